"""Writes tests/golden/shifted128_fgmres.json: the oracle's FGMRES(40) run on
the shifted 3-D 128^3 workload (20 negative eigenvalues, 8x8x8 boxes) with
the threshold local solvers of Sec. 6 -- ILDLT B_i after a minimum degree
ordering, ICT C in HID order (Sec. 5.2), drop tolerance 1e-4 -- k = 64 from
320 Lanczos steps (5k, Sec. 6), rtol 1e-8, at most 1000 iterations.

With --recursive it writes tests/golden/shifted128_fgmres_recursive.json
instead: the same run with the recursive SLR on C of Sec. 5.2 (the
leading HID level as the inner block diagonal, ICT at both levels, inner
rank 64 from 320 Lanczos steps) in place of the ICT factor of C, and at
most 3000 iterations.

Calls only the oracle and the input generators; about 25 minutes on one
core.  Run from the repository root: python tests/golden/make_shifted128_fgmres.py
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
import slr_inputs as si  # noqa: E402


def main(recursive: bool):
    pr = si.make_config("shifted3d_128")
    t0 = time.time()
    rec = dict(c_levels=2, k2=64) if recursive else {}
    maxit = 3000 if recursive else 1000
    P = O.setup(pr.csr, pr.part, pr.nparts, pr.k, pr.lanczos_steps, b_fact="ildlt", c_fact="ict", droptol=1e-4,
                c_order="hid", b_order="mindeg", v0=pr.v0(), **rec)
    t1 = time.time()
    xs, b = pr.rhs()
    r = O.solve(P, b[:, 0], "fgmres", rtol=1e-8, maxit=maxit, restart=40)
    t2 = time.time()
    out = {
        "workload": "shifted 3-D 7-point Laplacian 128^3, 20 negative eigenvalues, 8x8x8 boxes",
        "method": "ILDLT B_i (minimum degree order), ICT C (HID order), droptol 1e-4, k=64, 320 Lanczos steps, "
                  "FGMRES(40), rtol 1e-8, maxit 1000",
        "iters": int(r.iters), "converged": bool(r.converged), "true_relres": float(r.true_relres),
        "ritz_above_1": int(np.sum(P.ritz > 1.0)), "nnz_LB": int(P.FB.v.size),
        "theta": float(P.theta), "setup_s": round(t1 - t0, 1), "solve_s": round(t2 - t1, 1),
    }
    if recursive:
        inner = P.FC.inner
        out["method"] = out["method"].replace("ICT C (HID order)", "recursive SLR on C (HID order; ICT C1 and C2, "
                                              "inner k=64 from 320 Lanczos steps)").replace("maxit 1000",
                                                                                            "maxit 3000")
        out.update({"s1": int(P.FC.s1), "k2": int(inner.k), "theta2": float(inner.theta),
                    "lambda2": [float(v) for v in inner.lam],
                    "nnz_LC": int(inner.FB.v.size + inner.FC.v.size)})
        name = "shifted128_fgmres_recursive.json"
    else:
        out["nnz_LC"] = int(P.FC.v.size)
        name = "shifted128_fgmres.json"
    with open(os.path.join(ROOT, "tests", "golden", name), "w") as f:
        json.dump(out, f, indent=1)
    print(out)


if __name__ == "__main__":
    main("--recursive" in sys.argv[1:])
