"""Writes tests/golden/pcg_counts.json: the oracle's PCG iteration counts
(rtol 1e-8, x0 = 0, Sec. 6) on two full-size workloads, for the device's
counts to be held to:

- the 2-D diffusion 1024^2 workload (256 subdomains, k = 64 from 320
  Lanczos steps, IC(0) B_i and C, C in multicolour order, FP64 factors
  and U_k), right-hand-side columns 0, 7, 19 and 31, at most 3000
  iterations;
- the 2-D 512^2 serving matrix (64 subdomains, k = 32 from 160 steps,
  IC(0)/IC(0)) with C in multicolour and in subdomain order (the ordering
  of C's factor is a reading: the device uses the multicolour order), the
  workload's first right-hand side, at most 1000 iterations.

Calls only the oracle and the input generators; about 20 minutes on one
core.  Run from the repository root: python tests/golden/make_counts.py
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
import slr_inputs as si  # noqa: E402


def main():
    out = {}
    pr = si.make_config("diffusion2d_1024")
    t0 = time.time()
    P = O.setup(pr.csr, pr.part, pr.nparts, pr.k, pr.lanczos_steps, b_fact="ic0", c_fact="ic0",
                c_order="multicolor", v0=pr.v0())
    xs, b = pr.rhs()
    cols = [0, 7, 19, 31]
    its, rr = [], []
    for c in cols:
        r = O.solve(P, b[:, c], "pcg", rtol=1e-8, maxit=3000)
        its.append(int(r.iters))
        rr.append(float(r.true_relres))
        print("diffusion column", c, r.iters, r.converged, flush=True)
    out["diffusion2d_1024"] = {"method": "PCG, IC(0)/IC(0), C multicolour, FP64, k=64, 320 Lanczos steps",
                               "columns": cols, "iters": its, "true_relres": rr,
                               "seconds": round(time.time() - t0, 1)}
    pr = si.make_config("serve_lap2d_512")
    xs, b = pr.rhs()
    for order in ("multicolor", "subdomain"):
        t0 = time.time()
        P = O.setup(pr.csr, pr.part, pr.nparts, pr.k, pr.lanczos_steps, b_fact="ic0", c_fact="ic0",
                    c_order=order, v0=pr.v0())
        r = O.solve(P, b[:, 0], "pcg", rtol=1e-8, maxit=1000)
        out[f"serve_lap2d_512_{order}"] = {"method": f"PCG, IC(0)/IC(0), C {order}, FP64, k=32, 160 Lanczos steps",
                                           "iters": int(r.iters), "converged": bool(r.converged),
                                           "true_relres": float(r.true_relres),
                                           "seconds": round(time.time() - t0, 1)}
        print("serve 512", order, r.iters, r.converged, flush=True)
    with open(os.path.join(ROOT, "tests", "golden", "pcg_counts.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(out)


if __name__ == "__main__":
    main()
