"""Device parity on edge-based partitions (Sec. 2.1: nodes labelled -1 form
a vertex separator, the shared interface).  A separator row of E^T couples
to the interiors of several subdomains, so the device applies E^T as a
CSR product after the B kernel instead of in its epilogue.

Bars as for the other parity tests: FP64 apply <= 1e-12 relative per
column, FP32 <= 1e-5 (oracle on the same stored data and low-rank part);
converged Ritz values <= 1e-10 relative; solve counts within +-1 and true
relative residual <= 1e-8."""
import numpy as np
import pytest

import oracle as O
import slr_inputs as si

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

CASES = [
    (2, 40, 4, "ic0", "ic0", "multicolor", 1),
    (3, 25, 3, "ic0", "ic0", "subdomain", 1),
    (3, 25, 3, "ict", "ict", "hid", 1),
    (3, 25, 3, "ict", "ict", "hid", 2),
]


def _dev(x):
    return torch.tensor(np.asarray(x), dtype=torch.float64, device="cuda")


def _relerr(a, b):
    a = np.asarray(a).reshape(np.asarray(a).shape[0], -1)
    b = np.asarray(b).reshape(np.asarray(b).shape[0], -1)
    return np.linalg.norm(a - b, axis=0) / np.linalg.norm(b, axis=0)


def _problem(dim, N, q):
    csr = si.laplacian_3d(N) if dim == 3 else si.laplacian_2d(N)
    return csr, si.separator_partition(N, q, dim), q ** dim, si.lanczos_start(csr[3])


def _ritz_bounds(alpha, beta):
    mm = len(alpha)
    T = np.diag(alpha) + np.diag(beta[:mm - 1], 1) + np.diag(beta[:mm - 1], -1)
    ev, Y = np.linalg.eigh(T)
    return ev[::-1], beta[-1] * np.abs(Y[-1, ::-1])


def _converged_set(vals, bnds, tol=1e-9):
    v = np.sort(vals[bnds <= tol])[::-1]
    out = []
    for x in v:
        if not out or abs(out[-1] - x) > 1e-7 * max(1.0, abs(x)):
            out.append(x)
    return np.array(out)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("dim,N,q,bf,cf,co,lv", CASES)
def test_separator_partition_apply(dim, N, q, bf, cf, co, lv, prec):
    import paper_1505_04340_amd as P
    print(f"separator apply dim={dim} N={N} q={q} {bf}/{cf} {co} levels={lv} {prec}", flush=True)
    csr, part, p, v0 = _problem(dim, N, q)
    kw = dict(lanczos_steps=40, b_fact=bf, c_fact=cf, c_order=co, c_levels=lv, k2=4)
    G = P.SLR(csr, part, p, k=8, v0=v0, fact_prec=prec, uk_prec=prec, **kw)
    ex = G.export()
    lr2 = None
    if lv == 2:
        ei = G.export_inner()
        lr2 = (ei["U"], ei["lambda"], ei["theta"])
    Po = O.setup(csr, part, p, 8, v0=v0, fact_prec=prec, uk_prec=prec,
                 lowrank=(ex["U"], ex["lambda"], ex["theta"]), lowrank2=lr2, **kw)
    assert (ex["perm"] == Po.perm).all() and G.info["s"] == int(np.sum(part < 0))
    tol = 1e-12 if prec == "fp64" else 1e-5
    for nrhs, seed in ((1, 5), (3, 6)):
        r = np.random.default_rng(seed).uniform(-1, 1, (csr[3], nrhs))
        assert _relerr(G.apply(_dev(r)).cpu().numpy(), Po.apply(r)).max() <= tol


def test_separator_partition_lanczos_and_solves():
    """Lanczos on H (E^T through the CSR product) against the oracle's own,
    then PCG and FGMRES counts."""
    import paper_1505_04340_amd as P
    csr, part, p, v0 = _problem(3, 33, 4)
    kw = dict(lanczos_steps=80, b_fact="ic0", c_fact="ic0", c_order="multicolor")
    print("separator lanczos and solves 33^3, 4^3 boxes", flush=True)
    G = P.SLR(csr, part, p, k=16, v0=v0, **kw)
    Po = O.setup(csr, part, p, 16, v0=v0, **kw)
    ex = G.export()
    gv, gb = _ritz_bounds(ex["alpha"], ex["beta"])
    ov, ob = _ritz_bounds(Po.alpha, Po.beta)
    gs, os_ = _converged_set(gv[:17], gb[:17]), _converged_set(ov[:17], ob[:17])
    n = min(len(gs), len(os_))
    assert n >= 1 and np.all(np.abs(gs[:n] - os_[:n]) <= 1e-10 * np.abs(os_[:n])), (gs[:n], os_[:n])
    xs, b = si.rhs_from_solution(csr, 1, 7)
    A = O.sp.csr_matrix((csr[2], csr[1], csr[0]), shape=(csr[3], csr[3]))
    for method in ("pcg", "fgmres"):
        ro = O.solve(Po, b[:, 0], method)
        x, info = G.solve(_dev(b[:, 0]), method)
        rr = np.linalg.norm(b[:, 0] - A @ x.cpu().numpy()) / np.linalg.norm(b[:, 0])
        assert ro.converged and info[0]["status"] == 0 and rr <= 1e-8, (method, info, rr)
        assert abs(info[0]["iters"] - ro.iters) <= 1, (method, info[0]["iters"], ro.iters)
