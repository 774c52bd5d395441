"""Device parity of the recursive interface solver (Sec. 5.2): the solve
with C is itself an SLR preconditioner, with the lowest HID connector level
as its block diagonal, used in the factored form K K^T.

Bars as for the other parity tests: FP64 apply <= 1e-12 relative per
column and FP32 <= 1e-5, against the oracle on the same stored data and
the device's own low-rank parts (both levels); converged outer Ritz values
<= 1e-10 relative against the oracle's Lanczos on the same inner part;
inner Ritz values against the oracle's own inner Lanczos; solve counts
within +-1 of the oracle's own run and true relative residual <= 1e-8."""
import numpy as np
import pytest

import oracle as O
import slr_inputs as si

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

CASES = [
    ("lap3d_64", dict(N=16, boxes=2), "ic0", "ic0", "natural", 8, 4),
    ("lap3d_64", dict(N=24, boxes=3), "ict", "ict", "mindeg", 16, 8),
    ("shifted3d_128", dict(N=24, boxes=3, neg=10), "ildlt", "ict", "mindeg", 16, 8),
    ("diffusion2d_1024", dict(N=96, boxes=4), "ic0", "ic0", "natural", 8, 4),
]


def _dev(x):
    return torch.tensor(np.asarray(x), dtype=torch.float64, device="cuda")


def _relerr(a, b):
    a = np.asarray(a).reshape(np.asarray(a).shape[0], -1)
    b = np.asarray(b).reshape(np.asarray(b).shape[0], -1)
    return np.linalg.norm(a - b, axis=0) / np.linalg.norm(b, axis=0)


def _kw(bf, cf, bo, k, k2):
    return dict(lanczos_steps=5 * k, b_fact=bf, c_fact=cf, droptol=1e-3, c_order="hid", b_order=bo, c_levels=2,
                k2=k2)


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


@pytest.mark.parametrize("prec", ["fp64", "fp32", "mixed"])
@pytest.mark.parametrize("name,over,bf,cf,bo,k,k2", CASES)
def test_recursive_interface_apply(name, over, bf, cf, bo, k, k2, prec):
    """"mixed" is FP32 factors at both levels with a BF16 outer U_k (the
    inner U2 stays FP64)."""
    import paper_1505_04340_amd as P
    print(f"recursive apply {name} {over} {bf}/{cf} {bo} k={k} k2={k2} {prec}", flush=True)
    pr = si.make_config(name, **over)
    kw = _kw(bf, cf, bo, k, k2)
    fp, up = ("fp32", "bf16") if prec == "mixed" else (prec, prec)
    G = P.SLR(pr.csr, pr.part, pr.nparts, k=k, v0=pr.v0(), fact_prec=fp, uk_prec=up, **kw)
    ex, ei = G.export(), G.export_inner()
    assert G.info["k2"] == k2 and G.info["s1"] == ei["s1"] > 0
    Po = O.setup(pr.csr, pr.part, pr.nparts, k, v0=pr.v0(), fact_prec=fp, uk_prec=up,
                 lowrank=(ex["U"], ex["lambda"], ex["theta"]), lowrank2=(ei["U"], ei["lambda"], ei["theta"]), **kw)
    assert (ex["perm"] == Po.perm).all() and G.info["s1"] == Po.FC.s1
    if cf != "chol":
        assert G.info["nnz_LC"] == Po.FC.inner.FB.v.size + Po.FC.inner.FC.v.size
    tol = 1e-12 if prec == "fp64" else 1e-5
    for nrhs, seed in ((1, 3), (3, 4)):
        r = np.random.default_rng(seed).uniform(-1, 1, (pr.n, nrhs))
        z = G.apply(_dev(r)).cpu().numpy()
        assert _relerr(z, Po.apply(r)).max() <= tol


@pytest.mark.parametrize("name,over,bf,cf,bo,k,k2", CASES[:3])
def test_recursive_interface_lanczos(name, over, bf, cf, bo, k, k2):
    """The inner Lanczos (on H2 = L2^{-1} F^T C1^{-1} F L2^{-T}) against the
    oracle's own from the same start vector; the outer one (on K^T E^T
    B^{-1} E K) against the oracle's with the device's inner part."""
    import paper_1505_04340_amd as P
    print(f"recursive lanczos {name} {over}", flush=True)
    pr = si.make_config(name, **over)
    kw = _kw(bf, cf, bo, k, k2)
    G = P.SLR(pr.csr, pr.part, pr.nparts, k=k, v0=pr.v0(), reorth="full", **kw)
    ex, ei = G.export(), G.export_inner()
    Pown = O.setup(pr.csr, pr.part, pr.nparts, k, v0=pr.v0(), reorth="full", **kw)
    inner = Pown.FC.inner
    assert len(ei["ritz"]) == len(inner.ritz)
    assert np.allclose(ei["ritz"][:k2 + 1], inner.ritz[:k2 + 1], rtol=1e-9, atol=0)
    assert abs(ei["theta"] - inner.theta) <= 1e-9 * abs(inner.theta)
    # the same invariant subspace where the inner values are apart
    gap = np.abs(np.diff(inner.ritz[:k2 + 1]))
    if gap.min() > 1e-4:
        cosines = np.linalg.svd(ei["U"].T @ inner.U, compute_uv=False)
        assert cosines.min() > 1 - 1e-8
    Pi = O.setup(pr.csr, pr.part, pr.nparts, k, v0=pr.v0(), reorth="full",
                 lowrank2=(ei["U"], ei["lambda"], ei["theta"]), **kw)
    gv, gb = _ritz_bounds(ex["alpha"], ex["beta"])
    ov, ob = _ritz_bounds(Pi.alpha, Pi.beta)
    gs, os_ = _converged_set(gv[:k + 1], gb[:k + 1]), _converged_set(ov[:k + 1], ob[:k + 1])
    n = min(len(gs), len(os_))
    assert n >= 1
    assert np.all(np.abs(gs[:n] - os_[:n]) <= 1e-10 * np.abs(os_[:n])), (gs[:n], os_[:n])


@pytest.mark.parametrize("case", ["pcg", "fgmres"])
def test_recursive_interface_solve(case):
    """Solves with the recursive interface solver: the oracle's own run
    (its own Lanczos at both levels) gives the count."""
    import paper_1505_04340_amd as P
    if case == "pcg":
        pr = si.make_config("lap3d_64", N=32, boxes=4)
        k, k2, kw = 16, 8, _kw("ic0", "ic0", "natural", 16, 8)
    else:
        pr = si.make_config("shifted3d_128", N=32, boxes=4, neg=20)
        k, k2, kw = 32, 16, _kw("ildlt", "ict", "mindeg", 32, 16)
        kw["droptol"] = 1e-4
    print(f"recursive solve {case}", flush=True)
    Po = O.setup(pr.csr, pr.part, pr.nparts, k, v0=pr.v0(), **kw)
    G = P.SLR(pr.csr, pr.part, pr.nparts, k=k, v0=pr.v0(), **kw)
    xs, b = pr.rhs()
    ro = O.solve(Po, b[:, 0], case, maxit=1000)
    x, info = G.solve(_dev(b[:, 0]), case, maxit=1000)
    rr = np.linalg.norm(b[:, 0] - pr.scipy() @ x.cpu().numpy()) / np.linalg.norm(b[:, 0])
    assert ro.converged and info[0]["status"] == 0 and rr <= 1e-8, (info, rr)
    assert abs(info[0]["iters"] - ro.iters) <= 1, (info[0]["iters"], ro.iters)


@pytest.mark.parametrize("form", ["recursive", "separator", "separator_recursive"])
def test_batch_with_recursive_and_separator_contexts(form):
    """Continuous batching over a context with the recursive interface
    solver and/or an edge-based partition: every request's result and count
    are the same whether it runs alone or shares the batch with others that
    arrive while it is in flight, and each converges to 1e-8."""
    import paper_1505_04340_amd as P
    print(f"batch {form}", flush=True)
    if form == "recursive":
        pr = si.make_config("lap3d_64", N=24, boxes=3)
        csr, part, p, v0 = pr.csr, pr.part, pr.nparts, pr.v0()
        kw = _kw("ict", "ict", "mindeg", 16, 8)
    else:
        csr = si.laplacian_3d(25)
        part, p, v0 = si.separator_partition(25, 3, 3), 27, si.lanczos_start(csr[3])
        kw = dict(lanczos_steps=40, c_order="hid", b_fact="ict", c_fact="ict",
                  c_levels=2 if form == "separator_recursive" else 1, k2=4)
    G = P.SLR(csr, part, p, k=8 if form != "recursive" else 16, v0=v0, **kw)
    n = csr[3]
    rng = np.random.default_rng(11)
    reqs = [rng.uniform(-1, 1, (n, r)) for r in (1, 3, 2, 1)]
    alone = []
    for q, b in enumerate(reqs):
        bt = P.Batch(G, 4, "pcg", maxit=500)
        bt.admit(_dev(b), q)
        out = []
        while not out:
            bt.step(4)
            out = bt.poll()
        alone.append((out[0][1].cpu().numpy(), out[0][2]))
        bt.close()
    bt = P.Batch(G, 5, "pcg", maxit=500)
    got, pending, steps = {}, list(enumerate(reqs)), 0
    while len(got) < len(reqs):
        while pending and bt.admit(_dev(pending[0][1]), pending[0][0]) is not None:
            pending.pop(0)
        bt.step(3)
        steps += 1
        for tag, x, info in bt.poll():
            got[tag] = (x.cpu().numpy(), info)
        assert steps < 1000
    bt.close()
    for q in range(len(reqs)):
        (xa, ia), (xm, im) = alone[q], got[q]
        assert ia["status"] == 0 and im["status"] == 0 and im["relres"] <= 1e-8
        assert ia["iters"] == im["iters"]
        assert np.array_equal(xa.reshape(n, -1), xm.reshape(n, -1))
