"""Numeric refactorisation on the device (slr_refactor): same pattern, new
values.  The zero-fill factors of the B_i and of C are recomputed level by
level on the device and every stored coefficient is rewritten in place, so
the apply equals that of a fresh setup with the new values (given the same
low-rank part) bit for bit: the device takes the host factorisation's
operations in the same order (no contraction into fused multiply-adds,
correctly rounded division and square root).  The oracle with the new
values agrees to the apply bars (1e-12 FP64, 1e-5 FP32 factors).  A failed
pivot leaves every stored coefficient as it was."""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle as O
import slr_inputs as si

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

N, BOXES = 48, 3


def _dev(x):
    return torch.tensor(np.asarray(x), dtype=torch.float64, device="cuda")


def _relerr(a, b):
    return np.linalg.norm(a - b, axis=0) / np.linalg.norm(b, axis=0)


def _problem(seed):
    rng = np.random.default_rng(seed)
    return si.diffusion_2d(N, np.exp(rng.standard_normal((N + 2, N + 2))))


def _part():
    return si.random_cuts_2d(N, BOXES, BOXES, 3)


def _csr(t):
    indptr, indices, data, n = t
    return sp.csr_matrix((data, indices, indptr), shape=(n, n))


@pytest.mark.parametrize("fact_prec,b_fact", [("fp64", "ic0"), ("fp64", "ildlt0"), ("fp32", "ic0")])
def test_refactor_equals_fresh_setup(fact_prec, b_fact):
    import paper_1505_04340_amd as P
    A1, A2 = _problem(1), _problem(2)
    part = _part()
    kw = dict(b_fact=b_fact, c_fact="ic0", c_order="multicolor", fact_prec=fact_prec, uk_prec=fact_prec)
    G = P.SLR(A1, part, BOXES * BOXES, k=8, lanczos_steps=40, refactor=True, **kw)
    ex = G.export()
    lr = (ex["U"], ex["lambda"], ex["theta"])
    G.refactor(A2)
    F = P.SLR(A2, part, BOXES * BOXES, lowrank=lr, **kw)
    n = A2[3]
    r = np.random.default_rng(5).uniform(-1, 1, (n, 3))
    z = G.apply(_dev(r)).cpu().numpy()
    zf = F.apply(_dev(r)).cpu().numpy()
    print(f"[refactor] {fact_prec}/{b_fact}: bitwise equal to a fresh setup: {np.array_equal(z, zf)}")
    assert np.array_equal(z, zf)
    # the same values from device memory
    G.refactor_values(torch.tensor(A2[2], dtype=torch.float64, device="cuda"))
    assert np.array_equal(G.apply(_dev(r)).cpu().numpy(), zf)
    # the Krylov products use the new values
    x = np.random.default_rng(6).uniform(-1, 1, n)
    q = G.spmv(_dev(x)).cpu().numpy()
    assert np.abs(q - _csr(A2) @ x).max() <= 1e-12 * np.abs(_csr(A2) @ x).max()
    # the oracle with the new values and the same low-rank part
    rnd = O.round_fp32 if fact_prec == "fp32" else (lambda u: u)
    Po = O.setup(A2, part, BOXES * BOXES, 0, b_fact=b_fact, c_fact="ic0", c_order="multicolor",
                 fact_prec=fact_prec, lowrank=(rnd(ex["U"]), ex["lambda"], ex["theta"]))
    assert _relerr(z, Po.apply(r)).max() <= (1e-12 if fact_prec == "fp64" else 1e-5)
    # rebuild the low-rank part for the new matrix and solve
    G.update_lowrank(8, 40)
    xs = np.random.default_rng(7).uniform(-1, 1, n)
    b = _csr(A2) @ xs
    xx, info = G.solve(_dev(b), "pcg" if fact_prec == "fp64" else "fcg")
    assert info[0]["status"] == 0 and info[0]["relres"] <= 1e-8


def test_refactor_failed_pivot_keeps_coefficients():
    import paper_1505_04340_amd as P
    A1 = _problem(1)
    part = _part()
    G = P.SLR(A1, part, BOXES * BOXES, k=8, lanczos_steps=40, c_order="multicolor", refactor=True)
    ex = G.export()
    n = A1[3]
    r = np.random.default_rng(8).uniform(-1, 1, (n, 2))
    z0 = G.apply(_dev(r)).cpu().numpy()
    m = ex["m"]
    for node, code in ((int(ex["perm"][m // 2]), P.SLR_ERR_BREAKDOWN), (int(ex["perm"][m + 3]), P.SLR_ERR_C_NOT_SPD)):
        Ab = _csr(A1).tolil()
        Ab[node, node] = -1.0
        Ab = Ab.tocsr()
        Ab.sort_indices()
        with pytest.raises(P.SLRError) as ei:
            G.refactor(Ab)
        assert ei.value.code == code
        assert np.array_equal(G.apply(_dev(r)).cpu().numpy(), z0)
    # values that break symmetry, from the host and from device memory
    vals = np.array(A1[2], dtype=np.float64)
    off = int(np.flatnonzero(np.asarray(A1[1]) != np.repeat(np.arange(n), np.diff(A1[0])))[0])
    vals[off] *= 1.5
    with pytest.raises(P.SLRError) as ei:
        G.refactor((A1[0], A1[1], vals, n))
    assert ei.value.code == P.SLR_ERR_NOT_SYMMETRIC
    with pytest.raises(P.SLRError) as ei:
        G.refactor_values(torch.tensor(vals, device="cuda"))
    assert ei.value.code == P.SLR_ERR_NOT_SYMMETRIC
    assert np.array_equal(G.apply(_dev(r)).cpu().numpy(), z0)
    # refused: pattern change, no refactor option, live batch
    with pytest.raises(ValueError):
        G.refactor(_csr(A1) + sp.eye(n, format="csr") * 0 + sp.csr_matrix(([1.0], ([0], [n - 1])), shape=(n, n)))
    H = P.SLR(A1, part, BOXES * BOXES, k=4, lanczos_steps=20)
    with pytest.raises(ValueError):
        H.refactor(A1)
    bt = P.Batch(G, 2)
    with pytest.raises(P.SLRError):
        G.refactor(_problem(3))
    bt.close()
    G.refactor(_problem(3))
