"""slr_apply_dd_noalloc: the apply for callers that cannot allocate device
memory, with its scratch in the library's fixed per-GPU array.

Checked against slr_apply_dd (the existing entry point with allocated
scratch) on the same context and inputs: the two run the same kernels in
the same order, so the outputs must be equal bit for bit, which is within
the FP64 bar of 1e-12 and the FP32 / BF16 bar of 1e-5.  Two calls in a row,
the second with a smaller input, show that what the first call leaves in
the shared array does not leak into the second.  The mixed-precision
context and a second, smaller context exercise other kernels and layouts
on the same array; an nrhs whose scratch exceeds the array is refused
before any launch.
"""
import numpy as np
import pytest

import slr_inputs as si

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _dev(x):
    return torch.tensor(np.asarray(x), dtype=torch.float64, device="cuda")


def _slr(pr, **kw):
    import paper_1505_04340_amd as P
    args = dict(k=8, lanczos_steps=40, b_fact=pr.b_fact, c_fact=pr.c_fact, v0=pr.v0(), c_order="multicolor")
    args.update(kw)
    return P.SLR(pr.csr, pr.part, pr.nparts, **args)


def _rel(a, b):
    a = a.reshape(a.shape[0], -1)
    b = b.reshape(b.shape[0], -1)
    return float((np.linalg.norm(a - b, axis=0) / np.linalg.norm(b, axis=0)).max())


@pytest.mark.parametrize("prec", [("fp64", "fp64"), ("fp32", "bf16")])
def test_noalloc_apply_equals_apply_dd(prec):
    fact_prec, uk_prec = prec
    print(f"noalloc apply: lap3d N=32 boxes=4, {fact_prec}/{uk_prec}", flush=True)
    pr = si.make_config("lap3d_64", N=32, boxes=4)
    G = _slr(pr, fact_prec=fact_prec, uk_prec=uk_prec)
    rng = np.random.default_rng(5)
    tol = 1e-12 if fact_prec == "fp64" else 1e-5
    for nr in (6, 2):          # second call smaller than the first
        r = _dev(rng.uniform(-1, 1, (pr.n, nr)))
        z_ref = G.apply_dd(r).cpu().numpy()
        z = G.apply_dd_noalloc(r).cpu().numpy()
        assert _rel(z, z_ref) <= tol
        assert np.array_equal(z, z_ref), nr
    # single column (vector form)
    r1 = _dev(rng.uniform(-1, 1, pr.n))
    assert np.array_equal(G.apply_dd_noalloc(r1).cpu().numpy(), G.apply_dd(r1).cpu().numpy())


def test_noalloc_apply_second_context_and_size_limit():
    import paper_1505_04340_amd as P
    print("noalloc apply: lap3d N=32 then lap2d N=40, then the size limit", flush=True)
    pa = si.make_config("lap3d_64", N=32, boxes=4)
    pb = si.make_config("lap2d_64", N=40)
    Ga = _slr(pa)
    Gb = P.SLR(pb.csr, pb.part, pb.nparts, k=6, lanczos_steps=30, b_fact=pb.b_fact, c_fact=pb.c_fact, v0=pb.v0())
    rng = np.random.default_rng(6)
    ra = _dev(rng.uniform(-1, 1, (pa.n, 3)))
    rb = _dev(rng.uniform(-1, 1, (pb.n, 1)))
    za = Ga.apply_dd_noalloc(ra).cpu().numpy()
    zb = Gb.apply_dd_noalloc(rb).cpu().numpy()
    assert np.array_equal(za, Ga.apply_dd(ra).cpu().numpy())
    assert np.array_equal(zb, Gb.apply_dd(rb).cpu().numpy())
    assert np.array_equal(Ga.apply_dd_noalloc(ra[:, :1]).cpu().numpy().ravel(), za[:, 0])
    # scratch beyond the fixed array: refused with SLR_ERR_ARG, nothing launched
    s = Ga.info["s"]
    big = (64 << 20) // (16 * s) + 8
    rbig = torch.zeros((big, pa.n), dtype=torch.float64, device="cuda").t()
    with pytest.raises(P.SLRError) as e:
        Ga.apply_dd_noalloc(rbig)
    assert e.value.code == P.SLR_ERR_ARG
    assert np.array_equal(Ga.apply_dd_noalloc(ra).cpu().numpy(), za)


@pytest.mark.parametrize("form", ["recursive", "separator"])
def test_noalloc_apply_recursive_and_separator(form):
    """The recursive interface solver (its scratch: the second interface
    block and the inner rank-k partials) and an edge-based partition (the
    interior block z that the E^T product reads) on the fixed array."""
    import paper_1505_04340_amd as P
    print(f"noalloc apply: {form}", flush=True)
    if form == "recursive":
        pr = si.make_config("shifted3d_128", N=24, boxes=3, neg=10)
        G = P.SLR(pr.csr, pr.part, pr.nparts, k=8, lanczos_steps=40, b_fact="ildlt", c_fact="ict", c_order="hid",
                  c_levels=2, k2=4, v0=pr.v0())
        n = pr.n
    else:
        csr = si.laplacian_3d(25)
        part = si.separator_partition(25, 3, 3)
        G = P.SLR(csr, part, 27, k=8, lanczos_steps=40, v0=si.lanczos_start(csr[3]))
        n = csr[3]
    rng = np.random.default_rng(8)
    for nr in (4, 1):
        r = _dev(rng.uniform(-1, 1, (n, nr)))
        assert np.array_equal(G.apply_dd_noalloc(r).cpu().numpy(), G.apply_dd(r).cpu().numpy()), nr
