"""Boundary calls beyond setup / apply / solve: the serialised setup
(slr_export_setup / slr_import), the caller's allocator
(slr_set_allocator), slr_trim, the FGMRES workspace size, and the serving
loop's admission by device bytes against one shared budget."""
import numpy as np
import pytest
import scipy.sparse as sp

import slr_inputs as si

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _dev(x):
    return torch.tensor(np.asarray(x), dtype=torch.float64, device="cuda")


def _slr(pr, **kw):
    import paper_1505_04340_amd as P
    args = dict(k=8, lanczos_steps=40, b_fact=pr.b_fact, c_fact=pr.c_fact, v0=pr.v0())
    args.update(kw)
    return P.SLR(pr.csr, pr.part, pr.nparts, **args)


@pytest.mark.parametrize("form", ["fp64_multicolor", "mixed_multicolor", "fp64_subdomain"])
def test_export_import_round_trip(form):
    """An imported context applies and solves bit for bit like the exported
    one (the subdomain order takes the deep interface sweeps, the mixed form
    FP32 factors and BF16 U_k on matrix cores)."""
    import paper_1505_04340_amd as P
    print(f"export/import: {form}", flush=True)
    pr = si.make_config("lap3d_64", N=24, boxes=3)
    kw = {"fp64_multicolor": dict(c_order="multicolor"),
          "mixed_multicolor": dict(c_order="multicolor", fact_prec="fp32", uk_prec="bf16"),
          "fp64_subdomain": dict(c_order="subdomain")}[form]
    G = _slr(pr, **kw)
    blob = G.export_setup()
    Gi = P.SLR.import_setup(blob)
    for f in ("n", "m", "s", "p", "k", "c_levels", "nnz_LB", "nnz_LC", "nnz_E", "nnz_A", "lanczos_steps"):
        assert Gi.info[f] == G.info[f], f
    assert Gi.info["theta"] == G.info["theta"]
    ex, exi = G.export(), Gi.export()
    for f in ("perm", "lambda", "U", "alpha", "beta", "ritz"):
        assert np.array_equal(ex[f], exi[f]), f
    r = _dev(np.random.default_rng(3).uniform(-1, 1, (pr.n, 3)))
    assert torch.equal(G.apply(r), Gi.apply(r))
    xs, b = pr.rhs()
    method = "pcg" if form.startswith("fp64") else "fcg"
    x1, i1 = G.solve(_dev(b[:, 0]), method)
    x2, i2 = Gi.solve(_dev(b[:, 0]), method)
    assert i1 == i2 and i1[0]["status"] == 0
    assert torch.equal(x1, x2)
    # a second export of the imported context is the same bytes
    assert Gi.export_setup() == blob
    # damaged bytes are refused
    bad = bytearray(blob)
    bad[len(bad) // 2] ^= 0xFF
    with pytest.raises(P.SLRError) as e:
        P.SLR.import_setup(bytes(bad))
    assert e.value.code == P.SLR_ERR_ARG
    with pytest.raises(P.SLRError):
        P.SLR.import_setup(blob[:-9])


def test_export_after_refactor_takes_the_new_values():
    import paper_1505_04340_amd as P
    print("export after refactor", flush=True)
    pr = si.make_config("lap3d_64", N=20, boxes=2)
    G = _slr(pr, c_order="multicolor", refactor=True)
    A = pr.scipy().tocsr()
    A2 = (A + 0.5 * sp.identity(A.shape[0])).tocsr()
    A2.sort_indices()
    G.refactor(A2)
    Gi = P.SLR.import_setup(G.export_setup())
    r = _dev(np.random.default_rng(4).uniform(-1, 1, (pr.n, 2)))
    assert torch.equal(G.apply(r), Gi.apply(r))
    assert torch.equal(G.spmv(r), Gi.spmv(r))


def test_torch_allocator_owns_the_device_memory():
    """With PyTorch's allocator installed every device allocation of the
    library goes through it: free device memory drops by what PyTorch
    reserves (nothing else), the hook holds at least the context's
    device_bytes, and everything comes back at destroy.  Results equal those
    of a context built with hipMalloc."""
    import paper_1505_04340_amd as P
    print("torch allocator", flush=True)
    pr = si.make_config("lap3d_64", N=32, boxes=4)
    r = _dev(np.random.default_rng(5).uniform(-1, 1, (pr.n, 2)))
    xs, b = pr.rhs()
    G0 = _slr(pr, c_order="multicolor")
    z0 = G0.apply(r)
    x0, i0 = G0.solve(_dev(b[:, 0]), "fgmres")
    G0.close()
    torch.cuda.synchronize()
    hook = P.use_torch_allocator()
    try:
        a0 = hook.allocs
        free0, _ = torch.cuda.mem_get_info()
        res0 = torch.cuda.memory_reserved()
        G = _slr(pr, c_order="multicolor")
        z = G.apply(r)
        x, i1 = G.solve(_dev(b[:, 0]), "fgmres")
        bt = P.Batch(G, 3, "pcg")
        bt.admit(_dev(b[:, :1]), 0)
        bt.step(2)
        torch.cuda.synchronize()
        free1, _ = torch.cuda.mem_get_info()
        res1 = torch.cuda.memory_reserved()
        assert hook.allocs > a0
        assert hook.live_bytes() >= G.query()["device_bytes"]
        # no device memory beyond what PyTorch reserved (2 MiB granularity slack)
        assert (free0 - free1) - (res1 - res0) <= 4 << 20, (free0 - free1, res1 - res0)
        assert torch.equal(z, z0) and torch.equal(x, x0) and i1 == i0
        bt.close()
        G.close()
        torch.cuda.synchronize()
        assert hook.live_bytes() == 0 and hook.frees == hook.allocs
    finally:
        P.use_hip_allocator()


def test_trim_and_fgmres_workspace_bytes():
    import paper_1505_04340_amd as P
    print("trim and workspace bytes", flush=True)
    pr = si.make_config("lap3d_64", N=24, boxes=3)
    G = _slr(pr, c_order="multicolor")
    w10, w40 = G.workspace_bytes(1, "fgmres", restart=10), G.workspace_bytes(1, "fgmres", restart=40)
    assert w40 > w10 >= 2 * 11 * 8 * pr.n
    xs, b = pr.rhs()
    G.trim()
    d0 = G.query()["device_bytes"]
    x, i = G.solve(_dev(b[:, 0]), "fgmres", restart=40)
    d1 = G.query()["device_bytes"]
    assert d1 - d0 == w40, (d1 - d0, w40)
    G.trim()
    assert G.query()["device_bytes"] == d0
    x2, i2 = G.solve(_dev(b[:, 0]), "fgmres", restart=40)
    assert i2 == i and torch.equal(x, x2)


def test_service_admits_by_bytes_under_a_shared_budget():
    """A budget with room for about one batch beyond the resident
    preconditioners: batches are made and destroyed as requests of the two
    matrices come and go, the device bytes never pass the budget, and every
    result equals the same request solved alone."""
    import paper_1505_04340_amd as P
    from paper_1505_04340_amd import serve
    print("service admission by bytes", flush=True)
    prs = [si.make_config("serve_lap3d_64", N=20), si.make_config("serve_lap2d_256", N=48)]
    slrs = [P.SLR(pr.csr, pr.part, pr.nparts, k=8, lanczos_steps=40, c_order="multicolor",
                  fact_prec="fp32", uk_prec="bf16", v0=pr.v0()) for pr in prs]
    probe = [P.Batch(s, 4, "fcg") for s in slrs]
    per4 = max(b.bytes() for b in probe)
    for b in probe:
        b.close()
    resident = sum(s.query()["device_bytes"] for s in slrs)
    budget = resident + int(1.5 * per4)
    reqs = serve.make_requests([pr.n for pr in prs], 12, 3000.0, seed=8, max_rhs=4)
    svc = serve.Service(slrs, "fcg", hbm_budget_bytes=budget, max_cols=4, batch_cols=4, iters_per_round=3)
    svc.run(reqs)
    svc.close()
    assert svc.peak_bytes <= budget
    assert svc.batches_made > 2
    for rq in reqs:
        assert rq.info["status"] == 0
        bt = P.Batch(slrs[rq.matrix], 4, "fcg")
        bt.admit(rq.b, 0)
        out = []
        while not out:
            bt.step(4)
            out = bt.poll()
        bt.close()
        assert out[0][2]["iters"] == rq.info["iters"]
        assert torch.equal(out[0][1].reshape(rq.x.shape), rq.x)


@pytest.mark.parametrize("prec", [("fp64", "fp64"), ("fp32", "bf16")])
def test_autotune_keeps_results(prec):
    """slr_autotune picks the B kernel's launch shape for one and for several
    columns and the rank-k chunks: the apply still matches the oracle, and a
    column applied alone (the one-column shape) equals, bit for bit, the
    same column inside a 12-column apply (the several-column shape)."""
    import oracle as O
    fp, up = prec
    print(f"autotune: {fp}/{up}", flush=True)
    pr = si.make_config("diffusion2d_1024", N=192, boxes=6)
    Po = O.setup(pr.csr, pr.part, pr.nparts, 16, 80, b_fact=pr.b_fact, c_fact=pr.c_fact, c_order="multicolor",
                 fact_prec=fp, uk_prec=up, v0=pr.v0())
    G = _slr(pr, k=16, lanczos_steps=80, c_order="multicolor", fact_prec=fp, uk_prec=up,
             lowrank=(Po.U, Po.lam, Po.theta))
    t12 = G.autotune(12)
    t1 = G.autotune(1)
    assert t12["tune_b_threadsM"] in (0, 256, 512, 1024) and t1["tune_b_threads1"] in (0, 256, 512, 1024)
    assert t1["lr_chunks"] >= 128
    r = np.random.default_rng(9).uniform(-1, 1, (pr.n, 12))
    Z = G.apply(_dev(r)).cpu().numpy()
    zo = Po.apply(r)
    err = (np.linalg.norm(Z - zo, axis=0) / np.linalg.norm(zo, axis=0)).max()
    assert err <= (1e-12 if fp == "fp64" else 1e-5), err
    for j in (0, 5, 11):
        assert np.array_equal(G.apply(_dev(r[:, j])).cpu().numpy(), Z[:, j])
    Gi = type(G).import_setup(G.export_setup())
    assert Gi.info["lr_chunks"] == G.info["lr_chunks"]
    assert np.array_equal(Gi.apply(_dev(r)).cpu().numpy(), Z)


@pytest.mark.parametrize("prec", [("fp64", "fp64"), ("fp32", "bf16")])
def test_persistent_bsolve_plan_is_bitwise_the_same(prec):
    """The batching form's persistent launch (a resident grid walking a
    longest-first schedule of (subdomain, column group) items over
    subdomains of uneven size) gives the same bits as the plain grid, for
    several shapes, and survives the serialised setup."""
    fp, up = prec
    print(f"persistent B plan: {fp}/{up}", flush=True)
    pr = si.make_config("diffusion2d_1024", N=256, boxes=8)     # 64 subdomains of uneven size
    G = _slr(pr, k=16, lanczos_steps=80, c_order="multicolor", fact_prec=fp, uk_prec=up)
    r = _dev(np.random.default_rng(10).uniform(-1, 1, (pr.n, 32)))
    Z = G.apply(r).cpu().numpy()
    for threads, div, rmax in ((256, 4, 1), (512, 2, 2), (1024, 1, 4)):
        for mode in (1, 2, 0):
            G.set_bsolve_plan(True, threads, div, rmax, persistent=mode)
            assert G.info["tune_b_persistentM"] == mode
            assert np.array_equal(G.apply(r).cpu().numpy(), Z), (threads, div, rmax, mode)
    G.set_bsolve_plan(True, 512, 2, 2, persistent=2)
    Gi = type(G).import_setup(G.export_setup())
    assert Gi.info["tune_b_persistentM"] == 2
    assert np.array_equal(Gi.apply(r).cpu().numpy(), Z)
    G.set_bsolve_plan(True, 0)
    assert G.info["tune_b_persistentM"] == 0 and G.info["tune_b_threadsM"] == 0


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_column_results_do_not_depend_on_the_column_count(prec):
    """A column of a several-column apply equals, bit for bit, the same
    column applied alone, at column counts that take every register tile
    of the rank-k kernels (1, 4, 8 and 16 columns per pass) and several B
    kernel column groups: the batched service relies on this."""
    pr = si.make_config("lap3d_64", N=32, boxes=4)
    G = _slr(pr, k=16, lanczos_steps=80, c_order="multicolor", fact_prec=prec, uk_prec=prec)
    R = np.random.default_rng(91).uniform(-1, 1, (pr.n, 20))
    alone = np.column_stack([G.apply(_dev(R[:, j])).cpu().numpy() for j in range(20)])
    for nc in (5, 12, 20):
        Z = G.apply(_dev(R[:, :nc])).cpu().numpy()
        assert np.array_equal(Z, alone[:, :nc]), nc
