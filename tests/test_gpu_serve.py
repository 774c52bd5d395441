"""Serving form: continuous batching over several resident preconditioners.

Each request's result from the multi-matrix service (requests of 1..4
columns arriving while others are in flight, batches smaller than the
offered load so that admission waits) must equal, bit for bit, the same
request solved alone in a fresh batch of its matrix, and reach a true FP64
relative residual <= 1e-8 (checked on the host with scipy).  The plain
one-request-at-a-time form reaches the same residual bar.
"""
import numpy as np
import pytest

import slr_inputs as si

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _true_relres(A, x, b):
    x = x.reshape(A.shape[0], -1)
    b = b.reshape(A.shape[0], -1)
    return np.linalg.norm(b - A @ x, axis=0) / np.linalg.norm(b, axis=0)


def test_service_matches_solo_batches():
    import paper_1505_04340_amd as P
    from paper_1505_04340_amd import serve
    prs = [si.make_config("serve_lap3d_64", N=20), si.make_config("serve_lap2d_256", N=48)]
    slrs = [P.SLR(pr.csr, pr.part, pr.nparts, k=8, lanczos_steps=40, c_order="multicolor",
                  fact_prec="fp32", uk_prec="bf16", v0=pr.v0()) for pr in prs]
    ns = [pr.n for pr in prs]
    reqs = serve.make_requests(ns, 14, 2000.0, seed=5, max_rhs=4)
    svc = serve.Service(slrs, "fcg", max_cols=5, iters_per_round=3)
    svc.run(reqs)
    svc.close()
    for rq in reqs:
        assert rq.done >= rq.admitted >= rq.arrival - 1e-9
        assert rq.info["status"] == 0, rq.info
        bt = P.Batch(slrs[rq.matrix], 4, "fcg")
        assert bt.admit(rq.b, 0) is not None
        out = []
        guard = 0
        while not out:
            bt.step(4)
            out = bt.poll()
            guard += 1
            assert guard < 1000
        bt.close()
        x_alone, info_alone = out[0][1], out[0][2]
        assert info_alone["iters"] == rq.info["iters"]
        assert torch.equal(x_alone.reshape(rq.x.shape), rq.x)
        A = prs[rq.matrix].scipy()
        rr = _true_relres(A, rq.x.cpu().numpy(), rq.b.cpu().numpy())
        assert rr.max() <= 1e-8, (rq.tag, rr)
    sm = serve.summarize(reqs, max(r.done for r in reqs))
    assert sm["all_converged"] and sm["requests"] == 14


def test_plain_service_converges():
    import paper_1505_04340_amd as P
    from paper_1505_04340_amd import serve
    prs = [si.make_config("serve_lap3d_64", N=20), si.make_config("serve_lap2d_256", N=48)]
    slrs = [P.SLR(pr.csr, pr.part, pr.nparts, k=8, lanczos_steps=40, c_order="multicolor", v0=pr.v0())
            for pr in prs]
    reqs = serve.make_requests([pr.n for pr in prs], 6, 0.0, seed=6, max_rhs=3)
    serve.serve_plain(slrs, reqs, "pcg")
    for rq in reqs:
        assert rq.info["status"] == 0
        rr = _true_relres(prs[rq.matrix].scipy(), rq.x.cpu().numpy(), rq.b.cpu().numpy())
        assert rr.max() <= 1e-8, (rq.tag, rr)
