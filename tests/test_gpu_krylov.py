"""Device Krylov recurrences against the oracle's textbook CG (Sec. 6).

The device runs CG and flexible CG with one reduction phase per iteration
(gamma = r.z, delta = z.A z, and for the flexible form z.A p_prev, summed in
one pass).  In exact arithmetic its iterates are those of the two-reduction
recurrence the oracle runs, so after m iterations the two solutions agree to
rounding; a wrong alpha, beta or curvature term shows up at m = 3 already.
A CPU rehearsal of both recurrences on this problem agrees to 2e-16 after
30 iterations; the bar here, 1e-10, leaves room for the apply's own 1e-12.
"""
import numpy as np
import pytest

import oracle as O
import slr_inputs as si

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _dev(x):
    return torch.tensor(np.asarray(x), dtype=torch.float64, device="cuda")


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


@pytest.fixture(scope="module")
def lap3d32():
    """32^3 Laplacian, 4x4x4 boxes, IC(0) / IC(0), multicolour C; the device
    takes the oracle's (U_k, Lambda_k, theta) so both apply one preconditioner."""
    import paper_1505_04340_amd as P
    pr = si.make_config("lap3d_64", N=32, boxes=4)
    Po = O.setup(pr.csr, pr.part, pr.nparts, pr.k, pr.lanczos_steps, b_fact=pr.b_fact, c_fact=pr.c_fact,
                 v0=pr.v0(), c_order="multicolor")
    G = P.SLR(pr.csr, pr.part, pr.nparts, k=pr.k, lanczos_steps=pr.lanczos_steps, b_fact=pr.b_fact,
              c_fact=pr.c_fact, v0=pr.v0(), c_order="multicolor", lowrank=(Po.U, Po.lam, Po.theta))
    xs, b = pr.rhs()
    return P, pr, Po, G, b[:, 0]


@pytest.mark.parametrize("method", ["pcg", "fcg"])
@pytest.mark.parametrize("m", [3, 12, 30])
def test_iterate_after_m_steps_matches_oracle(lap3d32, method, m):
    P, pr, Po, G, b = lap3d32
    ro = O.pcg(Po.A, Po.apply, b, rtol=1e-8, maxit=m, flexible=method == "fcg")
    assert not ro.converged
    x, info = G.solve(_dev(b), method, rtol=1e-8, maxit=m)
    assert info[0]["status"] == P.SLR_ERR_NOCONV
    assert info[0]["iters"] == m
    err = _rel(x.cpu().numpy(), ro.x)
    assert err <= 1e-10, err


@pytest.mark.parametrize("method", ["pcg", "fcg"])
def test_converged_count_matches_oracle(lap3d32, method):
    P, pr, Po, G, b = lap3d32
    ro = O.pcg(Po.A, Po.apply, b, rtol=1e-8, maxit=300, flexible=method == "fcg")
    x, info = G.solve(_dev(b), method, rtol=1e-8, maxit=300)
    assert ro.converged and info[0]["status"] == 0
    assert abs(info[0]["iters"] - ro.iters) <= 1
    assert info[0]["relres"] <= 1e-8
    assert _rel(x.cpu().numpy(), ro.x) <= 1e-7


def test_zero_column_and_columns_alone(lap3d32):
    """A zero right-hand side is done at once with x = 0; the other columns
    take the iterations and the solution they take alone."""
    P, pr, Po, G, b = lap3d32
    _, b3 = si.rhs_from_solution(pr.csr, 3, 77)
    B = np.array(b3)
    B[:, 1] = 0.0
    X, info = G.solve(_dev(B), "pcg", rtol=1e-8, maxit=300)
    X = X.cpu().numpy()
    assert info[1]["status"] == 0 and info[1]["iters"] == 0
    assert np.all(X[:, 1] == 0.0)
    for j in (0, 2):
        x1, i1 = G.solve(_dev(B[:, j]), "pcg", rtol=1e-8, maxit=300)
        assert info[j]["status"] == 0 and info[j]["iters"] == i1[0]["iters"]
        assert _rel(X[:, j], x1.cpu().numpy()) <= 1e-12


@pytest.mark.parametrize("method", ["pcg", "fcg"])
def test_poll_period_does_not_change_the_solve(lap3d32, method):
    """The host polls convergence between blocks of iterations whose lengths
    follow the residual's decay, with the next block queued before each poll.
    Iterations queued past convergence must leave x, the count and the
    residual as they were: every poll period gives the same bits, converged
    or stopped by maxit (also at a maxit that ends inside a block)."""
    P, pr, Po, G, b = lap3d32
    _, b3 = si.rhs_from_solution(pr.csr, 3, 91)
    for rhs in (b, np.array(b3)):
        for maxit in (300, 13):
            ref = None
            for every in (1, 3, 8, 100):
                x, info = G.solve(_dev(rhs), method, rtol=1e-8, maxit=maxit, check_every=every)
                got = (x.cpu().numpy(), [(i["iters"], i["status"], i["relres"]) for i in info])
                if maxit == 13:
                    assert all(i["iters"] == 13 and i["status"] == P.SLR_ERR_NOCONV for i in info)
                else:
                    assert all(i["status"] == 0 for i in info)
                if ref is None:
                    ref = got
                    continue
                assert got[1] == ref[1], (every, got[1], ref[1])
                assert np.array_equal(got[0], ref[0]), every


def test_fgmres_iterate_inside_a_cycle_matches_oracle(lap3d32):
    """FGMRES with a restart shorter than the iteration limit, stopped by
    maxit inside the third cycle: the device iterate equals the oracle's
    (MGS Arnoldi there, CGS2 on the device: equal in exact arithmetic) to
    1e-10.  The device queues Arnoldi steps ahead of the host's flag reads
    and keeps its workspace between solves: a second solve on the same
    context with another restart gives the bits of a fresh context."""
    P, pr, Po, G, b = lap3d32
    print("fgmres inside a cycle: lap3d N=32", flush=True)
    ro = O.fgmres(Po.A, Po.apply, b, rtol=1e-12, maxit=23, restart=10)
    assert not ro.converged and ro.iters == 23
    x, info = G.solve(_dev(b), "fgmres", rtol=1e-12, maxit=23, restart=10)
    assert info[0]["iters"] == 23 and info[0]["status"] == P.SLR_ERR_NOCONV
    assert _rel(x.cpu().numpy(), ro.x) <= 1e-10
    x7, i7 = G.solve(_dev(b), "fgmres", rtol=1e-8, maxit=300, restart=7)
    Gf = P.SLR(pr.csr, pr.part, pr.nparts, k=pr.k, lanczos_steps=pr.lanczos_steps, b_fact=pr.b_fact,
               c_fact=pr.c_fact, v0=pr.v0(), c_order="multicolor", lowrank=(Po.U, Po.lam, Po.theta))
    xf, if_ = Gf.solve(_dev(b), "fgmres", rtol=1e-8, maxit=300, restart=7)
    assert i7 == if_
    assert np.array_equal(x7.cpu().numpy(), xf.cpu().numpy())
    ro7 = O.fgmres(Po.A, Po.apply, b, rtol=1e-8, maxit=300, restart=7)
    assert ro7.converged and i7[0]["status"] == 0 and i7[0]["relres"] <= 1e-8
    assert abs(i7[0]["iters"] - ro7.iters) <= 1
