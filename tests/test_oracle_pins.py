"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these re-type the oracle's formulas: each compares the oracle with
an independent dense computation, a closed form, a value the paper prints,
or an identity the method must satisfy (Li, Xi & Saad 2015).
"""
import json
import math
import os

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

import oracle as O
import slr_inputs as si

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _dense_blocks(P):
    Ad = P.Ap.toarray()
    m = P.m
    return Ad, Ad[:m, :m], Ad[:m, m:], Ad[m:, m:]


def _dense_H(P):
    """H = L^{-1} E^T B^{-1} E L^{-T} with L = chol(C), by dense algebra
    (eq. S, eq. H) -- independent of the oracle's sparse code."""
    _, B, E, C = _dense_blocks(P)
    L = np.linalg.cholesky(C)
    X = np.linalg.solve(B, E)
    H = sla.solve_triangular(L, E.T @ X, lower=True)
    H = sla.solve_triangular(L, H.T, lower=True).T
    return 0.5 * (H + H.T), L


def _tiny(N=12, boxes=2, **kw):
    csr = si.laplacian_2d(N)
    part = si.box_partition_2d(N, boxes, boxes)
    return csr, part, boxes * boxes


# ---------------------------------------------------------------- generators

def test_generator_closed_form_spectrum_2d_3d():
    """5/7-point Dirichlet eigenvalues 4 sum sin^2(j pi / (2(N+1))) (the
    unscaled stencil of Sec. 3.2)."""
    for N, d in ((9, 2), (5, 3)):
        csr = si.laplacian_2d(N) if d == 2 else si.laplacian_3d(N)
        A = sp.csr_matrix((csr[2], csr[1], csr[0]), shape=(csr[3],) * 2).toarray()
        l1 = 4 * np.sin(np.arange(1, N + 1) * np.pi / (2 * (N + 1))) ** 2
        grid = np.add.outer(l1, l1) if d == 2 else np.add.outer(np.add.outer(l1, l1), l1)
        assert np.allclose(np.sort(np.linalg.eigvalsh(A)), np.sort(grid.ravel()), atol=1e-12)


def test_shift_gives_requested_negative_count():
    N = 8
    s = si.shift_for_negative_count_3d(N, 4)
    csr = si.laplacian_3d(N, s)
    A = sp.csr_matrix((csr[2], csr[1], csr[0]), shape=(csr[3],) * 2).toarray()
    assert int((np.linalg.eigvalsh(A) < 0).sum()) == 4


# ------------------------------------------------------ classification, order

def test_classification_hand_drawn_6x6():
    """6x6 grid, 2x2 boxes of 3x3: a node is a local interface node iff it
    has a neighbour in another box (Sec. 2.1) -- lines x in {2,3} or
    y in {2,3}, drawn by hand."""
    csr = si.laplacian_2d(6)
    part = si.box_partition_2d(6, 2, 2)
    A = sp.csr_matrix((csr[2], csr[1], csr[0]), shape=(36, 36))
    iface, _ = O.classify(A, part, 4)
    expect = np.array([[x in (2, 3) or y in (2, 3) for x in range(6)] for y in range(6)]).ravel()
    assert (iface == expect).all()
    perm, off_b, off_y, _ = O.dd_ordering(A, part, 4)
    # box 0 interior: (0,0),(1,0),(0,1),(1,1)
    assert perm[:4].tolist() == [0, 1, 6, 7]
    assert off_b.tolist() == [0, 4, 8, 12, 16]
    assert off_y.tolist() == [0, 5, 10, 15, 20, 20]
    # interface of box 0 in ascending index: (2,0),(2,1),(0,2),(1,2),(2,2)
    assert perm[16:21].tolist() == [2, 8, 12, 13, 14]


def test_separator_labels_are_interface_and_neighbours_interior():
    A, part = si.separator_model(5, 3)
    M = sp.csr_matrix((A[2], A[1], A[0]), shape=(A[3],) * 2)
    iface, _ = O.classify(M, part, 2)
    assert iface.sum() == 5 and (iface == (part < 0)).all()


def test_multicolor_is_a_proper_colouring():
    pr = si.make_config("lap3d_64", N=16, boxes=2)
    A = pr.scipy()
    perm, off_b, off_y, colors = O.dd_ordering(A, pr.part, pr.nparts, "multicolor")
    m = off_b[-1]
    C = A[perm[m:]][:, perm[m:]].tocoo()
    assert (colors[C.row[C.row != C.col]] != colors[C.col[C.row != C.col]]).all()
    assert (np.diff(colors) >= 0).all()


# --------------------------------------------------------------- factorisations

def test_ic0_defining_property_and_tridiagonal_exactness():
    pr = si.make_config("lap3d_64", N=8, boxes=2)
    A = pr.scipy()
    F = O.factorize(sp.tril(A).tocsr() + sp.triu(A, 1).tocsr(), "ic0")
    L = sp.csr_matrix((F.v, F.ci, F.rp), shape=A.shape).toarray()
    LLt = L @ L.T
    Ad = A.toarray()
    mask = np.tril(Ad != 0)
    assert np.abs((LLt - Ad)[mask]).max() < 1e-13
    # IC(0) of a tridiagonal matrix has no dropped fill: it is the Cholesky factor
    T = sp.csr_matrix(sp.diags([-np.ones(29), 2.5 * np.ones(30), -np.ones(29)], [-1, 0, 1]))
    F1 = O.factorize(T, "ic0")
    L1 = sp.csr_matrix((F1.v, F1.ci, F1.rp), shape=T.shape).toarray()
    assert np.allclose(L1, np.linalg.cholesky(T.toarray()), atol=1e-14)


def test_ildlt0_defining_property_on_indefinite_pattern():
    csr = si.laplacian_3d(6, shift=5.5)
    A = sp.csr_matrix((csr[2], csr[1], csr[0]), shape=(csr[3],) * 2)
    F = O.factorize(A, "ildlt0")
    M = sp.csr_matrix((F.v, F.ci, F.rp), shape=A.shape).toarray()
    D = np.diag(M).copy()
    L = np.tril(M, -1) + np.eye(A.shape[0])
    Ad = A.toarray()
    mask = np.tril(Ad != 0)
    assert np.abs((L @ np.diag(D) @ L.T - Ad)[mask]).max() < 1e-12
    assert (D < 0).any()


def test_triangular_sweeps_match_dense_solves():
    pr = si.make_config("lap3d_64", N=8, boxes=2)
    A = pr.scipy()
    rng = np.random.default_rng(3)
    for kind in ("ic0", "ildlt0", "chol"):
        F = O.factorize(A, kind)
        L = F.dense_lower(0, A.shape[0])
        if kind == "ildlt0":
            D = np.diag(L).copy()
            L = np.tril(L, -1) + np.eye(A.shape[0])
        b = rng.standard_normal(A.shape[0])
        assert np.allclose(F.lower(b), sla.solve_triangular(L, b, lower=True), atol=1e-12)
        assert np.allclose(F.upper(b), sla.solve_triangular(L, b, lower=True, trans="T"), atol=1e-12)
        if kind == "chol":
            assert np.allclose(L @ L.T, A.toarray(), atol=1e-12)
            assert np.allclose(F.solve(b), np.linalg.solve(A.toarray(), b), atol=1e-10)


def test_exact_B_blocks_are_31x31_dirichlet_laplacians():
    """In the 64x64 / 2x2 configuration each interior block B_i is the
    5-point Laplacian of a 31x31 Dirichlet grid (closed-form spectrum)."""
    pr = si.make_config("lap2d_64")
    P = O.setup(pr.csr, pr.part, pr.nparts, 0, b_fact="chol", c_fact="chol")
    assert P.m == 4 * 961 and P.s == 252
    B0 = P.Ap[:961][:, :961].toarray()
    l1 = 4 * np.sin(np.arange(1, 32) * np.pi / 64) ** 2
    assert np.allclose(np.sort(np.linalg.eigvalsh(B0)), np.sort(np.add.outer(l1, l1).ravel()), atol=1e-11)


# -------------------------------------------------- operator H and spectrum

def test_G_matches_dense_H_and_lemma_bounds():
    """eq. H by dense algebra; Lemma (A SPD => 0 <= lambda(H) < 1)."""
    csr, part, p = _tiny(14)
    P = O.setup(csr, part, p, 0, b_fact="chol", c_fact="chol")
    H, _ = _dense_H(P)
    rng = np.random.default_rng(0)
    v = rng.standard_normal(P.s)
    assert np.allclose(P.G(v), H @ v, atol=1e-12)
    ev = np.linalg.eigvalsh(H)
    assert ev.min() > -1e-12 and ev.max() < 1.0


def test_lanczos_ritz_values_match_dense_spectrum_and_residual_bound():
    """Lanczos on H (Sec. 5.1): converged top Ritz values equal dense
    eigenvalues; Ritz residual ||H u - lambda u|| = beta_m |e_m^T y|."""
    pr = si.make_config("lap2d_64")
    P = O.setup(pr.csr, pr.part, pr.nparts, pr.k, pr.lanczos_steps, "chol", "chol", v0=pr.v0())
    H, _ = _dense_H(P)
    ev = np.sort(np.linalg.eigvalsh(H))[::-1]
    assert np.all(P.ritz < 1.0) and P.ritz.min() > -1e-12
    mm = P.steps
    T = np.diag(P.alpha) + np.diag(P.beta[:mm - 1], 1) + np.diag(P.beta[:mm - 1], -1)
    tev, Y = np.linalg.eigh(T)
    tev, Y = tev[::-1], Y[:, ::-1]
    near = np.abs(P.ritz[:, None] - ev[None, :]).min(axis=1)
    for i in range(pr.k + 1):
        bound = P.beta[-1] * abs(Y[-1, i])        # ||H u_i - lambda_i u_i||
        if i < pr.k:
            res = np.linalg.norm(H @ P.U[:, i] - P.lam[i] * P.U[:, i])
            assert abs(res - bound) < 1e-10
        # for symmetric H an eigenvalue lies within the residual of a Ritz value
        assert near[i] <= bound + 1e-12
    assert abs(P.ritz[0] - ev[0]) < 1e-12


def test_full_lanczos_equals_dense_spectrum_with_breakdown():
    """With steps >= s and distinct eigenvalues, Lanczos spans the space and
    every eigenvalue of H is recovered; it stops on beta ~ 0."""
    A, part = si.separator_model(24, 10)
    P = O.setup(A, part, 2, 8, 60, "chol", "chol")
    H, _ = _dense_H(P)
    assert P.steps == P.s == 24
    assert np.allclose(np.sort(P.ritz), np.sort(np.linalg.eigvalsh(H)), atol=1e-12)


# ------------------------------------------------------ the preconditioner

def _dense_lowrank(P, k, theta_mode="lambda_k1"):
    H, L = _dense_H(P)
    lam, U = np.linalg.eigh(H)
    lam, U = lam[::-1], U[:, ::-1]
    theta = lam[k] if (theta_mode == "lambda_k1" and k < len(lam)) else 0.0
    if theta_mode == "lambda_s":
        theta = lam[-1]
    return H, L, lam, U, theta


def test_P1_full_rank_exact_solves_make_M_equal_A():
    """k = s with exact B and C: S~ = S, so M = A (eq. M with eq. Sinv) and
    M^{-1} A x = x; PCG converges in one iteration."""
    csr, part, p = _tiny(12)
    P0 = O.setup(csr, part, p, 0, b_fact="chol", c_fact="chol")
    H, L, lam, U, _ = _dense_lowrank(P0, P0.s)
    P = O.setup(csr, part, p, 0, b_fact="chol", c_fact="chol", lowrank=(U, lam, 0.0))
    rng = np.random.default_rng(1)
    x = rng.uniform(-1, 1, P.A.shape[0])
    assert np.abs(P.apply(P.A @ x) - x).max() < 1e-11
    res = O.solve(P, P.A @ x, "pcg")
    assert res.iters == 1 and res.true_relres < 1e-12
    res = O.solve(P, P.A @ x, "fgmres")
    assert res.iters == 1 and res.true_relres < 1e-12


def test_P6_skt_form_equals_tildeSinv_and_schur_bruteforce():
    """Interface part of M^{-1}(0; g) equals S~^{-1} g with S~^{-1} built
    from ALL eigenvectors by eq. tildeSinv (Lambda~ = Lambda_k, theta on the
    tail, eq. main); the oracle uses only k of them (Prop. skt).  With
    k = s it equals S^{-1} g, S = C - E^T B^{-1} E formed densely (eq. Schur)."""
    csr, part, p = _tiny(14)
    P0 = O.setup(csr, part, p, 0, b_fact="chol", c_fact="chol")
    _, B, E, C = _dense_blocks(P0)
    S = C - E.T @ np.linalg.solve(B, E)
    for k in (3, 9):
        H, L, lam, U, theta = _dense_lowrank(P0, k)
        P = O.setup(csr, part, p, 0, b_fact="chol", c_fact="chol",
                    lowrank=(U[:, :k], lam[:k], theta))
        lt = np.concatenate([lam[:k], np.full(P.s - k, theta)])
        Linv = np.linalg.inv(L)
        St_inv = Linv.T @ U @ np.diag(1.0 / (1.0 - lt)) @ U.T @ Linv
        g = np.random.default_rng(k).standard_normal(P.s)
        r = np.concatenate([np.zeros(P.m), g])
        out = P.apply_dd(r)
        assert np.allclose(out[P.m:], St_inv @ g, atol=1e-11)
        assert np.allclose(out[:P.m], -np.linalg.solve(B, E @ out[P.m:]), atol=1e-11)
    H, L, lam, U, _ = _dense_lowrank(P0, P0.s)
    P = O.setup(csr, part, p, 0, b_fact="chol", c_fact="chol", lowrank=(U, lam, 0.0))
    g = np.random.default_rng(5).standard_normal(P.s)
    out = P.apply_dd(np.concatenate([np.zeros(P.m), g]))
    assert np.allclose(out[P.m:], np.linalg.solve(S, g), atol=1e-10)


def _spectrum_MinvA(P):
    n = P.A.shape[0]
    Ad = P.A.toarray()
    MA = np.column_stack([P.apply(Ad[:, j]) for j in range(n)])
    return np.sort(np.linalg.eigvals(MA).real)


@pytest.mark.parametrize("theta_mode", ["lambda_k1", "lambda_s", "zero"])
def test_P2_P7_spectrum_of_preconditioned_matrix(theta_mode):
    """eig(M^{-1}A) = {1}^(m+k) U {(1 - lambda_i)/(1 - theta)}_{i>k}
    (Prop. eigSS with eq. main; theta = 0 is eq. Lambda-1), and
    kappa(S S~^{-1}) = (1-lambda_s)/(1-lambda_{k+1}) for theta = lambda_{k+1}
    (Prop. kappa) and for theta = lambda_s alike (the condition number is
    the same for every theta in [lambda_s, lambda_{k+1}], Sec. 4)."""
    csr, part, p = _tiny(10)
    P0 = O.setup(csr, part, p, 0, b_fact="chol", c_fact="chol")
    k = 5
    H, L, lam, U, theta = _dense_lowrank(P0, k, theta_mode)
    P = O.setup(csr, part, p, 0, b_fact="chol", c_fact="chol", lowrank=(U[:, :k], lam[:k], theta))
    got = _spectrum_MinvA(P)
    expect = np.sort(np.concatenate([np.ones(P.m + k), (1 - lam[k:]) / (1 - theta)]))
    assert np.allclose(got, expect, atol=1e-9)
    if theta_mode in ("lambda_k1", "lambda_s"):
        sig = (1 - lam[k:]) / (1 - theta)
        kappa = max(sig.max(), 1.0) / min(sig.min(), 1.0)
        assert math.isclose(kappa, (1 - lam[-1]) / (1 - lam[k]), rel_tol=1e-12)


@pytest.mark.parametrize("eps", [0.3, 1.0])
def test_Lambda2_eps_spectrum_of_preconditioned_matrix(eps):
    """eq. Lambda-2: lambda~_i = 1 - (1 - lambda_i)/eps for i <= k and 0
    beyond make eig(S S~^{-1}) = {eps}^k U {1 - lambda_i}_{i>k}, so
    eig(M^{-1}A) = {1}^m U {eps}^k U {1 - lambda_i}_{i>k}; eps = 1 is
    eq. Lambda-1 (theta = 0)."""
    csr, part, p = _tiny(10)
    P0 = O.setup(csr, part, p, 0, b_fact="chol", c_fact="chol")
    k = 5
    H, L, lam, U, _ = _dense_lowrank(P0, k, "zero")
    P = O.setup(csr, part, p, 0, b_fact="chol", c_fact="chol", lowrank=(U[:, :k], lam[:k], 0.0),
                theta_mode="eps", eps=eps)
    got = _spectrum_MinvA(P)
    expect = np.sort(np.concatenate([np.ones(P.m), np.full(k, eps), 1 - lam[k:]]))
    assert np.allclose(got, expect, atol=1e-9)
    if eps == 1.0:
        Pz = O.setup(csr, part, p, 0, b_fact="chol", c_fact="chol", lowrank=(U[:, :k], lam[:k], 0.0),
                     theta_mode="zero")
        r = np.random.default_rng(3).standard_normal(P.A.shape[0])
        assert np.allclose(P.apply(r), Pz.apply(r), rtol=1e-13, atol=1e-13)


def test_condk_rank_selection():
    """eq. condk: with cond_K = K the rank is the number of eigenvalues of H
    above 1 - 1/K, and then kappa(S S~^{-1}) = (1 - lambda_s)/(1 - lambda_{k+1})
    <= K (theta = lambda_{k+1}).  Simple spectrum (random coefficients,
    uneven cuts) and as many Lanczos steps as interface nodes, so the Ritz
    values are the eigenvalues."""
    N = 14
    rng = np.random.default_rng(4)
    csr = si.diffusion_2d(N, np.exp(rng.standard_normal((N + 2, N + 2))))
    part = si.random_cuts_2d(N, 2, 2, 5)
    P0 = O.setup(csr, part, 4, 0, b_fact="chol", c_fact="chol")
    H, _ = _dense_H(P0)
    ev = np.sort(np.linalg.eigvalsh(H))[::-1]
    for K in (2.0, 5.0):
        want = int(np.sum(ev > 1 - 1 / K))
        P = O.setup(csr, part, 4, 20, P0.s, b_fact="chol", c_fact="chol", cond_K=K,
                    v0=si.lanczos_start(csr[3], 9))
        assert want < 20
        assert P.k == want
        assert np.allclose(P.ritz[:want + 1], ev[:want + 1], rtol=1e-9, atol=1e-12)
        sig = (1 - ev[want:]) / (1 - P.theta)
        kappa = max(sig.max(), 1.0) / min(sig.min(), 1.0)
        assert kappa <= K * (1 + 1e-9)
        assert math.isclose(kappa, (1 - ev[-1]) / (1 - ev[want]), rel_tol=1e-8)
        # eig(M^{-1}A) = {1}^(m+k) U {(1 - lambda_i)/(1 - theta)}_{i>k}
        spec = _spectrum_MinvA(P)
        assert np.allclose(spec, np.sort(np.concatenate([np.ones(P.m + want), sig])), atol=1e-7)


def test_theta_lambda_s_from_lanczos():
    """theta = lambda_s taken from Lanczos run to the full interface size is
    the smallest eigenvalue of H, and the condition number of S S~^{-1} is
    (1 - lambda_s)/(1 - lambda_{k+1}), as for theta = lambda_{k+1}.  The
    separator model of Sec. 3.2 has lambda_s > 0 (a vertex-based split
    usually has a singular H, lambda_s = 0, where this is eq. Lambda-1)."""
    A, part = si.separator_model(20, 10)
    P0 = O.setup(A, part, 2, 0, b_fact="chol", c_fact="chol")
    H, _ = _dense_H(P0)
    ev = np.sort(np.linalg.eigvalsh(H))[::-1]
    assert ev[-1] > 1e-3
    k = 6
    P = O.setup(A, part, 2, k, P0.s, b_fact="chol", c_fact="chol", theta_mode="lambda_s",
                v0=si.lanczos_start(A[3], 9))
    assert math.isclose(P.theta, ev[-1], rel_tol=1e-9)
    spec = _spectrum_MinvA(P)
    sig = (1 - ev[k:]) / (1 - P.theta)
    assert np.allclose(spec, np.sort(np.concatenate([np.ones(P.m + k), sig])), atol=1e-7)
    assert math.isclose(spec.max() / spec.min(), (1 - ev[-1]) / (1 - ev[k]), rel_tol=1e-7)


def test_grow_by_deflation_finds_the_next_eigenpairs():
    """Sec. 5.3: starting from the exact top-3 eigenpairs of H, deflated
    Lanczos run over the whole complement returns lambda_4..lambda_7 and
    keeps the old vectors; the grown preconditioner has the spectrum of the
    rank-7 one, {1}^(m+7) U {(1 - lambda_i)/(1 - lambda_8)}_{i>7}
    (Prop. eigSS).  Simple spectrum, so single-vector Lanczos sees every
    eigenvalue once."""
    N = 14
    rng = np.random.default_rng(4)
    csr = si.diffusion_2d(N, np.exp(rng.standard_normal((N + 2, N + 2))))
    part = si.random_cuts_2d(N, 2, 2, 5)
    P0 = O.setup(csr, part, 4, 0, b_fact="chol", c_fact="chol")
    H, L, lam, U, _ = _dense_lowrank(P0, 3)
    P = O.setup(csr, part, 4, 0, b_fact="chol", c_fact="chol", lowrank=(U[:, :3], lam[:3], lam[3]))
    v0 = si.lanczos_start(csr[3], 9)[P.perm[P.m:]]
    O.grow_lowrank(P, 4, P.s - 3, v0)
    assert P.k == 7
    assert np.array_equal(P.U[:, :3], U[:, :3])
    assert np.allclose(P.lam, lam[:7], rtol=1e-9, atol=1e-12)
    assert math.isclose(P.theta, lam[7], rel_tol=1e-9)
    assert np.allclose(P.U.T @ P.U, np.eye(7), atol=1e-10)
    assert np.allclose(np.abs(np.sum(P.U[:, 3:] * U[:, 3:7], axis=0)), 1.0, atol=1e-8)
    spec = _spectrum_MinvA(P)
    expect = np.sort(np.concatenate([np.ones(P.m + 7), (1 - lam[7:]) / (1 - lam[7])]))
    assert np.allclose(spec, expect, atol=1e-7)
    # a start vector inside span(U_k) is refused
    with pytest.raises(O.OracleError):
        O.grow_lowrank(P, 2, 10, P.U[:, 0] + 0.5 * P.U[:, 5])


def test_grow_from_nothing_is_plain_lanczos():
    """With no captured directions deflated Lanczos is the plain build
    (growth always reorthogonalises fully)."""
    csr, part, p = _tiny(12)
    v0 = si.lanczos_start(csr[3], 4)
    A = O.setup(csr, part, p, 5, 25, b_fact="ic0", c_fact="ic0", v0=v0, reorth="full")
    B = O.setup(csr, part, p, 0, b_fact="ic0", c_fact="ic0")
    O.grow_lowrank(B, 5, 25, v0[B.perm[B.m:]])
    assert B.k == A.k and np.array_equal(B.lam, A.lam) and B.theta == A.theta
    assert np.array_equal(B.U, A.U)


def _ritz_and_bounds(alpha, beta):
    mm = len(alpha)
    T = np.diag(alpha) + np.diag(beta[:mm - 1], 1) + np.diag(beta[:mm - 1], -1)
    ev, Y = np.linalg.eigh(T)
    return ev[::-1], beta[-1] * np.abs(Y[-1, ::-1])


def test_partial_reorthogonalisation_keeps_semiorthogonality():
    """Sec. 5.1: without reorthogonalisation the Lanczos vectors lose
    orthogonality once Ritz values converge; the partial scheme keeps
    max |V^T V - I| below sqrt(eps) while cleaning only a few steps, and its
    converged Ritz values equal those of full reorthogonalisation (semi-
    orthogonality makes T_m the projection of H up to O(eps ||H||))."""
    pr = si.make_config("diffusion2d_1024", N=96, boxes=4)
    P = O.setup(pr.csr, pr.part, pr.nparts, 0, b_fact=pr.b_fact, c_fact=pr.c_fact)
    v0 = pr.v0()[P.perm[P.m:]]
    steps = 150
    # no reorthogonalisation at all: the plain three-term recurrence
    Vp = np.zeros((P.s, steps))
    Vp[:, 0] = v0 / np.linalg.norm(v0)
    bprev = 0.0
    for j in range(steps - 1):
        w = P.G(Vp[:, j])
        a = Vp[:, j] @ w
        w = w - a * Vp[:, j] - (bprev * Vp[:, j - 1] if j else 0.0)
        bprev = np.linalg.norm(w)
        Vp[:, j + 1] = w / bprev
    assert np.abs(Vp.T @ Vp - np.eye(steps)).max() > 1e-4
    st = {}
    V, al, be = O.lanczos_pro(P.G, v0, steps, st)
    assert V.shape[1] == steps
    assert np.abs(V.T @ V - np.eye(steps)).max() <= math.sqrt(O.EPS)
    assert 0 < len(st["reorth"]) < steps // 4
    Vf, af, bf = O.lanczos(P.G, v0, steps)
    ep, bp = _ritz_and_bounds(al, be)
    ef, bfd = _ritz_and_bounds(af, bf)
    conv = (bp[:20] <= 1e-9) & (bfd[:20] <= 1e-9)
    assert conv.sum() >= 3
    assert np.all(np.abs(ep[:20] - ef[:20])[conv] <= 1e-10 * np.abs(ef[:20])[conv])


def test_partial_reorthogonalisation_spectrum_exact_problem():
    """With exact B and C solves and as many steps as interface nodes, the
    partial scheme's Ritz values are the eigenvalues of H (simple spectrum)
    and the rank-k preconditioner has the spectrum of Prop. eigSS."""
    N = 14
    rng = np.random.default_rng(4)
    csr = si.diffusion_2d(N, np.exp(rng.standard_normal((N + 2, N + 2))))
    part = si.random_cuts_2d(N, 2, 2, 5)
    P0 = O.setup(csr, part, 4, 0, b_fact="chol", c_fact="chol")
    H, _ = _dense_H(P0)
    ev = np.sort(np.linalg.eigvalsh(H))[::-1]
    k = 6
    P = O.setup(csr, part, 4, k, P0.s, b_fact="chol", c_fact="chol", v0=si.lanczos_start(csr[3], 9),
                reorth="partial")
    assert np.allclose(P.ritz[:k + 1], ev[:k + 1], rtol=1e-9, atol=1e-12)
    spec = _spectrum_MinvA(P)
    sig = (1 - ev[k:]) / (1 - P.theta)
    assert np.allclose(spec, np.sort(np.concatenate([np.ones(P.m + k), sig])), atol=1e-7)


def _dense_threshold_factor(A, tau, ldl):
    """Dense left-looking factorisation with the threshold rule written out
    on full matrices (independent of the oracle's sparse loops)."""
    n = A.shape[0]
    L = np.zeros((n, n))
    d = np.zeros(n)
    for j in range(n):
        w = A[j:, j].copy()
        nrm = np.abs(A[j:, j]).sum()
        for k in range(j):
            if L[j, k] != 0.0:
                f = L[j, k] * d[k] if ldl else L[j, k]
                w -= L[j:, k] * f
        d[j] = w[0] if ldl else np.sqrt(w[0])
        keep = np.abs(w[1:]) >= tau * nrm
        L[j + 1:, j] = np.where(keep, w[1:] / d[j], 0.0)
    return L, d


@pytest.mark.parametrize("kind", ["ict", "ildlt"])
def test_threshold_factors(kind):
    """ICT / ILDLT (Sec. 6 local solvers): no dropping is the exact
    factorisation (L L^T = M, L D L^T = M); an infinite tolerance keeps the
    diagonal only; the kept pattern and values follow the dense form of the
    rule (1-norm of the column of tril(M), updated values compared); with
    no fill possible (tridiagonal) they equal IC(0) / ILDL(0)."""
    import scipy.sparse as sp
    ldl = kind == "ildlt"
    rng = np.random.default_rng(11)
    N = 7
    csr = si.diffusion_2d(N, np.exp(rng.standard_normal((N + 2, N + 2))))
    M = sp.csr_matrix((csr[2], csr[1], csr[0]), shape=(csr[3], csr[3]))
    Md = M.toarray()

    def dense(F):
        Lf = sp.csr_matrix((F.v, F.ci, F.rp), shape=M.shape).toarray()
        dd = np.diag(Lf).copy()
        return Lf - np.diag(dd), dd

    Ls, dd = dense(O.factorize(M, kind, droptol=0.0))
    if ldl:
        Lu = Ls + np.eye(len(dd))
        assert np.abs(Lu @ np.diag(dd) @ Lu.T - Md).max() <= 1e-13 * np.abs(Md).max()
    else:
        Lf = Ls + np.diag(dd)
        assert np.allclose(Lf, np.linalg.cholesky(Md), rtol=1e-12, atol=1e-13)
    Ls, dd = dense(O.factorize(M, kind, droptol=1e300))
    assert not Ls.any()
    assert np.allclose(dd, np.diag(Md) if ldl else np.sqrt(np.diag(Md)), rtol=0, atol=0)
    for tau in (0.02, 0.1):
        Ls, dd = dense(O.factorize(M, kind, droptol=tau))
        Lr, dr = _dense_threshold_factor(Md, tau, ldl)
        assert np.array_equal(Ls != 0.0, np.tril(Lr, -1) != 0.0)
        assert np.allclose(Ls, np.tril(Lr, -1), rtol=1e-13, atol=1e-15)
        assert np.allclose(dd, dr, rtol=1e-13)
    T = si.laplacian_2d(1, Ny=30)
    T = sp.csr_matrix((T[2], T[1], T[0]), shape=(T[3], T[3]))
    Ft = O.factorize(T, kind, droptol=1e-12)
    F0 = O.factorize(T, "ildlt0" if ldl else "ic0")
    assert np.array_equal(Ft.ci, F0.ci) and np.allclose(Ft.v, F0.v, rtol=1e-15, atol=0)


def test_threshold_factors_without_dropping_give_exact_solves():
    """ICT for B and C with no dropping makes the SLR apply that of exact
    solves (eq. M with exact B and C)."""
    csr, part, p = _tiny(10)
    Pe = O.setup(csr, part, p, 5, 0, b_fact="chol", c_fact="chol", v0=si.lanczos_start(csr[3], 3))
    Pt = O.setup(csr, part, p, 0, b_fact="ict", c_fact="ict", droptol=0.0, lowrank=(Pe.U, Pe.lam, Pe.theta))
    r = np.random.default_rng(2).standard_normal(csr[3])
    assert np.allclose(Pt.apply(r), Pe.apply(r), rtol=1e-10, atol=1e-12)


def test_P3prime_inertia_counts_negative_eigenvalues():
    """Indefinite A with SPD B (exact solves): by Sylvester's law on
    eq. Schur, #{lambda(H) > 1} = #negative eigenvalues of A."""
    N = 10
    s = si.shift_for_negative_count_3d(N, 4)
    csr = si.laplacian_3d(N, s)
    part = si.box_partition_3d(N, 2)
    P = O.setup(csr, part, 8, 0, b_fact="chol", c_fact="chol")
    H, _ = _dense_H(P)
    A = P.A.toarray()
    nneg = int((np.linalg.eigvalsh(A) < 0).sum())
    assert nneg == 4
    assert int((np.linalg.eigvalsh(H) > 1).sum()) == nneg
    # the oracle's Lanczos sees them among its largest Ritz values
    Pl = O.setup(csr, part, 8, 8, 40, "chol", "chol", v0=si.lanczos_start(csr[3], 3))
    assert int((Pl.ritz > 1).sum()) >= 1
    assert np.all(np.abs(Pl.ritz[:3] - np.sort(np.linalg.eigvalsh(H))[::-1][:3]) < 1e-8)


def test_P4_two_domain_closed_form_matches_bruteforce():
    """eq. gammak0: eigenvalues of S^{-1} - C^{-1} in the separator model
    (Prop. of Sec. 3.2, eq. etak0) against dense brute force."""
    nx, ny = 20, 10
    A, part = si.separator_model(nx, ny)
    P = O.setup(A, part, 2, 0, b_fact="chol", c_fact="chol")
    _, B, E, C = _dense_blocks(P)
    S = C - E.T @ np.linalg.solve(B, E)
    got = np.sort(np.linalg.eigvalsh(np.linalg.inv(S) - np.linalg.inv(C)))
    kk = np.arange(1, nx + 1)
    eta = 1 + 2 * np.sin(kk * np.pi / (2 * (nx + 1))) ** 2
    th = np.arccosh(eta)
    gamma = np.sinh(ny * th) / (eta * (np.sinh((ny + 2) * th) - np.sinh(ny * th)))
    assert np.allclose(got, np.sort(gamma), rtol=1e-12, atol=1e-14)


def _separator_lambda(nx, ny):
    kk = np.arange(1, nx + 1)
    eta = 1 + 2 * np.sin(kk * np.pi / (2 * (nx + 1))) ** 2
    th = np.arccosh(eta)
    gamma = np.sinh(ny * th) / (eta * (np.sinh((ny + 2) * th) - np.sinh(ny * th)))
    zeta = 2 * eta * gamma
    return np.sort(zeta / (1 + zeta))[::-1]


def test_P4_fig_kappa_printed_values_from_closed_form():
    """The values printed with the kappa(theta) figure (Sec. 4) follow from
    the two-domain closed form: lambda(H) = zeta/(1+zeta), zeta = 2 eta gamma."""
    g = json.load(open(os.path.join(GOLDEN, "fig_kappa.json")))
    lam = _separator_lambda(g["nx"], g["ny"])
    k = g["k"]
    assert round(lam[-1], 5) == g["lambda_s"]
    assert round(lam[k], 5) == g["lambda_k1"]
    assert round((1 - lam[-1]) / (1 - lam[k]), 4) == g["kappa"]


@pytest.mark.slow
def test_P4_fig_kappa_through_oracle_lanczos():
    """The oracle's own Lanczos on the 256 x 513 separator grid, exact
    solves, k = 64, 5k = 320 >= s steps, reproduces the printed values."""
    g = json.load(open(os.path.join(GOLDEN, "fig_kappa.json")))
    A, part = si.separator_model(g["nx"], g["ny"])
    P = O.setup(A, part, 2, g["k"], 0, "chol", "chol", v0=si.lanczos_start(A[3], 7))
    assert P.steps == P.s == g["nx"]
    lam_s = P.ritz[-1]
    kappa = (1 - lam_s) / (1 - P.theta)
    assert round(lam_s, 5) == g["lambda_s"]
    assert round(P.theta, 5) == g["lambda_k1"]
    assert round(kappa, 4) == g["kappa"]
    assert np.allclose(P.ritz, _separator_lambda(g["nx"], g["ny"]), atol=1e-11)


# ------------------------------------------- minimum degree ordering of B_i

def _exact_fill(M):
    """nnz of the exact Cholesky factor (dense, |l_ij| > 1e-13 max|l|)."""
    L = np.linalg.cholesky(M.toarray())
    return int(np.sum(np.abs(L) > 1e-13 * np.abs(L).max()))


def test_min_degree_order_gives_no_fill_on_trees_and_eliminates_star_leaves_first():
    """Sec. 6 orders each B_i by (approximate) minimum degree.  Two exact
    consequences of the minimum degree rule: on a tree some leaf always has
    degree 1, so the order eliminates without any fill (the factor of the
    permuted matrix has exactly the pattern of its lower triangle), while a
    random labelling in natural order does fill; on a star the leaves go
    first in index order until one is left."""
    rng = np.random.default_rng(41)
    n = 300
    parent = [int(rng.integers(0, i)) for i in range(1, n)]
    lab = rng.permutation(n)
    rows = np.concatenate([lab[1:], lab[parent]])
    cols = np.concatenate([lab[parent], lab[1:]])
    T = sp.csr_matrix((-np.ones(2 * (n - 1)), (rows, cols)), shape=(n, n))
    M = (T + sp.diags(np.asarray(-T.sum(axis=1)).ravel() + 1.0)).tocsr()
    o = O.min_degree_order(M)
    assert sorted(o.tolist()) == list(range(n))
    Mp = M[o][:, o].tocsr()
    assert _exact_fill(Mp) == sp.tril(Mp).nnz
    assert _exact_fill(M) > sp.tril(M).nnz
    k = 40
    S = sp.lil_matrix((k, k))
    for i in range(1, k):
        S[0, i] = S[i, 0] = -1.0
    S.setdiag([float(k)] + [2.0] * (k - 1))
    # when one leaf is left, it and the centre both have degree 1: the
    # smaller index (the centre) goes first
    assert O.min_degree_order(S.tocsr()).tolist() == list(range(1, k - 1)) + [0, k - 1]


def test_min_degree_order_reduces_fill_and_exact_threshold_factor_in_that_order():
    """On a 31x31 Dirichlet Laplacian the exact factor in minimum degree
    order has far less fill than in natural (banded) order; with drop
    tolerance 0 the ICT and ILDLT factors in that order are the exact
    factors of the permuted matrix."""
    csr = si.laplacian_2d(31)
    A = sp.csr_matrix((csr[2], csr[1], csr[0]), shape=(csr[3], csr[3]))
    o = O.min_degree_order(A)
    Ap = A[o][:, o].tocsr()
    assert _exact_fill(Ap) < 0.6 * _exact_fill(A)
    F = O.factorize(Ap, "ict", None, "B", 0.0)
    Ld = sp.csr_matrix((F.v, F.ci, F.rp), shape=Ap.shape).toarray()
    assert np.allclose(Ld, np.linalg.cholesky(Ap.toarray()), atol=1e-12)
    Fl = O.factorize(Ap, "ildlt", None, "B", 0.0)
    x = np.random.default_rng(3).uniform(-1, 1, Ap.shape[0])
    assert np.allclose(Fl.solve(x), np.linalg.solve(Ap.toarray(), x), atol=1e-10)


def test_mindeg_interior_order_in_the_dd_ordering():
    """b_order='mindeg' only reorders inside each subdomain's interior: the
    groups (interiors by subdomain, interface) are those of the natural DD
    ordering, and the preconditioner with exact solves still makes
    M^{-1} A = I at full rank (P1)."""
    csr, part, p = _tiny(12)
    A = sp.csr_matrix((csr[2], csr[1], csr[0]), shape=(csr[3], csr[3]))
    pn, ob, oy, _ = O.dd_ordering(A, part, p)
    pm, ob2, oy2, _ = O.dd_ordering(A, part, p, b_order="mindeg")
    assert (ob == ob2).all() and (oy == oy2).all()
    for a, b in zip(ob[:-1], ob[1:]):
        assert sorted(pm[a:b]) == sorted(pn[a:b])
    assert (pm[ob[-1]:] == pn[ob[-1]:]).all()
    assert not (pm == pn).all()
    P0 = O.setup(csr, part, p, 0, b_fact="chol", c_fact="chol", b_order="mindeg")
    H, L, lam, U, _ = _dense_lowrank(P0, P0.s)
    P = O.setup(csr, part, p, 0, b_fact="chol", c_fact="chol", b_order="mindeg", lowrank=(U, lam, 0.0))
    x = np.random.default_rng(5).uniform(-1, 1, A.shape[0])
    assert np.abs(P.apply(A @ x) - x).max() < 1e-10


# ------------------------------------------------ HID ordering of C

@pytest.mark.parametrize("dim,N,q", [(3, 16, 2), (3, 18, 3), (3, 20, 4), (2, 40, 4), (2, 41, 5)])
def test_hid_order_makes_the_leading_block_of_C_block_diagonal(dim, N, q):
    """Sec. 5.2: for a recursive treatment C must have A's structure, its
    leading block block diagonal, which the HID ordering provides.  With
    the oracle's HID reading, the level-1 part of C splits into connected
    pieces that are contiguous in the order (so that block is block
    diagonal), one per pair of boxes sharing a face (3 q^2 (q-1) in 3-D,
    2 q (q-1) in 2-D);
    the interiors keep their order and the interface is a permutation of
    the natural one."""
    import scipy.sparse.csgraph  # noqa: F401
    csr = si.laplacian_3d(N) if dim == 3 else si.laplacian_2d(N)
    part = si.box_partition_3d(N, q) if dim == 3 else si.box_partition_2d(N, q, q)
    A = sp.csr_matrix((csr[2], csr[1], csr[0]), shape=(csr[3], csr[3]))
    pn, ob, oy, _ = O.dd_ordering(A, part, q ** dim)
    ph, ob2, _, lev = O.dd_ordering(A, part, q ** dim, c_order="hid")
    m = int(ob[-1])
    assert (ph[:m] == pn[:m]).all() and sorted(ph[m:]) == sorted(pn[m:])
    assert np.all(np.diff(lev) >= 0) and lev.min() == 2
    # the level-1 block: its connected components are the faces (a closed
    # count), and each is one contiguous range of the order (so the block
    # is block diagonal in this order)
    y = ph[m:]
    lvl1 = y[lev == 2]
    C1 = A[lvl1][:, lvl1].tocsr()
    ncomp, lab = sp.csgraph.connected_components(C1, directed=False)
    assert ncomp == (3 * q * q * (q - 1) if dim == 3 else 2 * q * (q - 1))
    starts = np.flatnonzero(np.concatenate([[True], np.diff(lab) != 0]))
    assert len(starts) == ncomp


# ------------------------------------------- recursive SLR on C (HID)

def _ml_problem(dim, N, q, **kw):
    csr = si.laplacian_3d(N) if dim == 3 else si.laplacian_2d(N)
    part = si.box_partition_3d(N, q) if dim == 3 else si.box_partition_2d(N, q, q)
    A = sp.csr_matrix((csr[2], csr[1], csr[0]), shape=(csr[3], csr[3]))
    return A, part, q ** dim


@pytest.mark.parametrize("dim,N,q,cf", [(3, 16, 2, "ic0"), (2, 40, 4, "ic0"), (3, 18, 3, "chol")])
def test_multilevel_c_factored_form_is_the_inner_slr_preconditioner(dim, N, q, cf):
    """Sec. 5.2: the recursive scheme applies SLR to C with C's leading HID
    level as the block diagonal B.  K K^T (K^T, K: what the outer level uses
    in place of L^{-1}, L^{-T}) must equal the eq. M preconditioner that
    setup builds for the matrix C on its own, with the connectors of that
    level as subdomains and every other interface node a separator node
    (Sec. 2.1, edge-based form) -- including its own Lanczos run from the
    same start vector; and K^T must be the transpose of K."""
    from scipy.sparse import csgraph
    A, part, p = _ml_problem(dim, N, q)
    P = O.setup(A, part, p, k=6, c_order="hid", c_levels=2, k2=4, c_fact=cf, b_fact=cf)
    ML = P.FC
    s1 = ML.s1
    assert 0 < s1 < P.s and ML.inner.k == 4
    nc, lab = csgraph.connected_components(P.C[:s1, :s1], directed=False)
    part2 = np.concatenate([lab, -np.ones(P.s - s1, dtype=np.int64)])
    v0 = O.splitmix64_uniform(A.shape[0], 7)
    P2 = O.setup(P.C, part2, nc, k=4, c_fact=cf, b_fact=cf, reorth="full",
                 v0=np.concatenate([np.zeros(s1), v0[P.perm[P.m + s1:]]]))
    assert (P2.perm == np.arange(P.s)).all()
    assert np.allclose(P2.lam, ML.inner.lam, rtol=0, atol=1e-13) and abs(P2.theta - ML.inner.theta) < 1e-13
    rng = np.random.default_rng(3)
    x, y = rng.standard_normal(P.s), rng.standard_normal(P.s)
    ref = P2.apply(x)
    assert np.abs(ML.upper(ML.lower(x)) - ref).max() <= 1e-12 * np.abs(ref).max()
    assert abs(x @ ML.lower(y) - ML.upper(x) @ y) <= 1e-12 * np.linalg.norm(x) * np.linalg.norm(y) * 10


def test_multilevel_exact_levels_make_M_equal_A():
    """With exact factors at both levels and every inner eigenpair, the inner
    SLR reproduces C (K^T C K = I); with every outer eigenpair as well,
    M = A (the P1 identity through the recursion)."""
    A, part, p = _ml_problem(2, 21, 3)
    P0 = O.setup(A, part, p, k=0, c_order="hid", c_levels=2, c_fact="chol", b_fact="chol",
                 lowrank2=(np.zeros((0, 0)), np.zeros(0), 0.0))
    s2 = P0.FC.s2
    inner = P0.FC.inner
    H2 = np.column_stack([inner.G(e) for e in np.eye(s2)])
    lam2, V2 = np.linalg.eigh(0.5 * (H2 + H2.T))
    lam2, V2 = lam2[::-1], V2[:, ::-1]
    assert lam2.max() < 1.0
    P1 = O.setup(A, part, p, k=0, c_order="hid", c_levels=2, c_fact="chol", b_fact="chol",
                 lowrank2=(V2, lam2, 0.0))
    ML = P1.FC
    K = np.column_stack([ML.upper(e) for e in np.eye(P1.s)])
    assert np.abs(K.T @ P1.C.toarray() @ K - np.eye(P1.s)).max() < 1e-10
    H = np.column_stack([P1.G(e) for e in np.eye(P1.s)])
    lam, U = np.linalg.eigh(0.5 * (H + H.T))
    lam, U = lam[::-1], U[:, ::-1]
    P = O.setup(A, part, p, k=0, c_order="hid", c_levels=2, c_fact="chol", b_fact="chol",
                lowrank2=(V2, lam2, 0.0), lowrank=(U, lam, 0.0))
    x = np.random.default_rng(5).uniform(-1, 1, A.shape[0])
    assert np.abs(P.apply(A @ x) - x).max() < 1e-10
    res = O.solve(P, A @ x, "pcg")
    assert res.iters == 1 and res.true_relres < 1e-11


def test_multilevel_planted_mistakes_fail_the_pins(monkeypatch):
    """The inner correction used as G2 instead of its square root, the
    F^T C1^{-1} coupling dropped from K^T, or L1^{-1} and L1^{-T} exchanged:
    each breaks the identity with the inner SLR preconditioner."""
    from scipy.sparse import csgraph
    A, part, p = _ml_problem(3, 16, 2)
    P = O.setup(A, part, p, k=4, c_order="hid", c_levels=2, k2=4)
    ML = P.FC
    s1 = ML.s1
    nc, lab = csgraph.connected_components(P.C[:s1, :s1], directed=False)
    part2 = np.concatenate([lab, -np.ones(P.s - s1, dtype=np.int64)])
    v0 = O.splitmix64_uniform(A.shape[0], 7)
    P2 = O.setup(P.C, part2, nc, k=4, reorth="full", v0=np.concatenate([np.zeros(s1), v0[P.perm[P.m + s1:]]]))
    x = np.random.default_rng(4).standard_normal(P.s)
    ref = P2.apply(x)

    def err():
        return np.abs(ML.upper(ML.lower(x)) - ref).max() / np.abs(ref).max()

    assert err() < 1e-12
    good_q = O.MultilevelC._q

    def q_without_root(self, v):
        # G2 itself: rho2 v + U2 D2 U2^T v
        d2 = (self.qd + self.sq) ** 2 - self.sq ** 2
        return self.sq ** 2 * v + self.inner.U @ (d2 * (self.inner.U.T @ v))
    monkeypatch.setattr(O.MultilevelC, "_q", q_without_root)
    assert err() > 1e-6
    monkeypatch.setattr(O.MultilevelC, "_q", good_q)
    good_lower = O.MultilevelC.lower

    def lower_no_coupling(self, v):
        a1 = self.inner.FB.lower(v[:self.s1])
        return np.concatenate([a1, self._q(self.inner.FC.lower(v[self.s1:]))])
    monkeypatch.setattr(O.MultilevelC, "lower", lower_no_coupling)
    assert err() > 1e-6
    monkeypatch.setattr(O.MultilevelC, "lower", good_lower)
    FB = ML.inner.FB
    lo, up = FB.lower, FB.upper
    monkeypatch.setattr(FB, "lower", up)
    monkeypatch.setattr(FB, "upper", lo)
    assert err() > 1e-6
    monkeypatch.setattr(FB, "lower", lo)
    monkeypatch.setattr(FB, "upper", up)
    assert err() < 1e-12


# --------------------------------------------------------------- Krylov

def test_krylov_iteration_counts_on_known_spectra():
    """CG / flexible CG / FGMRES take exactly d iterations on a matrix with
    d distinct eigenvalues (identity preconditioner), and with the exact
    inverse as preconditioner one iteration."""
    rng = np.random.default_rng(4)
    Q, _ = np.linalg.qr(rng.standard_normal((40, 40)))
    d = np.repeat([1.0, 3.0, 7.0], [10, 15, 15])
    A = sp.csr_matrix(Q @ np.diag(d) @ Q.T)
    b = rng.standard_normal(40)
    for fl in (False, True):
        r = O.pcg(A, lambda v: v, b, rtol=1e-10, flexible=fl)
        assert r.iters == 3 and r.true_relres < 1e-9
    r = O.fgmres(A, lambda v: v, b, rtol=1e-10)
    assert r.iters == 3 and r.true_relres < 1e-9
    Ainv = np.linalg.inv(A.toarray())
    assert O.pcg(A, lambda v: Ainv @ v, b).iters == 1
    # restart: GMRES(2) on 3 distinct eigenvalues needs more than 3 products
    r = O.fgmres(A, lambda v: v, b, rtol=1e-10, restart=2, maxit=200)
    assert r.converged and r.iters > 3


class _VariableJacobi:
    """A preconditioner that changes at every call: the j-th call applies
    diag(w_i / a_ii) with w_i = 1 + 0.3 ((i + j) mod 3), so the weights move
    between components from one call to the next (a plain rescaling of one
    fixed M would not test flexibility: CG absorbs it into the step
    length).  Flexible CG and flexible GMRES must keep their defining
    relations with it; the plain forms only keep them for a fixed M."""

    def __init__(self, A):
        self.d = A.diagonal()
        self.i = np.arange(A.shape[0])
        self.j = 0

    def __call__(self, v):
        w = 1.0 + 0.3 * ((self.i + self.j) % 3)
        self.j += 1
        return w * v / self.d


def _anorm(A, v):
    return math.sqrt(float(v @ (A @ v)))


def _local_a_orthogonality(A, ps):
    """max_j |p_j^T A p_{j-1}| / (||p_j||_A ||p_{j-1}||_A)."""
    return max(abs(float(ps[j] @ (A @ ps[j - 1]))) / (_anorm(A, ps[j]) * _anorm(A, ps[j - 1]))
               for j in range(1, len(ps)))


def test_flexible_cg_keeps_local_a_orthogonality_with_a_variable_preconditioner():
    """Flexible CG (Polak-Ribiere beta; Sec. 6 uses flexible outer iterations
    for the reduced-precision form): with a preconditioner that changes at
    every iteration, each search direction stays A-orthogonal to the
    previous one, |p_j^T A p_{j-1}| <= 1e-12 ||p_j||_A ||p_{j-1}||_A, and
    the iteration still converges.  The Fletcher-Reeves beta (the plain CG
    branch, the planted mistake) loses this property by orders of magnitude
    with the same preconditioner."""
    A = si.make_config("diffusion2d_1024", N=20, boxes=2).scipy()
    b = np.random.default_rng(31).uniform(-1, 1, A.shape[0])
    rec = {}
    r = O.pcg(A, _VariableJacobi(A), b, rtol=1e-10, maxit=400, flexible=True, record=rec)
    assert r.converged and r.true_relres <= 1e-9
    assert len(rec["p"]) == r.iters
    assert _local_a_orthogonality(A, rec["p"][:40]) <= 1e-12
    bad = {}
    O.pcg(A, _VariableJacobi(A), b, rtol=1e-10, maxit=40, flexible=False, record=bad)
    assert _local_a_orthogonality(A, bad["p"]) > 1e-4
    # with a fixed preconditioner both betas keep the property (consistency)
    fixed = {}
    O.pcg(A, lambda v: v / A.diagonal(), b, rtol=1e-10, maxit=40, flexible=False, record=fixed)
    assert _local_a_orthogonality(A, fixed["p"]) <= 1e-10


@pytest.mark.parametrize("restart", [60, 20])
def test_fgmres_arnoldi_relation_with_a_variable_preconditioner(restart):
    """Flexible GMRES stores the preconditioned vectors Z (Saad 1993): with a
    preconditioner that changes at every step, each cycle satisfies
    A Z_m = V_{m+1} Hbar_m, and the true residual of the updated iterate
    equals the least-squares estimate, ||b - A x_m|| = |g_{m+1}|, both to
    1e-12.  Updating with M(V_m y) instead of Z_m y (the planted mistake)
    breaks the second relation."""
    A = si.make_config("diffusion2d_1024", N=20, boxes=2).scipy()
    b = np.random.default_rng(32).uniform(-1, 1, A.shape[0])
    M = _VariableJacobi(A)
    rec = {}
    r = O.fgmres(A, M, b, rtol=1e-10, maxit=3000, restart=restart, record=rec)
    assert r.converged and r.true_relres <= 1e-9
    nb = np.linalg.norm(b)
    assert len(rec["cycles"]) >= 2
    for cy in rec["cycles"]:
        V, Z, Hb = cy["V"], cy["Z"], cy["Hbar"]
        assert np.abs(V.T @ V - np.eye(V.shape[1])).max() <= 1e-10
        lhs = A @ Z
        assert np.linalg.norm(lhs - V @ Hb) <= 1e-12 * np.linalg.norm(lhs)
        true = np.linalg.norm(b - A @ cy["x"])
        assert abs(true - cy["g"]) <= 1e-12 * nb, (true, cy["g"])
    # planted mistake on the first cycle: x0 + M(V y) with the
    # preconditioner's next state instead of x0 + Z y
    cy = rec["cycles"][0]
    wrong = cy["x0"] + M(cy["V"][:, :-1] @ cy["y"])
    assert abs(np.linalg.norm(b - A @ wrong) - cy["g"]) > 1e-3 * nb


def test_splitmix64_start_vector_matches_published_outputs():
    """The default Lanczos start vector (reading: SplitMix64 used as a
    counter-based generator keyed by node index) reproduces the published
    first outputs of the generator (tests/golden/splitmix64.json): entry i
    is 2 u - 1 with u the top 53 bits of output i + 1, over 2^53."""
    with open(os.path.join(GOLDEN, "splitmix64.json")) as f:
        g = json.load(f)
    outs = [int(x) for x in g["outputs"]]
    expect = np.array([2.0 * ((z >> 11) / 9007199254740992.0) - 1.0 for z in outs])
    got = O.splitmix64_uniform(len(outs), g["seed"])
    assert np.array_equal(got, expect)
    v = O.splitmix64_uniform(200000, 7)
    assert v.min() >= -1.0 and v.max() < 1.0 and abs(v.mean()) < 0.01 and abs(v.var() - 1.0 / 3.0) < 0.01


def test_pcg_solves_the_small_configuration():
    pr = si.make_config("lap2d_64")
    P = O.setup(pr.csr, pr.part, pr.nparts, pr.k, pr.lanczos_steps, "chol", "chol", v0=pr.v0())
    x, b = pr.rhs()
    r = O.solve(P, b[:, 0])
    assert r.converged and r.true_relres <= 1e-8
    assert np.abs(r.x - x[:, 0]).max() < 1e-6


# ------------------------------------------------------- precision emulation

def test_bf16_rounding_is_round_to_nearest_even():
    import torch
    rng = np.random.default_rng(9)
    x = np.concatenate([rng.standard_normal(2000), [1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -0.0, 1e-30]])
    ref = torch.tensor(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert (O.round_bf16(x) == ref).all()
    assert O.round_bf16(np.array([1.0 + 2 ** -8]))[0] == 1.0


# ------------------------------------------- planted mistakes must be caught

def test_planted_mistakes_fail_the_pins(monkeypatch):
    """A sign error, a transposed factor, or a dropped scalar in the apply
    breaks the M = A identity (P1); a wrong factor in G breaks eq. H."""
    csr, part, p = _tiny(10)
    P0 = O.setup(csr, part, p, 0, b_fact="chol", c_fact="chol")
    H, L, lam, U, _ = _dense_lowrank(P0, P0.s)
    x = np.random.default_rng(2).uniform(-1, 1, P0.A.shape[0])

    def p1_error(P):
        return np.abs(P.apply(P.A @ x) - x).max()

    good = O.setup(csr, part, p, 0, b_fact="chol", c_fact="chol", lowrank=(U, lam, 0.0))
    assert p1_error(good) < 1e-11
    orig = O.SLR.apply_dd

    def sign_flip(self, r):
        r2 = np.array(r, copy=True)
        E = self.E
        self.E = -E
        try:
            return orig(self, r2)
        finally:
            self.E = E
    monkeypatch.setattr(O.SLR, "apply_dd", sign_flip)
    assert p1_error(good) > 1e-3
    monkeypatch.setattr(O.SLR, "apply_dd", orig)

    # lower/upper swapped in the interface solve
    F = good.FC
    lo, up = F.lower, F.upper
    monkeypatch.setattr(F, "lower", up)
    monkeypatch.setattr(F, "upper", lo)
    assert p1_error(good) > 1e-3 or np.abs(good.G(np.ones(good.s)) - H @ np.ones(good.s)).max() > 1e-6
    monkeypatch.setattr(F, "lower", lo)
    monkeypatch.setattr(F, "upper", up)

    # dropped (1 - theta)^{-1} scaling with theta != 0
    k = 4
    H, L, lam, U, theta = _dense_lowrank(P0, k)
    Pk = O.setup(csr, part, p, 0, b_fact="chol", c_fact="chol", lowrank=(U[:, :k], lam[:k], theta))
    spec = _spectrum_MinvA(Pk)
    expect = np.sort(np.concatenate([np.ones(Pk.m + k), (1 - lam[k:]) / (1 - theta)]))
    assert np.allclose(spec, expect, atol=1e-9)
    Pk.theta = 0.0   # keeps the same U, lam: drops the theta scaling
    assert not np.allclose(_spectrum_MinvA(Pk), expect, atol=1e-6)
