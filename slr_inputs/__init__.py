"""Seeded synthetic workloads for the SLR preconditioner.

This module only builds *inputs*: sparse matrices of the model problems,
partition vectors, right-hand sides and Lanczos start vectors.  It holds
none of the preconditioner's arithmetic, so that both the CPU oracle and
the device library can consume the same data without sharing any code
path of the method itself.

Model problems follow the experiments section of Li, Xi & Saad (2015),
"Schur complement based domain decomposition preconditioners with
low-rank corrections" (Sec. 6.1, the PDE -Lap(u) - c u = f with 5/7-point
centred differences on the unit square/cube, Dirichlet boundary).  As in
Sec. 3.2 the 1/h^2 scaling is omitted, so the 5-point stencil has 4 on the
diagonal and -1 off it (6 and -1 for the 7-point stencil).

Grid numbering: node (x, y[, z]) has index x + N*y (+ N*N*z).
Matrices are returned as ``(indptr int64, indices int32, data float64, n)``
with sorted column indices and the full symmetric pattern.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp

__all__ = [
    "Problem", "laplacian_2d", "laplacian_3d", "diffusion_2d", "gaussian_field",
    "box_partition_2d", "box_partition_3d", "random_cuts_2d", "separator_model",
    "rhs_from_solution", "lanczos_start", "make_config", "CONFIG_NAMES",
    "shift_for_negative_count_3d",
]


def _to_csr(A: sp.spmatrix):
    A = sp.csr_matrix(A)
    A.sum_duplicates()
    A.sort_indices()
    return (A.indptr.astype(np.int64), A.indices.astype(np.int32),
            A.data.astype(np.float64), A.shape[0])


def _lap1d(N: int) -> sp.csr_matrix:
    e = np.ones(N)
    return sp.diags([-e[:-1], 2 * e, -e[:-1]], [-1, 0, 1], format="csr")


def laplacian_2d(N: int, shift: float = 0.0, Ny: int | None = None):
    """5-point Dirichlet Laplacian on an N x Ny grid, minus shift*I."""
    Ny = N if Ny is None else Ny
    A = sp.kron(sp.identity(Ny), _lap1d(N)) + sp.kron(_lap1d(Ny), sp.identity(N))
    if shift:
        A = A - shift * sp.identity(N * Ny)
    return _to_csr(A)


def laplacian_3d(N: int, shift: float = 0.0):
    """7-point Dirichlet Laplacian on an N^3 grid, minus shift*I."""
    I = sp.identity(N)
    T = _lap1d(N)
    A = (sp.kron(I, sp.kron(I, T)) + sp.kron(I, sp.kron(T, I))
         + sp.kron(T, sp.kron(I, I)))
    if shift:
        A = A - shift * sp.identity(N ** 3)
    return _to_csr(A)


def shift_for_negative_count_3d(N: int, count: int) -> float:
    """Shift s such that the 7-point Laplacian on N^3 minus s*I has exactly
    ``count`` negative eigenvalues: the midpoint between the count-th and
    (count+1)-th smallest closed-form eigenvalues
    4 sum_d sin^2(j_d pi / (2(N+1))).  Input-construction helper only."""
    lam1 = 4.0 * np.sin(np.arange(1, N + 1) * np.pi / (2 * (N + 1))) ** 2
    m = min(N, 12)
    l = lam1[:m]
    ev = np.sort((l[:, None, None] + l[None, :, None] + l[None, None, :]).ravel())
    if ev[count] - ev[count - 1] <= 0:
        raise ValueError("no spectral gap at this count")
    return 0.5 * (ev[count - 1] + ev[count])


def gaussian_field(N: int, corr_len: float, variance: float, seed: int,
                   torus: int = 2048) -> np.ndarray:
    """Stationary Gaussian random field g on the (N+2)^2 node lattice of
    spacing h = 1/(N+1) (boundary nodes included), covariance
    variance * exp(-r^2 / (2 corr_len^2)).  Sampled by FFT filtering of
    white noise on a ``torus`` x ``torus`` periodic lattice, then cropped."""
    M = max(torus, N + 2)
    h = 1.0 / (N + 1)
    rng = np.random.Generator(np.random.PCG64(seed))
    noise = rng.standard_normal((M, M))
    d = np.minimum(np.arange(M), M - np.arange(M)) * h
    r2 = d[:, None] ** 2 + d[None, :] ** 2
    cov = np.exp(-r2 / (2.0 * corr_len ** 2))
    spec = np.fft.fft2(cov).real
    spec = np.maximum(spec, 0.0)
    g = np.fft.ifft2(np.fft.fft2(noise) * np.sqrt(spec)).real
    g = g[: N + 2, : N + 2]
    g = g - g.mean()
    g = g * math.sqrt(variance) / g.std()
    return g


def diffusion_2d(N: int, a_nodes: np.ndarray):
    """5-point discretisation of -div(a grad u) on an N x N interior grid
    with Dirichlet boundary.  ``a_nodes`` has shape (N+2, N+2) and holds the
    coefficient on every lattice node, boundary included (row = y, col = x).
    The coefficient on the edge between two nodes is the harmonic mean of
    their nodal values; the stencil is unscaled (no 1/h^2)."""
    a = np.asarray(a_nodes, dtype=np.float64)
    assert a.shape == (N + 2, N + 2)
    hm = lambda p, q: 2.0 * p * q / (p + q)
    ai = a[1:-1, 1:-1]
    west = hm(ai, a[1:-1, :-2])
    east = hm(ai, a[1:-1, 2:])
    south = hm(ai, a[:-2, 1:-1])
    north = hm(ai, a[2:, 1:-1])
    diag = (west + east + south + north).ravel()
    idx = np.arange(N * N).reshape(N, N)
    rows, cols, vals = [np.arange(N * N)], [np.arange(N * N)], [diag]
    # east neighbour (x+1): edge coefficient east[y, x] for x < N-1
    rows.append(idx[:, :-1].ravel()); cols.append(idx[:, 1:].ravel()); vals.append(-east[:, :-1].ravel())
    rows.append(idx[:, 1:].ravel()); cols.append(idx[:, :-1].ravel()); vals.append(-east[:, :-1].ravel())
    rows.append(idx[:-1, :].ravel()); cols.append(idx[1:, :].ravel()); vals.append(-north[:-1, :].ravel())
    rows.append(idx[1:, :].ravel()); cols.append(idx[:-1, :].ravel()); vals.append(-north[:-1, :].ravel())
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(N * N, N * N))
    return _to_csr(A)


def _cuts(N: int, p: int, widths: np.ndarray | None = None) -> np.ndarray:
    """Owner strip (0..p-1) of every coordinate 0..N-1."""
    if widths is None:
        edges = np.array([(i * N) // p for i in range(p + 1)])
    else:
        c = np.concatenate([[0.0], np.cumsum(widths)])
        edges = np.rint(c / c[-1] * N).astype(np.int64)
    own = np.empty(N, dtype=np.int32)
    for i in range(p):
        own[edges[i]:edges[i + 1]] = i
    return own


def box_partition_2d(N: int, px: int, py: int, Ny: int | None = None) -> np.ndarray:
    Ny = N if Ny is None else Ny
    ox, oy = _cuts(N, px), _cuts(Ny, py)
    return (ox[None, :] + px * oy[:, None]).astype(np.int32).ravel()


def box_partition_3d(N: int, p: int) -> np.ndarray:
    o = _cuts(N, p)
    return (o[None, None, :] + p * o[None, :, None] + p * p * o[:, None, None]).astype(np.int32).ravel()


def random_cuts_2d(N: int, px: int, py: int, seed: int) -> np.ndarray:
    """Box partition with strip widths proportional to U[1, sqrt 2]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    wx = rng.uniform(1.0, math.sqrt(2.0), px)
    wy = rng.uniform(1.0, math.sqrt(2.0), py)
    ox, oy = _cuts(N, px, wx), _cuts(N, py, wy)
    return (ox[None, :] + px * oy[:, None]).astype(np.int32).ravel()


def _separator_cuts(N: int, q: int) -> np.ndarray:
    """Strip (0..q-1) of every coordinate 0..N-1, or -1 on the q-1 cut
    coordinates between strips (spread evenly)."""
    cut = [((k * (N + 1)) // q) - 1 for k in range(1, q)]
    own = np.empty(N, dtype=np.int32)
    strip = 0
    for x in range(N):
        if strip < q - 1 and x == cut[strip]:
            own[x] = -1
            strip += 1
        else:
            own[x] = strip
    return own


def separator_partition(N: int, q: int, dim: int) -> np.ndarray:
    """Edge-based partition of an N^dim grid into q^dim boxes: nodes on the
    cut lines (2-D) or planes (3-D) are separator nodes (label -1), the
    others carry their box's label (x fastest)."""
    o = _separator_cuts(N, q)
    if dim == 2:
        lab = np.where((o[None, :] < 0) | (o[:, None] < 0), -1, o[None, :] + q * o[:, None])
    else:
        lab = np.where((o[None, None, :] < 0) | (o[None, :, None] < 0) | (o[:, None, None] < 0), -1,
                       o[None, None, :] + q * o[None, :, None] + q * q * o[:, None, None])
    return lab.astype(np.int32).ravel()


def separator_model(nx: int, ny: int):
    """Two-domain model of Sec. 3.2: an nx x (2 ny + 1) grid split by the
    middle grid line.  Returns (csr, part) with part = -1 on the separator
    line (edge-based partitioning, vertex separator)."""
    A = laplacian_2d(nx, Ny=2 * ny + 1)
    y = np.repeat(np.arange(2 * ny + 1), nx)
    part = np.where(y < ny, 0, np.where(y > ny, 1, -1)).astype(np.int32)
    return A, part


def rhs_from_solution(csr, nrhs: int, seed: int):
    """x* ~ U[-1, 1] (PCG64 seed), b = A x*.  Column-major (n, nrhs)."""
    indptr, indices, data, n = csr
    rng = np.random.Generator(np.random.PCG64(seed))
    x = rng.uniform(-1.0, 1.0, size=(nrhs, n)).T.copy()
    A = sp.csr_matrix((data, indices, indptr), shape=(n, n))
    b = np.asfortranarray(A @ x)
    return np.asfortranarray(x), b


def lanczos_start(n: int, seed: int = 7) -> np.ndarray:
    """Lanczos start vector in original node order, U[-1, 1] from PCG64.
    The preconditioner uses its entries on the interface nodes."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(-1.0, 1.0, size=n)


@dataclass
class Problem:
    name: str
    csr: tuple
    part: np.ndarray
    nparts: int
    k: int
    lanczos_steps: int
    b_fact: str          # "chol" | "ic0" | "ildlt0"
    c_fact: str          # "chol" | "ic0"
    solver: str          # "pcg" | "fcg" | "fgmres"
    nrhs: int = 1
    rhs_seed: int = 0
    v0_seed: int = 7
    extra: dict = field(default_factory=dict)

    @property
    def n(self):
        return self.csr[3]

    def rhs(self):
        return rhs_from_solution(self.csr, self.nrhs, self.rhs_seed)

    def v0(self):
        return lanczos_start(self.n, self.v0_seed)

    def scipy(self):
        indptr, indices, data, n = self.csr
        return sp.csr_matrix((data, indices, indptr), shape=(n, n))


CONFIG_NAMES = ("lap2d_64", "lap3d_64", "shifted3d_128", "diffusion2d_1024",
                "serve_lap2d_256", "serve_lap2d_512", "serve_lap3d_64", "serve_lap3d_96")


def make_config(name: str, **over) -> Problem:
    """The workloads, by name and size:

    lap2d_64          2-D 5-pt Laplacian 64x64, 2x2 boxes, exact Cholesky B_i/C,
                      k=16 from 60 Lanczos steps, PCG, RHS seed 1001.
    lap3d_64          3-D 7-pt Laplacian 64^3, 4x4x4 boxes, IC(0)/IC(0), k=32,
                      160 Lanczos steps (5k), PCG, RHS seed 1002.
    shifted3d_128     3-D 7-pt Laplacian 128^3 minus sI with 20 negative
                      eigenvalues, 8x8x8 boxes, ILDL^T(0) B_i, IC(0) C, k=64,
                      320 steps, FGMRES(40), RHS seed 1003.
    diffusion2d_1024  -div(e^g grad u) on 1024^2, g Gaussian (corr 1/32, var 1,
                      seed 11), 16x16 random cuts (seed 12), IC(0)/IC(0), k=64,
                      320 steps, 32 RHS, flexible CG, RHS seed 1004.
    serve_*           serving matrices: 2-D 256^2 (4x4, k=16), 512^2 (8x8, k=32),
                      3-D 64^3 (4x4x4, k=32), 96^3 (6x6x6, k=32); IC(0)/IC(0).
    Keyword overrides replace Problem fields (e.g. a smaller N for tests).
    """
    N = over.pop("N", None)
    if name == "lap2d_64":
        N = N or 64
        pr = Problem(name, laplacian_2d(N), box_partition_2d(N, 2, 2), 4, 16, 60,
                     "chol", "chol", "pcg", 1, 1001)
    elif name == "lap3d_64":
        N = N or 64
        q = over.pop("boxes", 4)
        pr = Problem(name, laplacian_3d(N), box_partition_3d(N, q), q ** 3, 32, 160,
                     "ic0", "ic0", "pcg", 1, 1002)
    elif name == "shifted3d_128":
        N = N or 128
        q = over.pop("boxes", 8)
        cnt = over.pop("neg", 20)
        s = shift_for_negative_count_3d(N, cnt)
        pr = Problem(name, laplacian_3d(N, s), box_partition_3d(N, q), q ** 3, 64, 320,
                     "ildlt0", "ic0", "fgmres", 1, 1003, extra={"shift": s, "neg": cnt})
    elif name == "diffusion2d_1024":
        N = N or 1024
        q = over.pop("boxes", 16)
        g = gaussian_field(N, 1.0 / 32.0, 1.0, 11)
        pr = Problem(name, diffusion_2d(N, np.exp(g)), random_cuts_2d(N, q, q, 12), q * q,
                     64, 320, "ic0", "ic0", "fcg", 32, 1004)
    elif name.startswith("serve_"):
        table = {"serve_lap2d_256": (2, 256, 4, 16), "serve_lap2d_512": (2, 512, 8, 32),
                 "serve_lap3d_64": (3, 64, 4, 32), "serve_lap3d_96": (3, 96, 6, 32)}
        d, NN, q, k = table[name]
        NN = N or NN
        if d == 2:
            csr, part, p = laplacian_2d(NN), box_partition_2d(NN, q, q), q * q
        else:
            csr, part, p = laplacian_3d(NN), box_partition_3d(NN, q), q ** 3
        pr = Problem(name, csr, part, p, k, 5 * k, "ic0", "ic0", "pcg", 1, 1005)
    else:
        raise KeyError(name)
    for key, v in over.items():
        setattr(pr, key, v)
    return pr
