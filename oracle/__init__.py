"""CPU FP64 oracle of the SLR preconditioner hot path.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
benchmark's CPU-baseline leg may import this package.  It shares no code
with the device library (``paper_1505_04340_amd``) and never imports it.

Reference: R. Li, Y. Xi, Y. Saad, "Schur complement based domain
decomposition preconditioners with low-rank corrections" (2015).
Every function cites the passage it follows.  Readings where the paper is
silent are marked READING.

Plain, slow and step-by-step: scipy/numpy are used only for library
primitives (sparse permutation/slicing and mat-vec, banded Cholesky and
banded triangular solves for the exact factors, a symmetric tridiagonal
eigensolver, dot products); the incomplete factorisations and sparse
triangular sweeps are the plain C loops in ``sparse_loops.c``.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None


def build_c(force: bool = False) -> str:
    """Compile the oracle's C loops with gcc (plain -O2, no vector tricks)."""
    import subprocess
    src = os.path.join(_HERE, "sparse_loops.c")
    out = os.path.join(_HERE, "_sparse_loops.so")
    if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(src):
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-o", out + ".tmp", src, "-lm"])
        os.replace(out + ".tmp", out)
    return out


def _lib():
    global _LIB
    if _LIB is None:
        lib = ctypes.CDLL(build_c())
        P = ctypes.c_void_p
        I64 = ctypes.c_int64
        lib.orc_ic0.argtypes = [I64, P, P, P]
        lib.orc_ic0.restype = ctypes.c_int
        lib.orc_ildlt0.argtypes = [I64, P, P, P, P]
        lib.orc_ildlt0.restype = ctypes.c_int
        lib.orc_ict.argtypes = [I64, P, P, P, ctypes.c_double, ctypes.c_int, I64, P, P, P, P]
        lib.orc_ict.restype = ctypes.c_int
        lib.orc_lower_solve.argtypes = [I64, P, P, P, P, ctypes.c_int]
        lib.orc_upper_solve.argtypes = [I64, P, P, P, P, ctypes.c_int]
        lib.orc_diag_solve.argtypes = [I64, P, P, P]
        _LIB = lib
    return _LIB


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


class OracleError(RuntimeError):
    def __init__(self, code: str, msg: str):
        super().__init__(f"{code}: {msg}")
        self.code = code


# ---------------------------------------------------------------------------
# C1 / C2: classification and domain-decomposition ordering (Sec. 2.1)
# ---------------------------------------------------------------------------

def classify(A: sp.csr_matrix, part: np.ndarray, nparts: int):
    """Interior / interface labels (Sec. 2.1, local view of a subdomain).

    Vertex-based partitioning: a node is a local interface node when it is
    coupled to a node of another subdomain; otherwise it is interior.
    Edge-based partitioning: nodes labelled -1 form the vertex separator
    (shared interface); coupling to a separator node does not make a node
    an interface node.  Returns (is_interface bool[n], owner int[n]) with
    owner = -1 for separator nodes."""
    part = np.asarray(part)
    if part.shape != (A.shape[0],) or part.min() < -1 or part.max() >= nparts:
        raise OracleError("PARTITION", "labels out of range")
    rows = np.repeat(np.arange(A.shape[0]), np.diff(A.indptr))
    cols = A.indices
    pr, pc = part[rows], part[cols]
    cross = (pr >= 0) & (pc >= 0) & (pr != pc)
    iface = np.zeros(A.shape[0], dtype=bool)
    iface[rows[cross]] = True
    iface |= part < 0
    return iface, part.copy()


def greedy_colors(C: sp.csr_matrix) -> np.ndarray:
    """READING for the multicolour ordering of C: greedy colouring in the
    current row order, each node taking the smallest colour unused by its
    already-coloured neighbours."""
    n = C.shape[0]
    col = -np.ones(n, dtype=np.int64)
    for i in range(n):
        used = set(col[C.indices[C.indptr[i]:C.indptr[i + 1]]].tolist())
        c = 0
        while c in used:
            c += 1
        col[i] = c
    return col


def min_degree_order(M: sp.csr_matrix) -> np.ndarray:
    """READING for the AMD ordering of each B_i before ICT / ILDLT (Sec. 6
    reorders every B_i by approximate minimum degree to reduce fill): the
    minimum degree ordering that AMD approximates, with exact degrees.
    Eliminating a node joins its remaining neighbours into a clique (the
    elimination graph); each step eliminates the remaining node of smallest
    degree in that graph, the smallest index among equal degrees.  Returns
    the elimination order (new -> old local index)."""
    import heapq
    n = M.shape[0]
    adj = [set(M.indices[M.indptr[i]:M.indptr[i + 1]].tolist()) - {i} for i in range(n)]
    heap = [(len(adj[i]), i) for i in range(n)]
    heapq.heapify(heap)
    done = np.zeros(n, dtype=bool)
    order = []
    while heap:
        d, p = heapq.heappop(heap)
        if done[p] or d != len(adj[p]):
            continue            # stale entry
        done[p] = True
        order.append(p)
        nb = adj[p]
        for u in nb:
            adj[u].discard(p)
            adj[u] |= nb - {u}
            heapq.heappush(heap, (len(adj[u]), u))
        adj[p] = set()
    return np.array(order, dtype=np.int64)


def dd_ordering(A: sp.csr_matrix, part: np.ndarray, nparts: int, c_order: str = "subdomain",
                b_order: str = "natural"):
    """Global DD ordering of eq. (Global): interiors u_1..u_p by subdomain,
    then the interface y.  READING: ascending original index inside each
    group; interface grouped by owner subdomain 0..p-1 with separator nodes
    last (eq. Global2 with y = [y_1; ...; y_p]).  With c_order='multicolor'
    the interface is additionally stably sorted by greedy colour.  With
    b_order='mindeg' the interior of each subdomain is in the minimum degree
    order of its B_i (min_degree_order) instead of ascending index.
    Returns (perm new->old, interior offsets [p+1], interface offsets
    [p+2] (last group = separator), colours or None)."""
    iface, owner = classify(A, part, nparts)
    idx = np.arange(A.shape[0])
    inter = [idx[(~iface) & (owner == q)] for q in range(nparts)]
    if b_order == "mindeg":
        inter = [g[min_degree_order(A[g][:, g].tocsr())] for g in inter]
    elif b_order != "natural":
        raise OracleError("ARG", b_order)
    ifc = [idx[iface & (owner == q)] for q in range(nparts)] + [idx[iface & (owner < 0)]]
    off_b = np.concatenate([[0], np.cumsum([len(a) for a in inter])])
    off_y = np.concatenate([[0], np.cumsum([len(a) for a in ifc])])
    perm = np.concatenate(inter + ifc).astype(np.int64)
    colors = None
    if c_order == "hid":
        # READING of the HID ordering (Sec. 5.2 names the Hierarchical
        # Interface Decomposition of Henon and Saad for making C's leading
        # block block diagonal): the key of an interface node is the set of
        # subdomains met in its closed neighbourhood; nodes with equal keys
        # form a connector, whose level is the key's size.  Connectors are
        # taken by level, then by key, nodes by ascending index.
        m = off_b[-1]
        y = perm[m:]
        keys = []
        for i in y:
            nb = A.indices[A.indptr[i]:A.indptr[i + 1]]
            keys.append(tuple(sorted(set(np.asarray(part)[nb].tolist()) | {int(part[i])})))
        order = sorted(range(len(y)), key=lambda t: (len(keys[t]), keys[t], int(y[t])))
        perm = np.concatenate([perm[:m], y[order]])
        colors = np.array([len(keys[t]) for t in order], dtype=np.int64)
    elif c_order == "multicolor":
        m = off_b[-1]
        y = perm[m:]
        C = A[y][:, y].tocsr()
        colors = greedy_colors(C)
        order = np.argsort(colors, kind="stable")
        perm = np.concatenate([perm[:m], y[order]])
        colors = colors[order]
    elif c_order != "subdomain":
        raise OracleError("ARG", c_order)
    return perm, off_b, off_y, colors


# ---------------------------------------------------------------------------
# C3: local factorisations (Sec. 5.2)
# ---------------------------------------------------------------------------

@dataclass
class Factor:
    """L L^T (kind 'ic0' / 'chol') or L D L^T (kind 'ildlt0') of a block
    diagonal matrix.  For 'chol' each block is kept in LAPACK lower-band
    storage (band[i - j, j] = L[i, j])."""
    kind: str
    n: int
    rp: np.ndarray = None
    ci: np.ndarray = None
    v: np.ndarray = None
    blocks: list = field(default_factory=list)   # (start, lower band of L) for chol

    def round_to(self, prec: str):
        """READING (reduced precision): factors are computed in FP64 and the
        stored values rounded to nearest-even FP32."""
        if prec == "fp64":
            return
        if self.v is not None:
            self.v = self.v.astype(np.float32).astype(np.float64)
        self.blocks = [(s, L.astype(np.float32).astype(np.float64)) for s, L in self.blocks]

    def _band_solve(self, x: np.ndarray, trans: str) -> np.ndarray:
        for s, cb in self.blocks:
            nb = cb.shape[1]
            y, info = sla.lapack.dtbtrs(cb, x[s:s + nb].reshape(nb, 1), uplo="L", trans=trans)
            if info != 0:
                raise OracleError("BREAKDOWN", f"dtbtrs info {info}")
            x[s:s + nb] = y.ravel()
        return x

    def lower(self, x: np.ndarray) -> np.ndarray:
        """x <- L^{-1} x (unit L for LDL^T)."""
        x = np.array(x, dtype=np.float64, copy=True)
        if self.kind == "chol":
            return self._band_solve(x, "N")
        _lib().orc_lower_solve(self.n, _p(self.rp), _p(self.ci), _p(self.v), _p(x),
                               1 if self.kind in ("ildlt0", "ildlt") else 0)
        return x

    def upper(self, x: np.ndarray) -> np.ndarray:
        """x <- L^{-T} x."""
        x = np.array(x, dtype=np.float64, copy=True)
        if self.kind == "chol":
            return self._band_solve(x, "T")
        _lib().orc_upper_solve(self.n, _p(self.rp), _p(self.ci), _p(self.v), _p(x),
                               1 if self.kind in ("ildlt0", "ildlt") else 0)
        return x

    def dense_lower(self, a: int, b: int) -> np.ndarray:
        """Dense copy of the diagonal block [a, b) of L (tests only)."""
        if self.kind == "chol":
            for s, cb in self.blocks:
                if s == a and s + cb.shape[1] == b:
                    nb = cb.shape[1]
                    L = np.zeros((nb, nb))
                    for d in range(cb.shape[0]):
                        L[np.arange(d, nb), np.arange(0, nb - d)] = cb[d, :nb - d]
                    return L
            raise KeyError((a, b))
        M = sp.csr_matrix((self.v, self.ci, self.rp), shape=(self.n, self.n))
        return M[a:b][:, a:b].toarray()

    def solve(self, x: np.ndarray) -> np.ndarray:
        """x <- (L L^T)^{-1} x, or (L D L^T)^{-1} x."""
        y = self.lower(x)
        if self.kind in ("ildlt0", "ildlt"):
            _lib().orc_diag_solve(self.n, _p(self.rp), _p(self.v), _p(y))
        return self.upper(y)


def _tril_csr(M: sp.csr_matrix):
    T = sp.tril(M, format="csr")
    T.sort_indices()
    rp = T.indptr.astype(np.int64)
    ci = T.indices.astype(np.int32)
    v = T.data.astype(np.float64).copy()
    # the diagonal must be the last entry of each row
    for i in range(T.shape[0]):
        if rp[i + 1] == rp[i] or ci[rp[i + 1] - 1] != i:
            raise OracleError("BREAKDOWN", f"missing diagonal in row {i}")
    return rp, ci, v


def factorize(M: sp.csr_matrix, kind: str, block_offsets=None, what: str = "B", droptol: float = 0.0) -> Factor:
    """Factor a (block diagonal) symmetric matrix.

    'ic0'    incomplete Cholesky with zero fill: the unique lower L on the
             pattern of tril(M) with (L L^T)_ij = m_ij on that pattern.
    'ildlt0' incomplete L D L^T with zero fill, unit L.
    'ict' / 'ildlt'  threshold dropping (the local solvers of Sec. 6):
             left-looking by columns, an entry of column j is kept when its
             updated value is at least droptol times the 1-norm of column j
             of tril(M) (READING: the paper gives no dropping rule).
    'chol'   exact Cholesky of every diagonal block (banded LAPACK)."""
    n = M.shape[0]
    if kind == "chol":
        # exact Cholesky of every diagonal block, in LAPACK lower-band form
        offs = block_offsets if block_offsets is not None else [0, n]
        blocks = []
        Md = M.tocsr()
        for a, b in zip(offs[:-1], offs[1:]):
            if b > a:
                Bk = Md[a:b][:, a:b].tocoo()
                bw = int(max(0, (Bk.row - Bk.col).max()))
                ab = np.zeros((bw + 1, b - a))
                lo = Bk.row >= Bk.col
                ab[(Bk.row - Bk.col)[lo], Bk.col[lo]] = Bk.data[lo]
                try:
                    blocks.append((a, sla.cholesky_banded(ab, lower=True)))
                except np.linalg.LinAlgError:
                    raise OracleError("C_NOT_SPD" if what == "C" else "BREAKDOWN",
                                      "Cholesky failed")
        return Factor("chol", n, blocks=blocks)
    rp, ci, v = _tril_csr(M.tocsr())
    if kind in ("ict", "ildlt"):
        cap = 4 * len(ci) + n
        while True:
            orp = np.zeros(n + 1, dtype=np.int64)
            oci = np.zeros(cap, dtype=np.int32)
            ov = np.zeros(cap)
            need = ctypes.c_int64(0)
            rc = _lib().orc_ict(n, _p(rp), _p(ci), _p(v), float(droptol), 1 if kind == "ildlt" else 0, cap, _p(orp),
                                _p(oci), _p(ov), ctypes.byref(need))
            if rc != -(n + 1):
                break
            cap = int(need.value)
        if rc != 0:
            raise OracleError("C_NOT_SPD" if what == "C" else "BREAKDOWN", f"{kind} pivot failure in column {-rc - 1}")
        nz = int(orp[-1])
        return Factor(kind, n, orp, oci[:nz].copy(), ov[:nz].copy())
    if kind == "ic0":
        rc = _lib().orc_ic0(n, _p(rp), _p(ci), _p(v))
    elif kind == "ildlt0":
        d = np.zeros(n)
        rc = _lib().orc_ildlt0(n, _p(rp), _p(ci), _p(v), _p(d))
    else:
        raise OracleError("ARG", kind)
    if rc != 0:
        raise OracleError("C_NOT_SPD" if what == "C" else "BREAKDOWN",
                          f"{kind} pivot failure in row {-rc - 1}")
    return Factor(kind, n, rp, ci, v)


# ---------------------------------------------------------------------------
# Reduced-precision emulation helpers (stored-data rounding only)
# ---------------------------------------------------------------------------

def round_fp32(x):
    return np.asarray(x, dtype=np.float64).astype(np.float32).astype(np.float64)


def round_bf16(x):
    """READING: BF16 storage = round-to-nearest-even of the FP32-rounded value."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float64).astype(np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64).reshape(f.shape)


# ---------------------------------------------------------------------------
# The preconditioner
# ---------------------------------------------------------------------------

@dataclass
class SLR:
    A: sp.csr_matrix            # original matrix
    perm: np.ndarray            # new -> old
    off_b: np.ndarray
    off_y: np.ndarray
    m: int
    s: int
    Ap: sp.csr_matrix           # A in DD order
    E: sp.csr_matrix            # m x s
    C: sp.csr_matrix            # s x s
    FB: Factor
    FC: Factor
    k: int = 0
    U: np.ndarray = None        # s x k (C-factor order)
    lam: np.ndarray = None      # k Ritz values, descending
    theta: float = 0.0
    eps: float = 0.0            # > 0: the eq. Lambda-2 choice of Lambda~ (theta unused)
    ritz: np.ndarray = None     # all Ritz values of T_m, descending
    steps: int = 0
    reorth_steps: list = field(default_factory=list)   # partial reorthogonalisation: steps cleaned
    alpha: np.ndarray = None
    beta: np.ndarray = None
    colors: np.ndarray = None

    # -- products with the blocks -------------------------------------------------
    def G(self, v: np.ndarray) -> np.ndarray:
        """H v = L^{-1} E^T B^{-1} E L^{-T} v (eq. H), the operator Lanczos
        runs on (Sec. 5.1)."""
        t = self.FC.upper(v)
        e = self.E @ t
        z = self.FB.solve(e)
        g = self.E.T @ z
        return self.FC.lower(g)

    def apply_dd(self, r: np.ndarray) -> np.ndarray:
        """M^{-1} r in DD order, M of eq. (M) with S~^{-1} of eq. (skt).

        The inverse of the block factorisation needs two solves with B and
        one with S~ (Sec. 2.2):
          z  = B^{-1} f
          g' = g - E^T z
          S~^{-1} g' = L^{-T}[(1-theta)^{-1} w + U_k D U_k^T w], w = L^{-1} g',
                       D = diag((1-lambda_i)^{-1} - (1-theta)^{-1})   (eq. skt,
                       in the L-form used in its proof, Z_k = L^{-T} U_k)
          u  = B^{-1}(f - E y)."""
        r = np.asarray(r, dtype=np.float64)
        f, g = r[:self.m], r[self.m:]
        z = self.FB.solve(f)
        gp = g - self.E.T @ z
        w = self.FC.lower(gp)
        if self.eps > 0.0:
            # eq. Lambda-2: 1 - lambda~_i = (1 - lambda_i)/eps for i <= k,
            # lambda~_i = 0 beyond, so (I - Lambda~)^{-1} - I has the entries
            # eps/(1 - lambda_i) - 1 on the captured directions and 0 elsewhere
            rho, dsc = 1.0, (self.eps / (1.0 - self.lam) - 1.0) if self.k else None
        else:
            rho = 1.0 / (1.0 - self.theta)
            dsc = (1.0 / (1.0 - self.lam) - rho) if self.k else None
        wp = rho * w
        if self.k:
            c = self.U.T @ w
            c = c * dsc
            wp = wp + self.U @ c
        y = self.FC.upper(wp)
        u = self.FB.solve(f - self.E @ y)
        return np.concatenate([u, y])

    def apply(self, r: np.ndarray) -> np.ndarray:
        """M^{-1} r in original order (column-major block of vectors ok)."""
        r = np.asarray(r, dtype=np.float64)
        if r.ndim == 2:
            return np.column_stack([self.apply(r[:, j]) for j in range(r.shape[1])])
        out = np.empty_like(r)
        out[self.perm] = self.apply_dd(r[self.perm])
        return out


class MultilevelC:
    """Interface factor of the recursive SLR method (Sec. 5.2): instead of a
    factor of C, the SLR preconditioner is applied to C itself.

    In HID order C = [C1 F; F^T C2] with C1 the nodes of the lowest
    connector level, block diagonal (one block per connector).  The inner
    SLR takes B := C1, E := F and C := C2 = L2 L2^T, H2 = L2^{-1} F^T C1^{-1}
    F L2^{-T} (eq. H one level down) and (I - H2)^{-1} ~ G2 = rho2 I + U2 D2
    U2^T (eq. skt with theta2 = lambda_{k2+1}).  READING (the paper leaves
    the multilevel scheme to future work): so that the outer Lanczos keeps
    running on a symmetric operator, the inner preconditioner is written as
    M_C^{-1} = K K^T with
        K^T = [ L1^{-1}                          0          ]
              [ -Q2 L2^{-1} F^T C1^{-1} L1       Q2 L2^{-1} ],  applied as
    a1 = L1^{-1} v1, a2 = Q2 L2^{-1} (v2 - F^T L1^{-T} a1), and
    K w = (L1^{-T}(w1 - L1^{-1} F b2), b2 = L2^{-T} Q2 w2), where
    Q2 = G2^{1/2} = sqrt(rho2) I + U2 diag(sqrt(rho2 + d_i) - sqrt(rho2)) U2^T
    (U2 has orthonormal columns).  K K^T is the eq. M block inverse of the
    inner SLR, and the outer method uses K^T and K where a plain SLR uses
    L^{-1} and L^{-T}.  G2 must be positive definite: every lambda2_i and
    theta2 below 1."""

    def __init__(self, inner: "SLR"):
        self.inner = inner
        self.s1, self.s2 = inner.m, inner.s
        self.n = self.s1 + self.s2
        rho2 = 1.0 / (1.0 - inner.theta)
        if not rho2 > 0.0 or (inner.k and np.any(inner.lam >= 1.0)):
            raise OracleError("C_NOT_SPD", "inner low-rank correction is not positive definite (a Ritz value >= 1)")
        self.sq = math.sqrt(rho2)
        self.qd = (np.sqrt(1.0 / (1.0 - inner.lam)) - self.sq) if inner.k else np.zeros(0)

    def _q(self, x: np.ndarray) -> np.ndarray:
        """Q2 x = sqrt(rho2) x + U2 diag(qd) U2^T x."""
        out = self.sq * x
        if self.inner.k:
            out = out + self.inner.U @ (self.qd * (self.inner.U.T @ x))
        return out

    def lower(self, v: np.ndarray) -> np.ndarray:
        """K^T v (takes the place of L^{-1} v)."""
        P = self.inner
        v = np.asarray(v, dtype=np.float64)
        a1 = P.FB.lower(v[:self.s1])
        t = v[self.s1:] - P.E.T @ P.FB.upper(a1)
        return np.concatenate([a1, self._q(P.FC.lower(t))])

    def upper(self, w: np.ndarray) -> np.ndarray:
        """K w (takes the place of L^{-T} w)."""
        P = self.inner
        w = np.asarray(w, dtype=np.float64)
        b2 = P.FC.upper(self._q(w[self.s1:]))
        b1 = P.FB.upper(w[:self.s1] - P.FB.lower(P.E @ b2))
        return np.concatenate([b1, b2])

    def solve(self, x: np.ndarray) -> np.ndarray:
        """M_C^{-1} x = K K^T x."""
        return self.upper(self.lower(x))

    def round_to(self, prec: str):
        """The inner factors are rounded when they are built (before the
        inner Lanczos run), so there is nothing left to do here."""


def multilevel_c(C: sp.csr_matrix, lev: np.ndarray, c_fact: str, droptol: float, k2: int, steps2: int,
                 v0_2: np.ndarray, fact_prec: str = "fp64", lowrank2=None) -> MultilevelC:
    """Build the recursive interface solver of Sec. 5.2 from C in HID order
    (lev: the connector level of every interface node, non-decreasing).
    The nodes of the lowest level are C1, whose blocks (the connectors) are
    the connected pieces of its graph, each a contiguous range; both C1 and
    C2 are factored with c_fact and rounded to fact_prec; the inner Lanczos
    (full reorthogonalisation, steps2 steps from v0_2, the C2 entries of the
    outer start vector) gives U2, Lambda2 and theta2 = lambda_{k2+1}.
    lowrank2: optional (U2, lam2, theta2) used instead of that run."""
    from scipy.sparse import csgraph
    s = C.shape[0]
    lev = np.asarray(lev)
    s1 = int(np.sum(lev == lev.min())) if s else 0
    if s1 == 0 or s1 == s:
        raise OracleError("ARG", "the HID order has a single connector level: nothing to recurse on")
    C1 = C[:s1, :s1].tocsr()
    F = C[:s1, s1:].tocsr()
    C2 = C[s1:, s1:].tocsr()
    ncomp, lab = csgraph.connected_components(C1, directed=False)
    starts = np.flatnonzero(np.concatenate([[True], lab[1:] != lab[:-1]]))
    if len(starts) != ncomp:
        raise OracleError("ARG", "a connector of the leading level is not contiguous")
    off1 = np.concatenate([starts, [s1]])
    FB2 = factorize(C1, c_fact, off1, "C", droptol)
    FC2 = factorize(C2, c_fact, [0, s - s1], "C", droptol)
    FB2.round_to(fact_prec)
    FC2.round_to(fact_prec)
    inner = SLR(C, np.arange(s), off1, np.array([0, s - s1]), s1, s - s1, C, F, C2, FB2, FC2)
    if lowrank2 is not None:
        U2, lam2, th2 = lowrank2
        inner.U = np.array(U2, dtype=np.float64).reshape(s - s1, -1)
        inner.lam = np.array(lam2, dtype=np.float64)
        inner.k = inner.U.shape[1]
        inner.theta = float(th2)
    elif k2 > 0:
        lanczos_lowrank(inner, k2, steps2 or 5 * k2, np.asarray(v0_2, dtype=np.float64), "lambda_k1",
                        reorth="full")
    return MultilevelC(inner)


def setup(A, part, nparts: int, k: int, lanczos_steps: int = 0, b_fact: str = "ic0",
          c_fact: str = "ic0", c_order: str = "subdomain", theta_mode: str = "lambda_k1",
          fact_prec: str = "fp64", uk_prec: str = "fp64", v0: np.ndarray | None = None,
          lowrank=None, eps: float = 0.0, cond_K: float = 0.0, reorth: str = "partial",
          droptol: float = 1e-3, seed: int = 7, b_order: str = "natural", c_levels: int = 1,
          k2: int = 0, lanczos_steps2: int = 0, lowrank2=None) -> SLR:
    """Build the SLR preconditioner (Sec. 4 and Sec. 5).

    A: scipy CSR or (indptr, indices, data, n).  part: subdomain labels
    (-1 = separator).  lanczos_steps 0 means 5k (Sec. 6).  v0: Lanczos start
    vector in original node order (its interface entries are used); when
    it is None the start vector is splitmix64_uniform(n, seed).
    lowrank: optional (U, lam, theta) to use instead of running Lanczos.
    theta_mode "lambda_k1" (theta = lambda_{k+1}, Sec. 4), "lambda_s"
    (theta = smallest Ritz value, Sec. 4), "zero" (eq. Lambda-1) or "eps"
    (eq. Lambda-2 with parameter eps > 0).
    cond_K > 1: k becomes the smallest rank (at most the given k) with
    lambda_{k+1} <= 1 - 1/K among the Ritz values (eq. condk).  reorth:
    Lanczos with full ("full") or partial ("partial", Sec. 5.1)
    reorthogonalisation.  b_fact / c_fact "ict" (and "ildlt" for B): threshold
    factors with drop tolerance droptol (factorize).  b_order "natural" or
    "mindeg" (the minimum degree order of each B_i, dd_ordering).
    c_levels 2: the recursive SLR on C of Sec. 5.2 (MultilevelC, C in HID
    order) replaces the factor of C, with rank k2 (default k) from
    lanczos_steps2 (default 5 k2) inner Lanczos steps started from the
    start vector's entries on the inner interface; lowrank2 as lowrank for
    the inner level."""
    if theta_mode == "eps" and not eps > 0.0:
        raise OracleError("ARG", "theta_mode eps needs eps > 0")
    if isinstance(A, tuple):
        indptr, indices, data, n = A
        A = sp.csr_matrix((data, indices, indptr), shape=(n, n))
    A = sp.csr_matrix(A)
    if abs(A - A.T).max() > 0:
        raise OracleError("NOT_SYMMETRIC", "A must be symmetric")
    perm, off_b, off_y, colors = dd_ordering(A, part, nparts, c_order, b_order)
    m = int(off_b[-1])
    s = A.shape[0] - m
    Ap = A[perm][:, perm].tocsr()
    B = Ap[:m, :m].tocsr()
    E = Ap[:m, m:].tocsr()
    C = Ap[m:, m:].tocsr()
    FB = factorize(B, b_fact, off_b, "B", droptol)
    if v0 is None and (k > 0 or c_levels == 2):
        v0 = splitmix64_uniform(A.shape[0], seed)
    if c_levels == 2:
        if c_order != "hid":
            raise OracleError("ARG", "the recursive interface solver needs the HID order of C")
        kk2 = k2 if k2 > 0 else k
        s1 = int(np.sum(colors == colors.min())) if s else 0
        FC = multilevel_c(C, colors, c_fact, droptol, kk2, lanczos_steps2, np.asarray(v0)[perm[m + s1:]],
                          fact_prec, lowrank2)
    elif c_levels == 1:
        # exact C solve: one dense block; otherwise IC(0)
        FC = factorize(C, c_fact, [0, s], "C", droptol)
    else:
        raise OracleError("ARG", "c_levels is 1 or 2")
    FB.round_to(fact_prec)
    FC.round_to(fact_prec)
    P = SLR(A, perm, off_b, off_y, m, s, Ap, E, C, FB, FC, colors=colors)
    if lowrank is not None:
        U, lam, theta = lowrank
        P.U = np.array(U, dtype=np.float64).reshape(s, -1)
        P.lam = np.array(lam, dtype=np.float64)
        P.k = P.U.shape[1]
        P.theta = 0.0 if theta_mode == "eps" else float(theta)
    elif k > 0:
        steps = lanczos_steps or 5 * k
        lanczos_lowrank(P, k, steps, np.asarray(v0)[perm[m:]], theta_mode, cond_K, reorth)
    else:
        P.theta = 0.0
    if theta_mode == "eps":
        P.eps = float(eps)
        if P.k and np.any(np.abs(1.0 - P.lam) < 1e-12):
            raise OracleError("RITZ_SINGULAR", "Ritz value too close to 1")
    if uk_prec == "fp32":
        P.U = round_fp32(P.U)
    elif uk_prec == "bf16":
        P.U = round_bf16(P.U)
    return P


def splitmix64_uniform(n: int, seed: int) -> np.ndarray:
    """Default Lanczos start vector (Sec. 5.1 leaves the start vector open).

    READING: U[-1, 1) values from SplitMix64 (Steele, Lea and Flood,
    "Fast splittable pseudorandom number generators", OOPSLA 2014), used as
    a counter-based generator: the value of node i (original order) comes
    from the (i+1)-th output of the stream started at ``seed``, i.e. from the
    state seed + (i+1) * 0x9E3779B97F4A7C15 (mod 2^64) passed through the
    generator's mixing function; its top 53 bits give u in [0, 1) and the
    entry is 2u - 1.  Written from the published definition."""
    gamma = np.uint64(0x9E3779B97F4A7C15)
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + gamma * (np.arange(n, dtype=np.uint64) + np.uint64(1))
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    u = (z >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)
    return 2.0 * u - 1.0


def lanczos(G, v0: np.ndarray, steps: int, Z: np.ndarray | None = None):
    """Lanczos with full reorthogonalisation (Sec. 5.1).

    READING: full classical Gram-Schmidt applied twice (CGS2) replaces the
    paper's partial reorthogonalisation; stop after ``steps`` steps or when
    beta_j <= 1e-14 ||T_j||_inf.  Returns (V, alpha, beta) with V the
    orthonormal basis actually built (s x m) and beta of length m (its last
    entry is the residual norm beta_m of the final step).  Z (s x k0,
    orthonormal columns, optional): directions already captured; both
    Gram-Schmidt passes also run against them (deflation, Sec. 5.3)."""
    s = v0.shape[0]
    V = np.zeros((s, steps))
    alpha, beta = [], []
    V[:, 0] = v0 / np.linalg.norm(v0)
    tnorm = 0.0
    for j in range(steps):
        v = V[:, j]
        w = G(v)
        a = float(v @ w)
        w = w - a * v
        if j > 0:
            w = w - beta[j - 1] * V[:, j - 1]
        Q = V[:, :j + 1] if Z is None else np.hstack([Z, V[:, :j + 1]])
        for _ in range(2):
            h = Q.T @ w
            w = w - Q @ h
        b = float(np.linalg.norm(w))
        alpha.append(a)
        row = abs(a) + b + (beta[j - 1] if j > 0 else 0.0)
        tnorm = max(tnorm, row)
        if j + 1 == steps or b <= 1e-14 * tnorm:
            return V[:, :j + 1], np.array(alpha), np.array(beta + [b])
        beta.append(b)
        V[:, j + 1] = w / b


EPS = 2.0 ** -52


def lanczos_pro(G, v0: np.ndarray, steps: int, stats: dict | None = None):
    """Lanczos with partial reorthogonalisation (Sec. 5.1, the scheme of
    Parlett and Simon): the three-term recurrence, plus a classical
    Gram-Schmidt pass against all previous vectors only on steps where
    estimated orthogonality is lost.

    The estimates omega_{j+1,l} ~ v_{j+1}.v_l follow from the computed
    recurrence beta_j v_{j+1} = H v_j - alpha_j v_j - beta_{j-1} v_{j-1}
    taken against v_l and the same relation for v_l:
        beta_j om_{j+1,l} = beta_l om_{j,l+1} + (alpha_l - alpha_j) om_{j,l}
                            + beta_{l-1} om_{j,l-1} - beta_{j-1} om_{j-1,l},
    with om_{i,i} = 1.  READINGS (the paper only names the scheme): the
    rounding term e = eps sqrt(s) ||T_j|| is added to each estimate with
    its sign and om_{j+1,j} = e / beta_j (before the division); ||T_j|| is
    the running max of |alpha_i| + beta_i + beta_{i-1} with beta_i taken
    before any reorthogonalisation; when max_l |om_{j+1,l}| > sqrt(eps)
    the new vector and the one after it are reorthogonalised (one pass
    against all previous vectors) and their estimates reset to e / beta_j;
    alpha_j is not updated by the pass, beta_j is the norm after it.
    Stops as ``lanczos``.  stats (optional dict) receives "reorth", the
    list of reorthogonalised steps."""
    s = v0.shape[0]
    V = np.zeros((s, steps))
    alpha, beta = [], []
    V[:, 0] = v0 / np.linalg.norm(v0)
    tnorm = 0.0        # stopping test, as in lanczos
    tpro = 0.0         # ||T_j|| of the rounding term
    om_prev = np.zeros(0)      # om_{j-1, l}, l < j-1
    om_cur = np.zeros(0)       # om_{j, l},   l < j
    force = False
    done = []
    for j in range(steps):
        v = V[:, j]
        w = G(v)
        a = float(v @ w)
        w = w - a * v
        bm = beta[j - 1] if j > 0 else 0.0
        if j > 0:
            w = w - bm * V[:, j - 1]
        bpre = float(np.linalg.norm(w))
        tpro = max(tpro, abs(a) + bpre + bm)
        e = EPS * math.sqrt(s) * tpro

        def cur(l):            # om_{j,l} with the unit diagonal
            return 1.0 if l == j else om_cur[l]

        def prev(l):           # om_{j-1,l}
            return 1.0 if l == j - 1 else om_prev[l]

        new = np.zeros(j + 1)
        for l in range(j):
            t = beta[l] * cur(l + 1) + (alpha[l] - a) * cur(l) - bm * prev(l)
            if l > 0:
                t += beta[l - 1] * cur(l - 1)
            t += math.copysign(e, t)
            new[l] = t / bpre if bpre > 0 else 1.0
        psi = e / bpre if bpre > 0 else 1.0
        new[j] = psi
        big = bool(np.max(np.abs(new)) > math.sqrt(EPS))
        if force:
            do, force = True, False
        elif big:
            do, force = True, True
        else:
            do = False
        if do:
            Q = V[:, :j + 1]
            w = w - Q @ (Q.T @ w)
            new[:] = psi
            done.append(j)
        b = float(np.linalg.norm(w))
        alpha.append(a)
        tnorm = max(tnorm, abs(a) + b + bm)
        if j + 1 == steps or b <= 1e-14 * tnorm:
            if stats is not None:
                stats["reorth"] = done
            return V[:, :j + 1], np.array(alpha), np.array(beta + [b])
        beta.append(b)
        V[:, j + 1] = w / b
        om_prev, om_cur = om_cur, new


def lanczos_lowrank(P: SLR, k: int, steps: int, v0_iface: np.ndarray, theta_mode: str, cond_K: float = 0.0,
                    reorth: str = "partial"):
    """(U_k, Lambda_k, theta) from Lanczos on H (Sec. 5.1, eq. skt).

    The Ritz pairs of the tridiagonal T_m are sorted by decreasing value;
    the k largest give Lambda_k and U_k = V_m Y_k; theta = lambda_{k+1}
    (Sec. 4, the paper's choice), the smallest Ritz value (the lambda_s end
    of the interval of Sec. 4 over which the condition number is flat) or 0
    (eq. Lambda-1, truncation, and the eq. Lambda-2 form).  cond_K > 1: the rank is the number of Ritz values
    above 1 - 1/K, at most k (eq. condk: lambda_{k+1} <= 1 - 1/K).
    reorth: "full" (CGS2 every step) or "partial" (lanczos_pro)."""
    if reorth == "partial":
        st = {}
        V, alpha, beta = lanczos_pro(P.G, v0_iface, steps, st)
        P.reorth_steps = st["reorth"]
    else:
        V, alpha, beta = lanczos(P.G, v0_iface, steps)
    mm = V.shape[1]
    T = np.diag(alpha) + np.diag(beta[:mm - 1], 1) + np.diag(beta[:mm - 1], -1)
    ev, Y = np.linalg.eigh(T)
    ev, Y = ev[::-1], Y[:, ::-1]
    need = k + 1 if theta_mode in ("lambda_k1", "lambda_s") else k
    if mm < need:
        raise OracleError("LANCZOS_SHORT", f"{mm} Ritz pairs < {need}")
    if cond_K > 1.0:
        k = min(k, int(np.sum(ev > 1.0 - 1.0 / cond_K)))
    P.k = k
    P.lam = ev[:k].copy()
    P.U = V @ Y[:, :k]
    P.theta = float(ev[k]) if theta_mode == "lambda_k1" else float(ev[-1]) if theta_mode == "lambda_s" else 0.0
    P.ritz = ev
    P.steps = mm
    P.alpha, P.beta = alpha, beta
    if np.any(np.abs(1.0 - P.lam) < 1e-12) or abs(1.0 - P.theta) < 1e-12:
        raise OracleError("RITZ_SINGULAR", "Ritz value too close to 1")
    return P


def _take_ritz(ev, k, theta_mode, cond_K):
    """Rank and theta from descending Ritz values (Sec. 4, eq. condk)."""
    if cond_K > 1.0:
        k = min(k, int(np.sum(ev > 1.0 - 1.0 / cond_K)))
    theta = float(ev[k]) if theta_mode == "lambda_k1" else float(ev[-1]) if theta_mode == "lambda_s" else 0.0
    return k, theta


def grow_lowrank(P: SLR, k_add: int, steps: int, v0_iface: np.ndarray, theta_mode: str = "lambda_k1",
                 cond_K: float = 0.0):
    """Add up to k_add vectors to (U_k, Lambda_k) without discarding them
    (Sec. 5.3, improving an SLR preconditioner by deflation).

    READING: deflated Lanczos.  The start vector (interface entries,
    normalised) is orthogonalised twice against U_k, and every step's
    Gram-Schmidt passes include U_k, so the run sees H on the orthogonal
    complement of the captured directions.  Its k_add largest Ritz pairs
    are appended: U = [U_k, V_m Y], Lambda = [Lambda_k, new values], and
    theta follows theta_mode on the new run's Ritz values (lambda_{k+1} is
    the largest one not taken).  cond_K as in lanczos_lowrank, applied to
    the new values."""
    Z = P.U if P.k else None
    v = np.asarray(v0_iface, dtype=np.float64)
    nv = np.linalg.norm(v)
    if not nv > 0.0:
        raise OracleError("ARG", "Lanczos start vector is zero on the interface")
    v = v / nv
    if Z is not None:
        for _ in range(2):
            v = v - Z @ (Z.T @ v)
    if not np.linalg.norm(v) > 1e-12:
        raise OracleError("ARG", "start vector lies in the span of U_k")
    V, alpha, beta = lanczos(P.G, v, steps, Z)
    mm = V.shape[1]
    T = np.diag(alpha) + np.diag(beta[:mm - 1], 1) + np.diag(beta[:mm - 1], -1)
    ev, Y = np.linalg.eigh(T)
    ev, Y = ev[::-1], Y[:, ::-1]
    need = k_add + 1 if theta_mode in ("lambda_k1", "lambda_s") else k_add
    if mm < need:
        raise OracleError("LANCZOS_SHORT", f"{mm} Ritz pairs < {need}")
    ka, theta = _take_ritz(ev, k_add, theta_mode, cond_K)
    Unew = V @ Y[:, :ka]
    P.U = Unew if Z is None else np.hstack([Z, Unew])
    P.lam = np.concatenate([P.lam[:P.k] if P.k else np.zeros(0), ev[:ka]])
    P.k = P.U.shape[1]
    P.theta = 0.0 if theta_mode == "eps" else theta
    P.ritz = ev
    P.steps = mm
    P.alpha, P.beta = alpha, beta
    if np.any(np.abs(1.0 - P.lam) < 1e-12) or abs(1.0 - P.theta) < 1e-12:
        raise OracleError("RITZ_SINGULAR", "Ritz value too close to 1")
    return P


# ---------------------------------------------------------------------------
# C6: Krylov accelerators (Sec. 6: CG for SPD, GMRES(40) for indefinite;
#     stop when the residual norm is reduced by 1e-8, at most 300 its)
# ---------------------------------------------------------------------------

@dataclass
class SolveResult:
    x: np.ndarray
    iters: int
    converged: bool
    true_relres: float
    history: list


def _true_relres(A, x, b):
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(b - A @ x) / nb) if nb > 0 else 0.0


def pcg(A, M, b, rtol=1e-8, maxit=300, flexible=False, record: dict | None = None) -> SolveResult:
    """Preconditioned CG, x0 = 0.  READING: stop on the recurrence residual
    ||r_j|| <= rtol ||b||; the iteration count is the number of products
    with A.  flexible=True uses the Polak-Ribiere beta (flexible CG).
    record (optional dict) receives "p", the list of search directions in
    the order they are used (for the pins)."""
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b)
    r = b.copy()
    nb = np.linalg.norm(b)
    hist = [1.0]
    if nb == 0:
        return SolveResult(x, 0, True, 0.0, hist)
    z = M(r)
    p = z.copy()
    rz = float(r @ z)
    for it in range(1, maxit + 1):
        if record is not None:
            record.setdefault("p", []).append(p.copy())
        q = A @ p
        alpha = rz / float(p @ q)
        x += alpha * p
        r_old = r
        r = r - alpha * q
        rn = np.linalg.norm(r)
        hist.append(rn / nb)
        if rn <= rtol * nb:
            return SolveResult(x, it, True, _true_relres(A, x, b), hist)
        z = M(r)
        rz_new = float(r @ z)
        beta = (float(z @ (r - r_old)) if flexible else rz_new) / rz
        rz = rz_new
        p = z + beta * p
    return SolveResult(x, maxit, False, _true_relres(A, x, b), hist)


def fgmres(A, M, b, rtol=1e-8, maxit=300, restart=40, record: dict | None = None) -> SolveResult:
    """Right-preconditioned flexible GMRES(restart) (Saad 1993), x0 = 0,
    modified Gram-Schmidt Arnoldi, Givens rotations.  READING: stop when the
    least-squares residual estimate falls to rtol ||b||; the iteration count
    is the number of products with A.  record (optional dict) receives
    "cycles": per restart cycle the start x0, the bases V (n x (m+1)) and
    Z (n x m), the Hessenberg block Hbar ((m+1) x m) before the rotations,
    the least-squares solution y, the residual estimate |g_{m+1}| and the
    updated x (for the pins)."""
    b = np.asarray(b, dtype=np.float64)
    n = b.shape[0]
    x = np.zeros(n)
    nb = np.linalg.norm(b)
    hist = [1.0]
    if nb == 0:
        return SolveResult(x, 0, True, 0.0, hist)
    it = 0
    while True:
        r = b - A @ x
        beta = np.linalg.norm(r)
        V = np.zeros((n, restart + 1))
        Z = np.zeros((n, restart))
        H = np.zeros((restart + 1, restart))
        cs, sn = np.zeros(restart), np.zeros(restart)
        gvec = np.zeros(restart + 1)
        gvec[0] = beta
        V[:, 0] = r / beta
        j_done = 0
        done = False
        Hbar = np.zeros((restart + 1, restart)) if record is not None else None
        for j in range(restart):
            Z[:, j] = M(V[:, j])
            w = A @ Z[:, j]
            it += 1
            for i in range(j + 1):
                H[i, j] = float(w @ V[:, i])
                w = w - H[i, j] * V[:, i]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] > 0:
                V[:, j + 1] = w / H[j + 1, j]
            if Hbar is not None:
                Hbar[:j + 2, j] = H[:j + 2, j]
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = np.hypot(H[j, j], H[j + 1, j])
            cs[j], sn[j] = H[j, j] / den, H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            gvec[j + 1] = -sn[j] * gvec[j]
            gvec[j] = cs[j] * gvec[j]
            hist.append(abs(gvec[j + 1]) / nb)
            j_done = j + 1
            if abs(gvec[j + 1]) <= rtol * nb or it >= maxit:
                done = True
                break
        y = sla.solve_triangular(H[:j_done, :j_done], gvec[:j_done])
        x0 = x
        x = x + Z[:, :j_done] @ y
        if record is not None:
            record.setdefault("cycles", []).append(dict(
                x0=x0, V=V[:, :j_done + 1].copy(), Z=Z[:, :j_done].copy(), Hbar=Hbar[:j_done + 1, :j_done].copy(),
                y=y, g=abs(gvec[j_done]), x=x.copy()))
        if done:
            conv = hist[-1] <= rtol
            return SolveResult(x, it, conv, _true_relres(A, x, b), hist)


def solve(P: SLR, b: np.ndarray, method: str = "pcg", rtol=1e-8, maxit=300, restart=40):
    """Solve A x = b with the SLR preconditioner, in the original ordering."""
    A = P.A
    M = P.apply
    if method == "pcg":
        return pcg(A, M, b, rtol, maxit)
    if method == "fcg":
        return pcg(A, M, b, rtol, maxit, flexible=True)
    if method == "fgmres":
        return fgmres(A, M, b, rtol, maxit, restart)
    raise OracleError("ARG", method)
