"""MI355X (gfx950) Schur-complement low-rank (SLR) preconditioner.

Thin ctypes binding over the C ABI in include/slr.h (libslr.so, built
in-tree by ``paper_1505_04340_amd.build``).  Only argument marshalling
happens here: every step of setup's Lanczos build, the preconditioner
apply and the Krylov solves runs in the library's HIP kernels.  Device
memory and streams come from PyTorch-ROCm.

Method: Li, Xi & Saad, "Schur complement based domain decomposition
preconditioners with low-rank corrections" (2015).

The module-level functions carry the C names (slr_setup, slr_apply, ...);
``SLR`` and ``Batch`` wrap them for torch tensors.  Vectors are FP64 torch
tensors on the GPU of shape (n,) or (n, nrhs); they are passed to the
library column-major.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
# PyTorch first: the library must bind to the HIP runtime that PyTorch
# loads (loading the library first leaves device allocation failing).
import torch  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libslr.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python paper_1505_04340_amd/build.py` "
                      "(there is no CPU fallback)")
_lib = ctypes.CDLL(LIB_PATH)

# ---- constants (include/slr.h) -------------------------------------------------
SLR_OK, SLR_ERR_ARG, SLR_ERR_NOT_SYMMETRIC, SLR_ERR_PARTITION = 0, -1, -2, -3
SLR_ERR_BREAKDOWN, SLR_ERR_C_NOT_SPD, SLR_ERR_RITZ_SINGULAR, SLR_ERR_LANCZOS_SHORT = -4, -5, -6, -7
SLR_ERR_NOCONV, SLR_ERR_OOM, SLR_ERR_HIP, SLR_ERR_ADMIT = -8, -9, -10, -11
SLR_THETA_LAMBDA_K1, SLR_THETA_ZERO, SLR_THETA_EPS, SLR_THETA_LAMBDA_S = 0, 1, 2, 3
SLR_FACT_CHOL, SLR_FACT_IC0, SLR_FACT_ILDLT0, SLR_FACT_ICT, SLR_FACT_ILDLT = 0, 1, 2, 3, 4
SLR_CORDER_SUBDOMAIN, SLR_CORDER_MULTICOLOR = 0, 1
SLR_FP64, SLR_FP32, SLR_BF16 = 0, 1, 2
SLR_PCG, SLR_FCG, SLR_FGMRES = 0, 1, 2
SLR_REORTH_FULL, SLR_REORTH_PARTIAL = 0, 1

_FACT = {"chol": SLR_FACT_CHOL, "ic0": SLR_FACT_IC0, "ildlt0": SLR_FACT_ILDLT0, "ict": SLR_FACT_ICT,
         "ildlt": SLR_FACT_ILDLT}
_PREC = {"fp64": SLR_FP64, "fp32": SLR_FP32, "bf16": SLR_BF16}
SLR_CORDER_HID = 2
_CORD = {"subdomain": SLR_CORDER_SUBDOMAIN, "multicolor": SLR_CORDER_MULTICOLOR, "hid": SLR_CORDER_HID}
SLR_BORDER_NATURAL, SLR_BORDER_MINDEG = 0, 1
_BORD = {"natural": SLR_BORDER_NATURAL, "mindeg": SLR_BORDER_MINDEG}
_THETA = {"lambda_k1": SLR_THETA_LAMBDA_K1, "zero": SLR_THETA_ZERO, "eps": SLR_THETA_EPS, "lambda_s": SLR_THETA_LAMBDA_S}
_METHOD = {"pcg": SLR_PCG, "fcg": SLR_FCG, "fgmres": SLR_FGMRES}
_REORTH = {"full": SLR_REORTH_FULL, "partial": SLR_REORTH_PARTIAL}

_P = ctypes.c_void_p
_I32, _I64, _D, _U64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_uint64


class slr_csr(ctypes.Structure):
    _fields_ = [("n", _I64), ("nnz", _I64), ("rowptr", _P), ("col", _P), ("val", _P)]


class slr_opts(ctypes.Structure):
    _fields_ = [("k", _I32), ("lanczos_steps", _I32), ("theta_mode", _I32), ("b_fact", _I32),
                ("c_fact", _I32), ("c_order", _I32), ("fact_prec", _I32), ("uk_prec", _I32),
                ("seed", _U64), ("lanczos_v0", _P), ("k_in", _I32), ("U_in", _P),
                ("lambda_in", _P), ("theta_in", _D), ("eps", _D), ("cond_K", _D), ("reorth", _I32),
                ("refactor", _I32), ("droptol", _D), ("b_order", _I32), ("c_levels", _I32), ("k2", _I32),
                ("lanczos_steps2", _I32)]


class slr_solve_opts(ctypes.Structure):
    _fields_ = [("method", _I32), ("restart", _I32), ("maxit", _I32), ("check_every", _I32),
                ("rtol", _D)]


class slr_solve_info(ctypes.Structure):
    _fields_ = [("iters", _I32), ("status", _I32), ("relres", _D)]


class slr_info(ctypes.Structure):
    _fields_ = [("n", _I64), ("m", _I64), ("s", _I64), ("p", _I32), ("k", _I32),
                ("lanczos_steps", _I32), ("b_levels_max", _I32), ("c_levels", _I32),
                ("c_colors", _I32), ("nnz_LB", _I64), ("nnz_LC", _I64), ("nnz_E", _I64),
                ("nnz_A", _I64), ("m_min", _I64), ("m_max", _I64), ("theta", _D),
                ("setup_host_s", _D), ("setup_lanczos_s", _D), ("device_bytes", _I64),
                ("lanczos_reorth", _I32), ("tune_b_threads1", _I32), ("tune_b_lds_div1", _I32),
                ("tune_b_threadsM", _I32), ("tune_b_lds_divM", _I32), ("tune_b_rmaxM", _I32),
                ("lr_chunks", _I32), ("s1", _I64), ("k2", _I32), ("lanczos_steps2", _I32), ("c1_levels", _I32),
                ("c2_levels", _I32), ("theta2", _D), ("nnz_LC1", _I64), ("nnz_LC2", _I64), ("nnz_F", _I64),
                ("tune_b_persistentM", _I32), ("b_lds_level_order", _I32)]


def _sig(name, res, args):
    f = getattr(_lib, name)
    f.restype = res
    f.argtypes = args
    return f


slr_default_opts = _sig("slr_default_opts", None, [ctypes.POINTER(slr_opts)])
slr_default_solve_opts = _sig("slr_default_solve_opts", None, [ctypes.POINTER(slr_solve_opts)])
slr_setup = _sig("slr_setup", ctypes.c_int, [ctypes.POINTER(slr_csr), _P, _I32, ctypes.POINTER(slr_opts), _P,
                                             ctypes.POINTER(_P)])
slr_analyze = _sig("slr_analyze", ctypes.c_int, [ctypes.POINTER(slr_csr), _P, _I32, ctypes.POINTER(slr_opts),
                                                 ctypes.POINTER(slr_info), _P])
slr_update_lowrank = _sig("slr_update_lowrank", ctypes.c_int, [_P, _I32, _I32, _P, _P])
slr_grow_lowrank = _sig("slr_grow_lowrank", ctypes.c_int, [_P, _I32, _I32, _P, _P])
slr_refactor = _sig("slr_refactor", ctypes.c_int, [_P, _P, _I32, _P])
slr_time_kernel = _sig("slr_time_kernel", ctypes.c_int, [_P, _I32, _I32, _I32, _P, ctypes.POINTER(_D)])
slr_apply = _sig("slr_apply", ctypes.c_int, [_P, _P, _P, _I32, _P])
slr_apply_dd = _sig("slr_apply_dd", ctypes.c_int, [_P, _P, _P, _I32, _P])
slr_apply_dd_noalloc = _sig("slr_apply_dd_noalloc", ctypes.c_int, [_P, _P, _P, _I32, _P])
slr_solve = _sig("slr_solve", ctypes.c_int, [_P, _P, _P, _I32, ctypes.POINTER(slr_solve_opts),
                                             ctypes.POINTER(slr_solve_info), _P])
slr_solve_workspace_bytes = _sig("slr_solve_workspace_bytes", ctypes.c_size_t,
                                 [_P, _I32, ctypes.POINTER(slr_solve_opts)])
slr_trim = _sig("slr_trim", ctypes.c_int, [_P])
slr_autotune = _sig("slr_autotune", ctypes.c_int, [_P, _I32, _I32, _P])
slr_export_setup = _sig("slr_export_setup", ctypes.c_int, [_P, _P, ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t)])
slr_import = _sig("slr_import", ctypes.c_int, [_P, ctypes.c_size_t, _P, ctypes.POINTER(_P)])
SLR_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
SLR_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)
slr_set_allocator = _sig("slr_set_allocator", None, [SLR_ALLOC_FN, SLR_FREE_FN, _P])
slr_query = _sig("slr_query", ctypes.c_int, [_P, ctypes.POINTER(slr_info)])
slr_export = _sig("slr_export", ctypes.c_int, [_P, _P, _P, _P, _P, _P, _P])
slr_export_inner = _sig("slr_export_inner", ctypes.c_int, [_P, _P, _P, _P])
slr_set_bsolve_plan = _sig("slr_set_bsolve_plan", ctypes.c_int, [_P, _I32, _I32, _I32, _I32, _I32])
slr_spmv = _sig("slr_spmv", ctypes.c_int, [_P, _P, _P, _I32, _P])
slr_batch_create = _sig("slr_batch_create", ctypes.c_int, [_P, _I32, _I32, _D, _I32, ctypes.POINTER(_P)])
slr_batch_admit = _sig("slr_batch_admit", ctypes.c_int, [_P, _P, _P, _I32, _I64, _P])
slr_batch_step = _sig("slr_batch_step", ctypes.c_int, [_P, _I32, _P])
slr_batch_poll = _sig("slr_batch_poll", ctypes.c_int, [_P, _P, ctypes.POINTER(slr_solve_info), _I32, _P])
slr_batch_active = _sig("slr_batch_active", ctypes.c_int, [_P])
slr_batch_bytes = _sig("slr_batch_bytes", ctypes.c_size_t, [_P])
slr_batch_destroy = _sig("slr_batch_destroy", None, [_P])
slr_destroy = _sig("slr_destroy", None, [_P])
slr_strerror = _sig("slr_strerror", ctypes.c_char_p, [ctypes.c_int])
slr_last_error = _sig("slr_last_error", ctypes.c_char_p, [])
slr_device_lds_bytes = _sig("slr_device_lds_bytes", ctypes.c_int, [])

EXPORTED = ("slr_default_opts", "slr_default_solve_opts", "slr_setup", "slr_analyze", "slr_update_lowrank",
            "slr_grow_lowrank", "slr_refactor",
            "slr_time_kernel", "slr_apply", "slr_apply_dd", "slr_apply_dd_noalloc",
            "slr_solve", "slr_solve_workspace_bytes", "slr_query", "slr_export", "slr_export_inner", "slr_spmv",
            "slr_trim", "slr_export_setup", "slr_import", "slr_set_allocator", "slr_autotune", "slr_set_bsolve_plan",
            "slr_batch_create", "slr_batch_admit", "slr_batch_step", "slr_batch_poll",
            "slr_batch_active", "slr_batch_bytes", "slr_batch_destroy", "slr_destroy",
            "slr_strerror", "slr_last_error", "slr_device_lds_bytes")


class SLRError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        msg = slr_last_error().decode(errors="replace")
        super().__init__(f"{where}: {slr_strerror(code).decode()} ({code}): {msg}")


def _check(rc: int, where: str):
    if rc != SLR_OK:
        raise SLRError(rc, where)


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _colmajor(t):
    """(n,) or (n, r) FP64 CUDA tensor -> contiguous (r, n) storage."""
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64):
        raise TypeError("expected a float64 CUDA tensor")
    if t.dim() == 1:
        return t.contiguous().view(1, -1), True
    return t.t().contiguous(), False


def _csr_arrays(A):
    if isinstance(A, tuple):
        indptr, indices, data, n = A
    else:
        A = A.tocsr()
        indptr, indices, data, n = A.indptr, A.indices, A.data, A.shape[0]
    return (np.ascontiguousarray(indptr, dtype=np.int64), np.ascontiguousarray(indices, dtype=np.int32),
            np.ascontiguousarray(data, dtype=np.float64), int(n))


def _make_opts(k=16, lanczos_steps=0, theta_mode="lambda_k1", b_fact="ic0", c_fact="ic0",
               c_order="subdomain", fact_prec="fp64", uk_prec="fp64", seed=7, eps=0.0, cond_K=0.0,
               reorth=None, refactor=False, droptol=1e-3, b_order="natural", c_levels=1, k2=0, lanczos_steps2=0):
    o = slr_opts()
    slr_default_opts(ctypes.byref(o))
    o.k = k
    o.lanczos_steps = lanczos_steps
    o.theta_mode = _THETA[theta_mode]
    o.b_fact, o.c_fact = _FACT[b_fact], _FACT[c_fact]
    o.c_order = _CORD[c_order]
    o.fact_prec, o.uk_prec = _PREC[fact_prec], _PREC[uk_prec]
    o.seed = seed
    o.eps, o.cond_K = float(eps), float(cond_K)
    if reorth is not None:
        o.reorth = _REORTH[reorth]
    o.refactor = 1 if refactor else 0
    o.droptol = float(droptol)
    o.b_order = _BORD[b_order]
    o.c_levels, o.k2, o.lanczos_steps2 = int(c_levels), int(k2), int(lanczos_steps2)
    return o


class TorchAllocator:
    """Routes the library's device allocations through PyTorch's caching
    allocator (slr_set_allocator), so that PyTorch owns that memory.  Keeps
    count of the calls and of the bytes it holds for the library."""

    def __init__(self):
        import torch
        self._torch = torch
        self.allocs = 0
        self.frees = 0
        self.live = {}
        self._afn = SLR_ALLOC_FN(self._alloc)
        self._ffn = SLR_FREE_FN(self._free)

    def _alloc(self, nbytes, user):
        try:
            t = self._torch
            p = t.cuda.caching_allocator_alloc(int(nbytes), t.cuda.current_device(), t.cuda.current_stream())
        except Exception:
            return None
        self.allocs += 1
        self.live[p] = int(nbytes)
        return p

    def _free(self, ptr, user):
        self.frees += 1
        self.live.pop(ptr, None)
        self._torch.cuda.caching_allocator_delete(ptr)

    def live_bytes(self) -> int:
        return sum(self.live.values())

    def install(self):
        slr_set_allocator(self._afn, self._ffn, None)
        return self


_ALLOCATOR = None


def use_torch_allocator() -> TorchAllocator:
    """Install (once) and return the PyTorch allocator hook."""
    global _ALLOCATOR
    if _ALLOCATOR is None:
        _ALLOCATOR = TorchAllocator()
    return _ALLOCATOR.install()


def use_hip_allocator():
    """Back to hipMalloc / hipFree for new allocations (blocks made through
    the PyTorch hook are still freed through it)."""
    slr_set_allocator(SLR_ALLOC_FN(0), SLR_FREE_FN(0), None)


def analyze(A, part, nparts: int, **opts):
    """Host-only analysis (slr_analyze): (info dict, perm internal->original)."""
    indptr, indices, data, n = _csr_arrays(A)
    part = np.ascontiguousarray(part, dtype=np.int32)
    o = _make_opts(**opts)
    csr = slr_csr(n, int(indptr[-1]), indptr.ctypes.data, indices.ctypes.data, data.ctypes.data)
    info = slr_info()
    perm = np.empty(n, dtype=np.int64)
    _check(slr_analyze(ctypes.byref(csr), part.ctypes.data, nparts, ctypes.byref(o), ctypes.byref(info),
                       perm.ctypes.data), "slr_analyze")
    return {f: getattr(info, f) for f, _ in slr_info._fields_}, perm


class SLR:
    """An SLR preconditioner resident on the current GPU (slr_setup)."""

    def __init__(self, A, part, nparts: int, k: int = 16, lanczos_steps: int = 0,
                 theta_mode: str = "lambda_k1", b_fact: str = "ic0", c_fact: str = "ic0",
                 c_order: str = "subdomain", fact_prec: str = "fp64", uk_prec: str = "fp64",
                 v0=None, seed: int = 7, lowrank=None, eps: float = 0.0, cond_K: float = 0.0,
                 reorth: str | None = None, refactor: bool = False, droptol: float = 1e-3,
                 b_order: str = "natural", c_levels: int = 1, k2: int = 0, lanczos_steps2: int = 0,
                 stream=None):
        indptr, indices, data, n = _csr_arrays(A)
        self.n = n
        part = np.ascontiguousarray(part, dtype=np.int32)
        o = _make_opts(k, lanczos_steps, theta_mode, b_fact, c_fact, c_order, fact_prec, uk_prec, seed, eps, cond_K,
                       reorth, refactor, droptol, b_order, c_levels, k2, lanczos_steps2)
        keep = []
        if v0 is not None:
            v0 = np.ascontiguousarray(v0, dtype=np.float64)
            keep.append(v0)
            o.lanczos_v0 = v0.ctypes.data
        if lowrank is not None:
            U, lam, theta = lowrank
            U = np.asfortranarray(U, dtype=np.float64)
            lam = np.ascontiguousarray(lam, dtype=np.float64)
            keep += [U, lam]
            o.k_in = U.shape[1]
            o.U_in = U.ctypes.data
            o.lambda_in = lam.ctypes.data
            o.theta_in = float(theta)
        csr = slr_csr(n, int(indptr[-1]), indptr.ctypes.data, indices.ctypes.data, data.ctypes.data)
        h = _P()
        _check(slr_setup(ctypes.byref(csr), part.ctypes.data, nparts, ctypes.byref(o), _stream(stream),
                         ctypes.byref(h)), "slr_setup")
        self._pattern = (indptr, indices) if refactor else None
        self._h = h
        self.info = self.query()

    @classmethod
    def import_setup(cls, blob: bytes, stream=None) -> "SLR":
        """A context rebuilt from export_setup()'s bytes (slr_import)."""
        obj = cls.__new__(cls)
        buf = ctypes.create_string_buffer(bytes(blob), len(blob))
        h = _P()
        _check(slr_import(buf, len(blob), _stream(stream), ctypes.byref(h)), "slr_import")
        obj._h = h
        obj._pattern = None
        obj.info = obj.query()
        obj.n = obj.info["n"]
        return obj

    def export_setup(self) -> bytes:
        """The serialised preconditioner (slr_export_setup)."""
        nb = ctypes.c_size_t(0)
        _check(slr_export_setup(self._h, None, 0, ctypes.byref(nb)), "slr_export_setup")
        buf = ctypes.create_string_buffer(nb.value)
        _check(slr_export_setup(self._h, buf, nb.value, ctypes.byref(nb)), "slr_export_setup")
        return buf.raw[:nb.value]

    def autotune(self, nrhs: int = 1, reps: int = 3, stream=None) -> dict:
        """Pick the B kernel's launch shape for nrhs columns and the rank-k
        chunks by timing candidates (slr_autotune); returns the choice."""
        _check(slr_autotune(self._h, nrhs, reps, _stream(stream)), "slr_autotune")
        self.info = self.query()
        return {k: self.info[k] for k in ("tune_b_threads1", "tune_b_lds_div1", "tune_b_threadsM",
                                          "tune_b_lds_divM", "tune_b_rmaxM", "tune_b_persistentM", "lr_chunks")}

    def set_bsolve_plan(self, several: bool, threads: int = 0, lds_div: int = 1, rmax: int = 16,
                        persistent: int = 0):
        """Set the B kernel's launch shape (slr_set_bsolve_plan); threads=0
        restores the built-in plan; persistent 0, 1 or 2."""
        _check(slr_set_bsolve_plan(self._h, 1 if several else 0, threads, lds_div, rmax, int(persistent)),
               "slr_set_bsolve_plan")
        self.info = self.query()

    def trim(self):
        """Release the scratch kept between calls (slr_trim)."""
        _check(slr_trim(self._h), "slr_trim")
        self.info = self.query()

    def close(self):
        if getattr(self, "_h", None):
            slr_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def update_lowrank(self, k: int, lanczos_steps: int = 0, v0=None, stream=None):
        """Rebuild (U_k, Lambda_k, theta) on the device (slr_update_lowrank)."""
        p = None
        if v0 is not None:
            v0 = np.ascontiguousarray(v0, dtype=np.float64)
            p = v0.ctypes.data
        _check(slr_update_lowrank(self._h, k, lanczos_steps, p, _stream(stream)), "slr_update_lowrank")
        self.info = self.query()

    def refactor(self, A, stream=None):
        """New values of A with the pattern given at setup (slr_refactor):
        the factors and stored coefficients are recomputed on the device;
        the low-rank part is kept."""
        if self._pattern is None:
            raise ValueError("set up with refactor=True to refactor")
        indptr, indices, data, n = _csr_arrays(A)
        if n != self.n or not (np.array_equal(indptr, self._pattern[0])
                               and np.array_equal(indices, self._pattern[1])):
            raise ValueError("refactor needs the pattern given at setup")
        _check(slr_refactor(self._h, data.ctypes.data, 0, _stream(stream)), "slr_refactor")

    def refactor_values(self, values, stream=None):
        """As refactor, with the nnz values (setup's CSR order) given as an
        FP64 tensor on the GPU."""
        if self._pattern is None:
            raise ValueError("set up with refactor=True to refactor")
        import torch
        if values.dtype != torch.float64 or not values.is_cuda or values.numel() != len(self._pattern[1]):
            raise ValueError("values: FP64 CUDA tensor with one entry per stored entry of A")
        v = values.contiguous()
        _check(slr_refactor(self._h, ctypes.c_void_p(v.data_ptr()), 1, _stream(stream)), "slr_refactor")

    def grow_lowrank(self, k_add: int, lanczos_steps: int = 0, v0=None, stream=None):
        """Append up to k_add Ritz pairs from a deflated Lanczos run, keeping
        the current ones (slr_grow_lowrank)."""
        p = None
        if v0 is not None:
            v0 = np.ascontiguousarray(v0, dtype=np.float64)
            p = v0.ctypes.data
        _check(slr_grow_lowrank(self._h, k_add, lanczos_steps, p, _stream(stream)), "slr_grow_lowrank")
        self.info = self.query()

    STAGES = {"bsolve1": 0, "cfwd": 1, "lowrank": 2, "cbwd": 3, "bsolve2": 4, "apply": 5, "spmv": 6}

    def time_kernel(self, stage: str, nrhs: int = 1, reps: int = 20, stream=None) -> float:
        """Average ms per launch of one hot-path stage (slr_time_kernel)."""
        ms = _D()
        _check(slr_time_kernel(self._h, self.STAGES[stage], nrhs, reps, _stream(stream), ctypes.byref(ms)),
               "slr_time_kernel")
        return ms.value

    def query(self) -> dict:
        i = slr_info()
        _check(slr_query(self._h, ctypes.byref(i)), "slr_query")
        return {f: getattr(i, f) for f, _ in slr_info._fields_}

    def export(self) -> dict:
        inf = self.query()
        n, s, k, st = inf["n"], inf["s"], inf["k"], inf["lanczos_steps"]
        perm = np.empty(n, dtype=np.int64)
        ritz = np.empty(max(st, k), dtype=np.float64)
        lam = np.empty(k, dtype=np.float64)
        U = np.empty((s, k), dtype=np.float64, order="F")
        al = np.empty(st, dtype=np.float64)
        be = np.empty(st, dtype=np.float64)
        _check(slr_export(self._h, perm.ctypes.data, ritz.ctypes.data, lam.ctypes.data,
                          U.ctypes.data if k else None, al.ctypes.data, be.ctypes.data), "slr_export")
        return {"perm": perm, "ritz": ritz[:st] if st else ritz[:k], "lambda": lam, "U": U,
                "alpha": al, "beta": be, "theta": inf["theta"], "m": inf["m"], "s": s}

    def export_inner(self) -> dict:
        """The recursive interface solver's inner low-rank part
        (slr_export_inner): Ritz values, Lambda2, U2 and theta2."""
        inf = self.query()
        s2, k2, st = inf["s"] - inf["s1"], inf["k2"], inf["lanczos_steps2"]
        ritz = np.empty(max(st, 1), dtype=np.float64)
        lam = np.empty(max(k2, 1), dtype=np.float64)
        U = np.empty((s2, k2), dtype=np.float64, order="F")
        _check(slr_export_inner(self._h, ritz.ctypes.data, lam.ctypes.data, U.ctypes.data if k2 else None),
               "slr_export_inner")
        return {"ritz": ritz[:st], "lambda": lam[:k2], "U": U, "theta": inf["theta2"], "s1": inf["s1"]}

    def _call(self, fn, r, name, stream=None):
        import torch
        rc_, vec = _colmajor(r)
        out = torch.empty_like(rc_)
        _check(fn(self._h, ctypes.c_void_p(rc_.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                  rc_.shape[0], _stream(stream)), name)
        return out.view(-1) if vec else out.t()

    def apply(self, r, stream=None):
        """z = M^{-1} r (original order)."""
        return self._call(slr_apply, r, "slr_apply", stream)

    def apply_dd(self, r, stream=None):
        """z = M^{-1} r in the internal DD order."""
        return self._call(slr_apply_dd, r, "slr_apply_dd", stream)

    def apply_dd_noalloc(self, r, out=None, stream=None):
        """z = M^{-1} r in the internal DD order without any device
        allocation in the library (slr_apply_dd_noalloc); out (optional)
        receives z and must be an FP64 CUDA tensor shaped like r's
        column-major copy."""
        import torch
        rc_, vec = _colmajor(r)
        z = torch.empty_like(rc_) if out is None else out
        _check(slr_apply_dd_noalloc(self._h, ctypes.c_void_p(rc_.data_ptr()), ctypes.c_void_p(z.data_ptr()),
                                    rc_.shape[0], _stream(stream)), "slr_apply_dd_noalloc")
        return z.view(-1) if vec else z.t()

    def spmv(self, x, stream=None):
        return self._call(slr_spmv, x, "slr_spmv", stream)

    def solve(self, b, method: str = "pcg", rtol: float = 1e-8, maxit: int = 300, restart: int = 40,
              check_every: int = 8, stream=None, raise_noconv: bool = False):
        """x with A x = b; returns (x, [{'iters', 'status', 'relres'}, ...])."""
        import torch
        bc, vec = _colmajor(b)
        x = torch.empty_like(bc)
        so = slr_solve_opts()
        slr_default_solve_opts(ctypes.byref(so))
        so.method = _METHOD[method]
        so.rtol, so.maxit, so.restart, so.check_every = rtol, maxit, restart, check_every
        nr = bc.shape[0]
        infos = (slr_solve_info * nr)()
        rc = slr_solve(self._h, ctypes.c_void_p(bc.data_ptr()), ctypes.c_void_p(x.data_ptr()), nr,
                       ctypes.byref(so), infos, _stream(stream))
        if rc != SLR_OK and (rc != SLR_ERR_NOCONV or raise_noconv):
            raise SLRError(rc, "slr_solve")
        out = [{"iters": i.iters, "status": i.status, "relres": i.relres} for i in infos]
        return (x.view(-1) if vec else x.t()), out

    def workspace_bytes(self, nrhs: int, method: str = "pcg", restart: int = 40) -> int:
        so = slr_solve_opts()
        slr_default_solve_opts(ctypes.byref(so))
        so.method, so.restart = _METHOD[method], restart
        return int(slr_solve_workspace_bytes(self._h, nrhs, ctypes.byref(so)))


class Batch:
    """Continuous-batching solver state of one SLR context (slr_batch_*)."""

    def __init__(self, slr: SLR, max_cols: int, method: str = "pcg", rtol: float = 1e-8, maxit: int = 300):
        self.slr = slr
        h = _P()
        _check(slr_batch_create(slr.handle, max_cols, _METHOD[method], rtol, maxit, ctypes.byref(h)),
               "slr_batch_create")
        self._h = h
        self._keep = {}

    def admit(self, b, tag: int, stream=None):
        """Admit b (n,) or (n, r); returns the output tensor x or None when
        no slots are free (SLR_ERR_ADMIT)."""
        import torch
        bc, vec = _colmajor(b)
        x = torch.empty_like(bc)
        rc = slr_batch_admit(self._h, ctypes.c_void_p(bc.data_ptr()), ctypes.c_void_p(x.data_ptr()),
                             bc.shape[0], tag, _stream(stream))
        if rc == SLR_ERR_ADMIT:
            return None
        _check(rc, "slr_batch_admit")
        self._keep[tag] = (bc, x, vec)
        return x

    def step(self, iters: int = 1, stream=None):
        _check(slr_batch_step(self._h, iters, _stream(stream)), "slr_batch_step")

    def poll(self, max_done: int = 64, stream=None):
        """[(tag, x, info)] of finished requests."""
        tags = (ctypes.c_int64 * max_done)()
        infos = (slr_solve_info * max_done)()
        nd = slr_batch_poll(self._h, tags, infos, max_done, _stream(stream))
        if nd < 0:
            raise SLRError(nd, "slr_batch_poll")
        out = []
        for t in range(nd):
            bc, x, vec = self._keep.pop(tags[t])
            out.append((tags[t], x.view(-1) if vec else x.t(),
                        {"iters": infos[t].iters, "status": infos[t].status, "relres": infos[t].relres}))
        return out

    def active(self) -> int:
        return int(slr_batch_active(self._h))

    def bytes(self) -> int:
        return int(slr_batch_bytes(self._h))

    def close(self):
        if getattr(self, "_h", None):
            slr_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
