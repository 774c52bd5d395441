"""Host-only checks of the C ABI: the library loads, exports every symbol
that include/slr.h declares, and the Python structs match the C layout.
No device compute is called."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "slr.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(slr_[a-z_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    import paper_1505_04340_amd as P
    lib = ctypes.CDLL(P.LIB_PATH)
    names = _declared()
    assert len(names) >= 20
    for nm in names:
        assert hasattr(lib, nm), nm
    assert sorted(P.EXPORTED) == names


def test_binding_struct_layout_matches_header(tmp_path):
    """Every field offset and every struct size of the ctypes structs equals
    the C compiler's for include/slr.h."""
    import paper_1505_04340_amd as P
    structs = [P.slr_csr, P.slr_opts, P.slr_solve_opts, P.slr_solve_info, P.slr_info]
    exprs, want = [], []
    for st in structs:
        exprs.append(f"sizeof({st.__name__})")
        want.append(ctypes.sizeof(st))
        for f, _ in st._fields_:
            exprs.append(f"offsetof({st.__name__}, {f})")
            want.append(getattr(st, f).offset)
    src = tmp_path / "sz.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "slr.h"\nint main(void){\n' +
                   "".join(f'printf("%zu\\n", (size_t){e});\n' for e in exprs) + "return 0;}\n")
    exe = tmp_path / "sz"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    got = [int(x) for x in subprocess.check_output([str(exe)]).split()]
    assert got == want, [(e, g, w) for e, g, w in zip(exprs, got, want) if g != w]


def test_host_only_entry_points():
    import paper_1505_04340_amd as P
    o = P.slr_opts()
    P.slr_default_opts(ctypes.byref(o))
    assert (o.theta_mode, o.b_fact, o.c_fact, o.fact_prec) == (P.SLR_THETA_LAMBDA_K1, P.SLR_FACT_IC0,
                                                               P.SLR_FACT_IC0, P.SLR_FP64)
    assert (o.eps, o.cond_K) == (0.0, 0.0)
    so = P.slr_solve_opts()
    P.slr_default_solve_opts(ctypes.byref(so))
    assert (so.restart, so.maxit, so.rtol) == (40, 300, 1e-8)
    assert P.slr_strerror(P.SLR_ERR_NOCONV) == b"did not converge"
    # null arguments are rejected on the host without touching the device
    h = ctypes.c_void_p()
    assert P.slr_setup(None, None, 1, None, None, ctypes.byref(h)) == P.SLR_ERR_ARG
    assert b"null" in P.slr_last_error()
    assert P.slr_apply(None, None, None, 1, None) == P.SLR_ERR_ARG
    assert P.slr_batch_active(None) == 0
    # option checks come before any device work: eq. Lambda-2 needs eps > 0,
    # eq. condk needs K > 1
    import numpy as np
    rp = np.array([0, 1], dtype=np.int64)
    ci = np.array([0], dtype=np.int32)
    va = np.array([1.0])
    pa = np.array([0], dtype=np.int32)
    csr = P.slr_csr(1, 1, rp.ctypes.data, ci.ctypes.data, va.ctypes.data)
    for mode, eps, K, what in ((P.SLR_THETA_EPS, 0.0, 0.0, b"eps"), (P.SLR_THETA_LAMBDA_K1, 0.0, 0.5, b"cond_K"),
                               (7, 0.0, 0.0, b"theta_mode")):
        o.theta_mode, o.eps, o.cond_K = mode, eps, K
        assert P.slr_setup(ctypes.byref(csr), pa.ctypes.data, 1, ctypes.byref(o), None, ctypes.byref(h)) == P.SLR_ERR_ARG
        assert what in P.slr_last_error()
    # the device refactorisation takes incomplete factors only
    o.theta_mode, o.eps, o.cond_K = P.SLR_THETA_LAMBDA_K1, 0.0, 0.0
    o.refactor, o.b_fact = 1, P.SLR_FACT_CHOL
    assert P.slr_setup(ctypes.byref(csr), pa.ctypes.data, 1, ctypes.byref(o), None, ctypes.byref(h)) == P.SLR_ERR_ARG
    assert b"refactor" in P.slr_last_error()
    assert P.slr_refactor(None, None, 0, None) == P.SLR_ERR_ARG


def test_build_sources_are_gfx950_hip():
    from paper_1505_04340_amd import build
    assert build.ARCH == "gfx950" or os.environ.get("SLR_OFFLOAD_ARCH")
    srcs = build.sources()
    assert any(s.endswith(".hip") for s in srcs)
    assert "-packed-fp32-ops" in build.HIP_FLAGS
