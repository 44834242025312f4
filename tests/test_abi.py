"""The C-ABI library loads, exports every symbol its header declares, and validates arguments on
the host (no GPU needed for any of these)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mpspmv.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(\w+)\s*\(", text, flags=re.M)
    return sorted(set(n for n in names if n not in ("defined",)))


def test_library_exports_every_declared_symbol():
    from paper_1411_2377_amd import _lib
    names = declared_functions()
    assert "mpspmv_csr" in names and len(names) >= 4
    for n in names:
        assert hasattr(_lib.LIB, n), n
        assert n in _lib.SIGNATURES or n in _lib.SPECIAL, "binding lacks a signature for %s" % n


def test_host_validation_errors():
    from paper_1411_2377_amd import _lib
    a = _lib.MpCsr()
    a.row_dim, a.col_dim, a.nnz, a.prec = 4, 4, 0, 100
    a.row_ptr = 1234
    a.val.len, a.val.ld = 0, 0
    assert _lib.LIB.mp_validate_csr(ctypes.byref(a), 0) == _lib.MPS_EINVAL
    assert "precision" in _lib.last_error()
    a.prec = 256
    assert _lib.LIB.mp_validate_csr(ctypes.byref(a), 0) == _lib.MPS_OK
    a.nnz = 3
    a.val.len, a.val.ld = 3, 3
    assert _lib.LIB.mp_validate_csr(ctypes.byref(a), 0) == _lib.MPS_EINVAL   # null col_idx
    a.col_idx = 4321
    assert _lib.LIB.mp_validate_csr(ctypes.byref(a), 0) == _lib.MPS_EINVAL   # null val pointers
    a.val.limb, a.val.hdr = 1000, 2000
    assert _lib.LIB.mp_validate_csr(ctypes.byref(a), 0) == _lib.MPS_OK
    a.val.ld = 2
    assert _lib.LIB.mp_validate_csr(ctypes.byref(a), 0) == _lib.MPS_EINVAL   # ld < len
    a.val.ld = 3
    a.row_dim = -1
    assert _lib.LIB.mp_validate_csr(ctypes.byref(a), 0) == _lib.MPS_EINVAL
    a.row_dim = 4
    # SpMV argument checks happen before any device work
    x = _lib.MpVec(5000, 6000, 3, 3)   # wrong length (col_dim = 4)
    y = _lib.MpVec(7000, 8000, 4, 4)
    assert _lib.LIB.mpspmv_csr(ctypes.byref(a), ctypes.byref(x), ctypes.byref(y), 0, None, None) == _lib.MPS_EINVAL
    x.len, x.ld = 4, 4
    assert _lib.LIB.mpspmv_csr(ctypes.byref(a), ctypes.byref(x), ctypes.byref(y), 7, None, None) == _lib.MPS_EINVAL
    assert "mode" in _lib.last_error()
    yy = _lib.MpVec(5000, 6000, 4, 4)   # aliases x
    assert _lib.LIB.mpspmv_csr(ctypes.byref(a), ctypes.byref(x), ctypes.byref(yy), 0, None, None) == _lib.MPS_EINVAL
    assert "overlap" in _lib.last_error()


@pytest.mark.parametrize("prec", [64, 96, 3072, 16384, 0])
def test_unsupported_precisions_rejected(prec):
    from paper_1411_2377_amd import _lib
    a = _lib.MpCsr()
    a.row_dim, a.col_dim, a.nnz, a.prec = 1, 1, 0, prec
    a.row_ptr = 1
    assert _lib.LIB.mp_validate_csr(ctypes.byref(a), 0) == _lib.MPS_EINVAL


def test_batched_solver_host_validation():
    from paper_1411_2377_amd import _lib
    a = (_lib.MpCsr * 2)()
    for m in a:
        m.row_dim, m.col_dim, m.nnz, m.prec = 4, 4, 0, 256
        m.row_ptr = 1234
    b = (_lib.MpVec * 2)(_lib.MpVec(1000, 2000, 4, 4), _lib.MpVec(3000, 4000, 4, 4))
    x = (_lib.MpVec * 2)(_lib.MpVec(5000, 6000, 4, 4), _lib.MpVec(7000, 8000, 4, 4))
    o = _lib.MpSolveOpts()
    o.maxit = 10
    info = (_lib.MpSolveInfo * 2)()
    f = _lib.LIB.gpbicg_batched
    assert f(0, a, 1, b, x, ctypes.byref(o), info, None) == _lib.MPS_EINVAL
    assert f(2, a, 0, b, x, ctypes.byref(o), info, None) == _lib.MPS_EINVAL
    o.transpose = 1
    assert f(2, a, 1, b, x, ctypes.byref(o), info, None) == _lib.MPS_ENOTSUP
    o.transpose = 0
    a[1].prec = 128
    assert f(2, a, 1, b, x, ctypes.byref(o), info, None) == _lib.MPS_EINVAL
    assert "precision" in _lib.last_error()
    a[1].prec = 256
    a[1].col_dim = 5
    assert f(2, a, 1, b, x, ctypes.byref(o), info, None) == _lib.MPS_EINVAL
    assert "square" in _lib.last_error()
    a[1].col_dim = 4
    x[1] = _lib.MpVec(3000, 4000, 4, 4)   # aliases b[1]
    assert f(2, a, 1, b, x, ctypes.byref(o), info, None) == _lib.MPS_EINVAL
    assert "overlap" in _lib.last_error()


def test_variant_setter_validation():
    from paper_1411_2377_amd import _lib
    f = _lib.LIB.mp_plan_set_variant
    assert f(None, None, 0, 0, 16, 0) == _lib.MPS_EINVAL
    # the tuners refuse a missing plan or matrix before touching a device
    assert _lib.LIB.mp_plan_tune(None, None, 1, None) == _lib.MPS_EINVAL
    assert _lib.LIB.mp_plan_tune_x(None, None, None, None, 1, None) == _lib.MPS_EINVAL


def test_noalloc_size_limit_rejected_on_the_host():
    """x beyond what the static scratch array stages is refused before anything is enqueued."""
    from paper_1411_2377_amd import _lib
    for prec, max_x in ((128, 1 << 20), (256, 1 << 19), (512, 1 << 18), (1024, 1 << 17)):
        a = _lib.MpCsr()
        a.row_dim, a.col_dim, a.nnz, a.prec = 4, max_x + 1, 0, prec
        a.row_ptr = 1234
        a.val.len, a.val.ld = 0, 0
        x = _lib.MpVec(1 << 40, 1 << 41, max_x + 1, max_x + 1)
        y = _lib.MpVec(1 << 42, 1 << 43, 4, 4)
        assert _lib.LIB.mpspmv_csr_noalloc(ctypes.byref(a), ctypes.byref(x), ctypes.byref(y), 0, None) == _lib.MPS_ENOTSUP
        assert "scratch" in _lib.last_error()
        assert _lib.LIB.mpspmv_csr_noalloc(ctypes.byref(a), ctypes.byref(x), ctypes.byref(y), 5, None) == _lib.MPS_EINVAL
