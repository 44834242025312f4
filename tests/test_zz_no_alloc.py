"""The allocation-free product (mpspmv_csr_noalloc: x staged in the library's static scratch
array, no allocation in the call) against mpspmv_csr, bit for bit, through the C ABI: two calls
in a row at every precision and mode, the second on a smaller matrix; the edge-case matrices;
the power-law workload at full size (x of 500000 elements at p = 256, near the array's limit)."""
import ctypes

import pytest

import synth
from tests.test_gpu_spmv import edge_problem

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def lib():
    import paper_1411_2377_amd as M
    return M


def noalloc(M, A, x, y, mode):
    """One call of the C entry point into the caller's y; returns its status code."""
    a, xd, yd = A.desc(), x.desc(), y.desc()
    return M._lib.LIB.mpspmv_csr_noalloc(ctypes.byref(a), ctypes.byref(xd), ctypes.byref(yd),
                                         int(mode), M.api._stream(None))


def same_as_plain(M, A_h, x_h, mode):
    A = M.CSRMatrix.from_host(A_h)
    x = M.MPArray.from_host(x_h)
    y = M.MPArray.empty(A.n_rows, A.p)
    assert noalloc(M, A, x, y, mode) == 0, M.mp_last_error()
    want = M.mpspmv_csr(A, x, mode=mode)
    assert torch.equal(y.hdr, want.hdr) and torch.equal(y.limbs, want.limbs), \
        "allocation-free product differs from mpspmv_csr (n=%d, p=%d, mode %d)" % (A.n_rows, A.p, mode)


@pytest.mark.parametrize("p", [128, 256, 512, 1024])
@pytest.mark.parametrize("mode", [0, 1], ids=["seq", "exact"])
def test_two_calls_second_smaller(p, mode):
    M = lib()
    same_as_plain(M, *synth.config1(p=p, seed=11, n=5000, per_row=12), mode)
    same_as_plain(M, *synth.config1(p=p, seed=12, n=700, per_row=5), mode)
    same_as_plain(M, *edge_problem(p, seed=3 * p + mode), mode)
    assert M.mp_status() == 0


def test_powerlaw_full_then_small():
    M = lib()
    A_h, x_h, _ = synth.config3(p=256)
    for mode in (0, 1):
        same_as_plain(M, A_h, x_h, mode)
    same_as_plain(M, *synth.config1(p=256, seed=13, n=300, per_row=7), 0)
    assert M.mp_status() == 0
