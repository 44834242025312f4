"""The dense multiple-precision product (mp_gemv: the paper's dense MV with zeros stored, Sec. 3)
on the Lotkin-with-zeros workload, bit for bit: against the oracle's dense product in full at
moderate size, against the sparse product of the same matrix without its zeros at the
benchmark's size, on rectangular and empty shapes."""
import numpy as np
import pytest

import synth
from oracle import codec, dense
from tests.util import assert_bitwise

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def lib():
    import paper_1411_2377_amd as M
    return M


def gemv(M, D_h, rows, cols, x_h, mode):
    D = M.MPArray.from_host(D_h)
    y = M.mp_gemv(D, rows, cols, M.MPArray.from_host(x_h), mode=mode)
    return y.to_numpy()


@pytest.mark.parametrize("p", [128, 256, 512])
@pytest.mark.parametrize("mode", [0, 1], ids=["seq", "exact"])
@pytest.mark.parametrize("zero_pct", [0.0, 50.0, 90.0, 99.0])
def test_lotkin_dense_matches_oracle(p, mode, zero_pct):
    M = lib()
    n = 260 if p < 512 else 130
    D_h, C_h, x_h = synth.lotkin(n, p, zero_pct, seed=int(zero_pct) + p)
    yl, yh = gemv(M, D_h, n, n, x_h, mode)
    want = dense.gemv(n, n, codec.decode(D_h.limbs, D_h.hdr, p), codec.decode(x_h.limbs, x_h.hdr, p), p, mode)
    assert_bitwise(yl, yh, want, p, what="Lotkin n=%d, %g%% zeros" % (n, zero_pct))
    assert M.mp_status() == 0


@pytest.mark.parametrize("mode", [0, 1], ids=["seq", "exact"])
def test_lotkin_benchmark_size_dense_equals_sparse(mode):
    """n = 2000 (4M stored elements), 90% zeros, p = 256: b = A [1..n] by the sparse product,
    then A b by the dense and by the sparse product, which must agree bit for bit; sampled rows
    of A b against the oracle."""
    M = lib()
    p, n = 256, 2000
    D_h, C_h, x_h = synth.lotkin(n, p, 90.0, seed=11)
    A = M.CSRMatrix.from_host(C_h)
    D = M.MPArray.from_host(D_h)
    b = M.mpspmv_csr(A, M.MPArray.from_host(x_h), mode=mode)
    y_s = M.mpspmv_csr(A, b, mode=mode).to_numpy()
    y_d = M.mp_gemv(D, n, n, b, mode=mode).to_numpy()
    assert np.array_equal(y_s[0], y_d[0]) and np.array_equal(y_s[1], y_d[1])
    rows = np.array([0, 1, 2, 999, n - 1] + list(np.random.default_rng(0).integers(0, n, 12)))
    rows = np.unique(rows)
    bl, bh = b.to_numpy()
    bo = codec.decode(bl, bh, p)
    vals = codec.decode(D_h.limbs, D_h.hdr, p)
    want = []
    for i in rows:
        want += dense.gemv(1, n, vals[i * n:(i + 1) * n], bo, p, mode)
    assert_bitwise(y_d[0][:, rows], y_d[1][rows], want, p, what="A b rows")
    assert M.mp_status() == 0


def test_rectangular_and_empty():
    M = lib()
    p = 256
    rng = np.random.default_rng(5)
    rows, cols = 77, 513
    a = synth.mp_uniform(rng, rows * cols, p)
    a.hdr[rng.permutation(rows * cols)[:rows * cols // 3]] = synth.ZERO_HDR
    x = synth.mp_uniform(rng, cols, p)
    vals, xv = codec.decode(a.limbs, a.hdr, p), codec.decode(x.limbs, x.hdr, p)
    for mode in (0, 1):
        yl, yh = gemv(M, a, rows, cols, x, mode)
        assert_bitwise(yl, yh, dense.gemv(rows, cols, vals, xv, p, mode), p, what="77 x 513")
    # no columns: y = +0; no rows: nothing to do
    y = M.mp_gemv(M.MPArray.empty(0, p), 5, 0, M.MPArray.empty(0, p), mode=0).to_numpy()
    assert np.all(y[1] == np.int32(-(1 << 31)))
    M.mp_gemv(M.MPArray.empty(0, p), 0, 4, M.MPArray.from_host(synth.mp_ones(4, p)), mode=1)
    assert M.mp_status() == 0
