"""The wide precisions (p = 2048, 4096, 8192: numbers spread over a wavefront's lanes) against the
oracle, bit for bit: the sparse product in both modes and its transpose on edge-case rows, the
exact inner product (including an exact cancellation), y + alpha x, decimal constants, and BiCG,
GPBiCG, CGS and BiCGSTAB (every iterate, status and residual history; also the transposed system
and the breakdown exits)."""
from fractions import Fraction

import numpy as np
import pytest

import synth
from oracle import blas, codec, krylov, mpnum, spmv as ospmv
from tests.test_gpu_solvers import rhs_ones, run_both
from tests.test_gpu_spmv import edge_problem
from tests.util import assert_bitwise, oracle_spmv_rows

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

WIDE = [2048, 4096, 8192]


def lib():
    import paper_1411_2377_amd as M
    return M


@pytest.mark.parametrize("p", WIDE)
@pytest.mark.parametrize("mode", [0, 1], ids=["seq", "exact"])
def test_wide_product_and_transpose(p, mode):
    """Edge-case rows (empty, single, > 128 entries, stored zeros, -0, spreads up to 2000 bits,
    exact cancellations, all-ones mantissas): A x and A^T g against the oracle."""
    M = lib()
    A_h, x_h = edge_problem(p, seed=p + mode, n=45, m=60)
    A = M.CSRMatrix.from_host(A_h)
    y = M.mpspmv_csr(A, M.MPArray.from_host(x_h), mode=mode)
    yl, yh = y.to_numpy()
    assert_bitwise(yl, yh, oracle_spmv_rows(A_h, x_h, np.arange(A_h.n_rows), mode), p, what="A x p=%d" % p)
    g_h = synth.mp_uniform(np.random.default_rng(p), A_h.n_rows, p)
    P = M.mp_plan_create(A)
    t = M.mpspmv_csr_t(A, P, M.MPArray.from_host(g_h), mode=mode)
    tl, th = t.to_numpy()
    vals = codec.decode(A_h.vals.limbs, A_h.vals.hdr, p)
    want = ospmv.spmv_t(A_h.n_rows, A_h.n_cols, A_h.row_ptr.tolist(), A_h.col_idx.tolist(), vals,
                        codec.decode(g_h.limbs, g_h.hdr, p), p, mode)
    assert_bitwise(tl, th, want, p, what="A^T g p=%d" % p)
    assert M.mp_status() == 0


@pytest.mark.parametrize("p", WIDE)
def test_wide_dot_axpy_constants(p):
    M = lib()
    rng = np.random.default_rng(p + 1)
    n = 150
    x_h = synth.mp_uniform(rng, n, p)
    y_h = synth.mp_loguniform(rng, n, p, -40, 40)
    y_h.hdr[::13] = np.int32(-(1 << 31)) + (np.arange(len(y_h.hdr[::13])) % 2).astype(np.int32)  # +-0
    xo, yo = codec.decode(x_h.limbs, x_h.hdr, p), codec.decode(y_h.limbs, y_h.hdr, p)
    x, y = M.MPArray.from_host(x_h), M.MPArray.from_host(y_h)
    d = M.mp_dot(x, y).to_numpy()
    assert_bitwise(d[0], d[1], [blas.dot(xo, yo, p)], p, what="dot")
    # an exactly cancelling inner product: x . [y, -y] on [x, x] is +0
    xx = synth.mp_concat([x_h, x_h])
    yy = synth.mp_concat([y_h, synth.MPHost(y_h.limbs.copy(), y_h.hdr ^ np.int32(1), p)])
    d0 = M.mp_dot(M.MPArray.from_host(xx), M.MPArray.from_host(yy)).to_numpy()
    assert d0[1][0] == np.int32(-(1 << 31))
    a_h = synth.mp_uniform(rng, 1, p)
    M.mp_axpy(M.MPArray.from_host(a_h), x, y)
    yl, yh = y.to_numpy()
    assert_bitwise(yl, yh, blas.axpy(codec.decode(a_h.limbs, a_h.hdr, p)[0], xo, yo), p, what="axpy")
    for m_, e_ in ((1, -20), (1, -200), (-3, 7), (123456789, -3), (0, 5)):
        c = M.mp_const_decimal(m_, e_, p).to_numpy()
        want = mpnum.round_fraction(Fraction(m_) * Fraction(10) ** e_, p)
        assert_bitwise(c[0], c[1], [want], p, what="const %d e%d" % (m_, e_))
    assert M.mp_status() == 0


@pytest.mark.parametrize("p", WIDE)
@pytest.mark.parametrize("mode", [0, 1], ids=["seq", "exact"])
def test_wide_bicg_matches_oracle(p, mode):
    """BiCG on the 5 x 5 convection-diffusion operator, b = A * ones, to a relative 1e-200."""
    A_h, _ = synth.config2(p=p, m=5)
    b_h, b_o = rhs_ones(A_h)
    info, ref = run_both("bicg", A_h, b_h, mode, maxit=60, rtol=(1, -200), atol=(0, 0), b_oracle=b_o)
    assert info.status == 0


@pytest.mark.parametrize("solver", ["gpbicg", "cgs", "bicgstab"])
@pytest.mark.parametrize("p", WIDE)
@pytest.mark.parametrize("mode", [0, 1], ids=["seq", "exact"])
def test_wide_product_type_methods_match_oracle(solver, p, mode):
    """GPBiCG, CGS and BiCGSTAB on the 5 x 5 convection-diffusion operator, b = A * ones, to a
    relative 1e-200: every iterate, the status and the residual history bit for bit."""
    A_h, _ = synth.config2(p=p, m=5)
    b_h, b_o = rhs_ones(A_h)
    info, ref = run_both(solver, A_h, b_h, mode, maxit=80, rtol=(1, -200), atol=(0, 0), b_oracle=b_o)
    assert info.status == 0


@pytest.mark.parametrize("solver", ["bicg", "gpbicg", "cgs", "bicgstab"])
def test_wide_transposed_and_limit(solver):
    """A^T x = b at p = 2048 (iterates and history), and the iteration limit (NC)."""
    p = 2048
    A_h, _ = synth.config2(p=p, m=4)
    b_h = synth.mp_uniform(np.random.default_rng(5), A_h.n_rows, p)
    run_both(solver, A_h, b_h, 1, maxit=40, rtol=(1, -150), atol=(0, 0), transpose=True)
    info, ref = run_both(solver, A_h, b_h, 0, maxit=3, rtol=(1, -150), atol=(0, 0))
    assert info.status == 1 and info.iters == 3


def test_wide_breakdowns_zero_rhs_and_unsupported():
    """The sigma breakdown on the 2 x 2 swap matrix, BiCGSTAB's omega = 0 exit on a singular
    matrix, a zero right-hand side (converged after 0 iterations), and an entry point the wide
    path does not provide (the ILU(0)-preconditioned BiCGSTAB), refused."""
    M = lib()
    p = 4096
    one = synth.mp_from_ints([1, 1], p)
    swap = synth.CSRHost(2, 2, np.array([0, 1, 2], np.int32), np.array([1, 0], np.int32), one)
    for solver in ("bicg", "gpbicg", "cgs", "bicgstab"):
        info, ref = run_both(solver, swap, synth.mp_from_ints([1, 0], p), 0, maxit=10)
        assert info.status == krylov.BREAKDOWN_SIGMA and info.iters == 0
    sing = synth.CSRHost(2, 2, np.array([0, 2, 2], np.int32), np.array([0, 1], np.int32), one)
    info, ref = run_both("bicgstab", sing, synth.mp_from_ints([1, 1], p), 1, maxit=10)
    assert info.status == krylov.BREAKDOWN_ZETA and info.iters == 1
    A_h, _ = synth.config2(p=p, m=3)
    z = synth.mp_zeros(A_h.n_rows, p)
    for solver in ("gpbicg", "cgs", "bicgstab"):
        info, ref = run_both(solver, A_h, z, 0, maxit=5)
        assert info.status == krylov.CONVERGED and info.iters == 0
    A = M.CSRMatrix.from_host(A_h)
    with pytest.raises(M.MPError):
        M.ILU0(A)
    M.mp_status(raise_on_error=False)
