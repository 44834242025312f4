"""ILU(0) on the GPU against the oracle, bit for bit: the factors (row-wise, one RN per
operation), the preconditioner's applications K^{-1} r and K^{-T} r in both accumulation modes,
and BiCGSTAB and BiCG preconditioned by it (every iterate, status, residual history, every chunk
size)."""
from fractions import Fraction
import random

import numpy as np
import pytest

import synth
from oracle import codec, ilu, krylov, mpnum, spmv as ospmv
from tests.util import assert_bitwise

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def lib():
    import paper_1411_2377_amd as M
    return M


def rand_pattern(seed, n, p, density=0.08, dominance=True):
    """Random sparse matrix with every diagonal stored; off-diagonals uniform [-1, 1]; diagonally
    dominant (or not) by construction on the host (no MP arithmetic: the diagonal is a chopped
    rational)."""
    rng = np.random.default_rng(seed)
    rows, cols = [], []
    for i in range(n):
        cs = set(rng.choice(n, size=max(1, int(density * n)), replace=False).tolist()) | {i}
        for j in sorted(cs):
            rows.append(i)
            cols.append(j)
    rows, cols = np.array(rows), np.array(cols)
    vals = synth.mp_uniform(rng, len(rows), p)
    diag = np.flatnonzero(rows == cols)
    k = np.bincount(rows, minlength=n)
    dvals = synth.mp_from_rationals([(int(c) + 3, 1) if dominance else (1, 1) for c in k], p)
    vals.limbs[:, diag] = dvals.limbs
    vals.hdr[diag] = dvals.hdr
    rp = np.zeros(n + 1, np.int32)
    np.add.at(rp, rows + 1, 1)
    rp = np.cumsum(rp).astype(np.int32)
    return synth.CSRHost(n, n, rp, cols.astype(np.int32), vals)


def oracle_factors(A_h):
    p = A_h.vals.p
    vals = codec.decode(A_h.vals.limbs, A_h.vals.hdr, p)
    return ilu.ilu0(A_h.n_rows, A_h.row_ptr.tolist(), A_h.col_idx.tolist(), vals)


CASES = {
    "convdiff2d_24": lambda p: synth.config2(p=p, m=24)[0],
    "random_300": lambda p: rand_pattern(1, 300, p),
}


@pytest.mark.parametrize("p", [128, 256, 512, 1024])
@pytest.mark.parametrize("case", ["convdiff2d_24", "random_300"])
def test_factors_and_application(case, p):
    M = lib()
    A_h = CASES[case](p)
    n = A_h.n_rows
    A = M.CSRMatrix.from_host(A_h)
    K = M.ILU0(A)
    lu = oracle_factors(A_h)
    gl, gh = K.factors().to_numpy()
    assert_bitwise(gl, gh, lu, p, what="ILU(0) factors, %s" % case)
    r_h = synth.mp_uniform(np.random.default_rng(p), n, p)
    ro = codec.decode(r_h.limbs, r_h.hdr, p)
    rp, ci = A_h.row_ptr.tolist(), A_h.col_idx.tolist()
    r = M.MPArray.from_host(r_h)
    for mode in (0, 1):
        wl, wh = K.apply(r, mode=mode).to_numpy()
        assert_bitwise(wl, wh, ilu.apply(n, rp, ci, lu, ro, p, mode), p, what="K^-1 r mode %d" % mode)
        wl, wh = K.apply_t(r, mode=mode).to_numpy()
        assert_bitwise(wl, wh, ilu.apply_t(n, rp, ci, lu, ro, p, mode), p, what="K^-T r mode %d" % mode)
    assert M.mp_status() == 0


def test_factors_at_larger_size():
    """The 2-D convection-diffusion operator on a 96 x 96 grid (191 dependency levels), p = 256."""
    M = lib()
    A_h, _ = synth.config2(p=256, m=96)
    A = M.CSRMatrix.from_host(A_h)
    K = M.ILU0(A)
    gl, gh = K.factors().to_numpy()
    assert_bitwise(gl, gh, oracle_factors(A_h), 256, what="ILU(0) factors 96 x 96")


@pytest.mark.parametrize("mode", [0, 1], ids=["seq", "exact"])
def test_preconditioned_bicgstab_matches_oracle(mode):
    M = lib()
    p = 256
    A_h, _ = synth.config2(p=p, m=10)
    n = A_h.n_rows
    rp, ci = A_h.row_ptr.tolist(), A_h.col_idx.tolist()
    vals = codec.decode(A_h.vals.limbs, A_h.vals.hdr, p)
    xs = synth.mp_arange1(n, p)
    A = M.CSRMatrix.from_host(A_h)
    b = M.mpspmv_csr(A, M.MPArray.from_host(xs), mode=1)
    bo = ospmv.spmv_exact(rp, ci, vals, codec.decode(xs.limbs, xs.hdr, p), p)
    bl, bh = b.to_numpy()
    assert_bitwise(bl, bh, bo, p, what="b")
    K = M.ILU0(A)
    lu = ilu.ilu0(n, rp, ci, vals)
    c_rel = mpnum.round_fraction(Fraction(1, 10 ** 60), p)
    ref = krylov.bicgstab_precond(lambda v: ospmv.spmv(rp, ci, vals, v, p, mode),
                                  lambda v: ilu.apply(n, rp, ci, lu, v, p, mode), bo, c_rel,
                                  mpnum.zero(p), 100, p)
    assert ref.status == krylov.CONVERGED
    outs = []
    for chunk in (7, 0):
        x, info = M.bicgstab_ilu0(A, K, b, mode=mode, maxit=100, rtol=(1, -60), atol=(0, 0), chunk=chunk,
                                  hist=True)
        assert (info.status, info.iters) == (ref.status, ref.iters)
        xl, xh = x.to_numpy()
        assert_bitwise(xl, xh, ref.x, p, what="x")
        hl, hh = info.res_hist.to_numpy()
        assert_bitwise(hl[:, :ref.iters], hh[:ref.iters], ref.res_hist, p, what="history")
        outs.append(info.iters)
    plain = krylov.bicgstab(lambda v: ospmv.spmv(rp, ci, vals, v, p, mode), bo, c_rel, mpnum.zero(p), 200, p)
    assert ref.iters < plain.iters
    assert M.mp_status() == 0


@pytest.mark.parametrize("mode", [0, 1], ids=["seq", "exact"])
@pytest.mark.parametrize("case", ["convdiff2d_10", "random_120"])
def test_preconditioned_bicg_matches_oracle(case, mode):
    M = lib()
    p = 256
    A_h = synth.config2(p=p, m=10)[0] if case == "convdiff2d_10" else rand_pattern(5, 120, p, density=0.05)
    n = A_h.n_rows
    rp, ci = A_h.row_ptr.tolist(), A_h.col_idx.tolist()
    vals = codec.decode(A_h.vals.limbs, A_h.vals.hdr, p)
    xs = synth.mp_arange1(n, p)
    A = M.CSRMatrix.from_host(A_h)
    b = M.mpspmv_csr(A, M.MPArray.from_host(xs), mode=1)
    bo = ospmv.spmv_exact(rp, ci, vals, codec.decode(xs.limbs, xs.hdr, p), p)
    K = M.ILU0(A)
    lu = ilu.ilu0(n, rp, ci, vals)
    tp, ti, tv = ospmv.transpose(n, n, rp, ci, vals)
    c_rel = mpnum.round_fraction(Fraction(1, 10 ** 60), p)
    ref = krylov.bicg_precond(lambda v: ospmv.spmv(rp, ci, vals, v, p, mode),
                              lambda v: ospmv.spmv(tp, ti, tv, v, p, mode),
                              lambda v: ilu.apply(n, rp, ci, lu, v, p, mode),
                              lambda v: ilu.apply_t(n, rp, ci, lu, v, p, mode), bo, c_rel,
                              mpnum.zero(p), 150, p)
    assert ref.status == krylov.CONVERGED
    plan = M.Plan(A)
    for chunk in (5, 0):
        x, info = M.bicg_ilu0(A, K, b, plan=plan if chunk else None, mode=mode, maxit=150, rtol=(1, -60),
                              atol=(0, 0), chunk=chunk, hist=True)
        assert (info.status, info.iters) == (ref.status, ref.iters)
        xl, xh = x.to_numpy()
        assert_bitwise(xl, xh, ref.x, p, what="x")
        hl, hh = info.res_hist.to_numpy()
        assert_bitwise(hl[:, :ref.iters], hh[:ref.iters], ref.res_hist, p, what="history")
    assert M.mp_status() == 0


def test_preconditioned_bicg_limits():
    """maxit reached (NC after exactly maxit iterations, iterate as the oracle's), and the
    transposed system refused."""
    M = lib()
    p = 128
    A_h = synth.config2(p=p, m=6)[0]
    n = A_h.n_rows
    rp, ci = A_h.row_ptr.tolist(), A_h.col_idx.tolist()
    vals = codec.decode(A_h.vals.limbs, A_h.vals.hdr, p)
    A = M.CSRMatrix.from_host(A_h)
    bh = synth.mp_uniform(np.random.default_rng(3), n, p)
    b = M.MPArray.from_host(bh)
    K = M.ILU0(A)
    lu = ilu.ilu0(n, rp, ci, vals)
    tp, ti, tv = ospmv.transpose(n, n, rp, ci, vals)
    c_rel = mpnum.round_fraction(Fraction(1, 10 ** 30), p)
    ref = krylov.bicg_precond(lambda v: ospmv.spmv(rp, ci, vals, v, p, 0),
                              lambda v: ospmv.spmv(tp, ti, tv, v, p, 0),
                              lambda v: ilu.apply(n, rp, ci, lu, v, p, 0),
                              lambda v: ilu.apply_t(n, rp, ci, lu, v, p, 0),
                              codec.decode(bh.limbs, bh.hdr, p), c_rel, mpnum.zero(p), 3, p)
    assert ref.status == krylov.NOT_CONVERGED and ref.iters == 3
    x, info = M.bicg_ilu0(A, K, b, mode=0, maxit=3, rtol=(1, -30), atol=(0, 0), chunk=2)
    assert (info.status, info.iters) == (ref.status, ref.iters)
    xl, xh = x.to_numpy()
    assert_bitwise(xl, xh, ref.x, p, what="x after maxit")
    with pytest.raises(M.MPError):
        M.bicg_ilu0(A, K, b, mode=0, maxit=3, transpose=True)
    M.mp_status(raise_on_error=False)


def test_missing_diagonal_and_zero_pivot():
    M = lib()
    p = 128
    # row 1 stores no diagonal element
    A_h = synth.CSRHost(2, 2, np.array([0, 1, 2], np.int32), np.array([0, 0], np.int32),
                        synth.mp_from_ints([2, 1], p))
    with pytest.raises(M.MPError):
        M.ILU0(M.CSRMatrix.from_host(A_h))
    # a zero pivot: [[0, 1], [1, 1]] stores a zero diagonal in row 0
    A2 = synth.CSRHost(2, 2, np.array([0, 2, 4], np.int32), np.array([0, 1, 0, 1], np.int32),
                       synth.mp_from_ints([0, 1, 1, 1], p))
    with pytest.raises(M.MPError):
        M.ILU0(M.CSRMatrix.from_host(A2))
    M.mp_status(raise_on_error=False)
