"""GPU parity of the BiCG, GPBiCG, CGS and BiCGSTAB drivers against the oracle: every iterate is
deterministic, so the final x, the status, the iteration count and the residual history must
agree bit for bit, in both accumulation modes, for every graph chunk size."""
from fractions import Fraction

import numpy as np
import pytest

import synth
from oracle import codec, krylov, mpnum, spmv as ospmv
from tests.util import assert_bitwise

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def lib():
    import paper_1411_2377_amd as M
    return M


class OracleSystem:
    def __init__(self, A_h):
        self.A_h = A_h
        self.p = A_h.vals.p
        self.rp = A_h.row_ptr.tolist()
        self.ci = A_h.col_idx.tolist()
        self.vals = codec.decode(A_h.vals.limbs, A_h.vals.hdr, self.p)
        self.t = ospmv.transpose(A_h.n_rows, A_h.n_cols, self.rp, self.ci, self.vals)

    def mv(self, mode):
        return lambda v: ospmv.spmv(self.rp, self.ci, self.vals, v, self.p, mode)

    def rmv(self, mode):
        tp, ti, tv = self.t
        return lambda v: ospmv.spmv(tp, ti, tv, v, self.p, mode)


def consts(p, rtol, atol):
    c_rel = mpnum.round_fraction(Fraction(rtol[0]) * Fraction(10) ** rtol[1], p)
    c_abs = mpnum.round_fraction(Fraction(atol[0]) * Fraction(10) ** atol[1], p)
    return c_rel, c_abs


def run_both(solver, A_h, b_h, mode, maxit, rtol=(1, -20), atol=(1, -50), transpose=False,
             chunks=(16,), b_oracle=None):
    """Solve on the GPU with b_h and with the oracle with b_oracle (default: b_h decoded)."""
    M = lib()
    p = A_h.vals.p
    A = M.CSRMatrix.from_host(A_h)
    b = M.MPArray.from_host(b_h)
    plan = M.mp_plan_create(A)
    fn = getattr(M, solver)
    outs = []
    for ch in chunks:
        x, info = fn(A, b, plan=plan, mode=mode, maxit=maxit, rtol=rtol, atol=atol, chunk=ch,
                     transpose=transpose, hist=True)
        outs.append((x.to_numpy(), info, info.res_hist.to_numpy()))
    for o in outs[1:]:        # bit-identical for every chunk size (and eager launches)
        assert np.array_equal(o[0][0], outs[0][0][0]) and np.array_equal(o[0][1], outs[0][0][1])
        assert (o[1].status, o[1].iters) == (outs[0][1].status, outs[0][1].iters)
    (xl, xh), info, (hl, hh) = outs[0]
    S = OracleSystem(A_h)
    bo = b_oracle if b_oracle is not None else codec.decode(b_h.limbs, b_h.hdr, p)
    c_rel, c_abs = consts(p, rtol, atol)
    mv, rmv = (S.rmv(mode), S.mv(mode)) if transpose else (S.mv(mode), S.rmv(mode))
    if solver == "bicg":
        ref = krylov.bicg(mv, rmv, bo, c_rel, c_abs, maxit, p)
    else:
        ref = getattr(krylov, solver)(mv, bo, c_rel, c_abs, maxit, p)
    assert (info.status, info.iters) == (ref.status, ref.iters), (info, ref.status, ref.iters)
    assert_bitwise(xl, xh, ref.x, p, what="%s x" % solver)
    if ref.iters:
        assert_bitwise(hl[:, :ref.iters], hh[:ref.iters], ref.res_hist, p, what="%s history" % solver)
    return info, ref


def rhs_ones(A_h):
    """b = RN(A * ones) in EXACT mode, formed by each side on its own; the two must agree.
    Returns (the GPU's b as host arrays, the oracle's b as MP values)."""
    M = lib()
    p = A_h.vals.p
    ones = synth.mp_ones(A_h.n_cols, p)
    A = M.CSRMatrix.from_host(A_h)
    b = M.mpspmv_csr(A, M.MPArray.from_host(ones), mode=1)
    bl, bh = b.to_numpy()
    S = OracleSystem(A_h)
    want = ospmv.spmv_exact(S.rp, S.ci, S.vals, codec.decode(ones.limbs, ones.hdr, p), p)
    assert_bitwise(bl, bh, want, p, what="b = A*1")
    return synth.MPHost(bl, bh, p), want


@pytest.mark.parametrize("solver", ["bicg", "gpbicg", "cgs", "bicgstab"])
@pytest.mark.parametrize("mode", [0, 1], ids=["seq", "exact"])
def test_convdiff_small_fixed_iterations(solver, mode):
    A_h, _ = synth.config2(p=256, m=12)
    b_h, b_o = rhs_ones(A_h)
    run_both(solver, A_h, b_h, mode, maxit=30, rtol=(1, -60), atol=(0, 0), chunks=(7, 0, 1),
             b_oracle=b_o)


@pytest.mark.parametrize("solver", ["bicg", "gpbicg", "cgs", "bicgstab"])
@pytest.mark.parametrize("p", [128, 512, 1024])
def test_convergence_to_tolerance(solver, p):
    A_h, _ = synth.config2(p=p, m=6)
    b_h, b_o = rhs_ones(A_h)
    info, ref = run_both(solver, A_h, b_h, 1, maxit=400, rtol=(1, -20), atol=(1, -50), b_oracle=b_o)
    assert info.status == krylov.CONVERGED


@pytest.mark.parametrize("solver", ["bicg", "gpbicg", "cgs", "bicgstab"])
def test_transposed_solve(solver):
    A_h, _ = synth.config2(p=256, m=8)
    rng = np.random.default_rng(2)
    b_h = synth.mp_uniform(rng, A_h.n_rows, 256)
    run_both(solver, A_h, b_h, 0, maxit=12, rtol=(1, -40), atol=(0, 0), transpose=True)


def test_breakdown_and_not_converged():
    M = lib()
    p = 128
    one = synth.mp_from_ints([1, 1], p)
    A_h = synth.CSRHost(2, 2, np.array([0, 1, 2], np.int32), np.array([1, 0], np.int32), one)
    b_h = synth.mp_from_ints([1, 0], p)
    for solver, want in (("bicg", krylov.BREAKDOWN_SIGMA), ("gpbicg", krylov.BREAKDOWN_SIGMA),
                         ("cgs", krylov.BREAKDOWN_SIGMA), ("bicgstab", krylov.BREAKDOWN_SIGMA)):
        info, ref = run_both(solver, A_h, b_h, 0, maxit=10)
        assert info.status == want and info.iters == 0
    A2, _ = synth.config2(p=p, m=5)
    b2, b2o = rhs_ones(A2)
    info, ref = run_both("bicg", A2, b2, 0, maxit=1, b_oracle=b2o)
    assert info.status == krylov.NOT_CONVERGED and info.iters == 1
    for solver in ("cgs", "bicgstab"):
        info, ref = run_both(solver, A2, b2, 1, maxit=1, b_oracle=b2o)
        assert info.status == krylov.NOT_CONVERGED and info.iters == 1
    # a zero right-hand side meets the test at once
    z = synth.mp_zeros(A2.n_rows, p)
    for solver in ("gpbicg", "cgs", "bicgstab"):
        info, ref = run_both(solver, A2, z, 0, maxit=5)
        assert info.status == krylov.CONVERGED and info.iters == 0


def test_bicgstab_omega_zero_cases():
    """(t, t) = 0 gives omega = 0: on A = I the first half step already solves (one iteration,
    converged); on the singular A = [[1, 1], [0, 0]] with b = (1, 1), A s = 0 with s != 0 ends
    in the omega = 0 exit."""
    p = 256
    I3 = synth.CSRHost(3, 3, np.array([0, 1, 2, 3], np.int32), np.array([0, 1, 2], np.int32),
                       synth.mp_from_ints([1, 1, 1], p))
    info, ref = run_both("bicgstab", I3, synth.mp_from_ints([2, 3, 4], p), 0, maxit=10)
    assert info.status == krylov.CONVERGED and info.iters == 1
    sing = synth.CSRHost(2, 2, np.array([0, 2, 2], np.int32), np.array([0, 1], np.int32),
                         synth.mp_from_ints([1, 1], p))
    info, ref = run_both("bicgstab", sing, synth.mp_from_ints([1, 1], p), 1, maxit=10)
    assert info.status == krylov.BREAKDOWN_ZETA and info.iters == 1


@pytest.mark.parametrize("solver", ["bicg", "gpbicg"])
@pytest.mark.parametrize("mode", [0, 1], ids=["seq", "exact"])
def test_convdiff_full_size_first_iterations(solver, mode):
    """The 256 x 256 convection-diffusion workload at p = 256: the first two iterations in full."""
    A_h, _ = synth.config2()
    b_h, b_o = rhs_ones(A_h)
    run_both(solver, A_h, b_h, mode, maxit=2, rtol=(1, -20), atol=(1, -50), b_oracle=b_o)


@pytest.mark.parametrize("solver", ["bicg", "gpbicg", "cgs", "bicgstab"])
def test_scaled_3d_ill_conditioned_iterates(solver):
    """The row-scaled 3-D operator (d_i = 10^u, u ~ U(-15, 15); condition about 1e30) at
    p = 512 on an 8^3 grid: 40 iterations bit-identical to the oracle in EXACT mode."""
    A_h, xs_h, _ = synth.config5(p=512, m=8)
    M = lib()
    A = M.CSRMatrix.from_host(A_h)
    b = M.mpspmv_csr(A, M.MPArray.from_host(xs_h), mode=1)
    bl, bh = b.to_numpy()
    S = OracleSystem(A_h)
    b_o = ospmv.spmv_exact(S.rp, S.ci, S.vals, codec.decode(xs_h.limbs, xs_h.hdr, 512), 512)
    assert_bitwise(bl, bh, b_o, 512, what="b = A x*")
    run_both(solver, A_h, synth.MPHost(bl, bh, 512), 1, maxit=40, rtol=(1, -100), atol=(0, 0),
             b_oracle=b_o)


def test_profiled_solve_same_bits_and_counts():
    """A profiled solve (eager launches, timing events attached to the kernels) gives the bits
    of a graph-replayed one and counts every iteration kernel in its class: BiCG one fused SpMV,
    one A^T product, one direction and one update step per iteration; GPBiCG two fused SpMVs,
    one direction, one update and one t/s/y step; CGS one fused and one plain SpMV, one
    direction, one q/u^/x and one residual step; BiCGSTAB two fused SpMVs, one direction, one s
    and one x/r step."""
    M = lib()
    A_h, _ = synth.config2(p=256, m=12)
    b_h, _ = rhs_ones(A_h)
    A = M.CSRMatrix.from_host(A_h)
    b = M.MPArray.from_host(b_h)
    plan = M.mp_plan_create(A)
    for fn, per in ((M.bicg, (1, 1, 1, 1, 0)), (M.gpbicg, (2, 0, 1, 1, 1)), (M.cgs, (1, 1, 1, 1, 1)),
                    (M.bicgstab, (2, 0, 1, 1, 1))):
        for mode in (0, 1):
            kw = dict(plan=plan, mode=mode, maxit=10, rtol=(1, -60), atol=(0, 0))
            x0, i0 = fn(A, b, chunk=4, **kw)
            pr = M.SolveProfile()
            x1, i1 = fn(A, b, profile=pr, **kw)
            assert (i0.status, i0.iters) == (i1.status, i1.iters) == (krylov.NOT_CONVERGED, 10)
            (l0, h0), (l1, h1) = x0.to_numpy(), x1.to_numpy()
            assert np.array_equal(l0, l1) and np.array_equal(h0, h1)
            assert list(pr.launches) == [k * i1.iters for k in per], list(pr.launches)
            assert all((pr.us[k] > 0) == (per[k] > 0) for k in range(5))
