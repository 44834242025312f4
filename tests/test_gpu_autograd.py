"""Autograd wrappers: gradients bit-identical to the oracle's (A^T g, RN(g_i x_j), the adjoint
solve), central finite differences on the power-law workload, and the one-use limit."""
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


def packed(M, h):
    return M.autograd.pack(M.MPArray.from_host(h)).requires_grad_(True)


def bits_equal(a, b):
    """Packed MP tensors compared bit for bit (their float32 view may hold NaN patterns)."""
    return torch.equal(a.view(torch.int32), b.view(torch.int32))


def to_np(M, t, p):
    return M.autograd.unpack(t.detach(), p).to_numpy()


@pytest.mark.parametrize("mode", [0, 1], ids=["seq", "exact"])
@pytest.mark.parametrize("p", [128, 512])
def test_spmv_backward_matches_oracle(mode, p):
    M = lib()
    A_h, x_h = synth.config1(p=p, n=300, per_row=9)
    g_h = synth.mp_uniform(np.random.default_rng(7), A_h.n_rows, p)
    A = M.CSRMatrix.from_host(A_h)
    S = M.autograd.SparseStructure.of(A)
    vt, xt = packed(M, A_h.vals), packed(M, x_h)
    y = M.autograd.spmv(S, vt, xt, mode)
    y.backward(M.autograd.pack(M.MPArray.from_host(g_h)))
    gl, gh = to_np(M, xt.grad, p)
    vl, vh = to_np(M, vt.grad, p)
    rp, ci = A_h.row_ptr.tolist(), A_h.col_idx.tolist()
    vals = codec.decode(A_h.vals.limbs, A_h.vals.hdr, p)
    go = codec.decode(g_h.limbs, g_h.hdr, p)
    xo = codec.decode(x_h.limbs, x_h.hdr, p)
    assert_bitwise(gl, gh, ospmv.spmv_t(A_h.n_rows, A_h.n_cols, rp, ci, vals, go, p, mode), p, what="grad x")
    assert_bitwise(vl, vh, ospmv.grad_vals(rp, ci, go, xo, p), p, what="grad vals")
    yl, yh = to_np(M, y, p)
    assert_bitwise(yl, yh, ospmv.spmv(rp, ci, vals, xo, p, mode), p, what="forward")


def test_second_use_raises():
    M = lib()
    A_h, x_h = synth.config1(p=128, n=64, per_row=3)
    A = M.CSRMatrix.from_host(A_h)
    S = M.autograd.SparseStructure.of(A)
    vt, xt = packed(M, A_h.vals), packed(M, x_h)
    y = M.autograd.spmv(S, vt, xt, 0)      # kept alive: its graph node still holds vt
    with pytest.raises(RuntimeError):
        M.autograd.spmv(S, vt, packed(M, x_h), 0)
    assert y.requires_grad


def loss(M, A, x, g):
    """<g, A x> (EXACT product, exact inner product) as a Fraction."""
    y = M.mpspmv_csr(A, x, mode=1)
    d = M.mp_dot(g, y).to_numpy()
    return codec.decode(d[0], d[1], x.p)[0].to_fraction()


@pytest.mark.parametrize("p", [128, 256, 512])
def test_finite_differences_powerlaw(p):
    """Central differences of L(x, a) = <g, A x> on the power-law workload (n = 500000, mean
    20 / max 2000 entries per row): the loss is linear, so the difference quotient equals the
    gradient up to rounding.  Each L carries at most 2^-p sum_i |g_i y_i| from rounding y_i
    (EXACT mode) plus 2^-p |L| from the inner product, so
    |FD - grad| <= 2^-p (4 sum_i |g_i y_i| / |v+ - v-| + |grad|)."""
    M = lib()
    A_h, x_h, g_h = synth.config3(p=p)
    A = M.CSRMatrix.from_host(A_h)
    S = M.autograd.SparseStructure.of(A)
    vt, xt = packed(M, A_h.vals), packed(M, x_h)
    y = M.autograd.spmv(S, vt, xt, 1)
    y.backward(M.autograd.pack(M.MPArray.from_host(g_h)))
    gx = to_np(M, xt.grad, p)
    gv = to_np(M, vt.grad, p)
    g = M.MPArray.from_host(g_h)
    rng = np.random.default_rng(p)
    u = Fraction(1, 2 ** p)
    yl, yh = to_np(M, y, p)
    # sum_i |g_i y_i| in double is enough for a bound (relative slack 2^-40 is added)
    gd = np.array([float(v.to_fraction()) for v in codec.decode(g_h.limbs, g_h.hdr, p)])
    ydd = np.array([float(v.to_fraction()) for v in codec.decode(yl, yh, p)])
    s_abs = Fraction(float(np.sum(np.abs(gd * ydd)) * (1 + 2.0 ** -40)))

    xdev = M.MPArray.from_host(x_h)

    def fd(kind, idx):
        """(L(v + h) - L(v - h)) / (2h) with the entry changed in place on the device."""
        base = x_h if kind == "x" else A_h.vals
        dev = xdev if kind == "x" else A.vals
        v = codec.decode(base.limbs[:, [idx]], base.hdr[[idx]], p)[0]
        h = mpnum.MP(0, 1 << (p - 1), v.e - 12, p) if v.m else mpnum.round_fraction(Fraction(1, 2 ** 40), p)
        out = []
        for nv in (mpnum.add(v, h), mpnum.sub(v, h)):
            l, hh = codec.encode([nv], p)
            dev.limbs[:, idx] = torch.from_numpy(l[:, 0].view(np.int32)).to(dev.limbs.device)
            dev.hdr[idx] = int(hh[0])
            out.append((loss(M, A, xdev, g), nv))
        l, hh = codec.encode([v], p)
        dev.limbs[:, idx] = torch.from_numpy(l[:, 0].view(np.int32)).to(dev.limbs.device)
        dev.hdr[idx] = int(hh[0])
        (lp, vp), (lm, vm) = out
        dv = vp.to_fraction() - vm.to_fraction()
        return (lp - lm) / dv, 4 * u * s_abs / abs(dv)
    lengths = np.diff(A_h.row_ptr)
    for j in list(rng.integers(0, A_h.n_cols, 6)):
        want = codec.decode(gx[0][:, [j]], gx[1][[j]], p)[0].to_fraction()
        got, slack = fd("x", int(j))
        assert abs(got - want) <= slack + u * abs(want), (j, float(got), float(want))
    ks = list(rng.integers(0, A_h.nnz, 6)) + [int(A_h.row_ptr[int(np.argmax(lengths))])]
    for k in ks:
        want = codec.decode(gv[0][:, [k]], gv[1][[k]], p)[0].to_fraction()
        got, slack = fd("a", int(k))
        assert abs(got - want) <= slack + u * abs(want), (k, float(got), float(want))
        assert abs(got - want) <= abs(want) * Fraction(1, 2 ** (p // 3))   # and well inside p/3 bits


def approx_abs(h):
    """|v| of a host MP array in double, from the top limb (relative error below 2^-31)."""
    e = (h.hdr >> 1).astype(np.int64)
    top = h.limbs[h.limbs.shape[0] - 1].astype(np.float64)
    v = np.ldexp(top, (e - 32).clip(-1000, 1000))
    return np.where(h.hdr == np.int32(-(1 << 31)), 0.0, v)


def test_finite_differences_powerlaw_seq():
    """SEQ mode on the power-law workload at p = 256: the gradient of L(x) = <g, A x> (A^T g in
    SEQ order) against central differences of the SEQ loss.  Row i's SEQ sum is within
    gamma_k sum_j |a_ij x_j| of the exact one (k = row length + 1), and column j's transposed SEQ
    sum within gamma_k sum_i |a_ij g_i|, so
    |FD - grad| <= (2 sum_i |g_i| gamma_k_i T_i + 2^-p |L+| + 2^-p |L-|) / |v+ - v-| + gamma C_j."""
    M = lib()
    p = 256
    A_h, x_h, g_h = synth.config3(p=p)
    A = M.CSRMatrix.from_host(A_h)
    S = M.autograd.SparseStructure.of(A)
    vt, xt = packed(M, A_h.vals), packed(M, x_h)
    y = M.autograd.spmv(S, vt, xt, 0)
    y.backward(M.autograd.pack(M.MPArray.from_host(g_h)))
    gx = to_np(M, xt.grad, p)
    g = M.MPArray.from_host(g_h)
    u = 2.0 ** -p
    rows = np.repeat(np.arange(A_h.n_rows), np.diff(A_h.row_ptr))
    av, xv, gv = approx_abs(A_h.vals), approx_abs(x_h), approx_abs(g_h)
    T = np.bincount(rows, weights=av * xv[A_h.col_idx], minlength=A_h.n_rows)
    C = np.bincount(A_h.col_idx, weights=av * gv[rows], minlength=A_h.n_cols)
    k = np.diff(A_h.row_ptr).astype(np.float64) + 1
    kc = np.bincount(A_h.col_idx, minlength=A_h.n_cols).astype(np.float64) + 1
    row_err = float(np.sum(gv * (k * u / (1 - k * u)) * T)) * (1 + 2.0 ** -20)
    xdev = M.MPArray.from_host(x_h)

    def seq_loss(xd):
        yy = M.mpspmv_csr(A, xd, mode=0)
        d = M.mp_dot(g, yy).to_numpy()
        return codec.decode(d[0], d[1], p)[0].to_fraction()
    rng = np.random.default_rng(9)
    for j in [int(v) for v in rng.integers(0, A_h.n_cols, 6)] + [int(np.argmax(kc))]:
        v = codec.decode(x_h.limbs[:, [j]], x_h.hdr[[j]], p)[0]
        h = mpnum.MP(0, 1 << (p - 1), v.e - 12, p) if v.m else mpnum.round_fraction(Fraction(1, 2 ** 40), p)
        out = []
        for nv in (mpnum.add(v, h), mpnum.sub(v, h)):
            l, hh = codec.encode([nv], p)
            xdev.limbs[:, j] = torch.from_numpy(l[:, 0].view(np.int32)).to(xdev.limbs.device)
            xdev.hdr[j] = int(hh[0])
            out.append((seq_loss(xdev), nv))
        l, hh = codec.encode([v], p)
        xdev.limbs[:, j] = torch.from_numpy(l[:, 0].view(np.int32)).to(xdev.limbs.device)
        xdev.hdr[j] = int(hh[0])
        (lp, vp), (lm, vm) = out
        dv = vp.to_fraction() - vm.to_fraction()
        got = (lp - lm) / dv
        want = codec.decode(gx[0][:, [j]], gx[1][[j]], p)[0].to_fraction()
        slack = (Fraction(2 * row_err) + Fraction(u) * (abs(lp) + abs(lm))) / abs(dv) + \
            Fraction(float(kc[j] * u / (1 - kc[j] * u) * C[j] * (1 + 2.0 ** -20)))
        assert abs(got - want) <= slack, (j, float(got), float(want), float(slack))
        assert abs(got - want) <= abs(want) * Fraction(1, 2 ** (p // 3))


def test_solve_adjoint_matches_oracle_and_duality():
    """x = A^{-1} b (2-D convection-diffusion, 6 x 6 grid, p = 512, b = A [1..n], relative
    tolerance 1e-100); d(sum x)/db = lambda from one transposed solve, bit-identical to the
    oracle's transposed BiCG, <lambda, b> = sum x to the tolerance, and the value gradient
    -RN(lambda_i x_j) bit-identical."""
    M = lib()
    p = 512
    A_h, _ = synth.config2(p=p, m=6)
    xstar_h = synth.mp_arange1(A_h.n_rows, p)
    ones_h = synth.mp_ones(A_h.n_rows, p)
    A = M.CSRMatrix.from_host(A_h)
    b = M.mpspmv_csr(A, M.MPArray.from_host(xstar_h), mode=1)
    S = M.autograd.SparseStructure.of(A)
    vt = packed(M, A_h.vals)
    bt = M.autograd.pack(b).requires_grad_(True)
    opts = dict(mode=1, maxit=500, rtol=(1, -100), atol=(0, 0), chunk=32)
    xt = M.autograd.solve(S, vt, bt, **opts)
    xt.backward(M.autograd.pack(M.MPArray.from_host(ones_h)))
    lam = to_np(M, bt.grad, p)
    xs = to_np(M, xt, p)
    rp, ci = A_h.row_ptr.tolist(), A_h.col_idx.tolist()
    vals = codec.decode(A_h.vals.limbs, A_h.vals.hdr, p)
    tp, ti, tv = ospmv.transpose(A_h.n_rows, A_h.n_cols, rp, ci, vals)
    c_rel = mpnum.round_fraction(Fraction(1, 10 ** 100), p)
    ones = codec.decode(ones_h.limbs, ones_h.hdr, p)
    ref = krylov.bicg(lambda v: ospmv.spmv_exact(tp, ti, tv, v, p), lambda v: ospmv.spmv_exact(rp, ci, vals, v, p),
                      ones, c_rel, mpnum.zero(p), 500, p)
    assert ref.status == krylov.CONVERGED
    assert_bitwise(lam[0], lam[1], ref.x, p, what="adjoint lambda")
    bo = codec.decode(*b.to_numpy(), p)
    lb = sum(l.to_fraction() * v.to_fraction() for l, v in zip(ref.x, bo))
    sx = sum(v.to_fraction() for v in codec.decode(xs[0], xs[1], p))
    assert abs(lb - sx) <= Fraction(1, 10 ** 90) * abs(sx)
    gv = to_np(M, vt.grad, p)
    xo = codec.decode(xs[0], xs[1], p)
    assert_bitwise(gv[0], gv[1], ospmv.grad_vals(rp, ci, ref.x, xo, p, negate=True), p, what="grad vals (solve)")


def test_repeated_rounds_and_no_grad_calls():
    """The same leaves go through two forward + backward rounds of the product and of the solve
    (each use ends with its backward pass), a call under torch.no_grad() claims nothing, and a
    dropped output frees its inputs for another use; the gradients of every round are equal."""
    import gc
    M = lib()
    p = 256
    A_h, x_h = synth.config1(p=p, n=120, per_row=5)
    g_h = synth.mp_uniform(np.random.default_rng(3), A_h.n_rows, p)
    A = M.CSRMatrix.from_host(A_h)
    S = M.autograd.SparseStructure.of(A)
    vt, xt = packed(M, A_h.vals), packed(M, x_h)
    gt = M.autograd.pack(M.MPArray.from_host(g_h))
    grads = []
    for _ in range(2):
        vt.grad = xt.grad = None
        M.autograd.spmv(S, vt, xt, 1).backward(gt)
        grads.append((vt.grad.clone(), xt.grad.clone()))
    assert bits_equal(grads[0][0], grads[1][0]) and bits_equal(grads[0][1], grads[1][1])
    with torch.no_grad():
        M.autograd.spmv(S, vt, xt, 0)
    y = M.autograd.spmv(S, vt, xt, 0)        # not blocked by the no_grad call
    del y
    gc.collect()
    M.autograd.spmv(S, vt, xt, 0).backward(gt)   # the dropped output released its inputs

    C_h, _ = synth.config2(p=p, m=6)
    C = M.CSRMatrix.from_host(C_h)
    SC = M.autograd.SparseStructure.of(C)
    ct = packed(M, C_h.vals)
    bt = packed(M, synth.mp_uniform(np.random.default_rng(4), C_h.n_rows, p))
    ones = M.autograd.pack(M.MPArray.from_host(synth.mp_ones(C_h.n_rows, p)))
    opts = dict(mode=1, maxit=300, rtol=(1, -60), atol=(0, 0))
    sg = []
    for _ in range(2):
        ct.grad = bt.grad = None
        M.autograd.solve(SC, ct, bt, **opts).backward(ones)
        sg.append((ct.grad.clone(), bt.grad.clone()))
    assert bits_equal(sg[0][0], sg[1][0]) and bits_equal(sg[0][1], sg[1][1])


def test_unconverged_solve_has_no_gradient():
    """A solve stopped by its iteration limit raises in the forward pass; with
    require_converged=False the iterate is returned and the backward pass raises instead of
    returning an adjoint of a non-solution."""
    M = lib()
    p = 256
    C_h, _ = synth.config2(p=p, m=8)
    C = M.CSRMatrix.from_host(C_h)
    SC = M.autograd.SparseStructure.of(C)
    ct = packed(M, C_h.vals)
    bt = packed(M, synth.mp_uniform(np.random.default_rng(5), C_h.n_rows, p))
    opts = dict(mode=0, maxit=2, rtol=(1, -60), atol=(0, 0))
    with pytest.raises(M.autograd.MPSolveError):
        M.autograd.solve(SC, ct, bt, **opts)
    x = M.autograd.solve(SC, ct, bt, require_converged=False, **opts)
    ones = M.autograd.pack(M.MPArray.from_host(synth.mp_ones(C_h.n_rows, p)))
    with pytest.raises(M.autograd.MPSolveError):
        x.backward(ones)
