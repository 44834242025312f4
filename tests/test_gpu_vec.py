"""GPU parity of the transposed product, the value gradient, y + alpha x, the exact inner product
and the decimal constants, bit for bit against the oracle."""
from fractions import Fraction

import numpy as np
import pytest

import synth
from oracle import blas, codec, mpnum, spmv as ospmv
from tests.util import assert_bitwise, decode_vec

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def lib():
    import paper_1411_2377_amd as M
    return M


def host(arr):
    limbs, hdr = arr.to_numpy()
    return synth.MPHost(limbs, hdr, arr.p)


@pytest.mark.parametrize("p", [128, 256, 512, 1024])
@pytest.mark.parametrize("mode", [0, 1], ids=["seq", "exact"])
def test_transpose_product_random(p, mode):
    M = lib()
    rng = np.random.default_rng(p + mode)
    n, m = 700, 523
    lengths = rng.integers(0, 25, size=n)
    lengths[5] = 300                               # a row longer than one 128-entry chunk
    rp = np.zeros(n + 1, np.int64)
    np.cumsum(lengths, out=rp[1:])
    cols = synth._distinct_sorted_columns(rng, lengths, m)
    vals = synth.mp_uniform(rng, len(cols), p)
    A_h = synth.CSRHost(n, m, rp.astype(np.int32), cols.astype(np.int32), vals)
    x_h = synth.mp_uniform(rng, n, p)
    A = M.CSRMatrix.from_host(A_h)
    P = M.mp_plan_create(A)
    y = M.mpspmv_csr_t(A, P, M.MPArray.from_host(x_h), mode=mode)
    assert M.mp_status() == 0
    yl, yh = y.to_numpy()
    vals_o = codec.decode(A_h.vals.limbs, A_h.vals.hdr, p)
    x_o = codec.decode(x_h.limbs, x_h.hdr, p)
    want = ospmv.spmv_t(n, m, A_h.row_ptr.tolist(), A_h.col_idx.tolist(), vals_o, x_o, p, mode)
    assert_bitwise(yl, yh, want, p, what="A^T x")


@pytest.mark.parametrize("p", [128, 256, 512])
@pytest.mark.parametrize("mode", [0, 1], ids=["seq", "exact"])
def test_transpose_powerlaw_full_size_sampled(p, mode):
    """The power-law workload (n = 500000): A^T g on sampled columns (incl. the heaviest), with
    the plan's default variant and with its tuned variant (the benchmark's configuration)."""
    M = lib()
    A_h, x_h, g_h = synth.config3(p=p)
    A = M.CSRMatrix.from_host(A_h)
    P = M.mp_plan_create(A)
    g = M.MPArray.from_host(g_h)
    y = M.mpspmv_csr_t(A, P, g, mode=mode)
    P.tune(reps=1)
    y2 = M.mpspmv_csr_t(A, P, g, mode=mode)
    assert M.mp_status() == 0
    yl, yh = y.to_numpy()
    yl2, yh2 = y2.to_numpy()
    assert np.array_equal(yl, yl2) and np.array_equal(yh, yh2), "tuned variant differs"
    counts = np.bincount(A_h.col_idx, minlength=A_h.n_cols)
    rng = np.random.default_rng(1)
    cols = np.unique(np.concatenate([[0, A_h.n_cols - 1], np.argsort(counts)[-3:],
                                     rng.integers(0, A_h.n_cols, 40)]))
    # oracle: column j of A = entries with col_idx == j in ascending row order
    row_of = np.repeat(np.arange(A_h.n_rows), np.diff(A_h.row_ptr))
    want = []
    for j in cols:
        ks = np.nonzero(A_h.col_idx == j)[0]
        vals = codec.decode(A_h.vals.limbs[:, ks], A_h.vals.hdr[ks], p)
        gs = decode_vec(g_h, row_of[ks])
        pairs = [(v, gs[int(i)]) for v, i in zip(vals, row_of[ks])]
        if mode == 1:
            want.append(ospmv.exact_sum_of_products(pairs, p))
        else:
            acc = mpnum.zero(p)
            for a, b in pairs:
                acc = mpnum.add(acc, mpnum.mul(a, b))
            want.append(acc)
    assert_bitwise(yl, yh, want, p, rows=cols, what="A^T g power-law p=%d" % p)


@pytest.mark.parametrize("p", [128, 512])
def test_grad_vals_and_symmetric_transpose(p):
    M = lib()
    A_h, ones = synth.config2(p=p, m=24)
    rng = np.random.default_rng(3)
    g_h = synth.mp_uniform(rng, A_h.n_rows, p)
    x_h = synth.mp_uniform(rng, A_h.n_cols, p)
    A = M.CSRMatrix.from_host(A_h)
    P = M.mp_plan_create(A)
    gv = M.mp_grad_vals(A, P, M.MPArray.from_host(g_h), M.MPArray.from_host(x_h))
    gvn = M.mp_grad_vals(A, P, M.MPArray.from_host(g_h), M.MPArray.from_host(x_h), negate=True)
    gl, gh = gv.to_numpy()
    want = ospmv.grad_vals(A_h.row_ptr.tolist(), A_h.col_idx.tolist(), codec.decode(g_h.limbs, g_h.hdr, p),
                           codec.decode(x_h.limbs, x_h.hdr, p), p)
    assert_bitwise(gl, gh, want, p, what="grad vals")
    nl, nh = gvn.to_numpy()
    assert_bitwise(nl, nh, [w.neg() for w in want], p, what="negated grad vals")
    # a symmetric matrix (pattern and values) has A^T x == A x bitwise in both modes
    n = 50
    rows, cols_, vals = [], [], []
    rr = np.random.default_rng(5)
    dense = {}
    for i in range(n):
        for j in range(i, n):
            if i == j or rr.random() < 0.1:
                dense[(i, j)] = dense[(j, i)] = len(vals)
                vals.append(None)
    keys = sorted(dense)
    uniq = synth.mp_uniform(rr, len(vals), p)
    idx = np.array([dense[k] for k in keys])
    S_h = synth.CSRHost(n, n, np.concatenate([[0], np.cumsum(np.bincount([k[0] for k in keys], minlength=n))]).astype(np.int32),
                        np.array([k[1] for k in keys], np.int32), uniq.take(idx))
    S = M.CSRMatrix.from_host(S_h)
    SP = M.mp_plan_create(S)
    xs = M.MPArray.from_host(synth.mp_uniform(rr, n, p))
    for mode in (0, 1):
        a = M.mpspmv_csr(S, xs, mode=mode).to_numpy()
        b = M.mpspmv_csr_t(S, SP, xs, mode=mode).to_numpy()
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


@pytest.mark.parametrize("p", [128, 256, 512, 1024])
def test_axpy_dot_const(p):
    M = lib()
    rng = np.random.default_rng(p)
    n = 5000 + 37
    x_h = synth.mp_uniform(rng, n, p)
    y_h = synth.mp_loguniform(rng, n, p, -30, 30)
    y_h.hdr[::17] = np.int32(-(1 << 31)) + (np.arange(len(y_h.hdr[::17])) % 2).astype(np.int32)   # +-0
    a_h = synth.mp_uniform(rng, 1, p)
    x, y, a = M.MPArray.from_host(x_h), M.MPArray.from_host(y_h), M.MPArray.from_host(a_h)
    d = M.mp_dot(x, y).to_numpy()
    xo, yo = codec.decode(x_h.limbs, x_h.hdr, p), codec.decode(y_h.limbs, y_h.hdr, p)
    assert_bitwise(d[0], d[1], [blas.dot(xo, yo, p)], p, what="dot")
    # an exactly cancelling inner product: x . [y, -y] on [x, x]
    xx = synth.mp_concat([x_h, x_h])
    yy = synth.mp_concat([y_h, synth.MPHost(y_h.limbs.copy(), y_h.hdr ^ np.int32(1), p)])
    d0 = M.mp_dot(M.MPArray.from_host(xx), M.MPArray.from_host(yy)).to_numpy()
    assert d0[1][0] == np.int32(-(1 << 31))
    M.mp_axpy(a, x, y)
    yl, yh = y.to_numpy()
    assert_bitwise(yl, yh, blas.axpy(codec.decode(a_h.limbs, a_h.hdr, p)[0], xo, yo), p, what="axpy")
    for m_, e_ in ((1, -20), (1, -50), (1, -100), (-3, 7), (123456789, -3), (0, 5)):
        c = M.mp_const_decimal(m_, e_, p).to_numpy()
        want = mpnum.round_fraction(Fraction(m_) * Fraction(10) ** e_, p)
        assert_bitwise(c[0], c[1], [want], p, what="const %d e%d" % (m_, e_))


def test_dot_wide_span_and_long():
    """Products spanning ~2000 bits (the block-shared window) and a long vector (many blocks)."""
    M = lib()
    p = 256
    rng = np.random.default_rng(9)
    n = 300000
    x_h = synth.mp_uniform(rng, n, p)
    y_h = synth.mp_loguniform(rng, n, p, -300, 300)
    d = M.mp_dot(M.MPArray.from_host(x_h), M.MPArray.from_host(y_h)).to_numpy()
    xo, yo = codec.decode(x_h.limbs, x_h.hdr, p), codec.decode(y_h.limbs, y_h.hdr, p)
    assert_bitwise(d[0], d[1], [blas.dot(xo, yo, p)], p, what="wide dot")
    assert M.mp_status() == 0


@pytest.mark.parametrize("p", [128, 256, 512, 1024])
def test_dot_rounding_edge_cases(p):
    """Inner products whose exact sums sit on the rounding boundaries: ties to even, the
    all-ones mantissa that rounds up to the next power of two, exact cancellation, negative
    sums, borrows through many digits and windows of about 60 digits and of more."""
    from fractions import Fraction as F
    M = lib()
    h = F(1, 2 ** p)            # half an ulp of 1 is 2^-p
    cases = [
        ([F(1), h], [F(1), F(1)]),                          # tie, even: 1
        ([F(1), 3 * h / 2], [F(1), F(1)]),                  # above the tie: up
        ([1 - h, h / 2], [F(1), F(1)]),                      # all ones + half ulp: 1
        ([F(1, 3), F(1, 3)], [F(1), F(-1)]),                 # exact cancellation: +0
        ([F(1), h], [F(-1), F(-1)]),                         # negative tie: -1
        ([F(2) ** 100, F(-1), F(1, 2 ** 100)], [F(1), F(1), F(1)]),
        ([F(-(2 ** 60)), F(1, 2 ** 200), F(2 ** 60)], [F(1), F(1), F(1)]),
        ([F(2) ** 500, F(1, 2 ** 500)], [F(2) ** 200, F(-1, 2 ** 600)]),
        ([F(2) ** 450, F(-3, 2 ** 450)], [F(1), F(1)]),      # a window of about 60 digits
        ([F(2) ** 900, F(-3, 2 ** 900)], [F(2) ** 900, F(1, 2 ** 900)]),
        ([F(2) ** 1000, F(1, 2 ** 1000), F(-1)], [F(2) ** 1000, F(-1, 2 ** 1000), F(1)]),
    ]
    rng = np.random.default_rng(p + 1)
    for _ in range(12):   # random cancelling sums: sum of values and their near-negatives
        k = int(rng.integers(2, 9))
        xs = [F(int(rng.integers(-2 ** 40, 2 ** 40)), 2 ** int(rng.integers(0, 300))) for _ in range(k)]
        ys = [F(1)] * k
        xs = xs + [-v for v in xs[:-1]] + [F(1, 2 ** int(rng.integers(100, 700)))]
        ys = ys + ys[:-1] + [F(1)]
        cases.append((xs, ys))
    for i, (xs, ys) in enumerate(cases):
        x_h = synth.mp_from_rationals([(v.numerator, v.denominator) for v in xs], p)
        y_h = synth.mp_from_rationals([(v.numerator, v.denominator) for v in ys], p)
        d = M.mp_dot(M.MPArray.from_host(x_h), M.MPArray.from_host(y_h)).to_numpy()
        xo, yo = codec.decode(x_h.limbs, x_h.hdr, p), codec.decode(y_h.limbs, y_h.hdr, p)
        assert_bitwise(d[0], d[1], [blas.dot(xo, yo, p)], p, what="dot case %d" % i)


@pytest.mark.parametrize("p", [128, 256])
def test_dot_window_limit(p):
    """Two products 2^(2E) and 2^(-2E), an exponent span of 4E bits: a span inside the window
    limit of a stand-alone inner product (32 (1157 - 2L - 2) bits at p = 128, 32 (2048 - 2L - 2)
    above) rounds exactly, to the larger term; a wider span raises the window status and gives
    +0, and the next inner product is exact again (the ring was cleared)."""
    M = lib()
    nl = p // 32

    def powers(es):
        limbs = np.zeros((nl, len(es)), np.uint32)
        limbs[nl - 1] = np.uint32(0x80000000)
        return synth.MPHost(limbs, synth._hdr(np.array(es) + 1, np.zeros(len(es))), p)

    for E, fits in ((8000, True), (40000, False), (100, True)):
        xh = powers([E, -E])
        d = M.mp_dot(M.MPArray.from_host(xh), M.MPArray.from_host(xh)).to_numpy()
        flags = M.mp_status(raise_on_error=False)
        if fits:
            xo = codec.decode(xh.limbs, xh.hdr, p)
            assert flags == 0
            assert_bitwise(d[0], d[1], [blas.dot(xo, xo, p)], p, what="dot span %d" % E)
        else:
            assert flags & 2, flags          # MP_ST_WINDOW
            assert d[1][0] == np.int32(-(1 << 31))  # +0
