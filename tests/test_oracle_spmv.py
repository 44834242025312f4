"""Pins of the oracle's sparse products, transpose, gradients and inner products.

EXACT mode is checked against the definition computed a second way (Fraction sum, then the
brute-force-pinned Fraction rounding); SEQ mode against the classical error bound of recursive
summation and against invariants that hold bitwise; the transpose against the adjoint identity.
"""
from fractions import Fraction
import random

import numpy as np
import pytest

import synth
from oracle import blas, codec, mpnum, spmv
from oracle.mpnum import MP


def small_problem(seed, n=37, m=29, per_row=(0, 9), p=128, espan=30, zeros=0.1):
    rng = random.Random(seed)
    row_ptr = [0]
    col_idx = []
    vals = []
    for i in range(n):
        k = rng.randint(*per_row)
        cols = sorted(rng.sample(range(m), min(k, m)))
        for c in cols:
            col_idx.append(c)
            if rng.random() < zeros:
                vals.append(mpnum.zero(p, rng.randint(0, 1)))
            else:
                vals.append(MP(rng.randint(0, 1), rng.getrandbits(p) | (1 << (p - 1)),
                               rng.randint(-espan, espan), p))
        row_ptr.append(len(col_idx))
    x = []
    for j in range(m):
        if rng.random() < zeros:
            x.append(mpnum.zero(p, rng.randint(0, 1)))
        else:
            x.append(MP(rng.randint(0, 1), rng.getrandbits(p) | (1 << (p - 1)),
                        rng.randint(-espan, espan), p))
    return n, m, row_ptr, col_idx, vals, x


@pytest.mark.parametrize("p", [128, 256, 512])
def test_exact_is_rn_of_fraction_sum(p):
    for seed in range(6):
        n, m, rp, ci, vals, x = small_problem(seed, p=p, espan=[3, 30, 300][seed % 3])
        y = spmv.spmv_exact(rp, ci, vals, x, p)
        for i in range(n):
            s = spmv.exact_row_sum_fraction(rp, ci, vals, x, i)
            assert y[i] == mpnum.round_fraction(s, p)


@pytest.mark.parametrize("p", [128, 256])
def test_seq_error_bound(p):
    """|y_seq - sum| <= gamma_k * sum |a x|, gamma_k = k u / (1 - k u), u = 2^-p, k = nnz_i + 1."""
    u = Fraction(1, 2 ** p)
    for seed in range(6):
        n, m, rp, ci, vals, x = small_problem(seed + 10, p=p, espan=20)
        y = spmv.spmv_seq(rp, ci, vals, x, p)
        for i in range(n):
            k = rp[i + 1] - rp[i] + 1
            s = spmv.exact_row_sum_fraction(rp, ci, vals, x, i)
            mag = sum(abs(vals[t].to_fraction() * x[ci[t]].to_fraction()) for t in range(rp[i], rp[i + 1]))
            gamma = k * u / (1 - k * u)
            assert abs(y[i].to_fraction() - s) <= gamma * mag


def test_seq_is_fold_of_primitives_and_differs_from_exact():
    p = 128
    n, m, rp, ci, vals, x = small_problem(3, p=p, espan=60, per_row=(5, 12))
    y = spmv.spmv_seq(rp, ci, vals, x, p)
    ye = spmv.spmv_exact(rp, ci, vals, x, p)
    for i in range(n):
        acc = mpnum.zero(p)
        for t in range(rp[i], rp[i + 1]):
            acc = mpnum.add(acc, mpnum.mul(vals[t], x[ci[t]]))
        assert acc == y[i]
    assert any(a != b for a, b in zip(y, ye)), "wide exponent spread must separate the modes"


@pytest.mark.parametrize("mode", [spmv.SEQ, spmv.EXACT])
def test_invariants(mode):
    p = 256
    n, m, rp, ci, vals, x = small_problem(5, n=30, m=30, p=p)
    y = spmv.spmv(rp, ci, vals, x, p, mode)
    # x = 0 gives +0 everywhere (also with -0 entries)
    xz = [mpnum.zero(p, j & 1) for j in range(m)]
    assert all(v.key() == (0, 0, None) for v in spmv.spmv(rp, ci, vals, xz, p, mode))
    # identity
    ident_rp = list(range(m + 1))
    ident_ci = list(range(m))
    ones = [mpnum.from_int(1, p)] * m
    xnz = [v if v.m else mpnum.zero(p) for v in x]
    assert spmv.spmv(ident_rp, ident_ci, ones, xnz, p, mode) == xnz
    # powers of two scale exactly: A (2^k x) = 2^k (A x) and (2^k A) x = 2^k (A x)
    for k in (-7, 5):
        x2 = [MP(v.s, v.m, v.e + k, p) if v.m else v for v in x]
        a2 = [MP(v.s, v.m, v.e + k, p) if v.m else v for v in vals]
        y2 = [MP(v.s, v.m, v.e + k, p) if v.m else v for v in y]
        assert spmv.spmv(rp, ci, vals, x2, p, mode) == y2
        assert spmv.spmv(rp, ci, a2, x, p, mode) == y2
    # removing stored zeros changes nothing
    rp2, ci2, v2 = [0], [], []
    for i in range(n):
        for t in range(rp[i], rp[i + 1]):
            if vals[t].m:
                ci2.append(ci[t])
                v2.append(vals[t])
        rp2.append(len(ci2))
    assert spmv.spmv(rp2, ci2, v2, x, p, mode) == y
    # a row permutation permutes y
    perm = list(range(n))
    random.Random(1).shuffle(perm)
    rp3, ci3, v3 = [0], [], []
    for i in perm:
        ci3 += ci[rp[i]:rp[i + 1]]
        v3 += vals[rp[i]:rp[i + 1]]
        rp3.append(len(ci3))
    assert spmv.spmv(rp3, ci3, v3, x, p, mode) == [y[i] for i in perm]
    # diagonal matrix: y_i = RN(d_i x_i) in both modes
    d = [v for v in x]
    yd = spmv.spmv(ident_rp, ident_ci, d, x, p, mode)
    assert yd == [mpnum.mul(a, b) if (a.m and b.m) else mpnum.zero(p) for a, b in zip(d, x)]


def test_integer_inputs_seq_equals_exact():
    p = 128
    rng = random.Random(9)
    n = 20
    rp, ci, vals = [0], [], []
    for i in range(n):
        cols = sorted(rng.sample(range(n), 6))
        for c in cols:
            ci.append(c)
            vals.append(mpnum.from_int(rng.randint(-1000, 1000) or 1, p))
        rp.append(len(ci))
    x = [mpnum.from_int(rng.randint(-1000, 1000), p) for _ in range(n)]
    assert spmv.spmv_seq(rp, ci, vals, x, p) == spmv.spmv_exact(rp, ci, vals, x, p)


def test_exact_invariant_under_row_reordering():
    p = 128
    n, m, rp, ci, vals, x = small_problem(11, p=p, espan=80, per_row=(3, 9))
    y = spmv.spmv_exact(rp, ci, vals, x, p)
    # evaluate each row's exact sum in reversed storage order via the same definition
    for i in range(n):
        pairs = [(vals[t], x[ci[t]]) for t in range(rp[i + 1] - 1, rp[i] - 1, -1)]
        assert spmv.exact_sum_of_products(pairs, p) == y[i]


def test_transpose_involution_and_symmetric():
    p = 128
    n, m, rp, ci, vals, x = small_problem(12, n=25, m=31, p=p)
    tp, ti, tv = spmv.transpose(n, m, rp, ci, vals)
    rp2, ci2, v2 = spmv.transpose(m, n, tp, ti, tv)
    assert list(rp2) == list(rp) and list(ci2) == list(ci) and v2 == vals
    # brute-force transpose through a dense dict
    dense = {}
    for i in range(n):
        for t in range(rp[i], rp[i + 1]):
            dense[(i, ci[t])] = vals[t]
    for j in range(m):
        ent = [(ti[t], tv[t]) for t in range(tp[j], tp[j + 1])]
        assert ent == sorted(((i, v) for (i, jj), v in dense.items() if jj == j), key=lambda z: z[0])
    # symmetric matrix: A^T x == A x in both modes
    sym = {}
    rng = random.Random(4)
    for i in range(15):
        for j in range(i, 15):
            if rng.random() < 0.3 or i == j:
                v = MP(rng.randint(0, 1), rng.getrandbits(p) | (1 << (p - 1)), rng.randint(-5, 5), p)
                sym[(i, j)] = v
                sym[(j, i)] = v
    srp, sci, sv = [0], [], []
    for i in range(15):
        for j in range(15):
            if (i, j) in sym:
                sci.append(j)
                sv.append(sym[(i, j)])
        srp.append(len(sci))
    xs = x[:15]
    for mode in (spmv.SEQ, spmv.EXACT):
        assert spmv.spmv_t(15, 15, srp, sci, sv, xs, p, mode) == spmv.spmv(srp, sci, sv, xs, p, mode)


def test_adjoint_identity_exact_mode():
    """<g, A x> and <A^T g, x> agree to the rounding of each product component:
    |<g, RN(Ax)> - <RN(A^T g), x>| <= u (sum_i |g_i| |(Ax)_i| + sum_j |(A^T g)_j| |x_j|)."""
    p = 128
    u = Fraction(1, 2 ** p)
    n, m, rp, ci, vals, x = small_problem(13, n=40, m=33, p=p)
    _, _, _, _, _, g = small_problem(14, n=1, m=40, p=p)
    y = spmv.spmv_exact(rp, ci, vals, x, p)
    yt = spmv.spmv_t(n, m, rp, ci, vals, g, p, spmv.EXACT)
    lhs = sum(g[i].to_fraction() * y[i].to_fraction() for i in range(n))
    rhs = sum(yt[j].to_fraction() * x[j].to_fraction() for j in range(m))
    bound = u * (sum(abs(g[i].to_fraction() * y[i].to_fraction()) for i in range(n))
                 + sum(abs(yt[j].to_fraction() * x[j].to_fraction()) for j in range(m)))
    assert abs(lhs - rhs) <= bound


def test_grad_vals_and_dot_definitions():
    p = 256
    n, m, rp, ci, vals, x = small_problem(15, n=20, m=20, p=p)
    _, _, _, _, _, g = small_problem(16, n=1, m=20, p=p)
    gv = spmv.grad_vals(rp, ci, g, x, p)
    t = 0
    for i in range(n):
        for k in range(rp[i], rp[i + 1]):
            want = mpnum.round_fraction(g[i].to_fraction() * x[ci[k]].to_fraction(), p)
            if g[i].m == 0 or x[ci[k]].m == 0:
                # a zero factor: a zero whose sign is the xor of the factors' signs (IEEE RN)
                want = mpnum.zero(p, g[i].s ^ x[ci[k]].s)
            assert gv[t] == want, (t, gv[t], want)
            t += 1
    neg = spmv.grad_vals(rp, ci, g, x, p, negate=True)
    assert all(a == b.neg() for a, b in zip(neg, gv))
    d = blas.dot(g, x, p)
    assert d == mpnum.round_fraction(sum(a.to_fraction() * b.to_fraction() for a, b in zip(g, x)), p)


def test_codec_roundtrip_and_layout():
    p = 128
    rng = np.random.default_rng(0)
    h = synth.mp_uniform(rng, 50, p)
    vals = codec.decode(h.limbs, h.hdr, p)
    limbs, hdr = codec.encode(vals, p)
    assert np.array_equal(limbs, h.limbs) and np.array_equal(hdr, h.hdr)
    # the layout: limb k is bits [32k, 32k+32) of the mantissa, hdr = (e << 1) | s
    v = vals[3]
    assert int(h.limbs[p // 32 - 1, 3]) == v.m >> (p - 32)
    assert int(h.hdr[3]) == (v.e << 1) | v.s
    z = codec.decode(synth.mp_zeros(2, p).limbs, synth.mp_zeros(2, p).hdr, p)
    assert all(t.m == 0 and t.s == 0 for t in z)


def test_generators_values_match_their_recipe():
    """The chopped stencil coefficients are within one ulp below the exact rationals, and the
    structure has the documented shape."""
    p = 256
    A = synth.convdiff2d(8, p)
    vals = codec.decode(A.vals.limbs, A.vals.hdr, p)
    den = 2 * 9
    want = {Fraction(4), Fraction(-(den + 10), den), Fraction(-(den - 10), den)}
    got = set()
    for v in vals:
        f = v.to_fraction()
        match = [w for w in want if abs(f - w) < Fraction(2) ** (v.e - p) and abs(f) <= abs(w)]
        assert len(match) == 1
        got.add(match[0])
    assert got == want
    assert A.nnz == 5 * 64 - 4 * 8
    rp = A.row_ptr
    for i in range(A.n_rows):
        row = A.col_idx[rp[i]:rp[i + 1]]
        assert np.all(np.diff(row) > 0)


def _one_eps(p):
    """1 and eps = 2^-p: 1 + eps is the exact midpoint between 1 and its successor 1 + 2^(1-p)."""
    one = MP(0, 1 << (p - 1), 1, p)
    eps = MP(0, 1 << (p - 1), 1 - p, p)
    return one, eps


@pytest.mark.parametrize("p", [128, 256, 512])
def test_seq_order_is_storage_order_closed_form(p):
    """SEQ adds a row's products in ascending column order, one rounding per operation.

    Row [1, e, e, ..., e] (k copies of e = 2^-p, x = 1): in storage order every partial sum is the
    tie 1 + e, which rounds to the even neighbour 1, so y = 1 whatever k.  Any order that adds
    two of the small terms before the 1 (reversed, pairwise, sorted by magnitude) forms 2e
    exactly and returns 1 + 2^(1-p) or more.  Row [e, e, 1]: the small terms come first in
    storage order, so y = 1 + 2^(1-p), while the reversed order gives 1.  EXACT rounds the exact
    sum 1 + k e once."""
    one, eps = _one_eps(p)
    succ = MP(0, (1 << (p - 1)) + 1, 1, p)            # 1 + 2^(1-p)
    rows = [[one] + [eps] * k for k in (1, 2, 3, 7)] + [[eps, eps, one], [eps, one, eps]]
    rp, ci, vals = [0], [], []
    for r in rows:
        ci += list(range(len(r)))
        vals += r
        rp.append(len(ci))
    x = [one] * 8
    y = spmv.spmv_seq(rp, ci, vals, x, p)
    assert y[:4] == [one] * 4
    assert y[4] == succ            # e + e = 2e exactly, then 1 + 2e is representable
    assert y[5] == one             # (e + 1) ties to 1, then (1 + e) ties to 1
    # the same rows in reversed storage order give the other results
    rrp, rci, rvals = [0], [], []
    for r in rows:
        rci += list(range(len(r)))
        rvals += r[::-1]
        rrp.append(len(rci))
    yr = spmv.spmv_seq(rrp, rci, rvals, x, p)
    assert yr[1] == succ and yr[4] == one and yr[5] == one
    assert yr[3] == MP(0, (1 << (p - 1)) + 4, 1, p)   # 7e first: 1 + 7e -> tie at 1 + 3.5 ulp -> 1 + 4 ulp
    # EXACT: one rounding of 1 + k e
    ye = spmv.spmv_exact(rp, ci, vals, x, p)
    assert ye[0] == one                                # 1 + e: tie to even
    assert ye[1] == succ                               # 1 + 2e exactly
    assert ye[3] == MP(0, (1 << (p - 1)) + 4, 1, p)    # 1 + 7e: 3.5 ulp ties to 4 ulp (even)


@pytest.mark.parametrize("p", [128, 512])
def test_seq_transposed_order_is_ascending_original_row(p):
    """A^T x in SEQ mode sums each column of A over its original rows in ascending order.
    Column 0 holds (1, e, e) in rows 0, 1, 2 and column 1 holds (e, e, 1): with x = 1 the
    transposed product gives 1 and 1 + 2^(1-p) (descending original rows would swap them)."""
    one, eps = _one_eps(p)
    succ = MP(0, (1 << (p - 1)) + 1, 1, p)
    rp = [0, 2, 4, 6]
    ci = [0, 1, 0, 1, 0, 1]
    vals = [one, eps, eps, eps, eps, one]
    x = [one] * 3
    yt = spmv.spmv_t(3, 2, rp, ci, vals, x, p, spmv.SEQ)
    assert yt == [one, succ]
    tp, ti, tv = spmv.transpose(3, 2, rp, ci, vals)
    assert tp == [0, 3, 6] and ti == [0, 1, 2, 0, 1, 2]
    assert tv == [one, eps, eps, eps, eps, one]
