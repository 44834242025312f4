"""Pins of the oracle's dense product (the paper's dense MV with zeros stored, Sec. 3) and of
the Lotkin workload generator, against what the mathematics fixes:

* EXACT equals RN of the Fraction row sum;
* the stored zeros change nothing: the dense product equals the sparse product of the same
  matrix without its zeros, bitwise, in both modes (adding a zero product to a sum that is never
  -0 returns it unchanged);
* a row of integers times [1..n] sums exactly: the Lotkin matrix's first row gives n(n+1)/2;
* SEQ stays within the recursive-summation bound of the exact sum;
* the generator's elements are the p-bit truncations of 1/(i+j-1), with the requested number of
  zeros.
"""
from fractions import Fraction

import numpy as np
import pytest

import synth
from oracle import codec, dense, mpnum, spmv


def decode(h):
    return codec.decode(h.limbs, h.hdr, h.p)


@pytest.mark.parametrize("p", [128, 256])
def test_lotkin_generator(p):
    n = 12
    D, C, x = synth.lotkin(n, p, 40.0, seed=3)
    vals = decode(D)
    assert sum(v.is_zero() for v in vals) == round(0.4 * n * n)
    for idx, v in enumerate(vals):
        if v.is_zero():
            continue
        i, j = divmod(idx, n)
        want = Fraction(1) if i == 0 else Fraction(1, i + j + 1)
        f = v.to_fraction()
        ulp = Fraction(2) ** (v.e - p)
        assert f <= want < f + ulp, (i, j)
    # the CSR holds exactly the non-zero elements, row by row in ascending column order
    cv = decode(C.vals)
    k = 0
    for i in range(n):
        cols = [j for j in range(n) if not vals[i * n + j].is_zero()]
        assert C.col_idx[C.row_ptr[i]:C.row_ptr[i + 1]].tolist() == cols
        for j in cols:
            assert cv[k] == vals[i * n + j]
            k += 1
    assert [v.to_fraction() for v in decode(x)] == list(range(1, n + 1))


@pytest.mark.parametrize("mode", [spmv.SEQ, spmv.EXACT])
@pytest.mark.parametrize("zero_pct", [0.0, 50.0, 90.0])
def test_dense_equals_sparse_without_zeros(mode, zero_pct):
    p = 128
    n = 20
    D, C, x = synth.lotkin(n, p, zero_pct, seed=int(zero_pct) + mode)
    xv = decode(x)
    got = dense.gemv(n, n, decode(D), xv, p, mode)
    want = spmv.spmv(C.row_ptr.tolist(), C.col_idx.tolist(), decode(C.vals), xv, p, mode)
    assert got == want


def test_dense_exact_is_rounded_fraction_sum():
    p = 256
    n = 15
    rng = np.random.default_rng(4)
    a = synth.mp_uniform(rng, n * n, p)
    a.hdr[rng.permutation(n * n)[:60]] = synth.ZERO_HDR
    xs = synth.mp_uniform(rng, n, p)
    vals, xv = decode(a), decode(xs)
    y = dense.gemv(n, n, vals, xv, p, spmv.EXACT)
    for i in range(n):
        s = sum(vals[i * n + j].to_fraction() * xv[j].to_fraction() for j in range(n))
        assert y[i] == mpnum.round_fraction(s, p)


@pytest.mark.parametrize("mode", [spmv.SEQ, spmv.EXACT])
def test_integer_row_sums_exactly(mode):
    p = 128
    n = 40
    D, C, x = synth.lotkin(n, p, 0.0)
    y = dense.gemv(n, n, decode(D), decode(x), p, mode)
    assert y[0].to_fraction() == n * (n + 1) // 2


def test_seq_within_summation_bound():
    p = 128
    n = 30
    D, C, x = synth.lotkin(n, p, 30.0, seed=9)
    vals, xv = decode(D), decode(x)
    y = dense.gemv(n, n, vals, xv, p, spmv.SEQ)
    u = Fraction(1, 2 ** p)
    for i in range(n):
        terms = [vals[i * n + j].to_fraction() * xv[j].to_fraction() for j in range(n)]
        k = n + 1
        gamma = k * u / (1 - k * u)
        assert abs(y[i].to_fraction() - sum(terms)) <= gamma * sum(abs(t) for t in terms)
