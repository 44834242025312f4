"""Pins of the oracle's rounding and arithmetic primitives against things other than itself.

* brute force: at p = 2..5 every mantissa pair over a range of exponent offsets, the result is
  compared with an exhaustive search for the nearest p-bit number (ties to the even mantissa);
* mpmath at working precision p (its own correctly rounded nearest-even arithmetic);
* closed forms: ties, an all-ones mantissa carrying into a new exponent, total cancellation;
* characterisations: RN(a/b) and RN(sqrt a) are nearer than both neighbours.
"""
from fractions import Fraction
import itertools
import math
import random

import mpmath
import pytest

from oracle import mpnum
from oracle.mpnum import MP, add, div, mul, sqrt, sub


def mk(s, m, e, p):
    return MP(s, m, e, p)


def nearest_brute(v, p):
    """Nearest p-bit float to the exact non-zero rational v by exhaustive search."""
    sign = 1 if v < 0 else 0
    a = abs(v)
    e0 = math.frexp(float(a))[1]       # float estimate of the exponent, checked +-2
    best = None
    for e in range(e0 - 2, e0 + 3):
        for m in range(1 << (p - 1), 1 << p):
            c = Fraction(m) * Fraction(2) ** (e - p)
            d = abs(a - c)
            key = (d, m & 1)            # smaller distance first, then even mantissa
            if best is None or key < best[0]:
                best = (key, m, e)
    _, m, e = best
    return (sign, m, e)


def as_tuple(x):
    return (x.s, x.m, x.e)


@pytest.mark.parametrize("p", [2, 3, 4, 5])
def test_mul_add_sub_bruteforce(p):
    mants = range(1 << (p - 1), 1 << p)
    for ma, mb in itertools.product(mants, mants):
        for de in range(-(p + 3), p + 4):
            a = mk(0, ma, 0, p)
            for sb in (0, 1):
                b = mk(sb, mb, de, p)
                exact = a.to_fraction() * b.to_fraction()
                assert as_tuple(mul(a, b)) == nearest_brute(exact, p)
                exact = a.to_fraction() + b.to_fraction()
                r = add(a, b)
                if exact == 0:
                    assert r.m == 0 and r.s == 0
                else:
                    assert as_tuple(r) == nearest_brute(exact, p), (p, ma, mb, de, sb)
                exact = a.to_fraction() - b.to_fraction()
                r = sub(a, b)
                if exact == 0:
                    assert r.m == 0 and r.s == 0
                else:
                    assert as_tuple(r) == nearest_brute(exact, p)


@pytest.mark.parametrize("p", [2, 3, 4, 5])
def test_div_sqrt_bruteforce(p):
    mants = range(1 << (p - 1), 1 << p)
    for ma, mb in itertools.product(mants, mants):
        for de in (-3, 0, 1, 4):
            a = mk(1, ma, de, p)
            b = mk(0, mb, 0, p)
            assert as_tuple(div(a, b)) == nearest_brute(a.to_fraction() / b.to_fraction(), p)
    for ma in mants:
        for e in range(-5, 6):
            a = mk(0, ma, e, p)
            r = sqrt(a)
            # nearest p-bit number to sqrt(a), by brute force over candidates and exact squares
            v = a.to_fraction()
            cands = []
            e0 = math.frexp(math.sqrt(float(v)))[1]
            for ee in range(e0 - 2, e0 + 3):
                for m in mants:
                    cands.append((m, ee))
            # compare |sqrt(v) - c| via (c^2 vs v): the nearest c minimises |sqrt v - c|; use
            # exact midpoints: c is nearest iff mid_lo^2 <= v <= mid_hi^2 (strict on ties)
            sel = []
            allc = sorted(set(Fraction(m) * Fraction(2) ** (ee - p) for m, ee in cands))
            for i, c in enumerate(allc[1:-1], start=1):
                lo = (allc[i - 1] + c) / 2
                hi = (c + allc[i + 1]) / 2
                if lo * lo < v < hi * hi:
                    sel.append(c)
            assert len(sel) == 1
            assert r.to_fraction() == sel[0]


def test_round_scaled_matches_round_fraction():
    rng = random.Random(7)
    for p in (2, 3, 7, 64, 128, 256):
        for _ in range(300):
            n = rng.getrandbits(rng.randint(1, 3 * p)) | 1
            k = rng.randint(-300, 300)
            s = rng.randint(0, 1)
            v = Fraction(n) * Fraction(2) ** k * (-1 if s else 1)
            assert mpnum.round_scaled(s, n, k, p) == mpnum.round_fraction(v, p)


def to_mpf(x):
    if x.m == 0:
        return mpmath.mpf(0)
    v = mpmath.ldexp(mpmath.mpf(x.m), x.e - x.p)
    return -v if x.s else v


def from_mpf(v, p):
    """Exact rational value of an mpmath number (mantissa * 2^exponent)."""
    if v == 0:
        return Fraction(0)
    sign, man, exp, _ = mpmath.mpf(v)._mpf_
    f = Fraction(int(man)) * Fraction(2) ** int(exp)
    return -f if sign else f


def rand_mp(rng, p, espan=40):
    m = rng.getrandbits(p) | (1 << (p - 1))
    return MP(rng.randint(0, 1), m, rng.randint(-espan, espan), p)


@pytest.mark.parametrize("p", [128, 256, 512])
def test_against_mpmath(p):
    rng = random.Random(p)
    with mpmath.workprec(p):
        for _ in range(400):
            a = rand_mp(rng, p)
            b = rand_mp(rng, p, espan=rng.choice([2, 40, p + 40]))
            fa, fb = to_mpf(a), to_mpf(b)
            assert mul(a, b).to_fraction() == from_mpf(fa * fb, p)
            assert add(a, b).to_fraction() == from_mpf(fa + fb, p)
            assert sub(a, b).to_fraction() == from_mpf(fa - fb, p)
            assert div(a, b).to_fraction() == from_mpf(fa / fb, p)
            aa = MP(0, a.m, a.e, p)
            assert sqrt(aa).to_fraction() == from_mpf(mpmath.sqrt(to_mpf(aa)), p)


@pytest.mark.parametrize("p", [128, 256, 512])
def test_closed_form_ties_carries_cancellation(p):
    one = mpnum.from_int(1, p)
    half_ulp = mpnum.round_fraction(Fraction(1, 2 ** p), p)       # 2^-p, exact
    # 1 + 2^-p is a tie between 1 and 1 + 2^(1-p); the even mantissa is 1's
    assert add(one, half_ulp) == one
    # (1 + 2^(1-p)) + 2^-p is a tie; the even neighbour is 1 + 2^(2-p)
    onep = mpnum.round_fraction(1 + Fraction(2, 2 ** p), p)
    assert add(onep, half_ulp).to_fraction() == 1 + Fraction(4, 2 ** p)
    # (1 - 2^-p) has an all-ones mantissa; adding 2^-(p+1) is a tie, rounded up to 1 (a carry
    # into a new exponent)
    allones = mpnum.round_fraction(1 - Fraction(1, 2 ** p), p)
    assert allones.m == (1 << p) - 1 and allones.e == 0
    r = add(allones, mpnum.round_fraction(Fraction(1, 2 ** (p + 1)), p))
    assert r == one and r.e == 1
    # total cancellation: 1 - (1 - 2^-p) = 2^-p exactly (a shift by p bits)
    r = sub(one, allones)
    assert r.to_fraction() == Fraction(1, 2 ** p)
    # exact zero sum is +0
    r = add(allones, allones.neg())
    assert r.m == 0 and r.s == 0
    # multiply tie: M = 2 (mod 4), M >= 2^(p+1)/3, times 3: the (p+2)-bit product ends in 10
    rng = random.Random(p)
    for _ in range(50):
        m = rng.randrange((1 << (p + 1)) // 3 + 4, 1 << p)
        m = (m & ~3) | 2
        a = MP(0, m, 0, p)
        three = mpnum.from_int(3, p)
        q = (3 * m) >> 2
        if q & 1:
            q += 1
        expect = Fraction(q * 4) * Fraction(2) ** (-p)
        assert mul(a, three).to_fraction() == expect


def test_signed_zero_table():
    p = 128
    pz, nz = mpnum.zero(p, 0), mpnum.zero(p, 1)
    x = mpnum.from_int(5, p)
    assert add(pz, pz).key() == (0, 0, None)
    assert add(nz, nz).key() == (1, 0, None)
    assert add(pz, nz).key() == (0, 0, None)
    assert add(nz, pz).key() == (0, 0, None)
    assert add(x, nz) == x and add(nz, x) == x and add(x, pz) == x
    assert mul(nz, x).key() == (1, 0, None)
    assert mul(nz, x.neg()).key() == (0, 0, None)
    assert mul(x.neg(), pz).key() == (1, 0, None)
    assert sub(x, x).key() == (0, 0, None)
    assert div(nz, x).key() == (1, 0, None)
    assert sqrt(nz).key() == (1, 0, None)


def neighbours(r):
    p = r.p
    lo = r.to_fraction() - Fraction(2) ** (r.e - p) / (2 if r.m == (1 << (p - 1)) else 1)
    hi = r.to_fraction() + Fraction(2) ** (r.e - p)
    return lo, hi


@pytest.mark.parametrize("p", [128, 512])
def test_div_sqrt_nearest_characterisation(p):
    rng = random.Random(3 * p)
    for _ in range(200):
        a = rand_mp(rng, p)
        b = rand_mp(rng, p)
        v = a.to_fraction() / b.to_fraction()
        r = div(a, b)
        rr = abs(r.to_fraction())
        lo, hi = neighbours(MP(0, r.m, r.e, p))
        av = abs(v)
        assert abs(av - rr) <= abs(av - lo) and abs(av - rr) <= abs(av - hi)
        aa = MP(0, a.m, a.e, p)
        s = sqrt(aa)
        lo, hi = neighbours(s)
        sv = s.to_fraction()
        # s is nearest to sqrt(aa): the midpoints around s bracket sqrt(aa)
        assert ((lo + sv) / 2) ** 2 < aa.to_fraction() < ((sv + hi) / 2) ** 2


def test_range_error():
    p = 128
    big = MP(0, 1 << (p - 1), mpnum.EMAX, p)
    with pytest.raises(mpnum.MPRangeError):
        mul(big, big)
    tiny = MP(0, 1 << (p - 1), mpnum.EMIN, p)
    with pytest.raises(mpnum.MPRangeError):
        mul(tiny, tiny)
