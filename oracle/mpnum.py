"""Reference multiple-precision numbers: exact arithmetic, then one round-to-nearest.

TEST INFRASTRUCTURE ONLY. This package is the slow, obviously-correct CPU oracle for the
multiple-precision SpMV / Krylov path. Only the test suite, the smoke check and the CPU-baseline
leg of the benchmark may import it; the product path never does.

Number model (Kouya, Sec. 2: the MPFR number, IEEE-754-1985-like semantics, a p-bit mantissa
kept apart from the exponent, round-to-nearest mode):

    x = (-1)^s * M * 2^(e - p),   2^(p-1) <= M < 2^p     (mantissa in [1/2, 1), as MPFR)

A zero is M == 0 with its sign bit kept (IEEE signed zero).  The exponent range is MPFR's
default [1 - 2^30, 2^30 - 1]; a result outside it raises MPRangeError (the paper never leaves
it; no overflow/underflow emulation).  There are no NaN/Inf values.

Every operation computes the exact rational result and rounds it once, ties to even.  Nothing
here is blocked, fused or reordered; the only primitive used is Python's unbounded int.
"""
from fractions import Fraction
import math

EMIN = 1 - (1 << 30)
EMAX = (1 << 30) - 1


class MPRangeError(ArithmeticError):
    """The rounded result's exponent is outside [EMIN, EMAX]."""


class MP:
    """An immutable p-bit binary floating-point number (sign, mantissa, exponent)."""

    __slots__ = ("s", "m", "e", "p")

    def __init__(self, s, m, e, p):
        self.s = int(s) & 1
        self.m = int(m)
        self.e = int(e) if m else 0
        self.p = int(p)
        if m:
            assert (1 << (p - 1)) <= m < (1 << p), "mantissa not normalised"
            if not (EMIN <= e <= EMAX):
                raise MPRangeError(e)

    # ---- predicates and views -------------------------------------------------------
    def is_zero(self):
        return self.m == 0

    def to_fraction(self):
        """Exact rational value (a signed zero maps to 0)."""
        if self.m == 0:
            return Fraction(0)
        f = Fraction(self.m) * (Fraction(2) ** (self.e - self.p))
        return -f if self.s else f

    def key(self):
        """Bitwise identity: (sign, mantissa, exponent) with zeros keeping their sign."""
        return (self.s, self.m, self.e if self.m else None)

    def __eq__(self, other):
        return isinstance(other, MP) and self.p == other.p and self.key() == other.key()

    def __hash__(self):
        return hash(self.key())

    def __repr__(self):
        if self.m == 0:
            return "MP(%s0, p=%d)" % ("-" if self.s else "+", self.p)
        return "MP(%s0x%x * 2^(%d-%d))" % ("-" if self.s else "+", self.m, self.e, self.p)

    def neg(self):
        return MP(self.s ^ 1, self.m, self.e, self.p)


def zero(p, s=0):
    return MP(s, 0, 0, p)


# ---- rounding -----------------------------------------------------------------------
def round_scaled(sign, n, k, p):
    """RN_p of the exact dyadic value (-1)^sign * n * 2^k, for an integer n >= 1.

    Step by step as the definition of round-to-nearest-even: locate the leading bit, keep p
    bits, compare the discarded tail with one half of the last kept unit.
    """
    assert n > 0
    nb = n.bit_length()
    big_e = nb + k                      # 2^(E-1) <= |v| < 2^E
    drop = nb - p
    if drop <= 0:
        return MP(sign, n << (-drop), big_e, p)
    q = n >> drop
    r = n - (q << drop)
    half = 1 << (drop - 1)
    if r > half or (r == half and (q & 1)):
        q += 1
        if q == (1 << p):
            q >>= 1
            big_e += 1
    return MP(sign, q, big_e, p)


def round_fraction(v, p):
    """RN_p of an arbitrary rational v (a Fraction). An exact zero rounds to +0.

    Follows the textbook definition directly: find E with 2^(E-1) <= |v| < 2^E, scale |v| by
    2^(p-E), split into integer part q and fraction r, round up iff r > 1/2 or r == 1/2 with q
    odd, and renormalise if q reached 2^p.
    """
    v = Fraction(v)
    if v == 0:
        return zero(p)
    sign = 1 if v < 0 else 0
    a = -v if sign else v
    # E = floor(log2 a) + 1, found exactly from numerator/denominator bit lengths
    big_e = a.numerator.bit_length() - a.denominator.bit_length()
    while Fraction(2) ** big_e <= a:
        big_e += 1
    while Fraction(2) ** (big_e - 1) > a:
        big_e -= 1
    scaled = a * (Fraction(2) ** (p - big_e))      # in [2^(p-1), 2^p)
    q = scaled.numerator // scaled.denominator
    r = scaled - q
    if r > Fraction(1, 2) or (r == Fraction(1, 2) and (q & 1)):
        q += 1
        if q == (1 << p):
            q >>= 1
            big_e += 1
    return MP(sign, q, big_e, p)


def from_fraction(v, p):
    return round_fraction(v, p)


def from_int(v, p):
    return round_fraction(Fraction(int(v)), p)


def from_float(v, p):
    """Exact widening of an IEEE double (p >= 53 keeps every double exactly)."""
    return round_fraction(Fraction(float(v)), p)


# ---- the arithmetic primitives (RN, ties to even) -------------------------------------
def mul(a, b):
    """RN(a * b).  A zero factor gives a zero whose sign is the xor of the signs."""
    p = a.p
    s = a.s ^ b.s
    if a.m == 0 or b.m == 0:
        return zero(p, s)
    return round_scaled(s, a.m * b.m, a.e + b.e - 2 * p, p)


def add(a, b):
    """RN(a + b) with IEEE/MPFR signed-zero rules for round-to-nearest.

    (+0)+(+0)=+0, (-0)+(-0)=-0, (+0)+(-0)=+0, x+(+-0)=x, and an exact zero sum x+(-x)=+0.
    """
    p = a.p
    if a.m == 0 and b.m == 0:
        return zero(p, a.s & b.s)
    if a.m == 0:
        return b
    if b.m == 0:
        return a
    lo = min(a.e, b.e) - p
    na = a.m << (a.e - p - lo)
    nb = b.m << (b.e - p - lo)
    n = (-na if a.s else na) + (-nb if b.s else nb)
    if n == 0:
        return zero(p)
    return round_scaled(1 if n < 0 else 0, abs(n), lo, p)


def sub(a, b):
    """RN(a - b) = RN(a + (-b))."""
    return add(a, b.neg())


def div(a, b):
    """RN(a / b); b must be non-zero. 0/b is a zero with the xor sign."""
    p = a.p
    if b.m == 0:
        raise ZeroDivisionError("MP division by zero")
    s = a.s ^ b.s
    if a.m == 0:
        return zero(p, s)
    return round_fraction(Fraction(-1 if s else 1) * abs(a.to_fraction()) / abs(b.to_fraction()), p)


def sqrt(a):
    """RN(sqrt(a)) for a >= 0 (sqrt(+-0) = +-0).

    Integer square root of the scaled mantissa plus a remainder test: with the radicand
    written as R * 2^(2k), isqrt(R) carries p+1 significant bits, so the last one is the
    round bit and a non-zero remainder is the sticky information.  Ties cannot occur.
    """
    p = a.p
    if a.m == 0:
        return a
    if a.s:
        raise ValueError("sqrt of a negative MP number")
    # value = m * 2^(e-p) = R * 2^k2 with k2 even and 2^(2p) <= R < 2^(2p+2), so that
    # isqrt(R) has exactly p+1 bits.
    t = a.e - p                      # value = m * 2^t
    shift = p + 1                    # R = m * 2^shift has 2p+1 bits ...
    if (t - shift) % 2:
        shift += 1                   # ... or 2p+2 bits, so that the exponent k2 is even
    r_int = a.m << shift
    k2 = t - shift                   # value = r_int * 2^k2, k2 even
    s_root = math.isqrt(r_int)
    exact = (s_root * s_root == r_int)
    # s_root has p+1 bits (2^p <= s_root < 2^(p+1)); value = s_root' * 2^(k2/2)
    nbits = s_root.bit_length()
    assert nbits == p + 1, (nbits, p)
    q = s_root >> 1
    round_bit = s_root & 1
    sticky = not exact
    big_e = nbits + k2 // 2
    if round_bit and (sticky or (q & 1)):
        q += 1
        if q == (1 << p):
            q >>= 1
            big_e += 1
    return MP(0, q, big_e, p)


def le(a, b):
    """a <= b on the represented values."""
    return a.to_fraction() <= b.to_fraction()


def is_zero(a):
    return a.m == 0
