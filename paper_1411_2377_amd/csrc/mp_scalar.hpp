// Scalar p-bit operations used by the Krylov drivers on the device: RN division, RN square
// root, and the exact form of the stopping test ||r|| <= thr without a square root.
//
// Division is schoolbook long division on 32-bit digits (Knuth, TAOCP Vol. 2, Sec. 4.3.1,
// Algorithm D), with each quotient digit estimated in double precision from three remainder and
// two divisor digits, so that it is exact or one too large and at most one add-back fixes it.
// The square root is the binary digit-by-digit method on the scaled mantissa; a non-zero
// remainder is the sticky bit.
#pragma once
#include "mp_core.hpp"

namespace mp {

// Compare two N-limb unsigned integers: -1, 0, 1.
template <int N>
MPD int cmp_n(const uint32_t (&a)[N], const uint32_t (&b)[N]) {
#pragma unroll
  for (int i = N - 1; i >= 0; --i) {
    if (a[i] != b[i]) return a[i] < b[i] ? -1 : 1;
  }
  return 0;
}

// RN(a / b).  b == 0 sets kStDivZero and returns +0.
template <int L>
MPD Num<L> div_rn(const Num<L>& a, const Num<L>& b, uint32_t& st) {
  Num<L> r;
  if (is_zero(b)) {
    st |= kStDivZero;
    set_zero(r, 0);
    return r;
  }
  if (is_zero(a)) {
    set_zero(r, a.s ^ b.s);
    return r;
  }
  // u = M_a * 2^(p+1): limbs [0, L) zero, [L, 2L] = M_a << 1, plus one spare top limb.
  constexpr int NU = 2 * L + 1;
  uint32_t u[NU + 1];
#pragma unroll
  for (int i = 0; i < L; ++i) u[i] = 0;
  u[L] = a.m[0] << 1;
#pragma unroll
  for (int i = 1; i < L; ++i) u[L + i] = fshr(a.m[i], a.m[i - 1], 31);
  u[2 * L] = a.m[L - 1] >> 31;
  u[NU] = 0;
  const uint32_t* v = b.m;
  uint32_t q[NU - L + 1];
  // Trial digit: the top three remainder limbs times the reciprocal of the top two divisor
  // limbs, in double precision, plus 2^-17, truncated (and capped at 2^32 - 1).  The quotient
  // of the truncated operands exceeds the true one by less than 2^-30 (the divisor is
  // normalised) and the rounding errors stay below 2^-18, so the trial digit is the true digit
  // or one more: a single add-back (rare) makes it exact.
  const double rv = 1.0 / ((double)v[L - 1] * 4294967296.0 + (double)v[L - 2]);
#pragma unroll
  for (int j = NU - L; j >= 0; --j) {
    const double ud =
        ((double)u[j + L] * 4294967296.0 + (double)u[j + L - 1]) * 4294967296.0 + (double)u[j + L - 2];
    uint32_t qhat = (uint32_t)fmin(fma(ud, rv, 0x1p-17), 4294967295.0);
    // u[j .. j+L] -= qhat * v
    uint32_t c = 0, bw = 0;
#pragma unroll
    for (int i = 0; i < L; ++i) {
      const uint64_t t = (uint64_t)qhat * v[i] + c;
      c = (uint32_t)(t >> 32);
      u[j + i] = __builtin_subc(u[j + i], (uint32_t)t, bw, &bw);
    }
    u[j + L] = __builtin_subc(u[j + L], c, bw, &bw);
    if (bw) {  // the trial digit was one too large: add v back
      qhat -= 1;
      uint32_t cy = 0;
#pragma unroll
      for (int i = 0; i < L; ++i) u[i + j] = __builtin_addc(u[i + j], v[i], cy, &cy);
      u[j + L] += cy;
    }
    q[j] = qhat;
  }
  // quotient Q = q[0 .. L+1] (p+1 or p+2 bits); remainder in u[0 .. L)
  uint32_t rem = 0;
#pragma unroll
  for (int i = 0; i < L; ++i) rem |= u[i];
  const bool big = (q[L] >> 1) != 0;  // Q >= 2^(p+1)
  uint32_t rnd, sticky = rem;
  if (big) {
#pragma unroll
    for (int k = 0; k < L; ++k) r.m[k] = fshr(q[k + 1], q[k], 2);
    rnd = (q[0] >> 1) & 1u;
    sticky |= q[0] & 1u;
  } else {
#pragma unroll
    for (int k = 0; k < L; ++k) r.m[k] = fshr(q[k + 1], q[k], 1);
    rnd = q[0] & 1u;
  }
  int32_t e = a.e - b.e + (big ? 1 : 0);
  uint32_t cy = rnd & (uint32_t)((sticky != 0) | (r.m[0] & 1u));
#pragma unroll
  for (int k = 0; k < L; ++k) r.m[k] = __builtin_addc(r.m[k], 0u, cy, &cy);
  if (cy) {
    r.m[L - 1] = 0x80000000u;
    e += 1;
  }
  r.e = e;
  r.s = a.s ^ b.s;
  if (e > kEmax || e < kEmin) {
    st |= kStRange;
    set_zero(r, r.s);
  }
  return r;
}

// RN(sqrt(a)) for a >= 0 (a negative argument returns +0 and sets kStDivZero).
template <int L>
MPD Num<L> sqrt_rn(const Num<L>& a, uint32_t& st) {
  Num<L> r;
  if (is_zero(a)) return a;
  if (a.s) {
    st |= kStDivZero;
    set_zero(r, 0);
    return r;
  }
  // value = M * 2^(e-p) = R * 2^k2 with R = M << sh, sh in {p+1, p+2} so that k2 is even;
  // R has 2p+1 or 2p+2 bits and floor(sqrt(R)) has exactly p+1 bits.
  constexpr int NR = 2 * L + 1;
  const int32_t t = a.e - 32 * L;
  int sh = 32 * L + 1;
  if ((t - sh) & 1) sh += 1;
  const int32_t k2 = t - sh;
  uint32_t x[NR];  // R
#pragma unroll
  for (int i = 0; i < NR; ++i) x[i] = 0;
  // M << sh with sh = 32L + 1 or 32L + 2: limbs L.. hold M << (sh - 32L)
  const uint32_t bs = (uint32_t)(sh - 32 * L);
  x[L] = a.m[0] << bs;
#pragma unroll
  for (int i = 1; i < L; ++i) x[L + i] = fshr(a.m[i], a.m[i - 1], 32u - bs);
  x[2 * L] = a.m[L - 1] >> (32u - bs);
  uint32_t res[NR], bit[NR];
#pragma unroll
  for (int i = 0; i < NR; ++i) {
    res[i] = 0;
    bit[i] = 0;
  }
  // highest power of four <= R: R has nbits = 32L + bs + 32(L-1)... top bit index known
  const int topbit = 32 * L + (int)bs + 32 * L - 1;  // index of R's leading one
  const int b4 = topbit & ~1;
  for (int i = 0; i < NR; ++i) bit[i] = (i == (b4 >> 5)) ? (1u << (b4 & 31)) : 0u;
  for (int it = b4; it >= 0; it -= 2) {
    uint32_t tmp[NR];
    uint32_t cy = 0;
#pragma unroll
    for (int i = 0; i < NR; ++i) tmp[i] = __builtin_addc(res[i], bit[i], cy, &cy);
    const bool ge = cmp_n<NR>(x, tmp) >= 0;
    if (ge) {
      uint32_t bw = 0;
#pragma unroll
      for (int i = 0; i < NR; ++i) x[i] = __builtin_subc(x[i], tmp[i], bw, &bw);
    }
    // res = (res >> 1) (+ bit)
#pragma unroll
    for (int i = 0; i < NR - 1; ++i) res[i] = fshr(res[i + 1], res[i], 1);
    res[NR - 1] >>= 1;
    if (ge) {
      uint32_t c2 = 0;
#pragma unroll
      for (int i = 0; i < NR; ++i) res[i] = __builtin_addc(res[i], bit[i], c2, &c2);
    }
    // bit >>= 2
#pragma unroll
    for (int i = 0; i < NR - 1; ++i) bit[i] = fshr(bit[i + 1], bit[i], 2);
    bit[NR - 1] >>= 2;
  }
  // res = floor(sqrt(R)) with p+1 bits; remainder in x
  uint32_t rem = 0;
#pragma unroll
  for (int i = 0; i < NR; ++i) rem |= x[i];
#pragma unroll
  for (int k = 0; k < L; ++k) r.m[k] = fshr(res[k + 1], res[k], 1);
  const uint32_t rnd = res[0] & 1u;
  int32_t e = 32 * L + 1 + k2 / 2;
  uint32_t cy = rnd & (uint32_t)((rem != 0) | (r.m[0] & 1u));
#pragma unroll
  for (int k = 0; k < L; ++k) r.m[k] = __builtin_addc(r.m[k], 0u, cy, &cy);
  if (cy) {
    r.m[L - 1] = 0x80000000u;
    e += 1;
  }
  r.e = e;
  r.s = 0;
  return r;
}

// The stopping test RN(sqrt(q)) <= thr for q >= 0 (an RN'd inner product) and thr >= 0, decided
// exactly: with thr+ = thr + ulp(thr)/2, RN(sqrt q) <= thr  <=>  q < thr+^2 (the midpoint square
// is never a p-bit number, so equality cannot occur).  thr == 0 accepts only q == 0.
template <int L>
MPD bool sqrt_le(const Num<L>& q, const Num<L>& thr) {
  if (is_zero(q)) return true;
  if (is_zero(thr)) return false;
  // S = (2 M_thr + 1)^2, L+1 limbs squared into 2L+2 limbs
  uint32_t m2[L + 1];
  m2[0] = (thr.m[0] << 1) | 1u;
#pragma unroll
  for (int i = 1; i < L; ++i) m2[i] = fshr(thr.m[i], thr.m[i - 1], 31);
  m2[L] = thr.m[L - 1] >> 31;
  uint32_t S[2 * L + 2];
#pragma unroll
  for (int i = 0; i < 2 * L + 2; ++i) S[i] = 0;
#pragma unroll
  for (int i = 0; i <= L; ++i) {
    uint32_t c = 0;
#pragma unroll
    for (int j = 0; j <= L; ++j) {
      const uint64_t tt = (uint64_t)m2[i] * m2[j] + S[i + j] + c;
      S[i + j] = (uint32_t)tt;
      c = (uint32_t)(tt >> 32);
    }
    S[i + L + 1] = c;
  }
  // thr+^2 = S * 2^(2 e_t - 2p - 2); S has nb bits; q = M_q * 2^(e_q - p)
  uint32_t lz = 0;
  bool found = false;
#pragma unroll
  for (int i = 2 * L + 1; i >= 0; --i) {
    if (!found) {
      if (S[i]) {
        lz += __clz(S[i]);
        found = true;
      } else {
        lz += 32;
      }
    }
  }
  const int nb = 32 * (2 * L + 2) - (int)lz;
  const int64_t ER = (int64_t)nb + 2 * (int64_t)thr.e - 64 * L - 2;  // thr+^2 in [2^(ER-1), 2^ER)
  if ((int64_t)q.e < ER) return true;
  if ((int64_t)q.e > ER) return false;
  // same binade: compare M_q * 2^(nb - p) with S (both nb-bit integers)
  uint32_t Q[2 * L + 2];
#pragma unroll
  for (int i = 0; i < 2 * L + 2; ++i) Q[i] = 0;
  const int shq = nb - 32 * L;  // 32L+1 <= nb <= 64L+2  ->  1 <= shq <= 32L+2
  const int qq = shq >> 5, rr = shq & 31;
#pragma unroll
  for (int i = 0; i < 2 * L + 2; ++i) {
    const int src = i - qq;
    const uint32_t lo = (src - 1 >= 0 && src - 1 < L) ? q.m[src - 1] : 0u;
    const uint32_t hi = (src >= 0 && src < L) ? q.m[src] : 0u;
    Q[i] = rr ? fshr(hi, lo, 32u - (uint32_t)rr) : hi;
  }
  return cmp_n<2 * L + 2>(Q, S) < 0;
}

}  // namespace mp
