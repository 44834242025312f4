// Wide precisions (p = 2048, 4096, 8192; L = 64, 128, 256 limbs): one wavefront per number, the
// number's limbs in LDS, 64 limbs per step of a loop (limb tiles across the lanes).
//
// Building blocks, each called by all 64 lanes of a one-wavefront block:
//  * big integers of n limbs in LDS: addition / subtraction with carries resolved per 64 limbs
//    by two ballots (generate, propagate) and one 64-bit integer addition of the masks, carried
//    on to the next 64 limbs as a wave-uniform bit; shifts; the leading non-zero limb by ballots;
//  * the exact product by column sums (lane k sums the columns k, k + 64, ... in 96 bits), the
//    three words of each column then added into the limbs with carries passed lane to lane;
//  * RN of an exact magnitude: leading bit, p mantissa bits, round bit, sticky bits below it;
//  * RN addition (Y aligned below X with one guard limb and its shifted-out bits ORed into the
//    guard, added or subtracted, rounded), multiplication, division (restoring long division,
//    one quotient bit per step, p + 2 bits and the remainder as sticky) and square root (the
//    same, two radicand bits per step);
//  * exact sums: carry-save 64-bit digits in an LDS window at a 32-bit aligned anchor, each
//    product's 2L + 1 shifted limbs added by the lanes that own them, then carries, sign and one
//    RN rounding.
// Results are those of the fixed-width kernels and the oracle: one RN per operation, exact
// inner products and EXACT rows rounded once, SEQ rows folded in column order from +0.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <vector>

#include "../../include/mpspmv.h"
#include "api_internal.hpp"
#include "mp_core.hpp"
#include "wide_internal.hpp"

namespace {

using mp::fshr;
using mp::kEmax;
using mp::kEmin;
using mp::kStDivZero;
using mp::kStRange;
using mp::kStWindow;
using mp::kZeroE;

constexpr int kMaxL = 256;
constexpr int kBig = 2 * kMaxL + 8;  // limbs of the widest intermediate (a product plus headroom)
constexpr int kWinDigits = 4096;     // digits of an LDS window (an exact row or part of a dot)

struct WNum {
  int32_t e;   // kZeroE: zero
  uint32_t s;  // sign
};

MPD int lane_id() { return (int)(threadIdx.x & 63u); }
// one-wavefront blocks: orders the wavefront's LDS writes before other lanes' reads
MPD void wsync() { __syncthreads(); }

MPD uint64_t shfl_up64(uint64_t v) {
  const uint32_t lo = (uint32_t)__shfl_up((int)(uint32_t)v, 1, 64);
  const uint32_t hi = (uint32_t)__shfl_up((int)(uint32_t)(v >> 32), 1, 64);
  return ((uint64_t)hi << 32) | lo;
}
MPD uint64_t shfl64(uint64_t v, int src) {
  const uint32_t lo = (uint32_t)__shfl((int)(uint32_t)v, src, 64);
  const uint32_t hi = (uint32_t)__shfl((int)(uint32_t)(v >> 32), src, 64);
  return ((uint64_t)hi << 32) | lo;
}

// ---- big integers in LDS ------------------------------------------------------------------
MPD void big_set(uint32_t* d, int n, uint32_t v) {
  for (int j = lane_id(); j < n; j += 64) d[j] = v;
}
MPD void big_copy(uint32_t* d, const uint32_t* s, int n) {
  for (int j = lane_id(); j < n; j += 64) d[j] = s[j];
}

// index of the top non-zero limb of a[0..n), -1 if none
MPD int big_top(const uint32_t* a, int n) {
  const int ln = lane_id();
  for (int c0 = ((n - 1) >> 6) << 6; c0 >= 0; c0 -= 64) {
    const int j = c0 + ln;
    const uint64_t nz = __ballot(j < n && a[j] != 0u);
    if (nz) return c0 + 63 - (int)__clzll((long long)nz);
  }
  return -1;
}

MPD bool big_any(const uint32_t* a, int n) {
  const int ln = lane_id();
  for (int c0 = 0; c0 < n; c0 += 64)
    if (__ballot(c0 + ln < n && a[c0 + ln] != 0u)) return true;
  return false;
}

// d = a + (b or ~b) + cin over n limbs (d may be a or b: each limb is read and written by one
// lane); returns the carry out of limb n - 1
MPD uint32_t big_add(uint32_t* d, const uint32_t* a, const uint32_t* b, int n, bool inv_b, uint32_t cin) {
  const int ln = lane_id();
  uint32_t c = cin;
  for (int c0 = 0; c0 < n; c0 += 64) {
    const int j = c0 + ln;
    const bool in = j < n;
    const uint32_t x = in ? a[j] : 0u;
    const uint32_t y = in ? (inv_b ? ~b[j] : b[j]) : 0u;
    const uint32_t s0 = x + y;
    const uint64_t gen = __ballot(in && s0 < x);
    const uint64_t prop = __ballot(in && s0 == ~0u);
    // bit k: the carry into lane k (generated below it, or passed on by all-ones sums)
    const uint64_t car = ((((gen << 1) | (uint64_t)c)) + prop) ^ prop;
    if (in) d[j] = s0 + (uint32_t)((car >> ln) & 1ull);
    const int last = min(63, n - 1 - c0);
    c = (uint32_t)(((gen | (prop & car)) >> last) & 1ull);
  }
  return c;
}

// a = a + 1 over n limbs; returns the carry out
MPD uint32_t big_inc(uint32_t* a, int n) {
  const int ln = lane_id();
  uint32_t c = 1;
  for (int c0 = 0; c0 < n && c; c0 += 64) {
    const int j = c0 + ln;
    const bool in = j < n;
    const uint32_t x = in ? a[j] : 0u;
    const uint64_t prop = __ballot(in && x == ~0u);
    const uint64_t car = ((uint64_t)c + prop) ^ prop;
    if (in) a[j] = x + (uint32_t)((car >> ln) & 1ull);
    const int last = min(63, n - 1 - c0);
    c = (uint32_t)(((prop & car) >> last) & 1ull);
  }
  return c;
}

// a = -a (two's complement) over n limbs
MPD void big_neg(uint32_t* a, int n) {
  for (int j = lane_id(); j < n; j += 64) a[j] = ~a[j];
  wsync();
  big_inc(a, n);
}

// d[0..nd) = bits [s + 32 j, s + 32 j + 32) of x (x[i] = 0 outside [0, nx)), s >= 0 or < 0
// (a left shift); d must not alias x
MPD void big_window(uint32_t* d, int nd, const uint32_t* x, int nx, int64_t s) {
  const int64_t q = s >> 5;  // floor
  const uint32_t r = (uint32_t)(s & 31);
  for (int j = lane_id(); j < nd; j += 64) {
    const int64_t i = j + q;
    const uint32_t lo = (i >= 0 && i < nx) ? x[i] : 0u;
    const uint32_t hi = (i + 1 >= 0 && i + 1 < nx) ? x[i + 1] : 0u;
    d[j] = r ? fshr(hi, lo, r) : lo;
  }
}

// any non-zero bit of x below bit s (s >= 0)
MPD bool big_any_below(const uint32_t* x, int nx, int64_t s) {
  const int64_t q = min<int64_t>(s >> 5, nx);
  const uint32_t r = (uint32_t)(s & 31);
  if (big_any(x, (int)q)) return true;
  return r && q < nx && (x[q] & ((1u << r) - 1u)) != 0u;
}

// signed comparison helper: a >= b for n-limb magnitudes
MPD bool big_ge(const uint32_t* a, const uint32_t* b, int n) {
  const int ln = lane_id();
  for (int c0 = ((n - 1) >> 6) << 6; c0 >= 0; c0 -= 64) {
    const int j = c0 + ln;
    const uint64_t ne = __ballot(j < n && a[j] != b[j]);
    if (ne) {
      const int k = c0 + 63 - (int)__clzll((long long)ne);
      return a[k] > b[k];
    }
  }
  return true;
}

// p[0..La + Lb) = a * b exactly; c0, c1, c2 scratch of La + Lb + 2 words
MPD void big_mul(uint32_t* p, const uint32_t* a, int La, const uint32_t* b, int Lb, uint32_t* c0,
                 uint32_t* c1, uint32_t* c2) {
  const int n = La + Lb, ln = lane_id();
  big_set(c0, n + 2, 0u);
  big_set(c1, n + 2, 0u);
  big_set(c2, n + 2, 0u);
  wsync();
  for (int k = ln; k < n - 1; k += 64) {
    uint64_t lo = 0;
    uint32_t hi = 0;
    const int i0 = max(0, k - (Lb - 1)), i1 = min(k, La - 1);
    for (int i = i0; i <= i1; ++i) {
      const uint64_t pr = (uint64_t)a[i] * b[k - i];
      lo += pr;
      hi += (lo < pr) ? 1u : 0u;
    }
    c0[k] = (uint32_t)lo;
    c1[k + 1] = (uint32_t)(lo >> 32);
    c2[k + 2] = hi;
  }
  wsync();
  uint64_t cin = 0;
  for (int b0 = 0; b0 < n; b0 += 64) {
    const int j = b0 + ln;
    uint64_t v = (j < n) ? (uint64_t)c0[j] + c1[j] + c2[j] : 0ull;
    if (ln == 0) v += cin;
    uint32_t lo = (uint32_t)v;
    uint64_t c = v >> 32;
    uint64_t out = 0;
    while (__ballot(c != 0ull)) {
      const uint64_t from = shfl_up64(c);
      if (ln == 63) out += c;
      const uint64_t t = (uint64_t)lo + (ln ? from : 0ull);
      lo = (uint32_t)t;
      c = t >> 32;
    }
    if (j < n) p[j] = lo;
    cin = shfl64(out, 63);
  }
  wsync();
}

// ---- rounding -----------------------------------------------------------------------------
// RN_p of (-1)^sgn (m + f) 2^base, m = m[0..n) a non-negative integer and 0 <= f < 1 non-zero
// exactly when `sticky_in` (only with at least p + 1 bits in m); the mantissa goes to dst[0..L)
MPD WNum round_mag(uint32_t* dst, int L, const uint32_t* m, int n, int64_t base, uint32_t sgn,
                   bool sticky_in, uint32_t& st) {
  WNum out;
  const int top = big_top(m, n);
  if (top < 0) {
    big_set(dst, L, 0u);
    wsync();
    out.e = kZeroE;
    out.s = 0;
    return out;
  }
  const int64_t T = 32 * (int64_t)top + 31 - (int64_t)__clz((int)m[top]);  // leading bit
  const int64_t b0 = T - 32 * (int64_t)L + 1;                               // mantissa LSB
  big_window(dst, L, m, n, b0);
  bool sticky = sticky_in;
  uint32_t rnd = 0;
  const int64_t rb = b0 - 1;
  if (rb >= 0) {
    rnd = (m[rb >> 5] >> (uint32_t)(rb & 31)) & 1u;
    if (!sticky) sticky = big_any_below(m, n, rb);
  }
  wsync();
  int64_t e = b0 + base + 32 * (int64_t)L;
  if (rnd && (sticky || (dst[0] & 1u))) {
    if (big_inc(dst, L)) {  // 1.11..1 rounded up: 2^(p-1) one exponent up
      wsync();
      big_set(dst, L, 0u);
      wsync();
      if (lane_id() == 0) dst[L - 1] = 0x80000000u;
      e += 1;
    }
  }
  wsync();
  out.s = sgn;
  if (e > kEmax || e < kEmin) {
    st |= kStRange;
    big_set(dst, L, 0u);
    wsync();
    out.e = kZeroE;
    return out;
  }
  out.e = (int32_t)e;
  return out;
}

// ---- the operations -----------------------------------------------------------------------
// Workspace of one block: operands, results and scratch limbs (the exact window lives apart).
struct Lds {
  uint32_t x[kMaxL + 4], y[kMaxL + 4], acc[kMaxL + 4], t[kMaxL + 4];
  uint32_t p[kBig], s1[kBig], s2[kBig], s3[kBig], c0[kBig], c1[kBig], c2[kBig];
};

MPD WNum wide_mul(Lds& S, uint32_t* z, int L, const uint32_t* x, WNum xe, const uint32_t* y, WNum ye,
                  uint32_t& st) {
  if (xe.e == kZeroE || ye.e == kZeroE) {
    big_set(z, L, 0u);
    wsync();
    return WNum{kZeroE, xe.s ^ ye.s};
  }
  big_mul(S.p, x, L, y, L, S.c0, S.c1, S.c2);
  return round_mag(z, L, S.p, 2 * L, (int64_t)xe.e + ye.e - 64 * (int64_t)L, xe.s ^ ye.s, false, st);
}

// z = RN(x + (-1)^neg_y y); z must not alias x or y
MPD WNum wide_add(Lds& S, uint32_t* z, int L, const uint32_t* x, WNum xe, const uint32_t* y, WNum ye,
                  uint32_t& st) {
  const bool xz = xe.e == kZeroE, yz = ye.e == kZeroE;
  if (xz || yz) {
    const uint32_t* src = xz ? y : x;
    big_copy(z, src, L);
    wsync();
    if (xz && yz) return WNum{kZeroE, xe.s & ye.s};  // (-0) + (-0) = -0, else +0
    return xz ? ye : xe;
  }
  const bool sw = ye.e > xe.e;
  const uint32_t* X = sw ? y : x;
  const uint32_t* Y = sw ? x : y;
  const WNum Xn = sw ? ye : xe, Yn = sw ? xe : ye;
  const int64_t p = 32 * (int64_t)L;
  int64_t d = (int64_t)Xn.e - Yn.e;
  if (d > p + 2) d = p + 2;  // Y below a quarter of X's last unit: only its sticky bit counts
  // s1 = X 2^32 (guard limb below), s3 = Y 2^32, s2 = s3 >> d with the lost bits in bit 0
  const int ln = lane_id();
  if (ln == 0) {
    S.s1[0] = 0u;
    S.s3[0] = 0u;
  }
  for (int j = ln; j < L; j += 64) {
    S.s1[j + 1] = X[j];
    S.s3[j + 1] = Y[j];
  }
  wsync();
  big_window(S.s2, L + 1, S.s3, L + 1, d);
  const bool lost = big_any_below(S.s3, L + 1, d);
  wsync();
  if (lost && ln == 0) S.s2[0] |= 1u;
  wsync();
  uint32_t sgn = Xn.s;
  int n;
  if (Xn.s == Yn.s) {
    const uint32_t co = big_add(S.s1, S.s1, S.s2, L + 1, false, 0u);
    wsync();
    if (ln == 0) S.s1[L + 1] = co;
    n = L + 2;
  } else {
    const uint32_t nb = big_add(S.s1, S.s1, S.s2, L + 1, true, 1u);  // no borrow: |X| >= |Y|
    wsync();
    if (!nb) {
      big_neg(S.s1, L + 1);
      sgn ^= 1u;
    }
    n = L + 1;
  }
  wsync();
  return round_mag(z, L, S.s1, n, (int64_t)Xn.e - p - 32, sgn, false, st);
}

// z = RN(a / b): Q = floor(Ma 2^(p+1) / Mb) by long division in radix 2^32, the remainder's
// non-zero-ness as sticky.  R = 2 Ma first gives the top quotient digit (1, 2 or 3, by repeated
// subtraction); then each of the L steps shifts R up one limb, estimates the next digit from
// R's top two limbs over Mb's top limb (Mb is normalised, so the estimate is at most 2 too
// large: Knuth, TAOCP 4.3.1, algorithm D), subtracts digit x Mb and adds Mb back while the
// remainder is negative.
MPD WNum wide_div(Lds& S, uint32_t* z, int L, const uint32_t* a, WNum ae, const uint32_t* b, WNum be,
                  uint32_t& st) {
  if (be.e == kZeroE) {
    st |= kStDivZero;
    big_set(z, L, 0u);
    wsync();
    return WNum{kZeroE, 0u};
  }
  if (ae.e == kZeroE) {
    big_set(z, L, 0u);
    wsync();
    return WNum{kZeroE, ae.s ^ be.s};
  }
  const int p = 32 * L, n = L + 1, ln = lane_id();
  uint32_t* R = S.s1;
  uint32_t* U = S.s2;
  uint32_t* T = S.s3;
  uint32_t* H = S.c1;
  uint32_t* Q = S.p;
  uint32_t* B = S.c0;
  big_set(Q, L + 2, 0u);
  for (int j = ln; j < n; j += 64) {
    U[j] = j < L ? a[j] : 0u;
    B[j] = j < L ? b[j] : 0u;
  }
  wsync();
  big_window(R, n, U, n, -1);  // R = 2 Ma < 4 Mb
  wsync();
  uint32_t q0 = 0;
  for (int k = 0; k < 3; ++k) {
    const uint32_t nb = big_add(T, R, B, n, true, 1u);  // T = R - Mb
    wsync();
    if (!nb) break;
    uint32_t* t = R;
    R = T;
    T = t;
    ++q0;
  }
  const uint32_t dtop = B[L - 1];
  for (int j = 1; j <= L; ++j) {
    // U = R 2^32 (R < Mb, so U fits L + 1 limbs)
    for (int k = ln; k < n; k += 64) U[k] = k ? R[k - 1] : 0u;
    wsync();
    const uint64_t num = ((uint64_t)U[L] << 32) | U[L - 1];
    uint32_t qh = (uint32_t)min(num / dtop, (uint64_t)0xffffffffu);
    // T = qh * Mb: low words in place, high words one limb up, then added
    for (int k = ln; k < n; k += 64) {
      const uint64_t pr = (uint64_t)qh * (k < L ? B[k] : 0u);
      T[k] = (uint32_t)pr;
      H[k + 1] = (uint32_t)(pr >> 32);
    }
    if (ln == 0) H[0] = 0u;
    wsync();
    big_add(T, T, H, n, false, 0u);
    wsync();
    uint32_t nb = big_add(R, U, T, n, true, 1u);  // R = U - T (nb: no borrow)
    wsync();
    for (int k = 0; k < 3 && !nb; ++k) {  // the estimate was too large: add Mb back
      nb = big_add(R, R, B, n, false, 0u);
      wsync();
      --qh;
    }
    if (ln == 0) Q[L - j] = qh;
  }
  if (ln == 0) Q[L] = q0;
  wsync();
  const bool sticky = big_any(R, n);
  wsync();
  return round_mag(z, L, Q, L + 2, (int64_t)ae.e - be.e - p - 1, ae.s ^ be.s, sticky, st);
}

// z = RN(sqrt(a)) for a >= 0: N = Ma 2^k (2p + 2 or 2p + 3 bits, k making the exponent even),
// Q = isqrt(N) two radicand bits per step, the remainder as sticky
MPD WNum wide_sqrt(Lds& S, uint32_t* z, int L, const uint32_t* a, WNum ae, uint32_t& st) {
  if (ae.e == kZeroE) {
    big_set(z, L, 0u);
    wsync();
    return WNum{kZeroE, ae.s};
  }
  if (ae.s) {
    st |= kStDivZero;
    big_set(z, L, 0u);
    wsync();
    return WNum{kZeroE, 0u};
  }
  const int p = 32 * L, ln = lane_id();
  const int64_t E = (int64_t)ae.e - p;                       // a = Ma 2^E
  const int k = ((E - (p + 2)) & 1) ? p + 3 : p + 2;         // E - k even
  const int nbits = p + k;                                   // bits of N (Ma has p bits)
  const int n = L + 2;                                       // R < 2 Q + 1 < 2^(p + 3)
  uint32_t* R = S.s1;
  uint32_t* T = S.s2;
  uint32_t* U = S.s3;
  uint32_t* Q = S.p;
  uint32_t* Q4 = S.c0;
  big_set(R, n, 0u);
  big_set(Q, n, 0u);
  wsync();
  for (int pos = nbits - 2 + (nbits & 1); pos >= 0; pos -= 2) {
    // R = 4 R + the radicand bits pos + 1, pos (bit j of N is bit j - k of Ma)
    big_window(U, n, R, n, -2);
    wsync();
    const int j1 = pos + 1 - k, j0 = pos - k;
    uint32_t two = 0;
    if (j1 >= 0 && j1 < p) two |= ((a[j1 >> 5] >> (j1 & 31)) & 1u) << 1;
    if (j0 >= 0 && j0 < p) two |= (a[j0 >> 5] >> (j0 & 31)) & 1u;
    if (ln == 0) U[0] |= two;
    // Q4 = 4 Q + 1
    big_window(Q4, n, Q, n, -2);
    wsync();
    if (ln == 0) Q4[0] |= 1u;
    wsync();
    const uint32_t nb = big_add(T, U, Q4, n, true, 1u);  // T = R - (4 Q + 1)
    wsync();
    // Q = 2 Q + (R >= 4 Q + 1)
    big_window(Q4, n, Q, n, -1);
    wsync();
    if (ln == 0 && nb) Q4[0] |= 1u;
    wsync();
    big_copy(Q, Q4, n);
    big_copy(R, nb ? T : U, n);
    wsync();
  }
  const bool sticky = big_any(R, n);
  wsync();
  // sqrt(a) = sqrt(N) 2^((E - k) / 2)
  return round_mag(z, L, Q, n, (E - k) / 2, 0u, sticky, st);
}

// RN(sqrt q) <= thr for q, thr >= 0 (the stopping test), decided exactly: with thr+ = thr +
// ulp(thr)/2, RN(sqrt q) <= thr <=> q < thr+^2 (the midpoint square is never a p-bit number)
MPD bool wide_sqrt_le(Lds& S, int L, const uint32_t* q, WNum qe, const uint32_t* thr, WNum te) {
  if (qe.e == kZeroE) return true;
  if (te.e == kZeroE) return false;
  const int ln = lane_id();
  // c1 = 2 M_thr + 1 (L + 1 limbs); p = c1^2 (2L + 2 limbs)
  uint32_t* M2 = S.s3;
  big_window(M2, L + 1, thr, L, -1);
  wsync();
  if (ln == 0) M2[0] |= 1u;
  wsync();
  big_mul(S.p, M2, L + 1, M2, L + 1, S.c0, S.c1, S.c2);
  const int nS = 2 * L + 2;
  const int topS = big_top(S.p, nS);
  const int64_t nb = 32 * (int64_t)topS + 32 - (int64_t)__clz((int)S.p[topS]);
  const int64_t ER = nb + 2 * (int64_t)te.e - 64 * (int64_t)L - 2;  // thr+^2 in [2^(ER-1), 2^ER)
  if ((int64_t)qe.e < ER) return true;
  if ((int64_t)qe.e > ER) return false;
  // same binade: M_q 2^(nb - p) against the nb-bit integer in S.p
  big_window(S.s1, nS, q, L, -(nb - 32 * (int64_t)L));
  wsync();
  return !big_ge(S.s1, S.p, nS);
}

// ---- loads and stores ---------------------------------------------------------------------
MPD WNum load_num(uint32_t* d, int L, const uint32_t* limb, const int32_t* hdr, int64_t ld, int64_t i) {
  const int32_t h = hdr[i];
  WNum w{h >> 1, (uint32_t)h & 1u};
  for (int j = lane_id(); j < L; j += 64) d[j] = (w.e == kZeroE) ? 0u : limb[(int64_t)j * ld + i];
  wsync();
  return w;
}

MPD void store_num(const uint32_t* s, WNum w, int L, uint32_t* limb, int32_t* hdr, int64_t ld, int64_t i) {
  for (int j = lane_id(); j < L; j += 64) limb[(int64_t)j * ld + i] = s[j];
  if (lane_id() == 0) hdr[i] = mp::make_hdr(w.e, w.s);
}

// ---- exact sums -----------------------------------------------------------------------------
// win[(off >> 5) + j] += (-1)^s (P << (off & 31)) limb j, j = 0 .. 2L (each digit by one lane)
MPD void window_add(int64_t* win, const uint32_t* P, int L, uint32_t s, int64_t off) {
  const int64_t q = off >> 5;
  const uint32_t r = (uint32_t)(off & 31);
  for (int j = lane_id(); j <= 2 * L; j += 64) {
    const uint32_t lo = j > 0 ? P[j - 1] : 0u, hi = j < 2 * L ? P[j] : 0u;
    const uint32_t v = r ? fshr(hi, lo, 32u - r) : hi;
    win[q + j] += s ? -(int64_t)v : (int64_t)v;
  }
  wsync();
}

// Carry-save digits win[0..W) into magnitude limbs ml[0..W) and a sign (every lane).
MPD uint32_t window_normalize(uint32_t* ml, const int64_t* win, int W) {
  const int ln = lane_id();
  int64_t carry = 0;
  for (int c0 = 0; c0 < W; c0 += 64) {
    const int j = c0 + ln;
    int64_t d = (j < W) ? win[j] : 0;
    if (ln == 0) d += carry;
    uint32_t lo = (uint32_t)d;
    int64_t hi = d >> 32;
    int64_t out = 0;
    while (__ballot(hi != 0)) {
      const int64_t from = (int64_t)shfl_up64((uint64_t)hi);
      if (ln == 63) out += hi;
      const int64_t t = (int64_t)lo + (ln ? from : 0);
      lo = (uint32_t)t;
      hi = t >> 32;
    }
    if (j < W) ml[j] = lo;
    carry = (int64_t)shfl64((uint64_t)out, 63);
  }
  wsync();
  const uint32_t neg = carry < 0 ? 1u : 0u;
  if (neg) big_neg(ml, W);
  wsync();
  return neg;
}

}  // namespace

// ---- kernels ------------------------------------------------------------------------------
namespace wide_k {

struct SpmvA {
  int64_t n_rows;
  const int32_t* row_ptr;
  const int32_t* col_idx;
  const uint32_t* a_limb;
  const int32_t* a_hdr;
  int64_t a_ld;
  const uint32_t* x_limb;
  const int32_t* x_hdr;
  int64_t x_ld;
  uint32_t* y_limb;
  int32_t* y_hdr;
  int64_t y_ld;
  int L;
  uint32_t* status;
};

// SEQ rows: y_i = +0, then y_i = RN(y_i + RN(a_ik x_k)) in column order (zero products skipped:
// they leave y_i as it is)
__global__ void __launch_bounds__(64) spmv_seq(SpmvA A) {
  __shared__ Lds S;
  const int L = A.L;
  uint32_t st = 0;
  for (int64_t row = blockIdx.x; row < A.n_rows; row += gridDim.x) {
    WNum acc{kZeroE, 0u};
    big_set(S.acc, L, 0u);
    wsync();
    for (int32_t k = A.row_ptr[row]; k < A.row_ptr[row + 1]; ++k) {
      const int32_t ha = A.a_hdr[k];
      const int32_t col = A.col_idx[k];
      const int32_t hx = A.x_hdr[col];
      if (mp::hdr_is_zero(ha) || mp::hdr_is_zero(hx)) continue;
      const WNum a = load_num(S.x, L, A.a_limb, A.a_hdr, A.a_ld, k);
      const WNum x = load_num(S.y, L, A.x_limb, A.x_hdr, A.x_ld, col);
      const WNum t = wide_mul(S, S.t, L, S.x, a, S.y, x, st);
      const WNum r = wide_add(S, S.x, L, S.acc, acc, S.t, t, st);
      big_copy(S.acc, S.x, L);
      wsync();
      acc = r;
    }
    store_num(S.acc, acc, L, A.y_limb, A.y_hdr, A.y_ld, row);
    wsync();
  }
  if (st && lane_id() == 0) atomicOr(A.status, st);
}

// EXACT rows: the row's products in an LDS window at its 32-bit aligned exponent anchor, rounded
// once (a row spanning more than the window sets kStWindow and gives +0)
__global__ void __launch_bounds__(64) spmv_exact(SpmvA A) {
  __shared__ Lds S;
  __shared__ int64_t win[kWinDigits];
  __shared__ uint32_t ml[kWinDigits];
  const int L = A.L, ln = lane_id();
  uint32_t st = 0;
  for (int64_t row = blockIdx.x; row < A.n_rows; row += gridDim.x) {
    const int32_t rs = A.row_ptr[row], re = A.row_ptr[row + 1];
    int32_t lo = INT32_MAX, hi = INT32_MIN;
    for (int32_t k = rs + ln; k < re; k += 64) {
      const int32_t ha = A.a_hdr[k], hx = A.x_hdr[A.col_idx[k]];
      if (mp::hdr_is_zero(ha) || mp::hdr_is_zero(hx)) continue;
      const int32_t e = (ha >> 1) + (hx >> 1);
      lo = min(lo, e);
      hi = max(hi, e);
    }
    for (int o = 32; o > 0; o >>= 1) {
      lo = min(lo, __shfl_xor(lo, o, 64));
      hi = max(hi, __shfl_xor(hi, o, 64));
    }
    WNum y{kZeroE, 0u};
    big_set(S.acc, L, 0u);
    wsync();
    if (hi >= lo) {
      const int32_t anchor = lo & ~31;
      const int64_t W = (((int64_t)hi - anchor) >> 5) + 2 * L + 2;
      if (W > kWinDigits) {
        st |= kStWindow;
      } else {
        for (int j = ln; j < W; j += 64) win[j] = 0;
        wsync();
        for (int32_t k = rs; k < re; ++k) {
          const int32_t ha = A.a_hdr[k];
          const int32_t col = A.col_idx[k];
          const int32_t hx = A.x_hdr[col];
          if (mp::hdr_is_zero(ha) || mp::hdr_is_zero(hx)) continue;
          const WNum a = load_num(S.x, L, A.a_limb, A.a_hdr, A.a_ld, k);
          const WNum x = load_num(S.y, L, A.x_limb, A.x_hdr, A.x_ld, col);
          big_mul(S.p, S.x, L, S.y, L, S.c0, S.c1, S.c2);
          window_add(win, S.p, L, a.s ^ x.s, (int64_t)a.e + x.e - anchor);
        }
        const uint32_t neg = window_normalize(ml, win, (int)W);
        y = round_mag(S.acc, L, ml, (int)W, (int64_t)anchor - 64 * (int64_t)L, neg, false, st);
      }
    }
    store_num(S.acc, y, L, A.y_limb, A.y_hdr, A.y_ld, row);
    wsync();
  }
  if (st && ln == 0) atomicOr(A.status, st);
}

struct DotA {
  int64_t n, per_block;
  const uint32_t* x_limb;
  const int32_t* x_hdr;
  int64_t x_ld;
  const uint32_t* y_limb;
  const int32_t* y_hdr;
  int64_t y_ld;
  int L;
  int64_t* part;      // [blocks][kWinDigits] carry-save digits of each block's part
  int32_t* meta;      // [blocks][2]: anchor, digits (0: nothing; -1: too wide)
  uint32_t* out_limb;
  int32_t* out_hdr;
  int64_t out_ld;
  int nblocks;
  uint32_t* status;
};

// Each block's part of sum x_i y_i, exactly, as carry-save digits at its own anchor.
__global__ void __launch_bounds__(64) dot_parts(DotA A) {
  __shared__ Lds S;
  __shared__ int64_t win[kWinDigits];
  const int L = A.L, ln = lane_id();
  const int64_t i0 = (int64_t)blockIdx.x * A.per_block, i1 = min(A.n, i0 + A.per_block);
  int32_t lo = INT32_MAX, hi = INT32_MIN;
  for (int64_t i = i0 + ln; i < i1; i += 64) {
    const int32_t hx = A.x_hdr[i], hy = A.y_hdr[i];
    if (mp::hdr_is_zero(hx) || mp::hdr_is_zero(hy)) continue;
    const int32_t e = (hx >> 1) + (hy >> 1);
    lo = min(lo, e);
    hi = max(hi, e);
  }
  for (int o = 32; o > 0; o >>= 1) {
    lo = min(lo, __shfl_xor(lo, o, 64));
    hi = max(hi, __shfl_xor(hi, o, 64));
  }
  int32_t* meta = A.meta + 2 * blockIdx.x;
  if (hi < lo) {
    if (ln == 0) meta[1] = 0;
    return;
  }
  const int32_t anchor = lo & ~31;
  const int64_t W = (((int64_t)hi - anchor) >> 5) + 2 * L + 2;
  if (W > kWinDigits) {
    if (ln == 0) {
      meta[0] = anchor;
      meta[1] = -1;
    }
    return;
  }
  for (int j = ln; j < W; j += 64) win[j] = 0;
  wsync();
  for (int64_t i = i0; i < i1; ++i) {
    const int32_t hx = A.x_hdr[i], hy = A.y_hdr[i];
    if (mp::hdr_is_zero(hx) || mp::hdr_is_zero(hy)) continue;
    const WNum x = load_num(S.x, L, A.x_limb, A.x_hdr, A.x_ld, i);
    const WNum y = load_num(S.y, L, A.y_limb, A.y_hdr, A.y_ld, i);
    big_mul(S.p, S.x, L, S.y, L, S.c0, S.c1, S.c2);
    window_add(win, S.p, L, x.s ^ y.s, (int64_t)x.e + y.e - anchor);
  }
  int64_t* part = A.part + (int64_t)blockIdx.x * kWinDigits;
  for (int j = ln; j < W; j += 64) part[j] = win[j];
  if (ln == 0) {
    meta[0] = anchor;
    meta[1] = (int32_t)W;
  }
}

// The parts added at their anchors into one window, rounded once (one block).
__global__ void __launch_bounds__(64) dot_finish(DotA A) {
  __shared__ Lds S;
  __shared__ int64_t win[kWinDigits];
  __shared__ uint32_t ml[kWinDigits];
  const int L = A.L, ln = lane_id();
  uint32_t st = 0;
  int32_t lo = INT32_MAX;
  int64_t top = 0;
  bool wide = false, any = false;
  for (int b = 0; b < A.nblocks; ++b) {
    const int32_t w = A.meta[2 * b + 1];
    if (w < 0) wide = true;
    if (w > 0) {
      any = true;
      lo = min(lo, A.meta[2 * b]);
    }
  }
  WNum r{kZeroE, 0u};
  big_set(S.acc, L, 0u);
  wsync();
  if (wide) {
    st |= kStWindow;
  } else if (any) {
    for (int b = 0; b < A.nblocks; ++b) {
      const int32_t w = A.meta[2 * b + 1];
      if (w > 0) top = max(top, (((int64_t)A.meta[2 * b] - lo) >> 5) + w);
    }
    if (top > kWinDigits) {
      st |= kStWindow;
    } else {
      const int W = (int)top;
      for (int j = ln; j < W; j += 64) win[j] = 0;
      wsync();
      for (int b = 0; b < A.nblocks; ++b) {
        const int32_t w = A.meta[2 * b + 1];
        if (w <= 0) continue;
        const int64_t off = ((int64_t)A.meta[2 * b] - lo) >> 5;
        const int64_t* part = A.part + (int64_t)b * kWinDigits;
        for (int j = ln; j < w; j += 64) win[off + j] += part[j];
        wsync();
      }
      const uint32_t neg = window_normalize(ml, win, W);
      r = round_mag(S.acc, L, ml, W, (int64_t)lo - 64 * (int64_t)L, neg, false, st);
    }
  }
  store_num(S.acc, r, L, A.out_limb, A.out_hdr, A.out_ld, 0);
  if (st && ln == 0) atomicOr(A.status, st);
}

struct AxpyA {
  int kind;
  int64_t n;
  const uint32_t* a_limb;
  const int32_t* a_hdr;
  int64_t a_ld;
  const uint32_t* x_limb;
  const int32_t* x_hdr;
  int64_t x_ld;
  uint32_t* y_limb;
  int32_t* y_hdr;
  int64_t y_ld;
  int L;
  uint32_t* status;
};

// kind 0: y = y + RN(alpha x); 1: y = x + RN(alpha y); 2: y = y - RN(alpha x); 3: y = x - y
__global__ void __launch_bounds__(64) axpy(AxpyA A) {
  __shared__ Lds S;
  __shared__ uint32_t al[kMaxL + 4];
  const int L = A.L;
  uint32_t st = 0;
  const WNum alpha = A.kind == 3 ? WNum{kZeroE, 0u} : load_num(al, L, A.a_limb, A.a_hdr, A.a_ld, 0);
  for (int64_t i = blockIdx.x; i < A.n; i += gridDim.x) {
    const WNum x = load_num(S.x, L, A.x_limb, A.x_hdr, A.x_ld, i);
    const WNum y = load_num(S.y, L, A.y_limb, A.y_hdr, A.y_ld, i);
    WNum r;
    if (A.kind == 3) {
      WNum ny = y;
      ny.s ^= 1u;
      r = wide_add(S, S.acc, L, S.x, x, S.y, ny, st);
    } else {
      const bool on_y = A.kind == 1;
      WNum t = wide_mul(S, S.t, L, al, alpha, on_y ? S.y : S.x, on_y ? y : x, st);
      if (A.kind == 2) t.s ^= 1u;
      r = on_y ? wide_add(S, S.acc, L, S.x, x, S.t, t, st) : wide_add(S, S.acc, L, S.y, y, S.t, t, st);
    }
    store_num(S.acc, r, L, A.y_limb, A.y_hdr, A.y_ld, i);
    wsync();
  }
  if (st && lane_id() == 0) atomicOr(A.status, st);
}

enum ScalarOp { SC_DIV = 0, SC_MUL, SC_ADD, SC_SQRT, SC_ZERO, SC_CONV };

struct ScalarA {
  int op, L;
  int negb;  // SC_ADD: a - b
  const uint32_t* a_limb;
  const int32_t* a_hdr;
  int64_t a_ld;
  const uint32_t* b_limb;
  const int32_t* b_hdr;
  int64_t b_ld;
  uint32_t* o_limb;
  int32_t* o_hdr;
  int64_t o_ld;
  int32_t* flag;  // SC_ZERO: a == 0; SC_CONV: RN(sqrt a) <= b
  uint32_t* status;
};

__global__ void __launch_bounds__(64) scalar(ScalarA A) {
  __shared__ Lds S;
  __shared__ uint32_t r[kMaxL + 4];
  const int L = A.L;
  uint32_t st = 0;
  const WNum a = load_num(S.x, L, A.a_limb, A.a_hdr, A.a_ld, 0);
  const WNum b = (A.op == SC_SQRT || A.op == SC_ZERO) ? WNum{kZeroE, 0u}
                                                       : load_num(S.y, L, A.b_limb, A.b_hdr, A.b_ld, 0);
  WNum o{kZeroE, 0u};
  switch (A.op) {
    case SC_DIV: o = wide_div(S, r, L, S.x, a, S.y, b, st); break;
    case SC_MUL: o = wide_mul(S, r, L, S.x, a, S.y, b, st); break;
    case SC_ADD: {
      WNum bb = b;
      if (A.negb) bb.s ^= 1u;
      o = wide_add(S, r, L, S.x, a, S.y, bb, st);
      break;
    }
    case SC_SQRT: o = wide_sqrt(S, r, L, S.x, a, st); break;
    case SC_ZERO:
      if (lane_id() == 0) *A.flag = a.e == kZeroE ? 1 : 0;
      break;
    default: {
      const bool c = wide_sqrt_le(S, L, S.x, a, S.y, b);
      if (lane_id() == 0) *A.flag = c ? 1 : 0;
      break;
    }
  }
  if (A.op <= SC_SQRT) store_num(r, o, L, A.o_limb, A.o_hdr, A.o_ld, 0);
  if (st && lane_id() == 0) atomicOr(A.status, st);
}

// Element programs: per element, a few RN multiplications, additions and subtractions on
// registers loaded from vectors and scalars, in the order the program lists them (one RN per
// operation), the chosen registers stored back.  Operands 0..7 are element registers, 8..11
// scalars.
constexpr int kProgRegs = 8, kProgScalars = 4, kProgIns = 16, kProgIn = 7, kProgOut = 3;
enum ProgOp { PO_MUL = 0, PO_ADD, PO_SUB };

struct VRef {
  const uint32_t* limb;
  const int32_t* hdr;
  int64_t ld;
};

struct ProgA {
  int64_t n;
  int L;
  int n_in, n_sc, n_ins, n_out;
  VRef in[kProgIn];
  int in_reg[kProgIn];
  VRef sc[kProgScalars];
  int8_t op[kProgIns], dst[kProgIns], a[kProgIns], b[kProgIns];
  VRef out[kProgOut];
  int out_reg[kProgOut];
  uint32_t* status;
};

__global__ void __launch_bounds__(64) prog(ProgA P) {
  __shared__ Lds S;
  __shared__ uint32_t reg[kProgRegs + kProgScalars][kMaxL + 4];
  const int L = P.L;
  uint32_t st = 0;
  WNum w[kProgRegs + kProgScalars];
  for (int k = 0; k < P.n_sc; ++k)
    w[kProgRegs + k] = load_num(reg[kProgRegs + k], L, P.sc[k].limb, P.sc[k].hdr, P.sc[k].ld, 0);
  for (int64_t i = blockIdx.x; i < P.n; i += gridDim.x) {
    for (int k = 0; k < P.n_in; ++k)
      w[P.in_reg[k]] = load_num(reg[P.in_reg[k]], L, P.in[k].limb, P.in[k].hdr, P.in[k].ld, i);
    for (int t = 0; t < P.n_ins; ++t) {
      const int a = P.a[t], b = P.b[t], d = P.dst[t];
      WNum r;
      if (P.op[t] == PO_MUL) {
        r = wide_mul(S, S.acc, L, reg[a], w[a], reg[b], w[b], st);
      } else {
        WNum wb = w[b];
        if (P.op[t] == PO_SUB) wb.s ^= 1u;
        r = wide_add(S, S.acc, L, reg[a], w[a], reg[b], wb, st);
      }
      big_copy(reg[d], S.acc, L);
      wsync();
      w[d] = r;
    }
    for (int k = 0; k < P.n_out; ++k) {
      const int rr = P.out_reg[k];
      uint32_t* ol = const_cast<uint32_t*>(P.out[k].limb);
      int32_t* oh = const_cast<int32_t*>(P.out[k].hdr);
      store_num(reg[rr], w[rr], L, ol, oh, P.out[k].ld, i);
    }
    wsync();
  }
  if (st && lane_id() == 0) atomicOr(P.status, st);
}

// dst[k] = src[perm[k]] for every limb plane and the header
__global__ void __launch_bounds__(256) gather(const int32_t* perm, int64_t nnz, int L, const uint32_t* s_limb,
                                              const int32_t* s_hdr, int64_t s_ld, uint32_t* d_limb, int32_t* d_hdr) {
  const int64_t tot = nnz * (L + 1);
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < tot; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t k = t % nnz, q = t / nnz;
    const int64_t src = perm[k];
    if (q < L) d_limb[q * nnz + k] = s_limb[q * s_ld + src];
    else d_hdr[k] = s_hdr[src];
  }
}

// a plain copy of n elements (limbs and headers)
__global__ void __launch_bounds__(256) copy(int64_t n, int L, const uint32_t* s_limb, const int32_t* s_hdr, int64_t s_ld,
                                            uint32_t* d_limb, int32_t* d_hdr, int64_t d_ld) {
  const int64_t tot = n * (L + 1);
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < tot; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = t % n, q = t / n;
    if (q < L) d_limb[q * d_ld + i] = s_limb[q * s_ld + i];
    else d_hdr[i] = s_hdr[i];
  }
}

// +0 into n elements
__global__ void __launch_bounds__(256) zero(int64_t n, int L, uint32_t* d_limb, int32_t* d_hdr, int64_t d_ld) {
  const int64_t tot = n * (L + 1);
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < tot; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = t % n, q = t / n;
    if (q < L) d_limb[q * d_ld + i] = 0u;
    else d_hdr[i] = (int32_t)0x80000000u;
  }
}

}  // namespace wide_k

// ---- host side ----------------------------------------------------------------------------
namespace mpapi {

namespace {

unsigned grid_of(int64_t n, int64_t cap) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>(n, cap)); }

int launched(const char* what) {
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? MPS_OK : hip_fail(e, what);
}

// the dot's per-block parts (one allocation per device, kept until the process ends)
struct DotWs {
  int64_t* part = nullptr;
  int32_t* meta = nullptr;
};
constexpr int kDotBlocks = 256;  // partial windows of an inner product (its parallelism)
std::vector<DotWs> g_dot_ws;
std::mutex g_dot_mu;

int dot_ws(DotWs** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  std::lock_guard<std::mutex> lk(g_dot_mu);
  if ((int)g_dot_ws.size() <= dev) g_dot_ws.resize(dev + 1);
  DotWs& w = g_dot_ws[dev];
  if (!w.part) {
    e = hipMalloc((void**)&w.part, sizeof(int64_t) * (size_t)kDotBlocks * kWinDigits);
    if (e == hipSuccess) e = hipMalloc((void**)&w.meta, sizeof(int32_t) * 2 * kDotBlocks);
    if (e != hipSuccess) return fail(MPS_ENOMEM, "wide inner-product workspace: %s", hipGetErrorString(e));
  }
  *out = &w;
  return MPS_OK;
}

mp_vec elem(const mp_vec& v, int64_t i) {
  mp_vec r = v;
  r.limb = v.limb + i;
  r.hdr = v.hdr + i;
  r.len = 1;
  return r;
}

}  // namespace

int wide_limbs_of(int prec) {
  switch (prec) {
    case 2048: return 64;
    case 4096: return 128;
    case 8192: return 256;
    default: return 0;
  }
}

int wide_spmv(int L, int64_t n_rows, const int32_t* row_ptr, const int32_t* col_idx, const mp_vec& val,
              const mp_vec& x, const mp_vec& y, int mode, uint32_t* status, hipStream_t s) {
  if (n_rows == 0) return MPS_OK;
  wide_k::SpmvA a{n_rows, row_ptr, col_idx, val.limb, val.hdr, val.ld, x.limb, x.hdr, x.ld,
                  y.limb, y.hdr, y.ld, L, status};
  const unsigned g = grid_of(n_rows, 8192);
  if (mode == MP_SEQ)
    hipLaunchKernelGGL(wide_k::spmv_seq, dim3(g), dim3(64), 0, s, a);
  else
    hipLaunchKernelGGL(wide_k::spmv_exact, dim3(g), dim3(64), 0, s, a);
  return launched("wide sparse product");
}

int wide_dot(int L, const mp_vec& x, const mp_vec& y, const mp_vec& out, uint32_t* status, hipStream_t s) {
  DotWs* w;
  int r = dot_ws(&w);
  if (r) return r;
  const int64_t n = x.len;
  // a block forms its elements' products one after another: as many blocks as the parts allow
  const int nb = (int)std::max<int64_t>(1, std::min<int64_t>(kDotBlocks, n));
  const int64_t per = std::max<int64_t>(1, (n + nb - 1) / nb);
  wide_k::DotA a{n, per, x.limb, x.hdr, x.ld, y.limb, y.hdr, y.ld, L, w->part, w->meta,
                 out.limb, out.hdr, out.ld, nb, status};
  hipLaunchKernelGGL(wide_k::dot_parts, dim3(nb), dim3(64), 0, s, a);
  hipLaunchKernelGGL(wide_k::dot_finish, dim3(1), dim3(64), 0, s, a);
  return launched("wide inner product");
}

int wide_axpy(int L, int kind, const mp_vec& alpha, const mp_vec& x, const mp_vec& y, int64_t n,
              uint32_t* status, hipStream_t s) {
  if (n == 0) return MPS_OK;
  wide_k::AxpyA a{kind, n, alpha.limb, alpha.hdr, alpha.ld, x.limb, x.hdr, x.ld, y.limb, y.hdr, y.ld, L, status};
  hipLaunchKernelGGL(wide_k::axpy, dim3(grid_of(n, 8192)), dim3(64), 0, s, a);
  return launched("wide vector update");
}

int wide_gather(int L, const int32_t* perm, int64_t nnz, const mp_vec& src, uint32_t* dst_limb,
                int32_t* dst_hdr, hipStream_t s) {
  if (nnz == 0) return MPS_OK;
  const int64_t tot = nnz * (L + 1);
  hipLaunchKernelGGL(wide_k::gather, dim3(grid_of((tot + 255) / 256, 65536)), dim3(256), 0, s, perm, nnz, L,
                     src.limb, src.hdr, src.ld, dst_limb, dst_hdr);
  return launched("wide gather");
}

namespace {

int wcopy(int L, const mp_vec& src, const mp_vec& dst, int64_t n, hipStream_t s) {
  if (n == 0) return MPS_OK;
  const int64_t tot = n * (L + 1);
  hipLaunchKernelGGL(wide_k::copy, dim3(grid_of((tot + 255) / 256, 65536)), dim3(256), 0, s, n, L, src.limb, src.hdr,
                     src.ld, dst.limb, dst.hdr, dst.ld);
  return launched("wide copy");
}

int wzero(int L, const mp_vec& dst, int64_t n, hipStream_t s) {
  if (n == 0) return MPS_OK;
  const int64_t tot = n * (L + 1);
  hipLaunchKernelGGL(wide_k::zero, dim3(grid_of((tot + 255) / 256, 65536)), dim3(256), 0, s, n, L, dst.limb,
                     dst.hdr, dst.ld);
  return launched("wide zero");
}

int wscalar(int L, int op, const mp_vec& a, const mp_vec* b, const mp_vec* o, int32_t* flag, uint32_t* status,
            hipStream_t s, bool negb = false) {
  wide_k::ScalarA k{op, L, negb ? 1 : 0, a.limb, a.hdr, a.ld, b ? b->limb : nullptr, b ? b->hdr : nullptr,
                    b ? b->ld : 0, o ? o->limb : nullptr, o ? o->hdr : nullptr, o ? o->ld : 0, flag, status};
  hipLaunchKernelGGL(wide_k::scalar, dim3(1), dim3(64), 0, s, k);
  return launched("wide scalar operation");
}

// device buffers of a wide solve, freed on scope exit
struct WideBufs {
  std::vector<void*> ptrs;
  ~WideBufs() {
    for (void* p : ptrs) (void)hipFree(p);
  }
  int vec(int L, int64_t n, mp_vec* v) {
    uint32_t* l = nullptr;
    int32_t* h = nullptr;
    hipError_t e = hipMalloc((void**)&l, sizeof(uint32_t) * (size_t)L * std::max<int64_t>(1, n));
    if (e == hipSuccess) ptrs.push_back(l);
    if (e == hipSuccess) e = hipMalloc((void**)&h, sizeof(int32_t) * std::max<int64_t>(1, n));
    if (e == hipSuccess) ptrs.push_back(h);
    if (e != hipSuccess) return fail(MPS_ENOMEM, "wide solve buffers: %s", hipGetErrorString(e));
    *v = mp_vec{l, h, n, std::max<int64_t>(1, n)};
    return MPS_OK;
  }
};

}  // namespace

namespace {

// A host-driven wide solve: its vectors, scalar slots and the flag the host reads.
struct WSolve {
  int L;
  int64_t n;
  int mode;
  uint32_t* status;
  hipStream_t s;
  WideBufs B;
  mp_vec sc{};
  int32_t* dflag = nullptr;
  static constexpr int kSlots = 32;

  int init(int L_, int64_t n_, int mode_, uint32_t* st_, hipStream_t s_) {
    L = L_;
    n = n_;
    mode = mode_;
    status = st_;
    s = s_;
    int r = B.vec(L, kSlots, &sc);
    if (r) return r;
    hipError_t e = hipMalloc((void**)&dflag, sizeof(int32_t));
    if (e != hipSuccess) return fail(MPS_ENOMEM, "wide solve flag: %s", hipGetErrorString(e));
    B.ptrs.push_back(dflag);
    return MPS_OK;
  }
  mp_vec S(int k) const { return elem(sc, k); }
  int vec(mp_vec* v) { return B.vec(L, n, v); }
  int read_flag(bool* f) {
    int32_t h = 0;
    hipError_t e = hipMemcpyAsync(&h, dflag, 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "wide solve flag");
    *f = h != 0;
    return MPS_OK;
  }
  int is_zero(int k, bool* z) {
    int r = wscalar(L, wide_k::SC_ZERO, S(k), nullptr, nullptr, dflag, status, s);
    return r ? r : read_flag(z);
  }
  int conv(int q, int thr, bool* c) {
    const mp_vec t = S(thr);
    int r = wscalar(L, wide_k::SC_CONV, S(q), &t, nullptr, dflag, status, s);
    return r ? r : read_flag(c);
  }
  // slot o = a (op) b
  int scal(int op, int a, int b, int o, bool negb = false) {
    const mp_vec bv = S(b), ov = S(o);
    return wscalar(L, op, S(a), &bv, &ov, nullptr, status, s, negb);
  }
  int copy_slot(int from, int to) { return wcopy(L, S(from), S(to), 1, s); }
  int dot(const mp_vec& x, const mp_vec& y, int o) { return wide_dot(L, x, y, S(o), status, s); }
  int spmv(const WideOp& A, const mp_vec& in, const mp_vec& out) {
    return wide_spmv(L, A.n_out, A.row_ptr, A.col_idx, A.val, in, out, mode, status, s);
  }
  int set_const(int k, int64_t m, int64_t e10) {
    std::vector<uint32_t> l(L);
    int32_t h;
    if (!decimal_to_mp(m, e10, L, l.data(), &h)) return fail(MPS_EINVAL, "tolerance out of range");
    const mp_vec c = S(k);
    hipError_t e = hipSuccess;
    for (int q = 0; q < L && e == hipSuccess; ++q)
      e = hipMemcpyAsync(c.limb + (int64_t)q * c.ld, &l[q], 4, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(c.hdr, &h, 4, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return e == hipSuccess ? MPS_OK : hip_fail(e, "constant upload");
  }
};

// An element program under construction: inputs (vector -> register), scalars (slot ->
// operand 8 + k), instructions, outputs (register -> vector).
struct Prog {
  wide_k::ProgA a{};
  const WSolve* w;
  explicit Prog(const WSolve& ws) : w(&ws) {
    a.n = ws.n;
    a.L = ws.L;
    a.status = ws.status;
  }
  static wide_k::VRef ref(const mp_vec& v) { return wide_k::VRef{v.limb, v.hdr, v.ld}; }
  bool bad = false;  // a program beyond the kernel's table sizes (a bug here, reported by run)
  static bool reg_ok(int r) { return r >= 0 && r < wide_k::kProgRegs; }
  Prog& in(const mp_vec& v, int reg) {
    if (a.n_in >= wide_k::kProgIn || !reg_ok(reg)) return bad = true, *this;
    a.in[a.n_in] = ref(v);
    a.in_reg[a.n_in++] = reg;
    return *this;
  }
  int scalar(int slot) {  // operand index of a scalar slot
    if (a.n_sc >= wide_k::kProgScalars) return bad = true, 0;
    a.sc[a.n_sc] = ref(w->S(slot));
    return wide_k::kProgRegs + a.n_sc++;
  }
  Prog& op(int o, int d, int x, int y) {
    const int lim = wide_k::kProgRegs + wide_k::kProgScalars;
    if (a.n_ins >= wide_k::kProgIns || !reg_ok(d) || x < 0 || x >= lim || y < 0 || y >= lim)
      return bad = true, *this;
    a.op[a.n_ins] = (int8_t)o;
    a.dst[a.n_ins] = (int8_t)d;
    a.a[a.n_ins] = (int8_t)x;
    a.b[a.n_ins++] = (int8_t)y;
    return *this;
  }
  Prog& out(int reg, const mp_vec& v) {
    if (a.n_out >= wide_k::kProgOut || !reg_ok(reg)) return bad = true, *this;
    a.out[a.n_out] = ref(v);
    a.out_reg[a.n_out++] = reg;
    return *this;
  }
  int run() {
    if (bad) return fail(MPS_EINVAL, "wide element program exceeds its tables");
    if (a.n == 0) return MPS_OK;
    hipLaunchKernelGGL(wide_k::prog, dim3(grid_of(a.n, 8192)), dim3(64), 0, w->s, a);
    return launched("wide element program");
  }
};

enum { W_RHO, W_RHO_OLD, W_ALPHA, W_ALPHA_OLD, W_BETA, W_SIGMA, W_Q, W_Q0, W_NRM0, W_THR, W_CREL, W_CABS,
       W_T1, W_T2, W_T3, W_T4, W_ZETA, W_ZETA_OLD, W_ETA, W_MU1, W_MU2, W_MU3, W_MU4, W_MU5, W_TAU,
       W_OMEGA, W_OMEGA_OLD, W_TS, W_TT };

// The shared start of the methods: r = b - A x0 (or r = b, x = +0), r~ = r, q0 = (r, r),
// thr = RN(RN(c_rel RN(sqrt q0)) + c_abs); *done when r_0 already passes the test.
int wide_setup(WSolve& W, const WideOp& op, const mp_vec* b, mp_vec* x, const mp_solve_opts* o,
               const mp_vec& r, const mp_vec& rt, mp_solve_info* info, bool* done) {
  int rr;
  if ((rr = W.set_const(W_CREL, o->rtol_m, o->rtol_e10)) || (rr = W.set_const(W_CABS, o->atol_m, o->atol_e10)))
    return rr;
  if (o->use_x0) {
    if ((rr = W.spmv(op, *x, r))) return rr;
    if ((rr = wide_axpy(W.L, 3, W.S(W_T1), *b, r, W.n, W.status, W.s))) return rr;  // r = b - A x0
  } else {
    if ((rr = wzero(W.L, *x, W.n, W.s)) || (rr = wcopy(W.L, *b, r, W.n, W.s))) return rr;
  }
  if ((rr = wcopy(W.L, r, rt, W.n, W.s))) return rr;
  if ((rr = W.dot(r, r, W_Q0))) return rr;
  const mp_vec q0 = W.S(W_Q0), nrm0 = W.S(W_NRM0);
  if ((rr = wscalar(W.L, wide_k::SC_SQRT, q0, nullptr, &nrm0, nullptr, W.status, W.s))) return rr;
  if ((rr = W.scal(wide_k::SC_MUL, W_CREL, W_NRM0, W_T1)) || (rr = W.scal(wide_k::SC_ADD, W_T1, W_CABS, W_THR)))
    return rr;
  info->iters = 0;
  info->status = MP_NC;
  bool c = false;
  if ((rr = W.conv(W_Q0, W_THR, &c))) return rr;
  if (c) info->status = MP_CONVERGED;
  *done = c || o->maxit <= 0;
  return MPS_OK;
}

// the residual history entry of iteration i, the stopping test; *stop when converged
int wide_after(WSolve& W, const mp_solve_opts* o, int64_t i, mp_solve_info* info, bool* stop) {
  int rr;
  if (o->res_hist && o->res_hist->len > 0 && i - 1 < o->res_hist->len &&
      (rr = wcopy(W.L, W.S(W_Q), elem(*o->res_hist, i - 1), 1, W.s)))
    return rr;
  bool c = false;
  if ((rr = W.conv(W_Q, W_THR, &c))) return rr;
  info->iters = i;
  if (c) info->status = MP_CONVERGED;
  *stop = c;
  return MPS_OK;
}

int final_res(WSolve& W, mp_solve_info* info) {
  const int L = W.L;
  uint32_t qt = 0, q0t = 0;
  int32_t qh = 0, q0h = 0;
  const mp_vec qv = W.S(info->iters > 0 ? W_Q : W_Q0), q0v = W.S(W_Q0);
  hipError_t e = hipMemcpyAsync(&qh, qv.hdr, 4, hipMemcpyDeviceToHost, W.s);
  if (e == hipSuccess) e = hipMemcpyAsync(&q0h, q0v.hdr, 4, hipMemcpyDeviceToHost, W.s);
  if (e == hipSuccess) e = hipMemcpyAsync(&qt, qv.limb + (int64_t)(L - 1) * qv.ld, 4, hipMemcpyDeviceToHost, W.s);
  if (e == hipSuccess) e = hipMemcpyAsync(&q0t, q0v.limb + (int64_t)(L - 1) * q0v.ld, 4, hipMemcpyDeviceToHost, W.s);
  if (e == hipSuccess) e = hipStreamSynchronize(W.s);
  if (e != hipSuccess) return hip_fail(e, "wide solve readback");
  auto approx = [](uint32_t top, int32_t hd) {
    const int32_t ex = hd >> 1;
    if (ex == kZeroE) return 0.0;
    return std::ldexp((double)top, std::max(-1070, std::min(1020, ex - 32)));
  };
  const double a0 = approx(q0t, q0h), a1 = approx(qt, qh);
  info->final_rel_res = a0 > 0 ? std::sqrt(a1 / a0) : 0.0;
  return MPS_OK;
}

}  // namespace

// CGS (the same operations as the fixed-width cgs and the oracle's)
int wide_cgs(int L, const WideOp& op, const mp_vec* b, mp_vec* x, const mp_solve_opts* o, mp_solve_info* info,
             uint32_t* status, hipStream_t s) {
  WSolve W;
  int rr;
  mp_vec r, rt, u, p, q, vh, uh, qh;
  if ((rr = W.init(L, op.n_out, o->mode, status, s)) || (rr = W.vec(&r)) || (rr = W.vec(&rt)) ||
      (rr = W.vec(&u)) || (rr = W.vec(&p)) || (rr = W.vec(&q)) || (rr = W.vec(&vh)) || (rr = W.vec(&uh)) ||
      (rr = W.vec(&qh)))
    return rr;
  bool done = false;
  if ((rr = wide_setup(W, op, b, x, o, r, rt, info, &done))) return rr;
  for (int64_t i = 1; !done && i <= o->maxit; ++i) {
    bool z = false;
    if ((rr = W.dot(rt, r, W_RHO)) || (rr = W.is_zero(W_RHO, &z))) return rr;
    if (z) {
      info->status = MP_BREAKDOWN_RHO;
      info->iters = i - 1;
      break;
    }
    if (i == 1) {
      if ((rr = wcopy(L, r, u, W.n, s)) || (rr = wcopy(L, r, p, W.n, s))) return rr;
    } else {
      if ((rr = W.scal(wide_k::SC_DIV, W_RHO, W_RHO_OLD, W_BETA))) return rr;
      // u = r + beta q;  p = u + beta (q + beta p)
      Prog P(W);
      const int be = P.scalar(W_BETA);
      P.in(r, 0).in(q, 1).in(p, 2);
      P.op(wide_k::PO_MUL, 3, be, 1).op(wide_k::PO_ADD, 4, 0, 3);   // u
      P.op(wide_k::PO_MUL, 5, be, 2).op(wide_k::PO_ADD, 5, 1, 5).op(wide_k::PO_MUL, 5, be, 5)
          .op(wide_k::PO_ADD, 6, 4, 5);                              // p
      P.out(4, u).out(6, p);
      if ((rr = P.run())) return rr;
    }
    if ((rr = W.spmv(op, p, vh)) || (rr = W.dot(rt, vh, W_SIGMA)) || (rr = W.is_zero(W_SIGMA, &z))) return rr;
    if (z) {
      info->status = MP_BREAKDOWN_SIGMA;
      info->iters = i - 1;
      break;
    }
    if ((rr = W.scal(wide_k::SC_DIV, W_RHO, W_SIGMA, W_ALPHA))) return rr;
    {
      // q = u - alpha vh;  uh = u + q;  x = x + alpha uh
      Prog P(W);
      const int al = P.scalar(W_ALPHA);
      P.in(u, 0).in(vh, 1).in(*x, 2);
      P.op(wide_k::PO_MUL, 3, al, 1).op(wide_k::PO_SUB, 3, 0, 3)   // q
          .op(wide_k::PO_ADD, 4, 0, 3)                              // uh
          .op(wide_k::PO_MUL, 5, al, 4).op(wide_k::PO_ADD, 5, 2, 5);  // x
      P.out(3, q).out(4, uh).out(5, *x);
      if ((rr = P.run())) return rr;
    }
    if ((rr = W.spmv(op, uh, qh))) return rr;
    if ((rr = wide_axpy(L, 2, W.S(W_ALPHA), qh, r, W.n, status, s))) return rr;  // r = r - alpha qh
    if ((rr = W.dot(r, r, W_Q))) return rr;
    bool stop = false;
    if ((rr = wide_after(W, o, i, info, &stop))) return rr;
    if (stop) break;
    if ((rr = W.copy_slot(W_RHO, W_RHO_OLD))) return rr;
  }
  return final_res(W, info);
}

// BiCGSTAB
int wide_bicgstab(int L, const WideOp& op, const mp_vec* b, mp_vec* x, const mp_solve_opts* o,
                  mp_solve_info* info, uint32_t* status, hipStream_t s) {
  WSolve W;
  int rr;
  mp_vec r, rt, p, v, sv, t;
  if ((rr = W.init(L, op.n_out, o->mode, status, s)) || (rr = W.vec(&r)) || (rr = W.vec(&rt)) ||
      (rr = W.vec(&p)) || (rr = W.vec(&v)) || (rr = W.vec(&sv)) || (rr = W.vec(&t)))
    return rr;
  bool done = false;
  if ((rr = wide_setup(W, op, b, x, o, r, rt, info, &done))) return rr;
  for (int64_t i = 1; !done && i <= o->maxit; ++i) {
    bool z = false;
    if ((rr = W.dot(rt, r, W_RHO)) || (rr = W.is_zero(W_RHO, &z))) return rr;
    if (z) {
      info->status = MP_BREAKDOWN_RHO;
      info->iters = i - 1;
      break;
    }
    if (i == 1) {
      if ((rr = wcopy(L, r, p, W.n, s))) return rr;
    } else {
      // beta = (rho / rho_old)(alpha_old / omega_old); p = r + beta (p - omega_old v)
      if ((rr = W.scal(wide_k::SC_DIV, W_RHO, W_RHO_OLD, W_T1)) ||
          (rr = W.scal(wide_k::SC_DIV, W_ALPHA_OLD, W_OMEGA_OLD, W_T2)) ||
          (rr = W.scal(wide_k::SC_MUL, W_T1, W_T2, W_BETA)))
        return rr;
      Prog P(W);
      const int be = P.scalar(W_BETA), om = P.scalar(W_OMEGA_OLD);
      P.in(r, 0).in(p, 1).in(v, 2);
      P.op(wide_k::PO_MUL, 3, om, 2).op(wide_k::PO_SUB, 3, 1, 3).op(wide_k::PO_MUL, 3, be, 3)
          .op(wide_k::PO_ADD, 4, 0, 3);
      P.out(4, p);
      if ((rr = P.run())) return rr;
    }
    if ((rr = W.spmv(op, p, v)) || (rr = W.dot(rt, v, W_SIGMA)) || (rr = W.is_zero(W_SIGMA, &z))) return rr;
    if (z) {
      info->status = MP_BREAKDOWN_SIGMA;
      info->iters = i - 1;
      break;
    }
    if ((rr = W.scal(wide_k::SC_DIV, W_RHO, W_SIGMA, W_ALPHA))) return rr;
    {
      Prog P(W);  // s = r - alpha v
      const int al = P.scalar(W_ALPHA);
      P.in(r, 0).in(v, 1).op(wide_k::PO_MUL, 2, al, 1).op(wide_k::PO_SUB, 2, 0, 2).out(2, sv);
      if ((rr = P.run())) return rr;
    }
    if ((rr = W.spmv(op, sv, t)) || (rr = W.dot(t, sv, W_TS)) || (rr = W.dot(t, t, W_TT))) return rr;
    bool ttz = false;
    if ((rr = W.is_zero(W_TT, &ttz))) return rr;
    if (ttz) {
      if ((rr = wzero(L, W.S(W_OMEGA), 1, s))) return rr;
    } else if ((rr = W.scal(wide_k::SC_DIV, W_TS, W_TT, W_OMEGA))) {
      return rr;
    }
    {
      // x = (x + alpha p) + omega s;  r = s - omega t
      Prog P(W);
      const int al = P.scalar(W_ALPHA), om = P.scalar(W_OMEGA);
      P.in(*x, 0).in(p, 1).in(sv, 2).in(t, 3);
      P.op(wide_k::PO_MUL, 4, al, 1).op(wide_k::PO_ADD, 4, 0, 4).op(wide_k::PO_MUL, 5, om, 2)
          .op(wide_k::PO_ADD, 4, 4, 5)                              // x
          .op(wide_k::PO_MUL, 6, om, 3).op(wide_k::PO_SUB, 6, 2, 6);  // r
      P.out(4, *x).out(6, r);
      if ((rr = P.run())) return rr;
    }
    if ((rr = W.dot(r, r, W_Q))) return rr;
    bool stop = false;
    if ((rr = wide_after(W, o, i, info, &stop))) return rr;
    if (stop) break;
    bool oz = false;
    if ((rr = W.is_zero(W_OMEGA, &oz))) return rr;
    if (oz) {
      info->status = MP_BREAKDOWN_ZETA;
      break;
    }
    if ((rr = W.copy_slot(W_RHO, W_RHO_OLD)) || (rr = W.copy_slot(W_ALPHA, W_ALPHA_OLD)) ||
        (rr = W.copy_slot(W_OMEGA, W_OMEGA_OLD)))
      return rr;
  }
  return final_res(W, info);
}

// GPBiCG (Fig. 5 right, the readings of the fixed-width gpbicg)
int wide_gpbicg(int L, const WideOp& op, const mp_vec* b, mp_vec* x, const mp_solve_opts* o,
                mp_solve_info* info, uint32_t* status, hipStream_t s) {
  WSolve W;
  int rr;
  mp_vec r, rt, u, z, sv, w, t, p, q, v, y;
  if ((rr = W.init(L, op.n_out, o->mode, status, s)) || (rr = W.vec(&r)) || (rr = W.vec(&rt)) ||
      (rr = W.vec(&u)) || (rr = W.vec(&z)) || (rr = W.vec(&sv)) || (rr = W.vec(&w)) || (rr = W.vec(&t)) ||
      (rr = W.vec(&p)) || (rr = W.vec(&q)) || (rr = W.vec(&v)) || (rr = W.vec(&y)))
    return rr;
  bool done = false;
  if ((rr = wide_setup(W, op, b, x, o, r, rt, info, &done))) return rr;
  for (const mp_vec* vv : {&u, &z, &sv, &w, &t, &p, &q, &v})
    if ((rr = wzero(L, *vv, W.n, s))) return rr;
  if ((rr = wzero(L, W.S(W_BETA), 1, s))) return rr;
  for (int64_t i = 1; !done && i <= o->maxit; ++i) {
    bool zf = false;
    if ((rr = W.dot(rt, r, W_RHO)) || (rr = W.is_zero(W_RHO, &zf))) return rr;
    if (zf) {
      info->status = MP_BREAKDOWN_RHO;
      info->iters = i - 1;
      break;
    }
    if (i == 1) {
      if ((rr = wcopy(L, r, p, W.n, s))) return rr;
    } else {
      // beta = (rho / rho_old)(alpha_old / zeta_old); w = v + beta q; p = r + beta (p - u)
      if ((rr = W.scal(wide_k::SC_DIV, W_RHO, W_RHO_OLD, W_T1)) ||
          (rr = W.scal(wide_k::SC_DIV, W_ALPHA_OLD, W_ZETA_OLD, W_T2)) ||
          (rr = W.scal(wide_k::SC_MUL, W_T1, W_T2, W_BETA)))
        return rr;
      Prog P(W);
      const int be = P.scalar(W_BETA);
      P.in(v, 0).in(q, 1).in(r, 2).in(p, 3).in(u, 4);
      P.op(wide_k::PO_MUL, 5, be, 1).op(wide_k::PO_ADD, 5, 0, 5)                              // w
          .op(wide_k::PO_SUB, 6, 3, 4).op(wide_k::PO_MUL, 6, be, 6).op(wide_k::PO_ADD, 6, 2, 6);  // p
      P.out(5, w).out(6, p);
      if ((rr = P.run())) return rr;
    }
    if ((rr = W.spmv(op, p, q)) || (rr = W.dot(rt, q, W_SIGMA)) || (rr = W.is_zero(W_SIGMA, &zf))) return rr;
    if (zf) {
      info->status = MP_BREAKDOWN_SIGMA;
      info->iters = i - 1;
      break;
    }
    if ((rr = W.scal(wide_k::SC_DIV, W_RHO, W_SIGMA, W_ALPHA))) return rr;
    {
      // s = t - r (after the first iteration); t = r - alpha q
      Prog P(W);
      const int al = P.scalar(W_ALPHA);
      P.in(t, 0).in(r, 1).in(q, 2);
      if (i > 1) P.op(wide_k::PO_SUB, 3, 0, 1).out(3, sv);
      P.op(wide_k::PO_MUL, 4, al, 2).op(wide_k::PO_SUB, 4, 1, 4).out(4, t);
      if ((rr = P.run())) return rr;
    }
    if ((rr = W.spmv(op, t, v))) return rr;
    if (i == 1) {
      Prog P(W);  // y = alpha q - r
      const int al = P.scalar(W_ALPHA);
      P.in(q, 0).in(r, 1).op(wide_k::PO_MUL, 2, al, 0).op(wide_k::PO_SUB, 2, 2, 1).out(2, y);
      if ((rr = P.run())) return rr;
      if ((rr = W.dot(v, t, W_MU2)) || (rr = W.dot(v, v, W_MU5)) || (rr = W.is_zero(W_MU5, &zf))) return rr;
      if (zf) {
        info->status = MP_BREAKDOWN_TAU;
        info->iters = i - 1;
        break;
      }
      if ((rr = W.scal(wide_k::SC_DIV, W_MU2, W_MU5, W_ZETA)) || (rr = wzero(L, W.S(W_ETA), 1, s))) return rr;
    } else {
      Prog P(W);  // y = s - alpha (w - q)
      const int al = P.scalar(W_ALPHA);
      P.in(sv, 0).in(w, 1).in(q, 2);
      P.op(wide_k::PO_SUB, 3, 1, 2).op(wide_k::PO_MUL, 3, al, 3).op(wide_k::PO_SUB, 3, 0, 3).out(3, y);
      if ((rr = P.run())) return rr;
      if ((rr = W.dot(y, y, W_MU1)) || (rr = W.dot(v, t, W_MU2)) || (rr = W.dot(y, t, W_MU3)) ||
          (rr = W.dot(v, y, W_MU4)) || (rr = W.dot(v, v, W_MU5)))
        return rr;
      // tau = mu5 mu1 - mu4 mu4; zeta = (mu1 mu2 - mu3 mu4) / tau; eta = (mu5 mu3 - mu4 mu2) / tau
      if ((rr = W.scal(wide_k::SC_MUL, W_MU5, W_MU1, W_T1)) || (rr = W.scal(wide_k::SC_MUL, W_MU4, W_MU4, W_T2)) ||
          (rr = W.scal(wide_k::SC_ADD, W_T1, W_T2, W_TAU, true)) || (rr = W.is_zero(W_TAU, &zf)))
        return rr;
      if (zf) {
        info->status = MP_BREAKDOWN_TAU;
        info->iters = i - 1;
        break;
      }
      if ((rr = W.scal(wide_k::SC_MUL, W_MU1, W_MU2, W_T1)) || (rr = W.scal(wide_k::SC_MUL, W_MU3, W_MU4, W_T2)) ||
          (rr = W.scal(wide_k::SC_ADD, W_T1, W_T2, W_T3, true)) || (rr = W.scal(wide_k::SC_DIV, W_T3, W_TAU, W_ZETA)) ||
          (rr = W.scal(wide_k::SC_MUL, W_MU5, W_MU3, W_T1)) || (rr = W.scal(wide_k::SC_MUL, W_MU4, W_MU2, W_T2)) ||
          (rr = W.scal(wide_k::SC_ADD, W_T1, W_T2, W_T3, true)) || (rr = W.scal(wide_k::SC_DIV, W_T3, W_TAU, W_ETA)))
        return rr;
    }
    {
      // u = zeta q + eta (s + beta u);  z = (zeta r + eta z) - alpha u;  x = (x + alpha p) + z
      Prog P(W);
      const int ze = P.scalar(W_ZETA), et = P.scalar(W_ETA), be = P.scalar(W_BETA), al = P.scalar(W_ALPHA);
      P.in(q, 0).in(sv, 1).in(u, 2).in(r, 3).in(z, 4).in(*x, 5).in(p, 6);
      P.op(wide_k::PO_MUL, 7, be, 2).op(wide_k::PO_ADD, 7, 1, 7).op(wide_k::PO_MUL, 7, et, 7)
          .op(wide_k::PO_MUL, 1, ze, 0).op(wide_k::PO_ADD, 2, 1, 7)      // u (reg 2)
          .op(wide_k::PO_MUL, 7, ze, 3).op(wide_k::PO_MUL, 1, et, 4).op(wide_k::PO_ADD, 7, 7, 1)
          .op(wide_k::PO_MUL, 1, al, 2).op(wide_k::PO_SUB, 4, 7, 1)      // z (reg 4)
          .op(wide_k::PO_MUL, 7, al, 6).op(wide_k::PO_ADD, 7, 5, 7).op(wide_k::PO_ADD, 5, 7, 4);  // x (reg 5)
      P.out(2, u).out(4, z).out(5, *x);
      if ((rr = P.run())) return rr;
      // r = (t - eta y) - zeta v
      Prog R(W);
      const int ze2 = R.scalar(W_ZETA), et2 = R.scalar(W_ETA);
      R.in(t, 0).in(y, 1).in(v, 2);
      R.op(wide_k::PO_MUL, 3, et2, 1).op(wide_k::PO_SUB, 3, 0, 3).op(wide_k::PO_MUL, 4, ze2, 2)
          .op(wide_k::PO_SUB, 3, 3, 4).out(3, r);
      if ((rr = R.run())) return rr;
    }
    if ((rr = W.dot(r, r, W_Q))) return rr;
    bool stop = false;
    if ((rr = wide_after(W, o, i, info, &stop))) return rr;
    if (stop) break;
    if ((rr = W.is_zero(W_ZETA, &zf))) return rr;
    if (zf) {
      info->status = MP_BREAKDOWN_ZETA;
      break;
    }
    if ((rr = W.copy_slot(W_RHO, W_RHO_OLD)) || (rr = W.copy_slot(W_ALPHA, W_ALPHA_OLD)) ||
        (rr = W.copy_slot(W_ZETA, W_ZETA_OLD)))
      return rr;
  }
  return final_res(W, info);
}

int wide_bicg(int L, const WideOp& op, const WideOp& opT, const mp_vec* b, mp_vec* x,
              const mp_solve_opts* o, mp_solve_info* info, uint32_t* status, hipStream_t s) {
  const int64_t n = op.n_out;
  const int mode = o->mode;
  WideBufs B;
  mp_vec r, rt, p, pt, z, zt, sc;
  int rr;
  if ((rr = B.vec(L, n, &r)) || (rr = B.vec(L, n, &rt)) || (rr = B.vec(L, n, &p)) || (rr = B.vec(L, n, &pt)) ||
      (rr = B.vec(L, n, &z)) || (rr = B.vec(L, n, &zt)))
    return rr;
  // scalars: rho, rho_old, alpha, beta, sigma, q, q0, nrm0, thr, c_rel, c_abs, t
  enum { RHO, RHO_OLD, ALPHA, BETA, SIGMA, Q, Q0, NRM0, THR, CREL, CABS, TMP, NSC };
  if ((rr = B.vec(L, NSC, &sc))) return rr;
  int32_t* dflag = nullptr;
  hipError_t e = hipMalloc((void**)&dflag, sizeof(int32_t));
  if (e != hipSuccess) return fail(MPS_ENOMEM, "wide solve flag: %s", hipGetErrorString(e));
  B.ptrs.push_back(dflag);
  auto S = [&](int k) { return elem(sc, k); };
  // tolerance constants
  std::vector<uint32_t> m(L);
  int32_t h;
  for (int t = 0; t < 2; ++t) {
    const int64_t mm = t ? o->atol_m : o->rtol_m, ee = t ? o->atol_e10 : o->rtol_e10;
    if (!decimal_to_mp(mm, ee, L, m.data(), &h)) return fail(MPS_EINVAL, "tolerance out of range");
    const mp_vec c = S(t ? CABS : CREL);
    for (int k = 0; k < L; ++k) {
      e = hipMemcpyAsync(c.limb + (int64_t)k * c.ld, &m[k], 4, hipMemcpyHostToDevice, s);
      if (e != hipSuccess) return hip_fail(e, "tolerance upload");
    }
    e = hipMemcpyAsync(c.hdr, &h, 4, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "tolerance upload");
  }
  auto flag = [&](int32_t* out) -> int {
    hipError_t ee = hipMemcpyAsync(out, dflag, 4, hipMemcpyDeviceToHost, s);
    if (ee == hipSuccess) ee = hipStreamSynchronize(s);
    return ee == hipSuccess ? MPS_OK : hip_fail(ee, "wide solve flag");
  };
  auto spmv = [&](const WideOp& A, const mp_vec& in, const mp_vec& out) {
    return wide_spmv(L, A.n_out, A.row_ptr, A.col_idx, A.val, in, out, mode, status, s);
  };
  const mp_vec xv = *x;
  // r = b - A x0, or r = b and x = +0
  if (o->use_x0) {
    if ((rr = spmv(op, xv, r))) return rr;
    if ((rr = wide_axpy(L, 3, S(TMP), *b, r, n, status, s))) return rr;  // (alpha unused)
  } else {
    if ((rr = wzero(L, xv, n, s))) return rr;
    if ((rr = wcopy(L, *b, r, n, s))) return rr;
  }
  if ((rr = wcopy(L, r, rt, n, s))) return rr;
  // q0 = (r, r), thr = RN(RN(c_rel RN(sqrt q0)) + c_abs)
  const mp_vec q0 = S(Q0), nrm0 = S(NRM0), tmp = S(TMP), crel = S(CREL), cabs = S(CABS), thr = S(THR);
  if ((rr = wide_dot(L, r, r, q0, status, s))) return rr;
  if ((rr = wscalar(L, wide_k::SC_SQRT, q0, nullptr, &nrm0, nullptr, status, s))) return rr;
  if ((rr = wscalar(L, wide_k::SC_MUL, crel, &nrm0, &tmp, nullptr, status, s))) return rr;
  if ((rr = wscalar(L, wide_k::SC_ADD, tmp, &cabs, &thr, nullptr, status, s))) return rr;
  mp_vec hist{nullptr, nullptr, 0, 0};
  if (o->res_hist && o->res_hist->len > 0) hist = *o->res_hist;
  int32_t f = 0;
  if ((rr = wscalar(L, wide_k::SC_CONV, q0, &thr, nullptr, dflag, status, s)) || (rr = flag(&f))) return rr;
  info->iters = 0;
  info->status = MP_NC;
  if (f) {
    info->status = MP_CONVERGED;
  } else {
    for (int64_t i = 1; i <= o->maxit; ++i) {
      const mp_vec rho = S(RHO), rho_old = S(RHO_OLD), alpha = S(ALPHA), beta = S(BETA), sigma = S(SIGMA), q = S(Q);
      if ((rr = wide_dot(L, rt, r, rho, status, s))) return rr;
      if ((rr = wscalar(L, wide_k::SC_ZERO, rho, nullptr, nullptr, dflag, status, s)) || (rr = flag(&f))) return rr;
      if (f) {
        info->status = MP_BREAKDOWN_RHO;
        info->iters = i - 1;
        break;
      }
      if (i == 1) {
        if ((rr = wcopy(L, r, p, n, s)) || (rr = wcopy(L, rt, pt, n, s))) return rr;
      } else {
        if ((rr = wscalar(L, wide_k::SC_DIV, rho, &rho_old, &beta, nullptr, status, s))) return rr;
        if ((rr = wide_axpy(L, 1, beta, r, p, n, status, s)) || (rr = wide_axpy(L, 1, beta, rt, pt, n, status, s)))
          return rr;
      }
      if ((rr = spmv(op, p, z)) || (rr = spmv(opT, pt, zt))) return rr;
      if ((rr = wide_dot(L, pt, z, sigma, status, s))) return rr;
      if ((rr = wscalar(L, wide_k::SC_ZERO, sigma, nullptr, nullptr, dflag, status, s)) || (rr = flag(&f))) return rr;
      if (f) {
        info->status = MP_BREAKDOWN_SIGMA;
        info->iters = i - 1;
        break;
      }
      if ((rr = wscalar(L, wide_k::SC_DIV, rho, &sigma, &alpha, nullptr, status, s))) return rr;
      if ((rr = wide_axpy(L, 0, alpha, p, xv, n, status, s)) || (rr = wide_axpy(L, 2, alpha, z, r, n, status, s)) ||
          (rr = wide_axpy(L, 2, alpha, zt, rt, n, status, s)))
        return rr;
      if ((rr = wide_dot(L, r, r, q, status, s))) return rr;
      if (hist.limb && i - 1 < hist.len && (rr = wcopy(L, q, elem(hist, i - 1), 1, s))) return rr;
      if ((rr = wscalar(L, wide_k::SC_CONV, q, &thr, nullptr, dflag, status, s)) || (rr = flag(&f))) return rr;
      info->iters = i;
      if (f) {
        info->status = MP_CONVERGED;
        break;
      }
      if ((rr = wcopy(L, rho, rho_old, 1, s))) return rr;
    }
  }
  // display-only residual ratio
  std::vector<uint32_t> ql(L), q0l(L);
  int32_t qh = 0, q0h = 0;
  const mp_vec qv = S(info->iters > 0 ? Q : Q0), q0v = S(Q0);
  e = hipSuccess;
  if (e == hipSuccess) e = hipMemcpyAsync(&qh, qv.hdr, 4, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipMemcpyAsync(&q0h, q0v.hdr, 4, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipMemcpyAsync(&ql[L - 1], qv.limb + (int64_t)(L - 1) * qv.ld, 4, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipMemcpyAsync(&q0l[L - 1], q0v.limb + (int64_t)(L - 1) * q0v.ld, 4, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "wide solve readback");
  auto approx = [](uint32_t top, int32_t hd) {
    const int32_t ex = hd >> 1;
    if (ex == kZeroE) return 0.0;
    return std::ldexp((double)top, std::max(-1070, std::min(1020, ex - 32)));
  };
  const double a0 = approx(q0l[L - 1], q0h), a1 = approx(ql[L - 1], qh);
  info->final_rel_res = a0 > 0 ? std::sqrt(a1 / a0) : 0.0;
  return MPS_OK;
}

}  // namespace mpapi
