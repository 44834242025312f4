// Exact fixed-point accumulation of p-bit products ("superaccumulator") and its single final
// rounding.
//
// A window is an array of signed 64-bit digits; digit w carries weight 2^(32 w + base).  Each
// exact product (2L limbs) is shifted to its bit offset and its 32-bit pieces are added into the
// digits without carry propagation (carry-save), so the order of additions never matters and
// partial windows combine by plain integer addition.  With fewer than 2^31 addends per digit no
// digit overflows.  Finalisation propagates carries once, takes the sign, locates the leading
// bit and rounds to p bits with round and sticky bits: RN of the exact sum.
#pragma once
#include "mp_core.hpp"

namespace mp {

// Per-lane private window size used by the fast paths (spans up to 8 digits of exponent).
template <int L>
constexpr int window_fast_digits() { return 2 * L + 10; }

// Number of digits for products whose (e_a + e_b) spans [emin, emax]: the widest product sits
// at digit offset (span >> 5) and occupies 2L + 1 digits after the bit shift; one more digit of
// headroom absorbs the carries of up to 2^31 addends and the sign.
template <int L>
MPD int window_digits(int32_t emin, int32_t emax) {
  return (int)(((uint32_t)(emax - emin)) >> 5) + 2 * L + 2;
}

// Shift the exact product P (2L limbs) left by r bits (0 <= r < 32) into 2L + 1 limbs.
template <int L>
MPD void shift_product(const uint32_t (&P)[2 * L], uint32_t r, uint32_t (&sp)[2 * L + 1]) {
  sp[0] = P[0] << r;
#pragma unroll
  for (int j = 1; j < 2 * L; ++j) sp[j] = r ? fshr(P[j], P[j - 1], 32u - r) : P[j];
  sp[2 * L] = r ? (P[2 * L - 1] >> (32u - r)) : 0u;
}

// win[w * ws] += (-1)^s * (P << off) split in 32-bit digits (no carry propagation).  The adds
// are issued as LDS atomics without return: a window is private to its lane, but an atomic add
// needs no read-back, so the 2L + 1 adds of a product do not wait on one another.
template <int L>
MPD void window_add(int64_t* win, int ws, const uint32_t (&P)[2 * L], uint32_t s, uint32_t off) {
  uint32_t sp[2 * L + 1];
  shift_product<L>(P, off & 31u, sp);
  const int q = (int)(off >> 5);
#pragma unroll
  for (int j = 0; j <= 2 * L; ++j) {
    const int64_t v = s ? -(int64_t)sp[j] : (int64_t)sp[j];
    atomicAdd((unsigned long long*)&win[(q + j) * ws], (unsigned long long)v);
  }
}

// RN_p of a lane window of W <= WMAX digits at stride ws: digits read once, carried and signed
// in registers, the magnitude limbs written back and rounded.
template <int L, int WMAX>
MPD Num<L> lane_window_round(int64_t* win, int ws, int W, int64_t base, uint32_t& st);

// Same, with atomic adds (a window shared by several lanes).
template <int L>
MPD void window_add_atomic(int64_t* win, const uint32_t (&P)[2 * L], uint32_t s, uint32_t off) {
  uint32_t sp[2 * L + 1];
  shift_product<L>(P, off & 31u, sp);
  const int q = (int)(off >> 5);
#pragma unroll
  for (int j = 0; j <= 2 * L; ++j) {
    if (sp[j]) {
      const uint64_t v = s ? (uint64_t)(-(int64_t)sp[j]) : (uint64_t)sp[j];
      atomicAdd((unsigned long long*)&win[q + j], (unsigned long long)v);
    }
  }
}

// Digit w of a window lives at win[map(w)]: a stride (StrideMap) or a ring rotated so that
// window digit 0 is ring slot s0 (RingMap).
struct StrideMap {
  int ws;
  MPD int operator()(int w) const { return w * ws; }
};

template <int R>
struct RingMap {
  int ws, s0;
  MPD int operator()(int w) const { return (s0 + w >= R ? s0 + w - R : s0 + w) * ws; }
};

// Window accessor: digit w of a window (an LDS or private array, through an index map) is read
// with get(w) and written with set(w, v).
template <class Map>
struct MapWin {
  int64_t* win;
  Map map;
  MPD int64_t get(int w) const { return win[map(w)]; }
  MPD void set(int w, int64_t v) const { win[map(w)] = v; }
};

// RN_p of (-1)^sgn * sum_{w < nl} digit(w) 2^(32 w + base) for magnitude limbs (each digit
// holds a 32-bit limb; limb nl-1 is the top non-zero one, nl == 0 means zero).
template <int L, class Acc>
MPD Num<L> limbs_round_acc(const Acc& a, int nl, uint32_t sgn, int64_t base, uint32_t& st) {
  const int W = nl;
  const int top = nl - 1;
  Num<L> out;
  if (top < 0) {
    set_zero(out, 0);
    return out;
  }
  const int T = 32 * top + 31 - (int)__clz((uint32_t)a.get(top));  // leading bit index
  const int b0 = T - 32 * L + 1;                                     // mantissa LSB index
  auto limb_at = [&](int idx) -> uint32_t {
    return (idx >= 0 && idx < W) ? (uint32_t)a.get(idx) : 0u;
  };
  auto bits_at = [&](int b) -> uint32_t {  // the 32 bits starting at bit index b (b may be < 0)
    if (b <= -32) return 0u;
    if (b < 0) return limb_at(0) << (uint32_t)(-b);
    const int i = b >> 5;
    const uint32_t sh = (uint32_t)(b & 31);
    return sh ? fshr(limb_at(i + 1), limb_at(i), sh) : limb_at(i);
  };
#pragma unroll
  for (int k = 0; k < L; ++k) out.m[k] = bits_at(b0 + 32 * k);
  uint32_t rnd = 0, sticky = 0;
  const int rb = b0 - 1;
  if (rb >= 0) {
    rnd = (limb_at(rb >> 5) >> (rb & 31)) & 1u;
    const int ri = rb >> 5;
    const uint32_t below = (rb & 31) ? (limb_at(ri) & ((1u << (rb & 31)) - 1u)) : 0u;
    sticky = below;
    for (int w = 0; w < ri && !sticky; ++w) sticky |= limb_at(w);
  }
  int64_t e = (int64_t)b0 + base + 32 * L;
  uint32_t cy = rnd & (uint32_t)((sticky != 0) | (out.m[0] & 1u));
#pragma unroll
  for (int k = 0; k < L; ++k) out.m[k] = __builtin_addc(out.m[k], 0u, cy, &cy);
  if (cy) {
    out.m[L - 1] = 0x80000000u;
    e += 1;
  }
  out.s = sgn;
  if (e > kEmax || e < kEmin) {
    st |= kStRange;
    set_zero(out, sgn);
    return out;
  }
  out.e = (int32_t)e;
  return out;
}

template <int L, class Map>
MPD Num<L> limbs_round_map(const int64_t* win, Map map, int nl, uint32_t sgn, int64_t base,
                           uint32_t& st) {
  return limbs_round_acc<L>(MapWin<Map>{const_cast<int64_t*>(win), map}, nl, sgn, base, st);
}

template <int L>
MPD Num<L> limbs_round(const int64_t* win, int nl, uint32_t sgn, int64_t base, uint32_t& st,
                       int ws = 1) {
  return limbs_round_map<L>(win, StrideMap{ws}, nl, sgn, base, st);
}

// RN_p of the window value sum_w digit(w) * 2^(32 w + base) over W digits.  The digits are
// overwritten (they end up holding the 32-bit limbs of the magnitude).  An exact zero gives +0.
template <int L, class Acc>
MPD Num<L> window_finalize_acc(const Acc& a, int W, int64_t base, uint32_t& st) {
  int64_t c = 0;
  for (int w = 0; w < W; ++w) {
    const int64_t t = a.get(w) + c;
    a.set(w, (int64_t)(uint32_t)t);
    c = t >> 32;
  }
  const uint32_t sgn = (c < 0) ? 1u : 0u;
  if (sgn) {
    uint32_t cy = 1;
    for (int w = 0; w < W; ++w) a.set(w, (int64_t)__builtin_addc(~(uint32_t)a.get(w), 0u, cy, &cy));
  }
  int top = -1;
  for (int w = W - 1; w >= 0; --w) {
    if ((uint32_t)a.get(w) != 0u) {
      top = w;
      break;
    }
  }
  return limbs_round_acc<L>(a, top + 1, sgn, base, st);
}

template <int L, class Map>
MPD Num<L> window_finalize_map(int64_t* win, Map map, int W, int64_t base, uint32_t& st) {
  return window_finalize_acc<L>(MapWin<Map>{win, map}, W, base, st);
}

template <int L>
MPD Num<L> window_finalize(int64_t* win, int ws, int W, int64_t base, uint32_t& st) {
  return window_finalize_map<L>(win, StrideMap{ws}, W, base, st);
}

}  // namespace mp

namespace mp {

// RN_p of sum_w d_w 2^(32 w + base) for carry-save digits held one per lane of a wave (lane w
// holds digit w, |d_w| < 2^62; lanes past the window hold 0 and lane 63 must be headroom, so
// windows of at most 63 digits).  Every lane of the wave calls it and gets the result.
// Carries move up one lane per step until every digit is a 32-bit value (few steps unless a
// carry ripples); the sign is then lane 63's top bit; the magnitude, its leading bit, the
// mantissa limbs (lane k forms limb k), the round and sticky bits and the rounding carry are
// found with shuffles and lane masks.
template <int L>
MPD Num<L> wave_round(int64_t d, int64_t base, uint32_t& st) {
  const int lane = (int)(threadIdx.x & 63);
  const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;  // lanes under this one
  uint32_t lo = (uint32_t)d;
  int32_t c = (lane == 63) ? 0 : (int32_t)(d >> 32);
  while (__ballot(c != 0)) {
    const int32_t cin = __shfl_up(c, 1);
    const int64_t t = (int64_t)lo + (lane ? cin : 0);
    lo = (uint32_t)t;
    c = (lane == 63) ? 0 : (int32_t)(t >> 32);
  }
  const uint32_t neg = __shfl(lo, 63) >> 31;
  uint32_t m = lo;
  if (neg) {  // two's complement: ~lo plus a carry that passes every zero lane under this one
    const uint64_t nz = __ballot(lo != 0);
    m = ~lo + (((nz & below) == 0) ? 1u : 0u);
  }
  const uint64_t nzm = __ballot(m != 0);
  Num<L> out;
  if (nzm == 0) {
    set_zero(out, 0);
    return out;
  }
  const int top = 63 - (int)__clzll((long long)nzm);
  const uint32_t mtop = __shfl(m, top);
  const int b0 = 32 * top + 31 - (int)__clz((int)mtop) - 32 * L + 1;  // mantissa LSB bit index
  const int q0 = b0 >> 5;                                           // floor
  const uint32_t r0 = (uint32_t)(b0 & 31);
  const int i_lo = q0 + lane, i_hi = q0 + lane + 1;
  const uint32_t v_lo = __shfl(m, i_lo & 63), v_hi = __shfl(m, i_hi & 63);
  const uint32_t w_lo = (i_lo >= 0 && i_lo < 64) ? v_lo : 0u;
  const uint32_t w_hi = (i_hi >= 0 && i_hi < 64) ? v_hi : 0u;
  uint32_t limb = r0 ? fshr(w_hi, w_lo, r0) : w_lo;  // mantissa limb `lane` (lanes < L)
  uint32_t rnd = 0, sticky = 0;
  const int rb = b0 - 1;
  if (rb >= 0) {
    const int ri = rb >> 5;
    const uint32_t rs = (uint32_t)(rb & 31);
    const uint32_t mr = __shfl(m, ri);
    rnd = (mr >> rs) & 1u;
    const uint64_t under = ri ? (~0ull >> (64 - ri)) : 0ull;
    sticky = ((rs ? (mr & ((1u << rs) - 1u)) : 0u) != 0u || (nzm & under) != 0) ? 1u : 0u;
  }
  int64_t e = (int64_t)b0 + base + 32 * L;
  const uint32_t m0 = __shfl(limb, 0);
  if (rnd & (sticky | (m0 & 1u))) {
    constexpr uint64_t lmask = (L >= 64) ? ~0ull : ((1ull << L) - 1ull);
    const uint64_t ones = __ballot(limb == 0xFFFFFFFFu) & lmask;
    if (lane < L && (ones & below) == (below & lmask)) limb += 1u;
    if (ones == lmask) {  // all ones: the mantissa becomes 2^(p-1) one exponent up
      limb = (lane == L - 1) ? 0x80000000u : 0u;
      e += 1;
    }
  }
#pragma unroll
  for (int k = 0; k < L; ++k) out.m[k] = __shfl(limb, k);
  out.s = neg;
  if (e > kEmax || e < kEmin) {
    st |= kStRange;
    set_zero(out, neg);
    return out;
  }
  out.e = (int32_t)e;
  return out;
}

// Register-resident variants for windows of at most WMAX digits (the common case): the digits
// are read from LDS once, then carried, signed and rounded in registers with fully unrolled
// loops, avoiding a chain of dependent LDS round trips.
template <int WMAX>
struct RegWindow {
  uint32_t limb[WMAX];
  uint32_t neg;
  int nl;  // limbs up to and including the top non-zero one (0: the value is zero)
};

// Carry-propagate W <= WMAX carry-save digits into sign + magnitude limbs.
template <int WMAX>
MPD void reg_normalize(const int64_t* win, int ws, int W, RegWindow<WMAX>& R) {
  int64_t d[WMAX];
#pragma unroll
  for (int w = 0; w < WMAX; ++w) d[w] = (w < W) ? win[w * ws] : 0;
  int64_t c = 0;
#pragma unroll
  for (int w = 0; w < WMAX; ++w) {
    const int64_t t = d[w] + c;
    R.limb[w] = (uint32_t)t;
    c = t >> 32;
  }
  R.neg = (c < 0) ? 1u : 0u;
  if (R.neg) {
    uint32_t cy = 1;
#pragma unroll
    for (int w = 0; w < WMAX; ++w) R.limb[w] = __builtin_addc(~R.limb[w], 0u, cy, &cy);
  }
  int nl = 0;
#pragma unroll
  for (int w = 0; w < WMAX; ++w)
    if (R.limb[w] && w < W) nl = w + 1;
  R.nl = nl;
}

// RN_p of (-1)^neg * sum_w limb[w] 2^(32 w + base).
template <int L, int WMAX>
MPD Num<L> reg_round(const RegWindow<WMAX>& R, int64_t base, uint32_t& st) {
  Num<L> out;
  if (R.nl == 0) {
    set_zero(out, 0);
    return out;
  }
  uint32_t top_limb = 0;
#pragma unroll
  for (int w = 0; w < WMAX; ++w)
    if (w == R.nl - 1) top_limb = R.limb[w];
  const int T = 32 * (R.nl - 1) + 31 - (int)__clz(top_limb);
  const int b0 = T - 32 * L + 1;
  // mantissa limb k = bits [b0 + 32k, b0 + 32k + 32); b0 = 32 q0 + r0 (q0 may be negative)
  const int q0 = b0 >> 5;  // arithmetic shift: floor division
  const uint32_t r0 = (uint32_t)(b0 & 31);
  auto limb_at = [&](int idx) -> uint32_t {
    uint32_t v = 0;
#pragma unroll
    for (int w = 0; w < WMAX; ++w)
      if (w == idx) v = R.limb[w];
    return v;
  };
#pragma unroll
  for (int k = 0; k < L; ++k) {
    const uint32_t lo = limb_at(q0 + k), hi = limb_at(q0 + k + 1);
    out.m[k] = r0 ? fshr(hi, lo, r0) : lo;
  }
  // round bit at b0 - 1, sticky below it
  uint32_t rnd = 0, sticky = 0;
  const int rb = b0 - 1;
  if (rb >= 0) {
    const int ri = rb >> 5;
    const uint32_t rs = (uint32_t)(rb & 31);
#pragma unroll
    for (int w = 0; w < WMAX; ++w) {
      if (w < ri) sticky |= R.limb[w];
      if (w == ri) {
        rnd = (R.limb[w] >> rs) & 1u;
        sticky |= rs ? (R.limb[w] & ((1u << rs) - 1u)) : 0u;
      }
    }
  }
  int64_t e = (int64_t)b0 + base + 32 * L;
  uint32_t cy = rnd & (uint32_t)((sticky != 0) | (out.m[0] & 1u));
#pragma unroll
  for (int k = 0; k < L; ++k) out.m[k] = __builtin_addc(out.m[k], 0u, cy, &cy);
  if (cy) {
    out.m[L - 1] = 0x80000000u;
    e += 1;
  }
  out.s = R.neg;
  if (e > kEmax || e < kEmin) {
    st |= kStRange;
    set_zero(out, R.neg);
    return out;
  }
  out.e = (int32_t)e;
  return out;
}

// RN_p of sum_w win[w] 2^(32 w + base) for W carry-save digits in global memory (any W, one
// whole wavefront; every lane gets the result; the digits are overwritten; every access is
// device-coherent, like the adds that filled the window).  Three passes over
// the window, 64 digits at a time:
//  1. carries: each chunk's digits pass their high words one lane up until every digit is a
//     32-bit limb; lane 63's high word goes on to the next chunk, and the last chunk's is the
//     sign (the window's headroom digit keeps the sum inside W limbs of two's complement);
//  2. a negative sum is complemented into its magnitude (~limbs plus one, the one passing the
//     chunks' runs of all-ones limbs by lane masks);
//  3. the leading limb is found from the top, then the mantissa limbs, the round bit and the
//     sticky bits below it (every lower chunk, by ballots) are read, and rounding carries.
template <int L>
MPD Num<L> wave_window_round_global(int64_t* win, int W, int64_t base, uint32_t& st) {
  const int lane = (int)(threadIdx.x & 63);
  const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;  // lanes under this one
  int64_t carry = 0;  // into the chunk's lane 0 (wave-uniform)
  for (int c0 = 0; c0 < W; c0 += 64) {
    const int w = c0 + lane;
    int64_t d = (w < W) ? ld_dev(win + w) : 0;
    if (lane == 0) d += carry;
    uint32_t lo = (uint32_t)d;
    int64_t hi = d >> 32;
    int64_t out = 0;  // lane 63: what leaves the chunk
    while (__ballot(hi != 0)) {
      const int64_t from = __shfl_up(hi, 1);
      if (lane == 63) out += hi;
      const int64_t t = (int64_t)lo + (lane ? from : 0);
      lo = (uint32_t)t;
      hi = t >> 32;
    }
    if (w < W) st_dev(win + w, (int64_t)lo);
    carry = __shfl(out, 63);
  }
  wait_memory();
  const uint32_t neg = carry < 0 ? 1u : 0u;
  if (neg) {
    uint32_t cin = 1;  // the +1 of the two's complement, wave-uniform
    for (int c0 = 0; c0 < W; c0 += 64) {
      const int w = c0 + lane;
      const uint32_t m = (w < W) ? ~(uint32_t)ld_dev(win + w) : 0u;
      const uint64_t ones = __ballot(w < W && m == ~0u);
      // lane k gets the carry when every lane under it passes it on
      const bool gets = cin && ((ones & below) == below);
      if (w < W) st_dev(win + w, (int64_t)(m + (gets ? 1u : 0u)));
      cin = (cin && __ballot(w < W) == ones) ? 1u : 0u;
    }
  }
  wait_memory();
  // the leading non-zero limb
  int top = -1;
  for (int c0 = ((W - 1) / 64) * 64; c0 >= 0 && top < 0; c0 -= 64) {
    const int w = c0 + lane;
    const uint64_t nz = __ballot(w < W && (uint32_t)ld_dev(win + w) != 0u);
    if (nz) top = c0 + 63 - (int)__clzll((long long)nz);
  }
  Num<L> out;
  if (top < 0) {
    set_zero(out, 0);
    return out;
  }
  const uint32_t mtop = (uint32_t)ld_dev(win + top);
  const int b0 = 32 * top + 31 - (int)__clz((int)mtop) - 32 * L + 1;  // mantissa LSB bit index
  const int q0 = b0 >> 5;
  const uint32_t r0 = (uint32_t)(b0 & 31);
  auto limb_at = [&](int i) -> uint32_t { return (i >= 0 && i < W) ? (uint32_t)ld_dev(win + i) : 0u; };
  uint32_t limb = 0;
  if (lane < L) limb = r0 ? fshr(limb_at(q0 + lane + 1), limb_at(q0 + lane), r0) : limb_at(q0 + lane);
  uint32_t rnd = 0, sticky = 0;
  const int rb = b0 - 1;
  if (rb >= 0) {
    const int ri = rb >> 5;
    const uint32_t rs = (uint32_t)(rb & 31);
    const uint32_t mr = limb_at(ri);
    rnd = (mr >> rs) & 1u;
    sticky = (rs ? (mr & ((1u << rs) - 1u)) : 0u) != 0u ? 1u : 0u;
    for (int c0 = 0; c0 < ri && !sticky; c0 += 64) {
      const int w = c0 + lane;
      if (__ballot(w < ri && (uint32_t)ld_dev(win + w) != 0u)) sticky = 1u;
    }
  }
  int64_t e = (int64_t)b0 + base + 32 * L;
  const uint32_t m0 = __shfl(limb, 0);
  if (rnd & (sticky | (m0 & 1u))) {
    constexpr uint64_t lmask = (L >= 64) ? ~0ull : ((1ull << L) - 1ull);
    const uint64_t ones = __ballot(limb == 0xFFFFFFFFu) & lmask;
    if (lane < L && (ones & below) == (below & lmask)) limb += 1u;
    if (ones == lmask) {  // all ones: the mantissa becomes 2^(p-1) one exponent up
      limb = (lane == L - 1) ? 0x80000000u : 0u;
      e += 1;
    }
  }
#pragma unroll
  for (int k = 0; k < L; ++k) out.m[k] = __shfl(limb, k);
  out.s = neg;
  if (e > kEmax || e < kEmin) {
    st |= kStRange;
    set_zero(out, neg);
    return out;
  }
  out.e = (int32_t)e;
  return out;
}

template <int L, int WMAX>
MPD Num<L> lane_window_round(int64_t* win, int ws, int W, int64_t base, uint32_t& st) {
  RegWindow<WMAX> R;
  reg_normalize<WMAX>(win, ws, W, R);
#pragma unroll
  for (int w = 0; w < WMAX; ++w)
    if (w < W) win[w * ws] = (int64_t)R.limb[w];
  return limbs_round<L>(win, R.nl, R.neg, base, st, ws);
}

}  // namespace mp
