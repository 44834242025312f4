// Device limb arithmetic for p-bit binary floating point with round-to-nearest-even.
//
// Number model (Kouya, Sec. 2: the MPFR number with its mantissa kept apart from the exponent,
// IEEE-754-1985-like semantics, round-to-nearest):
//     x = (-1)^s * M * 2^(e - p),  2^(p-1) <= M < 2^p,  p = 32 * L
// M is held as L 32-bit limbs (m[0] least significant).  A zero has e == kZeroE and M == 0 and
// keeps its sign.  Exponents outside [kEmin, kEmax] (MPFR's default range) raise kStRange in the
// device status word; the paper never leaves that range.
//
// Storage (structure of arrays): limb k of element i at limb[k * ld + i]; hdr[i] = (e << 1) | s.
// A zero's header is INT32_MIN (+0) or INT32_MIN + 1 (-0); its limbs are ignored.
//
// All arithmetic is on 32-bit limbs with 32x32->64 multiplies and add/sub-with-carry chains.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define MPD __device__ __forceinline__

namespace mp {

constexpr int32_t kZeroE = -(1 << 30);
constexpr int32_t kEmin = 1 - (1 << 30);
constexpr int32_t kEmax = (1 << 30) - 1;

// device status word bits
constexpr uint32_t kStRange = 1u;    // a result exponent left [kEmin, kEmax]
constexpr uint32_t kStWindow = 2u;   // an exact accumulation needed a wider window than allowed
constexpr uint32_t kStDivZero = 4u;  // a scalar division by zero was requested

// Words per staged x record (the sparse product's copy of x, one record per element): the L
// limbs and the header, padded to a power of two so that a record sits in one cache line and
// loads as whole 16-byte pieces.  Host code sizes the staging buffers with it.
constexpr int x_rec_words_of(int L) { return L >= 32 ? 64 : (L >= 16 ? 32 : (L >= 8 ? 16 : 8)); }

template <int L>
struct Num {
  uint32_t m[L];
  int32_t e;
  uint32_t s;
};

MPD bool hdr_is_zero(int32_t h) { return (h >> 1) == kZeroE; }
MPD int32_t make_hdr(int32_t e, uint32_t s) { return (int32_t)(((uint32_t)e << 1) | (s & 1u)); }

template <int L>
MPD void set_zero(Num<L>& x, uint32_t s) {
#pragma unroll
  for (int k = 0; k < L; ++k) x.m[k] = 0;
  x.e = kZeroE;
  x.s = s;
}

template <int L>
MPD bool is_zero(const Num<L>& x) { return x.e == kZeroE; }

// Load element i.  The header and the limbs are requested together (one memory latency rather
// than a header read followed by dependent limb reads); a zero's limbs, whatever the buffer
// holds there, are replaced by 0.
template <int L>
MPD void load(Num<L>& x, const uint32_t* __restrict__ limb, const int32_t* __restrict__ hdr,
              int64_t ld, int64_t i) {
  const int32_t h = hdr[i];
  uint32_t m[L];
#pragma unroll
  for (int k = 0; k < L; ++k) m[k] = limb[(int64_t)k * ld + i];
  x.e = h >> 1;
  x.s = (uint32_t)h & 1u;
#pragma unroll
  for (int k = 0; k < L; ++k) x.m[k] = (x.e != kZeroE) ? m[k] : 0u;
}

template <int L>
MPD void store(const Num<L>& x, uint32_t* __restrict__ limb, int32_t* __restrict__ hdr,
               int64_t ld, int64_t i) {
  hdr[i] = make_hdr(x.e, x.s);
#pragma unroll
  for (int k = 0; k < L; ++k) limb[(int64_t)k * ld + i] = x.m[k];
}

// Device-coherent accesses for data that blocks of one launch exchange: relaxed device-scope
// atomic loads and stores, which bypass the per-XCD L2 copies, so they need neither the L2
// write-back of a device-scope release fence nor the invalidate of an acquire.
MPD uint32_t ld_dev(const uint32_t* p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }
MPD int32_t ld_dev(const int32_t* p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }
MPD void st_dev(uint32_t* p, uint32_t v) { __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }
MPD void st_dev(int32_t* p, int32_t v) { __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }
MPD int64_t ld_dev(const int64_t* p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }
MPD void st_dev(int64_t* p, int64_t v) { __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }

// Wait until every memory operation this wave has issued is complete.  Device-scope atomics and
// device-coherent stores are then performed at the device's coherence point, so an atomic the
// wave issues afterwards (a ticket) is observed after them: the ordering half of a release,
// without its L2 write-back (which the data exchanged this way does not need).
MPD void wait_memory() {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0);
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// Block barrier that orders LDS accesses only: this wave's LDS (and scalar-load) operations are
// complete (s_waitcnt lgkmcnt(0); the vector-memory and export counters are left alone), then
// s_barrier.  Global stores and atomics stay in flight across it (__syncthreads would wait for
// them: its workgroup fence waits for every outstanding memory operation).
MPD void lds_barrier() {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0xC07F);  // vmcnt 63, expcnt 7, lgkmcnt 0
  __builtin_amdgcn_s_barrier();
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

template <int L>
MPD void load_dev(Num<L>& x, const uint32_t* limb, const int32_t* hdr, int64_t ld, int64_t i) {
  const int32_t h = ld_dev(hdr + i);
  x.e = h >> 1;
  x.s = (uint32_t)h & 1u;
#pragma unroll
  for (int k = 0; k < L; ++k) x.m[k] = (x.e != kZeroE) ? ld_dev(limb + (int64_t)k * ld + i) : 0u;
}

template <int L>
MPD void store_dev(const Num<L>& x, uint32_t* limb, int32_t* hdr, int64_t ld, int64_t i) {
  st_dev(hdr + i, make_hdr(x.e, x.s));
#pragma unroll
  for (int k = 0; k < L; ++k) st_dev(limb + (int64_t)k * ld + i, x.m[k]);
}

// (hi:lo) >> s for 0 <= s < 32
MPD uint32_t fshr(uint32_t hi, uint32_t lo, uint32_t s) { return __builtin_amdgcn_alignbit(hi, lo, s); }

// ------------------------------------------------------------------------------------------
// Exact L x L limb product: p = a * b (2L limbs).  Row i is a[i] * b formed with one 32x32->64
// multiply-add per limb (the running carry is the added word), then added into p with a
// carry chain.
// ------------------------------------------------------------------------------------------
template <int L>
MPD void mul_full(const uint32_t (&a)[L], const uint32_t (&b)[L], uint32_t (&p)[2 * L]) {
#pragma unroll
  for (int i = 0; i < L; ++i) {
    uint32_t row[L + 1];
    uint32_t c = 0;
#pragma unroll
    for (int j = 0; j < L; ++j) {
      uint64_t t = (uint64_t)a[i] * b[j] + c;
      row[j] = (uint32_t)t;
      c = (uint32_t)(t >> 32);
    }
    row[L] = c;
    if (i == 0) {
#pragma unroll
      for (int j = 0; j <= L; ++j) p[j] = row[j];
    } else {
      uint32_t cy = 0;
#pragma unroll
      for (int j = 0; j < L; ++j) p[i + j] = __builtin_addc(p[i + j], row[j], cy, &cy);
      p[i + L] = row[L] + cy;
    }
  }
}

// Round the exact product (2L limbs, value P * 2^(e2 - 2p), P != 0 with its top bit at 2p-1 or
// 2p-2) to p bits, ties to even; straight-line code (selects).
template <int L>
MPD void round_product(const uint32_t (&pr)[2 * L], int32_t e2, uint32_t s, Num<L>& out,
                       uint32_t& st) {
  const bool top = (pr[2 * L - 1] >> 31) != 0;
  uint32_t m[L];
#pragma unroll
  for (int k = 0; k < L; ++k) m[k] = top ? pr[L + k] : fshr(pr[L + k], pr[L + k - 1], 31);
  const uint32_t rnd = top ? (pr[L - 1] >> 31) : ((pr[L - 1] >> 30) & 1u);
  uint32_t sticky = top ? (pr[L - 1] << 1) : (pr[L - 1] << 2);
#pragma unroll
  for (int k = 0; k < L - 1; ++k) sticky |= pr[k];
  int32_t e = top ? e2 : e2 - 1;
  uint32_t cy = rnd & (uint32_t)((sticky != 0) | (m[0] & 1u));
#pragma unroll
  for (int k = 0; k < L; ++k) m[k] = __builtin_addc(m[k], 0u, cy, &cy);
  m[L - 1] = cy ? 0x80000000u : m[L - 1];  // rounding carried out of the top: 2^p
  e += (int32_t)cy;
  const bool range = (e > kEmax) | (e < kEmin);
  st |= range ? kStRange : 0u;
#pragma unroll
  for (int k = 0; k < L; ++k) out.m[k] = range ? 0u : m[k];
  out.e = range ? kZeroE : e;
  out.s = s;
}

// RN(a * b).  The exact product is formed and rounded for every operand pair, and a zero
// factor then selects a zero with the xor sign: straight-line code (selects, no divergent
// branch), so the products of a wavefront's lanes run together whatever their data.  (The
// sparse products test their stored zeros first and skip the product.)
template <int L>
MPD Num<L> mul_rn(const Num<L>& a, const Num<L>& b, uint32_t& st) {
  const bool z = is_zero(a) | is_zero(b);
  uint32_t pr[2 * L];
  mul_full<L>(a.m, b.m, pr);
  // A zero factor's product (discarded below) is given a top bit, so that the exponent sum of
  // two zeros (INT32_MIN) is not decremented.
  pr[2 * L - 1] |= z ? 0x80000000u : 0u;
  uint32_t st1 = 0;
  Num<L> r;
  round_product<L>(pr, (int32_t)((uint32_t)a.e + (uint32_t)b.e), a.s ^ b.s, r, st1);
  st |= z ? 0u : st1;
#pragma unroll
  for (int k = 0; k < L; ++k) r.m[k] = z ? 0u : r.m[k];
  r.e = z ? kZeroE : r.e;
  return r;
}

// x (N limbs) >>= d, 0 <= d < 32N; bits shifted out are ORed into bit 0 (sticky).  Whole
// limbs move in log2(N) select stages.
template <int N>
MPD void shr_sticky(uint32_t (&x)[N], uint32_t d) {
  const uint32_t q = d >> 5, r = d & 31u;
  uint32_t sticky = 0;
#pragma unroll
  for (int bit = 1; bit < N; bit <<= 1) {
    const bool sh = (q & (uint32_t)bit) != 0;
    uint32_t lost = 0;
#pragma unroll
    for (int i = 0; i < bit; ++i) lost |= x[i];
    sticky |= sh ? lost : 0u;
#pragma unroll
    for (int i = 0; i < N; ++i) x[i] = sh ? ((i + bit < N) ? x[i + bit] : 0u) : x[i];
  }
  sticky |= r ? (x[0] << (32u - r)) : 0u;
#pragma unroll
  for (int i = 0; i < N - 1; ++i) x[i] = fshr(x[i + 1], x[i], r);
  x[N - 1] >>= r;
  x[0] |= (sticky != 0) ? 1u : 0u;
}

// x (N limbs) <<= d, 0 <= d < 32N
template <int N>
MPD void shl(uint32_t (&x)[N], uint32_t d) {
  const uint32_t q = d >> 5, r = d & 31u;
#pragma unroll
  for (int bit = 1; bit < N; bit <<= 1) {
    const bool sh = (q & (uint32_t)bit) != 0;
#pragma unroll
    for (int i = N - 1; i >= 0; --i) x[i] = sh ? ((i >= bit) ? x[i - bit] : 0u) : x[i];
  }
#pragma unroll
  for (int i = N - 1; i >= 1; --i) x[i] = r ? fshr(x[i], x[i - 1], 32u - r) : x[i];
  x[0] <<= r;
}

// leading zero bits of an N-limb integer (32N for zero)
template <int N>
MPD uint32_t clz_n(const uint32_t (&x)[N]) {
  uint32_t lz = 0;
  bool found = false;
#pragma unroll
  for (int i = N - 1; i >= 0; --i) {
    lz += found ? 0u : (uint32_t)__clz(x[i]);
    found |= x[i] != 0;
  }
  return lz;
}

// RN(a + b), IEEE/MPFR signed-zero rules for round-to-nearest.
//
// The operand with the larger exponent is X.  Both mantissas get one extra low limb (32 guard
// bits); Y's is shifted right by the exponent difference d with the shifted-out bits ORed into
// bit 0.  For d >= 2 an effective subtraction loses at most one leading bit, so that sticky
// bit always stays below the round bit (bit 31 of the guard limb); for d <= 1 no bit is
// shifted out and the difference is exact before normalisation.  For d >= p + 2, |Y| is below
// a quarter of X's last unit and the result is X: d is clamped there (Y then lands inside the
// guard limb, below its round bit, and rounding returns X).
//
// Mostly straight-line code: the subtraction is the addition of Y's complement, an addition that
// carried out is shifted right by one, a one-bit cancellation is shifted back, and zero
// operands, an exact zero and range errors are selected at the end.  Only the cases that need
// d <= 1 branch: a negative difference (negated) and a cancellation of more than one bit.
template <int L>
MPD Num<L> add_rn(const Num<L>& a, const Num<L>& b, uint32_t& st) {
  const bool az = is_zero(a), bz = is_zero(b);
  const bool sw = b.e > a.e;  // a zero's exponent is below every other one
  uint32_t xa[L + 1], ya[L + 1];
  xa[0] = 0;
  ya[0] = 0;
#pragma unroll
  for (int k = 0; k < L; ++k) {
    xa[k + 1] = sw ? b.m[k] : a.m[k];
    ya[k + 1] = sw ? a.m[k] : b.m[k];
  }
  const int32_t Xe = sw ? b.e : a.e, Ye = sw ? a.e : b.e;
  const uint32_t Xs = sw ? b.s : a.s, Ys = sw ? a.s : b.s;
  const uint32_t d = min((uint32_t)(Xe - Ye), (uint32_t)(32 * L + 2));
  shr_sticky<L + 1>(ya, d);
  const bool sub = Xs != Ys;
  const uint32_t mask = sub ? ~0u : 0u;
  uint32_t r[L + 1];
  uint32_t cy = sub ? 1u : 0u;
#pragma unroll
  for (int k = 0; k <= L; ++k) r[k] = __builtin_addc(xa[k], ya[k] ^ mask, cy, &cy);
  const bool neg = sub & (cy == 0);   // |Y| > |X| (d == 0 only: rare, so a branch)
  const bool ovf = !sub & (cy != 0);  // the sum carried out of the top limb
  if (neg) {
    uint32_t c2 = 1;
#pragma unroll
    for (int k = 0; k <= L; ++k) r[k] = __builtin_addc(~r[k], 0u, c2, &c2);
  }
  const uint32_t s = Xs ^ (neg ? 1u : 0u);
  int32_t e = Xe + (ovf ? 1 : 0);
  {
    const uint32_t lost = r[0] & 1u;
    uint32_t t[L + 1];
#pragma unroll
    for (int k = 0; k < L; ++k) t[k] = fshr(r[k + 1], r[k], 1);
    t[L] = (r[L] >> 1) | 0x80000000u;
    t[0] |= lost;
#pragma unroll
    for (int k = 0; k <= L; ++k) r[k] = ovf ? t[k] : r[k];
  }
  const uint32_t lz = clz_n<L + 1>(r);
  const bool zres = lz >= 32u * (L + 1);  // exact cancellation
  const uint32_t lzs = zres ? 0u : lz;
  if (lzs > 1) {  // a cancellation of more than one bit (d <= 1 only: a branch)
    shl<L + 1>(r, lzs);
  } else {
#pragma unroll
    for (int k = L; k >= 1; --k) r[k] = lzs ? fshr(r[k], r[k - 1], 31) : r[k];
    r[0] = lzs ? r[0] << 1 : r[0];
  }
  e -= (int32_t)lzs;
  const uint32_t rnd = r[0] >> 31;
  const uint32_t sticky = r[0] & 0x7fffffffu;
  uint32_t m[L];
#pragma unroll
  for (int k = 0; k < L; ++k) m[k] = r[k + 1];
  uint32_t c3 = rnd & (uint32_t)((sticky != 0) | (m[0] & 1u));
#pragma unroll
  for (int k = 0; k < L; ++k) m[k] = __builtin_addc(m[k], 0u, c3, &c3);
  m[L - 1] = c3 ? 0x80000000u : m[L - 1];
  e += (int32_t)c3;
  const bool bothz = az & bz;
  const bool range = !bothz & !zres & ((e > kEmax) | (e < kEmin));
  st |= range ? kStRange : 0u;
  const bool zr = bothz | zres | range;
  Num<L> out;
#pragma unroll
  for (int k = 0; k < L; ++k) out.m[k] = zr ? 0u : m[k];
  out.e = zr ? kZeroE : e;
  out.s = bothz ? (a.s & b.s) : zres ? 0u : s;  // x - x is +0; (-0) + (-0) is -0
  return out;
}

template <int L>
MPD Num<L> neg(const Num<L>& a) {
  Num<L> r = a;
  r.s ^= 1u;
  return r;
}

template <int L>
MPD Num<L> sub_rn(const Num<L>& a, const Num<L>& b, uint32_t& st) {
  return add_rn<L>(a, neg<L>(b), st);
}

}  // namespace mp
