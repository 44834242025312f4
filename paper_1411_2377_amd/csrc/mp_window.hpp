// Windowed SEQ chains: a long row's serial RN additions advanced up to 64 at a time by one
// wavefront, with exactly the results of the one-at-a-time chain.
//
// Let the running sum be Y = (-1)^s M u with M in [2^(p-1), 2^p) and u = 2^(E - p) its unit in
// the last place, and let the next product be t.  As long as the exact Y + t stays in Y's binade
// and on Y's side of zero, RN(Y + t) is the multiple of u nearest to Y + t, which is
// Y + RN_u(t): t rounded on its own to a multiple of u.  Over a run of steps that all stay in
// the binade, the chain is therefore a plain integer sum, M_k = M + sum_{i <= k} r_i with
// r_i = RN_u(t_i) / u, and integer sums can be formed in any order.  One round of the wavefront:
//  * lane i rounds its product t_i onto the grid of u (one shift of its mantissa by E - e_i,
//    round and sticky bits), giving r_i as an (L + 1)-word two's complement integer relative to
//    Y's sign;
//  * an inclusive prefix sum of the r_i over the lanes (DPP row shifts and row broadcasts, one
//    multi-word addition per stage) gives every M_i = M + sum_{j <= i} r_j;
//  * lane i's step is exact if 2^(p-1) < M_i < 2^p (the exact sum then lies strictly inside the
//    binade, because it differs from M_i by less than half a unit) and no earlier step failed;
//    steps whose product is zero add 0 and always pass;
//  * the steps up to the first failing lane are committed at once (M taken from the lane before
//    it), the failing step itself is done with the general RN addition, and the next round
//    starts after it.
// A step fails when its product lies above Y's binade or when the sum would leave the binade or
// cross zero.  A product that rounds half-way onto the grid is taken rounded towards zero in
// the prefix sum, then, in lane order, the sums from that step on move one unit when ties to
// even ask for it (the parity of that step's sum is known once the steps before it are).  A zero
// running sum takes the next non-zero product as it is (RN(+0 + t) = t).  On the power-law
// workload about one step in 80 fails, so a round commits some 40 steps.
#pragma once
#include "mp_core.hpp"

namespace mp {

// A DPP move that reads 0 where the source lane is outside the row or the row is masked off.
template <int CTRL, int ROWM>
MPD uint32_t win_dpp(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROWM, 0xf, true);
}

// v += (v of another lane, by the DPP pattern CTRL) over N words with carries.
template <int N, int CTRL, int ROWM>
MPD void win_scan_stage(uint32_t (&v)[N]) {
  uint32_t t[N];
#pragma unroll
  for (int i = 0; i < N; ++i) t[i] = win_dpp<CTRL, ROWM>(v[i]);
  uint32_t c = 0;
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] = __builtin_addc(v[i], t[i], c, &c);
}

// Inclusive prefix sum of N-word integers (mod 2^(32 N)) over the 64 lanes, in lane order:
// row shifts by 1, 2, 4 and 8 within each row of 16 lanes, then the last lane of row 0 (2) into
// row 1 (3), then lane 31 into rows 2 and 3.
template <int N>
MPD void win_scan(uint32_t (&v)[N]) {
  win_scan_stage<N, 0x111, 0xf>(v);  // row_shr:1
  win_scan_stage<N, 0x112, 0xf>(v);  // row_shr:2
  win_scan_stage<N, 0x114, 0xf>(v);  // row_shr:4
  win_scan_stage<N, 0x118, 0xf>(v);  // row_shr:8
  win_scan_stage<N, 0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
  win_scan_stage<N, 0x143, 0xc>(v);  // row_bcast:31 into rows 2 and 3
}

// r = (-1)^neg * RN(M / 2^d) as an (L + 1)-word two's complement integer, M an L-limb mantissa
// (not zero), d >= 0; *tie when M / 2^d lies exactly half-way between two integers.  The shift
// is of M * 2^32 (a guard word below), so the guard word's top bit is the round bit and its
// other bits, with every bit shifted out below it, the sticky bits.  Called by the lanes that
// have a product to place (the stages of whole-word shifts nobody needs are skipped).
template <int L>
MPD void win_align_round(const uint32_t (&m)[L], uint32_t d, bool neg, uint32_t (&r)[L + 1], bool& tie) {
  uint32_t w[L + 1];
  w[0] = 0u;
#pragma unroll
  for (int i = 0; i < L; ++i) w[i + 1] = m[i];
  const uint32_t q = min(d >> 5, (uint32_t)(L + 1));  // whole words
  uint32_t lost = 0u;
#pragma unroll
  for (int k = 1; k <= L + 1; k <<= 1) {
    const bool on = (q & (uint32_t)k) != 0u;
    if (k > 1 && __ballot(on) == 0ull) continue;  // no lane shifts by k words (the common case)
    uint32_t out = 0u;
#pragma unroll
    for (int j = 0; j < k && j <= L; ++j) out |= w[j];
    lost |= on ? out : 0u;
#pragma unroll
    for (int i = 0; i <= L; ++i) w[i] = on ? (i + k <= L ? w[i + k] : 0u) : w[i];
  }
  const uint32_t b = d & 31u;
  lost |= w[0] & ((1u << b) - 1u);
#pragma unroll
  for (int i = 0; i < L; ++i) w[i] = __builtin_amdgcn_alignbit(w[i + 1], w[i], b);
  w[L] >>= b;
  const bool rnd = (w[0] >> 31) != 0u;
  const bool sticky = ((w[0] << 1) | lost) != 0u;
  tie = rnd && !sticky;
  const uint32_t inc = (rnd && sticky) ? 1u : 0u;
  // (-1)^neg (S + inc) = (S ^ mask) + (neg ? 1 - inc : inc), S = w[1 .. L]
  const uint32_t mask = neg ? ~0u : 0u;
  uint32_t c = neg ? 1u - inc : inc;
#pragma unroll
  for (int i = 0; i < L; ++i) r[i] = __builtin_addc(w[i + 1] ^ mask, 0u, c, &c);
  r[L] = mask + c;
}

// 2^(p-1) < M < 2^p for an (L + 1)-word M: the step's exact sum lies inside the binade.
template <int L>
MPD bool win_inside(const uint32_t (&m)[L + 1]) {
  uint32_t below = 0u;
#pragma unroll
  for (int k = 0; k < L - 1; ++k) below |= m[k];
  return m[L] == 0u && (m[L - 1] >> 31) != 0u && (m[L - 1] != 0x80000000u || below != 0u);
}

// One windowed chain over the products t_i held by the lanes (lane i: product i of the window),
// steps i = start .. n - 1 in order, starting from the wave-uniform running sum y.  Every lane
// must call it together; y comes back wave-uniform.
template <int L>
MPD void win_chain(Num<L>& y, const Num<L>& t, int start, int n, uint32_t& st) {
  const int lane = (int)(threadIdx.x & 63u);
  while (start < n) {
    const bool act = lane >= start && lane < n;
    if (is_zero(y)) {
      // RN(+0 + t) = t, and a zero t leaves +0: the first non-zero product is taken as it is
      const uint64_t nz = __ballot(act && !is_zero(t));
      if (nz == 0ull) return;
      const int f = __ffsll((unsigned long long)nz) - 1;
#pragma unroll
      for (int k = 0; k < L; ++k) y.m[k] = (uint32_t)__shfl((int)t.m[k], f, 64);
      y.e = __shfl(t.e, f, 64);
      y.s = (uint32_t)__shfl((int)t.s, f, 64);
      start = f + 1;
      continue;
    }
    // r_i relative to y's sign (a half-way step rounded towards zero for now), the prefix sums,
    // and the first step the window cannot take
    uint32_t r[L + 1];
    bool big = false, tie = false;
    const bool live = act && !is_zero(t);
    const bool neg = t.s != y.s;
    if (live && t.e > y.e) {
      big = true;
#pragma unroll
      for (int k = 0; k <= L; ++k) r[k] = 0u;
    } else if (live) {
      win_align_round<L>(t.m, (uint32_t)(y.e - t.e), neg, r, tie);
    } else {
#pragma unroll
      for (int k = 0; k <= L; ++k) r[k] = 0u;
    }
    win_scan<L + 1>(r);
    uint32_t c = 0;
#pragma unroll
    for (int k = 0; k < L; ++k) r[k] = __builtin_addc(r[k], y.m[k], c, &c);
    r[L] += c;
    uint64_t fail = __ballot(act && (big || !win_inside<L>(r)));
    // Half-way steps before the first failure, in order: the exact sum lies half a unit beyond
    // M_i on the step's side, and ties to even keep M_i when it is even, else move it one unit
    // further; the sums after it move with it.
    uint64_t ties = __ballot(act && tie);
    while (ties) {
      const int g = __ffsll((unsigned long long)ties) - 1;
      if (fail && g >= __ffsll((unsigned long long)fail) - 1) break;
      ties &= ties - 1;
      if ((__shfl((int)r[0], g, 64) & 1) == 0) continue;
      const bool gneg = __shfl(neg ? 1 : 0, g, 64) != 0;
      const bool on = lane >= g;
      const uint32_t ext = (on && gneg) ? ~0u : 0u;  // -1 or +1 over L + 1 words
      uint32_t cc = 0;
      r[0] = __builtin_addc(r[0], on ? (gneg ? ~0u : 1u) : 0u, cc, &cc);
#pragma unroll
      for (int k = 1; k <= L; ++k) r[k] = __builtin_addc(r[k], ext, cc, &cc);
      fail = __ballot(act && (big || !win_inside<L>(r)));
    }
    const int f = fail ? __ffsll((unsigned long long)fail) - 1 : n;
    if (f > start) {  // steps start .. f - 1 hold: M from lane f - 1
#pragma unroll
      for (int k = 0; k < L; ++k) y.m[k] = (uint32_t)__shfl((int)r[k], f - 1, 64);
    }
    if (f >= n) return;
    // step f by the general RN addition (t_f is not zero)
    Num<L> tf;
#pragma unroll
    for (int k = 0; k < L; ++k) tf.m[k] = (uint32_t)__shfl((int)t.m[k], f, 64);
    tf.e = __shfl(t.e, f, 64);
    tf.s = (uint32_t)__shfl((int)t.s, f, 64);
    y = add_rn<L>(y, tf, st);
    start = f + 1;
  }
}

}  // namespace mp

namespace mp {

// ---- segmented windows: four chains per wavefront ----------------------------------------
// The same rounds with each row of 16 lanes (a DPP row) carrying its own chain: lane j of row
// g holds the g-th chain's product j, every lane holds its row's running sum, and the prefix
// sums stop at the row's edge.  Rows whose steps are done, or that have none, stay idle.

// Inclusive prefix sum of N-word integers within each row of 16 lanes.
template <int N>
MPD void win_scan16(uint32_t (&v)[N]) {
  win_scan_stage<N, 0x111, 0xf>(v);  // row_shr:1
  win_scan_stage<N, 0x112, 0xf>(v);  // row_shr:2
  win_scan_stage<N, 0x114, 0xf>(v);  // row_shr:4
  win_scan_stage<N, 0x118, 0xf>(v);  // row_shr:8
}

// The 16 bits of a wavefront mask that belong to this lane's row, as the low bits.
MPD uint32_t seg_bits(uint64_t m) { return (uint32_t)(m >> (threadIdx.x & 48u)) & 0xffffu; }

// Lowest set bit of each row's 16 bits of m.
MPD uint64_t seg_lowest(uint64_t m) {
  const uint32_t j = threadIdx.x & 15u;
  const uint32_t b = seg_bits(m);
  return __ballot(((b >> j) & 1u) != 0u && (b & ((1u << j) - 1u)) == 0u);
}

template <int L>
MPD Num<L> seg_take(const Num<L>& t, int src) {
  Num<L> o;
#pragma unroll
  for (int k = 0; k < L; ++k) o.m[k] = (uint32_t)__shfl((int)t.m[k], src, 64);
  o.e = __shfl(t.e, src, 64);
  o.s = (uint32_t)__shfl((int)t.s, src, 64);
  return o;
}

// Every row's chain over its products t (lane j: product j), steps start .. n - 1 of the row
// (n <= 16; start and n the same in all lanes of a row), from each row's running sum y.
template <int L>
MPD void win_chain_seg(Num<L>& y, const Num<L>& t, int n, uint32_t& st) {
  const int lane = (int)(threadIdx.x & 63u), j = lane & 15, base = lane & 48;
  int start = 0;
  while (__ballot(start < n) != 0ull) {
    // rows with a zero sum take their next non-zero product as it is
    if (__ballot(start < n && is_zero(y)) != 0ull) {
      const bool act = j >= start && j < n;
      const uint32_t nz = seg_bits(__ballot(act && !is_zero(t)));
      const bool zrow = start < n && is_zero(y);
      const int f = nz ? __ffs(nz) - 1 : 16;
      const Num<L> tf = seg_take<L>(t, base + min(f, 15));
      if (zrow) {
        if (f < n) {
          y = tf;
          start = f + 1;
        } else {
          start = n;
        }
      }
    }
    const bool work = start < n && !is_zero(y);
    const bool act = work && j >= start && j < n;
    uint32_t r[L + 1];
    bool big = false, tie = false;
    const bool live = act && !is_zero(t);
    const bool neg = t.s != y.s;
    if (live && t.e > y.e) {
      big = true;
#pragma unroll
      for (int k = 0; k <= L; ++k) r[k] = 0u;
    } else if (live) {
      win_align_round<L>(t.m, (uint32_t)(y.e - t.e), neg, r, tie);
    } else {
#pragma unroll
      for (int k = 0; k <= L; ++k) r[k] = 0u;
    }
    win_scan16<L + 1>(r);
    uint32_t c = 0;
#pragma unroll
    for (int k = 0; k < L; ++k) r[k] = __builtin_addc(r[k], y.m[k], c, &c);
    r[L] += c;
    uint64_t fail = __ballot(act && (big || !win_inside<L>(r)));
    // half-way steps before each row's first failure, in lane order (as in win_chain)
    uint64_t ties = __ballot(act && tie);
    while (ties) {
      const uint64_t low = seg_lowest(ties);
      const uint32_t fb = seg_bits(fail), gb = seg_bits(low);
      const int f = fb ? __ffs(fb) - 1 : 16;
      const int g = gb ? __ffs(gb) - 1 : 16;
      const bool pend = g < f;  // this row has a half-way step to settle
      const uint64_t pending = __ballot(pend);
      if (pending == 0ull) break;
      ties &= ~(low & pending);
      const int src = base + min(g, 15);
      const bool odd = (__shfl((int)r[0], src, 64) & 1) != 0;
      const bool gneg = __shfl(neg ? 1 : 0, src, 64) != 0;
      const bool on = pend && odd && j >= g;
      const uint32_t ext = (on && gneg) ? ~0u : 0u;
      uint32_t cc = 0;
      r[0] = __builtin_addc(r[0], on ? (gneg ? ~0u : 1u) : 0u, cc, &cc);
#pragma unroll
      for (int k = 1; k <= L; ++k) r[k] = __builtin_addc(r[k], ext, cc, &cc);
      fail = __ballot(act && (big || !win_inside<L>(r)));
    }
    const uint32_t fb = seg_bits(fail);
    const int f = fb ? __ffs(fb) - 1 : n;  // first failing step of the row, or n
    // the row's sum after its steps start .. f - 1: M from lane f - 1
    uint32_t mc[L];
    const int src = base + max(min(f, n) - 1, 0);
#pragma unroll
    for (int k = 0; k < L; ++k) mc[k] = (uint32_t)__shfl((int)r[k], src, 64);
    if (work && f > start) {
#pragma unroll
      for (int k = 0; k < L; ++k) y.m[k] = mc[k];
    }
    // step f by the general RN addition
    const bool exc = work && f < n;
    if (__ballot(exc) != 0ull) {
      const Num<L> tf = seg_take<L>(t, base + min(f, 15));
      uint32_t sta = 0;  // every row computes it; only a row that takes it reports its status
      const Num<L> ya = add_rn<L>(y, tf, sta);
      if (exc) {
        y = ya;
        st |= sta;
      }
    }
    if (work) start = exc ? f + 1 : n;
  }
}

}  // namespace mp
