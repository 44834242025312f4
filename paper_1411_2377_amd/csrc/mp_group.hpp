// Limb-parallel round-to-nearest addition: one p-bit number spread over a group of L consecutive
// lanes of a wavefront (lane w of the group holds limb w, w = 0 least significant; every lane of
// the group holds the exponent and the sign).  The wavefront holds 64 / L such numbers and adds
// a second operand to each of them at once.
//
// The result is the same RN(a + b) as add_rn in mp_core.hpp (same guard limb, sticky bit and
// ties-to-even rule, same signed-zero and range behaviour); only the data layout differs.  The
// addition is built for latency (a sparse row's SEQ sum is one long chain of them):
//  * the alignment shift of the smaller operand moves its limbs q places down the group (q =
//    whole limbs of the shift) with DPP row shifts by 1, 2, 4 and 8 lanes selected by the bits
//    of q, and the bits shifted out are OR-reduced into the guard lane by DPP row shifts;
//  * a limb's carry into the next lane is passed by one DPP row shift.  It moves on only through
//    a limb that became all ones, which random data almost never produces: when some lane of
//    the wavefront would pass a carry on, the exact carries are resolved instead from two
//    wavefront ballots (generate and propagate bits per limb) and one 64-bit addition of those
//    masks per parity of group (even- and odd-numbered groups apart, so no carry leaves its
//    group).  Rounding's increment is treated the same way;
//  * the group's top limb decides the normalisation, read by all lanes of the group from ballots.
//
// Every function here must be called by all 64 lanes of the wavefront together, and every lane
// exchange (group_limb, the DPP moves, __shfl) is made outside any data-dependent branch: a lane
// that skips the exchange would hand 0 instead of its value to the lanes reading from it.
#pragma once
#include "mp_core.hpp"

namespace mp {

template <int L>
struct Group {
  int lane;         // lane in the wavefront
  int w;            // limb index of this lane within its group
  int base;         // first lane of the group
  uint64_t start;   // first lanes of all groups
  uint64_t top;     // last lanes of all groups
  uint64_t even;    // lanes of groups 0, 2, 4, ...
  uint64_t odd;     // lanes of groups 1, 3, 5, ...
};

template <int L>
MPD Group<L> group_of_lane() {
  static_assert(L == 4 || L == 8 || L == 16, "groups of 4, 8 or 16 lanes");
  Group<L> G;
  G.lane = (int)(threadIdx.x & 63u);
  G.w = G.lane & (L - 1);
  G.base = G.lane - G.w;
  uint64_t st = 0, ev = 0;
#pragma unroll
  for (int b = 0; b < 64; b += L) {
    st |= 1ull << b;
    if (((b / L) & 1) == 0) ev |= ((L == 64 ? ~0ull : ((1ull << L) - 1)) << b);
  }
  G.start = st;
  G.top = st << (L - 1);
  G.even = ev;
  G.odd = ~ev;
  return G;
}

// bit `pos` of a wavefront mask
MPD bool mask_bit(uint64_t m, int pos) { return ((m >> pos) & 1ull) != 0; }

// This lane's group's L bits of a wavefront mask, as the low bits of a word.
template <int L>
MPD uint32_t group_bits(const Group<L>& G, uint64_t m) {
  return (uint32_t)((m >> G.base) & ((1ull << L) - 1));
}

// Carries into every limb of a per-group addition whose limbs generate (gen) or propagate
// (prop, disjoint from gen) a carry, with carry-in `cin` at the first lanes: bit k of the result
// is the carry into lane k.  Writing a_k for the carry lane k - 1 generates (or the carry-in),
// the carries c satisfy c_k = a_k | (prop_{k-1} & c_{k-1}), which is what the integer sum
// a + prop delivers: c = (a + prop) ^ prop.  Even and odd groups are added separately, so that
// no carry leaves a group.
template <int L>
MPD uint64_t group_carries(const Group<L>& G, uint64_t gen, uint64_t prop, uint64_t cin) {
  const uint64_t a = ((gen << 1) & ~G.start) | cin;
  const uint64_t pe = prop & G.even, po = prop & G.odd;
  const uint64_t ce = ((a & G.even) + pe) ^ pe;
  const uint64_t co = ((a & G.odd) + po) ^ po;
  return (ce & G.even) | (co & G.odd);
}

// The limb of lane base + i of the group (0 outside 0 <= i < L).
template <int L>
MPD uint32_t group_limb(const Group<L>& G, uint32_t v, int i) {
  const int src = G.base + min(max(i, 0), L - 1);
  const uint32_t t = (uint32_t)__shfl((int)v, src, 64);
  return (i >= 0 && i < L) ? t : 0u;
}

// The value of the next lane up / down within the lane's row of 16 (DPP row shifts; 0 past the
// row's end).  Groups of 4, 8 or 16 lanes never straddle a row, so within a group these are the
// limbs w + 1 and w - 1.
MPD uint32_t group_limb_above(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x101, 0xf, 0xf, true);  // row_shl:1
}
MPD uint32_t group_limb_below(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, true);  // row_shr:1
}

// DPP row shifts by a constant: the value of the lane k places up / down in the lane's row of 16
// (0 past the row's ends).
template <int K>
MPD uint32_t row_up(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x100 + K, 0xf, 0xf, true);  // row_shl:K
}
template <int K>
MPD uint32_t row_down(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x110 + K, 0xf, 0xf, true);  // row_shr:K
}

// The value of lane w + s of the group (0 <= s < 16; a lane past the row's end gives 0, a lane
// of the next group in the row its own value, which callers mask).  Every stage is executed by
// every lane; the bits of s select.
template <int L>
MPD uint32_t group_shift_down(uint32_t v, int s) {
  uint32_t t = row_up<1>(v);
  v = (s & 1) ? t : v;
  if constexpr (L > 2) {
    t = row_up<2>(v);
    v = (s & 2) ? t : v;
  }
  if constexpr (L > 4) {
    t = row_up<4>(v);
    v = (s & 4) ? t : v;
  }
  if constexpr (L > 8) {
    t = row_up<8>(v);
    v = (s & 8) ? t : v;
  }
  return v;
}

// OR of the values of lanes w .. w + L - 1 (in lane w = 0 of a group: the group's OR).
template <int L>
MPD uint32_t group_or_down(uint32_t v) {
  v |= row_up<1>(v);
  if constexpr (L > 2) v |= row_up<2>(v);
  if constexpr (L > 4) v |= row_up<4>(v);
  if constexpr (L > 8) v |= row_up<8>(v);
  return v;
}

// The value of the group's top lane (limb L - 1), in every lane of the group (every lane is a
// valid source, so the old value passed is never kept).
template <int L>
MPD uint32_t group_top(uint32_t v) {
  if constexpr (L == 4) {
    return (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, 0xFF, 0xf, 0xf, false);  // quad_perm 3,3,3,3
  } else if constexpr (L == 8) {
    const uint32_t t7 = (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x157, 0xf, 0xf, false);  // row_newbcast:7
    const uint32_t t15 = (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x15F, 0xf, 0xf, false);
    return (threadIdx.x & 8u) ? t15 : t7;
  } else {
    return (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x15F, 0xf, 0xf, false);  // row_newbcast:15
  }
}

// (am, ae, as) <- RN((am, ae, as) + (bm, be, bs)) for every group of the wavefront: the general
// algorithm (every carry resolved, negative differences, any cancellation).
template <int L>
MPD void group_add_exact(const Group<L>& G, uint32_t& am, int32_t& ae, uint32_t& as,
                         uint32_t bm, int32_t be, uint32_t bs, uint32_t& st) {
  const int w = G.w;
  const bool az = ae == kZeroE, bz = be == kZeroE;
  const bool sw = be > ae;  // a zero's exponent is below every other one
  const uint32_t Xm = sw ? bm : am, Ym = sw ? am : bm;
  const int32_t Xe = sw ? be : ae, Ye = sw ? ae : be;
  const uint32_t Xs = sw ? bs : as, Ys = sw ? as : bs;
  const uint32_t d = min((uint32_t)(Xe - Ye), (uint32_t)(32 * L + 2));
  const int q = (int)(d >> 5);
  const uint32_t r = d & 31u;

  // Y >> d, with one guard limb below limb 0 and the bits shifted out below it as a sticky bit.
  // Limbs w + q - 1, w + q and w + q + 1 of Y: B = limb w + max(q - 1, 0), then its neighbours.
  const uint32_t B = group_shift_down<L>(Ym, max(q - 1, 0));
  const uint32_t b_up1 = row_up<1>(B), b_up2 = row_up<2>(B), b_dn1 = row_down<1>(B);
  const uint32_t v0 = ((unsigned)(w + q - 1) < (unsigned)L) ? (q ? B : b_dn1) : 0u;
  const uint32_t v1 = (w + q < L) ? (q ? b_up1 : B) : 0u;
  const uint32_t v2 = (w + q + 1 < L) ? (q ? b_up2 : b_up1) : 0u;
  const uint32_t ysh = fshr(v2, v1, r);          // limb w of the shifted Y
  uint32_t gd = fshr(v1, v0, r);                 // its guard limb (used in lane w = 0)
  const uint32_t lost = (w + 2 <= q) ? Ym : ((w + 1 == q && r != 0u) ? (Ym << (32u - r)) : 0u);
  gd |= group_or_down<L>(lost) ? 1u : 0u;

  // X + Y or X - Y (the complement of Y plus one at the guard limb)
  const bool sub = Xs != Ys;
  const uint32_t mask = sub ? ~0u : 0u;
  const uint32_t y2 = ysh ^ mask, g2 = gd ^ mask;
  uint32_t rg = g2 + (sub ? 1u : 0u);            // guard limb of the sum (X's guard is 0)
  const bool cg = sub && g2 == ~0u;              // its carry into limb 0
  const uint32_t s0 = Xm + y2;
  const uint32_t gen = s0 < Xm ? 1u : 0u;
  const uint32_t gen_below = row_down<1>(gen);
  const uint32_t cin = (w == 0) ? (cg ? 1u : 0u) : gen_below;
  uint32_t rm;
  bool co;
  if (__ballot(cin != 0u && s0 == ~0u) == 0ull) {  // no carry moves past the limb it enters
    rm = s0 + cin;
    co = mask_bit(__ballot(w == L - 1 && gen != 0u), G.base + L - 1);
  } else {
    const uint64_t gm = __ballot(gen != 0u), pm = __ballot(s0 == ~0u);
    const uint64_t c = group_carries(G, gm, pm, __ballot(w == 0 && cg));
    rm = s0 + (mask_bit(c, G.lane) ? 1u : 0u);
    co = mask_bit((gm | (pm & c)) & G.top, G.base + L - 1);
  }
  const bool neg = sub && !co;  // |Y| > |X|: only when d == 0
  const bool ovf = !sub && co;  // the sum carried out of the top limb

  if (__ballot(neg) != 0ull) {  // negate the groups' (L + 1)-limb results (rare)
    const uint64_t p2 = __ballot(rm == 0u);
    const uint64_t c2 = group_carries(G, 0ull, p2, __ballot(w == 0 && rg == 0u));
    const uint32_t nrm = ~rm + (mask_bit(c2, G.lane) ? 1u : 0u);
    const uint32_t nrg = ~rg + 1u;
    rm = neg ? nrm : rm;
    rg = neg ? nrg : rg;
  }
  const uint32_t s = Xs ^ (neg ? 1u : 0u);
  int32_t e = Xe;

  // normalise: the carried-out sum moves right one bit; a sum whose top bit is clear moves left
  const uint64_t t31 = __ballot(w == L - 1 && (rm >> 31) != 0u);
  const uint64_t t30 = __ballot(w == L - 1 && (rm >> 30) == 1u);
  const bool lz0 = mask_bit(t31, G.base + L - 1), lz1 = mask_bit(t30, G.base + L - 1);
  const uint32_t up = group_limb_above(rm);  // limb w + 1 (this group's only for w < L - 1)
  const uint32_t dl = group_limb_below(rm);  // limb w - 1 (this group's only for w > 0)
  const bool l1 = !ovf && !lz0 && lz1;
  const uint32_t m_ovf = fshr(w == L - 1 ? 1u : up, rm, 1);
  const uint32_t g_ovf = fshr(rm, rg, 1) | (rg & 1u);
  const uint32_t m_l1 = fshr(rm, w == 0 ? rg : dl, 31);
  uint32_t nm = ovf ? m_ovf : (l1 ? m_l1 : rm);
  uint32_t ng = ovf ? g_ovf : (l1 ? (rg << 1) : rg);
  e += ovf ? 1 : (l1 ? -1 : 0);
  bool zres = false;
  const bool rare = !ovf && !lz0 && !lz1;  // a cancellation of two or more bits (d <= 1), or 0
  if (__ballot(rare) != 0ull) {
    const uint32_t nz = group_bits(G, __ballot(rm != 0u));
    const uint32_t guard = (uint32_t)__shfl((int)rg, G.base, 64);
    const int hb = nz ? 31 - (int)__clz(nz) : -1;  // highest non-zero limb
    const uint32_t hv = (uint32_t)__shfl((int)rm, G.base + max(hb, 0), 64);
    const bool allz = hb < 0 && guard == 0u;
    const uint32_t lz = hb >= 0 ? 32u * (uint32_t)(L - 1 - hb) + (uint32_t)__clz(hv)
                                : 32u * (uint32_t)L + (uint32_t)__clz(guard | 1u);
    const int q2 = (int)(lz >> 5);
    const uint32_t r2 = lz & 31u;
    // extended limbs: index 0 the guard, index i + 1 limb i; new index j takes j - q2 and
    // j - q2 - 1 shifted left by r2
    const int ja = w + 1 - q2, jb = w - q2;
    const uint32_t la = group_limb(G, rm, ja - 1), lb = group_limb(G, rm, jb - 1);
    const uint32_t ea = ja == 0 ? guard : (ja > 0 ? la : 0u);
    const uint32_t eb = jb == 0 ? guard : (jb > 0 ? lb : 0u);
    const uint32_t gn = q2 == 0 ? (guard << r2) : 0u;
    if (rare) {
      nm = r2 ? fshr(ea, eb, 32u - r2) : ea;
      ng = gn;
      e -= (int32_t)lz;
      zres = allz;
    }
  }

  // round to nearest, ties to even: guard bit 31 is the round bit, the rest of it the sticky
  // (lane 0's guard and limb); the increment moves past limb 0 only when that limb is all ones
  const bool inc = w == 0 && (ng >> 31) != 0u && ((ng & 0x7fffffffu) != 0u || (nm & 1u) != 0u);
  bool cout = false;
  if (__ballot(inc && nm == ~0u) == 0ull) {
    nm += inc ? 1u : 0u;
  } else {
    const uint64_t p3 = __ballot(nm == ~0u);
    const uint64_t c3 = group_carries(G, 0ull, p3, __ballot(inc));
    nm += mask_bit(c3, G.lane) ? 1u : 0u;
    cout = mask_bit(p3 & c3 & G.top, G.base + L - 1);  // 1.11..1 rounded up to 10..0
    nm = (cout && w == L - 1) ? 0x80000000u : nm;
  }
  e += cout ? 1 : 0;

  const bool bothz = az && bz;
  const bool range = !bothz && !zres && (e > kEmax || e < kEmin);
  st |= range ? kStRange : 0u;
  const bool zr = bothz || zres || range;
  am = zr ? 0u : nm;
  ae = zr ? kZeroE : e;
  as = bothz ? (as & bs) : (zres ? 0u : s);  // x - x is +0; (-0) + (-0) is -0
}

// The common case without a branch or a ballot, for the latency of a chain of additions: every
// carry stops in the limb it enters, the difference is not negative, at most one bit cancels,
// and rounding's increment stays in limb 0.  Returns false, leaving the operands as they were,
// when some group of the wavefront is not in that case; the result is otherwise the one
// group_add_exact forms.
template <int L>
MPD bool group_add_fast(const Group<L>& G, uint32_t& am, int32_t& ae, uint32_t& as,
                        uint32_t bm, int32_t be, uint32_t bs, uint32_t& st) {
  const int w = G.w;
  const bool az = ae == kZeroE, bz = be == kZeroE;
  const bool sw = be > ae;
  const uint32_t Xm = sw ? bm : am, Ym = sw ? am : bm;
  const int32_t Xe = sw ? be : ae, Ye = sw ? ae : be;
  const uint32_t Xs = sw ? bs : as, Ys = sw ? as : bs;
  const uint32_t d = min((uint32_t)(Xe - Ye), (uint32_t)(32 * L + 2));
  const int q = (int)(d >> 5);
  const uint32_t r = d & 31u;
  const uint32_t B = group_shift_down<L>(Ym, max(q - 1, 0));
  const uint32_t b_up1 = row_up<1>(B), b_up2 = row_up<2>(B), b_dn1 = row_down<1>(B);
  const uint32_t v0 = ((unsigned)(w + q - 1) < (unsigned)L) ? (q ? B : b_dn1) : 0u;
  const uint32_t v1 = (w + q < L) ? (q ? b_up1 : B) : 0u;
  const uint32_t v2 = (w + q + 1 < L) ? (q ? b_up2 : b_up1) : 0u;
  const uint32_t ysh = fshr(v2, v1, r);
  uint32_t gd = fshr(v1, v0, r);
  const uint32_t lost = (w + 2 <= q) ? Ym : ((w + 1 == q && r != 0u) ? (Ym << (32u - r)) : 0u);
  gd |= group_or_down<L>(lost) ? 1u : 0u;
  // a zero Y adds nothing whatever its sign (X + (+-0) = X)
  const bool sub = Xs != Ys && Ye != kZeroE;
  const uint32_t mask = sub ? ~0u : 0u;
  const uint32_t y2 = ysh ^ mask, g2 = gd ^ mask;
  const uint32_t rg = g2 + (sub ? 1u : 0u);
  const bool cg = sub && g2 == ~0u;
  const uint32_t s0 = Xm + y2;
  const uint32_t gen = s0 < Xm ? 1u : 0u;
  const uint32_t gen_below = row_down<1>(gen);
  const uint32_t cin = (w == 0) ? (cg ? 1u : 0u) : gen_below;
  const bool chain = cin != 0u && s0 == ~0u;
  const uint32_t rm = s0 + cin;
  // the top limb's two leading bits and its carry out, in one broadcast
  const uint32_t top = group_top<L>((rm & 0xC0000000u) | gen);
  const bool co = (top & 1u) != 0u;
  const bool neg = sub && !co;
  const bool ovf = !sub && co;
  const bool lz0 = (top >> 31) != 0u, lz1 = (top >> 30) == 1u;
  const uint32_t up = group_limb_above(rm);
  const uint32_t dl = group_limb_below(rm);
  const bool l1 = !ovf && !lz0 && lz1;
  const bool bothz = az && bz;
  const bool rare = !ovf && !lz0 && !lz1 && !bothz;
  const uint32_t m_ovf = fshr(w == L - 1 ? 1u : up, rm, 1);
  const uint32_t g_ovf = fshr(rm, rg, 1) | (rg & 1u);
  const uint32_t m_l1 = fshr(rm, w == 0 ? rg : dl, 31);
  uint32_t nm = ovf ? m_ovf : (l1 ? m_l1 : rm);
  const uint32_t ng = ovf ? g_ovf : (l1 ? (rg << 1) : rg);
  const int32_t e = Xe + (ovf ? 1 : (l1 ? -1 : 0));
  const bool inc = w == 0 && (ng >> 31) != 0u && ((ng & 0x7fffffffu) != 0u || (nm & 1u) != 0u);
  if (__ballot(chain || neg || rare || (inc && nm == ~0u)) != 0ull) return false;
  nm += inc ? 1u : 0u;
  const bool range = !bothz && (e > kEmax || e < kEmin);
  st |= range ? kStRange : 0u;
  const bool zr = bothz || range;
  am = zr ? 0u : nm;
  ae = zr ? kZeroE : e;
  as = bothz ? (as & bs) : Xs;
  return true;
}

// (am, ae, as) <- RN((am, ae, as) + (bm, be, bs)) for every group of the wavefront.
template <int L>
MPD void group_add_rn(const Group<L>& G, uint32_t& am, int32_t& ae, uint32_t& as,
                      uint32_t bm, int32_t be, uint32_t bs, uint32_t& st) {
  if (!group_add_fast<L>(G, am, ae, as, bm, be, bs, st)) group_add_exact<L>(G, am, ae, as, bm, be, bs, st);
}

}  // namespace mp
