// Vector, inner-product and scalar kernels of the BiCG and GPBiCG drivers (Kouya, Fig. 5, with
// K = I), and the plain vector entry points built on them.
//
// Scalars live in a small structure-of-arrays MP array (ld = kNumScalars), so every kernel reads
// them by slot.  A control block carries the iteration count and a done flag: once an epilogue
// sets done, every later kernel of the solve returns at once, so a captured iteration graph can
// be replayed past the stopping point without changing any result.  Every vector update is one
// RN per binary operation, evaluated in the order the oracle (and the listing) writes it.
#pragma once
#include "mp_core.hpp"
#include "mp_exact.hpp"
#include "mp_scalar.hpp"

namespace mp {

constexpr int kNumScalars = 32;
enum Slot {
  S_RHO = 0, S_RHO_OLD, S_ALPHA, S_BETA, S_SIGMA, S_Q, S_THR, S_CREL, S_CABS, S_ZETA, S_ETA,
  S_ALPHA_OLD, S_ZETA_OLD, S_MU1, S_MU2, S_MU3, S_MU4, S_MU5, S_TAU, S_DEN, S_Q0, S_NRM0,
  S_RHO_NEXT, S_RESULT
};

// solver outcomes (the values of the C header's MP_CONVERGED ...)
constexpr int kConverged = 0, kNotConverged = 1, kBreakRho = 2, kBreakSigma = 3, kBreakZeta = 4,
              kBreakTau = 5;

struct Ctl {
  int32_t done;
  int32_t status;
  int32_t iters;  // completed iterations
  int32_t maxit;
  uint32_t flags;
  int32_t hist_len;
  int32_t pad[2];
};

// Scalar slots of one solve: slot k of limb plane q at limb[q * ld + k].  A batch of solves
// keeps kNumScalars slots per solve side by side (ld = kNumScalars * number of solves).
struct Scalars {
  uint32_t* limb;
  int32_t* hdr;
  int64_t ld;
  __host__ __device__ Scalars at(int64_t pair) const {
    Scalars r;
    r.limb = limb + pair * kNumScalars;
    r.hdr = hdr + pair * kNumScalars;
    r.ld = ld;
    return r;
  }
};

// Several independent solves in one set of launches: every solve ("pair": a system and one
// right-hand side) owns a segment of the concatenated vectors that starts on a kTile boundary,
// so a tile (and every wavefront or block inside it) belongs to one solve.
constexpr int kTile = 512;
struct BatchMap {
  const int32_t* pair_of_tile;   // nullptr: a single solve
  const int32_t* tiles_of_pair;  // tiles in each solve's segment
  const int32_t* first_tile;     // first tile of each solve's segment
  int32_t* ndone;                // incremented once per solve that finishes
};

struct VecRef {
  uint32_t* limb;
  int32_t* hdr;
  int64_t ld;
};

template <int L>
MPD Num<L> sload(const Scalars& S, int slot) {
  Num<L> r;
  load<L>(r, S.limb, S.hdr, S.ld, slot);
  return r;
}

// Scalar read that sees values other blocks of the same launch stored with store_dev.
template <int L>
MPD Num<L> sload_dev(const Scalars& S, int slot) {
  Num<L> r;
  load_dev<L>(r, S.limb, S.hdr, S.ld, slot);
  return r;
}

template <int L>
MPD void sstore(const Scalars& S, int slot, const Num<L>& v) {
  store<L>(v, S.limb, S.hdr, S.ld, slot);
}

template <int L>
MPD Num<L> vload(const VecRef& v, int64_t i) {
  Num<L> r;
  load<L>(r, v.limb, v.hdr, v.ld, i);
  return r;
}

template <int L>
MPD void vstore(const VecRef& v, int64_t i, const Num<L>& x) {
  store<L>(x, v.limb, v.hdr, v.ld, i);
}

MPD bool solve_done(const Ctl* ctl) { return ctl && *(volatile const int32_t*)&ctl->done; }

MPD void finish(Ctl* ctl, int status) {
  ctl->status = status;
  ctl->done = 1;
}

// ------------------------------------------------------------------------------------------
// Driver epilogues, run by one thread after the inner products of a step are known (they read
// the scalars with device-coherent loads: other blocks of the launch stored some of them).
// ------------------------------------------------------------------------------------------
enum Epi {
  EPI_NONE = 0,
  EPI_SETUP,        // q0 = (r,r), rho = (rt,r): nrm0, thr = c_rel*nrm0 + c_abs, test r_0
  EPI_BICG_CONV,    // q = (r,r), rho' = (rt,r): stopping test, then beta = rho'/rho
  EPI_GP_CONV,      // q = (r,r), rho' = (rt,r): stopping test, zeta = 0 exit, beta
  EPI_CONV,         // q = (r,r): stopping test only (preconditioned BiCG)
  EPI_PRHO,         // rho' = (rt, K^{-1} r): zero exit, then beta = rho'/rho after the first
};

// Step prologues: scalars a step needs that follow from the inner products of the launch before
// it, formed at the start of the step by the first wavefront of every block (every block forms
// the same bits, so no block waits for another).
enum Pro {
  PRO_BICG_ALPHA = 1,  // sigma = (pt, z): alpha = rho / sigma (sigma = 0: breakdown)
  PRO_GP_ALPHA,        // den = (rt, q): alpha = rho / den (den = 0: breakdown)
  PRO_GP_ZETA,         // mu1..mu5: zeta, eta (and tau after the first iteration)
  PRO_STAB_OMEGA,      // BiCGSTAB: (t, s), (t, t): omega = (t, s) / (t, t), or 0 when (t, t) = 0
};

// Scalar operations of the prologues and epilogues, returning their status bits with the value.
// They are inlined into the (out-of-line) prologue and epilogue: a nested out-of-line call would
// save and restore the callee-saved registers through scratch memory on every operation.
template <int L>
struct NumSt {
  Num<L> v;
  uint32_t st;
};

template <int L>
MPD NumSt<L> s_mul(Num<L> a, Num<L> b) {
  NumSt<L> r;
  r.st = 0;
  r.v = mul_rn<L>(a, b, r.st);
  return r;
}

template <int L>
MPD NumSt<L> s_div(Num<L> a, Num<L> b) {
  NumSt<L> r;
  r.st = 0;
  r.v = div_rn<L>(a, b, r.st);
  return r;
}

template <int L>
MPD NumSt<L> s_add(Num<L> a, Num<L> b) {
  NumSt<L> r;
  r.st = 0;
  r.v = add_rn<L>(a, b, r.st);
  return r;
}

template <int L>
MPD NumSt<L> s_sub(Num<L> a, Num<L> b) {
  NumSt<L> r;
  r.st = 0;
  r.v = sub_rn<L>(a, b, r.st);
  return r;
}

template <int L>
MPD NumSt<L> s_sqrt(Num<L> a) {
  NumSt<L> r;
  r.st = 0;
  r.v = sqrt_rn<L>(a, r.st);
  return r;
}

template <int L>
MPD bool s_sqrt_le(Num<L> q, Num<L> thr) {
  return sqrt_le<L>(q, thr);
}

// A value held by lane `src`, to every lane.
template <int L>
MPD Num<L> shfl_num(const Num<L>& v, int src) {
  Num<L> r;
#pragma unroll
  for (int k = 0; k < L; ++k) r.m[k] = __shfl(v.m[k], src);
  r.e = __shfl(v.e, src);
  r.s = __shfl(v.s, src);
  return r;
}

// Scalars seen by an epilogue: read from a copy of the solve's slots in LDS (taken while the
// launch's inner products were rounded), written to the copy and to the slots.
template <int L>
struct ScalarView {
  uint32_t* cl;  // LDS copy: limb k of slot s at cl[s * L + k]
  int32_t* ch;   // LDS copy: header of slot s at ch[s]
  Scalars S;     // the slots in global memory
  MPD Num<L> get(int slot) const {
    Num<L> r;
    const int32_t h = ch[slot];
    r.e = h >> 1;
    r.s = (uint32_t)h & 1u;
#pragma unroll
    for (int k = 0; k < L; ++k) r.m[k] = cl[slot * L + k];
    return r;
  }
  MPD void put(int slot, const Num<L>& v) const {
    ch[slot] = make_hdr(v.e, v.s);
#pragma unroll
    for (int k = 0; k < L; ++k) cl[slot * L + k] = v.m[k];
    sstore<L>(S, slot, v);
  }
};

// iters, maxit, hist_len: the solve's control values as they stood when the launch began.
// Run by every lane of one wavefront: the formulas' values are formed in every lane (the two
// divisions of GPBiCG's beta side by side in lanes 0 and 1); lane 0 writes.  Returns the status
// bits in every lane.
template <int L>
MPD void epilogue_body(int epi, const ScalarView<L>& sv, Ctl* ctl, int iters, int maxit, int hist_len,
                       const VecRef& hist, uint32_t& st) {
  if (!ctl || epi == EPI_NONE) return;
  const bool w0 = (threadIdx.x & 63) == 0;
  auto mul = [&](const Num<L>& x, const Num<L>& y) { const NumSt<L> r = s_mul<L>(x, y); st |= r.st; return r.v; };
  auto add = [&](const Num<L>& x, const Num<L>& y) { const NumSt<L> r = s_add<L>(x, y); st |= r.st; return r.v; };
  auto put = [&](int slot, const Num<L>& v) {
    if (w0) sv.put(slot, v);
  };
  auto done = [&](int outcome) {
    if (w0) finish(ctl, outcome);
  };
  switch (epi) {
    case EPI_SETUP: {
      const Num<L> q0 = sv.get(S_Q0);
      const Num<L> nrm0 = [&] { const NumSt<L> r = s_sqrt<L>(q0); st |= r.st; return r.v; }();
      const Num<L> thr = add(mul(sv.get(S_CREL), nrm0), sv.get(S_CABS));
      put(S_NRM0, nrm0);
      put(S_THR, thr);
      if (s_sqrt_le<L>(q0, thr)) {
        done(kConverged);
      } else if (maxit <= 0) {
        done(kNotConverged);
      } else if (is_zero(sv.get(S_RHO))) {
        done(kBreakRho);
      }
      break;
    }
    case EPI_BICG_CONV:
    case EPI_GP_CONV: {
      const Num<L> q = sv.get(S_Q);
      const int i = iters + 1;
      if (w0) {
        if (hist.limb && i - 1 < hist_len) vstore<L>(hist, i - 1, q);
        ctl->iters = i;
      }
      if (s_sqrt_le<L>(q, sv.get(S_THR))) {
        done(kConverged);
        break;
      }
      if (epi == EPI_GP_CONV && is_zero(sv.get(S_ZETA))) {
        done(kBreakZeta);
        break;
      }
      if (i >= maxit) {
        done(kNotConverged);
        break;
      }
      const Num<L> rho = sv.get(S_RHO);
      const Num<L> rho_next = sv.get(S_RHO_NEXT);
      if (is_zero(rho_next)) {
        put(S_RHO_OLD, rho);
        put(S_RHO, rho_next);
        done(kBreakRho);
        break;
      }
      const Num<L> alpha = sv.get(S_ALPHA), zeta = sv.get(S_ZETA);
      // lane 0: rho' / rho; lane 1 (GPBiCG): alpha / zeta
      const int lane = threadIdx.x & 63;
      NumSt<L> dq;
      dq.st = 0;
      set_zero(dq.v, 0);
      if (lane == 0 || (lane == 1 && epi == EPI_GP_CONV))
        dq = s_div<L>(lane == 0 ? rho_next : alpha, lane == 0 ? rho : zeta);
      const Num<L> d0 = shfl_num<L>(dq.v, 0);
      st |= __shfl(dq.st, 0);
      put(S_RHO_OLD, rho);
      put(S_RHO, rho_next);
      if (epi == EPI_BICG_CONV) {
        put(S_BETA, d0);
      } else {
        const Num<L> d1 = shfl_num<L>(dq.v, 1);
        st |= __shfl(dq.st, 1);
        put(S_ALPHA_OLD, alpha);
        put(S_ZETA_OLD, zeta);
        put(S_BETA, mul(d0, d1));
      }
      break;
    }
    case EPI_CONV: {
      const Num<L> q = sv.get(S_Q);
      const int i = iters + 1;
      if (w0) {
        if (hist.limb && i - 1 < hist_len) vstore<L>(hist, i - 1, q);
        ctl->iters = i;
      }
      if (s_sqrt_le<L>(q, sv.get(S_THR))) {
        done(kConverged);
      } else if (i >= maxit) {
        done(kNotConverged);
      }
      break;
    }
    case EPI_PRHO: {
      const Num<L> rho_next = sv.get(S_RHO_NEXT);
      if (is_zero(rho_next)) {
        done(kBreakRho);
        break;
      }
      if (iters == 0) {
        put(S_RHO, rho_next);
        break;
      }
      const Num<L> rho = sv.get(S_RHO);
      const int lane = threadIdx.x & 63;
      NumSt<L> dq;
      dq.st = 0;
      set_zero(dq.v, 0);
      if (lane == 0) dq = s_div<L>(rho_next, rho);
      const Num<L> beta = shfl_num<L>(dq.v, 0);
      st |= __shfl(dq.st, 0);
      put(S_RHO_OLD, rho);
      put(S_RHO, rho_next);
      put(S_BETA, beta);
      break;
    }
    default:
      break;
  }
}

// The epilogue, once per launch in one wavefront.  Only plain values cross the call, so no
// caller object needs an address.  The update steps of BiCG and GPBiCG inline it (which spares
// them the register saves of a call); the others call the out-of-line copy below, which keeps
// their registers.
template <int L>
MPD uint32_t epilogue_impl(int epi, uint32_t* c_limb, int32_t* c_hdr, uint32_t* s_limb, int32_t* s_hdr,
                           int64_t s_ld, Ctl* ctl, int iters, int maxit, int hist_len, uint32_t* h_limb,
                           int32_t* h_hdr, int64_t h_ld) {
  ScalarView<L> sv;
  sv.cl = c_limb;
  sv.ch = c_hdr;
  sv.S = Scalars{s_limb, s_hdr, s_ld};
  VecRef hist;
  hist.limb = h_limb;
  hist.hdr = h_hdr;
  hist.ld = h_ld;
  uint32_t st = 0;
  epilogue_body<L>(epi, sv, ctl, iters, maxit, hist_len, hist, st);
  return st;
}

template <int L>
__device__ __attribute__((noinline)) uint32_t epilogue(int epi, uint32_t* c_limb, int32_t* c_hdr,
                                                      uint32_t* s_limb, int32_t* s_hdr, int64_t s_ld,
                                                      Ctl* ctl, int iters, int maxit, int hist_len,
                                                      uint32_t* h_limb, int32_t* h_hdr, int64_t h_ld) {
  return epilogue_impl<L>(epi, c_limb, c_hdr, s_limb, s_hdr, s_ld, ctl, iters, maxit, hist_len, h_limb,
                          h_hdr, h_ld);
}

// A step prologue, by every lane of one wavefront (independent operations run on different
// lanes at once): results to out (limbs of result k at o_limb[k * L ...], header at o_hdr[k]):
// alpha; or zeta, eta, tau.  Returns, in every lane, the status bits of the operations the
// formulas use in bits 0..7, a breakdown (its solver outcome + 1, or 0) in bits 8..15, and bit
// 16 when tau was formed.
// Inputs in i_limb / i_hdr (k-th at i_limb[k * L ...], i_hdr[k]): sigma or den, rho; or mu1..mu5.
template <int L>
MPD uint32_t prologue_body(int kind, uint32_t* i_limb, int32_t* i_hdr, int iters, uint32_t* o_limb,
                           int32_t* o_hdr) {
  const int lane = threadIdx.x & 63;
  uint32_t st = 0, brk = 0, tau_ok = 0;
  auto in = [&](int k) {
    Num<L> r;
    const int32_t h = i_hdr[k];
    r.e = h >> 1;
    r.s = (uint32_t)h & 1u;
#pragma unroll
    for (int i = 0; i < L; ++i) r.m[i] = i_limb[k * L + i];
    return r;
  };
  auto put = [&](int k, const Num<L>& v) {
    o_hdr[k] = make_hdr(v.e, v.s);
#pragma unroll
    for (int i = 0; i < L; ++i) o_limb[k * L + i] = v.m[i];
  };
  Num<L> zero;
  set_zero(zero, 0);
  if (lane < 3) put(lane, zero);
  switch (kind) {
    case PRO_BICG_ALPHA:
    case PRO_GP_ALPHA: {
      const Num<L> den = in(0), rho = in(1);
      if (is_zero(den)) {
        brk = kBreakSigma + 1;
      } else if (lane == 0) {
        const NumSt<L> q = s_div<L>(rho, den);
        st = q.st;
        put(0, q.v);
      }
      break;
    }
    case PRO_STAB_OMEGA: {
      const Num<L> ts = in(0), tt = in(1);
      if (!is_zero(tt) && lane == 0) {  // (t, t) = 0: t = 0, omega stays +0
        const NumSt<L> q = s_div<L>(ts, tt);
        st = q.st;
        put(0, q.v);
      }
      break;
    }
    case PRO_GP_ZETA: {
      const Num<L> mu1 = in(0), mu2 = in(1), mu3 = in(2), mu4 = in(3), mu5 = in(4);
      if (iters == 0) {  // first iteration: zeta = mu2 / mu5, eta = 0
        if (is_zero(mu5)) {
          brk = kBreakTau + 1;
        } else if (lane == 0) {
          const NumSt<L> z = s_div<L>(mu2, mu5);
          st = z.st;
          put(0, z.v);
        }
        break;
      }
      // lanes 0..5: mu5 mu1, mu4 mu4 | mu1 mu2, mu3 mu4 | mu5 mu3, mu4 mu2
      const Num<L> fa = lane == 0 ? mu5 : lane == 1 ? mu4 : lane == 2 ? mu1 : lane == 3 ? mu3 : lane == 4 ? mu5 : mu4;
      const Num<L> fb = lane == 0 ? mu1 : lane == 1 ? mu4 : lane == 2 ? mu2 : lane == 3 ? mu4 : lane == 4 ? mu3 : mu2;
      NumSt<L> pr;
      pr.st = 0;
      set_zero(pr.v, 0);
      if (lane < 6) pr = s_mul<L>(fa, fb);
      // lanes 0..2: tau, zeta's numerator, eta's numerator
      const Num<L> da = shfl_num<L>(pr.v, 2 * lane < 64 ? 2 * lane : 0);
      const Num<L> db = shfl_num<L>(pr.v, 2 * lane + 1 < 64 ? 2 * lane + 1 : 0);
      NumSt<L> df;
      df.st = 0;
      set_zero(df.v, 0);
      if (lane < 3) df = s_sub<L>(da, db);
      const Num<L> tau = shfl_num<L>(df.v, 0);
      const uint32_t st_tau = __shfl(pr.st, 0) | __shfl(pr.st, 1) | __shfl(df.st, 0);
      if (is_zero(tau)) {
        brk = kBreakTau + 1;
        st = st_tau;
        break;
      }
      // lanes 0, 1: zeta = zn / tau, eta = en / tau
      const Num<L> num = shfl_num<L>(df.v, lane < 2 ? lane + 1 : 0);
      NumSt<L> qt;
      qt.st = 0;
      set_zero(qt.v, 0);
      if (lane < 2) qt = s_div<L>(num, tau);
      if (lane < 2) put(lane, qt.v);
      if (lane == 0) put(2, tau);
      uint32_t all = 0;
#pragma unroll
      for (int k = 0; k < 6; ++k) all |= __shfl(pr.st, k);
      all |= __shfl(df.st, 1) | __shfl(df.st, 2) | __shfl(qt.st, 0) | __shfl(qt.st, 1);
      st = st_tau | all;
      tau_ok = 1;
      break;
    }
    default:
      break;
  }
  st = __shfl(st, 0);
  return (st & 0xFFu) | (brk << 8) | (tau_ok << 16);
}

// The same out of line: the prologue of zeta and eta is large, and the update step that runs it
// holds many values in registers (inlined there, it would spill them).  The alpha prologues are
// inlined, which spares their callers the register saves of a call.
template <int L>
__device__ __attribute__((noinline)) uint32_t prologue(int kind, uint32_t* i_limb, int32_t* i_hdr,
                                                      int iters, uint32_t* o_limb, int32_t* o_hdr) {
  return prologue_body<L>(kind, i_limb, i_hdr, iters, o_limb, o_hdr);
}

template <int L>
MPD Num<L> lds_num(const uint32_t* limb, const int32_t* hdr, int k) {
  Num<L> r;
  const int32_t h = hdr[k];
  r.e = h >> 1;
  r.s = (uint32_t)h & 1u;
#pragma unroll
  for (int i = 0; i < L; ++i) r.m[i] = limb[k * L + i];
  return r;
}

// A step's prologue results, for the last block's epilogue (scalar slot of result k, the LDS
// copies) and the breakdown it found (solver outcome + 1, or 0).
struct ProOut {
  int n;
  int slot[3];
  const uint32_t* limb;
  const int32_t* hdr;
  int brk;
  int nclr;     // inner-product slots the prologue read (its launch's last block clears them)
  int clr[3];
  const int32_t* clo;  // their exponent ranges (LDS)
  const int32_t* chi;
};

// ------------------------------------------------------------------------------------------
// Exact inner products.
//
// Every inner product owns a slot: a ring of int64 carry-save digits in global memory, 64
// exponent bins and (per solve) a ticket.  Digit d of an exact sum has weight 2^(32 d - 2p) and
// lives at ring position d mod 2^ring_log2, so a digit's place never depends on the other
// products and no exponent anchor is needed before accumulating.  Any kernel that holds both
// operands adds to a slot one "pass" at a time: a block forms one exact product per thread,
// finds the pass's exponent range, sums the products digit by digit in LDS and adds the sums
// to the ring with integer atomics (replicated `reps` times, by block, to spread contention),
// and folds its exponent range into the bins with integer atomic min/max.  Integer addition is
// associative, so the ring's content does not depend on the order of blocks or passes.  The
// last block of a launch (ticket) reads the bins, checks that the whole range fits the ring,
// takes the digits out of the ring (clearing it for the next use) and rounds once.
// ------------------------------------------------------------------------------------------
constexpr int kDotMaxND = 5;
constexpr int kDotThreads = 256;
constexpr int kDotSlots = 8;
constexpr int kAnchorBins = 64;

struct DotWork {
  int32_t* anchor;   // [nslots][kAnchorBins][2]: emin, emax; (INT32_MAX, INT32_MIN) when empty
  int64_t* win;      // [nslots][reps][1 << ring_log2] carry-save digits, zero between uses
  uint32_t* ticket;  // per solve, ngroups + 1 counters kTicketStride words apart (zero between
                     // launches): the finished blocks of each group, then the finished groups
  int ring_log2;
  int reps;          // a power of two
  int ngroups;       // a power of two
  int nslots;
};

// Counters on separate cache lines: atomics on one line are serialised.
constexpr int kTicketStride = 32;

MPD int64_t* slot_ring(const DotWork& w, int64_t slot) {
  return w.win + slot * ((int64_t)w.reps << w.ring_log2);
}

MPD int32_t wave_min(int32_t v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = min(v, __shfl_xor(v, o));
  return v;
}

MPD int32_t wave_max(int32_t v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = max(v, __shfl_xor(v, o));
  return v;
}

// Windows of at most this many digits are summed without atomics (one digit per thread group).
constexpr int kPassDigits = 64;
// Most ring replicas a slot may have.
constexpr int kMaxReps = 8;

template <int L, int NT>
struct PassLds {
  int64_t dwin[kPassDigits];  // the window of a narrow pass
  // block-shared window of a wide pass, or of a rounding
  int64_t win[((2 * L + 1) * (NT + 1) + 1) / 2];
  int32_t red[2 * (NT / 64)];
};

// Digits of the block-shared window a wide pass or a rounding can hold in LDS.
template <int L, int NT>
constexpr int lds_window_digits() { return ((2 * L + 1) * (NT + 1) + 1) / 2; }

// a[k] <- a[(k + r) mod D] for every k (a lane-dependent rotation of a register array, in
// log2 D conditional steps, so that no register is indexed by a lane-varying value).
template <int D>
MPD void rotate_digits(uint32_t (&a)[D], int r) {
#pragma unroll
  for (int b = 1; b < D; b <<= 1) {
    if (r & b) {
      uint32_t t[D];
#pragma unroll
      for (int k = 0; k < D; ++k) t[k] = a[(k + b) % D];
#pragma unroll
      for (int k = 0; k < D; ++k) a[k] = t[k];
    }
  }
}

// Add sum_u x_u * y_u over the block's NT threads (ok == false: no product) to the ring of
// `slot`, exactly.  Called by every thread of the block (it synchronises the block).
template <int L, int NT>
MPD void pass_dot(PassLds<L, NT>& S, bool ok, int32_t hx, int32_t hy, const uint32_t (&x)[L],
                  const uint32_t (&y)[L], const DotWork& dw, int64_t slot) {
  static_assert(NT % 64 == 0, "whole wavefronts");
  constexpr int NW = NT / 64;
  constexpr int G = kPassDigits;
  static_assert(NT >= G, "a thread per window digit");
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const bool nz = ok && !hdr_is_zero(hx) && !hdr_is_zero(hy);
  const int32_t e = nz ? (hx >> 1) + (hy >> 1) : 0;
  int32_t lo = wave_min(nz ? e : INT32_MAX), hi = wave_max(nz ? e : INT32_MIN);
  if (t < G) S.dwin[t] = 0;
  if (lane == 0) {
    S.red[wv] = lo;
    S.red[NW + wv] = hi;
  }
  lds_barrier();
#pragma unroll
  for (int k = 0; k < NW; ++k) {
    lo = min(lo, S.red[k]);
    hi = max(hi, S.red[NW + k]);
  }
  if (hi < lo) {  // no non-zero product in this pass (the same for every thread)
    lds_barrier();
    return;
  }
  const int W = (int)(((int64_t)hi - (lo & ~31)) >> 5) + 2 * L + 2;
  const int64_t mask = ((int64_t)1 << dw.ring_log2) - 1;
  int64_t* const ring =
      slot_ring(dw, slot) + ((int64_t)(blockIdx.x & (unsigned)(dw.reps - 1)) << dw.ring_log2);
  uint32_t pr[2 * L], sp[2 * L + 1];
  uint32_t sg = 0;
  if (nz) {
    mul_full<L>(x, y, pr);
    sg = (uint32_t)(hx ^ hy) & 1u;
    shift_product<L>(pr, (uint32_t)e & 31u, sp);  // window digits are ring digits: bit e & 31
  }
  if (W <= G) {
    // narrow pass: the products' digits are added into a window of G digits in LDS.  Lane t adds
    // its 2L + 1 digits starting from digit t mod (2L + 1), so lanes whose products share an
    // exponent add to different digits at each step (at most ceil(64 / (2L + 1)) per address).
    const int64_t wbase = (int64_t)(lo & ~31);
    if (nz) {
      constexpr int D = 2 * L + 1;
      const int q = (int)(((int64_t)e - wbase) >> 5);
      const int r = t % D;
      rotate_digits<D>(sp, r);
#pragma unroll
      for (int k = 0; k < D; ++k) {
        const int j = (r + k >= D) ? r + k - D : r + k;
        const int64_t v = sg ? -(int64_t)sp[k] : (int64_t)sp[k];
        atomicAdd((unsigned long long*)&S.dwin[q + j], (unsigned long long)v);
      }
    }
    lds_barrier();
    if (t < W) {
      const int64_t v = S.dwin[t];
      if (v) atomicAdd((unsigned long long*)&ring[((wbase >> 5) + t) & mask], (unsigned long long)v);
    }
  } else {
    // wide pass: a block-shared window in LDS (integer atomics) whose non-zero digits go to the
    // ring.  A pass spanning more than the window leaves out the products below it: the
    // launch's window is then wider than its rounding accepts, which reports kStWindow.
    constexpr int C = lds_window_digits<L, NT>();
    const int Wc = min(W, C);
    const int64_t wbase = (W <= C) ? (int64_t)(lo & ~31) : (int64_t)(hi & ~31) - 32 * (int64_t)(C - 2 * L - 2);
    for (int w = t; w < Wc; w += NT) S.win[w] = 0;
    lds_barrier();
    if (nz && (int64_t)e >= wbase) {
      const int q = (int)(((int64_t)e - wbase) >> 5);
#pragma unroll
      for (int j = 0; j <= 2 * L; ++j) {
        if (sp[j]) {
          const int64_t v = sg ? -(int64_t)sp[j] : (int64_t)sp[j];
          atomicAdd((unsigned long long*)&S.win[q + j], (unsigned long long)v);
        }
      }
    }
    lds_barrier();
    for (int w = t; w < Wc; w += NT) {
      const int64_t v = S.win[w];
      if (v) atomicAdd((unsigned long long*)&ring[((wbase >> 5) + w) & mask], (unsigned long long)v);
    }
  }
  if (t == 0) {
    int32_t* a = dw.anchor + 2 * (slot * kAnchorBins + (blockIdx.x & (kAnchorBins - 1)));
    atomicMin(&a[0], lo);
    atomicMax(&a[1], hi);
  }
  lds_barrier();  // the LDS is free for the next pass
}

// The exponent range of slot `slot`'s products (its 64 bins reduced by one wavefront; every
// lane gets it); the bins are reset for the slot's next use.
MPD void ring_range(const DotWork& dw, int64_t slot, int32_t& lo, int32_t& hi) {
  int32_t* b = dw.anchor + 2 * (slot * kAnchorBins + (threadIdx.x & 63));
  lo = wave_min(ld_dev(b));
  hi = wave_max(ld_dev(b + 1));
  st_dev(b, (int32_t)INT32_MAX);
  st_dev(b + 1, (int32_t)INT32_MIN);
}

// Window of a slot with products in [lo, hi]: digit 0 of weight 2^(base - 2p), W digits.
template <int L>
MPD int ring_window(int32_t lo, int32_t hi) { return (int)(((int64_t)hi - (lo & ~31)) >> 5) + 2 * L + 2; }

// Digit w of the window starting at ring position s0, summed over the replicas, which are
// cleared.
MPD int64_t ring_take(const DotWork& dw, int64_t* ring, int s0, int w) {
  const int64_t at = (s0 + w) & ((1 << dw.ring_log2) - 1);
  // every exchange is issued before any result is used: one memory round trip in all
  uint64_t got[kMaxReps];
#pragma unroll
  for (int c = 0; c < kMaxReps; ++c)
    got[c] = (c < dw.reps) ? atomicExch((unsigned long long*)&ring[((int64_t)c << dw.ring_log2) + at], 0ull) : 0ull;
  int64_t v = 0;
#pragma unroll
  for (int c = 0; c < kMaxReps; ++c) v += (int64_t)got[c];
  return v;
}

// RN_p of a slot whose window has at most 63 digits, by one whole wavefront (one digit per
// lane; every lane gets the result); the digits are cleared.
template <int L>
MPD Num<L> ring_round_narrow(const DotWork& dw, int64_t slot, int32_t lo, int32_t hi, uint32_t& st) {
  const int lane = threadIdx.x & 63;
  const int64_t base = (int64_t)(lo & ~31);
  const int W = ring_window<L>(lo, hi);
  const int s0 = (int)((base >> 5) & ((1 << dw.ring_log2) - 1));
  const int64_t dg = (lane < W) ? ring_take(dw, slot_ring(dw, slot), s0, lane) : 0;
  return wave_round<L>(dg, base - 64 * L, st);
}

// Digit w of the window starting at ring position s0, summed over the replicas (read only:
// every load is issued before any result is used).
MPD int64_t ring_sum(const DotWork& dw, const int64_t* ring, int s0, int w) {
  const int64_t at = (s0 + w) & ((1 << dw.ring_log2) - 1);
  int64_t got[kMaxReps];
#pragma unroll
  for (int c = 0; c < kMaxReps; ++c)
    got[c] = (c < dw.reps) ? ld_dev(ring + ((int64_t)c << dw.ring_log2) + at) : 0;
  int64_t v = 0;
#pragma unroll
  for (int c = 0; c < kMaxReps; ++c) v += got[c];
  return v;
}

// RN_p of the inner products of N slots, read from their rings and bins without clearing them
// (the kernel that formed them has ended), by one whole wavefront: every lane gets out[k] and
// the slot's exponent range (rlo[k], rhi[k]), which ring_clear_range takes.  The bins of all
// slots are read at once, then the windows' digits; windows of more than 63 digits are summed
// into `lds` (capacity `cap`) and rounded by lane 0.  A window wider than the ring or `cap` sets
// kStWindow and gives +0.
template <int L, int N>
MPD void ring_peek(const DotWork& dw, int64_t slot0, const int (&rs)[N], Num<L> (&out)[N],
                   int32_t (&rlo)[N], int32_t (&rhi)[N], int64_t* lds, int cap, uint32_t& st) {
  const int lane = threadIdx.x & 63;
  const int R = 1 << dw.ring_log2, mask = R - 1;
  int32_t lo[N], hi[N];
#pragma unroll
  for (int k = 0; k < N; ++k) {
    const int32_t* b = dw.anchor + 2 * ((slot0 + rs[k]) * kAnchorBins + lane);
    lo[k] = ld_dev(b);
    hi[k] = ld_dev(b + 1);
  }
#pragma unroll
  for (int k = 0; k < N; ++k) {
    lo[k] = wave_min(lo[k]);
    hi[k] = wave_max(hi[k]);
    rlo[k] = lo[k];
    rhi[k] = hi[k];
  }
  // every slot's digit loads are issued before any is used: one memory round trip
  int64_t got[N][kMaxReps];
#pragma unroll
  for (int k = 0; k < N; ++k) {
    const int W = hi[k] >= lo[k] ? ring_window<L>(lo[k], hi[k]) : 0;
    const int64_t at = ((((int64_t)(lo[k] & ~31)) >> 5) + lane) & mask;
    const int64_t* ring = slot_ring(dw, slot0 + rs[k]);
    const bool use = W <= 63 && lane < W;
#pragma unroll
    for (int c = 0; c < kMaxReps; ++c)
      got[k][c] = (use && c < dw.reps) ? ld_dev(ring + ((int64_t)c << dw.ring_log2) + at) : 0;
  }
  int64_t dg[N];
#pragma unroll
  for (int k = 0; k < N; ++k) {
    dg[k] = 0;
#pragma unroll
    for (int c = 0; c < kMaxReps; ++c) dg[k] += got[k][c];
  }
#pragma unroll
  for (int k = 0; k < N; ++k) {
    set_zero(out[k], 0);
    if (hi[k] < lo[k]) continue;
    const int64_t base = (int64_t)(lo[k] & ~31);
    const int W = ring_window<L>(lo[k], hi[k]);
    if (W > R || W > cap) {
      st |= kStWindow;
    } else if (W <= 63) {
      out[k] = wave_round<L>(dg[k], base - 64 * L, st);
    } else {
      const int s0 = (int)((base >> 5) & mask);
      for (int w = lane; w < W; w += 64) lds[w] = ring_sum(dw, slot_ring(dw, slot0 + rs[k]), s0, w);
      __builtin_amdgcn_s_waitcnt(0xC07F);  // this wavefront's LDS writes are done
      uint32_t st1 = 0;
      Num<L> r;
      set_zero(r, 0);
      if (lane == 0) r = window_finalize<L>(lds, 1, W, base - 64 * L, st1);
      out[k] = shfl_num<L>(r, 0);
      st |= __shfl(st1, 0);
      __builtin_amdgcn_s_waitcnt(0xC07F);
    }
  }
}

// Clear slot `slot`, whose products span [lo, hi] (its window's digits in every replica, or
// the whole ring when the window is wider than the ring or `cap`), and reset its bins, by one
// whole wavefront: stores only.
template <int L>
MPD void ring_clear_range(const DotWork& dw, int64_t slot, int32_t lo, int32_t hi, int cap) {
  const int lane = threadIdx.x & 63;
  int32_t* b = dw.anchor + 2 * (slot * kAnchorBins + lane);
  st_dev(b, (int32_t)INT32_MAX);
  st_dev(b + 1, (int32_t)INT32_MIN);
  if (hi < lo) return;
  const int R = 1 << dw.ring_log2, mask = R - 1;
  int64_t* const ring = slot_ring(dw, slot);
  const int W = ring_window<L>(lo, hi);
  if (W > R || W > cap) {
    for (int64_t k = lane; k < ((int64_t)dw.reps << dw.ring_log2); k += 64) st_dev(ring + k, (int64_t)0);
    return;
  }
  const int s0 = (int)((((int64_t)(lo & ~31)) >> 5) & mask);
  for (int k = lane; k < W * dw.reps; k += 64) {
    const int c = k / W, w = k - c * W;
    st_dev(ring + ((int64_t)c << dw.ring_log2) + ((s0 + w) & mask), (int64_t)0);
  }
}

// RN_p of a slot with a wider window (W > 63), by the whole block; thread 0 gets the result.
// The digits are summed into `lds` (capacity `cap` digits) and rounded there by thread 0.  A
// window wider than the ring or than `cap` sets kStWindow and gives +0 (the whole ring is
// cleared).
template <int L, int NT>
MPD Num<L> ring_round_wide(const DotWork& dw, int64_t slot, int32_t lo, int32_t hi, int64_t* lds,
                           int cap, uint32_t& st) {
  const int t = threadIdx.x;
  const int R = 1 << dw.ring_log2, mask = R - 1;
  int64_t* const ring = slot_ring(dw, slot);
  const int64_t base = (int64_t)(lo & ~31);
  const int W = ring_window<L>(lo, hi);
  const int s0 = (int)((base >> 5) & mask);
  Num<L> res;
  set_zero(res, 0);
  if (W > R || W > cap) {
    if (t == 0) st |= kStWindow;
    for (int64_t k = t; k < ((int64_t)dw.reps << dw.ring_log2); k += NT) st_dev(ring + k, (int64_t)0);
    return res;
  }
  for (int w = t; w < W; w += NT) lds[w] = ring_take(dw, ring, s0, w);
  __syncthreads();
  if (t == 0) res = window_finalize<L>(lds, 1, W, base - 64 * L, st);
  __syncthreads();
  return res;
}

// Where the last block of a launch puts the launch's inner products, and what it runs next.
struct DotOut {
  int nd;
  int slot[kDotMaxND];
  VecRef out[kDotMaxND];  // result d goes to element 0 of out[d] (in a batch: solve 0's scalar
                          // slot, moved to each solve's own slots)
  int sslot[kDotMaxND];   // the scalar slot out[d] is (the epilogue reads it), or -1
  int epi;
  VecRef hist;
};

// After a block's passes: take the solve's ticket; the last of its nblocks blocks rounds every
// inner product of the launch (wavefront k takes products k, k + NT/64, ...), stores them, and
// runs the driver epilogue.  Blocks exchange data only through device-scope atomics and
// device-coherent loads and stores, ordered by waiting for this wavefront's memory operations,
// so no cache write-back or invalidate is needed.
// Whether the calling block (number idx of the solve's nblocks blocks in this launch) is the last
// to finish; called by one thread after the block's memory operations are complete.  Blocks
// count in ngroups groups (idx mod ngroups), the last of each group counts in the group
// counter, so no counter sees more than about nblocks / ngroups contending atomics.  Each
// counter is reset by the block that completes it.
MPD bool last_block(const DotWork& dw, int pair, unsigned idx, unsigned nblocks) {
  const unsigned G = (unsigned)dw.ngroups;
  uint32_t* tk = dw.ticket + (int64_t)pair * (G + 1) * kTicketStride;
  const unsigned g = idx & (G - 1);
  const unsigned gsize = (nblocks - g + G - 1) / G;
  if (atomicAdd(&tk[g * kTicketStride], 1u) != gsize - 1) return false;
  st_dev(&tk[g * kTicketStride], 0u);
  const unsigned ng = min(G, nblocks);
  if (atomicAdd(&tk[G * kTicketStride], 1u) != ng - 1) return false;
  st_dev(&tk[G * kTicketStride], 0u);
  return true;
}

// EPI: whether the kernel can run a driver epilogue (kernels that never do are compiled without
// it, and keep their registers).
template <int L, int NT, bool EPI = true, bool EPI_INLINE = false>
MPD void dots_finish(const DotWork& dw, const DotOut& O, int pair, bool batched, unsigned idx,
                     unsigned nblocks, Ctl* ctl, const Scalars& S, int32_t* ndone, uint32_t* status,
                     uint32_t st, int64_t* lds, int cap, const ProOut* pro = nullptr) {
  constexpr int NW = NT / 64;
  static_assert(kNumScalars <= 32, "one lane per scalar slot, control values in lanes 32..34");
  __shared__ uint32_t s_last;
  __shared__ int32_t s_lo[kDotMaxND], s_hi[kDotMaxND];
  __shared__ uint32_t s_cl[kNumScalars * L];  // the solve's scalar slots, for the epilogue
  __shared__ int32_t s_ch[kNumScalars];
  __shared__ int32_t s_ctl[3];                // iters, maxit, hist_len
  const int t = threadIdx.x, wv = t >> 6, lane = t & 63;
  wait_memory();
  __syncthreads();
  if (t == 0) s_last = last_block(dw, pair, idx, nblocks) ? 1u : 0u;
  __syncthreads();
  if (!s_last) {
    if (st) atomicOr(status, st);
    return;
  }
  const int64_t slot0 = (int64_t)pair * kDotSlots;
  const int brk = pro ? pro->brk : 0;  // the step broke down: its products are not kept
  const bool epi_on = EPI && ctl != nullptr && O.epi != EPI_NONE && !brk;
  // the epilogue's inputs are requested first, so that they arrive while the rings are read
  uint32_t pm[L];
  int32_t ph = 0, pc = 0;
  if (epi_on && wv == 0) {
    if (lane < kNumScalars) {
      ph = ld_dev(S.hdr + lane);
#pragma unroll
      for (int k = 0; k < L; ++k) pm[k] = ld_dev(S.limb + (int64_t)k * S.ld + lane);
    } else if (lane == 32) {
      pc = ld_dev(&ctl->iters);
    } else if (lane == 33) {
      pc = ld_dev(&ctl->maxit);
    } else if (lane == 34) {
      pc = ld_dev(&ctl->hist_len);
    }
  }
  auto out_of = [&](const VecRef& o0) {
    VecRef o = o0;
    if (batched) {
      o.limb += (int64_t)pair * kNumScalars;
      o.hdr += (int64_t)pair * kNumScalars;
    }
    return o;
  };
  auto keep = [&](int dd, const Num<L>& res) {  // by one thread
    if (brk) return;
    const VecRef o = out_of(O.out[dd]);
    store_dev<L>(res, o.limb, o.hdr, o.ld, 0);
    const int ss = O.sslot[dd];
    if (ss >= 0) {
      s_ch[ss] = make_hdr(res.e, res.s);
#pragma unroll
      for (int k = 0; k < L; ++k) s_cl[ss * L + k] = res.m[k];
    }
  };
  // windows of at most 63 digits: one wavefront each
#pragma unroll
  for (int dd = 0; dd < kDotMaxND; ++dd) {
    if (dd < O.nd && wv == dd % NW) {
      int32_t lo, hi;
      ring_range(dw, slot0 + O.slot[dd], lo, hi);
      if (hi < lo || ring_window<L>(lo, hi) <= 63) {
        Num<L> res;
        if (hi < lo) set_zero(res, 0);
        else res = ring_round_narrow<L>(dw, slot0 + O.slot[dd], lo, hi, st);
        if (lane == 0) keep(dd, res);
      }
      if (lane == 0) {
        s_lo[dd] = lo;
        s_hi[dd] = hi;
      }
    }
  }
  __syncthreads();
  // wider windows: the whole block, one at a time
#pragma unroll
  for (int dd = 0; dd < kDotMaxND; ++dd) {
    if (dd < O.nd) {
      const int32_t lo = s_lo[dd], hi = s_hi[dd];
      if (hi >= lo && ring_window<L>(lo, hi) > 63) {
        const Num<L> res = ring_round_wide<L, NT>(dw, slot0 + O.slot[dd], lo, hi, lds, cap, st);
        if (t == 0) keep(dd, res);
      }
    }
  }
  if (pro) {  // the rings the step's prologue read
#pragma unroll
    for (int k = 0; k < 3; ++k)
      if (k < pro->nclr && wv == k % NW)
        ring_clear_range<L>(dw, slot0 + pro->clr[k], pro->clo[k], pro->chi[k], cap);
  }
  if (ctl && st) atomicOr(&ctl->flags, st);
  if (brk && t == 0) {
    finish(ctl, brk - 1);
    if (ndone) atomicAdd(ndone, 1);
  }
  if (!epi_on) {
    if (st) atomicOr(status, st);
    return;
  }
  if (wv == 0) {  // the prefetched slots, except those this launch just formed
    bool fresh = false;
#pragma unroll
    for (int dd = 0; dd < kDotMaxND; ++dd) fresh |= dd < O.nd && O.sslot[dd] == lane;
    if (pro) {
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        if (k < pro->n && pro->slot[k] == lane) {
          fresh = true;
          s_ch[lane] = pro->hdr[k];
#pragma unroll
          for (int i = 0; i < L; ++i) s_cl[lane * L + i] = pro->limb[k * L + i];
        }
      }
    }
    if (lane < kNumScalars && !fresh) {
      s_ch[lane] = ph;
#pragma unroll
      for (int k = 0; k < L; ++k) s_cl[lane * L + k] = pm[k];
    } else if (lane >= 32 && lane < 35) {
      s_ctl[lane - 32] = pc;
    }
  }
  lds_barrier();
  if constexpr (EPI) {
    if (wv == 0) {  // one wavefront
      const uint32_t st2 =
          EPI_INLINE ? epilogue_impl<L>(O.epi, s_cl, s_ch, S.limb, S.hdr, S.ld, ctl, s_ctl[0], s_ctl[1], s_ctl[2],
                                        O.hist.limb, O.hist.hdr, O.hist.ld)
                     : epilogue<L>(O.epi, s_cl, s_ch, S.limb, S.hdr, S.ld, ctl, s_ctl[0], s_ctl[1], s_ctl[2],
                                   O.hist.limb, O.hist.hdr, O.hist.ld);
      if (t == 0) {
        if (st2) atomicOr(&ctl->flags, st2);
        // the solve was running when the launch began (its blocks run only then)
        if (ndone && ctl->done) atomicAdd(ndone, 1);
        st |= st2;
      }
    }
  }
  if (st) atomicOr(status, st);
}

// Stand-alone inner products: blockIdx.y picks the product, blocks take 256-element passes.
struct DotArgs {
  int64_t n;
  VecRef x[kDotMaxND];
  VecRef y[kDotMaxND];
  DotOut o;
  DotWork w;
  Scalars S;
  Ctl* ctl;  // nullable
  uint32_t* status;
  BatchMap batch;  // batch.pair_of_tile == nullptr: one solve
};

template <int L>
__global__ void __launch_bounds__(kDotThreads) dot_kernel(DotArgs A) {
  __shared__ PassLds<L, kDotThreads> s;
  // batch: one block per 256 elements, so a block belongs to one solve
  const bool batched = A.batch.pair_of_tile != nullptr;
  const int pair = batched ? A.batch.pair_of_tile[((int64_t)blockIdx.x * kDotThreads) / kTile] : 0;
  Ctl* const ctl = A.ctl ? A.ctl + pair : nullptr;
  if (solve_done(ctl)) return;
  const int d = blockIdx.y;
  // operands picked by comparison: a dynamic index into the argument arrays would copy them
  // to scratch memory
  VecRef X = A.x[0], Y = A.y[0];
  int dslot = A.o.slot[0];
#pragma unroll
  for (int k = 1; k < kDotMaxND; ++k) {
    if (k == d) {
      X = A.x[k];
      Y = A.y[k];
      dslot = A.o.slot[k];
    }
  }
  const int64_t slot = (int64_t)pair * kDotSlots + dslot;
  const int32_t z = (int32_t)0x80000000;  // +0
  for (int64_t i0 = (int64_t)blockIdx.x * kDotThreads; i0 < A.n;
       i0 += (int64_t)gridDim.x * kDotThreads) {
    const int64_t i = i0 + threadIdx.x;
    const bool ok = i < A.n;
    const int32_t hx = ok ? X.hdr[i] : z, hy = ok ? Y.hdr[i] : z;
    uint32_t xm[L], ym[L];
#pragma unroll
    for (int q = 0; q < L; ++q) {
      xm[q] = ok ? X.limb[(int64_t)q * X.ld + i] : 0u;
      ym[q] = ok ? Y.limb[(int64_t)q * Y.ld + i] : 0u;
    }
    pass_dot<L, kDotThreads>(s, ok, hx, hy, xm, ym, A.w, slot);
  }
  // blocks of this solve: per product, all of them (one solve) or two per tile of its segment
  const unsigned per = batched ? 2u * (unsigned)A.batch.tiles_of_pair[pair] : gridDim.x;
  const unsigned bx = batched ? blockIdx.x - 2u * (unsigned)A.batch.first_tile[pair] : blockIdx.x;
  dots_finish<L, kDotThreads>(A.w, A.o, pair, batched, bx + per * blockIdx.y, per * gridDim.y, ctl,
                              A.S.at(pair), A.batch.ndone, A.status, 0u, s.win,
                              lds_window_digits<L, kDotThreads>());
}

// Reset anchors to empty.
static __global__ void dot_work_init_kernel(int32_t* anchor, int nslots) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (int64_t)nslots * kAnchorBins;
       i += (int64_t)gridDim.x * blockDim.x) {
    anchor[2 * i] = INT32_MAX;
    anchor[2 * i + 1] = INT32_MIN;
  }
}

// ------------------------------------------------------------------------------------------
// Element-wise kernels (one element per thread, grid-stride; those that end with inner products
// run block-uniform passes).
// ------------------------------------------------------------------------------------------
struct VecArgs {
  int64_t n;
  VecRef v[8];
  Scalars S;
  Ctl* ctl;
  uint32_t* status;
  BatchMap batch;   // batch: n is whole tiles and the grid has n / blockDim.x blocks
  // inner products the kernel forms from the vectors it writes (kernels that have them)
  DotWork dots;
  DotOut fd;
  int pro_sep;  // the step's prologue and epilogue run in launches of their own (batches)
};

// The solve a block works for: its control block, scalars, first inner-product slot and the
// number of blocks of the launch that work for it.
struct EwCtx {
  Ctl* ctl;
  Scalars S;
  int pair;
  int64_t abase;
  unsigned idx, nblocks;  // this block's number among the solve's blocks, and their count
};

MPD EwCtx ew_ctx(const VecArgs& A) {
  const bool batched = A.batch.pair_of_tile != nullptr;
  const int pair = batched ? A.batch.pair_of_tile[((int64_t)blockIdx.x * blockDim.x) / kTile] : 0;
  EwCtx c;
  c.ctl = A.ctl ? A.ctl + pair : nullptr;
  c.S = A.S.at(pair);
  c.pair = pair;
  c.abase = (int64_t)pair * kDotSlots;
  const unsigned per_tile = (unsigned)(kTile / (int)blockDim.x);
  c.nblocks = batched ? (unsigned)A.batch.tiles_of_pair[pair] * per_tile : gridDim.x;
  c.idx = batched ? blockIdx.x - (unsigned)A.batch.first_tile[pair] * per_tile : blockIdx.x;
  return c;
}

// A step prologue run at the start of an element-wise step: the first wavefront forms the
// values, the block reads them after a barrier.  Block 0 of the solve keeps them in the scalar slots (every
// block formed the same bits); the step's last block takes them from `pro`.
template <int L>
struct ProLds {
  uint32_t limb[3 * L];  // results
  int32_t hdr[3];
  uint32_t in_limb[5 * L];  // inputs
  int32_t in_hdr[5];
  int32_t rlo[3], rhi[3];   // exponent ranges of the rings read
  uint32_t word;
};

// A prologue by one wavefront: the inputs (inner products still in their rings, read with the
// SpMV's window limit, and scalar slots) into P.in_*, the results into P.limb / P.hdr; returns
// the prologue's word (status bits, breakdown, tau flag) in every lane.
template <int L>
MPD uint32_t prologue_wave(ProLds<L>& P, int kind, const Scalars& S, int iters, int64_t abase,
                           const DotWork& dw, int64_t* lds, int cap) {
  const int lane = threadIdx.x & 63;
  uint32_t st0 = 0;
  // the rings were filled by SpMV blocks (64 threads), whose passes hold at most this window
  const int pcap = min(cap, lds_window_digits<L, 64>());
  auto keep_in = [&](int k, const Num<L>& v) {
    if (lane == 0) {
      P.in_hdr[k] = make_hdr(v.e, v.s);
#pragma unroll
      for (int i = 0; i < L; ++i) P.in_limb[k * L + i] = v.m[i];
    }
  };
  if (kind == PRO_GP_ZETA) {  // mu1, mu3 from the t/s/y step; mu2, mu4, mu5 in rings 4, 6, 7
    const Num<L> mu1 = sload<L>(S, S_MU1), mu3 = sload<L>(S, S_MU3);  // requested first
    Num<L> mu[3];
    int32_t lo[3], hi[3];
    ring_peek<L, 3>(dw, abase, {4, 6, 7}, mu, lo, hi, lds, pcap, st0);
    if (lane == 0) {
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        P.rlo[k] = lo[k];
        P.rhi[k] = hi[k];
      }
    }
    keep_in(0, mu1);
    keep_in(1, mu[0]);
    keep_in(2, mu3);
    keep_in(3, mu[1]);
    keep_in(4, mu[2]);
  } else if (kind == PRO_STAB_OMEGA) {  // (t, s), (t, t) in rings 4 and 7
    Num<L> mu[2];
    int32_t lo[2], hi[2];
    ring_peek<L, 2>(dw, abase, {4, 7}, mu, lo, hi, lds, pcap, st0);
    if (lane == 0) {
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        P.rlo[k] = lo[k];
        P.rhi[k] = hi[k];
      }
    }
    keep_in(0, mu[0]);
    keep_in(1, mu[1]);
  } else {  // sigma or den in ring 0, rho
    const Num<L> rho = sload<L>(S, S_RHO);  // requested first
    Num<L> d[1];
    int32_t lo[1], hi[1];
    ring_peek<L, 1>(dw, abase, {0}, d, lo, hi, lds, pcap, st0);
    if (lane == 0) {
      P.rlo[0] = lo[0];
      P.rhi[0] = hi[0];
    }
    keep_in(0, d[0]);
    keep_in(1, rho);
  }
  __builtin_amdgcn_s_waitcnt(0xC07F);  // the inputs are in LDS for the whole wavefront
  const uint32_t w = (kind == PRO_GP_ZETA) ? prologue<L>(kind, P.in_limb, P.in_hdr, iters, P.limb, P.hdr)
                                            : prologue_body<L>(kind, P.in_limb, P.in_hdr, iters, P.limb, P.hdr);
  __builtin_amdgcn_s_waitcnt(0xC07F);  // and the results
  return w | (st0 & 0xFFu);
}

// The rings a prologue kind reads.
MPD int prologue_rings(int kind, int (&clr)[3]) {
  if (kind == PRO_GP_ZETA) {
    clr[0] = 4;
    clr[1] = 6;
    clr[2] = 7;
    return 3;
  }
  if (kind == PRO_STAB_OMEGA) {
    clr[0] = 4;
    clr[1] = 7;
    clr[2] = 0;
    return 2;
  }
  clr[0] = clr[1] = clr[2] = 0;
  return 1;
}

// The step prologue of an element-wise step.  sep: it ran in its own launch (prologue_kernel,
// for batches: one wavefront per solve instead of one per block), which kept the results in the
// scalar slots, finished a solve that broke down and cleared the rings.
template <int L>
MPD ProOut run_prologue(ProLds<L>& P, int kind, const EwCtx& c, const DotWork& dw, int64_t* lds,
                        int cap, int nres, const int (&slots)[3], uint32_t& st, bool sep = false) {
  ProOut o;
  o.nclr = 0;
  if (sep) {
    if (threadIdx.x == 0) {
      for (int k = 0; k < 3; ++k) {
        const Num<L> v = sload<L>(c.S, slots[k]);
        P.hdr[k] = make_hdr(v.e, v.s);
        for (int i = 0; i < L; ++i) P.limb[k * L + i] = v.m[i];
      }
    }
    __syncthreads();
    o.brk = 0;
    o.n = 0;
#pragma unroll
    for (int k = 0; k < 3; ++k) o.slot[k] = slots[k];
    o.limb = P.limb;
    o.hdr = P.hdr;
    return o;
  }
  if (threadIdx.x < 64) {  // one wavefront
    const uint32_t w = prologue_wave<L>(P, kind, c.S, c.ctl->iters, c.abase, dw, lds, cap);
    if (threadIdx.x == 0) P.word = w;
  }
  __syncthreads();
  const uint32_t w = P.word;
  if (threadIdx.x == 0) st |= w & 0xFFu;
  o.brk = (int)((w >> 8) & 0xFFu);
  o.n = (kind == PRO_GP_ZETA) ? (((w >> 16) & 1u) ? 3 : 2) : nres;
#pragma unroll
  for (int k = 0; k < 3; ++k) o.slot[k] = slots[k];
  o.limb = P.limb;
  o.hdr = P.hdr;
  o.nclr = prologue_rings(kind, o.clr);
  o.clo = P.rlo;
  o.chi = P.rhi;
  if (!o.brk && c.idx == 0 && threadIdx.x == 0) {
    for (int k = 0; k < o.n; ++k) sstore<L>(c.S, slots[k], lds_num<L>(P.limb, P.hdr, k));
  }
  return o;
}

// Step prologues of a batch in a launch of their own: one wavefront per solve forms the values,
// keeps them in the solve's scalar slots (or finishes a solve that broke down) and clears the
// rings it read.
struct ProArgs {
  int kind;
  Scalars S;
  Ctl* ctl;
  DotWork dots;
  int32_t* ndone;
  uint32_t* status;
};

template <int L>
__global__ void __launch_bounds__(64) prologue_kernel(ProArgs A) {
  __shared__ ProLds<L> pl;
  __shared__ int64_t lds[lds_window_digits<L, 64>()];
  const int pair = blockIdx.x;
  Ctl* const ctl = A.ctl + pair;
  if (solve_done(ctl)) return;
  const Scalars S = A.S.at(pair);
  const int64_t abase = (int64_t)pair * kDotSlots;
  const uint32_t w = prologue_wave<L>(pl, A.kind, S, ctl->iters, abase, A.dots, lds,
                                      lds_window_digits<L, 64>());
  const int brk = (int)((w >> 8) & 0xFFu);
  const uint32_t st = w & 0xFFu;
  if (threadIdx.x == 0) {
    if (brk) {
      finish(ctl, brk - 1);
      if (A.ndone) atomicAdd(A.ndone, 1);
    } else {
      const int n = (A.kind == PRO_GP_ZETA) ? (((w >> 16) & 1u) ? 3 : 2) : 1;
      const int slot0 = (A.kind == PRO_GP_ZETA) ? S_ZETA : S_ALPHA;
      const int slots[3] = {slot0, S_ETA, S_TAU};
      for (int k = 0; k < n; ++k) sstore<L>(S, slots[k], lds_num<L>(pl.limb, pl.hdr, k));
    }
    if (st) {
      atomicOr(&ctl->flags, st);
      atomicOr(A.status, st);
    }
  }
  int clr[3];
  const int nclr = prologue_rings(A.kind, clr);
  for (int k = 0; k < nclr; ++k)
    ring_clear_range<L>(A.dots, abase + clr[k], pl.rlo[k], pl.rhi[k], lds_window_digits<L, 64>());
}

// Driver epilogues of a batch in a launch of their own (the batch's element-wise steps are
// compiled without them): one wavefront per solve, after the step's inner products are rounded.
struct EpiArgs {
  int epi;
  Scalars S;
  Ctl* ctl;
  int32_t* ndone;
  uint32_t* status;
};

template <int L>
__global__ void __launch_bounds__(64) epilogue_kernel(EpiArgs A) {
  __shared__ uint32_t s_cl[kNumScalars * L];
  __shared__ int32_t s_ch[kNumScalars];
  const int pair = blockIdx.x, lane = threadIdx.x;
  Ctl* const ctl = A.ctl + pair;
  if (solve_done(ctl)) return;
  const Scalars S = A.S.at(pair);
  if (lane < kNumScalars) {
    s_ch[lane] = S.hdr[lane];
#pragma unroll
    for (int k = 0; k < L; ++k) s_cl[lane * L + k] = S.limb[(int64_t)k * S.ld + lane];
  }
  const int iters = ctl->iters, maxit = ctl->maxit, hist_len = ctl->hist_len;
  __builtin_amdgcn_s_waitcnt(0xC07F);  // the copy is in LDS for the whole wavefront
  const uint32_t st = epilogue<L>(A.epi, s_cl, s_ch, S.limb, S.hdr, S.ld, ctl, iters, maxit,
                                  hist_len, nullptr, nullptr, 0);
  if (lane == 0) {
    if (st) {
      atomicOr(&ctl->flags, st);
      atomicOr(A.status, st);
    }
    if (A.ndone && ctl->done) atomicAdd(A.ndone, 1);
  }
}

// The scalar slot as a one-element vector reference.
__host__ __device__ inline VecRef slot_ref(const Scalars& S, int slot) {
  VecRef r;
  r.limb = S.limb + slot;
  r.hdr = S.hdr + slot;
  r.ld = S.ld;
  return r;
}

#define MP_ELEMENTWISE_LOOP(A) \
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (A).n; \
       i += (int64_t)gridDim.x * blockDim.x)

// v0 <- v0 + v2[0] * v1   (mp_axpy: y <- y + alpha x)
template <int L>
__global__ void __launch_bounds__(256) axpy_kernel(VecArgs A) {
  const EwCtx c = ew_ctx(A);
  if (solve_done(c.ctl)) return;
  uint32_t st = 0;
  const Num<L> alpha = vload<L>(A.v[2], 0);
  MP_ELEMENTWISE_LOOP(A) {
    const Num<L> y = vload<L>(A.v[0], i), x = vload<L>(A.v[1], i);
    vstore<L>(A.v[0], i, add_rn<L>(y, mul_rn<L>(alpha, x, st), st));
  }
  if (st) atomicOr(A.status, st);
}

// v0 <- v1 (copy)
template <int L>
__global__ void __launch_bounds__(256) copy_kernel(VecArgs A) {
  const EwCtx c = ew_ctx(A);
  if (solve_done(c.ctl)) return;
  MP_ELEMENTWISE_LOOP(A) { vstore<L>(A.v[0], i, vload<L>(A.v[1], i)); }
}

// v0 <- +0
template <int L>
__global__ void __launch_bounds__(256) zero_kernel(VecArgs A) {
  const EwCtx c = ew_ctx(A);
  if (solve_done(c.ctl)) return;
  Num<L> z;
  set_zero(z, 0);
  MP_ELEMENTWISE_LOOP(A) { vstore<L>(A.v[0], i, z); }
}

// v0 <- v1 - v2
template <int L>
__global__ void __launch_bounds__(256) sub_kernel(VecArgs A) {
  const EwCtx c = ew_ctx(A);
  if (solve_done(c.ctl)) return;
  uint32_t st = 0;
  MP_ELEMENTWISE_LOOP(A) { vstore<L>(A.v[0], i, sub_rn<L>(vload<L>(A.v[1], i), vload<L>(A.v[2], i), st)); }
  if (st) atomicOr(A.status, st);
}

// BiCG directions: v = {p, pt, r, rt}. First iteration p = r, pt = rt; then p = r + beta p.
template <int L>
__global__ void __launch_bounds__(256) bicg_dir_kernel(VecArgs A) {
  const EwCtx c = ew_ctx(A);
  if (solve_done(c.ctl)) return;
  uint32_t st = 0;
  const bool first = c.ctl->iters == 0;
  const Num<L> beta = sload<L>(c.S, S_BETA);
  MP_ELEMENTWISE_LOOP(A) {
    // every operand is requested before the branch (p, pt are not used in the first iteration)
    const Num<L> r = vload<L>(A.v[2], i), rt = vload<L>(A.v[3], i);
    const Num<L> p = vload<L>(A.v[0], i), pt = vload<L>(A.v[1], i);
    if (first) {
      vstore<L>(A.v[0], i, r);
      vstore<L>(A.v[1], i, rt);
    } else {
      vstore<L>(A.v[0], i, add_rn<L>(r, mul_rn<L>(beta, p, st), st));
      vstore<L>(A.v[1], i, add_rn<L>(rt, mul_rn<L>(beta, pt, st), st));
    }
  }
  if (st) atomicOr(A.status, st);
}

// BiCG update: v = {x, r, rt, p, z, zt}: x += alpha p; r -= alpha z; rt -= alpha zt; then the
// inner products (r, r) and (rt, r) (fd slots 0 and 1) from the values just formed.  The loop
// is block-uniform: every pass ends with block-wide inner-product steps.
template <int L, bool SEP>
__global__ void __launch_bounds__(256) bicg_update_kernel(VecArgs A) {
  __shared__ PassLds<L, 256> lds;
  __shared__ ProLds<L> pl;
  const EwCtx c = ew_ctx(A);
  if (solve_done(c.ctl)) return;
  uint32_t st = 0;
  // alpha = rho / sigma, sigma = (pt, A p) from the product before
  const ProOut pro = run_prologue<L>(pl, PRO_BICG_ALPHA, c, A.dots, lds.win, lds_window_digits<L, 256>(), 1,
                                     {S_ALPHA, 0, 0}, st, SEP);
  const Num<L> alpha = lds_num<L>(pl.limb, pl.hdr, 0);
  for (int64_t i0 = (int64_t)blockIdx.x * 256; !pro.brk && i0 < A.n; i0 += (int64_t)gridDim.x * 256) {
    const int64_t i = i0 + threadIdx.x;
    const bool ok = i < A.n;
    Num<L> r, rt;
    set_zero(r, 0);
    set_zero(rt, 0);
    if (ok) {
      // A plain solve runs one wavefront per SIMD: every operand is requested before the first
      // store (the stores could alias the loads for all the compiler knows, so it would not move
      // a load above one).  Batched launches keep several wavefronts per SIMD resident instead,
      // with fewer registers: each operand is loaded where it is used.
      Num<L> r0, z, rt0, zt;
      const Num<L> x = vload<L>(A.v[0], i), p = vload<L>(A.v[3], i);
      if constexpr (!SEP) {
        r0 = vload<L>(A.v[1], i), z = vload<L>(A.v[4], i);
        rt0 = vload<L>(A.v[2], i), zt = vload<L>(A.v[5], i);
      }
      vstore<L>(A.v[0], i, add_rn<L>(x, mul_rn<L>(alpha, p, st), st));
      if constexpr (SEP) r0 = vload<L>(A.v[1], i), z = vload<L>(A.v[4], i);
      r = sub_rn<L>(r0, mul_rn<L>(alpha, z, st), st);
      vstore<L>(A.v[1], i, r);
      if constexpr (SEP) rt0 = vload<L>(A.v[2], i), zt = vload<L>(A.v[5], i);
      rt = sub_rn<L>(rt0, mul_rn<L>(alpha, zt, st), st);
      vstore<L>(A.v[2], i, rt);
    }
    const int32_t hr = make_hdr(r.e, r.s), hrt = make_hdr(rt.e, rt.s);
    pass_dot<L, 256>(lds, ok, hr, hr, r.m, r.m, A.dots, c.abase + A.fd.slot[0]);
    pass_dot<L, 256>(lds, ok, hrt, hr, rt.m, r.m, A.dots, c.abase + A.fd.slot[1]);
  }
  dots_finish<L, 256, !SEP, true>(A.dots, A.fd, c.pair, A.batch.pair_of_tile != nullptr, c.idx, c.nblocks, c.ctl,
                                  c.S, A.batch.ndone, A.status, st, lds.win, lds_window_digits<L, 256>(), &pro);
}

// GPBiCG direction: v = {p, w, r, v, q, u}.  First iteration p = r; then
// w = v + beta q, p = r + beta (p - u).
template <int L>
__global__ void __launch_bounds__(256) gp_dir_kernel(VecArgs A) {
  const EwCtx c = ew_ctx(A);
  if (solve_done(c.ctl)) return;
  uint32_t st = 0;
  const bool first = c.ctl->iters == 0;
  const Num<L> beta = sload<L>(c.S, S_BETA);
  MP_ELEMENTWISE_LOOP(A) {
    // every operand is requested before the branch (only r is used in the first iteration)
    const Num<L> r = vload<L>(A.v[2], i), q = vload<L>(A.v[4], i), v = vload<L>(A.v[3], i);
    const Num<L> p = vload<L>(A.v[0], i), u = vload<L>(A.v[5], i);
    if (first) {
      vstore<L>(A.v[0], i, r);
    } else {
      vstore<L>(A.v[1], i, add_rn<L>(v, mul_rn<L>(beta, q, st), st));
      const Num<L> pmu = sub_rn<L>(p, u, st);
      vstore<L>(A.v[0], i, add_rn<L>(r, mul_rn<L>(beta, pmu, st), st));
    }
  }
  if (st) atomicOr(A.status, st);
}

// GPBiCG t, s, y: v = {t, s, y, r, q, w}.  s = t - r (not in the first iteration),
// t = r - alpha q, y = alpha q - r (first) or s - alpha (w - q); then the inner products
// (y, y) and (y, t) (fd slots 0 and 1).
template <int L, bool SEP>
__global__ void __launch_bounds__(256) gp_tsy_kernel(VecArgs A) {
  __shared__ PassLds<L, 256> lds;
  __shared__ ProLds<L> pl;
  const EwCtx c = ew_ctx(A);
  if (solve_done(c.ctl)) return;
  uint32_t st = 0;
  const bool first = c.ctl->iters == 0;
  // alpha = rho / den, den = (rt, A p) from the product before
  const ProOut pro = run_prologue<L>(pl, PRO_GP_ALPHA, c, A.dots, lds.win, lds_window_digits<L, 256>(), 1,
                                     {S_ALPHA, 0, 0}, st, SEP);
  const Num<L> alpha = lds_num<L>(pl.limb, pl.hdr, 0);
  for (int64_t i0 = (int64_t)blockIdx.x * 256; !pro.brk && i0 < A.n; i0 += (int64_t)gridDim.x * 256) {
    const int64_t i = i0 + threadIdx.x;
    const bool ok = i < A.n;
    Num<L> tn, y;
    set_zero(tn, 0);
    set_zero(y, 0);
    if (ok) {
      // every operand is requested before the first store (t and w are not used in the first
      // iteration)
      const Num<L> r = vload<L>(A.v[3], i), q = vload<L>(A.v[4], i);
      const Num<L> t = vload<L>(A.v[0], i), w = vload<L>(A.v[5], i);
      const Num<L> aq = mul_rn<L>(alpha, q, st);
      Num<L> s;
      if (!first) {
        s = sub_rn<L>(t, r, st);
        vstore<L>(A.v[1], i, s);
      }
      tn = sub_rn<L>(r, aq, st);
      vstore<L>(A.v[0], i, tn);
      if (first) {
        y = sub_rn<L>(aq, r, st);
      } else {
        const Num<L> wq = sub_rn<L>(w, q, st);
        y = sub_rn<L>(s, mul_rn<L>(alpha, wq, st), st);
      }
      vstore<L>(A.v[2], i, y);
    }
    const int32_t hy = make_hdr(y.e, y.s), ht = make_hdr(tn.e, tn.s);
    pass_dot<L, 256>(lds, ok, hy, hy, y.m, y.m, A.dots, c.abase + A.fd.slot[0]);
    pass_dot<L, 256>(lds, ok, hy, ht, y.m, tn.m, A.dots, c.abase + A.fd.slot[1]);
  }
  dots_finish<L, 256, !SEP>(A.dots, A.fd, c.pair, A.batch.pair_of_tile != nullptr, c.idx, c.nblocks, c.ctl, c.S,
                      A.batch.ndone, A.status, st, lds.win, lds_window_digits<L, 256>(), &pro);
}

// GPBiCG update: v = {u, z, x, r, q, s, p, t} and v2 = {y, v} in w[]:
// u = zeta q + eta (s + beta u); z = zeta r + eta z - alpha u; x = x + alpha p + z;
// r = t - eta y - zeta v; then the inner products (r, r) and (rt, r) (fd slots 0 and 1).
struct GpUpdArgs {
  VecArgs a;
  VecRef y, v, rt;
};

template <int L, bool SEP>
__global__ void __launch_bounds__(256) gp_update_kernel(GpUpdArgs G) {
  __shared__ PassLds<L, 256> lds;
  __shared__ ProLds<L> pl;
  const VecArgs& A = G.a;
  const EwCtx c = ew_ctx(A);
  if (solve_done(c.ctl)) return;
  uint32_t st = 0;
  // zeta, eta (and tau) from mu1..mu5 of the two launches before
  const ProOut pro = run_prologue<L>(pl, PRO_GP_ZETA, c, A.dots, lds.win, lds_window_digits<L, 256>(), 3,
                                     {S_ZETA, S_ETA, S_TAU}, st, SEP);
  const Num<L> alpha = sload<L>(c.S, S_ALPHA), beta = sload<L>(c.S, S_BETA);
  const Num<L> zeta = lds_num<L>(pl.limb, pl.hdr, 0), eta = lds_num<L>(pl.limb, pl.hdr, 1);
  for (int64_t i0 = (int64_t)blockIdx.x * 256; !pro.brk && i0 < A.n; i0 += (int64_t)gridDim.x * 256) {
    const int64_t i = i0 + threadIdx.x;
    const bool ok = i < A.n;
    Num<L> rn, rt;
    set_zero(rn, 0);
    set_zero(rt, 0);
    if (ok) {
      // A plain solve requests every operand before the first store; batched launches load
      // each where it is used (see bicg_update_kernel).
      Num<L> r, z_old, x_old, p, t, y, v;
      rt = vload<L>(G.rt, i);
      const Num<L> q = vload<L>(A.v[4], i), s = vload<L>(A.v[5], i);
      const Num<L> u_old = vload<L>(A.v[0], i);
      if constexpr (!SEP) {
        r = vload<L>(A.v[3], i), z_old = vload<L>(A.v[1], i), x_old = vload<L>(A.v[2], i);
        p = vload<L>(A.v[6], i), t = vload<L>(A.v[7], i), y = vload<L>(G.y, i), v = vload<L>(G.v, i);
      }
      const Num<L> u = add_rn<L>(mul_rn<L>(zeta, q, st),
                                 mul_rn<L>(eta, add_rn<L>(s, mul_rn<L>(beta, u_old, st), st), st), st);
      vstore<L>(A.v[0], i, u);
      if constexpr (SEP) r = vload<L>(A.v[3], i), z_old = vload<L>(A.v[1], i);
      const Num<L> z = sub_rn<L>(add_rn<L>(mul_rn<L>(zeta, r, st), mul_rn<L>(eta, z_old, st), st),
                                 mul_rn<L>(alpha, u, st), st);
      vstore<L>(A.v[1], i, z);
      if constexpr (SEP) x_old = vload<L>(A.v[2], i), p = vload<L>(A.v[6], i);
      const Num<L> x = add_rn<L>(add_rn<L>(x_old, mul_rn<L>(alpha, p, st), st), z, st);
      vstore<L>(A.v[2], i, x);
      if constexpr (SEP) t = vload<L>(A.v[7], i), y = vload<L>(G.y, i), v = vload<L>(G.v, i);
      rn = sub_rn<L>(sub_rn<L>(t, mul_rn<L>(eta, y, st), st), mul_rn<L>(zeta, v, st), st);
      vstore<L>(A.v[3], i, rn);
    }
    const int32_t hr = make_hdr(rn.e, rn.s), hrt = make_hdr(rt.e, rt.s);
    pass_dot<L, 256>(lds, ok, hr, hr, rn.m, rn.m, A.dots, c.abase + A.fd.slot[0]);
    pass_dot<L, 256>(lds, ok, hrt, hr, rt.m, rn.m, A.dots, c.abase + A.fd.slot[1]);
  }
  dots_finish<L, 256, !SEP, true>(A.dots, A.fd, c.pair, A.batch.pair_of_tile != nullptr, c.idx, c.nblocks, c.ctl, c.S,
                      A.batch.ndone, A.status, st, lds.win, lds_window_digits<L, 256>(), &pro);
}

// ------------------------------------------------------------------------------------------
// CGS and BiCGSTAB steps (the paper's other product-type methods, K = I; one RN per operation
// in the order written).
// ------------------------------------------------------------------------------------------

// CGS direction: v = {u, p, r, q}.  First iteration u = p = r; then u = r + beta q,
// p = u + beta (q + beta p), beta = rho / rho_old (the stopping test's epilogue formed it).
template <int L>
__global__ void __launch_bounds__(256) cgs_dir_kernel(VecArgs A) {
  const EwCtx c = ew_ctx(A);
  if (solve_done(c.ctl)) return;
  uint32_t st = 0;
  const bool first = c.ctl->iters == 0;
  const Num<L> beta = sload<L>(c.S, S_BETA);
  MP_ELEMENTWISE_LOOP(A) {
    const Num<L> r = vload<L>(A.v[2], i), q = vload<L>(A.v[3], i), p = vload<L>(A.v[1], i);
    if (first) {
      vstore<L>(A.v[0], i, r);
      vstore<L>(A.v[1], i, r);
    } else {
      const Num<L> u = add_rn<L>(r, mul_rn<L>(beta, q, st), st);
      vstore<L>(A.v[0], i, u);
      const Num<L> qbp = add_rn<L>(q, mul_rn<L>(beta, p, st), st);
      vstore<L>(A.v[1], i, add_rn<L>(u, mul_rn<L>(beta, qbp, st), st));
    }
  }
  if (st) atomicOr(A.status, st);
}

// CGS q, u^, x: v = {q, uh, x, u, vh}.  alpha = rho / (r~, A p) (the product's inner product,
// still in its ring; zero: breakdown); q = u - alpha vh, u^ = u + q, x = x + alpha u^.
template <int L>
__global__ void __launch_bounds__(256) cgs_qux_kernel(VecArgs A) {
  __shared__ PassLds<L, 256> lds;
  __shared__ ProLds<L> pl;
  const EwCtx c = ew_ctx(A);
  if (solve_done(c.ctl)) return;
  uint32_t st = 0;
  const ProOut pro = run_prologue<L>(pl, PRO_BICG_ALPHA, c, A.dots, lds.win, lds_window_digits<L, 256>(), 1,
                                     {S_ALPHA, 0, 0}, st);
  const Num<L> alpha = lds_num<L>(pl.limb, pl.hdr, 0);
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; !pro.brk && i < A.n; i += (int64_t)gridDim.x * 256) {
    const Num<L> u = vload<L>(A.v[3], i), vh = vload<L>(A.v[4], i), x = vload<L>(A.v[2], i);
    const Num<L> q = sub_rn<L>(u, mul_rn<L>(alpha, vh, st), st);
    vstore<L>(A.v[0], i, q);
    const Num<L> uh = add_rn<L>(u, q, st);
    vstore<L>(A.v[1], i, uh);
    vstore<L>(A.v[2], i, add_rn<L>(x, mul_rn<L>(alpha, uh, st), st));
  }
  dots_finish<L, 256, false>(A.dots, A.fd, c.pair, false, c.idx, c.nblocks, c.ctl, c.S, A.batch.ndone,
                             A.status, st, lds.win, lds_window_digits<L, 256>(), &pro);
}

// CGS residual: v = {r, qh, rt}.  r = r - alpha qh, then the inner products (r, r) and (r~, r)
// (fd slots 0 and 1); the last block's epilogue runs the stopping test and forms beta.
template <int L>
__global__ void __launch_bounds__(256) cgs_r_kernel(VecArgs A) {
  __shared__ PassLds<L, 256> lds;
  const EwCtx c = ew_ctx(A);
  if (solve_done(c.ctl)) return;
  uint32_t st = 0;
  const Num<L> alpha = sload<L>(c.S, S_ALPHA);
  for (int64_t i0 = (int64_t)blockIdx.x * 256; i0 < A.n; i0 += (int64_t)gridDim.x * 256) {
    const int64_t i = i0 + threadIdx.x;
    const bool ok = i < A.n;
    Num<L> r, rt;
    set_zero(r, 0);
    set_zero(rt, 0);
    if (ok) {
      const Num<L> r0 = vload<L>(A.v[0], i), qh = vload<L>(A.v[1], i);
      rt = vload<L>(A.v[2], i);
      r = sub_rn<L>(r0, mul_rn<L>(alpha, qh, st), st);
      vstore<L>(A.v[0], i, r);
    }
    const int32_t hr = make_hdr(r.e, r.s), hrt = make_hdr(rt.e, rt.s);
    pass_dot<L, 256>(lds, ok, hr, hr, r.m, r.m, A.dots, c.abase + A.fd.slot[0]);
    pass_dot<L, 256>(lds, ok, hrt, hr, rt.m, r.m, A.dots, c.abase + A.fd.slot[1]);
  }
  dots_finish<L, 256, true>(A.dots, A.fd, c.pair, false, c.idx, c.nblocks, c.ctl, c.S, A.batch.ndone,
                            A.status, st, lds.win, lds_window_digits<L, 256>());
}

// BiCGSTAB direction: v = {p, r, v}.  First iteration p = r; then
// p = r + beta (p - omega v), beta = (rho / rho_old) (alpha / omega) (formed by the epilogue of
// the stopping test), omega in the zeta slot.
template <int L>
__global__ void __launch_bounds__(256) stab_dir_kernel(VecArgs A) {
  const EwCtx c = ew_ctx(A);
  if (solve_done(c.ctl)) return;
  uint32_t st = 0;
  const bool first = c.ctl->iters == 0;
  const Num<L> beta = sload<L>(c.S, S_BETA), omega = sload<L>(c.S, S_ZETA);
  MP_ELEMENTWISE_LOOP(A) {
    const Num<L> r = vload<L>(A.v[1], i), p = vload<L>(A.v[0], i), v = vload<L>(A.v[2], i);
    if (first) {
      vstore<L>(A.v[0], i, r);
    } else {
      const Num<L> d = sub_rn<L>(p, mul_rn<L>(omega, v, st), st);
      vstore<L>(A.v[0], i, add_rn<L>(r, mul_rn<L>(beta, d, st), st));
    }
  }
  if (st) atomicOr(A.status, st);
}

// BiCGSTAB s: v = {s, r, v}.  alpha = rho / (r~, A p) (zero: breakdown); s = r - alpha v.
template <int L>
__global__ void __launch_bounds__(256) stab_s_kernel(VecArgs A) {
  __shared__ PassLds<L, 256> lds;
  __shared__ ProLds<L> pl;
  const EwCtx c = ew_ctx(A);
  if (solve_done(c.ctl)) return;
  uint32_t st = 0;
  const ProOut pro = run_prologue<L>(pl, PRO_BICG_ALPHA, c, A.dots, lds.win, lds_window_digits<L, 256>(), 1,
                                     {S_ALPHA, 0, 0}, st);
  const Num<L> alpha = lds_num<L>(pl.limb, pl.hdr, 0);
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; !pro.brk && i < A.n; i += (int64_t)gridDim.x * 256) {
    const Num<L> r = vload<L>(A.v[1], i), v = vload<L>(A.v[2], i);
    vstore<L>(A.v[0], i, sub_rn<L>(r, mul_rn<L>(alpha, v, st), st));
  }
  dots_finish<L, 256, false>(A.dots, A.fd, c.pair, false, c.idx, c.nblocks, c.ctl, c.S, A.batch.ndone,
                             A.status, st, lds.win, lds_window_digits<L, 256>(), &pro);
}

// BiCGSTAB update: v = {x, r, p, s, t, rt, s^}.  omega = (t, s) / (t, t) (the product's inner
// products, still in their rings; 0 when (t, t) = 0); x = x + alpha p + omega s^ (s^ = s
// unless v[6] is given: the preconditioned direction K^{-1} s, with K^{-1} p in v[2]),
// r = s - omega t; then (r, r) and (r~, r) (fd slots 0 and 1); the last block's epilogue runs
// the stopping test, the omega = 0 exit and forms beta.
template <int L>
__global__ void __launch_bounds__(256) stab_xr_kernel(VecArgs A) {
  __shared__ PassLds<L, 256> lds;
  __shared__ ProLds<L> pl;
  const EwCtx c = ew_ctx(A);
  if (solve_done(c.ctl)) return;
  uint32_t st = 0;
  const ProOut pro = run_prologue<L>(pl, PRO_STAB_OMEGA, c, A.dots, lds.win, lds_window_digits<L, 256>(), 1,
                                     {S_ZETA, 0, 0}, st);
  const Num<L> omega = lds_num<L>(pl.limb, pl.hdr, 0);
  const Num<L> alpha = sload<L>(c.S, S_ALPHA);
  for (int64_t i0 = (int64_t)blockIdx.x * 256; i0 < A.n; i0 += (int64_t)gridDim.x * 256) {
    const int64_t i = i0 + threadIdx.x;
    const bool ok = i < A.n;
    Num<L> r, rt;
    set_zero(r, 0);
    set_zero(rt, 0);
    if (ok) {
      const Num<L> x = vload<L>(A.v[0], i), p = vload<L>(A.v[2], i), s = vload<L>(A.v[3], i);
      const Num<L> t = vload<L>(A.v[4], i);
      rt = vload<L>(A.v[5], i);
      const Num<L> sx = A.v[6].hdr ? vload<L>(A.v[6], i) : s;
      const Num<L> xa = add_rn<L>(x, mul_rn<L>(alpha, p, st), st);
      vstore<L>(A.v[0], i, add_rn<L>(xa, mul_rn<L>(omega, sx, st), st));
      r = sub_rn<L>(s, mul_rn<L>(omega, t, st), st);
      vstore<L>(A.v[1], i, r);
    }
    const int32_t hr = make_hdr(r.e, r.s), hrt = make_hdr(rt.e, rt.s);
    pass_dot<L, 256>(lds, ok, hr, hr, r.m, r.m, A.dots, c.abase + A.fd.slot[0]);
    pass_dot<L, 256>(lds, ok, hrt, hr, rt.m, r.m, A.dots, c.abase + A.fd.slot[1]);
  }
  dots_finish<L, 256, true>(A.dots, A.fd, c.pair, false, c.idx, c.nblocks, c.ctl, c.S, A.batch.ndone,
                            A.status, st, lds.win, lds_window_digits<L, 256>(), &pro);
}

// Write a constant into element 0 of a vector or a scalar slot (kernel arguments carry it).
template <int L>
struct ConstArgs {
  VecRef out;
  uint32_t m[L];
  int32_t hdr;
  int64_t count;  // places written: element j * step of out for j < count
  int64_t step;
};

template <int L>
__global__ void set_scalar_kernel(ConstArgs<L> A) {
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < A.count;
       j += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = j * A.step;
    A.out.hdr[i] = A.hdr;
#pragma unroll
    for (int k = 0; k < L; ++k) A.out.limb[(int64_t)k * A.out.ld + i] = A.m[k];
  }
}

// Initialise the control blocks of n solves.
static __global__ void ctl_init_kernel(Ctl* ctl, int n, int32_t maxit, int32_t hist_len) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    ctl[i].done = 0;
    ctl[i].status = kNotConverged;
    ctl[i].iters = 0;
    ctl[i].maxit = maxit;
    ctl[i].flags = 0;
    ctl[i].hist_len = hist_len;
  }
}

}  // namespace mp
