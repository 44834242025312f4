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
  EPI_BICG_SIGMA,   // sigma = (pt, z): alpha = rho / sigma
  EPI_BICG_CONV,    // q = (r,r), rho' = (rt,r): stopping test, then beta = rho'/rho
  EPI_GP_ALPHA,     // den = (rt, q): alpha = rho / den
  EPI_GP_ZETA,      // mu1..mu5: zeta, eta
  EPI_GP_CONV,      // q = (r,r), rho' = (rt,r): stopping test, zeta = 0 exit, beta
};

template <int L>
MPD void epilogue(int epi, const Scalars& S, Ctl* ctl, const VecRef& hist, uint32_t& st) {
  if (!ctl || epi == EPI_NONE) return;
  switch (epi) {
    case EPI_SETUP: {
      const Num<L> q0 = sload_dev<L>(S, S_Q0);
      const Num<L> nrm0 = sqrt_rn<L>(q0, st);
      const Num<L> thr = add_rn<L>(mul_rn<L>(sload_dev<L>(S, S_CREL), nrm0, st), sload_dev<L>(S, S_CABS), st);
      sstore<L>(S, S_NRM0, nrm0);
      sstore<L>(S, S_THR, thr);
      if (sqrt_le<L>(q0, thr)) {
        finish(ctl, kConverged);
      } else if (ctl->maxit <= 0) {
        finish(ctl, kNotConverged);
      } else if (is_zero(sload_dev<L>(S, S_RHO))) {
        finish(ctl, kBreakRho);
      }
      break;
    }
    case EPI_BICG_SIGMA: {
      const Num<L> sigma = sload_dev<L>(S, S_SIGMA);
      if (is_zero(sigma)) {
        finish(ctl, kBreakSigma);
      } else {
        sstore<L>(S, S_ALPHA, div_rn<L>(sload_dev<L>(S, S_RHO), sigma, st));
      }
      break;
    }
    case EPI_GP_ALPHA: {
      const Num<L> den = sload_dev<L>(S, S_DEN);
      if (is_zero(den)) {
        finish(ctl, kBreakSigma);
      } else {
        sstore<L>(S, S_ALPHA, div_rn<L>(sload_dev<L>(S, S_RHO), den, st));
      }
      break;
    }
    case EPI_GP_ZETA: {
      const Num<L> mu1 = sload_dev<L>(S, S_MU1), mu2 = sload_dev<L>(S, S_MU2), mu3 = sload_dev<L>(S, S_MU3);
      const Num<L> mu4 = sload_dev<L>(S, S_MU4), mu5 = sload_dev<L>(S, S_MU5);
      if (ctl->iters == 0) {  // first iteration: zeta = mu2 / mu5, eta = 0
        if (is_zero(mu5)) {
          finish(ctl, kBreakTau);
        } else {
          Num<L> eta;
          set_zero(eta, 0);
          sstore<L>(S, S_ZETA, div_rn<L>(mu2, mu5, st));
          sstore<L>(S, S_ETA, eta);
        }
      } else {
        const Num<L> tau = sub_rn<L>(mul_rn<L>(mu5, mu1, st), mul_rn<L>(mu4, mu4, st), st);
        if (is_zero(tau)) {
          finish(ctl, kBreakTau);
        } else {
          const Num<L> zn = sub_rn<L>(mul_rn<L>(mu1, mu2, st), mul_rn<L>(mu3, mu4, st), st);
          const Num<L> en = sub_rn<L>(mul_rn<L>(mu5, mu3, st), mul_rn<L>(mu4, mu2, st), st);
          sstore<L>(S, S_TAU, tau);
          sstore<L>(S, S_ZETA, div_rn<L>(zn, tau, st));
          sstore<L>(S, S_ETA, div_rn<L>(en, tau, st));
        }
      }
      break;
    }
    case EPI_BICG_CONV:
    case EPI_GP_CONV: {
      const Num<L> q = sload_dev<L>(S, S_Q);
      const int i = ctl->iters + 1;
      if (hist.limb && i - 1 < ctl->hist_len) vstore<L>(hist, i - 1, q);
      ctl->iters = i;
      if (sqrt_le<L>(q, sload_dev<L>(S, S_THR))) {
        finish(ctl, kConverged);
        break;
      }
      if (epi == EPI_GP_CONV && is_zero(sload_dev<L>(S, S_ZETA))) {
        finish(ctl, kBreakZeta);
        break;
      }
      if (i >= ctl->maxit) {
        finish(ctl, kNotConverged);
        break;
      }
      const Num<L> rho = sload_dev<L>(S, S_RHO);
      const Num<L> rho_next = sload_dev<L>(S, S_RHO_NEXT);
      sstore<L>(S, S_RHO_OLD, rho);
      sstore<L>(S, S_RHO, rho_next);
      if (is_zero(rho_next)) {
        finish(ctl, kBreakRho);
        break;
      }
      if (epi == EPI_BICG_CONV) {
        sstore<L>(S, S_BETA, div_rn<L>(rho_next, rho, st));
      } else {
        const Num<L> alpha = sload_dev<L>(S, S_ALPHA), zeta = sload_dev<L>(S, S_ZETA);
        sstore<L>(S, S_ALPHA_OLD, alpha);
        sstore<L>(S, S_ZETA_OLD, zeta);
        sstore<L>(S, S_BETA, mul_rn<L>(div_rn<L>(rho_next, rho, st), div_rn<L>(alpha, zeta, st), st));
      }
      break;
    }
    default:
      break;
  }
}

// ------------------------------------------------------------------------------------------
// Exact inner products.
//
// Every inner product owns a slot: an exponent anchor (the smallest and largest e_x + e_y over
// its non-zero products, kept with integer atomic min/max), a global carry-save window of int64
// digits, and an integer ticket.  The kernel that *produces* the operands fills the anchor while
// it writes them (the SpMV for products with its output, the vector updates for theirs), so the
// inner-product kernel starts with a global anchor: each block accumulates its exact products in
// per-lane LDS windows, sums them digit by digit and adds the digit sums to the slot's window
// with integer atomics (associative, hence order-independent and deterministic).  The last block
// rounds the window once, clears the slot for its next use and, once every inner product of the
// launch is done, runs the driver epilogue.  Lane windows are padded to an odd stride so that the
// per-lane adds and the per-digit sums hit distinct LDS banks.
// ------------------------------------------------------------------------------------------
constexpr int kDotMaxND = 5;
constexpr int kDotMaxBlocks = 128;
constexpr int kDotThreads = 256;
constexpr int kDotStride = kDotThreads + 1;
constexpr int kDotSlots = 8;

// block-shared window capacity (the per-lane windows' LDS reused as one array)
template <int L>
constexpr int dot_shared_digits() { return window_fast_digits<L>() * kDotStride; }

// Per-solve (or per-context) inner-product state.
// Anchors are spread over kAnchorBins bins per slot (a producing wave updates bin
// wave-index mod kAnchorBins) so that a thousand producing waves do not contend on one address;
// the inner-product kernel reduces the bins.
constexpr int kAnchorBins = 64;

struct DotWork {
  int32_t* anchor;    // [nslots][kAnchorBins][2]: emin, emax; (INT32_MAX, INT32_MIN) when empty
  int64_t* win;       // [nslots][win_stride] carry-save digits, zero between uses
  uint32_t* ticket;   // [nslots + number of solves]: entry nslots + k counts the finished blocks
                      // of solve k's current launch
  int64_t win_stride; // >= dot_shared_digits<L>()
  int nslots;
};

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

// Fold the exponent of the product of two headers into a running (emin, emax).
MPD void pair_exponent(int32_t h1, int32_t h2, int32_t& emin, int32_t& emax) {
  if (!hdr_is_zero(h1) && !hdr_is_zero(h2)) {
    const int32_t e = (h1 >> 1) + (h2 >> 1);
    emin = min(emin, e);
    emax = max(emax, e);
  }
}

// Publish a block's (emin, emax) to an anchor slot: wave reduction, then one lane per wave
// (an integer min/max is order-independent).
MPD int anchor_bin() {
  return (int)((blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) & (kAnchorBins - 1));
}

MPD void anchor_publish(int32_t* anchor, int slot, int32_t emin, int32_t emax) {
  emin = wave_min(emin);
  emax = wave_max(emax);
  if ((threadIdx.x & 63) == 0 && emax >= emin) {
    int32_t* a = anchor + 2 * ((int64_t)slot * kAnchorBins + anchor_bin());
    atomicMin(&a[0], emin);
    atomicMax(&a[1], emax);
  }
}

struct DotArgs {
  int64_t n;
  int nd;
  VecRef x[kDotMaxND];
  VecRef y[kDotMaxND];
  VecRef out[kDotMaxND];  // result d goes to element 0 of out[d]
  int slot[kDotMaxND];
  DotWork w;
  Scalars S;
  Ctl* ctl;  // nullable
  uint32_t* status;
  int epi;
  VecRef hist;
  BatchMap batch;  // batch.pair_of_tile == nullptr: one solve
};

// Anchor (smallest and largest e_x + e_y) of inner-product slot `slot`, its bins reduced by one
// wave; every lane gets it.
static_assert(kAnchorBins == 64, "one anchor bin per lane");
MPD void wave_anchor(const int32_t* anchor, int64_t slot, int32_t& emin, int32_t& emax) {
  const int32_t* b = anchor + 2 * (slot * kAnchorBins + (threadIdx.x & 63));
  emin = wave_min(ld_dev(b));
  emax = wave_max(ld_dev(b + 1));
}

// The two elements a thread takes per step: headers and limbs are loaded together (the limbs of
// a zero are loaded too, so no load waits for a header).
template <int L>
struct DotElems {
  int32_t hx[2], hy[2];
  uint32_t x[2][L], y[2][L];
};

template <int L>
MPD void dot_load(DotElems<L>& E, const VecRef& X, const VecRef& Y, int64_t i0, int64_t i1, bool h0,
                  bool h1) {
  const int32_t z = (int32_t)0x80000000;  // +0
  E.hx[0] = h0 ? X.hdr[i0] : z;
  E.hy[0] = h0 ? Y.hdr[i0] : z;
  E.hx[1] = h1 ? X.hdr[i1] : z;
  E.hy[1] = h1 ? Y.hdr[i1] : z;
#pragma unroll
  for (int q = 0; q < L; ++q) {
    E.x[0][q] = h0 ? X.limb[(int64_t)q * X.ld + i0] : 0u;
    E.y[0][q] = h0 ? Y.limb[(int64_t)q * Y.ld + i0] : 0u;
    E.x[1][q] = h1 ? X.limb[(int64_t)q * X.ld + i1] : 0u;
    E.y[1][q] = h1 ? Y.limb[(int64_t)q * Y.ld + i1] : 0u;
  }
}

template <int L>
__global__ void __launch_bounds__(kDotThreads) dot_kernel(DotArgs A) {
  constexpr int WF = window_fast_digits<L>();
  constexpr int WB = dot_shared_digits<L>();
  constexpr int WMAXF = 2 * L + 16;  // final windows up to this size are carried in registers
  __shared__ int64_t s_win[WB];
  __shared__ uint32_t s_last;
  // batch: block = one tile of one solve; otherwise a grid-stride pass over the whole vector
  const bool batched = A.batch.pair_of_tile != nullptr;
  const int pair = batched ? A.batch.pair_of_tile[blockIdx.x] : 0;
  Ctl* const ctl = A.ctl ? A.ctl + pair : nullptr;
  if (solve_done(ctl)) return;
  const Scalars S = A.S.at(pair);
  const int t = threadIdx.x;
  uint32_t st = 0;
  const int d = blockIdx.y;  // the inner products of one launch run side by side, one row each
  const int64_t slot0 = (int64_t)pair * kDotSlots;
  const unsigned nblocks = batched ? (unsigned)A.batch.tiles_of_pair[pair] : gridDim.x;

  // first elements in flight while the anchor is reduced (operands picked by comparison: a
  // dynamic index into the argument arrays would copy them to scratch memory)
  VecRef X = A.x[0], Y = A.y[0];
  int dslot = A.slot[0];
#pragma unroll
  for (int k = 1; k < kDotMaxND; ++k) {
    if (k == d) {
      X = A.x[k];
      Y = A.y[k];
      dslot = A.slot[k];
    }
  }
  const int64_t stride = batched ? (int64_t)(kTile / 2) : (int64_t)gridDim.x * kDotThreads;
  const int64_t n_end = batched ? (int64_t)(blockIdx.x + 1) * kTile : A.n;
  int64_t i0 = batched ? (int64_t)blockIdx.x * kTile + t : (int64_t)blockIdx.x * kDotThreads + t;
  DotElems<L> E;
  dot_load<L>(E, X, Y, i0, i0 + stride, i0 < n_end, i0 + stride < n_end);

  int32_t emin, emax;
  wave_anchor(A.w.anchor, slot0 + dslot, emin, emax);
  int64_t* gw = A.w.win + (slot0 + dslot) * A.w.win_stride;
  const bool any = emax >= emin;
  const int W = any ? window_digits<L>(emin, emax) : 0;
  const bool fits = W <= WB && W <= A.w.win_stride;
  if (any && !fits) st |= kStWindow;
  if (any && fits) {
    const bool fast = W <= WF;
    if (fast) {
      for (int w = 0; w < WF; ++w) s_win[w * kDotStride + t] = 0;
    } else {
      for (int w = t; w < W; w += kDotThreads) s_win[w] = 0;
      __syncthreads();
    }
    while (true) {
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        if (!hdr_is_zero(E.hx[k]) && !hdr_is_zero(E.hy[k])) {
          uint32_t pr[2 * L];
          mul_full<L>(E.x[k], E.y[k], pr);
          const uint32_t off = (uint32_t)((E.hx[k] >> 1) + (E.hy[k] >> 1) - emin);
          const uint32_t sg = (uint32_t)(E.hx[k] ^ E.hy[k]) & 1u;
          if (fast) window_add<L>(s_win + t, kDotStride, pr, sg, off);
          else window_add_atomic<L>(s_win, pr, sg, off);
        }
      }
      i0 += 2 * stride;
      if (i0 >= n_end) break;
      dot_load<L>(E, X, Y, i0, i0 + stride, true, i0 + stride < n_end);
    }
    __syncthreads();
    if (fast) {
      // digit w is summed over the 256 lane windows by TPD consecutive threads, then combined
      // with shuffles; the sum goes to the slot's global window
      constexpr int TPD = (WF <= 32) ? 8 : 4;
      constexpr int SEG = 64 / TPD;
      const int w = t / TPD, sub = t % TPD;
      int64_t a0 = 0, a1 = 0;
      if (w < W) {
        const int64_t* row = s_win + w * kDotStride + SEG * sub;
#pragma unroll
        for (int m = 0; m < kDotThreads / 64; ++m) {
#pragma unroll
          for (int k = 0; k < SEG; k += 2) {
            a0 += row[64 * m + k];
            a1 += row[64 * m + k + 1];
          }
        }
      }
      int64_t dsum = a0 + a1;
#pragma unroll
      for (int o = 1; o < TPD; o <<= 1) dsum += __shfl_xor(dsum, o);
      if (w < W && sub == 0 && dsum != 0)
        atomicAdd((unsigned long long*)&gw[w], (unsigned long long)dsum);
    } else {
      for (int w = t; w < W; w += kDotThreads) {
        const int64_t v = s_win[w];
        if (v) atomicAdd((unsigned long long*)&gw[w], (unsigned long long)v);
      }
    }
  }

  // One ticket per launch (per solve in a batch) counts the blocks of every inner product; the
  // window atomics of every wave are complete before it is taken, and the last block reads the
  // windows with atomics, so no cache write-back or invalidate is needed.
  wait_memory();
  __syncthreads();
  uint32_t* ticket = A.w.ticket + A.w.nslots + pair;
  if (t == 0) s_last = (atomicAdd(ticket, 1u) == nblocks * (unsigned)A.nd - 1) ? 1u : 0u;
  __syncthreads();
  if (!s_last) {
    if (st) atomicOr(A.status, st);
    return;
  }

  // The last block: wave k rounds inner products k and k + 4 when their windows have at most 63
  // digits (one per lane); wider windows are rounded afterwards by the whole block.
  const int wv = t >> 6, lane = t & 63;
  int32_t amin[kDotMaxND], amax[kDotMaxND];
#pragma unroll
  for (int dd = 0; dd < kDotMaxND; ++dd) {
    amin[dd] = INT32_MAX;
    amax[dd] = INT32_MIN;
    if (dd < A.nd) wave_anchor(A.w.anchor, slot0 + A.slot[dd], amin[dd], amax[dd]);
  }
  __syncthreads();  // every wave has its anchors: the bins may be reset
#pragma unroll
  for (int dd = 0; dd < kDotMaxND; ++dd) {
    if (dd < A.nd && wv == 0) {
      int32_t* b = A.w.anchor + 2 * ((slot0 + A.slot[dd]) * kAnchorBins + lane);
      st_dev(b, INT32_MAX);
      st_dev(b + 1, INT32_MIN);
    }
  }
#pragma unroll
  for (int dd = 0; dd < kDotMaxND; ++dd) {
    if (dd >= A.nd) continue;  // (continue, not break: the loop must unroll fully)
    const bool anyd = amax[dd] >= amin[dd];
    const int Wd = anyd ? window_digits<L>(amin[dd], amax[dd]) : 0;
    const bool fitsd = Wd <= WB && Wd <= A.w.win_stride;
    VecRef o = A.out[dd];  // batch: a scalar slot of solve 0, moved to this solve's slots
    if (batched) {
      o.limb += (int64_t)pair * kNumScalars;
      o.hdr += (int64_t)pair * kNumScalars;
    }
    int64_t* gwd = A.w.win + (slot0 + A.slot[dd]) * A.w.win_stride;
    if (wv == (dd & 3)) {
      if (anyd && fitsd && Wd <= 63) {
        const int64_t dg = (lane < Wd) ? (int64_t)atomicExch((unsigned long long*)&gwd[lane], 0ull) : 0;
        const Num<L> res = wave_round<L>(dg, (int64_t)amin[dd] - 64 * L, st);
        if (lane == 0) store_dev<L>(res, o.limb, o.hdr, o.ld, 0);
      } else if (!(anyd && fitsd) && lane == 0) {
        Num<L> res;
        set_zero(res, 0);
        store_dev<L>(res, o.limb, o.hdr, o.ld, 0);
      }
    }
    if (anyd && fitsd && Wd > 63) {  // block-uniform
      __syncthreads();
      for (int w = t; w < Wd; w += kDotThreads)
        s_win[w] = (int64_t)atomicExch((unsigned long long*)&gwd[w], 0ull);
      __syncthreads();
      if (t == 0) {
        Num<L> res;
        if (Wd <= WMAXF) {
          RegWindow<WMAXF> R;
          reg_normalize<WMAXF>(s_win, 1, Wd, R);
#pragma unroll
          for (int w = 0; w < WMAXF; ++w)
            if (w < Wd) s_win[w] = (int64_t)R.limb[w];
          res = limbs_round<L>(s_win, R.nl, R.neg, (int64_t)amin[dd] - 64 * L, st);
        } else {
          res = window_finalize<L>(s_win, 1, Wd, (int64_t)amin[dd] - 64 * L, st);
        }
        store_dev<L>(res, o.limb, o.hdr, o.ld, 0);
      }
    }
  }
  if (ctl && st) atomicOr(&ctl->flags, st);
  // every result is stored before the epilogue reads them
  wait_memory();
  __syncthreads();
  if (t == 0) {
    st_dev(ticket, 0u);
    uint32_t st2 = 0;
    const int was_done = ctl ? ctl->done : 0;
    epilogue<L>(A.epi, S, ctl, A.hist, st2);
    if (ctl && st2) atomicOr(&ctl->flags, st2);
    if (A.batch.ndone && ctl && !was_done && ctl->done) atomicAdd(A.batch.ndone, 1);
    st |= st2;
  }
  if (st) atomicOr(A.status, st);
}

// Anchors of stand-alone inner products (no producing kernel): one pass over the headers.
struct AnchorArgs {
  int64_t n;
  int nd;
  VecRef x[kDotMaxND];
  VecRef y[kDotMaxND];
  int slot[kDotMaxND];
  int32_t* anchor;
};

static __global__ void __launch_bounds__(256) dot_anchor_kernel(AnchorArgs A) {
  for (int d = 0; d < A.nd; ++d) {
    int32_t emin = INT32_MAX, emax = INT32_MIN;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < A.n;
         i += (int64_t)gridDim.x * blockDim.x)
      pair_exponent(A.x[d].hdr[i], A.y[d].hdr[i], emin, emax);
    anchor_publish(A.anchor, A.slot[d], emin, emax);
  }
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
// Element-wise kernels (one element per thread, grid-stride).
// ------------------------------------------------------------------------------------------
struct VecArgs {
  int64_t n;
  VecRef v[8];
  Scalars S;
  Ctl* ctl;
  uint32_t* status;
  int32_t* anchor;  // nullable: inner-product anchors filled for the products this kernel makes
  int aslot[2];
  BatchMap batch;   // batch: n is whole tiles and the grid has n / blockDim.x blocks
};

// The solve a block works for: its control block, scalars and first inner-product slot.
struct EwCtx {
  Ctl* ctl;
  Scalars S;
  int abase;
};

MPD EwCtx ew_ctx(const VecArgs& A) {
  const int pair =
      A.batch.pair_of_tile ? A.batch.pair_of_tile[((int64_t)blockIdx.x * blockDim.x) / kTile] : 0;
  EwCtx c;
  c.ctl = A.ctl ? A.ctl + pair : nullptr;
  c.S = A.S.at(pair);
  c.abase = pair * kDotSlots;
  return c;
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

// v0 <- v1, and the anchors of (v1, v1) and (v0, v1) = (v1, v1) (the solver setup's rt = r)
template <int L>
__global__ void __launch_bounds__(256) copy_anchor_kernel(VecArgs A) {
  const EwCtx c = ew_ctx(A);
  if (solve_done(c.ctl)) return;
  int32_t a0 = INT32_MAX, b0 = INT32_MIN;
  MP_ELEMENTWISE_LOOP(A) {
    const Num<L> r = vload<L>(A.v[1], i);
    vstore<L>(A.v[0], i, r);
    const int32_t h = make_hdr(r.e, r.s);
    pair_exponent(h, h, a0, b0);
  }
  if (A.anchor) {
    anchor_publish(A.anchor, c.abase + A.aslot[0], a0, b0);
    anchor_publish(A.anchor, c.abase + A.aslot[1], a0, b0);
  }
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
    const Num<L> r = vload<L>(A.v[2], i), rt = vload<L>(A.v[3], i);
    if (first) {
      vstore<L>(A.v[0], i, r);
      vstore<L>(A.v[1], i, rt);
    } else {
      vstore<L>(A.v[0], i, add_rn<L>(r, mul_rn<L>(beta, vload<L>(A.v[0], i), st), st));
      vstore<L>(A.v[1], i, add_rn<L>(rt, mul_rn<L>(beta, vload<L>(A.v[1], i), st), st));
    }
  }
  if (st) atomicOr(A.status, st);
}

// BiCG update: v = {x, r, rt, p, z, zt}: x += alpha p; r -= alpha z; rt -= alpha zt.
template <int L>
__global__ void __launch_bounds__(256) bicg_update_kernel(VecArgs A) {
  const EwCtx c = ew_ctx(A);
  if (solve_done(c.ctl)) return;
  uint32_t st = 0;
  const Num<L> alpha = sload<L>(c.S, S_ALPHA);
  int32_t a0 = INT32_MAX, b0 = INT32_MIN, a1 = INT32_MAX, b1 = INT32_MIN;
  MP_ELEMENTWISE_LOOP(A) {
    vstore<L>(A.v[0], i, add_rn<L>(vload<L>(A.v[0], i), mul_rn<L>(alpha, vload<L>(A.v[3], i), st), st));
    const Num<L> r = sub_rn<L>(vload<L>(A.v[1], i), mul_rn<L>(alpha, vload<L>(A.v[4], i), st), st);
    vstore<L>(A.v[1], i, r);
    const Num<L> rt = sub_rn<L>(vload<L>(A.v[2], i), mul_rn<L>(alpha, vload<L>(A.v[5], i), st), st);
    vstore<L>(A.v[2], i, rt);
    const int32_t hr = make_hdr(r.e, r.s), hrt = make_hdr(rt.e, rt.s);
    pair_exponent(hr, hr, a0, b0);
    pair_exponent(hrt, hr, a1, b1);
  }
  if (A.anchor) {
    anchor_publish(A.anchor, c.abase + A.aslot[0], a0, b0);
    anchor_publish(A.anchor, c.abase + A.aslot[1], a1, b1);
  }
  if (st) atomicOr(A.status, st);
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
    const Num<L> r = vload<L>(A.v[2], i);
    if (first) {
      vstore<L>(A.v[0], i, r);
    } else {
      const Num<L> q = vload<L>(A.v[4], i);
      vstore<L>(A.v[1], i, add_rn<L>(vload<L>(A.v[3], i), mul_rn<L>(beta, q, st), st));
      const Num<L> pmu = sub_rn<L>(vload<L>(A.v[0], i), vload<L>(A.v[5], i), st);
      vstore<L>(A.v[0], i, add_rn<L>(r, mul_rn<L>(beta, pmu, st), st));
    }
  }
  if (st) atomicOr(A.status, st);
}

// GPBiCG t, s, y: v = {t, s, y, r, q, w}.  s = t - r (not in the first iteration),
// t = r - alpha q, y = alpha q - r (first) or s - alpha (w - q).
template <int L>
__global__ void __launch_bounds__(256) gp_tsy_kernel(VecArgs A) {
  const EwCtx c = ew_ctx(A);
  if (solve_done(c.ctl)) return;
  uint32_t st = 0;
  const bool first = c.ctl->iters == 0;
  const Num<L> alpha = sload<L>(c.S, S_ALPHA);
  int32_t a0 = INT32_MAX, b0 = INT32_MIN, a1 = INT32_MAX, b1 = INT32_MIN;
  MP_ELEMENTWISE_LOOP(A) {
    const Num<L> r = vload<L>(A.v[3], i), q = vload<L>(A.v[4], i);
    const Num<L> aq = mul_rn<L>(alpha, q, st);
    Num<L> s;
    if (!first) {
      s = sub_rn<L>(vload<L>(A.v[0], i), r, st);
      vstore<L>(A.v[1], i, s);
    }
    const Num<L> tn = sub_rn<L>(r, aq, st);
    vstore<L>(A.v[0], i, tn);
    Num<L> y;
    if (first) {
      y = sub_rn<L>(aq, r, st);
    } else {
      const Num<L> wq = sub_rn<L>(vload<L>(A.v[5], i), q, st);
      y = sub_rn<L>(s, mul_rn<L>(alpha, wq, st), st);
    }
    vstore<L>(A.v[2], i, y);
    const int32_t hy = make_hdr(y.e, y.s), ht = make_hdr(tn.e, tn.s);
    pair_exponent(hy, hy, a0, b0);
    pair_exponent(hy, ht, a1, b1);
  }
  if (A.anchor) {
    anchor_publish(A.anchor, c.abase + A.aslot[0], a0, b0);
    anchor_publish(A.anchor, c.abase + A.aslot[1], a1, b1);
  }
  if (st) atomicOr(A.status, st);
}

// GPBiCG update: v = {u, z, x, r, q, s, p, t} and v2 = {y, v} in w[]:
// u = zeta q + eta (s + beta u); z = zeta r + eta z - alpha u; x = x + alpha p + z;
// r = t - eta y - zeta v.
struct GpUpdArgs {
  VecArgs a;
  VecRef y, v, rt;
};

template <int L>
__global__ void __launch_bounds__(256) gp_update_kernel(GpUpdArgs G) {
  const VecArgs& A = G.a;
  const EwCtx c = ew_ctx(A);
  if (solve_done(c.ctl)) return;
  uint32_t st = 0;
  const Num<L> alpha = sload<L>(c.S, S_ALPHA), beta = sload<L>(c.S, S_BETA);
  const Num<L> zeta = sload<L>(c.S, S_ZETA), eta = sload<L>(c.S, S_ETA);
  int32_t a0 = INT32_MAX, b0 = INT32_MIN, a1 = INT32_MAX, b1 = INT32_MIN;
  MP_ELEMENTWISE_LOOP(A) {
    const Num<L> q = vload<L>(A.v[4], i), s = vload<L>(A.v[5], i);
    const Num<L> u_old = vload<L>(A.v[0], i);
    const Num<L> u = add_rn<L>(mul_rn<L>(zeta, q, st),
                               mul_rn<L>(eta, add_rn<L>(s, mul_rn<L>(beta, u_old, st), st), st), st);
    vstore<L>(A.v[0], i, u);
    const Num<L> r = vload<L>(A.v[3], i);
    const Num<L> z = sub_rn<L>(add_rn<L>(mul_rn<L>(zeta, r, st), mul_rn<L>(eta, vload<L>(A.v[1], i), st), st),
                               mul_rn<L>(alpha, u, st), st);
    vstore<L>(A.v[1], i, z);
    const Num<L> x = add_rn<L>(add_rn<L>(vload<L>(A.v[2], i), mul_rn<L>(alpha, vload<L>(A.v[6], i), st), st), z, st);
    vstore<L>(A.v[2], i, x);
    const Num<L> t = vload<L>(A.v[7], i);
    const Num<L> rn = sub_rn<L>(sub_rn<L>(t, mul_rn<L>(eta, vload<L>(G.y, i), st), st),
                                mul_rn<L>(zeta, vload<L>(G.v, i), st), st);
    vstore<L>(A.v[3], i, rn);
    const int32_t hr = make_hdr(rn.e, rn.s), hrt = G.rt.hdr[i];
    pair_exponent(hr, hr, a0, b0);
    pair_exponent(hrt, hr, a1, b1);
  }
  if (A.anchor) {
    anchor_publish(A.anchor, c.abase + A.aslot[0], a0, b0);
    anchor_publish(A.anchor, c.abase + A.aslot[1], a1, b1);
  }
  if (st) atomicOr(A.status, st);
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
