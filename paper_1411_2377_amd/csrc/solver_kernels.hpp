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

struct Scalars {
  uint32_t* limb;  // [L][kNumScalars]
  int32_t* hdr;    // [kNumScalars]
};

struct VecRef {
  uint32_t* limb;
  int32_t* hdr;
  int64_t ld;
};

template <int L>
MPD Num<L> sload(const Scalars& S, int slot) {
  Num<L> r;
  load<L>(r, S.limb, S.hdr, kNumScalars, slot);
  return r;
}

template <int L>
MPD void sstore(const Scalars& S, int slot, const Num<L>& v) {
  store<L>(v, S.limb, S.hdr, kNumScalars, slot);
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
// Driver epilogues, run by one thread after the inner products of a step are known.
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
      const Num<L> q0 = sload<L>(S, S_Q0);
      const Num<L> nrm0 = sqrt_rn<L>(q0, st);
      const Num<L> thr = add_rn<L>(mul_rn<L>(sload<L>(S, S_CREL), nrm0, st), sload<L>(S, S_CABS), st);
      sstore<L>(S, S_NRM0, nrm0);
      sstore<L>(S, S_THR, thr);
      if (sqrt_le<L>(q0, thr)) {
        finish(ctl, kConverged);
      } else if (ctl->maxit <= 0) {
        finish(ctl, kNotConverged);
      } else if (is_zero(sload<L>(S, S_RHO))) {
        finish(ctl, kBreakRho);
      }
      break;
    }
    case EPI_BICG_SIGMA: {
      const Num<L> sigma = sload<L>(S, S_SIGMA);
      if (is_zero(sigma)) {
        finish(ctl, kBreakSigma);
      } else {
        sstore<L>(S, S_ALPHA, div_rn<L>(sload<L>(S, S_RHO), sigma, st));
      }
      break;
    }
    case EPI_GP_ALPHA: {
      const Num<L> den = sload<L>(S, S_DEN);
      if (is_zero(den)) {
        finish(ctl, kBreakSigma);
      } else {
        sstore<L>(S, S_ALPHA, div_rn<L>(sload<L>(S, S_RHO), den, st));
      }
      break;
    }
    case EPI_GP_ZETA: {
      const Num<L> mu1 = sload<L>(S, S_MU1), mu2 = sload<L>(S, S_MU2), mu3 = sload<L>(S, S_MU3);
      const Num<L> mu4 = sload<L>(S, S_MU4), mu5 = sload<L>(S, S_MU5);
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
      const Num<L> q = sload<L>(S, S_Q);
      const int i = ctl->iters + 1;
      if (hist.limb && i - 1 < ctl->hist_len) vstore<L>(hist, i - 1, q);
      ctl->iters = i;
      if (sqrt_le<L>(q, sload<L>(S, S_THR))) {
        finish(ctl, kConverged);
        break;
      }
      if (epi == EPI_GP_CONV && is_zero(sload<L>(S, S_ZETA))) {
        finish(ctl, kBreakZeta);
        break;
      }
      if (i >= ctl->maxit) {
        finish(ctl, kNotConverged);
        break;
      }
      const Num<L> rho = sload<L>(S, S_RHO);
      const Num<L> rho_next = sload<L>(S, S_RHO_NEXT);
      sstore<L>(S, S_RHO_OLD, rho);
      sstore<L>(S, S_RHO, rho_next);
      if (is_zero(rho_next)) {
        finish(ctl, kBreakRho);
        break;
      }
      if (epi == EPI_BICG_CONV) {
        sstore<L>(S, S_BETA, div_rn<L>(rho_next, rho, st));
      } else {
        const Num<L> alpha = sload<L>(S, S_ALPHA), zeta = sload<L>(S, S_ZETA);
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
// Exact inner products: up to kDotMaxND dots of length n in one launch (256-thread blocks).
// Each block forms the exact products of its elements in per-lane carry-save windows anchored
// at the block's smallest product exponent, sums the lane windows digit by digit, normalises
// the block sum to sign + magnitude limbs and writes that record out.  The last block to finish
// (integer ticket) aligns all records into one window, rounds once, stores the result and runs
// the driver epilogue.  Lane windows are padded to an odd stride so that both the per-lane
// adds and the per-digit sums hit distinct LDS banks.
// ------------------------------------------------------------------------------------------
constexpr int kDotMaxND = 5;
constexpr int kDotMaxBlocks = 128;
constexpr int kDotThreads = 256;
constexpr int kDotStride = kDotThreads + 1;

template <int L>
constexpr int dot_window_digits() { return window_fast_digits<L>(); }

// block-shared window capacity (the per-lane windows' LDS reused as one array)
template <int L>
constexpr int dot_shared_digits() { return window_fast_digits<L>() * kDotStride; }

template <int L>
constexpr int dot_rec_ints() { return 3 + dot_shared_digits<L>(); }

struct DotArgs {
  int64_t n;
  int nd;
  VecRef x[kDotMaxND];
  VecRef y[kDotMaxND];
  VecRef out[kDotMaxND];  // result d goes to element 0 of out[d]
  Scalars S;
  int32_t* part;     // [gridDim][kDotMaxND][dot_rec_ints]
  uint32_t* ticket;  // zero before the launch, reset by the last block
  Ctl* ctl;          // nullable
  uint32_t* status;
  int epi;
  VecRef hist;
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

MPD int64_t wave_max64(int64_t v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    const int64_t t = __shfl_xor(v, o);
    v = t > v ? t : v;
  }
  return v;
}

template <int L>
__global__ void __launch_bounds__(kDotThreads) dot_kernel(DotArgs A) {
  constexpr int WF = dot_window_digits<L>();
  constexpr int WB = dot_shared_digits<L>();
  constexpr int REC = dot_rec_ints<L>();
  constexpr int kRecPre = 3 + WF;          // record words staged in LDS by the last block
  constexpr int WMAXF = 2 * L + 16;        // final windows up to this size stay in registers
  static_assert(64 + (kDotMaxBlocks * kRecPre + 1) / 2 <= WB, "record staging must fit");
  __shared__ int64_t s_win[WB];
  // the last block stages record heads behind the first 64 window digits
  int32_t(*s_rec)[kRecPre] = reinterpret_cast<int32_t(*)[kRecPre]>(s_win + 64);
  __shared__ int64_t s_red[2][kDotThreads / 64];
  __shared__ int64_t s_part[kDotThreads / 64][64];
  __shared__ uint32_t s_last;
  if (solve_done(A.ctl)) return;
  const int t = threadIdx.x;
  const int wave = t >> 6;
  uint32_t st = 0;
  const int64_t stride = (int64_t)gridDim.x * kDotThreads;
  const int64_t first = (int64_t)blockIdx.x * kDotThreads + t;
  const int d = blockIdx.y;  // the dots of one launch run side by side, one grid row each

  do {
    const VecRef X = A.x[d], Y = A.y[d];
    // exponent range of the block's non-zero products
    int32_t emin = INT32_MAX, emax = INT32_MIN;
    for (int64_t i = first; i < A.n; i += stride) {
      const int32_t hx = X.hdr[i], hy = Y.hdr[i];
      if (!hdr_is_zero(hx) && !hdr_is_zero(hy)) {
        const int32_t e = (hx >> 1) + (hy >> 1);
        emin = min(emin, e);
        emax = max(emax, e);
      }
    }
    emin = wave_min(emin);
    emax = wave_max(emax);
    if ((t & 63) == 0) {
      s_red[0][wave] = emin;
      s_red[1][wave] = emax;
    }
    __syncthreads();
#pragma unroll
    for (int w = 0; w < kDotThreads / 64; ++w) {
      emin = min(emin, (int32_t)s_red[0][w]);
      emax = max(emax, (int32_t)s_red[1][w]);
    }
    __syncthreads();
    int32_t* rec = A.part + ((int64_t)blockIdx.x * kDotMaxND + d) * REC;
    if (emax < emin) {
      if (t == 0) rec[0] = 0;
      break;
    }
    const int W = window_digits<L>(emin, emax);
    if (W > WB) {
      st |= kStWindow;
      if (t == 0) rec[0] = 0;
      break;
    }
    const bool fast = W <= WF;
    if (fast) {
      for (int w = 0; w < WF; ++w) s_win[w * kDotStride + t] = 0;
    } else {
      for (int w = t; w < W; w += kDotThreads) s_win[w] = 0;
      __syncthreads();
    }
    // products, two elements at a time: both headers, then both limb sets in flight together
    for (int64_t i0 = first; i0 < A.n; i0 += 2 * stride) {
      const int64_t i1 = i0 + stride;
      const bool has1 = i1 < A.n;
      const int32_t hx0 = X.hdr[i0], hy0 = Y.hdr[i0];
      const int32_t hx1 = has1 ? X.hdr[i1] : (int32_t)0x80000000, hy1 = has1 ? Y.hdr[i1] : (int32_t)0x80000000;
      const bool nz0 = !hdr_is_zero(hx0) && !hdr_is_zero(hy0);
      const bool nz1 = !hdr_is_zero(hx1) && !hdr_is_zero(hy1);
      uint32_t x0[L], y0[L], x1[L], y1[L];
#pragma unroll
      for (int q = 0; q < L; ++q) {
        x0[q] = nz0 ? X.limb[(int64_t)q * X.ld + i0] : 0u;
        y0[q] = nz0 ? Y.limb[(int64_t)q * Y.ld + i0] : 0u;
        x1[q] = nz1 ? X.limb[(int64_t)q * X.ld + i1] : 0u;
        y1[q] = nz1 ? Y.limb[(int64_t)q * Y.ld + i1] : 0u;
      }
      if (nz0) {
        uint32_t pr[2 * L];
        mul_full<L>(x0, y0, pr);
        const uint32_t off = (uint32_t)((hx0 >> 1) + (hy0 >> 1) - emin);
        if (fast) window_add<L>(s_win + t, kDotStride, pr, (uint32_t)(hx0 ^ hy0) & 1u, off);
        else window_add_atomic<L>(s_win, pr, (uint32_t)(hx0 ^ hy0) & 1u, off);
      }
      if (nz1) {
        uint32_t pr[2 * L];
        mul_full<L>(x1, y1, pr);
        const uint32_t off = (uint32_t)((hx1 >> 1) + (hy1 >> 1) - emin);
        if (fast) window_add<L>(s_win + t, kDotStride, pr, (uint32_t)(hx1 ^ hy1) & 1u, off);
        else window_add_atomic<L>(s_win, pr, (uint32_t)(hx1 ^ hy1) & 1u, off);
      }
    }
    __syncthreads();
    if (fast) {
      // digit w is summed over the 256 lane windows by TPD consecutive threads (an odd row
      // stride keeps their reads on distinct banks), then combined with shuffles
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
      __syncthreads();
      if (w < W && sub == 0) s_win[w] = dsum;
      __syncthreads();
    }
    // normalise the block sum to sign + magnitude limbs (one lane)
    if (t == 0 && fast) {
      RegWindow<WF> R;
      reg_normalize<WF>(s_win, 1, W, R);
      rec[1] = emin;
      rec[2] = R.nl;
#pragma unroll
      for (int w = 0; w < WF; ++w)
        if (w < R.nl) rec[3 + w] = (int32_t)R.limb[w];
      rec[0] = R.nl ? (1 | ((int)R.neg << 1)) : 0;
    } else if (t == 0) {
      int64_t c = 0;
      for (int w = 0; w < W; ++w) {
        const int64_t v = s_win[w] + c;
        s_win[w] = (int64_t)(uint32_t)v;
        c = v >> 32;
      }
      const int neg = c < 0;
      if (neg) {
        uint32_t cy = 1;
        for (int w = 0; w < W; ++w) s_win[w] = (int64_t)__builtin_addc(~(uint32_t)s_win[w], 0u, cy, &cy);
      }
      int nl = W;
      while (nl > 0 && (uint32_t)s_win[nl - 1] == 0u) --nl;
      rec[1] = emin;
      rec[2] = nl;
      for (int w = 0; w < nl; ++w) rec[3 + w] = (int32_t)(uint32_t)s_win[w];
      rec[0] = nl ? (1 | (neg << 1)) : 0;
    }
    __syncthreads();
  } while (false);

  __threadfence();
  if (t == 0) s_last = (atomicAdd(&A.ticket[d], 1u) == gridDim.x - 1) ? 1u : 0u;
  __syncthreads();
  if (!s_last) {
    if (st) atomicOr(A.status, st);
    return;
  }
  __threadfence();
  const int G = gridDim.x;
  {
    // stage the head of every block record in LDS with independent coalesced loads (the fence
    // above makes the other blocks' writes visible); longer records are read on from memory
#pragma unroll 4
    for (int idx = t; idx < G * kRecPre; idx += kDotThreads) {
      const int b = idx / kRecPre, j = idx - b * kRecPre;
      s_rec[b][j] = A.part[((int64_t)b * kDotMaxND + d) * REC + j];
    }
    __syncthreads();
    int32_t gmin = INT32_MAX;
    int64_t gtop = INT64_MIN;
    for (int b = t; b < G; b += kDotThreads) {
      if (s_rec[b][0] & 1) {
        gmin = min(gmin, s_rec[b][1]);
        gtop = max(gtop, (int64_t)s_rec[b][1] + 32 * (int64_t)s_rec[b][2]);
      }
    }
    gmin = wave_min(gmin);
    gtop = wave_max64(gtop);
    if ((t & 63) == 0) {
      s_red[0][wave] = gmin;
      s_red[1][wave] = gtop;
    }
    __syncthreads();
#pragma unroll
    for (int w = 0; w < kDotThreads / 64; ++w) {
      gmin = min(gmin, (int32_t)s_red[0][w]);
      gtop = s_red[1][w] > gtop ? s_red[1][w] : gtop;
    }
    __syncthreads();
    Num<L> res;
    set_zero(res, 0);
    const int Wg = gtop != INT64_MIN ? (int)((gtop - (int64_t)gmin) >> 5) + 2 : 0;
    if (Wg > WB) st |= kStWindow;
    // a final window wider than 64 digits overwrites the staged records: read them from memory
    const bool staged = Wg <= 64;
    __syncthreads();
    if (Wg > 0 && Wg <= WB) {
      for (int w = t; w < Wg; w += kDotThreads) s_win[w] = 0;
      __syncthreads();
      // each lane adds its records, shifted to the common anchor, with integer LDS atomics
      for (int b = t; b < G; b += kDotThreads) {
        const int32_t* far = A.part + ((int64_t)b * kDotMaxND + d) * REC;
        const int32_t fl = staged ? s_rec[b][0] : far[0];
        if (!(fl & 1)) continue;
        const uint32_t off = (uint32_t)((staged ? s_rec[b][1] : far[1]) - gmin);
        const int nl = staged ? s_rec[b][2] : far[2];
        const int q = (int)(off >> 5);
        const uint32_t r = off & 31u;
        auto limb = [&](int j) -> uint32_t {
          if (j < 0 || j >= nl) return 0u;
          return (staged && 3 + j < kRecPre) ? (uint32_t)s_rec[b][3 + j] : (uint32_t)far[3 + j];
        };
        // start each record at a different digit so that the lanes' atomics spread over banks
        for (int jj = 0; jj <= nl; ++jj) {
          int j = jj + b;
          j %= (nl + 1);
          const uint32_t cur = limb(j), prev = limb(j - 1);
          const uint32_t v = r ? fshr(cur, prev, 32u - r) : cur;
          if (v) {
            const uint64_t add = (fl & 2) ? (uint64_t)(-(int64_t)v) : (uint64_t)v;
            atomicAdd((unsigned long long*)&s_win[q + j], (unsigned long long)add);
          }
        }
      }
      __syncthreads();
      if (t == 0) {
        if (Wg <= WMAXF) {
          // carries in registers, then the rounding reads the limbs back from LDS
          RegWindow<WMAXF> R;
          reg_normalize<WMAXF>(s_win, 1, Wg, R);
#pragma unroll
          for (int w = 0; w < WMAXF; ++w)
            if (w < Wg) s_win[w] = (int64_t)R.limb[w];
          res = limbs_round<L>(s_win, R.nl, R.neg, (int64_t)gmin - 64 * L, st);
        } else {
          res = window_finalize<L>(s_win, 1, Wg, (int64_t)gmin - 64 * L, st);
        }
      }
    }
    if (t == 0) vstore<L>(A.out[d], 0, res);
  }
  if (t == 0) {
    A.ticket[d] = 0;
    if (A.ctl && st) atomicOr(&A.ctl->flags, st);
    // the last dot to finish runs the driver epilogue
    __threadfence();
    if (atomicAdd(&A.ticket[kDotMaxND], 1u) == (unsigned)A.nd - 1) {
      __threadfence();
      uint32_t st2 = 0;
      epilogue<L>(A.epi, A.S, A.ctl, A.hist, st2);
      A.ticket[kDotMaxND] = 0;
      if (A.ctl && st2) atomicOr(&A.ctl->flags, st2);
      st |= st2;
    }
  }
  if (st) atomicOr(A.status, st);
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
};

// The scalar slot as a one-element vector reference.
__host__ __device__ inline VecRef slot_ref(const Scalars& S, int slot) {
  VecRef r;
  r.limb = S.limb + slot;
  r.hdr = S.hdr + slot;
  r.ld = kNumScalars;
  return r;
}

#define MP_ELEMENTWISE_LOOP(A) \
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (A).n; \
       i += (int64_t)gridDim.x * blockDim.x)

// v0 <- v0 + v2[0] * v1   (mp_axpy: y <- y + alpha x)
template <int L>
__global__ void __launch_bounds__(256) axpy_kernel(VecArgs A) {
  if (solve_done(A.ctl)) return;
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
  if (solve_done(A.ctl)) return;
  MP_ELEMENTWISE_LOOP(A) { vstore<L>(A.v[0], i, vload<L>(A.v[1], i)); }
}

// v0 <- +0
template <int L>
__global__ void __launch_bounds__(256) zero_kernel(VecArgs A) {
  if (solve_done(A.ctl)) return;
  Num<L> z;
  set_zero(z, 0);
  MP_ELEMENTWISE_LOOP(A) { vstore<L>(A.v[0], i, z); }
}

// v0 <- v1 - v2
template <int L>
__global__ void __launch_bounds__(256) sub_kernel(VecArgs A) {
  if (solve_done(A.ctl)) return;
  uint32_t st = 0;
  MP_ELEMENTWISE_LOOP(A) { vstore<L>(A.v[0], i, sub_rn<L>(vload<L>(A.v[1], i), vload<L>(A.v[2], i), st)); }
  if (st) atomicOr(A.status, st);
}

// BiCG directions: v = {p, pt, r, rt}. First iteration p = r, pt = rt; then p = r + beta p.
template <int L>
__global__ void __launch_bounds__(256) bicg_dir_kernel(VecArgs A) {
  if (solve_done(A.ctl)) return;
  uint32_t st = 0;
  const bool first = A.ctl->iters == 0;
  const Num<L> beta = sload<L>(A.S, S_BETA);
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
  if (solve_done(A.ctl)) return;
  uint32_t st = 0;
  const Num<L> alpha = sload<L>(A.S, S_ALPHA);
  MP_ELEMENTWISE_LOOP(A) {
    vstore<L>(A.v[0], i, add_rn<L>(vload<L>(A.v[0], i), mul_rn<L>(alpha, vload<L>(A.v[3], i), st), st));
    vstore<L>(A.v[1], i, sub_rn<L>(vload<L>(A.v[1], i), mul_rn<L>(alpha, vload<L>(A.v[4], i), st), st));
    vstore<L>(A.v[2], i, sub_rn<L>(vload<L>(A.v[2], i), mul_rn<L>(alpha, vload<L>(A.v[5], i), st), st));
  }
  if (st) atomicOr(A.status, st);
}

// GPBiCG direction: v = {p, w, r, v, q, u}.  First iteration p = r; then
// w = v + beta q, p = r + beta (p - u).
template <int L>
__global__ void __launch_bounds__(256) gp_dir_kernel(VecArgs A) {
  if (solve_done(A.ctl)) return;
  uint32_t st = 0;
  const bool first = A.ctl->iters == 0;
  const Num<L> beta = sload<L>(A.S, S_BETA);
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
  if (solve_done(A.ctl)) return;
  uint32_t st = 0;
  const bool first = A.ctl->iters == 0;
  const Num<L> alpha = sload<L>(A.S, S_ALPHA);
  MP_ELEMENTWISE_LOOP(A) {
    const Num<L> r = vload<L>(A.v[3], i), q = vload<L>(A.v[4], i);
    const Num<L> aq = mul_rn<L>(alpha, q, st);
    Num<L> s;
    if (!first) {
      s = sub_rn<L>(vload<L>(A.v[0], i), r, st);
      vstore<L>(A.v[1], i, s);
    }
    vstore<L>(A.v[0], i, sub_rn<L>(r, aq, st));
    if (first) {
      vstore<L>(A.v[2], i, sub_rn<L>(aq, r, st));
    } else {
      const Num<L> wq = sub_rn<L>(vload<L>(A.v[5], i), q, st);
      vstore<L>(A.v[2], i, sub_rn<L>(s, mul_rn<L>(alpha, wq, st), st));
    }
  }
  if (st) atomicOr(A.status, st);
}

// GPBiCG update: v = {u, z, x, r, q, s, p, t} and v2 = {y, v} in w[]:
// u = zeta q + eta (s + beta u); z = zeta r + eta z - alpha u; x = x + alpha p + z;
// r = t - eta y - zeta v.
struct GpUpdArgs {
  VecArgs a;
  VecRef y, v;
};

template <int L>
__global__ void __launch_bounds__(256) gp_update_kernel(GpUpdArgs G) {
  const VecArgs& A = G.a;
  if (solve_done(A.ctl)) return;
  uint32_t st = 0;
  const Num<L> alpha = sload<L>(A.S, S_ALPHA), beta = sload<L>(A.S, S_BETA);
  const Num<L> zeta = sload<L>(A.S, S_ZETA), eta = sload<L>(A.S, S_ETA);
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
  }
  if (st) atomicOr(A.status, st);
}

// Write a constant into element 0 of a vector or a scalar slot (kernel arguments carry it).
template <int L>
struct ConstArgs {
  VecRef out;
  uint32_t m[L];
  int32_t hdr;
};

template <int L>
__global__ void set_scalar_kernel(ConstArgs<L> A) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    A.out.hdr[0] = A.hdr;
#pragma unroll
    for (int k = 0; k < L; ++k) A.out.limb[(int64_t)k * A.out.ld] = A.m[k];
  }
}

// Initialise a solve's control block.
static __global__ void ctl_init_kernel(Ctl* ctl, int32_t maxit, int32_t hist_len) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    ctl->done = 0;
    ctl->status = kNotConverged;
    ctl->iters = 0;
    ctl->maxit = maxit;
    ctl->flags = 0;
    ctl->hist_len = hist_len;
  }
}

}  // namespace mp
