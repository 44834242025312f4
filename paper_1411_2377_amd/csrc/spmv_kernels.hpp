// Multiple-precision CSR sparse matrix-vector product kernels (y = A x).
//
// The paper's SpMV (Kouya, Sec. 2 and Sec. 3) is a loop of p-bit multiplies and adds over the
// stored entries of each CSR row.  Two deterministic accumulation modes are provided:
//   SEQ   y_i <- +0; y_i <- RN(y_i + RN(a_ij x_j)) over the row's entries in storage (ascending
//         column) order: the per-operation rounding of an MPFR loop.
//   EXACT y_i = RN(sum_j a_ij x_j): exact fixed-point accumulation, one final rounding.
//
// Work decomposition (one wavefront per block, 64 rows per block, lane l owns row r0 + l):
//   phase 1  the block's contiguous entry range is cut into chunks of CHUNK entries; consecutive
//            lanes take consecutive entries (coalesced structure-of-arrays limb loads, x
//            gathered), form the product (rounded for SEQ, exact 2L limbs for EXACT) and stage
//            it in LDS.  Products of stored zeros are not formed (zero fast path).
//   phase 2  each lane folds its own row's staged products in order: serial RN adds (SEQ), or
//            carry-save adds into its private LDS window (EXACT).
// EXACT rows whose products span more exponent range than the per-lane window holds are done
// afterwards by the whole block with a shared window (atomic carry-save adds); a row that does
// not fit even there raises kStWindow.
#pragma once
#include "mp_core.hpp"
#include "mp_exact.hpp"

namespace mp {

constexpr int kRowsPerBlock = 64;
// entries staged per phase-1 chunk (about 8 KB of rounded products in LDS at every precision)
template <int L>
constexpr int chunk_entries() { return 2048 / L; }

struct SpmvArgs {
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
  uint32_t* status;
  const int32_t* done;  // nullable: a set flag turns the launch into a no-op (solver graphs)
  // inner-product anchors for products of y with up to three vectors (pair_hdr[k] == nullptr
  // means y itself): the exponent range of y_i * w_i over the rows, published to anchor slots
  int npair;
  const int32_t* pair_hdr[3];
  int pair_slot[3];
  int32_t* anchor;
  // several right-hand sides / independent solves (nrhs == 1 and pair_of_tile == nullptr: one)
  int nrhs;                      // block b works on row block b / nrhs for right-hand side b % nrhs
  int64_t x_rstride, y_rstride;  // element offset between right-hand sides in x and y
  const int32_t* pair_of_tile;   // solve of each 512-element tile of y (done flags, anchors)
  const int32_t* done_base;      // &ctl[0].done; solve k's flag at done_base[k * done_stride]
  int64_t done_stride;
  int slots_per_pair;
};

// Row block, right-hand side and solve of this block; false if that solve is finished.
struct SpmvBlock {
  int64_t rb;
  int rhs;
  int pair;
};

MPD bool spmv_block(const SpmvArgs& A, SpmvBlock& B) {
  B.rhs = (int)(blockIdx.x % (unsigned)A.nrhs);
  B.rb = (int64_t)(blockIdx.x / (unsigned)A.nrhs);
  B.pair = 0;
  if (A.pair_of_tile) {
    B.pair = A.pair_of_tile[(B.rhs * A.y_rstride + B.rb * 64) / 512];
    if (*(volatile const int32_t*)&A.done_base[B.pair * A.done_stride]) return false;
  } else if (A.done && *(volatile const int32_t*)A.done) {
    return false;
  }
  return true;
}

// Fold row r's output header yh into the anchors of its requested products.
struct PairAcc {
  int32_t lo[3], hi[3];
};

MPD void pair_init(PairAcc& P) {
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    P.lo[k] = INT32_MAX;
    P.hi[k] = INT32_MIN;
  }
}

MPD void pair_fold(const SpmvArgs& A, PairAcc& P, int64_t row, int32_t yh) {
  // row: index into y (right-hand side offset included)
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    if (k < A.npair) {
      const int32_t hp = A.pair_hdr[k] ? A.pair_hdr[k][row] : yh;
      if (!hdr_is_zero(yh) && !hdr_is_zero(hp)) {
        const int32_t e = (yh >> 1) + (hp >> 1);
        P.lo[k] = min(P.lo[k], e);
        P.hi[k] = max(P.hi[k], e);
      }
    }
  }
}

MPD void pair_publish(const SpmvArgs& A, PairAcc& P, int pair) {
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    if (k < A.npair) {
      int32_t lo = P.lo[k], hi = P.hi[k];
#pragma unroll
      for (int o = 32; o >= 1; o >>= 1) {
        lo = min(lo, __shfl_xor(lo, o));
        hi = max(hi, __shfl_xor(hi, o));
      }
      if ((threadIdx.x & 63) == 0 && hi >= lo) {
        // bins of 64 per slot, spread by block (the inner-product kernel reduces them)
        const int64_t slot = (int64_t)pair * A.slots_per_pair + A.pair_slot[k];
        int32_t* a = A.anchor + 2 * (slot * 64 + (blockIdx.x & 63));
        atomicMin(&a[0], lo);
        atomicMax(&a[1], hi);
      }
    }
  }
}

template <int L>
__global__ void __launch_bounds__(64) spmv_seq_kernel(SpmvArgs A) {
  constexpr int kChunk = chunk_entries<L>();
  __shared__ int32_t s_rp[kRowsPerBlock + 1];
  __shared__ uint32_t s_m[L][kChunk];
  __shared__ int32_t s_e[kChunk];
  __shared__ uint32_t s_s[kChunk];

  SpmvBlock B;
  if (!spmv_block(A, B)) return;
  const int lane = threadIdx.x;
  const int64_t r0 = B.rb * kRowsPerBlock;
  const uint32_t* const x_limb = A.x_limb + B.rhs * A.x_rstride;
  const int32_t* const x_hdr = A.x_hdr + B.rhs * A.x_rstride;
  const int64_t yo = B.rhs * A.y_rstride;  // y (and paired vectors) offset of this right-hand side
  const int nr = (int)min((int64_t)kRowsPerBlock, A.n_rows - r0);
  for (int i = lane; i <= nr; i += 64) s_rp[i] = A.row_ptr[r0 + i];
  __syncthreads();
  const int kb = s_rp[0], ke = s_rp[nr];
  const bool has_row = lane < nr;
  const int rs = has_row ? s_rp[lane] : 0;
  const int re = has_row ? s_rp[lane + 1] : 0;
  uint32_t st = 0;
  Num<L> acc;
  set_zero(acc, 0);

  for (int c0 = kb; c0 < ke; c0 += kChunk) {
    const int cn = min(kChunk, ke - c0);
    for (int j = lane; j < cn; j += 64) {
      const int64_t k = c0 + j;
      const int32_t ha = A.a_hdr[k];
      const int32_t col = A.col_idx[k];
      const int32_t hx = x_hdr[col];
      Num<L> t;
      if (hdr_is_zero(ha) || hdr_is_zero(hx)) {
        set_zero(t, (uint32_t)(ha ^ hx) & 1u);
      } else {
        uint32_t am[L], xm[L], pr[2 * L];
#pragma unroll
        for (int q = 0; q < L; ++q) am[q] = A.a_limb[(int64_t)q * A.a_ld + k];
#pragma unroll
        for (int q = 0; q < L; ++q) xm[q] = x_limb[(int64_t)q * A.x_ld + col];
        mul_full<L>(am, xm, pr);
        round_product<L>(pr, (ha >> 1) + (hx >> 1), (uint32_t)(ha ^ hx) & 1u, t, st);
      }
#pragma unroll
      for (int q = 0; q < L; ++q) s_m[q][j] = t.m[q];
      s_e[j] = t.e;
      s_s[j] = t.s;
    }
    __syncthreads();
    const int lo = max(rs, c0), hi = min(re, c0 + cn);
    for (int k = lo; k < hi; ++k) {
      const int j = k - c0;
      Num<L> t;
#pragma unroll
      for (int q = 0; q < L; ++q) t.m[q] = s_m[q][j];
      t.e = s_e[j];
      t.s = s_s[j];
      acc = add_rn<L>(acc, t, st);
    }
    __syncthreads();
  }
  if (has_row) store<L>(acc, A.y_limb, A.y_hdr, A.y_ld, yo + r0 + lane);
  if (A.npair) {
    PairAcc P;
    pair_init(P);
    if (has_row) pair_fold(A, P, yo + r0 + lane, make_hdr(acc.e, acc.s));
    pair_publish(A, P, B.pair);
  }
  if (st) atomicOr(A.status, st);
}

template <int L>
__global__ void __launch_bounds__(64) spmv_exact_kernel(SpmvArgs A) {
  constexpr int WF = window_fast_digits<L>();
  constexpr int WB = WF * 64;  // digits of the shared window used for wide rows
  constexpr int kChunk = chunk_entries<L>();
  __shared__ int32_t s_rp[kRowsPerBlock + 1];
  __shared__ uint32_t s_p[2 * L][kChunk];
  __shared__ int32_t s_e[kChunk];
  __shared__ uint32_t s_s[kChunk];
  __shared__ int64_t s_win[WF * 64];

  SpmvBlock B;
  if (!spmv_block(A, B)) return;
  const int lane = threadIdx.x;
  const int64_t r0 = B.rb * kRowsPerBlock;
  const uint32_t* const x_limb = A.x_limb + B.rhs * A.x_rstride;
  const int32_t* const x_hdr = A.x_hdr + B.rhs * A.x_rstride;
  const int64_t yo = B.rhs * A.y_rstride;  // y (and paired vectors) offset of this right-hand side
  const int nr = (int)min((int64_t)kRowsPerBlock, A.n_rows - r0);
  for (int i = lane; i <= nr; i += 64) s_rp[i] = A.row_ptr[r0 + i];
  __syncthreads();
  const int kb = s_rp[0], ke = s_rp[nr];
  const bool has_row = lane < nr;
  const int rs = has_row ? s_rp[lane] : 0;
  const int re = has_row ? s_rp[lane + 1] : 0;
  uint32_t st = 0;

  // exponent range of this row's non-zero products
  int32_t emin = INT32_MAX, emax = INT32_MIN;
  for (int k = rs; k < re; ++k) {
    const int32_t ha = A.a_hdr[k];
    const int32_t hx = x_hdr[A.col_idx[k]];
    if (!hdr_is_zero(ha) && !hdr_is_zero(hx)) {
      const int32_t e = (ha >> 1) + (hx >> 1);
      emin = min(emin, e);
      emax = max(emax, e);
    }
  }
  const bool any = emax >= emin;
  const int W = any ? window_digits<L>(emin, emax) : 1;
  const bool wide = any && (W > WF);
  int64_t* mywin = s_win + lane;  // digit w at mywin[w * 64]
  for (int w = 0; w < WF; ++w) mywin[w * 64] = 0;

  for (int c0 = kb; c0 < ke; c0 += kChunk) {
    const int cn = min(kChunk, ke - c0);
    for (int j = lane; j < cn; j += 64) {
      const int64_t k = c0 + j;
      const int32_t ha = A.a_hdr[k];
      const int32_t col = A.col_idx[k];
      const int32_t hx = x_hdr[col];
      if (hdr_is_zero(ha) || hdr_is_zero(hx)) {
        s_e[j] = INT32_MIN;
      } else {
        uint32_t am[L], xm[L], pr[2 * L];
#pragma unroll
        for (int q = 0; q < L; ++q) am[q] = A.a_limb[(int64_t)q * A.a_ld + k];
#pragma unroll
        for (int q = 0; q < L; ++q) xm[q] = x_limb[(int64_t)q * A.x_ld + col];
        mul_full<L>(am, xm, pr);
#pragma unroll
        for (int q = 0; q < 2 * L; ++q) s_p[q][j] = pr[q];
        s_e[j] = (ha >> 1) + (hx >> 1);
        s_s[j] = (uint32_t)(ha ^ hx) & 1u;
      }
    }
    __syncthreads();
    if (!wide) {
      const int lo = max(rs, c0), hi = min(re, c0 + cn);
      for (int k = lo; k < hi; ++k) {
        const int j = k - c0;
        const int32_t e = s_e[j];
        if (e == INT32_MIN) continue;
        uint32_t pr[2 * L];
#pragma unroll
        for (int q = 0; q < 2 * L; ++q) pr[q] = s_p[q][j];
        window_add<L>(mywin, 64, pr, s_s[j], (uint32_t)(e - emin));
      }
    }
    __syncthreads();
  }
  Num<L> y;
  PairAcc P;
  pair_init(P);
  if (has_row && !wide) {
    if (any) {
      y = window_finalize<L>(mywin, 64, W, (int64_t)emin - 64 * L, st);
    } else {
      set_zero(y, 0);
    }
    store<L>(y, A.y_limb, A.y_hdr, A.y_ld, yo + r0 + lane);
    if (A.npair) pair_fold(A, P, yo + r0 + lane, make_hdr(y.e, y.s));
  }

  // wide rows: the whole block shares one window
  uint64_t pending = __ballot(has_row && wide);
  while (pending) {
    const int owner = __ffsll((unsigned long long)pending) - 1;
    pending &= pending - 1;
    __syncthreads();
    const int o_rs = s_rp[owner], o_re = s_rp[owner + 1];
    const int32_t o_emin = __shfl(emin, owner);
    const int o_W = __shfl(W, owner);
    if (o_W > WB) {
      if (lane == owner) {
        st |= kStWindow;
        set_zero(y, 0);
        store<L>(y, A.y_limb, A.y_hdr, A.y_ld, yo + r0 + lane);
      }
      continue;
    }
    for (int w = lane; w < o_W; w += 64) s_win[w] = 0;
    __syncthreads();
    for (int k = o_rs + lane; k < o_re; k += 64) {
      const int32_t ha = A.a_hdr[k];
      const int32_t col = A.col_idx[k];
      const int32_t hx = x_hdr[col];
      if (hdr_is_zero(ha) || hdr_is_zero(hx)) continue;
      uint32_t am[L], xm[L], pr[2 * L];
#pragma unroll
      for (int q = 0; q < L; ++q) am[q] = A.a_limb[(int64_t)q * A.a_ld + k];
#pragma unroll
      for (int q = 0; q < L; ++q) xm[q] = x_limb[(int64_t)q * A.x_ld + col];
      mul_full<L>(am, xm, pr);
      window_add_atomic<L>(s_win, pr, (uint32_t)(ha ^ hx) & 1u,
                           (uint32_t)((ha >> 1) + (hx >> 1) - o_emin));
    }
    __syncthreads();
    if (lane == owner) {
      y = window_finalize<L>(s_win, 1, o_W, (int64_t)o_emin - 64 * L, st);
      store<L>(y, A.y_limb, A.y_hdr, A.y_ld, yo + r0 + lane);
      if (A.npair) pair_fold(A, P, yo + r0 + lane, make_hdr(y.e, y.s));
    }
  }
  if (A.npair) pair_publish(A, P, B.pair);
  if (st) atomicOr(A.status, st);
}

}  // namespace mp
