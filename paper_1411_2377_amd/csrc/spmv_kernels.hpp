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
#include "mp_group.hpp"
#include "mp_window.hpp"
#include "solver_kernels.hpp"

namespace mp {

constexpr int kRowsPerBlock = 64;
// entries staged per phase-1 chunk (about 8 KB of rounded products in LDS at every precision)
template <int L>
constexpr int chunk_entries() { return 2048 / L; }

// Words per staged x record (x_rec_words_of in mp_core.hpp).
template <int L>
constexpr int x_rec_words() { return x_rec_words_of(L); }

// x_rec[i] = (limbs of x_i, header of x_i)
template <int L>
__global__ void __launch_bounds__(256) x_stage_kernel(const uint32_t* __restrict__ limb,
                                                      const int32_t* __restrict__ hdr, int64_t ld,
                                                      int64_t n, uint32_t* __restrict__ rec) {
  constexpr int S = x_rec_words<L>();
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    uint32_t w[L + 4];
#pragma unroll
    for (int q = 0; q < L; ++q) w[q] = limb[(int64_t)q * ld + i];
    w[L] = (uint32_t)hdr[i];
    w[L + 1] = w[L + 2] = w[L + 3] = 0u;
    uint4* out = reinterpret_cast<uint4*>(rec + i * S);
#pragma unroll
    for (int q = 0; q < (L + 4) / 4; ++q) out[q] = make_uint4(w[4 * q], w[4 * q + 1], w[4 * q + 2], w[4 * q + 3]);
  }
}


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
  // x staged as one record per element (limbs then header, x_rec_words<L>() words apart), or
  // nullptr: x is read in its own layout
  const uint32_t* x_rec;
  // rows in processing order (block b takes rows[b * RPW ...]), or nullptr: 0, 1, 2, ...
  const int32_t* rows;
  int pipe;  // SEQ: the pipelined kernel even when rows == nullptr
  // SEQ with a row order (plain products only): the first n_long rows of that order are summed
  // by lane groups in the first long_blocks blocks; the other blocks take the rows after them
  int64_t n_long;
  int64_t long_blocks;
  // or by windowed chains (window != 0): the first n_win of them one per wavefront in the first
  // win_blocks blocks, the others four per wavefront (16 lanes each)
  int window;
  int64_t n_win;
  int64_t win_blocks;
  // > 0: a dense row-major matrix with that many columns (row i holds entries i * dense_cols ...,
  // entry k sits in column k mod dense_cols); row_ptr and col_idx are then not read
  int32_t dense_cols;
  // several right-hand sides / independent solves (nrhs == 1 and pair_of_tile == nullptr: one)
  int nrhs;                      // block b works on row block b / nrhs for right-hand side b % nrhs
  int64_t x_rstride, y_rstride;  // element offset between right-hand sides in x and y
  const int32_t* pair_of_tile;   // solve of each 512-element tile of y (done flags, scalars)
  const int32_t* done_base;      // &ctl[0].done; solve k's flag at done_base[k * done_stride]
  int64_t done_stride;
  // inner products of y with up to three vectors (kernels instantiated with fused products):
  // (y, part[k]) into slot fd.slot[k]; part[k].hdr == nullptr means y itself
  VecRef part[3];
  DotOut fd;
  DotWork dots;
  Scalars S;
  Ctl* ctl;
  const int32_t* tiles_of_pair;
  const int32_t* first_tile;
  int32_t* ndone;
  // EXACT rows wider than the block's LDS window: kWideSlots windows of kWideDigits digits in
  // global memory, each taken under a lock (nullptr: such rows raise kStWindow)
  int64_t* wide_win;
  int32_t* wide_lock;
};

constexpr int kWideSlots = 16;
constexpr int kWideDigits = 1 << 16;
constexpr int kWideTries = 1 << 22;

// A free global window slot, taken with a compare-and-swap from `start` on (a holder releases
// its slot as soon as its row is rounded, without waiting on anything); -1 after kWideTries
// attempts.
MPD int wide_acquire(int32_t* lock, int start) {
  for (int t = 0; t < kWideTries; ++t) {
    const int s = (start + t) % kWideSlots;
    if (atomicCAS(lock + s, 0, 1) == 0) {
      wait_memory();
      return s;
    }
    if (s == kWideSlots - 1) __builtin_amdgcn_s_sleep(8);
  }
  return -1;
}

MPD void wide_release(int32_t* lock, int s) {
  wait_memory();
  atomicExch(lock + s, 0);
}

// Entry range of a row and column of an entry, from the CSR arrays or the dense shape.
MPD int row_begin(const SpmvArgs& A, int64_t row) {
  return A.dense_cols ? (int)(row * A.dense_cols) : A.row_ptr[row];
}
MPD int row_end(const SpmvArgs& A, int64_t row) {
  return A.dense_cols ? (int)((row + 1) * A.dense_cols) : A.row_ptr[row + 1];
}
MPD int32_t col_of(const SpmvArgs& A, int64_t k) {
  return A.dense_cols ? (int32_t)((uint32_t)k % (uint32_t)A.dense_cols) : A.col_idx[k];
}

// Row block (RPW rows), right-hand side and solve of this block; false if that solve is
// finished.  RPW divides 512, so a block's rows lie in one solve's tile.
struct SpmvBlock {
  int64_t rb;
  int rhs;
  int pair;
};

template <int RPW>
MPD bool spmv_block(const SpmvArgs& A, SpmvBlock& B) {
  B.rhs = (int)(blockIdx.x % (unsigned)A.nrhs);
  B.rb = (int64_t)(blockIdx.x / (unsigned)A.nrhs);
  B.pair = 0;
  if (A.pair_of_tile) {
    B.pair = A.pair_of_tile[(B.rhs * A.y_rstride + B.rb * RPW) / 512];
    if (*(volatile const int32_t*)&A.done_base[B.pair * A.done_stride]) return false;
  } else if (A.done && *(volatile const int32_t*)A.done) {
    return false;
  }
  return true;
}

// The inner products of the rows' results with the requested vectors, one pass each, added to
// their rings; the launch that uses them reads and rounds them (the kernel boundary orders
// every block's additions before it), so no block here waits for its additions or counts.  The
// lane of each row holds its result y; lanes without a row take part with no product.
template <int L, int NT>
MPD void spmv_fused_dots(const SpmvArgs& A, const SpmvBlock& B, bool has_row, int64_t yi,
                         const Num<L>& y, uint32_t st) {
  __shared__ PassLds<L, NT> lds;
  const int32_t hy = has_row ? make_hdr(y.e, y.s) : (int32_t)0x80000000;
  const int64_t slot0 = (int64_t)B.pair * kDotSlots;
  // every partner element is requested before the first pass (one memory latency in all)
  int32_t hw[3];
  uint32_t wm[3][L];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    hw[k] = hy;
#pragma unroll
    for (int q = 0; q < L; ++q) wm[k][q] = y.m[q];
    if (k < A.fd.nd && A.part[k].hdr && has_row) {
      hw[k] = A.part[k].hdr[yi];
#pragma unroll
      for (int q = 0; q < L; ++q) wm[k][q] = A.part[k].limb[(int64_t)q * A.part[k].ld + yi];
    }
  }
#pragma unroll
  for (int k = 0; k < 3; ++k)
    if (k < A.fd.nd) pass_dot<L, NT>(lds, has_row, hy, hw[k], y.m, wm[k], A.dots, slot0 + A.fd.slot[k]);
  if (st) atomicOr(A.status, st);
}

// x_j's header and limbs, from the staged records when there are any
template <int L>
MPD void load_x(const SpmvArgs& A, const uint32_t* x_limb, const int32_t* x_hdr, int32_t col,
                bool want_limbs, int32_t& hx, uint32_t (&xm)[L]) {
  if (A.x_rec) {
    const uint4* r = reinterpret_cast<const uint4*>(A.x_rec + (int64_t)col * x_rec_words<L>());
#pragma unroll
    for (int q = 0; q < L / 4; ++q) {
      const uint4 v = r[q];
      xm[4 * q] = v.x;
      xm[4 * q + 1] = v.y;
      xm[4 * q + 2] = v.z;
      xm[4 * q + 3] = v.w;
    }
    hx = (int32_t)A.x_rec[(int64_t)col * x_rec_words<L>() + L];
  } else {
    hx = x_hdr[col];
#pragma unroll
    for (int q = 0; q < L; ++q) xm[q] = want_limbs ? x_limb[(int64_t)q * A.x_ld + col] : 0u;
  }
}

// Exclusive prefix of each lane's count over the wave, into pre[lane] (pre[64] = total).
MPD void wave_prefix(int v, int32_t* pre) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int u = __shfl_up(v, o);
    if (lane >= o) v += u;
  }
  pre[lane + 1] = v;
  if (lane == 0) pre[0] = 0;
}

// ------------------------------------------------------------------------------------------
// Entry loads: a lane takes K entries of a chunk at once.  The column, header and (for a non-zero
// entry) the limbs of a_k are requested first, then x's header and limbs at that column, so every
// lane has 2K independent loads in flight per round trip instead of one chain per entry.  Stored
// zeros cost only their header and column (their limbs and x's limbs are not read).
// ------------------------------------------------------------------------------------------
template <int L>
constexpr int spmv_kper() { return L >= 16 ? 1 : 2; }

template <int L, int K>
struct EntryLoad {
  int32_t col[K], ha[K], hx[K];
  uint32_t am[K][L], xm[K][L];
};

template <int L, int K>
MPD void load_entries(EntryLoad<L, K>& E, const SpmvArgs& A, const uint32_t* x_limb,
                      const int32_t* x_hdr, const int64_t (&k)[K], const bool (&ok)[K]) {
  const int32_t z = (int32_t)0x80000000;  // +0
#pragma unroll
  for (int i = 0; i < K; ++i) {
    E.col[i] = ok[i] ? col_of(A, k[i]) : 0;
    E.ha[i] = ok[i] ? A.a_hdr[k[i]] : z;
  }
#pragma unroll
  for (int i = 0; i < K; ++i) {
    const bool nz = !hdr_is_zero(E.ha[i]);
#pragma unroll
    for (int q = 0; q < L; ++q) E.am[i][q] = nz ? A.a_limb[(int64_t)q * A.a_ld + k[i]] : 0u;
    if (ok[i]) {
      load_x<L>(A, x_limb, x_hdr, E.col[i], nz, E.hx[i], E.xm[i]);
    } else {
      E.hx[i] = z;
    }
  }
}

// SEQ.  A block takes RPW rows (consecutive, or the plan's rows sorted by length so that a
// block's rows have similar lengths).  Phase 1: all lanes form the rounded products of the rows'
// entries, taken in order (a compact numbering of the rows' entries, the row of each entry
// painted into LDS per chunk), with batched coalesced loads, and stage them in LDS.  Phase 2:
// each lane adds its row's staged products in storage order.
template <int L, int RPW, bool FUSE>
__global__ void __launch_bounds__(64, 4) spmv_seq_kernel(SpmvArgs A) {
  constexpr int K = spmv_kper<L>();
  constexpr int kChunk = 64 * K;
  __shared__ int32_t s_rs[RPW];
  __shared__ int32_t s_cp[65];          // compact entry prefix over the block's rows
  __shared__ uint8_t s_row[kChunk];     // row of each compact entry of the chunk
  __shared__ uint32_t s_m[L][kChunk];
  __shared__ int32_t s_e[kChunk];
  __shared__ uint32_t s_s[kChunk];

  SpmvBlock B;
  if (!spmv_block<RPW>(A, B)) return;
  const int lane = threadIdx.x;
  const int64_t r0 = B.rb * RPW;
  const uint32_t* const x_limb = A.x_limb + B.rhs * A.x_rstride;
  const int32_t* const x_hdr = A.x_hdr + B.rhs * A.x_rstride;
  const int64_t yo = B.rhs * A.y_rstride;  // y (and paired vectors) offset of this right-hand side
  const int nr = (int)min((int64_t)RPW, A.n_rows - r0);
  const bool has_row = lane < nr;
  const int64_t row = has_row ? (A.rows ? (int64_t)A.rows[r0 + lane] : r0 + lane) : 0;
  const int rs = has_row ? row_begin(A, row) : 0;
  const int re = has_row ? row_end(A, row) : 0;
  if (lane < RPW) s_rs[lane] = rs;
  wave_prefix(re - rs, s_cp);
  __syncthreads();
  const int cs = s_cp[lane], ce = s_cp[lane + 1], ntot = s_cp[64];
  uint32_t st = 0;
  Num<L> acc;
  set_zero(acc, 0);

  for (int c0 = 0; c0 < ntot; c0 += kChunk) {
    const int cn = min(kChunk, ntot - c0);
    for (int j = max(cs, c0); j < min(ce, c0 + cn); ++j) s_row[j - c0] = (uint8_t)lane;
    __syncthreads();
    // phase 1: rounded products of the chunk, staged in LDS
    int64_t k[K];
    bool ok[K];
#pragma unroll
    for (int i = 0; i < K; ++i) {
      const int j = lane + 64 * i;
      ok[i] = j < cn;
      const int r = ok[i] ? s_row[j] : 0;
      k[i] = (int64_t)s_rs[r] + (c0 + j - s_cp[r]);
    }
    EntryLoad<L, K> E;
    load_entries<L, K>(E, A, x_limb, x_hdr, k, ok);
#pragma unroll
    for (int i = 0; i < K; ++i) {
      if (!ok[i]) continue;
      const int j = lane + 64 * i;
      const int32_t ha = E.ha[i], hx = E.hx[i];
      Num<L> t;
      if (hdr_is_zero(ha) || hdr_is_zero(hx)) {
        set_zero(t, (uint32_t)(ha ^ hx) & 1u);
      } else {
        uint32_t pr[2 * L];
        mul_full<L>(E.am[i], E.xm[i], pr);
        round_product<L>(pr, (ha >> 1) + (hx >> 1), (uint32_t)(ha ^ hx) & 1u, t, st);
      }
#pragma unroll
      for (int q = 0; q < L; ++q) s_m[q][j] = t.m[q];
      s_e[j] = t.e;
      s_s[j] = t.s;
    }
    __syncthreads();
    // phase 2: each lane adds its row's products in storage order
    for (int j = max(cs, c0); j < min(ce, c0 + cn); ++j) {
      Num<L> t;
#pragma unroll
      for (int q = 0; q < L; ++q) t.m[q] = s_m[q][j - c0];
      t.e = s_e[j - c0];
      t.s = s_s[j - c0];
      // a zero product leaves the sum as it is (the sum is never -0), so it is not added
      if (!is_zero(t)) acc = add_rn<L>(acc, t, st);
    }
    __syncthreads();
  }
  if (has_row) store<L>(acc, A.y_limb, A.y_hdr, A.y_ld, yo + row);
  if constexpr (FUSE) {
    spmv_fused_dots<L, 64>(A, B, has_row, yo + row, acc, st);
  } else if (st) {
    atomicOr(A.status, st);
  }
}

MPD int32_t wave_min32(int32_t v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = min(v, __shfl_xor(v, o));
  return v;
}

MPD int32_t wave_max32(int32_t v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = max(v, __shfl_xor(v, o));
  return v;
}

// SEQ over rows taken by decreasing length (the plan's row order), so that a block's RPW rows
// have similar lengths.  The block is four wavefronts: lane r of the first adds row r's products
// in storage order (the serial RN chain the mode defines), while the other three form the rounded
// products of the next chunk — Q further entries of every row — into the other half of a
// double buffer in LDS.  The chains of the block's rows then advance together, and the products
// are computed off their critical path.
template <int RPW>
constexpr int seq_sorted_q() { return RPW >= 64 ? 4 : 8; }

// SEQ, the long rows at the head of the row order (decreasing length): 64 / L rows per block,
// each summed by a group of L lanes of the first wavefront, one limb per lane
// (group_add_rn: the same RN(y_i + t) as add_rn, with the limb loops spread over the lanes, so
// one step of the serial chain the mode defines costs a few dozen wavefront instructions
// instead of a few hundred).  The other three wavefronts form the rounded products of the next
// chunk, kGroupQ further entries of every row, into the other half of a double buffer in LDS.
constexpr int kGroupQ = 32;

template <int L>
__device__ void spmv_seq_group_rows(const SpmvArgs& A, int64_t blk, uint32_t& st) {
  constexpr int RG = 64 / L;            // rows per block: one per lane group
  constexpr int Q = kGroupQ;
  constexpr int NS = RG * Q;            // product slots per chunk: row r's t-th at r * Q + t
  constexpr int RS = Q * L + L;         // words per row in the limb buffer (padded: banks)
  __shared__ int32_t g_rs[RG], g_len[RG];
  __shared__ int32_t g_maxlen;
  __shared__ uint32_t g_m[2][RG * RS];  // row r, entry t, limb w at r * RS + t * L + w
  __shared__ int32_t g_h[2][RG * (Q + 1)];

  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int64_t r0 = blk * RG;
  const int nr = (int)min((int64_t)RG, A.n_long - r0);
  const uint32_t* const x_limb = A.x_limb;
  const int32_t* const x_hdr = A.x_hdr;
  if (wv == 0) {
    const bool hr = lane < nr;
    const int64_t row = hr ? (int64_t)A.rows[r0 + lane] : 0;
    const int rs = hr ? row_begin(A, row) : 0;
    const int len = hr ? row_end(A, row) - rs : 0;
    if (lane < RG) {
      g_rs[lane] = rs;
      g_len[lane] = len;
    }
    const int mx = wave_max32(len);
    if (lane == 0) g_maxlen = mx;
  }
  __syncthreads();
  const int maxlen = g_maxlen;
  const int nch = (maxlen + Q - 1) / Q;

  auto produce = [&](int c, int b) {
    for (int j = t - 64; j < NS; j += 192) {
      const int r = j / Q, o = j % Q, e = c * Q + o;
      int64_t k[1];
      bool ok[1];
      ok[0] = r < nr && e < g_len[r];
      k[0] = ok[0] ? (int64_t)g_rs[r] + e : 0;
      EntryLoad<L, 1> E;
      load_entries<L, 1>(E, A, x_limb, x_hdr, k, ok);
      const int32_t ha = E.ha[0], hx = E.hx[0];
      Num<L> p;
      if (!ok[0]) {
        set_zero(p, 0u);  // past the row's end: +0, which leaves the sum as it is
      } else if (hdr_is_zero(ha) || hdr_is_zero(hx)) {
        set_zero(p, (uint32_t)(ha ^ hx) & 1u);
      } else {
        uint32_t pr[2 * L];
        mul_full<L>(E.am[0], E.xm[0], pr);
        round_product<L>(pr, (ha >> 1) + (hx >> 1), (uint32_t)(ha ^ hx) & 1u, p, st);
      }
      if (r >= nr) continue;
#pragma unroll
      for (int w = 0; w < L; ++w) g_m[b][r * RS + o * L + w] = p.m[w];
      g_h[b][r * (Q + 1) + o] = make_hdr(p.e, p.s);
    }
  };

  const Group<L> G = group_of_lane<L>();
  const int gi = lane / L;
  const int g = min(gi, max(nr - 1, 0));  // groups without a row repeat the last one's (unstored)
  uint32_t am = 0u, as = 0u;
  int32_t ae = kZeroE;
  if (wv > 0 && nch > 0) produce(0, 0);
  // the chains are the block's critical path: their wavefront issues first
  if (wv == 0) __builtin_amdgcn_s_setprio(3);
  __syncthreads();
  for (int c = 0; c < nch; ++c) {
    const int b = c & 1;
    if (wv > 0) {
      if (c + 1 < nch) produce(c + 1, b ^ 1);
    } else {
      // rows that ended add the +0 products past their end (their sums are kept); the next
      // product is read from LDS while the current one is added
      const int qn = min(Q, maxlen - c * Q);
      uint32_t pm_next = g_m[b][g * RS + G.w];
      int32_t ph_next = g_h[b][g * (Q + 1)];
      for (int o = 0; o < qn; ++o) {
        const uint32_t pm = pm_next;
        const int32_t ph = ph_next;
        const int on = min(o + 1, Q - 1);
        pm_next = g_m[b][g * RS + on * L + G.w];
        ph_next = g_h[b][g * (Q + 1) + on];
        group_add_rn<L>(G, am, ae, as, pm, ph >> 1, (uint32_t)ph & 1u, st);
      }
    }
    __syncthreads();
  }
  if (wv == 0 && gi < nr) {
    const int64_t row = A.rows[r0 + gi];
    A.y_limb[(int64_t)G.w * A.y_ld + row] = am;
    if (G.w == 0) A.y_hdr[row] = make_hdr(ae, as);
  }
}

// SEQ, the long rows at the head of the row order, by windowed chains (mp_window.hpp): four rows
// per block, one per wavefront.  A wavefront forms its row's rounded products 64 at a time (lane
// i: entry i of the chunk; the next chunk's loads are issued before the chain runs) and advances
// the row's chain over them in windows.
template <int L>
__device__ void spmv_seq_window_rows(const SpmvArgs& A, int64_t blk, uint32_t& st) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t ri = blk * 4 + wv;
  if (ri >= A.n_win) return;  // the whole wavefront
  const int64_t row = A.rows ? (int64_t)A.rows[ri] : ri;
  const int rs = row_begin(A, row), len = row_end(A, row) - rs;
  Num<L> y;
  set_zero(y, 0u);
  int64_t k[1];
  bool ok[1];
  ok[0] = lane < len;
  k[0] = ok[0] ? (int64_t)rs + lane : 0;
  EntryLoad<L, 1> E;
  load_entries<L, 1>(E, A, A.x_limb, A.x_hdr, k, ok);
  for (int c0 = 0; c0 < len; c0 += 64) {
    Num<L> t;
    const int32_t ha = E.ha[0], hx = E.hx[0];
    if (!ok[0] || hdr_is_zero(ha) || hdr_is_zero(hx)) {
      set_zero(t, (uint32_t)(ha ^ hx) & 1u);
    } else {
      uint32_t pr[2 * L];
      mul_full<L>(E.am[0], E.xm[0], pr);
      round_product<L>(pr, (ha >> 1) + (hx >> 1), (uint32_t)(ha ^ hx) & 1u, t, st);
    }
    const int c1 = c0 + 64;
    if (c1 < len) {
      ok[0] = c1 + lane < len;
      k[0] = ok[0] ? (int64_t)rs + c1 + lane : 0;
      load_entries<L, 1>(E, A, A.x_limb, A.x_hdr, k, ok);
    }
    win_chain<L>(y, t, 0, min(64, len - c0), st);
  }
  if (lane == 0) store<L>(y, A.y_limb, A.y_hdr, A.y_ld, row);
}

// SEQ, the long rows by segmented windowed chains: sixteen rows per block, four per wavefront
// (one per row of 16 lanes).  Each wavefront forms its rows' rounded products 16 per row at a
// time (lane j of row g: entry j of the chunk of the g-th row; the next chunk's loads are issued
// before the chains run) and advances the four chains together.
template <int L>
__device__ void spmv_seq_seg_rows(const SpmvArgs& A, int64_t blk, uint32_t& st) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, j = lane & 15;
  const int64_t ri = A.n_win + blk * 16 + wv * 4 + (lane >> 4);
  const bool has = ri < A.n_long;
  const int64_t row = has ? (A.rows ? (int64_t)A.rows[ri] : ri) : 0;
  const int rs = has ? row_begin(A, row) : 0;
  const int len = has ? row_end(A, row) - rs : 0;
  const int maxlen = wave_max32(len);
  Num<L> y;
  set_zero(y, 0u);
  int64_t k[1];
  bool ok[1];
  ok[0] = j < len;
  k[0] = ok[0] ? (int64_t)rs + j : 0;
  EntryLoad<L, 1> E;
  load_entries<L, 1>(E, A, A.x_limb, A.x_hdr, k, ok);
  for (int c0 = 0; c0 < maxlen; c0 += 16) {
    Num<L> t;
    const int32_t ha = E.ha[0], hx = E.hx[0];
    if (!ok[0] || hdr_is_zero(ha) || hdr_is_zero(hx)) {
      set_zero(t, (uint32_t)(ha ^ hx) & 1u);
    } else {
      uint32_t pr[2 * L];
      mul_full<L>(E.am[0], E.xm[0], pr);
      round_product<L>(pr, (ha >> 1) + (hx >> 1), (uint32_t)(ha ^ hx) & 1u, t, st);
    }
    const int c1 = c0 + 16;
    if (c1 < maxlen) {
      ok[0] = c1 + j < len;
      k[0] = ok[0] ? (int64_t)rs + c1 + j : 0;
      load_entries<L, 1>(E, A, A.x_limb, A.x_hdr, k, ok);
    }
    win_chain_seg<L>(y, t, max(0, min(16, len - c0)), st);
  }
  if (has && j == 0) store<L>(y, A.y_limb, A.y_hdr, A.y_ld, row);
}

// GROUPS: the long rows are summed by lane groups (whose LDS buffers only this instantiation
// holds), else by windowed chains.
template <int L, int RPW, bool FUSE, bool GROUPS>
__global__ void __launch_bounds__(256) spmv_seq_sorted_kernel(SpmvArgs A) {
  if constexpr (!FUSE && L <= 16) {
    if ((int64_t)blockIdx.x < A.long_blocks) {
      uint32_t st = 0;
      if constexpr (GROUPS)
        spmv_seq_group_rows<L>(A, blockIdx.x, st);
      else if ((int64_t)blockIdx.x < A.win_blocks)
        spmv_seq_window_rows<L>(A, blockIdx.x, st);
      else
        spmv_seq_seg_rows<L>(A, blockIdx.x - A.win_blocks, st);
      if (st) atomicOr(A.status, st);
      return;
    }
  }
  constexpr int Q = seq_sorted_q<RPW>();
  constexpr int NS = RPW * Q;  // product slots per chunk: row r's t-th entry of the chunk at r*Q+t
  __shared__ int32_t s_rs[RPW], s_len[RPW];
  __shared__ int32_t s_maxlen;
  __shared__ uint32_t s_m[2][L][NS];
  __shared__ int32_t s_e[2][NS];
  __shared__ uint32_t s_s[2][NS];

  SpmvBlock B;
  if (!spmv_block<RPW>(A, B)) return;
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int64_t r0 = A.n_long + (B.rb - A.long_blocks) * RPW;
  const uint32_t* const x_limb = A.x_limb + B.rhs * A.x_rstride;
  const int32_t* const x_hdr = A.x_hdr + B.rhs * A.x_rstride;
  const int64_t yo = B.rhs * A.y_rstride;
  const int nr = (int)min((int64_t)RPW, A.n_rows - r0);
  const bool has_row = wv == 0 && lane < nr;
  const int64_t row = has_row ? (A.rows ? (int64_t)A.rows[r0 + lane] : r0 + lane) : 0;
  if (wv == 0) {
    const int rs = has_row ? row_begin(A, row) : 0;
    const int len = has_row ? row_end(A, row) - rs : 0;
    if (lane < RPW) {
      s_rs[lane] = rs;
      s_len[lane] = len;
    }
    const int mx = wave_max32(len);
    if (lane == 0) s_maxlen = mx;
  }
  __syncthreads();
  const int nch = (s_maxlen + Q - 1) / Q;
  uint32_t st = 0;

  // products of chunk c into buffer b by the threads of waves 1..3
  auto produce = [&](int c, int b) {
    for (int j = t - 64; j < NS; j += 192) {
      const int r = j / Q, o = c * Q + j % Q;
      int64_t k[1];
      bool ok[1];
      ok[0] = r < nr && o < s_len[r];
      k[0] = ok[0] ? (int64_t)s_rs[r] + o : 0;
      EntryLoad<L, 1> E;
      load_entries<L, 1>(E, A, x_limb, x_hdr, k, ok);
      if (!ok[0]) continue;
      const int32_t ha = E.ha[0], hx = E.hx[0];
      Num<L> p;
      if (hdr_is_zero(ha) || hdr_is_zero(hx)) {
        set_zero(p, (uint32_t)(ha ^ hx) & 1u);
      } else {
        uint32_t pr[2 * L];
        mul_full<L>(E.am[0], E.xm[0], pr);
        round_product<L>(pr, (ha >> 1) + (hx >> 1), (uint32_t)(ha ^ hx) & 1u, p, st);
      }
#pragma unroll
      for (int q = 0; q < L; ++q) s_m[b][q][j] = p.m[q];
      s_e[b][j] = p.e;
      s_s[b][j] = p.s;
    }
  };

  Num<L> acc;
  set_zero(acc, 0);
  if (wv > 0 && nch > 0) produce(0, 0);
  __syncthreads();
  for (int c = 0; c < nch; ++c) {
    const int b = c & 1;
    if (wv > 0) {
      if (c + 1 < nch) produce(c + 1, b ^ 1);
    } else if (has_row) {
      const int len = s_len[lane];
      for (int q = 0; q < Q && c * Q + q < len; ++q) {
        const int j = lane * Q + q;
        Num<L> p;
#pragma unroll
        for (int w = 0; w < L; ++w) p.m[w] = s_m[b][w][j];
        p.e = s_e[b][j];
        p.s = s_s[b][j];
        if (c == 0 && q == 0) {  // RN(+0 + p): p itself, +0 for a zero p (a uniform branch)
          acc = p;
          acc.s = is_zero(p) ? 0u : p.s;
        } else if (!is_zero(p)) {  // a zero product leaves the sum (never -0) as it is
          acc = add_rn<L>(acc, p, st);
        }
      }
    }
    __syncthreads();
  }
  if (has_row) store<L>(acc, A.y_limb, A.y_hdr, A.y_ld, yo + row);
  if constexpr (FUSE) {
    spmv_fused_dots<L, 256>(A, B, has_row, yo + row, acc, st);
  } else if (st) {
    atomicOr(A.status, st);
  }
}

// ------------------------------------------------------------------------------------------
// EXACT.  Every row's products are added, exactly, into a ring window of R int64 digits in LDS
// (carry-save: plain integer adds, so their order never matters).  Digit d of the exact sum has
// weight 2^(32 d - 2p) and lives in ring slot d mod R; a product with exponent e covers digits
// e >> 5 ... (e >> 5) + 2L.  The ring needs no base chosen in advance: it stays exact as long as
// the row's products span at most R digits (counting two of headroom), which each row checks
// from its exponent range once its products are in.
//
// Rows of at most kShortRow entries: all lanes take the block's short-row entries in order (long
// rows left out; coalesced loads), form the exact products and add them straight into the
// owner row's ring with LDS atomics, keeping the row's exponent range with LDS atomic min/max.
// Nothing is staged and no lane walks a row alone, so the work is spread evenly whatever the row
// lengths.  Each row then rounds its ring once.
//
// Longer rows, one at a time, with the whole wave: lane l takes entries l, l + 64, ... into ring
// column l mod RPW; the columns are summed digit by digit (one digit per lane) and rounded by
// the wave.  A row whose products span more than a ring is redone in a block-shared window at its
// exact exponent anchor (or raises kStWindow when even that is too narrow).
// ------------------------------------------------------------------------------------------
constexpr int kShortRow = 64;

// Ring slot of digit d.
template <int R>
MPD int ring_slot(int32_t d) {
  const int m = d % R;
  return m < 0 ? m + R : m;
}

// A product P * 2^(e - 64L) goes into the ring at digit (e - 1) >> 5 as P * 2^((e - 1) mod 32 + 1)
// in 2L + 1 digits: one funnel shift per digit by 31 - ((e - 1) mod 32), with no separate case
// for a shift of zero (an exponent that is a multiple of 32 anchors the product a digit lower).
MPD int32_t ring_digit(int32_t e) { return (e - 1) >> 5; }

// Ring digits needed by products with exponents in [lo, hi].
template <int L>
MPD int ring_span(int32_t lo, int32_t hi) { return ring_digit(hi) - ring_digit(lo) + 2 * L + 2; }

// Slots of a row's ring: R ring digits, then 2L + 2 overflow slots, so that a product's digits
// land in consecutive slots without wrapping (one base address, immediate offsets).  Overflow
// slot R + u stands for ring digit u; ring_fold adds it back before the row is read.
template <int L, int R>
constexpr int ring_slots() { return R + 2 * L + 2; }

// Add (-1)^s * P * 2^((e - 1) mod 32 + 1) at ring digit ring_digit(e) (slots WS apart) with LDS
// atomics.  A negative product X = sum_j x_j 2^(32 j) (D = 2L + 1 digits) is added as its
// digits' complements plus one, less one a digit above it: -X = sum_j (2^32 - 1 - x_j) 2^(32 j)
// + 1 - 2^(32 D).  Every digit's add is then a 32-bit value with no negation, and every lane issues
// the same adds (no per-digit branch); only negative products add the extra digit.  The row's
// window counts that digit (its headroom digit above the widest product).
template <int L, int R, int WS>
MPD void ring_add(int64_t* win, const uint32_t (&P)[2 * L], uint32_t s, int32_t e) {
  static_assert(2 * L + 2 <= R, "overflow slots fold onto distinct ring digits");
  const uint32_t sh = 31u - ((uint32_t)(e - 1) & 31u);
  uint32_t sp[2 * L + 1];
  sp[0] = fshr(P[0], 0u, sh);
#pragma unroll
  for (int j = 1; j < 2 * L; ++j) sp[j] = fshr(P[j], P[j - 1], sh);
  sp[2 * L] = fshr(0u, P[2 * L - 1], sh);
  const uint32_t mask = s ? ~0u : 0u;
  unsigned long long* const w = reinterpret_cast<unsigned long long*>(win + ring_slot<R>(ring_digit(e)) * WS);
  atomicAdd(&w[0], (unsigned long long)(sp[0] ^ mask) + (unsigned long long)(s & 1u));
#pragma unroll
  for (int j = 1; j <= 2 * L; ++j) atomicAdd(&w[j * WS], (unsigned long long)(sp[j] ^ mask));
  if (s) atomicAdd(&w[(2 * L + 1) * WS], ~0ull);
}

// Fold a row's overflow slots onto its ring digits (after every add has landed).
template <int L, int R, int WS>
MPD void ring_fold(int64_t* win) {
#pragma unroll
  for (int u = 0; u < 2 * L + 2; ++u) win[u * WS] += win[(R + u) * WS];
}

template <int L, int RPW, bool FUSE>
__global__ void __launch_bounds__(64, 4) spmv_exact_kernel(SpmvArgs A) {
  constexpr int R = window_fast_digits<L>();  // ring digits per row
  constexpr int RS = ring_slots<L, R>();        // with the overflow slots
  // digits of the block-shared exact window: the same for every variant, so that every variant
  // accepts the same rows
  constexpr int WB = R * 16;
  static_assert(RPW >= 16, "the shared window lives in the ring area");
  constexpr int K = spmv_kper<L>();
  constexpr int kChunk = 64 * K;
  __shared__ int32_t s_rs[RPW];
  __shared__ int32_t s_cp[65];          // compact (short-row) entry prefix
  __shared__ uint8_t s_row[kChunk];     // row of each compact entry of the chunk
  __shared__ int32_t s_lo[RPW], s_hi[RPW];
  __shared__ int64_t s_win[RS * RPW];   // ring slot d of row r at [d * RPW + r]

  SpmvBlock B;
  if (!spmv_block<RPW>(A, B)) return;
  const int lane = threadIdx.x;
  const int64_t r0 = B.rb * RPW;
  const uint32_t* const x_limb = A.x_limb + B.rhs * A.x_rstride;
  const int32_t* const x_hdr = A.x_hdr + B.rhs * A.x_rstride;
  const int64_t yo = B.rhs * A.y_rstride;  // y (and paired vectors) offset of this right-hand side
  const int nr = (int)min((int64_t)RPW, A.n_rows - r0);
  const bool has_row = lane < nr;
  const int64_t row = has_row ? (A.rows ? (int64_t)A.rows[r0 + lane] : r0 + lane) : 0;
  const int rs = has_row ? row_begin(A, row) : 0;
  const int re = has_row ? row_end(A, row) : 0;
  const bool is_short = has_row && re - rs <= kShortRow;
  for (int i = lane; i < RS * RPW; i += 64) s_win[i] = 0;
  if (lane < RPW) {
    s_rs[lane] = rs;
    s_lo[lane] = INT32_MAX;
    s_hi[lane] = INT32_MIN;
  }
  wave_prefix(is_short ? re - rs : 0, s_cp);  // compact positions of the short rows' entries
  __syncthreads();
  const int cs = s_cp[lane], ce = s_cp[lane + 1], ntot = s_cp[64];
  uint32_t st = 0;

  for (int c0 = 0; c0 < ntot; c0 += kChunk) {
    const int cn = min(kChunk, ntot - c0);
    for (int j = max(cs, c0); j < min(ce, c0 + cn); ++j) s_row[j - c0] = (uint8_t)lane;
    __syncthreads();
    int64_t k[K];
    bool ok[K];
    int rw[K];
#pragma unroll
    for (int i = 0; i < K; ++i) {
      const int j = lane + 64 * i;
      ok[i] = j < cn;
      rw[i] = ok[i] ? s_row[j] : 0;
      k[i] = (int64_t)s_rs[rw[i]] + (c0 + j - s_cp[rw[i]]);
    }
    EntryLoad<L, K> E;
    load_entries<L, K>(E, A, x_limb, x_hdr, k, ok);
#pragma unroll
    for (int i = 0; i < K; ++i) {
      if (!ok[i] || hdr_is_zero(E.ha[i]) || hdr_is_zero(E.hx[i])) continue;
      const int32_t e = (E.ha[i] >> 1) + (E.hx[i] >> 1);
      atomicMin(&s_lo[rw[i]], e);
      atomicMax(&s_hi[rw[i]], e);
      uint32_t pr[2 * L];
      mul_full<L>(E.am[i], E.xm[i], pr);
      ring_add<L, R, RPW>(s_win + rw[i], pr, (uint32_t)(E.ha[i] ^ E.hx[i]) & 1u, e);
    }
    __syncthreads();
  }

  Num<L> y;
  set_zero(y, 0);
  bool wide = false;
  int32_t lo = INT32_MAX, hi = INT32_MIN;
  if (is_short) {
    lo = s_lo[lane];
    hi = s_hi[lane];
    if (lo == INT32_MAX) {
      set_zero(y, 0);
    } else if (ring_span<L>(lo, hi) <= R) {
      ring_fold<L, R, RPW>(s_win + lane);
      y = window_finalize_map<L>(s_win + lane, RingMap<R>{RPW, ring_slot<R>(ring_digit(lo))},
                                 ring_span<L>(lo, hi), 32 * (int64_t)ring_digit(lo) - 64 * L, st);
    } else {
      wide = true;
    }
    if (!wide) store<L>(y, A.y_limb, A.y_hdr, A.y_ld, yo + row);
  }

  uint64_t pending = __ballot(has_row && (!is_short || wide));
  while (pending) {
    const int owner = __ffsll((unsigned long long)pending) - 1;
    pending &= pending - 1;
    const int o_rs = __shfl(rs, owner), o_re = __shfl(re, owner);
    int32_t emin = __shfl(lo, owner), emax = __shfl(hi, owner);  // known for a wide short row
    const bool known = __shfl(wide ? 1 : 0, owner) != 0;
    __syncthreads();
    Num<L> yr;
    set_zero(yr, 0);
    bool ring_ok = false;
    if (!known) {
      // lane rings: lane l adds into column l mod RPW
      for (int i = lane; i < RS * RPW; i += 64) s_win[i] = 0;
      __syncthreads();
      int32_t llo = INT32_MAX, lhi = INT32_MIN;
      for (int k0 = o_rs; k0 < o_re; k0 += kChunk) {
        int64_t k[K];
        bool ok[K];
#pragma unroll
        for (int i = 0; i < K; ++i) {
          k[i] = (int64_t)k0 + lane + 64 * i;
          ok[i] = k[i] < o_re;
        }
        EntryLoad<L, K> E;
        load_entries<L, K>(E, A, x_limb, x_hdr, k, ok);
#pragma unroll
        for (int i = 0; i < K; ++i) {
          if (!ok[i] || hdr_is_zero(E.ha[i]) || hdr_is_zero(E.hx[i])) continue;
          const int32_t e = (E.ha[i] >> 1) + (E.hx[i] >> 1);
          llo = min(llo, e);
          lhi = max(lhi, e);
          uint32_t pr[2 * L];
          mul_full<L>(E.am[i], E.xm[i], pr);
          ring_add<L, R, RPW>(s_win + (lane % RPW), pr, (uint32_t)(E.ha[i] ^ E.hx[i]) & 1u, e);
        }
      }
      emin = wave_min32(llo);
      emax = wave_max32(lhi);
      __syncthreads();
      if (lane < RPW) ring_fold<L, R, RPW>(s_win + lane);
      __syncthreads();
      if (emax >= emin && ring_span<L>(emin, emax) <= min(R, 63)) {  // a digit per lane
        ring_ok = true;
        int64_t dg = 0;
        if (lane < ring_span<L>(emin, emax)) {
          const int64_t* slot = s_win + ring_slot<R>(ring_digit(emin) + lane) * RPW;
#pragma unroll
          for (int c = 0; c < RPW; ++c) dg += slot[c];
        }
        yr = wave_round<L>(dg, 32 * (int64_t)ring_digit(emin) - 64 * L, st);
      }
    }
    if (!ring_ok && emax >= emin) {
      // the row's products span more than a ring: a block-shared window at the exact anchor
      const int W = window_digits<L>(emin, emax);
      if (W <= WB) {
        __syncthreads();
        for (int w = lane; w < W; w += 64) s_win[w] = 0;
        __syncthreads();
        for (int kk = o_rs + lane; kk < o_re; kk += 64) {
          const int32_t ha = A.a_hdr[kk];
          const int32_t col = col_of(A, kk);
          int32_t hx;
          uint32_t am[L], xm[L], pr[2 * L];
          load_x<L>(A, x_limb, x_hdr, col, true, hx, xm);
          if (hdr_is_zero(ha) || hdr_is_zero(hx)) continue;
#pragma unroll
          for (int q = 0; q < L; ++q) am[q] = A.a_limb[(int64_t)q * A.a_ld + kk];
          mul_full<L>(am, xm, pr);
          window_add_atomic<L>(s_win, pr, (uint32_t)(ha ^ hx) & 1u,
                               (uint32_t)((ha >> 1) + (hx >> 1) - emin));
        }
        __syncthreads();
        if (lane == owner) yr = window_finalize<L>(s_win, 1, W, (int64_t)emin - 64 * L, st);
      } else {
        // wider still: a window in global memory, every access device-coherent
        int slot = -1;
        if (A.wide_win && W <= kWideDigits) {
          if (lane == 0) slot = wide_acquire(A.wide_lock, (int)(blockIdx.x % kWideSlots));
          slot = __shfl(slot, 0);
        }
        if (slot < 0) {
          if (lane == owner) st |= kStWindow;
        } else {
          int64_t* const gw = A.wide_win + (int64_t)slot * kWideDigits;
          for (int w = lane; w < W; w += 64) st_dev(gw + w, (int64_t)0);
          wait_memory();
          for (int kk = o_rs + lane; kk < o_re; kk += 64) {
            const int32_t ha = A.a_hdr[kk];
            const int32_t col = col_of(A, kk);
            int32_t hx;
            uint32_t am[L], xm[L], pr[2 * L];
            load_x<L>(A, x_limb, x_hdr, col, true, hx, xm);
            if (hdr_is_zero(ha) || hdr_is_zero(hx)) continue;
#pragma unroll
            for (int q = 0; q < L; ++q) am[q] = A.a_limb[(int64_t)q * A.a_ld + kk];
            mul_full<L>(am, xm, pr);
            window_add_atomic<L>(gw, pr, (uint32_t)(ha ^ hx) & 1u, (uint32_t)((ha >> 1) + (hx >> 1) - emin));
          }
          wait_memory();
          yr = wave_window_round_global<L>(gw, W, (int64_t)emin - 64 * L, st);
          if (lane == 0) wide_release(A.wide_lock, slot);
        }
      }
    }
    if (lane == owner) {
      y = yr;
      store<L>(y, A.y_limb, A.y_hdr, A.y_ld, yo + row);
    }
  }
  if constexpr (FUSE) {
    spmv_fused_dots<L, 64>(A, B, has_row, yo + row, y, st);
  } else if (st) {
    atomicOr(A.status, st);
  }
}

}  // namespace mp
