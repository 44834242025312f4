// Transposed-product plan (CSR of A^T), A^T x, and the value gradient of a product.
//
// The plan is the explicit transpose in CSR form whose rows (the columns of A) list their
// entries in ascending original-row order, so a SEQ product with A^T accumulates in that order.
// It is built once: a stable radix sort of the entry indices by column (rocPRIM), the per-column
// entry counts (the paper's per-column non-zero numbers of its sparse structure, Sec. 2) and
// their prefix sum, and a gather of the values into structure-of-arrays order.
#include <hip/hip_runtime.h>

#include <algorithm>

#include <cstdio>
#include <cstring>
#include <vector>
#include <rocprim/rocprim.hpp>

#include "../../include/mpspmv.h"
#include "api_internal.hpp"
#include "mp_core.hpp"
#include "plan_internal.hpp"
#include "wide_internal.hpp"

namespace {

__global__ void row_of_kernel(const int32_t* __restrict__ row_ptr, int64_t n_rows,
                              int32_t* __restrict__ row_of) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_rows) return;
  for (int32_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) row_of[k] = (int32_t)i;
}

__global__ void iota_kernel(int32_t* __restrict__ v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) v[i] = (int32_t)i;
}

__global__ void count_kernel(const int32_t* __restrict__ col_idx, int64_t nnz,
                             int32_t* __restrict__ counts) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < nnz) atomicAdd(&counts[col_idx[k]], 1);
}

__global__ void transposed_index_kernel(const int32_t* __restrict__ perm,
                                        const int32_t* __restrict__ row_of, int64_t nnz,
                                        int32_t* __restrict__ t_col) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < nnz) t_col[t] = row_of[perm[t]];
}

template <int L>
__global__ void gather_values_kernel(const int32_t* __restrict__ perm, int64_t nnz,
                                     const uint32_t* __restrict__ src_limb,
                                     const int32_t* __restrict__ src_hdr, int64_t src_ld,
                                     uint32_t* __restrict__ dst_limb, int32_t* __restrict__ dst_hdr) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nnz) return;
  const int64_t k = perm[t];
  dst_hdr[t] = src_hdr[k];
#pragma unroll
  for (int q = 0; q < L; ++q) dst_limb[(int64_t)q * nnz + t] = src_limb[(int64_t)q * src_ld + k];
}

// rec[k] = (limbs of value k, its header), x_rec_words_of(L) words per record
template <int L>
__global__ void __launch_bounds__(256) value_records_kernel(int64_t nnz, const uint32_t* __restrict__ limb,
                                                            const int32_t* __restrict__ hdr, int64_t ld,
                                                            uint32_t* __restrict__ rec) {
  constexpr int S = mp::x_rec_words_of(L);
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nnz; k += (int64_t)gridDim.x * blockDim.x) {
    uint32_t w[L + 4];
#pragma unroll
    for (int q = 0; q < L; ++q) w[q] = limb[(int64_t)q * ld + k];
    w[L] = (uint32_t)hdr[k];
    w[L + 1] = w[L + 2] = w[L + 3] = 0u;
    uint4* out = reinterpret_cast<uint4*>(rec + k * S);
#pragma unroll
    for (int q = 0; q < (L + 4) / 4; ++q) out[q] = make_uint4(w[4 * q], w[4 * q + 1], w[4 * q + 2], w[4 * q + 3]);
  }
}

// dst[t] = record perm[t]
template <int L>
__global__ void __launch_bounds__(256) gather_records_kernel(const int32_t* __restrict__ perm, int64_t nnz,
                                                             const uint32_t* __restrict__ rec,
                                                             uint32_t* __restrict__ dst_limb,
                                                             int32_t* __restrict__ dst_hdr) {
  constexpr int S = mp::x_rec_words_of(L);
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < nnz; t += (int64_t)gridDim.x * blockDim.x) {
    const uint4* r = reinterpret_cast<const uint4*>(rec + (int64_t)perm[t] * S);
    uint32_t w[L + 4];
#pragma unroll
    for (int q = 0; q < (L + 4) / 4; ++q) {
      const uint4 v = r[q];
      w[4 * q] = v.x;
      w[4 * q + 1] = v.y;
      w[4 * q + 2] = v.z;
      w[4 * q + 3] = v.w;
    }
    dst_hdr[t] = (int32_t)w[L];
#pragma unroll
    for (int q = 0; q < L; ++q) dst_limb[(int64_t)q * nnz + t] = w[q];
  }
}

// gvals_k = (-1)^neg * RN(g_i x_j) for entry k = (i, j), in CSR order of A.
template <int L>
__global__ void grad_vals_kernel(int64_t nnz, const int32_t* __restrict__ row_of,
                                 const int32_t* __restrict__ col_idx, const uint32_t* g_limb,
                                 const int32_t* g_hdr, int64_t g_ld, const uint32_t* x_limb,
                                 const int32_t* x_hdr, int64_t x_ld, uint32_t* out_limb,
                                 int32_t* out_hdr, int64_t out_ld, uint32_t neg, uint32_t* status) {
  uint32_t st = 0;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nnz;
       k += (int64_t)gridDim.x * blockDim.x) {
    mp::Num<L> g, x;
    mp::load<L>(g, g_limb, g_hdr, g_ld, row_of[k]);
    mp::load<L>(x, x_limb, x_hdr, x_ld, col_idx[k]);
    mp::Num<L> r = mp::mul_rn<L>(g, x, st);
    r.s ^= neg;
    mp::store<L>(r, out_limb, out_hdr, out_ld, k);
  }
  if (st) atomicOr(status, st);
}

inline unsigned blocks_for(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

namespace mpapi {

int plan_free(mp_plan* P) {
  if (!P) return MPS_OK;
  hipFree(P->t_row_ptr);
  hipFree(P->t_col_idx);
  hipFree(P->perm);
  hipFree(P->row_of);
  hipFree(P->t_limb);
  hipFree(P->t_hdr);
  hipFree(P->x_rec);
  hipFree(P->row_order[0]);
  hipFree(P->row_order[1]);
  delete P;
  return MPS_OK;
}

int plan_row_order(mp_plan* P, int op, const int32_t* a_row_ptr) {
  if (P->row_order[op]) return MPS_OK;
  const int64_t n = op ? P->n_cols : P->n_rows;
  const int32_t* rp = op ? P->t_row_ptr : a_row_ptr;
  std::vector<int32_t> h(n + 1), order(n);
  hipError_t e = hipMemcpy(h.data(), rp, (size_t)(n + 1) * 4, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "row order");
  for (int64_t i = 0; i < n; ++i) order[i] = (int32_t)i;
  std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
    return h[a + 1] - h[a] > h[b + 1] - h[b];
  });
  e = hipMalloc((void**)&P->row_order[op], std::max<size_t>(4, (size_t)n * 4));
  if (e != hipSuccess) {
    P->row_order[op] = nullptr;
    return fail(MPS_ENOMEM, "row order: %s", hipGetErrorString(e));
  }
  e = hipMemcpy(P->row_order[op], order.data(), (size_t)n * 4, hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e, "row order");
  P->order_len[op].resize(n);
  for (int64_t i = 0; i < n; ++i) P->order_len[op][i] = h[order[i] + 1] - h[order[i]];
  return MPS_OK;
}

// Rows at the head of op's row order with at least min_len entries.
static int64_t rows_at_least(const mp_plan* P, int op, int min_len) {
  const std::vector<int32_t>& v = P->order_len[op];
  return std::lower_bound(v.begin(), v.end(), min_len, [](int32_t a, int m) { return a >= m; }) -
         v.begin();
}

SpmvVariant plan_variant(const mp_plan* P, int op, int mode) {
  SpmvVariant v;
  v.rpw = P->rpw[op][mode];
  if (P->stage[op][mode] && P->x_rec) {
    v.x_rec = P->x_rec;
    v.x_len = op ? P->n_rows : P->n_cols;
  }
  if (P->sorted[op][mode]) v.rows = P->row_order[op];
  if (v.rows && mode == MP_SEQ && P->group_min[op] > 0) {
    v.n_long = rows_at_least(P, op, P->group_min[op]);
    v.windows = P->windows[op];
    if (v.windows == 2) v.n_win = rows_at_least(P, op, 8 * P->group_min[op]);
  }
  return v;
}

int plan_x_rec(mp_plan* P) {
  if (P->x_rec) return MPS_OK;
  const int S = mp::x_rec_words_of(P->L);
  const int64_t n = std::max<int64_t>(1, std::max(P->n_rows, P->n_cols));
  hipError_t e = hipMalloc((void**)&P->x_rec, (size_t)n * S * 4);
  if (e != hipSuccess) {
    P->x_rec = nullptr;
    return fail(MPS_ENOMEM, "staged x buffer: %s", hipGetErrorString(e));
  }
  return MPS_OK;
}

template <int L>
void gather_via_records(mp_plan* P, const mp_csr* A, uint32_t* rec, unsigned g, hipStream_t s) {
  hipLaunchKernelGGL(value_records_kernel<L>, dim3(g), dim3(256), 0, s, P->nnz, A->val.limb, A->val.hdr,
                     A->val.ld, rec);
  hipLaunchKernelGGL(gather_records_kernel<L>, dim3(g), dim3(256), 0, s, P->perm, P->nnz, rec, P->t_limb, P->t_hdr);
}

int plan_gather(mp_plan* P, const mp_csr* A, hipStream_t s) {
  if (P->nnz == 0) return MPS_OK;
  if (P->L > 32) return wide_gather(P->L, P->perm, P->nnz, A->val, P->t_limb, P->t_hdr, s);
  const unsigned g = blocks_for(P->nnz, 256);
  // the values as one record per entry first (read and written in order), then the records
  // gathered in the transposed order: one cache line per entry instead of one per limb
  uint32_t* rec = nullptr;
  const size_t rec_bytes = (size_t)P->nnz * mp::x_rec_words_of(P->L) * 4;
  if (hipMallocAsync((void**)&rec, rec_bytes, s) == hipSuccess) {
    switch (P->L) {
      case 4: gather_via_records<4>(P, A, rec, g, s); break;
      case 8: gather_via_records<8>(P, A, rec, g, s); break;
      case 16: gather_via_records<16>(P, A, rec, g, s); break;
      case 32: gather_via_records<32>(P, A, rec, g, s); break;
    }
    hipError_t e = hipGetLastError();
    const hipError_t ef = hipFreeAsync(rec, s);
    if (e == hipSuccess) e = ef;
    return e == hipSuccess ? MPS_OK : hip_fail(e, "gather launch");
  }
  (void)hipGetLastError();  // no room for the records: gather limb by limb
  switch (P->L) {
    case 4: hipLaunchKernelGGL(gather_values_kernel<4>, dim3(g), dim3(256), 0, s, P->perm, P->nnz, A->val.limb, A->val.hdr, A->val.ld, P->t_limb, P->t_hdr); break;
    case 8: hipLaunchKernelGGL(gather_values_kernel<8>, dim3(g), dim3(256), 0, s, P->perm, P->nnz, A->val.limb, A->val.hdr, A->val.ld, P->t_limb, P->t_hdr); break;
    case 16: hipLaunchKernelGGL(gather_values_kernel<16>, dim3(g), dim3(256), 0, s, P->perm, P->nnz, A->val.limb, A->val.hdr, A->val.ld, P->t_limb, P->t_hdr); break;
    case 32: hipLaunchKernelGGL(gather_values_kernel<32>, dim3(g), dim3(256), 0, s, P->perm, P->nnz, A->val.limb, A->val.hdr, A->val.ld, P->t_limb, P->t_hdr); break;
  }
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? MPS_OK : hip_fail(e, "gather launch");
}

int plan_build(const mp_csr* A, hipStream_t s, mp_plan** out) {
  mp_plan* P = new mp_plan();
  P->L = limbs_of(A->prec) ? limbs_of(A->prec) : wide_limbs_of(A->prec);
  P->prec = A->prec;
  P->n_rows = A->row_dim;
  P->n_cols = A->col_dim;
  P->nnz = A->nnz;
  hipGetDevice(&P->device);
  const int64_t nnz = A->nnz;
  hipError_t e;
#define MPS_ALLOC(ptr, bytes)                                          \
  e = hipMalloc((void**)&(ptr), (bytes) > 0 ? (bytes) : 4);            \
  if (e != hipSuccess) {                                               \
    plan_free(P);                                                      \
    return fail(MPS_ENOMEM, "plan allocation: %s", hipGetErrorString(e)); \
  }
  MPS_ALLOC(P->t_row_ptr, (A->col_dim + 1) * 4);
  MPS_ALLOC(P->t_col_idx, nnz * 4);
  MPS_ALLOC(P->perm, nnz * 4);
  MPS_ALLOC(P->row_of, nnz * 4);
  MPS_ALLOC(P->t_limb, nnz * 4 * P->L);
  MPS_ALLOC(P->t_hdr, nnz * 4);
#undef MPS_ALLOC
  e = hipMemsetAsync(P->t_row_ptr, 0, (A->col_dim + 1) * 4, s);
  if (e != hipSuccess) { plan_free(P); return hip_fail(e, "hipMemsetAsync"); }
  if (nnz > 0) {
    uint32_t* keys_out = nullptr;
    int32_t* iota = nullptr;
    void* temp = nullptr;
    size_t temp_bytes = 0;
    e = hipMalloc((void**)&keys_out, nnz * 4);
    if (e == hipSuccess) e = hipMalloc((void**)&iota, nnz * 4);
    if (e != hipSuccess) {
      hipFree(keys_out);
      plan_free(P);
      return fail(MPS_ENOMEM, "plan scratch: %s", hipGetErrorString(e));
    }
    hipLaunchKernelGGL(row_of_kernel, dim3(blocks_for(A->row_dim, 256)), dim3(256), 0, s,
                       A->row_ptr, A->row_dim, P->row_of);
    hipLaunchKernelGGL(iota_kernel, dim3(blocks_for(nnz, 256)), dim3(256), 0, s, iota, nnz);
    hipLaunchKernelGGL(count_kernel, dim3(blocks_for(nnz, 256)), dim3(256), 0, s, A->col_idx,
                       nnz, P->t_row_ptr + 1);
    // stable sort of entry indices by column: ties keep ascending entry (= row) order
    unsigned end_bit = 1;
    while (end_bit < 31 && ((int64_t)1 << end_bit) < A->col_dim) ++end_bit;
    size_t scan_bytes = 0;
    e = rocprim::radix_sort_pairs(nullptr, temp_bytes, (const uint32_t*)A->col_idx, keys_out,
                                  (const int32_t*)iota, P->perm, (size_t)nnz, 0, end_bit, s);
    if (e == hipSuccess)
      e = rocprim::inclusive_scan(nullptr, scan_bytes, P->t_row_ptr + 1, P->t_row_ptr + 1,
                                  (size_t)A->col_dim, rocprim::plus<int32_t>(), s);
    if (scan_bytes > temp_bytes) temp_bytes = scan_bytes;
    if (e == hipSuccess) e = hipMalloc(&temp, temp_bytes > 0 ? temp_bytes : 4);
    if (e == hipSuccess)
      e = rocprim::radix_sort_pairs(temp, temp_bytes, (const uint32_t*)A->col_idx, keys_out,
                                    (const int32_t*)iota, P->perm, (size_t)nnz, 0, end_bit, s);
    // per-column counts -> row pointers of A^T (the sort is done with temp: same stream order)
    if (e == hipSuccess)
      e = rocprim::inclusive_scan(temp, scan_bytes, P->t_row_ptr + 1, P->t_row_ptr + 1,
                                  (size_t)A->col_dim, rocprim::plus<int32_t>(), s);
    if (e == hipSuccess)
      hipLaunchKernelGGL(transposed_index_kernel, dim3(blocks_for(nnz, 256)), dim3(256), 0, s,
                         P->perm, P->row_of, nnz, P->t_col_idx);
    if (e == hipSuccess) e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    else hipStreamSynchronize(s);
    hipFree(temp);
    hipFree(keys_out);
    hipFree(iota);
    if (e != hipSuccess) {
      plan_free(P);
      return hip_fail(e, "plan build");
    }
  }
  int r = plan_gather(P, A, s);
  if (r) {
    plan_free(P);
    return r;
  }
  *out = P;
  return MPS_OK;
}

int check_plan(const mp_plan* P, const mp_csr* A) {
  if (!P) return fail(MPS_EINVAL, "plan is required");
  if (P->n_rows != A->row_dim || P->n_cols != A->col_dim || P->nnz != A->nnz || P->prec != A->prec)
    return fail(MPS_EINVAL, "plan was built for a different matrix");
  return MPS_OK;
}

int grad_vals_launch(const mp_csr* A, const mp_plan* P, const mp_vec* g, const mp_vec* x,
                     mp_vec* out, int negate, uint32_t* status, hipStream_t s) {
  if (A->nnz == 0) return MPS_OK;
  const unsigned grid = (unsigned)std::min<int64_t>(blocks_for(A->nnz, 256), 65536);
  const uint32_t neg = negate ? 1u : 0u;
  switch (P->L) {
    case 4: MPS_LAUNCH_MAIN(true, true, grad_vals_kernel<4>, dim3(grid), dim3(256), 0, s, A->nnz, P->row_of, A->col_idx, g->limb, g->hdr, g->ld, x->limb, x->hdr, x->ld, out->limb, out->hdr, out->ld, neg, status); break;
    case 8: MPS_LAUNCH_MAIN(true, true, grad_vals_kernel<8>, dim3(grid), dim3(256), 0, s, A->nnz, P->row_of, A->col_idx, g->limb, g->hdr, g->ld, x->limb, x->hdr, x->ld, out->limb, out->hdr, out->ld, neg, status); break;
    case 16: MPS_LAUNCH_MAIN(true, true, grad_vals_kernel<16>, dim3(grid), dim3(256), 0, s, A->nnz, P->row_of, A->col_idx, g->limb, g->hdr, g->ld, x->limb, x->hdr, x->ld, out->limb, out->hdr, out->ld, neg, status); break;
    case 32: MPS_LAUNCH_MAIN(true, true, grad_vals_kernel<32>, dim3(grid), dim3(256), 0, s, A->nnz, P->row_of, A->col_idx, g->limb, g->hdr, g->ld, x->limb, x->hdr, x->ld, out->limb, out->hdr, out->ld, neg, status); break;
  }
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? MPS_OK : hip_fail(e, "grad_vals launch");
}

}  // namespace mpapi

using namespace mpapi;

namespace {

// Time every rows-per-block variant of the four products (A and A^T, both modes) on two random
// operands, one with random signs and one with the same magnitudes all positive (SEQ's long-row
// methods fare differently on sums that cancel and sums that only grow), and keep the variant
// with the least total time; every variant computes the same bits, so only speed changes.
template <int L>
__global__ void tune_fill_kernel(uint32_t* limb, int32_t* hdr, int32_t* hdr_pos, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    uint64_t h = 0x9e3779b97f4a7c15ull * (uint64_t)(i + 1);
    for (int k = 0; k < L; ++k) {
      h ^= h >> 29;
      h *= 0xbf58476d1ce4e5b9ull;
      h ^= h >> 32;
      limb[(int64_t)k * n + i] = (uint32_t)h | (k == L - 1 ? 0x80000000u : 0u);
    }
    // exponents as for values uniform on [-1, 1): 0 with probability 1/2, -1 with 1/4, ...
    const int32_t e = -(int32_t)__clz((int)(uint32_t)(h >> 20));
    hdr[i] = (int32_t)(((uint32_t)e << 1) | (uint32_t)((h >> 52) & 1));
    hdr_pos[i] = (int32_t)((uint32_t)e << 1);
  }
}

// xs[op]: the caller's operand for product op (nullptr: the two generated ones)
int tune_impl(mp_plan* P, const mp_csr* A, int reps, uint32_t* status, hipStream_t s,
              const mp_vec* const (&xs)[2] = {nullptr, nullptr}) {
  const int L = P->L;
  const int64_t nmax = std::max<int64_t>(1, std::max(P->n_rows, P->n_cols));
  uint32_t *xl = nullptr, *yl = nullptr;
  int32_t *xh = nullptr, *yh = nullptr, *xh_pos = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  struct Free {
    uint32_t **a, **b;
    int32_t **c, **d, **g;
    hipEvent_t *e, *f;
    ~Free() {
      hipFree(*a); hipFree(*b); hipFree(*c); hipFree(*d); hipFree(*g);
      if (*e) hipEventDestroy(*e);
      if (*f) hipEventDestroy(*f);
    }
  } fr{&xl, &yl, &xh, &yh, &xh_pos, &e0, &e1};
  hipError_t e = hipMalloc((void**)&xl, (size_t)L * nmax * 4);
  if (e == hipSuccess) e = hipMalloc((void**)&yl, (size_t)L * nmax * 4);
  if (e == hipSuccess) e = hipMalloc((void**)&xh, (size_t)nmax * 4);
  if (e == hipSuccess) e = hipMalloc((void**)&yh, (size_t)nmax * 4);
  if (e == hipSuccess) e = hipMalloc((void**)&xh_pos, (size_t)nmax * 4);
  if (e != hipSuccess) return fail(MPS_ENOMEM, "tune workspace: %s", hipGetErrorString(e));
  int r0 = plan_x_rec(P);
  if (!r0) r0 = plan_row_order(P, 0, A->row_ptr);
  if (!r0) r0 = plan_row_order(P, 1, nullptr);
  if (r0) return r0;
  if ((e = hipEventCreate(&e0)) != hipSuccess || (e = hipEventCreate(&e1)) != hipSuccess)
    return hip_fail(e, "tune events");
  const unsigned g = (unsigned)std::min<int64_t>(4096, (nmax + 255) / 256);
  switch (L) {
    case 4: hipLaunchKernelGGL(tune_fill_kernel<4>, dim3(g), dim3(256), 0, s, xl, xh, xh_pos, nmax); break;
    case 8: hipLaunchKernelGGL(tune_fill_kernel<8>, dim3(g), dim3(256), 0, s, xl, xh, xh_pos, nmax); break;
    case 16: hipLaunchKernelGGL(tune_fill_kernel<16>, dim3(g), dim3(256), 0, s, xl, xh, xh_pos, nmax); break;
    default: hipLaunchKernelGGL(tune_fill_kernel<32>, dim3(g), dim3(256), 0, s, xl, xh, xh_pos, nmax); break;
  }
  mp_vec tv{P->t_limb, P->t_hdr, P->nnz, P->nnz};
  for (int op = 0; op < 2; ++op) {
    const int64_t rows = op ? P->n_cols : P->n_rows, cols = op ? P->n_rows : P->n_cols;
    const int32_t* rp = op ? P->t_row_ptr : A->row_ptr;
    const int32_t* ci = op ? P->t_col_idx : A->col_idx;
    const mp_vec& val = op ? tv : A->val;
    mp_vec xv{xl, xh, cols, nmax}, yv{yl, yh, rows, nmax}, xv_pos{xl, xh_pos, cols, nmax};
    for (int mode = 0; mode < 2; ++mode) {
      float best = 0.f;
      int pick = default_rows_per_block(rows, P->nnz), pick_flags = 0, pick_gmin = 0;
      int pick_win = 0;
      // lane groups or windowed chains for the longest rows: SEQ with sorted rows only, when a
      // row is that long
      const int maxlen = P->order_len[op].empty() ? 0 : P->order_len[op][0];
      // (minimum row length, long-row method): none; lane groups from 128 or 512 entries;
      // windowed chains, a row per wavefront, from 256; windowed chains from 32, 64, 128 or
      // 192, four rows per wavefront below eight times that
      static const int kLongMin[8] = {0, 128, 512, 256, 32, 64, 128, 192};
      static const int kLongWin[8] = {0, 0, 0, 1, 2, 2, 2, 2};
      for (int gi = 0; gi < 8; ++gi)
      for (int flags = 0; flags < 4; ++flags) {
        const int gmin = kLongMin[gi];
        const int win = kLongWin[gi];
        if (gmin && (mode != MP_SEQ || !(flags & MP_VARIANT_SORTED_ROWS) || maxlen < gmin || P->L > 16)) continue;
        for (int rpw : {16, 32, 64}) {
          SpmvVariant var;
          var.rpw = rpw;
          if (flags & MP_VARIANT_STAGE_X) {
            var.x_rec = P->x_rec;
            var.x_len = cols;
          }
          if (flags & MP_VARIANT_SORTED_ROWS) var.rows = P->row_order[op];
          if (gmin) var.n_long = rows_at_least(P, op, gmin);
          var.windows = win;
          if (win == 2) var.n_win = rows_at_least(P, op, 8 * gmin);
          int rr = spmv_launch(L, rows, rp, ci, val, xv, yv, mode, status, nullptr, s, nullptr,
                               nullptr, &var);
          if (rr) return rr;
          float ms = 0.f;  // over the operands, the faster of two timed batches of reps launches
          for (int opnd = 0; opnd < (xs[op] ? 1 : 2); ++opnd) {
            const mp_vec& xo = xs[op] ? *xs[op] : (opnd ? xv_pos : xv);
            float mo = 0.f;
            for (int batch = 0; batch < 2; ++batch) {
              if ((e = hipEventRecord(e0, s)) != hipSuccess) return hip_fail(e, "tune");
              for (int k = 0; k < reps; ++k)
                if ((rr = spmv_launch(L, rows, rp, ci, val, xo, yv, mode, status, nullptr, s, nullptr,
                                      nullptr, &var)))
                  return rr;
              if ((e = hipEventRecord(e1, s)) != hipSuccess || (e = hipEventSynchronize(e1)) != hipSuccess)
                return hip_fail(e, "tune");
              float mb = 0.f;
              if ((e = hipEventElapsedTime(&mb, e0, e1)) != hipSuccess) return hip_fail(e, "tune");
              mo = batch == 0 ? mb : std::min(mo, mb);
            }
            ms += mo;
          }
          if (best == 0.f || ms < best) {
            best = ms;
            pick = rpw;
            pick_flags = flags;
            pick_gmin = gmin;
            pick_win = win;
          }
        }
      }
      P->rpw[op][mode] = pick;
      P->stage[op][mode] = (pick_flags & MP_VARIANT_STAGE_X) != 0;
      P->sorted[op][mode] = (pick_flags & MP_VARIANT_SORTED_ROWS) != 0;
      if (mode == MP_SEQ) {
        P->group_min[op] = pick_gmin;
        P->windows[op] = pick_win;
      }
    }
  }
  return MPS_OK;
}

// Tuning cache: one text line per product, "<key> <op> <mode> <rows per block> <flags>", keyed by
// a 64-bit FNV-1a hash of the matrix structure (precision, shape, row pointers, column
// indices), the device (architecture name, compute units) and the library build.
uint64_t fnv1a(uint64_t h, const void* p, size_t n) {
  const unsigned char* c = (const unsigned char*)p;
  for (size_t i = 0; i < n; ++i) {
    h ^= c[i];
    h *= 0x100000001b3ull;
  }
  return h;
}

int tune_key(const mp_plan* P, const mp_csr* A, uint64_t* key) {
  std::vector<int32_t> rp(A->row_dim + 1), ci(A->nnz);
  hipError_t e = hipMemcpy(rp.data(), A->row_ptr, rp.size() * 4, hipMemcpyDeviceToHost);
  if (e == hipSuccess && A->nnz) e = hipMemcpy(ci.data(), A->col_idx, ci.size() * 4, hipMemcpyDeviceToHost);
  hipDeviceProp_t prop;
  if (e == hipSuccess) e = hipGetDeviceProperties(&prop, P->device);
  if (e != hipSuccess) return hip_fail(e, "tuning cache key");
  uint64_t h = 0xcbf29ce484222325ull;
  const int64_t dims[4] = {A->prec, A->row_dim, A->col_dim, A->nnz};
  h = fnv1a(h, dims, sizeof(dims));
  h = fnv1a(h, rp.data(), rp.size() * 4);
  h = fnv1a(h, ci.data(), ci.size() * 4);
  h = fnv1a(h, prop.gcnArchName, strnlen(prop.gcnArchName, sizeof(prop.gcnArchName)));
  h = fnv1a(h, &prop.multiProcessorCount, sizeof(prop.multiProcessorCount));
  static const char build[] = __DATE__ " " __TIME__;
  h = fnv1a(h, build, sizeof(build));
  *key = h;
  return MPS_OK;
}

}  // namespace

extern "C" {

int mp_plan_tune_cached(mp_plan* plan, const mp_csr* A, int reps, const char* cache_path, int* hit,
                        void* stream) {
  clear_error();
  int r = check_csr(A, 0);
  if (r) return r;
  if ((r = check_plan(plan, A))) return r;
  if (!cache_path || !hit) return fail(MPS_EINVAL, "mp_plan_tune_cached: null path or hit flag");
  *hit = 0;
  uint64_t key = 0;
  if ((r = tune_key(plan, A, &key))) return r;
  int rpw[2][2], flags[2][2], seen = 0;
  if (FILE* f = fopen(cache_path, "r")) {
    char line[256];
    while (fgets(line, sizeof(line), f)) {
      unsigned long long k = 0;
      int op, mode, rv, fl;
      if (sscanf(line, "%llx %d %d %d %d", &k, &op, &mode, &rv, &fl) != 5 || k != key) continue;
      if (op < 0 || op > 1 || mode < 0 || mode > 1 || (rv != 0 && !valid_rows_per_block(rv)) ||
          (fl & ~(MP_VARIANT_STAGE_X | MP_VARIANT_SORTED_ROWS | MP_VARIANT_LANE_GROUPS | MP_VARIANT_WINDOWS |
                  MP_VARIANT_SEGMENTS | ~0xff)))
        continue;
      rpw[op][mode] = rv;
      flags[op][mode] = fl;
      seen |= 1 << (2 * op + mode);
    }
    fclose(f);
  }
  if (seen == 15) {
    for (int op = 0; op < 2; ++op)
      for (int mode = 0; mode < 2; ++mode)
        if ((r = mp_plan_set_variant(plan, A, op, mode, rpw[op][mode], flags[op][mode]))) return r;
    *hit = 1;
    return MPS_OK;
  }
  if (reps <= 0) reps = 3;
  DeviceCtx* ctx;
  if ((r = get_ctx(&ctx))) return r;
  if ((r = tune_impl(plan, A, reps, ctx->status, (hipStream_t)stream))) return r;
  FILE* f = fopen(cache_path, "a");
  if (!f) return fail(MPS_EINVAL, "mp_plan_tune_cached: cannot append to %s", cache_path);
  for (int op = 0; op < 2; ++op)
    for (int mode = 0; mode < 2; ++mode) {
      int rv = 0, fl = 0;
      mp_plan_get_variant(plan, op, mode, &rv, &fl);
      fprintf(f, "%016llx %d %d %d %d\n", (unsigned long long)key, op, mode, rv, fl);
    }
  fclose(f);
  return MPS_OK;
}

int mp_plan_create(const mp_csr* A, void* stream, mp_plan** plan) {
  clear_error();
  if (!plan) return fail(MPS_EINVAL, "plan: null output pointer");
  *plan = nullptr;
  int r = check_csr(A, 0, true);
  if (r) return r;
  return plan_build(A, (hipStream_t)stream, plan);
}

int mp_plan_destroy(mp_plan* plan) {
  clear_error();
  if (plan) hipDeviceSynchronize();
  return plan_free(plan);
}

int mp_plan_refresh(mp_plan* plan, const mp_csr* A, void* stream) {
  clear_error();
  int r = check_csr(A, 0, true);
  if (r) return r;
  if ((r = check_plan(plan, A))) return r;
  return plan_gather(plan, A, (hipStream_t)stream);
}

int mpspmv_csr_t(const mp_csr* A, const mp_vec* x, mp_vec* y, int mode, const mp_plan* plan,
                 void* stream) {
  clear_error();
  int r = check_csr(A, 0, true);
  if (r) return r;
  if ((r = check_plan(plan, A))) return r;
  if (mode != MP_SEQ && mode != MP_EXACT) return fail(MPS_EINVAL, "mode must be MP_SEQ or MP_EXACT");
  if ((r = check_vec(x, A->row_dim, "x"))) return r;
  if ((r = check_vec(y, A->col_dim, "y"))) return r;
  const int L = plan->L;
  if (vec_overlap(x, y, L) || vec_overlap(&A->val, y, L)) return fail(MPS_EINVAL, "y overlaps an input");
  DeviceCtx* ctx;
  if ((r = get_ctx(&ctx))) return r;
  mp_vec tv;
  tv.limb = plan->t_limb;
  tv.hdr = plan->t_hdr;
  tv.len = plan->nnz;
  tv.ld = plan->nnz;
  if (L > 32)
    return wide_spmv(L, A->col_dim, plan->t_row_ptr, plan->t_col_idx, tv, *x, *y, mode, ctx->status,
                     (hipStream_t)stream);
  const SpmvVariant var = plan_variant(plan, 1, mode);
  return spmv_launch(L, A->col_dim, plan->t_row_ptr, plan->t_col_idx, tv, *x, *y, mode,
                     ctx->status, nullptr, (hipStream_t)stream, nullptr, nullptr, &var);
}

int mp_plan_set_variant(mp_plan* plan, const mp_csr* A, int op, int mode, int rows_per_block,
                        int flags) {
  clear_error();
  if (!plan) return fail(MPS_EINVAL, "null plan");
  int r = check_csr(A, 0);
  if (r) return r;
  if ((r = check_plan(plan, A))) return r;
  if (op != 0 && op != 1) return fail(MPS_EINVAL, "op must be 0 (A) or 1 (A^T)");
  if (mode != MP_SEQ && mode != MP_EXACT) return fail(MPS_EINVAL, "mode must be MP_SEQ or MP_EXACT");
  if (rows_per_block != 0 && !valid_rows_per_block(rows_per_block))
    return fail(MPS_EINVAL, "rows per block must be 0, 16, 32 or 64");
  if (flags < 0 || (flags & 0xe0)) return fail(MPS_EINVAL, "unknown variant flags");
  if ((flags & MP_VARIANT_WINDOWS) && !(flags & MP_VARIANT_LANE_GROUPS))
    return fail(MPS_EINVAL, "MP_VARIANT_WINDOWS needs MP_VARIANT_LANE_GROUPS and a minimum row length");
  if ((flags & MP_VARIANT_SEGMENTS) && !(flags & MP_VARIANT_WINDOWS))
    return fail(MPS_EINVAL, "MP_VARIANT_SEGMENTS needs MP_VARIANT_WINDOWS");
  const int gmin = (flags & MP_VARIANT_LANE_GROUPS) ? (flags >> 8) : 0;
  if ((flags & MP_VARIANT_LANE_GROUPS) &&
      (mode != MP_SEQ || !(flags & MP_VARIANT_SORTED_ROWS) || gmin < 1))
    return fail(MPS_EINVAL, "lane groups need MP_SEQ, sorted rows and a minimum row length >= 1");
  if (!(flags & MP_VARIANT_LANE_GROUPS) && (flags >> 8))
    return fail(MPS_EINVAL, "a minimum row length without MP_VARIANT_LANE_GROUPS");
  if ((flags & MP_VARIANT_STAGE_X) && (r = plan_x_rec(plan))) return r;
  if ((flags & MP_VARIANT_SORTED_ROWS) && (r = plan_row_order(plan, op, A->row_ptr))) return r;
  plan->rpw[op][mode] = rows_per_block;
  plan->stage[op][mode] = (flags & MP_VARIANT_STAGE_X) != 0;
  plan->sorted[op][mode] = (flags & MP_VARIANT_SORTED_ROWS) != 0;
  if (mode == MP_SEQ) {
    plan->group_min[op] = gmin;
    plan->windows[op] = (gmin > 0 && (flags & MP_VARIANT_WINDOWS)) ? ((flags & MP_VARIANT_SEGMENTS) ? 2 : 1) : 0;
  }
  return MPS_OK;
}

int mp_plan_get_variant(const mp_plan* plan, int op, int mode, int* rows_per_block, int* flags) {
  clear_error();
  if (!plan || !rows_per_block || !flags) return fail(MPS_EINVAL, "null argument");
  if (op != 0 && op != 1) return fail(MPS_EINVAL, "op must be 0 (A) or 1 (A^T)");
  if (mode != MP_SEQ && mode != MP_EXACT) return fail(MPS_EINVAL, "mode must be MP_SEQ or MP_EXACT");
  const int64_t rows = op ? plan->n_cols : plan->n_rows;
  *rows_per_block = plan->rpw[op][mode] ? plan->rpw[op][mode] : default_rows_per_block(rows, plan->nnz);
  const bool srt = plan->sorted[op][mode] && plan->row_order[op];
  const int gmin = (srt && mode == MP_SEQ) ? plan->group_min[op] : 0;
  *flags = ((plan->stage[op][mode] && plan->x_rec) ? MP_VARIANT_STAGE_X : 0) |
           (srt ? MP_VARIANT_SORTED_ROWS : 0) | (gmin ? (MP_VARIANT_LANE_GROUPS | (gmin << 8)) : 0) |
           ((gmin && plan->windows[op]) ? MP_VARIANT_WINDOWS : 0) |
           ((gmin && plan->windows[op] == 2) ? MP_VARIANT_SEGMENTS : 0);
  return MPS_OK;
}

int mp_plan_tune(mp_plan* plan, const mp_csr* A, int reps, void* stream) {
  clear_error();
  int r = check_csr(A, 0);
  if (r) return r;
  if ((r = check_plan(plan, A))) return r;
  if (reps <= 0) reps = 3;
  DeviceCtx* ctx;
  if ((r = get_ctx(&ctx))) return r;
  return tune_impl(plan, A, reps, ctx->status, (hipStream_t)stream);
}

int mp_plan_tune_x(mp_plan* plan, const mp_csr* A, const mp_vec* x, const mp_vec* x_t, int reps, void* stream) {
  clear_error();
  int r = check_csr(A, 0);
  if (r) return r;
  if ((r = check_plan(plan, A))) return r;
  if (x && (r = check_vec(x, A->col_dim, "x"))) return r;
  if (x_t && (r = check_vec(x_t, A->row_dim, "x_t"))) return r;
  if (reps <= 0) reps = 3;
  DeviceCtx* ctx;
  if ((r = get_ctx(&ctx))) return r;
  const mp_vec* const xs[2] = {x, x_t};
  return tune_impl(plan, A, reps, ctx->status, (hipStream_t)stream, xs);
}

int mp_grad_vals(const mp_csr* A, const mp_plan* plan, const mp_vec* g, const mp_vec* x,
                 mp_vec* gvals, int negate, void* stream) {
  clear_error();
  int r = check_csr(A, 0);
  if (r) return r;
  if ((r = check_plan(plan, A))) return r;
  if ((r = check_vec(g, A->row_dim, "g"))) return r;
  if ((r = check_vec(x, A->col_dim, "x"))) return r;
  if ((r = check_vec(gvals, A->nnz, "gvals"))) return r;
  const int L = limbs_of(A->prec);
  if (vec_overlap(g, gvals, L) || vec_overlap(x, gvals, L)) return fail(MPS_EINVAL, "gvals overlaps an input");
  DeviceCtx* ctx;
  if ((r = get_ctx(&ctx))) return r;
  return grad_vals_launch(A, plan, g, x, gvals, negate, ctx->status, (hipStream_t)stream);
}

}  // extern "C"
