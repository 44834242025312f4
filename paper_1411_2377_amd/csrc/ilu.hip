// ILU(0) preconditioning (Kouya, Sec. 4.2 and Table 3: BiCGSTAB with the incomplete LU
// factorisation without fill-in as its preconditioner K = L U).
//
// Factorisation: row by row in the IKJ form, one RN per operation (a_ik <- a_ik / a_kk, then
// a_ij <- a_ij - a_ik a_kj over the columns j > k that rows i and k both store).  Row i needs the
// final rows k < i it stores, so the rows are grouped in levels (level of i = 1 + the highest
// level among those rows) and each level is one launch, one thread per row.
//
// Application K^{-1} r: the forward solve L y = r level by level, each level one sparse product
// over the augmented lower system (row i: +1 at column i, -l_ik at columns n + k) applied to
// x = [r; y], which the SEQ and EXACT kernels sum exactly as the rows r_i - sum l_ik y_k are
// defined (r_i first, then the terms in ascending column order; or exactly, rounded once); then
// the backward solve the same way on [y; w], each level followed by the division by u_ii.
//
// Transposed application K^{-T} r (BiCG's shadow system, Fig. 5 left): U^T y = r forward, then
// L^T w = y backward, over augmented systems built from the factors' columns (row i of U^T lists
// the u_ki of the rows k < i that store column i, in ascending k), each forward level followed by
// the division by u_ii.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "../../include/mpspmv.h"
#include "api_internal.hpp"
#include "ilu_internal.hpp"
#include "mp_core.hpp"
#include "mp_scalar.hpp"
#include "solver_kernels.hpp"
#include "spmv_internal.hpp"
#include "vec_internal.hpp"

namespace {

using mp::Num;

// One level of the factorisation: each thread takes one row of the level.
template <int L>
__global__ void __launch_bounds__(256) ilu_factor_kernel(const int32_t* __restrict__ rows, int64_t count,
                                                          const int32_t* __restrict__ row_ptr,
                                                          const int32_t* __restrict__ col_idx,
                                                          const int32_t* __restrict__ diag, uint32_t* lu_limb,
                                                          int32_t* lu_hdr, int64_t ld, int32_t* pivot_flag,
                                                          uint32_t* status) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= count) return;
  const int32_t i = rows[g];
  const int32_t rs = row_ptr[i], re = row_ptr[i + 1], di = diag[i];
  uint32_t st = 0;
  for (int32_t t = rs; t < di; ++t) {
    const int32_t k = col_idx[t];
    Num<L> piv, a;
    mp::load<L>(piv, lu_limb, lu_hdr, ld, diag[k]);
    mp::load<L>(a, lu_limb, lu_hdr, ld, t);
    if (mp::is_zero(piv)) {
      atomicOr(pivot_flag, 1);
      break;
    }
    a = mp::div_rn<L>(a, piv, st);
    mp::store<L>(a, lu_limb, lu_hdr, ld, t);
    // the stored columns j > k of row i that row k also stores (both rows ascending)
    int32_t q = diag[k] + 1;
    const int32_t qe = row_ptr[k + 1];
    for (int32_t u = t + 1; u < re; ++u) {
      const int32_t j = col_idx[u];
      while (q < qe && col_idx[q] < j) ++q;
      if (q < qe && col_idx[q] == j) {
        Num<L> aij, akj;
        mp::load<L>(aij, lu_limb, lu_hdr, ld, u);
        mp::load<L>(akj, lu_limb, lu_hdr, ld, q);
        mp::store<L>(mp::sub_rn<L>(aij, mp::mul_rn<L>(a, akj, st), st), lu_limb, lu_hdr, ld, u);
      }
    }
  }
  if (st) atomicOr(status, st);
}

// Values of the augmented triangular systems from the factors: +1, then the negated L (U) part
// of each row.
template <int L>
__global__ void __launch_bounds__(256) ilu_pack_kernel(int64_t n, const int32_t* __restrict__ row_ptr,
                                                        const int32_t* __restrict__ diag,
                                                        const uint32_t* __restrict__ lu_limb,
                                                        const int32_t* __restrict__ lu_hdr, int64_t ld,
                                                        const int32_t* __restrict__ rp_lo,
                                                        const int32_t* __restrict__ rp_up, uint32_t* lo_limb,
                                                        int32_t* lo_hdr, int64_t lo_ld, uint32_t* up_limb,
                                                        int32_t* up_hdr, int64_t up_ld) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  Num<L> one;
#pragma unroll
  for (int k = 0; k < L; ++k) one.m[k] = 0u;
  one.m[L - 1] = 0x80000000u;
  one.e = 1;
  one.s = 0;
  const int32_t rs = row_ptr[i], re = row_ptr[i + 1], di = diag[i];
  int64_t o = rp_lo[i];
  mp::store<L>(one, lo_limb, lo_hdr, lo_ld, o++);
  for (int32_t t = rs; t < di; ++t) {
    Num<L> v;
    mp::load<L>(v, lu_limb, lu_hdr, ld, t);
    mp::store<L>(mp::neg<L>(v), lo_limb, lo_hdr, lo_ld, o++);
  }
  o = rp_up[i];
  mp::store<L>(one, up_limb, up_hdr, up_ld, o++);
  for (int32_t t = di + 1; t < re; ++t) {
    Num<L> v;
    mp::load<L>(v, lu_limb, lu_hdr, ld, t);
    mp::store<L>(mp::neg<L>(v), up_limb, up_hdr, up_ld, o++);
  }
}

// Values of an augmented system from a map of its entries: +1 where src < 0, else the negated
// factor entry src.
template <int L>
__global__ void __launch_bounds__(256) ilu_pack_map_kernel(int64_t m, const int32_t* __restrict__ src,
                                                            const uint32_t* __restrict__ lu_limb,
                                                            const int32_t* __restrict__ lu_hdr, int64_t ld,
                                                            uint32_t* out_limb, int32_t* out_hdr, int64_t out_ld) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m) return;
  const int32_t t = src[e];
  Num<L> v;
  if (t < 0) {
#pragma unroll
    for (int k = 0; k < L; ++k) v.m[k] = 0u;
    v.m[L - 1] = 0x80000000u;
    v.e = 1;
    v.s = 0;
  } else {
    mp::load<L>(v, lu_limb, lu_hdr, ld, t);
    v = mp::neg<L>(v);
  }
  mp::store<L>(v, out_limb, out_hdr, out_ld, e);
}

// w_i <- RN(w_i / u_ii) for the rows of one level (w in place).
template <int L>
__global__ void __launch_bounds__(256) ilu_div_kernel(const int32_t* __restrict__ rows, int64_t count,
                                                       const int32_t* __restrict__ diag,
                                                       const uint32_t* __restrict__ lu_limb,
                                                       const int32_t* __restrict__ lu_hdr, int64_t ld,
                                                       uint32_t* w_limb, int32_t* w_hdr, int64_t w_ld,
                                                       const mp::Ctl* ctl, uint32_t* status) {
  if (mp::solve_done(ctl)) return;
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= count) return;
  const int32_t i = rows[g];
  Num<L> z, d;
  mp::load<L>(z, w_limb, w_hdr, w_ld, i);
  mp::load<L>(d, lu_limb, lu_hdr, ld, diag[i]);
  uint32_t st = 0;
  mp::store<L>(mp::div_rn<L>(z, d, st), w_limb, w_hdr, w_ld, i);
  if (st) atomicOr(status, st);
}

inline unsigned blocks_of(int64_t n) { return (unsigned)std::max<int64_t>(1, (n + 255) / 256); }

// Level sets: rows grouped by level (stable), and the first position of each level.
void levels(int64_t n, const std::vector<int32_t>& rp, const std::vector<int32_t>& ci, bool forward,
            std::vector<int32_t>& rows, std::vector<int64_t>& ptr) {
  std::vector<int32_t> lev(n, 0);
  int32_t top = 0;
  for (int64_t s = 0; s < n; ++s) {
    const int64_t i = forward ? s : n - 1 - s;
    int32_t l = 0;
    for (int32_t t = rp[i]; t < rp[i + 1]; ++t) {
      const int64_t j = ci[t];
      if (forward ? j < i : j > i) l = std::max(l, lev[j] + 1);
    }
    lev[i] = l;
    top = std::max(top, l);
  }
  std::vector<int64_t> cnt(top + 2, 0);
  for (int64_t i = 0; i < n; ++i) cnt[lev[i] + 1]++;
  for (int32_t l = 0; l <= top; ++l) cnt[l + 1] += cnt[l];
  ptr.assign(cnt.begin(), cnt.end());
  rows.assign(n, 0);
  std::vector<int64_t> fill(cnt.begin(), cnt.end() - 1);
  for (int64_t s = 0; s < n; ++s) {
    const int64_t i = forward ? s : n - 1 - s;
    rows[fill[lev[i]]++] = (int32_t)i;
  }
}

template <class T>
void free_dev(T*& p) {
  if (p) (void)hipFree(p);
  p = nullptr;
}

void ilu_free(mp_ilu* K) {
  if (!K) return;
  free_dev(K->row_ptr); free_dev(K->col_idx); free_dev(K->diag);
  free_dev(K->lu_limb); free_dev(K->lu_hdr);
  free_dev(K->rp_lo); free_dev(K->ci_lo); free_dev(K->rp_up); free_dev(K->ci_up);
  free_dev(K->v_lo_limb); free_dev(K->v_lo_hdr); free_dev(K->v_up_limb); free_dev(K->v_up_hdr);
  free_dev(K->fwd_rows); free_dev(K->bwd_rows);
  free_dev(K->rp_tu); free_dev(K->ci_tu); free_dev(K->rp_tl); free_dev(K->ci_tl);
  free_dev(K->v_tu_limb); free_dev(K->v_tu_hdr); free_dev(K->v_tl_limb); free_dev(K->v_tl_hdr);
  free_dev(K->tf_rows); free_dev(K->tb_rows);
  free_dev(K->aug_lo_limb); free_dev(K->aug_lo_hdr); free_dev(K->aug_up_limb); free_dev(K->aug_up_hdr);
  free_dev(K->pivot_flag);
  delete K;
}

}  // namespace

namespace mpapi {

int check_ilu(const mp_ilu* K, const mp_csr* A) {
  if (!K) return fail(MPS_EINVAL, "ILU(0) preconditioner is required");
  if (K->n != A->row_dim || K->nnz != A->nnz || K->prec != A->prec)
    return fail(MPS_EINVAL, "the preconditioner was built for a different matrix");
  return MPS_OK;
}

namespace {

// One triangular solve as level-by-level sparse products over an augmented system: x = [v; y]
// (v copied in first), each level's rows of y from their row sums, divided by u_ii after the
// level when `divide`.
struct TriSys {
  const int32_t* rp;
  const int32_t* ci;
  mp_vec val;
  const int32_t* rows;
  const std::vector<int64_t>* ptr;
  bool divide;
};

int tri_solve(const mp_ilu* K, const TriSys& T, uint32_t* aug_limb, int32_t* aug_hdr, const mp_vec& in,
              int mode, uint32_t* status, mp::Ctl* ctl, hipStream_t s) {
  const int L = K->L;
  const int64_t n = K->n;
  const int32_t* done = ctl ? &ctl->done : nullptr;
  const mp_vec x{aug_limb, aug_hdr, 2 * n, 2 * n};
  const mp_vec xv{aug_limb, aug_hdr, n, 2 * n};
  const mp_vec y{aug_limb + n, aug_hdr + n, n, 2 * n};
  mp::VecArgs a{};
  a.n = n;
  a.ctl = ctl;
  a.status = status;
  a.v[0] = ref(xv);
  a.v[1] = ref(in);
  int rr;
  if ((rr = launch_ew(L, EW_COPY, a, s))) return rr;
  const std::vector<int64_t>& ptr = *T.ptr;
  for (size_t l = 0; l + 1 < ptr.size(); ++l) {
    SpmvVariant var;
    var.rows = T.rows + ptr[l];
    const int64_t cnt = ptr[l + 1] - ptr[l];
    if ((rr = spmv_launch(L, cnt, T.rp, T.ci, T.val, x, y, mode, status, done, s, nullptr, nullptr, &var)))
      return rr;
    if (!T.divide) continue;
    const unsigned g = blocks_of(cnt);
    const int32_t* rows = T.rows + ptr[l];
    switch (L) {
      case 4: hipLaunchKernelGGL(ilu_div_kernel<4>, dim3(g), dim3(256), 0, s, rows, cnt, K->diag, K->lu_limb, K->lu_hdr, K->nnz, y.limb, y.hdr, y.ld, ctl, status); break;
      case 8: hipLaunchKernelGGL(ilu_div_kernel<8>, dim3(g), dim3(256), 0, s, rows, cnt, K->diag, K->lu_limb, K->lu_hdr, K->nnz, y.limb, y.hdr, y.ld, ctl, status); break;
      case 16: hipLaunchKernelGGL(ilu_div_kernel<16>, dim3(g), dim3(256), 0, s, rows, cnt, K->diag, K->lu_limb, K->lu_hdr, K->nnz, y.limb, y.hdr, y.ld, ctl, status); break;
      default: hipLaunchKernelGGL(ilu_div_kernel<32>, dim3(g), dim3(256), 0, s, rows, cnt, K->diag, K->lu_limb, K->lu_hdr, K->nnz, y.limb, y.hdr, y.ld, ctl, status); break;
    }
  }
  return MPS_OK;
}

// The two triangular solves of an application: first into the lower work vector's y, then from
// there into the upper one's, then out to w.
int two_solves(const mp_ilu* K, const TriSys& first, const TriSys& second, const mp_vec& r,
               const mp_vec& w, int mode, uint32_t* status, void* ctl_v, hipStream_t s) {
  const int64_t n = K->n;
  if (n == 0) return MPS_OK;
  mp::Ctl* ctl = static_cast<mp::Ctl*>(ctl_v);
  int rr;
  if ((rr = tri_solve(K, first, K->aug_lo_limb, K->aug_lo_hdr, r, mode, status, ctl, s))) return rr;
  const mp_vec y{K->aug_lo_limb + n, K->aug_lo_hdr + n, n, 2 * n};
  if ((rr = tri_solve(K, second, K->aug_up_limb, K->aug_up_hdr, y, mode, status, ctl, s))) return rr;
  mp::VecArgs a{};
  a.n = n;
  a.ctl = ctl;
  a.status = status;
  a.v[0] = ref(w);
  a.v[1] = ref(mp_vec{K->aug_up_limb + n, K->aug_up_hdr + n, n, 2 * n});
  if ((rr = launch_ew(K->L, EW_COPY, a, s))) return rr;
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? MPS_OK : hip_fail(e, "ILU(0) application");
}

}  // namespace

int ilu_apply(const mp_ilu* K, const mp_vec& r, const mp_vec& w, int mode, uint32_t* status,
              void* ctl, hipStream_t s) {
  const TriSys lo{K->rp_lo, K->ci_lo, mp_vec{K->v_lo_limb, K->v_lo_hdr, K->nnz_lo, K->nnz_lo},
                  K->fwd_rows, &K->fwd_ptr, false};
  const TriSys up{K->rp_up, K->ci_up, mp_vec{K->v_up_limb, K->v_up_hdr, K->nnz_up, K->nnz_up},
                  K->bwd_rows, &K->bwd_ptr, true};
  return two_solves(K, lo, up, r, w, mode, status, ctl, s);
}

int ilu_apply_t(const mp_ilu* K, const mp_vec& r, const mp_vec& w, int mode, uint32_t* status,
                void* ctl, hipStream_t s) {
  const TriSys tu{K->rp_tu, K->ci_tu, mp_vec{K->v_tu_limb, K->v_tu_hdr, K->nnz_tu, K->nnz_tu},
                  K->tf_rows, &K->tf_ptr, true};
  const TriSys tl{K->rp_tl, K->ci_tl, mp_vec{K->v_tl_limb, K->v_tl_hdr, K->nnz_tl, K->nnz_tl},
                  K->tb_rows, &K->tb_ptr, false};
  return two_solves(K, tu, tl, r, w, mode, status, ctl, s);
}

}  // namespace mpapi

using namespace mpapi;

extern "C" {

int mp_ilu0_create(const mp_csr* A, void* stream, mp_ilu** out) {
  clear_error();
  if (!out) return fail(MPS_EINVAL, "ilu: null output pointer");
  *out = nullptr;
  int r = check_csr(A, 0);
  if (r) return r;
  if (A->row_dim != A->col_dim) return fail(MPS_EINVAL, "A must be square");
  if (A->nnz + A->row_dim > INT32_MAX) return fail(MPS_EINVAL, "A too large for 32-bit entry indices");
  DeviceCtx* ctx;
  if ((r = get_ctx(&ctx))) return r;
  hipStream_t s = (hipStream_t)stream;
  const int64_t n = A->row_dim, nnz = A->nnz;
  const int L = limbs_of(A->prec);
  // structure on the host: diagonal positions, levels, augmented systems
  std::vector<int32_t> rp(n + 1), ci(nnz), dg(n);
  hipError_t e = hipMemcpy(rp.data(), A->row_ptr, (n + 1) * 4, hipMemcpyDeviceToHost);
  if (e == hipSuccess && nnz) e = hipMemcpy(ci.data(), A->col_idx, nnz * 4, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "ilu structure");
  std::vector<int32_t> rlo(n + 1, 0), rup(n + 1, 0), clo, cup;
  for (int64_t i = 0; i < n; ++i) {
    dg[i] = -1;
    for (int32_t t = rp[i]; t < rp[i + 1]; ++t)
      if (ci[t] == i) dg[i] = t;
    if (dg[i] < 0) return fail(MPS_EINVAL, "ILU(0): row %lld stores no diagonal entry", (long long)i);
    clo.push_back((int32_t)i);
    for (int32_t t = rp[i]; t < dg[i]; ++t) clo.push_back((int32_t)(n + ci[t]));
    cup.push_back((int32_t)i);
    for (int32_t t = dg[i] + 1; t < rp[i + 1]; ++t) cup.push_back((int32_t)(n + ci[t]));
    rlo[i + 1] = (int32_t)clo.size();
    rup[i + 1] = (int32_t)cup.size();
  }
  // the factors' columns: for column i, the rows k storing it (ascending) and their entries
  std::vector<int32_t> tp(n + 1, 0), tk(nnz), tt(nnz);
  for (int64_t t = 0; t < nnz; ++t) tp[ci[t] + 1]++;
  for (int64_t i = 0; i < n; ++i) tp[i + 1] += tp[i];
  {
    std::vector<int32_t> fill(tp.begin(), tp.end() - 1);
    for (int64_t k = 0; k < n; ++k)
      for (int32_t t = rp[k]; t < rp[k + 1]; ++t) {
        const int32_t f = fill[ci[t]]++;
        tk[f] = (int32_t)k;
        tt[f] = t;
      }
  }
  std::vector<int32_t> rtu(n + 1, 0), rtl(n + 1, 0), ctu, ctl_, stu, stl;
  for (int64_t i = 0; i < n; ++i) {
    ctu.push_back((int32_t)i);
    stu.push_back(-1);
    ctl_.push_back((int32_t)i);
    stl.push_back(-1);
    for (int32_t f = tp[i]; f < tp[i + 1]; ++f) {
      if (tk[f] < i) {
        ctu.push_back((int32_t)(n + tk[f]));
        stu.push_back(tt[f]);
      } else if (tk[f] > i) {
        ctl_.push_back((int32_t)(n + tk[f]));
        stl.push_back(tt[f]);
      }
    }
    rtu[i + 1] = (int32_t)ctu.size();
    rtl[i + 1] = (int32_t)ctl_.size();
  }
  mp_ilu* K = new mp_ilu();
  K->device = 0;
  (void)hipGetDevice(&K->device);
  K->L = L;
  K->prec = A->prec;
  K->n = n;
  K->nnz = nnz;
  K->nnz_lo = (int64_t)clo.size();
  K->nnz_up = (int64_t)cup.size();
  std::vector<int32_t> frows, brows;
  levels(n, rp, ci, true, frows, K->fwd_ptr);
  levels(n, rp, ci, false, brows, K->bwd_ptr);
  std::vector<int32_t> tfrows, tbrows;
  levels(n, tp, tk, true, tfrows, K->tf_ptr);
  levels(n, tp, tk, false, tbrows, K->tb_ptr);
  K->nnz_tu = (int64_t)ctu.size();
  K->nnz_tl = (int64_t)ctl_.size();
  int32_t *src_tu = nullptr, *src_tl = nullptr;
  auto alloc = [&](auto*& p, size_t bytes) {
    return hipMalloc((void**)&p, std::max<size_t>(bytes, 4));
  };
  e = alloc(K->row_ptr, (n + 1) * 4);
  if (e == hipSuccess) e = alloc(K->col_idx, nnz * 4);
  if (e == hipSuccess) e = alloc(K->diag, n * 4);
  if (e == hipSuccess) e = alloc(K->lu_limb, (size_t)L * nnz * 4);
  if (e == hipSuccess) e = alloc(K->lu_hdr, nnz * 4);
  if (e == hipSuccess) e = alloc(K->rp_lo, (n + 1) * 4);
  if (e == hipSuccess) e = alloc(K->ci_lo, K->nnz_lo * 4);
  if (e == hipSuccess) e = alloc(K->rp_up, (n + 1) * 4);
  if (e == hipSuccess) e = alloc(K->ci_up, K->nnz_up * 4);
  if (e == hipSuccess) e = alloc(K->v_lo_limb, (size_t)L * K->nnz_lo * 4);
  if (e == hipSuccess) e = alloc(K->v_lo_hdr, K->nnz_lo * 4);
  if (e == hipSuccess) e = alloc(K->v_up_limb, (size_t)L * K->nnz_up * 4);
  if (e == hipSuccess) e = alloc(K->v_up_hdr, K->nnz_up * 4);
  if (e == hipSuccess) e = alloc(K->fwd_rows, n * 4);
  if (e == hipSuccess) e = alloc(K->bwd_rows, n * 4);
  if (e == hipSuccess) e = alloc(K->aug_lo_limb, (size_t)L * 2 * n * 4);
  if (e == hipSuccess) e = alloc(K->aug_lo_hdr, 2 * n * 4);
  if (e == hipSuccess) e = alloc(K->aug_up_limb, (size_t)L * 2 * n * 4);
  if (e == hipSuccess) e = alloc(K->aug_up_hdr, 2 * n * 4);
  if (e == hipSuccess) e = alloc(K->pivot_flag, 4);
  if (e == hipSuccess) e = alloc(K->rp_tu, (n + 1) * 4);
  if (e == hipSuccess) e = alloc(K->ci_tu, K->nnz_tu * 4);
  if (e == hipSuccess) e = alloc(K->rp_tl, (n + 1) * 4);
  if (e == hipSuccess) e = alloc(K->ci_tl, K->nnz_tl * 4);
  if (e == hipSuccess) e = alloc(K->v_tu_limb, (size_t)L * K->nnz_tu * 4);
  if (e == hipSuccess) e = alloc(K->v_tu_hdr, K->nnz_tu * 4);
  if (e == hipSuccess) e = alloc(K->v_tl_limb, (size_t)L * K->nnz_tl * 4);
  if (e == hipSuccess) e = alloc(K->v_tl_hdr, K->nnz_tl * 4);
  if (e == hipSuccess) e = alloc(K->tf_rows, n * 4);
  if (e == hipSuccess) e = alloc(K->tb_rows, n * 4);
  if (e == hipSuccess) e = alloc(src_tu, K->nnz_tu * 4);
  if (e == hipSuccess) e = alloc(src_tl, K->nnz_tl * 4);
  auto free_src = [&] {
    free_dev(src_tu);
    free_dev(src_tl);
  };
  if (e != hipSuccess) {
    free_src();
    ilu_free(K);
    return fail(MPS_ENOMEM, "ILU(0) allocation: %s", hipGetErrorString(e));
  }
  e = hipMemcpyAsync(K->row_ptr, rp.data(), (n + 1) * 4, hipMemcpyHostToDevice, s);
  if (e == hipSuccess && nnz) e = hipMemcpyAsync(K->col_idx, ci.data(), nnz * 4, hipMemcpyHostToDevice, s);
  if (e == hipSuccess && n) e = hipMemcpyAsync(K->diag, dg.data(), n * 4, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(K->rp_lo, rlo.data(), (n + 1) * 4, hipMemcpyHostToDevice, s);
  if (e == hipSuccess && n) e = hipMemcpyAsync(K->ci_lo, clo.data(), clo.size() * 4, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(K->rp_up, rup.data(), (n + 1) * 4, hipMemcpyHostToDevice, s);
  if (e == hipSuccess && n) e = hipMemcpyAsync(K->ci_up, cup.data(), cup.size() * 4, hipMemcpyHostToDevice, s);
  if (e == hipSuccess && n) e = hipMemcpyAsync(K->fwd_rows, frows.data(), n * 4, hipMemcpyHostToDevice, s);
  if (e == hipSuccess && n) e = hipMemcpyAsync(K->bwd_rows, brows.data(), n * 4, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(K->rp_tu, rtu.data(), (n + 1) * 4, hipMemcpyHostToDevice, s);
  if (e == hipSuccess && n) e = hipMemcpyAsync(K->ci_tu, ctu.data(), ctu.size() * 4, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(K->rp_tl, rtl.data(), (n + 1) * 4, hipMemcpyHostToDevice, s);
  if (e == hipSuccess && n) e = hipMemcpyAsync(K->ci_tl, ctl_.data(), ctl_.size() * 4, hipMemcpyHostToDevice, s);
  if (e == hipSuccess && n) e = hipMemcpyAsync(src_tu, stu.data(), stu.size() * 4, hipMemcpyHostToDevice, s);
  if (e == hipSuccess && n) e = hipMemcpyAsync(src_tl, stl.data(), stl.size() * 4, hipMemcpyHostToDevice, s);
  if (e == hipSuccess && n) e = hipMemcpyAsync(K->tf_rows, tfrows.data(), n * 4, hipMemcpyHostToDevice, s);
  if (e == hipSuccess && n) e = hipMemcpyAsync(K->tb_rows, tbrows.data(), n * 4, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemsetAsync(K->pivot_flag, 0, 4, s);
  if (e != hipSuccess) {
    (void)hipStreamSynchronize(s);
    free_src();
    ilu_free(K);
    return hip_fail(e, "ILU(0) setup");
  }
  // the factors start as A's values
  mp::VecArgs a{};
  a.n = nnz;
  a.v[0] = mp::VecRef{K->lu_limb, K->lu_hdr, nnz};
  a.v[1] = ref(A->val);
  if ((r = launch_ew(L, EW_COPY, a, s))) {
    (void)hipStreamSynchronize(s);
    free_src();
    ilu_free(K);
    return r;
  }
  for (size_t l = 0; l + 1 < K->fwd_ptr.size(); ++l) {
    const int64_t cnt = K->fwd_ptr[l + 1] - K->fwd_ptr[l];
    const int32_t* rows = K->fwd_rows + K->fwd_ptr[l];
    const unsigned g = blocks_of(cnt);
    switch (L) {
      case 4: hipLaunchKernelGGL(ilu_factor_kernel<4>, dim3(g), dim3(256), 0, s, rows, cnt, K->row_ptr, K->col_idx, K->diag, K->lu_limb, K->lu_hdr, nnz, K->pivot_flag, ctx->status); break;
      case 8: hipLaunchKernelGGL(ilu_factor_kernel<8>, dim3(g), dim3(256), 0, s, rows, cnt, K->row_ptr, K->col_idx, K->diag, K->lu_limb, K->lu_hdr, nnz, K->pivot_flag, ctx->status); break;
      case 16: hipLaunchKernelGGL(ilu_factor_kernel<16>, dim3(g), dim3(256), 0, s, rows, cnt, K->row_ptr, K->col_idx, K->diag, K->lu_limb, K->lu_hdr, nnz, K->pivot_flag, ctx->status); break;
      default: hipLaunchKernelGGL(ilu_factor_kernel<32>, dim3(g), dim3(256), 0, s, rows, cnt, K->row_ptr, K->col_idx, K->diag, K->lu_limb, K->lu_hdr, nnz, K->pivot_flag, ctx->status); break;
    }
  }
  if (n) {
    switch (L) {
      case 4: hipLaunchKernelGGL(ilu_pack_kernel<4>, dim3(blocks_of(n)), dim3(256), 0, s, n, K->row_ptr, K->diag, K->lu_limb, K->lu_hdr, nnz, K->rp_lo, K->rp_up, K->v_lo_limb, K->v_lo_hdr, K->nnz_lo, K->v_up_limb, K->v_up_hdr, K->nnz_up); break;
      case 8: hipLaunchKernelGGL(ilu_pack_kernel<8>, dim3(blocks_of(n)), dim3(256), 0, s, n, K->row_ptr, K->diag, K->lu_limb, K->lu_hdr, nnz, K->rp_lo, K->rp_up, K->v_lo_limb, K->v_lo_hdr, K->nnz_lo, K->v_up_limb, K->v_up_hdr, K->nnz_up); break;
      case 16: hipLaunchKernelGGL(ilu_pack_kernel<16>, dim3(blocks_of(n)), dim3(256), 0, s, n, K->row_ptr, K->diag, K->lu_limb, K->lu_hdr, nnz, K->rp_lo, K->rp_up, K->v_lo_limb, K->v_lo_hdr, K->nnz_lo, K->v_up_limb, K->v_up_hdr, K->nnz_up); break;
      default: hipLaunchKernelGGL(ilu_pack_kernel<32>, dim3(blocks_of(n)), dim3(256), 0, s, n, K->row_ptr, K->diag, K->lu_limb, K->lu_hdr, nnz, K->rp_lo, K->rp_up, K->v_lo_limb, K->v_lo_hdr, K->nnz_lo, K->v_up_limb, K->v_up_hdr, K->nnz_up); break;
    }
  }
  if (n) {
    const int64_t mu = K->nnz_tu, ml = K->nnz_tl;
    switch (L) {
      case 4:
        hipLaunchKernelGGL(ilu_pack_map_kernel<4>, dim3(blocks_of(mu)), dim3(256), 0, s, mu, src_tu, K->lu_limb, K->lu_hdr, nnz, K->v_tu_limb, K->v_tu_hdr, mu);
        hipLaunchKernelGGL(ilu_pack_map_kernel<4>, dim3(blocks_of(ml)), dim3(256), 0, s, ml, src_tl, K->lu_limb, K->lu_hdr, nnz, K->v_tl_limb, K->v_tl_hdr, ml);
        break;
      case 8:
        hipLaunchKernelGGL(ilu_pack_map_kernel<8>, dim3(blocks_of(mu)), dim3(256), 0, s, mu, src_tu, K->lu_limb, K->lu_hdr, nnz, K->v_tu_limb, K->v_tu_hdr, mu);
        hipLaunchKernelGGL(ilu_pack_map_kernel<8>, dim3(blocks_of(ml)), dim3(256), 0, s, ml, src_tl, K->lu_limb, K->lu_hdr, nnz, K->v_tl_limb, K->v_tl_hdr, ml);
        break;
      case 16:
        hipLaunchKernelGGL(ilu_pack_map_kernel<16>, dim3(blocks_of(mu)), dim3(256), 0, s, mu, src_tu, K->lu_limb, K->lu_hdr, nnz, K->v_tu_limb, K->v_tu_hdr, mu);
        hipLaunchKernelGGL(ilu_pack_map_kernel<16>, dim3(blocks_of(ml)), dim3(256), 0, s, ml, src_tl, K->lu_limb, K->lu_hdr, nnz, K->v_tl_limb, K->v_tl_hdr, ml);
        break;
      default:
        hipLaunchKernelGGL(ilu_pack_map_kernel<32>, dim3(blocks_of(mu)), dim3(256), 0, s, mu, src_tu, K->lu_limb, K->lu_hdr, nnz, K->v_tu_limb, K->v_tu_hdr, mu);
        hipLaunchKernelGGL(ilu_pack_map_kernel<32>, dim3(blocks_of(ml)), dim3(256), 0, s, ml, src_tl, K->lu_limb, K->lu_hdr, nnz, K->v_tl_limb, K->v_tl_hdr, ml);
        break;
    }
  }
  int32_t piv = 0;
  e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpyAsync(&piv, K->pivot_flag, 4, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  free_src();
  if (e != hipSuccess) {
    ilu_free(K);
    return hip_fail(e, "ILU(0) factorisation");
  }
  if (piv) {
    ilu_free(K);
    return fail(MPS_EINVAL, "ILU(0): zero pivot");
  }
  *out = K;
  return MPS_OK;
}

int mp_ilu0_destroy(mp_ilu* ilu) {
  clear_error();
  if (ilu) (void)hipDeviceSynchronize();
  ilu_free(ilu);
  return MPS_OK;
}

int mp_ilu0_apply(const mp_ilu* ilu, const mp_vec* r, mp_vec* w, int mode, void* stream) {
  clear_error();
  if (!ilu) return fail(MPS_EINVAL, "null preconditioner");
  if (mode != MP_SEQ && mode != MP_EXACT) return fail(MPS_EINVAL, "mode must be MP_SEQ or MP_EXACT");
  int rr;
  if ((rr = check_vec(r, ilu->n, "r"))) return rr;
  if ((rr = check_vec(w, ilu->n, "w"))) return rr;
  if (vec_overlap(r, w, ilu->L)) return fail(MPS_EINVAL, "w overlaps r");
  DeviceCtx* ctx;
  if ((rr = get_ctx(&ctx))) return rr;
  return ilu_apply(ilu, *r, *w, mode, ctx->status, nullptr, (hipStream_t)stream);
}

int mp_ilu0_apply_t(const mp_ilu* ilu, const mp_vec* r, mp_vec* w, int mode, void* stream) {
  clear_error();
  if (!ilu) return fail(MPS_EINVAL, "null preconditioner");
  if (mode != MP_SEQ && mode != MP_EXACT) return fail(MPS_EINVAL, "mode must be MP_SEQ or MP_EXACT");
  int rr;
  if ((rr = check_vec(r, ilu->n, "r"))) return rr;
  if ((rr = check_vec(w, ilu->n, "w"))) return rr;
  if (vec_overlap(r, w, ilu->L)) return fail(MPS_EINVAL, "w overlaps r");
  DeviceCtx* ctx;
  if ((rr = get_ctx(&ctx))) return rr;
  return ilu_apply_t(ilu, *r, *w, mode, ctx->status, nullptr, (hipStream_t)stream);
}

int mp_ilu0_factors(const mp_ilu* ilu, mp_vec* lu, void* stream) {
  clear_error();
  if (!ilu) return fail(MPS_EINVAL, "null preconditioner");
  int rr;
  if ((rr = check_vec(lu, ilu->nnz, "lu"))) return rr;
  mp::VecArgs a{};
  a.n = ilu->nnz;
  a.v[0] = ref(*lu);
  a.v[1] = mp::VecRef{ilu->lu_limb, ilu->lu_hdr, ilu->nnz};
  return launch_ew(ilu->L, EW_COPY, a, (hipStream_t)stream);
}

}  // extern "C"
