// The ILU(0) preconditioner object behind mp_ilu* and its application K^{-1} r.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "../../include/mpspmv.h"

struct mp_ilu {
  int device = 0;
  int L = 0;
  int prec = 0;
  int64_t n = 0, nnz = 0;
  int32_t* row_ptr = nullptr;  // copy of A's pattern: [n + 1], [nnz]
  int32_t* col_idx = nullptr;
  int32_t* diag = nullptr;     // [n] entry index of each diagonal element
  uint32_t* lu_limb = nullptr; // [L][nnz] the factors in A's layout (L below, U on and above)
  int32_t* lu_hdr = nullptr;
  // augmented triangular systems: row i of the lower one holds (column i: +1) and
  // (column n + k: -l_ik) for the stored k < i; of the upper one (column i: +1) and
  // (column n + j: -u_ij) for the stored j > i; each is summed over x = [r; y] by the sparse
  // product, so that the row's sum is r_i - sum l_ik y_k in the product's accumulation mode
  int32_t *rp_lo = nullptr, *ci_lo = nullptr, *rp_up = nullptr, *ci_up = nullptr;
  uint32_t *v_lo_limb = nullptr, *v_up_limb = nullptr;
  int32_t *v_lo_hdr = nullptr, *v_up_hdr = nullptr;
  int64_t nnz_lo = 0, nnz_up = 0;
  // level sets: rows in order of level, and each level's first position (host)
  int32_t *fwd_rows = nullptr, *bwd_rows = nullptr;
  std::vector<int64_t> fwd_ptr, bwd_ptr;
  // the transposed factors' augmented systems, for K^{-T} r = L^{-T} (U^{-T} r): row i of the
  // first holds (column i: +1) and (column n + k: -u_ki) for the k < i whose row stores column
  // i, of the second (column i: +1) and (column n + k: -l_ki) for those k > i, both in
  // ascending k (the transpose's row order); U^T's rows are then divided by u_ii
  int32_t *rp_tu = nullptr, *ci_tu = nullptr, *rp_tl = nullptr, *ci_tl = nullptr;
  uint32_t *v_tu_limb = nullptr, *v_tl_limb = nullptr;
  int32_t *v_tu_hdr = nullptr, *v_tl_hdr = nullptr;
  int64_t nnz_tu = 0, nnz_tl = 0;
  int32_t *tf_rows = nullptr, *tb_rows = nullptr;  // level sets of U^T (forward), L^T (backward)
  std::vector<int64_t> tf_ptr, tb_ptr;
  // work vectors [r; y] and [y; w] (2n elements each; calls must not overlap in time)
  uint32_t *aug_lo_limb = nullptr, *aug_up_limb = nullptr;
  int32_t *aug_lo_hdr = nullptr, *aug_up_hdr = nullptr;
  int32_t* pivot_flag = nullptr;  // set by the factorisation on a zero pivot
};

namespace mpapi {
// w = K^{-1} r = U^{-1} (L^{-1} r) by level-scheduled launches on stream s; ctl (nullable, a
// solve's mp::Ctl): every launch is a no-op once the solve is done.
int ilu_apply(const mp_ilu* K, const mp_vec& r, const mp_vec& w, int mode, uint32_t* status,
              void* ctl, hipStream_t s);
// w = K^{-T} r = L^{-T} (U^{-T} r), the same way over the transposed factors' systems.
int ilu_apply_t(const mp_ilu* K, const mp_vec& r, const mp_vec& w, int mode, uint32_t* status,
                void* ctl, hipStream_t s);
int check_ilu(const mp_ilu* K, const mp_csr* A);
}  // namespace mpapi
