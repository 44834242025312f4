// The opaque plan object behind mp_plan* (transposed structure, permuted values).
#pragma once
#include <stdint.h>

struct mp_plan {
  int device = 0;
  int L = 0;
  int prec = 0;
  int64_t n_rows = 0, n_cols = 0, nnz = 0;
  int32_t* t_row_ptr = nullptr;  // [n_cols + 1]
  int32_t* t_col_idx = nullptr;  // [nnz] original row of each A^T entry, ascending per row of A^T
  int32_t* perm = nullptr;       // [nnz] original entry index of each A^T entry
  int32_t* row_of = nullptr;     // [nnz] row of each entry of A
  uint32_t* t_limb = nullptr;    // [L][nnz] values of A^T
  int32_t* t_hdr = nullptr;      // [nnz]
};

namespace mpapi {
int plan_build(const mp_csr* A, hipStream_t s, mp_plan** out);
int plan_free(mp_plan* P);
int check_plan(const mp_plan* P, const mp_csr* A);
}  // namespace mpapi
