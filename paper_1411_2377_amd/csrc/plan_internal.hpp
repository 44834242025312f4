// The opaque plan object behind mp_plan* (transposed structure, permuted values).
#pragma once
#include <stdint.h>

#include <vector>

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
  int rpw[2][2] = {{0, 0}, {0, 0}};  // SpMV rows per block for [A, A^T][mode]; 0: by shape
  bool stage[2][2] = {{false, false}, {false, false}};  // stage x as records for [op][mode]
  bool sorted[2][2] = {{false, false}, {false, false}}; // rows by length for [op][mode]
  uint32_t* x_rec = nullptr;     // [max(n_rows, n_cols)] staged x records (allocated on demand)
  int32_t* row_order[2] = {nullptr, nullptr};  // rows of A / A^T by length, longest first
  std::vector<int32_t> order_len[2];            // their lengths, in that order (host)
  int group_min[2] = {0, 0};  // SEQ with sorted rows: rows of at least this many entries are
                              // summed by lane groups (0: none), for [A, A^T]
  int windows[2] = {0, 0};  // ... by windowed chains instead (1: a row per wavefront, 2: four)
};

namespace mpapi {
struct SpmvVariant;
// allocate the plan's staged-x buffer if it has none
int plan_x_rec(mp_plan* P);
// build the plan's row order for op (0: A, whose row pointers are given; 1: A^T) if it has none
int plan_row_order(mp_plan* P, int op, const int32_t* a_row_ptr);
// the variant the plan holds for product op in mode
SpmvVariant plan_variant(const mp_plan* P, int op, int mode);
}

namespace mpapi {
int plan_build(const mp_csr* A, hipStream_t s, mp_plan** out);
int plan_free(mp_plan* P);
int check_plan(const mp_plan* P, const mp_csr* A);
}  // namespace mpapi
