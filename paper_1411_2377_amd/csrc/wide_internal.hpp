// Wide precisions: p = 2048, 4096 and 8192 bits (64, 128 and 256 limbs), the upper end of the
// paper's precision sweep (Sec. 4.1, Tables 1 and 2).  A number of this width does not fit one
// lane's registers, so every operation here is done by one whole wavefront on numbers held in
// LDS, 64 limbs at a time (limb tiles across the lanes): exact products by column sums, carries
// between lanes by ballots, rounding, long division in radix 2^32, square root bit by bit.  The
// operations and their results are those of the fixed-width path (RN per operation, exact inner
// products and EXACT row sums rounded once, SEQ rows folded in column order); only the data
// movement differs.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/mpspmv.h"

namespace mpapi {

// limbs of a wide precision (2048, 4096, 8192), else 0
int wide_limbs_of(int prec);

// y = A x (SEQ or EXACT) for wide precisions; row_ptr/col_idx/val as the sparse product's.
int wide_spmv(int L, int64_t n_rows, const int32_t* row_ptr, const int32_t* col_idx, const mp_vec& val,
              const mp_vec& x, const mp_vec& y, int mode, uint32_t* status, hipStream_t s);
// out = RN(sum x_i y_i), exact (same workspace rule as mp_dot: calls on one device do not overlap)
int wide_dot(int L, const mp_vec& x, const mp_vec& y, const mp_vec& out, uint32_t* status, hipStream_t s);
// element-wise y_i <- RN(y_i + RN(alpha x_i)) (kind 0), y_i <- RN(x_i + RN(alpha y_i)) (kind 1),
// y_i <- RN(y_i - RN(alpha x_i)) (kind 2); alpha a device scalar
int wide_axpy(int L, int kind, const mp_vec& alpha, const mp_vec& x, const mp_vec& y, int64_t n,
              uint32_t* status, hipStream_t s);
// transposed values: dst[k] = src[perm[k]] (L limbs per element)
int wide_gather(int L, const int32_t* perm, int64_t nnz, const mp_vec& src, uint32_t* dst_limb,
                int32_t* dst_hdr, hipStream_t s);
// BiCG (Fig. 5 left, K = I), GPBiCG (Fig. 5 right), CGS and BiCGSTAB for wide precisions, driven
// from the host (one synchronisation per inner product that decides a branch); each performs the
// operations of its fixed-width counterpart in the same order
struct WideOp {
  int64_t n_out;
  const int32_t* row_ptr;
  const int32_t* col_idx;
  mp_vec val;
};
int wide_bicg(int L, const WideOp& op, const WideOp& opT, const mp_vec* b, mp_vec* x,
              const mp_solve_opts* o, mp_solve_info* info, uint32_t* status, hipStream_t s);
int wide_gpbicg(int L, const WideOp& op, const mp_vec* b, mp_vec* x, const mp_solve_opts* o,
                mp_solve_info* info, uint32_t* status, hipStream_t s);
int wide_cgs(int L, const WideOp& op, const mp_vec* b, mp_vec* x, const mp_solve_opts* o, mp_solve_info* info,
             uint32_t* status, hipStream_t s);
int wide_bicgstab(int L, const WideOp& op, const mp_vec* b, mp_vec* x, const mp_solve_opts* o,
                  mp_solve_info* info, uint32_t* status, hipStream_t s);

}  // namespace mpapi
