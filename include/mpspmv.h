/*
 * mpspmv — multiple-precision sparse matrix-vector products and product-type Krylov solvers on
 * one AMD Instinct MI355X (gfx950).  C ABI.
 *
 * What is computed (Kouya, "A Highly Efficient Implementation of Multiple Precision Sparse
 * Matrix-Vector Multiplication and Its Application to Product-type Krylov Subspace Methods"):
 *   - y = A x over compressed sparse row storage with p-bit binary floating-point entries, every
 *     operation rounded to nearest (ties to even) as MPFR defines it (Sec. 2, Sec. 3);
 *   - the transposed product A^T x needed by BiCG (Sec. 4.1, Fig. 5 left);
 *   - the vector operations and inner products of BiCG and GPBiCG (Fig. 5) and the drivers with
 *     the stopping test (*) of Sec. 4.1.
 *
 * NUMBER FORMAT.  p = 32 L bits, L in {4, 8, 16} (p = 128, 256, 512).
 *   value = (-1)^s * M * 2^(e - p),  2^(p-1) <= M < 2^p  (mantissa in [1/2, 1), as MPFR)
 *   exponent range [1 - 2^30, 2^30 - 1] (MPFR's default); no NaN/Inf; signed zeros.
 * An array of N numbers (struct mp_vec) is stored as structure of arrays in device memory:
 *   limb[k * ld + i]  uint32, limb k (k = 0 least significant) of element i, ld >= N;
 *   hdr[i]            int32, (e << 1) | s; a zero has e = -2^30 (hdr = INT32_MIN for +0,
 *                     INT32_MIN + 1 for -0) and its limbs are never read.
 * A CSR matrix (struct mp_csr) mirrors the paper's sparse structure (Sec. 2: precision,
 * dimensions, total non-zero count, per-row entry ranges, column indices, element array):
 *   row_ptr[row_dim + 1] int32 device, row_ptr[0] = 0, non-decreasing, row_ptr[row_dim] = nnz;
 *   col_idx[nnz] int32 device, strictly ascending within each row, in [0, col_dim);
 *   val: mp_vec of length nnz.  Stored zeros are allowed (they take the zero fast path).
 *
 * ACCUMULATION MODES (mode argument):
 *   MP_SEQ   y_i <- +0, then y_i <- RN(y_i + RN(a_ij x_j)) over the row's entries in ascending
 *            column order (a loop of MPFR multiplies and adds);
 *   MP_EXACT y_i = RN(sum_j a_ij x_j), the sum formed exactly and rounded once.
 * Both are deterministic: results are bit-identical from run to run and for every launch shape.
 *
 * OWNERSHIP.  The caller allocates and owns every device array passed in.  The library never
 * frees caller memory.  It owns only what an mp_plan holds and one small per-device context
 * (status word, reduction workspace) created on first use.
 *
 * STREAMS AND ERRORS.  `stream` is a hipStream_t (NULL = the default stream).  Calls enqueue
 * work and return without synchronising unless stated.  Argument errors are detected on the
 * host before anything is enqueued and returned as MPS_EINVAL with a message for
 * mp_last_error().  Conditions found on the device (an exponent leaving the range, an exact
 * accumulation wider than supported) set bits in the per-device status word, read with
 * mp_status().  The library never aborts and never prints.
 */
#ifndef MPSPMV_H
#define MPSPMV_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* return codes */
#define MPS_OK 0
#define MPS_EINVAL (-1)  /* bad argument (checked on the host) */
#define MPS_ENOMEM (-2)  /* device allocation failed */
#define MPS_EHIP (-3)    /* a HIP runtime call failed */
#define MPS_ERANGE (-4)  /* a result exponent left [1 - 2^30, 2^30 - 1] (status word) */
#define MPS_ENOTSUP (-5) /* an exact accumulation needed a wider window than supported */

/* accumulation modes */
#define MP_SEQ 0
#define MP_EXACT 1

/* device status word bits (mp_status) */
#define MP_ST_RANGE 1u
#define MP_ST_WINDOW 2u
#define MP_ST_DIVZERO 4u

typedef struct {
  uint32_t *limb; /* device, [L][ld] limb planes */
  int32_t *hdr;   /* device, [len] headers */
  int64_t len;    /* number of elements */
  int64_t ld;     /* elements between consecutive limb planes, >= len */
} mp_vec;

typedef struct {
  int64_t row_dim, col_dim, nnz;
  int32_t prec;            /* 128, 256 or 512 */
  const int32_t *row_ptr;  /* device [row_dim + 1] */
  const int32_t *col_idx;  /* device [nnz] */
  mp_vec val;              /* [nnz] */
} mp_csr;

/* Message describing the last error returned on the calling thread ("" if none). */
const char *mp_last_error(void);

/* Host-side validation of a matrix descriptor: precision, sizes, pointers.  With
 * check_device_data != 0 it also copies row_ptr and col_idx to the host (synchronising) and
 * checks monotone row pointers and strictly ascending in-range columns.  Needs no GPU when
 * check_device_data == 0.  Returns MPS_OK or MPS_EINVAL. */
int mp_validate_csr(const mp_csr *A, int check_device_data);

/* y = A x (Sec. 2-3 of the paper) in the given mode.  x.len == col_dim, y.len == row_dim, all
 * at A->prec.  y must not overlap x or A.  Asynchronous on `stream`. */
int mpspmv_csr(const mp_csr *A, const mp_vec *x, mp_vec *y, int mode, void *stream);

/* Synchronise `stream`, then read and clear the calling device's status word into *flags
 * (MP_ST_* bits).  Returns MPS_OK, or MPS_ERANGE / MPS_ENOTSUP when such a bit was set. */
int mp_status(void *stream, uint32_t *flags);

#ifdef __cplusplus
}
#endif

#endif /* MPSPMV_H */
