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
 * NUMBER FORMAT.  p = 32 L bits, L in {4, 8, 16, 32} (p = 128, 256, 512, 1024), and the wide
 * precisions L in {64, 128, 256} (p = 2048, 4096, 8192) — the paper runs its solvers at 512 to
 * 8192 bits, Sec. 4.1, Tables 1 and 2.  The wide precisions are served by mpspmv_csr,
 * mpspmv_csr_t (with mp_plan_create / mp_plan_refresh / mp_plan_destroy), mp_dot, mp_axpy,
 * mp_const_decimal, mp_validate_csr, bicg, gpbicg, cgs and bicgstab (host-driven: one
 * synchronisation per inner product whose value decides a branch; opts->chunk and opts->profile
 * are ignored); the other entry points return MPS_EINVAL for them.  Each operation is done by one wavefront on numbers held in
 * LDS; an EXACT row or a block's share of an inner product must span at most
 * 32 (4096 - 2L - 2) bits (about 114,000 to 131,000; wider sets MP_ST_WINDOW and gives +0), and
 * inner products at these precisions on two streams of one device must not overlap.
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
 *
 * EXACT WINDOW LIMITS.  An EXACT row sum is supported when its non-zero products' exponents
 * e_a + e_x span at most 32 * (65536 - 2L - 2) bits (about 2.1 million; L = p/32): rows within
 * 32 * (16 R - 2L - 2) bits, R = 2L + 10 (about 8,900, 12,700, 20,400 and 35,700 bits at p =
 * 128, 256, 512, 1024), are summed in LDS, wider ones in one of 16 global-memory windows of
 * 65536 digits per device (8 MiB, allocated with the device's other state on the first call),
 * which a block takes under a lock and releases when the row is rounded.
 * mpspmv_csr_noalloc keeps the LDS limit.  An exact inner product (mp_dot, the solvers'
 * scalars) is supported when its products' exponents x_e + y_e span at most 32 * (W - 2L - 2)
 * bits, W = min(2048, 257 (2L + 1) / 2) digits for mp_dot and the solvers' vector steps
 * (about 36,700, 65,000, 64,400 and 63,400 bits at p = 128, 256, 512, 1024), W = min(2048,
 * 65 (2L + 1) / 2) digits for the products a solver forms inside its SpMV launches (about 9,000,
 * 17,100, 33,200 and 63,400 bits), and W = 256 digits in gpbicg_batched (about 7,900, 7,600,
 * 7,100 and 6,100 bits).  Wider sums set
 * MP_ST_WINDOW and give +0.
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
  int32_t prec;            /* 128, 256, 512 or 1024 */
  const int32_t *row_ptr;  /* device [row_dim + 1] */
  const int32_t *col_idx;  /* device [nnz] */
  mp_vec val;              /* [nnz] */
} mp_csr;

/* A dense matrix: rows x cols p-bit numbers, row-major (element (i, j) at index i * cols + j of
 * val), zeros stored as elements (the paper's dense format, Sec. 3). */
typedef struct {
  int64_t rows, cols;
  int32_t prec;  /* 128, 256, 512 or 1024 */
  mp_vec val;    /* rows * cols elements */
} mp_dense;

/* Opaque transposed-product plan: the CSR of A^T (rows = columns of A, entries in ascending
 * original-row order, built from the per-column non-zero counts of the paper's sparse
 * structure, Sec. 2) with A's values permuted into it.  Owned by the library. */
typedef struct mp_plan mp_plan;

/* Solver options.  Tolerances are decimal m * 10^e, turned into p-bit constants by exact
 * rounding: the stopping test (*) of Sec. 4.1 is ||r_k||_2 <= c_rel ||r_0||_2 + c_abs with
 * c_rel = RN_p(rtol_m 10^rtol_e10), c_abs = RN_p(atol_m 10^atol_e10) (the paper: 1e-20, 1e-50). */
typedef struct {
  int32_t mode;       /* MP_SEQ or MP_EXACT, for every product with A and A^T */
  int32_t transpose;  /* 0: solve A x = b; 1: solve A^T x = b (needs the plan) */
  int64_t maxit;      /* iteration limit (>= 0); reaching it returns MP_NC */
  int64_t rtol_m, rtol_e10;
  int64_t atol_m, atol_e10;
  int32_t chunk;      /* iterations per host poll of the device done flag, replayed from one
                         captured HIP graph; <= 0 launches every kernel eagerly instead.
                         Results are bit-identical for every value. */
  int32_t use_x0;     /* 0: x0 = +0 and x is output only; 1: x holds x0 on entry */
  mp_vec *res_hist;   /* nullable; element i-1 receives RN(r_i . r_i) after iteration i (up to
                         res_hist->len entries) — the residual history of Fig. 7 squared */
  struct mp_solve_profile *profile;  /* nullable; see below */
} mp_solve_opts;

/* Kernel timing of a solve (measurement only).  With opts->profile set, the iterations run
 * eagerly (as for chunk <= 0; the results do not change) and every iteration kernel is
 * bracketed by HIP events on the solver's stream; the durations, launch counts and algorithmic
 * bytes (the vectors and matrix entries the kernel must read and write once) are added to the
 * struct per kernel class: [0] sparse products that also form the step's inner products of
 * their output, [1] other sparse products, [2] direction steps, [3] update steps (with the
 * inner products they form), [4] the middle element-wise step (GPBiCG's t, s, y; CGS's q, u^, x;
 * BiCGSTAB's s). */
typedef struct mp_solve_profile {
  int64_t launches[5];
  double us[5];
  double bytes[5];
} mp_solve_profile;

/* solver outcome (mp_solve_info.status) */
#define MP_CONVERGED 0
#define MP_NC 1              /* not convergent within maxit (Tables 1-2: "NC") */
#define MP_BREAKDOWN_RHO 2   /* rho = 0: the listings' "exits" */
#define MP_BREAKDOWN_SIGMA 3 /* the denominator of alpha is 0 */
#define MP_BREAKDOWN_ZETA 4  /* GPBiCG: zeta = 0; BiCGSTAB: omega = 0 */
#define MP_BREAKDOWN_TAU 5   /* GPBiCG: tau = 0 (or mu5 = 0 in the first iteration) */

typedef struct {
  int32_t status;        /* MP_CONVERGED ... */
  int64_t iters;         /* completed iterations */
  double final_rel_res;  /* ||r|| / ||r_0|| in double, for display only */
} mp_solve_info;

/* Message describing the last error returned on the calling thread ("" if none). */
const char *mp_last_error(void);

/* Host-side validation of a matrix descriptor: precision, sizes, pointers.  With
 * check_device_data != 0 it also copies row_ptr and col_idx to the host (synchronising) and
 * checks monotone row pointers and strictly ascending in-range columns.  Needs no GPU when
 * check_device_data == 0.  Returns MPS_OK or MPS_EINVAL. */
int mp_validate_csr(const mp_csr *A, int check_device_data);

/* y = A x (Sec. 2-3 of the paper) in the given mode.  x.len == col_dim, y.len == row_dim, all
 * at A->prec.  y must not overlap x or A.  `plan` (nullable; built from A) supplies the kernel
 * variant chosen by mp_plan_tune; without one the variant follows A's shape.  The result bits do
 * not depend on the variant.  Asynchronous on `stream`. */
int mpspmv_csr(const mp_csr *A, const mp_vec *x, mp_vec *y, int mode, const mp_plan *plan,
               void *stream);

/* y = A x for a dense matrix (the dense multiple-precision MV the paper measures its sparse
 * product against, Sec. 3, on the Lotkin matrix with s% zeros), in the given mode: SEQ takes
 * every stored element of a row in ascending column order (y_i <- RN(y_i + RN(a_ij x_j)) from
 * y_i = +0), EXACT rounds the exact row sum once.  A stored zero takes the zero fast path: its
 * limbs and x's are not read, its product is not formed and (SEQ) not added, which gives the
 * same bits as adding it.  The result equals mpspmv_csr on the CSR of A's non-zero elements bit
 * for bit.  x.len == cols, y.len == rows; y must not overlap x or A; rows * cols < 2^31.
 * Asynchronous on `stream`.  Returns MPS_OK or MPS_EINVAL. */
int mp_gemv(const mp_dense *A, const mp_vec *x, mp_vec *y, int mode, void *stream);

/* y = A x as mpspmv_csr (same modes, same result bits), for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  The call allocates nothing, on the device or through any library: x is staged
 * (one record per element, as the MP_VARIANT_STAGE_X variant) into a file-scope device array of
 * 32 MiB + 256 bytes that every GPU the library runs on holds until the process ends, and rows
 * per block follow A's shape.  x.len (= col_dim) may be at most 1,048,576 at p = 128, 524,288 at
 * p = 256, 262,144 at p = 512 and 131,072 at p = 1024; larger x returns MPS_ENOTSUP before
 * anything is enqueued.
 * Device conditions go to a status word inside the same array, which mp_status reads and clears
 * together with the device's other status word.  All calls on one GPU share the array: calls
 * that overlap in time on one GPU (two streams, two threads) race and must be ordered by the
 * caller.  Other arguments, checks and return codes as mpspmv_csr. */
int mpspmv_csr_noalloc(const mp_csr *A, const mp_vec *x, mp_vec *y, int mode, void *stream);

/* Build the transposed-product plan of A (synchronises `stream`; allocates device memory).
 * The plan records A's shape and precision; its values are a copy: after changing A's values
 * in place call mp_plan_refresh.  Returns MPS_OK, MPS_EINVAL or MPS_ENOMEM. */
int mp_plan_create(const mp_csr *A, void *stream, mp_plan **plan);
int mp_plan_destroy(mp_plan *plan);
int mp_plan_refresh(mp_plan *plan, const mp_csr *A, void *stream);

/* y = A^T x, computed as the product with the plan's explicit transpose (SEQ sums over the
 * original rows in ascending order).  x.len == row_dim, y.len == col_dim. */
int mpspmv_csr_t(const mp_csr *A, const mp_vec *x, mp_vec *y, int mode, const mp_plan *plan,
                 void *stream);

/* Kernel variants (implementation tuning, not part of the paper's method).  The SpMV kernels
 * process `rows_per_block` rows (16, 32 or 64) per wavefront-sized block; with
 * MP_VARIANT_STAGE_X they first stage x as one contiguous record per element (one cache line per
 * gathered x_j instead of one per limb, which pays for scattered columns); with
 * MP_VARIANT_SORTED_ROWS the blocks take the rows in order of decreasing length (the plan holds
 * the order), so that a block's rows have similar lengths; MP_VARIANT_LANE_GROUPS (below) adds
 * lane groups for the longest rows of a SEQ product.  op 0 is the product with A, op 1
 * with A^T.  mp_plan_tune times every variant of the four products (both ops, both modes;
 * `reps` launches each, 0: 3) on a generated operand, synchronously on `stream`, and stores the
 * fastest in the plan; the plan then selects it for mpspmv_csr, mpspmv_csr_t and the solvers
 * given the plan.  Results are bit-identical for every variant.  mp_plan_set_variant forces a
 * variant (rows 0: by shape; A is the plan's matrix, read to order its rows);
 * mp_plan_get_variant reports the one in effect.  A plan whose variants stage x holds one
 * staging buffer: calls using it must not overlap in time (one stream at a time).  All return
 * MPS_OK or MPS_EINVAL (also MPS_ENOMEM, MPS_EHIP). */
#define MP_VARIANT_STAGE_X 1
#define MP_VARIANT_SORTED_ROWS 2
/* SEQ products with MP_VARIANT_SORTED_ROWS: the rows with at least n stored entries (flags
 * MP_VARIANT_LANE_GROUPS | MP_VARIANT_GROUP_MIN(n), 1 <= n < 2^23) are each summed by a group of
 * L lanes holding one limb each, so that the serial rounding chain of a long row advances many
 * times faster; the other rows as before.  Same result bits. */
#define MP_VARIANT_LANE_GROUPS 4
#define MP_VARIANT_GROUP_MIN(n) ((n) << 8)
/* With MP_VARIANT_LANE_GROUPS: those rows are summed instead by windowed chains, one wavefront
 * per row: up to 64 consecutive steps of the chain are taken at once as an integer prefix sum
 * of the products rounded onto the running sum's unit in the last place, exact while the sum
 * stays in its binade; a step that leaves it (or rounds half-way) is taken alone.  Same result
 * bits. */
#define MP_VARIANT_WINDOWS 8
/* With MP_VARIANT_WINDOWS: the rows of at least n but fewer than 8n entries four per wavefront,
 * one per row of 16 lanes (windows of up to 16 steps); the rows of 8n or more entries one per
 * wavefront as before.  Same result bits. */
#define MP_VARIANT_SEGMENTS 16
int mp_plan_tune(mp_plan *plan, const mp_csr *A, int reps, void *stream);
/* mp_plan_tune timing the products on the caller's operands: x (n_cols elements, device) for
 * y = A x and x_t (n_rows) for A^T x_t; a null pointer takes the generated operands for that
 * product.  The long-row methods of SEQ are data-dependent (the windowed chains take a step
 * alone where the running sum leaves its binade, which sums that cancel do often and sums of
 * one sign rarely), so the operand the products will see picks best.  x and x_t are only read.
 * Returns as mp_plan_tune, plus MPS_EINVAL for a bad operand. */
int mp_plan_tune_x(mp_plan *plan, const mp_csr *A, const mp_vec *x, const mp_vec *x_t, int reps,
                   void *stream);
int mp_plan_set_variant(mp_plan *plan, const mp_csr *A, int op, int mode, int rows_per_block,
                        int flags);
/* mp_plan_tune with a persistent cache: the text file `cache_path` maps a key (a hash of A's
 * precision, shape, row pointers and column indices, of the device's architecture and compute
 * unit count, and of the library build) to the variants of the four products.  On a hit
 * (*hit = 1) the cached variants are set and nothing is launched; otherwise the variants are
 * tuned as by mp_plan_tune and appended to the file (created if missing).  Synchronous (copies
 * A's structure to the host to form the key).  Returns as mp_plan_tune, plus MPS_EINVAL when
 * the file cannot be written. */
int mp_plan_tune_cached(mp_plan *plan, const mp_csr *A, int reps, const char *cache_path, int *hit,
                        void *stream);
int mp_plan_get_variant(const mp_plan *plan, int op, int mode, int *rows_per_block, int *flags);

/* gvals_k = RN(g_i x_j) for each stored entry k = (i, j) in A's CSR order (negated when
 * negate != 0): the gradient of <g, A x> with respect to the stored values.  Needs the plan
 * (for the row of each entry).  g.len == row_dim, x.len == col_dim, gvals.len == nnz. */
int mp_grad_vals(const mp_csr *A, const mp_plan *plan, const mp_vec *g, const mp_vec *x,
                 mp_vec *gvals, int negate, void *stream);

/* y_i <- RN(y_i + RN(alpha x_i)); alpha is a one-element device vector (the x + alpha p lines
 * of Fig. 5).  x.len == y.len. */
int mp_axpy(const mp_vec *alpha, const mp_vec *x, mp_vec *y, int prec, void *stream);

/* out[0] = RN(sum_i x_i y_i), the sum formed exactly (the inner products of Fig. 5).  Uses a
 * per-device workspace: calls on different streams of one device must not overlap. */
int mp_dot(const mp_vec *x, const mp_vec *y, mp_vec *out, int prec, void *stream);

/* out[0] = RN_p(m * 10^e10), |e10| <= 2000 (exact rounding of a decimal constant). */
int mp_const_decimal(int64_t m, int64_t e10, int prec, mp_vec *out, void *stream);

/* BiCG (Fig. 5 left, K = I) for A x = b (or A^T x = b).  The plan is used for the products
 * with A^T; pass NULL to have one built and freed inside the call.  Synchronous: returns
 * after the solve with *info filled.  Returns MPS_OK, MPS_EINVAL, MPS_ENOMEM, MPS_EHIP, or
 * MPS_ERANGE / MPS_ENOTSUP when a device condition was raised during the solve. */
int bicg(const mp_csr *A, const mp_plan *plan, const mp_vec *b, mp_vec *x,
         const mp_solve_opts *opts, mp_solve_info *info, void *stream);

/* GPBiCG (Fig. 5 right; Zhang's updates z = zeta r + eta z - alpha u and
 * r = t - eta y - zeta A t).  Same conventions as bicg; the plan is needed only when
 * opts->transpose != 0 (NULL: built inside the call). */
int gpbicg(const mp_csr *A, const mp_plan *plan, const mp_vec *b, mp_vec *x,
           const mp_solve_opts *opts, mp_solve_info *info, void *stream);

/* CGS (conjugate gradient squared) for A x = b (or A^T x = b), one of the product-type methods
 * of Sec. 4 (Tables 1 and 3; the paper names it without printing it), with K = I, the shadow
 * residual r~ = r_0 and the stopping test (*):  u = r + beta q, p = u + beta (q + beta p)
 * (u = p = r first), alpha = rho / (r~, A p), q = u - alpha A p, u^ = u + q, x = x + alpha u^,
 * r = r - alpha A u^, beta = rho' / rho.  Statuses: MP_BREAKDOWN_RHO (rho = 0),
 * MP_BREAKDOWN_SIGMA ((r~, A p) = 0).  Same conventions as gpbicg (plan needed only when
 * opts->transpose != 0). */
int cgs(const mp_csr *A, const mp_plan *plan, const mp_vec *b, mp_vec *x,
        const mp_solve_opts *opts, mp_solve_info *info, void *stream);

/* BiCGSTAB for A x = b (or A^T x = b), the other product-type method of Sec. 4 (Tables 1 and 3,
 * unpreconditioned here), K = I, r~ = r_0, stopping test (*):  p = r + beta (p - omega v)
 * (p = r first), v = A p, alpha = rho / (r~, v), s = r - alpha v, t = A s,
 * omega = (t, s) / (t, t) (0 when (t, t) = 0), x = x + alpha p + omega s, r = s - omega t,
 * beta = (rho' / rho) (alpha / omega).  Statuses: MP_BREAKDOWN_RHO, MP_BREAKDOWN_SIGMA
 * ((r~, v) = 0) and MP_BREAKDOWN_ZETA (omega = 0 without convergence: the next beta is
 * undefined).  Same conventions as gpbicg. */
int bicgstab(const mp_csr *A, const mp_plan *plan, const mp_vec *b, mp_vec *x,
             const mp_solve_opts *opts, mp_solve_info *info, void *stream);

/* ILU(0) preconditioner (Sec. 4.2, Table 3: the paper's left preconditioner for BiCGSTAB): the
 * incomplete LU factorisation without fill-in, K = L U (L unit lower, U upper triangular, both
 * on the sparsity pattern of the square matrix A, whose every row must store its diagonal
 * element).  The factors are computed row by row, one RN per operation: for each stored column
 * k < i of row i in ascending order, a_ik <- RN(a_ik / a_kk), then a_ij <- RN(a_ij - RN(a_ik a_kj))
 * for each stored column j > k of row i, in ascending order, that row k also stores.  The rows
 * are processed in dependency levels (one launch per level).  mp_ilu0_create factors A
 * (synchronises `stream`, copies A's structure to the host for the level sets, allocates device
 * memory owned by the object; MPS_EINVAL for a missing diagonal element or a zero pivot).
 * mp_ilu0_apply: w = K^{-1} r = U^{-1} L^{-1} r, each row's sum r_i - sum_k l_ik y_k (and
 * y_i - sum_j u_ij w_j, then one RN division by u_ii) in the given accumulation mode, as the
 * sparse product sums a row (SEQ: r_i first, then the products in ascending column order; EXACT:
 * exactly, one rounding); asynchronous, level by level; the object's work vectors are shared by
 * its calls, which must not overlap in time.  mp_ilu0_apply_t: w = K^{-T} r = L^{-T} U^{-T} r
 * (the shadow system's preconditioner in BiCG, Fig. 5 left): y_i = (r_i - sum_k u_ki y_k) / u_ii
 * over the rows k < i that store column i, then w_i = y_i - sum_k l_ki w_k over the rows k > i
 * that store column i, each sum over ascending k (the transpose's storage order) in the given
 * mode; same conventions and shared work vectors as mp_ilu0_apply.  mp_ilu0_factors copies the
 * factors into lu (A's CSR layout, nnz elements).  Returns MPS_OK, MPS_EINVAL, MPS_ENOMEM or
 * MPS_EHIP. */
typedef struct mp_ilu mp_ilu;
int mp_ilu0_create(const mp_csr *A, void *stream, mp_ilu **ilu);
int mp_ilu0_destroy(mp_ilu *ilu);
int mp_ilu0_apply(const mp_ilu *ilu, const mp_vec *r, mp_vec *w, int mode, void *stream);
int mp_ilu0_apply_t(const mp_ilu *ilu, const mp_vec *r, mp_vec *w, int mode, void *stream);
int mp_ilu0_factors(const mp_ilu *ilu, mp_vec *lu, void *stream);

/* BiCGSTAB preconditioned by ILU(0) (Sec. 4.2, Table 3), K applied to the two search
 * directions so that the residual of the stopping test (*) stays b - A x:  p^ = K^{-1} p,
 * v = A p^, alpha = rho / (r~, v), s = r - alpha v, s^ = K^{-1} s, t = A s^,
 * omega = (t, s) / (t, t) (0 when (t, t) = 0), x = x + alpha p^ + omega s^, r = s - omega t.
 * The triangular solves take opts->mode like the products.  opts->transpose must be 0
 * (MPS_ENOTSUP).  Otherwise as bicgstab. */
int bicgstab_ilu0(const mp_csr *A, const mp_ilu *ilu, const mp_vec *b, mp_vec *x,
                  const mp_solve_opts *opts, mp_solve_info *info, void *stream);

/* BiCG preconditioned by ILU(0) (Fig. 5 left with K = L U): w = K^{-1} r, w~ = K^{-T} r~,
 * rho = (r~, w), beta = rho / rho_old, p = w + beta p, p~ = w~ + beta p~ (first iteration:
 * p = w, p~ = w~), z = A p, z~ = A^T p~, alpha = rho / (p~, z), x += alpha p, r -= alpha z,
 * r~ -= alpha z~, and the stopping test (*) on r = b - A x.  The figure prints rho = (w~, w),
 * which applies K twice and loses BiCG's biorthogonality; this solve uses rho = (r~, K^{-1} r)
 * = (K^{-T} r~, r), equal to it for K = I.  The triangular solves take opts->mode like the
 * products; plan as for bicg (NULL: built and freed here); opts->transpose must be 0
 * (MPS_ENOTSUP).  Statuses and conventions as bicg. */
int bicg_ilu0(const mp_csr *A, const mp_plan *plan, const mp_ilu *ilu, const mp_vec *b, mp_vec *x,
              const mp_solve_opts *opts, mp_solve_info *info, void *stream);

/* Batched GPBiCG: nsys systems A[0..nsys-1] (square, same precision, sizes may differ), each
 * with nrhs right-hand sides, solved as nsys * nrhs independent GPBiCG solves (the method of
 * Fig. 5 right, K = I, applied to many systems) that share every kernel launch: one captured
 * iteration graph advances all of them, and each solve stops on its own test.  Solve
 * i = s * nrhs + k takes b[i] (length A[s].row_dim) and writes x[i]; info[i] receives its
 * outcome.  Every x[i] is bit-identical to what gpbicg(&A[s], NULL, &b[i], &x[i], opts, ...)
 * produces.  opts as for gpbicg, except that opts->transpose must be 0 and opts->res_hist NULL
 * (MPS_ENOTSUP otherwise).  The library builds a block-diagonal copy of the matrices and
 * concatenated work vectors (each system padded to a multiple of 512 rows) for the duration of
 * the call and frees them before returning.  Inner products in a batch support exponent spans of
 * about 7500 bits at p = 256 (MPS_ENOTSUP beyond).  Synchronous; returns as gpbicg, plus
 * MPS_ENOTSUP for batches of more than 2^20 solves or 2^31 - 1 rows or stored entries. */
int gpbicg_batched(int nsys, const mp_csr *A, int nrhs, const mp_vec *b, mp_vec *x,
                   const mp_solve_opts *opts, mp_solve_info *info, void *stream);

/* Kernel timer (measurement only, not part of the paper's method).  mp_timer_create makes a
 * pool of HIP events for up to max_launches kernels on the current device (MPS_EINVAL outside
 * 1..2^20, MPS_EHIP if event creation fails).  While a timer is selected on the calling thread
 * (mp_timer_select; NULL deselects), the main kernel of each later call on that thread -- the
 * sparse product's kernel of mpspmv_csr / mpspmv_csr_t (not the launch that stages x) and the
 * kernel of mp_grad_vals -- is launched with its own start and stop events; launches beyond the
 * pool are not timed.  mp_timer_read waits for the timed kernels, returns the sum of their
 * durations in microseconds and their number, and empties the pool for reuse.  The timer is
 * owned by the caller and freed by mp_timer_destroy (which also deselects it). */
typedef struct mp_timer mp_timer;
int mp_timer_create(int max_launches, mp_timer **timer);
int mp_timer_select(mp_timer *timer);
int mp_timer_read(mp_timer *timer, double *total_us, int64_t *launches);
int mp_timer_destroy(mp_timer *timer);

/* Synchronise `stream`, then read and clear the calling device's status word into *flags
 * (MP_ST_* bits).  Returns MPS_OK, or MPS_ERANGE / MPS_ENOTSUP when such a bit was set. */
int mp_status(void *stream, uint32_t *flags);

#ifdef __cplusplus
}
#endif

#endif /* MPSPMV_H */
