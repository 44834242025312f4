// C ABI of the multiple-precision SpMV / Krylov library (declarations in include/mpspmv.h).
#include <hip/hip_runtime.h>

#include <algorithm>

#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <vector>

#include "../../include/mpspmv.h"
#include "api_internal.hpp"
#include "wide_internal.hpp"
#include "plan_internal.hpp"
#include "spmv_internal.hpp"
#include "vec_internal.hpp"

namespace mpapi {

thread_local LaunchEvents* g_launch_events = nullptr;
thread_local KernelTimer* g_timer = nullptr;

static thread_local char g_err[512] = "";

int fail(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return code;
}

void clear_error() { g_err[0] = 0; }

int hip_fail(hipError_t e, const char* what) {
  return fail(MPS_EHIP, "%s: %s", what, hipGetErrorString(e));
}

// ---- per-device context -----------------------------------------------------------------
static std::mutex g_ctx_mu;
static std::vector<DeviceCtx*> g_ctx;

int get_ctx(DeviceCtx** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  std::lock_guard<std::mutex> lk(g_ctx_mu);
  if ((int)g_ctx.size() <= dev) g_ctx.resize(dev + 1, nullptr);
  if (!g_ctx[dev]) {
    DeviceCtx* c = new DeviceCtx();
    c->device = dev;
    e = hipMalloc((void**)&c->status, sizeof(uint32_t) * 4);
    if (e != hipSuccess) {
      delete c;
      return fail(MPS_ENOMEM, "hipMalloc(status): %s", hipGetErrorString(e));
    }
    e = hipMemset(c->status, 0, sizeof(uint32_t) * 4);
    if (e != hipSuccess) return hip_fail(e, "hipMemset(status)");
    int r = dot_work_alloc(1, kDotRingLog2, kDotReps, kDotGroups, &c->dot_anchor, &c->dot_win,
                           &c->dot_ticket, nullptr);
    if (r) return r;
    e = hipMalloc((void**)&c->wide_win, sizeof(int64_t) * (size_t)mp::kWideSlots * mp::kWideDigits);
    if (e == hipSuccess) e = hipMalloc((void**)&c->wide_lock, sizeof(int32_t) * mp::kWideSlots);
    if (e != hipSuccess) return fail(MPS_ENOMEM, "hipMalloc(wide windows): %s", hipGetErrorString(e));
    e = hipMemset(c->wide_lock, 0, sizeof(int32_t) * mp::kWideSlots);
    if (e != hipSuccess) return hip_fail(e, "hipMemset(wide locks)");
    e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
    g_ctx[dev] = c;
  }
  *out = g_ctx[dev];
  return MPS_OK;
}

// ---- validation ---------------------------------------------------------------------------
int limbs_of(int prec) {
  switch (prec) {
    case 128: return 4;
    case 256: return 8;
    case 512: return 16;
    case 1024: return 32;
    default: return 0;
  }
}

int check_vec(const mp_vec* v, int64_t want_len, const char* name) {
  if (!v) return fail(MPS_EINVAL, "%s: null descriptor", name);
  if (v->len != want_len)
    return fail(MPS_EINVAL, "%s: length %lld, expected %lld", name, (long long)v->len,
                (long long)want_len);
  if (v->len < 0 || v->ld < v->len) return fail(MPS_EINVAL, "%s: bad len/ld", name);
  if (v->len > 0 && (!v->limb || !v->hdr)) return fail(MPS_EINVAL, "%s: null pointer", name);
  return MPS_OK;
}

static bool overlap(const void* a, size_t na, const void* b, size_t nb) {
  const char* pa = (const char*)a;
  const char* pb = (const char*)b;
  if (!pa || !pb || na == 0 || nb == 0) return false;
  return pa < pb + nb && pb < pa + na;
}

bool vec_overlap(const mp_vec* a, const mp_vec* b, int L) {
  const size_t la = (size_t)((L - 1) * a->ld + a->len) * 4, lb = (size_t)((L - 1) * b->ld + b->len) * 4;
  return overlap(a->limb, la, b->limb, lb) || overlap(a->hdr, (size_t)a->len * 4, b->hdr, (size_t)b->len * 4) ||
         overlap(a->limb, la, b->hdr, (size_t)b->len * 4) || overlap(a->hdr, (size_t)a->len * 4, b->limb, lb);
}

int check_csr(const mp_csr* A, int check_device_data, bool wide_ok) {
  if (!A) return fail(MPS_EINVAL, "A: null descriptor");
  if (!limbs_of(A->prec) && !(wide_ok && wide_limbs_of(A->prec)))
    return fail(MPS_EINVAL, "A: precision %d not supported here (128, 256, 512, 1024%s)", A->prec,
                wide_ok ? ", 2048, 4096, 8192" : "");
  if (A->row_dim < 0 || A->col_dim < 0 || A->nnz < 0)
    return fail(MPS_EINVAL, "A: negative dimension");
  if (A->nnz > INT32_MAX || A->row_dim >= INT32_MAX || A->col_dim >= INT32_MAX)
    return fail(MPS_EINVAL, "A: sizes must fit 32-bit indices");
  if (!A->row_ptr) return fail(MPS_EINVAL, "A: null row_ptr");
  if (A->nnz > 0 && !A->col_idx) return fail(MPS_EINVAL, "A: null col_idx");
  int r = check_vec(&A->val, A->nnz, "A.val");
  if (r) return r;
  if (check_device_data) {
    std::vector<int32_t> rp(A->row_dim + 1), ci(A->nnz);
    hipError_t e = hipMemcpy(rp.data(), A->row_ptr, rp.size() * 4, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy(row_ptr)");
    if (A->nnz) {
      e = hipMemcpy(ci.data(), A->col_idx, ci.size() * 4, hipMemcpyDeviceToHost);
      if (e != hipSuccess) return hip_fail(e, "hipMemcpy(col_idx)");
    }
    if (rp[0] != 0 || rp[A->row_dim] != A->nnz)
      return fail(MPS_EINVAL, "A: row_ptr must start at 0 and end at nnz");
    for (int64_t i = 0; i < A->row_dim; ++i) {
      if (rp[i + 1] < rp[i]) return fail(MPS_EINVAL, "A: row_ptr decreases at row %lld", (long long)i);
      for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
        if (ci[k] < 0 || ci[k] >= A->col_dim)
          return fail(MPS_EINVAL, "A: column index out of range in row %lld", (long long)i);
        if (k > rp[i] && ci[k] <= ci[k - 1])
          return fail(MPS_EINVAL, "A: columns not strictly ascending in row %lld", (long long)i);
      }
    }
  }
  return MPS_OK;
}

// ---- SpMV launch ----------------------------------------------------------------------------
// Rows per block (one wavefront per block): fewer rows per block give more, shorter waves, which
// hides latency on short rows; more rows per block amortise a block's fixed work on long ones.
// Every variant computes the same bits.
int default_rows_per_block(int64_t n_rows, int64_t nnz) {
  const int64_t avg = n_rows > 0 ? nnz / n_rows : 0;
  return avg <= 8 ? 16 : avg <= 24 ? 32 : 64;
}

bool valid_rows_per_block(int rpw) { return rpw == 16 || rpw == 32 || rpw == 64; }

int spmv_launch(int L, int64_t n_rows, const int32_t* row_ptr, const int32_t* col_idx,
                const mp_vec& val, const mp_vec& x, const mp_vec& y, int mode, uint32_t* status,
                const int32_t* done, hipStream_t s, const SpmvFuse* fuse,
                const SpmvBatch* batch, const SpmvVariant* var, int32_t dense_cols) {
  if (n_rows == 0) return MPS_OK;
  const SpmvVariant plain;
  if (!var) var = &plain;
  int rpw = var->rpw;
  uint32_t* const x_rec = var->x_rec;
  const int64_t x_len = var->x_len;
  if (x_rec && batch && batch->nrhs != 1) return fail(MPS_EINVAL, "staged x takes one right-hand side");
  const SpmvBatch one;
  if (!batch) batch = &one;
  bool pipe = var->pipe;
  if (!valid_rows_per_block(rpw)) {
    rpw = default_rows_per_block(n_rows, val.len);
    // plain SEQ products with long rows (more than 24 entries on average): the pipelined
    // kernel with 16 rows per block, whose rows' rounding chains advance together (the one-lane
    // kernel stages a block's entries row after row, so its chains would run one at a time)
    if (mode == MP_SEQ && !var->rows && !(fuse && fuse->nd > 0) && batch->nrhs == 1 && !done &&
        val.len > 24 * n_rows) {
      pipe = true;
      rpw = 16;
    }
  }
  if ((n_rows + rpw - 1) / rpw * batch->nrhs + (n_rows + 3) / 4 > (int64_t)UINT32_MAX)
    return fail(MPS_ENOTSUP, "too many row blocks for one launch");
  mp::SpmvArgs a;
  a.n_rows = n_rows;
  a.row_ptr = row_ptr;
  a.col_idx = col_idx;
  a.a_limb = val.limb;
  a.a_hdr = val.hdr;
  a.a_ld = val.ld;
  a.x_limb = x.limb;
  a.x_hdr = x.hdr;
  a.x_ld = x.ld;
  a.y_limb = y.limb;
  a.y_hdr = y.hdr;
  a.y_ld = y.ld;
  a.status = status;
  a.done = done;
  a.nrhs = batch->nrhs;
  a.x_rstride = batch->rstride;
  a.y_rstride = batch->rstride;
  a.pair_of_tile = batch->pair_of_tile;
  a.done_base = batch->done_base;
  a.done_stride = batch->done_stride;
  a.x_rec = x_rec;
  a.rows = var->rows;
  a.pipe = pipe ? 1 : 0;
  a.n_long = 0;
  a.long_blocks = 0;
  a.window = 0;
  a.n_win = 0;
  a.win_blocks = 0;
  a.dense_cols = dense_cols;
  a.wide_win = nullptr;
  a.wide_lock = nullptr;
  if (mode == MP_EXACT && !var->no_wide) {
    DeviceCtx* ctx;
    const int r = get_ctx(&ctx);
    if (r) return r;
    a.wide_win = ctx->wide_win;
    a.wide_lock = ctx->wide_lock;
  }
  // (lane groups need a row order; windowed chains also take the rows in their own order)
  if (mode == MP_SEQ && (var->rows || (var->pipe && var->windows)) && var->n_long > 0 && !(fuse && fuse->nd > 0) &&
      batch->nrhs == 1 &&
      !batch->pair_of_tile && !done && L <= 16) {  // lane groups hold at most 16 limbs
    a.n_long = std::min<int64_t>(var->n_long, n_rows);
    a.window = var->windows;
    if (var->windows) {  // four rows per block (one per wavefront), then sixteen (four per wavefront)
      a.n_win = var->windows == 1 ? a.n_long : std::min<int64_t>(var->n_win, a.n_long);
      a.win_blocks = (a.n_win + 3) / 4;
      a.long_blocks = a.win_blocks + (a.n_long - a.n_win + 15) / 16;
    } else {  // one row per lane group
      a.long_blocks = (a.n_long + 64 / L - 1) / (64 / L);
    }
  }
  if (var->rows && batch->nrhs != 1) return fail(MPS_EINVAL, "a row order takes one right-hand side");
  a.fd = mp::DotOut{};
  a.dots = mp::DotWork{};
  a.S = mp::Scalars{};
  a.ctl = nullptr;
  a.tiles_of_pair = nullptr;
  a.first_tile = nullptr;
  a.ndone = nullptr;
  for (int k = 0; k < 3; ++k) a.part[k] = mp::VecRef{};
  if (fuse && fuse->nd > 0) {
    if (fuse->nd > 3) return fail(MPS_EINVAL, "at most three inner products per product");
    a.fd.nd = fuse->nd;
    a.fd.epi = fuse->epi;
    a.fd.hist = fuse->hist;
    for (int k = 0; k < fuse->nd; ++k) {
      a.part[k] = fuse->part[k];
      a.fd.slot[k] = fuse->slot[k];
      a.fd.out[k] = fuse->out[k];
      a.fd.sslot[k] = fuse->sslot[k];
    }
    a.dots = fuse->dots;
    a.S = fuse->S;
    a.ctl = fuse->ctl;
    a.tiles_of_pair = fuse->tiles_of_pair;
    a.first_tile = fuse->first_tile;
    a.ndone = fuse->ndone;
  }
  if (x_rec && x_len > 0) {
    const unsigned g = (unsigned)std::min<int64_t>(16384, (x_len + 255) / 256);
    switch (L) {
      case 4: MPS_LAUNCH(true, false, mp::x_stage_kernel<4>, dim3(g), dim3(256), 0, s, x.limb, x.hdr, x.ld, x_len, x_rec); break;
      case 8: MPS_LAUNCH(true, false, mp::x_stage_kernel<8>, dim3(g), dim3(256), 0, s, x.limb, x.hdr, x.ld, x_len, x_rec); break;
      case 16: MPS_LAUNCH(true, false, mp::x_stage_kernel<16>, dim3(g), dim3(256), 0, s, x.limb, x.hdr, x.ld, x_len, x_rec); break;
      case 32: MPS_LAUNCH(true, false, mp::x_stage_kernel<32>, dim3(g), dim3(256), 0, s, x.limb, x.hdr, x.ld, x_len, x_rec); break;
      default: return fail(MPS_EINVAL, "bad limb count");
    }
  }
  if (a.fd.nd > 0) {
    launch_spmv_fused(L, a, mode, rpw, s);
  } else {
    switch (L) {
      case 4: launch_spmv<4, false>(a, mode, rpw, s); break;
      case 8: launch_spmv<8, false>(a, mode, rpw, s); break;
      case 16: launch_spmv<16, false>(a, mode, rpw, s); break;
      case 32: launch_spmv<32, false>(a, mode, rpw, s); break;
      default: return fail(MPS_EINVAL, "bad limb count");
    }
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "spmv launch");
  return MPS_OK;
}

// ---- allocation-free product --------------------------------------------------------------
// mpspmv_csr_noalloc keeps its x staging buffer and its status word in `scratch`, a file-scope
// device array: each GPU the library runs on holds one copy until the process ends, so the call
// allocates nothing.  Word 0 is the status word of these calls (mp_status reads it beside the
// context's); the staged x records start at byte kScratchRecOffset.  Host code never passes the
// array's name to the device: the per-device address comes from hipGetSymbolAddress.
constexpr size_t kScratchRecOffset = 256;
constexpr size_t kScratchRecBytes = size_t(32) << 20;  // staged x records: 32 MiB
constexpr int kScratchMaxDevices = 64;
static std::mutex g_scratch_mu;
static uint32_t* g_scratch_ptr[kScratchMaxDevices] = {};

}  // namespace mpapi

static __device__ __align__(256) uint32_t scratch[(mpapi::kScratchRecOffset + mpapi::kScratchRecBytes) / 4];

namespace mpapi {

// The calling device's copy of `scratch`, resolved once per device with that device current.
static int scratch_ptr(uint32_t** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev < 0 || dev >= kScratchMaxDevices)
    return fail(MPS_ENOTSUP, "mpspmv_csr_noalloc: device %d beyond the first %d", dev, kScratchMaxDevices);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!p) return fail(MPS_EHIP, "hipGetSymbolAddress(scratch) returned no address");
    g_scratch_ptr[dev] = static_cast<uint32_t*>(p);
  }
  *out = g_scratch_ptr[dev];
  return MPS_OK;
}

// The scratch status word of a device whose scratch address was resolved (else nullptr).
static uint32_t* scratch_status(int dev) {
  if (dev < 0 || dev >= kScratchMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return g_scratch_ptr[dev];
}

// Elements of x the scratch array can stage at L limbs (records of 8, 16, 32 or 64 words).
static int64_t scratch_max_x(int L) {
  const int64_t rec_bytes = 4 * mp::x_rec_words_of(L);
  return (int64_t)(kScratchRecBytes / rec_bytes);
}

}  // namespace mpapi

using namespace mpapi;

extern "C" {

const char* mp_last_error(void) { return g_err; }

int mp_validate_csr(const mp_csr* A, int check_device_data) {
  clear_error();
  return check_csr(A, check_device_data, true);
}

int mpspmv_csr(const mp_csr* A, const mp_vec* x, mp_vec* y, int mode, const mp_plan* plan,
               void* stream) {
  clear_error();
  int r = check_csr(A, 0, true);
  if (r) return r;
  if (plan && (r = check_plan(plan, A))) return r;
  if (mode != MP_SEQ && mode != MP_EXACT) return fail(MPS_EINVAL, "mode must be MP_SEQ or MP_EXACT");
  if ((r = check_vec(x, A->col_dim, "x"))) return r;
  if ((r = check_vec(y, A->row_dim, "y"))) return r;
  const int WL = wide_limbs_of(A->prec);
  const int L = WL ? WL : limbs_of(A->prec);
  if (vec_overlap(x, y, L) || vec_overlap(&A->val, y, L))
    return fail(MPS_EINVAL, "y overlaps an input");
  DeviceCtx* ctx;
  if ((r = get_ctx(&ctx))) return r;
  if (WL)
    return wide_spmv(L, A->row_dim, A->row_ptr, A->col_idx, A->val, *x, *y, mode, ctx->status, (hipStream_t)stream);
  const SpmvVariant var = plan ? plan_variant(plan, 0, mode) : SpmvVariant{};
  return spmv_launch(L, A->row_dim, A->row_ptr, A->col_idx, A->val, *x, *y, mode, ctx->status,
                     nullptr, (hipStream_t)stream, nullptr, nullptr, &var);
}

int mp_gemv(const mp_dense* A, const mp_vec* x, mp_vec* y, int mode, void* stream) {
  clear_error();
  if (!A) return fail(MPS_EINVAL, "A: null descriptor");
  const int L = limbs_of(A->prec);
  if (!L) return fail(MPS_EINVAL, "A: precision %d not in {128, 256, 512, 1024}", A->prec);
  if (A->rows < 0 || A->cols < 0) return fail(MPS_EINVAL, "A: negative dimension");
  if (A->cols > 0 && A->rows > (int64_t)INT32_MAX / A->cols)
    return fail(MPS_EINVAL, "A: rows * cols must fit 32-bit entry indices");
  if (mode != MP_SEQ && mode != MP_EXACT) return fail(MPS_EINVAL, "mode must be MP_SEQ or MP_EXACT");
  int r;
  if ((r = check_vec(&A->val, A->rows * A->cols, "A.val"))) return r;
  if ((r = check_vec(x, A->cols, "x"))) return r;
  if ((r = check_vec(y, A->rows, "y"))) return r;
  if (vec_overlap(x, y, L) || vec_overlap(&A->val, y, L)) return fail(MPS_EINVAL, "y overlaps an input");
  DeviceCtx* ctx;
  if ((r = get_ctx(&ctx))) return r;
  if (A->rows == 0) return MPS_OK;
  if (A->cols == 0) {  // every row is empty: y = +0
    mp::VecArgs a{};
    a.n = A->rows;
    a.v[0] = ref(*y);
    return launch_ew(L, EW_ZERO, a, (hipStream_t)stream);
  }
  // SEQ: the four-wavefront pipelined kernel (products formed beside the rows' rounding chains),
  // 16 rows per block, and rows of 16 or more entries by windowed chains (four per wavefront,
  // one per wavefront from 128 entries); EXACT: rows per block by the row length
  SpmvVariant var;
  var.rpw = mode == MP_SEQ ? 16 : 0;
  var.pipe = mode == MP_SEQ;
  if (mode == MP_SEQ && L <= 16 && A->cols >= 16) {
    var.n_long = A->rows;
    var.windows = 2;
    var.n_win = A->cols >= 128 ? A->rows : 0;
  }
  return spmv_launch(L, A->rows, nullptr, nullptr, A->val, *x, *y, mode, ctx->status, nullptr,
                     (hipStream_t)stream, nullptr, nullptr, &var, (int32_t)A->cols);
}

int mpspmv_csr_noalloc(const mp_csr* A, const mp_vec* x, mp_vec* y, int mode, void* stream) {
  clear_error();
  int r = check_csr(A, 0);
  if (r) return r;
  if (mode != MP_SEQ && mode != MP_EXACT) return fail(MPS_EINVAL, "mode must be MP_SEQ or MP_EXACT");
  if ((r = check_vec(x, A->col_dim, "x"))) return r;
  if ((r = check_vec(y, A->row_dim, "y"))) return r;
  const int L = limbs_of(A->prec);
  if (vec_overlap(x, y, L) || vec_overlap(&A->val, y, L))
    return fail(MPS_EINVAL, "y overlaps an input");
  const int64_t max_x = scratch_max_x(L);
  if (A->col_dim > max_x)
    return fail(MPS_ENOTSUP,
                "mpspmv_csr_noalloc: x has %lld elements, the scratch array stages at most %lld "
                "at p = %d",
                (long long)A->col_dim, (long long)max_x, A->prec);
  uint32_t* sp;
  if ((r = scratch_ptr(&sp))) return r;
  SpmvVariant var;
  var.x_rec = sp + kScratchRecOffset / 4;
  var.x_len = A->col_dim;
  var.no_wide = true;  // the global windows are allocated memory
  return spmv_launch(L, A->row_dim, A->row_ptr, A->col_idx, A->val, *x, *y, mode, sp, nullptr,
                     (hipStream_t)stream, nullptr, nullptr, &var);
}

int mp_timer_create(int max_launches, mp_timer** out) {
  clear_error();
  if (!out || max_launches < 1 || max_launches > (1 << 20))
    return fail(MPS_EINVAL, "mp_timer_create: need 1 <= max_launches <= 2^20 and an output");
  KernelTimer* t = new KernelTimer();
  hipError_t e = hipGetDevice(&t->device);
  t->ev = new hipEvent_t[2 * (size_t)max_launches]();
  for (int i = 0; e == hipSuccess && i < 2 * max_launches; ++i) e = hipEventCreate(&t->ev[i]);
  if (e != hipSuccess) {
    for (int i = 0; i < 2 * max_launches; ++i)
      if (t->ev[i]) (void)hipEventDestroy(t->ev[i]);
    delete[] t->ev;
    delete t;
    return hip_fail(e, "mp_timer_create");
  }
  t->cap = max_launches;
  *out = reinterpret_cast<mp_timer*>(t);
  return MPS_OK;
}

int mp_timer_select(mp_timer* t) {
  clear_error();
  g_timer = reinterpret_cast<KernelTimer*>(t);
  return MPS_OK;
}

int mp_timer_read(mp_timer* t, double* total_us, int64_t* launches) {
  clear_error();
  KernelTimer* k = reinterpret_cast<KernelTimer*>(t);
  if (!k || !total_us || !launches) return fail(MPS_EINVAL, "mp_timer_read: null argument");
  double us = 0;
  for (int i = 0; i < k->used; ++i) {
    hipError_t e = hipEventSynchronize(k->ev[2 * i + 1]);
    float ms = 0;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, k->ev[2 * i], k->ev[2 * i + 1]);
    if (e != hipSuccess) return hip_fail(e, "mp_timer_read");
    us += 1e3 * (double)ms;
  }
  *total_us = us;
  *launches = k->used;
  k->used = 0;
  return MPS_OK;
}

int mp_timer_destroy(mp_timer* t) {
  clear_error();
  KernelTimer* k = reinterpret_cast<KernelTimer*>(t);
  if (!k) return MPS_OK;
  if (g_timer == k) g_timer = nullptr;
  for (int i = 0; i < 2 * k->cap; ++i) (void)hipEventDestroy(k->ev[i]);
  delete[] k->ev;
  delete k;
  return MPS_OK;
}

int mp_status(void* stream, uint32_t* flags) {
  clear_error();
  DeviceCtx* ctx;
  int r = get_ctx(&ctx);
  if (r) return r;
  hipError_t e = hipStreamSynchronize((hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  uint32_t h = 0;
  e = hipMemcpy(&h, ctx->status, 4, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpy(status)");
  e = hipMemset(ctx->status, 0, 4);
  if (e != hipSuccess) return hip_fail(e, "hipMemset(status)");
  if (uint32_t* sw = scratch_status(ctx->device)) {  // the allocation-free calls' status word
    uint32_t h2 = 0;
    e = hipMemcpy(&h2, sw, 4, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy(scratch status)");
    e = hipMemset(sw, 0, 4);
    if (e != hipSuccess) return hip_fail(e, "hipMemset(scratch status)");
    h |= h2;
  }
  if (flags) *flags = h;
  if (h & MP_ST_RANGE) return fail(MPS_ERANGE, "a result exponent left the range");
  if (h & MP_ST_WINDOW) return fail(MPS_ENOTSUP, "an exact accumulation was wider than supported");
  return MPS_OK;
}

}  // extern "C"
