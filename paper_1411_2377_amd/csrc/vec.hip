// Vector entry points (y <- y + alpha x, exact inner product) and the launch helpers that the
// Krylov drivers share.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "../../include/mpspmv.h"
#include "api_internal.hpp"
#include "solver_kernels.hpp"
#include "vec_internal.hpp"
#include "wide_internal.hpp"

namespace mpapi {

int dot_work_alloc(int nslots, int ring_log2, int reps, int ngroups, int32_t** anchor, int64_t** win,
                   uint32_t** ticket, hipStream_t s, int nsolves) {
  const size_t nwin = (size_t)nslots * reps << ring_log2;
  const size_t ntk = (size_t)nsolves * (ngroups + 1) * mp::kTicketStride;
  hipError_t e = hipMalloc((void**)anchor, (size_t)2 * nslots * mp::kAnchorBins * sizeof(int32_t));
  if (e == hipSuccess) e = hipMalloc((void**)win, nwin * sizeof(int64_t));
  if (e == hipSuccess) e = hipMalloc((void**)ticket, ntk * sizeof(uint32_t));
  if (e != hipSuccess) return fail(MPS_ENOMEM, "inner-product workspace: %s", hipGetErrorString(e));
  e = hipMemsetAsync(*win, 0, nwin * sizeof(int64_t), s);
  if (e == hipSuccess) e = hipMemsetAsync(*ticket, 0, ntk * sizeof(uint32_t), s);
  if (e != hipSuccess) return hip_fail(e, "inner-product workspace");
  const unsigned g = (unsigned)std::min<int64_t>(1024, ((int64_t)nslots * mp::kAnchorBins + 255) / 256);
  hipLaunchKernelGGL(mp::dot_work_init_kernel, dim3(g), dim3(256), 0, s, *anchor, nslots);
  e = hipGetLastError();
  if (e == hipSuccess && !s) e = hipDeviceSynchronize();
  return e == hipSuccess ? MPS_OK : hip_fail(e, "inner-product workspace init");
}

mp::VecRef ref(const mp_vec& v) {
  mp::VecRef r;
  r.limb = v.limb;
  r.hdr = v.hdr;
  r.ld = v.ld;
  return r;
}

// Blocks per inner product: one 256-element pass each, at most 2048 (more passes per block
// beyond that).
unsigned dot_grid(int64_t n) {
  const int64_t g = (n + mp::kDotThreads - 1) / mp::kDotThreads;
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(g, 2048));
}

mp::DotWork dot_work(int32_t* anchor, int64_t* win, uint32_t* ticket, int nslots, int ring_log2,
                     int reps, int ngroups) {
  mp::DotWork w;
  w.anchor = anchor;
  w.win = win;
  w.ticket = ticket;
  w.ring_log2 = ring_log2;
  w.reps = reps;
  w.ngroups = ngroups;
  w.nslots = nslots;
  return w;
}

unsigned ew_grid(int64_t n) {
  int64_t g = (n + 255) / 256;
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(g, 8192));
}

// A batch (vectors of whole kTile tiles, one solve per tile): one 256-thread block per half
// tile, one element per thread, so that every block belongs to one solve.
static unsigned ew_grid_of(const mp::VecArgs& a) {
  return a.batch.pair_of_tile ? (unsigned)(a.n / 256) : ew_grid(a.n);
}

int launch_dot(int L, const mp::DotArgs& a, hipStream_t s) {
  if (a.o.nd < 1 || a.o.nd > mp::kDotMaxND) return fail(MPS_EINVAL, "bad inner-product count");
  // a batch: one block per 256 elements (every block belongs to one solve)
  const unsigned g = a.batch.pair_of_tile ? (unsigned)(a.n / mp::kDotThreads) : dot_grid(a.n);
  const dim3 grid(g, a.o.nd);
  switch (L) {
    case 4: MPS_LAUNCH(true, true, mp::dot_kernel<4>, grid, dim3(mp::kDotThreads), 0, s, a); break;
    case 8: MPS_LAUNCH(true, true, mp::dot_kernel<8>, grid, dim3(mp::kDotThreads), 0, s, a); break;
    case 16: MPS_LAUNCH(true, true, mp::dot_kernel<16>, grid, dim3(mp::kDotThreads), 0, s, a); break;
    case 32: MPS_LAUNCH(true, true, mp::dot_kernel<32>, grid, dim3(mp::kDotThreads), 0, s, a); break;
    default: return fail(MPS_EINVAL, "bad limb count");
  }
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? MPS_OK : hip_fail(e, "dot launch");
}

#define MPS_EW_CASES(KERNEL, ARG)                                                             \
  switch (L) {                                                                                \
    case 4: MPS_LAUNCH(true, true, mp::KERNEL<4>, dim3(g), dim3(256), 0, s, ARG); break;          \
    case 8: MPS_LAUNCH(true, true, mp::KERNEL<8>, dim3(g), dim3(256), 0, s, ARG); break;          \
    case 16: MPS_LAUNCH(true, true, mp::KERNEL<16>, dim3(g), dim3(256), 0, s, ARG); break;        \
    case 32: MPS_LAUNCH(true, true, mp::KERNEL<32>, dim3(g), dim3(256), 0, s, ARG); break;        \
    default: return fail(MPS_EINVAL, "bad limb count");                                       \
  }

// the update steps: with their prologue and epilogue, or (batches) without
#define MPS_EW_CASES_SEP(KERNEL, ARG, SEP)                                                    \
  if (SEP) {                                                                                  \
    switch (L) {                                                                              \
      case 4: MPS_LAUNCH(true, true, (mp::KERNEL<4, true>), dim3(g), dim3(256), 0, s, ARG); break;   \
      case 8: MPS_LAUNCH(true, true, (mp::KERNEL<8, true>), dim3(g), dim3(256), 0, s, ARG); break;   \
      case 16: MPS_LAUNCH(true, true, (mp::KERNEL<16, true>), dim3(g), dim3(256), 0, s, ARG); break; \
      case 32: MPS_LAUNCH(true, true, (mp::KERNEL<32, true>), dim3(g), dim3(256), 0, s, ARG); break; \
      default: return fail(MPS_EINVAL, "bad limb count");                                     \
    }                                                                                         \
  } else {                                                                                    \
    switch (L) {                                                                              \
      case 4: MPS_LAUNCH(true, true, (mp::KERNEL<4, false>), dim3(g), dim3(256), 0, s, ARG); break;  \
      case 8: MPS_LAUNCH(true, true, (mp::KERNEL<8, false>), dim3(g), dim3(256), 0, s, ARG); break;  \
      case 16: MPS_LAUNCH(true, true, (mp::KERNEL<16, false>), dim3(g), dim3(256), 0, s, ARG); break; \
      case 32: MPS_LAUNCH(true, true, (mp::KERNEL<32, false>), dim3(g), dim3(256), 0, s, ARG); break; \
      default: return fail(MPS_EINVAL, "bad limb count");                                     \
    }                                                                                         \
  }

int launch_ew(int L, EwKind kind, const mp::VecArgs& a, hipStream_t s) {
  if (a.n == 0) return MPS_OK;
  const unsigned g = ew_grid_of(a);
  switch (kind) {
    case EW_AXPY: MPS_EW_CASES(axpy_kernel, a); break;
    case EW_COPY: MPS_EW_CASES(copy_kernel, a); break;
    case EW_ZERO: MPS_EW_CASES(zero_kernel, a); break;
    case EW_SUB: MPS_EW_CASES(sub_kernel, a); break;
    case EW_BICG_DIR: MPS_EW_CASES(bicg_dir_kernel, a); break;
    case EW_BICG_UPDATE: MPS_EW_CASES_SEP(bicg_update_kernel, a, a.pro_sep); break;
    case EW_GP_DIR: MPS_EW_CASES(gp_dir_kernel, a); break;
    case EW_GP_TSY: MPS_EW_CASES_SEP(gp_tsy_kernel, a, a.pro_sep); break;
    case EW_CGS_DIR: MPS_EW_CASES(cgs_dir_kernel, a); break;
    case EW_CGS_QUX: MPS_EW_CASES(cgs_qux_kernel, a); break;
    case EW_CGS_R: MPS_EW_CASES(cgs_r_kernel, a); break;
    case EW_STAB_DIR: MPS_EW_CASES(stab_dir_kernel, a); break;
    case EW_STAB_S: MPS_EW_CASES(stab_s_kernel, a); break;
    case EW_STAB_XR: MPS_EW_CASES(stab_xr_kernel, a); break;
    default: return fail(MPS_EINVAL, "bad element-wise kernel");
  }
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? MPS_OK : hip_fail(e, "element-wise launch");
}

int launch_gp_update(int L, const mp::GpUpdArgs& a, hipStream_t s) {
  if (a.a.n == 0) return MPS_OK;
  const unsigned g = ew_grid_of(a.a);
  MPS_EW_CASES_SEP(gp_update_kernel, a, a.a.pro_sep);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? MPS_OK : hip_fail(e, "gp_update launch");
}

int launch_epilogue(int L, const mp::EpiArgs& a, int npairs, hipStream_t s) {
  const dim3 g((unsigned)npairs);
  switch (L) {
    case 4: MPS_LAUNCH(true, true, mp::epilogue_kernel<4>, g, dim3(64), 0, s, a); break;
    case 8: MPS_LAUNCH(true, true, mp::epilogue_kernel<8>, g, dim3(64), 0, s, a); break;
    case 16: MPS_LAUNCH(true, true, mp::epilogue_kernel<16>, g, dim3(64), 0, s, a); break;
    case 32: MPS_LAUNCH(true, true, mp::epilogue_kernel<32>, g, dim3(64), 0, s, a); break;
    default: return fail(MPS_EINVAL, "bad limb count");
  }
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? MPS_OK : hip_fail(e, "epilogue launch");
}

int launch_prologue(int L, const mp::ProArgs& a, int npairs, hipStream_t s) {
  const dim3 g((unsigned)npairs);
  switch (L) {
    case 4: MPS_LAUNCH(true, true, mp::prologue_kernel<4>, g, dim3(64), 0, s, a); break;
    case 8: MPS_LAUNCH(true, true, mp::prologue_kernel<8>, g, dim3(64), 0, s, a); break;
    case 16: MPS_LAUNCH(true, true, mp::prologue_kernel<16>, g, dim3(64), 0, s, a); break;
    case 32: MPS_LAUNCH(true, true, mp::prologue_kernel<32>, g, dim3(64), 0, s, a); break;
    default: return fail(MPS_EINVAL, "bad limb count");
  }
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? MPS_OK : hip_fail(e, "prologue launch");
}

int set_scalar(int L, const mp::VecRef& out, const uint32_t* m, int32_t hdr, hipStream_t s,
               int64_t count, int64_t step) {
  const unsigned g = (unsigned)std::max<int64_t>(1, std::min<int64_t>(1024, (count + 255) / 256));
  switch (L) {
    case 4: {
      mp::ConstArgs<4> a;
      a.out = out; a.hdr = hdr; a.count = count; a.step = step;
      for (int k = 0; k < 4; ++k) a.m[k] = m[k];
      hipLaunchKernelGGL(mp::set_scalar_kernel<4>, dim3(g), dim3(256), 0, s, a);
      break;
    }
    case 8: {
      mp::ConstArgs<8> a;
      a.out = out; a.hdr = hdr; a.count = count; a.step = step;
      for (int k = 0; k < 8; ++k) a.m[k] = m[k];
      hipLaunchKernelGGL(mp::set_scalar_kernel<8>, dim3(g), dim3(256), 0, s, a);
      break;
    }
    case 16: {
      mp::ConstArgs<16> a;
      a.out = out; a.hdr = hdr; a.count = count; a.step = step;
      for (int k = 0; k < 16; ++k) a.m[k] = m[k];
      hipLaunchKernelGGL(mp::set_scalar_kernel<16>, dim3(g), dim3(256), 0, s, a);
      break;
    }
    case 32: {
      mp::ConstArgs<32> a;
      a.out = out; a.hdr = hdr; a.count = count; a.step = step;
      for (int k = 0; k < 32; ++k) a.m[k] = m[k];
      hipLaunchKernelGGL(mp::set_scalar_kernel<32>, dim3(g), dim3(256), 0, s, a);
      break;
    }
    default: return fail(MPS_EINVAL, "bad limb count");
  }
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? MPS_OK : hip_fail(e, "set_scalar launch");
}

int check_scalar(const mp_vec* v, const char* name) { return check_vec(v, 1, name); }

}  // namespace mpapi

using namespace mpapi;

extern "C" {

int mp_axpy(const mp_vec* alpha, const mp_vec* x, mp_vec* y, int prec, void* stream) {
  clear_error();
  const int WL = wide_limbs_of(prec);
  const int L = WL ? WL : limbs_of(prec);
  if (!L) return fail(MPS_EINVAL, "precision %d not in {128, 256, 512, 1024, 2048, 4096, 8192}", prec);
  int r;
  if ((r = check_scalar(alpha, "alpha"))) return r;
  if (!x || !y) return fail(MPS_EINVAL, "null vector");
  if ((r = check_vec(x, y->len, "x"))) return r;
  if ((r = check_vec(y, y->len, "y"))) return r;
  if (vec_overlap(x, y, L) || vec_overlap(alpha, y, L)) return fail(MPS_EINVAL, "y overlaps an input");
  DeviceCtx* ctx;
  if ((r = get_ctx(&ctx))) return r;
  mp::VecArgs a{};
  a.n = y->len;
  a.v[0] = ref(*y);
  a.v[1] = ref(*x);
  a.v[2] = ref(*alpha);
  a.ctl = nullptr;
  a.status = ctx->status;
  if (WL) return wide_axpy(L, 0, *alpha, *x, *y, y->len, ctx->status, (hipStream_t)stream);
  return launch_ew(L, EW_AXPY, a, (hipStream_t)stream);
}

int mp_dot(const mp_vec* x, const mp_vec* y, mp_vec* out, int prec, void* stream) {
  clear_error();
  const int WL = wide_limbs_of(prec);
  const int L = WL ? WL : limbs_of(prec);
  if (!L) return fail(MPS_EINVAL, "precision %d not in {128, 256, 512, 1024, 2048, 4096, 8192}", prec);
  int r;
  if (!x || !y) return fail(MPS_EINVAL, "null vector");
  if ((r = check_vec(y, x->len, "y"))) return r;
  if ((r = check_vec(x, x->len, "x"))) return r;
  if ((r = check_scalar(out, "out"))) return r;
  if (vec_overlap(x, out, L) || vec_overlap(y, out, L)) return fail(MPS_EINVAL, "out overlaps an input");
  DeviceCtx* ctx;
  if ((r = get_ctx(&ctx))) return r;
  if (WL) return wide_dot(L, *x, *y, *out, ctx->status, (hipStream_t)stream);
  mp::DotArgs a{};
  a.n = x->len;
  a.x[0] = ref(*x);
  a.y[0] = ref(*y);
  a.o.nd = 1;
  a.o.out[0] = ref(*out);
  a.o.sslot[0] = -1;
  a.o.slot[0] = 0;
  a.o.epi = mp::EPI_NONE;
  a.w = dot_work(ctx->dot_anchor, ctx->dot_win, ctx->dot_ticket, 1, kDotRingLog2, kDotReps, kDotGroups);
  a.ctl = nullptr;
  a.status = ctx->status;
  return launch_dot(L, a, (hipStream_t)stream);
}

}  // extern "C"
