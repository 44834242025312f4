// BiCG and GPBiCG drivers (Kouya, Fig. 5 with K = I; stopping test (*) of Sec. 4.1).
//
// The whole iteration stays on the device: the scalars (rho, alpha, beta, zeta, eta, ...) are
// formed by the epilogues of the inner-product kernels, the stopping test is the exact integer
// comparison q < (thr + ulp/2)^2 (no square root per iteration), and a done flag turns every
// later kernel into a no-op.  One iteration is captured as a HIP graph and replayed `chunk`
// times between host polls of the 32-byte control block; since replays past the stopping point
// do nothing, every result is bit-identical for every chunk size (and for eager launches).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <initializer_list>
#include <string>
#include <utility>
#include <vector>

#include "../../include/mpspmv.h"
#include "api_internal.hpp"
#include "ilu_internal.hpp"
#include "plan_internal.hpp"
#include "batch_kernels.hpp"
#include "spmv_internal.hpp"
#include "solver_kernels.hpp"
#include "vec_internal.hpp"
#include "wide_internal.hpp"

namespace mpapi {

// ---- exact decimal constants: RN_p(m * 10^e) --------------------------------------------
namespace {

struct Big {
  std::vector<uint32_t> d;  // little endian
  int bits() const {
    for (int i = (int)d.size() - 1; i >= 0; --i)
      if (d[i]) return 32 * i + 32 - __builtin_clz(d[i]);
    return 0;
  }
  int bit(int i) const {
    const int w = i >> 5;
    return (w < (int)d.size()) ? (int)((d[w] >> (i & 31)) & 1u) : 0;
  }
  void mul_small(uint32_t m) {
    uint64_t c = 0;
    for (auto& x : d) {
      const uint64_t t = (uint64_t)x * m + c;
      x = (uint32_t)t;
      c = t >> 32;
    }
    if (c) d.push_back((uint32_t)c);
  }
  void shl1_or(int b) {
    uint32_t c = (uint32_t)b;
    for (auto& x : d) {
      const uint32_t n = x >> 31;
      x = (x << 1) | c;
      c = n;
    }
    if (c) d.push_back(c);
  }
  int cmp(const Big& o) const {
    const size_t n = std::max(d.size(), o.d.size());
    for (size_t i = n; i-- > 0;) {
      const uint32_t a = i < d.size() ? d[i] : 0u, b = i < o.d.size() ? o.d[i] : 0u;
      if (a != b) return a < b ? -1 : 1;
    }
    return 0;
  }
  void sub(const Big& o) {  // *this >= o
    int64_t br = 0;
    for (size_t i = 0; i < d.size(); ++i) {
      const int64_t t = (int64_t)d[i] - (i < o.d.size() ? o.d[i] : 0u) - br;
      d[i] = (uint32_t)t;
      br = t < 0;
    }
  }
  bool zero() const {
    for (auto x : d)
      if (x) return false;
    return true;
  }
};

}  // namespace

// RN_p of |m| * 10^e10 into (limbs, hdr); returns false if out of the supported range.
bool decimal_to_mp(int64_t m, int64_t e10, int L, uint32_t* limbs, int32_t* hdr) {
  const int p = 32 * L;
  for (int k = 0; k < L; ++k) limbs[k] = 0;
  if (m == 0) {
    *hdr = (int32_t)0x80000000u;
    return true;
  }
  if (e10 > 2000 || e10 < -2000) return false;
  const int sign = m < 0;
  const uint64_t am = m < 0 ? (uint64_t)(-(m + 1)) + 1u : (uint64_t)m;
  Big N;
  N.d = {(uint32_t)am, (uint32_t)(am >> 32)};
  Big D;
  D.d = {1u};
  if (e10 >= 0)
    for (int64_t i = 0; i < e10; ++i) N.mul_small(10);
  else
    for (int64_t i = 0; i < -e10; ++i) D.mul_small(10);
  // Q = floor(N * 2^s / D) with at least p + 2 bits; sticky = remainder != 0
  int s = p + 3 + D.bits() - N.bits();
  if (s < 0) s = 0;
  Big Q, R;
  Q.d = {0u};
  R.d = {0u};
  const int xb = N.bits() + s;
  for (int i = xb - 1; i >= 0; --i) {
    const int b = (i >= s) ? N.bit(i - s) : 0;
    R.shl1_or(b);
    Q.shl1_or(0);
    if (R.cmp(D) >= 0) {
      R.sub(D);
      Q.d[0] |= 1u;
    }
  }
  const bool sticky = !R.zero();
  const int nq = Q.bits();
  const int drop = nq - p;  // >= 2
  // mantissa = Q >> drop; tail = low `drop` bits
  std::vector<uint32_t> mant(L, 0u);
  for (int i = 0; i < p; ++i)
    if (Q.bit(i + drop)) mant[i >> 5] |= 1u << (i & 31);
  const int half = Q.bit(drop - 1);
  bool rest = sticky;
  for (int i = 0; i < drop - 1 && !rest; ++i) rest = Q.bit(i) != 0;
  int64_t e = (int64_t)nq - s;  // value = Q * 2^-s, Q in [2^(nq-1), 2^nq)
  const bool up = half && (rest || (mant[0] & 1u));
  if (up) {
    uint64_t c = 1;
    for (int k = 0; k < L; ++k) {
      const uint64_t t = (uint64_t)mant[k] + c;
      mant[k] = (uint32_t)t;
      c = t >> 32;
    }
    if (c) {
      mant[L - 1] = 0x80000000u;
      e += 1;
    }
  }
  if (e > mp::kEmax || e < mp::kEmin) return false;
  for (int k = 0; k < L; ++k) limbs[k] = mant[k];
  *hdr = (int32_t)(((uint32_t)e << 1) | (uint32_t)sign);
  return true;
}

namespace {

double mp_to_double(const uint32_t* limbs, int32_t hdr, int L, int64_t ld) {
  const int32_t e = hdr >> 1;
  if (e == mp::kZeroE) return 0.0;
  const uint64_t top = ((uint64_t)limbs[(L - 1) * ld] << 32) | limbs[(L - 2) * ld];
  double v = std::ldexp((double)top, (int)std::max<int64_t>(-100000, std::min<int64_t>(100000, (int64_t)e - 64)));
  return (hdr & 1) ? -v : v;
}

// Device workspace of one solve, or of a batch of independent solves ("pairs") that share
// every launch: then the vectors are the pairs' segments side by side (each a whole number of
// mp::kTile tiles), and scalars, control blocks and inner-product slots are per pair.
struct Work {
  int L = 0;
  int64_t n = 0;
  int nvec = 0;
  int npairs = 1;
  int nrhs = 1;
  int64_t rstride = 0;       // batch: elements per right-hand side (all systems, padded)
  int ring_log2 = kDotRingLog2;  // inner-product rings: 2^ring_log2 digits, reps replicas,
  int reps = kDotReps;           // tickets in ngroups groups
  int ngroups = kDotGroups;
  int32_t* pair_of_tile = nullptr;
  int32_t* tiles_of_pair = nullptr;
  int32_t* first_tile = nullptr;
  int32_t* ndone = nullptr;
  int32_t* h_ndone = nullptr;  // pinned
  uint32_t* vlimb = nullptr;
  int32_t* vhdr = nullptr;
  mp::Scalars S{nullptr, nullptr, 0};
  mp::Ctl* ctl = nullptr;
  int32_t* anchor = nullptr;  // inner-product slots (see DotWork)
  int64_t* win = nullptr;
  uint32_t* ticket = nullptr;
  mp::Ctl* h_ctl = nullptr;  // pinned
  hipStream_t ws = nullptr;
  hipEvent_t ev = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  mp_solve_profile* prof = nullptr;  // kernel timing (eager launches)
  hipEvent_t pe0 = nullptr, pe1 = nullptr;

  mp::VecRef vec(int i) const {
    mp::VecRef r;
    r.limb = vlimb + (size_t)i * L * n;
    r.hdr = vhdr + (size_t)i * n;
    r.ld = n;
    return r;
  }
  mp_vec desc(int i) const {
    mp_vec v;
    v.limb = vlimb + (size_t)i * L * n;
    v.hdr = vhdr + (size_t)i * n;
    v.len = n;
    v.ld = n;
    return v;
  }
  bool batched() const { return pair_of_tile != nullptr; }
  mp::DotWork dots() const {
    return dot_work(anchor, win, ticket, npairs * mp::kDotSlots, ring_log2, reps, ngroups);
  }
  mp::BatchMap batch_map() const {
    mp::BatchMap b;
    b.pair_of_tile = pair_of_tile;
    b.tiles_of_pair = tiles_of_pair;
    b.first_tile = first_tile;
    b.ndone = ndone;
    return b;
  }
  ~Work() {
    if (exec) hipGraphExecDestroy(exec);
    if (graph) hipGraphDestroy(graph);
    if (ws) hipStreamSynchronize(ws);
    hipFree(pair_of_tile);
    hipFree(tiles_of_pair);
    hipFree(first_tile);
    hipFree(ndone);
    if (h_ndone) hipHostFree(h_ndone);
    hipFree(vlimb);
    hipFree(vhdr);
    hipFree(S.limb);
    hipFree(S.hdr);
    hipFree(ctl);
    hipFree(anchor);
    hipFree(win);
    hipFree(ticket);
    if (h_ctl) hipHostFree(h_ctl);
    if (ev) hipEventDestroy(ev);
    if (pe0) hipEventDestroy(pe0);
    if (pe1) hipEventDestroy(pe1);
    if (ws) hipStreamDestroy(ws);
  }
};

// Allocate the workspace of W.npairs solves (W.npairs, and for a batch the tile maps, set by
// the caller) with nvec work vectors of n elements.
int work_alloc(Work& W, int L, int64_t n, int nvec, hipStream_t user) {
  W.L = L;
  W.n = n;
  W.nvec = nvec;
  const int64_t nsc = (int64_t)W.npairs * mp::kNumScalars;
  W.S.ld = nsc;
  hipError_t e = hipMalloc((void**)&W.vlimb, std::max<size_t>(4, (size_t)nvec * L * n * 4));
  if (e == hipSuccess) e = hipMalloc((void**)&W.vhdr, std::max<size_t>(4, (size_t)nvec * n * 4));
  if (e == hipSuccess) e = hipMalloc((void**)&W.S.limb, (size_t)L * nsc * 4);
  if (e == hipSuccess) e = hipMalloc((void**)&W.S.hdr, (size_t)nsc * 4);
  if (e == hipSuccess) e = hipMalloc((void**)&W.ctl, sizeof(mp::Ctl) * W.npairs);
  if (e == hipSuccess && W.batched()) e = hipMalloc((void**)&W.ndone, sizeof(int32_t));
  if (e != hipSuccess) return fail(MPS_ENOMEM, "solver workspace: %s", hipGetErrorString(e));
  e = hipHostMalloc((void**)&W.h_ctl, sizeof(mp::Ctl) * W.npairs, hipHostMallocDefault);
  if (e == hipSuccess && W.batched()) e = hipHostMalloc((void**)&W.h_ndone, sizeof(int32_t), hipHostMallocDefault);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&W.ws, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&W.ev, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventRecord(W.ev, user);
  if (e == hipSuccess) e = hipStreamWaitEvent(W.ws, W.ev, 0);
  if (e == hipSuccess && W.ndone) e = hipMemsetAsync(W.ndone, 0, sizeof(int32_t), W.ws);
  if (e != hipSuccess) return hip_fail(e, "solver setup");
  int r = dot_work_alloc(W.npairs * mp::kDotSlots, W.ring_log2, W.reps, W.ngroups, &W.anchor, &W.win,
                         &W.ticket, W.ws, W.npairs);
  if (r) return r;
  // every scalar slot starts as +0
  mp::VecArgs a{};
  a.n = nsc;
  a.v[0].limb = W.S.limb;
  a.v[0].hdr = W.S.hdr;
  a.v[0].ld = nsc;
  return launch_ew(L, EW_ZERO, a, W.ws);
}

// Profiling: class of a launch and its algorithmic bytes.
// [0] sparse products that also form inner products, [1] other sparse products, [2] directions,
// [3] updates, [4] GPBiCG's t, s, y
enum ProfClass { PROF_SPMV_DOT = 0, PROF_SPMV = 1, PROF_DIR = 2, PROF_UPD = 3, PROF_TSY = 4 };

int prof_init(Work& W, mp_solve_profile* prof) {
  if (!prof) return MPS_OK;
  W.prof = prof;
  hipError_t e = hipEventCreate(&W.pe0);
  if (e == hipSuccess) e = hipEventCreate(&W.pe1);
  return e == hipSuccess ? MPS_OK : hip_fail(e, "profile events");
}

// Run `launch`; when profiling, have its kernels record their start and end on two events and
// add the kernel time, a launch and `bytes` to class c.
template <class F>
int timed(const Work& W, int c, double bytes, F&& launch) {
  if (!W.prof) return launch();
  LaunchEvents ev{W.pe0, W.pe1};
  g_launch_events = &ev;  // the kernels record their own start and end
  const int r = launch();
  g_launch_events = nullptr;
  if (r) return r;
  hipError_t e = hipEventSynchronize(W.pe1);
  float ms = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, W.pe0, W.pe1);
  if (e != hipSuccess) return hip_fail(e, "profile events");
  W.prof->launches[c] += 1;
  W.prof->us[c] += 1e3 * (double)ms;
  W.prof->bytes[c] += bytes;
  return MPS_OK;
}

// algorithmic bytes: k vectors of W.n elements; a sparse product (entries, x, y, row pointers)
double vec_bytes(const Work& W, int k) { return (double)k * W.n * (4.0 * W.L + 4.0); }
double spmv_bytes(const mp_csr* A, int L) {
  return (double)A->nnz * (4.0 * L + 8.0) + (double)(A->row_dim + A->col_dim) * (4.0 * L + 4.0) +
         4.0 * (double)(A->row_dim + 1);
}

// y = Aop v with the given arrays (Aop = A or A^T via the plan), no-op once done.
struct Op {
  int64_t n_out;
  const int32_t* row_ptr;
  const int32_t* col_idx;
  mp_vec val;
  SpmvVariant var[2];  // kernel variant per mode
};

// y = Aop x on the workspace stream; `gated`: a no-op once the solve is done (for a batch,
// the blocks of finished solves return at once).
int apply(const Work& W, const Op& op, int mode, const mp::VecRef& x, const mp::VecRef& y,
          uint32_t* status, bool gated, const SpmvFuse* fuse = nullptr) {
  mp_vec xv{x.limb, x.hdr, 0, x.ld}, yv{y.limb, y.hdr, 0, y.ld};
  if (W.batched()) {
    SpmvBatch b;
    b.nrhs = W.nrhs;
    b.rstride = W.rstride;
    b.pair_of_tile = W.pair_of_tile;
    b.done_base = &W.ctl->done;
    b.done_stride = (int64_t)(sizeof(mp::Ctl) / sizeof(int32_t));
    return spmv_launch(W.L, op.n_out, op.row_ptr, op.col_idx, op.val, xv, yv, mode, status,
                       nullptr, W.ws, fuse, &b, &op.var[mode]);
  }
  return spmv_launch(W.L, op.n_out, op.row_ptr, op.col_idx, op.val, xv, yv, mode, status,
                     gated ? &W.ctl->done : nullptr, W.ws, fuse, nullptr, &op.var[mode]);
}

// Inner products of an SpMV output y with up to three vectors ({nullptr}: y itself), each
// {partner, slot, scalar}; the launch's last block rounds them and runs epilogue epi.
struct FuseItem {
  mp::VecRef part;
  int slot;
  int scalar;
};

SpmvFuse fuse_of(const Work& W, int epi, std::initializer_list<FuseItem> list,
                 const mp::VecRef& hist = mp::VecRef{nullptr, nullptr, 0}) {
  SpmvFuse F;
  for (auto& it : list) {
    F.part[F.nd] = it.part;
    F.slot[F.nd] = it.slot;
    F.out[F.nd] = mp::slot_ref(W.S, it.scalar);
    F.sslot[F.nd] = it.scalar;
    ++F.nd;
  }
  F.epi = epi;
  F.hist = hist;
  F.dots = W.dots();
  F.S = W.S;
  F.ctl = W.ctl;
  F.tiles_of_pair = W.tiles_of_pair;
  F.first_tile = W.first_tile;
  F.ndone = W.ndone;
  return F;
}

mp::DotArgs dot_args(const Work& W, uint32_t* status, int epi) {
  mp::DotArgs a{};
  a.n = W.n;
  a.S = W.S;
  a.w = W.dots();
  a.ctl = W.ctl;
  a.status = status;
  a.o.epi = epi;
  a.batch = W.batch_map();
  return a;
}

// Element-wise step arguments; `fd`: the inner products the kernel forms ({slot, scalar} each)
// and the epilogue its launch ends with.
mp::VecArgs ew_args(const Work& W, uint32_t* status) {
  mp::VecArgs a{};
  a.n = W.n;
  a.S = W.S;
  a.ctl = W.ctl;
  a.status = status;
  a.batch = W.batch_map();
  a.dots = W.dots();
  return a;
}

void set_fd(const Work& W, mp::VecArgs& a, int epi, std::initializer_list<std::pair<int, int>> list,
            const mp::VecRef& hist = mp::VecRef{nullptr, nullptr, 0}) {
  a.fd.nd = 0;
  for (auto& it : list) {
    a.fd.slot[a.fd.nd] = it.first;
    a.fd.out[a.fd.nd] = mp::slot_ref(W.S, it.second);
    a.fd.sslot[a.fd.nd] = it.second;
    ++a.fd.nd;
  }
  a.fd.epi = epi;
  a.fd.hist = hist;
}

int check_solve_args(const mp_csr* A, const mp_vec* b, const mp_vec* x, const mp_solve_opts* o,
                     mp_solve_info* info) {
  int r = check_csr(A, 0);
  if (r) return r;
  if (A->row_dim != A->col_dim) return fail(MPS_EINVAL, "A must be square");
  if (!o || !info) return fail(MPS_EINVAL, "null opts/info");
  if (o->mode != MP_SEQ && o->mode != MP_EXACT) return fail(MPS_EINVAL, "mode must be MP_SEQ or MP_EXACT");
  if (o->maxit < 0 || o->maxit > INT32_MAX) return fail(MPS_EINVAL, "maxit out of range");
  if ((r = check_vec(b, A->row_dim, "b"))) return r;
  if ((r = check_vec(x, A->row_dim, "x"))) return r;
  const int L = limbs_of(A->prec);
  if (vec_overlap(b, x, L)) return fail(MPS_EINVAL, "x overlaps b");
  if (o->res_hist && o->res_hist->len > 0 && (!o->res_hist->limb || !o->res_hist->hdr))
    return fail(MPS_EINVAL, "res_hist: null pointer");
  return MPS_OK;
}

// Common setup: control block, tolerance constants, x0, r0 = b - A x0, rt = r0, q0, rho1.
// Vector slots used: 0 = r, 1 = rt, 2 = scratch.
int solve_setup(Work& W, const Op& Aop, const mp_vec* b, mp_vec* x, const mp_solve_opts* o,
                uint32_t* status) {
  const int L = W.L;
  hipLaunchKernelGGL(mp::ctl_init_kernel, dim3((W.npairs + 255) / 256), dim3(256), 0, W.ws, W.ctl,
                     W.npairs, (int32_t)o->maxit, (int32_t)(o->res_hist ? o->res_hist->len : 0));
  uint32_t m[32];
  int32_t h;
  if (!decimal_to_mp(o->rtol_m, o->rtol_e10, L, m, &h)) return fail(MPS_EINVAL, "rtol out of range");
  int r = set_scalar(L, mp::slot_ref(W.S, mp::S_CREL), m, h, W.ws, W.npairs, mp::kNumScalars);
  if (r) return r;
  if (!decimal_to_mp(o->atol_m, o->atol_e10, L, m, &h)) return fail(MPS_EINVAL, "atol out of range");
  if ((r = set_scalar(L, mp::slot_ref(W.S, mp::S_CABS), m, h, W.ws, W.npairs, mp::kNumScalars))) return r;
  mp::VecArgs a = ew_args(W, status);
  if (o->use_x0) {
    // r = b - Aop x0
    if ((r = apply(W, Aop, o->mode, ref(*x), W.vec(2), status, false))) return r;
    a.v[0] = W.vec(0);
    a.v[1] = ref(*b);
    a.v[2] = W.vec(2);
    if ((r = launch_ew(L, EW_SUB, a, W.ws))) return r;
  } else {
    // x0 = +0, r = b - A x0 = b exactly
    a.v[0] = ref(*x);
    if ((r = launch_ew(L, EW_ZERO, a, W.ws))) return r;
    a.v[0] = W.vec(0);
    a.v[1] = ref(*b);
    if ((r = launch_ew(L, EW_COPY, a, W.ws))) return r;
  }
  a.v[0] = W.vec(1);
  a.v[1] = W.vec(0);
  if ((r = launch_ew(L, EW_COPY, a, W.ws))) return r;
  mp::DotArgs d = dot_args(W, status, mp::EPI_SETUP);
  d.o.nd = 2;
  d.x[0] = W.vec(0);
  d.y[0] = W.vec(0);
  d.o.out[0] = mp::slot_ref(W.S, mp::S_Q0);
  d.o.sslot[0] = mp::S_Q0;
  d.o.slot[0] = 1;
  d.x[1] = W.vec(1);
  d.y[1] = W.vec(0);
  d.o.out[1] = mp::slot_ref(W.S, mp::S_RHO);
  d.o.sslot[1] = mp::S_RHO;
  d.o.slot[1] = 2;
  return launch_dot(L, d, W.ws);
}

// Wait for the enqueued work and report whether every solve of W is done.
int poll_done(Work& W, bool* done) {
  hipError_t e;
  if (W.batched())
    e = hipMemcpyAsync(W.h_ndone, W.ndone, sizeof(int32_t), hipMemcpyDeviceToHost, W.ws);
  else
    e = hipMemcpyAsync(W.h_ctl, W.ctl, sizeof(mp::Ctl), hipMemcpyDeviceToHost, W.ws);
  if (e == hipSuccess) e = hipStreamSynchronize(W.ws);
  if (e != hipSuccess) return hip_fail(e, "poll");
  *done = W.batched() ? (*W.h_ndone >= W.npairs) : (W.h_ctl->done != 0);
  return MPS_OK;
}

// Run iterations until the control block says done (graph replays, or eager when chunk <= 0).
template <class F>
int run_iterations(Work& W, const mp_solve_opts* o, F&& enqueue_iteration) {
  hipError_t e;
  int r;
  const int chunk = W.prof ? 0 : o->chunk;
  // the setup may already have finished the solve
  bool done = false;
  if ((r = poll_done(W, &done))) return r;
  if (done) return MPS_OK;
  if (chunk > 0) {
    e = hipStreamBeginCapture(W.ws, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
    r = enqueue_iteration();
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(W.ws, &g);
    if (r) {
      if (g) hipGraphDestroy(g);
      return r;
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    W.graph = g;
    e = hipGraphInstantiate(&W.exec, W.graph, nullptr, nullptr, 0);
    if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
  }
  int64_t launched = 0;
  const int64_t limit = o->maxit + 2;
  while (true) {
    const int batch = chunk > 0 ? chunk : 1;
    for (int c = 0; c < batch; ++c) {
      if (chunk > 0) {
        e = hipGraphLaunch(W.exec, W.ws);
        if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
      } else if ((r = enqueue_iteration())) {
        return r;
      }
      ++launched;
    }
    if ((r = poll_done(W, &done))) return r;
    if (done) break;
    if (launched > limit) return fail(MPS_EHIP, "solver did not reach its iteration limit");
  }
  return MPS_OK;
}

int finish_solve(Work& W, mp_solve_info* info, uint32_t* status) {
  info->status = W.h_ctl->status;
  info->iters = W.h_ctl->iters;
  // display-only residual ratio from q and q0
  std::vector<uint32_t> sl((size_t)W.L * mp::kNumScalars);
  std::vector<int32_t> sh(mp::kNumScalars);
  hipError_t e = hipMemcpyAsync(sl.data(), W.S.limb, sl.size() * 4, hipMemcpyDeviceToHost, W.ws);
  if (e == hipSuccess) e = hipMemcpyAsync(sh.data(), W.S.hdr, sh.size() * 4, hipMemcpyDeviceToHost, W.ws);
  if (e == hipSuccess) e = hipStreamSynchronize(W.ws);
  if (e != hipSuccess) return hip_fail(e, "result readback");
  const double q0 = mp_to_double(sl.data() + mp::S_Q0, sh[mp::S_Q0], W.L, W.S.ld);
  const double q = info->iters > 0 ? mp_to_double(sl.data() + mp::S_Q, sh[mp::S_Q], W.L, W.S.ld) : q0;
  info->final_rel_res = q0 > 0 ? std::sqrt(q / q0) : 0.0;
  const uint32_t fl = W.h_ctl->flags;
  if (fl & mp::kStRange) return fail(MPS_ERANGE, "a result exponent left the range during the solve");
  if (fl & mp::kStWindow) return fail(MPS_ENOTSUP, "an exact accumulation was wider than supported");
  (void)status;
  return MPS_OK;
}

struct OwnedPlan {
  mp_plan* p = nullptr;
  ~OwnedPlan() {
    if (p) plan_free(p);
  }
};

// The two products of a solve: Aop (the system matrix) and its transpose.
int make_ops(const mp_csr* A, const mp_plan* P, int transpose, Op* op, Op* opT) {
  Op a{A->row_dim, A->row_ptr, A->col_idx, A->val, {}};
  Op t{A->col_dim, nullptr, nullptr, A->val, {}};
  if (P) {
    for (int m = 0; m < 2; ++m) {
      a.var[m] = plan_variant(P, 0, m);
      t.var[m] = plan_variant(P, 1, m);
    }
    t.row_ptr = P->t_row_ptr;
    t.col_idx = P->t_col_idx;
    t.val.limb = P->t_limb;
    t.val.hdr = P->t_hdr;
    t.val.len = P->nnz;
    t.val.ld = P->nnz;
  }
  *op = transpose ? t : a;
  *opT = transpose ? a : t;
  return MPS_OK;
}

}  // namespace

int bicg_impl(const mp_csr* A, const mp_plan* plan, const mp_vec* b, mp_vec* x,
              const mp_solve_opts* o, mp_solve_info* info, hipStream_t user) {
  int r = check_solve_args(A, b, x, o, info);
  if (r) return r;
  DeviceCtx* ctx;
  if ((r = get_ctx(&ctx))) return r;
  OwnedPlan own;
  if (!plan) {
    if ((r = plan_build(A, user, &own.p))) return r;
    plan = own.p;
  } else if ((r = check_plan(plan, A))) {
    return r;
  }
  const int L = limbs_of(A->prec);
  Work W;
  // vectors: 0 r, 1 rt, 2 scratch/z, 3 p, 4 pt, 5 zt
  if ((r = work_alloc(W, L, A->row_dim, 6, user))) return r;
  Op op, opT;
  make_ops(A, plan, o->transpose, &op, &opT);
  uint32_t* st = ctx->status;
  if ((r = solve_setup(W, op, b, x, o, st))) return r;
  if ((r = prof_init(W, o->profile))) return r;
  const mp::VecRef R = W.vec(0), RT = W.vec(1), Z = W.vec(2), P = W.vec(3), PT = W.vec(4), ZT = W.vec(5);
  const mp::VecRef X = ref(*x);
  mp::VecRef hist{nullptr, nullptr, 0};
  if (o->res_hist && o->res_hist->len > 0) hist = ref(*o->res_hist);
  const double sp_bytes = spmv_bytes(A, L), dot1 = vec_bytes(W, 1);
  // per iteration: directions; z = A p with sigma = (pt, z); zt = A^T pt; the updates, which
  // first form alpha = rho / sigma, with (r, r) and (rt, r) (their last block: stopping test,
  // beta)
  auto iteration = [&]() -> int {
    int rr;
    mp::VecArgs a = ew_args(W, st);
    a.v[0] = P; a.v[1] = PT; a.v[2] = R; a.v[3] = RT;
    if ((rr = timed(W, PROF_DIR, vec_bytes(W, 6), [&] { return launch_ew(L, EW_BICG_DIR, a, W.ws); })))
      return rr;
    const SpmvFuse sig = fuse_of(W, mp::EPI_NONE, {{PT, 0, mp::S_SIGMA}});
    if ((rr = timed(W, PROF_SPMV_DOT, sp_bytes + dot1, [&] { return apply(W, op, o->mode, P, Z, st, true, &sig); })))
      return rr;
    if ((rr = timed(W, PROF_SPMV, sp_bytes, [&] { return apply(W, opT, o->mode, PT, ZT, st, true); })))
      return rr;
    a = ew_args(W, st);
    a.v[0] = X; a.v[1] = R; a.v[2] = RT; a.v[3] = P; a.v[4] = Z; a.v[5] = ZT;
    set_fd(W, a, mp::EPI_BICG_CONV, {{1, mp::S_Q}, {2, mp::S_RHO_NEXT}}, hist);
    return timed(W, PROF_UPD, vec_bytes(W, 9), [&] { return launch_ew(L, EW_BICG_UPDATE, a, W.ws); });
  };
  if ((r = run_iterations(W, o, iteration))) return r;
  return finish_solve(W, info, st);
}

// GPBiCG work vectors: 0 r, 1 rt, 2 scratch, 3 p, 4 q, 5 t, 6 v, 7 s, 8 w, 9 y, 10 u, 11 z
constexpr int kGpVectors = 12;

// Clear the vectors the first GPBiCG iteration reads before writing (u, z, s, w, t, p, q, v,
// y = +0; beta = +0 since the scalars were cleared).
int gp_clear(const Work& W, uint32_t* st) {
  mp::VecArgs a = ew_args(W, st);
  for (int i = 3; i < kGpVectors; ++i) {
    a.v[0] = W.vec(i);
    int r = launch_ew(W.L, EW_ZERO, a, W.ws);
    if (r) return r;
  }
  return MPS_OK;
}

// One GPBiCG iteration (Fig. 5 with K = I) on the workspace stream.
int gp_iteration(const Work& W, const Op& op, int mode, const mp::VecRef& X, const mp::VecRef& hist,
                 uint32_t* st, double sp_bytes) {
  const int L = W.L;
  const double dot1 = vec_bytes(W, 1);
  const mp::VecRef R = W.vec(0), RT = W.vec(1), P = W.vec(3), Q = W.vec(4), T = W.vec(5),
                   V = W.vec(6), S = W.vec(7), Wv = W.vec(8), Y = W.vec(9), U = W.vec(10),
                   Z = W.vec(11);
  const mp::VecRef self{nullptr, nullptr, 0};
  int rr;
  mp::VecArgs a = ew_args(W, st);
  a.v[0] = P; a.v[1] = Wv; a.v[2] = R; a.v[3] = V; a.v[4] = Q; a.v[5] = U;
  if ((rr = timed(W, PROF_DIR, vec_bytes(W, 7), [&] { return launch_ew(L, EW_GP_DIR, a, W.ws); }))) return rr;
  // q = A p with (rt, q)
  const SpmvFuse den = fuse_of(W, mp::EPI_NONE, {{RT, 0, mp::S_DEN}});
  if ((rr = timed(W, PROF_SPMV_DOT, sp_bytes + dot1, [&] { return apply(W, op, mode, P, Q, st, true, &den); }))) return rr;
  // a batch forms each solve's step prologue once, in a launch of its own
  auto prologue = [&](int kind) {
    mp::ProArgs pa{};
    pa.kind = kind;
    pa.S = W.S;
    pa.ctl = W.ctl;
    pa.dots = W.dots();
    pa.ndone = W.ndone;
    pa.status = st;
    return launch_prologue(L, pa, W.npairs, W.ws);
  };
  if (W.batched() && (rr = prologue(mp::PRO_GP_ALPHA))) return rr;
  // alpha = rho / (rt, q); t, s, y with (y, y) and (y, t)
  a = ew_args(W, st);
  a.pro_sep = W.batched() ? 1 : 0;
  a.v[0] = T; a.v[1] = S; a.v[2] = Y; a.v[3] = R; a.v[4] = Q; a.v[5] = Wv;
  set_fd(W, a, mp::EPI_NONE, {{3, mp::S_MU1}, {5, mp::S_MU3}});
  if ((rr = timed(W, PROF_TSY, vec_bytes(W, 7), [&] { return launch_ew(L, EW_GP_TSY, a, W.ws); }))) return rr;
  // v = A t with (v, t), (v, y), (v, v)
  const SpmvFuse mus =
      fuse_of(W, mp::EPI_NONE, {{T, 4, mp::S_MU2}, {Y, 6, mp::S_MU4}, {self, 7, mp::S_MU5}});
  if ((rr = timed(W, PROF_SPMV_DOT, sp_bytes + 2 * dot1, [&] { return apply(W, op, mode, T, V, st, true, &mus); }))) return rr;
  // zeta, eta from mu1..mu5; u, z, x, r with (r, r) and (rt, r) (their last block: stopping
  // test, beta)
  if (W.batched() && (rr = prologue(mp::PRO_GP_ZETA))) return rr;
  mp::GpUpdArgs g{};
  g.a = ew_args(W, st);
  g.a.pro_sep = W.batched() ? 1 : 0;
  g.a.v[0] = U; g.a.v[1] = Z; g.a.v[2] = X; g.a.v[3] = R; g.a.v[4] = Q; g.a.v[5] = S;
  g.a.v[6] = P; g.a.v[7] = T;
  set_fd(W, g.a, mp::EPI_GP_CONV, {{1, mp::S_Q}, {2, mp::S_RHO_NEXT}}, hist);
  g.y = Y;
  g.v = V;
  g.rt = RT;
  if ((rr = timed(W, PROF_UPD, vec_bytes(W, 15), [&] { return launch_gp_update(L, g, W.ws); }))) return rr;
  if (!W.batched()) return MPS_OK;
  mp::EpiArgs ea{};  // a batch runs the stopping test and beta in a launch of its own
  ea.epi = mp::EPI_GP_CONV;
  ea.S = W.S;
  ea.ctl = W.ctl;
  ea.ndone = W.ndone;
  ea.status = st;
  return launch_epilogue(L, ea, W.npairs, W.ws);
}

int gpbicg_impl(const mp_csr* A, const mp_plan* plan, const mp_vec* b, mp_vec* x,
                const mp_solve_opts* o, mp_solve_info* info, hipStream_t user) {
  int r = check_solve_args(A, b, x, o, info);
  if (r) return r;
  DeviceCtx* ctx;
  if ((r = get_ctx(&ctx))) return r;
  OwnedPlan own;
  if (o->transpose) {
    if (!plan) {
      if ((r = plan_build(A, user, &own.p))) return r;
      plan = own.p;
    } else if ((r = check_plan(plan, A))) {
      return r;
    }
  } else if (plan && (r = check_plan(plan, A))) {
    return r;
  }
  const int L = limbs_of(A->prec);
  Work W;
  if ((r = work_alloc(W, L, A->row_dim, kGpVectors, user))) return r;
  Op op, opT;
  make_ops(A, plan, o->transpose, &op, &opT);
  uint32_t* st = ctx->status;
  if ((r = solve_setup(W, op, b, x, o, st))) return r;
  if ((r = gp_clear(W, st))) return r;
  const mp::VecRef X = ref(*x);
  mp::VecRef hist{nullptr, nullptr, 0};
  if (o->res_hist && o->res_hist->len > 0) hist = ref(*o->res_hist);
  if ((r = prof_init(W, o->profile))) return r;
  const double sp_bytes = spmv_bytes(A, L);
  auto iteration = [&]() -> int { return gp_iteration(W, op, o->mode, X, hist, st, sp_bytes); };
  if ((r = run_iterations(W, o, iteration))) return r;
  return finish_solve(W, info, st);
}

// ---- CGS and BiCGSTAB -------------------------------------------------------------------
// The paper's other two product-type methods (Sec. 4, Tables 1 and 3), K = I, with the same
// setup, stopping test, graph replays and breakdown statuses as BiCG and GPBiCG.

namespace {

// Set up a solve whose plan is needed only for a transposed system (NULL: built here).
int plan_for(const mp_csr* A, const mp_plan*& plan, const mp_solve_opts* o, OwnedPlan& own,
             hipStream_t user) {
  int r;
  if (o->transpose) {
    if (!plan) {
      if ((r = plan_build(A, user, &own.p))) return r;
      plan = own.p;
    } else if ((r = check_plan(plan, A))) {
      return r;
    }
  } else if (plan && (r = check_plan(plan, A))) {
    return r;
  }
  return MPS_OK;
}

// Clear work vectors first..last-1 (those a first iteration reads before writing).
int clear_vectors(const Work& W, int first, int last, uint32_t* st) {
  mp::VecArgs a = ew_args(W, st);
  for (int i = first; i < last; ++i) {
    a.v[0] = W.vec(i);
    int r = launch_ew(W.L, EW_ZERO, a, W.ws);
    if (r) return r;
  }
  return MPS_OK;
}

}  // namespace

// CGS work vectors: 0 r, 1 rt, 2 A p and then A u^, 3 u, 4 p, 5 q, 6 u^
int cgs_impl(const mp_csr* A, const mp_plan* plan, const mp_vec* b, mp_vec* x,
             const mp_solve_opts* o, mp_solve_info* info, hipStream_t user) {
  int r = check_solve_args(A, b, x, o, info);
  if (r) return r;
  DeviceCtx* ctx;
  if ((r = get_ctx(&ctx))) return r;
  OwnedPlan own;
  if ((r = plan_for(A, plan, o, own, user))) return r;
  const int L = limbs_of(A->prec);
  Work W;
  if ((r = work_alloc(W, L, A->row_dim, 7, user))) return r;
  Op op, opT;
  make_ops(A, plan, o->transpose, &op, &opT);
  uint32_t* st = ctx->status;
  if ((r = solve_setup(W, op, b, x, o, st))) return r;
  if ((r = clear_vectors(W, 2, 7, st))) return r;
  if ((r = prof_init(W, o->profile))) return r;
  const mp::VecRef R = W.vec(0), RT = W.vec(1), AV = W.vec(2), U = W.vec(3), P = W.vec(4),
                   Q = W.vec(5), UH = W.vec(6);
  const mp::VecRef X = ref(*x);
  mp::VecRef hist{nullptr, nullptr, 0};
  if (o->res_hist && o->res_hist->len > 0) hist = ref(*o->res_hist);
  const double sp_bytes = spmv_bytes(A, L), dot1 = vec_bytes(W, 1);
  // per iteration: u, p; A p with (r~, A p); alpha, q, u^, x; A u^; r with (r, r) and (r~, r)
  // (their last block: stopping test, beta)
  auto iteration = [&]() -> int {
    int rr;
    mp::VecArgs a = ew_args(W, st);
    a.v[0] = U; a.v[1] = P; a.v[2] = R; a.v[3] = Q;
    if ((rr = timed(W, PROF_DIR, vec_bytes(W, 5), [&] { return launch_ew(L, EW_CGS_DIR, a, W.ws); })))
      return rr;
    const SpmvFuse sig = fuse_of(W, mp::EPI_NONE, {{RT, 0, mp::S_SIGMA}});
    if ((rr = timed(W, PROF_SPMV_DOT, sp_bytes + dot1, [&] { return apply(W, op, o->mode, P, AV, st, true, &sig); })))
      return rr;
    a = ew_args(W, st);
    a.v[0] = Q; a.v[1] = UH; a.v[2] = X; a.v[3] = U; a.v[4] = AV;
    set_fd(W, a, mp::EPI_NONE, {});
    if ((rr = timed(W, PROF_TSY, vec_bytes(W, 6), [&] { return launch_ew(L, EW_CGS_QUX, a, W.ws); })))
      return rr;
    if ((rr = timed(W, PROF_SPMV, sp_bytes, [&] { return apply(W, op, o->mode, UH, AV, st, true); })))
      return rr;
    a = ew_args(W, st);
    a.v[0] = R; a.v[1] = AV; a.v[2] = RT;
    set_fd(W, a, mp::EPI_BICG_CONV, {{1, mp::S_Q}, {2, mp::S_RHO_NEXT}}, hist);
    return timed(W, PROF_UPD, vec_bytes(W, 4), [&] { return launch_ew(L, EW_CGS_R, a, W.ws); });
  };
  if ((r = run_iterations(W, o, iteration))) return r;
  return finish_solve(W, info, st);
}

// BiCGSTAB work vectors: 0 r, 1 rt, 2 (unused), 3 p, 4 v = A p, 5 s, 6 t = A s
int bicgstab_impl(const mp_csr* A, const mp_plan* plan, const mp_vec* b, mp_vec* x,
                  const mp_solve_opts* o, mp_solve_info* info, hipStream_t user) {
  int r = check_solve_args(A, b, x, o, info);
  if (r) return r;
  DeviceCtx* ctx;
  if ((r = get_ctx(&ctx))) return r;
  OwnedPlan own;
  if ((r = plan_for(A, plan, o, own, user))) return r;
  const int L = limbs_of(A->prec);
  Work W;
  if ((r = work_alloc(W, L, A->row_dim, 7, user))) return r;
  Op op, opT;
  make_ops(A, plan, o->transpose, &op, &opT);
  uint32_t* st = ctx->status;
  if ((r = solve_setup(W, op, b, x, o, st))) return r;
  if ((r = clear_vectors(W, 2, 7, st))) return r;
  if ((r = prof_init(W, o->profile))) return r;
  const mp::VecRef R = W.vec(0), RT = W.vec(1), P = W.vec(3), V = W.vec(4), S = W.vec(5),
                   T = W.vec(6);
  const mp::VecRef X = ref(*x);
  const mp::VecRef self{nullptr, nullptr, 0};
  mp::VecRef hist{nullptr, nullptr, 0};
  if (o->res_hist && o->res_hist->len > 0) hist = ref(*o->res_hist);
  const double sp_bytes = spmv_bytes(A, L), dot1 = vec_bytes(W, 1);
  // per iteration: p; v = A p with (r~, v); alpha, s; t = A s with (t, s), (t, t); omega, x, r
  // with (r, r) and (r~, r) (their last block: stopping test, omega = 0 exit, beta)
  auto iteration = [&]() -> int {
    int rr;
    mp::VecArgs a = ew_args(W, st);
    a.v[0] = P; a.v[1] = R; a.v[2] = V;
    if ((rr = timed(W, PROF_DIR, vec_bytes(W, 4), [&] { return launch_ew(L, EW_STAB_DIR, a, W.ws); })))
      return rr;
    const SpmvFuse sig = fuse_of(W, mp::EPI_NONE, {{RT, 0, mp::S_SIGMA}});
    if ((rr = timed(W, PROF_SPMV_DOT, sp_bytes + dot1, [&] { return apply(W, op, o->mode, P, V, st, true, &sig); })))
      return rr;
    a = ew_args(W, st);
    a.v[0] = S; a.v[1] = R; a.v[2] = V;
    set_fd(W, a, mp::EPI_NONE, {});
    if ((rr = timed(W, PROF_TSY, vec_bytes(W, 3), [&] { return launch_ew(L, EW_STAB_S, a, W.ws); })))
      return rr;
    const SpmvFuse ts = fuse_of(W, mp::EPI_NONE, {{S, 4, mp::S_MU2}, {self, 7, mp::S_MU5}});
    if ((rr = timed(W, PROF_SPMV_DOT, sp_bytes + dot1, [&] { return apply(W, op, o->mode, S, T, st, true, &ts); })))
      return rr;
    a = ew_args(W, st);
    a.v[0] = X; a.v[1] = R; a.v[2] = P; a.v[3] = S; a.v[4] = T; a.v[5] = RT;
    set_fd(W, a, mp::EPI_GP_CONV, {{1, mp::S_Q}, {2, mp::S_RHO_NEXT}}, hist);
    return timed(W, PROF_UPD, vec_bytes(W, 8), [&] { return launch_ew(L, EW_STAB_XR, a, W.ws); });
  };
  if ((r = run_iterations(W, o, iteration))) return r;
  return finish_solve(W, info, st);
}

// BiCGSTAB with the ILU(0) preconditioner K on its two search directions (Sec. 4.2, Table 3):
// p^ = K^{-1} p, v = A p^, s = r - alpha v, s^ = K^{-1} s, t = A s^, omega = (t, s) / (t, t),
// x = x + alpha p^ + omega s^, r = s - omega t; the (*) test reads r = b - A x.
// Work vectors: 0 r, 1 rt, 2 p^, 3 p, 4 v, 5 s, 6 t, 7 s^
int bicgstab_ilu0_impl(const mp_csr* A, const mp_ilu* K, const mp_vec* b, mp_vec* x,
                       const mp_solve_opts* o, mp_solve_info* info, hipStream_t user) {
  int r = check_solve_args(A, b, x, o, info);
  if (r) return r;
  if (o->transpose) return fail(MPS_ENOTSUP, "the preconditioned solve takes A, not its transpose");
  if ((r = check_ilu(K, A))) return r;
  DeviceCtx* ctx;
  if ((r = get_ctx(&ctx))) return r;
  const int L = limbs_of(A->prec);
  Work W;
  if ((r = work_alloc(W, L, A->row_dim, 8, user))) return r;
  Op op, opT;
  make_ops(A, nullptr, 0, &op, &opT);
  uint32_t* st = ctx->status;
  if ((r = solve_setup(W, op, b, x, o, st))) return r;
  if ((r = clear_vectors(W, 2, 8, st))) return r;
  if ((r = prof_init(W, o->profile))) return r;
  const mp::VecRef R = W.vec(0), RT = W.vec(1), PH = W.vec(2), P = W.vec(3), V = W.vec(4),
                   S = W.vec(5), T = W.vec(6), SH = W.vec(7);
  const mp::VecRef X = ref(*x);
  const mp::VecRef self{nullptr, nullptr, 0};
  mp::VecRef hist{nullptr, nullptr, 0};
  if (o->res_hist && o->res_hist->len > 0) hist = ref(*o->res_hist);
  const double sp_bytes = spmv_bytes(A, L), dot1 = vec_bytes(W, 1);
  auto iteration = [&]() -> int {
    int rr;
    mp::VecArgs a = ew_args(W, st);
    a.v[0] = P; a.v[1] = R; a.v[2] = V;
    if ((rr = timed(W, PROF_DIR, vec_bytes(W, 4), [&] { return launch_ew(L, EW_STAB_DIR, a, W.ws); })))
      return rr;
    if ((rr = ilu_apply(K, W.desc(3), W.desc(2), o->mode, st, W.ctl, W.ws))) return rr;
    const SpmvFuse sig = fuse_of(W, mp::EPI_NONE, {{RT, 0, mp::S_SIGMA}});
    if ((rr = timed(W, PROF_SPMV_DOT, sp_bytes + dot1, [&] { return apply(W, op, o->mode, PH, V, st, true, &sig); })))
      return rr;
    a = ew_args(W, st);
    a.v[0] = S; a.v[1] = R; a.v[2] = V;
    set_fd(W, a, mp::EPI_NONE, {});
    if ((rr = timed(W, PROF_TSY, vec_bytes(W, 3), [&] { return launch_ew(L, EW_STAB_S, a, W.ws); })))
      return rr;
    if ((rr = ilu_apply(K, W.desc(5), W.desc(7), o->mode, st, W.ctl, W.ws))) return rr;
    const SpmvFuse ts = fuse_of(W, mp::EPI_NONE, {{S, 4, mp::S_MU2}, {self, 7, mp::S_MU5}});
    if ((rr = timed(W, PROF_SPMV_DOT, sp_bytes + dot1, [&] { return apply(W, op, o->mode, SH, T, st, true, &ts); })))
      return rr;
    a = ew_args(W, st);
    a.v[0] = X; a.v[1] = R; a.v[2] = PH; a.v[3] = S; a.v[4] = T; a.v[5] = RT; a.v[6] = SH;
    set_fd(W, a, mp::EPI_GP_CONV, {{1, mp::S_Q}, {2, mp::S_RHO_NEXT}}, hist);
    return timed(W, PROF_UPD, vec_bytes(W, 9), [&] { return launch_ew(L, EW_STAB_XR, a, W.ws); });
  };
  if ((r = run_iterations(W, o, iteration))) return r;
  return finish_solve(W, info, st);
}

// BiCG with the ILU(0) preconditioner K (Fig. 5 left): w = K^{-1} r, w~ = K^{-T} r~,
// rho = (r~, w) (zero: breakdown), beta = rho / rho_old, p = w + beta p, p~ = w~ + beta p~
// (first iteration: p = w, p~ = w~), z = A p with sigma = (p~, z), z~ = A^T p~, alpha = rho /
// sigma, x += alpha p, r -= alpha z, r~ -= alpha z~, (*) on r.
// Work vectors: 0 r, 1 rt, 2 z, 3 p, 4 pt, 5 zt, 6 w, 7 wt
int bicg_ilu0_impl(const mp_csr* A, const mp_plan* plan, const mp_ilu* K, const mp_vec* b, mp_vec* x,
                   const mp_solve_opts* o, mp_solve_info* info, hipStream_t user) {
  int r = check_solve_args(A, b, x, o, info);
  if (r) return r;
  if (o->transpose) return fail(MPS_ENOTSUP, "the preconditioned solve takes A, not its transpose");
  if ((r = check_ilu(K, A))) return r;
  DeviceCtx* ctx;
  if ((r = get_ctx(&ctx))) return r;
  OwnedPlan own;
  if (!plan) {
    if ((r = plan_build(A, user, &own.p))) return r;
    plan = own.p;
  } else if ((r = check_plan(plan, A))) {
    return r;
  }
  const int L = limbs_of(A->prec);
  Work W;
  if ((r = work_alloc(W, L, A->row_dim, 8, user))) return r;
  Op op, opT;
  make_ops(A, plan, 0, &op, &opT);
  uint32_t* st = ctx->status;
  if ((r = solve_setup(W, op, b, x, o, st))) return r;
  if ((r = clear_vectors(W, 2, 8, st))) return r;
  if ((r = prof_init(W, o->profile))) return r;
  const mp::VecRef R = W.vec(0), RT = W.vec(1), Z = W.vec(2), P = W.vec(3), PT = W.vec(4), ZT = W.vec(5),
                   Wv = W.vec(6), WT = W.vec(7);
  const mp::VecRef X = ref(*x);
  mp::VecRef hist{nullptr, nullptr, 0};
  if (o->res_hist && o->res_hist->len > 0) hist = ref(*o->res_hist);
  const double sp_bytes = spmv_bytes(A, L), dot1 = vec_bytes(W, 1);
  auto iteration = [&]() -> int {
    int rr;
    if ((rr = ilu_apply(K, W.desc(0), W.desc(6), o->mode, st, W.ctl, W.ws))) return rr;
    if ((rr = ilu_apply_t(K, W.desc(1), W.desc(7), o->mode, st, W.ctl, W.ws))) return rr;
    mp::DotArgs d = dot_args(W, st, mp::EPI_PRHO);
    d.o.nd = 1;
    d.x[0] = RT;
    d.y[0] = Wv;
    d.o.out[0] = mp::slot_ref(W.S, mp::S_RHO_NEXT);
    d.o.sslot[0] = mp::S_RHO_NEXT;
    d.o.slot[0] = 3;
    if ((rr = launch_dot(L, d, W.ws))) return rr;
    mp::VecArgs a = ew_args(W, st);
    a.v[0] = P; a.v[1] = PT; a.v[2] = Wv; a.v[3] = WT;
    if ((rr = timed(W, PROF_DIR, vec_bytes(W, 6), [&] { return launch_ew(L, EW_BICG_DIR, a, W.ws); })))
      return rr;
    const SpmvFuse sig = fuse_of(W, mp::EPI_NONE, {{PT, 0, mp::S_SIGMA}});
    if ((rr = timed(W, PROF_SPMV_DOT, sp_bytes + dot1, [&] { return apply(W, op, o->mode, P, Z, st, true, &sig); })))
      return rr;
    if ((rr = timed(W, PROF_SPMV, sp_bytes, [&] { return apply(W, opT, o->mode, PT, ZT, st, true); })))
      return rr;
    a = ew_args(W, st);
    a.v[0] = X; a.v[1] = R; a.v[2] = RT; a.v[3] = P; a.v[4] = Z; a.v[5] = ZT;
    // the update also forms (r~, r) in its second slot; this solve's rho comes from K^{-1} r
    set_fd(W, a, mp::EPI_CONV, {{1, mp::S_Q}, {2, mp::S_RHO_NEXT}}, hist);
    return timed(W, PROF_UPD, vec_bytes(W, 9), [&] { return launch_ew(L, EW_BICG_UPDATE, a, W.ws); });
  };
  if ((r = run_iterations(W, o, iteration))) return r;
  return finish_solve(W, info, st);
}

// BiCG, GPBiCG, CGS and BiCGSTAB at the wide precisions (2048, 4096, 8192 bits: the top of the
// paper's sweep, Sec. 4.1, Tables 1 and 2), driven from the host over the wide path's kernels
// (wide.hip).
enum WideMethod { WM_BICG, WM_GPBICG, WM_CGS, WM_BICGSTAB };
int wide_solve_impl(WideMethod m, const mp_csr* A, const mp_plan* plan, const mp_vec* b, mp_vec* x,
                    const mp_solve_opts* o, mp_solve_info* info, hipStream_t user) {
  int r = check_csr(A, 0, true);
  if (r) return r;
  if (A->row_dim != A->col_dim) return fail(MPS_EINVAL, "A must be square");
  if (!o || !info) return fail(MPS_EINVAL, "null opts/info");
  if (o->mode != MP_SEQ && o->mode != MP_EXACT) return fail(MPS_EINVAL, "mode must be MP_SEQ or MP_EXACT");
  if (o->maxit < 0 || o->maxit > INT32_MAX) return fail(MPS_EINVAL, "maxit out of range");
  if ((r = check_vec(b, A->row_dim, "b"))) return r;
  if ((r = check_vec(x, A->row_dim, "x"))) return r;
  const int L = wide_limbs_of(A->prec);
  if (vec_overlap(b, x, L)) return fail(MPS_EINVAL, "x overlaps b");
  if (o->res_hist && o->res_hist->len > 0 && (!o->res_hist->limb || !o->res_hist->hdr))
    return fail(MPS_EINVAL, "res_hist: null pointer");
  DeviceCtx* ctx;
  if ((r = get_ctx(&ctx))) return r;
  OwnedPlan own;
  if (plan) {
    if ((r = check_plan(plan, A))) return r;
  } else if (m == WM_BICG || o->transpose) {  // A^T is needed: build the transpose
    if ((r = plan_build(A, user, &own.p))) return r;
    plan = own.p;
  }
  const WideOp a{A->row_dim, A->row_ptr, A->col_idx, A->val};
  WideOp t = a;
  if (plan)
    t = WideOp{A->col_dim, plan->t_row_ptr, plan->t_col_idx, mp_vec{plan->t_limb, plan->t_hdr, plan->nnz, plan->nnz}};
  const WideOp& op = o->transpose ? t : a;
  switch (m) {
    case WM_BICG: return wide_bicg(L, op, o->transpose ? a : t, b, x, o, info, ctx->status, user);
    case WM_GPBICG: return wide_gpbicg(L, op, b, x, o, info, ctx->status, user);
    case WM_CGS: return wide_cgs(L, op, b, x, o, info, ctx->status, user);
    default: return wide_bicgstab(L, op, b, x, o, info, ctx->status, user);
  }
}

// ---- batched GPBiCG --------------------------------------------------------------------
// nsys systems, nrhs right-hand sides each: nsys * nrhs independent solves ("pairs", pair
// s * nrhs + k) advanced together.  The systems are concatenated into one block-diagonal CSR
// matrix whose diagonal blocks are padded to whole tiles with empty rows; vectors hold nrhs
// segments of rstride = sum of padded sizes, and pair (s, k) owns the tiles of system s in
// segment k.  Padding elements stay +0 (every update maps zeros to zeros and inner products skip
// zero products), so each pair computes exactly what a solve of its own system computes.

namespace {

int64_t padded_rows(int64_t n) {
  return std::max<int64_t>(mp::kTile, (n + mp::kTile - 1) / mp::kTile * mp::kTile);
}

int check_batched_args(int nsys, const mp_csr* A, int nrhs, const mp_vec* b, const mp_vec* x,
                       const mp_solve_opts* o, const mp_solve_info* info) {
  if (nsys <= 0 || nrhs <= 0) return fail(MPS_EINVAL, "nsys and nrhs must be positive");
  if (!A || !b || !x || !o || !info) return fail(MPS_EINVAL, "null argument");
  if (o->transpose) return fail(MPS_ENOTSUP, "batched solves take A, not its transpose");
  if (o->res_hist && o->res_hist->len > 0) return fail(MPS_ENOTSUP, "batched solves keep no residual history");
  if (o->profile) return fail(MPS_ENOTSUP, "batched solves take no profile");
  if (o->mode != MP_SEQ && o->mode != MP_EXACT) return fail(MPS_EINVAL, "mode must be MP_SEQ or MP_EXACT");
  if (o->maxit < 0 || o->maxit > INT32_MAX) return fail(MPS_EINVAL, "maxit out of range");
  int r;
  for (int s = 0; s < nsys; ++s) {
    if ((r = check_csr(&A[s], 0))) {
      const std::string m = mp_last_error();
      return fail(r, "system %d: %s", s, m.c_str());
    }
    if (A[s].row_dim != A[s].col_dim) return fail(MPS_EINVAL, "system %d is not square", s);
    if (A[s].prec != A[0].prec) return fail(MPS_EINVAL, "system %d: precisions differ", s);
    const int L = limbs_of(A[s].prec);
    for (int k = 0; k < nrhs; ++k) {
      const int64_t i = (int64_t)s * nrhs + k;
      if ((r = check_vec(&b[i], A[s].row_dim, "b")) || (r = check_vec(&x[i], A[s].row_dim, "x"))) {
        const std::string m = mp_last_error();
        return fail(r, "pair %lld: %s", (long long)i, m.c_str());
      }
      if (vec_overlap(&b[i], &x[i], L)) return fail(MPS_EINVAL, "pair %lld: x overlaps b", (long long)i);
    }
  }
  return MPS_OK;
}

// Concatenated block-diagonal matrix (device arrays owned here).
struct BlockDiag {
  int32_t* row_ptr = nullptr;
  int32_t* col_idx = nullptr;
  uint32_t* limb = nullptr;
  int32_t* hdr = nullptr;
  int64_t rows = 0, nnz = 0;
  ~BlockDiag() {
    hipFree(row_ptr);
    hipFree(col_idx);
    hipFree(limb);
    hipFree(hdr);
  }
};

int build_block_diag(int nsys, const mp_csr* A, int L, const std::vector<int64_t>& row_off,
                     BlockDiag& M, hipStream_t s) {
  std::vector<int64_t> nnz_off(nsys + 1, 0);
  for (int k = 0; k < nsys; ++k) nnz_off[k + 1] = nnz_off[k] + A[k].nnz;
  M.rows = row_off[nsys];
  M.nnz = nnz_off[nsys];
  if (M.nnz > INT32_MAX || M.rows > INT32_MAX)
    return fail(MPS_ENOTSUP, "the batch has more than 2^31 - 1 rows or stored entries");
  hipError_t e = hipMalloc((void**)&M.row_ptr, (size_t)(M.rows + 1) * 4);
  if (e == hipSuccess) e = hipMalloc((void**)&M.col_idx, std::max<size_t>(4, (size_t)M.nnz * 4));
  if (e == hipSuccess) e = hipMalloc((void**)&M.limb, std::max<size_t>(4, (size_t)M.nnz * L * 4));
  if (e == hipSuccess) e = hipMalloc((void**)&M.hdr, std::max<size_t>(4, (size_t)M.nnz * 4));
  if (e != hipSuccess) return fail(MPS_ENOMEM, "batched matrix: %s", hipGetErrorString(e));
  for (int k = 0; k < nsys; ++k) {
    const int64_t n = A[k].row_dim, np = row_off[k + 1] - row_off[k], nz = A[k].nnz;
    const bool last = k == nsys - 1;
    mp::BlockRowArgs ra{A[k].row_ptr, n, np + (last ? 1 : 0), (int32_t)nnz_off[k],
                        (int32_t)nz, M.row_ptr + row_off[k]};
    hipLaunchKernelGGL(mp::block_row_ptr_kernel, dim3((unsigned)std::min<int64_t>(4096, (np + 256) / 256)),
                       dim3(256), 0, s, ra);
    if (nz > 0) {
      mp::BlockColArgs ca{A[k].col_idx, nz, (int32_t)row_off[k], M.col_idx + nnz_off[k]};
      hipLaunchKernelGGL(mp::block_col_kernel, dim3((unsigned)std::min<int64_t>(4096, (nz + 255) / 256)),
                         dim3(256), 0, s, ca);
      e = hipMemcpy2DAsync(M.limb + nnz_off[k], (size_t)M.nnz * 4, A[k].val.limb,
                           (size_t)A[k].val.ld * 4, (size_t)nz * 4, (size_t)L, hipMemcpyDeviceToDevice, s);
      if (e == hipSuccess)
        e = hipMemcpyAsync(M.hdr + nnz_off[k], A[k].val.hdr, (size_t)nz * 4, hipMemcpyDeviceToDevice, s);
      if (e != hipSuccess) return hip_fail(e, "batched matrix copy");
    }
  }
  e = hipGetLastError();
  return e == hipSuccess ? MPS_OK : hip_fail(e, "batched matrix");
}

// gather (to_batch) the pairs' vectors into v, or scatter v back to them
int batch_copy(int L, bool to_batch, const mp::PairSeg* seg, const int32_t* pair_of_tile,
               const mp::VecRef& v, int64_t n, hipStream_t s) {
  const unsigned g = (unsigned)std::min<int64_t>(16384, (n + 255) / 256);
  const int gather = to_batch ? 1 : 0;
  switch (L) {
    case 4: hipLaunchKernelGGL(mp::batch_copy_kernel<4>, dim3(g), dim3(256), 0, s, seg, pair_of_tile, v, n, gather); break;
    case 8: hipLaunchKernelGGL(mp::batch_copy_kernel<8>, dim3(g), dim3(256), 0, s, seg, pair_of_tile, v, n, gather); break;
    case 16: hipLaunchKernelGGL(mp::batch_copy_kernel<16>, dim3(g), dim3(256), 0, s, seg, pair_of_tile, v, n, gather); break;
    case 32: hipLaunchKernelGGL(mp::batch_copy_kernel<32>, dim3(g), dim3(256), 0, s, seg, pair_of_tile, v, n, gather); break;
    default: return fail(MPS_EINVAL, "bad limb count");
  }
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? MPS_OK : hip_fail(e, "batch copy");
}

}  // namespace

int gpbicg_batched_impl(int nsys, const mp_csr* A, int nrhs, const mp_vec* b, mp_vec* x,
                        const mp_solve_opts* o, mp_solve_info* info, hipStream_t user) {
  int r = check_batched_args(nsys, A, nrhs, b, x, o, info);
  if (r) return r;
  DeviceCtx* ctx;
  if ((r = get_ctx(&ctx))) return r;
  const int L = limbs_of(A[0].prec);
  const int64_t npairs64 = (int64_t)nsys * nrhs;
  if (npairs64 > (1 << 20)) return fail(MPS_ENOTSUP, "more than 2^20 solves in one batch");
  // layout: padded row offsets, then the tile -> pair map of the nrhs segments
  std::vector<int64_t> row_off(nsys + 1, 0);
  for (int k = 0; k < nsys; ++k) row_off[k + 1] = row_off[k] + padded_rows(A[k].row_dim);
  const int64_t rstride = row_off[nsys];
  const int64_t n = rstride * nrhs;
  const int64_t ntiles = n / mp::kTile;
  if (ntiles > INT32_MAX / 2) return fail(MPS_ENOTSUP, "batch too large");
  std::vector<int32_t> pot((size_t)ntiles), top((size_t)npairs64), ftp((size_t)npairs64);
  std::vector<mp::PairSeg> seg_b((size_t)npairs64), seg_x((size_t)npairs64);
  for (int k = 0; k < nrhs; ++k)
    for (int sy = 0; sy < nsys; ++sy) {
      const int32_t pair = sy * nrhs + k;
      const int64_t off = (int64_t)k * rstride + row_off[sy];
      const int64_t nt = (row_off[sy + 1] - row_off[sy]) / mp::kTile;
      for (int64_t t = 0; t < nt; ++t) pot[(size_t)(off / mp::kTile + t)] = pair;
      top[pair] = (int32_t)nt;
      ftp[pair] = (int32_t)(off / mp::kTile);
      seg_b[pair] = mp::PairSeg{b[pair].limb, b[pair].hdr, b[pair].ld, A[sy].row_dim, off};
      seg_x[pair] = mp::PairSeg{x[pair].limb, x[pair].hdr, x[pair].ld, A[sy].row_dim, off};
    }
  Work W;
  W.npairs = (int)npairs64;
  W.nrhs = nrhs;
  W.rstride = rstride;
  W.ring_log2 = kBatchRingLog2;
  W.reps = kBatchReps;
  W.ngroups = kBatchGroups;
  mp::PairSeg* d_seg = nullptr;
  hipError_t e = hipMalloc((void**)&W.pair_of_tile, pot.size() * 4);
  if (e == hipSuccess) e = hipMalloc((void**)&W.tiles_of_pair, top.size() * 4);
  if (e == hipSuccess) e = hipMalloc((void**)&W.first_tile, ftp.size() * 4);
  if (e == hipSuccess) e = hipMalloc((void**)&d_seg, 2 * seg_b.size() * sizeof(mp::PairSeg));
  struct SegFree {
    mp::PairSeg* p;
    ~SegFree() { hipFree(p); }
  } seg_free{d_seg};
  if (e != hipSuccess) return fail(MPS_ENOMEM, "batch maps: %s", hipGetErrorString(e));
  // vectors 0..11 as in GPBiCG, 12 = x, 13 = b (concatenated)
  if ((r = work_alloc(W, L, n, kGpVectors + 2, user))) return r;
  e = hipMemcpyAsync(W.pair_of_tile, pot.data(), pot.size() * 4, hipMemcpyHostToDevice, W.ws);
  if (e == hipSuccess) e = hipMemcpyAsync(W.tiles_of_pair, top.data(), top.size() * 4, hipMemcpyHostToDevice, W.ws);
  if (e == hipSuccess) e = hipMemcpyAsync(W.first_tile, ftp.data(), ftp.size() * 4, hipMemcpyHostToDevice, W.ws);
  if (e == hipSuccess)
    e = hipMemcpyAsync(d_seg, seg_b.data(), seg_b.size() * sizeof(mp::PairSeg), hipMemcpyHostToDevice, W.ws);
  if (e == hipSuccess)
    e = hipMemcpyAsync(d_seg + seg_b.size(), seg_x.data(), seg_x.size() * sizeof(mp::PairSeg),
                       hipMemcpyHostToDevice, W.ws);
  if (e == hipSuccess) e = hipStreamSynchronize(W.ws);  // the host tables go out of scope below
  if (e != hipSuccess) return hip_fail(e, "batch maps upload");
  BlockDiag M;
  if ((r = build_block_diag(nsys, A, L, row_off, M, W.ws))) return r;
  Op op{M.rows, M.row_ptr, M.col_idx, mp_vec{M.limb, M.hdr, M.nnz, M.nnz}, {}};
  // SEQ: 64 rows per block in the pipelined kernel (one wavefront's chains advance while three
  // form the next products), rows in order; EXACT: rows per block by shape
  op.var[MP_SEQ].rpw = 64;
  op.var[MP_SEQ].pipe = true;
  uint32_t* st = ctx->status;
  const mp::VecRef X = W.vec(kGpVectors), B = W.vec(kGpVectors + 1);
  if ((r = batch_copy(L, true, d_seg, W.pair_of_tile, B, n, W.ws))) return r;
  if (o->use_x0 && (r = batch_copy(L, true, d_seg + seg_b.size(), W.pair_of_tile, X, n, W.ws))) return r;
  mp_vec bd = W.desc(kGpVectors + 1), xd = W.desc(kGpVectors);
  if ((r = solve_setup(W, op, &bd, &xd, o, st))) return r;
  if ((r = gp_clear(W, st))) return r;
  const mp::VecRef nohist{nullptr, nullptr, 0};
  auto iteration = [&]() -> int { return gp_iteration(W, op, o->mode, X, nohist, st, 0.0); };
  if ((r = run_iterations(W, o, iteration))) return r;
  if ((r = batch_copy(L, false, d_seg + seg_b.size(), W.pair_of_tile, X, n, W.ws))) return r;
  // per-pair outcomes
  std::vector<uint32_t> sl((size_t)L * W.S.ld);
  std::vector<int32_t> sh((size_t)W.S.ld);
  e = hipMemcpyAsync(W.h_ctl, W.ctl, sizeof(mp::Ctl) * W.npairs, hipMemcpyDeviceToHost, W.ws);
  if (e == hipSuccess) e = hipMemcpyAsync(sl.data(), W.S.limb, sl.size() * 4, hipMemcpyDeviceToHost, W.ws);
  if (e == hipSuccess) e = hipMemcpyAsync(sh.data(), W.S.hdr, sh.size() * 4, hipMemcpyDeviceToHost, W.ws);
  if (e == hipSuccess) e = hipStreamSynchronize(W.ws);
  if (e != hipSuccess) return hip_fail(e, "batched result readback");
  uint32_t fl = 0;
  for (int i = 0; i < W.npairs; ++i) {
    const mp::Ctl& c = W.h_ctl[i];
    info[i].status = c.status;
    info[i].iters = c.iters;
    const int64_t base = (int64_t)i * mp::kNumScalars;
    const double q0 = mp_to_double(sl.data() + base + mp::S_Q0, sh[base + mp::S_Q0], L, W.S.ld);
    const double q = c.iters > 0 ? mp_to_double(sl.data() + base + mp::S_Q, sh[base + mp::S_Q], L, W.S.ld) : q0;
    info[i].final_rel_res = q0 > 0 ? std::sqrt(q / q0) : 0.0;
    fl |= c.flags;
  }
  if (fl & mp::kStRange) return fail(MPS_ERANGE, "a result exponent left the range during a solve");
  if (fl & mp::kStWindow) return fail(MPS_ENOTSUP, "an exact accumulation was wider than supported");
  return MPS_OK;
}

}  // namespace mpapi

using namespace mpapi;

extern "C" {

int bicg(const mp_csr* A, const mp_plan* plan, const mp_vec* b, mp_vec* x,
         const mp_solve_opts* opts, mp_solve_info* info, void* stream) {
  clear_error();
  if (A && wide_limbs_of(A->prec)) return wide_solve_impl(WM_BICG, A, plan, b, x, opts, info, (hipStream_t)stream);
  return bicg_impl(A, plan, b, x, opts, info, (hipStream_t)stream);
}

int gpbicg(const mp_csr* A, const mp_plan* plan, const mp_vec* b, mp_vec* x,
           const mp_solve_opts* opts, mp_solve_info* info, void* stream) {
  clear_error();
  if (A && wide_limbs_of(A->prec)) return wide_solve_impl(WM_GPBICG, A, plan, b, x, opts, info, (hipStream_t)stream);
  return gpbicg_impl(A, plan, b, x, opts, info, (hipStream_t)stream);
}

int cgs(const mp_csr* A, const mp_plan* plan, const mp_vec* b, mp_vec* x,
        const mp_solve_opts* opts, mp_solve_info* info, void* stream) {
  clear_error();
  if (A && wide_limbs_of(A->prec)) return wide_solve_impl(WM_CGS, A, plan, b, x, opts, info, (hipStream_t)stream);
  return cgs_impl(A, plan, b, x, opts, info, (hipStream_t)stream);
}

int bicgstab(const mp_csr* A, const mp_plan* plan, const mp_vec* b, mp_vec* x,
             const mp_solve_opts* opts, mp_solve_info* info, void* stream) {
  clear_error();
  if (A && wide_limbs_of(A->prec)) return wide_solve_impl(WM_BICGSTAB, A, plan, b, x, opts, info, (hipStream_t)stream);
  return bicgstab_impl(A, plan, b, x, opts, info, (hipStream_t)stream);
}

int bicgstab_ilu0(const mp_csr* A, const mp_ilu* ilu, const mp_vec* b, mp_vec* x,
                  const mp_solve_opts* opts, mp_solve_info* info, void* stream) {
  clear_error();
  return bicgstab_ilu0_impl(A, ilu, b, x, opts, info, (hipStream_t)stream);
}

int bicg_ilu0(const mp_csr* A, const mp_plan* plan, const mp_ilu* ilu, const mp_vec* b, mp_vec* x,
              const mp_solve_opts* opts, mp_solve_info* info, void* stream) {
  clear_error();
  return bicg_ilu0_impl(A, plan, ilu, b, x, opts, info, (hipStream_t)stream);
}

int gpbicg_batched(int nsys, const mp_csr* A, int nrhs, const mp_vec* b, mp_vec* x,
                   const mp_solve_opts* opts, mp_solve_info* info, void* stream) {
  clear_error();
  return gpbicg_batched_impl(nsys, A, nrhs, b, x, opts, info, (hipStream_t)stream);
}

int mp_const_decimal(int64_t m, int64_t e10, int prec, mp_vec* out, void* stream) {
  clear_error();
  const int WL = wide_limbs_of(prec);
  const int L = WL ? WL : limbs_of(prec);
  if (!L) return fail(MPS_EINVAL, "precision %d not in {128, 256, 512, 1024, 2048, 4096, 8192}", prec);
  int r = check_vec(out, 1, "out");
  if (r) return r;
  std::vector<uint32_t> m_(L);
  int32_t h;
  if (!decimal_to_mp(m, e10, L, m_.data(), &h)) return fail(MPS_EINVAL, "constant out of range");
  if (!WL) return set_scalar(L, ref(*out), m_.data(), h, (hipStream_t)stream);
  // wide: the limbs one plane at a time (a synchronous upload of L + 1 words)
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = hipSuccess;
  for (int k = 0; k < L && e == hipSuccess; ++k)
    e = hipMemcpyAsync(out->limb + (int64_t)k * out->ld, &m_[k], 4, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(out->hdr, &h, 4, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  return e == hipSuccess ? MPS_OK : hip_fail(e, "constant upload");
}

}  // extern "C"
