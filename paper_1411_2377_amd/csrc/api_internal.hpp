// Internal helpers shared by the C-ABI translation units of the library.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/mpspmv.h"

#include <hip/hip_ext.h>

namespace mpapi {

// Kernel timing: while set on the calling thread, the launch helpers attach these events to the
// kernels they launch (the first kernel of a call records `start` when it begins, the last one
// records `stop` when it ends), so their difference is the kernels' own execution time.
struct LaunchEvents {
  hipEvent_t start = nullptr, stop = nullptr;
};
extern thread_local LaunchEvents* g_launch_events;

// hipLaunchKernelGGL, or with the timing events attached (`first`/`last`: whether this launch
// starts / ends the timed call)
#define MPS_LAUNCH(first, last, KERNEL, GRID, BLOCK, SHMEM, STREAM, ...)                        \
  do {                                                                                        \
    if (::mpapi::g_launch_events)                                                             \
      hipExtLaunchKernelGGL(KERNEL, GRID, BLOCK, SHMEM, STREAM,                               \
                            (first) ? ::mpapi::g_launch_events->start : nullptr,              \
                            (last) ? ::mpapi::g_launch_events->stop : nullptr, 0, __VA_ARGS__); \
    else                                                                                      \
      hipLaunchKernelGGL(KERNEL, GRID, BLOCK, SHMEM, STREAM, __VA_ARGS__);                    \
  } while (0)

// Kernel timer (measurement only, mp_timer_* in the C ABI): while one is selected on the calling
// thread, the main kernel of each library call (the sparse product's kernel, not its x staging;
// the value-gradient kernel) is launched with its own pair of events from the timer's pool.
struct KernelTimer {
  int device = 0;
  int cap = 0, used = 0;
  hipEvent_t* ev = nullptr;  // [2 * cap]
};
extern thread_local KernelTimer* g_timer;
// the next event pair of the selected timer (false: no timer selected, or its pool is full)
inline bool timer_next(hipEvent_t* e0, hipEvent_t* e1) {
  KernelTimer* t = g_timer;
  if (!t || t->used >= t->cap) return false;
  *e0 = t->ev[2 * t->used];
  *e1 = t->ev[2 * t->used + 1];
  ++t->used;
  return true;
}

// A call's main kernel: timed by the selected kernel timer if there is one, else as MPS_LAUNCH.
#define MPS_LAUNCH_MAIN(first, last, KERNEL, GRID, BLOCK, SHMEM, STREAM, ...)                   \
  do {                                                                                        \
    hipEvent_t mps_t0_, mps_t1_;                                                              \
    if (::mpapi::timer_next(&mps_t0_, &mps_t1_))                                               \
      hipExtLaunchKernelGGL(KERNEL, GRID, BLOCK, SHMEM, STREAM, mps_t0_, mps_t1_, 0, __VA_ARGS__); \
    else                                                                                      \
      MPS_LAUNCH(first, last, KERNEL, GRID, BLOCK, SHMEM, STREAM, __VA_ARGS__);               \
  } while (0)

struct DeviceCtx {
  int device = 0;
  uint32_t* status = nullptr;  // device status word (MP_ST_* bits)
  // inner-product state of the stand-alone mp_dot (one slot)
  int32_t* dot_anchor = nullptr;
  int64_t* dot_win = nullptr;
  uint32_t* dot_ticket = nullptr;
  // global windows (and their locks) of EXACT rows wider than a block's LDS window
  int64_t* wide_win = nullptr;
  int32_t* wide_lock = nullptr;
};

struct SpmvFuse;  // spmv_internal.hpp

// Several right-hand sides of a block-diagonal batch in one product launch: x and y hold nrhs
// segments of rstride elements each; the solve owning a 512-element tile of y decides whether
// its blocks run (done flags) and which scalars and inner-product slots they use.
struct SpmvBatch {
  int nrhs = 1;
  int64_t rstride = 0;
  const int32_t* pair_of_tile = nullptr;
  const int32_t* done_base = nullptr;
  int64_t done_stride = 0;
};

// Inner-product state (see the exact inner products in solver_kernels.hpp): rings of 2^11 digits
// (exponent spans up to 32 (2048 - 2L - 2) bits), 8 replicas, tickets in 64 groups; a batch of
// solves keeps 256-digit rings, 8 replicas and 16 groups per solve.
constexpr int kDotRingLog2 = 11, kDotReps = 8, kDotGroups = 64;  // replicas: at most 8
constexpr int kBatchRingLog2 = 8, kBatchReps = 8, kBatchGroups = 16;

// Allocate and clear inner-product state: `nslots` slots (each `reps` rings of 2^ring_log2
// digits and 64 exponent bins) and the tickets of `nsolves` solves.
int dot_work_alloc(int nslots, int ring_log2, int reps, int ngroups, int32_t** anchor, int64_t** win,
                   uint32_t** ticket, hipStream_t s, int nsolves = 1);

int fail(int code, const char* fmt, ...);
void clear_error();
int hip_fail(hipError_t e, const char* what);
// RN_p(m 10^e10) into L limbs and a header (false: out of range)
bool decimal_to_mp(int64_t m, int64_t e10, int L, uint32_t* limbs, int32_t* hdr);
int get_ctx(DeviceCtx** out);
int limbs_of(int prec);
int check_vec(const mp_vec* v, int64_t want_len, const char* name);
bool vec_overlap(const mp_vec* a, const mp_vec* b, int L);
// wide_ok: the precisions of the wide path (2048, 4096, 8192) are accepted too
int check_csr(const mp_csr* A, int check_device_data, bool wide_ok = false);
// Kernel variant of one product: rows per block (0: by shape), staged x (x_rec: a buffer of
// x_len records, the launch first stages x into it), rows in a given order (nullptr: in order),
// and for SEQ the pipelined kernel (always with a row order).
struct SpmvVariant {
  int rpw = 0;
  uint32_t* x_rec = nullptr;
  int64_t x_len = 0;
  const int32_t* rows = nullptr;
  bool pipe = false;  // SEQ: the four-wavefront pipelined kernel also without a row order
  int64_t n_long = 0;  // SEQ with a row order: its first n_long rows are summed by lane groups
  int windows = 0;  // ... or by windowed chains: 1 one row per wavefront; 2 the same for the
                    // first n_win rows, four per wavefront for the others
  int64_t n_win = 0;
  bool no_wide = false;  // EXACT: no global windows (rows wider than the LDS window raise kStWindow)
};
int spmv_launch(int L, int64_t n_rows, const int32_t* row_ptr, const int32_t* col_idx,
                const mp_vec& val, const mp_vec& x, const mp_vec& y, int mode, uint32_t* status,
                const int32_t* done, hipStream_t s, const SpmvFuse* fuse = nullptr,
                const SpmvBatch* batch = nullptr, const SpmvVariant* var = nullptr,
                int32_t dense_cols = 0);
// rows per block of the SpMV kernels: 16, 32 or 64 (0 or anything else: chosen from the shape)
int default_rows_per_block(int64_t n_rows, int64_t nnz);
bool valid_rows_per_block(int rpw);

}  // namespace mpapi
