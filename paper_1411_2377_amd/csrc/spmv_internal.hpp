// SpMV kernel dispatch shared by the plain product launch and the solver's fused launch.
#pragma once
#include <hip/hip_runtime.h>

#include "api_internal.hpp"
#include "spmv_kernels.hpp"

namespace mpapi {

// Inner products the solver takes of an SpMV's output y: (y, part[k]) for k < nd
// (part[k].hdr == nullptr: y itself) into slot[k]; the launch's last block rounds them into
// out[k] and runs the driver epilogue `epi`.
struct SpmvFuse {
  int nd = 0;
  mp::VecRef part[3] = {};
  int slot[3] = {0, 0, 0};
  mp::VecRef out[3] = {};
  int sslot[3] = {-1, -1, -1};  // the scalar slot of out[k], or -1
  int epi = 0;
  mp::VecRef hist = {};
  mp::DotWork dots = {};
  mp::Scalars S = {};
  mp::Ctl* ctl = nullptr;
  const int32_t* tiles_of_pair = nullptr;
  const int32_t* first_tile = nullptr;
  int32_t* ndone = nullptr;
};

template <int L, int RPW, bool FUSE>
void launch_spmv_rpw(const mp::SpmvArgs& a, int mode, hipStream_t s) {
  const unsigned grid = (unsigned)(a.long_blocks + (a.n_rows - a.n_long + RPW - 1) / RPW) * (unsigned)a.nrhs;
  if (mode == MP_SEQ && (a.rows || a.pipe)) {  // the four-wave pipelined kernel
    bool groups = false;  // the lane-group instantiation (its LDS buffers) only where it is used
    if constexpr (!FUSE && L <= 16) groups = a.long_blocks > 0 && !a.window;
    if constexpr (!FUSE && L <= 16) {
      if (groups) {
        MPS_LAUNCH_MAIN(!a.x_rec, true, (mp::spmv_seq_sorted_kernel<L, RPW, FUSE, true>), dim3(grid), dim3(256), 0, s, a);
        return;
      }
    }
    MPS_LAUNCH_MAIN(!a.x_rec, true, (mp::spmv_seq_sorted_kernel<L, RPW, FUSE, false>), dim3(grid), dim3(256), 0, s, a);
  } else if (mode == MP_SEQ)
    MPS_LAUNCH_MAIN(!a.x_rec, true, (mp::spmv_seq_kernel<L, RPW, FUSE>), dim3(grid), dim3(64), 0, s, a);
  else
    MPS_LAUNCH_MAIN(!a.x_rec, true, (mp::spmv_exact_kernel<L, RPW, FUSE>), dim3(grid), dim3(64), 0, s, a);
}

template <int L, bool FUSE>
void launch_spmv(const mp::SpmvArgs& a, int mode, int rpw, hipStream_t s) {
  switch (rpw) {
    case 16: launch_spmv_rpw<L, 16, FUSE>(a, mode, s); break;
    case 32: launch_spmv_rpw<L, 32, FUSE>(a, mode, s); break;
    default: launch_spmv_rpw<L, 64, FUSE>(a, mode, s); break;
  }
}

// The kernels with fused inner products (instantiated in their own translation unit).
void launch_spmv_fused(int L, const mp::SpmvArgs& a, int mode, int rpw, hipStream_t s);

}  // namespace mpapi
