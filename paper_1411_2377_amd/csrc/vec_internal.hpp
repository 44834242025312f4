// Launch helpers for the vector, inner-product and driver-step kernels.
#pragma once
#include <hip/hip_runtime.h>

#include "../../include/mpspmv.h"
#include "api_internal.hpp"
#include "solver_kernels.hpp"

namespace mpapi {

enum EwKind {
  EW_AXPY, EW_COPY, EW_ZERO, EW_SUB, EW_BICG_DIR, EW_BICG_UPDATE, EW_GP_DIR, EW_GP_TSY,
  EW_CGS_DIR, EW_CGS_QUX, EW_CGS_R, EW_STAB_DIR, EW_STAB_S, EW_STAB_XR
};

mp::VecRef ref(const mp_vec& v);
mp::DotWork dot_work(int32_t* anchor, int64_t* win, uint32_t* ticket, int nslots, int ring_log2,
                     int reps, int ngroups);
unsigned ew_grid(int64_t n);
int launch_dot(int L, const mp::DotArgs& a, hipStream_t s);
int launch_ew(int L, EwKind kind, const mp::VecArgs& a, hipStream_t s);
int launch_gp_update(int L, const mp::GpUpdArgs& a, hipStream_t s);
// step prologues of a batch: one wavefront per solve
int launch_prologue(int L, const mp::ProArgs& a, int npairs, hipStream_t s);
// driver epilogues of a batch: one wavefront per solve
int launch_epilogue(int L, const mp::EpiArgs& a, int npairs, hipStream_t s);
// write the constant to out and to count - 1 further places `step` elements apart
int set_scalar(int L, const mp::VecRef& out, const uint32_t* m, int32_t hdr, hipStream_t s,
               int64_t count = 1, int64_t step = 0);

}  // namespace mpapi
