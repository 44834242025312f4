// Internal helpers shared by the C-ABI translation units of the library.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/mpspmv.h"

namespace mpapi {

struct DeviceCtx {
  int device = 0;
  uint32_t* status = nullptr;  // device status word (MP_ST_* bits)
  // workspace of the stand-alone inner product entry point
  int32_t* dot_part = nullptr;
  uint32_t* dot_ticket = nullptr;
  uint32_t* scal_limb = nullptr;  // [16][32] scalar slots
  int32_t* scal_hdr = nullptr;    // [32]
};

// bytes of the inner-product partial-record workspace (largest precision)
size_t dot_workspace_bytes();

int fail(int code, const char* fmt, ...);
void clear_error();
int hip_fail(hipError_t e, const char* what);
int get_ctx(DeviceCtx** out);
int limbs_of(int prec);
int check_vec(const mp_vec* v, int64_t want_len, const char* name);
bool vec_overlap(const mp_vec* a, const mp_vec* b, int L);
int check_csr(const mp_csr* A, int check_device_data);
int spmv_launch(int L, int64_t n_rows, const int32_t* row_ptr, const int32_t* col_idx,
                const mp_vec& val, const mp_vec& x, const mp_vec& y, int mode, uint32_t* status,
                const int32_t* done, hipStream_t s);

}  // namespace mpapi
