// SpMV kernels that end with the solver's inner products of their output (the variants the
// Krylov drivers launch), compiled apart from the plain ones.
#include "spmv_internal.hpp"

namespace mpapi {

void launch_spmv_fused(int L, const mp::SpmvArgs& a, int mode, int rpw, hipStream_t s) {
  switch (L) {
    case 4: launch_spmv<4, true>(a, mode, rpw, s); break;
    case 8: launch_spmv<8, true>(a, mode, rpw, s); break;
    case 16: launch_spmv<16, true>(a, mode, rpw, s); break;
    case 32: launch_spmv<32, true>(a, mode, rpw, s); break;
    default: break;
  }
}

}  // namespace mpapi
