// Kernels that assemble a batch of independent solves: the block-diagonal concatenation of the
// systems' CSR matrices, and the gather / scatter of per-solve vectors into / out of the
// concatenated layout (each solve's segment is a whole number of kTile tiles; the elements past
// a system's size are +0).
#pragma once
#include "mp_core.hpp"
#include "solver_kernels.hpp"

namespace mp {

// One solve's vector: the caller's array and the solve's place in the concatenated vector.
struct PairSeg {
  uint32_t* limb;
  int32_t* hdr;
  int64_t ld;
  int64_t n;    // elements of the system
  int64_t off;  // first element of the segment in the concatenated vector
};

// out[i] = nnz_off + row_ptr[min(i, n)] for i < count (rows past n are empty padding rows).
struct BlockRowArgs {
  const int32_t* row_ptr;
  int64_t n;
  int64_t count;
  int32_t nnz_off;
  int32_t nnz;
  int32_t* out;
};

static __global__ void __launch_bounds__(256) block_row_ptr_kernel(BlockRowArgs A) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < A.count;
       i += (int64_t)gridDim.x * blockDim.x)
    A.out[i] = A.nnz_off + (i <= A.n ? A.row_ptr[i] : A.nnz);
}

// out[k] = col_idx[k] + col_off (the system's first column in the concatenated matrix).
struct BlockColArgs {
  const int32_t* col_idx;
  int64_t nnz;
  int32_t col_off;
  int32_t* out;
};

static __global__ void __launch_bounds__(256) block_col_kernel(BlockColArgs A) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < A.nnz;
       k += (int64_t)gridDim.x * blockDim.x)
    A.out[k] = A.col_idx[k] + A.col_off;
}

// gather: v[i] = the solve's element (or +0 past the system's size);
// scatter: the solve's element = v[i] for the elements inside the system.
template <int L>
__global__ void __launch_bounds__(256) batch_copy_kernel(const PairSeg* seg, const int32_t* pair_of_tile,
                                                         VecRef v, int64_t n, int gather) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const PairSeg g = seg[pair_of_tile[i / kTile]];
    const int64_t j = i - g.off;
    if (gather) {
      Num<L> x;
      if (j < g.n) load<L>(x, g.limb, g.hdr, g.ld, j);
      else set_zero(x, 0);
      store<L>(x, v.limb, v.hdr, v.ld, i);
    } else if (j < g.n) {
      Num<L> x;
      load<L>(x, v.limb, v.hdr, v.ld, i);
      store<L>(x, g.limb, g.hdr, g.ld, j);
    }
  }
}

}  // namespace mp
