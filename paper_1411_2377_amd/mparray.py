"""Device-resident MP arrays and CSR matrices (torch int32 storage, structure of arrays).

An MPArray of N numbers at p = 32 L bits is two torch tensors on the GPU:
  limbs  int32 [L, N]  (the bits of uint32 limb planes, plane k = limb k, k = 0 least significant)
  hdr    int32 [N]     (e << 1) | s, zeros have e = -2^30
PyTorch only provides the memory and the stream; all arithmetic is in libmpspmv.so.
"""
import numpy as np
import torch

from . import _lib


class MPArray:
    def __init__(self, limbs, hdr, p):
        assert limbs.dtype == torch.int32 and hdr.dtype == torch.int32
        assert limbs.dim() == 2 and limbs.shape[0] == p // 32 and limbs.shape[1] == hdr.shape[0]
        assert limbs.is_contiguous() and hdr.is_contiguous()
        self.limbs = limbs
        self.hdr = hdr
        self.p = int(p)

    @property
    def n(self):
        return int(self.hdr.shape[0])

    @property
    def device(self):
        return self.hdr.device

    @staticmethod
    def empty(n, p, device="cuda"):
        return MPArray(torch.empty((p // 32, n), dtype=torch.int32, device=device),
                       torch.empty(n, dtype=torch.int32, device=device), p)

    @staticmethod
    def zeros(n, p, device="cuda"):
        """+0 everywhere (header INT32_MIN)."""
        return MPArray(torch.zeros((p // 32, n), dtype=torch.int32, device=device),
                       torch.full((n,), -(1 << 31), dtype=torch.int32, device=device), p)

    @staticmethod
    def from_host(h, device="cuda"):
        """From a host container with .limbs (uint32 [L, N]), .hdr (int32 [N]) and .p."""
        limbs = torch.from_numpy(np.ascontiguousarray(h.limbs).view(np.int32)).to(device)
        hdr = torch.from_numpy(np.ascontiguousarray(h.hdr)).to(device)
        return MPArray(limbs.contiguous(), hdr.contiguous(), h.p)

    def to_numpy(self):
        """(limbs uint32 [L, N], hdr int32 [N]) on the host (synchronising copy)."""
        return (self.limbs.cpu().numpy().view(np.uint32).copy(), self.hdr.cpu().numpy().copy())

    def clone(self):
        return MPArray(self.limbs.clone(), self.hdr.clone(), self.p)

    def copy_(self, other):
        self.limbs.copy_(other.limbs)
        self.hdr.copy_(other.hdr)
        return self

    def slice(self, start, stop):
        """A view of elements [start, stop) (limb planes keep the parent's stride)."""
        return MPArrayView(self, start, stop)

    def desc(self):
        v = _lib.MpVec()
        v.limb = self.limbs.data_ptr()
        v.hdr = self.hdr.data_ptr()
        v.len = self.n
        v.ld = int(self.limbs.stride(0)) if self.n else 0
        return v


class MPArrayView:
    """Elements [start, stop) of an MPArray, as a descriptor with the parent's plane stride."""

    def __init__(self, parent, start, stop):
        self.parent = parent
        self.start = int(start)
        self.stop = int(stop)
        self.p = parent.p

    @property
    def n(self):
        return self.stop - self.start

    def desc(self):
        v = _lib.MpVec()
        v.limb = self.parent.limbs.data_ptr() + 4 * self.start
        v.hdr = self.parent.hdr.data_ptr() + 4 * self.start
        v.len = self.n
        v.ld = int(self.parent.limbs.stride(0))
        return v


class CSRMatrix:
    """CSR matrix with MP values on the device: row_ptr, col_idx int32; vals MPArray."""

    def __init__(self, n_rows, n_cols, row_ptr, col_idx, vals):
        assert row_ptr.dtype == torch.int32 and col_idx.dtype == torch.int32
        self.n_rows = int(n_rows)
        self.n_cols = int(n_cols)
        self.row_ptr = row_ptr.contiguous()
        self.col_idx = col_idx.contiguous()
        self.vals = vals
        self.p = vals.p

    @property
    def nnz(self):
        return int(self.col_idx.shape[0])

    @staticmethod
    def from_host(h, device="cuda"):
        """From a host container with n_rows, n_cols, row_ptr, col_idx, vals."""
        return CSRMatrix(h.n_rows, h.n_cols,
                         torch.from_numpy(np.ascontiguousarray(h.row_ptr, np.int32)).to(device),
                         torch.from_numpy(np.ascontiguousarray(h.col_idx, np.int32)).to(device),
                         MPArray.from_host(h.vals, device))

    def desc(self):
        a = _lib.MpCsr()
        a.row_dim = self.n_rows
        a.col_dim = self.n_cols
        a.nnz = self.nnz
        a.prec = self.p
        a.row_ptr = self.row_ptr.data_ptr()
        a.col_idx = self.col_idx.data_ptr() if self.nnz else 0
        a.val = self.vals.desc()
        return a
