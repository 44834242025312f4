"""Python entry points with the C ABI's names (argument marshalling only)."""
import ctypes

import torch

from . import _lib
from ._lib import MP_EXACT, MP_SEQ, check  # noqa: F401
from .mparray import CSRMatrix, MPArray  # noqa: F401


def _stream(stream=None):
    if stream is None:
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def mp_last_error():
    return _lib.last_error()


def mp_validate_csr(A, check_device_data=False):
    d = A.desc() if hasattr(A, "desc") else A
    return _lib.LIB.mp_validate_csr(ctypes.byref(d), int(bool(check_device_data)))


def mpspmv_csr(A, x, y=None, mode=MP_SEQ, stream=None):
    """y = A x; allocates y when not given.  Returns y."""
    if y is None:
        y = MPArray.empty(A.n_rows, A.p, device=x.device)
    a, xd, yd = A.desc(), x.desc(), y.desc()
    check(_lib.LIB.mpspmv_csr(ctypes.byref(a), ctypes.byref(xd), ctypes.byref(yd), int(mode),
                              _stream(stream)))
    return y


def mp_status(stream=None, raise_on_error=True):
    flags = ctypes.c_uint32(0)
    code = _lib.LIB.mp_status(_stream(stream), ctypes.byref(flags))
    if raise_on_error:
        check(code)
    return int(flags.value)
