"""ctypes binding of libmpspmv.so (the C ABI in include/mpspmv.h).

Argument marshalling only: every computation runs in the library's HIP kernels.  Importing this
module fails loudly when the library has not been built; there is no fallback path.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmpspmv.so")

MPS_OK = 0
MPS_EINVAL = -1
MPS_ENOMEM = -2
MPS_EHIP = -3
MPS_ERANGE = -4
MPS_ENOTSUP = -5

MP_SEQ = 0
MP_EXACT = 1

MP_ST_RANGE = 1
MP_ST_WINDOW = 2
MP_ST_DIVZERO = 4

MP_CONVERGED = 0
MP_NC = 1
MP_BREAKDOWN_RHO = 2
MP_BREAKDOWN_SIGMA = 3
MP_BREAKDOWN_ZETA = 4
MP_BREAKDOWN_TAU = 5


class MpVec(ctypes.Structure):
    _fields_ = [("limb", ctypes.c_void_p), ("hdr", ctypes.c_void_p),
                ("len", ctypes.c_int64), ("ld", ctypes.c_int64)]


class MpCsr(ctypes.Structure):
    _fields_ = [("row_dim", ctypes.c_int64), ("col_dim", ctypes.c_int64),
                ("nnz", ctypes.c_int64), ("prec", ctypes.c_int32),
                ("row_ptr", ctypes.c_void_p), ("col_idx", ctypes.c_void_p),
                ("val", MpVec)]


class MpDense(ctypes.Structure):
    _fields_ = [("rows", ctypes.c_int64), ("cols", ctypes.c_int64), ("prec", ctypes.c_int32),
                ("val", MpVec)]


class MpSolveProfile(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int64 * 5), ("us", ctypes.c_double * 5),
                ("bytes", ctypes.c_double * 5)]


class MpSolveOpts(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("transpose", ctypes.c_int32),
                ("maxit", ctypes.c_int64),
                ("rtol_m", ctypes.c_int64), ("rtol_e10", ctypes.c_int64),
                ("atol_m", ctypes.c_int64), ("atol_e10", ctypes.c_int64),
                ("chunk", ctypes.c_int32), ("use_x0", ctypes.c_int32),
                ("res_hist", ctypes.POINTER(MpVec)),
                ("profile", ctypes.POINTER(MpSolveProfile))]


class MpSolveInfo(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iters", ctypes.c_int64),
                ("final_rel_res", ctypes.c_double)]


class MPError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("mpspmv error %d: %s" % (code, msg))
        self.code = code


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("libmpspmv.so is not built (run: python -m paper_1411_2377_amd.build)")
    lib = ctypes.CDLL(LIB_PATH)
    lib.mp_last_error.restype = ctypes.c_char_p
    lib.mp_last_error.argtypes = []
    return lib


LIB = _load()

# every symbol the C header declares, with its ctypes signature
SIGNATURES = {
    "mp_validate_csr": [ctypes.POINTER(MpCsr), ctypes.c_int],
    "mpspmv_csr": [ctypes.POINTER(MpCsr), ctypes.POINTER(MpVec), ctypes.POINTER(MpVec),
                   ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p],
    "mp_gemv": [ctypes.POINTER(MpDense), ctypes.POINTER(MpVec), ctypes.POINTER(MpVec), ctypes.c_int,
                ctypes.c_void_p],
    "mpspmv_csr_noalloc": [ctypes.POINTER(MpCsr), ctypes.POINTER(MpVec), ctypes.POINTER(MpVec),
                           ctypes.c_int, ctypes.c_void_p],
    "mp_plan_tune": [ctypes.c_void_p, ctypes.POINTER(MpCsr), ctypes.c_int, ctypes.c_void_p],
    "mp_plan_tune_x": [ctypes.c_void_p, ctypes.POINTER(MpCsr), ctypes.POINTER(MpVec), ctypes.POINTER(MpVec),
                       ctypes.c_int, ctypes.c_void_p],
    "mp_plan_tune_cached": [ctypes.c_void_p, ctypes.POINTER(MpCsr), ctypes.c_int, ctypes.c_char_p,
                            ctypes.POINTER(ctypes.c_int), ctypes.c_void_p],
    "mp_plan_set_variant": [ctypes.c_void_p, ctypes.POINTER(MpCsr), ctypes.c_int, ctypes.c_int,
                            ctypes.c_int, ctypes.c_int],
    "mp_plan_get_variant": [ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                            ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)],
    "mp_status": [ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint32)],
    "mp_plan_create": [ctypes.POINTER(MpCsr), ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)],
    "mp_plan_destroy": [ctypes.c_void_p],
    "mp_plan_refresh": [ctypes.c_void_p, ctypes.POINTER(MpCsr), ctypes.c_void_p],
    "mpspmv_csr_t": [ctypes.POINTER(MpCsr), ctypes.POINTER(MpVec), ctypes.POINTER(MpVec),
                     ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p],
    "mp_grad_vals": [ctypes.POINTER(MpCsr), ctypes.c_void_p, ctypes.POINTER(MpVec),
                     ctypes.POINTER(MpVec), ctypes.POINTER(MpVec), ctypes.c_int, ctypes.c_void_p],
    "mp_axpy": [ctypes.POINTER(MpVec), ctypes.POINTER(MpVec), ctypes.POINTER(MpVec), ctypes.c_int,
                ctypes.c_void_p],
    "mp_dot": [ctypes.POINTER(MpVec), ctypes.POINTER(MpVec), ctypes.POINTER(MpVec), ctypes.c_int,
               ctypes.c_void_p],
    "mp_const_decimal": [ctypes.c_int64, ctypes.c_int64, ctypes.c_int, ctypes.POINTER(MpVec),
                         ctypes.c_void_p],
    "bicg": [ctypes.POINTER(MpCsr), ctypes.c_void_p, ctypes.POINTER(MpVec), ctypes.POINTER(MpVec),
             ctypes.POINTER(MpSolveOpts), ctypes.POINTER(MpSolveInfo), ctypes.c_void_p],
    "gpbicg": [ctypes.POINTER(MpCsr), ctypes.c_void_p, ctypes.POINTER(MpVec), ctypes.POINTER(MpVec),
               ctypes.POINTER(MpSolveOpts), ctypes.POINTER(MpSolveInfo), ctypes.c_void_p],
    "cgs": [ctypes.POINTER(MpCsr), ctypes.c_void_p, ctypes.POINTER(MpVec), ctypes.POINTER(MpVec),
            ctypes.POINTER(MpSolveOpts), ctypes.POINTER(MpSolveInfo), ctypes.c_void_p],
    "bicgstab": [ctypes.POINTER(MpCsr), ctypes.c_void_p, ctypes.POINTER(MpVec), ctypes.POINTER(MpVec),
                 ctypes.POINTER(MpSolveOpts), ctypes.POINTER(MpSolveInfo), ctypes.c_void_p],
    "mp_ilu0_create": [ctypes.POINTER(MpCsr), ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)],
    "mp_ilu0_destroy": [ctypes.c_void_p],
    "mp_ilu0_apply": [ctypes.c_void_p, ctypes.POINTER(MpVec), ctypes.POINTER(MpVec), ctypes.c_int,
                      ctypes.c_void_p],
    "mp_ilu0_apply_t": [ctypes.c_void_p, ctypes.POINTER(MpVec), ctypes.POINTER(MpVec), ctypes.c_int,
                        ctypes.c_void_p],
    "mp_ilu0_factors": [ctypes.c_void_p, ctypes.POINTER(MpVec), ctypes.c_void_p],
    "bicg_ilu0": [ctypes.POINTER(MpCsr), ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(MpVec),
                  ctypes.POINTER(MpVec), ctypes.POINTER(MpSolveOpts), ctypes.POINTER(MpSolveInfo),
                  ctypes.c_void_p],
    "bicgstab_ilu0": [ctypes.POINTER(MpCsr), ctypes.c_void_p, ctypes.POINTER(MpVec), ctypes.POINTER(MpVec),
                      ctypes.POINTER(MpSolveOpts), ctypes.POINTER(MpSolveInfo), ctypes.c_void_p],
    "gpbicg_batched": [ctypes.c_int, ctypes.POINTER(MpCsr), ctypes.c_int, ctypes.POINTER(MpVec),
                       ctypes.POINTER(MpVec), ctypes.POINTER(MpSolveOpts),
                       ctypes.POINTER(MpSolveInfo), ctypes.c_void_p],
    "mp_timer_create": [ctypes.c_int, ctypes.POINTER(ctypes.c_void_p)],
    "mp_timer_select": [ctypes.c_void_p],
    "mp_timer_read": [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)],
    "mp_timer_destroy": [ctypes.c_void_p],
}
OPTIONAL = {}
# symbols bound by hand above (non-int return types)
SPECIAL = {"mp_last_error"}


def _bind():
    for name, argtypes in list(SIGNATURES.items()) + list(OPTIONAL.items()):
        fn = getattr(LIB, name, None)
        if fn is None:
            if name in SIGNATURES:
                raise ImportError("libmpspmv.so lacks symbol %s" % name)
            continue
        fn.argtypes = argtypes
        fn.restype = ctypes.c_int


_bind()


def last_error():
    return LIB.mp_last_error().decode(errors="replace")


def check(code):
    if code != MPS_OK:
        raise MPError(code, last_error())
    return code
