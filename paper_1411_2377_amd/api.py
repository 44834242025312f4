"""Python entry points with the C ABI's names (argument marshalling only)."""
import ctypes
import os

import torch

from . import _lib
from ._lib import MP_EXACT, MP_SEQ, MPError, check  # noqa: F401
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


def mpspmv_csr(A, x, y=None, mode=MP_SEQ, plan=None, stream=None):
    """y = A x; allocates y when not given.  `plan` (optional) supplies tuned kernel variants.
    Returns y."""
    if y is None:
        y = MPArray.empty(A.n_rows, A.p, device=x.device)
    a, xd, yd = A.desc(), x.desc(), y.desc()
    check(_lib.LIB.mpspmv_csr(ctypes.byref(a), ctypes.byref(xd), ctypes.byref(yd), int(mode),
                              plan.handle if plan is not None else None, _stream(stream)))
    return y


def mp_gemv(vals, rows, cols, x, y=None, mode=MP_SEQ, stream=None):
    """y = A x for the dense row-major matrix A whose rows * cols elements are the MPArray vals
    (zeros stored).  Allocates y when not given.  Returns y."""
    if y is None:
        y = MPArray.empty(int(rows), vals.p, device=x.device)
    d = _lib.MpDense()
    d.rows, d.cols, d.prec = int(rows), int(cols), int(vals.p)
    d.val = vals.desc()
    xd, yd = x.desc(), y.desc()
    check(_lib.LIB.mp_gemv(ctypes.byref(d), ctypes.byref(xd), ctypes.byref(yd), int(mode),
                           _stream(stream)))
    return y


def mpspmv_csr_noalloc(A, x, y, mode=MP_SEQ, stream=None):
    """y = A x into the caller's y through the allocation-free entry point (x staged in the
    library's static scratch array; x.n bounded by its size).  Returns y."""
    a, xd, yd = A.desc(), x.desc(), y.desc()
    check(_lib.LIB.mpspmv_csr_noalloc(ctypes.byref(a), ctypes.byref(xd), ctypes.byref(yd),
                                      int(mode), _stream(stream)))
    return y


def mp_status(stream=None, raise_on_error=True):
    flags = ctypes.c_uint32(0)
    code = _lib.LIB.mp_status(_stream(stream), ctypes.byref(flags))
    if raise_on_error:
        check(code)
    return int(flags.value)


class Plan:
    """Transposed-product plan of a CSRMatrix (owns library memory; freed on close/GC)."""

    def __init__(self, A, stream=None):
        self.A = A
        self._h = ctypes.c_void_p()
        d = A.desc()
        check(_lib.LIB.mp_plan_create(ctypes.byref(d), _stream(stream), ctypes.byref(self._h)))

    @property
    def handle(self):
        return self._h

    def refresh(self, stream=None):
        d = self.A.desc()
        check(_lib.LIB.mp_plan_refresh(self._h, ctypes.byref(d), _stream(stream)))

    def tune(self, reps=3, stream=None, cache=None, x=None, x_t=None):
        """Time the SpMV kernel variants on this matrix and keep the fastest (synchronous).
        With cache=<file path> the choice is looked up in (or added to) that tuning cache;
        self.cache_hit tells which happened.  With x (and/or x_t, MPArrays) the products are
        timed on those operands instead of generated ones (no cache)."""
        d = self.A.desc()
        if x is not None or x_t is not None:
            xd = x.desc() if x is not None else None
            td = x_t.desc() if x_t is not None else None
            check(_lib.LIB.mp_plan_tune_x(self._h, ctypes.byref(d), ctypes.byref(xd) if xd else None,
                                          ctypes.byref(td) if td else None, int(reps), _stream(stream)))
            self.cache_hit = False
        elif cache is None:
            check(_lib.LIB.mp_plan_tune(self._h, ctypes.byref(d), int(reps), _stream(stream)))
            self.cache_hit = False
        else:
            hit = ctypes.c_int(0)
            check(_lib.LIB.mp_plan_tune_cached(self._h, ctypes.byref(d), int(reps),
                                               os.fsencode(cache), ctypes.byref(hit),
                                               _stream(stream)))
            self.cache_hit = bool(hit.value)
        return self.variants()

    def set_variant(self, op, mode, rows=0, stage_x=False, sorted_rows=False, group_min=0,
                    windows=False, segments=False):
        """Force a kernel variant: op 0 = A, 1 = A^T; rows in (0, 16, 32, 64), 0 = by shape;
        stage_x: gather x from staged records; sorted_rows: blocks take rows by decreasing
        length; group_min (SEQ with sorted rows): rows with at least that many entries are
        summed by lane groups (0: none), or with windows by windowed chains (a row per
        wavefront, or with segments four rows per wavefront)."""
        d = self.A.desc()
        flags = (1 if stage_x else 0) | (2 if sorted_rows else 0)
        if group_min:
            flags |= 4 | (int(group_min) << 8) | (8 if windows or segments else 0) | (16 if segments else 0)
        check(_lib.LIB.mp_plan_set_variant(self._h, ctypes.byref(d), int(op), int(mode), int(rows), flags))

    def variants(self):
        """{(op, mode): (rows per block, stage_x, sorted_rows, group_min, windows)} in effect;
        windows is 0, 1 (a row per wavefront) or 2 (four rows per wavefront)."""
        out = {}
        for op in (0, 1):
            for mode in (MP_SEQ, MP_EXACT):
                v, fl = ctypes.c_int(0), ctypes.c_int(0)
                check(_lib.LIB.mp_plan_get_variant(self._h, op, mode, ctypes.byref(v), ctypes.byref(fl)))
                gmin = (fl.value >> 8) if fl.value & 4 else 0
                win = (2 if fl.value & 16 else 1) if (gmin and fl.value & 8) else 0
                out[(op, mode)] = (v.value, bool(fl.value & 1), bool(fl.value & 2), gmin, win)
        return out

    def close(self):
        if self._h and self._h.value:
            _lib.LIB.mp_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mp_plan_create(A, stream=None):
    return Plan(A, stream)


def mpspmv_csr_t(A, plan, x, y=None, mode=MP_SEQ, stream=None):
    """y = A^T x (with the plan's explicit transpose); allocates y when not given."""
    if y is None:
        y = MPArray.empty(A.n_cols, A.p, device=x.device)
    a, xd, yd = A.desc(), x.desc(), y.desc()
    check(_lib.LIB.mpspmv_csr_t(ctypes.byref(a), ctypes.byref(xd), ctypes.byref(yd), int(mode),
                                plan.handle, _stream(stream)))
    return y


def mp_grad_vals(A, plan, g, x, out=None, negate=False, stream=None):
    """out_k = RN(g_i x_j) for each stored entry k = (i, j) (negated if asked)."""
    if out is None:
        out = MPArray.empty(A.nnz, A.p, device=x.device)
    a, gd, xd, od = A.desc(), g.desc(), x.desc(), out.desc()
    check(_lib.LIB.mp_grad_vals(ctypes.byref(a), plan.handle, ctypes.byref(gd), ctypes.byref(xd),
                                ctypes.byref(od), int(bool(negate)), _stream(stream)))
    return out


def mp_axpy(alpha, x, y, stream=None):
    """y <- y + alpha x (alpha a one-element MPArray), in place."""
    ad, xd, yd = alpha.desc(), x.desc(), y.desc()
    check(_lib.LIB.mp_axpy(ctypes.byref(ad), ctypes.byref(xd), ctypes.byref(yd), int(y.p),
                           _stream(stream)))
    return y


def mp_dot(x, y, out=None, stream=None):
    """out = RN(sum x_i y_i) as a one-element MPArray."""
    if out is None:
        out = MPArray.empty(1, x.p, device=x.device)
    xd, yd, od = x.desc(), y.desc(), out.desc()
    check(_lib.LIB.mp_dot(ctypes.byref(xd), ctypes.byref(yd), ctypes.byref(od), int(x.p),
                          _stream(stream)))
    return out


def mp_const_decimal(m, e10, p, device="cuda", stream=None):
    """RN_p(m * 10^e10) as a one-element MPArray."""
    out = MPArray.empty(1, p, device=device)
    od = out.desc()
    check(_lib.LIB.mp_const_decimal(int(m), int(e10), int(p), ctypes.byref(od), _stream(stream)))
    return out


class SolveInfo:
    def __init__(self, status, iters, final_rel_res, hist=None):
        self.status = status
        self.iters = iters
        self.final_rel_res = final_rel_res
        self.res_hist = hist

    def __repr__(self):
        return "SolveInfo(status=%d, iters=%d, rel_res=%.3g)" % (self.status, self.iters,
                                                                  self.final_rel_res)


def _opts(mode, maxit, rtol, atol, chunk, transpose, use_x0):
    o = _lib.MpSolveOpts()
    o.mode = int(mode)
    o.transpose = int(bool(transpose))
    o.maxit = int(maxit)
    o.rtol_m, o.rtol_e10 = int(rtol[0]), int(rtol[1])
    o.atol_m, o.atol_e10 = int(atol[0]), int(atol[1])
    o.chunk = int(chunk)
    o.use_x0 = int(use_x0)
    return o


def _solve(fn, A, b, x=None, plan=None, mode=MP_SEQ, maxit=1000, rtol=(1, -20), atol=(1, -50),
           chunk=16, transpose=False, x0=None, hist=False, profile=None, stream=None):
    if x is None:
        x = MPArray.empty(A.n_rows, A.p, device=b.device)
    use_x0 = 0
    if x0 is not None:
        x.copy_(x0)
        use_x0 = 1
    o = _opts(mode, maxit, rtol, atol, chunk, transpose, use_x0)
    if profile is not None:   # an MpSolveProfile to add kernel timings to
        o.profile = ctypes.pointer(profile)
    hist_arr = None
    if hist:
        hist_arr = MPArray.zeros(max(1, int(maxit)), A.p, device=b.device)
        hd = hist_arr.desc()
        o.res_hist = ctypes.pointer(hd)
    info = _lib.MpSolveInfo()
    a, bd, xd = A.desc(), b.desc(), x.desc()
    check(fn(ctypes.byref(a), plan.handle if plan is not None else None, ctypes.byref(bd),
             ctypes.byref(xd), ctypes.byref(o), ctypes.byref(info), _stream(stream)))
    return x, SolveInfo(info.status, info.iters, info.final_rel_res, hist_arr)


SolveProfile = _lib.MpSolveProfile


def bicg(A, b, **kw):
    """BiCG (K = I) for A x = b (or A^T x = b with transpose=True).  Returns (x, SolveInfo).
    profile=SolveProfile() collects per-class kernel timings (eager launches)."""
    return _solve(_lib.LIB.bicg, A, b, **kw)


def gpbicg(A, b, **kw):
    """GPBiCG for A x = b (or A^T x = b with transpose=True).  Returns (x, SolveInfo)."""
    return _solve(_lib.LIB.gpbicg, A, b, **kw)


def cgs(A, b, **kw):
    """CGS for A x = b (or A^T x = b with transpose=True).  Returns (x, SolveInfo)."""
    return _solve(_lib.LIB.cgs, A, b, **kw)


def bicgstab(A, b, **kw):
    """BiCGSTAB for A x = b (or A^T x = b with transpose=True).  Returns (x, SolveInfo)."""
    return _solve(_lib.LIB.bicgstab, A, b, **kw)


class ILU0:
    """The ILU(0) preconditioner of a square CSRMatrix (factored on creation; owns library
    memory, freed on close/GC)."""

    def __init__(self, A, stream=None):
        self.A = A
        self._h = ctypes.c_void_p()
        d = A.desc()
        check(_lib.LIB.mp_ilu0_create(ctypes.byref(d), _stream(stream), ctypes.byref(self._h)))

    @property
    def handle(self):
        return self._h

    def apply(self, r, w=None, mode=MP_SEQ, stream=None):
        """w = K^{-1} r.  Returns w."""
        if w is None:
            w = MPArray.empty(r.n, r.p, device=r.device)
        rd, wd = r.desc(), w.desc()
        check(_lib.LIB.mp_ilu0_apply(self._h, ctypes.byref(rd), ctypes.byref(wd), int(mode), _stream(stream)))
        return w

    def apply_t(self, r, w=None, mode=MP_SEQ, stream=None):
        """w = K^{-T} r.  Returns w."""
        if w is None:
            w = MPArray.empty(r.n, r.p, device=r.device)
        rd, wd = r.desc(), w.desc()
        check(_lib.LIB.mp_ilu0_apply_t(self._h, ctypes.byref(rd), ctypes.byref(wd), int(mode), _stream(stream)))
        return w

    def factors(self, stream=None):
        """The factors L (strictly below the diagonal) and U in A's CSR layout, as an MPArray."""
        lu = MPArray.empty(self.A.nnz, self.A.p, device=self.A.row_ptr.device)
        d = lu.desc()
        check(_lib.LIB.mp_ilu0_factors(self._h, ctypes.byref(d), _stream(stream)))
        return lu

    def close(self):
        if self._h and self._h.value:
            _lib.LIB.mp_ilu0_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def bicgstab_ilu0(A, ilu, b, **kw):
    """BiCGSTAB preconditioned by ILU(0) (an ILU0 of A).  Returns (x, SolveInfo)."""
    return _solve(_lib.LIB.bicgstab_ilu0, A, b, plan=_Handle(ilu.handle), **kw)


def bicg_ilu0(A, ilu, b, plan=None, **kw):
    """BiCG preconditioned by ILU(0) (an ILU0 of A), K^{-1} on r and K^{-T} on the shadow
    residual.  plan: a Plan of A (None: the library builds one).  Returns (x, SolveInfo)."""
    h = ilu.handle

    def fn(a, pl, bd, xd, o, info, s):
        return _lib.LIB.bicg_ilu0(a, pl, h, bd, xd, o, info, s)
    return _solve(fn, A, b, plan=plan, **kw)


class _Handle:
    def __init__(self, h):
        self.handle = h


def gpbicg_batched(As, bs, mode=MP_SEQ, maxit=1000, rtol=(1, -20), atol=(1, -50), chunk=16,
                   x0s=None, stream=None):
    """Batched GPBiCG: As is a list of nsys square CSRMatrix, bs a list of nsys lists of nrhs
    right-hand sides each.  Every solve is bit-identical to gpbicg(As[s], bs[s][k], ...).
    Returns (xs, infos) shaped like bs."""
    nsys = len(As)
    nrhs = len(bs[0]) if nsys else 0
    if nsys == 0 or nrhs == 0 or any(len(row) != nrhs for row in bs):
        raise ValueError("bs must hold nsys lists of the same positive length")
    xs = [[MPArray.empty(A.n_rows, A.p, device=row[0].device) for _ in row] for A, row in zip(As, bs)]
    use_x0 = 0
    if x0s is not None:
        for xr, x0r in zip(xs, x0s):
            for x, x0 in zip(xr, x0r):
                x.copy_(x0)
        use_x0 = 1
    o = _opts(mode, maxit, rtol, atol, chunk, False, use_x0)
    a_arr = (_lib.MpCsr * nsys)(*[A.desc() for A in As])
    n = nsys * nrhs
    b_arr = (_lib.MpVec * n)(*[b.desc() for row in bs for b in row])
    x_arr = (_lib.MpVec * n)(*[x.desc() for row in xs for x in row])
    infos = (_lib.MpSolveInfo * n)()
    check(_lib.LIB.gpbicg_batched(nsys, a_arr, nrhs, b_arr, x_arr, ctypes.byref(o), infos,
                                  _stream(stream)))
    out = [[SolveInfo(infos[s * nrhs + k].status, infos[s * nrhs + k].iters,
                      infos[s * nrhs + k].final_rel_res, None) for k in range(nrhs)]
           for s in range(nsys)]
    return xs, out


class KernelTimer:
    """Measurement only: HIP events attached to the main kernel of each library call made on
    this thread while the timer is selected (the sparse product's kernel, not its x staging)."""

    def __init__(self, max_launches=4096):
        self._h = ctypes.c_void_p()
        check(_lib.LIB.mp_timer_create(int(max_launches), ctypes.byref(self._h)))

    def select(self):
        check(_lib.LIB.mp_timer_select(self._h))
        return self

    @staticmethod
    def deselect():
        check(_lib.LIB.mp_timer_select(None))

    def read(self):
        """(total microseconds, launches) of the kernels timed since the last read."""
        us, n = ctypes.c_double(0), ctypes.c_int64(0)
        check(_lib.LIB.mp_timer_read(self._h, ctypes.byref(us), ctypes.byref(n)))
        return us.value, n.value

    def close(self):
        if self._h and self._h.value:
            _lib.LIB.mp_timer_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
