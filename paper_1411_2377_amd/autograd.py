"""torch.autograd wrappers: y = A x and x = A^{-1} b with hand-written backward passes.

Autograd only tracks floating-point tensors, so an MP array travels through the graph as a
float32 *bit view* of its packed int32 storage: a tensor of shape [L + 1, N] whose first L rows
are the limb planes and whose last row is the header row (zero-copy in both directions).  The
values are never touched by float arithmetic.

Backward passes (d<g, A x>/dx = A^T g, d<g, A x>/da_ij = g_i x_j; for x = A^{-1} b,
d<g, x>/db = A^{-T} g = lambda and d<g, x>/da_ij = -lambda_i x_j):
  * MPSpMV:  grad_x = mpspmv_csr_t(A, g) in the forward's mode; grad_vals = mp_grad_vals(g, x).
  * MPSolve: lambda = one transposed BiCG solve A^T lambda = g; grad_b = lambda;
             grad_vals = -RN(lambda_i x_j).

Limit: torch sums the gradients of a tensor used by several operations with float addition,
which would corrupt MP bits, so every MP tensor may feed at most one MP operation per backward
pass; a second use raises.  A use ends when its backward pass has run or when the graph node of
the operation is freed (no output depends on it any more); calls made with gradients disabled
(torch.no_grad) are not uses.

A solve's gradient is the adjoint of the solution, so it is only defined when the solve
converged: the forward raises MPSolveError when BiCG stops without meeting the stopping test
(unless require_converged=False is passed, for a forward value only), and the backward raises
when the forward or the transposed (adjoint) solve did not converge.
"""
import weakref

import torch

from . import _lib, api
from .mparray import CSRMatrix, MPArray

_USES = {}  # id(tensor) -> (weak reference to it, weak reference to the claiming graph node)


class MPSolveError(RuntimeError):
    """A solve inside the autograd graph did not converge (no adjoint gradient exists)."""


def pack(a):
    """MPArray -> float32 bit view [L + 1, N] (one copy into packed storage)."""
    L = a.p // 32
    buf = torch.empty((L + 1, a.n), dtype=torch.int32, device=a.device)
    buf[:L].copy_(a.limbs)
    buf[L].copy_(a.hdr)
    return buf.view(torch.float32)


def unpack(t, p):
    """float32 bit view [L + 1, N] -> MPArray over the same storage (no copy)."""
    t = t.contiguous()
    L = p // 32
    assert t.dim() == 2 and t.shape[0] == L + 1, "expected a packed MP tensor of %d rows" % (L + 1)
    i = t.view(torch.int32)
    return MPArray(i[:L], i[L], p)


def _in_use(t):
    ent = _USES.get(id(t))
    return ent is not None and ent[0]() is t and ent[1]() is not None


def _check_free(tensors, track):
    """The inputs this operation claims (those that need a gradient, when gradients are
    recorded), after checking that none of them already feeds a pending MP operation."""
    if not track:
        return []
    out = [t for t in tensors if t is not None and t.requires_grad]
    for t in out:
        if _in_use(t):
            raise RuntimeError("an MP tensor may feed only one MP operation per backward pass "
                               "(float gradient accumulation would corrupt it)")
    return out


def _claim(tensors, node):
    """Record the uses until the backward pass releases them or the graph `node` is freed."""
    ow = weakref.ref(node)
    keys = []
    for t in tensors:
        key = id(t)
        _USES[key] = (weakref.ref(t, lambda _r, k=key: _USES.pop(k, None)), ow)
        keys.append((key, weakref.ref(t)))
    return keys


def _release(keys):
    for key, tw in keys or ():
        ent = _USES.get(key)
        if ent is not None and ent[0]() is tw():
            _USES.pop(key, None)


class SparseStructure:
    """The fixed part of a CSR matrix (shape, row pointers, column indices) plus its plan."""

    def __init__(self, n_rows, n_cols, row_ptr, col_idx, p):
        self.n_rows, self.n_cols, self.p = int(n_rows), int(n_cols), int(p)
        self.row_ptr, self.col_idx = row_ptr, col_idx
        self._plan = None

    @staticmethod
    def of(A):
        return SparseStructure(A.n_rows, A.n_cols, A.row_ptr, A.col_idx, A.p)

    def matrix(self, vals):
        return CSRMatrix(self.n_rows, self.n_cols, self.row_ptr, self.col_idx, vals)

    def plan(self, A):
        if self._plan is None:
            self._plan = api.mp_plan_create(A)
        else:
            self._plan.A = A
            self._plan.refresh()
        return self._plan


class MPSpMV(torch.autograd.Function):
    @staticmethod
    def forward(ctx, vals_t, x_t, S, mode, track):
        claimed = _check_free((vals_t, x_t), track)
        A = S.matrix(unpack(vals_t, S.p))
        x = unpack(x_t, S.p)
        y = api.mpspmv_csr(A, x, mode=mode)
        ctx.save_for_backward(vals_t, x_t)
        ctx.S, ctx.mode = S, mode
        out = pack(y)
        ctx.claims = _claim(claimed, ctx)
        return out

    @staticmethod
    def backward(ctx, g_t):
        vals_t, x_t = ctx.saved_tensors
        S = ctx.S
        _release(ctx.claims)
        A = S.matrix(unpack(vals_t, S.p))
        g = unpack(g_t, S.p)
        P = S.plan(A)
        gx = gv = None
        if ctx.needs_input_grad[1]:
            gx = pack(api.mpspmv_csr_t(A, P, g, mode=ctx.mode))
        if ctx.needs_input_grad[0]:
            gv = pack(api.mp_grad_vals(A, P, g, unpack(x_t, S.p)))
        return gv, gx, None, None, None


class MPSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, vals_t, b_t, S, opts, track, require_converged):
        claimed = _check_free((vals_t, b_t), track)
        A = S.matrix(unpack(vals_t, S.p))
        P = S.plan(A)
        x, info = api.bicg(A, unpack(b_t, S.p), plan=P, **opts)
        if info.status != _lib.MP_CONVERGED and require_converged:
            raise MPSolveError("BiCG did not converge (status %d after %d iterations); pass "
                               "require_converged=False to use the iterate anyway"
                               % (info.status, info.iters))
        ctx.info = info
        xt = pack(x)
        ctx.save_for_backward(vals_t, xt)
        ctx.S, ctx.opts = S, opts
        ctx.claims = _claim(claimed, ctx)
        return xt

    @staticmethod
    def backward(ctx, g_t):
        vals_t, x_t = ctx.saved_tensors
        S = ctx.S
        _release(ctx.claims)
        if ctx.info.status != _lib.MP_CONVERGED:
            raise MPSolveError("no gradient through a solve that did not converge (status %d "
                               "after %d iterations)" % (ctx.info.status, ctx.info.iters))
        A = S.matrix(unpack(vals_t, S.p))
        P = S.plan(A)
        lam, info = api.bicg(A, unpack(g_t, S.p), plan=P, transpose=True, **ctx.opts)
        ctx.adjoint_info = info
        if info.status != _lib.MP_CONVERGED:
            raise MPSolveError("the adjoint (transposed) solve did not converge (status %d after "
                               "%d iterations): the gradient is undefined" % (info.status, info.iters))
        gb = pack(lam) if ctx.needs_input_grad[1] else None
        gv = None
        if ctx.needs_input_grad[0]:
            gv = pack(api.mp_grad_vals(A, P, lam, unpack(x_t, S.p), negate=True))
        return gv, gb, None, None, None, None


def spmv(S, vals_t, x_t, mode=api.MP_SEQ):
    """y = A x with A = (S, vals); packed MP tensors in and out."""
    return MPSpMV.apply(vals_t, x_t, S, mode, torch.is_grad_enabled())


def solve(S, vals_t, b_t, require_converged=True, **opts):
    """x = A^{-1} b by BiCG (options as api.bicg); backward is one transposed BiCG solve.
    Raises MPSolveError when the solve does not converge (require_converged=False returns the
    last iterate; its backward still raises)."""
    return MPSolve.apply(vals_t, b_t, S, opts, torch.is_grad_enabled(), bool(require_converged))
