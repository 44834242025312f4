"""Reference BiCG, GPBiCG, CGS and BiCGSTAB in p-bit RN arithmetic (TEST INFRASTRUCTURE ONLY).

Both follow the paper's Fig. 5 (BiCG left, GPBiCG right) with the preconditioner K = I, the
stopping test (*) of Sec. 4.1, ||r_k||_2 <= c_rel ||r_0||_2 + c_abs, and these readings of
the printed listings:
  * BiCG: the shadow direction update uses the previous shadow residual, and the second
    underlined product is with A^T (BiCG's shadow sequence), not with A.
  * GPBiCG: z = zeta r + eta z - alpha u and r = t - eta y - zeta v (with v = A t), which are the
    updates of Zhang's GPBiCG that keep the recursive residual equal to b - A x in exact
    arithmetic; the shadow residual is r_0; s = w = 0 and beta = 0 before the first iteration;
    the (*) test is applied to the updated residual, then the zeta = 0 exit.
  * x_0 = 0 unless given; a residual that already meets (*) returns x_0 after 0 iterations.
  * Breakdowns the listings do not name (a zero denominator in alpha, or tau = 0) stop the
    iteration with their own status instead of dividing by zero.
Every scalar expression is evaluated left to right with one RN per binary operation; inner
products are exact sums rounded once.

CGS and BiCGSTAB are the other two product-type methods the paper runs (Sec. 4, Tables 1 and 3)
without printing them; they follow their standard unpreconditioned forms (Sonneveld's CGS, van
der Vorst's BiCGSTAB) with K = I, the same shadow residual r~ = r_0, the same (*) test on the
updated residual, and these readings:
  * CGS: u = r + beta q, p = u + beta (q + beta p), q = u - alpha A p, u^ = u + q,
    x = x + alpha u^, r = r - alpha A u^; a zero (r~, A p) stops with the alpha breakdown.
  * BiCGSTAB: beta = (rho / rho_old) (alpha_old / omega_old), p = r + beta (p - omega_old v),
    v = A p, s = r - alpha v, t = A s, omega = (t, s) / (t, t), x = x + alpha p + omega s,
    r = s - omega t.  When (t, t) = 0 (t = A s = 0), omega is taken as 0: then x = x + alpha p
    and r = s, which meets (*) when s = 0 (A s = 0 with s != 0 needs a singular A); omega = 0
    stops after the (*) test (the zeta breakdown, as GPBiCG's zeta = 0 exit), since the next
    beta divides by it.
"""
from .blas import aymx, axpy, dot, xpby
from .mpnum import add, div, is_zero, le, mul, sqrt, sub, zero

CONVERGED = 0
NOT_CONVERGED = 1
BREAKDOWN_RHO = 2
BREAKDOWN_SIGMA = 3
BREAKDOWN_ZETA = 4
BREAKDOWN_TAU = 5


class SolveResult:
    def __init__(self, x, status, iters, res_hist):
        self.x = x
        self.status = status
        self.iters = iters
        self.res_hist = res_hist      # dot(r, r) after each iteration (RN'd), as MP


def _threshold(nrm0, c_rel, c_abs):
    return add(mul(c_rel, nrm0), c_abs)


def _converged(q, thr):
    """The (*) test on the residual whose squared norm (RN'd inner product) is q."""
    return le(sqrt(q), thr)


def bicg(matvec, rmatvec, b, c_rel, c_abs, maxit, p, x0=None, on_iter=None):
    """matvec(v) = A v and rmatvec(v) = A^T v, both in the chosen accumulation mode."""
    n = len(b)
    x = list(x0) if x0 is not None else [zero(p)] * n
    ax = matvec(x)
    r = [sub(bi, ai) for bi, ai in zip(b, ax)]
    rt = list(r)
    q0 = dot(r, r, p)
    thr = _threshold(sqrt(q0), c_rel, c_abs)
    hist = []
    if _converged(q0, thr):
        return SolveResult(x, CONVERGED, 0, hist)
    rho_old = None
    pv = pt = None
    for i in range(1, maxit + 1):
        rho = dot(rt, r, p)
        if is_zero(rho):
            return SolveResult(x, BREAKDOWN_RHO, i - 1, hist)
        if i == 1:
            pv, pt = list(r), list(rt)
        else:
            beta = div(rho, rho_old)
            pv = xpby(r, beta, pv)
            pt = xpby(rt, beta, pt)
        z = matvec(pv)
        zt = rmatvec(pt)
        sigma = dot(pt, z, p)
        if is_zero(sigma):
            return SolveResult(x, BREAKDOWN_SIGMA, i - 1, hist)
        alpha = div(rho, sigma)
        x = axpy(alpha, pv, x)
        r = aymx(alpha, z, r)
        rt = aymx(alpha, zt, rt)
        q = dot(r, r, p)
        hist.append(q)
        if on_iter is not None:
            on_iter(i, {"x": x, "r": r, "rt": rt, "p": pv, "pt": pt, "rho": rho,
                        "alpha": alpha, "sigma": sigma, "q": q})
        if _converged(q, thr):
            return SolveResult(x, CONVERGED, i, hist)
        rho_old = rho
    return SolveResult(x, NOT_CONVERGED, maxit, hist)


def gpbicg(matvec, b, c_rel, c_abs, maxit, p, x0=None, on_iter=None):
    n = len(b)
    zv = [zero(p)] * n
    x = list(x0) if x0 is not None else list(zv)
    ax = matvec(x)
    r = [sub(bi, ai) for bi, ai in zip(b, ax)]
    rt = list(r)
    q0 = dot(r, r, p)
    thr = _threshold(sqrt(q0), c_rel, c_abs)
    hist = []
    if _converged(q0, thr):
        return SolveResult(x, CONVERGED, 0, hist)
    u = list(zv)
    z = list(zv)
    s = list(zv)
    w = list(zv)
    t = list(zv)
    pv = list(zv)
    qv = list(zv)
    v = list(zv)
    beta = zero(p)
    rho_old = alpha_old = zeta_old = None
    for i in range(1, maxit + 1):
        rho = dot(rt, r, p)
        if is_zero(rho):
            return SolveResult(x, BREAKDOWN_RHO, i - 1, hist)
        if i == 1:
            pv = list(r)
        else:
            beta = mul(div(rho, rho_old), div(alpha_old, zeta_old))
            w = [add(vi, mul(beta, qi)) for vi, qi in zip(v, qv)]
            pv = [add(ri, mul(beta, sub(pi, ui))) for ri, pi, ui in zip(r, pv, u)]
        qv = matvec(pv)
        den = dot(rt, qv, p)
        if is_zero(den):
            return SolveResult(x, BREAKDOWN_SIGMA, i - 1, hist)
        alpha = div(rho, den)
        if i > 1:
            s = [sub(ti, ri) for ti, ri in zip(t, r)]
        t = [sub(ri, mul(alpha, qi)) for ri, qi in zip(r, qv)]
        v = matvec(t)
        if i == 1:
            y = [sub(mul(alpha, qi), ri) for qi, ri in zip(qv, r)]
            mu2 = dot(v, t, p)
            mu5 = dot(v, v, p)
            if is_zero(mu5):
                return SolveResult(x, BREAKDOWN_TAU, i - 1, hist)
            zeta = div(mu2, mu5)
            eta = zero(p)
        else:
            y = [sub(si, mul(alpha, sub(wi, qi))) for si, wi, qi in zip(s, w, qv)]
            mu1 = dot(y, y, p)
            mu2 = dot(v, t, p)
            mu3 = dot(y, t, p)
            mu4 = dot(v, y, p)
            mu5 = dot(v, v, p)
            tau = sub(mul(mu5, mu1), mul(mu4, mu4))
            if is_zero(tau):
                return SolveResult(x, BREAKDOWN_TAU, i - 1, hist)
            zeta = div(sub(mul(mu1, mu2), mul(mu3, mu4)), tau)
            eta = div(sub(mul(mu5, mu3), mul(mu4, mu2)), tau)
        u = [add(mul(zeta, qi), mul(eta, add(si, mul(beta, ui)))) for qi, si, ui in zip(qv, s, u)]
        z = [sub(add(mul(zeta, ri), mul(eta, zi)), mul(alpha, ui)) for ri, zi, ui in zip(r, z, u)]
        x = [add(add(xi, mul(alpha, pi)), zi) for xi, pi, zi in zip(x, pv, z)]
        r = [sub(sub(ti, mul(eta, yi)), mul(zeta, vi)) for ti, yi, vi in zip(t, y, v)]
        q = dot(r, r, p)
        hist.append(q)
        if on_iter is not None:
            on_iter(i, {"x": x, "r": r, "p": pv, "t": t, "u": u, "z": z, "alpha": alpha,
                        "zeta": zeta, "eta": eta, "beta": beta, "rho": rho, "q": q})
        if _converged(q, thr):
            return SolveResult(x, CONVERGED, i, hist)
        if is_zero(zeta):
            return SolveResult(x, BREAKDOWN_ZETA, i, hist)
        rho_old, alpha_old, zeta_old = rho, alpha, zeta
    return SolveResult(x, NOT_CONVERGED, maxit, hist)


def cgs(matvec, b, c_rel, c_abs, maxit, p, x0=None, on_iter=None):
    """Conjugate gradient squared: the BiCG residual polynomial applied twice."""
    n = len(b)
    x = list(x0) if x0 is not None else [zero(p)] * n
    ax = matvec(x)
    r = [sub(bi, ai) for bi, ai in zip(b, ax)]
    rt = list(r)
    q0 = dot(r, r, p)
    thr = _threshold(sqrt(q0), c_rel, c_abs)
    hist = []
    if _converged(q0, thr):
        return SolveResult(x, CONVERGED, 0, hist)
    rho_old = None
    qv = pv = None
    for i in range(1, maxit + 1):
        rho = dot(rt, r, p)
        if is_zero(rho):
            return SolveResult(x, BREAKDOWN_RHO, i - 1, hist)
        if i == 1:
            u = list(r)
            pv = list(u)
        else:
            beta = div(rho, rho_old)
            u = xpby(r, beta, qv)
            pv = [add(ui, mul(beta, add(qi, mul(beta, pi)))) for ui, qi, pi in zip(u, qv, pv)]
        vh = matvec(pv)
        sigma = dot(rt, vh, p)
        if is_zero(sigma):
            return SolveResult(x, BREAKDOWN_SIGMA, i - 1, hist)
        alpha = div(rho, sigma)
        qv = aymx(alpha, vh, u)
        uh = [add(ui, qi) for ui, qi in zip(u, qv)]
        x = axpy(alpha, uh, x)
        qh = matvec(uh)
        r = aymx(alpha, qh, r)
        q = dot(r, r, p)
        hist.append(q)
        if on_iter is not None:
            on_iter(i, {"x": x, "r": r, "u": u, "p": pv, "q": qv, "rho": rho, "alpha": alpha,
                        "sigma": sigma, "q2": q})
        if _converged(q, thr):
            return SolveResult(x, CONVERGED, i, hist)
        rho_old = rho
    return SolveResult(x, NOT_CONVERGED, maxit, hist)


def bicgstab(matvec, b, c_rel, c_abs, maxit, p, x0=None, on_iter=None):
    """BiCGSTAB: the BiCG polynomial times a product of local residual-minimising steps."""
    n = len(b)
    x = list(x0) if x0 is not None else [zero(p)] * n
    ax = matvec(x)
    r = [sub(bi, ai) for bi, ai in zip(b, ax)]
    rt = list(r)
    q0 = dot(r, r, p)
    thr = _threshold(sqrt(q0), c_rel, c_abs)
    hist = []
    if _converged(q0, thr):
        return SolveResult(x, CONVERGED, 0, hist)
    rho_old = alpha_old = omega_old = None
    pv = v = None
    for i in range(1, maxit + 1):
        rho = dot(rt, r, p)
        if is_zero(rho):
            return SolveResult(x, BREAKDOWN_RHO, i - 1, hist)
        if i == 1:
            pv = list(r)
        else:
            beta = mul(div(rho, rho_old), div(alpha_old, omega_old))
            pv = [add(ri, mul(beta, sub(pi, mul(omega_old, vi)))) for ri, pi, vi in zip(r, pv, v)]
        v = matvec(pv)
        sigma = dot(rt, v, p)
        if is_zero(sigma):
            return SolveResult(x, BREAKDOWN_SIGMA, i - 1, hist)
        alpha = div(rho, sigma)
        s = aymx(alpha, v, r)
        t = matvec(s)
        ts = dot(t, s, p)
        tt = dot(t, t, p)
        omega = zero(p) if is_zero(tt) else div(ts, tt)
        x = [add(add(xi, mul(alpha, pi)), mul(omega, si)) for xi, pi, si in zip(x, pv, s)]
        r = aymx(omega, t, s)
        q = dot(r, r, p)
        hist.append(q)
        if on_iter is not None:
            on_iter(i, {"x": x, "r": r, "p": pv, "s": s, "t": t, "rho": rho, "alpha": alpha,
                        "omega": omega, "sigma": sigma, "q": q})
        if _converged(q, thr):
            return SolveResult(x, CONVERGED, i, hist)
        if is_zero(omega):
            return SolveResult(x, BREAKDOWN_ZETA, i, hist)
        rho_old, alpha_old, omega_old = rho, alpha, omega
    return SolveResult(x, NOT_CONVERGED, maxit, hist)


def bicgstab_precond(matvec, psolve, b, c_rel, c_abs, maxit, p, x0=None, on_iter=None):
    """BiCGSTAB with a preconditioner K (psolve(v) = K^{-1} v), applied to the two search
    directions, so that the residual the (*) test reads stays b - A x:
    p^ = K^{-1} p, v = A p^, s = r - alpha v, s^ = K^{-1} s, t = A s^,
    omega = (t, s) / (t, t) (0 when (t, t) = 0), x = x + alpha p^ + omega s^, r = s - omega t.
    With psolve the identity this is bicgstab, operation for operation."""
    n = len(b)
    x = list(x0) if x0 is not None else [zero(p)] * n
    ax = matvec(x)
    r = [sub(bi, ai) for bi, ai in zip(b, ax)]
    rt = list(r)
    q0 = dot(r, r, p)
    thr = _threshold(sqrt(q0), c_rel, c_abs)
    hist = []
    if _converged(q0, thr):
        return SolveResult(x, CONVERGED, 0, hist)
    rho_old = alpha_old = omega_old = None
    pv = v = None
    for i in range(1, maxit + 1):
        rho = dot(rt, r, p)
        if is_zero(rho):
            return SolveResult(x, BREAKDOWN_RHO, i - 1, hist)
        if i == 1:
            pv = list(r)
        else:
            beta = mul(div(rho, rho_old), div(alpha_old, omega_old))
            pv = [add(ri, mul(beta, sub(pi, mul(omega_old, vi)))) for ri, pi, vi in zip(r, pv, v)]
        ph = psolve(pv)
        v = matvec(ph)
        sigma = dot(rt, v, p)
        if is_zero(sigma):
            return SolveResult(x, BREAKDOWN_SIGMA, i - 1, hist)
        alpha = div(rho, sigma)
        s = aymx(alpha, v, r)
        sh = psolve(s)
        t = matvec(sh)
        ts = dot(t, s, p)
        tt = dot(t, t, p)
        omega = zero(p) if is_zero(tt) else div(ts, tt)
        x = [add(add(xi, mul(alpha, pi)), mul(omega, si)) for xi, pi, si in zip(x, ph, sh)]
        r = aymx(omega, t, s)
        q = dot(r, r, p)
        hist.append(q)
        if on_iter is not None:
            on_iter(i, {"x": x, "r": r, "p": pv, "s": s, "t": t, "rho": rho, "alpha": alpha,
                        "omega": omega, "sigma": sigma, "q": q})
        if _converged(q, thr):
            return SolveResult(x, CONVERGED, i, hist)
        if is_zero(omega):
            return SolveResult(x, BREAKDOWN_ZETA, i, hist)
        rho_old, alpha_old, omega_old = rho, alpha, omega
    return SolveResult(x, NOT_CONVERGED, maxit, hist)


def bicg_precond(matvec, rmatvec, psolve, psolve_t, b, c_rel, c_abs, maxit, p, x0=None, on_iter=None):
    """BiCG with the left preconditioner K as the paper's Fig. 5 (left) lists it
    (psolve(v) = K^{-1} v, psolve_t(v) = K^{-T} v): w = K^{-1} r, w~ = K^{-T} r~,
    rho = (r~, w), p = w + beta p, p~ = w~ + beta p~ (first: p = w, p~ = w~), z = A p,
    z~ = A^T p~, alpha = rho / (p~, z), x += alpha p, r -= alpha z, r~ -= alpha z~, (*) on r.
    The listing prints rho = (w~, w) = (r~, K^{-1} K^{-1} r), which breaks BiCG's
    biorthogonality for K != I (it does not converge on a small convection-diffusion system that
    plain BiCG solves); rho = (r~, K^{-1} r) = (K^{-T} r~, r) is the preconditioned BiCG's
    coefficient.  With K = I the two forms agree and this is bicg, operation for operation."""
    n = len(b)
    x = list(x0) if x0 is not None else [zero(p)] * n
    ax = matvec(x)
    r = [sub(bi, ai) for bi, ai in zip(b, ax)]
    rt = list(r)
    q0 = dot(r, r, p)
    thr = _threshold(sqrt(q0), c_rel, c_abs)
    hist = []
    if _converged(q0, thr):
        return SolveResult(x, CONVERGED, 0, hist)
    rho_old = None
    pv = pt = None
    for i in range(1, maxit + 1):
        w = psolve(r)
        wt = psolve_t(rt)
        rho = dot(rt, w, p)
        if is_zero(rho):
            return SolveResult(x, BREAKDOWN_RHO, i - 1, hist)
        if i == 1:
            pv, pt = list(w), list(wt)
        else:
            beta = div(rho, rho_old)
            pv = xpby(w, beta, pv)
            pt = xpby(wt, beta, pt)
        z = matvec(pv)
        zt = rmatvec(pt)
        sigma = dot(pt, z, p)
        if is_zero(sigma):
            return SolveResult(x, BREAKDOWN_SIGMA, i - 1, hist)
        alpha = div(rho, sigma)
        x = axpy(alpha, pv, x)
        r = aymx(alpha, z, r)
        rt = aymx(alpha, zt, rt)
        q = dot(r, r, p)
        hist.append(q)
        if on_iter is not None:
            on_iter(i, {"x": x, "r": r, "rt": rt, "p": pv, "pt": pt, "rho": rho, "alpha": alpha,
                        "sigma": sigma, "q": q})
        if _converged(q, thr):
            return SolveResult(x, CONVERGED, i, hist)
        rho_old = rho
    return SolveResult(x, NOT_CONVERGED, maxit, hist)
