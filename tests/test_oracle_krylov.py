"""Pins of the oracle's BiCG / GPBiCG / CGS / BiCGSTAB against what the mathematics fixes.

* small well-conditioned systems converge (within a few times n iterations at p = 256) to the
  solution found by exact Gaussian elimination over the rationals;
* the recursively updated residual stays equal to b - A x up to rounding (this separates the
  corrected GPBiCG updates from the printed ones, which would drift);
* on a symmetric matrix BiCG's shadow residual equals its residual bitwise (BiCG is CG there);
* forced breakdowns and the not-converged exit;
* CGS and BiCGSTAB share BiCG's Lanczos coefficients: in exact arithmetic their alpha_i equal
  BiCG's alpha_i, and CGS's rho_i equal BiCG's rho_i (its residual polynomial is BiCG's squared),
  so at p = 512 the first iterations agree to far below the working precision of any planted
  mistake;
* BiCGSTAB's omega minimises ||s - omega t||: the new residual is orthogonal to t.
"""
from fractions import Fraction
import random

import pytest

from oracle import krylov, mpnum, spmv
from oracle.mpnum import MP


def rand_system(seed, n, p, sym=False, dominance=3):
    rng = random.Random(seed)
    dense = [[Fraction(0)] * n for _ in range(n)]
    for i in range(n):
        for j in range(n):
            if i != j and rng.random() < 0.5:
                dense[i][j] = Fraction(rng.randint(-100, 100), 64)
    if sym:
        for i in range(n):
            for j in range(i):
                dense[i][j] = dense[j][i]
    for i in range(n):
        dense[i][i] = sum(abs(v) for v in dense[i]) + dominance
    rp, ci, vals = [0], [], []
    for i in range(n):
        for j in range(n):
            if dense[i][j] != 0:
                ci.append(j)
                vals.append(mpnum.round_fraction(dense[i][j], p))
        rp.append(len(ci))
    return dense, rp, ci, vals


def gauss_solve(dense, b):
    n = len(b)
    a = [row[:] + [bi] for row, bi in zip(dense, b)]
    for c in range(n):
        piv = next(r for r in range(c, n) if a[r][c] != 0)
        a[c], a[piv] = a[piv], a[c]
        for r in range(n):
            if r != c and a[r][c] != 0:
                f = a[r][c] / a[c][c]
                a[r] = [x - f * y for x, y in zip(a[r], a[c])]
    return [a[i][n] / a[i][i] for i in range(n)]


def ops(rp, ci, vals, n, p, mode):
    return (lambda v: spmv.spmv(rp, ci, vals, v, p, mode),
            lambda v: spmv.spmv_t(n, n, rp, ci, vals, v, p, mode))


def solve_with(solver, mv, rmv, b, c_rel, c_abs, maxit, p, **kw):
    if solver == "bicg":
        return krylov.bicg(mv, rmv, b, c_rel, c_abs, maxit, p, **kw)
    return getattr(krylov, solver)(mv, b, c_rel, c_abs, maxit, p, **kw)


@pytest.mark.parametrize("solver", ["bicg", "gpbicg", "cgs", "bicgstab"])
@pytest.mark.parametrize("mode", [spmv.SEQ, spmv.EXACT])
def test_small_systems_reach_exact_solution(solver, mode):
    p = 256
    for seed, n in ((1, 4), (2, 6), (3, 8)):
        dense, rp, ci, vals = rand_system(seed, n, p)
        rng = random.Random(seed)
        b = [mpnum.from_int(rng.randint(-50, 50), p) for _ in range(n)]
        mv, rmv = ops(rp, ci, vals, n, p, mode)
        c_rel = mpnum.round_fraction(Fraction(1, 10 ** 60), p)
        c_abs = mpnum.zero(p)
        res = solve_with(solver, mv, rmv, b, c_rel, c_abs, 6 * n, p)
        assert res.status == krylov.CONVERGED, res.status
        # exact solution of the p-bit matrix
        adense = [[Fraction(0)] * n for _ in range(n)]
        for i in range(n):
            for t in range(rp[i], rp[i + 1]):
                adense[i][ci[t]] = vals[t].to_fraction()
        xs = gauss_solve(adense, [v.to_fraction() for v in b])
        err = max(abs(a.to_fraction() - e) for a, e in zip(res.x, xs))
        scale = max(abs(e) for e in xs)
        assert err <= scale * Fraction(1, 10 ** 50)


@pytest.mark.parametrize("solver", ["bicg", "gpbicg", "cgs", "bicgstab"])
def test_recursive_residual_tracks_true_residual(solver):
    p = 128
    n = 24
    dense, rp, ci, vals = rand_system(21, n, p, dominance=1)
    b = [mpnum.from_int(i + 1, p) for i in range(n)]
    mv, rmv = ops(rp, ci, vals, n, p, spmv.EXACT)
    c_rel = mpnum.round_fraction(Fraction(1, 10 ** 30), p)
    seen = []

    def hook(i, st):
        ax = spmv.spmv_exact(rp, ci, vals, st["x"], p)
        true_r = [bi.to_fraction() - a.to_fraction() for bi, a in zip(b, ax)]
        gap = max(abs(t - r.to_fraction()) for t, r in zip(true_r, st["r"]))
        seen.append(gap)
    solve_with(solver, mv, rmv, b, c_rel, mpnum.zero(p), 12, p, on_iter=hook)
    bn = max(abs(v.to_fraction()) for v in b)
    assert len(seen) >= 5
    assert max(seen) <= bn * Fraction(1, 2 ** (p - 40))


def test_printed_gpbicg_updates_would_drift():
    """Plant the printed (uncorrected) z and r updates in a copy of the oracle loop: the
    recursive residual then departs from b - A x, which the test above would catch."""
    p = 128
    n = 16
    dense, rp, ci, vals = rand_system(22, n, p, dominance=1)
    b = [mpnum.from_int(i + 1, p) for i in range(n)]
    mv = lambda v: spmv.spmv_exact(rp, ci, vals, v, p)  # noqa: E731
    import oracle.krylov as K
    gaps = []

    def hook(i, st):
        ax = mv(st["x"])
        gaps.append(max(abs(bi.to_fraction() - a.to_fraction() - r.to_fraction())
                        for bi, a, r in zip(b, ax, st["r"])))
    orig = K.gpbicg
    # run the correct oracle and a hand-planted wrong residual update for comparison
    res = orig(mv, b, mpnum.round_fraction(Fraction(1, 10 ** 30), p), mpnum.zero(p), 6, p, on_iter=hook)
    good = max(gaps)
    # planted mistake: r_i = t - eta y - zeta u  (u instead of v)
    wrong = []
    x = [mpnum.zero(p)] * n
    r = list(b)
    rt = list(r)
    u = z = s = w = t = pv = qv = v = [mpnum.zero(p)] * n
    beta = mpnum.zero(p)
    for i in range(1, 5):
        rho = K.dot(rt, r, p)
        if i == 1:
            pv = list(r)
        else:
            beta = K.mul(K.div(rho, rho_old), K.div(alpha_old, zeta_old))
            w = [K.add(vi, K.mul(beta, qi)) for vi, qi in zip(v, qv)]
            pv = [K.add(ri, K.mul(beta, K.sub(pi, ui))) for ri, pi, ui in zip(r, pv, u)]
        qv = mv(pv)
        alpha = K.div(rho, K.dot(rt, qv, p))
        if i > 1:
            s = [K.sub(ti, ri) for ti, ri in zip(t, r)]
        t = [K.sub(ri, K.mul(alpha, qi)) for ri, qi in zip(r, qv)]
        v = mv(t)
        if i == 1:
            y = [K.sub(K.mul(alpha, qi), ri) for qi, ri in zip(qv, r)]
            zeta = K.div(K.dot(v, t, p), K.dot(v, v, p))
            eta = mpnum.zero(p)
        else:
            y = [K.sub(si, K.mul(alpha, K.sub(wi, qi))) for si, wi, qi in zip(s, w, qv)]
            mu1, mu2, mu3, mu4, mu5 = (K.dot(y, y, p), K.dot(v, t, p), K.dot(y, t, p),
                                       K.dot(v, y, p), K.dot(v, v, p))
            tau = K.sub(K.mul(mu5, mu1), K.mul(mu4, mu4))
            zeta = K.div(K.sub(K.mul(mu1, mu2), K.mul(mu3, mu4)), tau)
            eta = K.div(K.sub(K.mul(mu5, mu3), K.mul(mu4, mu2)), tau)
        u = [K.add(K.mul(zeta, qi), K.mul(eta, K.add(si, K.mul(beta, ui)))) for qi, si, ui in zip(qv, s, u)]
        z = [K.sub(K.add(K.mul(zeta, ri), K.mul(eta, zi)), K.mul(alpha, ui)) for ri, zi, ui in zip(r, z, u)]
        x = [K.add(K.add(xi, K.mul(alpha, pi)), zi) for xi, pi, zi in zip(x, pv, z)]
        r = [K.sub(K.sub(ti, K.mul(eta, yi)), K.mul(zeta, ui)) for ti, yi, ui in zip(t, y, u)]
        ax = mv(x)
        wrong.append(max(abs(bi.to_fraction() - a.to_fraction() - ri.to_fraction())
                         for bi, a, ri in zip(b, ax, r)))
        rho_old, alpha_old, zeta_old = rho, alpha, zeta
    assert max(wrong) > 10 ** 6 * max(good, Fraction(1, 2 ** 200))


def test_bicg_symmetric_shadow_equals_residual():
    p = 256
    n = 10
    dense, rp, ci, vals = rand_system(31, n, p, sym=True)
    b = [mpnum.from_int(3 * i - 7, p) for i in range(n)]
    mv, rmv = ops(rp, ci, vals, n, p, spmv.SEQ)
    checks = []

    def hook(i, st):
        checks.append(st["rt"] == st["r"] and st["pt"] == st["p"])
    krylov.bicg(mv, rmv, b, mpnum.round_fraction(Fraction(1, 10 ** 40), p), mpnum.zero(p), 30, p,
                on_iter=hook)
    assert checks and all(checks)


def test_forced_breakdown_and_not_converged():
    p = 128
    one = mpnum.from_int(1, p)
    rp, ci, vals = [0, 1, 2], [1, 0], [one, one]          # A = [[0,1],[1,0]]
    b = [one, mpnum.zero(p)]                                 # b = e1
    mv, rmv = ops(rp, ci, vals, 2, p, spmv.SEQ)
    res = krylov.bicg(mv, rmv, b, mpnum.round_fraction(Fraction(1, 10 ** 20), p), mpnum.zero(p), 10, p)
    assert res.status == krylov.BREAKDOWN_SIGMA and res.iters == 0
    res = krylov.gpbicg(mv, b, mpnum.round_fraction(Fraction(1, 10 ** 20), p), mpnum.zero(p), 10, p)
    assert res.status == krylov.BREAKDOWN_SIGMA
    dense, rp, ci, vals = rand_system(5, 6, p)
    bb = [mpnum.from_int(i + 1, p) for i in range(6)]
    mv, rmv = ops(rp, ci, vals, 6, p, spmv.SEQ)
    res = krylov.bicg(mv, rmv, bb, mpnum.round_fraction(Fraction(1, 10 ** 30), p), mpnum.zero(p), 1, p)
    assert res.status == krylov.NOT_CONVERGED and res.iters == 1 and len(res.res_hist) == 1
    # zero right-hand side: r_0 = 0 already meets the test
    res = krylov.bicg(mv, rmv, [mpnum.zero(p)] * 6, mpnum.round_fraction(Fraction(1, 10 ** 30), p),
                      mpnum.zero(p), 5, p)
    assert res.status == krylov.CONVERGED and res.iters == 0


def test_convergence_test_without_sqrt_is_equivalent():
    """RN(sqrt q) <= thr  <=>  q < (thr + ulp(thr)/2)^2 for a positive p-bit thr."""
    rng = random.Random(2)
    for p in (128, 256):
        for _ in range(300):
            thr = MP(0, rng.getrandbits(p) | (1 << (p - 1)), rng.randint(-20, 20), p)
            mid = thr.to_fraction() + Fraction(2) ** (thr.e - p) / 2
            # q near mid^2 (both sides), and random ones
            base = mpnum.round_fraction(mid * mid, p)
            cands = [base, MP(0, base.m - 1, base.e, p) if base.m > (1 << (p - 1)) else base,
                     MP(0, base.m + 1, base.e, p) if base.m < (1 << p) - 1 else base,
                     MP(0, rng.getrandbits(p) | (1 << (p - 1)), rng.randint(-40, 40), p)]
            for q in cands:
                lhs = mpnum.le(mpnum.sqrt(q), thr)
                rhs = q.to_fraction() < mid * mid
                assert lhs == rhs


def test_cgs_bicgstab_share_bicg_lanczos_coefficients():
    """alpha_i of CGS and BiCGSTAB, and rho_i of CGS, equal BiCG's (exact-arithmetic identities
    of the product-type methods); at p = 512 the computed values agree to 1e-100 relative over
    the first iterations, while a planted mistake in CGS's direction update (q + p instead of
    q + beta p) breaks the agreement from the second iteration on."""
    p = 512
    n = 12
    dense, rp, ci, vals = rand_system(41, n, p, dominance=2)
    b = [mpnum.from_int(2 * i - 5, p) for i in range(n)]
    mv, rmv = ops(rp, ci, vals, n, p, spmv.EXACT)
    c_rel = mpnum.round_fraction(Fraction(1, 10 ** 140), p)
    logs = {}
    for solver in ("bicg", "cgs", "bicgstab"):
        rec = []
        solve_with(solver, mv, rmv, b, c_rel, mpnum.zero(p), 6, p,
                   on_iter=lambda i, st, rec=rec: rec.append((st["alpha"], st["rho"])))
        logs[solver] = rec
    tol = Fraction(1, 10 ** 100)

    def close(a, b):
        fa, fb = a.to_fraction(), b.to_fraction()
        return abs(fa - fb) <= tol * abs(fb)
    for i in range(6):
        assert close(logs["cgs"][i][0], logs["bicg"][i][0]), i
        assert close(logs["cgs"][i][1], logs["bicg"][i][1]), i
        assert close(logs["bicgstab"][i][0], logs["bicg"][i][0]), i
    # the planted mistake: p = u + beta (q + p)
    K = krylov
    x = [mpnum.zero(p)] * n
    r = list(b)
    rt = list(r)
    alphas = []
    rho_old = qv = pv = None
    for i in range(1, 4):
        rho = K.dot(rt, r, p)
        if i == 1:
            u = list(r)
            pv = list(u)
        else:
            beta = K.div(rho, rho_old)
            u = K.xpby(r, beta, qv)
            pv = [K.add(ui, K.mul(beta, K.add(qi, pi))) for ui, qi, pi in zip(u, qv, pv)]
        vh = mv(pv)
        alpha = K.div(rho, K.dot(rt, vh, p))
        alphas.append(alpha)
        qv = K.aymx(alpha, vh, u)
        uh = [K.add(ui, qi) for ui, qi in zip(u, qv)]
        x = K.axpy(alpha, uh, x)
        r = K.aymx(alpha, mv(uh), r)
        rho_old = rho
    assert close(alphas[0], logs["bicg"][0][0])
    assert not close(alphas[1], logs["bicg"][1][0])


def test_bicgstab_residual_orthogonal_to_t():
    """omega = (t, s) / (t, t) minimises ||s - omega t||, so r = s - omega t is orthogonal to t
    (to rounding) and ||r|| <= ||s||."""
    p = 256
    n = 16
    dense, rp, ci, vals = rand_system(42, n, p, dominance=1)
    b = [mpnum.from_int(i * i - 20, p) for i in range(n)]
    mv, rmv = ops(rp, ci, vals, n, p, spmv.SEQ)
    seen = []

    def hook(i, st):
        rt_ = spmv.exact_sum_of_products(list(zip(st["r"], st["t"])), p).to_fraction()
        rn = sum(v.to_fraction() ** 2 for v in st["r"])
        sn = sum(v.to_fraction() ** 2 for v in st["s"])
        tn = sum(v.to_fraction() ** 2 for v in st["t"])
        seen.append((rt_ * rt_, sn * tn, rn, sn))
    krylov.bicgstab(mv, b, mpnum.round_fraction(Fraction(1, 10 ** 50), p), mpnum.zero(p), 8, p, on_iter=hook)
    assert len(seen) >= 4
    for rt2, sntn, rn, sn in seen:
        assert rt2 <= sntn * Fraction(1, 2 ** (2 * p - 80))
        assert rn <= sn * (1 + Fraction(1, 2 ** (p - 20)))


def test_cgs_bicgstab_breakdowns_and_limits():
    p = 128
    one = mpnum.from_int(1, p)
    rp, ci, vals = [0, 1, 2], [1, 0], [one, one]          # A = [[0,1],[1,0]], b = e1
    b = [one, mpnum.zero(p)]
    mv, rmv = ops(rp, ci, vals, 2, p, spmv.SEQ)
    c_rel = mpnum.round_fraction(Fraction(1, 10 ** 20), p)
    for solver in ("cgs", "bicgstab"):
        res = solve_with(solver, mv, rmv, b, c_rel, mpnum.zero(p), 10, p)
        assert res.status == krylov.BREAKDOWN_SIGMA and res.iters == 0
    # A = I: BiCGSTAB's s = 0, t = 0: omega = 0, x = alpha p = b, converged in one iteration
    rp, ci, vals = [0, 1, 2, 3], [0, 1, 2], [one] * 3
    b3 = [mpnum.from_int(k + 2, p) for k in range(3)]
    mv, rmv = ops(rp, ci, vals, 3, p, spmv.SEQ)
    res = krylov.bicgstab(mv, b3, c_rel, mpnum.zero(p), 10, p)
    assert res.status == krylov.CONVERGED and res.iters == 1 and res.x == b3
    res = krylov.cgs(mv, b3, c_rel, mpnum.zero(p), 10, p)
    assert res.status == krylov.CONVERGED and res.iters == 1 and res.x == b3
    # singular A = [[1, 1], [0, 0]], b = (1, 1): alpha = 1, s = (-1, 1) with A s = 0, so
    # omega = 0, x = (1, 1), r = s != 0: the zeta breakdown after one iteration
    rp, ci, vals = [0, 2, 2], [0, 1], [one, one]
    mv, rmv = ops(rp, ci, vals, 2, p, spmv.SEQ)
    res = krylov.bicgstab(mv, [one, one], c_rel, mpnum.zero(p), 10, p)
    assert res.status == krylov.BREAKDOWN_ZETA and res.iters == 1
    dense, rp, ci, vals = rand_system(5, 6, p)
    bb = [mpnum.from_int(i + 1, p) for i in range(6)]
    mv, rmv = ops(rp, ci, vals, 6, p, spmv.SEQ)
    for solver in ("cgs", "bicgstab"):
        res = solve_with(solver, mv, rmv, bb, mpnum.round_fraction(Fraction(1, 10 ** 30), p), mpnum.zero(p), 1, p)
        assert res.status == krylov.NOT_CONVERGED and res.iters == 1 and len(res.res_hist) == 1
        res = solve_with(solver, mv, rmv, [mpnum.zero(p)] * 6, c_rel, mpnum.zero(p), 5, p)
        assert res.status == krylov.CONVERGED and res.iters == 0
