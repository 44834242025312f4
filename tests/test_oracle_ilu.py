"""Pins of the oracle's ILU(0) preconditioner and preconditioned BiCGSTAB against what the
mathematics fixes:

* the defining property of ILU(0): (L U)_ij = a_ij on A's pattern, to the rounding bound of
  the factorisation (a planted mistake, the pivot of the wrong row, breaks it);
* on a tridiagonal matrix ILU(0) is the complete LU factorisation (exact Fraction LU);
* a diagonal matrix is its own U and has no L;
* triangular solves: L y = r and U w = y to their rounding bounds; in EXACT mode each y_i is the
  rounded exact value; a diagonal U divides;
* preconditioned BiCGSTAB with the identity preconditioner is plain BiCGSTAB, bit for bit; with
  ILU(0) it solves small systems to their Gauss solution and needs fewer iterations;
* the transposed application K^{-T} is the adjoint of K^{-1} (a planted K^{-1} in its place
  fails); preconditioned BiCG with the identity preconditioner is plain BiCG, bit for bit, and
  with ILU(0) it reaches the exact solution.
"""
from fractions import Fraction
import random

import pytest

import synth
from oracle import codec, ilu, krylov, mpnum, spmv
from oracle.mpnum import MP


def rand_sparse(seed, n, p, density=0.35, dominance=2):
    rng = random.Random(seed)
    rp, ci, vals = [0], [], []
    for i in range(n):
        row = {}
        for j in range(n):
            if j != i and rng.random() < density:
                row[j] = Fraction(rng.randint(-90, 90), 32)
        row[i] = sum(abs(v) for v in row.values()) + dominance
        for j in sorted(row):
            if row[j] != 0:
                ci.append(j)
                vals.append(mpnum.round_fraction(row[j], p))
        rp.append(len(ci))
    return rp, ci, vals


def factors(n, rp, ci, lu):
    L = [[Fraction(0)] * n for _ in range(n)]
    U = [[Fraction(0)] * n for _ in range(n)]
    for i in range(n):
        L[i][i] = Fraction(1)
        for t in range(rp[i], rp[i + 1]):
            j = ci[t]
            (L if j < i else U)[i][j] = lu[t].to_fraction()
    return L, U


@pytest.mark.parametrize("p", [128, 256])
def test_lu_reproduces_a_on_its_pattern(p):
    n = 14
    rp, ci, vals = rand_sparse(p, n, p)
    lu = ilu.ilu0(n, rp, ci, vals)
    L, U = factors(n, rp, ci, lu)
    for i in range(n):
        for t in range(rp[i], rp[i + 1]):
            j = ci[t]
            prod = sum(L[i][k] * U[k][j] for k in range(n))
            mag = sum(abs(L[i][k] * U[k][j]) for k in range(n))
            assert abs(prod - vals[t].to_fraction()) <= mag * Fraction(4 * n, 2 ** p), (i, j)


def test_wrong_pivot_breaks_the_pattern_property():
    p = 128
    n = 10
    rp, ci, vals = rand_sparse(7, n, p)
    a = list(vals)
    diag = {i: next(t for t in range(rp[i], rp[i + 1]) if ci[t] == i) for i in range(n)}
    for i in range(n):                                  # planted: divide by a_ii, not a_kk
        for t in range(rp[i], rp[i + 1]):
            k = ci[t]
            if k >= i:
                break
            a[t] = mpnum.div(a[t], a[diag[i]])
            row_k = {ci[u]: u for u in range(rp[k], rp[k + 1])}
            for u in range(t + 1, rp[i + 1]):
                if ci[u] in row_k:
                    a[u] = mpnum.sub(a[u], mpnum.mul(a[t], a[row_k[ci[u]]]))
    L, U = factors(n, rp, ci, a)
    worst = max(abs(sum(L[i][k] * U[k][ci[t]] for k in range(n)) - vals[t].to_fraction())
                for i in range(n) for t in range(rp[i], rp[i + 1]))
    assert worst > Fraction(1, 10 ** 6)


def test_tridiagonal_is_complete_lu():
    p = 256
    n = 12
    rng = random.Random(3)
    dense = [[Fraction(0)] * n for _ in range(n)]
    for i in range(n):
        for j in (i - 1, i + 1):
            if 0 <= j < n:
                dense[i][j] = Fraction(rng.randint(-50, 50), 8)
        dense[i][i] = Fraction(rng.randint(200, 300), 4)
    rp, ci, vals = [0], [], []
    for i in range(n):
        for j in range(n):
            if dense[i][j] != 0:
                ci.append(j)
                vals.append(mpnum.round_fraction(dense[i][j], p))
        rp.append(len(ci))
    lu = ilu.ilu0(n, rp, ci, vals)
    # exact Doolittle LU of the p-bit matrix
    A = [[Fraction(0)] * n for _ in range(n)]
    for i in range(n):
        for t in range(rp[i], rp[i + 1]):
            A[i][ci[t]] = vals[t].to_fraction()
    Lx = [[Fraction(int(i == j)) for j in range(n)] for i in range(n)]
    Ux = [row[:] for row in A]
    for k in range(n):
        for i in range(k + 1, n):
            f = Ux[i][k] / Ux[k][k]
            Lx[i][k] = f
            Ux[i] = [a - f * b for a, b in zip(Ux[i], Ux[k])]
    for i in range(n):
        for t in range(rp[i], rp[i + 1]):
            j = ci[t]
            want = Lx[i][j] if j < i else Ux[i][j]
            assert abs(lu[t].to_fraction() - want) <= abs(want) * Fraction(1, 2 ** (p - 20))


def test_diagonal_matrix_and_its_solve():
    p = 128
    n = 6
    rng = random.Random(4)
    vals = [MP(rng.randint(0, 1), rng.getrandbits(p) | (1 << (p - 1)), rng.randint(-5, 5), p) for _ in range(n)]
    rp, ci = list(range(n + 1)), list(range(n))
    lu = ilu.ilu0(n, rp, ci, vals)
    assert lu == vals
    r = [MP(0, rng.getrandbits(p) | (1 << (p - 1)), rng.randint(-5, 5), p) for _ in range(n)]
    for mode in (spmv.SEQ, spmv.EXACT):
        w = ilu.apply(n, rp, ci, lu, r, p, mode)
        assert w == [mpnum.div(a, b) for a, b in zip(r, vals)]


@pytest.mark.parametrize("mode", [spmv.SEQ, spmv.EXACT])
def test_triangular_solves(mode):
    p = 256
    n = 16
    rp, ci, vals = rand_sparse(11, n, p, density=0.3)
    lu = ilu.ilu0(n, rp, ci, vals)
    L, U = factors(n, rp, ci, lu)
    rng = random.Random(5)
    r = [MP(rng.randint(0, 1), rng.getrandbits(p) | (1 << (p - 1)), rng.randint(-3, 3), p) for _ in range(n)]
    y = ilu.lower_solve(n, rp, ci, lu, r, p, mode)
    w = ilu.upper_solve(n, rp, ci, lu, y, p, mode)
    yf, wf = [v.to_fraction() for v in y], [v.to_fraction() for v in w]
    for i in range(n):
        terms = [L[i][k] * yf[k] for k in range(i)]
        exact = r[i].to_fraction() - sum(terms)
        if mode == spmv.EXACT:
            assert y[i] == mpnum.round_fraction(exact, p)
        mag = abs(r[i].to_fraction()) + sum(abs(t) for t in terms)
        assert abs(yf[i] - exact) <= mag * Fraction(n + 2, 2 ** p)
        upper = [U[i][j] * wf[j] for j in range(i + 1, n)]
        resid = yf[i] - sum(upper) - U[i][i] * wf[i]
        mag = abs(yf[i]) + sum(abs(t) for t in upper)
        assert abs(resid) <= mag * Fraction(n + 4, 2 ** p)


def test_identity_preconditioner_is_plain_bicgstab():
    p = 128
    n = 16
    rp, ci, vals = rand_sparse(21, n, p, dominance=1)
    b = [mpnum.from_int(i + 1, p) for i in range(n)]
    mv = lambda v: spmv.spmv(rp, ci, vals, v, p, spmv.SEQ)  # noqa: E731
    c_rel = mpnum.round_fraction(Fraction(1, 10 ** 30), p)
    a = krylov.bicgstab(mv, b, c_rel, mpnum.zero(p), 12, p)
    b2 = krylov.bicgstab_precond(mv, lambda v: list(v), b, c_rel, mpnum.zero(p), 12, p)
    assert (a.status, a.iters) == (b2.status, b2.iters)
    assert a.x == b2.x and a.res_hist == b2.res_hist


@pytest.mark.parametrize("mode", [spmv.SEQ, spmv.EXACT])
def test_ilu_bicgstab_solves_and_saves_iterations(mode):
    p = 256
    A_h, _ = synth.config2(p=p, m=8)
    n = A_h.n_rows
    rp, ci = A_h.row_ptr.tolist(), A_h.col_idx.tolist()
    vals = codec.decode(A_h.vals.limbs, A_h.vals.hdr, p)
    xs = [mpnum.from_int(i + 1, p) for i in range(n)]
    b = spmv.spmv_exact(rp, ci, vals, xs, p)
    lu = ilu.ilu0(n, rp, ci, vals)
    mv = lambda v: spmv.spmv(rp, ci, vals, v, p, mode)  # noqa: E731
    c_rel = mpnum.round_fraction(Fraction(1, 10 ** 60), p)
    pre = krylov.bicgstab_precond(mv, lambda v: ilu.apply(n, rp, ci, lu, v, p, mode), b, c_rel,
                                  mpnum.zero(p), 200, p)
    plain = krylov.bicgstab(mv, b, c_rel, mpnum.zero(p), 200, p)
    assert pre.status == krylov.CONVERGED and plain.status == krylov.CONVERGED
    assert pre.iters < plain.iters
    err = max(abs(a.to_fraction() - (i + 1)) for i, a in enumerate(pre.x))
    assert err <= Fraction(n, 10 ** 50)


@pytest.mark.parametrize("mode", [spmv.SEQ, spmv.EXACT])
def test_transposed_application_is_the_adjoint(mode):
    """<a, K^{-1} c> = <K^{-T} a, c> for the exact operators; the computed sides agree to the
    solves' rounding (p = 512, so far below any planted mistake's effect), and on a diagonal K
    both applications divide."""
    p = 512
    n = 14
    rp, ci, vals = rand_sparse(31, n, p, density=0.3)
    lu = ilu.ilu0(n, rp, ci, vals)
    rng = random.Random(6)
    a = [MP(rng.randint(0, 1), rng.getrandbits(p) | (1 << (p - 1)), rng.randint(-3, 3), p) for _ in range(n)]
    c = [MP(rng.randint(0, 1), rng.getrandbits(p) | (1 << (p - 1)), rng.randint(-3, 3), p) for _ in range(n)]
    kc = ilu.apply(n, rp, ci, lu, c, p, mode)
    kta = ilu.apply_t(n, rp, ci, lu, a, p, mode)
    lhs = sum(x.to_fraction() * y.to_fraction() for x, y in zip(a, kc))
    rhs = sum(x.to_fraction() * y.to_fraction() for x, y in zip(kta, c))
    scale = sum(abs(x.to_fraction() * y.to_fraction()) for x, y in zip(a, kc))
    assert abs(lhs - rhs) <= scale * Fraction(1, 2 ** (p - 40))
    # a planted mistake (K^{-1} in place of K^{-T}) is far off on a nonsymmetric factor
    wrong = ilu.apply(n, rp, ci, lu, a, p, mode)
    rw = sum(x.to_fraction() * y.to_fraction() for x, y in zip(wrong, c))
    assert abs(lhs - rw) > scale * Fraction(1, 10 ** 6)
    d = [MP(0, rng.getrandbits(p) | (1 << (p - 1)), rng.randint(-3, 3), p) for _ in range(n)]
    drp, dci = list(range(n + 1)), list(range(n))
    assert ilu.apply_t(n, drp, dci, d, a, p, mode) == ilu.apply(n, drp, dci, d, a, p, mode)


def test_identity_preconditioner_is_plain_bicg():
    p = 128
    n = 16
    rp, ci, vals = rand_sparse(22, n, p, dominance=1)
    b = [mpnum.from_int(i + 1, p) for i in range(n)]
    mv = lambda v: spmv.spmv(rp, ci, vals, v, p, spmv.EXACT)  # noqa: E731
    rmv = lambda v: spmv.spmv_t(n, n, rp, ci, vals, v, p, spmv.EXACT)  # noqa: E731
    c_rel = mpnum.round_fraction(Fraction(1, 10 ** 30), p)
    a = krylov.bicg(mv, rmv, b, c_rel, mpnum.zero(p), 12, p)
    ident = lambda v: list(v)  # noqa: E731
    b2 = krylov.bicg_precond(mv, rmv, ident, ident, b, c_rel, mpnum.zero(p), 12, p)
    assert (a.status, a.iters) == (b2.status, b2.iters)
    assert a.x == b2.x and a.res_hist == b2.res_hist


@pytest.mark.parametrize("mode", [spmv.SEQ, spmv.EXACT])
def test_ilu_bicg_solves(mode):
    p = 256
    A_h, _ = synth.config2(p=p, m=8)
    n = A_h.n_rows
    rp, ci = A_h.row_ptr.tolist(), A_h.col_idx.tolist()
    vals = codec.decode(A_h.vals.limbs, A_h.vals.hdr, p)
    xs = [mpnum.from_int(i + 1, p) for i in range(n)]
    b = spmv.spmv_exact(rp, ci, vals, xs, p)
    lu = ilu.ilu0(n, rp, ci, vals)
    mv = lambda v: spmv.spmv(rp, ci, vals, v, p, mode)  # noqa: E731
    rmv = lambda v: spmv.spmv_t(n, n, rp, ci, vals, v, p, mode)  # noqa: E731
    c_rel = mpnum.round_fraction(Fraction(1, 10 ** 60), p)
    pre = krylov.bicg_precond(mv, rmv, lambda v: ilu.apply(n, rp, ci, lu, v, p, mode),
                              lambda v: ilu.apply_t(n, rp, ci, lu, v, p, mode), b, c_rel,
                              mpnum.zero(p), 300, p)
    assert pre.status == krylov.CONVERGED
    err = max(abs(a.to_fraction() - (i + 1)) for i, a in enumerate(pre.x))
    assert err <= Fraction(n, 10 ** 50)
