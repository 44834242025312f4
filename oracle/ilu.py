"""Reference ILU(0) preconditioner (TEST INFRASTRUCTURE ONLY).

The preconditioner K the paper uses with BiCGSTAB (Sec. 4.2, Table 3): the incomplete LU
factorisation without fill-in, K = L U, L unit lower triangular and U upper triangular, both with
the sparsity pattern of A (every diagonal entry stored).  p-bit RN arithmetic, one rounding per
operation.

Factorisation, row by row (the IKJ form): for i = 0, 1, ..., n-1, for each stored column k < i
of row i in ascending order,
    a_ik <- RN(a_ik / a_kk);
    then for each stored column j > k of row i, in ascending order, that row k also stores:
    a_ij <- RN(a_ij - RN(a_ik * a_kj)).
The factors overwrite a copy of A's values in its CSR layout (L strictly below the diagonal,
U on and above it).  A zero pivot a_kk raises ZeroPivot.

K^T w = r (BiCG's shadow solve in Fig. 5) by the transposed solves U^T y = r (forward) and
L^T w = y (backward), whose rows are the columns of U and L taken in ascending original-row
order (the order of the transposed product).

K w = r by two triangular solves, each row's sum in the product's accumulation mode:
    forward  L y = r:   y_i = r_i - sum_{k<i} l_ik y_k
    backward U w = y:   w_i = (y_i - sum_{j>i} u_ij w_j) / u_ii   (rows in descending order)
SEQ: a sum from +0 of r_i (y_i), then of -RN(l_ik y_k) (-RN(u_ij w_j)) in ascending column
order, one RN per operation (the sparse product's SEQ sum of the row [r_i, -l_ik y_k ...]);
EXACT: the difference is formed exactly and rounded once.  Then one RN division by u_ii.
"""
from .mpnum import MP, add, div, is_zero, mul, sub, zero
from .spmv import EXACT, SEQ, exact_sum_of_products, transpose


class ZeroPivot(ArithmeticError):
    pass


def ilu0(n, row_ptr, col_idx, vals):
    """The ILU(0) factors of A in A's CSR layout (a new list of values)."""
    rp = [int(v) for v in row_ptr]
    ci = [int(v) for v in col_idx]
    a = list(vals)
    diag = []
    for i in range(n):
        ks = [k for k in range(rp[i], rp[i + 1]) if ci[k] == i]
        if not ks:
            raise ZeroPivot("row %d stores no diagonal entry" % i)
        diag.append(ks[0])
    for i in range(n):
        for t in range(rp[i], rp[i + 1]):
            k = ci[t]
            if k >= i:
                break
            piv = a[diag[k]]
            if is_zero(piv):
                raise ZeroPivot("zero pivot in row %d" % k)
            a[t] = div(a[t], piv)
            row_k = {ci[u]: u for u in range(rp[k], rp[k + 1])}
            for u in range(t + 1, rp[i + 1]):
                j = ci[u]
                if j in row_k:
                    a[u] = sub(a[u], mul(a[t], a[row_k[j]]))
    return a


def _row_sum(start, terms, p, mode):
    """start - sum of the products in terms ((a, b) pairs), in the given mode."""
    if mode == SEQ:
        acc = add(zero(p), start)
        for x, y in terms:
            acc = sub(acc, mul(x, y))
        return acc
    if mode == EXACT:
        one = MP(0, 1 << (p - 1), 1, p)
        return exact_sum_of_products([(start, one)] + [(x.neg(), y) for x, y in terms], p)
    raise ValueError("mode must be SEQ (0) or EXACT (1)")


def lower_solve(n, row_ptr, col_idx, lu, r, p, mode):
    """y with L y = r (L unit lower triangular, strictly lower part of lu)."""
    y = [None] * n
    for i in range(n):
        terms = [(lu[t], y[int(col_idx[t])]) for t in range(int(row_ptr[i]), int(row_ptr[i + 1]))
                 if int(col_idx[t]) < i]
        y[i] = _row_sum(r[i], terms, p, mode)
    return y


def upper_solve(n, row_ptr, col_idx, lu, y, p, mode):
    """w with U w = y (U the diagonal and upper part of lu)."""
    w = [None] * n
    for i in range(n - 1, -1, -1):
        d = None
        terms = []
        for t in range(int(row_ptr[i]), int(row_ptr[i + 1])):
            j = int(col_idx[t])
            if j == i:
                d = lu[t]
            elif j > i:
                terms.append((lu[t], w[j]))
        w[i] = div(_row_sum(y[i], terms, p, mode), d)
    return w


def apply(n, row_ptr, col_idx, lu, r, p, mode):
    """w = K^{-1} r = U^{-1} L^{-1} r."""
    return upper_solve(n, row_ptr, col_idx, lu, lower_solve(n, row_ptr, col_idx, lu, r, p, mode), p, mode)


def apply_t(n, row_ptr, col_idx, lu, r, p, mode):
    """w = K^{-T} r = L^{-T} U^{-T} r, through the explicit transpose of the factors (row i of
    the transpose lists column i of L and U, ascending original row)."""
    tp, ti, tv = transpose(n, n, row_ptr, col_idx, lu)
    y = [None] * n
    for i in range(n):                       # U^T y = r: entries k < i are u_ki, k == i is u_ii
        d = None
        terms = []
        for t in range(tp[i], tp[i + 1]):
            k = ti[t]
            if k == i:
                d = tv[t]
            elif k < i:
                terms.append((tv[t], y[k]))
        y[i] = div(_row_sum(r[i], terms, p, mode), d)
    w = [None] * n
    for i in range(n - 1, -1, -1):           # L^T w = y: entries k > i are l_ki
        terms = [(tv[t], w[ti[t]]) for t in range(tp[i], tp[i + 1]) if ti[t] > i]
        w[i] = _row_sum(y[i], terms, p, mode)
    return w

