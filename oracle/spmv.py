"""Reference multiple-precision sparse matrix-vector products (TEST INFRASTRUCTURE ONLY).

The matrix is in compressed sparse row form, as the paper's sparse structure (Sec. 2: per-row
non-zero counts, a one-dimensional array of the stored elements and their column indices):
row_ptr[n+1], col_idx[nnz] (strictly ascending within each row), vals = list of MP.

Two accumulation modes:
  SEQ   : y_i <- +0, then y_i <- RN(y_i + RN(a_ij * x_j)) for the stored entries of row i in
          ascending column order (the paper's SpMV is a loop of MPFR multiplies and adds, Sec. 2
          and Sec. 3; the paper does not print the loop, so storage order is the reading).
  EXACT : y_i = RN(sum_j a_ij * x_j), the sum formed exactly, rounded once.
"""
from fractions import Fraction

from .mpnum import MP, add, mul, round_scaled, zero

SEQ = 0
EXACT = 1


def spmv_seq(row_ptr, col_idx, vals, x, p):
    n = len(row_ptr) - 1
    y = []
    for i in range(n):
        acc = zero(p)
        for k in range(int(row_ptr[i]), int(row_ptr[i + 1])):
            acc = add(acc, mul(vals[k], x[int(col_idx[k])]))
        y.append(acc)
    return y


def exact_sum_of_products(pairs, p):
    """RN of the exact sum of a_k * b_k over the given (a, b) pairs; an exact zero gives +0."""
    terms = []
    for a, b in pairs:
        if a.m == 0 or b.m == 0:
            continue
        terms.append((a.s ^ b.s, a.m * b.m, a.e + b.e - 2 * p))
    if not terms:
        return zero(p)
    lo = min(t[2] for t in terms)
    n = 0
    for s, m, k in terms:
        v = m << (k - lo)
        n += -v if s else v
    if n == 0:
        return zero(p)
    return round_scaled(1 if n < 0 else 0, abs(n), lo, p)


def spmv_exact(row_ptr, col_idx, vals, x, p):
    n = len(row_ptr) - 1
    y = []
    for i in range(n):
        pairs = [(vals[k], x[int(col_idx[k])]) for k in range(int(row_ptr[i]), int(row_ptr[i + 1]))]
        y.append(exact_sum_of_products(pairs, p))
    return y


def spmv(row_ptr, col_idx, vals, x, p, mode):
    if mode == SEQ:
        return spmv_seq(row_ptr, col_idx, vals, x, p)
    if mode == EXACT:
        return spmv_exact(row_ptr, col_idx, vals, x, p)
    raise ValueError("mode must be SEQ (0) or EXACT (1)")


def transpose(n_rows, n_cols, row_ptr, col_idx, vals):
    """Explicit CSR of A^T with each new row's entries in ascending original-row order.

    The per-column counts are the paper's per-column non-zero numbers of the sparse structure.
    """
    counts = [0] * n_cols
    for j in col_idx:
        counts[int(j)] += 1
    t_ptr = [0] * (n_cols + 1)
    for j in range(n_cols):
        t_ptr[j + 1] = t_ptr[j] + counts[j]
    fill = list(t_ptr[:-1])
    t_idx = [0] * len(col_idx)
    t_vals = [None] * len(col_idx)
    for i in range(n_rows):                       # ascending i => ascending within new rows
        for k in range(int(row_ptr[i]), int(row_ptr[i + 1])):
            j = int(col_idx[k])
            t_idx[fill[j]] = i
            t_vals[fill[j]] = vals[k]
            fill[j] += 1
    return t_ptr, t_idx, t_vals


def spmv_t(n_rows, n_cols, row_ptr, col_idx, vals, x, p, mode):
    """y = A^T x  defined as the product with the explicit transpose (same mode)."""
    t_ptr, t_idx, t_vals = transpose(n_rows, n_cols, row_ptr, col_idx, vals)
    return spmv(t_ptr, t_idx, t_vals, x, p, mode)


def grad_vals(row_ptr, col_idx, g, x, p, negate=False):
    """d(<g, A x>)/d a_ij = g_i * x_j, one RN per stored entry, in CSR order of A."""
    out = []
    for i in range(len(row_ptr) - 1):
        for k in range(int(row_ptr[i]), int(row_ptr[i + 1])):
            v = mul(g[i], x[int(col_idx[k])])
            out.append(v.neg() if negate else v)
    return out


def exact_row_sum_fraction(row_ptr, col_idx, vals, x, i):
    """The exact rational sum of row i (for bound checks in tests)."""
    s = Fraction(0)
    for k in range(int(row_ptr[i]), int(row_ptr[i + 1])):
        s += vals[k].to_fraction() * x[int(col_idx[k])].to_fraction()
    return s
