"""Reference dense multiple-precision matrix-vector product (TEST INFRASTRUCTURE ONLY).

The dense product the paper sets against its sparse one (Sec. 3: the same matrix stored with all
of its n x m elements, zeros included, as MPFR numbers): y = A x with, for each row i,
  SEQ   : y_i <- +0, then y_i <- RN(y_i + RN(a_ij * x_j)) for j = 0, 1, ..., m - 1 (every
          stored element, zero or not, in ascending column order);
  EXACT : y_i = RN(sum_j a_ij * x_j), the sum formed exactly, rounded once.
vals is the row-major list of the n*m elements (element (i, j) at index i*m + j).
"""
from .mpnum import add, mul, zero
from .spmv import EXACT, SEQ, exact_sum_of_products


def gemv(n_rows, n_cols, vals, x, p, mode):
    y = []
    for i in range(n_rows):
        row = vals[i * n_cols:(i + 1) * n_cols]
        if mode == SEQ:
            acc = zero(p)
            for j in range(n_cols):
                acc = add(acc, mul(row[j], x[j]))
        elif mode == EXACT:
            acc = exact_sum_of_products(list(zip(row, x)), p)
        else:
            raise ValueError("mode must be SEQ (0) or EXACT (1)")
        y.append(acc)
    return y
