"""Reference vector operations (TEST INFRASTRUCTURE ONLY).

These are the non-SpMV lines of the paper's BiCG/GPBiCG listings (Fig. 5): scaled vector
updates, inner products and the residual norm.  One RN per binary operation; inner products
are formed exactly and rounded once.
"""
from .mpnum import add, mul, sqrt, sub
from .spmv import exact_sum_of_products


def axpy(alpha, x, y):
    """y_i + alpha * x_i  (RN after the multiply and after the add)."""
    return [add(yi, mul(alpha, xi)) for xi, yi in zip(x, y)]


def aymx(alpha, x, y):
    """y_i - alpha * x_i."""
    return [sub(yi, mul(alpha, xi)) for xi, yi in zip(x, y)]


def xpby(x, beta, y):
    """x_i + beta * y_i."""
    return [add(xi, mul(beta, yi)) for xi, yi in zip(x, y)]


def dot(x, y, p):
    """RN(sum_i x_i * y_i), the sum formed exactly."""
    return exact_sum_of_products(list(zip(x, y)), p)


def nrm2(x, p):
    """RN(sqrt(dot(x, x)))."""
    return sqrt(dot(x, x, p))
