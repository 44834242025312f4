"""Seeded synthetic inputs for the multiple-precision SpMV / Krylov path.

This module only *constructs* inputs in the storage format; it contains none of the method's
arithmetic (no rounding, no products, no sums of MP values).  Values are built directly from
random bits, or as exact short integers, or as the p-bit truncation (chop toward zero) of an
exact rational or of a double, which is an integer floor, not the round-to-nearest of the method.
Both the GPU path (tests, benchmark) and the oracle read the arrays produced here.

Storage of an MP array of N numbers at p = 32*L bits (structure of arrays):
  limbs uint32[L, N] (plane k = limb k of every mantissa, k = 0 least significant)
  hdr   int32[N]     (e << 1) | s, value = (-1)^s * M * 2^(e-p), 2^(p-1) <= M < 2^p;
                     a zero has e = -2^30 (hdr = INT32_MIN for +0, INT32_MIN + 1 for -0).
Sparse matrices are CSR: row_ptr int32[n+1], col_idx int32[nnz] strictly ascending per row.
"""
from dataclasses import dataclass
import math

import numpy as np

ZERO_E = -(1 << 30)
ZERO_HDR = np.int32(-(1 << 31))


@dataclass
class MPHost:
    limbs: np.ndarray   # uint32 [L, N]
    hdr: np.ndarray     # int32 [N]
    p: int

    @property
    def n(self):
        return int(self.hdr.shape[0])

    def take(self, idx):
        idx = np.asarray(idx)
        return MPHost(np.ascontiguousarray(self.limbs[:, idx]), self.hdr[idx].copy(), self.p)


@dataclass
class CSRHost:
    n_rows: int
    n_cols: int
    row_ptr: np.ndarray  # int32 [n+1]
    col_idx: np.ndarray  # int32 [nnz]
    vals: MPHost

    @property
    def nnz(self):
        return int(self.col_idx.shape[0])


# ---------------------------------------------------------------------------------------
# value constructors
# ---------------------------------------------------------------------------------------
def _hdr(e, s):
    e = np.asarray(e, dtype=np.int64)
    s = np.asarray(s, dtype=np.int64)
    return ((e << 1) | s).astype(np.int32)


def mp_zeros(n, p):
    return MPHost(np.zeros((p // 32, n), np.uint32), np.full(n, ZERO_HDR, np.int32), p)


def mp_uniform(rng, n, p, signed=True):
    """Uniform on [-1, 1] (or [0, 1)) truncated to p bits: P(value in [2^-k-1, 2^-k)) = 2^-k-1,
    uniform random mantissa bits below a leading one."""
    nl = p // 32
    limbs = rng.integers(0, 1 << 32, size=(nl, n), dtype=np.uint64).astype(np.uint32)
    limbs[nl - 1] |= np.uint32(0x80000000)
    e = 1 - rng.geometric(0.5, size=n).astype(np.int64)      # value in [2^(e-1), 2^e), e <= 0
    s = rng.integers(0, 2, size=n) if signed else np.zeros(n, np.int64)
    return MPHost(limbs, _hdr(e, s), p)


def mp_loguniform(rng, n, p, dec_lo, dec_hi, signed=True):
    """|v| = 10^U, U ~ U(dec_lo, dec_hi): exponent and the leading 53 mantissa bits come from the
    double 2^(U log2 10); the remaining p-53 bits are random."""
    nl = p // 32
    t = rng.uniform(dec_lo, dec_hi, size=n) * math.log2(10.0)
    fl = np.floor(t)
    lead = np.floor(np.exp2(t - fl) * 2.0 ** 52).astype(np.uint64)     # in [2^52, 2^53)
    lead = np.clip(lead, np.uint64(1 << 52), np.uint64((1 << 53) - 1))
    e = fl.astype(np.int64) + 1
    limbs = rng.integers(0, 1 << 32, size=(nl, n), dtype=np.uint64).astype(np.uint32)
    # place the 53 leading bits at the top: bits [p-53, p) = lead
    limbs[nl - 1] = (lead >> np.uint64(21)).astype(np.uint32)
    mid = (lead & np.uint64((1 << 21) - 1)) << np.uint64(11)
    limbs[nl - 2] = (mid.astype(np.uint32)) | (limbs[nl - 2] & np.uint32((1 << 11) - 1))
    s = rng.integers(0, 2, size=n) if signed else np.zeros(n, np.int64)
    return MPHost(limbs, _hdr(e, s), p)


def _enc_int(m, e, s, p, limbs, hdr, i):
    """Store one number with an already normalised p-bit integer mantissa m."""
    nl = p // 32
    if m == 0:
        hdr[i] = (ZERO_E << 1) | s
        for k in range(nl):
            limbs[k, i] = 0
        return
    assert (1 << (p - 1)) <= m < (1 << p)
    hdr[i] = (e << 1) | s
    for k in range(nl):
        limbs[k, i] = (m >> (32 * k)) & 0xFFFFFFFF


def chop_rational(num, den, p):
    """(s, M, e) of the p-bit truncation toward zero of num/den (integers, den > 0)."""
    if num == 0:
        return 0, 0, 0
    s = 1 if num < 0 else 0
    a = abs(num)
    e = a.bit_length() - den.bit_length()
    while (a << max(0, -e)) >= (den << max(0, e)):
        e += 1
    while (a << max(0, -(e - 1))) < (den << max(0, e - 1)):
        e -= 1
    # a/den in [2^(e-1), 2^e): M = floor(a/den * 2^(p-e))
    sh = p - e
    m = (a << sh) // den if sh >= 0 else a // (den << (-sh))
    return s, m, e


def mp_from_rationals(pairs, p):
    """Each (num, den) chopped to p bits."""
    n = len(pairs)
    limbs = np.zeros((p // 32, n), np.uint32)
    hdr = np.zeros(n, np.int32)
    for i, (num, den) in enumerate(pairs):
        s, m, e = chop_rational(int(num), int(den), p)
        _enc_int(m, e, s, p, limbs, hdr, i)
    return MPHost(limbs, hdr, p)


def mp_from_ints(vals, p):
    """Exact small integers (|v| < 2^p)."""
    vals = [int(v) for v in vals]
    n = len(vals)
    limbs = np.zeros((p // 32, n), np.uint32)
    hdr = np.zeros(n, np.int32)
    for i, v in enumerate(vals):
        s = 1 if v < 0 else 0
        a = abs(v)
        if a == 0:
            _enc_int(0, 0, s, p, limbs, hdr, i)
            continue
        nb = a.bit_length()
        _enc_int(a << (p - nb), nb, s, p, limbs, hdr, i)
    return MPHost(limbs, hdr, p)


def mp_arange1(n, p):
    """[1, 2, ..., n] exactly."""
    nl = p // 32
    k = np.arange(1, n + 1, dtype=np.int64)
    nb = np.floor(np.log2(k)).astype(np.int64) + 1
    # k < 2^31: mantissa = k << (p - nb); only the top limb (and the next) are non-zero
    limbs = np.zeros((nl, n), np.uint32)
    top = (k << (32 - nb)).astype(np.uint64)      # fits in 32 bits
    limbs[nl - 1] = top.astype(np.uint32)
    return MPHost(limbs, _hdr(nb, np.zeros(n, np.int64)), p)


def mp_ones(n, p):
    limbs = np.zeros((p // 32, n), np.uint32)
    limbs[p // 32 - 1] = np.uint32(0x80000000)
    return MPHost(limbs, _hdr(np.ones(n, np.int64), np.zeros(n, np.int64)), p)


def mp_concat(parts):
    p = parts[0].p
    return MPHost(np.concatenate([q.limbs for q in parts], axis=1),
                  np.concatenate([q.hdr for q in parts]), p)


# ---------------------------------------------------------------------------------------
# sparsity structures
# ---------------------------------------------------------------------------------------
def _rows_from_lengths(lengths):
    rp = np.zeros(len(lengths) + 1, np.int64)
    np.cumsum(lengths, out=rp[1:])
    return rp


def _distinct_sorted_columns(rng, lengths, n_cols):
    """Per row, `lengths[i]` distinct columns drawn uniformly without replacement, ascending."""
    lengths = np.asarray(lengths, np.int64)
    nnz = int(lengths.sum())
    row_of = np.repeat(np.arange(len(lengths), dtype=np.int64), lengths)
    cols = rng.integers(0, n_cols, size=nnz, dtype=np.int64)
    while True:
        order = np.lexsort((cols, row_of))
        cols = cols[order]
        dup = np.zeros(nnz, bool)
        dup[1:] = (cols[1:] == cols[:-1]) & (row_of[1:] == row_of[:-1])
        nd = int(dup.sum())
        if nd == 0:
            return cols
        cols[dup] = rng.integers(0, n_cols, size=nd, dtype=np.int64)


def csr_uniform(rng, n, per_row, p, vals_fn):
    lengths = np.full(n, per_row, np.int64)
    rp = _rows_from_lengths(lengths)
    cols = _distinct_sorted_columns(rng, lengths, n)
    return CSRHost(n, n, rp.astype(np.int32), cols.astype(np.int32), vals_fn(len(cols)))


def powerlaw_gamma(mean, kmax):
    """Exponent gamma of P(k) ~ k^-gamma on [1, kmax] with the given mean (bisection)."""
    k = np.arange(1, kmax + 1, dtype=np.float64)

    def m(g):
        w = k ** (-g)
        return float((w * k).sum() / w.sum())
    lo, hi = 0.5, 4.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if m(mid) > mean:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def powerlaw_lengths(rng, n, mean, kmax):
    g = powerlaw_gamma(mean, kmax)
    k = np.arange(1, kmax + 1, dtype=np.float64)
    w = k ** (-g)
    w /= w.sum()
    lengths = rng.choice(np.arange(1, kmax + 1), size=n, p=w).astype(np.int64)
    lengths[int(np.argmax(lengths))] = kmax
    return lengths


def stencil2d_pattern(m):
    """5-point stencil on an m x m grid in lexicographic order: (rows, cols, kind) with kind
    0 = centre, 1 = west, 2 = east, 3 = south, 4 = north; columns ascending in each row."""
    rows, cols, kind = [], [], []
    for gy in range(m):
        for gx in range(m):
            i = gy * m + gx
            ent = []
            if gy > 0:
                ent.append((i - m, 3))
            if gx > 0:
                ent.append((i - 1, 1))
            ent.append((i, 0))
            if gx < m - 1:
                ent.append((i + 1, 2))
            if gy < m - 1:
                ent.append((i + m, 4))
            for c, kd in ent:
                rows.append(i)
                cols.append(c)
                kind.append(kd)
    return np.array(rows, np.int64), np.array(cols, np.int64), np.array(kind, np.int64)


def stencil3d_pattern(m):
    """7-point stencil on an m^3 grid, lexicographic (x fastest); kind 0 centre, 1/2 -x/+x,
    3/4 -y/+y, 5/6 -z/+z; columns ascending in each row."""
    n = m ** 3
    idx = np.arange(n, dtype=np.int64)
    gx = idx % m
    gy = (idx // m) % m
    gz = idx // (m * m)
    offs = [(-m * m, gz > 0, 5), (-m, gy > 0, 3), (-1, gx > 0, 1), (0, np.ones(n, bool), 0),
            (1, gx < m - 1, 2), (m, gy < m - 1, 4), (m * m, gz < m - 1, 6)]
    R, C, K = [], [], []
    for off, ok, kd in offs:
        R.append(idx[ok])
        C.append(idx[ok] + off)
        K.append(np.full(int(ok.sum()), kd, np.int64))
    R = np.concatenate(R)
    C = np.concatenate(C)
    K = np.concatenate(K)
    order = np.lexsort((C, R))
    return R[order], C[order], K[order]


def _csr_from_coo_sorted(n, rows, cols):
    counts = np.bincount(rows, minlength=n)
    rp = _rows_from_lengths(counts)
    return rp.astype(np.int32), cols.astype(np.int32)


# ---------------------------------------------------------------------------------------
# the workloads
# ---------------------------------------------------------------------------------------
def config1(p=128, seed=1, n=1000, per_row=10):
    """Random CSR, n = 1000, 10 distinct uniformly placed columns per row, values and x
    uniform on [-1, 1] at p bits."""
    rng = np.random.default_rng(seed)
    A = csr_uniform(rng, n, per_row, p, lambda k: mp_uniform(rng, k, p))
    x = mp_uniform(rng, n, p)
    return A, x


def convdiff2d(m, p, peclet=10):
    """Nonsymmetric 2-D convection-diffusion, 5-point central differences on an m x m interior
    grid, h = 1/(m+1), convection (1, 1) * peclet: centre 4, west/south -1 - c, east/north
    -1 + c with c = peclet*h/2 = peclet/(2(m+1)); each coefficient chopped to p bits."""
    rows, cols, kind = stencil2d_pattern(m)
    den = 2 * (m + 1)
    coef = {0: (4, 1), 1: (-(den + peclet), den), 3: (-(den + peclet), den),
            2: (-(den - peclet), den), 4: (-(den - peclet), den)}
    table = mp_from_rationals([coef[k] for k in range(5)], p)
    vals = table.take(kind)
    rp, ci = _csr_from_coo_sorted(m * m, rows, cols)
    return CSRHost(m * m, m * m, rp, ci, vals)


def config2(p=256, m=256, peclet=10):
    """256 x 256 grid (n = 65536), p = 256; right-hand side is A * ones (formed by the solver
    side in EXACT mode), x0 = 0."""
    A = convdiff2d(m, p, peclet)
    return A, mp_ones(A.n_rows, p)


def config3(p=256, seed=3, n=500000, mean=20, kmax=2000):
    """Power-law row lengths (mean 20, max 2000), uniform distinct columns, |a| = 10^U with
    U ~ U(-8, 8) and random sign; x and the output cotangent g uniform on [-1, 1]."""
    rng = np.random.default_rng(seed)
    lengths = powerlaw_lengths(rng, n, mean, kmax)
    rp = _rows_from_lengths(lengths)
    cols = _distinct_sorted_columns(rng, lengths, n)
    vals = mp_loguniform(rng, len(cols), p, -8.0, 8.0)
    A = CSRHost(n, n, rp.astype(np.int32), cols.astype(np.int32), vals)
    x = mp_uniform(rng, n, p)
    g = mp_uniform(rng, n, p)
    return A, x, g


def banded_system(rng, n, bw, p):
    """Banded nonsymmetric matrix with bw diagonals (half-bandwidth (bw-1)/2): off-diagonals
    uniform on [-1, 1], diagonal a random value in [2^c, 2^(c+1)) with 2^c >= bw, which is
    larger than the sum of the off-diagonal magnitudes (strict diagonal dominance)."""
    h = (bw - 1) // 2
    i = np.arange(n, dtype=np.int64)
    R, C = [], []
    for off in range(-h, h + 1):
        ok = (i + off >= 0) & (i + off < n)
        R.append(i[ok])
        C.append(i[ok] + off)
    R = np.concatenate(R)
    C = np.concatenate(C)
    order = np.lexsort((C, R))
    R, C = R[order], C[order]
    vals = mp_uniform(rng, len(R), p)
    diag = np.nonzero(R == C)[0]
    c = int(math.ceil(math.log2(bw)))
    dv = mp_uniform(rng, len(diag), p, signed=False)
    dv.hdr[:] = _hdr(np.full(len(diag), c + 1, np.int64), np.zeros(len(diag), np.int64))
    vals.limbs[:, diag] = dv.limbs
    vals.hdr[diag] = dv.hdr
    rp, ci = _csr_from_coo_sorted(n, R, C)
    return CSRHost(n, n, rp, ci, vals)


def config4(p=256, seed=4, nsys=64, nrhs=16, n_lo=1000, n_hi=100000):
    """64 banded systems, n_k = round(n_lo * (n_hi/n_lo)^(k/(nsys-1))) in shuffled order,
    bandwidths from {7, 9, ..., 41}; per system nrhs true solutions: x*_0 = [1..n], the others
    uniform on [-1, 1] (right-hand sides b = A x* are formed by the solver side)."""
    rng = np.random.default_rng(seed)
    ks = np.arange(nsys)
    sizes = np.round(n_lo * (n_hi / n_lo) ** (ks / max(1, nsys - 1))).astype(np.int64)
    rng.shuffle(sizes)
    bws = rng.choice(np.arange(7, 42, 2), size=nsys)
    systems = []
    for n, bw in zip(sizes, bws):
        A = banded_system(rng, int(n), int(bw), p)
        xs = [mp_arange1(int(n), p)] + [mp_uniform(rng, int(n), p) for _ in range(nrhs - 1)]
        systems.append((A, xs))
    return systems


def convdiff3d_scaled(m, p, seed=5, peclet=10, dec=15.0):
    """7-point central convection-diffusion on m^3 (h = 1/(m+1), coefficients 6 and
    -1 -+ c, c = peclet/(2(m+1)), chopped to p/2 bits), left-scaled by d_i = 10^u_i,
    u_i ~ U(-dec, dec), with d_i carrying p/2 significant bits; each entry d_i * a_ij is then an
    exact product of two p/2-bit mantissas, so it is exactly representable at p bits."""
    rng = np.random.default_rng(seed)
    rows, cols, kind = stencil3d_pattern(m)
    n = m ** 3
    den = 2 * (m + 1)
    half = p // 2
    coef = {0: (6, 1)}
    for kd in (1, 3, 5):
        coef[kd] = (-(den + peclet), den)
    for kd in (2, 4, 6):
        coef[kd] = (-(den - peclet), den)
    cparts = {k: chop_rational(num, d, half) for k, (num, d) in coef.items()}
    d = mp_loguniform(rng, n, half, -dec, dec, signed=False)
    dl = d.limbs.astype(object)
    dm = [0] * n
    for k in range(d.limbs.shape[0] - 1, -1, -1):
        dm = [(a << 32) | int(b) for a, b in zip(dm, dl[k])]
    de = (d.hdr.astype(np.int64) >> 1).tolist()
    nnz = len(rows)
    limbs = np.zeros((p // 32, nnz), np.uint32)
    hdr = np.zeros(nnz, np.int32)
    for t in range(nnz):
        i = int(rows[t])
        cs, cm, ce = cparts[int(kind[t])]
        mm = dm[i] * cm                      # exact: two p/2-bit mantissas
        # value = mm * 2^(de - half) * 2^(ce - half); normalise mm to p bits exactly
        nb = mm.bit_length()
        m_norm = mm << (p - nb)
        e = de[i] + ce - 2 * half + nb
        _enc_int(m_norm, e, cs, p, limbs, hdr, t)
    rp, ci = _csr_from_coo_sorted(n, rows, cols)
    return CSRHost(n, n, rp, ci, MPHost(limbs, hdr, p))


def config5(p=512, m=64, seed=5):
    """3-D 7-point nonsymmetric operator on 64^3, row-scaled by 10^u, u ~ U(-15, 15), p = 512;
    true solution [1..n] (b = A x* formed by the solver side), adjoint right-hand side ones."""
    A = convdiff3d_scaled(m, p, seed=seed)
    return A, mp_arange1(A.n_rows, p), mp_ones(A.n_rows, p)


def lotkin(n, p, zero_pct, seed=6):
    """The Lotkin matrix of the paper's SpMV benchmark (first row all ones, a_ij = 1/(i+j-1)
    below it, 1-based), each element chopped to p bits, with round(zero_pct * n^2 / 100) of its
    n^2 elements (positions drawn with a seeded permutation) set to +0.  Returns the dense
    row-major array (n^2 elements, zeros stored), the CSR of its non-zero elements, and
    x = [1, 2, ..., n]."""
    rng = np.random.default_rng(seed)
    table = mp_from_rationals([(1, k) for k in range(1, 2 * n)], p)   # 1/k, k = 1 .. 2n-1
    i = np.arange(n, dtype=np.int64)[:, None]
    j = np.arange(n, dtype=np.int64)[None, :]
    k = np.where(i == 0, 1, i + j + 1)                                 # 1-based i + j - 1
    dense = table.take((k - 1).reshape(-1))
    nz = int(round(zero_pct * n * n / 100.0))
    zpos = rng.permutation(n * n)[:nz]
    dense.hdr[zpos] = ZERO_HDR
    dense.limbs[:, zpos] = 0
    keep = np.flatnonzero(dense.hdr != ZERO_HDR)
    rows = (keep // n).astype(np.int64)
    row_ptr = np.zeros(n + 1, np.int64)
    np.add.at(row_ptr, rows + 1, 1)
    row_ptr = np.cumsum(row_ptr).astype(np.int32)
    csr = CSRHost(n, n, row_ptr, (keep % n).astype(np.int32), dense.take(keep))
    return dense, csr, mp_arange1(n, p)
