"""GPU parity of y = A x (SEQ and EXACT) against the oracle, bit for bit.

Sizes: the random-CSR workload in full; edge-case matrices spanning several 64-row blocks and
128-entry chunks with a ragged tail; the convection-diffusion and power-law workloads at full
size, checked on sampled rows (always including the first, last and longest rows).
"""
import random

import numpy as np
import pytest

import synth
from oracle import codec, mpnum
from oracle.mpnum import MP
from tests.util import assert_bitwise, oracle_spmv_rows

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def lib():
    import paper_1411_2377_amd as M
    return M


def run(A_host, x_host, mode):
    M = lib()
    A = M.CSRMatrix.from_host(A_host)
    x = M.MPArray.from_host(x_host)
    y = M.mpspmv_csr(A, x, mode=mode)
    assert M.mp_status() == 0
    return y.to_numpy()


def edge_problem(p, seed, n=333, m=301):
    """Rows of every kind: empty, single, short, multi-chunk (> 128 entries); stored zeros,
    -0 entries, exponent spreads from 0 to ~2000 bits (the widest rows need the block-shared
    window), exact cancellations leaving a tiny remainder, all-ones mantissas."""
    rng = random.Random(seed)

    def rnd(e_lo, e_hi):
        return MP(rng.randint(0, 1), rng.getrandbits(p) | (1 << (p - 1)), rng.randint(e_lo, e_hi), p)
    x = []
    for j in range(m):
        r = rng.random()
        if j < 40 and j % 2 == 1:
            x.append(x[j - 1])                      # equal pairs for exact cancellations
        elif r < 0.05:
            x.append(mpnum.zero(p, rng.randint(0, 1)))
        elif r < 0.1:
            x.append(MP(rng.randint(0, 1), (1 << p) - 1, rng.randint(-5, 5), p))
        else:
            x.append(rnd(-20, 20))
    rp, ci, vals = [0], [], []
    for i in range(n):
        kind = i % 11
        row = {}
        if kind == 9:
            for t in rng.sample(range(20), 4):      # a x_2t - a x_2t+1 = 0 exactly
                v = rnd(-3, 3)
                row[2 * t] = v
                row[2 * t + 1] = v.neg()
            row[rng.randrange(40, m)] = rnd(-150, -100)
        else:
            k = {0: 0, 1: 1, 2: rng.randint(129, 300)}.get(kind, rng.randint(2, 24))
            spread = {3: 0, 4: 3, 5: 40, 6: 200, 7: 1000, 8: 2000}.get(kind, 10)
            for c in rng.sample(range(m), min(k, m)):
                if rng.random() < 0.08:
                    row[c] = mpnum.zero(p, rng.randint(0, 1))
                else:
                    row[c] = rnd(-spread, spread) if spread else rnd(0, 0)
        for c in sorted(row):
            ci.append(c)
            vals.append(row[c])
        rp.append(len(ci))
    vl, vh = codec.encode(vals, p)
    xl, xh = codec.encode(x, p)
    A = synth.CSRHost(n, m, np.array(rp, np.int32), np.array(ci, np.int32), synth.MPHost(vl, vh, p))
    return A, synth.MPHost(xl, xh, p)


@pytest.mark.parametrize("mode", [0, 1], ids=["seq", "exact"])
def test_random_csr_workload_full(mode):
    A, x = synth.config1()
    yl, yh = run(A, x, mode)
    want = oracle_spmv_rows(A, x, np.arange(A.n_rows), mode)
    assert_bitwise(yl, yh, want, A.vals.p, what="config1")


@pytest.mark.parametrize("p", [128, 256, 512, 1024])
@pytest.mark.parametrize("mode", [0, 1], ids=["seq", "exact"])
def test_edge_cases(p, mode):
    A, x = edge_problem(p, seed=p + mode)
    yl, yh = run(A, x, mode)
    want = oracle_spmv_rows(A, x, np.arange(A.n_rows), mode)
    assert_bitwise(yl, yh, want, p, what="edge p=%d" % p)


@pytest.mark.parametrize("mode", [0, 1], ids=["seq", "exact"])
def test_convdiff_full_size_sampled(mode):
    A, ones = synth.config2()
    rng = np.random.default_rng(0)
    x = synth.mp_uniform(rng, A.n_cols, A.vals.p)
    yl, yh = run(A, x, mode)
    rows = np.unique(np.concatenate([[0, 1, 255, 256, A.n_rows - 1], rng.integers(0, A.n_rows, 300)]))
    want = oracle_spmv_rows(A, x, rows, mode)
    assert_bitwise(yl, yh, want, A.vals.p, rows=rows, what="config2")
    # A * ones in EXACT mode as the solver right-hand side: spot rows again
    yl1, yh1 = run(A, ones, 1)
    want1 = oracle_spmv_rows(A, ones, rows, 1)
    assert_bitwise(yl1, yh1, want1, A.vals.p, rows=rows, what="config2 A*1")


@pytest.mark.parametrize("p", [128, 256, 512])
@pytest.mark.parametrize("mode", [0, 1], ids=["seq", "exact"])
def test_powerlaw_full_size_sampled(p, mode):
    """The power-law workload (n = 500000) with the default variant and with the tuned plan
    (the benchmark's configuration): sampled rows, including the longest, against the oracle."""
    A, x, g = synth.config3(p=p)
    yl, yh = run(A, x, mode)
    M = lib()
    Ad = M.CSRMatrix.from_host(A)
    P = M.mp_plan_create(Ad)
    P.tune(reps=1)
    yt = M.mpspmv_csr(Ad, M.MPArray.from_host(x), mode=mode, plan=P).to_numpy()
    assert M.mp_status() == 0
    assert np.array_equal(yt[0], yl) and np.array_equal(yt[1], yh), "tuned variant differs"
    lengths = np.diff(A.row_ptr)
    rng = np.random.default_rng(p)
    rows = np.unique(np.concatenate([[0, A.n_rows - 1, int(np.argmax(lengths))],
                                     np.argsort(lengths)[-5:], rng.integers(0, A.n_rows, 60)]))
    want = oracle_spmv_rows(A, x, rows, mode)
    assert_bitwise(yl, yh, want, p, rows=rows, what="config3 p=%d" % p)


def test_deterministic_and_invariants():
    M = lib()
    A_h, x_h = synth.config1(p=256)
    A = M.CSRMatrix.from_host(A_h)
    x = M.MPArray.from_host(x_h)
    for mode in (0, 1):
        y1 = M.mpspmv_csr(A, x, mode=mode).to_numpy()
        y2 = M.mpspmv_csr(A, x, mode=mode).to_numpy()
        assert np.array_equal(y1[0], y2[0]) and np.array_equal(y1[1], y2[1])
        # x = 0 (with -0 entries) gives +0 everywhere
        z = M.MPArray.zeros(A.n_cols, 256)
        z.hdr[1::2] = -(1 << 31) + 1
        yz = M.mpspmv_csr(A, z, mode=mode).to_numpy()
        assert np.all(yz[1] == np.int32(-(1 << 31)))
        # scaling x by 2^k scales y by 2^k exactly
        xs = x.clone()
        nz = (xs.hdr >> 1) != -(1 << 30)
        xs.hdr[nz] += 2 * 7
        ys = M.mpspmv_csr(A, xs, mode=mode).to_numpy()
        nzy = (y1[1] >> 1) != -(1 << 30)
        assert np.array_equal(ys[0], y1[0])
        assert np.array_equal(ys[1][nzy], y1[1][nzy] + 14)


def test_empty_shapes():
    M = lib()
    p = 128
    # nnz = 0 with rows: y = +0
    A = M.CSRMatrix(5, 3, torch.zeros(6, dtype=torch.int32, device="cuda"),
                    torch.zeros(0, dtype=torch.int32, device="cuda"), M.MPArray.empty(0, p))
    x = M.MPArray.zeros(3, p)
    y = M.mpspmv_csr(A, x, mode=1).to_numpy()
    assert np.all(y[1] == np.int32(-(1 << 31)))
    y = M.mpspmv_csr(A, x, mode=0).to_numpy()
    assert np.all(y[1] == np.int32(-(1 << 31)))
    # zero rows: nothing to do
    A0 = M.CSRMatrix(0, 3, torch.zeros(1, dtype=torch.int32, device="cuda"),
                     torch.zeros(0, dtype=torch.int32, device="cuda"), M.MPArray.empty(0, p))
    M.mpspmv_csr(A0, x, mode=0)
    torch.cuda.synchronize()


@pytest.mark.parametrize("p", [128, 256, 512, 1024])
def test_every_kernel_variant_same_bits(p):
    """Each rows-per-block variant of y = A x and y = A^T x, in both modes, matches the oracle
    bit for bit (edge-case matrix), and the tuner's pick changes nothing."""
    from tests.util import decode_vec
    from oracle import spmv as ospmv
    M = lib()
    A_h, x_h = edge_problem(p, seed=7 * p)
    A = M.CSRMatrix.from_host(A_h)
    x = M.MPArray.from_host(x_h)
    rng = np.random.default_rng(p)
    g_h = synth.mp_uniform(rng, A_h.n_rows, p)
    g = M.MPArray.from_host(g_h)
    P = M.mp_plan_create(A)
    vals = codec.decode(A_h.vals.limbs, A_h.vals.hdr, p)
    tp, ti, tv = ospmv.transpose(A_h.n_rows, A_h.n_cols, A_h.row_ptr.tolist(), A_h.col_idx.tolist(), vals)
    go = decode_vec(g_h)
    for mode in (0, 1):
        want = oracle_spmv_rows(A_h, x_h, np.arange(A_h.n_rows), mode)
        want_t = ospmv.spmv(tp, ti, tv, go, p, mode)
        combos = [(False, False, 0, 0), (True, False, 0, 0), (False, True, 0, 0), (True, True, 0, 0)]
        if mode == 0:   # lane groups / windowed chains (a row or four rows per wavefront) for
            # every non-empty row, rows of >= 2 and of >= 200
            combos += [(s, True, g, w) for w in (0, 1, 2) for s, g in ((False, 1), (True, 2), (True, 200))]
        kinds = ("lane groups", "windows", "segmented windows")
        for rows in (16, 32, 64):
            for stage, srt, gmin, win in combos:
                P.set_variant(0, mode, rows, stage, srt, gmin, win == 1, win == 2)
                P.set_variant(1, mode, rows, stage, srt, gmin, win == 1, win == 2)
                tag = "%d rows per block, staged x %s, sorted rows %s, %s from %d, mode %d" % (
                    rows, stage, srt, kinds[win], gmin, mode)
                yl, yh = M.mpspmv_csr(A, x, mode=mode, plan=P).to_numpy()
                assert_bitwise(yl, yh, want, p, what="A x, " + tag)
                tl, th = M.mpspmv_csr_t(A, P, g, mode=mode).to_numpy()
                assert_bitwise(tl, th, want_t, p, what="A^T g, " + tag)
    for kw in ({}, {"x": x, "x_t": g}):   # generated operands, then the products' own
        picks = P.tune(reps=1, **kw)
        assert {v[0] for v in picks.values()} <= {16, 32, 64}
        assert all(v[3] == 0 for (op, m), v in picks.items() if m == 1)   # lane groups: SEQ only
        for mode in (0, 1):
            yl, yh = M.mpspmv_csr(A, x, mode=mode, plan=P).to_numpy()
            want = oracle_spmv_rows(A_h, x_h, np.arange(A_h.n_rows), mode)
            assert_bitwise(yl, yh, want, p, what="tuned A x mode %d %s" % (mode, list(kw)))
    assert M.mp_status() == 0


def corner_rows(p, seed):
    """Rows whose SEQ partial sums hit the corners of RN addition (x = 1, so the products are
    the stored values): ties to even, the all-ones mantissa rounding up to a power of two,
    cancellations of one, several and p bits, exact zeros, signed zeros, operands far apart,
    and runs of values within a few binades of each other with mixed signs (differences of
    exponents 0, 1 and 2 between partial sum and term)."""
    rng = random.Random(seed)
    one = MP(0, 1 << (p - 1), 1, p)

    def pw(k, s=0):          # (-1)^s 2^k
        return MP(s, 1 << (p - 1), k + 1, p)

    def rnd(lo, hi, s=None):
        return MP(rng.randint(0, 1) if s is None else s, rng.getrandbits(p) | (1 << (p - 1)),
                  rng.randint(lo, hi), p)
    allones = MP(0, (1 << p) - 1, 0, p)                     # 1 - 2^-p
    rows = [
        [one, pw(-p), pw(-p)],                                # two ties to even: 1
        [MP(0, (1 << (p - 1)) | 1, 1, p), pw(-p)],            # 1 + 2^(1-p) + 2^-p: tie up
        [allones, pw(-p - 1)],                                # carries into a new binade
        [one, allones.neg()],                                 # cancellation of p bits
        [one, one.neg()],                                     # exact zero: +0
        [mpnum.zero(p, 1), mpnum.zero(p, 1)],                 # (-0) + (-0)
        [pw(100), one, pw(100, 1)],                           # large cancellation leaves 1
        [one, pw(-3000)],                                     # far apart
        [pw(-3000), one],
        [rnd(-2, 2) for _ in range(40)],
        [rnd(0, 2) for _ in range(300)],
        [rnd(-1, 1, 0) for _ in range(150)] + [rnd(-1, 1, 1) for _ in range(150)],
        [allones] * 64 + [allones.neg()] * 63,
        [rnd(-400, 400) for _ in range(257)],
    ]
    for _ in range(40):
        k = rng.randint(1, 90)
        rows.append([rnd(-3, 3) if rng.random() < 0.8 else mpnum.zero(p, rng.randint(0, 1))
                     for _ in range(k)])
    m = max(len(r) for r in rows)
    rp, ci, vals = [0], [], []
    for r in rows:
        ci.extend(range(len(r)))
        vals.extend(r)
        rp.append(len(ci))
    vl, vh = codec.encode(vals, p)
    xl, xh = codec.encode([one] * m, p)
    A = synth.CSRHost(len(rows), m, np.array(rp, np.int32), np.array(ci, np.int32), synth.MPHost(vl, vh, p))
    return A, synth.MPHost(xl, xh, p)


@pytest.mark.parametrize("p", [128, 256, 512, 1024])
def test_lane_group_rows_corner_sums(p):
    """Every row summed by lane groups (SEQ, sorted rows, rows of >= 1 entry), by windowed
    chains and by the one-lane chains: all equal the oracle bit for bit on the corner-case rows
    (whose ties, binade changes, cancellations and zeros are the windows' exception steps)."""
    M = lib()
    A_h, x_h = corner_rows(p, seed=p)
    A = M.CSRMatrix.from_host(A_h)
    x = M.MPArray.from_host(x_h)
    want = oracle_spmv_rows(A_h, x_h, np.arange(A_h.n_rows), 0)
    P = M.mp_plan_create(A)
    for rows, stage, gmin, win in ((16, False, 1, 0), (64, True, 1, 0), (32, False, 0, 0),
                                   (16, True, 1, 1), (64, False, 2, 1), (32, True, 1, 2), (16, False, 3, 2)):
        P.set_variant(0, 0, rows, stage, True, gmin, win == 1, win == 2)
        yl, yh = M.mpspmv_csr(A, x, mode=0, plan=P).to_numpy()
        assert_bitwise(yl, yh, want, p, what="corner rows, %s from %d" % (
            ("lane groups", "windows", "segmented windows")[win], gmin))
    assert M.mp_status() == 0


@pytest.mark.parametrize("p", [128, 256, 512])
@pytest.mark.parametrize("win", [0, 1, 2], ids=["groups", "windows", "segments"])
def test_powerlaw_lane_groups_sampled(p, win):
    """The power-law workload at full size with the longest rows summed by lane groups or by
    windowed chains (rows of >= 64 entries): sampled rows, always including the longest ones,
    equal the oracle."""
    M = lib()
    A_h, x_h, _ = synth.config3(p=p)
    A = M.CSRMatrix.from_host(A_h)
    x = M.MPArray.from_host(x_h)
    P = M.mp_plan_create(A)
    P.set_variant(0, 0, 16, True, True, 64, win == 1, win == 2)
    yl, yh = M.mpspmv_csr(A, x, mode=0, plan=P).to_numpy()
    lengths = np.diff(A_h.row_ptr)
    order = np.argsort(-lengths, kind="stable")
    rng = np.random.default_rng(p)
    rows = np.unique(np.concatenate([order[:6], order[np.sum(lengths >= 64) - 3:np.sum(lengths >= 64) + 3],
                                     rng.integers(0, A_h.n_rows, 40)]))
    want = oracle_spmv_rows(A_h, x_h, rows, 0)
    assert_bitwise(yl[:, rows], yh[rows], want, p, what="power-law rows by lane groups")
    assert M.mp_status() == 0


def wide_span_problem(p, seed):
    """EXACT rows whose products span far more bits than a block's LDS window: 48 rows of 8-60
    entries with exponents spread over +-60,000 bits (enough rows to contend for the global
    windows), rows whose largest products cancel exactly leaving terms 100,000 bits below them
    (positive and negative remainders), a row that cancels to exactly zero, and ordinary rows."""
    rng = np.random.default_rng(seed)
    m = 300
    x = synth.mp_uniform(rng, m, p)
    x.limbs[:, 1] = x.limbs[:, 0]          # x_0 == x_1: a_0 x_0 + (-a_0) x_1 cancels exactly
    x.hdr[1] = x.hdr[0]
    rows = []                              # (columns, exponents, signs); mantissas random
    for _ in range(48):
        k = int(rng.integers(8, 61))
        cols = np.sort(rng.choice(np.arange(2, m), size=k, replace=False))
        rows.append((cols, rng.integers(-60000, 60001, size=k), rng.integers(0, 2, size=k)))
    for sign_small in (0, 1):              # big cancelling pair, remainder 100,000 bits down
        cols = np.array([0, 1] + sorted(rng.choice(np.arange(2, m), size=5, replace=False).tolist()))
        exps = np.array([50000, 50000] + rng.integers(-50020, -49980, size=5).tolist())
        signs = np.array([0, 1] + [sign_small] * 5)
        rows.append((cols, exps, signs))
    rows.append((np.array([0, 1]), np.array([70000, 70000]), np.array([1, 0])))   # exactly zero
    for _ in range(8):                     # ordinary rows around them
        k = int(rng.integers(1, 20))
        cols = np.sort(rng.choice(np.arange(2, m), size=k, replace=False))
        rows.append((cols, rng.integers(-20, 21, size=k), rng.integers(0, 2, size=k)))
    rp = np.zeros(len(rows) + 1, np.int64)
    rp[1:] = np.cumsum([len(r[0]) for r in rows])
    nnz = int(rp[-1])
    vals = synth.mp_uniform(rng, nnz, p)
    exps = np.concatenate([r[1] for r in rows]).astype(np.int64)
    signs = np.concatenate([r[2] for r in rows]).astype(np.int64)
    vals.hdr[:] = ((exps << 1) | signs).astype(np.int32)
    # the cancelling pairs share one mantissa (and x_0 == x_1), so their products are negatives
    for i, r in enumerate(rows):
        if len(r[0]) >= 2 and r[0][0] == 0 and r[0][1] == 1:
            k0 = int(rp[i])
            vals.limbs[:, k0 + 1] = vals.limbs[:, k0]
    cols = np.concatenate([r[0] for r in rows]).astype(np.int32)
    A = synth.CSRHost(len(rows), m, rp.astype(np.int32), cols, vals)
    return A, x


@pytest.mark.parametrize("p", [128, 256, 1024])
def test_exact_rows_wider_than_lds_window(p):
    """Rows spanning up to ~120,000 bits (global-memory windows taken under locks) equal the
    oracle's exactly rounded sums, with no status raised; default and tuned variants."""
    M = lib()
    A_h, x_h = wide_span_problem(p, seed=p)
    want = oracle_spmv_rows(A_h, x_h, np.arange(A_h.n_rows), 1)
    yl, yh = run(A_h, x_h, 1)
    assert_bitwise(yl, yh, want, p, what="wide EXACT rows p=%d" % p)
    assert yh[48 + 2] == np.int32(-(1 << 31))          # the cancelling row is +0
    A = M.CSRMatrix.from_host(A_h)
    P = M.mp_plan_create(A)
    for rows in (16, 64):
        P.set_variant(0, 1, rows, True, False)
        yl2, yh2 = M.mpspmv_csr(A, M.MPArray.from_host(x_h), mode=1, plan=P).to_numpy()
        assert np.array_equal(yl2, yl) and np.array_equal(yh2, yh)
    assert M.mp_status() == 0
