"""Batched GPBiCG: many systems of uneven size, several right-hand sides each, advanced by one
set of launches.  Every solve of the batch must be bit-identical to a plain gpbicg call on its
own system (status, iteration count and every bit of x), in both accumulation modes; one member
is also pinned to the oracle."""
import numpy as np
import pytest

import synth
from oracle import codec, krylov
from tests.test_gpu_solvers import OracleSystem, consts
from tests.util import assert_bitwise

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def lib():
    import paper_1411_2377_amd as M
    return M


def banded_batch(sizes, nrhs, p, seed):
    rng = np.random.default_rng(seed)
    systems = []
    for n in sizes:
        bw = int(rng.choice(np.arange(7, 42, 2)))
        A_h = synth.banded_system(rng, int(n), bw, p)
        bs = [synth.mp_uniform(rng, int(n), p) for _ in range(nrhs)]
        systems.append((A_h, bs))
    return systems


def solve_batch_and_plain(systems, mode, maxit, rtol, atol=(0, 0), chunk=16, x0s=None):
    M = lib()
    As = [M.CSRMatrix.from_host(A_h) for A_h, _ in systems]
    bs = [[M.MPArray.from_host(b) for b in row] for _, row in systems]
    x0d = None
    if x0s is not None:
        x0d = [[M.MPArray.from_host(x) for x in row] for row in x0s]
    xs, infos = M.gpbicg_batched(As, bs, mode=mode, maxit=maxit, rtol=rtol, atol=atol,
                                 chunk=chunk, x0s=x0d)
    for s, (A, row) in enumerate(zip(As, bs)):
        for k, b in enumerate(row):
            x0 = x0d[s][k] if x0d is not None else None
            xp, ip = M.gpbicg(A, b, mode=mode, maxit=maxit, rtol=rtol, atol=atol, chunk=chunk,
                              x0=x0)
            got, want = infos[s][k], ip
            assert (got.status, got.iters) == (want.status, want.iters), (s, k, got, want)
            gl, gh = xs[s][k].to_numpy()
            pl, ph = xp.to_numpy()
            assert np.array_equal(gh, ph) and np.array_equal(gl, pl), \
                "system %d rhs %d: batched x differs from the plain solve" % (s, k)
    return xs, infos


@pytest.mark.parametrize("mode", [0, 1], ids=["seq", "exact"])
def test_batched_matches_plain(mode):
    # uneven sizes across tile boundaries (1, 511, 512, 513, 1500 rows)
    systems = banded_batch([40, 513, 1500, 512, 1, 511], nrhs=3, p=256, seed=11)
    xs, infos = solve_batch_and_plain(systems, mode, maxit=300, rtol=(1, -60), chunk=8)
    its = [i.iters for row in infos for i in row]
    # the 1 x 1 system is solved by the first step, after which t = 0 can end GPBiCG with a
    # tau breakdown (the plain solve does the same); every other solve converges
    assert all(i.status == krylov.CONVERGED for s, row in enumerate(infos) for i in row if s != 4), infos
    assert all(i.status in (krylov.CONVERGED, krylov.BREAKDOWN_TAU) for i in infos[4])
    assert len(set(its)) > 1  # the solves stop at different iterations


def test_batched_member_matches_oracle():
    p = 256
    systems = banded_batch([24, 70], nrhs=2, p=p, seed=12)
    rtol = (1, -60)
    xs, infos = solve_batch_and_plain(systems, 0, maxit=200, rtol=rtol)
    A_h, bs = systems[1]
    S = OracleSystem(A_h)
    c_rel, c_abs = consts(p, rtol, (0, 0))
    ref = krylov.gpbicg(S.mv(0), codec.decode(bs[1].limbs, bs[1].hdr, p), c_rel, c_abs, 200, p)
    info = infos[1][1]
    assert (info.status, info.iters) == (ref.status, ref.iters)
    xl, xh = xs[1][1].to_numpy()
    assert_bitwise(xl, xh, ref.x, p, what="batched gpbicg x")


def test_batched_edge_cases():
    """A zero right-hand side (done at setup), an iteration cap, a starting guess, p = 128 and
    p = 512, and eager launches (chunk 0)."""
    for p in (128, 512):
        systems = banded_batch([300, 5, 700], nrhs=2, p=p, seed=13)
        systems[0][1][0] = synth.mp_zeros(300, p)
        rng = np.random.default_rng(14)
        x0s = [[synth.mp_uniform(rng, A.n_rows, p) for _ in row] for A, row in systems]
        xs, infos = solve_batch_and_plain(systems, 1, maxit=6, rtol=(1, -60), chunk=0,
                                          x0s=x0s)
        statuses = {i.status for row in infos for i in row}
        assert krylov.NOT_CONVERGED in statuses
    systems = banded_batch([300, 64], nrhs=2, p=256, seed=15)
    systems[0][1][1] = synth.mp_zeros(300, 256)
    xs, infos = solve_batch_and_plain(systems, 0, maxit=50, rtol=(1, -30))
    assert (infos[0][1].status, infos[0][1].iters) == (krylov.CONVERGED, 0)


def test_batched_rejects_bad_arguments():
    M = lib()
    systems = banded_batch([10], nrhs=1, p=256, seed=16)
    A = M.CSRMatrix.from_host(systems[0][0])
    b = M.MPArray.from_host(systems[0][1][0])
    with pytest.raises(ValueError):
        M.gpbicg_batched([A], [[]])
    short = M.MPArray.from_host(synth.mp_zeros(9, 256))
    with pytest.raises(RuntimeError):
        M.gpbicg_batched([A], [[short]])
    xs, infos = M.gpbicg_batched([A], [[b]], maxit=100, rtol=(1, -60))
    assert infos[0][0].status == krylov.CONVERGED
