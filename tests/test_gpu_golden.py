"""Long runs at full size against stored expected values that only the oracle wrote
(tests/golden/make_golden.py, from the seeded inputs of synth/): every iterate is deterministic,
so status, iteration count, every residual-history entry and every bit of x must agree.

  * 2-D convection-diffusion 256 x 256, p = 256: 200 iterations of BiCG, GPBiCG, CGS and
    BiCGSTAB in SEQ and EXACT mode (the benchmark's solver runs, tuned plan, graph chunks of 25);
  * row-scaled 3-D operator 64^3, p = 512: the first 20 BiCG and GPBiCG iterations (EXACT);
  * the banded batch: its two smallest systems with all 16 right-hand sides (GPBiCG, SEQ, to
    1e-60), solved alone and inside the whole 64-system batch, and every member of the whole
    batch bit-identical to its plain solve;
  * the adjoint of a BiCG solve on a 16^3 row-scaled operator with decade spread 1 (x, lambda
    and the value gradient), and at full 64^3 size with the same spread the duality
    <lambda, b> = sum x (spread 1 is the widest of 0.5, 1 and 2 for which BiCG and its
    transposed solve reach 1e-100 at 64^3 and p = 512: about 6400 and 6800 iterations).
"""
import json
import os
from fractions import Fraction

import numpy as np
import pytest

import synth
from oracle import codec
from tests.util import digest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def lib():
    import paper_1411_2377_amd as M
    return M


def load(name):
    with open(os.path.join(GOLD, name + ".json")) as fh:
        return json.load(fh)


def check_run(gold, xl, xh, info, hist=None, what=""):
    """Status, iterations, residual history (first differing iteration named) and x."""
    assert (info.status, info.iters) == (gold["status"], gold["iters"]), \
        "%s: (status, iters) %s, oracle %s" % (what, (info.status, info.iters), (gold["status"], gold["iters"]))
    if hist is not None and "hist_digests" in gold:
        hl, hh = hist
        for i, want in enumerate(gold["hist_digests"]):
            got = digest(hl[:, i:i + 1], hh[i:i + 1])[:16]
            assert got == want, "%s: residual history differs first at iteration %d" % (what, i + 1)
    for idx, ent in gold.get("x_samples", {}).items():
        i = int(idx)
        assert int(xh[i]) == ent["hdr"] and [int(v) for v in xl[:, i]] == ent["limbs"], \
            "%s: x[%d] differs from the oracle's" % (what, i)
    assert digest(xl, xh) == gold["x_digest"], "%s: x differs from the oracle's" % what


@pytest.mark.parametrize("solver", ["bicg", "gpbicg", "cgs", "bicgstab"])
@pytest.mark.parametrize("mode", [0, 1], ids=["seq", "exact"])
def test_convdiff256_200_iterations(solver, mode):
    M = lib()
    gold = load("convdiff2d_256_p256_%s_%s" % (solver, "seq" if mode == 0 else "exact"))
    A_h, ones_h = synth.config2(p=256, m=256)
    A = M.CSRMatrix.from_host(A_h)
    b = M.mpspmv_csr(A, M.MPArray.from_host(ones_h), mode=M.MP_EXACT)
    assert digest(*b.to_numpy()) == gold["b_digest"], "b = A * ones differs from the oracle's"
    plan = M.mp_plan_create(A)
    plan.tune(reps=1)
    o = gold["opts"]
    fn = getattr(M, solver)
    x, info = fn(A, b, plan=plan, mode=mode, maxit=o["maxit"], rtol=tuple(o["rtol"]),
                 atol=tuple(o["atol"]), chunk=25, hist=True)
    xl, xh = x.to_numpy()
    check_run(gold, xl, xh, info, info.res_hist.to_numpy(), what="%s mode %d" % (solver, mode))
    assert M.mp_status() == 0


@pytest.fixture(scope="module")
def scaled3d_64():
    return synth.config5(p=512)


@pytest.mark.parametrize("solver", ["bicg", "gpbicg"])
def test_scaled3d_64_first_20_iterations(solver, scaled3d_64):
    M = lib()
    gold = load("scaled3d_64_p512_%s_exact_20it" % solver)
    A_h, xs_h, _ = scaled3d_64
    A = M.CSRMatrix.from_host(A_h)
    b = M.mpspmv_csr(A, M.MPArray.from_host(xs_h), mode=M.MP_EXACT)
    assert digest(*b.to_numpy()) == gold["b_digest"], "b = A x* differs from the oracle's"
    o = gold["opts"]
    fn = M.bicg if solver == "bicg" else M.gpbicg
    x, info = fn(A, b, mode=1, maxit=o["maxit"], rtol=tuple(o["rtol"]), atol=tuple(o["atol"]),
                 chunk=8, hist=True)
    xl, xh = x.to_numpy()
    check_run(gold, xl, xh, info, info.res_hist.to_numpy(), what="%s 64^3" % solver)
    assert M.mp_status() == 0


@pytest.fixture(scope="module")
def banded():
    systems = synth.config4(p=256)
    return systems


def _banded_device(M, systems):
    As, bs = [], []
    for A_h, xs in systems:
        A = M.CSRMatrix.from_host(A_h)
        As.append(A)
        bs.append([M.mpspmv_csr(A, M.MPArray.from_host(xt), mode=M.MP_EXACT) for xt in xs])
    return As, bs


def test_banded_whole_batch(banded):
    """All 64 systems x 16 right-hand sides in one batch: every member bit-identical to its plain
    solve, and the members of the two smallest systems equal to the oracle's stored solves."""
    M = lib()
    As, bs = _banded_device(M, banded)
    golds = [load("banded_smallest%d_p256_gpbicg_seq" % k) for k in (0, 1)]
    o = golds[0]["opts"]
    opts = dict(mode=M.MP_SEQ, maxit=o["maxit"], rtol=tuple(o["rtol"]), atol=tuple(o["atol"]), chunk=25)
    xs, infos = M.gpbicg_batched(As, bs, **opts)
    for gold in golds:
        s = gold["system"]
        assert As[s].n_rows == gold["n"] and As[s].nnz == gold["nnz"]
        for k, g in enumerate(gold["rhs"]):
            assert digest(*bs[s][k].to_numpy()) == g["b_digest"]
            xl, xh = xs[s][k].to_numpy()
            check_run(g, xl, xh, infos[s][k], what="batched system %d rhs %d" % (s, k))
            xp, ip = M.gpbicg(As[s], bs[s][k], **opts)
            pl, ph = xp.to_numpy()
            check_run(g, pl, ph, ip, what="plain system %d rhs %d" % (s, k))
    for s in range(len(As)):
        for k in range(len(bs[s])):
            xp, ip = M.gpbicg(As[s], bs[s][k], **opts)
            got = infos[s][k]
            assert (got.status, got.iters) == (ip.status, ip.iters), (s, k, got, ip)
            assert torch.equal(xp.limbs, xs[s][k].limbs) and torch.equal(xp.hdr, xs[s][k].hdr), \
                "system %d rhs %d: batched x differs from the plain solve" % (s, k)
    assert all(i.status == 0 for row in infos for i in row)
    assert M.mp_status() == 0


def test_adjoint_scaled3d_16_dec1():
    """x = A^-1 b and its adjoint lambda = A^-T ones (one transposed BiCG solve) through the
    autograd wrapper, and the value gradient -RN(lambda_i x_j), equal to the oracle's."""
    M = lib()
    gold = load("scaled3d_16_dec1_p512_adjoint")
    p = 512
    A_h = synth.convdiff3d_scaled(16, p, seed=5, dec=1.0)
    xs_h = synth.mp_arange1(A_h.n_rows, p)
    A = M.CSRMatrix.from_host(A_h)
    b = M.mpspmv_csr(A, M.MPArray.from_host(xs_h), mode=1)
    assert digest(*b.to_numpy()) == gold["b_digest"]
    S = M.autograd.SparseStructure.of(A)
    vt = M.autograd.pack(M.MPArray.from_host(A_h.vals)).requires_grad_(True)
    bt = M.autograd.pack(b).requires_grad_(True)
    o = gold["opts"]
    xt = M.autograd.solve(S, vt, bt, mode=1, maxit=o["maxit"], rtol=tuple(o["rtol"]),
                          atol=tuple(o["atol"]), chunk=32)
    xt.backward(M.autograd.pack(M.MPArray.from_host(synth.mp_ones(A_h.n_rows, p))))
    xl, xh = M.autograd.unpack(xt.detach(), p).to_numpy()
    ll, lh = M.autograd.unpack(bt.grad, p).to_numpy()
    gl, gh = M.autograd.unpack(vt.grad, p).to_numpy()
    fwd, adj = gold["forward"], gold["adjoint"]
    assert digest(xl, xh) == fwd["x_digest"], "x differs from the oracle's"
    assert digest(ll, lh) == adj["x_digest"], "lambda differs from the oracle's"
    assert digest(gl, gh) == gold["grad_vals_digest"], "value gradient differs from the oracle's"


def test_adjoint_scaled3d_64_dec1_duality():
    """At full 64^3 size (row scaling with decade spread 1, p = 512, tolerance 1e-100): both the
    solve and its adjoint converge and <lambda, b> = sum_i x_i to the tolerance."""
    M = lib()
    p = 512
    A_h = synth.convdiff3d_scaled(64, p, seed=5, dec=1.0)
    xs_h = synth.mp_arange1(A_h.n_rows, p)
    A = M.CSRMatrix.from_host(A_h)
    b = M.mpspmv_csr(A, M.MPArray.from_host(xs_h), mode=1)
    S = M.autograd.SparseStructure.of(A)
    vt = M.autograd.pack(M.MPArray.from_host(A_h.vals)).requires_grad_(True)
    bt = M.autograd.pack(b).requires_grad_(True)
    xt = M.autograd.solve(S, vt, bt, mode=1, maxit=10000, rtol=(1, -100), atol=(0, 0), chunk=64)
    xt.backward(M.autograd.pack(M.MPArray.from_host(synth.mp_ones(A_h.n_rows, p))))
    xo = codec.decode(*M.autograd.unpack(xt.detach(), p).to_numpy(), p)
    lo = codec.decode(*M.autograd.unpack(bt.grad, p).to_numpy(), p)
    bo = codec.decode(*b.to_numpy(), p)
    sx = sum(v.to_fraction() for v in xo)
    lb = sum(l.to_fraction() * v.to_fraction() for l, v in zip(lo, bo))
    assert abs(lb - sx) <= Fraction(1, 10 ** 90) * abs(sx)
    # and x is the solution [1..n] to about the tolerance times the condition
    assert abs(sx - Fraction(A_h.n_rows * (A_h.n_rows + 1), 2)) <= Fraction(1, 10 ** 60) * abs(sx)
