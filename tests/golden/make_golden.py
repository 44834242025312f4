"""Writes the stored expected values of the long solver parity cases (tests/golden/*.json).

Only the oracle (oracle/) computes them, on inputs from the seeded generators (synth/); nothing
here touches the GPU library.  Each case becomes one JSON file holding the workload and solver
options, the oracle's status and iteration count, SHA-256 digests (tests/util.py `digest`) of x
and of every residual-history entry in the storage layout, a few entries of x written out in
full (limbs and header, for a readable first difference), and the oracle's wall time.

Cases (the paper's Fig. 5 solvers with the stopping test of Sec. 4.1, K = I):
  convdiff2d_256_*   2-D convection-diffusion 256 x 256, p = 256, b = RN_exact(A * ones):
                     200 iterations of BiCG, GPBiCG, CGS and BiCGSTAB in SEQ and EXACT mode
                     (tolerance 1e-70, out of reach, so all 200 run);
  scaled3d_64_*      row-scaled 3-D operator 64^3, p = 512, b = RN_exact(A [1..n]): the first
                     20 iterations of BiCG and GPBiCG, EXACT (tolerance 1e-100);
  banded_*           the two smallest systems of the 64-system banded batch, all 16 right-hand
                     sides, GPBiCG SEQ to 1e-60 (maxit 5000);
  scaled3d_16_dec1_adjoint  a 16^3 row-scaled operator with decade spread 1, p = 512: the BiCG
                     solve of A x = A [1..n] to 1e-100, the adjoint lambda = A^-T ones (one
                     transposed BiCG) and the value gradient -RN(lambda_i x_j).

Usage: python tests/golden/make_golden.py [case-prefix ...]   (cases run in parallel processes)
"""
import json
import multiprocessing as mproc
import os
import sys
import time
from fractions import Fraction

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import codec, krylov, mpnum, spmv as ospmv  # noqa: E402
from tests.util import digest  # noqa: E402


def const(m, e10, p):
    return mpnum.round_fraction(Fraction(m) * Fraction(10) ** e10, p) if m else mpnum.zero(p)


def enc_digest(vals, p):
    return digest(*codec.encode(vals, p))


def entry(v, p):
    limbs, hdr = codec.encode([v], p)
    return {"limbs": [int(t) for t in limbs[:, 0]], "hdr": int(hdr[0])}


def samples(vals, p, n_extra=12, seed=0):
    n = len(vals)
    rng = np.random.default_rng(seed)
    idx = sorted(set([0, 1, n // 2, n - 1] + [int(i) for i in rng.integers(0, n, n_extra)]))
    return {str(i): entry(vals[i], p) for i in idx}


class System:
    def __init__(self, A_h):
        self.p = A_h.vals.p
        self.rp = A_h.row_ptr.tolist()
        self.ci = A_h.col_idx.tolist()
        self.vals = codec.decode(A_h.vals.limbs, A_h.vals.hdr, self.p)
        self.t = ospmv.transpose(A_h.n_rows, A_h.n_cols, self.rp, self.ci, self.vals)

    def mv(self, mode):
        return lambda v: ospmv.spmv(self.rp, self.ci, self.vals, v, self.p, mode)

    def rmv(self, mode):
        tp, ti, tv = self.t
        return lambda v: ospmv.spmv(tp, ti, tv, v, self.p, mode)


def solve(S, solver, mode, b, rtol, atol, maxit):
    p = S.p
    c_rel, c_abs = const(*rtol, p), const(*atol, p)
    if solver == "bicg":
        return krylov.bicg(S.mv(mode), S.rmv(mode), b, c_rel, c_abs, maxit, p)
    return getattr(krylov, solver)(S.mv(mode), b, c_rel, c_abs, maxit, p)


def result(ref, p, with_samples=True):
    out = {"status": ref.status, "iters": ref.iters, "x_digest": enc_digest(ref.x, p),
           "hist_digests": [enc_digest([q], p)[:16] for q in ref.res_hist]}
    if with_samples:
        out["x_samples"] = samples(ref.x, p)
    return out


def case_convdiff2d(solver, mode):
    p, m = 256, 256
    A_h, ones_h = synth.config2(p=p, m=m)
    S = System(A_h)
    b = ospmv.spmv_exact(S.rp, S.ci, S.vals, codec.decode(ones_h.limbs, ones_h.hdr, p), p)
    opts = {"rtol": [1, -70], "atol": [0, 0], "maxit": 200}
    t0 = time.time()
    ref = solve(S, solver, mode, b, opts["rtol"], opts["atol"], opts["maxit"])
    return {"workload": "2-D convection-diffusion 5-point, 256x256 grid, Peclet 10, p=256, "
                        "b = RN_exact(A * ones), x0 = 0",
            "solver": solver, "mode": mode, "opts": opts, "b_digest": enc_digest(b, p),
            "oracle_wall_s": round(time.time() - t0, 1), **result(ref, p)}


def case_scaled3d(solver):
    p = 512
    A_h, xs_h, _ = synth.config5(p=p)
    S = System(A_h)
    b = ospmv.spmv_exact(S.rp, S.ci, S.vals, codec.decode(xs_h.limbs, xs_h.hdr, p), p)
    opts = {"rtol": [1, -100], "atol": [0, 0], "maxit": 20}
    t0 = time.time()
    ref = solve(S, solver, ospmv.EXACT, b, opts["rtol"], opts["atol"], opts["maxit"])
    return {"workload": "3-D 7-point convection-diffusion 64^3, rows scaled by 10^u, "
                        "u ~ U(-15, 15), p=512, b = RN_exact(A [1..n]), x0 = 0",
            "solver": solver, "mode": ospmv.EXACT, "opts": opts, "b_digest": enc_digest(b, p),
            "oracle_wall_s": round(time.time() - t0, 1), **result(ref, p)}


def smallest_banded(k):
    """Index (in generation order) and data of the k-th smallest system of the banded batch."""
    systems = synth.config4(p=256)
    order = np.argsort([A.n_rows for A, _ in systems], kind="stable")
    s = int(order[k])
    return s, systems[s]


def case_banded(k):
    p = 256
    s, (A_h, xs) = smallest_banded(k)
    S = System(A_h)
    opts = {"rtol": [1, -60], "atol": [0, 0], "maxit": 5000}
    t0 = time.time()
    rhs = []
    for j, xt in enumerate(xs):
        b = ospmv.spmv_exact(S.rp, S.ci, S.vals, codec.decode(xt.limbs, xt.hdr, p), p)
        ref = solve(S, "gpbicg", ospmv.SEQ, b, opts["rtol"], opts["atol"], opts["maxit"])
        r = result(ref, p, with_samples=False)
        r["hist_digest"] = enc_digest(ref.res_hist, p) if ref.res_hist else ""
        del r["hist_digests"]
        r["b_digest"] = enc_digest(b, p)
        rhs.append(r)
    return {"workload": "banded batch (64 systems, seed 4): system %d of the generation order, "
                        "n=%d, p=256, b_k = RN_exact(A x*_k), 16 right-hand sides" % (s, A_h.n_rows),
            "system": s, "n": A_h.n_rows, "nnz": A_h.nnz, "solver": "gpbicg", "mode": ospmv.SEQ,
            "opts": opts, "oracle_wall_s": round(time.time() - t0, 1), "rhs": rhs}


def case_adjoint():
    p, m = 512, 16
    A_h = synth.convdiff3d_scaled(m, p, seed=5, dec=1.0)
    xs_h = synth.mp_arange1(A_h.n_rows, p)
    S = System(A_h)
    b = ospmv.spmv_exact(S.rp, S.ci, S.vals, codec.decode(xs_h.limbs, xs_h.hdr, p), p)
    opts = {"rtol": [1, -100], "atol": [0, 0], "maxit": 2000}
    c_rel, c_abs = const(1, -100, p), mpnum.zero(p)
    t0 = time.time()
    fwd = krylov.bicg(S.mv(1), S.rmv(1), b, c_rel, c_abs, opts["maxit"], p)
    ones = [mpnum.from_int(1, p)] * A_h.n_rows
    adj = krylov.bicg(S.rmv(1), S.mv(1), ones, c_rel, c_abs, opts["maxit"], p)
    gv = ospmv.grad_vals(S.rp, S.ci, adj.x, fwd.x, p, negate=True)
    return {"workload": "3-D 7-point convection-diffusion 16^3, rows scaled by 10^u, u ~ U(-1, 1), "
                        "p=512, b = RN_exact(A [1..n]); adjoint right-hand side ones",
            "mode": 1, "opts": opts, "b_digest": enc_digest(b, p),
            "oracle_wall_s": round(time.time() - t0, 1),
            "forward": result(fwd, p), "adjoint": result(adj, p),
            "grad_vals_digest": enc_digest(gv, p)}


CASES = {
    "convdiff2d_256_p256_bicg_seq": lambda: case_convdiff2d("bicg", 0),
    "convdiff2d_256_p256_bicg_exact": lambda: case_convdiff2d("bicg", 1),
    "convdiff2d_256_p256_gpbicg_seq": lambda: case_convdiff2d("gpbicg", 0),
    "convdiff2d_256_p256_gpbicg_exact": lambda: case_convdiff2d("gpbicg", 1),
    "convdiff2d_256_p256_cgs_seq": lambda: case_convdiff2d("cgs", 0),
    "convdiff2d_256_p256_cgs_exact": lambda: case_convdiff2d("cgs", 1),
    "convdiff2d_256_p256_bicgstab_seq": lambda: case_convdiff2d("bicgstab", 0),
    "convdiff2d_256_p256_bicgstab_exact": lambda: case_convdiff2d("bicgstab", 1),
    "scaled3d_64_p512_bicg_exact_20it": lambda: case_scaled3d("bicg"),
    "scaled3d_64_p512_gpbicg_exact_20it": lambda: case_scaled3d("gpbicg"),
    "banded_smallest0_p256_gpbicg_seq": lambda: case_banded(0),
    "banded_smallest1_p256_gpbicg_seq": lambda: case_banded(1),
    "scaled3d_16_dec1_p512_adjoint": case_adjoint,
}


def run(name):
    t0 = time.time()
    out = CASES[name]()
    out["case"] = name
    with open(os.path.join(HERE, name + ".json"), "w") as fh:
        json.dump(out, fh, indent=1, sort_keys=True)
        fh.write("\n")
    return name, round(time.time() - t0, 1)


def main():
    want = sys.argv[1:]
    names = [n for n in CASES if not want or any(n.startswith(w) for w in want)]
    with mproc.get_context("fork").Pool(min(len(names), os.cpu_count() or 1)) as pool:
        for name, dt in pool.imap_unordered(run, names):
            print("%s: %.1f s" % (name, dt), flush=True)


if __name__ == "__main__":
    main()
