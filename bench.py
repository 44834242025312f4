"""Benchmark: multiple-precision SpMV + BiCG/GPBiCG on one MI355X.

Workload: the nonsymmetric 2-D convection-diffusion operator, 5-point central differences on a
256 x 256 grid (n = 65536, nnz = 326656, global Peclet number 10), p = 256 bits, right-hand side
b = A * ones formed in EXACT mode, x0 = 0.  Synthetic (seeded) data; nothing is read from disk.

One step = one pass of the whole hot path on that matrix:
  * y = A x and y = A^T x in SEQ and in EXACT mode, and the value gradient RN(g_i x_j);
  * 200 BiCG iterations in SEQ mode and 200 in EXACT mode (2 products per iteration: A, A^T);
  * 200 GPBiCG iterations in SEQ mode and 200 in EXACT mode (2 products with A per iteration).
The stopping tolerance is set below what 200 iterations reach, so every solve runs all 200
iterations (status NC) and the work per step is fixed.

value = MP non-zeros per second = (stored entries x number of sparse products in a step) /
step time.  `roofline` reports the kernel with the largest share of the step (timed alone,
replayed back to back from a captured graph, with events on its stream) against the full-rate
integer VALU issue rate; `cpu_baseline` times the oracle on the host's cores.
"""
import argparse
import json
import multiprocessing as mproc
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

GRID = 256
PREC = 256
ITERS = 200
# MI355X: 256 CUs x 64 lanes x 2.4 GHz; v_mad_u64_u32 issues at full rate on gfx950 (a
# back-to-back microbenchmark of independent chains measured ~40 Tinst/s including the moves).
PEAK_MAD_TOPS = 256 * 64 * 2.4e9 / 1e12
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--kernel-reps", type=int, default=50)
    return ap.parse_args()


def build_problem(M, torch):
    import synth
    A_h, ones_h = synth.config2(p=PREC, m=GRID)
    A = M.CSRMatrix.from_host(A_h)
    ones = M.MPArray.from_host(ones_h)
    b = M.mpspmv_csr(A, ones, mode=M.MP_EXACT)
    import numpy as np
    rng = np.random.default_rng(0)
    x = M.MPArray.from_host(synth.mp_uniform(rng, A_h.n_cols, PREC))
    g = M.MPArray.from_host(synth.mp_uniform(rng, A_h.n_rows, PREC))
    plan = M.mp_plan_create(A)
    torch.cuda.synchronize()
    return A_h, A, b, x, g, plan


def one_step(M, A, b, x, g, plan, bufs):
    y, yt, gv = bufs
    nprod = 0
    for mode in (M.MP_SEQ, M.MP_EXACT):
        M.mpspmv_csr(A, x, y, mode=mode)
        M.mpspmv_csr_t(A, plan, g, yt, mode=mode)
        nprod += 2
    M.mp_grad_vals(A, plan, g, x, gv)
    infos = []
    for solver in (M.bicg, M.gpbicg):
        for mode in (M.MP_SEQ, M.MP_EXACT):
            _, info = solver(A, b, plan=plan, mode=mode, maxit=ITERS, rtol=(1, -70), atol=(0, 0),
                             chunk=25)
            infos.append(info)
            nprod += 2 * info.iters
    return nprod, infos


def time_kernel(M, torch, fn, reps):
    """Average duration of one launch: `reps` launches captured in a graph, replayed between
    two events on the capturing stream."""
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        for _ in range(3):
            fn()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        for _ in range(reps):
            fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(s):
        g.replay()
        torch.cuda.synchronize()
        e0.record(s)
        for _ in range(3):
            g.replay()
        e1.record(s)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / (3 * reps) * 1e-3   # seconds per launch


_CPU_PAYLOAD = {}


def _oracle_rows(args):
    """Oracle y_i for a block of rows (runs in a pool worker; the matrix is inherited)."""
    rows, mode = args
    from oracle import codec, spmv as ospmv
    A_h, x_h = _CPU_PAYLOAD["A"], _CPU_PAYLOAD["x"]
    p = A_h.vals.p
    rp = A_h.row_ptr
    ks = [k for i in rows for k in range(int(rp[i]), int(rp[i + 1]))]
    sub_rp = [0]
    for i in rows:
        sub_rp.append(sub_rp[-1] + int(rp[i + 1] - rp[i]))
    cols = A_h.col_idx[ks]
    vals = codec.decode(A_h.vals.limbs[:, ks], A_h.vals.hdr[ks], p)
    uc = sorted(set(int(c) for c in cols))
    xs = dict(zip(uc, codec.decode(x_h.limbs[:, uc], x_h.hdr[uc], p)))
    return len(ospmv.spmv(sub_rp, cols.tolist(), vals, xs, p, mode))


def cpu_baseline(A_h):
    """The oracle (pure-Python big integers) on the host's cores: one full y = A x in SEQ mode
    and one in EXACT mode, rows split into blocks over a process pool."""
    import numpy as np
    import synth
    cores = min(16, os.cpu_count() or 1)
    rng = np.random.default_rng(0)
    _CPU_PAYLOAD["A"] = A_h
    _CPU_PAYLOAD["x"] = synth.mp_uniform(rng, A_h.n_cols, PREC)
    blocks = np.array_split(np.arange(A_h.n_rows), cores * 4)
    ctx = mproc.get_context("fork")
    t0 = time.time()
    reps = 4
    with ctx.Pool(cores) as pool:
        for _ in range(reps):
            for mode in (0, 1):
                pool.map(_oracle_rows, [(blk, mode) for blk in blocks])
    dt = time.time() - t0
    return {"value": 2 * reps * A_h.nnz / dt, "unit": "MP nnz/s", "cores": cores, "kind": "oracle",
            "sample": "%d x (one full y = A x in SEQ and one in EXACT mode) on the 256x256 matrix "
                      "at p=256 (%d products), rows split over %d processes, %.1f s wall"
                      % (reps, 2 * reps * A_h.nnz, cores, dt)}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU: the path is a single-device kernel set and no "
              "multi-GPU run is part of this build (requested --gpus %d)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_1411_2377_amd as M
    torch.cuda.set_device(0)
    A_h, A, b, x, g, plan = build_problem(M, torch)
    y = M.MPArray.empty(A.n_rows, PREC)
    yt = M.MPArray.empty(A.n_cols, PREC)
    gv = M.MPArray.empty(A.nnz, PREC)
    bufs = (y, yt, gv)
    dres = M.MPArray.empty(1, PREC)
    for _ in range(args.warmup):
        one_step(M, A, b, x, g, plan, bufs)
    torch.cuda.synchronize()
    t0 = time.time()
    total = 0
    for _ in range(args.steps):
        nprod, infos = one_step(M, A, b, x, g, plan, bufs)
        total += nprod
    torch.cuda.synchronize()
    dt = time.time() - t0
    M.mp_status()
    ms_step = dt / args.steps * 1e3
    value = total * A.nnz / dt

    # per-component times (one extra pass, events around each part)
    comp = {}
    for name, fn in (
        ("spmv_seq_us", lambda: M.mpspmv_csr(A, x, y, mode=M.MP_SEQ)),
        ("spmv_exact_us", lambda: M.mpspmv_csr(A, x, y, mode=M.MP_EXACT)),
        ("spmv_t_seq_us", lambda: M.mpspmv_csr_t(A, plan, g, yt, mode=M.MP_SEQ)),
        ("spmv_t_exact_us", lambda: M.mpspmv_csr_t(A, plan, g, yt, mode=M.MP_EXACT)),
        ("grad_vals_us", lambda: M.mp_grad_vals(A, plan, g, x, gv)),
        ("dot_us", lambda: M.mp_dot(x, g, dres)),
    ):
        comp[name] = round(time_kernel(M, torch, fn, args.kernel_reps) * 1e6, 2)
    for sname, solver in (("bicg", M.bicg), ("gpbicg", M.gpbicg)):
        for mname, mode in (("seq", M.MP_SEQ), ("exact", M.MP_EXACT)):
            torch.cuda.synchronize()
            t1 = time.time()
            _, info = solver(A, b, plan=plan, mode=mode, maxit=ITERS, rtol=(1, -70), atol=(0, 0),
                             chunk=25)
            torch.cuda.synchronize()
            comp["%s_%s_ms_per_%d_it" % (sname, mname, ITERS)] = round((time.time() - t1) * 1e3, 2)
            comp["%s_%s_status_iters" % (sname, mname)] = [info.status, info.iters]

    # dominant sparse kernel against the integer-VALU roofline
    L = PREC // 32
    t_exact = comp["spmv_exact_us"] * 1e-6
    t_seq = comp["spmv_seq_us"] * 1e-6
    kname, tk = ("spmv_exact_kernel<8>", t_exact) if t_exact >= t_seq else ("spmv_seq_kernel<8>", t_seq)
    mads = A.nnz * L * L
    achieved = mads / tk / 1e12
    roofline = {"bound": "alu", "achieved": round(achieved, 4), "peak": round(PEAK_MAD_TOPS, 2),
                "unit": "TOP/s", "frac": round(achieved / PEAK_MAD_TOPS, 5), "traffic": None,
                "kernel": kname, "launch_us": round(tk * 1e6, 2),
                "ops_per_launch": mads,
                "op": "32x32->64-bit multiply-add, L^2 = 64 per stored entry at p = 256"}
    out = {
        "metric": "MP nonzeros/s for 256-bit MP-SpMV (+ % roofline); BiCG solve time, batched vs plain",
        "value": value,
        "unit": "MP nnz/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32 limbs (p=256 binary floating point, RN)",
        "data": "synthetic",
        "config": {"workload": "2-D convection-diffusion 5-point, 256x256 grid (n=65536, nnz=326656, "
                               "Peclet 10), p=256; SpMV/SpMV^T both modes + 200 BiCG + 200 GPBiCG "
                               "iterations per mode, b = A*ones",
                   "n": A.n_rows, "nnz": A.nnz, "prec_bits": PREC, "iters": ITERS},
        "components": comp,
        "roofline": roofline,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(A_h)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
