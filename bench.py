"""Benchmark: multiple-precision SpMV + BiCG/GPBiCG on one MI355X.

Workload (the step): the nonsymmetric 2-D convection-diffusion operator, 5-point central
differences on a 256 x 256 grid (n = 65536, nnz = 326656, global Peclet number 10), p = 256 bits,
right-hand side b = A * ones formed in EXACT mode, x0 = 0.  Synthetic (seeded) data; nothing is
read from disk.  A plan is built once (transpose, kernel variants tuned on this matrix).

One step = one pass of the whole hot path on that matrix:
  * y = A x and y = A^T x in SEQ and in EXACT mode, and the value gradient RN(g_i x_j);
  * 200 BiCG iterations in SEQ mode and 200 in EXACT mode (2 products per iteration: A, A^T);
  * 200 GPBiCG iterations in SEQ mode and 200 in EXACT mode (2 products with A per iteration).
The stopping tolerance is set below what 200 iterations reach, so every solve runs all 200
iterations (status NC) and the work per step is fixed.

value = MP non-zeros per second = (stored entries x number of sparse products in a step) /
step time.  `roofline` reports the kernel with the largest share of the step, timed live: one solve per
solver and mode runs with every iteration kernel bracketed by HIP events on the solver's stream
(eager launches, identical results); achieved = algorithmic bytes of those launches (vectors
read and written once; for a sparse product the matrix once, x and y once, the row pointers) /
their summed durations, against HBM bandwidth.  `components.spmv_roofline` gives the same for
the step's SpMV kernel timed alone.
`components` adds per-kernel times, the solver times, the power-law SpMV workload (n = 500000,
~9.9M stored entries, p = 256) with its roofline fractions, and optionally (--batched) the
batched-vs-plain GPBiCG comparison.  `cpu_baseline` times the oracle on the host's cores.
"""
import argparse
import hashlib
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
# MI355X: 256 CUs x 4 SIMD x 16 lanes at 2.4 GHz = 39.3 T lane-ops/s for full-rate integer VALU
# instructions; v_mad_u64_u32 (the 32x32->64 limb product) issues at half that rate (measured
# with independent chains), so the limb-product roofline is 19.66 T mads/s.
PEAK_MAD_TOPS = 256 * 4 * 16 * 2.4e9 / 2 / 1e12
# VALU issue slots: one wave64 instruction per SIMD every 4 cycles
VALU_ISSUE_PEAK = 256 * 4 * 2.4e9 / 4
HBM_PEAK_GBS = 8000.0
KERNEL_SOURCES = ("spmv_kernels.hpp", "solver_kernels.hpp", "mp_core.hpp", "mp_exact.hpp",
                  "mp_scalar.hpp")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-powerlaw", action="store_true")
    ap.add_argument("--batched", action="store_true", help="also time batched vs plain GPBiCG")
    ap.add_argument("--kernel-reps", type=int, default=50)
    ap.add_argument("--profile-pass", default="",
                    help="counter pass only: 'convdiff' or 'powerlaw' (copy calibration + SpMV launches)")
    return ap.parse_args()


def kernel_source_hash():
    h = hashlib.sha1()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1411_2377_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def spmv_bytes(n_rows, n_cols, nnz, L):
    """Algorithmic HBM bytes of one y = A x: entries (limbs, header, column), x and y once, row
    pointers."""
    return nnz * (4 * L + 8) + (n_rows + n_cols) * (4 * L + 4) + 4 * (n_rows + 1)


def build_problem(M, torch):
    import numpy as np
    import synth
    A_h, ones_h = synth.config2(p=PREC, m=GRID)
    A = M.CSRMatrix.from_host(A_h)
    ones = M.MPArray.from_host(ones_h)
    b = M.mpspmv_csr(A, ones, mode=M.MP_EXACT)
    rng = np.random.default_rng(0)
    x = M.MPArray.from_host(synth.mp_uniform(rng, A_h.n_cols, PREC))
    g = M.MPArray.from_host(synth.mp_uniform(rng, A_h.n_rows, PREC))
    plan = M.mp_plan_create(A)
    plan.tune()
    torch.cuda.synchronize()
    return A_h, A, b, x, g, plan


def one_step(M, A, b, x, g, plan, bufs):
    y, yt, gv = bufs
    nprod = 0
    for mode in (M.MP_SEQ, M.MP_EXACT):
        M.mpspmv_csr(A, x, y, mode=mode, plan=plan)
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


def time_kernel(torch, fn, reps):
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


def spmv_symbol(plan, op, mode, L, fused=False):
    """The kernel symbol (as rocprofv3 names it, without "void mp::" and the arguments) of the
    plan's variant of product op (0: A, 1: A^T) in a mode; fused: the solvers' instantiation,
    which ends with the inner products of its output."""
    rows, staged, srt = plan.variants()[(op, mode)]
    base = "spmv_exact_kernel" if mode else ("spmv_seq_sorted_kernel" if srt else "spmv_seq_kernel")
    return "%s<%d, %d, %s>" % (base, L, rows, "true" if fused else "false")


def spmv_kernel_name(plan, op, mode, L, fused=False):
    rows, staged, srt = plan.variants()[(op, mode)]
    return spmv_symbol(plan, op, mode, L, fused) + (" (x staged)" if staged else "")


def load_counters(kernel):
    """The committed counter summary's entry for a kernel symbol, when it was taken on the
    current kernel sources (else None)."""
    path = os.path.join(ROOT, "profiles", "traffic_counters.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    ent = d.get(kernel.split(" (")[0])
    if not ent or ent.get("kernel_source") != kernel_source_hash():
        return None
    return ent


def load_traffic(kernel):
    """HBM traffic per launch from the committed counter summary (FETCH_SIZE + WRITE_SIZE, each
    scaled by the plain-copy calibration), or None."""
    ent = load_counters(kernel)
    return None if ent is None else ent["fetch_bytes"] + ent["write_bytes"]


def valu_issue_frac(kernel, launch_us):
    """VALU instructions per launch from the committed counter summary over the VALU issue
    slots of a launch of the live duration, or None."""
    ent = load_counters(kernel)
    if ent is None or not ent.get("valu_instr"):
        return None
    return round(ent["valu_instr"] / (launch_us * 1e-6 * VALU_ISSUE_PEAK), 4)


def powerlaw_component(M, torch, reps):
    """The power-law workload (n = 500000, mean 20 and max 2000 entries per row, values
    log-uniform over 1e-8..1e8, x uniform on [-1, 1]) at p = 256: y = A x and A^T g in both
    modes with the tuned plan."""
    import synth
    A_h, x_h, g_h = synth.config3(p=PREC)
    A = M.CSRMatrix.from_host(A_h)
    x = M.MPArray.from_host(x_h)
    g = M.MPArray.from_host(g_h)
    y = M.MPArray.empty(A.n_rows, PREC)
    yt = M.MPArray.empty(A.n_cols, PREC)
    plan = M.mp_plan_create(A)
    plan.tune()
    L = PREC // 32
    out = {"workload": "power-law rows n=500000 nnz=%d p=256" % A.nnz}
    for mode, mname in ((M.MP_SEQ, "seq"), (M.MP_EXACT, "exact")):
        t = time_kernel(torch, lambda: M.mpspmv_csr(A, x, y, mode=mode, plan=plan), reps)
        tt = time_kernel(torch, lambda: M.mpspmv_csr_t(A, plan, g, yt, mode=mode), reps)
        by = spmv_bytes(A.n_rows, A.n_cols, A.nnz, L)
        out[mname] = {"spmv_us": round(t * 1e6, 1), "spmv_nnz_per_s": A.nnz / t,
                      "spmv_t_us": round(tt * 1e6, 1), "spmv_t_nnz_per_s": A.nnz / tt,
                      "hbm_frac": round(by / t / (HBM_PEAK_GBS * 1e9), 4),
                      "mad_frac": round(A.nnz * L * L / t / (PEAK_MAD_TOPS * 1e12), 4),
                      "variant": spmv_kernel_name(plan, 0, mode, L)}
    M.mp_status()
    return out


def batched_component(M, torch):
    """Batched GPBiCG on the banded workload (64 systems of 1000..100000 unknowns, bandwidths
    7..41, 16 right-hand sides each, p = 256, relative residual 1e-60) against plain solves of
    a sample of the same (system, right-hand side) pairs, extrapolated to all of them."""
    import numpy as np
    import synth
    systems = synth.config4(p=PREC)
    As, bs = [], []
    for A_h, xs in systems:
        A = M.CSRMatrix.from_host(A_h)
        As.append(A)
        bs.append([M.mpspmv_csr(A, M.MPArray.from_host(xt), mode=M.MP_EXACT) for xt in xs])
    torch.cuda.synchronize()
    opts = dict(mode=M.MP_SEQ, maxit=5000, rtol=(1, -60), atol=(0, 0), chunk=25)
    t0 = time.time()
    xs, infos = M.gpbicg_batched(As, bs, **opts)
    torch.cuda.synchronize()
    t_batched = time.time() - t0
    iters = [i.iters for row in infos for i in row]
    statuses = sorted({i.status for row in infos for i in row})
    rng = np.random.default_rng(0)
    sample = [(int(s), int(rng.integers(0, len(bs[0])))) for s in rng.choice(len(As), 8, replace=False)]
    t_plain, same = 0.0, True
    for s, k in sample:
        t1 = time.time()
        xp, ip = M.gpbicg(As[s], bs[s][k], **opts)
        torch.cuda.synchronize()
        t_plain += time.time() - t1
        same &= (ip.iters == infos[s][k].iters) and bool(
            torch.equal(xp.limbs, xs[s][k].limbs) and torch.equal(xp.hdr, xs[s][k].hdr))
    n_pairs = len(As) * len(bs[0])
    return {"workload": "64 banded systems n=1000..100000, 16 rhs each, p=256, GPBiCG to 1e-60",
            "batched_s": round(t_batched, 3), "plain_s_estimated": round(t_plain / len(sample) * n_pairs, 2),
            "plain_sample_pairs": len(sample), "speedup": round(t_plain / len(sample) * n_pairs / t_batched, 1),
            "iters_min_max": [min(iters), max(iters)], "statuses": statuses,
            "sample_bit_identical": same}


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


def cpu_baseline():
    """The oracle (pure-Python big integers) on the host's cores: one full y = A x in SEQ mode
    and one in EXACT mode, rows split into blocks over a process pool (run before the GPU is
    touched)."""
    import numpy as np
    import synth
    A_h, _ = synth.config2(p=PREC, m=GRID)
    cores = min(16, os.cpu_count() or 1)
    rng = np.random.default_rng(0)
    _CPU_PAYLOAD["A"] = A_h
    _CPU_PAYLOAD["x"] = synth.mp_uniform(rng, A_h.n_cols, PREC)
    blocks = np.array_split(np.arange(A_h.n_rows), cores * 4)
    ctx = mproc.get_context("fork")
    t0 = time.time()
    reps = 0
    with ctx.Pool(cores) as pool:   # whole products until about 10 s have passed
        while reps < 2 or time.time() - t0 < 10.0:
            for mode in (0, 1):
                pool.map(_oracle_rows, [(blk, mode) for blk in blocks])
            reps += 1
    dt = time.time() - t0
    return {"value": 2 * reps * A_h.nnz / dt, "unit": "MP nnz/s", "cores": cores, "kind": "oracle",
            "sample": "%d x (one full y = A x in SEQ and one in EXACT mode) on the 256x256 matrix "
                      "at p=256 (%d products), rows split over %d processes, %.1f s wall"
                      % (reps, 2 * reps * A_h.nnz, cores, dt)}


def profile_pass(M, torch, which):
    """Launches for a counter run: a plain copy of 256 MiB (the counters' calibration), then ten
    launches of each tuned SpMV kernel of the chosen workload and, for the step's workload, 20
    iterations of each solve of the step."""
    src = torch.empty(64 << 20, dtype=torch.int32, device="cuda").fill_(1)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    if which == "powerlaw":
        import synth
        A_h, x_h, g_h = synth.config3(p=PREC)
        A = M.CSRMatrix.from_host(A_h)
        x = M.MPArray.from_host(x_h)
        plan = M.mp_plan_create(A)
        plan.tune()
    else:
        A_h, A, b, x, g, plan = build_problem(M, torch)
    y = M.MPArray.empty(A.n_rows, PREC)
    names = {}
    for mode in (M.MP_SEQ, M.MP_EXACT):
        names[mode] = spmv_kernel_name(plan, 0, mode, PREC // 32)
        names["fused_%d" % mode] = spmv_kernel_name(plan, 0, mode, PREC // 32, fused=True)
        for _ in range(10):
            M.mpspmv_csr(A, x, y, mode=mode, plan=plan)
    if which != "powerlaw":   # the step's solver kernels in their step proportions (20 iterations)
        for solver in (M.bicg, M.gpbicg):
            for mode in (M.MP_SEQ, M.MP_EXACT):
                solver(A, b, plan=plan, mode=mode, maxit=20, rtol=(1, -70), atol=(0, 0), chunk=0)
        # then a few iterations with every variant of the solvers' SpMV instantiations, so that
        # each of their symbols has counters whichever variant a tuning run picks
        tuned = plan.variants()
        for mode in (M.MP_SEQ, M.MP_EXACT):
            for rows in (16, 32, 64):
                for srt in ((False, True) if mode == M.MP_SEQ else (False,)):
                    plan.set_variant(0, mode, rows=rows, stage_x=False, sorted_rows=srt)
                    for solver in (M.bicg, M.gpbicg):
                        solver(A, b, plan=plan, mode=mode, maxit=5, rtol=(1, -70), atol=(0, 0),
                               chunk=0)
            r, st, so = tuned[(0, mode)]
            plan.set_variant(0, mode, rows=r, stage_x=st, sorted_rows=so)
    torch.cuda.synchronize()
    print(json.dumps({"profile_pass": which, "variants": names, "kernel_source": kernel_source_hash(),
                      "copy_bytes": src.numel() * 4, "n_rows": A.n_rows, "n_cols": A.n_cols,
                      "nnz": A.nnz}))


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU: the path is a single-device kernel set and no "
              "multi-GPU run is part of this build (requested --gpus %d)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    cpu = None
    if not args.no_cpu_baseline and not args.profile_pass:
        cpu = cpu_baseline()
    import torch
    import paper_1411_2377_amd as M
    torch.cuda.set_device(0)
    if args.profile_pass:
        profile_pass(M, torch, args.profile_pass)
        return
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
    L = PREC // 32
    for name, fn in (
        ("spmv_seq_us", lambda: M.mpspmv_csr(A, x, y, mode=M.MP_SEQ, plan=plan)),
        ("spmv_exact_us", lambda: M.mpspmv_csr(A, x, y, mode=M.MP_EXACT, plan=plan)),
        ("spmv_t_seq_us", lambda: M.mpspmv_csr_t(A, plan, g, yt, mode=M.MP_SEQ)),
        ("spmv_t_exact_us", lambda: M.mpspmv_csr_t(A, plan, g, yt, mode=M.MP_EXACT)),
        ("grad_vals_us", lambda: M.mp_grad_vals(A, plan, g, x, gv)),
        ("dot_us", lambda: M.mp_dot(x, g, dres)),
    ):
        comp[name] = round(time_kernel(torch, fn, args.kernel_reps) * 1e6, 2)
    comp["variants"] = {"%s_%s" % ("A" if op == 0 else "At", "seq" if m == 0 else "exact"): v
                        for (op, m), v in plan.variants().items()}
    for sname, solver in (("bicg", M.bicg), ("gpbicg", M.gpbicg)):
        for mname, mode in (("seq", M.MP_SEQ), ("exact", M.MP_EXACT)):
            torch.cuda.synchronize()
            t1 = time.time()
            _, info = solver(A, b, plan=plan, mode=mode, maxit=ITERS, rtol=(1, -70), atol=(0, 0),
                             chunk=25)
            torch.cuda.synchronize()
            comp["%s_%s_ms_per_%d_it" % (sname, mname, ITERS)] = round((time.time() - t1) * 1e3, 2)
            comp["%s_%s_status_iters" % (sname, mname)] = [info.status, info.iters]
    if not args.no_powerlaw:
        comp["powerlaw_spmv"] = powerlaw_component(M, torch, max(3, args.kernel_reps // 10))
    if args.batched:
        comp["batched_gpbicg"] = batched_component(M, torch)

    # Kernel times of the step's solves, live: every iteration kernel of one solve per solver
    # and mode bracketed by HIP events on the solver's stream (eager launches, same results).
    prof = {}
    for sname, solver in (("bicg", M.bicg), ("gpbicg", M.gpbicg)):
        for mode in (M.MP_SEQ, M.MP_EXACT):
            pr = M.SolveProfile()
            solver(A, b, plan=plan, mode=mode, maxit=ITERS, rtol=(1, -70), atol=(0, 0), profile=pr)
            prof[(sname, mode)] = pr
    # per kernel symbol: the sparse products that form the step's inner products (one symbol per
    # mode, the tuned variant of A x in its solver instantiation), BiCG's A^T products, and each
    # element-wise step (directions, updates, GPBiCG's t/s/y)
    cand = {}
    for (sname, mode), pr in prof.items():
        names = {0: spmv_kernel_name(plan, 0, mode, L, fused=True),
                 1: spmv_kernel_name(plan, 1, mode, L),
                 2: "%s_dir_kernel<%d>" % ("bicg" if sname == "bicg" else "gp", L),
                 3: "%s_update_kernel<%d, false>" % ("bicg" if sname == "bicg" else "gp", L),
                 4: "gp_tsy_kernel<%d, false>" % L}
        for cls, kn in names.items():
            if pr.launches[cls] == 0:
                continue
            e = cand.setdefault(kn, [0.0, 0, 0.0])
            e[0] += pr.us[cls]; e[1] += pr.launches[cls]; e[2] += pr.bytes[cls]
    comp["solver_kernels"] = {k: {"total_us": round(v[0], 1), "launches": v[1],
                                  "avg_us": round(v[0] / max(1, v[1]), 2)} for k, v in cand.items()}
    kname = max(cand, key=lambda k: cand[k][0])
    tot_us, nl, nb = cand[kname]
    achieved = nb / (tot_us * 1e-6) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": load_traffic(kname), "kernel": kname,
                "launch_us": round(tot_us / max(1, nl), 2), "launches": nl,
                "algorithmic_bytes_per_launch": round(nb / max(1, nl)),
                "valu_issue_frac": valu_issue_frac(kname, tot_us / max(1, nl))}
    # the sparse product of the step alone (its roofline beside the dominant kernel's)
    smode = M.MP_EXACT if comp["spmv_exact_us"] >= comp["spmv_seq_us"] else M.MP_SEQ
    tk = comp["spmv_exact_us" if smode == M.MP_EXACT else "spmv_seq_us"] * 1e-6
    sname = spmv_kernel_name(plan, 0, smode, L)
    nbytes = spmv_bytes(A.n_rows, A.n_cols, A.nnz, L)
    comp["spmv_roofline"] = {"kernel": sname, "launch_us": round(tk * 1e6, 2), "bound": "hbm",
                             "achieved_gbs": round(nbytes / tk / 1e9, 1),
                             "frac": round(nbytes / tk / 1e9 / HBM_PEAK_GBS, 4),
                             "algorithmic_bytes": nbytes, "traffic": load_traffic(sname),
                             "mad_frac": round(A.nnz * L * L / tk / (PEAK_MAD_TOPS * 1e12), 4),
                             "valu_issue_frac": valu_issue_frac(sname, tk * 1e6)}
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
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out))


if __name__ == "__main__":
    main()
