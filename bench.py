"""Benchmark: multiple-precision sparse matrix-vector products on one MI355X (the method of
Kouya, arXiv 1411.2377: y = A x over CSR with every operation rounded to nearest at p bits).

Headline workload: the power-law matrix, n = 500000 rows and columns, row lengths from a
truncated power law (mean 20, longest row 2000), 9,932,151 stored entries, values log-uniform in
magnitude over 1e-8..1e8 with random signs, x uniform on [-1, 1], p = 256 bits (8 limbs);
seeded synthetic data, generated on the host and resident in HBM before timing.  A plan is built
and its kernel variants tuned (or read from a tuning cache, --tune-cache).

One step = y = A x in SEQ mode (per-operation rounding in column order) and y = A x in EXACT
mode (exact sum, one rounding): the two accumulation modes of the product.
value = MP non-zeros per second = 2 x stored entries / step time.

`roofline` describes the step's dominant kernel (the mode whose kernel takes longer): its
average launch duration comes from HIP events attached to the kernel launches themselves during
the timed steps (mp_timer_*, on the launch stream); achieved = algorithmic bytes per launch (the
matrix entries once: 4L + 8 bytes each; x and y once: 4L + 4 bytes per element; the row
pointers) / that duration, against the 8 TB/s HBM peak.  `mad_frac` gives the same launch
against the limb-product peak (L^2 32x32->64 multiply-adds per entry at 19.66 T/s).

`components`: both modes at p = 128, 256 and 512 with their variants, the transposed product
and value gradient (the autograd backward), cold-cache launches (after a 1 GiB write), 200
BiCG / GPBiCG / CGS / BiCGSTAB iterations per mode on the 256 x 256 convection-diffusion
operator with their per-kernel profile, the Lotkin-with-zeros dense vs sparse product (the
paper's SpMV benchmark), BiCGSTAB with and without ILU(0) (the paper's Table 3 comparison), and
batched GPBiCG on 64 banded systems x 16 right-hand sides against plain solves.  `cpu_baseline` times the oracle on a bounded sample of the headline workload's rows.

Other uses:
  --profile-pass powerlaw|convdiff   launches for a rocprofv3 counter pass only
  --summarize-stats FILE             text summary of a rocprofv3 *_kernel_stats.csv
  --summarize-counters DIR DIR       traffic summary of a FETCH_SIZE and a WRITE_SIZE pass
"""
import argparse
import glob
import hashlib
import json
import multiprocessing as mproc
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PREC = 256
GRID = 256
ITERS = 200
# MI355X: 256 CUs x 4 SIMD x 16 lanes at 2.4 GHz = 39.3 T lane-ops/s for full-rate integer VALU
# instructions; v_mad_u64_u32 (the 32x32->64 limb product) issues at half that rate (measured
# with independent chains), so the limb-product roofline is 19.66 T mads/s.
PEAK_MAD_TOPS = 256 * 4 * 16 * 2.4e9 / 2 / 1e12
# VALU issue slots: one wave64 instruction per SIMD every 4 cycles
VALU_ISSUE_PEAK = 256 * 4 * 2.4e9 / 4
HBM_PEAK_GBS = 8000.0
KERNEL_SOURCES = ("spmv_kernels.hpp", "solver_kernels.hpp", "mp_core.hpp", "mp_exact.hpp",
                  "mp_scalar.hpp", "mp_group.hpp", "mp_window.hpp")
WORKLOAD = ("power-law CSR n=500000 (row lengths mean 20, max 2000; 9932151 stored entries), "
            "values log-uniform 1e-8..1e8 with random sign, x uniform [-1,1], p=256; "
            "step = y = A x in SEQ mode + y = A x in EXACT mode")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--headline-only", action="store_true",
                    help="only the timed steps (for a kernel-trace profile of the same command)")
    ap.add_argument("--tune-cache", default="", help="tuning cache file (mp_plan_tune_cached)")
    ap.add_argument("--kernel-reps", type=int, default=10)
    ap.add_argument("--profile-pass", default="",
                    help="counter pass only: 'powerlaw' or 'convdiff' (copy calibration + launches)")
    ap.add_argument("--summarize-stats", default="")
    ap.add_argument("--summarize-counters", nargs=3, default=None,
                    metavar=("WORKLOAD", "FETCH_DIR", "WRITE_DIR"))
    ap.add_argument("--summarize-valu", nargs=2, default=None, metavar=("WORKLOAD", "DIR"),
                    help="instruction counts of an SQ_INSTS_VALU/SALU/LDS + SQ_WAVES pass")
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


def spmv_symbol(plan, op, mode, L, fused=False):
    """The kernel symbol (rocprofv3's name without "void mp::" and the arguments) of the plan's
    variant of product op (0: A, 1: A^T) in a mode; fused: the solvers' instantiation."""
    rows, staged, srt, gmin, win = plan.variants()[(op, mode)]
    tf = lambda b: "true" if b else "false"
    if mode == 0 and srt:  # the sorted kernel is instantiated apart for lane groups
        return "spmv_seq_sorted_kernel<%d, %d, %s, %s>" % (L, rows, tf(fused), tf(gmin and not win and not fused))
    base = "spmv_exact_kernel" if mode else "spmv_seq_kernel"
    return "%s<%d, %d, %s>" % (base, L, rows, tf(fused))


def spmv_kernel_name(plan, op, mode, L, fused=False):
    rows, staged, srt, gmin, win = plan.variants()[(op, mode)]
    return spmv_symbol(plan, op, mode, L, fused) + (" (x staged)" if staged else "") + \
        (" (rows of >= %d entries by %s)" % (gmin, ("lane groups", "windowed chains", "windowed chains, four rows per wavefront")[win])
         if gmin else "")


def load_counters(kernel, workload="powerlaw"):
    """The committed counter summary's entry for a kernel symbol in a workload's counter pass,
    when it was taken on the current kernel sources (else None)."""
    path = os.path.join(ROOT, "profiles", "traffic_counters.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    ent = d.get(workload, {}).get(kernel.split(" (")[0])
    if not ent or ent.get("kernel_source") != kernel_source_hash():
        return None
    return ent


def load_traffic(kernel):
    ent = load_counters(kernel)
    return None if ent is None else ent["fetch_bytes"] + ent["write_bytes"]


def valu_issue_frac(kernel, launch_us):
    ent = load_counters(kernel)
    if ent is None or not ent.get("valu_instr"):
        return None
    return round(ent["valu_instr"] / (launch_us * 1e-6 * VALU_ISSUE_PEAK), 4)


def roofline_entry(kernel, launch_us, nbytes, nnz, L):
    return {"bound": "hbm", "achieved": round(nbytes / (launch_us * 1e-6) / 1e9, 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(nbytes / (launch_us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4),
            "traffic": load_traffic(kernel), "kernel": kernel, "launch_us": round(launch_us, 2),
            "algorithmic_bytes_per_launch": nbytes,
            "mad_frac": round(nnz * L * L / (launch_us * 1e-6) / (PEAK_MAD_TOPS * 1e12), 4),
            "valu_issue_frac": valu_issue_frac(kernel, launch_us)}


# ---------------------------------------------------------------------------------------------
# CPU baseline: the oracle on sampled rows of the headline workload (forked before the GPU is
# touched)
# ---------------------------------------------------------------------------------------------
_CPU_PAYLOAD = {}


def _oracle_rows(args):
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
    t0 = time.time()
    ospmv.spmv(sub_rp, cols.tolist(), vals, xs, p, mode)
    return len(ks), time.time() - t0


def cpu_baseline(A_h, x_h, budget_s=12.0):
    """The oracle (pure-Python big integers) on the host's cores: rows drawn uniformly at random
    (seeded) from the headline matrix, each block of rows computed in SEQ and in EXACT mode, in a
    process pool, until about budget_s seconds have passed."""
    import numpy as np
    cores = min(16, os.cpu_count() or 1)
    _CPU_PAYLOAD["A"], _CPU_PAYLOAD["x"] = A_h, x_h
    rng = np.random.default_rng(0)
    ctx = mproc.get_context("fork")
    done_entries = 0
    done_rows = 0
    t0 = time.time()
    with ctx.Pool(cores) as pool:
        while time.time() - t0 < budget_s:
            blocks = [rng.integers(0, A_h.n_rows, 400) for _ in range(cores)]
            for n_ent, _ in pool.map(_oracle_rows, [(b, m) for b in blocks for m in (0, 1)]):
                done_entries += n_ent
            done_rows += 400 * cores
    dt = time.time() - t0
    return {"value": done_entries / dt, "unit": "MP nnz/s", "cores": cores, "kind": "oracle",
            "sample": "%d rows drawn uniformly (seeded) from the headline matrix, each in SEQ and in "
                      "EXACT mode (%d products of stored entries, p=256), rows split over %d "
                      "processes, %.1f s wall" % (done_rows, done_entries, cores, dt)}


# ---------------------------------------------------------------------------------------------
# GPU parts
# ---------------------------------------------------------------------------------------------
def upload_config3(M, p, tune_cache=""):
    import synth
    A_h, x_h, g_h = synth.config3(p=p)
    A = M.CSRMatrix.from_host(A_h)
    x = M.MPArray.from_host(x_h)
    g = M.MPArray.from_host(g_h)
    plan = M.mp_plan_create(A)
    plan.tune(cache=tune_cache or None)
    return A_h, A, x, g, plan


def timed_launches(M, torch, fn, reps, cold=None):
    """Average kernel duration (us) of fn's main kernel over reps launches (kernel timer)."""
    tm = M.KernelTimer(reps + 4)
    for _ in range(reps):
        if cold is not None:
            cold.add_(1)      # 1 GiB written between launches: nothing of the operands in cache
        tm.select()
        fn()
        M.KernelTimer.deselect()
    us, n = tm.read()
    tm.close()
    return us / max(1, n)


def precision_component(M, torch, p, reps, data=None, tune_cache=""):
    """Both modes of y = A x, A^T g and the value gradient on the power-law matrix at p bits."""
    A_h, A, x, g, plan = data if data is not None else upload_config3(M, p, tune_cache)
    L = p // 32
    y = M.MPArray.empty(A.n_rows, p)
    yt = M.MPArray.empty(A.n_cols, p)
    nb = spmv_bytes(A.n_rows, A.n_cols, A.nnz, L)
    out = {"nnz": A.nnz}
    for mode, mname in ((M.MP_SEQ, "seq"), (M.MP_EXACT, "exact")):
        t = timed_launches(M, torch, lambda: M.mpspmv_csr(A, x, y, mode=mode, plan=plan), reps)
        tt = timed_launches(M, torch, lambda: M.mpspmv_csr_t(A, plan, g, yt, mode=mode), reps)
        out[mname] = {"kernel": spmv_kernel_name(plan, 0, mode, L), "kernel_us": round(t, 1),
                      "nnz_per_s": A.nnz / (t * 1e-6),
                      "hbm_frac": round(nb / (t * 1e-6) / 1e9 / HBM_PEAK_GBS, 4),
                      "mad_frac": round(A.nnz * L * L / (t * 1e-6) / (PEAK_MAD_TOPS * 1e12), 4),
                      "transposed_kernel": spmv_kernel_name(plan, 1, mode, L),
                      "transposed_us": round(tt, 1), "transposed_nnz_per_s": A.nnz / (tt * 1e-6)}
    gv = M.MPArray.empty(A.nnz, p)
    tg = timed_launches(M, torch, lambda: M.mp_grad_vals(A, plan, g, x, gv), reps)
    out["grad_vals_us"] = round(tg, 1)
    M.mp_status()
    return out


def cold_component(M, torch, data, reps):
    """Kernel durations with a 1 GiB write before every launch (MALL and L2 hold nothing of the
    operands)."""
    A_h, A, x, g, plan = data
    y = M.MPArray.empty(A.n_rows, A.p)
    L = A.p // 32
    cold = torch.zeros(256 << 20, dtype=torch.int32, device="cuda")
    nb = spmv_bytes(A.n_rows, A.n_cols, A.nnz, L)
    out = {}
    for mode, mname in ((M.MP_SEQ, "seq"), (M.MP_EXACT, "exact")):
        t = timed_launches(M, torch, lambda: M.mpspmv_csr(A, x, y, mode=mode, plan=plan), reps, cold)
        out[mname] = {"kernel_us": round(t, 1), "nnz_per_s": A.nnz / (t * 1e-6),
                      "hbm_frac": round(nb / (t * 1e-6) / 1e9 / HBM_PEAK_GBS, 4)}
    del cold
    return out


def solver_component(M, torch):
    """200 BiCG and 200 GPBiCG iterations per mode on the 2-D convection-diffusion operator
    (256 x 256, Peclet 10, p = 256, b = A * ones in EXACT mode), with the per-kernel profile of
    one eager solve per solver and mode."""
    import synth
    A_h, ones_h = synth.config2(p=PREC, m=GRID)
    A = M.CSRMatrix.from_host(A_h)
    b = M.mpspmv_csr(A, M.MPArray.from_host(ones_h), mode=M.MP_EXACT)
    plan = M.mp_plan_create(A)
    plan.tune()
    L = PREC // 32
    out = {"workload": "2-D convection-diffusion 5-point 256x256 (n=65536, nnz=326656), Peclet 10, "
                       "p=256, b = A*ones; %d iterations (tolerance below reach)" % ITERS}
    for sname, solver in (("bicg", M.bicg), ("gpbicg", M.gpbicg), ("cgs", M.cgs), ("bicgstab", M.bicgstab)):
        for mname, mode in (("seq", M.MP_SEQ), ("exact", M.MP_EXACT)):
            solver(A, b, plan=plan, mode=mode, maxit=5, rtol=(1, -70), atol=(0, 0), chunk=25)
            torch.cuda.synchronize()
            t1 = time.time()
            _, info = solver(A, b, plan=plan, mode=mode, maxit=ITERS, rtol=(1, -70), atol=(0, 0),
                             chunk=25)
            torch.cuda.synchronize()
            dt = time.time() - t1
            out["%s_%s" % (sname, mname)] = {"ms": round(dt * 1e3, 2),
                                             "us_per_iter": round(dt * 1e6 / max(1, info.iters), 1),
                                             "status": info.status, "iters": info.iters}
    cand = {}
    for sname, solver in (("bicg", M.bicg), ("gpbicg", M.gpbicg)):
        for mode in (M.MP_SEQ, M.MP_EXACT):
            pr = M.SolveProfile()
            solver(A, b, plan=plan, mode=mode, maxit=ITERS, rtol=(1, -70), atol=(0, 0), profile=pr)
            names = {0: spmv_kernel_name(plan, 0, mode, L, fused=True),
                     1: spmv_kernel_name(plan, 1, mode, L),
                     2: "%s_dir_kernel<%d>" % ("bicg" if sname == "bicg" else "gp", L),
                     3: "%s_update_kernel<%d, false>" % ("bicg" if sname == "bicg" else "gp", L),
                     4: "gp_tsy_kernel<%d, false>" % L}
            for cls, kn in names.items():
                if pr.launches[cls] == 0:
                    continue
                e = cand.setdefault(kn, [0.0, 0, 0.0])
                e[0] += pr.us[cls]
                e[1] += pr.launches[cls]
                e[2] += pr.bytes[cls]
    out["kernels"] = {k: {"total_us": round(v[0], 1), "launches": v[1],
                          "avg_us": round(v[0] / max(1, v[1]), 2),
                          "hbm_frac": round(v[2] / (v[0] * 1e-6) / 1e9 / HBM_PEAK_GBS, 4)}
                      for k, v in cand.items()}
    M.mp_status()
    return out


def ilu_component(M, torch):
    """The paper's Table 3 comparison on a stand-in operator: BiCGSTAB and BiCGSTAB with ILU(0)
    to the (*) test of Sec. 4.1 (1e-20, 1e-50) on the 2-D convection-diffusion operator on a
    64 x 64 grid, p = 256, x* = [1..n], b = A x* (EXACT), both modes: iterations and times (the
    factorisation timed apart)."""
    import synth
    A_h, _ = synth.config2(p=PREC, m=64)
    A = M.CSRMatrix.from_host(A_h)
    b = M.mpspmv_csr(A, M.MPArray.from_host(synth.mp_arange1(A_h.n_rows, PREC)), mode=M.MP_EXACT)
    torch.cuda.synchronize()
    t0 = time.time()
    K = M.ILU0(A)
    torch.cuda.synchronize()
    out = {"workload": "2-D convection-diffusion 64x64 (n=4096), p=256, x* = [1..n], tolerance "
                       "1e-20 relative + 1e-50", "ilu0_factor_ms": round((time.time() - t0) * 1e3, 2)}
    for mname, mode in (("seq", M.MP_SEQ), ("exact", M.MP_EXACT)):
        for name, run in (("bicgstab", lambda: M.bicgstab(A, b, mode=mode, maxit=5000, chunk=25)),
                          ("bicgstab_ilu0", lambda: M.bicgstab_ilu0(A, K, b, mode=mode, maxit=5000, chunk=5))):
            torch.cuda.synchronize()
            t1 = time.time()
            _, info = run()
            torch.cuda.synchronize()
            out["%s_%s" % (name, mname)] = {"iters": info.iters, "status": info.status,
                                             "ms": round((time.time() - t1) * 1e3, 2)}
    M.mp_status()
    return out


def precision_sweep_component(M, torch):
    """The paper's precision sweep (Sec. 4.1, Tables 1-2: the same solve at 512 to 8192 bits):
    BiCG on the 2-D convection-diffusion operator on a 16 x 16 grid, b = A * ones (EXACT), SEQ
    products, 20 iterations (tolerance below reach), at p = 512 and 1024 (one number per lane)
    and 2048, 4096, 8192 (numbers across a wavefront); ms per iteration and the growth factor per
    doubling of p (the paper: about 2.8-2.9 per doubling for BiCG on cavity04 in MPFR)."""
    import synth
    out = {"workload": "2-D convection-diffusion 16x16 (n=256), BiCG, SEQ, 20 iterations"}
    prev = None
    for p in (512, 1024, 2048, 4096, 8192):
        A_h, ones = synth.config2(p=p, m=16)
        A = M.CSRMatrix.from_host(A_h)
        b = M.mpspmv_csr(A, M.MPArray.from_host(ones), mode=M.MP_EXACT)
        plan = M.mp_plan_create(A)
        M.bicg(A, b, plan=plan, mode=M.MP_SEQ, maxit=2, rtol=(1, -2000), atol=(0, 0), chunk=0)
        torch.cuda.synchronize()
        t0 = time.time()
        _, info = M.bicg(A, b, plan=plan, mode=M.MP_SEQ, maxit=20, rtol=(1, -2000), atol=(0, 0), chunk=0)
        torch.cuda.synchronize()
        ms = (time.time() - t0) * 1e3 / max(1, info.iters)
        e = {"ms_per_iter": round(ms, 3), "iters": info.iters, "status": info.status,
             "path": "one number per lane" if p <= 1024 else "numbers across a wavefront"}
        if prev:
            e["x_per_doubling"] = round(ms / prev, 2)
        out["p%d" % p] = e
        prev = ms
    M.mp_status()
    return out


def lotkin_component(M, torch, reps):
    """The paper's SpMV benchmark (Sec. 3): the Lotkin matrix (n = 2000) with s% of its elements
    set to zero, b = A [1..n] by the sparse product, then A b by the dense product (all n^2
    elements stored, zeros taking the fast path) and by the sparse product of the non-zero
    elements with a tuned plan; speedup = dense time / sparse time (SEQ mode).  Results are
    bit-identical."""
    import synth
    n = 2000
    out = {"workload": "Lotkin n=2000 with s%% zeros, y = A (A [1..n]) in SEQ mode; dense: %d stored "
                       "elements" % (n * n)}
    for p, zs in ((256, (50.0, 90.0, 99.0)), (128, (90.0,)), (512, (90.0,))):
        for z in zs:
            D_h, C_h, x_h = synth.lotkin(n, p, z, seed=6)
            A = M.CSRMatrix.from_host(C_h)
            D = M.MPArray.from_host(D_h)
            plan = M.mp_plan_create(A)
            plan.tune(reps=1)
            b = M.mpspmv_csr(A, M.MPArray.from_host(x_h), mode=M.MP_SEQ, plan=plan)
            plan.tune(reps=1, x=b)   # the variants timed on the operand they will see
            ys = M.MPArray.empty(n, p)
            yd = M.MPArray.empty(n, p)
            ts = timed_launches(M, torch, lambda: M.mpspmv_csr(A, b, ys, mode=M.MP_SEQ, plan=plan), reps)
            td = timed_launches(M, torch, lambda: M.mp_gemv(D, n, n, b, yd, mode=M.MP_SEQ), reps)
            same = bool(torch.equal(ys.limbs, yd.limbs) and torch.equal(ys.hdr, yd.hdr))
            out["p%d_zeros%g" % (p, z)] = {"nnz": A.nnz, "sparse_us": round(ts, 1), "dense_us": round(td, 1),
                                           "speedup": round(td / ts, 2), "same_bits": same}
            del A, D, b, ys, yd, plan
    M.mp_status()
    return out


def batched_component(M, torch):
    """Batched GPBiCG on the banded workload (64 systems of 1000..100000 unknowns, bandwidths
    7..41, 16 right-hand sides each, p = 256, SEQ products, relative residual 1e-60) against
    plain solves: one right-hand side of every system solved alone (bit-identity checked), the
    plain time of each system taken 16 times."""
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
    nrhs = len(bs[0])
    rng = np.random.default_rng(0)
    t_plain, same = 0.0, True
    for s in range(len(As)):
        k = int(rng.integers(0, nrhs))
        t1 = time.time()
        xp, ip = M.gpbicg(As[s], bs[s][k], **opts)
        torch.cuda.synchronize()
        t_plain += (time.time() - t1) * nrhs
        same &= (ip.iters == infos[s][k].iters) and bool(
            torch.equal(xp.limbs, xs[s][k].limbs) and torch.equal(xp.hdr, xs[s][k].hdr))
    return {"workload": "64 banded systems n=1000..100000 (sum 1405456), 16 rhs each, p=256, "
                        "GPBiCG (SEQ products) to relative residual 1e-60",
            "batched_s": round(t_batched, 3), "plain_s": round(t_plain, 2),
            "plain_method": "one right-hand side of each of the 64 systems solved alone, times 16",
            "speedup": round(t_plain / t_batched, 1),
            "iters_min_max": [min(iters), max(iters)], "statuses": statuses,
            "plain_bit_identical": same}


def headline(M, torch, args, data):
    """The timed steps: y = A x in SEQ and in EXACT mode per step, kernel durations from events
    attached to the two product kernels."""
    A_h, A, x, g, plan = data
    L = PREC // 32
    y_seq = M.MPArray.empty(A.n_rows, PREC)
    y_ex = M.MPArray.empty(A.n_rows, PREC)
    t_seq = M.KernelTimer(args.steps + 8)
    t_ex = M.KernelTimer(args.steps + 8)
    for _ in range(args.warmup):
        M.mpspmv_csr(A, x, y_seq, mode=M.MP_SEQ, plan=plan)
        M.mpspmv_csr(A, x, y_ex, mode=M.MP_EXACT, plan=plan)
    torch.cuda.synchronize()
    t0 = time.time()
    for _ in range(args.steps):
        t_seq.select()
        M.mpspmv_csr(A, x, y_seq, mode=M.MP_SEQ, plan=plan)
        t_ex.select()
        M.mpspmv_csr(A, x, y_ex, mode=M.MP_EXACT, plan=plan)
        M.KernelTimer.deselect()
    torch.cuda.synchronize()
    dt = time.time() - t0
    M.mp_status()
    us_seq, n_seq = t_seq.read()
    us_ex, n_ex = t_ex.read()
    k_seq, k_ex = us_seq / n_seq, us_ex / n_ex
    nb = spmv_bytes(A.n_rows, A.n_cols, A.nnz, L)
    dom_mode = M.MP_SEQ if k_seq >= k_ex else M.MP_EXACT
    roof = roofline_entry(spmv_kernel_name(plan, 0, dom_mode, L), max(k_seq, k_ex), nb, A.nnz, L)
    roof["launches"] = n_seq if dom_mode == M.MP_SEQ else n_ex
    modes = {}
    for mode, mname, k in ((M.MP_SEQ, "seq", k_seq), (M.MP_EXACT, "exact", k_ex)):
        e = roofline_entry(spmv_kernel_name(plan, 0, mode, L), k, nb, A.nnz, L)
        e["nnz_per_s"] = A.nnz / (k * 1e-6)
        modes[mname] = e
    return dt, roof, modes


def main():
    args = parse()
    if args.summarize_stats:
        summarize_stats(args.summarize_stats)
        return
    if args.summarize_counters:
        summarize_counters(*args.summarize_counters)
        return
    if args.summarize_valu:
        summarize_valu(*args.summarize_valu)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: the path is a single-device kernel set and no "
              "multi-GPU run is part of this build (requested --gpus %d)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    import synth
    A_h, x_h, g_h = synth.config3(p=PREC)
    cpu = None
    if not args.no_cpu_baseline and not args.profile_pass and not args.headline_only:
        cpu = cpu_baseline(A_h, x_h)
    import torch
    import paper_1411_2377_amd as M
    torch.cuda.set_device(0)
    if args.profile_pass:
        profile_pass(M, torch, args.profile_pass, args)
        return
    A = M.CSRMatrix.from_host(A_h)
    x = M.MPArray.from_host(x_h)
    g = M.MPArray.from_host(g_h)
    plan = M.mp_plan_create(A)
    plan.tune(cache=args.tune_cache or None)
    torch.cuda.synchronize()
    data = (A_h, A, x, g, plan)
    dt, roof, modes = headline(M, torch, args, data)
    value = 2 * A.nnz * args.steps / dt
    comp = {"modes": modes, "variants": {"%s_%s" % ("A" if op == 0 else "At", "seq" if m == 0 else "exact"): v
                                         for (op, m), v in plan.variants().items()},
            "tune_cache_hit": getattr(plan, "cache_hit", False)}
    if not args.headline_only:
        reps = args.kernel_reps
        comp["p256"] = precision_component(M, torch, PREC, reps, data)
        comp["cold_cache_p256"] = cold_component(M, torch, data, max(3, reps // 2))
        del data, A, x, g, plan
        torch.cuda.empty_cache()
        for p in (128, 512):
            comp["p%d" % p] = precision_component(M, torch, p, reps, tune_cache=args.tune_cache)
            torch.cuda.empty_cache()
        comp["solvers_convdiff256"] = solver_component(M, torch)
        comp["lotkin_dense_vs_sparse"] = lotkin_component(M, torch, reps)
        comp["ilu0_bicgstab"] = ilu_component(M, torch)
        comp["precision_sweep_bicg"] = precision_sweep_component(M, torch)
        comp["batched_gpbicg"] = batched_component(M, torch)
    out = {
        "metric": "MP nonzeros/s for 256-bit MP-SpMV (+ % roofline); BiCG solve time, batched vs plain",
        "value": value,
        "unit": "MP nnz/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32 limbs (p=256 binary floating point, RN)",
        "data": "synthetic",
        "config": {"workload": WORKLOAD, "n": A_h.n_rows, "nnz": A_h.nnz, "prec_bits": PREC,
                   "products_per_step": 2},
        "roofline": roof,
        "components": comp,
    }
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out))


# ---------------------------------------------------------------------------------------------
# counter passes and summaries of rocprofv3 output
# ---------------------------------------------------------------------------------------------
def profile_pass(M, torch, which, args):
    """Launches for a counter run: an elementwise kernel reading and writing 256 MiB (the
    counters' calibration), then ten
    launches of each tuned SpMV kernel of the workload (the power-law matrix at p = 256, or the
    256 x 256 operator followed by 20 iterations of each solve)."""
    src = torch.empty(64 << 20, dtype=torch.int32, device="cuda").fill_(1)
    dst = torch.empty_like(src)
    for _ in range(3):   # the calibration: one elementwise kernel reading and writing 256 MiB
        torch.bitwise_not(src, out=dst)
    torch.cuda.synchronize()
    import synth
    if which == "powerlaw":
        A_h, x_h, _ = synth.config3(p=PREC)
        A = M.CSRMatrix.from_host(A_h)
        x = M.MPArray.from_host(x_h)
        plan = M.mp_plan_create(A)
        plan.tune(cache=args.tune_cache or None)
    else:
        A_h, ones_h = synth.config2(p=PREC, m=GRID)
        A = M.CSRMatrix.from_host(A_h)
        x = M.MPArray.from_host(ones_h)
        plan = M.mp_plan_create(A)
        plan.tune(cache=args.tune_cache or None)
    y = M.MPArray.empty(A.n_rows, PREC)
    names = {}
    for mode in (M.MP_SEQ, M.MP_EXACT):
        names[mode] = spmv_kernel_name(plan, 0, mode, PREC // 32)
        for _ in range(10):
            M.mpspmv_csr(A, x, y, mode=mode, plan=plan)
    if which != "powerlaw":
        b = M.mpspmv_csr(A, x, mode=M.MP_EXACT)
        for solver in (M.bicg, M.gpbicg):
            for mode in (M.MP_SEQ, M.MP_EXACT):
                solver(A, b, plan=plan, mode=mode, maxit=20, rtol=(1, -70), atol=(0, 0), chunk=0)
    torch.cuda.synchronize()
    print(json.dumps({"profile_pass": which, "variants": names, "kernel_source": kernel_source_hash(),
                      "copy_bytes": src.numel() * 4, "n_rows": A.n_rows, "nnz": A.nnz}))


def _csv_rows(path):
    import csv
    with open(path) as fh:
        return list(csv.DictReader(fh))


def _short(name):
    n = name
    for pre in ("void ", "mp::", "(anonymous namespace)::"):
        n = n.replace(pre, "")
    return n.split("(")[0] if "(" in n and not n.startswith("(") else n


def summarize_stats(path):
    """Kernel table of a rocprofv3 --stats kernel summary (calls, total, average per kernel)."""
    rows = _csv_rows(path)
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    print("%-70s %6s %12s %10s %6s" % ("kernel", "calls", "total_us", "avg_us", "pct"))
    for r in rows:
        print("%-70s %6s %12.1f %10.2f %6.2f" % (_short(r["Name"])[:70], r["Calls"],
                                                 float(r["TotalDurationNs"]) / 1e3,
                                                 float(r["AverageNs"]) / 1e3, float(r["Percentage"])))


def _counter_means(d, counter):
    """Per kernel: mean over dispatches of the counter (summed over its instances) in bytes."""
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    per = {}
    for f in files:
        disp = {}
        for r in _csv_rows(f):
            if r["Counter_Name"] != counter:
                continue
            key = (r["Dispatch_Id"], r["Kernel_Name"])
            disp[key] = disp.get(key, 0.0) + float(r["Counter_Value"])
        for (_, name), v in disp.items():
            per.setdefault(_short(name), []).append(v * 1024.0)   # KiB -> bytes
    return {k: sum(v) / len(v) for k, v in per.items()}


def summarize_counters(workload, fetch_dir, write_dir):
    """FETCH_SIZE and WRITE_SIZE per dispatch, each scaled by what the same counter reads for
    the pass's plain 256 MiB copy; stored under the workload's name in
    profiles/traffic_counters.json and printed."""
    fe = _counter_means(fetch_dir, "FETCH_SIZE")
    wr = _counter_means(write_dir, "WRITE_SIZE")
    copy = [k for k in fe if "bitwise_not" in k]
    copy_bytes = 256 << 20
    f_fetch = fe[copy[0]] / copy_bytes if copy else 1.0
    f_write = wr.get(copy[0], copy_bytes) / copy_bytes if copy else 1.0
    path = os.path.join(ROOT, "profiles", "traffic_counters.json")
    d_all = json.load(open(path)) if os.path.exists(path) else {}
    d_all = {k: v for k, v in d_all.items() if k in ("powerlaw", "convdiff")}
    d = d_all.setdefault(workload, {})
    src = kernel_source_hash()
    print("calibration kernel %s: factors fetch %.4f write %.4f" % (copy[0] if copy else "-", f_fetch, f_write))
    print("%-60s %14s %14s %12s" % ("kernel (avg per dispatch)", "FETCH_MB", "WRITE_MB", "traffic_MB"))
    for k in sorted(set(fe) | set(wr)):
        fb, wb = fe.get(k, 0.0) / f_fetch, wr.get(k, 0.0) / f_write
        ent = d.get(k, {})
        if ent.get("kernel_source") not in (None, src):
            ent = {}
        ent.update({"fetch_bytes": round(fb), "write_bytes": round(wb), "kernel_source": src,
                    "workload": workload})
        d[k] = ent
        print("%-60s %14.2f %14.2f %12.2f" % (k[:60], fe.get(k, 0.0) / 1e6, wr.get(k, 0.0) / 1e6, (fb + wb) / 1e6))
    with open(path, "w") as fh:
        json.dump(d_all, fh, indent=1, sort_keys=True)
        fh.write("\n")


def summarize_valu(workload, d):
    """Per kernel: mean wavefront instruction counts per dispatch (SQ_INSTS_VALU, _SALU, _LDS,
    SQ_WAVES) and the mean dispatch duration the same pass recorded; VALU% is the share of the
    chip's VALU issue slots (one wave64 instruction per SIMD every 4 cycles) the dispatch used.
    valu_instr is stored under the workload in profiles/traffic_counters.json."""
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    per = {}
    for f in files:
        disp = {}
        for r in _csv_rows(f):
            key = (r["Dispatch_Id"], _short(r["Kernel_Name"]))
            e = disp.setdefault(key, {"dur": 0.0})
            e[r["Counter_Name"]] = e.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
            if "End_Timestamp" in r and "Start_Timestamp" in r:
                e["dur"] = (float(r["End_Timestamp"]) - float(r["Start_Timestamp"])) / 1e3
        for (_, name), e in disp.items():
            per.setdefault(name, []).append(e)
    path = os.path.join(ROOT, "profiles", "traffic_counters.json")
    d_all = json.load(open(path)) if os.path.exists(path) else {}
    dw = d_all.setdefault(workload, {})
    src = kernel_source_hash()
    cols = ("SQ_INSTS_VALU", "SQ_INSTS_SALU", "SQ_INSTS_LDS", "SQ_WAVES")
    print("%-48s %5s %9s %12s %10s %10s %8s %7s" % ("kernel (avg per dispatch)", "n", "dur_us",
                                                    "VALU_instr", "SALU", "LDS", "waves", "VALU%"))
    for k in sorted(per):
        es = per[k]
        avg = {c: sum(e.get(c, 0.0) for e in es) / len(es) for c in cols + ("dur",)}
        frac = avg["SQ_INSTS_VALU"] / (avg["dur"] * 1e-6 * VALU_ISSUE_PEAK) if avg["dur"] > 0 else 0.0
        print("%-48s %5d %9.2f %12.0f %10.0f %10.0f %8.0f %6.1f%%" % (
            k[:48], len(es), avg["dur"], avg["SQ_INSTS_VALU"], avg["SQ_INSTS_SALU"],
            avg["SQ_INSTS_LDS"], avg["SQ_WAVES"], 100 * frac))
        ent = dw.get(k, {})
        if ent.get("kernel_source") not in (None, src):
            ent = {}
        ent.update({"valu_instr": round(avg["SQ_INSTS_VALU"]), "kernel_source": src,
                    "workload": workload})
        dw[k] = ent
    with open(path, "w") as fh:
        json.dump(d_all, fh, indent=1, sort_keys=True)
        fh.write("\n")


if __name__ == "__main__":
    main()
