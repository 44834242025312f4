"""Build the HIP library libmpspmv.so in-tree for gfx950 (hipcc cross-compiles without a GPU).

Usage: python -m paper_1411_2377_amd.build   (or __graft_entry__.build())
"""
import os
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libmpspmv.so")
SOURCES = ["api.hip", "spmv_fused.hip", "plan.hip", "vec.hip", "solver.hip", "ilu.hip", "wide.hip"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # no packed FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
]


def sources():
    return [os.path.join(CSRC, s) for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]


def build(verbose=True, jobs=8):
    """Compile every source to an object in parallel, then link the shared library."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    bdir = os.path.join(HERE, "_build")
    os.makedirs(bdir, exist_ok=True)
    t0 = time.time()
    procs = []
    objs = []
    for src in sources():
        obj = os.path.join(bdir, os.path.basename(src) + ".o")
        objs.append(obj)
        cmd = [hipcc] + [f for f in HIPCC_FLAGS if f != "-shared"] + ["-c", src, "-o", obj]
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
    failed = False
    for src, p in procs:
        out, _ = p.communicate()
        text = out.decode(errors="replace")
        lines = [ln for ln in text.splitlines() if "packed-fp32-ops" not in ln]
        if p.returncode != 0:
            failed = True
            sys.stderr.write("\n".join(lines) + "\n")
        elif verbose and any(ln.strip() for ln in lines):
            sys.stderr.write("\n".join(lines) + "\n")
    if failed:
        raise RuntimeError("hipcc failed")
    tmp = OUT + ".tmp"
    cmd = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    subprocess.check_call(cmd)
    os.replace(tmp, OUT)
    if verbose:
        print("built %s in %.1fs" % (OUT, time.time() - t0))
    return OUT


if __name__ == "__main__":
    build()
