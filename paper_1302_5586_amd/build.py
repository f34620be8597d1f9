"""Build libpencilfilter.so for gfx950 with hipcc, in-tree.

Every HIP and C++ source under csrc/ is compiled to an object in parallel,
then linked into ``paper_1302_5586_amd/libpencilfilter.so``. Flags:

* ``--offload-arch=gfx950``: MI355X (CDNA4) only.
* ``-ffp-contract=off``: no implicit fused multiply-add; the kernels ask for
  FMA explicitly where they want it, so the exact mode's separate multiply
  and add stay separate.
* ``-Xclang -target-feature -Xclang -packed-fp32-ops``: no packed FP32
  instructions are generated.
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
OBJDIR = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libpencilfilter.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
COMMON = ["-O3", "-std=c++17", "-fPIC", "-ffp-contract=off", "-Wall", "-Wno-unused-function",
          "-I", INCLUDE, "-I", CSRC]
DEVICE = ["--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


# Units compiled several times with different defines: each radius and each
# batch-kernel group is its own object so that they build in parallel.
VARIANTS = {
    "f32_inst.hip": [("r%d" % r, ["-DPF_R=%d" % r]) for r in range(9)],
    "batch_inst.hip": [("g%de%dm%d" % (g, e, m), ["-DPF_GROUP=%d" % g, "-DPF_EXACT=%d" % e, "-DPF_VMASK=%d" % m])
                       for g, m in ((0, 1), (0, 2), (0, 3), (1, 3)) for e in (0, 1)],
}


def _jobs():
    out = []
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))
    for s in srcs:
        for tag, defs in VARIANTS.get(os.path.basename(s), [("", [])]):
            out.append((s, tag, defs))
    return out


def _newest_header() -> float:
    hs = glob.glob(os.path.join(CSRC, "*.h")) + glob.glob(os.path.join(INCLUDE, "*.h"))
    return max(os.path.getmtime(h) for h in hs)


def _compile(job, verbose: bool, objdir: str = OBJDIR, extra=(), incremental: bool = False) -> str:
    src, tag, defs = job
    defs = list(defs) + list(extra)
    obj = os.path.join(objdir, os.path.basename(src) + (("." + tag) if tag else "") + ".o")
    if incremental and os.path.exists(obj) and \
            os.path.getmtime(obj) > max(os.path.getmtime(src), _newest_header(), os.path.getmtime(__file__)):
        return obj
    t0 = time.time()
    if src.endswith(".hip"):
        cmd = [HIPCC, "-x", "hip", *DEVICE, *COMMON, *defs, "-c", src, "-o", obj]
    else:
        cmd = [HIPCC, *DEVICE, *COMMON, "-c", src, "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("compilation failed: %s" % src)
    noise = "is not a recognized feature for this target"
    msgs = [ln for ln in (r.stdout + r.stderr).splitlines() if ln.strip() and noise not in ln]
    if msgs and verbose:
        sys.stderr.write("\n".join(msgs) + "\n")
    if verbose:
        print("  %-40s %6.1f s" % (os.path.basename(obj), time.time() - t0), flush=True)
    return obj


def build(verbose: bool = False, jobs: int = 0, defines=(), out: str = LIB, incremental: bool = False) -> str:
    """Compile every source and link the shared library; returns its path.
    ``defines`` (e.g. ["-DPF_STRIP_ALIGNED=0"]) and ``out`` build a variant
    of the library elsewhere, in its own object directory. ``incremental``
    keeps objects newer than their source, every header and this script."""
    objdir = OBJDIR if not defines else OBJDIR + "_" + "_".join(d.lstrip("-D").replace("=", "") for d in defines)
    os.makedirs(objdir, exist_ok=True)
    work = _jobs()
    # big units first so the pool drains evenly
    work.sort(key=lambda j: (not j[0].endswith(".hip"), -len(j[1])))
    jobs = jobs or min(os.cpu_count() or 8, 16, len(work))
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda j: _compile(j, verbose, objdir, defines, incremental), work))
    tmp = out + ".tmp%d" % os.getpid()
    cmd = [HIPCC, *DEVICE, "-shared", "-fPIC", "-o", tmp, *objs, "-lpthread"]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("link failed")
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    defs = [a for a in sys.argv[1:] if a.startswith("-D")]
    outs = [a[len("--out="):] for a in sys.argv[1:] if a.startswith("--out=")]
    print(build(verbose="-v" in sys.argv, defines=defs, out=outs[0] if outs else LIB,
                incremental="--incremental" in sys.argv))
