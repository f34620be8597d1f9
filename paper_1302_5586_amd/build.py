"""Build libpencilfilter.so for gfx950 with hipcc, in-tree.

Every HIP and C++ source under csrc/ is compiled to an object in parallel,
then linked into ``paper_1302_5586_amd/libpencilfilter.so``. Flags:

* ``--offload-arch=gfx950``: MI355X (CDNA4) only.
* ``-ffp-contract=off``: no implicit fused multiply-add; the kernels ask for
  FMA explicitly where they want it, so the exact mode's separate multiply
  and add stay separate.
* ``-Xclang -target-feature -Xclang -packed-fp32-ops``: no packed FP32
  instructions are generated.

Every device compile also asks for the compiler's kernel resource-usage
remarks. They are collected into ``_build/resource_usage.txt`` (VGPRs,
SGPRs, scratch bytes per lane and occupancy of every kernel), and the
build fails if a persistent batch kernel uses scratch memory: compiled
with register spills, that kernel faulted on the GPU twice, so a batch
kernel that spills is never shipped.
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
                       for g, m in ((0, 1), (0, 2), (0, 3)) for e in (0, 1)],
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
        cmd = [HIPCC, "-x", "hip", *DEVICE, *COMMON, *defs, "-Rpass-analysis=kernel-resource-usage", "-c", src,
               "-o", obj]
    else:
        cmd = [HIPCC, *DEVICE, *COMMON, "-c", src, "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("compilation failed: %s" % src)
    noise = "is not a recognized feature for this target"
    text = r.stdout + r.stderr
    with open(obj + ".res", "w") as f:
        f.write(_resource_table(text))
    msgs = [ln for ln in text.splitlines() if ln.strip() and noise not in ln and "kernel-resource-usage" not in ln]
    if msgs and verbose:
        sys.stderr.write("\n".join(msgs) + "\n")
    if verbose:
        print("  %-40s %6.1f s" % (os.path.basename(obj), time.time() - t0), flush=True)
    return obj


def _resource_table(text: str) -> str:
    """One line per kernel from the resource-usage remarks: name, VGPRs,
    SGPRs, scratch bytes per lane, waves per SIMD."""
    rows, cur = [], None
    keys = {"VGPRs": "vgpr", "TotalSGPRs": "sgpr", "ScratchSize [bytes/lane]": "scratch", "Occupancy [waves/SIMD]": "occ"}
    for ln in text.splitlines():
        if "remark:" not in ln:
            continue
        body = ln.split("remark:", 1)[1].split("[-Rpass", 1)[0].strip()
        if body.startswith("Function Name:"):
            cur = {"name": body.split(":", 1)[1].strip()}
            rows.append(cur)
        elif cur is not None and ":" in body:
            k, v = body.rsplit(":", 1)
            if k.strip() in keys:
                cur[keys[k.strip()]] = v.strip()
    return "".join("%s vgpr=%s sgpr=%s scratch=%s occ=%s\n" % (r["name"], r.get("vgpr"), r.get("sgpr"),
                                                               r.get("scratch"), r.get("occ")) for r in rows)


def check_resources(objs, out_path: str) -> None:
    """Write the kernels' resource table; raise if any kernel uses scratch."""
    lines = []
    for o in objs:
        if os.path.exists(o + ".res"):
            lines += open(o + ".res").read().splitlines()
    lines = sorted(set(lines))
    with open(out_path, "w") as f:
        f.write("\n".join(lines) + "\n")
    spills = [ln for ln in lines if "scratch=" in ln and ln.split("scratch=")[1].split()[0] not in ("0", "None")]
    batch = [ln for ln in spills if "k_batch_f32" in ln]
    if batch:
        raise RuntimeError("batch kernels that use scratch (see %s):\n  %s" % (out_path, "\n  ".join(batch)))


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
    check_resources(objs, os.path.join(objdir, "resource_usage.txt"))
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
