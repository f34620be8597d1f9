"""Benchmark: Gpixel/s and % of the HBM roofline, batched vs plain, plus
p50/p99 latency of the served stream, on one MI355X.

One step = one replay of the batch plan over the 512-image batch (seeded
synthetic FP32 images, widths and heights log-uniform in [64, 2048], radius
1..4, Gaussian sigma in [0.5, 2.0); the 2D and separable tile bodies chosen
per image by the tune table), a single persistent launch captured in a
hipGraph. `value` is output Gpixel/s over the timed steps.

Printed as one JSON line with, besides the contract fields:
  roofline      the batch kernel's algorithmic bytes (8 per pixel) over its
                average duration from HIP events on its stream, against
                8 TB/s; `traffic` is filled from committed counter profiles
                when they match the current kernel, else null;
  plain         the same 512 images as 512 single-image launches (from
                Python, and replayed from a captured graph);
  large_2d / large_sep   the 4096x4096 5x5 Gaussian (2D and fused
                separable), buffers rotated over 1 GiB;
  chain         4 fused passes of a 3x3 Gaussian over 4096x4096, against 4
                single-pass launches;
  reduce        float64 sum of 4096x4096 FP32; histogram of 256 MiB uint8;
  inc           OP2 edge-to-cell increment on a 2048x2048 quad mesh;
  rgb_u8        1920x1080 planar RGB 7x7 integer filter;
  small         256x256 3x3 Gaussian: back-to-back throughput and the
                latency distribution of single calls;
  *_exact       the bit-reproducible mode (PF_FLAG_EXACT) at 4096x4096 and
                on the batch, beside the default mode;
  serve         open-loop Poisson arrivals at 2000 req/s (p50/p99/p99.9),
                a sweep of arrival rates up to saturation, and upload mode;
  cpu_baseline  the C oracle on all host cores and on one, over whole
                passes of the batch; cpu_per_config the same for every
                configuration.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
VALU_LANE_OPS = 256 * 4 * 16 * 2.4e9   # CUs x SIMDs x lanes x clock: dot4 lane-ops/s
MFMA_INT8_PEAK = 5.0e15        # MI355X dense int8 matrix ops/s, published
# Server settings for every served run: three streams keep a batch on the
# device while the next is packed; batches of up to 256 requests keep the
# per-batch host work small next to the kernel at saturation.
SERVE_STREAMS = 3
SERVE_MAX_BATCH = 256


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--serve-seconds", type=float, default=60.0)
    ap.add_argument("--serve-rate", type=float, default=2000.0)
    ap.add_argument("--tune", default=os.path.join(ROOT, "paper_1302_5586_amd", "tune_mi355x.json"))
    ap.add_argument("--autotune", default="",
                    help="tune the table (per class, then on the batch workload), write it to this path, and "
                         "bench with it")
    ap.add_argument("--skip", default="",
                    help="comma list of sections to skip: probes,exact,plain,large,chain,reduce,inc,small,rgb,serve,cpu")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run a plain 512 MiB device copy 4 times (reference for counter scaling)")
    return ap.parse_args()


KERNEL_SOURCES = ("paper_1302_5586_amd/csrc/filter_body.h", "paper_1302_5586_amd/csrc/pf_internal.h",
                  "paper_1302_5586_amd/csrc/dev_common.h", "paper_1302_5586_amd/csrc/batch_inst.hip",
                  "paper_1302_5586_amd/csrc/f32_inst.hip", "paper_1302_5586_amd/csrc/launch.hip",
                  "paper_1302_5586_amd/csrc/u8_mfma.hip")


def kernel_source_hash():
    """Hash of the kernel sources with comments and blank lines removed
    (comment edits do not invalidate the counters)."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        text = open(os.path.join(ROOT, f)).read()
        lines = [re.sub(r"//.*", "", ln).rstrip() for ln in text.splitlines()]
        h.update("\n".join(ln for ln in lines if ln).encode())
    return h.hexdigest()[:16]


def committed_traffic(tag):
    """HBM bytes per launch of a kernel from the committed counter profile
    (profiles/counters.json), or None when the kernel sources changed since
    the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "counters.json")
    if not os.path.exists(path):
        return None
    doc = json.load(open(path))
    if doc.get("source_hash") != kernel_source_hash():
        return None
    k = doc.get("kernels", {}).get(tag)
    return None if k is None else k.get("traffic_bytes")


def time_events(torch, fn, reps, stream):
    """Average ms per call from HIP events recorded on `stream` around
    `reps` back-to-back calls."""
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for i in range(reps):
        fn(i)
    b.record(stream)
    b.synchronize()
    return a.elapsed_time(b) / reps


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only (--gpus 1); multi-GPU sharding is design-only",
              file=sys.stderr)
        sys.exit(2)
    skip = set(s for s in args.skip.split(",") if s)

    import torch

    import paper_1302_5586_amd as pf
    import synth

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    pf.load()
    stream = torch.cuda.current_stream()
    if args.autotune:
        t0 = time.time()
        pf.autotune(r_max=pf.PF_R_MAX, reps=20)
        log("class autotune done (%.1f s)" % (time.time() - t0))
    elif os.path.exists(args.tune):
        pf.tune_load(args.tune)
        log("tune table: %s" % args.tune)
    else:
        log("tune table: built-in defaults")

    if args.calibrate_copy:
        # A plain copy of known size: its FETCH_SIZE / WRITE_SIZE per dispatch
        # scale the counters of the filter kernels to bytes.
        src = torch.ones(128 << 20, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(4):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("calibration copy: 4 x %d bytes read and written" % (src.numel() * 4))
        del src, dst

    # ---- batch workload (512 images, seed 3) --------------------------------
    t0 = time.time()
    b = synth.config_batch()
    kinds = [pf.KIND_SEP] * b.n
    filters = [np.concatenate([b.fx[i], b.fx[i]]) for i in range(b.n)]
    pk = pf.pack_batch(b.images, filters, kinds)
    log("batch generated: %d images, %d px (%.1f s)" % (b.n, b.pixels, time.time() - t0))
    x = torch.from_numpy(pk.pixels).to(dev)
    fl = torch.from_numpy(pk.filters).to(dev)
    out = torch.empty_like(x)
    if args.autotune:
        t0 = time.time()
        pf.autotune_batch(pk.h, pk.w, pk.r, pk.kind, pk.pix_off, pk.filt_off, x, fl, out, reps=20,
                          path=args.autotune)
        log("batch autotune done, table written to %s (%.1f s)" % (args.autotune, time.time() - t0))
    plan = pf.BatchPlan(pk.h, pk.w, pk.r, pk.kind, pk.pix_off, pk.filt_off, x.numel(), fl.numel(), graph=True)
    info = plan.info()
    variants = plan.variants()
    px = b.pixels
    alg_bytes = 8 * px

    for _ in range(args.warmup):
        plan.run(x, fl, out)
    torch.cuda.synchronize()
    # One event pair around the timed steps, on the stream the graph is
    # launched on: an event recorded between two graph launches held the
    # next launch back by about 20 us on MI355X (0.318 ms per step with
    # per-step events against 0.297 ms without), which is event overhead,
    # not the kernel's.
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    e0.record(stream)
    for _ in range(args.steps):
        plan.run(x, fl, out)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    k_avg_ms = e0.elapsed_time(e1) / args.steps
    ms_per_step = wall * 1000.0 / args.steps
    value = px * args.steps / wall / 1e9
    achieved = alg_bytes / (k_avg_ms * 1e-3) / 1e9
    log("batched: %.3f ms/step wall, kernel avg %.3f ms, %.1f Gpx/s, %.0f GB/s" % (ms_per_step, k_avg_ms, value, achieved))

    result = {
        "metric": "Gpixel/s + % HBM roofline, batched vs plain; p50/p99 request latency",
        "value": round(value, 3),
        "unit": "Gpixel/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded numpy PCG64 images; no dataset)",
        "config": {"workload": "batch of 512 FP32 images, sizes log-uniform 64..2048, r 1..4, Gaussian sigma "
                               "0.5..2.0, seed 3; one persistent launch replayed from a hipGraph",
                   "images": b.n, "pixels": px, "wave_tiles": info["tasks"], "grid": info["grid"],
                   "launches_per_step": info["launches"],
                   "variants": {name: int((variants == v).sum()) for v, name in
                                ((0, "direct"), (1, "separable"), (2, "separable_as_2d"))}},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": committed_traffic("k_batch_f32_batch512"),
                     "traffic_unit": "bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                     "traffic_source": "profiles/counters.json: rocprofv3 --pmc runs of this kernel source "
                                       "(null when the kernel sources changed since); not measured in this run",
                     "kernel": "k_batch_f32", "algorithmic_bytes_per_launch": alg_bytes,
                     "avg_kernel_ms": round(k_avg_ms, 4)},
    }

    # ---- the batch in the bit-reproducible mode ----------------------------------
    if "exact" not in skip:
        plan_x = pf.BatchPlan(pk.h, pk.w, pk.r, pk.kind, pk.pix_off, pk.filt_off, x.numel(), fl.numel(), graph=True,
                              exact=True)
        for _ in range(3):
            plan_x.run(x, fl, out)
        ms = time_events(torch, lambda _: plan_x.run(x, fl, out), max(5, args.steps), stream)
        result["batch_exact"] = {"value": round(px / (ms * 1e-3) / 1e9, 3), "unit": "Gpixel/s",
                                 "ms_per_step": round(ms, 4), "cost_vs_default": round(ms / k_avg_ms, 3),
                                 "frac_hbm": round(alg_bytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                                 "workload": "the same batch with PF_FLAG_EXACT (separate multiply and add per tap, "
                                             "bit-identical to the sequential program)"}
        log("batch exact: %.3f ms (x%.2f of default)" % (ms, ms / k_avg_ms))
        plan_x.close()

    # ---- plain: the same images as single-image launches ---------------------
    if "plain" not in skip:
        offs = pk.pix_off
        f_off = pk.filt_off
        views = []
        for i in range(b.n):
            n = int(pk.h[i]) * int(pk.w[i])
            k = 2 * int(pk.r[i]) + 1
            xi = x[offs[i]:offs[i] + n].view(int(pk.h[i]), int(pk.w[i]))
            oi = out[offs[i]:offs[i] + n].view(int(pk.h[i]), int(pk.w[i]))
            fx = fl[f_off[i]:f_off[i] + k]
            fy = fl[f_off[i] + k:f_off[i] + 2 * k]
            views.append((xi, fx, fy, oi))

        def plain_step(_):
            for xi, fx, fy, oi in views:
                pf.filter_sep(xi, fx, fy, out=oi)

        plain_step(0)
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        ms = time_events(torch, plain_step, max(3, args.steps // 4), stream)
        torch.cuda.synchronize()
        pv = px / (ms * 1e-3) / 1e9
        result["plain"] = {"value": round(pv, 3), "unit": "Gpixel/s", "ms_per_step": round(ms, 4),
                           "launches_per_step": b.n, "batched_speedup": round(value / pv, 3)}
        log("plain: %.3f ms/step, %.1f Gpx/s (batched x%.2f)" % (ms, pv, value / pv))
        # The same 512 launches captured once in a graph and replayed: the
        # GPU-side cost of separate kernels, without the host's per-call work.
        g = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream()
        side.wait_stream(stream)
        with torch.cuda.stream(side):
            plain_step(0)
        stream.wait_stream(side)
        torch.cuda.synchronize()
        with torch.cuda.graph(g):
            plain_step(0)
        torch.cuda.synchronize()
        for _ in range(3):
            g.replay()
        torch.cuda.synchronize()
        msg = time_events(torch, lambda _: g.replay(), max(5, args.steps), stream)
        pg = px / (msg * 1e-3) / 1e9
        result["plain"]["graph_replay"] = {"value": round(pg, 3), "unit": "Gpixel/s", "ms_per_step": round(msg, 4),
                                           "batched_speedup": round(value / pg, 3)}
        log("plain, 512 launches replayed from a graph: %.3f ms/step, %.1f Gpx/s (batched x%.2f)" % (
            msg, pg, value / pg))
        del g

    # ---- probes: what plain kernels sustain on this device ---------------------
    # An ALU rate (one instruction back to back on independent registers) and
    # a flat HBM copy of the 4096x4096 image's bytes: the filters' timings
    # are read against these as well as against the published peaks.
    probes = {}
    if "probes" not in skip:
        pbuf = torch.empty(4096 * 256, dtype=torch.int32, device=dev)
        for pname, op in (("dot4", pf.PROBE_DOT4), ("fma", pf.PROBE_FMA)):
            ops = pf.probe_alu(op, 4096, 200, pbuf)
            ms = time_events(torch, lambda i: pf.probe_alu(op, 4096, 200, pbuf), 5, stream)
            probes[pname + "_lane_ops_per_s"] = ops / (ms * 1e-3)
            log("probe %s: %.2f T lane-ops/s (%.3f of 256 CUs x 64 lanes x 2.4 GHz)" % (
                pname, ops / (ms * 1e-3) / 1e12, ops / (ms * 1e-3) / VALU_LANE_OPS))
        del pbuf
        n = 4096 * 4096
        nbuf = 8
        xs = [torch.ones(n, dtype=torch.float32, device=dev) for _ in range(nbuf)]
        os_ = [torch.empty_like(xs[0]) for _ in range(nbuf)]
        for i in range(nbuf):
            pf.probe_copy(xs[i], os_[i])
        ms = time_events(torch, lambda i: pf.probe_copy(xs[i % nbuf], os_[i % nbuf]), 64, stream)
        probes["copy_4096sq_us"] = ms * 1e3
        probes["copy_GBs"] = 8 * n / (ms * 1e-3) / 1e9
        log("probe copy 4096x4096 FP32: %.2f us, %.0f GB/s (%.3f of HBM)" % (
            ms * 1e3, probes["copy_GBs"], probes["copy_GBs"] / HBM_PEAK_GBS))
        del xs, os_
        result["probes"] = {
            "dot4_T_lane_ops_per_s": round(probes["dot4_lane_ops_per_s"] / 1e12, 2),
            "dot4_frac_of_derived_peak": round(probes["dot4_lane_ops_per_s"] / VALU_LANE_OPS, 4),
            "fma_T_lane_ops_per_s": round(probes["fma_lane_ops_per_s"] / 1e12, 2),
            "fma_frac_of_derived_peak": round(probes["fma_lane_ops_per_s"] / VALU_LANE_OPS, 4),
            "copy_4096sq_us": round(probes["copy_4096sq_us"], 2),
            "copy_GBs": round(probes["copy_GBs"], 1),
            "copy_frac_hbm": round(probes["copy_GBs"] / HBM_PEAK_GBS, 4),
            "workload": "4096 workgroups x 256 lanes x 200 x 128 instructions on 8 independent registers; flat "
                        "non-temporal copy of 4096x4096 FP32, buffers rotated over 1 GiB"}

    # ---- 4096x4096 5x5 Gaussian, plain filter ---------------------------------
    if "large" not in skip:
        cfg = synth.config_large()
        n = cfg.h * cfg.w
        nbuf = 8   # 8 x 128 MiB of in+out: the 256 MB last-level cache cannot serve it
        xs = [torch.from_numpy(cfg.image).to(dev) for _ in range(nbuf)]
        os_ = [torch.empty_like(xs[0]) for _ in range(nbuf)]
        f2 = torch.from_numpy(cfg.f2d).to(dev)
        g1 = torch.from_numpy(cfg.f1d).to(dev)
        g2 = g1.clone()
        for name, fn in (("large_2d", lambda i: pf.filter2d(xs[i % nbuf], f2, out=os_[i % nbuf])),
                         ("large_sep", lambda i: pf.filter_sep(xs[i % nbuf], g1, g2, out=os_[i % nbuf])),
                         ("large_2d_exact", lambda i: pf.filter2d(xs[i % nbuf], f2, exact=True, out=os_[i % nbuf])),
                         ("large_sep_exact",
                          lambda i: pf.filter_sep(xs[i % nbuf], g1, g2, exact=True, out=os_[i % nbuf]))):
            for i in range(nbuf):
                fn(i)
            ms = time_events(torch, fn, 64, stream)
            gbs = 8 * n / (ms * 1e-3) / 1e9
            result[name] = {"value": round(n / (ms * 1e-3) / 1e9, 3), "unit": "Gpixel/s", "us_per_call": round(ms * 1e3, 2),
                            "achieved_GBs": round(gbs, 1), "frac_hbm": round(gbs / HBM_PEAK_GBS, 4),
                            "workload": "4096x4096 FP32, 5x5 Gaussian sigma 1.5, seed 1, buffers rotated over 1 GiB"
                                        + ("; PF_FLAG_EXACT" if name.endswith("exact") else "")}
            if "copy_4096sq_us" in probes:
                # the copy probe moves the same 8 bytes per pixel
                result[name]["frac_of_copy_probe"] = round(probes["copy_4096sq_us"] / (ms * 1e3), 4)
            if name.endswith("exact"):
                base = result[name[:-len("_exact")]]["us_per_call"]
                result[name]["cost_vs_default"] = round(ms * 1e3 / base, 3)
            log("%s: %.2f us/call, %.0f GB/s (%.1f%% of HBM)" % (name, ms * 1e3, gbs, 100 * gbs / HBM_PEAK_GBS))
        del xs, os_

    # ---- chain: 4 passes of a 3x3 Gaussian over 4096x4096, fused ----------------
    if "chain" not in skip:
        cfg = synth.config_large()
        n = cfg.h * cfg.w
        passes = 4
        nbuf = 8
        xs = [torch.from_numpy(cfg.image).to(dev) for _ in range(nbuf)]
        os_ = [torch.empty_like(xs[0]) for _ in range(nbuf)]
        tmp = [torch.empty_like(xs[0]) for _ in range(2)]
        f3 = torch.from_numpy(synth.gaussian_2d(1, 1.0)).to(dev)

        def fused(i):
            pf.filter_chain(xs[i % nbuf], f3, passes, pf.BORDER_CLAMP, out=os_[i % nbuf])

        def unfused(i):
            src = xs[i % nbuf]
            for p in range(passes):
                dst = os_[i % nbuf] if p == passes - 1 else tmp[p % 2]
                pf.filter2d(src, f3, out=dst)
                src = dst

        res = {}
        for name, fn in (("fused", fused), ("unfused", unfused)):
            for i in range(nbuf):
                fn(i)
            res[name] = time_events(torch, fn, 32, stream)
        gbs = 8 * n / (res["fused"] * 1e-3) / 1e9
        result["chain"] = {"value": round(n * passes / (res["fused"] * 1e-3) / 1e9, 3),
                           "unit": "Gpixel-passes/s", "us_per_chain": round(res["fused"] * 1e3, 2),
                           "unfused_us_per_chain": round(res["unfused"] * 1e3, 2),
                           "speedup_vs_unfused": round(res["unfused"] / res["fused"], 3),
                           "achieved_GBs": round(gbs, 1), "frac_hbm": round(gbs / HBM_PEAK_GBS, 4),
                           "workload": "4096x4096 FP32 (seed 1), 4 passes of a 3x3 Gaussian sigma 1.0, clamp; "
                                       "fused (one launch) vs 4 single-pass launches"}
        log("chain: fused %.2f us, unfused %.2f us (x%.2f), %.0f GB/s (%.1f%% of HBM)" % (
            res["fused"] * 1e3, res["unfused"] * 1e3, res["unfused"] / res["fused"], gbs, 100 * gbs / HBM_PEAK_GBS))
        del xs, os_, tmp

    # ---- reductions: sum/mean of 4096x4096 FP32, histogram of 256 MiB uint8 ----
    if "reduce" not in skip:
        cfg = synth.config_large()
        n = cfg.h * cfg.w
        nbuf = 8
        xs = [torch.from_numpy(cfg.image).to(dev).reshape(-1) for _ in range(nbuf)]
        outs = torch.empty(2, dtype=torch.float64, device=dev)
        ws = pf._workspace(pf.load().pf_sum_workspace, n, dev)
        fn = lambda i: pf.sum_f32(xs[i % nbuf], out=outs, workspace=ws)  # noqa: E731
        for i in range(nbuf):
            fn(i)
        ms_sum = time_events(torch, fn, 64, stream)
        del xs
        nb = 256 << 20
        gen = torch.Generator(device=dev)
        gen.manual_seed(5)
        xb = torch.randint(0, 256, (nb,), dtype=torch.uint8, device=dev, generator=gen)
        hout = torch.empty(256, dtype=torch.int64, device=dev)
        hws = pf._workspace(pf.load().pf_hist_workspace, nb, dev)
        fn = lambda i: pf.hist256_u8(xb, out=hout, workspace=hws)  # noqa: E731
        fn(0)
        ms_hist = time_events(torch, fn, 16, stream)
        del xb
        sum_gbs = 4 * n / (ms_sum * 1e-3) / 1e9
        hist_gbs = nb / (ms_hist * 1e-3) / 1e9
        result["reduce"] = {"sum_us": round(ms_sum * 1e3, 2), "sum_GBs": round(sum_gbs, 1),
                            "sum_frac_hbm": round(sum_gbs / HBM_PEAK_GBS, 4),
                            "hist_us": round(ms_hist * 1e3, 2), "hist_GBs": round(hist_gbs, 1),
                            "hist_frac_hbm": round(hist_gbs / HBM_PEAK_GBS, 4),
                            "workload": "float64 sum and mean of 4096x4096 FP32 (seed 1, 8 rotating buffers); "
                                        "256-bin histogram of 256 MiB of uniform random bytes (torch seed 5)"}
        log("reduce: sum %.2f us (%.0f GB/s, %.1f%%), hist %.2f us (%.0f GB/s, %.1f%%)" % (
            ms_sum * 1e3, sum_gbs, 100 * sum_gbs / HBM_PEAK_GBS, ms_hist * 1e3, hist_gbs,
            100 * hist_gbs / HBM_PEAK_GBS))

    # ---- OP2 edge-to-cell increment on a 2048 x 2048 quad mesh ----------------
    if "inc" not in skip:
        m = synth.config_mesh()
        t0 = time.perf_counter()
        plan_inc = pf.IncPlan(m.ncells, m.edge_to_cells)
        plan_ms = (time.perf_counter() - t0) * 1e3
        ed = torch.from_numpy(m.edge).to(dev)
        cells = torch.from_numpy(m.cell).to(dev)
        e2c = torch.from_numpy(m.edge_to_cells.reshape(-1)).to(dev)
        fn = lambda i: plan_inc.run(ed, cells)  # noqa: E731
        fn(0)
        ms_plan = time_events(torch, fn, 50, stream)
        fn = lambda i: pf.edge_inc_atomic(e2c, ed, cells)  # noqa: E731
        fn(0)
        ms_atomic = time_events(torch, fn, 50, stream)
        # Bytes the plan run must move: each cell read and written (16 B), its
        # offset (4 B), and per increment an index (4 B) and an edge value (8 B).
        inc_bytes = 20 * m.ncells + 2 * m.nedges * 12
        gbs = inc_bytes / (ms_plan * 1e-3) / 1e9
        result["inc"] = {"value": round(m.nedges / (ms_plan * 1e-3) / 1e9, 3), "unit": "Gedge/s",
                         "plan_us": round(ms_plan * 1e3, 2), "atomic_us": round(ms_atomic * 1e3, 2),
                         "plan_build_ms": round(plan_ms, 1), "achieved_GBs": round(gbs, 1),
                         "frac_hbm": round(gbs / HBM_PEAK_GBS, 4),
                         "workload": "2048x2048 quad mesh, 4,194,304 cells, 8,384,512 edges, random cell numbering "
                                     "and edge order (seed 6), float64 values"}
        log("inc: plan %.2f us (%.0f GB/s, %.1f%%), atomic %.2f us, plan build %.0f ms" % (
            ms_plan * 1e3, gbs, 100 * gbs / HBM_PEAK_GBS, ms_atomic * 1e3, plan_ms))
        plan_inc.close()
        del ed, cells, e2c

    # ---- 256x256 3x3 Gaussian: throughput and single-call latency ------------
    if "small" not in skip:
        cfg = synth.config_small()
        n = cfg.h * cfg.w
        nbuf = 64
        xs = [torch.from_numpy(cfg.image).to(dev) for _ in range(nbuf)]
        os_ = [torch.empty_like(xs[0]) for _ in range(nbuf)]
        f2 = torch.from_numpy(cfg.f2d).to(dev)
        fn = lambda i: pf.filter2d(xs[i % nbuf], f2, out=os_[i % nbuf])  # noqa: E731
        for i in range(nbuf):
            fn(i)
        ms = time_events(torch, fn, 2000, stream)
        # single calls: events around each call on its stream, host wall time
        # from the call to the completion of a synchronize
        lat_ev, lat_host = [], []
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        for i in range(1000):
            t0 = time.perf_counter()
            e0.record(stream)
            fn(i)
            e1.record(stream)
            e1.synchronize()
            lat_host.append((time.perf_counter() - t0) * 1e6)
            lat_ev.append(e0.elapsed_time(e1) * 1e3)
        pc = lambda v, q: round(float(np.percentile(v, q)), 2)  # noqa: E731
        result["small"] = {"value": round(n / (ms * 1e-3) / 1e9, 3), "unit": "Gpixel/s",
                           "us_per_call_back_to_back": round(ms * 1e3, 3),
                           "frac_hbm": round(8 * n / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                           "single_call_event_us": {"p50": pc(lat_ev, 50), "p99": pc(lat_ev, 99),
                                                    "max": round(max(lat_ev), 2)},
                           "single_call_host_us": {"p50": pc(lat_host, 50), "p99": pc(lat_host, 99),
                                                   "max": round(max(lat_host), 2)},
                           "calls": 1000,
                           "workload": "256x256 FP32, 3x3 Gaussian sigma 1.0, seed 0; launch-bound (512 KiB)"}
        log("small: %.2f us/call back to back; single call p50 %.2f us (events), %.2f us (host)" % (
            ms * 1e3, pc(lat_ev, 50), pc(lat_host, 50)))
        del xs, os_

    # ---- 1080p RGB uint8 7x7 -------------------------------------------------
    if "rgb" not in skip:
        cfg = synth.config_rgb()
        xu = torch.from_numpy(cfg.image).to(dev)
        ou = torch.empty_like(xu)
        fu = torch.from_numpy(cfg.filt).to(dev)
        fn = lambda i: pf.filter2d_u8(xu, fu, cfg.shift, out=ou)  # noqa: E731
        fn(0)
        ms_host = time_events(torch, fn, 200, stream)

        def graph_ms():
            # A 6-10 us kernel launched back to back from Python is timed by
            # the host's launch rate as much as by the GPU: the rate reported
            # is that of the same calls captured once in a graph and replayed.
            side = torch.cuda.Stream()
            side.wait_stream(stream)
            with torch.cuda.stream(side):
                fn(0)
            stream.wait_stream(side)
            torch.cuda.synchronize()
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g):
                for _ in range(20):
                    fn(0)
            g.replay()
            torch.cuda.synchronize()
            t = time_events(torch, lambda i: g.replay(), 10, stream) / 20
            del g
            return t

        npx = cfg.c * cfg.h * cfg.w
        e = pf.tune_lookup(pf.KIND_U8, cfg.r, npx)
        ms = graph_ms()
        # The v_dot4 kernel at its tuned shape, for comparison.
        pf.tune_set([pf.TuneEntry(kind=pf.KIND_U8, r=cfg.r, size_class=2, variant=pf.VAR_DIRECT, rows_per_wave=16,
                                  waves_per_group=1, us=0.0, context=pf.TUNE_SINGLE)])
        ms_dot4 = graph_ms()
        pf.tune_set([e])
        dot4 = npx * (2 * cfg.r + 1) * ((2 * cfg.r + 1 + 3) // 4)
        ops = 2 * npx * (2 * cfg.r + 1) ** 2   # algorithmic int8 multiply-adds x 2
        result["rgb_u8"] = {"value": round(npx / (ms * 1e-3) / 1e9, 3), "unit": "Gpixel/s (pixels x channels)",
                            "variant": "mfma_i8" if e.variant == pf.VAR_MFMA else "dot4",
                            "rows_per_wave": e.rows_per_wave, "waves_per_group": e.waves_per_group,
                            "us_per_call": round(ms * 1e3, 2),
                            "us_per_call_from_python": round(ms_host * 1e3, 2),
                            "us_per_call_dot4": round(ms_dot4 * 1e3, 2),
                            "timing": "20 calls captured in a graph, replayed 10 times",
                            "achieved_GBs": round(2 * npx / (ms * 1e-3) / 1e9, 1),
                            "frac_hbm": round(2 * npx / (ms * 1e-3) / (HBM_PEAK_GBS * 1e9), 4),
                            "int8_TOPs_algorithmic": round(ops / (ms * 1e-3) / 1e12, 2),
                            "frac_mfma_int8_peak": round(ops / (ms * 1e-3) / MFMA_INT8_PEAK, 4),
                            "dot4_kernel_frac_alu_dot4": round(dot4 / (ms_dot4 * 1e-3) / VALU_LANE_OPS, 4),
                            "dot4_kernel_frac_of_dot4_probe": (
                                round(dot4 / (ms_dot4 * 1e-3) / probes["dot4_lane_ops_per_s"], 4)
                                if "dot4_lane_ops_per_s" in probes else None),
                            "workload": "3x1080x1920 uint8 planar, 7x7 int8 weights in -8..8, shift 6, seed 2"}
        log("rgb_u8: %.2f us/call (graph replay, %s), %.2f us/call from Python; v_dot4 kernel %.2f us" % (
            ms * 1e3, result["rgb_u8"]["variant"], ms_host * 1e3, ms_dot4 * 1e3))
        # Every radius on the same image: the matrix cores (16-row wave
        # tiles, four waves) against v_dot4 (16-row single-wave tiles), with
        # seeded int8 weights in -8..8.
        radii = {}
        wrng = np.random.default_rng(20)
        for r in range(1, pf.PF_U8_MFMA_R_MAX + 1):
            fr = torch.from_numpy(wrng.integers(-8, 9, (2 * r + 1, 2 * r + 1)).astype(np.int8)).to(dev)
            fn = lambda i, fr=fr: pf.filter2d_u8(xu, fr, cfg.shift, out=ou)  # noqa: E731
            t = {}
            for name, var, wpg in (("mfma_us", pf.VAR_MFMA, 4), ("dot4_us", pf.VAR_DIRECT, 1)):
                pf.tune_set([pf.TuneEntry(kind=pf.KIND_U8, r=r, size_class=2, variant=var, rows_per_wave=16,
                                          waves_per_group=wpg, us=0.0, context=pf.TUNE_SINGLE)])
                t[name] = round(graph_ms() * 1e3, 2)
            radii[str(r)] = t
        # Back to the table the run uses: the one it loaded, or the one an
        # autotuning run has written by now (the batch section writes it).
        pf.tune_reset()
        table = args.autotune if args.autotune else args.tune
        if os.path.exists(table):
            pf.tune_load(table)
        result["rgb_u8_radii"] = {"unit": "us per call (graph replay), 3x1080x1920 uint8", "by_radius": radii}
        log("rgb_u8 by radius (matrix cores / v_dot4, us): " + ", ".join(
            "r%s %.2f/%.2f" % (k, v["mfma_us"], v["dot4_us"]) for k, v in radii.items()))

    # ---- serving ------------------------------------------------------------
    if "serve" not in skip and args.serve_seconds > 0:
        tr = synth.arrival_trace(rate=args.serve_rate, duration=args.serve_seconds)
        pool = synth.serve_pool()
        offs = np.zeros(pool.n, np.int64)
        o = 0
        for i in range(pool.n):
            offs[i] = o
            o += int(pool.h[i] * pool.w[i])
            o = (o + 63) // 64 * 64
        arena = np.zeros(o, np.float32)
        for i in range(pool.n):
            arena[offs[i]:offs[i] + pool.images[i].size] = pool.images[i].ravel()
        pool_dev = torch.from_numpy(arena).to(dev)
        del arena
        # per-request Gaussian fx = fy, packed on the host
        fls, foffs = [], np.zeros(tr.n, np.int64)
        fo = 0
        for i in range(tr.n):
            g = synth.gaussian_1d(int(tr.r[i]), float(tr.sigma[i]))
            fls.append(g)
            fls.append(g)
            foffs[i] = fo
            fo += 2 * g.size
        flt = np.concatenate(fls)
        pi = tr.pool_index
        hh, ww = pool.h[pi], pool.w[pi]
        log("serve: %d requests over %.0f s at %.0f req/s" % (tr.n, args.serve_seconds, args.serve_rate))
        srv = pf.Server(64 << 30, n_streams=SERVE_STREAMS, max_batch=SERVE_MAX_BATCH, max_queue=1 << 20)
        st = srv.run_trace((tr.t * 1e9).astype(np.int64), hh, ww, tr.r, offs[pi], foffs, pool_dev, flt)
        srv.close()
        result["serve"] = {"requests": tr.n, "rate_req_s": args.serve_rate, "seconds": args.serve_seconds,
                           "p50_us": round(st["p50_us"], 1), "p99_us": round(st["p99_us"], 1),
                           "p999_us": round(st["p999_us"], 1), "max_us": round(st["max_us"], 1),
                           "gpx_per_s": round(st["gpx_per_s"], 4), "batches": st["batches"],
                           "mean_batch": round(st["mean_batch"], 2), "budget_bytes": 64 << 30,
                           "workload": "open-loop Poisson arrivals, seed 4; device-resident pool of 1024 images "
                                       "(seed 40) sized as the batch; r 1..4; separable Gaussians"}
        log("serve: p50 %.1f us p99 %.1f us, %.3f Gpx/s, mean batch %.2f" % (st["p50_us"], st["p99_us"],
                                                                          st["gpx_per_s"], st["mean_batch"]))
        # Arrival-rate sweep up to saturation (about 100,000 requests at
        # 2,000,000 req/s, about 630 Gpx/s offered, and 200,000 at 4,000,000
        # req/s, about 1,270 Gpx/s, both above what the GPU can drain): what
        # continuous batching sustains as the load grows; the plain section
        # above is the one-launch-per-image rate.
        def trace_filters(tr_):
            fls_, fo_ = [], np.zeros(tr_.n, np.int64)
            o_ = 0
            for i in range(tr_.n):
                g = synth.gaussian_1d(int(tr_.r[i]), float(tr_.sigma[i]))
                fls_ += [g, g]
                fo_[i] = o_
                o_ += 2 * g.size
            return np.concatenate(fls_), fo_

        sweep = []
        for rate, secs, seed in ((2.0e4, 3.0, 8), (2.0e5, 0.5, 9), (2.0e6, 0.05, 7), (4.0e6, 0.05, 12)):
            tr_ = synth.arrival_trace(rate=rate, duration=secs, seed=seed)
            flt_, fo_ = trace_filters(tr_)
            pi_ = tr_.pool_index
            srv = pf.Server(64 << 30, n_streams=SERVE_STREAMS, max_batch=SERVE_MAX_BATCH, max_queue=1 << 20)
            ss = srv.run_trace((tr_.t * 1e9).astype(np.int64), pool.h[pi_], pool.w[pi_], tr_.r, offs[pi_], fo_,
                               pool_dev, flt_)
            srv.close()
            sweep.append({"offered_req_s": rate, "seconds": secs, "requests": tr_.n,
                          "offered_gpx_s": round(float((pool.h[pi_].astype(np.float64) * pool.w[pi_]).sum()) / secs
                                                 / 1e9, 3),
                          "gpx_per_s": round(ss["gpx_per_s"], 3), "mean_batch": round(ss["mean_batch"], 2),
                          "p50_us": round(ss["p50_us"], 1), "p99_us": round(ss["p99_us"], 1),
                          "max_us": round(ss["max_us"], 1)})
            log("serve at %.0f req/s: %.1f Gpx/s, mean batch %.1f, p50 %.0f us p99 %.0f us" % (
                rate, ss["gpx_per_s"], ss["mean_batch"], ss["p50_us"], ss["p99_us"]))
        result["serve_sweep"] = {"points": sweep, "seeds": [8, 9, 7, 12], "n_streams": SERVE_STREAMS,
                                 "max_batch": SERVE_MAX_BATCH,
                                 "workload": "open-loop Poisson arrivals at each rate, same pool and request mix; "
                                             "the last two points are past saturation"}
        result["serve_saturation"] = dict(sweep[-1])
        # Upload mode: each request's image comes from host memory and is
        # copied into the server's arena at submit (PCIe-inclusive latency).
        up_secs = min(10.0, args.serve_seconds)
        tr_ = synth.arrival_trace(rate=args.serve_rate, duration=up_secs, seed=11)
        flt_, fo_ = trace_filters(tr_)
        pi_ = tr_.pool_index
        host_pool = [pool.images[i] for i in range(pool.n)]
        srv = pf.Server(64 << 30, n_streams=SERVE_STREAMS, max_batch=SERVE_MAX_BATCH, max_queue=1 << 20)
        t_start = time.perf_counter_ns()
        tickets = []
        for i in range(tr_.n):
            due = t_start + int(tr_.t[i] * 1e9)
            while time.perf_counter_ns() < due:
                pass
            k = 2 * int(tr_.r[i]) + 1
            tickets.append(srv.submit(host_pool[pi_[i]], int(tr_.r[i]), pf.KIND_SEP, flt_[fo_[i]:fo_[i] + 2 * k],
                                      arrival_ns=0))
            # release whatever finished (keeps the arena small)
            while len(tickets) > 256 and srv.poll(tickets[0]):
                srv.release(tickets.pop(0))
        for t in tickets:
            srv.wait(t)
            srv.release(t)
        su = srv.stats()
        srv.close()
        result["serve_upload"] = {"requests": tr_.n, "rate_req_s": args.serve_rate, "seconds": up_secs,
                                  "p50_us": round(su["p50_us"], 1), "p99_us": round(su["p99_us"], 1),
                                  "max_us": round(su["max_us"], 1), "gpx_per_s": round(su["gpx_per_s"], 4),
                                  "mean_batch": round(su["mean_batch"], 2),
                                  "workload": "as the served stream, but each image submitted from host memory "
                                              "(copied host to device inside the request; latency measured from "
                                              "submit)"}
        log("serve upload: p50 %.1f us p99 %.1f us" % (su["p50_us"], su["p99_us"]))
        # Mixed kinds: filters beside sum/mean and histogram requests on the
        # same server (the reductions batched with the filters), inputs
        # device-resident, latency measured from submit.
        mix_secs = min(5.0, args.serve_seconds)
        tr_ = synth.arrival_trace(rate=args.serve_rate, duration=mix_secs, seed=13)
        flt_, fo_ = trace_filters(tr_)
        pi_ = tr_.pool_index
        kinds = np.random.default_rng(14).choice(3, size=tr_.n, p=[0.6, 0.2, 0.2])
        gu = torch.Generator(device=dev).manual_seed(15)
        pool_u8 = torch.randint(0, 256, (int(offs[-1] + pool.h[-1] * pool.w[-1]),), dtype=torch.uint8, device=dev,
                                generator=gu)
        torch.cuda.synchronize()
        srv = pf.Server(64 << 30, n_streams=SERVE_STREAMS, max_batch=SERVE_MAX_BATCH, max_queue=1 << 20)
        t_start = time.perf_counter_ns()
        tickets = []
        for i in range(tr_.n):
            due = t_start + int(tr_.t[i] * 1e9)
            while time.perf_counter_ns() < due:
                pass
            j = int(pi_[i])
            o, hh_, ww_ = int(offs[j]), int(pool.h[j]), int(pool.w[j])
            if kinds[i] == 0:
                k = 2 * int(tr_.r[i]) + 1
                tk = srv.submit(pool_dev[o:o + hh_ * ww_].view(hh_, ww_), int(tr_.r[i]), pf.KIND_SEP,
                                flt_[fo_[i]:fo_[i] + 2 * k])
            elif kinds[i] == 1:
                tk = srv.submit_sum(pool_dev[o:o + hh_ * ww_])
            else:
                tk = srv.submit_hist(pool_u8[o:o + hh_ * ww_])
            tickets.append(tk)
            while len(tickets) > 256 and srv.poll(tickets[0]):
                srv.release(tickets.pop(0))
        for t in tickets:
            srv.wait(t)
            srv.release(t)
        sm = srv.stats()
        srv.close()
        del pool_u8
        result["serve_mixed"] = {"requests": tr_.n, "filters": int((kinds == 0).sum()), "sums": int((kinds == 1).sum()),
                                 "histograms": int((kinds == 2).sum()), "rate_req_s": args.serve_rate,
                                 "seconds": mix_secs, "p50_us": round(sm["p50_us"], 1),
                                 "p99_us": round(sm["p99_us"], 1), "max_us": round(sm["max_us"], 1),
                                 "filter_gpx_per_s": round(sm["gpx_per_s"], 4), "batches": sm["batches"],
                                 "mean_batch": round(sm["mean_batch"], 2),
                                 "workload": "Poisson arrivals (seed 13), 60% separable filters / 20% float64 "
                                             "sum+mean of an FP32 pool image / 20% 256-bin histogram of a uint8 "
                                             "image of the same size (seed 15); device-resident inputs; latency "
                                             "from submit"}
        log("serve mixed: p50 %.1f us p99 %.1f us, mean batch %.2f" % (sm["p50_us"], sm["p99_us"],
                                                                     sm["mean_batch"]))

    # ---- CPU baseline: the oracle on one core and on all host cores -----------
    if "cpu" not in skip:
        # The oracle's own C functions, unchanged, timed by its OpenMP driver
        # (oracle/time_oracle.c): one thread, then every host thread this
        # process may use (bands of output rows with their halo rows, one
        # image per task for the batch; bit-identical to one thread).
        # Median of 5 passes on one thread and of 15 on all threads: about
        # 25 s of CPU work for the batch, so the sample is bounded but not
        # a single short pass.
        import platform

        import oracle

        cores = len(os.sched_getaffinity(0))
        model = ""
        try:
            for ln in open("/proc/cpuinfo"):
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
        except OSError:
            pass
        cpu_info = {"nproc": os.cpu_count(), "threads_used": cores, "model": model or platform.processor(),
                    "omp_num_threads_env": os.environ.get("OMP_NUM_THREADS")}
        bpix = pk.pixels
        bout = np.empty_like(bpix)
        t1 = oracle.time_batch_sep(pk.h, pk.w, pk.r, pk.pix_off, bpix, pk.filters, pk.filt_off, bout, 1, 5)
        tn = oracle.time_batch_sep(pk.h, pk.w, pk.r, pk.pix_off, bpix, pk.filters, pk.filt_off, bout, cores, 15)
        result["cpu_baseline"] = {"value": round(px / tn / 1e9, 5), "unit": "Gpixel/s", "cores": cores,
                                  "kind": "oracle",
                                  "sample": "the whole 512-image batch (%d px), separable C oracle, one image per "
                                            "OpenMP task on %d threads, median of 15 passes (%.2f s each; "
                                            "with the 5 one-thread passes about %.0f s of CPU work)"
                                            % (px, cores, tn, 5 * t1 + 15 * tn * cores),
                                  "one_core": {"value": round(px / t1 / 1e9, 5), "unit": "Gpixel/s",
                                               "sample": "the whole batch on one thread, median of 5 (%.2f s)" % t1},
                                  "host": cpu_info}
        log("cpu oracle (batch): %.4f Gpx/s on %d threads, %.4f Gpx/s on one" % (px / tn / 1e9, cores, px / t1 / 1e9))
        per = {}
        cs, cl, cu = synth.config_small(), synth.config_large(), synth.config_rgb()
        cases = (("small_2d", "2d", cs.image, cs.f2d, cs.h * cs.w),
                 ("large_2d", "2d", cl.image, cl.f2d, cl.h * cl.w),
                 ("large_sep", "sep", cl.image, np.concatenate([cl.f1d, cl.f1d]), cl.h * cl.w),
                 ("rgb_u8", "u8", cu.image, cu.filt, cu.image.size))
        for name, kind, img, flt, npx in cases:
            o = np.empty_like(img)
            r1 = oracle.time_image(kind, img, flt, o, 1, 3)
            rn = oracle.time_image(kind, img, flt, o, cores, 3)
            per[name] = {"one_core_gpx_s": round(npx / r1 / 1e9, 5), "all_cores_gpx_s": round(npx / rn / 1e9, 5),
                         "one_core_s": round(r1, 4), "all_cores_s": round(rn, 4), "pixels": int(npx)}
        per["batch512_sep"] = {"one_core_gpx_s": round(px / t1 / 1e9, 5), "all_cores_gpx_s": round(px / tn / 1e9, 5),
                               "one_core_s": round(t1, 4), "all_cores_s": round(tn, 4), "pixels": int(px)}
        if "serve" in result:
            per["served_capacity"] = {"all_cores_gpx_s": round(px / tn / 1e9, 5),
                                      "offered_gpx_s": result["serve"]["gpx_per_s"],
                                      "note": "CPU capacity on the batch's image mix against the served stream's rate"}
        result["cpu_per_config"] = {"threads": cores, "host": cpu_info, "configs": per}
        log("cpu per config: %s" % ", ".join("%s %.3f/%.3f" % (k, v["one_core_gpx_s"], v["all_cores_gpx_s"])
                                              for k, v in per.items() if "one_core_gpx_s" in v))

    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
