#!/usr/bin/env python3
"""Benchmark of the Image-GS renderer hot path on one MI355X.

Workload: the texture-stack fit, 2048 x 2048 with n = 9 float32 channels (three synthetic
3-channel maps), N = 100,000 Gaussians, top-K = 10, 16 x 16 tiles.  One step is one fitting
iteration: binning (footprint bound, scan, pair emission, radix sort, tile ranges), forward
raster with the L1 loss and its gradient record fused in, adjoint raster with its per-Gaussian
reduction, and the fused Adam step, replayed as one HIP graph with all inputs resident in HBM.

Printed JSON line: ``value`` is Gaussian-pixel evaluations per second over whole fitting
iterations (E_fwd = sum over tiles of |S_j| times the tile's pixel count, per iteration); the
``roofline`` object reports the dominant raster kernel's algorithmic VALU work divided by its
average duration, timed live with HIP events on the stream it runs on; ``cpu_baseline`` is the
FP64 oracle timed on the host's cores over a sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("fwd+bwd Gaussian-pixel evals/s and fit iters/s at 2048², 100k G; "
          "×batched vs plain")
# VALU issue peak: 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz (one lane-op per lane per clock, packed
# FP32 disabled); the algorithmic work below is counted in the same lane-ops.
PEAK_LANE_OPS = 256 * 4 * 16 * 2.4e9
HBM_PEAK = 8.0e12


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def tile_pixels(H, W, tile=16):
    tx, ty = (W + tile - 1) // tile, (H + tile - 1) // tile
    wx = np.full(tx, tile)
    wx[-1] = W - tile * (tx - 1)
    hy = np.full(ty, tile)
    hy[-1] = H - tile * (ty - 1)
    return (hy[:, None] * wx[None, :]).ravel()


def fwd_valu_ops(e_fwd, hw, n, fused_l1=True):
    # per (pixel, candidate): 2 sub + 4 (two 2-term dot products) + 2 (squared norm) + 1 compare;
    # per pixel: K exps (4 each) and subs, K*n multiply-adds, n scalings, one reciprocal; the
    # fused L1 epilogue adds per channel a difference, its sign and magnitude, g.c_r and the two
    # loss sums (8 lane-ops).  The kernel skips candidates that provably cannot enter a list;
    # the count is the method's (every member of S_j ranked at every pixel of its tile).
    return 9.0 * e_fwd + (60.0 + 10.0 * n + (8.0 * n if fused_l1 else 0.0)) * hw


def bwd_valu_ops(e_bwd, n):
    # per retained (pixel, Gaussian): recompute e, q, w (~12 + exp), g.(c_i - c_r) (n+2),
    # five geometry products and n colour products, 5+n accumulations
    return (35.0 + 3.0 * n) * e_bwd


def cpu_model():
    """The host CPU's model name (as lscpu reports it), from /proc/cpuinfo."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.lower().startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline(params, H, W, K, grad_img, budget_s=15.0):
    """The FP64 oracle (forward + adjoint) on the host's cores: three timed runs over one whole
    frame of the workload on all threads (the median is reported), then one thread over an evenly
    strided sample of the frame's tiles sized to about a quarter of ``budget_s``."""
    from oracle import cref
    p64 = params.astype(np.float64)
    T = cref.num_tiles(H, W)
    tiles = np.arange(T, dtype=np.int32)
    counts, _ = cref.tile_lists(p64, H, W, tiles=tiles)
    e_tile = counts.astype(np.float64) * tile_pixels(H, W)
    cores = cref.max_threads()

    def timed(tl, nthreads):
        t0 = time.perf_counter()
        cref.render_tiles(p64, H, W, K, tiles=tl, grad_img=grad_img, want=("img",),
                          nthreads=nthreads)
        dt = time.perf_counter() - t0
        return float(e_tile[tl].sum()) / dt, dt

    runs = [timed(tiles, cores) for _ in range(3)]
    rates = sorted(r for r, _ in runs)
    frame_s = sorted(dt for _, dt in runs)[1]
    # one thread: a strided sample of tiles (every stride-th tile of the frame)
    stride = max(1, int(math.ceil(frame_s * cores / max(budget_s / 4.0, 0.5))))
    one_rate, one_dt = timed(tiles[::stride], 1)
    return {"value": rates[1], "unit": "Gaussian-pixel evals/s", "cores": cores, "kind": "oracle",
            "cpu_model": cpu_model(), "runs": [round(r, 1) for r in rates],
            "sample": f"median of 3 runs over one whole frame of the workload ({T} tiles, all "
                      f"pixels, {frame_s:.2f} s each) on {cores} threads, forward + adjoint in "
                      f"FP64 with a seeded upstream gradient",
            "one_core": {"value": one_rate, "unit": "Gaussian-pixel evals/s", "cores": 1,
                         "sample": f"every {stride}th tile of the frame ({len(tiles[::stride])} "
                                   f"tiles), one thread, {one_dt:.1f} s"}}


def paper_context(torch, dev, K=10):
    """Render and fit-iteration times at the paper's measured operating points (2048^2 RGB,
    10K and 50K Gaussians), for comparison with its A6000 timings (context only)."""
    from paper_2407_01866_amd import synth
    from paper_2407_01866_amd.fit import PlainFitter
    from paper_2407_01866_amd.render import Renderer
    out = {}
    tgt = torch.from_numpy(synth.gen_image(9000, 2048, 2048, 3, 200)).to(dev)
    for N in (10000, 50000):
        p = torch.from_numpy(synth.gen_gaussians(9500 + N, 2048, 2048, N, 3, 5.0, 5.0)).to(dev)
        r = Renderer(N, 3, 2048, 2048, K, device=dev)
        r.render(p, keep_state=False)
        img = torch.empty((3, 2048, 2048), device=dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(20):
            r.render_into(p, img, None)
        torch.cuda.synchronize()
        render_ms = (time.perf_counter() - t0) / 20 * 1e3
        rec = {"render_ms": round(render_ms, 4)}
        for key, wgt in (("fit_iter_ms_l1", 0.0), ("fit_iter_ms_l1_ssim", 0.1)):
            f = PlainFitter(tgt, p, K, headroom=3.0, ssim_weight=wgt)
            init = f.snapshot()
            f.advance_to(23, use_graph=False)      # sizes the pair buffer for this trajectory
            f.restore(init)
            f.capture()
            for _ in range(3):
                f.step()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(20):
                f.step()
            torch.cuda.synchronize()
            iter_ms = (time.perf_counter() - t0) / 20 * 1e3
            rec[key] = round(iter_ms, 4) if f.steps_done() == 23 else None
            del f
        out[f"N{N // 1000}k"] = rec
    out["paper_a6000"] = {"N10k": {"render_ms": 3.7, "fit_iter_ms": 18.74},
                          "N50k": {"render_ms": 4.5, "fit_iter_ms": 26.32},
                          "note": "Sec. 4.4, NVIDIA A6000, L1 + 0.1 SSIM loss (compare with "
                                  "fit_iter_ms_l1_ssim), Gaussians at init scale 5 px here"}
    return out


# Algorithmic work of the L1 + SSIM loss per image value (one channel of one pixel): the forward
# blurs five moments with a separable 11-tap window (5 x 11 horizontal + 5 x 11 vertical
# multiply-adds and 3 products) and evaluates the map and its three partial derivatives (about
# 30 operations); the adjoint blurs the three partials (3 x 22) and combines them with the L1
# sign (6).  Bytes: image and target read twice (16), three fp32 partial maps written and read
# (24), the gradient written (4).
SSIM_OPS_PER_VALUE = 5 * 11 * 2 + 3 + 30 + 3 * 22 + 6
SSIM_BYTES_PER_VALUE = 16 + 24 + 4


def _ssim_calls(torch, dev, w, image, target, calls):
    """Average duration of igs_l1_ssim_loss_grad (library phase timer: HIP events on the call's
    stream)."""
    from paper_2407_01866_amd import _native as nat
    n, H, W = w.n, w.H, w.W
    g = torch.empty_like(image)
    loss = torch.zeros(4, dtype=torch.float64, device=dev)
    ws = torch.empty(nat.igs_l1_ssim_workspace_size(n, H, W), dtype=torch.uint8, device=dev)
    for _ in range(3):
        nat.igs_l1_ssim_loss_grad(image, target, n, H, W, 0.1, g, loss, ws, ws.numel())
    torch.cuda.synchronize()
    nat.igs_timing_read(reset=True)
    nat.igs_timing_enable(True)
    torch.cuda._sleep(200_000_000)          # hold the stream while the calls are enqueued
    for _ in range(calls):
        nat.igs_l1_ssim_loss_grad(image, target, n, H, W, 0.1, g, loss, ws, ws.numel())
    ph = nat.igs_timing_read(reset=True)
    nat.igs_timing_enable(False)
    call_ms = ph["loss"][0] / ph["loss"][1]
    log(f"[bench] L1 + SSIM loss call: {call_ms:.4f} ms")
    return call_ms


def ssim_step(torch, dev, w, image, target, calls=20, iters=10):
    """The paper's full loss, L1 + 0.1 (1 - SSIM), at the benchmark workload: the loss-and-gradient
    call alone (HIP events on its stream, library phase timer) and a whole fitting iteration with
    it (render, loss, adjoint, Adam as one HIP graph)."""
    from paper_2407_01866_amd.fit import PlainFitter
    call_ms = _ssim_calls(torch, dev, w, image, target, calls)
    values = w.n * w.H * w.W
    ops = SSIM_OPS_PER_VALUE * values
    byts = SSIM_BYTES_PER_VALUE * values
    f = PlainFitter(target, torch.from_numpy(w.gaussians()).to(dev), w.K, ssim_weight=0.1)
    init = f.snapshot()
    f.advance_to(iters + 3, use_graph=False)
    f.restore(init)
    f.capture()
    for _ in range(3):
        f.step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(iters):
        f.step()
    torch.cuda.synchronize()
    iter_ms = (time.perf_counter() - t0) / iters * 1e3
    ok = f.steps_done() == iters + 3
    return {"loss": "L1 + 0.1 (1 - SSIM), 11x11 Gaussian window sigma 1.5",
            "loss_call_ms": round(call_ms, 4),
            "values_per_s": values / (call_ms * 1e-3),
            "roofline": {"bound": "alu+hbm", "alu_frac": round(ops / (call_ms * 1e-3) /
                                                              PEAK_LANE_OPS, 4),
                         "hbm_frac": round(byts / (call_ms * 1e-3) / HBM_PEAK, 4),
                         "work_per_call": f"{ops:.4g} lane-ops (fp64 forward moments), "
                                          f"{byts:.4g} B"},
            "fit_iter_ms": round(iter_ms, 4) if ok else None,
            "ssim_after_iters": round(f.ssim(), 6)}


def decode_step(torch, dev, w, params, M=1 << 22, calls=10):
    """Random access at the benchmark workload: binning alone (once per decoded set), then M
    points drawn uniformly over the image decoded per call (HIP events on the call's stream).
    Algorithmic work per point as the forward's per pixel: 9 lane-ops per member of the point's
    S_j (the mean |S_j| over the image, which uniform points sample) plus 60 + 10n for the
    blend."""
    from paper_2407_01866_amd import _native as nat
    from paper_2407_01866_amd.render import Renderer
    r = Renderer(w.N, w.n, w.H, w.W, w.K, device=dev)
    saved = r.bin(params)
    nat.igs_timing_read(reset=True)
    nat.igs_timing_enable(True)
    for _ in range(5):
        r.bin(params)
    ph = nat.igs_timing_read(reset=True)
    nat.igs_timing_enable(False)
    bin_ms = ph["binning"][0] / ph["binning"][1]
    g = torch.Generator(device=dev)
    g.manual_seed(123)
    pts = torch.stack([torch.rand(M, generator=g, device=dev) * w.W,
                       torch.rand(M, generator=g, device=dev) * w.H], dim=1).contiguous()
    out = torch.empty((M, w.n), device=dev)
    for _ in range(2):
        r.query_into(params, saved, pts, out)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda._sleep(200_000_000)
    e0.record()
    for _ in range(calls):
        r.query_into(params, saved, pts, out)
    e1.record()
    torch.cuda.synchronize()
    q_ms = e0.elapsed_time(e1) / calls
    st = r.status_of(saved).cpu()
    mean_sj = float(st[nat.STAT_EVALS_FWD]) / (w.H * w.W)
    ops = (9.0 * mean_sj + 60.0 + 10.0 * w.n) * M
    return {"bin_ms": round(bin_ms, 4), "points": M, "query_ms": round(q_ms, 4),
            "points_per_s": M / (q_ms * 1e-3), "mean_candidates_per_point": round(mean_sj, 2),
            "roofline": {"bound": "alu", "achieved": round(ops / (q_ms * 1e-3) / 1e12, 3),
                         "peak": round(PEAK_LANE_OPS / 1e12, 2), "unit": "Tlane-op/s",
                         "frac": round(ops / (q_ms * 1e-3) / PEAK_LANE_OPS, 4)}}


PROFILES = os.path.join(ROOT, "profiles")
TRAFFIC_FILE = os.path.join(PROFILES, "hbm_traffic_raster_texture-2048x2048-n9-N100000.txt")
KERNEL_SOURCES = {"raster_fwd": "raster_fwd.hip", "raster_bwd": "raster_bwd.hip",
                  "raster_fit": "raster_fit.hip"}
# headers whose device code the raster kernels inline
KERNEL_HEADERS = ("raster_tile.hpp", "raster_common.hpp")
PROFILE_CMDS = {
    "decode_trace": "rocprofv3 --kernel-trace --stats -f csv -d gpurun_out/qprof/trace -o t -- "
                    "python3 bench.py --decode-profile",
    "decode_sq": "rocprofv3 --pmc SQ_INSTS_VALU SQ_WAVES SQ_INSTS_LDS SQ_THREAD_CYCLES_VALU "
                 "SQ_INSTS_VMEM_RD SQ_WAIT_INST_ANY SQ_BUSY_CYCLES GRBM_GUI_ACTIVE "
                 "--kernel-include-regex query -f csv -d gpurun_out/qprof/sq -o p -- python3 "
                 "bench.py --decode-profile",
    "decode_fetch": "rocprofv3 --pmc FETCH_SIZE --kernel-include-regex query -f csv -d "
                    "gpurun_out/qprof/fetch -o p -- python3 bench.py --decode-profile",
    "decode_write": "rocprofv3 --pmc WRITE_SIZE --kernel-include-regex query -f csv -d "
                    "gpurun_out/qprof/write -o p -- python3 bench.py --decode-profile",
    "trace": "rocprofv3 --kernel-trace --stats -f csv -d gpurun_out/prof_trace -o trace -- "
             "python3 bench.py --steps 10 --warmup 3 --no-cpu-baseline --no-context --batch-iters 0 --large-iters 0 --no-ssim --no-decode "
             "--launch-config 0,0,1",
    "fetch": "rocprofv3 --pmc FETCH_SIZE --kernel-include-regex 'raster|elementwise' -f csv "
             "-d gpurun_out/pmc_fetch -o fetch -- python3 bench.py --steps 3 --warmup 1 "
             "--no-cpu-baseline --no-context --batch-iters 0 --large-iters 0 --no-ssim --no-decode --launch-config 0,0,1",
    "write": "rocprofv3 --pmc WRITE_SIZE (otherwise as fetch) -d gpurun_out/pmc_write -o write",
    "copy_fetch": "rocprofv3 --pmc FETCH_SIZE -f csv -d gpurun_out/pmc_copy_fetch -o cf -- "
                  "python3 bench.py --copy-calibration",
    "copy_write": "rocprofv3 --pmc WRITE_SIZE -f csv -d gpurun_out/pmc_copy_write -o cw -- "
                  "python3 bench.py --copy-calibration",
    "ssim": "rocprofv3 --kernel-trace --stats -f csv -d gpurun_out/prof_ssim -o ssim -- "
            "python3 bench.py --ssim-profile",
    "valu_ssim": "rocprofv3 --pmc SQ_ACTIVE_INST_VALU SQ_THREAD_CYCLES_VALU SQ_INSTS_VALU "
                 "SQ_INSTS_LDS SQ_WAVES SQ_WAIT_INST_LDS GRBM_GUI_ACTIVE GRBM_COUNT "
                 "--kernel-include-regex ssim -f csv -d gpurun_out/pmc_ssim -o s -- python3 "
                 "bench.py --ssim-profile",
    "valu": "rocprofv3 --pmc SQ_ACTIVE_INST_VALU SQ_THREAD_CYCLES_VALU SQ_INSTS_VALU SQ_INSTS_LDS "
            "SQ_WAVES SQ_BUSY_CYCLES GRBM_GUI_ACTIVE GRBM_COUNT --kernel-include-regex raster "
            "-f csv -d gpurun_out/pmc_valu -o valu -- python3 bench.py --steps 3 --warmup 1 "
            "--no-cpu-baseline --no-context --batch-iters 0 --large-iters 0 --no-ssim --no-decode "
            "--launch-config 0,0,1",
}
VALU_FILE = os.path.join(PROFILES, "valu_counters_raster_texture-2048x2048-n9-N100000.txt")


def kernel_source_hash(kernel):
    import hashlib
    h = hashlib.sha256()
    for name in (KERNEL_SOURCES[kernel],) + KERNEL_HEADERS:
        h.update(open(os.path.join(ROOT, "paper_2407_01866_amd", "csrc", name), "rb").read())
    return h.hexdigest()[:16]


def summarize_profiles(out_dir):
    """Write the committed text summaries of a profiling run (rocprofv3 CSVs under out_dir)."""
    import csv
    import collections
    os.makedirs(PROFILES, exist_ok=True)
    rows = list(csv.DictReader(open(os.path.join(out_dir, "prof_trace", "trace_kernel_stats.csv"))))
    # the spin kernel that holds the stream during the timed eager iterations is not ours
    rows = [r for r in rows if "spin_kernel" not in r["Name"]]
    total = sum(float(r["TotalDurationNs"]) for r in rows)
    for r in rows:
        r["Percentage"] = 100.0 * float(r["TotalDurationNs"]) / total
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    lines = ["# Kernel trace: fitting iteration, texture-2048x2048-n9-N100000 (2048^2, n=9, "
             "N=100k, K=10)", "", "Command (run from the repository root on the GPU box):", "",
             "    " + PROFILE_CMDS["trace"], "",
             "| kernel | calls | avg us | min us | max us | share % |", "|---|---|---|---|---|---|"]
    for r in rows[:20]:
        name = r["Name"].replace("igs::(anonymous namespace)::", "").replace("void ", "").split("(")[0]
        lines.append(f"| {name} | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
                     f"{float(r['MinNs']) / 1e3:.2f} | {float(r['MaxNs']) / 1e3:.2f} | "
                     f"{float(r['Percentage']):.2f} |")
    open(os.path.join(PROFILES, "kernel_trace_texture-2048x2048-n9-N100000.md"), "w").write(
        "\n".join(lines) + "\n")
    ssim_csv = os.path.join(out_dir, "prof_ssim", "ssim_kernel_stats.csv")
    if os.path.exists(ssim_csv):
        rows = [r for r in csv.DictReader(open(ssim_csv)) if "ssim" in r["Name"]]
        lines = ["# Kernel trace: L1 + 0.1 (1 - SSIM) loss and gradient, 2048^2, n=9 (the texture "
                 "workload's target against a render of its initial Gaussians)", "",
                 "Command (run from the repository root on the GPU box):", "",
                 "    " + PROFILE_CMDS["ssim"], "",
                 "| kernel | calls | avg us | min us | max us |", "|---|---|---|---|---|"]
        for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"])):
            name = r["Name"].replace("igs::(anonymous namespace)::", "").split("(")[0]
            lines.append(f"| {name} | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
                         f"{float(r['MinNs']) / 1e3:.2f} | {float(r['MaxNs']) / 1e3:.2f} |")
        open(os.path.join(PROFILES, "kernel_trace_ssim_texture-2048x2048-n9.md"), "w").write(
            "\n".join(lines) + "\n")

    valu_csv = os.path.join(out_dir, "pmc_valu", "valu_counter_collection.csv")
    if os.path.exists(valu_csv):
        import re
        per = collections.defaultdict(lambda: collections.defaultdict(list))
        for r in csv.DictReader(open(valu_csv)):
            m = re.search(r"(raster_\w+<[^>]*>)", r["Kernel_Name"])
            if m:
                per[m.group(1)][r["Counter_Name"]].append(float(r["Counter_Value"]))
        out = ["# VALU issue of the raster kernels, texture-2048x2048-n9-N100000 (per dispatch)",
               "# SQ_* summed over all SIMDs; GRBM_GUI_ACTIVE summed over the 8 XCDs.  A wave64",
               "# VALU instruction occupies a SIMD for 4 cycles (16 lanes, packed FP32 off), so",
               "# issue_busy = SQ_INSTS_VALU * 4 / 1024 SIMDs / (GRBM_GUI_ACTIVE / 8) and",
               "# active_lanes = SQ_THREAD_CYCLES_VALU / (64 SQ_INSTS_VALU).",
               "# command: " + PROFILE_CMDS["valu"]]
        for k, c in sorted(per.items()):
            a = {n: sum(v) / len(v) for n, v in c.items()}
            cyc = a["GRBM_GUI_ACTIVE"] / 8
            kern = next(f for f in KERNEL_SOURCES if f in k)
            out.append(f"kernel {k.replace(' ', '')} family {kern} source_sha256 "
                       f"{kernel_source_hash(kern)} dispatches {len(c['SQ_WAVES'])} "
                       f"valu_insts {a['SQ_INSTS_VALU']:.4g} lds_insts {a['SQ_INSTS_LDS']:.4g} "
                       f"cycles_per_xcd {cyc:.4g} "
                       f"issue_busy {a['SQ_INSTS_VALU'] * 4 / 1024 / cyc:.3f} "
                       f"active_lanes {a['SQ_THREAD_CYCLES_VALU'] / (64 * a['SQ_INSTS_VALU']):.3f} "
                       f"executed_lane_slots {64 * a['SQ_INSTS_VALU']:.4g}")
        open(VALU_FILE, "w").write("\n".join(out) + "\n")

    ssim_pmc = os.path.join(out_dir, "pmc_ssim", "s_counter_collection.csv")
    if os.path.exists(ssim_pmc):
        import re
        per = collections.defaultdict(lambda: collections.defaultdict(list))
        for r in csv.DictReader(open(ssim_pmc)):
            m = re.search(r"(ssim_\w+_kernel)", r["Kernel_Name"])
            if m:
                per[m.group(1)][r["Counter_Name"]].append(float(r["Counter_Value"]))
        values = 9 * 2048 * 2048
        out = ["# VALU issue of the SSIM stencils, L1 + 0.1 SSIM loss at 2048^2, n=9 (per dispatch)",
               "# issue_busy = SQ_INSTS_VALU * 4 / 1024 SIMDs / (GRBM_GUI_ACTIVE / 8); "
               "lane_ops_per_value = 64 SQ_INSTS_VALU / (n H W)",
               "# command: " + PROFILE_CMDS["valu_ssim"]]
        for k, c in sorted(per.items()):
            a = {n: sum(v) / len(v) for n, v in c.items()}
            cyc = a["GRBM_GUI_ACTIVE"] / 8
            out.append(f"kernel {k} dispatches {len(c['SQ_WAVES'])} valu_insts "
                       f"{a['SQ_INSTS_VALU']:.4g} cycles_per_xcd {cyc:.4g} issue_busy "
                       f"{a['SQ_INSTS_VALU'] * 4 / 1024 / cyc:.3f} active_lanes "
                       f"{a['SQ_THREAD_CYCLES_VALU'] / (64 * a['SQ_INSTS_VALU']):.3f} "
                       f"lane_ops_per_value {64 * a['SQ_INSTS_VALU'] / values:.4g}")
        open(os.path.join(PROFILES, "valu_counters_ssim_texture-2048x2048-n9.txt"), "w").write(
            "\n".join(out) + "\n")

    def counter(sub, fname):
        d = collections.defaultdict(list)
        for r in csv.DictReader(open(os.path.join(out_dir, sub, fname))):
            d[r["Kernel_Name"]].append(float(r["Counter_Value"]))
        return {k: sum(v) / len(v) for k, v in d.items()}

    cf = counter("pmc_copy_fetch", "cf_counter_collection.csv")
    cw = counter("pmc_copy_write", "cw_counter_collection.csv")
    copy_bytes = float(1 << 30)
    f_factor = copy_bytes / (1024.0 * max(v for k, v in cf.items() if "copy" in k.lower()))
    w_factor = copy_bytes / (1024.0 * max(v for k, v in cw.items() if "copy" in k.lower()))
    fetch = counter("pmc_fetch", "fetch_counter_collection.csv")
    write = counter("pmc_write", "write_counter_collection.csv")
    out = ["# HBM traffic of the raster kernels, texture-2048x2048-n9-N100000 (per dispatch)",
           "# FETCH_SIZE and WRITE_SIZE (KiB) from separate rocprofv3 --pmc passes, scaled by what the",
           "# same counters read for the runtime's copy of 1 GiB (bytes per counted KiB below).",
           "# commands: " + PROFILE_CMDS["fetch"], "#           " + PROFILE_CMDS["write"],
           "#           " + PROFILE_CMDS["copy_fetch"], "#           " + PROFILE_CMDS["copy_write"],
           f"copy_calibration fetch_bytes_per_kib {f_factor * 1024:.1f} write_bytes_per_kib {w_factor * 1024:.1f}"]
    for kern in KERNEL_SOURCES:
        fk = [v for k, v in fetch.items() if kern in k]
        wk = [v for k, v in write.items() if kern in k]
        if not fk or not wk:
            continue
        rb, wb = fk[0] * 1024 * f_factor, wk[0] * 1024 * w_factor
        out.append(f"kernel {kern} source_sha256 {kernel_source_hash(kern)} fetch_kib {fk[0]:.1f} "
                   f"write_kib {wk[0]:.1f} read_bytes {rb:.4g} write_bytes {wb:.4g} "
                   f"traffic_bytes {rb + wb:.4g}")
    open(TRAFFIC_FILE, "w").write("\n".join(out) + "\n")
    print("\n".join(out))
    qdir = os.path.join(out_dir, "qprof")
    if os.path.isdir(qdir):
        summarize_decode_profile(qdir, f_factor * 1024, w_factor * 1024)


def summarize_decode_profile(qdir, fetch_per_kib, write_per_kib):
    """The decode path's summary: kernel trace and SQ/traffic counters of `query_kernel` from the
    four rocprofv3 runs of bench.py --decode-profile under qdir."""
    import csv
    import collections
    import glob
    import hashlib
    import re

    def pmc(sub):
        f = glob.glob(os.path.join(qdir, sub, "**", "*counter_collection.csv"), recursive=True)[0]
        per = collections.defaultdict(list)
        for r in csv.DictReader(open(f)):
            if "query_kernel" in r["Kernel_Name"]:
                per[r["Counter_Name"]].append(float(r["Counter_Value"]))
        return {k: sum(v) / len(v) for k, v in per.items()}

    stats = glob.glob(os.path.join(qdir, "trace", "**", "*kernel_stats.csv"), recursive=True)[0]
    rows = [r for r in csv.DictReader(open(stats))
            if any(k in r["Name"] for k in ("query", "radix", "scan_block_kernel<unsigned int, unsigned int>"))]
    sq, fe, wr = pmc("sq"), pmc("fetch"), pmc("write")
    h = hashlib.sha256()
    for name in ("query.hip", "raster_common.hpp"):
        h.update(open(os.path.join(ROOT, "paper_2407_01866_amd", "csrc", name), "rb").read())
    cyc = sq["GRBM_GUI_ACTIVE"] / 8
    out = ["# Random-access decoding, texture-2048x2048-n9-N100000 (initial Gaussians): 4,194,304 "
           "uniform points per call",
           "# commands (from the repository root on the GPU box, TMPDIR=/tmp):"]
    out += ["#   " + PROFILE_CMDS[k] for k in ("decode_trace", "decode_sq", "decode_fetch",
                                             "decode_write")]
    out += [f"# bytes: FETCH_SIZE x {fetch_per_kib:.1f} and WRITE_SIZE x {write_per_kib:.1f} per "
            "counted KiB (the copy calibration of the raster traffic summary); issue_busy = "
            "SQ_INSTS_VALU x 4 cycles / 1024 SIMDs / (GRBM_GUI_ACTIVE / 8); active_lanes = "
            "SQ_THREAD_CYCLES_VALU / (64 SQ_INSTS_VALU)",
            f"source_sha256(query.hip+raster_common.hpp) {h.hexdigest()[:16]}"]
    for r in rows:
        name = re.sub(r"\(.*", "", r["Name"].replace("void ", "").replace(
            "igs::(anonymous namespace)::", ""))
        out.append(f"kernel {name} calls {r['Calls']} avg_us {float(r['AverageNs']) / 1e3:.2f}")
    out.append(f"query_kernel valu_insts {sq['SQ_INSTS_VALU']:.4g} waves {sq['SQ_WAVES']:.0f} "
               f"valu_per_wave {sq['SQ_INSTS_VALU'] / sq['SQ_WAVES']:.0f} vmem_rd_per_wave "
               f"{sq['SQ_INSTS_VMEM_RD'] / sq['SQ_WAVES']:.0f} issue_busy "
               f"{sq['SQ_INSTS_VALU'] * 4 / 1024 / cyc:.3f} active_lanes "
               f"{sq['SQ_THREAD_CYCLES_VALU'] / (64 * sq['SQ_INSTS_VALU']):.3f}")
    out.append(f"query_kernel fetch_kib {fe['FETCH_SIZE']:.4g} write_kib {wr['WRITE_SIZE']:.4g} "
               f"read_bytes {fe['FETCH_SIZE'] * fetch_per_kib:.4g} write_bytes "
               f"{wr['WRITE_SIZE'] * write_per_kib:.4g}")
    open(os.path.join(PROFILES, "query_decode_texture-2048x2048-n9-N100000.txt"), "w").write(
        "\n".join(out) + "\n")
    print("\n".join(out))


def measured_valu(kernel, fused=True):
    """(issue_busy, active_lanes, executed lane slots) of the kernel from the committed counter
    summary, or None when that summary is missing or was taken from another source."""
    if not os.path.exists(VALU_FILE):
        return None
    want = {"raster_fwd": "raster_fwd_kernel<10,true,false>",
            "raster_bwd": "raster_bwd_kernel<9,10,true>",
            "raster_fit": "raster_fit_kernel<9,10,false>"}[kernel]
    for line in open(VALU_FILE):
        f = line.split()
        if len(f) > 2 and f[0] == "kernel" and f[1] == want:
            kv = dict(zip(f[2::2], f[3::2]))
            if kv.get("source_sha256") != kernel_source_hash(kernel):
                return None
            return {"issue_busy": float(kv["issue_busy"]),
                    "active_lanes": float(kv["active_lanes"]),
                    "executed_lane_slots": float(kv["executed_lane_slots"])}
    return None


def measured_traffic(kernel):
    """HBM bytes per launch from the committed counter summary, or None when the kernel's source
    has changed since the counters were taken."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    for line in open(TRAFFIC_FILE):
        f = line.split()
        if len(f) > 2 and f[0] == "kernel" and f[1] == kernel:
            kv = dict(zip(f[2::2], f[3::2]))
            if kv.get("source_sha256") != kernel_source_hash(kernel):
                return None
            return float(kv["traffic_bytes"])
    return None


def timed_fit(fitter, iters, torch):
    """Untimed dry run of the trajectory (sizes the pair buffer), then the same iterations replayed
    from the initial state as one captured graph each; returns seconds."""
    init = fitter.snapshot()
    fitter.advance_to(iters, use_graph=True)
    fitter.restore(init)
    if fitter.graph is None:
        fitter.capture()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(iters):
        fitter.step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    if fitter.steps_done() != iters:
        raise RuntimeError("an iteration overflowed the pair buffer during a timed fit")
    return dt


def single_pass_step(torch, nat, w, target, params, cap, steps, warmup, ref_fit, e_fwd, e_bwd,
                     fixed_config=None):
    """The same fit (same initial state, trajectory and pair capacity) with the single-pass L1
    kernel in place of the fused forward + adjoint pair, under launch settings tuned on this
    fitter (or the fixed ones given): graph-replayed iterations, then the kernels timed with HIP
    events on eager launches; the parameters after warmup + steps iterations must equal the
    two-pass fitter's."""
    from paper_2407_01866_amd.fit import PlainFitter
    from paper_2407_01866_amd.tune import autotune
    f = PlainFitter(target, params, w.K, pair_capacity=cap, single_pass=True)
    init = f.snapshot()
    total = warmup + steps
    if fixed_config is not None:
        f.launch_config, tune_times = fixed_config, {}
    else:
        _, tune_times = autotune(f, iters=10, warmup=3)
    log(f"[bench] single-pass launch config {f.launch_config}: " +
        ", ".join(f"{c}={t * 1e3:.3f} ms" for c, t in tune_times.items()))
    f.restore(init)
    f.capture()
    for _ in range(warmup):
        f.step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        f.step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    if f.steps_done() != total:
        raise RuntimeError("an iteration overflowed the pair buffer during the single-pass run")
    same = bool(torch.equal(f.fit, ref_fit))
    f.restore(init)
    for _ in range(warmup):
        f.step_async()
    torch.cuda.synchronize()
    nat.igs_timing_read(reset=True)
    nat.igs_timing_enable(True)
    torch.cuda._sleep(int(2.4e9 * 0.2))
    for _ in range(steps):
        f.step_async()
    torch.cuda.synchronize()
    ph = nat.igs_timing_read(reset=True)
    nat.igs_timing_enable(False)
    if f.steps_done() != total:
        raise RuntimeError("an iteration overflowed the pair buffer during the timed kernels")
    avg = {k: (v[0] / v[1] if v[1] else 0.0) for k, v in ph.items()}
    # the kernel does the forward's and the adjoint's work
    ops = fwd_valu_ops(e_fwd, w.H * w.W, w.n, True) + bwd_valu_ops(e_bwd, w.n)
    ach = ops / (avg["raster_fit"] * 1e-3)
    roofline = {"bound": "alu", "kernel": "raster_fit", "achieved": round(ach / 1e12, 3),
                "peak": round(PEAK_LANE_OPS / 1e12, 2), "unit": "Tlane-op/s",
                "frac": round(ach / PEAK_LANE_OPS, 4), "traffic": measured_traffic("raster_fit"),
                "valu_counters": measured_valu("raster_fit"), "avg_ms": round(avg["raster_fit"], 4),
                "work_per_launch": f"{ops:.4g} VALU lane-ops"}
    return dt / steps * 1e3, avg, roofline, same, f.launch_config, tune_times


def batched_vs_plain(torch, dev, iters, count=64, single_pass=True, wl=None):
    """Uneven batch (H, W in {256, 512, 1024, 2048}, 5k-80k Gaussians), or the workloads wl: one
    BatchFitter vs the same images fitted one after another by graph-captured PlainFitters, both
    with the same iteration (single-pass L1 kernel, or the two-pass fused pair)."""
    from paper_2407_01866_amd import synth
    from paper_2407_01866_amd.fit import BatchFitter, PlainFitter
    if wl is None:
        wl = synth.batch_workloads(count)
    count = len(wl)
    log(f"[bench] batch of {count} images: generating inputs")
    targets = [torch.from_numpy(w.target()).to(dev) for w in wl]
    params = [torch.from_numpy(w.gaussians()).to(dev) for w in wl]
    from paper_2407_01866_amd.tune import autotune, current_config, set_config
    plain_cfg = current_config()
    bf = BatchFitter(targets, params, 10, single_pass=single_pass)
    init = bf.snapshot()
    bf.advance_to(3, use_graph=False)          # sizes the pair buffer before tuning
    bf.restore(init)
    batch_cfg, _ = autotune(bf, iters=3, warmup=1)
    t_batch = timed_fit(bf, iters, torch)
    p_batch = bf.psnrs()
    del bf
    log(f"[bench] batched ({batch_cfg}): {t_batch:.3f} s for {iters} iterations; sequential "
        f"plain fits ({plain_cfg})")
    set_config(plain_cfg)
    t_plain, p_plain = 0.0, []
    for t, p in zip(targets, params):
        pf = PlainFitter(t, p, 10, single_pass=single_pass)
        t_plain += timed_fit(pf, iters, torch)
        p_plain.append(pf.psnr())
        del pf
    dps = [abs(a - b) for a, b in zip(p_batch, p_plain)]
    pixels = sum(w.H * w.W for w in wl)
    return {"images": count, "iterations": iters, "pixels": pixels,
            "iteration": "single-pass" if single_pass else "two-pass",
            "launch_config_batched": list(batch_cfg), "launch_config_plain": list(plain_cfg),
            "gaussians": sum(w.N for w in wl),
            "batched_s": round(t_batch, 4), "sequential_plain_s": round(t_plain, 4),
            "batched_images_per_s": count / t_batch, "plain_images_per_s": count / t_plain,
            "speedup": t_plain / t_batch,
            "mean_psnr_batched": sum(p_batch) / count, "mean_psnr_plain": sum(p_plain) / count,
            "max_abs_dpsnr": max(dps), "mean_abs_dpsnr": sum(dps) / count,
            "psnr_match": max(dps) <= 0.1 and sum(dps) / count <= 0.02}


def large_config(torch, dev, iters, batch_iters, single_pass=True):
    """The large configuration: fit iterations at 4096^2 with 500k Gaussians (sigma 0.5-8 px),
    timed as graph replays after a dry run of the same trajectory, with their Gaussian-pixel
    evaluation rate; and 16 images of 1024^2 with 30k Gaussians each fitted batched against one
    after another."""
    from paper_2407_01866_amd import _native as nat
    from paper_2407_01866_amd import synth
    from paper_2407_01866_amd.fit import PlainFitter
    w = synth.workload(4)
    log(f"[bench] {w.name}: generating inputs")
    f = PlainFitter(torch.from_numpy(w.target()).to(dev), torch.from_numpy(w.gaussians()).to(dev),
                    w.K, single_pass=single_pass)
    init = f.snapshot()
    e_fwd = []
    for it in range(1, iters + 1):                 # dry run: sizes the pair buffer, counts work
        f.advance_to(it, use_graph=False)
        e_fwd.append(int(f.status()[nat.STAT_EVALS_FWD]))
    f.restore(init)
    dt = timed_fit(f, iters, torch)
    ms = dt / iters * 1e3
    plain = {"workload": w.name, "iterations": iters, "ms_per_iter": round(ms, 4),
             "fit_iters_per_s": round(1e3 / ms, 2), "E_fwd": float(np.mean(e_fwd)),
             "evals_per_s": float(np.mean(e_fwd)) / (ms * 1e-3), "psnr": round(f.psnr(), 3)}
    log(f"[bench] {w.name}: {ms:.3f} ms per iteration")
    del f
    batch = batched_vs_plain(torch, dev, batch_iters, single_pass=single_pass,
                             wl=synth.small_batch_workloads())
    return {"plain_4096": plain, "batched_16x1024": batch}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-context", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--batch-iters", type=int, default=100,
                    help="iterations of the batched-vs-plain comparison (0 skips it)")
    ap.add_argument("--batch-count", type=int, default=64)
    ap.add_argument("--large-iters", type=int, default=20,
                    help="iterations of the large configuration's legs (0 skips them)")
    ap.add_argument("--no-ssim", action="store_true",
                    help="skip the L1 + SSIM loss measurement")
    ap.add_argument("--no-single-pass", action="store_true",
                    help="skip the single-pass L1 fitting kernel's run")
    ap.add_argument("--no-decode", action="store_true",
                    help="skip the random-access decoding measurement")
    ap.add_argument("--ssim-profile", action="store_true",
                    help="only run 20 L1 + SSIM loss calls at the workload (for kernel traces)")
    ap.add_argument("--decode-profile", action="store_true",
                    help="only run 5 random-access decoding calls (4M points) on the workload's "
                         "initial Gaussians (for kernel traces)")
    ap.add_argument("--launch-config", metavar="P,W,C[,B,K]",
                    help="fixed launch settings (persistent, wgs_per_cu, fwd_cull[, fwd_batch, "
                         "k_unroll]) instead of autotuning (profiling runs use the autotuner's "
                         "choice)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (for scaling HBM counters)")
    ap.add_argument("--summarize-profiles", metavar="DIR",
                    help="write profiles/ summaries from a rocprofv3 output directory and exit")
    args = ap.parse_args()
    if args.summarize_profiles:
        summarize_profiles(args.summarize_profiles)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the path runs "
              "on a single MI355X)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2407_01866_amd import _native as nat
    from paper_2407_01866_amd import synth
    from paper_2407_01866_amd.fit import PlainFitter

    dev = torch.device("cuda:0")
    if args.copy_calibration:
        a = torch.empty(1 << 28, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        log("copied 1 GiB x3")
        return

    w = synth.workload(2)
    log(f"[bench] workload {w.name}: generating inputs")
    target = torch.from_numpy(w.target()).to(dev)
    params = torch.from_numpy(w.gaussians()).to(dev)
    fitter = PlainFitter(target, params, w.K)
    if args.ssim_profile:
        fitter.step_async()                     # a rendered image of the workload
        _ssim_calls(torch, dev, w, fitter.image, target, 20)
        return
    if args.decode_profile:
        log(json.dumps(decode_step(torch, dev, w, params, calls=5)))
        return
    init = fitter.snapshot()
    # dry run of the same trajectory, one iteration at a time: sizes the pair buffer for every
    # iteration and records each iteration's work counts (the timed run repeats the trajectory)
    total = args.warmup + args.steps
    log(f"[bench] dry run of {total} iterations")
    evals = []
    for it in range(1, total + 1):
        fitter.advance_to(it, use_graph=False)
        st = fitter.status().clone()
        evals.append((int(st[nat.STAT_EVALS_FWD]), int(st[nat.STAT_EVALS_BWD]),
                      int(st[nat.STAT_PAIRS])))
    peak_pairs = max(e[2] for e in evals)
    fitter.r.set_capacity(int(peak_pairs * 1.25) + 1024)
    fitter.saved = fitter.r.new_saved()
    fitter.graph = None
    fitter.restore(init)
    # result-invariant launch settings, chosen by timing this fitter (state restored afterwards)
    from paper_2407_01866_amd.tune import autotune, set_config
    if args.launch_config:
        set_config(tuple(int(v) for v in args.launch_config.split(",")))
        tuned = nat.igs_get_launch_config().as_tuple()
        fitter.launch_config = tuned
        tune_times = {}
    else:
        tuned, tune_times = autotune(fitter, iters=10, warmup=3)
    log(f"[bench] autotuned launch config {tuned}: " +
        ", ".join(f"{c}={t * 1e3:.3f} ms" for c, t in tune_times.items()))
    fitter.restore(init)
    fitter.capture()
    log(f"[bench] pair capacity {fitter.r.cap} (peak need {peak_pairs}); warmup {args.warmup}")
    for _ in range(args.warmup):
        fitter.step()
    torch.cuda.synchronize()
    log(f"[bench] timing {args.steps} graph-replayed fit iterations")
    t0 = time.perf_counter()
    for _ in range(args.steps):
        fitter.step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    if fitter.steps_done() != total:
        raise RuntimeError("an iteration overflowed the pair buffer during the timed run")
    timed = evals[args.warmup:]
    e_fwd = float(np.mean([e[0] for e in timed]))
    e_bwd = float(np.mean([e[1] for e in timed]))
    pairs = float(np.mean([e[2] for e in timed]))
    ms_per_step = dt / args.steps * 1e3
    value = e_fwd / (ms_per_step * 1e-3)

    # live per-phase timing with HIP events on the launch stream (eager launches: events cannot
    # be recorded inside the captured graph).  A spin kernel holds the stream while the timed
    # iterations are enqueued, so that the kernels then run back to back and the events time the
    # kernels rather than the host's launch rate.
    log("[bench] per-kernel HIP-event timing (same trajectory, eager launches)")
    fitter.restore(init)
    for _ in range(args.warmup):
        fitter.step_async()
    torch.cuda.synchronize()
    nat.igs_timing_read(reset=True)
    nat.igs_timing_enable(True)
    torch.cuda._sleep(int(2.4e9 * 0.2))      # ~0.2 s of device time at 2.4 GHz
    for _ in range(args.steps):
        fitter.step_async()
    torch.cuda.synchronize()
    ph = nat.igs_timing_read(reset=True)
    nat.igs_timing_enable(False)
    if fitter.steps_done() != total:
        raise RuntimeError("an iteration overflowed the pair buffer during the timed kernels")
    avg = {k: (v[0] / v[1] if v[1] else 0.0) for k, v in ph.items()}
    hw = w.H * w.W
    ops = {"raster_fwd": fwd_valu_ops(e_fwd, hw, w.n, fitter.fused),
           "raster_bwd": bwd_valu_ops(e_bwd, w.n)}
    dom = max(ops, key=lambda k: avg[k])
    achieved = ops[dom] / (avg[dom] * 1e-3)
    fwdbwd_ms = (avg["binning"] + avg["raster_fwd"] + avg["loss"] + avg["raster_bwd"] +
                 avg["grad_reduce"])
    roofline = {"bound": "alu", "kernel": dom, "achieved": round(achieved / 1e12, 3),
                "peak": round(PEAK_LANE_OPS / 1e12, 2), "unit": "Tlane-op/s",
                "frac": round(achieved / PEAK_LANE_OPS, 4), "traffic": measured_traffic(dom),
                "valu_counters": measured_valu(dom),
                "avg_ms": round(avg[dom], 4),
                "work_per_launch": f"{ops[dom]:.4g} VALU lane-ops"}

    other = "raster_bwd" if dom == "raster_fwd" else "raster_fwd"
    roofline_bwd = {"kernel": other, "achieved": round(ops[other] / (avg[other] * 1e-3) / 1e12, 3),
                    "peak": round(PEAK_LANE_OPS / 1e12, 2), "unit": "Tlane-op/s",
                    "frac": round(ops[other] / (avg[other] * 1e-3) / PEAK_LANE_OPS, 4),
                    "traffic": measured_traffic(other), "valu_counters": measured_valu(other),
                    "avg_ms": round(avg[other], 4),
                    "work_per_launch": f"{ops[other]:.4g} VALU lane-ops"}
    single = None
    if not args.no_single_pass:
        log("[bench] single-pass L1 fitting kernel (same trajectory)")
        single = single_pass_step(torch, nat, w, target, params, fitter.r.cap, args.steps,
                                  args.warmup, fitter.fit, e_fwd, e_bwd,
                                  tuned if args.launch_config else None)
    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] CPU oracle baseline")
        g = synth.gen_grad_image(1, w.n, w.H, w.W).astype(np.float64) / (w.n * w.H * w.W)
        cpu = cpu_baseline(w.gaussians(), w.H, w.W, w.K, g, args.cpu_budget)
    decode = None
    if not args.no_decode:
        log("[bench] random-access decoding")
        decode = decode_step(torch, dev, w, fitter.rend)
    ssim = None
    if not args.no_ssim:
        log("[bench] L1 + SSIM loss")
        ssim = ssim_step(torch, dev, w, fitter.image, fitter.target)
    ctx = None if args.no_context else paper_context(torch, dev)
    batch = None
    if args.batch_iters > 0:
        batch = batched_vs_plain(torch, dev, args.batch_iters, args.batch_count,
                                 single_pass=not args.no_single_pass)
    large = None
    if args.large_iters > 0:
        large = large_config(torch, dev, args.large_iters, 2 * args.large_iters,
                             single_pass=not args.no_single_pass)

    two_pass_step = ("binning + render fused with the L1 loss + adjoint + gradient reduction + "
                     "Adam (HIP graph)" if fitter.fused else
                     "binning + render + L1 gradient + adjoint + gradient reduction + Adam "
                     "(HIP graph)")
    def config_record(cfg, times):
        return {"persistent": cfg[0], "wgs_per_cu": cfg[1], "fwd_cull": cfg[2],
                "fwd_batch": cfg[3] or 192, "k_unroll": cfg[4],
                "autotune_ms": {str(c): round(t * 1e3, 4) for c, t in times.items()}}

    two_pass = {"step": two_pass_step, "ms_per_step": ms_per_step,
                "launch_config": config_record(tuned, tune_times),
                "fit_iters_per_s": 1e3 / ms_per_step,
                "fwd_bwd_evals_per_s": e_fwd / (fwdbwd_ms * 1e-3),
                "phase_ms": {k: round(v, 4) for k, v in avg.items() if v > 0},
                "roofline": roofline, "roofline_adjoint": roofline_bwd}
    if single is not None:
        # the headline step: the single-pass kernel (same loss, gradient and trajectory)
        sp_ms, sp_avg, sp_roof, same, sp_cfg, sp_times = single
        if not same:
            raise RuntimeError("the single-pass fit diverged from the two-pass fit")
        head = {"step": "binning + single-pass render, L1 loss and adjoint + gradient reduction "
                        "+ Adam (HIP graph)", "ms_per_step": sp_ms, "fit_iters_per_s": 1e3 / sp_ms,
                "fwd_bwd_evals_per_s": e_fwd / ((sp_avg["binning"] + sp_avg["raster_fit"] +
                                                 sp_avg["loss"] + sp_avg["grad_reduce"]) * 1e-3),
                "phase_ms": {k: round(v, 4) for k, v in sp_avg.items() if v > 0},
                "launch_config": config_record(sp_cfg, sp_times), "roofline": sp_roof}
    else:
        head, two_pass = two_pass, None
    ms_per_step = head["ms_per_step"]
    value = e_fwd / (ms_per_step * 1e-3)
    out = {
        "metric": METRIC, "value": value, "unit": "Gaussian-pixel evals/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "H": w.H, "W": w.W, "n": w.n, "N": w.N, "K": w.K,
                   "tile": 16, "step": head["step"]},
        "fit_iters_per_s": head["fit_iters_per_s"],
        "fwd_bwd_evals_per_s": head["fwd_bwd_evals_per_s"],
        "phase_ms": head["phase_ms"],
        "E_fwd": e_fwd, "E_bwd": e_bwd, "pairs": pairs,
        "E_fwd_first_last": [evals[args.warmup][0], evals[-1][0]],
        "launch_config": head["launch_config"],
        "roofline": head["roofline"],
        "two_pass": two_pass, "cpu_baseline": cpu, "ssim_step": ssim, "decode": decode,
        "paper_context": ctx, "batched_vs_plain": batch, "large_config": large,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
