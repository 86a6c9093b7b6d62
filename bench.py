#!/usr/bin/env python3
"""Frames/s of the full per-frame hot path on one MI355X.

One step = one frame of the whole path over a resident synthetic scene:
project/cull/count -> prefix sum -> scatter into tile lists -> per-tile ray
cast into the (depth, id) G-buffer -> SSAO + shading into RGBA8, i.e. one
vtx_render call through the C ABI.  Inputs are resident in device memory
before the timed region starts.

Prints ONE JSON line.  Besides frames/s it reports atom-fragments/s, the
p50/p99 latency of single synchronous frames, per-kernel device times from
HIP events recorded on the render stream inside the timed region, the
roofline of the dominant kernel, and the CPU oracle timed on the host.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
# 256 CUs x 64 lanes x 2.4 GHz: one non-packed VALU op per lane per clock
ALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
# algorithmic per-unit work (lane-ops): per shaded pixel, per SSAO sample,
# per sphere / cylinder fragment, per primitive projected
OPS_PIXEL, OPS_SAMPLE, OPS_SPHERE_FRAG, OPS_CYL_FRAG, OPS_PRIM = 40, 25, 20, 50, 60


def workload(name):
    from paper_2501_12750_amd import scenes
    if name == "ball_and_stick":
        return scenes.ball_and_stick()
    if name == "whole_cell":
        return scenes.whole_cell()
    if name == "plain_small":
        return scenes.plain_small()
    raise SystemExit(f"unknown workload {name}")


def cpu_baseline(wl, budget_s=12.0):
    """The oracle (FP64 C splatter + SSAO + shading) on the host cores, end to
    end, for as many whole frames as fit the budget (at least one)."""
    from oracle import osplat
    osplat.build(force=False)
    threads = osplat.default_threads()
    n = 0
    t0 = time.perf_counter()
    while True:
        osplat.render(wl.scene, wl.camera, wl.options, wl.width, wl.height, nthreads=threads)
        n += 1
        el = time.perf_counter() - t0
        if el >= budget_s or el / n * (n + 1) > 3 * budget_s:
            break
    return {"value": n / el, "unit": "frames/s", "cores": threads, "kind": "oracle",
            "sample": f"{n} full {wl.width}x{wl.height} frame(s) of the same scene and camera, "
                      f"FP64 footprint splatter with accept sets + SSAO + shading, {el:.1f} s"}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="ball_and_stick", choices=["ball_and_stick", "whole_cell", "plain_small"])
    ap.add_argument("--tile", type=int, default=0, help="tile size (0 = library default)")
    ap.add_argument("--latency-frames", type=int, default=50)
    ap.add_argument("--kernel-events", choices=["timed", "separate"], default="separate",
                    help="record the per-kernel HIP events inside the timed region, or in a separate "
                         "pass of the same length after it")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy-mb", type=int, default=0,
                    help="before timing, run one device copy of this many MiB (reference for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the renderer has no multi-GPU path "
              "(--gpus must be 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2501_12750_amd import vtx

    def log(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    t0 = time.perf_counter()
    wl = workload(args.workload)
    if args.tile:
        wl.options.tile_size = args.tile
    W, H = wl.width, wl.height
    log(f"workload {wl.name}: {wl.scene.n_atoms} atoms, {wl.scene.n_bonds} bonds, {W}x{H}, "
        f"generated in {time.perf_counter() - t0:.1f} s")
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    ds = vtx.DeviceScene(wl.scene)
    frame = vtx.Frame(W, H)
    stream = torch.cuda.current_stream()

    # exact fragment counts of this scene and camera (early-outs off), untimed
    import dataclasses
    opts_stats = dataclasses.replace(wl.options, flags=vtx.VTX_FLAG_STATS)
    vtx.vtx_render(*ds.args(), wl.camera, opts_stats, W, H, frame.rgba, frame.depth, frame.id, stream)
    st = vtx.vtx_read_stats(stream)
    ids = frame.id.cpu().numpy().view(np.uint32)
    hit_px = int(np.count_nonzero(ids != 0xFFFFFFFF))
    log(f"stats {st}, hit pixels {hit_px}")

    if args.calibrate_copy_mb:
        src = torch.empty(args.calibrate_copy_mb << 18, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"calibration copy of {args.calibrate_copy_mb} MiB done")
        del src, dst

    opts_t = dataclasses.replace(wl.options, flags=vtx.VTX_FLAG_TIMING)
    for _ in range(args.warmup):
        vtx.vtx_render(*ds.args(), wl.camera, wl.options, W, H, frame.rgba, frame.depth, frame.id, stream)
    torch.cuda.synchronize()
    vtx.vtx_reset_timings(stream)
    log(f"warmup {args.warmup} done; timing {args.steps} steps")

    opts_main = opts_t if args.kernel_events == "timed" else wl.options
    torch.cuda.synchronize()
    ts = time.perf_counter()
    for _ in range(args.steps):
        vtx.vtx_render(*ds.args(), wl.camera, opts_main, W, H, frame.rgba, frame.depth, frame.id, stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - ts
    if args.kernel_events == "separate":
        for _ in range(args.steps):
            vtx.vtx_render(*ds.args(), wl.camera, opts_t, W, H, frame.rgba, frame.depth, frame.id, stream)
    timings = vtx.vtx_read_timings(stream)
    st_after = vtx.vtx_read_stats(stream)
    ms_per_step = elapsed / args.steps * 1e3
    fps = args.steps / elapsed
    log(f"timed: {ms_per_step:.3f} ms/frame, {fps:.1f} frames/s; kernels {timings}")

    # latency of single frames submitted and awaited one at a time
    lat = []
    for _ in range(args.latency_frames):
        a = time.perf_counter()
        vtx.vtx_render(*ds.args(), wl.camera, wl.options, W, H, frame.rgba, frame.depth, frame.id, stream)
        stream.synchronize()
        lat.append((time.perf_counter() - a) * 1e3)
    lat = np.array(lat)

    # roofline of each kernel; the dominant one goes in the JSON's roofline
    N, M = wl.scene.n_atoms, wl.scene.n_bonds
    K = int(wl.options.ssao_samples)
    f_total = st["fragments_hit"]
    f_cyl = st.get("fragments_hit_bond", 0)
    f_sph = f_total - f_cyl
    per_kernel = {
        "project": ("hbm", 16.0 * N + 8.0 * M, timings["ms_project"]),
        "resolve": ("alu", float(OPS_SPHERE_FRAG * f_sph + OPS_CYL_FRAG * f_cyl), timings["ms_resolve"]),
        "shade": ("alu", float((OPS_PIXEL + OPS_SAMPLE * K) * hit_px), timings["ms_shade"]),
        "scatter": ("hbm", 12.0 * st["visible"] + 4.0 * st["pairs"], timings["ms_scatter"]),
        "scan": ("hbm", 4.0 * (W // max(1, wl.options.tile_size or 16) + 1) * (H // max(1, wl.options.tile_size or 16) + 1) * 3, timings["ms_scan"]),
    }
    kern = {}
    for k, (bound, work, ms) in per_kernel.items():
        if ms <= 0:
            continue
        if bound == "hbm":
            ach, peak, unit = work / (ms * 1e-3) / 1e9, HBM_PEAK_GBS, "GB/s"
        else:
            ach, peak, unit = work / (ms * 1e-3) / 1e12, ALU_PEAK_TOPS, "Tops/s"
        kern[k] = {"bound": bound, "ms": round(ms, 5), "achieved": round(ach, 3), "peak": round(peak, 2),
                   "unit": unit, "frac": round(ach / peak, 4)}
    dom = max(kern, key=lambda k: kern[k]["ms"])
    roof = dict(kern[dom])
    roof.pop("ms")
    roof = {"kernel": dom, **roof, "traffic": None}

    out = {
        "metric": "frames/s",
        "value": round(fps, 3),
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wl.name, "atoms": N, "bonds": M, "width": W, "height": H,
                   "ssao_samples": K, "tile_size": wl.options.tile_size or 16},
        "atom_fragments_per_s": round(f_total * fps, 1),
        "atom_fragments": f_total,
        "latency_ms": ({"p50": round(float(np.percentile(lat, 50)), 4),
                        "p99": round(float(np.percentile(lat, 99)), 4), "frames": int(lat.size)}
                       if lat.size else None),
        "kernels": kern,
        "roofline": roof,
        "bins": {"visible": st["visible"], "pairs": st["pairs"], "overflow_tiles": st_after["overflow_tiles"]},
    }
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(wl)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
