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


ROOT = os.path.dirname(os.path.abspath(__file__))
TRAFFIC_FILES = {"ball_and_stick_1000k_1920x1080": "hbm_traffic_ball_and_stick_1M_1080p.txt",
                 "whole_cell_100M_3840x2160": "hbm_traffic_whole_cell_100M_4k.txt"}
KERNEL_SOURCES = {"k_resolve": "resolve.hip", "k_count": "bin.hip", "k_scatter": "bin.hip",
                  "k_shade": "shade.hip", "k_cluster_cull": "scene.hip"}


def sources_sha(kernel):
    """sha256[:16] of a kernel's source file followed by the shared internal header."""
    import hashlib
    f = KERNEL_SOURCES.get(kernel.split("<")[0])
    if f is None:
        return None
    h = hashlib.sha256()
    for name in (f, "vtx_internal.h"):
        with open(os.path.join(ROOT, "paper_2501_12750_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload_name, kernels):
    """HBM bytes per launch of the named kernels, summed, from the committed
    rocprofv3 FETCH_SIZE/WRITE_SIZE summary of this workload; None when there
    is none or when any of the kernels' sources changed since it was taken."""
    fname = TRAFFIC_FILES.get(workload_name)
    if fname is None:
        return None
    path = os.path.join(ROOT, "profiles", fname)
    if not os.path.exists(path):
        return None
    rows = {}
    with open(path) as fh:
        for line in fh:
            parts = line.split()
            if len(parts) == 6 and parts[0].startswith("k_"):
                rows[parts[0]] = (float(parts[4]), parts[5])
    total = 0.0
    for k in kernels:
        if k not in rows or rows[k][1] != sources_sha(k):
            return None
        total += rows[k][0]
    return total


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


def frame_tile(tile, W, H):
    """The tile edge the library uses: the requested one (16 by default),
    doubled while the frame would have more tiles than its binner holds."""
    t = tile or 16
    while ((W + t - 1) // t) * ((H + t - 1) // t) > 15360 and t < 64:
        t *= 2
    return t


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="ball_and_stick", choices=["ball_and_stick", "whole_cell", "plain_small"])
    ap.add_argument("--tile", type=int, default=0, help="tile size (0 = library default)")
    ap.add_argument("--path", choices=["scene", "plain"], default="scene",
                    help="scene: the molecule is a resident scene (vtx_scene_create before timing, "
                         "vtx_render_scene per frame); plain: vtx_render on the caller's arrays each frame")
    ap.add_argument("--compare-plain", type=int, default=1,
                    help="with --path scene, also time the plain vtx_render path (reported beside)")
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
    ctx = rs = None
    if args.path == "scene":
        ctx = vtx.vtx_context_create(0, 0)
        t1 = time.perf_counter()
        rs = vtx.ResidentScene(ctx, ds)
        log(f"resident scene built in {time.perf_counter() - t1:.2f} s")

    def render(opts):
        if rs is not None:
            vtx.vtx_render_scene(rs.handle, wl.camera, opts, W, H, frame.rgba, frame.depth, frame.id, stream)
        else:
            vtx.vtx_render(*ds.args(), wl.camera, opts, W, H, frame.rgba, frame.depth, frame.id, stream)

    # exact fragment counts of this scene and camera (early-outs off), untimed
    import dataclasses
    opts_stats = dataclasses.replace(wl.options, flags=vtx.VTX_FLAG_STATS)
    render(opts_stats)
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
        render(wl.options)
    torch.cuda.synchronize()
    vtx.vtx_reset_timings(stream)
    log(f"warmup {args.warmup} done; timing {args.steps} steps")

    opts_main = opts_t if args.kernel_events == "timed" else wl.options
    torch.cuda.synchronize()
    ts = time.perf_counter()
    for _ in range(args.steps):
        render(opts_main)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - ts
    if args.kernel_events == "separate":
        for _ in range(args.steps):
            render(opts_t)
    timings = vtx.vtx_read_timings(stream)
    st_after = vtx.vtx_read_stats(stream)
    ms_per_step = elapsed / args.steps * 1e3
    fps = args.steps / elapsed
    log(f"timed: {ms_per_step:.3f} ms/frame, {fps:.1f} frames/s; kernels {timings}")

    # latency of single frames submitted and awaited one at a time
    lat = []
    for _ in range(args.latency_frames):
        a = time.perf_counter()
        render(wl.options)
        stream.synchronize()
        lat.append((time.perf_counter() - a) * 1e3)
    lat = np.array(lat)

    plain = None
    if rs is not None and args.compare_plain:
        for _ in range(args.warmup):
            vtx.vtx_render(*ds.args(), wl.camera, wl.options, W, H, frame.rgba, frame.depth, frame.id, stream)
        torch.cuda.synchronize()
        a = time.perf_counter()
        for _ in range(args.steps):
            vtx.vtx_render(*ds.args(), wl.camera, wl.options, W, H, frame.rgba, frame.depth, frame.id, stream)
        torch.cuda.synchronize()
        pe = time.perf_counter() - a
        plain = {"frames_per_s": round(args.steps / pe, 3), "ms_per_frame": round(pe / args.steps * 1e3, 4)}
        log(f"plain vtx_render: {plain}")

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
        "scan": ("hbm", 12.0 * ((W + frame_tile(wl.options.tile_size, W, H) - 1) // frame_tile(wl.options.tile_size, W, H))
                 * ((H + frame_tile(wl.options.tile_size, W, H) - 1) // frame_tile(wl.options.tile_size, W, H)), timings["ms_scan"]),
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
    tile = frame_tile(wl.options.tile_size, W, H)
    launched = {"project": (["k_cluster_cull", "k_count<SceneSource>"] if rs is not None else ["k_count<PlainSource>"]),
                "scatter": ["k_scatter"], "resolve": [f"k_resolve<{tile}>"], "shade": ["k_shade"], "scan": []}
    traffic = measured_traffic(wl.name, launched[dom]) if launched[dom] else None
    roof = {"kernel": dom, "launches": launched[dom], **roof,
            "traffic": None if traffic is None else round(traffic)}

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
                   "ssao_samples": K, "tile_size": frame_tile(wl.options.tile_size, W, H),
                   "path": "resident scene (vtx_render_scene)" if rs is not None else "vtx_render"},
        "plain_vtx_render": plain,
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
    if rs is not None:
        rs.close()
        vtx.vtx_context_destroy(ctx)


if __name__ == "__main__":
    main()
