#!/usr/bin/env python3
"""Frames/s of the full per-frame hot path on one MI355X.

One step is one pass of the whole path over synthetic inputs already resident
in device memory: cluster test and project/cull/count -> prefix sum ->
scatter into tile lists -> per-tile ray cast into the (depth, id) G-buffer ->
SSAO + shading into RGBA8.

Workloads:
  whole_cell (default)      100M atoms, 3840x2160, SSAO 16; one step = one frame
                            (vtx_render_scene, or vtx_render with --path plain);
                            the ball-and-stick frame is timed after it and
                            reported under its own key (--also)
  ball_and_stick            1M atoms + 1.04M bonds, 1920x1080, SSAO 16; one
                            step = one frame
  trajectory                50k atoms x 64 trajectory frames x 4 orbit
                            viewports (720p..1440p) = 256 renders; one step =
                            one vtx_render_batch call of all 256
  served                    Poisson arrivals (200/s, 60 s) of session frames on
                            24 resident scenes of 1e4..1e7 atoms at 720p/1080p/4K,
                            rendered by vtx_server (continuous batching);
                            frames/s and arrival-to-completion p50/p99
  plain_small               4096 atoms, 256x256 (the small parity case)

Prints ONE JSON line: frames/s (renders/s for the batch) with the contract
fields, atom-fragments/s, p50/p99 latency, per-kernel device times (each
kernel dispatched with its own start and stop events on the render stream),
the roofline of the dominant kernel and of the whole frame, the step's
share of the VALU issue slots (its counted instructions from the committed
rocprofv3 summary over the measured step time), the resolve's
skip rate (ray tests the early-outs leave, from a counting frame), the other
launch form of the same renders side by side, and the CPU oracle timed on
the host.
"""
from __future__ import annotations

import argparse
import dataclasses
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
                 "whole_cell_100M_3840x2160": "hbm_traffic_whole_cell_100M_4k.txt",
                 "trajectory_50k_64x4": "hbm_traffic_trajectory_50k_64x4.txt",
                 "ses_globule_50k_h0.5": "hbm_traffic_ses_globule_50k_h0.5.txt"}
KERNEL_SOURCES = {"k_resolve": "resolve.hip", "k_resolve_tail": "resolve.hip", "k_refine": "resolve.hip",
                  "k_count": "bin.hip", "k_layers": "bin.hip", "k_tile_offsets": "bin.hip",
                  "k_scatter": "bin.hip", "k_shade": "shade.hip", "k_cluster_cull": "scene.hip",
                  "k_ses_mark": "ses.hip", "k_ses_edt_x_lds": "ses.hip", "k_ses_edt_yz_lds": "ses.hip",
                  "k_ses_count": "ses.hip", "k_ses_emit": "ses.hip", "k_scan_sums": "scan.hip",
                  "k_scan_top": "scan.hip", "k_scan_apply": "scan.hip"}
# the launches of one vtx_ses call on the benchmark's grid (windows of at
# most 32 steps: the distance passes staged through LDS)
SES_KERNELS = ["k_ses_mark", "k_ses_edt_x_lds<32>", "k_ses_edt_yz_lds<false>", "k_ses_edt_yz_lds<true>",
               "k_ses_count", "k_scan_sums", "k_scan_top", "k_scan_apply", "k_ses_emit"]


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def sources_sha(kernel):
    """sha256[:16] of a kernel's source file followed by the shared headers."""
    import hashlib
    f = KERNEL_SOURCES.get(kernel.split("<")[0])
    if f is None:
        return None
    h = hashlib.sha256()
    for name in (f, "prims.h", "vtx_internal.h"):
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


VALU_FILES = {"ball_and_stick_1000k_1920x1080": "valu_ball_and_stick_1M_1080p.txt",
              "whole_cell_100M_3840x2160": "valu_whole_cell_100M_4k.txt",
              "trajectory_50k_64x4": "valu_trajectory_50k_64x4.txt"}


def measured_valu(workload_name, kernels):
    """VALU wave instructions per launch of the named kernels (SQ_INSTS_VALU),
    summed, from the committed rocprofv3 counter summary of this workload;
    None when there is none or when any of the kernels' sources changed since
    it was taken."""
    fname = VALU_FILES.get(workload_name)
    if fname is None:
        return None
    path = os.path.join(ROOT, "profiles", fname)
    if not os.path.exists(path):
        return None
    rows = {}
    with open(path) as fh:
        for line in fh:
            if line.startswith("k_"):
                rest = line[44:].split()
                if len(rest) == 9:
                    rows[line[:44].replace(" ", "")] = (float(rest[7]), rest[8])
    total = 0.0
    for k in kernels:
        if k not in rows or rows[k][1] != sources_sha(k):
            return None
        total += rows[k][0]
    return total


def frame_tile(tile, W, H):
    """The tile edge the library uses: the requested one (16 by default),
    doubled while the frame would have more tiles than its binner holds."""
    t = tile or 16
    while ((W + t - 1) // t) * ((H + t - 1) // t) > 15360 and t < 64:
        t *= 2
    return t


def n_tiles(tile, W, H):
    t = frame_tile(tile, W, H)
    return ((W + t - 1) // t) * ((H + t - 1) // t)


# ---------------------------------------------------------------------------
# runners: one step of each workload, in each launch form
# ---------------------------------------------------------------------------
class Render:
    """One camera view of a scene frame into its own device images."""

    def __init__(self, vtx, frame_index, camera, options, W, H):
        self.frame_index, self.camera, self.options = frame_index, camera, options
        self.W, self.H = W, H
        self.out = vtx.Frame(W, H)


class SingleRunner:
    """One frame per step: vtx_render_scene on a resident scene, or vtx_render."""

    def __init__(self, vtx, wl, path, stream):
        self.vtx, self.wl, self.stream, self.path = vtx, wl, stream, path
        self.ds = vtx.DeviceScene(wl.scene)
        self.renders = [Render(vtx, 0, wl.camera, wl.options, wl.width, wl.height)]
        self.ctx = self.rs = None
        if path == "scene":
            self.ctx = vtx.vtx_context_create(0, 0)
            t1 = time.perf_counter()
            self.rs = vtx.ResidentScene(self.ctx, self.ds)
            log(f"resident scene built in {time.perf_counter() - t1:.2f} s")
        self.launch_form = "resident scene, vtx_render_scene per frame" if path == "scene" else "vtx_render per frame"
        self.other_forms = [("vtx_render per frame (caller's arrays)", self.other_step)] if path == "scene" else []

    def step(self, flags=0):
        r = self.renders[0]
        o = dataclasses.replace(r.options, flags=flags) if flags else r.options
        if self.rs is not None:
            self.vtx.vtx_render_scene(self.rs.handle, r.camera, o, r.W, r.H, r.out.rgba, r.out.depth, r.out.id,
                                      self.stream)
        else:
            self.vtx.vtx_render(*self.ds.args(), r.camera, o, r.W, r.H, r.out.rgba, r.out.depth, r.out.id,
                                self.stream)

    def other_step(self):
        r = self.renders[0]
        self.vtx.vtx_render(*self.ds.args(), r.camera, r.options, r.W, r.H, r.out.rgba, r.out.depth, r.out.id,
                            self.stream)

    def autotune(self, cache):
        if self.rs is None:
            raise SystemExit("--autotune needs the resident-scene path")
        r = self.renders[0]
        job = self.vtx.make_job(self.rs.handle, 0, r.camera, r.options, r.W, r.H, r.out.rgba, r.out.depth, r.out.id)
        return self.vtx.vtx_autotune(self.ctx, [job], cache, self.stream)

    def close(self):
        if self.rs is not None:
            self.rs.close()
            self.vtx.vtx_context_destroy(self.ctx)


class BatchRunner:
    """All renders of a trajectory workload per step: one vtx_render_batch call
    (the other form: one call per render)."""

    def __init__(self, vtx, scene0, frames, cams, opts, viewports, stream):
        import torch
        self.vtx, self.stream = vtx, stream
        self.ctx = vtx.vtx_context_create(0, 0)
        self.rs = vtx.ResidentScene(self.ctx, vtx.DeviceScene(scene0))
        if len(frames) > 1:
            self.rs.add_frames(torch.from_numpy(np.ascontiguousarray(frames[1:])).to("cuda"), len(frames) - 1)
        self.renders = []
        for f in range(len(frames)):
            for k in range(len(cams)):
                W, H = viewports[k]
                self.renders.append(Render(vtx, f, cams[k], opts, W, H))
        self.arrays = {}
        self.graph = None   # captured at the first step (after any tuning)
        self.launch_form = (f"hipGraph of the {len(self.renders)}-render batch (vtx_batch_graph_launch: one graph "
                            f"launch per step)")
        self.other_forms = [("vtx_render_batch of the same renders, launched eagerly", self.eager_step),
                            ("one vtx_render_batch call per render (single-render launches)", self.per_render_step)]

    def jobs(self, flags):
        if flags not in self.arrays:
            v = self.vtx
            js = [v.make_job(self.rs.handle, r.frame_index, r.camera,
                             dataclasses.replace(r.options, flags=flags), r.W, r.H, r.out.rgba, r.out.depth, r.out.id)
                  for r in self.renders]
            self.arrays[flags] = ((v.vtx_job * len(js))(*js), [(v.vtx_job * 1)(j) for j in js])
        return self.arrays[flags]

    def step(self, flags=0):
        if flags == 0:
            if self.graph is None:
                self.graph = self.vtx.vtx_batch_graph_create(self.ctx, self.jobs(0)[0])
            self.vtx.vtx_batch_graph_launch(self.graph, self.stream)
        else:   # statistics and per-kernel events run the same kernels eagerly
            self.vtx.vtx_render_batch(self.ctx, self.jobs(flags)[0], self.stream)

    def eager_step(self):
        self.vtx.vtx_render_batch(self.ctx, self.jobs(0)[0], self.stream)

    def per_render_step(self):
        for one in self.jobs(0)[1]:
            self.vtx.vtx_render_batch(self.ctx, one, self.stream)

    def autotune(self, cache):
        return self.vtx.vtx_autotune(self.ctx, self.jobs(0)[0], cache, self.stream)

    def close(self):
        if self.graph is not None:
            self.vtx.vtx_batch_graph_destroy(self.graph)
        self.rs.close()
        self.vtx.vtx_context_destroy(self.ctx)


def _build_served_scene(spec):
    scene, centre, radius = spec.build()
    return scene, centre, radius


def build_served(args, scenes):
    """Generates the served mix's scene pool on the host cores (before the
    process touches the GPU)."""
    import concurrent.futures as cf
    import multiprocessing as mp
    pool, reqs = scenes.served_mix(duration_s=args.serve_seconds, rate_hz=args.serve_rate)
    t0 = time.perf_counter()
    used = sorted({r.scene for r in reqs})
    with cf.ProcessPoolExecutor(max_workers=min(8, len(used)), mp_context=mp.get_context("spawn")) as ex:
        built = dict(zip(used, ex.map(_build_served_scene, [pool[k] for k in used])))
    log(f"served pool: {len(used)} scenes, {sum(built[k][0].n_atoms for k in used) / 1e6:.1f}M atoms, "
        f"generated in {time.perf_counter() - t0:.1f} s; {len(reqs)} requests over {args.serve_seconds:.0f} s")
    return pool, reqs, used, built


def run_served(args, vtx, scenes, torch, stream):
    """The served mix: Poisson arrivals of session frames on a pool of 24
    resident scenes; latency is arrival -> device completion.  --serve-mode
    server renders them through the library's server (continuous batching);
    plain replays the same arrival trace with one vtx_render_scene per
    request on one stream, completion taken from an event after each render
    (device time, referred to the host clock through an event recorded at
    the start)."""
    pool, reqs, used, built = args.served_inputs
    plain = args.serve_mode == "plain"
    dev_scenes = {k: vtx.DeviceScene(built[k][0]) for k in used}
    budget = int(args.serve_budget_gb * (1 << 30)) if args.serve_budget_gb > 0 else 0
    ctx = vtx.vtx_context_create(0, budget)
    upload = torch.cuda.Stream()
    server = None if plain else vtx.vtx_server_create(ctx, args.serve_max_batch, 2, stream)
    opts = scenes.Options(ssao_samples=16, ssao_radius=2.0)
    pending = []                        # plain: (event, ticket) in submission order
    ref_ev = torch.cuda.Event(enable_timing=True)
    ref_ev.record(stream)
    stream.synchronize()
    t_ref = vtx.vtx_clock_s()
    hbm_peak = 0
    outs = {res: [vtx.Frame(*res) for _ in range(48)] for res in scenes.SERVE_RESOLUTIONS}
    slot_next = {res: 0 for res in outs}
    slot_busy = {}                      # (res, slot) -> ticket
    resident = {}                       # pool index -> ResidentScene
    last_use = {}
    outstanding = {}                    # pool index -> in-flight requests
    ticket_info = {}
    done = []
    created = evicted = 0

    def finish(c):
        info = ticket_info.pop(c["ticket"])
        outstanding[info["scene"]] -= 1
        slot_busy.pop(info["slot"], None)
        c.update(info)
        done.append(c)

    def collect(wait_ms=0):
        if not plain:
            for c in vtx.vtx_server_poll(server, 512, wait_ms):
                finish(c)
            return
        if wait_ms and pending:
            pending[0][0].synchronize()
        while pending and pending[0][0].query():
            ev, tk = pending.pop(0)
            t = t_ref + ref_ev.elapsed_time(ev) / 1e3
            finish({"ticket": tk, "status": 0, "done_s": t, "launch_s": ticket_info[tk]["submit"]})

    def ensure_resident(k):
        nonlocal created, evicted
        if k in resident:
            return resident[k]
        while True:
            try:
                rs = vtx.ResidentScene(ctx, dev_scenes[k], stream=upload)
                created += 1
                resident[k] = rs
                nonlocal hbm_peak
                hbm_peak = max(hbm_peak, vtx.vtx_context_bytes_in_use(ctx))
                return rs
            except vtx.VtxError as e:
                if e.code != vtx.VTX_EBUSY:
                    raise
                idle = [j for j in resident if outstanding.get(j, 0) == 0]
                if not idle:
                    collect(5)
                    continue
                j = min(idle, key=lambda j: last_use.get(j, 0.0))
                resident.pop(j).close()
                evicted += 1

    start = vtx.vtx_clock_s() + 0.5
    for r in reqs:
        arrival = start + r.t
        while True:
            collect()
            dt = arrival - vtx.vtx_clock_s()
            if dt <= 0:
                break
            time.sleep(min(dt, 0.002))
        rs = ensure_resident(r.scene)
        res = (r.width, r.height)
        slot = None
        while slot is None:
            cand = (res, slot_next[res])
            slot_next[res] = (slot_next[res] + 1) % len(outs[res])
            if cand not in slot_busy:
                slot = cand
            else:
                collect(1)
        fr = outs[res][slot[1]]
        sc, centre, radius = built[r.scene]
        cam = scenes.orbit_camera(centre, radius, r.angle)
        if plain:
            tk = len(ticket_info) + len(done)
            sub = vtx.vtx_clock_s()
            vtx.vtx_render_scene(rs.handle, cam, opts, r.width, r.height, fr.rgba, fr.depth, fr.id, stream)
            ev = torch.cuda.Event(enable_timing=True)
            ev.record(stream)
            pending.append((ev, tk))
        else:
            sub = None
            job = vtx.make_job(rs.handle, 0, cam, opts, r.width, r.height, fr.rgba, fr.depth, fr.id)
            tk = vtx.vtx_server_submit(server, job)
        ticket_info[tk] = {"arrival": arrival, "scene": r.scene, "slot": slot, "t": r.t,
                           "pixels": r.width * r.height, "submit": sub}
        slot_busy[slot] = tk
        outstanding[r.scene] = outstanding.get(r.scene, 0) + 1
        last_use[r.scene] = arrival
    if plain:
        stream.synchronize()
        collect()
        sst = {"completed": len(done), "batches": len(done)}
    else:
        vtx.vtx_server_drain(server)
        collect()
        sst = vtx.vtx_server_stats_read(server)
        vtx.vtx_server_destroy(server)
    for rs in resident.values():
        rs.close()
    vtx.vtx_context_destroy(ctx)

    warm = args.serve_warmup
    lat = np.array([(c["done_s"] - c["arrival"]) * 1e3 for c in done if c["t"] >= warm])
    q = np.array([(c["launch_s"] - c["arrival"]) * 1e3 for c in done if c["t"] >= warm])
    bad = sum(1 for c in done if c["status"] != 0)
    span = max(c["done_s"] for c in done) - (start + warm)
    n_after = sum(1 for c in done if c["t"] >= warm)
    px = sum(c["pixels"] for c in done if c["t"] >= warm)
    fps = n_after / span
    out = {
        "metric": "frames/s",
        "value": round(fps, 3),
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": len(reqs),
        "warmup": sum(1 for r in reqs if r.t < warm),
        "ms_per_step": round(1e3 / fps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"served_mix_{len(pool)}scenes_{args.serve_rate:.0f}hz_{args.serve_seconds:.0f}s"
                               + ("_plain" if plain else ""),
                   "scenes": len(used), "atoms_min": min(built[k][0].n_atoms for k in used),
                   "atoms_max": max(built[k][0].n_atoms for k in used),
                   "resolutions": [list(x) for x in scenes.SERVE_RESOLUTIONS], "ssao_samples": 16,
                   "arrival_rate_hz": args.serve_rate, "mean_session_frames": 8,
                   "hbm_budget_bytes": budget or "full", "hbm_scenes_peak_bytes": hbm_peak,
                   "max_batch": args.serve_max_batch,
                   "launch": ("one vtx_render_scene per request, one stream" if plain else
                              "vtx_server: continuous batching into vtx_render_batch, 2 batches in flight")},
        "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 3), "p99": round(float(np.percentile(lat, 99)), 3),
                       "mean": round(float(lat.mean()), 3), "queue_p50": round(float(np.percentile(q, 50)), 3),
                       "frames": int(lat.size), "measured_from": "arrival", "to": "device completion (host callback)"},
        "megapixels_per_s": round(px / span / 1e6, 2),
        "server": {**sst, "mean_batch": round(sst["completed"] / max(1, sst["batches"]), 2)},
        "residency": {"scenes_created": created, "scenes_evicted": evicted},
        "failed_requests": bad,
    }
    print(json.dumps(out), flush=True)


def cpu_baseline(renders, scene_of, budget_s=12.0):
    """The oracle (FP64 C splatter + SSAO + shading) on the host cores, end to
    end.  Whole renders of the workload, in order, as many as fit the budget
    (at least one) when one render fits it.  Otherwise a sample of the first
    render: its fixed part (the oracle projects every primitive for any
    window), timed on a 1-pixel window, plus three full-width strips of 32
    rows at a quarter, half and three quarters of the height, whose time less
    three fixed parts gives the cost per pixel (each strip pixel is ray-cast
    and shaded once, as in a full frame; SSAO samples that leave a strip are
    not looked up); the frame's time is the fixed part plus that cost times
    its pixels."""
    from oracle import osplat
    osplat.build(force=False)
    threads = osplat.default_threads()
    r0 = renders[0]

    def timed(win, halo):
        a = time.perf_counter()
        osplat.render(scene_of(r0), r0.camera, r0.options, r0.W, r0.H, window=win, halo=halo, nthreads=threads)
        return time.perf_counter() - a

    fixed = timed((r0.W // 2, r0.H // 2, 1, 1), 0)
    rows = min(32, r0.H)
    strips = [(0, max(0, min(r0.H - rows, int(r0.H * f) - rows // 2)), r0.W, rows) for f in (0.25, 0.5, 0.75)]
    t1 = timed(strips[0], 0)
    per_px1 = max(t1 - fixed, 0.0) / (r0.W * rows)
    if fixed + per_px1 * r0.W * r0.H > budget_s:
        t_rest = sum(timed(w, 0) for w in strips[1:])
        px = 3 * r0.W * rows
        per_px = max(t1 + t_rest - 3 * fixed, 0.0) / px
        t_frame = fixed + per_px * r0.W * r0.H
        return {"value": 1.0 / t_frame, "unit": "frames/s", "cores": threads, "kind": "oracle",
                "sample": f"the first {r0.W}x{r0.H} render: fixed part {fixed:.2f} s (1-pixel window), three "
                          f"{r0.W}x{rows} strips at 1/4, 1/2, 3/4 of the height "
                          f"({t1 + t_rest:.2f} s for {px} px: {per_px * 1e6:.2f} us per pixel); frame time "
                          f"extrapolated to {t_frame:.1f} s; FP64 footprint splatter with accept sets + SSAO + "
                          f"shading"}
    n = 0
    px = 0
    t0 = time.perf_counter()
    while True:
        r = renders[n % len(renders)]
        osplat.render(scene_of(r), r.camera, r.options, r.W, r.H, nthreads=threads)
        n += 1
        px += r.W * r.H
        el = time.perf_counter() - t0
        if el >= budget_s or el / n * (n + 1) > 3 * budget_s:
            break
    sizes = sorted({f"{r.W}x{r.H}" for r in renders[:n]})
    return {"value": n / el, "unit": "frames/s", "cores": threads, "kind": "oracle",
            "sample": f"the first {n} render(s) of the workload ({', '.join(sizes)}; {px / 1e6:.1f} Mpx), "
                      f"FP64 footprint splatter with accept sets + SSAO + shading, {el:.1f} s"}


def frame_roofline(N, M, st, K, renders, ms_per_step):
    """The whole frame against its roofline, as the method's algorithmic cost
    per frame (summed over the step's renders): bytes B = 16 N + 8 M +
    8 (N_vis + M_vis) + 16 W H + 4 (covered pixels); lane-ops = 60 (N + M) +
    20 F_sphere + 50 F_cylinder + 25 K W H + 40 W H (F: every atom-fragment,
    the plain z-buffer count).  Roofline time = max(B / HBM peak,
    lane-ops / ALU peak); frac = roofline time / measured time."""
    f_cyl = st.get("fragments_hit_bond", 0)
    f_sph = st["fragments_hit"] - f_cyl
    px = sum(r.W * r.H for r in renders)
    covered = sum(int((r.out.id != -1).sum().item()) for r in renders)
    R = len(renders)
    B = 16.0 * N * R + 8.0 * M * R + 8.0 * st["visible"] + 16.0 * px + 4.0 * covered
    ops = (OPS_PRIM * (N + M) * R + OPS_SPHERE_FRAG * f_sph + OPS_CYL_FRAG * f_cyl + OPS_SAMPLE * K * px +
           OPS_PIXEL * px)
    t_hbm = B / (HBM_PEAK_GBS * 1e9) * 1e3
    t_alu = ops / (ALU_PEAK_TOPS * 1e12) * 1e3
    t_roof = max(t_hbm, t_alu)
    return {"bytes": round(B), "lane_ops": round(ops), "t_hbm_ms": round(t_hbm, 4), "t_alu_ms": round(t_alu, 4),
            "bound": "hbm" if t_hbm >= t_alu else "alu", "roofline_ms": round(t_roof, 4),
            "measured_ms": round(ms_per_step, 4), "frac": round(t_roof / ms_per_step, 4)}


def run_workload(args, workload, vtx, scenes, torch, stream, steps_arg, warmup_arg, cpu=True):
    """Times one workload (a single-frame scene or the trajectory batch) and
    returns its JSON record."""
    t0 = time.perf_counter()
    batch = workload == "trajectory"
    if batch:
        scene0, frames, cams, opts, viewports = scenes.trajectory()
        if args.tile:
            opts = dataclasses.replace(opts, tile_size=args.tile)
        name = f"trajectory_{scene0.n_atoms // 1000}k_{len(frames)}x{len(cams)}"
        runner = BatchRunner(vtx, scene0, frames, cams, opts, viewports, stream)
        N, M = scene0.n_atoms, scene0.n_bonds

        def scene_of(r):
            return scenes.Scene(frames[r.frame_index], scene0.radii, scene0.colors, scene0.bonds)
        config = {"workload": name, "atoms": N, "bonds": M, "trajectory_frames": len(frames),
                  "viewports": [list(v) for v in viewports], "renders_per_step": len(runner.renders),
                  "ssao_samples": int(opts.ssao_samples)}
        steps = steps_arg or 10
        warmup = warmup_arg if warmup_arg >= 0 else 2
    else:
        wl = {"ball_and_stick": scenes.ball_and_stick, "whole_cell": scenes.whole_cell,
              "plain_small": scenes.plain_small}[workload]()
        if args.tile:
            wl.options = dataclasses.replace(wl.options, tile_size=args.tile)
        name = wl.name
        runner = SingleRunner(vtx, wl, args.path, stream)
        N, M = wl.scene.n_atoms, wl.scene.n_bonds

        def scene_of(r):
            return wl.scene
        config = {"workload": name, "atoms": N, "bonds": M, "width": wl.width, "height": wl.height,
                  "ssao_samples": int(wl.options.ssao_samples),
                  "tile_size": frame_tile(wl.options.tile_size, wl.width, wl.height)}
        steps = steps_arg or 200
        warmup = warmup_arg if warmup_arg >= 0 else 20
    config["launch"] = runner.launch_form
    R = len(runner.renders)
    if args.autotune and not args.tile and (batch or args.path == "scene"):
        tuning = runner.autotune(args.tuning_cache)
        log(f"autotune: {tuning}")
        for r in runner.renders:
            r.tuned_tile = tuning["tile_size"]
        config["tile_size"] = tuning["tile_size"]
        config["autotune"] = tuning
    log(f"workload {name}: {N} atoms, {M} bonds, {R} render(s) per step, set up in {time.perf_counter() - t0:.1f} s")

    # exact fragment counts of these renders (early-outs off), untimed; then
    # the ray tests the normal frames run (early-outs on), untimed
    runner.step(vtx.VTX_FLAG_STATS)
    st = vtx.vtx_read_stats(stream)
    hit_px = int(sum(int((r.out.id != -1).sum().item()) for r in runner.renders))
    log(f"stats {st}, hit pixels {hit_px}")
    runner.step(vtx.VTX_FLAG_COUNT)
    stc = vtx.vtx_read_stats(stream)
    log(f"counted frame {stc}")

    if args.calibrate_copy_mb:
        src = torch.empty(args.calibrate_copy_mb << 18, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"calibration copy of {args.calibrate_copy_mb} MiB done")
        del src, dst

    for _ in range(warmup):
        runner.step()
    torch.cuda.synchronize()
    vtx.vtx_reset_timings(stream)
    log(f"warmup {warmup} done; timing {steps} steps")

    main_flags = vtx.VTX_FLAG_TIMING if args.kernel_events == "timed" else 0
    torch.cuda.synchronize()
    ts = time.perf_counter()
    for _ in range(steps):
        runner.step(main_flags)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - ts
    if args.kernel_events == "separate":
        for _ in range(steps):
            runner.step(vtx.VTX_FLAG_TIMING)
    timings = vtx.vtx_read_timings(stream)
    st_after = vtx.vtx_read_stats(stream)
    ms_per_step = elapsed / steps * 1e3
    fps = steps * R / elapsed
    log(f"timed: {ms_per_step:.3f} ms/step, {fps:.1f} frames/s; kernels {timings}")

    # latency of single steps submitted and awaited one at a time
    lat = []
    for _ in range(args.latency_frames if not batch else min(args.latency_frames, 20)):
        a = time.perf_counter()
        runner.step()
        stream.synchronize()
        lat.append((time.perf_counter() - a) * 1e3)
    lat = np.array(lat)

    other = []
    for form, fn in (runner.other_forms if args.compare else []):
        for _ in range(max(1, warmup)):
            fn()
        torch.cuda.synchronize()
        o_steps = max(1, steps // 2) if batch else steps
        a = time.perf_counter()
        for _ in range(o_steps):
            fn()
        torch.cuda.synchronize()
        pe = time.perf_counter() - a
        other.append({"launch": form, "frames_per_s": round(o_steps * R / pe, 3),
                      "ms_per_step": round(pe / o_steps * 1e3, 4)})
        log(f"other launch form: {other[-1]}")

    # roofline of each kernel (per step = sums over the step's renders, device
    # time of each kernel from its own dispatch events); the dominant one goes
    # in the JSON's roofline
    K = int(runner.renders[0].options.ssao_samples)
    f_total = st["fragments_hit"]
    f_cyl = st.get("fragments_hit_bond", 0)
    f_sph = f_total - f_cyl
    t_cyl = stc.get("fragments_tested_bond", 0)
    t_sph = stc["fragments_tested"] - t_cyl

    def eff_tile(r):
        return frame_tile(getattr(r, "tuned_tile", 0) or r.options.tile_size, r.W, r.H)
    tiles = sum(n_tiles(eff_tile(r), r.W, r.H) for r in runner.renders)
    per_kernel = {
        "project": ("hbm", (16.0 * N + 8.0 * M) * R, timings["ms_project"]),
        "resolve": ("alu", float(OPS_SPHERE_FRAG * f_sph + OPS_CYL_FRAG * f_cyl), timings["ms_resolve"]),
        "shade": ("alu", float((OPS_PIXEL + OPS_SAMPLE * K) * hit_px), timings["ms_shade"]),
        "scatter": ("hbm", 12.0 * st["visible"] + 4.0 * st["pairs"], timings["ms_scatter"]),
        "scan": ("hbm", 12.0 * tiles, timings["ms_scan"]),
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
    if "resolve" in kern:
        # the resolve priced on the ray tests the timed frames run (early-outs
        # on), beside the plain z-buffer pricing above
        done = float(OPS_SPHERE_FRAG * t_sph + OPS_CYL_FRAG * t_cyl)
        ach = done / (timings["ms_resolve"] * 1e-3) / 1e12
        kern["resolve"].update({
            "frac_work_done": round(ach / ALU_PEAK_TOPS, 4),
            "tests_all": st["fragments_tested"], "tests_done": stc["fragments_tested"],
            "skip_rate": round(1.0 - stc["fragments_tested"] / max(1, st["fragments_tested"]), 4),
            "tests_done_per_atom_fragment": round(stc["fragments_tested"] / max(1, f_total), 4),
            "early_outs": {k: stc[k] for k in ("fragments_skipped", "records_culled", "lists_stopped",
                                               "chunks_stopped")}})
    dom = max(kern, key=lambda k: kern[k]["ms"])
    roof = {k: v for k, v in kern[dom].items() if k in ("bound", "achieved", "peak", "unit", "frac")}
    scene_path = batch or runner.path == "scene"
    res_tiles = sorted({eff_tile(r) for r in runner.renders})
    # the launches of each stage, named as the kernel trace names them (template
    # arguments: launch form; count: scene, rest pass, atoms only; resolve:
    # tile, counting, two-pass; shade: noise)
    form = "JobList" if batch else "OneJob"
    atoms_only = "true" if M == 0 else "false"
    noise = "true" if getattr(runner.renders[0].options, "ssao_noise", 0) else "false"
    launched = {"project": ([f"k_cluster_cull<{form}>", f"k_count<{form},true,false,{atoms_only}>"] if scene_path
                            else [f"k_count<{form},false,false,false>"]),
                "scatter": [f"k_scatter<{form}>"],
                "resolve": ([k for t in res_tiles for k in (f"k_resolve<{t},{form},false,false>",
                                                             f"k_resolve_tail<{t},{form},false,false>")] +
                            (["k_refine<JobList>"] if batch else [])),
                "shade": [f"k_shade<{form},{noise}>"],
                "scan": []}
    traffic = measured_traffic(name, launched[dom]) if (launched[dom] and scene_path) else None
    roof = {"kernel": dom, "launches": launched[dom], **roof, "traffic": None if traffic is None else round(traffic),
            "timing": "per-kernel dispatch events (hipExtLaunchKernel start/stop), mean over the timed steps"}
    # the whole step against the chip's VALU issue slots: the counted VALU
    # wave instructions of every launch of the step (committed counter
    # summary), 4 cycles each on 1024 SIMDs at 2.4 GHz, over the measured step
    frame_rl = frame_roofline(N, M, st, K, runner.renders, ms_per_step)
    frame_valu = None
    if scene_path:
        step_kernels = (launched["project"] + [f"k_layers<{form}>", f"k_tile_offsets<{form}>"] + launched["scatter"] +
                        launched["resolve"] + launched["shade"])
        v = measured_valu(name, step_kernels)
        if v is not None:
            frame_valu = {"valu_wave_instr": round(v), "issue_frac": round(v * 4 / (ms_per_step * 1e-3 * 1024 * 2.4e9), 4),
                          "lane_instr_per_priced_lane_op": round(v * 64 / max(1.0, frame_rl["lane_ops"]), 3),
                          "source": "profiles/" + VALU_FILES[name],
                          "launches": step_kernels}

    out = {
        "metric": "frames/s",
        "value": round(fps, 3),
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": config,
        "other_launch_forms": other,
        "atom_fragments_per_s": round(f_total * steps / elapsed, 1),
        "atom_fragments_per_step": f_total,
        "latency_ms": ({"p50": round(float(np.percentile(lat, 50)), 4),
                        "p99": round(float(np.percentile(lat, 99)), 4), "steps": int(lat.size)}
                       if lat.size else None),
        "kernels": kern,
        "roofline": roof,
        "frame_roofline": frame_rl,
        "frame_valu": frame_valu,
        "bins": {"visible": st["visible"], "pairs": st["pairs"], "overflow_tiles": st_after["overflow_tiles"]},
    }
    if cpu and not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(runner.renders, scene_of)
    runner.close()
    return out


def run_ses(args, vtx, scenes, torch, stream, cpu=True):
    """The solvent excluded surface of the 50k-atom protein-like globule
    (frame 0 of the trajectory workload, van der Waals radii, probe 1.4 A) on
    a 0.5 A grid reaching the probe radius and two steps past every atom:
    one vtx_ses call per step (SAS marking, the three distance passes, the
    triangle counts, their scan and the emission)."""
    scene0, _, _, _, _ = scenes.trajectory(n_frames=1)
    pos, rad = scene0.positions, scene0.radii
    probe, h = 1.4, 0.5
    lo = np.min(pos - rad[:, None], axis=0) - probe - 2 * h
    hi = np.max(pos + rad[:, None], axis=0) + probe + 2 * h
    dims = tuple(int(d) for d in np.ceil((hi - lo) / h).astype(int) + 1)
    origin = lo.astype(np.float32)
    npts = int(np.prod(dims))
    ncubes = int(np.prod([d - 1 for d in dims]))
    dp = torch.from_numpy(np.ascontiguousarray(pos)).cuda()
    dr = torch.from_numpy(np.ascontiguousarray(rad)).cuda()
    field = torch.empty(dims[::-1], dtype=torch.float32, device="cuda")
    cap = 4_000_000
    tri = torch.empty((cap, 9), dtype=torch.float32, device="cuda")
    ntri = torch.zeros(1, dtype=torch.int64, device="cuda")

    def step():
        vtx.vtx_ses(dp, dr, pos.shape[0], probe, origin, h, dims, field, tri, cap, ntri, stream)
    for _ in range(3):
        step()
    torch.cuda.synchronize()
    n_tri = int(ntri.item())
    steps = 20
    a = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - a) / steps * 1e3
    # algorithmic bytes: the mark (1 B), three distance passes (4 B written
    # each, 1 + 4 + 4 B read), the field read by the count and the emission
    # (4 B each), per cube the count written, scanned and read (12 B), and
    # 36 B per triangle written; the atoms (16 B each)
    B = 16.0 * pos.shape[0] + (1 + 12 + 9 + 8) * npts + 12.0 * ncubes + 36.0 * n_tri
    out = {"value": round(1e3 / ms, 3), "unit": "surfaces/s", "ms_per_step": round(ms, 4), "steps": steps,
           "config": {"workload": f"ses_globule_{pos.shape[0] // 1000}k_h{h}", "atoms": int(pos.shape[0]),
                      "probe": probe, "spacing": h, "grid": list(dims), "triangles": n_tri},
           "roofline": {"bound": "hbm", "achieved": round(B / (ms * 1e-3) / 1e9, 3), "peak": HBM_PEAK_GBS,
                        "unit": "GB/s", "frac": round(B / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4), "bytes": round(B),
                        "timing": "whole vtx_ses call, host clock over synchronized steps"}}
    traffic = measured_traffic(out["config"]["workload"], SES_KERNELS)
    out["roofline"]["traffic"] = None if traffic is None else round(traffic)
    log(f"ses: {out}")
    if cpu and not args.no_cpu_baseline:
        # the oracle on a slab of the grid (one eighth of its z extent through
        # the middle), scaled to the whole grid
        from oracle import oses
        nz = max(2, dims[2] // 8)
        z0 = (dims[2] - nz) // 2
        sub_origin = (origin + np.array([0.0, 0.0, h * z0])).astype(np.float32)
        sub_dims = (dims[0], dims[1], nz)
        a = time.perf_counter()
        ref = oses.ses_field(pos, rad, probe, sub_origin, np.float32(h), sub_dims)
        oses.marching_cubes(ref["f"], sub_origin, np.float32(h))
        el = time.perf_counter() - a
        t_full = el * (dims[2] - 1) / (nz - 1)
        out["cpu_baseline"] = {"value": 1.0 / t_full, "unit": "surfaces/s", "cores": 1, "kind": "oracle",
                               "sample": f"the oracle (NumPy + scipy k-d tree, one core) on the {dims[0]}x{dims[1]}x"
                                         f"{nz} middle slab of the grid ({el:.1f} s), scaled by the cube layers "
                                         f"({dims[2] - 1} / {nz - 1})"}
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=0, help="timed steps (0: 200 frames, or 10 batches)")
    ap.add_argument("--warmup", type=int, default=-1, help="untimed steps first (-1: 20 frames, or 2 batches)")
    ap.add_argument("--workload", default="whole_cell",
                    choices=["ball_and_stick", "whole_cell", "trajectory", "served", "plain_small"])
    ap.add_argument("--also", default="ball_and_stick,ses",
                    help="comma-separated workloads also timed and reported under their own key "
                         "(\"\" for none; default: ball_and_stick and ses (the solvent excluded surface "
                         "of the 50k-atom globule) beside the whole cell)")
    ap.add_argument("--serve-seconds", type=float, default=60.0, help="served mix: arrival window")
    ap.add_argument("--serve-warmup", type=float, default=5.0, help="served mix: arrivals excluded from stats")
    ap.add_argument("--serve-rate", type=float, default=200.0, help="served mix: frame requests per second")
    ap.add_argument("--serve-budget-gb", type=float, default=0.0,
                    help="served mix: HBM budget of resident scenes (0 = the full memory)")
    ap.add_argument("--serve-max-batch", type=int, default=64)
    ap.add_argument("--serve-mode", choices=["server", "plain"], default="server",
                    help="served mix: the library's server, or one vtx_render_scene per request")
    ap.add_argument("--tile", type=int, default=0, help="tile size (0 = library default)")
    ap.add_argument("--path", choices=["scene", "plain"], default="scene",
                    help="single-frame workloads: scene = resident scene (vtx_scene_create before timing, "
                         "vtx_render_scene per frame); plain = vtx_render on the caller's arrays each frame")
    ap.add_argument("--compare", type=int, default=1,
                    help="also time the other launch form of the same renders (reported beside)")
    ap.add_argument("--latency-frames", type=int, default=50)
    ap.add_argument("--kernel-events", choices=["timed", "separate"], default="separate",
                    help="per-kernel device times: every kernel dispatched with its own start and stop "
                         "events, in a pass of the same length right after the timed one (separate), or "
                         "in the timed steps themselves (timed: the events add ~5 us per kernel to the "
                         "frame time)")
    ap.add_argument("--autotune", type=int, default=1,
                    help="1: choose the tile size with vtx_autotune on the workload's renders before timing "
                         "(resident-scene and batch forms; renders that leave tile_size at 0 then use it); "
                         "0: the library default (16, raised for large images)")
    ap.add_argument("--tuning-cache", default=None, help="JSON cache file for --autotune")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy-mb", type=int, default=0,
                    help="before timing, run one device copy of this many MiB (reference for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the renderer has no multi-GPU path "
              "(--gpus must be 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2501_12750_amd import scenes, vtx

    if args.workload == "served":
        args.served_inputs = build_served(args, scenes)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    if args.workload == "served":
        run_served(args, vtx, scenes, torch, torch.cuda.Stream())
        return
    out = run_workload(args, args.workload, vtx, scenes, torch, stream, args.steps, args.warmup)
    for extra in [w for w in args.also.split(",") if w and w != args.workload]:
        if extra == "ses":
            rec = run_ses(args, vtx, scenes, torch, stream)
            out[rec["config"]["workload"]] = rec
            continue
        if extra not in ("ball_and_stick", "whole_cell", "trajectory", "plain_small"):
            raise SystemExit(f"--also: unknown workload {extra}")
        log(f"also timing {extra}")
        rec = run_workload(args, extra, vtx, scenes, torch, stream, 0, -1, cpu=False)
        out[rec["config"]["workload"]] = {k: rec[k] for k in ("value", "unit", "ms_per_step", "config",
                                                               "other_launch_forms", "atom_fragments_per_s",
                                                               "latency_ms", "kernels", "roofline",
                                                               "frame_roofline", "frame_valu", "bins")}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
