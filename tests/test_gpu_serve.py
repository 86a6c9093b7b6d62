"""Served renders (vtx_server_*): a frame served among many others equals the
same frame rendered alone (needs an MI355X)."""
import math

import numpy as np
import pytest

from paper_2501_12750_amd import scenes

pytestmark = pytest.mark.gpu

SIZES = [(320, 180), (333, 221), (640, 360), (96, 54)]


@pytest.fixture(scope="module")
def vtx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    from paper_2501_12750_amd import vtx as v
    return v


@pytest.fixture(scope="module")
def pool():
    specs = [scenes.ServedScene("vdw", 6000, 11), scenes.ServedScene("ball_and_stick", 5000, 12),
             scenes.ServedScene("vdw", 30000, 13), scenes.ServedScene("ball_and_stick", 20000, 14)]
    return [s.build() for s in specs]


def requests(n, n_scenes, seed):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        W, H = SIZES[int(rng.integers(len(SIZES)))]
        out.append((int(rng.integers(n_scenes)), W, H, float(rng.uniform(0, 2 * math.pi))))
    return out


def alone(vtx, rs, cam, opts, W, H):
    import torch
    fr = rs.render(cam, opts, W, H)
    torch.cuda.synchronize()
    return fr.numpy()


def assert_identical(a, b, what):
    for k in ("depth", "id", "rgba"):
        assert np.array_equal(a[k], b[k]), f"{what}: {k} differs at {np.count_nonzero(a[k] != b[k])} pixels"


def test_served_frames_equal_frames_rendered_alone(vtx, pool):
    import torch
    ctx = vtx.vtx_context_create(0, 0)
    rss = [vtx.ResidentScene(ctx, vtx.DeviceScene(sc)) for sc, _, _ in pool]
    opts = scenes.Options(ssao_samples=16, ssao_radius=2.0)
    stream = torch.cuda.Stream()
    server = vtx.vtx_server_create(ctx, 16, 2, stream)
    reqs = requests(48, len(pool), 7)
    frames, tickets = [], {}
    for i, (k, W, H, ang) in enumerate(reqs):
        sc, c, r = pool[k]
        fr = vtx.Frame(W, H)
        frames.append(fr)
        cam = scenes.orbit_camera(c, r, ang)
        tickets[vtx.vtx_server_submit(server, vtx.make_job(rss[k].handle, 0, cam, opts, W, H, fr.rgba, fr.depth,
                                                           fr.id))] = i
    vtx.vtx_server_drain(server)
    done = vtx.vtx_server_poll(server, 1000)
    st = vtx.vtx_server_stats_read(server)
    vtx.vtx_server_destroy(server)
    assert len(done) == len(reqs) and all(c["status"] == 0 for c in done)
    assert sorted(tickets[c["ticket"]] for c in done) == list(range(len(reqs)))
    assert all(c["submit_s"] <= c["launch_s"] <= c["done_s"] for c in done)
    print(st, flush=True)
    assert st["completed"] == len(reqs) and st["batches"] < len(reqs) and st["max_batch_seen"] > 1
    torch.cuda.synchronize()
    for i, (k, W, H, ang) in enumerate(reqs):
        sc, c, r = pool[k]
        ref = alone(vtx, rss[k], scenes.orbit_camera(c, r, ang), opts, W, H)
        assert_identical(frames[i].numpy(), ref, f"request {i}")
        assert np.count_nonzero(ref["id"] != 0xFFFFFFFF) > 0
    for rs in rss:
        rs.close()
    vtx.vtx_context_destroy(ctx)


def test_served_under_a_small_budget_with_eviction(vtx, pool):
    """The budget holds the largest scene but not all of them: scenes are
    created on first use and the least recently used idle one is evicted
    when a new one does not fit."""
    import torch
    need = [vtx.vtx_scene_footprint_bytes(sc.n_atoms, sc.n_bonds) for sc, _, _ in pool]
    budget = max(need) + min(need)
    ctx = vtx.vtx_context_create(0, budget)
    opts = scenes.Options(ssao_samples=8, ssao_radius=2.0)
    stream = torch.cuda.Stream()
    server = vtx.vtx_server_create(ctx, 8, 2, stream)
    resident, last, evicted = {}, {}, 0
    rng = np.random.default_rng(3)
    checked = 0
    for session in range(10):
        k = int(rng.integers(len(pool)))
        if k not in resident:
            while True:
                try:
                    resident[k] = vtx.ResidentScene(ctx, vtx.DeviceScene(pool[k][0]))
                    break
                except vtx.VtxError as e:
                    assert e.code == vtx.VTX_EBUSY
                    j = min(resident, key=lambda j: last[j])
                    resident.pop(j).close()
                    evicted += 1
        assert vtx.vtx_context_bytes_in_use(ctx) <= budget
        sc, c, r = pool[k]
        W, H = SIZES[session % len(SIZES)]
        frames = [vtx.Frame(W, H) for _ in range(4)]
        angles = [0.3 * session + 0.05 * f for f in range(4)]
        for fr, a in zip(frames, angles):
            vtx.vtx_server_submit(server, vtx.make_job(resident[k].handle, 0, scenes.orbit_camera(c, r, a), opts,
                                                       W, H, fr.rgba, fr.depth, fr.id))
        vtx.vtx_server_drain(server)     # the session's frames are done before its scene may go
        assert all(x["status"] == 0 for x in vtx.vtx_server_poll(server, 100))
        torch.cuda.synchronize()
        for fr, a in zip(frames, angles):
            assert_identical(fr.numpy(), alone(vtx, resident[k], scenes.orbit_camera(c, r, a), opts, W, H),
                             f"session {session}")
            checked += 1
        last[k] = session
    vtx.vtx_server_destroy(server)
    assert evicted > 0 and checked == 40
    for rs in resident.values():
        rs.close()
    assert vtx.vtx_context_bytes_in_use(ctx) == 0
    vtx.vtx_context_destroy(ctx)


def test_server_refuses_bad_requests_and_finishes_its_queue(vtx, pool):
    import torch
    ctx = vtx.vtx_context_create(0, 0)
    rs = vtx.ResidentScene(ctx, vtx.DeviceScene(pool[0][0]))
    opts = scenes.Options()
    stream = torch.cuda.Stream()
    server = vtx.vtx_server_create(ctx, 4, 1, stream)
    sc, c, r = pool[0]
    cam = scenes.orbit_camera(c, r, 0.0)
    fr = vtx.Frame(64, 64)
    bad = vtx.make_job(rs.handle, 3, cam, opts, 64, 64, fr.rgba, fr.depth, fr.id)       # no frame 3
    with pytest.raises(vtx.VtxError) as e:
        vtx.vtx_server_submit(server, bad)
    assert e.value.code == vtx.VTX_EINVAL
    frames = [vtx.Frame(64, 64) for _ in range(12)]
    for f in frames:
        vtx.vtx_server_submit(server, vtx.make_job(rs.handle, 0, cam, opts, 64, 64, f.rgba, f.depth, f.id))
    vtx.vtx_server_destroy(server)        # renders the queue before it stops
    torch.cuda.synchronize()
    ref = alone(vtx, rs, cam, opts, 64, 64)
    for f in frames:
        assert_identical(f.numpy(), ref, "queued at destroy")
    with pytest.raises(vtx.VtxError):
        vtx.vtx_server_create(ctx, 0, 1, stream)
    rs.close()
    vtx.vtx_context_destroy(ctx)
