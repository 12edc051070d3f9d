"""Serving: requests over several device-resident scenes, traced by one persistent kernel
fed from a work queue, give the same result as tracing each request alone. Needs an
MI355X."""
import sys
import time

import numpy as np
import pytest

from paper_2601_20429_amd import inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
from paper_2601_20429_amd import grtx  # noqa: E402

AMIN = float(np.float32(1.0 / 255.0))


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    yield
    torch.cuda.synchronize()


def wait_all(srv, tickets, limit_s):
    t0 = time.time()
    pending = set(tickets)
    while pending and time.time() - t0 < limit_s:
        pending = {t for t in pending if srv.poll(t) is None}
        time.sleep(0.001)
    assert not pending, "requests did not finish"


def alone(bvh, cam, k=16, T_min=1e-3, **kw):
    o, d = grtx.pinhole_rays(cam)
    out = grtx.trace(bvh, o, d, k=k, T_min=T_min, **kw)
    torch.cuda.synchronize()
    return out


def test_mix_equals_alone():
    say("serving mix vs alone")
    scenes = [inputs.cluster_scene(10 + i, n, 3) for i, n in enumerate([20_000, 50_000, 100_000])]
    bvhs = [grtx.build(grtx.SceneTensors.from_scene(s, "cuda"), alpha_min=AMIN) for s in scenes]
    torch.cuda.synchronize()
    srv = grtx.Server(memory_budget=40 << 30, k=16, T_min=1e-3)
    ids = [srv.add_scene(b) for b in bvhs]
    rng = np.random.default_rng(50)
    reqs = []
    # sizes include ragged ones (edge tiles partly outside the image)
    sizes = [(64, 64), (128, 96), (200, 160), (96, 72), (100, 75), (37, 53)]
    for j in range(24):
        sid = int(rng.integers(len(ids)))
        w, h = sizes[int(rng.integers(len(sizes)))]
        cam = inputs.Camera(inputs.random_orbit_eye(rng), (0.0, 0.0, 0.0), (0.0, 0.0, 1.0), 60.0, w, h)
        reqs.append((sid, cam, srv.submit(sid, cam)))
        if j % 5 == 4:
            time.sleep(0.002)  # let some requests arrive while others run
    wait_all(srv, [t for _, _, t in reqs], 60)
    st = srv.stats()
    say(st)
    assert st["completed"] == 24 and st["p99_ms"] >= st["p50_ms"] > 0
    assert 1 <= st["launches"] < 24  # requests joined running launches
    for sid, cam, t in reqs:
        got = srv.result(t)
        ref = alone(bvhs[sid], cam)
        for key in ["rgb", "depth", "opacity"]:
            assert torch.equal(got[key], ref[key]), (t, cam.width, cam.height, key)
        srv.release(t)
    assert srv.stats()["bytes_in_use"] == 0
    srv.close()


def test_requests_join_the_running_launch():
    """Requests submitted while a long request is being traced join its launch: one
    launch serves them all, each result equal to its camera traced alone."""
    say("serving join")
    scene = inputs.cluster_scene(21, 500_000, 3)
    bvh = grtx.build(grtx.SceneTensors.from_scene(scene, "cuda"), alpha_min=AMIN)
    torch.cuda.synchronize()
    srv = grtx.Server(memory_budget=16 << 30, k=16, T_min=1e-3)
    srv.add_scene(bvh)
    rng = np.random.default_rng(52)
    cams = [inputs.Camera(inputs.random_orbit_eye(rng), (0.0, 0.0, 0.0), (0.0, 0.0, 1.0), 60.0, w, h)
            for w, h in [(1920, 1080), (128, 128), (64, 48), (256, 200), (31, 17)]]
    tickets = [srv.submit(0, c) for c in cams]
    wait_all(srv, tickets, 60)
    st = srv.stats()
    say(st)
    assert st["completed"] == len(cams) and st["launches"] == 1
    for cam, t in zip(cams, tickets):
        got = srv.result(t)
        ref = alone(bvh, cam)
        for key in ["rgb", "depth", "opacity"]:
            assert torch.equal(got[key], ref[key]), (cam.width, key)
        srv.release(t)
    srv.close()


def test_admission_under_memory_pressure():
    """With a budget that holds one request's outputs, the second request waits in the
    queue until the first is released, a third is withdrawn while queued (never traced
    or counted), and the second's result equals its camera traced alone."""
    say("serving admission")
    scene = inputs.cluster_scene(12, 50_000, 3)
    bvh = grtx.build(grtx.SceneTensors.from_scene(scene, "cuda"), alpha_min=AMIN)
    torch.cuda.synchronize()
    rng = np.random.default_rng(53)
    cams = [inputs.Camera(inputs.random_orbit_eye(rng), (0.0, 0.0, 0.0), (0.0, 0.0, 1.0), 60.0, 256, 256)
            for _ in range(3)]
    rb = grtx.request_bytes(cams[0])
    # the budget's fixed part (kernel pool, queue, scene copy), read from a probe server
    probe = grtx.Server(memory_budget=16 << 30, k=16, T_min=1e-3)
    probe.add_scene(bvh)
    t = probe.submit(0, cams[0])
    wait_all(probe, [t], 30)
    fixed = (16 << 30) - probe.stats()["bytes_available"]
    probe.release(t)
    probe.close()
    srv = grtx.Server(memory_budget=fixed + rb + rb // 2, k=16, T_min=1e-3)
    srv.add_scene(bvh)
    a, b, c = (srv.submit(0, cam) for cam in cams)
    wait_all(srv, [a], 30)
    time.sleep(0.05)
    assert srv.poll(b) is None and srv.poll(c) is None  # both wait for memory
    assert srv.stats()["bytes_in_use"] == rb
    srv.release(c)  # withdrawn while queued
    got_a = srv.result(a)
    srv.release(a)
    wait_all(srv, [b], 30)
    got_b = srv.result(b)
    st = srv.stats()
    say(st)
    assert st["submitted"] == 2 and st["completed"] == 2 and st["bytes_in_use"] == rb
    assert st["bytes_arena"] <= st["bytes_available"]
    for cam, got in [(cams[0], got_a), (cams[1], got_b)]:
        ref = alone(bvh, cam)
        for key in ["rgb", "depth", "opacity"]:
            assert torch.equal(got[key], ref[key]), key
    srv.release(b)
    assert srv.stats()["bytes_in_use"] == 0
    srv.close()


def test_served_requests_match_oracle():
    """The serving workload's scenes (100k, 500k, 1M and 3M Gaussians) at each of its
    resolutions (256x256, 512x512, 800x800, 1920x1080), all sixteen requests in one mix:
    every served image equals the request's camera traced alone bit for bit, and that trace
    matches the oracle on sampled pixels by the per-ray rule (which chains the served
    output to the oracle)."""
    import oracle
    from tests import parity
    cfg = inputs.SERVE
    say("serving vs oracle")
    scenes = [inputs.cluster_scene(seed, n, 3) for seed, n in zip(cfg["scene_seeds"], cfg["scene_sizes"])]
    bvhs = [grtx.build(grtx.SceneTensors.from_scene(s, "cuda"), alpha_min=AMIN) for s in scenes]
    torch.cuda.synchronize()
    srv = grtx.Server(memory_budget=64 << 30, k=cfg["k"], T_min=cfg["T_min"])
    ids = [srv.add_scene(b) for b in bvhs]
    rng = np.random.default_rng(51)
    reqs = []
    for sid in ids:
        for w, h in cfg["resolutions"]:
            cam = inputs.Camera(inputs.random_orbit_eye(rng), (0.0, 0.0, 0.0), (0.0, 0.0, 1.0), 60.0, w, h)
            reqs.append((sid, cam, srv.submit(sid, cam)))
    t0 = time.time()
    pending = {t for _, _, t in reqs}
    while pending and time.time() - t0 < 120:
        pending = {t for t in pending if srv.poll(t) is None}
        time.sleep(0.001)
    assert not pending, "requests did not finish"
    for j, (sid, cam, t) in enumerate(reqs):
        got = srv.result(t)
        o, d = grtx.pinhole_rays(cam)
        alone = grtx.trace(bvhs[sid], o, d, k=cfg["k"], T_min=cfg["T_min"], image_width=cam.width, hit_capacity=512)
        torch.cuda.synchronize()
        for key in ["rgb", "depth", "opacity"]:
            assert torch.equal(got[key], alone[key]), (t, key)
        srv.release(t)
        idx = inputs.ray_subsample(200 + j, cam.n_rays, 48)
        ti = torch.from_numpy(idx).cuda()
        sub = {key: v.index_select(0, ti).cpu().numpy() for key, v in alone.items()}
        so, sd = o.index_select(0, ti).cpu().numpy(), d.index_select(0, ti).cpu().numpy()
        ref = oracle.render(scenes[sid], so, sd, AMIN, cfg["T_min"], cap=512)
        s = parity.compare_render(scenes[sid], so, sd, sub, ref, AMIN, cfg["T_min"],
                                  label=f"served scene {cfg['scene_sizes'][sid]} {cam.width}x{cam.height}")
        say(cfg["scene_sizes"][sid], f"{cam.width}x{cam.height}", s)
    assert srv.stats()["bytes_in_use"] == 0
    srv.close()


def test_request_too_large_is_refused():
    say("serving capacity")
    scene = inputs.cluster_scene(10, 20_000, 3)
    bvh = grtx.build(grtx.SceneTensors.from_scene(scene, "cuda"), alpha_min=AMIN)
    srv = grtx.Server(memory_budget=16 << 30, k=16, max_request_rays=1 << 16)
    srv.add_scene(bvh)
    with pytest.raises(grtx.GrtxError) as e:
        srv.submit(0, inputs.orbit_camera(512, 512))  # more pixels than a request may hold
    assert e.value.status == grtx.ERR_CAPACITY
    t = srv.submit(0, inputs.orbit_camera(64, 64))
    wait_all(srv, [t], 30)
    srv.release(t)
    srv.close()
    with pytest.raises(grtx.GrtxError) as e:
        grtx.Server(memory_budget=1 << 20, k=16)  # cannot hold the kernel's checkpoint pool
    assert e.value.status == grtx.ERR_CAPACITY
