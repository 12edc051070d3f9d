"""Serving: requests over several device-resident scenes, packed into shared launches,
give the same result as tracing each request alone. Needs an MI355X."""
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


def test_mix_equals_alone():
    say("serving mix vs alone")
    scenes = [inputs.cluster_scene(10 + i, n, 3) for i, n in enumerate([20_000, 50_000, 100_000])]
    bvhs = [grtx.build(grtx.SceneTensors.from_scene(s, "cuda"), alpha_min=AMIN) for s in scenes]
    torch.cuda.synchronize()
    srv = grtx.Server(memory_budget=40 << 30, slots=2, k=16, T_min=1e-3)
    ids = [srv.add_scene(b) for b in bvhs]
    rng = np.random.default_rng(50)
    reqs = []
    for j in range(24):
        sid = int(rng.integers(len(ids)))
        w, h = [(64, 64), (128, 96), (200, 160), (96, 72)][int(rng.integers(4))]
        cam = inputs.Camera(inputs.random_orbit_eye(rng), (0.0, 0.0, 0.0), (0.0, 0.0, 1.0), 60.0, w, h)
        reqs.append((sid, cam, srv.submit(sid, cam)))
        if j % 5 == 4:
            time.sleep(0.002)  # let some requests arrive while others run
    t0 = time.time()
    pending = {t for _, _, t in reqs}
    while pending and time.time() - t0 < 60:
        pending = {t for t in pending if srv.poll(t) is None}
        time.sleep(0.001)
    assert not pending, "requests did not finish"
    st = srv.stats()
    say(st)
    assert st["completed"] == 24 and st["p99_ms"] >= st["p50_ms"] > 0
    launches = {}
    for sid, cam, t in reqs:
        got = srv.result(t)
        launches.setdefault(got["t_launch"], 0)
        launches[got["t_launch"]] += 1
        o, d = grtx.pinhole_rays(cam)
        alone = grtx.trace(bvhs[sid], o, d, k=16, T_min=1e-3)
        torch.cuda.synchronize()
        for key in ["rgb", "depth", "opacity"]:
            assert torch.equal(got[key], alone[key]), (t, key)
        srv.release(t)
    assert max(launches.values()) > 1  # several requests shared one launch
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
    srv = grtx.Server(memory_budget=64 << 30, slots=2, k=cfg["k"], T_min=cfg["T_min"])
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
    pool = 0
    srv = grtx.Server(memory_budget=8 << 30, slots=1, k=16, max_batch_rays=1 << 16)
    srv.add_scene(bvh)
    with pytest.raises(grtx.GrtxError) as e:
        srv.submit(0, inputs.orbit_camera(512, 512))  # more rays than one batch holds
    assert e.value.status == grtx.ERR_CAPACITY
    t = srv.submit(0, inputs.orbit_camera(64, 64))
    t0 = time.time()
    while srv.poll(t) is None and time.time() - t0 < 30:
        time.sleep(0.001)
    assert srv.poll(t) is not None
    srv.release(t)
    srv.close()
    with pytest.raises(grtx.GrtxError) as e:
        grtx.Server(memory_budget=1 << 20, slots=2, k=16)  # cannot hold the checkpoint pools
    assert e.value.status == grtx.ERR_CAPACITY
