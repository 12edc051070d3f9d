"""Benchmark: Gaussian ray tracing of a 100k-Gaussian scene at 800x800, k = 16, on one GPU.

One step is the whole hot path over one frame: pinhole ray generation, the LBVH build
over the Gaussians (setup, Morton codes, radix sort, radix tree, refit) and the
multi-round checkpointed trace with blending. Inputs (scene parameters) are resident on
the GPU before timing starts. Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
# algorithmic bytes per unit of work: what one node fetch, leaf test, blended hit, list
# entry and ray must move at least
B_NODE = 64          # node record: four quantized child boxes + four child references
B_LEAF = 48          # unit-sphere transform of a leaf (3 x float4)
B_BLEND_INST = 64    # full instance record re-read for blending
B_LIST = 16          # one checkpoint / eviction entry written and read back (8 B each way)
B_RAY = 24 + 20      # ray in (origin, direction); rgb, depth, opacity out


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def run_serving(n_requests, rates):
    """Serving workload: four device-resident scenes (100k, 500k, 1M, 3M Gaussians), Poisson
    arrivals, each a random camera on the radius-3 sphere at a resolution drawn from
    {256^2, 512^2, 800^2, 1920x1080}, k = 16; latency is submission to result. One server,
    one run of `n_requests` per arrival rate (requests/s)."""
    import threading

    import numpy as np
    import torch

    from paper_2601_20429_amd import grtx, inputs

    cfg = inputs.SERVE
    amin = float(np.float32(cfg["alpha_min"]))
    bvhs, tensors = [], []
    for seed, n in zip(cfg["scene_seeds"], cfg["scene_sizes"]):
        st = grtx.SceneTensors.from_scene(inputs.cluster_scene(seed, n, 3), "cuda")
        tensors.append(st)
        bvhs.append(grtx.build(st, alpha_min=amin))
    torch.cuda.synchronize()
    srv = grtx.Server(memory_budget=96 << 30, slots=2, k=cfg["k"], T_min=cfg["T_min"])
    ids = [srv.add_scene(b) for b in bvhs]
    # warm the server's streams with one request per scene (pools, code objects)
    warm = [srv.submit(i, inputs.orbit_camera(64, 64)) for i in ids]
    while any(srv.poll(t) is None for t in warm):
        time.sleep(0.001)
    for t in warm:
        srv.release(t)

    def measure(rate):
        rng = np.random.default_rng(cfg["arrival_seed"])
        gaps = rng.exponential(1.0 / rate, n_requests)
        plan = []
        for j in range(n_requests):
            w, h = cfg["resolutions"][int(rng.integers(len(cfg["resolutions"])))]
            cam = inputs.Camera(inputs.random_orbit_eye(rng), (0.0, 0.0, 0.0), (0.0, 0.0, 1.0), 60.0, w, h)
            plan.append((float(gaps[:j + 1].sum()), ids[int(rng.integers(len(ids)))], cam))
        tickets = []

        def submitter():
            t0 = time.perf_counter()
            for at, sid, cam in plan:
                dt = at - (time.perf_counter() - t0)
                if dt > 0:
                    time.sleep(dt)
                tickets.append(srv.submit(sid, cam))

        th = threading.Thread(target=submitter)
        th.start()
        done = 0
        lat, wait, service, pixels = [], [], [], 0
        t_first, t_last = None, None
        while done < n_requests:
            for j, t in enumerate(list(tickets)):
                if t > 0:
                    r = srv.poll(t)
                    if r is not None:
                        lat.append(r["t_done"] - r["t_submit"])
                        wait.append(r["t_admit"] - r["t_submit"])
                        service.append(r["t_done"] - r["t_admit"])
                        pixels += r["width"] * r["height"]
                        t_first = r["t_submit"] if t_first is None else min(t_first, r["t_submit"])
                        t_last = r["t_done"] if t_last is None else max(t_last, r["t_done"])
                        srv.release(t)
                        tickets[j] = -1
                        done += 1
            time.sleep(0.0005)
        th.join()
        lat, wait, service = (np.array(x) * 1e3 for x in (lat, wait, service))
        offered = sum(c.width * c.height for _, _, c in plan) / plan[-1][0] / 1e6
        return dict(workload=cfg["name"] if rate == cfg["rate"] else f"serve-4scenes-poisson{rate:g}",
                    rate=rate, requests=n_requests, p50_ms=float(np.percentile(lat, 50)),
                    p99_ms=float(np.percentile(lat, 99)), mean_ms=float(lat.mean()), max_ms=float(lat.max()),
                    queue_wait_p50_ms=float(np.percentile(wait, 50)),
                    service_p50_ms=float(np.percentile(service, 50)),
                    service_p99_ms=float(np.percentile(service, 99)),
                    mrays_s=pixels / (t_last - t_first) / 1e6, rays=pixels, offered_mrays_s=offered,
                    scenes=list(cfg["scene_sizes"]),
                    note="latency = submission to completion of each timed request; "
                         "service = admission to completion")

    out = [measure(r) for r in rates]
    srv.close()
    return out


def time_launch(fn, stream, reps):
    """Mean duration (ms) of what `fn` enqueues on `stream`, from HIP events on that stream."""
    import torch
    fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        fn()
        e1.record(stream)
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    return sum(ts) / len(ts)


def run_proxy(st, cam, cfg, k, stream):
    """The same frame traced over the 20-face proxy BVH (one BVH leaf per triangle) and over
    instances of one shared icosahedron (one leaf per Gaussian)."""
    import numpy as np
    import torch

    from paper_2601_20429_amd import grtx
    amin = float(np.float32(cfg["alpha_min"]))
    o, d = grtx.pinhole_rays(cam)
    t0 = time.perf_counter()
    pb = grtx.build(st, alpha_min=amin, kind=grtx.PROXY20)
    torch.cuda.synchronize()
    build_ms = (time.perf_counter() - t0) * 1e3
    res = {}
    for m, name in [(grtx.CHECKPOINT, "checkpoint"), (grtx.RESTART, "restart")]:
        out = grtx.trace(pb, o, d, k=k, T_min=cfg["T_min"], mode=m, image_width=cam.width)
        ms = time_launch(lambda: grtx.trace(pb, o, d, k=k, T_min=cfg["T_min"], mode=m, image_width=cam.width,
                                            out=out), stream, 3)
        s = grtx.trace(pb, o, d, k=k, T_min=cfg["T_min"], mode=m, image_width=cam.width, stats=True)
        stt = s["stats"].to(torch.int64).sum(0).cpu().numpy()
        res[f"proxy_{name}_trace_ms"] = ms
        res[f"proxy_{name}_mrays_s"] = cam.n_rays / (ms * 1e-3) / 1e6
        res[f"proxy_{name}_nodes_per_ray"] = float(stt[0] + stt[1]) / cam.n_rays
    info = pb.info()
    res["proxy_build_ms"] = build_ms
    res["proxy_bvh_bytes"] = int(info["device_bytes"])
    del pb
    # instances of one shared icosahedron: the proxy's keys with the sphere's BVH size
    ib = grtx.build(st, alpha_min=amin, kind=grtx.ICO_INSTANCE)
    for m, name in [(grtx.CHECKPOINT, "checkpoint"), (grtx.RESTART, "restart")]:
        out = grtx.trace(ib, o, d, k=k, T_min=cfg["T_min"], mode=m, image_width=cam.width)
        ms = time_launch(lambda: grtx.trace(ib, o, d, k=k, T_min=cfg["T_min"], mode=m, image_width=cam.width,
                                            out=out), stream, 3)
        s = grtx.trace(ib, o, d, k=k, T_min=cfg["T_min"], mode=m, image_width=cam.width, stats=True)
        stt = s["stats"].to(torch.int64).sum(0).cpu().numpy()
        res[f"ico_{name}_trace_ms"] = ms
        res[f"ico_{name}_mrays_s"] = cam.n_rays / (ms * 1e-3) / 1e6
        res[f"ico_{name}_nodes_per_ray"] = float(stt[0] + stt[1]) / cam.n_rays
    res["ico_bvh_bytes"] = int(ib.info()["device_bytes"])
    return res


def run_secondary(bvh, cam, k, stream):
    """Secondary rays: the 100k scene with a glass sphere and a mirror. The primary rays
    end at the objects (t_far); the reflected and refracted rays continue from there with
    the transmittance left. Each ray type is traced in checkpoint and restart mode (the
    checkpoint speedup per ray type), and the whole chain (object rays, bounded trace,
    gathering, continuation trace, composite) is timed end to end."""
    import torch

    from paper_2601_20429_amd import grtx, inputs
    cfg = inputs.SECONDARY
    T_min = cfg["T_min"]
    objs = inputs.secondary_objects(cfg["objects_seed"])
    o, d = grtx.pinhole_rays(cam)
    ob = grtx.object_rays(objs, o, d)
    res = dict(workload=cfg["name"], primary_rays=cam.n_rays)
    res["object_rays_ms"] = time_launch(lambda: grtx.object_rays(objs, o, d), stream, 5)

    def trace_both(label, oo, dd, **kw):
        out = None
        for m, name in [(grtx.CHECKPOINT, "checkpoint"), (grtx.RESTART, "restart")]:
            out = grtx.trace(bvh, oo, dd, k=k, T_min=T_min, mode=m, **kw)
            ms = time_launch(lambda: grtx.trace(bvh, oo, dd, k=k, T_min=T_min, mode=m, out=out, **kw), stream, 5)
            stt = grtx.trace(bvh, oo, dd, k=k, T_min=T_min, mode=m, stats=True, **kw)["stats"]
            stt = stt.to(torch.int64).sum(0).cpu().numpy()
            n = int(oo.shape[0])
            res[f"{label}_{name}_ms"] = ms
            res[f"{label}_{name}_mrays_s"] = n / (ms * 1e-3) / 1e6
            res[f"{label}_{name}_nodes_per_ray"] = float(stt[0] + stt[1]) / n
        res[f"{label}_checkpoint_speedup"] = res[f"{label}_restart_ms"] / res[f"{label}_checkpoint_ms"]
        return out

    prim = trace_both("primary", o, d, image_width=cam.width, t_far=ob["t_far"])
    cont = grtx.continue_rays(ob["kind"], prim["opacity"], ob["next_o"], ob["next_d"], T_min)
    res["secondary_rays"] = int(cont["index"].shape[0])
    res["gather_ms"] = time_launch(lambda: grtx.continue_rays(ob["kind"], prim["opacity"], ob["next_o"],
                                                              ob["next_d"], T_min), stream, 5)
    sec = trace_both("secondary", cont["origins"], cont["dirs"], transmittance=cont["transmittance"])
    base = {key: v.clone() for key, v in prim.items()}

    def composite():
        for key in base:
            prim[key].copy_(base[key])
        grtx.continue_composite(cont, ob["path"], sec, prim)

    res["composite_ms_with_reset"] = time_launch(composite, stream, 5)
    for m, name in [(grtx.CHECKPOINT, "checkpoint"), (grtx.RESTART, "restart")]:
        ms = time_launch(lambda: grtx.trace_with_objects(bvh, o, d, objs, k=k, T_min=T_min, mode=m,
                                                         image_width=cam.width), stream, 3)
        res[f"chain_{name}_ms"] = ms
        res[f"chain_{name}_mrays_s"] = (cam.n_rays + res["secondary_rays"]) / (ms * 1e-3) / 1e6
    for m, name in [(grtx.CHECKPOINT, "checkpoint"), (grtx.RESTART, "restart")]:
        fo = grtx.trace_with_objects(bvh, o, d, objs, k=k, T_min=T_min, mode=m, image_width=cam.width, fused=True)
        ms = time_launch(lambda: grtx.trace(bvh, o, d, k=k, T_min=T_min, mode=m, image_width=cam.width,
                                            t_far=ob["t_far"], continuation=ob, out=fo), stream, 5)
        res[f"fused_{name}_trace_ms"] = ms
        res[f"fused_{name}_mrays_s"] = (cam.n_rays + res["secondary_rays"]) / (ms * 1e-3) / 1e6
    res["note"] = ("chain_ms includes the host wait for the number of continuation rays; fused_trace_ms is the one "
                   "trace launch that continues the rays itself (object rays excluded, "
                   f"{res['object_rays_ms']:.3f} ms)")
    return res


def run_two_streams(st, cam, cfg, k, steps, warmup=2):
    """The same step (raygen + build + trace of one frame) issued on two streams in turn, so
    that consecutive frames overlap: the next frame's build and first rays fill the GPU
    while the last rays of the previous frame finish. Reported beside the sequential step
    as whole-job throughput of the same work."""
    import numpy as np
    import torch

    from paper_2601_20429_amd import grtx
    amin = float(np.float32(cfg["alpha_min"]))
    dev = torch.device("cuda:0")
    streams = [torch.cuda.Stream(device=dev), torch.cuda.Stream(device=dev)]
    R = cam.n_rays
    outs = [dict(rgb=torch.empty((R, 3), dtype=torch.float32, device=dev),
                 depth=torch.empty(R, dtype=torch.float32, device=dev),
                 opacity=torch.empty(R, dtype=torch.float32, device=dev)) for _ in streams]

    def step(i):
        s = streams[i % 2]
        with torch.cuda.stream(s):
            oo, dd = grtx.pinhole_rays(cam, device=dev, stream=s)
            bvh = grtx.build(st, alpha_min=amin, stream=s)
            grtx.trace(bvh, oo, dd, k=k, T_min=cfg["T_min"], image_width=cam.width, out=outs[i % 2], stream=s)
        return bvh, oo, dd

    keep = [step(i) for i in range(warmup)]
    torch.cuda.synchronize()
    keep.clear()
    t0 = time.perf_counter()
    keep = [step(i) for i in range(steps)]
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    keep.clear()
    return dict(two_stream_step_ms=ms, two_stream_mrays_s=R / (ms * 1e-3) / 1e6)


def run_ksweep(bvh, o, d, cam, cfg, stream, ks=(4, 8, 16, 32, 64)):
    """k-buffer size sweep on the same frame, checkpoint and restart: trace time and
    per-ray fetches and rounds (the cost of re-traversal against the cost of larger
    buffers)."""
    import torch

    from paper_2601_20429_amd import grtx
    res = {}
    for k in ks:
        for m, name in [(grtx.CHECKPOINT, "checkpoint"), (grtx.RESTART, "restart")]:
            out = grtx.trace(bvh, o, d, k=k, T_min=cfg["T_min"], mode=m, image_width=cam.width)
            ms = time_launch(lambda: grtx.trace(bvh, o, d, k=k, T_min=cfg["T_min"], mode=m, image_width=cam.width,
                                                out=out), stream, 3)
            stt = grtx.trace(bvh, o, d, k=k, T_min=cfg["T_min"], mode=m, image_width=cam.width, stats=True)["stats"]
            stt = stt.to(torch.int64).sum(0).cpu().numpy()
            R = cam.n_rays
            res[f"k{k}_{name}"] = dict(ms=round(ms, 3), mrays_s=round(R / (ms * 1e-3) / 1e6, 2),
                                       nodes_per_ray=round(float(stt[0] + stt[1]) / R, 1),
                                       rounds_per_ray=round(float(stt[2]) / R, 3))
    return res


def run_scene3m(stream, ks=(16, 32)):
    """Largest workload: 3M Gaussians, 1920x1080 primary rays (8x8 tiles) plus 2M
    incoherent rays, k = 16 and 32, checkpointing. Rates count both ray sets."""
    import numpy as np
    import torch

    from paper_2601_20429_amd import grtx, inputs
    cfg = inputs.SCENE3M
    amin = float(np.float32(cfg["alpha_min"]))
    st = grtx.SceneTensors.from_scene(inputs.cluster_scene(cfg["seed"], cfg["n"], 3), "cuda")
    cam = inputs.orbit_camera(cfg["width"], cfg["height"])
    po, pd = grtx.pinhole_rays(cam)
    io, id_ = (torch.from_numpy(a).cuda() for a in inputs.incoherent_rays(cfg["incoherent_seed"], cfg["incoherent"]))
    bvh = grtx.build(st, alpha_min=amin)
    build_ms = time_launch(lambda: grtx.build(st, alpha_min=amin), stream, 3)
    res = dict(workload=cfg["name"], build_ms=build_ms, rays=cam.n_rays + cfg["incoherent"])
    for k in ks:
        for label, o, d, w in [("primary", po, pd, cam.width), ("incoherent", io, id_, 0)]:
            out = grtx.trace(bvh, o, d, k=k, T_min=cfg["T_min"], image_width=w)
            ms = time_launch(lambda: grtx.trace(bvh, o, d, k=k, T_min=cfg["T_min"], image_width=w, out=out),
                             stream, 3)
            stt = grtx.trace(bvh, o, d, k=k, T_min=cfg["T_min"], image_width=w, stats=True)["stats"]
            stt = stt.to(torch.int64).sum(0).cpu().numpy()
            n = int(o.shape[0])
            res[f"k{k}_{label}_ms"] = ms
            res[f"k{k}_{label}_mrays_s"] = n / (ms * 1e-3) / 1e6
            res[f"k{k}_{label}_nodes_per_ray"] = float(stt[0] + stt[1]) / n
            del out
        res[f"k{k}_mrays_s"] = res["rays"] / ((res[f"k{k}_primary_ms"] + res[f"k{k}_incoherent_ms"]) * 1e-3) / 1e6
    return res


def run_backward(stream):
    """Differentiation workload: 200k Gaussians, 512x512 rays, k = 16; the forward pass keeps
    each ray's blended ids, the backward kernel replays them."""
    import numpy as np
    import torch

    from paper_2601_20429_amd import grtx, inputs
    cfg = inputs.DIFF200K
    st = grtx.SceneTensors.from_scene(inputs.cluster_scene(cfg["seed"], cfg["n"], 3), "cuda")
    cam = inputs.orbit_camera(cfg["width"], cfg["height"])
    o, d = grtx.pinhole_rays(cam)
    bvh = grtx.build(st, alpha_min=float(np.float32(cfg["alpha_min"])))
    fwd = grtx.trace(bvh, o, d, k=cfg["k"], T_min=cfg["T_min"], hit_capacity=256)
    g_rgb = torch.ones_like(fwd["rgb"])
    f_ms = time_launch(lambda: grtx.trace(bvh, o, d, k=cfg["k"], T_min=cfg["T_min"], hit_capacity=256, out=fwd),
                       stream, 3)
    b_ms = time_launch(lambda: grtx.trace_backward(bvh, o, d, fwd, grad_rgb=g_rgb, k=cfg["k"], T_min=cfg["T_min"]),
                       stream, 3)
    R = cam.n_rays
    return dict(workload=cfg["name"], forward_with_ids_ms=f_ms, backward_ms=b_ms,
                backward_mrays_s=R / (b_ms * 1e-3) / 1e6,
                note="backward_ms includes zeroing the gradient arrays")


def kernel_k(k):
    return 4 if k <= 4 else 8 if k <= 8 else 16 if k <= 16 else 32 if k <= 32 else 64


TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "k_trace_k16_scene100k_hbm_traffic.txt")
TRACE_SOURCES = [os.path.join(ROOT, "paper_2601_20429_amd", "csrc", f) for f in ("trace.hip", "grtx_internal.h")]


def source_digest():
    import hashlib
    h = hashlib.sha256()
    for f in TRACE_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(args):
    """HBM bytes per launch of the timed kernel from the committed counter summary
    (FETCH_SIZE + WRITE_SIZE, scaled by the copy-kernel calibration), or None when that
    summary was taken on other kernel sources or another launch configuration."""
    if args.k != 16 or args.mode != "checkpoint" or not os.path.exists(TRAFFIC_PROFILE):
        return None
    fields = {}
    with open(TRAFFIC_PROFILE) as fh:
        for line in fh:
            if ":" in line and not line.startswith(" "):
                key, _, val = line.partition(":")
                fields[key.strip()] = val.strip()
    if fields.get("source_sha256") != source_digest():
        return None
    try:
        return float(fields["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--k", type=int, default=16)
    ap.add_argument("--mode", choices=["checkpoint", "restart"], default="checkpoint")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-compare", action="store_true", help="skip the restart-mode comparison run")
    ap.add_argument("--cpu-rays", type=int, default=196608)
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--calibrate-copy-gib", type=float, default=0.0,
                    help="first copy this many GiB device-to-device (a reference kernel for HBM counters)")
    ap.add_argument("--serve-requests", type=int, default=200)
    ap.add_argument("--serve-low-rate", type=float, default=30.0,
                    help="second serving run at this arrival rate (requests/s), below the server's capacity")
    ap.add_argument("--no-proxy", action="store_true", help="skip the 20-face proxy BVH comparison")
    ap.add_argument("--no-backward", action="store_true", help="skip the backward-pass timing")
    ap.add_argument("--no-scene3m", action="store_true", help="skip the 3M-Gaussian workload")
    ap.add_argument("--no-ksweep", action="store_true", help="skip the k-buffer size sweep")
    ap.add_argument("--no-secondary", action="store_true", help="skip the secondary-ray workload")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); sharding the rays over "
              "several GPUs is not built", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2601_20429_amd import grtx, inputs

    cfg = inputs.SCENE100K
    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    amin = float(np.float32(cfg["alpha_min"]))
    scene = inputs.cluster_scene(cfg["seed"], cfg["n"], 3)
    st = grtx.SceneTensors.from_scene(scene, dev)
    cam = inputs.orbit_camera(cfg["width"], cfg["height"])
    R = cam.n_rays
    mode = grtx.CHECKPOINT if args.mode == "checkpoint" else grtx.RESTART
    stream = torch.cuda.current_stream()
    o = torch.empty((R, 3), dtype=torch.float32, device=dev)
    d = torch.empty((R, 3), dtype=torch.float32, device=dev)
    out = dict(rgb=torch.empty((R, 3), dtype=torch.float32, device=dev),
               depth=torch.empty(R, dtype=torch.float32, device=dev),
               opacity=torch.empty(R, dtype=torch.float32, device=dev))
    trace_ev = []

    def step(m, record=False):
        oo, dd = grtx.pinhole_rays(cam, device=dev)
        bvh = grtx.build(st, alpha_min=amin)
        if record:
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
        grtx.trace(bvh, oo, dd, k=args.k, T_min=cfg["T_min"], mode=m, image_width=cam.width, out=out)
        if record:
            e1.record(stream)
            trace_ev.append((e0, e1))
        return bvh

    def timed(m, steps, warmup):
        keep = []
        for _ in range(warmup):
            keep.append(step(m))
        torch.cuda.synchronize()
        keep.clear()
        trace_ev.clear()
        t0 = time.perf_counter()
        for _ in range(steps):
            keep.append(step(m, record=True))
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        ktimes = [a.elapsed_time(b) for a, b in trace_ev]
        keep.clear()
        return (t1 - t0) * 1e3 / steps, float(np.mean(ktimes)), float(np.median(ktimes))

    if args.calibrate_copy_gib > 0:
        nb = int(args.calibrate_copy_gib * (1 << 30)) // 4
        src = torch.ones(nb, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"calibration copy: {nb * 4} bytes read and written")
        del src, dst
    log(f"scene {cfg['n']} Gaussians, {cam.width}x{cam.height} rays, k={args.k}, mode={args.mode}")
    ms, k_mean, k_med = timed(mode, args.steps, args.warmup)
    mrays = R / (ms * 1e-3) / 1e6
    log(f"step {ms:.3f} ms ({mrays:.1f} Mrays/s); trace kernel mean {k_mean:.3f} ms median {k_med:.3f} ms")

    # counters of the same launch configuration (deterministic, so an untimed run with the
    # per-ray counters enabled sees exactly the timed work)
    bvh = grtx.build(st, alpha_min=amin)
    oo, dd = grtx.pinhole_rays(cam, device=dev)
    sout = grtx.trace(bvh, oo, dd, k=args.k, T_min=cfg["T_min"], mode=mode, image_width=cam.width, stats=True)
    torch.cuda.synchronize()
    stt = sout["stats"].to(torch.int64).sum(0).cpu().numpy()
    nodes, leaves, rounds, blended, deferred, free, evicted, fallbacks = [int(x) for x in stt[:8]]
    alg_bytes = (B_NODE * nodes + B_LEAF * leaves + (B_BLEND_INST + 4 * 3 * (scene.sh_degree + 1) ** 2) * blended
                 + B_LIST * (deferred + evicted) + B_RAY * R)
    achieved = alg_bytes / (k_mean * 1e-3) / 1e9
    extra = dict(nodes_per_ray=(nodes + leaves) / R, internal_nodes_per_ray=nodes / R, leaf_tests_per_ray=leaves / R,
                 rounds_per_ray=rounds / R, blended_per_ray=blended / R, deferred_per_ray=deferred / R,
                 fetch_free_per_ray=free / R, evicted_per_ray=evicted / R, fallbacks=fallbacks,
                 trace_kernel_ms=k_mean, trace_kernel_ms_median=k_med,
                 trace_only_mrays_s=R / (k_mean * 1e-3) / 1e6, algorithmic_bytes_per_ray=alg_bytes / R)
    log("counters", json.dumps(extra))

    if not args.no_compare:
        other = grtx.RESTART if mode == grtx.CHECKPOINT else grtx.CHECKPOINT
        ms2, k2, _ = timed(other, max(3, args.steps // 2), 1)
        sout2 = grtx.trace(bvh, oo, dd, k=args.k, T_min=cfg["T_min"], mode=other, image_width=cam.width,
                           stats=True)
        torch.cuda.synchronize()
        s2 = sout2["stats"].to(torch.int64).sum(0).cpu().numpy()
        name = "restart" if other == grtx.RESTART else "checkpoint"
        extra[f"{name}_step_ms"] = ms2
        extra[f"{name}_mrays_s"] = R / (ms2 * 1e-3) / 1e6
        extra[f"{name}_trace_kernel_ms"] = k2
        extra[f"{name}_nodes_per_ray"] = float(s2[0] + s2[1]) / R
        log(f"{name}: step {ms2:.3f} ms, trace {k2:.3f} ms, nodes/ray {extra[f'{name}_nodes_per_ray']:.1f}")

    info = bvh.info()
    extra["bvh_bytes"] = int(info["device_bytes"])
    if not args.no_compare:
        extra.update(run_two_streams(st, cam, cfg, args.k, args.steps))
        log(f"two streams: step {extra['two_stream_step_ms']:.3f} ms ({extra['two_stream_mrays_s']:.1f} Mrays/s)")
    if not args.no_proxy:
        extra.update(run_proxy(st, cam, cfg, args.k, stream))
        log("proxy", json.dumps({k: v for k, v in extra.items() if k.startswith(("proxy", "ico"))}))
    if not args.no_secondary:
        extra["secondary"] = run_secondary(bvh, cam, args.k, stream)
        log("secondary", json.dumps(extra["secondary"]))
    backward = None
    if not args.no_backward:
        backward = run_backward(stream)
        log("backward", json.dumps(backward))

    if not args.no_ksweep:
        extra["ksweep"] = run_ksweep(bvh, oo, dd, cam, cfg, stream)
        log("ksweep", json.dumps(extra["ksweep"]))

    scene3m = None
    if not args.no_scene3m:
        scene3m = run_scene3m(stream)
        log("scene3m", json.dumps(scene3m))

    serving = None
    if not args.no_serving:
        serving, below = run_serving(args.serve_requests, (inputs.SERVE["rate"], args.serve_low_rate))
        log("serving", json.dumps(serving))
        log("serving below capacity", json.dumps(below))
        extra["serving_below_capacity"] = below

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        cores = min(16, os.cpu_count() or 1)
        ro, rd = oracle.pinhole_rays(cam)
        idx = inputs.ray_subsample(99, R, args.cpu_rays)
        ro, rd = ro[idx].astype(np.float32), rd[idx].astype(np.float32)
        t0 = time.perf_counter()
        oracle.render(scene, ro, rd, amin, cfg["T_min"], nthreads=cores)
        dt = time.perf_counter() - t0
        cpu_model = ""
        try:
            with open("/proc/cpuinfo") as f:
                cpu_model = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), "")
        except OSError:
            pass
        cpu = dict(value=len(idx) / dt / 1e6, unit="Mrays/s", cores=cores, kind="oracle",
                   sample=f"{len(idx)} of the {R} primary rays (seeded subsample) against all {cfg['n']} "
                          f"Gaussians, FP64 brute force, {dt:.1f} s",
                   host_cpu=cpu_model, host_threads_visible=os.cpu_count())
        log("cpu baseline", json.dumps(cpu))

    rec = {
        "metric": "Mrays/s and nodes visited/ray at k=16; p50/p99 frame latency (serving)",
        "value": mrays,
        "unit": "Mrays/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": cfg["name"], "gaussians": cfg["n"], "width": cam.width, "height": cam.height,
                   "rays": R, "k": args.k, "mode": args.mode, "sh_degree": 3, "bvh": "sphere-instance LBVH",
                   "step": "raygen + LBVH build + trace"},
        "nodes_per_ray": extra["nodes_per_ray"],
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(args),
                     "kernel": f"k_trace<{kernel_k(args.k)}>"},
        "cpu_baseline": cpu,
        "serving": serving,
        "backward": backward,
        "scene3m": scene3m,
        "extra": extra,
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
