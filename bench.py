"""Benchmark: Gaussian ray tracing of the 3M-Gaussian workload on one GPU.

One step is the whole hot path over one batch of the workload (3M Gaussians, SH degree 3,
1920x1080 primary rays plus 2M incoherent rays, k = 16, checkpointed tracing): pinhole
ray generation, the LBVH build over the Gaussians (setup, Morton codes, radix sort, radix
tree, refit, treelet restructuring, four-wide records) and the multi-round trace with
blending of both ray sets. Inputs (scene parameters, incoherent rays) are resident on the
GPU before timing starts. The value is rays per second over the step (both ray sets).
Beside it: the same step in restart-from-root mode and at k = 32, the 100k-Gaussian
frame (restart, proxy BVH, k sweep, secondary rays), the backward pass and serving.
Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline] [--headline-only]
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
B_LEAF = 48          # unit-sphere transform of a leaf (3 x float4); a proxy triangle is 48 B too
B_BLEND_INST = 64    # full instance record re-read for blending
B_LIST = 16          # one checkpoint / eviction entry written and read back (8 B each way)
B_RAY = 24 + 20      # ray in (origin, direction); rgb, depth, opacity out
STAT_NAMES = ("nodes", "leaves", "rounds", "blended", "deferred", "fetch_free", "evicted", "fallbacks",
              "stack_drops")


def alg_bytes(c, sh_degree, rays):
    """Algorithmic bytes of a trace from its summed per-ray counters `c` (dict)."""
    return (B_NODE * c["nodes"] + B_LEAF * c["leaves"]
            + (B_BLEND_INST + 4 * 3 * (sh_degree + 1) ** 2) * c["blended"]
            + B_LIST * (c["deferred"] + c["evicted"]) + B_RAY * rays)


def stat_sums(out):
    import torch
    v = out["stats"].to(torch.int64).sum(0).cpu().numpy()
    return {name: int(x) for name, x in zip(STAT_NAMES, v)}


def per_ray(c, rays):
    return dict(nodes_per_ray=(c["nodes"] + c["leaves"]) / rays, internal_nodes_per_ray=c["nodes"] / rays,
                leaf_tests_per_ray=c["leaves"] / rays, rounds_per_ray=c["rounds"] / rays,
                blended_per_ray=c["blended"] / rays, deferred_per_ray=c["deferred"] / rays,
                fetch_free_per_ray=c["fetch_free"] / rays, evicted_per_ray=c["evicted"] / rays,
                fallbacks=c["fallbacks"], stack_drops=c["stack_drops"])


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def run_serving(n_requests, rates, sweep=(0.5, 0.7, 0.85, 1.0)):
    """Serving workload: four device-resident scenes (100k, 500k, 1M, 3M Gaussians), Poisson
    arrivals, each a random camera on the radius-3 sphere at a resolution drawn from
    {256^2, 512^2, 800^2, 1920x1080}, k = 16; latency is submission to result. One server
    (one persistent kernel fed from its queue). Runs of `n_requests` each: all submitted at
    once (sustained capacity: pixels over the span from the first submission to the last
    result), then at each arrival rate of `rates` (requests/s), then at the fractions
    `sweep` of the measured capacity in requests/s; a run's latency is bounded when the
    queue does not grow over it (mean latency of the last third of the requests at most
    1.5x that of the first third plus 20 ms)."""
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
    srv = grtx.Server(memory_budget=96 << 30, k=cfg["k"], T_min=cfg["T_min"])
    ids = [srv.add_scene(b) for b in bvhs]
    # warm the server (code objects, arena, tile orders of every resolution)
    warm = [srv.submit(i, inputs.orbit_camera(w, h)) for i in ids for w, h in cfg["resolutions"]]
    while any(srv.poll(t) is None for t in warm):
        time.sleep(0.001)
    for t in warm:
        srv.release(t)

    def measure(rate, label):
        rng = np.random.default_rng(cfg["arrival_seed"])
        gaps = rng.exponential(1.0 / rate, n_requests) if rate > 0 else np.zeros(n_requests)
        plan = []
        for j in range(n_requests):
            w, h = cfg["resolutions"][int(rng.integers(len(cfg["resolutions"])))]
            cam = inputs.Camera(inputs.random_orbit_eye(rng), (0.0, 0.0, 0.0), (0.0, 0.0, 1.0), 60.0, w, h)
            plan.append((float(gaps[:j + 1].sum()), ids[int(rng.integers(len(ids)))], cam))
        tickets = []
        launches0 = srv.stats()["launches"]

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
        lat = [None] * n_requests
        wait, pixels = [], 0
        t_first, t_last = None, None
        while done < n_requests:
            for j, t in enumerate(list(tickets)):
                if t > 0:
                    r = srv.poll(t)
                    if r is not None:
                        lat[j] = r["t_done"] - r["t_submit"]
                        wait.append(r["t_admit"] - r["t_submit"])
                        pixels += r["width"] * r["height"]
                        t_first = r["t_submit"] if t_first is None else min(t_first, r["t_submit"])
                        t_last = r["t_done"] if t_last is None else max(t_last, r["t_done"])
                        srv.release(t)
                        tickets[j] = -1
                        done += 1
            time.sleep(0.0005)
        th.join()
        lat = np.array(lat) * 1e3
        wait = np.array(wait) * 1e3
        third = n_requests // 3
        early, late = float(lat[:third].mean()), float(lat[-third:].mean())
        span = t_last - t_first
        offered = sum(c.width * c.height for _, _, c in plan) / plan[-1][0] / 1e6 if rate > 0 else None
        return dict(workload=label, rate=rate if rate > 0 else None, requests=n_requests,
                    p50_ms=float(np.percentile(lat, 50)), p99_ms=float(np.percentile(lat, 99)),
                    mean_ms=float(lat.mean()), max_ms=float(lat.max()),
                    queue_wait_p50_ms=float(np.percentile(wait, 50)),
                    early_mean_ms=early, late_mean_ms=late, bounded=bool(late <= 1.5 * early + 20.0),
                    mrays_s=pixels / span / 1e6, requests_s=n_requests / span, rays=pixels,
                    offered_mrays_s=offered, launches=srv.stats()["launches"] - launches0)

    cap = measure(0.0, "serve-4scenes-saturated")
    log("serving capacity", json.dumps(cap))
    runs = []
    for r in rates:
        runs.append(measure(r, cfg["name"] if r == cfg["rate"] else f"serve-4scenes-poisson{r:g}"))
        log("serving", json.dumps(runs[-1]))
    swept = []
    for f in sweep:
        rate = round(f * cap["requests_s"], 1)
        swept.append(measure(rate, f"serve-4scenes-poisson{rate:g}"))
        log("serving sweep", json.dumps(swept[-1]))
    ok = [m["rate"] for m in swept + runs if m["bounded"]]
    summary = dict(capacity_mrays_s=cap["mrays_s"], capacity_requests_s=cap["requests_s"],
                   max_bounded_rate=max(ok) if ok else None, scenes=list(cfg["scene_sizes"]),
                   note="latency = submission to result; one persistent kernel fed from a work queue; "
                        "bounded = no latency growth over the run")
    srv.close()
    return summary, cap, runs, swept


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
        c = stat_sums(grtx.trace(pb, o, d, k=k, T_min=cfg["T_min"], mode=m, image_width=cam.width, stats=True))
        res[f"proxy_{name}_trace_ms"] = ms
        res[f"proxy_{name}_mrays_s"] = cam.n_rays / (ms * 1e-3) / 1e6
        res[f"proxy_{name}_nodes_per_ray"] = float(c["nodes"] + c["leaves"]) / cam.n_rays
        res[f"proxy_{name}_algorithmic_GBs"] = alg_bytes(c, st.sh_degree, cam.n_rays) / (ms * 1e-3) / 1e9
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
        c = stat_sums(grtx.trace(ib, o, d, k=k, T_min=cfg["T_min"], mode=m, image_width=cam.width, stats=True))
        res[f"ico_{name}_trace_ms"] = ms
        res[f"ico_{name}_mrays_s"] = cam.n_rays / (ms * 1e-3) / 1e6
        res[f"ico_{name}_nodes_per_ray"] = float(c["nodes"] + c["leaves"]) / cam.n_rays
        res[f"ico_{name}_algorithmic_GBs"] = alg_bytes(c, st.sh_degree, cam.n_rays) / (ms * 1e-3) / 1e9
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


def run_single_round(bvh, sets, T_min, stream, caps=(512, 1024, 2048)):
    """Single-round tracing (collect every hit of a ray, then sort and blend) for each list
    capacity: time, nodes per ray and the rays whose hits overflowed the list (incomplete
    results). `sets` = [(label, origins, dirs, image_width)]."""
    from paper_2601_20429_amd import grtx
    res = {}
    for cap in caps:
        for label, o, d, w in sets:
            kw = dict(k=16, T_min=T_min, mode=grtx.SINGLE_ROUND, collect_capacity=cap, image_width=w)
            out = grtx.trace(bvh, o, d, **kw)
            ms = time_launch(lambda: grtx.trace(bvh, o, d, out=out, **kw), stream, 2)
            c = stat_sums(grtx.trace(bvh, o, d, stats=True, **kw))
            n = int(o.shape[0])
            res[f"cap{cap}_{label}"] = dict(ms=round(ms, 3), mrays_s=round(n / (ms * 1e-3) / 1e6, 2),
                                            nodes_per_ray=round((c["nodes"] + c["leaves"]) / n, 1),
                                            incomplete_rays=c["fallbacks"])
            del out
    return res


def run_backward(stream):
    """Differentiation workload: 200k Gaussians, 512x512 rays, k = 16; the forward pass keeps
    each ray's blended ids, the backward pass replays them (and, timed separately, traces
    the rays again itself when given no list)."""
    import numpy as np
    import torch

    from paper_2601_20429_amd import grtx, inputs
    cfg = inputs.DIFF200K
    st = grtx.SceneTensors.from_scene(inputs.cluster_scene(cfg["seed"], cfg["n"], 3), "cuda")
    cam = inputs.orbit_camera(cfg["width"], cfg["height"])
    o, d = grtx.pinhole_rays(cam)
    bvh = grtx.build(st, alpha_min=float(np.float32(cfg["alpha_min"])))
    cap = 256
    W = cam.width  # the rays form an image: 8x8 tile scheduling
    fwd = grtx.trace(bvh, o, d, k=cfg["k"], T_min=cfg["T_min"], hit_capacity=cap, image_width=W)
    g_rgb = torch.ones_like(fwd["rgb"])
    grads = dict(means=torch.zeros_like(st.means), scales=torch.zeros_like(st.scales),
                 quats=torch.zeros_like(st.quats), opacities=torch.zeros_like(st.opacities),
                 sh=torch.zeros_like(st.sh))
    f_ms = time_launch(lambda: grtx.trace(bvh, o, d, k=cfg["k"], T_min=cfg["T_min"], hit_capacity=cap, out=fwd,
                                          image_width=W), stream, 3)
    b_ms = time_launch(lambda: grtx.trace_backward(bvh, o, d, fwd, grad_rgb=g_rgb, grads=grads, k=cfg["k"],
                                                   T_min=cfg["T_min"]), stream, 5)
    r_ms = time_launch(lambda: grtx.trace_backward(bvh, o, d, None, grad_rgb=g_rgb, grads=grads, k=cfg["k"],
                                                   T_min=cfg["T_min"], hit_capacity=cap, image_width=W), stream, 3)
    R = cam.n_rays
    counts = fwd["hit_counts"].clamp(max=cap)
    P = int(counts.sum())
    ids = fwd["hit_ids"][fwd["hit_ids"] >= 0]
    touched = int(torch.unique(ids).numel())
    ncoef = 3 * (st.sh_degree + 1) ** 2
    params = 4 * (3 + 3 + 4 + 1 + ncoef)  # one Gaussian's parameters (or gradients)
    passes = (max(1, int(np.ceil(np.log2(st.n + 1)))) + 7) // 8
    per_record = params + 4 + (64 + 12) + passes * 2 * 12 + (64 + 4 + 12)
    alg = P * per_record + R * (24 + 20 + 12) + touched * 2 * params
    return dict(workload=cfg["name"], forward_with_ids_ms=f_ms, backward_ms=b_ms,
                backward_mrays_s=R / (b_ms * 1e-3) / 1e6, backward_retrace_ms=r_ms,
                hit_records=P, records_per_ray=P / R, touched_gaussians=touched,
                algorithmic_bytes=alg, algorithmic_GBs=alg / (b_ms * 1e-3) / 1e9,
                algorithmic_frac=alg / (b_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                note=("bytes per hit record: the Gaussian's parameters re-read, its id, the 64-B record and "
                      "its 12-B sort key written, the sort passes, the record, order and ray direction read "
                      "back; per ray: ray, forward outputs, output gradient; per touched Gaussian: its "
                      "gradient read and written. backward_retrace_ms traces the rays again inside the call"))


def kernel_k(k):
    return 4 if k <= 4 else 8 if k <= 8 else 16 if k <= 16 else 32 if k <= 32 else 64


TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "k_trace_k16_scene3m_hbm_traffic.txt")
# what the traced launch's traffic depends on: the trace kernel, its list sizes and device
# helpers, and the build of the tree it walks
TRACE_SOURCES = [os.path.join(ROOT, "paper_2601_20429_amd", "csrc", f) for f in ("trace.hip", "trace_common.h", "build.hip")]


def source_digest():
    import hashlib
    h = hashlib.sha256()
    for f in TRACE_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def profile_fields(path):
    """`key: value` lines of a committed counter summary."""
    fields = {}
    if not os.path.exists(path):
        return fields
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith(" "):
                key, _, val = line.partition(":")
                fields[key.strip()] = val.strip()
    return fields


def measured_traffic(args):
    """HBM bytes per launch of the timed trace kernel from the committed counter summary
    (FETCH_SIZE + WRITE_SIZE of the step's one launch, scaled by the copy-kernel
    calibration), or None when that summary was taken on other kernel sources or another
    launch configuration."""
    if args.k != 16 or args.mode != "checkpoint":
        return None
    fields = profile_fields(TRAFFIC_PROFILE)
    if fields.get("source_sha256") != source_digest():
        return None
    try:
        return float(fields["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


class Workload3M:
    """The 3M-Gaussian workload, resident on the GPU: scene parameters, one ray buffer that
    holds the 2M incoherent rays followed by the 1920x1080 frame's rays (written by the
    step's ray generation), and one output buffer."""

    def __init__(self, dev):
        import numpy as np
        import torch

        from paper_2601_20429_amd import grtx, inputs
        self.cfg = cfg = inputs.SCENE3M
        self.amin = float(np.float32(cfg["alpha_min"]))
        self.scene = inputs.cluster_scene(cfg["seed"], cfg["n"], 3)
        self.st = grtx.SceneTensors.from_scene(self.scene, dev)
        self.cam = inputs.orbit_camera(cfg["width"], cfg["height"])
        io, id_ = inputs.incoherent_rays(cfg["incoherent_seed"], cfg["incoherent"])
        self.n_prim, self.n_inc = self.cam.n_rays, cfg["incoherent"]
        self.rays = self.n_prim + self.n_inc
        self.o = torch.empty((self.rays, 3), dtype=torch.float32, device=dev)
        self.d = torch.empty((self.rays, 3), dtype=torch.float32, device=dev)
        self.o[:self.n_inc] = torch.from_numpy(io)
        self.d[:self.n_inc] = torch.from_numpy(id_)
        self.io, self.id = self.o[:self.n_inc], self.d[:self.n_inc]
        self.po, self.pd = self.o[self.n_inc:], self.d[self.n_inc:]
        self.dev = dev
        self.out = self.outputs(self.rays)

    def outputs(self, R):
        import torch
        return dict(rgb=torch.empty((R, 3), dtype=torch.float32, device=self.dev),
                    depth=torch.empty(R, dtype=torch.float32, device=self.dev),
                    opacity=torch.empty(R, dtype=torch.float32, device=self.dev))

    def trace_kw(self, k, mode):
        return dict(k=k, T_min=self.cfg["T_min"], mode=mode, image_width=self.cam.width, image_begin=self.n_inc)

    def step(self, k, mode, events=None):
        """One step: raygen + build + one trace launch over both ray sets (the incoherent
        rays first, then the frame's 8x8 tiles); with `events` (a list), HIP events on the
        launch stream bracket the trace call."""
        import torch

        from paper_2601_20429_amd import grtx
        stream = torch.cuda.current_stream()
        grtx.pinhole_rays(self.cam, out=(self.po, self.pd))
        bvh = grtx.build(self.st, alpha_min=self.amin)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)] if events is not None else None
        if ev:
            ev[0].record(stream)
        grtx.trace(bvh, self.o, self.d, out=self.out, **self.trace_kw(k, mode))
        if ev:
            ev[1].record(stream)
            events.append(ev)
        return bvh

    def timed(self, k, mode, steps, warmup):
        """Step time (ms, host clock over `steps` synchronised steps) and the mean duration
        (ms, HIP events) of the step's trace launch."""
        import numpy as np
        import torch
        keep = [self.step(k, mode) for _ in range(warmup)]
        torch.cuda.synchronize()
        keep.clear()
        ev = []
        t0 = time.perf_counter()
        for _ in range(steps):
            keep.append(self.step(k, mode, ev))
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        trace = float(np.mean([a.elapsed_time(b) for a, b in ev]))
        keep.clear()
        return ms, trace

    def alone(self, k, mode, reps=3):
        """Launch time (ms, HIP events) of each ray set traced on its own (a diagnostic:
        the step traces both in one launch)."""
        import torch

        from paper_2601_20429_amd import grtx
        stream = torch.cuda.current_stream()
        grtx.pinhole_rays(self.cam, out=(self.po, self.pd))
        bvh = grtx.build(self.st, alpha_min=self.amin)
        op, oi = self.outputs(self.n_prim), self.outputs(self.n_inc)
        kw = dict(k=k, T_min=self.cfg["T_min"], mode=mode)
        for _ in range(2):
            grtx.trace(bvh, self.po, self.pd, image_width=self.cam.width, out=op, **kw)
            grtx.trace(bvh, self.io, self.id, out=oi, **kw)
        tp = time_launch(lambda: grtx.trace(bvh, self.po, self.pd, image_width=self.cam.width, out=op, **kw),
                         stream, reps)
        ti = time_launch(lambda: grtx.trace(bvh, self.io, self.id, out=oi, **kw), stream, reps)
        return tp, ti

    def other_seeds(self, k, seeds=(34, 35, 36), reps=2):
        """The step's launch, checkpointed, with other seeds of the same incoherent-ray
        distribution in place of the step's (whether the checkpoint lists hold the heaviest
        rays of other draws too): launch time (HIP events), rays that fell back to a
        restart round, and the costliest ray's node and leaf visits."""
        import torch

        from paper_2601_20429_amd import grtx, inputs
        stream = torch.cuda.current_stream()
        grtx.pinhole_rays(self.cam, out=(self.po, self.pd))
        bvh = grtx.build(self.st, alpha_min=self.amin)
        o, d = torch.empty_like(self.o), torch.empty_like(self.d)
        o[self.n_inc:], d[self.n_inc:] = self.po, self.pd
        out = self.outputs(self.rays)
        kw = self.trace_kw(k, grtx.CHECKPOINT)
        res = {}
        for sd in seeds:
            io, id_ = inputs.incoherent_rays(sd, self.n_inc)
            o[:self.n_inc] = torch.from_numpy(io).to(self.dev)
            d[:self.n_inc] = torch.from_numpy(id_).to(self.dev)
            ms = time_launch(lambda: grtx.trace(bvh, o, d, out=out, **kw), stream, reps)
            st = grtx.trace(bvh, o, d, stats=True, **kw)["stats"].to(torch.int64)
            vis = st[:, grtx.STAT_NODES] + st[:, grtx.STAT_LEAVES]
            res[f"incoherent_seed_{sd}"] = dict(trace_ms=ms, fallbacks=int(st[:, grtx.STAT_FALLBACKS].sum()),
                                                max_visits_per_ray=int(vis.max()))
            del st, vis
        return res

    def two_streams(self, k, steps, warmup=2):
        """The step issued on the launch stream and a second stream in turn, each with its
        own ray and output buffers, so that a frame's ray generation and build overlap the
        previous frame's trace: whole-job throughput of the same work, reported beside the
        sequential step."""
        import torch

        from paper_2601_20429_amd import grtx
        streams = [torch.cuda.current_stream(), torch.cuda.Stream(device=self.o.device)]
        o2, d2 = torch.empty_like(self.o), torch.empty_like(self.d)
        o2[:self.n_inc], d2[:self.n_inc] = self.io, self.id
        bufs = [(self.o, self.d, self.out), (o2, d2, self.outputs(self.rays))]
        torch.cuda.synchronize()

        def step(i):
            s = streams[i % 2]
            o, d, out = bufs[i % 2]
            with torch.cuda.stream(s):
                grtx.pinhole_rays(self.cam, out=(o[self.n_inc:], d[self.n_inc:]), stream=s)
                bvh = grtx.build(self.st, alpha_min=self.amin, stream=s)
                grtx.trace(bvh, o, d, out=out, stream=s, **self.trace_kw(k, grtx.CHECKPOINT))
            return bvh

        keep = [step(i) for i in range(warmup)]
        torch.cuda.synchronize()
        keep.clear()
        t0 = time.perf_counter()
        keep = [step(i) for i in range(steps)]
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        keep.clear()
        return dict(step_ms=ms, mrays_s=self.rays / (ms * 1e-3) / 1e6)

    def counters(self, k, mode):
        """Summed per-ray counters of each ray set in the step's launch, from an untimed run
        with the counters on: the timed launch's work, except for the few rays whose
        checkpoint lists fill and are compacted at a point that follows the scheduling."""
        import torch

        from paper_2601_20429_amd import grtx
        grtx.pinhole_rays(self.cam, out=(self.po, self.pd))
        bvh = grtx.build(self.st, alpha_min=self.amin)
        st = grtx.trace(bvh, self.o, self.d, stats=True, **self.trace_kw(k, mode))["stats"]
        cp = stat_sums({"stats": st[self.n_inc:]})
        ci = stat_sums({"stats": st[:self.n_inc]})
        torch.cuda.synchronize()
        info = bvh.info()
        return cp, ci, info

    def summary(self, k, mode, steps, warmup, alone=True):
        ms, tt = self.timed(k, mode, steps, warmup)
        tp, ti = self.alone(k, mode) if alone else (None, None)
        cp, ci, info = self.counters(k, mode)
        bp = alg_bytes(cp, 3, self.n_prim)
        bi = alg_bytes(ci, 3, self.n_inc)
        return dict(k=k, mode="checkpoint" if mode == 0 else "restart", step_ms=ms,
                    mrays_s=self.rays / (ms * 1e-3) / 1e6,
                    trace_ms=tt, trace_mrays_s=self.rays / (tt * 1e-3) / 1e6,
                    primary_alone_ms=tp, incoherent_alone_ms=ti,
                    primary_alone_mrays_s=self.n_prim / (tp * 1e-3) / 1e6 if tp else None,
                    incoherent_alone_mrays_s=self.n_inc / (ti * 1e-3) / 1e6 if ti else None,
                    primary=per_ray(cp, self.n_prim), incoherent=per_ray(ci, self.n_inc),
                    nodes_per_ray=(cp["nodes"] + cp["leaves"] + ci["nodes"] + ci["leaves"]) / self.rays,
                    algorithmic_bytes_primary=bp, algorithmic_bytes_incoherent=bi,
                    trace_algorithmic_GBs=(bp + bi) / (tt * 1e-3) / 1e9,
                    tree_depth=info["depth"], bvh_bytes=info["device_bytes"])


def run_frame100k(args, stream):
    """The 100k-Gaussian 800x800 frame (k = 16): step (raygen + build + trace), the
    trace's counters, restart mode, two streams in turn, the proxy BVHs, the k sweep and
    the secondary-ray workload."""
    import numpy as np
    import torch

    from paper_2601_20429_amd import grtx, inputs
    cfg = inputs.SCENE100K
    dev = torch.device("cuda:0")
    amin = float(np.float32(cfg["alpha_min"]))
    st = grtx.SceneTensors.from_scene(inputs.cluster_scene(cfg["seed"], cfg["n"], 3), dev)
    cam = inputs.orbit_camera(cfg["width"], cfg["height"])
    R = cam.n_rays
    out = dict(rgb=torch.empty((R, 3), dtype=torch.float32, device=dev),
               depth=torch.empty(R, dtype=torch.float32, device=dev),
               opacity=torch.empty(R, dtype=torch.float32, device=dev))
    res = dict(workload=cfg["name"])

    def timed(m, steps, warmup):
        ev = []

        def step(record):
            oo, dd = grtx.pinhole_rays(cam, device=dev)
            bvh = grtx.build(st, alpha_min=amin)
            if record:
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
            grtx.trace(bvh, oo, dd, k=args.k, T_min=cfg["T_min"], mode=m, image_width=cam.width, out=out)
            if record:
                e1.record(stream)
                ev.append((e0, e1))
            return bvh
        keep = [step(False) for _ in range(warmup)]
        torch.cuda.synchronize()
        keep.clear()
        t0 = time.perf_counter()
        keep = [step(True) for _ in range(steps)]
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        return ms, float(np.mean([a.elapsed_time(b) for a, b in ev]))

    bvh = grtx.build(st, alpha_min=amin)
    oo, dd = grtx.pinhole_rays(cam, device=dev)
    for m, name in [(grtx.CHECKPOINT, "checkpoint"), (grtx.RESTART, "restart")]:
        ms, kms = timed(m, args.steps, 2)
        c = stat_sums(grtx.trace(bvh, oo, dd, k=args.k, T_min=cfg["T_min"], mode=m, image_width=cam.width,
                                 stats=True))
        res[name] = dict(step_ms=ms, mrays_s=R / (ms * 1e-3) / 1e6, trace_ms=kms,
                         trace_mrays_s=R / (kms * 1e-3) / 1e6,
                         trace_algorithmic_GBs=alg_bytes(c, 3, R) / (kms * 1e-3) / 1e9,
                         algorithmic_bytes_per_ray=alg_bytes(c, 3, R) / R, **per_ray(c, R))
        log(f"100k {name}: step {ms:.3f} ms, trace {kms:.3f} ms, nodes/ray {res[name]['nodes_per_ray']:.1f}")
    res["checkpoint_speedup_trace"] = res["restart"]["trace_ms"] / res["checkpoint"]["trace_ms"]
    res["bvh_bytes"] = int(bvh.info()["device_bytes"])
    if not args.no_compare:
        res.update(run_two_streams(st, cam, cfg, args.k, args.steps))
    if not args.no_proxy:
        res.update(run_proxy(st, cam, cfg, args.k, stream))
        log("proxy", json.dumps({k: v for k, v in res.items() if k.startswith(("proxy", "ico"))}))
    if not args.no_secondary:
        res["secondary"] = run_secondary(bvh, cam, args.k, stream)
        log("secondary", json.dumps(res["secondary"]))
    if not args.no_ksweep:
        res["ksweep"] = run_ksweep(bvh, oo, dd, cam, cfg, stream)
        log("ksweep", json.dumps(res["ksweep"]))
        res["single_round"] = run_single_round(bvh, [("primary", oo, dd, cam.width)], cfg["T_min"], stream)
        log("single round", json.dumps(res["single_round"]))
    return res


def cpu_baseline(work, sample_rays):
    """The oracle (FP64 brute force over every ray/Gaussian pair) on a seeded sample of the
    step's rays, on the host threads this process may use; beside it the oracle's CPU model
    of the method on the same rays, in checkpoint and restart mode (its rate, node visits
    against distinct nodes visited, and the checkpoint a ray carries between rounds)."""
    import numpy as np

    import oracle
    from paper_2601_20429_amd import inputs
    threads = int(os.environ.get("OMP_NUM_THREADS") or 0) or len(os.sched_getaffinity(0))
    po, pd = oracle.pinhole_rays(work.cam)
    io, id_ = inputs.incoherent_rays(work.cfg["incoherent_seed"], work.cfg["incoherent"])
    idx = inputs.ray_subsample(99, work.rays, sample_rays)
    ip, ii = idx[idx < work.n_prim], idx[idx >= work.n_prim] - work.n_prim
    ro = np.concatenate([po[ip].astype(np.float32), io[ii]])
    rd = np.concatenate([pd[ip].astype(np.float32), id_[ii]])
    t0 = time.perf_counter()
    oracle.render(work.scene, ro, rd, work.amin, work.cfg["T_min"], nthreads=threads)
    dt = time.perf_counter() - t0
    cpu_model = ""
    try:
        with open("/proc/cpuinfo") as f:
            cpu_model = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), "")
    except OSError:
        pass
    # the oracle's CPU model of the method (FP64 binary-BVH traversal in rounds of k, with
    # checkpoints) on the same rays; its BVH build is timed apart with a one-ray call
    t0 = time.perf_counter()
    oracle.model_render(work.scene, ro[:1], rd[:1], 16, oracle.CHECKPOINT, oracle.RULE_KBUF_MAX, work.amin,
                        work.cfg["T_min"], nthreads=threads, distinct=False)
    t_build = time.perf_counter() - t0
    t0 = time.perf_counter()
    oracle.model_render(work.scene, ro, rd, 16, oracle.CHECKPOINT, oracle.RULE_KBUF_MAX, work.amin,
                        work.cfg["T_min"], nthreads=threads, distinct=False)
    t_model = time.perf_counter() - t0
    # (untimed: the same rays with distinct visits counted, in both modes)
    mc, mr = (oracle.model_render(work.scene, ro, rd, 16, m, oracle.RULE_KBUF_MAX, work.amin, work.cfg["T_min"],
                                  nthreads=threads) for m in (oracle.CHECKPOINT, oracle.RESTART))

    def visits(m):
        # per ray on the binary tree: visits of nodes and leaves, distinct ones, and the
        # largest checkpoint carried between rounds (8 B per deferred node or evicted hit)
        c = m["counts"].astype(np.float64)
        v, u = c[:, 0] + c[:, 1], c[:, 4]
        return dict(visits_per_ray=float(v.mean()), distinct_per_ray=float(u.mean()),
                    visits_per_distinct=float(v.sum() / max(u.sum(), 1.0)), rounds_per_ray=float(m["rounds"].mean()),
                    checkpoint_bytes_per_ray_mean=float(8 * c[:, 5].mean()),
                    checkpoint_bytes_per_ray_max=float(8 * c[:, 5].max()))
    model = dict(value=len(idx) / max(t_model - t_build, 1e-9) / 1e6, unit="Mrays/s", cores=threads,
                 kind="cpu model of the method (FP64, binary radix-tree BVH, k = 16, checkpoints)",
                 build_s=t_build, sample="the same rays",
                 checkpoint=visits(mc), restart=visits(mr))
    return dict(value=len(idx) / dt / 1e6, unit="Mrays/s", cores=threads, kind="oracle",
                sample=f"{len(idx)} of the step's {work.rays} rays ({len(ip)} primary, {len(ii)} incoherent; "
                       f"seeded subsample) against all {work.cfg['n']} Gaussians, FP64 brute force, {dt:.1f} s",
                host_cpu=cpu_model, host_threads_visible=os.cpu_count(), cpu_model_of_method=model,
                whole_frames=cpu_whole_frames(threads))


def cpu_whole_frames(threads):
    """The oracle and its CPU model of the method over whole frames of the two smaller
    workloads: the plain 1k-Gaussian 64x64 frame at k = 4 (both), and the 100k-Gaussian
    800x800 frame at k = 16 (the model; the brute force would take hours)."""
    import numpy as np

    import oracle
    from paper_2601_20429_amd import inputs
    out = {}
    for cfg, brute in ((inputs.PLAIN, True), (inputs.SCENE100K, False)):
        scene = inputs.make_workload_scene(cfg)
        o, d = oracle.pinhole_rays(inputs.orbit_camera(cfg["width"], cfg["height"]))
        o, d = o.astype(np.float32), d.astype(np.float32)
        amin = float(np.float32(cfg["alpha_min"]))
        res = dict(rays=int(o.shape[0]), k=cfg["k"], cores=threads)
        if brute:
            t0 = time.perf_counter()
            oracle.render(scene, o, d, amin, cfg["T_min"], nthreads=threads)
            res["oracle_mrays_s"] = o.shape[0] / (time.perf_counter() - t0) / 1e6
        t0 = time.perf_counter()
        oracle.model_render(scene, o, d, cfg["k"], oracle.CHECKPOINT, oracle.RULE_KBUF_MAX, amin, cfg["T_min"],
                            nthreads=threads, distinct=False)
        res["cpu_model_mrays_s"] = o.shape[0] / (time.perf_counter() - t0) / 1e6
        res["note"] = "the CPU model's rate includes its BVH build"
        out[cfg["name"]] = res
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--k", type=int, default=16)
    ap.add_argument("--mode", choices=["checkpoint", "restart"], default="checkpoint")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-compare", action="store_true", help="skip the restart-mode and k = 32 runs of the step")
    ap.add_argument("--cpu-rays", type=int, default=8192)
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--calibrate-copy-gib", type=float, default=0.0,
                    help="first copy this many GiB device-to-device (a reference kernel for HBM counters)")
    ap.add_argument("--serve-requests", type=int, default=200)
    ap.add_argument("--serve-low-rate", type=float, default=30.0,
                    help="second serving run at this arrival rate (requests/s), below the server's capacity")
    ap.add_argument("--no-frame100k", action="store_true", help="skip the 100k-Gaussian frame measurements")
    ap.add_argument("--no-proxy", action="store_true", help="skip the 20-face proxy BVH comparison")
    ap.add_argument("--no-backward", action="store_true", help="skip the backward-pass timing")
    ap.add_argument("--no-ksweep", action="store_true", help="skip the k-buffer size sweep")
    ap.add_argument("--no-secondary", action="store_true", help="skip the secondary-ray workload")
    ap.add_argument("--headline-only", action="store_true",
                    help="only the timed step and its counters (for profiler runs)")
    ap.add_argument("--backward-only", action="store_true",
                    help="only the backward-pass timing, printed as its JSON object (for profiler runs)")
    ap.add_argument("--serving-only", action="store_true",
                    help="only the serving runs, printed as one JSON object (for profiler runs)")
    ap.add_argument("--frame100k-only", action="store_true",
                    help="only the 100k-Gaussian frame in checkpoint and restart mode, printed as its JSON "
                         "object (for profiler runs)")
    ap.add_argument("--with-secondary", action="store_true",
                    help="with --frame100k-only: also the secondary-ray workload")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); sharding the rays over "
              "several GPUs is not built", file=sys.stderr)
        sys.exit(2)
    if args.headline_only:
        args.no_cpu_baseline = args.no_compare = args.no_serving = args.no_frame100k = True
        args.no_backward = True

    import torch

    from paper_2601_20429_amd import grtx, inputs

    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    mode = grtx.CHECKPOINT if args.mode == "checkpoint" else grtx.RESTART
    if args.calibrate_copy_gib > 0:
        nb = int(args.calibrate_copy_gib * (1 << 30)) // 4
        src = torch.ones(nb, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"calibration copy: {nb * 4} bytes read and written")
        del src, dst

    if args.backward_only:
        print(json.dumps(run_backward(stream)), flush=True)
        return
    if args.frame100k_only:
        args.no_compare = args.no_proxy = args.no_ksweep = True
        args.no_secondary = not args.with_secondary
        print(json.dumps(run_frame100k(args, stream)), flush=True)
        return
    if args.serving_only:
        summary, cap, runs, swept = run_serving(args.serve_requests, (inputs.SERVE["rate"], args.serve_low_rate))
        print(json.dumps(dict(summary=summary, saturated=cap, runs=runs, sweep=swept)), flush=True)
        return

    work = Workload3M(dev)
    log(f"workload {work.cfg['name']}: {work.cfg['n']} Gaussians, {work.n_prim} + {work.n_inc} rays, k={args.k}, "
        f"mode={args.mode}")
    # (profiler runs see only the step's launches: no separate launches of each ray set)
    head = work.summary(args.k, mode, args.steps, args.warmup, alone=not args.headline_only)
    log("headline", json.dumps(head))
    extra = dict(headline=head)
    # the dominant kernel: the trace, one launch per step over both ray sets
    launch_ms = head["trace_ms"]
    launch_bytes = head["algorithmic_bytes_primary"] + head["algorithmic_bytes_incoherent"]
    achieved = launch_bytes / (launch_ms * 1e-3) / 1e9
    traffic = measured_traffic(args)
    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                "kernel": f"k_trace<{kernel_k(args.k)}, 0, false>",
                "per_launch": "the step's one launch: 2M incoherent rays, then the 1920x1080 frame's 8x8 tiles",
                "algorithmic_bytes_per_launch": launch_bytes, "launch_ms": launch_ms,
                "hbm_measured_GBs": None if traffic is None else traffic / (launch_ms * 1e-3) / 1e9,
                "hbm_measured_frac": None if traffic is None else traffic / (launch_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                "limiter": profile_fields(TRAFFIC_PROFILE).get("limiter")}

    if not args.no_compare:
        other = grtx.RESTART if mode == grtx.CHECKPOINT else grtx.CHECKPOINT
        extra["restart" if other == grtx.RESTART else "checkpoint"] = cmp = work.summary(
            args.k, other, max(3, args.steps // 2), 1)
        log("compare", json.dumps(cmp))
        extra["k32"] = k32 = work.summary(32, mode, max(3, args.steps // 2), 1)
        log("k32", json.dumps(k32))
        bvh3 = grtx.build(work.st, alpha_min=work.amin)
        grtx.pinhole_rays(work.cam, out=(work.po, work.pd))
        extra["single_round"] = run_single_round(
            bvh3, [("primary", work.po, work.pd, work.cam.width), ("incoherent", work.io, work.id, 0)],
            work.cfg["T_min"], stream, caps=(2048,))
        log("single round", json.dumps(extra["single_round"]))
        del bvh3
        if mode == grtx.CHECKPOINT:
            extra["checkpoint_speedup_step"] = cmp["step_ms"] / head["step_ms"]
            extra["checkpoint_speedup_trace"] = cmp["trace_ms"] / head["trace_ms"]
        extra["other_incoherent_seeds"] = work.other_seeds(args.k)
        log("other seeds", json.dumps(extra["other_incoherent_seeds"]))
        if mode == grtx.CHECKPOINT:
            extra["two_streams"] = work.two_streams(args.k, max(4, args.steps))
            log("two streams", json.dumps(extra["two_streams"]))

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(work, args.cpu_rays)
        log("cpu baseline", json.dumps(cpu))
    del work
    torch.cuda.empty_cache()

    if not args.no_frame100k:
        extra["scene100k"] = run_frame100k(args, stream)
    backward = None
    if not args.no_backward:
        backward = run_backward(stream)
        log("backward", json.dumps(backward))
    serving = None
    if not args.no_serving:
        summary, cap, runs, swept = run_serving(args.serve_requests, (inputs.SERVE["rate"], args.serve_low_rate))
        serving = dict(runs[0], **summary)
        extra["serving_saturated"] = cap
        extra["serving_below_capacity"] = runs[1:]
        extra["serving_sweep"] = swept
        log("serving summary", json.dumps(summary))
    extra["paper_reference"] = (
        "paper (Vulkan-Sim, 8 SMs at 1365 MHz; 6 scenes of 0.76-2.43 M Gaussians at 128x128, k = 8): "
        "GRTX 4.36x over the 20-triangle baseline on average, checkpointing alone 1.94x, 2.37x fewer node "
        "fetches from checkpointing; no absolute rays/s is given")

    rec = {
        "metric": "Mrays/s and nodes visited/ray at k=16; p50/p99 frame latency (serving)",
        "value": head["mrays_s"],
        "unit": "Mrays/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["step_ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": inputs.SCENE3M["name"], "gaussians": 3_000_000, "primary_rays": 1920 * 1080,
                   "incoherent_rays": 2_000_000, "k": args.k, "mode": args.mode, "sh_degree": 3,
                   "bvh": "sphere-instance LBVH", "step": "raygen + LBVH build + one trace launch over both ray sets"},
        "nodes_per_ray": head["nodes_per_ray"],
        "roofline": roofline,
        "cpu_baseline": cpu,
        "serving": serving,
        "backward": backward,
        "extra": extra,
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
