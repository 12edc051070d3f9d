"""GPU path vs the FP64 oracle, through the C ABI. Needs an MI355X and the built library."""
import math
import sys

import numpy as np
import pytest

import oracle
from paper_2601_20429_amd import inputs
from tests import parity
from tests.helpers import dc_colour, load_golden, make_scene, walkthrough_scene

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_2601_20429_amd import grtx  # noqa: E402

AMIN = float(np.float32(1.0 / 255.0))  # the library's binary32 alpha_min, as a real number
T_MIN = 1e-3


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    oracle.lib()
    yield
    torch.cuda.synchronize()


def dev(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def build(scene, kind=grtx.SPHERE_INSTANCE, plain_lbvh=False):
    st = grtx.SceneTensors.from_scene(scene, "cuda")
    return grtx.build(st, kind=kind, alpha_min=AMIN, plain_lbvh=plain_lbvh)


def render(bvh, o, d, k=16, mode=grtx.CHECKPOINT, cap=256, **kw):
    out = grtx.trace(bvh, dev(o), dev(d), k=k, T_min=T_MIN, mode=mode, hit_capacity=cap, stats=True, **kw)
    torch.cuda.synchronize()
    return {key: v.cpu().numpy() for key, v in out.items()}


def oracle_rays(cam):
    o, d = oracle.pinhole_rays(cam)
    return o.astype(np.float32), d.astype(np.float32)


# ------------------------------------------------------------------------ build

@pytest.mark.parametrize("case", ["n1", "n2", "n3", "n100", "plain1k", "dups257", "scene100k", "scene1100k",
                                  "scene3m"])
def test_topology_bit_exact(case):
    """Morton codes, the stable sort's permutation and the plain radix tree (child and
    parent arrays, and its depth) bit for bit against the oracle. Above 1,048,576 keys
    (1.1M, and the 3M-Gaussian workload) the radix sort takes its scan-kernel path."""
    say("topology", case)
    if case == "plain1k":
        scene = inputs.small_scene(1, 1000)
    elif case == "scene100k":
        scene = inputs.cluster_scene(2, 100_000, 0)
    elif case == "scene1100k":
        scene = inputs.cluster_scene(6, 1_100_000, 0)
    elif case == "scene3m":
        scene = inputs.cluster_scene(inputs.SCENE3M["seed"], inputs.SCENE3M["n"], 0)
    else:
        n = int(case[1:] if case[0] == "n" else case[4:])
        rng = np.random.default_rng(n)
        means = rng.uniform(-1, 1, (n, 3))
        if case.startswith("dups"):
            means[::3] = means[0]
        scene = make_scene(means, [0.05] * 3, quats=rng.standard_normal((n, 4)), opac=0.5)
    bvh = build(scene, plain_lbvh=True)
    t = bvh.export_topology()
    torch.cuda.synchronize()
    ref = oracle.lbvh_topology(scene.means)
    n = scene.n
    assert (t["morton"].cpu().numpy().view(np.uint64) == ref["codes"]).all()
    assert (t["perm"].cpu().numpy().view(np.uint32) == ref["perm"]).all()
    if n > 1:
        assert (t["child"].cpu().numpy().view(np.uint32) == ref["child"]).all()
    assert (t["parent"].cpu().numpy().view(np.uint32) == ref["parent"]).all()
    info = bvh.info()
    assert info["leaves"] == n and info["internal_nodes"] == max(n - 1, 0)
    assert info["restructured"] == 0 and info["depth"] == tree_depth(ref["child"], n)


def tree_depth(child, n):
    """Internal nodes on the longest root-to-leaf path of a tree given by its child array
    (bit 31 = leaf), by a breadth-first walk from the root (node 0)."""
    if n < 2:
        return 0
    child = np.asarray(child, np.uint32).reshape(-1, 2)
    level, depth = np.array([0], np.int64), 0
    while level.size:
        depth += 1
        c = child[level].ravel()
        level = (c[(c & 0x80000000) == 0]).astype(np.int64)
    return depth


def _check_tree(t, n):
    """A valid binary tree over n leaves: every node but the root is the child of exactly
    one internal node, parents agree, and every internal box is the exact union of its
    children's boxes. Returns the surface-area cost (internal 1.2 x area, leaf 1.0 x area)
    relative to the root's area."""
    child = t["child"].cpu().numpy().view(np.uint32).astype(np.int64)
    parent = t["parent"].cpu().numpy().view(np.uint32).astype(np.int64)
    boxes = t["boxes"].cpu().numpy().astype(np.float64)
    nint = n - 1
    uid = np.where(child & 0x80000000, nint + (child & 0x7FFFFFFF), child)
    seen = np.bincount(uid.ravel(), minlength=nint + n)
    assert seen[0] == 0 and (seen[1:] == 1).all()
    for k in range(2):
        assert (parent[uid[:, k]] == np.arange(nint)).all()
    assert parent[0] == 0xFFFFFFFF
    lo = np.minimum(boxes[uid[:, 0], :3], boxes[uid[:, 1], :3])
    hi = np.maximum(boxes[uid[:, 0], 3:], boxes[uid[:, 1], 3:])
    assert (boxes[:nint, :3] == lo).all() and (boxes[:nint, 3:] == hi).all()
    e = np.maximum(boxes[:, 3:] - boxes[:, :3], 0)
    area = e[:, 0] * e[:, 1] + e[:, 1] * e[:, 2] + e[:, 2] * e[:, 0]
    return (1.2 * area[:nint].sum() + area[nint:].sum()) / area[0]


@pytest.mark.parametrize("case", ["n2", "n3", "n5", "n100", "dups257", "plain1k", "scene100k", "proxy2k",
                                  "scene1100k"])
def test_restructured_tree_valid_and_cheaper(case):
    """Treelet restructuring keeps a valid tree over the same sorted leaves (Morton codes
    and permutation unchanged), with exact boxes, and never raises the surface-area cost."""
    say("restructured tree", case)
    kind = grtx.SPHERE_INSTANCE
    if case == "plain1k":
        scene = inputs.small_scene(1, 1000)
    elif case == "scene100k":
        scene = inputs.cluster_scene(2, 100_000, 0)
    elif case == "proxy2k":
        scene, kind = inputs.cluster_scene(2, 2000, 0), grtx.PROXY20
    elif case == "scene1100k":  # above a million leaves: the pass over the top of the tree runs too
        scene = inputs.cluster_scene(6, 1_100_000, 0)
    else:
        n = int(case[1:] if case[0] == "n" else case[4:])
        rng = np.random.default_rng(n)
        means = rng.uniform(-1, 1, (n, 3))
        if case.startswith("dups"):
            means[::3] = means[0]
        scene = make_scene(means, [0.05] * 3, quats=rng.standard_normal((n, 4)), opac=0.5)
    a = build(scene, kind, plain_lbvh=True)
    b = build(scene, kind)
    ta, tb = a.export_topology(), b.export_topology()
    torch.cuda.synchronize()
    n = a.info()["leaves"]
    assert torch.equal(ta["morton"], tb["morton"]) and torch.equal(ta["perm"], tb["perm"])
    assert torch.equal(ta["boxes"][n - 1:], tb["boxes"][n - 1:])  # leaf boxes
    ca, cb = _check_tree(ta, n), _check_tree(tb, n)
    assert cb <= ca * (1 + 1e-6), (ca, cb)
    say(dict(case=case, sah_plain=round(ca, 2), sah_restructured=round(cb, 2)))


@pytest.mark.parametrize("kind,n", [(grtx.SPHERE_INSTANCE, 100_000), (grtx.PROXY20, 20_000),
                                    (grtx.ICO_INSTANCE, 100_000), (grtx.SPHERE_INSTANCE, 1_100_000)])
def test_restructured_tree_renders_identically(kind, n):
    """Results do not depend on the tree: the plain radix tree and the restructured one
    give bit-identical outputs and hit lists, in both modes."""
    say("restructured renders", kind, n)
    scene = inputs.cluster_scene(2, n, 3)
    cam = inputs.orbit_camera(160, 120)
    o, d = grtx.pinhole_rays(cam)
    a = build(scene, kind, plain_lbvh=True)
    b = build(scene, kind)
    for mode in (grtx.CHECKPOINT, grtx.RESTART):
        ra = grtx.trace(a, o, d, k=8, T_min=T_MIN, mode=mode, image_width=cam.width, hit_capacity=128, stats=True)
        rb = grtx.trace(b, o, d, k=8, T_min=T_MIN, mode=mode, image_width=cam.width, hit_capacity=128, stats=True)
        torch.cuda.synchronize()
        for key in ("rgb", "depth", "opacity", "hit_ids", "hit_counts"):
            assert torch.equal(ra[key], rb[key]), (mode, key)
        fa = int(ra["stats"][:, grtx.STAT_NODES].sum())
        fb = int(rb["stats"][:, grtx.STAT_NODES].sum())
        say(dict(mode=mode, node_fetches_plain=fa, node_fetches_restructured=fb))


@pytest.mark.parametrize("case", ["scene100k", "proxy100k", "scene1100k", "scene3m"])
def test_tree_depth_within_stack_bound(case):
    """The build measures the depth of the tree it keeps; every kept tree fits the trace's
    traversal stack (3 entries per level), and traces over it lose no stack entry. The
    measured depth equals a breadth-first walk of the exported child array."""
    say("tree depth", case)
    kind, n, seed = grtx.SPHERE_INSTANCE, 100_000, 2
    if case == "proxy100k":
        kind = grtx.PROXY20
    elif case == "scene1100k":
        n, seed = 1_100_000, 6
    elif case == "scene3m":
        n, seed = inputs.SCENE3M["n"], inputs.SCENE3M["seed"]
    scene = inputs.cluster_scene(seed, n, 3)
    bvh = build(scene, kind)
    info = bvh.info()
    t = bvh.export_topology()
    torch.cuda.synchronize()
    m = info["leaves"]
    assert 0 < info["depth"] <= grtx.MAX_TREE_DEPTH
    assert info["restructured"] == 1
    assert info["depth"] == tree_depth(t["child"].cpu().numpy().view(np.uint32), m)
    cam = inputs.orbit_camera(256, 256)
    po, pd = grtx.pinhole_rays(cam)
    io, id_ = (dev(a) for a in inputs.incoherent_rays(33, 16384))
    drops = 0
    for o, d, w in [(po, pd, cam.width), (io, id_, 0)]:
        for mode in (grtx.CHECKPOINT, grtx.RESTART):
            st = grtx.trace(bvh, o, d, k=16, T_min=T_MIN, mode=mode, image_width=w, stats=True)["stats"]
            torch.cuda.synchronize()
            drops += int(st[:, grtx.STAT_STACK_DROPS].sum())
    say(dict(case=case, leaves=m, depth=info["depth"], stack_drops=drops))
    assert drops == 0


def test_too_deep_restructured_tree_falls_back_to_plain():
    """A restructured tree deeper than the build's max_depth is replaced on the device by
    the plain radix tree: the same topology and boxes as a plain build, identical images."""
    say("depth fallback")
    scene = inputs.cluster_scene(2, 100_000, 3)
    plain = build(scene, plain_lbvh=True)
    restr = build(scene)
    dp, dr = plain.info()["depth"], restr.info()["depth"]
    assert restr.info()["restructured"] == 1 and dr > 1
    st = grtx.SceneTensors.from_scene(scene, "cuda")
    fb = grtx.build(st, alpha_min=AMIN, max_depth=dr - 1)
    info = fb.info()
    say(dict(plain_depth=dp, restructured_depth=dr, fallback=info))
    assert info["restructured"] == 0 and info["depth"] == dp
    a, b = plain.export_topology(), fb.export_topology()
    for key in ("child", "parent", "morton", "perm", "boxes"):
        assert torch.equal(a[key], b[key]), key
    cam = inputs.orbit_camera(128, 96)
    o, d = grtx.pinhole_rays(cam)
    ra = grtx.trace(plain, o, d, k=16, T_min=T_MIN, image_width=cam.width, hit_capacity=128)
    rb = grtx.trace(fb, o, d, k=16, T_min=T_MIN, image_width=cam.width, hit_capacity=128)
    torch.cuda.synchronize()
    for key in ("rgb", "depth", "opacity", "hit_ids", "hit_counts"):
        assert torch.equal(ra[key], rb[key]), key


def test_boxes_conservative_and_tight():
    say("boxes")
    scene = inputs.cluster_scene(2, 20_000, 0)
    bvh = build(scene)
    t = bvh.export_topology()
    boxes = t["boxes"].cpu().numpy().astype(np.float64)
    child = t["child"].cpu().numpy().view(np.uint32)
    perm = t["perm"].cpu().numpy().view(np.uint32)
    n = scene.n
    lo, hi, act = oracle.gaussian_aabb(scene, AMIN)
    leaf = boxes[n - 1:]
    olo, ohi = lo[perm], hi[perm]
    assert (leaf[:, :3] <= olo).all() and (leaf[:, 3:] >= ohi).all()
    ext = np.maximum(ohi - olo, 1e-30)
    assert ((leaf[:, 3:] - leaf[:, :3]) <= ext * (1 + 2 ** -6) + 1e-6).all()
    # internal boxes are the exact union of their children
    for i in range(n - 1):
        cb = []
        for c in child[i]:
            idx = (n - 1 + (c & 0x7FFFFFFF)) if c & 0x80000000 else c
            cb.append(boxes[idx])
        cb = np.array(cb)
        assert (boxes[i, :3] == cb[:, :3].min(0)).all() and (boxes[i, 3:] == cb[:, 3:].max(0)).all()


def test_pinhole_rays_match_oracle():
    say("pinhole")
    cam = inputs.orbit_camera(97, 61, eye=(0.3, -3.0, 0.8), fov_y_deg=55.0)
    o, d = grtx.pinhole_rays(cam)
    torch.cuda.synchronize()
    ro, rd = oracle.pinhole_rays(cam)
    np.testing.assert_allclose(o.cpu().numpy(), ro, atol=1e-6)
    np.testing.assert_allclose(d.cpu().numpy(), rd, atol=2e-6)


# ------------------------------------------------------------------------ tracing parity

@pytest.mark.parametrize("mode", [grtx.CHECKPOINT, grtx.RESTART])
def test_plain_scene_parity(mode):
    """1k Gaussians, 64x64 pinhole camera at radius 3, k=4, alpha_min 1/255, T_min 1e-3."""
    say("plain parity mode", mode)
    scene = inputs.small_scene(1, 1000)
    o, d = oracle_rays(inputs.orbit_camera(64, 64))
    g = render(build(scene), o, d, k=4, mode=mode, cap=256)
    ref = oracle.render(scene, o, d, AMIN, T_MIN, cap=256)
    s = parity.compare_render(scene, o, d, g, ref, AMIN, T_MIN, label=f"plain mode={mode}")
    say(s)


@pytest.mark.parametrize("mode", [grtx.CHECKPOINT, grtx.RESTART])
def test_scene100k_parity_sampled(mode):
    """100k-Gaussian SH-degree-3 scene, sampled 800x800 primary rays, k=16."""
    say("scene100k parity mode", mode)
    scene = inputs.cluster_scene(2, 100_000, 3)
    o, d = oracle_rays(inputs.orbit_camera(800, 800))
    idx = inputs.ray_subsample(99, o.shape[0], 1536)
    o, d = o[idx], d[idx]
    g = render(build(scene), o, d, k=16, mode=mode, cap=512)
    ref = oracle.render(scene, o, d, AMIN, T_MIN, cap=512)
    s = parity.compare_render(scene, o, d, g, ref, AMIN, T_MIN, label=f"100k mode={mode}")
    say(s)


def test_incoherent_rays_parity():
    """Origins inside the scene box, directions uniform on the sphere."""
    say("incoherent")
    scene = inputs.cluster_scene(2, 100_000, 3)
    o, d = inputs.incoherent_rays(33, 1024)
    g = render(build(scene), o, d, k=16, cap=512)
    ref = oracle.render(scene, o, d, AMIN, T_MIN, cap=512)
    s = parity.compare_render(scene, o, d, g, ref, AMIN, T_MIN, label="incoherent")
    say(s)


def test_modes_and_k_bit_identical():
    """Checkpointing only removes redundant work: every k and both modes give the same
    bits, and repeated runs are deterministic."""
    say("modes/k identity")
    scene = inputs.cluster_scene(2, 100_000, 3)
    cam = inputs.orbit_camera(160, 120)
    o, d = grtx.pinhole_rays(cam)
    bvh = build(scene)
    base = None
    for k in [16, 1, 2, 4, 8, 32, 64]:
        for mode in [grtx.CHECKPOINT, grtx.RESTART]:
            out = grtx.trace(bvh, o, d, k=k, T_min=T_MIN, mode=mode, image_width=cam.width, hit_capacity=128)
            torch.cuda.synchronize()
            cur = {kk: v.cpu().numpy() for kk, v in out.items()}
            if base is None:
                base = cur
                continue
            for key in ["rgb", "depth", "opacity", "hit_counts", "hit_ids"]:
                assert np.array_equal(cur[key], base[key]), (k, mode, key)


@pytest.mark.parametrize("cap", [2048, 512])
def test_single_round_equals_checkpoint(cap):
    """Single-round mode (collect all hits, then sort and blend) blends the same hits in
    the same order as the checkpointed k-buffer trace on every ray whose hits fit its list
    (here all of them: primary rays of the 100k scene and incoherent rays), with colour,
    depth and opacity equal up to rounding (1e-5; the accumulation runs in another kernel,
    so a ray whose transmittance ends within rounding of T_min may stop one hit apart:
    at most a fraction 1e-3 of the rays)."""
    say("single round", cap)
    scene = inputs.cluster_scene(2, 100_000, 3)
    cam = inputs.orbit_camera(160, 120)
    po, pd = grtx.pinhole_rays(cam)
    io, id_ = (dev(a) for a in inputs.incoherent_rays(33, 4096))
    bvh = build(scene)
    for o, d, w in [(po, pd, cam.width), (io, id_, 0)]:
        a = grtx.trace(bvh, o, d, k=16, T_min=T_MIN, image_width=w, hit_capacity=512, stats=True)
        b = grtx.trace(bvh, o, d, k=16, T_min=T_MIN, image_width=w, hit_capacity=512, stats=True,
                       mode=grtx.SINGLE_ROUND, collect_capacity=cap)
        torch.cuda.synchronize()
        over = int(b["stats"][:, grtx.STAT_FALLBACKS].sum())
        say(dict(rays=int(o.shape[0]), overflowed=over, nodes_single=float(b["stats"][:, :2].sum()) / o.shape[0],
                 nodes_checkpoint=float(a["stats"][:, :2].sum()) / o.shape[0]))
        flag = b["stats"][:, grtx.STAT_FALLBACKS].bool()  # hits beyond the list: incomplete
        if cap >= 2048:
            assert over == 0
        same = (a["hit_counts"] == b["hit_counts"]) & (a["hit_ids"] == b["hit_ids"]).all(1)
        R = int(o.shape[0])
        apart = ~same & ~flag
        assert int(apart.sum()) <= max(1, R // 1000), int(apart.sum())
        same = same & ~flag
        T_b = 1 - b["opacity"][apart]
        assert bool(((T_b - T_MIN).abs() < 1e-5).all())
        for key in ("rgb", "depth", "opacity"):
            err = float((a[key][same] - b[key][same]).abs().max())
            say(key, "max |single - checkpoint|", err)
            assert err <= 1e-5, key
        assert torch.equal(b["stats"][:, grtx.STAT_ROUNDS], torch.ones_like(b["stats"][:, 0]))


def test_single_round_plain_parity_and_overflow():
    """The plain 1k-Gaussian case in single-round mode against the oracle; with a list of
    8 hits the rays with more hits are flagged, and the others still equal the k-buffer
    trace."""
    say("single round plain")
    scene = inputs.small_scene(1, 1000)
    o, d = oracle_rays(inputs.orbit_camera(64, 64))
    bvh = build(scene)
    g = render(bvh, o, d, k=4, mode=grtx.SINGLE_ROUND, cap=256)
    assert int(g["stats"][:, grtx.STAT_FALLBACKS].sum()) == 0
    ref = oracle.render(scene, o, d, AMIN, T_MIN, cap=256)
    say(parity.compare_render(scene, o, d, g, ref, AMIN, T_MIN, label="single round plain"))
    small = grtx.trace(bvh, dev(o), dev(d), k=4, T_min=T_MIN, mode=grtx.SINGLE_ROUND, collect_capacity=8,
                       stats=True)
    full = grtx.trace(bvh, dev(o), dev(d), k=4, T_min=T_MIN, stats=True)
    torch.cuda.synchronize()
    flag = small["stats"][:, grtx.STAT_FALLBACKS].bool()
    n = int(flag.sum())
    say(dict(flagged=n, rays=o.shape[0]))
    assert 0 < n < o.shape[0]
    for key in ("rgb", "depth", "opacity"):
        assert float((small[key][~flag] - full[key][~flag]).abs().max()) <= 1e-5, key


def test_round_structure():
    """Per-round content: round r blends the sorted hits of ranks [(r-1)k, rk), so the
    number of rounds follows from the oracle's blended and total hit counts."""
    say("rounds")
    scene = inputs.cluster_scene(2, 100_000, 3)
    o, d = oracle_rays(inputs.orbit_camera(800, 800))
    idx = inputs.ray_subsample(7, o.shape[0], 1024)
    o, d = o[idx], d[idx]
    ref = oracle.render(scene, o, d, AMIN, T_MIN, cap=512)
    bvh = build(scene)
    for k in [4, 16]:
        for mode in [grtx.RESTART, grtx.CHECKPOINT]:
            g = render(bvh, o, d, k=k, mode=mode, cap=512)
            rounds = g["stats"][:, grtx.STAT_ROUNDS]
            for r in range(len(idx)):
                if int(g["hit_counts"][r]) != int(ref["nblend"][r]):
                    continue  # an allowed exception shifted the list; checked elsewhere
                nb, H = int(ref["nblend"][r]), int(ref["nhits"][r])
                ert = nb > 0 and ref["tafter"][r, nb - 1] < T_MIN
                if ert:
                    want = (math.ceil(nb / k),)
                elif mode == grtx.RESTART:
                    want = (H // k + 1,)
                else:
                    want = (max(1, math.ceil(H / k)), H // k + 1)
                assert int(rounds[r]) in want, (k, mode, r, nb, H, ert, int(rounds[r]))


def test_walkthrough_example():
    """Sec. IV-B walkthrough with k = 4: round 1 ends with primitive 33 (t 2.85) as the
    farthest k-buffer entry and primitive 5 (t 3.2) beyond it; round 2 blends 5 first."""
    say("walkthrough")
    scene, g = walkthrough_scene()
    o = np.float32([g["ray"]["origin"]])
    d = np.float32([g["ray"]["direction"]])
    bvh = build(scene)
    for mode in [grtx.CHECKPOINT, grtx.RESTART]:
        r = render(bvh, o, d, k=g["paper_values"]["k"], mode=mode, cap=16)
        n = int(r["hit_counts"][0])
        assert r["hit_ids"][0, :n].tolist() == g["expected_blend_order"]
        assert r["stats"][0, grtx.STAT_ROUNDS] == g["expected_rounds_k4"]
        if mode == grtx.CHECKPOINT:
            st = r["stats"][0]
            # primitive 5 left round 1 either as an evicted hit or inside a deferred node
            assert st[grtx.STAT_EVICTED] + st[grtx.STAT_DEFERRED] >= 1
            assert st[grtx.STAT_FALLBACKS] == 0
        o32 = float(np.float32(g["opacity"]))
        cols = {e["id"]: np.asarray(e["rgb"]) for e in g["on_ray"]}
        want = sum(o32 * (1 - o32) ** j * dc_colour(cols[i]) for j, i in enumerate(g["expected_blend_order"]))
        np.testing.assert_allclose(r["rgb"][0], want, atol=1e-5)


@pytest.mark.parametrize("o_,n", [(0.5, 20), (0.3, 40), (0.95, 6)])
def test_stacked_slabs_early_termination(o_, n):
    say("slabs", o_, n)
    sig = 0.01
    o32 = float(np.float32(o_))
    rho = math.sqrt(2 * math.log(o32 / AMIN))
    means = [[1.0 + i * 2.5 * rho * sig, 0.0, 0.0] for i in range(n)]
    scene = make_scene(means, [sig] * 3, opac=o_, rgb=[0.2, 0.6, 0.9])
    nstar = math.ceil(math.log(T_MIN) / math.log(1 - o32))
    m = min(n, nstar)
    for k in [1, 4, 16]:
        r = render(build(scene), np.zeros((1, 3), np.float32), np.float32([[1, 0, 0]]), k=k, cap=128)
        assert int(r["hit_counts"][0]) == m
        assert r["opacity"][0] == pytest.approx(1 - (1 - o32) ** m, abs=1e-6)
        np.testing.assert_allclose(r["rgb"][0], dc_colour([0.2, 0.6, 0.9]) * (1 - (1 - o32) ** m), atol=1e-5)


def test_list_overflow_falls_back_to_restart():
    """Checkpoint lists of capacity 1 overflow; the ray restarts from the root for that
    round and the image is unchanged."""
    say("overflow")
    scene = inputs.cluster_scene(2, 100_000, 3)
    cam = inputs.orbit_camera(96, 96)
    o, d = grtx.pinhole_rays(cam)
    bvh = build(scene)
    a = grtx.trace(bvh, o, d, k=8, mode=grtx.CHECKPOINT, stats=True)
    b = grtx.trace(bvh, o, d, k=8, mode=grtx.CHECKPOINT, stats=True, defer_capacity=1, evict_capacity=1)
    torch.cuda.synchronize()
    for key in ["rgb", "depth", "opacity"]:
        assert torch.equal(a[key], b[key]), key
    fa = int(a["stats"][:, grtx.STAT_FALLBACKS].sum())
    fb = int(b["stats"][:, grtx.STAT_FALLBACKS].sum())
    assert fb > fa and fb > 0, (fa, fb)


@pytest.mark.parametrize("caps", [(8, 8), (24, 16), (64, 40)])
def test_full_lists_compact_and_keep_results(caps):
    """Rays that start at Gaussian centres inside dense clusters defer and evict more than
    small lists hold: a full list is compacted (the near entries stay, the limit comes down)
    and the ray restarts from the root only if its blending reaches the limit. Colour,
    depth, opacity and the blended hits equal the default lists' bit for bit, and the oracle
    by the per-ray rule."""
    say("compaction", caps)
    scene = inputs.cluster_scene(2, 100_000, 3)
    rng = np.random.default_rng(71)
    pick = rng.choice(scene.n, 768, replace=False)
    o = scene.means[pick].astype(np.float32)
    d = rng.normal(size=(768, 3))
    d = (d / np.linalg.norm(d, axis=1, keepdims=True)).astype(np.float32)
    bvh = build(scene)
    a = render(bvh, o, d, k=8, cap=512)
    b = render(bvh, o, d, k=8, cap=512, defer_capacity=caps[0], evict_capacity=caps[1])
    for key in ["rgb", "depth", "opacity", "hit_counts", "hit_ids"]:
        assert np.array_equal(a[key], b[key]), (caps, key)
    assert int(b["stats"][:, grtx.STAT_DEFERRED].max()) > caps[0]  # more entries than a list holds went through
    ref = oracle.render(scene, o, d, AMIN, T_MIN, cap=512)
    s = parity.compare_render(scene, o, d, b, ref, AMIN, T_MIN, label=f"compaction {caps}")
    say(s, "fallbacks", int(b["stats"][:, grtx.STAT_FALLBACKS].sum()))


def test_degenerate_inputs():
    say("degenerate")
    o = np.float32([[0, -3, 0], [0, -3, 0]])
    d = np.float32([[0, 1, 0], [1, 0, 0]])
    empty = make_scene(np.zeros((0, 3)), [0.1] * 3)
    bvh = build(empty)
    r = grtx.trace(bvh, dev(o), dev(d), bg=(0.1, 0.2, 0.3))
    torch.cuda.synchronize()
    np.testing.assert_array_equal(r["rgb"].cpu().numpy(), np.float32([[0.1, 0.2, 0.3]] * 2))
    one = make_scene([[0.0, 0.0, 0.0]], [0.1] * 3, opac=0.5, rgb=[1, 0, 0])
    r = render(build(one), o, d, k=4, cap=4)
    ref = oracle.render(one, o, d, AMIN, T_MIN)
    np.testing.assert_allclose(r["rgb"], ref["rgb"], atol=1e-5)
    assert r["hit_counts"].tolist() == [1, 0]
    # zero rays is a no-op
    z = grtx.trace(build(one), dev(np.zeros((0, 3))), dev(np.zeros((0, 3))))
    assert z["rgb"].shape == (0, 3)
    # a Gaussian with opacity at or below alpha_min is never hit
    faint = make_scene([[0.0, 0.0, 0.0]], [0.1] * 3, opac=AMIN)
    r = render(build(faint), o, d, k=4, cap=4)
    assert r["hit_counts"].tolist() == [0, 0]


def test_full_size_scene100k_sampled():
    """The benchmark's trace launch: all 800x800 primary rays, 100k Gaussians, k=16,
    checkpointing, 8x8 tile scheduling; sampled pixels against the oracle. The rays are
    the oracle's pinhole rays rounded to binary32 (the GPU's own ray generator is checked
    separately), so both sides trace identical rays."""
    say("full-size 800x800")
    scene = inputs.cluster_scene(2, 100_000, 3)
    cam = inputs.orbit_camera(800, 800)
    ro, rd = oracle_rays(cam)
    bvh = build(scene)
    out = grtx.trace(bvh, dev(ro), dev(rd), k=16, T_min=T_MIN, image_width=800, hit_capacity=512, stats=True)
    torch.cuda.synchronize()
    g = {k: v.cpu().numpy() for k, v in out.items()}
    assert np.isfinite(g["rgb"]).all() and (g["hit_counts"] <= 512).all()
    assert (g["stats"][:, grtx.STAT_ROUNDS] >= 1).all()  # every ray was finished
    idx = inputs.ray_subsample(123, ro.shape[0], 768)
    sub = {k: v[idx] for k, v in g.items()}
    ref = oracle.render(scene, ro[idx], rd[idx], AMIN, T_MIN, cap=512)
    s = parity.compare_render(scene, ro[idx], rd[idx], sub, ref, AMIN, T_MIN, label="full-size")
    say(s)


@pytest.mark.parametrize("k", [16, 32])
def test_scene3m_full_size_sampled(k):
    """The largest workload at full size: 3M Gaussians, all 1920x1080 primary rays (8x8
    tile scheduling) and 2M incoherent rays (origins uniform in the scene box, directions
    uniform on the sphere), k = 16 and 32, checkpointing; sampled rays of both sets against
    the oracle's brute force over all 3M Gaussians."""
    cfg = inputs.SCENE3M
    say("scene 3M full size, k", k)
    scene = inputs.cluster_scene(cfg["seed"], cfg["n"], 3)
    cam = inputs.orbit_camera(cfg["width"], cfg["height"])
    ro, rd = oracle_rays(cam)
    io, id_ = inputs.incoherent_rays(cfg["incoherent_seed"], cfg["incoherent"])
    bvh = build(scene)
    # one launch, as the benchmark's step traces them: the incoherent rays, then the image
    n_inc = io.shape[0]
    out = grtx.trace(bvh, dev(np.concatenate([io, ro])), dev(np.concatenate([id_, rd])), k=k, T_min=T_MIN,
                     image_width=cfg["width"], image_begin=n_inc, hit_capacity=512, stats=True)
    torch.cuda.synchronize()
    assert bool(torch.isfinite(out["rgb"]).all())
    assert int(out["stats"][:, grtx.STAT_ROUNDS].min()) >= 1  # every ray was finished
    for label, o, d, first, seed in [("primary", ro, rd, n_inc, 7), ("incoherent", io, id_, 0, 8)]:
        idx = inputs.ray_subsample(seed, o.shape[0], 192)
        ti = torch.from_numpy(idx + first).cuda()
        sub = {name: v.index_select(0, ti).cpu().numpy() for name, v in out.items()}
        ref = oracle.render(scene, o[idx], d[idx], AMIN, T_MIN, cap=512)
        s = parity.compare_render(scene, o[idx], d[idx], sub, ref, AMIN, T_MIN, label=f"3M {label} k={k}")
        say(s)
    del out


def test_scene3m_restart_equals_checkpoint():
    """The largest workload's one launch (2M incoherent rays, then the 1920x1080 frame's
    tiles), k = 16, in both modes: restart from the root gives bit-identical colour, depth,
    opacity, hit lists and blended counts, and fetches more nodes on both ray sets (the
    comparison of Sec. V-B at full size)."""
    cfg = inputs.SCENE3M
    say("scene 3M restart against checkpoint")
    scene = inputs.cluster_scene(cfg["seed"], cfg["n"], 3)
    cam = inputs.orbit_camera(cfg["width"], cfg["height"])
    ro, rd = oracle_rays(cam)
    io, id_ = inputs.incoherent_rays(cfg["incoherent_seed"], cfg["incoherent"])
    bvh = build(scene)
    n_inc = io.shape[0]
    o, d = dev(np.concatenate([io, ro])), dev(np.concatenate([id_, rd]))
    kw = dict(k=16, T_min=T_MIN, image_width=cfg["width"], image_begin=n_inc, hit_capacity=64, stats=True)
    a = grtx.trace(bvh, o, d, mode=grtx.CHECKPOINT, **kw)
    b = grtx.trace(bvh, o, d, mode=grtx.RESTART, **kw)
    torch.cuda.synchronize()
    for key in ("rgb", "depth", "opacity", "hit_ids", "hit_counts"):
        assert torch.equal(a[key], b[key]), key
    assert torch.equal(a["stats"][:, grtx.STAT_BLENDED], b["stats"][:, grtx.STAT_BLENDED])
    for label, sl in (("incoherent", slice(0, n_inc)), ("primary", slice(n_inc, None))):
        fa = int(a["stats"][sl, grtx.STAT_NODES].sum())
        fb = int(b["stats"][sl, grtx.STAT_NODES].sum())
        say(dict(set=label, node_fetches_checkpoint=fa, node_fetches_restart=fb))
        assert fb > fa, label
    del a, b


def test_two_streams_in_turn_equal_one_stream():
    """Frames issued on two streams in turn (ray generation, build and trace each; every
    stream with its own scratch arena and checkpoint pool, consecutive frames overlapping
    on the device) give the same outputs and hit lists, bit for bit, as one stream."""
    say("two streams in turn")
    scene = inputs.cluster_scene(2, 100_000, 3)
    st = grtx.SceneTensors.from_scene(scene, "cuda")
    cam = inputs.orbit_camera(320, 240)
    kw = dict(k=16, T_min=T_MIN, image_width=cam.width, hit_capacity=64)
    o, d = grtx.pinhole_rays(cam)
    ref = grtx.trace(grtx.build(st, alpha_min=AMIN), o, d, **kw)
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    keep, outs = [], []
    for i in range(6):
        s = streams[i % 2]
        with torch.cuda.stream(s):
            oi, di = grtx.pinhole_rays(cam, stream=s)
            bvh = grtx.build(st, alpha_min=AMIN, stream=s)
            outs.append(grtx.trace(bvh, oi, di, stream=s, **kw))
        keep.append((bvh, oi, di))
    torch.cuda.synchronize()
    for i, out in enumerate(outs):
        for key in ("rgb", "depth", "opacity", "hit_ids", "hit_counts"):
            assert torch.equal(out[key], ref[key]), (i, key)


def test_image_part_that_does_not_divide_into_rows():
    """Rays after image_begin that do not divide into rows of image_width are all taken as
    free rays (scheduling only): outputs, hit lists and blended counts bit-equal to a trace
    that declares no image."""
    say("ragged image part")
    scene = inputs.cluster_scene(2, 100_000, 3)
    bvh = build(scene)
    o, d = (dev(a) for a in inputs.incoherent_rays(45, 10_007))
    kw = dict(k=16, T_min=T_MIN, hit_capacity=128, stats=True)
    a = grtx.trace(bvh, o, d, image_width=100, image_begin=3, **kw)  # 10,004 rays: not rows of 100
    b = grtx.trace(bvh, o, d, **kw)
    torch.cuda.synchronize()
    for key in ("rgb", "depth", "opacity", "hit_ids", "hit_counts"):
        assert torch.equal(a[key], b[key]), key
    assert torch.equal(a["stats"][:, grtx.STAT_BLENDED], b["stats"][:, grtx.STAT_BLENDED])


@pytest.mark.parametrize("width,height,n_free", [(160, 120, 70_000), (100, 37, 5_003), (64, 64, 0)])
def test_image_after_free_rays_one_launch(width, height, n_free):
    """Rays that form no image and an image traced in one launch (image_begin): each ray's
    outputs, hit list, blended count and (where no ray restarted after a list compaction)
    rounds are bit-equal to those of its own set traced alone
    (scheduling only; 70,000 free rays are enough for the density ordering, 5,003 are
    not; a 100x37 image has ragged tiles), and sampled rays of both parts match the
    oracle. With image_begin = count every ray is a free ray."""
    say("image after free rays", width, height, n_free)
    scene = inputs.cluster_scene(2, 100_000, 3)
    cam = inputs.orbit_camera(width, height)
    po, pd = oracle_rays(cam)
    fo, fd = inputs.incoherent_rays(44, n_free) if n_free else (np.zeros((0, 3), np.float32),) * 2
    bvh = build(scene)
    ho, hd = np.concatenate([fo, po]), np.concatenate([fd, pd])
    o, d = dev(ho), dev(hd)
    kw = dict(k=16, T_min=T_MIN, hit_capacity=256, stats=True)
    both = grtx.trace(bvh, o, d, image_width=width, image_begin=n_free, **kw)
    img = grtx.trace(bvh, dev(po), dev(pd), image_width=width, **kw)
    free = grtx.trace(bvh, dev(fo), dev(fd), **kw) if n_free else None
    flat = grtx.trace(bvh, o, d, image_width=width, image_begin=o.shape[0], **kw)  # no image part
    torch.cuda.synchronize()
    for key in ("rgb", "depth", "opacity", "hit_ids", "hit_counts"):
        assert torch.equal(both[key][n_free:], img[key]), key
        assert torch.equal(flat[key], both[key]), key
        if free is not None:
            assert torch.equal(both[key][:n_free], free[key]), key
    # counters that do not follow the scheduling (the others count work, which depends on
    # when a full checkpoint list was compacted)
    alone = torch.cat([free["stats"], img["stats"]]) if free is not None else img["stats"]
    for other in (alone, flat["stats"]):
        for f in (grtx.STAT_BLENDED, grtx.STAT_STACK_DROPS):
            assert torch.equal(both["stats"][:, f], other[:, f]), f
        # rounds too, where neither launch restarted a ray from the root after a compaction
        ok = (both["stats"][:, grtx.STAT_FALLBACKS] == 0) & (other[:, grtx.STAT_FALLBACKS] == 0)
        assert torch.equal(both["stats"][ok, grtx.STAT_ROUNDS], other[ok, grtx.STAT_ROUNDS])
    g = {key: v.cpu().numpy() for key, v in both.items()}
    for first, n, seed in [(0, n_free, 3), (n_free, po.shape[0], 4)]:
        if n == 0:
            continue
        idx = inputs.ray_subsample(seed, n, 256) + first
        ref = oracle.render(scene, ho[idx], hd[idx], AMIN, T_MIN, cap=256)
        sub = {key: v[idx] for key, v in g.items()}
        say(parity.compare_render(scene, ho[idx], hd[idx], sub, ref, AMIN, T_MIN,
                                  label=f"one launch {width}x{height}+{n_free}"))


# ------------------------------------------------------------------------ proxy-mesh baseline

@pytest.mark.parametrize("mode", [grtx.CHECKPOINT, grtx.RESTART])
def test_proxy_plain_parity(mode):
    """20-triangle bounding-icosahedron BVH against the oracle's proxy-key mode."""
    say("proxy plain mode", mode)
    scene = inputs.small_scene(1, 1000)
    o, d = oracle_rays(inputs.orbit_camera(64, 64))
    g = render(build(scene, grtx.PROXY20), o, d, k=4, mode=mode, cap=256)
    ref = oracle.render(scene, o, d, AMIN, T_MIN, key_mode=1, cap=256)
    s = parity.compare_render(scene, o, d, g, ref, AMIN, T_MIN, label=f"proxy plain mode={mode}",
                              key_mode=1)
    say(s)


def test_proxy_scene100k_parity_sampled():
    say("proxy 100k")
    scene = inputs.cluster_scene(2, 100_000, 3)
    o, d = oracle_rays(inputs.orbit_camera(800, 800))
    idx = inputs.ray_subsample(99, o.shape[0], 1024)
    o, d = o[idx], d[idx]
    bvh = build(scene, grtx.PROXY20)
    assert bvh.info()["leaves"] == 20 * scene.n
    g = render(bvh, o, d, k=16, cap=512)
    ref = oracle.render(scene, o, d, AMIN, T_MIN, key_mode=1, cap=512)
    s = parity.compare_render(scene, o, d, g, ref, AMIN, T_MIN, label="proxy 100k", key_mode=1)
    say(s)
    g2 = render(bvh, o, d, k=16, mode=grtx.RESTART, cap=512)
    for key in ["rgb", "depth", "hit_ids", "hit_counts"]:
        assert np.array_equal(g[key], g2[key]), key


# ------------------------------------------------------------------ instanced icosahedron

@pytest.mark.parametrize("mode", [grtx.CHECKPOINT, grtx.RESTART])
def test_ico_instance_plain_parity(mode):
    """Instances of one shared icosahedron (inradius 1 in each Gaussian's unit frame): the
    same keys as the 20-triangle proxy mesh, checked against the oracle's proxy-key mode."""
    say("ico instance plain mode", mode)
    scene = inputs.small_scene(1, 1000)
    o, d = oracle_rays(inputs.orbit_camera(64, 64))
    bvh = build(scene, grtx.ICO_INSTANCE)
    assert bvh.info()["leaves"] == scene.n
    g = render(bvh, o, d, k=4, mode=mode, cap=256)
    ref = oracle.render(scene, o, d, AMIN, T_MIN, key_mode=1, cap=256)
    s = parity.compare_render(scene, o, d, g, ref, AMIN, T_MIN, label=f"ico plain mode={mode}", key_mode=1)
    say(s)


def test_ico_instance_scene100k_parity_sampled():
    """100k scene-scale Gaussians, sampled primary and incoherent rays, k = 16: against the
    oracle's proxy key, and checkpoint equal to restart; the images equal the proxy mesh's
    up to the allowed exceptions."""
    say("ico instance 100k")
    scene = inputs.cluster_scene(2, 100_000, 3)
    o, d = oracle_rays(inputs.orbit_camera(800, 800))
    idx = inputs.ray_subsample(98, o.shape[0], 768)
    io, id_ = inputs.incoherent_rays(77, 256)
    o, d = np.concatenate([o[idx], io]), np.concatenate([d[idx], id_])
    bvh = build(scene, grtx.ICO_INSTANCE)
    g = render(bvh, o, d, k=16, cap=512)
    ref = oracle.render(scene, o, d, AMIN, T_MIN, key_mode=1, cap=512)
    s = parity.compare_render(scene, o, d, g, ref, AMIN, T_MIN, label="ico 100k", key_mode=1)
    say(s)
    g2 = render(bvh, o, d, k=16, mode=grtx.RESTART, cap=512)
    for key in ["rgb", "depth", "hit_ids", "hit_counts"]:
        assert np.array_equal(g[key], g2[key]), key


def test_proxy_topology_and_boxes():
    say("proxy topology")
    from tests.test_oracle_pins import _check_radix_tree
    scene = inputs.cluster_scene(5, 400, 0)
    bvh = build(scene, grtx.PROXY20, plain_lbvh=True)
    t = bvh.export_topology()
    m = 20 * scene.n
    codes = t["morton"].cpu().numpy().view(np.uint64)
    perm = t["perm"].cpu().numpy().view(np.uint32)
    assert np.array_equal(np.sort(perm), np.arange(m, dtype=np.uint32))
    _check_radix_tree(codes, perm, t["child"].cpu().numpy().view(np.uint32), t["parent"].cpu().numpy().view(np.uint32), m)
    # every leaf box holds its triangle (FP64 icosahedron of the oracle mapped to world)
    boxes = t["boxes"].cpu().numpy().astype(np.float64)[m - 1:]
    v, f = oracle.icosahedron()
    from tests.helpers import quat_to_matrix_scipy, rho_of
    for p in range(0, m, 7):
        gi, face = divmod(int(perm[p]), 20)
        q = scene.quats[gi].astype(np.float64)
        R = quat_to_matrix_scipy(q / np.linalg.norm(q))
        o = float(scene.opacities[gi])
        if o <= AMIN:
            continue
        sc = scene.scales[gi].astype(np.float64) * rho_of(o, AMIN)
        W = scene.means[gi].astype(np.float64) + (v * sc) @ R.T
        # the library numbers faces its own way: the box must hold one face of the mesh,
        # and be no larger than that face's box plus the padding
        ok = False
        for tri in W[f]:
            lo, hi = tri.min(0), tri.max(0)
            inside = (lo >= boxes[p, :3] - 1e-6).all() and (hi <= boxes[p, 3:] + 1e-6).all()
            tight = ((boxes[p, 3:] - boxes[p, :3]) <= (hi - lo) * (1 + 2 ** -9) + 1e-4).all()
            ok = ok or (inside and tight)
        assert ok, (p, boxes[p])
