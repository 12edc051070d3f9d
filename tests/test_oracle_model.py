"""The CPU model of the method in the oracle (rounds of k-buffer hit collection over a
BVH, resuming from checkpoint lists or from the root; Sec. III-B and IV) against the
brute-force definition, the paper's per-round structure and its walkthrough (Sec. IV-B).
CPU only."""
import numpy as np
import pytest

import oracle
from paper_2601_20429_amd import inputs
from paper_2601_20429_amd.inputs import Scene
from tests.helpers import load_golden, walkthrough_scene

AMIN = float(np.float32(1.0 / 255.0))
T_MIN = 1e-3
MODES = [oracle.CHECKPOINT, oracle.RESTART]
RULES = [oracle.RULE_KBUF_MAX, oracle.RULE_PAPER]


def dense_tiny(seed, n, dup=0):
    """The plain-method generator with Gaussians six times larger, so that rays meet many
    of them; `dup` Gaussians repeated exactly (equal keys, ordered by id)."""
    s = inputs.small_scene(seed, n)
    f = lambda a: np.ascontiguousarray(a, np.float32)
    sc = Scene(s.means, f(s.scales * 6.0), s.quats, s.opacities, s.sh, 0)
    if dup:
        idx = np.concatenate([np.arange(n), np.arange(dup)])
        sc = sc.subset(idx)
    return sc


def rays(seed, n_cam, n_inc):
    cam = inputs.orbit_camera(n_cam, n_cam)
    o, d = oracle.pinhole_rays(cam)
    io, id_ = inputs.incoherent_rays(seed, n_inc, box=1.0)
    return (np.concatenate([o.astype(np.float32), io]), np.concatenate([d.astype(np.float32), id_]))


def check_same(scene, o, d, k, mode, rule, cap=512):
    ref = oracle.render(scene, o, d, AMIN, T_MIN, cap=cap)
    m = oracle.model_render(scene, o, d, k, mode, rule, AMIN, T_MIN, cap=cap)
    assert np.array_equal(m["nblend"], ref["nblend"])
    for r in range(o.shape[0]):
        nb = min(int(ref["nblend"][r]), cap)
        assert np.array_equal(m["ids"][r, :nb], ref["ids"][r, :nb]), r
    # the same hits in the same order through the same arithmetic
    for key in ("rgb", "depth", "opacity"):
        assert np.array_equal(m[key], ref[key]), key
    return ref, m


@pytest.mark.parametrize("n,dup", [(1, 0), (2, 0), (17, 0), (64, 0), (40, 8)])
def test_model_equals_brute_force(n, dup):
    """On tiny random scenes (one Gaussian, two, 17, 64, and 40 with 8 repeated exactly),
    the model blends exactly the brute force's hits in its order for every k, both modes
    and both t_max rules: the BVH, the rounds and the checkpoints lose, repeat and reorder
    nothing."""
    scene = dense_tiny(10 + n, n, dup)
    o, d = rays(20 + n, 8, 96)
    for k in (1, 2, 4, 16):
        for mode in MODES:
            for rule in RULES:
                check_same(scene, o, d, k, mode, rule)


def test_model_rounds_blend_consecutive_ranks():
    """Round r blends the hits of sorted ranks (r-1)k .. rk-1 (each round collects the k
    nearest hits not yet blended), and the ray takes ceil(n/k) rounds for n blended hits,
    or one more when the last round filled its k-buffer and found nothing beyond. With
    checkpoints no node or leaf is visited twice."""
    scene = dense_tiny(31, 64)
    o, d = rays(32, 8, 96)
    for k in (1, 3, 4, 16):
        for mode in MODES:
            for rule in RULES:
                m = oracle.model_render(scene, o, d, k, mode, rule, AMIN, T_MIN, cap=512)
                c = m["counts"]
                if mode == oracle.CHECKPOINT:  # no node or leaf visited twice
                    assert np.array_equal(c[:, 0] + c[:, 1], c[:, 4]), (k, rule)
                for r in range(o.shape[0]):
                    nb = int(m["nblend"][r])
                    assert np.array_equal(m["round_of"][r, :nb], np.arange(nb) // k + 1), (k, mode, rule, r)
                    want = {max(1, -(-nb // k)), nb // k + 1}
                    assert int(m["rounds"][r]) in want, (k, mode, rule, r, nb, int(m["rounds"][r]))


def test_model_scene100k_and_checkpoint_saves_fetches():
    """A 100k-Gaussian SH-degree-3 scene: primary and incoherent rays at k = 16 match the
    brute force in both modes. Checkpointing visits every node and leaf at most once and
    fewer in all than restart from root, whose rays of several rounds visit some twice."""
    scene = inputs.cluster_scene(2, 100_000, 3)
    cam = inputs.orbit_camera(64, 64)
    po, pd = oracle.pinhole_rays(cam)
    idx = inputs.ray_subsample(5, po.shape[0], 24)
    io, id_ = inputs.incoherent_rays(33, 24)
    o = np.concatenate([po[idx].astype(np.float32), io])
    d = np.concatenate([pd[idx].astype(np.float32), id_])
    fetched = {}
    for mode in MODES:
        _, m = check_same(scene, o, d, 16, mode, oracle.RULE_KBUF_MAX)
        c = m["counts"]
        visits = c[:, 0] + c[:, 1]
        fetched[mode] = int(visits.sum())
        if mode == oracle.RESTART:
            assert int(c[:, 2].sum()) == 0 and int(c[:, 3].sum()) == 0 and int(c[:, 5].sum()) == 0
            # rays of several rounds walk the top of the tree again each round
            multi = m["rounds"] > 1
            assert multi.any() and (visits[multi] > c[multi, 4]).all()
        else:
            # checkpointing visits no node and no leaf twice
            assert np.array_equal(visits, c[:, 4])
    assert fetched[oracle.CHECKPOINT] < fetched[oracle.RESTART], fetched


def test_walkthrough_round_one_state():
    """Sec. IV-B: with k = 4 the k-buffer ends round 1 holding the four nearest hits, the
    farthest being primitive 33 at t = 2.85; primitive 5 at t = 3.2 was turned away into
    the eviction list, and under the paper's rule t_max moved from infinity to 3.2. The far
    Gaussian beyond it waits in a checkpoint (a deferred node, or the eviction list), and
    round 2 blends primitive 5 first. Under the k-buffer-maximum rule t_max is 2.85 and
    primitive 5 may wait in a deferred node instead; the image is the same."""
    scene, g = walkthrough_scene()
    pv = g["paper_values"]
    o = np.float32(g["ray"]["origin"])
    d = np.float32(g["ray"]["direction"])
    k = pv["k"]
    perm = oracle.lbvh_topology(scene.means)["perm"]
    far = [e["id"] for e in g["on_ray"] if e["t_entry"] > pv["rejected_hit"]["t_hit"]]

    def under_deferred(st, gid):
        pos = int(np.nonzero(perm == gid)[0][0])
        return bool(((st["deferred_first"] <= pos) & (pos <= st["deferred_last"])).any())

    for rule in RULES:
        st = oracle.model_round_state(scene, o, d, k, 1, oracle.CHECKPOINT, rule, AMIN, T_MIN)
        assert st["kbuf_ids"].tolist() == g["expected_round1_ids_k4"]
        assert st["kbuf_ids"][-1] == pv["farthest_in_kbuffer"]["id"]
        assert st["kbuf_t"][-1] == pytest.approx(pv["farthest_in_kbuffer"]["t_hit"], abs=1e-5)
        rej = pv["rejected_hit"]["id"]
        if rule == oracle.RULE_PAPER:
            assert rej in st["evicted_ids"].tolist()
            assert st["tmax_id"] == rej
            assert st["tmax_t"] == pytest.approx(pv["t_max_after"], abs=1e-5)
        else:
            assert rej in st["evicted_ids"].tolist() or under_deferred(st, rej)
            assert st["tmax_id"] == pv["farthest_in_kbuffer"]["id"]
            assert st["tmax_t"] == pytest.approx(pv["farthest_in_kbuffer"]["t_hit"], abs=1e-5)
        for gid in far:
            assert gid in st["evicted_ids"].tolist() or under_deferred(st, gid), (rule, gid)
        m = oracle.model_render(scene, o[None], d[None], k, oracle.CHECKPOINT, rule, AMIN, T_MIN, cap=16)
        nb = int(m["nblend"][0])
        assert m["ids"][0, :nb].tolist() == g["expected_blend_order"]
        assert m["round_of"][0, :nb].tolist() == [1, 1, 1, 1, 2, 2]
        assert int(m["rounds"][0]) == g["expected_rounds_k4"]
