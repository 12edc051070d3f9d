"""Backward kernel vs FP64 central finite differences of the oracle, through the C ABI
and the autograd Function. Needs an MI355X and the built library."""
import copy
import sys

import numpy as np
import pytest

import oracle
from paper_2601_20429_amd import inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
from paper_2601_20429_amd import autograd, grtx  # noqa: E402

AMIN = float(np.float32(1.0 / 255.0))
T_MIN = 1e-3


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    yield
    torch.cuda.synchronize()


def _as64(scene):
    s = copy.copy(scene)
    for f in ["means", "scales", "quats", "opacities", "sh"]:
        setattr(s, f, getattr(scene, f).astype(np.float64))
    return s


LOSSES = {  # weights of the rgb, depth and opacity terms of L = sum w * (x - x_target)^2
    "rgb": (1.0, 0.0, 0.0),
    "depth": (0.0, 1.0, 0.0),
    "opacity": (0.0, 0.0, 1.0),
    "all": (1.0, 0.1, 1.0),
}


def _loss(out, tgt, w):
    return (w[0] * ((out["rgb"] - tgt["rgb"]) ** 2).sum() + w[1] * ((out["depth"] - tgt["depth"]) ** 2).sum()
            + w[2] * ((out["opacity"] - tgt["opacity"]) ** 2).sum())


def _loss_oracle(scene64, o, d, tgt, w):
    r = oracle.render(scene64, o, d, AMIN, T_MIN, cap=256)
    return float(_loss(r, tgt, w)), r["ids"], r["nblend"]


@pytest.mark.parametrize("loss", list(LOSSES))
def test_gradients_match_oracle_finite_differences(loss):
    """L = sum of squared differences to a target over a 32x32 image of a 500-Gaussian
    SH-degree-3 scene, on colour, depth, opacity or all three; the target is the oracle's
    render of the scene with means + N(0, 0.01^2). The GPU's FP32 gradients for mean,
    scale, rotation, opacity and SH must match FP64 central differences of the oracle
    wherever the perturbation leaves every ray's blended list unchanged:
    |g - fd| <= 0.03 |fd| + 2e-3 rms(fd), with at least 4 such checks per parameter group."""
    say("fd gradients", loss)
    w = LOSSES[loss]
    scene = inputs.fd_scene(5, 500)
    cam = inputs.orbit_camera(32, 32)
    o, d = oracle.pinhole_rays(cam)
    o, d = o.astype(np.float32), d.astype(np.float32)
    tgt = oracle.render(inputs.perturbed_means(scene, 44), o, d, AMIN, T_MIN)

    st = grtx.SceneTensors.from_scene(scene, "cuda")
    params = [st.means.clone().requires_grad_(), st.scales.clone().requires_grad_(),
              st.quats.clone().requires_grad_(), st.opacities.clone().requires_grad_(),
              st.sh.clone().requires_grad_()]
    settings = autograd.RenderSettings(sh_degree=3, k=8, T_min=T_MIN, alpha_min=AMIN, hit_capacity=256)
    rgb, depth, opac = autograd.render(*params, torch.from_numpy(o).cuda(), torch.from_numpy(d).cuda(), settings)
    t_gpu = {k: torch.from_numpy(np.asarray(v, np.float64)).float().cuda() for k, v in tgt.items()
             if k in ("rgb", "depth", "opacity")}
    L = _loss(dict(rgb=rgb, depth=depth, opacity=opac), t_gpu, w)
    L.backward()
    torch.cuda.synchronize()
    g = {name: p.grad.cpu().numpy().astype(np.float64) for name, p in
         zip(["means", "scales", "quats", "opacities", "sh"], params)}

    s64 = _as64(scene)
    L0, ids0, nb0 = _loss_oracle(s64, o, d, tgt, w)
    assert abs(L0 - float(L.detach())) < 1e-3 * max(1.0, abs(L0))
    used = np.unique(np.concatenate([ids0[r, :nb0[r]] for r in range(len(nb0))]))
    assert used.size > 50
    rng = np.random.default_rng(0)
    checks = []
    for field, width in [("means", 3), ("scales", 3), ("quats", 4), ("opacities", 1), ("sh", 48)]:
        found = 0
        for _ in range(40):
            if found == 8:
                break
            i = int(rng.choice(used))
            j = int(rng.integers(width))
            arr = getattr(s64, field)
            flat = arr.reshape(arr.shape[0], -1)
            h = 1e-5 * max(1.0, abs(flat[i, j])) if field != "scales" else 1e-4 * abs(flat[i, j])
            res = []
            lists = []
            for sgn in (+1, -1):
                sp = copy.copy(s64)
                a2 = arr.copy()
                a2.reshape(a2.shape[0], -1)[i, j] += sgn * h
                setattr(sp, field, a2)
                Lp, ids, nb = _loss_oracle(sp, o, d, tgt, w)
                res.append(Lp)
                lists.append((ids, nb))
            same = all(np.array_equal(nb, nb0) and all(np.array_equal(ids[r, :nb[r]], ids0[r, :nb0[r]])
                                                       for r in range(len(nb0))) for ids, nb in lists)
            if not same:
                continue  # the perturbation changes a blended list: not differentiable there
            fd = (res[0] - res[1]) / (2 * h)
            gg = g[field].reshape(g[field].shape[0], -1)[i, j]
            checks.append((field, i, j, gg, fd))
            found += 1
    fds = np.array([c[4] for c in checks])
    rms = float(np.sqrt((fds ** 2).mean()))
    bad = [c for c in checks if abs(c[3] - c[4]) > 0.03 * abs(c[4]) + 2e-3 * rms]
    say(f"{loss}: {len(checks)} checked, rms fd {rms:.3e}, bad {len(bad)}")
    for f in ["means", "scales", "quats", "opacities", "sh"]:
        cs = [c for c in checks if c[0] == f]
        err = max((abs(c[3] - c[4]) / (abs(c[4]) + 1e-12) for c in cs), default=float("nan"))
        say(loss, f, len(cs), "max rel err", f"{err:.2e}")
        assert len(cs) >= 4, (loss, f, len(cs))
    assert rms > 0
    assert not bad, bad[:6]


def test_backward_retraces_without_a_hit_list():
    """Without the forward's hit-id list the backward pass traces the rays again: the
    gradients equal those from the listed forward bit for bit, also when the rays are
    scheduled as an image."""
    say("backward re-trace")
    scene = inputs.cluster_scene(7, 20_000, 3)
    st = grtx.SceneTensors.from_scene(scene, "cuda")
    o, d = grtx.pinhole_rays(inputs.orbit_camera(128, 96))
    bvh = grtx.build(st, alpha_min=AMIN)
    fwd = grtx.trace(bvh, o, d, k=16, T_min=T_MIN, hit_capacity=256)
    g_rgb = torch.rand_like(fwd["rgb"])
    g_dep = torch.rand_like(fwd["depth"])
    a, ta = grtx.trace_backward(bvh, o, d, fwd, grad_rgb=g_rgb, grad_depth=g_dep, k=16, T_min=T_MIN)
    b, tb = grtx.trace_backward(bvh, o, d, None, grad_rgb=g_rgb, grad_depth=g_dep, k=16, T_min=T_MIN,
                                hit_capacity=256)
    # the same re-trace scheduled as a 128-wide image, and a forward traced that way
    c, tc = grtx.trace_backward(bvh, o, d, None, grad_rgb=g_rgb, grad_depth=g_dep, k=16, T_min=T_MIN,
                                hit_capacity=256, image_width=128)
    fwd_img = grtx.trace(bvh, o, d, k=16, T_min=T_MIN, hit_capacity=256, image_width=128)
    torch.cuda.synchronize()
    assert int(ta.item()) == 0 and int(tb.item()) == 0 and int(tc.item()) == 0
    for key in a:
        assert torch.equal(a[key], b[key]), key
        assert torch.equal(a[key], c[key]), key
    for key in fwd:
        assert torch.equal(fwd[key], fwd_img[key]), key
    assert float(a["means"].abs().sum()) > 0


def test_backward_is_repeatable_and_finite_at_scale():
    """200k-Gaussian scene, 512x512 rays, k = 16: gradients are finite and two runs are
    bit-identical (the per-Gaussian sums run in a fixed order)."""
    say("backward 200k 512x512")
    cfg = inputs.DIFF200K
    scene = inputs.cluster_scene(cfg["seed"], cfg["n"], 3)
    st = grtx.SceneTensors.from_scene(scene, "cuda")
    o, d = grtx.pinhole_rays(inputs.orbit_camera(cfg["width"], cfg["height"]))
    bvh = grtx.build(st, alpha_min=AMIN)
    fwd = grtx.trace(bvh, o, d, k=16, T_min=T_MIN, hit_capacity=256)
    g_rgb = torch.ones_like(fwd["rgb"])
    g1, tr1 = grtx.trace_backward(bvh, o, d, fwd, grad_rgb=g_rgb, k=16, T_min=T_MIN)
    g2, tr2 = grtx.trace_backward(bvh, o, d, fwd, grad_rgb=g_rgb, k=16, T_min=T_MIN)
    torch.cuda.synchronize()
    assert int(tr1.item()) == 0
    for k in g1:
        a, b = g1[k], g2[k]
        assert torch.isfinite(a).all(), k
        assert torch.equal(a, b), k
    assert float(g1["opacities"].abs().sum()) > 0
