"""Pins for the oracle's secondary rays: a glass sphere that refracts and a mirror that
reflects (ray continuation at a surface, Sec. II-A; the secondary-ray experiment of
Sec. VI), and for rays bounded by a surface or starting with a transmittance below one.

The geometry is pinned by closed forms (the deviation of a ray through a sphere, the
law of reflection, total internal reflection), the compositing of continued rays by two
identities that hold exactly: a mirror is equivalent to the scene's reflection seen
straight through the mirror plane, and a glass sphere of index 1 in empty space is
invisible."""
import math

import numpy as np
import pytest

import oracle
from paper_2601_20429_amd import inputs
from tests.helpers import dc_colour, make_scene, quat_to_matrix_scipy, rho_of

AMIN = 1.0 / 255.0


def _objects(sphere=None, mirror=None, eps=1e-4):
    d = {"eps": eps}
    if sphere is not None:
        d["sphere"] = sphere
    if mirror is not None:
        d["mirror"] = mirror
    return d


# ---------------------------------------------------------------- geometry

@pytest.mark.parametrize("ior", [1.33, 1.5, 2.4])
@pytest.mark.parametrize("b", [0.0, 0.2, 0.55, 0.9, 0.999])
def test_sphere_refraction_matches_snell_deviation(ior, b):
    """A ray at impact parameter b through a unit sphere: incidence theta_i = asin(b),
    refraction theta_t = asin(b / ior); the ray leaves deviated by 2 (theta_i - theta_t)
    towards the axis, from the far end of a chord of length 2 cos(theta_t)."""
    c = np.array([0.3, -0.2, 0.1])
    o = c + np.array([-5.0, b, 0.0])
    d = np.array([1.0, 0.0, 0.0])
    ob = oracle.object_rays(_objects(sphere=[*c, 1.0, ior]), o[None], d[None])
    ti, tt = math.asin(b), math.asin(b / ior)
    dev = 2.0 * (ti - tt)
    t_in = 5.0 - math.sqrt(1.0 - b * b)
    chord = 2.0 * math.cos(tt)
    p1 = c + np.array([-math.sqrt(1.0 - b * b), b, 0.0])
    inside = np.array([math.cos(ti - tt), -math.sin(ti - tt), 0.0])
    assert ob["kind"][0] == 2
    assert ob["t_far"][0] == pytest.approx(t_in, abs=1e-12)
    assert ob["path"][0] == pytest.approx(t_in + chord, abs=1e-9)
    np.testing.assert_allclose(ob["next_o"][0], p1 + chord * inside, atol=1e-9)
    np.testing.assert_allclose(ob["next_d"][0], [math.cos(dev), -math.sin(dev), 0.0], atol=1e-9)
    assert np.linalg.norm(ob["next_d"][0]) == pytest.approx(1.0, abs=1e-12)


def test_index_one_sphere_passes_rays_straight():
    rng = np.random.default_rng(3)
    c = np.array([0.1, 0.2, -0.3])
    o = rng.uniform(-3, 3, (200, 3))
    d = rng.normal(size=(200, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    ob = oracle.object_rays(_objects(sphere=[*c, 0.7, 1.0]), o, d)
    for r in range(200):
        f = o[r] - c
        bq = f @ d[r]
        disc = bq * bq - (f @ f - 0.49)
        roots = [-bq - math.sqrt(disc), -bq + math.sqrt(disc)] if disc >= 0 else []
        ahead = [t for t in roots if t > 1e-4]
        if not ahead:
            assert ob["kind"][r] == 0 and np.isinf(ob["t_far"][r])
            continue
        assert ob["kind"][r] == 2
        assert ob["t_far"][r] == pytest.approx(ahead[0], abs=1e-12)
        np.testing.assert_allclose(ob["next_d"][r], d[r], atol=1e-12)
        np.testing.assert_allclose(ob["next_o"][r], o[r] + roots[1] * d[r], atol=1e-9)
        assert ob["path"][r] == pytest.approx(roots[1], abs=1e-9)


@pytest.mark.parametrize("side", [1.0, -1.0])
def test_mirror_reflection_and_extent(side):
    """Law of reflection on both faces: the component along the normal flips, the
    tangential part is kept, the angle of reflection equals the angle of incidence; rays
    that meet the plane outside the rectangle, or run away from it, pass."""
    mir = [0.5, -0.25, 0.0, 0.8, 0.0, 0.0, 0.0, 0.4, 0.0]   # z = 0, x in [-0.3, 1.3], y in [-0.65, 0.15]
    o = np.array([[0.2, -0.1, 2.0 * side], [2.0, 0.0, 1.0 * side], [0.5, -0.25, 1.0 * side]])
    d = np.array([[0.3, -0.1, -1.0 * side], [0.0, 0.0, -1.0 * side], [0.0, 0.0, 1.0 * side]])
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    ob = oracle.object_rays(_objects(mirror=mir), o, d)
    t = 2.0 / abs(d[0, 2])
    assert ob["kind"].tolist() == [1, 0, 0]
    assert ob["t_far"][0] == pytest.approx(t, abs=1e-12) and ob["path"][0] == pytest.approx(t, abs=1e-12)
    np.testing.assert_allclose(ob["next_o"][0], o[0] + t * d[0], atol=1e-12)
    np.testing.assert_allclose(ob["next_d"][0], d[0] * [1, 1, -1], atol=1e-12)
    assert np.isinf(ob["t_far"][1]) and np.isinf(ob["t_far"][2])


def test_total_internal_reflection_inside_sphere():
    """Inside a sphere every chord meets the surface at the same angle. Beyond the
    critical angle asin(1/ior) the ray is reflected on every chord and ends inside
    (kind 3) after the last allowed chord; below it, it leaves with sin(out) = ior
    sin(in)."""
    ior, r = 1.5, 1.0
    crit = math.asin(1.0 / ior)
    for th, trapped in [(crit + 0.2, True), (crit - 0.3, False)]:
        # start at the centre's side: a chord through the point at distance r sin(th)
        # from the centre, heading +x, meets the surface at incidence th
        o = np.array([[0.0, r * math.sin(th), 0.0]])
        d = np.array([[1.0, 0.0, 0.0]])
        ob = oracle.object_rays(_objects(sphere=[0.0, 0.0, 0.0, r, ior]), o, d)
        t_exit = r * math.cos(th)
        assert ob["t_far"][0] == pytest.approx(t_exit, abs=1e-12)
        if trapped:
            assert ob["kind"][0] == 3
            assert ob["path"][0] == pytest.approx(t_exit + 8 * 2 * r * math.cos(th), abs=1e-9)
            assert not ob["next_d"][0].any()
        else:
            assert ob["kind"][0] == 2
            n = ob["next_o"][0] / r
            cos_out = float(ob["next_d"][0] @ n)
            assert math.sqrt(max(0.0, 1 - cos_out ** 2)) == pytest.approx(ior * math.sin(th), abs=1e-9)


def test_continuation_rays_leave_their_surface():
    """The eps rule: a continuation ray does not meet the surface it starts on again."""
    cam = inputs.orbit_camera(32, 24)
    o, d = oracle.pinhole_rays(cam)
    objs = _objects(sphere=[0.3, 0.0, 0.2, 0.5, 1.5], mirror=[-0.6, 0.5, -0.1, 0.0, 0.8, 0.5, 0.6, 0.0, 0.0])
    ob = oracle.object_rays(objs, o, d)
    assert (ob["kind"] == 1).sum() > 20 and (ob["kind"] == 2).sum() > 20
    sel = ob["kind"] == 1
    again = oracle.object_rays(_objects(mirror=objs["mirror"]), ob["next_o"][sel], ob["next_d"][sel])
    assert (again["kind"] == 0).all()
    sel = ob["kind"] == 2
    again = oracle.object_rays(_objects(sphere=objs["sphere"]), ob["next_o"][sel], ob["next_d"][sel])
    assert (again["kind"] == 0).all()


# ---------------------------------------------------------------- bounded rays, starting transmittance

@pytest.mark.parametrize("o,n,m", [(0.5, 12, 3), (0.3, 30, 17), (0.9, 6, 0)])
def test_bounded_stack_of_slabs(o, n, m):
    """n identical Gaussians along the ray; a surface just after the m-th entry: exactly
    m are blended (T = (1-o)^m) and the background stays hidden."""
    sig = 0.01
    o32 = float(np.float32(o))
    rho = rho_of(o32, AMIN)
    gap = 2.5 * rho * sig
    means = [[1.0 + i * gap, 0.0, 0.0] for i in range(n)]
    rgb = [0.2, 0.6, 0.9]
    sc = make_scene(means, [sig] * 3, opac=o, rgb=rgb)
    entries = [1.0 + i * gap - rho * float(np.float32(sig)) for i in range(n)]
    t_far = entries[m] - 1e-6 if m < n else 100.0
    r = oracle.render(sc, np.zeros((1, 3)), [[1, 0, 0]], AMIN, 1e-6, bg=(1.0, 1.0, 1.0), t_far=[t_far])
    c = dc_colour(rgb)
    assert r["nblend"][0] == m
    assert 1 - r["opacity"][0] == pytest.approx((1 - o32) ** m, rel=1e-12)
    np.testing.assert_allclose(r["rgb"][0], c * (1 - (1 - o32) ** m), rtol=1e-12, atol=1e-15)


@pytest.mark.parametrize("tau", [1.0, 0.5, 0.02, 1.5e-3])
def test_starting_transmittance_scales_and_shortens(tau):
    """A ray that starts with transmittance tau: every weight scales by tau and early
    termination comes after the first n with tau (1-o)^n < T_min."""
    o, n, T_min = 0.4, 40, 1e-3
    sig = 0.01
    o32 = float(np.float32(o))
    rho = rho_of(o32, AMIN)
    means = [[1.0 + i * 2.5 * rho * sig, 0.0, 0.0] for i in range(n)]
    sc = make_scene(means, [sig] * 3, opac=o, rgb=[0.7, 0.1, 0.4])
    r = oracle.render(sc, np.zeros((1, 3)), [[1, 0, 0]], AMIN, T_min, trans0=[tau])
    nstar = next(k for k in range(1, n + 1) if tau * (1 - o32) ** k < T_min)
    assert r["nblend"][0] == nstar
    assert 1 - r["opacity"][0] == pytest.approx(tau * (1 - o32) ** nstar, rel=1e-12)
    np.testing.assert_allclose(r["rgb"][0], tau * dc_colour([0.7, 0.1, 0.4]) * (1 - (1 - o32) ** nstar), rtol=1e-12)


def test_bound_applies_to_the_proxy_key():
    """The surface bound compares the key that orders the hits: in proxy-key mode the
    icosahedron entry, which precedes the ellipsoid entry. A ray through the centre of one
    Gaussian bounded between the two entries blends it with the proxy key only."""
    sig, o = 0.05, 0.8
    sc = make_scene([[2.0, 0.0, 0.0]], [sig] * 3, opac=o, rgb=[0.9, 0.2, 0.1])
    ray_o, ray_d = np.zeros((1, 3)), np.array([[1.0, 0.0, 0.0]])
    hp = oracle.ray_hits(sc, ray_o[0], ray_d[0], AMIN, key_mode=1)
    hs = oracle.ray_hits(sc, ray_o[0], ray_d[0], AMIN, key_mode=0)
    t_proxy, t_sphere = float(hp["t"][0]), float(hs["t"][0])
    rho = rho_of(float(np.float32(o)), AMIN) * float(np.float32(sig))
    assert t_sphere == pytest.approx(2.0 - rho, abs=1e-9) and t_proxy < t_sphere - 1e-4
    t_far = [0.5 * (t_proxy + t_sphere)]
    rp = oracle.render(sc, ray_o, ray_d, AMIN, key_mode=1, t_far=t_far, cap=2)
    rs = oracle.render(sc, ray_o, ray_d, AMIN, key_mode=0, t_far=t_far, cap=2)
    assert rp["nblend"][0] == 1 and rs["nblend"][0] == 0
    assert rp["opacity"][0] == pytest.approx(float(np.float32(o)), rel=1e-12)


# ---------------------------------------------------------------- identities of the whole chain

def _scene_above_plane(seed, n, zmin):
    rng = np.random.default_rng(seed)
    means = np.column_stack([rng.uniform(-1.5, 1.5, n), rng.uniform(-1.5, 1.5, n), rng.uniform(0.35, 1.6, n)])
    scales = np.exp(rng.normal(-3.5, 0.4, (n, 3)))
    quats = rng.normal(size=(n, 4))
    opac = 1 / (1 + np.exp(-rng.normal(0, 1.5, n)))
    sh = rng.normal(0, 0.3, (n, 16, 3))
    sc = make_scene(means, scales, quats, opac, sh=sh, sh_degree=3)
    lo, _, _ = oracle.gaussian_aabb(sc, AMIN)
    keep = lo[:, 2] > zmin
    return inputs.Scene(sc.means[keep].copy(), sc.scales[keep].copy(), sc.quats[keep].copy(),
                        sc.opacities[keep].copy(), sc.sh[keep].copy(), 3)


def test_mirror_equals_reflected_scene_seen_straight():
    """Unfolding: a ray reflected by the plane z = 0 sees what the straight ray sees in
    the scene reflected through that plane. With every Gaussian above the plane, the
    two-segment render (primary ray bounded by the mirror, continuation from the mirror
    with the remaining transmittance) equals a plain render of the scene plus its mirror
    image: colour, depth along the bent path, opacity and background."""
    sc = _scene_above_plane(21, 400, 0.02)
    n = sc.n
    # reflection H = diag(1, 1, -1): mean z -> -z; rotation R -> H R H, which is the
    # quaternion (w, -x, -y, z); real SH Y_lm(x, y, -z) = (-1)^(l+m) Y_lm(x, y, z)
    H = np.diag([1.0, 1.0, -1.0])
    q2 = sc.quats * np.array([1, -1, -1, 1], np.float32)
    for i in range(0, n, 37):
        np.testing.assert_allclose(quat_to_matrix_scipy(q2[i]), H @ quat_to_matrix_scipy(sc.quats[i]) @ H, atol=1e-6)
    parity = np.array([(-1.0) ** (l + m) for l in range(4) for m in range(-l, l + 1)], np.float32)
    v = np.array([0.3, -0.5, 0.7])
    v /= np.linalg.norm(v)
    for l in range(4):
        for m in range(-l, l + 1):
            assert oracle.sh_basis(l, m, v * [1, 1, -1]) == pytest.approx(parity[l * l + l + m] * oracle.sh_basis(l, m, v),
                                                                          abs=1e-14)
    refl = inputs.Scene(sc.means * np.array([1, 1, -1], np.float32), sc.scales.copy(), q2,
                        sc.opacities.copy(), sc.sh * parity[None, :, None], 3)
    both = inputs.Scene(np.concatenate([sc.means, refl.means]), np.concatenate([sc.scales, refl.scales]),
                        np.concatenate([sc.quats, refl.quats]), np.concatenate([sc.opacities, refl.opacities]),
                        np.concatenate([sc.sh, refl.sh]), 3)
    cam = inputs.Camera((0.0, -3.0, 1.5), (0.0, 0.0, 0.0), (0.0, 0.0, 1.0), 40.0, 24, 16)
    o, d = oracle.pinhole_rays(cam)
    assert (d[:, 2] < -0.1).all()  # every ray meets the plane inside the mirror
    mirror = [0.0, 0.0, 0.0, 50.0, 0.0, 0.0, 0.0, 50.0, 0.0]
    bg = (0.2, 0.3, 0.4)
    lv = []
    two = oracle.render_with_objects(sc, o, d, _objects(mirror=mirror), bounces=1, bg=bg, levels=lv)
    one = oracle.render(both, o, d, AMIN, 1e-3, bg=bg)
    assert (lv[0]["objects"]["kind"] == 1).all() and len(lv) == 2
    assert lv[1]["out"]["nblend"].sum() > 100 and lv[0]["out"]["nblend"].sum() > 100
    np.testing.assert_allclose(two["rgb"], one["rgb"], atol=1e-10)
    np.testing.assert_allclose(two["depth"], one["depth"], atol=1e-9)
    np.testing.assert_allclose(two["opacity"], one["opacity"], atol=1e-12)


def test_index_one_glass_in_empty_space_is_invisible():
    """A glass sphere of index 1 that no Gaussian reaches changes nothing: the primary
    segment ends at the entry point, the continuation starts at the exit point with the
    same direction and transmittance, and their sum is the plain render."""
    sc0 = inputs.small_scene(1, 1000)
    c, rad = np.array([0.1, -0.2, 0.2]), 0.45
    lo, hi, _ = oracle.gaussian_aabb(sc0, AMIN)
    gap = np.linalg.norm(np.maximum(np.maximum(lo - c, c - hi), 0.0), axis=1)
    keep = gap > rad + 1e-3
    sc = inputs.Scene(sc0.means[keep].copy(), sc0.scales[keep].copy(), sc0.quats[keep].copy(),
                      sc0.opacities[keep].copy(), sc0.sh[keep].copy(), sc0.sh_degree)
    o, d = oracle.pinhole_rays(inputs.orbit_camera(32, 32))
    bg = (0.1, 0.5, 0.9)
    lv = []
    two = oracle.render_with_objects(sc, o, d, _objects(sphere=[*c, rad, 1.0]), bounces=1, bg=bg, levels=lv)
    one = oracle.render(sc, o, d, AMIN, 1e-3, bg=bg)
    through = lv[0]["objects"]["kind"] == 2
    assert through.sum() > 50
    np.testing.assert_allclose(two["rgb"], one["rgb"], atol=1e-12)
    np.testing.assert_allclose(two["depth"], one["depth"], atol=1e-10)
    np.testing.assert_allclose(two["opacity"], one["opacity"], atol=1e-12)


def test_second_bounce_chain():
    """Two bounces: mirror then glass. Each level's continuation rays are the previous
    level's object rays (kind 1 or 2 with T >= T_min), and a ray that meets no second
    object ends unbounded, as with one bounce."""
    sc = inputs.small_scene(1, 1000)
    # a mirror at 45 degrees sends the camera's rays along +x, into the glass sphere
    objs = _objects(sphere=[0.9, 0.45, 0.0, 0.35, 1.5], mirror=[-0.4, 0.45, 0.0, 0.5, 0.5, 0.0, 0.0, 0.0, 0.6])
    o, d = oracle.pinhole_rays(inputs.orbit_camera(48, 48))
    lv1, lv2 = [], []
    one = oracle.render_with_objects(sc, o, d, objs, bounces=1, levels=lv1)
    two = oracle.render_with_objects(sc, o, d, objs, bounces=2, levels=lv2)
    assert len(lv2) == 3
    ob2 = lv2[1]["objects"]
    multi = np.isin(ob2["kind"], (1, 2, 3))
    assert multi.sum() > 0
    # rays whose continuation meets no further object render identically
    T1 = 1 - lv1[0]["out"]["opacity"]
    cont = np.flatnonzero(np.isin(lv1[0]["objects"]["kind"], (1, 2)) & (T1 >= 1e-3))
    same = np.ones(o.shape[0], bool)
    same[cont[multi]] = False
    np.testing.assert_allclose(two["rgb"][same], one["rgb"][same], atol=1e-12)
    assert np.abs(two["rgb"][~same] - one["rgb"][~same]).max() > 1e-3
