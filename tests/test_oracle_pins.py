"""Pins for the FP64 oracle: closed forms, invariants, brute force and the paper's worked
example. None of these re-types the oracle's own formulas; each checks a consequence
that a dropped term, a wrong sign or index, or a transposed operand would break."""
import math

import numpy as np
import pytest

import oracle
from paper_2601_20429_amd import inputs
from tests.helpers import Y00, dc_colour, load_golden, make_scene, quat_to_matrix_scipy, rho_of, walkthrough_scene

AMIN = 1.0 / 255.0


# ---------------------------------------------------------------- Eq. 2 closed forms

@pytest.mark.parametrize("o,sigma,dist", [(0.5, 0.05, 2.0), (0.9, 0.2, 3.5), (0.02, 0.01, 1.25)])
def test_isotropic_ray_through_centre(o, sigma, dist):
    """Ray through the centre of an isotropic Gaussian: alpha = o, t_alpha = |mu - o|,
    entry t0 = t_alpha - rho*sigma."""
    sc = make_scene([[0.0, dist, 0.0]], [sigma] * 3, opac=o, rgb=[0.25, 0.5, 0.75])
    h = oracle.ray_hits(sc, [0, 0, 0], [0, 1, 0], AMIN)
    o32, s32 = float(np.float32(o)), float(np.float32(sigma))
    d32 = float(np.float32(dist))
    assert h["ids"].tolist() == [0]
    assert h["alpha"][0] == pytest.approx(o32, rel=1e-12)
    assert h["talpha"][0] == pytest.approx(d32, rel=1e-12)
    assert h["t"][0] == pytest.approx(d32 - rho_of(o32, AMIN) * s32, rel=1e-12)
    r = oracle.render(sc, np.zeros((1, 3)), [[0, 1, 0]], AMIN)
    c = dc_colour(np.float32([0.25, 0.5, 0.75]).astype(np.float64))
    np.testing.assert_allclose(r["rgb"][0], o32 * c, rtol=1e-12)
    assert r["depth"][0] == pytest.approx(o32 * d32, rel=1e-12)
    assert r["opacity"][0] == pytest.approx(o32, rel=1e-12)


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_offset_along_principal_axis(axis):
    """A ray along principal axis k, offset by b along principal axis j != k:
    alpha = o exp(-b^2 / (2 s_j^2)); a hit iff b <= rho s_j."""
    rng = np.random.default_rng(11 + axis)
    q = rng.standard_normal(4)
    q /= np.linalg.norm(q)
    q32 = q.astype(np.float32)
    R = quat_to_matrix_scipy(q32.astype(np.float64) / np.linalg.norm(q32.astype(np.float64)))
    s = np.float32([0.03, 0.08, 0.15]).astype(np.float64)
    o = float(np.float32(0.7))
    mu = np.array([0.2, -0.1, 0.3])
    j, k = axis, (axis + 1) % 3
    rho = rho_of(o, AMIN)
    ej, ek = R[:, j], R[:, k]
    for frac in [0.0, 0.3, 0.9, 0.999, 1.001, 1.5]:
        b = frac * rho * s[j]
        origin = mu + b * ej - 4.0 * ek
        sc = make_scene([mu], s, quats=q32, opac=o)
        o32 = origin.astype(np.float32).astype(np.float64)
        d32 = ek.astype(np.float32).astype(np.float64)
        h = oracle.ray_hits(sc, o32, d32, AMIN)
        # exact offset of the float32 ray from the float32 centre along e_j
        mu32 = np.float32(mu).astype(np.float64)
        dvec = d32 / np.linalg.norm(d32)
        rel = mu32 - o32
        perp = rel - np.dot(rel, dvec) * dvec
        # Mahalanobis distance^2 of the closest approach = sum_j (perp.e_j / s_j)^2 for
        # a direction exactly along e_k; the float32 direction is within 1e-7 of it
        m2 = sum((np.dot(perp, R[:, a]) / s[a]) ** 2 for a in range(3) if a != k)
        if frac < 0.99:
            assert h["ids"].tolist() == [0]
            assert h["alpha"][0] == pytest.approx(o * math.exp(-0.5 * m2), rel=1e-5)
            assert h["alpha"][0] == pytest.approx(o * math.exp(-0.5 * (b / s[j]) ** 2), rel=1e-4)
        elif frac > 1.0:
            assert h["ids"].size == 0


def test_talpha_is_argmax_of_response():
    """t_alpha of Eq. 2 is where o*G(o + t d) peaks along the ray: compare with a dense
    sampling plus golden-section refinement of the response, with G built from scipy's
    rotation of the quaternion (an independent route to Sigma)."""
    rng = np.random.default_rng(3)
    for trial in range(20):
        q = rng.standard_normal(4).astype(np.float32)
        s = np.exp(rng.normal(-1.5, 0.5, 3)).astype(np.float32)
        mu = rng.uniform(-0.5, 0.5, 3).astype(np.float32)
        o = np.float32(rng.uniform(0.2, 0.99))
        origin = np.float32([0.0, -3.0, 0.0]) + rng.uniform(-0.05, 0.05, 3).astype(np.float32)
        d = (mu - origin) + rng.normal(0, 0.05, 3)
        d = (d / np.linalg.norm(d)).astype(np.float32)
        sc = make_scene([mu], s, quats=q, opac=o)
        h = oracle.ray_hits(sc, origin, d, AMIN)
        R = quat_to_matrix_scipy(q.astype(np.float64) / np.linalg.norm(q.astype(np.float64)))
        Sig = R @ np.diag(s.astype(np.float64) ** 2) @ R.T
        Si = np.linalg.inv(Sig)
        od, dd, md = origin.astype(np.float64), d.astype(np.float64), mu.astype(np.float64)

        def resp(t):
            x = od + t * dd - md
            return float(o) * math.exp(-0.5 * x @ Si @ x)

        ts = np.linspace(0.0, 6.0, 60001)
        vals = np.array([resp(t) for t in ts])
        i = int(np.argmax(vals))
        a, b = ts[max(i - 1, 0)], ts[min(i + 1, len(ts) - 1)]
        g = (math.sqrt(5) - 1) / 2
        for _ in range(200):
            c1, c2 = b - g * (b - a), a + g * (b - a)
            if resp(c1) > resp(c2):
                b = c2
            else:
                a = c1
        tstar = 0.5 * (a + b)
        if h["ids"].size:
            assert h["talpha"][0] == pytest.approx(tstar, abs=1e-7)
            assert h["alpha"][0] == pytest.approx(resp(tstar), rel=1e-9)
            assert resp(tstar) >= AMIN * (1 - 1e-9)
        else:
            assert resp(tstar) < AMIN * (1 + 1e-9)


def test_hit_iff_peak_alpha_reaches_threshold():
    """The bounding ellipsoid is the alpha_min level set: a ray (starting outside every
    ellipsoid) hits a Gaussian exactly when its peak alpha along the ray is >= alpha_min."""
    sc = inputs.small_scene(1, 300)
    rng = np.random.default_rng(5)
    eye = np.float32([0.0, -4.0, 0.0])
    for r in range(40):
        tgt = rng.uniform(-1, 1, 3)
        d = ((tgt - eye) / np.linalg.norm(tgt - eye)).astype(np.float32)
        h = oracle.ray_hits(sc, eye, d, AMIN)
        hit = set(h["ids"].tolist())
        for i in range(sc.n):
            a = oracle.composite_list(sc, eye, d, [i], AMIN)["opacity"]
            if abs(a - AMIN) < 1e-9:
                continue
            assert (i in hit) == (a >= AMIN), (r, i, a)


# ---------------------------------------------------------------- Eq. 1 + early termination

@pytest.mark.parametrize("o,n", [(0.5, 4), (0.5, 20), (0.3, 30), (0.95, 5), (0.1, 80)])
def test_stacked_identical_slabs(o, n):
    """n identical Gaussians along the ray with disjoint supports, ray through their
    centres: alpha = o each; T after m hits = (1-o)^m; early termination after
    n* = ceil(ln T_min / ln(1-o)) hits; C = c (1 - (1-o)^min(n, n*))."""
    T_min = 1e-3
    sig = 0.01
    o32 = float(np.float32(o))
    rho = rho_of(o32, AMIN)
    gap = 2.5 * rho * sig
    means = [[1.0 + i * gap, 0.0, 0.0] for i in range(n)]
    rgb = [0.2, 0.6, 0.9]
    sc = make_scene(means, [sig] * 3, opac=o, rgb=rgb)
    r = oracle.render(sc, np.zeros((1, 3)), [[1, 0, 0]], AMIN, T_min, cap=n)
    nstar = math.ceil(math.log(T_min) / math.log(1 - o32))
    m = min(n, nstar)
    c = dc_colour(rgb)
    assert r["nblend"][0] == m
    assert r["opacity"][0] == pytest.approx(1 - (1 - o32) ** m, rel=1e-12)
    np.testing.assert_allclose(r["rgb"][0], c * (1 - (1 - o32) ** m), rtol=1e-12)
    np.testing.assert_allclose(r["tafter"][0, :m], (1 - o32) ** np.arange(1, m + 1), rtol=1e-12)
    assert r["ids"][0, :m].tolist() == list(range(m))


def test_background_and_empty():
    sc = make_scene([[0.0, 5.0, 0.0]], [0.1] * 3, opac=0.5)
    r = oracle.render(sc, np.zeros((2, 3)), [[1, 0, 0], [0, 1, 0]], AMIN, bg=(0.1, 0.2, 0.3))
    np.testing.assert_allclose(r["rgb"][0], [0.1, 0.2, 0.3], rtol=0, atol=0)
    assert r["opacity"][0] == 0.0 and r["depth"][0] == 0.0
    o32 = float(np.float32(0.5))
    np.testing.assert_allclose(r["rgb"][1], o32 * 0.5 + (1 - o32) * np.array([0.1, 0.2, 0.3]), rtol=1e-12)


def test_inactive_and_behind():
    """o <= alpha_min is never hit; a Gaussian behind the origin, or one containing the
    origin, is not a hit (front-face rule)."""
    means = [[0.0, 2.0, 0.0], [0.0, -2.0, 0.0], [0.0, 0.0, 0.0], [0.0, 3.0, 0.0]]
    sc = make_scene(means, [0.1] * 3, opac=[0.5, 0.5, 0.5, 0.5 * AMIN])
    h = oracle.ray_hits(sc, [0, 0, 0], [0, 1, 0], AMIN)
    assert h["ids"].tolist() == [0]


def test_ties_sorted_by_index():
    """Identical Gaussians have identical distance; they are ordered by index."""
    means = [[0.0, 2.0, 0.0]] * 3 + [[0.0, 1.0, 0.0]]
    sc = make_scene(means, [0.05] * 3, opac=[0.4, 0.4, 0.4, 0.2], rgb=[[0.1, 0, 0], [0, 0.2, 0], [0, 0, 0.3], [1, 1, 1]])
    h = oracle.ray_hits(sc, [0, 0, 0], [0, 1, 0], AMIN)
    assert h["ids"].tolist() == [3, 0, 1, 2]
    assert h["t"][1] == h["t"][2] == h["t"][3]


def test_composite_list_reproduces_render():
    sc = inputs.cluster_scene(8, 2000, 3)
    cam = inputs.orbit_camera(24, 24)
    o, d = oracle.pinhole_rays(cam)
    r = oracle.render(sc, o, d, AMIN, 1e-3, cap=512)
    for i in range(0, o.shape[0], 37):
        nb = r["nblend"][i]
        c = oracle.composite_list(sc, o[i], d[i], r["ids"][i, :nb], AMIN)
        np.testing.assert_allclose(c["rgb"], r["rgb"][i], rtol=1e-12, atol=1e-15)
        assert c["depth"] == pytest.approx(r["depth"][i], rel=1e-12, abs=1e-15)


# ---------------------------------------------------------------- spherical harmonics

def _sphere_quadrature(nt=24, nph=48):
    x, w = np.polynomial.legendre.leggauss(nt)
    ph = (np.arange(nph) + 0.5) * 2 * np.pi / nph
    pts, wts = [], []
    for xi, wi in zip(x, w):
        st = math.sqrt(1 - xi * xi)
        for p in ph:
            pts.append([st * math.cos(p), st * math.sin(p), xi])
            wts.append(wi * 2 * np.pi / nph)
    return np.array(pts), np.array(wts)


def test_sh_orthonormal():
    pts, wts = _sphere_quadrature()
    lm = [(l, m) for l in range(4) for m in range(-l, l + 1)]
    Y = np.array([[oracle.sh_basis(l, m, p) for p in pts] for (l, m) in lm])
    G = (Y * wts) @ Y.T
    np.testing.assert_allclose(G, np.eye(len(lm)), atol=1e-10)


def test_sh_known_values():
    """Band 0 is constant; band 1 is proportional to (y, z, x) with the Condon-Shortley
    sign (-, +, -) for m = (-1, 0, 1)."""
    c1 = math.sqrt(3 / (4 * math.pi))
    rng = np.random.default_rng(2)
    for _ in range(10):
        v = rng.standard_normal(3)
        v /= np.linalg.norm(v)
        assert oracle.sh_basis(0, 0, v) == pytest.approx(1 / (2 * math.sqrt(math.pi)), rel=1e-14)
        assert oracle.sh_basis(1, -1, v) == pytest.approx(-c1 * v[1], abs=1e-14)
        assert oracle.sh_basis(1, 0, v) == pytest.approx(c1 * v[2], abs=1e-14)
        assert oracle.sh_basis(1, 1, v) == pytest.approx(-c1 * v[0], abs=1e-14)
    # zonal harmonic at the pole: Y_l0(z) = sqrt((2l+1)/4pi)
    for l in range(4):
        assert oracle.sh_basis(l, 0, [0, 0, 1]) == pytest.approx(math.sqrt((2 * l + 1) / (4 * math.pi)), rel=1e-14)


def test_view_dependent_colour_uses_ray_direction():
    """A degree-1 coefficient on Y_1,0 changes colour with the z component of the ray
    direction only (Sec. III-A: colour from SH and ray direction)."""
    sh = np.zeros((1, 4, 3))
    sh[0, 2, :] = [0.3, 0.3, 0.3]
    sc = make_scene([[0.0, 0.0, 0.0]], [0.2] * 3, opac=0.5, sh=sh, sh_degree=1)
    c1 = math.sqrt(3 / (4 * math.pi))
    for dz in [-0.6, 0.0, 0.6]:
        d = np.array([0.0, math.sqrt(1 - dz * dz), dz])
        o = -3.0 * d
        r = oracle.render(sc, o[None], d[None], AMIN)
        dd = d / np.linalg.norm(d)
        want = max(0.0, 0.5 + c1 * dd[2] * float(np.float32(0.3)))
        assert r["rgb"][0, 0] / r["opacity"][0] == pytest.approx(want, rel=1e-9)


# ---------------------------------------------------------------- camera and rotation

def test_pinhole_geometry():
    cam = inputs.orbit_camera(33, 21, eye=(0.0, -3.0, 0.0), fov_y_deg=60.0)
    o, d = oracle.pinhole_rays(cam)
    np.testing.assert_allclose(np.linalg.norm(d, axis=1), 1.0, rtol=1e-14)
    np.testing.assert_allclose(o, np.tile([0.0, -3.0, 0.0], (o.shape[0], 1)))
    centre = 10 * 33 + 16
    np.testing.assert_allclose(d[centre], [0, 1, 0], atol=1e-15)
    top = 0 * 33 + 16
    ang = math.atan2(d[top][2], d[top][1])
    assert math.tan(ang) == pytest.approx((1 - 1 / 21) * math.tan(math.radians(30)), rel=1e-12)
    right = 10 * 33 + 32
    assert d[right][0] > 0 and abs(d[right][2]) < 1e-15
    assert math.tan(math.atan2(d[right][0], d[right][1])) == pytest.approx(
        (1 - 1 / 33) * math.tan(math.radians(30)) * 33 / 21, rel=1e-12)


def test_aabb_and_quaternion_convention():
    """Identity rotation: half-extent rho*s per axis. A 90-degree turn about z swaps the
    x and y extents. Quaternions need not be normalised."""
    s = [0.1, 0.02, 0.05]
    c = math.cos(math.pi / 4)
    sc = make_scene([[0, 0, 0]] * 3, s, quats=[[1, 0, 0, 0], [c, 0, 0, c], [2 * c, 0, 0, 2 * c]], opac=0.6)
    lo, hi, act = oracle.gaussian_aabb(sc, AMIN)
    rho = rho_of(float(np.float32(0.6)), AMIN)
    s32 = np.float32(s).astype(np.float64)
    np.testing.assert_allclose(hi[0], rho * s32, rtol=1e-12)
    np.testing.assert_allclose(hi[1], rho * s32[[1, 0, 2]], rtol=1e-6)
    np.testing.assert_allclose(hi[2], hi[1], rtol=1e-12)
    np.testing.assert_allclose(lo, -hi)
    assert act.all()


def test_aabb_contains_ellipsoid_samples():
    sc = inputs.cluster_scene(9, 200, 0)
    lo, hi, act = oracle.gaussian_aabb(sc, AMIN)
    rng = np.random.default_rng(1)
    for i in range(sc.n):
        if not act[i]:
            continue
        R = quat_to_matrix_scipy(sc.quats[i].astype(np.float64) / np.linalg.norm(sc.quats[i].astype(np.float64)))
        rho = rho_of(float(sc.opacities[i]), AMIN)
        u = rng.standard_normal((64, 3))
        u /= np.linalg.norm(u, axis=1, keepdims=True)
        x = sc.means[i].astype(np.float64) + (u * sc.scales[i].astype(np.float64) * rho) @ R.T
        assert (x >= lo[i] - 1e-12).all() and (x <= hi[i] + 1e-12).all()
        # tight: the extreme sample along each axis comes close to the box
        assert ((x.max(0) - hi[i]) > -0.5 * (hi[i] - lo[i])).all()


# ---------------------------------------------------------------- worked example

def test_walkthrough_order():
    """Sec. IV-B walkthrough: hits along the ray come in distance order, with primitive
    33 at t = 2.85 immediately before primitive 5 at t = 3.2."""
    sc, g = walkthrough_scene()
    h = oracle.ray_hits(sc, g["ray"]["origin"], g["ray"]["direction"], g["alpha_min"])
    assert h["ids"].tolist() == g["expected_blend_order"]
    want_t = [e["t_entry"] for e in g["on_ray"]]
    np.testing.assert_allclose(h["t"], want_t, atol=2e-6)
    pv = g["paper_values"]
    i33 = h["ids"].tolist().index(pv["farthest_in_kbuffer"]["id"])
    assert h["t"][i33] == pytest.approx(pv["farthest_in_kbuffer"]["t_hit"], abs=2e-6)
    assert h["ids"][i33 + 1] == pv["rejected_hit"]["id"]
    assert h["t"][i33 + 1] == pytest.approx(pv["rejected_hit"]["t_hit"], abs=2e-6)
    assert i33 + 1 == pv["k"]  # the rejected hit is the (k+1)-th closest
    r = oracle.render(sc, np.float32([g["ray"]["origin"]]), np.float32([g["ray"]["direction"]]),
                      g["alpha_min"], g["T_min"], cap=8)
    o32 = float(np.float32(g["opacity"]))
    assert r["nblend"][0] == 6
    cols = {e["id"]: np.asarray(e["rgb"], np.float64) for e in g["on_ray"]}
    want = sum(o32 * (1 - o32) ** j * dc_colour(cols[i]) for j, i in enumerate(g["expected_blend_order"]))
    np.testing.assert_allclose(r["rgb"][0], want, rtol=1e-12)


# ---------------------------------------------------------------- proxy mesh

def test_icosahedron_is_regular_with_unit_inradius():
    v, f = oracle.icosahedron()
    assert len({tuple(sorted(x)) for x in f.tolist()}) == 20
    edges = {tuple(sorted((a, b))) for tri in f.tolist() for a, b in [(tri[0], tri[1]), (tri[1], tri[2]), (tri[2], tri[0])]}
    assert len(edges) == 30  # V - E + F = 2
    L = [np.linalg.norm(v[a] - v[b]) for a, b in edges]
    np.testing.assert_allclose(L, L[0], rtol=1e-12)
    for tri in f:
        a, b, c = v[tri]
        n = np.cross(b - a, c - a)
        n /= np.linalg.norm(n)
        assert n @ a == pytest.approx(1.0, rel=1e-12)  # outward, at distance 1
    # circumradius / inradius of the regular icosahedron
    np.testing.assert_allclose(np.linalg.norm(v, axis=1), math.sqrt(15 - 6 * math.sqrt(5)), rtol=1e-12)


def test_proxy_key_bounds_sphere_key():
    """The icosahedron contains the bounding ellipsoid: its entry distance is <= the
    ellipsoid's, equal along a face normal through the centre, and smaller by
    rho*sigma*(R/r - 1) along a vertex direction."""
    sc = inputs.cluster_scene(12, 300, 0)
    rng = np.random.default_rng(4)
    for _ in range(20):
        eye = np.float32([0, -3.5, 0])
        tgt = sc.means[rng.integers(sc.n)]
        d = ((tgt - eye) / np.linalg.norm(tgt - eye)).astype(np.float32)
        hs = oracle.ray_hits(sc, eye, d, AMIN, key_mode=0)
        hp = oracle.ray_hits(sc, eye, d, AMIN, key_mode=1)
        assert set(hs["ids"].tolist()) == set(hp["ids"].tolist())
        ts = dict(zip(hs["ids"].tolist(), hs["t"]))
        for i, t in zip(hp["ids"].tolist(), hp["t"]):
            assert t <= ts[i] + 1e-12
    v, f = oracle.icosahedron()
    sig, o = 0.1, 0.5
    rho = rho_of(float(np.float32(o)), AMIN)
    s32 = float(np.float32(sig))
    a, b, c = v[f[0]]
    nrm = np.cross(b - a, c - a)
    nrm /= np.linalg.norm(nrm)
    one = make_scene([[0, 0, 0]], [sig] * 3, opac=o)
    for direction, extra in [(-nrm, 1.0), (-v[0] / np.linalg.norm(v[0]), np.linalg.norm(v[0]))]:
        d = direction.astype(np.float32)
        eye = (-3.0 * d).astype(np.float32)
        hp = oracle.ray_hits(one, eye, d, AMIN, key_mode=1)
        ta = oracle.ray_hits(one, eye, d, AMIN, key_mode=0)["talpha"][0]
        assert hp["t"][0] == pytest.approx(ta - extra * rho * s32, abs=1e-6)


# ---------------------------------------------------------------- LBVH reference

def _deinterleave(code):
    q = [0, 0, 0]
    for b in range(21):
        q[0] |= ((code >> (3 * b + 2)) & 1) << b
        q[1] |= ((code >> (3 * b + 1)) & 1) << b
        q[2] |= ((code >> (3 * b)) & 1) << b
    return q


def test_morton_quantisation():
    rng = np.random.default_rng(0)
    m = rng.uniform(-2, 3, (500, 3)).astype(np.float32)
    codes = oracle.morton(m)
    lo, hi = m.min(0).astype(np.float64), m.max(0).astype(np.float64)
    for i in range(m.shape[0]):
        q = _deinterleave(int(codes[i]))
        exact = (m[i].astype(np.float64) - lo) / (hi - lo) * 2 ** 21
        for a in range(3):
            # binary32 steps: ulp(mu - lo) * scale + ulp(product) stays below 2 units
            assert abs(q[a] - min(exact[a], 2 ** 21 - 1)) <= 2.0
    # extremes: the corner points map to all-zero / all-one coordinates
    m2 = np.float32([[0, 0, 0], [1, 2, 3], [0.5, 1, 1.5]])
    c2 = oracle.morton(m2)
    assert int(c2[0]) == 0 and int(c2[1]) == 2 ** 63 - 1
    assert _deinterleave(int(c2[2])) == [2 ** 20] * 3
    # only x varies -> only bits 3b+2 are used, in x order
    m3 = np.zeros((50, 3), np.float32)
    m3[:, 0] = rng.uniform(0, 1, 50)
    c3 = oracle.morton(m3)
    assert all((int(c) & ~sum(1 << (3 * b + 2) for b in range(21))) == 0 for c in c3)
    assert (np.argsort(c3, kind="stable") == np.argsort(m3[:, 0], kind="stable")).all()


def _check_radix_tree(codes, perm, child, parent, n):
    """Structural check of a binary radix tree with internal node i numbered by one of its
    range endpoints, using Python integers for the 95-bit keys (code, position)."""
    keys = [(int(codes[i]) << 32) | i for i in range(n)]
    assert all(keys[i] < keys[i + 1] for i in range(n - 1))
    rng_of = {}

    def walk(ref):
        if ref & 0x80000000:
            p = ref & 0x7FFFFFFF
            return p, p
        a0, a1 = walk(int(child[ref, 0]))
        b0, b1 = walk(int(child[ref, 1]))
        assert a1 + 1 == b0
        first, last = a0, b1
        assert ref in (first, last)
        hb = (keys[first] ^ keys[last]).bit_length() - 1
        assert all(((keys[i] >> hb) & 1) == 0 for i in range(first, a1 + 1))
        assert all(((keys[i] >> hb) & 1) == 1 for i in range(b0, last + 1))
        rng_of[ref] = (first, last)
        return first, last

    if n == 1:
        return
    assert walk(0) == (0, n - 1)
    assert len(rng_of) == n - 1
    for i in range(n - 1):
        for c in child[i]:
            c = int(c)
            idx = (n - 1 + (c & 0x7FFFFFFF)) if c & 0x80000000 else c
            assert parent[idx] == i
    assert parent[0] == 0xFFFFFFFF


@pytest.mark.parametrize("n,dup", [(1, False), (2, False), (3, False), (17, False), (300, False), (64, True), (257, True)])
def test_lbvh_reference_topology(n, dup):
    rng = np.random.default_rng(n)
    m = rng.uniform(-1, 1, (n, 3)).astype(np.float32)
    if dup:
        m[::3] = m[0]  # many equal codes: split by position
    t = oracle.lbvh_topology(m)
    codes = oracle.morton(m)
    assert (t["perm"] == np.argsort(codes, kind="stable")).all()
    assert (t["codes"] == codes[t["perm"]]).all()
    _check_radix_tree(t["codes"], t["perm"], t["child"], t["parent"], n)


@pytest.mark.parametrize("n,dup", [(2, False), (3, False), (100, False), (1000, False), (4000, False), (257, True),
                                   (3000, True)])
def test_lbvh_bisection_equals_linear_split_search(n, dup):
    """The oracle's split search by bisection (used at the 1.1M and 3M sizes) gives exactly
    the tree of the linear search over each key range (the definition as written)."""
    rng = np.random.default_rng(1000 + n)
    m = rng.uniform(-1, 1, (n, 3)).astype(np.float32)
    if dup:
        m[::3] = m[0]
        m[1::7] = m[1]
    a = oracle.lbvh_topology(m, linear=True)
    b = oracle.lbvh_topology(m)
    for key in ("codes", "perm", "child", "parent"):
        assert np.array_equal(a[key], b[key]), key
    _check_radix_tree(b["codes"], b["perm"], b["child"], b["parent"], n)


def test_oracle_finite_difference_matches_closed_form_gradient():
    """Central differences of the oracle with FP64 inputs reproduce a closed-form
    derivative: for a ray along x at distance b from an isotropic Gaussian's centre,
    alpha = o exp(-b^2 / 2s^2), so d alpha / d mu_y = -alpha b / s^2 and
    d alpha / d s = alpha b^2 / s^3."""
    import copy
    s0, o0, b = 0.1, 0.6, 0.07
    base = make_scene([[1.0, b, 0.0]], [s0] * 3, opac=o0)
    sc = copy.deepcopy(base)
    sc.means = base.means.astype(np.float64)
    sc.scales = base.scales.astype(np.float64)
    sc.opacities = base.opacities.astype(np.float64)
    o32, s32, b32 = float(base.opacities[0]), float(base.scales[0, 0]), float(base.means[0, 1])
    alpha = o32 * math.exp(-0.5 * b32 ** 2 / s32 ** 2)
    h = 1e-6

    def opac(scene):
        return oracle.render(scene, np.zeros((1, 3)), np.array([[1.0, 0.0, 0.0]]), AMIN)["opacity"][0]

    sp, sm = copy.deepcopy(sc), copy.deepcopy(sc)
    sp.means = sc.means.copy(); sp.means[0, 1] += h
    sm.means = sc.means.copy(); sm.means[0, 1] -= h
    assert (opac(sp) - opac(sm)) / (2 * h) == pytest.approx(-alpha * b32 / s32 ** 2, rel=1e-6)
    sp, sm = copy.deepcopy(sc), copy.deepcopy(sc)
    sp.scales = sc.scales + h
    sm.scales = sc.scales - h
    # isotropic scale change: only the two axes across the ray matter for the offset in y
    want = alpha * b32 ** 2 / s32 ** 3
    assert (opac(sp) - opac(sm)) / (2 * h) == pytest.approx(want, rel=1e-6)
