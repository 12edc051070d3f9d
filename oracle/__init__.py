"""FP64 CPU oracle for 3D Gaussian ray tracing -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import this
package. The product path (the HIP library and its Python binding) never imports it.

The numerical work lives in ``grtx_oracle.c`` (plain C, FP64, brute force over every
ray/Gaussian pair); this module compiles it with gcc on first use and wraps it with
ctypes. Each wrapper names the part of the paper it follows; the C file's header states
the full definition.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "grtx_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

GCC_CMD = ["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
           "-pthread", _SRC, "-o", _LIB_PATH, "-lm"]


def build(force: bool = False) -> str:
    """Compile the oracle's C source into ``oracle/liboracle.so``."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp"
        cmd = GCC_CMD[:-3] + ["-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _p(a, ctype):
    return None if a is None else a.ctypes.data_as(C.POINTER(ctype))


def lib():
    global _lib
    with _lock:
        if _lib is None:
            build()
            L = C.CDLL(_LIB_PATH)
            f, d, i32, i64, u32, u64 = C.c_float, C.c_double, C.c_int32, C.c_int64, C.c_uint32, C.c_uint64
            PF, PD = C.POINTER(f), C.POINTER(d)
            L.oracle_render.restype = C.c_int
            L.oracle_render.argtypes = [PD, PD, PD, PD, PD, i64, C.c_int, i64, PD, PD, PD, PD, d, d, d, PD,
                                        C.c_int, PD, PD, PD, C.POINTER(i32), C.POINTER(i32), C.POINTER(i32), PD,
                                        PD, C.c_int, C.c_int]
            L.oracle_ray_hits.restype = i64
            L.oracle_ray_hits.argtypes = [PD, PD, PD, PD, i64, PD, PD, d, d, d, C.c_int, C.POINTER(i64), PD, PD,
                                          PD, i64]
            L.oracle_composite_list.restype = C.c_int
            L.oracle_composite_list.argtypes = [PD, PD, PD, PD, PD, i64, C.c_int, PD, PD, C.POINTER(i32), i64,
                                                d, d, PD, PD, PD, PD]
            L.oracle_object_rays.restype = C.c_int
            L.oracle_object_rays.argtypes = [PD, PD, d, i64, PD, PD, d, PD, PD, PD, PD, C.POINTER(i32)]
            L.oracle_gaussian_aabb.restype = C.c_int
            L.oracle_gaussian_aabb.argtypes = [PD, PD, PD, PD, i64, d, PD, PD, C.POINTER(i32)]
            L.oracle_pinhole_rays.restype = C.c_int
            L.oracle_pinhole_rays.argtypes = [PD, PD, PD, d, C.c_int, C.c_int, PD, PD]
            L.oracle_morton.restype = C.c_int
            L.oracle_morton.argtypes = [i64, PF, C.POINTER(u64)]
            L.oracle_lbvh_topology_search.restype = C.c_int
            L.oracle_lbvh_topology_search.argtypes = [i64, PF, C.POINTER(u64), C.POINTER(u32), C.POINTER(u32),
                                                      C.POINTER(u32), C.c_int]
            L.oracle_sh_basis.restype = d
            L.oracle_sh_basis.argtypes = [C.c_int, C.c_int, PD]
            L.oracle_icosahedron.restype = C.c_int
            L.oracle_icosahedron.argtypes = [PD, C.POINTER(i32)]
            L.oracle_model_render.restype = C.c_int
            L.oracle_model_render.argtypes = [PD, PD, PD, PD, PD, i64, C.c_int, i64, PD, PD, d, d, C.c_int, C.c_int,
                                              C.c_int, C.c_int, C.c_int, PD, PD, PD, C.POINTER(i32),
                                              C.POINTER(i32), C.POINTER(i32), C.POINTER(i32), C.POINTER(i64),
                                              C.c_int]
            L.oracle_model_round_state.restype = C.c_int
            L.oracle_model_round_state.argtypes = [PD, PD, PD, PD, PD, i64, C.c_int, PD, PD, d, d, C.c_int, C.c_int,
                                                   C.c_int, C.c_int, C.POINTER(i64), PD, C.POINTER(i32),
                                                   C.POINTER(i64), PD, C.POINTER(i32), C.c_int, C.POINTER(i64),
                                                   C.POINTER(i64), PD, C.POINTER(i32), C.c_int, PD, C.POINTER(i64)]
            _lib = L
    return _lib


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _f64(a):
    """Widen to FP64 (exact for float32 inputs; FP64 inputs pass through)."""
    return np.ascontiguousarray(a, dtype=np.float64)


def _scene_args(scene):
    return (_f64(scene.means), _f64(scene.scales), _f64(scene.quats), _f64(scene.opacities),
            _f64(scene.sh.reshape(scene.n, -1)) if scene.sh is not None else None)


def render(scene, origins, dirs, alpha_min=1.0 / 255.0, T_min=1e-3, t_near=0.0, bg=(0.0, 0.0, 0.0),
           key_mode=0, cap=0, nthreads=None, t_far=None, trans0=None):
    """Brute-force FP64 render of the given rays (Eq. 1, Eq. 2, Sec. III-A). Scene and rays
    are taken as given (float32 values are widened exactly; FP64 values are used as is).

    key_mode 0 orders hits by ellipsoid entry distance, 1 by bounding-icosahedron entry
    distance. With cap > 0 also returns, per ray, the first `cap` blended ids, the
    transmittance after each and each hit's key distance. t_far [R] bounds the rays (hits
    need key < t_far; bounded rays get no background); trans0 [R] is the transmittance
    each ray starts with (both optional)."""
    L = lib()
    if nthreads is None:
        nthreads = min(16, os.cpu_count() or 1)
    o = _f64(origins).reshape(-1, 3)
    d = _f64(dirs).reshape(-1, 3)
    R = o.shape[0]
    m, s, q, op, sh = _scene_args(scene)
    rgb = np.zeros((R, 3), np.float64)
    depth = np.zeros(R, np.float64)
    opac = np.zeros(R, np.float64)
    nblend = np.zeros(R, np.int32)
    nhits = np.zeros(R, np.int32)
    ids = np.full((R, max(cap, 1)), -1, np.int32) if cap > 0 else None
    tafter = np.zeros((R, max(cap, 1)), np.float64) if cap > 0 else None
    tkey = np.zeros((R, max(cap, 1)), np.float64) if cap > 0 else None
    bga = np.asarray(bg, np.float64)
    tf = None if t_far is None else _f64(t_far).reshape(R)
    t0 = None if trans0 is None else _f64(trans0).reshape(R)
    rc = L.oracle_render(_p(m, C.c_double), _p(s, C.c_double), _p(q, C.c_double), _p(op, C.c_double),
                         _p(sh, C.c_double), scene.n, scene.sh_degree, R, _p(o, C.c_double), _p(d, C.c_double),
                         _p(tf, C.c_double), _p(t0, C.c_double), alpha_min, T_min, t_near, _p(bga, C.c_double), key_mode,
                         _p(rgb, C.c_double), _p(depth, C.c_double), _p(opac, C.c_double),
                         _p(nblend, C.c_int32), _p(nhits, C.c_int32), _p(ids, C.c_int32),
                         _p(tafter, C.c_double), _p(tkey, C.c_double), cap, nthreads)
    if rc != 0:
        raise RuntimeError(f"oracle_render failed ({rc})")
    out = dict(rgb=rgb, depth=depth, opacity=opac, nblend=nblend, nhits=nhits)
    if cap > 0:
        out.update(ids=ids, tafter=tafter, tkey=tkey)
    return out


def ray_hits(scene, origin, direction, alpha_min=1.0 / 255.0, t_near=0.0, key_mode=0, t_far=np.inf):
    """All hits of one ray with key in (t_near, t_far), sorted by (key distance, id): ids,
    key, alpha, t_alpha."""
    L = lib()
    m, s, q, op, _ = _scene_args(scene)
    o = _f64(origin).reshape(3)
    d = _f64(direction).reshape(3)
    cap = scene.n
    ids = np.zeros(max(cap, 1), np.int64)
    tk = np.zeros(max(cap, 1), np.float64)
    al = np.zeros(max(cap, 1), np.float64)
    ta = np.zeros(max(cap, 1), np.float64)
    nh = L.oracle_ray_hits(_p(m, C.c_double), _p(s, C.c_double), _p(q, C.c_double), _p(op, C.c_double), scene.n,
                           _p(o, C.c_double), _p(d, C.c_double), alpha_min, t_near, float(t_far), key_mode,
                           _p(ids, C.c_int64), _p(tk, C.c_double), _p(al, C.c_double), _p(ta, C.c_double), cap)
    if nh < 0:
        raise RuntimeError("oracle_ray_hits failed")
    return dict(ids=ids[:nh], t=tk[:nh], alpha=al[:nh], talpha=ta[:nh])


def composite_list(scene, origin, direction, ids, alpha_min=1.0 / 255.0, bg=(0.0, 0.0, 0.0), trans0=1.0):
    """Composite an explicit ordered id list along one ray (Eq. 1 with Eq. 2 alphas),
    starting from transmittance trans0."""
    L = lib()
    m, s, q, op, sh = _scene_args(scene)
    o = _f64(origin).reshape(3)
    d = _f64(direction).reshape(3)
    lst = np.ascontiguousarray(ids, np.int32)
    rgb = np.zeros(3, np.float64)
    dep = np.zeros(1, np.float64)
    opa = np.zeros(1, np.float64)
    bga = np.asarray(bg, np.float64)
    rc = L.oracle_composite_list(_p(m, C.c_double), _p(s, C.c_double), _p(q, C.c_double), _p(op, C.c_double),
                                 _p(sh, C.c_double), scene.n, scene.sh_degree, _p(o, C.c_double), _p(d, C.c_double),
                                 _p(lst, C.c_int32), lst.size, alpha_min, float(trans0), _p(bga, C.c_double),
                                 _p(rgb, C.c_double), _p(dep, C.c_double), _p(opa, C.c_double))
    if rc != 0:
        raise RuntimeError("oracle_composite_list failed")
    return dict(rgb=rgb, depth=float(dep[0]), opacity=float(opa[0]))


def object_rays(objects, origins, dirs, t_near=0.0):
    """Where each ray meets the glass sphere or the mirror of `objects` (a dict with
    optional "sphere" = (cx, cy, cz, r, ior), "mirror" = (m, u, v) as 9 numbers, "eps")
    and the continuation ray there (Sec. II-A; the secondary-ray experiment of Sec. VI).
    Returns t_far, next_o, next_d, path and kind (0 none, 1 mirror, 2 glass, 3 glass
    without a way out)."""
    L = lib()
    o = _f64(origins).reshape(-1, 3)
    d = _f64(dirs).reshape(-1, 3)
    R = o.shape[0]
    sph = objects.get("sphere")
    mir = objects.get("mirror")
    sph = None if sph is None else _f64(sph).reshape(5)
    mir = None if mir is None else _f64(mir).reshape(9)
    out = dict(t_far=np.zeros(R), next_o=np.zeros((R, 3)), next_d=np.zeros((R, 3)), path=np.zeros(R),
               kind=np.zeros(R, np.int32))
    rc = L.oracle_object_rays(_p(sph, C.c_double), _p(mir, C.c_double), float(objects.get("eps", 1e-4)), R,
                              _p(o, C.c_double), _p(d, C.c_double), t_near, _p(out["t_far"], C.c_double),
                              _p(out["next_o"], C.c_double), _p(out["next_d"], C.c_double),
                              _p(out["path"], C.c_double), _p(out["kind"], C.c_int32))
    if rc != 0:
        raise RuntimeError("oracle_object_rays failed")
    return out


def render_with_objects(scene, origins, dirs, objects, bounces=1, alpha_min=1.0 / 255.0, T_min=1e-3, t_near=0.0,
                        bg=(0.0, 0.0, 0.0), key_mode=0, trans0=None, nthreads=None, levels=None):
    """Render rays through a scene with a glass sphere and a mirror, following up to
    `bounces` object interactions per ray. Each ray segment is an ordinary render bounded
    by t_far; a segment that reaches its surface with T >= T_min continues as the
    continuation ray, starting from that transmittance, and its result is added:
      rgb   = rgb_1 + rgb_2
      depth = depth_1 + depth_2 + path * (T_1 - T_2)   (distances along the bent path)
      opacity = opacity_2                              (1 - the final transmittance)
    With `levels` (a list) each level's rays and outputs are appended to it."""
    o = _f64(origins).reshape(-1, 3)
    d = _f64(dirs).reshape(-1, 3)
    R = o.shape[0]
    if bounces > 0:
        ob = object_rays(objects, o, d, t_near)
        t_far = ob["t_far"]
    else:
        ob = None
        t_far = None
    out = render(scene, o, d, alpha_min, T_min, t_near, bg, key_mode, nthreads=nthreads, t_far=t_far,
                 trans0=trans0)
    if levels is not None:
        levels.append(dict(origins=o, dirs=d, objects=ob, out={k: v.copy() for k, v in out.items()}, trans0=trans0))
    if ob is None:
        return out
    T1 = 1.0 - out["opacity"]
    cont = np.flatnonzero(((ob["kind"] == 1) | (ob["kind"] == 2)) & (T1 >= T_min))
    if cont.size == 0:
        return out
    sub = render_with_objects(scene, ob["next_o"][cont], ob["next_d"][cont], objects, bounces - 1, alpha_min, T_min,
                              0.0, bg, key_mode, trans0=T1[cont], nthreads=nthreads, levels=levels)
    T2 = 1.0 - sub["opacity"]
    out["rgb"][cont] += sub["rgb"]
    out["depth"][cont] += sub["depth"] + ob["path"][cont] * (T1[cont] - T2)
    out["opacity"][cont] = sub["opacity"]
    return out


def gaussian_aabb(scene, alpha_min=1.0 / 255.0):
    """FP64 axis-aligned bounds of each Gaussian's bounding ellipsoid."""
    L = lib()
    m, s, q, op, _ = _scene_args(scene)
    lo = np.zeros((scene.n, 3), np.float64)
    hi = np.zeros((scene.n, 3), np.float64)
    act = np.zeros(scene.n, np.int32)
    L.oracle_gaussian_aabb(_p(m, C.c_double), _p(s, C.c_double), _p(q, C.c_double), _p(op, C.c_double), scene.n,
                           alpha_min, _p(lo, C.c_double), _p(hi, C.c_double), _p(act, C.c_int32))
    return lo, hi, act.astype(bool)


def pinhole_rays(camera):
    """FP64 pinhole primary rays, one per pixel centre, row-major from the top row."""
    L = lib()
    W, H = camera.width, camera.height
    o = np.zeros((W * H, 3), np.float64)
    d = np.zeros((W * H, 3), np.float64)
    eye = np.asarray(camera.eye, np.float64)
    tgt = np.asarray(camera.target, np.float64)
    up = np.asarray(camera.up, np.float64)
    rc = L.oracle_pinhole_rays(_p(eye, C.c_double), _p(tgt, C.c_double), _p(up, C.c_double), camera.fov_y_deg,
                               W, H, _p(o, C.c_double), _p(d, C.c_double))
    if rc != 0:
        raise RuntimeError("oracle_pinhole_rays failed")
    return o, d


def morton(means):
    L = lib()
    m = _f32(means).reshape(-1, 3)
    codes = np.zeros(m.shape[0], np.uint64)
    L.oracle_morton(m.shape[0], _p(m, C.c_float), _p(codes, C.c_uint64))
    return codes


def lbvh_topology(means, linear=False):
    """Sorted Morton codes, permutation, child [(n-1),2] and parent [2n-1] arrays. Each
    node's split is found by bisection, or with `linear` by testing every position of its
    key range (the definition as written, quadratic; small sizes)."""
    L = lib()
    m = _f32(means).reshape(-1, 3)
    n = m.shape[0]
    codes = np.zeros(n, np.uint64)
    perm = np.zeros(n, np.uint32)
    child = np.zeros((max(n - 1, 1), 2), np.uint32)
    parent = np.zeros(max(2 * n - 1, 1), np.uint32)
    rc = L.oracle_lbvh_topology_search(n, _p(m, C.c_float), _p(codes, C.c_uint64), _p(perm, C.c_uint32),
                                       _p(child, C.c_uint32), _p(parent, C.c_uint32), 1 if linear else 0)
    if rc != 0:
        raise RuntimeError("oracle_lbvh_topology failed")
    return dict(codes=codes, perm=perm, child=child[: max(n - 1, 0)], parent=parent[: max(2 * n - 1, 0)])


def sh_basis(l, m, direction):
    L = lib()
    d = np.ascontiguousarray(direction, np.float64).reshape(3)
    return L.oracle_sh_basis(l, m, _p(d, C.c_double))


def icosahedron():
    L = lib()
    v = np.zeros((12, 3), np.float64)
    f = np.zeros((20, 3), np.int32)
    L.oracle_icosahedron(_p(v, C.c_double), _p(f, C.c_int32))
    return v, f


# --------------------------------------------------------------------------------------
# CPU model of the method (multi-round k-buffer traversal with checkpoints)

CHECKPOINT, RESTART = 0, 1
RULE_KBUF_MAX, RULE_PAPER = 0, 1


def model_render(scene, origins, dirs, k, mode=CHECKPOINT, rule=RULE_KBUF_MAX, alpha_min=1.0 / 255.0,
                 T_min=1e-3, cap=0, nthreads=None, distinct=True):
    """The method itself on the CPU in FP64 (Sec. III-B, IV): rounds of k-buffer hit
    collection over the oracle's radix tree with exact Gaussian boxes, each round blended
    front to back, resuming from checkpoint lists (mode CHECKPOINT) or from the root
    (RESTART). rule: the round's cull distance t_max once the k-buffer is full, its
    farthest key (RULE_KBUF_MAX) or the nearest key it rejected or pushed out (RULE_PAPER,
    the walkthrough of Sec. IV-B). t_near = 0, black background.
    Returns rgb, depth, opacity, nblend, rounds and counts [R,6] (internal nodes visited,
    leaves tested, nodes deferred, hits evicted, distinct nodes and leaves visited, and the
    largest checkpoint carried between rounds in entries; the distinct count only with
    `distinct`, which costs a visit bitmap per thread); with cap > 0 also the first `cap`
    blended ids and the round that blended each (round_of)."""
    L = lib()
    if nthreads is None:
        nthreads = min(16, os.cpu_count() or 1)
    o = _f64(origins).reshape(-1, 3)
    d = _f64(dirs).reshape(-1, 3)
    R = o.shape[0]
    m, s, q, op, sh = _scene_args(scene)
    rgb = np.zeros((R, 3), np.float64)
    depth = np.zeros(R, np.float64)
    opac = np.zeros(R, np.float64)
    nblend = np.zeros(R, np.int32)
    rounds = np.zeros(R, np.int32)
    counts = np.zeros((R, 6), np.int64)
    ids = np.full((R, max(cap, 1)), -1, np.int32) if cap > 0 else None
    round_of = np.zeros((R, max(cap, 1)), np.int32) if cap > 0 else None
    rc = L.oracle_model_render(_p(m, C.c_double), _p(s, C.c_double), _p(q, C.c_double), _p(op, C.c_double),
                               _p(sh, C.c_double), scene.n, scene.sh_degree, R, _p(o, C.c_double),
                               _p(d, C.c_double), alpha_min, T_min, k, mode, rule, cap, nthreads,
                               _p(rgb, C.c_double), _p(depth, C.c_double), _p(opac, C.c_double),
                               _p(nblend, C.c_int32), _p(ids, C.c_int32), _p(round_of, C.c_int32),
                               _p(rounds, C.c_int32), _p(counts, C.c_int64), 1 if distinct else 0)
    if rc != 0:
        raise RuntimeError(f"oracle_model_render failed ({rc})")
    out = dict(rgb=rgb, depth=depth, opacity=opac, nblend=nblend, rounds=rounds, counts=counts)
    if cap > 0:
        out.update(ids=ids, round_of=round_of)
    return out


def model_round_state(scene, origin, direction, k, round_, mode=CHECKPOINT, rule=RULE_KBUF_MAX,
                      alpha_min=1.0 / 255.0, T_min=1e-3, cap=256):
    """One ray's state at the end of round `round_` of the CPU model, before that round
    blends: the k-buffer (ids, distances), the eviction list (ids, distances), the deferred
    nodes (the range of sorted leaf positions under each, in oracle_lbvh_topology's order,
    and its entry distance) and t_max (distance, id; inf while the k-buffer was not full).
    None if the ray finishes earlier."""
    L = lib()
    o = _f64(origin).reshape(3)
    d = _f64(direction).reshape(3)
    m, s, q, op, sh = _scene_args(scene)
    kid = np.zeros(k, np.int64)
    kt = np.zeros(k, np.float64)
    eid = np.zeros(cap, np.int64)
    et = np.zeros(cap, np.float64)
    df = np.zeros(cap, np.int64)
    dl = np.zeros(cap, np.int64)
    dt = np.zeros(cap, np.float64)
    nk, ne, nd = C.c_int32(0), C.c_int32(0), C.c_int32(0)
    tt, ti = C.c_double(0.0), C.c_int64(0)
    rc = L.oracle_model_round_state(_p(m, C.c_double), _p(s, C.c_double), _p(q, C.c_double), _p(op, C.c_double),
                                    _p(sh, C.c_double), scene.n, scene.sh_degree, _p(o, C.c_double),
                                    _p(d, C.c_double), alpha_min, T_min, k, mode, rule, round_,
                                    _p(kid, C.c_int64), _p(kt, C.c_double), C.byref(nk), _p(eid, C.c_int64),
                                    _p(et, C.c_double), C.byref(ne), cap, _p(df, C.c_int64), _p(dl, C.c_int64),
                                    _p(dt, C.c_double), C.byref(nd), cap, C.byref(tt), C.byref(ti))
    if rc != 0:
        return None
    if ne.value > cap or nd.value > cap:
        raise RuntimeError("model_round_state: lists longer than cap")
    return dict(kbuf_ids=kid[:nk.value], kbuf_t=kt[:nk.value], evicted_ids=eid[:ne.value], evicted_t=et[:ne.value],
                deferred_first=df[:nd.value], deferred_last=dl[:nd.value], deferred_t=dt[:nd.value],
                tmax_t=tt.value, tmax_id=ti.value)
