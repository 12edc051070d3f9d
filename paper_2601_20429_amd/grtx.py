"""Python binding of libgrtx.so (include/grtx.h): argument marshalling only.

Every computation runs in the HIP library. PyTorch supplies device memory and the
current HIP stream; tensors are passed to the C ABI as raw device pointers. If the
library is not built the import of this module still works, but every call raises.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libgrtx.so")

OK = 0
ERR_INVALID_ARG = 1
ERR_OUT_OF_MEMORY = 2
ERR_DEVICE = 3
ERR_CAPACITY = 4
ERR_NOT_READY = 5
ERR_INTERNAL = 6

SPHERE_INSTANCE = 0
PROXY20 = 1
ICO_INSTANCE = 2
CHECKPOINT = 0
RESTART = 1
SINGLE_ROUND = 2

STAT_NODES, STAT_LEAVES, STAT_ROUNDS, STAT_BLENDED, STAT_DEFERRED, STAT_FETCH_FREE, STAT_EVICTED, \
    STAT_FALLBACKS, STAT_STACK_DROPS = range(9)
STATS_FIELDS = 9
MAX_TREE_DEPTH = 96
OBJECT_NONE, OBJECT_MIRROR, OBJECT_GLASS, OBJECT_GLASS_TRAPPED = range(4)


class GrtxError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"grtx status {status}: {msg}")
        self.status = status


class _Gaussians(C.Structure):
    _fields_ = [("means", C.c_void_p), ("scales", C.c_void_p), ("quats", C.c_void_p), ("opacities", C.c_void_p),
                ("sh", C.c_void_p), ("count", C.c_int64), ("sh_degree", C.c_int32), ("reserved", C.c_int32)]


class _BuildParams(C.Structure):
    _fields_ = [("alpha_min", C.c_float), ("plain_lbvh", C.c_int32), ("max_depth", C.c_int32),
                ("reserved", C.c_int32)]


class _BvhInfo(C.Structure):
    _fields_ = [("gaussians", C.c_int64), ("leaves", C.c_int64), ("internal_nodes", C.c_int64),
                ("device_bytes", C.c_int64), ("kind", C.c_int32), ("sh_degree", C.c_int32),
                ("alpha_min", C.c_float), ("root_lo", C.c_float * 3), ("root_hi", C.c_float * 3),
                ("depth", C.c_int32), ("restructured", C.c_int32)]


class _Rays(C.Structure):
    _fields_ = [("origins", C.c_void_p), ("dirs", C.c_void_p), ("count", C.c_int64), ("t_near", C.c_float),
                ("image_width", C.c_int32), ("t_far", C.c_void_p), ("transmittance", C.c_void_p),
                ("next_origins", C.c_void_p), ("next_dirs", C.c_void_p), ("path", C.c_void_p), ("kind", C.c_void_p),
                ("image_begin", C.c_int64)]


class _Objects(C.Structure):
    _fields_ = [("sphere_center", C.c_float * 3), ("sphere_radius", C.c_float), ("sphere_ior", C.c_float),
                ("mirror_center", C.c_float * 3), ("mirror_u", C.c_float * 3), ("mirror_v", C.c_float * 3),
                ("surface_eps", C.c_float)]


class _TraceParams(C.Structure):
    _fields_ = [("k", C.c_int32), ("T_min", C.c_float), ("mode", C.c_int32), ("bg", C.c_float * 3),
                ("defer_capacity", C.c_int32), ("evict_capacity", C.c_int32), ("collect_capacity", C.c_int32),
                ("reserved", C.c_int32)]


class _TraceOutputs(C.Structure):
    _fields_ = [("rgb", C.c_void_p), ("depth", C.c_void_p), ("opacity", C.c_void_p), ("stats", C.c_void_p),
                ("hit_ids", C.c_void_p), ("hit_counts", C.c_void_p), ("hit_capacity", C.c_int32),
                ("reserved", C.c_int32)]


class _GaussianGrads(C.Structure):
    _fields_ = [("means", C.c_void_p), ("scales", C.c_void_p), ("quats", C.c_void_p), ("opacities", C.c_void_p),
                ("sh", C.c_void_p)]


class _Camera(C.Structure):
    _fields_ = [("eye", C.c_float * 3), ("target", C.c_float * 3), ("up", C.c_float * 3), ("fov_y_deg", C.c_float),
                ("width", C.c_int32), ("height", C.c_int32)]


class _ServeConfig(C.Structure):
    _fields_ = [("memory_budget", C.c_int64), ("k", C.c_int32), ("T_min", C.c_float), ("mode", C.c_int32),
                ("max_request_rays", C.c_int32), ("bg", C.c_float * 3), ("idle_exit_us", C.c_int32)]


class _Request(C.Structure):
    _fields_ = [("scene_id", C.c_int32), ("width", C.c_int32), ("height", C.c_int32), ("eye", C.c_float * 3),
                ("target", C.c_float * 3), ("up", C.c_float * 3), ("fov_y_deg", C.c_float)]


class _RequestResult(C.Structure):
    _fields_ = [("rgb", C.c_void_p), ("depth", C.c_void_p), ("opacity", C.c_void_p), ("width", C.c_int32),
                ("height", C.c_int32), ("t_submit", C.c_double), ("t_admit", C.c_double),
                ("t_launch", C.c_double), ("t_done", C.c_double)]


class _ServeStats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("rays_completed", C.c_int64),
                ("bytes_in_use", C.c_int64), ("bytes_available", C.c_int64), ("bytes_arena", C.c_int64),
                ("launches", C.c_int64), ("p50_ms", C.c_double),
                ("p99_ms", C.c_double), ("mean_ms", C.c_double), ("max_ms", C.c_double), ("busy_s", C.c_double),
                ("mrays_per_s", C.c_double)]


# Every symbol the header declares, with its ctypes signature.
_SIGNATURES = {
    "grtx_build": (C.c_int, [C.POINTER(_Gaussians), C.c_int, C.POINTER(_BuildParams), C.c_void_p,
                             C.POINTER(C.c_void_p)]),
    "grtx_bvh_get_info": (C.c_int, [C.c_void_p, C.POINTER(_BvhInfo)]),
    "grtx_bvh_export_topology": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                           C.c_void_p, C.c_void_p]),
    "grtx_bvh_destroy": (C.c_int, [C.c_void_p]),
    "grtx_pinhole_rays": (C.c_int, [C.POINTER(_Camera), C.c_void_p, C.c_void_p, C.c_void_p]),
    "grtx_trace": (C.c_int, [C.c_void_p, C.POINTER(_Rays), C.POINTER(_TraceParams), C.POINTER(_TraceOutputs),
                             C.c_void_p]),
    "grtx_trace_noalloc": (C.c_int, [C.c_void_p, C.POINTER(_Rays), C.POINTER(_TraceParams),
                                     C.POINTER(_TraceOutputs), C.c_void_p]),
    "grtx_trace_backward": (C.c_int, [C.c_void_p, C.POINTER(_Gaussians), C.POINTER(_Rays), C.POINTER(_TraceParams),
                                      C.POINTER(_TraceOutputs), C.c_void_p, C.c_void_p, C.c_void_p,
                                      C.POINTER(_GaussianGrads), C.c_void_p, C.c_void_p]),
    "grtx_object_rays": (C.c_int, [C.POINTER(_Objects), C.POINTER(_Rays), C.c_void_p, C.c_void_p, C.c_void_p,
                                   C.c_void_p, C.c_void_p, C.c_void_p]),
    "grtx_continue_rays": (C.c_int, [C.c_int64, C.c_void_p, C.c_void_p, C.c_float, C.c_void_p, C.c_void_p,
                                     C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(C.c_int64),
                                     C.c_void_p]),
    "grtx_continue_composite": (C.c_int, [C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                          C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "grtx_serve_request_bytes": (C.c_int, [C.POINTER(_Request), C.POINTER(C.c_int64)]),
    "grtx_serve_create": (C.c_int, [C.POINTER(_ServeConfig), C.POINTER(C.c_void_p)]),
    "grtx_serve_add_scene": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(C.c_int32)]),
    "grtx_serve_submit": (C.c_int, [C.c_void_p, C.POINTER(_Request), C.POINTER(C.c_uint64)]),
    "grtx_serve_poll": (C.c_int, [C.c_void_p, C.c_uint64, C.POINTER(_RequestResult)]),
    "grtx_serve_copy_result": (C.c_int, [C.c_void_p, C.c_uint64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "grtx_serve_release": (C.c_int, [C.c_void_p, C.c_uint64]),
    "grtx_serve_get_stats": (C.c_int, [C.c_void_p, C.POINTER(_ServeStats)]),
    "grtx_serve_destroy": (C.c_int, [C.c_void_p]),
    "grtx_last_error": (C.c_char_p, []),
    "grtx_version": (C.c_int32, []),
}

_lib = None


def lib():
    """Load libgrtx.so. Raises if the library has not been built: there is no fallback."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2601_20429_amd.build`")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(status):
    if status != OK:
        raise GrtxError(status, lib().grtx_last_error().decode(errors="replace"))


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def _dev_f32(x, device):
    t = torch.as_tensor(x, dtype=torch.float32, device=device)
    return t.contiguous()


@dataclass
class SceneTensors:
    means: torch.Tensor
    scales: torch.Tensor
    quats: torch.Tensor
    opacities: torch.Tensor
    sh: torch.Tensor
    sh_degree: int

    @staticmethod
    def from_scene(scene, device="cuda"):
        return SceneTensors(_dev_f32(scene.means, device), _dev_f32(scene.scales, device),
                            _dev_f32(scene.quats, device), _dev_f32(scene.opacities, device),
                            _dev_f32(scene.sh, device).reshape(scene.n, (int(scene.sh_degree) + 1) ** 2, 3),
                            int(scene.sh_degree))

    @property
    def n(self):
        return int(self.means.shape[0])


class Bvh:
    """Owner of a grtx_bvh handle. Keeps the borrowed scene tensors alive."""

    def __init__(self, handle, scene: SceneTensors, kind: int, alpha_min: float):
        self.handle = handle
        self.scene = scene
        self.kind = kind
        self.alpha_min = alpha_min

    def close(self):
        if self.handle:
            _check(lib().grtx_bvh_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            if self.handle:
                lib().grtx_bvh_destroy(self.handle)
        except Exception:
            pass

    def info(self):
        inf = _BvhInfo()
        _check(lib().grtx_bvh_get_info(self.handle, C.byref(inf)))
        return dict(gaussians=inf.gaussians, leaves=inf.leaves, internal_nodes=inf.internal_nodes,
                    device_bytes=inf.device_bytes, kind=inf.kind, sh_degree=inf.sh_degree,
                    alpha_min=inf.alpha_min, root_lo=list(inf.root_lo), root_hi=list(inf.root_hi),
                    depth=inf.depth, restructured=inf.restructured)

    def export_topology(self, stream=None):
        inf = self.info()
        n, m = inf["leaves"], inf["internal_nodes"]
        dev = self.scene.means.device
        child = torch.empty((max(m, 1), 2), dtype=torch.int32, device=dev)
        parent = torch.empty(max(m + n, 1), dtype=torch.int32, device=dev)
        morton = torch.empty(max(n, 1), dtype=torch.int64, device=dev)
        perm = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
        boxes = torch.empty((max(m + n, 1), 6), dtype=torch.float32, device=dev)
        _check(lib().grtx_bvh_export_topology(self.handle, _ptr(child), _ptr(parent), _ptr(morton), _ptr(perm),
                                              _ptr(boxes), _stream(stream)))
        return dict(child=child[:m], parent=parent[:m + n], morton=morton[:n], perm=perm[:n], boxes=boxes[:m + n])


def build(scene: SceneTensors, kind: int = SPHERE_INSTANCE, alpha_min: float = 1.0 / 255.0, stream=None,
          plain_lbvh: bool = False, max_depth: int = 0) -> Bvh:
    """grtx_build. plain_lbvh keeps the radix tree as the LBVH construction gives it (no
    treelet restructuring); traced results are the same either way. A restructured tree
    deeper than max_depth (0 = MAX_TREE_DEPTH) is replaced by the plain one."""
    g = _Gaussians(scene.means.data_ptr(), scene.scales.data_ptr(), scene.quats.data_ptr(),
                   scene.opacities.data_ptr(), scene.sh.data_ptr(), scene.n, scene.sh_degree, 0)
    p = _BuildParams(alpha_min, 1 if plain_lbvh else 0, max_depth)
    h = C.c_void_p()
    _check(lib().grtx_build(C.byref(g), kind, C.byref(p), _stream(stream), C.byref(h)))
    return Bvh(h, scene, kind, alpha_min)


def pinhole_rays(camera, device="cuda", stream=None, out=None):
    """Pinhole rays of `camera` in row-major pixel order: origins, unit directions [W*H,3]
    float32; into `out` = (origins, dirs) when given (contiguous, float32)."""
    n = camera.width * camera.height
    if out is not None:
        o, d = out
        for t in (o, d):
            if t.shape != (n, 3) or t.dtype != torch.float32 or not t.is_contiguous():
                raise ValueError(f"pinhole_rays: out tensors must be contiguous float32 [{n},3]")
    else:
        o = torch.empty((n, 3), dtype=torch.float32, device=device)
        d = torch.empty((n, 3), dtype=torch.float32, device=device)
    cam = _Camera((C.c_float * 3)(*camera.eye), (C.c_float * 3)(*camera.target), (C.c_float * 3)(*camera.up),
                  camera.fov_y_deg, camera.width, camera.height)
    _check(lib().grtx_pinhole_rays(C.byref(cam), _ptr(o), _ptr(d), _stream(stream)))
    return o, d


def trace(bvh: Bvh, origins: torch.Tensor, dirs: torch.Tensor, k: int = 16, T_min: float = 1e-3,
          mode: int = CHECKPOINT, bg=(0.0, 0.0, 0.0), t_near: float = 0.0, image_width: int = 0,
          image_begin: int = 0, stats: bool = False, hit_capacity: int = 0, defer_capacity: int = 0, evict_capacity: int = 0,
          out=None, stream=None, t_far: torch.Tensor = None, transmittance: torch.Tensor = None,
          continuation: dict = None, collect_capacity: int = 0, _entry: str = "grtx_trace"):
    """Render rays; returns dict(rgb [R,3], depth [R], opacity [R], and optionally stats
    [R,9] int32, hit_ids [R,cap] int32, hit_counts [R] int32). t_far [R] bounds the rays at
    a surface; transmittance [R] is what each ray starts with (both optional float32).
    continuation: the dict of `object_rays` (next_o, next_d, path, kind); rays that reach
    their surface then go on along their continuation ray in the same launch.
    image_width > 0: rays image_begin.. form a row-major image of that width, traced after
    the rays before image_begin (scheduling only).
    mode SINGLE_ROUND collects up to `collect_capacity` hits per ray (0 = 2048), then sorts
    and blends them."""
    R = int(origins.shape[0])
    dev = origins.device
    if out is None:
        out = dict(rgb=torch.empty((R, 3), dtype=torch.float32, device=dev),
                   depth=torch.empty(R, dtype=torch.float32, device=dev),
                   opacity=torch.empty(R, dtype=torch.float32, device=dev))
        if stats:
            out["stats"] = torch.empty((R, STATS_FIELDS), dtype=torch.int32, device=dev)
        if hit_capacity > 0:
            out["hit_ids"] = torch.full((R, hit_capacity), -1, dtype=torch.int32, device=dev)
            out["hit_counts"] = torch.empty(R, dtype=torch.int32, device=dev)
    rays = _Rays(origins.data_ptr() if R else None, dirs.data_ptr() if R else None, R, t_near, image_width,
                 t_far.data_ptr() if t_far is not None and R else None,
                 transmittance.data_ptr() if transmittance is not None and R else None)
    rays.image_begin = image_begin
    if continuation is not None and R:
        rays.next_origins = continuation["next_o"].data_ptr()
        rays.next_dirs = continuation["next_d"].data_ptr()
        rays.path = continuation["path"].data_ptr()
        rays.kind = continuation["kind"].data_ptr()
    prm = _TraceParams(k, T_min, mode, (C.c_float * 3)(*bg), defer_capacity, evict_capacity, collect_capacity)
    o = _TraceOutputs(out["rgb"].data_ptr() if R else None, out["depth"].data_ptr() if R else None,
                      out["opacity"].data_ptr() if R else None,
                      out["stats"].data_ptr() if "stats" in out and R else None,
                      out["hit_ids"].data_ptr() if "hit_ids" in out and R else None,
                      out["hit_counts"].data_ptr() if "hit_counts" in out and R else None,
                      int(out["hit_ids"].shape[1]) if "hit_ids" in out else 0, 0)
    _check(getattr(lib(), _entry)(bvh.handle, C.byref(rays), C.byref(prm), C.byref(o), _stream(stream)))
    return out


def trace_noalloc(bvh: Bvh, origins: torch.Tensor, dirs: torch.Tensor, out: dict, **kw):
    """grtx_trace_noalloc: `trace` into the caller's preallocated outputs `out` (rgb, depth,
    opacity, optionally stats / hit_ids / hit_counts) without any device allocation by the
    library; the same keyword arguments as `trace`."""
    return trace(bvh, origins, dirs, out=out, _entry="grtx_trace_noalloc", **kw)


def _objects(objects: dict):
    """grtx_objects from a dict with optional "sphere" = (cx, cy, cz, r, ior), "mirror" =
    (m, u, v) as 9 numbers and "eps"."""
    sph = list(objects.get("sphere") or (0.0, 0.0, 0.0, 0.0, 1.0))
    mir = list(objects.get("mirror") or (0.0,) * 9)
    f3 = lambda a: (C.c_float * 3)(*[float(x) for x in a])
    return _Objects(f3(sph[0:3]), float(sph[3]), float(sph[4]), f3(mir[0:3]), f3(mir[3:6]), f3(mir[6:9]),
                    float(objects.get("eps", 0.0)))


def object_rays(objects: dict, origins: torch.Tensor, dirs: torch.Tensor, t_near: float = 0.0, stream=None):
    """grtx_object_rays: t_far [R], next_o / next_d [R,3], path [R], kind [R] int32."""
    R = int(origins.shape[0])
    dev = origins.device
    out = dict(t_far=torch.empty(R, dtype=torch.float32, device=dev),
               next_o=torch.empty((R, 3), dtype=torch.float32, device=dev),
               next_d=torch.empty((R, 3), dtype=torch.float32, device=dev),
               path=torch.empty(R, dtype=torch.float32, device=dev),
               kind=torch.empty(R, dtype=torch.int32, device=dev))
    rays = _Rays(origins.data_ptr() if R else None, dirs.data_ptr() if R else None, R, t_near, 0, None, None)
    ob = _objects(objects)
    _check(lib().grtx_object_rays(C.byref(ob), C.byref(rays), _ptr(out["t_far"]), _ptr(out["next_o"]),
                                  _ptr(out["next_d"]), _ptr(out["path"]), _ptr(out["kind"]), _stream(stream)))
    return out


def continue_rays(kind, opacity, next_o, next_d, T_min: float = 1e-3, stream=None):
    """grtx_continue_rays: the continuing rays (origins, dirs [n,3], transmittance [n],
    index [n] int32) of segments that reached their surface."""
    R = int(kind.shape[0])
    dev = kind.device
    co = torch.empty((R, 3), dtype=torch.float32, device=dev)
    cd = torch.empty((R, 3), dtype=torch.float32, device=dev)
    ct = torch.empty(R, dtype=torch.float32, device=dev)
    ci = torch.empty(R, dtype=torch.int32, device=dev)
    n = C.c_int64()
    _check(lib().grtx_continue_rays(R, _ptr(kind), _ptr(opacity), T_min, _ptr(next_o), _ptr(next_d), _ptr(co),
                                    _ptr(cd), _ptr(ct), _ptr(ci), C.byref(n), _stream(stream)))
    m = int(n.value)
    return dict(origins=co[:m], dirs=cd[:m], transmittance=ct[:m], index=ci[:m])


def continue_composite(cont: dict, path, cont_out: dict, out: dict, stream=None):
    """grtx_continue_composite: add the continuation results `cont_out` of the rays in
    `cont` to the segment outputs `out` (rgb, depth, opacity, in place)."""
    n = int(cont["index"].shape[0])
    _check(lib().grtx_continue_composite(n, _ptr(cont["index"]), _ptr(cont["transmittance"]), _ptr(path),
                                         _ptr(cont_out["rgb"]), _ptr(cont_out["depth"]), _ptr(cont_out["opacity"]),
                                         _ptr(out["rgb"]), _ptr(out["depth"]), _ptr(out["opacity"]),
                                         _stream(stream)))
    return out


def trace_with_objects(bvh: Bvh, origins: torch.Tensor, dirs: torch.Tensor, objects: dict, bounces: int = 1,
                       t_near: float = 0.0, T_min: float = 1e-3, transmittance: torch.Tensor = None,
                       levels: list = None, stream=None, fused: bool = False, **trace_kw):
    """Render rays through a scene holding a glass sphere and a mirror, following up to
    `bounces` object interactions per ray: object rays, the bounded trace, the gathered
    continuation rays traced from the transmittance left, and their composite. Returns
    the outputs of `trace`; with `levels` (a list) each level's rays and outputs are
    appended to it. fused (one bounce): the continuation runs inside the same trace
    launch instead."""
    if fused:
        if bounces != 1 or levels is not None:
            raise ValueError("the fused continuation follows exactly one bounce and records no levels")
        ob = object_rays(objects, origins, dirs, t_near, stream=stream)
        return trace(bvh, origins, dirs, T_min=T_min, t_near=t_near, t_far=ob["t_far"],
                     transmittance=transmittance, continuation=ob, stream=stream, **trace_kw)
    if bounces <= 0:
        out = trace(bvh, origins, dirs, T_min=T_min, t_near=t_near, transmittance=transmittance, stream=stream,
                    **trace_kw)
        if levels is not None:
            levels.append(dict(origins=origins, dirs=dirs, objects=None, out=out, transmittance=transmittance))
        return out
    ob = object_rays(objects, origins, dirs, t_near, stream=stream)
    out = trace(bvh, origins, dirs, T_min=T_min, t_near=t_near, t_far=ob["t_far"], transmittance=transmittance,
                stream=stream, **trace_kw)
    if levels is not None:
        levels.append(dict(origins=origins, dirs=dirs, objects=ob, out={k: v.clone() for k, v in out.items()},
                           transmittance=transmittance))
    cont = continue_rays(ob["kind"], out["opacity"], ob["next_o"], ob["next_d"], T_min, stream=stream)
    if cont["index"].shape[0] == 0:
        return out
    kw = {k: v for k, v in trace_kw.items() if k not in ("image_width", "out")}
    sub = trace_with_objects(bvh, cont["origins"], cont["dirs"], objects, bounces - 1, 0.0, T_min,
                             cont["transmittance"], levels, stream, **kw)
    continue_composite(cont, ob["path"], sub, out, stream=stream)
    return out


def _gaussians(scene: SceneTensors):
    return _Gaussians(scene.means.data_ptr(), scene.scales.data_ptr(), scene.quats.data_ptr(),
                      scene.opacities.data_ptr(), scene.sh.data_ptr(), scene.n, scene.sh_degree, 0)


def trace_backward(bvh: Bvh, origins, dirs, fwd: dict = None, grad_rgb=None, grad_depth=None, grad_opacity=None,
                   grads: dict = None, k: int = 16, T_min: float = 1e-3, mode: int = CHECKPOINT,
                   bg=(0.0, 0.0, 0.0), t_near: float = 0.0, hit_capacity: int = 0, stream=None,
                   image_width: int = 0):
    """Accumulate dL/d(parameters) into `grads` (dict of tensors shaped like the scene
    arrays; allocated as zeros when None). `fwd` holds rgb, depth, opacity, hit_ids and
    hit_counts of the forward call; when None the library traces the rays again with
    lists of `hit_capacity` entries (0 = 256), scheduled as an image of `image_width` when
    given. Returns (grads, truncated_rays tensor)."""
    sc = bvh.scene
    dev = sc.means.device
    if grads is None:
        grads = dict(means=torch.zeros_like(sc.means), scales=torch.zeros_like(sc.scales),
                     quats=torch.zeros_like(sc.quats), opacities=torch.zeros_like(sc.opacities),
                     sh=torch.zeros_like(sc.sh))
    truncated = torch.zeros(1, dtype=torch.int32, device=dev)
    R = int(origins.shape[0])
    rays = _Rays(origins.data_ptr() if R else None, dirs.data_ptr() if R else None, R, t_near, image_width, None, None)
    prm = _TraceParams(k, T_min, mode, (C.c_float * 3)(*bg), 0, 0)
    if fwd is None:
        o = _TraceOutputs(None, None, None, None, None, None, int(hit_capacity), 0)
    else:
        o = _TraceOutputs(fwd["rgb"].data_ptr(), fwd["depth"].data_ptr(), fwd["opacity"].data_ptr(), None,
                          fwd["hit_ids"].data_ptr(), fwd["hit_counts"].data_ptr(), int(fwd["hit_ids"].shape[1]), 0)
    gg = _GaussianGrads(grads["means"].data_ptr(), grads["scales"].data_ptr(), grads["quats"].data_ptr(),
                        grads["opacities"].data_ptr(), grads["sh"].data_ptr())
    g = _gaussians(sc)
    _check(lib().grtx_trace_backward(bvh.handle, C.byref(g), C.byref(rays), C.byref(prm), C.byref(o),
                                     _ptr(grad_rgb), _ptr(grad_depth), _ptr(grad_opacity), C.byref(gg),
                                     _ptr(truncated), _stream(stream)))
    return grads, truncated


def _request(scene_id, camera):
    return _Request(scene_id, camera.width, camera.height, (C.c_float * 3)(*camera.eye),
                    (C.c_float * 3)(*camera.target), (C.c_float * 3)(*camera.up), camera.fov_y_deg)


def request_bytes(camera):
    b = C.c_int64()
    _check(lib().grtx_serve_request_bytes(C.byref(_request(0, camera)), C.byref(b)))
    return int(b.value)


class Server:
    """Render server: one persistent trace kernel fed from a request queue (grtx_serve_*)."""

    def __init__(self, memory_budget, k=16, T_min=1e-3, mode=CHECKPOINT, max_request_rays=0, bg=(0.0, 0.0, 0.0),
                 idle_exit_us=0):
        cfg = _ServeConfig(int(memory_budget), k, T_min, mode, max_request_rays, (C.c_float * 3)(*bg),
                           int(idle_exit_us))
        h = C.c_void_p()
        _check(lib().grtx_serve_create(C.byref(cfg), C.byref(h)))
        self.handle = h
        self._bvhs = []

    def add_scene(self, bvh: Bvh) -> int:
        sid = C.c_int32()
        _check(lib().grtx_serve_add_scene(self.handle, bvh.handle, C.byref(sid)))
        self._bvhs.append(bvh)
        return int(sid.value)

    def submit(self, scene_id, camera) -> int:
        t = C.c_uint64()
        _check(lib().grtx_serve_submit(self.handle, C.byref(_request(scene_id, camera)), C.byref(t)))
        return int(t.value)

    def poll(self, ticket):
        """None while pending; else a dict of timestamps and the image size."""
        r = _RequestResult()
        st = lib().grtx_serve_poll(self.handle, ticket, C.byref(r))
        if st == ERR_NOT_READY:
            return None
        _check(st)
        return dict(width=r.width, height=r.height, t_submit=r.t_submit, t_admit=r.t_admit, t_launch=r.t_launch,
                    t_done=r.t_done)

    def result(self, ticket, device="cuda", stream=None):
        info = self.poll(ticket)
        if info is None:
            return None
        n = info["width"] * info["height"]
        out = dict(rgb=torch.empty((n, 3), dtype=torch.float32, device=device),
                   depth=torch.empty(n, dtype=torch.float32, device=device),
                   opacity=torch.empty(n, dtype=torch.float32, device=device))
        _check(lib().grtx_serve_copy_result(self.handle, ticket, _ptr(out["rgb"]), _ptr(out["depth"]),
                                            _ptr(out["opacity"]), _stream(stream)))
        out.update(info)
        return out

    def release(self, ticket):
        _check(lib().grtx_serve_release(self.handle, ticket))

    def stats(self):
        st = _ServeStats()
        _check(lib().grtx_serve_get_stats(self.handle, C.byref(st)))
        return {f: getattr(st, f) for f, _ in _ServeStats._fields_}

    def close(self):
        if self.handle:
            _check(lib().grtx_serve_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            if self.handle:
                lib().grtx_serve_destroy(self.handle)
        except Exception:
            pass


def version():
    return int(lib().grtx_version())
