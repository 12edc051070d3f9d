// Secondary rays: where rays meet a glass sphere or a mirror, the rays that continue
// from there, and the compositing of a continued path. A ray tracer follows light past
// a surface by casting a new ray from the hit point (Sec. II-A); the paper's
// secondary-ray experiment places a glass sphere and a rectangular mirror in each scene
// and traces the reflected and refracted rays through the Gaussians (Sec. VI).
//
// All three steps are elementwise over rays and HBM-bound (a few dozen bytes per ray);
// one thread per ray, coalesced float loads and stores.
#include <hip/hip_runtime.h>

#include <cmath>

#include "grtx_internal.h"

namespace grtx {
namespace {

constexpr int kObjBlock = 256;
constexpr int kMaxInside = 8;  // chords a ray may follow inside the glass

struct ObjArgs {
  float3 c;       // sphere centre
  float rad;      // sphere radius (<= 0: no sphere)
  float ior;      // relative index of refraction
  float3 m;       // mirror centre
  float3 u, v;    // mirror half-axes (orthogonal)
  float3 n;       // unit mirror normal
  float inv_uu, inv_vv;
  int has_mirror;
  float tmin;     // t_near + surface eps
};

__device__ __forceinline__ float3 f3(float x, float y, float z) { return make_float3(x, y, z); }
__device__ __forceinline__ float3 sub3(float3 a, float3 b) { return f3(a.x - b.x, a.y - b.y, a.z - b.z); }
__device__ __forceinline__ float3 axpy3(float a, float3 x, float3 y) {
  return f3(fmaf(a, x.x, y.x), fmaf(a, x.y, y.y), fmaf(a, x.z, y.z));
}
__device__ __forceinline__ float3 scale3(float a, float3 x) { return f3(a * x.x, a * x.y, a * x.z); }
__device__ __forceinline__ float dot3(float3 a, float3 b) { return fmaf(a.x, b.x, fmaf(a.y, b.y, a.z * b.z)); }
__device__ __forceinline__ float3 cross3(float3 a, float3 b) {
  return f3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ float3 unit3(float3 a) { return scale3(1.f / sqrtf(dot3(a, a)), a); }

// Both roots of |o + t d - c| = r (t0 <= t1). The discriminant comes from the distance
// of the centre to the line, |f x d|^2, which avoids the cancellation of |f|^2 - r^2.
__device__ __forceinline__ bool sphere_roots(const ObjArgs& A, float3 o, float3 d, float* t0, float* t1) {
  const float3 f = sub3(o, A.c);
  const float a = dot3(d, d);
  const float b = dot3(f, d);
  const float3 fx = cross3(f, d);
  const float disc = a * A.rad * A.rad - dot3(fx, fx);
  if (!(disc >= 0.f)) return false;
  const float sq = sqrtf(disc);
  const float ia = 1.f / a;
  *t0 = (-b - sq) * ia;
  *t1 = (-b + sq) * ia;
  return true;
}

// Snell's law for unit d at a surface whose unit normal n faces the ray, eta = n1 / n2;
// false on total internal reflection.
__device__ __forceinline__ bool refract3(float3 d, float3 n, float eta, float3* out) {
  const float ci = -dot3(d, n);
  const float k = 1.f - eta * eta * (1.f - ci * ci);
  if (k < 0.f) return false;
  *out = unit3(axpy3(eta * ci - sqrtf(k), n, scale3(eta, d)));
  return true;
}

__device__ __forceinline__ float3 reflect3(float3 d, float3 n) { return unit3(axpy3(-2.f * dot3(d, n), n, d)); }

__global__ void __launch_bounds__(kObjBlock) k_object_rays(ObjArgs A, const float* __restrict__ ro,
                                                           const float* __restrict__ rd, int64_t count,
                                                           float* __restrict__ t_far, float* __restrict__ next_o,
                                                           float* __restrict__ next_d, float* __restrict__ path,
                                                           int32_t* __restrict__ kind) {
  const int64_t i = blockIdx.x * (int64_t)kObjBlock + threadIdx.x;
  if (i >= count) return;
  const float3 o = f3(ro[3 * i], ro[3 * i + 1], ro[3 * i + 2]);
  const float3 d = f3(rd[3 * i], rd[3 * i + 1], rd[3 * i + 2]);
  float ts = INFINITY, tm = INFINITY, t0, t1;
  if (A.rad > 0.f && sphere_roots(A, o, d, &t0, &t1)) ts = t0 > A.tmin ? t0 : t1 > A.tmin ? t1 : INFINITY;
  if (A.has_mirror) {
    const float dn = dot3(d, A.n);
    if (dn != 0.f) {
      const float th = dot3(sub3(A.m, o), A.n) / dn;
      if (th > A.tmin) {
        const float3 q = sub3(axpy3(th, d, o), A.m);
        const float x = dot3(q, A.u) * A.inv_uu, y = dot3(q, A.v) * A.inv_vv;
        if (fabsf(x) <= 1.f && fabsf(y) <= 1.f) tm = th;
      }
    }
  }
  float3 po = f3(0.f, 0.f, 0.f), pd = f3(0.f, 0.f, 0.f);
  float len = 0.f, tf = INFINITY;
  int k = GRTX_OBJECT_NONE;
  if (tm < ts) {
    po = axpy3(tm, d, o);
    pd = reflect3(d, A.n);
    len = tf = tm;
    k = GRTX_OBJECT_MIRROR;
  } else if (ts < INFINITY) {
    const float inv_r = 1.f / A.rad;
    float3 p = axpy3(ts, d, o), dir = d;
    len = tf = ts;
    k = GRTX_OBJECT_GLASS_TRAPPED;
    bool inside = true;
    const float3 n = scale3(inv_r, sub3(p, A.c));
    if (dot3(dir, n) < 0.f) {
      // entering: refract in, or, where the index forbids entry, reflect away
      float3 in;
      if (refract3(dir, n, 1.f / A.ior, &in)) {
        dir = in;
        if (!sphere_roots(A, p, dir, &t0, &t1)) t1 = 0.f;
        len += t1;
        p = axpy3(t1, dir, p);
      } else {
        po = p;
        pd = reflect3(dir, n);
        k = GRTX_OBJECT_GLASS;
        inside = false;
      }
    }
    // at the surface from inside: refract out, or reflect along another chord
    for (int seg = 0; inside && seg < kMaxInside; ++seg) {
      const float3 nout = scale3(inv_r, sub3(p, A.c));
      float3 out;
      if (refract3(dir, scale3(-1.f, nout), A.ior, &out)) {
        po = p;
        pd = out;
        k = GRTX_OBJECT_GLASS;
        break;
      }
      dir = reflect3(dir, nout);
      if (!sphere_roots(A, p, dir, &t0, &t1)) t1 = 0.f;
      len += t1;
      p = axpy3(t1, dir, p);
    }
  }
  t_far[i] = tf;
  path[i] = len;
  kind[i] = k;
  next_o[3 * i] = po.x;
  next_o[3 * i + 1] = po.y;
  next_o[3 * i + 2] = po.z;
  next_d[3 * i] = pd.x;
  next_d[3 * i + 1] = pd.y;
  next_d[3 * i + 2] = pd.z;
}

// A ray continues when it met a mirror or left the glass and its segment was not ended
// by early termination (its transmittance at the surface is at least T_min).
__global__ void __launch_bounds__(kObjBlock) k_cont_flags(const int32_t* __restrict__ kind,
                                                          const float* __restrict__ opac, float T_min,
                                                          int64_t count, uint32_t* __restrict__ flags) {
  const int64_t i = blockIdx.x * (int64_t)kObjBlock + threadIdx.x;
  if (i >= count) return;
  const int k = kind[i];
  flags[i] = (k == GRTX_OBJECT_MIRROR || k == GRTX_OBJECT_GLASS) && 1.f - opac[i] >= T_min ? 1u : 0u;
}

__global__ void __launch_bounds__(kObjBlock) k_cont_scatter(const uint32_t* __restrict__ flags,
                                                            const uint32_t* __restrict__ offs, int64_t count,
                                                            const float* __restrict__ next_o,
                                                            const float* __restrict__ next_d,
                                                            const float* __restrict__ opac, float* __restrict__ co,
                                                            float* __restrict__ cd, float* __restrict__ ct,
                                                            int32_t* __restrict__ ci) {
  const int64_t i = blockIdx.x * (int64_t)kObjBlock + threadIdx.x;
  if (i >= count || !flags[i]) return;
  const int64_t j = offs[i];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    co[3 * j + a] = next_o[3 * i + a];
    cd[3 * j + a] = next_d[3 * i + a];
  }
  ct[j] = 1.f - opac[i];
  ci[j] = (int32_t)i;
}

__global__ void __launch_bounds__(kObjBlock) k_cont_composite(int64_t n, const int32_t* __restrict__ idx,
                                                              const float* __restrict__ trans,
                                                              const float* __restrict__ path,
                                                              const float* __restrict__ crgb,
                                                              const float* __restrict__ cdepth,
                                                              const float* __restrict__ copac, float* rgb,
                                                              float* depth, float* opac) {
  const int64_t j = blockIdx.x * (int64_t)kObjBlock + threadIdx.x;
  if (j >= n) return;
  const int64_t i = idx[j];
  rgb[3 * i] += crgb[3 * j];
  rgb[3 * i + 1] += crgb[3 * j + 1];
  rgb[3 * i + 2] += crgb[3 * j + 2];
  // the continuation's weights sum to T_start - T_end; its distances start at path[i]
  depth[i] += cdepth[j] + path[i] * (trans[j] - (1.f - copac[j]));
  opac[i] = copac[j];
}

unsigned int grid_of(int64_t n) { return (unsigned int)((n + kObjBlock - 1) / kObjBlock); }

}  // namespace

grtx_status object_rays(const grtx_objects* obj, const grtx_rays* r, float* t_far, float* next_o, float* next_d,
                        float* path, int32_t* kind, hipStream_t s) {
  const int64_t n = r->count;
  if (n == 0) return GRTX_OK;
  ObjArgs A{};
  A.c = make_float3(obj->sphere_center[0], obj->sphere_center[1], obj->sphere_center[2]);
  A.rad = obj->sphere_radius;
  A.ior = obj->sphere_ior;
  A.m = make_float3(obj->mirror_center[0], obj->mirror_center[1], obj->mirror_center[2]);
  A.u = make_float3(obj->mirror_u[0], obj->mirror_u[1], obj->mirror_u[2]);
  A.v = make_float3(obj->mirror_v[0], obj->mirror_v[1], obj->mirror_v[2]);
  // the mirror's unit normal and inverse squared half-axes, once on the host
  const double u[3] = {obj->mirror_u[0], obj->mirror_u[1], obj->mirror_u[2]};
  const double v[3] = {obj->mirror_v[0], obj->mirror_v[1], obj->mirror_v[2]};
  const double c[3] = {u[1] * v[2] - u[2] * v[1], u[2] * v[0] - u[0] * v[2], u[0] * v[1] - u[1] * v[0]};
  const double cl = std::sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
  A.has_mirror = cl > 0.0;
  if (A.has_mirror) {
    A.n = make_float3((float)(c[0] / cl), (float)(c[1] / cl), (float)(c[2] / cl));
    A.inv_uu = (float)(1.0 / (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]));
    A.inv_vv = (float)(1.0 / (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]));
  }
  A.tmin = r->t_near + (obj->surface_eps > 0.f ? obj->surface_eps : 1e-4f);
  hipLaunchKernelGGL(k_object_rays, dim3(grid_of(n)), dim3(kObjBlock), 0, s, A, r->origins, r->dirs, n, t_far,
                     next_o, next_d, path, kind);
  GRTX_LAUNCH_CHECK();
  return GRTX_OK;
}

grtx_status continue_rays(int64_t count, const int32_t* kind, const float* opacity, float T_min,
                          const float* next_o, const float* next_d, float* co, float* cd, float* ct, int32_t* ci,
                          int64_t* n_cont, hipStream_t s) {
  if (count == 0) {
    *n_cont = 0;
    return GRTX_OK;
  }
  Scratch sc(s);
  uint32_t* flags = nullptr;
  GRTX_TRY(sc.get(&flags, 2 * (size_t)count));
  uint32_t* offs = flags + count;
  grtx_status st = GRTX_OK;
  hipLaunchKernelGGL(k_cont_flags, dim3(grid_of(count)), dim3(kObjBlock), 0, s, kind, opacity, T_min, count, flags);
  if (hipGetLastError() != hipSuccess) {
    set_error("continue_rays: flag kernel launch failed");
    st = GRTX_ERR_DEVICE;
  }
  if (st == GRTX_OK) st = exclusive_scan_u32(flags, offs, count, s);
  if (st == GRTX_OK) {
    hipLaunchKernelGGL(k_cont_scatter, dim3(grid_of(count)), dim3(kObjBlock), 0, s, flags, offs, count, next_o,
                       next_d, opacity, co, cd, ct, ci);
    if (hipGetLastError() != hipSuccess) {
      set_error("continue_rays: scatter kernel launch failed");
      st = GRTX_ERR_DEVICE;
    }
  }
  uint32_t tail[2] = {0u, 0u};
  if (st == GRTX_OK &&
      (hipMemcpyAsync(&tail[0], offs + count - 1, sizeof(uint32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
       hipMemcpyAsync(&tail[1], flags + count - 1, sizeof(uint32_t), hipMemcpyDeviceToHost, s) != hipSuccess)) {
    set_error("continue_rays: reading the count failed");
    st = GRTX_ERR_DEVICE;
  }
  const hipError_t es = hipStreamSynchronize(s);
  if (st != GRTX_OK) return st;
  if (es != hipSuccess) {
    set_error("continue_rays: %s", hipGetErrorString(es));
    return GRTX_ERR_DEVICE;
  }
  *n_cont = (int64_t)tail[0] + tail[1];
  return GRTX_OK;
}

grtx_status continue_composite(int64_t n, const int32_t* idx, const float* trans, const float* path,
                               const float* crgb, const float* cdepth, const float* copac, float* rgb, float* depth,
                               float* opac, hipStream_t s) {
  if (n == 0) return GRTX_OK;
  hipLaunchKernelGGL(k_cont_composite, dim3(grid_of(n)), dim3(kObjBlock), 0, s, n, idx, trans, path, crgb, cdepth,
                     copac, rgb, depth, opac);
  GRTX_LAUNCH_CHECK();
  return GRTX_OK;
}

}  // namespace grtx
