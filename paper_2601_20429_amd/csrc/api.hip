// C ABI entry points: argument validation, handle lifetimes, error reporting.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstring>
#include <new>

#include "grtx_internal.h"

namespace grtx {

static thread_local char g_err[1024] = "";

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
}

void clear_error() { g_err[0] = '\0'; }

}  // namespace grtx

using grtx::set_error;

#define CHECK_ARG(cond, ...)        \
  do {                              \
    if (!(cond)) {                  \
      set_error(__VA_ARGS__);       \
      return GRTX_ERR_INVALID_ARG;  \
    }                               \
  } while (0)

extern "C" {

const char* grtx_last_error(void) { return grtx::g_err; }

int32_t grtx_version(void) { return GRTX_VERSION; }

grtx_status grtx_build(const grtx_gaussians* g, grtx_bvh_kind kind, const grtx_build_params* p, void* stream,
                       grtx_bvh** out) {
  grtx::clear_error();
  CHECK_ARG(g && p && out, "grtx_build: null argument");
  CHECK_ARG(g->count >= 0, "grtx_build: negative Gaussian count");
  CHECK_ARG(g->count < (int64_t)0x7FFFFFFF / 20, "grtx_build: too many Gaussians (%lld)", (long long)g->count);
  CHECK_ARG(g->sh_degree >= 0 && g->sh_degree <= 3, "grtx_build: sh_degree must be 0..3, got %d", g->sh_degree);
  CHECK_ARG(kind == GRTX_BVH_SPHERE_INSTANCE || kind == GRTX_BVH_PROXY20 || kind == GRTX_BVH_ICO_INSTANCE,
            "grtx_build: unknown kind %d", (int)kind);
  CHECK_ARG(p->alpha_min > 0.f && p->alpha_min < 1.f, "grtx_build: alpha_min must be in (0,1)");
  CHECK_ARG(p->max_depth >= 0 && p->max_depth <= GRTX_MAX_TREE_DEPTH, "grtx_build: max_depth must be 0..%d",
            GRTX_MAX_TREE_DEPTH);
  if (g->count > 0)
    CHECK_ARG(g->means && g->scales && g->quats && g->opacities && g->sh, "grtx_build: null Gaussian array");
  grtx_bvh* h = new (std::nothrow) grtx_bvh();
  if (!h) {
    set_error("grtx_build: host allocation failed");
    return GRTX_ERR_OUT_OF_MEMORY;
  }
  grtx_status st =
      grtx::build_bvh(g, kind, p->alpha_min, p->plain_lbvh == 0, p->max_depth > 0 ? p->max_depth : GRTX_MAX_TREE_DEPTH,
                      static_cast<hipStream_t>(stream), &h->impl);
  if (st != GRTX_OK) {
    char msg[1024];
    std::strncpy(msg, grtx::g_err, sizeof msg - 1);
    msg[sizeof msg - 1] = 0;
    for (void* q : h->impl.allocations) (void)hipFree(q);
    delete h;
    set_error("%s", msg);
    return st;
  }
  *out = h;
  return GRTX_OK;
}

grtx_status grtx_bvh_get_info(const grtx_bvh* bvh, grtx_bvh_info* out) {
  grtx::clear_error();
  CHECK_ARG(bvh && out, "grtx_bvh_get_info: null argument");
  const grtx::Bvh& b = bvh->impl;
  grtx_bvh_info info{};
  info.gaussians = b.n_gauss;
  info.leaves = b.n_leaves;
  info.internal_nodes = b.n_leaves > 1 ? b.n_leaves - 1 : 0;
  info.device_bytes = (int64_t)b.bytes;
  info.kind = b.kind;
  info.sh_degree = b.sh_degree;
  info.alpha_min = b.alpha_min;
  if (b.n_leaves > 0) {
    float box[6];
    uint32_t depth[2] = {0u, 0u};
    GRTX_HIP(hipStreamSynchronize(b.build_stream));
    GRTX_HIP(hipMemcpy(box, b.root_box, sizeof box, hipMemcpyDeviceToHost));
    GRTX_HIP(hipMemcpy(depth, b.depth, sizeof depth, hipMemcpyDeviceToHost));
    for (int a = 0; a < 3; ++a) {
      info.root_lo[a] = box[a];
      info.root_hi[a] = box[3 + a];
    }
    info.depth = (int32_t)depth[0];
    info.restructured = (int32_t)depth[1];
  }
  *out = info;
  return GRTX_OK;
}

grtx_status grtx_bvh_export_topology(const grtx_bvh* bvh, uint32_t* child, uint32_t* parent, uint64_t* morton,
                                     uint32_t* perm, float* boxes, void* stream) {
  grtx::clear_error();
  CHECK_ARG(bvh, "grtx_bvh_export_topology: null handle");
  return grtx::export_topology(&bvh->impl, child, parent, morton, perm, boxes, static_cast<hipStream_t>(stream));
}

grtx_status grtx_bvh_destroy(grtx_bvh* bvh) {
  grtx::clear_error();
  if (!bvh) return GRTX_OK;
  grtx_status st = GRTX_OK;
  for (void* q : bvh->impl.allocations) {
    hipError_t e = hipFree(q);
    if (e != hipSuccess && st == GRTX_OK) {
      set_error("grtx_bvh_destroy: hipFree failed: %s", hipGetErrorString(e));
      st = GRTX_ERR_DEVICE;
    }
  }
  delete bvh;
  return st;
}

grtx_status grtx_pinhole_rays(const grtx_camera* cam, float* origins, float* dirs, void* stream) {
  grtx::clear_error();
  CHECK_ARG(cam && origins && dirs, "grtx_pinhole_rays: null argument");
  CHECK_ARG(cam->width > 0 && cam->height > 0, "grtx_pinhole_rays: image size must be positive");
  CHECK_ARG(cam->fov_y_deg > 0.f && cam->fov_y_deg < 180.f, "grtx_pinhole_rays: fov must be in (0,180)");
  return grtx::pinhole_rays(cam, origins, dirs, static_cast<hipStream_t>(stream));
}

// Host-side checks shared by grtx_trace and grtx_trace_noalloc.
static grtx_status check_trace_args(const char* fn, const grtx_bvh* bvh, const grtx_rays* rays,
                                    const grtx_trace_params* p, const grtx_trace_outputs* out) {
  CHECK_ARG(bvh && rays && p && out, "%s: null argument", fn);
  CHECK_ARG(rays->count >= 0 && rays->count < ((int64_t)1 << 40), "%s: bad ray count", fn);
  CHECK_ARG(p->k >= 1 && p->k <= 64, "%s: k must be 1..64, got %d", fn, p->k);
  CHECK_ARG(p->T_min >= 0.f && p->T_min < 1.f, "%s: T_min must be in [0,1)", fn);
  CHECK_ARG(p->mode == GRTX_MODE_CHECKPOINT || p->mode == GRTX_MODE_RESTART || p->mode == GRTX_MODE_SINGLE_ROUND,
            "%s: unknown mode %d", fn, p->mode);
  CHECK_ARG(p->collect_capacity >= 0 && p->collect_capacity <= 8192, "%s: collect_capacity must be 0..8192", fn);
  CHECK_ARG(p->defer_capacity >= 0 && p->evict_capacity >= 0 && p->defer_capacity <= (1 << 20) &&
                p->evict_capacity <= (1 << 20),
            "%s: list capacities must be 0..2^20", fn);
  CHECK_ARG(rays->t_near >= 0.f && std::isfinite(rays->t_near), "%s: t_near must be finite and >= 0", fn);
  CHECK_ARG(rays->image_width >= 0, "%s: negative image width", fn);
  CHECK_ARG(rays->image_begin >= 0 && rays->image_begin <= rays->count, "%s: image_begin must be 0..count", fn);
  CHECK_ARG(rays->image_begin == 0 || rays->image_width > 0, "%s: image_begin given without image_width", fn);
  {
    int64_t n_free = 0, image_h = 0;
    const int64_t work = grtx::trace_work_items(rays, &n_free, &image_h);
    CHECK_ARG(work <= grtx::kMaxTraceWork,
              "%s: %lld rays make %lld work items (an image's 8x8 tiles count whole); one launch takes at most "
              "2^31-1", fn, (long long)rays->count, (long long)work);
  }
  {
    const int nc = !!rays->next_origins + !!rays->next_dirs + !!rays->path + !!rays->kind;
    CHECK_ARG(nc == 0 || nc == 4, "%s: give all four continuation arrays or none", fn);
    CHECK_ARG(nc == 0 || (rays->t_far && rays->t_near == 0.f), "%s: continuation rays need t_far and t_near = 0",
              fn);
  }
  if (rays->count > 0) {
    CHECK_ARG(rays->origins && rays->dirs, "%s: null ray arrays", fn);
    CHECK_ARG(out->rgb && out->depth && out->opacity, "%s: null output arrays", fn);
    CHECK_ARG(!out->hit_ids || out->hit_capacity > 0, "%s: hit_ids given with hit_capacity <= 0", fn);
  }
  return GRTX_OK;
}

grtx_status grtx_trace_noalloc(const grtx_bvh* bvh, const grtx_rays* rays, const grtx_trace_params* p,
                               const grtx_trace_outputs* out, void* stream) {
  grtx::clear_error();
  grtx_status st = check_trace_args("grtx_trace_noalloc", bvh, rays, p, out);
  if (st != GRTX_OK) return st;
  return grtx::trace_noalloc(&bvh->impl, rays, p, out, static_cast<hipStream_t>(stream));
}

grtx_status grtx_trace(const grtx_bvh* bvh, const grtx_rays* rays, const grtx_trace_params* p,
                       const grtx_trace_outputs* out, void* stream) {
  grtx::clear_error();
  grtx_status st = check_trace_args("grtx_trace", bvh, rays, p, out);
  if (st != GRTX_OK) return st;
  return grtx::trace(&bvh->impl, rays, p, out, static_cast<hipStream_t>(stream));
}

grtx_status grtx_trace_backward(const grtx_bvh* bvh, const grtx_gaussians* g, const grtx_rays* rays,
                                const grtx_trace_params* p, const grtx_trace_outputs* fwd, const float* grad_rgb,
                                const float* grad_depth, const float* grad_opacity, const grtx_gaussian_grads* grads,
                                uint32_t* truncated_rays, void* stream) {
  grtx::clear_error();
  CHECK_ARG(bvh && g && rays && p && fwd && grads, "grtx_trace_backward: null argument");
  CHECK_ARG(g->count == bvh->impl.n_gauss && g->sh_degree == bvh->impl.sh_degree,
            "grtx_trace_backward: Gaussians differ from those the structure was built from");
  CHECK_ARG(rays->count >= 0 && rays->count <= grtx::kMaxTraceWork, "grtx_trace_backward: bad ray count");
  if (rays->count > 0 && g->count > 0) {
    CHECK_ARG(g->means && g->scales && g->quats && g->opacities && g->sh, "grtx_trace_backward: null Gaussian array");
    CHECK_ARG(rays->origins && rays->dirs, "grtx_trace_backward: null ray arrays");
    CHECK_ARG(!fwd->hit_ids || (fwd->rgb && fwd->depth && fwd->opacity && fwd->hit_counts && fwd->hit_capacity > 0),
              "grtx_trace_backward: with a hit-id list the forward outputs need rgb, depth, opacity and hit counts");
    CHECK_ARG(fwd->hit_capacity >= 0, "grtx_trace_backward: negative hit capacity");
    CHECK_ARG(p->k >= 1 && p->k <= 64 && p->T_min >= 0.f && p->T_min < 1.f &&
                  (p->mode == GRTX_MODE_CHECKPOINT || p->mode == GRTX_MODE_RESTART ||
                   p->mode == GRTX_MODE_SINGLE_ROUND) &&
                  p->collect_capacity >= 0 && p->collect_capacity <= 8192 && p->defer_capacity >= 0 &&
                  p->evict_capacity >= 0 && p->defer_capacity <= (1 << 20) && p->evict_capacity <= (1 << 20),
              "grtx_trace_backward: bad trace parameters");
    CHECK_ARG(grad_rgb || grad_depth || grad_opacity, "grtx_trace_backward: no output gradient given");
    CHECK_ARG(!rays->t_far && !rays->transmittance && !rays->kind,
              "grtx_trace_backward: rays with t_far, a starting transmittance or continuation rays are not "
              "supported");
    CHECK_ARG(grads->means && grads->scales && grads->quats && grads->opacities && grads->sh,
              "grtx_trace_backward: null gradient array");
  }
  static thread_local unsigned int* own = nullptr;
  static thread_local int own_dev = -1;
  unsigned int* tr = truncated_rays;
  if (!tr) {
    int dev = 0;
    GRTX_HIP(hipGetDevice(&dev));
    if (!own || own_dev != dev) {
      GRTX_HIP(hipMalloc(&own, sizeof(unsigned int)));
      own_dev = dev;
    }
    tr = own;
  }
  return grtx::trace_backward(&bvh->impl, g, rays, p, fwd, grad_rgb, grad_depth, grad_opacity, grads, tr,
                              static_cast<hipStream_t>(stream));
}

grtx_status grtx_object_rays(const grtx_objects* obj, const grtx_rays* rays, float* t_far, float* next_origins,
                             float* next_dirs, float* path, int32_t* kind, void* stream) {
  grtx::clear_error();
  CHECK_ARG(obj && rays, "grtx_object_rays: null argument");
  CHECK_ARG(rays->count >= 0 && rays->count < ((int64_t)1 << 40), "grtx_object_rays: bad ray count");
  CHECK_ARG(rays->t_near >= 0.f && std::isfinite(rays->t_near), "grtx_object_rays: t_near must be finite and >= 0");
  CHECK_ARG(obj->surface_eps >= 0.f && std::isfinite(obj->surface_eps), "grtx_object_rays: bad surface_eps");
  bool finite = std::isfinite(obj->sphere_radius) && std::isfinite(obj->sphere_ior);
  for (int a = 0; a < 3; ++a)
    finite = finite && std::isfinite(obj->sphere_center[a]) && std::isfinite(obj->mirror_center[a]) &&
             std::isfinite(obj->mirror_u[a]) && std::isfinite(obj->mirror_v[a]);
  CHECK_ARG(finite, "grtx_object_rays: non-finite object parameter");
  CHECK_ARG(obj->sphere_radius <= 0.f || obj->sphere_ior > 0.f, "grtx_object_rays: sphere_ior must be positive");
  {
    double uu = 0, vv = 0, uv = 0;
    for (int a = 0; a < 3; ++a) {
      uu += (double)obj->mirror_u[a] * obj->mirror_u[a];
      vv += (double)obj->mirror_v[a] * obj->mirror_v[a];
      uv += (double)obj->mirror_u[a] * obj->mirror_v[a];
    }
    CHECK_ARG(std::fabs(uv) <= 1e-4 * std::sqrt(uu * vv), "grtx_object_rays: mirror half-axes must be orthogonal");
  }
  if (rays->count > 0) {
    CHECK_ARG(rays->origins && rays->dirs, "grtx_object_rays: null ray arrays");
    CHECK_ARG(t_far && next_origins && next_dirs && path && kind, "grtx_object_rays: null output array");
  }
  return grtx::object_rays(obj, rays, t_far, next_origins, next_dirs, path, kind, static_cast<hipStream_t>(stream));
}

grtx_status grtx_continue_rays(int64_t count, const int32_t* kind, const float* opacity, float T_min,
                               const float* next_origins, const float* next_dirs, float* cont_origins,
                               float* cont_dirs, float* cont_transmittance, int32_t* cont_index, int64_t* n_cont,
                               void* stream) {
  grtx::clear_error();
  CHECK_ARG(n_cont, "grtx_continue_rays: null n_cont");
  CHECK_ARG(count >= 0 && count <= ((int64_t)1 << 24), "grtx_continue_rays: count must be 0..2^24");
  CHECK_ARG(T_min >= 0.f && T_min < 1.f, "grtx_continue_rays: T_min must be in [0,1)");
  if (count > 0)
    CHECK_ARG(kind && opacity && next_origins && next_dirs && cont_origins && cont_dirs && cont_transmittance &&
                  cont_index,
              "grtx_continue_rays: null array");
  return grtx::continue_rays(count, kind, opacity, T_min, next_origins, next_dirs, cont_origins, cont_dirs,
                             cont_transmittance, cont_index, n_cont, static_cast<hipStream_t>(stream));
}

grtx_status grtx_continue_composite(int64_t n, const int32_t* cont_index, const float* cont_transmittance,
                                    const float* path, const float* cont_rgb, const float* cont_depth,
                                    const float* cont_opacity, float* rgb, float* depth, float* opacity,
                                    void* stream) {
  grtx::clear_error();
  CHECK_ARG(n >= 0 && n < ((int64_t)1 << 31), "grtx_continue_composite: n must be 0..2^31-1");
  if (n > 0)
    CHECK_ARG(cont_index && cont_transmittance && path && cont_rgb && cont_depth && cont_opacity && rgb && depth &&
                  opacity,
              "grtx_continue_composite: null array");
  return grtx::continue_composite(n, cont_index, cont_transmittance, path, cont_rgb, cont_depth, cont_opacity, rgb,
                                  depth, opacity, static_cast<hipStream_t>(stream));
}

grtx_status grtx_serve_request_bytes(const grtx_request* r, int64_t* bytes) {
  grtx::clear_error();
  CHECK_ARG(r && bytes, "grtx_serve_request_bytes: null argument");
  CHECK_ARG(r->width > 0 && r->height > 0, "grtx_serve_request_bytes: image size must be positive");
  *bytes = grtx::request_bytes(r);
  return GRTX_OK;
}

grtx_status grtx_serve_create(const grtx_serve_config* cfg, grtx_server** out) {
  grtx::clear_error();
  CHECK_ARG(cfg && out, "grtx_serve_create: null argument");
  CHECK_ARG(cfg->memory_budget > 0, "grtx_serve_create: memory_budget must be positive");
  CHECK_ARG(cfg->k >= 1 && cfg->k <= 64, "grtx_serve_create: k must be 1..64");
  CHECK_ARG(cfg->T_min >= 0.f && cfg->T_min < 1.f, "grtx_serve_create: T_min must be in [0,1)");
  CHECK_ARG(cfg->mode == GRTX_MODE_CHECKPOINT || cfg->mode == GRTX_MODE_RESTART, "grtx_serve_create: unknown mode");
  CHECK_ARG(cfg->max_request_rays >= 0 && cfg->max_request_rays <= (1 << grtx::kServePixelBits),
            "grtx_serve_create: max_request_rays must be 0..2^22");
  CHECK_ARG(cfg->idle_exit_us >= 0 && cfg->idle_exit_us <= 10000000, "grtx_serve_create: idle_exit_us must be 0..1e7");
  grtx::Server* sv = nullptr;
  grtx_status st = grtx::serve_create(cfg, &sv);
  if (st != GRTX_OK) return st;
  grtx_server* h = new (std::nothrow) grtx_server{sv};
  if (!h) {
    grtx::serve_destroy(sv);
    set_error("grtx_serve_create: host allocation failed");
    return GRTX_ERR_OUT_OF_MEMORY;
  }
  *out = h;
  return GRTX_OK;
}

grtx_status grtx_serve_add_scene(grtx_server* s, const grtx_bvh* bvh, int32_t* scene_id) {
  grtx::clear_error();
  CHECK_ARG(s && bvh && scene_id, "grtx_serve_add_scene: null argument");
  return grtx::serve_add_scene(s->impl, &bvh->impl, scene_id);
}

grtx_status grtx_serve_submit(grtx_server* s, const grtx_request* r, uint64_t* ticket) {
  grtx::clear_error();
  CHECK_ARG(s && r && ticket, "grtx_serve_submit: null argument");
  CHECK_ARG(r->width > 0 && r->height > 0, "grtx_serve_submit: image size must be positive");
  CHECK_ARG(r->fov_y_deg > 0.f && r->fov_y_deg < 180.f, "grtx_serve_submit: fov must be in (0,180)");
  return grtx::serve_submit(s->impl, r, ticket);
}

grtx_status grtx_serve_poll(grtx_server* s, uint64_t ticket, grtx_request_result* res) {
  grtx::clear_error();
  CHECK_ARG(s && res, "grtx_serve_poll: null argument");
  return grtx::serve_poll(s->impl, ticket, res);
}

grtx_status grtx_serve_copy_result(grtx_server* s, uint64_t ticket, float* rgb, float* depth, float* opacity,
                                   void* stream) {
  grtx::clear_error();
  CHECK_ARG(s, "grtx_serve_copy_result: null argument");
  grtx_request_result r{};
  grtx_status st = grtx::serve_poll(s->impl, ticket, &r);
  if (st != GRTX_OK) return st;
  const size_t n = (size_t)r.width * r.height;
  hipStream_t hs = static_cast<hipStream_t>(stream);
  if (rgb) GRTX_HIP(hipMemcpyAsync(rgb, r.rgb, sizeof(float) * 3 * n, hipMemcpyDeviceToDevice, hs));
  if (depth) GRTX_HIP(hipMemcpyAsync(depth, r.depth, sizeof(float) * n, hipMemcpyDeviceToDevice, hs));
  if (opacity) GRTX_HIP(hipMemcpyAsync(opacity, r.opacity, sizeof(float) * n, hipMemcpyDeviceToDevice, hs));
  return GRTX_OK;
}

grtx_status grtx_serve_release(grtx_server* s, uint64_t ticket) {
  grtx::clear_error();
  CHECK_ARG(s, "grtx_serve_release: null argument");
  return grtx::serve_release(s->impl, ticket);
}

grtx_status grtx_serve_get_stats(grtx_server* s, grtx_serve_stats* st) {
  grtx::clear_error();
  CHECK_ARG(s && st, "grtx_serve_get_stats: null argument");
  return grtx::serve_stats(s->impl, st);
}

grtx_status grtx_serve_destroy(grtx_server* s) {
  grtx::clear_error();
  if (!s) return GRTX_OK;
  grtx_status st = grtx::serve_destroy(s->impl);
  delete s;
  return st;
}

}  // extern "C"
