// Serving: continuous batching of render requests over several device-resident scenes.
//
// Scenes are merged once into one device scene set (node, leaf and Gaussian indices
// offset per scene; one root entry per scene), so one trace launch can mix rays of any
// scenes: each ray carries its scene index and starts at that scene's root. A worker
// thread admits queued requests while their memory fits the budget, packs every admitted
// request into the next batch (rays of all its requests generated on the device, in 8x8
// tiles per image), and launches the batch on a free stream; batches on different
// streams overlap on the device, so requests that arrive while one batch runs go out in
// the next one without waiting for it. Completion is observed with events; latency is
// measured from submission to the completion of the request's batch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "grtx_internal.h"

namespace grtx {
namespace {

constexpr int kBlock = 256;
constexpr int kMaxBatchRequests = 1024;

// ------------------------------------------------------------------ scene-set merge

__device__ __forceinline__ uint32_t rebase(uint32_t r, uint32_t node_base, uint32_t leaf_base) {
  if (r == kNoChild) return r;
  return (r & kLeafFlag) ? (kLeafFlag | ((r & ~kLeafFlag) + leaf_base)) : r + node_base;
}

__global__ void k_merge_nodes(const float4* __restrict__ src, int64_t n, uint32_t node_base, uint32_t leaf_base,
                              float4* __restrict__ dst) {
  int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x;
  if (i >= n) return;
  const float4* a = src + (int64_t)kNodeF4 * i;
  float4* b = dst + (int64_t)kNodeF4 * i;
  float4 q1 = a[1], q2 = a[2];
  q1.z = __uint_as_float(rebase(__float_as_uint(q1.z), node_base, leaf_base));
  q1.w = __uint_as_float(rebase(__float_as_uint(q1.w), node_base, leaf_base));
  q2.x = __uint_as_float(rebase(__float_as_uint(q2.x), node_base, leaf_base));
  q2.y = __uint_as_float(rebase(__float_as_uint(q2.y), node_base, leaf_base));
  b[0] = a[0];
  b[1] = q1;
  b[2] = q2;
  b[3] = a[3];
}

__global__ void k_merge_inst(const float4* __restrict__ src, int64_t n, uint32_t gauss_base,
                             float4* __restrict__ dst) {
  int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x;
  if (i >= n) return;
  dst[4 * i + 0] = src[4 * i + 0];
  dst[4 * i + 1] = src[4 * i + 1];
  dst[4 * i + 2] = src[4 * i + 2];
  float4 q = src[4 * i + 3];
  q.z = __uint_as_float(__float_as_uint(q.z) + gauss_base);
  dst[4 * i + 3] = q;
}

__global__ void k_merge_root(const float* __restrict__ src, uint32_t node_base, uint32_t leaf_base,
                             float* __restrict__ dst) {
  if (threadIdx.x < 6) dst[threadIdx.x] = src[threadIdx.x];
  if (threadIdx.x == 6) {
    dst[6] = __uint_as_float(rebase(__float_as_uint(src[6]), node_base, leaf_base));
  }
  if (threadIdx.x == 7) dst[7] = 0.f;
}

// ------------------------------------------------------------------ batch rays and outputs

// One request of a batch, as the device sees it.
struct ReqDev {
  float eye[3];
  float fwd[3];
  float right[3];  // right * tan(fov/2) * aspect
  float up[3];     // true up * tan(fov/2)
  int32_t width, height;
  int64_t ray_offset;  // first batch ray of the request
  int32_t scene;
  int32_t tiled;       // rays in 8x8 tiles (width and height multiples of 8)
  const uint32_t* order;  // tile processing order (centre-out) when tiled
  float* rgb;          // request outputs, row-major pixels
  float* depth;
  float* opacity;
};

__device__ __forceinline__ int find_request(const ReqDev* __restrict__ rq, int nreq, int64_t i) {
  int lo = 0, hi = nreq - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (rq[mid].ray_offset <= i) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ int64_t pixel_of(const ReqDev& q, int64_t j) {
  if (!q.tiled) return j;
  const int64_t tiles_x = q.width / 8;
  const int64_t tile = q.order[j >> 6];
  const int within = (int)(j & 63);
  const int64_t ty = tile / tiles_x, tx = tile - ty * tiles_x;
  return (ty * 8 + (within >> 3)) * q.width + tx * 8 + (within & 7);
}

// Rays of every request of the batch; the arithmetic is the single-camera generator's.
__global__ void __launch_bounds__(kBlock) k_batch_rays(const ReqDev* __restrict__ rq, int nreq, int64_t total,
                                                       float* __restrict__ origins, float* __restrict__ dirs,
                                                       int32_t* __restrict__ ray_scene) {
  int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x;
  if (i >= total) return;
  const ReqDev& q = rq[find_request(rq, nreq, i)];
  const int64_t pix = pixel_of(q, i - q.ray_offset);
  const int W = q.width, H = q.height;
  const int y = (int)(pix / W), x = (int)(pix - (int64_t)y * W);
  float sx = 2.f * ((float)x + 0.5f) / (float)W - 1.f;
  float sy = 1.f - 2.f * ((float)y + 0.5f) / (float)H;
  float dx = q.fwd[0] + sx * q.right[0] + sy * q.up[0];
  float dy = q.fwd[1] + sx * q.right[1] + sy * q.up[1];
  float dz = q.fwd[2] + sx * q.right[2] + sy * q.up[2];
  float inv = 1.f / sqrtf(dx * dx + dy * dy + dz * dz);
  origins[3 * i + 0] = q.eye[0];
  origins[3 * i + 1] = q.eye[1];
  origins[3 * i + 2] = q.eye[2];
  dirs[3 * i + 0] = dx * inv;
  dirs[3 * i + 1] = dy * inv;
  dirs[3 * i + 2] = dz * inv;
  ray_scene[i] = q.scene;
}

__global__ void __launch_bounds__(kBlock) k_batch_scatter(const ReqDev* __restrict__ rq, int nreq, int64_t total,
                                                          const float* __restrict__ rgb,
                                                          const float* __restrict__ depth,
                                                          const float* __restrict__ opac) {
  int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x;
  if (i >= total) return;
  const ReqDev& q = rq[find_request(rq, nreq, i)];
  const int64_t pix = pixel_of(q, i - q.ray_offset);
  q.rgb[3 * pix + 0] = rgb[3 * i + 0];
  q.rgb[3 * pix + 1] = rgb[3 * i + 1];
  q.rgb[3 * pix + 2] = rgb[3 * i + 2];
  q.depth[pix] = depth[i];
  q.opacity[pix] = opac[i];
}

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

}  // namespace

// Bytes a request holds while admitted: its rays (origins, directions, scene index), the
// batch outputs and its own outputs.
int64_t request_bytes(const grtx_request* r) {
  const int64_t n = (int64_t)r->width * r->height;
  return n * (24 + 4 + 20 + 20);
}

struct Server {
  grtx_serve_config cfg{};
  int device = 0;
  double t0 = 0.0;
  // merged scene set
  std::vector<const Bvh*> scenes;
  bool frozen = false;
  float4* nodes = nullptr;
  float4* inst = nullptr;
  float* sh = nullptr;
  float* roots = nullptr;
  int sh_degree = -1;
  int64_t total_leaves = 0, total_nodes = 0, total_gauss = 0;
  std::vector<void*> scene_allocs;
  int64_t scene_bytes = 0;
  // slots: one stream each, with batch buffers
  struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    float* rays = nullptr;     // origins then directions
    int32_t* rscene = nullptr;
    float* out = nullptr;      // rgb, depth, opacity
    ReqDev* table_dev = nullptr;
    ReqDev* table_host = nullptr;  // pinned
    int64_t cap = 0;
    bool busy = false;
    std::vector<uint64_t> tickets;
    int64_t rays_in_batch = 0;
  };
  std::vector<Slot> slots;
  int64_t pool_bytes_per_slot = 0;
  // requests
  struct Req {
    grtx_request r{};
    int64_t rays = 0, bytes = 0;
    double t_submit = 0, t_admit = 0, t_launch = 0, t_done = 0;
    float* out = nullptr;
    int state = 0;  // 0 queued, 1 admitted, 2 launched, 3 done, 4 failed
  };
  std::mutex mu;
  std::condition_variable cv;
  std::deque<uint64_t> queued, admitted;
  std::unordered_map<uint64_t, Req> reqs;
  uint64_t next_ticket = 1;
  int64_t in_use = 0, available = 0;
  std::vector<double> latencies;
  int64_t submitted = 0, completed = 0, rays_completed = 0;
  double first_launch = -1.0, last_done = 0.0;
  std::atomic<bool> stop{false};
  std::thread worker;
  char worker_error[512] = "";
};

namespace {

template <class T>
grtx_status sv_alloc(Server* sv, T** p, size_t count) {
  void* q = nullptr;
  GRTX_HIP(hipMalloc(&q, std::max<size_t>(count, 1) * sizeof(T)));
  sv->scene_allocs.push_back(q);
  sv->scene_bytes += (int64_t)(std::max<size_t>(count, 1) * sizeof(T));
  *p = static_cast<T*>(q);
  return GRTX_OK;
}

#define SV_TRY(x)                    \
  do {                               \
    grtx_status st_ = (x);           \
    if (st_ != GRTX_OK) return st_;  \
  } while (0)

grtx_status freeze(Server* sv) {
  if (sv->frozen) return GRTX_OK;
  hipStream_t s = sv->slots[0].stream;
  SV_TRY(sv_alloc(sv, &sv->nodes, kNodeF4 * (size_t)std::max<int64_t>(sv->total_nodes, 1)));
  SV_TRY(sv_alloc(sv, &sv->inst, 4 * (size_t)sv->total_gauss));
  const int ncoef = (sv->sh_degree + 1) * (sv->sh_degree + 1);
  SV_TRY(sv_alloc(sv, &sv->sh, (size_t)sv->total_gauss * 3 * ncoef));
  SV_TRY(sv_alloc(sv, &sv->roots, 8 * sv->scenes.size()));
  int64_t node_base = 0, leaf_base = 0, gauss_base = 0;
  for (size_t i = 0; i < sv->scenes.size(); ++i) {
    const Bvh* b = sv->scenes[i];
    const int64_t slots = b->node_slots;
    if (slots > 0)
      hipLaunchKernelGGL(k_merge_nodes, dim3((unsigned)((slots + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, b->nodes,
                         slots, (uint32_t)node_base, (uint32_t)leaf_base, sv->nodes + kNodeF4 * node_base);
    hipLaunchKernelGGL(k_merge_inst, dim3((unsigned)((b->n_gauss + kBlock - 1) / kBlock)), dim3(kBlock), 0, s,
                       b->inst, b->n_gauss, (uint32_t)gauss_base, sv->inst + 4 * leaf_base);
    GRTX_HIP(hipMemcpyAsync(sv->sh + gauss_base * 3 * ncoef, b->sh, sizeof(float) * 3 * ncoef * b->n_gauss,
                            hipMemcpyDeviceToDevice, s));
    hipLaunchKernelGGL(k_merge_root, dim3(1), dim3(64), 0, s, b->roots, (uint32_t)node_base, (uint32_t)leaf_base,
                       sv->roots + 8 * i);
    GRTX_LAUNCH_CHECK();
    node_base += slots;
    leaf_base += b->n_leaves;
    gauss_base += b->n_gauss;
  }
  GRTX_HIP(hipStreamSynchronize(s));
  sv->available -= sv->scene_bytes;
  sv->frozen = true;
  return GRTX_OK;
}

void camera_basis(const grtx_request& r, ReqDev& q) {
  double f[3], rr[3], u[3];
  for (int a = 0; a < 3; ++a) f[a] = (double)r.target[a] - r.eye[a];
  double fl = std::sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
  for (double& x : f) x /= fl;
  rr[0] = f[1] * r.up[2] - f[2] * r.up[1];
  rr[1] = f[2] * r.up[0] - f[0] * r.up[2];
  rr[2] = f[0] * r.up[1] - f[1] * r.up[0];
  double rl = std::sqrt(rr[0] * rr[0] + rr[1] * rr[1] + rr[2] * rr[2]);
  for (double& x : rr) x /= rl;
  u[0] = rr[1] * f[2] - rr[2] * f[1];
  u[1] = rr[2] * f[0] - rr[0] * f[2];
  u[2] = rr[0] * f[1] - rr[1] * f[0];
  double th = std::tan(0.5 * (double)r.fov_y_deg * M_PI / 180.0);
  double aspect = (double)r.width / (double)r.height;
  for (int a = 0; a < 3; ++a) {
    q.eye[a] = r.eye[a];
    q.fwd[a] = (float)f[a];
    q.right[a] = (float)(rr[a] * th * aspect);
    q.up[a] = (float)(u[a] * th);
  }
  q.width = r.width;
  q.height = r.height;
  q.tiled = (r.width % 8 == 0 && r.height % 8 == 0) ? 1 : 0;
}

// Launch one batch on `slot` with the tickets in `batch` (lock not held).
grtx_status launch_batch(Server* sv, Server::Slot& slot, const std::vector<uint64_t>& batch,
                         const std::vector<Server::Req>& rq) {
  int64_t total = 0;
  for (const auto& r : rq) total += r.rays;
  if (total > slot.cap) {
    if (slot.rays) GRTX_HIP(hipFree(slot.rays));
    if (slot.rscene) GRTX_HIP(hipFree(slot.rscene));
    if (slot.out) GRTX_HIP(hipFree(slot.out));
    GRTX_HIP(hipMalloc(&slot.rays, sizeof(float) * 6 * total));
    GRTX_HIP(hipMalloc(&slot.rscene, sizeof(int32_t) * total));
    GRTX_HIP(hipMalloc(&slot.out, sizeof(float) * 5 * total));
    slot.cap = total;
  }
  int64_t off = 0;
  for (size_t i = 0; i < rq.size(); ++i) {
    ReqDev& q = slot.table_host[i];
    camera_basis(rq[i].r, q);
    q.order = nullptr;
    if (q.tiled) GRTX_TRY(centre_out_order(sv->device, q.width / 8, q.height / 8, &q.order));
    q.ray_offset = off;
    q.scene = rq[i].r.scene_id;
    const int64_t n = rq[i].rays;
    q.rgb = rq[i].out;
    q.depth = rq[i].out + 3 * n;
    q.opacity = rq[i].out + 4 * n;
    off += n;
  }
  hipStream_t s = slot.stream;
  const int nreq = (int)rq.size();
  GRTX_HIP(hipMemcpyAsync(slot.table_dev, slot.table_host, sizeof(ReqDev) * nreq, hipMemcpyHostToDevice, s));
  float* o = slot.rays;
  float* d = slot.rays + 3 * total;
  const unsigned grid = (unsigned)((total + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_batch_rays, dim3(grid), dim3(kBlock), 0, s, slot.table_dev, nreq, total, o, d, slot.rscene);
  GRTX_LAUNCH_CHECK();
  TraceScene sc{sv->nodes, sv->inst, nullptr, sv->sh, sv->sh_degree, sv->roots, slot.rscene,
                GRTX_BVH_SPHERE_INSTANCE, sv->total_leaves};
  grtx_rays rays{o, d, total, 0.f, 0};
  grtx_trace_params p{};
  p.k = sv->cfg.k;
  p.T_min = sv->cfg.T_min;
  p.mode = sv->cfg.mode;
  for (int a = 0; a < 3; ++a) p.bg[a] = sv->cfg.bg[a];
  p.defer_capacity = kServeDeferCap;  // what the slot pools were reserved for
  p.evict_capacity = kServeEvictCap;
  grtx_trace_outputs out{};
  out.rgb = slot.out;
  out.depth = slot.out + 3 * total;
  out.opacity = slot.out + 4 * total;
  SV_TRY(launch_trace(sc, &rays, &p, &out, s));
  hipLaunchKernelGGL(k_batch_scatter, dim3(grid), dim3(kBlock), 0, s, slot.table_dev, nreq, total, out.rgb, out.depth,
                     out.opacity);
  GRTX_LAUNCH_CHECK();
  GRTX_HIP(hipEventRecord(slot.done, s));
  slot.rays_in_batch = total;
  (void)batch;
  return GRTX_OK;
}

void admit_locked(Server* sv) {
  while (!sv->queued.empty()) {
    auto it = sv->reqs.find(sv->queued.front());
    if (it == sv->reqs.end()) {  // released while queued
      sv->queued.pop_front();
      continue;
    }
    auto& r = it->second;
    if (sv->in_use + r.bytes > sv->available) break;  // first come, first served
    void* q = nullptr;
    if (hipMalloc(&q, sizeof(float) * 5 * r.rays) != hipSuccess) break;
    r.out = static_cast<float*>(q);
    sv->in_use += r.bytes;
    r.state = 1;
    r.t_admit = now_s() - sv->t0;
    sv->admitted.push_back(sv->queued.front());
    sv->queued.pop_front();
  }
}

void worker_main(Server* sv) {
  (void)hipSetDevice(sv->device);
  while (!sv->stop.load()) {
    bool progressed = false;
    // completions
    for (auto& slot : sv->slots) {
      if (!slot.busy) continue;
      hipError_t q = hipEventQuery(slot.done);
      if (q == hipErrorNotReady) continue;
      std::lock_guard<std::mutex> g(sv->mu);
      const double t = now_s() - sv->t0;
      for (uint64_t tk : slot.tickets) {
        auto it = sv->reqs.find(tk);
        if (it == sv->reqs.end()) continue;
        it->second.state = q == hipSuccess ? 3 : 4;
        it->second.t_done = t;
        if (q == hipSuccess) {
          sv->latencies.push_back(t - it->second.t_submit);
          ++sv->completed;
          sv->rays_completed += it->second.rays;
        }
      }
      if (q != hipSuccess) snprintf(sv->worker_error, sizeof sv->worker_error, "batch failed: %s", hipGetErrorString(q));
      sv->last_done = t;
      slot.tickets.clear();
      slot.busy = false;
      progressed = true;
      sv->cv.notify_all();
    }
    // admission and launch
    for (auto& slot : sv->slots) {
      if (slot.busy) continue;
      std::vector<uint64_t> batch;
      std::vector<Server::Req> rq;
      {
        std::lock_guard<std::mutex> g(sv->mu);
        admit_locked(sv);
        int64_t rays = 0;
        const double t_launch = now_s() - sv->t0;
        while (!sv->admitted.empty() && (int)batch.size() < kMaxBatchRequests) {
          auto& r = sv->reqs[sv->admitted.front()];
          if (!batch.empty() && rays + r.rays > sv->cfg.max_batch_rays) break;
          batch.push_back(sv->admitted.front());
          sv->admitted.pop_front();
          r.state = 2;
          r.t_launch = t_launch;
          rays += r.rays;
          rq.push_back(r);
        }
        if (!batch.empty() && sv->first_launch < 0) sv->first_launch = rq.front().t_launch;
      }
      if (batch.empty()) break;
      grtx_status st = launch_batch(sv, slot, batch, rq);
      std::lock_guard<std::mutex> g(sv->mu);
      if (st != GRTX_OK) {
        snprintf(sv->worker_error, sizeof sv->worker_error, "launch failed: %s", grtx_last_error());
        for (uint64_t tk : batch) sv->reqs[tk].state = 4;
        sv->cv.notify_all();
      } else {
        slot.tickets = batch;
        slot.busy = true;
      }
      progressed = true;
    }
    if (!progressed) {
      std::unique_lock<std::mutex> lk(sv->mu);
      sv->cv.wait_for(lk, std::chrono::microseconds(50));
    }
  }
}

}  // namespace

grtx_status serve_create(const grtx_serve_config* cfg, Server** out) {
  auto* sv = new Server();
  sv->cfg = *cfg;
  if (sv->cfg.slots <= 0) sv->cfg.slots = 2;
  if (sv->cfg.max_batch_rays <= 0) sv->cfg.max_batch_rays = 1 << 23;
  sv->t0 = now_s();
  hipError_t e = hipGetDevice(&sv->device);
  if (e != hipSuccess) {
    set_error("grtx_serve_create: %s", hipGetErrorString(e));
    delete sv;
    return GRTX_ERR_DEVICE;
  }
  // the checkpoint pool of each slot's trace launches counts against the budget
  const int K = cfg->k <= 4 ? 4 : cfg->k <= 8 ? 8 : cfg->k <= 16 ? 16 : cfg->k <= 32 ? 32 : 64;
  sv->pool_bytes_per_slot = trace_pool_bytes(K, kServeDeferCap, kServeEvictCap);
  sv->available = cfg->memory_budget - sv->cfg.slots * sv->pool_bytes_per_slot;
  if (sv->available <= 0) {
    set_error("grtx_serve_create: budget %lld bytes is below the %d slots' checkpoint pools (%lld bytes each)",
              (long long)cfg->memory_budget, sv->cfg.slots, (long long)sv->pool_bytes_per_slot);
    delete sv;
    return GRTX_ERR_CAPACITY;
  }
  sv->slots.resize(sv->cfg.slots);
  for (auto& slot : sv->slots) {
    if (hipStreamCreateWithFlags(&slot.stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&slot.done, hipEventDisableTiming) != hipSuccess ||
        hipMalloc(&slot.table_dev, sizeof(ReqDev) * kMaxBatchRequests) != hipSuccess ||
        hipHostMalloc(&slot.table_host, sizeof(ReqDev) * kMaxBatchRequests, hipHostMallocDefault) != hipSuccess) {
      set_error("grtx_serve_create: stream/buffer setup failed");
      serve_destroy(sv);
      return GRTX_ERR_DEVICE;
    }
  }
  sv->worker = std::thread(worker_main, sv);
  *out = sv;
  return GRTX_OK;
}

grtx_status serve_add_scene(Server* sv, const Bvh* b, int32_t* scene_id) {
  std::lock_guard<std::mutex> g(sv->mu);
  if (sv->frozen) {
    set_error("grtx_serve_add_scene: scenes must be added before the first request");
    return GRTX_ERR_INVALID_ARG;
  }
  if (b->kind != GRTX_BVH_SPHERE_INSTANCE || b->n_gauss == 0) {
    set_error("grtx_serve_add_scene: serving takes non-empty unit-sphere instance structures");
    return GRTX_ERR_INVALID_ARG;
  }
  if (sv->sh_degree >= 0 && b->sh_degree != sv->sh_degree) {
    set_error("grtx_serve_add_scene: all scenes must share one SH degree");
    return GRTX_ERR_INVALID_ARG;
  }
  if (sv->total_leaves + b->n_leaves >= (int64_t)kLeafFlag) {
    set_error("grtx_serve_add_scene: scene set too large");
    return GRTX_ERR_CAPACITY;
  }
  GRTX_HIP(hipStreamSynchronize(b->build_stream));
  sv->sh_degree = b->sh_degree;
  sv->scenes.push_back(b);
  sv->total_nodes += b->node_slots;
  sv->total_leaves += b->n_leaves;
  sv->total_gauss += b->n_gauss;
  *scene_id = (int32_t)sv->scenes.size() - 1;
  return GRTX_OK;
}

grtx_status serve_submit(Server* sv, const grtx_request* r, uint64_t* ticket) {
  std::lock_guard<std::mutex> g(sv->mu);
  if (r->scene_id < 0 || r->scene_id >= (int32_t)sv->scenes.size()) {
    set_error("grtx_serve_submit: unknown scene %d", r->scene_id);
    return GRTX_ERR_INVALID_ARG;
  }
  if (!sv->frozen) SV_TRY(freeze(sv));
  Server::Req q;
  q.r = *r;
  q.rays = (int64_t)r->width * r->height;
  q.bytes = request_bytes(r);
  if (q.bytes > sv->available || q.rays > sv->cfg.max_batch_rays) {
    set_error("grtx_serve_submit: request needs %lld bytes / %lld rays; the server holds %lld bytes / %lld rays",
              (long long)q.bytes, (long long)q.rays, (long long)sv->available, (long long)sv->cfg.max_batch_rays);
    return GRTX_ERR_CAPACITY;
  }
  q.t_submit = now_s() - sv->t0;
  const uint64_t t = sv->next_ticket++;
  sv->reqs.emplace(t, q);
  sv->queued.push_back(t);
  ++sv->submitted;
  sv->cv.notify_all();
  *ticket = t;
  return GRTX_OK;
}

grtx_status serve_poll(Server* sv, uint64_t ticket, grtx_request_result* res) {
  std::lock_guard<std::mutex> g(sv->mu);
  auto it = sv->reqs.find(ticket);
  if (it == sv->reqs.end()) {
    set_error("grtx_serve_poll: unknown ticket %llu", (unsigned long long)ticket);
    return GRTX_ERR_INVALID_ARG;
  }
  const Server::Req& q = it->second;
  if (q.state == 4) {
    set_error("grtx_serve_poll: %s", sv->worker_error);
    return GRTX_ERR_DEVICE;
  }
  if (q.state != 3) return GRTX_ERR_NOT_READY;
  grtx_request_result r{};
  r.rgb = q.out;
  r.depth = q.out + 3 * q.rays;
  r.opacity = q.out + 4 * q.rays;
  r.width = q.r.width;
  r.height = q.r.height;
  r.t_submit = q.t_submit;
  r.t_admit = q.t_admit;
  r.t_launch = q.t_launch;
  r.t_done = q.t_done;
  *res = r;
  return GRTX_OK;
}

grtx_status serve_release(Server* sv, uint64_t ticket) {
  std::lock_guard<std::mutex> g(sv->mu);
  auto it = sv->reqs.find(ticket);
  if (it == sv->reqs.end()) {
    set_error("grtx_serve_release: unknown ticket %llu", (unsigned long long)ticket);
    return GRTX_ERR_INVALID_ARG;
  }
  if (it->second.state == 1 || it->second.state == 2) {
    set_error("grtx_serve_release: request %llu is still in flight", (unsigned long long)ticket);
    return GRTX_ERR_NOT_READY;
  }
  if (it->second.state == 0) {
    // withdrawn before admission: it leaves the queue and is never launched or counted
    auto q = std::find(sv->queued.begin(), sv->queued.end(), ticket);
    if (q != sv->queued.end()) sv->queued.erase(q);
    --sv->submitted;
  }
  if (it->second.out) {
    GRTX_HIP(hipFree(it->second.out));
    sv->in_use -= it->second.bytes;
  }
  sv->reqs.erase(it);
  sv->cv.notify_all();
  return GRTX_OK;
}

grtx_status serve_stats(Server* sv, grtx_serve_stats* st) {
  std::lock_guard<std::mutex> g(sv->mu);
  grtx_serve_stats s{};
  s.submitted = sv->submitted;
  s.completed = sv->completed;
  s.rays_completed = sv->rays_completed;
  s.bytes_in_use = sv->in_use;
  s.bytes_available = sv->available;
  std::vector<double> l = sv->latencies;
  if (!l.empty()) {
    std::sort(l.begin(), l.end());
    auto pct = [&](double p) {
      double idx = p * (double)(l.size() - 1);
      size_t lo = (size_t)std::floor(idx), hi = (size_t)std::ceil(idx);
      return 1e3 * (l[lo] + (l[hi] - l[lo]) * (idx - (double)lo));
    };
    s.p50_ms = pct(0.50);
    s.p99_ms = pct(0.99);
    double sum = 0.0;
    for (double x : l) sum += x;
    s.mean_ms = 1e3 * sum / (double)l.size();
    s.max_ms = 1e3 * l.back();
  }
  if (sv->first_launch >= 0 && sv->last_done > sv->first_launch) {
    s.busy_s = sv->last_done - sv->first_launch;
    s.mrays_per_s = (double)sv->rays_completed / s.busy_s / 1e6;
  }
  *st = s;
  return GRTX_OK;
}

grtx_status serve_destroy(Server* sv) {
  if (sv->worker.joinable()) {
    sv->stop.store(true);
    sv->cv.notify_all();
    sv->worker.join();
  }
  for (auto& slot : sv->slots) {
    if (slot.stream) (void)hipStreamSynchronize(slot.stream);
    if (slot.rays) (void)hipFree(slot.rays);
    if (slot.rscene) (void)hipFree(slot.rscene);
    if (slot.out) (void)hipFree(slot.out);
    if (slot.table_dev) (void)hipFree(slot.table_dev);
    if (slot.table_host) (void)hipHostFree(slot.table_host);
    if (slot.done) (void)hipEventDestroy(slot.done);
    if (slot.stream) (void)hipStreamDestroy(slot.stream);
  }
  for (auto& kv : sv->reqs)
    if (kv.second.out) (void)hipFree(kv.second.out);
  for (void* p : sv->scene_allocs) (void)hipFree(p);
  delete sv;
  return GRTX_OK;
}

}  // namespace grtx
