// Serving: render requests over several device-resident scenes, traced by one persistent
// kernel that takes work from a queue the host appends to.
//
// Scenes are merged once into one device scene set (node, leaf and Gaussian indices
// offset per scene; one root entry per scene), so one launch can trace rays of any scene:
// each ray carries its scene index and starts at that scene's root. A worker thread
// admits queued requests first come, first served while their outputs fit the memory
// budget (their outputs are placed in a pooled device arena) and publishes each admitted
// request to the work queue; the serving kernel, launched when work is published and no
// launch is running, takes the requests' 8x8 pixel tiles as its lanes fall idle,
// generates their rays from the request's camera, writes each pixel's outputs, and raises
// the request's flag in host memory when its last pixel is written. A request that arrives
// while the kernel runs joins it: its tiles go to the next lanes that fall idle. The
// kernel ends once no work has been taken for the idle time (or the server stops), and
// the next publication starts it again. Latency is measured from submission to the
// worker seeing the request's flag.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "camera.h"
#include "grtx_internal.h"

namespace grtx {
namespace {

constexpr int kBlock = 256;
// Output arena: device memory in chunks of at least this size, grown as admission needs
// and kept until the server is destroyed; request outputs are placed first-fit.
constexpr int64_t kArenaChunk = (int64_t)1 << 30;
constexpr int64_t kArenaAlign = 256;
// Wall-clock interval between the kernel's reads of the host's published count.
constexpr int kPollMicros = 4;
constexpr int kDefaultIdleMicros = 2000;

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


double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

}  // namespace

// Bytes a request holds while admitted: its outputs (rgb, depth, opacity).
int64_t request_bytes(const grtx_request* r) {
  const int64_t n = (int64_t)r->width * r->height;
  return n * 20;
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
  // work queue and kernel
  hipStream_t stream = nullptr;
  hipEvent_t kernel_done = nullptr;
  bool kernel_running = false;
  ServeHost* host = nullptr;      // fine-grained pinned host memory
  ServeHost* host_dev = nullptr;  // its device address
  ServeDev* dev = nullptr;
  void* pool = nullptr;
  int64_t fixed_bytes = 0;        // kernel pool and queue
  uint64_t poll_ticks = 0, idle_ticks = 0;
  uint64_t published = 0;         // requests published so far (request numbers)
  uint64_t slot_ticket[kServeRing] = {};  // ticket of the request in each slot (0: free)
  std::vector<int> in_flight;     // slots of published, unfinished requests
  int64_t launches = 0;
  // output arena
  struct Chunk {
    char* base = nullptr;
    int64_t size = 0;
    std::map<int64_t, int64_t> free;  // offset -> length, coalesced
  };
  std::vector<Chunk> chunks;
  int64_t arena_bytes = 0;
  // requests
  struct Req {
    grtx_request r{};
    int64_t rays = 0, bytes = 0;
    double t_submit = 0, t_admit = 0, t_launch = 0, t_done = 0;
    const uint32_t* order = nullptr;
    float* out = nullptr;
    int chunk = -1;
    int64_t offset = 0, span = 0;
    int state = 0;  // 0 queued, 1 admitted and published, 3 done, 4 failed
  };
  std::mutex mu;
  std::condition_variable cv;
  std::deque<uint64_t> queued;
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
  hipStream_t s = sv->stream;
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

// First-fit placement of `bytes` in the arena's chunks; false if no free range holds it.
bool arena_place(Server* sv, int64_t bytes, int* chunk, int64_t* offset, int64_t* span) {
  const int64_t need = (bytes + kArenaAlign - 1) / kArenaAlign * kArenaAlign;
  for (size_t c = 0; c < sv->chunks.size(); ++c) {
    auto& fl = sv->chunks[c].free;
    for (auto it = fl.begin(); it != fl.end(); ++it) {
      if (it->second < need) continue;
      const int64_t off = it->first, len = it->second;
      fl.erase(it);
      if (len > need) fl.emplace(off + need, len - need);
      *chunk = (int)c;
      *offset = off;
      *span = need;
      return true;
    }
  }
  return false;
}

void arena_free(Server* sv, int chunk, int64_t offset, int64_t span) {
  auto& fl = sv->chunks[chunk].free;
  auto it = fl.emplace(offset, span).first;
  auto nx = std::next(it);
  if (nx != fl.end() && it->first + it->second == nx->first) {
    it->second += nx->second;
    fl.erase(nx);
  }
  if (it != fl.begin()) {
    auto pv = std::prev(it);
    if (pv->first + pv->second == it->first) {
      pv->second += it->second;
      fl.erase(it);
    }
  }
}

// Write request `rq` (admitted, ticket t) into its ring slot and publish it (lock held).
void publish_locked(Server* sv, uint64_t t, Server::Req& rq) {
  const uint64_t j = sv->published;
  const int slot = (int)(j % kServeRing);
  ServeDesc& d = sv->host->ring[slot];
  CameraFrame cf;
  camera_frame(rq.r.eye, rq.r.target, rq.r.up, rq.r.fov_y_deg, rq.r.width, rq.r.height, &cf);
  const int tiles_x = (rq.r.width + 7) / 8, tiles_y = (rq.r.height + 7) / 8;
  d.seq = (uint32_t)j;
  d.n_work = (uint32_t)((int64_t)tiles_x * tiles_y * 64);
  d.width = rq.r.width;
  d.height = rq.r.height;
  d.tiles_x = tiles_x;
  d.scene = rq.r.scene_id;
  d.n_pixels = (uint32_t)rq.rays;
  d.pad = 0;
  d.order = reinterpret_cast<uint64_t>(rq.order);
  d.out = reinterpret_cast<uint64_t>(rq.out);
  for (int a = 0; a < 3; ++a) {
    d.eye[a] = cf.eye[a];
    d.fwd[a] = cf.fwd[a];
    d.right[a] = cf.right[a];
    d.up[a] = cf.up[a];
  }
  sv->host->done[slot] = 0;
  // the descriptor and the cleared flag reach memory before the count that publishes them
  std::atomic_thread_fence(std::memory_order_release);
  __atomic_store_n(&sv->host->published, j + 1, __ATOMIC_RELEASE);
  sv->published = j + 1;
  sv->slot_ticket[slot] = t;
  sv->in_flight.push_back(slot);
  rq.state = 1;
  rq.t_admit = rq.t_launch = now_s() - sv->t0;
  if (sv->first_launch < 0) sv->first_launch = rq.t_launch;
}

// Admit and publish queued requests, first come, first served, while their outputs fit
// the budget and the arena and the next ring slot is free (lock held). Returns the
// arena growth the head of the queue waits for (0 if none).
int64_t admit_locked(Server* sv) {
  while (!sv->queued.empty()) {
    auto it = sv->reqs.find(sv->queued.front());
    if (it == sv->reqs.end()) {  // released while queued
      sv->queued.pop_front();
      continue;
    }
    Server::Req& r = it->second;
    if (sv->in_use + r.bytes > sv->available) return 0;  // waits for releases
    if (sv->slot_ticket[sv->published % kServeRing] != 0) return 0;  // ring slot still busy
    int chunk = -1;
    int64_t off = 0, span = 0;
    if (!arena_place(sv, r.bytes, &chunk, &off, &span)) {
      // a new chunk, if the budget still has room for one that holds the request
      const int64_t room = sv->available - sv->arena_bytes;
      const int64_t want = std::min(room, std::max(kArenaChunk, (r.bytes + kArenaAlign - 1) / kArenaAlign * kArenaAlign));
      return want >= r.bytes ? want : 0;
    }
    r.chunk = chunk;
    r.offset = off;
    r.span = span;
    r.out = reinterpret_cast<float*>(sv->chunks[chunk].base + off);
    sv->in_use += r.bytes;
    const uint64_t t = it->first;
    sv->queued.pop_front();
    publish_locked(sv, t, r);
  }
  return 0;
}

// Mark the in-flight requests failed (their launch failed or did not finish; lock held).
void fail_in_flight_locked(Server* sv, const char* why) {
  snprintf(sv->worker_error, sizeof sv->worker_error, "%s", why);
  for (int slot : sv->in_flight) {
    auto it = sv->reqs.find(sv->slot_ticket[slot]);
    if (it != sv->reqs.end()) it->second.state = 4;
    sv->slot_ticket[slot] = 0;
  }
  sv->in_flight.clear();
  sv->cv.notify_all();
}

void worker_main(Server* sv) {
  (void)hipSetDevice(sv->device);
  while (!sv->stop.load()) {
    bool progressed = false;
    // the launch ended: every flag it raised is in host memory by now
    if (sv->kernel_running) {
      const hipError_t q = hipEventQuery(sv->kernel_done);
      if (q != hipErrorNotReady) {
        sv->kernel_running = false;
        progressed = true;
        if (q != hipSuccess) {
          std::lock_guard<std::mutex> g(sv->mu);
          char msg[256];
          snprintf(msg, sizeof msg, "serving kernel failed: %s", hipGetErrorString(q));
          fail_in_flight_locked(sv, msg);
        }
      }
    }
    int64_t grow = 0;
    {
      std::lock_guard<std::mutex> g(sv->mu);
      // completions
      const double t = now_s() - sv->t0;
      for (size_t i = 0; i < sv->in_flight.size();) {
        const int slot = sv->in_flight[i];
        if (__atomic_load_n(&sv->host->done[slot], __ATOMIC_ACQUIRE) == 0) {
          ++i;
          continue;
        }
        auto it = sv->reqs.find(sv->slot_ticket[slot]);
        if (it != sv->reqs.end()) {
          it->second.state = 3;
          it->second.t_done = t;
          sv->latencies.push_back(t - it->second.t_submit);
          ++sv->completed;
          sv->rays_completed += it->second.rays;
        }
        sv->last_done = t;
        sv->slot_ticket[slot] = 0;
        sv->in_flight[i] = sv->in_flight.back();
        sv->in_flight.pop_back();
        progressed = true;
      }
      if (progressed) sv->cv.notify_all();
      // admission and publication
      const uint64_t before = sv->published;
      grow = admit_locked(sv);
      if (sv->published != before) progressed = true;
    }
    if (grow > 0) {
      // a new arena chunk, allocated without the lock (no device synchronisation)
      void* p = nullptr;
      const hipError_t e = hipMalloc(&p, (size_t)grow);
      std::lock_guard<std::mutex> g(sv->mu);
      if (e == hipSuccess) {
        Server::Chunk c;
        c.base = static_cast<char*>(p);
        c.size = grow;
        c.free.emplace(0, grow);
        sv->chunks.push_back(std::move(c));
        sv->arena_bytes += grow;
        progressed = true;
      } else {
        (void)hipGetLastError();
        snprintf(sv->worker_error, sizeof sv->worker_error, "arena growth of %lld bytes failed", (long long)grow);
      }
    }
    // (re)start the kernel while published work is unfinished
    if (!sv->kernel_running) {
      bool pending;
      {
        std::lock_guard<std::mutex> g(sv->mu);
        pending = !sv->in_flight.empty();
      }
      if (pending) {
        ServeLaunch L{};
        L.scene = TraceScene{sv->nodes, sv->inst, nullptr, sv->sh, sv->sh_degree, sv->roots, nullptr,
                             GRTX_BVH_SPHERE_INSTANCE, sv->total_leaves};
        L.k = sv->cfg.k;
        L.T_min = sv->cfg.T_min;
        L.mode = sv->cfg.mode;
        for (int a = 0; a < 3; ++a) L.bg[a] = sv->cfg.bg[a];
        L.host = sv->host_dev;
        L.dev = sv->dev;
        L.pool = sv->pool;
        L.poll_ticks = sv->poll_ticks;
        L.idle_ticks = sv->idle_ticks;
        grtx_status st = launch_serve(L, sv->stream);
        if (st == GRTX_OK && hipEventRecord(sv->kernel_done, sv->stream) != hipSuccess) st = GRTX_ERR_DEVICE;
        if (st == GRTX_OK) {
          sv->kernel_running = true;
          ++sv->launches;
        } else {
          std::lock_guard<std::mutex> g(sv->mu);
          char msg[256];
          snprintf(msg, sizeof msg, "serving launch failed: %s", grtx_last_error());
          fail_in_flight_locked(sv, msg);
        }
        progressed = true;
      }
    }
    if (!progressed) {
      std::unique_lock<std::mutex> lk(sv->mu);
      sv->cv.wait_for(lk, std::chrono::microseconds(sv->in_flight.empty() ? 200 : 20));
    }
  }
  // stop: the kernel finishes the published work and leaves
  __atomic_store_n(&sv->host->stop, 1u, __ATOMIC_RELEASE);
  (void)hipStreamSynchronize(sv->stream);
}

}  // namespace

grtx_status serve_create(const grtx_serve_config* cfg, Server** out) {
  auto* sv = new Server();
  sv->cfg = *cfg;
  if (sv->cfg.max_request_rays <= 0) sv->cfg.max_request_rays = 1 << kServePixelBits;
  if (sv->cfg.idle_exit_us <= 0) sv->cfg.idle_exit_us = kDefaultIdleMicros;
  sv->t0 = now_s();
  hipError_t e = hipGetDevice(&sv->device);
  int clock_khz = 0;
  if (e == hipSuccess) e = hipDeviceGetAttribute(&clock_khz, hipDeviceAttributeWallClockRate, sv->device);
  if (e != hipSuccess || clock_khz <= 0) {
    set_error("grtx_serve_create: %s", e != hipSuccess ? hipGetErrorString(e) : "no wall clock rate");
    delete sv;
    return GRTX_ERR_DEVICE;
  }
  sv->poll_ticks = std::max<uint64_t>(1, (uint64_t)clock_khz * kPollMicros / 1000);
  sv->idle_ticks = std::max<uint64_t>(1, (uint64_t)clock_khz * (uint64_t)sv->cfg.idle_exit_us / 1000);
  // the kernel's checkpoint pool and the queue count against the budget
  const int64_t pool_bytes = serve_pool_bytes(cfg->k);
  sv->fixed_bytes = pool_bytes + (int64_t)sizeof(ServeDev);
  sv->available = cfg->memory_budget - sv->fixed_bytes;
  if (pool_bytes <= 0 || sv->available <= 0) {
    set_error("grtx_serve_create: budget %lld bytes is below the serving kernel's checkpoint pool (%lld bytes)",
              (long long)cfg->memory_budget, (long long)pool_bytes);
    delete sv;
    return GRTX_ERR_CAPACITY;
  }
  if (hipStreamCreateWithFlags(&sv->stream, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&sv->kernel_done, hipEventDisableTiming) != hipSuccess ||
      hipHostMalloc(reinterpret_cast<void**>(&sv->host), sizeof(ServeHost),
                    hipHostMallocCoherent | hipHostMallocMapped) != hipSuccess ||
      hipHostGetDevicePointer(reinterpret_cast<void**>(&sv->host_dev), sv->host, 0) != hipSuccess ||
      hipMalloc(reinterpret_cast<void**>(&sv->dev), sizeof(ServeDev)) != hipSuccess ||
      hipMalloc(&sv->pool, (size_t)pool_bytes) != hipSuccess) {
    (void)hipGetLastError();
    set_error("grtx_serve_create: stream/queue setup failed");
    serve_destroy(sv);
    return GRTX_ERR_DEVICE;
  }
  std::memset(static_cast<void*>(sv->host), 0, sizeof(ServeHost));
  {
    // empty queue: nothing published, every claim counter naming no request and past any
    // request's items
    std::vector<ServeDev> init(1);
    ServeDev& q = init[0];
    std::memset(static_cast<void*>(&q), 0, sizeof(ServeDev));
    for (auto& sl : q.slot) sl.claim = ((uint64_t)kServeNoRequest << 32) | 0x80000000u;
    if (hipMemcpy(sv->dev, &q, sizeof(ServeDev), hipMemcpyHostToDevice) != hipSuccess) {
      (void)hipGetLastError();
      set_error("grtx_serve_create: queue setup failed");
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
  if (sv->total_leaves + b->n_leaves >= (int64_t)kLeafFlag || sv->total_nodes + b->node_slots >= (int64_t)kLeafFlag) {
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
  CameraFrame cf;
  if (!camera_frame(r->eye, r->target, r->up, r->fov_y_deg, r->width, r->height, &cf)) {
    set_error("grtx_serve_submit: degenerate eye/target/up");
    return GRTX_ERR_INVALID_ARG;
  }
  const int64_t rays = (int64_t)r->width * r->height;
  if (rays > sv->cfg.max_request_rays) {
    set_error("grtx_serve_submit: request of %lld rays; the server takes at most %d", (long long)rays,
              sv->cfg.max_request_rays);
    return GRTX_ERR_CAPACITY;
  }
  // the tile order of this image size (made once per size, outside the server's lock)
  const uint32_t* order = nullptr;
  SV_TRY(centre_out_order(sv->device, (r->width + 7) / 8, (r->height + 7) / 8, &order));
  std::lock_guard<std::mutex> g(sv->mu);
  if (r->scene_id < 0 || r->scene_id >= (int32_t)sv->scenes.size()) {
    set_error("grtx_serve_submit: unknown scene %d", r->scene_id);
    return GRTX_ERR_INVALID_ARG;
  }
  if (!sv->frozen) SV_TRY(freeze(sv));
  Server::Req q;
  q.r = *r;
  q.rays = rays;
  q.bytes = request_bytes(r);
  q.order = order;
  if (q.bytes > sv->available) {
    set_error("grtx_serve_submit: request needs %lld bytes; the server holds %lld bytes for outputs",
              (long long)q.bytes, (long long)sv->available);
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
  Server::Req& q = it->second;
  if (q.state == 1) {
    set_error("grtx_serve_release: request %llu is still in flight", (unsigned long long)ticket);
    return GRTX_ERR_NOT_READY;
  }
  if (q.state == 0) {
    // withdrawn before admission: it leaves the queue and is never published or counted
    auto p = std::find(sv->queued.begin(), sv->queued.end(), ticket);
    if (p != sv->queued.end()) sv->queued.erase(p);
    --sv->submitted;
  }
  if (q.chunk >= 0) {
    arena_free(sv, q.chunk, q.offset, q.span);
    sv->in_use -= q.bytes;
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
  s.bytes_arena = sv->arena_bytes;
  s.launches = sv->launches;
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
  } else if (sv->host) {
    __atomic_store_n(&sv->host->stop, 1u, __ATOMIC_RELEASE);
  }
  if (sv->stream) (void)hipStreamSynchronize(sv->stream);
  for (auto& c : sv->chunks) (void)hipFree(c.base);
  if (sv->pool) (void)hipFree(sv->pool);
  if (sv->dev) (void)hipFree(sv->dev);
  if (sv->host) (void)hipHostFree(sv->host);
  if (sv->kernel_done) (void)hipEventDestroy(sv->kernel_done);
  if (sv->stream) (void)hipStreamDestroy(sv->stream);
  for (void* p : sv->scene_allocs) (void)hipFree(p);
  delete sv;
  return GRTX_OK;
}

}  // namespace grtx
