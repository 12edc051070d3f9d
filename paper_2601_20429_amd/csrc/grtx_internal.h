// Internal declarations shared by the HIP sources of the library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "grtx.h"

namespace grtx {

// Work items of one trace launch: the rays before image_begin one each, then the image's
// 8x8 tiles 64 each (the image being rays image_begin..count-1 in rows of image_width;
// rays that do not divide into such rows are all taken one by one). The launch's work
// counter and ray indices are 32-bit, so a launch takes at most 2^31-1 items.
inline int64_t trace_work_items(const grtx_rays* r, int64_t* n_free, int64_t* image_h) {
  const int64_t R = r->count;
  const int64_t n_img = R - r->image_begin;
  if (r->image_width > 0 && r->image_begin >= 0 && n_img > 0 && n_img % r->image_width == 0) {
    *n_free = r->image_begin;
    *image_h = n_img / r->image_width;
    const int64_t tiles_x = ((int64_t)r->image_width + 7) / 8, tiles_y = (*image_h + 7) / 8;
    return r->image_begin + tiles_x * tiles_y * 64;
  }
  *n_free = R;
  *image_h = 0;
  return R;
}
constexpr int64_t kMaxTraceWork = 0x7FFFFFFF;

// ---------------------------------------------------------------------------------------
// Device data layout
// ---------------------------------------------------------------------------------------
//
// Node record, 64 B (4 x float4), one per internal node of the binary radix tree that the
// traversal can reach (root at position 0). A record lists up to four descendants that
// partition its leaves: starting from the node's two children, the internal entry of
// largest surface area is replaced by its two children until there are four; its
// internal entries are the positions of their own records. The children's boxes
// are stored on an 8-bit grid over the node's own box: per axis a an origin o_a (the box
// minimum) and a power-of-two step s_a with extent / s_a <= 254; child j's planes are
// o_a + q * s_a with q rounded outward (lo down, hi up), so each stored box contains
// the child's exact box.
//   q0 = (o.x, o.y, o.z, s.x)
//   q1 = (s.y, s.z, ref0, ref1)
//   q2 = (ref2, ref3, qlo.x, qlo.y)
//   q3 = (qlo.z, qhi.x, qhi.y, qhi.z)
// ref = internal node index, kLeafFlag | leaf, or kNoChild (as uint bits); each q word
// holds one plane of the four children, child j in byte j.
constexpr int kNodeF4 = 4;

// Instance record (SPHERE_INSTANCE leaf), 64 B, in sorted-leaf order:
//   q0 = (A00, A01, A02, mu.x)   A = rho^-1 S^-1 R^T maps the bounding ellipsoid of the
//   q1 = (A10, A11, A12, mu.y)   Gaussian onto the unit sphere: u = A (x - mu)
//   q2 = (A20, A21, A22, mu.z)
//   q3 = (o, log2(o/alpha_min), gaussian id bits, active bits)
//
// Proxy triangle record (PROXY20 leaf), 48 B, in sorted-leaf order:
//   q0 = (v0.x, v0.y, v0.z, gaussian id bits)
//   q1 = (v1.x, v1.y, v1.z, 0)
//   q2 = (v2.x, v2.y, v2.z, 0)
// For PROXY20 the instance records are stored in Gaussian order instead.
constexpr uint32_t kLeafFlag = 0x80000000u;
constexpr uint32_t kNoParent = 0xFFFFFFFFu;
// Cut of the radix tree kept for cost estimates of image traces: the largest subtrees of at
// most max(1, leaves / kCutDiv) leaves, at most kCutCap of them.
constexpr int64_t kCutDiv = 2048;
constexpr int kCutCap = 16384;
// Density grid kept for ordering rays that form no image: leaves per cell of a
// kDensityRes^3 grid over the leaf centres' bounds (`dbox`: lo xyz, hi xyz).
constexpr int kDensityRes = 64;
constexpr int kDensityCells = kDensityRes * kDensityRes * kDensityRes;
__device__ __forceinline__ int density_axis(float p, float lo, float hi) {
  const float e = hi - lo;
  const int c = e > 0.f ? (int)((p - lo) / e * (float)kDensityRes) : 0;
  return c < 0 ? 0 : c >= kDensityRes ? kDensityRes - 1 : c;
}
// Cell of point (x, y, z) in the grid over box (lo xyz, hi xyz); points outside are clamped.
__device__ __forceinline__ int density_cell(float x, float y, float z, const float* box) {
  return density_axis(x, box[0], box[3]) +
         kDensityRes * (density_axis(y, box[1], box[4]) + kDensityRes * density_axis(z, box[2], box[5]));
}
constexpr uint32_t kNoChild = 0xFFFFFFFFu;
// Per-ray capacities of the checkpoint (deferred node) and eviction lists of the serving
// kernel's pool (the trace's defaults live with the trace kernel): 2048/512 served the
// four-scene mix 2% faster than 1024/256 (fewer list compactions on the 1M and 3M
// scenes), and 4096/1024 no faster.
constexpr int kServeDeferCap = 2048;
constexpr int kServeEvictCap = 512;

// ---------------------------------------------------------------------------------------
// Serving work queue
// ---------------------------------------------------------------------------------------
//
// Requests are numbered j = 0, 1, ... in publication order and live in ring slot
// j % kServeRing from publication until the kernel reports them finished; the host
// publishes request j only once the request before it in that slot has finished. A
// request's work items are its 8x8 pixel tiles x 64 (items of a ragged edge tile that
// fall outside the image are skipped). A served ray's id is slot << kServePixelBits |
// pixel, so a request holds at most 2^kServePixelBits pixels.
constexpr int kServeRing = 1024;
constexpr int kServePixelBits = 22;

// One request as the host publishes it (fine-grained host memory, read by the kernel).
struct ServeDesc {
  uint32_t seq;       // request number j
  uint32_t n_work;    // work items: tiles x 64
  int32_t width, height, tiles_x, scene;
  uint32_t n_pixels;  // width x height: rays whose outputs complete the request
  uint32_t pad;
  uint64_t order;     // device address of the tile order (uint32 per tile), 0 for row-major
  uint64_t out;       // device address of the outputs: rgb [n,3], depth [n], opacity [n]
  float eye[3], fwd[3], right[3], up[3];
};

// Host side of the queue, in fine-grained (coherent) pinned host memory.
struct ServeHost {
  uint64_t published;           // requests published; written after their descriptors
  uint32_t stop;                // set by the host: finish the published work, then exit
  uint32_t pad;
  uint32_t done[kServeRing];    // set to 1 by the kernel when the slot's request finished
  ServeDesc ring[kServeRing];
};

// Per ring slot on the device: the claim counter, (request << 32) | work items claimed
// (it may run past the request's items: claims beyond them are empty), and the count of
// the request's finished rays, on separate 64-B lines.
struct alignas(128) ServeSlot {
  uint64_t claim;
  uint32_t pad0[14];
  uint32_t done;
  uint32_t pad1[15];
};

// Device side of the queue (device memory; read with device-scope atomic loads, written
// with atomics, so every XCD sees one value).
//   state: bit 63 closing (no more requests are taken), bits 32..62 requests published
//          to the kernel, bits 0..31 the request whose items are being handed out.
//   A request's descriptor and claim counter are set up (by the lane that reads the
//   host's count, under poll_lock) before the published count covers it.
constexpr uint64_t kServeClosing = 1ull << 63;
constexpr uint32_t kServeNoRequest = 0xFFFFFFFFu;
struct ServeDev {
  uint64_t state;
  uint64_t pad_a[7];
  uint64_t last_poll;     // wall clock of the last read of the host's count
  uint64_t inited;        // requests whose descriptor and claim counter are set up
  uint32_t poll_lock;
  uint32_t pad_b[11];
  ServeSlot slot[kServeRing];
  ServeDesc desc[kServeRing];
};

struct Bvh {
  int device = 0;
  grtx_bvh_kind kind = GRTX_BVH_SPHERE_INSTANCE;
  int64_t n_gauss = 0;
  int64_t n_leaves = 0;
  int sh_degree = 0;
  float alpha_min = 0.f;
  float4* nodes = nullptr;   // [node_slots][kNodeF4]: the reachable records (positions, see k_layout_top)
  int64_t node_slots = 0;    // positions of `nodes` (some unused between subtree blocks)
  float4* inst = nullptr;    // [n_gauss][4]
  float4* tris = nullptr;    // PROXY20: [n_leaves][3]
  uint64_t* codes = nullptr; // [n_leaves] sorted Morton codes
  uint32_t* perm = nullptr;  // [n_leaves]
  uint32_t* child = nullptr; // [n_leaves-1][2]
  uint32_t* parent = nullptr;// [2 n_leaves - 1]
  float* boxes = nullptr;    // [2 n_leaves - 1][6]
  float* root_box = nullptr; // device [6] (points into boxes)
  float* roots = nullptr;    // device [8]: root box, root reference bits, 0
  float4* cut = nullptr;     // [kCutCap][2]: subtree boxes (lo, leaf count) (hi, 0), see k_cut_write
  uint32_t* n_cut = nullptr; // device [1]: entries of `cut` (may exceed kCutCap; read the minimum)
  uint32_t* depth = nullptr; // device [2]: tree depth in internal nodes, 1 if restructured
  uint32_t* density = nullptr;  // [kDensityCells] leaves per grid cell
  float* dbox = nullptr;        // device [6]: the grid's box
  const float* opacities = nullptr; // borrowed
  const float* sh = nullptr;        // borrowed
  hipStream_t build_stream = nullptr;
  size_t bytes = 0;
  std::vector<void*> allocations;
};

// ---------------------------------------------------------------------------------------
// Errors
// ---------------------------------------------------------------------------------------
void set_error(const char* fmt, ...);
void clear_error();

// Propagate a non-OK status from a library call.
#define GRTX_TRY(x)                  \
  do {                               \
    grtx_status st_ = (x);           \
    if (st_ != GRTX_OK) return st_;  \
  } while (0)

#define GRTX_HIP(call)                                                                  \
  do {                                                                                  \
    hipError_t e_ = (call);                                                             \
    if (e_ != hipSuccess) {                                                             \
      ::grtx::set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), __FILE__, \
                        __LINE__);                                                      \
      return e_ == hipErrorOutOfMemory ? GRTX_ERR_OUT_OF_MEMORY : GRTX_ERR_DEVICE;      \
    }                                                                                   \
  } while (0)

#define GRTX_LAUNCH_CHECK()                                                             \
  do {                                                                                  \
    hipError_t e_ = hipGetLastError();                                                  \
    if (e_ != hipSuccess) {                                                             \
      ::grtx::set_error("kernel launch failed: %s (%s:%d)", hipGetErrorString(e_),      \
                        __FILE__, __LINE__);                                            \
      return GRTX_ERR_DEVICE;                                                           \
    }                                                                                   \
  } while (0)

// ---------------------------------------------------------------------------------------
// Host entry points implemented in the .hip sources
// ---------------------------------------------------------------------------------------
grtx_status build_bvh(const grtx_gaussians* g, grtx_bvh_kind kind, float alpha_min, bool restructure_tree,
                      int max_depth, hipStream_t s, Bvh* b);
grtx_status export_topology(const Bvh* b, uint32_t* child, uint32_t* parent, uint64_t* morton, uint32_t* perm,
                            float* boxes, hipStream_t s);
grtx_status pinhole_rays(const grtx_camera* cam, float* origins, float* dirs, hipStream_t s);
grtx_status trace(const Bvh* b, const grtx_rays* r, const grtx_trace_params* p, const grtx_trace_outputs* o,
                  hipStream_t s);
// The same trace with every device buffer beyond the inputs and outputs taken from the
// library's static per-device scratch (no allocation; row-major tile order).
grtx_status trace_noalloc(const Bvh* b, const grtx_rays* r, const grtx_trace_params* p, const grtx_trace_outputs* o,
                          hipStream_t s);

// What the trace kernel reads of a scene, or of several scenes merged into one address
// space (serving): then `ray_scene` gives each ray's scene and `roots` holds one root
// entry (8 floats) per scene.
struct TraceScene {
  const float4* nodes;
  const float4* inst;
  const float4* tris;
  const float* sh;
  int sh_degree;
  const float* roots;
  const int32_t* ray_scene;
  grtx_bvh_kind kind;
  int64_t n_leaves;
  const float4* cut = nullptr;      // subtree cut for tile cost estimates, or null
  const uint32_t* n_cut = nullptr;
  const uint32_t* density = nullptr;  // density grid for ray order estimates, or null
  const float* dbox = nullptr;
};
grtx_status launch_trace(const TraceScene& sc, const grtx_rays* r, const grtx_trace_params* p,
                         const grtx_trace_outputs* o, hipStream_t s);
// Single-round mode of launch_trace (single.hip).
grtx_status trace_single_round(const TraceScene& b, const grtx_rays* r, const grtx_trace_params* p,
                               const grtx_trace_outputs* o, hipStream_t s);
// The serving kernel: a persistent trace launch over the merged scene set that takes
// requests from the work queue until the host stops it or no work has been taken for
// `idle_ticks` of the device wall clock (then it sets `closing` and its waves exit once
// their rays are done). `pool` holds serve_pool_bytes(k) bytes.
struct ServeLaunch {
  TraceScene scene;
  int k;
  float T_min;
  int mode;
  float bg[3];
  ServeHost* host;
  ServeDev* dev;
  void* pool;
  uint64_t poll_ticks;
  uint64_t idle_ticks;
};
grtx_status launch_serve(const ServeLaunch& L, hipStream_t s);
int64_t serve_pool_bytes(int k);
// Centre-out processing order of the 8x8 tiles of a tiles_x x tiles_y image (device array,
// kept until the process ends).
grtx_status centre_out_order(int device, int tiles_x, int tiles_y, const uint32_t** out);

struct Server;
int64_t request_bytes(const grtx_request* r);
grtx_status serve_create(const grtx_serve_config* cfg, Server** out);
grtx_status serve_add_scene(Server* sv, const Bvh* b, int32_t* scene_id);
grtx_status serve_submit(Server* sv, const grtx_request* r, uint64_t* ticket);
grtx_status serve_poll(Server* sv, uint64_t ticket, grtx_request_result* res);
grtx_status serve_release(Server* sv, uint64_t ticket);
grtx_status serve_stats(Server* sv, grtx_serve_stats* st);
grtx_status serve_destroy(Server* sv);
// Stream-ordered scratch memory for one call. Regions come from a per-(device, stream)
// arena in last-in-first-out order and return to it when the Scratch ends, so calls on one
// stream reuse the same memory without an allocation or a free each time (the work that
// used a region is ordered before any later use on that stream). A request beyond the
// arena is met by hipMallocAsync and freed in stream order; when the outermost scratch of
// a stream ends, the arena grows to the largest demand seen. A stream must be driven by
// one host thread at a time.
struct ScratchArena;
class Scratch {
 public:
  explicit Scratch(hipStream_t s);
  ~Scratch();
  Scratch(const Scratch&) = delete;
  Scratch& operator=(const Scratch&) = delete;
  grtx_status raw(void** p, size_t bytes);
  template <class T>
  grtx_status get(T** p, size_t count) {
    void* q = nullptr;
    grtx_status st = raw(&q, (count > 0 ? count : 1) * sizeof(T));
    if (st == GRTX_OK) *p = static_cast<T*>(q);
    return st;
  }

 private:
  ScratchArena* arena_ = nullptr;
  hipStream_t s_;
  size_t mark_ = 0, logical_mark_ = 0;
  std::vector<void*> extra_;
};

// Device utilities of the build, reused by the backward pass (stream-ordered scratch).
// Exclusive prefix sum of n uint32 values.
grtx_status exclusive_scan_u32(const uint32_t* in, uint32_t* out, int64_t n, hipStream_t s);
// Stable LSD radix sort of (keys, vals) by the low key_bits bits of the keys, in place. With
// `n_dev` the first *n_dev (at most n) pairs are sorted, n being the host's bound.
grtx_status sort_by_key(uint64_t* keys, uint32_t* vals, int64_t n, int key_bits, hipStream_t s,
                        const uint32_t* n_dev = nullptr);
// The same with caller-owned temporaries (tkeys, tvals of n entries); *kres / *vres receive
// the arrays that hold the result (the inputs or the temporaries), so nothing is copied.
grtx_status sort_by_key_into(uint64_t* keys, uint32_t* vals, uint64_t* tkeys, uint32_t* tvals, int64_t n,
                             int key_bits, hipStream_t s, const uint32_t* n_dev, uint64_t** kres, uint32_t** vres);

// Secondary rays (objects.hip).
grtx_status object_rays(const grtx_objects* obj, const grtx_rays* r, float* t_far, float* next_o, float* next_d,
                        float* path, int32_t* kind, hipStream_t s);
grtx_status continue_rays(int64_t count, const int32_t* kind, const float* opacity, float T_min,
                          const float* next_o, const float* next_d, float* co, float* cd, float* ct, int32_t* ci,
                          int64_t* n_cont, hipStream_t s);
grtx_status continue_composite(int64_t n, const int32_t* idx, const float* trans, const float* path,
                               const float* crgb, const float* cdepth, const float* copac, float* rgb, float* depth,
                               float* opac, hipStream_t s);

grtx_status trace_backward(const Bvh* bvh, const grtx_gaussians* g, const grtx_rays* r, const grtx_trace_params* p,
                           const grtx_trace_outputs* fwd, const float* grad_rgb, const float* grad_depth,
                           const float* grad_opacity, const grtx_gaussian_grads* grads, unsigned int* truncated,
                           hipStream_t s);

}  // namespace grtx

struct grtx_bvh {
  grtx::Bvh impl;
};

struct grtx_server {
  grtx::Server* impl;
};
