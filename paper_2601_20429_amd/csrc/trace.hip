// Multi-round k-buffer Gaussian ray tracing with traversal checkpointing, for gfx950.
//
// What one ray computes (Sec. III-A; Listing 1; Sec. IV-B):
//   round r: traverse the BVH, keeping the k closest hits beyond the last blended one in
//   a sorted k-buffer (any-hit insertion sort; a hit beyond the farthest entry of a full
//   buffer is rejected and t_max shrinks to the buffer's farthest entry); blend the
//   k-buffer front to back (Eq. 1, alpha at the maximum response, Eq. 2, colour from SH
//   and the ray direction); stop once the transmittance falls below T_min (early ray
//   termination) or fewer than k hits remain.
//   CHECKPOINT mode: nodes whose entry distance exceeds t_max are written to the ray's
//   destination checkpoint list, and hits rejected from the k-buffer to its eviction
//   list; the next round first moves the k closest evicted hits into the k-buffer and
//   then resumes traversal from the source list (the previous destination list) instead
//   of the root. Entries whose stored distance already exceeds t_max are carried to the
//   new destination list without fetching the node.
//   RESTART mode: every round starts at the root with the interval (last blended hit,
//   t_max] and nothing is kept between rounds (the multi-round baseline).
//
// How it maps to CDNA4 (there is no RT unit, so the RT unit's job is done by the wave):
//   - persistent waves; each lane owns one ray at a time across all of its rounds;
//     idle lanes are refilled with a ballot + one atomic per wave; rays are taken in
//     8x8 pixel tiles when the rays form an image;
//   - the k-buffer is a register array of 64-bit keys (distance bits << 32 | leaf),
//     kept sorted; a key is inserted by comparing it with every entry at once (statically
//     indexed, no dependent chain);
//   - the traversal stack is per lane: the top kLdsStack entries in LDS, the rest in a
//     per-wave HBM region, where each lane also keeps its checkpoint and eviction lists
//     in a contiguous block of its own (its appends and reads walk its own cache lines);
//     k-buffers are parked there [entry][lane] for the blend;
//   - hit keys use the leaf's sorted position, whose Morton order keeps neighbouring
//     Gaussians close in memory; ties in distance are broken by that position.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <memory>
#include <mutex>
#include <numeric>
#include <tuple>
#include <vector>

#include "camera.h"
#include "grtx_internal.h"
#include "trace_common.h"

namespace grtx {
namespace {

// Waves per SIMD the trace kernel is register-budgeted for up to k = 32 (at most 170
// VGPRs): three, which k <= 32 reach with a few dozen bytes of scratch per lane on cold
// paths; k = 64 is held to two (256 VGPRs).
#ifndef GRTX_MIN_WAVES
#define GRTX_MIN_WAVES 3
#endif
// Idle or finished lanes that end a traversal burst for a refill: 32 for structures of up
// to a million leaves, 16 above (on the 3M-Gaussian workload 16 was 5% faster on its
// incoherent rays than 32, and 12 or 8 no better; on a 100k-Gaussian frame 32 is 1% faster
// than 16).
constexpr int kRefillSmall = 32;
constexpr int kRefillLarge = 16;
// Deferred-node list appends gather in LDS and go out to the lane's HBM block kStage
// entries at a time (one contiguous write of kStage x 8 B instead of kStage scattered
// 8-B writes from the wave). List capacities are rounded up to a multiple of kStage.
#ifndef GRTX_STAGE
#define GRTX_STAGE 8
#endif
constexpr int kStage = GRTX_STAGE;
// Eviction-list appends gathered the same way, kStageE entries at a time (0: written one
// by one); kStageE divides kStage. Two entries (16-B writes) measured 1-2% faster than
// single entries on the 3M-Gaussian workload; four (with a smaller LDS stack or deferred
// stage, to keep three workgroups per CU) were slower. The serving kernel, whose LDS also
// holds its request copies, writes them one by one.
#ifndef GRTX_EVICT_STAGE
#define GRTX_EVICT_STAGE 2
#endif
constexpr int kStageE = GRTX_EVICT_STAGE;
// Traversal iterations between checks for list room (a power of two).
constexpr int kRoomEvery = 8;
#ifndef GRTX_CHUNKS
#define GRTX_CHUNKS 1
#endif
// Work queues. One shared queue keeps a launch's heaviest-first order; one per XCD (8)
// measured slower.
constexpr int kChunks = GRTX_CHUNKS;
// Default per-ray capacities of the checkpoint (deferred node) and eviction lists. An entry
// that finds its list full is dropped and lowers the ray's key limit to its smallest key;
// the ray goes on from its checkpoint and falls back to a restart-from-root round (which
// the other lanes of its wave wait for) only if its blending reaches that limit. At
// 256/128 such rounds are rare on a 100k-Gaussian scene. Structures
// of more than a million leaves defer several hundred nodes per ray, and rays that start
// inside a 3M-Gaussian scene over a thousand, with a long tail: at 2048/512, 2% of such
// rays fell back and the launch took 9% longer than at 8192/2048. At 8192/2048 a few of
// the heaviest rays of 2M still fell back on three of four seeds of incoherent rays, each
// restart costing its ray tens of thousands of visits and the launch 18-37%; at
// 12288/3072 none did on any of them. The lists are per lane, not per ray: 12288/3072
// costs about 48 GB at k = 16 for 3072 waves, affordable in 288 GB. The allocation-free
// entry point, whose lists share a fixed scratch, keeps 2048/512 there so that enough
// workgroups fit.
constexpr int kDefaultDeferCap = 256;
constexpr int kDefaultEvictCap = 128;
constexpr int kLargeDeferCap = 12288;
constexpr int kLargeEvictCap = 3072;
constexpr int kNoAllocLargeDeferCap = 2048;
constexpr int kNoAllocLargeEvictCap = 512;
constexpr int64_t kLargeScene = 1000000;
inline int default_defer_cap(int64_t n_leaves, bool noalloc) {
  return n_leaves <= kLargeScene ? kDefaultDeferCap : noalloc ? kNoAllocLargeDeferCap : kLargeDeferCap;
}
inline int default_evict_cap(int64_t n_leaves, bool noalloc) {
  return n_leaves <= kLargeScene ? kDefaultEvictCap : noalloc ? kNoAllocLargeEvictCap : kLargeEvictCap;
}


enum : int { kIdle = 0, kTrav = 1, kEnd = 2 };

struct TraceArgs {
  const float4* nodes;
  const float4* inst;
  const float4* tris;
  const float* sh;
  const float* roots;         // per scene: root box (lo xyz, hi xyz), root ref bits, 0
  const int32_t* ray_scene;   // per ray scene index, or null (scene 0)
  int sh_degree;
  const float* ray_o;
  const float* ray_d;
  const float* ray_tfar;      // per ray surface distance, or null (unbounded)
  const float* ray_trans;     // per ray starting transmittance, or null (1)
  const float* ray_next_o;    // continuation rays (all four, or all null)
  const float* ray_next_d;
  const float* ray_path;
  const int32_t* ray_kind;
  int64_t n_rays;
  int64_t n_work;
  int64_t n_free;             // rays 0..n_free-1 form no image; the image's rays follow
  int image_w;
  int image_h;
  int tiles_x;
  float t_near;
  int k;
  float T_min;
  int mode;
  float bg0, bg1, bg2;
  float* rgb;
  float* depth;
  float* opac;
  uint32_t* stats;
  int32_t* hit_ids;
  int32_t* hit_counts;
  int hit_cap;
  uint2* pool;
  int64_t rows_per_wave;
  int cap_d;
  int cap_e;
  unsigned int* counter;  // kChunks work counters
  int64_t chunk_len;      // work items per chunk (a multiple of 64)
  const uint32_t* tile_order;  // processing order of the 8x8 tiles, or null (row-major)
  const uint32_t* ray_order;   // processing order of rays that form no image, or null
  int refill;                  // idle lanes that end a traversal burst
  ServeHost* sv_host;          // serving kernel: the work queue (host and device sides)
  ServeDev* sv_dev;
  uint64_t sv_poll_ticks;      // wall-clock ticks between reads of the host's count
  uint64_t sv_idle_ticks;      // wall-clock ticks without work before the launch winds down
};

template <int K>
__device__ __forceinline__ uint64_t kbuf_insert(uint64_t (&kb)[K], uint64_t x) {
  // The buffer is sorted, so "x < kb[j]" holds from x's place on: every compare is against
  // x itself (independent, one per entry) and entry j takes x at that place, its
  // predecessor after it, and stays before it. Returns the entry pushed out (or x).
  bool lt[K];
#pragma unroll
  for (int j = 0; j < K; ++j) lt[j] = x < kb[j];
  const uint64_t out = lt[K - 1] ? kb[K - 1] : x;
#pragma unroll
  for (int j = K - 1; j > 0; --j) kb[j] = lt[j - 1] ? kb[j - 1] : (lt[j] ? x : kb[j]);
  kb[0] = lt[0] ? x : kb[0];
  return out;
}

template <int K>
__device__ __forceinline__ void kbuf_reset(uint64_t (&kb)[K], int k) {
#pragma unroll
  for (int j = 0; j < K; ++j) kb[j] = j < K - k ? 0ull : kEmptyKey;
}

// Proxy leaf: front-facing crossing of a triangle of the bounding icosahedron. Each edge
// function is d . (P x Q) over the edge's end points relative to the ray origin, with
// contraction off: the two triangles that share an edge evaluate it with P and Q swapped
// and get exactly opposite values, so a ray never slips between two faces of a mesh.
// Front-facing (outward normal against the ray) means all three are <= 0.
__device__ __forceinline__ bool proxy_hit(float4 A4, float4 B4, float4 C4, float ox, float oy, float oz, float dx,
                                          float dy, float dz, float* tout) {
#pragma clang fp contract(off)
  const float ax = A4.x - ox, ay = A4.y - oy, az = A4.z - oz;
  const float bx = B4.x - ox, by = B4.y - oy, bz = B4.z - oz;
  const float cx = C4.x - ox, cy = C4.y - oy, cz = C4.z - oz;
  const float sAB = dx * (ay * bz - az * by) + dy * (az * bx - ax * bz) + dz * (ax * by - ay * bx);
  const float sBC = dx * (by * cz - bz * cy) + dy * (bz * cx - bx * cz) + dz * (bx * cy - by * cx);
  const float sCA = dx * (cy * az - cz * ay) + dy * (cz * ax - cx * az) + dz * (cx * ay - cy * ax);
  const float sum = sAB + sBC + sCA;
  // barycentric weights of A, B, C are sBC, sCA, sAB (over their sum)
  *tout = (sBC * (ax * dx + ay * dy + az * dz) + sCA * (bx * dx + by * dy + bz * dz) +
           sAB * (cx * dx + cy * dy + cz * dz)) / sum;
  return sAB <= 0.f && sBC <= 0.f && sCA <= 0.f && sum < 0.f;
}

// Leaf tests: unit sphere of an instance, a world-space proxy triangle, or the shared
// icosahedron (inradius 1) of an instance.
enum : int { kLeafSphere = 0, kLeafTri = 1, kLeafIco = 2 };

// Face normals of the regular icosahedron with vertices at the cyclic permutations of
// (0, +-1, +-phi): the directions (+-1, +-1, +-1) and the cyclic permutations of
// (+-1/phi, 0, +-phi), all of length sqrt(3). Scaled to inradius 1 every face plane is
// n . x = 1 with n the unit normal.
constexpr float kPhi = (float)1.6180339887498948482;
constexpr float kInvPhi = (float)0.6180339887498948482;
constexpr float kInvSqrt3 = (float)0.57735026918962576451;

// Entry distance of the ray through the icosahedron in the unit frame of an instance
// record (rows of A with mu in the fourth lane): the convex-polytope slab test, entry =
// the last crossing of a face plane met from outside, exit = the first crossing from
// inside. The ray parameter is the world one (the map is affine). A ray starting inside
// has its entry behind the origin and is rejected by the caller's t > t_near test.
__device__ __forceinline__ bool ico_entry(float4 r0, float4 r1, float4 r2, float ox, float oy, float oz, float dx,
                                          float dy, float dz, float* tout) {
  const float fx = ox - r0.w, fy = oy - r1.w, fz = oz - r2.w;
  const float u[3] = {r0.x * fx + r0.y * fy + r0.z * fz, r1.x * fx + r1.y * fy + r1.z * fz,
                      r2.x * fx + r2.y * fy + r2.z * fz};
  const float v[3] = {r0.x * dx + r0.y * dy + r0.z * dz, r1.x * dx + r1.y * dy + r1.z * dz,
                      r2.x * dx + r2.y * dy + r2.z * dz};
  float te = -INFINITY, tx = INFINITY;
  bool outside_parallel = false;
  auto face = [&](float nx, float ny, float nz) __attribute__((always_inline)) {
    const float nu = nx * u[0] + ny * u[1] + nz * u[2];
    const float nv = nx * v[0] + ny * v[1] + nz * v[2];
    const float t = (1.f - nu) / nv;
    if (nv < 0.f) te = fmaxf(te, t);
    if (nv > 0.f) tx = fminf(tx, t);
    if (nv == 0.f && nu > 1.f) outside_parallel = true;
  };
#pragma unroll
  for (int q = 0; q < 8; ++q)
    face((q & 1 ? -kInvSqrt3 : kInvSqrt3), (q & 2 ? -kInvSqrt3 : kInvSqrt3), (q & 4 ? -kInvSqrt3 : kInvSqrt3));
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const float a = (q & 1 ? -kInvPhi : kInvPhi) * kInvSqrt3, b = (q & 2 ? -kPhi : kPhi) * kInvSqrt3;
    face(a, 0.f, b);
    face(0.f, b, a);
    face(b, a, 0.f);
  }
  *tout = te;
  return !outside_parallel && te <= tx;
}

// ------------------------------------------------------------------ serving work queue
// Host memory is read with system-scope loads (they bypass the GPU's caches); the
// device-side queue with device-scope atomics, so that all XCDs see one value; served
// outputs are written with device-scope stores, which write through the XCD's L2.
__device__ __forceinline__ uint32_t ld_sys(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
__device__ __forceinline__ uint64_t ld_sys64(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
__device__ __forceinline__ uint32_t ld_dev(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t ld_dev64(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_dev(float* p, float v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Device wall clock (constant rate, hipDeviceAttributeWallClockRate kHz).
__device__ __forceinline__ uint64_t wall_clock() { return __builtin_amdgcn_s_memrealtime(); }
// Wait until this wave's earlier memory writes are complete.
__device__ __forceinline__ void wait_writes() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

__device__ __forceinline__ void st_dev_u32(uint32_t* p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t state_cur(uint64_t st) { return (uint32_t)st; }
__device__ __forceinline__ uint32_t state_pub(uint64_t st) { return (uint32_t)(st >> 32) & 0x7FFFFFFFu; }
typedef unsigned long long ull;

// Descriptors the poller sets up per read of the host's count (bounds one lane's work).
constexpr int kServePollBatch = 64;

// Set up the requests the host has published since the last read: copy their
// descriptors into the device ring, start their claim counters, then raise the published
// count in the state word. One lane at a time (poll_lock), at most once per poll_ticks
// over the launch. A stop from the host closes the queue once everything published has
// been handed out.
__device__ __forceinline__ void serve_poll(ServeDev* q, const ServeHost* h, uint64_t poll_ticks) {
  const uint64_t now = wall_clock();
  if (now - ld_dev64(&q->last_poll) < poll_ticks) return;  // (a clock behind wraps: poll)
  if (atomicCAS(&q->poll_lock, 0u, 1u) != 0u) return;
  atomicExch(reinterpret_cast<ull*>(&q->last_poll), (ull)now);
  const uint64_t hp = ld_sys64(&h->published);
  const uint32_t stop = ld_sys(&h->stop);
  const uint64_t inited = ld_dev64(&q->inited);
  const uint64_t upto = hp < inited + kServePollBatch ? hp : inited + kServePollBatch;
  for (uint64_t j = inited; j < upto; ++j) {
    const uint32_t slot = (uint32_t)(j % kServeRing);
    const uint32_t* src = reinterpret_cast<const uint32_t*>(&h->ring[slot]);
    uint32_t* dst = reinterpret_cast<uint32_t*>(&q->desc[slot]);
    uint32_t v[sizeof(ServeDesc) / 4];
#pragma unroll
    for (int i = 0; i < (int)(sizeof(ServeDesc) / 4); ++i) v[i] = ld_sys(src + i);
#pragma unroll
    for (int i = 0; i < (int)(sizeof(ServeDesc) / 4); ++i) st_dev_u32(dst + i, v[i]);
    wait_writes();  // the descriptor is in place before its counter names the request
    atomicExch(reinterpret_cast<ull*>(&q->slot[slot].claim), (ull)(j << 32));
  }
  if (upto > inited) atomicExch(reinterpret_cast<ull*>(&q->inited), (ull)upto);
  // the state word also changes when the current request moves on or the queue closes;
  // each failed swap means one of those happened
  uint64_t st = ld_dev64(&q->state);
  for (int a = 0; a < 1024 && state_pub(st) < (uint32_t)upto; ++a) {
    const uint64_t nst = (st & (kServeClosing | 0xFFFFFFFFull)) | ((uint64_t)((uint32_t)upto & 0x7FFFFFFFu) << 32);
    const uint64_t seen = atomicCAS(reinterpret_cast<ull*>(&q->state), (ull)st, (ull)nst);
    if (seen == st) {
      st = nst;
      break;
    }
    st = seen;
  }
  if (stop && upto == hp && state_cur(st) >= state_pub(st)) atomicOr(reinterpret_cast<ull*>(&q->state), (ull)kServeClosing);
  atomicExch(&q->poll_lock, 0u);
}

// One lane claims up to `cnt` work items for its wave. Fast path: one atomic add on the
// claim counter of the wave's current request (*myj, in LDS); a counter that names a
// later request (the slot was reused) hands out that request's items, which are just as
// much unclaimed. When the request has no items left, the state word moves past it (if
// it still names it) and the request it names next becomes the wave's. Returns the
// number of items claimed (0: none now; *closed is set when the queue is closing);
// *j_out / *o_out receive their request and first item, and the wave's descriptor copy
// `wd` (LDS) then holds that request.
__device__ __forceinline__ uint32_t serve_claim(ServeDev* q, const ServeHost* h, uint32_t cnt, uint64_t poll_ticks,
                                                uint32_t* myj, ServeDesc* wd, uint32_t* j_out, uint32_t* o_out,
                                                uint32_t* closed) {
  *closed = 0;
  for (int attempt = 0; attempt < 4; ++attempt) {
    const uint32_t jj = *myj;
    if (jj != kServeNoRequest) {
      const uint64_t old = atomicAdd(reinterpret_cast<ull*>(&q->slot[jj % kServeRing].claim), (ull)cnt);
      const uint32_t seq = (uint32_t)(old >> 32), o = (uint32_t)old;
      if ((int32_t)(seq - jj) >= 0) {
        if (wd->seq != seq) {
          const uint32_t* src = reinterpret_cast<const uint32_t*>(&q->desc[seq % kServeRing]);
          uint32_t v[sizeof(ServeDesc) / 4];
#pragma unroll
          for (int i = 0; i < (int)(sizeof(ServeDesc) / 4); ++i) v[i] = ld_dev(src + i);
          uint32_t* dst = reinterpret_cast<uint32_t*>(wd);
#pragma unroll
          for (int i = 0; i < (int)(sizeof(ServeDesc) / 4); ++i) dst[i] = v[i];
        }
        const uint32_t n = wd->seq == seq ? wd->n_work : 0u;
        if (o < n) {
          *myj = seq;
          *j_out = seq;
          *o_out = o;
          return cnt < n - o ? cnt : n - o;
        }
        uint64_t st = ld_dev64(&q->state);
        for (int a = 0; a < 4 && state_cur(st) == seq; ++a) {
          const uint64_t seen = atomicCAS(reinterpret_cast<ull*>(&q->state), (ull)st,
                                          (ull)((st & ~0xFFFFFFFFull) | (uint32_t)(seq + 1)));
          if (seen == st) break;
          st = seen;
        }
      }
      *myj = kServeNoRequest;
    }
    uint64_t st = ld_dev64(&q->state);
    if (st & kServeClosing) {
      *closed = 1;
      return 0;
    }
    if (state_cur(st) >= state_pub(st)) {
      serve_poll(q, h, poll_ticks);
      st = ld_dev64(&q->state);
      if (st & kServeClosing) {
        *closed = 1;
        return 0;
      }
      if (state_cur(st) >= state_pub(st)) return 0;
    }
    *myj = state_cur(st);
  }
  return 0;
}

// The kernel's arguments, read again from the argument segment (scalar loads) at each use
// site inside the ray loop: the empty asm statement hides that the pointer is the same every
// time, so the compiler does not hold every field in scalar registers for the whole kernel
// (too many: they were spilled into vector-register lanes and read back with VALU
// instructions). The trace kernel takes one argument, so it sits at offset 0.
typedef const __attribute__((address_space(4))) TraceArgs KernArgs;
__device__ __forceinline__ KernArgs& kernel_args() {
  auto p = (KernArgs*)__builtin_amdgcn_kernarg_segment_ptr();
  asm volatile("" : "+s"(p));
  return *p;
}

// SERVE: the serving kernel. Work comes from the serving queue instead of the ray arrays:
// each ray is generated from its request's camera, its outputs go to the request's
// buffers, and the lane that completes a request raises its flag in host memory. Idle
// waves wait for new requests and leave once the queue closes.
template <int K, int LEAF, bool STATS, bool SERVE = false>
__global__ void __launch_bounds__(kTraceBlock)
    __attribute__((amdgpu_waves_per_eu(K <= 32 ? GRTX_MIN_WAVES : 2, 8))) k_trace(TraceArgs Args) {
  __shared__ uint2 s_stack[kLdsStack * kTraceBlock];
  __shared__ uint2 s_dst[kStage * kTraceBlock];  // destination node-list entries not yet written out
  constexpr int kStageEv = SERVE ? 0 : kStageE;
  __shared__ uint2 s_edst[kStageEv > 0 ? kStageEv * kTraceBlock : 1];  // eviction-list entries likewise
  __shared__ uint32_t s_stat[STATS ? GRTX_STATS_FIELDS : 1][kTraceBlock];  // per-lane counters
  // serving: each wave's copy of its current request, each lane's output address and its
  // request's pixel count
  __shared__ ServeDesc s_desc[SERVE ? kWaves : 1];
  __shared__ uint32_t s_myj[SERVE ? kWaves : 1];
  __shared__ uint32_t s_out[SERVE ? 3 : 1][SERVE ? kTraceBlock : 1];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const uint64_t lt_mask = lane ? (~0ull >> (64 - lane)) : 0ull;
  const int gwave = __builtin_amdgcn_readfirstlane((int)((blockIdx.x * kTraceBlock + tid) >> 6));
  // The wave's region: first each lane's own entries, lane l at [l * rowK, (l + 1) * rowK):
  // [0, kSpillRows) stack spill, two node lists of cap_d entries and two hit lists of
  // cap_e entries (ping-pong source/destination, selected by `par`); a lane's appends and
  // reads walk its own lines. Then K rows holding the k-buffers while they are blended,
  // entry j of lane l at row j, column l: all blending lanes write row j together.
  uint2* const wbase = Args.pool + (int64_t)gwave * Args.rows_per_wave * 64;
  const int rowN = kSpillRows;
  const int rowE = kSpillRows + 2 * Args.cap_d;
  const int rowK = rowE + 2 * Args.cap_e;
  uint2* const park = wbase + (int64_t)rowK * 64 + lane;
// k-buffer park entry j of this lane, at 64-bit offsets from one base (`pk`, see below)
#define PARK(j) pk[(int64_t)(j) * 64]
#define LROW(r) wbase[(uint32_t)lane * (uint32_t)rowK + (uint32_t)(r)]
#define STAT(f)                        \
  do {                                 \
    if constexpr (STATS) ++s_stat[f][tid]; \
  } while (0)
  const bool ckpt = Args.mode == GRTX_MODE_CHECKPOINT;
  const float tnear = Args.t_near;

  int state = kIdle;
  int ray = -1;
  int sid = 0;  // scene of the lane's ray
  float ox = 0, oy = 0, oz = 0, dx = 0, dy = 0, dz = 0, ix = 0, iy = 0, iz = 0;
  float oix = 0, oiy = 0, oiz = 0;  // origin times inverse direction, for the slab fma
  float tfar = INFINITY;  // the ray ends on a surface there: keys must stay below it
  uint64_t kb[K];
  kbuf_reset(kb, Args.k);
  uint64_t tmin = 0;  // key of the last blended hit
  float C0 = 0, C1 = 0, C2 = 0, Dp = 0, T = 1;
  uint32_t cur_ref = 0;  // item in hand: internal node or leaf (has_cur)
  float cur_t = 0;
  int has_cur = 0;  // per-lane flags held as integers: fewer live lane masks in SGPRs
  uint64_t key = 0;      // hit key waiting for the k-buffer (have_key)
  int have_key = 0;
  int sp = 0;
  int par = 0;                              // which list of each pair is the source
  int nsrc_n = 0, nsrc_i = 0, ndst_n = 0;   // deferred nodes
  int esrc_n = 0, esrc_i = 0, edst_n = 0;   // evicted hits
  // Every hit nearer than `lim` is either blended, in the k-buffer, in a list, or in a
  // deferred subtree; hits from distance `lim` on may have been dropped by a full list
  // (infinity: none).
  float lim = INFINITY;
  int nblend = 0;
  bool exhausted = false;
  int chunk = (int)(blockIdx.x % kChunks);
  int chunks_tried = 0;
  int room_tick = 0;  // traversal iterations of the wave, for the list-room check
  bool nowork = false;       // serving: the last claim found no work
  uint64_t idle_since = 0;   // serving: when the wave last ran out of rays (lane 0)
  if constexpr (SERVE) {
    if (lane == 0) {
      s_desc[tid >> 6].seq = ~0u;
      s_myj[tid >> 6] = kServeNoRequest;
    }
  }

  auto root_start = [&]() __attribute__((always_inline)) {
    // (Re)start at the root; subtrees that end before tmin are culled.
    const float* rb = Args.roots + 8 * sid;
    Slab s = slab(rb[0], rb[1], rb[2], rb[3], rb[4], rb[5], ox, oy, oz, ix, iy, iz);
    float tlo = fmaxf(tnear, key_t(tmin));
    const float tf = fminf(s.tf, tfar);
    has_cur = s.tn <= tf && tf >= tlo;
    cur_ref = __float_as_uint(rb[6]);
    cur_t = s.tn;
    sp = 0;
  };

  // the destination node list's chunk at `pos` (a multiple of kStage) from LDS to HBM
  auto flush_dst = [&](int pos) __attribute__((always_inline)) {
    uint4* q = reinterpret_cast<uint4*>(&LROW(rowN + (par ^ 1) * Args.cap_d + pos));
#pragma unroll
    for (int j = 0; j < kStage / 2; ++j) {
      const uint2 a = s_dst[(2 * j) * kTraceBlock + tid], b = s_dst[(2 * j + 1) * kTraceBlock + tid];
      q[j] = make_uint4(a.x, a.y, b.x, b.y);
    }
  };

  // A nearly full destination list is compacted in place (from the top of the traversal
  // loop, so that the appends in the node and leaf steps always find room): the entries
  // nearer than a threshold stay, the rest are dropped and the limit comes down to the
  // threshold. The threshold starts halfway between the nearest and the farthest entry and
  // halves its distance to the nearest until at most three quarters of the entries stay
  // (after four halvings none stay). Entries a ray needs before early termination are
  // usually the near ones, so it seldom reaches the limit. `row0` is the list's first row,
  // `n` its length (all of it in HBM). Returns the entries kept.
  auto compact = [&](int row0, int n) __attribute__((always_inline)) -> int {
    if (n == 0) return 0;
    // eight entries per step, their four 16-B loads in flight together (a list's rows are
    // a multiple of 8 long and 16-B aligned, so a step may read past n inside the list)
    float lo = INFINITY, hi = 0.f;
#pragma unroll 1
    for (int i = 0; i < n; i += 8) {
      uint4 v[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) v[q] = *reinterpret_cast<const uint4*>(&LROW(row0 + i + 2 * q));
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const float a = __uint_as_float(v[q].y), b = __uint_as_float(v[q].w);
        if (i + 2 * q < n) lo = fminf(lo, a), hi = fmaxf(hi, a);
        if (i + 2 * q + 1 < n) lo = fminf(lo, b), hi = fmaxf(hi, b);
      }
    }
    float thr = fminf(lo + 0.5f * (hi - lo), lim);
    int m = n;
#pragma unroll 1
    for (int it = 0; it < 4; ++it) {
      int w = 0;
#pragma unroll 1
      for (int i = 0; i < m; i += 8) {
        uint4 v[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) v[q] = *reinterpret_cast<const uint4*>(&LROW(row0 + i + 2 * q));
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          if (i + 2 * q < m && __uint_as_float(v[q].y) < thr) LROW(row0 + w++) = make_uint2(v[q].x, v[q].y);
          if (i + 2 * q + 1 < m && __uint_as_float(v[q].w) < thr) LROW(row0 + w++) = make_uint2(v[q].z, v[q].w);
        }
      }
      m = w;
      if (4 * m <= 3 * n) break;
      thr = lo + 0.5f * (thr - lo);
    }
    if (4 * m > 3 * n) {
      m = 0;
      thr = lo;
    }
    lim = fminf(lim, thr);
    return m;
  };

  // (Entries at or beyond the limit may still be appended: the next compaction drops
  // them. One that finds its list full is dropped at once and lowers the limit to it:
  // every hit of a subtree lies at its entry distance or beyond.)
  auto defer = [&](uint32_t ref, float t) __attribute__((always_inline)) {
    if (!ckpt) return;
    if (ndst_n == Args.cap_d) {
      lim = fminf(lim, t);
      return;
    }
    s_dst[(ndst_n & (kStage - 1)) * kTraceBlock + tid] = make_uint2(ref, __float_as_uint(t));
    ++ndst_n;
    if ((ndst_n & (kStage - 1)) == 0) flush_dst(ndst_n - kStage);
    STAT(GRTX_STAT_DEFERRED);
  };

  // the destination eviction list's chunk at `pos` (a multiple of kStageEv) from LDS to HBM
  auto flush_evict = [&](int pos) __attribute__((always_inline)) {
    if constexpr (kStageEv > 0) {
      uint4* q = reinterpret_cast<uint4*>(&LROW(rowE + (par ^ 1) * Args.cap_e + pos));
#pragma unroll
      for (int j = 0; j < kStageEv / 2; ++j) {
        const uint2 a = s_edst[(2 * j) * kTraceBlock + tid], b = s_edst[(2 * j + 1) * kTraceBlock + tid];
        q[j] = make_uint4(a.x, a.y, b.x, b.y);
      }
    }
  };

  auto evict = [&](uint64_t k64) __attribute__((always_inline)) {
    if (!ckpt) return;
    if (edst_n == Args.cap_e) {
      lim = fminf(lim, key_t(k64));
      return;
    }
    if constexpr (kStageEv > 0) {
      s_edst[(edst_n & (kStageEv - 1)) * kTraceBlock + tid] = make_uint2((uint32_t)k64, (uint32_t)(k64 >> 32));
      ++edst_n;
      if ((edst_n & (kStageEv - 1)) == 0) flush_evict(edst_n - kStageEv);
    } else {
      LROW(rowE + (par ^ 1) * Args.cap_e + edst_n) = make_uint2((uint32_t)k64, (uint32_t)(k64 >> 32));
      ++edst_n;
    }
    STAT(GRTX_STAT_EVICTED);
  };

  // Room for kRoomEvery traversal iterations' appends (each appends at most five deferred
  // nodes: one carried entry and four children; and at most one evicted hit), made by
  // compaction; the partial staging chunk goes out first and its survivors come back to
  // LDS. (Lists shorter than that margin are compacted at every check; an append that
  // still finds its list full is dropped and lowers the limit.)
  auto make_room = [&]() __attribute__((always_inline)) {
    if (ndst_n > Args.cap_d - 5 * kRoomEvery) {
      const int row0 = rowN + (par ^ 1) * Args.cap_d;
      if (ndst_n & (kStage - 1)) flush_dst(ndst_n & ~(kStage - 1));
      ndst_n = compact(row0, ndst_n);
#pragma unroll 1
      for (int j = ndst_n & ~(kStage - 1); j < ndst_n; ++j) s_dst[(j & (kStage - 1)) * kTraceBlock + tid] = LROW(row0 + j);
    }
    if (edst_n > Args.cap_e - kRoomEvery) {
      const int row0 = rowE + (par ^ 1) * Args.cap_e;
      if constexpr (kStageEv > 0) {
        if (edst_n & (kStageEv - 1)) flush_evict(edst_n & ~(kStageEv - 1));
      }
      edst_n = compact(row0, edst_n);
      if constexpr (kStageEv > 0) {
#pragma unroll 1
        for (int j = edst_n & ~(kStageEv - 1); j < edst_n; ++j)
          s_edst[(j & (kStageEv - 1)) * kTraceBlock + tid] = LROW(row0 + j);
      }
    }
  };

  auto push = [&](uint32_t ref, float t) __attribute__((always_inline)) {
    // At most three entries per visited record are pending (see kMaxStack), so
    // sp < kMaxStack always; the bound keeps memory safe, and an entry it would drop is
    // counted (GRTX_STAT_STACK_DROPS, zero on every tree the build keeps).
    uint2 e = make_uint2(ref, __float_as_uint(t));
    if (sp < kLdsStack)
      s_stack[sp * kTraceBlock + tid] = e;
    else if (sp < kMaxStack)
      LROW(sp - kLdsStack) = e;
    else
      STAT(GRTX_STAT_STACK_DROPS);
    sp = sp < kMaxStack ? sp + 1 : sp;
  };

  auto pop = [&]() __attribute__((always_inline)) -> uint2 {
    // Two loads of different types in two branches: one load through a selected pointer
    // (what the compiler makes of two alike loads) is a flat load, which waits on LDS and
    // HBM alike.
    --sp;
    uint2 e;
    if (sp < kLdsStack) {
      e = s_stack[sp * kTraceBlock + tid];
    } else {
      const uint64_t v = *reinterpret_cast<const uint64_t*>(&LROW(sp - kLdsStack));
      e = make_uint2((uint32_t)v, (uint32_t)(v >> 32));
    }
    return e;
  };

  while (true) {
    KernArgs& A = kernel_args();
    // ---------------------------------------------------------------- refill idle lanes
    // Serving: one lane claims work items of one request for the wave's idle lanes
    // (serve_claim), which generate their rays from the request's camera.
    // Otherwise the work items are split into kChunks contiguous chunks, each with its own
    // counter (one chunk by default). With several, a wave starts on chunk
    // blockIdx % kChunks (workgroups are dealt round-robin to the 8 XCDs) and moves on to
    // the next chunk when its own is drained.
    if constexpr (SERVE) {
      const uint64_t idle = __ballot(state == kIdle);
      if (idle && !exhausted) {
        const int leader = __ffsll((unsigned long long)idle) - 1;
        uint32_t take = 0, j = 0, o = 0, closed = 0;
        if (lane == leader)
          take = serve_claim(A.sv_dev, A.sv_host, (uint32_t)__popcll(idle), A.sv_poll_ticks, &s_myj[tid >> 6],
                             &s_desc[tid >> 6], &j, &o, &closed);
        take = __shfl(take, leader);
        j = __shfl(j, leader);
        o = __shfl(o, leader);
        closed = __shfl(closed, leader);
        nowork = take == 0;
        if (closed) exhausted = true;
        const uint32_t rank = (uint32_t)__popcll(idle & lt_mask);
        if (state == kIdle && rank < take) {
          const ServeDesc& d = s_desc[tid >> 6];
          const uint32_t w = o + rank;
          const uint32_t* order = reinterpret_cast<const uint32_t*>(d.order);
          const uint32_t tile = order ? order[w >> 6] : w >> 6;
          const uint32_t ty = tile / (uint32_t)d.tiles_x, tx = tile - ty * (uint32_t)d.tiles_x;
          const int px = (int)(tx * 8 + (w & 7)), py = (int)(ty * 8 + ((w >> 3) & 7));
          if (px < d.width && py < d.height) {
            const uint32_t pix = (uint32_t)py * (uint32_t)d.width + (uint32_t)px;
            ray = (int)(((j % kServeRing) << kServePixelBits) | pix);
            s_out[0][tid] = (uint32_t)d.out;
            s_out[1][tid] = (uint32_t)(d.out >> 32);
            s_out[2][tid] = d.n_pixels;
            sid = d.scene;
            ox = d.eye[0]; oy = d.eye[1]; oz = d.eye[2];
            pinhole_dir(d.fwd[0], d.fwd[1], d.fwd[2], d.right[0], d.right[1], d.right[2], d.up[0], d.up[1], d.up[2], px,
                        py, d.width, d.height, &dx, &dy, &dz);
            ix = safe_inv(dx); iy = safe_inv(dy); iz = safe_inv(dz);
            oix = ox * ix; oiy = oy * iy; oiz = oz * iz;
            tfar = INFINITY;
            kbuf_reset(kb, A.k);
            tmin = 0;
            C0 = C1 = C2 = Dp = 0.f;
            T = 1.f;
            nblend = 0;
            par = 0;
            nsrc_n = nsrc_i = ndst_n = 0;
            esrc_n = esrc_i = edst_n = 0;
            lim = INFINITY;
            have_key = false;
            root_start();
            state = kTrav;
          }
        }
      }
      if (__ballot(state != kIdle) == 0) {
        if (exhausted) break;
        if (nowork) {
          // nothing to trace: wait for new requests (checking about every 14 us at first,
          // every 110 us after 100 us), and once this wave has found no work for
          // idle_ticks, close the queue: every wave leaves when its rays are done, and the
          // host starts a new launch for later requests
          uint32_t quit = 0, naps = 4;
          if (lane == 0) {
            const uint64_t now = wall_clock();
            if (idle_since == 0) idle_since = now;
            if (now - idle_since > A.sv_idle_ticks) {
              atomicOr(reinterpret_cast<ull*>(&A.sv_dev->state), (ull)kServeClosing);
              quit = 1;
            }
            if (now - idle_since > 25 * A.sv_poll_ticks) naps = 32;
          }
          if (__shfl(quit, 0)) break;
          naps = __shfl(naps, 0);
#pragma unroll 1
          for (uint32_t z = 0; z < naps; ++z) __builtin_amdgcn_s_sleep(127);
          continue;
        }
      }
      idle_since = 0;
    } else if (!exhausted) {
      uint64_t idle = __ballot(state == kIdle);
      if (idle) {
        int cnt = __popcll(idle);
        int leader = __ffsll((unsigned long long)idle) - 1;
        unsigned int base = 0;
        int64_t avail = 0;
        while (true) {
          if (lane == leader) base = atomicAdd(A.counter + chunk, (unsigned int)cnt);
          base = __shfl(base, leader);
          avail = A.chunk_len - (int64_t)base;
          if (avail > 0) break;
          chunk = chunk + 1 == kChunks ? 0 : chunk + 1;
          if (++chunks_tried == kChunks) {
            exhausted = true;
            break;
          }
        }
        if (state == kIdle && !exhausted) {
          int64_t rank = __popcll(idle & lt_mask);
          int64_t w = (int64_t)chunk * A.chunk_len + base + rank;
          int r = -1;
          if (rank < avail && w < A.n_work) {
            if (w < A.n_free) {
              r = A.ray_order ? (int)A.ray_order[w] : (int)w;
            } else {
              const int64_t wi = w - A.n_free;
              int64_t tile = A.tile_order ? (int64_t)A.tile_order[wi >> 6] : wi >> 6;
              int within = (int)(wi & 63);
              int64_t ty = tile / A.tiles_x, tx = tile - ty * A.tiles_x;
              int64_t px = tx * 8 + (within & 7), py = ty * 8 + (within >> 3);
              if (px < A.image_w && py < A.image_h) r = (int)(A.n_free + py * A.image_w + px);
            }
          }
          if (r >= 0) {
            ray = r;
            sid = A.ray_scene ? A.ray_scene[r] : 0;
            const float* ro = A.ray_o + 3 * (int64_t)r;
            const float* rd = A.ray_d + 3 * (int64_t)r;
            ox = ro[0]; oy = ro[1]; oz = ro[2];
            dx = rd[0]; dy = rd[1]; dz = rd[2];
            ix = safe_inv(dx); iy = safe_inv(dy); iz = safe_inv(dz);
            oix = ox * ix; oiy = oy * iy; oiz = oz * iz;
            tfar = A.ray_tfar ? A.ray_tfar[r] : INFINITY;
            kbuf_reset(kb, A.k);
            tmin = 0;
            C0 = C1 = C2 = Dp = 0.f;
            T = A.ray_trans ? A.ray_trans[r] : 1.f;
            nblend = 0;
            par = 0;
            nsrc_n = nsrc_i = ndst_n = 0;
            esrc_n = esrc_i = edst_n = 0;
            lim = INFINITY;
            have_key = false;
            if constexpr (STATS) {
#pragma unroll
              for (int f = 0; f < GRTX_STATS_FIELDS; ++f) s_stat[f][tid] = 0u;
            }
            root_start();
            state = kTrav;
          }
        }
      }
    }
    if constexpr (!SERVE) {
      if (__ballot(state != kIdle) == 0) {
        if (exhausted) break;
      }
    }

    // ---------------------------------------------------------------- traversal
    // Each iteration runs a node step for the lanes holding an internal node (they descend
    // one record) and then a leaf step for the lanes holding a leaf, including a leaf the
    // node step has just reached, or a pending hit key (the leaf is tested and every key
    // goes through the k-buffer insertion). Both steps in one iteration ("if-if" in Aila
    // and Laine's terms) measured faster here than alternating whole-wave node and leaf
    // steps: every traversing lane progresses in every iteration.
    while (true) {
      const uint64_t trav = __ballot(state == kTrav);
      if (!trav) break;
      const uint64_t waiting = __ballot(state == kEnd) | (exhausted || nowork ? 0ull : __ballot(state == kIdle));
      if (__popcll(waiting) >= A.refill) break;
      if ((++room_tick & (kRoomEvery - 1)) == 0 && state == kTrav && ckpt) make_room();
      const uint64_t tmax = kb[K - 1];
      const float tmax_t = key_t(tmax);
      if (state == kTrav && !has_cur && !have_key) {
        // acquire: evicted hits of earlier rounds first, then the stack, then the source
        // checkpoint list; entries already beyond t_max are carried without a fetch
        if (esrc_i < esrc_n) {
          uint2 v = LROW(rowE + par * A.cap_e + esrc_i);
          ++esrc_i;
          key = ((uint64_t)v.y << 32) | v.x;
          have_key = true;
        } else {
          uint2 e;
          bool got = true;
          if (sp > 0) {
            e = pop();
          } else if (nsrc_i < nsrc_n) {
            e = LROW(rowN + par * A.cap_d + nsrc_i);
            ++nsrc_i;
          } else {
            got = false;
            state = kEnd;
          }
          if (got) {
            float t = __uint_as_float(e.y);
            if (t > tmax_t) {
              defer(e.x, t);
              STAT(GRTX_STAT_FETCH_FREE);
            } else {
              cur_ref = e.x;
              cur_t = t;
              has_cur = true;
            }
          }
        }
      }
      const bool nodey = state == kTrav && has_cur && !(cur_ref & kLeafFlag);
      if (__ballot(nodey) != 0) {
        if (nodey) {
          // ------------------------------------------------ node step: four children
          // Slab distances straight from the 8-bit planes: t = q * (s * inv) + (o - ray) * inv.
          // A child's entry is raised to at least the entry of the node in hand, so entries
          // never decrease along a path whatever the rounding, and a node whose entry exceeds
          // t_max holds no key at or below t_max (keys are clamped to their leaf's entry).
          const float4* np = A.nodes + kNodeF4 * (int64_t)cur_ref;
          const float4 q0 = np[0], q1 = np[1], q2 = np[2], q3 = np[3];
          STAT(GRTX_STAT_NODES);
          const float tlo = fmaxf(tnear, key_t(tmin));
          const float Ax = q0.w * ix, Ay = q1.x * iy, Az = q1.y * iz;
          // (record origin - ray origin) * inv as one fma per axis; the rounding differs from
          // the subtract-then-multiply form by a few ulps, far inside the leaf boxes' padding
          const float Bx = fmaf(q0.x, ix, -oix), By = fmaf(q0.y, iy, -oiy), Bz = fmaf(q0.z, iz, -oiz);
          const uint32_t wlx = __float_as_uint(q2.z), wly = __float_as_uint(q2.w), wlz = __float_as_uint(q3.x);
          const uint32_t whx = __float_as_uint(q3.y), why = __float_as_uint(q3.z), whz = __float_as_uint(q3.w);
          // The entry plane of an axis is the low one where the ray's direction is positive
          // (t grows with the plane coordinate, and the rounding of fma keeps that order), so
          // the planes are chosen once per record instead of a min and a max per child.
          const uint32_t wnx = ix < 0.f ? whx : wlx, wfx = ix < 0.f ? wlx : whx;
          const uint32_t wny = iy < 0.f ? why : wly, wfy = iy < 0.f ? wly : why;
          const uint32_t wnz = iz < 0.f ? whz : wlz, wfz = iz < 0.f ? wlz : whz;
          uint32_t c[4] = {__float_as_uint(q1.z), __float_as_uint(q1.w), __float_as_uint(q2.x), __float_as_uint(q2.y)};
          float t[4];
  #pragma unroll
          for (int j = 0; j < 4; ++j) {
            const float tnx = fmaf((float)((wnx >> (8 * j)) & 0xFFu), Ax, Bx);
            const float tfx = fmaf((float)((wfx >> (8 * j)) & 0xFFu), Ax, Bx);
            const float tny = fmaf((float)((wny >> (8 * j)) & 0xFFu), Ay, By);
            const float tfy = fmaf((float)((wfy >> (8 * j)) & 0xFFu), Ay, By);
            const float tnz = fmaf((float)((wnz >> (8 * j)) & 0xFFu), Az, Bz);
            const float tfz = fmaf((float)((wfz >> (8 * j)) & 0xFFu), Az, Bz);
            const float tn = fmaxf(fmaxf(tnx, tny), tnz);
            const float tf = fminf(fminf(fminf(tfx, tfy), tfz), tfar);
            const float te = fmaxf(tn, cur_t);
            bool v = c[j] != kNoChild && fmaxf(tn, tlo) <= tf;  // entered, and not ended before tlo
            if (v && te > tmax_t) {
              defer(c[j], te);
              v = false;
            }
            t[j] = v ? te : INFINITY;
          }
          // near-to-far order of the children still in play (sorting network on (t, ref))
          auto cswap = [&](int a, int b) __attribute__((always_inline)) {
            const bool sw = t[b] < t[a];
            const float ta = t[a], tb = t[b];
            const uint32_t ca = c[a], cb = c[b];
            t[a] = sw ? tb : ta;
            t[b] = sw ? ta : tb;
            c[a] = sw ? cb : ca;
            c[b] = sw ? ca : cb;
          };
          cswap(0, 1);
          cswap(2, 3);
          cswap(0, 2);
          cswap(1, 3);
          cswap(1, 2);
          if (t[3] < INFINITY) push(c[3], t[3]);
          if (t[2] < INFINITY) push(c[2], t[2]);
          if (t[1] < INFINITY) push(c[1], t[1]);
          has_cur = t[0] < INFINITY;
          cur_ref = c[0];
          cur_t = t[0];
        }
      }
      // lanes holding a leaf (also one just reached by the node step above) or a key
      const bool leafy = state == kTrav && (have_key || (has_cur && (cur_ref & kLeafFlag)));
      if (__ballot(leafy)) {
        // ------------------------------------------------ leaf step
        if (leafy && !have_key) {
          const uint32_t p = cur_ref & ~kLeafFlag;
          STAT(GRTX_STAT_LEAVES);
          has_cur = false;
          // A key never precedes the entry of the leaf's own box, so every ancestor's
          // entry distance bounds the keys below it exactly.
          if constexpr (LEAF == kLeafTri) {
            const float4* tp = A.tris + 3 * (int64_t)p;
            float4 a4 = tp[0], b4 = tp[1], c4 = tp[2];
            float tt;
            const bool hit = proxy_hit(a4, b4, c4, ox, oy, oz, dx, dy, dz, &tt);
            key = make_key(fmaxf(tt, cur_t), __float_as_uint(a4.w));
            have_key = hit && tt > tnear && tt < tfar && key > tmin;
          } else if constexpr (LEAF == kLeafIco) {
            const float4* ip = A.inst + 4 * (int64_t)p;
            float tt;
            const bool hit = ico_entry(ip[0], ip[1], ip[2], ox, oy, oz, dx, dy, dz, &tt);
            key = make_key(fmaxf(tt, cur_t), p);
            have_key = hit && tt > tnear && tt < tfar && key > tmin;
          } else {
            const float4* ip = A.inst + 4 * (int64_t)p;
            float4 r0 = ip[0], r1 = ip[1], r2 = ip[2];
            SphereHit h = sphere_terms(r0, r1, r2, ox, oy, oz, dx, dy, dz);
            if (h.a > 0.f && h.c2 <= h.a) {
              const float t0 = (-h.b - __builtin_amdgcn_sqrtf(fmaxf(h.a - h.c2, 0.f))) * __builtin_amdgcn_rcpf(h.a);
              key = make_key(fmaxf(t0, cur_t), p);
              have_key = t0 > tnear && t0 < tfar && key > tmin;
            }
          }
        }
        // any-hit: keys beyond the farthest entry of a full k-buffer are rejected into
        // the eviction list; otherwise the key is inserted and the entry it pushes out of
        // a full buffer is evicted. The insertion runs under a wave-uniform branch with the
        // empty key (a no-op) on lanes without a key, so the registers update in place.
        const bool ins = have_key && key <= tmax;
        if (__ballot(ins)) {
          uint64_t out = kbuf_insert(kb, ins ? key : kEmptyKey);
          if (ins && out != kEmptyKey) evict(out);
        }
        if (have_key && !ins) evict(key);
        have_key = false;
      }
    }

    // ---------------------------------------------------------------- round end: blend
    if (state == kEnd) {
      STAT(GRTX_STAT_ROUNDS);
      const int ncoef = (A.sh_degree + 1) * (A.sh_degree + 1);
      bool ert = false;
      // Blend in key order. The k-buffer is parked in the lane's rows so that the blend
      // loop indexes memory rather than a register array.
      const uint64_t last = kb[K - 1];
      // The base gets an offset that passes through an empty asm statement (it is zero), so
      // that the compiler cannot hoist the K entry addresses out of the ray loop
      // (where they would be spilled); the offsets fold into the store and load
      // instructions, and the pointer stays a global one.
      int opaque_zero = 0;
      asm volatile("" : "+s"(opaque_zero));
      uint2* const pk = park + opaque_zero;
#pragma unroll
      for (int j = 0; j < K; ++j)
        if (j >= K - A.k) PARK(j) = make_uint2((uint32_t)kb[j], (uint32_t)(kb[j] >> 32));
      // proxy keys carry the Gaussian id: a mesh crossed exactly on an edge reports the
      // same Gaussian twice with adjacent keys; only the first is blended
      uint32_t prev_id = tmin == 0ull ? 0xFFFFFFFFu : (uint32_t)tmin;
      // the next entry's key is read while the current one blends; blending stops at the
      // first hit at or beyond the limit (hits there may be missing), and `lastp` is the last
      // key taken
      uint2 kv = PARK(K - A.k);
      uint64_t lastp = tmin;
      bool stopped = false;
#pragma unroll 1
      for (int j = K - A.k; j < K && !ert; ++j) {
        const uint64_t x = ((uint64_t)kv.y << 32) | kv.x;
        if (x == kEmptyKey) break;
        if (key_t(x) >= lim) {
          stopped = true;
          break;
        }
        lastp = x;
        kv = PARK(j + 1 < K ? j + 1 : j);  // unconditional: no join right after the load
        const uint32_t p = (uint32_t)x;
        const float4* ip = A.inst + 4 * (int64_t)p;
        float4 r0 = ip[0], r1 = ip[1], r2 = ip[2], r3 = ip[3];
        SphereHit h = sphere_terms(r0, r1, r2, ox, oy, oz, dx, dy, dz);
        bool blend = true;
        if constexpr (LEAF != kLeafSphere) {
          // a proxy hit counts only if the ray meets the bounding ellipsoid itself
          blend = p != prev_id && h.a > 0.f && h.c2 <= h.a;
          prev_id = p;
        }
        if (blend) {
          // hardware reciprocal and exp2 (about 1 ulp each); the exponent lies in
          // [-log2(o / alpha_min), 0], far from the denormal range a library exp2f guards
          const float inva = __builtin_amdgcn_rcpf(h.a);
          const float cperp = h.c2 * inva;
          const float talpha = -h.b * inva;
          const float alpha = r3.x * __builtin_amdgcn_exp2f(-r3.y * cperp);
          const uint32_t gid = __float_as_uint(r3.z);
          float c[3] = {0.5f, 0.5f, 0.5f};
          const float dn = rsqrtf(dx * dx + dy * dy + dz * dz);
          float Y[16];
          sh_basis(dx * dn, dy * dn, dz * dn, A.sh_degree, Y);
          if (A.sh_degree == 3) {
            // all twelve loads in flight at once, then the sums
            const float4* sp4 = reinterpret_cast<const float4*>(A.sh + (int64_t)gid * 48);
            float4 shv[12];
#pragma unroll
            for (int q = 0; q < 12; ++q) shv[q] = sp4[q];
#pragma unroll
            for (int q = 0; q < 12; ++q) {
              const float* vv = reinterpret_cast<const float*>(&shv[q]);
#pragma unroll
              for (int e = 0; e < 4; ++e) {
                const int f = 4 * q + e;
                c[f % 3] += Y[f / 3] * vv[e];
              }
            }
          } else {
            const float* sc = A.sh + (int64_t)gid * 3 * ncoef;
#pragma unroll
            for (int f = 0; f < 16; ++f) {
              if (f < ncoef) {
                c[0] += Y[f] * sc[3 * f + 0];
                c[1] += Y[f] * sc[3 * f + 1];
                c[2] += Y[f] * sc[3 * f + 2];
              }
            }
          }
          const float w = T * alpha;
          C0 += w * fmaxf(c[0], 0.f);
          C1 += w * fmaxf(c[1], 0.f);
          C2 += w * fmaxf(c[2], 0.f);
          Dp += w * talpha;
          T *= (1.f - alpha);
          if (A.hit_ids && nblend < A.hit_cap) A.hit_ids[(int64_t)ray * A.hit_cap + nblend] = (int32_t)gid;
          ++nblend;
          if (T < A.T_min) ert = true;
        }  // blend
      }
      // every path below starts the buffer afresh (a finished lane's on its next ray), so
      // the old entries are dead from the park on and hold no registers through the blend
      kbuf_reset(kb, A.k);
      const bool full = last != kEmptyKey;
      // with a limit, "no hit left" holds only below it
      const bool limited = lim != INFINITY;
      const bool done = ert || (!limited && (!full || (ckpt && ndst_n == 0 && edst_n == 0)));
      // A segment that reached its surface with T >= T_min goes on along its reflected or
      // refracted ray in the same lane: colour, transmittance and the hit list carry over,
      // and the continuation's distances start at the bent path length.
      bool cont = false;
      if (done && A.ray_kind && tfar != INFINITY && T >= A.T_min) {
        const int kd = A.ray_kind[ray];
        cont = kd == GRTX_OBJECT_MIRROR || kd == GRTX_OBJECT_GLASS;
      }
      if (cont) {
        const float* no = A.ray_next_o + 3 * (int64_t)ray;
        const float* nd = A.ray_next_d + 3 * (int64_t)ray;
        ox = no[0]; oy = no[1]; oz = no[2];
        dx = nd[0]; dy = nd[1]; dz = nd[2];
        ix = safe_inv(dx); iy = safe_inv(dy); iz = safe_inv(dz);
        oix = ox * ix; oiy = oy * iy; oiz = oz * iz;
        Dp = fmaf(A.ray_path[ray], T, Dp);
        tfar = INFINITY;
        tmin = 0;
        par = 0;
        nsrc_n = nsrc_i = ndst_n = 0;
        esrc_n = esrc_i = edst_n = 0;
        lim = INFINITY;
        root_start();
        state = kTrav;
      } else if (done && SERVE) {
        // served ray: outputs to the request's buffers, written through to device scope;
        // then one count per request among the lanes finishing here, and the lane whose
        // count completes a request resets its counter and raises its flag in host memory
        const uint32_t slot = (uint32_t)ray >> kServePixelBits;
        const uint32_t pix = (uint32_t)ray & ((1u << kServePixelBits) - 1u);
        float* out = reinterpret_cast<float*>(((uint64_t)s_out[1][tid] << 32) | s_out[0][tid]);
        const uint32_t n = s_out[2][tid];
        st_dev(out + 3 * (int64_t)pix + 0, C0 + T * A.bg0);
        st_dev(out + 3 * (int64_t)pix + 1, C1 + T * A.bg1);
        st_dev(out + 3 * (int64_t)pix + 2, C2 + T * A.bg2);
        st_dev(out + 3 * (int64_t)n + pix, Dp);
        st_dev(out + 4 * (int64_t)n + pix, 1.f - T);
        wait_writes();
        uint64_t fin = __ballot(true);
        while (fin) {
          const int l0 = __ffsll((unsigned long long)fin) - 1;
          const uint32_t s0 = __shfl(slot, l0);
          const uint64_t same = __ballot(slot == s0);
          if (lane == l0) {
            const uint32_t c = (uint32_t)__popcll(same);
            if (atomicAdd(&A.sv_dev->slot[s0].done, c) + c == n) {
              atomicExch(&A.sv_dev->slot[s0].done, 0u);
              wait_writes();
              __hip_atomic_store(&A.sv_host->done[s0], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            }
          }
          fin &= ~same;
        }
        state = kIdle;
      } else if (done) {
        // the background shows only through rays that no surface ends
        const float bgT = tfar == INFINITY ? T : 0.f;
        A.rgb[3 * (int64_t)ray + 0] = C0 + bgT * A.bg0;
        A.rgb[3 * (int64_t)ray + 1] = C1 + bgT * A.bg1;
        A.rgb[3 * (int64_t)ray + 2] = C2 + bgT * A.bg2;
        // a continued ray (its bound was lifted): the continuation's weights sum to
        // T_switch - T, so take path * T back off
        if (A.ray_kind && tfar == INFINITY && A.ray_tfar[ray] != INFINITY) Dp = fmaf(-A.ray_path[ray], T, Dp);
        A.depth[ray] = Dp;
        A.opac[ray] = 1.f - T;
        if (A.hit_counts) A.hit_counts[ray] = nblend;
        if constexpr (STATS) {
          s_stat[GRTX_STAT_BLENDED][tid] = (uint32_t)nblend;
          uint32_t* st = A.stats + (int64_t)ray * GRTX_STATS_FIELDS;
#pragma unroll
          for (int f = 0; f < GRTX_STATS_FIELDS; ++f) st[f] = s_stat[f][tid];
        }
        state = kIdle;
      } else {
        tmin = lastp;
        if (!ckpt || stopped || (limited && (!full || (ndst_n == 0 && edst_n == 0)))) {
          // restart from the root beyond the last blended hit: restart mode, or a
          // checkpoint whose lists dropped entries and whose remaining keys below the
          // limit are all blended
          if (ckpt) STAT(GRTX_STAT_FALLBACKS);
          lim = INFINITY;
          nsrc_n = nsrc_i = ndst_n = 0;
          esrc_n = esrc_i = edst_n = 0;
          root_start();
        } else {
          // resume: this round's destination lists become the next round's sources (the
          // last, partial chunk of deferred nodes goes out first)
          if (ndst_n & (kStage - 1)) flush_dst(ndst_n & ~(kStage - 1));
          if constexpr (kStageEv > 0) {
            if (edst_n & (kStageEv - 1)) flush_evict(edst_n & ~(kStageEv - 1));
          }
          par ^= 1;
          nsrc_n = ndst_n;
          nsrc_i = 0;
          ndst_n = 0;
          esrc_n = edst_n;
          esrc_i = 0;
          edst_n = 0;
          has_cur = false;
          sp = 0;
        }
        state = kTrav;
      }
    }
  }
#undef PARK
#undef LROW
#undef STAT
}

__global__ void k_reset_counter(unsigned int* c) {
  if (threadIdx.x < kChunks) c[threadIdx.x] = 0u;
}

// Per-tile cost estimate from the tree's subtree cut: the leaf counts of the cut subtrees
// whose boxes the tile's centre ray crosses (how many Gaussians lie near the ray). A block
// takes kEstTiles tiles (positions of the base order) in slices of threads that share out
// the cut, read in chunks through LDS. The key is the estimate's eighth-octave bucket,
// largest first, for a one-pass stable sort that keeps the base order within a bucket.
constexpr int kEstTiles = 8;
constexpr int kEstSlices = 256 / kEstTiles;
__global__ void __launch_bounds__(256) k_tile_estimate(const float4* __restrict__ cut,
                                                       const uint32_t* __restrict__ n_cut,
                                                       const float* __restrict__ ro, const float* __restrict__ rd,
                                                       int w, int h, int tiles_x, int64_t n_tiles,
                                                       const uint32_t* __restrict__ base,
                                                       uint64_t* __restrict__ keys, uint32_t* __restrict__ vals) {
  __shared__ float4 s_cut[2 * 256];
  __shared__ float part[kEstSlices][kEstTiles];
  const int ti = threadIdx.x % kEstTiles, sl = threadIdx.x / kEstTiles;
  const int64_t i = blockIdx.x * (int64_t)kEstTiles + ti;
  float ox = 0.f, oy = 0.f, oz = 0.f, ix = 0.f, iy = 0.f, iz = 0.f;
  if (i < n_tiles) {
    const int64_t t = base[i];
    const int64_t ty = t / tiles_x, tx = t - ty * tiles_x;
    const int64_t px = tx * 8 + 4 < w ? tx * 8 + 4 : w - 1, py = ty * 8 + 4 < h ? ty * 8 + 4 : h - 1;
    const int64_t r = py * w + px;
    ox = ro[3 * r];
    oy = ro[3 * r + 1];
    oz = ro[3 * r + 2];
    ix = safe_inv(rd[3 * r]);
    iy = safe_inv(rd[3 * r + 1]);
    iz = safe_inv(rd[3 * r + 2]);
  }
  const int n = (int)min(*n_cut, (uint32_t)kCutCap);
  float acc = 0.f;
  for (int c0 = 0; c0 < n; c0 += 256) {
    const int m = min(256, n - c0);
    __syncthreads();
    if ((int)threadIdx.x < m) {
      s_cut[2 * threadIdx.x] = cut[2 * (c0 + threadIdx.x)];
      s_cut[2 * threadIdx.x + 1] = cut[2 * (c0 + threadIdx.x) + 1];
    }
    __syncthreads();
    for (int j = sl; j < m; j += kEstSlices) {
      const float4 lo = s_cut[2 * j], hi = s_cut[2 * j + 1];
      const Slab sb = slab(lo.x, lo.y, lo.z, hi.x, hi.y, hi.z, ox, oy, oz, ix, iy, iz);
      if (sb.tn <= sb.tf && sb.tf >= 0.f) acc += lo.w;
    }
  }
  part[sl][ti] = acc;
  __syncthreads();
  if (sl == 0 && i < n_tiles) {
    float sum = 0.f;
    for (int q = 0; q < kEstSlices; ++q) sum += part[q][ti];
    const int b = min(255, (int)(8.f * log2f(1.f + sum)));
    keys[i] = (uint64_t)(255 - b);
    vals[i] = base[i];
  }
}

// Tile order for rays that continue past an object: the tiles holding such rays go first.
// Those rays run longest (two segments); started last, they would set the end of the
// launch, while rows of tiles in image order keep neighbouring rays together.
__global__ void __launch_bounds__(256) k_tile_heavy(const int32_t* __restrict__ kind, const uint32_t* __restrict__ base,
                                                    int w, int h, int tiles_x, int64_t n_tiles,
                                                    uint32_t* __restrict__ flag) {
  const int64_t i = blockIdx.x * (int64_t)256 + threadIdx.x;
  if (i >= n_tiles) return;
  const int64_t t = base[i];
  const int64_t ty = t / tiles_x, tx = t - ty * tiles_x;
  uint32_t f = 0;
  for (int j = 0; j < 64; ++j) {
    const int64_t px = tx * 8 + (j & 7), py = ty * 8 + (j >> 3);
    if (px < w && py < h) {
      const int k = kind[py * w + px];
      f |= (k == GRTX_OBJECT_MIRROR || k == GRTX_OBJECT_GLASS) ? 1u : 0u;
    }
  }
  flag[i] = f;
}

// Stable partition of the base order: flagged tiles first.
__global__ void __launch_bounds__(256) k_tile_order(const uint32_t* __restrict__ base, const uint32_t* __restrict__ flag,
                                                    const uint32_t* __restrict__ pos, int64_t n_tiles,
                                                    uint32_t* __restrict__ order) {
  const int64_t i = blockIdx.x * (int64_t)256 + threadIdx.x;
  if (i >= n_tiles) return;
  const int64_t heavy = (int64_t)pos[n_tiles - 1] + flag[n_tiles - 1];
  const int64_t dst = flag[i] ? (int64_t)pos[i] : heavy + (i - (int64_t)pos[i]);
  order[dst] = base[i];
}

// Outputs of rays that meet nothing (a structure without leaves).
// Order of rays that form no image: the few rays that start where the leaves are densest
// run longest (one that starts inside a dense cluster enters the box of every Gaussian
// around its origin), and started late they set the end of the launch. Each ray gets a
// bucket of the density at its origin (quarter octaves of the leaf count of its grid cell;
// 0 outside the grid or in an empty cell); the top buckets that together hold at most
// kHeavyFrac of the rays go first, and every other ray keeps the caller's order after them.
// (Ordering all rays by cost was slower than the caller's order: the heaviest then run
// together and their waves diverge the most.)
constexpr int kOrderBuckets = 128;
constexpr float kHeavyFrac = 0.02f;
constexpr int64_t kOrderMinRays = 65536;

__global__ void k_zero_u32(uint32_t* p, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0u;
}

__global__ void __launch_bounds__(256) k_ray_bucket(const float* __restrict__ ro, int64_t R, const float* __restrict__ box,
                                                    const uint32_t* __restrict__ density, uint32_t* __restrict__ bucket,
                                                    uint32_t* __restrict__ hist) {
  __shared__ uint32_t h[kOrderBuckets];
  for (int i = threadIdx.x; i < kOrderBuckets; i += 256) h[i] = 0u;
  __syncthreads();
  const int64_t r = blockIdx.x * (int64_t)256 + threadIdx.x;
  if (r < R) {
    const float x = ro[3 * r], y = ro[3 * r + 1], z = ro[3 * r + 2];
    const bool inside = x >= box[0] && y >= box[1] && z >= box[2] && x <= box[3] && y <= box[4] && z <= box[5];
    const uint32_t d = inside ? density[density_cell(x, y, z, box)] : 0u;
    const int q = d == 0u ? 0 : 1 + (int)(4.f * log2f((float)d));
    const uint32_t bk = (uint32_t)(q < kOrderBuckets ? q : kOrderBuckets - 1);
    bucket[r] = bk;
    atomicAdd(&h[bk], 1u);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kOrderBuckets; i += 256)
    if (h[i]) atomicAdd(&hist[i], h[i]);
}

__global__ void k_ray_split(const uint32_t* __restrict__ hist, int64_t R, uint32_t* __restrict__ thr) {
  if (threadIdx.x != 0) return;
  const uint64_t cap = (uint64_t)(kHeavyFrac * (float)R);
  uint64_t acc = 0;
  uint32_t t = kOrderBuckets;  // none
  for (int b = kOrderBuckets - 1; b >= 1; --b) {
    if (acc + hist[b] > cap) break;
    acc += hist[b];
    t = (uint32_t)b;
  }
  *thr = t;
}

__global__ void __launch_bounds__(256) k_ray_flags(const uint32_t* __restrict__ bucket, int64_t R,
                                                   const uint32_t* __restrict__ thr, uint32_t* __restrict__ flag) {
  const int64_t r = blockIdx.x * (int64_t)256 + threadIdx.x;
  if (r < R) flag[r] = bucket[r] >= *thr ? 1u : 0u;
}

__global__ void __launch_bounds__(256) k_ray_order(const uint32_t* __restrict__ flag, const uint32_t* __restrict__ pos,
                                                   int64_t R, uint32_t* __restrict__ order) {
  const int64_t r = blockIdx.x * (int64_t)256 + threadIdx.x;
  if (r >= R) return;
  const uint32_t heavy = pos[R - 1] + flag[R - 1];
  order[flag[r] ? pos[r] : heavy + (uint32_t)r - pos[r]] = (uint32_t)r;
}

__global__ void __launch_bounds__(256) k_fill_background(float* rgb, float* depth, float* opac, uint32_t* stats,
                                                         int32_t* hit_counts, const float* tfar,
                                                         const float* trans, int64_t n, float b0, float b1,
                                                         float b2) {
  int64_t i = blockIdx.x * (int64_t)256 + threadIdx.x;
  if (i >= n) return;
  const float T = trans ? trans[i] : 1.f;
  const float bgT = !tfar || tfar[i] == INFINITY ? T : 0.f;
  rgb[3 * i] = bgT * b0;
  rgb[3 * i + 1] = bgT * b1;
  rgb[3 * i + 2] = bgT * b2;
  depth[i] = 0.f;
  opac[i] = 1.f - T;
  if (hit_counts) hit_counts[i] = 0;
  if (stats)
    for (int f = 0; f < GRTX_STATS_FIELDS; ++f) stats[i * GRTX_STATS_FIELDS + f] = 0u;
}

// ------------------------------------------------------------------ per-stream pools

struct Pool {
  void* ptr = nullptr;
  size_t bytes = 0;
  unsigned int* counter = nullptr;
};

std::mutex g_pool_lock;
std::map<std::pair<int, hipStream_t>, Pool> g_pools;

template <int K, int LEAF>
grtx_status launch(const TraceArgs& a, int blocks, hipStream_t s) {
  if (a.stats)
    hipLaunchKernelGGL((k_trace<K, LEAF, true>), dim3(blocks), dim3(kTraceBlock), 0, s, a);
  else
    hipLaunchKernelGGL((k_trace<K, LEAF, false>), dim3(blocks), dim3(kTraceBlock), 0, s, a);
  GRTX_LAUNCH_CHECK();
  return GRTX_OK;
}

// Resident workgroups per CU of one kernel variant (the counting variant holds its
// counters in LDS and may fit fewer; each launch takes its own kernel's figure, results
// do not depend on it).
template <int K, int LEAF>
int blocks_per_cu(bool stats) {
  int nb = 0;
  const hipError_t e = stats ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_trace<K, LEAF, true>, kTraceBlock, 0)
                             : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_trace<K, LEAF, false>, kTraceBlock, 0);
  return e == hipSuccess ? std::max(1, nb) : 1;
}

template <int LEAF>
int blocks_per_cu_k(int K, bool stats) {
  return K == 4 ? blocks_per_cu<4, LEAF>(stats) : K == 8 ? blocks_per_cu<8, LEAF>(stats)
       : K == 16 ? blocks_per_cu<16, LEAF>(stats) : K == 32 ? blocks_per_cu<32, LEAF>(stats)
       : blocks_per_cu<64, LEAF>(stats);
}

// List capacities as the kernel uses them: the default for the structure's size when 0,
// rounded up to whole LDS staging chunks.
inline int stage_round(int c) { return (c + kStage - 1) / kStage * kStage; }

template <int LEAF>
grtx_status launch_k(int K, const TraceArgs& a, int blocks, hipStream_t s) {
  switch (K) {
    case 4: return launch<4, LEAF>(a, blocks, s);
    case 8: return launch<8, LEAF>(a, blocks, s);
    case 16: return launch<16, LEAF>(a, blocks, s);
    case 32: return launch<32, LEAF>(a, blocks, s);
    default: return launch<64, LEAF>(a, blocks, s);
  }
}

// The serving kernel leaves this many CUs' worth of workgroup slots free, so that other
// work on the device (copies of results, other streams' kernels) is not shut out while it
// runs.
constexpr int kServeSpareCUs = 8;

template <int K>
int serve_blocks_per_cu() {
  int nb = 0;
  const hipError_t e =
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_trace<K, kLeafSphere, false, true>, kTraceBlock, 0);
  return e == hipSuccess ? std::max(1, nb) : 1;
}

inline int serve_k(int k) { return k <= 4 ? 4 : k <= 8 ? 8 : k <= 16 ? 16 : k <= 32 ? 32 : 64; }

int serve_blocks(int K) {
  int device = 0, cus = 0;
  if (hipGetDevice(&device) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) return 0;
  const int bpc = K == 4 ? serve_blocks_per_cu<4>() : K == 8 ? serve_blocks_per_cu<8>()
                : K == 16 ? serve_blocks_per_cu<16>() : K == 32 ? serve_blocks_per_cu<32>() : serve_blocks_per_cu<64>();
  return std::max(1, cus - kServeSpareCUs) * bpc;
}

inline int64_t serve_rows(int K) {
  return kSpillRows + 2 * (int64_t)stage_round(kServeDeferCap) + 2 * (int64_t)stage_round(kServeEvictCap) + K;
}

}  // namespace

int64_t serve_pool_bytes(int k) {
  const int K = serve_k(k);
  return (int64_t)serve_blocks(K) * kWaves * serve_rows(K) * 64 * (int64_t)sizeof(uint2);
}

namespace {
// Reopen the queue for a new launch (stream-ordered after the previous one).
__global__ void k_serve_reopen(ServeDev* q) {
  if (threadIdx.x == 0) atomicAnd(reinterpret_cast<unsigned long long*>(&q->state), ~(unsigned long long)kServeClosing);
}
}  // namespace

grtx_status launch_serve(const ServeLaunch& L, hipStream_t s) {
  const int K = serve_k(L.k);
  const int blocks = serve_blocks(K);
  if (blocks <= 0) {
    set_error("serving: no device");
    return GRTX_ERR_DEVICE;
  }
  TraceArgs a{};
  a.nodes = L.scene.nodes;
  a.inst = L.scene.inst;
  a.sh = L.scene.sh;
  a.roots = L.scene.roots;
  a.sh_degree = L.scene.sh_degree;
  a.t_near = 0.f;
  a.k = L.k;
  a.T_min = L.T_min;
  a.mode = L.mode;
  a.bg0 = L.bg[0];
  a.bg1 = L.bg[1];
  a.bg2 = L.bg[2];
  a.pool = static_cast<uint2*>(L.pool);
  a.rows_per_wave = serve_rows(K);
  a.cap_d = stage_round(kServeDeferCap);
  a.cap_e = stage_round(kServeEvictCap);
  a.sv_host = L.host;
  a.sv_dev = L.dev;
  a.sv_poll_ticks = L.poll_ticks;
  a.sv_idle_ticks = L.idle_ticks;
  a.refill = L.scene.n_leaves > kLargeScene ? kRefillLarge : kRefillSmall;
  hipLaunchKernelGGL(k_serve_reopen, dim3(1), dim3(64), 0, s, L.dev);
  switch (K) {
    case 4: hipLaunchKernelGGL((k_trace<4, kLeafSphere, false, true>), dim3(blocks), dim3(kTraceBlock), 0, s, a); break;
    case 8: hipLaunchKernelGGL((k_trace<8, kLeafSphere, false, true>), dim3(blocks), dim3(kTraceBlock), 0, s, a); break;
    case 16: hipLaunchKernelGGL((k_trace<16, kLeafSphere, false, true>), dim3(blocks), dim3(kTraceBlock), 0, s, a); break;
    case 32: hipLaunchKernelGGL((k_trace<32, kLeafSphere, false, true>), dim3(blocks), dim3(kTraceBlock), 0, s, a); break;
    default: hipLaunchKernelGGL((k_trace<64, kLeafSphere, false, true>), dim3(blocks), dim3(kTraceBlock), 0, s, a); break;
  }
  GRTX_LAUNCH_CHECK();
  return GRTX_OK;
}

// Centre-out tile order of an image: rings of tiles by distance from the image centre,
// each ring by angle. Rays near the centre of an object-centred view cross the most
// Gaussians; started first, they no longer set the end of the launch, and the tiles in
// flight together stay one compact region. Computed once per (device, tile grid) on the
// host and kept on the device until the process ends.
std::mutex g_order_lock;
std::map<std::tuple<int, int, int>, uint32_t*> g_orders;

grtx_status centre_out_order(int device, int tiles_x, int tiles_y, const uint32_t** out) {
  std::lock_guard<std::mutex> g(g_order_lock);
  auto& slot = g_orders[std::make_tuple(device, tiles_x, tiles_y)];
  if (!slot) {
    const int64_t n = (int64_t)tiles_x * tiles_y;
    std::vector<uint32_t> order(n);
    std::iota(order.begin(), order.end(), 0u);
    std::vector<std::pair<int64_t, double>> key(n);
    const double cx = 0.5 * (tiles_x - 1), cy = 0.5 * (tiles_y - 1);
    for (int64_t t = 0; t < n; ++t) {
      const double dx = (double)(t % tiles_x) - cx, dy = (double)(t / tiles_x) - cy;
      key[t] = {(int64_t)std::floor(std::sqrt(dx * dx + dy * dy)), std::atan2(dy, dx)};
    }
    std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) { return key[a] < key[b]; });
    uint32_t* d = nullptr;
    GRTX_HIP(hipMalloc(reinterpret_cast<void**>(&d), sizeof(uint32_t) * (size_t)n));
    GRTX_HIP(hipMemcpy(d, order.data(), sizeof(uint32_t) * (size_t)n, hipMemcpyHostToDevice));
    slot = d;
  }
  *out = slot;
  return GRTX_OK;
}

grtx_status trace(const Bvh* b, const grtx_rays* r, const grtx_trace_params* p, const grtx_trace_outputs* o,
                  hipStream_t s) {
  TraceScene sc{b->nodes, b->inst, b->tris, b->sh, b->sh_degree, b->roots, nullptr, b->kind, b->n_leaves, b->cut,
                b->n_cut, b->density, b->dbox};
  return launch_trace(sc, r, p, o, s);
}

grtx_status launch_trace_in(const TraceScene& b, const grtx_rays* r, const grtx_trace_params* p,
                            const grtx_trace_outputs* o, hipStream_t s, bool noalloc);

// Scratch of the allocation-free entry point (grtx_trace_noalloc): the work counters in
// the first 256 bytes, then the per-wave checkpoint regions. Each device that runs the
// library holds its own copy until the process ends; calls on one device share it.
constexpr size_t kNoAllocBytes = (size_t)GRTX_NOALLOC_SCRATCH_MB << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

// Device address of `scratch` on each device (the host-side name is only a handle for the
// runtime), looked up once per device with that device current.
constexpr int kMaxDevices = 64;
std::mutex g_noalloc_lock;
void* g_noalloc_ptr[kMaxDevices] = {};

grtx_status noalloc_scratch(int device, void** out) {
  if (device < 0 || device >= kMaxDevices) {
    set_error("grtx_trace_noalloc: device %d beyond the %d supported", device, kMaxDevices);
    return GRTX_ERR_INVALID_ARG;
  }
  std::lock_guard<std::mutex> g(g_noalloc_lock);
  if (!g_noalloc_ptr[device]) {
    void* ptr = nullptr;
    GRTX_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    g_noalloc_ptr[device] = ptr;
  }
  *out = g_noalloc_ptr[device];
  return GRTX_OK;
}

grtx_status launch_trace(const TraceScene& b, const grtx_rays* r, const grtx_trace_params* p,
                         const grtx_trace_outputs* o, hipStream_t s) {
  return launch_trace_in(b, r, p, o, s, false);
}

grtx_status trace_noalloc(const Bvh* b, const grtx_rays* r, const grtx_trace_params* p, const grtx_trace_outputs* o,
                          hipStream_t s) {
  TraceScene sc{b->nodes, b->inst, b->tris, b->sh, b->sh_degree, b->roots, nullptr, b->kind, b->n_leaves, nullptr,
                nullptr};
  return launch_trace_in(sc, r, p, o, s, true);
}

grtx_status launch_trace_in(const TraceScene& b, const grtx_rays* r, const grtx_trace_params* p,
                            const grtx_trace_outputs* o, hipStream_t s, bool noalloc) {
  const int64_t R = r->count;
  if (R == 0) return GRTX_OK;
  if (p->mode == GRTX_MODE_SINGLE_ROUND) {
    if (noalloc) {
      set_error("grtx_trace_noalloc: single-round mode needs scratch for its hit lists");
      return GRTX_ERR_INVALID_ARG;
    }
    if (b.n_leaves > 0) return trace_single_round(b, r, p, o, s);
  }
  if (b.n_leaves == 0) {
    hipLaunchKernelGGL(k_fill_background, dim3((unsigned)((R + 255) / 256)), dim3(256), 0, s, o->rgb, o->depth,
                       o->opacity, o->stats, o->hit_counts, r->t_far, r->transmittance, R, p->bg[0], p->bg[1],
                       p->bg[2]);
    GRTX_LAUNCH_CHECK();
    return GRTX_OK;
  }
  int device = 0;
  GRTX_HIP(hipGetDevice(&device));
  hipDeviceProp_t prop;
  static thread_local int cached_dev = -1;
  static thread_local int cached_cus = 0;
  if (cached_dev != device) {
    GRTX_HIP(hipGetDeviceProperties(&prop, device));
    cached_dev = device;
    cached_cus = prop.multiProcessorCount;
  }
  const int K = p->k <= 4 ? 4 : p->k <= 8 ? 8 : p->k <= 16 ? 16 : p->k <= 32 ? 32 : 64;
  const int leaf = b.kind == GRTX_BVH_PROXY20 ? kLeafTri : b.kind == GRTX_BVH_ICO_INSTANCE ? kLeafIco : kLeafSphere;
  const bool stats = o->stats != nullptr;
  int bpc = leaf == kLeafTri ? blocks_per_cu_k<kLeafTri>(K, stats)
          : leaf == kLeafIco ? blocks_per_cu_k<kLeafIco>(K, stats) : blocks_per_cu_k<kLeafSphere>(K, stats);
  int blocks = cached_cus * bpc;
  // never more waves than rays need
  int64_t need_blocks = (R + kTraceBlock - 1) / kTraceBlock;
  if (blocks > need_blocks) blocks = (int)std::max<int64_t>(1, need_blocks);

  // restart rounds keep no lists: their lanes hold only the stack spill and the park
  const bool lists = p->mode == GRTX_MODE_CHECKPOINT;
  const int cap_d =
      lists ? stage_round(p->defer_capacity > 0 ? p->defer_capacity : default_defer_cap(b.n_leaves, noalloc)) : 0;
  const int cap_e =
      lists ? stage_round(p->evict_capacity > 0 ? p->evict_capacity : default_evict_cap(b.n_leaves, noalloc)) : 0;
  const int64_t rows = kSpillRows + 2 * (int64_t)cap_d + 2 * (int64_t)cap_e + K;
  const size_t need = (size_t)blocks * kWaves * rows * 64 * sizeof(uint2) + 256;

  Pool fixed;
  Pool* pool = nullptr;
  if (noalloc) {
    // the static scratch: as many workgroups as fit in it, none beyond it
    const size_t per_block = (size_t)kWaves * rows * 64 * sizeof(uint2);
    const int64_t fit = (int64_t)((kNoAllocBytes - 256) / per_block);
    if (fit < 1) {
      set_error("grtx_trace_noalloc: one workgroup's checkpoint lists (%zu bytes at k-buffer %d, capacities %d/%d) "
                "exceed the %zu-byte scratch; lower the list capacities",
                per_block, K, cap_d, cap_e, kNoAllocBytes - 256);
      return GRTX_ERR_CAPACITY;
    }
    if (blocks > fit) blocks = (int)fit;
    GRTX_TRY(noalloc_scratch(device, &fixed.ptr));
    fixed.bytes = kNoAllocBytes;
    fixed.counter = reinterpret_cast<unsigned int*>(fixed.ptr);
    pool = &fixed;
  } else {
    std::lock_guard<std::mutex> g(g_pool_lock);
    pool = &g_pools[{device, s}];
    if (pool->bytes < need) {
      if (pool->ptr) GRTX_HIP(hipFreeAsync(pool->ptr, s));
      pool->ptr = nullptr;
      pool->bytes = 0;
      // some room to grow into, at most 1 GiB of it
      size_t want = need + std::min<size_t>(need / 4, (size_t)1 << 30);
      GRTX_HIP(hipMallocAsync(&pool->ptr, want, s));
      pool->bytes = want;
      pool->counter = reinterpret_cast<unsigned int*>(pool->ptr);
    }
  }

  TraceArgs a{};
  a.nodes = b.nodes;
  a.inst = b.inst;
  a.tris = b.tris;
  a.sh = b.sh;
  a.roots = b.roots;
  a.ray_scene = b.ray_scene;
  a.sh_degree = b.sh_degree;
  a.ray_o = r->origins;
  a.ray_d = r->dirs;
  a.ray_tfar = r->t_far;
  a.ray_trans = r->transmittance;
  a.ray_next_o = r->next_origins;
  a.ray_next_d = r->next_dirs;
  a.ray_path = r->path;
  a.ray_kind = r->kind;
  a.n_rays = R;
  a.t_near = r->t_near;
  // rays 0..image_begin-1 form no image and are taken first; the image's rays follow
  int64_t image_h = 0;
  a.n_work = trace_work_items(r, &a.n_free, &image_h);
  if (a.n_work > kMaxTraceWork) {  // (the ABI layer refuses such launches first)
    set_error("trace: %lld work items exceed one launch's 2^31-1", (long long)a.n_work);
    return GRTX_ERR_INVALID_ARG;
  }
  a.image_h = (int)image_h;
  a.image_w = image_h > 0 ? r->image_width : 0;
  a.tiles_x = (a.image_w + 7) / 8;
  a.k = p->k;
  a.T_min = p->T_min;
  a.mode = p->mode;
  a.bg0 = p->bg[0];
  a.bg1 = p->bg[1];
  a.bg2 = p->bg[2];
  a.rgb = o->rgb;
  a.depth = o->depth;
  a.opac = o->opacity;
  a.stats = o->stats;
  a.hit_ids = o->hit_ids;
  a.hit_counts = o->hit_counts;
  a.hit_cap = o->hit_ids ? o->hit_capacity : 0;
  a.counter = pool->counter;
  a.pool = reinterpret_cast<uint2*>(reinterpret_cast<char*>(pool->ptr) + 256);
  a.rows_per_wave = rows;
  a.cap_d = cap_d;
  a.cap_e = cap_e;
  a.refill = b.n_leaves > kLargeScene ? kRefillLarge : kRefillSmall;
  a.chunk_len = ((a.n_work + 64 * kChunks - 1) / (64 * kChunks)) * 64;
  uint32_t* order_buf = nullptr;
  // (the allocation-free path keeps the tiles in row-major order: no scratch, same results)
  std::unique_ptr<Scratch> order_scratch;
  if (!noalloc) order_scratch.reset(new Scratch(s));
  const int64_t F = a.n_free;
  if (a.image_w > 0 && !noalloc) {
    // Tiles heaviest first, so that the longest rays do not start last: by estimated cost
    // where the structure carries a subtree cut, centre-out within equal estimates.
    const int64_t nt = (a.n_work - F) / 64;
    const uint32_t* base = nullptr;
    GRTX_TRY(centre_out_order(device, a.tiles_x, (int)(nt / a.tiles_x), &base));
    // scratch: estimate keys (8 B) and order (4 B) per tile, then three more words per tile
    // for the continuation partition
    GRTX_TRY(order_scratch->get(&order_buf, 6 * (size_t)nt));
    if (b.cut) {
      uint64_t* keys = reinterpret_cast<uint64_t*>(order_buf);
      uint32_t* est_order = order_buf + 2 * nt;
      hipLaunchKernelGGL(k_tile_estimate, dim3((unsigned)((nt + kEstTiles - 1) / kEstTiles)), dim3(256), 0, s, b.cut,
                         b.n_cut, r->origins + 3 * F, r->dirs + 3 * F, a.image_w, a.image_h, a.tiles_x, nt, base,
                         keys, est_order);
      GRTX_TRY(sort_by_key(keys, est_order, nt, 8, s));
      base = est_order;
    }
    a.tile_order = base;
    if (r->kind) {
      // rays that go on past an object run longest: their tiles first
      uint32_t* flag = order_buf + 3 * nt;
      uint32_t* pos = flag + nt;
      uint32_t* order = pos + nt;
      const unsigned g = (unsigned)((nt + 255) / 256);
      hipLaunchKernelGGL(k_tile_heavy, dim3(g), dim3(256), 0, s, r->kind + F, base, a.image_w, a.image_h, a.tiles_x,
                         nt, flag);
      GRTX_TRY(exclusive_scan_u32(flag, pos, nt, s));
      hipLaunchKernelGGL(k_tile_order, dim3(g), dim3(256), 0, s, base, flag, pos, nt, order);
      a.tile_order = order;
    }
  }
  if (!noalloc && b.density && F >= kOrderMinRays) {
    // heaviest rays first (see k_ray_bucket)
    uint32_t* buf = nullptr;
    GRTX_TRY(order_scratch->get(&buf, 4 * (size_t)F + kOrderBuckets + 1));
    uint32_t *bucket = buf, *flag = buf + F, *pos = buf + 2 * F, *order = buf + 3 * F;
    uint32_t *hist = buf + 4 * F, *thr = hist + kOrderBuckets;
    const unsigned g = (unsigned)((F + 255) / 256);
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(256), 0, s, hist, kOrderBuckets);
    hipLaunchKernelGGL(k_ray_bucket, dim3(g), dim3(256), 0, s, r->origins, F, b.dbox, b.density, bucket, hist);
    hipLaunchKernelGGL(k_ray_split, dim3(1), dim3(64), 0, s, hist, F, thr);
    hipLaunchKernelGGL(k_ray_flags, dim3(g), dim3(256), 0, s, bucket, F, thr, flag);
    GRTX_TRY(exclusive_scan_u32(flag, pos, F, s));
    hipLaunchKernelGGL(k_ray_order, dim3(g), dim3(256), 0, s, flag, pos, F, order);
    GRTX_LAUNCH_CHECK();
    a.ray_order = order;
  }
  hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(64), 0, s, pool->counter);
  return leaf == kLeafTri ? launch_k<kLeafTri>(K, a, blocks, s)
       : leaf == kLeafIco ? launch_k<kLeafIco>(K, a, blocks, s) : launch_k<kLeafSphere>(K, a, blocks, s);
}

}  // namespace grtx
