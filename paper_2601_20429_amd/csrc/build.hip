// LBVH construction over Gaussians on gfx950 (Sec. IV-A: one leaf per Gaussian holding
// its world->unit-sphere transform; the baseline's 20-triangle proxy mesh per Gaussian).
//
// Pipeline, all on one stream, no host synchronisation:
//   bounds of the centroids (two-stage min/max, exact)
//   63-bit Morton codes (binary32 quantisation with fp contraction off, so the codes are
//     an exact integer function of the inputs)
//   stable LSD radix sort of (code, index), 8 passes of 8 bits
//   radix tree over the sorted (code, position) keys (Karras 2012, one thread per node)
//   leaf records and leaf boxes in sorted order
//   bottom-up refit with per-node arrival counters (exact min/max)
//   treelet restructuring by surface-area cost (5-leaf treelets, one workgroup per subtree
//     of at most 256 leaves; beyond a million leaves three passes over the subtrees and
//     one over the nodes above them), unless the plain radix tree is asked for
//   collapse to four-wide quantised node records, and a subtree cut kept for the trace's
//     per-tile cost estimates
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <cmath>
#include <type_traits>

#include "camera.h"
#include "grtx_internal.h"

namespace grtx {
namespace {

constexpr int kBlock = 256;

// ------------------------------------------------------------------ centroid bounds

__global__ void __launch_bounds__(kBlock) k_bounds_partial(const float* __restrict__ pts, int64_t n,
                                                           float* __restrict__ partial) {
  float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
    for (int a = 0; a < 3; ++a) {
      float v = pts[3 * i + a];
      lo[a] = fminf(lo[a], v);
      hi[a] = fmaxf(hi[a], v);
    }
  }
  __shared__ float s[6][kBlock];
  for (int a = 0; a < 3; ++a) {
    s[a][threadIdx.x] = lo[a];
    s[3 + a][threadIdx.x] = hi[a];
  }
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w)
      for (int a = 0; a < 3; ++a) {
        s[a][threadIdx.x] = fminf(s[a][threadIdx.x], s[a][threadIdx.x + w]);
        s[3 + a][threadIdx.x] = fmaxf(s[3 + a][threadIdx.x], s[3 + a][threadIdx.x + w]);
      }
    __syncthreads();
  }
  if (threadIdx.x < 6) partial[blockIdx.x * 6 + threadIdx.x] = s[threadIdx.x][0];
}

__global__ void __launch_bounds__(kBlock) k_bounds_final(const float* __restrict__ partial, int nparts,
                                                         float* __restrict__ out) {
  __shared__ float s[6][kBlock];
  float v[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
  for (int i = threadIdx.x; i < nparts; i += kBlock)
    for (int a = 0; a < 3; ++a) {
      v[a] = fminf(v[a], partial[i * 6 + a]);
      v[3 + a] = fmaxf(v[3 + a], partial[i * 6 + 3 + a]);
    }
  for (int a = 0; a < 6; ++a) s[a][threadIdx.x] = v[a];
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w)
      for (int a = 0; a < 3; ++a) {
        s[a][threadIdx.x] = fminf(s[a][threadIdx.x], s[a][threadIdx.x + w]);
        s[3 + a][threadIdx.x] = fmaxf(s[3 + a][threadIdx.x], s[3 + a][threadIdx.x + w]);
      }
    __syncthreads();
  }
  if (threadIdx.x < 6) out[threadIdx.x] = s[threadIdx.x][0];
}

// ------------------------------------------------------------------ Morton codes

__device__ __forceinline__ uint64_t spread3(uint32_t v) {
  uint64_t x = v & 0x1FFFFFu;
  x = (x | (x << 32)) & 0x1F00000000FFFFull;
  x = (x | (x << 16)) & 0x1F0000FF0000FFull;
  x = (x | (x << 8)) & 0x100F00F00F00F00Full;
  x = (x | (x << 4)) & 0x10C30C30C30C30C3ull;
  x = (x | (x << 2)) & 0x1249249249249249ull;
  return x;
}

__device__ __forceinline__ uint32_t quantise(float v, float lo, float scale) {
#pragma clang fp contract(off)
  float rel = v - lo;
  float pos = rel * scale;
  float fl = floorf(pos);
  return fl <= 0.f ? 0u : (fl >= 2097151.f ? 2097151u : (uint32_t)fl);
}

__global__ void __launch_bounds__(kBlock) k_morton(const float* __restrict__ pts, int64_t n,
                                                   const float* __restrict__ bounds, uint64_t* __restrict__ codes,
                                                   uint32_t* __restrict__ idx) {
#pragma clang fp contract(off)
  int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x;
  if (i >= n) return;
  uint32_t q[3];
  for (int a = 0; a < 3; ++a) {
    float lo = bounds[a], hi = bounds[3 + a];
    float ext = hi - lo;
    float scale = ext > 0.f ? 2097152.f / ext : 0.f;  // correctly rounded division
    q[a] = quantise(pts[3 * i + a], lo, scale);
  }
  codes[i] = (spread3(q[0]) << 2) | (spread3(q[1]) << 1) | spread3(q[2]);
  idx[i] = (uint32_t)i;
}

// ------------------------------------------------------------------ radix sort (stable LSD)

// Keys per thread: 16 for large sorts; 4 up to kRadixSmall keys, so that a sort of a few
// hundred thousand keys still spreads over ~100 workgroups instead of ~25.
constexpr int kRadixItems = 16;
constexpr int kRadixItemsSmall = 4;
constexpr int64_t kRadixSmall = (int64_t)256 * kBlock * kRadixItemsSmall;
// Up to this many workgroups, each scatter workgroup derives its own offsets from the
// histogram table (a digit's counts over all workgroups), so no scan launch is needed.
constexpr int kRadixFusedBlocks = 256;

// `n_dev` (may be null) holds the number of keys on the device when the host knows only a
// bound `n` (the grid is sized for the bound; workgroups past the count see no keys).
__global__ void __launch_bounds__(kBlock) k_radix_hist(const uint64_t* __restrict__ keys, int64_t n, int shift,
                                                       int items, uint32_t* __restrict__ hist, int nblocks,
                                                       bool fused, const uint32_t* __restrict__ n_dev) {
  if (n_dev) n = min(n, (int64_t)*n_dev);
  __shared__ uint32_t s_cnt[256];
  s_cnt[threadIdx.x] = 0;
  __syncthreads();
  int64_t base = (int64_t)blockIdx.x * kBlock * items;
  for (int r = 0; r < items; ++r) {
    int64_t i = base + r * kBlock + threadIdx.x;
    if (i < n) atomicAdd(&s_cnt[(keys[i] >> shift) & 255u], 1u);
  }
  __syncthreads();
  // digit-major ([digit][workgroup]) for the scan; workgroup-major rows for the fused scatter
  hist[fused ? (size_t)blockIdx.x * 256 + threadIdx.x : (size_t)threadIdx.x * nblocks + blockIdx.x] = s_cnt[threadIdx.x];
}

// Exclusive scan of `n` uint32 in chunks of kScanChunk.
constexpr int kScanItems = 16;
constexpr int kScanChunk = kBlock * kScanItems;

__device__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* s_tmp, uint32_t* total) {
  // Hillis-Steele over kBlock values in LDS.
  s_tmp[threadIdx.x] = v;
  __syncthreads();
  for (int off = 1; off < kBlock; off <<= 1) {
    uint32_t add = threadIdx.x >= off ? s_tmp[threadIdx.x - off] : 0u;
    __syncthreads();
    s_tmp[threadIdx.x] += add;
    __syncthreads();
  }
  uint32_t incl = s_tmp[threadIdx.x];
  *total = s_tmp[kBlock - 1];
  __syncthreads();
  return incl - v;
}

__global__ void __launch_bounds__(kBlock) k_scan_reduce(const uint32_t* __restrict__ in, int64_t n,
                                                        uint32_t* __restrict__ partial) {
  __shared__ uint32_t s[kBlock];
  int64_t base = (int64_t)blockIdx.x * kScanChunk + (int64_t)threadIdx.x * kScanItems;
  uint32_t acc = 0;
  for (int j = 0; j < kScanItems; ++j)
    if (base + j < n) acc += in[base + j];
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = s[0];
}

// One block: exclusive scan of up to kScanChunk partials in place.
__global__ void __launch_bounds__(kBlock) k_scan_partials(uint32_t* __restrict__ partial, int n) {
  __shared__ uint32_t s[kBlock];
  uint32_t v[kScanItems];
  uint32_t acc = 0;
  for (int j = 0; j < kScanItems; ++j) {
    int i = threadIdx.x * kScanItems + j;
    v[j] = i < n ? partial[i] : 0u;
    acc += v[j];
  }
  uint32_t tot;
  uint32_t run = block_exclusive_scan(acc, s, &tot);
  for (int j = 0; j < kScanItems; ++j) {
    int i = threadIdx.x * kScanItems + j;
    if (i < n) partial[i] = run;
    run += v[j];
  }
}

__global__ void __launch_bounds__(kBlock) k_scan_down(const uint32_t* __restrict__ in, int64_t n,
                                                      const uint32_t* __restrict__ partial,
                                                      uint32_t* __restrict__ out) {
  __shared__ uint32_t s[kBlock];
  int64_t base = (int64_t)blockIdx.x * kScanChunk + (int64_t)threadIdx.x * kScanItems;
  uint32_t v[kScanItems];
  uint32_t acc = 0;
  for (int j = 0; j < kScanItems; ++j) {
    v[j] = base + j < n ? in[base + j] : 0u;
    acc += v[j];
  }
  uint32_t tot;
  uint32_t run = block_exclusive_scan(acc, s, &tot) + (partial ? partial[blockIdx.x] : 0u);
  for (int j = 0; j < kScanItems; ++j) {
    if (base + j < n) out[base + j] = run;
    run += v[j];
  }
}

// Exclusive scan of up to a few chunks in one workgroup, chunk after chunk with a running
// carry: one launch where the three-kernel scan would spend two more on a tiny partial pass.
constexpr int kScanLoopChunks = 8;
__global__ void __launch_bounds__(kBlock) k_scan_loop(const uint32_t* __restrict__ in, int64_t n,
                                                      uint32_t* __restrict__ out) {
  __shared__ uint32_t s[kBlock];
  uint32_t carry = 0;
  for (int64_t c0 = 0; c0 < n; c0 += kScanChunk) {
    const int64_t base = c0 + (int64_t)threadIdx.x * kScanItems;
    uint32_t v[kScanItems];
    uint32_t acc = 0;
    for (int j = 0; j < kScanItems; ++j) {
      v[j] = base + j < n ? in[base + j] : 0u;
      acc += v[j];
    }
    uint32_t tot;
    uint32_t run = block_exclusive_scan(acc, s, &tot) + carry;
    for (int j = 0; j < kScanItems; ++j) {
      if (base + j < n) out[base + j] = run;
      run += v[j];
    }
    carry += tot;
    __syncthreads();
  }
}

// `offsets` is either the scanned histogram table ([digit][workgroup], exclusive), or, with
// `fused`, the raw counts in workgroup-major rows: then thread d adds digit d's counts of the
// workgroups before this one, and a block scan over the 256 digit totals gives the digit's
// start.
__global__ void __launch_bounds__(kBlock) k_radix_scatter(const uint64_t* __restrict__ keys_in,
                                                          const uint32_t* __restrict__ vals_in, int64_t n, int shift,
                                                          int items, const uint32_t* __restrict__ offsets,
                                                          int nblocks, bool fused, uint64_t* __restrict__ keys_out,
                                                          uint32_t* __restrict__ vals_out,
                                                          const uint32_t* __restrict__ n_dev) {
  if (n_dev) n = min(n, (int64_t)*n_dev);
  if ((int64_t)blockIdx.x * kBlock * items >= n) return;  // the whole workgroup is past the keys
  __shared__ uint32_t s_off[256];
  __shared__ uint32_t s_wcnt[kBlock / 64][256];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const uint64_t lt_mask = lane ? (~0ull >> (64 - lane)) : 0ull;
  if (fused) {
    uint32_t before = 0, total = 0;
#pragma unroll 8
    for (int b = 0; b < nblocks; ++b) {
      const uint32_t c = offsets[(size_t)b * 256 + threadIdx.x];
      total += c;
      before += b < (int)blockIdx.x ? c : 0u;
    }
    uint32_t all;
    const uint32_t start = block_exclusive_scan(total, &s_wcnt[0][0], &all);
    s_off[threadIdx.x] = start + before;
  } else {
    s_off[threadIdx.x] = offsets[(size_t)threadIdx.x * nblocks + blockIdx.x];
  }
  int64_t base = (int64_t)blockIdx.x * kBlock * items;
  for (int r = 0; r < items; ++r) {
    for (int w = 0; w < kBlock / 64; ++w) s_wcnt[w][threadIdx.x] = 0u;
    __syncthreads();
    int64_t i = base + r * kBlock + threadIdx.x;
    bool valid = i < n;
    uint64_t key = valid ? keys_in[i] : 0ull;
    uint32_t val = valid ? vals_in[i] : 0u;
    uint32_t digit = (uint32_t)(key >> shift) & 255u;
    uint64_t peers = __ballot(valid);
    for (int b = 0; b < 8; ++b) {
      bool bit = (digit >> b) & 1u;
      uint64_t m = __ballot(valid && bit);
      peers &= bit ? m : ~m;
    }
    uint32_t rank = __popcll(peers & lt_mask);
    if (valid && rank == 0) s_wcnt[wave][digit] = (uint32_t)__popcll(peers);
    __syncthreads();
    if (valid) {
      uint32_t pos = s_off[digit] + rank;
      for (int w = 0; w < wave; ++w) pos += s_wcnt[w][digit];
      keys_out[pos] = key;
      vals_out[pos] = val;
    }
    __syncthreads();
    uint32_t add = 0;
    for (int w = 0; w < kBlock / 64; ++w) add += s_wcnt[w][threadIdx.x];
    s_off[threadIdx.x] += add;
    __syncthreads();
  }
}

// ------------------------------------------------------------------ radix tree (Karras)

__device__ __forceinline__ int prefix_len(const uint64_t* __restrict__ codes, int64_t n, int64_t i, int64_t j) {
  if (j < 0 || j >= n) return -1;
  uint64_t a = codes[i], b = codes[j];
  if (a != b) return __clzll(a ^ b);
  return 64 + __clz((uint32_t)i ^ (uint32_t)j);
}

__global__ void __launch_bounds__(kBlock) k_karras(const uint64_t* __restrict__ codes, int64_t n,
                                                   uint32_t* __restrict__ child, uint32_t* __restrict__ parent,
                                                   uint2* __restrict__ range, uint32_t* __restrict__ count,
                                                   uint32_t* __restrict__ arrivals) {
  int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x;
  if (i >= n - 1) return;
  // the refit's arrival counters (n - 1 nodes, then the ready-list length) start at zero
  arrivals[i] = 0u;
  if (i == 0) arrivals[n - 1] = 0u;
  int d = prefix_len(codes, n, i, i + 1) - prefix_len(codes, n, i, i - 1) > 0 ? 1 : -1;
  int dmin = prefix_len(codes, n, i, i - d);
  int64_t lmax = 2;
  while (prefix_len(codes, n, i, i + lmax * d) > dmin) lmax <<= 1;
  int64_t l = 0;
  for (int64_t t = lmax >> 1; t >= 1; t >>= 1)
    if (prefix_len(codes, n, i, i + (l + t) * d) > dmin) l += t;
  int64_t j = i + l * d;
  int dnode = prefix_len(codes, n, i, j);
  int64_t s = 0;
  int64_t t = l;
  do {
    t = (t + 1) >> 1;
    if (prefix_len(codes, n, i, i + (s + t) * d) > dnode) s += t;
  } while (t > 1);
  int64_t gamma = i + s * d + (d < 0 ? -1 : 0);
  int64_t lo = i < j ? i : j, hi = i < j ? j : i;
  uint32_t left, right;
  if (lo == gamma) {
    left = kLeafFlag | (uint32_t)gamma;
    parent[(n - 1) + gamma] = (uint32_t)i;
  } else {
    left = (uint32_t)gamma;
    parent[gamma] = (uint32_t)i;
  }
  if (hi == gamma + 1) {
    right = kLeafFlag | (uint32_t)(gamma + 1);
    parent[(n - 1) + gamma + 1] = (uint32_t)i;
  } else {
    right = (uint32_t)(gamma + 1);
    parent[gamma + 1] = (uint32_t)i;
  }
  child[2 * i] = left;
  child[2 * i + 1] = right;
  range[i] = make_uint2((uint32_t)lo, (uint32_t)hi);
  count[i] = (uint32_t)(hi - lo + 1);  // leaves below the node
  if (i == 0) parent[0] = kNoParent;
}

// ------------------------------------------------------------------ leaves

struct GaussIn {
  const float* means;
  const float* scales;
  const float* quats;
  const float* opac;
};

__device__ __forceinline__ void quat_rot(const float* q4, float R[3][3]) {
  float w = q4[0], x = q4[1], y = q4[2], z = q4[3];
  float inv = rsqrtf(w * w + x * x + y * y + z * z);
  w *= inv; x *= inv; y *= inv; z *= inv;
  R[0][0] = 1.f - 2.f * (y * y + z * z); R[0][1] = 2.f * (x * y - w * z);       R[0][2] = 2.f * (x * z + w * y);
  R[1][0] = 2.f * (x * y + w * z);       R[1][1] = 1.f - 2.f * (x * x + z * z); R[1][2] = 2.f * (y * z - w * x);
  R[2][0] = 2.f * (x * z - w * y);       R[2][1] = 2.f * (y * z + w * x);       R[2][2] = 1.f - 2.f * (x * x + y * y);
}

// Relative padding of the leaf boxes: the box must contain the bounding ellipsoid as the
// leaf test sees it in binary32 (rounding of R, rho and of the transformed ray).
constexpr float kBoxPad = 1.0f + 1.0f / 128.0f;

struct GaussGeom {
  float R[3][3];
  float s[3];
  float rho;
  float o;
  bool active;
};

__device__ __forceinline__ GaussGeom gauss_geom(const GaussIn& g, int64_t i, float alpha_min) {
  GaussGeom G;
  quat_rot(g.quats + 4 * i, G.R);
  for (int a = 0; a < 3; ++a) G.s[a] = g.scales[3 * i + a];
  G.o = g.opac[i];
  G.active = G.o > alpha_min && G.s[0] > 0.f && G.s[1] > 0.f && G.s[2] > 0.f;
  G.rho = G.active ? sqrtf(2.f * logf(G.o / alpha_min)) : 0.f;
  return G;
}

// Box of the bounding ellipsoid scaled by `scale` about mu (1 for the sphere leaf; the
// icosahedron's circumradius over its inradius for the icosahedron instance leaf, whose
// mesh lies inside that scaled ellipsoid).
__device__ __forceinline__ void gauss_box(const GaussIn& g, int64_t i, const GaussGeom& G, float scale, float lo[3],
                                          float hi[3]) {
  for (int j = 0; j < 3; ++j) {
    float m = g.means[3 * i + j];
    float h = 0.f;
    if (G.active) {
      float v = 0.f;
      for (int k = 0; k < 3; ++k) v += G.R[j][k] * G.R[j][k] * G.s[k] * G.s[k];
      h = G.rho * sqrtf(v) * (kBoxPad * scale);
    }
    lo[j] = m - h;
    hi[j] = m + h;
  }
}

// Sphere leaves: instance record and box for sorted position p.
__global__ void __launch_bounds__(kBlock) k_sphere_leaves(GaussIn g, const uint32_t* __restrict__ perm, int64_t n,
                                                          float alpha_min, float box_scale, float4* __restrict__ inst,
                                                          float* __restrict__ boxes) {
  int64_t p = blockIdx.x * (int64_t)kBlock + threadIdx.x;
  if (p >= n) return;
  uint32_t i = perm[p];
  GaussGeom G = gauss_geom(g, i, alpha_min);
  float4 r[4];
  float* rr = reinterpret_cast<float*>(r);
  for (int a = 0; a < 3; ++a) {
    // row a of A = column a of R / (rho s_a)
    float sc = G.active ? 1.f / (G.rho * G.s[a]) : 0.f;
    rr[4 * a + 0] = G.R[0][a] * sc;
    rr[4 * a + 1] = G.R[1][a] * sc;
    rr[4 * a + 2] = G.R[2][a] * sc;
    rr[4 * a + 3] = g.means[3 * i + a];
  }
  rr[12] = G.o;
  rr[13] = G.active ? log2f(G.o / alpha_min) : 0.f;
  rr[14] = __uint_as_float(i);
  rr[15] = __uint_as_float(G.active ? 1u : 0u);
  for (int q = 0; q < 4; ++q) inst[4 * p + q] = r[q];
  float lo[3], hi[3];
  gauss_box(g, i, G, box_scale, lo, hi);
  float* bx = boxes + ((n - 1) + p) * 6;
  for (int a = 0; a < 3; ++a) {
    bx[a] = lo[a];
    bx[3 + a] = hi[a];
  }
}

// ------------------------------------------------------------------ proxy mesh (baseline)

// Regular icosahedron of inradius 1 (its faces touch the unit sphere from outside):
// vertices and outward-wound faces, derived on the host from the definition.
struct Ico {
  float v[12][3];
  unsigned char f[20][3];
};

// Instance record in Gaussian order (used by the proxy BVH's blending).
__device__ __forceinline__ void write_instance(const GaussIn& g, uint32_t i, const GaussGeom& G, float alpha_min,
                                               float4* __restrict__ dst) {
  float r[16];
  for (int a = 0; a < 3; ++a) {
    float sc = G.active ? 1.f / (G.rho * G.s[a]) : 0.f;
    r[4 * a + 0] = G.R[0][a] * sc;
    r[4 * a + 1] = G.R[1][a] * sc;
    r[4 * a + 2] = G.R[2][a] * sc;
    r[4 * a + 3] = g.means[3 * i + a];
  }
  r[12] = G.o;
  r[13] = G.active ? log2f(G.o / alpha_min) : 0.f;
  r[14] = __uint_as_float(i);
  r[15] = __uint_as_float(G.active ? 1u : 0u);
  for (int q = 0; q < 4; ++q) dst[q] = make_float4(r[4 * q], r[4 * q + 1], r[4 * q + 2], r[4 * q + 3]);
}

// Relative and absolute padding of a triangle's box: the binary32 hit distance of a ray
// crossing the triangle must stay inside the box's slab interval.
constexpr float kTriPadRel = 1.0f / 1024.0f;
constexpr float kTriPadAbs = 1.0f / 131072.0f;

// One thread per Gaussian: instance record (Gaussian order), 20 world triangles
// mu + R diag(rho s) v_ico with their boxes and box centres (triangle order 20 g + face).
__global__ void __launch_bounds__(kBlock) k_proxy_setup(GaussIn g, int64_t n, float alpha_min, Ico ico,
                                                        float4* __restrict__ inst, float4* __restrict__ tri,
                                                        float* __restrict__ tbox, float* __restrict__ cent) {
  int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x;
  if (i >= n) return;
  GaussGeom G = gauss_geom(g, i, alpha_min);
  write_instance(g, (uint32_t)i, G, alpha_min, inst + 4 * i);
  float w[12][3];
  for (int v = 0; v < 12; ++v)
    for (int a = 0; a < 3; ++a) {
      float acc = 0.f;
      for (int k = 0; k < 3; ++k) acc += G.R[a][k] * (G.rho * G.s[k] * ico.v[v][k]);
      w[v][a] = g.means[3 * i + a] + acc;  // inactive: rho = 0, a point at mu
    }
  for (int f = 0; f < 20; ++f) {
    const int64_t t = 20 * i + f;
    const float* A = w[ico.f[f][0]];
    const float* B = w[ico.f[f][1]];
    const float* C = w[ico.f[f][2]];
    tri[3 * t + 0] = make_float4(A[0], A[1], A[2], __uint_as_float((uint32_t)i));
    tri[3 * t + 1] = make_float4(B[0], B[1], B[2], 0.f);
    tri[3 * t + 2] = make_float4(C[0], C[1], C[2], 0.f);
    for (int a = 0; a < 3; ++a) {
      float lo = fminf(A[a], fminf(B[a], C[a]));
      float hi = fmaxf(A[a], fmaxf(B[a], C[a]));
      float pad = (hi - lo) * kTriPadRel + (fabsf(lo) + fabsf(hi)) * kTriPadAbs;
      tbox[6 * t + a] = lo - pad;
      tbox[6 * t + 3 + a] = hi + pad;
      cent[3 * t + a] = 0.5f * (lo + hi);
    }
  }
}

// Gather triangle records and boxes into sorted-leaf order.
__global__ void __launch_bounds__(kBlock) k_proxy_leaves(const uint32_t* __restrict__ perm, int64_t m,
                                                         const float4* __restrict__ tri_in,
                                                         const float* __restrict__ box_in,
                                                         float4* __restrict__ tri_out, float* __restrict__ boxes) {
  int64_t p = blockIdx.x * (int64_t)kBlock + threadIdx.x;
  if (p >= m) return;
  uint32_t t = perm[p];
  for (int q = 0; q < 3; ++q) tri_out[3 * p + q] = tri_in[3 * (int64_t)t + q];
  float* bx = boxes + ((m - 1) + p) * 6;
  for (int a = 0; a < 6; ++a) bx[a] = box_in[6 * (int64_t)t + a];
}

// ------------------------------------------------------------------ refit

// Refit in two phases. An internal node of the radix tree covers a contiguous range of
// sorted leaves. "Small" nodes (at most `small` leaves) take their children's boxes
// straight from the leaf boxes of the two sub-ranges: no ordering between threads is
// needed. The few "top" nodes above them are refitted bottom-up by one workgroup, which
// orders its threads with workgroup-scope atomics; a grid-wide bottom-up pass would need a
// device-scope fence per node, which on a multi-XCD part writes back the whole L2.
// The limit grows with the tree: 128 leaves up to a million leaves; 1024 above, where the
// top phase would otherwise walk tens of thousands of nodes in one workgroup (at 3M leaves
// the two phases took 0.24 + 0.71 ms with 128, 0.58 + 0.10 ms with 1024).
inline int64_t refit_small_limit(int64_t m) { return m > ((int64_t)1 << 20) ? 1024 : 128; }
constexpr int kTopBlock = 1024;

__device__ __forceinline__ bool is_small(uint32_t c, const uint2* __restrict__ range, int64_t small) {
  if (c & kLeafFlag) return true;
  uint2 r = range[c];
  return (int64_t)r.y - r.x + 1 <= small;
}

__device__ __forceinline__ void range_box(const float* __restrict__ leaf_boxes, uint32_t lo, uint32_t hi, float b[6]) {
  b[0] = b[1] = b[2] = INFINITY;
  b[3] = b[4] = b[5] = -INFINITY;
  uint32_t q = lo;
  for (; q + 3 <= hi; q += 4) {
    float v[4][6];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int a = 0; a < 6; ++a) v[u][a] = leaf_boxes[(int64_t)(q + u) * 6 + a];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        b[a] = fminf(b[a], v[u][a]);
        b[3 + a] = fmaxf(b[3 + a], v[u][3 + a]);
      }
  }
  for (; q <= hi; ++q)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      b[a] = fminf(b[a], leaf_boxes[(int64_t)q * 6 + a]);
      b[3 + a] = fmaxf(b[3 + a], leaf_boxes[(int64_t)q * 6 + 3 + a]);
    }
}

__device__ __forceinline__ void write_box(float* __restrict__ boxes, uint32_t node, const float (&b0)[6],
                                          const float (&b1)[6]) {
  float* nb = boxes + (int64_t)node * 6;
  for (int a = 0; a < 3; ++a) {
    nb[a] = fminf(b0[a], b1[a]);
    nb[3 + a] = fmaxf(b0[3 + a], b1[3 + a]);
  }
}

// Phase 1: every small internal node; also lists the top nodes whose children are both
// small (the top phase starts there).
__global__ void __launch_bounds__(kBlock) k_refit_small(int64_t n, const uint32_t* __restrict__ child,
                                                        const uint2* __restrict__ range, float* __restrict__ boxes,
                                                        uint32_t* __restrict__ ready,
                                                        uint32_t* __restrict__ n_ready, int64_t small) {
  const int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x;
  bool top_ready = false;
  if (i < n - 1) {
    const uint2 r = range[i];
    const uint32_t c0 = child[2 * i], c1 = child[2 * i + 1];
    if ((int64_t)r.y - r.x + 1 <= small) {
      const uint32_t split = c0 & ~kLeafFlag;  // last leaf of the left child
      float b0[6], b1[6];
      const float* leaf_boxes = boxes + (n - 1) * 6;
      range_box(leaf_boxes, r.x, split, b0);
      range_box(leaf_boxes, split + 1, r.y, b1);
      write_box(boxes, (uint32_t)i, b0, b1);
    } else {
      top_ready = is_small(c0, range, small) && is_small(c1, range, small);
    }
  }
  const uint64_t m = __ballot(top_ready);
  if (m) {
    const int lane = threadIdx.x & 63;
    const int leader = __ffsll((unsigned long long)m) - 1;
    uint32_t base = 0;
    if (lane == leader) base = atomicAdd(n_ready, (uint32_t)__popcll(m));
    base = __shfl(base, leader);
    if (top_ready) ready[base + __popcll(m & ((1ull << lane) - 1))] = (uint32_t)i;
  }
}

__device__ __forceinline__ void child_box(const float* boxes, int64_t n, uint32_t c, float b[6]) {
  const int64_t idx = (c & kLeafFlag) ? (n - 1) + (c & ~kLeafFlag) : c;
#pragma unroll
  for (int a = 0; a < 6; ++a) b[a] = boxes[idx * 6 + a];
}

// Phase 2: one workgroup. A thread starts at a ready top node and climbs; at a parent with
// two top children the first arrival stops and the second continues.
__global__ void __launch_bounds__(kTopBlock) k_refit_top(int64_t n, const uint32_t* __restrict__ child,
                                                         const uint32_t* __restrict__ parent,
                                                         const uint2* __restrict__ range, float* boxes,
                                                         const uint32_t* __restrict__ ready,
                                                         const uint32_t* __restrict__ n_ready,
                                                         uint32_t* __restrict__ arrivals, int64_t small) {
  const uint32_t cnt = *n_ready;
  for (uint32_t w = threadIdx.x; w < cnt; w += kTopBlock) {
    uint32_t node = ready[w];
    while (true) {
      const uint32_t c0 = child[2 * (int64_t)node], c1 = child[2 * (int64_t)node + 1];
      float b0[6], b1[6];
      child_box(boxes, n, c0, b0);
      child_box(boxes, n, c1, b1);
      write_box(boxes, node, b0, b1);
      const uint32_t p = parent[node];
      if (p == kNoParent) break;
      const bool two =
          !is_small(child[2 * (int64_t)p], range, small) && !is_small(child[2 * (int64_t)p + 1], range, small);
      // release this node's box to the sibling's thread; acquire the sibling's box
      if (two && __hip_atomic_fetch_add(&arrivals[p], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_WORKGROUP) == 0u)
        break;
      node = p;
    }
  }
}

// Four-wide node records (layout in grtx_internal.h), written once every box is final.
__global__ void __launch_bounds__(kBlock) k_wide(int64_t n, const uint32_t* __restrict__ child,
                                                 const float* __restrict__ boxes, float4* __restrict__ nodes) {
  const int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x;
  if (i >= n - 1) return;
  // Start from the two children and open the internal entry of largest surface area
  // until there are four entries or none is internal (greedy collapse; every internal
  // node has a record, so a record may list nodes from any depth below it).
  uint32_t ref[4] = {child[2 * i], child[2 * i + 1], kNoChild, kNoChild};
  int cnt = 2;
  while (cnt < 4) {
    int best = -1;
    float best_area = -1.f;
    for (int j = 0; j < cnt; ++j) {
      if (ref[j] & kLeafFlag) continue;
      const float* bb = boxes + 6 * (int64_t)ref[j];
      const float ex = bb[3] - bb[0], ey = bb[4] - bb[1], ez = bb[5] - bb[2];
      const float area = ex * ey + ey * ez + ez * ex;
      if (area > best_area) {
        best_area = area;
        best = j;
      }
    }
    if (best < 0) break;
    const uint32_t c = ref[best];
    ref[best] = child[2 * (int64_t)c];
    ref[cnt++] = child[2 * (int64_t)c + 1];
  }
  const float* own = boxes + 6 * i;  // the union of the children's boxes
  float org[3], step[3];
  uint32_t wlo[3] = {0u, 0u, 0u}, whi[3] = {0u, 0u, 0u};
  for (int a = 0; a < 3; ++a) {
    org[a] = own[a];
    const double ext = (double)own[3 + a] - (double)own[a];
    int e = -126;
    if (ext > 0.0) {
      (void)frexp(ext / 254.0, &e);  // ext / 254 <= 2^e
      e = e < -126 ? -126 : e;
    }
    step[a] = ldexpf(1.0f, e);
  }
  for (int j = 0; j < cnt; ++j) {
    float b[6];
    child_box(boxes, n, ref[j], b);
    for (int a = 0; a < 3; ++a) {
      const double s = (double)step[a];
      double ql = floor(((double)b[a] - (double)org[a]) / s);
      double qh = ceil(((double)b[3 + a] - (double)org[a]) / s);
      ql = ql < 0.0 ? 0.0 : ql > 255.0 ? 255.0 : ql;
      qh = qh < 0.0 ? 0.0 : qh > 255.0 ? 255.0 : qh;
      wlo[a] |= (uint32_t)ql << (8 * j);
      whi[a] |= (uint32_t)qh << (8 * j);
    }
  }
  float4* r = nodes + (int64_t)kNodeF4 * i;
  r[0] = make_float4(org[0], org[1], org[2], step[0]);
  r[1] = make_float4(step[1], step[2], __uint_as_float(ref[0]), __uint_as_float(ref[1]));
  r[2] = make_float4(__uint_as_float(ref[2]), __uint_as_float(ref[3]), __uint_as_float(wlo[0]),
                     __uint_as_float(wlo[1]));
  r[3] = make_float4(__uint_as_float(wlo[2]), __uint_as_float(whi[0]), __uint_as_float(whi[1]),
                     __uint_as_float(whi[2]));
}

// ------------------------------------------------------------------ record layout
// Only the records that the traversal can reach are kept, about a third of the radix
// tree's internal nodes: the root's, and recursively those its entries list (a record's
// opened entries are interior to it). They are laid out breadth first: the records of
// nodes above kLayoutLeaves leaves by one workgroup, level by level, from position 0;
// each node of at most kLayoutLeaves leaves that such a record lists starts a task, a
// block of (leaves - 1) positions (the most records its subtree can have) reserved after
// the first `top_cap` positions, which one wave fills breadth first. So the records a
// ray meets near each other lie near each other, and the lines fetched hold live records
// only. `qold` maps each position of the top levels to the radix-tree node whose record it
// holds.
constexpr int64_t kLayoutLeaves = 128;
constexpr int kLayoutBlock = 1024;

// Reserve and record a task for internal node c (leaf count cnt); returns its position.
__device__ __forceinline__ uint32_t new_task(uint32_t c, uint32_t cnt, uint32_t top_cap, uint32_t* task_cursor,
                                             uint32_t* n_tasks, uint2* tasks) {
  const uint32_t start = top_cap + atomicAdd(task_cursor, cnt - 1u);
  tasks[atomicAdd(n_tasks, 1u)] = make_uint2(c, start);
  return start;
}

// Copy the record of radix-tree node `old` to position `pos` with its internal entries
// replaced by the positions `pos_of` assigns them.
template <class F>
__device__ __forceinline__ void place_record(const float4* __restrict__ wide, uint32_t old, uint32_t pos,
                                             float4* __restrict__ nodes, F&& pos_of) {
  const float4* src = wide + (int64_t)kNodeF4 * old;
  float4 q0 = src[0], q1 = src[1], q2 = src[2], q3 = src[3];
  uint32_t r[4] = {__float_as_uint(q1.z), __float_as_uint(q1.w), __float_as_uint(q2.x), __float_as_uint(q2.y)};
#pragma unroll
  for (int j = 0; j < 4; ++j)
    if (r[j] != kNoChild && !(r[j] & kLeafFlag)) r[j] = pos_of(r[j]);
  q1.z = __uint_as_float(r[0]);
  q1.w = __uint_as_float(r[1]);
  q2.x = __uint_as_float(r[2]);
  q2.y = __uint_as_float(r[3]);
  float4* dst = nodes + (int64_t)kNodeF4 * pos;
  dst[0] = q0;
  dst[1] = q1;
  dst[2] = q2;
  dst[3] = q3;
}

// The top levels (one workgroup; its counters live in LDS until the end). Root = radix-tree
// node 0 at position 0; with at most kLayoutLeaves leaves in all, the root itself is the
// only task (top_cap = 0).
__global__ void __launch_bounds__(kLayoutBlock) k_layout_top(int64_t m, const float4* __restrict__ wide,
                                                             const uint32_t* __restrict__ count, uint32_t top_cap,
                                                             float4* __restrict__ nodes, uint32_t* __restrict__ qold,
                                                             uint2* __restrict__ tasks, uint32_t* __restrict__ ctr) {
  __shared__ uint32_t s_next, s_cursor, s_tasks;
  if (m <= kLayoutLeaves) {
    if (threadIdx.x == 0) {
      ctr[0] = (uint32_t)(m - 1);
      ctr[1] = 1u;
      tasks[0] = make_uint2(0u, 0u);
    }
    return;
  }
  if (threadIdx.x == 0) {
    s_cursor = 0u;
    s_tasks = 0u;
    qold[0] = 0u;
    s_next = 1u;
  }
  __syncthreads();
  uint32_t begin = 0, end = 1;
  while (begin < end) {
    for (uint32_t q = begin + threadIdx.x; q < end; q += kLayoutBlock) {
      place_record(wide, qold[q], q, nodes, [&](uint32_t c) {
        const uint32_t cnt = count[c];
        if (cnt > (uint32_t)kLayoutLeaves) {
          const uint32_t pos = atomicAdd(&s_next, 1u);
          qold[pos] = c;
          return pos;
        }
        return new_task(c, cnt, top_cap, &s_cursor, &s_tasks, tasks);
      });
    }
    __syncthreads();
    begin = end;
    end = s_next;
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    ctr[0] = s_cursor;
    ctr[1] = s_tasks;
  }
}

// The tasks: one wave fills a block breadth first, a level at a time. The records of one
// level belong to disjoint subtrees of two leaves or more, so a block of at most
// kLayoutLeaves leaves has at most kLayoutLeaves / 2 = 64 records per level: one per lane.
// Each lane places its record, its internal entries taking the next positions in lane and
// entry order (the order a sequential breadth-first fill gives), and passes their
// radix-tree nodes through LDS to the lanes that place them on the next level.
static_assert(kLayoutLeaves / 2 <= 64, "a level of a layout block must fit one wave");
__global__ void __launch_bounds__(kBlock) k_layout_tasks(const float4* __restrict__ wide, const uint2* __restrict__ tasks,
                                                         const uint32_t* __restrict__ ctr, float4* __restrict__ nodes) {
  __shared__ uint32_t s_next[kBlock / 64][64];
  const uint32_t n = ctr[1];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const uint64_t below = lane ? ~0ull >> (64 - lane) : 0ull;
  for (uint32_t t = blockIdx.x * (kBlock / 64) + w; t < n; t += gridDim.x * (kBlock / 64)) {
    const uint2 task = tasks[t];
    uint32_t begin = task.y, width = 1, old = task.x;
    while (width > 0) {
      const bool mine = (uint32_t)lane < width;
      float4 q0{}, q1{}, q2{}, q3{};
      if (mine) {
        const float4* src = wide + (int64_t)kNodeF4 * old;
        q0 = src[0];
        q1 = src[1];
        q2 = src[2];
        q3 = src[3];
      }
      uint32_t r[4] = {__float_as_uint(q1.z), __float_as_uint(q1.w), __float_as_uint(q2.x), __float_as_uint(q2.y)};
      bool in[4];
      uint32_t below_n = 0, total = 0;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        in[j] = mine && r[j] != kNoChild && !(r[j] & kLeafFlag);
        const uint64_t m = __ballot(in[j]);
        below_n += (uint32_t)__popcll(m & below);
        total += (uint32_t)__popcll(m);
      }
      const uint32_t nbeg = begin + width;
      asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");  // last level's reads of s_next are done
      if (mine) {
        uint32_t k = below_n;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          if (in[j]) {
            s_next[w][k] = r[j];
            r[j] = nbeg + k;
            ++k;
          }
        }
        q1.z = __uint_as_float(r[0]);
        q1.w = __uint_as_float(r[1]);
        q2.x = __uint_as_float(r[2]);
        q2.y = __uint_as_float(r[3]);
        float4* dst = nodes + (int64_t)kNodeF4 * (begin + (uint32_t)lane);
        dst[0] = q0;
        dst[1] = q1;
        dst[2] = q2;
        dst[3] = q3;
      }
      asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");  // this level's writes to s_next are done
      width = total < 64u ? total : 64u;  // (total <= 64 by the bound above)
      old = (uint32_t)lane < width ? s_next[w][lane] : 0u;
      begin = nbeg;
    }
  }
}

// ------------------------------------------------------------------ density grid
// Leaves per cell of a kDensityRes^3 grid over the leaf centres' bounds. A thread counts
// kDensityRun consecutive sorted leaves and adds each run of equal cells with one atomic.
constexpr int kDensityRun = 16;
__global__ void __launch_bounds__(kBlock) k_density(const float* __restrict__ pts, const uint32_t* __restrict__ perm,
                                                    int64_t m, const float* __restrict__ bounds,
                                                    uint32_t* __restrict__ grid) {
  const int64_t i0 = (blockIdx.x * (int64_t)kBlock + threadIdx.x) * kDensityRun;
  if (i0 >= m) return;
  int cur = -1;
  uint32_t run = 0;
  const int64_t i1 = i0 + kDensityRun < m ? i0 + kDensityRun : m;
  for (int64_t i = i0; i < i1; ++i) {
    const float* p = pts + 3 * (int64_t)perm[i];
    const int c = density_cell(p[0], p[1], p[2], bounds);
    if (c == cur) {
      ++run;
    } else {
      if (run) atomicAdd(grid + cur, run);
      cur = c;
      run = 1;
    }
  }
  if (run) atomicAdd(grid + cur, run);
}

// ------------------------------------------------------------------ pinhole rays

__global__ void __launch_bounds__(kBlock) k_pinhole(CameraFrame cf, int W, int H, float* __restrict__ origins,
                                                    float* __restrict__ dirs) {
  int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x;
  if (i >= (int64_t)W * H) return;
  int y = (int)(i / W), x = (int)(i - (int64_t)y * W);
  float dx, dy, dz;
  pinhole_dir(cf.fwd[0], cf.fwd[1], cf.fwd[2], cf.right[0], cf.right[1], cf.right[2], cf.up[0], cf.up[1], cf.up[2], x, y,
              W, H, &dx, &dy, &dz);
  origins[3 * i + 0] = cf.eye[0];
  origins[3 * i + 1] = cf.eye[1];
  origins[3 * i + 2] = cf.eye[2];
  dirs[3 * i + 0] = dx;
  dirs[3 * i + 1] = dy;
  dirs[3 * i + 2] = dz;
}

inline unsigned grid_for(int64_t n) { return (unsigned)std::max<int64_t>(1, (n + kBlock - 1) / kBlock); }



grtx_status radix_sort(uint64_t* keys, uint32_t* vals, uint64_t* tkeys, uint32_t* tvals, int64_t n, Scratch& sc,
                       hipStream_t s, int passes = 8, const uint32_t* n_dev = nullptr, uint64_t** kres = nullptr,
                       uint32_t** vres = nullptr) {
  const int items = n <= kRadixSmall ? kRadixItemsSmall : kRadixItems;
  const int64_t tile = (int64_t)kBlock * items;
  int nblocks = (int)((n + tile - 1) / tile);
  const bool fused = nblocks <= kRadixFusedBlocks;
  int64_t hn = (int64_t)256 * nblocks;
  uint32_t *hist = nullptr, *offs = nullptr, *part = nullptr;
  int nparts = (int)((hn + kScanChunk - 1) / kScanChunk);
  if (nparts > kScanChunk) {
    set_error("radix sort: %lld keys exceed the supported size", (long long)n);
    return GRTX_ERR_INVALID_ARG;
  }
  GRTX_TRY(sc.get(&hist, hn));
  GRTX_TRY(sc.get(&offs, hn));
  GRTX_TRY(sc.get(&part, nparts));
  uint64_t* kin = keys;
  uint32_t* vin = vals;
  uint64_t* kout = tkeys;
  uint32_t* vout = tvals;
  for (int pass = 0; pass < passes; ++pass) {
    int shift = 8 * pass;
    hipLaunchKernelGGL(k_radix_hist, dim3(nblocks), dim3(kBlock), 0, s, kin, n, shift, items, hist, nblocks, fused,
                       n_dev);
    if (fused) {
      // the scatter turns the counts into offsets itself
    } else if (nparts > 1 && nparts <= kScanLoopChunks) {
      hipLaunchKernelGGL(k_scan_loop, dim3(1), dim3(kBlock), 0, s, hist, hn, offs);
    } else if (nparts > 1) {
      hipLaunchKernelGGL(k_scan_reduce, dim3(nparts), dim3(kBlock), 0, s, hist, hn, part);
      hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(kBlock), 0, s, part, nparts);
      hipLaunchKernelGGL(k_scan_down, dim3(nparts), dim3(kBlock), 0, s, hist, hn, part, offs);
    } else {
      hipLaunchKernelGGL(k_scan_down, dim3(1), dim3(kBlock), 0, s, hist, hn, (const uint32_t*)nullptr, offs);
    }
    hipLaunchKernelGGL(k_radix_scatter, dim3(nblocks), dim3(kBlock), 0, s, kin, vin, n, shift, items,
                       fused ? hist : offs, nblocks, fused, kout, vout, n_dev);
    GRTX_LAUNCH_CHECK();
    std::swap(kin, kout);
    std::swap(vin, vout);
  }
  if (kres) {  // the caller takes the result where the last pass left it
    *kres = kin;
    *vres = vin;
  } else if (kin != keys) {  // an odd number of passes leaves the result in the temporaries
    GRTX_HIP(hipMemcpyAsync(keys, kin, sizeof(uint64_t) * n, hipMemcpyDeviceToDevice, s));
    GRTX_HIP(hipMemcpyAsync(vals, vin, sizeof(uint32_t) * n, hipMemcpyDeviceToDevice, s));
  }
  return GRTX_OK;
}

// Root entry: the root's box and reference (internal node 0, or leaf 0 for one leaf).
// ------------------------------------------------------------------ treelet restructuring
// One bottom-up pass over the radix tree that rebuilds, at every internal node, the
// treelet of the node and its largest descendants (up to kTreeletLeaves treelet leaves,
// opened by largest surface area) into the binary topology of least surface-area cost,
// found by dynamic programming over the subsets of the treelet leaves (restructuring after
// Karras and Aila's treelet optimisation). Leaves keep their sorted positions, so the
// leaf order of the instances and every traced result are unchanged; only internal nodes
// are rewired, each keeping its index. A node is processed by the second of the two
// threads that reach it from its children, after both subtrees are final.
constexpr int kTreeletLeaves = 5;
constexpr float kCostNode = 1.2f;  // surface-area cost of visiting an internal node
constexpr float kCostLeaf = 1.f;   // ... of testing a leaf

__device__ __forceinline__ float half_area(const float* __restrict__ b) {
  const float ex = fmaxf(b[3] - b[0], 0.f), ey = fmaxf(b[4] - b[1], 0.f), ez = fmaxf(b[5] - b[2], 0.f);
  return ex * ey + ey * ez + ez * ex;
}

__device__ __forceinline__ uint32_t node_of(uint32_t c, int64_t nint) {
  return (c & kLeafFlag) ? (uint32_t)(nint + (c & ~kLeafFlag)) : c;
}
__device__ __forceinline__ uint32_t ref_of(uint32_t u, int64_t nint) {
  return (int64_t)u >= nint ? kLeafFlag | (uint32_t)(u - nint) : u;
}

// Per-thread work arrays of the subset dynamic programme live in LDS, entry-major
// ([entry][thread]), so that lanes index them independently; NS threads per workgroup,
// one per leaf of its subtree.
constexpr int kSets = 1 << kTreeletLeaves;
template <int NS>
struct TreeletLds {
  float copt[kSets][NS];
  uint8_t split[kSets][NS];
  int stack_set[kTreeletLeaves][NS];
  uint32_t stack_node[kTreeletLeaves][NS];
};
// Subtree size of the per-subtree pass: 256 leaves, 128 above a million leaves. Smaller
// subtrees give shorter bottom-up chains and twice the workgroups per CU (at 3M leaves the
// two passes took 1.43 + 0.30 ms against 1.59 + 0.23 ms, trace time unchanged), but leave
// more nodes above them untouched where no second pass runs (100k: 0.7% more node visits
// per ray).
inline int subtree_leaves(int64_t m) { return m > ((int64_t)1 << 20) ? 128 : 256; }
// Per-subtree passes: one, three above a million leaves. Each further pass rebuilds the
// treelets the previous one left, and skips treelet roots of fewer than kLaterPassLeaves
// leaves (doubled per pass), where little is left to gain (after Karras and Aila's
// repeated passes with a growing minimum). At 3M leaves the three passes cut node visits
// per ray by 2.6% and trace time by 5%, for 4 ms more build; at 100k the trace gains less
// than the pass costs.
inline int treelet_passes(int64_t m) { return m > ((int64_t)1 << 20) ? 3 : 1; }
constexpr uint32_t kLaterPassLeaves = 4;

// Subset dynamic programme over NL treelet leaves, unrolled at compile time so that every
// subset and split index is a constant (the costs stay in registers); the chosen splits and
// costs then go to the thread's LDS column for the rebuild.
template <int NL, class Lds>
__device__ __forceinline__ void treelet_dp(const float (&lb)[kTreeletLeaves][6], const float (&lcost)[kTreeletLeaves],
                                           Lds& L, int tid) {
  float copt[1 << NL];
#pragma unroll
  for (int S = 1; S < (1 << NL); ++S) {
    if ((S & (S - 1)) == 0) {
      copt[S] = lcost[__builtin_ctz(S)];
      L.copt[S][tid] = copt[S];
      continue;
    }
    float b[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
#pragma unroll
    for (int q = 0; q < NL; ++q)
      if (S >> q & 1) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          b[a] = fminf(b[a], lb[q][a]);
          b[3 + a] = fmaxf(b[3 + a], lb[q][3 + a]);
        }
      }
    float best = INFINITY;
    int bp = 0;
#pragma unroll
    for (int P = 1; P < S; ++P) {
      if ((P & S) != P || !(P & S & -S)) continue;  // each split once: the part holding the lowest leaf
      const float c = copt[P] + copt[S ^ P];
      if (c < best) {
        best = c;
        bp = P;
      }
    }
    copt[S] = kCostNode * half_area(b) + best;
    L.copt[S][tid] = copt[S];
    L.split[S][tid] = (uint8_t)bp;
  }
}

template <class Lds>
__device__ __forceinline__ void restructure(uint32_t p, int64_t nint, uint32_t* __restrict__ child, uint32_t* __restrict__ parent,
                            float* __restrict__ boxes, float* __restrict__ cost, uint32_t* __restrict__ count,
                            Lds& L, int tid) {
  // treelet leaves (registers, constant indices only) and its internal nodes
  uint32_t leaf[kTreeletLeaves], inner[kTreeletLeaves - 1];
  float larea[kTreeletLeaves];
#pragma unroll
  for (int q = 0; q < kTreeletLeaves; ++q) {
    leaf[q] = 0u;
    larea[q] = -1.f;
  }
#pragma unroll
  for (int q = 0; q < kTreeletLeaves - 1; ++q) inner[q] = p;
  int nl = 2;
  leaf[0] = node_of(child[2 * (int64_t)p], nint);
  leaf[1] = node_of(child[2 * (int64_t)p + 1], nint);
  larea[0] = half_area(boxes + 6 * (int64_t)leaf[0]);
  larea[1] = half_area(boxes + 6 * (int64_t)leaf[1]);
#pragma unroll
  for (int step = 0; step < kTreeletLeaves - 2; ++step) {
    // open the internal treelet leaf of largest surface area
    int best = -1;
    float ba = -1.f;
#pragma unroll
    for (int q = 0; q < kTreeletLeaves; ++q)
      if (q < nl && (int64_t)leaf[q] < nint && larea[q] > ba) {
        ba = larea[q];
        best = q;
      }
    if (best < 0) break;
    uint32_t x = 0u;
#pragma unroll
    for (int q = 0; q < kTreeletLeaves; ++q)
      if (q == best) x = leaf[q];
    inner[step + 1] = x;
    const uint32_t c0 = node_of(child[2 * (int64_t)x], nint), c1 = node_of(child[2 * (int64_t)x + 1], nint);
    const float a0 = half_area(boxes + 6 * (int64_t)c0), a1 = half_area(boxes + 6 * (int64_t)c1);
#pragma unroll
    for (int q = 0; q < kTreeletLeaves; ++q) {
      if (q == best) {
        leaf[q] = c0;
        larea[q] = a0;
      }
      if (q == nl) {
        leaf[q] = c1;
        larea[q] = a1;
      }
    }
    ++nl;
  }
  // the treelet leaves' boxes, counts and costs, read once
  float lb[kTreeletLeaves][6];
  uint32_t lcnt[kTreeletLeaves];
  float lcost[kTreeletLeaves];
#pragma unroll
  for (int q = 0; q < kTreeletLeaves; ++q) {
    if (q < nl) {
      const float* bq = boxes + 6 * (int64_t)leaf[q];
#pragma unroll
      for (int a = 0; a < 6; ++a) lb[q][a] = bq[a];
      lcnt[q] = (int64_t)leaf[q] >= nint ? 1u : count[leaf[q]];
      lcost[q] = cost[leaf[q]];
    } else {
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        lb[q][a] = INFINITY;
        lb[q][3 + a] = -INFINITY;
      }
      lcnt[q] = 0u;
      lcost[q] = 0.f;
    }
  }
  auto set_box = [&](int S, float b[6]) __attribute__((always_inline)) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      b[a] = INFINITY;
      b[3 + a] = -INFINITY;
    }
#pragma unroll
    for (int q = 0; q < kTreeletLeaves; ++q)
      if (S >> q & 1) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          b[a] = fminf(b[a], lb[q][a]);
          b[3 + a] = fmaxf(b[3 + a], lb[q][3 + a]);
        }
      }
  };
  // optimal cost of every subset of the treelet leaves and the split that reaches it
  const int full = (1 << nl) - 1;
  if (nl == kTreeletLeaves) treelet_dp<kTreeletLeaves>(lb, lcost, L, tid);
  else if (nl == 4) treelet_dp<4>(lb, lcost, L, tid);
  else if (nl == 3) treelet_dp<3>(lb, lcost, L, tid);
  else treelet_dp<2>(lb, lcost, L, tid);
  // rebuild top-down, reusing the treelet's internal nodes (p stays the root)
  int sp = 0, next = 1;
  L.stack_set[0][tid] = full;
  L.stack_node[0][tid] = p;
  sp = 1;
  while (sp > 0) {
    --sp;
    const int S = L.stack_set[sp][tid];
    const uint32_t node = L.stack_node[sp][tid];
    const int P = L.split[S][tid];
    for (int k = 0; k < 2; ++k) {
      const int X = k == 0 ? P : S ^ P;
      uint32_t c = 0u;
      if ((X & (X - 1)) == 0) {
#pragma unroll
        for (int q = 0; q < kTreeletLeaves; ++q)
          if (X == (1 << q)) c = leaf[q];
      } else {
#pragma unroll
        for (int q = 1; q < kTreeletLeaves - 1; ++q)
          if (q == next) c = inner[q];
        ++next;
        L.stack_set[sp][tid] = X;
        L.stack_node[sp][tid] = c;
        ++sp;
      }
      child[2 * (int64_t)node + k] = ref_of(c, nint);
      parent[c] = node;
    }
    float b[6];
    set_box(S, b);
    uint32_t cnt = 0;
#pragma unroll
    for (int q = 0; q < kTreeletLeaves; ++q)
      if (S >> q & 1) cnt += lcnt[q];
    float* nb = boxes + 6 * (int64_t)node;
#pragma unroll
    for (int a = 0; a < 6; ++a) nb[a] = b[a];
    cost[node] = L.copt[S][tid];
    count[node] = cnt;
  }
}

// The pass runs per subtree of at most NS leaves whose parent has more (the
// nodes above keep the radix tree's topology): one workgroup takes a subtree, its threads
// its leaves (a contiguous run [lo, hi] of sorted positions). The subtree's internal nodes
// are exactly the indices lo..hi-1 of the radix tree (each internal node is numbered after
// one end of its range), and restructuring only permutes them, so the arrival counters of
// the bottom-up hand-over sit in LDS at index - lo, ordered with workgroup-scope fences.
// Workgroups draw subtrees from a queue.
template <int NS>
__global__ void __launch_bounds__(NS) k_treelet(int64_t m, const uint32_t* __restrict__ roots,
                                                            const uint32_t* __restrict__ n_roots,
                                                            unsigned int* __restrict__ queue,
                                                            const uint2* __restrict__ range, uint32_t* child,
                                                            uint32_t* parent, float* boxes, float* cost,
                                                            uint32_t* count, uint32_t min_leaves) {
  __shared__ TreeletLds<NS> L;
  __shared__ uint32_t s_item;
  __shared__ uint32_t s_arrive[NS];
  const int64_t nint = m - 1;
  const uint32_t nr = *n_roots;
  const int tid = threadIdx.x;
  while (true) {
    if (tid == 0) s_item = atomicAdd(queue, 1u);
    __syncthreads();
    const uint32_t item = s_item;
    __syncthreads();
    if (item >= nr) return;
    const uint32_t r = roots[item];
    const int64_t lo = (int64_t)r < nint ? (int64_t)range[r].x : (int64_t)r - nint;
    const int64_t n = (int64_t)r < nint ? (int64_t)range[r].y - range[r].x + 1 : 1;
    s_arrive[tid] = 0u;
    __syncthreads();
    if ((int64_t)tid < n) {
      const uint32_t u = (uint32_t)(nint + lo + tid);
      cost[u] = kCostLeaf * half_area(boxes + 6 * (int64_t)u);
      if (u != r) {
        uint32_t p = parent[u];
        while (true) {
          // the first thread to arrive leaves; the second sees both subtrees
          if ((uint64_t)((int64_t)p - lo) >= (uint64_t)NS) break;  // outside the run: never
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
          if (atomicAdd(&s_arrive[p - lo], 1u) == 0u) break;
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
          if (min_leaves == 0u || count[p] >= min_leaves) {
            restructure(p, nint, child, parent, boxes, cost, count, L, tid);
          } else {
            // kept as it is; its cost follows its children's
            cost[p] = kCostNode * half_area(boxes + 6 * (int64_t)p) + cost[node_of(child[2 * (int64_t)p], nint)] +
                      cost[node_of(child[2 * (int64_t)p + 1], nint)];
          }
          if (p == r) break;
          p = parent[p];
        }
      }
    }
    __syncthreads();
  }
}

// The nodes above the subtrees, in a second pass for trees of more than kTopPassLeaves
// leaves (below that the top part is a few hundred nodes and the pass costs more than it
// saves): a thread per subtree root walks up, the second arrival at a node restructures
// it. Threads of different workgroups hand over here, so the counters are agent-scope
// atomics in global memory.
constexpr int64_t kTopPassLeaves = (int64_t)1 << 20;
template <int NS>
__global__ void __launch_bounds__(NS) k_treelet_top(int64_t m, const uint32_t* __restrict__ roots,
                                                                const uint32_t* __restrict__ n_roots,
                                                                uint32_t* child, uint32_t* parent, float* boxes,
                                                                float* cost, uint32_t* count,
                                                                uint32_t* arrivals) {
  __shared__ TreeletLds<NS> L;
  const int tid = threadIdx.x;
  const int64_t k = blockIdx.x * (int64_t)NS + tid;
  if (k >= (int64_t)*n_roots) return;
  const int64_t nint = m - 1;
  uint32_t p = parent[roots[k]];
  while (p != kNoParent) {
    if (__hip_atomic_fetch_add(arrivals + p, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) == 0u) return;
    restructure(p, nint, child, parent, boxes, cost, count, L, tid);
    p = parent[p];
  }
}

// Subtree roots for the restructuring pass: nodes of at most `limit` leaves whose parent
// has more (or that are the root), listed in node order.
__global__ void k_subtree_roots(int64_t nn, const uint32_t* __restrict__ flag, const uint32_t* __restrict__ pos,
                                uint32_t* __restrict__ roots, uint32_t* __restrict__ n_roots) {
  const int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x;
  if (i >= nn) return;
  if (i == nn - 1) *n_roots = pos[i] + flag[i];
  if (flag[i]) roots[pos[i]] = (uint32_t)i;
}


// Cut of the tree for per-tile cost estimates of image traces (the trace takes the
// heaviest tiles first): every node of at most `cut` leaves whose parent has more (or that
// is the root). Nodes are numbered internal first, then leaves, as in `parent`.
__device__ __forceinline__ uint32_t leaves_below(int64_t i, int64_t nint, const uint32_t* __restrict__ count) {
  return i < nint ? count[i] : 1u;
}

__global__ void k_cut_flags(int64_t nn, int64_t nint, const uint32_t* __restrict__ parent,
                            const uint32_t* __restrict__ range, uint32_t cut, uint32_t* __restrict__ flag) {
  const int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x;
  if (i >= nn) return;
  const uint32_t p = parent[i];
  const bool big_parent = p == kNoParent || leaves_below(p, nint, range) > cut;
  flag[i] = leaves_below(i, nint, range) <= cut && big_parent ? 1u : 0u;
}

// Records (lo xyz, leaf count) (hi xyz, 0) of the cut nodes, in node order, up to kCutCap.
__global__ void k_cut_write(int64_t nn, int64_t nint, const uint32_t* __restrict__ flag,
                            const uint32_t* __restrict__ pos, const uint32_t* __restrict__ range,
                            const float* __restrict__ boxes, float4* __restrict__ cutrec, uint32_t* __restrict__ n_cut) {
  const int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x;
  if (i >= nn) return;
  if (i == nn - 1) *n_cut = pos[i] + flag[i];
  if (!flag[i] || pos[i] >= (uint32_t)kCutCap) return;
  const float* bx = boxes + 6 * i;
  cutrec[2 * (int64_t)pos[i]] = make_float4(bx[0], bx[1], bx[2], (float)leaves_below(i, nint, range));
  cutrec[2 * (int64_t)pos[i] + 1] = make_float4(bx[3], bx[4], bx[5], 0.f);
}

__global__ void k_write_root(const float* __restrict__ box, uint32_t ref, float* __restrict__ roots) {
  if (threadIdx.x < 6) roots[threadIdx.x] = box[threadIdx.x];
  if (threadIdx.x == 6) roots[6] = __uint_as_float(ref);
  if (threadIdx.x == 7) roots[7] = 0.f;
}

__global__ void __launch_bounds__(kBlock) k_fill_u32(uint32_t* p, int64_t n, uint32_t v) {
  int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x;
  if (i < n) p[i] = v;
}

// ------------------------------------------------------------------ tree depth
// Depth of the tree in internal nodes on the longest root-to-leaf path, which bounds the
// trace's traversal stack (a four-wide record leaves at most three entries pending per
// level). One thread per leaf climbs towards the root carrying the number of internal
// nodes below it on its path and raises the per-node maximum `h`; it stops where a path at
// least as long has already been recorded, so most climbs end after a few steps. The
// root is node 0. A climb longer than `cap` stops there and records cap + 1 at the root
// (the tree is then too deep whatever its exact depth).
__global__ void __launch_bounds__(kBlock) k_tree_height(int64_t m, const uint32_t* __restrict__ parent,
                                                        uint32_t* __restrict__ h, int cap,
                                                        const uint32_t* __restrict__ only_if) {
  if (only_if && *only_if == 0u) return;
  const int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x;
  if (i >= m) return;
  uint32_t p = parent[(m - 1) + i];
  uint32_t d = 1;
  while (p != kNoParent) {
    if (d > (uint32_t)cap) {
      atomicMax(h, (uint32_t)cap + 1u);
      return;
    }
    if (atomicMax(h + p, d) >= d) return;
    ++d;
    p = parent[p];
  }
}

// Saved topology of the plain radix tree, put back when the restructured tree is deeper
// than `max_depth` (the plain tree over distinct 95-bit keys is at most 96 deep): child,
// parent, the internal boxes and leaf counts. `deep[0]` records the decision for the
// later kernels, which also recompute the depth of the tree put back into `h2`.
struct PlainTree {
  const uint32_t* child;
  const uint32_t* parent;
  const float* boxes;
  const uint32_t* count;
};
__global__ void __launch_bounds__(kBlock) k_restore_plain(int64_t m, const uint32_t* __restrict__ h, int max_depth,
                                                          PlainTree saved, uint32_t* __restrict__ child,
                                                          uint32_t* __restrict__ parent, float* __restrict__ boxes,
                                                          uint32_t* __restrict__ count, uint32_t* __restrict__ h2,
                                                          uint32_t* __restrict__ deep) {
  const bool too_deep = h[0] > (uint32_t)max_depth;
  const int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x;
  if (i == 0) deep[0] = too_deep ? 1u : 0u;
  if (!too_deep) return;
  const int64_t nint = m - 1;
  if (i < nint) {
    child[2 * i] = saved.child[2 * i];
    child[2 * i + 1] = saved.child[2 * i + 1];
    for (int a = 0; a < 6; ++a) boxes[6 * i + a] = saved.boxes[6 * i + a];
    count[i] = saved.count[i];
    h2[i] = 0u;
  }
  if (i < 2 * m - 1) parent[i] = saved.parent[i];
}

// Final depth and kind of the tree: out[0] = depth, out[1] = 1 if the restructured tree
// was kept. `deep` and `h2` are null when no restructuring ran.
__global__ void k_depth_store(const uint32_t* __restrict__ h, const uint32_t* __restrict__ deep,
                              const uint32_t* __restrict__ h2, uint32_t* __restrict__ out) {
  if (threadIdx.x != 0) return;
  const bool restored = deep && deep[0] != 0u;
  out[0] = restored ? h2[0] : h[0];
  out[1] = deep && !restored ? 1u : 0u;
}

}  // namespace

// Build over `n` points (centroids) whose leaf boxes/records are produced by `leaves`.
// Icosahedron of inradius 1, from its definition: the 12 points (0,+-1,+-phi) and their
// cyclic permutations; faces are the vertex triples at mutual distance 2 (the edge), wound
// so that (B-A) x (C-A) points away from the centre; scaled so face planes are at distance 1.
static Ico make_icosahedron() {
  const double phi = 0.5 * (1.0 + std::sqrt(5.0));
  double v[12][3];
  int nv = 0;
  for (int sa = -1; sa <= 1; sa += 2)
    for (int sb = -1; sb <= 1; sb += 2) {
      const double p[3] = {0.0, (double)sa, sb * phi};
      for (int rot = 0; rot < 3; ++rot) {
        for (int a = 0; a < 3; ++a) v[nv][a] = p[(a + 3 - rot) % 3];
        ++nv;
      }
    }
  Ico ico{};
  int nf = 0;
  double inr = 0.0;
  for (int i = 0; i < 12; ++i)
    for (int j = i + 1; j < 12; ++j)
      for (int k = j + 1; k < 12; ++k) {
        auto d2 = [&](int x, int y) {
          double s2 = 0.0;
          for (int a = 0; a < 3; ++a) s2 += (v[x][a] - v[y][a]) * (v[x][a] - v[y][a]);
          return s2;
        };
        if (std::fabs(d2(i, j) - 4.0) > 1e-9 || std::fabs(d2(j, k) - 4.0) > 1e-9 || std::fabs(d2(i, k) - 4.0) > 1e-9)
          continue;
        double e1[3], e2[3], nrm[3], cen = 0.0;
        for (int a = 0; a < 3; ++a) {
          e1[a] = v[j][a] - v[i][a];
          e2[a] = v[k][a] - v[i][a];
        }
        nrm[0] = e1[1] * e2[2] - e1[2] * e2[1];
        nrm[1] = e1[2] * e2[0] - e1[0] * e2[2];
        nrm[2] = e1[0] * e2[1] - e1[1] * e2[0];
        for (int a = 0; a < 3; ++a) cen += nrm[a] * v[i][a];
        bool out = cen > 0.0;
        ico.f[nf][0] = (unsigned char)i;
        ico.f[nf][1] = (unsigned char)(out ? j : k);
        ico.f[nf][2] = (unsigned char)(out ? k : j);
        double nl = std::sqrt(nrm[0] * nrm[0] + nrm[1] * nrm[1] + nrm[2] * nrm[2]);
        inr = std::fabs(cen) / nl;
        ++nf;
      }
  for (int i = 0; i < 12; ++i)
    for (int a = 0; a < 3; ++a) ico.v[i][a] = (float)(v[i][a] / inr);
  return ico;
}

struct ScratchArena {
  char* base = nullptr;
  size_t cap = 0;
  size_t top = 0;      // bytes handed out from the arena
  size_t logical = 0;  // bytes handed out in total, overflow included
  size_t high = 0;     // largest `logical` seen
  int depth = 0;       // live Scratch objects
};

namespace {
std::mutex g_arena_lock;
std::map<std::pair<int, hipStream_t>, ScratchArena> g_arenas;
}  // namespace

Scratch::Scratch(hipStream_t s) : s_(s) {
  int dev = 0;
  (void)hipGetDevice(&dev);
  {
    std::lock_guard<std::mutex> g(g_arena_lock);
    arena_ = &g_arenas[{dev, s}];
  }
  mark_ = arena_->top;
  logical_mark_ = arena_->logical;
  ++arena_->depth;
}

grtx_status Scratch::raw(void** p, size_t bytes) {
  bytes = (bytes + 255) & ~(size_t)255;
  ScratchArena& a = *arena_;
  a.logical += bytes;
  a.high = std::max(a.high, a.logical);
  if (a.base && a.top + bytes <= a.cap) {
    *p = a.base + a.top;
    a.top += bytes;
    return GRTX_OK;
  }
  void* q = nullptr;
  GRTX_HIP(hipMallocAsync(&q, bytes, s_));
  extra_.push_back(q);
  *p = q;
  return GRTX_OK;
}

Scratch::~Scratch() {
  for (void* q : extra_) (void)hipFreeAsync(q, s_);
  ScratchArena& a = *arena_;
  a.top = mark_;
  a.logical = logical_mark_;
  if (--a.depth == 0 && a.high > a.cap) {
    if (a.base) (void)hipFreeAsync(a.base, s_);
    a.base = nullptr;
    a.cap = 0;
    const size_t want = a.high + a.high / 4;
    void* q = nullptr;
    if (hipMallocAsync(&q, want, s_) == hipSuccess) {
      a.base = static_cast<char*>(q);
      a.cap = want;
    } else {
      (void)hipGetLastError();
    }
  }
}

grtx_status build_bvh(const grtx_gaussians* g, grtx_bvh_kind kind, float alpha_min, bool restructure_tree,
                      int max_depth, hipStream_t s, Bvh* b) {
  b->kind = kind;
  b->n_gauss = g->count;
  b->sh_degree = g->sh_degree;
  b->alpha_min = alpha_min;
  b->opacities = g->opacities;
  b->sh = g->sh;
  b->build_stream = s;
  GRTX_HIP(hipGetDevice(&b->device));
  const bool proxy = kind == GRTX_BVH_PROXY20;
  const int64_t n = g->count;
  const int64_t m = proxy ? 20 * n : n;  // leaves
  b->n_leaves = m;
  if (n == 0) return GRTX_OK;
  GaussIn gi{g->means, g->scales, g->quats, g->opacities};
  const int64_t nint = m - 1;
  // node record positions: the top levels in [0, top_cap), then one block per subtree task
  // (a tree's nodes above kLayoutLeaves leaves can number up to m - 1 when it is lopsided)
  const int64_t top_cap = m > kLayoutLeaves ? m : 0;
  const int64_t node_slots = nint > 0 ? top_cap + m : 0;
  if (node_slots >= (int64_t)kLeafFlag) {
    set_error("build: %lld leaves exceed the node positions a record reference can hold", (long long)m);
    return GRTX_ERR_INVALID_ARG;
  }
  b->node_slots = node_slots;
  // every array the handle owns in one allocation (each hipMalloc costs host time per frame)
  auto layout = [&](auto&& put) {
    put(&b->codes, m);
    put(&b->perm, m);
    put(&b->child, 2 * std::max<int64_t>(nint, 1));
    put(&b->parent, 2 * m - 1);
    put(&b->boxes, 6 * (2 * m - 1));
    put(&b->nodes, kNodeF4 * std::max<int64_t>(node_slots, 1));
    put(&b->inst, 4 * n);
    if (proxy) put(&b->tris, 3 * m);
    put(&b->roots, 8);
    put(&b->cut, 2 * (int64_t)kCutCap);
    put(&b->n_cut, 1);
    put(&b->depth, 2);
    put(&b->density, kDensityCells);
    put(&b->dbox, 6);
  };
  size_t total = 0;
  layout([&](auto** p, int64_t count) {
    total = (total + 255) & ~(size_t)255;
    total += (size_t)std::max<int64_t>(count, 1) * sizeof(**p);
  });
  void* block = nullptr;
  GRTX_HIP(hipMalloc(&block, total));
  b->allocations.push_back(block);
  b->bytes += total;
  size_t off = 0;
  layout([&](auto** p, int64_t count) {
    off = (off + 255) & ~(size_t)255;
    *p = reinterpret_cast<std::remove_reference_t<decltype(*p)>>(static_cast<char*>(block) + off);
    off += (size_t)std::max<int64_t>(count, 1) * sizeof(**p);
  });
  b->root_box = b->boxes;  // node 0: the root, or the only leaf when m == 1

  Scratch sc(s);
  float *partial = nullptr, *bounds = nullptr, *cent = nullptr, *tbox = nullptr;
  float4* ttmp = nullptr;
  uint64_t* tkeys = nullptr;
  uint32_t *tvals = nullptr, *arrivals = nullptr;
  int nparts = (int)std::min<int64_t>(1024, (m + kBlock - 1) / kBlock);
  GRTX_TRY(sc.get(&partial, 6 * nparts));
  GRTX_TRY(sc.get(&bounds, 6));
  GRTX_TRY(sc.get(&tkeys, m));
  GRTX_TRY(sc.get(&tvals, m));
  uint2* range = nullptr;
  uint32_t* ready = nullptr;
  uint32_t* count = nullptr;  // leaves below each internal node
  float* sah = nullptr;       // surface-area cost of each node's subtree (restructuring)
  GRTX_TRY(sc.get(&arrivals, nint + 1));  // per internal node, then the ready-list length
  GRTX_TRY(sc.get(&range, std::max<int64_t>(nint, 1)));
  GRTX_TRY(sc.get(&ready, std::max<int64_t>(nint, 1)));
  GRTX_TRY(sc.get(&count, std::max<int64_t>(nint, 1)));
  const float* points = g->means;
  if (proxy) {
    GRTX_TRY(sc.get(&cent, 3 * m));
    GRTX_TRY(sc.get(&tbox, 6 * m));
    GRTX_TRY(sc.get(&ttmp, 3 * m));
    static const Ico ico = make_icosahedron();
    hipLaunchKernelGGL(k_proxy_setup, dim3(grid_for(n)), dim3(kBlock), 0, s, gi, n, alpha_min, ico, b->inst, ttmp,
                       tbox, cent);
    points = cent;
  }
  hipLaunchKernelGGL(k_bounds_partial, dim3(nparts), dim3(kBlock), 0, s, points, m, partial);
  hipLaunchKernelGGL(k_bounds_final, dim3(1), dim3(kBlock), 0, s, partial, nparts, bounds);
  hipLaunchKernelGGL(k_morton, dim3(grid_for(m)), dim3(kBlock), 0, s, points, m, bounds, b->codes, b->perm);
  GRTX_LAUNCH_CHECK();
  GRTX_TRY(radix_sort(b->codes, b->perm, tkeys, tvals, m, sc, s));
  // leaves per cell of the density grid, over the leaf centres' bounds (in sorted order, so
  // that a thread's leaves mostly share a cell)
  GRTX_HIP(hipMemcpyAsync(b->dbox, bounds, 6 * sizeof(float), hipMemcpyDeviceToDevice, s));
  hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(kDensityCells)), dim3(kBlock), 0, s, b->density, (int64_t)kDensityCells,
                     0u);
  hipLaunchKernelGGL(k_density, dim3(grid_for((m + kDensityRun - 1) / kDensityRun)), dim3(kBlock), 0, s, points,
                     b->perm, m, bounds, b->density);
  if (proxy) {
    hipLaunchKernelGGL(k_proxy_leaves, dim3(grid_for(m)), dim3(kBlock), 0, s, b->perm, m, ttmp, tbox, b->tris,
                       b->boxes);
  } else {
    float box_scale = 1.f;
    if (kind == GRTX_BVH_ICO_INSTANCE) {
      static const Ico ico = make_icosahedron();
      box_scale = std::sqrt(ico.v[0][0] * ico.v[0][0] + ico.v[0][1] * ico.v[0][1] + ico.v[0][2] * ico.v[0][2]);
    }
    hipLaunchKernelGGL(k_sphere_leaves, dim3(grid_for(m)), dim3(kBlock), 0, s, gi, b->perm, m, alpha_min, box_scale,
                       b->inst, b->boxes);
  }
  if (nint > 0) {
    hipLaunchKernelGGL(k_karras, dim3(grid_for(nint)), dim3(kBlock), 0, s, b->codes, m, b->child, b->parent,
                       range, count, arrivals);
    hipLaunchKernelGGL(k_refit_small, dim3(grid_for(nint)), dim3(kBlock), 0, s, m, b->child, range, b->boxes,
                       ready, arrivals + nint, refit_small_limit(m));
    hipLaunchKernelGGL(k_refit_top, dim3(1), dim3(kTopBlock), 0, s, m, b->child, b->parent, range, b->boxes,
                       ready, arrivals + nint, arrivals, refit_small_limit(m));
    const bool restructure = restructure_tree && nint > 1 && 2 * m - 1 <= (int64_t)kScanChunk * kScanChunk;
    PlainTree saved{};
    if (restructure) {
      // keep the plain tree in case the restructured one comes out too deep
      uint32_t *sc_child = nullptr, *sc_parent = nullptr, *sc_count = nullptr;
      float* sc_boxes = nullptr;
      GRTX_TRY(sc.get(&sc_child, 2 * nint));
      GRTX_TRY(sc.get(&sc_parent, 2 * m - 1));
      GRTX_TRY(sc.get(&sc_boxes, 6 * nint));
      GRTX_TRY(sc.get(&sc_count, nint));
      GRTX_HIP(hipMemcpyAsync(sc_child, b->child, sizeof(uint32_t) * 2 * nint, hipMemcpyDeviceToDevice, s));
      GRTX_HIP(hipMemcpyAsync(sc_parent, b->parent, sizeof(uint32_t) * (2 * m - 1), hipMemcpyDeviceToDevice, s));
      GRTX_HIP(hipMemcpyAsync(sc_boxes, b->boxes, sizeof(float) * 6 * nint, hipMemcpyDeviceToDevice, s));
      GRTX_HIP(hipMemcpyAsync(sc_count, count, sizeof(uint32_t) * nint, hipMemcpyDeviceToDevice, s));
      saved = PlainTree{sc_child, sc_parent, sc_boxes, sc_count};
    }
    if (restructure) {
      const int64_t nn = 2 * m - 1;
      uint32_t *rflag = nullptr, *rpos = nullptr, *roots = nullptr, *nroots = nullptr;
      GRTX_TRY(sc.get(&sah, nn));
      GRTX_TRY(sc.get(&rflag, nn));
      GRTX_TRY(sc.get(&rpos, nn));
      GRTX_TRY(sc.get(&roots, m));
      GRTX_TRY(sc.get(&nroots, 2));  // count, then the work queue
      const int ns = subtree_leaves(m);
      hipLaunchKernelGGL(k_cut_flags, dim3(grid_for(nn)), dim3(kBlock), 0, s, nn, nint, b->parent, count,
                         (uint32_t)ns, rflag);
      GRTX_TRY(exclusive_scan_u32(rflag, rpos, nn, s));
      hipLaunchKernelGGL(k_subtree_roots, dim3(grid_for(nn)), dim3(kBlock), 0, s, nn, rflag, rpos, roots, nroots);
      hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(kBlock), 0, s, nroots + 1, 1, 0u);
      int dev = 0, cus = 0;
      GRTX_HIP(hipGetDevice(&dev));
      GRTX_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
      // workgroups: four per CU at 256 threads, eight at 128 (the queue hands out subtrees)
      const unsigned groups = (unsigned)std::max(1, 4 * cus * (256 / ns));
      // a subtree keeps its root, its leaves and its set of internal nodes through a pass, so
      // later passes take the same roots (the queue is reset for each)
      for (int pass = 0; pass < treelet_passes(m); ++pass) {
        const uint32_t min_leaves = pass == 0 ? 0u : kLaterPassLeaves << (pass - 1);
        if (pass > 0) hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(kBlock), 0, s, nroots + 1, 1, 0u);
        if (ns == 256)
          hipLaunchKernelGGL(k_treelet<256>, dim3(groups), dim3(256), 0, s, m, roots, nroots, nroots + 1, range,
                             b->child, b->parent, b->boxes, sah, count, min_leaves);
        else
          hipLaunchKernelGGL(k_treelet<128>, dim3(groups), dim3(128), 0, s, m, roots, nroots, nroots + 1, range,
                             b->child, b->parent, b->boxes, sah, count, min_leaves);
      }
      if (m > kTopPassLeaves) {
        hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(nint + 1)), dim3(kBlock), 0, s, arrivals, nint + 1, 0u);
        const unsigned top_groups = (unsigned)((m + ns - 1) / ns);
        if (ns == 256)
          hipLaunchKernelGGL(k_treelet_top<256>, dim3(top_groups), dim3(256), 0, s, m, roots, nroots, b->child,
                             b->parent, b->boxes, sah, count, arrivals);
        else
          hipLaunchKernelGGL(k_treelet_top<128>, dim3(top_groups), dim3(128), 0, s, m, roots, nroots, b->child,
                             b->parent, b->boxes, sah, count, arrivals);
      }
    }
    // depth of the tree (the refit's arrival counters are free again and hold the heights)
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(nint)), dim3(kBlock), 0, s, arrivals, nint, 0u);
    hipLaunchKernelGGL(k_tree_height, dim3(grid_for(m)), dim3(kBlock), 0, s, m, b->parent, arrivals,
                       restructure ? max_depth : GRTX_MAX_TREE_DEPTH, (const uint32_t*)nullptr);
    uint32_t *deep = nullptr, *h2 = nullptr;
    if (restructure) {
      GRTX_TRY(sc.get(&deep, 1));
      GRTX_TRY(sc.get(&h2, nint));
      hipLaunchKernelGGL(k_restore_plain, dim3(grid_for(2 * m - 1)), dim3(kBlock), 0, s, m, arrivals, max_depth, saved,
                         b->child, b->parent, b->boxes, count, h2, deep);
      hipLaunchKernelGGL(k_tree_height, dim3(grid_for(m)), dim3(kBlock), 0, s, m, b->parent, h2, GRTX_MAX_TREE_DEPTH,
                         deep);
    }
    hipLaunchKernelGGL(k_depth_store, dim3(1), dim3(64), 0, s, arrivals, deep, h2, b->depth);
    // four-wide records of every internal node, then the reachable ones laid out
    float4* wide = nullptr;
    uint32_t *qold = nullptr, *ctr = nullptr;
    uint2* tasks = nullptr;
    GRTX_TRY(sc.get(&wide, kNodeF4 * nint));
    GRTX_TRY(sc.get(&qold, node_slots));
    GRTX_TRY(sc.get(&tasks, m));
    GRTX_TRY(sc.get(&ctr, 2));
    hipLaunchKernelGGL(k_wide, dim3(grid_for(nint)), dim3(kBlock), 0, s, m, b->child, b->boxes, wide);
    hipLaunchKernelGGL(k_layout_top, dim3(1), dim3(kLayoutBlock), 0, s, m, wide, count, (uint32_t)top_cap, b->nodes,
                       qold, tasks, ctr);
    // a wave per task; the tasks number about m / 64 (a grid-stride loop takes any more)
    hipLaunchKernelGGL(k_layout_tasks, dim3((unsigned)std::min<int64_t>(2048, m / (64 * (kBlock / 64)) + 1)),
                       dim3(kBlock), 0, s, wide, tasks, ctr, b->nodes);
  } else {
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(kBlock), 0, s, b->parent, 1, kNoParent);
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(kBlock), 0, s, b->depth, 2, 0u);
  }
  hipLaunchKernelGGL(k_write_root, dim3(1), dim3(64), 0, s, b->root_box, m == 1 ? (kLeafFlag | 0u) : 0u, b->roots);
  if (2 * m - 1 > (int64_t)kScanChunk * kScanChunk) {
    // beyond one scan's reach: no cut, the trace keeps its centre-out order
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(kBlock), 0, s, b->n_cut, 1, 0u);
  } else {
    const int64_t nn = 2 * m - 1;
    uint32_t *cflag = nullptr, *cpos = nullptr;
    GRTX_TRY(sc.get(&cflag, nn));
    GRTX_TRY(sc.get(&cpos, nn));
    const uint32_t cut = (uint32_t)std::max<int64_t>(1, m / kCutDiv);
    hipLaunchKernelGGL(k_cut_flags, dim3(grid_for(nn)), dim3(kBlock), 0, s, nn, nint, b->parent, count, cut, cflag);
    GRTX_TRY(exclusive_scan_u32(cflag, cpos, nn, s));
    hipLaunchKernelGGL(k_cut_write, dim3(grid_for(nn)), dim3(kBlock), 0, s, nn, nint, cflag, cpos, count, b->boxes,
                       b->cut, b->n_cut);
  }
  GRTX_LAUNCH_CHECK();
  return GRTX_OK;
}

grtx_status export_topology(const Bvh* b, uint32_t* child, uint32_t* parent, uint64_t* morton, uint32_t* perm,
                            float* boxes, hipStream_t s) {
  const int64_t n = b->n_leaves;
  if (n == 0) return GRTX_OK;
  const int64_t nint = n - 1;
  if (child && nint > 0) GRTX_HIP(hipMemcpyAsync(child, b->child, sizeof(uint32_t) * 2 * nint, hipMemcpyDeviceToDevice, s));
  if (parent) GRTX_HIP(hipMemcpyAsync(parent, b->parent, sizeof(uint32_t) * (2 * n - 1), hipMemcpyDeviceToDevice, s));
  if (morton) GRTX_HIP(hipMemcpyAsync(morton, b->codes, sizeof(uint64_t) * n, hipMemcpyDeviceToDevice, s));
  if (perm) GRTX_HIP(hipMemcpyAsync(perm, b->perm, sizeof(uint32_t) * n, hipMemcpyDeviceToDevice, s));
  if (boxes) GRTX_HIP(hipMemcpyAsync(boxes, b->boxes, sizeof(float) * 6 * (2 * n - 1), hipMemcpyDeviceToDevice, s));
  return GRTX_OK;
}

grtx_status pinhole_rays(const grtx_camera* cam, float* origins, float* dirs, hipStream_t s) {
  CameraFrame cf;
  if (!camera_frame(cam->eye, cam->target, cam->up, cam->fov_y_deg, cam->width, cam->height, &cf)) {
    set_error("pinhole camera: degenerate eye/target/up");
    return GRTX_ERR_INVALID_ARG;
  }
  int64_t n = (int64_t)cam->width * cam->height;
  hipLaunchKernelGGL(k_pinhole, dim3(grid_for(n)), dim3(kBlock), 0, s, cf, cam->width, cam->height, origins, dirs);
  GRTX_LAUNCH_CHECK();
  return GRTX_OK;
}

grtx_status exclusive_scan_u32(const uint32_t* in, uint32_t* out, int64_t n, hipStream_t s) {
  if (n <= 0) return GRTX_OK;
  Scratch sc(s);
  const int nparts = (int)((n + kScanChunk - 1) / kScanChunk);
  if (nparts > kScanChunk) {
    set_error("scan: %lld values exceed the supported size", (long long)n);
    return GRTX_ERR_INVALID_ARG;
  }
  if (nparts > 1 && nparts <= kScanLoopChunks) {
    hipLaunchKernelGGL(k_scan_loop, dim3(1), dim3(kBlock), 0, s, in, n, out);
  } else if (nparts > 1) {
    uint32_t* part = nullptr;
    GRTX_TRY(sc.get(&part, nparts));
    hipLaunchKernelGGL(k_scan_reduce, dim3(nparts), dim3(kBlock), 0, s, in, n, part);
    hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(kBlock), 0, s, part, nparts);
    hipLaunchKernelGGL(k_scan_down, dim3(nparts), dim3(kBlock), 0, s, in, n, part, out);
  } else {
    hipLaunchKernelGGL(k_scan_down, dim3(1), dim3(kBlock), 0, s, in, n, (const uint32_t*)nullptr, out);
  }
  GRTX_LAUNCH_CHECK();
  return GRTX_OK;
}

grtx_status sort_by_key_into(uint64_t* keys, uint32_t* vals, uint64_t* tkeys, uint32_t* tvals, int64_t n,
                             int key_bits, hipStream_t s, const uint32_t* n_dev, uint64_t** kres, uint32_t** vres) {
  *kres = keys;
  *vres = vals;
  if (n <= 1) return GRTX_OK;
  Scratch sc(s);
  const int passes = std::max(1, std::min(8, (key_bits + 7) / 8));
  return radix_sort(keys, vals, tkeys, tvals, n, sc, s, passes, n_dev, kres, vres);
}

grtx_status sort_by_key(uint64_t* keys, uint32_t* vals, int64_t n, int key_bits, hipStream_t s,
                        const uint32_t* n_dev) {
  if (n <= 1) return GRTX_OK;
  Scratch sc(s);
  uint64_t* tkeys = nullptr;
  uint32_t* tvals = nullptr;
  GRTX_TRY(sc.get(&tkeys, n));
  GRTX_TRY(sc.get(&tvals, n));
  const int passes = std::max(1, std::min(8, (key_bits + 7) / 8));
  return radix_sort(keys, vals, tkeys, tvals, n, sc, s, passes, n_dev);
}

}  // namespace grtx
