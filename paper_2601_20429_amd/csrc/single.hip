// Single-round tracing: the alternative to multi-round k-buffer tracing that the paper
// weighs it against (Sec. III-C, Observation II). One traversal per ray collects every hit,
// unsorted and without early termination, into a list; the list is then sorted and blended
// front to back with early termination.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "grtx_internal.h"
#include "trace_common.h"

namespace grtx {
namespace {

__global__ void k_zero_counter(unsigned int* c) {
  if (threadIdx.x == 0) *c = 0u;
}

// The single-round alternative to the k-buffer rounds (Sec. III-C, Observation II): one
// traversal collects every hit of a ray, unsorted and without early termination, into a
// list of `cap` keys; then the list is sorted and blended front to back with early
// termination. Collection: persistent waves as in k_trace, without t_max (every box the
// ray crosses beyond t_near is entered). A ray with more hits than `cap` keeps the first
// `cap` in traversal order, which need not be the closest: its result is incomplete, and
// its GRTX_STAT_FALLBACKS counter is set to 1.
struct CollectArgs {
  const float4* nodes;
  const float4* inst;
  const float* roots;
  const float* ray_o;
  const float* ray_d;
  int64_t ray0;      // first ray of this chunk
  int64_t n_rays;    // rays in this chunk
  float t_near;
  int cap;
  uint64_t* keys;    // [n_rays][cap], chunk-local
  uint32_t* counts;  // [n_rays], all hits (may exceed cap)
  uint32_t* stats;   // [R][GRTX_STATS_FIELDS] or null (global ray index)
  uint2* spill;      // per wave: [kSpillRows][64]
  unsigned int* counter;
};

__global__ void __launch_bounds__(kTraceBlock) k_collect(CollectArgs A) {
  __shared__ uint2 s_stack[kLdsStack * kTraceBlock];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const uint64_t lt_mask = lane ? (~0ull >> (64 - lane)) : 0ull;
  const int64_t gwave = (blockIdx.x * (int64_t)kTraceBlock + tid) >> 6;
  uint2* const spill = A.spill + gwave * (int64_t)kSpillRows * 64 + lane;
  bool live = false, exhausted = false;
  int64_t ray = 0;
  float ox = 0, oy = 0, oz = 0, dx = 0, dy = 0, dz = 0, ix = 0, iy = 0, iz = 0, oix = 0, oiy = 0, oiz = 0;
  uint32_t cur_ref = 0, n_hits = 0, n_nodes = 0, n_leaves = 0;
  float cur_t = 0;
  bool has_cur = false;
  int sp = 0;
  while (true) {
    if (!exhausted) {
      const uint64_t idle = __ballot(!live);
      if (idle) {
        const int leader = __ffsll((unsigned long long)idle) - 1;
        unsigned int base = 0;
        if (lane == leader) base = atomicAdd(A.counter, (unsigned int)__popcll(idle));
        base = __shfl(base, leader);
        if ((int64_t)base >= A.n_rays) exhausted = true;
        if (!live) {
          const int64_t r = (int64_t)base + __popcll(idle & lt_mask);
          if (r < A.n_rays) {
            ray = r;
            const float* ro = A.ray_o + 3 * (A.ray0 + r);
            const float* rd = A.ray_d + 3 * (A.ray0 + r);
            ox = ro[0]; oy = ro[1]; oz = ro[2];
            dx = rd[0]; dy = rd[1]; dz = rd[2];
            ix = safe_inv(dx); iy = safe_inv(dy); iz = safe_inv(dz);
            oix = ox * ix; oiy = oy * iy; oiz = oz * iz;
            const Slab sb = slab(A.roots[0], A.roots[1], A.roots[2], A.roots[3], A.roots[4], A.roots[5], ox, oy, oz,
                                 ix, iy, iz);
            has_cur = sb.tn <= sb.tf && sb.tf >= A.t_near;
            cur_ref = __float_as_uint(A.roots[6]);
            cur_t = sb.tn;
            sp = 0;
            n_hits = n_nodes = n_leaves = 0;
            live = true;
          }
        }
      }
    }
    if (__ballot(live) == 0) {
      if (exhausted) break;
      continue;
    }
    // one node step and one leaf step per iteration, as in k_trace
    if (live && !has_cur) {
      if (sp > 0) {
        --sp;
        const uint2 e = sp < kLdsStack ? s_stack[sp * kTraceBlock + tid] : spill[(int64_t)(sp - kLdsStack) * 64];
        cur_ref = e.x;
        cur_t = __uint_as_float(e.y);
        has_cur = true;
      } else {
        A.counts[ray] = n_hits;
        if (A.stats) {
          uint32_t* st = A.stats + (A.ray0 + ray) * GRTX_STATS_FIELDS;
          st[GRTX_STAT_NODES] = n_nodes;
          st[GRTX_STAT_LEAVES] = n_leaves;
        }
        live = false;
      }
    }
    if (live && has_cur && !(cur_ref & kLeafFlag)) {
      const float4* np = A.nodes + kNodeF4 * (int64_t)cur_ref;
      const float4 q0 = np[0], q1 = np[1], q2 = np[2], q3 = np[3];
      ++n_nodes;
      const float Ax = q0.w * ix, Ay = q1.x * iy, Az = q1.y * iz;
      const float Bx = fmaf(q0.x, ix, -oix), By = fmaf(q0.y, iy, -oiy), Bz = fmaf(q0.z, iz, -oiz);
      const uint32_t wlx = __float_as_uint(q2.z), wly = __float_as_uint(q2.w), wlz = __float_as_uint(q3.x);
      const uint32_t whx = __float_as_uint(q3.y), why = __float_as_uint(q3.z), whz = __float_as_uint(q3.w);
      const uint32_t wnx = ix < 0.f ? whx : wlx, wfx = ix < 0.f ? wlx : whx;
      const uint32_t wny = iy < 0.f ? why : wly, wfy = iy < 0.f ? wly : why;
      const uint32_t wnz = iz < 0.f ? whz : wlz, wfz = iz < 0.f ? wlz : whz;
      const uint32_t c[4] = {__float_as_uint(q1.z), __float_as_uint(q1.w), __float_as_uint(q2.x),
                             __float_as_uint(q2.y)};
      has_cur = false;
      const float pt = cur_t;  // entry of the node in hand
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const float tn = fmaxf(fmaxf(fmaf((float)((wnx >> (8 * j)) & 0xFFu), Ax, Bx),
                                     fmaf((float)((wny >> (8 * j)) & 0xFFu), Ay, By)),
                               fmaf((float)((wnz >> (8 * j)) & 0xFFu), Az, Bz));
        const float tf = fminf(fminf(fmaf((float)((wfx >> (8 * j)) & 0xFFu), Ax, Bx),
                                     fmaf((float)((wfy >> (8 * j)) & 0xFFu), Ay, By)),
                               fmaf((float)((wfz >> (8 * j)) & 0xFFu), Az, Bz));
        // the same entry distances as k_trace's (raised to the entry of the node in hand)
        const float te = fmaxf(tn, pt);
        if (c[j] != kNoChild && fmaxf(tn, A.t_near) <= tf) {
          if (!has_cur) {
            cur_ref = c[j];
            cur_t = te;
            has_cur = true;
          } else {
            const uint2 e = make_uint2(c[j], __float_as_uint(te));
            if (sp < kLdsStack)
              s_stack[sp * kTraceBlock + tid] = e;
            else if (sp < kMaxStack)
              spill[(int64_t)(sp - kLdsStack) * 64] = e;
            sp = sp < kMaxStack ? sp + 1 : sp;
          }
        }
      }
    }
    if (live && has_cur && (cur_ref & kLeafFlag)) {
      const uint32_t p = cur_ref & ~kLeafFlag;
      has_cur = false;
      ++n_leaves;
      const float4* ip = A.inst + 4 * (int64_t)p;
      const SphereHit h = sphere_terms(ip[0], ip[1], ip[2], ox, oy, oz, dx, dy, dz);
      if (h.a > 0.f && h.c2 <= h.a) {
        const float t0 = (-h.b - __builtin_amdgcn_sqrtf(fmaxf(h.a - h.c2, 0.f))) * __builtin_amdgcn_rcpf(h.a);
        if (t0 > A.t_near) {
          if (n_hits < (uint32_t)A.cap) A.keys[ray * A.cap + n_hits] = make_key(fmaxf(t0, cur_t), p);
          ++n_hits;
        }
      }
    }
  }
}

// Sort and blend: one wave per ray. The keys go through LDS (padded with the empty key to
// a power of two) and a bitonic sort; then, 64 hits at a time, each lane computes its
// hit's alpha, depth and colour as k_trace's blend does, and the accumulation runs over
// the 64 in key order with k_trace's expressions (the compiler may round them apart by
// contracting differently in the two kernels).
struct BlendArgs {
  const float4* inst;
  const float* sh;
  int sh_degree;
  const float* ray_o;
  const float* ray_d;
  int64_t ray0;
  int cap;
  int cap_pow2;
  const uint64_t* keys;
  const uint32_t* counts;
  float T_min;
  float bg0, bg1, bg2;
  float* rgb;
  float* depth;
  float* opac;
  uint32_t* stats;
  int32_t* hit_ids;
  int32_t* hit_counts;
  int hit_cap;
};

__global__ void __launch_bounds__(64) k_sort_blend(BlendArgs A) {
  extern __shared__ uint64_t s_keys[];
  const int lane = threadIdx.x;
  const int64_t r = blockIdx.x;
  const int64_t gr = A.ray0 + r;
  const uint32_t total = A.counts[r];
  const int n = (int)min(total, (uint32_t)A.cap);
  int P = 64;
  while (P < n) P <<= 1;
  for (int j = lane; j < P; j += 64) s_keys[j] = j < n ? A.keys[r * A.cap + j] : kEmptyKey;
  __syncthreads();
  for (int size = 2; size <= P; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int j = lane; j < P; j += 64) {
        const int o = j ^ stride;
        if (o > j) {
          const bool up = (j & size) == 0;
          const uint64_t a = s_keys[j], b = s_keys[o];
          if ((a > b) == up) {
            s_keys[j] = b;
            s_keys[o] = a;
          }
        }
      }
      __syncthreads();
    }
  }
  const float ox = A.ray_o[3 * gr], oy = A.ray_o[3 * gr + 1], oz = A.ray_o[3 * gr + 2];
  const float dx = A.ray_d[3 * gr], dy = A.ray_d[3 * gr + 1], dz = A.ray_d[3 * gr + 2];
  const int ncoef = (A.sh_degree + 1) * (A.sh_degree + 1);
  float T = 1.f, C0 = 0.f, C1 = 0.f, C2 = 0.f, Dp = 0.f;
  int nblend = 0;
  bool ert = false;
  for (int base = 0; base < n && !ert; base += 64) {
    const int j = base + lane;
    float alpha = 0.f, talpha = 0.f, c[3] = {0.5f, 0.5f, 0.5f};
    uint32_t gid = 0;
    if (j < n) {
      const uint32_t p = (uint32_t)s_keys[j];
      const float4* ip = A.inst + 4 * (int64_t)p;
      const float4 r0 = ip[0], r1 = ip[1], r2 = ip[2], r3 = ip[3];
      const SphereHit h = sphere_terms(r0, r1, r2, ox, oy, oz, dx, dy, dz);
      const float inva = __builtin_amdgcn_rcpf(h.a);
      const float cperp = h.c2 * inva;
      talpha = -h.b * inva;
      alpha = r3.x * __builtin_amdgcn_exp2f(-r3.y * cperp);
      gid = __float_as_uint(r3.z);
      const float dn = rsqrtf(dx * dx + dy * dy + dz * dz);
      float Y[16];
      sh_basis(dx * dn, dy * dn, dz * dn, A.sh_degree, Y);
      if (A.sh_degree == 3) {
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
    }
    const int m = min(64, n - base);
    for (int q = 0; q < m; ++q) {  // wave-uniform: every lane runs the same accumulation
      const float a = __shfl(alpha, q), ta = __shfl(talpha, q);
      const float k0 = __shfl(c[0], q), k1 = __shfl(c[1], q), k2 = __shfl(c[2], q);
      const float w = T * a;
      C0 += w * fmaxf(k0, 0.f);
      C1 += w * fmaxf(k1, 0.f);
      C2 += w * fmaxf(k2, 0.f);
      Dp += w * ta;
      T *= (1.f - a);
      if (A.hit_ids && lane == q && nblend < A.hit_cap) A.hit_ids[gr * A.hit_cap + nblend] = (int32_t)gid;
      ++nblend;
      if (T < A.T_min) {
        ert = true;
        break;
      }
    }
  }
  if (lane == 0) {
    A.rgb[3 * gr + 0] = C0 + T * A.bg0;
    A.rgb[3 * gr + 1] = C1 + T * A.bg1;
    A.rgb[3 * gr + 2] = C2 + T * A.bg2;
    A.depth[gr] = Dp;
    A.opac[gr] = 1.f - T;
    if (A.hit_counts) A.hit_counts[gr] = nblend;
    if (A.stats) {
      uint32_t* st = A.stats + gr * GRTX_STATS_FIELDS;
      st[GRTX_STAT_ROUNDS] = 1u;
      st[GRTX_STAT_BLENDED] = (uint32_t)nblend;
      for (int f = GRTX_STAT_DEFERRED; f < GRTX_STATS_FIELDS; ++f) st[f] = 0u;
      st[GRTX_STAT_FALLBACKS] = total > (uint32_t)A.cap ? 1u : 0u;  // the list overflowed
    }
  }
}

}  // namespace

// Single-round tracing (the baseline of Sec. III-C, Observation II): collect, then sort
// and blend, in chunks of rays whose lists fit kCollectChunkBytes of scratch.
constexpr size_t kCollectChunkBytes = (size_t)8 << 30;
constexpr int kCollectDefaultCap = 2048;
constexpr int kCollectMaxCap = 8192;  // the sort's LDS: 8 B per padded key, 64 KB at most

grtx_status trace_single_round(const TraceScene& b, const grtx_rays* r, const grtx_trace_params* p,
                               const grtx_trace_outputs* o, hipStream_t s) {
  if (b.kind != GRTX_BVH_SPHERE_INSTANCE || b.ray_scene) {
    set_error("grtx_trace: single-round mode takes one unit-sphere instance structure");
    return GRTX_ERR_INVALID_ARG;
  }
  if (r->t_far || r->transmittance || r->kind) {
    set_error("grtx_trace: single-round mode takes unbounded rays that start with transmittance 1");
    return GRTX_ERR_INVALID_ARG;
  }
  const int64_t R = r->count;
  const int cap = p->collect_capacity > 0 ? p->collect_capacity : kCollectDefaultCap;
  if (cap > kCollectMaxCap) {
    set_error("grtx_trace: collect_capacity %d exceeds %d", cap, kCollectMaxCap);
    return GRTX_ERR_INVALID_ARG;
  }
  int P2 = 64;
  while (P2 < cap) P2 <<= 1;
  int device = 0, cus = 0, nb = 0;
  GRTX_HIP(hipGetDevice(&device));
  GRTX_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device));
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_collect, kTraceBlock, 0) != hipSuccess) nb = 1;
  const int64_t chunk = std::max<int64_t>(1, std::min<int64_t>(R, (int64_t)(kCollectChunkBytes / (8 * (size_t)cap))));
  const int64_t blocks = std::min<int64_t>((int64_t)cus * std::max(1, nb), (chunk + kTraceBlock - 1) / kTraceBlock);
  Scratch sc(s);
  uint64_t* keys = nullptr;
  uint32_t *counts = nullptr, *counter = nullptr;
  uint2* spill = nullptr;
  GRTX_TRY(sc.get(&keys, chunk * (int64_t)cap));
  GRTX_TRY(sc.get(&counts, chunk));
  GRTX_TRY(sc.get(&counter, 64));
  GRTX_TRY(sc.get(&spill, blocks * kWaves * (int64_t)kSpillRows * 64));
  CollectArgs ca{};
  ca.nodes = b.nodes;
  ca.inst = b.inst;
  ca.roots = b.roots;
  ca.ray_o = r->origins;
  ca.ray_d = r->dirs;
  ca.t_near = r->t_near;
  ca.cap = cap;
  ca.keys = keys;
  ca.counts = counts;
  ca.stats = o->stats;
  ca.spill = spill;
  ca.counter = counter;
  BlendArgs ba{};
  ba.inst = b.inst;
  ba.sh = b.sh;
  ba.sh_degree = b.sh_degree;
  ba.ray_o = r->origins;
  ba.ray_d = r->dirs;
  ba.cap = cap;
  ba.cap_pow2 = P2;
  ba.keys = keys;
  ba.counts = counts;
  ba.T_min = p->T_min;
  ba.bg0 = p->bg[0];
  ba.bg1 = p->bg[1];
  ba.bg2 = p->bg[2];
  ba.rgb = o->rgb;
  ba.depth = o->depth;
  ba.opac = o->opacity;
  ba.stats = o->stats;
  ba.hit_ids = o->hit_ids;
  ba.hit_counts = o->hit_counts;
  ba.hit_cap = o->hit_ids ? o->hit_capacity : 0;
  for (int64_t c0 = 0; c0 < R; c0 += chunk) {
    const int64_t n = std::min(chunk, R - c0);
    ca.ray0 = ba.ray0 = c0;
    ca.n_rays = n;
    hipLaunchKernelGGL(k_zero_counter, dim3(1), dim3(64), 0, s, counter);
    hipLaunchKernelGGL(k_collect, dim3((unsigned)std::min<int64_t>(blocks, (n + kTraceBlock - 1) / kTraceBlock)),
                       dim3(kTraceBlock), 0, s, ca);
    hipLaunchKernelGGL(k_sort_blend, dim3((unsigned)n), dim3(64), (size_t)P2 * sizeof(uint64_t), s, ba);
    GRTX_LAUNCH_CHECK();
  }
  return GRTX_OK;
}

}  // namespace grtx
