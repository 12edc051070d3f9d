// Backward pass of the Gaussian ray tracer for gfx950.
//
// The forward image of a ray is front-to-back compositing (Eq. 1) of its blended hits,
// in blend order, with alpha at the point of maximum response (Eq. 2) and colour from
// SH at the ray direction:
//   C = sum_i T_i a_i c_i + T_N bg,   D = sum_i T_i a_i t_i,   O = 1 - T_N,
//   T_i = prod_{j<i} (1 - a_j).
// With S_i = sum_{j>i} T_j a_j c_j + T_N bg (everything behind hit i):
//   dC/dc_i = T_i a_i,  dC/da_i = T_i c_i - S_i / (1 - a_i),
//   dD/dt_i = T_i a_i,  dD/da_i = T_i t_i - (sum_{j>i} T_j a_j t_j) / (1 - a_i),
//   dO/da_i = T_N / (1 - a_i).
// The suffix sums come from the forward outputs (C, D, T_N) minus running prefix sums,
// so one pass in blend order suffices. Per hit, with M = S^-1 R^T, f = o - mu,
// u = M f, v = M d, t = -(u.v)/(v.v), p = u + t v (closest approach in the whitened
// frame), m2 = |p|^2 and a = opacity * exp(-m2/2):
//   dm2/du = 2p, dm2/dv = 2 t p, dt/du = -v/(v.v), dt/dv = -(u + 2 t v)/(v.v),
//   dL/dM = g_u f^T + g_v d^T, dL/dmu = -M^T g_u, dL/ds_i = -(1/s_i) sum_j g_M[i][j] M[i][j],
//   dL/dR[j][i] = g_M[i][j] / s_i, then through R(q/|q|) to q; dL/do = dL/da * a / o;
//   dL/dsh[l,m,ch] = dL/dc_ch * [c_ch > 0] * Y_lm(d).
// The sum over rays is done without atomics and in a fixed order: a first kernel writes
// one 64-byte record per (ray, blended hit) with the hit's gradients of mean, scale,
// rotation and opacity and the three colour factors dL/dc * T a [c > 0]; the records
// are sorted by Gaussian (stable radix sort, so ray order is kept inside a Gaussian);
// one wave per Gaussian then sums its records (dL/dsh = colour factor x Y(ray direction))
// and adds the totals to the caller's arrays. Results are deterministic.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "grtx_internal.h"

namespace grtx {
namespace {

constexpr int kBlock = 128;

constexpr double cx_sqrt(double x) {
  double r = x > 1.0 ? x : 1.0;
  for (int i = 0; i < 100; ++i) r = 0.5 * (r + x / r);
  return r;
}
constexpr double kPi = 3.14159265358979323846;
// K_l^m = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!)
constexpr double Klm(int l, double fac_ratio) { return cx_sqrt((2.0 * l + 1.0) / (4.0 * kPi) * fac_ratio); }
constexpr float B00 = (float)Klm(0, 1.0);
constexpr float B1 = (float)Klm(1, 1.0);
constexpr float B20 = (float)(Klm(2, 1.0) * 0.5);
constexpr float B21 = (float)(cx_sqrt(2.0) * Klm(2, 1.0 / 6.0) * 3.0);
constexpr float B22 = (float)(cx_sqrt(2.0) * Klm(2, 1.0 / 24.0) * 3.0);
constexpr float B30 = (float)(Klm(3, 1.0) * 0.5);
constexpr float B31 = (float)(cx_sqrt(2.0) * Klm(3, 1.0 / 12.0) * 0.5);
constexpr float B32 = (float)(cx_sqrt(2.0) * Klm(3, 1.0 / 120.0) * 15.0);
constexpr float B33 = (float)(cx_sqrt(2.0) * Klm(3, 1.0 / 720.0) * 15.0);

// Real SH basis (orthonormal, Condon-Shortley phase) as polynomials of the unit direction.
__device__ __forceinline__ void basis(float x, float y, float z, int L, float* Y) {
  Y[0] = B00;
  if (L < 1) return;
  Y[1] = -B1 * y;
  Y[2] = B1 * z;
  Y[3] = -B1 * x;
  if (L < 2) return;
  const float xx = x * x, yy = y * y, zz = z * z;
  Y[4] = B22 * 2.f * x * y;
  Y[5] = -B21 * y * z;
  Y[6] = B20 * (3.f * zz - 1.f);
  Y[7] = -B21 * x * z;
  Y[8] = B22 * (xx - yy);
  if (L < 3) return;
  Y[9] = -B33 * (3.f * xx * y - yy * y);
  Y[10] = B32 * 2.f * x * y * z;
  Y[11] = -B31 * y * (15.f * zz - 3.f);
  Y[12] = B30 * (5.f * zz * z - 3.f * z);
  Y[13] = -B31 * x * (15.f * zz - 3.f);
  Y[14] = B32 * z * (xx - yy);
  Y[15] = -B33 * (xx * x - 3.f * x * yy);
}

struct BwdArgs {
  const float* means;
  const float* scales;
  const float* quats;
  const float* opac;
  const float* sh;
  int sh_degree;
  const float* ray_o;
  const float* ray_d;
  int64_t n_rays;
  const float* rgb;
  const float* depth;
  const float* opacity;
  const int32_t* hit_ids;
  const int32_t* hit_counts;
  int hit_cap;
  float bg0, bg1, bg2;
  const float* g_rgb;
  const float* g_depth;
  const float* g_opacity;
  int64_t n_gauss;
  const uint32_t* pair_off;  // per ray: first record
  float4* rec;               // per (ray, hit): 4 x float4
  uint64_t* key;             // per record: Gaussian index
  uint32_t* val;             // per record: its own index (permuted by the sort)
  unsigned int* truncated;
};

// Record layout: q0 = (dmu.xyz, ds.x), q1 = (ds.yz, dq.wx), q2 = (dq.yz, do, gc.r),
// q3 = (gc.g, gc.b, ray index bits, 0).

// Records per ray (the blended hits the forward pass listed, at most hit_cap).
__global__ void __launch_bounds__(kBlock) k_bwd_count(const int32_t* __restrict__ hit_counts, int64_t n, int cap,
                                                      uint32_t* __restrict__ cnt, unsigned int* truncated) {
  const int64_t r = blockIdx.x * (int64_t)kBlock + threadIdx.x;
  if (r >= n) return;
  int c = hit_counts[r];
  if (c > cap) {
    atomicAdd(truncated, 1u);
    c = cap;
  }
  cnt[r] = (uint32_t)(c < 0 ? 0 : c);
}

__global__ void __launch_bounds__(kBlock) k_bwd_pairs(BwdArgs A) {
  const int64_t r = blockIdx.x * (int64_t)kBlock + threadIdx.x;
  if (r >= A.n_rays) return;
  const float ox = A.ray_o[3 * r], oy = A.ray_o[3 * r + 1], oz = A.ray_o[3 * r + 2];
  const float dx = A.ray_d[3 * r], dy = A.ray_d[3 * r + 1], dz = A.ray_d[3 * r + 2];
  int n = A.hit_counts[r];
  n = n > A.hit_cap ? A.hit_cap : n;
  if (n <= 0) return;
  const uint32_t base = A.pair_off[r];
  const float TN = 1.f - A.opacity[r];
  const float bg[3] = {A.bg0, A.bg1, A.bg2};
  float Cf[3], gC[3];
  for (int ch = 0; ch < 3; ++ch) {
    Cf[ch] = A.rgb[3 * r + ch];  // includes T_N * bg
    gC[ch] = A.g_rgb ? A.g_rgb[3 * r + ch] : 0.f;
  }
  const float Df = A.depth[r];
  const float gD = A.g_depth ? A.g_depth[r] : 0.f;
  const float gO = A.g_opacity ? A.g_opacity[r] : 0.f;
  const float dn = rsqrtf(dx * dx + dy * dy + dz * dz);
  float Y[16];
  basis(dx * dn, dy * dn, dz * dn, A.sh_degree, Y);
  const int ncoef = (A.sh_degree + 1) * (A.sh_degree + 1);

  float T = 1.f, Cacc[3] = {0.f, 0.f, 0.f}, Dacc = 0.f;
  // The hits of a ray are replayed in order, one at a time, and the longest ray sets the
  // kernel's end: each step reads the next hit's id ahead and issues all of its own hit's
  // parameter loads (SH included) together, so fewer memory latencies separate two steps.
  int32_t i_cur = A.hit_ids[r * A.hit_cap];
  asm volatile("" ::"v"(i_cur));  // (in hand on entry too: the loop head then waits for nothing)
  for (int h = 0; h < n; ++h) {
    const int32_t i_ahead = A.hit_ids[r * A.hit_cap + (h + 1 < n ? h + 1 : h)];  // (the last re-reads its own)
    const int64_t i = i_cur;
    if (i < 0 || i >= A.n_gauss) {  // not a Gaussian of this scene: an empty record, sorted last
      const uint32_t pi = base + (uint32_t)h;
      for (int q = 0; q < 4; ++q) A.rec[4 * (int64_t)pi + q] = make_float4(0.f, 0.f, 0.f, 0.f);
      A.key[pi] = (uint64_t)A.n_gauss;
      A.val[pi] = pi;
      i_cur = i_ahead;
      continue;
    }
    float4 shv[12];
    if (A.sh_degree == 3) {
      const float4* sp4 = reinterpret_cast<const float4*>(A.sh + i * 48);
#pragma unroll
      for (int q = 0; q < 12; ++q) shv[q] = sp4[q];
    }
    // ---- recompute the hit
    const float4 q4 = reinterpret_cast<const float4*>(A.quats)[i];
    const float qn = sqrtf(q4.x * q4.x + q4.y * q4.y + q4.z * q4.z + q4.w * q4.w);
    const float w = q4.x / qn, x = q4.y / qn, y = q4.z / qn, z = q4.w / qn;
    float R[3][3];
    R[0][0] = 1.f - 2.f * (y * y + z * z); R[0][1] = 2.f * (x * y - w * z);       R[0][2] = 2.f * (x * z + w * y);
    R[1][0] = 2.f * (x * y + w * z);       R[1][1] = 1.f - 2.f * (x * x + z * z); R[1][2] = 2.f * (y * z - w * x);
    R[2][0] = 2.f * (x * z - w * y);       R[2][1] = 2.f * (y * z + w * x);       R[2][2] = 1.f - 2.f * (x * x + y * y);
    const float s[3] = {A.scales[3 * i], A.scales[3 * i + 1], A.scales[3 * i + 2]};
    float M[3][3];  // S^-1 R^T
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) M[a][b] = R[b][a] / s[a];
    const float f[3] = {ox - A.means[3 * i], oy - A.means[3 * i + 1], oz - A.means[3 * i + 2]};
    const float dv[3] = {dx, dy, dz};
    float u[3], v[3];
    for (int a = 0; a < 3; ++a) {
      u[a] = M[a][0] * f[0] + M[a][1] * f[1] + M[a][2] * f[2];
      v[a] = M[a][0] * dv[0] + M[a][1] * dv[1] + M[a][2] * dv[2];
    }
    const float vv = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
    const float uv = u[0] * v[0] + u[1] * v[1] + u[2] * v[2];
    const float ta = -uv / vv;
    const float p[3] = {u[0] + ta * v[0], u[1] + ta * v[1], u[2] + ta * v[2]};
    const float m2 = p[0] * p[0] + p[1] * p[1] + p[2] * p[2];
    const float o = A.opac[i];
    const float G = expf(-0.5f * m2);
    const float alpha = o * G;
    float c[3];
    bool pos[3];
    float acc[3] = {0.5f, 0.5f, 0.5f};
    if (A.sh_degree == 3) {
      // the 48 coefficients, loaded above as twelve 16-B loads
#pragma unroll
      for (int q = 0; q < 12; ++q) {
        const float* vv = reinterpret_cast<const float*>(&shv[q]);
#pragma unroll
        for (int e = 0; e < 4; ++e) acc[(4 * q + e) % 3] += Y[(4 * q + e) / 3] * vv[e];
      }
    } else {
      const float* shp = A.sh + i * 3 * ncoef;
      for (int ch = 0; ch < 3; ++ch)
        for (int k = 0; k < 16; ++k)
          if (k < ncoef) acc[ch] += Y[k] * shp[3 * k + ch];
    }
    for (int ch = 0; ch < 3; ++ch) {
      pos[ch] = acc[ch] > 0.f;
      c[ch] = pos[ch] ? acc[ch] : 0.f;
    }
    // ---- compositing derivatives
    const float wgt = T * alpha;
    for (int ch = 0; ch < 3; ++ch) Cacc[ch] += wgt * c[ch];
    Dacc += wgt * ta;
    const float inv1ma = 1.f / (1.f - alpha);
    float gA = 0.f;
    for (int ch = 0; ch < 3; ++ch) {
      const float behind = Cf[ch] - Cacc[ch];  // S_i (includes T_N bg)
      gA += gC[ch] * (T * c[ch] - behind * inv1ma);
    }
    gA += gD * (T * ta - (Df - Dacc) * inv1ma);
    gA += gO * (TN * inv1ma);
    const float gT = gD * wgt;  // dL/dt_alpha
    T *= (1.f - alpha);
    // ---- SH: the colour factors (dL/dsh = factor x Y is formed per Gaussian)
    float gcol[3];
    for (int ch = 0; ch < 3; ++ch) gcol[ch] = pos[ch] ? gC[ch] * wgt : 0.f;
    (void)bg;
    // ---- alpha -> opacity, m2
    const float g_op = gA * G;
    const float gm2 = gA * (-0.5f * alpha);
    float gu[3], gv[3];
    for (int a = 0; a < 3; ++a) {
      gu[a] = gm2 * 2.f * p[a] - gT * v[a] / vv;
      gv[a] = gm2 * 2.f * ta * p[a] - gT * (u[a] + 2.f * ta * v[a]) / vv;
    }
    // ---- u = M f, v = M d
    float gM[3][3];
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) gM[a][b] = gu[a] * f[b] + gv[a] * dv[b];
    float g_mu[3], g_s[3];
    for (int b = 0; b < 3; ++b) g_mu[b] = -(M[0][b] * gu[0] + M[1][b] * gu[1] + M[2][b] * gu[2]);
    float gR[3][3];
    for (int a = 0; a < 3; ++a) {
      float gs = 0.f;
      for (int b = 0; b < 3; ++b) {
        gs += gM[a][b] * M[a][b];
        gR[b][a] = gM[a][b] / s[a];
      }
      g_s[a] = -gs / s[a];
    }
    // ---- R(qhat) -> qhat -> q
    const float gw = 2.f * (-z * gR[0][1] + y * gR[0][2] + z * gR[1][0] - x * gR[1][2] - y * gR[2][0] + x * gR[2][1]);
    const float gx = 2.f * (y * gR[0][1] + z * gR[0][2] + y * gR[1][0] - 2.f * x * gR[1][1] - w * gR[1][2] +
                            z * gR[2][0] + w * gR[2][1] - 2.f * x * gR[2][2]);
    const float gy = 2.f * (-2.f * y * gR[0][0] + x * gR[0][1] + w * gR[0][2] + x * gR[1][0] + z * gR[1][2] -
                            w * gR[2][0] + z * gR[2][1] - 2.f * y * gR[2][2]);
    const float gz = 2.f * (-2.f * z * gR[0][0] - w * gR[0][1] + x * gR[0][2] + w * gR[1][0] - 2.f * z * gR[1][1] +
                            y * gR[1][2] + x * gR[2][0] + y * gR[2][1]);
    const float dot = w * gw + x * gx + y * gy + z * gz;
    // the id read ahead is in hand before this step's stores go out (an empty asm that
    // takes it as an input), so the next step does not wait for them
    asm volatile("" ::"v"(i_ahead));
    const uint32_t pi = base + (uint32_t)h;
    float4* rp = A.rec + 4 * (int64_t)pi;
    rp[0] = make_float4(g_mu[0], g_mu[1], g_mu[2], g_s[0]);
    rp[1] = make_float4(g_s[1], g_s[2], (gw - w * dot) / qn, (gx - x * dot) / qn);
    rp[2] = make_float4((gy - y * dot) / qn, (gz - z * dot) / qn, g_op, gcol[0]);
    rp[3] = make_float4(gcol[1], gcol[2], __uint_as_float((uint32_t)r), 0.f);
    A.key[pi] = (uint64_t)i;
    A.val[pi] = pi;
    i_cur = i_ahead;
  }
}

// Total number of records: the last ray's offset plus its count.
__global__ void k_bwd_total(const uint32_t* __restrict__ off, const uint32_t* __restrict__ cnt, int64_t R,
                            uint32_t* __restrict__ total) {
  if (threadIdx.x == 0) *total = off[R - 1] + cnt[R - 1];
}

// Per Gaussian: [first[g], last[g]) in the sorted records (empty when untouched). The
// number of records is read on the device; a fixed grid strides over them.
__global__ void __launch_bounds__(kBlock) k_bwd_segments(const uint64_t* __restrict__ key,
                                                         const uint32_t* __restrict__ total, int64_t n_gauss,
                                                         uint32_t* __restrict__ first, uint32_t* __restrict__ last) {
  const int64_t P = *total;
  for (int64_t p = blockIdx.x * (int64_t)kBlock + threadIdx.x; p < P; p += (int64_t)gridDim.x * kBlock) {
    const uint64_t k = key[p];
    if (k >= (uint64_t)n_gauss) continue;
    if (p == 0 || key[p - 1] != k) first[k] = (uint32_t)p;
    if (p == P - 1 || key[p + 1] != k) last[k] = (uint32_t)(p + 1);
  }
}

struct ReduceArgs {
  const float4* rec;
  const uint32_t* order;  // sorted position -> record
  const uint32_t* first;
  const uint32_t* last;
  const float* ray_d;
  int sh_degree;
  int64_t n_gauss;
  float* d_means;
  float* d_scales;
  float* d_quats;
  float* d_opac;
  float* d_sh;
};

__device__ __forceinline__ float wave_sum(float v) {
  // fixed butterfly: the same order on every run
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// One wave per Gaussian: lanes take the Gaussian's records in sorted order with stride 64,
// sum them, and the wave adds the totals to the caller's arrays (no other wave writes
// them, so plain read-add-write).
__global__ void __launch_bounds__(kBlock) k_bwd_reduce(ReduceArgs A) {
  const int64_t g = (blockIdx.x * (int64_t)kBlock + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (g >= A.n_gauss) return;
  const uint32_t b = A.first[g], e = A.last[g];
  if (e <= b) return;
  const int ncoef = (A.sh_degree + 1) * (A.sh_degree + 1);
  float acc[11];
  float sh[16][3];
#pragma unroll
  for (int q = 0; q < 11; ++q) acc[q] = 0.f;
#pragma unroll
  for (int k = 0; k < 16; ++k) sh[k][0] = sh[k][1] = sh[k][2] = 0.f;
  for (uint32_t p = b + lane; p < e; p += 64) {
    const float4* rp = A.rec + 4 * (int64_t)A.order[p];
    const float4 q0 = rp[0], q1 = rp[1], q2 = rp[2], q3 = rp[3];
    acc[0] += q0.x; acc[1] += q0.y; acc[2] += q0.z; acc[3] += q0.w;
    acc[4] += q1.x; acc[5] += q1.y; acc[6] += q1.z; acc[7] += q1.w;
    acc[8] += q2.x; acc[9] += q2.y; acc[10] += q2.z;
    const int64_t r = __float_as_uint(q3.z);
    const float dx = A.ray_d[3 * r], dy = A.ray_d[3 * r + 1], dz = A.ray_d[3 * r + 2];
    const float dn = rsqrtf(dx * dx + dy * dy + dz * dz);
    float Y[16];
    basis(dx * dn, dy * dn, dz * dn, A.sh_degree, Y);
    const float gc[3] = {q2.w, q3.x, q3.y};
#pragma unroll
    for (int k = 0; k < 16; ++k)
      if (k < ncoef) {
        sh[k][0] += gc[0] * Y[k];
        sh[k][1] += gc[1] * Y[k];
        sh[k][2] += gc[2] * Y[k];
      }
  }
#pragma unroll
  for (int q = 0; q < 11; ++q) acc[q] = wave_sum(acc[q]);
#pragma unroll
  for (int k = 0; k < 16; ++k)
    if (k < ncoef) {
      sh[k][0] = wave_sum(sh[k][0]);
      sh[k][1] = wave_sum(sh[k][1]);
      sh[k][2] = wave_sum(sh[k][2]);
    }
  if (lane == 0) {
    for (int a = 0; a < 3; ++a) A.d_means[3 * g + a] += acc[a];
    for (int a = 0; a < 3; ++a) A.d_scales[3 * g + a] += acc[3 + a];
    for (int a = 0; a < 4; ++a) A.d_quats[4 * g + a] += acc[6 + a];
    A.d_opac[g] += acc[10];
    for (int k = 0; k < 16; ++k)
      if (k < ncoef)
        for (int ch = 0; ch < 3; ++ch) A.d_sh[g * 3 * ncoef + 3 * k + ch] += sh[k][ch];
  }
}

__global__ void k_zero_u32(unsigned int* p) { *p = 0u; }

__global__ void __launch_bounds__(kBlock) k_fill_u32_bwd(uint32_t* p, int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x;
  if (i < n) p[i] = 0u;
}

inline unsigned grid(int64_t n, int per = kBlock) { return (unsigned)std::max<int64_t>(1, (n + per - 1) / per); }


}  // namespace

// Hit-list capacity of the re-trace when the forward outputs carry no list.
constexpr int kRetraceCap = 256;

grtx_status trace_backward(const Bvh* bvh, const grtx_gaussians* g, const grtx_rays* r, const grtx_trace_params* p,
                           const grtx_trace_outputs* fwd, const float* grad_rgb, const float* grad_depth,
                           const float* grad_opacity, const grtx_gaussian_grads* grads, unsigned int* truncated,
                           hipStream_t s) {
  const int64_t R = r->count;
  const int64_t N = g->count;
  hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(1), 0, s, truncated);
  GRTX_LAUNCH_CHECK();
  if (R == 0 || N == 0) return GRTX_OK;
  const bool retrace = fwd->hit_ids == nullptr;
  const int cap = !retrace ? fwd->hit_capacity : (fwd->hit_capacity > 0 ? fwd->hit_capacity : kRetraceCap);
  // every record of the pass lives in scratch sized for the bound rays x cap, so that the
  // host never waits for the actual number (which stays on the device)
  const int64_t Pmax = R * (int64_t)cap;
  if (Pmax >= ((int64_t)1 << 32) - 1) {
    set_error("trace_backward: %lld rays x %d listed hits exceed 2^32 records", (long long)R, cap);
    return GRTX_ERR_INVALID_ARG;
  }
  Scratch sc(s);
  grtx_trace_outputs fo = *fwd;
  if (retrace) {
    // the blended ids are not given: trace again with a list (the trace is deterministic,
    // so its outputs equal the forward's)
    float* outs = nullptr;
    GRTX_TRY(sc.get(&outs, 5 * R));
    GRTX_TRY(sc.get(&fo.hit_ids, Pmax));
    GRTX_TRY(sc.get(&fo.hit_counts, R));
    fo.rgb = outs;
    fo.depth = outs + 3 * R;
    fo.opacity = outs + 4 * R;
    fo.stats = nullptr;
    fo.hit_capacity = cap;
    GRTX_TRY(trace(bvh, r, p, &fo, s));
  }
  // 1. records per ray, their offsets and the total (on the device)
  uint32_t *cnt = nullptr, *off = nullptr, *total = nullptr;
  GRTX_TRY(sc.get(&cnt, R));
  GRTX_TRY(sc.get(&off, R));
  GRTX_TRY(sc.get(&total, 1));
  hipLaunchKernelGGL(k_bwd_count, dim3(grid(R)), dim3(kBlock), 0, s, fo.hit_counts, R, cap, cnt, truncated);
  GRTX_LAUNCH_CHECK();
  GRTX_TRY(exclusive_scan_u32(cnt, off, R, s));
  hipLaunchKernelGGL(k_bwd_total, dim3(1), dim3(64), 0, s, off, cnt, R, total);
  // 2. one record per (ray, blended hit)
  BwdArgs a{};
  a.means = g->means;
  a.scales = g->scales;
  a.quats = g->quats;
  a.opac = g->opacities;
  a.sh = g->sh;
  a.sh_degree = g->sh_degree;
  a.ray_o = r->origins;
  a.ray_d = r->dirs;
  a.n_rays = R;
  a.rgb = fo.rgb;
  a.depth = fo.depth;
  a.opacity = fo.opacity;
  a.hit_ids = fo.hit_ids;
  a.hit_counts = fo.hit_counts;
  a.hit_cap = cap;
  a.bg0 = p->bg[0];
  a.bg1 = p->bg[1];
  a.bg2 = p->bg[2];
  a.g_rgb = grad_rgb;
  a.g_depth = grad_depth;
  a.g_opacity = grad_opacity;
  a.n_gauss = N;
  a.pair_off = off;
  GRTX_TRY(sc.get(&a.rec, 4 * Pmax));
  GRTX_TRY(sc.get(&a.key, Pmax));
  GRTX_TRY(sc.get(&a.val, Pmax));
  a.truncated = truncated;
  hipLaunchKernelGGL(k_bwd_pairs, dim3(grid(R)), dim3(kBlock), 0, s, a);
  GRTX_LAUNCH_CHECK();
  // 3. group by Gaussian, keeping ray order inside a Gaussian
  int bits = 1;  // keys are 0..N (N marks a record of no Gaussian)
  while (bits < 63 && ((int64_t)1 << bits) <= N) ++bits;
  uint64_t *tkeys = nullptr, *skey = nullptr;
  uint32_t *tvals = nullptr, *sval = nullptr;
  GRTX_TRY(sc.get(&tkeys, Pmax));
  GRTX_TRY(sc.get(&tvals, Pmax));
  GRTX_TRY(sort_by_key_into(a.key, a.val, tkeys, tvals, Pmax, bits, s, total, &skey, &sval));
  // 4. segments and per-Gaussian sums
  uint32_t *first = nullptr, *last = nullptr;
  GRTX_TRY(sc.get(&first, N));
  GRTX_TRY(sc.get(&last, N));
  hipLaunchKernelGGL(k_fill_u32_bwd, dim3(grid(N)), dim3(kBlock), 0, s, first, N);
  hipLaunchKernelGGL(k_fill_u32_bwd, dim3(grid(N)), dim3(kBlock), 0, s, last, N);
  hipLaunchKernelGGL(k_bwd_segments, dim3((unsigned)std::min<int64_t>(4096, grid(Pmax))), dim3(kBlock), 0, s, skey,
                     total, N, first, last);
  ReduceArgs ra{};
  ra.rec = a.rec;
  ra.order = sval;
  ra.first = first;
  ra.last = last;
  ra.ray_d = r->dirs;
  ra.sh_degree = g->sh_degree;
  ra.n_gauss = N;
  ra.d_means = grads->means;
  ra.d_scales = grads->scales;
  ra.d_quats = grads->quats;
  ra.d_opac = grads->opacities;
  ra.d_sh = grads->sh;
  hipLaunchKernelGGL(k_bwd_reduce, dim3(grid(N * 64)), dim3(kBlock), 0, s, ra);
  GRTX_LAUNCH_CHECK();
  return GRTX_OK;
}

}  // namespace grtx
