// Device helpers and constants shared by the trace kernels (k_trace) and the single-round
// kernels: ray keys, slab test, unit-sphere leaf terms, real spherical harmonics, and the
// per-lane stack sizes. Included inside namespace grtx's anonymous namespace of each
// source, so every file gets its own copies.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "grtx_internal.h"

namespace grtx {
namespace {

#ifndef GRTX_LDS_STACK
#define GRTX_LDS_STACK 16
#endif
constexpr int kTraceBlock = 256;
constexpr int kWaves = kTraceBlock / 64;
constexpr int kLdsStack = GRTX_LDS_STACK;  // per-lane stack entries held in LDS
// The build keeps no tree deeper than GRTX_MAX_TREE_DEPTH internal nodes on a path (it
// measures the restructured tree and falls back to the plain radix tree, at most 96 deep
// over distinct 95-bit keys); a record's children lie one to three levels below it, so a
// path visits at most that many records, each leaving at most three entries pending.
constexpr int kMaxStack = 3 * GRTX_MAX_TREE_DEPTH + 16;
constexpr int kSpillRows = kMaxStack - kLdsStack;
constexpr uint64_t kEmptyKey = (0x7F800000ull << 32) | 0xFFFFFFFFull;  // (+inf, max)

__device__ __forceinline__ float key_t(uint64_t k) { return __uint_as_float((uint32_t)(k >> 32)); }
__device__ __forceinline__ uint64_t make_key(float t, uint32_t id) {
  return ((uint64_t)__float_as_uint(t) << 32) | id;
}

// Robust reciprocal for the slab test: zero components become a huge finite value of
// the same sign, so that 0 * inv never produces NaN.
__device__ __forceinline__ float safe_inv(float d) {
  const float tiny = 1e-20f;
  float ad = fabsf(d);
  return 1.0f / copysignf(ad > tiny ? ad : tiny, d);
}

struct Slab {
  float tn, tf;
};

__device__ __forceinline__ Slab slab(float lox, float loy, float loz, float hix, float hiy, float hiz, float ox,
                                     float oy, float oz, float ix, float iy, float iz) {
  float t0x = (lox - ox) * ix, t1x = (hix - ox) * ix;
  float t0y = (loy - oy) * iy, t1y = (hiy - oy) * iy;
  float t0z = (loz - oz) * iz, t1z = (hiz - oz) * iz;
  Slab s;
  s.tn = fmaxf(fmaxf(fminf(t0x, t1x), fminf(t0y, t1y)), fminf(t0z, t1z));
  s.tf = fminf(fminf(fmaxf(t0x, t1x), fmaxf(t0y, t1y)), fmaxf(t0z, t1z));
  return s;
}

// Real spherical harmonics up to band 3 (orthonormal, Condon-Shortley phase) as
// polynomials in the unit direction. Y_l^m = sqrt(2) K_l^|m| (-1)^m (cos|sin)(|m| phi)
// sin^|m|(theta) P_l^(|m|)(cos theta), with K_l^m = sqrt((2l+1)/(4 pi) (l-|m|)!/(l+|m|)!)
// and P_l^(m) the m-th derivative of the Legendre polynomial.
constexpr double cx_sqrt(double x) {
  double r = x > 1.0 ? x : 1.0;
  for (int i = 0; i < 100; ++i) r = 0.5 * (r + x / r);
  return r;
}
constexpr double kPi = 3.14159265358979323846;
constexpr double K(int l, int am, double fac_ratio) { return cx_sqrt((2.0 * l + 1.0) / (4.0 * kPi) * fac_ratio); }
constexpr float SH00 = (float)K(0, 0, 1.0);
constexpr float SH1 = (float)K(1, 0, 1.0);                                   // sqrt(3/4pi)
constexpr float SH20 = (float)(K(2, 0, 1.0) * 0.5);                          // K20 / 2 * (3z^2 - 1)
constexpr float SH21 = (float)(cx_sqrt(2.0) * K(2, 1, 1.0 / 6.0) * 3.0);     // -xz, -yz
constexpr float SH22 = (float)(cx_sqrt(2.0) * K(2, 2, 1.0 / 24.0) * 3.0);    // (x^2-y^2), 2xy
constexpr float SH30 = (float)(K(3, 0, 1.0) * 0.5);                          // (5z^3 - 3z)
constexpr float SH31 = (float)(cx_sqrt(2.0) * K(3, 1, 1.0 / 12.0) * 0.5);    // -(15z^2-3) x|y
constexpr float SH32 = (float)(cx_sqrt(2.0) * K(3, 2, 1.0 / 120.0) * 15.0);  // z (x^2-y^2), 2xyz
constexpr float SH33 = (float)(cx_sqrt(2.0) * K(3, 3, 1.0 / 720.0) * 15.0);  // -(x^3-3xy^2), -(3x^2y-y^3)

__device__ __forceinline__ void sh_basis(float x, float y, float z, int L, float* Y) {
  Y[0] = SH00;
  if (L < 1) return;
  Y[1] = -SH1 * y;
  Y[2] = SH1 * z;
  Y[3] = -SH1 * x;
  if (L < 2) return;
  float xx = x * x, yy = y * y, zz = z * z;
  Y[4] = SH22 * 2.f * x * y;
  Y[5] = -SH21 * y * z;
  Y[6] = SH20 * (3.f * zz - 1.f);
  Y[7] = -SH21 * x * z;
  Y[8] = SH22 * (xx - yy);
  if (L < 3) return;
  Y[9] = -SH33 * (3.f * xx * y - yy * y);
  Y[10] = SH32 * 2.f * x * y * z;
  Y[11] = -SH31 * y * (15.f * zz - 3.f);
  Y[12] = SH30 * (5.f * zz * z - 3.f * z);
  Y[13] = -SH31 * x * (15.f * zz - 3.f);
  Y[14] = SH32 * z * (xx - yy);
  Y[15] = -SH33 * (xx * x - 3.f * x * yy);
}

// Sphere leaf: ray in the unit-sphere frame of instance record (r0, r1, r2).
struct SphereHit {
  float a, b, c2;  // v.v, u.v, |u x v|^2
};

__device__ __forceinline__ SphereHit sphere_terms(float4 r0, float4 r1, float4 r2, float ox, float oy, float oz,
                                                  float dx, float dy, float dz) {
  float fx = ox - r0.w, fy = oy - r1.w, fz = oz - r2.w;
  float ux = r0.x * fx + r0.y * fy + r0.z * fz;
  float uy = r1.x * fx + r1.y * fy + r1.z * fz;
  float uz = r2.x * fx + r2.y * fy + r2.z * fz;
  float vx = r0.x * dx + r0.y * dy + r0.z * dz;
  float vy = r1.x * dx + r1.y * dy + r1.z * dz;
  float vz = r2.x * dx + r2.y * dy + r2.z * dz;
  float cx = uy * vz - uz * vy, cy = uz * vx - ux * vz, cz = ux * vy - uy * vx;
  SphereHit h;
  h.a = vx * vx + vy * vy + vz * vz;
  h.b = ux * vx + uy * vy + uz * vz;
  h.c2 = cx * cx + cy * cy + cz * cz;
  return h;
}

}  // namespace
}  // namespace grtx
