// Pinhole camera rays, shared by the ray generator and the serving path's in-kernel ray
// generation: both go through these two functions, so a served pixel's ray is the same
// bits as the one grtx_pinhole_rays writes for it.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

namespace grtx {

// Camera frame: eye, unit forward, right scaled by tan(fov_y / 2) * aspect, true up
// scaled by tan(fov_y / 2). Computed in double on the host, stored in float. False for a
// degenerate frame (eye on target, or up parallel to the view direction).
struct CameraFrame {
  float eye[3], fwd[3], right[3], up[3];
};

inline bool camera_frame(const float eye[3], const float target[3], const float up[3], float fov_y_deg, int width,
                         int height, CameraFrame* out) {
  double f[3], r[3], u[3];
  for (int a = 0; a < 3; ++a) f[a] = (double)target[a] - eye[a];
  const double fl = std::sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
  if (!(fl > 0.0)) return false;
  for (double& x : f) x /= fl;
  r[0] = f[1] * up[2] - f[2] * up[1];
  r[1] = f[2] * up[0] - f[0] * up[2];
  r[2] = f[0] * up[1] - f[1] * up[0];
  const double rl = std::sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
  if (!(rl > 0.0)) return false;
  for (double& x : r) x /= rl;
  u[0] = r[1] * f[2] - r[2] * f[1];
  u[1] = r[2] * f[0] - r[0] * f[2];
  u[2] = r[0] * f[1] - r[1] * f[0];
  const double th = std::tan(0.5 * (double)fov_y_deg * M_PI / 180.0);
  const double aspect = (double)width / (double)height;
  for (int a = 0; a < 3; ++a) {
    out->eye[a] = eye[a];
    out->fwd[a] = (float)f[a];
    out->right[a] = (float)(r[a] * th * aspect);
    out->up[a] = (float)(u[a] * th);
  }
  return true;
}

// Unit direction through the centre of pixel (x, y) of a W x H image (row 0 at the top).
__device__ __forceinline__ void pinhole_dir(float fx, float fy, float fz, float rx, float ry, float rz, float ux,
                                            float uy, float uz, int x, int y, int W, int H, float* dx, float* dy,
                                            float* dz) {
  const float sx = 2.f * ((float)x + 0.5f) / (float)W - 1.f;
  const float sy = 1.f - 2.f * ((float)y + 0.5f) / (float)H;
  const float ex = fx + sx * rx + sy * ux;
  const float ey = fy + sx * ry + sy * uy;
  const float ez = fz + sx * rz + sy * uz;
  const float inv = 1.f / sqrtf(ex * ex + ey * ey + ez * ez);
  *dx = ex * inv;
  *dy = ey * inv;
  *dz = ez * inv;
}

}  // namespace grtx
