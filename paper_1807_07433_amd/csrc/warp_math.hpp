// Perspective-warp sample (Sec. II-A): the warped target at column u of row v is
// the target row v linearly interpolated at x = u - s(u, v), s = a0 + a1 v + a2 u - delta.
// Computed in double and rounded once, so every kernel that needs a warped value
// (plain warp, fused batch kernel, adjoint) produces the same float.
#pragma once

#include "rsv_internal.hpp"

namespace rsv {

struct WarpTap {
  int c0, c1;     // clamped source columns
  double f;       // interpolation fraction
};

__device__ __forceinline__ double plane_shift(const rsv_plane& pl, int u, int v) {
  return pl.a0 + pl.a1 * static_cast<double>(v) + pl.a2 * static_cast<double>(u) - pl.delta;
}

__device__ __forceinline__ WarpTap warp_tap(const rsv_plane& pl, int u, int v, int W) {
  double x = static_cast<double>(u) - plane_shift(pl, u, v);
  x = fmin(fmax(x, -2.0), static_cast<double>(W) + 1.0);  // keeps floor() in int range
  const double x0 = floor(x);
  WarpTap t;
  t.f = x - x0;
  const int i0 = static_cast<int>(x0);
  t.c0 = clampi(i0, 0, W - 1);
  t.c1 = clampi(i0 + 1, 0, W - 1);
  return t;
}

template <typename T>
__device__ __forceinline__ float warp_sample(const T* __restrict__ right, int64_t pitch, int W,
                                             const rsv_plane& pl, int u, int v) {
  const WarpTap t = warp_tap(pl, u, v, W);
  const T* row = right + static_cast<int64_t>(v) * pitch;
  const double i0 = static_cast<double>(row[t.c0]);
  const double i1 = static_cast<double>(row[t.c1]);
  return static_cast<float>(i0 + t.f * (i1 - i0));
}

}  // namespace rsv
