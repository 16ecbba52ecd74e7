// Selection arithmetic shared by the plain select kernel and the batch tail kernel:
// Eq. 12 on the winner and its neighbours, and post-processing + triangulation
// (Sec. II-C, II-D), so both forms round identically.
#pragma once

#include <math.h>

#include "rsv_internal.hpp"

namespace rsv {

// Eq. 12: d + (a(d-1) - a(d+1)) / (2a(d-1) + 2a(d+1) - 4a(d)); ends of the range unrefined.
__device__ __forceinline__ float parabola(int arg, float best, float am, float ap, int D) {
  if (arg <= 0 || arg >= D - 1) return static_cast<float>(arg);
  const float den = 2.f * am + 2.f * ap - 4.f * best;
  return static_cast<float>(arg) + (am - ap) / den;
}

// d_f = d_s + s(u - d_s, v); xyz = (x, y, z) or NaN when invalid or d_f <= 0.  FP64, one rounding.
__device__ __forceinline__ void postprocess_point(float dsub, bool valid, int u, int v, const rsv_plane& pl,
                                                  const rsv_camera& cam, float* dfin, float* xyz) {
  const double ds = static_cast<double>(dsub);
  const double df = ds + (pl.a0 + pl.a1 * static_cast<double>(v) +
                          pl.a2 * (static_cast<double>(u) - ds) - pl.delta);
  if (dfin) *dfin = static_cast<float>(df);
  if (xyz) {
    if (valid && df > 0.0) {
      const double z = cam.f * cam.baseline / df;
      xyz[0] = static_cast<float>((static_cast<double>(u) - cam.u0) * z / cam.f);
      xyz[1] = static_cast<float>((static_cast<double>(v) - cam.v0) * z / cam.f);
      xyz[2] = static_cast<float>(z);
    } else {
      xyz[0] = xyz[1] = xyz[2] = NAN;
    }
  }
}

}  // namespace rsv
