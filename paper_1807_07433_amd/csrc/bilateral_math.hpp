// Bilateral weight of Eq. 9-10, shared by the aggregation, batch and adjoint kernels
// so all of them use the same float for the same pixel pair:
//   w = exp(-(dx^2 + dy^2) / gamma_d^2 - ((g_q - g_p) / 255)^2 / gamma_r^2)
// (the product of the two exponentials written as one).
#pragma once

#include "rsv_internal.hpp"

namespace rsv {

__device__ __forceinline__ float bilateral_weight(float gq, float gp, int dy, int dx, float inv_gd2,
                                                  float inv_gr2) {
  const float dg = (gq - gp) * (1.f / 255.f);
  const float r2 = static_cast<float>(dy * dy + dx * dx);
  return expf(-(r2 * inv_gd2 + dg * dg * inv_gr2));
}

// d w / d g_q for the same weight (and -that for g_p).
__device__ __forceinline__ float bilateral_weight_dgq(float w, float gq, float gp, float inv_gr2) {
  const float dg = (gq - gp) * (1.f / 255.f);
  return w * (-2.f * dg * inv_gr2 * (1.f / 255.f));
}

}  // namespace rsv
