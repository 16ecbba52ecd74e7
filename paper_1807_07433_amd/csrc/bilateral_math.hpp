// Bilateral weight of Eq. 9-10, shared by the aggregation, batch and adjoint kernels
// so all of them use the same float for the same pixel pair.  In base 2:
//   w = exp(-(dx^2 + dy^2) / gamma_d^2 - ((g_q - g_p) / 255)^2 / gamma_r^2)
//     = 2^-(s + (h_q - h_p)^2),   s = (dx^2 + dy^2) kd,   h = g sr,
//   kd = log2(e) / gamma_d^2,   sr = sqrt(log2(e)) / (255 gamma_r),
// evaluated with the hardware base-2 exponential.  Guides enter as h = g sr (the
// kernels scale a guide value once when they stage it), so a weight costs one
// subtraction, one FMA and one exponential.  The spatial exponent s of a window
// offset is a constant the kernels may tabulate; s = +inf (outside the window) or
// h_q = +inf (outside the image) gives w = 0.
#pragma once

#include <cmath>

#include "rsv_internal.hpp"

namespace rsv {

constexpr double kLog2e = 1.4426950408889634074;
constexpr float kLn2f = 0.693147180559945309f;

struct BilateralK {
  float kd, sr;
};

inline BilateralK bilateral_constants(float gamma_d, float gamma_r) {
  const double gd = gamma_d, gr = 255.0 * static_cast<double>(gamma_r);
  return BilateralK{static_cast<float>(kLog2e / (gd * gd)), static_cast<float>(std::sqrt(kLog2e) / gr)};
}

// h = g sr, the guide in the weight's scale.
__device__ __forceinline__ float guide_scaled(float g, const BilateralK& k) { return g * k.sr; }

__device__ __forceinline__ float spatial_exponent(int dy, int dx, float kd) {
  return static_cast<float>(dy * dy + dx * dx) * kd;
}

// w from scaled guides h_q, h_p and the spatial exponent s of the offset.
__device__ __forceinline__ float bilateral_weight_s(float hq, float hp, float s) {
  const float dh = hq - hp;
  return __builtin_amdgcn_exp2f(-fmaf(dh, dh, s));
}

__device__ __forceinline__ float bilateral_weight(float gq, float gp, int dy, int dx, const BilateralK& k) {
  return bilateral_weight_s(guide_scaled(gq, k), guide_scaled(gp, k), spatial_exponent(dy, dx, k.kd));
}

// d w / d g_q for the same weight (and -that for g_p): w ln2 (-2 (h_q - h_p) sr).
__device__ __forceinline__ float bilateral_weight_dgq(float w, float gq, float gp, const BilateralK& k) {
  return w * (-2.f * kLn2f * k.sr * (guide_scaled(gq, k) - guide_scaled(gp, k)));
}

}  // namespace rsv
