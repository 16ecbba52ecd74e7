// ZNCC arithmetic shared by the plain cost kernel and the fused batch kernel
// (Sec. II-B.1, Eq. 3-5).  With n = (2r+1)^2, S = sum of a block and Q = sum of
// squares, e = sqrt(n Q - S^2) = n * sigma.  For left block values l_i and
// target block values r_i:
//     c = sum_i (n l_i - S_l) r_i / (e_l e_r)
// which is Eq. 3 rewritten with the left block centred (the centred values sum to
// zero, so mu_r drops out).  For uint8 images n l_i - S_l is an exact integer.
// Any constant may be subtracted from the r_i without changing the sum (the cost
// tile subtracts 128), which keeps the FP32 products small.
//
// The FP32 sum's rounding error grows with sum_i |n l_i - S_l| |r_i| <= 128 n e_l, so
// its error in c scales as 1 / e_r: it stays near 1e-7 for textured target blocks and
// reaches 1e-4 only for nearly flat ones.  Target blocks with sigma below
// kExactSigma are therefore marked (their 1/e_r is stored negated) and their entries
// are recomputed exactly in FP64 (cost_tile.hpp).
#pragma once

#include "rsv_internal.hpp"

namespace rsv {

// 1 / e, or 0 when the block std-dev e / n is below sigma_min.
__device__ __forceinline__ float inv_block_norm(double n, double S, double Q, float sigma_min) {
  const double e2 = n * Q - S * S;
  if (!(e2 > 0.0)) return 0.f;
  const double e = sqrt(e2);
  if (e < n * static_cast<double>(sigma_min)) return 0.f;
  return static_cast<float>(1.0 / e);
}

// Left block of width K = 2R+1 read from a row-major tile: produces the centred
// values n*l - S (FP32) and 1/e_l.  INT: the tile holds integers in [0, 255] (a
// uint8 image), so S, Q and n*l - S are exact in FP32 (all below 2^24) and equal
// the FP64 sums bit for bit; otherwise they are formed in FP64.
template <int R, bool INT>
struct LeftBlock {
  static constexpr int K = 2 * R + 1;
  static constexpr int N = K * K;
  static_assert(!INT || N * 255 * 255 < (1 << 24), "integer block sums must stay exact in FP32");
  float c[K][K];
  float inv;

  __device__ __forceinline__ void load(const float* tile, int stride, float sigma_min) {
    if constexpr (INT) {
      float S = 0.f, Q = 0.f;
#pragma unroll
      for (int j = 0; j < K; ++j)
#pragma unroll
        for (int k = 0; k < K; ++k) {
          const float x = tile[j * stride + k];
          c[j][k] = x;
          S += x;
          Q = fmaf(x, x, Q);
        }
      inv = inv_block_norm(static_cast<double>(N), static_cast<double>(S), static_cast<double>(Q), sigma_min);
#pragma unroll
      for (int j = 0; j < K; ++j)
#pragma unroll
        for (int k = 0; k < K; ++k) c[j][k] = fmaf(static_cast<float>(N), c[j][k], -S);
    } else {
      double S = 0.0, Q = 0.0;
#pragma unroll
      for (int j = 0; j < K; ++j)
#pragma unroll
        for (int k = 0; k < K; ++k) {
          const float x = tile[j * stride + k];
          c[j][k] = x;
          S += static_cast<double>(x);
          Q = fma(static_cast<double>(x), static_cast<double>(x), Q);
        }
      inv = inv_block_norm(static_cast<double>(N), S, Q, sigma_min);
#pragma unroll
      for (int j = 0; j < K; ++j)
#pragma unroll
        for (int k = 0; k < K; ++k)
          c[j][k] = static_cast<float>(static_cast<double>(N) * static_cast<double>(c[j][k]) - S);
    }
  }
};

// Target blocks with a std-dev below this (grey levels) take the exact FP64 path.
constexpr double kExactSigma = 1.0;

// 1/e_r of a target block, negated where its std-dev is below kExactSigma (the
// entries that pair with it are recomputed in FP64); 0 below sigma_min.
__device__ __forceinline__ float target_inv(double n, double S, double Q, float sigma_min) {
  const float inv = inv_block_norm(n, S, Q, sigma_min);
  return (inv > 0.f && static_cast<double>(inv) * n * kExactSigma > 1.0) ? -inv : inv;
}

// Signed 1/e_r (target_inv) of two vertically adjacent target blocks: the one whose
// top-left corner is tile[0] and the one a row below.  They share 2R rows, which are
// summed once.
template <int R>
__device__ __forceinline__ void target_inv_pair(const float* tile, int stride, float sigma_min,
                                                float& inv0, float& inv1) {
  constexpr int K = 2 * R + 1;
  double St = 0.0, Qt = 0.0, Sm = 0.0, Qm = 0.0, Sb = 0.0, Qb = 0.0;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const double t = static_cast<double>(tile[k]);
    const double b = static_cast<double>(tile[K * stride + k]);
    St += t;
    Qt = fma(t, t, Qt);
    Sb += b;
    Qb = fma(b, b, Qb);
  }
#pragma unroll
  for (int j = 1; j < K; ++j)
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const double x = static_cast<double>(tile[j * stride + k]);
      Sm += x;
      Qm = fma(x, x, Qm);
    }
  inv0 = target_inv(static_cast<double>(K * K), St + Sm, Qt + Qm, sigma_min);
  inv1 = target_inv(static_cast<double>(K * K), Sm + Sb, Qm + Qb, sigma_min);
}

}  // namespace rsv
