// One 16 x 16 output tile of the bilateral aggregation (Sec. II-B.2, Eq. 8-10) on
// the matrix cores, shared by the plain aggregation kernel and the batch kernel.
// NT threads (1024 or 512): wave w owns patches w, w + NT/64, ... of the 16 patches,
// patch k sitting at (k / 4, k % 4); every patch runs the same MFMA sequence
// whatever NT is, so both forms give the same floats.  The cost tile plus halo for 16
// disparities at a time is staged in LDS as fp16 hi / lo planes (double-buffered,
// next tile's global loads in flight during the current tile's MFMAs).  For every
// disparity tile t the sink receives, per lane, the aggregated values of pixels
// (patch row g = lane / 16, columns 0..3) at disparity 16 t + lane % 16.
#pragma once

#include "aggregate_mfma.hpp"

namespace rsv {

template <int A>
__host__ __device__ inline size_t agg_tile_lds_bytes() {
  using G = AggGeo<A>;
  return sizeof(float) * G::GT * G::GT + 2 /*hi,lo*/ * 2 /*buffers*/ * 16 * G::PLANE * sizeof(_Float16);
}

// guide_at(Y, X): guide intensity at in-image (Y, X).
// sink(t, pp, lane, vals): vals[e] = A[16 t + lane % 16][by + 4 pp.pr + lane / 16][bx + 4 pp.pc + e]
// (values for disparities >= D or pixels outside the image are meaningless).
template <int A, int NT, typename GuideAt, typename Sink>
__device__ __forceinline__ void agg_tile(const float* __restrict__ cost, int H, int W, int D, float igd2,
                                         float igr2, int by, int bx, GuideAt guide_at, Sink& sink,
                                         unsigned char* smem) {
  using G = AggGeo<A>;
  constexpr int NW = NT / 64;               // waves
  constexpr int PPW = 16 / NW;              // patches per wave
  constexpr int SPT = (G::RAW + NT - 1) / NT;  // staged tile positions per thread
  float* gt = reinterpret_cast<float*>(smem);
  _Float16* hi = reinterpret_cast<_Float16*>(smem + sizeof(float) * G::GT * G::GT);
  _Float16* lo = hi + 2 * 16 * G::PLANE;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t plane = static_cast<int64_t>(H) * W;

  for (int i = tid; i < G::GT * G::GT; i += NT) {
    const int r = i / G::GT, c = i - r * G::GT;
    const int Y = by - A + r, X = bx - A + c;
    gt[i] = (Y >= 0 && Y < H && X >= 0 && X < W) ? guide_at(Y, X) : 0.f;
  }

  // Thread tid owns tile positions tid, tid + NT, ... (< RAW) and moves their 16
  // disparities of one tile: global -> registers -> LDS hi / lo planes.
  const float* src[SPT];
  bool sok[SPT];
#pragma unroll
  for (int q = 0; q < SPT; ++q) {
    const int i = tid + q * NT;
    const int sr = i / G::TC, sc = i - sr * G::TC;
    const int sY = by - A + sr, sX = bx - A + sc;
    sok[q] = i < G::RAW && sY >= 0 && sY < H && sX >= 0 && sX < W;
    src[q] = cost + (sok[q] ? static_cast<int64_t>(sY) * W + sX : 0);
  }
  float pre[SPT][16];
  auto fetch = [&](int t) {
#pragma unroll
    for (int q = 0; q < SPT; ++q)
#pragma unroll
      for (int dd = 0; dd < 16; ++dd) {
        const int d = 16 * t + dd;
        pre[q][dd] = (sok[q] && d < D) ? src[q][d * plane] : 0.f;
      }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int q = 0; q < SPT; ++q) {
      const int i = tid + q * NT;
      if (i < G::RAW) {
        _Float16* h = hi + buf * 16 * G::PLANE + i;
        _Float16* l = lo + buf * 16 * G::PLANE + i;
#pragma unroll
        for (int dd = 0; dd < 16; ++dd) split_store(pre[q][dd], h, l, dd * G::PLANE);
      }
    }
  };

  fetch(0);
  store(0);
  __syncthreads();

  PatchPos pp[PPW];
  half8_t whi[PPW][G::KS], wlo[PPW][G::KS];
  float4_t iz[PPW];
#pragma unroll
  for (int k = 0; k < PPW; ++k) {
    const int patch = wave + k * NW;
    pp[k] = PatchPos{patch >> 2, patch & 3};
    iz[k] = patch_weights<A>(whi[k], wlo[k], pp[k], lane, by, bx, H, W, igd2, igr2,
                             [&](int r, int c) { return gt[r * G::GT + c]; });
  }

  const int ndt = (D + 15) >> 4;
  for (int t = 0; t < ndt; ++t) {
    const int buf = t & 1;
    if (t + 1 < ndt) fetch(t + 1);
#pragma unroll
    for (int k = 0; k < PPW; ++k) {
      const float4_t acc =
          patch_mfma<A>(whi[k], wlo[k], hi + buf * 16 * G::PLANE, lo + buf * 16 * G::PLANE, pp[k], lane);
      float4_t vals;
#pragma unroll
      for (int e = 0; e < 4; ++e) vals[e] = acc[e] * iz[k][e];
      sink(t, pp[k], lane, vals);
    }
    if (t + 1 < ndt) store(buf ^ 1);
    __syncthreads();
  }
}

}  // namespace rsv
