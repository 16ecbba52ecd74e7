// rsv_aggregate: bilateral cost aggregation (Sec. II-B.2, Eq. 8-10).
//
// The weights of Eq. 9-10 depend on the pixel pair only, not on d.  Each thread
// owns one output pixel, computes its (2A+1)^2 weights once into registers
// (zero for taps outside the image) together with 1 / sum(w), and then walks the
// disparity slices: slice d of the cost volume is staged tile-plus-halo in LDS
// (double-buffered) and the thread forms its weighted sum from there.
#include "bilateral_math.hpp"

namespace rsv {

constexpr int kAggT = 16;

template <int A, typename TG>
__global__ __launch_bounds__(kAggT* kAggT) void aggregate_kernel(
    const float* __restrict__ cost, const TG* __restrict__ guide, int64_t gpitch, int H, int W,
    int D, float inv_gd2, float inv_gr2, float* __restrict__ agg) {
  constexpr int K = 2 * A + 1;
  constexpr int TT = kAggT + 2 * A;
  __shared__ float tile[2][TT * TT];
  const int tx = threadIdx.x, ty = threadIdx.y;
  const int tid = ty * kAggT + tx;
  const int ub = blockIdx.x * kAggT, vb = blockIdx.y * kAggT;
  const int u = ub + tx, v = vb + ty;
  const bool inside = (u < W) && (v < H);

  // Eq. 9-10 weights; intensities scaled by 1/255 inside the range term.
  float w[K][K];
  float z = 0.f;
  const float gp = pixel(guide, gpitch, clampi(v, 0, H - 1), clampi(u, 0, W - 1));
#pragma unroll
  for (int j = 0; j < K; ++j)
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int y = v + j - A, x = u + k - A;
      float wt = 0.f;
      if (x >= 0 && x < W && y >= 0 && y < H)
        wt = bilateral_weight(pixel(guide, gpitch, y, x), gp, j - A, k - A, inv_gd2, inv_gr2);
      w[j][k] = wt;
      z += wt;
    }
  const float invz = 1.f / z;

  const int64_t plane = static_cast<int64_t>(H) * W;
  auto stage = [&](int d, float* dst) {
    const float* src = cost + d * plane;
    for (int i = tid; i < TT * TT; i += kAggT * kAggT) {
      const int r = i / TT, c = i - r * TT;
      const int y = vb - A + r, x = ub - A + c;
      dst[i] = (x >= 0 && x < W && y >= 0 && y < H) ? src[static_cast<int64_t>(y) * W + x] : 0.f;
    }
  };
  stage(0, tile[0]);
  __syncthreads();
  for (int d = 0; d < D; ++d) {
    const float* cur = tile[d & 1];
    if (d + 1 < D) stage(d + 1, tile[(d + 1) & 1]);
    float acc = 0.f;
#pragma unroll
    for (int j = 0; j < K; ++j)
#pragma unroll
      for (int k = 0; k < K; ++k) acc = fmaf(w[j][k], cur[(ty + j) * TT + tx + k], acc);
    if (inside) agg[d * plane + static_cast<int64_t>(v) * W + u] = acc * invz;
    __syncthreads();
  }
}

template <int A, typename TG>
int launch_agg(const float* cost, const rsv_image& g, const rsv_params* p, float* agg,
               hipStream_t st) {
  const dim3 block(kAggT, kAggT);
  const dim3 grid((g.width + kAggT - 1) / kAggT, (g.height + kAggT - 1) / kAggT);
  const float inv_gd2 = 1.f / (p->gamma_d * p->gamma_d);
  const float inv_gr2 = 1.f / (p->gamma_r * p->gamma_r);
  aggregate_kernel<A, TG><<<grid, block, 0, st>>>(cost, static_cast<const TG*>(g.data), g.pitch,
                                                  g.height, g.width, p->D, inv_gd2, inv_gr2, agg);
  return check_launch();
}

template <typename TG>
int dispatch_agg(const float* cost, const rsv_image& g, const rsv_params* p, float* agg,
                 hipStream_t st) {
  switch (p->agg_radius) {
    case 1: return launch_agg<1, TG>(cost, g, p, agg, st);
    case 2: return launch_agg<2, TG>(cost, g, p, agg, st);
    case 3: return launch_agg<3, TG>(cost, g, p, agg, st);
    case 4: return launch_agg<4, TG>(cost, g, p, agg, st);
    case 5: return launch_agg<5, TG>(cost, g, p, agg, st);
    case 6: return launch_agg<6, TG>(cost, g, p, agg, st);
    default: return RSV_E_PARAM;
  }
}

}  // namespace rsv

extern "C" int rsv_aggregate(const float* cost, rsv_image guide, const rsv_params* p, float* agg,
                             void* stream) {
  using namespace rsv;
  if (int s = validate_image(guide)) return s;
  if (int s = validate_agg_params(p)) return s;
  if (!cost || !agg) return RSV_E_NULL;
  if (!aligned(cost, 4) || !aligned(agg, 4)) return RSV_E_ALIGN;
  if (cost == agg) return RSV_E_PARAM;
  hipStream_t st = as_stream(stream);
  if (guide.dtype == RSV_U8) return dispatch_agg<uint8_t>(cost, guide, p, agg, st);
  return dispatch_agg<float>(cost, guide, p, agg, st);
}
