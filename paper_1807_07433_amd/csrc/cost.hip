// rsv_cost_volume: ZNCC reference and target cost volumes (Sec. II-B.1, Eq. 3-5).
//
// One thread owns one left-block centre (u, v) and walks d = 0 .. D-1.  Its left
// block (centred) stays in registers; the target block slides one column left per
// step, so each step reads one new column of 2R+1 values from LDS into a ring of
// registers and spends (2R+1)^2 FMAs.  The value computed for (u, v, d) is written
// to cost_ref[d][v][u] and to cost_tar[d][v][u - d], which is the identity stated
// after Eq. 5; threads with u >= W (up to W + D - 2) exist only to fill the target
// volume where x + d leaves the image, reading the left image clamped.
//
// Tile per block: 64 consecutive centres u x 4 rows.  LDS holds the left tile
// (64 + 2R columns), the warped tile (64 + D - 1 + 2R columns) and 1/e_r of every
// target centre the block visits.
#include "zncc_math.hpp"

namespace rsv {

constexpr int kCostTW = 64;
constexpr int kCostTH = 4;

inline size_t cost_lds_bytes(int D, int R) {
  const int rows = kCostTH + 2 * R;
  const int wt = kCostTW + D - 1 + 2 * R;
  const int lw = kCostTW + 2 * R;
  const int nt = kCostTW + D - 1;
  return sizeof(float) * (static_cast<size_t>(rows) * wt + static_cast<size_t>(rows) * lw +
                          static_cast<size_t>(kCostTH) * nt);
}

template <int R, typename TL>
__global__ __launch_bounds__(kCostTW* kCostTH) void cost_volume_kernel(
    const TL* __restrict__ left, int64_t lpitch, const float* __restrict__ warped, int H, int W,
    int D, float sigma_min, float* __restrict__ cost_ref, float* __restrict__ cost_tar) {
  constexpr int K = 2 * R + 1;
  extern __shared__ float smem[];
  const int tx = threadIdx.x, ty = threadIdx.y;
  const int tid = ty * kCostTW + tx;
  const int nthreads = kCostTW * kCostTH;
  const int u0 = blockIdx.x * kCostTW;
  const int v0 = blockIdx.y * kCostTH;
  const int rows = kCostTH + 2 * R;
  const int wtw = kCostTW + D - 1 + 2 * R;  // warped tile width
  const int ltw = kCostTW + 2 * R;          // left tile width
  const int nt = kCostTW + D - 1;           // target centres visited by the block
  float* wt = smem;
  float* lt = wt + rows * wtw;
  float* ir = lt + rows * ltw;
  const int cw0 = u0 - (D - 1) - R;  // global column of warped tile column 0

  for (int i = tid; i < rows * wtw; i += nthreads) {
    const int r = i / wtw, c = i - r * wtw;
    const int y = clampi(v0 - R + r, 0, H - 1);
    const int x = clampi(cw0 + c, 0, W - 1);
    wt[i] = warped[static_cast<int64_t>(y) * W + x];
  }
  for (int i = tid; i < rows * ltw; i += nthreads) {
    const int r = i / ltw, c = i - r * ltw;
    const int y = clampi(v0 - R + r, 0, H - 1);
    const int x = clampi(u0 - R + c, 0, W - 1);
    lt[i] = pixel(left, lpitch, y, x);
  }
  __syncthreads();
  // 1/e_r for target centres x = u0 - (D-1) + c, rows v0 + r.
  for (int i = tid; i < kCostTH * nt; i += nthreads) {
    const int r = i / nt, c = i - r * nt;
    ir[i] = target_inv<R>(wt + r * wtw + c, wtw, sigma_min);
  }

  LeftBlock<R> lb;
  lb.load(lt + ty * ltw + tx, ltw, sigma_min);
  __syncthreads();

  const int u = u0 + tx;
  const int v = v0 + ty;
  const bool row_ok = v < H;
  const int64_t plane = static_cast<int64_t>(H) * W;
  const int64_t rowoff = static_cast<int64_t>(v) * W;
  const float* wrow = wt + ty * wtw + tx + (D - 1);  // window column k at step d: wrow[k - d]
  const float* irow = ir + ty * nt + tx + (D - 1);   // 1/e_r of centre u - d: irow[-d]

  float win[K][K];  // ring: window column k at step d0 + t lives in slot (k - t) mod K
#pragma unroll
  for (int j = 0; j < K; ++j)
#pragma unroll
    for (int k = 0; k < K; ++k) win[j][k] = wrow[j * wtw + k] - lb.shift;

  for (int d0 = 0; d0 < D; d0 += K) {
#pragma unroll
    for (int t = 0; t < K; ++t) {
      const int d = d0 + t;
      if (d >= D) break;
      if (d > 0) {
        const int slot = (K - t) % K;
#pragma unroll
        for (int j = 0; j < K; ++j) {
#pragma unroll
          for (int s = 0; s < K; ++s)
            if (s == slot) win[j][s] = wrow[j * wtw - d] - lb.shift;
        }
      }
      float num = 0.f;
#pragma unroll
      for (int j = 0; j < K; ++j)
#pragma unroll
        for (int k = 0; k < K; ++k) num = fmaf(lb.c[j][k], win[j][(k - t + K) % K], num);
      const float c = (num * lb.inv) * irow[-d];
      if (row_ok) {
        if (u < W) cost_ref[d * plane + rowoff + u] = c;
        const int x = u - d;
        if (cost_tar && x >= 0 && x < W) cost_tar[d * plane + rowoff + x] = c;
      }
    }
  }
}

template <int R, typename TL>
int launch_cost(const rsv_image& left, const float* warped, const rsv_params* p, float* cref,
                float* ctar, hipStream_t st) {
  const int H = left.height, W = left.width, D = p->D;
  const size_t lds = cost_lds_bytes(D, R);
  const dim3 block(kCostTW, kCostTH);
  const dim3 grid((W + D - 1 + kCostTW - 1) / kCostTW, (H + kCostTH - 1) / kCostTH);
  auto kern = cost_volume_kernel<R, TL>;
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       static_cast<int>(lds));
    if (e != hipSuccess) {
      set_hip_error(e);
      return RSV_E_HIP;
    }
  }
  kern<<<grid, block, lds, st>>>(static_cast<const TL*>(left.data), left.pitch, warped, H, W, D,
                                 p->sigma_min, cref, ctar);
  return check_launch();
}

template <typename TL>
int dispatch_cost(const rsv_image& left, const float* warped, const rsv_params* p, float* cref,
                  float* ctar, hipStream_t st) {
  switch (p->block_radius) {
    case 1: return launch_cost<1, TL>(left, warped, p, cref, ctar, st);
    case 2: return launch_cost<2, TL>(left, warped, p, cref, ctar, st);
    case 3: return launch_cost<3, TL>(left, warped, p, cref, ctar, st);
    case 4: return launch_cost<4, TL>(left, warped, p, cref, ctar, st);
    default: return RSV_E_PARAM;
  }
}

}  // namespace rsv

extern "C" int rsv_cost_volume(rsv_image left, const float* warped, const rsv_params* p,
                               float* cost_ref, float* cost_tar, void* stream) {
  using namespace rsv;
  if (int s = validate_image(left)) return s;
  if (int s = validate_cost_params(p)) return s;
  if (!warped || !cost_ref) return RSV_E_NULL;
  if (!aligned(warped, 4) || !aligned(cost_ref, 4) || (cost_tar && !aligned(cost_tar, 4)))
    return RSV_E_ALIGN;
  const int K = 2 * p->block_radius + 1;
  if (left.height < K || left.width < K) return RSV_E_SHAPE;
  hipStream_t st = as_stream(stream);
  if (left.dtype == RSV_U8) return dispatch_cost<uint8_t>(left, warped, p, cost_ref, cost_tar, st);
  return dispatch_cost<float>(left, warped, p, cost_ref, cost_tar, st);
}
