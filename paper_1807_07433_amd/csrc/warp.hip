// rsv_warp: perspective transformation of the target image (Sec. II-A).
#include "warp_math.hpp"

namespace rsv {

template <typename T>
__global__ __launch_bounds__(256) void warp_kernel(const T* __restrict__ right, int64_t pitch,
                                                   int H, int W, rsv_plane pl,
                                                   float* __restrict__ out) {
  const int u = blockIdx.x * blockDim.x + threadIdx.x;
  const int v = blockIdx.y;
  if (u >= W || v >= H) return;
  out[static_cast<int64_t>(v) * W + u] = warp_sample(right, pitch, W, pl, u, v);
}

}  // namespace rsv

extern "C" int rsv_warp(rsv_image right, rsv_plane plane, float* warped, void* stream) {
  using namespace rsv;
  if (int s = validate_image(right)) return s;
  if (!warped) return RSV_E_NULL;
  if (!aligned(warped, 4)) return RSV_E_ALIGN;
  const dim3 block(256);
  const dim3 grid((right.width + 255) / 256, right.height);
  hipStream_t st = as_stream(stream);
  if (right.dtype == RSV_U8)
    warp_kernel<uint8_t><<<grid, block, 0, st>>>(static_cast<const uint8_t*>(right.data), right.pitch,
                                                 right.height, right.width, plane, warped);
  else
    warp_kernel<float><<<grid, block, 0, st>>>(static_cast<const float*>(right.data), right.pitch,
                                               right.height, right.width, plane, warped);
  return check_launch();
}
