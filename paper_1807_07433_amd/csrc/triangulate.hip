// rsv_triangulate: post-processing (Sec. II-C) and 3-D reconstruction (Sec. II-D).
// The warp shift is added back at the matched target column, d_f = d_s + s(u - d_s, v),
// and the rectified pinhole model gives z = f T / d_f, x = (u - u0) z / f,
// y = (v - v0) z / f.  Arithmetic in double, rounded once.
#include <math.h>

#include "select_math.hpp"

namespace rsv {

__global__ __launch_bounds__(256) void triangulate_kernel(const float* __restrict__ dsub,
                                                          const uint8_t* __restrict__ valid,
                                                          int H, int W, rsv_plane pl,
                                                          rsv_camera cam, float* __restrict__ dfin,
                                                          float* __restrict__ xyz) {
  const int u = blockIdx.x * blockDim.x + threadIdx.x;
  const int v = blockIdx.y;
  if (u >= W || v >= H) return;
  const int64_t i = static_cast<int64_t>(v) * W + u;
  postprocess_point(dsub[i], valid[i] != 0, u, v, pl, cam, dfin ? dfin + i : nullptr,
                    xyz ? xyz + 3 * i : nullptr);
}

}  // namespace rsv

extern "C" int rsv_triangulate(const float* disp_sub, const uint8_t* valid, int32_t height,
                               int32_t width, rsv_plane plane, rsv_camera cam, float* disp_final,
                               float* xyz, void* stream) {
  using namespace rsv;
  if (!disp_sub || !valid) return RSV_E_NULL;
  if (!disp_final && !xyz) return RSV_E_NULL;
  if (height < 1 || width < 1) return RSV_E_SHAPE;
  if (!(cam.f > 0.0) || !(cam.baseline > 0.0)) return RSV_E_PARAM;
  if (!aligned(disp_sub, 4) || (disp_final && !aligned(disp_final, 4)) || (xyz && !aligned(xyz, 4)))
    return RSV_E_ALIGN;
  triangulate_kernel<<<dim3((width + 255) / 256, height), dim3(256), 0, as_stream(stream)>>>(
      disp_sub, valid, height, width, plane, cam, disp_final, xyz);
  return check_launch();
}
