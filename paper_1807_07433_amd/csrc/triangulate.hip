// rsv_triangulate: post-processing (Sec. II-C) and 3-D reconstruction (Sec. II-D).
// The warp shift is added back at the matched target column, d_f = d_s + s(u - d_s, v),
// and the rectified pinhole model gives z = f T / d_f, x = (u - u0) z / f,
// y = (v - v0) z / f.  Arithmetic in double, rounded once.
#include <math.h>

#include "warp_math.hpp"

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
  const double ds = static_cast<double>(dsub[i]);
  const double df = ds + (pl.a0 + pl.a1 * static_cast<double>(v) +
                          pl.a2 * (static_cast<double>(u) - ds) - pl.delta);
  if (dfin) dfin[i] = static_cast<float>(df);
  if (xyz) {
    float* o = xyz + 3 * i;
    if (valid[i] && df > 0.0) {
      const double z = cam.f * cam.baseline / df;
      o[0] = static_cast<float>((static_cast<double>(u) - cam.u0) * z / cam.f);
      o[1] = static_cast<float>((static_cast<double>(v) - cam.v0) * z / cam.f);
      o[2] = static_cast<float>(z);
    } else {
      o[0] = o[1] = o[2] = NAN;
    }
  }
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
