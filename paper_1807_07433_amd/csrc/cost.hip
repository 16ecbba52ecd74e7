// rsv_cost_volume, rsv_cost_volume_joint: ZNCC reference and target cost volumes
// (Sec. II-B.1, Eq. 3-5), as two dense volumes or as one joint volume.
// One block per tile of 64 left-block centres x cost_tile_rows<R>() rows: the direct
// tile (cost_tile.hpp) for 3x3 and 5x5 blocks, the sliding-sum tile (cost_box.hpp)
// for 7x7 and 9x9.  The grid spans centres u = 0 .. W + D - 2 so that the target
// volume is filled where x + d leaves the image.
#include "cost_box.hpp"

namespace rsv {

template <int R, typename TL, bool TAR>
__global__ __launch_bounds__(cost_tile_threads<R>(), cost_uses_box<R>() ? 1 : 4) void cost_volume_kernel(
    const TL* __restrict__ left, int64_t lpitch, const float* __restrict__ warped, int H, int W,
    int D, float sigma_min, CostOut out) {
  extern __shared__ __align__(16) unsigned char smem[];
  auto warped_at = [&](int y, int x) { return warped[static_cast<int64_t>(y) * W + x]; };
  cost_tile_for<R, TAR>(left, lpitch, warped_at, H, W, D, sigma_min, blockIdx.x * kCostTW,
                        blockIdx.y * cost_tile_rows<R>(), out, smem);
}

template <int R, typename TL>
int launch_cost(const rsv_image& left, const float* warped, const rsv_params* p, const CostOut& out,
                hipStream_t st) {
  const int H = left.height, W = left.width, D = p->D;
  const size_t lds = cost_tile_lds(R, D);
  const dim3 block(cost_tile_threads<R>());
  const dim3 grid((W + D - 1 + kCostTW - 1) / kCostTW, (H + cost_tile_rows<R>() - 1) / cost_tile_rows<R>());
  auto kern = out.tar ? cost_volume_kernel<R, TL, true> : cost_volume_kernel<R, TL, false>;
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
    if (e != hipSuccess) {
      set_hip_error(e);
      return RSV_E_HIP;
    }
  }
  kern<<<grid, block, lds, st>>>(static_cast<const TL*>(left.data), left.pitch, warped, H, W, D,
                                 p->sigma_min, out);
  return check_launch();
}

template <typename TL>
int dispatch_cost(const rsv_image& left, const float* warped, const rsv_params* p, const CostOut& out,
                  hipStream_t st) {
  switch (p->block_radius) {
    case 1: return launch_cost<1, TL>(left, warped, p, out, st);
    case 2: return launch_cost<2, TL>(left, warped, p, out, st);
    case 3: return launch_cost<3, TL>(left, warped, p, out, st);
    case 4: return launch_cost<4, TL>(left, warped, p, out, st);
    default: return RSV_E_PARAM;
  }
}

int run_cost(const rsv_image& left, const float* warped, const rsv_params* p, const CostOut& out,
             void* stream) {
  hipStream_t st = as_stream(stream);
  if (left.dtype == RSV_U8) return dispatch_cost<uint8_t>(left, warped, p, out, st);
  return dispatch_cost<float>(left, warped, p, out, st);
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
  return run_cost(left, warped, p, cost_out_dual(cost_ref, cost_tar, left.height, left.width), stream);
}

extern "C" int rsv_cost_volume_joint(rsv_image left, const float* warped, const rsv_params* p,
                                     float* joint, int64_t row_stride, void* stream) {
  using namespace rsv;
  if (int s = validate_image(left)) return s;
  if (int s = validate_cost_params(p)) return s;
  if (!warped || !joint) return RSV_E_NULL;
  if (!aligned(warped, 4) || !aligned(joint, 4)) return RSV_E_ALIGN;
  const int K = 2 * p->block_radius + 1;
  if (left.height < K || left.width < K) return RSV_E_SHAPE;
  if (row_stride < static_cast<int64_t>(left.width) + p->D - 1 ||
      static_cast<int64_t>(left.height) * row_stride > INT32_MAX)
    return RSV_E_SHAPE;
  return run_cost(left, warped, p, cost_out_joint(joint, row_stride, left.height, left.width, p->D), stream);
}
