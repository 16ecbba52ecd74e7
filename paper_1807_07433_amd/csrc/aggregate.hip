// rsv_aggregate, rsv_aggregate_strided, rsv_aggregate_argmax: bilateral cost
// aggregation (Sec. II-B.2, Eq. 8-10) of a dense volume or of any strided view (e.g.
// of the joint cost volume), writing the aggregated volume or only its argmax over d
// (the target volume's use in Sec. II-B.3).
//
// The weights of Eq. 9-10 depend on the pixel pair only, never on d, so the
// aggregation of a 4 x 4 patch over 16 disparities is a small matrix product with a
// banded weight matrix, run on the matrix cores (aggregate_mfma.hpp).  Each block
// owns a 16 x 16 output tile.  Its cost tiles come into LDS by direct loads
// (agg_tile_dma.hpp; rho <= 5, W >= 4) or through registers (agg_tile.hpp), and its
// results leave one 16-disparity tile at a time through a sink: the volume's planes
// (non-temporal stores) or the running argmax (argmax_sink.hpp).
#include <climits>

#include "agg_tile_dma.hpp"
#include "argmax_sink.hpp"
#include "select_math.hpp"
#include "wta_sink.hpp"

namespace rsv {

// Output rows per block: 16 (1024 threads, one block per CU).  8-row tiles of 512
// threads run two blocks per CU but measured about 5% slower (more halo per output,
// two barriers per disparity tile with a single output buffer).
constexpr int kAggTileRows = 16;

// Tiles are taken in runs of kAggXcdRun per XCD (xcd_run_item, rsv_internal.hpp): each
// XCD works through runs of horizontally adjacent tiles, which share halo columns in its
// L2, while the whole GPU stays on one stretch of the image (the shared cache holds its
// rows).  At 1280x720, runs of 40 measured 1.5% faster than one band of the image per
// XCD and equal to runs of 20; enumerating the tiles in strips of 4 tile rows, column by
// column, measured about 4% slower than bands.
constexpr int kAggXcdRun = 40;

// agg_tile sink that writes each 16-disparity tile into the output volume: thread i
// moves 4 consecutive pixels of one row of one plane (a wave covers 16 rows or a
// whole 8 x 16 plane tile, 64-byte row segments), as one float4 store when rows are
// 16-byte aligned.
template <int TY>
struct VolumeSink {
  float* agg;
  int H, W, D, by, bx;
  bool vec4;

  __device__ __forceinline__ void operator()(int t, const float* o) {
    using G = AggGeo<1, TY>;  // NT and OST do not depend on the radius
    for (int i = threadIdx.x; i < 64 * TY; i += G::NT) {
      const int dd = i / (4 * TY), rem = i - dd * (4 * TY);
      const int row = rem >> 2, c4 = (rem & 3) << 2;
      const int d = 16 * t + dd, Y = by + row, X = bx + c4;
      if (d < D && Y < H && X < W) {
        const float4_t v = *reinterpret_cast<const float4_t*>(o + dd * G::OST + row * 16 + c4);
        float* p = agg + d * (static_cast<int64_t>(H) * W) + static_cast<int64_t>(Y) * W + X;
        // Non-temporal: the aggregated volume is read only by a later kernel, and
        // allocating it in the caches evicts the cost volume the next aggregation
        // still reads (with the joint volume both aggregations read the same one).
        if (vec4 && X + 3 < W) {
          __builtin_nontemporal_store(v, reinterpret_cast<float4_t*>(p));
        } else {
#pragma unroll
          for (int e = 0; e < 4; ++e)
            if (X + e < W) __builtin_nontemporal_store(v[e], p + e);
        }
      }
    }
  }
};

// ARG: write the argmax map `disp` instead of the volume `agg`.
template <int A, int TY, typename TG, bool ARG>
__global__ __launch_bounds__(64 * TY, 4) void aggregate_kernel(
    const float* __restrict__ cost, int64_t cps, int crs, const TG* __restrict__ guide, int64_t gpitch,
    int H, int W, int D, BilateralK bk, bool vec4, float* __restrict__ agg, int32_t* __restrict__ disp) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int tiles_x = (W + 15) >> 4, tiles_y = (H + TY - 1) / TY;
  const int tile = xcd_run_item<kAggXcdRun>(blockIdx.x, tiles_x * tiles_y);
  const int by = (tile / tiles_x) * TY, bx = (tile % tiles_x) * 16;
  auto guide_at = [&](int Y, int X) { return pixel(guide, gpitch, Y, X); };
  if constexpr (ARG) {
    static_assert(TY == 16, "the argmax sink covers 16 x 16 pixels");
    ArgmaxSink sink{D, reinterpret_cast<float*>(smem + agg_tile_lds_bytes<A, TY>())};
    agg_tile<A, TY>(cost, cps, crs, H, W, D, bk, by, bx, guide_at, sink, smem);
    sink.finish(disp, H, W, by, bx);
  } else {
    VolumeSink<TY> sink{agg, H, W, D, by, bx, vec4};
    agg_tile<A, TY>(cost, cps, crs, H, W, D, bk, by, bx, guide_at, sink, smem);
  }
}

// The same tile with its cost tiles loaded straight into LDS ahead of use
// (agg_tile_dma.hpp): used when its buffers fit one CU's LDS (rho <= 5) and W >= 4.
template <int A, typename TG, bool ARG>
__global__ __launch_bounds__(1024) void aggregate_dma_kernel(
    const float* __restrict__ cost, int64_t cps, int crs, const TG* __restrict__ guide, int64_t gpitch,
    int H, int W, int D, BilateralK bk, bool vec4, float* __restrict__ agg, int32_t* __restrict__ disp) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int tiles_x = (W + 15) >> 4, tiles_y = (H + 15) >> 4;
  const int tile = xcd_run_item<kAggXcdRun>(blockIdx.x, tiles_x * tiles_y);
  const int by = (tile / tiles_x) * 16, bx = (tile % tiles_x) * 16;
  auto guide_at = [&](int Y, int X) { return pixel(guide, gpitch, Y, X); };
  if constexpr (ARG) {
    ArgmaxSink sink{D};
    agg_tile_dma<A>(cost, cps, crs, H, W, D, bk, by, bx, guide_at, sink, smem, lds_address(smem));
    sink.finish(disp, H, W, by, bx);
  } else {
    VolumeSink<16> sink{agg, H, W, D, by, bx, vec4};
    agg_tile_dma<A>(cost, cps, crs, H, W, D, bk, by, bx, guide_at, sink, smem, lds_address(smem));
  }
}

template <int A, typename TG, bool ARG>
int launch_agg_dma(const float* cost, int64_t cps, int crs, const rsv_image& g, const rsv_params* p,
                   float* agg, int32_t* disp, hipStream_t st) {
  const int tiles = ((g.width + 15) / 16) * ((g.height + 15) / 16);
  const BilateralK bk = bilateral_constants(p->gamma_d, p->gamma_r);
  const bool vec4 = (g.width % 4) == 0 && aligned(agg, 16);
  const size_t lds = agg_tile_dma_lds_bytes<A>();
  auto kern = aggregate_dma_kernel<A, TG, ARG>;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
  if (e != hipSuccess) {
    set_hip_error(e);
    return RSV_E_HIP;
  }
  kern<<<dim3(tiles), dim3(1024), lds, st>>>(cost, cps, crs, static_cast<const TG*>(g.data), g.pitch,
                                             g.height, g.width, p->D, bk, vec4, agg, disp);
  return check_launch();
}

// The reference aggregation with the selection folded in: the LDS-loaded tile feeds
// RefQuadSink, and each pixel's four lanes end with the winner (ties to the lowest
// d), Eq. 12 on it and its neighbours, and Eq. 11 against the target map `dtar`
// (complete before this launch), written as the select kernels write them.
template <int A, typename TG>
__global__ __launch_bounds__(1024) void aggregate_select_kernel(
    const float* __restrict__ cost, int64_t cps, int crs, const TG* __restrict__ guide, int64_t gpitch,
    int H, int W, int D, BilateralK bk, int tau, const int32_t* __restrict__ dtar,
    int32_t* __restrict__ dref, float* __restrict__ dsub, uint8_t* __restrict__ valid) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int tiles_x = (W + 15) >> 4, tiles_y = (H + 15) >> 4;
  const int tile = xcd_run_item<kAggXcdRun>(blockIdx.x, tiles_x * tiles_y);
  const int by = (tile / tiles_x) * 16, bx = (tile % tiles_x) * 16;
  auto guide_at = [&](int Y, int X) { return pixel(guide, gpitch, Y, X); };
  RefQuadSink sink{D};
  agg_tile_dma<A>(cost, cps, crs, H, W, D, bk, by, bx, guide_at, sink, smem, lds_address(smem));
  if ((threadIdx.x & 3) != 0) return;  // the four lanes of a pixel hold the same result
  const int q = threadIdx.x >> 2;
  const int Y = by + (q >> 4), X = bx + (q & 15);
  if (Y >= H || X >= W) return;
  const int64_t row = static_cast<int64_t>(Y) * W, i = row + X;
  const int a = sink.arg, x = X - a;
  dref[i] = a;
  dsub[i] = parabola(a, sink.best, sink.am, sink.ap, D);
  valid[i] = (x >= 0 && abs(a - dtar[row + (x < 0 ? 0 : x)]) <= tau) ? 1 : 0;
}

template <int A, typename TG>
int launch_agg_select(const float* cost, int64_t cps, int crs, const rsv_image& g, const rsv_params* p,
                      const int32_t* dtar, int32_t* dref, float* dsub, uint8_t* valid, hipStream_t st) {
  if constexpr (agg_dma_fits<A>()) {
    const int tiles = ((g.width + 15) / 16) * ((g.height + 15) / 16);
    const BilateralK bk = bilateral_constants(p->gamma_d, p->gamma_r);
    const size_t lds = agg_tile_dma_lds_bytes<A>();
    auto kern = aggregate_select_kernel<A, TG>;
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
    if (e != hipSuccess) {
      set_hip_error(e);
      return RSV_E_HIP;
    }
    kern<<<dim3(tiles), dim3(1024), lds, st>>>(cost, cps, crs, static_cast<const TG*>(g.data), g.pitch, g.height,
                                               g.width, p->D, bk, p->lr_threshold, dtar, dref, dsub, valid);
    return check_launch();
  } else {
    return RSV_E_PARAM;  // the LDS-loaded tile does not fit this radius
  }
}

template <typename TG>
int dispatch_agg_select(const float* cost, int64_t cps, int crs, const rsv_image& g, const rsv_params* p,
                        const int32_t* dtar, int32_t* dref, float* dsub, uint8_t* valid, hipStream_t st) {
  switch (p->agg_radius) {
    case 1: return launch_agg_select<1, TG>(cost, cps, crs, g, p, dtar, dref, dsub, valid, st);
    case 2: return launch_agg_select<2, TG>(cost, cps, crs, g, p, dtar, dref, dsub, valid, st);
    case 3: return launch_agg_select<3, TG>(cost, cps, crs, g, p, dtar, dref, dsub, valid, st);
    case 4: return launch_agg_select<4, TG>(cost, cps, crs, g, p, dtar, dref, dsub, valid, st);
    case 5: return launch_agg_select<5, TG>(cost, cps, crs, g, p, dtar, dref, dsub, valid, st);
    default: return RSV_E_PARAM;
  }
}

// ------------------------------------------- both views in one launch
// Items come row by row of tiles, the reference tiles of a tile row next to its
// target tiles, so both views' reads of the same rows of the joint volume come close
// together in time; XCDs take the items in runs of kViewsXcdRun (one tile row of both
// views at 1280 columns).  One launch of 2T tiles also leaves one partial last round of
// blocks instead of two.  Measured at 1280x720, D = 64 against the target argmax and
// the reference selection as two launches: 0.469 -> 0.443 ms (runs of 80; 20: 0.456,
// 40: 0.447); later, with the conversion beside the MFMAs, runs of 80 / 160 / 240 / 320
// gave 0.433 / 0.430 / 0.433 / 0.431 ms, and interleaving the two views tile by tile
// instead of row by row gained nothing.
constexpr int kViewsXcdRun = 160;

template <int A, typename TGR>
__global__ __launch_bounds__(1024) void aggregate_views_kernel(
    const float* __restrict__ cref, int64_t rps, int rrs, const float* __restrict__ ctar, int64_t tps, int trs,
    const TGR* __restrict__ gref, int64_t grp, const float* __restrict__ gtar, int64_t gtp, int H, int W, int D,
    BilateralK bk, int32_t* __restrict__ dtar, int32_t* __restrict__ dref, float* __restrict__ dsub) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int tiles_x = (W + 15) >> 4, tiles_y = (H + 15) >> 4;
  const int k = xcd_run_item<kViewsXcdRun>(blockIdx.x, 2 * tiles_x * tiles_y);
  const int ty = k / (2 * tiles_x), r = k - ty * 2 * tiles_x;
  const bool ref = r < tiles_x;  // uniform per block
  const int by = ty * 16, bx = (ref ? r : r - tiles_x) * 16;
  if (ref) {
    auto guide_at = [&](int Y, int X) { return pixel(gref, grp, Y, X); };
    RefQuadSink sink{D};
    agg_tile_dma<A>(cref, rps, rrs, H, W, D, bk, by, bx, guide_at, sink, smem, lds_address(smem));
    const int q = threadIdx.x >> 2;
    const int Y = by + (q >> 4), X = bx + (q & 15);
    if ((threadIdx.x & 3) == 0 && Y < H && X < W) {  // the four lanes of a pixel hold the same result
      const int64_t i = static_cast<int64_t>(Y) * W + X;
      dref[i] = sink.arg;
      dsub[i] = parabola(sink.arg, sink.best, sink.am, sink.ap, D);
    }
  } else {
    auto guide_at = [&](int Y, int X) { return pixel(gtar, gtp, Y, X); };
    ArgmaxSink sink{D};
    agg_tile_dma<A>(ctar, tps, trs, H, W, D, bk, by, bx, guide_at, sink, smem, lds_address(smem));
    sink.finish(dtar, H, W, by, bx);
  }
}

// Both views on the register-staged tile (agg_tile.hpp), for windows the LDS-loaded
// tile does not take (rho = 6, or W < 4): the item order of the kernel above, and per
// block the select kernel's scan over d through WtaSink (wta_sink.hpp), so the maps
// equal those of the unfused path (aggregation, then selection) bit for bit.
template <int A, typename TGR>
__global__ __launch_bounds__(1024) void aggregate_views_rs_kernel(
    const float* __restrict__ cref, int64_t rps, int rrs, const float* __restrict__ ctar, int64_t tps, int trs,
    const TGR* __restrict__ gref, int64_t grp, const float* __restrict__ gtar, int64_t gtp, int H, int W, int D,
    BilateralK bk, int32_t* __restrict__ dtar, int32_t* __restrict__ dref, float* __restrict__ dsub) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int tiles_x = (W + 15) >> 4, tiles_y = (H + 15) >> 4;
  const int k = xcd_run_item<kViewsXcdRun>(blockIdx.x, 2 * tiles_x * tiles_y);
  const int ty = k / (2 * tiles_x), r = k - ty * 2 * tiles_x;
  const bool ref = r < tiles_x;  // uniform per block
  const int by = ty * 16, bx = (ref ? r : r - tiles_x) * 16;
  WtaState* st = reinterpret_cast<WtaState*>(smem + agg_tile_lds_bytes<A, 16>());
  WtaSink sink{st, D, ref};
  if (ref) {
    auto guide_at = [&](int Y, int X) { return pixel(gref, grp, Y, X); };
    agg_tile<A, 16>(cref, rps, rrs, H, W, D, bk, by, bx, guide_at, sink, smem);
  } else {
    auto guide_at = [&](int Y, int X) { return pixel(gtar, gtp, Y, X); };
    agg_tile<A, 16>(ctar, tps, trs, H, W, D, bk, by, bx, guide_at, sink, smem);
  }
  // thread q < 256 wrote its own pixel's state in the last sink call
  if (threadIdx.x < 256) {
    const int q = threadIdx.x;
    const int Y = by + (q >> 4), X = bx + (q & 15);
    if (Y < H && X < W) {
      const int64_t i = static_cast<int64_t>(Y) * W + X;
      if (ref) {
        dref[i] = st->arg[q];
        dsub[i] = parabola(st->arg[q], st->best[q], st->am[q], st->ap[q], D);
      } else {
        dtar[i] = st->arg[q];
      }
    }
  }
}

template <int A, typename TGR>
int launch_agg_views_rs(const float* cref, int64_t rps, int rrs, const float* ctar, int64_t tps, int trs,
                        const rsv_image& gr, const rsv_image& gt, const rsv_params* p, int32_t* dtar, int32_t* dref,
                        float* dsub, hipStream_t st) {
  const int tiles = ((gr.width + 15) / 16) * ((gr.height + 15) / 16);
  const BilateralK bk = bilateral_constants(p->gamma_d, p->gamma_r);
  const size_t lds = agg_tile_lds_bytes<A, 16>() + sizeof(WtaState);
  auto kern = aggregate_views_rs_kernel<A, TGR>;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                                     static_cast<int>(lds));
  if (e != hipSuccess) {
    set_hip_error(e);
    return RSV_E_HIP;
  }
  kern<<<dim3(2 * tiles), dim3(1024), lds, st>>>(cref, rps, rrs, ctar, tps, trs, static_cast<const TGR*>(gr.data),
                                                 gr.pitch, static_cast<const float*>(gt.data), gt.pitch, gr.height,
                                                 gr.width, p->D, bk, dtar, dref, dsub);
  return check_launch();
}

template <int A, typename TGR>
int launch_agg_views(const float* cref, int64_t rps, int rrs, const float* ctar, int64_t tps, int trs,
                     const rsv_image& gr, const rsv_image& gt, const rsv_params* p, int32_t* dtar, int32_t* dref,
                     float* dsub, hipStream_t st) {
  if constexpr (agg_dma_fits<A>()) {
    const int tiles = ((gr.width + 15) / 16) * ((gr.height + 15) / 16);
    const BilateralK bk = bilateral_constants(p->gamma_d, p->gamma_r);
    const size_t lds = agg_tile_dma_lds_bytes<A>();
    auto kern = aggregate_views_kernel<A, TGR>;
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
    if (e != hipSuccess) {
      set_hip_error(e);
      return RSV_E_HIP;
    }
    kern<<<dim3(2 * tiles), dim3(1024), lds, st>>>(cref, rps, rrs, ctar, tps, trs, static_cast<const TGR*>(gr.data),
                                                   gr.pitch, static_cast<const float*>(gt.data), gt.pitch, gr.height,
                                                   gr.width, p->D, bk, dtar, dref, dsub);
    return check_launch();
  } else {
    return RSV_E_PARAM;
  }
}

template <typename TGR>
int dispatch_agg_views(const float* cref, int64_t rps, int rrs, const float* ctar, int64_t tps, int trs,
                       const rsv_image& gr, const rsv_image& gt, const rsv_params* p, int32_t* dtar, int32_t* dref,
                       float* dsub, hipStream_t st) {
  if (p->agg_radius > 5 || gr.width < 4) {  // the register-staged tile
    switch (p->agg_radius) {
      case 1: return launch_agg_views_rs<1, TGR>(cref, rps, rrs, ctar, tps, trs, gr, gt, p, dtar, dref, dsub, st);
      case 2: return launch_agg_views_rs<2, TGR>(cref, rps, rrs, ctar, tps, trs, gr, gt, p, dtar, dref, dsub, st);
      case 3: return launch_agg_views_rs<3, TGR>(cref, rps, rrs, ctar, tps, trs, gr, gt, p, dtar, dref, dsub, st);
      case 4: return launch_agg_views_rs<4, TGR>(cref, rps, rrs, ctar, tps, trs, gr, gt, p, dtar, dref, dsub, st);
      case 5: return launch_agg_views_rs<5, TGR>(cref, rps, rrs, ctar, tps, trs, gr, gt, p, dtar, dref, dsub, st);
      case 6: return launch_agg_views_rs<6, TGR>(cref, rps, rrs, ctar, tps, trs, gr, gt, p, dtar, dref, dsub, st);
      default: return RSV_E_PARAM;
    }
  }
  switch (p->agg_radius) {
    case 1: return launch_agg_views<1, TGR>(cref, rps, rrs, ctar, tps, trs, gr, gt, p, dtar, dref, dsub, st);
    case 2: return launch_agg_views<2, TGR>(cref, rps, rrs, ctar, tps, trs, gr, gt, p, dtar, dref, dsub, st);
    case 3: return launch_agg_views<3, TGR>(cref, rps, rrs, ctar, tps, trs, gr, gt, p, dtar, dref, dsub, st);
    case 4: return launch_agg_views<4, TGR>(cref, rps, rrs, ctar, tps, trs, gr, gt, p, dtar, dref, dsub, st);
    case 5: return launch_agg_views<5, TGR>(cref, rps, rrs, ctar, tps, trs, gr, gt, p, dtar, dref, dsub, st);
    default: return RSV_E_PARAM;
  }
}

// ------------------------------------------------- restricted search (Sec. IV)
// Each pixel aggregates only the window of `width` disparities around its calculated
// (unaggregated winner-take-all) disparity, lo = clamp(coarse - radius, 0, D - width).
// A block aggregates the consecutive 16-disparity tiles that cover all its pixels'
// windows widened by one on each side (Eq. 12's neighbours; clamped to the range),
// and the sinks take each pixel's winner inside its own window.  Every aggregated
// value is the full method's float (same tile, same arithmetic).

// The window of the thread's pixel (thread i covers pixel i / 4 of the 16 x 16 block),
// and the block's tile range [t_first, t_first + t_count).  Pixels outside the image
// do not widen the range.
__device__ __forceinline__ void restricted_tiles(const int32_t* __restrict__ coarse, int H, int W, int D,
                                                 int radius, int width, int by, int bx, int* s_range, int& lo,
                                                 int& hi, int& t_first, int& t_count) {
  const int p = threadIdx.x >> 2;
  const int Y = by + (p >> 4), X = bx + (p & 15);
  const bool in = Y < H && X < W;
  const int c = in ? coarse[static_cast<int64_t>(Y) * W + X] : 0;
  lo = clampi(c - radius, 0, D - width);
  hi = lo + width - 1;
  int mn = in ? lo : INT_MAX, mx = in ? hi : -1;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    mn = min(mn, __shfl_xor(mn, off));
    mx = max(mx, __shfl_xor(mx, off));
  }
  if (threadIdx.x == 0) {
    s_range[0] = INT_MAX;
    s_range[1] = -1;
  }
  __syncthreads();
  if ((threadIdx.x & 63) == 0) {
    atomicMin(&s_range[0], mn);
    atomicMax(&s_range[1], mx);
  }
  __syncthreads();
  const int dlo = max(s_range[0] - 1, 0), dhi = min(s_range[1] + 1, D - 1);
  t_first = __builtin_amdgcn_readfirstlane(dlo >> 4);
  t_count = __builtin_amdgcn_readfirstlane((dhi >> 4) - (dlo >> 4) + 1);
}

template <int A, typename TG>
__global__ __launch_bounds__(1024) void aggregate_restricted_argmax_kernel(
    const float* __restrict__ cost, int64_t cps, int crs, const TG* __restrict__ guide, int64_t gpitch, int H,
    int W, int D, BilateralK bk, const int32_t* __restrict__ coarse, int radius, int width,
    int32_t* __restrict__ disp) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int s_range[2];
  const int tiles_x = (W + 15) >> 4, tiles_y = (H + 15) >> 4;
  const int tile = xcd_run_item<kAggXcdRun>(blockIdx.x, tiles_x * tiles_y);
  const int by = (tile / tiles_x) * 16, bx = (tile % tiles_x) * 16;
  int lo, hi, t_first, t_count;
  restricted_tiles(coarse, H, W, D, radius, width, by, bx, s_range, lo, hi, t_first, t_count);
  if (t_count <= 0) return;  // no pixel of the block in the image
  auto guide_at = [&](int Y, int X) { return pixel(guide, gpitch, Y, X); };
  ArgmaxSink sink{D};
  sink.lo = lo;
  sink.hi = hi;
  agg_tile_dma<A>(cost, cps, crs, H, W, D, bk, by, bx, guide_at, sink, smem, lds_address(smem), t_first, t_count);
  sink.finish(disp, H, W, by, bx);
}

template <int A, typename TG>
__global__ __launch_bounds__(1024) void aggregate_restricted_select_kernel(
    const float* __restrict__ cost, int64_t cps, int crs, const TG* __restrict__ guide, int64_t gpitch, int H,
    int W, int D, BilateralK bk, const int32_t* __restrict__ coarse, int radius, int width, int tau,
    const int32_t* __restrict__ dtar, int32_t* __restrict__ dref, float* __restrict__ dsub,
    uint8_t* __restrict__ valid) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int s_range[2];
  const int tiles_x = (W + 15) >> 4, tiles_y = (H + 15) >> 4;
  const int tile = xcd_run_item<kAggXcdRun>(blockIdx.x, tiles_x * tiles_y);
  const int by = (tile / tiles_x) * 16, bx = (tile % tiles_x) * 16;
  int lo, hi, t_first, t_count;
  restricted_tiles(coarse, H, W, D, radius, width, by, bx, s_range, lo, hi, t_first, t_count);
  if (t_count <= 0) return;
  auto guide_at = [&](int Y, int X) { return pixel(guide, gpitch, Y, X); };
  RefQuadSink sink{D};
  sink.lo = lo;
  sink.hi = hi;
  agg_tile_dma<A>(cost, cps, crs, H, W, D, bk, by, bx, guide_at, sink, smem, lds_address(smem), t_first, t_count);
  if ((threadIdx.x & 3) != 0) return;
  const int q = threadIdx.x >> 2;
  const int Y = by + (q >> 4), X = bx + (q & 15);
  if (Y >= H || X >= W) return;
  const int64_t row = static_cast<int64_t>(Y) * W, i = row + X;
  const int a = sink.arg, x = X - a;
  dref[i] = a;
  dsub[i] = parabola(a, sink.best, sink.am, sink.ap, D);
  valid[i] = (x >= 0 && abs(a - dtar[row + (x < 0 ? 0 : x)]) <= tau) ? 1 : 0;
}

// Both views' restricted aggregations in one launch, in aggregate_views_kernel's
// item order: reference tiles as aggregate_restricted_select_kernel without Eq. 11
// (winner in the window and Eq. 12), target tiles as the restricted argmax.
template <int A, typename TGR>
__global__ __launch_bounds__(1024) void aggregate_restricted_views_kernel(
    const float* __restrict__ cref, int64_t rps, int rrs, const float* __restrict__ ctar, int64_t tps, int trs,
    const TGR* __restrict__ gref, int64_t grp, const float* __restrict__ gtar, int64_t gtp, int H, int W, int D,
    BilateralK bk, const int32_t* __restrict__ coarse_ref, const int32_t* __restrict__ coarse_tar, int radius,
    int width, int32_t* __restrict__ dtar, int32_t* __restrict__ dref, float* __restrict__ dsub) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int s_range[2];
  const int tiles_x = (W + 15) >> 4, tiles_y = (H + 15) >> 4;
  const int k = xcd_run_item<kViewsXcdRun>(blockIdx.x, 2 * tiles_x * tiles_y);
  const int ty = k / (2 * tiles_x), r = k - ty * 2 * tiles_x;
  const bool ref = r < tiles_x;  // uniform per block
  const int by = ty * 16, bx = (ref ? r : r - tiles_x) * 16;
  int lo, hi, t_first, t_count;
  restricted_tiles(ref ? coarse_ref : coarse_tar, H, W, D, radius, width, by, bx, s_range, lo, hi, t_first,
                   t_count);
  if (t_count <= 0) return;  // no pixel of the block in the image
  if (ref) {
    auto guide_at = [&](int Y, int X) { return pixel(gref, grp, Y, X); };
    RefQuadSink sink{D};
    sink.lo = lo;
    sink.hi = hi;
    agg_tile_dma<A>(cref, rps, rrs, H, W, D, bk, by, bx, guide_at, sink, smem, lds_address(smem), t_first,
                    t_count);
    const int q = threadIdx.x >> 2;
    const int Y = by + (q >> 4), X = bx + (q & 15);
    if ((threadIdx.x & 3) == 0 && Y < H && X < W) {
      const int64_t i = static_cast<int64_t>(Y) * W + X;
      dref[i] = sink.arg;
      dsub[i] = parabola(sink.arg, sink.best, sink.am, sink.ap, D);
    }
  } else {
    auto guide_at = [&](int Y, int X) { return pixel(gtar, gtp, Y, X); };
    ArgmaxSink sink{D};
    sink.lo = lo;
    sink.hi = hi;
    agg_tile_dma<A>(ctar, tps, trs, H, W, D, bk, by, bx, guide_at, sink, smem, lds_address(smem), t_first,
                    t_count);
    sink.finish(dtar, H, W, by, bx);
  }
}

template <int A, typename TGR>
int launch_restricted_views(const float* cref, int64_t rps, int rrs, const float* ctar, int64_t tps, int trs,
                            const rsv_image& gr, const rsv_image& gt, const rsv_params* p, const int32_t* cc_ref,
                            const int32_t* cc_tar, int radius, int32_t* dtar, int32_t* dref, float* dsub,
                            hipStream_t st) {
  if constexpr (agg_dma_fits<A>()) {
    const int tiles = ((gr.width + 15) / 16) * ((gr.height + 15) / 16);
    const BilateralK bk = bilateral_constants(p->gamma_d, p->gamma_r);
    const size_t lds = agg_tile_dma_lds_bytes<A>();
    const int width = 2 * radius + 1 < p->D ? 2 * radius + 1 : p->D;
    auto kern = aggregate_restricted_views_kernel<A, TGR>;
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
    if (e != hipSuccess) {
      set_hip_error(e);
      return RSV_E_HIP;
    }
    kern<<<dim3(2 * tiles), dim3(1024), lds, st>>>(cref, rps, rrs, ctar, tps, trs, static_cast<const TGR*>(gr.data),
                                                   gr.pitch, static_cast<const float*>(gt.data), gt.pitch, gr.height,
                                                   gr.width, p->D, bk, cc_ref, cc_tar, radius, width, dtar, dref,
                                                   dsub);
    return check_launch();
  } else {
    return RSV_E_PARAM;
  }
}

template <typename TGR>
int dispatch_restricted_views(const float* cref, int64_t rps, int rrs, const float* ctar, int64_t tps, int trs,
                              const rsv_image& gr, const rsv_image& gt, const rsv_params* p, const int32_t* cc_ref,
                              const int32_t* cc_tar, int radius, int32_t* dtar, int32_t* dref, float* dsub,
                              hipStream_t st) {
#define RSV_RV(A) \
  launch_restricted_views<A, TGR>(cref, rps, rrs, ctar, tps, trs, gr, gt, p, cc_ref, cc_tar, radius, dtar, dref, dsub, st)
  switch (p->agg_radius) {
    case 1: return RSV_RV(1);
    case 2: return RSV_RV(2);
    case 3: return RSV_RV(3);
    case 4: return RSV_RV(4);
    case 5: return RSV_RV(5);
    default: return RSV_E_PARAM;
  }
#undef RSV_RV
}

// Argument checks shared by the two-view entry points.
int validate_views(const float* cost_ref, int64_t rps, int64_t rrs, const float* cost_tar, int64_t tps, int64_t trs,
                   const rsv_image& gr, const rsv_image& gt, const rsv_params* p, const int32_t* dtar,
                   const int32_t* dref, const float* dsub) {
  if (int s = validate_image(gr)) return s;
  if (int s = validate_image(gt)) return s;
  if (int s = validate_agg_params(p)) return s;
  if (int s = validate_select_params(p)) return s;
  if (!cost_ref || !cost_tar || !dtar || !dref || !dsub) return RSV_E_NULL;
  if (!aligned(cost_ref, 4) || !aligned(cost_tar, 4) || !aligned(dtar, 4) || !aligned(dref, 4) || !aligned(dsub, 4))
    return RSV_E_ALIGN;
  if (gt.dtype != RSV_F32) return RSV_E_DTYPE;
  if (gt.width != gr.width || gt.height != gr.height) return RSV_E_SHAPE;
  const int64_t H = gr.height, W = gr.width;
  for (int64_t rs : {rrs, trs})
    if (rs < W || (H - 1) * rs + W > kAggMaxPixels) return RSV_E_SHAPE;
  for (int64_t ps : {rps, tps})
    if (ps < 1 || ps > kAggMaxPixels) return RSV_E_SHAPE;
  return RSV_OK;
}

template <int A, typename TG, bool SEL>
int launch_restricted(const float* cost, int64_t cps, int crs, const rsv_image& g, const rsv_params* p,
                      const int32_t* coarse, int radius, const int32_t* dtar, int32_t* dref, float* dsub,
                      uint8_t* valid, hipStream_t st) {
  if constexpr (agg_dma_fits<A>()) {
    const int tiles = ((g.width + 15) / 16) * ((g.height + 15) / 16);
    const BilateralK bk = bilateral_constants(p->gamma_d, p->gamma_r);
    const size_t lds = agg_tile_dma_lds_bytes<A>();
    const int width = 2 * radius + 1 < p->D ? 2 * radius + 1 : p->D;
    auto kern_sel = aggregate_restricted_select_kernel<A, TG>;
    auto kern_arg = aggregate_restricted_argmax_kernel<A, TG>;
    const void* kern = SEL ? reinterpret_cast<const void*>(kern_sel) : reinterpret_cast<const void*>(kern_arg);
    hipError_t e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
    if (e != hipSuccess) {
      set_hip_error(e);
      return RSV_E_HIP;
    }
    const TG* gd = static_cast<const TG*>(g.data);
    if constexpr (SEL)
      kern_sel<<<dim3(tiles), dim3(1024), lds, st>>>(cost, cps, crs, gd, g.pitch, g.height, g.width, p->D, bk,
                                                     coarse, radius, width, p->lr_threshold, dtar, dref, dsub,
                                                     valid);
    else
      kern_arg<<<dim3(tiles), dim3(1024), lds, st>>>(cost, cps, crs, gd, g.pitch, g.height, g.width, p->D, bk,
                                                     coarse, radius, width, dref);
    return check_launch();
  } else {
    return RSV_E_PARAM;  // the LDS-loaded tile does not fit this radius
  }
}

template <typename TG, bool SEL>
int dispatch_restricted(const float* cost, int64_t cps, int crs, const rsv_image& g, const rsv_params* p,
                        const int32_t* coarse, int radius, const int32_t* dtar, int32_t* dref, float* dsub,
                        uint8_t* valid, hipStream_t st) {
  switch (p->agg_radius) {
    case 1: return launch_restricted<1, TG, SEL>(cost, cps, crs, g, p, coarse, radius, dtar, dref, dsub, valid, st);
    case 2: return launch_restricted<2, TG, SEL>(cost, cps, crs, g, p, coarse, radius, dtar, dref, dsub, valid, st);
    case 3: return launch_restricted<3, TG, SEL>(cost, cps, crs, g, p, coarse, radius, dtar, dref, dsub, valid, st);
    case 4: return launch_restricted<4, TG, SEL>(cost, cps, crs, g, p, coarse, radius, dtar, dref, dsub, valid, st);
    case 5: return launch_restricted<5, TG, SEL>(cost, cps, crs, g, p, coarse, radius, dtar, dref, dsub, valid, st);
    default: return RSV_E_PARAM;
  }
}

// SEL: the reference form (winner, Eq. 12, Eq. 11 against dtar); else the target
// argmax written to dref.
int run_restricted(bool sel, const float* cost, int64_t cps, int64_t crs, const rsv_image& guide,
                   const rsv_params* p, const int32_t* coarse, int radius, const int32_t* dtar, int32_t* dref,
                   float* dsub, uint8_t* valid, void* stream) {
  if (int s = validate_image(guide)) return s;
  if (int s = validate_agg_params(p)) return s;
  if (sel)
    if (int s = validate_select_params(p)) return s;
  if (!cost || !coarse || !dref || (sel && (!dtar || !dsub || !valid))) return RSV_E_NULL;
  if (!aligned(cost, 4) || !aligned(coarse, 4) || !aligned(dref, 4) || (sel && (!aligned(dtar, 4) ||
                                                                              !aligned(dsub, 4))))
    return RSV_E_ALIGN;
  if (radius < 0) return RSV_E_PARAM;
  if (p->agg_radius > 5) return RSV_E_PARAM;
  if (guide.width < 4 || crs < guide.width || cps < 1 || cps > kAggMaxPixels ||
      static_cast<int64_t>(guide.height - 1) * crs + guide.width > kAggMaxPixels)
    return RSV_E_SHAPE;
  hipStream_t st = as_stream(stream);
  const int rs = static_cast<int>(crs);
  if (guide.dtype == RSV_U8)
    return sel ? dispatch_restricted<uint8_t, true>(cost, cps, rs, guide, p, coarse, radius, dtar, dref, dsub, valid, st)
               : dispatch_restricted<uint8_t, false>(cost, cps, rs, guide, p, coarse, radius, dtar, dref, dsub, valid, st);
  return sel ? dispatch_restricted<float, true>(cost, cps, rs, guide, p, coarse, radius, dtar, dref, dsub, valid, st)
             : dispatch_restricted<float, false>(cost, cps, rs, guide, p, coarse, radius, dtar, dref, dsub, valid, st);
}

template <int A, typename TG, bool ARG>
int launch_agg(const float* cost, int64_t cps, int crs, const rsv_image& g, const rsv_params* p,
               float* agg, int32_t* disp, hipStream_t st) {
  if constexpr (agg_dma_fits<A>()) {
    if (g.width >= 4) return launch_agg_dma<A, TG, ARG>(cost, cps, crs, g, p, agg, disp, st);
  }
  constexpr int TY = kAggTileRows;
  const int tiles = ((g.width + 15) / 16) * ((g.height + TY - 1) / TY);
  const BilateralK bk = bilateral_constants(p->gamma_d, p->gamma_r);
  const bool vec4 = (g.width % 4) == 0 && aligned(agg, 16);
  const size_t lds = agg_tile_lds_bytes<A, TY>() + (ARG ? 2 * 256 * sizeof(float) : 0);
  auto kern = aggregate_kernel<A, TY, TG, ARG>;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
  if (e != hipSuccess) {
    set_hip_error(e);
    return RSV_E_HIP;
  }
  kern<<<dim3(tiles), dim3(64 * TY), lds, st>>>(cost, cps, crs, static_cast<const TG*>(g.data), g.pitch,
                                                g.height, g.width, p->D, bk, vec4, agg, disp);
  return check_launch();
}

template <typename TG, bool ARG>
int dispatch_agg(const float* cost, int64_t cps, int crs, const rsv_image& g, const rsv_params* p,
                 float* agg, int32_t* disp, hipStream_t st) {
  switch (p->agg_radius) {
    case 1: return launch_agg<1, TG, ARG>(cost, cps, crs, g, p, agg, disp, st);
    case 2: return launch_agg<2, TG, ARG>(cost, cps, crs, g, p, agg, disp, st);
    case 3: return launch_agg<3, TG, ARG>(cost, cps, crs, g, p, agg, disp, st);
    case 4: return launch_agg<4, TG, ARG>(cost, cps, crs, g, p, agg, disp, st);
    case 5: return launch_agg<5, TG, ARG>(cost, cps, crs, g, p, agg, disp, st);
    case 6: return launch_agg<6, TG, ARG>(cost, cps, crs, g, p, agg, disp, st);
    default: return RSV_E_PARAM;
  }
}

// One output: the volume agg, or (agg null) the argmax map disp.
int run_agg(const float* cost, int64_t cps, int64_t crs, const rsv_image& guide, const rsv_params* p,
            float* agg, int32_t* disp, void* stream) {
  if (int s = validate_image(guide)) return s;
  if (int s = validate_agg_params(p)) return s;
  if (!cost || (!agg && !disp)) return RSV_E_NULL;
  if (!aligned(cost, 4) || (agg && !aligned(agg, 4)) || (disp && !aligned(disp, 4))) return RSV_E_ALIGN;
  if (cost == agg || static_cast<const void*>(cost) == static_cast<const void*>(disp)) return RSV_E_PARAM;
  // element offsets inside 16 disparity planes stay below 2^31
  if (crs < guide.width || cps < 1 || cps > kAggMaxPixels ||
      static_cast<int64_t>(guide.height - 1) * crs + guide.width > kAggMaxPixels)
    return RSV_E_SHAPE;
  hipStream_t st = as_stream(stream);
  const int rs = static_cast<int>(crs);
  if (agg) {
    if (guide.dtype == RSV_U8) return dispatch_agg<uint8_t, false>(cost, cps, rs, guide, p, agg, nullptr, st);
    return dispatch_agg<float, false>(cost, cps, rs, guide, p, agg, nullptr, st);
  }
  if (guide.dtype == RSV_U8) return dispatch_agg<uint8_t, true>(cost, cps, rs, guide, p, nullptr, disp, st);
  return dispatch_agg<float, true>(cost, cps, rs, guide, p, nullptr, disp, st);
}

}  // namespace rsv

extern "C" int rsv_aggregate(const float* cost, rsv_image guide, const rsv_params* p, float* agg,
                             void* stream) {
  using namespace rsv;
  if (int s = validate_image(guide)) return s;
  if (!agg) return RSV_E_NULL;
  return run_agg(cost, static_cast<int64_t>(guide.height) * guide.width, guide.width, guide, p, agg, nullptr,
                 stream);
}

extern "C" int rsv_aggregate_strided(const float* cost, int64_t plane_stride, int64_t row_stride,
                                     rsv_image guide, const rsv_params* p, float* agg, void* stream) {
  if (!agg) return RSV_E_NULL;
  return rsv::run_agg(cost, plane_stride, row_stride, guide, p, agg, nullptr, stream);
}

extern "C" int rsv_aggregate_argmax(const float* cost, int64_t plane_stride, int64_t row_stride,
                                    rsv_image guide, const rsv_params* p, int32_t* disp, void* stream) {
  if (!disp) return RSV_E_NULL;
  return rsv::run_agg(cost, plane_stride, row_stride, guide, p, nullptr, disp, stream);
}

extern "C" int rsv_aggregate_select(const float* cost, int64_t plane_stride, int64_t row_stride, rsv_image guide,
                                    const rsv_params* p, const int32_t* disp_tar, int32_t* disp_ref,
                                    float* disp_sub, uint8_t* valid, void* stream) {
  using namespace rsv;
  if (int s = validate_image(guide)) return s;
  if (int s = validate_agg_params(p)) return s;
  if (int s = validate_select_params(p)) return s;
  if (!cost || !disp_tar || !disp_ref || !disp_sub || !valid) return RSV_E_NULL;
  if (!aligned(cost, 4) || !aligned(disp_tar, 4) || !aligned(disp_ref, 4) || !aligned(disp_sub, 4))
    return RSV_E_ALIGN;
  if (p->agg_radius > 5) return RSV_E_PARAM;
  if (guide.width < 4 || row_stride < guide.width || plane_stride < 1 || plane_stride > kAggMaxPixels ||
      static_cast<int64_t>(guide.height - 1) * row_stride + guide.width > kAggMaxPixels)
    return RSV_E_SHAPE;
  hipStream_t st = as_stream(stream);
  const int rs = static_cast<int>(row_stride);
  if (guide.dtype == RSV_U8)
    return dispatch_agg_select<uint8_t>(cost, plane_stride, rs, guide, p, disp_tar, disp_ref, disp_sub, valid, st);
  return dispatch_agg_select<float>(cost, plane_stride, rs, guide, p, disp_tar, disp_ref, disp_sub, valid, st);
}

extern "C" int rsv_aggregate_views(const float* cost_ref, int64_t ref_plane_stride, int64_t ref_row_stride,
                                   const float* cost_tar, int64_t tar_plane_stride, int64_t tar_row_stride,
                                   rsv_image guide_ref, rsv_image guide_tar, const rsv_params* p,
                                   int32_t* disp_tar, int32_t* disp_ref, float* disp_sub, void* stream) {
  using namespace rsv;
  if (int s = validate_views(cost_ref, ref_plane_stride, ref_row_stride, cost_tar, tar_plane_stride, tar_row_stride,
                             guide_ref, guide_tar, p, disp_tar, disp_ref, disp_sub))
    return s;
  hipStream_t st = as_stream(stream);
  const int rrs = static_cast<int>(ref_row_stride), trs = static_cast<int>(tar_row_stride);
  if (guide_ref.dtype == RSV_U8)
    return dispatch_agg_views<uint8_t>(cost_ref, ref_plane_stride, rrs, cost_tar, tar_plane_stride, trs, guide_ref,
                                       guide_tar, p, disp_tar, disp_ref, disp_sub, st);
  return dispatch_agg_views<float>(cost_ref, ref_plane_stride, rrs, cost_tar, tar_plane_stride, trs, guide_ref,
                                   guide_tar, p, disp_tar, disp_ref, disp_sub, st);
}

extern "C" int rsv_aggregate_restricted_views(const float* cost_ref, int64_t ref_plane_stride,
                                              int64_t ref_row_stride, const float* cost_tar,
                                              int64_t tar_plane_stride, int64_t tar_row_stride, rsv_image guide_ref,
                                              rsv_image guide_tar, const rsv_params* p, const int32_t* coarse_ref,
                                              const int32_t* coarse_tar, int32_t radius, int32_t* disp_tar,
                                              int32_t* disp_ref, float* disp_sub, void* stream) {
  using namespace rsv;
  if (int s = validate_views(cost_ref, ref_plane_stride, ref_row_stride, cost_tar, tar_plane_stride, tar_row_stride,
                             guide_ref, guide_tar, p, disp_tar, disp_ref, disp_sub))
    return s;
  if (!coarse_ref || !coarse_tar) return RSV_E_NULL;
  if (!aligned(coarse_ref, 4) || !aligned(coarse_tar, 4)) return RSV_E_ALIGN;
  if (radius < 0) return RSV_E_PARAM;
  hipStream_t st = as_stream(stream);
  const int rrs = static_cast<int>(ref_row_stride), trs = static_cast<int>(tar_row_stride);
  if (guide_ref.dtype == RSV_U8)
    return dispatch_restricted_views<uint8_t>(cost_ref, ref_plane_stride, rrs, cost_tar, tar_plane_stride, trs,
                                              guide_ref, guide_tar, p, coarse_ref, coarse_tar, radius, disp_tar,
                                              disp_ref, disp_sub, st);
  return dispatch_restricted_views<float>(cost_ref, ref_plane_stride, rrs, cost_tar, tar_plane_stride, trs, guide_ref,
                                          guide_tar, p, coarse_ref, coarse_tar, radius, disp_tar, disp_ref, disp_sub,
                                          st);
}

extern "C" int rsv_aggregate_restricted_argmax(const float* cost, int64_t plane_stride, int64_t row_stride,
                                               rsv_image guide, const rsv_params* p, const int32_t* coarse,
                                               int32_t radius, int32_t* disp, void* stream) {
  return rsv::run_restricted(false, cost, plane_stride, row_stride, guide, p, coarse, radius, nullptr, disp,
                             nullptr, nullptr, stream);
}

extern "C" int rsv_aggregate_restricted_select(const float* cost, int64_t plane_stride, int64_t row_stride,
                                               rsv_image guide, const rsv_params* p, const int32_t* coarse,
                                               int32_t radius, const int32_t* disp_tar, int32_t* disp_ref,
                                               float* disp_sub, uint8_t* valid, void* stream) {
  return rsv::run_restricted(true, cost, plane_stride, row_stride, guide, p, coarse, radius, disp_tar, disp_ref,
                             disp_sub, valid, stream);
}
