// rsv_select_subpixel, rsv_select_subpixel_ref: winner-take-all on the aggregated
// volumes (Sec. II-B.3), the left-right consistency check (Sec. II-B.4, Eq. 11) and
// the parabola subpixel refinement (Eq. 12).
//
// Two launches: a scan kernel in which each thread walks d for one pixel in both
// aggregated volumes at once, or in the reference volume only when the target
// disparities are given (coalesced loads across the row, 256-pixel row segments per
// block), keeping the target argmax and, for the reference volume, the best, second
// best and the neighbours of the running best (ties go to the lowest d); then the
// left-right check on the two disparity maps, which reads the target disparity at
// u - d of any segment once every scan has finished.
#include <math.h>

#include "select_math.hpp"

namespace rsv {

constexpr int kSelThreads = 256;
constexpr int kSelUnroll = 16;

// Walk d = 0 .. D-1 of one pixel in both volumes (stride `plane`; pt null: the
// reference volume only): loads run ahead of the compare chains in chunks of
// kSelUnroll, then of 4, then singly.  Every value is read once, so the loads are
// non-temporal.
template <bool TAR, bool TOP2>
__device__ __forceinline__ void scan_pair(const float* __restrict__ pr, const float* __restrict__ pt,
                                          int64_t plane, int D, Scan& s, int& targ) {
  bool need_next = false;
  float prev = 0.f, tbest = 0.f;
  targ = 0;
  auto consume = [&](float a, float b, int d) {
    if (d == 0) {
      scan_init(s, need_next, prev, a);
      tbest = wta_key(b);
      targ = 0;
    } else {
      scan_step<TOP2>(s, need_next, prev, a, d);
      if (TAR && wta_key(b) > tbest) {
        tbest = wta_key(b);
        targ = d;
      }
    }
  };
  auto load_t = [&](int d) { return TAR ? __builtin_nontemporal_load(pt + d * plane) : 0.f; };
  int d = 0;
  for (; d + kSelUnroll <= D; d += kSelUnroll) {
    float a[kSelUnroll], b[kSelUnroll];
#pragma unroll
    for (int i = 0; i < kSelUnroll; ++i) {
      a[i] = __builtin_nontemporal_load(pr + (d + i) * plane);
      b[i] = load_t(d + i);
    }
#pragma unroll
    for (int i = 0; i < kSelUnroll; ++i) consume(a[i], b[i], d + i);
  }
  for (; d + 4 <= D; d += 4) {
    float a[4], b[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      a[i] = __builtin_nontemporal_load(pr + (d + i) * plane);
      b[i] = load_t(d + i);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) consume(a[i], b[i], d + i);
  }
  for (; d < D; ++d) consume(__builtin_nontemporal_load(pr + d * plane), load_t(d), d);
}

// TAR: scan the target volume too and write dtar; otherwise dtar is an input.  TOP2:
// write the best and second-best values to top2.
template <bool TAR, bool TOP2>
__global__ __launch_bounds__(kSelThreads) void select_scan_kernel(
    const float* __restrict__ aref, const float* __restrict__ atar, int H, int W, int D,
    int32_t* __restrict__ dref, int32_t* __restrict__ dtar, float* __restrict__ dsub,
    float* __restrict__ top2) {
  const int u = blockIdx.x * kSelThreads + threadIdx.x;
  const int v = blockIdx.y;
  if (u >= W) return;
  const int64_t plane = static_cast<int64_t>(H) * W;
  const int64_t i = static_cast<int64_t>(v) * W + u;
  Scan s;
  int ta;
  scan_pair<TAR, TOP2>(aref + i, TAR ? atar + i : nullptr, plane, D, s, ta);
  dref[i] = s.arg;
  if (TAR) dtar[i] = ta;
  dsub[i] = parabola(s.arg, s.best, s.am, s.ap, D);
  if (TOP2) {
    top2[i] = s.best;
    top2[plane + i] = s.second;
  }
}

// Eq. 11 with tolerance tau: the target disparity at the matched column u - d.
__global__ __launch_bounds__(kSelThreads) void lr_check_kernel(const int32_t* __restrict__ dref,
                                                              const int32_t* __restrict__ dtar, int W,
                                                              int tau, uint8_t* __restrict__ valid) {
  const int u = blockIdx.x * kSelThreads + threadIdx.x;
  if (u >= W) return;
  const int64_t row = static_cast<int64_t>(blockIdx.y) * W;
  const int a = dref[row + u];
  const int x = u - a;
  valid[row + u] = (x >= 0 && abs(a - dtar[row + (x < 0 ? 0 : x)]) <= tau) ? 1 : 0;
}

// Winner-take-all of an unaggregated cost view, the disparities the restricted
// search of Sec. IV centres its windows on: first maximum over d (wta_key order) of
// cost[d * cps + v * crs + u], one thread per pixel, loads in chunks of kSelUnroll
// ahead of the compare chain (coalesced across the row).
__global__ __launch_bounds__(kSelThreads) void cost_argmax_kernel(const float* __restrict__ cost, int64_t cps,
                                                                 int64_t crs, int W, int D,
                                                                 int32_t* __restrict__ disp) {
  const int u = blockIdx.x * kSelThreads + threadIdx.x;
  if (u >= W) return;
  const int v = blockIdx.y;
  const float* c = cost + static_cast<int64_t>(v) * crs + u;
  float b = wta_key(c[0]);
  int a = 0;
  int d = 1;
  for (; d + kSelUnroll <= D; d += kSelUnroll) {
    float x[kSelUnroll];
#pragma unroll
    for (int i = 0; i < kSelUnroll; ++i) x[i] = wta_key(c[(d + i) * cps]);
#pragma unroll
    for (int i = 0; i < kSelUnroll; ++i)
      if (x[i] > b) {
        b = x[i];
        a = d + i;
      }
  }
  for (; d < D; ++d) {
    const float x = wta_key(c[d * cps]);
    if (x > b) {
      b = x;
      a = d;
    }
  }
  disp[static_cast<int64_t>(v) * W + u] = a;
}

// The same for two views in one pass (e.g. both views of one joint volume): per
// thread the scans of pixel u in both, their loads interleaved, so that where the
// views share a volume its lines are fetched once for both.
__global__ __launch_bounds__(kSelThreads) void cost_argmax2_kernel(const float* __restrict__ c0, int64_t cps0,
                                                                  int64_t crs0, const float* __restrict__ c1,
                                                                  int64_t cps1, int64_t crs1, int W, int D,
                                                                  int32_t* __restrict__ d0,
                                                                  int32_t* __restrict__ d1) {
  const int u = blockIdx.x * kSelThreads + threadIdx.x;
  if (u >= W) return;
  const int v = blockIdx.y;
  const float* p0 = c0 + static_cast<int64_t>(v) * crs0 + u;
  const float* p1 = c1 + static_cast<int64_t>(v) * crs1 + u;
  float b0 = wta_key(p0[0]), b1 = wta_key(p1[0]);
  int a0 = 0, a1 = 0;
  int d = 1;
  for (; d + kSelUnroll <= D; d += kSelUnroll) {
    float x0[kSelUnroll], x1[kSelUnroll];
#pragma unroll
    for (int i = 0; i < kSelUnroll; ++i) {
      x0[i] = wta_key(p0[(d + i) * cps0]);
      x1[i] = wta_key(p1[(d + i) * cps1]);
    }
#pragma unroll
    for (int i = 0; i < kSelUnroll; ++i) {
      if (x0[i] > b0) {
        b0 = x0[i];
        a0 = d + i;
      }
      if (x1[i] > b1) {
        b1 = x1[i];
        a1 = d + i;
      }
    }
  }
  for (; d < D; ++d) {
    const float y0 = wta_key(p0[d * cps0]), y1 = wta_key(p1[d * cps1]);
    if (y0 > b0) {
      b0 = y0;
      a0 = d;
    }
    if (y1 > b1) {
      b1 = y1;
      a1 = d;
    }
  }
  const int64_t i = static_cast<int64_t>(v) * W + u;
  d0[i] = a0;
  d1[i] = a1;
}

}  // namespace rsv

namespace rsv {

// With agg_tar: both scans; without: disp_tar is the target argmax map, given.
int run_select(const float* agg_ref, const float* agg_tar, int32_t height, int32_t width, const rsv_params* p,
               int32_t* disp_ref, int32_t* disp_tar, float* disp_sub, uint8_t* valid, float* top2,
               void* stream) {
  if (int s = validate_select_params(p)) return s;
  if (!agg_ref || !disp_ref || !disp_tar || !disp_sub || !valid) return RSV_E_NULL;
  if (height < 1 || width < 1) return RSV_E_SHAPE;
  if (static_cast<int64_t>(height) * width > INT32_MAX) return RSV_E_SHAPE;
  if (!aligned(agg_ref, 4) || !aligned(agg_tar, 4) || !aligned(disp_ref, 4) ||
      !aligned(disp_tar, 4) || !aligned(disp_sub, 4) || (top2 && !aligned(top2, 4)))
    return RSV_E_ALIGN;
  const dim3 grid((width + kSelThreads - 1) / kSelThreads, height);
  auto kern = agg_tar ? (top2 ? select_scan_kernel<true, true> : select_scan_kernel<true, false>)
                      : (top2 ? select_scan_kernel<false, true> : select_scan_kernel<false, false>);
  kern<<<grid, dim3(kSelThreads), 0, as_stream(stream)>>>(agg_ref, agg_tar, height, width, p->D, disp_ref,
                                                          disp_tar, disp_sub, top2);
  if (int st = check_launch()) return st;
  lr_check_kernel<<<grid, dim3(kSelThreads), 0, as_stream(stream)>>>(disp_ref, disp_tar, width,
                                                                    p->lr_threshold, valid);
  return check_launch();
}

}  // namespace rsv

extern "C" int rsv_lr_check(const int32_t* disp_ref, const int32_t* disp_tar, int32_t height, int32_t width,
                            int32_t tau, uint8_t* valid, void* stream) {
  using namespace rsv;
  if (!disp_ref || !disp_tar || !valid) return RSV_E_NULL;
  if (!aligned(disp_ref, 4) || !aligned(disp_tar, 4)) return RSV_E_ALIGN;
  if (height < 1 || width < 1) return RSV_E_SHAPE;
  if (tau < 0) return RSV_E_PARAM;
  const dim3 grid((width + kSelThreads - 1) / kSelThreads, height);
  lr_check_kernel<<<grid, dim3(kSelThreads), 0, as_stream(stream)>>>(disp_ref, disp_tar, width, tau, valid);
  return check_launch();
}

extern "C" int rsv_select_subpixel(const float* agg_ref, const float* agg_tar, int32_t height,
                                   int32_t width, const rsv_params* p, int32_t* disp_ref,
                                   int32_t* disp_tar, float* disp_sub, uint8_t* valid, float* top2,
                                   void* stream) {
  if (int s = rsv::validate_select_params(p)) return s;
  if (!agg_tar) return RSV_E_NULL;
  return rsv::run_select(agg_ref, agg_tar, height, width, p, disp_ref, disp_tar, disp_sub, valid, top2, stream);
}

extern "C" int rsv_select_subpixel_ref(const float* agg_ref, const int32_t* disp_tar, int32_t height,
                                       int32_t width, const rsv_params* p, int32_t* disp_ref, float* disp_sub,
                                       uint8_t* valid, float* top2, void* stream) {
  return rsv::run_select(agg_ref, nullptr, height, width, p, disp_ref, const_cast<int32_t*>(disp_tar),
                         disp_sub, valid, top2, stream);
}

extern "C" int rsv_cost_argmax(const float* cost, int64_t plane_stride, int64_t row_stride, int32_t height,
                               int32_t width, int32_t D, int32_t* disp, void* stream) {
  using namespace rsv;
  if (!cost || !disp) return RSV_E_NULL;
  if (height < 1 || width < 1 || D < 1 || D > RSV_MAX_D || row_stride < width || plane_stride < 1)
    return RSV_E_SHAPE;
  if (!aligned(cost, 4) || !aligned(disp, 4)) return RSV_E_ALIGN;
  const dim3 grid((width + kSelThreads - 1) / kSelThreads, height);
  cost_argmax_kernel<<<grid, dim3(kSelThreads), 0, as_stream(stream)>>>(cost, plane_stride, row_stride, width, D,
                                                                        disp);
  return check_launch();
}

extern "C" int rsv_cost_argmax_views(const float* cost_ref, int64_t ref_plane_stride, int64_t ref_row_stride,
                                     const float* cost_tar, int64_t tar_plane_stride, int64_t tar_row_stride,
                                     int32_t height, int32_t width, int32_t D, int32_t* disp_ref, int32_t* disp_tar,
                                     void* stream) {
  using namespace rsv;
  if (!cost_ref || !cost_tar || !disp_ref || !disp_tar) return RSV_E_NULL;
  if (height < 1 || width < 1 || D < 1 || D > RSV_MAX_D || ref_row_stride < width || tar_row_stride < width ||
      ref_plane_stride < 1 || tar_plane_stride < 1)
    return RSV_E_SHAPE;
  if (!aligned(cost_ref, 4) || !aligned(cost_tar, 4) || !aligned(disp_ref, 4) || !aligned(disp_tar, 4))
    return RSV_E_ALIGN;
  const dim3 grid((width + kSelThreads - 1) / kSelThreads, height);
  cost_argmax2_kernel<<<grid, dim3(kSelThreads), 0, as_stream(stream)>>>(cost_ref, ref_plane_stride, ref_row_stride,
                                                                         cost_tar, tar_plane_stride, tar_row_stride,
                                                                         width, D, disp_ref, disp_tar);
  return check_launch();
}
