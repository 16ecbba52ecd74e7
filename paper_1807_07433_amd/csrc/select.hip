// rsv_select_subpixel: winner-take-all on both aggregated volumes (Sec. II-B.3),
// the left-right consistency check (Sec. II-B.4, Eq. 11) and the parabola subpixel
// refinement (Eq. 12).
//
// Each thread walks d for one pixel in both aggregated volumes at once (coalesced
// loads across the row), keeping the target argmax and, for the reference volume,
// the best, second best and the neighbours of the running best.  Ties go to the
// lowest d: a later d replaces the best only when strictly greater.
#include <math.h>

#include "select_math.hpp"

namespace rsv {

constexpr int kSelThreads = 1024;
constexpr int kSelMaxW = 16384;
constexpr int kSelUnroll = 8;

struct Scan {
  float best, second, am, ap;
  int arg;
};

// One step of the reference scan at disparity d with value a (strictly greater
// replaces the best, so ties keep the lowest d).
__device__ __forceinline__ void scan_step(Scan& s, bool& need_next, float& prev, float a, int d) {
  if (need_next) {
    s.ap = a;
    need_next = false;
  }
  if (a > s.best) {
    s.second = s.best;
    s.best = a;
    s.arg = d;
    s.am = prev;
    need_next = true;
  } else if (a > s.second) {
    s.second = a;
  }
  prev = a;
}

// Walk d = 0 .. D-1 of one pixel in both volumes (stride `plane`), loads for both
// running ahead of the compare chains in groups of kSelUnroll.
__device__ __forceinline__ void scan_pair(const float* __restrict__ pr, const float* __restrict__ pt,
                                          int64_t plane, int D, Scan& s, int& targ) {
  s.best = pr[0];
  s.second = -INFINITY;
  s.am = 0.f;
  s.ap = 0.f;
  s.arg = 0;
  bool need_next = true;  // the value after the current best is its right neighbour
  float prev = s.best;
  float tbest = pt[0];
  targ = 0;
  int d = 1;
  for (; d + kSelUnroll <= D; d += kSelUnroll) {
    float a[kSelUnroll], b[kSelUnroll];
#pragma unroll
    for (int i = 0; i < kSelUnroll; ++i) {
      a[i] = pr[(d + i) * plane];
      b[i] = pt[(d + i) * plane];
    }
#pragma unroll
    for (int i = 0; i < kSelUnroll; ++i) {
      scan_step(s, need_next, prev, a[i], d + i);
      if (b[i] > tbest) {
        tbest = b[i];
        targ = d + i;
      }
    }
  }
  for (; d < D; ++d) {
    scan_step(s, need_next, prev, pr[d * plane], d);
    const float b = pt[d * plane];
    if (b > tbest) {
      tbest = b;
      targ = d;
    }
  }
}

// One block per image row, walking the row in chunks of kSelThreads columns from
// left to right.  The left-right lookup at u - d only reaches columns of the
// current or an earlier chunk, whose target disparities are already in LDS.
__global__ __launch_bounds__(kSelThreads) void select_kernel(
    const float* __restrict__ aref, const float* __restrict__ atar, int H, int W, int D, int tau,
    int32_t* __restrict__ dref, int32_t* __restrict__ dtar, float* __restrict__ dsub,
    uint8_t* __restrict__ valid, float* __restrict__ top2) {
  extern __shared__ int32_t ltar[];
  const int v = blockIdx.x;
  const int64_t plane = static_cast<int64_t>(H) * W;
  const int64_t row = static_cast<int64_t>(v) * W;
  for (int c0 = 0; c0 < W; c0 += kSelThreads) {
    const int u = c0 + threadIdx.x;
    Scan s{};
    int ta = 0;
    if (u < W) {
      scan_pair(aref + row + u, atar + row + u, plane, D, s, ta);
      ltar[u] = ta;
      dtar[row + u] = ta;
    }
    __syncthreads();
    if (u < W) {
      const int x = u - s.arg;
      const bool ok = (x >= 0) && (abs(s.arg - ltar[x < 0 ? 0 : x]) <= tau);
      dref[row + u] = s.arg;
      dsub[row + u] = parabola(s.arg, s.best, s.am, s.ap, D);
      valid[row + u] = ok ? 1 : 0;
      if (top2) {
        top2[row + u] = s.best;
        top2[plane + row + u] = s.second;
      }
    }
  }
}

}  // namespace rsv

extern "C" int rsv_select_subpixel(const float* agg_ref, const float* agg_tar, int32_t height,
                                   int32_t width, const rsv_params* p, int32_t* disp_ref,
                                   int32_t* disp_tar, float* disp_sub, uint8_t* valid, float* top2,
                                   void* stream) {
  using namespace rsv;
  if (int s = validate_select_params(p)) return s;
  if (!agg_ref || !agg_tar || !disp_ref || !disp_tar || !disp_sub || !valid) return RSV_E_NULL;
  if (height < 1 || width < 1 || width > kSelMaxW) return RSV_E_SHAPE;
  if (!aligned(agg_ref, 4) || !aligned(agg_tar, 4) || !aligned(disp_ref, 4) ||
      !aligned(disp_tar, 4) || !aligned(disp_sub, 4) || (top2 && !aligned(top2, 4)))
    return RSV_E_ALIGN;
  const size_t lds = sizeof(int32_t) * static_cast<size_t>(width);
  select_kernel<<<dim3(height), dim3(kSelThreads), lds, as_stream(stream)>>>(
      agg_ref, agg_tar, height, width, p->D, p->lr_threshold, disp_ref, disp_tar, disp_sub, valid,
      top2);
  return check_launch();
}
