// rsv_select_subpixel: winner-take-all on both aggregated volumes (Sec. II-B.3),
// the left-right consistency check (Sec. II-B.4, Eq. 11) and the parabola subpixel
// refinement (Eq. 12).
//
// One block per image row.  Pass 1 scans the target volume for every pixel of the
// row (threads stride over u, each walking d with coalesced loads) and keeps the
// target disparities of the row in LDS.  Pass 2 scans the reference volume,
// keeping best / second-best and the neighbours of the running best, then checks
// the match against the target row in LDS and refines.  Ties go to the lowest d:
// a later d replaces the best only when strictly greater.
#include <math.h>

#include "select_math.hpp"

namespace rsv {

constexpr int kSelThreads = 256;
constexpr int kSelMaxW = 16384;

struct Scan {
  float best, second, am, ap;
  int arg;
};

// Walk d = 0 .. D-1 of column `p` (stride `plane`).  Loads run ahead of the
// compare chain in groups of 8.
__device__ __forceinline__ Scan scan_column(const float* __restrict__ p, int64_t plane, int D) {
  Scan s;
  s.best = p[0];
  s.second = -INFINITY;
  s.am = 0.f;
  s.ap = 0.f;
  s.arg = 0;
  bool need_next = true;  // the value after the current best is its right neighbour
  float prev = s.best;
  int d = 1;
  for (; d + 8 <= D; d += 8) {
    float a[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) a[i] = p[(d + i) * plane];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      if (need_next) {
        s.ap = a[i];
        need_next = false;
      }
      if (a[i] > s.best) {
        s.second = s.best;
        s.best = a[i];
        s.arg = d + i;
        s.am = prev;
        need_next = true;
      } else if (a[i] > s.second) {
        s.second = a[i];
      }
      prev = a[i];
    }
  }
  for (; d < D; ++d) {
    const float a = p[d * plane];
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
  return s;
}

__device__ __forceinline__ int argmax_column(const float* __restrict__ p, int64_t plane, int D) {
  float best = p[0];
  int arg = 0;
  int d = 1;
  for (; d + 8 <= D; d += 8) {
    float a[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) a[i] = p[(d + i) * plane];
#pragma unroll
    for (int i = 0; i < 8; ++i)
      if (a[i] > best) {
        best = a[i];
        arg = d + i;
      }
  }
  for (; d < D; ++d) {
    const float a = p[d * plane];
    if (a > best) {
      best = a;
      arg = d;
    }
  }
  return arg;
}

__global__ __launch_bounds__(kSelThreads) void select_kernel(
    const float* __restrict__ aref, const float* __restrict__ atar, int H, int W, int D, int tau,
    int32_t* __restrict__ dref, int32_t* __restrict__ dtar, float* __restrict__ dsub,
    uint8_t* __restrict__ valid, float* __restrict__ top2) {
  extern __shared__ int32_t ltar[];
  const int v = blockIdx.x;
  const int64_t plane = static_cast<int64_t>(H) * W;
  const int64_t row = static_cast<int64_t>(v) * W;
  for (int u = threadIdx.x; u < W; u += kSelThreads) {
    const int a = argmax_column(atar + row + u, plane, D);
    ltar[u] = a;
    dtar[row + u] = a;
  }
  __syncthreads();
  for (int u = threadIdx.x; u < W; u += kSelThreads) {
    const Scan s = scan_column(aref + row + u, plane, D);
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
