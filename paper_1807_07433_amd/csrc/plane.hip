// rsv_plane_ransac: the road-plane estimation of Sec. II-A.  The plane of
// disparities d = a0 + a1 v + a2 u (Eq. 2 with the u-term of the roll-fitted plane)
// is fitted to the valid pixels of a disparity map by least squares inside RANSAC:
//   1. hypotheses: one thread per draw of 3 pixels (the draws are an input), the
//      plane through them by Cramer's rule in FP64 (-1 count: the pixels are
//      collinear in (u, v), an exact integer test, or a draw is out of range);
//   2. scoring: every valid pixel against every hypothesis, |d - (a0 + a1 v + a2 u)|
//      <= threshold in FP64, one lane per pixel, the hypotheses as scalar operands,
//      one global add per hypothesis and block;
//   3. the best hypothesis (most inliers, ties to the lowest index; a block-wide
//      reduction in every block of the next launch), then the FP64
//      normal-equation sums of its inliers in coordinates centred on the image
//      (well conditioned), block partial sums and one atomic per sum and block;
//   4. one thread solves the 3 x 3 system and moves the plane back to image
//      coordinates.
#include <algorithm>
#include <climits>

#include "rsv_internal.hpp"

namespace rsv {

constexpr int kPlaneThreads = 256;
constexpr int kPlaneMaxK = RSV_PLANE_MAX_K;
constexpr int kPlaneSums = 9;  // n, Su, Sv, Suu, Suv, Svv, Sd, Sud, Svd

// d - (a0 + a1 v + a2 u), with the same roundings wherever an inlier is decided.
__device__ __forceinline__ double plane_residual(double a0, double a1, double a2, double d, double v, double u) {
  return d - fma(a2, u, fma(a1, v, a0));
}

struct PlaneWs {
  double* planes;  // [K][3]: a0, a1, a2
  double* sums;    // [kPlaneSums]
};

inline PlaneWs plane_ws(void* ws, int K) {
  double* p = static_cast<double*>(ws);
  return PlaneWs{p, p + 3 * K};
}

__global__ __launch_bounds__(kPlaneThreads) void plane_hypothesis_kernel(const float* __restrict__ disp, int H, int W,
                                                                         const int32_t* __restrict__ samples, int K,
                                                                         double* __restrict__ planes,
                                                                         int32_t* __restrict__ counts,
                                                                         double* __restrict__ sums) {
  const int k = blockIdx.x * kPlaneThreads + threadIdx.x;
  if (k < kPlaneSums && blockIdx.x == 0) sums[k] = 0.0;
  if (k >= K) return;
  const int64_t n = static_cast<int64_t>(H) * W;
  int64_t s[3];
  bool ok = true;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    s[i] = samples[3 * k + i];
    ok = ok && s[i] >= 0 && s[i] < n;
  }
  int64_t u[3] = {0, 0, 0}, v[3] = {0, 0, 0};
  double d[3] = {0.0, 0.0, 0.0};
  if (ok) {
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      v[i] = s[i] / W;
      u[i] = s[i] - v[i] * W;
      d[i] = disp[s[i]];
    }
  }
  // twice the signed area of the (u, v) triangle: the determinant of [1 v u] rows
  const int64_t det = (v[1] - v[0]) * (u[2] - u[0]) - (v[2] - v[0]) * (u[1] - u[0]);
  if (!ok || det == 0) {
    counts[k] = -1;
    planes[3 * k] = planes[3 * k + 1] = planes[3 * k + 2] = __builtin_nan("");
    return;
  }
  const double dd1 = d[1] - d[0], dd2 = d[2] - d[0];
  const double det_d = static_cast<double>(det);
  const double a1 = (dd1 * static_cast<double>(u[2] - u[0]) - dd2 * static_cast<double>(u[1] - u[0])) / det_d;
  const double a2 = (static_cast<double>(v[1] - v[0]) * dd2 - static_cast<double>(v[2] - v[0]) * dd1) / det_d;
  planes[3 * k] = d[0] - a1 * static_cast<double>(v[0]) - a2 * static_cast<double>(u[0]);
  planes[3 * k + 1] = a1;
  planes[3 * k + 2] = a2;
  counts[k] = 0;
}

// One lane per pixel, kPlaneRun pixels per lane held as doubles in registers (NaN
// disparity where invalid or past the end, so they never count); the hypotheses of
// blockIdx.y's chunk are wave-uniform values the FP64 instructions read as scalar
// operands.  Per 64 pixels and hypothesis: two FMAs, a subtraction and a compare whose
// wave mask is popcounted into a scalar count.  The block's 4 waves (4 * 64 *
// kPlaneRun consecutive pixels) merge their counts in LDS: one global add per
// hypothesis and block.
constexpr int kPlaneRun = 16;
constexpr int kPlaneChunk = 32;
constexpr int kPlaneBlockPix = kPlaneThreads * kPlaneRun;

__global__ __launch_bounds__(kPlaneThreads) void plane_score_kernel(const float* __restrict__ disp,
                                                                    const uint8_t* __restrict__ valid, int64_t n,
                                                                    int W, const double* __restrict__ planes,
                                                                    int K, double thr,
                                                                    int32_t* __restrict__ counts) {
  __shared__ int sc[kPlaneChunk];
  if (threadIdx.x < kPlaneChunk) sc[threadIdx.x] = 0;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // 32-bit index arithmetic: n < 2^31, so every index below fits an unsigned
  const uint32_t base = static_cast<uint32_t>(blockIdx.x) * kPlaneBlockPix + wave * 64 * kPlaneRun + lane;
  double d[kPlaneRun], v[kPlaneRun], u[kPlaneRun];
#pragma unroll
  for (int j = 0; j < kPlaneRun; ++j) {
    const uint32_t i = base + j * 64;
    d[j] = __builtin_nan("");
    v[j] = u[j] = 0.0;
    if (i < n && valid[i]) {
      const uint32_t vi = i / static_cast<uint32_t>(W);
      d[j] = disp[i];
      v[j] = static_cast<double>(vi);
      u[j] = static_cast<double>(i - vi * W);
    }
  }
  __syncthreads();
  const int k0 = blockIdx.y * kPlaneChunk;
  const int k1 = min(K, k0 + kPlaneChunk);
  // the next hypothesis's plane is loaded while this one is scored
  double n0 = planes[3 * k0], n1 = planes[3 * k0 + 1], n2 = planes[3 * k0 + 2];
  for (int k = k0; k < k1; ++k) {
    const double a0 = n0, a1 = n1, a2 = n2;
    const int kn = min(k + 1, k1 - 1);
    n0 = planes[3 * kn];
    n1 = planes[3 * kn + 1];
    n2 = planes[3 * kn + 2];
    int cnt = 0;
#pragma unroll
    for (int j = 0; j < kPlaneRun; ++j)
      cnt += __popcll(__ballot(fabs(plane_residual(a0, a1, a2, d[j], v[j], u[j])) <= thr));
    if (lane == 0 && cnt) atomicAdd(&sc[k - k0], cnt);
  }
  __syncthreads();
  if (threadIdx.x < k1 - k0 && sc[threadIdx.x]) atomicAdd(&counts[k0 + threadIdx.x], sc[threadIdx.x]);
}

// The best hypothesis (most inliers, the lowest index among equals) by a block-wide
// reduction over the counts; every thread returns it.
__device__ int block_best_hypothesis(const int32_t* __restrict__ counts, int K) {
  __shared__ int bk[kPlaneThreads], bc[kPlaneThreads];
  int k_best = 0, c_best = INT_MIN;
  for (int k = threadIdx.x; k < K; k += kPlaneThreads) {
    const int c = counts[k];
    if (c > c_best) {  // k rises: equal counts keep the lower index
      c_best = c;
      k_best = k;
    }
  }
  bk[threadIdx.x] = k_best;
  bc[threadIdx.x] = c_best;
  __syncthreads();
  for (int s = kPlaneThreads / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      const int c = bc[threadIdx.x + s], k = bk[threadIdx.x + s];
      if (c > bc[threadIdx.x] || (c == bc[threadIdx.x] && k < bk[threadIdx.x])) {
        bc[threadIdx.x] = c;
        bk[threadIdx.x] = k;
      }
    }
    __syncthreads();
  }
  const int r = bk[0];
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(kPlaneThreads) void plane_sums_kernel(const float* __restrict__ disp,
                                                                   const uint8_t* __restrict__ valid, int H, int W,
                                                                   const double* __restrict__ planes,
                                                                   const int32_t* __restrict__ counts, int K,
                                                                   double thr, double* __restrict__ sums,
                                                                   int32_t* __restrict__ best_out) {
  __shared__ double red[kPlaneSums][kPlaneThreads];
  const int s_best = block_best_hypothesis(counts, K);
  if (blockIdx.x == 0 && threadIdx.x == 0) *best_out = s_best;
  if (counts[s_best] < 0) return;  // every hypothesis degenerate: the sums stay 0, the plane NaN
  const double a0 = planes[3 * s_best], a1 = planes[3 * s_best + 1], a2 = planes[3 * s_best + 2];
  const double cu = 0.5 * (W - 1), cv = 0.5 * (H - 1);
  double acc[kPlaneSums] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  const int64_t n = static_cast<int64_t>(H) * W;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kPlaneThreads + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * kPlaneThreads) {
    if (!valid[i]) continue;
    const uint32_t vi = static_cast<uint32_t>(i) / static_cast<uint32_t>(W);
    const double v = static_cast<double>(vi), u = static_cast<double>(i - vi * W);
    const double d = disp[i];
    if (!(fabs(plane_residual(a0, a1, a2, d, v, u)) <= thr)) continue;
    const double x = u - cu, y = v - cv;
    acc[0] += 1.0;
    acc[1] += x;
    acc[2] += y;
    acc[3] += x * x;
    acc[4] += x * y;
    acc[5] += y * y;
    acc[6] += d;
    acc[7] += x * d;
    acc[8] += y * d;
  }
#pragma unroll
  for (int j = 0; j < kPlaneSums; ++j) red[j][threadIdx.x] = acc[j];
  __syncthreads();
  for (int s = kPlaneThreads / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s)
#pragma unroll
      for (int j = 0; j < kPlaneSums; ++j) red[j][threadIdx.x] += red[j][threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x < kPlaneSums) atomicAdd(&sums[threadIdx.x], red[threadIdx.x][0]);
}

// Solves [n Sy Sx; Sy Syy Sxy; Sx Sxy Sxx] (b0, b1, b2) = (Sd, Syd, Sxd) for the centred
// plane d = b0 + b1 y + b2 x (Gaussian elimination with partial pivoting), then
// a1 = b1, a2 = b2, a0 = b0 - b1 cv - b2 cu.  best[0] = the hypothesis, best[1] = its
// inliers (the refit's points).
__global__ void plane_solve_kernel(const double* __restrict__ sums, int H, int W, double* __restrict__ plane,
                                   int32_t* __restrict__ best) {
  const double* s = sums;
  double m[3][4] = {{s[0], s[2], s[1], s[6]}, {s[2], s[5], s[4], s[8]}, {s[1], s[4], s[3], s[7]}};
  for (int c = 0; c < 3; ++c) {
    int p = c;
    for (int r = c + 1; r < 3; ++r)
      if (fabs(m[r][c]) > fabs(m[p][c])) p = r;
    for (int j = 0; j < 4; ++j) {
      const double t = m[c][j];
      m[c][j] = m[p][j];
      m[p][j] = t;
    }
    for (int r = c + 1; r < 3; ++r) {
      const double f = m[r][c] / m[c][c];
      for (int j = c; j < 4; ++j) m[r][j] -= f * m[c][j];
    }
  }
  double b[3];
  for (int r = 2; r >= 0; --r) {
    double t = m[r][3];
    for (int j = r + 1; j < 3; ++j) t -= m[r][j] * b[j];
    b[r] = t / m[r][r];
  }
  const double cu = 0.5 * (W - 1), cv = 0.5 * (H - 1);
  plane[0] = b[0] - b[1] * cv - b[2] * cu;
  plane[1] = b[1];
  plane[2] = b[2];
  best[1] = static_cast<int32_t>(s[0]);  // best[0]: written by plane_sums_kernel
}

}  // namespace rsv

extern "C" size_t rsv_plane_ransac_workspace_bytes(int32_t K) {
  if (K < 1 || K > rsv::kPlaneMaxK) return 0;
  return sizeof(double) * (3 * static_cast<size_t>(K) + rsv::kPlaneSums);
}

extern "C" int rsv_plane_ransac(const float* disp, const uint8_t* valid, int32_t height, int32_t width,
                                const int32_t* samples, int32_t K, float threshold, double* plane,
                                int32_t* counts, int32_t* best, void* workspace, void* stream) {
  using namespace rsv;
  if (!disp || !valid || !samples || !plane || !counts || !best || !workspace) return RSV_E_NULL;
  if (height < 1 || width < 1 || static_cast<int64_t>(height) * width > INT32_MAX) return RSV_E_SHAPE;
  if (K < 1 || K > kPlaneMaxK) return RSV_E_SHAPE;
  if (!(threshold >= 0.f)) return RSV_E_PARAM;
  if (!aligned(disp, 4) || !aligned(samples, 4) || !aligned(plane, 8) || !aligned(counts, 4) ||
      !aligned(best, 4) || !aligned(workspace, 8))
    return RSV_E_ALIGN;
  hipStream_t st = as_stream(stream);
  const PlaneWs ws = plane_ws(workspace, K);
  plane_hypothesis_kernel<<<(K + kPlaneThreads - 1) / kPlaneThreads, kPlaneThreads, 0, st>>>(
      disp, height, width, samples, K, ws.planes, counts, ws.sums);
  if (int s = check_launch()) return s;
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    cus = 256;  // only sizes the grid
  const int64_t n = static_cast<int64_t>(height) * width;
  const dim3 grid(static_cast<unsigned>((n + kPlaneBlockPix - 1) / kPlaneBlockPix),
                  (K + kPlaneChunk - 1) / kPlaneChunk);
  plane_score_kernel<<<grid, kPlaneThreads, 0, st>>>(disp, valid, n, width, ws.planes, K,
                                                     static_cast<double>(threshold), counts);
  if (int s = check_launch()) return s;
  const int blocks = static_cast<int>(std::min<int64_t>(cus, (n + kPlaneThreads - 1) / kPlaneThreads));
  plane_sums_kernel<<<blocks, kPlaneThreads, 0, st>>>(disp, valid, height, width, ws.planes, counts, K,
                                                      static_cast<double>(threshold), ws.sums, best);
  if (int s = check_launch()) return s;
  plane_solve_kernel<<<1, 1, 0, st>>>(ws.sums, height, width, plane, best);
  return check_launch();
}
