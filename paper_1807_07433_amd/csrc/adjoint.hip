// The differentiable form: the loss
//     L(theta, I_l, I_r) = sum over p in Omega of A_ref(p, d*(p))
// (aggregated reference cost of Eq. 8 at frozen disparities d* on a frozen pixel
// set Omega), its value from a cost volume (rsv_selected_aggregate_sum) and its
// gradient with respect to the warp plane (Sec. II-A) and both images
// (rsv_cost_adjoint).
//
// The chain rule runs through the bilateral weights (guide = left image, Eq. 10),
// the ZNCC of Eq. 3-5 and the linear-interpolation warp:
//   dL/dc(q, d)  = G(q, d) = sum over p in win(q), p in Omega, d*(p) = d of w(p, q) / Z(p)
//   dL/dw(p, q)  = (c(q, d*(p)) - A(p)) / Z(p)
//   G dc/dl_i    = a (r_i - mu_r) - b (l_i - mu_l),  G dc/dr_i = a (l_i - mu_l) - g (r_i - mu_r)
//   with a = G / sqrt(S_ll S_rr), b = G c / S_ll, g = G c / S_rr.
// The weights are recomputed (never stored), and so is A(p): the cost volume (any
// strided view, e.g. the reference view of the joint volume) supplies c, and no
// aggregated volume is needed.  One block covers 16 x 8 reference pixels q.  It
// stages the left tile, the warped tile and the statistics of every target block its
// pixels meet (mean and 1/sqrt(S_rr), once per block); gathers G(q, .) for its pixels
// into private LDS columns (64 disparities at a time); keeps each pixel's left-block
// gradient in registers across disparities and scatters the warped-block gradient
// into an LDS accumulator; then flushes both with float atomics.  Accumulators are
// indexed by block position, not pixel, so clamp-to-edge reads are folded onto their
// edge pixel only at the flush.  The warped-image gradient goes through the transpose
// of the interpolation into the right image, and its shift derivative
// -(I1 - I0) (1, v, u) into the plane gradient.
#include <climits>
#include <mutex>

#include "bilateral_math.hpp"
#include "warp_math.hpp"

namespace rsv {

constexpr int kAdjTX = 16;
constexpr int kAdjTY = 16;
constexpr int kAdjThreads = kAdjTX * kAdjTY;
constexpr int kAdjSlots = 16;  // disparities gathered per pass over a pixel's window
constexpr int kAdjMaxD = 256;

__global__ void adjoint_zero_kernel(float* __restrict__ a, float* __restrict__ b, int64_t n,
                                    double* __restrict__ gp, double* __restrict__ loss) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) {
    a[i] = 0.f;
    b[i] = 0.f;
  }
  if (i < 3) gp[i] = 0.0;
  if (i == 0 && loss) *loss = 0.0;
}

// Sum of the Eq. 9-10 weights of the window of (u, v), in window order, with the
// aggregation kernels' weight function; taps outside the image are skipped.
template <int A, typename T>
__device__ __forceinline__ float window_weight_sum(const T* __restrict__ g, int64_t gpitch, int H, int W,
                                                   int v, int u, float gp, const BilateralK& bk) {
  constexpr int K = 2 * A + 1;
  float z = 0.f;
#pragma unroll
  for (int j = 0; j < K; ++j)
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int y = v + j - A, x = u + k - A;
      float wt = 0.f;
      if (x >= 0 && x < W && y >= 0 && y < H)
        wt = bilateral_weight(pixel(g, gpitch, y, x), gp, j - A, k - A, bk);
      z += wt;
    }
  return z;
}

// 1 / sum of the Eq. 9-10 weights of each pixel's window.
template <int A>
__global__ __launch_bounds__(256) void zinv_kernel(const float* __restrict__ g, int64_t gpitch, int H,
                                                   int W, BilateralK bk,
                                                   float* __restrict__ zinv) {
  const int u = blockIdx.x * blockDim.x + threadIdx.x;
  const int v = blockIdx.y;
  if (u >= W || v >= H) return;
  const float z = window_weight_sum<A>(g, gpitch, H, W, v, u, pixel(g, gpitch, v, u), bk);
  zinv[static_cast<int64_t>(v) * W + u] = 1.f / z;
}

struct AdjLayout {
  int hl, ltw, lth, wtw, wth, ztw, zth, tsw;
  size_t off_ts, off_lt, off_wt, off_zt, off_dt, off_gl, off_gw, off_col, bytes;
};

// off_col holds, in turn, the row pass of the window disparity range (2 x zth x TX
// ints), the gathered G(q, .) (kAdjSlots x threads floats) and the block reduction
// (4 x threads doubles).
__host__ __device__ inline AdjLayout adj_layout(int R, int A, int D) {
  AdjLayout L;
  L.hl = R > A ? R : A;
  L.ltw = kAdjTX + 2 * L.hl;
  L.lth = kAdjTY + 2 * L.hl;
  L.wtw = kAdjTX + D - 1 + 2 * R;
  L.wth = kAdjTY + 2 * R;
  L.ztw = kAdjTX + 2 * A;
  L.zth = kAdjTY + 2 * A;
  L.tsw = kAdjTX + D - 1;  // target block centres per tile row
  size_t o = 0;
  L.off_ts = o;  // 8-byte items first
  o += sizeof(float2) * L.tsw * kAdjTY;
  L.off_lt = o;
  o += sizeof(float) * L.ltw * L.lth;
  L.off_wt = o;
  o += sizeof(float) * L.wtw * L.wth;
  L.off_zt = o;
  o += sizeof(float) * L.ztw * L.zth;
  L.off_dt = o;
  o += sizeof(int) * L.ztw * L.zth;
  L.off_gl = o;
  o += sizeof(float) * L.ltw * L.lth;
  L.off_gw = o;
  o += sizeof(float) * L.wtw * L.wth;
  o = (o + 7) & ~size_t(7);
  L.off_col = o;
  size_t col = sizeof(float) * kAdjSlots * kAdjThreads;
  const size_t red = sizeof(double) * 4 * kAdjThreads, rng = sizeof(int) * 2 * L.zth * kAdjTX;
  col = col > red ? col : red;
  col = col > rng ? col : rng;
  o += col;
  L.bytes = o;
  return L;
}

template <int R, int A>
__global__ __launch_bounds__(kAdjThreads) void adjoint_kernel(
    const float* __restrict__ left, int64_t lpitch, const float* __restrict__ right, int64_t rpitch,
    int H, int W, int D, rsv_plane pl, BilateralK bk, float sigma_min,
    const float* __restrict__ cost, int64_t cps, int64_t crs, const int32_t* __restrict__ disp,
    const uint8_t* __restrict__ mask, const float* __restrict__ zinv, float* __restrict__ gleft,
    float* __restrict__ gright, double* __restrict__ gplane, double* __restrict__ loss) {
  constexpr int K = 2 * R + 1;
  constexpr int N = K * K;
  constexpr int KA = 2 * A + 1;
  extern __shared__ __align__(16) unsigned char smem[];
  const AdjLayout Ly = adj_layout(R, A, D);
  float2* ts = reinterpret_cast<float2*>(smem + Ly.off_ts);
  float* lt = reinterpret_cast<float*>(smem + Ly.off_lt);
  float* wt = reinterpret_cast<float*>(smem + Ly.off_wt);
  float* zt = reinterpret_cast<float*>(smem + Ly.off_zt);
  int* dt = reinterpret_cast<int*>(smem + Ly.off_dt);
  float* gl = reinterpret_cast<float*>(smem + Ly.off_gl);
  float* gw = reinterpret_cast<float*>(smem + Ly.off_gw);
  float* col = reinterpret_cast<float*>(smem + Ly.off_col);
  int* rmn = reinterpret_cast<int*>(smem + Ly.off_col);
  int* rmx = rmn + Ly.zth * kAdjTX;
  double* red = reinterpret_cast<double*>(smem + Ly.off_col);

  const int tid = threadIdx.x;
  const int tx = tid % kAdjTX, ty = tid / kAdjTX;
  const int x0 = blockIdx.x * kAdjTX, y0 = blockIdx.y * kAdjTY;
  const int qx = x0 + tx, qy = y0 + ty;
  const bool in = qx < W && qy < H;
  const int hl = Ly.hl;
  const int lx0 = x0 - hl, ly0 = y0 - hl;                // left tile / grad-left origin
  const int wx0 = x0 - (D - 1) - R, wy0 = y0 - R;        // warped tile / grad-warped origin
  const int zx0 = x0 - A, zy0 = y0 - A;                  // Omega tile origin

  // Tiles hold clamp-to-edge reads at every position of the tile.
  for (int i = tid; i < Ly.ltw * Ly.lth; i += kAdjThreads) {
    const int r = i / Ly.ltw, c = i - r * Ly.ltw;
    lt[i] = left[static_cast<int64_t>(clampi(ly0 + r, 0, H - 1)) * lpitch + clampi(lx0 + c, 0, W - 1)];
    gl[i] = 0.f;
  }
  for (int i = tid; i < Ly.wtw * Ly.wth; i += kAdjThreads) {
    const int r = i / Ly.wtw, c = i - r * Ly.wtw;
    wt[i] = warp_sample(right, rpitch, W, pl, clampi(wx0 + c, 0, W - 1), clampi(wy0 + r, 0, H - 1));
    gw[i] = 0.f;
  }
  for (int i = tid; i < Ly.ztw * Ly.zth; i += kAdjThreads) {
    const int r = i / Ly.ztw, c = i - r * Ly.ztw;
    const int y = zy0 + r, x = zx0 + c;
    const bool ok = x >= 0 && x < W && y >= 0 && y < H;
    const int64_t gi = static_cast<int64_t>(y) * W + x;
    zt[i] = ok ? zinv[gi] : 0.f;
    const int dv = ok ? disp[gi] : -1;
    dt[i] = (ok && mask[gi] && dv >= 0 && dv < D) ? dv : -1;  // out-of-range d: not in Omega
  }
  __syncthreads();

  // Statistics of every target block the tile's pixels meet: the block centred on
  // tile row r, column x0 - (D - 1) + c (mean, and 1/sqrt(S_rr), or 0 where the block
  // std-dev is below sigma_min and the correlation is the constant 0).
  for (int i = tid; i < Ly.tsw * kAdjTY; i += kAdjThreads) {
    const int r = i / Ly.tsw, c = i - r * Ly.tsw;
    const float* tb = wt + r * Ly.wtw + c;
    double S = 0.0, Q = 0.0;
#pragma unroll
    for (int j = 0; j < K; ++j)
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const double x = tb[j * Ly.wtw + k];
        S += x;
        Q = fma(x, x, Q);
      }
    const double srr = fmax(Q - S * S / N, 0.0);
    const bool ok = sqrt(srr / N) >= static_cast<double>(sigma_min);
    ts[i] = make_float2(static_cast<float>(S / N), ok ? static_cast<float>(1.0 / sqrt(srr)) : 0.f);
  }
  // Range of the Omega disparities in each pixel's window, row pass (columns tx .. tx + 2A
  // of every Omega tile row): the gathers below take kAdjSlots disparities at a time.
  for (int i = tid; i < Ly.zth * kAdjTX; i += kAdjThreads) {
    const int r = i / kAdjTX, c = i - r * kAdjTX;
    int mn = INT_MAX, mx = -1;
#pragma unroll
    for (int k = 0; k < KA; ++k) {
      const int dp = dt[r * Ly.ztw + c + k];
      if (dp >= 0) {
        mn = min(mn, dp);
        mx = max(mx, dp);
      }
    }
    rmn[i] = mn;
    rmx[i] = mx;
  }

  // Left block of q (clamp-to-edge reads) and its statistics; its centred values are
  // read back from the tile (minus the mean) where needed.
  double S = 0.0, Q = 0.0;
  const float* lb0 = lt + (ty + hl - R) * Ly.ltw + tx + hl - R;
#pragma unroll
  for (int j = 0; j < K; ++j)
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const float x = lb0[j * Ly.ltw + k];
      S += x;
      Q = fma(static_cast<double>(x), static_cast<double>(x), Q);
    }
  const double sll = fmax(Q - S * S / N, 0.0);
  const bool okl = sqrt(sll / N) >= static_cast<double>(sigma_min);
  const float mul = static_cast<float>(S / N);
  const float inv_l = okl ? static_cast<float>(1.0 / sqrt(sll)) : 0.f;
  const float gq = lt[(ty + hl) * Ly.ltw + tx + hl];
  __syncthreads();  // target statistics and the row ranges complete

  int dmin = INT_MAX, dmax = -1;
#pragma unroll
  for (int j = 0; j < KA; ++j) {
    dmin = min(dmin, rmn[(ty + j) * kAdjTX + tx]);
    dmax = max(dmax, rmx[(ty + j) * kAdjTX + tx]);
  }
  if (!in) dmax = -1;  // no gathers outside the image
  if (dmax < 0) dmin = 0;  // no Omega pixel in the window: one pass (for A(q) alone)
  __syncthreads();  // the ranges' memory becomes the gather columns

  const int my_d = dt[(ty + A) * Ly.ztw + tx + A];
  const float zq = zt[(ty + A) * Ly.ztw + tx + A];
  const float* cd = cost + (my_d >= 0 ? my_d : 0) * cps;
  const bool has_p = in && my_d >= 0;
  float* mycol = col + tid;
  // ZNCC adjoint of (q, d) with weight G = dL/dc(q, d): the left-block gradient is
  // kept in registers across disparities (sum_d a_d (r - mu_r) and the scalar
  // sum_d b_d), the warped-block gradient goes to the LDS accumulator.
  float gacc[K][K];
#pragma unroll
  for (int j = 0; j < K; ++j)
#pragma unroll
    for (int k = 0; k < K; ++k) gacc[j][k] = 0.f;
  float bsum = 0.f;
  const float* cq = cost + static_cast<int64_t>(qy) * crs + qx;
  auto apply = [&](int d, float G) {
    const int tc = tx - d + (D - 1);  // target block column in the tile
    const float2 st = ts[ty * Ly.tsw + tc];
    if (st.y == 0.f) return;  // flat target block: c == 0
    const float c = cq[static_cast<int64_t>(d) * cps];
    const float a = G * inv_l * st.y;
    const float g = G * c * st.y * st.y;
    bsum = fmaf(G * c, inv_l * inv_l, bsum);
    const float* tb = wt + ty * Ly.wtw + tc;
    float* gb = gw + ty * Ly.wtw + tc;
#pragma unroll
    for (int j = 0; j < K; ++j)
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const float r = tb[j * Ly.wtw + k] - st.x;
        gacc[j][k] = fmaf(a, r, gacc[j][k]);
        atomicAdd(&gb[j * Ly.wtw + k], fmaf(a, lb0[j * Ly.ltw + k] - mul, -g * r));
      }
  };

  // One pass per kAdjSlots disparities of the window's range.  The first pass also
  // forms A(q) at q's own disparity (q in the role of p; w(p, q) = w(q, p)) and its
  // loss term.  G(q, d) = sum over p of w(p, q) / Z(p), p in win(q), d*(p) = d.
  double loss_part = 0.0;
  float Aq = 0.f;
  for (int base = dmin, first = 1; first || base <= dmax; base += kAdjSlots, first = 0) {
#pragma unroll
    for (int s = 0; s < kAdjSlots; ++s) mycol[s * kAdjThreads] = 0.f;
    float num = 0.f;
    if (in) {
#pragma unroll 1
      for (int j = 0; j < KA; ++j)
#pragma unroll
        for (int k = 0; k < KA; ++k) {
          const int Y = qy + j - A, X = qx + k - A;
          if (X >= 0 && X < W && Y >= 0 && Y < H) {
            const float gx = lt[(Y - ly0) * Ly.ltw + X - lx0];
            const float w = bilateral_weight(gx, gq, j - A, k - A, bk);
            if (first && has_p) num = fmaf(w, cd[Y * crs + X], num);
            const int zi = (ty + j) * Ly.ztw + tx + k;
            const int ds = dt[zi] - base;
            if (static_cast<unsigned>(ds) < static_cast<unsigned>(kAdjSlots)) mycol[ds * kAdjThreads] += w * zt[zi];
          }
        }
    }
    if (first && has_p) {
      Aq = num * zq;
      loss_part = Aq;
    }
    if (in && okl) {
#pragma unroll 1
      for (int s = 0; s < kAdjSlots; ++s) {
        const float G = mycol[s * kAdjThreads];
        if (G != 0.f && base + s < D) apply(base + s, G);
      }
    }
  }
  // dL/dw(q, p') = (c(p', d*(q)) - A(q)) / Z(q) for p' in win(q), through the guide:
  // t(q, p') = dL/dw * dw/dg(p') goes to g(p') and -t to g(q).  The sum over p' for q
  // is formed here; the sums over q for each p' are gathered below by the owner of p'
  // (no LDS atomics: one float atomic per LDS address costs about one lane at a time).
  if (has_p) {
    float s = 0.f;
#pragma unroll 1
    for (int j = 0; j < KA; ++j)
#pragma unroll
      for (int k = 0; k < KA; ++k) {
        const int Y = qy + j - A, X = qx + k - A;
        if (X >= 0 && X < W && Y >= 0 && Y < H) {
          const float gx = lt[(Y - ly0) * Ly.ltw + X - lx0];
          const float w = bilateral_weight(gx, gq, j - A, k - A, bk);
          s += (cd[Y * crs + X] - Aq) * zq * bilateral_weight_dgq(w, gx, gq, bk);
        }
      }
    atomicAdd(&gl[(qy - ly0) * Ly.ltw + qx - lx0], -s);
  }
  __syncthreads();  // every pixel's gathers are done: the columns take its left-block gradient
  // The left-block gradient of q, -bsum (l - mu_l) + gacc, goes to the left tile one
  // block row at a time: each q writes its row j, then the owner of each position of
  // the row band sums the (up to K) values aimed at it.
  float* rowv = col;  // [K][threads]
#pragma unroll
  for (int j = 0; j < K; ++j) {
#pragma unroll
    for (int k = 0; k < K; ++k)
      rowv[k * kAdjThreads + tid] = (in && okl) ? fmaf(-bsum, lb0[j * Ly.ltw + k] - mul, gacc[j][k]) : 0.f;
    __syncthreads();
    // positions: tile rows hl - R + j + ty' (ty' = 0 .. 15), columns hl - R + c (c = 0 .. 15 + 2R)
    constexpr int BW = kAdjTX + 2 * R;
    for (int i = tid; i < kAdjTY * BW; i += kAdjThreads) {
      const int qyl = i / BW, c = i - qyl * BW;  // q row in the block, tile column offset
      float acc = 0.f;
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const int qxl = c - k;  // q column in the block
        if (qxl >= 0 && qxl < kAdjTX) acc += rowv[k * kAdjThreads + qyl * kAdjTX + qxl];
      }
      gl[(qyl + hl - R + j) * Ly.ltw + c + hl - R] += acc;
    }
    __syncthreads();
  }
  // per q: A(q), 1 / Z(q) (0 where q is not in Omega), d*(q), guide at q
  float4* qinfo = reinterpret_cast<float4*>(col);
  qinfo[tid] = make_float4(Aq, has_p ? zq : 0.f, __int_as_float(has_p ? my_d : 0), gq);
  __syncthreads();
  // Owner gather: position p' of the left tile adds sum over the block's q with p' in
  // win(q) of t(q, p') (the weight and its derivative as in the scatter form).
  for (int i = tid; i < Ly.ltw * Ly.lth; i += kAdjThreads) {
    const int r = i / Ly.ltw, c = i - r * Ly.ltw;
    const int Y = ly0 + r, X = lx0 + c;  // p'
    if (X < 0 || X >= W || Y < 0 || Y >= H) continue;
    const int j0 = max(Y - (y0 + kAdjTY - 1), -A), j1 = min(Y - y0, A);  // dy = Y - q.y
    const int k0 = X - (x0 + kAdjTX - 1), k1 = X - x0;                    // dx = X - q.x
    if (j0 > j1 || k0 > A || k1 < -A) continue;
    const float gx = lt[i];
    const float* cp = cost + static_cast<int64_t>(Y) * crs + X;
    float acc = 0.f;
    int dlast = -1;
    float clast = 0.f;
    for (int dy = j0; dy <= j1; ++dy) {
      const float4* qrow = qinfo + (Y - dy - y0) * kAdjTX + X - x0;  // q = p' - (dy, dx): qrow[-dx]
#pragma unroll
      for (int dx = -A; dx <= A; ++dx) {
        if (dx < k0 || dx > k1) continue;
        const float4 qv = qrow[-dx];
        if (qv.y == 0.f) continue;
        const int dq = __float_as_int(qv.z);
        if (dq != dlast) {
          clast = cp[static_cast<int64_t>(dq) * cps];
          dlast = dq;
        }
        const float w = bilateral_weight(gx, qv.w, dy, dx, bk);
        acc += (clast - qv.x) * qv.y * bilateral_weight_dgq(w, gx, qv.w, bk);
      }
    }
    gl[i] += acc;
  }
  __syncthreads();

  // Flush: left-image gradient; positions outside the image belong to their
  // clamp-to-edge pixel.
  for (int i = tid; i < Ly.ltw * Ly.lth; i += kAdjThreads) {
    const float g = gl[i];
    if (g == 0.f) continue;
    const int r = i / Ly.ltw, c = i - r * Ly.ltw;
    const int Y = clampi(ly0 + r, 0, H - 1), X = clampi(lx0 + c, 0, W - 1);
    atomicAdd(&gleft[static_cast<int64_t>(Y) * W + X], g);
  }
  // Flush: warped-image gradient through the warp transpose, and the plane gradient.
  double t0 = 0.0, t1 = 0.0, t2 = 0.0;
  for (int i = tid; i < Ly.wtw * Ly.wth; i += kAdjThreads) {
    const float g = gw[i];
    if (g == 0.f) continue;
    const int r = i / Ly.wtw, c = i - r * Ly.wtw;
    const int Y = clampi(wy0 + r, 0, H - 1), X = clampi(wx0 + c, 0, W - 1);
    const WarpTap tap = warp_tap(pl, X, Y, W);
    const float* row = right + static_cast<int64_t>(Y) * rpitch;
    const double i0 = row[tap.c0], i1 = row[tap.c1];
    atomicAdd(&gright[static_cast<int64_t>(Y) * W + tap.c0], static_cast<float>(g * (1.0 - tap.f)));
    atomicAdd(&gright[static_cast<int64_t>(Y) * W + tap.c1], static_cast<float>(g * tap.f));
    const double t = -static_cast<double>(g) * (i1 - i0);
    t0 += t;
    t1 += t * Y;
    t2 += t * X;
  }
  red[tid] = t0;
  red[kAdjThreads + tid] = t1;
  red[2 * kAdjThreads + tid] = t2;
  red[3 * kAdjThreads + tid] = loss_part;
  __syncthreads();
  for (int s = kAdjThreads / 2; s > 0; s >>= 1) {
    if (tid < s)
      for (int m = 0; m < 4; ++m) red[m * kAdjThreads + tid] += red[m * kAdjThreads + tid + s];
    __syncthreads();
  }
  if (tid == 0) {
    atomicAdd(&gplane[0], red[0]);
    atomicAdd(&gplane[1], red[kAdjThreads]);
    atomicAdd(&gplane[2], red[2 * kAdjThreads]);
    if (loss) atomicAdd(loss, red[3 * kAdjThreads]);
  }
}

struct AdjointArgs {
  rsv_image l, r;
  rsv_plane pl;
  const rsv_params* p;
  const float* cost;
  int64_t cps, crs;
  const int32_t* disp;
  const uint8_t* mask;
  float *gl, *gr;
  double *gp, *loss;
  float* zinv;
};

template <int R, int A>
int launch_adjoint(const AdjointArgs& a, hipStream_t st) {
  const int H = a.l.height, W = a.l.width, D = a.p->D;
  const BilateralK bk = bilateral_constants(a.p->gamma_d, a.p->gamma_r);
  const int64_t n = static_cast<int64_t>(H) * W;
  adjoint_zero_kernel<<<dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, st>>>(a.gl, a.gr, n,
                                                                                           a.gp, a.loss);
  if (int s = check_launch()) return s;
  zinv_kernel<A><<<dim3((W + 255) / 256, H), dim3(256), 0, st>>>(
      static_cast<const float*>(a.l.data), a.l.pitch, H, W, bk, a.zinv);
  if (int s = check_launch()) return s;
  const AdjLayout Ly = adj_layout(R, A, D);
  auto kern = adjoint_kernel<R, A>;
  if (Ly.bytes > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       static_cast<int>(Ly.bytes));
    if (e != hipSuccess) {
      set_hip_error(e);
      return RSV_E_HIP;
    }
  }
  const dim3 grid((W + kAdjTX - 1) / kAdjTX, (H + kAdjTY - 1) / kAdjTY);
  kern<<<grid, dim3(kAdjThreads), Ly.bytes, st>>>(
      static_cast<const float*>(a.l.data), a.l.pitch, static_cast<const float*>(a.r.data), a.r.pitch, H, W, D,
      a.pl, bk, a.p->sigma_min, a.cost, a.cps, a.crs, a.disp, a.mask, a.zinv, a.gl, a.gr, a.gp, a.loss);
  return check_launch();
}

template <int R>
int dispatch_adjoint_a(const AdjointArgs& a, hipStream_t st) {
  switch (a.p->agg_radius) {
    case 1: return launch_adjoint<R, 1>(a, st);
    case 2: return launch_adjoint<R, 2>(a, st);
    case 3: return launch_adjoint<R, 3>(a, st);
    case 4: return launch_adjoint<R, 4>(a, st);
    case 5: return launch_adjoint<R, 5>(a, st);
    case 6: return launch_adjoint<R, 6>(a, st);
    default: return RSV_E_PARAM;
  }
}

// Checks of a strided view cost(d, v, u) = cost[d*plane_stride + v*row_stride + u]
// over D x H x W (32-bit offsets within a plane, 64-bit across planes).
inline int validate_cost_view(const float* cost, int64_t plane_stride, int64_t row_stride, int H, int W,
                              int D) {
  if (!cost) return RSV_E_NULL;
  if (row_stride < W || plane_stride < 1) return RSV_E_SHAPE;
  if (static_cast<int64_t>(H - 1) * row_stride + W > INT32_MAX) return RSV_E_SHAPE;
  if (plane_stride > INT64_MAX / (D > 0 ? D : 1)) return RSV_E_SHAPE;
  if (!aligned(cost, 4)) return RSV_E_ALIGN;
  return RSV_OK;
}

int validate_adjoint(const rsv_image& left, const rsv_image& right, const rsv_params* p, const float* cost,
                     int64_t cps, int64_t crs, const int32_t* disp, const uint8_t* mask, const float* gl,
                     const float* gr, const double* gp, const double* loss) {
  if (int s = validate_image(left)) return s;
  if (int s = validate_image(right)) return s;
  if (int s = validate_cost_params(p)) return s;
  if (int s = validate_agg_params(p)) return s;
  if (left.dtype != RSV_F32 || right.dtype != RSV_F32) return RSV_E_DTYPE;
  if (!disp || !mask || !gl || !gr || !gp) return RSV_E_NULL;
  if (left.height != right.height || left.width != right.width) return RSV_E_SHAPE;
  if (p->D > kAdjMaxD) return RSV_E_SHAPE;
  const int K = 2 * p->block_radius + 1;
  if (left.height < K || left.width < K) return RSV_E_SHAPE;
  if (int s = validate_cost_view(cost, cps, crs, left.height, left.width, p->D)) return s;
  if (!aligned(disp, 4) || !aligned(gl, 4) || !aligned(gr, 4) || !aligned(gp, 8) || (loss && !aligned(loss, 8)))
    return RSV_E_ALIGN;
  return RSV_OK;
}

int run_adjoint(const AdjointArgs& a, hipStream_t st) {
  switch (a.p->block_radius) {
    case 1: return dispatch_adjoint_a<1>(a, st);
    case 2: return dispatch_adjoint_a<2>(a, st);
    case 3: return dispatch_adjoint_a<3>(a, st);
    case 4: return dispatch_adjoint_a<4>(a, st);
    default: return RSV_E_PARAM;
  }
}

// Loss of the differentiable form from a cost volume: per pixel p in Omega the
// aggregation of Eq. 8 at its one selected disparity (the weights of Eq. 9-10, the
// same window sums as the adjoint), summed in double; one atomic per block.
template <int A, typename T>
__global__ __launch_bounds__(256) void selected_aggregate_sum_kernel(
    const float* __restrict__ cost, int64_t cps, int64_t crs, const T* __restrict__ g, int64_t gpitch,
    int H, int W, int D, BilateralK bk, const int32_t* __restrict__ disp, const uint8_t* __restrict__ mask,
    double* __restrict__ out) {
  constexpr int K = 2 * A + 1;
  __shared__ double red[256];
  const int u = blockIdx.x * 16 + threadIdx.x % 16;
  const int v = blockIdx.y * 16 + threadIdx.x / 16;
  double part = 0.0;
  if (u < W && v < H) {
    const int64_t i = static_cast<int64_t>(v) * W + u;
    const int d = disp[i];
    if (mask[i] && d >= 0 && d < D) {
      const float gp = pixel(g, gpitch, v, u);
      const float z = window_weight_sum<A>(g, gpitch, H, W, v, u, gp, bk);
      const float* cd = cost + d * cps;
      float num = 0.f;
#pragma unroll
      for (int j = 0; j < K; ++j)
#pragma unroll
        for (int k = 0; k < K; ++k) {
          const int y = v + j - A, x = u + k - A;
          if (x >= 0 && x < W && y >= 0 && y < H)
            num = fmaf(bilateral_weight(pixel(g, gpitch, y, x), gp, j - A, k - A, bk), cd[y * crs + x], num);
        }
      part = num * (1.f / z);
    }
  }
  red[threadIdx.x] = part;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicAdd(out, red[0]);
}

template <typename T>
int launch_selected_aggregate_sum(const float* cost, int64_t cps, int64_t crs, const rsv_image& guide,
                                  const rsv_params* p, const int32_t* disp, const uint8_t* mask, double* out,
                                  hipStream_t st) {
  const int H = guide.height, W = guide.width;
  const BilateralK bk = bilateral_constants(p->gamma_d, p->gamma_r);
  const dim3 grid((W + 15) / 16, (H + 15) / 16);
  const T* g = static_cast<const T*>(guide.data);
#define RSV_SAS(A_)                                                                                   \
  case A_:                                                                                            \
    selected_aggregate_sum_kernel<A_, T><<<grid, 256, 0, st>>>(cost, cps, crs, g, guide.pitch, H, W,  \
                                                               p->D, bk, disp, mask, out);            \
    break;
  switch (p->agg_radius) {
    RSV_SAS(1) RSV_SAS(2) RSV_SAS(3) RSV_SAS(4) RSV_SAS(5) RSV_SAS(6)
    default: return RSV_E_PARAM;
  }
#undef RSV_SAS
  return check_launch();
}

// Sum of agg[disp(p)][p] over pixels with mask(p) != 0 (the loss of the
// differentiable form).  Block partial sums in double, then one atomic per block.
__global__ __launch_bounds__(256) void selected_sum_kernel(const float* __restrict__ agg,
                                                           const int32_t* __restrict__ disp,
                                                           const uint8_t* __restrict__ mask, int H,
                                                           int W, int D, double* __restrict__ out) {
  __shared__ double red[256];
  const int64_t n = static_cast<int64_t>(H) * W;
  double s = 0.0;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * 256) {
    const int d = disp[i];
    if (mask[i] && d >= 0 && d < D) s += agg[d * n + i];
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicAdd(out, red[0]);
}

__global__ void zero_double_kernel(double* p) { *p = 0.0; }

}  // namespace rsv

extern "C" int rsv_selected_cost_sum(const float* agg_ref, const int32_t* disp, const uint8_t* mask,
                                     int32_t height, int32_t width, int32_t D, double* out,
                                     void* stream) {
  using namespace rsv;
  if (!agg_ref || !disp || !mask || !out) return RSV_E_NULL;
  if (height < 1 || width < 1 || D < 1 || D > RSV_MAX_D) return RSV_E_SHAPE;
  if (!aligned(agg_ref, 4) || !aligned(disp, 4) || !aligned(out, 8)) return RSV_E_ALIGN;
  hipStream_t st = as_stream(stream);
  zero_double_kernel<<<1, 1, 0, st>>>(out);
  if (int s = check_launch()) return s;
  const int64_t n = static_cast<int64_t>(height) * width;
  const int blocks = static_cast<int>((n + 255) / 256 < 1024 ? (n + 255) / 256 : 1024);
  selected_sum_kernel<<<blocks, 256, 0, st>>>(agg_ref, disp, mask, height, width, D, out);
  return check_launch();
}

extern "C" int rsv_selected_aggregate_sum(const float* cost, int64_t plane_stride, int64_t row_stride,
                                          rsv_image guide, const rsv_params* p, const int32_t* disp,
                                          const uint8_t* mask, double* out, void* stream) {
  using namespace rsv;
  if (int s = validate_image(guide)) return s;
  if (int s = validate_agg_params(p)) return s;
  if (!disp || !mask || !out) return RSV_E_NULL;
  if (int s = validate_cost_view(cost, plane_stride, row_stride, guide.height, guide.width, p->D)) return s;
  if (!aligned(disp, 4) || !aligned(out, 8)) return RSV_E_ALIGN;
  hipStream_t st = as_stream(stream);
  zero_double_kernel<<<1, 1, 0, st>>>(out);
  if (int s = check_launch()) return s;
  if (guide.dtype == RSV_U8)
    return launch_selected_aggregate_sum<uint8_t>(cost, plane_stride, row_stride, guide, p, disp, mask, out, st);
  return launch_selected_aggregate_sum<float>(cost, plane_stride, row_stride, guide, p, disp, mask, out, st);
}

extern "C" size_t rsv_cost_adjoint_workspace_bytes(int32_t height, int32_t width) {
  if (height < 1 || width < 1) return 0;
  return sizeof(float) * static_cast<size_t>(height) * static_cast<size_t>(width);
}

extern "C" int rsv_cost_adjoint(rsv_image left, rsv_image right, rsv_plane plane, const rsv_params* p,
                                const float* cost, int64_t plane_stride, int64_t row_stride,
                                const int32_t* disp, const uint8_t* mask, float* grad_left,
                                float* grad_right, double* grad_plane, double* loss, void* workspace,
                                void* stream) {
  using namespace rsv;
  if (int s = validate_adjoint(left, right, p, cost, plane_stride, row_stride, disp, mask, grad_left,
                               grad_right, grad_plane, loss))
    return s;
  if (!workspace) return RSV_E_NULL;
  if (!aligned(workspace, 4)) return RSV_E_ALIGN;
  const AdjointArgs a{left, right, plane, p, cost, plane_stride, row_stride, disp, mask,
                      grad_left, grad_right, grad_plane, loss, static_cast<float*>(workspace)};
  return run_adjoint(a, as_stream(stream));
}

// ------------------------------------------------------- no-allocation variant
// rsv_cost_adjoint_noalloc keeps the adjoint's workspace (1 / sum of the window
// weights per pixel) in a file-scope device array instead of a caller buffer.  Each
// GPU holds its own copy for the life of the process.  In host code `scratch` names
// only a host-side stand-in, so its device address is resolved with
// hipGetSymbolAddress, once per device with that device current, and only that
// address is passed to kernels.
namespace rsv {
namespace {
constexpr size_t kAdjScratchBytes = RSV_ADJOINT_NOALLOC_MAX_PIXELS * sizeof(float);
static __device__ __align__(256) float scratch[RSV_ADJOINT_NOALLOC_MAX_PIXELS];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float* g_scratch_dev[kMaxDevices] = {};

// The device address of the current device's scratch array (resolved on first use).
int current_scratch(float** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    set_hip_error(e);
    return RSV_E_HIP;
  }
  if (dev < 0 || dev >= kMaxDevices) {
    set_hip_error(hipErrorInvalidDevice);
    return RSV_E_HIP;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      set_hip_error(e != hipSuccess ? e : hipErrorInvalidSymbol);
      return RSV_E_HIP;
    }
    g_scratch_dev[dev] = static_cast<float*>(ptr);
  }
  *out = g_scratch_dev[dev];
  return RSV_OK;
}
}  // namespace
}  // namespace rsv

extern "C" int rsv_cost_adjoint_noalloc(rsv_image left, rsv_image right, rsv_plane plane, const rsv_params* p,
                                        const float* cost, int64_t plane_stride, int64_t row_stride,
                                        const int32_t* disp, const uint8_t* mask, float* grad_left,
                                        float* grad_right, double* grad_plane, double* loss, void* stream) {
  using namespace rsv;
  if (int s = validate_adjoint(left, right, p, cost, plane_stride, row_stride, disp, mask, grad_left,
                               grad_right, grad_plane, loss))
    return s;
  if (rsv_cost_adjoint_workspace_bytes(left.height, left.width) > kAdjScratchBytes) return RSV_E_SHAPE;
  float* ws = nullptr;
  if (int s = current_scratch(&ws)) return s;
  const AdjointArgs a{left, right, plane, p, cost, plane_stride, row_stride, disp, mask,
                      grad_left, grad_right, grad_plane, loss, ws};
  return run_adjoint(a, as_stream(stream));
}
