// One tile of the ZNCC cost volumes (Sec. II-B.1, Eq. 3-5), shared by the plain
// cost kernel and the batch kernel so both produce the same float for every entry.
//
// The tile is 64 consecutive left-block centres u (u may run past W, up to
// W + D - 2, to fill the target volume) times TH rows.  Each thread owns one centre
// and walks d = 0 .. D-1: its centred left block stays in registers and the target
// block slides one column left per step through a register ring, so a step reads
// one new column of 2R+1 values from LDS and spends (2R+1)^2 FMAs.  The value for
// (u, v, d) is written to ref[d * ref_plane + v * ref_row + u] (u < ref_cols) and,
// for the dual layout, to tar[d][v][u - d] (0 <= u - d < W): the identity stated
// after Eq. 5.  The joint layout (ref_cols = W + D - 1, no tar) holds both volumes
// in one: the target one is its view with plane stride ref_plane + 1.
// The warped tile is stored minus 128 (kWarpShift): the centred left values sum to
// zero, so the dot product is unchanged while its FP32 terms stay small.  Entries
// whose target block is nearly flat (std-dev below 1 grey level, see zncc_math.hpp)
// are recomputed exactly in FP64 from the tiles, since there the FP32 sum's
// rounding, divided by a small e_r, could reach 1e-4.  Its row
// stride is a compile-time constant so the column reads use immediate offsets.
#pragma once

#include <type_traits>

#include "zncc_math.hpp"

namespace rsv {

constexpr int kCostTW = 64;
constexpr int kWarpStride = kCostTW + RSV_MAX_D - 1 + 2 * RSV_MAX_BLOCK_RADIUS + 1;  // 584
constexpr float kWarpShift = 128.f;

// Where a cost tile writes its values.
struct CostOut {
  float* ref;         // ref[d * ref_plane + v * ref_row + u] for u < ref_cols
  int64_t ref_plane;
  uint32_t ref_row;
  int ref_cols;
  float* tar;         // dense [D][H][W] target volume, or null
};

// Both volumes dense [D][H][W] (tar may be null).
__host__ __device__ inline CostOut cost_out_dual(float* ref, float* tar, int H, int W) {
  return CostOut{ref, static_cast<int64_t>(H) * W, static_cast<uint32_t>(W), W, tar};
}

// Row stride the library's own joint volumes use: W + D - 1 centres rounded up to 64,
// so every 64-centre row segment is 256-byte aligned.
__host__ __device__ inline int64_t joint_row_stride(int W, int D) {
  return (static_cast<int64_t>(W) + D - 1 + 63) / 64 * 64;
}

// The joint volume [D][H][row] over centres u = 0 .. W + D - 2.
__host__ __device__ inline CostOut cost_out_joint(float* joint, int64_t row, int H, int W, int D) {
  return CostOut{joint, H * row, static_cast<uint32_t>(row), W + D - 1, nullptr};
}

__host__ __device__ inline size_t cost_tile_lds_floats(int D, int R, int TH) {
  const size_t rows = TH + 2 * R;
  // warped tile, left tile, 1/e_r of the target centres, one flag word
  return rows * kWarpStride + rows * (kCostTW + 2 * R) + static_cast<size_t>(TH) * (kCostTW + D - 1) + 1;
}

// The volume is written through a global-address-space pointer.  Where the output
// pointer is loaded from memory (the batch kernel's pair descriptors) rather than
// passed as a kernel argument, the compiler cannot tell it is global and would emit
// flat stores, which also count in the LDS counter: every wait for the window's LDS
// reads would then wait for the stores as well.
typedef __attribute__((address_space(1))) float global_float;
__device__ __forceinline__ global_float* to_global(float* p) { return (global_float*)p; }

// warped_at(y, x) returns the warped target at in-image (y, x).  TAR: out.tar may be
// non-null (the dual layout); with TAR false the target stores are not compiled.
template <int R, int TH, bool TAR, typename TL, typename WarpAt>
__device__ __forceinline__ void cost_tile(const TL* __restrict__ left, int64_t lpitch, WarpAt warped_at,
                                          int H, int W, int D, float sigma_min, int u0, int v0,
                                          const CostOut& out, float* smem) {
  constexpr int K = 2 * R + 1;
  constexpr int NT = kCostTW * TH;
  const int tid = opaque_tid();
  const int tx = tid % kCostTW, ty = tid / kCostTW;
  constexpr int wtw = kWarpStride;          // warped tile row stride
  const int rows = TH + 2 * R;
  const int wtc = kCostTW + D - 1 + 2 * R;  // warped tile columns in use
  const int ltw = kCostTW + 2 * R;          // left tile width
  const int nt = kCostTW + D - 1;           // target centres visited by the tile
  float* wt = smem;
  float* lt = wt + rows * wtw;
  float* ir = lt + rows * ltw;
  int* flat = reinterpret_cast<int*>(ir + TH * nt);  // any target block on the exact path
  const int cw0 = u0 - (D - 1) - R;  // global column of warped tile column 0
  if (tid == 0) *flat = 0;

  // Thread (tx, ty) fills columns tx, tx + 64, ... of rows ty, ty + TH, ...
  for (int r = ty; r < rows; r += TH) {
    const int y = clampi(v0 - R + r, 0, H - 1);
    for (int c = tx; c < wtc; c += kCostTW)
      wt[r * wtw + c] = warped_at(y, clampi(cw0 + c, 0, W - 1)) - kWarpShift;
    for (int c = tx; c < ltw; c += kCostTW)
      lt[r * ltw + c] = pixel(left, lpitch, y, clampi(u0 - R + c, 0, W - 1));
  }
  __syncthreads();
  // 1/e_r for target centres x = u0 - (D-1) + c, rows v0 + r, two rows per thread:
  // thread t takes rows 2 (t / 128) and 2 (t / 128) + 1 of columns t % 128, + 128, ...
  static_assert(TH % 2 == 0 && NT / (TH / 2) == 128, "target rows are taken in pairs");
  {
    const int r = 2 * (tid >> 7);
    for (int c = tid & 127; c < nt; c += 128) {
      float i0, i1;
      target_inv_pair<R>(wt + r * wtw + c, wtw, sigma_min, i0, i1);
      ir[r * nt + c] = i0;
      ir[(r + 1) * nt + c] = i1;
      if (i0 < 0.f || i1 < 0.f) *flat = 1;
    }
  }

  LeftBlock<R, std::is_same<TL, uint8_t>::value> lb;
  lb.load(lt + ty * ltw + tx, ltw, sigma_min);
  __syncthreads();

  const int u = u0 + tx;
  const int v = v0 + ty;
  const bool row_ok = v < H;
  const int64_t plane = static_cast<int64_t>(H) * W;
  // Stores go to a per-disparity base that is the same for the whole workgroup plus
  // this thread's element offset: v * ref_row + u, and v * W + u for C_tar, whose
  // base is moved back by d so that column u - d has that offset.
  float* const cost_ref = out.ref;
  float* const cost_tar = out.tar;
  const int64_t ref_plane = out.ref_plane;
  const uint32_t roff = static_cast<uint32_t>(v) * out.ref_row + static_cast<uint32_t>(u);
  const uint32_t toff = static_cast<uint32_t>(v) * static_cast<uint32_t>(W) + static_cast<uint32_t>(u);
  const bool ref_ok = row_ok && u < out.ref_cols;
  const bool tar_ok = TAR && row_ok && cost_tar != nullptr;
  const float* wrow = wt + ty * wtw + tx + (D - 1);  // window column k at step d: wrow[k - d]
  const float* irow = ir + ty * nt + tx + (D - 1);   // 1/e_r of centre u - d: irow[-d]

  // The entry recomputed in FP64 from the unshifted images: (n l - S_l) and the
  // products are exact for uint8 and float images alike, so only the final scaling
  // rounds.  Used for target blocks marked by target_inv (std-dev below kExactSigma).
  auto exact = [&](int d, float inv_r) -> float {
    const float* lb0 = lt + ty * ltw + tx;
    double S = 0.0;
#pragma unroll 1
    for (int j = 0; j < K; ++j)
#pragma unroll 1
      for (int k = 0; k < K; ++k) S += static_cast<double>(lb0[j * ltw + k]);
    double num = 0.0;
#pragma unroll 1
    for (int j = 0; j < K; ++j) {
      const int y = clampi(v - R + j, 0, H - 1);
#pragma unroll 1
      for (int k = 0; k < K; ++k) {
        const double l = fma(static_cast<double>(K * K), static_cast<double>(lb0[j * ltw + k]), -S);
        num = fma(l, static_cast<double>(warped_at(y, clampi(u - d - R + k, 0, W - 1))), num);
      }
    }
    return static_cast<float>(num * (static_cast<double>(lb.inv) * static_cast<double>(inv_r)));
  };
  // Blocks of 3x3 and 5x5 meet nearly flat target blocks far more often (a few per
  // thousand tiles of the road frame, each costing the whole tile a pass over d), so
  // there the same sum is unrolled, reads the warped tile (minus 128: the shift drops
  // out, the left factors summing to zero) and takes S_l once per thread.
  auto exact_small = [&](int d, float inv_r, double S) -> float {
    const float* lb0 = lt + ty * ltw + tx;
    double num = 0.0;
#pragma unroll
    for (int j = 0; j < K; ++j)
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const double l = fma(static_cast<double>(K * K), static_cast<double>(lb0[j * ltw + k]), -S);
        num = fma(l, static_cast<double>(wrow[j * wtw + k - d]), num);
      }
    return static_cast<float>(num * (static_cast<double>(lb.inv) * static_cast<double>(inv_r)));
  };

  float win[K][K];  // ring: window column k at step d0 + t lives in slot (k - t) mod K
#pragma unroll
  for (int j = 0; j < K; ++j)
#pragma unroll
    for (int k = 0; k < K; ++k) win[j][k] = wrow[j * wtw + k];

  for (int d0 = 0; d0 < D; d0 += K) {
#pragma unroll
    for (int t = 0; t < K; ++t) {
      const int d = d0 + t;
      if (d >= D) break;
      if (d > 0) {
        const int slot = (K - t) % K;
#pragma unroll
        for (int j = 0; j < K; ++j) {
#pragma unroll
          for (int s = 0; s < K; ++s)
            if (s == slot) win[j][s] = wrow[j * wtw - d];
        }
      }
      float num = 0.f;
#pragma unroll
      for (int j = 0; j < K; ++j)
#pragma unroll
        for (int k = 0; k < K; ++k) num = fmaf(lb.c[j][k], win[j][(k - t + K) % K], num);
      // (negative 1/e_r: a nearly flat target block, rewritten below)
      const float c = (num * lb.inv) * irow[-d];
      if (ref_ok) to_global(cost_ref + d * ref_plane)[roff] = c;
      if constexpr (TAR) {
        const int64_t pd = d * plane;
        if (tar_ok && static_cast<unsigned>(u - d) < static_cast<unsigned>(W)) to_global(cost_tar + (pd - d))[toff] = c;
      }
    }
  }
  if (*flat) {  // uniform; never taken on textured images at 7x7 and larger blocks
    double S = 0.0;
    if constexpr (R <= 2) {
      const float* lb0 = lt + ty * ltw + tx;
#pragma unroll
      for (int j = 0; j < K; ++j)
#pragma unroll
        for (int k = 0; k < K; ++k) S += static_cast<double>(lb0[j * ltw + k]);
    }
#pragma unroll 1
    for (int d = 0; d < D; ++d) {
      const float inv_r = irow[-d];
      if (!(inv_r < 0.f)) continue;
      float c;
      if constexpr (R <= 2)
        c = exact_small(d, -inv_r, S);
      else
        c = exact(d, -inv_r);
      if (ref_ok) to_global(cost_ref + d * ref_plane)[roff] = c;
      if constexpr (TAR) {
        const int64_t pd = d * plane;
        if (tar_ok && static_cast<unsigned>(u - d) < static_cast<unsigned>(W)) to_global(cost_tar + (pd - d))[toff] = c;
      }
    }
  }
}

}  // namespace rsv
