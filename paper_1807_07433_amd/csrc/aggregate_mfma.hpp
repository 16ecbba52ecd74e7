// Bilateral aggregation (Sec. II-B.2, Eq. 8-10) as a banded contraction on the
// matrix cores.  For a 4 x 4 patch of output pixels p and 16 disparities d:
//     A[d][p] = (sum_q w(p, q) C[d][q]) / Z(p),   Z(p) = sum_q w(p, q)
// where q runs over the union of the 16 windows: (4 + 2A) rows x 16 columns (the
// columns outside a pixel's window carry zero weight).  One v_mfma_f32_16x16x32_f16
// consumes two union rows (K = 32): M = 16 pixels, N = 16 disparities.  Weights and
// costs are each split into fp16 hi + lo parts (x = hi + lo to about 2^-22
// relative, |C| <= 1, 0 <= w <= 1), and hi*hi + hi*lo + lo*hi is accumulated in
// fp32, so the result matches an fp32 weighted sum to ~1e-7.  The weights are
// computed once per patch and stay in registers for every disparity tile.
//
// Lane layout of v_mfma_f32_16x16x32_f16 (wave64; l = lane, i = l % 16, g = l / 16):
//   A operand: A[i][8g + e], e = 0..7      B operand: B[8g + e][l % 16]
//   result:    C[4g + e][l % 16], e = 0..3
// K index 8g + e of K-step s maps to union row 2s + g/2, union column 8 (g % 2) + e.
#pragma once

#include "bilateral_math.hpp"
#include "fp16_split.hpp"

namespace rsv {

// Geometry of the LDS tiles of a TY x 16 output block at (by, bx) (TY = 16 or 8
// rows: TY / 4 x 4 patches).  The staged cost and guide tiles start at row by - A
// and column bx - A - PAD; PAD makes that column even, so four consecutive tile
// columns are one 8-byte aligned pair of float2 loads whenever the image width is
// even.  Union column c of patch column pc is tile column 4 pc + c.
template <int A, int TY>
struct AggGeo {
  static_assert(TY == 16 || TY == 8, "tile height");
  static constexpr int PAD = A & 1;
  static constexpr int NP = TY;              // patches (TY / 4 rows of 4)
  static constexpr int NT = 64 * NP;         // threads: one wave per patch
  static constexpr int UR = 4 + 2 * A;       // union rows of one patch
  static constexpr int KS = UR / 2;          // K-steps of 32
  static constexpr int TR = TY + 2 * A;      // tile rows
  static constexpr int TC = 28;              // tile columns: patch 3's union ends at 12 + 16
  static constexpr int RAW = TR * TC;
  static constexpr int CPR = TC / 4;         // 4-column chunks per tile row
  static constexpr int NCH = TR * CPR;       // chunks per disparity plane
  // halves per disparity plane; PLANE % 8 == 4 (an odd number of dword pairs) puts
  // the 16 planes read by one group of 16 lanes on distinct bank pairs
  static constexpr int PLANE = RAW + ((4 - RAW % 8) + 8) % 8;
  // spatial exponent table, indexed by (union row - py + 3, union column - px + 3)
  static constexpr int SKR = UR + 3, SKC = 19;
  static constexpr int SKN = (SKR * SKC + 3) & ~3;
  // output tile: floats per disparity (TY * 16 + 4: the planes written by
  // consecutive lanes start on distinct 4-bank groups); double-buffered for TY = 16,
  // single for TY = 8 so that two blocks fit one CU's LDS
  static constexpr int OST = TY * 16 + 4;
  static constexpr int NOB = TY == 16 ? 2 : 1;
  static_assert(2 * A + PAD <= 12, "a pixel's window must fit the 16 union columns");
};

// Largest H * W the aggregation tile accepts: its loads address 16 disparity planes
// from one base with 32-bit offsets.
constexpr int64_t kAggMaxPixels = int64_t(1) << 26;

struct PatchPos {
  int pr, pc;  // patch row / column inside the 16 x 16 block (0..3)
};

// Weights w of one lane for one patch, split into hi / lo fp16 parts (w <= 1).
// gt: guide tile of scaled guides h = g sr (+inf outside the image); skt: spatial
// exponent table (+inf outside the window).  Returns 1 / Z for the four output pixels this lane
// receives from the MFMA (patch row g = lane / 16, columns 0..3).
template <int A, int TY>
__device__ __forceinline__ float4_t patch_weights(half8_t* whi, half8_t* wlo, const PatchPos& pp,
                                                  int lane, bool pin, const float* gt, const float* skt) {
  using G = AggGeo<A, TY>;
  const int i = lane & 15, g = lane >> 4;
  const int py = i >> 2, px = i & 3;
  const float gp = pin ? gt[(4 * pp.pr + py + A) * G::TC + 4 * pp.pc + px + A + G::PAD] : 0.f;
  const float* gq = gt + (4 * pp.pr + (g >> 1)) * G::TC + 4 * pp.pc + 8 * (g & 1);
  const float* sk = skt + ((g >> 1) - py + 3) * G::SKC + 8 * (g & 1) - px + 3;
#pragma unroll
  for (int s = 0; s < G::KS; ++s) {
    float wt[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) wt[e] = bilateral_weight_s(gq[2 * s * G::TC + e], gp, sk[2 * s * G::SKC + e]);
#pragma unroll
    for (int e = 0; e < 8; e += 2) {
      half2_t h, l;
      split2(wt[e], wt[e + 1], h, l);
      whi[s][e] = h[0];
      whi[s][e + 1] = h[1];
      wlo[s][e] = l[0];
      wlo[s][e + 1] = l[1];
    }
  }
  // Each pixel's weight sum (Eq. 8's normaliser) as the product of its weights with a
  // matrix of ones, on the matrix pipe, which is idle while the weights are computed:
  // sum of hi + lo over the window, the same split weights the products use.  Lane l
  // ends with the sums of pixels 4 (l >> 4) + e, the layout of the tile's accumulator.
  half8_t ones;
#pragma unroll
  for (int e = 0; e < 8; ++e) ones[e] = static_cast<_Float16>(1.f);
  float4_t za = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int s = 0; s < G::KS; ++s) {
    za = __builtin_amdgcn_mfma_f32_16x16x32_f16(whi[s], ones, za, 0, 0, 0);
    za = __builtin_amdgcn_mfma_f32_16x16x32_f16(wlo[s], ones, za, 0, 0, 0);
  }
  float4_t iz;
#pragma unroll
  for (int e = 0; e < 4; ++e) iz[e] = za[e] > 0.f ? 1.f / za[e] : 0.f;
  return iz;
}

__device__ __forceinline__ half8_t lds_load8(const _Float16* p) {
  // two 8-byte LDS reads (the address is 8-byte aligned, not always 16)
  const half4_t a = *reinterpret_cast<const half4_t*>(p);
  const half4_t b = *reinterpret_cast<const half4_t*>(p + 4);
  half8_t r;
  r[0] = a[0]; r[1] = a[1]; r[2] = a[2]; r[3] = a[3];
  r[4] = b[0]; r[5] = b[1]; r[6] = b[2]; r[7] = b[3];
  return r;
}

// acc += W' x C over all K-steps for one patch and one 16-disparity tile held in
// LDS as hi / lo planes.
template <int A, int TY>
__device__ __forceinline__ float4_t patch_mfma(const half8_t* whi, const half8_t* wlo,
                                               const _Float16* hi, const _Float16* lo,
                                               const PatchPos& pp, int lane) {
  using G = AggGeo<A, TY>;
  const int j = lane & 15, g = lane >> 4;
  const int base = j * G::PLANE + (4 * pp.pr + (g >> 1)) * G::TC + 4 * pp.pc + 8 * (g & 1);
  float4_t acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int s = 0; s < G::KS; ++s) {
    const int off = base + 2 * s * G::TC;
    const half8_t bh = lds_load8(hi + off);
    const half8_t bl = lds_load8(lo + off);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(whi[s], bh, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(whi[s], bl, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(wlo[s], bh, acc, 0, 0, 0);
  }
  return acc;
}

// patch_mfma with `then(s)` called after K-step s's MFMAs are issued: independent
// work placed there (the next tile's conversion) issues while the matrix pipe runs.
template <int A, int TY, typename Then>
__device__ __forceinline__ float4_t patch_mfma_then(const half8_t* whi, const half8_t* wlo,
                                                    const _Float16* hi, const _Float16* lo,
                                                    const PatchPos& pp, int lane, Then then) {
  using G = AggGeo<A, TY>;
  const int j = lane & 15, g = lane >> 4;
  const int base = j * G::PLANE + (4 * pp.pr + (g >> 1)) * G::TC + 4 * pp.pc + 8 * (g & 1);
  float4_t acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int s = 0; s < G::KS; ++s) {
    const int off = base + 2 * s * G::TC;
    const half8_t bh = lds_load8(hi + off);
    const half8_t bl = lds_load8(lo + off);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(whi[s], bh, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(whi[s], bl, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(wlo[s], bh, acc, 0, 0, 0);
    then(s);
  }
  return acc;
}

}  // namespace rsv
