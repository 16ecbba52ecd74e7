// Sinks of the aggregation tiles for volumes that are only needed through their
// winner-take-all results (Sec. II-B.3): the target volume's argmax (rsv_aggregate_argmax
// and the batch kernel's target items) and the reference volume's winner with its
// neighbours for Eq. 12 (rsv_aggregate_select and the batch kernel's reference tiles).
// Both take, per pixel, a window [lo, hi] of candidate disparities: the whole range
// for the full method, or the restricted search of Sec. IV (rsv_aggregate_restricted_*).
#pragma once

#include "aggregate_mfma.hpp"
#include "select_math.hpp"

namespace rsv {

// Winners are compared as (key, d) pairs, key = wta_key(value): the larger key, and
// the lower d between equal keys.  (-inf, INT_MAX) stands for "no candidate".  This
// order is total, so the lanes' winners of consecutive disparity ranges merge in any
// grouping into the winner of one scan over d (the select kernel's).
__device__ __forceinline__ bool wta_better(float kb, int db, float ka, int da) {
  return kb > ka || (kb == ka && db < da);
}

// The first maximum (wta_key order) over the candidates among the four disparities
// 16 t + 4 q .. + 3 of tile t held in the output tile o for pixel p: the key and d,
// (-inf, INT_MAX) when none of them lies in [lo, hi].
__device__ __forceinline__ void lane_scan(const float* o, int t, int q, int p, int lo, int hi, float& b,
                                          int& a) {
  using G = AggGeo<1, 16>;
  float v[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) v[k] = o[(4 * q + k) * G::OST + p];  // all read, then compared
  b = -INFINITY;
  a = 0x7fffffff;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int d = 16 * t + 4 * q + k;
    const float key = wta_key(v[k]);
    if (d >= lo && d <= hi && (key > b || a == 0x7fffffff)) {
      b = key;
      a = d;
    }
  }
}

// (b, a) <- the better of (b, a) and the quad lane selected by the DPP quad_perm
// pattern PERM (wta_better).
template <int PERM>
__device__ __forceinline__ void quad_merge(float& b, int& a) {
  const float ob = __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(b), PERM, 0xF, 0xF, false));
  const int oa = __builtin_amdgcn_mov_dpp(a, PERM, 0xF, 0xF, false);
  if (wta_better(ob, oa, b, a)) {
    b = ob;
    a = oa;
  }
}

// The candidates of tile t for this thread's pixel, merged over its quad: thread i
// covers pixel i / 4 and disparities 4 (i % 4) .. + 3; all four lanes of a quad end
// with the tile's winner ((-inf, INT_MAX): no candidate in this tile).
__device__ __forceinline__ void tile_winner(const float* o, int t, int lo, int hi, float& b, int& a) {
  const int i = threadIdx.x, p = i >> 2, q = i & 3;
  lane_scan(o, t, q, p, lo, hi, b, a);
  quad_merge<0xB1>(b, a);  // lanes i ^ 1, then i ^ 2 (no LDS traffic)
  quad_merge<0x4E>(b, a);
}

// agg_tile sink for a volume that is only needed through its argmax over d (the
// target volume of Sec. II-B.3): the 16 x 16 pixels' running winner, nothing written
// until the end; the select kernel's order (the first maximum over d of wta_key).
// Two forms:
// * state null (the LDS-loaded tile): the quad lanes of a pixel take the tile's
//   winner (tile_winner), then the running winner is replaced only when beaten; the
//   candidates are d in [lo, hi] (lo = 0, hi = D - 1 for the full method).
// * state in LDS (the register-staged tile, whose registers are full): thread p <
//   256 scans pixel p's 16 values in order against the winner kept in LDS (full
//   range only).
struct ArgmaxSink {
  int D;
  float* state = nullptr;  // [2][256]: best, then arg bits
  int lo = 0, hi = D - 1;
  float best = -INFINITY;
  int arg = 0x7fffffff;

  __device__ __forceinline__ void operator()(int t, const float* o) {
    using G = AggGeo<1, 16>;
    if (state) {
      const int p = threadIdx.x;
      if (p >= 256) return;
      float b = t == 0 ? -INFINITY : state[p];
      int a = t == 0 ? 0 : __float_as_int(state[256 + p]);
      const int n = min(16, D - 16 * t);
      for (int dd = 0; dd < n; ++dd) {
        const float v = wta_key(o[dd * G::OST + p]);
        if ((t == 0 && dd == 0) || v > b) {
          b = v;
          a = 16 * t + dd;
        }
      }
      state[p] = b;
      state[256 + p] = __int_as_float(a);
      return;
    }
    float b;
    int a;
    tile_winner(o, t, lo, hi, b, a);
    if (wta_better(b, a, best, arg)) {
      best = b;
      arg = a;
    }
  }

  // Writes the winners after the last call: one thread per in-image pixel.
  __device__ __forceinline__ void finish(int32_t* disp, int H, int W, int by, int bx) const {
    int p;
    int a;
    if (state) {
      p = threadIdx.x;
      if (p >= 256) return;
      a = __float_as_int(state[256 + p]);  // written by this thread
    } else {
      if (threadIdx.x & 3) return;
      p = threadIdx.x >> 2;
      a = arg;
    }
    const int Y = by + (p >> 4), X = bx + (p & 15);
    if (Y < H && X < W) disp[static_cast<int64_t>(Y) * W + X] = a;
  }
};

// agg_tile_dma sink for the reference volume: the select kernel's scan result (first
// maximum over d of wta_key, and the values at d - 1 and d + 1) from all 1024
// threads, in registers; shared by rsv_aggregate_select, the restricted search and
// the batch kernel's reference tiles.  The quad lanes of a pixel take the tile's
// winner among the candidates d in [lo, hi] (tile_winner).  When it replaces the
// running one, its neighbours are read from the output tile, still in LDS; at the
// tile's edges they are the previous tile's last value and the next tile's first
// (the caller's tiles are consecutive and reach one disparity past every window on
// both sides, or the range's ends).  The winner, its value and the values at d - 1
// and d + 1 are exactly the scan's wherever Eq. 12 uses them (0 < d < D - 1).
struct RefQuadSink {
  int D;
  int lo = 0, hi = D - 1;
  float best = -INFINITY, am = 0.f, ap = 0.f, lastv = 0.f;
  int arg = 0x7fffffff;
  bool pend = false;

  __device__ __forceinline__ void operator()(int t, const float* o) {
    using G = AggGeo<1, 16>;
    const int p = threadIdx.x >> 2;
    float b;
    int a;
    tile_winner(o, t, lo, hi, b, a);
    if (pend) {  // the running winner sat at d = 16 t - 1: its right neighbour is d = 16 t
      ap = o[p];
      pend = false;
    }
    if (wta_better(b, a, best, arg)) {  // a real candidate: a is in tile t
      const int k = a - 16 * t;  // the winner's place in the tile, 0 .. 15
      best = b;
      arg = a;
      am = k > 0 ? o[(k - 1) * G::OST + p] : lastv;
      pend = k == 15;
      if (!pend) ap = o[(k + 1) * G::OST + p];
    }
    lastv = o[15 * G::OST + p];
  }
};

}  // namespace rsv
