// Sinks of the aggregation tiles for volumes that are only needed through their
// winner-take-all results (Sec. II-B.3): the target volume's argmax (rsv_aggregate_argmax
// and the batch kernel's target items) and the reference volume's winner with its
// neighbours for Eq. 12 (rsv_aggregate_select and the batch kernel's reference tiles).
#pragma once

#include "aggregate_mfma.hpp"

namespace rsv {

// (b, a) <- the better of (b, a) and the quad lane selected by the DPP quad_perm
// pattern PERM: the larger value, the lower d on ties.
template <int PERM>
__device__ __forceinline__ void quad_merge(float& b, int& a) {
  const float ob = __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(b), PERM, 0xF, 0xF, false));
  const int oa = __builtin_amdgcn_mov_dpp(a, PERM, 0xF, 0xF, false);
  if (ob > b || (ob == b && oa < a)) {
    b = ob;
    a = oa;
  }
}

// agg_tile sink for a volume that is only needed through its argmax over d (the
// target volume of Sec. II-B.3): the 16 x 16 pixels' running winner, nothing written
// until the end; the select kernel's order (the first maximum over d).  Two forms:
// * state null (the LDS-loaded tile): thread i covers pixel i / 4 and disparities
//   4 (i % 4) .. + 3 of the tile: its first maximum, then the quad's (lower d on
//   ties), then against the earlier tiles' winner (replaced only when strictly
//   greater).  All four threads of a quad keep the same winner in registers.
// * state in LDS (the register-staged tile, whose registers are full): thread p <
//   256 scans pixel p's 16 values in order against the winner kept in LDS.
struct ArgmaxSink {
  int D;
  float* state = nullptr;  // [2][256]: best, then arg bits
  float best = -INFINITY;
  int arg = 0;

  __device__ __forceinline__ void operator()(int t, const float* o) {
    using G = AggGeo<1, 16>;
    if (state) {
      const int p = threadIdx.x;
      if (p >= 256) return;
      float b = t == 0 ? -INFINITY : state[p];
      int a = t == 0 ? 0 : __float_as_int(state[256 + p]);
      const int n = min(16, D - 16 * t);
      for (int dd = 0; dd < n; ++dd) {
        const float v = o[dd * G::OST + p];
        if ((t == 0 && dd == 0) || v > b) {
          b = v;
          a = 16 * t + dd;
        }
      }
      state[p] = b;
      state[256 + p] = __int_as_float(a);
      return;
    }
    const int i = threadIdx.x, p = i >> 2, q = i & 3;
    float b = -INFINITY;
    int a = 0x7fffffff;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int d = 16 * t + 4 * q + k;
      const float v = o[(4 * q + k) * G::OST + p];
      if (d < D && v > b) {
        b = v;
        a = d;
      }
    }
    // the quad's lanes i ^ 1, then i ^ 2 (DPP quad permutations, no LDS traffic)
    quad_merge<0xB1>(b, a);
    quad_merge<0x4E>(b, a);
    if (t == 0 || b > best) {
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
// maximum over d, ties to the lowest d, and the values at d - 1 and d + 1) from all
// 1024 threads, in registers; shared by rsv_aggregate_select and the batch kernel's
// reference tiles.  Thread i covers pixel i / 4 and disparities 4 (i % 4) .. + 3 of
// each 16-disparity tile: its first maximum, then two quad permutations merge the four
// (larger value, lower d on ties).  When the tile's winner replaces the running one,
// its neighbours are read from the output tile, still in LDS; at the tile's edges they
// are the previous tile's last value and the next tile's first.  The winner, its value
// and the values at d - 1 and d + 1 are exactly the scan's wherever Eq. 12 uses them
// (0 < d < D - 1).
struct RefQuadSink {
  int D;
  float best = -INFINITY, am = 0.f, ap = 0.f, lastv = 0.f;
  int arg = 0;
  bool pend = false;

  __device__ __forceinline__ void operator()(int t, const float* o) {
    using G = AggGeo<1, 16>;
    const int i = threadIdx.x, p = i >> 2, q = i & 3;
    float b = -INFINITY;
    int a = 0x7fffffff;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int d = 16 * t + 4 * q + k;
      const float v = o[(4 * q + k) * G::OST + p];
      if (d < D && v > b) {
        b = v;
        a = d;
      }
    }
    quad_merge<0xB1>(b, a);
    quad_merge<0x4E>(b, a);
    if (pend) {  // the running winner sat at d = 16 t - 1: its right neighbour is d = 16 t
      ap = o[p];
      pend = false;
    }
    if (t == 0 || b > best) {
      const int k = a - 16 * t;  // the winner's place in the tile
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
