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
// reference tiles.  Thread i covers pixel i / 4 and disparities
// 4 (i % 4) .. + 3 of each 16-disparity tile: its first maximum with the values beside
// it (from the quad's neighbouring lanes, or from the previous tile's last value),
// then two quad permutations merge the four (larger value, lower d on ties).  A
// winner at a tile's last disparity takes its right neighbour from the next tile.
// The winner, its value and the values at d - 1 and d + 1 are exactly the scan's
// wherever Eq. 12 uses them (0 < d < D - 1).
struct RefQuadSink {
  int D;
  float best = -INFINITY, am = 0.f, ap = 0.f, lastv = 0.f;
  int arg = 0;
  bool pend = false;

  template <int PERM>
  static __device__ __forceinline__ float dppf(float x) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), PERM, 0xF, 0xF, false));
  }
  template <int PERM>
  static __device__ __forceinline__ int dppi(int x) {
    return __builtin_amdgcn_mov_dpp(x, PERM, 0xF, 0xF, false);
  }
  template <int PERM>
  static __device__ __forceinline__ void merge(float& b, int& a, float& m, float& n, int& pd) {
    const float ob = dppf<PERM>(b), om = dppf<PERM>(m), on = dppf<PERM>(n);
    const int oa = dppi<PERM>(a), opd = dppi<PERM>(pd);
    if (ob > b || (ob == b && oa < a)) {
      b = ob;
      a = oa;
      m = om;
      n = on;
      pd = opd;
    }
  }

  __device__ __forceinline__ void operator()(int t, const float* o) {
    using G = AggGeo<1, 16>;
    const int i = threadIdx.x, p = i >> 2, q = i & 3;
    float v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = o[(4 * q + k) * G::OST + p];
    // quad lanes: the previous lane's last value, the next lane's first, the tile's
    // first (d = 16 t) and last (d = 16 t + 15) values
    const float prevq = dppf<0x90>(v[3]);  // quad_perm [0, 0, 1, 2]
    const float nextq = dppf<0xF9>(v[0]);  // quad_perm [1, 2, 3, 3]
    const float first = dppf<0x00>(v[0]);
    const float last = dppf<0xFF>(v[3]);
    const float left = q == 0 ? lastv : prevq;
    float b = -INFINITY, m = 0.f, n = 0.f;
    int a = 0x7fffffff, pd = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int d = 16 * t + 4 * q + k;
      if (d < D && v[k] > b) {
        b = v[k];
        a = d;
        m = k == 0 ? left : v[k - 1];
        n = k == 3 ? nextq : v[k + 1];
        pd = (k == 3 && q == 3) ? 1 : 0;
      }
    }
    merge<0xB1>(b, a, m, n, pd);
    merge<0x4E>(b, a, m, n, pd);
    if (pend) {  // the running winner sat at d = 16 t - 1: its right neighbour is d = 16 t
      ap = first;
      pend = false;
    }
    if (t == 0 || b > best) {
      best = b;
      arg = a;
      am = m;
      ap = n;
      pend = pd != 0;
    }
    lastv = last;
  }
};

}  // namespace rsv
