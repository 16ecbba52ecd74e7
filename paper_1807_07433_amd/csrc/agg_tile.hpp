// One TY x 16 output tile (TY = 16 or 8) of the bilateral aggregation (Sec. II-B.2,
// Eq. 8-10) on the matrix cores, shared by the plain aggregation kernel and the
// batch kernel.  64 * TY threads: wave w owns patch w, sitting at (w / 4, w % 4);
// every patch runs the same MFMA sequence whatever the tile height, so all forms
// give the same floats.
//
// Per disparity tile t of 16: the cost tile plus halo is staged in LDS as fp16 hi /
// lo planes, each thread moving 4-column chunks (two float2 loads, one 8-byte LDS
// store per plane).  The MFMA results, scaled by 1/Z, are transposed through an LDS
// output tile out[dd * OST + y * 16 + x] = A[16 t + dd][by + y][bx + x], which the
// sink reads after a barrier: sink(t, out) is called by every thread.  Staging and
// output tiles are both double-buffered, so one barrier per disparity tile orders
//     loads of t+1 issued -> MFMAs of t -> output t -> staging t+1 -> barrier -> sink t
// and the sink's global stores drain while the next tile's MFMAs run.
#pragma once

#include "aggregate_mfma.hpp"

namespace rsv {

template <int A, int TY>
__host__ __device__ inline size_t agg_tile_lds_bytes() {
  using G = AggGeo<A, TY>;
  return sizeof(float) * (G::NOB * 16 * G::OST + G::RAW + G::SKN) +
         (2 /*hi,lo*/ * 2 /*buffers*/ * 16 * G::PLANE + 4 * 64 /*dummy*/) * sizeof(_Float16);
}

// cost(d, Y, X) = cost[d * cps + Y * crs + X] (a dense volume: cps = H W, crs = W).
// guide_at(Y, X): guide intensity at in-image (Y, X).
// Values for disparities >= D or pixels outside the image are meaningless.
template <int A, int TY, typename GuideAt, typename Sink>
__device__ __forceinline__ void agg_tile(const float* __restrict__ cost, int64_t cps, int crs, int H,
                                         int W, int D,
                                         const BilateralK& bk, int by, int bx, GuideAt guide_at,
                                         Sink& sink, unsigned char* smem) {
  using G = AggGeo<A, TY>;
  constexpr int NT = G::NT;
  constexpr int NW = NT / 64;                    // waves
  constexpr int PPW = G::NP / NW;                // patches per wave
  constexpr int NITEM = 16 * G::NCH;             // (disparity, chunk) items per tile
  constexpr int SPT = (NITEM + NT - 1) / NT;     // items per thread
  float* out = reinterpret_cast<float*>(smem);  // NOB output tiles
  float* gt = out + G::NOB * 16 * G::OST;
  float* skt = gt + G::RAW;
  _Float16* hi = reinterpret_cast<_Float16*>(skt + G::SKN);
  _Float16* lo = hi + 2 * 16 * G::PLANE;
  const int tid = opaque_tid(), lane = tid & 63, wave = tid >> 6;
  _Float16* dummy = lo + 2 * 16 * G::PLANE + 4 * lane;  // store target of surplus items
  const int x0 = bx - A - G::PAD;  // image column of tile column 0 (even)

  // Item q of this thread: disparity dd of the tile, chunk k = 4 columns of one row.
  // meta = dd | in-image column mask << 4 (bit e: column X + e) | (offset of the
  // chunk in the hi / lo planes + 1, 0 past the item list) << 8; eoff = dd * cps +
  // Y * crs + X, the element offset from the tile's first disparity plane (32-bit
  // for cps and H * crs <= 2^26), added to a per-tile uniform base.  The fetch and
  // store steps read opaque copies of meta, so that the decisions derived from it are
  // recomputed per tile rather than hoisted out of the tile loop as lane masks
  // (which, at radius 6, spilled and were reloaded from scratch every tile).
  static_assert(2 * 16 * G::PLANE + 1 < (1 << 24), "plane offset field");
  int eoff[SPT];
  unsigned meta[SPT];
#pragma unroll
  for (int q = 0; q < SPT; ++q) {
    const int it = tid + q * NT;
    const int dd = it / G::NCH, k = it - dd * G::NCH;
    const int row = k / G::CPR, c4 = 4 * (k - row * G::CPR);
    const int Y = by - A + row, X = x0 + c4;
    unsigned m = 0;
    if (it < NITEM && Y >= 0 && Y < H)
#pragma unroll
      for (int e = 0; e < 4; ++e) m |= (X + e >= 0 && X + e < W) ? (1u << e) : 0u;
    const unsigned ldso1 = it < NITEM ? static_cast<unsigned>(dd * G::PLANE + 4 * k) + 1u : 0u;
    meta[q] = static_cast<unsigned>(dd) | (m << 4) | (ldso1 << 8);
    eoff[q] = m ? dd * static_cast<int>(cps) + Y * crs + X : 0;
  }
  float4_t pre[SPT];
  // The load form is chosen per wave (uniform branch): whole 4-column chunks as one
  // 16-byte load when every lane has one, else per-column predicated loads.  No
  // register is then written on one path while the other path's loads are pending.
  // A chunk start is only 4-byte aligned (odd strides, e.g. a target view of a joint
  // volume, or odd widths); gfx950 serves such 16-byte global loads.  Past the last
  // disparity tile nothing is loaded.
  auto fetch = [&](int t) {
    const float* base = cost + static_cast<int64_t>(16 * t) * cps;
#pragma unroll
    for (int q = 0; q < SPT; ++q) {
      float4_t v = {0.f, 0.f, 0.f, 0.f};
      unsigned mq = meta[q];
      asm volatile("" : "+v"(mq));
      const unsigned m = mq >> 4 & 15u;
      const unsigned mm = 16 * t + static_cast<int>(mq & 15u) < D ? m : 0u;
      const float* p = base + eoff[q];  // column X of the chunk (X may be < 0 at the border)
      if (__all(mm == 0xFu)) {
        const float4_a4 a = *reinterpret_cast<const float4_a4*>(p);
        v[0] = a[0]; v[1] = a[1]; v[2] = a[2]; v[3] = a[3];
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e)
          if (mm & (1u << e)) v[e] = p[e];
      }
      pre[q] = v;
    }
  };
  // Every thread stores every item (surplus ones to its dummy slot), so all loads of
  // the fetch are consumed on every path.
  auto store = [&](int buf) {
#pragma unroll
    for (int q = 0; q < SPT; ++q) {
      half4_t h, l;
      split4(pre[q], h, l);
      unsigned mq = meta[q];
      asm volatile("" : "+v"(mq));
      const unsigned ldso1 = mq >> 8;
      const bool real = ldso1 != 0;
      const int ldso = static_cast<int>(ldso1) - 1;
      *reinterpret_cast<half4_t*>(real ? hi + buf * 16 * G::PLANE + ldso : dummy) = h;
      *reinterpret_cast<half4_t*>(real ? lo + buf * 16 * G::PLANE + ldso : dummy) = l;
    }
  };

  fetch(0);
  // the guide and spatial tables are staged while tile 0 loads
  for (int i = tid; i < G::RAW; i += NT) {
    const int r = i / G::TC, c = i - r * G::TC;
    const int Y = by - A + r, X = x0 + c;
    gt[i] = (Y >= 0 && Y < H && X >= 0 && X < W) ? guide_scaled(guide_at(Y, X), bk) : INFINITY;
  }
  for (int i = tid; i < G::SKR * G::SKC; i += NT) {
    const int a = i / G::SKC, b = i - a * G::SKC;
    const int dy = a - 3 - A, dx = b - 3 - A - G::PAD;
    skt[i] = (dy >= -A && dy <= A && dx >= -A && dx <= A) ? spatial_exponent(dy, dx, bk.kd) : INFINITY;
  }
  store(0);
  __syncthreads();
  fetch(1);  // in flight while the weights are computed

  PatchPos pp[PPW];
  half8_t whi[PPW][G::KS], wlo[PPW][G::KS];
  float4_t iz[PPW];
#pragma unroll
  for (int k = 0; k < PPW; ++k) {
    const int patch = wave + k * NW;
    pp[k] = PatchPos{patch >> 2, patch & 3};
    const int i = lane & 15;
    const bool pin = by + 4 * pp[k].pr + (i >> 2) < H && bx + 4 * pp[k].pc + (i & 3) < W;
    iz[k] = patch_weights<A, TY>(whi[k], wlo[k], pp[k], lane, pin, gt, skt);
  }

  const int ndt = (D + 15) >> 4;
  for (int t = 0; t < ndt; ++t) {
    const int buf = t & 1;
    float* o = out + (G::NOB == 2 ? buf : 0) * 16 * G::OST;
    float4_t vals[PPW];
#pragma unroll
    for (int k = 0; k < PPW; ++k) {
      const float4_t acc = patch_mfma<A, TY>(whi[k], wlo[k], hi + buf * 16 * G::PLANE,
                                             lo + buf * 16 * G::PLANE, pp[k], lane);
#pragma unroll
      for (int e = 0; e < 4; ++e) vals[k][e] = acc[e] * iz[k][e];
    }
    // a single output tile was read by the sink of tile t - 1 after the last barrier
    if (G::NOB == 1) __syncthreads();
#pragma unroll
    for (int k = 0; k < PPW; ++k)
      *reinterpret_cast<float4_t*>(o + (lane & 15) * G::OST + (4 * pp[k].pr + (lane >> 4)) * 16 +
                                   4 * pp[k].pc) = vals[k];
    // Keep the staging store (which waits for the loads) after the MFMAs: without
    // this fence the scheduler moves its conversions into the MFMA chain and the
    // loads' latency is no longer hidden.
    __builtin_amdgcn_sched_barrier(0);
    // staging buffer buf ^ 1 was last read by the MFMAs of tile t - 1 and (double
    // buffering) output tile buf by the sink of tile t - 2, both before the previous
    // barrier
    store(buf ^ 1);
    __syncthreads();
    sink(t, static_cast<const float*>(o));
    fetch(t + 2);  // in flight during the next tile's MFMAs
  }
}

}  // namespace rsv
