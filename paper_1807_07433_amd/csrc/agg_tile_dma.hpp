// The aggregation tile of agg_tile.hpp with the cost tiles brought into LDS by
// direct global-to-LDS loads (global_load_lds_dwordx4).  Same weights, same fp16
// split of the same floats, same MFMA sequence per patch, so it produces the same
// aggregated floats as agg_tile.
//
// Register staging holds only one tile in flight, and at the aggregation's rate a
// disparity tile's loads take longer than its MFMAs; these loads need no registers.
// LDS holds
//     raw      the fp32 cost tile as loaded (16 B per 4-column chunk, item order)
//     hl[2]    two pairs of fp16 hi / lo planes: the MFMAs read one while the next
//              tile is converted into the other
//     out      the transposed output tile
// Every thread converts exactly the chunks its own loads brought in, so a thread
// needs no barrier between its loads landing and its conversion, nor between its
// conversion and reloading its raw chunks.  Iteration t:
//     MFMAs(t) from hl[t % 2], with this thread's part of tile t+1 converted from
//     raw into hl[(t+1) % 2] between the last K-steps (its loads waited for just
//     before) -> tile t+2's loads into raw -> barrier -> output(t) -> barrier ->
//     sink(t)
// so the conversion runs beside the matrix pipe instead of in a phase of its own,
// and tile t+2's loads are in flight during the output, the sink and the first
// K-steps of tile t+1.
//
// The loads are issued with inline assembly and waited for by hand ("no vector-memory
// operations outstanding": the wave's only loads in flight at that point are the
// ones being waited for, plus any stores of the previous sink).  Lanes whose chunk has
// no data (rows outside the image, disparities >= D) load a valid address anyway and
// are masked when converting; lanes past the item list issue nothing.  Border chunks
// load the in-row chunk [Xc, Xc + 3], Xc = clamp(X, 0, W - 4), and the conversion
// picks their columns from it.  Needs W >= 4.  The cost volume is read as
// cost[d * cps + Y * crs + X], as in agg_tile.
#pragma once

#include "agg_tile.hpp"

namespace rsv {

// LDS layout: out | raw | hi0 | lo0 | hi1 | lo1 | guide tile | spatial table.  The
// last two are read only by the weight computation, before the first sink call; from
// then on a sink may use the LDS from agg_tile_dma_spare_offset on.
template <int A>
__host__ __device__ constexpr size_t agg_tile_dma_spare_offset() {
  using G = AggGeo<A, 16>;
  return sizeof(float) * 16 * G::OST + 16 * G::NCH * 16 /*raw: B per chunk*/ +
         2 /*buffers*/ * 2 /*hi,lo*/ * 16 * G::PLANE * sizeof(_Float16);
}

template <int A>
__host__ __device__ constexpr size_t agg_tile_dma_lds_bytes() {
  using G = AggGeo<A, 16>;
  return agg_tile_dma_spare_offset<A>() + sizeof(float) * (G::RAW + G::SKN);
}

// The LDS-loaded tile fits one CU's 160 KiB of LDS up to radius 5.
template <int A>
constexpr bool agg_dma_fits() {
  return agg_tile_dma_lds_bytes<A>() <= 160 * 1024;
}

// One 16-byte-per-lane global-to-LDS load: lane l's 16 bytes at base + voff (a
// uniform base in SGPRs, a 32-bit byte offset per lane) go to LDS byte address
// lds_wave + 16 l (lds_wave is the wave's destination base, uniform).  The
// destination goes through m0, which the statement saves and restores itself (the
// compiler reserves m0 and does not honour it as a clobber).
// lds_wave is taken from its first lane inside the statement, so it may sit in a
// vector register (inside device functions the compiler does not always keep it
// scalar).
__device__ __forceinline__ void lds_dma16(const float* base, uint32_t voff, uint32_t lds_wave) {
  uint32_t saved, dst;
  asm volatile(
      "s_mov_b32 %0, m0\n\t"
      "v_readfirstlane_b32 %1, %4\n\t"
      "s_mov_b32 m0, %1\n\t"
      "global_load_lds_dwordx4 %2, %3\n\t"
      "s_mov_b32 m0, %0"
      : "=&s"(saved), "=&s"(dst)
      : "v"(voff), "s"(base), "v"(lds_wave)
      : "memory");
}

// s_waitcnt vmcnt(n); the memory clobber keeps LDS reads of the loaded data after it.
template <int N>
__device__ __forceinline__ void wait_vm() {
  static_assert(N >= 0 && N < 16, "vmcnt");
  asm volatile("s_waitcnt vmcnt(%0)" ::"n"(N) : "memory");
}

// LDS byte address of a pointer into the workgroup's LDS (use it where the pointer is
// known to address LDS, e.g. on a kernel's __shared__ array).
__device__ __forceinline__ uint32_t lds_address(const void* p) {
  typedef const __attribute__((address_space(3))) char* lds_ptr;
  return static_cast<uint32_t>(reinterpret_cast<uintptr_t>((lds_ptr)p));
}

template <int A, typename GuideAt, typename Sink>
__device__ __forceinline__ void agg_tile_dma(const float* __restrict__ cost, int64_t cps, int crs, int H,
                                             int W, int D,
                                             const BilateralK& bk, int by, int bx, GuideAt guide_at,
                                             Sink& sink, unsigned char* smem, uint32_t smem_lds,
                                             int t_first = 0, int t_count = -1) {
  // smem_lds: LDS byte address of smem (lds_address in the kernel), so that device
  // functions holding smem as a generic pointer can address the DMA destinations.
  // t_first, t_count: the disparity tiles to aggregate (uniform over the block), by
  // default all of them; the sink is called with each tile's absolute index.
  using G = AggGeo<A, 16>;
  constexpr int NT = G::NT;                      // 1024
  constexpr int NITEM = 16 * G::NCH;             // (disparity, chunk) items per tile
  constexpr int SPT = (NITEM + NT - 1) / NT;     // items per thread
  static_assert(SPT <= 3, "wait counts below assume at most 3 loads per wave and tile");
  float* out = reinterpret_cast<float*>(smem);
  float* raw = out + 16 * G::OST;                // 16 B aligned: 16 * OST is a multiple of 4
  _Float16* hl0 = reinterpret_cast<_Float16*>(raw + 4 * NITEM);  // hi | lo of buffer 0
  _Float16* hl1 = hl0 + 2 * 16 * G::PLANE;
  float* gt = reinterpret_cast<float*>(smem + agg_tile_dma_spare_offset<A>());
  float* skt = gt + G::RAW;
  const int tid = opaque_tid(), lane = tid & 63, wave = tid >> 6;
  const int x0 = bx - A - G::PAD;

  // Item q of this thread: chunk k (4 columns of one row) of disparity dd.
  // meta = dd | in-image column mask << 4 | (X - Xc + 3) << 8; eoff = element offset
  // of the loaded chunk [Xc, Xc + 3] from the tile's first plane (0 for rows outside).
  int eoff[SPT], ldso[SPT];
  unsigned meta[SPT];
#pragma unroll
  for (int q = 0; q < SPT; ++q) {
    const int it = tid + q * NT;
    const int dd = it / G::NCH, k = it - dd * G::NCH;
    const int row = k / G::CPR, c4 = 4 * (k - row * G::CPR);
    const int Y = by - A + row, X = x0 + c4;
    const bool yok = it < NITEM && Y >= 0 && Y < H;
    unsigned m = 0;
    if (yok)
#pragma unroll
      for (int e = 0; e < 4; ++e) m |= (X + e >= 0 && X + e < W) ? (1u << e) : 0u;
    const int Xc = X < 0 ? 0 : (X > W - 4 ? W - 4 : X);
    // every in-image column of the chunk lies in [Xc, Xc + 3], so |X - Xc| <= 3 when
    // m != 0; chunks wholly outside keep shift 0
    const int sh = m ? X - Xc : 0;
    meta[q] = static_cast<unsigned>(dd) | (m << 4) | (static_cast<unsigned>(sh + 3) << 8);
    eoff[q] = yok ? dd * static_cast<int>(cps) + Y * crs + Xc : 0;
    ldso[q] = it < NITEM ? dd * G::PLANE + 4 * k : -1;
  }

  // Byte offsets from the tile's first plane fit 32 bits: eoff <= 15 cps + (H-1) crs +
  // W - 1 < 2^30 under the 2^26 limits on cps and (H-1) crs + W.
  auto issue = [&](int t) {
    const float* base = uniform(cost + static_cast<int64_t>(16 * t) * cps);
#pragma unroll
    for (int q = 0; q < SPT; ++q) {
      if (q * NT + 64 * wave < NITEM) {  // uniform per wave
        const int d = 16 * t + static_cast<int>(meta[q] & 15u);
        const bool ok = (meta[q] >> 4 & 15u) != 0 && d < D;
        const uint32_t voff = ok ? 4u * static_cast<uint32_t>(eoff[q]) : 0u;  // plane 16 t exists
        const uint32_t dst = __builtin_amdgcn_readfirstlane(
            smem_lds + static_cast<uint32_t>(reinterpret_cast<const unsigned char*>(raw + 4 * (q * NT + 64 * wave)) -
                                             smem));
        if (tid + q * NT < NITEM) lds_dma16(base, voff, dst);
      }
    }
  };
  // item q of this thread, tile t: raw -> hi / lo
  auto convert = [&](int q, int t, _Float16* hi, _Float16* lo) {
    if (ldso[q] >= 0) {
      const int it = tid + q * NT;
      float4_t v = *reinterpret_cast<const float4_t*>(raw + 4 * it);
      // An opaque copy of the item's metadata: the decisions below are recomputed from
      // it on every tile.  Otherwise the compiler hoists them out of the tile loop as
      // dozens of lane masks, which spill to VGPR lanes and are read back every tile.
      unsigned mq = meta[q];
      asm volatile("" : "+v"(mq));
      const unsigned m = (16 * t + static_cast<int>(mq & 15u) < D) ? (mq >> 4 & 15u) : 0u;
      const int sh = static_cast<int>(mq >> 8) - 3;  // column X + e is loaded element e + sh
      if (m != 0xFu || sh != 0) {
        float4_t w = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int s = e + sh;
          float x = 0.f;
#pragma unroll
          for (int j = 0; j < 4; ++j)
            if (s == j) x = v[j];
          w[e] = (m >> e & 1u) ? x : 0.f;
        }
        v = w;
      }
      half4_t h, l;
      split4(v, h, l);
      *reinterpret_cast<half4_t*>(hi + ldso[q]) = h;
      *reinterpret_cast<half4_t*>(lo + ldso[q]) = l;
    }
  };

  const int ndt = t_count < 0 ? (D + 15) >> 4 : t_count;  // tiles t_first .. t_first + ndt - 1
  static_assert(G::KS > SPT, "the conversion of the next tile rides on the last SPT K-steps");
  issue(t_first);
  // The guide and spatial tables are staged while the first tile loads (the wait
  // for the guide loads also waits for that tile).
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
  wait_vm<0>();
#pragma unroll
  for (int q = 0; q < SPT; ++q) convert(q, t_first, hl0, hl0 + 16 * G::PLANE);
  if (ndt > 1) issue(t_first + 1);  // into the chunks this thread has just converted
  __syncthreads();  // hi / lo of the first tile, guide and spatial tables ready

  PatchPos pp;
  half8_t whi[G::KS], wlo[G::KS];
  pp = PatchPos{wave >> 2, wave & 3};
  const int i16 = lane & 15;
  const bool pin = by + 4 * pp.pr + (i16 >> 2) < H && bx + 4 * pp.pc + (i16 & 3) < W;
  const float4_t iz = patch_weights<A, 16>(whi, wlo, pp, lane, pin, gt, skt);

  for (int t = 0; t < ndt; ++t) {
    _Float16* cur = (t & 1) ? hl1 : hl0;
    _Float16* nxt = (t & 1) ? hl0 : hl1;
    const bool more = t + 1 < ndt;
    // K-step s: after its MFMAs are issued, the next tile's loads are waited for
    // (s = KS - SPT - 1) and its item q converted (s = KS - SPT + q), beside the
    // matrix pipe
    const float4_t acc = patch_mfma_then<A, 16>(whi, wlo, cur, cur + 16 * G::PLANE, pp, lane, [&](int s) {
      if (!more) return;
      if (s == G::KS - SPT - 1) wait_vm<0>();
#pragma unroll
      for (int q = 0; q < SPT; ++q)
        if (s == G::KS - SPT + q) convert(q, t_first + t + 1, nxt, nxt + 16 * G::PLANE);
    });
    if (t + 2 < ndt) issue(t_first + t + 2);
    float4_t vals;
#pragma unroll
    for (int e = 0; e < 4; ++e) vals[e] = acc[e] * iz[e];
    __syncthreads();  // hi / lo of tile t+1 ready; tile t's planes and the output tile (sink t-1) free
    *reinterpret_cast<float4_t*>(out + (lane & 15) * G::OST + (4 * pp.pr + (lane >> 4)) * 16 + 4 * pp.pc) =
        vals;
    __syncthreads();  // output t ready
    sink(t_first + t, static_cast<const float*>(out));
  }
  wait_vm<0>();  // nothing may be in flight into LDS when the block's LDS is reused
}

}  // namespace rsv
