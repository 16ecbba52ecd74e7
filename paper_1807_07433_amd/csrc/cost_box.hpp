// The ZNCC cost tile for blocks of 7x7 and larger (Sec. II-B.1, Eq. 3-5), shared by
// the plain cost kernel and the batch kernels so both produce the same float for every
// entry (cost_tile_for below picks it or the direct tile of cost_tile.hpp by radius).
//
// A tile is 64 consecutive left-block centres u (u may run past W, up to W + D - 2,
// to fill the target volume) times kBoxTH rows, for every disparity, worked by one
// block of kBoxWaves waves.  An entry needs, at its centre (u, v), the window sum
// over the (2R+1)^2 block of the products P_d(y, x) = l(y, x) r(y, x - d) (l the left
// image, r the warped target, both clamped to the image edge).  Neighbouring centres
// share most of their windows, so the tile forms these sums as sliding sums instead
// of a (2R+1)^2-term dot product per entry:
//   1. horizontal: h(y, u) = sum over k of P_d(y, u + k), for every row y of the tile
//      and its halo; a lane takes a run of 8 centres of one row and slides along it
//      (2 FMAs per step, the left values held in registers);
//   2. vertical: a lane takes one centre column and slides the window down the
//      kBoxTH rows (2 additions per step), then forms the entry.
// Everything is FP64.  The product of a uint8 left value and an FP32 warped value is
// exact, so are all partial sums, and so is the numerator n sum - S_l S_r (Eq. 3 with
// the means multiplied out); the entry's only rounding is the scaling by 1/e_l and
// 1/e_r.  (For float left images the products are still exact and the sums carry
// FP64 rounding.)
// The waves take the disparities in turn (wave w: d = w, w + kBoxWaves, ...), each
// with its own LDS buffer of h, so no block barrier separates disparities.
// Disparities come in chunks of kBoxDC: per chunk the block loads the warped rows the
// chunk reads and S_r and 1/e_r of every target centre it meets, so LDS use does not
// depend on D.
// The value for (u, v, d) is written to ref[d * ref_plane + v * ref_row + u]
// (u < ref_cols) and, for the dual layout, to tar[d][v][u - d] (0 <= u - d < W): the
// identity stated after Eq. 5.  The joint layout (ref_cols = W + D - 1, no tar) holds
// both volumes in one: the target one is its view with plane stride ref_plane + 1.
#pragma once

#include "cost_tile.hpp"

namespace rsv {

constexpr int kBoxTH = 16;                    // rows per tile
constexpr int kBoxWaves = 8;
constexpr int kBoxThreads = 64 * kBoxWaves;
constexpr int kBoxDC = 64;                    // disparities per chunk
constexpr int kBoxTC = kCostTW + kBoxDC - 1;  // target centres a chunk meets per row
constexpr int kBoxTCS = 128;                  // their row stride in LDS
constexpr int kBoxRun = 8;                    // centres per lane in the horizontal pass
static_assert(kBoxTH % 4 == 0 && kBoxTCS >= kBoxTC, "target statistics: 4 rows per item");

// LDS layout of one tile, in bytes.
template <int R>
struct BoxGeo {
  static constexpr int K = 2 * R + 1;
  static constexpr int ROWS = kBoxTH + 2 * R;  // tile rows with the block halo
  static constexpr int LW = kCostTW + 2 * R;    // left tile width
  static constexpr int WS = kBoxTC + 2 * R;    // warped columns one chunk reads
  // warped row stride, 1 mod 32 words: a half-wave of the horizontal pass (8 rows x 4
  // runs 8 columns apart) then reads distinct banks
  static constexpr int WSP = (WS + 30) / 32 * 32 + 1;
  static constexpr int JOBS = ROWS * (kCostTW / kBoxRun);  // horizontal runs per disparity
  static constexpr int PASSES = (JOBS + 63) / 64;
  // h is stored column-major, [centre][row], with an odd column stride: the horizontal
  // pass's lanes (8 rows x 4 runs per half-wave) and the vertical pass's lanes (one
  // column each) then hit distinct banks
  static constexpr int HS = ROWS | 1;
  static constexpr size_t ts_off = 0;                                         // double [TH][TCS]: S_r
  static constexpr size_t ti_off = ts_off + 8 * kBoxTH * kBoxTCS;           // float [TH][TCS]: 1/e_r
  static constexpr size_t wt_off = ti_off + 4 * kBoxTH * kBoxTCS;           // float [ROWS][WSP]
  static constexpr size_t hb_off = (wt_off + 4 * ROWS * WSP + 15) / 16 * 16;  // double [waves][TW][HS]
  static constexpr size_t bytes = hb_off + 8 * kBoxWaves * kCostTW * HS;
  // set-up scratch, inside the h buffers: the left tile, its row sums and squares,
  // S_l and 1/e_l of every centre
  static constexpr size_t lt_off = hb_off;                                    // float [ROWS][LW]
  static constexpr size_t lr_off = (lt_off + 4 * ROWS * LW + 15) / 16 * 16;   // double [2][ROWS][TW]
  static constexpr size_t ls_off = lr_off + 16 * ROWS * kCostTW;              // double [TH][TW]
  static constexpr size_t li_off = ls_off + 8 * kBoxTH * kCostTW;            // float [TH][TW]
  static_assert(li_off + 4 * kBoxTH * kCostTW <= bytes, "set-up scratch fits in the h buffers");
  static_assert(bytes <= 160 * 1024, "one tile fits in LDS");
};

// BoxGeo<R>::bytes for a runtime R (0 outside 1 .. RSV_MAX_BLOCK_RADIUS).
inline size_t box_tile_lds_bytes(int R) {
  switch (R) {
    case 1: return BoxGeo<1>::bytes;
    case 2: return BoxGeo<2>::bytes;
    case 3: return BoxGeo<3>::bytes;
    case 4: return BoxGeo<4>::bytes;
    default: return 0;
  }
}

// Word 3 of a gfx9 buffer resource for raw 32-bit accesses (32-bit data format).
constexpr int kBufferWord3 = 0x00020000;

// Stores x at byte offset off of the window [row, row + bytes): offsets outside it
// (negative ones included, as unsigned) are dropped by the buffer unit's range check.
__device__ __forceinline__ void store_row(float* row, int bytes, int off, float x) {
  const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(row, 0, bytes, kBufferWord3);
  __builtin_amdgcn_raw_buffer_store_b32(__float_as_int(x), rs, off, 0, 0);
}

// LDS accesses of one wave take effect in the order the wave issues them, so a wave
// reading back what it wrote needs only the compiler to keep that order.
__device__ __forceinline__ void wave_lds_order() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// warped_at(y, x) returns the warped target at in-image (y, x).  TAR: out.tar may be
// non-null (the dual layout); with TAR false the target stores are not compiled.
// Needs BoxGeo<R>::bytes of LDS at smem and kBoxThreads threads.
template <int R, bool TAR, typename TL, typename WarpAt>
__device__ __forceinline__ void cost_box_tile(const TL* __restrict__ left, int64_t lpitch, WarpAt warped_at,
                                          int H, int W, int D, float sigma_min, int u0, int v0,
                                          const CostOut& out, unsigned char* smem) {
  using G = BoxGeo<R>;
  constexpr int K = G::K, ROWS = G::ROWS, LW = G::LW, HS = G::HS, NT = kBoxThreads, TW = kCostTW;
  constexpr int NL = kBoxRun + 2 * R;  // left / warped values of one horizontal run
  constexpr double n = K * K;
  const int tid = opaque_tid();
  const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // d is uniform per wave
  double* const ts = reinterpret_cast<double*>(smem + G::ts_off);
  float* const ti = reinterpret_cast<float*>(smem + G::ti_off);
  float* const wt = reinterpret_cast<float*>(smem + G::wt_off);
  double* const hb = reinterpret_cast<double*>(smem + G::hb_off) + wave * kCostTW * HS;

  // ---- set-up: the left tile, S_l and 1/e_l of every centre, the runs' left values
  double lv[G::PASSES][NL];  // pass p: row (lane % 8) + 8 p, centres 8 (lane / 8) ..
  double sl[kBoxTH];        // S_l of this lane's centre column, rows 0 .. TH - 1
  float il[kBoxTH];         // 1/e_l
  {
    float* const lt = reinterpret_cast<float*>(smem + G::lt_off);
    double* const lr = reinterpret_cast<double*>(smem + G::lr_off);
    double* const ls = reinterpret_cast<double*>(smem + G::ls_off);
    float* const li = reinterpret_cast<float*>(smem + G::li_off);
#pragma unroll 1
    for (int i = tid; i < ROWS * LW; i += NT) {
      const int r = i / LW, c = i - r * LW;
      lt[i] = pixel(left, lpitch, clampi(v0 - R + r, 0, H - 1), clampi(u0 - R + c, 0, W - 1));
    }
    __syncthreads();
#pragma unroll 1
    for (int i = tid; i < ROWS * TW; i += NT) {  // row sums of the K columns right of c
      const int r = i / TW, c = i - r * TW;
      double s = 0.0, q = 0.0;
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const double x = lt[r * LW + c + k];
        s += x;
        q = fma(x, x, q);
      }
      lr[i] = s;
      lr[ROWS * TW + i] = q;
    }
    __syncthreads();
#pragma unroll 1
    for (int i = tid; i < kBoxTH * TW; i += NT) {
      double s = 0.0, q = 0.0;
#pragma unroll
      for (int j = 0; j < K; ++j) {
        s += lr[i + j * TW];
        q += lr[ROWS * TW + i + j * TW];
      }
      ls[i] = s;
      li[i] = inv_block_norm(n, s, q, sigma_min);
    }
#pragma unroll
    for (int p = 0; p < G::PASSES; ++p) {
      const int jy = (lane & 7) + 8 * p, jq = lane >> 3;
      const bool on = jy < ROWS;
      const float* src = lt + (on ? jy * LW + jq * kBoxRun : 0);
#pragma unroll
      for (int m = 0; m < NL; ++m) lv[p][m] = on ? static_cast<double>(src[m]) : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int v = 0; v < kBoxTH; ++v) {
      sl[v] = ls[v * TW + lane];
      il[v] = li[v * TW + lane];
    }
  }

  const int u = u0 + lane;
  const int ref_bytes = 4 * max(0, out.ref_cols - u0);  // the tile's part of a volume row
  const int tar_bytes = 4 * W;
  const int64_t plane = static_cast<int64_t>(H) * W;
#pragma unroll 1
  for (int dc = 0; dc < D; dc += kBoxDC) {
    __syncthreads();  // the set-up, or the previous chunk, is done with LDS
    // warped rows: tile column c is image column cw0 + c
    const int cw0 = u0 - R - (dc + kBoxDC - 1);
#pragma unroll 1
    for (int i = tid; i < ROWS * G::WS; i += NT) {
      const int r = i / G::WS, c = i - r * G::WS;
      wt[r * G::WSP + c] = warped_at(clampi(v0 - R + r, 0, H - 1), clampi(cw0 + c, 0, W - 1));
    }
    __syncthreads();
    // S_r and 1/e_r of target centre x = cw0 + R + t (table column t, block over warped
    // columns t .. t + 2R), four rows v = 4g .. 4g + 3 per item
#pragma unroll 1
    for (int i = tid; i < kBoxTC * (kBoxTH / 4); i += NT) {
      const int g = i / kBoxTC, t = i - g * kBoxTC;
      double hs[4 + 2 * R], hq[4 + 2 * R];
#pragma unroll
      for (int y = 0; y < 4 + 2 * R; ++y) {
        const float* w = wt + (4 * g + y) * G::WSP + t;
        double s = 0.0, q = 0.0;
#pragma unroll
        for (int k = 0; k < K; ++k) {
          const double x = w[k];
          s += x;
          q = fma(x, x, q);
        }
        hs[y] = s;
        hq[y] = q;
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        double S = 0.0, Q = 0.0;
#pragma unroll
        for (int j = 0; j < K; ++j) {
          S += hs[v + j];
          Q += hq[v + j];
        }
        ts[(4 * g + v) * kBoxTCS + t] = S;
        ti[(4 * g + v) * kBoxTCS + t] = inv_block_norm(n, S, Q, sigma_min);
      }
    }
    __syncthreads();

    const int dend = min(D, dc + kBoxDC);
#pragma unroll 1
    for (int d = dc + wave; d < dend; d += kBoxWaves) {
      // centre c's target block at d starts at warped column c + off; its statistics
      // sit in table column c + off
      const int off = dc + kBoxDC - 1 - d;
      // 1. horizontal sums h(y, c) over the K products right of c
#pragma unroll
      for (int p = 0; p < G::PASSES; ++p) {
        const int y = (lane & 7) + 8 * p, c0 = (lane >> 3) * kBoxRun;
        if (8 * (p + 1) <= ROWS || y < ROWS) {
          const float* wr = wt + y * G::WSP + c0 + off;
          double wv[NL];
#pragma unroll
          for (int m = 0; m < NL; ++m) wv[m] = wr[m];
          double h = 0.0;
#pragma unroll
          for (int m = 0; m < K; ++m) h = fma(lv[p][m], wv[m], h);
          double hh[kBoxRun];
          hh[0] = h;
#pragma unroll
          for (int i = 1; i < kBoxRun; ++i) {
            h = fma(lv[p][i + 2 * R], wv[i + 2 * R], h);
            h = fma(-lv[p][i - 1], wv[i - 1], h);
            hh[i] = h;
          }
#pragma unroll
          for (int i = 0; i < kBoxRun; ++i) hb[(c0 + i) * HS + y] = hh[i];
        }
      }
      wave_lds_order();
      // 2. vertical sums down this lane's column, and the entries.  Stores go through
      // a buffer window per row: a row at or past H gets an empty window, and columns
      // outside the volume fall outside the window, whose range check drops them, so
      // the row loop has no branches and its LDS reads can be issued early.
      double hsum = 0.0;
#pragma unroll
      for (int y = 0; y < K; ++y) hsum += hb[lane * HS + y];
      const double* tsr = ts + lane + off;
      const float* tir = ti + lane + off;
      float* const rbase = out.ref + d * out.ref_plane + u0;
#pragma unroll
      for (int v = 0; v < kBoxTH; ++v) {
        if (v > 0) hsum = (hsum + hb[lane * HS + v + 2 * R]) - hb[lane * HS + v - 1];
        const double num = fma(n, hsum, -(sl[v] * tsr[v * kBoxTCS]));
        const float c = (static_cast<float>(num) * il[v]) * tir[v * kBoxTCS];
        const bool row_in = v0 + v < H;  // uniform
        store_row(rbase + static_cast<int64_t>(v0 + v) * out.ref_row, row_in ? ref_bytes : 0, lane * 4, c);
        if constexpr (TAR)
          store_row(out.tar + d * plane + static_cast<int64_t>(v0 + v) * W, row_in ? tar_bytes : 0, (u - d) * 4, c);
      }
      wave_lds_order();  // the next disparity's horizontal pass rewrites h
    }
  }
}

// ------------------------------------------------------------ tile by block radius
// The sliding-sum tile issues about 2 (2R + 3) + 12 operations per entry against the
// direct tile's (2R + 1)^2 + 3, but each of its disparities is a chain of LDS round
// trips, which the direct tile does not have.  Measured at 1280x720, D = 64 (direct
// tile, then this one): 3x3 0.057 / 0.090 ms, 5x5 0.090-0.093 / 0.099 ms, 7x7
// 0.117-0.121 / 0.106 ms, 9x9 0.210 / 0.120 ms.  Blocks of 7x7 and larger take it.
template <int R>
constexpr bool cost_uses_box() { return R >= 3; }
constexpr int kDirectTH = 4;  // rows of a direct tile (64 x 4 centres, 256 threads)
template <int R>
constexpr int cost_tile_rows() { return cost_uses_box<R>() ? kBoxTH : kDirectTH; }
template <int R>
constexpr int cost_tile_threads() { return cost_uses_box<R>() ? kBoxThreads : kCostTW * kDirectTH; }
inline int cost_tile_rows_rt(int R) { return R >= 3 ? kBoxTH : kDirectTH; }
inline int cost_tile_threads_rt(int R) { return R >= 3 ? kBoxThreads : kCostTW * kDirectTH; }
// LDS bytes of one tile for block radius R and D disparities.
inline size_t cost_tile_lds(int R, int D) {
  return R >= 3 ? box_tile_lds_bytes(R) : sizeof(float) * cost_tile_lds_floats(D, R, kDirectTH);
}

// One tile of cost_tile_rows<R>() rows at (u0, v0), with cost_tile_threads<R>() threads
// and cost_tile_lds(R, D) bytes of LDS at smem.
template <int R, bool TAR, typename TL, typename WarpAt>
__device__ __forceinline__ void cost_tile_for(const TL* __restrict__ left, int64_t lpitch, WarpAt warped_at,
                                              int H, int W, int D, float sigma_min, int u0, int v0,
                                              const CostOut& out, unsigned char* smem) {
  if constexpr (cost_uses_box<R>())
    cost_box_tile<R, TAR>(left, lpitch, warped_at, H, W, D, sigma_min, u0, v0, out, smem);
  else
    cost_tile<R, kDirectTH, TAR>(left, lpitch, warped_at, H, W, D, sigma_min, u0, v0, out,
                                 reinterpret_cast<float*>(smem));
}

}  // namespace rsv
