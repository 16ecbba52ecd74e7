// Batched form: many stereo pairs of uneven size and disparity range in one
// persistent, hipGraph-captured launch.
//
// A plan holds, per pair, the two cost volumes and the running WTA state, plus one
// global work list.  The persistent kernel (512-thread workgroups) pulls items from
// an atomic counter:
//   COST (pair, band, column tile): warp + ZNCC for 8 rows x 64 centres, the same
//       arithmetic as rsv_cost_volume (shared cost_tile), writing C_ref and C_tar;
//       then marks the band one tile closer to complete.
//   AGG (pair, tile row, tile column, ref|tar): bilateral aggregation of a 16 x 16
//       tile on the matrix cores (shared agg_tile, same arithmetic as rsv_aggregate)
//       with winner-take-all folded in: per pixel the running best, second best and
//       the winner's neighbours, updated disparity tile by disparity tile exactly as
//       a scan over d in increasing order would (ties keep the lowest d).  No
//       aggregated volume is written.
// An AGG item waits (bounded spin) until the cost bands under its window are
// complete.  Items are listed so that every item an AGG item waits for comes earlier
// in the list, and an item is only taken by a running workgroup, so every wait ends;
// a wait that exceeds its spin limit sets an error flag instead of hanging.
// A tail kernel then applies the left-right check (Eq. 11), the parabola (Eq. 12),
// post-processing and triangulation per pixel, with the plain path's functions.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <new>
#include <vector>

#include "agg_tile.hpp"
#include "cost_tile.hpp"
#include "select_math.hpp"
#include "warp_math.hpp"

namespace rsv {

constexpr int kBatchThreads = 512;
constexpr int kBandRows = kBatchThreads / kCostTW;  // 8
constexpr int kSpinLimit = 1 << 22;

enum : int { kItemCost = 0, kItemAggRef = 1, kItemAggTar = 2 };

struct PairDev {
  const uint8_t* left;
  const uint8_t* right;
  int64_t lpitch, rpitch;
  int H, W, D, nbands, ncol_tiles, tiles_x;
  rsv_plane plane;
  rsv_camera cam;
  float* cref;
  float* ctar;
  int32_t* ref_arg;
  float* ref_best;
  float* ref_am;
  float* ref_ap;
  int32_t* tar_arg;
  int32_t* band_done;
  int32_t* disp_ref;
  int32_t* disp_tar;
  float* disp_sub;
  uint8_t* valid;
  float* disp_final;
  float* xyz;
};

struct BatchArgs {
  const PairDev* pairs;
  const int4* items;  // {pair, kind, a, b}
  int n_items;
  int* head;
  int* err;
  float igd2, igr2, sigma_min;
  int tau;
};

// Running WTA state of the 256 pixels of one AGG tile, in LDS.
struct WtaState {
  float best[256], second[256], am[256], ap[256], last[256];
  int arg[256], need_ap[256];
};

__device__ __forceinline__ void argmax16(float& v, int& j) {
  // max over the 16 lanes of a lane group; ties -> lowest j
#pragma unroll
  for (int m = 1; m < 16; m <<= 1) {
    const float ov = __shfl_xor(v, m);
    const int oj = __shfl_xor(j, m);
    if (ov > v || (ov == v && oj < j)) {
      v = ov;
      j = oj;
    }
  }
}

__device__ __forceinline__ float max16(float v) {
#pragma unroll
  for (int m = 1; m < 16; m <<= 1) v = fmaxf(v, __shfl_xor(v, m));
  return v;
}

// Sink for agg_tile: folds each 16-disparity tile into the per-pixel scan state.
struct WtaSink {
  WtaState* st;
  int D;
  bool full;  // reference volume: keep second best and neighbours; target: argmax only

  __device__ __forceinline__ void operator()(int t, const PatchPos& pp, int lane, const float4_t& vals) {
    const int j = lane & 15, g = lane >> 4;
    const int base = lane & ~15;
    const int d = 16 * t + j;
    const int jl = min(15, D - 1 - 16 * t);  // last valid lane of this tile
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const float v = d < D ? vals[e] : -INFINITY;
      float m = v;
      int jm = j;
      argmax16(m, jm);
      const int pix = (4 * pp.pr + g) * 16 + 4 * pp.pc + e;
      const float v_first = __shfl(v, base);
      const float v_last = __shfl(v, base + jl);
      float sec = 0.f, vm1 = 0.f, vp1 = 0.f;
      if (full) {
        sec = max16(j == jm ? -INFINITY : v);
        vm1 = __shfl(v, base + (jm > 0 ? jm - 1 : 0));
        vp1 = __shfl(v, base + (jm < 15 ? jm + 1 : 15));
      }
      if (j == 0) {
        if (t == 0) {
          st->best[pix] = -INFINITY;
          st->second[pix] = -INFINITY;
          st->arg[pix] = -1;
          st->am[pix] = 0.f;
          st->ap[pix] = 0.f;
          st->need_ap[pix] = 0;
          st->last[pix] = 0.f;
        }
        float best = st->best[pix];
        if (full && st->need_ap[pix]) {
          st->ap[pix] = v_first;
          st->need_ap[pix] = 0;
        }
        if (m > best) {
          if (full) {
            st->second[pix] = fmaxf(best, sec);
            st->am[pix] = jm > 0 ? vm1 : st->last[pix];
            if (jm < jl) {
              st->ap[pix] = vp1;
              st->need_ap[pix] = 0;
            } else {
              st->need_ap[pix] = 1;
            }
          }
          st->best[pix] = m;
          st->arg[pix] = 16 * t + jm;
        } else if (full) {
          st->second[pix] = fmaxf(st->second[pix], m);
        }
        st->last[pix] = v_last;
      }
    }
  }
};

__device__ __forceinline__ void release_fence() { __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent"); }
__device__ __forceinline__ void acquire_fence() { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent"); }

template <int R, int A>
__global__ __launch_bounds__(kBatchThreads) void batch_kernel(BatchArgs args) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int s_item;
  WtaState* st = reinterpret_cast<WtaState*>(smem);
  unsigned char* work = smem + ((sizeof(WtaState) + 15) & ~size_t(15));
  const int tid = threadIdx.x;

  for (;;) {
    if (tid == 0) s_item = atomicAdd(args.head, 1);
    __syncthreads();
    const int it = s_item;
    __syncthreads();
    if (it >= args.n_items) break;
    const int4 w = args.items[it];
    const PairDev P = args.pairs[w.x];
    if (w.y == kItemCost) {
      const int v0 = w.z * kBandRows, u0 = w.w * kCostTW;
      auto warped_at = [&](int y, int x) { return warp_sample(P.right, P.rpitch, P.W, P.plane, x, y); };
      cost_tile<R, kBandRows>(P.left, P.lpitch, warped_at, P.H, P.W, P.D, args.sigma_min, u0, v0, P.cref,
                              P.ctar, reinterpret_cast<float*>(work));
      release_fence();
      __syncthreads();
      if (tid == 0) __hip_atomic_fetch_add(P.band_done + w.z, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      const int ty = w.z, tx = w.w;
      const int by = 16 * ty, bx = 16 * tx;
      if (tid == 0) {
        const int b_lo = max(0, (by - A) / kBandRows);
        const int b_hi = min(P.nbands - 1, (by + 15 + A) / kBandRows);
        for (int b = b_lo; b <= b_hi; ++b) {
          int spins = 0;
          while (__hip_atomic_load(P.band_done + b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) <
                 P.ncol_tiles) {
            __builtin_amdgcn_s_sleep(2);
            if (++spins > kSpinLimit) {
              atomicExch(args.err, 1);
              break;
            }
          }
        }
      }
      __syncthreads();
      acquire_fence();
      const bool full = w.y == kItemAggRef;
      WtaSink sink{st, P.D, full};
      if (full) {
        auto guide = [&](int Y, int X) { return pixel(P.left, P.lpitch, Y, X); };
        agg_tile<A, kBatchThreads>(P.cref, P.H, P.W, P.D, args.igd2, args.igr2, by, bx, guide, sink, work);
      } else {
        auto guide = [&](int Y, int X) { return warp_sample(P.right, P.rpitch, P.W, P.plane, X, Y); };
        agg_tile<A, kBatchThreads>(P.ctar, P.H, P.W, P.D, args.igd2, args.igr2, by, bx, guide, sink, work);
      }
      // agg_tile ends with a barrier: the state is complete
      for (int q = tid; q < 256; q += kBatchThreads) {
        const int Y = by + (q >> 4), X = bx + (q & 15);
        if (Y < P.H && X < P.W) {
          const int64_t i = static_cast<int64_t>(Y) * P.W + X;
          if (full) {
            P.ref_arg[i] = st->arg[q];
            P.ref_best[i] = st->best[q];
            P.ref_am[i] = st->am[q];
            P.ref_ap[i] = st->ap[q];
          } else {
            P.tar_arg[i] = st->arg[q];
          }
        }
      }
    }
    __syncthreads();  // LDS is reused by the next item
  }
}

// Left-right check, Eq. 12, post-processing and 3-D points for every pixel of every pair.
__global__ __launch_bounds__(256) void batch_tail_kernel(const PairDev* pairs, int tau) {
  const PairDev P = pairs[blockIdx.y];
  const int64_t n = static_cast<int64_t>(P.H) * P.W;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * 256) {
    const int v = static_cast<int>(i / P.W), u = static_cast<int>(i - static_cast<int64_t>(v) * P.W);
    const int arg = P.ref_arg[i];
    const int x = u - arg;
    const bool ok = (x >= 0) && (abs(arg - P.tar_arg[static_cast<int64_t>(v) * P.W + (x < 0 ? 0 : x)]) <= tau);
    const float ds = parabola(arg, P.ref_best[i], P.ref_am[i], P.ref_ap[i], P.D);
    if (P.disp_ref) P.disp_ref[i] = arg;
    if (P.disp_tar) P.disp_tar[i] = P.tar_arg[i];
    P.disp_sub[i] = ds;
    P.valid[i] = ok ? 1 : 0;
    postprocess_point(ds, ok, u, v, P.plane, P.cam, P.disp_final ? P.disp_final + i : nullptr,
                      P.xyz ? P.xyz + 3 * i : nullptr);
  }
}

__global__ void batch_reset_kernel(int* head, int* err, int32_t* counters, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) {
    *head = 0;
    *err = 0;
  }
  if (i < n) counters[i] = 0;
}

}  // namespace rsv

// ------------------------------------------------------------------ host side
struct rsv_batch_plan {
  int n_pairs = 0;
  int R = 0, A = 0;
  rsv_tuning tuning{};
  void* dev_mem = nullptr;       // one allocation: pair table, items, counters, workspace
  rsv::PairDev* d_pairs = nullptr;
  int4* d_items = nullptr;
  int* d_head = nullptr;
  int* d_err = nullptr;
  int32_t* d_counters = nullptr;
  int n_counters = 0;
  int n_items = 0;
  int max_pixels = 0;
  rsv::BatchArgs args{};
  hipStream_t capture_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int grid = 0;
};

namespace rsv {
namespace {

template <int R, int A>
const void* batch_kernel_ptr() {
  return reinterpret_cast<const void*>(batch_kernel<R, A>);
}

const void* pick_batch_kernel(int R, int A) {
#define RSV_BK(r)                                             \
  switch (A) {                                                \
    case 1: return batch_kernel_ptr<r, 1>();                  \
    case 2: return batch_kernel_ptr<r, 2>();                  \
    case 3: return batch_kernel_ptr<r, 3>();                  \
    case 4: return batch_kernel_ptr<r, 4>();                  \
    case 5: return batch_kernel_ptr<r, 5>();                  \
    case 6: return batch_kernel_ptr<r, 6>();                  \
    default: return nullptr;                                  \
  }
  switch (R) {
    case 1: RSV_BK(1)
    case 2: RSV_BK(2)
    case 3: RSV_BK(3)
    case 4: RSV_BK(4)
    default: return nullptr;
  }
#undef RSV_BK
}

size_t batch_lds_bytes(int R, int A, int maxD) {
  size_t agg = 0;
  switch (A) {
    case 1: agg = agg_tile_lds_bytes<1>(); break;
    case 2: agg = agg_tile_lds_bytes<2>(); break;
    case 3: agg = agg_tile_lds_bytes<3>(); break;
    case 4: agg = agg_tile_lds_bytes<4>(); break;
    case 5: agg = agg_tile_lds_bytes<5>(); break;
    default: agg = agg_tile_lds_bytes<6>(); break;
  }
  const size_t cost = sizeof(float) * cost_tile_lds_floats(maxD, R, kBandRows);
  return ((sizeof(WtaState) + 15) & ~size_t(15)) + std::max(agg, cost);
}

int validate_pair(const rsv_pair_desc& pd, int K) {
  if (int s = validate_image(pd.left)) return s;
  if (int s = validate_image(pd.right)) return s;
  if (pd.left.dtype != RSV_U8 || pd.right.dtype != RSV_U8) return RSV_E_DTYPE;
  if (pd.left.height != pd.right.height || pd.left.width != pd.right.width) return RSV_E_SHAPE;
  if (pd.left.height < K || pd.left.width < K) return RSV_E_SHAPE;
  if (pd.D < 1 || pd.D > RSV_MAX_D) return RSV_E_SHAPE;
  if (pd.left.width > 16384) return RSV_E_SHAPE;
  if (!pd.disp_sub || !pd.valid) return RSV_E_NULL;
  if (!(pd.camera.f > 0.0) || !(pd.camera.baseline > 0.0)) return RSV_E_PARAM;
  return RSV_OK;
}

}  // namespace
}  // namespace rsv

extern "C" void rsv_tuning_default(rsv_tuning* t) {
  if (!t) return;
  t->lag_bands = 1;
  t->grid_blocks = 0;
  t->reserved[0] = t->reserved[1] = 0;
}

extern "C" int rsv_batch_plan_create(const rsv_pair_desc* pairs, int32_t n, const rsv_params* p,
                                     const rsv_tuning* tuning, rsv_batch_plan** out) {
  using namespace rsv;
  if (!pairs || !p || !out) return RSV_E_NULL;
  *out = nullptr;
  if (n < 1) return RSV_E_SHAPE;
  if (int s = validate_cost_params(p)) return s;
  if (int s = validate_agg_params(p)) return s;
  if (int s = validate_select_params(p)) return s;
  const int R = p->block_radius, A = p->agg_radius, K = 2 * R + 1;
  rsv_tuning tn;
  rsv_tuning_default(&tn);
  if (tuning) tn = *tuning;
  if (tn.lag_bands < 0 || tn.lag_bands > 8 || tn.grid_blocks < 0) return RSV_E_PARAM;
  int maxD = 0;
  for (int i = 0; i < n; ++i) {
    if (int s = validate_pair(pairs[i], K)) return s;
    maxD = std::max(maxD, pairs[i].D);
  }

  // ---- sizes and the work list
  std::vector<PairDev> pd(n);
  std::vector<int4> items;
  size_t ws_bytes = 0;
  int n_counters = 0, max_pixels = 0;
  auto align = [](size_t x) { return (x + 255) & ~size_t(255); };
  std::vector<size_t> off_cref(n), off_ctar(n), off_maps(n);
  std::vector<int> off_cnt(n);
  for (int i = 0; i < n; ++i) {
    const rsv_pair_desc& q = pairs[i];
    const int H = q.left.height, W = q.left.width, D = q.D;
    const size_t N = static_cast<size_t>(H) * W;
    off_cref[i] = ws_bytes;
    ws_bytes = align(ws_bytes + sizeof(float) * N * D);
    off_ctar[i] = ws_bytes;
    ws_bytes = align(ws_bytes + sizeof(float) * N * D);
    off_maps[i] = ws_bytes;
    ws_bytes = align(ws_bytes + N * (sizeof(int32_t) * 2 + sizeof(float) * 3));
    off_cnt[i] = n_counters;
    const int nb = (H + kBandRows - 1) / kBandRows;
    n_counters += nb;
    max_pixels = std::max<int>(max_pixels, static_cast<int>(N));
    PairDev& P = pd[i];
    P.left = static_cast<const uint8_t*>(q.left.data);
    P.right = static_cast<const uint8_t*>(q.right.data);
    P.lpitch = q.left.pitch;
    P.rpitch = q.right.pitch;
    P.H = H;
    P.W = W;
    P.D = D;
    P.nbands = nb;
    P.ncol_tiles = (W + D - 1 + kCostTW - 1) / kCostTW;
    P.tiles_x = (W + 15) / 16;
    P.plane = q.plane;
    P.cam = q.camera;
    P.disp_ref = q.disp_ref;
    P.disp_tar = q.disp_tar;
    P.disp_sub = q.disp_sub;
    P.valid = q.valid;
    P.disp_final = q.disp_final;
    P.xyz = q.xyz;
    // work list: cost bands in order; an aggregation tile row follows the cost band
    // that completes its window, delayed by lag_bands bands
    const int nty = (H + 15) / 16;
    int next_row = 0;
    auto last_band = [&](int ty) { return std::min(nb - 1, (16 * ty + 15 + A) / kBandRows); };
    for (int b = 0; b < nb; ++b) {
      for (int ct = 0; ct < P.ncol_tiles; ++ct) items.push_back(make_int4(i, kItemCost, b, ct));
      while (next_row < nty && last_band(next_row) + tn.lag_bands <= b) {
        for (int tx = 0; tx < P.tiles_x; ++tx) {
          items.push_back(make_int4(i, kItemAggRef, next_row, tx));
          items.push_back(make_int4(i, kItemAggTar, next_row, tx));
        }
        ++next_row;
      }
    }
    for (; next_row < nty; ++next_row)
      for (int tx = 0; tx < P.tiles_x; ++tx) {
        items.push_back(make_int4(i, kItemAggRef, next_row, tx));
        items.push_back(make_int4(i, kItemAggTar, next_row, tx));
      }
  }

  rsv_batch_plan* plan = new (std::nothrow) rsv_batch_plan();
  if (!plan) return RSV_E_NOMEM;
  plan->n_pairs = n;
  plan->R = R;
  plan->A = A;
  plan->tuning = tn;
  plan->n_items = static_cast<int>(items.size());
  plan->n_counters = n_counters;
  plan->max_pixels = max_pixels;

  size_t off = 0;
  const size_t o_pairs = off;
  off = align(off + sizeof(PairDev) * n);
  const size_t o_items = off;
  off = align(off + sizeof(int4) * items.size());
  const size_t o_ctl = off;
  off = align(off + sizeof(int) * 2);
  const size_t o_cnt = off;
  off = align(off + sizeof(int32_t) * n_counters);
  const size_t o_ws = off;
  off += ws_bytes;
  hipError_t e = hipMalloc(&plan->dev_mem, off);
  if (e != hipSuccess) {
    set_hip_error(e);
    delete plan;
    return RSV_E_NOMEM;
  }
  unsigned char* base = static_cast<unsigned char*>(plan->dev_mem);
  plan->d_pairs = reinterpret_cast<PairDev*>(base + o_pairs);
  plan->d_items = reinterpret_cast<int4*>(base + o_items);
  plan->d_head = reinterpret_cast<int*>(base + o_ctl);
  plan->d_err = plan->d_head + 1;
  plan->d_counters = reinterpret_cast<int32_t*>(base + o_cnt);
  for (int i = 0; i < n; ++i) {
    PairDev& P = pd[i];
    const size_t N = static_cast<size_t>(P.H) * P.W;
    P.cref = reinterpret_cast<float*>(base + o_ws + off_cref[i]);
    P.ctar = reinterpret_cast<float*>(base + o_ws + off_ctar[i]);
    unsigned char* m = base + o_ws + off_maps[i];
    P.ref_arg = reinterpret_cast<int32_t*>(m);
    P.tar_arg = P.ref_arg + N;
    P.ref_best = reinterpret_cast<float*>(P.tar_arg + N);
    P.ref_am = P.ref_best + N;
    P.ref_ap = P.ref_am + N;
    P.band_done = plan->d_counters + off_cnt[i];
  }
  auto fail = [&](hipError_t err) {
    set_hip_error(err);
    rsv_batch_plan_destroy(plan);
    return RSV_E_HIP;
  };
  if ((e = hipMemcpy(plan->d_pairs, pd.data(), sizeof(PairDev) * n, hipMemcpyHostToDevice)) != hipSuccess)
    return fail(e);
  if ((e = hipMemcpy(plan->d_items, items.data(), sizeof(int4) * items.size(), hipMemcpyHostToDevice)) !=
      hipSuccess)
    return fail(e);

  const void* kern = pick_batch_kernel(R, A);
  if (!kern) {
    rsv_batch_plan_destroy(plan);
    return RSV_E_PARAM;
  }
  const size_t lds = batch_lds_bytes(R, A, maxD);
  if ((e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds))) !=
      hipSuccess)
    return fail(e);
  int dev = 0, cus = 0;
  hipGetDevice(&dev);
  hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  int per_cu = 0;
  if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, kBatchThreads, lds)) != hipSuccess)
    return fail(e);
  if (per_cu < 1) {
    rsv_batch_plan_destroy(plan);
    return RSV_E_PARAM;
  }
  plan->grid = tn.grid_blocks > 0 ? tn.grid_blocks : cus * per_cu;

  BatchArgs& a = plan->args;
  a.pairs = plan->d_pairs;
  a.items = plan->d_items;
  a.n_items = plan->n_items;
  a.head = plan->d_head;
  a.err = plan->d_err;
  a.igd2 = 1.f / (p->gamma_d * p->gamma_d);
  a.igr2 = 1.f / (p->gamma_r * p->gamma_r);
  a.sigma_min = p->sigma_min;
  a.tau = p->lr_threshold;

  // graph: reset counters -> persistent kernel -> tail
  if ((e = hipStreamCreateWithFlags(&plan->capture_stream, hipStreamNonBlocking)) != hipSuccess) return fail(e);
  if ((e = hipStreamBeginCapture(plan->capture_stream, hipStreamCaptureModeThreadLocal)) != hipSuccess)
    return fail(e);
  const int nrc = std::max(1, n_counters);
  batch_reset_kernel<<<(nrc + 255) / 256, 256, 0, plan->capture_stream>>>(plan->d_head, plan->d_err,
                                                                          plan->d_counters, n_counters);
  void* kargs[] = {&plan->args};
  hipLaunchKernel(kern, dim3(plan->grid), dim3(kBatchThreads), kargs, lds, plan->capture_stream);
  const int tail_x = std::min(1024, (max_pixels + 255) / 256);
  batch_tail_kernel<<<dim3(tail_x, n), 256, 0, plan->capture_stream>>>(plan->d_pairs, p->lr_threshold);
  hipError_t le = hipGetLastError();
  e = hipStreamEndCapture(plan->capture_stream, &plan->graph);
  if (le != hipSuccess) return fail(le);
  if (e != hipSuccess) return fail(e);
  if ((e = hipGraphInstantiate(&plan->exec, plan->graph, nullptr, nullptr, 0)) != hipSuccess) return fail(e);
  *out = plan;
  return RSV_OK;
}

extern "C" int rsv_batch_run(rsv_batch_plan* plan, void* stream) {
  using namespace rsv;
  if (!plan || !plan->exec) return RSV_E_NULL;
  hipError_t e = hipGraphLaunch(plan->exec, as_stream(stream));
  if (e != hipSuccess) {
    set_hip_error(e);
    return RSV_E_HIP;
  }
  return RSV_OK;
}

extern "C" int rsv_batch_error(rsv_batch_plan* plan, int32_t* flag) {
  using namespace rsv;
  if (!plan || !flag) return RSV_E_NULL;
  int v = 0;
  hipError_t e = hipMemcpy(&v, plan->d_err, sizeof(int), hipMemcpyDeviceToHost);
  if (e != hipSuccess) {
    set_hip_error(e);
    return RSV_E_HIP;
  }
  *flag = v;
  return RSV_OK;
}

extern "C" int rsv_batch_plan_info(const rsv_batch_plan* plan, int32_t* n_items, int32_t* grid_blocks,
                                   int64_t* workspace_bytes) {
  if (!plan) return RSV_E_NULL;
  if (n_items) *n_items = plan->n_items;
  if (grid_blocks) *grid_blocks = plan->grid;
  if (workspace_bytes) {
    size_t sz = 0;
    hipMemPtrGetInfo(plan->dev_mem, &sz);
    *workspace_bytes = static_cast<int64_t>(sz);
  }
  return RSV_OK;
}

extern "C" int rsv_batch_plan_destroy(rsv_batch_plan* plan) {
  if (!plan) return RSV_E_NULL;
  if (plan->exec) hipGraphExecDestroy(plan->exec);
  if (plan->graph) hipGraphDestroy(plan->graph);
  if (plan->capture_stream) hipStreamDestroy(plan->capture_stream);
  if (plan->dev_mem) hipFree(plan->dev_mem);
  delete plan;
  return RSV_OK;
}

extern "C" int rsv_autotune(const rsv_pair_desc* pairs, int32_t n, const rsv_params* p, rsv_tuning* out,
                            float* best_ms, void* stream) {
  using namespace rsv;
  if (!pairs || !p || !out) return RSV_E_NULL;
  hipStream_t st = as_stream(stream);
  rsv_tuning best;
  rsv_tuning_default(&best);
  float best_t = 1e30f;
  int cus = 0, dev = 0;
  hipGetDevice(&dev);
  hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  hipEvent_t e0, e1;
  hipEventCreate(&e0);
  hipEventCreate(&e1);
  int status = RSV_OK;
  const int lags[] = {0, 1, 2, 4};
  const int grids[] = {cus, 2 * cus, 4 * cus};
  for (int lag : lags)
    for (int g : grids) {
      rsv_tuning t;
      rsv_tuning_default(&t);
      t.lag_bands = lag;
      t.grid_blocks = g;
      rsv_batch_plan* plan = nullptr;
      int s = rsv_batch_plan_create(pairs, n, p, &t, &plan);
      if (s != RSV_OK) {
        status = s;
        continue;
      }
      rsv_batch_run(plan, st);  // warm-up
      hipEventRecord(e0, st);
      const int reps = 3;
      for (int r = 0; r < reps; ++r) rsv_batch_run(plan, st);
      hipEventRecord(e1, st);
      hipEventSynchronize(e1);
      float ms = 0.f;
      hipEventElapsedTime(&ms, e0, e1);
      ms /= reps;
      int32_t err = 0;
      rsv_batch_error(plan, &err);
      rsv_batch_plan_destroy(plan);
      if (!err && ms < best_t) {
        best_t = ms;
        best = t;
      }
    }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (best_t >= 1e30f) return status != RSV_OK ? status : RSV_E_HIP;
  *out = best;
  if (best_ms) *best_ms = best_t;
  return RSV_OK;
}
