// Batched form: many stereo pairs of uneven size and disparity range in one
// hipGraph launch.
//
// A plan holds, per pair, the warped right image, the joint cost volume and the
// selection maps, plus the work lists, and captures the graph
//     reset counters -> warp -> cost kernel -> [persistent aggregation kernel] ->
//     tile kernel -> tail kernel.
//   warp: every pixel of every pair, with rsv_warp's arithmetic;
//   cost items (pair, band of 4 rows, 64-centre column tiles): ZNCC with the
//       arithmetic of rsv_cost_volume_joint (shared cost_tile), persistent over a
//       work queue or one workgroup per tile;
//   target and reference tiles (rho <= 5, W >= 4): one workgroup per (pair, 16 x 16
//       tile) on the LDS-loaded tile (agg_tile_dma) reading views of the joint
//       volume, one launch, each pair's target and reference tiles side by side in
//       the list.  The target tile keeps only the argmax over d (rsv_aggregate_argmax's
//       arithmetic); the reference tile feeds each 16-disparity tile of aggregated
//       values, from LDS, through the select kernel's scan step (running best, its d
//       and its neighbours, ties keep the lowest d), with the scan state in the LDS
//       of the weight tables;
//   the persistent kernel takes the tiles the LDS-loaded tile cannot (rho = 6 or
//       W < 4), reference and target, on the register-staged tile (agg_tile), both
//       through the scan sink (a target tile through its argmax part only).  Its list is cut into 8 contiguous stretches, one queue per XCD
//       (workgroups are dealt to the XCDs round-robin), so neighbouring tiles share
//       an L2; a workgroup whose queue is empty takes items from the next queues, in
//       chunks of 4 neighbours, one atomic per chunk.  It is left out when its list
//       is empty.
// No aggregated volume is written.  The tail applies the left-right check (Eq. 11),
// the parabola (Eq. 12), post-processing and triangulation per pixel, with the plain
// path's functions.  Every output therefore equals the plain path's bit for bit.
// The kernel boundaries replace any cross-workgroup wait.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <new>
#include <vector>

#include "agg_tile.hpp"
#include "agg_tile_dma.hpp"
#include "argmax_sink.hpp"
#include "cost_box.hpp"
#include "select_math.hpp"
#include "warp_math.hpp"
#include "wta_sink.hpp"

namespace rsv {

constexpr int kAggItemThreads = 1024;
constexpr int kAggQueues = 8;  // one per XCD

enum : int { kItemCost = 0, kItemAggRef = 1, kItemAggTar = 2 };

struct PairDev {
  const uint8_t* left;
  const uint8_t* right;
  int64_t lpitch, rpitch;
  int H, W, D, nbands, ncol_tiles, tiles_x;
  rsv_plane plane;
  rsv_camera cam;
  float* warped;
  float* joint;  // joint cost volume [D][H][jrow]: C_L and C_R are its views
  int64_t jrow;
  int32_t* ref_arg;
  int32_t* tar_arg;
  int32_t* disp_ref;
  int32_t* disp_tar;
  float* disp_sub;
  uint8_t* valid;
  float* disp_final;
  float* xyz;
};

// Work queues over one item list: queue q holds items [qbeg[q], qbeg[q + 1]) and
// head[q] counts the items taken from it.
struct BatchArgs {
  const PairDev* pairs;
  const int4* items;  // {pair, kind, a, b}
  const int* qbeg;    // nq + 1 entries
  int nq;
  int* head;          // nq counters
  BilateralK bk;
  float sigma_min;
};

// Items are claimed in chunks of kChunk consecutive list entries: one atomic per
// chunk, and a chunk's items are neighbours (they share halo data in L2).
constexpr int kChunk = 4;

// First item of a chunk from queue q, or -1 when the queue is exhausted (the
// counter still advances).
__device__ __forceinline__ int take(const BatchArgs& a, int q) {
  const int it = a.qbeg[q] + kChunk * atomicAdd(&a.head[q], 1);
  return it < a.qbeg[q + 1] ? it : -1;
}

// A chunk for the workgroup: from the home queue, else from the following queues.
__device__ int claim(const BatchArgs& a, int home, int* end) {
  for (int k = 0; k < a.nq; ++k) {
    const int q = (home + k) % a.nq;
    const int it = take(a, q);
    if (it >= 0) {
      *end = min(it + kChunk, a.qbeg[q + 1]);
      return it;
    }
  }
  return -1;
}

// Runs body(item) for every item this workgroup obtains.
template <typename Body>
__device__ __forceinline__ void for_each_item(const BatchArgs& a, int home, int* slot, Body body) {
  for (;;) {
    if (threadIdx.x == 0) {
      int end = 0;
      slot[0] = claim(a, home, &end);
      slot[1] = end;
    }
    __syncthreads();
    const int first = __builtin_amdgcn_readfirstlane(slot[0]);
    const int end = __builtin_amdgcn_readfirstlane(slot[1]);
    __syncthreads();
    if (first < 0) return;
    for (int it = first; it < end; ++it) {
      body(it);
      __syncthreads();  // the item's LDS is free for the next one
    }
  }
}

// The warped right image of every pair (rsv_warp's arithmetic); grid (x, pair).
__global__ __launch_bounds__(256) void batch_warp_kernel(const PairDev* pairs) {
  const PairDev* pd = pairs + blockIdx.y;
  const int W = pd->W;
  const int64_t n = static_cast<int64_t>(pd->H) * W;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * 256) {
    const int v = static_cast<int>(i / W), u = static_cast<int>(i - static_cast<int64_t>(v) * W);
    pd->warped[i] = warp_sample(pd->right, pd->rpitch, W, pd->plane, u, v);
  }
}

// Cost item {pair, tiles << 8, band, first column tile}: `tiles` consecutive tiles of
// 64 centres x cost_tile_rows<R>() rows.
template <int R>
__device__ __forceinline__ void batch_cost_item(const BatchArgs& args, int4 w, unsigned char* cwork) {
  const PairDev* pd = uniform(args.pairs + uniform(w.x));
  const float* warped = uniform(pd->warped);
  const int W = uniform(pd->W), H = uniform(pd->H), D = uniform(pd->D);
  auto warped_at = [&](int y, int x) { return as_global(warped)[static_cast<int64_t>(y) * W + x]; };
  const int c0 = uniform(w.w);
  const int last = min(c0 + (uniform(w.y) >> 8), uniform(pd->ncol_tiles));
  const int v0 = uniform(w.z) * cost_tile_rows<R>();
  const uint8_t* left = uniform(pd->left);
  const int64_t lpitch = uniform(pd->lpitch);
  const CostOut out = cost_out_joint(uniform(pd->joint), uniform(pd->jrow), H, W, D);
  for (int ct = c0; ct < last; ++ct) {
    if (ct > c0) __syncthreads();  // LDS is reused by the next tile
    cost_tile_for<R, false>(left, lpitch, warped_at, H, W, D, args.sigma_min, ct * kCostTW, v0,
                            out, cwork);
  }
}

template <int R>
__global__ __launch_bounds__(cost_tile_threads<R>()) void batch_cost_kernel(BatchArgs args) {
  extern __shared__ __align__(16) unsigned char cwork[];
  __shared__ int s_item[2];
  for_each_item(args, 0, s_item, [&](int it) { batch_cost_item<R>(args, args.items[it], cwork); });
}

// The same work with one workgroup per cost item (no queue): without the item loop
// the kernel keeps the plain cost kernel's register budget and occupancy.
template <int R>
__global__ __launch_bounds__(cost_tile_threads<R>(), cost_uses_box<R>() ? 1 : 4) void batch_cost_grid_kernel(BatchArgs args) {
  extern __shared__ __align__(16) unsigned char cwork[];
  const int4 w = args.items[blockIdx.x];  // one tile: {pair, 1 << 8, band, column tile}
  const PairDev* pd = uniform(args.pairs + uniform(w.x));
  const float* warped = uniform(pd->warped);
  const int W = uniform(pd->W), H = uniform(pd->H), D = uniform(pd->D);
  auto warped_at = [&](int y, int x) { return as_global(warped)[static_cast<int64_t>(y) * W + x]; };
  cost_tile_for<R, false>(uniform(pd->left), uniform(pd->lpitch), warped_at, H, W, D, args.sigma_min,
                          uniform(w.w) * kCostTW, uniform(w.z) * cost_tile_rows<R>(),
                          cost_out_joint(uniform(pd->joint), uniform(pd->jrow), H, W, D), cwork);
}

// One pair's cost tiles, the pair's descriptor a kernel argument (block b: band
// b / ncol_tiles, column tile b % ncol_tiles); used by the per-pair launch schedule.
template <int R>
__global__ __launch_bounds__(cost_tile_threads<R>(), cost_uses_box<R>() ? 1 : 4) void batch_pair_cost_kernel(PairDev P, float sigma_min) {
  extern __shared__ __align__(16) unsigned char cwork[];
  const float* warped = P.warped;
  const int W = P.W;
  auto warped_at = [&](int y, int x) { return as_global(warped)[static_cast<int64_t>(y) * W + x]; };
  const int band = static_cast<int>(blockIdx.x) / P.ncol_tiles;
  const int ct = static_cast<int>(blockIdx.x) - band * P.ncol_tiles;
  cost_tile_for<R, false>(P.left, P.lpitch, warped_at, P.H, W, P.D, sigma_min, ct * kCostTW,
                                 band * cost_tile_rows<R>(), cost_out_joint(P.joint, P.jrow, P.H, W, P.D), cwork);
}

template <int A>
__device__ __noinline__ void batch_agg_item(const BatchArgs& args, int4 w, unsigned char* smem) {
  // the item and the pair's fields are the same for the whole workgroup
  const PairDev* pd = uniform(args.pairs + uniform(w.x));
  const int H = uniform(pd->H), W = uniform(pd->W), D = uniform(pd->D);
  const int by = 16 * uniform(w.z), bx = 16 * uniform(w.w);
  const bool full = uniform(w.y) == kItemAggRef;
  WtaState* st = reinterpret_cast<WtaState*>(smem + agg_tile_lds_bytes<A, 16>());
  WtaSink sink{st, D, full};
  // reference: guided by the left image; target: by the warped right image (one
  // branch per guide pixel, uniform per item)
  const uint8_t* left = uniform(pd->left);
  const float* warped = uniform(pd->warped);
  const int64_t lpitch = uniform(pd->lpitch);
  // the joint volume's reference view, or its target view (plane stride one longer)
  const float* cost = uniform(pd->joint);
  const int jrow = static_cast<int>(uniform(pd->jrow));
  const int64_t cps = static_cast<int64_t>(H) * jrow + (full ? 0 : 1);
  auto guide = [&](int Y, int X) {
    return full ? pixel(left, lpitch, Y, X) : warped[static_cast<int64_t>(Y) * W + X];
  };
  agg_tile<A, 16>(cost, cps, jrow, H, W, D, args.bk, by, bx, guide, sink, smem);
  // each thread < 256 wrote its own pixel's state in the last sink call
  if (threadIdx.x < 256) {
    const int q = threadIdx.x;
    const int Y = by + (q >> 4), X = bx + (q & 15);
    if (Y < H && X < W) {
      const int64_t i = static_cast<int64_t>(Y) * W + X;
      if (full) {  // the winner and Eq. 12 on it (the left-right check waits for the tail)
        uniform(pd->ref_arg)[i] = st->arg[q];
        uniform(pd->disp_sub)[i] = parabola(st->arg[q], st->best[q], st->am[q], st->ap[q], D);
      } else {
        uniform(pd->tar_arg)[i] = st->arg[q];
      }
    }
  }
}

template <int A>
__global__ __launch_bounds__(kAggItemThreads) void batch_agg_kernel(BatchArgs args) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int s_item[2];
  const int home = static_cast<int>(blockIdx.x % static_cast<unsigned>(args.nq));
  for_each_item(args, home, s_item, [&](int it) { batch_agg_item<A>(args, args.items[it], smem); });
}

// Target-volume tiles on the LDS-loaded tile (rho <= 5, W >= 4): only the argmax over
// d is kept, in registers (ArgmaxSink), as in rsv_aggregate_argmax.  P holds the
// pair's descriptor (wave-uniform values).
template <int A>
__device__ __forceinline__ void batch_tar_tile(const PairDev& P, const BilateralK& bk, int by, int bx,
                                               unsigned char* smem) {
  const int H = P.H, W = P.W, D = P.D;
  const float* warped = P.warped;
  const int jrow = static_cast<int>(P.jrow);
  auto guide = [&](int Y, int X) { return as_global(warped)[static_cast<int64_t>(Y) * W + X]; };
  ArgmaxSink sink{D};
  agg_tile_dma<A>(P.joint, static_cast<int64_t>(H) * jrow + 1, jrow, H, W, D, bk, by, bx, guide, sink, smem,
                  lds_address(smem));
  sink.finish(P.tar_arg, H, W, by, bx);
}

// Reference-volume tiles on the LDS-loaded tile (rho <= 5, W >= 4): the select
// kernel's scan result from all 1024 threads (RefQuadSink).
template <int A>
__device__ __forceinline__ void batch_ref_tile(const PairDev& P, const BilateralK& bk, int by, int bx,
                                               unsigned char* smem) {
  const int H = P.H, W = P.W, D = P.D;
  const uint8_t* left = P.left;
  const int64_t lpitch = P.lpitch;
  const int jrow = static_cast<int>(P.jrow);
  auto guide = [&](int Y, int X) { return pixel(left, lpitch, Y, X); };
  RefQuadSink sink{D};
  agg_tile_dma<A>(P.joint, static_cast<int64_t>(H) * jrow, jrow, H, W, D, bk, by, bx, guide, sink, smem,
                  lds_address(smem));
  if ((threadIdx.x & 3) == 0) {  // the four lanes of a pixel hold the same result
    const int q = threadIdx.x >> 2;
    const int Y = by + (q >> 4), X = bx + (q & 15);
    if (Y < H && X < W) {
      const int64_t i = static_cast<int64_t>(Y) * W + X;
      P.ref_arg[i] = sink.arg;  // the winner and Eq. 12 on it
      P.disp_sub[i] = parabola(sink.arg, sink.best, sink.am, sink.ap, D);
    }
  }
}

// The pair descriptor of an item, read into wave-uniform registers.
__device__ __forceinline__ PairDev load_pair(const PairDev* pd) {
  PairDev P;
  P.left = uniform(pd->left);
  P.lpitch = uniform(pd->lpitch);
  P.H = uniform(pd->H);
  P.W = uniform(pd->W);
  P.D = uniform(pd->D);
  P.warped = uniform(pd->warped);
  P.joint = uniform(pd->joint);
  P.jrow = uniform(pd->jrow);
  P.ref_arg = uniform(pd->ref_arg);
  P.tar_arg = uniform(pd->tar_arg);
  P.disp_sub = uniform(pd->disp_sub);
  return P;
}

// The tile items {pair, kind, tile row, tile column} of the LDS-loaded tile, one
// workgroup per item, target or reference by the item's kind (uniform per workgroup).
// The list holds each pair's target tiles next to its reference tiles, so both passes
// over a pair's joint cost volume run close together in time.  A kernel of its own
// (no item loop), so the tile keeps a kernel's register budget.
template <int A>
__global__ __launch_bounds__(1024) void batch_tile_kernel(BatchArgs args) {
  extern __shared__ __align__(16) unsigned char smem[];
  // each XCD takes runs of 8 neighbouring tiles (they share halos in its L2), all XCDs
  // near the same stretch of the list (one pair's volume in the shared cache)
  const int4 w = args.items[xcd_run_item<8>(blockIdx.x, gridDim.x)];
  const PairDev P = load_pair(args.pairs + uniform(w.x));
  const int by = 16 * uniform(w.z), bx = 16 * uniform(w.w);
  if (uniform(w.y) == kItemAggRef)
    batch_ref_tile<A>(P, args.bk, by, bx, smem);
  else
    batch_tar_tile<A>(P, args.bk, by, bx, smem);
}

// One pair's tiles of both views, the pair's descriptor a kernel argument: no item
// list and no descriptor load before the tile's first loads.  Tiles in the order of
// rsv_aggregate_views (a tile row of reference tiles, then of target tiles), XCDs in
// runs of 80.  Used by the per-pair launch schedule.
template <int A>
__global__ __launch_bounds__(1024) void batch_pair_tile_kernel(PairDev P, BilateralK bk) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int tiles_x = (P.W + 15) >> 4, tiles_y = (P.H + 15) >> 4;
  const int k = xcd_run_item<80>(blockIdx.x, 2 * tiles_x * tiles_y);
  const int ty = k / (2 * tiles_x), r = k - ty * 2 * tiles_x;
  if (r < tiles_x)
    batch_ref_tile<A>(P, bk, 16 * ty, 16 * r, smem);
  else
    batch_tar_tile<A>(P, bk, 16 * ty, 16 * (r - tiles_x), smem);
}

// Left-right check, post-processing and 3-D points for every pixel of every pair (the
// reference tiles wrote the winner and its Eq. 12 refinement).
__global__ __launch_bounds__(256) void batch_tail_kernel(const PairDev* pairs, int tau) {
  const PairDev P = pairs[blockIdx.y];
  const int64_t n = static_cast<int64_t>(P.H) * P.W;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * 256) {
    const int v = static_cast<int>(i / P.W), u = static_cast<int>(i - static_cast<int64_t>(v) * P.W);
    const int arg = P.ref_arg[i];
    const int x = u - arg;
    const bool ok = (x >= 0) && (abs(arg - P.tar_arg[static_cast<int64_t>(v) * P.W + (x < 0 ? 0 : x)]) <= tau);
    const float ds = P.disp_sub[i];
    if (P.disp_ref) P.disp_ref[i] = arg;
    if (P.disp_tar) P.disp_tar[i] = P.tar_arg[i];
    P.valid[i] = ok ? 1 : 0;
    postprocess_point(ds, ok, u, v, P.plane, P.cam, P.disp_final ? P.disp_final + i : nullptr,
                      P.xyz ? P.xyz + 3 * i : nullptr);
  }
}

__global__ void batch_reset_kernel(int* heads, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) heads[i] = 0;
}

}  // namespace rsv

// ------------------------------------------------------------------ host side
// Default device memory for cost volumes.  On the 64-pair mixed batch (pairs up to
// 1920x1080 with D = 128, 1.1 GB of volume) groups of at most 1 GiB, i.e. mostly one
// pair, ran 46.5 ms against 47.9 ms with every volume resident (21.9 GiB): the next
// group's cost volumes are computed while the current one is aggregated, and each
// group's volumes are read back soon after they are written.
constexpr int32_t kDefaultVolumeBudgetMiB = 2048;

struct rsv_batch_plan {
  int n_pairs = 0;
  rsv_tuning tuning{};
  void* dev_mem = nullptr;  // one allocation: pair table, item lists, counters, workspace
  rsv::PairDev* d_pairs = nullptr;
  int* d_heads = nullptr;   // per group: [cost, aggregation queues]
  // agg: items of the persistent aggregation kernel; tar / ref: of the tile kernels
  int n_cost_items = 0, n_agg_items = 0, n_tile_items = 0;
  int n_groups = 1;
  int cost_grid = 0, agg_grid = 0;  // largest launch of a group
  hipStream_t capture_stream = nullptr, capture_stream2 = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace rsv {
namespace {

template <int R>
const void* pair_cost_kernel_ptr() {
  return reinterpret_cast<const void*>(batch_pair_cost_kernel<R>);
}

template <int R>
const void* cost_kernel_ptr(bool grid) {
  return grid ? reinterpret_cast<const void*>(batch_cost_grid_kernel<R>)
              : reinterpret_cast<const void*>(batch_cost_kernel<R>);
}
template <int A>
const void* agg_kernel_ptr() {
  return reinterpret_cast<const void*>(batch_agg_kernel<A>);
}

const void* pick_cost_kernel(int R, bool grid) {
  switch (R) {
    case 1: return cost_kernel_ptr<1>(grid);
    case 2: return cost_kernel_ptr<2>(grid);
    case 3: return cost_kernel_ptr<3>(grid);
    case 4: return cost_kernel_ptr<4>(grid);
    default: return nullptr;
  }
}

const void* pick_pair_cost_kernel(int R) {
  switch (R) {
    case 1: return pair_cost_kernel_ptr<1>();
    case 2: return pair_cost_kernel_ptr<2>();
    case 3: return pair_cost_kernel_ptr<3>();
    case 4: return pair_cost_kernel_ptr<4>();
    default: return nullptr;
  }
}

const void* pick_agg_kernel(int A, size_t* lds) {
  switch (A) {
    case 1: *lds = agg_tile_lds_bytes<1, 16>() + sizeof(WtaState); return agg_kernel_ptr<1>();
    case 2: *lds = agg_tile_lds_bytes<2, 16>() + sizeof(WtaState); return agg_kernel_ptr<2>();
    case 3: *lds = agg_tile_lds_bytes<3, 16>() + sizeof(WtaState); return agg_kernel_ptr<3>();
    case 4: *lds = agg_tile_lds_bytes<4, 16>() + sizeof(WtaState); return agg_kernel_ptr<4>();
    case 5: *lds = agg_tile_lds_bytes<5, 16>() + sizeof(WtaState); return agg_kernel_ptr<5>();
    case 6: *lds = agg_tile_lds_bytes<6, 16>() + sizeof(WtaState); return agg_kernel_ptr<6>();
    default: return nullptr;
  }
}

// The tile kernel for radius A (null when the LDS-loaded tile does not fit: rho = 6),
// with its LDS bytes.
template <int A>
const void* tile_kernel_ptr(size_t* lds) {
  if constexpr (agg_dma_fits<A>()) {
    *lds = agg_tile_dma_lds_bytes<A>();
    return reinterpret_cast<const void*>(batch_tile_kernel<A>);
  } else {
    return nullptr;
  }
}

template <int A>
const void* pair_tile_kernel_ptr() {
  if constexpr (agg_dma_fits<A>())
    return reinterpret_cast<const void*>(batch_pair_tile_kernel<A>);
  else
    return nullptr;
}

const void* pick_pair_tile_kernel(int A) {
  switch (A) {
    case 1: return pair_tile_kernel_ptr<1>();
    case 2: return pair_tile_kernel_ptr<2>();
    case 3: return pair_tile_kernel_ptr<3>();
    case 4: return pair_tile_kernel_ptr<4>();
    case 5: return pair_tile_kernel_ptr<5>();
    default: return nullptr;
  }
}

const void* pick_tile_kernel(int A, size_t* lds) {
  switch (A) {
    case 1: return tile_kernel_ptr<1>(lds);
    case 2: return tile_kernel_ptr<2>(lds);
    case 3: return tile_kernel_ptr<3>(lds);
    case 4: return tile_kernel_ptr<4>(lds);
    case 5: return tile_kernel_ptr<5>(lds);
    case 6: return tile_kernel_ptr<6>(lds);
    default: return nullptr;
  }
}

int validate_pair(const rsv_pair_desc& pd, int K) {
  if (int s = validate_image(pd.left)) return s;
  if (int s = validate_image(pd.right)) return s;
  if (pd.left.dtype != RSV_U8 || pd.right.dtype != RSV_U8) return RSV_E_DTYPE;
  if (pd.left.height != pd.right.height || pd.left.width != pd.right.width) return RSV_E_SHAPE;
  if (pd.left.height < K || pd.left.width < K) return RSV_E_SHAPE;
  if (pd.D < 1 || pd.D > RSV_MAX_D) return RSV_E_SHAPE;
  // the joint cost volume's target view: plane stride H * row stride + 1 (32-bit tile offsets)
  if (pd.left.height * joint_row_stride(pd.left.width, pd.D) + 1 > kAggMaxPixels) return RSV_E_SHAPE;
  if (!pd.disp_sub || !pd.valid) return RSV_E_NULL;
  if (!(pd.camera.f > 0.0) || !(pd.camera.baseline > 0.0)) return RSV_E_PARAM;
  return RSV_OK;
}

}  // namespace
}  // namespace rsv

extern "C" void rsv_tuning_default(rsv_tuning* t) {
  if (!t) return;
  t->largest_first = 1;
  t->cost_tiles_per_item = 2;
  t->cost_blocks_per_cu = 0;
  t->agg_blocks_per_cu = 0;
  t->per_pair_launches = 1;
  t->volume_budget_mib = kDefaultVolumeBudgetMiB;
}

extern "C" int rsv_batch_plan_create(const rsv_pair_desc* pairs, int32_t n, const rsv_params* p,
                                     const rsv_tuning* tuning, rsv_batch_plan** out) {
  using namespace rsv;
  if (!pairs || !p || !out) return RSV_E_NULL;
  *out = nullptr;
  if (n < 1) return RSV_E_SHAPE;
  rsv_params pc = *p;  // D comes from each pair; validate the shared parameters only
  pc.D = 1;
  if (int s = validate_cost_params(&pc)) return s;
  if (int s = validate_agg_params(&pc)) return s;
  if (int s = validate_select_params(&pc)) return s;
  const int R = p->block_radius, A = p->agg_radius, K = 2 * R + 1;
  rsv_tuning tn;
  rsv_tuning_default(&tn);
  if (tuning) tn = *tuning;
  if (tn.cost_tiles_per_item < 1 || tn.cost_tiles_per_item > 16 || tn.cost_blocks_per_cu < -1 ||
      tn.agg_blocks_per_cu < 0 || tn.volume_budget_mib < 0)
    return RSV_E_PARAM;
  int maxD = 0;
  for (int i = 0; i < n; ++i) {
    if (int s = validate_pair(pairs[i], K)) return s;
    maxD = std::max(maxD, pairs[i].D);
  }

  // pair order: as given, or largest W*H*D first (the big pairs do not end the queue)
  std::vector<int> order(n);
  for (int i = 0; i < n; ++i) order[i] = i;
  if (tn.largest_first)
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
      const double wa = double(pairs[a].left.width) * pairs[a].left.height * pairs[a].D;
      const double wb = double(pairs[b].left.width) * pairs[b].left.height * pairs[b].D;
      return wa > wb;
    });

  std::vector<PairDev> pd(n);
  std::vector<int4> cost_items, agg_items, tile_items;
  size_t tile_lds = 0;
  const void* tk = pick_tile_kernel(A, &tile_lds);
  int max_pixels = 0;
  auto align = [](size_t x) { return (x + 255) & ~size_t(255); };
  std::vector<size_t> off_joint(n), off_maps(n), vol(n);
  std::vector<int64_t> jrows(n);
  for (int i = 0; i < n; ++i) {
    const rsv_pair_desc& q = pairs[i];
    jrows[i] = joint_row_stride(q.left.width, q.D);
    vol[i] = align(sizeof(float) * static_cast<size_t>(q.D) * q.left.height * jrows[i]);
  }
  // Groups of consecutive pairs (in list order) whose joint volumes are resident
  // together: one group without a budget; with one, groups of at most half the
  // budget (at least one pair each) alternating between two slots, so that group
  // g + 1's cost volumes are computed while group g is aggregated.
  const size_t budget = static_cast<size_t>(tn.volume_budget_mib) << 20;
  std::vector<int> group_first{0};  // list positions where groups start
  std::vector<size_t> in_group(n);  // volume offset of list position k inside its group
  size_t slot_bytes = 0, cur = 0;
  for (int k = 0; k < n; ++k) {
    const size_t v = vol[order[k]];
    if (budget && k > group_first.back() && cur + v > budget / 2) {
      group_first.push_back(k);
      cur = 0;
    }
    in_group[k] = cur;
    cur += v;
    slot_bytes = std::max(slot_bytes, cur);
  }
  const int n_groups = static_cast<int>(group_first.size());
  group_first.push_back(n);
  const int n_slots = n_groups > 1 ? 2 : 1;
  size_t ws_bytes = slot_bytes * n_slots;
  for (int g = 0; g < n_groups; ++g)
    for (int k = group_first[g]; k < group_first[g + 1]; ++k)
      off_joint[order[k]] = slot_bytes * (g % n_slots) + in_group[k];
  for (int i = 0; i < n; ++i) {
    const rsv_pair_desc& q = pairs[i];
    const int H = q.left.height, W = q.left.width, D = q.D;
    const size_t N = static_cast<size_t>(H) * W;
    off_maps[i] = ws_bytes;
    ws_bytes = align(ws_bytes + N * (sizeof(int32_t) * 2 + sizeof(float)));  // winners, warped image
    max_pixels = std::max<int>(max_pixels, static_cast<int>(N));
    PairDev& P = pd[i];
    P.left = static_cast<const uint8_t*>(q.left.data);
    P.right = static_cast<const uint8_t*>(q.right.data);
    P.lpitch = q.left.pitch;
    P.rpitch = q.right.pitch;
    P.H = H;
    P.W = W;
    P.D = D;
    P.nbands = (H + cost_tile_rows_rt(R) - 1) / cost_tile_rows_rt(R);
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
  }
  // agg items: per pair, row by row of tiles, the reference tiles then the target
  // tiles of the row, so both views' reads of the same rows of a pair's joint volume
  // come close together (49.9 instead of 50.9 ms per 64-pair batch with one view after
  // the other); one tile per cost item when the cost kernel runs one workgroup per item
  const bool grid_cost = tn.cost_blocks_per_cu < 0 || tn.per_pair_launches != 0;
  const int cost_tiles = grid_cost ? 1 : tn.cost_tiles_per_item;
  // per pair (in list order): its ranges of the cost and tile lists
  std::vector<int> cost_beg, cost_end, tile_beg, tile_end, agg_end;
  for (int i : order) {
    const PairDev& P = pd[i];
    cost_beg.push_back(static_cast<int>(cost_items.size()));
    tile_beg.push_back(static_cast<int>(tile_items.size()));
    for (int b = 0; b < P.nbands; ++b)
      for (int ct = 0; ct < P.ncol_tiles; ct += cost_tiles)
        cost_items.push_back(make_int4(i, kItemCost | (cost_tiles << 8), b, ct));
    for (int ty = 0; ty < (P.H + 15) / 16; ++ty)
      for (int kind : {kItemAggRef, kItemAggTar})
        for (int tx = 0; tx < P.tiles_x; ++tx) {
          // tiles go to the tile kernels when the LDS-loaded tile applies, else to the
          // persistent kernel
          const int4 it = make_int4(i, kind, ty, tx);
          if (tk && P.W >= 4)
            tile_items.push_back(it);
          else
            agg_items.push_back(it);
        }
    cost_end.push_back(static_cast<int>(cost_items.size()));
    tile_end.push_back(static_cast<int>(tile_items.size()));
    agg_end.push_back(static_cast<int>(agg_items.size()));
  }
  // per group: its ranges of the three lists, queue boundaries ([cost begin, cost end);
  // 8 equal stretches of its agg items) and queue counters
  constexpr int kQB = 2 + kAggQueues + 1, kHB = 1 + kAggQueues;
  std::vector<int> qbeg(static_cast<size_t>(kQB) * n_groups);
  std::vector<int> g_cost(n_groups + 1), g_tile(n_groups + 1), g_agg(n_groups + 1);
  for (int g = 0; g <= n_groups; ++g) {
    const int k = group_first[g];
    g_cost[g] = k < n ? cost_beg[k] : static_cast<int>(cost_items.size());
    g_tile[g] = k < n ? tile_beg[k] : static_cast<int>(tile_items.size());
    g_agg[g] = k == 0 ? 0 : agg_end[k - 1];
  }
  for (int g = 0; g < n_groups; ++g) {
    int* qb = qbeg.data() + static_cast<size_t>(kQB) * g;
    qb[0] = g_cost[g];
    qb[1] = g_cost[g + 1];
    const int na = g_agg[g + 1] - g_agg[g];
    for (int q = 0; q <= kAggQueues; ++q)
      qb[2 + q] = g_agg[g] + static_cast<int>((static_cast<int64_t>(na) * q) / kAggQueues);
  }

  rsv_batch_plan* plan = new (std::nothrow) rsv_batch_plan();
  if (!plan) return RSV_E_NOMEM;
  plan->n_pairs = n;
  plan->tuning = tn;
  plan->n_cost_items = static_cast<int>(cost_items.size());
  plan->n_agg_items = static_cast<int>(agg_items.size());
  plan->n_tile_items = static_cast<int>(tile_items.size());

  size_t off = 0;
  const size_t o_pairs = off;
  off = align(off + sizeof(PairDev) * n);
  const size_t o_ci = off;
  off = align(off + sizeof(int4) * cost_items.size());
  const size_t o_ai = off;
  off = align(off + sizeof(int4) * agg_items.size());
  const size_t o_ti = off;
  off = align(off + sizeof(int4) * tile_items.size());
  const size_t o_heads = off;
  off = align(off + sizeof(int) * kHB * n_groups);
  const size_t o_qbeg = off;
  off = align(off + sizeof(int) * qbeg.size());
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
  plan->d_heads = reinterpret_cast<int*>(base + o_heads);
  for (int i = 0; i < n; ++i) {
    PairDev& P = pd[i];
    const size_t N = static_cast<size_t>(P.H) * P.W;
    P.joint = reinterpret_cast<float*>(base + o_ws + off_joint[i]);
    P.jrow = jrows[i];
    unsigned char* m = base + o_ws + off_maps[i];
    P.ref_arg = reinterpret_cast<int32_t*>(m);
    P.tar_arg = P.ref_arg + N;
    P.warped = reinterpret_cast<float*>(P.tar_arg + N);
  }
  auto fail = [&](hipError_t err) {
    set_hip_error(err);
    rsv_batch_plan_destroy(plan);
    return RSV_E_HIP;
  };
  if ((e = hipMemcpy(plan->d_pairs, pd.data(), sizeof(PairDev) * n, hipMemcpyHostToDevice)) != hipSuccess)
    return fail(e);
  if ((e = hipMemcpy(base + o_ci, cost_items.data(), sizeof(int4) * cost_items.size(),
                     hipMemcpyHostToDevice)) != hipSuccess)
    return fail(e);
  if (!tile_items.empty() && (e = hipMemcpy(base + o_ti, tile_items.data(), sizeof(int4) * tile_items.size(),
                                             hipMemcpyHostToDevice)) != hipSuccess)
    return fail(e);
  if ((e = hipMemcpy(base + o_ai, agg_items.data(), sizeof(int4) * agg_items.size(),
                     hipMemcpyHostToDevice)) != hipSuccess)
    return fail(e);
  if ((e = hipMemcpy(base + o_qbeg, qbeg.data(), sizeof(int) * qbeg.size(), hipMemcpyHostToDevice)) !=
      hipSuccess)
    return fail(e);

  const bool cost_grid_mode = grid_cost;
  const void* ck = pick_cost_kernel(R, cost_grid_mode);
  size_t agg_lds = 0;
  const void* ak = pick_agg_kernel(A, &agg_lds);
  if (!ck || !ak) {
    rsv_batch_plan_destroy(plan);
    return RSV_E_PARAM;
  }
  const size_t cost_lds = cost_tile_lds(R, maxD);
  if ((e = hipFuncSetAttribute(ck, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(cost_lds))) !=
      hipSuccess)
    return fail(e);
  const void* pck = pick_pair_cost_kernel(R);  // non-null: R was validated above
  if ((e = hipFuncSetAttribute(pck, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(cost_lds))) !=
      hipSuccess)
    return fail(e);
  if (tk && (e = hipFuncSetAttribute(tk, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    static_cast<int>(tile_lds))) != hipSuccess)
    return fail(e);
  const void* ptk = pick_pair_tile_kernel(A);
  if (ptk && (e = hipFuncSetAttribute(ptk, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     static_cast<int>(tile_lds))) != hipSuccess)
    return fail(e);
  if ((e = hipFuncSetAttribute(ak, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(agg_lds))) !=
      hipSuccess)
    return fail(e);
  int dev = 0, cus = 0, cost_fit = 0, agg_fit = 0;
  if ((e = hipGetDevice(&dev)) != hipSuccess) return fail(e);
  if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return fail(e);
  if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&cost_fit, ck, cost_tile_threads_rt(R), cost_lds)) != hipSuccess)
    return fail(e);
  if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&agg_fit, ak, kAggItemThreads, agg_lds)) != hipSuccess)
    return fail(e);
  if (cost_fit < 1 || agg_fit < 1) {
    rsv_batch_plan_destroy(plan);
    return RSV_E_PARAM;
  }
  const int cpc = tn.cost_blocks_per_cu > 0 ? std::min(tn.cost_blocks_per_cu, cost_fit) : cost_fit;
  const int apc = tn.agg_blocks_per_cu > 0 ? std::min(tn.agg_blocks_per_cu, agg_fit) : agg_fit;
  // launch sizes of one group's cost and persistent aggregation kernels
  auto cost_blocks = [&](int g) {
    const int items = g_cost[g + 1] - g_cost[g];
    return cost_grid_mode ? items : std::min(cus * cpc, items);
  };
  auto agg_blocks = [&](int g) { return std::min(cus * apc, g_agg[g + 1] - g_agg[g]); };
  plan->n_groups = n_groups;
  plan->cost_grid = 0;
  plan->agg_grid = 0;
  for (int g = 0; g < n_groups; ++g) {
    plan->cost_grid = std::max(plan->cost_grid, cost_blocks(g));
    plan->agg_grid = std::max(plan->agg_grid, agg_blocks(g));
  }

  const int* d_qbeg = reinterpret_cast<const int*>(base + o_qbeg);
  BatchArgs ca{};
  ca.pairs = plan->d_pairs;
  ca.items = reinterpret_cast<const int4*>(base + o_ci);
  ca.nq = 1;
  ca.sigma_min = p->sigma_min;
  ca.bk = bilateral_constants(p->gamma_d, p->gamma_r);
  BatchArgs aa = ca;
  aa.items = reinterpret_cast<const int4*>(base + o_ai);
  aa.nq = kAggQueues;
  BatchArgs ta = ca;
  ta.items = reinterpret_cast<const int4*>(base + o_ti);

  // graph: reset counters -> warp -> per group: cost kernel -> [persistent aggregation
  // kernel] -> tile kernel -> tail.  Groups alternate between two streams (two volume
  // slots): group g + 1's launches may run beside group g's, group g + 2's follow
  // group g's on the same stream, which frees the slot they share.
  if ((e = hipStreamCreateWithFlags(&plan->capture_stream, hipStreamNonBlocking)) != hipSuccess) return fail(e);
  if (n_groups > 1) {
    if ((e = hipStreamCreateWithFlags(&plan->capture_stream2, hipStreamNonBlocking)) != hipSuccess) return fail(e);
    if ((e = hipEventCreateWithFlags(&plan->fork, hipEventDisableTiming)) != hipSuccess) return fail(e);
    if ((e = hipEventCreateWithFlags(&plan->join, hipEventDisableTiming)) != hipSuccess) return fail(e);
  }
  if ((e = hipStreamBeginCapture(plan->capture_stream, hipStreamCaptureModeThreadLocal)) != hipSuccess)
    return fail(e);
  hipError_t cap = hipSuccess;  // first failure while capturing; the capture is ended either way
  auto note = [&](hipError_t r) {
    if (r != hipSuccess && cap == hipSuccess) cap = r;
  };
  batch_reset_kernel<<<1, 256, 0, plan->capture_stream>>>(plan->d_heads, kHB * n_groups);
  const int tail_x = std::min(1024, (max_pixels + 255) / 256);
  batch_warp_kernel<<<dim3(tail_x, n), 256, 0, plan->capture_stream>>>(plan->d_pairs);
  note(hipGetLastError());
  if (n_groups > 1) {
    note(hipEventRecord(plan->fork, plan->capture_stream));
    note(hipStreamWaitEvent(plan->capture_stream2, plan->fork, 0));
  }
  for (int g = 0; g < n_groups; ++g) {
    hipStream_t gs = (g & 1) ? plan->capture_stream2 : plan->capture_stream;
    BatchArgs c = ca, a = aa;
    c.qbeg = d_qbeg + static_cast<size_t>(kQB) * g;
    c.head = plan->d_heads + static_cast<size_t>(kHB) * g;
    a.qbeg = c.qbeg + 2;
    a.head = c.head + 1;
    if (tn.per_pair_launches) {
      // pair after pair: its cost items, then its tiles, each launch over its own range
      // of the lists (one workgroup per item); the persistent kernel's tiles after them
      for (int k = group_first[g]; k < group_first[g + 1]; ++k) {
        PairDev Pc = pd[order[k]];
        float sm = p->sigma_min;
        void* cargs[] = {&Pc, &sm};
        note(hipLaunchKernel(pck, dim3(Pc.nbands * Pc.ncol_tiles), dim3(cost_tile_threads_rt(R)), cargs, cost_lds, gs));
        if (tile_end[k] > tile_beg[k]) {  // all of the pair's tiles, both views
          PairDev P = pd[order[k]];
          BilateralK bk = ca.bk;
          void* pargs[] = {&P, &bk};
          note(hipLaunchKernel(ptk, dim3(tile_end[k] - tile_beg[k]), dim3(1024), pargs, tile_lds, gs));
        }
      }
      if (agg_blocks(g) > 0) {
        void* aargs[] = {&a};
        note(hipLaunchKernel(ak, dim3(agg_blocks(g)), dim3(kAggItemThreads), aargs, agg_lds, gs));
      }
    } else {
      if (cost_grid_mode) c.items += g_cost[g];  // one workgroup per item of the group
      void* cargs[] = {&c};
      if (cost_blocks(g) > 0)
        note(hipLaunchKernel(ck, dim3(cost_blocks(g)), dim3(cost_tile_threads_rt(R)), cargs, cost_lds, gs));
      if (agg_blocks(g) > 0) {
        void* aargs[] = {&a};
        note(hipLaunchKernel(ak, dim3(agg_blocks(g)), dim3(kAggItemThreads), aargs, agg_lds, gs));
      }
      if (g_tile[g + 1] > g_tile[g]) {
        BatchArgs t = ta;
        t.items += g_tile[g];
        void* targs[] = {&t};
        note(hipLaunchKernel(tk, dim3(g_tile[g + 1] - g_tile[g]), dim3(1024), targs, tile_lds, gs));
      }
    }
  }
  if (n_groups > 1) {
    note(hipEventRecord(plan->join, plan->capture_stream2));
    note(hipStreamWaitEvent(plan->capture_stream, plan->join, 0));
  }
  batch_tail_kernel<<<dim3(tail_x, n), 256, 0, plan->capture_stream>>>(plan->d_pairs, p->lr_threshold);
  note(hipGetLastError());
  e = hipStreamEndCapture(plan->capture_stream, &plan->graph);
  if (cap != hipSuccess) return fail(cap);
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

extern "C" int rsv_batch_plan_info(const rsv_batch_plan* plan, int32_t* n_items, int32_t* grid_blocks,
                                   int64_t* workspace_bytes) {
  if (!plan) return RSV_E_NULL;
  if (n_items) {
    n_items[0] = plan->n_cost_items;
    n_items[1] = plan->n_agg_items + plan->n_tile_items;
  }
  if (grid_blocks) {
    grid_blocks[0] = plan->cost_grid;
    grid_blocks[1] = plan->agg_grid;
  }
  if (workspace_bytes) {
    size_t sz = 0;
    if (hipMemPtrGetInfo(plan->dev_mem, &sz) != hipSuccess) sz = 0;
    *workspace_bytes = static_cast<int64_t>(sz);
  }
  return RSV_OK;
}

extern "C" int rsv_batch_plan_destroy(rsv_batch_plan* plan) {
  if (!plan) return RSV_E_NULL;
  // teardown: failures here leave nothing to undo
  if (plan->exec) (void)hipGraphExecDestroy(plan->exec);
  if (plan->graph) (void)hipGraphDestroy(plan->graph);
  if (plan->capture_stream) (void)hipStreamDestroy(plan->capture_stream);
  if (plan->capture_stream2) (void)hipStreamDestroy(plan->capture_stream2);
  if (plan->fork) (void)hipEventDestroy(plan->fork);
  if (plan->join) (void)hipEventDestroy(plan->join);
  if (plan->dev_mem) (void)hipFree(plan->dev_mem);
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
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return RSV_E_HIP;
  int status = RSV_OK;
  // mean time of 3 runs after a warm-up, or 1e30 if the plan cannot be built
  auto time_plan = [&](const rsv_tuning& t) {
    rsv_batch_plan* plan = nullptr;
    const int s = rsv_batch_plan_create(pairs, n, p, &t, &plan);
    if (s != RSV_OK) {
      status = s;
      return 1e30f;
    }
    const int reps = 3;
    int run = rsv_batch_run(plan, st);  // warm-up
    float ms = 0.f;
    bool ok = run == RSV_OK && hipEventRecord(e0, st) == hipSuccess;
    for (int r = 0; ok && r < reps; ++r) ok = rsv_batch_run(plan, st) == RSV_OK;
    ok = ok && hipEventRecord(e1, st) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
         hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
    rsv_batch_plan_destroy(plan);
    if (!ok) {
      status = RSV_E_HIP;
      return 1e30f;
    }
    return ms / reps;
  };
  for (int lf = 0; lf <= 1; ++lf)
    for (int tiles : {1, 2, 4})
      for (int cpc : {-1, 0, 2})
        for (int pp : {0, 1}) {
        if (cpc < 0 && tiles != 1) continue;  // one tile per item there
        if (pp && cpc >= 0) continue;         // per-pair launches run one workgroup per cost item
        rsv_tuning t;
        rsv_tuning_default(&t);
        t.largest_first = lf;
        t.cost_tiles_per_item = tiles;
        t.cost_blocks_per_cu = cpc;
        t.per_pair_launches = pp;
        const float ms = time_plan(t);
        if (ms < best_t) {
          best_t = ms;
          best = t;
        }
      }
  // then the volume budget, on the fastest launch shape
  if (best_t < 1e30f) {
    const rsv_tuning shape = best;
    for (int mib : {0, 512, 4096}) {
      rsv_tuning t = shape;
      t.volume_budget_mib = mib;
      const float ms = time_plan(t);
      if (ms < best_t) {
        best_t = ms;
        best = t;
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (best_t >= 1e30f) return status != RSV_OK ? status : RSV_E_HIP;
  *out = best;
  if (best_ms) *best_ms = best_t;
  return RSV_OK;
}
