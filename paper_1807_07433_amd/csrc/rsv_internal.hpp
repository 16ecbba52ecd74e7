// Internal helpers shared by the HIP translation units of librsv.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rsv.h"

namespace rsv {

// ------------------------------------------------------------------ host side
void set_hip_error(hipError_t e);

// Records the launch status of the last kernel; returns RSV_OK or RSV_E_HIP.
inline int check_launch() {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_hip_error(e);
    return RSV_E_HIP;
  }
  return RSV_OK;
}

inline bool aligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

inline int validate_image(const rsv_image& im) {
  if (!im.data) return RSV_E_NULL;
  if (im.dtype != RSV_U8 && im.dtype != RSV_F32) return RSV_E_DTYPE;
  if (im.height < 1 || im.width < 1 || im.pitch < im.width) return RSV_E_SHAPE;
  // pixel indices within one plane are 32-bit in the kernels
  if (static_cast<int64_t>(im.height) * im.width > INT32_MAX) return RSV_E_SHAPE;
  if (im.dtype == RSV_F32 && !aligned(im.data, 4)) return RSV_E_ALIGN;
  return RSV_OK;
}

inline int validate_d(const rsv_params* p) {
  if (!p) return RSV_E_NULL;
  if (p->D < 1 || p->D > RSV_MAX_D) return RSV_E_SHAPE;
  return RSV_OK;
}

inline int validate_cost_params(const rsv_params* p) {
  if (int s = validate_d(p)) return s;
  if (p->block_radius < RSV_MIN_BLOCK_RADIUS || p->block_radius > RSV_MAX_BLOCK_RADIUS)
    return RSV_E_PARAM;
  if (!(p->sigma_min >= 0.f)) return RSV_E_PARAM;
  return RSV_OK;
}

inline int validate_agg_params(const rsv_params* p) {
  if (int s = validate_d(p)) return s;
  if (p->agg_radius < RSV_MIN_AGG_RADIUS || p->agg_radius > RSV_MAX_AGG_RADIUS) return RSV_E_PARAM;
  if (!(p->gamma_d > 0.f) || !(p->gamma_r > 0.f)) return RSV_E_PARAM;
  return RSV_OK;
}

inline int validate_select_params(const rsv_params* p) {
  if (int s = validate_d(p)) return s;
  if (p->lr_threshold < 0) return RSV_E_PARAM;
  return RSV_OK;
}

inline int validate_all_params(const rsv_params* p) {
  if (int s = validate_cost_params(p)) return s;
  if (int s = validate_agg_params(p)) return s;
  return validate_select_params(p);
}

inline hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

// ----------------------------------------------------------------- device side
// Wave-uniform copies (the value of the first active lane), for values the compiler
// cannot prove uniform, e.g. arguments of a non-inlined device function.
__device__ __forceinline__ int uniform(int x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ int64_t uniform(int64_t x) {
  const uint64_t u = static_cast<uint64_t>(x);
  const uint32_t lo = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(u));
  const uint32_t hi = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(u >> 32));
  return static_cast<int64_t>((static_cast<uint64_t>(hi) << 32) | lo);
}
template <typename T>
__device__ __forceinline__ T* uniform(T* p) {
  return reinterpret_cast<T*>(uniform(static_cast<int64_t>(reinterpret_cast<uintptr_t>(p))));
}

// threadIdx.x as a value the compiler cannot see through.  A tile function called
// once per work item of a persistent loop derives its per-thread indices from it,
// so they are recomputed per item instead of being hoisted out of the loop and kept
// live (which costs registers and occupancy).
__device__ __forceinline__ int opaque_tid() {
  int t = static_cast<int>(threadIdx.x);
  asm volatile("" : "+v"(t));
  return t;
}

__device__ __forceinline__ int clampi(int x, int lo, int hi) { return x < lo ? lo : (x > hi ? hi : x); }

// A device pointer into global memory, read as such.  Where a pointer is loaded from
// memory (the batch kernels' pair descriptors) rather than passed as a kernel
// argument, the compiler cannot tell it is global and emits flat accesses, which also
// count in the LDS counter, so waits for LDS reads would wait for them too.
template <typename T>
__device__ __forceinline__ const __attribute__((address_space(1))) T* as_global(const T* p) {
  return (const __attribute__((address_space(1))) T*)p;
}

template <typename T>
__device__ __forceinline__ float pixel(const T* img, int64_t pitch, int v, int u) {
  return static_cast<float>(as_global(img)[static_cast<int64_t>(v) * pitch + u]);
}

// Work item of block b in runs of M: blocks are dealt round-robin to the 8 XCDs, and
// within each group of 8 M consecutive items XCD x takes the M items x M .. x M + M - 1.
// Neighbouring items share an L2 while the whole GPU stays on one stretch of the list
// (one pair's volume in the shared cache).  The last partial group of m items is cut
// into 8 contiguous chunks the same way (XCD x takes m / 8 items, one more for
// x < m % 8), so its neighbours share an L2 too: dealing it round-robin instead cost
// 15 % more L2 fetches in the two-view aggregation at 1280x720, whose last 800 of 7200
// items form such a group.  A bijection of [0, n).
template <int M>
__device__ __forceinline__ int xcd_run_item(int b, int n) {
  constexpr int G = 8 * M;
  const int g = b / G;
  const int r = b - g * G;
  const int x = r & 7, i = r >> 3;
  if ((g + 1) * G <= n) return g * G + x * M + i;
  const int m = n - g * G;
  const int q = m >> 3, e = m & 7;
  return g * G + x * q + (x < e ? x : e) + i;
}

}  // namespace rsv
