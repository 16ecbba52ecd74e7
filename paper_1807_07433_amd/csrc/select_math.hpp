// Selection arithmetic shared by the plain select kernel and the batch tail kernel:
// Eq. 12 on the winner and its neighbours, and post-processing + triangulation
// (Sec. II-C, II-D), so both forms round identically.
#pragma once

#include <math.h>

#include "rsv_internal.hpp"

namespace rsv {

// The winner-take-all order (Sec. II-B.3) compares keys: the value itself, or -inf
// for a NaN (from non-finite inputs), so a NaN never beats a number.  A later d
// replaces the running best only when its key is strictly greater, so a pixel's
// winner is the first maximum of its non-NaN values (the first d if all are NaN).
// The order is a total preorder on (key, lower d first), so merging the winners of
// disparity ranges in any grouping gives the same winner as one scan: the tile sinks'
// parallel merges match the select kernel's scan.
__device__ __forceinline__ float wta_key(float v) { return v == v ? v : -INFINITY; }

// Running state of the reference-volume scan over d = 0, 1, ... of one pixel: the
// best key (wta_key) and its d, the second best, and the best's neighbours (values).
// Ties keep the lowest d: a later d replaces the best only when its key is greater.
struct Scan {
  float best, second, am, ap;
  int arg;
};

// The scan after d = 0 with value a.  need_next: the next value is the best's right
// neighbour; prev: the value at the previous d.
__device__ __forceinline__ void scan_init(Scan& s, bool& need_next, float& prev, float a) {
  s.best = wta_key(a);
  s.second = -INFINITY;
  s.am = 0.f;
  s.ap = 0.f;
  s.arg = 0;
  need_next = true;
  prev = a;
}

// One step of the scan at disparity d >= 1 with value a.  SECOND: also track the
// second best (only the optional top-two output reads it).
template <bool SECOND = true>
__device__ __forceinline__ void scan_step(Scan& s, bool& need_next, float& prev, float a, int d) {
  if (need_next) {
    s.ap = a;
    need_next = false;
  }
  const float k = wta_key(a);
  if (k > s.best) {
    if (SECOND) s.second = s.best;
    s.best = k;
    s.arg = d;
    s.am = prev;
    need_next = true;
  } else if (SECOND && k > s.second) {
    s.second = k;
  }
  prev = a;
}

// Eq. 12: d + (a(d-1) - a(d+1)) / (2a(d-1) + 2a(d+1) - 4a(d)); ends of the range unrefined,
// and so is a winner that is not a maximum of its neighbours (the restricted search's
// winner at a window edge can have a larger value just outside; the full method's
// winner never does, so there this test never fires).
__device__ __forceinline__ float parabola(int arg, float best, float am, float ap, int D) {
  if (arg <= 0 || arg >= D - 1) return static_cast<float>(arg);
  if (am > best || ap > best) return static_cast<float>(arg);
  // Eq. 12 written with the gaps below the peak, x = c(d) - c(d-1) and
  // y = c(d) - c(d+1): the offset (x - y) / (2 (x + y)) equals
  // (c(d-1) - c(d+1)) / (2c(d-1) + 2c(d+1) - 4c(d)), and since x, y >= 0 at a
  // maximum the rounded quotient stays within [-1/2, 1/2] (the direct form's
  // denominator can round to 0 when a neighbour is within an ulp of the peak).
  const float x = best - am, y = best - ap;
  const float s = x + y;
  if (!(s > 0.f)) return static_cast<float>(arg);
  return static_cast<float>(arg) + (x - y) / (2.f * s);
}

// d_f = d_s + s(u - d_s, v); xyz = (x, y, z) or NaN when invalid or d_f <= 0.  FP64, one rounding.
__device__ __forceinline__ void postprocess_point(float dsub, bool valid, int u, int v, const rsv_plane& pl,
                                                  const rsv_camera& cam, float* dfin, float* xyz) {
  const double ds = static_cast<double>(dsub);
  const double df = ds + (pl.a0 + pl.a1 * static_cast<double>(v) +
                          pl.a2 * (static_cast<double>(u) - ds) - pl.delta);
  if (dfin) *dfin = static_cast<float>(df);
  if (xyz) {
    if (valid && df > 0.0) {
      const double z = cam.f * cam.baseline / df;
      xyz[0] = static_cast<float>((static_cast<double>(u) - cam.u0) * z / cam.f);
      xyz[1] = static_cast<float>((static_cast<double>(v) - cam.v0) * z / cam.f);
      xyz[2] = static_cast<float>(z);
    } else {
      xyz[0] = xyz[1] = xyz[2] = NAN;
    }
  }
}

}  // namespace rsv
