// Winner-take-all sink for the register-staged aggregation tile (agg_tile.hpp):
// the select kernel's scan over d (Sec. II-B.3, Eq. 12's neighbours) for the tile's
// 256 pixels, 16 disparities at a time, its state in LDS.  Shared by the batch's
// aggregation items and the two-view launch for windows the LDS-loaded tile does not
// take, so both give the select kernel's maps bit for bit.
#pragma once

#include "agg_tile.hpp"
#include "select_math.hpp"

namespace rsv {

// Scan state of the 256 pixels of one aggregation item, in LDS between disparity
// tiles (kept out of registers, which the tile needs).
struct WtaState {
  float best[256], am[256], ap[256], prev[256];
  int arg[256], need_next[256];
};

// agg_tile sink that runs the select kernel's scan over d for the tile's 256
// pixels, 16 disparities at a time: thread p < 256 owns pixel p (row p / 16,
// column p % 16).
struct WtaSink {
  WtaState* st;
  int D;
  bool full;  // reference volume: best and its neighbours; target: argmax only (the
              // batch has no top-two output, so no second best is kept)

  __device__ __forceinline__ void operator()(int t, const float* o) {
    const int p = threadIdx.x;
    if (p >= 256) return;
    Scan s;
    bool need_next = false;
    float prev = 0.f;
    if (t > 0) {
      s.best = st->best[p];
      s.arg = st->arg[p];
      if (full) {
        s.am = st->am[p];
        s.ap = st->ap[p];
        prev = st->prev[p];
        need_next = st->need_next[p] != 0;
      }
    }
    const int n = min(16, D - 16 * t);
    for (int dd = 0; dd < n; ++dd) {
      const float a = o[dd * AggGeo<1, 16>::OST + p];
      const int d = 16 * t + dd;
      if (full) {
        if (d == 0)
          scan_init(s, need_next, prev, a);
        else
          scan_step<false>(s, need_next, prev, a, d);
      } else if (d == 0 || wta_key(a) > s.best) {
        s.best = wta_key(a);
        s.arg = d;
      }
    }
    st->best[p] = s.best;
    st->arg[p] = s.arg;
    if (full) {
      st->am[p] = s.am;
      st->ap[p] = s.ap;
      st->prev[p] = prev;
      st->need_next[p] = need_next ? 1 : 0;
    }
  }
};

}  // namespace rsv
