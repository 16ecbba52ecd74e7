/*
 * rsv.h -- C ABI of the road-surface stereo library (gfx950 / MI355X).
 *
 * The library computes the dense stereo path of Fan et al., "Real-Time Stereo
 * Vision for Road Surface 3-D Reconstruction" (arXiv 1807.07433): the perspective
 * warp of the target image (Sec. II-A), ZNCC reference and target cost volumes
 * (Sec. II-B.1, Eq. 3-5), bilateral cost aggregation (Sec. II-B.2, Eq. 8-10),
 * winner-take-all with the left-right check (Sec. II-B.3/4, Eq. 11), parabola
 * subpixel refinement (Eq. 12), post-processing (Sec. II-C) and triangulation
 * (Sec. II-D).  Two further forms sit on the same kernels: a batched form (one
 * graph launch over many pairs of uneven size and disparity range, no aggregated
 * volume in memory), and the adjoint of the aggregated reference cost for
 * gradient-based refinement of the plane.  Also: the restricted search of Sec. IV
 * (aggregation only around a calculated disparity) and the road-plane fit of
 * Sec. II-A (RANSAC with a least-squares refit).
 *
 * Conventions for every call
 *   - All array pointers are DEVICE pointers (hipMalloc'd or torch tensors) unless
 *     a comment says "host".  The caller owns every buffer; stateless calls never
 *     allocate or free.  Only a batch plan owns device memory (see rsv_batch_*).
 *   - Images are row-major [height][pitch] with pitch >= width (in elements).
 *     Volumes are dense row-major [D][height][width] float32; maps are dense
 *     [height][width].
 *   - `stream` is a hipStream_t (NULL = the default stream).  Calls only enqueue
 *     work and return; results are visible after the caller synchronises.
 *   - Arguments are validated on the host before anything is launched; a call
 *     that returns an error has launched nothing.  Kernel faults surface at the
 *     caller's next synchronisation.  Stateless calls are re-entrant.
 *   - Stateless calls launch kernels only: no memset, copy, allocation or
 *     synchronisation, so a sequence of them may be captured into a HIP graph on
 *     `stream` and replayed (the buffers are bound at capture).
 *   - Return value: RSV_OK (0) or a negative rsv_status.
 */
#ifndef RSV_H_
#define RSV_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  RSV_OK = 0,
  RSV_E_NULL = -1,   /* a required pointer is NULL                                   */
  RSV_E_SHAPE = -2,  /* size out of range: H or W < block width, D < 1 or D > RSV_MAX_D,
                        pitch < width, image sizes disagree                          */
  RSV_E_PARAM = -3,  /* radius unsupported, gamma <= 0, sigma_min < 0, threshold < 0  */
  RSV_E_DTYPE = -4,  /* unknown or unsupported image element type                    */
  RSV_E_ALIGN = -5,  /* pointer not aligned to its element size                      */
  RSV_E_HIP = -6,    /* a HIP runtime call failed; see rsv_last_hip_error()          */
  RSV_E_NOMEM = -7   /* device allocation failed (batch plans only)                  */
} rsv_status;

typedef enum { RSV_U8 = 0, RSV_F32 = 1 } rsv_dtype;

enum {
  RSV_MAX_D = 512,          /* largest residual disparity search range               */
  RSV_MIN_BLOCK_RADIUS = 1, /* NCC block radius range (block width 2r+1: 3x3 .. 9x9) */
  RSV_MAX_BLOCK_RADIUS = 4,
  RSV_MIN_AGG_RADIUS = 1,   /* bilateral window radius range (3x3 .. 13x13)          */
  RSV_MAX_AGG_RADIUS = 6
};

/* An image in device memory: element (v, u) is at data[v * pitch + u]. */
typedef struct {
  const void* data;
  int32_t dtype;   /* rsv_dtype: uint8 grey levels or float32 on the same 0..255 scale */
  int32_t height;
  int32_t width;
  int64_t pitch;   /* elements between row starts */
} rsv_image;

/* Warp plane: shift s(u, v) = a0 + a1*v + a2*u - delta pixels (Eq. 2 gives
 * a0 = alpha0, a1 = alpha1; a2 is the u-slope left by the road's roll, Sec. II-A;
 * delta keeps the residual disparities non-negative). */
typedef struct {
  double a0, a1, a2, delta;
} rsv_plane;

/* Rectified pinhole pair (Sec. II-D): focal length f and principal point (u0, v0)
 * in pixels, baseline in metres. */
typedef struct {
  double f, baseline, u0, v0;
} rsv_camera;

/* Method parameters (Sec. II-B).  gamma_r applies to intensities divided by 255. */
typedef struct {
  int32_t D;             /* residual disparity search range, d = 0 .. D-1         */
  int32_t block_radius;  /* NCC block radius (block width 2*block_radius+1)       */
  int32_t agg_radius;    /* bilateral window radius                                */
  int32_t lr_threshold;  /* left-right check tolerance in pixels (0 = Eq. 11 exact) */
  float gamma_d;         /* spatial parameter of Eq. 9                             */
  float gamma_r;         /* range parameter of Eq. 10                              */
  float sigma_min;       /* block std-dev below which the correlation is 0         */
} rsv_params;

/* ------------------------------------------------------------------ plain path */

/* Perspective warp of the target image into the reference view (Sec. II-A, last
 * paragraph).  warped[v][u] = linear interpolation of row v of `right` at column
 * u - s(u, v), clamp-to-edge, written I0 + f*(I1 - I0).
 *   right   target image, u8 or f32, any pitch
 *   warped  out, float32 [H][W] dense
 * Errors: RSV_E_NULL, RSV_E_DTYPE, RSV_E_SHAPE (H or W < 1, pitch < W). */
int rsv_warp(rsv_image right, rsv_plane plane, float* warped, void* stream);

/* ZNCC cost volumes (Sec. II-B.1, Eq. 3-5).  With clamp-to-edge blocks B of width
 * 2*block_radius+1:
 *   cost_ref[d][v][u] = zncc(B_left(u, v), B_warped(u - d, v))
 *   cost_tar[d][v][x] = zncc(B_left(x + d, v), B_warped(x, v))
 * so cost_tar[d][v][x] == cost_ref[d][v][x + d] bit for bit wherever x + d < W
 * (the identity stated after Eq. 5); beyond that the left block reads are clamped.
 * The correlation is 0 where either block std-dev is below sigma_min.
 *   left      reference image, u8 or f32
 *   warped    float32 [H][W] dense (output of rsv_warp)
 *   cost_ref  out, float32 [D][H][W]
 *   cost_tar  out, float32 [D][H][W], or NULL to skip the target volume
 * Errors: RSV_E_NULL, RSV_E_DTYPE, RSV_E_SHAPE, RSV_E_PARAM (block_radius,
 * sigma_min), RSV_E_ALIGN. */
int rsv_cost_volume(rsv_image left, const float* warped, const rsv_params* p,
                    float* cost_ref, float* cost_tar, void* stream);

/* Both ZNCC volumes of rsv_cost_volume as one joint volume (Sec. II-B.1, Eq. 3-5 and
 * the identity stated after Eq. 5):
 *   joint[d][v][u] = zncc(B_left(u, v), B_warped(u - d, v)),  u = 0 .. W + D - 2
 * (left blocks clamp-to-edge past column W - 1).  The two volumes are its views:
 *   cost_ref[d][v][u] = joint[d*(H*row_stride)     + v*row_stride + u]
 *   cost_tar[d][v][x] = joint[d*(H*row_stride + 1) + v*row_stride + x]   (= joint[d][v][x + d])
 * bit for bit equal to rsv_cost_volume's outputs, with 4 B written per entry instead
 * of 8.  Aggregate the views with rsv_aggregate_strided.
 *   joint       out, float32 [D][H][row_stride]; columns >= W + D - 1 are not written
 *   row_stride  elements, >= W + D - 1; a multiple of 64 keeps every 64-centre row
 *               segment 256-byte aligned
 * Errors: as rsv_cost_volume; RSV_E_SHAPE also for row_stride < W + D - 1 or
 * H*row_stride > 2^31 - 1. */
int rsv_cost_volume_joint(rsv_image left, const float* warped, const rsv_params* p,
                          float* joint, int64_t row_stride, void* stream);

/* Bilateral cost aggregation (Sec. II-B.2, Eq. 8-10) of one volume:
 *   agg[d][v][u] = sum_q w(p, q) cost[d][q] / sum_q w(p, q),  p = (u, v),
 *   w = exp(-|q - p|^2 / gamma_d^2) * exp(-((g(q) - g(p)) / 255)^2 / gamma_r^2)
 * over the (2*agg_radius+1)^2 window; taps outside the image are skipped.  Call it
 * once per volume: guide = left image for cost_ref, warped image for cost_tar.
 *   cost   float32 [D][H][W];  guide  u8 or f32 image of the same H, W
 *   agg    out, float32 [D][H][W] (must not alias cost)
 * Errors: RSV_E_NULL, RSV_E_DTYPE, RSV_E_SHAPE (also H*W > 2^26), RSV_E_PARAM
 * (agg_radius, gammas), RSV_E_ALIGN. */
int rsv_aggregate(const float* cost, rsv_image guide, const rsv_params* p, float* agg,
                  void* stream);

/* rsv_aggregate on a strided view of a cost volume (Sec. II-B.2, Eq. 8-10):
 *   cost(d, v, u) = cost[d*plane_stride + v*row_stride + u],  d < D, v < H, u < W,
 * e.g. the reference and target views of rsv_cost_volume_joint's volume.  Only the
 * view's elements are read; views may overlap themselves (the target view does).
 *   agg    out, float32 [D][H][W] dense, outside the view
 * Errors: as rsv_aggregate; RSV_E_SHAPE also for row_stride < W, plane_stride < 1,
 * plane_stride > 2^26 or (H-1)*row_stride + W > 2^26. */
int rsv_aggregate_strided(const float* cost, int64_t plane_stride, int64_t row_stride,
                          rsv_image guide, const rsv_params* p, float* agg, void* stream);

/* The winner-take-all disparity of an aggregated volume that is needed for nothing
 * else (the target volume, Sec. II-B.3): the aggregation of rsv_aggregate_strided's
 * view, reduced over d as it is computed, without writing the volume:
 *   disp[v][u] = argmax_d agg(d, v, u), ties -> lowest d
 * bit for bit the disp_tar that rsv_select_subpixel computes from rsv_aggregate's
 * volume.
 *   disp   out, int32 [H][W] dense
 * Errors: as rsv_aggregate_strided (RSV_E_NULL for disp). */
int rsv_aggregate_argmax(const float* cost, int64_t plane_stride, int64_t row_stride,
                         rsv_image guide, const rsv_params* p, int32_t* disp, void* stream);

/* Disparity selection and refinement (Sec. II-B.3 and II-B.4):
 *   disp_ref = argmax_d agg_ref, disp_tar = argmax_d agg_tar (ties -> lowest d);
 *   valid    = (u - disp_ref >= 0) && |disp_ref - disp_tar(u - disp_ref, v)| <= lr_threshold
 *              (Eq. 11 with a tolerance);
 *   disp_sub = d + (a(d-1) - a(d+1)) / (2a(d-1) + 2a(d+1) - 4a(d)) on agg_ref (Eq. 12),
 *              d itself at d = 0 or D-1.
 *   agg_ref, agg_tar  float32 [D][H][W]
 *   disp_ref, disp_tar  out, int32 [H][W];  disp_sub out, float32 [H][W]
 *   valid    out, uint8 [H][W] (1 = passes the check)
 *   top2     out, float32 [2][H][W]: best and second-best agg_ref value, or NULL
 * Errors: RSV_E_NULL, RSV_E_SHAPE, RSV_E_PARAM, RSV_E_ALIGN. */
int rsv_select_subpixel(const float* agg_ref, const float* agg_tar, int32_t height,
                        int32_t width, const rsv_params* p, int32_t* disp_ref,
                        int32_t* disp_tar, float* disp_sub, uint8_t* valid, float* top2,
                        void* stream);

/* rsv_select_subpixel with the target disparities given (e.g. from
 * rsv_aggregate_argmax) instead of the target volume: WTA and Eq. 12 on agg_ref,
 * Eq. 11 against disp_tar.  Outputs equal rsv_select_subpixel's bit for bit.
 *   disp_tar  int32 [H][W], read
 * Errors: as rsv_select_subpixel. */
int rsv_select_subpixel_ref(const float* agg_ref, const int32_t* disp_tar, int32_t height,
                            int32_t width, const rsv_params* p, int32_t* disp_ref,
                            float* disp_sub, uint8_t* valid, float* top2, void* stream);

/* The reference aggregation with the selection folded in (Sec. II-B.2 to II-B.4,
 * Eq. 8-12): rsv_aggregate_strided's view aggregated with the guide, and per pixel
 * the winner-take-all disparity, Eq. 12 on it and Eq. 11 against disp_tar, as the
 * aggregation is computed; no aggregated volume is written.  Outputs equal those of
 * rsv_aggregate_strided followed by rsv_select_subpixel_ref bit for bit.  Runs
 * where the cost tiles are loaded straight into LDS: agg_radius <= 5 and W >= 4
 * (callers fall back to those two calls otherwise).
 *   cost(d, v, u) = cost[d*plane_stride + v*row_stride + u] (the reference view)
 *   guide     the left image (u8 or f32)
 *   disp_tar  int32 [H][W], read: the target disparities (rsv_aggregate_argmax),
 *             complete before this call's work starts on the stream
 *   disp_ref  out, int32 [H][W];  disp_sub out, float32 [H][W];  valid out, uint8 [H][W]
 * Errors: as rsv_aggregate_strided and rsv_select_subpixel; RSV_E_PARAM also for
 * agg_radius > 5, RSV_E_SHAPE also for W < 4. */
int rsv_aggregate_select(const float* cost, int64_t plane_stride, int64_t row_stride,
                         rsv_image guide, const rsv_params* p, const int32_t* disp_tar,
                         int32_t* disp_ref, float* disp_sub, uint8_t* valid, void* stream);

/* Both views' aggregation in one launch (Sec. II-B.2 and II-B.3, Eq. 8-10 and 12):
 * the target view reduced to its winner-take-all map as rsv_aggregate_argmax does, and
 * the reference view to its winner and Eq. 12 as rsv_aggregate_select does; the
 * left-right check (Eq. 11) is left to rsv_lr_check, which needs the complete target
 * map.  disp_tar, disp_ref and disp_sub equal those of rsv_aggregate_argmax followed
 * by rsv_select_subpixel_ref (the winner and Eq. 12) bit for bit; no aggregated volume
 * is written.  Every window radius and width: where agg_radius <= 5 and W >= 4 the
 * cost tiles are loaded straight into LDS; otherwise the register-staged tile of
 * rsv_aggregate runs, with the selection's scan over d kept in LDS.
 *   cost_ref(d, v, u) = cost_ref[d*ref_plane_stride + v*ref_row_stride + u] (the
 *             reference view), cost_tar likewise (the target view; e.g. both views of
 *             one joint volume)
 *   guide_ref the left image (u8 or f32);  guide_tar the warped right image (f32),
 *             of the same H, W
 *   disp_tar, disp_ref out, int32 [H][W];  disp_sub out, float32 [H][W]
 * Errors: RSV_E_NULL, RSV_E_ALIGN, RSV_E_PARAM (radii out of range, lr_threshold < 0),
 * RSV_E_SHAPE (row stride < W, plane stride < 1, (H - 1) * row stride + W or a plane
 * stride above 2^26, guides of different sizes), RSV_E_DTYPE for a guide_tar that is
 * not float32, RSV_E_HIP. */
int rsv_aggregate_views(const float* cost_ref, int64_t ref_plane_stride, int64_t ref_row_stride,
                        const float* cost_tar, int64_t tar_plane_stride, int64_t tar_row_stride,
                        rsv_image guide_ref, rsv_image guide_tar, const rsv_params* p,
                        int32_t* disp_tar, int32_t* disp_ref, float* disp_sub, void* stream);

/* Left-right consistency check (Sec. II-B.4, Eq. 11) of two winner-take-all maps:
 *   valid(u, v) = (u - disp_ref >= 0) && |disp_ref - disp_tar(u - disp_ref, v)| <= tau
 * with disp_ref = disp_ref(u, v), as the select kernels compute it.
 *   disp_ref, disp_tar  int32 [H][W], read;  valid out, uint8 [H][W]
 * Errors: RSV_E_NULL, RSV_E_ALIGN (int32 maps not 4-byte aligned), RSV_E_SHAPE
 * (H or W < 1), RSV_E_PARAM (tau < 0), RSV_E_HIP. */
int rsv_lr_check(const int32_t* disp_ref, const int32_t* disp_tar, int32_t height, int32_t width,
                 int32_t tau, uint8_t* valid, void* stream);

/* ------------------------------------------- restricted search (Sec. IV)
 * The paper's proposed speed-up: bilateral filtering only on the disparities around
 * an already calculated disparity instead of on the whole cost volume.  Here the
 * calculated disparity of a pixel is the winner-take-all of its unaggregated
 * correlation (rsv_cost_argmax), and its window is the width = min(2*radius + 1, D)
 * disparities lo .. lo + width - 1, lo = clamp(coarse - radius, 0, D - width).  The
 * aggregated values in a window are the full method's floats; the winner is the first
 * maximum inside the window. */

/* Winner-take-all of an unaggregated cost view (Sec. II-B.3's rule on Eq. 3's c):
 *   disp[v][u] = argmax_d cost[d*plane_stride + v*row_stride + u], ties -> lowest d
 * (e.g. the reference and target views of rsv_cost_volume_joint's volume).
 *   disp  out, int32 [H][W]
 * Errors: RSV_E_NULL, RSV_E_SHAPE (H, W, D < 1, D > RSV_MAX_D, row_stride < W,
 * plane_stride < 1), RSV_E_ALIGN. */
int rsv_cost_argmax(const float* cost, int64_t plane_stride, int64_t row_stride, int32_t height,
                    int32_t width, int32_t D, int32_t* disp, void* stream);

/* rsv_cost_argmax of two views in one pass: disp_ref of cost_ref and disp_tar of
 * cost_tar, each bit for bit rsv_cost_argmax's.  Where the two are views of one joint
 * volume (rsv_cost_volume_joint), a thread reads entry (d, v, u) of both views, whose
 * lines the other view's threads also read, so the volume is fetched about once.
 *   disp_ref, disp_tar  out, int32 [H][W]
 * Errors: as rsv_cost_argmax, for either view. */
int rsv_cost_argmax_views(const float* cost_ref, int64_t ref_plane_stride, int64_t ref_row_stride,
                          const float* cost_tar, int64_t tar_plane_stride, int64_t tar_row_stride,
                          int32_t height, int32_t width, int32_t D, int32_t* disp_ref, int32_t* disp_tar,
                          void* stream);

/* rsv_aggregate_argmax restricted to each pixel's window around coarse[v][u]: the
 * first maximum over the window of the aggregation of Eq. 8-10.
 *   coarse  int32 [H][W], read (any values; clamped into the range as above)
 *   radius  >= 0;  disp out, int32 [H][W]
 * Runs where the LDS-loaded tile does (agg_radius <= 5, W >= 4).
 * Errors: as rsv_aggregate_argmax; RSV_E_PARAM also for radius < 0 or agg_radius > 5,
 * RSV_E_SHAPE also for W < 4. */
int rsv_aggregate_restricted_argmax(const float* cost, int64_t plane_stride, int64_t row_stride,
                                    rsv_image guide, const rsv_params* p, const int32_t* coarse,
                                    int32_t radius, int32_t* disp, void* stream);

/* rsv_aggregate_select restricted to each pixel's window around coarse[v][u]: the
 * winner inside the window, Eq. 12 on it with the aggregated values at d - 1 and d + 1
 * (also computed where they leave the window), Eq. 11 against disp_tar.
 * Errors: as rsv_aggregate_select; RSV_E_PARAM also for radius < 0. */
int rsv_aggregate_restricted_select(const float* cost, int64_t plane_stride, int64_t row_stride,
                                    rsv_image guide, const rsv_params* p, const int32_t* coarse,
                                    int32_t radius, const int32_t* disp_tar, int32_t* disp_ref,
                                    float* disp_sub, uint8_t* valid, void* stream);

/* Both views' restricted aggregations in one launch, as rsv_aggregate_views does for
 * the full range: the target view's winner inside each pixel's window around
 * coarse_tar (rsv_aggregate_restricted_argmax's disp), the reference view's winner
 * inside its window around coarse_ref and Eq. 12 on it (rsv_aggregate_restricted_
 * select's disp_ref and disp_sub), bit for bit; the left-right check is rsv_lr_check's.
 *   cost_ref / cost_tar, guide_ref / guide_tar  as rsv_aggregate_views
 *   coarse_ref, coarse_tar  int32 [H][W], read;  radius >= 0
 *   disp_tar, disp_ref out, int32 [H][W];  disp_sub out, float32 [H][W]
 * Errors: as rsv_aggregate_views; RSV_E_NULL and RSV_E_ALIGN also for the coarse maps,
 * RSV_E_PARAM also for radius < 0. */
int rsv_aggregate_restricted_views(const float* cost_ref, int64_t ref_plane_stride, int64_t ref_row_stride,
                                   const float* cost_tar, int64_t tar_plane_stride, int64_t tar_row_stride,
                                   rsv_image guide_ref, rsv_image guide_tar, const rsv_params* p,
                                   const int32_t* coarse_ref, const int32_t* coarse_tar, int32_t radius,
                                   int32_t* disp_tar, int32_t* disp_ref, float* disp_sub, void* stream);

/* Road-plane estimation (Sec. II-A): the plane of disparities d = a0 + a1 v + a2 u
 * that the warp of Eq. 2 uses (a0, a1 as in Eq. 2; a2 the term of the roll-fitted
 * plane), fitted by least squares inside RANSAC to the valid pixels of a disparity
 * map (e.g. the previous frame's post-processed disparities).
 *   disp     float32 [H][W], read; valid uint8 [H][W] (nonzero = a correspondence)
 *   samples  int32 [K][3], the random draws: linear pixel indices v*W + u, 1 <= K <=
 *            RSV_PLANE_MAX_K (drawing them is the caller's; an index out of range or
 *            three pixels on one line of the image make the hypothesis degenerate)
 *   threshold  inlier bound |d - (a0 + a1 v + a2 u)| <= threshold (>= 0), in FP64
 *   plane    out, double[3] (a0, a1, a2): the least-squares plane of the inliers of
 *            the best hypothesis (most inliers, ties to the lowest index)
 *   counts   out, int32 [K]: inliers per hypothesis, -1 where degenerate
 *   best     out, int32[2]: the best hypothesis and its inlier count
 *   workspace  device, rsv_plane_ransac_workspace_bytes(K) bytes, 8-byte aligned
 * All outputs are device memory written on the stream.  With no non-degenerate
 * hypothesis or fewer than 3 non-collinear inliers the plane holds non-finite values.
 * The roll angle is atan(-a2 / a1).
 * Errors: RSV_E_NULL, RSV_E_SHAPE (H or W < 1, H*W > 2^31 - 1, K out of range),
 * RSV_E_PARAM (threshold < 0 or NaN), RSV_E_ALIGN. */
enum { RSV_PLANE_MAX_K = 1024 };
size_t rsv_plane_ransac_workspace_bytes(int32_t K);
int rsv_plane_ransac(const float* disp, const uint8_t* valid, int32_t height, int32_t width,
                     const int32_t* samples, int32_t K, float threshold, double* plane, int32_t* counts,
                     int32_t* best, void* workspace, void* stream);

/* Post-processing (Sec. II-C) and 3-D reconstruction (Sec. II-D):
 *   disp_final = disp_sub + s(u - disp_sub, v)            (every pixel)
 *   xyz[v][u]  = (x, y, z), z = f*baseline/disp_final, x = (u-u0) z/f, y = (v-v0) z/f,
 *                NaN where valid == 0 or disp_final <= 0.
 *   disp_final out, float32 [H][W];  xyz out, float32 [H][W][3] (either may be NULL)
 * Errors: RSV_E_NULL, RSV_E_SHAPE, RSV_E_PARAM (f or baseline <= 0). */
int rsv_triangulate(const float* disp_sub, const uint8_t* valid, int32_t height,
                    int32_t width, rsv_plane plane, rsv_camera cam, float* disp_final,
                    float* xyz, void* stream);

/* ------------------------------------------------------------ batched form */

/* One stereo pair of a batch.  Pairs may differ in size and in D; all share the
 * rsv_params of the plan (p->D is ignored).  The plan keeps the pointers: inputs and
 * outputs must stay valid while the plan is used. */
typedef struct {
  rsv_image left, right;  /* uint8 pair of the same H, W (W <= 16384), any pitch */
  rsv_plane plane;
  rsv_camera camera;
  int32_t D;              /* this pair's residual search range, 1 .. RSV_MAX_D        */
  int32_t reserved;
  int32_t* disp_ref;      /* out int32 [H][W] or NULL                                 */
  int32_t* disp_tar;      /* out int32 [H][W] or NULL                                 */
  float* disp_sub;        /* out float32 [H][W]                                       */
  uint8_t* valid;         /* out uint8 [H][W]                                         */
  float* disp_final;      /* out float32 [H][W] or NULL                               */
  float* xyz;             /* out float32 [H][W][3] or NULL                            */
} rsv_pair_desc;

/* Launch shape of a plan (rsv_tuning_default fills the defaults). */
typedef struct {
  int32_t largest_first;        /* 1: queue the pairs by decreasing W*H*D; 0: as given    */
  int32_t cost_tiles_per_item;  /* cost work item = this many tiles of 64 centres x 4
                                   rows (3x3, 5x5 blocks) or x 16 rows (7x7, 9x9)
                                   (1 .. 16; 1 when cost_blocks_per_cu = -1)               */
  int32_t cost_blocks_per_cu;   /* persistent cost workgroups per CU; 0 = as many as fit
                                   (default); -1 = one workgroup per cost item, no queue */
  int32_t agg_blocks_per_cu;    /* persistent aggregation workgroups per CU; 0 = as fit  */
  int32_t per_pair_launches;    /* 1 (default): each pair's cost launch and then its tile
                                   launch, pair after pair within a group, each kernel
                                   taking the pair's descriptor as an argument (implies
                                   one cost workgroup per tile); 0: one launch per phase
                                   and group over the item lists                        */
  int32_t volume_budget_mib;    /* 0: every pair's joint cost volume resident at once;
                                   > 0 (default 2048): device memory for cost volumes, MiB:
                                   the pairs run in groups of consecutive pairs whose
                                   volumes fit half of it (a larger pair forms a group of
                                   its own), alternating between two slots on two graph
                                   branches, so that one group's volumes are computed
                                   while the previous group is aggregated               */
} rsv_tuning;

typedef struct rsv_batch_plan rsv_batch_plan;

void rsv_tuning_default(rsv_tuning* t);

/* Builds a plan for the whole batch: device workspace for every pair's warped image
 * and selection state, the joint cost volumes of the pairs in flight
 * (rsv_cost_volume_joint's layout, row stride W + D - 1 rounded up to 64), the work
 * lists, and a hipGraph of
 *   [reset queue counters] -> [warp every pair] -> per group of pairs: [cost kernel]
 *   -> [tile kernel] -> [per-pixel tail]
 * (one group without a volume budget; with one, groups alternate between two volume
 * slots on two graph branches, see rsv_tuning).  The cost kernel runs ZNCC (the
 * arithmetic of rsv_cost_volume_joint): persistent over a work queue, one workgroup
 * per tile, or, in the per-pair schedule (the default), one launch per pair taking the
 * pair's descriptor as an argument.  Where agg_radius <= 5 and W >= 4 the tile kernel
 * takes one workgroup per (pair, 16 x 16 block, view), the LDS-loaded aggregation tile
 * of rsv_aggregate_views (reference view: winner and Eq. 12; target view: its argmax),
 * per pair in the per-pair schedule; otherwise a persistent kernel pulls (pair, block,
 * view) items from per-XCD atomic counters and runs rsv_aggregate's tile with
 * winner-take-all fused in.  No aggregated volume is written.  The tail runs the
 * left-right check, post-processing and triangulation (those of rsv_lr_check and
 * rsv_triangulate).  Every output equals the plain path's bit for bit.
 *   pairs, n   the batch (host array, copied)
 *   p          shared parameters (block_radius, agg_radius, gammas, lr_threshold,
 *              sigma_min); p->D is ignored
 *   tuning     launch shape, or NULL for the defaults (see rsv_autotune)
 *   out        host pointer receiving the plan
 * The plan owns its device memory and graph: the cost volumes (about
 * 4 * sum(H*(W+D)*D) bytes, or two slots of at most half the tuning's volume budget
 * each, or of the largest pair's volume if that is larger) plus 12 bytes per pixel.
 * Errors: RSV_E_NULL, RSV_E_SHAPE (also H * row stride + 1 > 2^26 for a pair),
 * RSV_E_PARAM, RSV_E_DTYPE (pairs must be uint8), RSV_E_NOMEM, RSV_E_HIP. */
int rsv_batch_plan_create(const rsv_pair_desc* pairs, int32_t n, const rsv_params* p,
                          const rsv_tuning* tuning, rsv_batch_plan** out);

/* Launches the plan's graph on `stream` (one hipGraphLaunch).  A plan must not run
 * concurrently on two streams. */
int rsv_batch_run(rsv_batch_plan* plan, void* stream);

/* Host arrays n_items[2] and grid_blocks[2] receive the cost / aggregation item
 * counts and persistent workgroup counts; *workspace_bytes the plan's device bytes.
 * Any pointer may be NULL. */
int rsv_batch_plan_info(const rsv_batch_plan* plan, int32_t* n_items, int32_t* grid_blocks,
                        int64_t* workspace_bytes);

int rsv_batch_plan_destroy(rsv_batch_plan* plan);

/* Times candidate launch shapes (pair order x cost tiles per item x cost workgroups
 * per CU x per-pair launches, at the default volume budget; then volume budgets of
 * 0, 512 and 4096 MiB on the fastest shape) on this batch, each with its own
 * temporary plan, and returns the fastest in *out and its time in *best_ms (may be
 * NULL).  Writes the pairs' outputs.  Synchronises `stream`. */
int rsv_autotune(const rsv_pair_desc* pairs, int32_t n, const rsv_params* p, rsv_tuning* out,
                 float* best_ms, void* stream);

/* ------------------------------------------------------ differentiable form */

/* Loss of the differentiable form: sum of agg_ref[disp(p)][p] over the pixels p with
 * mask(p) != 0 and 0 <= disp(p) < D (the aggregated reference cost of Eq. 8 at the
 * selected disparities, Sec. II-B.3).
 *   agg_ref  float32 [D][H][W];  disp int32 [H][W];  mask uint8 [H][W]
 *   out      device double[1], overwritten
 * Errors: RSV_E_NULL, RSV_E_SHAPE, RSV_E_ALIGN. */
int rsv_selected_cost_sum(const float* agg_ref, const int32_t* disp, const uint8_t* mask,
                          int32_t height, int32_t width, int32_t D, double* out, void* stream);

/* The same loss from a cost volume, with no aggregated volume (Sec. II-B.2, Eq. 8-10,
 * at one disparity per pixel): sum over the pixels p with mask(p) != 0 and
 * 0 <= disp(p) < D of
 *   A(p) = sum_q w(p, q) cost(disp(p), q) / sum_q w(p, q)
 * over p's (2*agg_radius+1)^2 window inside the image, w of Eq. 9-10 with the guide,
 * accumulated in float per pixel and in double over pixels.  Equal to
 * rsv_selected_cost_sum on rsv_aggregate's volume to float rounding.
 *   cost(d, v, u) = cost[d*plane_stride + v*row_stride + u]  (e.g. the reference
 *                   view of rsv_cost_volume_joint's volume)
 *   guide    the left image (u8 or f32), H x W
 *   disp, mask  int32 / uint8 [H][W];  out  device double[1], overwritten
 * Errors: RSV_E_NULL, RSV_E_DTYPE, RSV_E_SHAPE (row_stride < W, plane_stride < 1,
 * (H-1)*row_stride + W > 2^31 - 1), RSV_E_PARAM (agg_radius, gammas), RSV_E_ALIGN. */
int rsv_selected_aggregate_sum(const float* cost, int64_t plane_stride, int64_t row_stride,
                               rsv_image guide, const rsv_params* p, const int32_t* disp,
                               const uint8_t* mask, double* out, void* stream);

/* Bytes of device workspace rsv_cost_adjoint needs for an H x W pair (0 if invalid). */
size_t rsv_cost_adjoint_workspace_bytes(int32_t height, int32_t width);

/* Adjoint of the loss above with disp and mask held fixed: gradients with respect to
 * the warp plane (a0, a1, a2) of Sec. II-A and both input images, through the warp,
 * the ZNCC of Eq. 3-5 and the bilateral aggregation of Eq. 8-10.  The weights and
 * the aggregated costs A(p) are recomputed from the images and the cost volume, never
 * stored; the weights' dependence on the left image is included.
 *   left, right   float32 images the forward ran on (same H, W)
 *   plane, p      the forward's plane and parameters (D <= 256)
 *   cost(d, v, u) = cost[d*plane_stride + v*row_stride + u]: the forward's reference
 *                 cost volume (rsv_cost_volume's cost_ref, or the reference view of
 *                 rsv_cost_volume_joint's volume)
 *   disp, mask    int32 / uint8 [H][W]; pixels with mask == 0 or disp outside [0, D)
 *                 are not in the loss
 *   grad_left, grad_right  out float32 [H][W] (dense), overwritten
 *   grad_plane    out device double[3] = dL/d(a0, a1, a2), overwritten
 *   loss          out device double[1] (the loss of rsv_selected_aggregate_sum), or NULL
 *   workspace     device buffer of rsv_cost_adjoint_workspace_bytes(H, W) bytes, owned
 *                 by the caller; its contents are scratch
 * Results are sums of float atomics: equal to rounding, not bit for bit, run to run.
 * Errors: RSV_E_NULL, RSV_E_DTYPE (images not float32), RSV_E_SHAPE (also D > 256,
 * H or W < block width, the cost view's strides as rsv_selected_aggregate_sum),
 * RSV_E_PARAM, RSV_E_ALIGN. */
int rsv_cost_adjoint(rsv_image left, rsv_image right, rsv_plane plane, const rsv_params* p,
                     const float* cost, int64_t plane_stride, int64_t row_stride,
                     const int32_t* disp, const uint8_t* mask, float* grad_left,
                     float* grad_right, double* grad_plane, double* loss, void* workspace,
                     void* stream);

/* rsv_cost_adjoint for callers that cannot allocate device memory (code under HIP
 * graph capture, serving loops, harnesses that forbid hipMalloc): the same arguments
 * without `workspace`, and the same results (to float rounding, as any two runs).
 * The workspace lives in a static device array inside the library, of
 * RSV_ADJOINT_NOALLOC_MAX_PIXELS floats (8 MiB); every GPU the library runs this call
 * on keeps its copy until the process ends.  The call uses the array of the calling
 * thread's current device, so `stream` must belong to that device.  It allocates and
 * frees nothing; its first call on a device resolves the array's device address.
 * All calls on one GPU share that array, and nothing in it needs clearing between
 * calls (every element a call reads it first writes), so calls that overlap on one
 * GPU (concurrent streams or threads) race and must be serialised by the caller.
 * Errors: as rsv_cost_adjoint; RSV_E_SHAPE also for H*W > RSV_ADJOINT_NOALLOC_MAX_PIXELS;
 * RSV_E_HIP if the current device or the array's address cannot be obtained. */
enum { RSV_ADJOINT_NOALLOC_MAX_PIXELS = 1 << 21 };
int rsv_cost_adjoint_noalloc(rsv_image left, rsv_image right, rsv_plane plane, const rsv_params* p,
                             const float* cost, int64_t plane_stride, int64_t row_stride,
                             const int32_t* disp, const uint8_t* mask, float* grad_left,
                             float* grad_right, double* grad_plane, double* loss, void* stream);

/* --------------------------------------------------------------- diagnostics */

/* Text for a status code (static storage, never NULL). */
const char* rsv_status_string(int status);

/* hipError_t of the last failing HIP call made by this thread (0 if none). */
int rsv_last_hip_error(void);

/* Library version as major*10000 + minor*100 + patch. */
int rsv_version(void);

#ifdef __cplusplus
}
#endif

#endif /* RSV_H_ */
