/*
 * pmsref.h -- plain FP64 CPU reference ("the oracle") of equirectangular
 * PatchMatch-Stereo densification (Surmann, Thurow, Slomma,
 * "PatchMatch-Stereo-Panorama, a fast dense reconstruction from 360 degree
 * video images", Sec. III).
 *
 * TEST INFRASTRUCTURE. Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark load this library. The GPU library never
 * links, includes or calls it, and it shares no source with the GPU library.
 *
 * Everything is double precision and single-image-size: every image of one
 * call is W x H with W == 2H, row-major, one value per pixel, intensities as
 * given (the caller scales 8-bit images by 1/255 before the call).
 *
 * Camera model (the paper fixes none; this is the reading used throughout):
 *   longitude  lam(x) = 2*pi*(x + 0.5)/W - pi
 *   latitude   phi(y) = pi/2 - pi*(y + 0.5)/H
 *   bearing    b      = (cos phi sin lam, -sin phi, cos phi cos lam)
 * in a camera frame with x right, y down, z forward. Poses are world->camera:
 * X_cam = R X_world + t, R row-major.
 *
 * Parity status of each function is stated at its definition in pmsref.c.
 */
#ifndef PMSREF_H
#define PMSREF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PMSREF_MAX_VIEWS 16
#define PMSREF_MAX_OFFSETS 16
#define PMSREF_MAX_SAMPLES 1024

typedef struct {
    double R[9]; /* row-major, world -> camera */
    double t[3];
} pmsref_pose;

typedef struct {
    int32_t patch_size;    /* odd; patch radius r = (patch_size-1)/2       */
    int32_t patch_stride;  /* sample spacing s; offsets -r, -r+s, ..., r   */
    int32_t iterations;    /* red+black sweeps                             */
    int32_t refine_trials; /* random refinement trials per pixel per sweep */
    double depth_min, depth_max; /* range along the unit ray, metres      */
    int32_t top_k;               /* views averaged; 0 => ceil(N/2)        */
    double ncc_var_floor;        /* variance floor on scaled intensities  */
    double refine_sigma_logdepth0; /* <=0 => 0.5*ln(depth_max/depth_min)  */
    double refine_depth_shrink;    /* per-trial factor on the log range   */
    double refine_sigma_normal0;   /* initial normal perturbation width   */
    double refine_normal_shrink;   /* per-trial factor on the normal width*/
    int32_t n_offsets;             /* propagation neighbourhood size      */
    int32_t offsets[PMSREF_MAX_OFFSETS][2]; /* (dx, dy), odd |dx|+|dy|    */
    double geo_px;        /* reprojection threshold, pixels               */
    double geo_rel_depth; /* relative depth threshold                     */
    int32_t geo_min_views; /* views that must agree; 0 => min(2, #maps)   */
    uint64_t seed;
    int32_t median_radius; /* median post-filter window radius; 0 = off   */
    double median_rel;     /* drop where |d - median| > median_rel * median */
} pmsref_params;

/* Fill the default parameters (11x11 patch sampled every 2nd pixel,
   8 iterations, 6 refinement trials, 0.3-30 m, 8-neighbourhood). */
void pmsref_default_params(pmsref_params *p);

/* 0 on success, otherwise a negative code; pmsref_check_params only
   validates and never writes anything. */
int pmsref_check_params(const pmsref_params *p, int W, int H, int n_views);

/* --- camera model --------------------------------------------------------*/
void pmsref_unproject(int W, int H, double x, double y, double b[3]);
void pmsref_project(int W, int H, const double Y[3], double *x, double *y);
double pmsref_sample(const double *img, int W, int H, double x, double y);

/* --- relative pose: ref camera -> neighbour camera -----------------------*/
void pmsref_relative_pose(const pmsref_pose *ref, const pmsref_pose *nbr,
                          double R[9], double t[3]);

/* --- counter-based RNG: Philox4x64 with 10 rounds ------------------------*/
void pmsref_philox4x64_10(uint64_t key0, uint64_t key1, const uint64_t ctr[4],
                          uint64_t out[4]);
/* Blocks for counters (ctr0 + i, 0, 0, 0), i < n, into out[4n]. */
void pmsref_philox4x64_10_stream(uint64_t key0, uint64_t key1, uint64_t ctr0, long n,
                                 uint64_t *out);
/* Four uniforms in [0,1) with 24 bits each for (seed, pixel, iter, stage). */
void pmsref_uniforms(uint64_t seed, uint64_t pixel, uint64_t iteration,
                     uint64_t stage, double u[4]);

/* --- patch -----------------------------------------------------------------
   Number of samples of the patch, and its offsets in row-major order. */
int pmsref_patch_offsets(const pmsref_params *p, int32_t *dx, int32_t *dy);

/* --- one view, one hypothesis ----------------------------------------------
   Cost 1 - NCC in [0, 2] of hypothesis (depth d, normal n) at ref pixel
   (x, y) against neighbour image `nbr` under relative pose (R, t); 2 when the
   view is invalid. When r_out/s_out are non-null the P reference and warped
   neighbour samples are written there (only if every sample warped), and
   *vr_out / *vs_out receive the two variances. Returns the cost. */
double pmsref_view_cost(int W, int H, const double *ref, const double *nbr,
                        const double R[9], const double t[3],
                        const pmsref_params *p, int x, int y, double d,
                        const double n[3], double *r_out, double *s_out,
                        double *vr_out, double *vs_out);

/* Aggregate over views: mean of the top_k smallest view costs. */
double pmsref_aggregate(const double *view_costs, int n_views, int top_k);

/* --- whole-image cost of caller-given hypotheses --------------------------
   depth/normal are H*W and 3*H*W (planar nx, ny, nz). cost_out H*W receives
   the aggregated cost (2 at invalid pixels or depth <= 0); per_view_out,
   if non-null, n_views*H*W per-view costs. Returns 0 or a negative code. */
int pmsref_eval_cost(int W, int H, const double *ref, int n_views,
                     const double *const *nbrs, const pmsref_pose *ref_pose,
                     const pmsref_pose *nbr_poses, const pmsref_params *p,
                     const double *depth, const double *normal,
                     double *cost_out, double *per_view_out, int n_threads);

/* --- one red-black update of one pixel ------------------------------------
   State arrays are H*W depth, 3*H*W normal (planar), H*W cost. The update of
   pixel (x, y) in iteration `iteration` (1-based) reads only the state of
   opposite-colour pixels and of the pixel itself, and returns the new plane
   and cost in d_out, n_out, cost_out without writing the state. */
int pmsref_update_pixel(int W, int H, const double *ref, int n_views,
                        const double *const *nbrs, const pmsref_pose *ref_pose,
                        const pmsref_pose *nbr_poses, const pmsref_params *p,
                        const double *depth, const double *normal,
                        const double *cost, int iteration, int x, int y,
                        double *d_out, double n_out[3], double *cost_out);

/* One half-sweep (colour 0: even x+y, 1: odd) restricted to rows [y0, y1):
   the listed pixels' updates go to the *_out arrays, every other pixel is
   copied from the input state. */
int pmsref_halfsweep_rows(int W, int H, const double *ref, int n_views,
                          const double *const *nbrs, const pmsref_pose *ref_pose,
                          const pmsref_pose *nbr_poses, const pmsref_params *p,
                          const double *depth, const double *normal,
                          const double *cost, int iteration, int colour, int y0,
                          int y1, double *depth_out, double *normal_out,
                          double *cost_out, int n_threads);

/* --- decision-noise study hook (off by default) -----------------------------
   With amplitude a > 0, every matching cost that takes part in an accept
   decision -- the initial cost of a pixel and each propagation and
   refinement candidate's cost in a half-sweep -- has a deterministic
   pseudo-random offset, uniform in [-a, a] and keyed on (pixel, iteration,
   candidate slot), added before it is compared or stored (invalid costs of
   2 are left alone). It models an implementation whose cost evaluations
   carry independent rounding errors of up to a, so that the oracle's own
   sensitivity to such errors can be measured. a = 0, the default, leaves
   every result exactly as described above. Process-wide; set it only while
   no other call runs. */
void pmsref_set_decision_noise(double amplitude);

/* --- geometric consistency ------------------------------------------------
   Filters (depth, normal, cost) of the reference in place against n_maps
   depth maps of other keyframes. If err_px/err_depth/agree are non-null they
   receive, per map and pixel (n_maps*H*W), the reprojection error in pixels,
   the relative depth error and the 0/1 agreement (-1 where not evaluated). */
int pmsref_consistency(int W, int H, double *depth, double *normal,
                       double *cost, const pmsref_pose *ref_pose, int n_maps,
                       const double *const *maps, const pmsref_pose *map_poses,
                       const pmsref_params *p, double *err_px,
                       double *err_depth, int32_t *agree, int n_threads);

/* --- full densification ------------------------------------------------------
   Random initialisation, `iterations` red-black sweeps with propagation and
   random refinement, then (when n_maps > 0) geometric consistency. Outputs:
   depth H*W (0 = invalid), normal 3*H*W planar (0 = invalid), cost H*W
   (2 = invalid). init_depth/init_normal, when non-null, replace the random
   initial plane at every pixel whose init depth lies in the depth range and
   whose normal faces the camera. order_seed != 0 processes the pixels of each
   half-sweep in a seeded random order on one thread (the result must not
   depend on it). iterations_done_cb may be null. */
int pmsref_densify(int W, int H, const double *ref, int n_views,
                   const double *const *nbrs, const pmsref_pose *ref_pose,
                   const pmsref_pose *nbr_poses, const pmsref_params *p,
                   const double *init_depth, const double *init_normal,
                   int n_maps, const double *const *maps,
                   const pmsref_pose *map_poses, double *depth_out,
                   double *normal_out, double *cost_out, int n_threads,
                   uint64_t order_seed);

/* --- view filter (Sec. III-A, Eq. 1) ----------------------------------------
   Camera centres ca, cb (world) and n world points (3n doubles, seen by
   both keyframes). Counts the points whose angle between the directions to
   the two centres lies in [min_deg, max_deg] (in_range) among the points
   not at a centre (counted). Returns 1 to accept the keyframe (counted > 0
   and in_range >= min_frac * counted), 0 to reject, negative on error. */
int pmsref_view_filter(const double ca[3], const double cb[3], const double *points, long n,
                       double min_deg, double max_deg, double min_frac, long *in_range,
                       long *counted);

/* --- dense point-cloud fusion (Sec. III, point-cloud thread) ----------------
   Every pixel with depth > 0 of the n_maps W x H maps (camera poses[m]) is a
   world point; of the points in one cubic voxel of edge `voxel` (floor of
   each coordinate / voxel) the first in (map, pixel) order is kept:
   keep[m * H * W + pixel] = 1 (n_maps * H * W bytes), *n_kept = their count.
   Returns 0 or a negative code. */
int pmsref_fuse(int W, int H, int n_maps, const double *const *depths, const pmsref_pose *poses,
                double voxel, uint8_t *keep, long *n_kept);
/* Completeness: every kept point (keep may be null: all) marks the nearest
   pixel of a Wc x Hc equirectangular image at view_pose; cover (Wc*Hc
   bytes) receives the marks; returns the number of marked pixels. */
long pmsref_coverage(int W, int H, int n_maps, const double *const *depths,
                     const pmsref_pose *poses, const uint8_t *keep, const pmsref_pose *view_pose,
                     int Wc, int Hc, uint8_t *cover);

/* --- median post-filter (Sec. III-C, item 2) -------------------------------
   A median-filtered copy of the depth map is compared with the map: where a
   valid depth deviates from the median of the valid depths in its
   (2 median_radius + 1)^2 window (longitude wrapping, rows beyond the image
   left out; the lower median for an even count) by more than median_rel
   times that median, the pixel is removed (depth 0, normal 0, cost 2).
   Decisions use the unfiltered map only. No-op for median_radius 0. */
int pmsref_median_filter(int W, int H, double *depth, double *normal, double *cost,
                         const pmsref_params *p);

/* --- plane-map warping (Sec. III-B) ------------------------------------------
   Carries the plane map (src_depth H*W, 0 = none; src_normal 3*H*W planar)
   of the keyframe at src_pose into the keyframe at dst_pose: each valid
   source pixel claims the destination pixel nearest to the projection of its
   plane point, the nearest claim wins (float range, then lower source
   index), and its plane (rotated normal) is re-intersected with the
   destination pixel's ray. Outputs dst_depth (0 = no plane) and dst_normal
   (0 = none); only depths in [depth_min, depth_max] with the normal facing
   the destination camera are kept. Returns 0 or a negative code. */
int pmsref_warp_planes(int W, int H, const double *src_depth, const double *src_normal,
                       const pmsref_pose *src_pose, const pmsref_pose *dst_pose,
                       const pmsref_params *p, double *dst_depth, double *dst_normal);

/* Pixels per row-band for which pmsref_update_pixel is defined (valid rows). */
int pmsref_pixel_valid(int W, int H, const pmsref_params *p, int x, int y);

#ifdef __cplusplus
}
#endif
#endif
