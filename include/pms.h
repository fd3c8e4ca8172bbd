/*
 * pms.h -- C ABI of libpms, the gfx950 (MI355X) implementation of
 * equirectangular PatchMatch-Stereo densification after Surmann, Thurow,
 * Slomma, "PatchMatch-Stereo-Panorama, a fast dense reconstruction from 360
 * degree video images" (Sec. III, "Proposed method").
 *
 * The problem statement (Sec. III, first paragraph): a keyframe and its
 * neighbouring keyframes, each an equirectangular 360 degree image with a
 * 6-DoF pose from SLAM, are turned into a dense 360 degree depth image on the
 * GPU; once depth maps of further keyframes exist, a consistency filter
 * removes outliers (Sec. III, paragraph on the densification thread).
 *
 * Conventions shared by every call
 * --------------------------------
 * Images:  W x H with W == 2H, H <= PMS_MAX_HEIGHT, row-major, one
 *          channel, pitch in bytes.
 *          float32, float16 or uint8 (uint8 is scaled by 1/255; the NCC
 *          variance floor applies to the scaled values). All images of one
 *          call have the same W and H.
 * Camera:  equirectangular, pixel centres on integer coordinates:
 *            longitude lam = 2 pi (x + 0.5)/W - pi,
 *            latitude  phi = pi/2 - pi (y + 0.5)/H,
 *            bearing   b   = (cos phi sin lam, -sin phi, cos phi cos lam)
 *          in a frame with x right, y down, z forward.
 * Poses:   world -> camera, X_cam = R X_world + t, R row-major, double.
 *          Relative poses are composed in double on the host, once per
 *          keyframe pair, and rounded to float for the kernels.
 * Planes:  per pixel, depth = range along the unit ray in metres (0 marks
 *          an invalid pixel), normal = unit vector in the reference camera
 *          frame facing the camera (0 when invalid), cost = aggregated
 *          1 - NCC in [0, 2] (2 when invalid). Each is a separate float32
 *          H x W plane with its own pitch in elements.
 * Valid pixels: rows r <= y <= H-1-r for patch radius r; every column (the
 *          longitude wraps around the seam). Other rows are written invalid.
 * Pointers: image, plane and output pointers are DEVICE pointers the caller
 *          owns (e.g. from PyTorch); pose and parameter structs are HOST
 *          memory read before the call returns. Inputs must stay alive until
 *          the stream reaches the enqueued work.
 * Streams: `stream` is a hipStream_t (0 = the null stream). Every call only
 *          enqueues work on it and returns; the caller synchronises.
 * Errors:  every call validates all arguments on the host before it enqueues
 *          anything; on any error nothing is written. PMS_ERR_DEVICE carries
 *          the HIP error text in pms_last_error(). A context is not
 *          thread-safe: use one per stream.
 */
#ifndef PMS_H
#define PMS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PMS_OK = 0,
    PMS_ERR_INVALID_ARG = 1,
    PMS_ERR_OUT_OF_MEMORY = 2,
    PMS_ERR_DEVICE = 3,
    PMS_ERR_UNSUPPORTED = 4,
    PMS_ERR_BUDGET = 5
} pms_status;

typedef enum { PMS_F32 = 0, PMS_F16 = 1, PMS_U8 = 2 } pms_dtype;

#define PMS_MAX_VIEWS 8      /* neighbours per call                        */
#define PMS_MAX_MAPS 8       /* consistency depth maps per call            */
#define PMS_MAX_OFFSETS 16   /* propagation neighbourhood                  */
#define PMS_MAX_SAMPLES 64   /* samples per patch                          */
#define PMS_MAX_TRIALS 16    /* refinement trials per pixel and sweep      */
#define PMS_MAX_BATCH 256    /* jobs per batch                             */
#define PMS_MAX_TOP_K 4      /* views averaged (top_k, or ceil(N/2))       */
#define PMS_MAX_HEIGHT 5791  /* image rows: a neighbour's re-laid-out copy,
                                (H + 1) x (2W + 4) cells of 16 bytes, stays
                                under 2 GiB (32-bit byte offsets)          */

typedef struct {
    const void *data;    /* device pointer                                 */
    int32_t width;       /* W == 2 * height                                */
    int32_t height;
    int64_t pitch_bytes; /* >= width * element size                        */
    int32_t dtype;       /* pms_dtype                                      */
} pms_image;

typedef struct {
    float *data;         /* device pointer to an H x W float32 plane       */
    int64_t pitch_elems; /* >= W                                           */
} pms_plane;

typedef struct {
    double R[9]; /* world -> camera rotation, row-major                    */
    double t[3]; /* world -> camera translation                            */
} pms_pose;

typedef struct {
    int32_t patch_size;    /* odd >= 3; patch radius r = (patch_size-1)/2   */
    int32_t patch_stride;  /* s >= 1 dividing 2r; samples at -r, -r+s, ..., r
                              in x and y (row-major), at most 64 samples   */
    int32_t iterations;    /* red + black sweeps                            */
    int32_t refine_trials; /* random refinement trials per pixel per sweep */
    double depth_min;      /* 0 < depth_min < depth_max, metres            */
    double depth_max;
    int32_t top_k;         /* views averaged; 0 => ceil(N/2); at most
                              PMS_MAX_TOP_K (PMS_ERR_UNSUPPORTED above)     */
    double ncc_var_floor;  /* a view whose patch variance is below this is
                              invalid (cost 2)                              */
    double refine_sigma_logdepth0; /* <= 0 => 0.5 ln(depth_max/depth_min)   */
    double refine_depth_shrink;    /* log-depth half-width factor per trial */
    double refine_sigma_normal0;   /* normal perturbation half-width        */
    double refine_normal_shrink;   /* its factor per trial                  */
    int32_t n_offsets;             /* propagation neighbours, table order  */
    int32_t offsets[PMS_MAX_OFFSETS][2]; /* (dx, dy) with odd |dx| + |dy|  */
    double geo_px;        /* consistency: reprojection error bound, pixels */
    double geo_rel_depth; /* consistency: relative range error bound       */
    int32_t geo_min_views; /* maps that must agree; 0 => min(2, #maps)     */
    uint64_t seed;        /* key of the counter-based RNG                   */
    int32_t median_radius; /* median post-filter (Sec. III-C item 2): window
                              (2r+1)^2, 0..8; 0 = off (default)             */
    double median_rel;     /* removes depths deviating from the window's
                              median by more than this fraction (0.05)      */
} pms_params;

typedef struct pms_context pms_context;

/* One keyframe densification job: the arguments of pms_densify gathered in
   one struct (same meaning, same rules). The arrays it points to are host
   memory read before the call that takes the job returns. */
typedef struct {
    pms_image ref;
    pms_pose ref_pose;
    const pms_image *nbrs;      /* n_nbrs images of ref's size and dtype     */
    const pms_pose *nbr_poses;
    int32_t n_nbrs;             /* 1 .. PMS_MAX_VIEWS                        */
    const pms_plane *maps;      /* consistency maps; null when n_maps == 0   */
    const pms_pose *map_poses;
    int32_t n_maps;             /* 0 .. PMS_MAX_MAPS                         */
    const pms_params *params;
    pms_plane depth_out;
    pms_plane normal_out[3];
    pms_plane cost_out;
    /* Optional initial planes (Sec. III-B, plane-map warping: typically
       pms_warp_planes of the previous keyframe's result). init_depth.data
       == NULL means a random initialisation everywhere; otherwise the four
       planes share one pitch, and at every valid pixel whose init depth lies
       in [depth_min, depth_max] and whose normal faces the camera the
       supplied plane replaces the random one. */
    pms_plane init_depth;
    pms_plane init_normal[3];
} pms_job;

/* Launch schedule of a context: the tile one 256-thread workgroup serves and
   the lanes that share one pixel. A wave of 64 lanes holds 64 /
   lanes_per_pixel pixels as wave_rows rows; a workgroup holds waves_x x
   (4 / waves_x) waves. The tile shape never changes a result;
   lanes_per_pixel (2, 4 or 8; 2 is used for 36-sample patches only, 8 for
   64-sample patches only, 4 for every other patch) changes the order of
   the patch sums and therefore the last bits of the costs. */
typedef struct {
    int32_t wave_rows;       /* 1, 2, 4, 8 or 16; default 4 */
    int32_t waves_x;         /* 1, 2 or 4; default 2        */
    int32_t lanes_per_pixel; /* 2, 4 or 8; default 4        */
} pms_schedule;

typedef struct pms_batch pms_batch;
typedef struct pms_server pms_server;

/* Defaults: 11x11 patch sampled every 2nd pixel, 8 iterations, 6 refinement
   trials (Sec. III-C, item 1), 0.3-30 m, the 8-neighbourhood of Sec. III-C
   with its inner ring moved out to distance 3 and the outer ring at 5, 1 px /
   1% consistency. Never fails for a non-null pointer. */
pms_status pms_default_params(pms_params *out);

/* Creates a context on HIP device `device`. The context owns only scratch
   memory (plane state, reference patch statistics, re-laid-out neighbour
   images, argument tables: one block sized on first use and grown when a
   call needs more, never above scratch_budget_bytes, 0 = no limit; plus the
   bearing tables of each image size it has seen). device == -1
   makes a validation-only context: every call checks its arguments as usual
   and then returns PMS_ERR_DEVICE instead of launching (no GPU needed). */
pms_status pms_context_create(int32_t device, size_t scratch_budget_bytes, pms_context **out);
pms_status pms_context_destroy(pms_context *ctx);

/* Densifies one reference keyframe (Sec. III and III-B/C):
   random initialisation, `iterations` red-black sweeps of propagation and
   random refinement scored by the plane-induced warp and NCC against
   n_nbrs neighbours, the median post-filter when median_radius > 0 (a
   valid depth is removed if it deviates from the lower median of the valid
   depths of its window -- longitude wrapping, rows beyond the image left
   out -- by more than median_rel times that median; decided on the
   unfiltered map), and -- when n_maps > 0 -- the geometric-consistency
   filter against the depth maps of n_maps other keyframes (maps[k] is a
   W x H plane of ranges, 0 = no depth, for the camera at map_poses[k]).
   Writes depth_out, normal_out[0..2] (nx, ny, nz) and cost_out. */
pms_status pms_densify(pms_context *ctx, const pms_image *ref, const pms_pose *ref_pose,
                       const pms_image *nbrs, const pms_pose *nbr_poses, int32_t n_nbrs,
                       const pms_plane *maps, const pms_pose *map_poses, int32_t n_maps,
                       const pms_params *params, pms_plane depth_out,
                       const pms_plane normal_out[3], pms_plane cost_out, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
   capture, tight serving loops, harnesses that forbid hipMalloc): the same
   arguments, validation and results as pms_densify, but the call's working
   memory -- bearing tables, argument tables, plane state, patch statistics
   and the re-laid-out neighbour images -- lives in a fixed scratch array of
   PMS_NOALLOC_SCRATCH_BYTES compiled into the library. Each GPU the library
   runs on holds its own copy until the process ends; its address is looked
   up once per device by pms_context_create. The call makes no device or
   pinned-host allocation (no hipMalloc, hipFree, hipHostMalloc or stream-
   ordered allocation) and records no profiling events; it uploads its
   tables with one copy from a pageable host buffer of the context, and only
   the host-side plan bookkeeping uses ordinary heap containers.
   Limit: returns PMS_ERR_BUDGET, enqueuing nothing, when the call needs
   more than PMS_NOALLOC_SCRATCH_BYTES (about 24 B x (W + H) of tables plus
   28 B per pixel of state plus the neighbour copies: e.g. 960 x 480 with up
   to 6 neighbours fits). Every call on one GPU shares that GPU's array and
   leaves its contents behind (nothing in it needs clearing: each call
   writes every scratch word it reads): calls that can run at the same time
   on one GPU -- on different streams, or from different contexts or
   threads without ordering -- race and give undefined results; calls
   enqueued on one stream are ordered and safe. */
#define PMS_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)
pms_status pms_densify_noalloc(pms_context *ctx, const pms_image *ref, const pms_pose *ref_pose,
                               const pms_image *nbrs, const pms_pose *nbr_poses, int32_t n_nbrs,
                               const pms_plane *maps, const pms_pose *map_poses, int32_t n_maps,
                               const pms_params *params, pms_plane depth_out,
                               const pms_plane normal_out[3], pms_plane cost_out, void *stream);

/* Densifies n_jobs (1 .. PMS_MAX_BATCH) keyframes of any mix of sizes,
   neighbour counts and parameters together: every step of the method runs
   as one launch over the tiles of all jobs still at that step, so small
   keyframes share the GPU instead of under-filling it. Each job's outputs
   are bitwise those of pms_densify on that job alone with the same context
   schedule. No output plane may be shared by two jobs or be a consistency
   map of the batch. Neighbour images that appear in several jobs (same
   pointer, size, pitch and dtype) are re-laid out once. */
pms_status pms_densify_batch(pms_context *ctx, const pms_job *jobs, int32_t n_jobs,
                             void *stream);

/* A batch prepared once and run many times: pms_batch_create validates the
   jobs, allocates the batch's own device memory (plane state for every job,
   re-laid-out images, argument tables) and uploads the tables; the images
   and output planes are referenced, not copied, and must stay valid until
   pms_batch_destroy (their contents may change between runs).
   pms_batch_run only enqueues kernels on `stream`; with use_graph != 0 the
   whole batch is captured into a HIP graph on its first run and every run
   is one graph launch. pms_batch_destroy waits for the device. */
pms_status pms_batch_create(pms_context *ctx, const pms_job *jobs, int32_t n_jobs,
                            pms_batch **out);
pms_status pms_batch_run(pms_batch *batch, int32_t use_graph, void *stream);
pms_status pms_batch_bytes(const pms_batch *batch, size_t *bytes);
pms_status pms_batch_destroy(pms_batch *batch);

/* Schedule of a context (applies to every later call on it). */
pms_status pms_get_schedule(const pms_context *ctx, pms_schedule *out);
pms_status pms_set_schedule(pms_context *ctx, const pms_schedule *s);

/* Autotuner: densifies the jobs (as one batch) under every tile shape (and,
   with try_lanes != 0, every lanes_per_pixel value), timing the
   initialisation and half-sweep kernels over `reps` runs after one warm-up,
   and leaves the fastest schedule set on the context. Synchronous; the
   jobs' output planes receive the last run's results. */
pms_status pms_autotune(pms_context *ctx, const pms_job *jobs, int32_t n_jobs, int32_t reps,
                        int32_t try_lanes, pms_schedule *best_out, double *best_ms_out,
                        void *stream);

/* Serving loop with continuous batching. A server owns one device arena of
   arena_bytes (allocated once, at create) from which every admitted job
   takes its plane state and the re-laid-out copies of its neighbour images
   (shared, reference-counted, between jobs that name the same image).
   pms_server_submit validates a job, copies its host-side description and
   queues it (PMS_ERR_BUDGET if the job alone could never fit the arena);
   its device buffers must stay valid, and its images unchanged, until the
   job is done. Each pms_server_step is one tick on `stream`: waiting jobs
   are admitted in submission order while their memory fits and fewer than
   max_jobs run, then every running job advances by one half-sweep -- newly
   admitted ones are laid out, get their patch statistics and random
   initialisation first; the ones that complete their sweeps write their
   outputs and run the consistency filter -- with one launch per step kind
   and kernel variant over all jobs. A job's results are bitwise those of
   pms_densify on it alone (same context schedule). At most two ticks are
   in flight: a step waits for the tick before the previous one. Use one
   stream per server; consistency maps must be final when their job is
   submitted. */
pms_status pms_server_create(pms_context *ctx, size_t arena_bytes, int32_t max_jobs,
                             pms_server **out);
pms_status pms_server_submit(pms_server *server, const pms_job *job, int64_t *ticket);
pms_status pms_server_step(pms_server *server, void *stream, int32_t *active_out,
                           int32_t *waiting_out);
/* state: 0 waiting, 1 running (or enqueued but not finished on the device),
   2 done -- reported once; the ticket is then forgotten. */
pms_status pms_server_poll(pms_server *server, int64_t ticket, int32_t *state);
/* Ticks run, the sum over ticks of running jobs (mean occupancy =
   job_ticks / ticks), and the arena bytes in use now and at most. */
pms_status pms_server_stats(const pms_server *server, int64_t *ticks, int64_t *job_ticks,
                            size_t *arena_used, size_t *arena_peak);
pms_status pms_server_destroy(pms_server *server);

/* The matching cost alone (Sec. III-C: rectangular reference patch, any
   shape in the neighbours) for caller-given hypotheses: cost_out receives the
   aggregated cost at every pixel (2 where the pixel is invalid or depth <= 0);
   per_view_out, if non-null, points to n_nbrs planes of per-view costs. */
pms_status pms_eval_cost(pms_context *ctx, const pms_image *ref, const pms_pose *ref_pose,
                         const pms_image *nbrs, const pms_pose *nbr_poses, int32_t n_nbrs,
                         const pms_params *params, pms_plane depth_in,
                         const pms_plane normal_in[3], pms_plane cost_out,
                         const pms_plane *per_view_out, void *stream);

/* One half-sweep of Sec. III-C (propagation from the opposite colour, then
   random refinement) on a caller-held state: colour 0 updates pixels with
   even x + y, colour 1 odd; `iteration` (>= 1) keys the refinement draws.
   The state planes are read and written in place. */
pms_status pms_halfsweep(pms_context *ctx, const pms_image *ref, const pms_pose *ref_pose,
                         const pms_image *nbrs, const pms_pose *nbr_poses, int32_t n_nbrs,
                         const pms_params *params, int32_t iteration, int32_t colour,
                         pms_plane depth_io, const pms_plane normal_io[3], pms_plane cost_io,
                         void *stream);

/* The geometric-consistency filter alone (Sec. III: it runs as soon as a
   window of five keyframes has depth maps) on a caller-held W x H result,
   in place. */
pms_status pms_consistency(pms_context *ctx, int32_t width, int32_t height,
                           const pms_pose *ref_pose, const pms_plane *maps,
                           const pms_pose *map_poses, int32_t n_maps, const pms_params *params,
                           pms_plane depth_io, const pms_plane normal_io[3], pms_plane cost_io,
                           void *stream);

/* Plane-map warping (Sec. III-B: the optimised plane map of the preceding
   keyframe initialises the current one). Every valid pixel of the source
   map (src_depth > 0, rows r .. H-1-r) carries its plane point into the
   destination camera (relative pose composed in FP64) and claims the
   destination pixel nearest to its projection; of several claims the
   nearest point wins (its range rounded to float, ties to the lower source
   pixel index, so the result does not depend on scheduling). The winning
   plane -- normal rotated into the destination frame, through the moved
   point -- is re-intersected with the destination pixel's own ray and kept
   if it faces the camera with a depth in [depth_min, depth_max]. Writes
   dst_depth (0 where no plane arrives) and dst_normal (0 there). Both maps
   are width x height (width == 2 height); src and dst planes must not
   overlap. Uses 8 bytes per pixel of context scratch. */
pms_status pms_warp_planes(pms_context *ctx, int32_t width, int32_t height,
                           const pms_pose *src_pose, pms_plane src_depth,
                           const pms_plane src_normal[3], const pms_pose *dst_pose,
                           const pms_params *params, pms_plane dst_depth,
                           const pms_plane dst_normal[3], void *stream);

/* View filter (Sec. III-A, Eq. 1): for n_points sparse world points
   (device memory, 3 doubles each, points seen by both keyframes) counts
   those whose angle between the directions to the two camera centres
   centre_a and centre_b (world, host) lies in [min_deg, max_deg]
   (counts_out[0]) and those not at a centre (counts_out[1]); counts_out is
   two uint64 in device memory, overwritten. The keyframe is accepted when
   counts_out[0] >= 0.2 counts_out[1] (the paper's 20%, 6 and 60 degrees).
   Angles in FP64. Uses 16 KB of context scratch (spread counters). */
pms_status pms_view_filter(pms_context *ctx, const double centre_a[3], const double centre_b[3],
                           const double *points, int64_t n_points, double min_deg,
                           double max_deg, uint64_t *counts_out, void *stream);

/* Dense point-cloud fusion (Sec. III: the point-cloud thread buffers four
   consistent keyframes and erases duplicate points). Every pixel with depth
   > 0 of the n_maps (1 .. PMS_MAX_MAPS) width x height depth planes, taken
   at poses[m], is a world point; of the points in one cubic voxel of edge
   `voxel` metres (floor of each world coordinate / voxel) the first in
   (map, pixel) order is kept. Writes keep_out[m * H * W + y * W + x] = 1
   for kept points, else 0 (device, n_maps * H * W bytes) and the number of
   kept points to n_kept_out (device uint64). Points more than 2^20 voxels
   from the first map's camera centre along an axis are not kept (with
   depths up to depth_max around nearby cameras this needs voxel <
   depth_max / 2^20, i.e. 0.05 mm at 50 m); world coordinates themselves may
   be anywhere. Uses context scratch: a hash table of 16-byte slots, the
   power of two at or above 5/4 n_maps W H, 4 bytes per point and 16 KB of
   spread counters; a table
   above 2^31 slots is rejected (PMS_ERR_INVALID_ARG). The result does not
   depend on scheduling. */
pms_status pms_fuse(pms_context *ctx, int32_t width, int32_t height, int32_t n_maps,
                    const pms_plane *depths, const pms_pose *poses, double voxel,
                    uint8_t *keep_out, uint64_t *n_kept_out, void *stream);

/* Completeness of fused points seen from one camera (the paper renders
   depth panoramas of the cloud at 720 x 360): every point of the maps (as
   in pms_fuse) whose keep byte is set (keep == NULL: every point) marks the
   pixel of an out_width x out_height equirectangular image at view_pose
   nearest to its projection. Writes cover_out (device, out_width *
   out_height bytes, 1 = marked) and the number of marked pixels to
   n_covered_out (device uint64). Uses 16 KB of context scratch (spread
   counters). */
pms_status pms_coverage(pms_context *ctx, int32_t width, int32_t height, int32_t n_maps,
                        const pms_plane *depths, const pms_pose *poses, const uint8_t *keep,
                        const pms_pose *view_pose, int32_t out_width, int32_t out_height,
                        uint8_t *cover_out, uint64_t *n_covered_out, void *stream);

/* Philox4x64-10 blocks for counters (ctr0 + i, 0, 0, 0), i < n, with key
   (key0, key1), written to the device buffer out[4n] -- the generator the
   kernels draw hypotheses from, exposed for testing. */
pms_status pms_philox_stream(pms_context *ctx, uint64_t key0, uint64_t key1, uint64_t ctr0,
                             int64_t n, uint64_t *out, void *stream);

/* Per-kernel timing with HIP events around each launch (off by default).
   pms_profile_read synchronises on the recorded events, returns the launch
   count and total milliseconds of kernel `name` ("halfsweep", "init",
   "refstats", "finalize", "consistency", "eval", "io" for the image
   re-layout and state copies, "batch" for whole graph launches, "median",
   and one entry per call of the calls beside densification: "warp",
   "fuse", "coverage", "view_filter") since the last read, and clears them.
   A graph launch is timed as one "batch". */
pms_status pms_profile_enable(pms_context *ctx, int32_t on);

/* Executed-work counters of the half-sweeps (Sec. III-C: propagation and
   refinement), for measuring throughput against the work actually done.
   While enabled, every half-sweep launch of the context runs a variant that
   counts, per pixel update, the candidates it considers, skips and scores
   and the (pixel, candidate, view) NCC evaluations it executes, and adds
   them to device counters (one atomic per counter and workgroup). Results
   are bit for bit those of the uncounted kernels. pms_work_count_enable
   allocates the counters on first use (zeroed); pms_work_count_read
   synchronises the device, copies the totals since the last reset into
   *out (all zero if never enabled) and zeroes them when reset != 0.
   Invariants: prop_candidates + refine_trials = skipped_geometry +
   skipped_repeat + scored; view_evals + views_pruned = n_views x (scored -
   facing_rejects) for a job with n_views neighbours. */
#define PMS_WORK_FIELDS 9
typedef struct {
    int64_t pixels;           /* pixel updates                                */
    int64_t prop_candidates;  /* propagation offsets considered             */
    int64_t refine_trials;    /* refinement trials considered                */
    int64_t skipped_geometry; /* dropped unscored: neighbour outside the band
                                 or invalid, plane behind the ray or depth out
                                 of range, refined normal not facing          */
    int64_t skipped_repeat;   /* propagation candidates equal to the current
                                 plane or the previous candidate             */
    int64_t scored;           /* candidates whose cost was evaluated          */
    int64_t facing_rejects;   /* scored planes not facing every sample ray   */
    int64_t view_evals;       /* NCC evaluations executed (P samples each)   */
    int64_t views_pruned;     /* views skipped by the top-k bound            */
} pms_work_counts;
pms_status pms_work_count_enable(pms_context *ctx, int32_t on);
pms_status pms_work_count_read(pms_context *ctx, pms_work_counts *out, int32_t reset);
pms_status pms_profile_read(pms_context *ctx, const char *name, int64_t *launches,
                            double *total_ms);

const char *pms_status_string(pms_status s);
/* Text of the last error on this context ("" if none); valid until the next
   call on the context. */
const char *pms_last_error(const pms_context *ctx);

#ifdef __cplusplus
}
#endif
#endif
