/*
 * pmsref.c -- plain FP64 CPU reference ("the oracle") of equirectangular
 * PatchMatch-Stereo densification, after Surmann et al., Sec. III
 * ("Proposed method"), subsections B (Initialisation) and C (Parallel 360
 * degree PatchMatch).
 *
 * TEST INFRASTRUCTURE. Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark load this library; the GPU library shares
 * no source with it.
 *
 * The paper is a systems paper: beyond the view-filter equation it prints no
 * formula for the densifier. Every step below is written from the method it
 * names (PatchMatch stereo with slanted plane hypotheses, red-black parallel
 * propagation after Galliani et al., random refinement with a shrinking
 * search range) and from the readings listed at each function where the
 * paper is silent. The code is deliberately slow and direct: every sample
 * recomputes its bearing with sin/cos, NCC is two-pass, sorting is insertion
 * sort. Threads only split the pixels of one half-sweep, whose updates are
 * independent by construction (each pixel reads only opposite-colour pixels
 * and itself), so the result does not depend on the thread count or order.
 *
 * Parity pins (tests/test_oracle_*.py):
 *   camera model       closed forms, round trip, poles, seam      pinned
 *   bilinear sample    torch grid_sample on a wrap-padded copy    pinned
 *   relative pose      transform of explicit points               pinned
 *   plane warp         analytic plane/point, t=0, yaw-only shift  pinned
 *   NCC                affine identities, numpy.corrcoef          pinned
 *   aggregation        N=2 -> min, view permutation invariance    pinned
 *   Philox4x64-10      numpy.random.Philox bit stream             pinned
 *   random plane       distribution moments, facing constraint    pinned
 *   propagation/refine brute-force plane sweep on a textured
 *                      sphere, ground truth of rendered scenes,
 *                      pixel-order invariance                     pinned
 *   refinement widths, neighbourhood table, top-k rule,
 *   consistency vote count                                        parity
 *                      unpinned against the paper (it prints no values)
 *   consistency        ground-truth maps kept, scaled maps
 *                      dropped, closed-form reprojection error    pinned
 */
#include "pmsref.h"

#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

static const double PI = 3.14159265358979323846;

/* ------------------------------------------------------------------------ */
/* parameters                                                               */
/* ------------------------------------------------------------------------ */

void pmsref_default_params(pmsref_params *p)
{
    static const int32_t nb[8][2] = {{-3, 0}, {3, 0}, {0, -3}, {0, 3},
                                     {-5, 0}, {5, 0}, {0, -5}, {0, 5}};
    memset(p, 0, sizeof *p);
    p->patch_size = 11;
    p->patch_stride = 2;
    p->iterations = 8;
    p->refine_trials = 6; /* Sec. III-C item 1: six random hypothesis tests */
    p->depth_min = 0.3;
    p->depth_max = 30.0;
    p->top_k = 0;
    p->ncc_var_floor = 1e-6;
    p->refine_sigma_logdepth0 = 0.0;
    p->refine_depth_shrink = 0.25;
    p->refine_sigma_normal0 = 1.0;
    p->refine_normal_shrink = 0.5;
    /* Sec. III-C: 8-neighbourhood of the red-black scheme with the inner ring
       moved outwards. An offset must keep the opposite colour, i.e. have odd
       |dx|+|dy|, so the inner ring moves from distance 1 to distance 3 and
       the outer ring stays at distance 5. */
    p->n_offsets = 8;
    memcpy(p->offsets, nb, sizeof nb);
    p->geo_px = 1.0;
    p->geo_rel_depth = 0.01;
    p->geo_min_views = 0;
    p->seed = 0;
    p->median_radius = 0;
    p->median_rel = 0.05;
}

static int patch_radius(const pmsref_params *p) { return (p->patch_size - 1) / 2; }

int pmsref_patch_offsets(const pmsref_params *p, int32_t *dx, int32_t *dy)
{
    int r = patch_radius(p), s = p->patch_stride, n = 0;
    for (int oy = -r; oy <= r; oy += s)
        for (int ox = -r; ox <= r; ox += s) {
            if (dx) dx[n] = ox;
            if (dy) dy[n] = oy;
            ++n;
        }
    return n;
}

int pmsref_check_params(const pmsref_params *p, int W, int H, int n_views)
{
    if (!p) return -1;
    if (H < 1 || W != 2 * H) return -2;
    if (n_views < 0 || n_views > PMSREF_MAX_VIEWS) return -3;
    if (p->patch_size < 3 || p->patch_size % 2 == 0) return -4;
    if (p->patch_stride < 1 || (p->patch_size - 1) % p->patch_stride != 0) return -5;
    if (pmsref_patch_offsets(p, NULL, NULL) > PMSREF_MAX_SAMPLES) return -6;
    if (p->iterations < 0 || p->refine_trials < 0 || p->refine_trials > 16) return -7;
    if (!(p->depth_min > 0.0) || !(p->depth_max > p->depth_min) || !isfinite(p->depth_max))
        return -8;
    if (p->top_k < 0 || p->top_k > n_views) return -9;
    if (!(p->ncc_var_floor >= 0.0) || !isfinite(p->ncc_var_floor)) return -10;
    if (!isfinite(p->refine_sigma_logdepth0) || !(p->refine_depth_shrink > 0.0) ||
        !isfinite(p->refine_depth_shrink) || !(p->refine_sigma_normal0 >= 0.0) ||
        !isfinite(p->refine_sigma_normal0) || !(p->refine_normal_shrink > 0.0) ||
        !isfinite(p->refine_normal_shrink))
        return -11;
    if (p->n_offsets < 0 || p->n_offsets > PMSREF_MAX_OFFSETS) return -12;
    for (int k = 0; k < p->n_offsets; ++k) {
        int ox = p->offsets[k][0], oy = p->offsets[k][1];
        if (((ox < 0 ? -ox : ox) + (oy < 0 ? -oy : oy)) % 2 != 1) return -13;
        if (oy <= -H || oy >= H || ox <= -W || ox >= W) return -13;
    }
    if (!(p->geo_px >= 0.0) || !(p->geo_rel_depth >= 0.0) || p->geo_min_views < 0) return -14;
    if (p->median_radius < 0 || p->median_radius > 8 || !(p->median_rel >= 0.0) || !isfinite(p->median_rel))
        return -15;
    return 0;
}

int pmsref_pixel_valid(int W, int H, const pmsref_params *p, int x, int y)
{
    int r = patch_radius(p);
    return x >= 0 && x < W && y >= r && y <= H - 1 - r;
}

/* ------------------------------------------------------------------------ */
/* camera model (Sec. III-C: the rectangular reference patch takes any      */
/* shape in the neighbours because of the equirectangular projection)       */
/* ------------------------------------------------------------------------ */

void pmsref_unproject(int W, int H, double x, double y, double b[3])
{
    double lam = 2.0 * PI * (x + 0.5) / W - PI;
    double phi = PI / 2.0 - PI * (y + 0.5) / H;
    b[0] = cos(phi) * sin(lam);
    b[1] = -sin(phi);
    b[2] = cos(phi) * cos(lam);
}

void pmsref_project(int W, int H, const double Y[3], double *x, double *y)
{
    double lam = atan2(Y[0], Y[2]);
    double phi = atan2(-Y[1], hypot(Y[0], Y[2]));
    *x = W * (lam + PI) / (2.0 * PI) - 0.5;
    *y = H * (PI / 2.0 - phi) / PI - 0.5;
}

static int wrap_index(double fx, int W)
{
    double m = fx - W * floor(fx / W);
    int i = (int)m;
    if (i >= W) i -= W; /* m can round up to W */
    if (i < 0) i += W;
    return i;
}

static int clamp_index(double fy, int H)
{
    if (fy < 0.0) return 0;
    if (fy > H - 1) return H - 1;
    return (int)fy;
}

/* Bilinear interpolation with the longitude wrapping around the seam and the
   latitude clamped at the poles (no cross-pole wrap). */
double pmsref_sample(const double *img, int W, int H, double x, double y)
{
    double fx = floor(x), fy = floor(y);
    double ax = x - fx, ay = y - fy;
    int x0 = wrap_index(fx, W), x1 = wrap_index(fx + 1.0, W);
    int y0 = clamp_index(fy, H), y1 = clamp_index(fy + 1.0, H);
    double top = (1.0 - ax) * img[(size_t)y0 * W + x0] + ax * img[(size_t)y0 * W + x1];
    double bot = (1.0 - ax) * img[(size_t)y1 * W + x0] + ax * img[(size_t)y1 * W + x1];
    return (1.0 - ay) * top + ay * bot;
}

/* ------------------------------------------------------------------------ */
/* poses (Sec. III: keyframe poses come from the SLAM thread)               */
/* ------------------------------------------------------------------------ */

void pmsref_relative_pose(const pmsref_pose *ref, const pmsref_pose *nbr, double R[9],
                          double t[3])
{
    /* X_ref = R_r X_w + t_r and X_nbr = R_n X_w + t_n give
       X_nbr = (R_n R_r^T) X_ref + (t_n - R_n R_r^T t_r). */
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = 0.0;
            for (int k = 0; k < 3; ++k) s += nbr->R[3 * i + k] * ref->R[3 * j + k];
            R[3 * i + j] = s;
        }
    for (int i = 0; i < 3; ++i) {
        double s = 0.0;
        for (int k = 0; k < 3; ++k) s += R[3 * i + k] * ref->t[k];
        t[i] = nbr->t[i] - s;
    }
}

/* ------------------------------------------------------------------------ */
/* Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two     */
/* 64x64->128 multiplications with a Weyl-sequence key schedule.            */
/* ------------------------------------------------------------------------ */

static uint64_t mul_hi_lo(uint64_t a, uint64_t b, uint64_t *hi)
{
    unsigned __int128 prod = (unsigned __int128)a * b;
    *hi = (uint64_t)(prod >> 64);
    return (uint64_t)prod;
}

void pmsref_philox4x64_10(uint64_t key0, uint64_t key1, const uint64_t ctr[4], uint64_t out[4])
{
    uint64_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    for (int round = 0; round < 10; ++round) {
        uint64_t hi0, hi1;
        uint64_t lo0 = mul_hi_lo(0xD2E7470EE14C6C93ULL, c0, &hi0);
        uint64_t lo1 = mul_hi_lo(0xCA5A826395121157ULL, c2, &hi1);
        uint64_t n0 = hi1 ^ c1 ^ key0;
        uint64_t n2 = hi0 ^ c3 ^ key1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        key0 += 0x9E3779B97F4A7C15ULL;
        key1 += 0xBB67AE8584CAA73BULL;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

void pmsref_philox4x64_10_stream(uint64_t key0, uint64_t key1, uint64_t ctr0, long n,
                                 uint64_t *out)
{
    for (long i = 0; i < n; ++i) {
        uint64_t ctr[4] = {ctr0 + (uint64_t)i, 0, 0, 0};
        pmsref_philox4x64_10(key0, key1, ctr, out + 4 * i);
    }
}

void pmsref_uniforms(uint64_t seed, uint64_t pixel, uint64_t iteration, uint64_t stage,
                     double u[4])
{
    uint64_t ctr[4] = {pixel, iteration, stage, 0}, w[4];
    pmsref_philox4x64_10(seed, 0, ctr, w);
    for (int i = 0; i < 4; ++i) u[i] = (double)(w[i] >> 40) * (1.0 / 16777216.0);
}

/* ------------------------------------------------------------------------ */
/* matching cost                                                            */
/* ------------------------------------------------------------------------ */

static double dot3(const double a[3], const double b[3])
{
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

/* One view of one plane hypothesis at one reference pixel.
   Plane: the point X_p = d b_p on the pixel's ray with normal n, i.e. the
   set {X : n.X = c} with c = n.X_p. Each reference sample ray b_q meets it
   at X_q = (c / n.b_q) b_q; X_q is moved into the neighbour and projected
   (the patch warp of Sec. III-C). The cost is 1 - NCC of the reference and
   warped samples. The paper does not name its matching cost; plain
   unweighted NCC is used. A view is invalid (cost 2) when the plane is not
   in front of every sample ray or a variance falls below the floor. */
double pmsref_view_cost(int W, int H, const double *ref, const double *nbr, const double R[9],
                        const double t[3], const pmsref_params *p, int x, int y, double d,
                        const double n[3], double *r_out, double *s_out, double *vr_out,
                        double *vs_out)
{
    int32_t dx[PMSREF_MAX_SAMPLES], dy[PMSREF_MAX_SAMPLES];
    double rs[PMSREF_MAX_SAMPLES], ss[PMSREF_MAX_SAMPLES];
    int P = pmsref_patch_offsets(p, dx, dy);
    double bp[3];
    pmsref_unproject(W, H, x, y, bp);
    double c = d * dot3(n, bp);
    if (!(c < 0.0)) return 2.0;
    for (int q = 0; q < P; ++q) {
        int xq = wrap_index((double)(x + dx[q]), W);
        int yq = y + dy[q];
        if (yq < 0 || yq >= H) return 2.0;
        double bq[3], X[3], Y[3], u, v;
        pmsref_unproject(W, H, xq, yq, bq);
        double den = dot3(n, bq);
        if (!(den < 0.0)) return 2.0;
        double lambda = c / den;
        for (int i = 0; i < 3; ++i) X[i] = lambda * bq[i];
        for (int i = 0; i < 3; ++i) Y[i] = R[3 * i] * X[0] + R[3 * i + 1] * X[1] + R[3 * i + 2] * X[2] + t[i];
        pmsref_project(W, H, Y, &u, &v);
        ss[q] = pmsref_sample(nbr, W, H, u, v);
        rs[q] = ref[(size_t)yq * W + xq];
    }
    double mr = 0.0, ms = 0.0;
    for (int q = 0; q < P; ++q) {
        mr += rs[q];
        ms += ss[q];
    }
    mr /= P;
    ms /= P;
    double vr = 0.0, vs = 0.0, cov = 0.0;
    for (int q = 0; q < P; ++q) {
        vr += (rs[q] - mr) * (rs[q] - mr);
        vs += (ss[q] - ms) * (ss[q] - ms);
        cov += (rs[q] - mr) * (ss[q] - ms);
    }
    vr /= P;
    vs /= P;
    cov /= P;
    if (r_out) memcpy(r_out, rs, sizeof(double) * P);
    if (s_out) memcpy(s_out, ss, sizeof(double) * P);
    if (vr_out) *vr_out = vr;
    if (vs_out) *vs_out = vs;
    if (vr < p->ncc_var_floor || vs < p->ncc_var_floor) return 2.0;
    double ncc = cov / sqrt(vr * vs);
    if (ncc > 1.0) ncc = 1.0;
    if (ncc < -1.0) ncc = -1.0;
    return 1.0 - ncc;
}

/* Several neighbours (Sec. III-C matches against the two adjacent
   keyframes): the mean of the k smallest view costs, k = top_k or
   ceil(N/2). */
double pmsref_aggregate(const double *view_costs, int n_views, int top_k)
{
    double c[PMSREF_MAX_VIEWS];
    int k = top_k > 0 ? top_k : (n_views + 1) / 2;
    if (n_views <= 0) return 2.0;
    if (k > n_views) k = n_views;
    for (int j = 0; j < n_views; ++j) {
        double v = view_costs[j];
        int i = j;
        while (i > 0 && c[i - 1] > v) {
            c[i] = c[i - 1];
            --i;
        }
        c[i] = v;
    }
    double s = 0.0;
    for (int i = 0; i < k; ++i) s += c[i];
    return s / k;
}

/* Everything a pixel update needs, fixed for one call. */
typedef struct {
    int W, H, n_views;
    const double *ref;
    const double *const *nbrs;
    double R[PMSREF_MAX_VIEWS][9];
    double t[PMSREF_MAX_VIEWS][3];
    const pmsref_params *p;
} job_t;

static void job_init(job_t *J, int W, int H, const double *ref, int n_views,
                     const double *const *nbrs, const pmsref_pose *ref_pose,
                     const pmsref_pose *nbr_poses, const pmsref_params *p)
{
    J->W = W;
    J->H = H;
    J->n_views = n_views;
    J->ref = ref;
    J->nbrs = nbrs;
    J->p = p;
    for (int j = 0; j < n_views; ++j) pmsref_relative_pose(ref_pose, &nbr_poses[j], J->R[j], J->t[j]);
}

static double hyp_cost(const job_t *J, int x, int y, double d, const double n[3], double *per_view)
{
    double vc[PMSREF_MAX_VIEWS];
    for (int j = 0; j < J->n_views; ++j) {
        vc[j] = pmsref_view_cost(J->W, J->H, J->ref, J->nbrs[j], J->R[j], J->t[j], J->p, x, y, d,
                                 n, NULL, NULL, NULL, NULL);
        if (per_view) per_view[j] = vc[j];
    }
    return pmsref_aggregate(vc, J->n_views, J->p->top_k);
}

/* ------------------------------------------------------------------------ */
/* simple thread split                                                      */
/* ------------------------------------------------------------------------ */

typedef void (*range_fn)(void *ctx, long begin, long end);
typedef struct {
    range_fn fn;
    void *ctx;
    long begin, end;
} range_task;

static void *range_thread(void *arg)
{
    range_task *t = (range_task *)arg;
    t->fn(t->ctx, t->begin, t->end);
    return NULL;
}

static int thread_count(int n_threads)
{
    if (n_threads > 0) return n_threads;
    long n = sysconf(_SC_NPROCESSORS_ONLN);
    return n > 0 ? (int)n : 1;
}

static void parallel_for(long n, int n_threads, range_fn fn, void *ctx)
{
    int T = thread_count(n_threads);
    if (T > 256) T = 256;
    if (T <= 1 || n < 2 * T) {
        fn(ctx, 0, n);
        return;
    }
    pthread_t th[256];
    range_task tasks[256];
    char running[256];
    for (int i = 0; i < T; ++i) {
        tasks[i].fn = fn;
        tasks[i].ctx = ctx;
        tasks[i].begin = n * i / T;
        tasks[i].end = n * (i + 1) / T;
    }
    for (int i = 1; i < T; ++i) {
        running[i] = pthread_create(&th[i], NULL, range_thread, &tasks[i]) == 0;
        if (!running[i]) fn(ctx, tasks[i].begin, tasks[i].end); /* could not start: run here */
    }
    fn(ctx, tasks[0].begin, tasks[0].end);
    for (int i = 1; i < T; ++i)
        if (running[i]) pthread_join(th[i], NULL);
}

/* ------------------------------------------------------------------------ */
/* whole-image cost of given hypotheses                                     */
/* ------------------------------------------------------------------------ */

typedef struct {
    const job_t *J;
    const double *depth, *normal;
    double *cost, *per_view;
} eval_ctx;

static void eval_range(void *vctx, long begin, long end)
{
    eval_ctx *E = (eval_ctx *)vctx;
    const job_t *J = E->J;
    long HW = (long)J->W * J->H;
    for (long i = begin; i < end; ++i) {
        int x = (int)(i % J->W), y = (int)(i / J->W);
        double pv[PMSREF_MAX_VIEWS];
        double c = 2.0;
        for (int j = 0; j < J->n_views; ++j) pv[j] = 2.0;
        if (pmsref_pixel_valid(J->W, J->H, J->p, x, y) && E->depth[i] > 0.0) {
            double n[3] = {E->normal[i], E->normal[HW + i], E->normal[2 * HW + i]};
            c = hyp_cost(J, x, y, E->depth[i], n, pv);
        }
        E->cost[i] = c;
        if (E->per_view)
            for (int j = 0; j < J->n_views; ++j) E->per_view[(long)j * HW + i] = pv[j];
    }
}

int pmsref_eval_cost(int W, int H, const double *ref, int n_views, const double *const *nbrs,
                     const pmsref_pose *ref_pose, const pmsref_pose *nbr_poses,
                     const pmsref_params *p, const double *depth, const double *normal,
                     double *cost_out, double *per_view_out, int n_threads)
{
    int rc = pmsref_check_params(p, W, H, n_views);
    if (rc) return rc;
    if (n_views < 1 || !ref || !nbrs || !ref_pose || !nbr_poses || !depth || !normal || !cost_out)
        return -1;
    job_t J;
    job_init(&J, W, H, ref, n_views, nbrs, ref_pose, nbr_poses, p);
    eval_ctx E = {&J, depth, normal, cost_out, per_view_out};
    parallel_for((long)W * H, n_threads, eval_range, &E);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* random plane hypothesis (Sec. III-B: random initialisation)              */
/* ------------------------------------------------------------------------ */

/* Depth uniform in inverse depth over [depth_min, depth_max]; normal uniform
   on the sphere, flipped to face the camera. */
static void random_plane(const job_t *J, int x, int y, double *d, double n[3])
{
    const pmsref_params *p = J->p;
    double u[4], bp[3];
    pmsref_uniforms(p->seed, (uint64_t)y * J->W + x, 0, 0, u);
    pmsref_unproject(J->W, J->H, x, y, bp);
    double rho = 1.0 / p->depth_max + u[0] * (1.0 / p->depth_min - 1.0 / p->depth_max);
    *d = 1.0 / rho;
    double z = 2.0 * u[1] - 1.0, a = 2.0 * PI * u[2];
    double s = sqrt(fmax(0.0, 1.0 - z * z));
    n[0] = s * cos(a);
    n[1] = s * sin(a);
    n[2] = z;
    double nb = dot3(n, bp);
    if (nb > 0.0) {
        n[0] = -n[0];
        n[1] = -n[1];
        n[2] = -n[2];
    } else if (nb == 0.0) {
        n[0] = -bp[0];
        n[1] = -bp[1];
        n[2] = -bp[2];
    }
}

/* ------------------------------------------------------------------------ */
/* red-black update of one pixel (Sec. III-C)                               */
/* ------------------------------------------------------------------------ */

/* Decision-noise study hook (see pmsref.h): off unless set. The offset of
   (pixel, iteration, slot) is splitmix64 of a key made of the three, mapped
   to [-a, a]; slot 0 is the initial cost, 1 + k propagation candidate k,
   1 + PMSREF_MAX_OFFSETS + k refinement trial k. */
static double g_decision_noise = 0.0;

void pmsref_set_decision_noise(double amplitude) { g_decision_noise = amplitude; }

static uint64_t mix64(uint64_t z)
{
    z += 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

static double with_noise(double c, long pixel, int iteration, int slot)
{
    if (g_decision_noise <= 0.0 || !(c < 2.0)) return c;
    uint64_t k = mix64((uint64_t)pixel);
    k = mix64(k ^ ((uint64_t)iteration << 32 | (uint64_t)(uint32_t)slot));
    double u = (double)(k >> 11) * (1.0 / 9007199254740992.0); /* [0, 1) */
    return c + g_decision_noise * (2.0 * u - 1.0);
}

static void update_one(const job_t *J, const double *depth, const double *normal,
                       const double *cost, int iteration, int x, int y, double *d_out,
                       double n_out[3], double *c_out)
{
    const pmsref_params *p = J->p;
    int W = J->W;
    long HW = (long)W * J->H;
    long i = (long)y * W + x;
    double best_d = depth[i];
    double best_n[3] = {normal[i], normal[HW + i], normal[2 * HW + i]};
    double best_c = cost[i];
    double bp[3];
    pmsref_unproject(W, J->H, x, y, bp);

    /* Propagation: each opposite-colour neighbour's plane is intersected with
       this pixel's ray; the first strictly cheaper candidate in table order
       wins ties. */
    for (int k = 0; k < p->n_offsets; ++k) {
        int qx = (int)(((long)x + p->offsets[k][0]) % W);
        if (qx < 0) qx += W;
        int qy = y + p->offsets[k][1];
        if (!pmsref_pixel_valid(W, J->H, p, qx, qy)) continue;
        long qi = (long)qy * W + qx;
        double dq = depth[qi];
        if (!(dq > 0.0)) continue;
        double nq[3] = {normal[qi], normal[HW + qi], normal[2 * HW + qi]};
        double bq[3];
        pmsref_unproject(W, J->H, qx, qy, bq);
        double cq = dq * dot3(nq, bq);
        double den = dot3(nq, bp);
        if (!(den < 0.0)) continue;
        double dd = cq / den;
        if (!(dd >= p->depth_min && dd <= p->depth_max)) continue;
        double c = with_noise(hyp_cost(J, x, y, dd, nq, NULL), i, iteration, 1 + k);
        if (c < best_c) {
            best_c = c;
            best_d = dd;
            best_n[0] = nq[0];
            best_n[1] = nq[1];
            best_n[2] = nq[2];
        }
    }

    /* Random refinement (Sec. III-C item 1): trials around the current best,
       the search range shrinking from trial to trial; only a strictly lower
       cost is accepted. */
    double sd0 = p->refine_sigma_logdepth0 > 0.0 ? p->refine_sigma_logdepth0
                                                 : 0.5 * log(p->depth_max / p->depth_min);
    for (int k = 0; k < p->refine_trials; ++k) {
        double u[4];
        pmsref_uniforms(p->seed, (uint64_t)i, (uint64_t)iteration, (uint64_t)(16 + k), u);
        double sd = sd0 * pow(p->refine_depth_shrink, k);
        double sn = p->refine_sigma_normal0 * pow(p->refine_normal_shrink, k);
        double dd = best_d * exp((2.0 * u[0] - 1.0) * sd);
        if (dd < p->depth_min) dd = p->depth_min;
        if (dd > p->depth_max) dd = p->depth_max;
        double nn[3] = {best_n[0] + sn * (2.0 * u[1] - 1.0), best_n[1] + sn * (2.0 * u[2] - 1.0),
                        best_n[2] + sn * (2.0 * u[3] - 1.0)};
        double len = sqrt(dot3(nn, nn));
        if (!(len > 0.0)) continue;
        nn[0] /= len;
        nn[1] /= len;
        nn[2] /= len;
        if (!(dot3(nn, bp) < 0.0)) continue;
        double c = with_noise(hyp_cost(J, x, y, dd, nn, NULL), i, iteration,
                              1 + PMSREF_MAX_OFFSETS + k);
        if (c < best_c) {
            best_c = c;
            best_d = dd;
            best_n[0] = nn[0];
            best_n[1] = nn[1];
            best_n[2] = nn[2];
        }
    }
    *d_out = best_d;
    n_out[0] = best_n[0];
    n_out[1] = best_n[1];
    n_out[2] = best_n[2];
    *c_out = best_c;
}

int pmsref_update_pixel(int W, int H, const double *ref, int n_views, const double *const *nbrs,
                        const pmsref_pose *ref_pose, const pmsref_pose *nbr_poses,
                        const pmsref_params *p, const double *depth, const double *normal,
                        const double *cost, int iteration, int x, int y, double *d_out,
                        double n_out[3], double *cost_out)
{
    int rc = pmsref_check_params(p, W, H, n_views);
    if (rc) return rc;
    if (n_views < 1 || !pmsref_pixel_valid(W, H, p, x, y)) return -1;
    job_t J;
    job_init(&J, W, H, ref, n_views, nbrs, ref_pose, nbr_poses, p);
    update_one(&J, depth, normal, cost, iteration, x, y, d_out, n_out, cost_out);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* geometric consistency                                                    */
/* ------------------------------------------------------------------------ */

typedef struct {
    int W, H, n_maps, min_views;
    double *depth, *normal, *cost;
    const double *const *maps;
    double R[PMSREF_MAX_VIEWS][9], t[PMSREF_MAX_VIEWS][3];
    const pmsref_params *p;
    double *err_px, *err_depth;
    int32_t *agree;
    char *keep;
} geo_ctx;

static void geo_range(void *vctx, long begin, long end)
{
    geo_ctx *G = (geo_ctx *)vctx;
    int W = G->W, H = G->H;
    long HW = (long)W * H;
    for (long i = begin; i < end; ++i) {
        int x = (int)(i % W), y = (int)(i / W);
        double d = G->depth[i];
        G->keep[i] = 0;
        for (int j = 0; j < G->n_maps; ++j) {
            if (G->err_px) G->err_px[(long)j * HW + i] = -1.0;
            if (G->err_depth) G->err_depth[(long)j * HW + i] = -1.0;
            if (G->agree) G->agree[(long)j * HW + i] = -1;
        }
        if (!pmsref_pixel_valid(W, H, G->p, x, y) || !(d > 0.0)) continue;
        double bp[3], X[3];
        pmsref_unproject(W, H, x, y, bp);
        for (int k = 0; k < 3; ++k) X[k] = d * bp[k];
        int votes = 0;
        for (int j = 0; j < G->n_maps; ++j) {
            const double *R = G->R[j], *t = G->t[j];
            double Y[3], u, v;
            for (int k = 0; k < 3; ++k) Y[k] = R[3 * k] * X[0] + R[3 * k + 1] * X[1] + R[3 * k + 2] * X[2] + t[k];
            pmsref_project(W, H, Y, &u, &v);
            /* nearest neighbour pixel, halves rounded up */
            int xi = wrap_index(floor(u + 0.5), W);
            int yi = clamp_index(floor(v + 0.5), H);
            double dj = G->maps[j][(long)yi * W + xi];
            int ok = 0;
            double epx = INFINITY, ed = INFINITY;
            if (dj > 0.0) {
                double bj[3], Z[3], Xb[3], xb, yb;
                pmsref_unproject(W, H, xi, yi, bj);
                for (int k = 0; k < 3; ++k) Z[k] = dj * bj[k] - t[k];
                /* back into the reference frame: X' = R^T (Z - t) */
                for (int k = 0; k < 3; ++k) Xb[k] = R[k] * Z[0] + R[3 + k] * Z[1] + R[6 + k] * Z[2];
                pmsref_project(W, H, Xb, &xb, &yb);
                double ddx = xb - x;
                ddx -= W * floor((ddx + 0.5 * W) / W); /* fold into [-W/2, W/2) */
                double ddy = yb - y;
                epx = sqrt(ddx * ddx + ddy * ddy);
                ed = fabs(sqrt(dot3(Xb, Xb)) - d) / d;
                ok = (epx <= G->p->geo_px) && (ed <= G->p->geo_rel_depth);
            }
            votes += ok;
            if (G->err_px) G->err_px[(long)j * HW + i] = epx;
            if (G->err_depth) G->err_depth[(long)j * HW + i] = ed;
            if (G->agree) G->agree[(long)j * HW + i] = ok;
        }
        G->keep[i] = votes >= G->min_views;
    }
}

int pmsref_consistency(int W, int H, double *depth, double *normal, double *cost,
                       const pmsref_pose *ref_pose, int n_maps, const double *const *maps,
                       const pmsref_pose *map_poses, const pmsref_params *p, double *err_px,
                       double *err_depth, int32_t *agree, int n_threads)
{
    int rc = pmsref_check_params(p, W, H, 0);
    if (rc) return rc;
    if (n_maps < 1 || n_maps > PMSREF_MAX_VIEWS || !depth || !normal || !cost || !maps ||
        !ref_pose || !map_poses)
        return -1;
    long HW = (long)W * H;
    geo_ctx G;
    memset(&G, 0, sizeof G);
    G.W = W;
    G.H = H;
    G.n_maps = n_maps;
    G.min_views = p->geo_min_views > 0 ? p->geo_min_views : (n_maps < 2 ? n_maps : 2);
    G.depth = depth;
    G.normal = normal;
    G.cost = cost;
    G.maps = maps;
    G.p = p;
    G.err_px = err_px;
    G.err_depth = err_depth;
    G.agree = agree;
    for (int j = 0; j < n_maps; ++j) pmsref_relative_pose(ref_pose, &map_poses[j], G.R[j], G.t[j]);
    G.keep = (char *)malloc((size_t)HW);
    if (!G.keep) return -20;
    parallel_for(HW, n_threads, geo_range, &G);
    for (long i = 0; i < HW; ++i)
        if (!G.keep[i]) {
            depth[i] = 0.0;
            normal[i] = normal[HW + i] = normal[2 * HW + i] = 0.0;
            cost[i] = 2.0;
        }
    free(G.keep);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* full densification                                                       */
/* ------------------------------------------------------------------------ */

typedef struct {
    const job_t *J;
    double *depth, *normal, *cost;
    const double *init_depth, *init_normal;
} init_ctx;

static void init_range(void *vctx, long begin, long end)
{
    init_ctx *C = (init_ctx *)vctx;
    const job_t *J = C->J;
    const pmsref_params *p = J->p;
    long HW = (long)J->W * J->H;
    for (long i = begin; i < end; ++i) {
        int x = (int)(i % J->W), y = (int)(i / J->W);
        if (!pmsref_pixel_valid(J->W, J->H, p, x, y)) {
            C->depth[i] = 0.0;
            C->normal[i] = C->normal[HW + i] = C->normal[2 * HW + i] = 0.0;
            C->cost[i] = 2.0;
            continue;
        }
        double d, n[3];
        random_plane(J, x, y, &d, n);
        if (C->init_depth && C->init_normal) {
            /* a supplied plane replaces the random one where it is usable */
            double di = C->init_depth[i];
            double ni[3] = {C->init_normal[i], C->init_normal[HW + i], C->init_normal[2 * HW + i]};
            double bp[3];
            pmsref_unproject(J->W, J->H, x, y, bp);
            if (di >= p->depth_min && di <= p->depth_max && dot3(ni, bp) < 0.0) {
                d = di;
                n[0] = ni[0];
                n[1] = ni[1];
                n[2] = ni[2];
            }
        }
        C->depth[i] = d;
        C->normal[i] = n[0];
        C->normal[HW + i] = n[1];
        C->normal[2 * HW + i] = n[2];
        C->cost[i] = with_noise(hyp_cost(J, x, y, d, n, NULL), i, 0, 0);
    }
}

typedef struct {
    const job_t *J;
    const double *depth, *normal, *cost;
    const long *pix;
    int iteration;
    double *nd, *nn, *nc; /* per listed pixel: new depth, normal (3), cost */
} sweep_ctx;

static void sweep_range(void *vctx, long begin, long end)
{
    sweep_ctx *S = (sweep_ctx *)vctx;
    for (long k = begin; k < end; ++k) {
        long i = S->pix[k];
        int x = (int)(i % S->J->W), y = (int)(i / S->J->W);
        update_one(S->J, S->depth, S->normal, S->cost, S->iteration, x, y, &S->nd[k],
                   &S->nn[3 * k], &S->nc[k]);
    }
}

int pmsref_halfsweep_rows(int W, int H, const double *ref, int n_views, const double *const *nbrs,
                          const pmsref_pose *ref_pose, const pmsref_pose *nbr_poses,
                          const pmsref_params *p, const double *depth, const double *normal,
                          const double *cost, int iteration, int colour, int y0, int y1,
                          double *depth_out, double *normal_out, double *cost_out, int n_threads)
{
    int rc = pmsref_check_params(p, W, H, n_views);
    if (rc) return rc;
    if (n_views < 1 || (colour != 0 && colour != 1) || y0 < 0 || y1 > H || y0 > y1) return -1;
    long HW = (long)W * H;
    job_t J;
    job_init(&J, W, H, ref, n_views, nbrs, ref_pose, nbr_poses, p);
    memcpy(depth_out, depth, sizeof(double) * (size_t)HW);
    memcpy(normal_out, normal, sizeof(double) * 3 * (size_t)HW);
    memcpy(cost_out, cost, sizeof(double) * (size_t)HW);
    long cap = (long)(y1 - y0) * W / 2 + 1;
    long *pix = (long *)malloc(sizeof(long) * (size_t)cap);
    double *nd = (double *)malloc(sizeof(double) * (size_t)cap);
    double *nn = (double *)malloc(sizeof(double) * 3 * (size_t)cap);
    double *nc = (double *)malloc(sizeof(double) * (size_t)cap);
    if (!pix || !nd || !nn || !nc) {
        free(pix);
        free(nd);
        free(nn);
        free(nc);
        return -20;
    }
    long np = 0;
    for (int y = y0; y < y1; ++y)
        for (int x = 0; x < W; ++x)
            if (((x + y) & 1) == colour && pmsref_pixel_valid(W, H, p, x, y)) pix[np++] = (long)y * W + x;
    sweep_ctx S = {&J, depth, normal, cost, pix, iteration, nd, nn, nc};
    parallel_for(np, n_threads, sweep_range, &S);
    for (long k = 0; k < np; ++k) {
        long i = pix[k];
        depth_out[i] = nd[k];
        normal_out[i] = nn[3 * k];
        normal_out[HW + i] = nn[3 * k + 1];
        normal_out[2 * HW + i] = nn[3 * k + 2];
        cost_out[i] = nc[k];
    }
    free(pix);
    free(nd);
    free(nn);
    free(nc);
    return 0;
}

static uint64_t splitmix64(uint64_t *s)
{
    uint64_t z = (*s += 0x9E3779B97F4A7C15ULL);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

int pmsref_densify(int W, int H, const double *ref, int n_views, const double *const *nbrs,
                   const pmsref_pose *ref_pose, const pmsref_pose *nbr_poses,
                   const pmsref_params *p, const double *init_depth, const double *init_normal,
                   int n_maps, const double *const *maps, const pmsref_pose *map_poses,
                   double *depth_out, double *normal_out, double *cost_out, int n_threads,
                   uint64_t order_seed)
{
    int rc = pmsref_check_params(p, W, H, n_views);
    if (rc) return rc;
    if (n_views < 1 || !ref || !nbrs || !ref_pose || !nbr_poses || !depth_out || !normal_out ||
        !cost_out)
        return -1;
    if (n_maps < 0 || n_maps > PMSREF_MAX_VIEWS || (n_maps > 0 && (!maps || !map_poses)))
        return -1;
    long HW = (long)W * H;
    job_t J;
    job_init(&J, W, H, ref, n_views, nbrs, ref_pose, nbr_poses, p);

    double *depth = depth_out, *normal = normal_out, *cost = cost_out;
    init_ctx IC = {&J, depth, normal, cost, init_depth, init_normal};
    parallel_for(HW, n_threads, init_range, &IC);

    long *pix = (long *)malloc(sizeof(long) * (size_t)(HW / 2 + 1));
    double *nd = (double *)malloc(sizeof(double) * (size_t)(HW / 2 + 1));
    double *nn = (double *)malloc(sizeof(double) * 3 * (size_t)(HW / 2 + 1));
    double *nc = (double *)malloc(sizeof(double) * (size_t)(HW / 2 + 1));
    if (!pix || !nd || !nn || !nc) {
        free(pix);
        free(nd);
        free(nn);
        free(nc);
        return -20;
    }
    for (int it = 1; it <= p->iterations; ++it)
        for (int colour = 0; colour < 2; ++colour) {
            /* red = even x+y first, then black */
            long np = 0;
            for (long i = 0; i < HW; ++i) {
                int x = (int)(i % W), y = (int)(i / W);
                if (((x + y) & 1) == colour && pmsref_pixel_valid(W, H, p, x, y)) pix[np++] = i;
            }
            if (order_seed == 0) {
                sweep_ctx S = {&J, depth, normal, cost, pix, it, nd, nn, nc};
                parallel_for(np, n_threads, sweep_range, &S);
                for (long k = 0; k < np; ++k) {
                    long i = pix[k];
                    depth[i] = nd[k];
                    normal[i] = nn[3 * k];
                    normal[HW + i] = nn[3 * k + 1];
                    normal[2 * HW + i] = nn[3 * k + 2];
                    cost[i] = nc[k];
                }
            } else {
                /* seeded random order, written in place one pixel at a time */
                uint64_t s = order_seed ^ ((uint64_t)it << 32) ^ (uint64_t)colour;
                for (long k = np - 1; k > 0; --k) {
                    long j = (long)(splitmix64(&s) % (uint64_t)(k + 1));
                    long tmp = pix[k];
                    pix[k] = pix[j];
                    pix[j] = tmp;
                }
                for (long k = 0; k < np; ++k) {
                    long i = pix[k];
                    int x = (int)(i % W), y = (int)(i / W);
                    double d1, n1[3], c1;
                    update_one(&J, depth, normal, cost, it, x, y, &d1, n1, &c1);
                    depth[i] = d1;
                    normal[i] = n1[0];
                    normal[HW + i] = n1[1];
                    normal[2 * HW + i] = n1[2];
                    cost[i] = c1;
                }
            }
        }
    free(pix);
    free(nd);
    free(nn);
    free(nc);

    rc = pmsref_median_filter(W, H, depth, normal, cost, p);
    if (rc) return rc;
    if (n_maps > 0)
        return pmsref_consistency(W, H, depth, normal, cost, ref_pose, n_maps, maps, map_poses, p,
                                  NULL, NULL, NULL, n_threads);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* plane-map warping (Sec. III-B: the optimised plane map of the preceding  */
/* keyframe initialises the current one; after Shen 2013). The paper's      */
/* listing of the step is a figure that is not in the text; the reading:    */
/* every valid source pixel carries its plane point X = d b into the        */
/* destination camera (Y = R X + t, relative pose composed in FP64), where  */
/* it claims the nearest pixel; of the claims on one pixel the nearest point */
/* wins (range rounded to float, ties to the lower source index, so that    */
/* the choice is the one a float z-buffer makes); the winner's plane,       */
/* normal R n through Y, is re-intersected with the claimed pixel's own     */
/* ray. Parity: pinned by tests (identity, exact yaw shift, analytic        */
/* planes, occlusion by a nearer plane, back-facing planes).                */
/* ------------------------------------------------------------------------ */

int pmsref_warp_planes(int W, int H, const double *src_depth, const double *src_normal,
                       const pmsref_pose *src_pose, const pmsref_pose *dst_pose,
                       const pmsref_params *p, double *dst_depth, double *dst_normal)
{
    int rc = pmsref_check_params(p, W, H, 0);
    if (rc) return rc;
    if (!src_depth || !src_normal || !src_pose || !dst_pose || !dst_depth || !dst_normal) return -1;
    long HW = (long)W * H;
    double R[9], t[3];
    pmsref_relative_pose(src_pose, dst_pose, R, t);
    uint64_t *best = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)HW);
    if (!best) return -20;
    for (long i = 0; i < HW; ++i) best[i] = UINT64_MAX;
    /* claims */
    for (long i = 0; i < HW; ++i) {
        int x = (int)(i % W), y = (int)(i / W);
        double d = src_depth[i];
        if (!pmsref_pixel_valid(W, H, p, x, y) || !(d > 0.0)) continue;
        double b[3], X[3], Y[3];
        pmsref_unproject(W, H, x, y, b);
        for (int k = 0; k < 3; ++k) X[k] = d * b[k];
        for (int k = 0; k < 3; ++k) Y[k] = R[3 * k] * X[0] + R[3 * k + 1] * X[1] + R[3 * k + 2] * X[2] + t[k];
        double range = sqrt(dot3(Y, Y));
        if (!(range > 0.0)) continue;
        double u, v;
        pmsref_project(W, H, Y, &u, &v);
        int xi = wrap_index(floor(u + 0.5), W);
        int yi = clamp_index(floor(v + 0.5), H);
        if (!pmsref_pixel_valid(W, H, p, xi, yi)) continue;
        float rf = (float)range;
        uint32_t bits;
        memcpy(&bits, &rf, sizeof bits);
        uint64_t key = ((uint64_t)bits << 32) | (uint64_t)(uint32_t)i;
        long j = (long)yi * W + xi;
        if (key < best[j]) best[j] = key;
    }
    /* resolution: the winning plane at each claimed pixel */
    for (long j = 0; j < HW; ++j) {
        dst_depth[j] = 0.0;
        dst_normal[j] = dst_normal[HW + j] = dst_normal[2 * HW + j] = 0.0;
        if (best[j] == UINT64_MAX) continue;
        long i = (long)(best[j] & 0xffffffffu);
        int x = (int)(i % W), y = (int)(i / W);
        int xd = (int)(j % W), yd = (int)(j / W);
        double b[3], X[3], Y[3], n[3], nd[3], bd[3];
        pmsref_unproject(W, H, x, y, b);
        for (int k = 0; k < 3; ++k) X[k] = src_depth[i] * b[k];
        for (int k = 0; k < 3; ++k) Y[k] = R[3 * k] * X[0] + R[3 * k + 1] * X[1] + R[3 * k + 2] * X[2] + t[k];
        for (int k = 0; k < 3; ++k) n[k] = src_normal[(long)k * HW + i];
        for (int k = 0; k < 3; ++k) nd[k] = R[3 * k] * n[0] + R[3 * k + 1] * n[1] + R[3 * k + 2] * n[2];
        pmsref_unproject(W, H, xd, yd, bd);
        double den = dot3(nd, bd);
        if (!(den < 0.0)) continue;
        double dd = dot3(nd, Y) / den;
        if (!(dd >= p->depth_min && dd <= p->depth_max)) continue;
        dst_depth[j] = dd;
        for (int k = 0; k < 3; ++k) dst_normal[(long)k * HW + j] = nd[k];
    }
    free(best);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* median post-filter (Sec. III-C, item 2: a depth whose distance from the  */
/* median of its window exceeds a threshold is dropped from the map).       */
/* Window, median of an even count and the relative                         */
/* threshold are readings. Parity: pinned by tests (flat maps, an isolated  */
/* outlier, brute force against numpy on random maps, the seam, the exact   */
/* threshold).                                                              */
/* ------------------------------------------------------------------------ */

static int cmp_double(const void *a, const void *b)
{
    double x = *(const double *)a, y = *(const double *)b;
    return (x > y) - (x < y);
}

int pmsref_median_filter(int W, int H, double *depth, double *normal, double *cost,
                         const pmsref_params *p)
{
    if (!p || !depth || !normal || !cost) return -1;
    int R = p->median_radius;
    if (R <= 0) return 0;
    long HW = (long)W * H;
    double *copy = (double *)malloc(sizeof(double) * (size_t)HW);
    char *drop = (char *)calloc((size_t)HW, 1);
    double win[17 * 17];
    if (!copy || !drop) {
        free(copy);
        free(drop);
        return -20;
    }
    memcpy(copy, depth, sizeof(double) * (size_t)HW);
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            double d = copy[(long)y * W + x];
            if (!(d > 0.0)) continue;
            int n = 0;
            for (int dy = -R; dy <= R; ++dy) {
                int yy = y + dy;
                if (yy < 0 || yy >= H) continue;
                for (int dx = -R; dx <= R; ++dx) {
                    int xx = ((x + dx) % W + W) % W;
                    double v = copy[(long)yy * W + xx];
                    if (v > 0.0) win[n++] = v;
                }
            }
            qsort(win, (size_t)n, sizeof(double), cmp_double);
            double m = win[(n - 1) / 2];
            if (fabs(d - m) > p->median_rel * m) drop[(long)y * W + x] = 1;
        }
    for (long i = 0; i < HW; ++i)
        if (drop[i]) {
            depth[i] = 0.0;
            normal[i] = normal[HW + i] = normal[2 * HW + i] = 0.0;
            cost[i] = 2.0;
        }
    free(copy);
    free(drop);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* view filter (Sec. III-A, Eq. 1): the triangulation angle theta_p at each  */
/* sparse point p seen by both keyframes, between the directions from p to  */
/* the two camera centres; the candidate keyframe is accepted when at least */
/* min_frac of the points have theta_p within [min_deg, max_deg]. Points at */
/* a camera centre have no angle and are not counted. Parity: pinned by     */
/* tests (points on the perpendicular bisector with closed-form angles,     */
/* collinear points, mixtures with known fractions).                         */
/* ------------------------------------------------------------------------ */

int pmsref_view_filter(const double ca[3], const double cb[3], const double *points, long n,
                       double min_deg, double max_deg, double min_frac, long *in_range,
                       long *counted)
{
    if (!ca || !cb || (n > 0 && !points) || n < 0 || !in_range || !counted) return -1;
    long k = 0, c = 0;
    for (long i = 0; i < n; ++i) {
        const double *p = points + 3 * i;
        double a[3] = {ca[0] - p[0], ca[1] - p[1], ca[2] - p[2]};
        double b[3] = {cb[0] - p[0], cb[1] - p[1], cb[2] - p[2]};
        double la = sqrt(dot3(a, a)), lb = sqrt(dot3(b, b));
        if (!(la > 0.0) || !(lb > 0.0)) continue;
        double cs = dot3(a, b) / (la * lb);
        cs = cs > 1.0 ? 1.0 : (cs < -1.0 ? -1.0 : cs);
        double deg = acos(cs) * 180.0 / PI;
        ++c;
        if (deg >= min_deg && deg <= max_deg) ++k;
    }
    *in_range = k;
    *counted = c;
    return c > 0 && (double)k >= min_frac * (double)c;
}

/* ------------------------------------------------------------------------ */
/* dense point-cloud fusion (Sec. III: the point-cloud thread buffers four  */
/* consistent keyframes, erases duplicates and adds the points to the      */
/* map). Reading: every valid pixel of the buffered depth maps is a world  */
/* point; points falling into the same cubic voxel of edge `voxel` are      */
/* duplicates, of which the first in (map, pixel) order is kept. Parity:    */
/* pinned by tests (duplicate maps, brute force with numpy's unique, one    */
/* huge voxel, coverage of analytic point sets).                            */
/* ------------------------------------------------------------------------ */

static void world_point(int W, int H, const pmsref_pose *pose, int x, int y, double d, double Xw[3])
{
    double b[3], Xc[3];
    pmsref_unproject(W, H, x, y, b);
    for (int k = 0; k < 3; ++k) Xc[k] = d * b[k] - pose->t[k];
    /* X_w = R^T (X_c - t) */
    for (int k = 0; k < 3; ++k)
        Xw[k] = pose->R[k] * Xc[0] + pose->R[3 + k] * Xc[1] + pose->R[6 + k] * Xc[2];
}

typedef struct {
    int64_t v[3];
    long order; /* map * H * W + pixel */
} voxel_entry;

static int cmp_voxel(const void *a, const void *b)
{
    const voxel_entry *p = (const voxel_entry *)a, *q = (const voxel_entry *)b;
    for (int k = 0; k < 3; ++k)
        if (p->v[k] != q->v[k]) return p->v[k] < q->v[k] ? -1 : 1;
    return (p->order > q->order) - (p->order < q->order);
}

int pmsref_fuse(int W, int H, int n_maps, const double *const *depths, const pmsref_pose *poses,
                double voxel, uint8_t *keep, long *n_kept)
{
    if (W < 2 || H < 1 || W != 2 * H || n_maps < 1 || !depths || !poses || !keep || !n_kept ||
        !(voxel > 0.0))
        return -1;
    long HW = (long)W * H;
    voxel_entry *e = (voxel_entry *)malloc(sizeof(voxel_entry) * (size_t)(HW * n_maps));
    if (!e) return -20;
    long n = 0;
    memset(keep, 0, (size_t)(HW * n_maps));
    for (int m = 0; m < n_maps; ++m)
        for (long i = 0; i < HW; ++i) {
            double d = depths[m][i];
            if (!(d > 0.0)) continue;
            double X[3];
            world_point(W, H, &poses[m], (int)(i % W), (int)(i / W), d, X);
            for (int k = 0; k < 3; ++k) e[n].v[k] = (int64_t)floor(X[k] / voxel);
            e[n].order = (long)m * HW + i;
            ++n;
        }
    qsort(e, (size_t)n, sizeof(voxel_entry), cmp_voxel);
    long kept = 0;
    for (long j = 0; j < n; ++j)
        if (j == 0 || e[j].v[0] != e[j - 1].v[0] || e[j].v[1] != e[j - 1].v[1] || e[j].v[2] != e[j - 1].v[2]) {
            keep[e[j].order] = 1;
            ++kept;
        }
    free(e);
    *n_kept = kept;
    return 0;
}

/* Completeness of a point cloud seen from one camera (the paper renders
   depth panoramas of the fused cloud at 720 x 360): every kept point of the
   maps marks the pixel of a Wc x Hc equirectangular image at view_pose
   nearest to its projection; returns the number of marked pixels. */
long pmsref_coverage(int W, int H, int n_maps, const double *const *depths,
                     const pmsref_pose *poses, const uint8_t *keep, const pmsref_pose *view_pose,
                     int Wc, int Hc, uint8_t *cover)
{
    if (!depths || !poses || !view_pose || !cover || Wc < 2 || Hc < 1) return -1;
    long HW = (long)W * H;
    memset(cover, 0, (size_t)Wc * Hc);
    for (int m = 0; m < n_maps; ++m)
        for (long i = 0; i < HW; ++i) {
            double d = depths[m][i];
            if (!(d > 0.0) || (keep && !keep[(long)m * HW + i])) continue;
            double X[3], Y[3], u, v;
            world_point(W, H, &poses[m], (int)(i % W), (int)(i / W), d, X);
            for (int k = 0; k < 3; ++k)
                Y[k] = view_pose->R[3 * k] * X[0] + view_pose->R[3 * k + 1] * X[1] +
                       view_pose->R[3 * k + 2] * X[2] + view_pose->t[k];
            if (!(dot3(Y, Y) > 0.0)) continue;
            pmsref_project(Wc, Hc, Y, &u, &v);
            int xi = wrap_index(floor(u + 0.5), Wc);
            int yi = clamp_index(floor(v + 0.5), Hc);
            cover[(long)yi * Wc + xi] = 1;
        }
    long c = 0;
    for (long j = 0; j < (long)Wc * Hc; ++j) c += cover[j];
    return c;
}
