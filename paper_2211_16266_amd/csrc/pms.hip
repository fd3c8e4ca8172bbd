// pms.hip -- host side of libpms: argument validation, FP64 pose
// composition, scratch management and kernel launches behind the C ABI
// declared in include/pms.h.
#include "pms.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "pms_kernels.hpp"

namespace {

constexpr int kNumKernelKinds = 7;
const char *const kKernelNames[kNumKernelKinds] = {"refstats", "init", "halfsweep", "finalize",
                                                   "consistency", "eval", "io"};
enum KernelKind { KK_REFSTATS, KK_INIT, KK_HALFSWEEP, KK_FINALIZE, KK_CONSISTENCY, KK_EVAL, KK_IO };

struct TimedLaunch {
    int kind;
    hipEvent_t start, stop;
};

}  // namespace

struct pms_context {
    int device = 0;
    size_t budget = 0;
    // scratch: [state float4 | cost float | stats float2] for `cap_pixels`
    // pixels, then the bearing tables for (tab_W, tab_H)
    void *scratch = nullptr;
    size_t scratch_bytes = 0;
    long long cap_pixels = 0;
    float4 *state = nullptr;
    float *cost = nullptr;
    float2 *stats = nullptr;
    float2 *tab_row = nullptr;
    float2 *tab_col = nullptr;
    double2 *tab_row64 = nullptr;
    double2 *tab_col64 = nullptr;
    int tab_W = 0, tab_H = 0;
    void *pad[pms::MAXV] = {};  // re-laid-out neighbour images
    int pad_Wp = 0;
    int pad_bytes = 0;
    std::string last_error;
    bool profiling = false;
    std::vector<TimedLaunch> launches;
    std::vector<hipEvent_t> event_pool;
};

namespace {

pms_status fail(pms_context *ctx, pms_status s, const std::string &msg)
{
    if (ctx) ctx->last_error = msg;
    return s;
}

pms_status hip_fail(pms_context *ctx, hipError_t e, const char *what)
{
    return fail(ctx, PMS_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

size_t dtype_size(int dt)
{
    switch (dt) {
    case PMS_F32: return 4;
    case PMS_F16: return 2;
    case PMS_U8: return 1;
    default: return 0;
    }
}

bool finite_pose(const pms_pose &p)
{
    for (double v : p.R)
        if (!std::isfinite(v)) return false;
    for (double v : p.t)
        if (!std::isfinite(v)) return false;
    return true;
}

int patch_samples(const pms_params &p)
{
    const int r = (p.patch_size - 1) / 2;
    const int side = 2 * r / p.patch_stride + 1;
    return side * side;
}

// Checks every parameter; `n_views` = 0 skips the view-dependent checks.
bool check_params(pms_context *ctx, const pms_params *p, int W, int H, int n_views,
                  pms_status *st)
{
    auto bad = [&](const char *m) {
        *st = fail(ctx, PMS_ERR_INVALID_ARG, m);
        return false;
    };
    if (!p) return bad("params is null");
    if (p->patch_size < 3 || p->patch_size % 2 == 0) return bad("patch_size must be odd and >= 3");
    if (p->patch_stride < 1 || (p->patch_size - 1) % p->patch_stride != 0)
        return bad("patch_stride must divide patch_size - 1");
    if (patch_samples(*p) > PMS_MAX_SAMPLES) {
        *st = fail(ctx, PMS_ERR_UNSUPPORTED, "more than 64 samples per patch");
        return false;
    }
    if (p->iterations < 0) return bad("iterations < 0");
    if (p->refine_trials < 0 || p->refine_trials > PMS_MAX_TRIALS) return bad("refine_trials out of range");
    if (!(p->depth_min > 0.0) || !(p->depth_max > p->depth_min) || !std::isfinite(p->depth_max))
        return bad("need 0 < depth_min < depth_max < inf");
    if (n_views > 0 && (p->top_k < 0 || p->top_k > n_views)) return bad("top_k out of range");
    if (!(p->ncc_var_floor >= 0.0) || !std::isfinite(p->ncc_var_floor)) return bad("bad ncc_var_floor");
    if (!std::isfinite(p->refine_sigma_logdepth0) || !(p->refine_depth_shrink > 0.0) ||
        !std::isfinite(p->refine_depth_shrink) || !(p->refine_sigma_normal0 >= 0.0) ||
        !std::isfinite(p->refine_sigma_normal0) || !(p->refine_normal_shrink > 0.0) ||
        !std::isfinite(p->refine_normal_shrink))
        return bad("bad refinement widths");
    if (p->n_offsets < 0 || p->n_offsets > PMS_MAX_OFFSETS) return bad("n_offsets out of range");
    for (int k = 0; k < p->n_offsets; ++k) {
        const int ox = p->offsets[k][0], oy = p->offsets[k][1];
        if ((std::abs(ox) + std::abs(oy)) % 2 != 1)
            return bad("a propagation offset must have odd |dx|+|dy| (opposite colour)");
        if (oy <= -H || oy >= H || ox <= -W || ox >= W) return bad("propagation offset too large");
    }
    if (!(p->geo_px >= 0.0) || !(p->geo_rel_depth >= 0.0) || p->geo_min_views < 0)
        return bad("bad consistency thresholds");
    return true;
}

bool check_image(pms_context *ctx, const pms_image &im, int W, int H, int dtype, const char *what,
                 pms_status *st)
{
    char buf[160];
    if (!im.data) {
        std::snprintf(buf, sizeof buf, "%s: null data", what);
        *st = fail(ctx, PMS_ERR_INVALID_ARG, buf);
        return false;
    }
    if (im.width != W || im.height != H) {
        std::snprintf(buf, sizeof buf, "%s: size %dx%d differs from %dx%d", what, im.width,
                      im.height, W, H);
        *st = fail(ctx, PMS_ERR_INVALID_ARG, buf);
        return false;
    }
    if (im.dtype != dtype) {
        std::snprintf(buf, sizeof buf, "%s: dtype differs from the reference", what);
        *st = fail(ctx, PMS_ERR_INVALID_ARG, buf);
        return false;
    }
    if (im.pitch_bytes < (int64_t)W * (int64_t)dtype_size(dtype)) {
        std::snprintf(buf, sizeof buf, "%s: pitch too small", what);
        *st = fail(ctx, PMS_ERR_INVALID_ARG, buf);
        return false;
    }
    return true;
}

bool check_plane(pms_context *ctx, const pms_plane &p, int W, const char *what, pms_status *st)
{
    if (!p.data || p.pitch_elems < W) {
        *st = fail(ctx, PMS_ERR_INVALID_ARG, std::string(what) + ": null data or pitch < width");
        return false;
    }
    return true;
}

bool check_ref_and_views(pms_context *ctx, const pms_image *ref, const pms_pose *ref_pose,
                         const pms_image *nbrs, const pms_pose *nbr_poses, int n_nbrs,
                         pms_status *st)
{
    if (!ref) {
        *st = fail(ctx, PMS_ERR_INVALID_ARG, "ref is null");
        return false;
    }
    const int W = ref->width, H = ref->height;
    if (H < 1 || W != 2 * H) {
        *st = fail(ctx, PMS_ERR_INVALID_ARG, "images must be W x H with W == 2H >= 2");
        return false;
    }
    if (dtype_size(ref->dtype) == 0) {
        *st = fail(ctx, PMS_ERR_INVALID_ARG, "unknown dtype");
        return false;
    }
    if (!check_image(ctx, *ref, W, H, ref->dtype, "ref", st)) return false;
    if (n_nbrs < 1 || n_nbrs > PMS_MAX_VIEWS) {
        *st = fail(ctx, PMS_ERR_INVALID_ARG, "n_nbrs must be in [1, 8]");
        return false;
    }
    if (!nbrs || !nbr_poses || !ref_pose) {
        *st = fail(ctx, PMS_ERR_INVALID_ARG, "null neighbour or pose array");
        return false;
    }
    for (int j = 0; j < n_nbrs; ++j)
        if (!check_image(ctx, nbrs[j], W, H, ref->dtype, "neighbour", st)) return false;
    if (!finite_pose(*ref_pose)) {
        *st = fail(ctx, PMS_ERR_INVALID_ARG, "non-finite reference pose");
        return false;
    }
    for (int j = 0; j < n_nbrs; ++j)
        if (!finite_pose(nbr_poses[j])) {
            *st = fail(ctx, PMS_ERR_INVALID_ARG, "non-finite neighbour pose");
            return false;
        }
    return true;
}

// X_nbr = (R_n R_r^T) X_ref + (t_n - R_n R_r^T t_r), composed in FP64.
pms::ViewPoseD relative_pose64(const pms_pose &ref, const pms_pose &nbr)
{
    pms::ViewPoseD out;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = 0.0;
            for (int k = 0; k < 3; ++k) s += nbr.R[3 * i + k] * ref.R[3 * j + k];
            out.R[3 * i + j] = s;
        }
    for (int i = 0; i < 3; ++i)
        out.t[i] = nbr.t[i] - (out.R[3 * i] * ref.t[0] + out.R[3 * i + 1] * ref.t[1] + out.R[3 * i + 2] * ref.t[2]);
    return out;
}

// The same, rounded once to float (consistency filter).
pms::ViewPoseF relative_pose(const pms_pose &ref, const pms_pose &nbr)
{
    double R[9], t[3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = 0.0;
            for (int k = 0; k < 3; ++k) s += nbr.R[3 * i + k] * ref.R[3 * j + k];
            R[3 * i + j] = s;
        }
    for (int i = 0; i < 3; ++i) t[i] = nbr.t[i] - (R[3 * i] * ref.t[0] + R[3 * i + 1] * ref.t[1] + R[3 * i + 2] * ref.t[2]);
    pms::ViewPoseF out;
    for (int i = 0; i < 9; ++i) out.R[i] = (float)R[i];
    for (int i = 0; i < 3; ++i) out.t[i] = (float)t[i];
    return out;
}

size_t pad_elem_size(int dtype) { return dtype == PMS_F16 ? 2 : 4; }

// Grows the scratch block to hold W x H pixels of state, the bearing tables
// and n_pad re-laid-out neighbour images of `pad_elem` bytes per value.
pms_status ensure_scratch(pms_context *ctx, int W, int H, int n_pad, size_t pad_elem,
                          hipStream_t stream)
{
    const long long npx = (long long)W * H;
    const size_t state_b = (size_t)npx * sizeof(float4);
    const size_t cost_b = (size_t)npx * sizeof(float);
    const size_t stats_b = (size_t)npx * sizeof(float2);
    const size_t tabs_b = (size_t)(W + H) * (sizeof(float2) + sizeof(double2));
    const int Wp = 2 * W + 4;
    const size_t pad_b = (size_t)(H + 2) * Wp * pad_elem;
    auto align = [](size_t v) { return (v + 255) & ~(size_t)255; };
    const size_t need = align(state_b) + align(cost_b) + align(stats_b) + align(tabs_b) +
                        (size_t)n_pad * align(pad_b);
    if (ctx->device < 0) return fail(ctx, PMS_ERR_DEVICE, "validation-only context cannot launch");
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_fail(ctx, e, "hipSetDevice");
    if (need > ctx->scratch_bytes) {
        if (ctx->budget && need > ctx->budget)
            return fail(ctx, PMS_ERR_BUDGET, "scratch for this image size exceeds the context budget");
        if (ctx->scratch) {
            // earlier work may still use the old block
            e = hipDeviceSynchronize();
            if (e != hipSuccess) return hip_fail(ctx, e, "hipDeviceSynchronize");
            (void)hipFree(ctx->scratch);
            ctx->scratch = nullptr;
            ctx->scratch_bytes = 0;
        }
        e = hipMalloc(&ctx->scratch, need);
        if (e != hipSuccess) {
            ctx->scratch = nullptr;
            return fail(ctx, PMS_ERR_OUT_OF_MEMORY, "hipMalloc of scratch failed");
        }
        ctx->scratch_bytes = need;
        ctx->tab_W = ctx->tab_H = 0;
    }
    char *base = static_cast<char *>(ctx->scratch);
    ctx->state = reinterpret_cast<float4 *>(base);
    base += align(state_b);
    ctx->cost = reinterpret_cast<float *>(base);
    base += align(cost_b);
    ctx->stats = reinterpret_cast<float2 *>(base);
    base += align(stats_b);
    float2 *tabs = reinterpret_cast<float2 *>(base);
    base += align(tabs_b);
    for (int j = 0; j < pms::MAXV; ++j) {
        ctx->pad[j] = j < n_pad ? static_cast<void *>(base) : nullptr;
        if (j < n_pad) base += align(pad_b);
    }
    ctx->pad_Wp = Wp;
    ctx->pad_bytes = (int)pad_b;
    if (ctx->tab_W != W || ctx->tab_H != H || ctx->tab_row != tabs) {
        ctx->tab_row = tabs;
        ctx->tab_col = tabs + H;
        ctx->tab_row64 = reinterpret_cast<double2 *>(tabs + W + H);
        ctx->tab_col64 = ctx->tab_row64 + H;
        const int n = W > H ? W : H;
        hipLaunchKernelGGL(pms::k_tables, dim3((n + 255) / 256), dim3(256), 0, stream, W, H,
                           ctx->tab_row, ctx->tab_col, ctx->tab_row64, ctx->tab_col64);
        e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(ctx, e, "k_tables launch");
        ctx->tab_W = W;
        ctx->tab_H = H;
    }
    ctx->cap_pixels = npx;
    return PMS_OK;
}

hipEvent_t take_event(pms_context *ctx)
{
    if (!ctx->event_pool.empty()) {
        hipEvent_t e = ctx->event_pool.back();
        ctx->event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

struct LaunchTimer {
    pms_context *ctx;
    int kind;
    hipStream_t stream;
    hipEvent_t a = nullptr, b = nullptr;
    LaunchTimer(pms_context *c, int k, hipStream_t s) : ctx(c), kind(k), stream(s)
    {
        if (ctx->profiling) {
            a = take_event(ctx);
            b = take_event(ctx);
            if (a) (void)hipEventRecord(a, stream);
        }
    }
    ~LaunchTimer()
    {
        if (ctx->profiling && a && b) {
            (void)hipEventRecord(b, stream);
            ctx->launches.push_back({kind, a, b});
        }
    }
};

void fill_common(pms::SweepArgs &A, const pms_context *ctx, const pms_image *ref,
                 const pms_pose *ref_pose, const pms_image *nbrs, const pms_pose *nbr_poses,
                 int n_nbrs, const pms_params *p)
{
    std::memset(&A, 0, sizeof A);
    const int W = ref->width, H = ref->height;
    A.W = W;
    A.H = H;
    A.r = (p->patch_size - 1) / 2;
    A.stride = p->patch_stride;
    A.side = 2 * A.r / A.stride + 1;
    A.P = A.side * A.side;
    A.inv_P = (float)(1.0 / A.P);
    A.n_views = n_nbrs;
    A.top_k = p->top_k > 0 ? p->top_k : (n_nbrs + 1) / 2;
    A.k_float = (float)A.top_k;
    A.var_floor = (float)p->ncc_var_floor;
    A.dmin = (float)p->depth_min;
    A.dmax = (float)p->depth_max;
    A.inv_dmin = (float)(1.0 / p->depth_min);
    A.inv_dmax = (float)(1.0 / p->depth_max);
    const double PI = 3.14159265358979323846;
    A.kx = (float)(W / (2.0 * PI));
    A.cx = (float)(W / 2.0 - 0.5);
    A.ky = (float)(-H / PI);
    A.cy = (float)(H / 2.0 - 0.5);
    // chord between bearings r pixels apart in x and y is at most their
    // angular distance, r (2 pi / W) + r (pi / H) = 2r (2 pi / W)
    A.patch_chord = (float)(2.0 * A.r * (2.0 * PI / W) * 1.001);
    A.n_offsets = p->n_offsets;
    for (int k = 0; k < p->n_offsets; ++k) {
        A.off_x[k] = p->offsets[k][0];
        A.off_y[k] = p->offsets[k][1];
    }
    A.refine_trials = p->refine_trials;
    const double sd0 = p->refine_sigma_logdepth0 > 0.0 ? p->refine_sigma_logdepth0
                                                       : 0.5 * std::log(p->depth_max / p->depth_min);
    for (int k = 0; k < p->refine_trials; ++k) {
        A.sd[k] = (float)(sd0 * std::pow(p->refine_depth_shrink, k));
        A.sn[k] = (float)(p->refine_sigma_normal0 * std::pow(p->refine_normal_shrink, k));
    }
    A.seed = p->seed;
    A.ref.ptr = ref->data;
    A.ref.pitch = ref->pitch_bytes;
    for (int j = 0; j < n_nbrs; ++j) {
        A.pad[j] = ctx->pad[j];
        A.pose[j] = relative_pose64(*ref_pose, nbr_poses[j]);
        A.posef[j] = relative_pose(*ref_pose, nbr_poses[j]);
    }
    A.Wp = ctx->pad_Wp;
    A.pad_bytes = ctx->pad_bytes;
    A.tab_row = ctx->tab_row;
    A.tab_col = ctx->tab_col;
    A.tab_row64 = ctx->tab_row64;
    A.tab_col64 = ctx->tab_col64;
    A.stats = ctx->stats;
    A.state = ctx->state;
    A.cost = ctx->cost;
}

// Lanes per pixel, samples per lane, and whether every lane owns exactly
// that many samples: a function of the patch size alone, so results never
// depend on launch shapes.
struct Variant {
    int lpp, spl;
    bool full;
};

#ifndef PMS_P36_LPP
#define PMS_P36_LPP 4
#endif

Variant pick_variant(int P)
{
    if (P == 36 && PMS_P36_LPP == 2) return {2, 18, true};
    if (P % 4 == 0 && (P / 4 == 9 || P / 4 == 16)) return {4, P / 4, true};
    const int need = (P + 3) / 4;
    return {4, need <= 4 ? 4 : need <= 9 ? 9 : need <= 13 ? 13 : 16, false};
}

// Tiles and grid for a launch over `cols` x `rows` pixels in (32/LPP) x 8
// tiles; the grid is padded to a multiple of the 8 XCDs.
dim3 tile_grid(pms::SweepArgs &A, int cols, int rows)
{
    const int tx = 32 / pick_variant(A.P).lpp;
    A.tiles_x = (cols + tx - 1) / tx;
    A.tiles_y = (rows + pms::TILE_Y - 1) / pms::TILE_Y;
    const int tiles = A.tiles_x * A.tiles_y;
    A.tiles_per_xcd = (tiles + 7) / 8;
    return dim3(8 * A.tiles_per_xcd);
}

template <int DT, int LPP, int SPL, bool FULL>
void launch_kernel(int kind, const pms::SweepArgs &A, dim3 grid, hipStream_t s)
{
    switch (kind) {
    case KK_INIT: hipLaunchKernelGGL((pms::k_init<DT, LPP, SPL, FULL>), grid, dim3(pms::BLOCK), 0, s, A); break;
    case KK_HALFSWEEP: hipLaunchKernelGGL((pms::k_halfsweep<DT, LPP, SPL, FULL>), grid, dim3(pms::BLOCK), 0, s, A); break;
    case KK_EVAL: hipLaunchKernelGGL((pms::k_eval<DT, LPP, SPL, FULL>), grid, dim3(pms::BLOCK), 0, s, A); break;
    default: break;
    }
}

template <int DT>
void launch_variant(int kind, const Variant &v, const pms::SweepArgs &A, dim3 grid, hipStream_t s)
{
    if (v.lpp == 2) launch_kernel<DT, 2, 18, true>(kind, A, grid, s);
    else if (v.full && v.spl == 9) launch_kernel<DT, 4, 9, true>(kind, A, grid, s);
    else if (v.full && v.spl == 16) launch_kernel<DT, 4, 16, true>(kind, A, grid, s);
    else if (v.spl == 4) launch_kernel<DT, 4, 4, false>(kind, A, grid, s);
    else if (v.spl == 9) launch_kernel<DT, 4, 9, false>(kind, A, grid, s);
    else if (v.spl == 13) launch_kernel<DT, 4, 13, false>(kind, A, grid, s);
    else launch_kernel<DT, 4, 16, false>(kind, A, grid, s);
}

pms_status launch(pms_context *ctx, int kind, int dtype, const pms::SweepArgs &A, dim3 grid,
                  hipStream_t s)
{
    LaunchTimer timer(ctx, kind, s);
    const Variant v = pick_variant(A.P);
    switch (dtype) {
    case PMS_F32: launch_variant<pms::DT_F32>(kind, v, A, grid, s); break;
    case PMS_F16: launch_variant<pms::DT_F16>(kind, v, A, grid, s); break;
    default: launch_variant<pms::DT_U8>(kind, v, A, grid, s); break;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(ctx, e, kKernelNames[kind]);
    return PMS_OK;
}

// Re-lays out the neighbour images into the context's scratch.
pms_status launch_pad(pms_context *ctx, const pms_image *nbrs, int n_nbrs, hipStream_t s)
{
    LaunchTimer timer(ctx, KK_IO, s);
    const int W = nbrs[0].width, H = nbrs[0].height, Wp = ctx->pad_Wp;
    const long long n = (long long)(H + 2) * Wp;
    dim3 grid((unsigned)((n + pms::BLOCK - 1) / pms::BLOCK));
    for (int j = 0; j < n_nbrs; ++j) {
        pms::ImgRef src{nbrs[j].data, nbrs[j].pitch_bytes};
        switch (nbrs[j].dtype) {
        case PMS_F32:
            hipLaunchKernelGGL(pms::k_pad<pms::DT_F32>, grid, dim3(pms::BLOCK), 0, s, src, W, H, Wp,
                               static_cast<float *>(ctx->pad[j]));
            break;
        case PMS_F16:
            hipLaunchKernelGGL(pms::k_pad<pms::DT_F16>, grid, dim3(pms::BLOCK), 0, s, src, W, H, Wp,
                               static_cast<__half *>(ctx->pad[j]));
            break;
        default:
            hipLaunchKernelGGL(pms::k_pad<pms::DT_U8>, grid, dim3(pms::BLOCK), 0, s, src, W, H, Wp,
                               static_cast<float *>(ctx->pad[j]));
            break;
        }
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(ctx, e, "pad");
    return PMS_OK;
}

pms_status launch_refstats(pms_context *ctx, int dtype, const pms::SweepArgs &A, hipStream_t s)
{
    LaunchTimer timer(ctx, KK_REFSTATS, s);
    const long long n = (long long)A.W * A.H;
    dim3 grid((unsigned)((n + pms::BLOCK - 1) / pms::BLOCK));
    switch (dtype) {
    case PMS_F32: hipLaunchKernelGGL(pms::k_refstats<pms::DT_F32>, grid, dim3(pms::BLOCK), 0, s, A); break;
    case PMS_F16: hipLaunchKernelGGL(pms::k_refstats<pms::DT_F16>, grid, dim3(pms::BLOCK), 0, s, A); break;
    default: hipLaunchKernelGGL(pms::k_refstats<pms::DT_U8>, grid, dim3(pms::BLOCK), 0, s, A); break;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(ctx, e, "refstats");
    return PMS_OK;
}

pms::IoArgs io_args(pms_context *ctx, int W, int H, int r, pms_plane depth,
                    const pms_plane normal[3], pms_plane cost)
{
    pms::IoArgs io;
    io.W = W;
    io.H = H;
    io.r = r;
    io.state = ctx->state;
    io.cost = ctx->cost;
    io.depth = depth.data;
    io.n0 = normal[0].data;
    io.n1 = normal[1].data;
    io.n2 = normal[2].data;
    io.cplane = cost.data;
    io.pd = depth.pitch_elems;
    io.pn0 = normal[0].pitch_elems;
    io.pn1 = normal[1].pitch_elems;
    io.pn2 = normal[2].pitch_elems;
    io.pc = cost.pitch_elems;
    return io;
}

bool check_outputs(pms_context *ctx, int W, pms_plane depth, const pms_plane normal[3],
                   pms_plane cost, pms_status *st)
{
    if (!normal) {
        *st = fail(ctx, PMS_ERR_INVALID_ARG, "normal planes are null");
        return false;
    }
    return check_plane(ctx, depth, W, "depth", st) && check_plane(ctx, normal[0], W, "normal[0]", st) &&
           check_plane(ctx, normal[1], W, "normal[1]", st) &&
           check_plane(ctx, normal[2], W, "normal[2]", st) && check_plane(ctx, cost, W, "cost", st);
}

bool check_maps(pms_context *ctx, const pms_plane *maps, const pms_pose *map_poses, int n_maps,
                int W, pms_status *st)
{
    if (n_maps < 0 || n_maps > PMS_MAX_MAPS) {
        *st = fail(ctx, PMS_ERR_INVALID_ARG, "n_maps must be in [0, 8]");
        return false;
    }
    if (n_maps == 0) return true;
    if (!maps || !map_poses) {
        *st = fail(ctx, PMS_ERR_INVALID_ARG, "null consistency maps or poses");
        return false;
    }
    for (int k = 0; k < n_maps; ++k) {
        if (!check_plane(ctx, maps[k], W, "consistency map", st)) return false;
        if (!finite_pose(map_poses[k])) {
            *st = fail(ctx, PMS_ERR_INVALID_ARG, "non-finite map pose");
            return false;
        }
    }
    return true;
}

pms_status launch_consistency(pms_context *ctx, int W, int H, int r, const pms_pose *ref_pose,
                              const pms_plane *maps, const pms_pose *map_poses, int n_maps,
                              const pms_params *p, pms_plane depth, const pms_plane normal[3],
                              pms_plane cost, hipStream_t s)
{
    pms::GeoArgs G;
    std::memset(&G, 0, sizeof G);
    G.W = W;
    G.H = H;
    G.r = r;
    G.n_maps = n_maps;
    G.min_views = p->geo_min_views > 0 ? p->geo_min_views : (n_maps < 2 ? n_maps : 2);
    G.geo_px = (float)p->geo_px;
    G.geo_rel = (float)p->geo_rel_depth;
    const double PI = 3.14159265358979323846;
    G.kx = (float)(W / (2.0 * PI));
    G.cx = (float)(W / 2.0 - 0.5);
    G.ky = (float)(-H / PI);
    G.cy = (float)(H / 2.0 - 0.5);
    G.tab_row = ctx->tab_row;
    G.tab_col = ctx->tab_col;
    for (int k = 0; k < n_maps; ++k) {
        G.pose[k] = relative_pose(*ref_pose, map_poses[k]);
        G.map[k] = maps[k].data;
        G.map_pitch[k] = maps[k].pitch_elems;
    }
    G.depth = depth.data;
    G.n0 = normal[0].data;
    G.n1 = normal[1].data;
    G.n2 = normal[2].data;
    G.cost = cost.data;
    G.pd = depth.pitch_elems;
    G.pn0 = normal[0].pitch_elems;
    G.pn1 = normal[1].pitch_elems;
    G.pn2 = normal[2].pitch_elems;
    G.pc = cost.pitch_elems;
    LaunchTimer timer(ctx, KK_CONSISTENCY, s);
    const long long n = (long long)W * H;
    hipLaunchKernelGGL(pms::k_consistency, dim3((unsigned)((n + pms::BLOCK - 1) / pms::BLOCK)),
                       dim3(pms::BLOCK), 0, s, G);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(ctx, e, "consistency");
    return PMS_OK;
}

pms_status launch_io(pms_context *ctx, int which, const pms::IoArgs &io, int colour, hipStream_t s)
{
    LaunchTimer timer(ctx, which == 0 ? KK_FINALIZE : KK_IO, s);
    const long long n = (long long)io.W * io.H;
    dim3 grid((unsigned)((n + pms::BLOCK - 1) / pms::BLOCK));
    if (which == 0)
        hipLaunchKernelGGL(pms::k_finalize, grid, dim3(pms::BLOCK), 0, s, io);
    else if (which == 1)
        hipLaunchKernelGGL(pms::k_load_state, grid, dim3(pms::BLOCK), 0, s, io);
    else
        hipLaunchKernelGGL(pms::k_store_colour, grid, dim3(pms::BLOCK), 0, s, io, colour);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(ctx, e, "state io");
    return PMS_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------

extern "C" {

pms_status pms_default_params(pms_params *out)
{
    if (!out) return PMS_ERR_INVALID_ARG;
    std::memset(out, 0, sizeof *out);
    out->patch_size = 11;
    out->patch_stride = 2;
    out->iterations = 8;
    out->refine_trials = 6;
    out->depth_min = 0.3;
    out->depth_max = 30.0;
    out->top_k = 0;
    out->ncc_var_floor = 1e-6;
    out->refine_sigma_logdepth0 = 0.0;
    out->refine_depth_shrink = 0.25;
    out->refine_sigma_normal0 = 1.0;
    out->refine_normal_shrink = 0.5;
    static const int32_t ring[8][2] = {{-3, 0}, {3, 0}, {0, -3}, {0, 3},
                                       {-5, 0}, {5, 0}, {0, -5}, {0, 5}};
    out->n_offsets = 8;
    std::memcpy(out->offsets, ring, sizeof ring);
    out->geo_px = 1.0;
    out->geo_rel_depth = 0.01;
    out->geo_min_views = 0;
    out->seed = 0;
    return PMS_OK;
}

pms_status pms_context_create(int32_t device, size_t scratch_budget_bytes, pms_context **out)
{
    if (!out) return PMS_ERR_INVALID_ARG;
    *out = nullptr;
    if (device != -1) {
        int n = 0;
        if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return PMS_ERR_DEVICE;
    }
    pms_context *ctx = new (std::nothrow) pms_context();
    if (!ctx) return PMS_ERR_OUT_OF_MEMORY;
    ctx->device = device;
    ctx->budget = scratch_budget_bytes;
    *out = ctx;
    return PMS_OK;
}

pms_status pms_context_destroy(pms_context *ctx)
{
    if (!ctx) return PMS_ERR_INVALID_ARG;
    if (ctx->device >= 0) {
        (void)hipSetDevice(ctx->device);
        (void)hipDeviceSynchronize();
    }
    if (ctx->scratch) (void)hipFree(ctx->scratch);
    for (auto &l : ctx->launches) {
        (void)hipEventDestroy(l.start);
        (void)hipEventDestroy(l.stop);
    }
    for (auto e : ctx->event_pool) (void)hipEventDestroy(e);
    delete ctx;
    return PMS_OK;
}

pms_status pms_densify(pms_context *ctx, const pms_image *ref, const pms_pose *ref_pose,
                       const pms_image *nbrs, const pms_pose *nbr_poses, int32_t n_nbrs,
                       const pms_plane *maps, const pms_pose *map_poses, int32_t n_maps,
                       const pms_params *params, pms_plane depth_out,
                       const pms_plane normal_out[3], pms_plane cost_out, void *stream)
{
    if (!ctx) return PMS_ERR_INVALID_ARG;
    ctx->last_error.clear();
    pms_status st = PMS_OK;
    if (!check_ref_and_views(ctx, ref, ref_pose, nbrs, nbr_poses, n_nbrs, &st)) return st;
    const int W = ref->width, H = ref->height;
    if (!check_params(ctx, params, W, H, n_nbrs, &st)) return st;
    if (!check_outputs(ctx, W, depth_out, normal_out, cost_out, &st)) return st;
    if (!check_maps(ctx, maps, map_poses, n_maps, W, &st)) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if ((st = ensure_scratch(ctx, W, H, n_nbrs, pad_elem_size(ref->dtype), s)) != PMS_OK) return st;

    pms::SweepArgs A;
    fill_common(A, ctx, ref, ref_pose, nbrs, nbr_poses, n_nbrs, params);
    if ((st = launch_pad(ctx, nbrs, n_nbrs, s)) != PMS_OK) return st;
    if ((st = launch_refstats(ctx, ref->dtype, A, s)) != PMS_OK) return st;
    dim3 g_all = tile_grid(A, W, H);
    if ((st = launch(ctx, KK_INIT, ref->dtype, A, g_all, s)) != PMS_OK) return st;
    pms::SweepArgs B = A;
    const int rows = H - 2 * A.r;
    if (rows > 0) {
        dim3 g_half = tile_grid(B, W / 2, rows);
        for (int it = 1; it <= params->iterations; ++it)
            for (int colour = 0; colour < 2; ++colour) {
                B.iteration = it;
                B.colour = colour;
                if ((st = launch(ctx, KK_HALFSWEEP, ref->dtype, B, g_half, s)) != PMS_OK) return st;
            }
    }
    pms::IoArgs io = io_args(ctx, W, H, A.r, depth_out, normal_out, cost_out);
    if ((st = launch_io(ctx, 0, io, 0, s)) != PMS_OK) return st;
    if (n_maps > 0)
        return launch_consistency(ctx, W, H, A.r, ref_pose, maps, map_poses, n_maps, params,
                                  depth_out, normal_out, cost_out, s);
    return PMS_OK;
}

pms_status pms_eval_cost(pms_context *ctx, const pms_image *ref, const pms_pose *ref_pose,
                         const pms_image *nbrs, const pms_pose *nbr_poses, int32_t n_nbrs,
                         const pms_params *params, pms_plane depth_in,
                         const pms_plane normal_in[3], pms_plane cost_out,
                         const pms_plane *per_view_out, void *stream)
{
    if (!ctx) return PMS_ERR_INVALID_ARG;
    ctx->last_error.clear();
    pms_status st = PMS_OK;
    if (!check_ref_and_views(ctx, ref, ref_pose, nbrs, nbr_poses, n_nbrs, &st)) return st;
    const int W = ref->width, H = ref->height;
    if (!check_params(ctx, params, W, H, n_nbrs, &st)) return st;
    if (!check_outputs(ctx, W, depth_in, normal_in, cost_out, &st)) return st;
    const int64_t pitch = depth_in.pitch_elems;
    if (normal_in[0].pitch_elems != pitch || normal_in[1].pitch_elems != pitch ||
        normal_in[2].pitch_elems != pitch)
        return fail(ctx, PMS_ERR_INVALID_ARG, "depth_in and normal_in must share one pitch");
    if (per_view_out) {
        for (int j = 0; j < n_nbrs; ++j) {
            if (!check_plane(ctx, per_view_out[j], W, "per_view_out", &st)) return st;
            if (per_view_out[j].pitch_elems != cost_out.pitch_elems)
                return fail(ctx, PMS_ERR_INVALID_ARG, "per_view_out must share cost_out's pitch");
        }
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    if ((st = ensure_scratch(ctx, W, H, n_nbrs, pad_elem_size(ref->dtype), s)) != PMS_OK) return st;
    pms::SweepArgs A;
    fill_common(A, ctx, ref, ref_pose, nbrs, nbr_poses, n_nbrs, params);
    if ((st = launch_pad(ctx, nbrs, n_nbrs, s)) != PMS_OK) return st;
    A.in_depth = depth_in.data;
    A.in_n0 = normal_in[0].data;
    A.in_n1 = normal_in[1].data;
    A.in_n2 = normal_in[2].data;
    A.in_pitch = pitch;
    A.out_cost = cost_out.data;
    A.out_pitch = cost_out.pitch_elems;
    for (int j = 0; j < n_nbrs; ++j) A.view_out[j] = per_view_out ? per_view_out[j].data : nullptr;
    if ((st = launch_refstats(ctx, ref->dtype, A, s)) != PMS_OK) return st;
    dim3 g = tile_grid(A, W, H);
    return launch(ctx, KK_EVAL, ref->dtype, A, g, s);
}

pms_status pms_halfsweep(pms_context *ctx, const pms_image *ref, const pms_pose *ref_pose,
                         const pms_image *nbrs, const pms_pose *nbr_poses, int32_t n_nbrs,
                         const pms_params *params, int32_t iteration, int32_t colour,
                         pms_plane depth_io, const pms_plane normal_io[3], pms_plane cost_io,
                         void *stream)
{
    if (!ctx) return PMS_ERR_INVALID_ARG;
    ctx->last_error.clear();
    pms_status st = PMS_OK;
    if (!check_ref_and_views(ctx, ref, ref_pose, nbrs, nbr_poses, n_nbrs, &st)) return st;
    const int W = ref->width, H = ref->height;
    if (!check_params(ctx, params, W, H, n_nbrs, &st)) return st;
    if (!check_outputs(ctx, W, depth_io, normal_io, cost_io, &st)) return st;
    if (iteration < 1) return fail(ctx, PMS_ERR_INVALID_ARG, "iteration must be >= 1");
    if (colour != 0 && colour != 1) return fail(ctx, PMS_ERR_INVALID_ARG, "colour must be 0 or 1");
    hipStream_t s = static_cast<hipStream_t>(stream);
    if ((st = ensure_scratch(ctx, W, H, n_nbrs, pad_elem_size(ref->dtype), s)) != PMS_OK) return st;
    pms::SweepArgs A;
    fill_common(A, ctx, ref, ref_pose, nbrs, nbr_poses, n_nbrs, params);
    if ((st = launch_pad(ctx, nbrs, n_nbrs, s)) != PMS_OK) return st;
    pms::IoArgs io = io_args(ctx, W, H, A.r, depth_io, normal_io, cost_io);
    if ((st = launch_io(ctx, 1, io, 0, s)) != PMS_OK) return st;
    if ((st = launch_refstats(ctx, ref->dtype, A, s)) != PMS_OK) return st;
    const int rows = H - 2 * A.r;
    if (rows > 0) {
        dim3 g = tile_grid(A, W / 2, rows);
        A.iteration = iteration;
        A.colour = colour;
        if ((st = launch(ctx, KK_HALFSWEEP, ref->dtype, A, g, s)) != PMS_OK) return st;
    }
    return launch_io(ctx, 2, io, colour, s);
}

pms_status pms_consistency(pms_context *ctx, int32_t width, int32_t height,
                           const pms_pose *ref_pose, const pms_plane *maps,
                           const pms_pose *map_poses, int32_t n_maps, const pms_params *params,
                           pms_plane depth_io, const pms_plane normal_io[3], pms_plane cost_io,
                           void *stream)
{
    if (!ctx) return PMS_ERR_INVALID_ARG;
    ctx->last_error.clear();
    pms_status st = PMS_OK;
    if (height < 1 || width != 2 * height)
        return fail(ctx, PMS_ERR_INVALID_ARG, "size must be W x H with W == 2H >= 2");
    if (!ref_pose || !finite_pose(*ref_pose))
        return fail(ctx, PMS_ERR_INVALID_ARG, "null or non-finite reference pose");
    if (!check_params(ctx, params, width, height, 0, &st)) return st;
    if (n_maps < 1) return fail(ctx, PMS_ERR_INVALID_ARG, "need at least one map");
    if (!check_maps(ctx, maps, map_poses, n_maps, width, &st)) return st;
    if (!check_outputs(ctx, width, depth_io, normal_io, cost_io, &st)) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if ((st = ensure_scratch(ctx, width, height, 0, 4, s)) != PMS_OK) return st;
    return launch_consistency(ctx, width, height, (params->patch_size - 1) / 2, ref_pose, maps,
                              map_poses, n_maps, params, depth_io, normal_io, cost_io, s);
}

pms_status pms_philox_stream(pms_context *ctx, uint64_t key0, uint64_t key1, uint64_t ctr0,
                             int64_t n, uint64_t *out, void *stream)
{
    if (!ctx) return PMS_ERR_INVALID_ARG;
    ctx->last_error.clear();
    if (n < 0 || (n > 0 && !out)) return fail(ctx, PMS_ERR_INVALID_ARG, "bad n or null out");
    if (n == 0) return PMS_OK;
    if (n > (int64_t)1 << 31) return fail(ctx, PMS_ERR_INVALID_ARG, "n too large");
    if (ctx->device < 0) return fail(ctx, PMS_ERR_DEVICE, "validation-only context cannot launch");
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_fail(ctx, e, "hipSetDevice");
    hipLaunchKernelGGL(pms::k_philox, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                       static_cast<hipStream_t>(stream), (unsigned long long)key0,
                       (unsigned long long)key1, (unsigned long long)ctr0, (long long)n,
                       reinterpret_cast<unsigned long long *>(out));
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(ctx, e, "philox");
    return PMS_OK;
}

pms_status pms_profile_enable(pms_context *ctx, int32_t on)
{
    if (!ctx) return PMS_ERR_INVALID_ARG;
    ctx->profiling = on != 0;
    return PMS_OK;
}

pms_status pms_profile_read(pms_context *ctx, const char *name, int64_t *launches, double *total_ms)
{
    if (!ctx || !name || !launches || !total_ms) return PMS_ERR_INVALID_ARG;
    int kind = -1;
    for (int k = 0; k < kNumKernelKinds; ++k)
        if (std::strcmp(name, kKernelNames[k]) == 0) kind = k;
    if (kind < 0) return fail(ctx, PMS_ERR_INVALID_ARG, "unknown kernel name");
    *launches = 0;
    *total_ms = 0.0;
    std::vector<TimedLaunch> keep;
    for (auto &l : ctx->launches) {
        if (l.kind != kind) {
            keep.push_back(l);
            continue;
        }
        hipError_t e = hipEventSynchronize(l.stop);
        if (e != hipSuccess) return hip_fail(ctx, e, "hipEventSynchronize");
        float ms = 0.0f;
        e = hipEventElapsedTime(&ms, l.start, l.stop);
        if (e != hipSuccess) return hip_fail(ctx, e, "hipEventElapsedTime");
        *launches += 1;
        *total_ms += ms;
        ctx->event_pool.push_back(l.start);
        ctx->event_pool.push_back(l.stop);
    }
    ctx->launches.swap(keep);
    return PMS_OK;
}

const char *pms_status_string(pms_status s)
{
    switch (s) {
    case PMS_OK: return "ok";
    case PMS_ERR_INVALID_ARG: return "invalid argument";
    case PMS_ERR_OUT_OF_MEMORY: return "out of memory";
    case PMS_ERR_DEVICE: return "device error";
    case PMS_ERR_UNSUPPORTED: return "unsupported";
    case PMS_ERR_BUDGET: return "scratch budget exceeded";
    default: return "unknown status";
    }
}

const char *pms_last_error(const pms_context *ctx)
{
    return ctx ? ctx->last_error.c_str() : "";
}

}  // extern "C"
