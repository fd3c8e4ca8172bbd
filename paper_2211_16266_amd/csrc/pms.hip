// pms.hip -- host side of libpms: argument validation, FP64 pose
// composition, device memory and the launch plans behind the C ABI declared
// in include/pms.h.
//
// Every computation is described as a plan: a table of per-job kernel
// arguments (JobArgs), per-launch entry lists naming which job (and, for a
// half-sweep, which iteration and colour) each range of workgroups serves,
// and the ordered list of launches. One keyframe (pms_densify), a batch of
// uneven keyframes (pms_densify_batch, pms_batch_*) and the serving loop's
// ticks (pms_server_*) all run through the same kernels; a pixel's
// arithmetic does not depend on which other jobs share its launch or on the
// tile shape.
#include "pms.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <tuple>
#include <utility>
#include <vector>

#include "pms_kernels.hpp"

namespace {

constexpr int kNumKernelKinds = 13;
const char *const kKernelNames[kNumKernelKinds] = {"refstats", "init", "halfsweep", "finalize",
                                                   "consistency", "eval", "io", "batch", "warp",
                                                   "median", "fuse", "coverage", "view_filter"};
enum KernelKind {
    KK_REFSTATS, KK_INIT, KK_HALFSWEEP, KK_FINALIZE, KK_CONSISTENCY, KK_EVAL, KK_IO, KK_GRAPH, KK_WARP,
    KK_MEDIAN, KK_FUSE, KK_COVER, KK_VIEW
};

struct TimedLaunch {
    int kind;
    hipEvent_t start, stop;
};

// Bearing tables of one image size, built once per context and size.
struct Tables {
    float2 *row = nullptr, *col = nullptr;
    double2 *row64 = nullptr, *col64 = nullptr;
};

// Pinned host buffers for argument uploads, reused in turn; a buffer is
// rewritten only after the copy that last read it has run.
constexpr int kStagingSlots = 4;
struct Staging {
    void *host = nullptr;
    size_t cap = 0;
    hipEvent_t done = nullptr;
};

// Tile shape and patch schedule used by every launch of a context.
struct Schedule {
    int wy_log2 = 2;  // a wave covers 2^wy_log2 pixel rows
    int bx_log2 = 1;  // a workgroup holds 2^bx_log2 waves side by side
    int lpp = 0;      // lanes per pixel: 2 for 36-sample patches, 8 for
                      // 64-sample ones, 0 for 4 everywhere
};

}  // namespace

struct pms_context {
    int device = 0;
    size_t budget = 0;
    // device block of the calls that run one plan at a time: argument
    // tables first, then per-job plane state and re-laid-out images
    void *work = nullptr;  // stream-ordered allocation (hipMallocAsync)
    size_t work_bytes = 0;
    hipEvent_t work_used = nullptr;  // recorded after the last plan using it
    std::map<std::pair<int, int>, Tables> tables;
    Staging staging[kStagingSlots];
    int staging_next = 0;
    Schedule sched;
    hipStream_t capture_stream = nullptr;
    bool capturing = false;
    std::string last_error;
    bool profiling = false;
    // executed-work counters of the half-sweeps (pms_work_count_*)
    bool work_counts_on = false;
    unsigned long long *work_counts = nullptr;
    std::vector<char> noalloc_host;  // pageable upload buffer of pms_densify_noalloc
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
    if (p->top_k > PMS_MAX_TOP_K || (p->top_k == 0 && (n_views + 1) / 2 > PMS_MAX_TOP_K)) {
        *st = fail(ctx, PMS_ERR_UNSUPPORTED, "more than 4 views averaged");
        return false;
    }
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
    if (p->median_radius < 0 || p->median_radius > 8 || !(p->median_rel >= 0.0) ||
        !std::isfinite(p->median_rel))
        return bad("median_radius must be in [0, 8] and median_rel >= 0");
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
    if (H > PMS_MAX_HEIGHT) {
        *st = fail(ctx, PMS_ERR_INVALID_ARG, "image height above PMS_MAX_HEIGHT");
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
    out.tnorm = (float)(std::sqrt(t[0] * t[0] + t[1] * t[1] + t[2] * t[2]) * (1.0 + 1e-6));
    return out;
}

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// A re-laid-out image holds (H + 1) rows of 2W + 4 bilinear cells: 16 bytes
// (corner value and its three differences in FP32) for FP32 images, 8 bytes
// for FP16 (the four corners as halves) and 8-bit ones (corner and three
// differences of the raw values, as halves).
size_t pad_elem_size(int dtype) { return dtype == PMS_F32 ? sizeof(float4) : dtype == PMS_F16 ? sizeof(pms::Cell8) : sizeof(pms::Cell8d); }
long long pad_cells(int W, int H) { return (long long)(H + 1) * (2 * (long long)W + 4); }

pms_status set_device(pms_context *ctx)
{
    if (ctx->device < 0) return fail(ctx, PMS_ERR_DEVICE, "validation-only context cannot launch");
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_fail(ctx, e, "hipSetDevice");
    return PMS_OK;
}

// Bearing tables of a W x H image: per row sin/cos of the latitude, per
// column sin/cos of the longitude, FP64 and rounded to FP32, laid out as
// [row f32 | col f32 | row f64 | col f64].
size_t tables_bytes(int W, int H) { return ((size_t)W + H) * (sizeof(float2) + sizeof(double2)); }

void fill_tables_host(int W, int H, char *host)
{
    const size_t n = (size_t)W + H;
    float2 *row = reinterpret_cast<float2 *>(host);
    float2 *col = row + H;
    double2 *row64 = reinterpret_cast<double2 *>(row + n);
    double2 *col64 = row64 + H;
    const double PI = 3.14159265358979323846;
    for (int i = 0; i < H; ++i) {
        const double phi = PI / 2.0 - PI * (i + 0.5) / H;
        row64[i] = make_double2(std::sin(phi), std::cos(phi));
        row[i] = make_float2((float)row64[i].x, (float)row64[i].y);
    }
    for (int i = 0; i < W; ++i) {
        const double lam = 2.0 * PI * (i + 0.5) / W - PI;
        col64[i] = make_double2(std::sin(lam), std::cos(lam));
        col[i] = make_float2((float)col64[i].x, (float)col64[i].y);
    }
}

// The table pointers of a block laid out by fill_tables_host at `dev`.
Tables tables_at(void *dev, int W, int H)
{
    const size_t n = (size_t)W + H;
    Tables t;
    t.row = static_cast<float2 *>(dev);
    t.col = t.row + H;
    t.row64 = reinterpret_cast<double2 *>(t.row + n);
    t.col64 = t.row64 + H;
    return t;
}

// Bearing tables computed on the host once per size and kept for the
// context's lifetime.
pms_status get_tables(pms_context *ctx, int W, int H, Tables *out)
{
    auto it = ctx->tables.find({W, H});
    if (it != ctx->tables.end()) {
        *out = it->second;
        return PMS_OK;
    }
    std::vector<char> host(tables_bytes(W, H));
    fill_tables_host(W, H, host.data());
    void *dev = nullptr;
    hipError_t e = hipMalloc(&dev, host.size());
    if (e != hipSuccess) return fail(ctx, PMS_ERR_OUT_OF_MEMORY, "hipMalloc of bearing tables failed");
    e = hipMemcpy(dev, host.data(), host.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(dev);
        return hip_fail(ctx, e, "bearing table upload");
    }
    const Tables t = tables_at(dev, W, H);
    ctx->tables[{W, H}] = t;
    *out = t;
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
        if (kind >= 0 && ctx->profiling && !ctx->capturing) {
            a = take_event(ctx);
            b = take_event(ctx);
            if (a) (void)hipEventRecord(a, stream);
        }
    }
    ~LaunchTimer()
    {
        if (a && b) {
            (void)hipEventRecord(b, stream);
            ctx->launches.push_back({kind, a, b});
        }
    }
};

// Lanes per pixel, samples per lane, and whether every lane owns exactly
// that many samples: a function of the patch size and the context's
// schedule, never of the launch.
struct Variant {
    int lpp, spl;
    bool full;
};

Variant pick_variant(int P, const Schedule &sc)
{
    if (P == 36 && sc.lpp == 2) return {2, 18, true};
    if (P == 64 && sc.lpp == 8) return {8, 8, true};
    if (P % 4 == 0 && (P / 4 == 9 || P / 4 == 16)) return {4, P / 4, true};
    const int need = (P + 3) / 4;
    return {4, need <= 4 ? 4 : need <= 9 ? 9 : need <= 13 ? 13 : 16, false};
}

int ilog2(int v)
{
    int l = 0;
    while ((1 << (l + 1)) <= v) ++l;
    return l;
}

enum Mode { MODE_DENSIFY, MODE_EVAL, MODE_SWEEP, MODE_GEO };

// One validated job of a plan.
struct JobSpec {
    int mode = MODE_DENSIFY;
    int W = 0, H = 0;
    const pms_image *ref = nullptr;
    const pms_pose *ref_pose = nullptr;
    const pms_image *nbrs = nullptr;
    const pms_pose *nbr_poses = nullptr;
    int n_nbrs = 0;
    const pms_plane *maps = nullptr;
    const pms_pose *map_poses = nullptr;
    int n_maps = 0;
    const pms_params *p = nullptr;
    pms_plane depth{}, normal[3]{}, cost{};  // outputs, or in/out planes
    pms_plane depth_in{}, normal_in[3]{};    // MODE_EVAL hypotheses
    pms_plane init_depth{}, init_normal[3]{};  // MODE_DENSIFY initial planes (optional)
    const pms_plane *per_view = nullptr;     // MODE_EVAL, nullable
    int iteration = 0, colour = 0;           // MODE_SWEEP
};

// Tile geometry of one job under a schedule.
struct Geometry {
    Variant v;
    int r, wx_log2, wy_log2, bx_log2, tile_w, tile_h;
    int tiles_x_all, tiles_y_all, tiles_x_half, tiles_y_half;
};

Geometry geometry(const JobSpec &J, const Schedule &sc)
{
    Geometry g;
    g.v = pick_variant(patch_samples(*J.p), sc);
    g.r = (J.p->patch_size - 1) / 2;
    const int pix_log2 = ilog2(64 / g.v.lpp);  // pixels per wave
    g.wy_log2 = std::min(sc.wy_log2, pix_log2);
    g.wx_log2 = pix_log2 - g.wy_log2;
    g.bx_log2 = sc.bx_log2;
    g.tile_w = (1 << g.wx_log2) << g.bx_log2;
    g.tile_h = (1 << g.wy_log2) * (4 >> g.bx_log2);
    g.tiles_x_all = (J.W + g.tile_w - 1) / g.tile_w;
    g.tiles_y_all = (J.H + g.tile_h - 1) / g.tile_h;
    const int rows = J.H - 2 * g.r;
    g.tiles_x_half = (J.W / 2 + g.tile_w - 1) / g.tile_w;
    g.tiles_y_half = rows > 0 ? (rows + g.tile_h - 1) / g.tile_h : 0;
    return g;
}

// A launch of a plan: kernel kind, the entry list it walks, and for the
// state hooks the job they copy.
enum IoSub { IO_PAD = 0, IO_LOAD = 1, IO_STORE = 2 };
struct Rec {
    int kind;
    int sub;
    int dtype;
    Variant v;
    size_t entry_off;
    int n_entries;
    int total;  // workgroup slots per XCD (the grid is 8 x total)
    int job, colour;
};

struct Plan {
    std::vector<pms::JobArgs> jobs;
    std::vector<pms::PadJob> pads;
    std::vector<pms::Entry> entries;
    std::vector<Rec> recs;
    size_t off_pads = 0, off_entries = 0, args_bytes = 0, total_bytes = 0;
};

// Appends a launch over (job, tiles, iteration, colour) items.
void add_rec(Plan &P, int kind, int sub, int dtype, Variant v,
             const std::vector<std::tuple<int, int, int, int>> &items)
{
    Rec R{};
    R.kind = kind;
    R.sub = sub;
    R.dtype = dtype;
    R.v = v;
    R.entry_off = P.entries.size();
    int first = 0;
    for (auto &it : items) {
        const int tiles = std::get<1>(it);
        if (tiles <= 0) continue;
        const int per_xcd = (tiles + 7) / 8;
        P.entries.push_back({std::get<0>(it), first, tiles, per_xcd, std::get<2>(it), std::get<3>(it)});
        first += per_xcd;
    }
    R.n_entries = (int)(P.entries.size() - R.entry_off);
    if (R.n_entries == 0) {
        P.entries.resize(R.entry_off);
        return;
    }
    P.entries.push_back({-1, first, 0, 0, 0, 0});
    R.total = first;
    P.recs.push_back(R);
}

long long blocks_of(long long n) { return (n + pms::BLOCK - 1) / pms::BLOCK; }
// workgroups of the median filter: one per MED_TW x MED_TH tile
int median_tiles(int W, int H)
{
    return ((W + pms::MED_TW - 1) / pms::MED_TW) * ((H + pms::MED_TH - 1) / pms::MED_TH);
}
// grid of a counting kernel over n items (at least one workgroup: every
// workgroup adds its count, zero included, after a barrier)
unsigned count_grid(long long n) { return (unsigned)std::max(1LL, std::min(blocks_of(n), (long long)pms::COUNT_GRID)); }

using GroupKey = std::tuple<int, int, int, int>;  // dtype, lpp, spl, full
GroupKey group_key(const JobSpec &J, const Geometry &g)
{
    return GroupKey(J.ref->dtype, g.v.lpp, g.v.spl, g.v.full ? 1 : 0);
}

void fill_sweep_args(pms::SweepArgs &A, const JobSpec &J, const Geometry &g, const Tables &T)
{
    const pms_params *p = J.p;
    const int W = J.W, H = J.H;
    A.W = W;
    A.H = H;
    A.r = g.r;
    A.stride = p->patch_stride;
    A.side = 2 * A.r / A.stride + 1;
    A.P = A.side * A.side;
    A.inv_P = (float)(1.0 / A.P);
    A.n_views = J.n_nbrs;
    A.top_k = p->top_k > 0 ? p->top_k : (J.n_nbrs + 1) / 2;
    A.inv_k = (float)(1.0 / A.top_k);
    A.var_floor = (float)p->ncc_var_floor;
    A.var_floor_s = (float)(J.ref->dtype == PMS_U8 ? p->ncc_var_floor * 255.0 * 255.0 : p->ncc_var_floor);
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
    // |b_q - b_p| <= sqrt(dphi^2 + dlam^2) <= sqrt(2) r (2 pi / W) for the
    // samples within r pixels of the centre (rows and columns both span
    // 2 pi / W per pixel)
    A.patch_chord = (float)(std::sqrt(2.0) * A.r * (2.0 * PI / W) * 1.001);
    A.n_offsets = p->n_offsets;
    for (int k = 0; k < p->n_offsets; ++k) {
        A.off_x[k] = p->offsets[k][0];
        A.off_y[k] = p->offsets[k][1];
    }
    A.refine_trials = p->refine_trials;
    const double sd0 = p->refine_sigma_logdepth0 > 0.0 ? p->refine_sigma_logdepth0
                                                       : 0.5 * std::log(p->depth_max / p->depth_min);
    for (int k = 0; k < p->refine_trials; ++k) {
        // (in log2 units: the kernel scales the depth by a power of two)
        A.sd[k] = (float)(sd0 * std::pow(p->refine_depth_shrink, k) / std::log(2.0));
        A.sn[k] = (float)(p->refine_sigma_normal0 * std::pow(p->refine_normal_shrink, k));
    }
    A.seed = p->seed;
    A.wx_log2 = g.wx_log2;
    A.bx_log2 = g.bx_log2;
    A.tile_w = g.tile_w;
    A.tile_h = g.tile_h;
    A.tiles_x_all = g.tiles_x_all;
    A.tiles_x_half = g.tiles_x_half;
    A.ref_dtype = J.ref->dtype;
    // the half-sweep test hook starts from caller-given costs
    A.own_costs = J.mode == MODE_SWEEP ? 0 : 1;
    A.ref.ptr = J.ref->data;
    A.ref.pitch = J.ref->pitch_bytes;
    for (int j = 0; j < J.n_nbrs; ++j) {
        A.pose[j] = relative_pose64(*J.ref_pose, J.nbr_poses[j]);
        A.posef[j] = relative_pose(*J.ref_pose, J.nbr_poses[j]);
    }
    A.Wp = 2 * W + 4;
    A.pad_bytes = (int)((size_t)pad_cells(W, H) * pad_elem_size(J.ref->dtype));
    A.tab_row = T.row;
    A.tab_col = T.col;
    A.tab_row64 = T.row64;
    A.tab_col64 = T.col64;
    if (J.mode == MODE_DENSIFY && J.init_depth.data) {
        A.init_depth = J.init_depth.data;
        A.init_n0 = J.init_normal[0].data;
        A.init_n1 = J.init_normal[1].data;
        A.init_n2 = J.init_normal[2].data;
        A.init_pitch = J.init_depth.pitch_elems;
    }
}

void fill_io(pms::IoArgs &io, const JobSpec &J, int r, float4 *state, float *cost)
{
    io.W = J.W;
    io.H = J.H;
    io.r = r;
    io.state = state;
    io.cost = cost;
    io.depth = J.depth.data;
    io.n0 = J.normal[0].data;
    io.n1 = J.normal[1].data;
    io.n2 = J.normal[2].data;
    io.cplane = J.cost.data;
    io.pd = J.depth.pitch_elems;
    io.pn0 = J.normal[0].pitch_elems;
    io.pn1 = J.normal[1].pitch_elems;
    io.pn2 = J.normal[2].pitch_elems;
    io.pc = J.cost.pitch_elems;
    io.median_radius = J.p->median_radius;
    io.median_rel = J.p->median_rel;
}

void fill_geo(pms::GeoArgs &G, const JobSpec &J, int r, const Tables &T)
{
    const int W = J.W, H = J.H;
    G.W = W;
    G.H = H;
    G.r = r;
    G.n_maps = J.n_maps;
    G.min_views = J.p->geo_min_views > 0 ? J.p->geo_min_views : (J.n_maps < 2 ? J.n_maps : 2);
    G.geo_px = (float)J.p->geo_px;
    G.geo_rel = (float)J.p->geo_rel_depth;
    const double PI = 3.14159265358979323846;
    G.kx = (float)(W / (2.0 * PI));
    G.cx = (float)(W / 2.0 - 0.5);
    G.ky = (float)(-H / PI);
    G.cy = (float)(H / 2.0 - 0.5);
    G.tab_row = T.row;
    G.tab_col = T.col;
    for (int k = 0; k < J.n_maps; ++k) {
        G.pose[k] = relative_pose(*J.ref_pose, J.map_poses[k]);
        G.map[k] = J.maps[k].data;
        G.map_pitch[k] = J.maps[k].pitch_elems;
    }
    G.depth = J.depth.data;
    G.n0 = J.normal[0].data;
    G.n1 = J.normal[1].data;
    G.n2 = J.normal[2].data;
    G.cost = J.cost.data;
    G.pd = J.depth.pitch_elems;
    G.pn0 = J.normal[0].pitch_elems;
    G.pn1 = J.normal[1].pitch_elems;
    G.pn2 = J.normal[2].pitch_elems;
    G.pc = J.cost.pitch_elems;
}

// Builds the plan of `specs`. With base == nullptr only sizes and launches
// are final (used to size the device block); with the block's address every
// pointer in the tables is final too. `fixed` (all jobs of one size) names
// bearing tables the caller placed itself instead of the context's.
pms_status build_plan(pms_context *ctx, const std::vector<JobSpec> &specs, char *base, Plan &P,
                      const Tables *fixed = nullptr)
{
    P = Plan();
    const int n = (int)specs.size();
    std::vector<Geometry> geo(n);
    std::vector<Tables> tabs(n);
    for (int i = 0; i < n; ++i) {
        if (fixed) {
            tabs[i] = *fixed;
        } else {
            pms_status st = get_tables(ctx, specs[i].W, specs[i].H, &tabs[i]);
            if (st != PMS_OK) return st;
        }
        if (specs[i].mode != MODE_GEO) geo[i] = geometry(specs[i], ctx->sched);
        else geo[i].r = (specs[i].p->patch_size - 1) / 2;
    }
    // distinct neighbour images, each re-laid out once
    std::map<std::tuple<const void *, int, int, long long, int>, int> pad_index;
    std::vector<std::vector<int>> job_pads(n);
    for (int i = 0; i < n; ++i) {
        const JobSpec &J = specs[i];
        if (J.mode == MODE_GEO) continue;
        for (int j = 0; j < J.n_nbrs; ++j) {
            const pms_image &im = J.nbrs[j];
            auto key = std::make_tuple(im.data, (int)im.width, (int)im.height, (long long)im.pitch_bytes,
                                       (int)im.dtype);
            auto it = pad_index.find(key);
            int idx;
            if (it == pad_index.end()) {
                idx = (int)P.pads.size();
                pad_index[key] = idx;
                pms::PadJob pj;
                std::memset(&pj, 0, sizeof pj);
                pj.src.ptr = im.data;
                pj.src.pitch = im.pitch_bytes;
                pj.W = im.width;
                pj.H = im.height;
                pj.Wp = 2 * im.width + 4;
                pj.dtype = im.dtype;
                P.pads.push_back(pj);
            } else {
                idx = it->second;
            }
            job_pads[i].push_back(idx);
        }
    }

    // launches, in dependency order
    using Items = std::vector<std::tuple<int, int, int, int>>;
    const Variant none{0, 0, false};
    {
        Items items;
        for (size_t k = 0; k < P.pads.size(); ++k)
            items.emplace_back((int)k, (int)blocks_of(pad_cells(P.pads[k].W, P.pads[k].H)), 0, 0);
        add_rec(P, KK_IO, IO_PAD, 0, none, items);
    }
    {
        Items items;
        for (int i = 0; i < n; ++i)
            if (specs[i].mode != MODE_GEO)
                items.emplace_back(i, (int)blocks_of((long long)specs[i].W * specs[i].H), 0, 0);
        add_rec(P, KK_REFSTATS, 0, 0, none, items);
    }
    for (int i = 0; i < n; ++i)
        if (specs[i].mode == MODE_SWEEP) {
            Rec R{};
            R.kind = KK_IO;
            R.sub = IO_LOAD;
            R.job = i;
            R.total = 1;
            P.recs.push_back(R);
        }
    // tile launches, one per group of jobs sharing a kernel instance
    std::map<GroupKey, std::vector<int>> groups;
    for (int i = 0; i < n; ++i)
        if (specs[i].mode != MODE_GEO) groups[group_key(specs[i], geo[i])].push_back(i);
    auto group_variant = [&](const std::vector<int> &js) { return geo[js[0]].v; };
    for (auto &kv : groups) {
        Items init, eval;
        for (int i : kv.second) {
            const int tiles = geo[i].tiles_x_all * geo[i].tiles_y_all;
            if (specs[i].mode == MODE_DENSIFY) init.emplace_back(i, tiles, 0, 0);
            if (specs[i].mode == MODE_EVAL) eval.emplace_back(i, tiles, 0, 0);
        }
        add_rec(P, KK_INIT, 0, std::get<0>(kv.first), group_variant(kv.second), init);
        add_rec(P, KK_EVAL, 0, std::get<0>(kv.first), group_variant(kv.second), eval);
    }
    int max_steps = 0;
    for (int i = 0; i < n; ++i)
        if (specs[i].mode == MODE_DENSIFY) max_steps = std::max(max_steps, 2 * specs[i].p->iterations);
        else if (specs[i].mode == MODE_SWEEP) max_steps = std::max(max_steps, 1);
    for (int s = 0; s < max_steps; ++s)
        for (auto &kv : groups) {
            Items items;
            for (int i : kv.second) {
                const int tiles = geo[i].tiles_x_half * geo[i].tiles_y_half;
                if (specs[i].mode == MODE_DENSIFY && s < 2 * specs[i].p->iterations)
                    items.emplace_back(i, tiles, s / 2 + 1, s % 2);
                if (specs[i].mode == MODE_SWEEP && s == 0)
                    items.emplace_back(i, tiles, specs[i].iteration, specs[i].colour);
            }
            add_rec(P, KK_HALFSWEEP, 0, std::get<0>(kv.first), group_variant(kv.second), items);
        }
    {
        Items items;
        for (int i = 0; i < n; ++i)
            if (specs[i].mode == MODE_DENSIFY)
                items.emplace_back(i, (int)blocks_of((long long)specs[i].W * specs[i].H), 0, 0);
        add_rec(P, KK_FINALIZE, 0, 0, none, items);
    }
    {
        Items items;
        for (int i = 0; i < n; ++i)
            if (specs[i].mode == MODE_DENSIFY && specs[i].p->median_radius > 0)
                items.emplace_back(i, median_tiles(specs[i].W, specs[i].H), 0, 0);
        add_rec(P, KK_MEDIAN, 0, 0, none, items);
    }
    for (int i = 0; i < n; ++i)
        if (specs[i].mode == MODE_SWEEP) {
            Rec R{};
            R.kind = KK_IO;
            R.sub = IO_STORE;
            R.job = i;
            R.colour = specs[i].colour;
            R.total = 1;
            P.recs.push_back(R);
        }
    {
        Items items;
        for (int i = 0; i < n; ++i)
            if ((specs[i].mode == MODE_DENSIFY && specs[i].n_maps > 0) || specs[i].mode == MODE_GEO)
                items.emplace_back(i, (int)blocks_of((long long)specs[i].W * specs[i].H), 0, 0);
        add_rec(P, KK_CONSISTENCY, 0, 0, none, items);
    }

    // layout: argument tables, then per-job state, then re-laid-out images
    size_t off = align256((size_t)n * sizeof(pms::JobArgs));
    P.off_pads = off;
    off += align256(P.pads.size() * sizeof(pms::PadJob));
    P.off_entries = off;
    off += align256(P.entries.size() * sizeof(pms::Entry));
    P.args_bytes = off;
    P.jobs.resize(n);
    for (int i = 0; i < n; ++i) {
        const JobSpec &J = specs[i];
        pms::JobArgs &JA = P.jobs[i];
        std::memset(&JA, 0, sizeof JA);
        const long long npx = (long long)J.W * J.H;
        float4 *state = nullptr;
        float *cost = nullptr;
        if (J.mode == MODE_DENSIFY || J.mode == MODE_SWEEP) {
            state = reinterpret_cast<float4 *>(base + off);
            off += align256((size_t)npx * sizeof(float4));
            cost = reinterpret_cast<float *>(base + off);
            off += align256((size_t)npx * sizeof(float));
        }
        if (J.mode != MODE_GEO) {
            fill_sweep_args(JA.s, J, geo[i], tabs[i]);
            JA.s.stats = reinterpret_cast<const float2 *>(base + off);
            off += align256((size_t)npx * sizeof(float2));
            JA.s.state = state;
            JA.s.cost = cost;
        }
        if (J.mode == MODE_EVAL) {
            JA.s.in_depth = J.depth_in.data;
            JA.s.in_n0 = J.normal_in[0].data;
            JA.s.in_n1 = J.normal_in[1].data;
            JA.s.in_n2 = J.normal_in[2].data;
            JA.s.in_pitch = J.depth_in.pitch_elems;
            JA.s.out_cost = J.cost.data;
            JA.s.out_pitch = J.cost.pitch_elems;
            for (int j = 0; j < J.n_nbrs; ++j) JA.s.view_out[j] = J.per_view ? J.per_view[j].data : nullptr;
        }
        if (J.mode == MODE_DENSIFY || J.mode == MODE_SWEEP) fill_io(JA.io, J, geo[i].r, state, cost);
        if ((J.mode == MODE_DENSIFY && J.n_maps > 0) || J.mode == MODE_GEO) fill_geo(JA.g, J, geo[i].r, tabs[i]);
    }
    for (auto &pj : P.pads) {
        pj.dst = base + off;
        off += align256((size_t)pad_cells(pj.W, pj.H) * pad_elem_size(pj.dtype));
    }
    for (int i = 0; i < n; ++i)
        for (size_t j = 0; j < job_pads[i].size(); ++j) P.jobs[i].s.pad[j] = P.pads[job_pads[i][j]].dst;
    P.total_bytes = off;
    return PMS_OK;
}

// Writes the argument tables of a plan into `dst` (args_bytes).
void pack_args(const Plan &P, char *dst)
{
    std::memset(dst, 0, P.args_bytes);
    std::memcpy(dst, P.jobs.data(), P.jobs.size() * sizeof(pms::JobArgs));
    std::memcpy(dst + P.off_pads, P.pads.data(), P.pads.size() * sizeof(pms::PadJob));
    std::memcpy(dst + P.off_entries, P.entries.data(), P.entries.size() * sizeof(pms::Entry));
}

// Copies a plan's argument tables to `dev` on `s` through the staging ring.
pms_status upload_args(pms_context *ctx, const Plan &P, void *dev, hipStream_t s)
{
    Staging &sl = ctx->staging[ctx->staging_next];
    ctx->staging_next = (ctx->staging_next + 1) % kStagingSlots;
    hipError_t e;
    if (sl.done) {
        e = hipEventSynchronize(sl.done);
        if (e != hipSuccess) return hip_fail(ctx, e, "staging wait");
    } else {
        e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming);
        if (e != hipSuccess) return hip_fail(ctx, e, "hipEventCreate");
    }
    if (sl.cap < P.args_bytes) {
        if (sl.host) (void)hipHostFree(sl.host);
        sl.host = nullptr;
        sl.cap = 0;
        const size_t cap = std::max(P.args_bytes, (size_t)1 << 16);
        e = hipHostMalloc(&sl.host, cap, hipHostMallocDefault);
        if (e != hipSuccess) return fail(ctx, PMS_ERR_OUT_OF_MEMORY, "hipHostMalloc of staging failed");
        sl.cap = cap;
    }
    pack_args(P, static_cast<char *>(sl.host));
    e = hipMemcpyAsync(dev, sl.host, P.args_bytes, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(ctx, e, "argument upload");
    e = hipEventRecord(sl.done, s);
    if (e != hipSuccess) return hip_fail(ctx, e, "hipEventRecord");
    return PMS_OK;
}

// The half-sweep variant that also counts its executed work.
template <int DT>
void launch_counted_dt(const Variant &v, const pms::Launch &L, dim3 grid, hipStream_t s)
{
    using namespace pms;
    if (v.lpp == 2) hipLaunchKernelGGL((k_halfsweep_counted<DT, 2, 18, true>), grid, dim3(BLOCK), 0, s, L);
    else if (v.lpp == 8) hipLaunchKernelGGL((k_halfsweep_counted<DT, 8, 8, true>), grid, dim3(BLOCK), 0, s, L);
    else if (v.full && v.spl == 9) hipLaunchKernelGGL((k_halfsweep_counted<DT, 4, 9, true>), grid, dim3(BLOCK), 0, s, L);
    else if (v.full && v.spl == 16) hipLaunchKernelGGL((k_halfsweep_counted<DT, 4, 16, true>), grid, dim3(BLOCK), 0, s, L);
    else if (v.spl == 4) hipLaunchKernelGGL((k_halfsweep_counted<DT, 4, 4, false>), grid, dim3(BLOCK), 0, s, L);
    else if (v.spl == 9) hipLaunchKernelGGL((k_halfsweep_counted<DT, 4, 9, false>), grid, dim3(BLOCK), 0, s, L);
    else if (v.spl == 13) hipLaunchKernelGGL((k_halfsweep_counted<DT, 4, 13, false>), grid, dim3(BLOCK), 0, s, L);
    else hipLaunchKernelGGL((k_halfsweep_counted<DT, 4, 16, false>), grid, dim3(BLOCK), 0, s, L);
}

template <int KIND, int DT>
void launch_tiles_dt(const Variant &v, const pms::Launch &L, dim3 grid, hipStream_t s)
{
    using namespace pms;
    if (KIND == TK_HALFSWEEP && L.counts) launch_counted_dt<DT>(v, L, grid, s);
    else if (v.lpp == 2) hipLaunchKernelGGL((k_tiles<KIND, DT, 2, 18, true>), grid, dim3(BLOCK), 0, s, L);
    else if (v.lpp == 8) hipLaunchKernelGGL((k_tiles<KIND, DT, 8, 8, true>), grid, dim3(BLOCK), 0, s, L);
    else if (v.full && v.spl == 9) hipLaunchKernelGGL((k_tiles<KIND, DT, 4, 9, true>), grid, dim3(BLOCK), 0, s, L);
    else if (v.full && v.spl == 16) hipLaunchKernelGGL((k_tiles<KIND, DT, 4, 16, true>), grid, dim3(BLOCK), 0, s, L);
    else if (v.spl == 4) hipLaunchKernelGGL((k_tiles<KIND, DT, 4, 4, false>), grid, dim3(BLOCK), 0, s, L);
    else if (v.spl == 9) hipLaunchKernelGGL((k_tiles<KIND, DT, 4, 9, false>), grid, dim3(BLOCK), 0, s, L);
    else if (v.spl == 13) hipLaunchKernelGGL((k_tiles<KIND, DT, 4, 13, false>), grid, dim3(BLOCK), 0, s, L);
    else hipLaunchKernelGGL((k_tiles<KIND, DT, 4, 16, false>), grid, dim3(BLOCK), 0, s, L);
}

template <int KIND>
void launch_tiles(int dtype, const Variant &v, const pms::Launch &L, dim3 grid, hipStream_t s)
{
    if (dtype == PMS_F32) launch_tiles_dt<KIND, pms::DT_F32>(v, L, grid, s);
    else if (dtype == PMS_F16) launch_tiles_dt<KIND, pms::DT_F16>(v, L, grid, s);
    else launch_tiles_dt<KIND, pms::DT_U8>(v, L, grid, s);
}

// Enqueues every launch of a plan whose tables sit at `dev`; `timed` = false
// records no profiling events even when the context profiles.
pms_status enqueue_plan(pms_context *ctx, const Plan &P, char *dev, hipStream_t s, bool timed = true)
{
    for (const Rec &R : P.recs) {
        LaunchTimer timer(ctx, timed ? R.kind : -1, s);
        if (R.kind == KK_IO && R.sub != IO_PAD) {
            const pms::IoArgs &io = P.jobs[R.job].io;
            dim3 grid((unsigned)blocks_of((long long)io.W * io.H));
            if (R.sub == IO_LOAD) hipLaunchKernelGGL(pms::k_load_state, grid, dim3(pms::BLOCK), 0, s, io);
            else hipLaunchKernelGGL(pms::k_store_colour, grid, dim3(pms::BLOCK), 0, s, io, R.colour);
        } else {
            pms::Launch L;
            L.table = R.kind == KK_IO ? static_cast<const void *>(dev + P.off_pads) : static_cast<const void *>(dev);
            L.entries = reinterpret_cast<const pms::Entry *>(dev + P.off_entries) + R.entry_off;
            L.n_entries = R.n_entries;
            L.slots = R.total;
            L.counts = R.kind == KK_HALFSWEEP && ctx->work_counts_on ? ctx->work_counts : nullptr;
            dim3 grid(8u * (unsigned)L.slots);
            switch (R.kind) {
            case KK_IO: hipLaunchKernelGGL(pms::k_pad, grid, dim3(pms::BLOCK), 0, s, L); break;
            case KK_REFSTATS: hipLaunchKernelGGL(pms::k_refstats, grid, dim3(pms::BLOCK), 0, s, L); break;
            case KK_INIT: launch_tiles<pms::TK_INIT>(R.dtype, R.v, L, grid, s); break;
            case KK_HALFSWEEP: launch_tiles<pms::TK_HALFSWEEP>(R.dtype, R.v, L, grid, s); break;
            case KK_EVAL: launch_tiles<pms::TK_EVAL>(R.dtype, R.v, L, grid, s); break;
            case KK_FINALIZE: hipLaunchKernelGGL(pms::k_finalize, grid, dim3(pms::BLOCK), 0, s, L); break;
            case KK_MEDIAN: hipLaunchKernelGGL(pms::k_median, grid, dim3(pms::BLOCK), 0, s, L); break;
            case KK_CONSISTENCY: hipLaunchKernelGGL(pms::k_consistency, grid, dim3(pms::BLOCK), 0, s, L); break;
            default: break;
            }
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(ctx, e, kKernelNames[R.kind]);
    }
    return PMS_OK;
}

// Grows the context's device block to `need` bytes, stream-ordered on `s`:
// the old block is released after the last work that used it (the event
// recorded behind it, whatever stream that ran on), with no host wait.
pms_status ensure_work(pms_context *ctx, size_t need, hipStream_t s)
{
    if (need <= ctx->work_bytes) return PMS_OK;
    if (ctx->budget && need > ctx->budget)
        return fail(ctx, PMS_ERR_BUDGET, "device memory for this call exceeds the context budget");
    hipError_t e;
    if (ctx->work) {
        if (ctx->work_used) {
            e = hipStreamWaitEvent(s, ctx->work_used, 0);
            if (e != hipSuccess) return hip_fail(ctx, e, "hipStreamWaitEvent");
        }
        e = hipFreeAsync(ctx->work, s);
        if (e != hipSuccess) return hip_fail(ctx, e, "hipFreeAsync of the work block");
        ctx->work = nullptr;
        ctx->work_bytes = 0;
    }
    e = hipMallocAsync(&ctx->work, need, s);
    if (e != hipSuccess) {
        ctx->work = nullptr;
        return fail(ctx, PMS_ERR_OUT_OF_MEMORY, "hipMallocAsync of the work block failed");
    }
    ctx->work_bytes = need;
    return PMS_OK;
}

// Records, behind the work just enqueued on `s`, that the context's block
// is in use up to here (a later growth on any stream waits for it).
pms_status mark_work_used(pms_context *ctx, hipStream_t s)
{
    if (!ctx->work_used) {
        hipError_t e = hipEventCreateWithFlags(&ctx->work_used, hipEventDisableTiming);
        if (e != hipSuccess) return hip_fail(ctx, e, "hipEventCreate");
    }
    hipError_t e = hipEventRecord(ctx->work_used, s);
    return e == hipSuccess ? PMS_OK : hip_fail(ctx, e, "hipEventRecord");
}

// Runs validated jobs through the context's own block on `s`.
pms_status run_specs(pms_context *ctx, const std::vector<JobSpec> &specs, hipStream_t s)
{
    pms_status st = set_device(ctx);
    if (st != PMS_OK) return st;
    Plan P;
    if ((st = build_plan(ctx, specs, nullptr, P)) != PMS_OK) return st;
    if ((st = ensure_work(ctx, P.total_bytes, s)) != PMS_OK) return st;
    char *base = static_cast<char *>(ctx->work);
    if ((st = build_plan(ctx, specs, base, P)) != PMS_OK) return st;
    if ((st = upload_args(ctx, P, base, s)) != PMS_OK) return st;
    if ((st = enqueue_plan(ctx, P, base, s)) != PMS_OK) return st;
    return mark_work_used(ctx, s);
}

// ---------------------------------------------------------------------------
// Fixed scratch of pms_densify_noalloc: one array per GPU, compiled into the
// library. Host code must never pass `scratch` itself to a kernel or a copy
// (in host code it names a host-side stand-in); it uses the device address
// hipGetSymbolAddress returned for the current device, kept in
// g_scratch_ptr. Layout of one call: [bearing tables | plan block].
// ---------------------------------------------------------------------------

static __device__ __align__(256) unsigned char scratch[PMS_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};
hipError_t g_scratch_err[kMaxDevices] = {};
bool g_scratch_done[kMaxDevices] = {};

// Looks up this device's copy of the scratch array once per device, with
// the device current. Called at context creation.
void scratch_setup(int device)
{
    if (device < 0 || device >= kMaxDevices) return;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_done[device]) return;
    int prev = 0;
    hipError_t e = hipGetDevice(&prev);
    if (e == hipSuccess) e = hipSetDevice(device);
    void *ptr = nullptr;
    if (e == hipSuccess) e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e == hipSuccess && !ptr) e = hipErrorInvalidSymbol;
    (void)hipSetDevice(prev);
    g_scratch_ptr[device] = e == hipSuccess ? ptr : nullptr;
    g_scratch_err[device] = e;
    g_scratch_done[device] = true;
}

// Runs one validated job through the device's scratch array: no device or
// pinned-host allocation. The argument and bearing tables go up in one copy
// from the context's pageable host buffer (HIP stages a pageable source
// before the call returns, so the buffer may be rewritten by the next call).
pms_status run_noalloc(pms_context *ctx, const std::vector<JobSpec> &specs, hipStream_t s)
{
    pms_status st = set_device(ctx);
    if (st != PMS_OK) return st;
    const int dev = ctx->device;
    void *base = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        if (dev >= kMaxDevices || !g_scratch_done[dev])
            return fail(ctx, PMS_ERR_DEVICE, "scratch array of this device was not set up");
        if (!g_scratch_ptr[dev]) return hip_fail(ctx, g_scratch_err[dev], "hipGetSymbolAddress(scratch)");
        base = g_scratch_ptr[dev];
    }
    const int W = specs[0].W, H = specs[0].H;
    const size_t tab_bytes = align256(tables_bytes(W, H));
    Tables T = tables_at(base, W, H);
    Plan P;
    if ((st = build_plan(ctx, specs, nullptr, P, &T)) != PMS_OK) return st;
    if (tab_bytes + P.total_bytes > PMS_NOALLOC_SCRATCH_BYTES)
        return fail(ctx, PMS_ERR_BUDGET,
                    "this call needs " + std::to_string(tab_bytes + P.total_bytes) +
                        " bytes of scratch, more than PMS_NOALLOC_SCRATCH_BYTES (" +
                        std::to_string((size_t)PMS_NOALLOC_SCRATCH_BYTES) + ")");
    char *block = static_cast<char *>(base) + tab_bytes;
    if ((st = build_plan(ctx, specs, block, P, &T)) != PMS_OK) return st;
    const size_t upload = tab_bytes + P.args_bytes;
    if (ctx->noalloc_host.size() < upload) ctx->noalloc_host.resize(upload);
    char *host = ctx->noalloc_host.data();
    std::memset(host, 0, tab_bytes);
    fill_tables_host(W, H, host);
    pack_args(P, host + tab_bytes);
    hipError_t e = hipMemcpyAsync(base, host, upload, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(ctx, e, "argument upload");
    return enqueue_plan(ctx, P, block, s, false);
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

// Validates one densification job and fills its spec.
bool densify_spec(pms_context *ctx, const pms_image *ref, const pms_pose *ref_pose,
                  const pms_image *nbrs, const pms_pose *nbr_poses, int n_nbrs,
                  const pms_plane *maps, const pms_pose *map_poses, int n_maps,
                  const pms_params *params, pms_plane depth_out, const pms_plane normal_out[3],
                  pms_plane cost_out, JobSpec &J, pms_status *st)
{
    if (!check_ref_and_views(ctx, ref, ref_pose, nbrs, nbr_poses, n_nbrs, st)) return false;
    const int W = ref->width, H = ref->height;
    if (!check_params(ctx, params, W, H, n_nbrs, st)) return false;
    if (!check_outputs(ctx, W, depth_out, normal_out, cost_out, st)) return false;
    if (!check_maps(ctx, maps, map_poses, n_maps, W, st)) return false;
    J = JobSpec();
    J.mode = MODE_DENSIFY;
    J.W = W;
    J.H = H;
    J.ref = ref;
    J.ref_pose = ref_pose;
    J.nbrs = nbrs;
    J.nbr_poses = nbr_poses;
    J.n_nbrs = n_nbrs;
    J.maps = maps;
    J.map_poses = map_poses;
    J.n_maps = n_maps;
    J.p = params;
    J.depth = depth_out;
    for (int k = 0; k < 3; ++k) J.normal[k] = normal_out[k];
    J.cost = cost_out;
    return true;
}

bool job_spec(pms_context *ctx, const pms_job &jb, JobSpec &J, pms_status *st)
{
    if (!densify_spec(ctx, &jb.ref, &jb.ref_pose, jb.nbrs, jb.nbr_poses, jb.n_nbrs, jb.maps,
                      jb.map_poses, jb.n_maps, jb.params, jb.depth_out, jb.normal_out,
                      jb.cost_out, J, st))
        return false;
    if (jb.init_depth.data) {
        const int W = jb.ref.width;
        if (!check_outputs(ctx, W, jb.init_depth, jb.init_normal, jb.init_depth, st)) return false;
        const int64_t pitch = jb.init_depth.pitch_elems;
        for (int k = 0; k < 3; ++k)
            if (jb.init_normal[k].pitch_elems != pitch) {
                *st = fail(ctx, PMS_ERR_INVALID_ARG, "init_depth and init_normal must share one pitch");
                return false;
            }
        J.init_depth = jb.init_depth;
        for (int k = 0; k < 3; ++k) J.init_normal[k] = jb.init_normal[k];
    }
    return true;
}

// Output planes of one batch must not be read as another job's consistency
// map or written by two jobs.
bool check_batch_aliasing(pms_context *ctx, const std::vector<JobSpec> &specs, pms_status *st)
{
    std::vector<const float *> outs;
    for (auto &J : specs) {
        outs.push_back(J.depth.data);
        for (int k = 0; k < 3; ++k) outs.push_back(J.normal[k].data);
        outs.push_back(J.cost.data);
    }
    std::vector<const float *> sorted = outs;
    std::sort(sorted.begin(), sorted.end());
    if (std::adjacent_find(sorted.begin(), sorted.end()) != sorted.end()) {
        *st = fail(ctx, PMS_ERR_INVALID_ARG, "two output planes of a batch share one buffer");
        return false;
    }
    for (auto &J : specs) {
        for (int k = 0; k < J.n_maps; ++k)
            if (std::binary_search(sorted.begin(), sorted.end(), (const float *)J.maps[k].data)) {
                *st = fail(ctx, PMS_ERR_INVALID_ARG,
                           "a consistency map of a batch is an output plane of the same batch");
                return false;
            }
        const float *init[4] = {J.init_depth.data, J.init_normal[0].data, J.init_normal[1].data,
                                J.init_normal[2].data};
        if (init[0])
            for (auto p : init)
                if (std::binary_search(sorted.begin(), sorted.end(), p)) {
                    *st = fail(ctx, PMS_ERR_INVALID_ARG,
                               "an initial plane of a batch is an output plane of the same batch");
                    return false;
                }
    }
    return true;
}

bool batch_specs(pms_context *ctx, const pms_job *jobs, int n_jobs, std::vector<JobSpec> &specs,
                 pms_status *st)
{
    if (n_jobs < 1 || n_jobs > PMS_MAX_BATCH || !jobs) {
        *st = fail(ctx, PMS_ERR_INVALID_ARG, "need 1 <= n_jobs <= PMS_MAX_BATCH and a job array");
        return false;
    }
    specs.resize(n_jobs);
    for (int i = 0; i < n_jobs; ++i) {
        if (!job_spec(ctx, jobs[i], specs[i], st)) {
            ctx->last_error = "job " + std::to_string(i) + ": " + ctx->last_error;
            return false;
        }
    }
    return check_batch_aliasing(ctx, specs, st);
}

}  // namespace

// A batch plan with its own device block, uploaded once; running it only
// enqueues kernels (optionally as one graph launch).
struct pms_batch {
    pms_context *ctx = nullptr;
    Plan plan;
    void *block = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

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
    out->median_radius = 0;
    out->median_rel = 0.05;
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
    scratch_setup(device);
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
    if (ctx->work) {
        (void)hipFreeAsync(ctx->work, nullptr);
        (void)hipStreamSynchronize(nullptr);
    }
    if (ctx->work_used) (void)hipEventDestroy(ctx->work_used);
    if (ctx->work_counts) (void)hipFree(ctx->work_counts);
    for (auto &kv : ctx->tables) (void)hipFree(kv.second.row);
    for (auto &sl : ctx->staging) {
        if (sl.host) (void)hipHostFree(sl.host);
        if (sl.done) (void)hipEventDestroy(sl.done);
    }
    if (ctx->capture_stream) (void)hipStreamDestroy(ctx->capture_stream);
    for (auto &l : ctx->launches) {
        (void)hipEventDestroy(l.start);
        (void)hipEventDestroy(l.stop);
    }
    for (auto e : ctx->event_pool) (void)hipEventDestroy(e);
    delete ctx;
    return PMS_OK;
}

pms_status pms_get_schedule(const pms_context *ctx, pms_schedule *out)
{
    if (!ctx || !out) return PMS_ERR_INVALID_ARG;
    out->wave_rows = 1 << ctx->sched.wy_log2;
    out->waves_x = 1 << ctx->sched.bx_log2;
    out->lanes_per_pixel = ctx->sched.lpp == 0 ? 4 : ctx->sched.lpp;
    return PMS_OK;
}

pms_status pms_set_schedule(pms_context *ctx, const pms_schedule *s)
{
    if (!ctx || !s) return PMS_ERR_INVALID_ARG;
    ctx->last_error.clear();
    auto pow2 = [](int v) { return v > 0 && (v & (v - 1)) == 0; };
    if (!pow2(s->wave_rows) || s->wave_rows > 16)
        return fail(ctx, PMS_ERR_INVALID_ARG, "wave_rows must be 1, 2, 4, 8 or 16");
    if (!pow2(s->waves_x) || s->waves_x > 4)
        return fail(ctx, PMS_ERR_INVALID_ARG, "waves_x must be 1, 2 or 4");
    if (s->lanes_per_pixel != 2 && s->lanes_per_pixel != 4 && s->lanes_per_pixel != 8)
        return fail(ctx, PMS_ERR_INVALID_ARG, "lanes_per_pixel must be 2, 4 or 8");
    ctx->sched.wy_log2 = ilog2(s->wave_rows);
    ctx->sched.bx_log2 = ilog2(s->waves_x);
    ctx->sched.lpp = s->lanes_per_pixel == 4 ? 0 : s->lanes_per_pixel;
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
    std::vector<JobSpec> specs(1);
    if (!densify_spec(ctx, ref, ref_pose, nbrs, nbr_poses, n_nbrs, maps, map_poses, n_maps, params,
                      depth_out, normal_out, cost_out, specs[0], &st))
        return st;
    if (!check_batch_aliasing(ctx, specs, &st)) return st;
    return run_specs(ctx, specs, static_cast<hipStream_t>(stream));
}

pms_status pms_densify_noalloc(pms_context *ctx, const pms_image *ref, const pms_pose *ref_pose,
                               const pms_image *nbrs, const pms_pose *nbr_poses, int32_t n_nbrs,
                               const pms_plane *maps, const pms_pose *map_poses, int32_t n_maps,
                               const pms_params *params, pms_plane depth_out,
                               const pms_plane normal_out[3], pms_plane cost_out, void *stream)
{
    if (!ctx) return PMS_ERR_INVALID_ARG;
    ctx->last_error.clear();
    pms_status st = PMS_OK;
    std::vector<JobSpec> specs(1);
    if (!densify_spec(ctx, ref, ref_pose, nbrs, nbr_poses, n_nbrs, maps, map_poses, n_maps, params,
                      depth_out, normal_out, cost_out, specs[0], &st))
        return st;
    if (!check_batch_aliasing(ctx, specs, &st)) return st;
    return run_noalloc(ctx, specs, static_cast<hipStream_t>(stream));
}

pms_status pms_densify_batch(pms_context *ctx, const pms_job *jobs, int32_t n_jobs, void *stream)
{
    if (!ctx) return PMS_ERR_INVALID_ARG;
    ctx->last_error.clear();
    pms_status st = PMS_OK;
    std::vector<JobSpec> specs;
    if (!batch_specs(ctx, jobs, n_jobs, specs, &st)) return st;
    return run_specs(ctx, specs, static_cast<hipStream_t>(stream));
}

pms_status pms_batch_create(pms_context *ctx, const pms_job *jobs, int32_t n_jobs, pms_batch **out)
{
    if (!ctx || !out) return PMS_ERR_INVALID_ARG;
    *out = nullptr;
    ctx->last_error.clear();
    pms_status st = PMS_OK;
    std::vector<JobSpec> specs;
    if (!batch_specs(ctx, jobs, n_jobs, specs, &st)) return st;
    if ((st = set_device(ctx)) != PMS_OK) return st;
    pms_batch *b = new (std::nothrow) pms_batch();
    if (!b) return fail(ctx, PMS_ERR_OUT_OF_MEMORY, "batch allocation failed");
    b->ctx = ctx;
    if ((st = build_plan(ctx, specs, nullptr, b->plan)) != PMS_OK) {
        delete b;
        return st;
    }
    if (ctx->budget && b->plan.total_bytes > ctx->budget) {
        delete b;
        return fail(ctx, PMS_ERR_BUDGET, "device memory for this batch exceeds the context budget");
    }
    hipError_t e = hipMalloc(&b->block, b->plan.total_bytes);
    if (e != hipSuccess) {
        delete b;
        return fail(ctx, PMS_ERR_OUT_OF_MEMORY, "hipMalloc of the batch block failed");
    }
    char *base = static_cast<char *>(b->block);
    if ((st = build_plan(ctx, specs, base, b->plan)) != PMS_OK) {
        (void)hipFree(b->block);
        delete b;
        return st;
    }
    std::vector<char> args(b->plan.args_bytes);
    pack_args(b->plan, args.data());
    e = hipMemcpy(base, args.data(), args.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(b->block);
        delete b;
        return hip_fail(ctx, e, "batch argument upload");
    }
    *out = b;
    return PMS_OK;
}

pms_status pms_batch_run(pms_batch *b, int32_t use_graph, void *stream)
{
    if (!b) return PMS_ERR_INVALID_ARG;
    pms_context *ctx = b->ctx;
    ctx->last_error.clear();
    pms_status st = set_device(ctx);
    if (st != PMS_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    char *base = static_cast<char *>(b->block);
    if (!use_graph) return enqueue_plan(ctx, b->plan, base, s);
    hipError_t e;
    if (!b->exec) {
        if (!ctx->capture_stream) {
            e = hipStreamCreateWithFlags(&ctx->capture_stream, hipStreamNonBlocking);
            if (e != hipSuccess) return hip_fail(ctx, e, "hipStreamCreate");
        }
        e = hipStreamBeginCapture(ctx->capture_stream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return hip_fail(ctx, e, "hipStreamBeginCapture");
        ctx->capturing = true;
        st = enqueue_plan(ctx, b->plan, base, ctx->capture_stream);
        ctx->capturing = false;
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(ctx->capture_stream, &g);
        if (st != PMS_OK) {
            if (g) (void)hipGraphDestroy(g);
            return st;
        }
        if (e != hipSuccess) return hip_fail(ctx, e, "hipStreamEndCapture");
        e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            (void)hipGraphDestroy(g);
            b->exec = nullptr;
            return hip_fail(ctx, e, "hipGraphInstantiate");
        }
        b->graph = g;
    }
    LaunchTimer timer(ctx, KK_GRAPH, s);
    e = hipGraphLaunch(b->exec, s);
    if (e != hipSuccess) return hip_fail(ctx, e, "hipGraphLaunch");
    return PMS_OK;
}

pms_status pms_batch_bytes(const pms_batch *b, size_t *bytes)
{
    if (!b || !bytes) return PMS_ERR_INVALID_ARG;
    *bytes = b->plan.total_bytes;
    return PMS_OK;
}

pms_status pms_batch_destroy(pms_batch *b)
{
    if (!b) return PMS_ERR_INVALID_ARG;
    if (b->ctx->device >= 0) {
        (void)hipSetDevice(b->ctx->device);
        (void)hipDeviceSynchronize();
    }
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->block) (void)hipFree(b->block);
    delete b;
    return PMS_OK;
}

pms_status pms_autotune(pms_context *ctx, const pms_job *jobs, int32_t n_jobs, int32_t reps,
                        int32_t try_lanes, pms_schedule *best_out, double *best_ms_out,
                        void *stream)
{
    if (!ctx) return PMS_ERR_INVALID_ARG;
    ctx->last_error.clear();
    pms_status st = PMS_OK;
    if (reps < 1) return fail(ctx, PMS_ERR_INVALID_ARG, "reps must be >= 1");
    std::vector<JobSpec> specs;
    if (!batch_specs(ctx, jobs, n_jobs, specs, &st)) return st;
    if ((st = set_device(ctx)) != PMS_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const Schedule keep = ctx->sched;
    const bool keep_prof = ctx->profiling;
    // earlier timings stay with the caller
    std::vector<TimedLaunch> earlier;
    earlier.swap(ctx->launches);
    double best = 1e300;
    Schedule best_s = keep;
    // times one candidate schedule; whatever happens, every event it
    // recorded is waited for and returned to the pool
    auto measure = [&](const Schedule &c, double *ms_out) -> pms_status {
        ctx->sched = c;
        ctx->profiling = false;
        pms_status r = run_specs(ctx, specs, s);  // warm-up
        ctx->profiling = true;
        for (int k = 0; k < reps && r == PMS_OK; ++k) r = run_specs(ctx, specs, s);
        ctx->profiling = false;
        double ms = 0.0;
        for (auto &l : ctx->launches) {
            hipError_t e = hipEventSynchronize(l.stop);
            if (e != hipSuccess && r == PMS_OK) r = hip_fail(ctx, e, "hipEventSynchronize");
            float t = 0.0f;
            if (e == hipSuccess && hipEventElapsedTime(&t, l.start, l.stop) == hipSuccess &&
                (l.kind == KK_INIT || l.kind == KK_HALFSWEEP))
                ms += t;
            ctx->event_pool.push_back(l.start);
            ctx->event_pool.push_back(l.stop);
        }
        ctx->launches.clear();
        *ms_out = ms / reps;
        return r;
    };
    const int lanes[3] = {0, 2, 8};
    for (int li = 0; li < (try_lanes ? 3 : 1) && st == PMS_OK; ++li)
        for (int wy = 0; wy <= 4 && st == PMS_OK; ++wy)
            for (int bx = 0; bx <= 2 && st == PMS_OK; ++bx) {
                Schedule c;
                c.wy_log2 = wy;
                c.bx_log2 = bx;
                c.lpp = try_lanes ? lanes[li] : keep.lpp;
                double ms = 0.0;
                st = measure(c, &ms);
                if (st == PMS_OK && ms < best) {
                    best = ms;
                    best_s = c;
                }
            }
    ctx->launches.swap(earlier);
    ctx->profiling = keep_prof;
    if (st != PMS_OK) {
        ctx->sched = keep;
        return st;
    }
    ctx->sched = best_s;
    if (best_out) (void)pms_get_schedule(ctx, best_out);
    if (best_ms_out) *best_ms_out = best;
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
    std::vector<JobSpec> specs(1);
    JobSpec &J = specs[0];
    J.mode = MODE_EVAL;
    J.W = W;
    J.H = H;
    J.ref = ref;
    J.ref_pose = ref_pose;
    J.nbrs = nbrs;
    J.nbr_poses = nbr_poses;
    J.n_nbrs = n_nbrs;
    J.p = params;
    J.depth_in = depth_in;
    for (int k = 0; k < 3; ++k) J.normal_in[k] = normal_in[k];
    J.cost = cost_out;
    J.per_view = per_view_out;
    return run_specs(ctx, specs, static_cast<hipStream_t>(stream));
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
    std::vector<JobSpec> specs(1);
    JobSpec &J = specs[0];
    J.mode = MODE_SWEEP;
    J.W = W;
    J.H = H;
    J.ref = ref;
    J.ref_pose = ref_pose;
    J.nbrs = nbrs;
    J.nbr_poses = nbr_poses;
    J.n_nbrs = n_nbrs;
    J.p = params;
    J.depth = depth_io;
    for (int k = 0; k < 3; ++k) J.normal[k] = normal_io[k];
    J.cost = cost_io;
    J.iteration = iteration;
    J.colour = colour;
    return run_specs(ctx, specs, static_cast<hipStream_t>(stream));
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
    std::vector<JobSpec> specs(1);
    JobSpec &J = specs[0];
    J.mode = MODE_GEO;
    J.W = width;
    J.H = height;
    J.ref_pose = ref_pose;
    J.maps = maps;
    J.map_poses = map_poses;
    J.n_maps = n_maps;
    J.p = params;
    J.depth = depth_io;
    for (int k = 0; k < 3; ++k) J.normal[k] = normal_io[k];
    J.cost = cost_io;
    return run_specs(ctx, specs, static_cast<hipStream_t>(stream));
}

pms_status pms_warp_planes(pms_context *ctx, int32_t width, int32_t height,
                           const pms_pose *src_pose, pms_plane src_depth,
                           const pms_plane src_normal[3], const pms_pose *dst_pose,
                           const pms_params *params, pms_plane dst_depth,
                           const pms_plane dst_normal[3], void *stream)
{
    if (!ctx) return PMS_ERR_INVALID_ARG;
    ctx->last_error.clear();
    pms_status st = PMS_OK;
    if (height < 1 || width != 2 * height)
        return fail(ctx, PMS_ERR_INVALID_ARG, "size must be W x H with W == 2H >= 2");
    if (!src_pose || !dst_pose || !finite_pose(*src_pose) || !finite_pose(*dst_pose))
        return fail(ctx, PMS_ERR_INVALID_ARG, "null or non-finite pose");
    if (!check_params(ctx, params, width, height, 0, &st)) return st;
    if (!check_outputs(ctx, width, src_depth, src_normal, src_depth, &st)) return st;
    if (!check_outputs(ctx, width, dst_depth, dst_normal, dst_depth, &st)) return st;
    const float *srcs[4] = {src_depth.data, src_normal[0].data, src_normal[1].data, src_normal[2].data};
    const float *dsts[4] = {dst_depth.data, dst_normal[0].data, dst_normal[1].data, dst_normal[2].data};
    for (auto a : srcs)
        for (auto b : dsts)
            if (a == b) return fail(ctx, PMS_ERR_INVALID_ARG, "source and destination planes overlap");
    if ((st = set_device(ctx)) != PMS_OK) return st;
    Tables T;
    if ((st = get_tables(ctx, width, height, &T)) != PMS_OK) return st;
    const long long npx = (long long)width * height;
    if ((st = ensure_work(ctx, (size_t)npx * sizeof(unsigned long long), static_cast<hipStream_t>(stream))) != PMS_OK)
        return st;
    pms::WarpArgs A;
    std::memset(&A, 0, sizeof A);
    A.W = width;
    A.H = height;
    A.r = (params->patch_size - 1) / 2;
    const pms::ViewPoseD rel = relative_pose64(*src_pose, *dst_pose);
    for (int k = 0; k < 9; ++k) A.R[k] = rel.R[k];
    for (int k = 0; k < 3; ++k) A.t[k] = rel.t[k];
    A.dmin = params->depth_min;
    A.dmax = params->depth_max;
    A.sd = src_depth.data;
    A.sn0 = src_normal[0].data;
    A.sn1 = src_normal[1].data;
    A.sn2 = src_normal[2].data;
    A.psd = src_depth.pitch_elems;
    A.psn0 = src_normal[0].pitch_elems;
    A.psn1 = src_normal[1].pitch_elems;
    A.psn2 = src_normal[2].pitch_elems;
    A.dd = dst_depth.data;
    A.dn0 = dst_normal[0].data;
    A.dn1 = dst_normal[1].data;
    A.dn2 = dst_normal[2].data;
    A.pdd = dst_depth.pitch_elems;
    A.pdn0 = dst_normal[0].pitch_elems;
    A.pdn1 = dst_normal[1].pitch_elems;
    A.pdn2 = dst_normal[2].pitch_elems;
    A.zbuf = static_cast<unsigned long long *>(ctx->work);
    A.tab_row64 = T.row64;
    A.tab_col64 = T.col64;
    hipStream_t s = static_cast<hipStream_t>(stream);
    dim3 grid((unsigned)blocks_of(npx));
    {
        LaunchTimer timer(ctx, KK_WARP, s);
        hipLaunchKernelGGL(pms::k_warp_clear, grid, dim3(pms::BLOCK), 0, s, A);
        hipLaunchKernelGGL(pms::k_warp_splat, grid, dim3(pms::BLOCK), 0, s, A);
        hipLaunchKernelGGL(pms::k_warp_resolve, grid, dim3(pms::BLOCK), 0, s, A);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(ctx, e, "warp");
    return mark_work_used(ctx, s);
}

pms_status pms_view_filter(pms_context *ctx, const double centre_a[3], const double centre_b[3],
                           const double *points, int64_t n_points, double min_deg,
                           double max_deg, uint64_t *counts_out, void *stream)
{
    if (!ctx) return PMS_ERR_INVALID_ARG;
    ctx->last_error.clear();
    if (!centre_a || !centre_b || !counts_out || n_points < 0 || (n_points > 0 && !points))
        return fail(ctx, PMS_ERR_INVALID_ARG, "null centre, points or counts, or n_points < 0");
    for (int k = 0; k < 3; ++k)
        if (!std::isfinite(centre_a[k]) || !std::isfinite(centre_b[k]))
            return fail(ctx, PMS_ERR_INVALID_ARG, "non-finite camera centre");
    if (!(min_deg <= max_deg) || !std::isfinite(min_deg) || !std::isfinite(max_deg))
        return fail(ctx, PMS_ERR_INVALID_ARG, "need finite min_deg <= max_deg");
    pms_status st = set_device(ctx);
    if (st != PMS_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    unsigned long long *counts = reinterpret_cast<unsigned long long *>(counts_out);
    // the spread counters in the context's block
    if ((st = ensure_work(ctx, pms::COUNT_SPREAD_BYTES, s)) != PMS_OK) return st;
    unsigned long long *spread = static_cast<unsigned long long *>(ctx->work);
    {
        LaunchTimer timer(ctx, KK_VIEW, s);
        hipLaunchKernelGGL(pms::k_count_clear, dim3(1), dim3(2 * pms::COUNT_SPREAD), 0, s, spread);
        // cosines of the bounds; 2 / -2 where a bound admits / rejects every
        // angle in [0, 180]
        const double deg2rad = 3.14159265358979323846 / 180.0;
        const double cmin = min_deg < 0.0 ? 2.0 : (min_deg > 180.0 ? -2.0 : std::cos(min_deg * deg2rad));
        const double cmax = max_deg > 180.0 ? -2.0 : (max_deg < 0.0 ? 2.0 : std::cos(max_deg * deg2rad));
        if (n_points > 0)
            hipLaunchKernelGGL(pms::k_view_filter, dim3(count_grid(n_points)), dim3(pms::BLOCK), 0,
                               s, centre_a[0], centre_a[1], centre_a[2], centre_b[0], centre_b[1],
                               centre_b[2], points, (long long)n_points, min_deg, max_deg, cmin, cmax,
                               spread);
        hipLaunchKernelGGL(pms::k_count_gather, dim3(1), dim3(pms::COUNT_SPREAD), 0, s, spread, counts,
                           counts + 1);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(ctx, e, "view filter");
    return mark_work_used(ctx, s);
}

}  // extern "C"

namespace {

// Validates the maps of pms_fuse / pms_coverage and fills their part of
// the arguments.
pms_status fuse_args(pms_context *ctx, int W, int H, int n_maps, const pms_plane *depths,
                     const pms_pose *poses, pms::FuseArgs &A)
{
    if (H < 1 || W != 2 * H) return fail(ctx, PMS_ERR_INVALID_ARG, "size must be W x H with W == 2H >= 2");
    if (n_maps < 1 || n_maps > PMS_MAX_MAPS || !depths || !poses)
        return fail(ctx, PMS_ERR_INVALID_ARG, "need 1 <= n_maps <= 8 maps and poses");
    pms_status st = PMS_OK;
    for (int m = 0; m < n_maps; ++m) {
        if (!check_plane(ctx, depths[m], W, "depth map", &st)) return st;
        if (!finite_pose(poses[m])) return fail(ctx, PMS_ERR_INVALID_ARG, "non-finite map pose");
    }
    if ((st = set_device(ctx)) != PMS_OK) return st;
    Tables T;
    if ((st = get_tables(ctx, W, H, &T)) != PMS_OK) return st;
    std::memset(&A, 0, sizeof A);
    A.W = W;
    A.H = H;
    A.n_maps = n_maps;
    for (int m = 0; m < n_maps; ++m) {
        A.depth[m] = depths[m].data;
        A.pitch[m] = depths[m].pitch_elems;
        for (int k = 0; k < 9; ++k) A.pose[m].R[k] = poses[m].R[k];
        for (int k = 0; k < 3; ++k) A.pose[m].t[k] = poses[m].t[k];
    }
    A.tab_row64 = T.row64;
    A.tab_col64 = T.col64;
    return PMS_OK;
}

}  // namespace

extern "C" {

pms_status pms_fuse(pms_context *ctx, int32_t width, int32_t height, int32_t n_maps,
                    const pms_plane *depths, const pms_pose *poses, double voxel,
                    uint8_t *keep_out, uint64_t *n_kept_out, void *stream)
{
    if (!ctx) return PMS_ERR_INVALID_ARG;
    ctx->last_error.clear();
    if (!keep_out || !n_kept_out) return fail(ctx, PMS_ERR_INVALID_ARG, "null keep or count output");
    if (!(voxel > 0.0) || !std::isfinite(voxel)) return fail(ctx, PMS_ERR_INVALID_ARG, "voxel must be > 0");
    pms::FuseArgs A;
    pms_status st = fuse_args(ctx, width, height, n_maps, depths, poses, A);
    if (st != PMS_OK) return st;
    const long long points = (long long)width * height * n_maps;
    unsigned long long cap = 1024;
    // load at most 0.8 if every point had a voxel of its own; a window's
    // maps share most voxels, so the usual load is far lower
    while (cap < (unsigned long long)points + (unsigned long long)points / 4) cap <<= 1;
    // (32-bit slot indices, all below the NO_CLAIM marker)
    if (cap > (1ULL << 31)) return fail(ctx, PMS_ERR_INVALID_ARG, "too many points for one fusion call");
    // the table, one claimed-slot index per point, then the spread counters
    const size_t table_bytes = (size_t)cap * 2 * sizeof(unsigned long long);
    const size_t spread_off = (table_bytes + (size_t)points * sizeof(unsigned) + 255) & ~(size_t)255;
    if ((st = ensure_work(ctx, spread_off + pms::COUNT_SPREAD_BYTES, static_cast<hipStream_t>(stream))) != PMS_OK)
        return st;
    A.voxel = voxel;
    {
        // camera centre of the first map, -R^T t, in voxel coordinates
        const pms_pose &P = poses[0];
        for (int k = 0; k < 3; ++k) {
            const double c = -(P.R[k] * P.t[0] + P.R[3 + k] * P.t[1] + P.R[6 + k] * P.t[2]);
            A.origin[k] = std::floor(c / voxel);
        }
        if (!(std::fabs(A.origin[0]) < 4.0e15 && std::fabs(A.origin[1]) < 4.0e15 && std::fabs(A.origin[2]) < 4.0e15))
            return fail(ctx, PMS_ERR_INVALID_ARG, "first camera too far from the world origin for this voxel size");
    }
    A.slots = static_cast<unsigned long long *>(ctx->work);
    A.mask = cap - 1;
    A.claim = reinterpret_cast<unsigned *>(static_cast<char *>(ctx->work) + table_bytes);
    A.spread = reinterpret_cast<unsigned long long *>(static_cast<char *>(ctx->work) + spread_off);
    A.keep = keep_out;
    A.count = reinterpret_cast<unsigned long long *>(n_kept_out);
    hipStream_t s = static_cast<hipStream_t>(stream);
    {
        LaunchTimer timer(ctx, KK_FUSE, s);
        hipLaunchKernelGGL(pms::k_fuse_clear, dim3((unsigned)blocks_of((long long)cap)), dim3(pms::BLOCK), 0, s, A);
        // one launch per map, in map order; one wave per FUSE_TILE x
        // FUSE_TILE tile
        const long long tiles = (long long)((width + pms::FUSE_TILE - 1) / pms::FUSE_TILE) *
                                ((height + pms::FUSE_TILE - 1) / pms::FUSE_TILE);
        for (int m = 0; m < n_maps; ++m)
            hipLaunchKernelGGL(pms::k_fuse_insert,
                               dim3((unsigned)((tiles + pms::BLOCK / 64 - 1) / (pms::BLOCK / 64))), dim3(pms::BLOCK),
                               0, s, A, m);
        hipLaunchKernelGGL(pms::k_fuse_mark, dim3(count_grid(points)), dim3(pms::BLOCK), 0, s, A);
        hipLaunchKernelGGL(pms::k_count_gather, dim3(1), dim3(pms::COUNT_SPREAD), 0, s, A.spread, A.count,
                           (unsigned long long *)nullptr);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(ctx, e, "fuse");
    return mark_work_used(ctx, s);
}

pms_status pms_coverage(pms_context *ctx, int32_t width, int32_t height, int32_t n_maps,
                        const pms_plane *depths, const pms_pose *poses, const uint8_t *keep,
                        const pms_pose *view_pose, int32_t out_width, int32_t out_height,
                        uint8_t *cover_out, uint64_t *n_covered_out, void *stream)
{
    if (!ctx) return PMS_ERR_INVALID_ARG;
    ctx->last_error.clear();
    if (!cover_out || !n_covered_out || !view_pose || !finite_pose(*view_pose))
        return fail(ctx, PMS_ERR_INVALID_ARG, "null output or bad view pose");
    if (out_height < 1 || out_width != 2 * out_height)
        return fail(ctx, PMS_ERR_INVALID_ARG, "panorama must be W x H with W == 2H");
    pms::FuseArgs A;
    pms_status st = fuse_args(ctx, width, height, n_maps, depths, poses, A);
    if (st != PMS_OK) return st;
    for (int k = 0; k < 9; ++k) A.view.R[k] = view_pose->R[k];
    for (int k = 0; k < 3; ++k) A.view.t[k] = view_pose->t[k];
    A.Wc = out_width;
    A.Hc = out_height;
    A.cover = cover_out;
    A.keep_in = keep;
    A.count = reinterpret_cast<unsigned long long *>(n_covered_out);
    const long long points = (long long)width * height * n_maps;
    const long long pix = (long long)out_width * out_height;
    hipStream_t s = static_cast<hipStream_t>(stream);
    // the spread counters in the context's block
    if ((st = ensure_work(ctx, pms::COUNT_SPREAD_BYTES, s)) != PMS_OK) return st;
    A.spread = static_cast<unsigned long long *>(ctx->work);
    {
        LaunchTimer timer(ctx, KK_COVER, s);
        hipLaunchKernelGGL(pms::k_cover_clear, dim3((unsigned)blocks_of(pix)), dim3(pms::BLOCK), 0, s, A);
        // one wave per COVER_SPAN points
        const long long waves = (points + pms::COVER_SPAN - 1) / pms::COVER_SPAN;
        hipLaunchKernelGGL(pms::k_cover_mark, dim3((unsigned)((waves + pms::BLOCK / 64 - 1) / (pms::BLOCK / 64))),
                           dim3(pms::BLOCK), 0, s, A);
        hipLaunchKernelGGL(pms::k_cover_count, dim3(count_grid(pix)), dim3(pms::BLOCK), 0, s, A);
        hipLaunchKernelGGL(pms::k_count_gather, dim3(1), dim3(pms::COUNT_SPREAD), 0, s, A.spread, A.count,
                           (unsigned long long *)nullptr);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(ctx, e, "coverage");
    return mark_work_used(ctx, s);
}

pms_status pms_philox_stream(pms_context *ctx, uint64_t key0, uint64_t key1, uint64_t ctr0,
                             int64_t n, uint64_t *out, void *stream)
{
    if (!ctx) return PMS_ERR_INVALID_ARG;
    ctx->last_error.clear();
    if (n < 0 || (n > 0 && !out)) return fail(ctx, PMS_ERR_INVALID_ARG, "bad n or null out");
    if (n == 0) return PMS_OK;
    if (n > (int64_t)1 << 31) return fail(ctx, PMS_ERR_INVALID_ARG, "n too large");
    pms_status st = set_device(ctx);
    if (st != PMS_OK) return st;
    hipLaunchKernelGGL(pms::k_philox, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                       static_cast<hipStream_t>(stream), (unsigned long long)key0,
                       (unsigned long long)key1, (unsigned long long)ctr0, (long long)n,
                       reinterpret_cast<unsigned long long *>(out));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(ctx, e, "philox");
    return PMS_OK;
}

pms_status pms_profile_enable(pms_context *ctx, int32_t on)
{
    if (!ctx) return PMS_ERR_INVALID_ARG;
    ctx->profiling = on != 0;
    return PMS_OK;
}

pms_status pms_work_count_enable(pms_context *ctx, int32_t on)
{
    if (!ctx) return PMS_ERR_INVALID_ARG;
    ctx->last_error.clear();
    if (on && !ctx->work_counts) {
        pms_status st = set_device(ctx);
        if (st != PMS_OK) return st;
        void *p = nullptr;
        if (hipMalloc(&p, PMS_WORK_FIELDS * sizeof(unsigned long long)) != hipSuccess)
            return fail(ctx, PMS_ERR_OUT_OF_MEMORY, "hipMalloc of the work counters failed");
        hipError_t e = hipMemset(p, 0, PMS_WORK_FIELDS * sizeof(unsigned long long));
        if (e != hipSuccess) {
            (void)hipFree(p);
            return hip_fail(ctx, e, "hipMemset of the work counters");
        }
        ctx->work_counts = static_cast<unsigned long long *>(p);
    }
    ctx->work_counts_on = on != 0;
    return PMS_OK;
}

pms_status pms_work_count_read(pms_context *ctx, pms_work_counts *out, int32_t reset)
{
    if (!ctx || !out) return PMS_ERR_INVALID_ARG;
    ctx->last_error.clear();
    std::memset(out, 0, sizeof *out);
    if (!ctx->work_counts) return PMS_OK;
    pms_status st = set_device(ctx);
    if (st != PMS_OK) return st;
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(ctx, e, "hipDeviceSynchronize");
    unsigned long long v[PMS_WORK_FIELDS];
    e = hipMemcpy(v, ctx->work_counts, sizeof v, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(ctx, e, "work counter read");
    static_assert(PMS_WORK_FIELDS == pms::WC_FIELDS, "counter fields");
    int64_t *dst = &out->pixels;
    for (int f = 0; f < PMS_WORK_FIELDS; ++f) dst[f] = (int64_t)v[f];
    if (reset) {
        e = hipMemset(ctx->work_counts, 0, sizeof v);
        if (e != hipSuccess) return hip_fail(ctx, e, "hipMemset of the work counters");
    }
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

// ---------------------------------------------------------------------------
// serving loop: continuous batching of keyframe jobs
// ---------------------------------------------------------------------------

namespace {

// First-fit allocator over one device arena (offsets, 256-byte granules).
class Arena {
  public:
    void reset(size_t bytes)
    {
        free_.clear();
        size_ = bytes & ~(size_t)255;
        if (size_) free_[0] = size_;
        used_ = 0;
    }
    bool alloc(size_t bytes, size_t *off)
    {
        bytes = align256(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it)
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes;
                const size_t at = it->first + bytes;
                free_.erase(it);
                if (rest) free_[at] = rest;
                used_ += bytes;
                return true;
            }
        return false;
    }
    void release(size_t off, size_t bytes)
    {
        bytes = align256(bytes);
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t size() const { return size_; }
    size_t used() const { return used_; }

  private:
    std::map<size_t, size_t> free_;
    size_t size_ = 0, used_ = 0;
};

using ImageKey = std::tuple<const void *, int, int, long long, int>;

struct CachedPad {
    size_t off = 0, bytes = 0;
    int refs = 0;
    bool laid_out = false;  // its re-layout is already enqueued
    pms::PadJob job;
};

enum ServerJobState { SJ_WAITING = 0, SJ_RUNNING = 1, SJ_DONE = 2 };

// A submitted job with its own copies of everything the caller passed by
// host pointer.
struct ServerJob {
    int64_t ticket = 0;
    pms_job job{};
    std::vector<pms_image> nbrs;
    std::vector<pms_pose> nbr_poses, map_poses;
    std::vector<pms_plane> maps;
    pms_params params{};
    JobSpec spec;
    Geometry geo{};
    size_t bytes = 0;      // plane state, cost and patch statistics
    size_t pad_need = 0;   // re-laid-out images not yet cached at submission
    size_t off = 0;
    int slot = -1;
    int steps_done = 0;    // half-sweeps enqueued
    bool fresh = false;    // admitted in the tick being built
    std::vector<ImageKey> pads;
    int state = SJ_WAITING;
    hipEvent_t done = nullptr;  // recorded after the job's last launch
};

}  // namespace

struct pms_server {
    pms_context *ctx = nullptr;
    void *block = nullptr;        // argument region, then the arena
    size_t args_bytes = 0;
    size_t off_pads = 0, off_entries = 0;
    int max_jobs = 0, max_pads = 0, max_entries = 0;
    Arena arena;
    char *arena_base = nullptr;
    std::map<ImageKey, CachedPad> pads;
    std::vector<pms::JobArgs> table;  // host mirror of the device job table
    std::vector<int> slot_free;
    std::vector<ServerJob *> waiting;  // FIFO
    std::vector<ServerJob *> running;
    std::map<int64_t, ServerJob *> jobs;  // every job not yet collected
    int64_t next_ticket = 1;
    std::vector<hipEvent_t> tick_events;  // ring: limits ticks in flight
    int tick_next = 0;
    std::vector<hipEvent_t> spare_events;
    // statistics
    int64_t ticks = 0, job_ticks = 0;
    size_t peak_bytes = 0;
};

namespace {

constexpr int kTicksInFlight = 2;

// Arena bytes of a job's own buffers.
size_t job_state_bytes(const JobSpec &J)
{
    const size_t npx = (size_t)J.W * J.H;
    return align256(npx * sizeof(float4)) + align256(npx * sizeof(float)) + align256(npx * sizeof(float2));
}

ImageKey image_key(const pms_image &im)
{
    return ImageKey(im.data, (int)im.width, (int)im.height, (long long)im.pitch_bytes, (int)im.dtype);
}

size_t pad_bytes_of(const pms_image &im)
{
    return align256((size_t)pad_cells(im.width, im.height) * pad_elem_size(im.dtype));
}

void server_release(pms_server *S, ServerJob *J)
{
    S->arena.release(J->off, J->bytes);
    for (auto &k : J->pads) {
        auto it = S->pads.find(k);
        if (it != S->pads.end() && --it->second.refs == 0) {
            S->arena.release(it->second.off, it->second.bytes);
            S->pads.erase(it);
        }
    }
    J->pads.clear();
    S->slot_free.push_back(J->slot);
    J->slot = -1;
}

// Tries to give the waiting job its memory and a table slot.
bool server_admit(pms_server *S, ServerJob *J)
{
    if (S->slot_free.empty()) return false;
    size_t off = 0;
    if (!S->arena.alloc(J->bytes, &off)) return false;
    std::vector<ImageKey> fresh_keys;
    std::vector<ImageKey> keys;
    for (int j = 0; j < J->job.n_nbrs; ++j) {
        ImageKey k = image_key(J->nbrs[j]);
        if (std::find(keys.begin(), keys.end(), k) != keys.end()) continue;
        keys.push_back(k);
        if (S->pads.count(k)) continue;
        size_t poff = 0;
        const size_t pb = pad_bytes_of(J->nbrs[j]);
        if (!S->arena.alloc(pb, &poff)) {
            // roll back
            for (auto &fk : fresh_keys) {
                S->arena.release(S->pads[fk].off, S->pads[fk].bytes);
                S->pads.erase(fk);
            }
            S->arena.release(off, J->bytes);
            return false;
        }
        CachedPad cp;
        cp.off = poff;
        cp.bytes = pb;
        std::memset(&cp.job, 0, sizeof cp.job);
        const pms_image &im = J->nbrs[j];
        cp.job.src.ptr = im.data;
        cp.job.src.pitch = im.pitch_bytes;
        cp.job.W = im.width;
        cp.job.H = im.height;
        cp.job.Wp = 2 * im.width + 4;
        cp.job.dtype = im.dtype;
        cp.job.dst = S->arena_base + poff;
        S->pads[k] = cp;
        fresh_keys.push_back(k);
    }
    for (auto &k : keys) S->pads[k].refs += 1;
    J->pads = keys;
    J->off = off;
    J->slot = S->slot_free.back();
    S->slot_free.pop_back();
    S->peak_bytes = std::max(S->peak_bytes, S->arena.used());
    return true;
}

// Fills the job's table slot (host mirror).
pms_status server_fill_slot(pms_server *S, ServerJob *J)
{
    Tables T;
    pms_status st = get_tables(S->ctx, J->spec.W, J->spec.H, &T);
    if (st != PMS_OK) return st;
    pms::JobArgs &JA = S->table[J->slot];
    std::memset(&JA, 0, sizeof JA);
    char *base = S->arena_base + J->off;
    const size_t npx = (size_t)J->spec.W * J->spec.H;
    float4 *state = reinterpret_cast<float4 *>(base);
    float *cost = reinterpret_cast<float *>(base + align256(npx * sizeof(float4)));
    const float2 *stats = reinterpret_cast<const float2 *>(base + align256(npx * sizeof(float4)) +
                                                            align256(npx * sizeof(float)));
    fill_sweep_args(JA.s, J->spec, J->geo, T);
    JA.s.state = state;
    JA.s.cost = cost;
    JA.s.stats = stats;
    for (int j = 0; j < J->job.n_nbrs; ++j) JA.s.pad[j] = S->pads[image_key(J->nbrs[j])].job.dst;
    fill_io(JA.io, J->spec, J->geo.r, state, cost);
    if (J->job.n_maps > 0) fill_geo(JA.g, J->spec, J->geo.r, T);
    return PMS_OK;
}

}  // namespace

extern "C" {

pms_status pms_server_create(pms_context *ctx, size_t arena_bytes, int32_t max_jobs, pms_server **out)
{
    if (!ctx || !out) return PMS_ERR_INVALID_ARG;
    *out = nullptr;
    ctx->last_error.clear();
    if (max_jobs < 1 || max_jobs > PMS_MAX_BATCH)
        return fail(ctx, PMS_ERR_INVALID_ARG, "max_jobs must be in [1, PMS_MAX_BATCH]");
    if (arena_bytes < ((size_t)1 << 20)) return fail(ctx, PMS_ERR_INVALID_ARG, "arena below 1 MiB");
    pms_status st = set_device(ctx);
    if (st != PMS_OK) return st;
    pms_server *S = new (std::nothrow) pms_server();
    if (!S) return fail(ctx, PMS_ERR_OUT_OF_MEMORY, "server allocation failed");
    S->ctx = ctx;
    S->max_jobs = max_jobs;
    S->max_pads = max_jobs * PMS_MAX_VIEWS;
    // per tick: pads, refstats, init and half-sweep per group, finalize,
    // consistency; each list with its sentinel
    S->max_entries = S->max_pads + 8 * (max_jobs + 1) * 4;
    S->off_pads = align256((size_t)max_jobs * sizeof(pms::JobArgs));
    S->off_entries = S->off_pads + align256((size_t)S->max_pads * sizeof(pms::PadJob));
    S->args_bytes = S->off_entries + align256((size_t)S->max_entries * sizeof(pms::Entry));
    const size_t total = S->args_bytes + arena_bytes;
    if (ctx->budget && total > ctx->budget) {
        delete S;
        return fail(ctx, PMS_ERR_BUDGET, "server arena exceeds the context budget");
    }
    hipError_t e = hipMalloc(&S->block, total);
    if (e != hipSuccess) {
        delete S;
        return fail(ctx, PMS_ERR_OUT_OF_MEMORY, "hipMalloc of the server arena failed");
    }
    S->arena_base = static_cast<char *>(S->block) + S->args_bytes;
    S->arena.reset(arena_bytes);
    S->table.resize(max_jobs);
    std::memset(S->table.data(), 0, S->table.size() * sizeof(pms::JobArgs));
    for (int i = max_jobs - 1; i >= 0; --i) S->slot_free.push_back(i);
    S->tick_events.assign(kTicksInFlight, nullptr);
    *out = S;
    return PMS_OK;
}

pms_status pms_server_submit(pms_server *S, const pms_job *job, int64_t *ticket)
{
    if (!S || !job || !ticket) return PMS_ERR_INVALID_ARG;
    pms_context *ctx = S->ctx;
    ctx->last_error.clear();
    pms_status st = PMS_OK;
    JobSpec probe;
    if (!job_spec(ctx, *job, probe, &st)) return st;
    std::vector<JobSpec> one{probe};
    if (!check_batch_aliasing(ctx, one, &st)) return st;
    ServerJob *J = new (std::nothrow) ServerJob();
    if (!J) return fail(ctx, PMS_ERR_OUT_OF_MEMORY, "job allocation failed");
    J->job = *job;
    J->nbrs.assign(job->nbrs, job->nbrs + job->n_nbrs);
    J->nbr_poses.assign(job->nbr_poses, job->nbr_poses + job->n_nbrs);
    if (job->n_maps > 0) {
        J->maps.assign(job->maps, job->maps + job->n_maps);
        J->map_poses.assign(job->map_poses, job->map_poses + job->n_maps);
    }
    J->params = *job->params;
    J->job.nbrs = J->nbrs.data();
    J->job.nbr_poses = J->nbr_poses.data();
    J->job.maps = J->maps.empty() ? nullptr : J->maps.data();
    J->job.map_poses = J->map_poses.empty() ? nullptr : J->map_poses.data();
    J->job.params = &J->params;
    job_spec(ctx, J->job, J->spec, &st);
    J->geo = geometry(J->spec, ctx->sched);
    J->bytes = job_state_bytes(J->spec);
    size_t need = J->bytes;
    for (int j = 0; j < J->job.n_nbrs; ++j) need += pad_bytes_of(J->nbrs[j]);
    if (need > S->arena.size()) {
        delete J;
        return fail(ctx, PMS_ERR_BUDGET, "this job alone needs more than the server arena");
    }
    J->ticket = S->next_ticket++;
    S->waiting.push_back(J);
    S->jobs[J->ticket] = J;
    *ticket = J->ticket;
    return PMS_OK;
}

// One tick: admit waiting jobs that fit (in arrival order), then advance
// every admitted job by one step -- re-layout, patch statistics and the
// random initialisation for the newly admitted ones, one half-sweep for all
// (each at its own iteration and colour), output and consistency for those
// that finish -- with one launch per step kind and kernel variant.
pms_status pms_server_step(pms_server *S, void *stream, int32_t *active_out, int32_t *waiting_out)
{
    if (!S) return PMS_ERR_INVALID_ARG;
    pms_context *ctx = S->ctx;
    ctx->last_error.clear();
    pms_status st = set_device(ctx);
    if (st != PMS_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e;
    // bound the ticks in flight
    hipEvent_t &slot_ev = S->tick_events[S->tick_next];
    if (slot_ev) {
        e = hipEventSynchronize(slot_ev);
        if (e != hipSuccess) return hip_fail(ctx, e, "tick wait");
    }
    // admission, first come first served: a job that does not fit holds
    // back the ones behind it
    while (!S->waiting.empty()) {
        ServerJob *J = S->waiting.front();
        if (!server_admit(S, J)) break;
        S->waiting.erase(S->waiting.begin());
        J->state = SJ_RUNNING;
        J->fresh = true;
        if ((st = server_fill_slot(S, J)) != PMS_OK) return st;
        S->running.push_back(J);
    }
    if (active_out) *active_out = (int32_t)S->running.size();
    if (waiting_out) *waiting_out = (int32_t)S->waiting.size();
    if (S->running.empty()) return PMS_OK;

    Plan P;
    P.jobs = S->table;
    P.off_pads = S->off_pads;
    P.off_entries = S->off_entries;
    P.args_bytes = S->args_bytes;
    using Items = std::vector<std::tuple<int, int, int, int>>;
    const Variant none{0, 0, false};
    {
        Items items;
        for (auto &kv : S->pads)
            if (!kv.second.laid_out) {
                items.emplace_back((int)P.pads.size(),
                                   (int)blocks_of(pad_cells(kv.second.job.W, kv.second.job.H)), 0, 0);
                P.pads.push_back(kv.second.job);
                kv.second.laid_out = true;
            }
        add_rec(P, KK_IO, IO_PAD, 0, none, items);
    }
    std::map<GroupKey, std::vector<ServerJob *>> groups;
    for (ServerJob *J : S->running) groups[group_key(J->spec, J->geo)].push_back(J);
    {
        Items items;
        for (ServerJob *J : S->running)
            if (J->fresh) items.emplace_back(J->slot, (int)blocks_of((long long)J->spec.W * J->spec.H), 0, 0);
        add_rec(P, KK_REFSTATS, 0, 0, none, items);
    }
    for (auto &kv : groups) {
        Items items;
        for (ServerJob *J : kv.second)
            if (J->fresh) items.emplace_back(J->slot, J->geo.tiles_x_all * J->geo.tiles_y_all, 0, 0);
        add_rec(P, KK_INIT, 0, std::get<0>(kv.first), kv.second[0]->geo.v, items);
    }
    for (auto &kv : groups) {
        Items items;
        for (ServerJob *J : kv.second)
            if (J->steps_done < 2 * J->params.iterations) {
                items.emplace_back(J->slot, J->geo.tiles_x_half * J->geo.tiles_y_half,
                                   J->steps_done / 2 + 1, J->steps_done % 2);
                J->steps_done += 1;
            }
        add_rec(P, KK_HALFSWEEP, 0, std::get<0>(kv.first), kv.second[0]->geo.v, items);
    }
    std::vector<ServerJob *> finishing, still;
    for (ServerJob *J : S->running) {
        J->fresh = false;
        if (J->steps_done >= 2 * J->params.iterations) finishing.push_back(J);
        else still.push_back(J);
    }
    {
        Items fin, med, geo;
        for (ServerJob *J : finishing) {
            const int blocks = (int)blocks_of((long long)J->spec.W * J->spec.H);
            fin.emplace_back(J->slot, blocks, 0, 0);
            if (J->params.median_radius > 0) med.emplace_back(J->slot, median_tiles(J->spec.W, J->spec.H), 0, 0);
            if (J->job.n_maps > 0) geo.emplace_back(J->slot, blocks, 0, 0);
        }
        add_rec(P, KK_FINALIZE, 0, 0, none, fin);
        add_rec(P, KK_MEDIAN, 0, 0, none, med);
        add_rec(P, KK_CONSISTENCY, 0, 0, none, geo);
    }
    if ((int)P.pads.size() > S->max_pads || (int)P.entries.size() > S->max_entries)
        return fail(ctx, PMS_ERR_UNSUPPORTED, "tick exceeds the server's table sizes");
    char *dev = static_cast<char *>(S->block);
    if ((st = upload_args(ctx, P, dev, s)) != PMS_OK) return st;
    if ((st = enqueue_plan(ctx, P, dev, s)) != PMS_OK) return st;
    // the tick's event: completion of every job finishing in it
    if (!slot_ev) {
        e = hipEventCreateWithFlags(&slot_ev, hipEventDisableTiming);
        if (e != hipSuccess) return hip_fail(ctx, e, "hipEventCreate");
    }
    e = hipEventRecord(slot_ev, s);
    if (e != hipSuccess) return hip_fail(ctx, e, "hipEventRecord");
    S->tick_next = (S->tick_next + 1) % kTicksInFlight;
    for (ServerJob *J : finishing) {
        if (!S->spare_events.empty()) {
            J->done = S->spare_events.back();
            S->spare_events.pop_back();
        } else {
            e = hipEventCreateWithFlags(&J->done, hipEventDisableTiming);
            if (e != hipSuccess) return hip_fail(ctx, e, "hipEventCreate");
        }
        e = hipEventRecord(J->done, s);
        if (e != hipSuccess) return hip_fail(ctx, e, "hipEventRecord");
        J->state = SJ_DONE;
        // later ticks on this stream run after this one, so the memory can
        // be handed out again right away
        server_release(S, J);
    }
    S->ticks += 1;
    S->job_ticks += (int64_t)S->running.size();
    S->running.swap(still);
    return PMS_OK;
}

pms_status pms_server_poll(pms_server *S, int64_t ticket, int32_t *state)
{
    if (!S || !state) return PMS_ERR_INVALID_ARG;
    auto it = S->jobs.find(ticket);
    if (it == S->jobs.end()) return fail(S->ctx, PMS_ERR_INVALID_ARG, "unknown or collected ticket");
    ServerJob *J = it->second;
    if (J->state != SJ_DONE) {
        *state = J->state;
        return PMS_OK;
    }
    hipError_t e = hipEventQuery(J->done);
    if (e == hipErrorNotReady) {
        *state = SJ_RUNNING;
        return PMS_OK;
    }
    if (e != hipSuccess) return hip_fail(S->ctx, e, "hipEventQuery");
    *state = SJ_DONE;
    S->spare_events.push_back(J->done);
    S->jobs.erase(it);
    delete J;
    return PMS_OK;
}

pms_status pms_server_stats(const pms_server *S, int64_t *ticks, int64_t *job_ticks,
                            size_t *arena_used, size_t *arena_peak)
{
    if (!S) return PMS_ERR_INVALID_ARG;
    if (ticks) *ticks = S->ticks;
    if (job_ticks) *job_ticks = S->job_ticks;
    if (arena_used) *arena_used = S->arena.used();
    if (arena_peak) *arena_peak = S->peak_bytes;
    return PMS_OK;
}

pms_status pms_server_destroy(pms_server *S)
{
    if (!S) return PMS_ERR_INVALID_ARG;
    if (S->ctx->device >= 0) {
        (void)hipSetDevice(S->ctx->device);
        (void)hipDeviceSynchronize();
    }
    for (auto &kv : S->jobs) {
        if (kv.second->done) (void)hipEventDestroy(kv.second->done);
        delete kv.second;
    }
    for (auto e : S->tick_events)
        if (e) (void)hipEventDestroy(e);
    for (auto e : S->spare_events) (void)hipEventDestroy(e);
    if (S->block) (void)hipFree(S->block);
    delete S;
    return PMS_OK;
}

}  // extern "C"
