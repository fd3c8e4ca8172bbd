// pms_kernels.hpp -- gfx950 kernels of equirectangular PatchMatch-Stereo
// densification (Surmann et al., Sec. III-B/C). Included once, by pms.hip.
//
// Work decomposition
//   * One reference pixel is served by LPP (2, 4 or 8) adjacent lanes of a
//     wave64 inside one half row of 8 lanes. Each lane owns every LPP-th
//     patch sample: its bearing, its centred reference value and, per view,
//     its warped neighbour value stay in VGPRs; patch sums are reduced
//     inside the group with DPP adds (quad_perm, then row_half_mirror for 8
//     lanes), so the reduction order depends on the patch and the context's
//     schedule only, never on the launch.
//   * A workgroup of 256 threads covers a (32/LPP) x 8 tile of pixels of one
//     colour (red-black sweep) or of all pixels (init / cost evaluation); tiles are
//     handed out so that each XCD walks a contiguous band of rows and keeps
//     the matching part of the neighbour images in its own L2.
//   * Neighbour images are re-laid out once per call as bilinear cells (a
//     corner value and its three differences in FP32, 16 bytes; 8 bytes of
//     halves for FP16 and 8-bit images): every row is repeated around the
//     seam to width 2W + 4 (columns -W/2-2 .. 3W/2+1), and the first and
//     last rows are repeated once more above and below (the clamped pole
//     taps). Any warped sample then reads its whole 2x2 neighbourhood as
//     one buffer load at an offset from its anchor, with no seam or pole
//     test; the buffer descriptor's range check (and, in the ragged-patch
//     variants, a clamp of the offset) keeps every load inside the storage
//     whatever the inputs.
//   * Precision split: what is shared by all samples of one (pixel,
//     hypothesis, view) -- relative pose, plane homography, anchor rotation,
//     warped centre ray and its latitude offset -- is formed in FP64 (on
//     MI355X an FP64 FMA issues at the FP32 rate); each sample then works in
//     FP32 on small quantities only: its bearing minus the centre bearing
//     (formed in FP64 at set-up), the homography applied to that difference,
//     and local angles. A shared rounding would shift the whole patch
//     coherently, which NCC feels most; per-sample roundings of small
//     offsets do not.
//
// Warp. With the plane {X : n.X = c}, c = d (n.b_p) < 0, the neighbour ray of
// sample bearing b_q is a positive multiple of M b_q, M = (-c) R - t n^T,
// whenever the plane lies in front of the sample ray (n.b_q < 0); its pixel
// equals that of R X_q + t with X_q = (c / n.b_q) b_q.
//
// Anchored coordinates. A pixel coordinate near 1920 carries only ~1e-4 px
// in FP32, which is felt by NCC at the 1e-4 level. Each (pixel, hypothesis,
// view) therefore picks an anchor pixel (U0, V0) next to the warped patch
// centre: M is turned about the vertical by the anchor column's longitude, so
// a sample's longitude offset is atan2 of the turned ray, and its latitude
// offset from the anchor row is atan2 of sin/cos of the difference, which is
// the centre's (FP64) plus a small per-sample increment. The offsets are
// small and carry FP32 relative precision; only integers are added to the
// anchor.
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace pms {

constexpr int MAXV = 8;       // neighbour views per launch
constexpr int MAXK = 4;       // views averaged (top_k)
constexpr int MAXOFF = 16;    // propagation offsets
constexpr int MAXTRIAL = 16;  // refinement trials
constexpr int BLOCK = 256;    // threads per workgroup (4 waves)

// Occupancy target of the PatchMatch kernels (waves per SIMD). Up to 9
// samples per lane: exactly 3 (168 VGPRs; measured at 1920x960, 4
// neighbours: 51.3 ms per keyframe, against 54.2 ms at exactly 4 waves,
// 59.8 ms at 2, and 58 ms when the compiler may choose between 3 and 8),
// at least 3 for the per-view cost evaluation. 13 and 16 samples per lane:
// exactly 2, with up to 256 VGPRs for a view's gathers in flight together
// (at 3 waves they spill 240-330 bytes per lane, or wait after each
// gather: the 3840x1920 8-bit courtyard then takes 1013 ms per keyframe
// instead of 847).
#define PMS_OCCUPANCY(KIND, SPL) \
    __attribute__((amdgpu_waves_per_eu((SPL) <= 9 ? 3 : 2, (SPL) <= 9 ? ((KIND) == TK_EVAL ? 8 : 3) : 2)))
// Re-laid-out neighbour image: H + 1 rows of 2W + 4 bilinear cells (16 or
// 8 bytes, see Cell8); logical column x is stored at x + W/2 + 2, logical
// row y at y + 1.

// dtype codes of the C ABI
constexpr int DT_F32 = 0, DT_F16 = 1, DT_U8 = 2;

struct ViewPoseF {
    float R[9];
    float t[3];
    float tnorm;  // |t|, rounded up
};

struct ViewPoseD {
    double R[9];
    double t[3];
};

struct ImgRef {
    const void *ptr;
    long long pitch;  // bytes
};

// Everything a sweep / init / eval launch needs; passed by value.
struct SweepArgs {
    int W, H, r, stride, side, P;
    float inv_P;
    int n_views, top_k;
    float inv_k;  // fl(1 / top_k)
    float var_floor;     // of the reference patch variance
    float var_floor_s;   // of the warped samples' variance, in their cells'
                         // units (8-bit cells hold raw 0..255: x 255^2)
    float dmin, dmax, inv_dmin, inv_dmax;
    float kx, cx, ky, cy;  // u = lam * kx + cx, v = phi * ky + cy
    float patch_chord;     // bound on |b_q - b_p| over the patch, with a margin
    int n_offsets;
    int off_x[MAXOFF], off_y[MAXOFF];
    int refine_trials;
    float sd[MAXTRIAL], sn[MAXTRIAL];  // per trial: log2-depth and normal spread
    unsigned long long seed;
    // tile shape: a wave covers (1 << wx_log2) x ((64 / LPP) >> wx_log2)
    // pixels, a workgroup (1 << bx_log2) x (4 >> bx_log2) waves
    int wx_log2, bx_log2;
    int tile_w, tile_h;      // tile size in pixels
    int tiles_x_all;         // tiles per tile row over all pixels
    int tiles_x_half;        // ... over the pixels of one colour
    int ref_dtype;
    int own_costs;           // stored costs were computed by these kernels
    ImgRef ref;
    ViewPoseD pose[MAXV];    // relative poses in FP64 (warped centre ray)
    ViewPoseF posef[MAXV];   // the same rounded (homography on offsets)
    const void *pad[MAXV];  // re-laid-out neighbours, (H + 1) x Wp bilinear cells
    int Wp;                 // their pitch in elements, 2W + 4
    int pad_bytes;          // bytes of one re-laid-out image
    const float2 *tab_row;  // per row (sin phi, cos phi)
    const float2 *tab_col;  // per column (sin lam, cos lam)
    const double2 *tab_row64;
    const double2 *tab_col64;
    const float2 *stats;    // per pixel (mean, variance) of the reference patch
    float4 *state;          // per pixel (nx, ny, nz, depth)
    float *cost;            // per pixel aggregated cost
    // caller planes (eval)
    const float *in_depth;
    const float *in_n0, *in_n1, *in_n2;
    long long in_pitch;
    float *out_cost;
    long long out_pitch;
    float *view_out[MAXV];
    // initial planes (e.g. the previous keyframe's map carried over); null
    // for a random initialisation everywhere
    const float *init_depth;
    const float *init_n0, *init_n1, *init_n2;
    long long init_pitch;
};

// A bilinear cell of a re-laid-out neighbour image, for the corners a, b
// (row r0) and e, f (row r1). FP32 images: the corner value and its three
// differences a, b - a, e - a, (f - e) - (b - a) in FP32 (float4, 16
// bytes). FP16 images: the four corner values as halves (a, b | e, f), 8
// bytes, exact. 8-bit images: the corner value and its three differences
// as halves of the raw values 0..255, 8 bytes, exact (integers within
// +-510).
struct Cell8 {
    unsigned ab, ef;
};
struct Cell8d {
    unsigned lo, hi;
};

template <int DT>
struct Storage;
template <>
struct Storage<DT_F32> {
    using ref_t = float;
    using pad_t = float4;
};
template <>
struct Storage<DT_F16> {
    using ref_t = __half;
    using pad_t = Cell8;
};
template <>
struct Storage<DT_U8> {
    using ref_t = uint8_t;
    using pad_t = Cell8d;
};

// log2 of a cell's size in bytes: sample offsets are cell index << shift
template <typename PT>
constexpr int cell_shift()
{
    static_assert(sizeof(PT) == 16 || sizeof(PT) == 8, "cells are 8 or 16 bytes");
    return sizeof(PT) == 16 ? 4 : 3;
}

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------

// Sum over the LPP lanes of a pixel: quad_perm [1,0,3,2], then (LPP >= 4)
// [2,3,0,1], then (LPP = 8) row_half_mirror, which pairs each lane of one
// quad with a lane of the other quad of its 8. Every lane of the group
// ends with the same bits ((a+b)+(c+d) == (b+a)+(d+c) exactly, and the
// last step adds the two quads' equal sums in either order).
template <int LPP>
__device__ __forceinline__ float group_sum(float v)
{
    v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xB1, 0xF, 0xF, true));
    if (LPP >= 4) v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x4E, 0xF, 0xF, true));
    if (LPP == 8) v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x141, 0xF, 0xF, true));
    return v;
}

template <int LPP>
__device__ __forceinline__ int group_and(int v)
{
    v &= __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, true);
    if (LPP >= 4) v &= __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, true);
    if (LPP == 8) v &= __builtin_amdgcn_mov_dpp(v, 0x141, 0xF, 0xF, true);
    return v;
}

template <typename T>
__device__ __forceinline__ float load_px(const ImgRef &im, int x, int y);

template <>
__device__ __forceinline__ float load_px<float>(const ImgRef &im, int x, int y)
{
    return reinterpret_cast<const float *>(static_cast<const char *>(im.ptr) + (long long)y * im.pitch)[x];
}

template <>
__device__ __forceinline__ float load_px<__half>(const ImgRef &im, int x, int y)
{
    return __half2float(
        reinterpret_cast<const __half *>(static_cast<const char *>(im.ptr) + (long long)y * im.pitch)[x]);
}

template <>
__device__ __forceinline__ float load_px<uint8_t>(const ImgRef &im, int x, int y)
{
    return (float)(static_cast<const uint8_t *>(im.ptr) + (long long)y * im.pitch)[x] * (1.0f / 255.0f);
}

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void *p, int bytes)
{
    // raw buffer (stride 0), gfx9 descriptor word 3
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, bytes, 0x00020000);
}

// Halves of a 32-bit word as floats (exact).
__device__ __forceinline__ float half_lo(unsigned w)
{
    return (float)__builtin_bit_cast(_Float16, (unsigned short)(w & 0xffffu));
}
__device__ __forceinline__ float half_hi(unsigned w)
{
    return (float)__builtin_bit_cast(_Float16, (unsigned short)(w >> 16));
}

// lo + t (hi - lo) for the two halves of w, as fl(t hi + fl(lo - t lo)) in
// FP32: the compiler makes each step one v_fma_mix_f32, which reads the
// half operand exactly.
__device__ __forceinline__ float lerp_halves(unsigned w, float t)
{
    const float lo = half_lo(w), hi = half_hi(w);
    return fmaf(t, hi, fmaf(-t, lo, lo));
}

// A bilinear sample is one buffer load of the cell at byte offset `off` of a
// re-laid-out neighbour image (load_cell) and its blend with the fractions
// au, av along x and y (blend_cell); the two are separate so that a view's
// gathers can all be issued before the first blend.
template <typename PT>
struct CellBits {
    using type = uint2;
};
template <>
struct CellBits<float4> {
    using type = float4;
};

template <typename PT>
__device__ __forceinline__ typename CellBits<PT>::type load_cell(__amdgpu_buffer_rsrc_t r, int off)
{
    if constexpr (sizeof(PT) == 16)
        return __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
    else
        return __builtin_bit_cast(uint2, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}

template <typename PT>
__device__ __forceinline__ float blend_cell(typename CellBits<PT>::type q, float au, float av)
{
    if constexpr (__is_same(PT, float4)) {
        // FP32 corner and differences: three FMAs
        const float top = fmaf(au, q.y, q.x);
        const float dv = fmaf(au, q.w, q.z);
        return fmaf(av, dv, top);
    } else if constexpr (__is_same(PT, Cell8d)) {
        // corner and differences in halves: the same three FMAs, two mixed
        const float top = fmaf(au, half_hi(q.x), half_lo(q.x));
        const float dv = fmaf(au, half_hi(q.y), half_lo(q.y));
        return fmaf(av, dv, top);
    } else {
        // four corner halves: six FMAs, four mixed
        const float top = lerp_halves(q.x, au);
        const float bot = lerp_halves(q.y, au);
        return fmaf(av, bot, fmaf(-av, top, top));
    }
}

__device__ __forceinline__ void bearing(const SweepArgs &A, int x, int y, float b[3])
{
    float2 rw = A.tab_row[y], cl = A.tab_col[x];
    b[0] = rw.y * cl.x;
    b[1] = -rw.x;
    b[2] = rw.y * cl.y;
}

// min(max(x, 0), hi) in one instruction (hi >= 0, the same in every lane).
__device__ __forceinline__ int clamp0_int(int x, int hi)
{
    int r;
    asm("v_med3_i32 %0, %1, 0, %2" : "=v"(r) : "v"(x), "s"(hi));
    return r;
}

// floor(x) as an integer in one instruction (x finite and in int range).
__device__ __forceinline__ int floor_int(float x)
{
    int r;
    asm("v_cvt_flr_i32_f32 %0, %1" : "=v"(r) : "v"(x));
    return r;
}

// atan(t) for |t| <= tan(pi/8): t + t s P(s), s = t^2, with a degree-2 P
// fitted for minimum relative error (7.1e-7 in FP32; atan_coeffs.py): a
// sample 5 px from its anchor lands within 4e-6 px of the exact angle's
// position. Odd in t bit for bit: round-to-nearest is symmetric.
constexpr float TAN_PI_8 = 0.41421356f;
// tan(pi/8) less a margin for the rounding of the range test itself
constexpr float SHORT_RANGE = 0.4141f;

__device__ __forceinline__ float atan_core(float t)
{
    const float s = t * t;
    float p = fmaf(s, -1.122516319e-01f, 1.971414387e-01f);
    p = fmaf(p, s, -3.332550824e-01f);
    return fmaf(t * s, p, t);
}

// G(u) = 1 / (1 + sqrt(1 + u)) for u in [0, tan^2(pi/8)], so that
// y2 sqrt(1 + tau^2) = y2 + y2 u G(u) with u = tau^2: degree 3, fitted for
// minimum relative error (2.8e-7 in exact arithmetic, 3.3e-7 evaluated in
// FP32; hz_coeffs.py). The error enters the length through y2 u G(u) only,
// so the length itself is off by at most 2.7e-8 of it, below its FP32
// rounding.
__device__ __forceinline__ float hz_core(float u)
{
    float p = fmaf(u, -3.114441782e-02f, 6.170029193e-02f);
    p = fmaf(p, u, -1.249734089e-01f);
    return fmaf(p, u, 4.999998510e-01f);
}

// atan2 for any arguments (both zero give 0): octant reduction to t in
// [0, 1], then t > tan(pi/8) is mapped to (t - 1) / (t + 1) in (-tan(pi/8), 0]
// with atan t = pi/4 + atan((t - 1) / (t + 1)).
__device__ __forceinline__ float atan2_full(float y, float x)
{
    const float ax = fabsf(x), ay = fabsf(y);
    const float mx = fmaxf(fmaxf(ax, ay), 1e-30f);
    const float mn = fminf(ax, ay);
    const float t = mn * __builtin_amdgcn_rcpf(mx);
    const bool big = t > TAN_PI_8;
    const float u = big ? (t - 1.0f) * __builtin_amdgcn_rcpf(t + 1.0f) : t;
    float r = atan_core(u) + (big ? 0.78539816339744831f : 0.0f);
    r = ay > ax ? 1.57079632679489662f - r : r;
    r = x < 0.0f ? 3.14159265358979324f - r : r;
    return copysignf(r, y);
}

// atan2 to within 8.2e-5 rad for any arguments (both zero give 0), for the
// choice of an anchor pixel, which needs the angle only to a small fraction
// of a pixel: octant reduction to t in [0, 1] and a degree-3 polynomial
// fitted there for minimum absolute error (atan_coeffs.py, fit_anchor).
__device__ __forceinline__ float atan2_anchor(float y, float x)
{
    const float ax = fabsf(x), ay = fabsf(y);
    const float mx = fmaxf(fmaxf(ax, ay), 1e-30f);
    const float mn = fminf(ax, ay);
    const float t = mn * __builtin_amdgcn_rcpf(mx);
    const float u = t * t;
    float p = fmaf(u, -3.898651525e-02f, 1.462644637e-01f);
    p = fmaf(p, u, -3.211749792e-01f);
    p = fmaf(p, u, 9.992138147e-01f);
    float r = t * p;
    r = ay > ax ? 1.57079632679489662f - r : r;
    r = x < 0.0f ? 3.14159265358979324f - r : r;
    return copysignf(r, y);
}

// For x > 1e-30 and |y| rcp(x) <= tan(pi/8), atan2_full(y, x) computes
// exactly copysign(atan_core(|y| rcp(x)), y) = atan_core(y rcp(x)). Sample
// angles measured from the anchor take this short form when a bound shows
// that all of them qualify; the forms agree bit for bit where both apply,
// so no result depends on which path a wave takes.

// Philox4x64-10 (Salmon et al., SC'11), counter (c0, c1, c2, c3), key (k0, k1).
__device__ __forceinline__ void philox4x64_10(unsigned long long k0, unsigned long long k1,
                                              unsigned long long c[4])
{
    const unsigned long long M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        unsigned long long lo0 = M0 * c[0], hi0 = __umul64hi(M0, c[0]);
        unsigned long long lo1 = M1 * c[2], hi1 = __umul64hi(M1, c[2]);
        unsigned long long n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
        k0 += 0x9E3779B97F4A7C15ULL;
        k1 += 0xBB67AE8584CAA73BULL;
    }
}

// Four 24-bit uniforms in [0,1) for (seed; pixel, iteration, stage).
__device__ __forceinline__ void uniforms(unsigned long long seed, unsigned long long pixel,
                                         unsigned long long iteration, unsigned long long stage,
                                         float u[4])
{
    unsigned long long c[4] = {pixel, iteration, stage, 0ULL};
    philox4x64_10(seed, 0ULL, c);
#pragma unroll
    for (int i = 0; i < 4; ++i) u[i] = (float)(unsigned int)(c[i] >> 40) * (1.0f / 16777216.0f);
}

// ---------------------------------------------------------------------------
// per-pixel patch context held by the 4 lanes of a quad
// ---------------------------------------------------------------------------

template <int SPL>
struct Patch {
    float b[SPL][3];  // sample bearing minus the pixel's bearing (FP64, rounded)
    float rc[SPL];    // reference samples minus the patch mean (0 if not owned)
    float wt[SPL];    // 1 for a sample this lane owns, else 0
    double bp64[3];   // bearing of the pixel itself
    float bp[3];      // the same, rounded
    float var_r;      // reference patch variance
};

template <typename TR, int LPP, int SPL>
__device__ __forceinline__ void patch_setup(const SweepArgs &A, int x, int y, int lane,
                                            Patch<SPL> &pt)
{
    {
        const double2 rw = A.tab_row64[y], cl = A.tab_col64[x];
        pt.bp64[0] = rw.y * cl.x;
        pt.bp64[1] = -rw.x;
        pt.bp64[2] = rw.y * cl.y;
        for (int a = 0; a < 3; ++a) pt.bp[a] = (float)pt.bp64[a];
    }
    float2 st = A.stats[(long long)y * A.W + x];
    pt.var_r = st.y;
#pragma unroll
    for (int i = 0; i < SPL; ++i) {
        const int q = lane + LPP * i;
        if (q < A.P) {
            const int row = q / A.side;
            const int col = q - row * A.side;
            int xq = x - A.r + col * A.stride;
            xq = xq < 0 ? xq + A.W : (xq >= A.W ? xq - A.W : xq);
            const int yq = y - A.r + row * A.stride;
            const double2 rw = A.tab_row64[yq], cl = A.tab_col64[xq];
            pt.b[i][0] = (float)(rw.y * cl.x - pt.bp64[0]);
            pt.b[i][1] = (float)(-rw.x - pt.bp64[1]);
            pt.b[i][2] = (float)(rw.y * cl.y - pt.bp64[2]);
            pt.rc[i] = load_px<TR>(A.ref, xq, yq) - st.x;
            pt.wt[i] = 1.0f;
        } else {
            // the pixel's own ray, so that the unused slot stays finite
            pt.b[i][0] = 0.0f;
            pt.b[i][1] = 0.0f;
            pt.b[i][2] = 0.0f;
            pt.rc[i] = 0.0f;
            pt.wt[i] = 0.0f;
        }
    }
}

constexpr int SHORT_LON = 1, SHORT_LAT = 2;

// Everything a (pixel, hypothesis, view) shares between its samples.
struct ViewSetup {
    float h[9];          // homography turned by -lam0, on bearing offsets
    float y0c, y2c;      // turned warped centre ray, x and z
    float kc;            // its horizontal length minus y2c
    float sdc, cdc;      // sin / cos of (centre latitude - phi0), scaled
    float sp0, cp0;      // sin / cos of the anchor latitude phi0
    int base;            // byte offset of the anchor in the re-laid-out storage
    int short_ok;        // SHORT_LON / SHORT_LAT: every sample's longitude /
                         // latitude offset is in the short atan range
};

// The job's relative poses, staged in LDS once per workgroup: every lane of
// a pixel sets up another view, so reading them from the argument table
// would take vector loads per lane and view set-up.
struct PoseStage {
    ViewPoseD d[MAXV];
    ViewPoseF f[MAXV];
};

__device__ __forceinline__ PoseStage &pose_stage()
{
    __shared__ PoseStage stage;
    return stage;
}

// Copies the poses of A's views into the stage; every thread of the
// workgroup calls it (it ends with a workgroup barrier).
__device__ __forceinline__ void stage_poses(const SweepArgs &A)
{
    PoseStage &S = pose_stage();
    const int nd = A.n_views * (int)(sizeof(ViewPoseD) / sizeof(double));
    const int nf = A.n_views * (int)(sizeof(ViewPoseF) / sizeof(float));
    const double *srcd = reinterpret_cast<const double *>(A.pose);
    const float *srcf = reinterpret_cast<const float *>(A.posef);
    for (int i = threadIdx.x; i < nd; i += BLOCK) reinterpret_cast<double *>(S.d)[i] = srcd[i];
    for (int i = threadIdx.x; i < nf; i += BLOCK) reinterpret_cast<float *>(S.f)[i] = srcf[i];
    __syncthreads();
}

// R_j b_p of the views a lane sets up (view jb + lane in round jb / LPP):
// it does not depend on the plane, so each lane forms it once per pixel and
// keeps it in LDS (its own slots; registers are spoken for).
template <int LPP>
__device__ __forceinline__ double (&ray_stage())[MAXV / LPP][3][BLOCK]
{
    __shared__ double stage[MAXV / LPP][3][BLOCK];
    return stage;
}

template <int LPP>
__device__ __forceinline__ void stage_rays(const SweepArgs &A, const double bp[3], int lane)
{
    for (int jb = 0; jb < A.n_views; jb += LPP) {
        if (jb + lane >= A.n_views) break;
        const ViewPoseD &V = pose_stage().d[jb + lane];
#pragma unroll
        for (int a = 0; a < 3; ++a)
            ray_stage<LPP>()[jb / LPP][a][threadIdx.x] =
                fma(V.R[3 * a], bp[0], fma(V.R[3 * a + 1], bp[1], V.R[3 * a + 2] * bp[2]));
    }
}

// Sets up view j for plane (n, c) at the pixel of `pt`; mc = -c. Reads the
// poses from the workgroup's stage and R_j b_p from the lane's ray stage.
template <int LPP, int SPL, int SH>
__device__ __forceinline__ void view_setup(const SweepArgs &A, const Patch<SPL> &pt, int j, double mc,
                                           double nbp, float n0, float n1, float n2, ViewSetup &o)
{
    const ViewPoseD &V = pose_stage().d[j];
    const ViewPoseF &Vf = pose_stage().f[j];
    // warped centre ray in FP64: M b_p = (-c) R b_p - t (n . b_p), where
    // M = (-c) R - t n^T is a positive multiple of the plane homography
    double yc[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double rb = ray_stage<LPP>()[j / LPP][a][threadIdx.x];
        yc[a] = fma(mc, rb, -V.t[a] * nbp);
    }
    // anchor: the pixel nearest to the warped centre, up to the error of
    // the anchor atan2 (a pixel next to it at worst; the short-form tests
    // below use the centre's actual offset from it)
    const float lamc = atan2_anchor((float)yc[0], (float)yc[2]);
    const float phic = atan2_anchor((float)-yc[1], __builtin_amdgcn_sqrtf((float)(yc[0] * yc[0] + yc[2] * yc[2])));
    int U0 = (int)floorf(fmaf(lamc, A.kx, A.cx) + 0.5f);
    U0 = U0 >= A.W ? U0 - A.W : (U0 < 0 ? U0 + A.W : U0);
    int V0 = (int)floorf(fmaf(phic, A.ky, A.cy) + 0.5f);
    V0 = V0 < 0 ? 0 : (V0 > A.H - 1 ? A.H - 1 : V0);
    const double2 lam0 = A.tab_col64[U0];  // (sin, cos) of the anchor longitude
    const double2 phi0 = A.tab_row64[V0];  // (sin, cos) of the anchor latitude
    {
        // anchor position in the re-laid-out storage ((H + 1) rows of Wp
        // cells, the image starting at row 1, column W/2 + 2)
        const int U0p = U0 + (A.W >> 1) + 2, V0p = V0 + 1;
        o.base = (V0p * A.Wp + U0p) << SH;
    }
    // centre turned about the vertical by -lam0 (FP64). Its longitude is
    // within a pixel and a half of lam0 (half a pixel, plus the anchor
    // atan2's error), so yr2 > 0 and tau = yr0 / yr2 is small, and the
    // horizontal length yr2 sqrt(1 + tau^2) is yr2 + q - q^2 / (2 yr2), q =
    // yr2 tau^2 / 2, to FP64 precision (the next term is yr2 tau^6 / 16).
    const double yr0 = fma(lam0.y, yc[0], -lam0.x * yc[2]);
    const double yr2 = fma(lam0.x, yc[0], lam0.y * yc[2]);
    o.y0c = (float)yr0;
    o.y2c = (float)yr2;
    const float ry2 = __builtin_amdgcn_rcpf(o.y2c);
    const float q = 0.5f * o.y0c * o.y0c * ry2;
    const double hzc = yr2 + (double)fmaf(-0.5f * q * q, ry2, q);
    // centre: sin and cos of (latitude - phi0), scaled by the ray length
    o.sdc = (float)fma(-yc[1], phi0.y, -hzc * phi0.x);
    o.cdc = (float)fma(hzc, phi0.y, -yc[1] * phi0.x);
    o.kc = (float)(hzc - yr2);
    o.sp0 = (float)phi0.x;
    o.cp0 = (float)phi0.y;
    const float sl0 = (float)lam0.x, cl0 = (float)lam0.y;
    // the homography turned by -lam0, in FP32: it only maps the small
    // offsets of the sample bearings from the centre bearing
    const float mcf = (float)mc;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const float nk = k == 0 ? n0 : k == 1 ? n1 : n2;
        const float m0 = fmaf(mcf, Vf.R[k], -Vf.t[0] * nk);
        const float m1 = fmaf(mcf, Vf.R[3 + k], -Vf.t[1] * nk);
        const float m2 = fmaf(mcf, Vf.R[6 + k], -Vf.t[2] * nk);
        o.h[k] = fmaf(cl0, m0, -sl0 * m2);
        o.h[3 + k] = m1;
        o.h[6 + k] = fmaf(sl0, m0, cl0 * m2);
    }
    // Every sample offset e = h (b_q - b_p) satisfies |e| <= |M|_2 |b_q - b_p|
    // (turning keeps norms), and the spectral norm of M = (-c) R - t n^T is
    // at most -c + |t| for a rotation R and a unit n; the patch chord bounds
    // |b_q - b_p|. Where the centre and that bound keep an angle of every
    // sample in the short form's range, the short form of that angle equals
    // the general one bit for bit.
    const float E = (mcf + Vf.tnorm) * A.patch_chord;
    const float lon_den = o.y2c - E, lat_den = o.cdc - E;
    const bool lon_ok = lon_den > 1e-30f && fabsf(o.y0c) + E <= SHORT_RANGE * lon_den;
    const bool lat_ok = lat_den > 1e-30f && fabsf(o.sdc) + E <= SHORT_RANGE * lat_den;
    o.short_ok = (lon_ok ? SHORT_LON : 0) | (lat_ok ? SHORT_LAT : 0);
}

// Per-lane staging of view set-ups in LDS, one array per field (a lane's
// slot is its thread index), so that every lane of a pixel can read the
// set-up another lane of the same pixel prepared. Only lanes of one wave
// exchange data, and a wave's LDS operations complete in order.
constexpr int SETUP_WORDS = 18;

struct SetupLds {
    float w[SETUP_WORDS][BLOCK];
};

__device__ __forceinline__ void put_setup(SetupLds &L, int slot, const ViewSetup &v)
{
#pragma unroll
    for (int k = 0; k < 9; ++k) L.w[k][slot] = v.h[k];
    L.w[9][slot] = v.y0c;
    L.w[10][slot] = v.y2c;
    L.w[11][slot] = v.kc;
    L.w[12][slot] = v.sdc;
    L.w[13][slot] = v.cdc;
    L.w[14][slot] = v.sp0;
    L.w[15][slot] = v.cp0;
    L.w[16][slot] = __int_as_float(v.base);
    L.w[17][slot] = __int_as_float(v.short_ok);
}

__device__ __forceinline__ void get_setup(const SetupLds &L, int slot, ViewSetup &v)
{
#pragma unroll
    for (int k = 0; k < 9; ++k) v.h[k] = L.w[k][slot];
    v.y0c = L.w[9][slot];
    v.y2c = L.w[10][slot];
    v.kc = L.w[11][slot];
    v.sdc = L.w[12][slot];
    v.cdc = L.w[13][slot];
    v.sp0 = L.w[14][slot];
    v.cp0 = L.w[15][slot];
    v.base = __float_as_int(L.w[16][slot]);
    v.short_ok = __float_as_int(L.w[17][slot]);
}

// Warps the lane's samples into one view and bilinear-samples it: s[i] and
// their (masked) sum. LON / LAT select the short atan form for the
// longitude / latitude offset from the anchor; callers take a short form
// only where it equals the general one bit for bit.
template <typename PT, bool LON, bool LAT, int SPL, bool FULL>
__device__ __forceinline__ float warp_samples(const SweepArgs &A, const Patch<SPL> &pt, const ViewSetup &V,
                                              __amdgpu_buffer_rsrc_t img, int last, float s[SPL])
{
    const float y0c = V.y0c, y2c = V.y2c, kc = V.kc, sdc = V.sdc, cdc = V.cdc;
    const float sp0 = V.sp0, cp0 = V.cp0;
    float sum;
    typename CellBits<PT>::type q[SPL];
    float fu[SPL], fv[SPL];
#pragma unroll
    for (int i = 0; i < SPL; ++i) {
        const float bx = pt.b[i][0], by = pt.b[i][1], bz = pt.b[i][2];
        // the turned homography on the offset from the centre bearing; the
        // x row starts from the centre's x, which is small as well (the
        // anchor is within a pixel and a half of the centre's longitude)
        const float y0 = fmaf(V.h[0], bx, fmaf(V.h[1], by, fmaf(V.h[2], bz, y0c)));
        const float e1 = fmaf(V.h[3], bx, fmaf(V.h[4], by, V.h[5] * bz));
        const float e2 = fmaf(V.h[6], bx, fmaf(V.h[7], by, V.h[8] * bz));
        const float y2 = y2c + e2;
        // tangent of the longitude offset, and hz - hzc without cancellation:
        // with u = tau^2, hz = y2 + y2 u G(u) and hzc = y2c + kc, so
        // hz - hzc = (e2 - kc) + y2 u G(u) while |tau| <= tan(pi/8) (always
        // in the short form; the general form takes the same expression
        // there, so both agree bit for bit). Beyond that the sample lies
        // over 22 degrees of longitude from the anchor (a grazing warp) and
        // the plain difference of the lengths is accurate enough.
        const float tau = y0 * __builtin_amdgcn_rcpf(y2);
        const float u = tau * tau;
        float dhz = fmaf(y2 * u, hz_core(u), e2 - kc);
        if (!LON && !(y2 > 0.0f && fabsf(tau) <= TAN_PI_8))
            dhz = __builtin_amdgcn_sqrtf(fmaf(y0, y0, y2 * y2)) - (y2c + kc);
        const float sd = fmaf(-dhz, sp0, fmaf(-e1, cp0, sdc));
        const float cd = fmaf(dhz, cp0, fmaf(-e1, sp0, cdc));
        // longitude - lam0 and latitude - phi0
        const float dl = LON ? atan_core(tau) : atan2_full(y0, y2);
        const float dp = LAT ? atan_core(sd * __builtin_amdgcn_rcpf(cd)) : atan2_full(sd, cd);
        const float ul = dl * A.kx, vl = dp * A.ky;
        // whole and fractional pixel offsets from the anchor
        const float au = __builtin_amdgcn_fractf(ul), av = __builtin_amdgcn_fractf(vl);
        // |ul| <= W/2 keeps the column inside the repeated storage and the
        // latitude stays within the poles, so the cell lies inside the
        // storage. Whatever the inputs, no load leaves it: an offset past
        // the end (a negative one wraps to a large unsigned value) fails the
        // buffer descriptor's range check and reads zeros. The clamp into
        // the storage is kept where it is free, in the ragged variants (13
        // samples: 7% faster with it, register allocation), and left out of
        // the full ones (1-2% faster without).
        int off = (int)(((unsigned)(__mul24(floor_int(vl), A.Wp) + floor_int(ul)) << cell_shift<PT>()) +
                        (unsigned)V.base);
        if (!FULL) off = clamp0_int(off, last);
        q[i] = load_cell<PT>(img, off);
        fu[i] = au;
        fv[i] = av;
    }
    // Every gather of the view is in flight before the first blend. With 13
    // or 16 samples per lane the compiler would otherwise wait for each
    // gather before issuing the next; the empty asm with a memory clobber
    // keeps the loads above it (3840x1920 courtyard: 845 -> 808 ms per
    // keyframe). With 9 it already issues them together.
    if (SPL > 9) asm volatile("" ::: "memory");
#pragma unroll
    for (int i = 0; i < SPL; ++i) {
        s[i] = blend_cell<PT>(q[i], fu[i], fv[i]);
        const float si = FULL ? s[i] : s[i] * pt.wt[i];
        // (the first term starts the sum: 0 + x costs an addition)
        sum = i == 0 ? si : sum + si;
    }
    return sum;
}

// Aggregated cost of plane (d, n) at the pixel of `pt`: per view, warp every
// sample, bilinear-sample the neighbour, two-pass NCC, cost = 1 - NCC or 2
// when invalid; then the mean of the top_k smallest view costs. All lanes of
// the pixel return the same value. FULL: every lane owns SPL samples (P is
// a multiple of LPP), so no slot is masked. When VIEWS is set, the pixel's
// first lane writes each view's cost to A.view_out[j][out_index].
//
// Views are taken LPP at a time: lane l of the pixel prepares the set-up of
// view jb + l (the FP64 centre ray, the anchor, the turned homography) and
// stages it in LDS; every lane then reads each view's set-up from the slot
// of the lane that made it.
//
// `bound`: the caller only uses the result if it is below `bound`. Once the
// views still to come are fewer than top_k, the aggregate is at least the
// same ascending sum with those views at cost 0; when that is already
// >= bound the remaining views are skipped and a value >= bound returned.
// Float addition and multiplication by fl(1/top_k) round monotonically, so
// every decision the caller takes is the one the full evaluation gives.
// Work a half-sweep actually executes, counted per pixel when the launch
// asks for it (instrumentation only; the decisions are the same either way).
enum WorkField {
    WC_PIXELS,        // pixel updates
    WC_PROP,          // propagation candidates considered (offsets)
    WC_TRIALS,        // refinement trials considered
    WC_SKIP_GEOMETRY, // candidates dropped before scoring: neighbour outside
                      // the band or invalid, plane behind the pixel's ray or
                      // its depth out of range, refined normal not facing
    WC_SKIP_REPEAT,   // propagation candidates equal to the current plane or
                      // to the previous candidate (same cost, cannot win)
    WC_SCORED,        // candidates scored (evaluate calls)
    WC_FACING,        // scored planes not facing every sample ray (cost 2,
                      // no view evaluated)
    WC_VIEWS,         // (pixel, candidate, view) NCC evaluations executed
    WC_PRUNED,        // views skipped by the top-k bound
    WC_FIELDS
};
struct WorkCount {
    unsigned v[WC_FIELDS];
};

template <typename PT, int LPP, int SPL, bool FULL, bool VIEWS, bool COUNT = false>
__device__ __forceinline__ float evaluate(const SweepArgs &A, const Patch<SPL> &pt, float d,
                                          float n0, float n1, float n2, int lane,
                                          long long out_index, float bound = 3.0f,
                                          WorkCount *wc = nullptr)
{
    if (COUNT) wc->v[WC_SCORED]++;
    const double n64[3] = {(double)n0, (double)n1, (double)n2};
    const double nbp = n64[0] * pt.bp64[0] + n64[1] * pt.bp64[1] + n64[2] * pt.bp64[2];
    const double c64 = (double)d * nbp;
    const float nbpf = (float)nbp;
    int ok = c64 < 0.0;
    // |n . (b_q - b_p)| <= |b_q - b_p| <= patch_chord (which carries a
    // margin far above the rounding of den), so a plane with n . b_p below
    // -patch_chord faces every sample ray; the per-sample test below then
    // finds the same
    if (!__all(nbpf < -A.patch_chord)) {
#pragma unroll
        for (int i = 0; i < SPL; ++i) {
            // n . b_q = n . b_p + n . (b_q - b_p)
            const float den = fmaf(n0, pt.b[i][0], fmaf(n1, pt.b[i][1], fmaf(n2, pt.b[i][2], nbpf)));
            ok &= FULL ? (den < 0.0f) : (den < 0.0f || pt.wt[i] == 0.0f);
        }
    }
    ok = group_and<LPP>(ok);
    if (!ok) {
        if (VIEWS && lane == 0)
            for (int j = 0; j < A.n_views; ++j) A.view_out[j][out_index] = 2.0f;
        if (COUNT) wc->v[WC_FACING]++;
        return 2.0f;
    }
    // the offset of the last cell
    const int last = A.pad_bytes - (int)sizeof(PT);
    // the top_k smallest view costs, ascending, as bit patterns: costs are
    // non-negative floats, whose order is that of their bits as unsigned
    unsigned top[MAXK];
#pragma unroll
    for (int i = 0; i < MAXK; ++i) top[i] = 0x40400000u;  // 3.0f

    __shared__ SetupLds setup_lds;
    const int slot0 = (int)threadIdx.x - lane;  // slot of the pixel's first lane
    for (int jb = 0; jb < A.n_views; jb += LPP) {
        if (jb + lane < A.n_views) {
            // (recomputed per round rather than kept live across the
            // sample loops)
            const double nbp_r = (double)n0 * pt.bp64[0] + (double)n1 * pt.bp64[1] + (double)n2 * pt.bp64[2];
            ViewSetup mine;
            view_setup<LPP, SPL, cell_shift<PT>()>(A, pt, jb + lane, -((double)d * nbp_r), nbp_r, n0, n1, n2, mine);
            put_setup(setup_lds, threadIdx.x, mine);
        }
        __builtin_amdgcn_wave_barrier();
        const int nr = min(LPP, A.n_views - jb);
        for (int t = 0; t < nr; ++t) {
            const int j = jb + t;
            if (COUNT) wc->v[WC_VIEWS]++;
            ViewSetup V;
            get_setup(setup_lds, slot0 + t, V);
            const __amdgpu_buffer_rsrc_t img = make_rsrc(A.pad[j], A.pad_bytes);
            float s[SPL];
            float sum;
            if (__all(V.short_ok & SHORT_LAT)) {
                if (__all(V.short_ok & SHORT_LON))
                    sum = warp_samples<PT, true, true, SPL, FULL>(A, pt, V, img, last, s);
                else
                    sum = warp_samples<PT, false, true, SPL, FULL>(A, pt, V, img, last, s);
            } else {
                sum = warp_samples<PT, false, false, SPL, FULL>(A, pt, V, img, last, s);
            }
            sum = group_sum<LPP>(sum);
            const float ms = sum * A.inv_P;
            float m2 = 0.0f, cv = 0.0f;
#pragma unroll
            for (int i = 0; i < SPL; ++i) {
                const float e = FULL ? s[i] - ms : (s[i] - ms) * pt.wt[i];
                m2 = fmaf(e, e, m2);
                cv = fmaf(pt.rc[i], e, cv);
            }
            m2 = group_sum<LPP>(m2);
            cv = group_sum<LPP>(cv);
            const float vs = m2 * A.inv_P, cov = cv * A.inv_P;
            float cj;
            if (pt.var_r < A.var_floor || vs < A.var_floor_s) {
                cj = 2.0f;
            } else {
                float ncc = cov * __builtin_amdgcn_rsqf(pt.var_r * vs);
                ncc = fminf(fmaxf(ncc, -1.0f), 1.0f);
                cj = 1.0f - ncc;
            }
            if (VIEWS && lane == 0) A.view_out[j][out_index] = cj;
            // the next round overwrites the slots read above
            __builtin_amdgcn_wave_barrier();
            // insertion into the ascending list of the MAXK smallest costs so
            // far; slots past top_k only collect larger costs and are never
            // summed
            unsigned cb = __float_as_uint(cj);
            if (A.top_k <= 2) {
                // (the usual two of four views: the other slots stay at 3)
                top[1] = min(top[1], max(top[0], cb));
                top[0] = min(top[0], cb);
            } else {
#pragma unroll
                for (int i = 0; i < MAXK; ++i) {
                    const unsigned lo = min(top[i], cb), hi = max(top[i], cb);
                    top[i] = lo;
                    cb = hi;
                }
            }
            if (!VIEWS) {
                const int have = A.top_k - (A.n_views - 1 - j);  // evaluated costs in the bound
                if (have > 0) {
                    float lb = 0.0f;
#pragma unroll
                    for (int i = 0; i < MAXK; ++i) {
                        if (i >= have) break;
                        lb += __uint_as_float(top[i]);
                    }
                    if (lb * A.inv_k >= bound) {
                        if (COUNT) wc->v[WC_PRUNED] += A.n_views - 1 - j;
                        return lb * A.inv_k;
                    }
                }
            }
        }
    }
    // the mean as sum x fl(1/k): monotone in the sum like the bound above
    float acc = 0.0f;
#pragma unroll
    for (int i = 0; i < MAXK; ++i) {
        if (i >= A.top_k) break;
        acc += __uint_as_float(top[i]);
    }
    return acc * A.inv_k;
}

// ---------------------------------------------------------------------------
// launches over job tables
// ---------------------------------------------------------------------------

// Plane state <-> caller planes.
struct IoArgs {
    int W, H, r;
    float4 *state;
    float *cost;
    float *depth, *n0, *n1, *n2, *cplane;
    long long pd, pn0, pn1, pn2, pc;  // pitches in elements
    int median_radius;                // median post-filter (0 = off)
    double median_rel;
};

// Geometric consistency of one keyframe against up to MAXV depth maps.
struct GeoArgs {
    int W, H, r, n_maps, min_views;
    float geo_px, geo_rel;
    float kx, cx, ky, cy;
    const float2 *tab_row, *tab_col;
    ViewPoseF pose[MAXV];
    const float *map[MAXV];
    long long map_pitch[MAXV];
    float *depth, *n0, *n1, *n2, *cost;
    long long pd, pn0, pn1, pn2, pc;
};

// Everything the kernels know about one keyframe job.
struct JobArgs {
    SweepArgs s;
    IoArgs io;
    GeoArgs g;
};

// One neighbour image to re-lay out.
struct PadJob {
    ImgRef src;
    int W, H, Wp, dtype;
    void *dst;
};

// A launch covers a list of entries. Entry e has `tiles` tiles (or blocks),
// split into 8 runs of per_xcd = ceil(tiles / 8), one per XCD; on every XCD
// it owns the workgroup slots [first_e, first_{e+1}) (the list ends with a
// sentinel whose `first` is the slot count). It names its job and, for a
// half-sweep, the job's iteration and colour, so jobs at different stages
// of their sweep can share one launch.
struct Entry {
    int job, first, tiles, per_xcd, iteration, colour;
};

struct Launch {
    const void *table;      // JobArgs[] or PadJob[]
    const Entry *entries;   // n_entries + 1 entries
    int n_entries;
    int slots;              // workgroup slots per XCD; the grid is 8 * slots
    unsigned long long *counts;  // half-sweeps: work counters, or null
};

// The tables are written before a launch and only read by it: reading them
// through the constant address space lets every (wave-uniform) access be a
// scalar load.
#define PMS_CONSTANT __attribute__((address_space(4)))

template <typename T>
__device__ __forceinline__ const T *const_view(const void *base, int i)
{
    const PMS_CONSTANT T *p = (const PMS_CONSTANT T *)base;
    return (const T *)(p + i);
}

// Entry and tile of this workgroup. The 8 XCDs receive workgroups round
// robin; slot = blockIdx / 8 on XCD x = blockIdx % 8 serves tile
// x * per_xcd + (slot - first) of its entry, so every XCD walks one
// contiguous band of rows of each job and keeps the matching rows of that
// job's neighbour images in its own L2. Returns false for the few slots
// past an entry's last tile.
__device__ __forceinline__ bool block_entry(const Launch &L, int &e, int &local)
{
    const int bid = blockIdx.x;
    const int slot = bid >> 3;
    const Entry *E = const_view<Entry>(L.entries, 0);
    if (slot >= E[L.n_entries].first) return false;
    int lo = 0, hi = L.n_entries - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (E[mid].first <= slot) lo = mid;
        else hi = mid - 1;
    }
    e = lo;
    local = (bid & 7) * E[lo].per_xcd + (slot - E[lo].first);
    return local < E[lo].tiles;
}

// Position of this thread's pixel inside its job's tile.
template <int LPP>
__device__ __forceinline__ void tile_pixel(const SweepArgs &A, int tid, int &dx, int &dy, int &lane)
{
    lane = tid & (LPP - 1);
    const int wave = tid >> 6;
    const int piw = (tid & 63) / LPP;
    const int wx = 1 << A.wx_log2;
    const int wy = (64 / LPP) >> A.wx_log2;
    dx = (wave & ((1 << A.bx_log2) - 1)) * wx + (piw & (wx - 1));
    dy = (wave >> A.bx_log2) * wy + (piw >> A.wx_log2);
}

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------

// Bearing tables in FP64, also rounded to FP32.
__global__ void k_tables(int W, int H, float2 *row, float2 *col, double2 *row64, double2 *col64)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const double PI = 3.14159265358979323846;
    if (i < H) {
        const double phi = PI / 2.0 - PI * (i + 0.5) / H;
        const double sp = sin(phi), cp = cos(phi);
        row64[i] = make_double2(sp, cp);
        row[i] = make_float2((float)sp, (float)cp);
    }
    if (i < W) {
        const double lam = 2.0 * PI * (i + 0.5) / W - PI;
        const double sl = sin(lam), cl = cos(lam);
        col64[i] = make_double2(sl, cl);
        col[i] = make_float2((float)sl, (float)cl);
    }
}

// Re-lays out neighbour images as bilinear cells. Storage row py stands for
// image row clamp(py - 1, 0, H - 1) (the rows above the first and below
// the last repeat them: the clamped pole taps), storage column px for image
// column c = (px - W/2 - 2) mod W. Cell (px, py) holds, with a = I(c, r0),
// b = I(c + 1, r0), e = I(c, r1), f = I(c + 1, r1) for the rows r0, r1 of
// storage rows py and py + 1: (a, b - a, e - a, (f - e) - (b - a)) in FP32
// (16-bit values widen exactly; 8-bit ones are scaled to [0, 1]).
template <typename TS>
__device__ __forceinline__ void pad_one(const PadJob &J, long long i)
{
    const int py = (int)(i / J.Wp), px = (int)(i - (long long)py * J.Wp);
    int sx = px - (J.W >> 1) - 2;
    sx = sx < 0 ? sx + J.W : sx;
    sx = sx >= J.W ? sx - J.W : sx;
    const int sx1 = sx + 1 == J.W ? 0 : sx + 1;
    const int r0 = py == 0 ? 0 : py - 1;
    const int r1 = py >= J.H ? J.H - 1 : py;
    const float a = load_px<TS>(J.src, sx, r0);
    const float b = load_px<TS>(J.src, sx1, r0);
    const float e = load_px<TS>(J.src, sx, r1);
    const float f = load_px<TS>(J.src, sx1, r1);
    static_cast<float4 *>(J.dst)[i] = make_float4(a, b - a, e - a, (f - e) - (b - a));
}

// FP16 images: the four corner halves, copied.
__device__ __forceinline__ unsigned half_bits(const ImgRef &im, int x, int y)
{
    return reinterpret_cast<const unsigned short *>(static_cast<const char *>(im.ptr) + (long long)y * im.pitch)[x];
}

__device__ __forceinline__ void pad_one_f16(const PadJob &J, long long i)
{
    const int py = (int)(i / J.Wp), px = (int)(i - (long long)py * J.Wp);
    int sx = px - (J.W >> 1) - 2;
    sx = sx < 0 ? sx + J.W : sx;
    sx = sx >= J.W ? sx - J.W : sx;
    const int sx1 = sx + 1 == J.W ? 0 : sx + 1;
    const int r0 = py == 0 ? 0 : py - 1;
    const int r1 = py >= J.H ? J.H - 1 : py;
    Cell8 c;
    c.ab = half_bits(J.src, sx, r0) | half_bits(J.src, sx1, r0) << 16;
    c.ef = half_bits(J.src, sx, r1) | half_bits(J.src, sx1, r1) << 16;
    static_cast<Cell8 *>(J.dst)[i] = c;
}

// 8-bit images: corner and differences of the raw values, as halves.
__device__ __forceinline__ int raw_u8(const ImgRef &im, int x, int y)
{
    return (static_cast<const uint8_t *>(im.ptr) + (long long)y * im.pitch)[x];
}

__device__ __forceinline__ unsigned half_of_int(int v)
{
    return __builtin_bit_cast(unsigned short, (_Float16)(float)v);
}

__device__ __forceinline__ void pad_one_u8(const PadJob &J, long long i)
{
    const int py = (int)(i / J.Wp), px = (int)(i - (long long)py * J.Wp);
    int sx = px - (J.W >> 1) - 2;
    sx = sx < 0 ? sx + J.W : sx;
    sx = sx >= J.W ? sx - J.W : sx;
    const int sx1 = sx + 1 == J.W ? 0 : sx + 1;
    const int r0 = py == 0 ? 0 : py - 1;
    const int r1 = py >= J.H ? J.H - 1 : py;
    const int a = raw_u8(J.src, sx, r0), b = raw_u8(J.src, sx1, r0);
    const int e = raw_u8(J.src, sx, r1), f = raw_u8(J.src, sx1, r1);
    Cell8d c;
    c.lo = half_of_int(a) | half_of_int(b - a) << 16;
    c.hi = half_of_int(e - a) | half_of_int((f - e) - (b - a)) << 16;
    static_cast<Cell8d *>(J.dst)[i] = c;
}

__global__ __launch_bounds__(BLOCK) void k_pad(Launch L)
{
    int e, local;
    if (!block_entry(L, e, local)) return;
    const Entry &E = *const_view<Entry>(L.entries, e);
    const PadJob &J = *const_view<PadJob>(L.table, E.job);
    const long long i = (long long)local * BLOCK + threadIdx.x;
    if (i >= (long long)(J.H + 1) * J.Wp) return;
    if (J.dtype == DT_F16) pad_one_f16(J, i);
    else if (J.dtype == DT_U8) pad_one_u8(J, i);
    else pad_one<float>(J, i);
}

// Reference patch mean and variance per valid pixel (two-pass, FP32).
template <typename TR>
__device__ __forceinline__ void refstats_one(const SweepArgs &A, long long i)
{
    const int y = (int)(i / A.W), x = (int)(i - (long long)y * A.W);
    float2 out = make_float2(0.0f, 0.0f);
    if (y >= A.r && y <= A.H - 1 - A.r) {
        float sum = 0.0f;
        for (int q = 0; q < A.P; ++q) {
            int row = q / A.side, col = q - row * A.side;
            int xq = x - A.r + col * A.stride;
            xq = xq < 0 ? xq + A.W : (xq >= A.W ? xq - A.W : xq);
            sum += load_px<TR>(A.ref, xq, y - A.r + row * A.stride);
        }
        const float m = sum * A.inv_P;
        float v = 0.0f;
        for (int q = 0; q < A.P; ++q) {
            int row = q / A.side, col = q - row * A.side;
            int xq = x - A.r + col * A.stride;
            xq = xq < 0 ? xq + A.W : (xq >= A.W ? xq - A.W : xq);
            const float e = load_px<TR>(A.ref, xq, y - A.r + row * A.stride) - m;
            v = fmaf(e, e, v);
        }
        out = make_float2(m, v * A.inv_P);
    }
    const_cast<float2 *>(A.stats)[i] = out;
}

__global__ __launch_bounds__(BLOCK) void k_refstats(Launch L)
{
    int e, local;
    if (!block_entry(L, e, local)) return;
    const SweepArgs &A = const_view<JobArgs>(L.table, const_view<Entry>(L.entries, e)->job)->s;
    const long long i = (long long)local * BLOCK + threadIdx.x;
    if (i >= (long long)A.W * A.H) return;
    if (A.ref_dtype == DT_F16) refstats_one<__half>(A, i);
    else if (A.ref_dtype == DT_U8) refstats_one<uint8_t>(A, i);
    else refstats_one<float>(A, i);
}

// Initialisation (Sec. III-B): depth uniform in inverse depth, normal
// uniform on the sphere turned towards the camera -- or the supplied plane
// (plane-map warping) where it is usable -- and its cost.
template <int DT, int LPP, int SPL, bool FULL>
__device__ __forceinline__ void init_tile(const SweepArgs &A, int tile)
{
    using TR = typename Storage<DT>::ref_t;
    using PT = typename Storage<DT>::pad_t;
    int dx, dy, lane;
    tile_pixel<LPP>(A, threadIdx.x, dx, dy, lane);
    const int ty = tile / A.tiles_x_all, tx = tile - ty * A.tiles_x_all;
    const int x = tx * A.tile_w + dx, y = ty * A.tile_h + dy;
    if (x >= A.W || y >= A.H) return;
    const long long idx = (long long)y * A.W + x;
    if (y < A.r || y > A.H - 1 - A.r) {
        if (lane == 0) {
            A.state[idx] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            A.cost[idx] = 2.0f;
        }
        return;
    }
    Patch<SPL> pt;
    patch_setup<TR, LPP, SPL>(A, x, y, lane, pt);
    stage_rays<LPP>(A, pt.bp64, lane);
    float u[4];
    uniforms(A.seed, (unsigned long long)idx, 0ULL, 0ULL, u);
    const float rho = fmaf(u[0], A.inv_dmin - A.inv_dmax, A.inv_dmax);
    const float d_rand = 1.0f / rho;
    const float z = 2.0f * u[1] - 1.0f, a = 6.283185307179586f * u[2];
    const float s = sqrtf(fmaxf(0.0f, 1.0f - z * z));
    float sa, ca;
    sincosf(a, &sa, &ca);
    float n0 = s * ca, n1 = s * sa, n2 = z;
    // the side is decided in FP64 with the FP64 bearing, as every later
    // test of a plane facing the camera is (negation is exact, so the
    // flipped normal faces it in FP64 too)
    const double nb = (double)n0 * pt.bp64[0] + (double)n1 * pt.bp64[1] + (double)n2 * pt.bp64[2];
    if (nb > 0.0) {
        n0 = -n0;
        n1 = -n1;
        n2 = -n2;
    } else if (nb == 0.0) {
        n0 = -pt.bp[0];
        n1 = -pt.bp[1];
        n2 = -pt.bp[2];
    }
    float d = d_rand;
    if (A.init_depth) {
        // a supplied plane replaces the random one where it is usable: depth
        // in range and the normal facing the camera (tested in FP64)
        const long long pi = (long long)y * A.init_pitch + x;
        const float di = A.init_depth[pi];
        const float m0 = A.init_n0[pi], m1 = A.init_n1[pi], m2 = A.init_n2[pi];
        const double mb = (double)m0 * pt.bp64[0] + (double)m1 * pt.bp64[1] + (double)m2 * pt.bp64[2];
        if (di >= A.dmin && di <= A.dmax && mb < 0.0) {
            d = di;
            n0 = m0;
            n1 = m1;
            n2 = m2;
        }
    }
    const float c = evaluate<PT, LPP, SPL, FULL, false>(A, pt, d, n0, n1, n2, lane, 0);
    if (lane == 0) {
        A.state[idx] = make_float4(n0, n1, n2, d);
        A.cost[idx] = c;
    }
}

// One half-sweep (Sec. III-C): propagation from the opposite-colour
// neighbourhood, then random refinement; strictly cheaper candidates win, the
// first in table order on ties. Pixels of the other colour are only read.
template <int DT, int LPP, int SPL, bool FULL, bool COUNT = false>
__device__ __forceinline__ void halfsweep_tile(const SweepArgs &A, int tile, int iteration, int colour,
                                               WorkCount *wc = nullptr)
{
    using TR = typename Storage<DT>::ref_t;
    using PT = typename Storage<DT>::pad_t;
    int dx, dy, lane;
    tile_pixel<LPP>(A, threadIdx.x, dx, dy, lane);
    const int ty = tile / A.tiles_x_half, tx = tile - ty * A.tiles_x_half;
    const int k = tx * A.tile_w + dx;
    const int y = A.r + ty * A.tile_h + dy;
    if (k >= (A.W >> 1) || y > A.H - 1 - A.r) return;
    const int x = 2 * k + ((y + colour) & 1);
    // (32 bits: images hold fewer than 2^31 pixels; one register less to
    // keep through the evaluations)
    const unsigned idx = (unsigned)y * (unsigned)A.W + (unsigned)x;
    if (COUNT) {
        wc->v[WC_PIXELS] = 1;
        wc->v[WC_PROP] = A.n_offsets;
        wc->v[WC_TRIALS] = A.refine_trials;
    }

    Patch<SPL> pt;
    patch_setup<TR, LPP, SPL>(A, x, y, lane, pt);
    stage_rays<LPP>(A, pt.bp64, lane);
    const float4 cur = A.state[idx];
    float bd = cur.w, bn0 = cur.x, bn1 = cur.y, bn2 = cur.z;
    float bc = A.cost[idx];

    // the previous propagation candidate (a repeat of it, or of the current
    // plane, scores exactly the same cost again and cannot win under the
    // strict rule, so it is not evaluated a second time)
    float pd = -1.0f, pn0 = 0.0f, pn1 = 0.0f, pn2 = 0.0f;
    bool loaded = true;  // the current plane is still the one read from the state
    for (int o = 0; o < A.n_offsets; ++o) {
        int qx = x + A.off_x[o];
        qx = qx < 0 ? qx + A.W : (qx >= A.W ? qx - A.W : qx);
        const int qy = y + A.off_y[o];
        if (qy < A.r || qy > A.H - 1 - A.r) {
            if (COUNT) wc->v[WC_SKIP_GEOMETRY]++;
            continue;
        }
        const float4 sq = A.state[(long long)qy * A.W + qx];
        if (!(sq.w > 0.0f)) {
            if (COUNT) wc->v[WC_SKIP_GEOMETRY]++;
            continue;
        }
        float bq[3];
        bearing(A, qx, qy, bq);
        const float cq = sq.w * (sq.x * bq[0] + sq.y * bq[1] + sq.z * bq[2]);
        const float den = sq.x * pt.bp[0] + sq.y * pt.bp[1] + sq.z * pt.bp[2];
        if (!(den < 0.0f)) {
            if (COUNT) wc->v[WC_SKIP_GEOMETRY]++;
            continue;
        }
        const float dd = cq * __builtin_amdgcn_rcpf(den);
        if (!(dd >= A.dmin && dd <= A.dmax)) {
            if (COUNT) wc->v[WC_SKIP_GEOMETRY]++;
            continue;
        }
        // (the stored cost of the current plane is this evaluation's result
        // only when these kernels computed it)
        const bool same_best = (A.own_costs || !loaded) &&
                               __float_as_uint(dd) == __float_as_uint(bd) && __float_as_uint(sq.x) == __float_as_uint(bn0) &&
                               __float_as_uint(sq.y) == __float_as_uint(bn1) && __float_as_uint(sq.z) == __float_as_uint(bn2);
        const bool same_prev = __float_as_uint(dd) == __float_as_uint(pd) && __float_as_uint(sq.x) == __float_as_uint(pn0) &&
                               __float_as_uint(sq.y) == __float_as_uint(pn1) && __float_as_uint(sq.z) == __float_as_uint(pn2);
        if (same_best || same_prev) {
            if (COUNT) wc->v[WC_SKIP_REPEAT]++;
            continue;
        }
        pd = dd;
        pn0 = sq.x;
        pn1 = sq.y;
        pn2 = sq.z;
        const float c = evaluate<PT, LPP, SPL, FULL, false, COUNT>(A, pt, dd, sq.x, sq.y, sq.z, lane, 0, bc, wc);
        if (c < bc) {
            bc = c;
            bd = dd;
            bn0 = sq.x;
            bn1 = sq.y;
            bn2 = sq.z;
            loaded = false;
        }
    }

    // The draws of a trial do not depend on earlier trials: each of the LPP
    // lanes of the pixel computes every LPP-th trial's Philox block and
    // stages it in LDS, and the trial reads its four uniforms from the slot
    // of the lane that drew them (the lanes of a pixel always take the same
    // branches; only lanes of one wave exchange data, in order).
    __shared__ float4 draws_lds[BLOCK];
    const int slot0 = (int)threadIdx.x - lane;
    for (int t = 0; t < A.refine_trials; ++t) {
        const int j = t & (LPP - 1);
        if (j == 0) {
            // (opaque, so that the first round's products are recomputed
            // here rather than held in registers through the evaluations)
            unsigned pix = idx;
            asm volatile("" : "+v"(pix));
            float drawn[4];
            uniforms(A.seed, (unsigned long long)pix, (unsigned long long)iteration, (unsigned long long)(16 + t + lane), drawn);
            __builtin_amdgcn_wave_barrier();
            draws_lds[threadIdx.x] = make_float4(drawn[0], drawn[1], drawn[2], drawn[3]);
            __builtin_amdgcn_wave_barrier();
        }
        const float4 uv = draws_lds[slot0 + j];
        const float u[4] = {uv.x, uv.y, uv.z, uv.w};
        // depth x e^((2u - 1) sigma) as a power of two (|exponent| stays far
        // inside the range where v_exp_f32 is exact to an ulp)
        float dd = bd * __builtin_amdgcn_exp2f((2.0f * u[0] - 1.0f) * A.sd[t]);
        dd = fminf(fmaxf(dd, A.dmin), A.dmax);
        float m0 = fmaf(A.sn[t], 2.0f * u[1] - 1.0f, bn0);
        float m1 = fmaf(A.sn[t], 2.0f * u[2] - 1.0f, bn1);
        float m2 = fmaf(A.sn[t], 2.0f * u[3] - 1.0f, bn2);
        const float len2 = m0 * m0 + m1 * m1 + m2 * m2;
        if (!(len2 > 0.0f)) {
            if (COUNT) wc->v[WC_SKIP_GEOMETRY]++;
            continue;
        }
        const float il = __builtin_amdgcn_rsqf(len2);
        m0 *= il;
        m1 *= il;
        m2 *= il;
        if (!(m0 * pt.bp[0] + m1 * pt.bp[1] + m2 * pt.bp[2] < 0.0f)) {
            if (COUNT) wc->v[WC_SKIP_GEOMETRY]++;
            continue;
        }
        const float c = evaluate<PT, LPP, SPL, FULL, false, COUNT>(A, pt, dd, m0, m1, m2, lane, 0, bc, wc);
        if (c < bc) {
            bc = c;
            bd = dd;
            bn0 = m0;
            bn1 = m1;
            bn2 = m2;
        }
    }
    if (COUNT && lane != 0)
        for (int f = 0; f < WC_FIELDS; ++f) wc->v[f] = 0;
    if (lane == 0) {
        A.state[idx] = make_float4(bn0, bn1, bn2, bd);
        A.cost[idx] = bc;
    }
}

// Cost of caller-given hypotheses at every pixel (the matching cost alone).
template <int DT, int LPP, int SPL, bool FULL>
__device__ __forceinline__ void eval_tile(const SweepArgs &A, int tile)
{
    using TR = typename Storage<DT>::ref_t;
    using PT = typename Storage<DT>::pad_t;
    int dx, dy, lane;
    tile_pixel<LPP>(A, threadIdx.x, dx, dy, lane);
    const int ty = tile / A.tiles_x_all, tx = tile - ty * A.tiles_x_all;
    const int x = tx * A.tile_w + dx, y = ty * A.tile_h + dy;
    if (x >= A.W || y >= A.H) return;
    const long long pin = (long long)y * A.in_pitch + x;
    const long long pout = (long long)y * A.out_pitch + x;
    const float d = A.in_depth[pin];
    if (y < A.r || y > A.H - 1 - A.r || !(d > 0.0f)) {
        if (lane == 0) {
            A.out_cost[pout] = 2.0f;
            for (int j = 0; j < A.n_views; ++j)
                if (A.view_out[j]) A.view_out[j][pout] = 2.0f;
        }
        return;
    }
    Patch<SPL> pt;
    patch_setup<TR, LPP, SPL>(A, x, y, lane, pt);
    stage_rays<LPP>(A, pt.bp64, lane);
    float c;
    if (A.view_out[0])
        c = evaluate<PT, LPP, SPL, FULL, true>(A, pt, d, A.in_n0[pin], A.in_n1[pin], A.in_n2[pin], lane, pout);
    else
        c = evaluate<PT, LPP, SPL, FULL, false>(A, pt, d, A.in_n0[pin], A.in_n1[pin], A.in_n2[pin], lane, pout);
    if (lane == 0) A.out_cost[pout] = c;
}

enum TileKind { TK_INIT = 0, TK_HALFSWEEP = 1, TK_EVAL = 2 };

// The PatchMatch kernels: every workgroup serves one tile of one job.
template <int KIND, int DT, int LPP, int SPL, bool FULL>
__global__ __launch_bounds__(BLOCK) PMS_OCCUPANCY(KIND, SPL) void k_tiles(Launch L)
{
    int e, local;
    if (!block_entry(L, e, local)) return;
    const Entry &E = *const_view<Entry>(L.entries, e);
    const SweepArgs &A = const_view<JobArgs>(L.table, E.job)->s;
    stage_poses(A);
    if (KIND == TK_INIT) init_tile<DT, LPP, SPL, FULL>(A, local);
    else if (KIND == TK_HALFSWEEP) halfsweep_tile<DT, LPP, SPL, FULL>(A, local, E.iteration, E.colour);
    else eval_tile<DT, LPP, SPL, FULL>(A, local);
}

// The half-sweep with its executed work counted: per workgroup the pixels'
// counts are summed in LDS and added to L.counts (WC_FIELDS 64-bit
// counters) with one atomic per field.
template <int DT, int LPP, int SPL, bool FULL>
__global__ __launch_bounds__(BLOCK) PMS_OCCUPANCY(TK_HALFSWEEP, SPL) void k_halfsweep_counted(Launch L)
{
    __shared__ unsigned wg[WC_FIELDS];
    int e, local;
    if (!block_entry(L, e, local)) return;
    if (threadIdx.x < WC_FIELDS) wg[threadIdx.x] = 0;
    const Entry &E = *const_view<Entry>(L.entries, e);
    const SweepArgs &A = const_view<JobArgs>(L.table, E.job)->s;
    stage_poses(A);  // (its barrier also orders the zeroing above)
    WorkCount wc;
    for (int f = 0; f < WC_FIELDS; ++f) wc.v[f] = 0;
    halfsweep_tile<DT, LPP, SPL, FULL, true>(A, local, E.iteration, E.colour, &wc);
    for (int f = 0; f < WC_FIELDS; ++f)
        if (wc.v[f]) atomicAdd(&wg[f], wc.v[f]);
    __syncthreads();
    if (threadIdx.x < WC_FIELDS) atomicAdd(&L.counts[threadIdx.x], (unsigned long long)wg[threadIdx.x]);
}

// Caller planes from the plane state (invalid pixels: depth and normal 0,
// cost 2).
__device__ __forceinline__ void finalize_one(const IoArgs &A, long long i)
{
    const int y = (int)(i / A.W), x = (int)(i - (long long)y * A.W);
    const float4 s = A.state[i];
    const bool ok = y >= A.r && y <= A.H - 1 - A.r && s.w > 0.0f;
    A.depth[(long long)y * A.pd + x] = ok ? s.w : 0.0f;
    A.n0[(long long)y * A.pn0 + x] = ok ? s.x : 0.0f;
    A.n1[(long long)y * A.pn1 + x] = ok ? s.y : 0.0f;
    A.n2[(long long)y * A.pn2 + x] = ok ? s.z : 0.0f;
    A.cplane[(long long)y * A.pc + x] = ok ? A.cost[i] : 2.0f;
}

__global__ __launch_bounds__(BLOCK) void k_finalize(Launch L)
{
    int e, local;
    if (!block_entry(L, e, local)) return;
    const IoArgs &A = const_view<JobArgs>(L.table, const_view<Entry>(L.entries, e)->job)->io;
    const long long i = (long long)local * BLOCK + threadIdx.x;
    if (i >= (long long)A.W * A.H) return;
    finalize_one(A, i);
}

// Median post-filter (Sec. III-C, item 2): a valid depth (from the plane
// state, i.e. before any removal) that deviates from the lower median of the
// valid depths in its (2R+1)^2 window (longitude wrapping, rows beyond the
// image left out) by more than median_rel times that median is removed from
// the output planes. The k-th smallest of the window is found by bisection
// on the bit pattern: positive floats order like their bits.
__device__ __forceinline__ float state_depth(const IoArgs &A, int x, int y)
{
    if (y < A.r || y > A.H - 1 - A.r) return 0.0f;
    const float d = A.state[(long long)y * A.W + x].w;
    return d > 0.0f ? d : 0.0f;
}

// Drops the pixel's output when its depth d deviates from the window's
// median (bit pattern m_bits) by more than median_rel of it.
__device__ __forceinline__ void median_reject(const IoArgs &A, int x, int y, float d, unsigned m_bits)
{
    const double m = (double)__uint_as_float(m_bits);
    if (fabs((double)d - m) > A.median_rel * m) {
        A.depth[(long long)y * A.pd + x] = 0.0f;
        A.n0[(long long)y * A.pn0 + x] = 0.0f;
        A.n1[(long long)y * A.pn1 + x] = 0.0f;
        A.n2[(long long)y * A.pn2 + x] = 0.0f;
        A.cplane[(long long)y * A.pc + x] = 2.0f;
    }
}

// Lower median of up to 25 window values (0 = invalid; n valid): sorted
// in registers as bit patterns (positive floats order like their bits),
// invalid ones as +inf so that they sort last, through Batcher's odd-even
// merge sorting network for 32 slots restricted to its 140 comparators
// among the first 25 (each dropped one would compare a slot with a +inf
// slot above it and change nothing; the restricted network sorts all 2^25
// zero-one inputs). Returns the bit pattern of the ((n - 1) / 2)-th
// smallest.
__device__ __forceinline__ unsigned lower_median25(const float v[25], int n)
{
    const int k = (n - 1) / 2;
    unsigned u[25];
#pragma unroll
    for (int q = 0; q < 25; ++q) u[q] = v[q] > 0.0f ? __float_as_uint(v[q]) : 0x7f800000u;
#pragma unroll
    for (int p = 1; p < 32; p <<= 1)
#pragma unroll
        for (int kk = p; kk >= 1; kk >>= 1)
#pragma unroll
            for (int j = kk % p; j + kk < 32; j += 2 * kk)
#pragma unroll
                for (int i = 0; i < kk; ++i) {
                    const int a = i + j, b = i + j + kk;
                    if (b < 25 && a / (2 * p) == b / (2 * p)) {
                        const unsigned lo = min(u[a], u[b]), hi = max(u[a], u[b]);
                        u[a] = lo;
                        u[b] = hi;
                    }
                }
    unsigned m = u[0];
#pragma unroll
    for (int q = 1; q < 13; ++q) m = q == k ? u[q] : m;
    return m;
}

// Windows wider than 5x5: read from the plane state, the k-th smallest by
// bisection on the bit pattern.
__device__ __forceinline__ void median_wide(const IoArgs &A, int x, int y, float d)
{
    const int R = A.median_radius;
    const int y0 = max(y - R, 0), y1 = min(y + R, A.H - 1);
    int n = 0;
    for (int yy = y0; yy <= y1; ++yy)
        for (int dx = -R; dx <= R; ++dx) {
            // (a window wider than the image wraps more than once)
            const int xx = ((x + dx) % A.W + A.W) % A.W;
            n += state_depth(A, xx, yy) > 0.0f ? 1 : 0;
        }
    const int k = (n - 1) / 2;
    // smallest bit pattern b with #{v <= b} > k
    unsigned lo = 1u, hi = 0x7f800000u;
    while (lo < hi) {
        const unsigned mid = lo + ((hi - lo) >> 1);
        int c = 0;
        for (int yy = y0; yy <= y1; ++yy)
            for (int dx = -R; dx <= R; ++dx) {
                const int xx = ((x + dx) % A.W + A.W) % A.W;
                const float v = state_depth(A, xx, yy);
                c += (v > 0.0f && __float_as_uint(v) <= mid) ? 1 : 0;
            }
        if (c > k) hi = mid;
        else lo = mid + 1;
    }
    median_reject(A, x, y, d, lo);
}

// One workgroup per tile of MED_TW x MED_TH pixels. Windows up to 5x5 (the
// default) read the tile's depths and a 2-pixel halo from LDS: staged once
// per tile from the plane state, the longitude wrapping around the seam,
// rows beyond the image and outside the valid band as 0; each pixel then
// takes its 25 values from LDS into registers.
constexpr int MED_TW = 64, MED_TH = 4;
static_assert(MED_TW * MED_TH == BLOCK, "one pixel per thread");

__global__ __launch_bounds__(BLOCK) void k_median(Launch L)
{
    int e, local;
    if (!block_entry(L, e, local)) return;
    const IoArgs &A = const_view<JobArgs>(L.table, const_view<Entry>(L.entries, e)->job)->io;
    const int tiles_x = (A.W + MED_TW - 1) / MED_TW;
    const int ty = local / tiles_x, tx = local - ty * tiles_x;
    const int x0 = tx * MED_TW, y0 = ty * MED_TH;
    const int x = x0 + (int)(threadIdx.x % MED_TW), y = y0 + (int)(threadIdx.x / MED_TW);
    const bool pixel = x < A.W && y < A.H;
    const int R = A.median_radius;
    if (R > 2) {
        if (!pixel) return;
        const float d = state_depth(A, x, y);
        if (d > 0.0f) median_wide(A, x, y, d);
        return;
    }
    constexpr int SW = MED_TW + 4, SH = MED_TH + 4;
    __shared__ float tile[SH][SW];
    for (int c = threadIdx.x; c < SW * SH; c += BLOCK) {
        const int r = c / SW, col = c - r * SW;
        const int yy = y0 - 2 + r;
        int xx = x0 - 2 + col;
        // (the halo wraps around the seam; more than once on images
        // narrower than the window)
        if (xx < 0 || xx >= A.W) xx = (xx % A.W + A.W) % A.W;
        tile[r][col] = yy >= 0 && yy < A.H ? state_depth(A, xx, yy) : 0.0f;
    }
    __syncthreads();
    if (!pixel) return;
    const int lx = x - x0 + 2, ly = y - y0 + 2;
    const float d = tile[ly][lx];
    if (!(d > 0.0f)) return;
    float v[25];
    int n = 0;
#pragma unroll
    for (int dy = -2; dy <= 2; ++dy)
#pragma unroll
        for (int dx = -2; dx <= 2; ++dx) {
            const float vv = abs(dy) <= R && abs(dx) <= R ? tile[ly + dy][lx + dx] : 0.0f;
            v[(dy + 2) * 5 + dx + 2] = vv;
            n += vv > 0.0f ? 1 : 0;
        }
    median_reject(A, x, y, d, lower_median25(v, n));
}

// Plane state from caller planes (test hook).
__global__ __launch_bounds__(BLOCK) void k_load_state(IoArgs A)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long long)A.W * A.H) return;
    const int y = (int)(i / A.W), x = (int)(i - (long long)y * A.W);
    A.state[i] = make_float4(A.n0[(long long)y * A.pn0 + x], A.n1[(long long)y * A.pn1 + x],
                             A.n2[(long long)y * A.pn2 + x], A.depth[(long long)y * A.pd + x]);
    A.cost[i] = A.cplane[(long long)y * A.pc + x];
}

// Writes back only the pixels of one colour (the ones a half-sweep changed).
__global__ __launch_bounds__(BLOCK) void k_store_colour(IoArgs A, int colour)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long long)A.W * A.H) return;
    const int y = (int)(i / A.W), x = (int)(i - (long long)y * A.W);
    if (((x + y) & 1) != colour || y < A.r || y > A.H - 1 - A.r) return;
    const float4 s = A.state[i];
    A.depth[(long long)y * A.pd + x] = s.w;
    A.n0[(long long)y * A.pn0 + x] = s.x;
    A.n1[(long long)y * A.pn1 + x] = s.y;
    A.n2[(long long)y * A.pn2 + x] = s.z;
    A.cplane[(long long)y * A.pc + x] = A.cost[i];
}

// ---------------------------------------------------------------------------
// geometric consistency
// ---------------------------------------------------------------------------

__device__ __forceinline__ void project(const GeoArgs &A, float y0, float y1, float y2, float &u,
                                        float &v)
{
    const float lam = atan2f(y0, y2);
    const float phi = atan2f(-y1, sqrtf(y0 * y0 + y2 * y2));
    u = fmaf(lam, A.kx, A.cx);
    v = fmaf(phi, A.ky, A.cy);
}

// Per pixel and map: project the pixel's point into the map's camera, read
// the nearest depth there, move that point back into the reference and
// require both the reprojection error (pixels, longitude folded across the
// seam) and the relative range error to be within bounds; keep the pixel if
// at least min_views maps agree.
__device__ __forceinline__ void consistency_one(const GeoArgs &A, long long i)
{
    const int y = (int)(i / A.W), x = (int)(i - (long long)y * A.W);
    const long long id = (long long)y * A.pd + x;
    const float d = A.depth[id];
    int votes = 0;
    if (y >= A.r && y <= A.H - 1 - A.r && d > 0.0f) {
        float2 rw = A.tab_row[y], cl = A.tab_col[x];
        const float X0 = d * rw.y * cl.x, X1 = -d * rw.x, X2 = d * rw.y * cl.y;
        for (int j = 0; j < A.n_maps; ++j) {
            const ViewPoseF &P = A.pose[j];
            const float Y0 = fmaf(P.R[0], X0, fmaf(P.R[1], X1, fmaf(P.R[2], X2, P.t[0])));
            const float Y1 = fmaf(P.R[3], X0, fmaf(P.R[4], X1, fmaf(P.R[5], X2, P.t[1])));
            const float Y2 = fmaf(P.R[6], X0, fmaf(P.R[7], X1, fmaf(P.R[8], X2, P.t[2])));
            float u, v;
            project(A, Y0, Y1, Y2, u, v);
            u = fminf(fmaxf(u, -0.5f), (float)A.W - 0.5f);
            v = fminf(fmaxf(v, -0.5f), (float)A.H - 0.5f);
            int xi = (int)floorf(u + 0.5f);
            xi = xi >= A.W ? xi - A.W : xi;
            int yi = (int)floorf(v + 0.5f);
            yi = yi > A.H - 1 ? A.H - 1 : (yi < 0 ? 0 : yi);
            const float dj = A.map[j][(long long)yi * A.map_pitch[j] + xi];
            if (!(dj > 0.0f)) continue;
            float2 rj = A.tab_row[yi], cj = A.tab_col[xi];
            const float Z0 = dj * rj.y * cj.x - P.t[0];
            const float Z1 = -dj * rj.x - P.t[1];
            const float Z2 = dj * rj.y * cj.y - P.t[2];
            const float B0 = fmaf(P.R[0], Z0, fmaf(P.R[3], Z1, P.R[6] * Z2));
            const float B1 = fmaf(P.R[1], Z0, fmaf(P.R[4], Z1, P.R[7] * Z2));
            const float B2 = fmaf(P.R[2], Z0, fmaf(P.R[5], Z1, P.R[8] * Z2));
            float ub, vb;
            project(A, B0, B1, B2, ub, vb);
            float ddx = ub - (float)x;
            ddx -= (float)A.W * floorf((ddx + 0.5f * (float)A.W) / (float)A.W);
            const float ddy = vb - (float)y;
            const float epx = sqrtf(ddx * ddx + ddy * ddy);
            const float ed = fabsf(sqrtf(B0 * B0 + B1 * B1 + B2 * B2) - d) / d;
            votes += (epx <= A.geo_px && ed <= A.geo_rel) ? 1 : 0;
        }
    }
    if (votes < A.min_views || !(d > 0.0f) || y < A.r || y > A.H - 1 - A.r) {
        A.depth[id] = 0.0f;
        A.n0[(long long)y * A.pn0 + x] = 0.0f;
        A.n1[(long long)y * A.pn1 + x] = 0.0f;
        A.n2[(long long)y * A.pn2 + x] = 0.0f;
        A.cost[(long long)y * A.pc + x] = 2.0f;
    }
}

__global__ __launch_bounds__(BLOCK) void k_consistency(Launch L)
{
    int e, local;
    if (!block_entry(L, e, local)) return;
    const GeoArgs &A = const_view<JobArgs>(L.table, const_view<Entry>(L.entries, e)->job)->g;
    const long long i = (long long)local * BLOCK + threadIdx.x;
    if (i >= (long long)A.W * A.H) return;
    consistency_one(A, i);
}

// ---------------------------------------------------------------------------
// plane-map warping (Sec. III-B): the previous keyframe's plane map carried
// into the current keyframe
// ---------------------------------------------------------------------------

struct WarpArgs {
    int W, H, r;
    double R[9], t[3];  // source camera -> destination camera, FP64
    double dmin, dmax;
    const float *sd, *sn0, *sn1, *sn2;
    long long psd, psn0, psn1, psn2;
    float *dd, *dn0, *dn1, *dn2;
    long long pdd, pdn0, pdn1, pdn2;
    unsigned long long *zbuf;  // per destination pixel: (float range bits << 32) | source index
    const double2 *tab_row64, *tab_col64;
};

__global__ __launch_bounds__(BLOCK) void k_warp_clear(WarpArgs A)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < (long long)A.W * A.H) A.zbuf[i] = ~0ULL;
}

__device__ __forceinline__ void warp_point(const WarpArgs &A, int x, int y, float d, double Y[3])
{
    const double2 rw = A.tab_row64[y], cl = A.tab_col64[x];
    const double X0 = (double)d * (rw.y * cl.x), X1 = (double)d * -rw.x, X2 = (double)d * (rw.y * cl.y);
#pragma unroll
    for (int k = 0; k < 3; ++k) Y[k] = A.R[3 * k] * X0 + A.R[3 * k + 1] * X1 + A.R[3 * k + 2] * X2 + A.t[k];
}

// Nearest pixel of a Wc x Hc equirectangular image to direction Y, in FP64:
// u = Wc (atan2(Y0, Y2) + pi) / (2 pi) - 0.5, v = Hc (pi/2 - atan2(-Y1,
// |(Y0, Y2)|)) / pi - 0.5, the column floor(u + 1/2) wrapped, the row
// floor(v + 1/2) clamped.
__device__ __forceinline__ void nearest_pixel64(const double Y[3], int Wc, int Hc, int &xi, int &yi)
{
    const double PI = 3.14159265358979323846;
    const double lam = atan2(Y[0], Y[2]);
    const double phi = atan2(-Y[1], hypot(Y[0], Y[2]));
    const double u = Wc * (lam + PI) / (2.0 * PI) - 0.5;
    const double v = Hc * (PI / 2.0 - phi) / PI - 0.5;
    double fx = floor(u + 0.5);
    fx -= Wc * floor(fx / Wc);
    xi = (int)fx;
    xi = xi >= Wc ? xi - Wc : (xi < 0 ? xi + Wc : xi);
    const double fy = floor(v + 0.5);
    yi = fy < 0.0 ? 0 : (fy > Hc - 1 ? Hc - 1 : (int)fy);
}

// The same decision from FP32 angles (atan2_full), taken only where it
// provably equals the FP64 one: the FP32 pipeline (Y rounded to FP32,
// atan2_full within 1e-6 rad of the angle, a few FP32 roundings of values
// below Wc + 1) puts u + 1/2 within 3e-7 Wc + 1e-4 of its FP64 value, and
// v + 1/2 within 3e-7 Hc + 1e-4, so when both lie farther than 4e-6 Wc +
// 1e-3 (4e-6 Hc + 1e-3) from an integer, the floors agree. Otherwise, and
// where the ray is too close to a pole for the FP32 lengths, it falls back
// to nearest_pixel64: the result is that of the FP64 formulas.
__device__ __forceinline__ void nearest_pixel(const double Y[3], int Wc, int Hc, int &xi, int &yi)
{
    const float y0 = (float)Y[0], y1 = (float)Y[1], y2 = (float)Y[2];
    const float hz = __builtin_amdgcn_sqrtf(fmaf(y0, y0, y2 * y2));
    const float lam = atan2_full(y0, y2), phi = atan2_full(-y1, hz);
    const float fu = fmaf((float)Wc * 0.15915494f, lam, 0.5f * (float)Wc);
    const float fv = fmaf(-(float)Hc * 0.31830989f, phi, 0.5f * (float)Hc);
    const float gu = fmaf(4e-6f, (float)Wc, 1e-3f), gv = fmaf(4e-6f, (float)Hc, 1e-3f);
    const float ru = fu - floorf(fu), rv = fv - floorf(fv);
    if (!(hz > 1e-18f * fabsf(y1)) || !(ru > gu && ru < 1.0f - gu) || !(rv > gv && rv < 1.0f - gv)) {
        nearest_pixel64(Y, Wc, Hc, xi, yi);
        return;
    }
    int x = (int)floorf(fu);
    x = x >= Wc ? x - Wc : (x < 0 ? x + Wc : x);
    const int y = (int)floorf(fv);
    xi = x;
    yi = y < 0 ? 0 : (y > Hc - 1 ? Hc - 1 : y);
}

// Each valid source pixel claims the destination pixel nearest to the
// projection of its plane point; the smallest key (nearest point, then the
// lower source index) wins, so the outcome does not depend on the order of
// the 64-bit atomics.
__global__ __launch_bounds__(BLOCK) void k_warp_splat(WarpArgs A)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long long)A.W * A.H) return;
    const int y = (int)(i / A.W), x = (int)(i - (long long)y * A.W);
    if (y < A.r || y > A.H - 1 - A.r) return;
    const float d = A.sd[(long long)y * A.psd + x];
    if (!(d > 0.0f)) return;
    double Y[3];
    warp_point(A, x, y, d, Y);
    const double range = sqrt(Y[0] * Y[0] + Y[1] * Y[1] + Y[2] * Y[2]);
    if (!(range > 0.0)) return;
    // (the guarded FP32 decision of nearest_pixel gained nothing here: the
    // splat's time goes to its random 64-bit atomics)
    int xi, yi;
    nearest_pixel64(Y, A.W, A.H, xi, yi);
    if (yi < A.r || yi > A.H - 1 - A.r) return;
    const unsigned long long key =
        ((unsigned long long)__float_as_uint((float)range) << 32) | (unsigned long long)(unsigned)i;
    atomicMin(&A.zbuf[(long long)yi * A.W + xi], key);
}

// The winning plane (normal R n through the moved point) re-intersected
// with the destination pixel's ray; kept if it faces the camera and its
// depth is in range.
__global__ __launch_bounds__(BLOCK) void k_warp_resolve(WarpArgs A)
{
    const long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= (long long)A.W * A.H) return;
    const int yd = (int)(j / A.W), xd = (int)(j - (long long)yd * A.W);
    const unsigned long long key = A.zbuf[j];
    float od = 0.0f, o0 = 0.0f, o1 = 0.0f, o2 = 0.0f;
    if (key != ~0ULL) {
        const long long i = (long long)(key & 0xffffffffULL);
        const int y = (int)(i / A.W), x = (int)(i - (long long)y * A.W);
        const float d = A.sd[(long long)y * A.psd + x];
        double Y[3];
        warp_point(A, x, y, d, Y);
        const double n0 = A.sn0[(long long)y * A.psn0 + x], n1 = A.sn1[(long long)y * A.psn1 + x],
                     n2 = A.sn2[(long long)y * A.psn2 + x];
        double nd[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) nd[k] = A.R[3 * k] * n0 + A.R[3 * k + 1] * n1 + A.R[3 * k + 2] * n2;
        const double2 rw = A.tab_row64[yd], cl = A.tab_col64[xd];
        const double b0 = rw.y * cl.x, b1 = -rw.x, b2 = rw.y * cl.y;
        const double den = nd[0] * b0 + nd[1] * b1 + nd[2] * b2;
        if (den < 0.0) {
            const double dd = (nd[0] * Y[0] + nd[1] * Y[1] + nd[2] * Y[2]) / den;
            if (dd >= A.dmin && dd <= A.dmax) {
                od = (float)dd;
                o0 = (float)nd[0];
                o1 = (float)nd[1];
                o2 = (float)nd[2];
            }
        }
    }
    A.dd[(long long)yd * A.pdd + xd] = od;
    A.dn0[(long long)yd * A.pdn0 + xd] = o0;
    A.dn1[(long long)yd * A.pdn1 + xd] = o1;
    A.dn2[(long long)yd * A.pdn2 + xd] = o2;
}

// ---------------------------------------------------------------------------
// view filter (Sec. III-A, Eq. 1)
// ---------------------------------------------------------------------------

// Counters of the counting kernels (view filter, fuse marks, coverage),
// spread over COUNT_SPREAD slots a cache line apart per counter: workgroup
// w adds its sums to slot w % COUNT_SPREAD with one atomic each, so the
// atomics of different slots proceed in parallel instead of serialising on
// one address (at one address, ~13 ns each: 2048 of them were most of a
// 29 us view filter), and k_count_gather adds the slots up.
constexpr int COUNT_SPREAD = 64;
static_assert(BLOCK >= 2 * COUNT_SPREAD, "a clearing workgroup covers every slot");
constexpr int COUNT_PAD = 16;  // unsigned long longs per slot (128 bytes)
constexpr size_t COUNT_SPREAD_BYTES = 2 * COUNT_SPREAD * COUNT_PAD * sizeof(unsigned long long);

__device__ __forceinline__ unsigned long long *count_slot(unsigned long long *spread, int counter, int slot)
{
    return spread + ((size_t)counter * COUNT_SPREAD + slot) * COUNT_PAD;
}

// Zeroes both counters' slots (one workgroup of 2 * COUNT_SPREAD threads).
__global__ void k_count_clear(unsigned long long *spread)
{
    if (threadIdx.x < 2 * COUNT_SPREAD)
        *count_slot(spread, (int)threadIdx.x / COUNT_SPREAD, (int)threadIdx.x % COUNT_SPREAD) = 0ULL;
}

// out0 (and out1, unless null) = the sums of the two counters' slots (one
// wave of COUNT_SPREAD threads).
__global__ void k_count_gather(unsigned long long *spread, unsigned long long *out0, unsigned long long *out1)
{
    static_assert(COUNT_SPREAD == 64, "one slot per lane of a wave");
    unsigned long long c0 = *count_slot(spread, 0, (int)threadIdx.x);
    unsigned long long c1 = *count_slot(spread, 1, (int)threadIdx.x);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        c0 += __shfl_xor(c0, o, 64);
        c1 += __shfl_xor(c1, o, 64);
    }
    if (threadIdx.x == 0) {
        *out0 = c0;
        if (out1) *out1 = c1;
    }
}

// Workgroups of the counting kernels, which walk their items with a grid
// stride.
constexpr int COUNT_GRID = 8192;

// Adds the workgroup's sums of c0 and c1 to slot blockIdx.x % COUNT_SPREAD
// of the two spread counters with one atomic each; every thread of the
// workgroup must call it.
__device__ __forceinline__ void block_count_add(unsigned long long *spread, unsigned c0, unsigned c1)
{
    __shared__ unsigned part[2][BLOCK / 64];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        c0 += __shfl_xor(c0, o, 64);
        c1 += __shfl_xor(c1, o, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        part[0][threadIdx.x >> 6] = c0;
        part[1][threadIdx.x >> 6] = c1;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t0 = 0, t1 = 0;
        for (int w = 0; w < BLOCK / 64; ++w) {
            t0 += part[0][w];
            t1 += part[1][w];
        }
        const int slot = (int)(blockIdx.x % COUNT_SPREAD);
        if (t0) atomicAdd(count_slot(spread, 0, slot), t0);
        if (t1) atomicAdd(count_slot(spread, 1, slot), t1);
    }
}

// Per sparse point the angle between the directions to the two camera
// centres (FP64); counts of points in [min_deg, max_deg] and of points not
// at a centre. The angle decreases with its cosine: with cmin, cmax the
// cosines of the bounds (2 or -2 where a bound admits or rejects every
// angle), angle >= min_deg is cos < cmin and angle <= max_deg is cos >
// cmax wherever the cosine lies farther than 1e-9 from the bound's (the
// rounding of either form is below 1e-15); within that band the angle
// itself decides, in degrees as before.
__global__ __launch_bounds__(BLOCK) void k_view_filter(double ax, double ay, double az, double bx,
                                                       double by, double bz, const double *pts,
                                                       long long n, double min_deg, double max_deg,
                                                       double cmin, double cmax,
                                                       unsigned long long *spread)
{
    unsigned n_range = 0, n_counted = 0;
    for (long long i = (long long)blockIdx.x * BLOCK + threadIdx.x; i < n; i += (long long)gridDim.x * BLOCK) {
        const double px = pts[3 * i], py = pts[3 * i + 1], pz = pts[3 * i + 2];
        const double a0 = ax - px, a1 = ay - py, a2 = az - pz;
        const double b0 = bx - px, b1 = by - py, b2 = bz - pz;
        const double la = sqrt(a0 * a0 + a1 * a1 + a2 * a2), lb = sqrt(b0 * b0 + b1 * b1 + b2 * b2);
        if (la > 0.0 && lb > 0.0) {
            double cs = (a0 * b0 + a1 * b1 + a2 * b2) / (la * lb);
            cs = cs > 1.0 ? 1.0 : (cs < -1.0 ? -1.0 : cs);
            bool in;
            if (fabs(cs - cmin) > 1e-9 && fabs(cs - cmax) > 1e-9) {
                in = cs < cmin && cs > cmax;
            } else {
                const double deg = acos(cs) * (180.0 / 3.14159265358979323846);
                in = deg >= min_deg && deg <= max_deg;
            }
            n_counted += 1;
            n_range += in ? 1 : 0;
        }
    }
    block_count_add(spread, n_range, n_counted);
}

// ---------------------------------------------------------------------------
// dense point-cloud fusion (Sec. III, point-cloud thread): voxel
// de-duplication of the points of buffered depth maps, and the coverage of a
// panorama by the kept points (the paper's completeness measure)
// ---------------------------------------------------------------------------

constexpr unsigned long long EMPTY_KEY = ~0ULL;

struct FuseArgs {
    int W, H, n_maps;
    double voxel;
    double origin[3];  // voxel coordinates of the first map's camera centre
    const float *depth[MAXV];
    long long pitch[MAXV];
    ViewPoseD pose[MAXV];  // world -> camera of each map
    const double2 *tab_row64, *tab_col64;
    // hash table of 16-byte slots: voxel key at [2h], first (map, pixel) at
    // [2h + 1], so that a point's claim and order share one cache line
    unsigned long long *slots;
    unsigned long long mask;          // capacity - 1 (a power of two, <= 2^31)
    unsigned *claim;                  // per point: its voxel's slot, or NO_CLAIM
    unsigned char *keep;              // n_maps x H x W
    unsigned long long *count;        // the output count
    unsigned long long *spread;       // its spread slots (k_count_gather)
    // coverage
    ViewPoseD view;
    int Wc, Hc;
    unsigned char *cover;
    const unsigned char *keep_in;     // null: every valid pixel
};

__device__ __forceinline__ bool fuse_point(const FuseArgs &A, int m, long long i, double X[3])
{
    const int y = (int)(i / A.W), x = (int)(i - (long long)y * A.W);
    const float d = A.depth[m][(long long)y * A.pitch[m] + x];
    if (!(d > 0.0f)) return false;
    const double2 rw = A.tab_row64[y], cl = A.tab_col64[x];
    const ViewPoseD &P = A.pose[m];
    const double c0 = (double)d * (rw.y * cl.x) - P.t[0];
    const double c1 = (double)d * -rw.x - P.t[1];
    const double c2 = (double)d * (rw.y * cl.y) - P.t[2];
#pragma unroll
    for (int k = 0; k < 3; ++k) X[k] = P.R[k] * c0 + P.R[3 + k] * c1 + P.R[6 + k] * c2;
    return true;
}

// Voxel coordinates relative to the first camera's voxel (an exact integer
// difference, so voxels are the world's), packed 21 bits each (offset
// 2^20); false beyond that.
__device__ __forceinline__ bool voxel_key(const FuseArgs &A, const double X[3], unsigned long long &key)
{
    key = 0ULL;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double v = floor(X[k] / A.voxel) - A.origin[k];
        if (!(v >= -1048576.0 && v < 1048576.0)) return false;
        key = (key << 21) | (unsigned long long)((long long)v + 1048576LL);
    }
    return true;
}

__device__ __forceinline__ unsigned long long hash64(unsigned long long k)
{
    k ^= k >> 33;
    k *= 0xff51afd7ed558ccdULL;
    k ^= k >> 33;
    k *= 0xc4ceb9fe1a85ec53ULL;
    k ^= k >> 33;
    return k;
}

__global__ __launch_bounds__(BLOCK) void k_fuse_clear(FuseArgs A)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i <= (long long)A.mask) {
        A.slots[2 * i] = EMPTY_KEY;
        A.slots[2 * i + 1] = EMPTY_KEY;
    }
    // (the grid has at least 4 workgroups: capacity >= 1024)
    if (i < 2 * COUNT_SPREAD) *count_slot(A.spread, (int)i / COUNT_SPREAD, (int)i % COUNT_SPREAD) = 0ULL;
}

// Each point claims its voxel's slot (linear probing; the table holds at
// least 5/4 as many slots as points, so a free slot is always found) and
// lowers the slot's value to its (map, pixel) order. A slot's key, once
// written, never changes: a plain read that shows a key is final, and only
// a slot that reads as empty (possibly a stale copy) needs the CAS.
//
// One launch per map, in map order. A slot whose order already names an
// earlier map (written by an earlier launch, so final) keeps that order,
// which every point of this map exceeds: such points only read.
//
// A wave takes an 8 x 8 pixel tile of the map. Neighbouring pixels often
// fall into one voxel: a point whose left or upper neighbour in the tile
// (both of lower order) has the same voxel leaves the claim to it. Every
// skipped point has a lower-order point of its voxel in the wave, and the
// lowest-order one of the wave never skips, so each slot still ends with
// its voxel's lowest order, with fewer contended atomics. Every point of
// the map records the slot it claimed, or NO_CLAIM (no valid voxel, or a
// lower-order point of its voxel exists: such a point is never the first
// of its voxel).
constexpr int FUSE_TILE = 8;
constexpr unsigned NO_CLAIM = 0xffffffffu;

__global__ __launch_bounds__(BLOCK) void k_fuse_insert(FuseArgs A, int m)
{
    const int lane = (int)(threadIdx.x & 63u);
    const int wave = (int)(blockIdx.x * (BLOCK / 64) + (threadIdx.x >> 6));
    const int tiles_x = (A.W + FUSE_TILE - 1) / FUSE_TILE;
    const int ty = wave / tiles_x, tx = wave - ty * tiles_x;
    const int x = tx * FUSE_TILE + lane % FUSE_TILE, y = ty * FUSE_TILE + lane / FUSE_TILE;
    const long long HW = (long long)A.W * A.H;
    const long long g = (long long)m * HW + (long long)y * A.W + x;
    const bool in_range = x < A.W && y < A.H;
    unsigned long long key = 0ULL;
    bool have = false;
    if (in_range) {
        double X[3];
        have = fuse_point(A, m, (long long)y * A.W + x, X) && voxel_key(A, X, key);
    }
    const unsigned lo = (unsigned)key, hi = (unsigned)(key >> 32);
    const int hv = have ? 1 : 0;
    const unsigned l_lo = __shfl_up(lo, 1, 64), l_hi = __shfl_up(hi, 1, 64);
    const int l_have = __shfl_up(hv, 1, 64);
    const unsigned u_lo = __shfl_up(lo, FUSE_TILE, 64), u_hi = __shfl_up(hi, FUSE_TILE, 64);
    const int u_have = __shfl_up(hv, FUSE_TILE, 64);
    const bool left = lane % FUSE_TILE != 0 && l_have && l_lo == lo && l_hi == hi;
    const bool up = lane >= FUSE_TILE && u_have && u_lo == lo && u_hi == hi;
    if (!have || left || up) {
        if (in_range) A.claim[g] = NO_CLAIM;
        return;
    }
    const unsigned long long first = (unsigned long long)m * (unsigned long long)HW;
    unsigned long long h = hash64(key) & A.mask;
    for (unsigned long long probe = 0; probe <= A.mask; ++probe) {
        // key and order in one 16-byte read. It may race with this launch's
        // atomics and see either half stale; a stale key reads as empty
        // and an order of this map is not below `first`, so such a read
        // only sends the point on to the CAS and the atomic min, which are
        // exact. Only what earlier launches wrote can skip them.
        const ulonglong2 sl = *reinterpret_cast<const ulonglong2 *>(&A.slots[2 * h]);
        if (sl.x == key && sl.y < first) {
            A.claim[g] = NO_CLAIM;
            return;
        }
        unsigned long long prev = sl.x;
        if (prev == EMPTY_KEY) prev = atomicCAS(&A.slots[2 * h], EMPTY_KEY, key);
        if (prev == EMPTY_KEY || prev == key) {
            atomicMin(&A.slots[2 * h + 1], (unsigned long long)g);
            A.claim[g] = (unsigned)h;
            return;
        }
        h = (h + 1) & A.mask;
    }
    // (not reached: the table always has a free slot)
    A.claim[g] = NO_CLAIM;
}

// keep = this point is the first of its voxel: it claimed a slot and the
// slot's lowest order is its own. The workgroup adds its count.
__global__ __launch_bounds__(BLOCK) void k_fuse_mark(FuseArgs A)
{
    const long long HW = (long long)A.W * A.H, n = HW * A.n_maps;
    unsigned n_kept = 0;
    for (long long g = (long long)blockIdx.x * BLOCK + threadIdx.x; g < n; g += (long long)gridDim.x * BLOCK) {
        const unsigned h = A.claim[g];
        const bool kept = h != NO_CLAIM && A.slots[2 * (unsigned long long)h + 1] == (unsigned long long)g;
        A.keep[g] = kept ? 1 : 0;
        n_kept += kept ? 1 : 0;
    }
    block_count_add(A.spread, n_kept, 0);
}

__global__ __launch_bounds__(BLOCK) void k_cover_clear(FuseArgs A)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < (long long)A.Wc * A.Hc) A.cover[i] = 0;
    // (the grid has at least one workgroup of BLOCK >= 2 COUNT_SPREAD threads)
    if (i < 2 * COUNT_SPREAD) *count_slot(A.spread, (int)i / COUNT_SPREAD, (int)i % COUNT_SPREAD) = 0ULL;
}

// Marks the panorama pixel of point g (a kept point of the maps).
__device__ __forceinline__ void cover_point(const FuseArgs &A, long long g)
{
    const long long HW = (long long)A.W * A.H;
    const int m = (int)(g / HW);
    double X[3];
    if (!fuse_point(A, m, g - (long long)m * HW, X)) return;
    double Y[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) Y[k] = A.view.R[3 * k] * X[0] + A.view.R[3 * k + 1] * X[1] + A.view.R[3 * k + 2] * X[2] + A.view.t[k];
    if (!(Y[0] * Y[0] + Y[1] * Y[1] + Y[2] * Y[2] > 0.0)) return;
    int xi, yi;
    nearest_pixel(Y, A.Wc, A.Hc, xi, yi);
    A.cover[(long long)yi * A.Wc + xi] = 1;
}

// A wave takes COVER_SPAN consecutive points: it collects the indices of
// those with their keep byte set (or depth > 0 without keep bytes) in LDS,
// in order, and then projects them 64 at a time, so that the FP64
// projection runs on full waves although most points are not kept.
constexpr int COVER_SPAN = 256;

__global__ __launch_bounds__(BLOCK) void k_cover_mark(FuseArgs A)
{
    __shared__ long long list[BLOCK / 64][COVER_SPAN];
    const int lane = (int)(threadIdx.x & 63u), w = (int)(threadIdx.x >> 6);
    const long long HW = (long long)A.W * A.H, n = HW * A.n_maps;
    const long long base = ((long long)blockIdx.x * (BLOCK / 64) + w) * COVER_SPAN;
    int total = 0;
#pragma unroll
    for (int c = 0; c < COVER_SPAN / 64; ++c) {
        const long long g = base + c * 64 + lane;
        bool f = false;
        if (g < n) {
            if (A.keep_in) {
                f = A.keep_in[g] != 0;
            } else {
                const int m = (int)(g / HW);
                const long long i = g - (long long)m * HW;
                const int y = (int)(i / A.W), x = (int)(i - (long long)y * A.W);
                f = A.depth[m][(long long)y * A.pitch[m] + x] > 0.0f;
            }
        }
        const unsigned long long mask = __ballot(f);
        // rank of this lane among the flagged lanes below it
        const int r = __builtin_amdgcn_mbcnt_hi((unsigned)(mask >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)mask, 0u));
        if (f) list[w][total + r] = g;
        total += __popcll(mask);
    }
    // (a wave's LDS writes complete before its reads)
    __builtin_amdgcn_wave_barrier();
    for (int j = lane; j < total; j += 64) cover_point(A, list[w][j]);
}

__global__ __launch_bounds__(BLOCK) void k_cover_count(FuseArgs A)
{
    const long long n = (long long)A.Wc * A.Hc;
    unsigned c = 0;
    for (long long i = (long long)blockIdx.x * BLOCK + threadIdx.x; i < n; i += (long long)gridDim.x * BLOCK)
        c += A.cover[i] ? 1 : 0;
    block_count_add(A.spread, c, 0);
}

// Test hook: raw Philox blocks.
__global__ void k_philox(unsigned long long k0, unsigned long long k1, unsigned long long ctr0,
                         long long n, unsigned long long *out)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    unsigned long long c[4] = {ctr0 + (unsigned long long)i, 0ULL, 0ULL, 0ULL};
    philox4x64_10(k0, k1, c);
    out[4 * i + 0] = c[0];
    out[4 * i + 1] = c[1];
    out[4 * i + 2] = c[2];
    out[4 * i + 3] = c[3];
}

}  // namespace pms
