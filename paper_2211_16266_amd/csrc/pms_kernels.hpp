// pms_kernels.hpp -- gfx950 kernels of equirectangular PatchMatch-Stereo
// densification (Surmann et al., Sec. III-B/C). Included once, by pms.hip.
//
// Work decomposition
//   * One reference pixel is served by LPP (2 or 4) adjacent lanes of a
//     wave64 inside one DPP quad. Each lane owns every LPP-th patch sample:
//     its bearing, its centred reference value and, per view, its warped
//     neighbour value stay in VGPRs; patch sums are reduced inside the group
//     with quad_perm DPP adds, so the reduction order depends on the patch
//     only. LPP is chosen from the patch size alone.
//   * A workgroup of 256 threads covers a (32/LPP) x 8 tile of pixels of one
//     colour (red-black sweep) or of all pixels (init / cost evaluation); tiles are
//     handed out so that each XCD walks a contiguous band of rows and keeps
//     the matching part of the neighbour images in its own L2.
//   * Neighbour images are re-laid out once per call: every row is repeated
//     around the seam to width 2W + 4 (columns -W/2-2 .. 3W/2+1), and the
//     first and last rows are repeated once more above and below (the
//     clamped pole taps). Any warped sample then reads its two bilinear rows
//     as two 8-byte buffer loads at an offset built by one add and one clamp
//     per axis, with no seam or pole test; buffer loads carry the image size,
//     so no address can leave the image.
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
constexpr int MAXOFF = 16;    // propagation offsets
constexpr int MAXTRIAL = 16;  // refinement trials
constexpr int BLOCK = 256;    // threads per workgroup (4 waves)

// Occupancy target of the PatchMatch kernels (waves per SIMD): 4 for up to
// 9 samples per lane, where the compiler would otherwise settle for 3 waves
// to avoid a couple of spill slots outside the sample loop; the larger
// variants keep the compiler's choice.
#define PMS_OCCUPANCY(SPL) __attribute__((amdgpu_waves_per_eu((SPL) <= 9 ? 4 : 1, 8)))
// Re-laid-out neighbour image: H + 2 rows of 2W + 4 values;
// logical column x is stored at x + W/2 + 2, logical row y at y + 1.

// dtype codes of the C ABI
constexpr int DT_F32 = 0, DT_F16 = 1, DT_U8 = 2;

struct ViewPoseF {
    float R[9];
    float t[3];
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
    float k_float;
    float var_floor;
    float dmin, dmax, inv_dmin, inv_dmax;
    float kx, cx, ky, cy;  // u = lam * kx + cx, v = phi * ky + cy
    float patch_chord;     // bound on |b_q - b_p| over the patch
    int n_offsets;
    int off_x[MAXOFF], off_y[MAXOFF];
    int refine_trials;
    float sd[MAXTRIAL], sn[MAXTRIAL];
    unsigned long long seed;
    // tile shape: a wave covers (1 << wx_log2) x ((64 / LPP) >> wx_log2)
    // pixels, a workgroup (1 << bx_log2) x (4 >> bx_log2) waves
    int wx_log2, bx_log2;
    int tile_w, tile_h;      // tile size in pixels
    int tiles_x_all;         // tiles per tile row over all pixels
    int tiles_x_half;        // ... over the pixels of one colour
    int ref_dtype;
    ImgRef ref;
    ViewPoseD pose[MAXV];    // relative poses in FP64 (warped centre ray)
    ViewPoseF posef[MAXV];   // the same rounded (homography on offsets)
    const void *pad[MAXV];  // re-laid-out neighbours, (H + 2) x Wp elements
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
};

template <int DT>
struct Storage;
template <>
struct Storage<DT_F32> {
    using ref_t = float;
    using pad_t = float;
};
template <>
struct Storage<DT_F16> {
    using ref_t = __half;
    using pad_t = __half;
};
template <>
struct Storage<DT_U8> {
    using ref_t = uint8_t;
    using pad_t = float;  // 8-bit neighbours are widened (and scaled) once
};

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------

// Sum over the LPP lanes of a pixel: quad_perm [1,0,3,2], then (LPP = 4)
// [2,3,0,1]. Every lane of the group ends with the same bits
// ((a+b)+(c+d) == (b+a)+(d+c) exactly).
template <int LPP>
__device__ __forceinline__ float group_sum(float v)
{
    v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xB1, 0xF, 0xF, true));
    if (LPP == 4) v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x4E, 0xF, 0xF, true));
    return v;
}

template <int LPP>
__device__ __forceinline__ int group_and(int v)
{
    v &= __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, true);
    if (LPP == 4) v &= __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, true);
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

// Two horizontally adjacent values of a re-laid-out image at a byte offset.
template <typename P>
__device__ __forceinline__ float2 load_pair(__amdgpu_buffer_rsrc_t r, int byte_off);

template <>
__device__ __forceinline__ float2 load_pair<float>(__amdgpu_buffer_rsrc_t r, int byte_off)
{
    return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, byte_off, 0, 0));
}

template <>
__device__ __forceinline__ float2 load_pair<__half>(__amdgpu_buffer_rsrc_t r, int byte_off)
{
    const __half2 h = __builtin_bit_cast(__half2, __builtin_amdgcn_raw_buffer_load_b32(r, byte_off, 0, 0));
    return __half22float2(h);
}

__device__ __forceinline__ void bearing(const SweepArgs &A, int x, int y, float b[3])
{
    float2 rw = A.tab_row[y], cl = A.tab_col[x];
    b[0] = rw.y * cl.x;
    b[1] = -rw.x;
    b[2] = rw.y * cl.y;
}

// atan(t) for |t| <= tan(pi/8): t + t s P(s), s = t^2, with a degree-3 P
// fitted for minimum relative error (8e-8 in FP32; atan_coeffs.py). Odd in
// t bit for bit: round-to-nearest is symmetric.
constexpr float TAN_PI_8 = 0.41421356f;
// tan(pi/8) less a margin for the rounding of the range test itself
constexpr float SHORT_RANGE = 0.4141f;

__device__ __forceinline__ float atan_core(float t)
{
    const float s = t * t;
    float p = fmaf(s, 8.053722978e-02f, -1.387767941e-01f);
    p = fmaf(p, s, 1.997770965e-01f);
    p = fmaf(p, s, -3.333294988e-01f);
    return fmaf(t * s, p, t);
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

// Aggregated cost of plane (d, n) at the pixel of `pt`: per view, warp every
// sample, bilinear-sample the neighbour, two-pass NCC, cost = 1 - NCC or 2
// when invalid; then the mean of the top_k smallest view costs. All lanes of
// the pixel return the same value. FULL: every lane owns SPL samples (P is
// a multiple of LPP), so no slot is masked. When VIEWS is set, the pixel's
// first lane writes each view's cost to A.view_out[j][out_index].
//
// `bound`: the caller only uses the result if it is below `bound`. Once the
// views still to come are fewer than top_k, the aggregate is at least the
// same ascending sum with those views at cost 0; when that is already
// >= bound the remaining views are skipped and a value >= bound returned.
// Float addition and division round monotonically, so every decision the
// caller takes is the one the full evaluation gives.
template <typename PT, int LPP, int SPL, bool FULL, bool VIEWS>
__device__ __forceinline__ float evaluate(const SweepArgs &A, const Patch<SPL> &pt, float d,
                                          float n0, float n1, float n2, int lane,
                                          long long out_index, float bound = 3.0f)
{
    const double n64[3] = {(double)n0, (double)n1, (double)n2};
    const double nbp = n64[0] * pt.bp64[0] + n64[1] * pt.bp64[1] + n64[2] * pt.bp64[2];
    const double c64 = (double)d * nbp;
    const float nbpf = (float)nbp;
    int ok = c64 < 0.0;
#pragma unroll
    for (int i = 0; i < SPL; ++i) {
        // n . b_q = n . b_p + n . (b_q - b_p)
        const float den = fmaf(n0, pt.b[i][0], fmaf(n1, pt.b[i][1], fmaf(n2, pt.b[i][2], nbpf)));
        ok &= FULL ? (den < 0.0f) : (den < 0.0f || pt.wt[i] == 0.0f);
    }
    ok = group_and<LPP>(ok);
    if (!ok) {
        if (VIEWS && lane == 0)
            for (int j = 0; j < A.n_views; ++j) A.view_out[j][out_index] = 2.0f;
        return 2.0f;
    }
    const double mc = -c64;
    const int rowb = A.Wp * (int)sizeof(PT);
    // the top_k smallest view costs, ascending, as bit patterns: costs are
    // non-negative floats, whose order is that of their bits as unsigned
    unsigned top[MAXV];
#pragma unroll
    for (int i = 0; i < MAXV; ++i) top[i] = 0x40400000u;  // 3.0f

    for (int j = 0; j < A.n_views; ++j) {
        const ViewPoseD &V = A.pose[j];
        const ViewPoseF &Vf = A.posef[j];
        const __amdgpu_buffer_rsrc_t img = make_rsrc(A.pad[j], A.pad_bytes);
        // warped centre ray in FP64: M b_p = (-c) R b_p - t (n . b_p), where
        // M = (-c) R - t n^T is a positive multiple of the plane homography
        double yc[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const double rb = fma(V.R[3 * a], pt.bp64[0], fma(V.R[3 * a + 1], pt.bp64[1], V.R[3 * a + 2] * pt.bp64[2]));
            yc[a] = fma(mc, rb, -V.t[a] * nbp);
        }
        // anchor: the pixel nearest to the warped centre
        const float lamc = atan2_full((float)yc[0], (float)yc[2]);
        const float phic = atan2_full((float)-yc[1], __builtin_amdgcn_sqrtf((float)(yc[0] * yc[0] + yc[2] * yc[2])));
        int U0 = (int)floorf(fmaf(lamc, A.kx, A.cx) + 0.5f);
        U0 = U0 >= A.W ? U0 - A.W : (U0 < 0 ? U0 + A.W : U0);
        int V0 = (int)floorf(fmaf(phic, A.ky, A.cy) + 0.5f);
        V0 = V0 < 0 ? 0 : (V0 > A.H - 1 ? A.H - 1 : V0);
        const double2 lam0 = A.tab_col64[U0];  // (sin, cos) of the anchor longitude
        const double2 phi0 = A.tab_row64[V0];  // (sin, cos) of the anchor latitude
        const int U0p = U0 + (A.W >> 1) + 2;   // anchor in re-laid-out storage
        const int V0p = V0 + 1;
        // centre turned about the vertical by -lam0 (FP64). Its longitude is
        // within half a pixel of lam0, so yr2 > 0 and |yr0| << yr2, and the
        // horizontal length is yr2 + yr0^2 / (2 yr2) to FP64 precision.
        const double yr0 = fma(lam0.y, yc[0], -lam0.x * yc[2]);
        const double yr2 = fma(lam0.x, yc[0], lam0.y * yc[2]);
        const float y0c = (float)yr0, y2c = (float)yr2;
        const double hzc = yr2 + (double)(0.5f * y0c * y0c / y2c);
        // centre: sin and cos of (latitude - phi0), scaled by the ray length
        const float sdc = (float)fma(-yc[1], phi0.y, -hzc * phi0.x);
        const float cdc = (float)fma(hzc, phi0.y, -yc[1] * phi0.x);
        const float hzcf = (float)hzc;
        const float sp0 = (float)phi0.x, cp0 = (float)phi0.y;
        const float sl0 = (float)lam0.x, cl0 = (float)lam0.y;
        // the homography turned by -lam0, in FP32: it only maps the small
        // offsets of the sample bearings from the centre bearing
        const float mcf = (float)mc;
        float h[9];
        float mf2 = 0.0f;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const float m0 = fmaf(mcf, Vf.R[k], -Vf.t[0] * (k == 0 ? n0 : k == 1 ? n1 : n2));
            const float m1 = fmaf(mcf, Vf.R[3 + k], -Vf.t[1] * (k == 0 ? n0 : k == 1 ? n1 : n2));
            const float m2 = fmaf(mcf, Vf.R[6 + k], -Vf.t[2] * (k == 0 ? n0 : k == 1 ? n1 : n2));
            h[k] = fmaf(cl0, m0, -sl0 * m2);
            h[3 + k] = m1;
            h[6 + k] = fmaf(sl0, m0, cl0 * m2);
            mf2 = fmaf(m0, m0, fmaf(m1, m1, fmaf(m2, m2, mf2)));
        }
        float s[SPL];
        float sum = 0.0f;
        // Every sample offset e = h (b_q - b_p) satisfies |e| <= |M|_F dmax
        // (turning keeps the norm). If the centre and that bound keep both
        // angles of every sample in the short form's range, the wave takes
        // the short form, which then equals the general one bit for bit.
        const float E = __builtin_amdgcn_sqrtf(mf2) * A.patch_chord;
        const float lon_den = y2c - E, lat_den = cdc - E;
        const bool short_ok = lon_den > 1e-30f && fabsf(y0c) + E <= SHORT_RANGE * lon_den &&
                              lat_den > 1e-30f && fabsf(sdc) + E <= SHORT_RANGE * lat_den;
        // (compiled in for up to 9 samples per lane only: the larger variants
        // cannot hold both copies at their occupancy)
        if (SPL <= 9 && __all(short_ok)) {
    #pragma unroll
            for (int i = 0; i < SPL; ++i) {
                const float bx = pt.b[i][0], by = pt.b[i][1], bz = pt.b[i][2];
                // the turned homography on the offset from the centre bearing
                const float e0 = fmaf(h[0], bx, fmaf(h[1], by, h[2] * bz));
                const float e1 = fmaf(h[3], bx, fmaf(h[4], by, h[5] * bz));
                const float e2 = fmaf(h[6], bx, fmaf(h[7], by, h[8] * bz));
                const float y0 = y0c + e0, y2 = y2c + e2;
                const float hz = __builtin_amdgcn_sqrtf(fmaf(y0, y0, y2 * y2));
                // hz - hzc without cancellation
                const float dhz = fmaf(e0, y0 + y0c, e2 * (y2 + y2c)) * __builtin_amdgcn_rcpf(hz + hzcf);
                const float sd = fmaf(-dhz, sp0, fmaf(-e1, cp0, sdc));
                const float cd = fmaf(dhz, cp0, fmaf(-e1, sp0, cdc));
                // longitude - lam0 and latitude - phi0
                const float dl = atan_core(y0 * __builtin_amdgcn_rcpf(y2));
                const float dp = atan_core(sd * __builtin_amdgcn_rcpf(cd));
                const float ul = dl * A.kx, vl = dp * A.ky;
                const float fu = floorf(ul), fv = floorf(vl);
                const float au = ul - fu, av = vl - fv;
                // |ul| <= W/2 keeps the column inside the repeated storage; the
                // latitude stays within the poles, so this clamp only guards
                // against rounding
                const int xi = U0p + (int)fu;
                const int yi = min(max(V0p + (int)fv, 0), A.H);
                const int off = (int)(__umul24((unsigned)yi, (unsigned)A.Wp) + (unsigned)xi) * (int)sizeof(PT);
                const float2 p0 = load_pair<PT>(img, off);
                const float2 p1 = load_pair<PT>(img, off + rowb);
                const float top_r = fmaf(au, p0.y - p0.x, p0.x);
                const float bot_r = fmaf(au, p1.y - p1.x, p1.x);
                s[i] = fmaf(av, bot_r - top_r, top_r);
                sum += FULL ? s[i] : s[i] * pt.wt[i];
            }
        } else {
    #pragma unroll
            for (int i = 0; i < SPL; ++i) {
                const float bx = pt.b[i][0], by = pt.b[i][1], bz = pt.b[i][2];
                // the turned homography on the offset from the centre bearing
                const float e0 = fmaf(h[0], bx, fmaf(h[1], by, h[2] * bz));
                const float e1 = fmaf(h[3], bx, fmaf(h[4], by, h[5] * bz));
                const float e2 = fmaf(h[6], bx, fmaf(h[7], by, h[8] * bz));
                const float y0 = y0c + e0, y2 = y2c + e2;
                const float hz = __builtin_amdgcn_sqrtf(fmaf(y0, y0, y2 * y2));
                // hz - hzc without cancellation
                const float dhz = fmaf(e0, y0 + y0c, e2 * (y2 + y2c)) * __builtin_amdgcn_rcpf(hz + hzcf);
                const float sd = fmaf(-dhz, sp0, fmaf(-e1, cp0, sdc));
                const float cd = fmaf(dhz, cp0, fmaf(-e1, sp0, cdc));
                // longitude - lam0 and latitude - phi0
                const float dl = atan2_full(y0, y2);
                const float dp = atan2_full(sd, cd);
                const float ul = dl * A.kx, vl = dp * A.ky;
                const float fu = floorf(ul), fv = floorf(vl);
                const float au = ul - fu, av = vl - fv;
                // |ul| <= W/2 keeps the column inside the repeated storage; the
                // latitude stays within the poles, so this clamp only guards
                // against rounding
                const int xi = U0p + (int)fu;
                const int yi = min(max(V0p + (int)fv, 0), A.H);
                const int off = (int)(__umul24((unsigned)yi, (unsigned)A.Wp) + (unsigned)xi) * (int)sizeof(PT);
                const float2 p0 = load_pair<PT>(img, off);
                const float2 p1 = load_pair<PT>(img, off + rowb);
                const float top_r = fmaf(au, p0.y - p0.x, p0.x);
                const float bot_r = fmaf(au, p1.y - p1.x, p1.x);
                s[i] = fmaf(av, bot_r - top_r, top_r);
                sum += FULL ? s[i] : s[i] * pt.wt[i];
            }
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
        if (pt.var_r < A.var_floor || vs < A.var_floor) {
            cj = 2.0f;
        } else {
            float ncc = cov * __builtin_amdgcn_rsqf(pt.var_r * vs);
            ncc = fminf(fmaxf(ncc, -1.0f), 1.0f);
            cj = 1.0f - ncc;
        }
        if (VIEWS && lane == 0) A.view_out[j][out_index] = cj;
        unsigned cb = __float_as_uint(cj);
#pragma unroll
        for (int i = 0; i < MAXV; ++i)
            if (i < A.top_k) {
                const unsigned lo = min(top[i], cb), hi = max(top[i], cb);
                top[i] = lo;
                cb = hi;
            }
        if (!VIEWS) {
            const int have = A.top_k - (A.n_views - 1 - j);  // evaluated costs in the bound
            if (have > 0) {
                float lb = 0.0f;
#pragma unroll
                for (int i = 0; i < MAXV; ++i)
                    if (i < have) lb += __uint_as_float(top[i]);
                if (lb / A.k_float >= bound) return lb / A.k_float;
            }
        }
    }
    float acc = 0.0f;
#pragma unroll
    for (int i = 0; i < MAXV; ++i)
        if (i < A.top_k) acc += __uint_as_float(top[i]);
    return acc / A.k_float;
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

// A launch covers a list of entries; entry e owns the logical blocks
// [first_e, first_{e+1}) (the list ends with a sentinel holding the total)
// and names its job and, for a half-sweep, the job's iteration and colour.
// Jobs at different stages of their sweep can share one launch.
struct Entry {
    int job, first, iteration, colour;
};

struct Launch {
    const void *table;      // JobArgs[] or PadJob[]
    const Entry *entries;   // n_entries + 1 entries
    int n_entries;
    int per_xcd;            // logical blocks per XCD; the grid is 8 * per_xcd
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

// Logical block of this workgroup: the 8 XCDs receive workgroups round
// robin, and logical block t = xcd * per_xcd + slot gives each XCD a
// contiguous run of tiles (rows of one job), whose neighbour image rows then
// stay in that XCD's L2. Returns false past the last entry.
__device__ __forceinline__ bool block_entry(const Launch &L, int &e, int &local)
{
    const int bid = blockIdx.x;
    const int t = (bid & 7) * L.per_xcd + (bid >> 3);
    const Entry *E = const_view<Entry>(L.entries, 0);
    if (t >= E[L.n_entries].first) return false;
    int lo = 0, hi = L.n_entries - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (E[mid].first <= t) lo = mid;
        else hi = mid - 1;
    }
    e = lo;
    local = t - E[lo].first;
    return true;
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

// Re-lays out neighbour images: storage row py holds image row
// clamp(py - 1, 0, H - 1), storage column px holds image column
// (px - W/2 - 2) mod W. 16-bit images keep their values; the others are
// widened to FP32 (8-bit ones scaled to [0, 1]).
template <typename TS, typename TD>
__device__ __forceinline__ void pad_one(const PadJob &J, long long i)
{
    const int py = (int)(i / J.Wp), px = (int)(i - (long long)py * J.Wp);
    int sx = px - (J.W >> 1) - 2;
    sx = sx < 0 ? sx + J.W : sx;
    sx = sx >= J.W ? sx - J.W : sx;
    const int sy = py == 0 ? 0 : (py > J.H ? J.H - 1 : py - 1);
    if constexpr (std::is_same<TS, __half>::value)
        static_cast<__half *>(J.dst)[i] =
            reinterpret_cast<const __half *>(static_cast<const char *>(J.src.ptr) + (long long)sy * J.src.pitch)[sx];
    else
        static_cast<float *>(J.dst)[i] = load_px<TS>(J.src, sx, sy);
}

__global__ __launch_bounds__(BLOCK) void k_pad(Launch L)
{
    int e, local;
    if (!block_entry(L, e, local)) return;
    const Entry &E = *const_view<Entry>(L.entries, e);
    const PadJob &J = *const_view<PadJob>(L.table, E.job);
    const long long i = (long long)local * BLOCK + threadIdx.x;
    if (i >= (long long)(J.H + 2) * J.Wp) return;
    if (J.dtype == DT_F16) pad_one<__half, __half>(J, i);
    else if (J.dtype == DT_U8) pad_one<uint8_t, float>(J, i);
    else pad_one<float, float>(J, i);
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

// Random initialisation (Sec. III-B): depth uniform in inverse depth, normal
// uniform on the sphere turned towards the camera, and its cost.
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
    float u[4];
    uniforms(A.seed, (unsigned long long)idx, 0ULL, 0ULL, u);
    const float rho = fmaf(u[0], A.inv_dmin - A.inv_dmax, A.inv_dmax);
    const float d = 1.0f / rho;
    const float z = 2.0f * u[1] - 1.0f, a = 6.283185307179586f * u[2];
    const float s = sqrtf(fmaxf(0.0f, 1.0f - z * z));
    float sa, ca;
    sincosf(a, &sa, &ca);
    float n0 = s * ca, n1 = s * sa, n2 = z;
    const float nb = n0 * pt.bp[0] + n1 * pt.bp[1] + n2 * pt.bp[2];
    if (nb > 0.0f) {
        n0 = -n0;
        n1 = -n1;
        n2 = -n2;
    } else if (nb == 0.0f) {
        n0 = -pt.bp[0];
        n1 = -pt.bp[1];
        n2 = -pt.bp[2];
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
template <int DT, int LPP, int SPL, bool FULL>
__device__ __forceinline__ void halfsweep_tile(const SweepArgs &A, int tile, int iteration, int colour)
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
    const long long idx = (long long)y * A.W + x;

    Patch<SPL> pt;
    patch_setup<TR, LPP, SPL>(A, x, y, lane, pt);
    const float4 cur = A.state[idx];
    float bd = cur.w, bn0 = cur.x, bn1 = cur.y, bn2 = cur.z;
    float bc = A.cost[idx];

    for (int o = 0; o < A.n_offsets; ++o) {
        int qx = x + A.off_x[o];
        qx = qx < 0 ? qx + A.W : (qx >= A.W ? qx - A.W : qx);
        const int qy = y + A.off_y[o];
        if (qy < A.r || qy > A.H - 1 - A.r) continue;
        const float4 sq = A.state[(long long)qy * A.W + qx];
        if (!(sq.w > 0.0f)) continue;
        float bq[3];
        bearing(A, qx, qy, bq);
        const float cq = sq.w * (sq.x * bq[0] + sq.y * bq[1] + sq.z * bq[2]);
        const float den = sq.x * pt.bp[0] + sq.y * pt.bp[1] + sq.z * pt.bp[2];
        if (!(den < 0.0f)) continue;
        const float dd = cq / den;
        if (!(dd >= A.dmin && dd <= A.dmax)) continue;
        const float c = evaluate<PT, LPP, SPL, FULL, false>(A, pt, dd, sq.x, sq.y, sq.z, lane, 0, bc);
        if (c < bc) {
            bc = c;
            bd = dd;
            bn0 = sq.x;
            bn1 = sq.y;
            bn2 = sq.z;
        }
    }

    for (int t = 0; t < A.refine_trials; ++t) {
        float u[4];
        uniforms(A.seed, (unsigned long long)idx, (unsigned long long)iteration,
                 (unsigned long long)(16 + t), u);
        float dd = bd * expf((2.0f * u[0] - 1.0f) * A.sd[t]);
        dd = fminf(fmaxf(dd, A.dmin), A.dmax);
        float m0 = fmaf(A.sn[t], 2.0f * u[1] - 1.0f, bn0);
        float m1 = fmaf(A.sn[t], 2.0f * u[2] - 1.0f, bn1);
        float m2 = fmaf(A.sn[t], 2.0f * u[3] - 1.0f, bn2);
        const float len = sqrtf(m0 * m0 + m1 * m1 + m2 * m2);
        if (!(len > 0.0f)) continue;
        m0 /= len;
        m1 /= len;
        m2 /= len;
        if (!(m0 * pt.bp[0] + m1 * pt.bp[1] + m2 * pt.bp[2] < 0.0f)) continue;
        const float c = evaluate<PT, LPP, SPL, FULL, false>(A, pt, dd, m0, m1, m2, lane, 0, bc);
        if (c < bc) {
            bc = c;
            bd = dd;
            bn0 = m0;
            bn1 = m1;
            bn2 = m2;
        }
    }
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
__global__ __launch_bounds__(BLOCK) PMS_OCCUPANCY(SPL) void k_tiles(Launch L)
{
    int e, local;
    if (!block_entry(L, e, local)) return;
    const Entry &E = *const_view<Entry>(L.entries, e);
    const SweepArgs &A = const_view<JobArgs>(L.table, E.job)->s;
    if (KIND == TK_INIT) init_tile<DT, LPP, SPL, FULL>(A, local);
    else if (KIND == TK_HALFSWEEP) halfsweep_tile<DT, LPP, SPL, FULL>(A, local, E.iteration, E.colour);
    else eval_tile<DT, LPP, SPL, FULL>(A, local);
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
