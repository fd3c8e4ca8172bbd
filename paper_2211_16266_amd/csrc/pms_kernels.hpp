// pms_kernels.hpp -- gfx950 kernels of equirectangular PatchMatch-Stereo
// densification (Surmann et al., Sec. III-B/C). Included once, by pms.hip.
//
// Work decomposition
//   * One reference pixel is served by LPP = 4 adjacent lanes of a wave64
//     (one DPP quad). Each lane owns every 4th patch sample: its bearing,
//     its centred reference value and, per view, its warped neighbour value
//     stay in VGPRs; patch sums are reduced inside the quad with two DPP
//     quad_perm adds, so the reduction order depends on the patch only.
//   * A workgroup of 256 threads covers an 8x8 tile of pixels of one colour
//     (red-black sweep) or of all pixels (init / cost evaluation); tiles are
//     handed out so that each XCD walks a contiguous band of rows and keeps
//     the matching part of the neighbour images in its own L2.
//   * Everything is FP32 except the bearing tables, which are computed in
//     FP64 once per image size and rounded.
//
// The warp of a sample is written in homography form: with the plane
// {X : n.X = c}, c = d (n.b_p) < 0, the neighbour ray of sample bearing b_q is
// proportional to H b_q, H = R + t n^T / c, with a positive factor whenever
// the plane lies in front of the sample ray (n.b_q < 0), so the projected
// pixel equals that of R X_q + t with X_q = (c / n.b_q) b_q.
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pms {

constexpr int LPP = 4;        // lanes per pixel (one DPP quad)
constexpr int MAXV = 8;       // neighbour views per launch
constexpr int MAXOFF = 16;    // propagation offsets
constexpr int MAXTRIAL = 16;  // refinement trials
constexpr int TILE = 8;       // 8x8 pixel tile per 256-thread workgroup
constexpr int BLOCK = 256;

struct ViewPoseF {
    float R[9];
    float t[3];
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
    int n_offsets;
    int off_x[MAXOFF], off_y[MAXOFF];
    int refine_trials;
    float sd[MAXTRIAL], sn[MAXTRIAL];
    unsigned long long seed;
    int iteration, colour;
    int tiles_x, tiles_y, tiles_per_xcd;
    ImgRef ref;
    ImgRef nbr[MAXV];
    ViewPoseF pose[MAXV];
    const float2 *tab_row;  // per row (sin phi, cos phi)
    const float2 *tab_col;  // per column (sin lam, cos lam)
    const float2 *stats;    // per pixel (mean, variance) of the reference patch
    float4 *state;          // per pixel (nx, ny, nz, depth)
    float *cost;            // per pixel aggregated cost
    // caller planes (eval: inputs/outputs; halfsweep io packing)
    const float *in_depth;
    const float *in_n0, *in_n1, *in_n2;
    long long in_pitch;
    float *out_cost;
    long long out_pitch;
    float *view_out[MAXV];
};

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------

__device__ __forceinline__ float quad_sum(float v)
{
    // quad_perm [1,0,3,2] then [2,3,0,1]: every lane of the quad ends with the
    // same bits ((a+b)+(c+d) == (b+a)+(d+c) exactly)
    v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xB1, 0xF, 0xF, true));
    v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x4E, 0xF, 0xF, true));
    return v;
}

__device__ __forceinline__ int quad_and(int v)
{
    v &= __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, true);
    v &= __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, true);
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

// Bilinear sample; longitude wraps around the seam, latitude taps clamp to
// the first/last row. Coordinates are clamped to the image first, which also
// maps NaN to the border, so every tap is in bounds.
template <typename T>
__device__ __forceinline__ float bilinear(const ImgRef &im, int W, int H, float u, float v)
{
    u = fminf(fmaxf(u, -0.5f), (float)W - 0.5f);
    v = fminf(fmaxf(v, -0.5f), (float)H - 0.5f);
    float fu = floorf(u), fv = floorf(v);
    float au = u - fu, av = v - fv;
    int x0 = (int)fu, y0 = (int)fv;
    int x1 = x0 + 1, y1 = y0 + 1;
    x0 = x0 < 0 ? W - 1 : x0;
    x1 = x1 >= W ? 0 : x1;
    y0 = y0 < 0 ? 0 : y0;
    y1 = y1 > H - 1 ? H - 1 : y1;
    float p00 = load_px<T>(im, x0, y0), p01 = load_px<T>(im, x1, y0);
    float p10 = load_px<T>(im, x0, y1), p11 = load_px<T>(im, x1, y1);
    float top = fmaf(au, p01 - p00, p00);
    float bot = fmaf(au, p11 - p10, p10);
    return fmaf(av, bot - top, top);
}

__device__ __forceinline__ void bearing(const SweepArgs &A, int x, int y, float b[3])
{
    float2 rw = A.tab_row[y], cl = A.tab_col[x];
    b[0] = rw.y * cl.x;
    b[1] = -rw.x;
    b[2] = rw.y * cl.y;
}

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
    float b[SPL][3];  // sample bearings
    float rc[SPL];    // reference samples minus the patch mean
    int nmine;        // samples owned by this lane (<= SPL)
    float bp[3];      // bearing of the pixel itself
    float var_r;      // reference patch variance
};

template <typename T, int SPL>
__device__ __forceinline__ void patch_setup(const SweepArgs &A, int x, int y, int lane,
                                            Patch<SPL> &pt)
{
    bearing(A, x, y, pt.bp);
    float2 st = A.stats[(long long)y * A.W + x];
    pt.var_r = st.y;
    pt.nmine = (A.P - lane + LPP - 1) / LPP;
#pragma unroll
    for (int i = 0; i < SPL; ++i) {
        int q = lane + LPP * i;
        if (q < A.P) {
            int row = q / A.side;
            int col = q - row * A.side;
            int xq = x - A.r + col * A.stride;
            xq = xq < 0 ? xq + A.W : (xq >= A.W ? xq - A.W : xq);
            int yq = y - A.r + row * A.stride;
            bearing(A, xq, yq, pt.b[i]);
            pt.rc[i] = load_px<T>(A.ref, xq, yq) - st.x;
        } else {
            pt.b[i][0] = pt.bp[0];
            pt.b[i][1] = pt.bp[1];
            pt.b[i][2] = pt.bp[2];
            pt.rc[i] = 0.0f;
        }
    }
}

// Aggregated cost of plane (d, n) at the pixel of `pt`: per view, warp every
// sample, bilinear-sample the neighbour, two-pass NCC, cost = 1 - NCC or 2
// when invalid; then the mean of the top_k smallest view costs. All 4 lanes
// of the quad return the same value. When VIEWS is set, lane 0 of the quad
// writes each view's cost to A.view_out[j][out_index].
template <typename T, int SPL, bool VIEWS>
__device__ __forceinline__ float evaluate(const SweepArgs &A, const Patch<SPL> &pt, float d,
                                          float n0, float n1, float n2, int lane,
                                          long long out_index)
{
    float c = d * (n0 * pt.bp[0] + n1 * pt.bp[1] + n2 * pt.bp[2]);
    int ok = c < 0.0f;
#pragma unroll
    for (int i = 0; i < SPL; ++i)
        if (i < pt.nmine) ok &= (n0 * pt.b[i][0] + n1 * pt.b[i][1] + n2 * pt.b[i][2]) < 0.0f;
    ok = quad_and(ok);
    if (!ok) {
        if (VIEWS && lane == 0)
            for (int j = 0; j < A.n_views; ++j) A.view_out[j][out_index] = 2.0f;
        return 2.0f;
    }
    const float ic = 1.0f / c;
    float top[MAXV];
#pragma unroll
    for (int i = 0; i < MAXV; ++i) top[i] = 3.0f;

    for (int j = 0; j < A.n_views; ++j) {
        const ViewPoseF &V = A.pose[j];
        const float t0 = V.t[0] * ic, t1 = V.t[1] * ic, t2 = V.t[2] * ic;
        const float h00 = fmaf(t0, n0, V.R[0]), h01 = fmaf(t0, n1, V.R[1]), h02 = fmaf(t0, n2, V.R[2]);
        const float h10 = fmaf(t1, n0, V.R[3]), h11 = fmaf(t1, n1, V.R[4]), h12 = fmaf(t1, n2, V.R[5]);
        const float h20 = fmaf(t2, n0, V.R[6]), h21 = fmaf(t2, n1, V.R[7]), h22 = fmaf(t2, n2, V.R[8]);
        float s[SPL];
        float sum = 0.0f;
#pragma unroll
        for (int i = 0; i < SPL; ++i) {
            s[i] = 0.0f;
            if (i < pt.nmine) {
                const float bx = pt.b[i][0], by = pt.b[i][1], bz = pt.b[i][2];
                const float y0 = fmaf(h00, bx, fmaf(h01, by, h02 * bz));
                const float y1 = fmaf(h10, bx, fmaf(h11, by, h12 * bz));
                const float y2 = fmaf(h20, bx, fmaf(h21, by, h22 * bz));
                const float lam = atan2f(y0, y2);
                const float hz = __builtin_sqrtf(fmaf(y0, y0, y2 * y2));
                const float phi = atan2f(-y1, hz);
                const float u = fmaf(lam, A.kx, A.cx);
                const float v = fmaf(phi, A.ky, A.cy);
                s[i] = bilinear<T>(A.nbr[j], A.W, A.H, u, v);
                sum += s[i];
            }
        }
        sum = quad_sum(sum);
        const float ms = sum * A.inv_P;
        float m2 = 0.0f, cv = 0.0f;
#pragma unroll
        for (int i = 0; i < SPL; ++i)
            if (i < pt.nmine) {
                const float e = s[i] - ms;
                m2 = fmaf(e, e, m2);
                cv = fmaf(pt.rc[i], e, cv);
            }
        m2 = quad_sum(m2);
        cv = quad_sum(cv);
        const float vs = m2 * A.inv_P, cov = cv * A.inv_P;
        float cj;
        if (pt.var_r < A.var_floor || vs < A.var_floor) {
            cj = 2.0f;
        } else {
            float ncc = cov / sqrtf(pt.var_r * vs);
            ncc = fminf(fmaxf(ncc, -1.0f), 1.0f);
            cj = 1.0f - ncc;
        }
        if (VIEWS && lane == 0) A.view_out[j][out_index] = cj;
        // insert into the ascending list of the smallest costs
#pragma unroll
        for (int i = 0; i < MAXV; ++i) {
            const float lo = fminf(top[i], cj), hi = fmaxf(top[i], cj);
            top[i] = lo;
            cj = hi;
        }
    }
    float acc = 0.0f;
#pragma unroll
    for (int i = 0; i < MAXV; ++i)
        if (i < A.top_k) acc += top[i];
    return acc / A.k_float;
}

// Tile scheduling: logical tile t = xcd * tiles_per_xcd + slot, so that the
// consecutive workgroups one XCD receives cover a contiguous band of tiles.
__device__ __forceinline__ bool tile_of_block(const SweepArgs &A, int &tx, int &ty)
{
    const int bid = blockIdx.x;
    const int t = (bid & 7) * A.tiles_per_xcd + (bid >> 3);
    if (t >= A.tiles_x * A.tiles_y) return false;
    ty = t / A.tiles_x;
    tx = t - ty * A.tiles_x;
    return true;
}

// Position of this thread's pixel inside an 8x8 tile: 4 waves of 4x4 pixels.
__device__ __forceinline__ void tile_pixel(int tid, int &dx, int &dy, int &lane)
{
    lane = tid & (LPP - 1);
    const int pix = tid >> 2;
    const int wave = pix >> 4;
    dx = ((wave & 1) << 2) + (pix & 3);
    dy = ((wave >> 1) << 2) + ((pix >> 2) & 3);
}

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------

// Bearing tables in FP64, rounded once.
__global__ void k_tables(int W, int H, float2 *row, float2 *col)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const double PI = 3.14159265358979323846;
    if (i < H) {
        double phi = PI / 2.0 - PI * (i + 0.5) / H;
        row[i] = make_float2((float)sin(phi), (float)cos(phi));
    }
    if (i < W) {
        double lam = 2.0 * PI * (i + 0.5) / W - PI;
        col[i] = make_float2((float)sin(lam), (float)cos(lam));
    }
}

// Reference patch mean and variance per valid pixel (two-pass, FP32).
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_refstats(SweepArgs A)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long long)A.W * A.H) return;
    const int y = (int)(i / A.W), x = (int)(i - (long long)y * A.W);
    float2 out = make_float2(0.0f, 0.0f);
    if (y >= A.r && y <= A.H - 1 - A.r) {
        float sum = 0.0f;
        for (int q = 0; q < A.P; ++q) {
            int row = q / A.side, col = q - row * A.side;
            int xq = x - A.r + col * A.stride;
            xq = xq < 0 ? xq + A.W : (xq >= A.W ? xq - A.W : xq);
            sum += load_px<T>(A.ref, xq, y - A.r + row * A.stride);
        }
        const float m = sum * A.inv_P;
        float v = 0.0f;
        for (int q = 0; q < A.P; ++q) {
            int row = q / A.side, col = q - row * A.side;
            int xq = x - A.r + col * A.stride;
            xq = xq < 0 ? xq + A.W : (xq >= A.W ? xq - A.W : xq);
            const float e = load_px<T>(A.ref, xq, y - A.r + row * A.stride) - m;
            v = fmaf(e, e, v);
        }
        out = make_float2(m, v * A.inv_P);
    }
    const_cast<float2 *>(A.stats)[i] = out;
}

// Random initialisation (Sec. III-B): depth uniform in inverse depth, normal
// uniform on the sphere turned towards the camera, and its cost.
template <typename T, int SPL>
__global__ __launch_bounds__(BLOCK) void k_init(SweepArgs A)
{
    int tx, ty, dx, dy, lane;
    if (!tile_of_block(A, tx, ty)) return;
    tile_pixel(threadIdx.x, dx, dy, lane);
    const int x = tx * TILE + dx, y = ty * TILE + dy;
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
    patch_setup<T, SPL>(A, x, y, lane, pt);
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
    const float c = evaluate<T, SPL, false>(A, pt, d, n0, n1, n2, lane, 0);
    if (lane == 0) {
        A.state[idx] = make_float4(n0, n1, n2, d);
        A.cost[idx] = c;
    }
}

// One half-sweep (Sec. III-C): propagation from the opposite-colour
// neighbourhood, then random refinement; strictly cheaper candidates win, the
// first in table order on ties. Pixels of the other colour are only read.
template <typename T, int SPL>
__global__ __launch_bounds__(BLOCK) void k_halfsweep(SweepArgs A)
{
    int tx, ty, dx, dy, lane;
    if (!tile_of_block(A, tx, ty)) return;
    tile_pixel(threadIdx.x, dx, dy, lane);
    const int k = tx * TILE + dx;
    const int y = A.r + ty * TILE + dy;
    if (k >= (A.W >> 1) || y > A.H - 1 - A.r) return;
    const int x = 2 * k + ((y + A.colour) & 1);
    const long long idx = (long long)y * A.W + x;

    Patch<SPL> pt;
    patch_setup<T, SPL>(A, x, y, lane, pt);
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
        const float c = evaluate<T, SPL, false>(A, pt, dd, sq.x, sq.y, sq.z, lane, 0);
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
        uniforms(A.seed, (unsigned long long)idx, (unsigned long long)A.iteration,
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
        const float c = evaluate<T, SPL, false>(A, pt, dd, m0, m1, m2, lane, 0);
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
template <typename T, int SPL>
__global__ __launch_bounds__(BLOCK) void k_eval(SweepArgs A)
{
    int tx, ty, dx, dy, lane;
    if (!tile_of_block(A, tx, ty)) return;
    tile_pixel(threadIdx.x, dx, dy, lane);
    const int x = tx * TILE + dx, y = ty * TILE + dy;
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
    patch_setup<T, SPL>(A, x, y, lane, pt);
    float c;
    if (A.view_out[0])
        c = evaluate<T, SPL, true>(A, pt, d, A.in_n0[pin], A.in_n1[pin], A.in_n2[pin], lane, pout);
    else
        c = evaluate<T, SPL, false>(A, pt, d, A.in_n0[pin], A.in_n1[pin], A.in_n2[pin], lane, pout);
    if (lane == 0) A.out_cost[pout] = c;
}

// Plane state <-> caller planes.
struct IoArgs {
    int W, H, r;
    float4 *state;
    float *cost;
    float *depth, *n0, *n1, *n2, *cplane;
    long long pd, pn0, pn1, pn2, pc;  // pitches in elements
};

__global__ __launch_bounds__(BLOCK) void k_finalize(IoArgs A)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long long)A.W * A.H) return;
    const int y = (int)(i / A.W), x = (int)(i - (long long)y * A.W);
    const float4 s = A.state[i];
    const bool ok = y >= A.r && y <= A.H - 1 - A.r && s.w > 0.0f;
    A.depth[(long long)y * A.pd + x] = ok ? s.w : 0.0f;
    A.n0[(long long)y * A.pn0 + x] = ok ? s.x : 0.0f;
    A.n1[(long long)y * A.pn1 + x] = ok ? s.y : 0.0f;
    A.n2[(long long)y * A.pn2 + x] = ok ? s.z : 0.0f;
    A.cplane[(long long)y * A.pc + x] = ok ? A.cost[i] : 2.0f;
}

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
__global__ __launch_bounds__(BLOCK) void k_consistency(GeoArgs A)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long long)A.W * A.H) return;
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
