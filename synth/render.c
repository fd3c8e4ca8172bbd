/*
 * render.c -- seeded synthetic equirectangular scenes for testing and
 * benchmarking the densifier: ray casting against a few analytic primitive
 * types, a Lambertian solid value-noise texture, supersampled pixels, and
 * ground-truth range and normal per pixel centre.
 *
 * This is an INPUT GENERATOR. It holds none of the densifier's arithmetic
 * (no warping, no matching cost, no propagation); it only defines what the
 * synthetic cameras see. Its equirectangular camera uses the pixel-centre
 * convention that the densifier documents:
 *   lam = 2 pi (x + 0.5) / W - pi,  phi = pi/2 - pi (y + 0.5) / H,
 *   ray = (cos phi sin lam, -sin phi, cos phi cos lam)  (x right, y down,
 *   z forward), poses world -> camera with X_c = R X_w + t.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

#define PRIM_ROOM 0   /* axis-aligned box seen from inside: lo[3], hi[3]        */
#define PRIM_SPHERE 1 /* centre[3], radius                                     */
#define PRIM_QUAD 2   /* centre[3], u[3], v[3] (unit, orthogonal), half_u, half_v */
#define PRIM_BOX 3    /* solid axis-aligned box seen from outside: lo[3], hi[3] */
#define PRIM_PLANE 4  /* point[3], unit normal[3] (infinite)                   */
#define PRIM_STRIDE 16

typedef struct {
    int W, H, ss;
    double Rt[9]; /* camera -> world rotation (R transposed) */
    double C[3];  /* camera centre in world coordinates */
    int n_prims;
    const int32_t *types;
    const double *prm;
    int n_octaves;
    double base_freq, lo, hi, sky;
    uint64_t tex_seed;
    float *image, *depth, *normal;
} scene_t;

static const double PI = 3.14159265358979323846;

static uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

static double lattice(int64_t i, int64_t j, int64_t k, uint64_t seed, int octave)
{
    uint64_t h = seed * 0x9E3779B97F4A7C15ULL + (uint64_t)octave * 0xD1B54A32D192ED03ULL;
    h = mix64(h ^ (uint64_t)i);
    h = mix64(h ^ ((uint64_t)j * 0xABC98388FB8FAC03ULL));
    h = mix64(h ^ ((uint64_t)k * 0x8CB92BA72F3D8DD7ULL));
    return (double)(h >> 11) * (1.0 / 9007199254740992.0);
}

/* Trilinearly interpolated value noise, octaves at doubling frequency and
   halving amplitude, normalised to [lo, hi]. */
static double texture(const scene_t *S, const double p[3])
{
    double sum = 0.0, amp = 1.0, norm = 0.0, f = S->base_freq;
    for (int o = 0; o < S->n_octaves; ++o) {
        double q[3] = {p[0] * f + 17.31 * o, p[1] * f + 5.77 * o, p[2] * f + 11.13 * o};
        double fl[3] = {floor(q[0]), floor(q[1]), floor(q[2])};
        double a[3] = {q[0] - fl[0], q[1] - fl[1], q[2] - fl[2]};
        int64_t i0 = (int64_t)fl[0], j0 = (int64_t)fl[1], k0 = (int64_t)fl[2];
        double v = 0.0;
        for (int c = 0; c < 8; ++c) {
            int di = c & 1, dj = (c >> 1) & 1, dk = (c >> 2) & 1;
            double w = (di ? a[0] : 1.0 - a[0]) * (dj ? a[1] : 1.0 - a[1]) * (dk ? a[2] : 1.0 - a[2]);
            v += w * lattice(i0 + di, j0 + dj, k0 + dk, S->tex_seed, o);
        }
        sum += amp * v;
        norm += amp;
        amp *= 0.5;
        f *= 2.0;
    }
    return S->lo + (S->hi - S->lo) * (sum / norm);
}

static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

/* Nearest hit along o + s d (d unit) with s > 1e-9; returns s or INFINITY and
   the surface normal facing the ray. */
static double cast(const scene_t *S, const double o[3], const double d[3], double nrm[3])
{
    double best = INFINITY;
    for (int k = 0; k < S->n_prims; ++k) {
        const double *q = S->prm + (size_t)k * PRIM_STRIDE;
        double s = INFINITY, n[3] = {0, 0, 0};
        switch (S->types[k]) {
        case PRIM_ROOM: {
            double smin = INFINITY;
            int axis = -1;
            for (int a = 0; a < 3; ++a) {
                if (d[a] > 0.0) {
                    double v = (q[3 + a] - o[a]) / d[a];
                    if (v < smin) smin = v, axis = a;
                } else if (d[a] < 0.0) {
                    double v = (q[a] - o[a]) / d[a];
                    if (v < smin) smin = v, axis = a;
                }
            }
            if (axis >= 0 && smin > 1e-9) {
                s = smin;
                n[axis] = d[axis] > 0.0 ? -1.0 : 1.0;
            }
            break;
        }
        case PRIM_SPHERE: {
            double oc[3] = {o[0] - q[0], o[1] - q[1], o[2] - q[2]};
            double b = dot3(oc, d), c = dot3(oc, oc) - q[3] * q[3];
            double disc = b * b - c;
            if (disc >= 0.0) {
                double r = sqrt(disc);
                double s0 = -b - r, s1 = -b + r;
                double sh = s0 > 1e-9 ? s0 : (s1 > 1e-9 ? s1 : INFINITY);
                if (sh < INFINITY) {
                    s = sh;
                    for (int a = 0; a < 3; ++a) n[a] = (o[a] + s * d[a] - q[a]) / q[3];
                }
            }
            break;
        }
        case PRIM_QUAD: {
            const double *c = q, *u = q + 3, *v = q + 6;
            double pn[3] = {u[1] * v[2] - u[2] * v[1], u[2] * v[0] - u[0] * v[2],
                            u[0] * v[1] - u[1] * v[0]};
            double den = dot3(pn, d);
            if (fabs(den) > 1e-12) {
                double co[3] = {c[0] - o[0], c[1] - o[1], c[2] - o[2]};
                double sh = dot3(pn, co) / den;
                if (sh > 1e-9) {
                    double h[3] = {o[0] + sh * d[0] - c[0], o[1] + sh * d[1] - c[1],
                                   o[2] + sh * d[2] - c[2]};
                    if (fabs(dot3(h, u)) <= q[9] && fabs(dot3(h, v)) <= q[10]) {
                        s = sh;
                        for (int a = 0; a < 3; ++a) n[a] = pn[a];
                    }
                }
            }
            break;
        }
        case PRIM_BOX: {
            double t0 = -INFINITY, t1 = INFINITY;
            int ax0 = -1;
            double sg0 = 0.0;
            int miss = 0;
            for (int a = 0; a < 3 && !miss; ++a) {
                if (d[a] == 0.0) {
                    if (o[a] < q[a] || o[a] > q[3 + a]) miss = 1;
                    continue;
                }
                double ta = (q[a] - o[a]) / d[a], tb = (q[3 + a] - o[a]) / d[a];
                double sg = -1.0; /* normal of the entry face */
                if (ta > tb) {
                    double tmp = ta;
                    ta = tb;
                    tb = tmp;
                    sg = 1.0;
                }
                if (ta > t0) t0 = ta, ax0 = a, sg0 = sg;
                if (tb < t1) t1 = tb;
            }
            if (!miss && t0 <= t1 && t0 > 1e-9 && ax0 >= 0) {
                s = t0;
                n[ax0] = sg0;
            }
            break;
        }
        case PRIM_PLANE: {
            double den = dot3(q + 3, d);
            if (fabs(den) > 1e-12) {
                double co[3] = {q[0] - o[0], q[1] - o[1], q[2] - o[2]};
                double sh = dot3(q + 3, co) / den;
                if (sh > 1e-9) {
                    s = sh;
                    for (int a = 0; a < 3; ++a) n[a] = q[3 + a];
                }
            }
            break;
        }
        default:
            break;
        }
        if (s < best) {
            best = s;
            if (dot3(n, d) > 0.0) n[0] = -n[0], n[1] = -n[1], n[2] = -n[2];
            nrm[0] = n[0];
            nrm[1] = n[1];
            nrm[2] = n[2];
        }
    }
    return best;
}

static void ray_dir(const scene_t *S, double x, double y, double dw[3], double dc[3])
{
    double lam = 2.0 * PI * (x + 0.5) / S->W - PI;
    double phi = PI / 2.0 - PI * (y + 0.5) / S->H;
    dc[0] = cos(phi) * sin(lam);
    dc[1] = -sin(phi);
    dc[2] = cos(phi) * cos(lam);
    for (int i = 0; i < 3; ++i) dw[i] = S->Rt[3 * i] * dc[0] + S->Rt[3 * i + 1] * dc[1] + S->Rt[3 * i + 2] * dc[2];
}

typedef struct {
    const scene_t *S;
    int y0, y1;
} band_t;

static void *render_band(void *arg)
{
    band_t *B = (band_t *)arg;
    const scene_t *S = B->S;
    int W = S->W, H = S->H, ss = S->ss;
    size_t HW = (size_t)W * H;
    for (int y = B->y0; y < B->y1; ++y)
        for (int x = 0; x < W; ++x) {
            size_t i = (size_t)y * W + x;
            double acc = 0.0;
            for (int sy = 0; sy < ss; ++sy)
                for (int sx = 0; sx < ss; ++sx) {
                    double ox = (sx + 0.5) / ss - 0.5, oy = (sy + 0.5) / ss - 0.5;
                    double dw[3], dc[3], n[3];
                    ray_dir(S, x + ox, y + oy, dw, dc);
                    double s = cast(S, S->C, dw, n);
                    if (s < INFINITY) {
                        double p[3] = {S->C[0] + s * dw[0], S->C[1] + s * dw[1], S->C[2] + s * dw[2]};
                        acc += texture(S, p);
                    } else {
                        acc += S->sky;
                    }
                }
            S->image[i] = (float)(acc / (ss * ss));
            if (S->depth || S->normal) {
                double dw[3], dc[3], n[3];
                ray_dir(S, x, y, dw, dc);
                double s = cast(S, S->C, dw, n);
                int hit = s < INFINITY;
                if (S->depth) S->depth[i] = hit ? (float)s : 0.0f;
                if (S->normal) {
                    /* world normal into the camera frame: n_c = R n_w */
                    for (int a = 0; a < 3; ++a) {
                        double v = hit ? (S->Rt[a] * n[0] + S->Rt[3 + a] * n[1] + S->Rt[6 + a] * n[2]) : 0.0;
                        S->normal[a * HW + i] = (float)v;
                    }
                }
            }
        }
    return NULL;
}

int synth_render(int W, int H, int ss, const double R[9], const double t[3], int n_prims,
                 const int32_t *types, const double *prm, int n_octaves, double base_freq,
                 double lo, double hi, uint64_t tex_seed, double sky, float *image, float *depth,
                 float *normal, int n_threads)
{
    if (W <= 0 || H <= 0 || ss <= 0 || !image || n_prims < 0) return -1;
    scene_t S;
    memset(&S, 0, sizeof S);
    S.W = W;
    S.H = H;
    S.ss = ss;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) S.Rt[3 * i + j] = R[3 * j + i];
    for (int i = 0; i < 3; ++i) S.C[i] = -(S.Rt[3 * i] * t[0] + S.Rt[3 * i + 1] * t[1] + S.Rt[3 * i + 2] * t[2]);
    S.n_prims = n_prims;
    S.types = types;
    S.prm = prm;
    S.n_octaves = n_octaves;
    S.base_freq = base_freq;
    S.lo = lo;
    S.hi = hi;
    S.sky = sky;
    S.tex_seed = tex_seed;
    S.image = image;
    S.depth = depth;
    S.normal = normal;
    int T = n_threads > 0 ? n_threads : (int)sysconf(_SC_NPROCESSORS_ONLN);
    if (T < 1) T = 1;
    if (T > 64) T = 64;
    if (T > H) T = H;
    pthread_t th[64];
    band_t bands[64];
    int ok[64];
    for (int k = 0; k < T; ++k) {
        bands[k].S = &S;
        bands[k].y0 = H * k / T;
        bands[k].y1 = H * (k + 1) / T;
    }
    for (int k = 1; k < T; ++k) {
        ok[k] = pthread_create(&th[k], NULL, render_band, &bands[k]) == 0;
        if (!ok[k]) render_band(&bands[k]);
    }
    render_band(&bands[0]);
    for (int k = 1; k < T; ++k)
        if (ok[k]) pthread_join(th[k], NULL);
    return 0;
}
