/*
 * glint_oracle.c -- plain, slow FP64 CPU oracle for image-based glint lighting
 * (Kneiphof & Klein, "Real-Time Image-based Lighting of Glints", EGSR 2025).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may link, load or
 * call this file; only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark do.  It shares no code, header, table or helper with the
 * HIP library: every routine here is written independently from the paper.
 *
 * Precision: every step runs in IEEE double, except where the paper fixes
 * the precision.  The paper designs the gating probabilities of the
 * dual-gated Gaussian (Sec. 6, Alg. "Dual-gated Gaussian", paragraph
 * "Numeric Gating Issues") for 32-bit floats: the bias constant
 * eps = 10^-3.54 is tuned for FP32.  Those thresholds, and the decisions
 * taken on them, are evaluated in float here.  Stored textures (the
 * unfiltered indicator lerp factor, the source mip chain, the prefiltered
 * pyramid, the lookup tables) are 32-bit float values, as the paper's
 * textures are; the oracle rounds to float exactly where a texture is
 * written and computes everything else in double.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC (see build.py).
 * -ffp-contract=off keeps every float expression rounded as written.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <float.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_EINVAL 1

/* ------------------------------------------------------------------------ */
/* Cube-map conventions (texture addressing is an implementation reading:   */
/* the paper delegates environment filtering to standard real-time IBL).    */
/* Faces +X,-X,+Y,-Y,+Z,-Z; texel (x,y) of a face of size n has face        */
/* coordinates s = 2(x+1/2)/n - 1, t = 2(y+1/2)/n - 1.                        */
/* ------------------------------------------------------------------------ */
static void face_to_dir(int face, double s, double t, double d[3])
{
    switch (face) {
    case 0: d[0] = 1.0;  d[1] = -t;   d[2] = -s;   break;
    case 1: d[0] = -1.0; d[1] = -t;   d[2] = s;    break;
    case 2: d[0] = s;    d[1] = 1.0;  d[2] = t;    break;
    case 3: d[0] = s;    d[1] = -1.0; d[2] = -t;   break;
    case 4: d[0] = s;    d[1] = -t;   d[2] = 1.0;  break;
    default: d[0] = -s;  d[1] = -t;   d[2] = -1.0; break;
    }
}

/* Owning face of a direction (largest |component|, ties to x then y). */
static int dir_to_face(const double d[3], double *s, double *t)
{
    double ax = fabs(d[0]), ay = fabs(d[1]), az = fabs(d[2]);
    if (ax >= ay && ax >= az) {
        if (d[0] >= 0.0) { *s = -d[2] / ax; *t = -d[1] / ax; return 0; }
        *s = d[2] / ax; *t = -d[1] / ax; return 1;
    }
    if (ay >= az) {
        if (d[1] >= 0.0) { *s = d[0] / ay; *t = d[2] / ay; return 2; }
        *s = d[0] / ay; *t = -d[2] / ay; return 3;
    }
    if (d[2] >= 0.0) { *s = d[0] / az; *t = -d[1] / az; return 4; }
    *s = -d[0] / az; *t = -d[1] / az; return 5;
}

static int64_t level_offset(int R, int level)
{
    int64_t off = 0;
    for (int s = 0; s < level; ++s) { int64_t n = R >> s; off += 6 * n * n; }
    return off;
}

/* ------------------------------------------------------------------------ */
/* Sec. 5 "Discrete Radiance Levels" and "Fuzzy Indicator Functions".        */
/* ------------------------------------------------------------------------ */

/* Brightness of one texel.  The paper only considers brightness when
 * building the partition (Sec. 4, paragraph "Light Partition"); it does not
 * define it, so Rec. 709 luminance is used.  Non-finite or negative
 * channels count as 0. */
static double sane(float c) { return (isfinite(c) && c > 0.0f) ? (double)c : 0.0; }

static double luminance(const float *rgb)
{
    return 0.2126 * sane(rgb[0]) + 0.7152 * sane(rgb[1]) + 0.0722 * sane(rgb[2]);
}

/* Radiance levels, Sec. 5: L(1) = 0 and, for k > 1,
 * L(k) = exp(lerp(log min, log max, (k-1)/(K-1))), with min clipped to >= ell.
 * Zero-based index k here.  level_mode 2 is the alternative reading in which
 * the first non-zero level equals the clipped minimum. */
static void radiance_levels(double lmin, double lmax, int K, int level_mode, double *L)
{
    double a = log(lmin), b = log(lmax);
    L[0] = 0.0;
    for (int k = 1; k < K; ++k) {
        double f;
        if (level_mode == 2) f = (K > 2) ? (double)(k - 1) / (double)(K - 2) : 1.0;
        else f = (double)k / (double)(K - 1);
        L[k] = exp(a + f * (b - a));
        if (L[k] > lmax) L[k] = lmax; /* keeps the levels monotone when min ~ max */
    }
    L[K - 1] = lmax;
}

/* Exact solid angle of texel (x, y) of a cube face of size R: the area
 * element dA / (1 + s^2 + t^2)^(3/2) of the unit cube face integrated over
 * the texel, from its antiderivative atan2(s t, sqrt(s^2 + t^2 + 1)). */
static double corner_F(double s, double t) { return atan2(s * t, sqrt(s * s + t * t + 1.0)); }

static double texel_solid_angle(int R, int x, int y)
{
    double s0 = 2.0 * x / R - 1.0, s1 = 2.0 * (x + 1) / R - 1.0;
    double t0 = 2.0 * y / R - 1.0, t1 = 2.0 * (y + 1) / R - 1.0;
    return corner_F(s1, t1) - corner_F(s0, t1) - corner_F(s1, t0) + corner_F(s0, t0);
}

typedef struct {
    double y, w;
} yw_t;

static int cmp_yw(const void *a, const void *b)
{
    double ya = ((const yw_t *)a)->y, yb = ((const yw_t *)b)->y;
    return (ya > yb) - (ya < yb);
}

/* Quantile levels: the configuration's wording "regions by radiance
 * quantiles" (the paper's own levels are the log-lerp above).  Level k,
 * 1 <= k <= K-2 (zero-based), is the solid-angle-weighted quantile of the
 * texel luminance at q = k/(K-1): the smallest texel luminance y whose
 * weighted distribution function C(y) = sum of the solid angles of the
 * texels with Y <= y reaches q W (W the total), clipped to [lmin, lmax]
 * like the log-lerp levels; L(0) = 0 and L(K-1) = lmax.  margin[k]
 * (optional) is the distance of q W to the nearer of C(L(k)) and
 * C(just below L(k)), over W: the room a differently rounded sum has before
 * it would pick another texel value. */
static int quantile_levels(const float *env, int R, int K, double lmin, double lmax, double *L, double *margin)
{
    int64_t n = 6LL * R * R;
    yw_t *a = (yw_t *)malloc(sizeof(yw_t) * (size_t)n);
    if (!a) return ORC_EINVAL;
    for (int f = 0; f < 6; ++f)
        for (int y = 0; y < R; ++y)
            for (int x = 0; x < R; ++x) {
                int64_t i = ((int64_t)f * R + y) * R + x;
                a[i].y = luminance(env + 3 * i);
                a[i].w = texel_solid_angle(R, x, y);
            }
    qsort(a, (size_t)n, sizeof(yw_t), cmp_yw);
    double W = 0.0;
    for (int64_t i = 0; i < n; ++i) W += a[i].w;
    L[0] = 0.0;
    if (margin) margin[0] = INFINITY;
    for (int k = 1; k <= K - 2; ++k) {
        double tau = (double)k / (double)(K - 1) * W;
        double cum = 0.0, below = 0.0;
        int64_t i = 0;
        /* walk runs of equal luminance: C jumps by the whole run */
        while (i < n) {
            int64_t j = i;
            double run = 0.0;
            while (j < n && a[j].y == a[i].y) run += a[j++].w;
            below = cum;
            cum += run;
            if (cum >= tau || j == n) break;
            i = j;
        }
        double q = a[i].y;
        if (q < lmin) q = lmin;
        if (q > lmax) q = lmax;
        L[k] = q;
        if (margin) {
            double m1 = (cum - tau) / W, m2 = (tau - below) / W;
            margin[k] = m1 < m2 ? m1 : m2;
        }
    }
    L[K - 1] = lmax;
    if (margin) margin[K - 1] = INFINITY;
    free(a);
    return ORC_OK;
}

int orc_partition(const float *env, int R, int K, double ell, int level_mode, int weight_space,
                  double *levels, uint8_t *ind_j, float *ind_t)
{
    if (R < 1 || K < 2 || K > 16 || !(ell > 0.0) || level_mode < 0 || level_mode > 2) return ORC_EINVAL;
    int64_t n = 6LL * R * R;
    double ymin = INFINITY, ymax = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double y = luminance(env + 3 * i);
        if (y < ymin) ymin = y;
        if (y > ymax) ymax = y;
    }
    double lmin = ymin > ell ? ymin : ell;
    double lmax = ymax;
    if (lmax < lmin) lmax = lmin;
    if (level_mode == 1) {
        if (quantile_levels(env, R, K, lmin, lmax, levels, NULL)) return ORC_EINVAL;
    } else {
        radiance_levels(lmin, lmax, K, level_mode, levels);
    }
    for (int64_t i = 0; i < n; ++i) {
        double y = luminance(env + 3 * i);
        if (y > levels[K - 1]) y = levels[K - 1];
        /* Eq. (wkdefpractice): j with L(j) <= y < L(j+1); the top interval
         * is closed. */
        int j = 0;
        for (int k = 1; k <= K - 2; ++k)
            if (levels[k] <= y) j = k;
        double lo = levels[j], hi = levels[j + 1], t;
        if (weight_space == 1 && j >= 1) {
            double dl = log(hi) - log(lo);
            t = dl > 0.0 ? (log(y) - log(lo)) / dl : 1.0;
        } else {
            double dl = hi - lo;
            t = dl > 0.0 ? (y - lo) / dl : 1.0;
        }
        if (t < 0.0) t = 0.0;
        if (t > 1.0) t = 1.0;
        ind_j[i] = (uint8_t)j;
        ind_t[i] = (float)t;
    }
    return ORC_OK;
}

/* Quantile levels with their margins (for the tests). */
int orc_quantile_levels(const float *env, int R, int K, double ell, double *levels, double *margin)
{
    if (R < 1 || K < 2 || K > 16 || !(ell > 0.0)) return ORC_EINVAL;
    int64_t n = 6LL * R * R;
    double ymin = INFINITY, ymax = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double y = luminance(env + 3 * i);
        if (y < ymin) ymin = y;
        if (y > ymax) ymax = y;
    }
    double lmin = ymin > ell ? ymin : ell;
    double lmax = ymax < lmin ? lmin : ymax;
    return quantile_levels(env, R, K, lmin, lmax, levels, margin);
}

/* ------------------------------------------------------------------------ */
/* Source mip chain of the environment filter: K indicator channels followed */
/* by RGB radiance.  Level 0 is exact (dense weights 1-t and t, Eq.          */
/* (wkdefpractice)); level s+1 is the mean of the 2x2 children of level s,   */
/* stored as float.                                                          */
/* ------------------------------------------------------------------------ */
typedef struct {
    const float *env;
    const uint8_t *ind_j;
    const float *ind_t;
    const float *chain; /* levels >= 1, float, [C] per texel, C = K + 3 */
    int R, K, M;
} src_chain;

static void level0_texel(const src_chain *c, int face, int x, int y, double *out)
{
    int64_t i = ((int64_t)face * c->R + y) * c->R + x;
    for (int k = 0; k < c->K; ++k) out[k] = 0.0;
    int j = c->ind_j[i];
    double t = (double)c->ind_t[i];
    out[j] = 1.0 - t;
    out[j + 1] = t;
    out[c->K + 0] = sane(c->env[3 * i + 0]);
    out[c->K + 1] = sane(c->env[3 * i + 1]);
    out[c->K + 2] = sane(c->env[3 * i + 2]);
}

static void chain_texel(const src_chain *c, int level, int face, int x, int y, double *out)
{
    if (level == 0) { level0_texel(c, face, x, y, out); return; }
    int C = c->K + 3;
    int64_t n = c->R >> level;
    const float *p = c->chain + (level_offset(c->R, level) - 6LL * c->R * c->R
                                 + ((int64_t)face * n + y) * n + x) * C;
    for (int k = 0; k < C; ++k) out[k] = (double)p[k];
}

int orc_mipchain(const float *env, const uint8_t *ind_j, const float *ind_t, int R, int K, int M,
                 float *chain)
{
    if (R < 1 || K < 2 || K > 16 || M < 1 || (R >> (M - 1)) < 1) return ORC_EINVAL;
    src_chain c = {env, ind_j, ind_t, chain, R, K, M};
    int C = K + 3;
    double a[19], b[19], d[19], e[19];
    for (int s = 1; s < M; ++s) {
        int64_t n = R >> s;
        float *dst = chain + (level_offset(R, s) - 6LL * R * R) * C;
        for (int f = 0; f < 6; ++f)
            for (int y = 0; y < n; ++y)
                for (int x = 0; x < n; ++x) {
                    chain_texel(&c, s - 1, f, 2 * x, 2 * y, a);
                    chain_texel(&c, s - 1, f, 2 * x + 1, 2 * y, b);
                    chain_texel(&c, s - 1, f, 2 * x, 2 * y + 1, d);
                    chain_texel(&c, s - 1, f, 2 * x + 1, 2 * y + 1, e);
                    float *o = dst + ((f * n + y) * n + x) * C;
                    for (int k = 0; k < C; ++k)
                        o[k] = (float)(((a[k] + b[k]) + (d[k] + e[k])) * 0.25);
                }
    }
    return ORC_OK;
}

/* Seams.  A bilinear footprint reaches at most one texel beyond a face.
 * A texel off one edge of the face is re-projected through the 3-D
 * direction of its (extended) centre to the nearest texel of the face that
 * owns that direction -- the adjacent texel across the edge.  The texel off
 * two edges (beyond a cube corner) has no single neighbour: it takes the
 * mean of the three texels that meet at that cube corner.  With this rule
 * the bilinear lookup is continuous across edges and corners, so it does
 * not depend on which face a direction lying on an edge is assigned to. */
static void reproject_one(int face, int x, int y, int n, int *f2, int *x2, int *y2)
{
    double d[3], s, t;
    face_to_dir(face, 2.0 * (x + 0.5) / n - 1.0, 2.0 * (y + 0.5) / n - 1.0, d);
    *f2 = dir_to_face(d, &s, &t);
    int a = (int)floor((s + 1.0) * 0.5 * n);
    int b = (int)floor((t + 1.0) * 0.5 * n);
    *x2 = a < 0 ? 0 : (a > n - 1 ? n - 1 : a);
    *y2 = b < 0 ? 0 : (b > n - 1 ? n - 1 : b);
}

/* Resolves texel (x, y) of `face` (x, y in [-1, n]) to 1 or 3 in-face
 * texels; returns the count. */
static int resolve_texel(int face, int x, int y, int n, int fo[3], int xo[3], int yo[3])
{
    int xin = x >= 0 && x < n, yin = y >= 0 && y < n;
    if (xin && yin) { fo[0] = face; xo[0] = x; yo[0] = y; return 1; }
    int xc = x < 0 ? 0 : (x > n - 1 ? n - 1 : x);
    int yc = y < 0 ? 0 : (y > n - 1 ? n - 1 : y);
    if (xin || yin) { reproject_one(face, x, y, n, &fo[0], &xo[0], &yo[0]); return 1; }
    fo[0] = face; xo[0] = xc; yo[0] = yc;
    reproject_one(face, x, yc, n, &fo[1], &xo[1], &yo[1]);
    reproject_one(face, xc, y, n, &fo[2], &xo[2], &yo[2]);
    return 3;
}

static void chain_texel_seamless(const src_chain *c, int level, int face, int x, int y, double *out)
{
    int n = c->R >> level;
    int fo[3], xo[3], yo[3];
    int cnt = resolve_texel(face, x, y, n, fo, xo, yo);
    if (cnt == 1) { chain_texel(c, level, fo[0], xo[0], yo[0], out); return; }
    double a[20], b[20], d[20];
    chain_texel(c, level, fo[0], xo[0], yo[0], a);
    chain_texel(c, level, fo[1], xo[1], yo[1], b);
    chain_texel(c, level, fo[2], xo[2], yo[2], d);
    for (int k = 0; k < c->K + 3; ++k) out[k] = ((a[k] + b[k]) + d[k]) / 3.0;
}

typedef void (*texel_fn)(const void *src, int level, int face, int x, int y, double *out);

/* Bilinear lookup of one mip level in direction d (C channels). */
static void bilinear(texel_fn fn, const void *src, int R, int level, int C, const double d[3], double *out)
{
    int n = R >> level;
    double s, t;
    int face = dir_to_face(d, &s, &t);
    double x = (s + 1.0) * 0.5 * n - 0.5;
    double y = (t + 1.0) * 0.5 * n - 0.5;
    double x0 = floor(x), y0 = floor(y);
    double fx = x - x0, fy = y - y0;
    int ix = (int)x0, iy = (int)y0;
    double v00[20], v10[20], v01[20], v11[20];
    fn(src, level, face, ix, iy, v00);
    fn(src, level, face, ix + 1, iy, v10);
    fn(src, level, face, ix, iy + 1, v01);
    fn(src, level, face, ix + 1, iy + 1, v11);
    for (int k = 0; k < C; ++k) {
        double top = (1.0 - fx) * v00[k] + fx * v10[k];
        double bot = (1.0 - fx) * v01[k] + fx * v11[k];
        out[k] = (1.0 - fy) * top + fy * bot;
    }
}

/* Trilinear lookup: linear blend of the two mip levels around lod. */
static void trilinear(texel_fn fn, const void *src, int R, int M, int C, const double d[3], double lod,
                      double *out)
{
    if (lod < 0.0) lod = 0.0;
    if (lod > M - 1) lod = M - 1;
    double l0 = floor(lod);
    int s0 = (int)l0;
    int s1 = s0 + 1 < M ? s0 + 1 : M - 1;
    double f = lod - l0;
    double a[20], b[20];
    bilinear(fn, src, R, s0, C, d, a);
    bilinear(fn, src, R, s1, C, d, b);
    for (int k = 0; k < C; ++k) out[k] = (1.0 - f) * a[k] + f * b[k];
}

static void chain_fn(const void *src, int level, int face, int x, int y, double *out)
{
    chain_texel_seamless((const src_chain *)src, level, face, x, y, out);
}

/* ------------------------------------------------------------------------ */
/* Sec. 5 "Integrated NDF", Eq. (rtiblndf) with the kernel of Eq. (rtibl):   */
/* each indicator channel (and RGB) is filtered with the same real-time IBL  */
/* kernel, assuming n = v = r.  Reading of the delegated kernel: GGX          */
/* importance sampling of T Hammersley taps, tap weight <r,l>+, filtered      */
/* importance sampling for the source lod, roughness alpha_m = (m/(M-1))^2.   */
/* ------------------------------------------------------------------------ */
static double radical_inverse(uint32_t j)
{
    uint32_t b = j;
    b = (b << 16) | (b >> 16);
    b = ((b & 0x55555555u) << 1) | ((b & 0xAAAAAAAAu) >> 1);
    b = ((b & 0x33333333u) << 2) | ((b & 0xCCCCCCCCu) >> 2);
    b = ((b & 0x0F0F0F0Fu) << 4) | ((b & 0xF0F0F0F0u) >> 4);
    b = ((b & 0x00FF00FFu) << 8) | ((b & 0xFF00FF00u) >> 8);
    return (double)b * 2.3283064365386963e-10; /* 2^-32 */
}

typedef struct { double hx, hy, hz, w, lod; } tap_t;

/* Tap table for roughness alpha (the prefilter uses alpha_m = (m/(M-1))^2;
 * the filter sampled at an arbitrary alpha uses the same construction). */
static void make_taps_alpha(double alpha, int M, int T, int R, tap_t *taps)
{
    double a2 = alpha * alpha;
    double omega_p = 4.0 * M_PI / (6.0 * (double)R * (double)R);
    for (int j = 0; j < T; ++j) {
        double uphi = (double)j / (double)T;
        double uth = radical_inverse((uint32_t)j);
        double c2 = (1.0 - uth) / (1.0 + (a2 - 1.0) * uth);
        double ct = sqrt(c2);
        double st = sqrt(fmax(0.0, 1.0 - c2));
        double phi = 2.0 * M_PI * uphi;
        taps[j].hx = st * cos(phi);
        taps[j].hy = st * sin(phi);
        taps[j].hz = ct;
        taps[j].w = fmax(0.0, 2.0 * c2 - 1.0);
        double den = 1.0 + (a2 - 1.0) * c2;
        double D = a2 / (M_PI * den * den);
        double omega_s = 4.0 / ((double)T * D);
        double lod = 0.5 * log2(omega_s / omega_p) + 1.0;
        if (lod < 0.0) lod = 0.0;
        if (lod > M - 1) lod = M - 1;
        taps[j].lod = lod;
    }
}

static void make_taps(int m, int M, int T, int R, tap_t *taps)
{
    double a = (double)m / (double)(M - 1);
    make_taps_alpha(a * a, M, T, R, taps);
}

/* Orthonormal basis around r (Duff et al. 2017, branchless construction). */
static void onb(const double r[3], double t1[3], double t2[3])
{
    double sgn = copysign(1.0, r[2]);
    double a = -1.0 / (sgn + r[2]);
    double b = r[0] * r[1] * a;
    t1[0] = 1.0 + sgn * r[0] * r[0] * a; t1[1] = sgn * b; t1[2] = -sgn * r[0];
    t2[0] = b; t2[1] = sgn + r[1] * r[1] * a; t2[2] = -r[1];
}

/* Filter all K+3 channels around the unit direction r with a tap table. */
static void filter_dir(const src_chain *c, int T, const double r[3], const tap_t *taps, double *out)
{
    int C = c->K + 3;
    double t1[3], t2[3];
    onb(r, t1, t2);
    double acc[20] = {0}, wsum = 0.0, v[20];
    for (int j = 0; j < T; ++j) {
        if (!(taps[j].w > 0.0)) continue;
        double h[3], l[3];
        for (int i = 0; i < 3; ++i) h[i] = taps[j].hx * t1[i] + taps[j].hy * t2[i] + taps[j].hz * r[i];
        for (int i = 0; i < 3; ++i) l[i] = 2.0 * taps[j].hz * h[i] - r[i];
        trilinear(chain_fn, c, c->R, c->M, C, l, taps[j].lod, v);
        for (int k = 0; k < C; ++k) acc[k] += taps[j].w * v[k];
        wsum += taps[j].w;
    }
    for (int k = 0; k < C; ++k) out[k] = acc[k] / wsum;
}

/* Filter one output texel (mip m >= 1): its centre direction, normalised. */
static void filter_texel(const src_chain *c, int T, int m, int face, int x, int y, const tap_t *taps,
                         double *out)
{
    int n = c->R >> m;
    double r[3];
    face_to_dir(face, 2.0 * (x + 0.5) / n - 1.0, 2.0 * (y + 0.5) / n - 1.0, r);
    double len = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
    r[0] /= len; r[1] /= len; r[2] /= len;
    filter_dir(c, T, r, taps, out);
}

/* Prefiltered pyramid values (double, K indicator channels then RGB) of the
 * requested texels.  texel_ids index the mip-major pyramid
 * [m][face][y][x]; mip 0 is the unfiltered level (alpha = 0). */
int orc_prefilter_texels(const float *env, const uint8_t *ind_j, const float *ind_t, const float *chain,
                         int R, int K, int M, int T, const int64_t *texel_ids, int64_t count, double *out,
                         int threads)
{
    if (R < 1 || K < 2 || K > 16 || M < 1 || (R >> (M - 1)) < 1 || T < 1) return ORC_EINVAL;
    src_chain c = {env, ind_j, ind_t, chain, R, K, M};
    int C = K + 3;
    tap_t *taps = (tap_t *)malloc(sizeof(tap_t) * (size_t)T * (size_t)M);
    for (int m = 1; m < M; ++m) make_taps(m, M, T, R, taps + (size_t)m * T);
    int64_t total = level_offset(R, M);
    int bad = 0;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 64) num_threads(threads > 0 ? threads : 1) reduction(| : bad)
#endif
    for (int64_t q = 0; q < count; ++q) {
        int64_t id = texel_ids[q];
        if (id < 0 || id >= total) { bad = 1; continue; }
        int m = 0;
        while (m + 1 < M && id >= level_offset(R, m + 1)) ++m;
        int64_t rem = id - level_offset(R, m);
        int64_t n = R >> m;
        int face = (int)(rem / (n * n));
        int y = (int)((rem / n) % n), x = (int)(rem % n);
        if (m == 0) level0_texel(&c, face, x, y, out + q * C);
        else filter_texel(&c, T, m, face, x, y, taps + (size_t)m * T, out + q * C);
    }
    (void)threads;
    free(taps);
    return bad ? ORC_EINVAL : ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Lookup tables (once per BRDF model).                                      */
/* S(mu_o, alpha) = E_D / D_H: Sec. 5 "Integrated NDF" defines the visible    */
/* reflecting microfacet area E_D = integral over the upper hemisphere of     */
/* D(h)/(4<h,l>) dl; Sec. 3.2 defines the total microfacet area D_H.  In      */
/* half-vector measure E_D integrates D over h whose mirror direction is     */
/* above the surface.  E_rho (split sum, Sec. 3.4 Eq. (rtibl)) uses Schlick  */
/* Fresnel and height-correlated Smith masking-shadowing (Sec. 7).           */
/* Quadrature (a reading; the paper gives none): GGX half vectors            */
/* parameterised by s in (0,1), cos^2(theta_h) = s^2/(a^2 + (1-a^2) s^2), in  */
/* which D dw_h = q(s) ds dphi / pi with q = sqrt(a^2 + (1-a^2) s^2); the     */
/* valid azimuths form one arc |phi| < phi_max(s).  Midpoint rules.           */
/* Grid: 64 x 64 cells over (mu_o, sqrt(alpha)), cell centred, [alpha][mu].   */
/* ------------------------------------------------------------------------ */
#define LUT_N 64
#define LUT_NS_S 4096
#define LUT_NS_E 512
#define LUT_NPHI_E 64

/* cos(phi) threshold above which the reflected direction is above the
 * horizon; returns phi_max / pi in [0,1]. */
static double arc_fraction(double mu, double sin_o, double ch, double sh)
{
    double rhs = mu * (1.0 - 2.0 * ch * ch) / (2.0 * ch);
    double den = sin_o * sh;
    if (!(den > 0.0)) return rhs < 0.0 ? 1.0 : 0.0;
    double c = rhs / den;
    if (c <= -1.0) return 1.0;
    if (c >= 1.0) return 0.0;
    return acos(c) / M_PI;
}

static double smith_lambda(double mu, double a2)
{
    double m2 = mu * mu;
    return 0.5 * (-1.0 + sqrt(1.0 + a2 * (1.0 - m2) / m2));
}

static void lut_cell(int ia, int im, double *S, double *A, double *B)
{
    double mu = ((double)im + 0.5) / LUT_N;
    double sa = ((double)ia + 0.5) / LUT_N;
    double alpha = sa * sa;
    double a2 = alpha * alpha;
    double sin_o = sqrt(1.0 - mu * mu);
    /* S */
    double num = 0.0, den = 0.0;
    for (int i = 0; i < LUT_NS_S; ++i) {
        double s = ((double)i + 0.5) / LUT_NS_S;
        double q = sqrt(a2 + (1.0 - a2) * s * s);
        double ch = s / q;
        double sh = alpha * sqrt(1.0 - s * s) / q;
        num += q * arc_fraction(mu, sin_o, ch, sh);
        den += q;
    }
    *S = num / den;
    /* E_rho = F0 * A + B */
    double lam_o = smith_lambda(mu, a2);
    double sa_acc = 0.0, sb_acc = 0.0;
    for (int i = 0; i < LUT_NS_E; ++i) {
        double s = ((double)i + 0.5) / LUT_NS_E;
        double q = sqrt(a2 + (1.0 - a2) * s * s);
        double ch = s / q;
        double sh = alpha * sqrt(1.0 - s * s) / q;
        double frac = arc_fraction(mu, sin_o, ch, sh);
        if (!(frac > 0.0)) continue;
        double phimax = frac * M_PI;
        double w = (q / M_PI) * (1.0 / LUT_NS_E) * (2.0 * phimax / LUT_NPHI_E);
        for (int b = 0; b < LUT_NPHI_E; ++b) {
            double phi = ((double)b + 0.5) / LUT_NPHI_E * phimax;
            double vh = sin_o * sh * cos(phi) + mu * ch;
            double mu_i = 2.0 * vh * ch - mu;
            if (!(mu_i > 0.0) || !(vh > 0.0)) continue;
            double g2 = 1.0 / (1.0 + lam_o + smith_lambda(mu_i, a2));
            double x = 1.0 - vh;
            double fc = x * x * x * x * x;
            double base = g2 * vh / mu * w;
            sa_acc += (1.0 - fc) * base;
            sb_acc += fc * base;
        }
    }
    *A = sa_acc;
    *B = sb_acc;
}

/* cells[i] = ia * 64 + im. */
int orc_lut_cells(const int *cells, int64_t count, double *S, double *A, double *B, int threads)
{
    int bad = 0;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 4) num_threads(threads > 0 ? threads : 1) reduction(| : bad)
#endif
    for (int64_t q = 0; q < count; ++q) {
        int c = cells[q];
        if (c < 0 || c >= LUT_N * LUT_N) { bad = 1; continue; }
        lut_cell(c / LUT_N, c % LUT_N, S + q, A + q, B + q);
    }
    (void)threads;
    return bad ? ORC_EINVAL : ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Inverse standard normal CDF: Wichura, "Algorithm AS 241: The percentage   */
/* points of the normal distribution", Applied Statistics 37 (1988),         */
/* PPND16 (about 1e-16 relative accuracy).                                   */
/* ------------------------------------------------------------------------ */
double orc_ppnd16(double p)
{
    double q = p - 0.5, r, val;
    if (fabs(q) <= 0.425) {
        r = 0.180625 - q * q;
        val = q * (((((((r * 2509.0809287301226727 + 33430.575583588128105) * r + 67265.770927008700853) * r
                        + 45921.953931549871457) * r + 13731.693765509461125) * r + 1971.5909503065514427) * r
                     + 133.14166789178437745) * r + 3.387132872796366608)
              / (((((((r * 5226.495278852545925 + 28729.085735721942674) * r + 39307.89580009271061) * r
                     + 21213.794301586595867) * r + 5394.1960214247511077) * r + 687.1870074920579083) * r
                  + 42.313330701600911252) * r + 1.0);
        return val;
    }
    r = q < 0.0 ? p : 1.0 - p;
    if (r <= 0.0) return q < 0.0 ? -INFINITY : INFINITY;
    r = sqrt(-log(r));
    if (r <= 5.0) {
        r -= 1.6;
        val = (((((((r * 7.7454501427834140764e-4 + 0.0227238449892691845833) * r + 0.24178072517745061177) * r
                   + 1.27045825245236838258) * r + 3.64784832476320460504) * r + 5.7694972214606914055) * r
                + 4.6303378461565452959) * r + 1.42343711074968357734)
              / (((((((r * 1.05075007164441684324e-9 + 5.475938084995344946e-4) * r + 0.0151986665636164571966) * r
                     + 0.14810397642748007459) * r + 0.68976733498510000455) * r + 1.6763848301838038494) * r
                  + 2.05319162663775882187) * r + 1.0);
    } else {
        r -= 5.0;
        val = (((((((r * 2.01033439929228813265e-7 + 2.71155556874348757815e-5) * r + 0.0012426609473880784386) * r
                   + 0.026532189526576123093) * r + 0.29656057182850489123) * r + 1.7848265399172913358) * r
                + 5.4637849111641143699) * r + 6.6579046435011037772)
              / (((((((r * 2.04426310338993978564e-15 + 1.4215117583164458887e-7) * r + 1.8463183175100546818e-5) * r
                     + 7.868691311456132591e-4) * r + 0.0148753612908506148525) * r + 0.13692988092273580531) * r
                  + 0.59983220655588793769) * r + 1.0);
    }
    return q < 0.0 ? -val : val;
}

/* ------------------------------------------------------------------------ */
/* Per-footprint random numbers: the PCG-family 4-D hash "pcg4d" of          */
/* Jarzynski & Olano, "Hash Functions for GPU Rendering", JCGT 9(3), 2020.    */
/* xi = ((h >> 9) + 1/2) 2^-23 lies in (0,1) and is exact in float.           */
/* ------------------------------------------------------------------------ */
static void pcg4d(uint32_t v[4])
{
    for (int i = 0; i < 4; ++i) v[i] = v[i] * 1664525u + 1013904223u;
    v[0] += v[1] * v[3]; v[1] += v[2] * v[0]; v[2] += v[0] * v[1]; v[3] += v[1] * v[2];
    for (int i = 0; i < 4; ++i) v[i] ^= v[i] >> 16;
    v[0] += v[1] * v[3]; v[1] += v[2] * v[0]; v[2] += v[0] * v[1]; v[3] += v[1] * v[2];
}

static float to_unit(uint32_t h) { return ((float)(h >> 9) + 0.5f) * 1.1920928955078125e-07f; }

/* One hash serves two tree nodes: nodes 2i and 2i+1 of a lattice vertex
 * take (x, y) and (z, w) of pcg4d(a, b, key | i, seed ^ surf * phi); the
 * key names the lattice (its upper 16 bits: level << 16 for the lattices of
 * vertices 1 and 6, the footprint cell vertex for the full grid). */
static void hash_xi_key(uint32_t seed, uint32_t surf, uint32_t key, int64_t a, int64_t b, int node, float *xi1,
                        float *xi2)
{
    uint32_t v[4];
    v[0] = (uint32_t)a;
    v[1] = (uint32_t)b;
    v[2] = key | (((uint32_t)node >> 1) & 0xFFFFu);
    v[3] = seed ^ (surf * 0x9E3779B9u);
    pcg4d(v);
    *xi1 = to_unit(v[(node & 1) ? 2 : 0]);
    *xi2 = to_unit(v[(node & 1) ? 3 : 1]);
}

void orc_hash_xi(uint32_t seed, uint32_t surf, int32_t level, int64_t a, int64_t b, int node, float *xi1,
                 float *xi2)
{
    hash_xi_key(seed, surf, ((uint32_t)level & 0xFFFFu) << 16, a, b, node, xi1, xi2);
}

/* The raw hash on n 4-word inputs (in and out [n][4]), for the quality
 * checks of the hash itself. */
void orc_pcg4d(const uint32_t *in, uint32_t *out, int64_t n)
{
    for (int64_t i = 0; i < n; ++i) {
        uint32_t v[4] = {in[4 * i], in[4 * i + 1], in[4 * i + 2], in[4 * i + 3]};
        pcg4d(v);
        for (int k = 0; k < 4; ++k) out[4 * i + k] = v[k];
    }
}

/* ------------------------------------------------------------------------ */
/* Sec. 6, Alg. "Dual-gated Gaussian".  Gating probabilities and masks in    */
/* float (the paper's precision for them); the Gaussian in double.  The      */
/* bias of paragraph "Numeric Gating Issues": c = max(1, eps/p) gives        */
/* c*p = max(p, eps) and N/c = N*min(1, p/eps); this form equals the         */
/* algorithm's and stays defined at p = 0.                                   */
/* ------------------------------------------------------------------------ */
#define EPS_GATE 2.8840315031266055e-04 /* 10^-3.54 */

typedef struct {
    float P_nN, P_n1, P_nbN, P_nb1;
    float th[4];      /* the four mask thresholds as compared with xi1 */
    float th_scale[4];/* magnitude of the terms behind each threshold */
} gate_t;

/* sym = 0: Alg. "Dual-gated Gaussian" as printed, where only the power
 * (1-p)^N2 carries the bias.  sym = 1: the bias on both powers, P(n=N)
 * taken as (1 - max(q, eps))^(N2 min(1, q/eps)) with q = 1 - p the other
 * side's probability computed on its own (not as 1 - float(p)). */
static void gate_probs(float Nf, float pf, float qf, int sym, gate_t *g)
{
    const float eps = (float)EPS_GATE;
    float N2 = fmaxf(2.0f, Nf);
    float cN = fminf(fmaxf(Nf - 1.0f, 0.0f), 1.0f);
    float cp = fmaxf(pf, eps);
    float ex = N2 * fminf(1.0f, pf / eps);
    float d1 = fmaxf(0.0f, 1.0f - fabsf(1.0f - Nf));
    float pow_n = sym ? powf(1.0f - fmaxf(qf, eps), N2 * fminf(1.0f, qf / eps)) : powf(pf, N2);
    float pow_nb = powf(1.0f - cp, ex);
    g->P_nN = cN * pow_n;
    g->P_nbN = cN * pow_nb;
    g->P_n1 = d1 * pf;
    g->P_nb1 = d1 * (1.0f - pf);
    g->th[0] = g->P_nN;
    g->th[1] = g->P_nN + g->P_n1;
    g->th[2] = 1.0f - g->P_nbN;
    g->th[3] = (1.0f - g->P_nbN) - g->P_nb1;
    g->th_scale[0] = g->P_nN;
    g->th_scale[1] = g->P_nN + g->P_n1;
    g->th_scale[2] = g->P_nbN;
    g->th_scale[3] = g->P_nbN + g->P_nb1;
}

/* Flag: xi1 within the band in which a conforming float evaluation of the
 * same thresholds (powf within 2 ulp, then the same float operations) might
 * decide differently. */
static int gate_band_flag(const gate_t *g, float xi1)
{
    for (int i = 0; i < 4; ++i) {
        double band = 9.5367431640625e-07 * (double)g->th_scale[i] + 5.9604644775390625e-08;
        if (fabs((double)xi1 - (double)g->th[i]) <= band) return 1;
    }
    return 0;
}

/* float rounding of x is ambiguous if x sits within 1e-12 (relative) of a
 * rounding boundary; then a double that agrees to ~1e-15 elsewhere could
 * round to the other neighbour. */
static int round_flag(double x)
{
    double e = fabs(x) * 1e-12 + 1e-300;
    return (float)(x - e) != (float)(x + e);
}

typedef struct {
    double n, nb;
    uint8_t code;
    int flag;
    /* the count varies continuously with the value of a Gaussian draw (of
     * this node or above), whose last bits follow those of p: such a count
     * can land on an integer on one implementation and just below it on
     * another.  Counts formed from gating constants, clamp bounds, the
     * floor of the prior single gate and N_P do not. */
    int n_cont, nb_cont;
} node_out;

/* N_exact: N is computed exactly on every conforming implementation (the
 * root count N_P = density * area, an exact double product of two floats),
 * so its float rounding cannot differ. */
static void dual_gated(double N, double p, double q, int sym, float xi1, float xi2, int N_exact, int N_cont,
                       node_out *o)
{
    float Nf = (float)N, pf = (float)p, qf = (float)q;
    gate_t g;
    gate_probs(Nf, pf, qf, sym, &g);
    int B_nN = xi1 < g.th[0];
    int B_n1N = xi1 < g.th[1];
    int B_nbN = g.th[2] <= xi1;
    int B_nb1N = g.th[3] <= xi1;
    int B_G = (Nf > 1.0f) && !B_n1N && !B_nb1N;
    double N2 = N > 2.0 ? N : 2.0;
    double mu = 1.0 + (N2 - 2.0) * p;
    double sig = sqrt((N2 - 2.0) * p * (1.0 - p));
    double x = mu + sig * orc_ppnd16((double)xi2);
    double G = x < 1.0 ? 1.0 : (x > N2 - 1.0 ? N2 - 1.0 : x);
    double Gb = N2 - G;
    o->n = (B_nN ? N2 - 1.0 : 0.0) + (B_n1N ? 1.0 : 0.0) + (B_G ? G : 0.0);
    o->nb = (B_nbN ? N2 - 1.0 : 0.0) + (B_nb1N ? 1.0 : 0.0) + (B_G ? Gb : 0.0);
    /* per term: N2 follows N above 2; G and N2 - G follow the draw unless
     * G is clamped (G = 1, N2 - G = N2 - 1; or G = N2 - 1, N2 - G = 1) or
     * degenerate (N2 = 2: mean 1, spread 0, G = 1) */
    int N2_cont = N_cont && N > 2.0;
    int G_cont, Gb_cont;
    if (x < 1.0 || N2 <= 2.0) {
        G_cont = 0;
        Gb_cont = N2_cont;
    } else if (x > N2 - 1.0) {
        G_cont = N2_cont;
        Gb_cont = 0;
    } else {
        G_cont = Gb_cont = 1;
    }
    o->n_cont = (B_nN && N2_cont) || (B_G && G_cont);
    o->nb_cont = (B_nbN && N2_cont) || (B_G && Gb_cont);
    o->code = (uint8_t)(B_nN | (B_n1N << 1) | (B_nbN << 2) | (B_nb1N << 3) | (B_G << 4));
    o->flag = gate_band_flag(&g, xi1) | ((round_flag(p) | (sym && round_flag(q))) << 1) |
              ((!N_exact && round_flag(N)) << 2);
}

/* Sec. 6 paragraphs "Single-Gated Gaussians" and "Gating Generalization".
 * form 1, Eq. (gated): one gate, passed with probability min(N p, P_any),
 * P_any = 1 - (1-p)^N, the power taken with the bias of paragraph "Numeric
 * Gating Issues" (the paper names the single gate among those it fixes):
 * (1 - max(p, eps))^(N min(1, p/eps)).  Past the gate the count is the
 * Gaussian of mean 1 + (N1-1) p and variance (N1-1) p (1-p), N1 = max(N, 1),
 * clamped to [1, N1] (so exactly 1 for N <= 1).
 * form 2, Eq. (oldgated), the prior form: gate probability P_any without
 * the bias and without the N < 1 generalisation, and the floor of the same
 * clamped Gaussian.
 * Both forms: the negative count is what remains, max(N - n, 0).  The gate
 * is evaluated in float, as the dual gate; the Gaussian in double. */
static void single_gated(int form, double N, double p, float xi1, float xi2, int N_exact, int N_cont,
                         node_out *o)
{
    const float eps = (float)EPS_GATE;
    float Nf = (float)N, pf = (float)p;
    float th;
    if (form == 1) {
        float cp = fmaxf(pf, eps);
        float ex = Nf * fminf(1.0f, pf / eps);
        float pany = 1.0f - powf(1.0f - cp, ex);
        float np = Nf * pf;
        th = np < pany ? np : pany;
    } else {
        th = 1.0f - powf(1.0f - pf, Nf);
    }
    int hit = xi1 < th;
    int gauss = hit && N > 1.0;
    double N1 = N > 1.0 ? N : 1.0;
    double n = hit ? 1.0 : 0.0;
    int fl = 0;
    if (gauss) {
        double mu = 1.0 + (N1 - 1.0) * p;
        double sig = sqrt((N1 - 1.0) * p * (1.0 - p));
        double x = mu + sig * orc_ppnd16((double)xi2);
        n = x < 1.0 ? 1.0 : (x > N1 ? N1 : x);
        if (form == 2) {
            /* the floor decides an integer: flag a Gaussian value (not a
             * clamp bound, which is exact) next to one */
            double d = fabs(x - floor(x + 0.5));
            double band = 8.0 * (nextafter(fabs(x), INFINITY) - fabs(x));
            fl |= (x > 1.0 && x < N1 && d < (band > 1e-5 ? band : 1e-5)) << 3;
            n = floor(n);
        }
    }
    double r = N - n;
    o->n = n;
    o->nb = r > 0.0 ? r : 0.0;
    /* past the gate: n is exact when clamped to a bound or floored (the
     * floor's own ambiguity is flagged above) */
    /* n: a gate constant, the floor (its own ambiguity flagged above) or a
     * clamp bound, else the draw; the rest N - n follows both (0 when n
     * reaches N) */
    o->n_cont = gauss && form != 2 && n != 1.0 && (n != N1 || N_cont);
    o->nb_cont = o->nb > 0.0 && (N_cont || o->n_cont);
    o->code = (uint8_t)(hit | (gauss << 4));
    double bandg = 9.5367431640625e-07 * (double)th + 5.9604644775390625e-08;
    fl |= fabs((double)xi1 - (double)th) <= bandg;
    o->flag = fl | (round_flag(p) << 1) | ((!N_exact && round_flag(N)) << 2);
}

/* The binomial approximation selected by `sampler`: 0 dual-gated (Alg.
 * "Dual-gated Gaussian"), 1 single-gated Eq. (gated), 2 Eq. (oldgated),
 * 3 dual-gated with the bias on both powers (q: the negative side's
 * probability, 1 - p in exact arithmetic). */
static void sample_node(int sampler, double N, double p, double q, float xi1, float xi2, int N_exact, int N_cont,
                        node_out *o)
{
    if (sampler == 0 || sampler == 3) dual_gated(N, p, q, sampler == 3, xi1, xi2, N_exact, N_cont, o);
    else single_gated(sampler, N, p, xi1, xi2, N_exact, N_cont, o);
}

/* A sampled count is "near an integer" if it lies within 1e-5 of one
 * without being one, or, for counts so large that a double's spacing
 * approaches that band (beyond ~1e10), within 8 units in the last place:
 * there the evaluation order alone moves a count by a few ulps.  A count
 * that varies with a Gaussian draw (node_out.n_cont) and is itself an
 * integer is near one too: another evaluation order lands just below it. */
static int near_int_flag(double v, int cont)
{
    double d = fabs(v - floor(v + 0.5));
    double band = 8.0 * (nextafter(fabs(v), INFINITY) - fabs(v));
    return (d > 0.0 || cont) && d < (band > 1e-5 ? band : 1e-5);
}

/* Sec. 6 (a multinomial drawn "hierarchically" from binomials), second
 * shape: a sequential chain.  Node i (0 <= i <= K-2) draws the facets of
 * bin i out of the N_i that reach it, with p_node = p_i / S_i, S_i the
 * suffix sum p_i + S_{i+1} (S_{K-1} = p_{K-1}, evaluated from the last bin
 * down), p_node = 0 when S_i = 0; bin i receives the positive count n and
 * the negative count nb goes on to node i+1 (N_0 = N_P); bin K-1 receives
 * what reaches it. */
static int multinomial_chain(int sampler, double NP, int root_exact, const double *p, int K, uint32_t seed,
                             uint32_t surf, uint32_t key, int64_t a, int64_t b, double *M, uint8_t *codes)
{
    double S[16];
    S[K - 1] = p[K - 1];
    for (int k = K - 2; k >= 0; --k) S[k] = p[k] + S[k + 1];
    double N = NP;
    int exact = root_exact, cont = 0, flag = 0;
    for (int i = 0; i < K - 1; ++i) {
        double pn = S[i] > 0.0 ? p[i] / S[i] : 0.0;
        if (pn > 1.0) pn = 1.0;
        double qn = S[i] > 0.0 ? S[i + 1] / S[i] : 0.0; /* the bins after i */
        if (qn > 1.0) qn = 1.0;
        float xi1, xi2;
        hash_xi_key(seed, surf, key, a, b, i, &xi1, &xi2);
        node_out o;
        sample_node(sampler, N, pn, qn, xi1, xi2, exact, cont, &o);
        codes[i] = o.code;
        flag |= o.flag;
        M[i] = o.n;
        flag |= near_int_flag(M[i], o.n_cont) << 3;
        N = o.nb;
        exact = exact && !(o.code & 16);
        cont = o.nb_cont;
    }
    M[K - 1] = N;
    flag |= near_int_flag(N, cont) << 3;
    return flag;
}

/* Sec. 6 (hierarchical multinomial from recursive binomials): balanced binary
 * tree over the K bins, nodes numbered breadth first (heap order); node i
 * splits [lo,hi) at the midpoint; the left child receives the positive count
 * n, the right child the negative count nb.  p_node = S_left / S_node.
 * tree = 1 selects the sequential chain above instead. */
static int multinomial(int sampler, int tree, double NP, int root_exact, const double *p, int K, uint32_t seed,
                       uint32_t surf, uint32_t key, int64_t a, int64_t b, double *M, uint8_t *codes)
{
    if (tree == 1) return multinomial_chain(sampler, NP, root_exact, p, K, seed, surf, key, a, b, M, codes);
    int nodes = K - 1;
    double Nn[32];
    int lo_[32], hi_[32], exact[32], cont[32];
    int flag = 0;
    /* exact[i]: node i's count is formed by exact operations on exact values
     * (the root product, then gating outcomes without a Gaussian draw);
     * cont[i]: it varies with a Gaussian draw's value (node_out). */
    Nn[0] = NP; lo_[0] = 0; hi_[0] = K; exact[0] = root_exact; cont[0] = 0;
    for (int i = 0; i < nodes; ++i) {
        int lo = lo_[i], hi = hi_[i], mid = lo + (hi - lo) / 2;
        double sl = 0.0, sr = 0.0;
        for (int k = lo; k < mid; ++k) sl += p[k];
        for (int k = mid; k < hi; ++k) sr += p[k];
        double st = sl + sr;
        double pn = st > 0.0 ? sl / st : 0.0;
        if (pn > 1.0) pn = 1.0;
        double qn = st > 0.0 ? sr / st : 0.0; /* the right child's share */
        if (qn > 1.0) qn = 1.0;
        float xi1, xi2;
        hash_xi_key(seed, surf, key, a, b, i, &xi1, &xi2);
        node_out o;
        sample_node(sampler, Nn[i], pn, qn, xi1, xi2, exact[i], cont[i], &o);
        codes[i] = o.code;
        flag |= o.flag;
        int c1 = 2 * i + 1, c2 = 2 * i + 2;
        Nn[c1] = o.n; lo_[c1] = lo; hi_[c1] = mid;
        Nn[c2] = o.nb; lo_[c2] = mid; hi_[c2] = hi;
        exact[c1] = exact[c2] = exact[i] && !(o.code & 16);
        cont[c1] = o.n_cont;
        cont[c2] = o.nb_cont;
    }
    /* leaves: heap slots nodes .. 2K-2 hold single bins, in order, for a
     * power-of-two K */
    for (int k = 0; k < K; ++k) {
        M[k] = Nn[nodes + k];
        flag |= near_int_flag(M[k], cont[nodes + k]) << 3;
    }
    return flag;
}

/* ------------------------------------------------------------------------ */
/* Pyramid lookup for shading (Sec. 5: the prefiltered map is read at the    */
/* reflection direction and the roughness lod).                              */
/* ------------------------------------------------------------------------ */
typedef struct {
    const float *pyr; /* mip-major [m][6][n][n][C] */
    int R, C;
} pyr_src;

static void pyr_texel_at(const pyr_src *src, int level, int face, int x, int y, double *out)
{
    int n = src->R >> level;
    const float *p = src->pyr + (level_offset(src->R, level) + ((int64_t)face * n + y) * n + x) * src->C;
    for (int k = 0; k < src->C; ++k) out[k] = (double)p[k];
}

static void pyr_texel(const void *srcv, int level, int face, int x, int y, double *out)
{
    const pyr_src *src = (const pyr_src *)srcv;
    int n = src->R >> level;
    int fo[3], xo[3], yo[3];
    int cnt = resolve_texel(face, x, y, n, fo, xo, yo);
    if (cnt == 1) { pyr_texel_at(src, level, fo[0], xo[0], yo[0], out); return; }
    double a[20], b[20], d[20];
    pyr_texel_at(src, level, fo[0], xo[0], yo[0], a);
    pyr_texel_at(src, level, fo[1], xo[1], yo[1], b);
    pyr_texel_at(src, level, fo[2], xo[2], yo[2], d);
    for (int k = 0; k < src->C; ++k) out[k] = ((a[k] + b[k]) + d[k]) / 3.0;
}

static double lut_bilinear(const float *lut, int stride, int comp, double mu, double sa)
{
    double x = mu * LUT_N - 0.5, y = sa * LUT_N - 0.5;
    if (x < 0.0) x = 0.0;
    if (x > LUT_N - 1) x = LUT_N - 1;
    if (y < 0.0) y = 0.0;
    if (y > LUT_N - 1) y = LUT_N - 1;
    double x0 = floor(x), y0 = floor(y);
    if (x0 > LUT_N - 2) x0 = LUT_N - 2;
    if (y0 > LUT_N - 2) y0 = LUT_N - 2;
    double fx = x - x0, fy = y - y0;
    int ix = (int)x0, iy = (int)y0;
#define LV(j, i) ((double)lut[((j) * LUT_N + (i)) * stride + comp])
    double top = (1.0 - fx) * LV(iy, ix) + fx * LV(iy, ix + 1);
    double bot = (1.0 - fx) * LV(iy + 1, ix) + fx * LV(iy + 1, ix + 1);
#undef LV
    return (1.0 - fy) * top + fy * bot;
}

/* Lattice of the footprint grid (Sec. 3.3, used as a black box by the
 * paper; reading: one uv lattice per footprint scale).  level0 =
 * floor(log2(area)/2), computed exactly from the binary exponent. */
static int lattice_level(double area, double *frac)
{
    int e;
    double m = frexp(area, &e); /* area = m 2^e, m in [0.5,1) */
    (void)m;
    int l0 = (e - 1) >= 0 ? (e - 1) / 2 : -((-(e - 1) + 1) / 2);
    double lam = 0.5 * log2(area);
    double t = lam - (double)l0;
    if (t < 0.0) t = 0.0;
    if (t > 1.0) t = 1.0;
    *frac = t;
    return l0;
}

typedef struct {
    const float *nx, *ny, *nz, *vx, *vy, *vz, *u, *v, *area, *ax, *ay, *density, *f0r, *f0g, *f0b;
    const uint32_t *surf;
    const float *vis; /* optional visibility in [0, 1] (NULL: unoccluded) */
    const float *tx, *ty, *tz; /* optional tangent (the alpha_x axis) */
    const float *dudx, *dudy, *dvdx, *dvdy; /* optional uv Jacobian of the pixel (footprint grid) */
} gbuf_t;

/* ------------------------------------------------------------------------ */
/* Footprint grid (Sec. 3.3, "Binomial Sampling with Anisotropic Grids"):    */
/* the pixel footprint is described by its length, anisotropy and            */
/* orientation; its microfacets are distributed over the vertices of the     */
/* tetrahedral cell around it in that space, and at each such vertex a       */
/* triangle grid in uv interpolates the outcomes drawn at its vertices.      */
/* The layout is this library's (the paper treats the grid as a black box):  */
/*  - footprint: ellipse of J J^T, J = [[du/dx, du/dy], [dv/dx, dv/dy]]:      */
/*    length s_maj = sqrt(largest eigenvalue), s_min = |det J| / s_maj,       */
/*    clamped to s_maj / 16, anisotropy A = s_maj / s_min in [1, 16],         */
/*    orientation theta of the major axis in [0, pi);                         */
/*  - grid coordinates g = (log2 s_maj, log2 A, 8 theta / pi), orientation    */
/*    periodic with 8 cells; Kuhn cell: axes sorted by decreasing fraction    */
/*    (ties in axis order), weights (1 - f1, f1 - f2, f2 - f3, f3);            */
/*  - vertex (l, a, o): footprint of length 2^l, anisotropy 2^a, orientation */
/*    o pi / 8; its count is N_P times the ratio of its uv area 4^l / 2^a to  */
/*    the pixel's s_maj s_min;                                                */
/*  - uv triangle grid of that vertex: uv rotated by -theta_o and scaled by   */
/*    (2^-l, 2^(a-l)) (one cell per footprint), unit squares split along the  */
/*    diagonal, barycentric weights;                                          */
/*  - random numbers keyed by (lattice x, lattice y, l, a, o).                */
/* 12 draws per pixel; the output is normalised by the weighted count         */
/* sum_i w_i N_i.  flag: a cell, triangle or ordering decision within 1e-9    */
/* of its boundary (implementations may decide differently there).           */
/* ------------------------------------------------------------------------ */
#define FG_ORIENT 8
#define FG_AMAX 16.0

typedef struct {
    int valid, flag;
    double w[12], r[12];
    uint32_t key[12];
    int64_t a[12], b[12];
} fgrid_t;

static int near_int_1e9(double x)
{
    return fabs(x - floor(x + 0.5)) < 1e-9 * (1.0 + fabs(x));
}

static void footprint_grid(double uu, double vv, double j00, double j01, double j10, double j11, fgrid_t *G)
{
    double m11 = j00 * j00 + j01 * j01, m22 = j10 * j10 + j11 * j11, m12 = j00 * j10 + j01 * j11;
    double h = 0.5 * (m11 - m22);
    double disc = sqrt(h * h + m12 * m12);
    double smaj = sqrt(0.5 * (m11 + m22) + disc);
    G->flag = 0;
    G->valid = isfinite(smaj) && smaj > 1e-12;
    if (!G->valid) return;
    double smin = fabs(j00 * j11 - j01 * j10) / smaj;
    int clamped = !(smin > smaj / FG_AMAX);
    double sminc = clamped ? smaj / FG_AMAX : smin;
    double A = smaj / sminc;
    double th = 0.5 * atan2(2.0 * m12, m11 - m22);
    if (th < 0.0) th += M_PI;
    /* a clamped anisotropy is exactly log2(16) = 4 on every implementation */
    double g[3] = {log2(smaj), clamped ? 4.0 : log2(A), th * ((double)FG_ORIENT / M_PI)};
    int base[3];
    double f[3];
    for (int c = 0; c < 3; ++c) {
        double fl = floor(g[c]);
        base[c] = (int)fl;
        f[c] = g[c] - fl;
        if (!(c == 1 && clamped)) G->flag |= near_int_1e9(g[c]);
    }
    int ord[3] = {0, 1, 2};
    for (int i = 1; i < 3; ++i)
        for (int j = i; j > 0 && f[ord[j]] > f[ord[j - 1]]; --j) {
            int t = ord[j]; ord[j] = ord[j - 1]; ord[j - 1] = t;
        }
    G->flag |= fabs(f[ord[0]] - f[ord[1]]) < 1e-9 || fabs(f[ord[1]] - f[ord[2]]) < 1e-9;
    double wt[4] = {1.0 - f[ord[0]], f[ord[0]] - f[ord[1]], f[ord[1]] - f[ord[2]], f[ord[2]]};
    int cv[3] = {base[0], base[1], base[2]};
    for (int i = 0; i < 4; ++i) {
        if (i > 0) cv[ord[i - 1]] += 1;
        int l = cv[0], ai = cv[1], o = ((cv[2] % FG_ORIENT) + FG_ORIENT) % FG_ORIENT;
        double li = ldexp(1.0, l), Ai = ldexp(1.0, ai), thi = (double)o * (M_PI / (double)FG_ORIENT);
        double ratio = (li * li / Ai) / (smaj * sminc);
        uint32_t key = (((uint32_t)l & 0xFFu) << 24) | (((uint32_t)ai & 0xFu) << 20) | (((uint32_t)o & 0xFu) << 16);
        double cs = cos(thi), sn = sin(thi);
        double X = (cs * uu + sn * vv) / li;
        double Y = (cs * vv - sn * uu) * Ai / li;
        double fxl = floor(X), fyl = floor(Y);
        double fx = X - fxl, fy = Y - fyl;
        G->flag |= near_int_1e9(X) | near_int_1e9(Y) | (fabs(fx - fy) < 1e-9);
        int64_t ix = (int64_t)fxl, iy = (int64_t)fyl;
        for (int c = 0; c < 3; ++c) {
            int64_t a, b;
            double bw;
            if (fx >= fy) {
                if (c == 0) { a = ix; b = iy; bw = 1.0 - fx; }
                else if (c == 1) { a = ix + 1; b = iy; bw = fx - fy; }
                else { a = ix + 1; b = iy + 1; bw = fy; }
            } else {
                if (c == 0) { a = ix; b = iy; bw = 1.0 - fy; }
                else if (c == 1) { a = ix; b = iy + 1; bw = fy - fx; }
                else { a = ix + 1; b = iy + 1; bw = fx; }
            }
            G->w[3 * i + c] = wt[i] * bw;
            G->r[3 * i + c] = ratio;
            G->key[3 * i + c] = key;
            G->a[3 * i + c] = a;
            G->b[3 * i + c] = b;
        }
    }
}

/* Anisotropic lookup: the future work of Sec. 8 (several samples of the
 * prefiltered map for anisotropic distributions) as this library designs
 * it.  T taps of isotropic roughness a_t = max(a_min, a_max / T) lie along
 * the lobe's major axis at the stratified quantiles u_j = (2j+1)/T - 1 of
 * the GGX slope marginal of scale s = sqrt(a_max^2 - a_t^2): slope
 * x_j = s u_j / sqrt(1 - u_j^2), microfacet normal
 * h_j = (n - x_j d) / sqrt(1 + x_j^2),
 * direction w_j = 2 <v, h_j> h_j - v, read at lod sqrt(a_t)(M-1); the taps
 * are averaged with weights <n, w_j>+ (the cosine of the filter kernel,
 * whose half vectors the quantiles stand for).  d is the tangent made
 * orthogonal to n (the alpha_x axis),
 * or n x d when alpha_y > alpha_x; a tangent parallel to n is replaced by
 * the first axis of the frame onb(n). */
static void aniso_lookup(const pyr_src *ind, const pyr_src *rgbs, int R, int M, int K, int T, int read_ind,
                         const double n[3], const double v[3], const double t[3], double ax, double ay, double *F,
                         double *rgb)
{
    double tn = t[0] * n[0] + t[1] * n[1] + t[2] * n[2];
    double tt[3] = {t[0] - tn * n[0], t[1] - tn * n[1], t[2] - tn * n[2]};
    double tl = sqrt(tt[0] * tt[0] + tt[1] * tt[1] + tt[2] * tt[2]);
    if (tl > 1e-12) {
        for (int c = 0; c < 3; ++c) tt[c] /= tl;
    } else {
        double b2[3];
        onb(n, tt, b2);
    }
    double bt[3] = {n[1] * tt[2] - n[2] * tt[1], n[2] * tt[0] - n[0] * tt[2], n[0] * tt[1] - n[1] * tt[0]};
    double amin = ax < ay ? ax : ay, amax = ax < ay ? ay : ax;
    const double *d = ax >= ay ? tt : bt;
    double at = amax / (double)T;
    if (at < amin) at = amin;
    double s2 = amax * amax - at * at;
    double s = s2 > 0.0 ? sqrt(s2) : 0.0;
    double lod = sqrt(at) * (double)(M - 1);
    for (int k = 0; k < K; ++k) F[k] = 0.0;
    for (int c = 0; c < 4; ++c) rgb[c] = 0.0;
    double wsum = 0.0;
    for (int j = 0; j < T; ++j) {
        double u = (double)(2 * j + 1) / (double)T - 1.0;
        double x = s * u / sqrt(1.0 - u * u);
        /* n and d are orthonormal, so |n - x d| = sqrt(1 + x^2) */
        double hl = sqrt(1.0 + x * x);
        double h[3] = {(n[0] - x * d[0]) / hl, (n[1] - x * d[1]) / hl, (n[2] - x * d[2]) / hl};
        double vh = v[0] * h[0] + v[1] * h[1] + v[2] * h[2];
        double w[3] = {2.0 * vh * h[0] - v[0], 2.0 * vh * h[1] - v[1], 2.0 * vh * h[2] - v[2]};
        double cw = w[0] * n[0] + w[1] * n[1] + w[2] * n[2];
        cw = cw > 0.0 ? cw : 0.0;
        double fj[20], cj[4];
        if (read_ind) {
            trilinear(pyr_texel, ind, R, M, K, w, lod, fj);
            for (int k = 0; k < K; ++k) F[k] += cw * fj[k];
        }
        trilinear(pyr_texel, rgbs, R, M, 4, w, lod, cj);
        for (int c = 0; c < 4; ++c) rgb[c] += cw * cj[c];
        wsum += cw;
    }
    if (wsum > 0.0) { /* else every tap is below the horizon: nothing reflected */
        for (int k = 0; k < K; ++k) F[k] /= wsum;
        for (int c = 0; c < 4; ++c) rgb[c] /= wsum;
    }
}

/* Shades the requested pixels.  Outputs (double): radiance [n][3], counts
 * [n][V][K], probs [n][K]; codes [n][V][K-1]; flags [n], a bit mask of the
 * reasons a conforming implementation may take a different discrete branch
 * or integer part on this pixel: 1 = xi1 within the tolerance band of a
 * float gating threshold, 2 = a node probability on a float rounding
 * boundary, 4 = a node count on a float rounding boundary, 8 = a sampled
 * count within 1e-5 of an integer (without being one), 16 = a footprint
 * grid decision (cell, ordering, triangle) within 1e-9 of its boundary. */
static int shade_impl(const float *const *gb, const float *ind_pyr, const float *rgb_pyr, const double *levels,
                      const float *lut_S, const float *lut_E, int R, int K, int M, uint32_t seed, int V,
                      int sampler, int tree, int prob_mode, double gamma, int lobe_taps, const int64_t *pix, int64_t count,
                      const double *Fext, double *radiance, double *counts, uint8_t *codes, double *probs,
                      uint8_t *flags, int threads)
{
    if (R < 1 || K < 2 || K > 16 || (K & (K - 1)) || M < 1 || (R >> (M - 1)) < 1 || (V != 1 && V != 6 && V != 12) ||
        (V == 12 && (!gb[20] || !gb[21] || !gb[22] || !gb[23])) ||
        sampler < 0 || sampler > 3 || tree < 0 || tree > 1 || prob_mode < 0 || prob_mode > 1 ||
        (prob_mode == 1 && !(gamma > 0.0 && gamma <= 1.0)) ||
        !(lobe_taps == 0 || lobe_taps == 2 || lobe_taps == 4 || lobe_taps == 8) ||
        (lobe_taps && (!gb[17] || !gb[18] || !gb[19])))
        return ORC_EINVAL;
    gbuf_t g = {gb[0], gb[1], gb[2], gb[3], gb[4], gb[5], gb[6], gb[7], gb[8], gb[9], gb[10], gb[11],
                gb[12], gb[13], gb[14], (const uint32_t *)gb[15], gb[16], gb[17], gb[18], gb[19],
                gb[20], gb[21], gb[22], gb[23]};
    /* prob_mode 1 (the comparison of Sec. 7 "Comparison with Previous Work",
     * after Wang et al. 2020): every facet reflects with one probability
     * gamma, independent of the map; this is the two-bin case of the same
     * machinery with p = (1 - gamma, gamma) and levels (0, 1). */
    if (prob_mode == 1) K = 2;
    static const double unit_levels[2] = {0.0, 1.0};
    if (prob_mode == 1) levels = unit_levels;
    pyr_src ps_ind = {ind_pyr, R, K};
    pyr_src ps_rgb = {rgb_pyr, R, 4};
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 256) num_threads(threads > 0 ? threads : 1)
#endif
    for (int64_t q = 0; q < count; ++q) {
        int64_t i = pix[q];
        double *rad = radiance + 3 * q;
        double *cnt = counts ? counts + q * V * K : NULL;
        uint8_t *cod = codes ? codes + q * V * (K - 1) : NULL;
        double *pr = probs ? probs + q * K : NULL;
        rad[0] = rad[1] = rad[2] = 0.0;
        if (cnt) for (int k = 0; k < V * K; ++k) cnt[k] = 0.0;
        if (cod) memset(cod, 0, (size_t)V * (K - 1));
        if (pr) for (int k = 0; k < K; ++k) pr[k] = 0.0;
        flags[q] = 0;
        uint32_t surf = g.surf[i];
        if (surf == 0xFFFFFFFFu) continue;
        /* Sec. 3.2: stratified count N_P = N |P|. */
        double NP = (double)g.density[i] * (double)g.area[i];
        double n[3] = {g.nx[i], g.ny[i], g.nz[i]}, v[3] = {g.vx[i], g.vy[i], g.vz[i]};
        double mu = n[0] * v[0] + n[1] * v[1] + n[2] * v[2];
        double wr[3];
        for (int c = 0; c < 3; ++c) wr[c] = 2.0 * mu * n[c] - v[c];
        double aeff = sqrt((double)g.ax[i] * (double)g.ay[i]);
        double sa = sqrt(aeff);
        double lod = sa * (double)(M - 1);
        /* Sec. 4 Eq. (probhk) with Sec. 5 Eq. (rtiblndf): p_k = S F_k / sum F for
         * k >= 2 (one-based); the zero-radiance bin absorbs the rest. */
        double F[20], rgb[4];
        if (lobe_taps) {
            double t[3] = {g.tx[i], g.ty[i], g.tz[i]};
            aniso_lookup(&ps_ind, &ps_rgb, R, M, K, lobe_taps, prob_mode == 0 && !Fext, n, v, t, (double)g.ax[i],
                         (double)g.ay[i], F, rgb);
            if (prob_mode == 0 && Fext)
                for (int k = 0; k < K; ++k) F[k] = Fext[q * K + k];
        } else {
            if (prob_mode == 0) {
                if (Fext)
                    for (int k = 0; k < K; ++k) F[k] = Fext[q * K + k];
                else
                    trilinear(pyr_texel, &ps_ind, R, M, K, wr, lod, F);
            }
            trilinear(pyr_texel, &ps_rgb, R, M, 4, wr, lod, rgb);
        }
        double A = lut_bilinear(lut_E, 2, 0, mu, sa);
        double B = lut_bilinear(lut_E, 2, 1, mu, sa);
        /* Sec. 8 "Limitations & Future Work": occlusion attenuates the
         * reflection probabilities rather than the output.  A visibility v
         * scales p_k (k >= 1); occluded facets join bin 0.  The normalisation
         * below keeps the unattenuated p, so the expected output is v times
         * the smooth radiance while each glint keeps its brightness. */
        double vis = g.vis ? (double)g.vis[i] : 1.0;
        double p[16], pa[16];
        double rest = 0.0;
        if (prob_mode == 1) {
            p[1] = gamma;
        } else {
            double sumF = 0.0;
            for (int k = 0; k < K; ++k) sumF += F[k];
            double S = lut_bilinear(lut_S, 1, 0, mu, sa);
            for (int k = 1; k < K; ++k) p[k] = sumF > 0.0 ? S * F[k] / sumF : 0.0;
        }
        for (int k = 1; k < K; ++k) {
            pa[k] = p[k] * vis;
            rest += pa[k];
        }
        pa[0] = 1.0 - rest;
        if (pr) for (int k = 0; k < K; ++k) pr[k] = pa[k];
        /* Sec. 3.3 Eq. (anisogrid): weighted sum of independent multinomial
         * draws at lattice vertices; vertices 1 and 6 draw N_i = N_P, the
         * footprint grid (12) its vertices' own counts. */
        double lt;
        int l0 = lattice_level((double)g.area[i], &lt);
        double Msum[16] = {0};
        int flag = 0;
        double uu = (double)g.u[i], vv = (double)g.v[i];
        fgrid_t fg;
        double Nbar = NP; /* the normalisation's count */
        if (V == 12) {
            footprint_grid(uu, vv, g.dudx[i], g.dudy[i], g.dvdx[i], g.dvdy[i], &fg);
            if (!fg.valid) { /* no footprint: nothing is drawn */
                flags[q] = 0;
                continue;
            }
            flag |= fg.flag << 4;
            Nbar = 0.0;
            for (int vi = 0; vi < 12; ++vi) Nbar += fg.w[vi] * (NP * fg.r[vi]);
        }
        for (int vi = 0; vi < V; ++vi) {
            int lev = 0;
            int64_t a, b;
            double w;
            double Nv = NP;
            uint32_t key;
            if (V == 12) {
                w = fg.w[vi];
                Nv = NP * fg.r[vi];
                key = fg.key[vi];
                a = fg.a[vi];
                b = fg.b[vi];
            } else if (V == 1) {
                lev = l0;
                a = (int64_t)floor(ldexp(uu, -lev) + 0.5);
                b = (int64_t)floor(ldexp(vv, -lev) + 0.5);
                w = 1.0;
            } else {
                int side = vi / 3, corner = vi % 3;
                lev = l0 + side;
                double x = ldexp(uu, -lev), y = ldexp(vv, -lev);
                double fxl = floor(x), fyl = floor(y);
                double fx = x - fxl, fy = y - fyl;
                int64_t ix = (int64_t)fxl, iy = (int64_t)fyl;
                double bw;
                if (fx >= fy) {
                    if (corner == 0) { a = ix; b = iy; bw = 1.0 - fx; }
                    else if (corner == 1) { a = ix + 1; b = iy; bw = fx - fy; }
                    else { a = ix + 1; b = iy + 1; bw = fy; }
                } else {
                    if (corner == 0) { a = ix; b = iy; bw = 1.0 - fy; }
                    else if (corner == 1) { a = ix; b = iy + 1; bw = fy - fx; }
                    else { a = ix + 1; b = iy + 1; bw = fx; }
                }
                w = (side == 0 ? 1.0 - lt : lt) * bw;
            }
            if (V != 12) key = ((uint32_t)lev & 0xFFFFu) << 16;
            double Mv[16];
            uint8_t cv[16];
            flag |= multinomial(sampler, tree, Nv, V != 12, pa, K, seed, surf, key, a, b, Mv, cv);
            for (int k = 0; k < K; ++k) Msum[k] += w * Mv[k];
            if (cnt) for (int k = 0; k < K; ++k) cnt[vi * K + k] = Mv[k];
            if (cod) for (int k = 0; k < K - 1; ++k) cod[vi * (K - 1) + k] = cv[k];
        }
        /* Sec. 4 Eq. (iblglints:fin). */
        double num = 0.0, den = 0.0;
        for (int k = 0; k < K; ++k) num += levels[k] * Msum[k];
        for (int k = 1; k < K; ++k) den += levels[k] * p[k];
        den *= Nbar;
        double gmod = (num > 0.0 && den > 0.0) ? num / den : 0.0;
        const float *f0[3] = {g.f0r, g.f0g, g.f0b};
        for (int c = 0; c < 3; ++c) {
            double Erho = (double)f0[c][i] * A + B;
            rad[c] = Erho * rgb[c] * gmod;
        }
        flags[q] = (uint8_t)flag;
    }
    (void)threads;
    return ORC_OK;
}

int orc_shade_pixels(const float *const *gb, const float *ind_pyr, const float *rgb_pyr, const double *levels,
                     const float *lut_S, const float *lut_E, int R, int K, int M, uint32_t seed, int V, int sampler,
                     int tree, int prob_mode, double gamma, int lobe_taps, const int64_t *pix, int64_t count,
                     double *radiance, double *counts, uint8_t *codes, double *probs, uint8_t *flags, int threads)
{
    return shade_impl(gb, ind_pyr, rgb_pyr, levels, lut_S, lut_E, R, K, M, seed, V, sampler, tree, prob_mode, gamma,
                      lobe_taps, pix, count, NULL, radiance, counts, codes, probs, flags, threads);
}

/* As orc_shade_pixels, with the K filtered indicator values of each requested
 * pixel given (F [count][K], e.g. a learned surrogate's output) instead of
 * read from the indicator pyramid; RGB still comes from the RGB pyramid.
 * ind_pyr is not read. */
int orc_shade_pixels_given_F(const float *const *gb, const double *F, const float *rgb_pyr, const double *levels,
                             const float *lut_S, const float *lut_E, int R, int K, int M, uint32_t seed, int V,
                             int sampler, int tree, const int64_t *pix, int64_t count, double *radiance,
                             double *counts, uint8_t *codes, double *probs, uint8_t *flags, int threads)
{
    if (!F) return ORC_EINVAL;
    return shade_impl(gb, NULL, rgb_pyr, levels, lut_S, lut_E, R, K, M, seed, V, sampler, tree, 0, 1.0, 0, pix,
                      count, F,
                      radiance, counts, codes, probs, flags, threads);
}

/* Exposed pieces for the definition tests. */
void orc_gate_probs(float N, float p, float *out4)
{
    gate_t g;
    gate_probs(N, p, 1.0f - p, 0, &g);
    out4[0] = g.P_nN; out4[1] = g.P_n1; out4[2] = g.P_nbN; out4[3] = g.P_nb1;
}

/* The gating probabilities with the bias on both powers (q given). */
void orc_gate_probs_symmetric(float N, float p, float q, float *out4)
{
    gate_t g;
    gate_probs(N, p, q, 1, &g);
    out4[0] = g.P_nN; out4[1] = g.P_n1; out4[2] = g.P_nbN; out4[3] = g.P_nb1;
}

void orc_dual_gated(double N, double p, float xi1, float xi2, double *n, double *nb, uint8_t *code)
{
    node_out o;
    dual_gated(N, p, 1.0 - p, 0, xi1, xi2, 0, 1, &o);
    *n = o.n; *nb = o.nb; *code = o.code;
}

/* The hierarchical multinomial of one draw (Sec. 6) on given probabilities
 * p[K] (K a power of two <= 16): leaf counts M[K], node codes[K-1]; returns
 * the draw's flags (bit 8: a count near an integer). */
int orc_multinomial(int sampler, int tree, double NP, const double *p, int K, uint32_t seed, uint32_t surf,
                    int32_t level, int64_t a, int64_t b, double *M, uint8_t *codes)
{
    if (sampler < 0 || sampler > 3 || tree < 0 || tree > 1 || K < 2 || K > 16 || (tree == 0 && (K & (K - 1))))
        return -1;
    return multinomial(sampler, tree, NP, 1, p, K, seed, surf, ((uint32_t)level & 0xFFFFu) << 16, a, b, M, codes);
}

/* One binomial draw per element with the given random words: xi1 from h1,
 * xi2 from h2 (as the hash outputs are mapped).  N and p are inputs, so
 * their float roundings are shared; flags keep bits 1 (gate band) and 8
 * (floor next to an integer). */
int orc_sample_binomial(int sampler, const double *N, const double *p, const uint32_t *h1, const uint32_t *h2,
                        int64_t count, double *n, double *nb, uint8_t *code, uint8_t *flags, int threads)
{
    if (sampler < 0 || sampler > 3 || count < 0) return ORC_EINVAL;
#ifdef _OPENMP
#pragma omp parallel for schedule(static) num_threads(threads > 0 ? threads : 1)
#endif
    for (int64_t i = 0; i < count; ++i) {
        node_out o;
        sample_node(sampler, N[i], p[i], 1.0 - p[i], to_unit(h1[i]), to_unit(h2[i]), 1, 0, &o);
        n[i] = o.n;
        nb[i] = o.nb;
        code[i] = o.code;
        flags[i] = (uint8_t)(o.flag & 9);
    }
    (void)threads;
    return ORC_OK;
}

/* The footprint grid's 12 draws of one pixel (weights, count ratios, hash
 * keys, lattice vertices); returns -1 for a degenerate Jacobian, else the
 * boundary flag. */
int orc_footprint_grid(double u, double v, double j00, double j01, double j10, double j11, double *w, double *r,
                       uint32_t *key, int64_t *a, int64_t *b)
{
    fgrid_t G;
    footprint_grid(u, v, j00, j01, j10, j11, &G);
    if (!G.valid) return -1;
    for (int i = 0; i < 12; ++i) {
        w[i] = G.w[i]; r[i] = G.r[i]; key[i] = G.key[i]; a[i] = G.a[i]; b[i] = G.b[i];
    }
    return G.flag;
}

void orc_face_dir(int face, double s, double t, double *d) { face_to_dir(face, s, t, d); }
int orc_dir_face(const double *d, double *st)
{
    return dir_to_face(d, &st[0], &st[1]);
}

int orc_lattice_level(double area, double *frac) { return lattice_level(area, frac); }

void orc_taps(int m, int M, int T, int R, double *out5)
{
    tap_t *t = (tap_t *)malloc(sizeof(tap_t) * (size_t)T);
    make_taps(m, M, T, R, t);
    for (int j = 0; j < T; ++j) {
        out5[5 * j + 0] = t[j].hx; out5[5 * j + 1] = t[j].hy; out5[5 * j + 2] = t[j].hz;
        out5[5 * j + 3] = t[j].w; out5[5 * j + 4] = t[j].lod;
    }
    free(t);
}

/* Trilinear lookup of a float pyramid (mip-major, C channels per texel) at
 * the given directions and lods: the addressing used by the filter's taps
 * and by shading.  out: [count][C]. */
void orc_pyramid_lookup(const float *pyr, int R, int M, int C, const double *dirs, const double *lods,
                        int64_t count, double *out)
{
    pyr_src ps = {pyr, R, C};
    for (int64_t q = 0; q < count; ++q) trilinear(pyr_texel, &ps, R, M, C, dirs + 3 * q, lods[q], out + q * C);
}

/* The filter of Eq. (rtiblndf) evaluated at arbitrary (direction, alpha):
 * the same quadrature as the pyramid's mips, at a continuous roughness.
 * Training targets of the learned surrogate and the reference its error and
 * the pyramid's interpolation error are measured against.  out: [n][K+3]. */
int orc_sample_filter(const float *env, const uint8_t *ind_j, const float *ind_t, const float *chain, int R, int K,
                      int M, int T, const double *dirs, const double *alphas, int64_t count, double *out, int threads)
{
    if (R < 1 || K < 2 || K > 16 || M < 1 || (R >> (M - 1)) < 1 || T < 1) return ORC_EINVAL;
    src_chain c = {env, ind_j, ind_t, chain, R, K, M};
    int C = K + 3;
    int bad = 0;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 16) num_threads(threads > 0 ? threads : 1) reduction(| : bad)
#endif
    for (int64_t q = 0; q < count; ++q) {
        double alpha = alphas[q];
        if (!(alpha > 0.0)) { bad = 1; continue; }
        tap_t taps[1024];
        if (T > 1024) { bad = 1; continue; }
        make_taps_alpha(alpha, M, T, R, taps);
        double r[3] = {dirs[3 * q], dirs[3 * q + 1], dirs[3 * q + 2]};
        double len = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
        r[0] /= len; r[1] /= len; r[2] /= len;
        filter_dir(&c, T, r, taps, out + q * C);
    }
    (void)threads;
    return bad ? ORC_EINVAL : ORC_OK;
}
