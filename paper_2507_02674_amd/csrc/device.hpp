// Device-side building blocks of the glint kernels (gfx950).
//
// Cube addressing, seam handling, the pcg4d hash, the AS 241 inverse normal
// CDF and the float gating probabilities of the dual-gated Gaussian.  Every
// routine is evaluated in double except the gating (float, the precision the
// paper tunes its bias constant for, Sec. 6 "Numeric Gating Issues").
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace glint {

constexpr int kLutN = 64;

struct d3 {
    double x, y, z;
};

// Orthonormal frame (t1, t2) around the unit vector r (branchless form of
// Duff et al. 2017).
__device__ __forceinline__ void onb(const d3 &r, d3 &t1, d3 &t2)
{
    const double sgn = copysign(1.0, r.z);
    const double ea = -1.0 / (sgn + r.z);
    const double eb = r.x * r.y * ea;
    t1 = {1.0 + sgn * r.x * r.x * ea, sgn * eb, -sgn * r.x};
    t2 = {eb, sgn + r.y * r.y * ea, -r.y};
}

// Direction of face coordinates (s, t) in [-1,1]^2 (unnormalised).
__device__ __forceinline__ d3 face_dir(int face, double s, double t)
{
    switch (face) {
    case 0: return {1.0, -t, -s};
    case 1: return {-1.0, -t, s};
    case 2: return {s, 1.0, t};
    case 3: return {s, -1.0, -t};
    case 4: return {s, -t, 1.0};
    default: return {-s, -t, -1.0};
    }
}

// Owning face of d (largest |component|, ties to x then y) and its face
// coordinates.  The major axis is chosen first so only two (IEEE, correctly
// rounded) double divisions are emitted; negation is exact, so the
// quotients equal the per-face formulas.
__device__ __forceinline__ int dir_face(const d3 &d, double &s, double &t)
{
    const double ax = fabs(d.x), ay = fabs(d.y), az = fabs(d.z);
    int face;
    double ma, sc, tc;
    if (ax >= ay && ax >= az) {
        face = d.x >= 0.0 ? 0 : 1;
        ma = ax;
        sc = d.x >= 0.0 ? -d.z : d.z;
        tc = -d.y;
    } else if (ay >= az) {
        face = d.y >= 0.0 ? 2 : 3;
        ma = ay;
        sc = d.x;
        tc = d.y >= 0.0 ? d.z : -d.z;
    } else {
        face = d.z >= 0.0 ? 4 : 5;
        ma = az;
        sc = d.z >= 0.0 ? d.x : -d.x;
        tc = -d.y;
    }
    s = sc / ma;
    t = tc / ma;
    return face;
}

__host__ __device__ __forceinline__ int64_t level_offset(int R, int level)
{
    int64_t off = 0;
    for (int s = 0; s < level; ++s) {
        const int64_t n = R >> s;
        off += 6 * n * n;
    }
    return off;
}

// Seams.  A bilinear footprint reaches at most one texel beyond a face.  A
// texel off one edge is re-projected through the 3-D direction of its
// extended centre to the nearest texel of the owning face (the adjacent
// texel across the edge); the texel off two edges (beyond a cube corner)
// is the mean of the three texels meeting at that corner.  This keeps the
// lookup continuous across edges and corners.

__device__ __forceinline__ int64_t reproject_one(int face, int x, int y, int n)
{
    const double inv = ldexp(1.0, -__builtin_ctz((unsigned)n)); // 1/n, exact for n a power of two
    const d3 d = face_dir(face, 2.0 * ((double)x + 0.5) * inv - 1.0, 2.0 * ((double)y + 0.5) * inv - 1.0);
    double s, t;
    const int f2 = dir_face(d, s, t);
    int a = (int)floor((s + 1.0) * 0.5 * (double)n);
    int b = (int)floor((t + 1.0) * 0.5 * (double)n);
    a = a < 0 ? 0 : (a > n - 1 ? n - 1 : a);
    b = b < 0 ? 0 : (b > n - 1 ? n - 1 : b);
    return ((int64_t)f2 * n + b) * n + a;
}

// The same re-projection for a texel one step beyond an edge, in integer
// form (the shading lookup's footprints cross edges often; the filter keeps
// the form above, which measures faster in its kernel).
// Scaled by n, the extended texel centre's direction has integer
// components (face_dir with s = 2x+1-n, t = 2y+1-n and the major axis n),
// so its owning face and texel follow exactly from integer arithmetic
// (floor((num + den) n / (2 den)); the quotient is never an integer there,
// so a floating-point evaluation of the same steps lands on the same
// texel).  The result is affine in the position i along the
// edge: texel (a1 i + an (n-1), b1 i + bn (n-1)) of face f2.  The 24 maps
// (face, edge: 0 x = -1, 1 x = n, 2 y = -1, 3 y = n) are derived here at
// compile time from this file's cube convention.
struct EdgeMap {
    int f2, a1, an, b1, bn;
};

struct EdgeTexel {
    int f2, a, b;
};

constexpr EdgeTexel edge_texel_int(int face, int x, int y, long n)
{
    const long s = 2 * x + 1 - n, t = 2 * y + 1 - n, m = n;
    long d[3] = {0, 0, 0};
    switch (face) { // face_dir, scaled by n
    case 0: d[0] = m; d[1] = -t; d[2] = -s; break;
    case 1: d[0] = -m; d[1] = -t; d[2] = s; break;
    case 2: d[0] = s; d[1] = m; d[2] = t; break;
    case 3: d[0] = s; d[1] = -m; d[2] = -t; break;
    case 4: d[0] = s; d[1] = -t; d[2] = m; break;
    default: d[0] = -s; d[1] = -t; d[2] = -m; break;
    }
    const long ax = d[0] < 0 ? -d[0] : d[0], ay = d[1] < 0 ? -d[1] : d[1], az = d[2] < 0 ? -d[2] : d[2];
    int f2 = 0;
    long ma = 1, sc = 0, tc = 0;
    if (ax >= ay && ax >= az) { // dir_face, numerators over the major magnitude
        f2 = d[0] >= 0 ? 0 : 1; ma = ax; sc = d[0] >= 0 ? -d[2] : d[2]; tc = -d[1];
    } else if (ay >= az) {
        f2 = d[1] >= 0 ? 2 : 3; ma = ay; sc = d[0]; tc = d[1] >= 0 ? d[2] : -d[2];
    } else {
        f2 = d[2] >= 0 ? 4 : 5; ma = az; sc = d[2] >= 0 ? d[0] : -d[0]; tc = -d[1];
    }
    long a = (sc + ma) * n / (2 * ma), b = (tc + ma) * n / (2 * ma); // numerators >= 0: floor
    a = a < 0 ? 0 : (a > n - 1 ? n - 1 : a);
    b = b < 0 ? 0 : (b > n - 1 ? n - 1 : b);
    return {f2, (int)a, (int)b};
}

constexpr EdgeMap derive_edge_map(int face, int e)
{
    const long n = 8; // the maps are affine in i; two positions fix them
    const int x0 = e == 0 ? -1 : (e == 1 ? (int)n : 0), y0 = e == 2 ? -1 : (e == 3 ? (int)n : 0);
    const int x1 = e <= 1 ? x0 : 1, y1 = e <= 1 ? 1 : y0;
    const EdgeTexel p = edge_texel_int(face, x0, y0, n), q = edge_texel_int(face, x1, y1, n);
    const int a1 = q.a - p.a, b1 = q.b - p.b;
    return {p.f2, a1, p.a / (int)(n - 1), b1, p.b / (int)(n - 1)};
}

struct EdgeMaps {
    EdgeMap m[24];
};

constexpr EdgeMaps derive_edge_maps()
{
    EdgeMaps t{};
    for (int f = 0; f < 6; ++f)
        for (int e = 0; e < 4; ++e) t.m[4 * f + e] = derive_edge_map(f, e);
    return t;
}

constexpr EdgeMaps kEdgeMaps = derive_edge_maps();

// a self-check of the affine form at another size
constexpr bool edge_maps_consistent()
{
    for (int f = 0; f < 6; ++f)
        for (int e = 0; e < 4; ++e)
            for (int i = 0; i < 32; ++i) {
                const long n = 32;
                const int x = e == 0 ? -1 : (e == 1 ? (int)n : i), y = e == 2 ? -1 : (e == 3 ? (int)n : i);
                const EdgeTexel r = edge_texel_int(f, x, y, n);
                const EdgeMap m = kEdgeMaps.m[4 * f + e];
                if (r.f2 != m.f2 || r.a != m.a1 * i + m.an * (int)(n - 1) || r.b != m.b1 * i + m.bn * (int)(n - 1))
                    return false;
            }
    return true;
}
static_assert(edge_maps_consistent(), "edge maps are not affine in the position along the edge");

// Flat index (within the level) of texel (x, y) of `face` one step beyond
// exactly one edge (x or y in range).
__device__ __forceinline__ int64_t reproject_edge(int face, int x, int y, int n)
{
    const int e = x < 0 ? 0 : (x >= n ? 1 : (y < 0 ? 2 : 3));
    const int i = e <= 1 ? y : x;
    const EdgeMap m = kEdgeMaps.m[4 * face + e];
    const int a = m.a1 * i + m.an * (n - 1), b = m.b1 * i + m.bn * (n - 1);
    return ((int64_t)m.f2 * n + b) * n + a;
}

// The 24 edge maps packed 9 bits each, seven to a 64-bit word (f2: 3 bits,
// a1 + 1: 2, an: 1, b1 + 1: 2, bn: 1), so a lane can decode its map from
// four constants without a memory access.
struct EdgeWords {
    unsigned long long w[4];
};

constexpr EdgeWords pack_edge_maps()
{
    EdgeWords p{};
    for (int i = 0; i < 24; ++i) {
        const EdgeMap m = kEdgeMaps.m[i];
        const unsigned long long v = (unsigned long long)m.f2 | (unsigned long long)(m.a1 + 1) << 3 |
                                     (unsigned long long)m.an << 5 | (unsigned long long)(m.b1 + 1) << 6 |
                                     (unsigned long long)m.bn << 8;
        p.w[i / 7] |= v << (9 * (i % 7));
    }
    return p;
}

constexpr EdgeWords kEdgeWords = pack_edge_maps();

constexpr bool edge_words_consistent()
{
    for (int i = 0; i < 24; ++i) {
        const unsigned v = (unsigned)(kEdgeWords.w[i / 7] >> (9 * (i % 7))) & 511u;
        const EdgeMap m = kEdgeMaps.m[i];
        if ((int)(v & 7u) != m.f2 || (int)((v >> 3) & 3u) - 1 != m.a1 || (int)((v >> 5) & 1u) != m.an ||
            (int)((v >> 6) & 3u) - 1 != m.b1 || (int)((v >> 8) & 1u) != m.bn)
            return false;
    }
    return true;
}
static_assert(edge_words_consistent(), "edge map packing lost a field");

// reproject_edge in 32-bit arithmetic with the maps decoded from kEdgeWords.
__device__ __forceinline__ int reproject_edge_alu(int face, int x, int y, int n)
{
    const int e = x < 0 ? 0 : (x >= n ? 1 : (y < 0 ? 2 : 3));
    const int i = e <= 1 ? y : x;
    const int id = 4 * face + e, wi = id / 7;
    const unsigned long long w = wi == 0 ? kEdgeWords.w[0]
                                         : (wi == 1 ? kEdgeWords.w[1] : (wi == 2 ? kEdgeWords.w[2] : kEdgeWords.w[3]));
    const unsigned v = (unsigned)(w >> (9 * (id - 7 * wi))) & 511u;
    const int f2 = (int)(v & 7u), a1 = (int)((v >> 3) & 3u) - 1, an = (int)((v >> 5) & 1u);
    const int b1 = (int)((v >> 6) & 3u) - 1, bn = (int)((v >> 8) & 1u);
    const int a = a1 * i + an * (n - 1), b = b1 * i + bn * (n - 1);
    return (f2 * n + b) * n + a;
}

// resolve_texel with the integer edge maps (the same texels as
// reproject_edge), in 32-bit arithmetic without memory accesses (levels of
// fewer than 2^31 / 6 texels per face).
__device__ __forceinline__ int resolve_texel_edge(int face, int x, int y, int n, int (&idx)[3])
{
    const bool xin = (unsigned)x < (unsigned)n, yin = (unsigned)y < (unsigned)n;
    if (xin && yin) {
        idx[0] = (face * n + y) * n + x;
        return 1;
    }
    if (xin || yin) {
        idx[0] = reproject_edge_alu(face, x, y, n);
        return 1;
    }
    const int xc = x < 0 ? 0 : n - 1, yc = y < 0 ? 0 : n - 1;
    idx[0] = (face * n + yc) * n + xc;
    idx[1] = reproject_edge_alu(face, x, yc, n);
    idx[2] = reproject_edge_alu(face, xc, y, n);
    return 3;
}

// Resolves texel (x, y), x and y in [-1, n], of `face` to 1 or 3 flat
// indices within the level; returns the count.
__device__ __forceinline__ int resolve_texel(int face, int x, int y, int n, int64_t (&idx)[3])
{
    const bool xin = (unsigned)x < (unsigned)n, yin = (unsigned)y < (unsigned)n;
    if (xin && yin) {
        idx[0] = ((int64_t)face * n + y) * n + x;
        return 1;
    }
    if (xin || yin) {
        idx[0] = reproject_one(face, x, y, n);
        return 1;
    }
    const int xc = x < 0 ? 0 : n - 1, yc = y < 0 ? 0 : n - 1;
    idx[0] = ((int64_t)face * n + yc) * n + xc;
    idx[1] = reproject_one(face, x, yc, n);
    idx[2] = reproject_one(face, xc, y, n);
    return 3;
}


// Footprint of a direction on one level: face coordinates are computed once
// per direction (dir_face) and shared by every level.
struct face_st {
    int face;
    double s, t;
};

// Same face choice as dir_face, with one reciprocal instead of two
// divisions (s and t may differ from the quotients by an ulp of double; the
// seamless bilinear lookup is continuous, so lookups move by ~1e-16).
__device__ __forceinline__ face_st locate(const d3 &d)
{
    const double ax = fabs(d.x), ay = fabs(d.y), az = fabs(d.z);
    face_st f;
    double ma, sc, tc;
    if (ax >= ay && ax >= az) {
        f.face = d.x >= 0.0 ? 0 : 1;
        ma = ax;
        sc = d.x >= 0.0 ? -d.z : d.z;
        tc = -d.y;
    } else if (ay >= az) {
        f.face = d.y >= 0.0 ? 2 : 3;
        ma = ay;
        sc = d.x;
        tc = d.y >= 0.0 ? d.z : -d.z;
    } else {
        f.face = d.z >= 0.0 ? 4 : 5;
        ma = az;
        sc = d.z >= 0.0 ? d.x : -d.x;
        tc = -d.y;
    }
    const double inv = 1.0 / ma;
    f.s = sc * inv;
    f.t = tc * inv;
    return f;
}

struct bilin {
    int x0, y0;
    double fx, fy;
};

__device__ __forceinline__ bilin bilinear_at(const face_st &f, int n)
{
    const double x = (f.s + 1.0) * 0.5 * (double)n - 0.5;
    const double y = (f.t + 1.0) * 0.5 * (double)n - 0.5;
    const double x0 = floor(x), y0 = floor(y);
    bilin b;
    b.x0 = (int)x0;
    b.y0 = (int)y0;
    b.fx = x - x0;
    b.fy = y - y0;
    return b;
}

// Base-2 radical inverse of a 32-bit index (exact in double).
__device__ __forceinline__ double radical_inverse(uint32_t j)
{
    return (double)__builtin_bitreverse32(j) * 2.3283064365386963e-10;
}

// ---------------------------------------------------------------------------
// pcg4d (Jarzynski & Olano, "Hash Functions for GPU Rendering", JCGT 2020).
// ---------------------------------------------------------------------------
struct u4 {
    uint32_t x, y, z, w;
};

__device__ __forceinline__ u4 pcg4d(u4 v)
{
    v.x = v.x * 1664525u + 1013904223u;
    v.y = v.y * 1664525u + 1013904223u;
    v.z = v.z * 1664525u + 1013904223u;
    v.w = v.w * 1664525u + 1013904223u;
    v.x += v.y * v.w; v.y += v.z * v.x; v.z += v.x * v.y; v.w += v.y * v.z;
    v.x ^= v.x >> 16; v.y ^= v.y >> 16; v.z ^= v.z >> 16; v.w ^= v.w >> 16;
    v.x += v.y * v.w; v.y += v.z * v.x; v.z += v.x * v.y; v.w += v.y * v.z;
    return v;
}

// (h >> 9 + 1/2) 2^-23: exact float in (0, 1).
__device__ __forceinline__ float hash_unit(uint32_t h)
{
    return ((float)(h >> 9) + 0.5f) * 1.1920928955078125e-07f;
}

// ---------------------------------------------------------------------------
// Inverse standard normal CDF, AS 241 PPND16 (Wichura 1988), double.
// ---------------------------------------------------------------------------
// Central region of AS 241 (|p - 1/2| <= 0.425), q = p - 1/2.
__device__ __forceinline__ double ppnd16_central(double q)
{
    const double r = 0.180625 - q * q;
    const double num = (((((((r * 2509.0809287301226727 + 33430.575583588128105) * r + 67265.770927008700853) * r
                            + 45921.953931549871457) * r + 13731.693765509461125) * r + 1971.5909503065514427) * r
                         + 133.14166789178437745) * r + 3.387132872796366608);
    const double den = (((((((r * 5226.495278852545925 + 28729.085735721942674) * r + 39307.89580009271061) * r
                            + 21213.794301586595867) * r + 5394.1960214247511077) * r + 687.1870074920579083) * r
                         + 42.313330701600911252) * r + 1.0);
    return q * num / den;
}

// Tails of AS 241 (|p - 1/2| > 0.425).
__device__ __forceinline__ double ppnd16_tail(double p, double q)
{
    double r = q < 0.0 ? p : 1.0 - p;
    r = sqrt(-log(r));
    double num, den;
    if (r <= 5.0) {
        r -= 1.6;
        num = (((((((r * 7.7454501427834140764e-4 + 0.0227238449892691845833) * r + 0.24178072517745061177) * r
                   + 1.27045825245236838258) * r + 3.64784832476320460504) * r + 5.7694972214606914055) * r
                + 4.6303378461565452959) * r + 1.42343711074968357734);
        den = (((((((r * 1.05075007164441684324e-9 + 5.475938084995344946e-4) * r + 0.0151986665636164571966) * r
                   + 0.14810397642748007459) * r + 0.68976733498510000455) * r + 1.6763848301838038494) * r
                + 2.05319162663775882187) * r + 1.0);
    } else {
        r -= 5.0;
        num = (((((((r * 2.01033439929228813265e-7 + 2.71155556874348757815e-5) * r + 0.0012426609473880784386) * r
                   + 0.026532189526576123093) * r + 0.29656057182850489123) * r + 1.7848265399172913358) * r
                + 5.4637849111641143699) * r + 6.6579046435011037772);
        den = (((((((r * 2.04426310338993978564e-15 + 1.4215117583164458887e-7) * r + 1.8463183175100546818e-5) * r
                   + 7.868691311456132591e-4) * r + 0.0148753612908506148525) * r + 0.13692988092273580531) * r
                + 0.59983220655588793769) * r + 1.0);
    }
    const double val = num / den;
    return q < 0.0 ? -val : val;
}

// Standard normal quantile, AS 241 PPND16 (Wichura 1988), double.
__device__ __forceinline__ double ppnd16(double p)
{
    const double q = p - 0.5;
    if (fabs(q) <= 0.425) return ppnd16_central(q);
    return ppnd16_tail(p, q);
}

// The quantile's tails for the hash-derived uniforms: xi = (h9 + 1/2) 2^-23
// with h9 = h >> 9 is in a tail exactly when h9 < kTailLo or h9 > kTailHi;
// a table of those 2 kTailLo values (built with ppnd16_tail) replaces the
// divergent tail evaluation in shading.
constexpr uint32_t kTailLo = 629146u, kTailHi = 7759461u;
constexpr int64_t kTailEntries = 2 * (int64_t)kTailLo;

__device__ __forceinline__ bool tail_index(uint32_t h9, uint32_t &idx)
{
    if (h9 < kTailLo) {
        idx = h9;
        return true;
    }
    if (h9 > kTailHi) {
        idx = h9 - (kTailHi + 1u) + kTailLo;
        return true;
    }
    return false;
}

// ---------------------------------------------------------------------------
// Float gating thresholds of the dual-gated Gaussian.  With c = max(1, eps/p)
// the biased power (1 - c p)^(N2/c) equals (1 - max(p, eps))^(N2 min(1, p/eps)),
// a form that is also defined at p = 0.  Contraction is off so each
// operation rounds as written.
// ---------------------------------------------------------------------------
struct gate_f {
    float th_nN;   // P(n = N)
    float th_n1N;  // P(n = N) + P(n = 1)
    float th_nbN;  // 1 - P(nbar = N)
    float th_nb1N; // (1 - P(nbar = N)) - P(nbar = 1)
};

// sym: the bias also on the first power, P(n = N) = (1 - max(q, eps))^(N2
// min(1, q/eps)) with q the negative side's probability computed on its own
// (the printed algorithm takes p^N2, which float rounds to 1 when q < 2^-25).
__device__ __forceinline__ gate_f gate_thresholds(float Nf, float pf, float qf, bool sym)
{
#pragma clang fp contract(off)
    const float eps = 2.8840315031266055e-04f; // 10^-3.54
    const float N2 = fmaxf(2.0f, Nf);
    const float cN = fminf(fmaxf(Nf - 1.0f, 0.0f), 1.0f);
    const float cp = fmaxf(pf, eps);
    const float ex = N2 * fminf(1.0f, pf / eps);
    const float d1 = fmaxf(0.0f, 1.0f - fabsf(1.0f - Nf));
    const float P_nN = cN * (sym ? powf(1.0f - fmaxf(qf, eps), N2 * fminf(1.0f, qf / eps)) : powf(pf, N2));
    const float P_nbN = cN * powf(1.0f - cp, ex);
    const float P_n1 = d1 * pf;
    const float P_nb1 = d1 * (1.0f - pf);
    gate_f g;
    g.th_nN = P_nN;
    g.th_n1N = P_nN + P_n1;
    g.th_nbN = 1.0f - P_nbN;
    g.th_nb1N = (1.0f - P_nbN) - P_nb1;
    return g;
}

// The four gating decisions of a node (xi1 against the thresholds of
// gate_thresholds), computed first from powers evaluated with the hardware
// log2/exp2: their relative error is below 2^-17 whenever the power is
// above 2^-64 (both instructions are within one ulp of the result and the
// exponent's magnitude is then at most 64), so a decision whose xi1 lies
// farther than 2^-14 P + 2^-22 from its approximate threshold equals the
// decision from the exactly rounded thresholds.  Only when some xi1 is that
// close (or a value is not finite) are the thresholds evaluated with powf.
struct gate_d {
    bool nN, n1N, nbN, nb1N;
};

__device__ __forceinline__ gate_d gate_decide(float Nf, float pf, float qf, bool sym, float xi1,
                                              bool exact_only = false)
{
#pragma clang fp contract(off)
    const float eps = 2.8840315031266055e-04f; // 10^-3.54
    const float N2 = fmaxf(2.0f, Nf);
    const float cN = fminf(fmaxf(Nf - 1.0f, 0.0f), 1.0f);
    const float cp = fmaxf(pf, eps);
    const float ex = N2 * fminf(1.0f, pf / eps);
    const float d1 = fmaxf(0.0f, 1.0f - fabsf(1.0f - Nf));
    const float bN = 1.0f - cp;
    const float bA = sym ? 1.0f - fmaxf(qf, eps) : pf;
    const float eA = sym ? N2 * fminf(1.0f, qf / eps) : N2;
    const float P_nN = cN * __builtin_amdgcn_exp2f(eA * __builtin_amdgcn_logf(bA));
    const float P_nbN = cN * __builtin_amdgcn_exp2f(ex * __builtin_amdgcn_logf(bN));
    const float P_n1 = d1 * pf;
    const float P_nb1 = d1 * (1.0f - pf);
    const float t_nN = P_nN, t_n1N = P_nN + P_n1;
    const float t_nbN = 1.0f - P_nbN, t_nb1N = (1.0f - P_nbN) - P_nb1;
    const float mN = 6.103515625e-05f * P_nN + 2.384185791015625e-07f;   // 2^-14 P + 2^-22
    const float mB = 6.103515625e-05f * P_nbN + 2.384185791015625e-07f;
    const bool robust = !exact_only && fabsf(xi1 - t_nN) > mN && fabsf(xi1 - t_n1N) > mN &&
                        fabsf(xi1 - t_nbN) > mB && fabsf(xi1 - t_nb1N) > mB;
    gate_d d;
    if (robust) {
        d.nN = xi1 < t_nN;
        d.n1N = xi1 < t_n1N;
        d.nbN = t_nbN <= xi1;
        d.nb1N = t_nb1N <= xi1;
    } else {
        const gate_f g = gate_thresholds(Nf, pf, qf, sym);
        d.nN = xi1 < g.th_nN;
        d.n1N = xi1 < g.th_n1N;
        d.nbN = g.th_nbN <= xi1;
        d.nb1N = g.th_nb1N <= xi1;
    }
    return d;
}

// Gate threshold of the single-gated Gaussian (Sec. 6): form 1, Eq. (gated),
// min(N p, 1 - (1-p)^N) with the power biased as in the dual gate; form 2,
// Eq. (oldgated), the prior 1 - (1-p)^N without bias.  float, powf.
__device__ __forceinline__ float single_gate_threshold(int form, float Nf, float pf)
{
#pragma clang fp contract(off)
    if (form == 1) {
        const float eps = 2.8840315031266055e-04f; // 10^-3.54
        const float cp = fmaxf(pf, eps);
        const float ex = Nf * fminf(1.0f, pf / eps);
        const float pany = 1.0f - powf(1.0f - cp, ex);
        const float np = Nf * pf;
        return np < pany ? np : pany;
    }
    return 1.0f - powf(1.0f - pf, Nf);
}

// The single gate's decision xi1 < threshold, first from the power taken
// with the hardware log2/exp2 (the bound of gate_decide: relative error
// below 2^-17 above 2^-64, and the minimum with the exact N p moves the
// threshold by no more than the power), falling back to powf within
// 2^-14 P + 2^-22 of the approximate threshold.
__device__ __forceinline__ bool single_gate_decide(int form, float Nf, float pf, float xi1, bool exact_only)
{
#pragma clang fp contract(off)
    if (!exact_only) {
        float base, ex;
        if (form == 1) {
            const float eps = 2.8840315031266055e-04f; // 10^-3.54
            base = 1.0f - fmaxf(pf, eps);
            ex = Nf * fminf(1.0f, pf / eps);
        } else {
            base = 1.0f - pf;
            ex = Nf;
        }
        const float P = __builtin_amdgcn_exp2f(ex * __builtin_amdgcn_logf(base));
        const float pany = 1.0f - P;
        float th = pany;
        if (form == 1) {
            const float np = Nf * pf;
            th = np < pany ? np : pany;
        }
        const float margin = 6.103515625e-05f * P + 2.384185791015625e-07f; // 2^-14 P + 2^-22
        if (fabsf(xi1 - th) > margin) return xi1 < th;
    }
    return xi1 < single_gate_threshold(form, Nf, pf);
}

// Learned-surrogate inputs of a lookup (the project's extension, not the
// paper's): the reflection direction, then (ln alpha - c) / h for alpha_x
// and alpha_y, where c and h map [ln 0.02, ln 0.5] onto [-1, 1].
__device__ __forceinline__ void surrogate_features(double wx, double wy, double wz, double ax, double ay, float *out)
{
    const double lo = -3.912023005428146, hi = -0.6931471805599453; // ln 0.02, ln 0.5
    const double c = 0.5 * (lo + hi), h = 0.5 * (hi - lo);
    out[0] = (float)wx;
    out[1] = (float)wy;
    out[2] = (float)wz;
    out[3] = (float)((log(ax) - c) / h);
    out[4] = (float)((log(ay) - c) / h);
}

} // namespace glint
