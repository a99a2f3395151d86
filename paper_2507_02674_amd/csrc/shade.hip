// Per-pixel glint shading (Sec. 3.2, Sec. 3.3 Eq. (anisogrid), Sec. 4
// Eq. (probhk) and Eq. (iblglints:fin), Sec. 6 Alg. "Dual-gated Gaussian").
//
// One thread per pixel.  The footprint count, the reflection probabilities
// (trilinear pyramid lookup), the tree probabilities and the Gaussian draw
// are double; the gating thresholds and masks are float, as the paper's bias
// constant assumes.  The multinomial tree is walked depth by depth in place
// over a register array of K counts (compile-time K, static indices).
#include "device.hpp"
#include "internal.hpp"

namespace glint {

constexpr int kShadeThreads = 256;

template <int DT>
__device__ __forceinline__ double load_value(const void *base, int64_t i);

template <>
__device__ __forceinline__ double load_value<0>(const void *base, int64_t i)
{
    return (double)static_cast<const float *>(base)[i];
}
template <>
__device__ __forceinline__ double load_value<1>(const void *base, int64_t i)
{
    return (double)static_cast<const _Float16 *>(base)[i];
}
template <>
__device__ __forceinline__ double load_value<2>(const void *base, int64_t i)
{
    return (double)__uint_as_float((uint32_t)static_cast<const uint16_t *>(base)[i] << 16);
}
template <>
__device__ __forceinline__ double load_value<3>(const void *base, int64_t i)
{
    return (double)static_cast<const uint16_t *>(base)[i] * (1.0 / 65535.0);
}

// One pyramid texel: K indicator channels (stored type DT) and RGB, as double.
template <int K, int DT>
__device__ __forceinline__ void load_texel(const void *__restrict__ ind, const float *__restrict__ rgb, int64_t t,
                                           double (&v)[K + 3])
{
    if constexpr (DT == 0 && K % 4 == 0) {
        const float4 *p = reinterpret_cast<const float4 *>(static_cast<const float *>(ind) + t * K);
#pragma unroll
        for (int q = 0; q < K / 4; ++q) {
            const float4 f = p[q];
            v[4 * q] = f.x; v[4 * q + 1] = f.y; v[4 * q + 2] = f.z; v[4 * q + 3] = f.w;
        }
    } else if constexpr (DT != 0 && K % 8 == 0) {
        const uint4 *p = reinterpret_cast<const uint4 *>(static_cast<const uint16_t *>(ind) + t * K);
#pragma unroll
        for (int q = 0; q < K / 8; ++q) {
            const uint4 u = p[q];
            const uint32_t w[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const uint16_t h = (uint16_t)(w[e / 2] >> (16 * (e % 2)));
                double val;
                if constexpr (DT == 1) val = (double)__builtin_bit_cast(_Float16, h);
                else if constexpr (DT == 2) val = (double)__uint_as_float((uint32_t)h << 16);
                else val = (double)h * (1.0 / 65535.0);
                v[8 * q + e] = val;
            }
        }
    } else {
#pragma unroll
        for (int k = 0; k < K; ++k) v[k] = load_value<DT>(ind, t * K + k);
    }
    const float4 c = reinterpret_cast<const float4 *>(rgb)[t];
    v[K] = c.x; v[K + 1] = c.y; v[K + 2] = c.z;
}

// acc += w * (texel (x, y) of `face` on the pyramid level at `base`) with the
// seam rule: beyond a cube corner the texel is the mean of the three texels
// meeting there, added as three terms of weight w/3.
template <int K, int DT>
__device__ __forceinline__ void accumulate_pyr(const void *__restrict__ ind, const float *__restrict__ rgb,
                                               int64_t base, int face, int x, int y, int n, double w,
                                               double (&acc)[K + 3])
{
    int64_t idx[3];
    const int cnt = resolve_texel(face, x, y, n, idx);
    const double wc = cnt == 3 ? w / 3.0 : w;
#pragma unroll 1
    for (int e = 0; e < cnt; ++e) {
        double v[K + 3];
        load_texel<K, DT>(ind, rgb, base + (e == 0 ? idx[0] : (e == 1 ? idx[1] : idx[2])), v);
#pragma unroll
        for (int k = 0; k < K + 3; ++k) acc[k] += wc * v[k];
    }
}

__device__ __forceinline__ double lut_bilinear(const float *__restrict__ lut, int stride, int comp, double mu,
                                               double sa)
{
    double x = mu * kLutN - 0.5, y = sa * kLutN - 0.5;
    x = x < 0.0 ? 0.0 : (x > kLutN - 1 ? kLutN - 1 : x);
    y = y < 0.0 ? 0.0 : (y > kLutN - 1 ? kLutN - 1 : y);
    double x0 = floor(x), y0 = floor(y);
    x0 = x0 > kLutN - 2 ? kLutN - 2 : x0;
    y0 = y0 > kLutN - 2 ? kLutN - 2 : y0;
    const double fx = x - x0, fy = y - y0;
    const int ix = (int)x0, iy = (int)y0;
    const double v00 = lut[(iy * kLutN + ix) * stride + comp];
    const double v01 = lut[(iy * kLutN + ix + 1) * stride + comp];
    const double v10 = lut[((iy + 1) * kLutN + ix) * stride + comp];
    const double v11 = lut[((iy + 1) * kLutN + ix + 1) * stride + comp];
    const double top = (1.0 - fx) * v00 + fx * v01;
    const double bot = (1.0 - fx) * v10 + fx * v11;
    return (1.0 - fy) * top + fy * bot;
}

struct ShadeArgs {
    glint_gbuffer g;
    int64_t P;
    const void *ind_pyr;
    const float *rgb_pyr;
    const double *levels;
    const float *lut_S;
    const float *lut_E;
    int R, M;
    uint32_t seed;
    float *radiance;
    double *counts;
    uint8_t *codes;
    double *probs;
    const float *F;      // surrogate form: filtered indicator values [P][K] (else null)
    const double *qtail; // quantile tail table (else null: tails evaluated inline)
    int exact_gating;    // 1: gating thresholds always through powf (verification)
    int sampler;         // GLINT_SAMPLER_*: node sampler of the multinomial tree
    double gamma;        // constant reflection probability (prob_mode GLINT_PROBS_CONSTANT)
    int lobe_taps;       // anisotropic lookup taps (2, 4, 8; 0: isotropic lookup)
};

// The same arguments with every pointer typed as global memory.  Pointers
// read from memory (the batched launch's per-view table) have no known
// address space, so loads through them would be generic (flat) loads with
// 64-bit addresses in vector registers; read through this layout they are
// global loads, as for kernel arguments.
#define GLINT_GLOBAL(T) __attribute__((address_space(1))) T
struct GBufferG {
    const GLINT_GLOBAL(float) *nx, *ny, *nz, *vx, *vy, *vz, *u, *v, *area, *ax, *ay, *density, *f0r, *f0g, *f0b;
    const GLINT_GLOBAL(uint32_t) *surf_id;
    const GLINT_GLOBAL(float) *visibility, *tx, *ty, *tz, *dudx, *dudy, *dvdx, *dvdy;
};

struct ShadeArgsG {
    GBufferG g;
    int64_t P;
    const GLINT_GLOBAL(void) *ind_pyr;
    const GLINT_GLOBAL(float) *rgb_pyr;
    const GLINT_GLOBAL(double) *levels;
    const GLINT_GLOBAL(float) *lut_S;
    const GLINT_GLOBAL(float) *lut_E;
    int R, M;
    uint32_t seed;
    GLINT_GLOBAL(float) *radiance;
    GLINT_GLOBAL(double) *counts;
    GLINT_GLOBAL(uint8_t) *codes;
    GLINT_GLOBAL(double) *probs;
    const GLINT_GLOBAL(float) *F;
    const GLINT_GLOBAL(double) *qtail;
    int exact_gating;
    int sampler;
    double gamma;
    int lobe_taps;
};
static_assert(sizeof(GBufferG) == sizeof(glint_gbuffer) && offsetof(GBufferG, dvdy) == offsetof(glint_gbuffer, dvdy) &&
                  offsetof(GBufferG, surf_id) == offsetof(glint_gbuffer, surf_id),
              "GBufferG mirrors glint_gbuffer");
static_assert(sizeof(ShadeArgsG) == sizeof(ShadeArgs) && offsetof(ShadeArgsG, P) == offsetof(ShadeArgs, P) &&
                  offsetof(ShadeArgsG, seed) == offsetof(ShadeArgs, seed) &&
                  offsetof(ShadeArgsG, qtail) == offsetof(ShadeArgs, qtail) &&
                  offsetof(ShadeArgsG, gamma) == offsetof(ShadeArgs, gamma) &&
                  offsetof(ShadeArgsG, lobe_taps) == offsetof(ShadeArgs, lobe_taps),
              "ShadeArgsG mirrors ShadeArgs");

// acc += w * trilinear lookup of the pyramid (KL indicator channels, then
// RGB) in direction dir at lod (clamped to [0, M-1]).
template <int KL, int DT, class Args>
__device__ __forceinline__ void pyramid_trilinear(const Args &A, const d3 &dir, double lod, double w,
                                                  double (&acc)[KL + 3])
{
    lod = lod < 0.0 ? 0.0 : (lod > (double)(A.M - 1) ? (double)(A.M - 1) : lod);
    const double l0f = floor(lod);
    const int s0 = (int)l0f;
    const int s1 = s0 + 1 < A.M ? s0 + 1 : A.M - 1;
    const double fr = lod - l0f;
    const face_st fs = locate(dir);
    const int nlev = fr > 0.0 ? 2 : 1;
#pragma unroll 1
    for (int li = 0; li < nlev; ++li) {
        const int s = li == 0 ? s0 : s1;
        const double lw = w * (li == 0 ? 1.0 - fr : fr);
        const int ns = A.R >> s;
        const bilin bl = bilinear_at(fs, ns);
        const int64_t base = level_offset(A.R, s);
        const double w4[4] = {lw * ((1.0 - bl.fy) * (1.0 - bl.fx)), lw * ((1.0 - bl.fy) * bl.fx),
                              lw * (bl.fy * (1.0 - bl.fx)), lw * (bl.fy * bl.fx)};
        // the four texels of the footprint; one beyond a face edge is the
        // neighbouring face's texel (one index, as inside the face), one
        // beyond a cube corner needs the three-texel mean below
        int64_t tt[4];
        bool corner = false;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int x = bl.x0 + (c & 1), y = bl.y0 + (c >> 1);
            const bool xin = (unsigned)x < (unsigned)ns, yin = (unsigned)y < (unsigned)ns;
            if (xin && yin) tt[c] = base + ((int64_t)fs.face * ns + y) * ns + x;
            else if (xin || yin) tt[c] = base + reproject_edge(fs.face, x, y, ns);
            else corner = true;
        }
        if (!corner) {
            // four loads in flight
            double v[4][KL + 3];
#pragma unroll
            for (int c = 0; c < 4; ++c) load_texel<KL, DT>((const void *)A.ind_pyr, (const float *)A.rgb_pyr, tt[c], v[c]);
#pragma unroll
            for (int c = 0; c < 4; ++c)
#pragma unroll
                for (int k = 0; k < KL + 3; ++k) acc[k] += w4[c] * v[c][k];
        } else {
            // a cube corner: one copy of the seam rule
#pragma unroll 1
            for (int c = 0; c < 4; ++c)
                accumulate_pyr<KL, DT>((const void *)A.ind_pyr, (const float *)A.rgb_pyr, base, fs.face, bl.x0 + (c & 1), bl.y0 + (c >> 1), ns,
                                       c == 0 ? w4[0] : (c == 1 ? w4[1] : (c == 2 ? w4[2] : w4[3])), acc);
        }
    }
}

// One dual-gated Gaussian draw (Alg. "Dual-gated Gaussian").
// xi2 = (h9 + 1/2) 2^-23; qtail: the quantile's tail table (or null: the
// tails are evaluated here).
__device__ __forceinline__ void dual_gated(double N, double p, double q, bool sym, float xi1, float xi2,
                                           uint32_t h9, const double *__restrict__ qtail, bool exact_gating,
                                           double &n, double &nb, uint32_t &code)
{
    // Rounded as written (no fused multiply-add): at N ~ 1e12 one ulp of mu
    // is ~1e-4, so every operation must round as in the definition for the
    // counts' integer parts to agree.
#pragma clang fp contract(off)
    // the tail value is fetched first so its latency overlaps the gating
    uint32_t tidx = 0;
    const bool tail = tail_index(h9, tidx);
    double ztab = 0.0;
    if (qtail && tail) ztab = qtail[tidx];
    const gate_d gd = gate_decide((float)N, (float)p, (float)q, sym, xi1, exact_gating);
    const bool BnN = gd.nN;
    const bool Bn1N = gd.n1N;
    const bool BnbN = gd.nbN;
    const bool Bnb1N = gd.nb1N;
    const bool BG = ((float)N > 1.0f) && !Bn1N && !Bnb1N;
    const double N2 = N > 2.0 ? N : 2.0;
    double G = 0.0, Gb = 0.0;
    if (BG) {
        const double mu = 1.0 + (N2 - 2.0) * p;
        const double sig = sqrt((N2 - 2.0) * p * (1.0 - p));
        const double xd = (double)xi2, q = xd - 0.5;
        const double z = !tail ? ppnd16_central(q) : (qtail ? ztab : ppnd16_tail(xd, q));
        const double x = mu + sig * z;
        G = x < 1.0 ? 1.0 : (x > N2 - 1.0 ? N2 - 1.0 : x);
        Gb = N2 - G;
    }
    n = (BnN ? N2 - 1.0 : 0.0) + (Bn1N ? 1.0 : 0.0) + (BG ? G : 0.0);
    nb = (BnbN ? N2 - 1.0 : 0.0) + (Bnb1N ? 1.0 : 0.0) + (BG ? Gb : 0.0);
    code = (uint32_t)BnN | ((uint32_t)Bn1N << 1) | ((uint32_t)BnbN << 2) | ((uint32_t)Bnb1N << 3) |
           ((uint32_t)BG << 4);
}

// Single-gated Gaussian (Sec. 6 "Single-Gated Gaussians", "Gating
// Generalization"): form 1 Eq. (gated), form 2 the prior Eq. (oldgated)
// (floor, no bias, no N < 1 generalisation).  The negative count is what
// remains, max(N - n, 0).
__device__ __forceinline__ void single_gated(int form, double N, double p, float xi1, float xi2, uint32_t h9,
                                             const double *__restrict__ qtail, bool exact_gating, double &n,
                                             double &nb, uint32_t &code)
{
#pragma clang fp contract(off)
    uint32_t tidx = 0;
    const bool tail = tail_index(h9, tidx);
    double ztab = 0.0;
    if (qtail && tail) ztab = qtail[tidx];
    const bool hit = single_gate_decide(form, (float)N, (float)p, xi1, exact_gating);
    const bool BG = hit && N > 1.0;
    double c = hit ? 1.0 : 0.0;
    if (BG) {
        const double mu = 1.0 + (N - 1.0) * p;
        const double sig = sqrt((N - 1.0) * p * (1.0 - p));
        const double xd = (double)xi2, q = xd - 0.5;
        const double z = !tail ? ppnd16_central(q) : (qtail ? ztab : ppnd16_tail(xd, q));
        const double x = mu + sig * z;
        c = x < 1.0 ? 1.0 : (x > N ? N : x);
        if (form == 2) c = floor(c);
    }
    n = c;
    const double r = N - c;
    nb = r > 0.0 ? r : 0.0;
    code = (uint32_t)hit | ((uint32_t)BG << 4);
}

// SG: a single-gated form (`sampler` says which); else the dual gate, with
// the bias on both powers when SYM (GLINT_SAMPLER_DUAL_SYMMETRIC).  Both are
// compile-time switches, so each kernel carries only its own form: a
// runtime choice between the two dual forms keeps the right shares of a
// whole tree depth live and costs the default kernel a third of its
// occupancy (236 instead of 166 registers).
// q: the node's negative-side probability (1 - p in exact arithmetic),
// read only when SYM.
template <bool SG, bool SYM = false>
__device__ __forceinline__ void node_sample(int sampler, double N, double p, double q, float xi1, float xi2,
                                            uint32_t h9, const double *__restrict__ qtail, bool exact_gating,
                                            double &n, double &nb, uint32_t &code)
{
    static_assert(!(SG && SYM), "the symmetric bias is a form of the dual gate");
    if constexpr (SG) single_gated(sampler, N, p, xi1, xi2, h9, qtail, exact_gating, n, nb, code);
    else dual_gated(N, p, q, SYM, xi1, xi2, h9, qtail, exact_gating, n, nb, code);
}

// Hierarchical multinomial over K bins: balanced binary tree, nodes in
// breadth-first (heap) order; node i covers a contiguous run of bins, its
// probability is S_left / S_node, its left child 2i+1 receives the positive
// count n and its right child 2i+2 the negative count nbar.
//
// Code shape: the depth loop is unrolled (log2 K copies of the sampler); the
// nodes of one depth run in a loop that is not unrolled.  The loop consumes
// its inputs from the front of small register queues and appends the two
// child counts at the back, shifting with static indices, so no register
// array is indexed dynamically.
template <int K, bool SG, bool SYM>
__device__ __forceinline__ void multinomial(double NP, const double (&p)[K], uint32_t seed_mix, uint32_t key, int64_t a,
                                            int64_t b, const double *__restrict__ qtail, bool exact_gating,
                                            int sampler, double (&leaf)[K], uint8_t *codes)
{
    double Q[K]; // counts of the current depth, in node order
    Q[0] = NP;
    // one hash per node pair: node 2i takes (x, y), node 2i+1 the (z, w)
    // carried over (nodes run in increasing order across the depths)
    uint32_t carry_z = 0, carry_w = 0;
#pragma unroll
    for (int k = 1; k < K; ++k) Q[k] = 0.0;
#pragma unroll
    for (int d = 0; (1 << d) < K; ++d) {
        const int nd = 1 << d, width = K >> d;
        double P[K / 2], Qr[K / 2]; // node probabilities (left, right share) of this depth, in node order
#pragma unroll
        for (int j = 0; j < nd; ++j) {
            const int lo = j * width, mid = lo + width / 2, hi = lo + width;
            double sl = 0.0, sr = 0.0;
#pragma unroll
            for (int k = lo; k < mid; ++k) sl += p[k];
#pragma unroll
            for (int k = mid; k < hi; ++k) sr += p[k];
            const double st = sl + sr;
            const double q = st > 0.0 ? sl / st : 0.0;
            P[j] = q > 1.0 ? 1.0 : q;
            if constexpr (SYM) {
                const double r = st > 0.0 ? sr / st : 0.0;
                Qr[j] = r > 1.0 ? 1.0 : r;
            } else {
                Qr[j] = 0.0;
            }
        }
        double Rq[K];
#pragma unroll
        for (int k = 0; k < K; ++k) Rq[k] = 0.0;
#pragma unroll 1
        for (int j = 0; j < nd; ++j) {
            const double N = Q[0], pj = P[0], qj = Qr[0];
#pragma unroll
            for (int k = 0; k + 1 < nd; ++k) { Q[k] = Q[k + 1]; P[k] = P[k + 1]; Qr[k] = Qr[k + 1]; }
            const int node = nd - 1 + j;
            uint32_t hx, hy;
            if ((node & 1) == 0) {
                const u4 h = pcg4d({(uint32_t)a, (uint32_t)b, key | ((uint32_t)node >> 1),
                                    seed_mix});
                hx = h.x;
                hy = h.y;
                carry_z = h.z;
                carry_w = h.w;
            } else {
                hx = carry_z;
                hy = carry_w;
            }
            double n, nb;
            uint32_t code;
            node_sample<SG, SYM>(sampler, N, pj, qj, hash_unit(hx), hash_unit(hy), hy >> 9, qtail, exact_gating, n,
                                 nb, code);
            if (codes) codes[node] = (uint8_t)code;
#pragma unroll
            for (int k = 0; k + 2 < 2 * nd; ++k) Rq[k] = Rq[k + 2];
            Rq[2 * nd - 2] = n;
            Rq[2 * nd - 1] = nb;
        }
#pragma unroll
        for (int k = 0; k < 2 * nd; ++k) Q[k] = Rq[k];
    }
#pragma unroll
    for (int k = 0; k < K; ++k) leaf[k] = Q[k];
}

// The second shape of the hierarchical multinomial (tree = 1): a sequential
// chain.  Node i draws bin i's facets out of those that reach it with
// probability p_i / S_i, S_i = p_i + S_{i+1} the suffix sum (from the last
// bin down); the negative count goes on to node i+1 and bin K-1 keeps what
// reaches it.  One copy of the sampler in a loop that is not unrolled; the
// node probabilities and the bins' counts move through register queues with
// static indices.
template <int K, bool SG, bool SYM>
__device__ __forceinline__ void multinomial_chain(double NP, const double (&p)[K], uint32_t seed_mix, uint32_t key,
                                                  int64_t a, int64_t b, const double *__restrict__ qtail,
                                                  bool exact_gating, int sampler, double (&leaf)[K], uint8_t *codes)
{
    double S[K];
    S[K - 1] = p[K - 1];
#pragma unroll
    for (int k = K - 2; k >= 0; --k) S[k] = p[k] + S[k + 1];
    double P[K - 1], Qr[K - 1]; // bin k's share of S_k and that of the bins after it
#pragma unroll
    for (int k = 0; k < K - 1; ++k) {
        const double q = S[k] > 0.0 ? p[k] / S[k] : 0.0;
        P[k] = q > 1.0 ? 1.0 : q;
        if constexpr (SYM) {
            const double r = S[k] > 0.0 ? S[k + 1] / S[k] : 0.0;
            Qr[k] = r > 1.0 ? 1.0 : r;
        } else {
            Qr[k] = 0.0;
        }
    }
    double Mq[K];
#pragma unroll
    for (int k = 0; k < K; ++k) Mq[k] = 0.0;
    double N = NP;
    uint32_t carry_z = 0, carry_w = 0;
#pragma unroll 1
    for (int node = 0; node < K - 1; ++node) {
        const double pj = P[0], qj = Qr[0];
#pragma unroll
        for (int k = 0; k + 1 < K - 1; ++k) { P[k] = P[k + 1]; Qr[k] = Qr[k + 1]; }
        uint32_t hx, hy;
        if ((node & 1) == 0) {
            const u4 h = pcg4d({(uint32_t)a, (uint32_t)b, key | ((uint32_t)node >> 1), seed_mix});
            hx = h.x;
            hy = h.y;
            carry_z = h.z;
            carry_w = h.w;
        } else {
            hx = carry_z;
            hy = carry_w;
        }
        double n, nb;
        uint32_t code;
        node_sample<SG, SYM>(sampler, N, pj, qj, hash_unit(hx), hash_unit(hy), hy >> 9, qtail, exact_gating, n, nb,
                             code);
        if (codes) codes[node] = (uint8_t)code;
#pragma unroll
        for (int k = 0; k + 1 < K; ++k) Mq[k] = Mq[k + 1];
        Mq[K - 1] = n;
        N = nb;
    }
    // Mq[1..K-1] hold the counts of bins 0..K-2 in order
#pragma unroll
    for (int k = 0; k + 1 < K; ++k) leaf[k] = Mq[k + 1];
    leaf[K - 1] = N;
}

// Footprint grid (Sec. 3.3 "Binomial Sampling with Anisotropic Grids"; the
// paper uses the grid as a black box, the layout is this library's): the
// pixel footprint, the ellipse of J J^T for the uv Jacobian J, by length
// log2 s_maj, anisotropy log2(s_maj / s_min) (s_min clamped to s_maj / 16)
// and orientation 8 theta / pi (periodic); a Kuhn tetrahedron of that grid
// (axes by decreasing fraction, ties in axis order) gives 4 vertices with
// weights; each vertex (l, a, o) draws with its own count N_P 4^l 2^-a /
// (s_maj s_min) on the uv triangle grid of its footprint (uv rotated by
// -o pi/8, scaled by (2^-l, 2^(a-l))), 3 triangle vertices each.
struct FootGrid {
    bool valid;
    double smaj, sminc;
    double wt[4];
    int l[4], a[4], o[4];
};

__device__ __forceinline__ FootGrid footprint_grid(double j00, double j01, double j10, double j11)
{
    FootGrid G;
    const double m11 = j00 * j00 + j01 * j01, m22 = j10 * j10 + j11 * j11, m12 = j00 * j10 + j01 * j11;
    const double h = 0.5 * (m11 - m22);
    const double disc = sqrt(h * h + m12 * m12);
    const double smaj = sqrt(0.5 * (m11 + m22) + disc);
    G.valid = isfinite(smaj) && smaj > 1e-12;
    if (!G.valid) return G;
    const double smin = fabs(j00 * j11 - j01 * j10) / smaj;
    const bool clamped = !(smin > smaj / 16.0);
    const double sminc = clamped ? smaj / 16.0 : smin;
    const double A = smaj / sminc;
    double th = 0.5 * atan2(2.0 * m12, m11 - m22);
    if (th < 0.0) th += M_PI;
    const double g[3] = {log2(smaj), clamped ? 4.0 : log2(A), th * (8.0 / M_PI)};
    int base[3];
    double f[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double fl = floor(g[c]);
        base[c] = (int)fl;
        f[c] = g[c] - fl;
    }
    // axes by decreasing fraction, ties in axis order (insertion sort)
    int o0 = 0, o1 = 1, o2 = 2;
    if (f[o1] > f[o0]) { const int t = o0; o0 = o1; o1 = t; }
    if (f[o2] > f[o1]) {
        const int t = o1; o1 = o2; o2 = t;
        if (f[o1] > f[o0]) { const int t2 = o0; o0 = o1; o1 = t2; }
    }
    G.smaj = smaj;
    G.sminc = sminc;
    G.wt[0] = 1.0 - f[o0];
    G.wt[1] = f[o0] - f[o1];
    G.wt[2] = f[o1] - f[o2];
    G.wt[3] = f[o2];
    int cv[3] = {base[0], base[1], base[2]};
    const int ord[3] = {o0, o1, o2};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        if (i > 0) cv[ord[i - 1]] += 1;
        G.l[i] = cv[0];
        G.a[i] = cv[1];
        G.o[i] = ((cv[2] % 8) + 8) % 8;
    }
    return G;
}

// Shades pixel i of the view described by A (all of rows b1-b5).  SURR: the
// K filtered indicator values come from A.F (a learned surrogate's output)
// and only RGB is read from the pyramid.  PC: constant reflection
// probability A.gamma (K = 2, levels (0, 1)), no indicator lookup.
template <int K, int DT, int V, bool SURR = false, bool SG = false, bool PC = false, bool AN = false,
          bool CH = false, bool SYM = false, class Args = ShadeArgs>
__device__ __forceinline__ void shade_pixel(const Args &A, int64_t i)
{
    static_assert(!PC || (K == 2 && !SURR), "constant probabilities use two bins");
    constexpr int KL = (SURR || PC) ? 0 : K; // indicator channels read from the pyramid
    const uint32_t surf = A.g.surf_id[i];
    if (surf == GLINT_NO_SURFACE) {
        A.radiance[3 * i] = 0.0f; A.radiance[3 * i + 1] = 0.0f; A.radiance[3 * i + 2] = 0.0f;
        if (A.counts) for (int k = 0; k < V * K; ++k) A.counts[i * V * K + k] = 0.0;
        if (A.codes) for (int k = 0; k < V * (K - 1); ++k) A.codes[i * V * (K - 1) + k] = 0;
        if (A.probs) for (int k = 0; k < K; ++k) A.probs[i * K + k] = 0.0;
        return;
    }
    const double area = (double)A.g.area[i];
    const double NP = (double)A.g.density[i] * area; // Sec. 3.2: stratified count
    const d3 n = {(double)A.g.nx[i], (double)A.g.ny[i], (double)A.g.nz[i]};
    const d3 v = {(double)A.g.vx[i], (double)A.g.vy[i], (double)A.g.vz[i]};
    const double mu = n.x * v.x + n.y * v.y + n.z * v.z;
    const d3 wr = {2.0 * mu * n.x - v.x, 2.0 * mu * n.y - v.y, 2.0 * mu * n.z - v.z};
    const double aeff = sqrt((double)A.g.ax[i] * (double)A.g.ay[i]);
    const double sa = sqrt(aeff);
    // trilinear pyramid lookup of the K indicator channels and RGB
    double acc[KL + 3];
#pragma unroll
    for (int k = 0; k < KL + 3; ++k) acc[k] = 0.0;
    if constexpr (AN) {
        // anisotropic lookup: lobe_taps isotropic lookups along the lobe's
        // major axis (layout in the header), averaged
        const int T = A.lobe_taps;
        const double ax = (double)A.g.ax[i], ay = (double)A.g.ay[i];
        d3 t = {(double)A.g.tx[i], (double)A.g.ty[i], (double)A.g.tz[i]};
        const double tn = t.x * n.x + t.y * n.y + t.z * n.z;
        t = {t.x - tn * n.x, t.y - tn * n.y, t.z - tn * n.z};
        const double tl = sqrt(t.x * t.x + t.y * t.y + t.z * t.z);
        if (tl > 1e-12) {
            t = {t.x / tl, t.y / tl, t.z / tl};
        } else {
            d3 b2;
            onb(n, t, b2);
        }
        const d3 bt = {n.y * t.z - n.z * t.y, n.z * t.x - n.x * t.z, n.x * t.y - n.y * t.x};
        const double amin = ax < ay ? ax : ay, amax = ax < ay ? ay : ax;
        const d3 d = ax >= ay ? t : bt;
        double at = amax / (double)T;
        at = at < amin ? amin : at;
        const double s2 = amax * amax - at * at;
        const double sp = s2 > 0.0 ? sqrt(s2) : 0.0;
        const double lodt = sqrt(at) * (double)(A.M - 1);
        double wsum = 0.0;
#pragma unroll 1
        for (int j = 0; j < T; ++j) {
            const double u = (double)(2 * j + 1) / (double)T - 1.0;
            const double x = sp * u / sqrt(1.0 - u * u);
            const double hl = sqrt(1.0 + x * x); // |n - x d| for orthonormal n, d
            const d3 h = {(n.x - x * d.x) / hl, (n.y - x * d.y) / hl, (n.z - x * d.z) / hl};
            const double vh = v.x * h.x + v.y * h.y + v.z * h.z;
            const d3 w = {2.0 * vh * h.x - v.x, 2.0 * vh * h.y - v.y, 2.0 * vh * h.z - v.z};
            double cw = w.x * n.x + w.y * n.y + w.z * n.z;
            cw = cw > 0.0 ? cw : 0.0;
            if (cw > 0.0) pyramid_trilinear<KL, DT>(A, w, lodt, cw, acc);
            wsum += cw;
        }
        if (wsum > 0.0) { // else every tap is below the horizon: nothing reflected
#pragma unroll
            for (int k = 0; k < KL + 3; ++k) acc[k] /= wsum;
        }
    } else {
        pyramid_trilinear<KL, DT>(A, wr, sa * (double)(A.M - 1), 1.0, acc);
    }
    const double rgb[3] = {acc[KL], acc[KL + 1], acc[KL + 2]};
    const double EA = lut_bilinear((const float *)A.lut_E, 2, 0, mu, sa);
    const double EB = lut_bilinear((const float *)A.lut_E, 2, 1, mu, sa);

    // Sec. 4 Eq. (probhk) with Sec. 5 Eq. (rtiblndf); the normalisation of
    // Eq. (iblglints:fin) uses these (unattenuated) probabilities
    double p[K];
    double den = 0.0;
    if constexpr (PC) {
        p[1] = A.gamma;
        den = A.gamma;
    } else {
        double F[K];
        if constexpr (SURR) {
#pragma unroll
            for (int k = 0; k < K; ++k) F[k] = (double)A.F[i * K + k];
        } else {
#pragma unroll
            for (int k = 0; k < K; ++k) F[k] = acc[k];
        }
        double sumF = 0.0;
#pragma unroll
        for (int k = 0; k < K; ++k) sumF += F[k];
        const double S = lut_bilinear((const float *)A.lut_S, 1, 0, mu, sa);
        const double scale = sumF > 0.0 ? S / sumF : 0.0;
#pragma unroll
        for (int k = 1; k < K; ++k) {
            p[k] = scale * F[k];
            den += A.levels[k] * p[k];
        }
    }
    // occlusion attenuates the probabilities (occluded facets join bin 0),
    // not the output
    const double vis = A.g.visibility ? (double)A.g.visibility[i] : 1.0;
    double rest = 0.0;
#pragma unroll
    for (int k = 1; k < K; ++k) {
        p[k] = p[k] * vis;
        rest += p[k];
    }
    p[0] = 1.0 - rest;
    if (A.probs) {
#pragma unroll
        for (int k = 0; k < K; ++k) A.probs[i * K + k] = p[k];
    }

    // footprint lattice: level l0 = floor(log2(area)/2) from the exponent
    int e;
    (void)frexp(area, &e);
    const int l0 = (e - 1) >= 0 ? (e - 1) / 2 : -((-(e - 1) + 1) / 2);
    double lt = 0.5 * log2(area) - (double)l0;
    lt = lt < 0.0 ? 0.0 : (lt > 1.0 ? 1.0 : lt);
    const uint32_t seed_mix = A.seed ^ (surf * 0x9E3779B9u);
    const double uu = (double)A.g.u[i], vv = (double)A.g.v[i];

    double Msum[K];
#pragma unroll
    for (int k = 0; k < K; ++k) Msum[k] = 0.0;
    double Nbar = NP; // the normalisation's count
    FootGrid fg;
    if constexpr (V == 12) {
        fg = footprint_grid((double)A.g.dudx[i], (double)A.g.dudy[i], (double)A.g.dvdx[i], (double)A.g.dvdy[i]);
        if (!fg.valid) { // no footprint: nothing is drawn
            A.radiance[3 * i] = 0.0f; A.radiance[3 * i + 1] = 0.0f; A.radiance[3 * i + 2] = 0.0f;
            if (A.counts) for (int k = 0; k < V * K; ++k) A.counts[i * V * K + k] = 0.0;
            if (A.codes) for (int k = 0; k < V * (K - 1); ++k) A.codes[i * V * (K - 1) + k] = 0;
            return;
        }
    }
    // the 6 and 12 draws run in a loop (code size: measured faster than
    // unrolled copies of the tree)
#pragma unroll 1
    for (int vi = 0; vi < V; ++vi) {
        int lev = 0;
        int64_t a, b;
        double w;
        double Nv = NP;
        uint32_t key;
        if constexpr (V == 12) {
            const int ti = vi / 3, corner = vi % 3;
            // the cell vertex's entries by selection (static indices: no
            // private array for the runtime index)
            const int gl = ti == 0 ? fg.l[0] : (ti == 1 ? fg.l[1] : (ti == 2 ? fg.l[2] : fg.l[3]));
            const int ga = ti == 0 ? fg.a[0] : (ti == 1 ? fg.a[1] : (ti == 2 ? fg.a[2] : fg.a[3]));
            const int go = ti == 0 ? fg.o[0] : (ti == 1 ? fg.o[1] : (ti == 2 ? fg.o[2] : fg.o[3]));
            const double gw = ti == 0 ? fg.wt[0] : (ti == 1 ? fg.wt[1] : (ti == 2 ? fg.wt[2] : fg.wt[3]));
            const double li = ldexp(1.0, gl), Ai = ldexp(1.0, ga);
            const double thi = (double)go * (M_PI / 8.0);
            const double ratio = (li * li / Ai) / (fg.smaj * fg.sminc);
            key = (((uint32_t)gl & 0xFFu) << 24) | (((uint32_t)ga & 0xFu) << 20) | (((uint32_t)go & 0xFu) << 16);
            const double cs = cos(thi), sn = sin(thi);
            const double X = (cs * uu + sn * vv) / li;
            const double Y = (cs * vv - sn * uu) * Ai / li;
            const double fxl = floor(X), fyl = floor(Y);
            const double fx = X - fxl, fy = Y - fyl;
            const int64_t ix = (int64_t)fxl, iy = (int64_t)fyl;
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
            w = gw * bw;
            Nv = NP * ratio;
            Nbar = vi == 0 ? w * Nv : Nbar + w * Nv;
        } else if (V == 1) {
            lev = l0;
            a = (int64_t)floor(ldexp(uu, -lev) + 0.5);
            b = (int64_t)floor(ldexp(vv, -lev) + 0.5);
            w = 1.0;
        } else {
            const int side = vi / 3, corner = vi % 3;
            lev = l0 + side;
            const double x = ldexp(uu, -lev), y = ldexp(vv, -lev);
            const double fxl = floor(x), fyl = floor(y);
            const double fx = x - fxl, fy = y - fyl;
            const int64_t ix = (int64_t)fxl, iy = (int64_t)fyl;
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
        if constexpr (V != 12) key = ((uint32_t)lev & 0xFFFFu) << 16;
        double Mv[K];
        uint8_t *cod = A.codes ? (uint8_t *)A.codes + (i * V + vi) * (K - 1) : nullptr;
        if constexpr (CH)
            multinomial_chain<K, SG, SYM>(Nv, p, seed_mix, key, a, b, (const double *)A.qtail, A.exact_gating != 0,
                                     A.sampler, Mv, cod);
        else
            multinomial<K, SG, SYM>(Nv, p, seed_mix, key, a, b, (const double *)A.qtail, A.exact_gating != 0, A.sampler,
                               Mv, cod);
#pragma unroll
        for (int k = 0; k < K; ++k) Msum[k] += w * Mv[k];
        if (A.counts) {
#pragma unroll
            for (int k = 0; k < K; ++k) A.counts[(i * V + vi) * K + k] = Mv[k];
        }
    }

    // Sec. 4 Eq. (iblglints:fin)
    double num = 0.0;
    if constexpr (PC) {
        num = Msum[1];
    } else {
#pragma unroll
        for (int k = 1; k < K; ++k) num += A.levels[k] * Msum[k];
    }
    den *= Nbar;
    const double gmod = (num > 0.0 && den > 0.0) ? num / den : 0.0;
    const double f0[3] = {(double)A.g.f0r[i], (double)A.g.f0g[i], (double)A.g.f0b[i]};
#pragma unroll
    for (int c = 0; c < 3; ++c) A.radiance[3 * i + c] = (float)((f0[c] * EA + EB) * rgb[c] * gmod);
}

// The footprint grid and the anisotropic lookup carry more state per lane;
// asking for two waves per SIMD keeps them at <= 256 registers.
template <int K, int DT, int V, bool SURR = false, bool SG = false, bool PC = false, bool AN = false,
          bool CH = false, bool SYM = false>
__global__ void __launch_bounds__(kShadeThreads, (V == 12 || AN) ? 2 : 1) k_shade(ShadeArgs A)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= A.P) return;
    shade_pixel<K, DT, V, SURR, SG, PC, AN, CH, SYM>(A, i);
}

// All views of one (K, V) group in one launch: block b shades tile b of the
// concatenated views (tile = blockDim.x pixels); tile0[v] is the first tile
// of view v (ascending), so the view is found by a scan of <= n_views entries.
template <int K, int DT, int V, bool SURR = false>
__global__ void __launch_bounds__(kShadeThreads, 1) k_shade_views(const ShadeArgs *__restrict__ views,
                                                     const int64_t *__restrict__ tile0, int n_views)
{
    __shared__ int s_view;
    const int64_t b = blockIdx.x;
    if (threadIdx.x < 64) {
        // the view is the number of views v >= 1 whose first tile is <= b
        // (tile0 ascending, tile0[0] = 0): one load per lane and a ballot
        // per 64 views instead of a serial scan
        int v = 0;
        for (int base = 1; base < n_views; base += 64) {
            const int u = base + (int)threadIdx.x;
            v += __popcll(__ballot(u < n_views && tile0[u] <= b));
        }
        if (threadIdx.x == 0) s_view = v;
    }
    __syncthreads();
    // uniform across the block: the view's arguments go to scalar registers
    const ShadeArgsG A = reinterpret_cast<const ShadeArgsG *>(views)[__builtin_amdgcn_readfirstlane(s_view)];
    const int64_t i = (b - tile0[s_view]) * blockDim.x + threadIdx.x;
    if (i >= A.P) return;
    shade_pixel<K, DT, V, SURR, false, false, false, false, false, ShadeArgsG>(A, i);
}

// SYM: the dual gate with the bias on both powers (the sampler decides
// which instantiation runs; the single-gated kernels exist once, SYM false).
template <int K, int DT, bool SYM>
static hipError_t launch_shade_kd(const ShadeArgs &a, int V, hipStream_t stream)
{
    const unsigned blocks = (unsigned)((a.P + kShadeThreads - 1) / kShadeThreads);
    if (V == 12) {
        // footprint grid: float32 pyramid, dual gate, one lookup (the API checks)
        if constexpr (DT == 0) {
            GLINT_LAUNCH("k_shade", (k_shade<K, 0, 12, false, false, false, false, false, SYM>), dim3(blocks),
                         dim3(kShadeThreads), 0, stream, a);
            return hipGetLastError();
        }
        return hipErrorInvalidValue;
    }
    if (a.lobe_taps > 0) {
        // anisotropic lookups: float32 pyramid, dual gate (the API checks)
        if constexpr (DT == 0) {
            if (V == 1)
                GLINT_LAUNCH("k_shade", (k_shade<K, 0, 1, false, false, false, true, false, SYM>), dim3(blocks),
                             dim3(kShadeThreads), 0, stream, a);
            else
                GLINT_LAUNCH("k_shade", (k_shade<K, 0, 6, false, false, false, true, false, SYM>), dim3(blocks),
                             dim3(kShadeThreads), 0, stream, a);
            return hipGetLastError();
        }
        return hipErrorInvalidValue;
    }
    if (a.sampler == GLINT_SAMPLER_SINGLE || a.sampler == GLINT_SAMPLER_SINGLE_FLOOR) {
        // single-gated forms: float32 pyramids only (the API checks)
        if constexpr (DT == 0 && !SYM) {
            if (V == 1)
                GLINT_LAUNCH("k_shade", (k_shade<K, 0, 1, false, true>), dim3(blocks), dim3(kShadeThreads), 0, stream, a);
            else
                GLINT_LAUNCH("k_shade", (k_shade<K, 0, 6, false, true>), dim3(blocks), dim3(kShadeThreads), 0, stream, a);
            return hipGetLastError();
        }
        return hipErrorInvalidValue;
    }
    if (V == 1)
        GLINT_LAUNCH("k_shade", (k_shade<K, DT, 1, false, false, false, false, false, SYM>), dim3(blocks),
                     dim3(kShadeThreads), 0, stream, a);
    else
        GLINT_LAUNCH("k_shade", (k_shade<K, DT, 6, false, false, false, false, false, SYM>), dim3(blocks),
                     dim3(kShadeThreads), 0, stream, a);
    return hipGetLastError();
}

size_t shade_args_bytes() { return sizeof(ShadeArgs); }

// Fills the device-side descriptor of one view (host memory, copied later).
void make_shade_args(void *out, const glint_gbuffer &g, int64_t P, const glint_env &env,
                     const glint_shade_params &sp, float *radiance, const float *F)
{
    ShadeArgs a;
    a.g = g;
    a.P = P;
    a.ind_pyr = env.ind_pyr;
    a.rgb_pyr = env.rgb_pyr;
    a.levels = env.levels;
    a.lut_S = env.lut_S;
    a.lut_E = env.lut_E;
    a.R = env.R;
    a.M = env.num_mips;
    a.seed = sp.seed;
    a.radiance = radiance;
    a.counts = nullptr;
    a.codes = nullptr;
    a.probs = nullptr;
    a.F = F;
    a.qtail = env.quantile_tail;
    a.exact_gating = sp.exact_gating;
    a.sampler = sp.sampler;
    a.gamma = (double)sp.gamma;
    a.lobe_taps = sp.lobe_taps;
    *static_cast<ShadeArgs *>(out) = a;
}

hipError_t launch_shade_views(int K, int dtype, int V, bool surrogate, const void *views, const int64_t *tile0,
                              int n_views, int64_t tiles, int tile_px, hipStream_t stream)
{
    // k_shade_views finds a block's view with its first wave
    if (tile_px < 64 || tile_px % 64 != 0 || tile_px > kShadeThreads) return hipErrorInvalidValue;
    const ShadeArgs *va = static_cast<const ShadeArgs *>(views);
    if (surrogate) {
        // the indicator pyramid is not read, so its storage type does not matter
#define GLINT_SVS(KK, VV)                                                                                    \
    if (K == KK && V == VV) {                                                                                \
        GLINT_LAUNCH("k_shade_views", (k_shade_views<KK, 0, VV, true>), dim3((unsigned)tiles), dim3(tile_px), \
                     0, stream, va, tile0, n_views);                                                         \
        return hipGetLastError();                                                                            \
    }
        GLINT_SVS(2, 1) GLINT_SVS(4, 1) GLINT_SVS(8, 1) GLINT_SVS(16, 1)
        GLINT_SVS(2, 6) GLINT_SVS(4, 6) GLINT_SVS(8, 6) GLINT_SVS(16, 6)
#undef GLINT_SVS
        return hipErrorInvalidValue;
    }
#define GLINT_SV(KK, DD, VV)                                                                                 \
    if (K == KK && dtype == DD && V == VV) {                                                                 \
        GLINT_LAUNCH("k_shade_views", (k_shade_views<KK, DD, VV>), dim3((unsigned)tiles), dim3(tile_px), 0,  \
                     stream, va, tile0, n_views);                                                            \
        return hipGetLastError();                                                                            \
    }
#define GLINT_SV_K(KK) GLINT_SV(KK, 0, 1) GLINT_SV(KK, 1, 1) GLINT_SV(KK, 2, 1) GLINT_SV(KK, 3, 1) \
    GLINT_SV(KK, 0, 6) GLINT_SV(KK, 1, 6) GLINT_SV(KK, 2, 6) GLINT_SV(KK, 3, 6)
    GLINT_SV_K(2)
    GLINT_SV_K(4)
    GLINT_SV_K(8)
    GLINT_SV_K(16)
#undef GLINT_SV_K
#undef GLINT_SV
    return hipErrorInvalidValue;
}

hipError_t launch_shade(const glint_gbuffer &g, int64_t P, const glint_env &env, const glint_shade_params &sp,
                        const float *F, float *radiance, const glint_shade_debug *dbg, hipStream_t stream)
{
    ShadeArgs a;
    a.g = g;
    a.P = P;
    a.ind_pyr = env.ind_pyr;
    a.rgb_pyr = env.rgb_pyr;
    a.levels = env.levels;
    a.lut_S = env.lut_S;
    a.lut_E = env.lut_E;
    a.R = env.R;
    a.M = env.num_mips;
    a.seed = sp.seed;
    a.radiance = radiance;
    a.counts = dbg ? dbg->counts : nullptr;
    a.codes = dbg ? dbg->codes : nullptr;
    a.probs = dbg ? dbg->probs : nullptr;
    a.F = F;
    a.qtail = env.quantile_tail;
    a.exact_gating = sp.exact_gating;
    a.sampler = sp.sampler;
    a.gamma = (double)sp.gamma;
    a.lobe_taps = sp.lobe_taps;
    const int K = env.K, DT = (int)env.dtype, V = sp.vertices;
    const bool sym = sp.sampler == GLINT_SAMPLER_DUAL_SYMMETRIC;
    if (sp.tree == GLINT_TREE_CHAIN) {
        // sequential chain: float32 pyramid, dual gate, map probabilities, one
        // lookup, 1 or 6 vertices (the API checks)
        const unsigned blocks = (unsigned)((P + kShadeThreads - 1) / kShadeThreads);
#define GLINT_CH(KK)                                                                                         \
    if (K == KK) {                                                                                           \
        if (V == 1 && !sym)                                                                                  \
            GLINT_LAUNCH("k_shade", (k_shade<KK, 0, 1, false, false, false, false, true>), dim3(blocks),     \
                         dim3(kShadeThreads), 0, stream, a);                                                 \
        else if (V == 1)                                                                                     \
            GLINT_LAUNCH("k_shade", (k_shade<KK, 0, 1, false, false, false, false, true, true>),             \
                         dim3(blocks), dim3(kShadeThreads), 0, stream, a);                                   \
        else if (!sym)                                                                                       \
            GLINT_LAUNCH("k_shade", (k_shade<KK, 0, 6, false, false, false, false, true>), dim3(blocks),     \
                         dim3(kShadeThreads), 0, stream, a);                                                 \
        else                                                                                                 \
            GLINT_LAUNCH("k_shade", (k_shade<KK, 0, 6, false, false, false, false, true, true>),             \
                         dim3(blocks), dim3(kShadeThreads), 0, stream, a);                                   \
        return hipGetLastError();                                                                            \
    }
        GLINT_CH(2)
        GLINT_CH(4)
        GLINT_CH(8)
        GLINT_CH(16)
#undef GLINT_CH
        return hipErrorInvalidValue;
    }
    if (sp.prob_mode == GLINT_PROBS_CONSTANT) {
        // two bins, indicator pyramid not read
        const unsigned blocks = (unsigned)((P + kShadeThreads - 1) / kShadeThreads);
        const bool sg = sp.sampler == GLINT_SAMPLER_SINGLE || sp.sampler == GLINT_SAMPLER_SINGLE_FLOOR;
        if (V == 1 && sym)
            GLINT_LAUNCH("k_shade", (k_shade<2, 0, 1, false, false, true, false, false, true>), dim3(blocks),
                         dim3(kShadeThreads), 0, stream, a);
        else if (V != 1 && sym)
            GLINT_LAUNCH("k_shade", (k_shade<2, 0, 6, false, false, true, false, false, true>), dim3(blocks),
                         dim3(kShadeThreads), 0, stream, a);
        else if (V == 1 && !sg)
            GLINT_LAUNCH("k_shade", (k_shade<2, 0, 1, false, false, true>), dim3(blocks), dim3(kShadeThreads), 0,
                         stream, a);
        else if (V == 1)
            GLINT_LAUNCH("k_shade", (k_shade<2, 0, 1, false, true, true>), dim3(blocks), dim3(kShadeThreads), 0,
                         stream, a);
        else if (!sg)
            GLINT_LAUNCH("k_shade", (k_shade<2, 0, 6, false, false, true>), dim3(blocks), dim3(kShadeThreads), 0,
                         stream, a);
        else
            GLINT_LAUNCH("k_shade", (k_shade<2, 0, 6, false, true, true>), dim3(blocks), dim3(kShadeThreads), 0,
                         stream, a);
        return hipGetLastError();
    }
    if (F) {
        // surrogate form: the indicator pyramid is not read, so its storage type does not matter
        const unsigned blocks = (unsigned)((P + kShadeThreads - 1) / kShadeThreads);
#define GLINT_SF(KK)                                                                                        \
    if (K == KK) {                                                                                          \
        if (sp.sampler == GLINT_SAMPLER_SINGLE || sp.sampler == GLINT_SAMPLER_SINGLE_FLOOR) {               \
            if (V == 1)                                                                                     \
                GLINT_LAUNCH("k_shade_surrogate", (k_shade<KK, 0, 1, true, true>), dim3(blocks),            \
                             dim3(kShadeThreads), 0, stream, a);                                            \
            else                                                                                            \
                GLINT_LAUNCH("k_shade_surrogate", (k_shade<KK, 0, 6, true, true>), dim3(blocks),            \
                             dim3(kShadeThreads), 0, stream, a);                                            \
        } else if (sym && V == 1)                                                                           \
            GLINT_LAUNCH("k_shade_surrogate", (k_shade<KK, 0, 1, true, false, false, false, false, true>),  \
                         dim3(blocks), dim3(kShadeThreads), 0, stream, a);                                  \
        else if (sym)                                                                                       \
            GLINT_LAUNCH("k_shade_surrogate", (k_shade<KK, 0, 6, true, false, false, false, false, true>),  \
                         dim3(blocks), dim3(kShadeThreads), 0, stream, a);                                  \
        else if (V == 1)                                                                                    \
            GLINT_LAUNCH("k_shade_surrogate", (k_shade<KK, 0, 1, true>), dim3(blocks), dim3(kShadeThreads), \
                         0, stream, a);                                                                     \
        else                                                                                                \
            GLINT_LAUNCH("k_shade_surrogate", (k_shade<KK, 0, 6, true>), dim3(blocks), dim3(kShadeThreads), \
                         0, stream, a);                                                                     \
        return hipGetLastError();                                                                           \
    }
        GLINT_SF(2)
        GLINT_SF(4)
        GLINT_SF(8)
        GLINT_SF(16)
#undef GLINT_SF
        return hipErrorInvalidValue;
    }
#define GLINT_SH(KK, DD)                                                                                     \
    if (K == KK && DT == DD)                                                                                 \
        return sym ? launch_shade_kd<KK, DD, true>(a, V, stream) : launch_shade_kd<KK, DD, false>(a, V, stream);
#define GLINT_SH_K(KK) GLINT_SH(KK, 0) GLINT_SH(KK, 1) GLINT_SH(KK, 2) GLINT_SH(KK, 3)
    GLINT_SH_K(2)
    GLINT_SH_K(4)
    GLINT_SH_K(8)
    GLINT_SH_K(16)
#undef GLINT_SH_K
#undef GLINT_SH
    return hipErrorInvalidValue;
}

// One binomial draw per element with given random words (the sampler of
// every tree node, exposed for distribution checks and timing).
__global__ void __launch_bounds__(256) k_sample_binomial(int sampler, int exact_gating, const double *__restrict__ N,
                                                         const double *__restrict__ p, const uint32_t *__restrict__ h1,
                                                         const uint32_t *__restrict__ h2, int64_t count,
                                                         const double *__restrict__ qtail, double *__restrict__ n,
                                                         double *__restrict__ nb, uint8_t *__restrict__ code)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const uint32_t b = h2[i];
    double a, c;
    uint32_t cd;
    if (sampler == GLINT_SAMPLER_DUAL)
        node_sample<false>(sampler, N[i], p[i], 1.0 - p[i], hash_unit(h1[i]), hash_unit(b), b >> 9, qtail,
                           exact_gating != 0, a, c, cd);
    else if (sampler == GLINT_SAMPLER_DUAL_SYMMETRIC)
        node_sample<false, true>(sampler, N[i], p[i], 1.0 - p[i], hash_unit(h1[i]), hash_unit(b), b >> 9, qtail,
                                 exact_gating != 0, a, c, cd);
    else
        node_sample<true>(sampler, N[i], p[i], 1.0 - p[i], hash_unit(h1[i]), hash_unit(b), b >> 9, qtail,
                          exact_gating != 0, a, c, cd);
    n[i] = a;
    nb[i] = c;
    code[i] = (uint8_t)cd;
}

hipError_t launch_sample_binomial(int sampler, int exact_gating, const double *N, const double *p, const uint32_t *h1,
                                  const uint32_t *h2, int64_t count, const double *qtail, double *n, double *nb,
                                  uint8_t *code, hipStream_t stream)
{
    const int64_t blocks = (count + 255) / 256;
    if (blocks > 0x7FFFFFFF) return hipErrorInvalidValue;
    GLINT_LAUNCH("k_sample_binomial", k_sample_binomial, dim3((unsigned)blocks), dim3(256), 0, stream, sampler,
                 exact_gating, N, p, h1, h2, count, qtail, n, nb, code);
    return hipGetLastError();
}

} // namespace glint
