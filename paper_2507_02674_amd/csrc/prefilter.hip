// Environment prefilter of the K indicator channels and RGB (Sec. 5,
// "Integrated NDF", Eq. (rtiblndf), with the real-time IBL kernel of
// Sec. 3.4, Eq. (rtibl), n = v = r).
//
// Source mip chain: level 0 is virtual (dense weights 1-t, t expanded from
// the packed indicator plus RGB from the map); levels >= 1 are stored float
// in CP/4 planes of float4 (CP = K+3 rounded up to 4): plane q of a level
// holds channels 4q..4q+3 of every texel record, so lanes that read
// neighbouring texels of one plane touch a third as many cache lines as with
// 48-byte interleaved records.  Each face has a one-texel border that holds
// the seam rule's value (the adjacent face's texel beyond an edge, the mean
// of the three texels that meet at a corner), so bilinear footprints on
// levels >= 1 never leave the stored face:
//
//   k_chain_tiles   per 32x32 tile of level 0: mip 0 of the output pyramid
//                   (alpha = 0, the dense level) and chain levels 1..5 via
//                   LDS, each level the float-rounded 2x2 mean (double sums
//                   in a fixed order) of the one above;
//   k_chain_level   one level per launch (levels the tiles did not reach
//                   whose parent face is larger than 8 texels, R >= 512);
//   k_chain_finish  the remaining coarse levels of all faces through LDS in
//                   one block, and the border rings of every stored level;
//   k_prefilter     mips >= 1: a group of G lanes per output texel splits
//                   the T taps, sums each tap's trilinear corners in float
//                   and the taps in double, reduces across the group with
//                   cross-lane shuffles; the tap table of the
//                   block's mip lives in LDS.  Blocks are mip-homogeneous and
//                   remapped so consecutive tiles share an XCD's L2.
#include "device.hpp"
#include "internal.hpp"

namespace glint {

constexpr int kChainThreads = 256;
// Tuning knobs of the filter kernels (build-time; results do not depend on
// them beyond the order of the group's double sums).  Measured on the
// 6x256^2, K=8, T=64 frame: 2 lanes per texel with both trilinear levels
// loaded together is the fastest of 1, 2, 4, 8 lanes with and without it
// (the kernel is bound by vector-cache tag throughput, not by the ALUs).
#ifndef GLINT_FILTER_LANES
#define GLINT_FILTER_LANES 2
#endif
#ifndef GLINT_FILTER_MIN_WAVES
#define GLINT_FILTER_MIN_WAVES 1
#endif
#ifndef GLINT_FILTER_LEVEL_UNROLL
#define GLINT_FILTER_LEVEL_UNROLL 1
#endif
constexpr int kFilterThreads = 256;
constexpr int kGroup = GLINT_FILTER_LANES; // lanes per output texel

__host__ __device__ constexpr int chain_stride(int K) { return (K + 3 + 3) & ~3; }

// Records of stored chain level s >= 1 (face size n = R >> s plus border).
__host__ __device__ inline int64_t chain_level_records(int R, int s)
{
    const int64_t n = R >> s;
    return 6 * (n + 2) * (n + 2);
}

// Records before stored level s >= 1 (level 1 starts the chain).
__host__ __device__ inline int64_t chain_level_base(int R, int s)
{
    int64_t o = 0;
    for (int q = 1; q < s; ++q) o += chain_level_records(R, q);
    return o;
}

// Record of texel (x, y), x, y in [-1, n], of `face` within its level.
__host__ __device__ inline int64_t chain_rec(int face, int x, int y, int n)
{
    return ((int64_t)face * (n + 2) + (y + 1)) * (n + 2) + (x + 1);
}

// Floats per float4 plane of a stored level of face size n.
__host__ __device__ inline int64_t chain_plane(int n)
{
    return 6LL * (n + 2) * (n + 2) * 4;
}

// Writes the CP floats of record `rec`.
template <int CP>
__device__ __forceinline__ void store_record(float *__restrict__ lvl, int64_t plane, int64_t rec, const float (&out)[CP])
{
#pragma unroll
    for (int q = 0; q < CP / 4; ++q)
        *reinterpret_cast<float4 *>(lvl + q * plane + rec * 4) =
            make_float4(out[4 * q], out[4 * q + 1], out[4 * q + 2], out[4 * q + 3]);
}

// ---------------------------------------------------------------------------
// storage types of the indicator pyramid
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint16_t f32_to_bf16(float f)
{
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x7FFFFFu)) return (uint16_t)((u >> 16) | 0x40u);
    u += 0x7FFFu + ((u >> 16) & 1u); // round to nearest even
    return (uint16_t)(u >> 16);
}

template <int DT>
__device__ __forceinline__ void store_value(void *base, int64_t i, double v);

template <>
__device__ __forceinline__ void store_value<0>(void *base, int64_t i, double v)
{
    static_cast<float *>(base)[i] = (float)v;
}
template <>
__device__ __forceinline__ void store_value<1>(void *base, int64_t i, double v)
{
    static_cast<_Float16 *>(base)[i] = (_Float16)v;
}
template <>
__device__ __forceinline__ void store_value<2>(void *base, int64_t i, double v)
{
    static_cast<uint16_t *>(base)[i] = f32_to_bf16((float)v);
}
template <>
__device__ __forceinline__ void store_value<3>(void *base, int64_t i, double v)
{
    double c = v < 0.0 ? 0.0 : (v > 1.0 ? 1.0 : v);
    static_cast<uint16_t *>(base)[i] = (uint16_t)rint(c * 65535.0);
}

// ---------------------------------------------------------------------------
// level-0 texel: dense weights + RGB
// ---------------------------------------------------------------------------
template <int K>
struct Level0 {
    const float *env;
    const uint8_t *ind_j;
    const float *ind_t;

    __device__ __forceinline__ void load(int64_t i, double (&v)[K + 3]) const
    {
        const int j = ind_j[i];
        const double t = (double)ind_t[i];
        const double omt = 1.0 - t;
#pragma unroll
        for (int k = 0; k < K; ++k) v[k] = k == j ? omt : (k == j + 1 ? t : 0.0);
        const float *e = env + 3 * i;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const float x = e[c];
            v[K + c] = (__builtin_isfinite(x) && x > 0.0f) ? (double)x : 0.0;
        }
    }

    // acc += w * (dense texel i), without materialising the dense texel
    __device__ __forceinline__ void add(int64_t i, double w, double (&acc)[K + 3]) const
    {
        const int j = ind_j[i];
        const double t = (double)ind_t[i];
        const double wt = w * t, wo = w * (1.0 - t);
#pragma unroll
        for (int k = 0; k < K; ++k) acc[k] += k == j ? wo : (k == j + 1 ? wt : 0.0);
        const float *e = env + 3 * i;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const float x = e[c];
            acc[K + c] += w * ((__builtin_isfinite(x) && x > 0.0f) ? (double)x : 0.0);
        }
    }
};

template <int K>
__device__ __forceinline__ void load_chain(const float *__restrict__ lvl, int64_t plane, int64_t i,
                                           double (&v)[K + 3])
{
    constexpr int CP = chain_stride(K);
    float buf[CP];
#pragma unroll
    for (int q = 0; q < CP / 4; ++q) {
        const float4 f = *reinterpret_cast<const float4 *>(lvl + q * plane + i * 4);
        buf[4 * q] = f.x; buf[4 * q + 1] = f.y; buf[4 * q + 2] = f.z; buf[4 * q + 3] = f.w;
    }
#pragma unroll
    for (int k = 0; k < K + 3; ++k) v[k] = (double)buf[k];
}

// acc += w * (texel (x, y) of `face` on level 0, the virtual level) with the
// seam rule: beyond a cube corner the texel is the mean of the three texels
// meeting there, added as three terms of weight w/3.
template <int K>
__device__ __forceinline__ void accumulate_texel0(const Level0<K> &l0, int face, int x, int y, int n, double w,
                                                  double (&acc)[K + 3])
{
    int64_t idx[3];
    const int cnt = resolve_texel(face, x, y, n, idx);
    const double wc = cnt == 3 ? w / 3.0 : w;
#pragma unroll 1
    for (int e = 0; e < cnt; ++e) l0.add(e == 0 ? idx[0] : (e == 1 ? idx[1] : idx[2]), wc, acc);
}

// ---------------------------------------------------------------------------
// chain level s (>= 1) from level s-1
// ---------------------------------------------------------------------------
template <int K>
__global__ void __launch_bounds__(kChainThreads) k_chain_level(Level0<K> l0, const float *__restrict__ src,
                                                                float *__restrict__ dst, int n)
{
    constexpr int C = K + 3, CP = chain_stride(K);
    const int64_t total = 6LL * n * n;
    const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= total) return;
    const int x = (int)(o % n), y = (int)((o / n) % n), f = (int)(o / ((int64_t)n * n));
    const int m = 2 * n;
    double a[C], b[C], c[C], d[C];
    if (src == nullptr) {
        const int64_t c00 = ((int64_t)f * m + 2 * y) * m + 2 * x;
        l0.load(c00, a); l0.load(c00 + 1, b); l0.load(c00 + m, c); l0.load(c00 + m + 1, d);
    } else {
        const int64_t c00 = chain_rec(f, 2 * x, 2 * y, m), ps = chain_plane(m);
        load_chain<K>(src, ps, c00, a); load_chain<K>(src, ps, c00 + 1, b);
        load_chain<K>(src, ps, c00 + m + 2, c); load_chain<K>(src, ps, c00 + m + 3, d);
    }
    float out[CP];
    {
#pragma clang fp contract(off)
#pragma unroll
        for (int k = 0; k < C; ++k) out[k] = (float)(((a[k] + b[k]) + (c[k] + d[k])) * 0.25);
    }
#pragma unroll
    for (int k = C; k < CP; ++k) out[k] = 0.0f;
    store_record<CP>(dst, chain_plane(n), chain_rec(f, x, y, n), out);
}

// ---------------------------------------------------------------------------
// fused chain: a block owns a T x T tile of level 0 (T = min(32, R)); it
// writes mip 0 of the output pyramid for the tile and builds chain levels
// 1..log2(T) through LDS (each level rounded to float before the next, sums
// in double in a fixed order).  The coarser levels are built the same way by
// later launches.
// ---------------------------------------------------------------------------
constexpr int kTile = 32;

template <int K>
__device__ __forceinline__ void mean4_store(const double (&a)[K + 3], const double (&b)[K + 3],
                                            const double (&c)[K + 3], const double (&d)[K + 3], float *lds_out,
                                            float *__restrict__ gl_lvl, int64_t plane, int64_t rec)
{
    constexpr int C = K + 3, CP = chain_stride(K);
    float out[CP];
    {
#pragma clang fp contract(off)
#pragma unroll
        for (int k = 0; k < C; ++k) out[k] = (float)(((a[k] + b[k]) + (c[k] + d[k])) * 0.25);
    }
#pragma unroll
    for (int k = C; k < CP; ++k) out[k] = 0.0f;
#pragma unroll
    for (int k = 0; k < CP; ++k) lds_out[k] = out[k];
    store_record<CP>(gl_lvl, plane, rec, out);
}

template <int K>
__device__ __forceinline__ void lds_texel(const float *p, double (&v)[K + 3])
{
#pragma unroll
    for (int k = 0; k < K + 3; ++k) v[k] = (double)p[k];
}

// Reduces a square LDS level of side `side` (records of CP floats) into the
// next level (side/2), storing it to LDS `dst` and to the chain level whose
// face-local origin is (ox, oy) with face size n.
template <int K>
__device__ __forceinline__ void reduce_lds_level(const float *src, float *dst, int side, int face, int ox, int oy,
                                                 int n, float *__restrict__ level_base)
{
    constexpr int CP = chain_stride(K);
    const int half = side / 2;
    for (int o = threadIdx.x; o < half * half; o += blockDim.x) {
        const int x = o % half, y = o / half;
        double a[K + 3], b[K + 3], c[K + 3], d[K + 3];
        lds_texel<K>(src + ((2 * y) * side + 2 * x) * CP, a);
        lds_texel<K>(src + ((2 * y) * side + 2 * x + 1) * CP, b);
        lds_texel<K>(src + ((2 * y + 1) * side + 2 * x) * CP, c);
        lds_texel<K>(src + ((2 * y + 1) * side + 2 * x + 1) * CP, d);
        mean4_store<K>(a, b, c, d, dst + o * CP, level_base, chain_plane(n), chain_rec(face, ox + x, oy + y, n));
    }
}

template <int K, int DT>
__global__ void __launch_bounds__(256) k_chain_tiles(Level0<K> l0, int R, int M, float *__restrict__ chain,
                                                     void *__restrict__ ind_pyr, float *__restrict__ rgb_pyr)
{
    constexpr int CP = chain_stride(K);
    __shared__ float s_a[(kTile / 2) * (kTile / 2) * CP];
    __shared__ float s_b[(kTile / 4) * (kTile / 4) * CP];
    const int T = R < kTile ? R : kTile;
    const int tiles = R / T;
    const int face = blockIdx.x / (tiles * tiles);
    const int tx = blockIdx.x % tiles, ty = (blockIdx.x / tiles) % tiles;
    // mip 0 of the pyramid: the dense level, T*T texels of this tile
    for (int o = threadIdx.x; o < T * T; o += blockDim.x) {
        const int x = tx * T + o % T, y = ty * T + o / T;
        const int64_t i = ((int64_t)face * R + y) * R + x;
        double v[K + 3];
        l0.load(i, v);
#pragma unroll
        for (int k = 0; k < K; ++k) store_value<DT>(ind_pyr, i * K + k, v[k]);
        reinterpret_cast<float4 *>(rgb_pyr)[i] = make_float4((float)v[K], (float)v[K + 1], (float)v[K + 2], 0.0f);
    }
    if (M < 2 || T < 2) return;
    // level 1 from level 0
    {
        const int half = T / 2, n1 = R / 2;
        float *base1 = chain; // level 1 starts the chain
        for (int o = threadIdx.x; o < half * half; o += blockDim.x) {
            const int x = o % half, y = o / half;
            const int gx = tx * T + 2 * x, gy = ty * T + 2 * y;
            const int64_t c00 = ((int64_t)face * R + gy) * R + gx;
            double a[K + 3], b[K + 3], c[K + 3], d[K + 3];
            l0.load(c00, a); l0.load(c00 + 1, b); l0.load(c00 + R, c); l0.load(c00 + R + 1, d);
            mean4_store<K>(a, b, c, d, s_a + o * CP, base1, chain_plane(n1),
                           chain_rec(face, tx * half + x, ty * half + y, n1));
        }
    }
    __syncthreads();
    // levels 2.. within the tile, ping-ponging between the two LDS buffers
    int side = T / 2;
    float *src = s_a, *dst = s_b;
    for (int s = 2; s < M && side >= 2; ++s) {
        const int n = R >> s, half = side / 2;
        float *lvl = chain + chain_level_base(R, s) * CP;
        reduce_lds_level<K>(src, dst, side, face, tx * half, ty * half, n, lvl);
        __syncthreads();
        float *t = src; src = dst; dst = t;
        side = half;
    }
}

// Position `pos` in [0, 4n + 4) of a face's border ring -> texel (x, y), x or
// y in {-1, n}: top row (x = -1..n), bottom row, left column, right column.
__device__ __forceinline__ void ring_texel(int pos, int n, int &x, int &y)
{
    if (pos < n + 2) {
        x = pos - 1;
        y = -1;
    } else if (pos < 2 * (n + 2)) {
        x = pos - (n + 2) - 1;
        y = n;
    } else if (pos < 2 * (n + 2) + n) {
        x = -1;
        y = pos - 2 * (n + 2);
    } else {
        x = n;
        y = pos - 2 * (n + 2) - n;
    }
}

// The seam rule's value of a border texel from the interior texels it
// resolves to (cnt = 1: one texel copied; cnt = 3: the float-rounded mean
// ((a + b) + c) / 3 with sums in double).  Plane q of texel e is the float4
// at p_e + q * ps: ps is the plane size in global memory, 4 in LDS records.
// All three records are read whatever cnt is (p1 = p2 = p0 for an edge
// texel), so the reads are issued together.
template <int K>
__device__ __forceinline__ void ring_value(int cnt, const float *p0, const float *p1, const float *p2, int64_t ps,
                                           float (&out)[chain_stride(K)])
{
    constexpr int C = K + 3, CP = chain_stride(K);
    float a[CP], b[CP], c[CP];
#pragma unroll
    for (int q = 0; q < CP / 4; ++q) {
        const float4 u = *reinterpret_cast<const float4 *>(p0 + q * ps);
        const float4 v = *reinterpret_cast<const float4 *>(p1 + q * ps);
        const float4 w = *reinterpret_cast<const float4 *>(p2 + q * ps);
        a[4 * q] = u.x; a[4 * q + 1] = u.y; a[4 * q + 2] = u.z; a[4 * q + 3] = u.w;
        b[4 * q] = v.x; b[4 * q + 1] = v.y; b[4 * q + 2] = v.z; b[4 * q + 3] = v.w;
        c[4 * q] = w.x; c[4 * q + 1] = w.y; c[4 * q + 2] = w.z; c[4 * q + 3] = w.w;
    }
    if (cnt == 1) {
#pragma unroll
        for (int k = 0; k < CP; ++k) out[k] = a[k];
    } else {
#pragma clang fp contract(off)
#pragma unroll
        for (int k = 0; k < C; ++k) out[k] = (float)((((double)a[k] + (double)b[k]) + (double)c[k]) / 3.0);
#pragma unroll
        for (int k = C; k < CP; ++k) out[k] = 0.0f;
    }
}

// Border ring texel r of stored level s (face size n) from the level's
// interior in global memory.
template <int K>
__device__ __forceinline__ void border_from_global(int r, int s, int n, int R, float *__restrict__ chain)
{
    constexpr int CP = chain_stride(K);
    const int face = r / (4 * n + 4);
    int x, y;
    ring_texel(r - face * (4 * n + 4), n, x, y);
    float *lvl = chain + chain_level_base(R, s) * CP;
    int idx[3];
    const int cnt = resolve_texel_edge(face, x, y, n, idx);
    const int lg = __builtin_ctz((unsigned)n);
    const float *p[3];
#pragma unroll
    for (int e = 0; e < 3; ++e) {
        const int i = e < cnt ? idx[e] : idx[0];
        const int f = i >> (2 * lg), rem = i & (n * n - 1);
        p[e] = lvl + chain_rec(f, rem & (n - 1), rem >> lg, n) * 4;
    }
    const int64_t pl = chain_plane(n);
    float out[CP];
    ring_value<K>(cnt, p[0], p[1], p[2], pl, out);
    store_record<CP>(lvl, pl, chain_rec(face, x, y, n), out);
}

// Builds coarse level s (face size n = 2^lg, all six faces) from the level
// above it in LDS (`src`, face size 2n, records of CP floats): texel
// o = (f * n + y) * n + x is the float-rounded mean of its 2x2 texels,
// ((a + b) + (c + d)) / 4 in double, kept in LDS (`dst`) and stored.  Thread
// t of the block takes texels t', t' + 256, ... with t' = t, or with
// t' = 255 - t when `reversed` (so the pass can share the block with a ring
// pass on the low waves).
template <int K>
__device__ __forceinline__ void coarse_reduce(const float *src, float *dst, int lg, float *__restrict__ lvl,
                                              bool reversed)
{
    constexpr int C = K + 3, CP = chain_stride(K);
    const int n = 1 << lg, side = 2 * n;
    const int t = reversed ? (int)blockDim.x - 1 - (int)threadIdx.x : (int)threadIdx.x;
    for (int o = t; o < 6 * n * n; o += blockDim.x) {
        const int f = o >> (2 * lg), rem = o & (n * n - 1), x = rem & (n - 1), y = rem >> lg;
        const float *q = src + ((f * side + 2 * y) * side + 2 * x) * CP;
        double a[C], b[C], c[C], d[C];
        lds_texel<K>(q, a);
        lds_texel<K>(q + CP, b);
        lds_texel<K>(q + side * CP, c);
        lds_texel<K>(q + (side + 1) * CP, d);
        mean4_store<K>(a, b, c, d, dst + o * CP, lvl, chain_plane(n), chain_rec(f, x, y, n));
    }
}

// Border rings of coarse level s (face size n = 2^lg) from its LDS copy.
template <int K>
__device__ __forceinline__ void coarse_rings(const float *lds, int lg, float *__restrict__ lvl)
{
    constexpr int CP = chain_stride(K);
    const int n = 1 << lg;
    const int64_t pl = chain_plane(n);
    for (int r = threadIdx.x; r < 6 * (4 * n + 4); r += blockDim.x) {
        const int face = r / (4 * n + 4);
        int x, y;
        ring_texel(r - face * (4 * n + 4), n, x, y);
        int idx[3];
        const int cnt = resolve_texel_edge(face, x, y, n, idx);
        float out[CP];
        ring_value<K>(cnt, lds + idx[0] * CP, lds + (cnt == 3 ? idx[1] : idx[0]) * CP,
                      lds + (cnt == 3 ? idx[2] : idx[0]) * CP, 4, out);
        store_record<CP>(lvl, pl, chain_rec(face, x, y, n), out);
    }
}

// The rest of the chain after the tiles (and any per-level launches), in one
// launch.  Block 0 (when first < M) loads level first - 1 of all six faces
// (faces of <= 8 texels) into LDS and builds levels first..M-1 there; the
// border rings of a level are written by the low waves while the high waves
// build the next level.  Every other block covers the border rings of levels
// 1..first-1, one ring texel per thread, read from the stored interiors.
// The blocks do not depend on each other.
template <int K>
__global__ void __launch_bounds__(256) k_chain_finish(int R, int M, int first, float *__restrict__ chain)
{
    constexpr int CP = chain_stride(K);
    extern __shared__ float s_dyn[];
    const int coarse_blocks = first < M ? 1 : 0;
    if ((int)blockIdx.x >= coarse_blocks) {
        int r = (int)(blockIdx.x - coarse_blocks) * (int)blockDim.x + (int)threadIdx.x;
        int s = 1, n = R >> 1;
        while (s < first && r >= 6 * (4 * n + 4)) {
            r -= 6 * (4 * n + 4);
            ++s;
            n = R >> s;
        }
        if (s < first) border_from_global<K>(r, s, n, R, chain);
        return;
    }
    const int n0 = R >> (first - 1), lg0 = __builtin_ctz((unsigned)n0);
    const int t0 = 6 * n0 * n0;
    float *src = s_dyn, *dst = s_dyn + t0 * CP;
    {
        // level first-1 (<= 6 * 8 * 8 records) into LDS: every float4 of
        // the thread's share is loaded before any is stored, so the loads
        // are in flight together
        constexpr int kPlanes = CP / 4, kLoads = (6 * 8 * 8 * kPlanes + 255) / 256;
        const float *lvl0 = chain + chain_level_base(R, first - 1) * CP;
        const int64_t pl0 = chain_plane(n0);
        const int total = t0 * kPlanes; // float4 units: texel tex, plane q
        float4 v[kLoads];
        // past the end a lane repeats the last unit (the same value to the
        // same place), so neither loop has a branch that a load could sink into
#pragma unroll
        for (int j = 0; j < kLoads; ++j) {
            const int o = min((int)threadIdx.x + j * 256, total - 1);
            const int tex = o / kPlanes, q = o - tex * kPlanes;
            const int f = tex >> (2 * lg0), rem = tex & (n0 * n0 - 1);
            v[j] = *reinterpret_cast<const float4 *>(lvl0 + q * pl0 + chain_rec(f, rem & (n0 - 1), rem >> lg0, n0) * 4);
        }
#pragma unroll
        for (int j = 0; j < kLoads; ++j) {
            const int o = min((int)threadIdx.x + j * 256, total - 1);
            const int tex = o / kPlanes, q = o - tex * kPlanes;
            *reinterpret_cast<float4 *>(src + tex * CP + q * 4) = v[j];
        }
    }
    __syncthreads();
    coarse_reduce<K>(src, dst, lg0 - 1, chain + chain_level_base(R, first) * CP, false);
    __syncthreads();
    for (int s = first, lg = lg0 - 1; s < M; ++s, --lg) {
        float *t = src; src = dst; dst = t; // src: level s
        coarse_rings<K>(src, lg, chain + chain_level_base(R, s) * CP);
        // the next level reads level s too and writes the buffer of level
        // s - 1, which nothing reads any more
        if (s + 1 < M) coarse_reduce<K>(src, dst, lg - 1, chain + chain_level_base(R, s + 1) * CP, true);
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// filtered mips
// ---------------------------------------------------------------------------
struct Tap {
    double hx, hy, hz, w, lod;
};

struct FilterLaunch {
    int R, M, T;
    int nmips;              // filtered mips (M - 1)
    int block_start[16];    // first logical block of mip 1 + q; block_start[nmips] = total
    int texels[16];         // output texels of mip 1 + q
    int xcd_chunk;          // logical blocks per XCD (grid = 8 * xcd_chunk)
};

__device__ __forceinline__ void make_tap_alpha(int j, double alpha, int M, int T, int R, Tap &tp)
{
    const double a2 = alpha * alpha;
    const double uphi = (double)j / (double)T;
    const double uth = radical_inverse((uint32_t)j);
    const double c2 = (1.0 - uth) / (1.0 + (a2 - 1.0) * uth);
    const double ct = sqrt(c2);
    const double st = sqrt(fmax(0.0, 1.0 - c2));
    double sp, cp;
    sincospi(2.0 * uphi, &sp, &cp);
    tp.hx = st * cp;
    tp.hy = st * sp;
    tp.hz = ct;
    tp.w = fmax(0.0, 2.0 * c2 - 1.0);
    const double den = 1.0 + (a2 - 1.0) * c2;
    const double D = a2 / (3.14159265358979323846 * den * den);
    const double omega_s = 4.0 / ((double)T * D);
    const double omega_p = 4.0 * 3.14159265358979323846 / (6.0 * (double)R * (double)R);
    double lod = 0.5 * log2(omega_s / omega_p) + 1.0;
    lod = lod < 0.0 ? 0.0 : (lod > (double)(M - 1) ? (double)(M - 1) : lod);
    tp.lod = lod;
}

// Tap j of mip m (roughness (m/(M-1))^2).
__device__ __forceinline__ void make_tap(int j, int m, int M, int T, int R, Tap &tp)
{
    const double a = (double)m / (double)(M - 1);
    make_tap_alpha(j, a * a, M, T, R, tp);
}

// Orthonormal basis around the unit direction r (Duff et al. 2017).

// acc += W_j * (trilinear chain lookup at the tap's mirror direction, lod_j).
template <int K>
__device__ __forceinline__ void accumulate_tap(const Tap &tp, const d3 &r, const d3 &t1, const d3 &t2, int R,
                                               const Level0<K> &l0, const float *__restrict__ chain,
                                               const int64_t *lvl_off, double (&acc)[K + 3])
{
    constexpr int C = K + 3, CP = chain_stride(K);
    const d3 h = {tp.hx * t1.x + tp.hy * t2.x + tp.hz * r.x, tp.hx * t1.y + tp.hy * t2.y + tp.hz * r.y,
                  tp.hx * t1.z + tp.hy * t2.z + tp.hz * r.z};
    const d3 l = {2.0 * tp.hz * h.x - r.x, 2.0 * tp.hz * h.y - r.y, 2.0 * tp.hz * h.z - r.z};
    const face_st fs = locate(l);
    const double l0f = floor(tp.lod);
    const int s0 = (int)l0f;
    const double fr = tp.lod - l0f;
    const int nlev = fr > 0.0 ? 2 : 1; // fr > 0 implies s0 + 1 <= M - 1
#if GLINT_FILTER_LEVEL_UNROLL
    if (s0 >= 1) {
        // both stored levels at once (the second repeats the first with weight 0 when lod is whole)
        const int s1 = nlev == 2 ? s0 + 1 : s0;
        const int n0 = R >> s0, n1 = R >> s1;
        const bilin b0 = bilinear_at(fs, n0), b1 = bilinear_at(fs, n1);
        const double lw0 = tp.w * (1.0 - fr), lw1 = tp.w * fr;
        const double w8[8] = {lw0 * ((1.0 - b0.fy) * (1.0 - b0.fx)), lw0 * ((1.0 - b0.fy) * b0.fx),
                              lw0 * (b0.fy * (1.0 - b0.fx)),         lw0 * (b0.fy * b0.fx),
                              lw1 * ((1.0 - b1.fy) * (1.0 - b1.fx)), lw1 * ((1.0 - b1.fy) * b1.fx),
                              lw1 * (b1.fy * (1.0 - b1.fx)),         lw1 * (b1.fy * b1.fx)};
        const float *lv0 = chain + lvl_off[s0], *lv1 = chain + lvl_off[s1];
        const int64_t a0 = chain_rec(fs.face, b0.x0, b0.y0, n0), a1 = chain_rec(fs.face, b1.x0, b1.y0, n1);
        const int64_t p0 = chain_plane(n0), p1 = chain_plane(n1);
        const float *src[8] = {lv0 + a0 * 4, lv0 + (a0 + 1) * 4, lv0 + (a0 + n0 + 2) * 4, lv0 + (a0 + n0 + 3) * 4,
                               lv1 + a1 * 4, lv1 + (a1 + 1) * 4, lv1 + (a1 + n1 + 2) * 4, lv1 + (a1 + n1 + 3) * 4};
        float4 raw[8][CP / 4];
#pragma unroll
        for (int c = 0; c < 8; ++c)
#pragma unroll
            for (int q4 = 0; q4 < CP / 4; ++q4)
                raw[c][q4] = *reinterpret_cast<const float4 *>(src[c] + q4 * (c < 4 ? p0 : p1));
        // the tap's eight weighted corners are summed in float (eight
        // non-negative terms, weights rounded once: relative error below
        // 9 * 2^-24), the taps in double
        float tsum[C];
#pragma unroll
        for (int k = 0; k < C; ++k) tsum[k] = 0.0f;
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const float *f = reinterpret_cast<const float *>(raw[c]);
            const float wf = (float)w8[c];
#pragma unroll
            for (int k = 0; k < C; ++k) tsum[k] = __builtin_fmaf(wf, f[k], tsum[k]);
        }
#pragma unroll
        for (int k = 0; k < C; ++k) acc[k] += (double)tsum[k];
        return;
    }
#endif
#pragma unroll 1
    for (int li = 0; li < nlev; ++li) {
        const int s = s0 + li;
        const int ns = R >> s;
        const bilin bl = bilinear_at(fs, ns);
        const double lw = tp.w * (li ? fr : 1.0 - fr);
        const double w4[4] = {lw * ((1.0 - bl.fy) * (1.0 - bl.fx)), lw * ((1.0 - bl.fy) * bl.fx),
                              lw * (bl.fy * (1.0 - bl.fx)), lw * (bl.fy * bl.fx)};
        const float *lvl = chain + lvl_off[s]; // global pointer arithmetic: global loads
        if (s > 0) {
            // stored level: the bordered face holds the whole footprint
            const int64_t t0 = chain_rec(fs.face, bl.x0, bl.y0, ns), pl = chain_plane(ns);
            const int64_t tt[4] = {t0, t0 + 1, t0 + ns + 2, t0 + ns + 3};
            float4 raw[4][CP / 4];
#pragma unroll
            for (int c = 0; c < 4; ++c)
#pragma unroll
                for (int q4 = 0; q4 < CP / 4; ++q4)
                    raw[c][q4] = *reinterpret_cast<const float4 *>(lvl + q4 * pl + tt[c] * 4);
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const float *f = reinterpret_cast<const float *>(raw[c]);
#pragma unroll
                for (int k = 0; k < C; ++k) acc[k] += w4[c] * (double)f[k];
            }
        } else if (bl.x0 >= 0 && bl.x0 + 1 < ns && bl.y0 >= 0 && bl.y0 + 1 < ns) {
            // level 0 (virtual), footprint inside the face
            const int64_t t0 = ((int64_t)fs.face * ns + bl.y0) * ns + bl.x0;
            const int64_t tt[4] = {t0, t0 + 1, t0 + ns, t0 + ns + 1};
#pragma unroll
            for (int c = 0; c < 4; ++c) l0.add(tt[c], w4[c], acc);
        } else {
            // level 0 across a seam: one copy of the seam rule
#pragma unroll 1
            for (int c = 0; c < 4; ++c)
                accumulate_texel0<K>(l0, fs.face, bl.x0 + (c & 1), bl.y0 + (c >> 1), ns,
                                     c == 0 ? w4[0] : (c == 1 ? w4[1] : (c == 2 ? w4[2] : w4[3])), acc);
        }
    }
}

template <int K, int DT>
__global__ void __launch_bounds__(kFilterThreads, GLINT_FILTER_MIN_WAVES) k_prefilter(FilterLaunch fl, Level0<K> l0,
                                                               const float *__restrict__ chain,
                                                               void *__restrict__ ind_pyr,
                                                               float *__restrict__ rgb_pyr)
{
    constexpr int C = K + 3, CP = chain_stride(K);
    extern __shared__ Tap s_taps[];
    __shared__ double s_wsum;
    __shared__ int64_t s_lvl[16]; // float offset of each chain level (0 for level 0)

    // XCD-aware remap: hardware dispatches block b to XCD b % 8; give each
    // XCD a contiguous range of logical blocks (neighbouring texels share
    // source texels in that XCD's L2).  The grid is padded to 8 * xcd_chunk
    // blocks, so this is a bijection; padding blocks land past the last
    // mip's texels and stay inactive.
    const int b = (int)blockIdx.x;
    const int lb = (b % 8) * fl.xcd_chunk + b / 8;
    int q = 0;
    while (q + 1 < fl.nmips && lb >= fl.block_start[q + 1]) ++q;
    const int m = q + 1;
    for (int j = threadIdx.x; j < fl.T; j += blockDim.x) make_tap(j, m, fl.M, fl.T, fl.R, s_taps[j]);
    if (threadIdx.x < fl.M)
        s_lvl[threadIdx.x] = threadIdx.x == 0 ? 0 : chain_level_base(fl.R, threadIdx.x) * CP;
    __syncthreads();
    if (threadIdx.x == 0) {
        double ws = 0.0;
        for (int j = 0; j < fl.T; ++j)
            if (s_taps[j].w > 0.0) ws += s_taps[j].w;
        s_wsum = ws;
    }
    __syncthreads();

    const int n = fl.R >> m;
    const int64_t texel = (int64_t)(lb - fl.block_start[q]) * (kFilterThreads / kGroup) + threadIdx.x / kGroup;
    const int sub = threadIdx.x % kGroup;
    const bool active = texel < fl.texels[q];
    double acc[C];
#pragma unroll
    for (int k = 0; k < C; ++k) acc[k] = 0.0;

    int x = 0, y = 0, f = 0;
    if (active) {
        x = (int)(texel % n);
        y = (int)((texel / n) % n);
        f = (int)(texel / ((int64_t)n * n));
        const double inv = 1.0 / (double)n;
        d3 r = face_dir(f, 2.0 * ((double)x + 0.5) * inv - 1.0, 2.0 * ((double)y + 0.5) * inv - 1.0);
        const double len = sqrt(r.x * r.x + r.y * r.y + r.z * r.z);
        r.x /= len; r.y /= len; r.z /= len;
        d3 t1, t2;
        onb(r, t1, t2);
#pragma unroll 1
        for (int j = sub; j < fl.T; j += kGroup) {
            const Tap tp = s_taps[j];
            if (!(tp.w > 0.0)) continue;
            accumulate_tap<K>(tp, r, t1, t2, fl.R, l0, chain, s_lvl, acc);
        }
    }
    // reduce over the group's lanes
#pragma unroll
    for (int k = 0; k < C; ++k) {
#pragma unroll
        for (int o = kGroup / 2; o >= 1; o >>= 1) acc[k] += __shfl_xor(acc[k], o, kGroup);
    }
    if (active && sub == 0) {
        const double ws = s_wsum;
        const int64_t out = level_offset(fl.R, m) + ((int64_t)f * n + y) * n + x;
#pragma unroll
        for (int k = 0; k < K; ++k) store_value<DT>(ind_pyr, out * K + k, acc[k] / ws);
        reinterpret_cast<float4 *>(rgb_pyr)[out] =
            make_float4((float)(acc[K] / ws), (float)(acc[K + 1] / ws), (float)(acc[K + 2] / ws), 0.0f);
    }
}

// The filter at arbitrary (direction, alpha): the mip quadrature with the
// tap table built per sample (8 lanes per sample; the weight sum is reduced
// across the group).
//   MODE 0: a0 = alpha [n]; out0 = filtered values [n][K+3].
//   MODE 1: a0 = alpha_x, a1 = alpha_y [n], filtered at sqrt(alpha_x alpha_y);
//           out0 = surrogate inputs [n][5], out1 = F_k / sum F [n][K].
//   MODE 2: the lookups of G-buffer pixels (reflection direction
//           2<n,v>n - v and sqrt(alpha_x alpha_y), as shading computes
//           them); out0 = filtered indicator values [n][K] (0 for
//           background pixels).
template <int K, int MODE>
__global__ void __launch_bounds__(kFilterThreads) k_sample_filter(int R, int M, int T, Level0<K> l0,
                                                                   const float *__restrict__ chain,
                                                                   const float *__restrict__ dirs,
                                                                   const float *__restrict__ a0,
                                                                   const float *__restrict__ a1, glint_gbuffer g,
                                                                   int64_t n, float *__restrict__ out0,
                                                                   float *__restrict__ out1)
{
    constexpr int C = K + 3, CP = chain_stride(K);
    __shared__ int64_t s_lvl[16];
    if (threadIdx.x < M) s_lvl[threadIdx.x] = threadIdx.x == 0 ? 0 : chain_level_base(R, threadIdx.x) * CP;
    __syncthreads();
    const int64_t q = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kGroup;
    const int sub = threadIdx.x % kGroup;
    const bool active = q < n && (MODE != 2 || g.surf_id[q] != GLINT_NO_SURFACE);
    double acc[C];
#pragma unroll
    for (int k = 0; k < C; ++k) acc[k] = 0.0;
    double wsum = 0.0;
    d3 r = {0.0, 0.0, 1.0};
    if (active) {
        double alpha;
        if constexpr (MODE == 2) {
            const d3 nn = {(double)g.nx[q], (double)g.ny[q], (double)g.nz[q]};
            const d3 vv = {(double)g.vx[q], (double)g.vy[q], (double)g.vz[q]};
            const double mu = nn.x * vv.x + nn.y * vv.y + nn.z * vv.z;
            r = {2.0 * mu * nn.x - vv.x, 2.0 * mu * nn.y - vv.y, 2.0 * mu * nn.z - vv.z};
            alpha = sqrt((double)g.ax[q] * (double)g.ay[q]);
        } else {
            r = {(double)dirs[3 * q], (double)dirs[3 * q + 1], (double)dirs[3 * q + 2]};
            alpha = MODE == 0 ? (double)a0[q] : sqrt((double)a0[q] * (double)a1[q]);
        }
        const double len = sqrt(r.x * r.x + r.y * r.y + r.z * r.z);
        const d3 u = {r.x / len, r.y / len, r.z / len};
        d3 t1, t2;
        onb(u, t1, t2);
#pragma unroll 1
        for (int j = sub; j < T; j += kGroup) {
            Tap tp;
            make_tap_alpha(j, alpha, M, T, R, tp);
            if (!(tp.w > 0.0)) continue;
            wsum += tp.w;
            accumulate_tap<K>(tp, u, t1, t2, R, l0, chain, s_lvl, acc);
        }
    }
#pragma unroll
    for (int k = 0; k < C; ++k) {
#pragma unroll
        for (int o = kGroup / 2; o >= 1; o >>= 1) acc[k] += __shfl_xor(acc[k], o, kGroup);
    }
    for (int o = kGroup / 2; o >= 1; o >>= 1) wsum += __shfl_xor(wsum, o, kGroup);
    if constexpr (MODE == 2) {
        if (q < n && sub == 0) {
#pragma unroll
            for (int k = 0; k < K; ++k) out0[q * K + k] = active ? (float)(acc[k] / wsum) : 0.0f;
        }
        return;
    }
    if (!active || sub != 0) return;
    if constexpr (MODE == 0) {
#pragma unroll
        for (int k = 0; k < C; ++k) out0[q * C + k] = (float)(acc[k] / wsum);
    } else {
        const double len = sqrt(r.x * r.x + r.y * r.y + r.z * r.z);
        float f[5];
        surrogate_features(r.x / len, r.y / len, r.z / len, (double)a0[q], (double)a1[q], f);
#pragma unroll
        for (int c = 0; c < 5; ++c) out0[q * 5 + c] = f[c];
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < K; ++k) s += acc[k];
#pragma unroll
        for (int k = 0; k < K; ++k) out1[q * K + k] = s > 0.0 ? (float)(acc[k] / s) : 1.0f / (float)K;
    }
}

hipError_t launch_sample_filter(const float *env, const uint8_t *ind_j, const float *ind_t, const void *workspace,
                                int R, int K, int M, int T, int mode, const float *dirs, const float *a0,
                                const float *a1, const glint_gbuffer *g, int64_t n, float *out0, float *out1,
                                hipStream_t stream)
{
    const float *chain = static_cast<const float *>(workspace);
    const unsigned blocks = (unsigned)((n * kGroup + kFilterThreads - 1) / kFilterThreads);
    glint_gbuffer gb{};
    if (g) gb = *g;
#define GLINT_SF(KK)                                                                                          \
    if (K == KK) {                                                                                            \
        Level0<KK> l0{env, ind_j, ind_t};                                                                     \
        if (mode == 0)                                                                                        \
            GLINT_LAUNCH("k_sample_filter", (k_sample_filter<KK, 0>), dim3(blocks), dim3(kFilterThreads), 0,  \
                         stream, R, M, T, l0, chain, dirs, a0, a1, gb, n, out0, out1);                        \
        else if (mode == 1)                                                                                   \
            GLINT_LAUNCH("k_sample_filter", (k_sample_filter<KK, 1>), dim3(blocks), dim3(kFilterThreads), 0,  \
                         stream, R, M, T, l0, chain, dirs, a0, a1, gb, n, out0, out1);                        \
        else                                                                                                  \
            GLINT_LAUNCH("k_filter_pixels", (k_sample_filter<KK, 2>), dim3(blocks), dim3(kFilterThreads), 0,  \
                         stream, R, M, T, l0, chain, dirs, a0, a1, gb, n, out0, out1);                        \
        return hipGetLastError();                                                                             \
    }
    GLINT_SF(2)
    GLINT_SF(4)
    GLINT_SF(8)
    GLINT_SF(16)
#undef GLINT_SF
    return hipErrorInvalidValue;
}

size_t chain_bytes(int R, int K, int M)
{
    return (size_t)chain_level_base(R, M) * chain_stride(K) * sizeof(float);
}

template <int K, int DT>
static hipError_t launch_prefilter_t(const float *env, const uint8_t *ind_j, const float *ind_t, int R, int M,
                                     int T, float *chain, void *ind_pyr, float *rgb_pyr, hipStream_t stream)
{
    Level0<K> l0{env, ind_j, ind_t};
    // mip 0 of the pyramid and chain levels 1..log2(T) per tile, then the
    // coarser chain levels per face
    const int tile = R < kTile ? R : kTile;
    const int tiles = R / tile;
    {
        GLINT_LAUNCH("k_chain_tiles", (k_chain_tiles<K, DT>), dim3(6 * tiles * tiles), dim3(256), 0, stream, l0, R, M, chain,
                           ind_pyr, rgb_pyr);
    }
    int tile_levels = 0;
    while ((1 << (tile_levels + 1)) <= tile) ++tile_levels; // log2(tile)
    // levels the tiles did not build: per-level launches while the parent
    // face is larger than 8 texels, then one launch that computes the rest
    // and writes every border ring
    int first = M;
    for (int s = tile_levels + 1; s < M; ++s) {
        const int parent = R >> (s - 1);
        if (parent <= 8) { // 6 (8^2 + 4^2) records of <= 20 floats: 38 KB of LDS
            first = s;
            break;
        }
        const int n = R >> s;
        const int64_t total = 6LL * n * n;
        const float *src = chain + chain_level_base(R, s - 1) * chain_stride(K);
        float *dst = chain + chain_level_base(R, s) * chain_stride(K);
        GLINT_LAUNCH("k_chain_level", k_chain_level<K>, dim3((unsigned)((total + kChainThreads - 1) / kChainThreads)),
                           dim3(kChainThreads), 0, stream, l0, src, dst, n);
    }
    if (M > 1) {
        int64_t ring = 0;
        for (int s = 1; s < first; ++s) ring += 6LL * (4 * (R >> s) + 4);
        const int coarse_blocks = first < M ? 1 : 0;
        const int n0 = R >> (first - 1);
        const size_t shm = coarse_blocks ? sizeof(float) * (size_t)chain_stride(K) * 6 *
                                               (size_t)(n0 * n0 + (n0 / 2) * (n0 / 2))
                                         : 0;
        GLINT_LAUNCH("k_chain_finish", k_chain_finish<K>, dim3((unsigned)(coarse_blocks + (ring + 255) / 256)),
                     dim3(256), shm, stream, R, M, first, chain);
    }
    if (M > 1) {
        FilterLaunch fl{};
        fl.R = R; fl.M = M; fl.T = T; fl.nmips = M - 1;
        const int per_block = kFilterThreads / kGroup;
        int total = 0;
        for (int q = 0; q < M - 1; ++q) {
            const int n = R >> (q + 1);
            fl.texels[q] = 6 * n * n;
            fl.block_start[q] = total;
            total += (fl.texels[q] + per_block - 1) / per_block;
        }
        fl.block_start[M - 1] = total;
        fl.xcd_chunk = (total + 7) / 8;
        const size_t shm = sizeof(Tap) * (size_t)T;
        GLINT_LAUNCH("k_prefilter", (k_prefilter<K, DT>), dim3(8 * fl.xcd_chunk), dim3(kFilterThreads), shm, stream, fl, l0,
                           chain, ind_pyr, rgb_pyr);
    }
    return hipGetLastError();
}

hipError_t launch_prefilter(const float *env, const uint8_t *ind_j, const float *ind_t, int R, int K, int M, int T,
                            int dtype, void *workspace, void *ind_pyr, float *rgb_pyr, hipStream_t stream)
{
    float *chain = static_cast<float *>(workspace);
#define GLINT_PF(KK, DD)                                                                                     \
    if (K == KK && dtype == DD)                                                                              \
        return launch_prefilter_t<KK, DD>(env, ind_j, ind_t, R, M, T, chain, ind_pyr, rgb_pyr, stream);
#define GLINT_PF_K(KK) GLINT_PF(KK, 0) GLINT_PF(KK, 1) GLINT_PF(KK, 2) GLINT_PF(KK, 3)
    GLINT_PF_K(2)
    GLINT_PF_K(4)
    GLINT_PF_K(8)
    GLINT_PF_K(16)
#undef GLINT_PF_K
#undef GLINT_PF
    return hipErrorInvalidValue;
}

} // namespace glint
