// Environment partition: radiance levels and fuzzy indicators (Sec. 5,
// "Discrete Radiance Levels" and "Fuzzy Indicator Functions",
// Eq. (wkdefpractice)).
//
// Log-lerp levels (the paper's, level_mode 0 and 2): two launches, no
// atomics, no host round trip:
//   k_minmax     grid-stride luminance min/max, one (min, max) pair per block;
//   k_indicators every block re-reduces the pairs (<= 1024, from L2), builds
//                the K levels in LDS (block 0 also stores them) and writes the
//                packed indicator (j, t) of its texels.
// Luminance and levels are double; the partition is HBM-bound (12 B read
// twice + 5 B written per texel).
//
// Quantile levels (level_mode 1): level k is the smallest texel luminance
// whose solid-angle-weighted distribution function reaches k/(K-1).  A radix
// select over the 64-bit patterns of the luminance (non-negative doubles
// order as their bit patterns), one byte per pass, for all K-2 quantiles at
// once: each pass histograms the byte below the prefixes chosen so far
// (quantiles that share a prefix share a histogram), weighted by the texel
// solid angle in fixed point (2^-55 units: integer sums, exact and
// independent of order), and the last block to finish picks each
// quantile's byte.  The solid angles come from a table of one face quadrant
// (the four mirror images of a texel have the same solid angle), rebuilt per
// call.  Launches: k_minmax, k_qinit, 8 x k_qpass, k_indicators.
#include "device.hpp"
#include "internal.hpp"

namespace glint {

constexpr int kPartThreads = 256;

__device__ __forceinline__ double sane(float c)
{
    return (__builtin_isfinite(c) && c > 0.0f) ? (double)c : 0.0;
}

// Rec. 709 luminance, evaluated left to right without contraction.
__device__ __forceinline__ double luminance(const float *p)
{
#pragma clang fp contract(off)
    return 0.2126 * sane(p[0]) + 0.7152 * sane(p[1]) + 0.0722 * sane(p[2]);
}

__device__ __forceinline__ void block_minmax(double &mn, double &mx, double *s_mn, double *s_mx)
{
    for (int o = 32; o >= 1; o >>= 1) {
        mn = fmin(mn, __shfl_xor(mn, o, 64));
        mx = fmax(mx, __shfl_xor(mx, o, 64));
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) { s_mn[wave] = mn; s_mx[wave] = mx; }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < (int)(blockDim.x >> 6); ++w) {
            mn = fmin(mn, s_mn[w]);
            mx = fmax(mx, s_mx[w]);
        }
        s_mn[0] = mn;
        s_mx[0] = mx;
    }
    __syncthreads();
    mn = s_mn[0];
    mx = s_mx[0];
}

__global__ void __launch_bounds__(kPartThreads) k_minmax(const float *__restrict__ env, int64_t n,
                                                          double *__restrict__ pairs)
{
    __shared__ double s_mn[kPartThreads / 64], s_mx[kPartThreads / 64];
    double mn = __builtin_inf(), mx = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double y = luminance(env + 3 * i);
        mn = fmin(mn, y);
        mx = fmax(mx, y);
    }
    block_minmax(mn, mx, s_mn, s_mx);
    if (threadIdx.x == 0) {
        pairs[2 * blockIdx.x] = mn;
        pairs[2 * blockIdx.x + 1] = mx;
    }
}

// ---------------------------------------------------------------------------
// Quantile levels (level_mode 1)

constexpr double kQScale = 36028797018963968.0; // 2^55: fixed-point unit of the solid angles

struct QState {
    unsigned long long W;               // total weight (fixed point)
    unsigned int ticket;                // blocks of the current pass that are done
    int n_groups;                       // distinct prefixes among the quantiles
    unsigned long long prefix[16];      // quantile k: the bytes chosen so far (lower bytes 0)
    unsigned long long below[16];       // weight of the texels below the prefix's range
    int group[16];                      // quantile k -> histogram of its prefix
    unsigned long long gprefix[16];     // prefix of each group
    double lev[16];                     // final levels (after the last pass)
};

struct QLayout {
    size_t state, hist, table, total;
};

__host__ __device__ inline int quadrant_side(int R) { return (R + 1) / 2; }

QLayout quantile_layout(int R)
{
    QLayout q;
    const size_t pairs = ((size_t)16 * kMaxPartitionBlocks + 255) & ~(size_t)255;
    q.state = pairs;
    q.hist = q.state + ((sizeof(QState) + 255) & ~(size_t)255);
    q.table = q.hist + (size_t)16 * 256 * sizeof(unsigned long long);
    const size_t h = (size_t)quadrant_side(R);
    q.total = q.table + h * h * sizeof(unsigned long long);
    return q;
}

__device__ __forceinline__ double corner_F(double s, double t) { return atan2(s * t, sqrt(s * s + t * t + 1.0)); }

// Solid angle of every texel of one face quadrant (x, y < ceil(R/2)) in
// fixed point; block 0 also clears the selection state and histograms.
__global__ void __launch_bounds__(kPartThreads) k_qinit(int R, int K, unsigned long long *__restrict__ table,
                                                         QState *__restrict__ st,
                                                         unsigned long long *__restrict__ hist)
{
    const int h = quadrant_side(R);
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < h * h) {
        const int x = i % h, y = i / h;
        const double inv = 2.0 / (double)R;
        const double s0 = x * inv - 1.0, s1 = (x + 1) * inv - 1.0, t0 = y * inv - 1.0, t1 = (y + 1) * inv - 1.0;
        const double om = corner_F(s1, t1) - corner_F(s0, t1) - corner_F(s1, t0) + corner_F(s0, t0);
        table[i] = (unsigned long long)__double2ull_rn(om * kQScale);
    }
    if (blockIdx.x == 0) {
        for (int b = threadIdx.x; b < 16 * 256; b += blockDim.x) hist[b] = 0ull;
        if (threadIdx.x < 16) {
            st->prefix[threadIdx.x] = 0ull;
            st->below[threadIdx.x] = 0ull;
            st->group[threadIdx.x] = 0;
            st->gprefix[threadIdx.x] = 0ull;
            st->lev[threadIdx.x] = 0.0;
        }
        if (threadIdx.x == 0) {
            st->W = 0ull;
            st->ticket = 0u;
            st->n_groups = 1;
        }
    }
}

__device__ __forceinline__ unsigned long long load_coherent(const unsigned long long *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// One radix-select pass over the byte at bit `shift` (56, 48, ..., 0).
__global__ void __launch_bounds__(kPartThreads) k_qpass(const float *__restrict__ env, int R, int K, int shift,
                                                         const unsigned long long *__restrict__ table,
                                                         QState *__restrict__ st,
                                                         unsigned long long *__restrict__ hist,
                                                         const double *__restrict__ pairs, int npairs, double ell)
{
    __shared__ unsigned long long lh[16][256];
    __shared__ unsigned long long s_gp[16];
    __shared__ int s_ng, s_last;
    __shared__ unsigned long long s_scan[256];
    __shared__ double s_mn[kPartThreads / 64], s_mx[kPartThreads / 64];
    if (threadIdx.x == 0) s_ng = st->n_groups;
    if (threadIdx.x < 16) s_gp[threadIdx.x] = st->gprefix[threadIdx.x];
    __syncthreads();
    const int ng = s_ng;
    for (int b = threadIdx.x; b < ng * 256; b += blockDim.x) lh[b >> 8][b & 255] = 0ull;
    __syncthreads();
    const int h = quadrant_side(R);
    const int64_t n = 6LL * R * R;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const unsigned long long key = (unsigned long long)__double_as_longlong(luminance(env + 3 * i));
        const int64_t rem = i % ((int64_t)R * R);
        const int y = (int)(rem / R), x = (int)(rem % R);
        const int qx = x < R - 1 - x ? x : R - 1 - x, qy = y < R - 1 - y ? y : R - 1 - y;
        const unsigned long long w = table[qy * h + qx];
        const int digit = (int)((key >> shift) & 255ull);
        for (int g = 0; g < ng; ++g) {
            const bool match = shift == 56 || (key >> (shift + 8)) == (s_gp[g] >> (shift + 8));
            if (match) atomicAdd(&lh[g][digit], w);
        }
    }
    __syncthreads();
    for (int b = threadIdx.x; b < ng * 256; b += blockDim.x) {
        const unsigned long long v = lh[b >> 8][b & 255];
        if (v) atomicAdd(&hist[b], v);
    }
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) s_last = atomicAdd(&st->ticket, 1u) == gridDim.x - 1;
    __syncthreads();
    if (!s_last) return;
    __threadfence();
    // last block: pick each quantile's byte.  The state written by earlier
    // launches is read directly; what this block changes lives in LDS until
    // thread 0 writes it back at the end.
    __shared__ unsigned long long s_prefix[16], s_below[16];
    __shared__ unsigned long long s_W;
    const int t = threadIdx.x; // 256 threads, one bin each
    if (t < 16) {
        s_prefix[t] = st->prefix[t];
        s_below[t] = st->below[t];
    }
    if (shift == 56) {
        // every texel matched the empty prefix: the histogram's total is W
        s_scan[t] = load_coherent(&hist[t]);
        __syncthreads();
        for (int o = 128; o >= 1; o >>= 1) {
            if (t < o) s_scan[t] += s_scan[t + o];
            __syncthreads();
        }
        if (t == 0) s_W = s_scan[0];
    } else if (t == 0) {
        s_W = st->W;
    }
    __syncthreads();
    const unsigned long long W = s_W;
    for (int k = 1; k <= K - 2; ++k) {
        const int g = st->group[k];
        s_scan[t] = load_coherent(&hist[g * 256 + t]);
        __syncthreads();
        for (int o = 1; o < 256; o <<= 1) { // inclusive scan (Hillis-Steele)
            const unsigned long long add = t >= o ? s_scan[t - o] : 0ull;
            __syncthreads();
            s_scan[t] += add;
            __syncthreads();
        }
        const unsigned long long below = s_below[k];
        // smallest byte whose cumulative weight reaches k W / (K-1):
        // (K-1)(below + incl) >= k W, exact in 64 bits (W < 2^59, K <= 16)
        const bool reach = (unsigned long long)(K - 1) * (below + s_scan[t]) >= (unsigned long long)k * W;
        const int d = __syncthreads_count(!reach); // reach is monotone in the byte
        if (t == 0) {
            const int dd = d < 255 ? d : 255;
            s_prefix[k] |= (unsigned long long)dd << shift;
            s_below[k] = below + (dd > 0 ? s_scan[dd - 1] : 0ull);
        }
        __syncthreads();
    }
    // every thread clears the bins it read (b = t mod 256)
    for (int b = t; b < 16 * 256; b += blockDim.x) hist[b] = 0ull;
    if (t == 0) {
        st->W = W;
        int ngr = 0;
        unsigned long long gp[16];
        for (int k = 1; k <= K - 2; ++k) {
            int g = 0;
            while (g < ngr && gp[g] != s_prefix[k]) ++g;
            if (g == ngr) gp[ngr++] = s_prefix[k];
            st->group[k] = g;
        }
        for (int g = 0; g < ngr; ++g) st->gprefix[g] = gp[g];
        for (int k = 0; k < 16; ++k) {
            st->prefix[k] = s_prefix[k];
            st->below[k] = s_below[k];
        }
        st->n_groups = ngr > 0 ? ngr : 1;
        st->ticket = 0u;
    }
    if (shift == 0) {
        // final levels, clipped like the log-lerp levels
        double mn = __builtin_inf(), mx = 0.0;
        for (int i = t; i < npairs; i += blockDim.x) {
            mn = fmin(mn, pairs[2 * i]);
            mx = fmax(mx, pairs[2 * i + 1]);
        }
        block_minmax(mn, mx, s_mn, s_mx);
        if (t < K) {
            const double lmin = mn > ell ? mn : ell;
            const double lmax = mx < lmin ? lmin : mx;
            double v;
            if (t == 0) v = 0.0;
            else if (t == K - 1) v = lmax;
            else {
                v = __longlong_as_double((long long)s_prefix[t]);
                v = v < lmin ? lmin : (v > lmax ? lmax : v);
            }
            st->lev[t] = v;
        }
    }
}

__global__ void __launch_bounds__(kPartThreads) k_indicators(const float *__restrict__ env, int64_t n,
                                                              const double *__restrict__ pairs, int npairs, int K,
                                                              double ell, int level_mode, int weight_space,
                                                              const QState *__restrict__ qst,
                                                              double *__restrict__ levels_out,
                                                              uint8_t *__restrict__ ind_j,
                                                              float *__restrict__ ind_t)
{
    __shared__ double s_mn[kPartThreads / 64], s_mx[kPartThreads / 64];
    __shared__ double L[16];
    double mn = __builtin_inf(), mx = 0.0;
    for (int i = threadIdx.x; i < npairs; i += blockDim.x) {
        mn = fmin(mn, pairs[2 * i]);
        mx = fmax(mx, pairs[2 * i + 1]);
    }
    block_minmax(mn, mx, s_mn, s_mx);
    if (level_mode == 1 && threadIdx.x < K) {
        const double v = qst->lev[threadIdx.x];
        L[threadIdx.x] = v;
        if (blockIdx.x == 0) levels_out[threadIdx.x] = v;
    } else if (threadIdx.x < K) {
        const int k = threadIdx.x;
        const double lmin = mn > ell ? mn : ell;
        const double lmax = mx < lmin ? lmin : mx;
        double v;
        if (k == 0) {
            v = 0.0;
        } else if (k == K - 1) {
            v = lmax;
        } else {
            const double f = level_mode == 2 ? (double)(k - 1) / (double)(K - 2) : (double)k / (double)(K - 1);
            const double a = log(lmin), b = log(lmax);
            v = exp(a + f * (b - a));
            v = v > lmax ? lmax : v; // monotone levels when min ~ max
        }
        L[k] = v;
        if (blockIdx.x == 0) levels_out[k] = v;
    }
    __syncthreads();
    const double top = L[K - 1];
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double y = luminance(env + 3 * i);
        y = y > top ? top : y;
        int j = 0;
        for (int k = 1; k <= K - 2; ++k)
            j = L[k] <= y ? k : j;
        const double lo = L[j], hi = L[j + 1];
        double t;
        if (weight_space == 1 && j >= 1) {
            const double dl = log(hi) - log(lo);
            t = dl > 0.0 ? (log(y) - log(lo)) / dl : 1.0;
        } else {
            const double dl = hi - lo;
            t = dl > 0.0 ? (y - lo) / dl : 1.0;
        }
        t = t < 0.0 ? 0.0 : (t > 1.0 ? 1.0 : t);
        ind_j[i] = (uint8_t)j;
        ind_t[i] = (float)t;
    }
}

int partition_blocks(int R)
{
    const int64_t n = 6LL * R * R;
    int64_t b = (n + kPartThreads * 4 - 1) / (kPartThreads * 4);
    return (int)(b < 1 ? 1 : (b > kMaxPartitionBlocks ? kMaxPartitionBlocks : b));
}

size_t partition_workspace_bytes(int R) { return quantile_layout(R).total; }

size_t partition_workspace_bytes_mode(int R, int level_mode)
{
    // the log-lerp modes use the (min, max) pairs only; the selection state
    // that follows them is addressed but not read
    const QLayout q = quantile_layout(R);
    return (level_mode == 1) ? q.total : q.hist;
}

hipError_t launch_partition(const float *env, int R, int K, double ell, int level_mode, int weight_space,
                            void *workspace, double *levels, uint8_t *ind_j, float *ind_t, hipStream_t stream)
{
    const int64_t n = 6LL * R * R;
    const int blocks = partition_blocks(R);
    double *pairs = static_cast<double *>(workspace);
    const QLayout ql = quantile_layout(R);
    char *ws = static_cast<char *>(workspace);
    QState *qst = reinterpret_cast<QState *>(ws + ql.state);
    // two levels have no quantile between them: the same as the log-lerp levels
    const int mode = (level_mode == 1 && K == 2) ? 0 : level_mode;
    {
        GLINT_LAUNCH("k_minmax", k_minmax, dim3(blocks), dim3(kPartThreads), 0, stream, env, n, pairs);
    }
    if (mode == 1) {
        unsigned long long *hist = reinterpret_cast<unsigned long long *>(ws + ql.hist);
        unsigned long long *table = reinterpret_cast<unsigned long long *>(ws + ql.table);
        const int h = quadrant_side(R);
        const unsigned tb = (unsigned)((h * h + kPartThreads - 1) / kPartThreads);
        GLINT_LAUNCH("k_qinit", k_qinit, dim3(tb), dim3(kPartThreads), 0, stream, R, K, table, qst, hist);
        for (int shift = 56; shift >= 0; shift -= 8) {
            GLINT_LAUNCH("k_qpass", k_qpass, dim3(blocks), dim3(kPartThreads), 0, stream, env, R, K, shift, table,
                         qst, hist, pairs, blocks, ell);
        }
    }
    {
        GLINT_LAUNCH("k_indicators", k_indicators, dim3(blocks), dim3(kPartThreads), 0, stream, env, n, pairs, blocks, K, ell,
                           mode, weight_space, qst, levels, ind_j, ind_t);
    }
    return hipGetLastError();
}

} // namespace glint
