// Environment partition: radiance levels and fuzzy indicators (Sec. 5,
// "Discrete Radiance Levels" and "Fuzzy Indicator Functions",
// Eq. (wkdefpractice)).
//
// Two launches, no atomics, no host round trip:
//   k_minmax     grid-stride luminance min/max, one (min, max) pair per block;
//   k_indicators every block re-reduces the pairs (<= 1024, from L2), builds
//                the K levels in LDS (block 0 also stores them) and writes the
//                packed indicator (j, t) of its texels.
// Luminance and levels are double; the partition is HBM-bound (12 B read
// twice + 5 B written per texel).
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

__global__ void __launch_bounds__(kPartThreads) k_indicators(const float *__restrict__ env, int64_t n,
                                                              const double *__restrict__ pairs, int npairs, int K,
                                                              double ell, int level_mode, int weight_space,
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
    if (threadIdx.x < K) {
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

hipError_t launch_partition(const float *env, int R, int K, double ell, int level_mode, int weight_space,
                            void *workspace, double *levels, uint8_t *ind_j, float *ind_t, hipStream_t stream)
{
    const int64_t n = 6LL * R * R;
    const int blocks = partition_blocks(R);
    double *pairs = static_cast<double *>(workspace);
    {
        GLINT_LAUNCH("k_minmax", k_minmax, dim3(blocks), dim3(kPartThreads), 0, stream, env, n, pairs);
    }
    {
        GLINT_LAUNCH("k_indicators", k_indicators, dim3(blocks), dim3(kPartThreads), 0, stream, env, n, pairs, blocks, K, ell,
                           level_mode, weight_space, levels, ind_j, ind_t);
    }
    return hipGetLastError();
}

} // namespace glint
