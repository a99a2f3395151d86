// Lookup tables, once per BRDF model: S = E_D / D_H (Sec. 5, "Integrated
// NDF": visible reflecting facet area over the total facet area of
// Sec. 3.2) and the split-sum albedo E_rho = F0 A + B (Sec. 3.4, Eq. (rtibl);
// Schlick Fresnel, height-correlated Smith, Sec. 7).
//
// One workgroup per (sqrt(alpha), mu_o) cell; midpoint quadrature in GGX
// half-vector coordinates s in (0,1): cos^2(theta_h) = s^2/(a^2 + (1-a^2)s^2),
// D dw_h = q(s) ds dphi / pi with q = sqrt(a^2 + (1-a^2) s^2); the azimuths
// whose mirror direction stays above the horizon form one arc |phi| <
// phi_max(s).  S: 4096 nodes in s with the arc length in closed form;
// E_rho: 512 x 64 nodes over (s, phi in the arc).  Double throughout.
#include "device.hpp"
#include "internal.hpp"

namespace glint {

constexpr int kLutThreads = 256;
constexpr int kNsS = 4096;
constexpr int kNsE = 512;
constexpr int kNphiE = 64;
constexpr double kPi = 3.14159265358979323846;

__device__ __forceinline__ double arc_fraction(double mu, double sin_o, double ch, double sh)
{
    const double rhs = mu * (1.0 - 2.0 * ch * ch) / (2.0 * ch);
    const double den = sin_o * sh;
    if (!(den > 0.0)) return rhs < 0.0 ? 1.0 : 0.0;
    const double c = rhs / den;
    if (c <= -1.0) return 1.0;
    if (c >= 1.0) return 0.0;
    return acos(c) / kPi;
}

__device__ __forceinline__ double smith_lambda(double mu, double a2)
{
    const double m2 = mu * mu;
    return 0.5 * (-1.0 + sqrt(1.0 + a2 * (1.0 - m2) / m2));
}

__device__ __forceinline__ double block_sum(double v, double *s_buf)
{
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) s_buf[wave] = v;
    __syncthreads();
    double t = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += s_buf[w];
    return t;
}

__global__ void __launch_bounds__(kLutThreads) k_lut(float *__restrict__ lut_S, float *__restrict__ lut_E)
{
    __shared__ double s_buf[kLutThreads / 64];
    const int cell = blockIdx.x;
    const int ia = cell / kLutN, im = cell % kLutN;
    const double mu = ((double)im + 0.5) / kLutN;
    const double sa = ((double)ia + 0.5) / kLutN;
    const double alpha = sa * sa;
    const double a2 = alpha * alpha;
    const double sin_o = sqrt(1.0 - mu * mu);

    double num = 0.0, den = 0.0;
    for (int i = threadIdx.x; i < kNsS; i += blockDim.x) {
        const double s = ((double)i + 0.5) / kNsS;
        const double q = sqrt(a2 + (1.0 - a2) * s * s);
        const double ch = s / q;
        const double sh = alpha * sqrt(1.0 - s * s) / q;
        num += q * arc_fraction(mu, sin_o, ch, sh);
        den += q;
    }
    num = block_sum(num, s_buf);
    den = block_sum(den, s_buf);

    const double lam_o = smith_lambda(mu, a2);
    double A = 0.0, B = 0.0;
    for (int i = threadIdx.x; i < kNsE; i += blockDim.x) {
        const double s = ((double)i + 0.5) / kNsE;
        const double q = sqrt(a2 + (1.0 - a2) * s * s);
        const double ch = s / q;
        const double sh = alpha * sqrt(1.0 - s * s) / q;
        const double frac = arc_fraction(mu, sin_o, ch, sh);
        if (!(frac > 0.0)) continue;
        const double phimax = frac * kPi;
        const double w = (q / kPi) * (1.0 / kNsE) * (2.0 * phimax / kNphiE);
        for (int b = 0; b < kNphiE; ++b) {
            const double phi = ((double)b + 0.5) / kNphiE * phimax;
            const double vh = sin_o * sh * cos(phi) + mu * ch;
            const double mu_i = 2.0 * vh * ch - mu;
            if (!(mu_i > 0.0) || !(vh > 0.0)) continue;
            const double g2 = 1.0 / (1.0 + lam_o + smith_lambda(mu_i, a2));
            const double x = 1.0 - vh;
            const double fc = x * x * x * x * x;
            const double base = g2 * vh / mu * w;
            A += (1.0 - fc) * base;
            B += fc * base;
        }
    }
    A = block_sum(A, s_buf);
    B = block_sum(B, s_buf);
    if (threadIdx.x == 0) {
        lut_S[cell] = (float)(num / den);
        lut_E[2 * cell] = (float)A;
        lut_E[2 * cell + 1] = (float)B;
    }
}

// Quantile of every tail uniform the hash can produce (see tail_index).
__global__ void __launch_bounds__(256) k_quantile_tail(double *__restrict__ table)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kTailEntries) return;
    const uint32_t h9 = i < (int64_t)kTailLo ? (uint32_t)i : (uint32_t)(i - kTailLo) + kTailHi + 1u;
    const float xi = ((float)h9 + 0.5f) * 1.1920928955078125e-07f;
    const double xd = (double)xi;
    table[i] = ppnd16_tail(xd, xd - 0.5);
}

hipError_t launch_quantile_table(double *table, hipStream_t stream)
{
    GLINT_LAUNCH("k_quantile_tail", k_quantile_tail, dim3((unsigned)((kTailEntries + 255) / 256)), dim3(256), 0,
                 stream, table);
    return hipGetLastError();
}

hipError_t launch_luts(float *lut_S, float *lut_E, hipStream_t stream)
{
    GLINT_LAUNCH("k_lut", k_lut, dim3(kLutN * kLutN), dim3(kLutThreads), 0, stream, lut_S, lut_E);
    return hipGetLastError();
}

} // namespace glint
