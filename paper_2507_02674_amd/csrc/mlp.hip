// Learned surrogate of the indicator pyramid lookup (not from the paper: the
// project's own extension).  A small MLP maps (reflection direction,
// scaled ln alpha_x, ln alpha_y) to the K normalised filtered indicator
// values F_k / sum F; the plain filter provides its training targets.
//
// Network 5 -> 64 -> 64 -> 64 -> K, SiLU hidden units, softmax output.
// Dense layers run on the matrix cores (v_mfma_f32_32x32x16_bf16): bfloat16
// weights and activations, float32 accumulation.  One wave computes a tile
// of 32 rows (samples or pixels) through all layers out of LDS.
//
// Parameter layout (flat float32 master, bfloat16 copy, padded for the
// 32x32x16 tiles): W1 [64][16] (inputs 5..15 zero), b1 [64], W2 [64][64],
// b2 [64], W3 [64][64], b3 [64], W4 [32][64] (rows K..31 zero), b4 [32].
#include "device.hpp"
#include "internal.hpp"

namespace glint {

namespace {

typedef __attribute__((__vector_size__(8 * sizeof(short)))) short bf16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;

constexpr int kH = 64, kIn = 16, kOut = 32;
constexpr int oW1 = 0, ob1 = oW1 + kH * kIn, oW2 = ob1 + kH, ob2 = oW2 + kH * kH, oW3 = ob2 + kH,
              ob3 = oW3 + kH * kH, oW4 = ob3 + kH, ob4 = oW4 + kOut * kH, kParams = ob4 + kOut;

// LDS row strides (bf16 elements).  Rows are read as 16-byte vectors by 32
// lanes; strides of 24, 40 and 72 elements (12, 20, 36 dwords) put any 16
// consecutive rows on disjoint banks.
constexpr int kLdW1 = 24, kLdX = 40, kLdH = 72, kLdO = 40;
constexpr int sW1 = 0, sW2 = sW1 + kH * kLdW1, sW3 = sW2 + kH * kLdH, sW4 = sW3 + kH * kLdH,
              kWLds = sW4 + kOut * kLdH; // bf16 weights staged in LDS (no biases)

// Biases staged in LDS by the inference kernels: b1, b2, b3 (64 each), b4 (32).
constexpr int kBiasLds = 3 * kH + kOut;
// Offset from b1 in the parameter layout of staged bias c (b1, b2, b3 and
// b4 are separated by the weight matrices).
__device__ __forceinline__ int bias_src(int c)
{
    return c < kH ? c : (c < 2 * kH ? (ob2 - ob1) + (c - kH) : (c < 3 * kH ? (ob3 - ob1) + (c - 2 * kH) : (ob4 - ob1) + (c - 3 * kH)));
}

constexpr int kInferWaves = 4;     // waves per block of the inference kernels
constexpr int kInferMaxBlocks = 768; // one round at 3 blocks per CU (256 CUs)

__device__ __forceinline__ uint16_t to_bf16(float f)
{
    return __builtin_bit_cast(uint16_t, (__bf16)f); // round to nearest even (v_cvt_pk_bf16_f32)
}

typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef float f32x2_t __attribute__((ext_vector_type(2)));

// Two floats to two packed bfloat16, a in the low half (one two-source
// v_cvt_pk_bf16_f32, round to nearest even like to_bf16).
__device__ __forceinline__ uint32_t pack_bf16x2(float a, float b)
{
    return __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2_t){a, b}, bf16x2_t));
}

// Four floats to four packed bfloat16 (two conversions of two).
__device__ __forceinline__ uint2 pack_bf16x4(float a, float b, float c, float d)
{
    return make_uint2(pack_bf16x2(a, b), pack_bf16x2(c, d));
}

__device__ __forceinline__ float from_bf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// Logistic function with the hardware exp and reciprocal (a few ulp; the
// result is rounded to bfloat16 or scales a bfloat16 error signal).
__device__ __forceinline__ float sigmoid(float z) { return __builtin_amdgcn_rcpf(1.0f + __expf(-z)); }

__device__ __forceinline__ float silu(float z) { return z * sigmoid(z); }

__device__ __forceinline__ float dsilu(float z)
{
    const float s = sigmoid(z);
    return s * (1.0f + z * (1.0f - s));
}

// acc (32 x 32 tile) += A[r][k] B[k][c] over k in [0, Kd), Kd a multiple of
// 16; A(r, k) = a[r * ars + k * acs], B(k, c) = b[k * brs + c * bcs] (bf16
// bit patterns in LDS).  Lane l supplies A[l%32][8(l/32)+j] and
// B[8(l/32)+j][l%32], j < 8.  AV / BV: the eight values are contiguous
// (acs == 1 / brs == 1, 16-byte aligned) and are read as one vector.
template <bool AV, bool BV>
__device__ __forceinline__ void tile_mma(const uint16_t *a, int ars, int acs, const uint16_t *b, int brs, int bcs,
                                         int Kd, f32x16 &acc)
{
    const int l = threadIdx.x & 63, r = l & 31, kg = (l >> 5) * 8;
    for (int k0 = 0; k0 < Kd; k0 += 16) {
        bf16x8 av, bv;
        if constexpr (AV) {
            av = *reinterpret_cast<const bf16x8 *>(a + r * ars + k0 + kg);
        } else {
#pragma unroll
            for (int j = 0; j < 8; ++j) av[j] = (short)a[r * ars + (k0 + kg + j) * acs];
        }
        if constexpr (BV) {
            bv = *reinterpret_cast<const bf16x8 *>(b + r * bcs + k0 + kg);
        } else {
#pragma unroll
            for (int j = 0; j < 8; ++j) bv[j] = (short)b[(k0 + kg + j) * brs + r * bcs];
        }
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, acc, 0, 0, 0);
    }
}

// Row / column of accumulator i of this lane in the 32 x 32 tile.
__device__ __forceinline__ int acc_row(int i) { return 8 * (i >> 2) + 4 * ((threadIdx.x & 63) >> 5) + (i & 3); }
__device__ __forceinline__ int acc_col() { return threadIdx.x & 31; }

__device__ __forceinline__ void zero(f32x16 &acc)
{
#pragma unroll
    for (int i = 0; i < 16; ++i) acc[i] = 0.0f;
}

// Stages the bf16 weights (16-byte chunks) into LDS; all threads of the block.
__device__ __forceinline__ void stage_weights(const uint16_t *__restrict__ wb, uint16_t *s_w)
{
    constexpr int c1 = kH * kIn / 8, c2 = c1 + kH * kH / 8, c3 = c2 + kH * kH / 8, c4 = c3 + kOut * kH / 8;
    for (int c = threadIdx.x; c < c4; c += blockDim.x) {
        int src, dst;
        if (c < c1) {
            const int n = c >> 1, q = c & 1;
            src = oW1 + n * kIn + 8 * q;
            dst = sW1 + n * kLdW1 + 8 * q;
        } else if (c < c2) {
            const int e = c - c1, n = e >> 3, q = e & 7;
            src = oW2 + n * kH + 8 * q;
            dst = sW2 + n * kLdH + 8 * q;
        } else if (c < c3) {
            const int e = c - c2, n = e >> 3, q = e & 7;
            src = oW3 + n * kH + 8 * q;
            dst = sW3 + n * kLdH + 8 * q;
        } else {
            const int e = c - c3, n = e >> 3, q = e & 7;
            src = oW4 + n * kH + 8 * q;
            dst = sW4 + n * kLdH + 8 * q;
        }
        *reinterpret_cast<uint4 *>(s_w + dst) = *reinterpret_cast<const uint4 *>(wb + src);
    }
}

// Transposed product tile: acc[t] = sum_k W[n0 + u][k] in[r][k] with
// u = 8(t/4) + 4(lane/32) + t%4 and r = lane%32: the weights are the
// first operand and the activations the second, so both are read as
// 16-byte rows, and each lane ends with four runs of four consecutive units
// of one sample (stored as 8-byte bfloat16 quads).
__device__ __forceinline__ void unit_mma(const uint16_t *W, int ldw, const uint16_t *in, int ldi, int Kd, int n0,
                                         f32x16 &acc)
{
    const int l = threadIdx.x & 63, r = l & 31, kg = (l >> 5) * 8;
    for (int k0 = 0; k0 < Kd; k0 += 16) {
        const bf16x8 a = *reinterpret_cast<const bf16x8 *>(W + (n0 + r) * ldw + k0 + kg);
        const bf16x8 b = *reinterpret_cast<const bf16x8 *>(in + r * ldi + k0 + kg);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
    }
}

__device__ __forceinline__ void unit_tile(const uint16_t *W, int ldw, const uint16_t *in, int ldi, int Kd, int n0,
                                          f32x16 &acc)
{
    zero(acc);
    unit_mma(W, ldw, in, ldi, Kd, n0, acc);
}

// unit_tile with each accumulator starting at its unit's bias (bias in LDS,
// indexed by unit): the pre-activation b + sum_k W x leaves the matrix cores
// whole, with no separate additions.
__device__ __forceinline__ void unit_tile_biased(const uint16_t *W, int ldw, const uint16_t *in, int ldi, int Kd,
                                                 int n0, const float *bias, f32x16 &acc)
{
    const int h = (threadIdx.x & 63) >> 5;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const float4 b4 = *reinterpret_cast<const float4 *>(bias + n0 + 8 * q + 4 * h);
        acc[4 * q] = b4.x;
        acc[4 * q + 1] = b4.y;
        acc[4 * q + 2] = b4.z;
        acc[4 * q + 3] = b4.w;
    }
    unit_mma(W, ldw, in, ldi, Kd, n0, acc);
}

// out[r][n] = bf16(silu(in[r][:Kd] . W[n][:Kd] + bias[n])) for the 32 samples
// and 64 units; z[r][n] keeps the float pre-activation when z is non-null.
__device__ __forceinline__ void dense_silu(const uint16_t *in, int ldi, int Kd, const uint16_t *W, int ldw,
                                           const float *__restrict__ bias, uint16_t *out, float *z)
{
    const int r = threadIdx.x & 31, h = (threadIdx.x & 63) >> 5;
#pragma unroll
    for (int n0 = 0; n0 < kH; n0 += 32) {
        f32x16 acc;
        unit_tile(W, ldw, in, ldi, Kd, n0, acc);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int n = n0 + 8 * q + 4 * h;
            const float4 b4 = *reinterpret_cast<const float4 *>(bias + n);
            const float z0 = acc[4 * q] + b4.x, z1 = acc[4 * q + 1] + b4.y, z2 = acc[4 * q + 2] + b4.z,
                        z3 = acc[4 * q + 3] + b4.w;
            if (z) *reinterpret_cast<float4 *>(z + r * kH + n) = make_float4(z0, z1, z2, z3);
            *reinterpret_cast<uint2 *>(out + r * kLdH + n) = pack_bf16x4(silu(z0), silu(z1), silu(z2), silu(z3));
        }
    }
}

// Output layer in registers: logit[4q + i] = h[r][:] . W4[u][:] + b4[u] for
// u = 8q + 4(lane/32) + i (16 of the 32 padded outputs; the lane with the
// other half is lane ^ 32).
__device__ __forceinline__ void dense_out(const uint16_t *hin, const uint16_t *W4, const float *__restrict__ b4,
                                          float (&logit)[16])
{
    f32x16 acc;
    unit_tile_biased(W4, kLdH, hin, kLdH, kH, 0, b4, acc);
#pragma unroll
    for (int j = 0; j < 16; ++j) logit[j] = acc[j];
}

__device__ __forceinline__ int out_unit(int j) { return 8 * (j >> 2) + 4 * ((threadIdx.x & 63) >> 5) + (j & 3); }

// Softmax over the first K outputs of each sample, across the lane pair
// (lane, lane ^ 32): y[j] for this lane's units (0 for units >= K).
__device__ __forceinline__ void softmax_pair(const float (&logit)[16], int K, float (&y)[16])
{
    float mx = -3.4e38f;
#pragma unroll
    for (int j = 0; j < 16; ++j)
        if (out_unit(j) < K) mx = fmaxf(mx, logit[j]);
    mx = fmaxf(mx, __shfl_xor(mx, 32, 64));
    float se = 0.0f;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        y[j] = out_unit(j) < K ? __expf(logit[j] - mx) : 0.0f;
        se += y[j];
    }
    se += __shfl_xor(se, 32, 64);
    const float inv = 1.0f / se;
#pragma unroll
    for (int j = 0; j < 16; ++j) y[j] *= inv;
}

// Per-wave LDS of the inference kernels: one buffer of 32 rows that holds
// the inputs (columns 0..15), then each hidden layer in turn (the output
// layer and softmax stay in registers).  One buffer instead of three keeps
// the block at 3 per CU.
struct InferTile {
    uint16_t h[32 * kLdH];
};

// One hidden layer in place: both 32-unit tiles are computed from the
// buffer before any output is written back into it (the wave's LDS
// operations complete in order).
__device__ __forceinline__ void dense_silu_inplace(uint16_t *buf, int Kd, const uint16_t *W, int ldw,
                                                   const float *__restrict__ bias)
{
    const int r = threadIdx.x & 31, h = (threadIdx.x & 63) >> 5;
    f32x16 acc[2];
    unit_tile_biased(W, ldw, buf, kLdH, Kd, 0, bias, acc[0]);
    unit_tile_biased(W, ldw, buf, kLdH, Kd, 32, bias, acc[1]);
#pragma unroll
    for (int t = 0; t < 2; ++t) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int n = 32 * t + 8 * q + 4 * h;
            *reinterpret_cast<uint2 *>(buf + r * kLdH + n) =
                pack_bf16x4(silu(acc[t][4 * q]), silu(acc[t][4 * q + 1]), silu(acc[t][4 * q + 2]),
                            silu(acc[t][4 * q + 3]));
        }
    }
}

// Per-wave LDS of the training kernel (one wave per block).
struct TrainTile {
    uint16_t x[32 * kLdX];    // inputs, bf16 (cols 5.. zero)
    uint16_t h[3][32 * kLdH]; // h1..h3, bf16
    float z[3][32 * kH];      // z1..z3, float
    uint16_t dz[2][32 * kLdH]; // hidden error signals (ping-pong), bf16
    uint16_t dz4[32 * kLdO];  // output error signal, bf16 (cols K.. zero)
};

} // namespace

// ---------------------------------------------------------------------------
// training: one wave per 32 samples; per-block partial gradients
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(64) k_mlp_grad(const float *__restrict__ x, const float *__restrict__ target,
                                                 const double *__restrict__ levels, float lam, int B, int K,
                                                 const float *__restrict__ w, const uint16_t *__restrict__ wb,
                                                 float *__restrict__ partial, float *__restrict__ loss_partial)
{
    __shared__ __attribute__((aligned(16))) uint16_t s_w[kWLds];
    __shared__ __attribute__((aligned(16))) TrainTile t;
    const int lane = threadIdx.x;
    const int row0 = blockIdx.x * 32;
    stage_weights(wb, s_w);
    for (int i = lane; i < 32 * kLdX; i += 64) {
        const int r = i / kLdX, c = i % kLdX;
        t.x[i] = (c < 5 && row0 + r < B) ? to_bf16(x[(int64_t)(row0 + r) * 5 + c]) : (uint16_t)0;
    }
    __syncthreads();
    const uint16_t *W1 = s_w + sW1, *W2 = s_w + sW2, *W3 = s_w + sW3, *W4 = s_w + sW4;
    dense_silu(t.x, kLdX, kIn, W1, kLdW1, w + ob1, t.h[0], t.z[0]);
    __syncthreads(); // one-wave block: orders the LDS writes before the next layer reads them
    dense_silu(t.h[0], kLdH, kH, W2, kLdH, w + ob2, t.h[1], t.z[1]);
    __syncthreads();
    dense_silu(t.h[1], kLdH, kH, W3, kLdH, w + ob3, t.h[2], t.z[2]);
    __syncthreads();
    // output layer, softmax, loss and the output error signal, in registers
    // (sample r = lane % 32, 16 of its outputs per lane, the other 16 in
    // lane ^ 32): (y - t) / B, plus, with levels, lam (y' - t') / B for the
    // radiance-weighted distributions y'_k = L_k y_k / sum_{j>=1} L_j y_j,
    // t' likewise, over the bins k >= 1
    float logit[16], y[16];
    dense_out(t.h[2], W4, w + ob4, logit);
    softmax_pair(logit, K, y);
    float loss = 0.0f;
    {
        const int r = lane & 31;
        const bool valid = row0 + r < B;
        float tv[16], Lk[16];
        float tws = 0.0f, yws = 0.0f;
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const int o = out_unit(j);
            tv[j] = (o < K && valid) ? target[(int64_t)(row0 + r) * K + o] : 0.0f;
            Lk[j] = (levels && o >= 1 && o < K) ? (float)levels[o] : 0.0f;
            tws += tv[j] * Lk[j];
            yws += y[j] * Lk[j];
        }
        tws += __shfl_xor(tws, 32, 64);
        yws += __shfl_xor(yws, 32, 64);
        const bool rad = levels && valid && tws > 0.0f && yws > 0.0f;
        const float itw = rad ? 1.0f / tws : 0.0f, iyw = rad ? 1.0f / yws : 0.0f;
        float d[16];
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const int o = out_unit(j);
            d[j] = 0.0f;
            if (o < K && valid) {
                const float tk = tv[j];
                float dj = y[j] - tk;
                loss -= tk * logf(fmaxf(y[j], 1e-30f));
                if (rad && o >= 1) {
                    const float yp = y[j] * Lk[j] * iyw, tp = tk * Lk[j] * itw;
                    dj += lam * (yp - tp);
                    loss -= lam * tp * logf(fmaxf(yp, 1e-30f));
                }
                d[j] = dj / (float)B;
            }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q)
            *reinterpret_cast<uint2 *>(t.dz4 + r * kLdO + out_unit(4 * q)) =
                pack_bf16x4(d[4 * q], d[4 * q + 1], d[4 * q + 2], d[4 * q + 3]);
    }
    __syncthreads();
    float *P = partial + (int64_t)blockIdx.x * kParams;

    // output layer: dW4[n][k] = sum_r dz4[r][n] h3[r][k]; db4[n] = sum_r dz4[r][n]
#pragma unroll 1
    for (int k0 = 0; k0 < kH; k0 += 32) {
        f32x16 acc;
        zero(acc);
        tile_mma<false, false>(t.dz4, 1, kLdO, t.h[2] + k0, kLdH, 1, 32, acc);
#pragma unroll
        for (int i = 0; i < 16; ++i) P[oW4 + acc_row(i) * kH + k0 + acc_col()] = acc[i];
    }
    if (lane < kOut) {
        float s = 0.0f;
        for (int r = 0; r < 32; ++r) s += from_bf16(t.dz4[r * kLdO + lane]);
        P[ob4 + lane] = s;
    }
    // dz3 = (dz4 W4) * silu'(z3)
#pragma unroll 1
    for (int n0 = 0; n0 < kH; n0 += 32) {
        f32x16 acc;
        zero(acc);
        tile_mma<true, false>(t.dz4, kLdO, 1, W4 + n0, kLdH, 1, kOut, acc);
        const int n = n0 + acc_col();
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int r = acc_row(i);
            t.dz[0][r * kLdH + n] = to_bf16(acc[i] * dsilu(t.z[2][r * kH + n]));
        }
    }
    __syncthreads();
    // hidden layers 3, 2, 1
    const uint16_t *Wl[3] = {W1, W2, W3};
    const int ldw[3] = {kLdW1, kLdH, kLdH};
    const int oW[3] = {oW1, oW2, oW3}, ob[3] = {ob1, ob2, ob3};
    int cur = 0;
#pragma unroll 1
    for (int layer = 2; layer >= 0; --layer) {
        const uint16_t *dzl = t.dz[cur];
        const uint16_t *in = layer == 0 ? t.x : t.h[layer - 1];
        const int in_ld = layer == 0 ? kLdX : kLdH;
        const int in_n = layer == 0 ? kIn : kH; // columns of W_layer
        // dW[n][k] = sum_r dz[r][n] in[r][k]
#pragma unroll 1
        for (int m0 = 0; m0 < kH; m0 += 32) {
#pragma unroll 1
            for (int k0 = 0; k0 < in_n; k0 += 32) {
                f32x16 acc;
                zero(acc);
                tile_mma<false, false>(dzl + m0, 1, kLdH, in + k0, in_ld, 1, 32, acc);
                const int k = k0 + acc_col();
#pragma unroll
                for (int i = 0; i < 16; ++i) {
                    const int n = m0 + acc_row(i);
                    if (k < in_n) P[oW[layer] + n * in_n + k] = acc[i];
                }
            }
        }
        {
            float s = 0.0f; // 64 units, one per lane
            for (int r = 0; r < 32; ++r) s += from_bf16(dzl[r * kLdH + lane]);
            P[ob[layer] + lane] = s;
        }
        if (layer > 0) {
            // dz_{layer-1} = (dz W_layer) * silu'(z_{layer-1})
            uint16_t *dzn = t.dz[cur ^ 1];
#pragma unroll 1
            for (int n0 = 0; n0 < kH; n0 += 32) {
                f32x16 acc;
                zero(acc);
                tile_mma<true, false>(dzl, kLdH, 1, Wl[layer] + n0, ldw[layer], 1, kH, acc);
                const int n = n0 + acc_col();
#pragma unroll
                for (int i = 0; i < 16; ++i) {
                    const int r = acc_row(i);
                    dzn[r * kLdH + n] = to_bf16(acc[i] * dsilu(t.z[layer - 1][r * kH + n]));
                }
            }
            cur ^= 1;
        }
        __syncthreads();
    }
    for (int o = 32; o >= 1; o >>= 1) loss += __shfl_xor(loss, o, 64);
    if (lane == 0) loss_partial[blockIdx.x] = loss;
}

__device__ __forceinline__ bool mlp_pad(int p, int K)
{
    if (p < ob1) return (p - oW1) % kIn >= 5;
    if (p >= oW4 && p < ob4) return (p - oW4) / kH >= K;
    if (p >= ob4) return (p - ob4) >= K;
    return false;
}

// Sum of the per-block partial gradients of parameter p: a block of 256
// threads covers 64 parameters (lane) x 4 slices (wave); slice s adds the
// partials s, s + 4, ... in order, and the four slice sums are combined as
// (s0 + s1) + (s2 + s3) (a fixed order: results are deterministic).  Every
// thread of the block must call it (a barrier); p >= kParams contribute 0.
constexpr int kReduceParams = 64, kReduceSlices = 4;

__device__ __forceinline__ float reduce_partials(const float *__restrict__ partial, int blocks, int p)
{
    __shared__ float s_part[kReduceSlices][kReduceParams];
    const int lane = threadIdx.x % kReduceParams, slice = threadIdx.x / kReduceParams;
    float g = 0.0f;
    if (p < kParams)
        for (int b = slice; b < blocks; b += kReduceSlices) g += partial[(int64_t)b * kParams + p];
    s_part[slice][lane] = g;
    __syncthreads();
    return (s_part[0][lane] + s_part[1][lane]) + (s_part[2][lane] + s_part[3][lane]);
}

__device__ __forceinline__ void reduce_loss(const float *__restrict__ loss_partial, int blocks, int B,
                                            float *__restrict__ loss_out)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        float s = 0.0f;
        for (int b = 0; b < blocks; ++b) s += loss_partial[b];
        *loss_out = s / (float)B;
    }
}

// Gradient reduction and one Adam step (beta 0.9, 0.999, eps 1e-8) on the
// float master, then its bfloat16 copy; pad entries stay 0.
__global__ void __launch_bounds__(kReduceParams * kReduceSlices) k_mlp_adam(
    const float *__restrict__ partial, int blocks, int K, float *__restrict__ w, uint16_t *__restrict__ wb,
    float *__restrict__ m, float *__restrict__ v, int step, float lr, const float *__restrict__ loss_partial, int B,
    float *__restrict__ loss_out)
{
    reduce_loss(loss_partial, blocks, B, loss_out);
    const int p = blockIdx.x * kReduceParams + (int)(threadIdx.x % kReduceParams);
    const float g = reduce_partials(partial, blocks, p);
    if (threadIdx.x >= kReduceParams || p >= kParams) return; // slice 0 writes
    if (mlp_pad(p, K)) {
        w[p] = 0.0f;
        wb[p] = 0;
        m[p] = 0.0f;
        v[p] = 0.0f;
        return;
    }
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float mm = b1 * m[p] + (1.0f - b1) * g;
    const float vv = b2 * v[p] + (1.0f - b2) * g * g;
    m[p] = mm;
    v[p] = vv;
    const float mh = mm / (1.0f - powf(b1, (float)step));
    const float vh = vv / (1.0f - powf(b2, (float)step));
    const float nw = w[p] - lr * mh / (sqrtf(vh) + eps);
    w[p] = nw;
    wb[p] = to_bf16(nw);
}

// Gradient reduction only (the gradient entry point).
__global__ void __launch_bounds__(kReduceParams * kReduceSlices) k_mlp_sum(
    const float *__restrict__ partial, int blocks, const float *__restrict__ loss_partial, int B,
    float *__restrict__ grad, float *__restrict__ loss_out)
{
    reduce_loss(loss_partial, blocks, B, loss_out);
    const int p = blockIdx.x * kReduceParams + (int)(threadIdx.x % kReduceParams);
    const float g = reduce_partials(partial, blocks, p);
    if (threadIdx.x < kReduceParams && p < kParams) grad[p] = g;
}

// Zeroes the pad entries of the float master and writes the bf16 copy.
__global__ void __launch_bounds__(256) k_mlp_prepare(float *__restrict__ w, uint16_t *__restrict__ wb, int K)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= kParams) return;
    const float v = mlp_pad(p, K) ? 0.0f : w[p];
    w[p] = v;
    wb[p] = to_bf16(v);
}

// ---------------------------------------------------------------------------
// inference: kInferWaves waves per block share the staged weights (one
// block barrier after staging); wave w of block b then runs tiles
// (b * waves + w) + it * (grid * waves) in its own LDS tile, so the layers
// are ordered within the wave only.
// ---------------------------------------------------------------------------
// Orders a wave's LDS writes before its later LDS reads (all lanes of one
// wave): the writes complete (lgkmcnt 0) and the compiler moves no memory
// operation across.
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_s_waitcnt(0xC07F); // lgkmcnt(0), other counters unchanged
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

struct InferInput {
    const float *x;   // [B][5] features (src 0), or null
    glint_gbuffer g;  // G-buffer (src 1)
};

// Features of a surface pixel: reflection direction and scaled ln alphas.
// (float arithmetic: the inputs are rounded to bfloat16 before use).
__device__ __forceinline__ void pixel_features(const glint_gbuffer &g, int64_t i, float *f)
{
    const float nx = g.nx[i], ny = g.ny[i], nz = g.nz[i], vx = g.vx[i], vy = g.vy[i], vz = g.vz[i];
    const float mu = nx * vx + ny * vy + nz * vz;
    const float c = -2.3025850929940457f, h = 1.6094379124341003f; // centre, half width of [ln 0.02, ln 0.5]
    f[0] = 2.0f * mu * nx - vx;
    f[1] = 2.0f * mu * ny - vy;
    f[2] = 2.0f * mu * nz - vz;
    f[3] = (__logf(g.ax[i]) - c) / h;
    f[4] = (__logf(g.ay[i]) - c) / h;
}

template <int SRC>
__global__ void __launch_bounds__(64 * kInferWaves) k_mlp_infer(InferInput in, int64_t B, int K,
                                                                const float *__restrict__ w,
                                                                const uint16_t *__restrict__ wb,
                                                                float *__restrict__ out)
{
    __shared__ __attribute__((aligned(16))) uint16_t s_w[kWLds];
    __shared__ __attribute__((aligned(16))) float s_b[kBiasLds];
    __shared__ __attribute__((aligned(16))) InferTile s_t[kInferWaves];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    InferTile &t = s_t[wave];
    stage_weights(wb, s_w);
    // the biases too: read from global memory they are 28 16-byte loads per
    // lane and tile through the vector-memory path (the kernel's bound)
    for (int c = threadIdx.x; c < kBiasLds; c += blockDim.x) s_b[c] = w[ob1 + bias_src(c)];
    __syncthreads(); // the staged weights and biases are shared by the block's waves
    const uint16_t *W1 = s_w + sW1, *W2 = s_w + sW2, *W3 = s_w + sW3, *W4 = s_w + sW4;
    const int64_t tiles = (B + 31) / 32;
    const int64_t stride = (int64_t)gridDim.x * kInferWaves;
    const int64_t first = (int64_t)blockIdx.x * kInferWaves;
    const int64_t iters = first < tiles ? (tiles - first + stride - 1) / stride : 0;
    for (int64_t it = 0; it < iters; ++it) {
        const int64_t row0 = (first + wave + it * stride) * 32;
        wave_lds_sync(); // the previous tile's output layer has read the buffer
        bool needed = false; // this lane's row is a sample or a surface pixel
        if (lane < 32) {
            const int64_t i = row0 + lane;
            float f[5] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
            if (i < B) {
                if constexpr (SRC == 0) {
                    needed = true;
#pragma unroll
                    for (int c = 0; c < 5; ++c) f[c] = in.x[i * 5 + c];
                } else {
                    needed = in.g.surf_id[i] != GLINT_NO_SURFACE;
                    if (needed) pixel_features(in.g, i, f);
                }
            }
            uint4 *xr = reinterpret_cast<uint4 *>(t.h + lane * kLdH);
            const uint2 lo = pack_bf16x4(f[0], f[1], f[2], f[3]);
            xr[0] = make_uint4(lo.x, lo.y, (uint32_t)to_bf16(f[4]), 0u);
            xr[1] = make_uint4(0u, 0u, 0u, 0u);
        }
        // a tile with no sample and no surface pixel (background) skips the
        // network
        const bool active = __ballot(needed) != 0;
        wave_lds_sync();
        if (active) dense_silu_inplace(t.h, kIn, W1, kLdW1, s_b);
        wave_lds_sync();
        if (active) dense_silu_inplace(t.h, kH, W2, kLdH, s_b + kH);
        wave_lds_sync();
        if (active) dense_silu_inplace(t.h, kH, W3, kLdH, s_b + 2 * kH);
        wave_lds_sync();
        float logit[16], y[16];
#pragma unroll
        for (int j = 0; j < 16; ++j) y[j] = 0.0f;
        if (active) {
            dense_out(t.h, W4, s_b + 3 * kH, logit);
            softmax_pair(logit, K, y);
        }
        const int64_t i = row0 + (lane & 31);
        if (i < B) {
            bool keep = true;
            if constexpr (SRC == 1) keep = in.g.surf_id[i] != GLINT_NO_SURFACE;
#pragma unroll
            for (int j = 0; j < 16; ++j)
                if (out_unit(j) < K) out[i * K + out_unit(j)] = keep ? y[j] : 0.0f;
        }
    }
}

int mlp_params() { return kParams; }

static unsigned infer_blocks(int64_t B)
{
    const int64_t tiles = (B + 31) / 32;
    int64_t blocks = (tiles + kInferWaves - 1) / kInferWaves;
    if (blocks > kInferMaxBlocks) blocks = kInferMaxBlocks;
    return (unsigned)(blocks < 1 ? 1 : blocks);
}

hipError_t launch_mlp_prepare(float *w, uint16_t *wb, int K, hipStream_t stream)
{
    GLINT_LAUNCH("k_mlp_prepare", k_mlp_prepare, dim3((kParams + 255) / 256), dim3(256), 0, stream, w, wb, K);
    return hipGetLastError();
}

hipError_t launch_mlp_grad_step(const float *x, const float *target, const double *levels, float lam, int B, int K,
                                float *w, uint16_t *wb, float *m, float *v, int step, float lr, float *partial,
                                float *loss_partial, float *loss_out, hipStream_t stream)
{
    const int blocks = (B + 31) / 32;
    {
        GLINT_LAUNCH("k_mlp_grad", k_mlp_grad, dim3(blocks), dim3(64), 0, stream, x, target, levels, lam, B, K, w,
                     wb, partial, loss_partial);
    }
    GLINT_LAUNCH("k_mlp_adam", k_mlp_adam, dim3((kParams + kReduceParams - 1) / kReduceParams),
                 dim3(kReduceParams * kReduceSlices), 0, stream, partial, blocks, K, w, wb, m,
                       v, step, lr, loss_partial, B, loss_out);
    return hipGetLastError();
}

hipError_t launch_mlp_gradient(const float *x, const float *target, const double *levels, float lam, int B, int K,
                               const float *w, const uint16_t *wb, float *partial, float *loss_partial, float *grad,
                               float *loss_out, hipStream_t stream)
{
    const int blocks = (B + 31) / 32;
    {
        GLINT_LAUNCH("k_mlp_grad", k_mlp_grad, dim3(blocks), dim3(64), 0, stream, x, target, levels, lam, B, K, w,
                     wb, partial, loss_partial);
    }
    GLINT_LAUNCH("k_mlp_sum", k_mlp_sum, dim3((kParams + kReduceParams - 1) / kReduceParams),
                 dim3(kReduceParams * kReduceSlices), 0, stream, partial, blocks, loss_partial, B,
                       grad, loss_out);
    return hipGetLastError();
}

hipError_t launch_mlp_forward(const float *x, int64_t B, int K, const float *w, const uint16_t *wb, float *probs,
                              hipStream_t stream)
{
    InferInput in{};
    in.x = x;
    GLINT_LAUNCH("k_mlp_infer", k_mlp_infer<0>, dim3(infer_blocks(B)), dim3(64 * kInferWaves), 0, stream, in, B, K, w, wb,
                       probs);
    return hipGetLastError();
}

hipError_t launch_mlp_lookup(const glint_gbuffer &g, int64_t P, int K, const float *w, const uint16_t *wb, float *F,
                             hipStream_t stream)
{
    InferInput in{};
    in.g = g;
    GLINT_LAUNCH("k_mlp_lookup", k_mlp_infer<1>, dim3(infer_blocks(P)), dim3(64 * kInferWaves), 0, stream, in, P, K, w, wb,
                       F);
    return hipGetLastError();
}

} // namespace glint
