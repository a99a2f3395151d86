// Internal launcher interface between the C ABI and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "glint.h"
#include "profile.hpp"

namespace glint {

constexpr int kMaxPartitionBlocks = 1024;

int partition_blocks(int R);
size_t partition_workspace_bytes(int R); // every level mode
size_t partition_workspace_bytes_mode(int R, int level_mode);
hipError_t launch_partition(const float *env, int R, int K, double ell, int level_mode, int weight_space,
                            void *workspace, double *levels, uint8_t *ind_j, float *ind_t, hipStream_t stream);

size_t chain_bytes(int R, int K, int M);
hipError_t launch_prefilter(const float *env, const uint8_t *ind_j, const float *ind_t, int R, int K, int M, int T,
                            int dtype, void *workspace, void *ind_pyr, float *rgb_pyr, hipStream_t stream);

// mode 0: filter at alpha = a0 -> out0 [n][K+3]; mode 1: training pairs at
// alpha = sqrt(a0 a1) -> out0 features [n][5], out1 targets [n][K]; mode 2:
// the lookups of the G-buffer g's pixels -> out0 [n][K].
hipError_t launch_sample_filter(const float *env, const uint8_t *ind_j, const float *ind_t, const void *workspace,
                                int R, int K, int M, int T, int mode, const float *dirs, const float *a0,
                                const float *a1, const glint_gbuffer *g, int64_t n, float *out0, float *out1,
                                hipStream_t stream);

hipError_t launch_luts(float *lut_S, float *lut_E, hipStream_t stream);
hipError_t launch_quantile_table(double *table, hipStream_t stream);

// learned surrogate
int mlp_params();
hipError_t launch_mlp_prepare(float *w, uint16_t *wb, int K, hipStream_t stream);
// levels: null (soft-label cross-entropy only) or the K radiance levels of
// the radiance-weighted term, with weight lam
hipError_t launch_mlp_grad_step(const float *x, const float *target, const double *levels, float lam, int B, int K,
                                float *w, uint16_t *wb, float *m, float *v, int step, float lr, float *partial,
                                float *loss_partial, float *loss_out, hipStream_t stream);
hipError_t launch_mlp_gradient(const float *x, const float *target, const double *levels, float lam, int B, int K,
                               const float *w, const uint16_t *wb, float *partial, float *loss_partial, float *grad,
                               float *loss_out, hipStream_t stream);
hipError_t launch_mlp_forward(const float *x, int64_t B, int K, const float *w, const uint16_t *wb, float *probs,
                              hipStream_t stream);
hipError_t launch_mlp_lookup(const glint_gbuffer &g, int64_t P, int K, const float *w, const uint16_t *wb, float *F,
                             hipStream_t stream);

// F: null for the plain form; else the surrogate's filtered indicator values [P][K].
hipError_t launch_shade(const glint_gbuffer &g, int64_t P, const glint_env &env, const glint_shade_params &sp,
                        const float *F, float *radiance, const glint_shade_debug *dbg, hipStream_t stream);

hipError_t launch_sample_binomial(int sampler, int exact_gating, const double *N, const double *p, const uint32_t *h1,
                                  const uint32_t *h2, int64_t count, const double *qtail, double *n, double *nb,
                                  uint8_t *code, hipStream_t stream);

// batched shading: per-view descriptors (device copies of make_shade_args
// output) and the first tile of each view
size_t shade_args_bytes();
void make_shade_args(void *out, const glint_gbuffer &g, int64_t P, const glint_env &env,
                     const glint_shade_params &sp, float *radiance, const float *F);
hipError_t launch_shade_views(int K, int dtype, int V, bool surrogate, const void *views, const int64_t *tile0,
                              int n_views, int64_t tiles, int tile_px, hipStream_t stream);

} // namespace glint
