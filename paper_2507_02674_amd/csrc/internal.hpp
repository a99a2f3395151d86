// Internal launcher interface between the C ABI and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "glint.h"

namespace glint {

constexpr int kMaxPartitionBlocks = 1024;

int partition_blocks(int R);
hipError_t launch_partition(const float *env, int R, int K, double ell, int level_mode, int weight_space,
                            void *workspace, double *levels, uint8_t *ind_j, float *ind_t, hipStream_t stream);

size_t chain_bytes(int R, int K, int M);
hipError_t launch_prefilter(const float *env, const uint8_t *ind_j, const float *ind_t, int R, int K, int M, int T,
                            int dtype, void *workspace, void *ind_pyr, float *rgb_pyr, hipStream_t stream);

hipError_t launch_luts(float *lut_S, float *lut_E, hipStream_t stream);

hipError_t launch_shade(const glint_gbuffer &g, int64_t P, const glint_env &env, const glint_shade_params &sp,
                        float *radiance, const glint_shade_debug *dbg, hipStream_t stream);

// batched shading: per-view descriptors (device copies of make_shade_args
// output) and the first tile of each view
size_t shade_args_bytes();
void make_shade_args(void *out, const glint_gbuffer &g, int64_t P, const glint_env &env,
                     const glint_shade_params &sp, float *radiance);
hipError_t launch_shade_views(int K, int dtype, int V, const void *views, const int64_t *tile0, int n_views,
                              int64_t tiles, int tile_px, hipStream_t stream);

} // namespace glint
