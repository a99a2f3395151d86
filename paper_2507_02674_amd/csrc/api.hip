// C ABI of the glint library: argument validation, context, error reporting.
// Every entry point validates on the host before launching anything.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <new>

#include "batched.hpp"
#include "device.hpp"
#include "internal.hpp"

struct glint_ctx_s {
    int device;
    int num_cu;
    glint::BatchedCache batched;
};

namespace {

thread_local char g_err[512] = "";

int fail(int code, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

int ok()
{
    g_err[0] = '\0';
    return GLINT_OK;
}

int device_status(hipError_t e, const char *what)
{
    if (e != hipSuccess) return fail(GLINT_EDEVICE, "%s: %s", what, hipGetErrorString(e));
    return ok();
}

bool pow2(int x) { return x > 0 && (x & (x - 1)) == 0; }

int log2i(int x)
{
    int l = 0;
    while ((1 << (l + 1)) <= x) ++l;
    return l;
}

int check_ctx(glint_ctx ctx)
{
    if (!ctx) return fail(GLINT_EINVAL, "null context");
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) return fail(GLINT_EDEVICE, "hipGetDevice failed");
    if (cur != ctx->device && hipSetDevice(ctx->device) != hipSuccess)
        return fail(GLINT_EDEVICE, "hipSetDevice(%d) failed", ctx->device);
    return GLINT_OK;
}

int check_R(int R)
{
    if (!pow2(R) || R > 4096) return fail(GLINT_EINVAL, "face size R=%d must be a power of two in [1, 4096]", R);
    return GLINT_OK;
}

int check_mips(int R, int M)
{
    if (M < 1 || M > log2i(R) + 1) return fail(GLINT_EINVAL, "num_mips=%d must be in [1, log2(R)+1=%d]", M, log2i(R) + 1);
    return GLINT_OK;
}

int check_tree_K(int K)
{
    if (K < 2 || K > 16) return fail(GLINT_EINVAL, "K=%d must be in [2, 16]", K);
    if (!pow2(K)) return fail(GLINT_EUNSUPPORTED, "K=%d: filtering and shading support K in {2,4,8,16}", K);
    return GLINT_OK;
}

int check_dtype(int dt)
{
    if (dt < GLINT_F32 || dt > GLINT_UNORM16) return fail(GLINT_EINVAL, "unknown pyramid dtype %d", dt);
    return GLINT_OK;
}

int check_partition(const float *env, int R, const glint_partition_params *pp, const void *workspace,
                    const double *levels, const uint8_t *ind_j, const float *ind_t)
{
    if (!pp || !env || !workspace || !levels || !ind_j || !ind_t) return fail(GLINT_EINVAL, "null pointer argument");
    if (int rc = check_R(R)) return rc;
    if (pp->K < 2 || pp->K > 16) return fail(GLINT_EINVAL, "K=%d must be in [2, 16]", pp->K);
    if (!(pp->ell > 0.0)) return fail(GLINT_EINVAL, "ell must be > 0");
    if (pp->level_mode != 0 && pp->level_mode != 2)
        return fail(pp->level_mode == 1 ? GLINT_EUNSUPPORTED : GLINT_EINVAL, "level_mode %d not available",
                    pp->level_mode);
    if (pp->level_mode == 2 && pp->K < 3) return fail(GLINT_EINVAL, "level_mode 2 needs K >= 3");
    if (pp->weight_space != 0 && pp->weight_space != 1) return fail(GLINT_EINVAL, "weight_space must be 0 or 1");
    if (reinterpret_cast<uintptr_t>(workspace) % 8) return fail(GLINT_EINVAL, "workspace must be 8-byte aligned");
    return GLINT_OK;
}

int check_prefilter(const float *env, const uint8_t *ind_j, const float *ind_t, int R, int K,
                    const glint_prefilter_params *fp, const void *workspace, const void *ind_pyr,
                    const float *rgb_pyr)
{
    if (!fp || !env || !ind_j || !ind_t || !workspace || !ind_pyr || !rgb_pyr)
        return fail(GLINT_EINVAL, "null pointer argument");
    if (int rc = check_R(R)) return rc;
    if (int rc = check_tree_K(K)) return rc;
    if (int rc = check_mips(R, fp->num_mips)) return rc;
    if (int rc = check_dtype(fp->dtype)) return rc;
    if (fp->taps < 1 || fp->taps > 1024) return fail(GLINT_EINVAL, "taps=%d must be in [1, 1024]", fp->taps);
    if (reinterpret_cast<uintptr_t>(workspace) % 16 || reinterpret_cast<uintptr_t>(rgb_pyr) % 16)
        return fail(GLINT_EINVAL, "workspace and rgb_pyr must be 16-byte aligned");
    return GLINT_OK;
}

int check_gbuffer(const glint_gbuffer *g)
{
    if (!g) return fail(GLINT_EINVAL, "null G-buffer");
    const void *fields[] = {g->nx, g->ny, g->nz, g->vx, g->vy, g->vz, g->u, g->v, g->area, g->ax, g->ay,
                            g->density, g->f0r, g->f0g, g->f0b, g->surf_id};
    for (const void *f : fields)
        if (!f) return fail(GLINT_EINVAL, "null G-buffer field");
    return GLINT_OK;
}

} // namespace

extern "C" {

int glint_version(void) { return GLINT_VERSION; }

const char *glint_last_error(void) { return g_err; }

int glint_create(int device, glint_ctx *out)
{
    if (!out) return fail(GLINT_EINVAL, "null output pointer");
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess) return fail(GLINT_EDEVICE, "hipGetDeviceCount failed");
    if (device < 0 || device >= count) return fail(GLINT_EINVAL, "device %d out of range (count %d)", device, count);
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess)
        return fail(GLINT_EDEVICE, "hipGetDeviceProperties(%d) failed", device);
    glint_ctx c = new (std::nothrow) glint_ctx_s;
    if (!c) return fail(GLINT_ENOMEM, "context allocation failed");
    c->device = device;
    c->num_cu = prop.multiProcessorCount;
    *out = c;
    return ok();
}

void glint_destroy(glint_ctx ctx) { delete ctx; }

int glint_sync(glint_ctx ctx)
{
    if (int rc = check_ctx(ctx)) return rc;
    return device_status(hipDeviceSynchronize(), "hipDeviceSynchronize");
}

size_t glint_partition_workspace_bytes(int R)
{
    if (!pow2(R) || R > 4096) return 0;
    return sizeof(double) * 2 * (size_t)glint::partition_blocks(R);
}

int glint_partition_env(glint_ctx ctx, const float *env, int R, const glint_partition_params *pp, void *workspace,
                        double *levels, uint8_t *ind_j, float *ind_t, void *stream)
{
    if (int rc = check_ctx(ctx)) return rc;
    if (int rc = check_partition(env, R, pp, workspace, levels, ind_j, ind_t)) return rc;
    return device_status(glint::launch_partition(env, R, pp->K, pp->ell, pp->level_mode, pp->weight_space,
                                                 workspace, levels, ind_j, ind_t, (hipStream_t)stream),
                         "glint_partition_env launch");
}

int64_t glint_pyramid_texels(int R, int num_mips)
{
    if (!pow2(R) || R > 4096 || num_mips < 1 || num_mips > log2i(R) + 1) return 0;
    return glint::level_offset(R, num_mips);
}

size_t glint_prefilter_workspace_bytes(int R, int K, const glint_prefilter_params *fp)
{
    if (!fp || !pow2(R) || R > 4096 || K < 2 || K > 16 || fp->num_mips < 1 || fp->num_mips > log2i(R) + 1)
        return 0;
    size_t b = glint::chain_bytes(R, K, fp->num_mips);
    return b < 16 ? 16 : b;
}

int glint_prefilter(glint_ctx ctx, const float *env, const uint8_t *ind_j, const float *ind_t, int R, int K,
                    const glint_prefilter_params *fp, void *workspace, void *ind_pyr, float *rgb_pyr, void *stream)
{
    if (int rc = check_ctx(ctx)) return rc;
    if (int rc = check_prefilter(env, ind_j, ind_t, R, K, fp, workspace, ind_pyr, rgb_pyr)) return rc;
    return device_status(glint::launch_prefilter(env, ind_j, ind_t, R, K, fp->num_mips, fp->taps, (int)fp->dtype,
                                                 workspace, ind_pyr, rgb_pyr, (hipStream_t)stream),
                         "glint_prefilter launch");
}

int glint_build_luts(glint_ctx ctx, float *lut_S, float *lut_E, void *stream)
{
    if (int rc = check_ctx(ctx)) return rc;
    if (!lut_S || !lut_E) return fail(GLINT_EINVAL, "null pointer argument");
    return device_status(glint::launch_luts(lut_S, lut_E, (hipStream_t)stream), "glint_build_luts launch");
}

int glint_shade(glint_ctx ctx, const glint_gbuffer *g, int64_t P, const glint_env *env,
                const glint_shade_params *sp, float *radiance, const glint_shade_debug *dbg, void *stream)
{
    if (int rc = check_ctx(ctx)) return rc;
    if (!g || !env || !sp) return fail(GLINT_EINVAL, "null pointer argument");
    if (P < 0) return fail(GLINT_EINVAL, "num_pixels must be >= 0");
    if (int rc = check_R(env->R)) return rc;
    if (int rc = check_tree_K(env->K)) return rc;
    if (int rc = check_mips(env->R, env->num_mips)) return rc;
    if (int rc = check_dtype(env->dtype)) return rc;
    if (sp->vertices != 1 && sp->vertices != 6) return fail(GLINT_EINVAL, "vertices must be 1 or 6");
    if (P == 0) return ok();
    if (!radiance || !env->ind_pyr || !env->rgb_pyr || !env->levels || !env->lut_S || !env->lut_E)
        return fail(GLINT_EINVAL, "null pointer argument");
    if (int rc = check_gbuffer(g)) return rc;
    if (reinterpret_cast<uintptr_t>(env->rgb_pyr) % 16) return fail(GLINT_EINVAL, "rgb_pyr must be 16-byte aligned");
    if (P > ((int64_t)1 << 40)) return fail(GLINT_EINVAL, "num_pixels too large");
    return device_status(glint::launch_shade(*g, P, *env, *sp, radiance, dbg, (hipStream_t)stream),
                         "glint_shade launch");
}

size_t glint_batched_workspace_bytes(int n_views)
{
    if (n_views < 1 || n_views > 4096) return 0;
    return glint::batched_workspace_bytes(n_views);
}

int glint_frame_batched(glint_ctx ctx, const glint_env_task *envs, int n_env, const glint_view *views, int n_views,
                        void *workspace, void *stream)
{
    if (int rc = check_ctx(ctx)) return rc;
    if (!envs || !views || !workspace) return fail(GLINT_EINVAL, "null pointer argument");
    if (n_env < 1 || n_env > 64) return fail(GLINT_EINVAL, "n_env=%d must be in [1, 64]", n_env);
    if (n_views < 1 || n_views > 4096) return fail(GLINT_EINVAL, "n_views=%d must be in [1, 4096]", n_views);
    if (reinterpret_cast<uintptr_t>(workspace) % 256) return fail(GLINT_EINVAL, "workspace must be 256-byte aligned");
    for (int e = 0; e < n_env; ++e) {
        const glint_env_task &t = envs[e];
        if (int rc = check_partition(t.env, t.R, &t.partition, t.partition_workspace, t.levels, t.ind_j, t.ind_t))
            return rc;
        if (int rc = check_prefilter(t.env, t.ind_j, t.ind_t, t.R, t.partition.K, &t.prefilter,
                                     t.prefilter_workspace, t.ind_pyr, t.rgb_pyr))
            return rc;
        if (!t.lut_S || !t.lut_E) return fail(GLINT_EINVAL, "environment %d: null LUT", e);
        if (t.prefilter.dtype != envs[0].prefilter.dtype)
            return fail(GLINT_EINVAL, "all environments of one call must share the pyramid dtype");
    }
    for (int v = 0; v < n_views; ++v) {
        const glint_view &w = views[v];
        if (w.env_index < 0 || w.env_index >= n_env) return fail(GLINT_EINVAL, "view %d: env_index out of range", v);
        if (w.num_pixels < 0 || w.num_pixels > ((int64_t)1 << 40))
            return fail(GLINT_EINVAL, "view %d: bad num_pixels", v);
        if (w.shade.vertices != 1 && w.shade.vertices != 6) return fail(GLINT_EINVAL, "view %d: vertices", v);
        if (!w.radiance) return fail(GLINT_EINVAL, "view %d: null radiance", v);
        if (int rc = check_gbuffer(&w.gbuf)) return rc;
    }
    return device_status(glint::frame_batched(ctx->batched, envs, n_env, views, n_views, workspace,
                                              (hipStream_t)stream),
                         "glint_frame_batched");
}

int glint_batched_tile_px(glint_ctx ctx) { return ctx ? ctx->batched.last_tile_px : 0; }

} // extern "C"
