// C ABI of the glint library: argument validation, context, error reporting.
// Every entry point validates on the host before launching anything.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <map>
#include <mutex>
#include <new>
#include <string>

#include "batched.hpp"
#include "device.hpp"
#include "internal.hpp"

struct glint_ctx_s {
    int device;
    int num_cu;
    void *scratch; // device address of this GPU's copy of `scratch` below
    glint::BatchedCache batched;
    glint::Profiler prof;
    // bf16 parameter copies written in this context (glint_surrogate_prepare
    // or glint_surrogate_train_step), with their K
    std::mutex sur_mu;
    std::map<const void *, int> prepared;
};

// Workspace of glint_partition_env_noalloc: a file-scope device array, one
// copy per GPU, held until the process ends.  Host code uses the device
// address that hipGetSymbolAddress returns for the current GPU (kept per
// device below), never the array's name.  Every call on one GPU shares it.
constexpr size_t kNoallocScratchBytes = 2304 * 1024;
static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on `device` (looked up once per device, with
// that device current).
hipError_t scratch_address(int device, void **out)
{
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        int prev = -1;
        hipError_t e = hipGetDevice(&prev);
        if (e != hipSuccess) return e;
        if (prev != device && (e = hipSetDevice(device)) != hipSuccess) return e;
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (prev != device) {
            const hipError_t e2 = hipSetDevice(prev);
            if (e == hipSuccess) e = e2;
        }
        if (e != hipSuccess) return e;
        g_scratch_ptr[device] = p;
    }
    *out = g_scratch_ptr[device];
    return hipSuccess;
}

// Error messages: per thread the last one of any call, and per (thread,
// context) the last one of a call on that context.  Every entry point that
// takes a context names it first (check_ctx or enter), so fail() and ok()
// know where to record.
thread_local char g_err[512] = "";
thread_local glint_ctx g_cur = nullptr;
thread_local std::map<glint_ctx, std::string> *g_ctx_err = nullptr;

void enter(glint_ctx ctx) { g_cur = ctx; }

std::map<glint_ctx, std::string> &ctx_errors()
{
    if (!g_ctx_err) g_ctx_err = new std::map<glint_ctx, std::string>(); // lives as long as the thread
    return *g_ctx_err;
}

int fail(int code, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    if (g_cur) ctx_errors()[g_cur] = g_err;
    return code;
}

int ok()
{
    g_err[0] = '\0';
    if (g_cur && g_ctx_err) {
        auto it = g_ctx_err->find(g_cur);
        if (it != g_ctx_err->end()) it->second.clear();
    }
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
    enter(ctx);
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
    if (pp->level_mode < 0 || pp->level_mode > 2) return fail(GLINT_EINVAL, "level_mode %d not available", pp->level_mode);
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

int check_surrogate(int K, const void *w, const void *w_bf16)
{
    if (K < 2 || K > 32) return fail(GLINT_EINVAL, "surrogate K=%d must be in [2, 32]", K);
    if (!w || !w_bf16) return fail(GLINT_EINVAL, "null surrogate parameters");
    if (reinterpret_cast<uintptr_t>(w_bf16) % 16 || reinterpret_cast<uintptr_t>(w) % 4)
        return fail(GLINT_EINVAL, "w_bf16 must be 16-byte aligned");
    return GLINT_OK;
}

void mark_prepared(glint_ctx ctx, const void *w_bf16, int K)
{
    std::lock_guard<std::mutex> lock(ctx->sur_mu);
    ctx->prepared[w_bf16] = K;
}

// GLINT_ENOTTRAINED unless w_bf16 was written for K in this context.
int check_prepared(glint_ctx ctx, const void *w_bf16, int K)
{
    std::lock_guard<std::mutex> lock(ctx->sur_mu);
    auto it = ctx->prepared.find(w_bf16);
    if (it == ctx->prepared.end())
        return fail(GLINT_ENOTTRAINED, "surrogate parameters at %p were never prepared (glint_surrogate_prepare) "
                    "or trained (glint_surrogate_train_step) in this context", w_bf16);
    if (it->second != K)
        return fail(GLINT_ENOTTRAINED, "surrogate parameters at %p were prepared for K=%d, not K=%d", w_bf16,
                    it->second, K);
    return GLINT_OK;
}

int check_batch(int B, const float *x, const float *target, const void *workspace)
{
    if (B < 1 || B > (1 << 20)) return fail(GLINT_EINVAL, "batch size %d must be in [1, 2^20]", B);
    if (!x || !target || !workspace) return fail(GLINT_EINVAL, "null pointer argument");
    if (reinterpret_cast<uintptr_t>(workspace) % 16) return fail(GLINT_EINVAL, "workspace must be 16-byte aligned");
    return GLINT_OK;
}

// Bytes of the per-block partial gradients (a multiple of 256).
size_t surrogate_partial_bytes(size_t blocks)
{
    return (blocks * (size_t)glint::mlp_params() * sizeof(float) + 255) & ~(size_t)255;
}

} // namespace

extern "C" {

int glint_version(void) { return GLINT_VERSION; }

const char *glint_last_error(glint_ctx ctx)
{
    if (!ctx) return g_err;
    if (!g_ctx_err) return "";
    auto it = g_ctx_err->find(ctx);
    return it == g_ctx_err->end() ? "" : it->second.c_str();
}

int glint_create(int device, glint_ctx *out)
{
    enter(nullptr);
    if (!out) return fail(GLINT_EINVAL, "null output pointer");
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess) return fail(GLINT_EDEVICE, "hipGetDeviceCount failed");
    if (device < 0 || device >= count) return fail(GLINT_EINVAL, "device %d out of range (count %d)", device, count);
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess)
        return fail(GLINT_EDEVICE, "hipGetDeviceProperties(%d) failed", device);
    if (device >= kMaxDevices) return fail(GLINT_EINVAL, "device %d beyond the library's %d", device, kMaxDevices);
    void *scr = nullptr;
    if (hipError_t e = scratch_address(device, &scr); e != hipSuccess)
        return fail(GLINT_EDEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", device, hipGetErrorString(e));
    glint_ctx c = new (std::nothrow) glint_ctx_s;
    if (!c) return fail(GLINT_ENOMEM, "context allocation failed");
    c->device = device;
    c->num_cu = prop.multiProcessorCount;
    c->scratch = scr;
    *out = c;
    return ok();
}

void glint_destroy(glint_ctx ctx)
{
    if (g_ctx_err) g_ctx_err->erase(ctx); // this thread's record (others keep a stale entry, never read)
    if (g_cur == ctx) g_cur = nullptr;
    delete ctx;
}

int glint_sync(glint_ctx ctx)
{
    if (int rc = check_ctx(ctx)) return rc;
    glint::ProfScope prof_scope(&ctx->prof);
    return device_status(hipDeviceSynchronize(), "hipDeviceSynchronize");
}

size_t glint_partition_workspace_bytes(int R)
{
    if (!pow2(R) || R > 4096) return 0;
    return glint::partition_workspace_bytes(R);
}

int glint_partition_env(glint_ctx ctx, const float *env, int R, const glint_partition_params *pp, void *workspace,
                        double *levels, uint8_t *ind_j, float *ind_t, void *stream)
{
    if (int rc = check_ctx(ctx)) return rc;
    glint::ProfScope prof_scope(&ctx->prof);
    if (int rc = check_partition(env, R, pp, workspace, levels, ind_j, ind_t)) return rc;
    return device_status(glint::launch_partition(env, R, pp->K, pp->ell, pp->level_mode, pp->weight_space,
                                                 workspace, levels, ind_j, ind_t, (hipStream_t)stream),
                         "glint_partition_env launch");
}

int glint_partition_env_noalloc(glint_ctx ctx, const float *env, int R, const glint_partition_params *pp,
                                double *levels, uint8_t *ind_j, float *ind_t, void *stream)
{
    if (int rc = check_ctx(ctx)) return rc;
    glint::ProfScope prof_scope(&ctx->prof);
    if (int rc = check_partition(env, R, pp, ctx->scratch, levels, ind_j, ind_t)) return rc;
    const size_t need = glint::partition_workspace_bytes_mode(R, pp->level_mode);
    if (need > kNoallocScratchBytes)
        return fail(GLINT_EINVAL, "R=%d with level_mode %d needs %zu bytes of scratch; the allocation-free call "
                    "holds %zu (level_mode 1 up to R = 1024)", R, pp->level_mode, need, kNoallocScratchBytes);
    return device_status(glint::launch_partition(env, R, pp->K, pp->ell, pp->level_mode, pp->weight_space,
                                                 ctx->scratch, levels, ind_j, ind_t, (hipStream_t)stream),
                         "glint_partition_env_noalloc launch");
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
    glint::ProfScope prof_scope(&ctx->prof);
    if (int rc = check_prefilter(env, ind_j, ind_t, R, K, fp, workspace, ind_pyr, rgb_pyr)) return rc;
    return device_status(glint::launch_prefilter(env, ind_j, ind_t, R, K, fp->num_mips, fp->taps, (int)fp->dtype,
                                                 workspace, ind_pyr, rgb_pyr, (hipStream_t)stream),
                         "glint_prefilter launch");
}

static bool dual_sampler(int s) { return s == GLINT_SAMPLER_DUAL || s == GLINT_SAMPLER_DUAL_SYMMETRIC; }

// view >= 0 names the batched view in the message
static int check_shade_params(const glint_shade_params &sp, int view)
{
    const char *what = nullptr;
    if (sp.vertices != 1 && sp.vertices != 6 && sp.vertices != 12) what = "vertices must be 1, 6 or 12";
    else if (sp.exact_gating != 0 && sp.exact_gating != 1) what = "exact_gating must be 0 or 1";
    else if (sp.sampler < GLINT_SAMPLER_DUAL || sp.sampler > GLINT_SAMPLER_DUAL_SYMMETRIC) what = "unknown sampler";
    else if (sp.prob_mode != GLINT_PROBS_ENV && sp.prob_mode != GLINT_PROBS_CONSTANT) what = "unknown prob_mode";
    else if (sp.prob_mode == GLINT_PROBS_CONSTANT && !(sp.gamma > 0.0f && sp.gamma <= 1.0f))
        what = "gamma must be in (0, 1]";
    else if (sp.lobe_taps != 0 && sp.lobe_taps != 2 && sp.lobe_taps != 4 && sp.lobe_taps != 8)
        what = "lobe_taps must be 0, 2, 4 or 8";
    else if (sp.tree != GLINT_TREE_BALANCED && sp.tree != GLINT_TREE_CHAIN)
        what = "tree must be GLINT_TREE_BALANCED or GLINT_TREE_CHAIN";
    if (!what) return GLINT_OK;
    if (view >= 0) return fail(GLINT_EINVAL, "view %d: %s", view, what);
    return fail(GLINT_EINVAL, "%s", what);
}

int glint_build_luts(glint_ctx ctx, float *lut_S, float *lut_E, void *stream)
{
    if (int rc = check_ctx(ctx)) return rc;
    glint::ProfScope prof_scope(&ctx->prof);
    if (!lut_S || !lut_E) return fail(GLINT_EINVAL, "null pointer argument");
    return device_status(glint::launch_luts(lut_S, lut_E, (hipStream_t)stream), "glint_build_luts launch");
}

size_t glint_quantile_table_bytes(void) { return (size_t)glint::kTailEntries * sizeof(double); }

int glint_build_quantile_table(glint_ctx ctx, double *table, void *stream)
{
    if (int rc = check_ctx(ctx)) return rc;
    glint::ProfScope prof_scope(&ctx->prof);
    if (!table) return fail(GLINT_EINVAL, "null pointer argument");
    if (reinterpret_cast<uintptr_t>(table) % 8) return fail(GLINT_EINVAL, "table must be 8-byte aligned");
    return device_status(glint::launch_quantile_table(table, (hipStream_t)stream), "glint_build_quantile_table");
}

int glint_sample_binomial(glint_ctx ctx, int sampler, int exact_gating, const double *N, const double *p,
                          const uint32_t *h1, const uint32_t *h2, int64_t count, const double *quantile_tail,
                          double *n, double *nbar, uint8_t *code, void *stream)
{
    if (int rc = check_ctx(ctx)) return rc;
    glint::ProfScope prof_scope(&ctx->prof);
    if (sampler < GLINT_SAMPLER_DUAL || sampler > GLINT_SAMPLER_DUAL_SYMMETRIC)
        return fail(GLINT_EINVAL, "unknown sampler %d", sampler);
    if (exact_gating != 0 && exact_gating != 1) return fail(GLINT_EINVAL, "exact_gating must be 0 or 1");
    if (count < 0 || count > ((int64_t)1 << 40)) return fail(GLINT_EINVAL, "bad count %lld", (long long)count);
    if (count == 0) return ok();
    if (!N || !p || !h1 || !h2 || !n || !nbar || !code) return fail(GLINT_EINVAL, "null pointer argument");
    return device_status(glint::launch_sample_binomial(sampler, exact_gating, N, p, h1, h2, count, quantile_tail, n,
                                                       nbar, code, (hipStream_t)stream),
                         "glint_sample_binomial launch");
}

int glint_shade(glint_ctx ctx, const glint_gbuffer *g, int64_t P, const glint_env *env,
                const glint_shade_params *sp, float *radiance, const glint_shade_debug *dbg, void *stream)
{
    if (int rc = check_ctx(ctx)) return rc;
    glint::ProfScope prof_scope(&ctx->prof);
    if (!g || !env || !sp) return fail(GLINT_EINVAL, "null pointer argument");
    if (P < 0) return fail(GLINT_EINVAL, "num_pixels must be >= 0");
    if (int rc = check_R(env->R)) return rc;
    if (int rc = check_tree_K(env->K)) return rc;
    if (int rc = check_mips(env->R, env->num_mips)) return rc;
    if (int rc = check_dtype(env->dtype)) return rc;
    if (int rc = check_shade_params(*sp, -1)) return rc;
    const bool constant = sp->prob_mode == GLINT_PROBS_CONSTANT;
    if (!dual_sampler(sp->sampler) && env->dtype != GLINT_F32 && !constant)
        return fail(GLINT_EUNSUPPORTED, "single-gated samplers need a float32 pyramid");
    if (sp->lobe_taps > 0 && (env->dtype != GLINT_F32 || !dual_sampler(sp->sampler) || constant))
        return fail(GLINT_EUNSUPPORTED, "anisotropic lookups need a float32 pyramid, the dual gate and the map's "
                    "probabilities");
    if (sp->vertices == 12 &&
        (env->dtype != GLINT_F32 || !dual_sampler(sp->sampler) || constant || sp->lobe_taps != 0))
        return fail(GLINT_EUNSUPPORTED, "the footprint grid needs a float32 pyramid, the dual gate, the map's "
                    "probabilities and one lookup");
    if (sp->tree == GLINT_TREE_CHAIN &&
        (env->dtype != GLINT_F32 || !dual_sampler(sp->sampler) || constant || sp->lobe_taps != 0 ||
         sp->vertices == 12))
        return fail(GLINT_EUNSUPPORTED, "the sequential chain needs a float32 pyramid, the dual gate, the map's "
                    "probabilities, one lookup and 1 or 6 vertices");
    if (P == 0) return ok();
    if (!radiance || !env->rgb_pyr || !env->lut_E ||
        (!constant && (!env->ind_pyr || !env->levels || !env->lut_S)))
        return fail(GLINT_EINVAL, "null pointer argument");
    if (int rc = check_gbuffer(g)) return rc;
    if (sp->lobe_taps > 0 && (!g->tx || !g->ty || !g->tz))
        return fail(GLINT_EINVAL, "anisotropic lookups need the G-buffer tangent");
    if (sp->vertices == 12 && (!g->dudx || !g->dudy || !g->dvdx || !g->dvdy))
        return fail(GLINT_EINVAL, "the footprint grid needs the G-buffer uv Jacobian");
    if (reinterpret_cast<uintptr_t>(env->rgb_pyr) % 16) return fail(GLINT_EINVAL, "rgb_pyr must be 16-byte aligned");
    if (P > ((int64_t)1 << 40)) return fail(GLINT_EINVAL, "num_pixels too large");
    return device_status(glint::launch_shade(*g, P, *env, *sp, nullptr, radiance, dbg, (hipStream_t)stream),
                         "glint_shade launch");
}

int glint_sample_filter(glint_ctx ctx, const float *env, const uint8_t *ind_j, const float *ind_t, int R, int K,
                        const glint_prefilter_params *fp, const void *workspace, const float *dirs,
                        const float *alphas, int64_t n, float *out, void *stream)
{
    if (int rc = check_ctx(ctx)) return rc;
    glint::ProfScope prof_scope(&ctx->prof);
    if (!fp || !env || !ind_j || !ind_t || !workspace) return fail(GLINT_EINVAL, "null pointer argument");
    if (int rc = check_R(R)) return rc;
    if (int rc = check_tree_K(K)) return rc;
    if (int rc = check_mips(R, fp->num_mips)) return rc;
    if (fp->taps < 1 || fp->taps > 1024) return fail(GLINT_EINVAL, "taps=%d must be in [1, 1024]", fp->taps);
    if (n < 0 || n > ((int64_t)1 << 36)) return fail(GLINT_EINVAL, "bad sample count %lld", (long long)n);
    if (reinterpret_cast<uintptr_t>(workspace) % 16) return fail(GLINT_EINVAL, "workspace must be 16-byte aligned");
    if (n == 0) return ok();
    if (!dirs || !alphas || !out) return fail(GLINT_EINVAL, "null pointer argument");
    return device_status(glint::launch_sample_filter(env, ind_j, ind_t, workspace, R, K, fp->num_mips, fp->taps, 0,
                                                     dirs, alphas, nullptr, nullptr, n, out, nullptr,
                                                     (hipStream_t)stream),
                         "glint_sample_filter launch");
}

int glint_surrogate_samples(glint_ctx ctx, const float *env, const uint8_t *ind_j, const float *ind_t, int R,
                            int K, const glint_prefilter_params *fp, const void *workspace, const float *dirs,
                            const float *ax, const float *ay, int64_t n, float *x, float *target, void *stream)
{
    if (int rc = check_ctx(ctx)) return rc;
    glint::ProfScope prof_scope(&ctx->prof);
    if (!fp || !env || !ind_j || !ind_t || !workspace) return fail(GLINT_EINVAL, "null pointer argument");
    if (int rc = check_R(R)) return rc;
    if (int rc = check_tree_K(K)) return rc;
    if (int rc = check_mips(R, fp->num_mips)) return rc;
    if (fp->taps < 1 || fp->taps > 1024) return fail(GLINT_EINVAL, "taps=%d must be in [1, 1024]", fp->taps);
    if (n < 0 || n > ((int64_t)1 << 36)) return fail(GLINT_EINVAL, "bad sample count %lld", (long long)n);
    if (reinterpret_cast<uintptr_t>(workspace) % 16) return fail(GLINT_EINVAL, "workspace must be 16-byte aligned");
    if (n == 0) return ok();
    if (!dirs || !ax || !ay || !x || !target) return fail(GLINT_EINVAL, "null pointer argument");
    return device_status(glint::launch_sample_filter(env, ind_j, ind_t, workspace, R, K, fp->num_mips, fp->taps, 1,
                                                     dirs, ax, ay, nullptr, n, x, target, (hipStream_t)stream),
                         "glint_surrogate_samples launch");
}

int glint_filter_pixels(glint_ctx ctx, const float *env, const uint8_t *ind_j, const float *ind_t, int R, int K,
                        const glint_prefilter_params *fp, const void *workspace, const glint_gbuffer *g, int64_t P,
                        float *F, void *stream)
{
    if (int rc = check_ctx(ctx)) return rc;
    glint::ProfScope prof_scope(&ctx->prof);
    if (!fp || !env || !ind_j || !ind_t || !workspace) return fail(GLINT_EINVAL, "null pointer argument");
    if (int rc = check_R(R)) return rc;
    if (int rc = check_tree_K(K)) return rc;
    if (int rc = check_mips(R, fp->num_mips)) return rc;
    if (fp->taps < 1 || fp->taps > 1024) return fail(GLINT_EINVAL, "taps=%d must be in [1, 1024]", fp->taps);
    if (P < 0 || P > ((int64_t)1 << 36)) return fail(GLINT_EINVAL, "bad pixel count %lld", (long long)P);
    if (reinterpret_cast<uintptr_t>(workspace) % 16) return fail(GLINT_EINVAL, "workspace must be 16-byte aligned");
    if (P == 0) return ok();
    if (!F) return fail(GLINT_EINVAL, "null pointer argument");
    if (int rc = check_gbuffer(g)) return rc;
    return device_status(glint::launch_sample_filter(env, ind_j, ind_t, workspace, R, K, fp->num_mips, fp->taps, 2,
                                                     nullptr, nullptr, nullptr, g, P, F, nullptr,
                                                     (hipStream_t)stream),
                         "glint_filter_pixels launch");
}

int glint_surrogate_params(void) { return glint::mlp_params(); }

size_t glint_surrogate_workspace_bytes(int batch)
{
    if (batch < 1 || batch > (1 << 20)) return 0;
    const size_t blocks = (size_t)(batch + 31) / 32;
    return surrogate_partial_bytes(blocks) + ((blocks * sizeof(float) + 255) & ~(size_t)255);
}

int glint_surrogate_prepare(glint_ctx ctx, int K, float *w, uint16_t *w_bf16, void *stream)
{
    if (int rc = check_ctx(ctx)) return rc;
    glint::ProfScope prof_scope(&ctx->prof);
    if (int rc = check_surrogate(K, w, w_bf16)) return rc;
    const int rc = device_status(glint::launch_mlp_prepare(w, w_bf16, K, (hipStream_t)stream),
                                 "glint_surrogate_prepare launch");
    if (rc == GLINT_OK) mark_prepared(ctx, w_bf16, K);
    return rc;
}

int glint_surrogate_forward(glint_ctx ctx, int K, const float *w, const uint16_t *w_bf16, const float *x,
                            int64_t B, float *probs, void *stream)
{
    if (int rc = check_ctx(ctx)) return rc;
    glint::ProfScope prof_scope(&ctx->prof);
    if (int rc = check_surrogate(K, w, w_bf16)) return rc;
    if (B < 0 || B > ((int64_t)1 << 36)) return fail(GLINT_EINVAL, "bad batch size %lld", (long long)B);
    if (int rc = check_prepared(ctx, w_bf16, K)) return rc;
    if (B == 0) return ok();
    if (!x || !probs) return fail(GLINT_EINVAL, "null pointer argument");
    return device_status(glint::launch_mlp_forward(x, B, K, w, w_bf16, probs, (hipStream_t)stream),
                         "glint_surrogate_forward launch");
}

static int check_radiance_weight(const double *levels, float lam)
{
    if (!(lam >= 0.0f) || !(lam <= 1e3f)) return fail(GLINT_EINVAL, "radiance_weight must be in [0, 1000]");
    if (lam > 0.0f && !levels) return fail(GLINT_EINVAL, "a radiance weight needs the levels");
    return GLINT_OK;
}

int glint_surrogate_gradient(glint_ctx ctx, int K, const float *w, const uint16_t *w_bf16, const float *x,
                             const float *target, const double *levels, float radiance_weight, int B,
                             void *workspace, float *grad, float *loss, void *stream)
{
    if (int rc = check_ctx(ctx)) return rc;
    glint::ProfScope prof_scope(&ctx->prof);
    if (int rc = check_surrogate(K, w, w_bf16)) return rc;
    if (int rc = check_batch(B, x, target, workspace)) return rc;
    if (!grad || !loss) return fail(GLINT_EINVAL, "null pointer argument");
    if (int rc = check_radiance_weight(levels, radiance_weight)) return rc;
    if (int rc = check_prepared(ctx, w_bf16, K)) return rc;
    const size_t blocks = (size_t)(B + 31) / 32;
    float *partial = static_cast<float *>(workspace);
    float *loss_partial = reinterpret_cast<float *>(static_cast<char *>(workspace) + surrogate_partial_bytes(blocks));
    return device_status(glint::launch_mlp_gradient(x, target, radiance_weight > 0.0f ? levels : nullptr,
                                                    radiance_weight, B, K, w, w_bf16, partial, loss_partial, grad,
                                                    loss, (hipStream_t)stream),
                         "glint_surrogate_gradient launch");
}

int glint_surrogate_train_step(glint_ctx ctx, int K, float *w, uint16_t *w_bf16, float *m, float *v, int step,
                               float lr, const float *x, const float *target, const double *levels,
                               float radiance_weight, int B, void *workspace, float *loss, void *stream)
{
    if (int rc = check_ctx(ctx)) return rc;
    glint::ProfScope prof_scope(&ctx->prof);
    if (int rc = check_surrogate(K, w, w_bf16)) return rc;
    if (int rc = check_batch(B, x, target, workspace)) return rc;
    if (!m || !v || !loss) return fail(GLINT_EINVAL, "null pointer argument");
    if (step < 1) return fail(GLINT_EINVAL, "step must be >= 1");
    if (!(lr >= 0.0f) || !(lr < 1.0f)) return fail(GLINT_EINVAL, "learning rate must be in [0, 1)");
    if (int rc = check_radiance_weight(levels, radiance_weight)) return rc;
    if (int rc = check_prepared(ctx, w_bf16, K)) return rc;
    const size_t blocks = (size_t)(B + 31) / 32;
    float *partial = static_cast<float *>(workspace);
    float *loss_partial = reinterpret_cast<float *>(static_cast<char *>(workspace) + surrogate_partial_bytes(blocks));
    return device_status(glint::launch_mlp_grad_step(x, target, radiance_weight > 0.0f ? levels : nullptr,
                                                     radiance_weight, B, K, w, w_bf16, m, v, step, lr, partial,
                                                     loss_partial, loss, (hipStream_t)stream),
                         "glint_surrogate_train_step launch");
}

size_t glint_shade_surrogate_workspace_bytes(int64_t P, int K)
{
    if (P < 0 || P > ((int64_t)1 << 40) || K < 2 || K > 16) return 0;
    const size_t b = (size_t)P * (size_t)K * sizeof(float);
    return b < 256 ? 256 : (b + 255) & ~(size_t)255;
}

int glint_shade_surrogate(glint_ctx ctx, const glint_gbuffer *g, int64_t P, const glint_env *env, const float *w,
                          const uint16_t *w_bf16, const glint_shade_params *sp, void *workspace, float *radiance,
                          const glint_shade_debug *dbg, void *stream)
{
    if (int rc = check_ctx(ctx)) return rc;
    glint::ProfScope prof_scope(&ctx->prof);
    if (!g || !env || !sp) return fail(GLINT_EINVAL, "null pointer argument");
    if (P < 0) return fail(GLINT_EINVAL, "num_pixels must be >= 0");
    if (int rc = check_R(env->R)) return rc;
    if (int rc = check_tree_K(env->K)) return rc;
    if (int rc = check_mips(env->R, env->num_mips)) return rc;
    if (int rc = check_surrogate(env->K, w, w_bf16)) return rc;
    if (int rc = check_shade_params(*sp, -1)) return rc;
    if (sp->prob_mode != GLINT_PROBS_ENV || sp->lobe_taps != 0 || sp->vertices == 12 ||
        sp->tree != GLINT_TREE_BALANCED)
        return fail(GLINT_EUNSUPPORTED, "the surrogate form computes the map's probabilities with one lookup and "
                    "the balanced tree");
    if (int rc = check_prepared(ctx, w_bf16, env->K)) return rc;
    if (P == 0) return ok();
    if (!radiance || !workspace || !env->rgb_pyr || !env->levels || !env->lut_S || !env->lut_E)
        return fail(GLINT_EINVAL, "null pointer argument");
    if (int rc = check_gbuffer(g)) return rc;
    if (reinterpret_cast<uintptr_t>(env->rgb_pyr) % 16 || reinterpret_cast<uintptr_t>(workspace) % 16)
        return fail(GLINT_EINVAL, "rgb_pyr and workspace must be 16-byte aligned");
    if (P > ((int64_t)1 << 40)) return fail(GLINT_EINVAL, "num_pixels too large");
    float *F = static_cast<float *>(workspace);
    hipError_t e = glint::launch_mlp_lookup(*g, P, env->K, w, w_bf16, F, (hipStream_t)stream);
    if (e != hipSuccess) return device_status(e, "glint_shade_surrogate network launch");
    return device_status(glint::launch_shade(*g, P, *env, *sp, F, radiance, dbg, (hipStream_t)stream),
                         "glint_shade_surrogate launch");
}

int glint_shade_given_F(glint_ctx ctx, const glint_gbuffer *g, int64_t P, const glint_env *env, const float *F,
                        const glint_shade_params *sp, float *radiance, const glint_shade_debug *dbg, void *stream)
{
    if (int rc = check_ctx(ctx)) return rc;
    glint::ProfScope prof_scope(&ctx->prof);
    if (!g || !env || !sp) return fail(GLINT_EINVAL, "null pointer argument");
    if (P < 0) return fail(GLINT_EINVAL, "num_pixels must be >= 0");
    if (int rc = check_R(env->R)) return rc;
    if (int rc = check_tree_K(env->K)) return rc;
    if (int rc = check_mips(env->R, env->num_mips)) return rc;
    if (int rc = check_shade_params(*sp, -1)) return rc;
    if (sp->prob_mode != GLINT_PROBS_ENV || sp->lobe_taps != 0 || sp->vertices == 12 ||
        sp->tree != GLINT_TREE_BALANCED)
        return fail(GLINT_EUNSUPPORTED, "given filtered values are one lookup's, shaded with the map's "
                    "probabilities and the balanced tree");
    if (P == 0) return ok();
    if (!radiance || !F || !env->rgb_pyr || !env->levels || !env->lut_S || !env->lut_E)
        return fail(GLINT_EINVAL, "null pointer argument");
    if (int rc = check_gbuffer(g)) return rc;
    if (reinterpret_cast<uintptr_t>(env->rgb_pyr) % 16 || reinterpret_cast<uintptr_t>(F) % 4)
        return fail(GLINT_EINVAL, "rgb_pyr must be 16-byte and F 4-byte aligned");
    if (P > ((int64_t)1 << 40)) return fail(GLINT_EINVAL, "num_pixels too large");
    return device_status(glint::launch_shade(*g, P, *env, *sp, F, radiance, dbg, (hipStream_t)stream),
                         "glint_shade_given_F launch");
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
    glint::ProfScope prof_scope(&ctx->prof);
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
        if ((t.surrogate_w == nullptr) != (t.surrogate_w_bf16 == nullptr))
            return fail(GLINT_EINVAL, "environment %d: surrogate weights and their bf16 copy go together", e);
        if (t.surrogate_w) {
            if (int rc = check_surrogate(t.partition.K, t.surrogate_w, t.surrogate_w_bf16)) return rc;
            if (int rc = check_prepared(ctx, t.surrogate_w_bf16, t.partition.K)) return rc;
        }
    }
    for (int v = 0; v < n_views; ++v) {
        const glint_view &w = views[v];
        if (w.env_index < 0 || w.env_index >= n_env) return fail(GLINT_EINVAL, "view %d: env_index out of range", v);
        if (w.num_pixels < 0 || w.num_pixels > ((int64_t)1 << 40))
            return fail(GLINT_EINVAL, "view %d: bad num_pixels", v);
        if (int rc = check_shade_params(w.shade, v)) return rc;
        if (w.shade.sampler != GLINT_SAMPLER_DUAL || w.shade.prob_mode != GLINT_PROBS_ENV ||
            w.shade.lobe_taps != 0 || w.shade.vertices == 12 || w.shade.tree != GLINT_TREE_BALANCED)
            return fail(GLINT_EUNSUPPORTED, "view %d: batched frames use the dual-gated sampler, the balanced tree "
                        "and the map's probabilities with one lookup", v);
        if (!w.radiance) return fail(GLINT_EINVAL, "view %d: null radiance", v);
        if (envs[w.env_index].surrogate_w &&
            (!w.surrogate_F || reinterpret_cast<uintptr_t>(w.surrogate_F) % 16))
            return fail(GLINT_EINVAL, "view %d: its environment has a surrogate; surrogate_F must be a 16-byte "
                                      "aligned [num_pixels][K] buffer", v);
        if (int rc = check_gbuffer(&w.gbuf)) return rc;
    }
    return device_status(glint::frame_batched(ctx->batched, envs, n_env, views, n_views, workspace,
                                              (hipStream_t)stream),
                         "glint_frame_batched");
}

int glint_batched_tile_px(glint_ctx ctx)
{
    enter(ctx);
    return ctx ? ctx->batched.last_tile_px : 0;
}

int glint_profile_enable(glint_ctx ctx, int enable)
{
    if (int rc = check_ctx(ctx)) return rc;
    ctx->prof.reset();
    ctx->prof.enabled = enable != 0;
    // events for 1024 timed launches up front: creating them is slow and
    // would otherwise land inside the caller's timed region
    if (ctx->prof.enabled) ctx->prof.reserve(2048);
    return ok();
}

int glint_profile_select(glint_ctx ctx, const char *kernels)
{
    enter(ctx);
    if (!ctx) return fail(GLINT_EINVAL, "null context");
    ctx->prof.only = kernels ? kernels : "";
    return ok();
}

int glint_profile_collect(glint_ctx ctx, int *n_kernels)
{
    if (int rc = check_ctx(ctx)) return rc;
    if (!n_kernels) return fail(GLINT_EINVAL, "null pointer argument");
    const hipError_t e = ctx->prof.collect();
    *n_kernels = (int)ctx->prof.summary.size();
    return device_status(e, "glint_profile_collect");
}

int glint_profile_entry(glint_ctx ctx, int i, const char **name, double *total_ms, int64_t *launches)
{
    enter(ctx);
    if (!ctx) return fail(GLINT_EINVAL, "null context");
    if (i < 0 || i >= (int)ctx->prof.summary.size()) return fail(GLINT_EINVAL, "profile entry %d out of range", i);
    if (!name || !total_ms || !launches) return fail(GLINT_EINVAL, "null pointer argument");
    *name = ctx->prof.summary[i].name;
    *total_ms = ctx->prof.summary[i].total_ms;
    *launches = ctx->prof.summary[i].launches;
    return ok();
}

} // extern "C"
