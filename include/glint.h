/*
 * glint.h -- C ABI of the MI355X (gfx950) glint hot path.
 *
 * Real-time image-based lighting of glints (Kneiphof & Klein, EGSR 2025):
 *   per frame, the environment map is split into K area lights of constant
 *   radiance and each light's (fuzzy) indicator is filtered with the IBL
 *   kernel into a roughness pyramid (Sec. 5); per pixel, the footprint's
 *   microfacet count N_P (Sec. 3.2), the K reflection probabilities (Sec. 4,
 *   Eq. (probhk) with Eq. (rtiblndf)) and a hierarchical multinomial of
 *   dual-gated Gaussian binomials (Sec. 6, Alg. "Dual-gated Gaussian") give
 *   the glint radiance of Eq. (iblglints:fin).
 *
 * Conventions for every entry point:
 *   - Returns GLINT_OK (0) or a positive error code; nothing is thrown.
 *     glint_last_error(ctx) returns the message of the calling thread's
 *     last failed call on ctx (glint_last_error(NULL): of any call).
 *   - Pointers marked "device" are HIP device pointers (e.g. torch CUDA
 *     tensors' data_ptr()); the caller owns every buffer.  Entry points that
 *     take a stream never allocate device memory and never synchronise:
 *     work is enqueued on `stream` (a hipStream_t; NULL = default stream).
 *     Device faults surface on a later call or on glint_sync().
 *   - Arguments are validated on the host before anything is launched; a
 *     rejected call launches nothing and leaves every output untouched.
 *   - Concurrent calls on different streams must not share output buffers
 *     or workspaces.
 *
 * Cube-map layout: env[face][y][x][3] float32 RGB radiance, faces
 * +X,-X,+Y,-Y,+Z,-Z, texel centre s = 2(x+1/2)/R - 1, t = 2(y+1/2)/R - 1,
 * direction +X:(1,-t,-s) -X:(-1,-t,s) +Y:(s,1,t) -Y:(s,-1,-t) +Z:(s,-t,1)
 * -Z:(-s,-t,-1).  Pyramids are mip-major: mip m (face size R >> m) starts at
 * texel offset sum_{s<m} 6 (R>>s)^2, then [face][y][x].
 */
#ifndef GLINT_H
#define GLINT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GLINT_VERSION 1

enum glint_status {
    GLINT_OK = 0,
    GLINT_EINVAL = 1,       /* invalid argument (size, null pointer, option) */
    GLINT_EUNSUPPORTED = 2, /* valid but not implemented (option value) */
    GLINT_EDEVICE = 3,      /* HIP runtime error (launch, device query) */
    GLINT_ENOMEM = 4,       /* host allocation failed (context only) */
    GLINT_ENOTTRAINED = 5   /* surrogate parameters never prepared or trained in this context */
};

typedef enum glint_dtype {
    GLINT_F32 = 0,    /* 32-bit float */
    GLINT_F16 = 1,    /* IEEE half, round to nearest even */
    GLINT_BF16 = 2,   /* bfloat16, round to nearest even */
    GLINT_UNORM16 = 3 /* 16-bit unsigned normalised: round(v * 65535) */
} glint_dtype;

typedef struct glint_ctx_s *glint_ctx;

/* Library version (GLINT_VERSION of the build). */
int glint_version(void);

/* Message of the calling thread's last failed call on ctx ("" if its last
 * call on ctx succeeded or it made none); with ctx = NULL, of the thread's
 * last call of any entry point (including glint_create).  The string stays
 * valid until the thread's next call on the same context. */
const char *glint_last_error(glint_ctx ctx);

/* Creates a context bound to HIP device `device` (queries its properties).
 * *out receives the context.  GLINT_EINVAL for a bad device index or a null
 * out pointer; GLINT_EDEVICE if the device cannot be queried. */
int glint_create(int device, glint_ctx *out);
void glint_destroy(glint_ctx ctx);

/* Waits for all work on the context's device; reports device faults. */
int glint_sync(glint_ctx ctx);

/* ------------------------------------------------------------------------
 * Environment partition (Sec. 5, "Discrete Radiance Levels", "Fuzzy
 * Indicator Functions", Eq. (wkdefpractice)).
 *
 * Brightness of a texel is Rec. 709 luminance of its RGB (non-finite or
 * negative channels count as 0).  With Lmin = max(ell, min Y) and
 * Lmax = max(max Y, Lmin): levels[0] = 0, levels[K-1] = Lmax and, for
 * 1 <= k <= K-2:
 *   level_mode 0 (the paper's): min(Lmax, exp(lerp(ln Lmin, ln Lmax, k/(K-1))));
 *   level_mode 2: the same with (k-1)/(K-2), so that levels[1] = Lmin;
 *   level_mode 1 (regions by radiance quantiles): the solid-angle-weighted
 *     quantile of Y at q = k/(K-1), i.e. the smallest texel luminance y
 *     with C(y) >= q W, C(y) the total solid angle of the texels with
 *     Y <= y and W that of the sphere, clipped to [Lmin, Lmax].  Solid
 *     angles are exact per texel (from the antiderivative
 *     atan2(s t, sqrt(s^2 + t^2 + 1)) of the cube face's area element)
 *     and summed in 2^-55 fixed point, so the result does not depend on
 *     the summation order.
 * Each texel stores the interval
 * index j (largest j <= K-2 with levels[j] <= min(Y, Lmax)) and the lerp
 * factor t in [0,1] (linear space, weight_space 0, the paper's choice; log
 * space for j >= 1 with weight_space 1); the fuzzy indicator weights are
 * w_j = 1 - t, w_{j+1} = t.  t = 1 when levels[j+1] == levels[j].
 * ------------------------------------------------------------------------ */
typedef struct glint_partition_params {
    int K;            /* number of radiance levels, 2..16 */
    double ell;       /* lower clip of the minimum radiance (> 0), e.g. 1e-3 */
    int level_mode;   /* 0 (paper), 1 (radiance quantiles) or 2 */
    int weight_space; /* 0 linear (paper) or 1 log */
} glint_partition_params;

/* Device workspace (bytes) glint_partition_env needs for a face size R
 * (any level mode; the quantile mode's solid-angle table of one face
 * quadrant grows as R^2 / 4 * 8 bytes: 128 KB at R = 256, 32 MB at 4096). */
size_t glint_partition_workspace_bytes(int R);

/* env: device [6][R][R][3] float32.  workspace: device, at least
 * glint_partition_workspace_bytes(R) bytes, 8-byte aligned, no initial
 * contents required.  Outputs (device): levels [K] double,
 * ind_j [6][R][R] uint8, ind_t [6][R][R] float32.
 * GLINT_EINVAL: R not a power of two in [1, 4096], K outside 2..16,
 * ell <= 0, an option out of range, or a null pointer. */
int glint_partition_env(glint_ctx ctx, const float *env, int R, const glint_partition_params *params,
                        void *workspace, double *levels, uint8_t *ind_j, float *ind_t, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * operation as glint_partition_env without the workspace argument.  Its
 * workspace is a scratch array of 2,359,296 bytes that the library holds on
 * each GPU until the process ends (looked up per device by glint_create);
 * this call allocates nothing.  Every call on one GPU shares that array and
 * leaves its contents behind (each call rebuilds what it reads), so calls
 * that overlap on one GPU -- on different streams, threads or contexts --
 * race and must be ordered by the caller.  Arguments, outputs and errors as
 * glint_partition_env; GLINT_EINVAL also when the face size needs more
 * scratch than the array holds (level_mode 1 above R = 1024; levels modes 0
 * and 2 fit every R). */
int glint_partition_env_noalloc(glint_ctx ctx, const float *env, int R, const glint_partition_params *params,
                                double *levels, uint8_t *ind_j, float *ind_t, void *stream);

/* ------------------------------------------------------------------------
 * Prefilter (Sec. 5 "Integrated NDF", Eq. (rtiblndf) with the real-time IBL
 * kernel of Sec. 3.4, Eq. (rtibl), assuming n = v = r).  The K indicator
 * channels and RGB are filtered with the same kernel.
 *
 * Source: a mip chain of the dense indicator weights + RGB (level 0 exact,
 * level s+1 the float-stored 2x2 mean of level s).  Mip m of the output
 * (roughness alpha_m = (m/(M-1))^2; mip 0 is the unfiltered level) is
 *   F(r) = sum_j W_j v(l_j, lod_j) / sum_j W_j
 * over T GGX-importance-sampled Hammersley taps around r (tap j: azimuth
 * 2 pi j/T, cos^2 theta = (1-u)/(1+(alpha^2-1)u) with u the base-2 radical
 * inverse of j), l_j the mirror of r about the tap's half vector,
 * W_j = <r,l_j>+, lod_j = clamp(log2(Omega_s/Omega_p)/2 + 1, 0, M-1) with
 * Omega_s = 4/(T D(h_j)) and Omega_p = 4 pi/(6 R^2) (filtered importance
 * sampling), v a trilinear lookup of the chain.  Seams: a texel one step
 * beyond a face edge is the nearest texel of the face that owns its centre's
 * direction (the adjacent texel); the texel beyond a cube corner is the mean
 * of the three texels meeting there, so lookups are continuous.  Shading
 * reads the pyramid with the same rule.  The eight weighted corners of one
 * tap's trilinear lookup are summed in float (non-negative terms: relative
 * error below 9 * 2^-24), the taps and the normalisation in double; results
 * are rounded once to the stored type.
 * ------------------------------------------------------------------------ */
typedef struct glint_prefilter_params {
    int num_mips;      /* M, 1 <= M <= log2(R) + 1 */
    int taps;          /* T, 1..1024 (never tuned: it changes results) */
    glint_dtype dtype; /* storage type of the indicator pyramid */
} glint_prefilter_params;

/* Texels of an M-level pyramid of face size R: sum_m 6 (R>>m)^2. */
int64_t glint_pyramid_texels(int R, int num_mips);

/* Device workspace (bytes) for the source mip chain. */
size_t glint_prefilter_workspace_bytes(int R, int K, const glint_prefilter_params *params);

/* env: device [6][R][R][3] float32; ind_j, ind_t: device, as written by
 * glint_partition_env.  workspace: device, >= glint_prefilter_workspace_bytes,
 * 16-byte aligned.  Outputs (device): ind_pyr [texels][K] of params->dtype;
 * rgb_pyr [texels][4] float32 (RGB, 4th channel 0).
 * GLINT_EINVAL: bad R, K, M, T or dtype, or a null pointer. */
int glint_prefilter(glint_ctx ctx, const float *env, const uint8_t *ind_j, const float *ind_t, int R, int K,
                    const glint_prefilter_params *params, void *workspace, void *ind_pyr, float *rgb_pyr,
                    void *stream);

/* ------------------------------------------------------------------------
 * The filter of Sec. 5 at arbitrary (direction, roughness): the same
 * quadrature as glint_prefilter (tap table built for the given alpha rather
 * than alpha_m = (m/(M-1))^2, trilinear lookups of the source chain), for
 * checking the pyramid and for producing training targets of the learned
 * surrogate.  workspace: the prefilter workspace that the most recent
 * glint_prefilter call for the same env, R, K and params filled (it holds
 * the source mip chain); it is only read.  dirs: device [n][3] float32
 * directions (normalised here, need not be unit).
 * ------------------------------------------------------------------------ */

/* alphas: device [n] float32 GGX roughness in (0, 1].  out: device
 * [n][K+3] float32, the K filtered indicator values then RGB.
 * GLINT_EINVAL: bad R, K, M, T, n < 0 or a null pointer (n = 0: no-op). */
int glint_sample_filter(glint_ctx ctx, const float *env, const uint8_t *ind_j, const float *ind_t, int R, int K,
                        const glint_prefilter_params *params, const void *workspace, const float *dirs,
                        const float *alphas, int64_t n, float *out, void *stream);

/* Training pairs of the learned surrogate (see below): for each sample the
 * filter at alpha = sqrt(alpha_x alpha_y) (the isotropic roughness that
 * shading uses), x [n][5] = surrogate inputs of (dir, alpha_x, alpha_y)
 * and target [n][K] = F_k / sum F (1/K each if sum F = 0).  ax, ay: device
 * [n] float32 in (0, 1].  The caller draws dirs, ax and ay (e.g. dirs
 * uniform on the sphere, ln alpha uniform in [ln 0.02, ln 0.5]). */
int glint_surrogate_samples(glint_ctx ctx, const float *env, const uint8_t *ind_j, const float *ind_t, int R,
                            int K, const glint_prefilter_params *params, const void *workspace, const float *dirs,
                            const float *ax, const float *ay, int64_t n, float *x, float *target, void *stream);

/* ------------------------------------------------------------------------
 * Learned surrogate of the indicator lookup (an extension, not the
 * paper's method).  An MLP maps x = (w_x, w_y, w_z, (ln alpha_x - c)/h,
 * (ln alpha_y - c)/h), c and h mapping [ln 0.02, ln 0.5] onto [-1, 1], to
 * softmax probabilities that stand in for F_k / sum F in Eq. (probhk):
 * 5 -> 64 -> 64 -> 64 -> K, SiLU hidden units.  The dense layers run on
 * the matrix cores with bfloat16 weights and activations (round to nearest
 * even) and float32 accumulation; biases, softmax and the error signals'
 * scaling are float32.
 *
 * Parameters: a flat float32 master of glint_surrogate_params() entries,
 * padded for 32 x 32 x 16 matrix tiles:
 *   W1 [64][16] (columns 5..15 zero), b1 [64], W2 [64][64], b2 [64],
 *   W3 [64][64], b3 [64], W4 [32][64] (rows K..31 zero), b4 [32] (K.. zero)
 * and a bfloat16 copy (uint16_t bit patterns, same layout, 16-byte aligned)
 * that the matrix cores read.  Loss: mean over the batch of the soft-label
 * cross-entropy -sum_k t_k ln y_k, plus, with the radiance levels L given
 * and weight lam > 0, lam times the cross-entropy -sum_{k>=1} t'_k ln y'_k
 * of the radiance-weighted distributions over the bins k >= 1,
 * y'_k = L_k y_k / sum_{j>=1} L_j y_j and t'_k likewise (samples with
 * sum_{j>=1} L_j t_j = 0 add no such term).  The glint radiance of a pixel
 * moves with sum_k L_k |dp_k| / sum_k L_k p_k (Eq. (iblglints:fin)), so the
 * second term weights each bin's relative error by its radiance.
 * ------------------------------------------------------------------------ */

/* Entries of the padded parameter layout (11488). */
int glint_surrogate_params(void);

/* Device workspace (bytes) of glint_surrogate_gradient and
 * glint_surrogate_train_step for a batch of B samples (per-block partial
 * gradients); 0 if B is outside 1..2^20. */
size_t glint_surrogate_workspace_bytes(int batch);

/* Zeroes the pad entries of the master w (device) and writes the bfloat16
 * copy w_bf16 (device).  Call after writing or loading w.  The context
 * records w_bf16 (its address) and K: the calls below that read the
 * network return GLINT_ENOTTRAINED for a w_bf16 that was never prepared or
 * updated by glint_surrogate_train_step in this context, or was prepared
 * for another K (a host-side check of the address, not of the contents). */
int glint_surrogate_prepare(glint_ctx ctx, int K, float *w, uint16_t *w_bf16, void *stream);

/* Forward pass: x device [B][5] float32 -> probs device [B][K] float32.
 * K in 2..32; GLINT_EINVAL for bad sizes or null pointers. */
int glint_surrogate_forward(glint_ctx ctx, int K, const float *w, const uint16_t *w_bf16, const float *x,
                            int64_t B, float *probs, void *stream);

/* Gradient of the mean loss over the batch: grad device [params] float32
 * (pad entries 0), loss device float32 scalar.  x [B][5], target [B][K];
 * levels: device [K] double (e.g. from glint_partition_env) or NULL, used
 * when radiance_weight (lam, in [0, 1000]) is > 0; workspace device,
 * >= glint_surrogate_workspace_bytes(B), 16-byte aligned.  The per-block
 * partial gradients are summed in a fixed order, so results are
 * deterministic. */
int glint_surrogate_gradient(glint_ctx ctx, int K, const float *w, const uint16_t *w_bf16, const float *x,
                             const float *target, const double *levels, float radiance_weight, int B,
                             void *workspace, float *grad, float *loss, void *stream);

/* One training step: the gradient as above, then Adam (beta1 0.9, beta2
 * 0.999, eps 1e-8, bias correction with step >= 1) on the master w with
 * moments m, v (device [params] float32, zero before step 1), then the
 * bfloat16 copy is refreshed.  loss receives the batch loss before the
 * update.  lr: the step's learning rate (schedules are the caller's). */
int glint_surrogate_train_step(glint_ctx ctx, int K, float *w, uint16_t *w_bf16, float *m, float *v, int step,
                               float lr, const float *x, const float *target, const double *levels,
                               float radiance_weight, int B, void *workspace, float *loss, void *stream);

/* ------------------------------------------------------------------------
 * Lookup tables, once per BRDF model (isotropic GGX, Schlick Fresnel,
 * height-correlated Smith), on a 64 x 64 cell-centred grid over
 * (sqrt(alpha) rows, mu_o = <n,v> columns):
 *   lut_S[a][m]      = E_D / D_H, the visible reflecting facet area of
 *                      Sec. 5 over the total facet area of Sec. 3.2;
 *   lut_E[a][m][0,1] = split-sum albedo E_rho = F0 * [0] + [1] (Sec. 3.4).
 * Midpoint quadrature in GGX half-vector coordinates (double), stored float.
 * Outputs: device float32 arrays [64][64] and [64][64][2].
 * ------------------------------------------------------------------------ */
int glint_build_luts(glint_ctx ctx, float *lut_S, float *lut_E, void *stream);

/* ------------------------------------------------------------------------
 * Tail table of the Gaussian quantile (an implementation aid, same results).
 * Shading draws xi2 = (h9 + 1/2) 2^-23 from the 23-bit hash value h9; the
 * quantile (AS 241) takes its tail branch (|xi2 - 1/2| > 0.425) exactly for
 * h9 < 629146 or h9 > 7759461.  The table holds the quantile of those
 * 1,258,292 values (double, low tail then high tail, ascending h9),
 * computed by the same device code as the per-draw evaluation, so shading
 * with or without it gives bit-identical results; with it, a draw in a tail
 * is one load instead of a divergent log, square root and rational function.
 * Build once per context; `table` is device memory of
 * glint_quantile_table_bytes() bytes, 8-byte aligned.
 * ------------------------------------------------------------------------ */
size_t glint_quantile_table_bytes(void);
int glint_build_quantile_table(glint_ctx ctx, double *table, void *stream);

/* ------------------------------------------------------------------------
 * Binomial approximations b(N, p) of Sec. 6, one draw per element, with the
 * random numbers given: xi1 = ((h1 >> 9) + 1/2) 2^-23 decides the gates and
 * xi2 = ((h2 >> 9) + 1/2) 2^-23 the Gaussian, as the shading kernel maps its
 * hash outputs.  N >= 0 and p in [0, 1] are real.
 *  GLINT_SAMPLER_DUAL: Alg. "Dual-gated Gaussian" with the bias of
 *    paragraph "Numeric Gating Issues" (the node sampler of glint_shade).
 *  GLINT_SAMPLER_SINGLE: Eq. (gated), the single-gated Gaussian generalised
 *    to real N: gate passed with probability min(N p, 1 - (1-p)^N), the
 *    power with the same bias; past it, the Gaussian of mean 1 + (N1-1) p
 *    and variance (N1-1) p (1-p), N1 = max(N, 1), clamped to [1, N1].
 *  GLINT_SAMPLER_SINGLE_FLOOR: Eq. (oldgated), the prior form: gate
 *    probability 1 - (1-p)^N without bias, floor of the same clamped
 *    Gaussian.
 *  GLINT_SAMPLER_DUAL_SYMMETRIC: the dual gate with the bias of "Numeric
 *    Gating Issues" on both powers: P(n = N) = (1 - max(q, eps))^(N2
 *    min(1, q/eps)) with q the negative side's probability computed on its
 *    own (here 1 - p in double; in shading the tree node's right share
 *    S_right / S), instead of p^N2.  The printed algorithm biases only
 *    (1 - p)^N2; in a multinomial tree the rare side of a node may be
 *    either child (the bright bins sit on the right), and for q < 2^-25
 *    float(p) = 1 makes p^N2 = 1: no facet ever reaches that side, however
 *    large N.  This form keeps those draws within the paper's error
 *    bound.
 * Single-gated forms return nbar = max(N - n, 0).  Gates are evaluated in
 * float (the decisions of powf thresholds; exact_gating = 1 evaluates powf
 * for every draw), the Gaussian (AS 241) in double.
 * All arrays are device memory of `count` elements; quantile_tail may be
 * NULL (see glint_build_quantile_table).  code: bits as in
 * glint_shade_debug for the dual form; 1 = gate passed, 16 = Gaussian for
 * the single forms.  GLINT_EINVAL: unknown sampler, count < 0 or a null
 * array (count = 0 is a no-op).
 * ------------------------------------------------------------------------ */
#define GLINT_SAMPLER_DUAL 0
#define GLINT_SAMPLER_SINGLE 1
#define GLINT_SAMPLER_SINGLE_FLOOR 2
#define GLINT_SAMPLER_DUAL_SYMMETRIC 3
int glint_sample_binomial(glint_ctx ctx, int sampler, int exact_gating, const double *N, const double *p,
                          const uint32_t *h1, const uint32_t *h2, int64_t count, const double *quantile_tail,
                          double *n, double *nbar, uint8_t *code, void *stream);

/* ------------------------------------------------------------------------
 * Per-pixel glint shading (Sec. 3.2, Sec. 3.3 Eq. (anisogrid), Sec. 4
 * Eq. (probhk) and Eq. (iblglints:fin), Sec. 6 Alg. "Dual-gated Gaussian").
 *
 * Per pixel: N_P = density * area (stratified count); w_r = 2<n,v>n - v;
 * alpha = sqrt(alpha_x alpha_y); F = trilinear pyramid lookup at (w_r,
 * lod = sqrt(alpha)(M-1)); p_k = S F_k / sum F for k >= 1 and
 * p_0 = 1 - sum_{k>=1} p_k (level 0 has zero radiance and absorbs facets
 * that reflect nothing); L_o = (F0 A + B) RGB(w_r, lod).
 * Counts: a balanced binary tree over the K bins (K a power of two, nodes
 * in breadth-first order), node probability S_left / S_node, the left child
 * receiving the positive count n and the right child the negative count
 * nbar of the dual-gated Gaussian (or of the single-gated forms, selected
 * by params->sampler, see glint_sample_binomial).  With tree =
 * GLINT_TREE_CHAIN the multinomial is a sequential chain instead (Sec. 6
 * does not fix the shape): node i (0..K-2) draws bin i's count out of the
 * N_i facets that reach it with probability p_i / S_i, S_i = p_i + S_{i+1}
 * (S_{K-1} = p_{K-1}), nbar goes on to node i+1 (N_0 = N_P) and bin K-1
 * keeps what reaches it; the node ids of the hash are 0..K-2 in chain
 * order.  Gating probabilities and masks are
 * evaluated in float with the bias c = max(1, eps/p), eps = 10^-3.54
 * (Sec. 6 "Numeric Gating Issues"); the Gaussian quantile (AS 241) and all
 * other arithmetic in double.  Random numbers per (surface, lattice vertex,
 * node) from the pcg4d hash (Jarzynski & Olano 2020), one hash per pair of
 * nodes: node 2i takes outputs (x, y), node 2i+1 outputs (z, w).
 * Lattice (the footprint grid of Sec. 3.3, used as a black box by the
 * paper): level l0 = floor(log2(area)/2) on the uv plane, spacing 2^l0.
 * vertices = 1: the nearest vertex; vertices = 6: the 3 vertices of the uv
 * triangle containing the point at levels l0 and l0+1, barycentric weights
 * times (1-f, f), f = log2(area)/2 - l0.  Each vertex draws with N_i = N_P;
 * the counts are blended with the weights.
 * vertices = 12, the footprint grid (Sec. 3.3 describes the footprint by
 * length, anisotropy and orientation and distributes its facets over a
 * tetrahedral cell of that space; the layout is this library's): with
 * J = [[du/dx, du/dy], [dv/dx, dv/dy]], s_maj = sqrt(largest eigenvalue of
 * J J^T), s_min = max(|det J| / s_maj, s_maj / 16), theta in [0, pi) the
 * major axis; grid coordinates (log2 s_maj, log2(s_maj/s_min), 8 theta/pi)
 * (orientation periodic, 8 cells); the Kuhn tetrahedron (axes by
 * decreasing fraction, ties in axis order) gives 4 vertices (l, a, o) with
 * weights (1-f1, f1-f2, f2-f3, f3); vertex (l, a, o) draws
 * N_i = N_P (4^l / 2^a) / (s_maj s_min) facets at the 3 vertices of the uv
 * triangle grid of its footprint (uv rotated by -o pi/8, scaled by
 * (2^-l, 2^(a-l)), squares split along the diagonal, barycentric weights),
 * hash key (lattice x, lattice y, l << 24 | a << 20 | o << 16 | node/2);
 * the radiance is normalised by sum_i w_i N_i instead of N_P.  A zero
 * Jacobian draws nothing (radiance 0).
 * Radiance = L_o * sum_k L_k M_k / (N_P sum_k L_k p_k) (0 if either sum is 0).
 * Occlusion (Sec. 8 "Limitations & Future Work": attenuate the
 * probabilities, not the output): with gbuf->visibility, the tree samples
 * with p'_k = v p_k (k >= 1), p'_0 = 1 - sum_{k>=1} p'_k, while the
 * normalisation keeps the unattenuated p_k, so the expected radiance is
 * v L_o and each glint keeps its brightness.
 * Anisotropic lookup (Sec. 8 names several samples of the prefiltered map
 * as the way to anisotropic distributions; the tap layout is this
 * library's): with lobe_taps = T, F and RGB are the mean, weighted by
 * <n, w_j>+, of T trilinear lookups at lod sqrt(a_t)(M-1),
 * a_t = max(a_min, a_max/T), in directions
 * w_j = 2<v,h_j>h_j - v, h_j = (n - x_j d)/sqrt(1+x_j^2), x_j = s u_j/sqrt(1-u_j^2),
 * u_j = (2j+1)/T - 1, s = sqrt(a_max^2 - a_t^2), d the tangent made
 * orthogonal to n (n x d when alpha_y > alpha_x).  S and E_rho stay at
 * alpha = sqrt(alpha_x alpha_y).
 * prob_mode = GLINT_PROBS_CONSTANT (Sec. 7 "Comparison with Previous Work",
 * after Wang et al. 2020): p = (1 - gamma, gamma) and levels (0, 1) for
 * every pixel, i.e. the two-bin case of the same path; the indicator
 * pyramid, env->levels and lut_S are not read, env->K and env->dtype are
 * ignored and the debug outputs are laid out for K = 2.
 * ------------------------------------------------------------------------ */
#define GLINT_NO_SURFACE 0xFFFFFFFFu

typedef struct glint_gbuffer {
    /* device float32 arrays of num_pixels entries each (structure of arrays) */
    const float *nx, *ny, *nz; /* unit surface normal */
    const float *vx, *vy, *vz; /* unit vector towards the viewer */
    const float *u, *v;        /* surface uv (lattice coordinates) */
    const float *area;         /* footprint area |P| (> 0) */
    const float *ax, *ay;      /* GGX roughness alpha_x, alpha_y */
    const float *density;      /* microfacets per unit area N */
    const float *f0r, *f0g, *f0b; /* Fresnel reflectance at normal incidence */
    const uint32_t *surf_id;   /* surface id (hash input); GLINT_NO_SURFACE = background */
    const float *visibility;   /* optional (NULL: unoccluded): unoccluded fraction v in [0, 1] of the
                                  pixel's reflection lobe; scales the reflection probabilities, see
                                  glint_shade */
    const float *tx, *ty, *tz; /* optional surface tangent, the axis of alpha_x (needed only for
                                  anisotropic lookups, glint_shade_params.lobe_taps > 0) */
    const float *dudx, *dudy, *dvdx, *dvdy; /* optional uv Jacobian of the pixel footprint (needed
                                  only for the footprint grid, vertices = 12) */
} glint_gbuffer;

typedef struct glint_env {
    const void *ind_pyr;   /* device [texels][K], dtype below (from glint_prefilter) */
    const float *rgb_pyr;  /* device [texels][4] float32 */
    const double *levels;  /* device [K] (from glint_partition_env) */
    const float *lut_S;    /* device [64][64] */
    const float *lut_E;    /* device [64][64][2] */
    int R, K, num_mips;
    glint_dtype dtype;
    const double *quantile_tail; /* device table from glint_build_quantile_table, or NULL
                                    (then the quantile's tails are evaluated per draw) */
} glint_env;

typedef struct glint_shade_params {
    uint32_t seed;    /* material seed mixed into the hash */
    int vertices;     /* 1, 6 or 12 (the footprint grid; float32 pyramid, dual gate, map
                         probabilities, one lookup; needs the G-buffer uv Jacobian) */
    int exact_gating; /* 0: gating decisions from hardware log2/exp2 powers, re-evaluated with powf
                         only within a safety margin of a threshold (same decisions); 1: always
                         powf (for verification) */
    int sampler;      /* binomial approximation at every tree node (see glint_sample_binomial):
                         GLINT_SAMPLER_DUAL (the paper's method), GLINT_SAMPLER_DUAL_SYMMETRIC,
                         GLINT_SAMPLER_SINGLE, GLINT_SAMPLER_SINGLE_FLOOR; the single-gated forms
                         need a float32 pyramid; glint_frame_batched runs GLINT_SAMPLER_DUAL only
                         (GLINT_EUNSUPPORTED for the others) */
    int prob_mode;    /* GLINT_PROBS_ENV: p_k from the map (the paper's method);
                         GLINT_PROBS_CONSTANT: every facet reflects with probability gamma,
                         independent of the map (the comparison of Sec. 7) */
    float gamma;      /* in (0, 1], GLINT_PROBS_CONSTANT only */
    int lobe_taps;    /* 0: one lookup at alpha = sqrt(alpha_x alpha_y); 2, 4 or 8: anisotropic
                         lookup with that many taps along the lobe (see glint_shade; needs the
                         G-buffer tangent; float32 pyramid, dual-gated sampler, GLINT_PROBS_ENV) */
    int tree;         /* shape of the hierarchical multinomial: GLINT_TREE_BALANCED (binary tree,
                         the default) or GLINT_TREE_CHAIN (sequential chain; float32 pyramid,
                         dual-gated sampler, GLINT_PROBS_ENV, one lookup, vertices 1 or 6, plain
                         form; not in glint_frame_batched) */
} glint_shade_params;

#define GLINT_PROBS_ENV 0
#define GLINT_PROBS_CONSTANT 1
#define GLINT_TREE_BALANCED 0
#define GLINT_TREE_CHAIN 1

/* Optional per-pixel outputs for verification (each pointer may be NULL). */
typedef struct glint_shade_debug {
    double *counts; /* device [P][vertices][K]: multinomial counts per vertex */
    uint8_t *codes; /* device [P][vertices][K-1]: gating mask bits per node:
                       1 n=N, 2 n in {1,N}, 4 nbar=N, 8 nbar in {1,N}, 16 Gaussian */
    double *probs;  /* device [P][K]: reflection probabilities p_k */
} glint_shade_debug;

/* radiance: device [P][3] float32 (background pixels get 0).  debug may be
 * NULL.  GLINT_EINVAL: P < 0, K not in {2,4,8,16}, bad R/M/dtype/vertices or
 * a null pointer (P = 0 is a no-op). */
int glint_shade(glint_ctx ctx, const glint_gbuffer *gbuf, int64_t num_pixels, const glint_env *env,
                const glint_shade_params *params, float *radiance, const glint_shade_debug *debug,
                void *stream);

/* Device workspace (bytes) of glint_shade_surrogate: the surrogate's
 * outputs for num_pixels pixels ([P][K] float32). */
size_t glint_shade_surrogate_workspace_bytes(int64_t num_pixels, int K);

/* Surrogate form of glint_shade: F_k / sum F of each surface pixel comes
 * from the network at (w_r, alpha_x, alpha_y) instead of the indicator
 * pyramid, which is not read (env->ind_pyr may be NULL; env->dtype is
 * ignored); RGB, S and E_rho are read as in glint_shade and the rest of
 * the pixel's arithmetic is unchanged.  w, w_bf16: parameters for env->K.
 * workspace: device, >= glint_shade_surrogate_workspace_bytes, 16-byte
 * aligned.  Errors as glint_shade. */
int glint_shade_surrogate(glint_ctx ctx, const glint_gbuffer *gbuf, int64_t num_pixels, const glint_env *env,
                          const float *w, const uint16_t *w_bf16, const glint_shade_params *params,
                          void *workspace, float *radiance, const glint_shade_debug *debug, void *stream);

/* The filter at the lookup of every G-buffer pixel: reflection direction
 * 2<n,v>n - v and alpha = sqrt(alpha_x alpha_y), computed as glint_shade
 * computes them, at that continuous roughness (no mip interpolation).
 * F: device [P][K] float32, the K filtered indicator values per pixel (0
 * for background pixels).  With glint_shade_given_F this shades with the
 * plain filter itself: the reference that the pyramid's and the
 * surrogate's errors are measured against.  Errors as glint_sample_filter,
 * plus GLINT_EINVAL for a G-buffer with a null field. */
int glint_filter_pixels(glint_ctx ctx, const float *env, const uint8_t *ind_j, const float *ind_t, int R, int K,
                        const glint_prefilter_params *params, const void *workspace, const glint_gbuffer *gbuf,
                        int64_t num_pixels, float *F, void *stream);

/* Shading with the K filtered indicator values of every pixel given
 * (F [num_pixels][K] float32, device; any positive scale): p_k =
 * S F_k / sum F as in glint_shade, RGB, S and E_rho read from env, the
 * indicator pyramid not read (env->ind_pyr may be NULL, env->dtype is
 * ignored).  This is the second step of glint_shade_surrogate; with F from
 * glint_sample_filter at each pixel's reflection direction and
 * sqrt(alpha_x alpha_y) it shades with the plain filter itself (no mip
 * interpolation), the reference the surrogate and the pyramid are judged
 * against.  Errors as glint_shade_surrogate. */
int glint_shade_given_F(glint_ctx ctx, const glint_gbuffer *gbuf, int64_t num_pixels, const glint_env *env,
                        const float *F, const glint_shade_params *params, float *radiance,
                        const glint_shade_debug *debug, void *stream);

/* ------------------------------------------------------------------------
 * Batched frame: several environment maps and many views of uneven size,
 * with mixed K, materials and vertex counts, in one graph launch.  The
 * result is defined as glint_partition_env + glint_prefilter for every
 * environment followed by glint_shade (or glint_shade_surrogate, for views
 * of an environment that carries surrogate parameters) for every view (no
 * debug outputs); outputs are bit-identical to those calls.
 *
 * The first call for a given argument set (compared byte-wise, including
 * the pointers) is a set-up call: it times the shading launch for each
 * candidate tile size (pixels per workgroup: 64, 128, 256; results do not
 * depend on the choice) and keeps the fastest per (K, dtype, vertices,
 * form, size class) in the context, uploads the view descriptors into
 * `workspace`, and captures the frame into a HIP graph: one branch per
 * environment on the context's side streams (the maps are filtered
 * concurrently) and one shading launch per (K, vertices, plain/surrogate)
 * group, covering all views of the group, on a branch of its own that
 * waits only for the environments those views are lit by (a group's
 * shading overlaps the filtering of the other maps and the other groups'
 * shading).  The set-up
 * call synchronises the stream and lets the HIP runtime allocate graph
 * objects.  Later calls with the same arguments enqueue exactly one
 * hipGraphLaunch and allocate nothing.  A workspace holds the descriptors of
 * one argument set: a set-up call drops every graph captured on the same
 * workspace, so alternating argument sets on one workspace repeats the
 * set-up each time (give each set its own workspace to keep both graphs).
 * Every environment's outputs and every view's radiance must be distinct
 * buffers; env_index selects the environment a view is lit by.
 * ------------------------------------------------------------------------ */
typedef struct glint_env_task {
    const float *env;               /* device [6][R][R][3] */
    int R;
    glint_partition_params partition;
    glint_prefilter_params prefilter;
    void *partition_workspace;      /* device, >= glint_partition_workspace_bytes(R) */
    void *prefilter_workspace;      /* device, >= glint_prefilter_workspace_bytes(R, K, &prefilter) */
    double *levels;                 /* outputs, as glint_partition_env / glint_prefilter */
    uint8_t *ind_j;
    float *ind_t;
    void *ind_pyr;
    float *rgb_pyr;
    const float *lut_S, *lut_E;     /* device LUTs from glint_build_luts */
    const double *quantile_tail;    /* device table from glint_build_quantile_table, or NULL */
    /* Surrogate form (NULL, NULL: plain form): the parameters of a network
     * for this environment's K (see glint_shade_surrogate); views lit by
     * this environment are shaded with it. */
    const float *surrogate_w;
    const uint16_t *surrogate_w_bf16;
} glint_env_task;

typedef struct glint_view {
    glint_gbuffer gbuf;
    int64_t num_pixels;
    int env_index;                  /* 0 .. n_env-1 */
    glint_shade_params shade;
    float *radiance;                /* device [num_pixels][3] */
    float *surrogate_F;             /* device [num_pixels][K] f32 workspace, 16-byte aligned, when the
                                       view's environment has a surrogate (else ignored) */
} glint_view;

/* Device workspace (bytes) for n_views views; the workspace passed to
 * glint_frame_batched must be 256-byte aligned. */
size_t glint_batched_workspace_bytes(int n_views);

/* GLINT_EINVAL for null pointers, n_env outside 1..64, n_views outside
 * 1..4096, an env_index out of range, or any per-environment or per-view
 * argument glint_partition_env / glint_prefilter / glint_shade would
 * reject; GLINT_EUNSUPPORTED for a view whose shading parameters ask for
 * another sampler than GLINT_SAMPLER_DUAL, constant probabilities, the
 * anisotropic lookup, the footprint grid or the sequential chain.  All
 * environments in one call share one pyramid dtype. */
int glint_frame_batched(glint_ctx ctx, const glint_env_task *envs, int n_env, const glint_view *views,
                        int n_views, void *workspace, void *stream);

/* Tile size (pixels per workgroup) the autotuner chose for the largest
 * (K, vertices) group of the most recent set-up call; 0 before any. */
int glint_batched_tile_px(glint_ctx ctx);

/* ------------------------------------------------------------------------
 * Per-kernel timing, for benchmarks and profiling.  While enabled, every
 * kernel that an entry point of this context launches (outside a stream
 * capture) is bracketed by two HIP events recorded on its launch stream;
 * the events travel with the dispatch, but the runtime adds a few
 * microseconds per timed launch, so time only the kernels of interest.
 * ------------------------------------------------------------------------ */

/* Enables (1) or disables (0) timing; either way drops every record. */
int glint_profile_enable(glint_ctx ctx, int enable);

/* Restricts timing to the kernels named in `kernels` (comma-separated, e.g.
 * "k_prefilter,k_shade"); NULL or "" times every kernel. */
int glint_profile_select(glint_ctx ctx, const char *kernels);

/* Waits for the recorded events (synchronising with the streams they were
 * recorded on), adds their durations to per-kernel totals and stores the
 * number of distinct kernels in *n_kernels. */
int glint_profile_collect(glint_ctx ctx, int *n_kernels);

/* Entry i < *n_kernels of the totals: kernel name (a static string owned
 * by the library), total milliseconds and number of launches. */
int glint_profile_entry(glint_ctx ctx, int i, const char **name, double *total_ms, int64_t *launches);

#ifdef __cplusplus
}
#endif

#endif /* GLINT_H */
