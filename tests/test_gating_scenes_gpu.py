"""Scenes for the gating comparisons of Sec. 7 ("Improved Single-Gated
Gaussians", "Numeric Gating Issues"; Sec. 6 "Gating Generalization"),
built from environment maps instead of the paper's directional and point
lights, on the GPU against the oracle.

Wide light, N < 1 (Fig. result_nlt1): a large area light at the zenith
(its own radiance level) above a glossy plane whose microfacet count per
footprint sweeps 0.03 .. 100 and 1e6 over the rows.
* single binomial, the paper's setting: each pixel's facets reflecting the
  light are b(N_P, p) with p the light's reflection probability from the
  map; Eq. (oldgated) passes its gate with probability 1 - (1-p)^N >> N p
  when p is large and N < 1 and so overestimates the light's facets (mean
  count over N p well above 1), Eq. (gated) and the dual gate do not;
* whole multinomial (shading): the dual gate's glint radiance stays at the
  smooth value on average for every N; the single-gated node samplers of
  the tree overestimate it for N < 1.

Tiny probability (Fig. result_smallp): the light's reflection probability
gamma sweeps 1e-12 .. 1e-3 over the columns (the comparison method's
constant-probability mode, a narrow light seen off-specular) and N_P
1e3 .. 1e13 over the rows.
* single binomial: Eq. (oldgated)'s gate 1 - (1-gamma)^N is 0 in float for
  gamma < 2^-25 whatever N (banding that does not converge); with the bias
  Eq. (gated) and the dual gate give N gamma on average;
* tree (K = 2: the light is the node's right side, probability q = gamma):
  the printed dual gate evaluates P(n = N) = p^N with p = 1 - q, which float
  rounds to 1 for q < 2^-25, so no facet reaches the light; with the bias
  on both powers (GLINT_SAMPLER_DUAL_SYMMETRIC) the light's count converges
  to N gamma.
"""
import math

import numpy as np
import pytest

import oracle
import synth
from paper_2507_02674_amd import glint as G
from tests import gpu_util as U
from tests.test_modes_gpu import check_draws, check_pixels, gpu_draw, oracle_env

pytestmark = pytest.mark.gpu

DUAL, SINGLE, FLOOR, SYM = (G.GLINT_SAMPLER_DUAL, G.GLINT_SAMPLER_SINGLE, G.GLINT_SAMPLER_SINGLE_FLOOR,
                            G.GLINT_SAMPLER_DUAL_SYMMETRIC)


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU; the library has no CPU fallback")
    c = G.glint_create(0)
    yield c
    G.glint_destroy(c)


@pytest.fixture(scope="module")
def qtail(ctx):
    return U.quantile_table(ctx)


def wide_light_scene():
    """Sky 0.05, an area light of radius 25 degrees at the zenith whose
    luminance is the map's third radiance level (K = 4, so its facets form
    their own bin), a small bright sun near the horizon (the top level)."""
    L2 = math.exp(math.log(0.05) + 2.0 / 3.0 * (math.log(1e4) - math.log(0.05)))
    env = synth.disc_env(64, [(90.0, 0.0, 25.0, L2), (5.0, 180.0, 2.0, 1e4)], 0.05)
    Ns = np.concatenate([10.0 ** np.linspace(-1.52, 2.03, 15), [1.03e6]])
    W = 2048
    g = synth.sweep_plane(np.full(W, 90.0), Ns, alpha=0.05)
    return env, g, Ns, W


def test_wide_light_below_one_facet(ctx, qtail):
    R, K, M = 64, 4, 7
    U.log("wide light scene, N < 1")
    env, g, Ns, W = wide_light_scene()
    levels, ind, rgb = oracle_env(env, K, M)
    S, E = oracle.lut_tables()
    mean_g = {}
    for s in (DUAL, SYM, SINGLE, FLOOR):
        gpu = U.shade(ctx, g, ind, rgb, levels, S, E, R, K, M, seed=7, qtail=qtail, sampler=s)
        orc = oracle.shade(g, ind, rgb, levels, S, E, R, K, M, 7, 1, sampler=s)
        check_pixels(gpu, orc, f"wide light sampler {s}", max_flagged=0.25 if s == FLOOR else 5e-3)
        mean_g[s] = gpu["radiance"][:, 1].reshape(len(Ns), W).astype(np.float64).mean(1)
        probs = gpu["probs"]
    ref = mean_g[DUAL][-1]  # N = 1e6: the smooth value
    rel = {s: mean_g[s] / ref for s in mean_g}
    for i, N in enumerate(Ns):
        U.log(f"  N={N:9.3g}  mean glint radiance / smooth: dual {rel[DUAL][i]:.3f}  dual-sym {rel[SYM][i]:.3f}  "
              f"Eq.(gated) {rel[SINGLE][i]:.3f}  Eq.(oldgated) {rel[FLOOR][i]:.3f}")
    # the dual gates: unbiased on average at every N (statistical error of a
    # row: the glints of a row are ~N W p Poisson events)
    p_light = float(probs[0, 2])
    for i, N in enumerate(Ns[:-1]):
        tol = 5.0 / math.sqrt(max(N * W * p_light, 1.0)) + 0.03
        assert abs(rel[DUAL][i] - 1.0) < tol and abs(rel[SYM][i] - 1.0) < tol, (N, rel[DUAL][i], rel[SYM][i])
    # the tree's single-gated samplers overestimate below one facet
    low = Ns < 0.3
    assert np.all(rel[FLOOR][low] > 2.0) and np.all(rel[SINGLE][low] > 2.0)

    # the single binomial of the paper's figure: facets reflecting the area
    # light out of N_P, p = the light's probability from the map
    rng = np.random.default_rng(3)
    P = len(g["nx"])
    NP = np.repeat(Ns, W)
    p = probs[:, 2].astype(np.float64)
    h1 = rng.integers(0, 2 ** 32, P, dtype=np.uint32)
    h2 = rng.integers(0, 2 ** 32, P, dtype=np.uint32)
    for s, name in ((DUAL, "dual"), (SINGLE, "Eq.(gated)"), (FLOOR, "Eq.(oldgated)")):
        d = gpu_draw(ctx, s, NP, p, h1, h2, qtail)
        check_draws(d, oracle.sample_binomial(s, NP, p, h1, h2), f"wide light draws {name}", max_flagged=0.3)
        ratio = d["n"].reshape(len(Ns), W).mean(1) / (Ns * p_light)
        U.log(f"  single binomial {name}: mean n / (N p) for N = {Ns[0]:.3g}, {Ns[4]:.3g}, {Ns[8]:.3g}: "
              f"{ratio[0]:.3f}, {ratio[4]:.3f}, {ratio[8]:.3f}")
        # below one facet the dual gate's P(n = 1) = N p and Eq. (gated)'s
        # min(N p, .) are exact means (above, the dual gate's mean may sit
        # up to |1 - 2p| facets off, Alg. "Dual-gated Gaussian")
        tol = np.array([5.0 / math.sqrt(max(N * W * p_light, 1.0)) + 0.03 for N in Ns])
        if s == FLOOR:
            assert np.all(ratio[low] > 1.5), ratio
        else:
            assert np.all(np.abs(ratio[low] - 1.0) < tol[low]), ratio


def test_tiny_probability_banding(ctx, qtail):
    R, K, M = 32, 2, 6
    U.log("tiny reflection probability scene")
    env = synth.make_env(R, 5)
    levels, ind, rgb = oracle_env(env, 4, M)  # the two-bin mode reads only RGB and the LUTs
    S, E = oracle.lut_tables()
    gammas = 10.0 ** np.linspace(-12.0, -3.0, 37)
    Ns = 10.0 ** np.linspace(3.05, 13.05, 11)
    W = len(gammas)
    g = synth.sweep_plane(np.full(W, 60.0), Ns, alpha=0.1)
    NP = np.repeat(Ns, W)
    # shading in the two-bin mode, one call per column's gamma (the mode takes one gamma per call)
    counts = {DUAL: np.zeros((len(Ns), W)), SYM: np.zeros((len(Ns), W))}
    for c, gamma in enumerate(gammas):
        col = synth.subsample_gbuf(g, np.arange(c, len(g["nx"]), W))
        for s in (DUAL, SYM):
            gpu = U.shade(ctx, col, ind, rgb, levels, S, E, R, 4, M, seed=7, qtail=qtail, sampler=s,
                          prob_mode=G.GLINT_PROBS_CONSTANT, gamma=float(gamma))
            orc = oracle.shade(col, ind, rgb, levels, S, E, R, 4, M, 7, 1, sampler=s, prob_mode=1,
                               gamma=float(gamma))
            check_pixels(gpu, orc, f"gamma={gamma:.1e} sampler {s}", max_flagged=0.2)
            counts[s][:, c] = gpu["counts"][:, 0, 1]
    gf = np.array([float(np.float32(x)) for x in gammas])
    tiny = gf < 2.0 ** -25
    expect = 1.0 + (Ns[:, None] - 2.0) * gf[None, :]  # Gaussian branch mean of Alg. "Dual-gated Gaussian"
    U.log(f"  light facets, printed dual gate, gamma < 2^-25 and N gamma >= 20: "
          f"{counts[DUAL][:, tiny][(Ns[:, None] * gf[None, tiny]) >= 20].sum():.0f}")
    big = (Ns[:, None] * gf[None, :]) >= 20
    # banding: no light facet at all below 2^-25 with the printed gate ...
    assert np.all(counts[DUAL][:, tiny] == 0)
    # ... while above it the light gets its share, and the symmetric bias
    # gives the Gaussian branch's count everywhere N gamma is large
    sel = big & ~tiny[None, :]
    assert np.all(counts[DUAL][sel] > 0)
    selt = big & tiny[None, :]
    assert selt.sum() > 20
    r = counts[SYM][selt] / expect[selt]
    U.log(f"  symmetric bias, gamma < 2^-25: light count / (1 + (N-2) gamma): mean {r.mean():.3f}")
    assert abs(r.mean() - 1.0) < 0.1

    # the single binomial: the light's facets out of N, p = gamma
    rng = np.random.default_rng(5)
    Pn = len(Ns) * W
    p = np.tile(gf, len(Ns))
    h1 = rng.integers(0, 2 ** 32, Pn, dtype=np.uint32)
    h2 = rng.integers(0, 2 ** 32, Pn, dtype=np.uint32)
    n = {}
    for s in (DUAL, SINGLE, FLOOR):
        d = gpu_draw(ctx, s, NP, p, h1, h2, qtail)
        check_draws(d, oracle.sample_binomial(s, NP, p, h1, h2), f"tiny p draws sampler {s}", max_flagged=0.3)
        n[s] = d["n"].reshape(len(Ns), W)
    # Eq. (oldgated): no facet at all below 2^-25, whatever N
    assert np.all(n[FLOOR][:, tiny] == 0)
    for s in (DUAL, SINGLE):
        rr = n[s][selt] / (Ns[:, None] * gf[None, :])[selt]
        U.log(f"  single binomial sampler {s}, gamma < 2^-25: mean n / (N gamma) = {rr.mean():.3f}")
        assert abs(rr.mean() - 1.0) < 0.15
