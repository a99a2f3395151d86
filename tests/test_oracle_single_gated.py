"""Pins of the oracle's binomial approximations against what Sec. 6 and
App. B fix: the single-gated Gaussian of Eq. (gated) and its prior form
Eq. (oldgated), next to the dual-gated Gaussian of Alg. "Dual-gated
Gaussian".  Random words are stratified grids, so every probability below
is a deterministic fraction."""
import math

import numpy as np
import pytest

import oracle

DUAL, SINGLE, FLOOR = 0, 1, 2


def words(n):
    """n stratified 32-bit words whose mapped value ((h >> 9) + 1/2) 2^-23
    runs over a uniform grid of (0, 1)."""
    step = (1 << 23) // n
    j = np.arange(n, dtype=np.uint64) * step + step // 2
    return (j << np.uint64(9)).astype(np.uint32)


def grid2(n):
    h1, h2 = np.meshgrid(words(n), words(n), indexing="ij")
    return h1.ravel(), h2.ravel()


def draw(sampler, N, p, h1, h2):
    m = len(h1)
    return oracle.sample_binomial(sampler, np.full(m, float(N)), np.full(m, float(p)), h1, h2)


@pytest.mark.parametrize("N", [0.1, 0.5, 0.9, 1.5, 3.0, 10.0, 1000.0])
@pytest.mark.parametrize("p", [0.01, 0.2, 0.5, 0.9])
def test_single_gate_probability_is_min_of_Np_and_any_hit(N, p):
    """Eq. (gated) with App. B: the gate passes with probability N p for
    N < 1 and 1 - (1-p)^N for N > 1 (p above the bias threshold, so the
    power is unbiased)."""
    G = 1 << 16
    h1 = words(G)
    o = draw(SINGLE, N, p, h1, np.full(G, 1 << 31, np.uint32))
    hit = (o["code"] & 1).astype(bool)
    want = N * p if N < 1 else 1.0 - (1.0 - p) ** N
    assert abs(hit.mean() - want) <= 2.0 / G + 2e-6 * want


@pytest.mark.parametrize("N", [0.05, 0.3, 0.7, 0.999])
def test_single_gated_below_one_is_one_facet_or_none(N):
    """Gating generalisation: for N < 1 the count is exactly 1 (a single
    facet, inside the footprint and oriented) or 0; the mean is N p."""
    p = 0.6
    h1, h2 = grid2(256)
    o = draw(SINGLE, N, p, h1, h2)
    hit = (o["code"] & 1).astype(bool)
    assert set(np.unique(o["n"])) <= {0.0, 1.0}
    assert np.all(o["n"][hit] == 1.0) and np.all(o["n"][~hit] == 0.0)
    assert np.all(o["nb"][hit] == 0.0) and np.all(o["nb"][~hit] == N)
    assert not np.any(o["code"] & 16)
    assert abs(o["n"].mean() - N * p) <= 1.0 / 256 + 1e-6


def test_single_gated_gaussian_branch():
    """Past the gate and for N > 1: mean 1 + (N-1) p, variance (N-1) p (1-p)
    (no clamping at these N, p), counts in [1, N] and n + nbar = N."""
    N, p = 1e6, 0.3
    h1, h2 = grid2(1024)
    o = draw(SINGLE, N, p, h1, h2)
    hit = (o["code"] & 1).astype(bool)
    assert hit.all()  # (1-p)^N underflows
    assert np.all(o["code"] & 16)
    n = o["n"]
    mu, var = 1 + (N - 1) * p, (N - 1) * p * (1 - p)
    assert abs(n.mean() - mu) < 1e-3 * math.sqrt(var)
    assert abs(n.var() / var - 1) < 2e-2
    assert n.min() >= 1 and n.max() <= N
    np.testing.assert_allclose(n + o["nb"], N, rtol=1e-15)


def test_single_gated_clamps_to_range():
    """Small N: both Gaussian tails are clamped to [1, N]."""
    N, p = 3.0, 0.7
    h1, h2 = grid2(256)
    n = draw(SINGLE, N, p, h1, h2)["n"]
    assert n.min() == 0.0 and n.max() == N and np.any(n == 1.0)
    assert np.all((n == 0) | ((n >= 1) & (n <= N)))


def test_prior_form_overestimates_below_one():
    """Eq. (oldgated) gates with 1 - (1-p)^N, which exceeds N p for N < 1
    (App. B): the glint brightness is overestimated, the artefact the
    generalisation removes (Sec. 7 "Improved Single-Gated Gaussians")."""
    N, p = 0.5, 0.6
    G = 1 << 16
    h1 = words(G)
    h2 = np.full(G, 1 << 31, np.uint32)
    old = draw(FLOOR, N, p, h1, h2)["n"].mean()
    new = draw(SINGLE, N, p, h1, h2)["n"].mean()
    assert abs(new - N * p) <= 2.0 / G
    assert abs(old - (1 - (1 - p) ** N)) <= 2.0 / G + 1e-6
    assert old > new + 0.05


def test_prior_form_floors_counts():
    h1, h2 = grid2(128)
    n = draw(FLOOR, 37.5, 0.4, h1, h2)["n"]
    assert np.all(n == np.floor(n)) and n.max() <= 37


@pytest.mark.parametrize("Np", [0.1, 1.0, 10.0])
@pytest.mark.parametrize("p", [1e-9, 1e-12])
def test_bias_keeps_small_p_gate_alive(Np, p):
    """Sec. 6 "Numeric Gating Issues": in float, 1 - p rounds to 1 for
    p below ~6e-8, so the unbiased gate 1 - (1-p)^N never passes; with the
    bias the gate probability is ~1 - exp(-N p)."""
    N = Np / p
    G = 1 << 14
    h1 = words(G)
    h2 = np.full(G, 1 << 31, np.uint32)
    biased = (draw(SINGLE, N, p, h1, h2)["code"] & 1).mean()
    prior = (draw(FLOOR, N, p, h1, h2)["code"] & 1).mean()
    assert prior == 0.0
    assert abs(biased - (1 - math.exp(-Np))) < 2e-3


def wasserstein_to_binomial(n, N, p):
    from scipy.stats import binom
    u = (np.arange(len(n)) + 0.5) / len(n)
    return float(np.abs(np.sort(n) - binom.ppf(u, N, p)).mean())


@pytest.mark.parametrize("N", [2, 3, 4, 5, 8])
def test_dual_gated_is_closer_to_the_binomial_for_small_N(N):
    """Fig. "gatingplot": for small N the dual-gated Gaussian is closer to
    b(N, p) than the single-gated one (Wasserstein-1 distance of the
    distributions over a stratified grid of both random numbers)."""
    h1, h2 = grid2(128)
    for p in (0.05, 0.1, 0.3, 0.5, 0.7, 0.9):
        dual = wasserstein_to_binomial(draw(DUAL, N, p, h1, h2)["n"], N, p)
        single = wasserstein_to_binomial(draw(SINGLE, N, p, h1, h2)["n"], N, p)
        assert dual < single, (N, p, dual, single)


@pytest.mark.parametrize("N", [2.0, 3.0, 5.0, 12.0])
def test_dual_gated_symmetric_single_gated_not(N):
    """Fig. "gatingplot": the dual-gated draw is symmetric (the positive
    count at p is distributed as the negative count at 1-p), the single-gated
    one is not."""
    h1, h2 = grid2(128)
    p = 0.3
    a = draw(DUAL, N, p, h1, h2)
    b = draw(DUAL, N, 1 - p, h1, h2)
    assert np.abs(np.sort(a["n"]) - np.sort(b["nb"])).mean() < 1e-3 * N
    a = draw(SINGLE, N, p, h1, h2)
    b = draw(SINGLE, N, 1 - p, h1, h2)
    assert np.abs(np.sort(a["n"]) - np.sort(b["nb"])).mean() > 0.05


def test_all_samplers_agree_for_large_N():
    """Sec. 7 "Dual-Gated Gaussians": for large N the approximations
    coincide (relative difference of the means and spreads)."""
    N, p = 1e5, 0.4
    h1, h2 = grid2(256)
    ms = [draw(s, N, p, h1, h2)["n"] for s in (DUAL, SINGLE, FLOOR)]
    for m in ms[1:]:
        assert abs(m.mean() - ms[0].mean()) / (N * p) < 1e-4
        assert abs(m.std() / ms[0].std() - 1) < 1e-2


def test_shade_single_gated_conserves_counts():
    """The multinomial tree with the single gate: each node splits N into n
    and N - n, except that a passed gate at N < 1 yields one facet (excess
    below 1 per node), so the leaf counts sum to N_P up to K - 1."""
    import synth
    R, K, M = 16, 8, 5
    env = synth.make_env(R, 6)
    levels, ij, it = oracle.partition(env, K)
    chain = oracle.mipchain(env, ij, it, K, M)
    ind, rgb = oracle.split_pyramid(oracle.prefilter(env, ij, it, chain, K, M, 64), K)
    S, E = oracle.lut_tables()
    g = synth.scene_frame(96, 54, seed=3, density_decades=(2.0, 9.0))
    hit = np.nonzero(g["surf_id"] != synth.NO_SURFACE)[0][::5]
    out = oracle.shade(g, ind, rgb, levels, S, E, R, K, M, 5, 1, pixels=hit, sampler=SINGLE)
    NP = g["density"][hit].astype(np.float64) * g["area"][hit]
    tot = out["counts"][:, 0].sum(axis=1)
    assert np.all(tot >= NP * (1 - 1e-12)) and np.all(tot <= NP * (1 + 1e-12) + (K - 1))
    big = NP > 1e4
    assert big.sum() > 100
    # the sampler changes the counts, not the probabilities
    dual = oracle.shade(g, ind, rgb, levels, S, E, R, K, M, 5, 1, pixels=hit)
    np.testing.assert_array_equal(out["probs"], dual["probs"])
    assert not np.array_equal(out["counts"], dual["counts"])
    floor = oracle.shade(g, ind, rgb, levels, S, E, R, K, M, 5, 1, pixels=hit, sampler=FLOOR)
    assert np.all(floor["counts"][:, 0] >= 0)
