"""Pins of the oracle's two changes to the reflection probabilities:
occlusion that attenuates the probabilities instead of the output (Sec. 8
"Limitations & Future Work"), and the map-independent constant probability
of the comparison method (Sec. 7 "Comparison with Previous Work")."""
import numpy as np
import pytest

import oracle
import synth

R, K, M = 16, 8, 5


@pytest.fixture(scope="module")
def setup():
    env = synth.make_env(R, 6)
    levels, ij, it = oracle.partition(env, K)
    chain = oracle.mipchain(env, ij, it, K, M)
    ind, rgb = oracle.split_pyramid(oracle.prefilter(env, ij, it, chain, K, M, 64), K)
    S, E = oracle.lut_tables()
    g = synth.scene_frame(128, 72, seed=3, density_decades=(2.0, 7.0))
    hit = np.nonzero(g["surf_id"] != synth.NO_SURFACE)[0]
    return dict(env=env, levels=levels, ind=ind, rgb=rgb, S=S, E=E, g=g, hit=hit)


def run(s, g, **kw):
    return oracle.shade(g, s["ind"], s["rgb"], s["levels"], s["S"], s["E"], R, K, M, 9, 1, pixels=s["hit"], **kw)


def with_vis(g, v):
    h = dict(g)
    h["visibility"] = np.broadcast_to(np.float32(v), g["nx"].shape).copy() if np.isscalar(v) else v
    return h


def test_full_visibility_is_the_unoccluded_path(setup):
    a = run(setup, setup["g"])
    b = run(setup, with_vis(setup["g"], 1.0))
    for k in ("radiance", "counts", "codes", "probs", "flags"):
        assert np.array_equal(a[k], b[k]), k


def test_zero_visibility_reflects_nothing(setup):
    out = run(setup, with_vis(setup["g"], 0.0))
    assert np.all(out["radiance"] == 0)
    NP = setup["g"]["density"][setup["hit"]].astype(np.float64) * setup["g"]["area"][setup["hit"]]
    big = NP > 2  # below 2 facets the dual gate dithers the count to an integer
    np.testing.assert_allclose(out["counts"][big, 0, 0], NP[big], rtol=1e-12)
    assert np.all(out["counts"][:, 0, 1:] == 0)
    np.testing.assert_array_equal(out["probs"][:, 0], 1.0)


def test_visibility_scales_probabilities_and_expected_radiance(setup):
    """p'_k = v p_k for k >= 1 and the frame's radiance scales by ~v (the
    normalisation keeps the unattenuated probabilities)."""
    a = run(setup, setup["g"])
    b = run(setup, with_vis(setup["g"], 0.5))
    np.testing.assert_allclose(b["probs"][:, 1:], 0.5 * a["probs"][:, 1:], rtol=1e-15)
    np.testing.assert_allclose(b["probs"].sum(1), 1.0, rtol=1e-12)
    ratio = b["radiance"].sum() / a["radiance"].sum()
    assert abs(ratio - 0.5) < 0.03, ratio


def test_occlusion_is_not_an_output_multiplier(setup):
    """Attenuated probabilities change how many facets glint, not how bright
    a glint is: where a pixel holds less than one facet, occlusion v = 1/4
    makes ~4x fewer pixels glint while the glints that remain keep their
    radiance (an output multiplier would dim every glint instead)."""
    g = synth.scene_frame(256, 144, seed=3, density_decades=(1.0, 3.0))
    hit = np.nonzero(g["surf_id"] != synth.NO_SURFACE)[0]
    s = dict(setup, hit=hit)
    a = run(s, g)["radiance"].sum(1)
    b = run(s, with_vis(g, 0.25))["radiance"].sum(1)
    assert not np.allclose(b, 0.25 * a, rtol=1e-3)
    NP = g["density"][hit].astype(np.float64) * g["area"][hit]
    sparse = NP < 1
    assert sparse.sum() > 10000
    la, lb = a[sparse] > 0, b[sparse] > 0
    assert abs(lb.mean() / la.mean() - 0.25) < 0.05
    assert abs(np.median(b[sparse][lb]) / np.median(a[sparse][la]) - 1) < 0.2


def test_constant_probability_layout_and_counts(setup):
    gamma = 0.05
    out = run(setup, setup["g"], prob_mode=1, gamma=gamma)
    g32 = float(np.float32(gamma))
    assert out["counts"].shape[2] == 2 and out["probs"].shape[1] == 2
    np.testing.assert_array_equal(out["probs"][:, 1], g32)
    np.testing.assert_array_equal(out["probs"][:, 0], 1.0 - g32)
    NP = setup["g"]["density"][setup["hit"]].astype(np.float64) * setup["g"]["area"][setup["hit"]]
    big = NP > 2
    np.testing.assert_allclose(out["counts"][big, 0].sum(1), NP[big], rtol=1e-12)
    # E[M_1] ~ N gamma (the gated Gaussians' small-N bias aside: a ratio of
    # sums, dominated by the large counts)
    m = out["counts"][big, 0, 1].sum() / (NP[big].sum() * g32)
    assert abs(m - 1) < 0.02, m


def test_constant_probability_is_independent_of_the_map(setup):
    """The comparison method's glints do not depend on the map: counts are
    identical for two different maps, and the output is the smooth radiance
    times the same factor."""
    s2 = dict(setup)
    env2 = synth.make_env(R, 11)
    levels, ij, it = oracle.partition(env2, K)
    chain = oracle.mipchain(env2, ij, it, K, M)
    s2["ind"], s2["rgb"] = oracle.split_pyramid(oracle.prefilter(env2, ij, it, chain, K, M, 64), K)
    a = run(setup, setup["g"], prob_mode=1, gamma=0.1)
    b = run(s2, setup["g"], prob_mode=1, gamma=0.1)
    assert np.array_equal(a["counts"], b["counts"]) and np.array_equal(a["codes"], b["codes"])
    # the factor radiance / smooth radiance is the same on both maps
    sm_a = run(setup, setup["g"], prob_mode=1, gamma=1.0)["radiance"]
    sm_b = run(s2, setup["g"], prob_mode=1, gamma=1.0)["radiance"]
    ok = (sm_a.sum(1) > 1e-6) & (sm_b.sum(1) > 1e-6)
    np.testing.assert_allclose(a["radiance"][ok] / sm_a[ok], b["radiance"][ok] / sm_b[ok], rtol=1e-9, atol=1e-12)


def test_constant_probability_one_is_the_smooth_radiance(setup):
    """gamma = 1: every facet reflects, the count is N_P and the output is
    the smooth BRDF's radiance L_o = E_rho RGB."""
    out = run(setup, setup["g"], prob_mode=1, gamma=1.0)
    NP = setup["g"]["density"][setup["hit"]].astype(np.float64) * setup["g"]["area"][setup["hit"]]
    big = NP > 2
    np.testing.assert_allclose(out["counts"][big, 0, 1], NP[big], rtol=1e-15)
    # the map's glints average to the smooth radiance over the frame (counts
    # are unbiased draws of N_P p_k)
    env_mode = run(setup, setup["g"])
    ratio = env_mode["radiance"][big].sum() / out["radiance"][big].sum()
    assert abs(ratio - 1) < 0.05, ratio


def test_invalid_modes_rejected(setup):
    with pytest.raises(ValueError):
        run(setup, setup["g"], prob_mode=1, gamma=0.0)
    with pytest.raises(ValueError):
        run(setup, setup["g"], prob_mode=2)
