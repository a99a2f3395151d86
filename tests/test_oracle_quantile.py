"""Pins of the quantile radiance levels (level_mode 1): the configuration's
"K regions by radiance quantiles", next to the paper's log-lerp levels of
Sec. 5 "Discrete Radiance Levels".  Level k (1 <= k <= K-2) is the smallest
texel luminance whose solid-angle-weighted distribution function reaches
q = k/(K-1); L(0) = 0 and L(K-1) = max.

Pinned by the definition checked against independent numpy sums over the
exact texel solid angles, by a closed form (faces of constant luminance:
the distribution is a staircase of steps 1/6) and by Archimedes' hat-box
theorem (the height of a uniformly distributed direction is uniform on
[-1, 1], so a map whose luminance is affine in the height has affine
quantiles); a quantile by texel count instead of solid angle fails it.
"""
import math

import numpy as np
import pytest

import oracle
import synth
from oracle import definitions as defs
from tests.test_oracle_env import luminance_np


def weighted_cdf(Y, om, y):
    return om[Y <= y].sum()


@pytest.mark.parametrize("K", [3, 4, 8, 16])
@pytest.mark.parametrize("seed", [1, 2, 7])
def test_quantile_levels_are_the_smallest_values_reaching_q(K, seed):
    R = 32
    env = synth.make_env(R, seed)
    levels, margin = oracle.quantile_levels(env, K)
    lv, _, _ = oracle.partition(env, K, 1e-3, level_mode=1)
    assert np.array_equal(levels, lv)
    Y = luminance_np(env).reshape(-1)
    om = defs.texel_solid_angles(R).reshape(-1)
    W = om.sum()
    assert W == pytest.approx(4 * math.pi, rel=1e-12)
    vals = np.unique(Y)
    assert levels[0] == 0.0 and levels[-1] == Y.max()
    assert np.all(np.diff(levels) >= 0)
    for k in range(1, K - 1):
        q = k / (K - 1)
        L = levels[k]
        assert L in vals  # a texel's own luminance (no clip is active on these maps)
        assert weighted_cdf(Y, om, L) >= q * W * (1 - 1e-12)
        below = vals[vals < L]
        if below.size:
            assert weighted_cdf(Y, om, below[-1]) < q * W
        assert margin[k] > 0


def test_quantile_levels_constant_faces_closed_form():
    """Each face at its own constant luminance: C is a staircase of steps
    1/6, so level k is the ceil(6k/(K-1))-th smallest face value (K = 8:
    6k/7 is never an integer, no tie with a step)."""
    R, K = 16, 8
    face_y = np.array([3.0, 0.5, 7.0, 1.5, 12.0, 0.25])
    env = np.empty((6, R, R, 3), np.float32)
    for f in range(6):
        env[f] = face_y[f]  # grey: luminance = value (coefficients sum to 1)
    levels, margin = oracle.quantile_levels(env, K)
    srt = np.sort(face_y)
    for k in range(1, K - 1):
        assert levels[k] == pytest.approx(srt[math.ceil(6 * k / (K - 1)) - 1], rel=1e-6), k
        assert margin[k] > 0.01
    assert levels[-1] == pytest.approx(12.0, rel=1e-6)


def test_quantile_levels_archimedes():
    """Luminance 2 + y (y the height of the texel direction): the height of
    a direction uniform on the sphere is uniform on [-1, 1], so the
    solid-angle quantile at q is 2 + (2q - 1), up to the texel resolution.
    A quantile by texel count is far off (the cube's texels crowd towards
    the face corners)."""
    R, K = 128, 8
    d = defs.face_dirs(R)
    Y = 2.0 + d[..., 1]
    env = np.repeat(Y[..., None], 3, axis=-1).astype(np.float32)
    levels, _ = oracle.quantile_levels(env, K)
    for k in range(1, K - 1):
        q = k / (K - 1)
        assert abs(levels[k] - (2.0 + 2 * q - 1)) < 0.02, (k, levels[k])
    # the count quantile differs measurably somewhere: the weighting matters
    Yf = np.sort(luminance_np(env).reshape(-1))
    count_q = [Yf[math.ceil(k / (K - 1) * Yf.size) - 1] for k in range(1, K - 1)]
    assert max(abs(c - (2.0 + 2 * (k + 1) / (K - 1) - 1)) for k, c in enumerate(count_q)) > 0.03


def test_quantile_levels_degenerate_maps():
    K = 4
    lv, ind_j, ind_t = oracle.partition(synth.uniform_env(8, 2.0), K, 1e-3, level_mode=1)
    assert np.all(lv[1:] == pytest.approx(2.0, rel=1e-15))
    assert np.all(ind_j == K - 2) and np.all(ind_t == 1.0)
    # everything below ell: levels clipped to ell
    lv, _, _ = oracle.partition(synth.uniform_env(8, 1e-6), K, 1e-3, level_mode=1)
    assert np.all(lv[1:] == 1e-3)
    # one face: R = 1 (six texels of equal solid angle)
    env = np.arange(1, 19, dtype=np.float32).reshape(6, 1, 1, 3)
    lv, margin = oracle.quantile_levels(env, 8)
    Y = np.sort(luminance_np(env).reshape(-1))
    for k in range(1, 7):
        assert lv[k] == Y[math.ceil(6 * k / 7) - 1]


@pytest.mark.parametrize("K", [4, 8])
def test_quantile_indicators_reconstruct_luminance(K):
    env = synth.make_env(32, 4)
    levels, ind_j, ind_t = oracle.partition(env, K, 1e-3, level_mode=1)
    Y = np.minimum(luminance_np(env), levels[-1])
    w = defs.dense_level0(ind_j, ind_t, env, K)[..., :K]
    assert np.abs(w.sum(-1) - 1.0).max() == 0.0
    j = ind_j.astype(int)
    lo, hi = levels[j], levels[j + 1]
    assert np.all((lo <= Y) & (Y <= hi))
    t = ind_t.astype(np.float64)
    rec = (1 - t) * lo + t * hi
    assert np.all(np.abs(rec - Y) <= 2 ** -23 * hi + 1e-300)
