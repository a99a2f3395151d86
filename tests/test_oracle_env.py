"""Pins of the oracle's per-frame environment steps (Sec. 5) and lookup tables.

Partition: closed forms and invariants of the radiance levels and fuzzy
indicators.  Filter: partition of unity, uniform environment, identity at mip
0, brute-force kernel sum.  LUTs: closed-form D_H, direct integrals over
incident directions, mirror limit.
"""
import math

import numpy as np
import pytest

import oracle
import synth
from oracle import definitions as defs


def luminance_np(env):
    e = env.astype(np.float64)
    e = np.where(np.isfinite(e) & (e > 0), e, 0.0)
    return 0.2126 * e[..., 0] + 0.7152 * e[..., 1] + 0.0722 * e[..., 2]


@pytest.mark.parametrize("K", [2, 4, 8, 16])
def test_levels_closed_form(K):
    env = synth.make_env(32, 3)
    ell = 1e-3
    levels, ind_j, ind_t = oracle.partition(env, K, ell)
    Y = luminance_np(env)
    assert levels[0] == 0.0
    assert levels[-1] == Y.max()  # top level is the maximum radiance exactly
    assert np.all(np.diff(levels) > 0)
    if K > 2:
        # log-linear spacing: constant ratio between consecutive non-zero levels,
        # whose product telescopes to max / min
        ratios = levels[2:] / levels[1:-1]
        assert np.allclose(ratios, ratios[0], rtol=1e-12)
        lmin = max(Y.min(), ell)
        assert ratios[0] ** (K - 1) == pytest.approx(Y.max() / lmin, rel=1e-10)
        assert levels[1] == pytest.approx(lmin * ratios[0], rel=1e-12)


@pytest.mark.parametrize("K", [4, 8])
@pytest.mark.parametrize("weight_space", [0, 1])
def test_indicators_partition_of_unity_and_reconstruction(K, weight_space):
    env = synth.make_env(32, 5)
    levels, ind_j, ind_t = oracle.partition(env, K, 1e-3, weight_space=weight_space)
    Y = np.minimum(luminance_np(env), levels[-1])
    w = defs.dense_level0(ind_j, ind_t, env, K)[..., :K]
    assert np.all(w >= 0)
    assert np.abs(w.sum(-1) - 1.0).max() == 0.0
    j = ind_j.astype(int)
    lo, hi = levels[j], levels[j + 1]
    assert np.all((lo <= Y) & (Y <= hi))
    t = ind_t.astype(np.float64)
    if weight_space == 0:
        # Eq. (wkdefpractice): L_i = lerp(L(j), L(j+1), w(j+1)) (float-stored t)
        rec = (1 - t) * lo + t * hi
        assert np.all(np.abs(rec - Y) <= 2 ** -23 * hi + 1e-300)
    else:
        sel = j >= 1
        rec = np.exp((1 - t[sel]) * np.log(lo[sel]) + t[sel] * np.log(hi[sel]))
        assert np.all(np.abs(rec - Y[sel]) <= 1e-6 * hi[sel])


def test_partition_degenerate_inputs():
    R, K = 8, 4
    # uniform environment: every level above 0 equals the radiance; all weight
    # on the top level
    env = synth.uniform_env(R, 2.0)
    levels, ind_j, ind_t = oracle.partition(env, K, 1e-3)
    assert np.all(levels[1:] == pytest.approx(2.0, rel=1e-15))
    assert np.all(ind_j == K - 2) and np.all(ind_t == 1.0)
    # negative, NaN and Inf channels count as zero radiance
    env = synth.make_env(R, 1)
    env[0, 0, 0] = [-5.0, np.nan, np.inf]
    levels, ind_j, ind_t = oracle.partition(env, K, 1e-3)
    assert ind_j[0, 0, 0] == 0 and ind_t[0, 0, 0] == 0.0
    assert np.isfinite(levels).all()
    # everything below ell: clipped minimum, defined levels
    env = synth.uniform_env(R, 1e-6)
    levels, ind_j, ind_t = oracle.partition(env, K, 1e-3)
    assert np.all(levels[1:] == pytest.approx(1e-3))
    assert np.all(ind_j == 0)


def test_cube_conventions_round_trip():
    rng = np.random.default_rng(0)
    for _ in range(500):
        d = rng.normal(size=3)
        f, s, t = oracle.dir_face(d)
        back = oracle.face_dir(f, s, t)
        assert np.allclose(back / np.linalg.norm(back), d / np.linalg.norm(d), atol=1e-14)
        assert -1.0 <= s <= 1.0 and -1.0 <= t <= 1.0
    axes = [(1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)]
    for f, a in enumerate(axes):
        assert oracle.dir_face(np.array(a, float))[0] == f


def test_mipchain_is_mean_of_children():
    env = synth.make_env(16, 2)
    K, M = 4, 5
    levels, ind_j, ind_t = oracle.partition(env, K)
    chain = oracle.mipchain(env, ind_j, ind_t, K, M)
    lev = defs.dense_level0(ind_j, ind_t, env, K)
    off = 0
    for s in range(1, M):
        n = 16 >> s
        got = chain[off:off + 6 * n * n].reshape(6, n, n, K + 3).astype(np.float64)
        off += 6 * n * n
        want = lev.reshape(6, n, 2, n, 2, K + 3).mean(axis=(2, 4))
        assert np.abs(got - want).max() <= 2 ** -23 * (np.abs(want).max() + 1)
        lev = got
    # the coarsest level averages the whole face: equals the face mean of level 0
    top = chain[-6:].astype(np.float64).reshape(6, K + 3)
    full = defs.dense_level0(ind_j, ind_t, env, K).mean(axis=(1, 2))
    assert np.allclose(top, full, rtol=1e-5, atol=1e-7)


def _frame_pyramid(R, K, M, T, seed=1, env=None):
    env = synth.make_env(R, seed) if env is None else env
    levels, ind_j, ind_t = oracle.partition(env, K)
    chain = oracle.mipchain(env, ind_j, ind_t, K, M)
    pyr = oracle.prefilter(env, ind_j, ind_t, chain, K, M, T)
    return env, ind_j, ind_t, chain, pyr


def test_uniform_environment_filters_to_one():
    R, K, M = 16, 4, 5
    env = synth.uniform_env(R, 3.0)
    _, ind_j, ind_t, chain, pyr = _frame_pyramid(R, K, M, 64, env=env)
    assert np.all(pyr[:, K - 1] == 1.0)
    assert np.all(pyr[:, :K - 1] == 0.0)
    assert np.allclose(pyr[:, K:], 3.0, rtol=1e-15)


def test_filter_partition_of_unity_and_identity_mip0():
    R, K, M = 32, 4, 6
    env, ind_j, ind_t, chain, pyr = _frame_pyramid(R, K, M, 64)
    assert np.abs(pyr[:, :K].sum(1) - 1).max() < 1e-6
    assert np.all(pyr[:, :K] >= 0)
    n0 = 6 * R * R
    dense = defs.dense_level0(ind_j, ind_t, env, K).reshape(n0, K + 3)
    assert np.array_equal(pyr[:n0], dense)


def test_filter_against_brute_force_kernel_sum():
    """The quadrature approximates the kernel integral; the error against the
    direct sum over all texels (parity unpinned: the paper gives no number) must
    shrink as the tap count grows."""
    R, K, M = 32, 4, 6
    env = synth.make_env(R, 1)
    levels, ind_j, ind_t = oracle.partition(env, K)
    chain = oracle.mipchain(env, ind_j, ind_t, K, M)
    dense = defs.dense_level0(ind_j, ind_t, env, K)
    rng = np.random.default_rng(3)
    errs = {}
    for T in (16, 64, 256):
        e = []
        for m in (2, 3, 4):
            n = R >> m
            base = oracle.level_offset(R, m)
            ids = base + rng.choice(6 * n * n, 6, replace=False)
            got = oracle.prefilter(env, ind_j, ind_t, chain, K, M, T, texel_ids=ids)
            alpha = (m / (M - 1)) ** 2
            for q, tid in enumerate(ids):
                rem = tid - base
                f, y, x = rem // (n * n), (rem // n) % n, rem % n
                r = oracle.face_dir(int(f), 2 * (x + 0.5) / n - 1, 2 * (y + 0.5) / n - 1)
                want = defs.brute_force_filter(dense, r, alpha)
                e.append(np.abs(got[q, :K] - want[:K]).max())
        errs[T] = float(np.mean(e))
    assert errs[256] < errs[16]
    assert errs[64] < 0.08, errs


def test_tap_table_matches_ggx_importance_sampling():
    """Tap half vectors follow D(h) cos(h): the GGX inverse CDF; tap weights
    <r,l>+ = 2 cos^2 - 1; the lod follows filtered importance sampling with
    pdf_l = D/4 (n = v = r)."""
    R, M, T = 256, 8, 64
    for m in (1, 4, 7):
        alpha = (m / (M - 1)) ** 2
        taps = oracle.taps(m, M, T, R)
        h = taps[:, :3]
        assert np.allclose(np.linalg.norm(h, axis=1), 1.0, atol=1e-14)
        assert np.allclose(taps[:, 3], np.maximum(0, 2 * h[:, 2] ** 2 - 1), atol=1e-14)
        # normalisation of the NDF used for the lod: integral of D cos = 1
        from scipy import integrate
        val, _ = integrate.quad(lambda th: float(defs.ggx_D(np.array(math.cos(th)), alpha)) * math.cos(th)
                                * math.sin(th) * 2 * math.pi, 0, math.pi / 2, limit=200, points=[alpha])
        assert val == pytest.approx(1.0, rel=1e-7)
        D = defs.ggx_D(h[:, 2], alpha)
        lod = np.clip(0.5 * np.log2((4.0 / (T * D)) / (4 * math.pi / (6 * R * R))) + 1, 0, M - 1)
        assert np.allclose(taps[:, 4], lod, atol=1e-12)
        # empirical CDF of the taps' cos^2 against the GGX CDF of D cos
        c2 = np.sort(h[:, 2] ** 2)
        a2 = alpha * alpha
        u = np.array([(1 - c) / (1 + (a2 - 1) * c) for c in c2])  # fraction of mass with larger cos
        ks = np.max(np.abs(np.sort(1 - u) - (np.arange(T) + 0.5) / T))
        assert ks < 1.5 / T


def test_total_facet_area_closed_form():
    from scipy import integrate
    for alpha in (0.02, 0.1, 0.3, 0.7, 1.0):
        val, _ = integrate.quad(lambda th: float(defs.ggx_D(np.array(math.cos(th)), alpha)) * math.sin(th)
                                * 2 * math.pi, 0, math.pi / 2, limit=400, points=[alpha])
        assert defs.total_facet_area(alpha) == pytest.approx(val, rel=1e-8)
        assert defs.total_facet_area(alpha) >= 1.0


@pytest.mark.parametrize("ia,im", [(10, 63), (20, 40), (20, 6), (40, 30), (50, 60), (63, 10)])
def test_lut_against_direct_integrals(ia, im):
    S, A, B = oracle.luts(np.array([ia * 64 + im]))
    mu = (im + 0.5) / 64
    alpha = ((ia + 0.5) / 64) ** 2
    ED = defs.visible_facet_area(mu, alpha)
    assert S[0] == pytest.approx(ED / defs.total_facet_area(alpha), abs=2e-4)
    a_ref, b_ref = defs.split_sum_albedo(mu, alpha)
    assert A[0] == pytest.approx(a_ref, abs=2e-4)
    assert B[0] == pytest.approx(b_ref, abs=2e-4)


def test_lut_limits():
    S, A, B = oracle.luts()
    S = S.reshape(64, 64)
    A = A.reshape(64, 64)
    B = B.reshape(64, 64)
    assert np.all(S <= 1.0 + 1e-12) and np.all(S > 0)
    # smooth limit at normal incidence: every facet reflects upward
    assert S[0, 63] > 0.9999
    # mirror limit (alpha -> 0): E_rho -> Schlick F(mu) with G2 -> 1
    mu = (np.arange(64) + 0.5) / 64
    fc = (1 - mu) ** 5
    assert np.allclose(A[0, 16:], 1 - fc[16:], atol=2e-3)
    assert np.allclose(B[0, 16:], fc[16:], atol=2e-3)
    # roughness reduces the visible reflecting area
    assert np.all(np.diff(S[:, 40]) <= 1e-9)


@pytest.mark.parametrize("R,M", [(4, 3), (16, 5)])
def test_lookup_continuous_across_edges_and_corners(R, M):
    """A seamless cube lookup is a continuous function of direction: on face
    edges (|x| = |y| etc.) and at cube corners a tiny perturbation of the
    direction may change the owning face but not the value."""
    rng = np.random.default_rng(5)
    n_tex = oracle.pyramid_texels(R, M)
    pyr = rng.random((n_tex, 3)).astype(np.float32)
    dirs = []
    for _ in range(300):
        a, b = rng.uniform(0.2, 1.0, 2)
        sx, sy, sz = rng.choice([-1.0, 1.0], 3)
        kind = rng.integers(4)
        if kind == 0:
            d = np.array([sx * a, sy * a, sz * b * a])      # |x| = |y|
        elif kind == 1:
            d = np.array([sx * a, sy * b * a, sz * a])      # |x| = |z|
        elif kind == 2:
            d = np.array([sx * b * a, sy * a, sz * a])      # |y| = |z|
        else:
            d = np.array([sx, sy, sz]) * a                 # cube corner
        dirs.append(d)
    dirs = np.array(dirs)
    for lod in (0.0, 0.5, float(M - 1)):
        base = oracle.pyramid_lookup(pyr, R, M, dirs, lod)
        for eps in (1e-12, -1e-12):
            for axis in range(3):
                p = dirs.copy()
                p[:, axis] *= 1 + eps
                got = oracle.pyramid_lookup(pyr, R, M, p, lod)
                assert np.abs(got - base).max() < 1e-9


def test_lookup_interpolates_texel_centres():
    """At a texel centre of level s the lookup returns that texel exactly."""
    R, M = 8, 4
    rng = np.random.default_rng(6)
    pyr = rng.random((oracle.pyramid_texels(R, M), 2)).astype(np.float32)
    for s in range(M):
        n = R >> s
        for f in range(6):
            for (x, y) in ((0, 0), (n - 1, 0), (n // 2, n - 1)):
                d = oracle.face_dir(f, 2 * (x + 0.5) / n - 1, 2 * (y + 0.5) / n - 1)
                got = oracle.pyramid_lookup(pyr, R, M, d[None], float(s))[0]
                want = pyr[oracle.level_offset(R, s) + (f * n + y) * n + x]
                assert np.allclose(got, want, atol=1e-7)
