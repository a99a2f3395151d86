"""Pins of the surrogate's FP64 definition (oracle/mlp.py): finite-difference
gradients, softmax/cross-entropy identities, layout round trip, Adam."""
import numpy as np
import pytest

from oracle import mlp


def test_layout_and_parameter_count():
    assert mlp.real_params(8) == 9224
    rng = np.random.default_rng(0)
    w = rng.normal(size=mlp.N_PARAMS)
    p = mlp.unpack(w, 8)
    back = mlp.pack(p, 8)
    keep = back != 0
    assert np.array_equal(back[keep], w[keep])
    assert np.count_nonzero(back) == mlp.real_params(8)


@pytest.mark.parametrize("K", [4, 8])
def test_radiance_weighted_loss_gradient_matches_finite_differences(K):
    """The loss with the radiance-weighted term: its gradient against central
    differences of the loss itself; a sample whose target reflects nothing
    above level 0 contributes only the plain term."""
    rng = np.random.default_rng(7)
    w = mlp.init(K, seed=8).astype(np.float64)
    w += rng.normal(scale=0.05, size=w.shape) * (mlp.pack(mlp.unpack(np.ones(mlp.N_PARAMS), K), K) != 0)
    x = rng.normal(size=(12, 5))
    t = rng.dirichlet(np.ones(K), size=12)
    t[3] = 0.0
    t[3, 0] = 1.0
    levels = np.concatenate([[0.0], np.sort(10.0 ** rng.uniform(-2, 3, K - 1))])
    lam = 0.7
    loss, g = mlp.loss_and_grad(w, x, t, K, levels=levels, lam=lam)
    idx = np.nonzero(g)[0]
    pick = rng.choice(idx, 60, replace=False)
    h = 1e-6
    for i in pick:
        wp, wm = w.copy(), w.copy()
        wp[i] += h
        wm[i] -= h
        fd = (mlp.loss_and_grad(wp, x, t, K, levels=levels, lam=lam)[0] -
              mlp.loss_and_grad(wm, x, t, K, levels=levels, lam=lam)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])
    # the term is the cross-entropy of the L-weighted distributions: zero
    # gradient contribution when the network matches the target exactly
    y, _ = mlp.forward(w, x, K)
    _, g_self = mlp.loss_and_grad(w, x, y, K, levels=levels, lam=lam)
    assert np.abs(g_self).max() < 1e-12
    base, _ = mlp.loss_and_grad(w, x, t, K)
    yp, tp, ok = mlp.radiance_weighted(y, t, levels)
    assert not ok[3] and ok.sum() == 11
    assert loss == pytest.approx(base - lam * np.sum(tp[ok] * np.log(yp[ok])) / 12, rel=1e-12)


@pytest.mark.parametrize("K", [4, 8])
def test_gradient_matches_finite_differences(K):
    rng = np.random.default_rng(1)
    w = mlp.init(K, seed=3).astype(np.float64)
    w += rng.normal(scale=0.05, size=w.shape) * (mlp.pack(mlp.unpack(np.ones(mlp.N_PARAMS), K), K) != 0)
    x = rng.normal(size=(16, 5))
    t = rng.dirichlet(np.ones(K), size=16)
    loss, g = mlp.loss_and_grad(w, x, t, K)
    idx = np.nonzero(g)[0]
    pick = rng.choice(idx, 60, replace=False)
    h = 1e-6
    for i in pick:
        wp, wm = w.copy(), w.copy()
        wp[i] += h
        wm[i] -= h
        fd = (mlp.loss_and_grad(wp, x, t, K)[0] - mlp.loss_and_grad(wm, x, t, K)[0]) / (2 * h)
        assert fd == pytest.approx(g[i], rel=1e-5, abs=1e-9)


def test_softmax_cross_entropy_identities():
    K = 8
    rng = np.random.default_rng(2)
    w = mlp.init(K).astype(np.float64)
    x = rng.normal(size=(32, 5))
    y, _ = mlp.forward(w, x, K)
    assert np.allclose(y.sum(1), 1.0) and np.all(y > 0)
    # cross-entropy against its own output is the entropy; the gradient of the
    # logits vanishes there
    loss, g = mlp.loss_and_grad(w, x, y, K)
    assert loss == pytest.approx(-np.mean(np.sum(y * np.log(y), 1)), rel=1e-12)
    assert np.abs(g).max() < 1e-12


def test_adam_first_step_moves_by_lr():
    g = np.array([1e-3, -2.0, 5.0])
    w, m, v = mlp.adam(np.zeros(3), np.zeros(3), np.zeros(3), g, 1, 1e-3)
    assert np.allclose(w, -1e-3 * np.sign(g), rtol=1e-4)


def test_bf16_rounding():
    assert mlp.bf16(1.0) == 1.0
    assert mlp.bf16(1.0 + 2 ** -9) == 1.0          # tie to even
    assert mlp.bf16(1.0 + 3 * 2 ** -9) == 1.0 + 2 ** -7
    x = np.random.default_rng(3).normal(size=1000)
    assert np.all(np.abs(mlp.bf16(x) - x) <= 2 ** -8 * np.abs(x))


def _perturbed(K, seed, scale=0.05):
    rng = np.random.default_rng(seed)
    w = mlp.init(K, seed=seed + 1).astype(np.float64)
    mask = mlp.pack(mlp.unpack(np.ones(mlp.N_PARAMS), K), K) != 0
    return (w + rng.normal(scale=scale, size=w.shape) * mask).astype(np.float32).astype(np.float64), rng


@pytest.mark.parametrize("K,B", [(8, 600), (4, 64), (16, 37), (8, 4096)])
def test_bfloat16_mirror_fits_the_rounding_error_model(K, B):
    """The tolerance model of the GPU parity tests (tests/mlp_bounds.py)
    against the bfloat16 mirror of the kernels, which rounds exactly where
    they round: the deviations from FP64 are of the order of the model's
    sigma (root-mean-square ratio between 0.05 and 2) and never beyond the
    8 sigma the GPU tests allow."""
    from tests import mlp_bounds as MB
    w, rng = _perturbed(K, 5)
    d = rng.normal(size=(B, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    la = rng.uniform(np.log(0.02), np.log(0.5), size=(B, 2))
    x = mlp.features(d, np.exp(la[:, 0]), np.exp(la[:, 1])).astype(np.float32).astype(np.float64)
    t = rng.dirichlet(np.ones(K) * 0.5, size=B)
    y64, sy, _ = MB.forward_sigma(w, x, K)
    ref, _ = mlp.forward(w, x, K, bf=False)
    np.testing.assert_allclose(y64, ref, rtol=1e-12, atol=1e-15)
    ybf, _ = mlp.forward(w, x, K, bf=True)
    r = np.abs(ybf - y64) / sy
    rms = float(np.sqrt(np.mean(r * r)))
    assert r.max() < 8 and 0.05 < rms < 2, (r.max(), rms)
    levels = np.concatenate([[0.0], np.sort(10.0 ** rng.uniform(-2, 3, K - 1))])
    for lv, lam in ((None, 0.0), (levels, 1.0)):
        g64, sg = MB.gradient_sigma(w, x, t, K, levels=lv, lam=lam)
        _, gref = mlp.loss_and_grad(w, x, t, K, bf=False, levels=lv, lam=lam)
        np.testing.assert_allclose(g64, gref, rtol=1e-10, atol=1e-14)
        _, gbf = mlp.loss_and_grad(w, x, t, K, bf=True, levels=lv, lam=lam)
        nz = sg > 0
        assert np.all(gbf[~nz] == 0) and np.all(g64[~nz] == 0)
        r = np.abs(gbf - g64)[nz] / sg[nz]
        rms = float(np.sqrt(np.mean(r * r)))
        assert r.max() < 8 and 0.02 < rms < 2, (lam, r.max(), rms)
