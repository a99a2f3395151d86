"""Pins of the oracle's anisotropic lookup (several samples of the
prefiltered map along the lobe, the future work of Sec. 8; tap layout in
include/glint.h): reductions to the isotropic lookup, symmetries, and a
brute-force anisotropic filter of the source map that it approximates
better than the single lookup at alpha = sqrt(alpha_x alpha_y)."""
import numpy as np
import pytest

import oracle
import synth

R, K, M = 64, 8, 7


@pytest.fixture(scope="module")
def scene():
    env = synth.make_env(R, 7)
    levels, ij, it = oracle.partition(env, K)
    chain = oracle.mipchain(env, ij, it, K, M)
    ind, rgb = oracle.split_pyramid(oracle.prefilter(env, ij, it, chain, K, M, 64), K)
    S, E = oracle.lut_tables()
    return dict(env=env, ij=ij, it=it, levels=levels, ind=ind, rgb=rgb, S=S, E=E)


def gbuf(n, v, t, ax, ay):
    P = len(n)
    g = {k: np.zeros(P, np.float32) for k in oracle.GBUF_FIELDS}
    for c, k in enumerate("xyz"):
        g["n" + k], g["v" + k], g["t" + k] = (a[:, c].astype(np.float32) for a in (n, v, t))
    g["u"][:] = np.arange(P) * 0.37
    g["area"][:] = 1e-4
    g["ax"][:], g["ay"][:] = ax, ay
    g["density"][:] = 1e8
    g["f0r"][:] = g["f0g"][:] = g["f0b"][:] = 0.9
    g["surf_id"] = np.ones(P, np.uint32)
    return g


def frames(P, seed, normal_incidence=False):
    rng = np.random.default_rng(seed)
    n = rng.normal(size=(P, 3))
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    if normal_incidence:
        v = n.copy()
    else:
        v = n + 0.6 * rng.normal(size=(P, 3))
        v /= np.linalg.norm(v, axis=1, keepdims=True)
        flip = (v * n).sum(1) < 0.1
        v[flip] = n[flip]
    t = rng.normal(size=(P, 3))
    t -= (t * n).sum(1, keepdims=True) * n
    t /= np.linalg.norm(t, axis=1, keepdims=True)
    return n, v, t


def shade(s, g, T):
    return oracle.shade(g, s["ind"], s["rgb"], s["levels"], s["S"], s["E"], R, K, M, 3, 1, lobe_taps=T)


def test_isotropic_roughness_reduces_to_one_lookup(scene):
    """alpha_x = alpha_y: a_t = alpha, s = 0, every tap reads w_r at the
    same lod, so the lookup is the single isotropic one."""
    n, v, t = frames(300, 1)
    g = gbuf(n, v, t, 0.12, 0.12)
    a = shade(scene, g, 0)
    for T in (2, 4, 8):
        b = shade(scene, g, T)
        np.testing.assert_allclose(b["probs"], a["probs"], rtol=1e-13, atol=1e-15)
        np.testing.assert_allclose(b["radiance"], a["radiance"], rtol=1e-12, atol=1e-30)


def test_axis_swap_and_tangent_sign_symmetries(scene):
    """Swapping alpha_x and alpha_y while turning the tangent by 90 degrees,
    or flipping the tangent, describes the same lobe."""
    n, v, t = frames(300, 2)
    b = np.cross(n, t)
    a = shade(scene, gbuf(n, v, t, 0.4, 0.05), 8)
    c = shade(scene, gbuf(n, v, b, 0.05, 0.4), 8)
    d = shade(scene, gbuf(n, v, -t, 0.4, 0.05), 8)
    for o in (c, d):
        np.testing.assert_allclose(o["probs"], a["probs"], rtol=1e-6, atol=1e-12)
    # the tangent's float rounding differs after the turn, so only close
    np.testing.assert_allclose(d["probs"], a["probs"], rtol=1e-12, atol=1e-15)


def test_degenerate_tangent_uses_a_frame_of_n(scene):
    """A tangent parallel to the normal falls back to the frame onb(n):
    results are finite and probabilities sum to one."""
    n, v, t = frames(100, 4)
    out = shade(scene, gbuf(n, v, n.copy(), 0.4, 0.05), 4)
    assert np.all(np.isfinite(out["radiance"]))
    np.testing.assert_allclose(out["probs"].sum(1), 1.0, rtol=1e-12)


def brute_force(scene, n, t, ax, ay):
    """Normalised indicator values of the anisotropic filter kernel
    D(h) <r, l>+ (the isotropic kernel of the prefilter with the anisotropic
    GGX D; n = v = r) summed over every texel of the unfiltered source map
    (texel solid angle (2/R)^2 / |d|^3)."""
    d = np.zeros((6, R, R, 3))
    om = np.zeros((6, R, R))
    for f in range(6):
        for y in range(R):
            for x in range(R):
                e = oracle.face_dir(f, 2 * (x + 0.5) / R - 1, 2 * (y + 0.5) / R - 1)
                L = np.linalg.norm(e)
                d[f, y, x], om[f, y, x] = e / L, (2.0 / R) ** 2 / L ** 3
    W = np.zeros((6, R, R, K))
    ij, it = scene["ij"], scene["it"]
    for k in range(K):
        W[..., k] = np.where(ij == k, 1 - it, 0) + np.where(ij + 1 == k, it, 0)
    d, om, W = d.reshape(-1, 3), om.reshape(-1), W.reshape(-1, K)
    b = np.cross(n, t)
    out = []
    for i in range(len(n)):
        cl = d @ n[i]
        h = d + n[i]
        h /= np.linalg.norm(h, axis=1, keepdims=True)
        hx, hy, hz = h @ t[i], h @ b[i], h @ n[i]
        D = 1.0 / (np.pi * ax * ay * (hx ** 2 / ax ** 2 + hy ** 2 / ay ** 2 + hz ** 2) ** 2)
        w = np.where(cl > 0, D * cl, 0.0) * om
        out.append((w[:, None] * W).sum(0) / w.sum())
    return np.array(out)


@pytest.mark.parametrize("ax,ay", [(0.5, 0.02), (0.05, 0.3), (0.4, 0.05)])
def test_closer_to_the_anisotropic_filter_than_one_lookup(scene, ax, ay):
    """At normal incidence (where the prefilter's n = v = r holds), eight
    taps reproduce the brute-force anisotropic filter markedly better than
    the single lookup at sqrt(alpha_x alpha_y): L1 error of the normalised
    reflecting-bin distribution F_k / sum_{j>=1} F_j."""
    n, v, t = frames(200, 5, normal_incidence=True)
    ref = brute_force(scene, n, t, ax, ay)[:, 1:]
    ref /= ref.sum(1, keepdims=True)
    g = gbuf(n, v, t, ax, ay)

    def err(T):
        p = shade(scene, g, T)["probs"][:, 1:]
        return np.abs(p / p.sum(1, keepdims=True) - ref).sum(1).mean()

    e1, e8 = err(0), err(8)
    assert e8 < 0.8 * e1, (e1, e8)
