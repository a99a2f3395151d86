"""GPU parity of the learned surrogate and of the filter sampler, through the C ABI.

* glint_sample_filter / glint_surrogate_samples against the oracle's filter
  at arbitrary (direction, alpha) (float outputs of double sums: 1e-5
  relative); at a mip's roughness and a texel's centre direction the sampler
  reproduces the stored pyramid texel.
* glint_surrogate_forward / _gradient / _train_step against the plain FP64
  definition (oracle/mlp.py, bf=False), element by element, within 8
  standard deviations of a bfloat16 rounding-error model of that definition
  (tests/mlp_bounds.py); and, tighter, against the same definition rounded
  at the points where the matrix cores are fed (bf=True), where only float
  accumulation order and a rare bfloat16 rounding-boundary flip remain.
* glint_surrogate_train_step = the gradient followed by Adam.
* glint_shade_surrogate: the network's per-pixel outputs against the
  oracle's forward pass, and the shading given those outputs against the
  oracle's shading given the same values (the parity bar of the plain path).
"""
import numpy as np
import pytest

import oracle
import synth
from oracle import mlp
from paper_2507_02674_amd import glint as G
from tests import gpu_util as U

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU; the library has no CPU fallback")
    c = G.glint_create(0)
    yield c
    G.glint_destroy(c)


def upload_params(ctx, w, K):
    import torch
    wt = U.dev(np.asarray(w, dtype=np.float32))
    wb = torch.empty(wt.numel(), dtype=torch.int16, device="cuda")
    G.glint_surrogate_prepare(ctx, K, wt, wb)
    return wt, wb


def random_inputs(n, seed):
    rng = np.random.default_rng(seed)
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    la = rng.uniform(np.log(0.02), np.log(0.5), size=(n, 2))
    return mlp.features(d, np.exp(la[:, 0]), np.exp(la[:, 1])).astype(np.float32)


def env_setup(ctx, R=32, K=4, M=6, T=64, seed=3):
    """Plain filter state on the GPU plus the oracle's own chain."""
    import torch
    from paper_2507_02674_amd.pipeline import EnvPipeline
    env = synth.make_env(R, seed)
    pipe = EnvPipeline(ctx, R, K, M, T)
    pipe.build_luts()
    et = torch.from_numpy(env).cuda()
    pipe.run(et)
    torch.cuda.synchronize()
    return env, et, pipe


# --- filter sampler -----------------------------------------------------------------

@pytest.mark.parametrize("K", [4, 8])
def test_sample_filter_matches_oracle(ctx, K):
    import torch
    U.log(f"sample_filter K={K}")
    env, et, pipe = env_setup(ctx, K=K)
    rng = np.random.default_rng(5)
    n = 777  # ragged against the 32-sample groups of a block
    d = rng.normal(size=(n, 3)).astype(np.float32)
    alphas = np.exp(rng.uniform(np.log(0.01), np.log(1.0), size=n)).astype(np.float32)
    alphas[:5] = [1e-4, 0.04, 0.25, 0.64, 1.0]
    out = torch.empty((n, K + 3), dtype=torch.float32, device="cuda")
    G.glint_sample_filter(ctx, et, pipe.ind_j, pipe.ind_t, pipe.R, K, pipe.fp, pipe.filt_ws, U.dev(d),
                          U.dev(alphas), out)
    got = U.host(out)
    levels, ind_j, ind_t = oracle.partition(env, K)
    chain = oracle.mipchain(env, ind_j, ind_t, K, pipe.M)
    ref = oracle.sample_filter(env, ind_j, ind_t, chain, K, pipe.M, pipe.T, d.astype(np.float64),
                               alphas.astype(np.float64))
    np.testing.assert_allclose(got, ref, rtol=1e-5, atol=1e-7)


def test_sample_filter_reproduces_pyramid_texels(ctx):
    """At alpha_m = (m/(M-1))^2 and a texel centre the sampler is the prefilter."""
    import torch
    env, et, pipe = env_setup(ctx, K=4)
    R, M, K = pipe.R, pipe.M, pipe.K
    rng = np.random.default_rng(6)
    dirs, alphas, tex = [], [], []
    for m in range(1, M):
        n = R >> m
        for _ in range(40):
            f, x, y = rng.integers(6), rng.integers(n), rng.integers(n)
            d = oracle.face_dir(int(f), 2.0 * (x + 0.5) / n - 1.0, 2.0 * (y + 0.5) / n - 1.0)
            dirs.append(d)
            alphas.append((m / (M - 1)) ** 2)
            tex.append(G.glint_pyramid_texels(R, m) + (f * n + y) * n + x)
    d = np.asarray(dirs, dtype=np.float32)
    a = np.asarray(alphas, dtype=np.float32)
    out = torch.empty((len(a), K + 3), dtype=torch.float32, device="cuda")
    G.glint_sample_filter(ctx, et, pipe.ind_j, pipe.ind_t, R, K, pipe.fp, pipe.filt_ws, U.dev(d), U.dev(a), out)
    got = U.host(out)
    ind, rgb = U.host(pipe.ind_pyr), U.host(pipe.rgb_pyr)
    tex = np.asarray(tex)
    np.testing.assert_allclose(got[:, :K], ind[tex], rtol=2e-6, atol=1e-7)
    np.testing.assert_allclose(got[:, K:], rgb[tex, :3], rtol=2e-6, atol=1e-7)


def test_surrogate_samples_match_oracle(ctx):
    import torch
    env, et, pipe = env_setup(ctx, K=8)
    K, n = 8, 500
    rng = np.random.default_rng(7)
    d = (rng.normal(size=(n, 3)) * 3.0).astype(np.float32)  # not unit: the sampler normalises
    ax = np.exp(rng.uniform(np.log(0.02), np.log(0.5), n)).astype(np.float32)
    ay = np.exp(rng.uniform(np.log(0.02), np.log(0.5), n)).astype(np.float32)
    x = torch.empty((n, 5), dtype=torch.float32, device="cuda")
    t = torch.empty((n, K), dtype=torch.float32, device="cuda")
    G.glint_surrogate_samples(ctx, et, pipe.ind_j, pipe.ind_t, pipe.R, K, pipe.fp, pipe.filt_ws, U.dev(d),
                              U.dev(ax), U.dev(ay), x, t)
    gx, gt = U.host(x), U.host(t)
    d64 = d.astype(np.float64)
    u = d64 / np.linalg.norm(d64, axis=1, keepdims=True)
    np.testing.assert_allclose(gx, mlp.features(u, ax.astype(np.float64), ay.astype(np.float64)), rtol=1e-6,
                               atol=1e-6)
    levels, ind_j, ind_t = oracle.partition(env, K)
    chain = oracle.mipchain(env, ind_j, ind_t, K, pipe.M)
    ref = oracle.sample_filter(env, ind_j, ind_t, chain, K, pipe.M, pipe.T, d64,
                               np.sqrt(ax.astype(np.float64) * ay.astype(np.float64)))[:, :K]
    ref = ref / ref.sum(1, keepdims=True)
    np.testing.assert_allclose(gt, ref, rtol=1e-5, atol=1e-7)
    assert np.allclose(gt.sum(1), 1.0, atol=1e-5)


# --- network ------------------------------------------------------------------------

@pytest.mark.parametrize("K,B", [(8, 4096), (4, 1000), (16, 33), (8, 1)])
def test_forward_matches_oracle(ctx, K, B):
    import torch
    U.log(f"surrogate forward K={K} B={B}")
    w = mlp.init(K, seed=11)
    rng = np.random.default_rng(12)
    w = (w + rng.normal(scale=0.02, size=w.shape) * (mlp.pack(mlp.unpack(np.ones(mlp.N_PARAMS), K), K) != 0))
    w = w.astype(np.float32)
    wt, wb = upload_params(ctx, w, K)
    x = random_inputs(B, 13)
    probs = torch.empty((B, K), dtype=torch.float32, device="cuda")
    G.glint_surrogate_forward(ctx, K, wt, wb, U.dev(x), probs)
    got = U.host(probs).astype(np.float64)
    ref, _ = mlp.forward(w.astype(np.float64), x.astype(np.float64), K, bf=True)
    err = np.abs(got - ref)
    U.log(f"  max abs err {err.max():.2e}, mean {err.mean():.2e}")
    assert err.max() < 3e-3 and err.mean() < 2e-5
    # the bf16 copy is the master rounded to nearest even, pads zero
    wb_host = U.host(wb).view(np.uint16)
    assert np.array_equal(wb_host, U.encode(U.host(wt).astype(np.float64), G.GLINT_BF16))
    assert np.all(U.host(wt)[mlp.pack(mlp.unpack(np.ones(mlp.N_PARAMS), K), K) == 0] == 0)


@pytest.mark.parametrize("K,B", [(8, 1000), (4, 64), (16, 37)])
def test_gradient_matches_oracle(ctx, K, B):
    import torch
    U.log(f"surrogate gradient K={K} B={B}")
    rng = np.random.default_rng(21)
    w = mlp.init(K, seed=22).astype(np.float64)
    mask = mlp.pack(mlp.unpack(np.ones(mlp.N_PARAMS), K), K) != 0
    w = (w + rng.normal(scale=0.05, size=w.shape) * mask).astype(np.float32)
    wt, wb = upload_params(ctx, w, K)
    x = random_inputs(B, 23)
    t = rng.dirichlet(np.ones(K) * 0.5, size=B).astype(np.float32)
    ws = torch.empty(G.glint_surrogate_workspace_bytes(B) // 4, dtype=torch.float32, device="cuda")
    grad = torch.empty(mlp.N_PARAMS, dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    G.glint_surrogate_gradient(ctx, K, wt, wb, U.dev(x), U.dev(t), ws, grad, loss)
    g = U.host(grad).astype(np.float64)
    rl, rg = mlp.loss_and_grad(w.astype(np.float64), x.astype(np.float64), t.astype(np.float64), K, bf=True)
    assert float(U.host(loss)[0]) == pytest.approx(rl, rel=1e-5)
    assert np.all(g[~mask] == 0)
    for name, (o, n) in mlp.OFF.items():
        a, b = g[o:o + n], rg[o:o + n]
        rel = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)
        U.log(f"  {name}: rel L2 err {rel:.2e}")
        assert rel < 3e-3, name
    # deterministic: a second evaluation is bit-identical
    grad2 = torch.empty_like(grad)
    G.glint_surrogate_gradient(ctx, K, wt, wb, U.dev(x), U.dev(t), ws, grad2, loss)
    assert np.array_equal(U.host(grad2), U.host(grad))


# --- against the plain FP64 definition (bf=False), element by element ----------------

def _fp64_case(K, B, seed):
    rng = np.random.default_rng(seed)
    w = mlp.init(K, seed=seed + 1).astype(np.float64)
    mask = mlp.pack(mlp.unpack(np.ones(mlp.N_PARAMS), K), K) != 0
    w = (w + rng.normal(scale=0.05, size=w.shape) * mask).astype(np.float32)
    x = random_inputs(B, seed + 2)
    t = rng.dirichlet(np.ones(K) * 0.5, size=B).astype(np.float32)
    return w, x, t, mask


@pytest.mark.parametrize("K,B", [(8, 4096), (4, 1000), (16, 33)])
def test_forward_matches_fp64_definition(ctx, K, B):
    """Every output within 8 sigma of the bfloat16 rounding-error model
    (tests/mlp_bounds.py) of the plain FP64 network."""
    import torch
    from tests import mlp_bounds as MB
    w, x, _, _ = _fp64_case(K, B, 41)
    wt, wb = upload_params(ctx, w, K)
    probs = torch.empty((B, K), dtype=torch.float32, device="cuda")
    G.glint_surrogate_forward(ctx, K, wt, wb, U.dev(x), probs)
    got = U.host(probs).astype(np.float64)
    y64, sy, _ = MB.forward_sigma(w.astype(np.float64), x.astype(np.float64), K)
    r = np.abs(got - y64) / (sy + 6e-8 * y64)
    U.log(f"  forward vs FP64: max {r.max():.2f} sigma, rms {np.sqrt(np.mean(r * r)):.3f}")
    assert r.max() < 8.0


def _levels(K, seed):
    rng = np.random.default_rng(seed)
    return np.concatenate([[0.0], np.sort(10.0 ** rng.uniform(-2, 3, K - 1))])


@pytest.mark.parametrize("K,B,lam", [(8, 1000, 0.0), (4, 64, 0.0), (16, 37, 0.0), (8, 4096, 0.0), (8, 1000, 1.0),
                                     (16, 300, 2.5)])
def test_gradient_matches_fp64_definition(ctx, K, B, lam):
    """Every gradient entry within 8 sigma of the rounding-error model of the
    plain FP64 gradient (pads exactly zero); the loss within 1e-3; with
    lam > 0 the loss carries the radiance-weighted term."""
    import torch
    from tests import mlp_bounds as MB
    w, x, t, mask = _fp64_case(K, B, 51)
    t[5] = 0.0
    t[5, 0] = 1.0  # reflects nothing above level 0: no radiance-weighted term
    lv = _levels(K, 52) if lam > 0 else None
    wt, wb = upload_params(ctx, w, K)
    ws = torch.empty(G.glint_surrogate_workspace_bytes(B) // 4, dtype=torch.float32, device="cuda")
    grad = torch.empty(mlp.N_PARAMS, dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    G.glint_surrogate_gradient(ctx, K, wt, wb, U.dev(x), U.dev(t), ws, grad, loss,
                               levels=U.dev(lv) if lv is not None else None, radiance_weight=lam)
    g = U.host(grad).astype(np.float64)
    g64, sg = MB.gradient_sigma(w.astype(np.float64), x.astype(np.float64), t.astype(np.float64), K, levels=lv,
                                lam=lam)
    l64, _ = mlp.loss_and_grad(w.astype(np.float64), x.astype(np.float64), t.astype(np.float64), K, levels=lv,
                               lam=lam)
    assert float(U.host(loss)[0]) == pytest.approx(l64, rel=1e-3)
    assert np.all(g[~mask] == 0)
    r = np.abs(g - g64)[mask] / (sg[mask] + 6e-8 * np.abs(g64[mask]) + 1e-30)
    U.log(f"  gradient vs FP64: max {r.max():.2f} sigma, rms {np.sqrt(np.mean(r * r)):.3f}")
    assert r.max() < 8.0


def test_adam_step_matches_fp64_definition(ctx):
    """One training step (step 1) against FP64 Adam on the FP64 gradient:
    the first step moves every weight by lr sign(g) (|g| >> eps), so where
    the model makes the gradient's sign certain (|g64| > 8 sigma) the step
    agrees to float rounding; elsewhere it is within 2 lr."""
    import torch
    from tests import mlp_bounds as MB
    K, B, lr = 8, 2048, 1e-3
    w, x, t, mask = _fp64_case(K, B, 61)
    wt, wb = upload_params(ctx, w, K)
    ws = torch.empty(G.glint_surrogate_workspace_bytes(B) // 4, dtype=torch.float32, device="cuda")
    m = torch.zeros(mlp.N_PARAMS, dtype=torch.float32, device="cuda")
    v = torch.zeros_like(m)
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    G.glint_surrogate_train_step(ctx, K, wt, wb, m, v, 1, lr, U.dev(x), U.dev(t), ws, loss)
    got = U.host(wt).astype(np.float64)
    g64, sg = MB.gradient_sigma(w.astype(np.float64), x.astype(np.float64), t.astype(np.float64), K)
    w64, _, _ = mlp.adam(w.astype(np.float64), np.zeros(mlp.N_PARAMS), np.zeros(mlp.N_PARAMS), g64, 1, lr)
    sure = mask & (np.abs(g64) > 8.0 * sg) & (np.abs(g64) > 1e-6)
    assert sure.sum() > 0.5 * mask.sum()
    err = np.abs(got - w64)
    # float rounding of the update and of w, plus the update's sensitivity
    # lr eps / (|g| + eps)^2 to the gradient's deviation (eps = 1e-8)
    fl = 2.0 ** -23 * np.abs(w64) + lr * 1e-5 + lr * 1e-8 * 8.0 * sg / (np.abs(g64) + 1e-8) ** 2
    assert np.all(err[sure] <= fl[sure]), err[sure].max()
    assert np.all(err[mask] <= 2 * lr + fl[mask])
    assert np.all(got[~mask] == 0)
    U.log(f"  Adam step 1: {int(sure.sum())}/{int(mask.sum())} weights with a certain sign agree to float rounding")


def test_train_step_is_gradient_then_adam(ctx):
    import torch
    K, B = 8, 512
    rng = np.random.default_rng(31)
    w = mlp.init(K, seed=32)
    wt, wb = upload_params(ctx, w, K)
    x, t = U.dev(random_inputs(B, 33)), U.dev(rng.dirichlet(np.ones(K), size=B).astype(np.float32))
    ws = torch.empty(G.glint_surrogate_workspace_bytes(B) // 4, dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    m = torch.zeros(mlp.N_PARAMS, dtype=torch.float32, device="cuda")
    v = torch.zeros_like(m)
    wh, mh, vh = U.host(wt).astype(np.float64), np.zeros(mlp.N_PARAMS), np.zeros(mlp.N_PARAMS)
    for step, lr in ((1, 1e-3), (2, 5e-4), (3, 2e-4)):
        grad = torch.empty(mlp.N_PARAMS, dtype=torch.float32, device="cuda")
        G.glint_surrogate_gradient(ctx, K, wt, wb, x, t, ws, grad, loss)
        g = U.host(grad).astype(np.float64)
        G.glint_surrogate_train_step(ctx, K, wt, wb, m, v, step, lr, x, t, ws, loss)
        wh, mh, vh = mlp.adam(wh, mh, vh, g, step, lr)
        np.testing.assert_allclose(U.host(wt), wh, rtol=0, atol=lr * 1e-3 + 1e-7)
        wh = U.host(wt).astype(np.float64)  # continue from the device's state
        mh, vh = U.host(m).astype(np.float64), U.host(v).astype(np.float64)


def test_training_reduces_loss_on_filter_targets(ctx):
    from paper_2507_02674_amd.pipeline import Surrogate
    U.log("surrogate training on a 32^2 map, K=8")
    env, et, pipe = env_setup(ctx, R=32, K=8, M=6)
    sur = Surrogate(ctx, 8)
    sur.init(seed=7)
    x, t = sur.samples(pipe, et, 1 << 15, seed=1)
    xv, tv = sur.samples(pipe, et, 4096, seed=2)
    p0 = U.host(sur.forward(xv)).astype(np.float64)
    loss0 = float(U.host(sur.gradient(xv, tv)[1])[0])
    curve = sur.fit(x, t, batch=1024, lr=3e-3, lr_min=1e-4, steps=600, log_every=100)
    loss1 = float(U.host(sur.gradient(xv, tv)[1])[0])
    U.log(f"  held-out loss {loss0:.4f} -> {loss1:.4f}; training curve {curve}")
    p1 = U.host(sur.forward(xv)).astype(np.float64)
    tvh = U.host(tv).astype(np.float64)
    e0, e1 = np.abs(p0 - tvh).mean(), np.abs(p1 - tvh).mean()
    base = np.abs(tvh.mean(0, keepdims=True) - tvh).mean()
    U.log(f"  held-out mean |F - F_filter|: init {e0:.4f}, trained {e1:.4f}, constant predictor {base:.4f}")
    assert loss1 < loss0 - 0.05
    assert e1 < 0.5 * base


# --- surrogate shading --------------------------------------------------------------

def test_shade_surrogate_matches_oracle(ctx):
    import torch
    from paper_2507_02674_amd.pipeline import Surrogate, SurrogateShader
    K, R, M = 8, 64, 7
    U.log("shade_surrogate 200x120, K=8")
    env, et, pipe = env_setup(ctx, R=R, K=K, M=M, seed=4)
    sur = Surrogate(ctx, K)
    sur.init(seed=5)
    x, t = sur.samples(pipe, et, 1 << 13, seed=3)
    sur.fit(x, t, batch=512, lr=3e-3, steps=50)
    gb = synth.scene_frame(200, 120, seed=9)
    sh = SurrogateShader(ctx, gb, sur, seed=17, vertices=1)
    P = sh.P
    dbg = dict(counts=torch.empty((P, 1, K), dtype=torch.float64, device="cuda"),
               codes=torch.empty((P, 1, K - 1), dtype=torch.uint8, device="cuda"),
               probs=torch.empty((P, K), dtype=torch.float64, device="cuda"))
    sh.run(pipe.env_struct(), debug=dbg)
    F = U.host(sh.F)[: P * K].reshape(P, K).astype(np.float64)
    surf = gb["surf_id"] != G.GLINT_NO_SURFACE
    # (1) network outputs per pixel vs the oracle's forward pass at the pixel's inputs
    n = np.stack([gb["nx"], gb["ny"], gb["nz"]], 1).astype(np.float64)
    v = np.stack([gb["vx"], gb["vy"], gb["vz"]], 1).astype(np.float64)
    mu = np.sum(n * v, 1, keepdims=True)
    wr = 2.0 * mu * n - v
    xs = mlp.features(wr[surf], gb["ax"][surf].astype(np.float64), gb["ay"][surf].astype(np.float64))
    ref, _ = mlp.forward(U.host(sur.w).astype(np.float64), xs.astype(np.float32).astype(np.float64), K, bf=True)
    err = np.abs(F[surf] - ref)
    U.log(f"  network: max abs err {err.max():.2e}, mean {err.mean():.2e}")
    assert err.max() < 3e-3 and err.mean() < 2e-5
    assert np.all(F[~surf] == 0)
    # (2) shading given those values vs the oracle's shading given the same values
    pix = np.nonzero(surf)[0]
    pix = pix[:: max(1, len(pix) // 6000)]
    rgb = U.host(pipe.rgb_pyr)
    S, E = U.host(pipe.lut_S), U.host(pipe.lut_E)
    orc = oracle.shade(gb, None, rgb, U.host(pipe.levels), S, E, R, K, M, 17, 1, pixels=pix, F=F[pix])
    gpu = dict(radiance=U.host(sh.radiance)[pix], probs=U.host(dbg["probs"])[pix],
               codes=U.host(dbg["codes"])[pix], counts=U.host(dbg["counts"])[pix])
    from tests.test_parity_gpu import check_shade
    check_shade(gpu, orc, K, "surrogate shading")
    bg = np.nonzero(~surf)[0]
    assert np.all(U.host(sh.radiance)[bg] == 0)


def test_surrogate_rejects_bad_arguments(ctx):
    import torch
    K = 8
    wt, wb = upload_params(ctx, mlp.init(K), K)
    x = U.dev(random_inputs(64, 1))
    probs = torch.empty((64, K), dtype=torch.float32, device="cuda")
    with pytest.raises(G.GlintError):
        G.glint_surrogate_forward(ctx, 33, wt, wb, x, probs)
    with pytest.raises(G.GlintError):
        G.glint_surrogate_forward(ctx, 1, wt, wb, x, probs)
    odd = torch.empty(wb.numel() + 8, dtype=torch.int16, device="cuda")[1:1 + wb.numel()]
    with pytest.raises(G.GlintError):
        G.glint_surrogate_forward(ctx, K, wt, odd, x, probs)
    assert G.glint_surrogate_workspace_bytes(0) == 0
    assert G.glint_surrogate_workspace_bytes((1 << 20) + 1) == 0
    ws = torch.empty(G.glint_surrogate_workspace_bytes(64) // 4, dtype=torch.float32, device="cuda")
    m = torch.zeros(mlp.N_PARAMS, dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    t = torch.full((64, K), 1.0 / K, dtype=torch.float32, device="cuda")
    with pytest.raises(G.GlintError):
        G.glint_surrogate_train_step(ctx, K, wt, wb, m, m.clone(), 0, 1e-3, x, t, ws, loss)
    for lv, lam in ((None, 1.0), (U.dev(_levels(K, 3)), -1.0)):  # a radiance weight needs levels; lam >= 0
        with pytest.raises(G.GlintError) as e:
            G.glint_surrogate_train_step(ctx, K, wt, wb, m, m.clone(), 1, 1e-3, x, t, ws, loss, levels=lv,
                                         radiance_weight=lam)
        assert e.value.code == G.GLINT_EINVAL
    # empty batch is a no-op for the forward pass
    G.glint_surrogate_forward(ctx, K, wt, wb, x[:0], probs)
    # parameters never prepared in this context, or prepared for another K
    raw = torch.zeros_like(wb)
    for call in (lambda: G.glint_surrogate_forward(ctx, K, wt, raw, x, probs),
                 lambda: G.glint_surrogate_forward(ctx, 4, wt, wb, x, probs[:, :4].contiguous()),
                 lambda: G.glint_surrogate_train_step(ctx, K, wt, raw, m, m.clone(), 1, 1e-3, x, t, ws, loss),
                 lambda: G.glint_surrogate_gradient(ctx, K, wt, raw, x, t, ws, m.clone(), loss)):
        with pytest.raises(G.GlintError) as e:
            call()
        assert e.value.code == G.GLINT_ENOTTRAINED
    other = G.glint_create(0)
    try:
        with pytest.raises(G.GlintError) as e:
            G.glint_surrogate_forward(other, K, wt, wb, x, probs)
        assert e.value.code == G.GLINT_ENOTTRAINED
        # per-context messages: the failure stays recorded on `other`, the
        # successful call below clears ctx's record only
        assert "never prepared" in G.glint_last_error(other)
        G.glint_surrogate_forward(ctx, K, wt, wb, x, probs)
        assert G.glint_last_error(ctx) == ""
        assert "never prepared" in G.glint_last_error(other)
        G.glint_surrogate_prepare(other, K, wt, wb)
        G.glint_surrogate_forward(other, K, wt, wb, x, probs)
        assert G.glint_last_error(other) == ""
    finally:
        G.glint_destroy(other)


def test_checkpoint_resume_reproduces_training(ctx, tmp_path):
    """Weights, Adam moments and the step counter saved mid-training; a fresh
    surrogate loaded from the file continues with identical losses and
    bit-identical weights (the kernels are deterministic)."""
    from paper_2507_02674_amd.pipeline import Surrogate, load_surrogate, save_surrogate
    env, et, pipe = env_setup(ctx, R=32, K=8, M=6)
    a = Surrogate(ctx, 8)
    a.init(seed=3)
    x, t = a.samples(pipe, et, 1 << 13, seed=4)
    a.fit(x, t, batch=512, lr=2e-3, steps=30, seed=5)
    path = str(tmp_path / "sur.ckpt")
    save_surrogate(a, path)
    curve_a = a.fit(x, t, batch=512, lr=2e-3, steps=30, seed=6, log_every=1)
    b = Surrogate(ctx, 8)
    load_surrogate(b, path)
    assert b.step == 30
    curve_b = b.fit(x, t, batch=512, lr=2e-3, steps=30, seed=6, log_every=1)
    assert curve_a == curve_b
    assert np.array_equal(U.host(a.w), U.host(b.w)) and np.array_equal(U.host(a.wb), U.host(b.wb))


def test_fallback_to_plain_filter_on_bad_weights(ctx):
    """The guard keeps the surrogate while its probe error is small and falls
    back to the plain form (identical radiance) when the weights are corrupted."""
    import torch
    from paper_2507_02674_amd.pipeline import GuardedShader, Shader, Surrogate, SurrogateShader
    env, et, pipe = env_setup(ctx, R=32, K=8, M=6)
    sur = Surrogate(ctx, 8)
    sur.init(seed=7)
    x, t = sur.samples(pipe, et, 1 << 15, seed=1)
    sur.fit(x, t, batch=1024, lr=3e-3, lr_min=1e-4, steps=400)
    gb = synth.scene_frame(96, 64, seed=3)
    guard = GuardedShader(SurrogateShader(ctx, gb, sur, seed=5), Shader(ctx, gb, seed=5), every=2, threshold=0.03)
    guard.run(pipe, et)
    U.log(f"  probe error trained {guard.last_error:.4f}")
    assert guard.use_surrogate
    with torch.no_grad():
        sur.w.copy_(torch.randn_like(sur.w) * 0.5)
    G.glint_surrogate_prepare(ctx, 8, sur.w, sur.wb)
    guard.run(pipe, et)  # frame 1: no check yet
    assert guard.use_surrogate
    guard.run(pipe, et)  # frame 2: check -> fall back
    U.log(f"  probe error corrupted {guard.last_error:.4f}")
    assert not guard.use_surrogate
    plain = Shader(ctx, gb, seed=5)
    plain.run(pipe.env_struct())
    assert np.array_equal(U.host(guard.radiance), U.host(plain.radiance))
