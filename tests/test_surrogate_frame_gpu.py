"""The learned surrogate on the frame workload (1920x1080, cube map
6x256x256, K = 8), trained with the workload's schedule (2^22 samples of
the plain filter, 20 epochs of batch 4096) by the library's own kernels.

Accuracy is the mean relative radiance error sum |L - L_ref| / sum |L_ref|
over the glint pixels and RGB, with the same hash draws.  The judge
L_ref is shading with the plain filter evaluated at each pixel's lookup
(glint_filter_pixels + glint_shade_given_F): the quantity the network
replaces, Sec. 5 Eq. (rtiblndf), at the pixel's own roughness.

* the network meets the 1e-2 bar against that filter and against the plain
  float32 pyramid path;
* what it gains over the method without it: its error against the filter
  is below the pyramid's (the pyramid interpolates between mips at
  alpha_m = (m/(M-1))^2 and between texels; the network is trained at
  continuous roughness and direction);
* the per-pixel filter itself matches the oracle's filter on sampled
  pixels (parity of glint_filter_pixels).
"""
import numpy as np
import pytest

import oracle
import synth
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


@pytest.fixture(scope="module")
def frame(ctx):
    import torch
    from paper_2507_02674_amd.pipeline import EnvPipeline, FilterShader, Shader, Surrogate, SurrogateShader
    w = synth.WORKLOADS["frame"]
    env_np, g = w.env(), w.gbuf()
    env = torch.from_numpy(env_np).cuda()
    pipe = EnvPipeline(ctx, w.R, w.K, w.M, w.T)
    pipe.build_luts()
    pipe.run(env)
    ref = FilterShader(ctx, g, w.K, seed=w.hash_seed)
    ref.run(pipe, env)
    pyr = Shader(ctx, g, seed=w.hash_seed)
    pyr.run(pipe.env_struct())
    U.log("surrogate frame: training 20 epochs over 2^22 samples")
    sur = Surrogate(ctx, w.K)
    sur.init(seed=7)
    sur.train(pipe, env)
    net = SurrogateShader(ctx, g, sur, seed=w.hash_seed)
    net.run(pipe.env_struct())
    torch.cuda.synchronize()
    hit = torch.from_numpy(g["surf_id"] != synth.NO_SURFACE).cuda()
    return dict(w=w, env_np=env_np, env=env, g=g, pipe=pipe, ref=ref, pyr=pyr, sur=sur, net=net, hit=hit)


def test_surrogate_meets_the_radiance_bar_and_beats_the_pyramid(frame):
    from paper_2507_02674_amd.pipeline import relative_l1
    f = frame
    e_net = relative_l1(f["net"].radiance, f["ref"].radiance, f["hit"])
    e_pyr = relative_l1(f["pyr"].radiance, f["ref"].radiance, f["hit"])
    e_np = relative_l1(f["net"].radiance, f["pyr"].radiance, f["hit"])
    U.log(f"  mean relative radiance error: network vs filter {e_net:.3e}, pyramid vs filter {e_pyr:.3e}, "
          f"network vs pyramid {e_np:.3e}")
    assert e_net <= 1e-2 and e_np <= 1e-2
    assert e_net < e_pyr


def test_probabilities_closer_to_the_filter_than_the_pyramid(frame):
    """The same comparison on the reflection probabilities themselves:
    radiance-weighted relative error sum_k L_k |p_k - p_k^ref| / sum_k L_k p_k^ref
    and mean absolute error, per pixel, averaged."""
    import torch
    f = frame
    w, P, K = f["w"], f["ref"].P, f["w"].K
    out = {}
    for name, run in (("ref", lambda d: G.glint_shade_given_F(f["ref"].ctx, f["ref"].gb, P, f["pipe"].env_struct(),
                                                              f["ref"].F, f["ref"].sp, f["ref"].radiance, d)),
                      ("pyr", lambda d: f["pyr"].run(f["pipe"].env_struct(), debug=d)),
                      ("net", lambda d: f["net"].run(f["pipe"].env_struct(), debug=d))):
        d = {"probs": torch.empty((P, K), dtype=torch.float64, device="cuda")}
        run(d)
        out[name] = d["probs"][f["hit"]]
    torch.cuda.synchronize()
    lv = f["pipe"].levels.double()[1:]
    ref = out["ref"]
    den = (ref[:, 1:] * lv).sum(1).clamp_min(1e-300)
    rw = {k: float((((out[k] - ref)[:, 1:].abs() * lv).sum(1) / den).mean()) for k in ("pyr", "net")}
    ma = {k: float((out[k] - ref).abs().mean()) for k in ("pyr", "net")}
    U.log(f"  radiance-weighted p error: pyramid {rw['pyr']:.3e}, network {rw['net']:.3e}; "
          f"mean |dp|: pyramid {ma['pyr']:.3e}, network {ma['net']:.3e}")
    assert rw["net"] < rw["pyr"]


def test_filter_pixels_matches_the_oracle_filter(ctx, frame):
    """glint_filter_pixels against the oracle's filter at the same lookups
    (directions and roughness computed in double from the G-buffer), on
    2000 sampled pixels of the frame (float outputs of double sums)."""
    f = frame
    w, g = f["w"], f["g"]
    rng = np.random.default_rng(4)
    hit = np.nonzero(g["surf_id"] != synth.NO_SURFACE)[0]
    pix = rng.choice(hit, 2000, replace=False)
    n = np.stack([g["nx"], g["ny"], g["nz"]], 1)[pix].astype(np.float64)
    v = np.stack([g["vx"], g["vy"], g["vz"]], 1)[pix].astype(np.float64)
    mu = (n * v).sum(1, keepdims=True)
    r = 2 * mu * n - v
    r /= np.linalg.norm(r, axis=1, keepdims=True)
    alpha = np.sqrt(g["ax"][pix].astype(np.float64) * g["ay"][pix].astype(np.float64))
    pipe = f["pipe"]
    ij, it = U.host(pipe.ind_j), U.host(pipe.ind_t)
    chain = oracle.mipchain(f["env_np"], ij, it, w.K, w.M)
    o = oracle.sample_filter(f["env_np"], ij, it, chain, w.K, w.M, w.T, r, alpha)
    got = U.host(f["ref"].F)[pix].astype(np.float64)
    np.testing.assert_allclose(got, o[:, :w.K], rtol=1e-5, atol=1e-7)
    bg = np.nonzero(g["surf_id"] == synth.NO_SURFACE)[0][:100]
    assert np.all(U.host(f["ref"].F)[bg] == 0)


def test_fine_tuning_follows_rotating_suns(ctx, frame):
    """Rotating suns (sun s's azimuth +2 (s+1) degrees per frame): at frame
    4 the network trained on frame 0 has drifted; 200 fine-tuning steps per
    frame on the new frames' filter bring it back under the bar."""
    import torch
    from paper_2507_02674_amd.pipeline import FilterShader, Surrogate, SurrogateShader, relative_l1
    f = frame
    w, g = f["w"], f["g"]
    tuned = Surrogate(ctx, w.K)
    tuned.restore(f["sur"].state())
    pipe = f["pipe"]
    ref = FilterShader(ctx, g, w.K, seed=w.hash_seed)
    for fr in range(1, 5):
        env = torch.from_numpy(synth.make_env(w.R, w.env_seed, frame=fr)).cuda()
        pipe.run(env)
        tuned.fine_tune(pipe, env, seed=100 + fr)
    ref.run(pipe, env)
    frozen_sh = SurrogateShader(ctx, g, f["sur"], seed=w.hash_seed)
    tuned_sh = SurrogateShader(ctx, g, tuned, seed=w.hash_seed)
    frozen_sh.run(pipe.env_struct())
    tuned_sh.run(pipe.env_struct())
    torch.cuda.synchronize()
    e_frozen = relative_l1(frozen_sh.radiance, ref.radiance, f["hit"])
    e_tuned = relative_l1(tuned_sh.radiance, ref.radiance, f["hit"])
    U.log(f"  frame 4: frozen {e_frozen:.3e}, fine-tuned {e_tuned:.3e}")
    assert e_tuned < e_frozen and e_tuned <= 1e-2
    pipe.run(f["env"])  # leave the module's map as it was
