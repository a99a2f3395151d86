"""The overlapped frame pipeline (environment work of later frames on one
stream beside the shading of frame f on another, buffer sets reused in
turn) gives every frame exactly the radiance of the serial path."""
import numpy as np
import pytest

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


@pytest.mark.parametrize("buffers", [2, 3])
def test_overlapped_frames_equal_serial_frames(ctx, buffers):
    import torch
    from paper_2507_02674_amd.pipeline import EnvPipeline, FramePipeline, Shader
    R, K, M, T = 32, 8, 6, 64
    U.log(f"frame pipeline buffers={buffers}")
    envs = [torch.from_numpy(synth.make_env(R, s)).cuda() for s in (3, 4, 5, 6, 7)]
    g = synth.scene_frame(192, 108, seed=2, density_decades=(2.0, 8.0))
    shader = Shader(ctx, g, seed=5)
    frames = FramePipeline(lambda: EnvPipeline(ctx, R, K, M, T), shader, overlap=True, buffers=buffers)
    frames.build_luts()
    n = 11
    got = [torch.empty_like(shader.radiance) for _ in range(n)]
    for f in range(n):
        frames.step(envs[f % len(envs)])
        with torch.cuda.stream(frames.s_shade):
            got[f].copy_(shader.radiance)
    torch.cuda.synchronize()
    # serial reference on the default stream, one buffer set
    ref_pipe = EnvPipeline(ctx, R, K, M, T)
    ref_pipe.build_luts()
    ref_sh = Shader(ctx, g, seed=5)
    for f in range(n):
        ref_pipe.run(envs[f % len(envs)])
        ref_sh.run(ref_pipe.env_struct())
        torch.cuda.synchronize()
        assert torch.equal(got[f], ref_sh.radiance), f
    # consecutive frames differ (the maps differ), so equality is not vacuous
    assert not torch.equal(got[0], got[1])


def test_frames_wait_for_the_callers_stream(ctx):
    """Tables built on the caller's stream behind a long-running kernel are
    complete before any frame reads them (the pipeline's streams do not
    synchronise with the caller's stream by themselves)."""
    import torch
    from paper_2507_02674_amd.pipeline import EnvPipeline, FramePipeline, Shader
    R, K, M, T = 32, 8, 6, 64
    U.log("frame pipeline behind a busy caller stream")
    env = torch.from_numpy(synth.make_env(R, 3)).cuda()
    g = synth.scene_frame(192, 108, seed=2, density_decades=(2.0, 8.0))
    shader = Shader(ctx, g, seed=5)
    frames = FramePipeline(lambda: EnvPipeline(ctx, R, K, M, T), shader, overlap=True, buffers=3)
    # finite but wrong tables (S = 0 reflects nothing) until build_luts runs
    for p in frames.pipes:
        for t in (p.lut_S, p.lut_E, p.qtail):
            t.zero_()
    torch.cuda.synchronize()
    torch.cuda._sleep(50_000_000)  # a bounded spin on the caller's stream (~20 ms)
    frames.build_luts()
    got = []
    for f in range(3):
        frames.step(env)
        with torch.cuda.stream(frames.s_shade):
            got.append(shader.radiance.clone())
    torch.cuda.synchronize()
    ref_pipe = EnvPipeline(ctx, R, K, M, T)
    ref_pipe.build_luts()
    ref_pipe.run(env)
    ref_sh = Shader(ctx, g, seed=5)
    ref_sh.run(ref_pipe.env_struct())
    torch.cuda.synchronize()
    for f in range(3):
        assert torch.equal(got[f], ref_sh.radiance), f


def test_frames_keep_the_callers_map_alive(ctx):
    """A map dropped by the caller right after step() is not overwritten
    before the environment stream has read it (the frame equals the serial
    frame of the same map), with many frames over freshly uploaded maps."""
    import torch
    from paper_2507_02674_amd.pipeline import EnvPipeline, FramePipeline, Shader
    R, K, M, T = 32, 8, 6, 64
    U.log("frame pipeline over dropped maps")
    maps = [synth.make_env(R, s) for s in (3, 4)]
    g = synth.scene_frame(96, 54, seed=2, density_decades=(2.0, 8.0))
    shader = Shader(ctx, g, seed=5)
    frames = FramePipeline(lambda: EnvPipeline(ctx, R, K, M, T), shader, overlap=True, buffers=3)
    frames.build_luts()
    got = []
    for f in range(40):
        env = torch.from_numpy(maps[f % 2]).cuda()
        frames.step(env)
        del env
        # allocations on the caller's stream that would reuse a freed map
        junk = torch.full((6, R, R, 3), -1.0, device="cuda")
        del junk
        with torch.cuda.stream(frames.s_shade):
            got.append(shader.radiance.clone())
    torch.cuda.synchronize()
    ref = []
    for m in maps:
        p = EnvPipeline(ctx, R, K, M, T)
        p.build_luts()
        p.run(torch.from_numpy(m).cuda())
        sh = Shader(ctx, g, seed=5)
        sh.run(p.env_struct())
        torch.cuda.synchronize()
        ref.append(sh.radiance.clone())
    for f in range(40):
        assert torch.equal(got[f], ref[f % 2]), f
