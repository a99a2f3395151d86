"""The allocation-free partition entry point (glint_partition_env_noalloc)
against glint_partition_env, through the C ABI: bit-identical outputs on
calls in a row (the second on a smaller map), both level modes, and the
size limit of its scratch array."""
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


def outputs(R, K):
    import torch
    return (torch.full((K,), -1.0, dtype=torch.float64, device="cuda"),
            torch.full((6, R, R), 255, dtype=torch.uint8, device="cuda"),
            torch.full((6, R, R), -1.0, dtype=torch.float32, device="cuda"))


def noalloc(ctx, env, K, level_mode, ws=0):
    R = env.shape[1]
    lv, ij, it = outputs(R, K)
    G.glint_partition_env_noalloc(ctx, U.dev(env), R, G.PartitionParams(K, 1e-3, level_mode, ws), lv, ij, it)
    return U.host(lv), U.host(ij), U.host(it)


@pytest.mark.parametrize("level_mode", [0, 1, 2])
def test_noalloc_partition_equals_workspace_call(ctx, level_mode):
    U.log(f"noalloc partition level_mode={level_mode}")
    cases = [(256, 8, 2), (32, 4, 7)] if level_mode != 2 else [(64, 8, 3), (16, 4, 5)]
    for R, K, seed in cases:  # the second call is smaller
        env = synth.make_env(R, seed)
        a = noalloc(ctx, env, K, level_mode)
        b = U.partition(ctx, env, K, 1e-3, level_mode, 0)
        for x, y in zip(a, b):
            assert np.array_equal(x, y), (R, K)


def test_noalloc_partition_largest_sizes_and_limits(ctx):
    import torch
    U.log("noalloc partition limits")
    env = synth.make_env(1024, 4)
    a = noalloc(ctx, env, 16, 1, ws=1)  # the largest quantile-mode map
    b = U.partition(ctx, env, 16, 1e-3, 1, 1)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    lv, ij, it = outputs(8, 4)
    big = torch.zeros((6, 2048, 2048, 3), dtype=torch.float32, device="cuda")
    lv2, ij2, it2 = outputs(2048, 4)
    with pytest.raises(G.GlintError) as e:
        G.glint_partition_env_noalloc(ctx, big, 2048, G.PartitionParams(4, 1e-3, 1, 0), lv2, ij2, it2)
    assert e.value.code == G.GLINT_EINVAL and "scratch" in str(e.value)
    with pytest.raises(G.GlintError) as e:
        G.glint_partition_env_noalloc(ctx, U.dev(synth.make_env(8, 1)), 8, G.PartitionParams(1, 1e-3, 0, 0), lv, ij,
                                      it)
    assert e.value.code == G.GLINT_EINVAL
    # the log-lerp mode fits the largest face size (R = 4096)
    del big
    gen = torch.Generator(device="cuda").manual_seed(3)
    env = torch.rand((6, 4096, 4096, 3), generator=gen, device="cuda") * 100.0
    lv, ij, it = outputs(4096, 8)
    G.glint_partition_env_noalloc(ctx, env, 4096, G.PartitionParams(8, 1e-3, 0, 0), lv, ij, it)
    lv2, ij2, it2 = outputs(4096, 8)
    ws = torch.empty(G.glint_partition_workspace_bytes(4096) // 8, dtype=torch.float64, device="cuda")
    G.glint_partition_env(ctx, env, 4096, G.PartitionParams(8, 1e-3, 0, 0), ws, lv2, ij2, it2)
    torch.cuda.synchronize()
    assert torch.equal(lv, lv2) and torch.equal(ij, ij2) and torch.equal(it, it2)
