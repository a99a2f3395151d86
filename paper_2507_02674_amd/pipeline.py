"""Buffer management around the C ABI: one environment + one frame on one GPU.

PyTorch provides device memory and the stream; all compute is in libglint's
kernels (partition -> prefilter -> shade).  Buffers are allocated once at
construction so a frame enqueues kernels only.
"""
from __future__ import annotations

import torch

from . import glint as G

DTYPE_BYTES = {G.GLINT_F32: 4, G.GLINT_F16: 2, G.GLINT_BF16: 2, G.GLINT_UNORM16: 2}
_TORCH_STORAGE = {G.GLINT_F32: torch.float32, G.GLINT_F16: torch.float16, G.GLINT_BF16: torch.int16,
                  G.GLINT_UNORM16: torch.int16}


class EnvPipeline:
    """Per-frame environment work for a cube map of face size R."""

    def __init__(self, ctx, R, K, num_mips, taps=64, dtype=G.GLINT_F32, ell=1e-3, level_mode=0,
                 weight_space=0, device="cuda"):
        self.ctx, self.R, self.K, self.M, self.T, self.dtype = ctx, R, K, num_mips, taps, dtype
        self.pp = G.PartitionParams(K, ell, level_mode, weight_space)
        self.fp = G.PrefilterParams(num_mips, taps, dtype)
        nbytes = G.glint_partition_workspace_bytes(R)
        self.part_ws = torch.empty(max(nbytes // 8, 1), dtype=torch.float64, device=device)
        fbytes = G.glint_prefilter_workspace_bytes(R, K, self.fp)
        self.filt_ws = torch.empty(max(fbytes // 4, 4), dtype=torch.float32, device=device)
        self.levels = torch.empty(K, dtype=torch.float64, device=device)
        self.ind_j = torch.empty((6, R, R), dtype=torch.uint8, device=device)
        self.ind_t = torch.empty((6, R, R), dtype=torch.float32, device=device)
        self.texels = G.glint_pyramid_texels(R, num_mips)
        self.ind_pyr = torch.empty((self.texels, K), dtype=_TORCH_STORAGE[dtype], device=device)
        self.rgb_pyr = torch.empty((self.texels, 4), dtype=torch.float32, device=device)
        self.lut_S = torch.empty((G.LUT_N, G.LUT_N), dtype=torch.float32, device=device)
        self.lut_E = torch.empty((G.LUT_N, G.LUT_N, 2), dtype=torch.float32, device=device)

    def build_luts(self, stream=None):
        G.glint_build_luts(self.ctx, self.lut_S, self.lut_E, stream)

    def partition(self, env, stream=None):
        G.glint_partition_env(self.ctx, env, self.R, self.pp, self.part_ws, self.levels, self.ind_j, self.ind_t,
                              stream)

    def prefilter(self, env, stream=None):
        G.glint_prefilter(self.ctx, env, self.ind_j, self.ind_t, self.R, self.K, self.fp, self.filt_ws,
                          self.ind_pyr, self.rgb_pyr, stream)

    def run(self, env, stream=None):
        self.partition(env, stream)
        self.prefilter(env, stream)

    def env_struct(self):
        return G.make_env(self.ind_pyr, self.rgb_pyr, self.levels, self.lut_S, self.lut_E, self.R, self.K,
                          self.M, self.dtype)


class Shader:
    """Per-pixel glint shading of a fixed G-buffer."""

    def __init__(self, ctx, gbuf: dict, seed=1, vertices=1, device="cuda"):
        self.ctx = ctx
        self.fields = {k: (v if isinstance(v, torch.Tensor) else torch.from_numpy(v)).to(device)
                       for k, v in gbuf.items()}
        if self.fields["surf_id"].dtype != torch.int32:
            self.fields["surf_id"] = self.fields["surf_id"].view(torch.int32) \
                if self.fields["surf_id"].dtype == torch.uint32 else self.fields["surf_id"].to(torch.int32)
        self.P = int(self.fields["nx"].numel())
        self.gb = G.make_gbuffer(self.fields)
        self.sp = G.ShadeParams(seed, vertices)
        self.vertices = vertices
        self.radiance = torch.empty((self.P, 3), dtype=torch.float32, device=device)

    def run(self, env: G.Env, stream=None, debug=None):
        G.glint_shade(self.ctx, self.gb, self.P, env, self.sp, self.radiance, debug, stream)


class BatchedFrame:
    """Many environments and views in one graph launch (glint_frame_batched).

    envs: list of (env tensor [6,R,R,3], K, M, T); views: list of
    (gbuf dict, env_index, seed, vertices).  Allocates every buffer once."""

    def __init__(self, ctx, envs, views, dtype=G.GLINT_F32, ell=1e-3, device="cuda"):
        self.ctx = ctx
        self.pipes, self.env_tensors = [], []
        for (env, K, M, T) in envs:
            R = int(env.shape[1])
            pipe = EnvPipeline(ctx, R, K, M, T, dtype, ell, device=device)
            pipe.build_luts()
            self.pipes.append(pipe)
            self.env_tensors.append(env)
        self.shaders = [Shader(ctx, gb, seed=seed, vertices=V, device=device) for (gb, _, seed, V) in views]
        self.env_index = [e for (_, e, _, _) in views]
        self.tasks = []
        for pipe, env in zip(self.pipes, self.env_tensors):
            self.tasks.append(G.EnvTask(env.data_ptr(), pipe.R, pipe.pp, pipe.fp, pipe.part_ws.data_ptr(),
                                        pipe.filt_ws.data_ptr(), pipe.levels.data_ptr(), pipe.ind_j.data_ptr(),
                                        pipe.ind_t.data_ptr(), pipe.ind_pyr.data_ptr(), pipe.rgb_pyr.data_ptr(),
                                        pipe.lut_S.data_ptr(), pipe.lut_E.data_ptr()))
        self.view_structs = [G.View(sh.gb, sh.P, e, sh.sp, sh.radiance.data_ptr())
                             for sh, e in zip(self.shaders, self.env_index)]
        nbytes = G.glint_batched_workspace_bytes(len(views))
        self.workspace = torch.empty(nbytes // 8 + 64, dtype=torch.float64, device=device)
        # 256-byte aligned view into the workspace
        off = (-self.workspace.data_ptr()) % 256 // 8
        self.ws = self.workspace[off:]

    @property
    def total_pixels(self):
        return sum(sh.P for sh in self.shaders)

    def run(self, stream=None):
        G.glint_frame_batched(self.ctx, self.tasks, self.view_structs, self.ws, stream)
