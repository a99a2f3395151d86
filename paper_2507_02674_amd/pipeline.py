"""Buffer management around the C ABI: one environment + one frame on one GPU.

PyTorch provides device memory and the stream; all compute is in libglint's
kernels (partition -> prefilter -> shade).  Buffers are allocated once at
construction so a frame enqueues kernels only.
"""
from __future__ import annotations

import math

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
        self.qtail = torch.empty(G.glint_quantile_table_bytes() // 8, dtype=torch.float64, device=device)

    def build_luts(self, stream=None):
        """Lookup tables once per BRDF model, and the quantile's tail table."""
        G.glint_build_luts(self.ctx, self.lut_S, self.lut_E, stream)
        G.glint_build_quantile_table(self.ctx, self.qtail, stream)

    def partition(self, env, stream=None):
        G.glint_partition_env(self.ctx, env, self.R, self.pp, self.part_ws, self.levels, self.ind_j, self.ind_t,
                              stream)

    def prefilter(self, env, stream=None):
        G.glint_prefilter(self.ctx, env, self.ind_j, self.ind_t, self.R, self.K, self.fp, self.filt_ws,
                          self.ind_pyr, self.rgb_pyr, stream)

    def run(self, env, stream=None):
        self.partition(env, stream)
        self.prefilter(env, stream)

    def env_struct(self, quantile_table=True):
        return G.make_env(self.ind_pyr, self.rgb_pyr, self.levels, self.lut_S, self.lut_E, self.R, self.K,
                          self.M, self.dtype, self.qtail if quantile_table else None)


class Shader:
    """Per-pixel glint shading of a fixed G-buffer."""

    def __init__(self, ctx, gbuf: dict, seed=1, vertices=1, device="cuda", sampler=G.GLINT_SAMPLER_DUAL,
                 prob_mode=G.GLINT_PROBS_ENV, gamma=1.0, lobe_taps=0, tree=G.GLINT_TREE_BALANCED):
        self.ctx = ctx
        self.fields = {k: (v if isinstance(v, torch.Tensor) else torch.from_numpy(v)).to(device)
                       for k, v in gbuf.items()}
        if self.fields["surf_id"].dtype != torch.int32:
            self.fields["surf_id"] = self.fields["surf_id"].view(torch.int32) \
                if self.fields["surf_id"].dtype == torch.uint32 else self.fields["surf_id"].to(torch.int32)
        self.P = int(self.fields["nx"].numel())
        self.gb = G.make_gbuffer(self.fields)
        self.sp = G.ShadeParams(seed, vertices, 0, sampler, prob_mode, gamma, lobe_taps, tree)
        self.vertices = vertices
        self.radiance = torch.empty((self.P, 3), dtype=torch.float32, device=device)

    def run(self, env: G.Env, stream=None, debug=None):
        G.glint_shade(self.ctx, self.gb, self.P, env, self.sp, self.radiance, debug, stream)


class BatchedFrame:
    """Many environments and views in one graph launch (glint_frame_batched).

    envs: list of (env tensor [6,R,R,3], K, M, T); views: list of
    (gbuf dict, env_index, seed, vertices); surrogates: optional list (one
    per environment) of Surrogate or None: views of an environment with a
    surrogate are shaded with it.  Allocates every buffer once."""

    def __init__(self, ctx, envs, views, dtype=G.GLINT_F32, ell=1e-3, device="cuda", surrogates=None):
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
        self.surrogates = list(surrogates) if surrogates is not None else [None] * len(envs)
        self.tasks = []
        for pipe, env, sur in zip(self.pipes, self.env_tensors, self.surrogates):
            self.tasks.append(G.EnvTask(env.data_ptr(), pipe.R, pipe.pp, pipe.fp, pipe.part_ws.data_ptr(),
                                        pipe.filt_ws.data_ptr(), pipe.levels.data_ptr(), pipe.ind_j.data_ptr(),
                                        pipe.ind_t.data_ptr(), pipe.ind_pyr.data_ptr(), pipe.rgb_pyr.data_ptr(),
                                        pipe.lut_S.data_ptr(), pipe.lut_E.data_ptr(), pipe.qtail.data_ptr(),
                                        sur.w.data_ptr() if sur is not None else None,
                                        sur.wb.data_ptr() if sur is not None else None))
        self.F = []
        for sh, e in zip(self.shaders, self.env_index):
            sur = self.surrogates[e]
            self.F.append(torch.empty(max(1, sh.P * sur.K), dtype=torch.float32, device=device)
                          if sur is not None else None)
        self.view_structs = [G.View(sh.gb, sh.P, e, sh.sp, sh.radiance.data_ptr(),
                                    F.data_ptr() if F is not None else None)
                             for sh, e, F in zip(self.shaders, self.env_index, self.F)]
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


class Surrogate:
    """Parameters of the learned surrogate for one environment (float32 master,
    bfloat16 copy, Adam moments) and its training loop.

    The network's layout is the C ABI's padded one (glint_surrogate_params()
    entries).  Training data come from the plain filter through
    glint_surrogate_samples; every step runs in the library's kernels."""

    HIDDEN, IN_PAD, OUT_PAD = 64, 16, 32
    LN_LO, LN_HI = math.log(0.02), math.log(0.5)

    def __init__(self, ctx, K, device="cuda"):
        self.ctx, self.K, self.device = ctx, K, device
        self.n = G.glint_surrogate_params()
        self.w = torch.zeros(self.n, dtype=torch.float32, device=device)
        self.wb = torch.zeros(self.n, dtype=torch.int16, device=device)
        self.m = torch.zeros_like(self.w)
        self.v = torch.zeros_like(self.w)
        self.step = 0
        self.loss = torch.zeros(1, dtype=torch.float32, device=device)
        self.ws = None
        self.ws_batch = 0

    # layout: W1 [64][16], b1, W2 [64][64], b2, W3 [64][64], b3, W4 [32][64], b4 [32]
    def offsets(self):
        H, I, O = self.HIDDEN, self.IN_PAD, self.OUT_PAD
        off, o = {}, 0
        for name, n in (("W1", H * I), ("b1", H), ("W2", H * H), ("b2", H), ("W3", H * H), ("b3", H),
                        ("W4", O * H), ("b4", O)):
            off[name] = (o, n)
            o += n
        return off

    def init(self, seed=7):
        """He-uniform weights (seeded, drawn on the host), zero biases."""
        gen = torch.Generator().manual_seed(seed)
        H, I, O, K = self.HIDDEN, self.IN_PAD, self.OUT_PAD, self.K
        host = torch.zeros(self.n, dtype=torch.float32)
        off = self.offsets()
        for name, (rows, fan_in, ld) in (("W1", (H, 5, I)), ("W2", (H, H, H)), ("W3", (H, H, H)),
                                         ("W4", (K, H, H))):
            lim = math.sqrt(6.0 / fan_in)
            wmat = (torch.rand((rows, fan_in), generator=gen, dtype=torch.float64) * 2.0 - 1.0) * lim
            o = off[name][0]
            view = host[o:o + off[name][1]].view(-1, ld)
            view[:rows, :fan_in] = wmat.float()
        self.load(host)

    def load(self, host_w):
        self.w.copy_(torch.as_tensor(host_w, dtype=torch.float32).reshape(-1))
        self.m.zero_()
        self.v.zero_()
        self.step = 0
        G.glint_surrogate_prepare(self.ctx, self.K, self.w, self.wb)

    def _workspace(self, batch):
        if self.ws is None or self.ws_batch < batch:
            nbytes = G.glint_surrogate_workspace_bytes(batch)
            self.ws = torch.empty(nbytes // 4 + 64, dtype=torch.float32, device=self.device)
            self.ws_batch = batch
        return self.ws

    def forward(self, x, probs=None):
        if probs is None:
            probs = torch.empty((x.shape[0], self.K), dtype=torch.float32, device=self.device)
        G.glint_surrogate_forward(self.ctx, self.K, self.w, self.wb, x, probs)
        return probs

    def gradient(self, x, target, levels=None, lam=0.0):
        """Gradient of the loss; levels (device [K] double) and lam > 0 add
        the radiance-weighted term."""
        grad = torch.empty(self.n, dtype=torch.float32, device=self.device)
        G.glint_surrogate_gradient(self.ctx, self.K, self.w, self.wb, x, target, self._workspace(x.shape[0]), grad,
                                   self.loss, levels=levels, radiance_weight=lam)
        return grad, self.loss

    def train_step(self, x, target, lr, levels=None, lam=0.0):
        self.step += 1
        G.glint_surrogate_train_step(self.ctx, self.K, self.w, self.wb, self.m, self.v, self.step, lr, x, target,
                                     self._workspace(x.shape[0]), self.loss, levels=levels, radiance_weight=lam)
        return self.loss

    @staticmethod
    def draw_lookups(n, seed, device="cuda"):
        """Random lookups: directions uniform on the sphere, ln alpha_x and
        ln alpha_y independently uniform on [ln 0.02, ln 0.5] (host-seeded)."""
        gen = torch.Generator().manual_seed(seed)
        d = torch.randn((n, 3), generator=gen, dtype=torch.float64)
        d = d / d.norm(dim=1, keepdim=True)
        la = torch.rand((n, 2), generator=gen, dtype=torch.float64) * (Surrogate.LN_HI - Surrogate.LN_LO) + \
            Surrogate.LN_LO
        a = la.exp()
        return (d.float().contiguous().to(device), a[:, 0].float().contiguous().to(device),
                a[:, 1].float().contiguous().to(device))

    def samples(self, pipe, env, n, seed):
        """Training pairs (x [n][5], target [n][K]) from the plain filter of pipe."""
        dirs, ax, ay = self.draw_lookups(n, seed, self.device)
        x = torch.empty((n, 5), dtype=torch.float32, device=self.device)
        t = torch.empty((n, self.K), dtype=torch.float32, device=self.device)
        G.glint_surrogate_samples(self.ctx, env, pipe.ind_j, pipe.ind_t, pipe.R, pipe.K, pipe.fp, pipe.filt_ws, dirs,
                                  ax, ay, x, t)
        return x, t

    def fit(self, x, t, epochs=1, batch=4096, lr=1e-3, lr_min=1e-5, seed=7, log_every=0, steps=None, levels=None,
            lam=0.0):
        """Adam over shuffled mini-batches with a cosine learning-rate
        schedule; returns the list of (step, loss) read back every
        log_every steps (the device loss is read only then).  levels and
        lam > 0: the radiance-weighted loss term."""
        n = x.shape[0]
        per_epoch = max(1, n // batch)
        total = steps if steps is not None else epochs * per_epoch
        gen = torch.Generator().manual_seed(seed)
        curve = []
        s = 0
        while s < total:
            perm = torch.randperm(n, generator=gen).to(self.device)
            xs, ts = x.index_select(0, perm), t.index_select(0, perm)
            for b in range(per_epoch):
                if s >= total:
                    break
                lr_s = lr_min + 0.5 * (lr - lr_min) * (1.0 + math.cos(math.pi * s / max(1, total)))
                self.train_step(xs[b * batch:(b + 1) * batch], ts[b * batch:(b + 1) * batch], lr_s, levels, lam)
                s += 1
                if log_every and (s % log_every == 0 or s == total):
                    curve.append((s, float(self.loss.item())))
        return curve

    # Training schedule of the surrogate workload: 2^22 filter samples, 20
    # epochs of batch 4096 (20,480 Adam steps), cosine learning rate
    # 5e-3 -> 1e-5, radiance-weighted loss term of weight 1.
    TRAIN = dict(samples=1 << 22, epochs=20, batch=4096, lr=5e-3, lr_min=1e-5, lam=1.0)
    FINE_TUNE = dict(samples=1 << 18, steps=200, batch=4096, lr=5e-4, lr_min=1e-5, lam=1.0)

    def train(self, pipe, env, seed=1, log_every=0, **over):
        """Trains on the plain filter of pipe's current map (fresh weights
        not implied: call init first).  Returns the loss curve."""
        c = dict(self.TRAIN, **over)
        x, t = self.samples(pipe, env, c["samples"], seed=seed)
        steps = c["epochs"] * max(1, c["samples"] // c["batch"])
        return self.fit(x, t, batch=c["batch"], lr=c["lr"], lr_min=c["lr_min"], steps=steps, seed=seed,
                        log_every=log_every, levels=pipe.levels, lam=c["lam"])

    def fine_tune(self, pipe, env, seed=1, **over):
        """A few Adam steps on fresh samples of pipe's current map (the
        map moved since the weights were trained): by default 200 steps
        over 2^18 samples, learning rate 5e-4 -> 1e-5."""
        c = dict(self.FINE_TUNE, **over)
        x, t = self.samples(pipe, env, c["samples"], seed=seed)
        return self.fit(x, t, batch=c["batch"], lr=c["lr"], lr_min=c["lr_min"], steps=c["steps"], seed=seed,
                        levels=pipe.levels, lam=c["lam"])

    def state(self):
        """Host copy of (w, m, v, step) for checkpoints."""
        return dict(w=self.w.cpu(), m=self.m.cpu(), v=self.v.cpu(), step=self.step, K=self.K)

    def restore(self, st):
        if int(st["K"]) != self.K:
            raise ValueError("checkpoint K does not match")
        self.w.copy_(st["w"])
        self.m.copy_(st["m"])
        self.v.copy_(st["v"])
        self.step = int(st["step"])
        G.glint_surrogate_prepare(self.ctx, self.K, self.w, self.wb)


class SurrogateShader(Shader):
    """Shading with the surrogate in place of the indicator pyramid lookup."""

    def __init__(self, ctx, gbuf: dict, surrogate: Surrogate, seed=1, vertices=1, device="cuda",
                 sampler=G.GLINT_SAMPLER_DUAL):
        super().__init__(ctx, gbuf, seed=seed, vertices=vertices, device=device, sampler=sampler)
        self.sur = surrogate
        nbytes = G.glint_shade_surrogate_workspace_bytes(self.P, surrogate.K)
        self.F = torch.empty(nbytes // 4, dtype=torch.float32, device=device)

    def run(self, env: G.Env, stream=None, debug=None):
        G.glint_shade_surrogate(self.ctx, self.gb, self.P, env, self.sur.w, self.sur.wb, self.sp, self.F,
                                self.radiance, debug, stream)


class FilterShader(Shader):
    """Shading with the plain filter evaluated at every pixel's lookup
    (glint_filter_pixels + glint_shade_given_F): no mip interpolation, the
    reference the pyramid and the surrogate are judged against."""

    def __init__(self, ctx, gbuf: dict, K, seed=1, vertices=1, device="cuda"):
        super().__init__(ctx, gbuf, seed=seed, vertices=vertices, device=device)
        self.K = K
        self.F = torch.empty((max(self.P, 1), K), dtype=torch.float32, device=device)

    def run(self, pipe: EnvPipeline, env, stream=None, debug=None):
        G.glint_filter_pixels(self.ctx, env, pipe.ind_j, pipe.ind_t, pipe.R, pipe.K, pipe.fp, pipe.filt_ws, self.gb,
                              self.P, self.F, stream)
        G.glint_shade_given_F(self.ctx, self.gb, self.P, pipe.env_struct(), self.F, self.sp, self.radiance, debug,
                              stream)


def relative_l1(a, b, mask=None):
    """Mean relative radiance error sum |a - b| / sum |b| over the masked
    pixels and the three channels (a: radiance to judge, b: reference)."""
    a, b = a.double(), b.double()
    if mask is not None:
        a, b = a[mask], b[mask]
    den = b.abs().sum()
    return float((a - b).abs().sum() / den) if float(den) > 0 else 0.0


class FramePipeline:
    """Per-frame path with the environment work of later frames overlapping
    the shading of frame f: `buffers` sets of environment buffers used in
    turn (three by default, so the environment stream can run up to two
    frames ahead), the environment kernels on one stream and shading on
    another, ordered by events (a buffer set is refilled only after the
    shading that read it).  Both streams are non-blocking pool streams: each
    frame first waits for the work already enqueued on the caller's current
    stream (the lookup tables of build_luts, the map, the G-buffer), and
    the frame's radiance is complete once s_shade reaches it.

    env_factory() -> EnvPipeline, shader: Shader or SurrogateShader."""

    def __init__(self, env_factory, shader, overlap=True, buffers=3):
        self.nbuf = max(2, buffers) if overlap else 1
        self.pipes = [env_factory() for _ in range(self.nbuf)]
        self.shader = shader
        self.overlap = overlap
        self.s_env = torch.cuda.Stream() if overlap else None
        self.s_shade = torch.cuda.Stream() if overlap else None
        self.frame = 0
        # events reused frame after frame (creating them costs host time):
        # a wait enqueued on a stream waits for the event's latest record
        self._caller_ev = torch.cuda.Event()
        self._env_done = [torch.cuda.Event() for _ in range(self.nbuf)]
        self._shade_done = [torch.cuda.Event() for _ in range(self.nbuf)]
        self._recorded = [False] * self.nbuf
        self._env_structs = [p.env_struct() for p in self.pipes]

    def build_luts(self):
        for p in self.pipes:
            p.build_luts()

    def step(self, env):
        """Enqueues one frame (no synchronisation)."""
        if not self.overlap:
            p = self.pipes[0]
            p.run(env)
            self.shader.run(p.env_struct())
            self.frame += 1
            return
        b = self.frame % self.nbuf
        p = self.pipes[b]
        # a wait that the host already sees satisfied is not enqueued: each
        # costs the queue a barrier packet
        caller = torch.cuda.current_stream()
        if not caller.query():
            self._caller_ev.record(caller)
            self.s_env.wait_event(self._caller_ev)
            self.s_shade.wait_event(self._caller_ev)
        if self._recorded[b] and not self._shade_done[b].query():
            # the buffer set is refilled only after the shading that read it
            self.s_env.wait_event(self._shade_done[b])
        # the caller may drop the map once step returns: its memory is not
        # reused before the environment stream has read it
        env.record_stream(self.s_env)
        p.run(env, stream=self.s_env)
        self._env_done[b].record(self.s_env)
        self.s_shade.wait_event(self._env_done[b])
        self.shader.run(self._env_structs[b], stream=self.s_shade)
        self._shade_done[b].record(self.s_shade)
        self._recorded[b] = True
        self.frame += 1

    def streams(self):
        return [self.s_env, self.s_shade] if self.overlap else [torch.cuda.current_stream()]

    def last_env(self):
        return self.pipes[(self.frame - 1) % len(self.pipes)]


# --- surrogate checkpoints ---------------------------------------------------------

CKPT_MAGIC = b"GLSGCKPT"
CKPT_VERSION = 1


def pack_checkpoint(w, m, v, step: int, K: int) -> bytes:
    """Versioned binary of the surrogate's training state: header (magic,
    version, K, parameter count, step, dtype code 0 = float32), then the
    float32 master weights and the two Adam moments, then a CRC32 of
    everything before it."""
    import struct
    import zlib

    import numpy as np
    arrs = [np.ascontiguousarray(np.asarray(a, dtype=np.float32)).reshape(-1) for a in (w, m, v)]
    n = arrs[0].size
    if any(a.size != n for a in arrs):
        raise ValueError("weights and moments differ in size")
    body = CKPT_MAGIC + struct.pack("<IIIqI", CKPT_VERSION, K, n, step, 0) + b"".join(a.tobytes() for a in arrs)
    return body + struct.pack("<I", zlib.crc32(body) & 0xFFFFFFFF)


def unpack_checkpoint(blob: bytes) -> dict:
    """Inverse of pack_checkpoint; raises ValueError on a bad magic, version,
    size or CRC."""
    import struct
    import zlib

    import numpy as np
    head = len(CKPT_MAGIC) + struct.calcsize("<IIIqI")
    if len(blob) < head + 4 or blob[:len(CKPT_MAGIC)] != CKPT_MAGIC:
        raise ValueError("not a surrogate checkpoint")
    version, K, n, step, dtype = struct.unpack("<IIIqI", blob[len(CKPT_MAGIC):head])
    if version != CKPT_VERSION or dtype != 0:
        raise ValueError(f"unsupported checkpoint version {version} / dtype {dtype}")
    if len(blob) != head + 3 * 4 * n + 4:
        raise ValueError("checkpoint size does not match its header")
    (crc,) = struct.unpack("<I", blob[-4:])
    if zlib.crc32(blob[:-4]) & 0xFFFFFFFF != crc:
        raise ValueError("checkpoint CRC mismatch")
    arr = np.frombuffer(blob, dtype=np.float32, count=3 * n, offset=head).reshape(3, n)
    return dict(w=arr[0].copy(), m=arr[1].copy(), v=arr[2].copy(), step=int(step), K=int(K))


def save_surrogate(sur: "Surrogate", path: str) -> None:
    st = sur.state()
    blob = pack_checkpoint(st["w"].numpy(), st["m"].numpy(), st["v"].numpy(), st["step"], st["K"])
    with open(path, "wb") as f:
        f.write(blob)


def load_surrogate(sur: "Surrogate", path: str) -> None:
    with open(path, "rb") as f:
        st = unpack_checkpoint(f.read())
    sur.restore({k: (torch.from_numpy(val) if hasattr(val, "dtype") else val) for k, val in st.items()})


# --- surrogate fallback -----------------------------------------------------------

class GuardedShader:
    """Surrogate shading with a fallback to the plain form: every `every`
    frames the network's F_k/sum F on a fixed probe set of lookups is
    compared with the plain filter of the current map (glint_surrogate_samples
    and glint_surrogate_forward); while the mean absolute error exceeds
    `threshold` the plain shader (indicator pyramid) is used."""

    def __init__(self, surrogate_shader: "SurrogateShader", plain_shader: Shader, probe=4096, every=8,
                 threshold=0.02, seed=99):
        self.sur_sh, self.plain_sh = surrogate_shader, plain_shader
        self.sur = surrogate_shader.sur
        self.every, self.threshold = every, threshold
        self.dirs, self.ax, self.ay = Surrogate.draw_lookups(probe, seed, surrogate_shader.radiance.device)
        K = self.sur.K
        self.x = torch.empty((probe, 5), dtype=torch.float32, device=self.dirs.device)
        self.t = torch.empty((probe, K), dtype=torch.float32, device=self.dirs.device)
        self.y = torch.empty((probe, K), dtype=torch.float32, device=self.dirs.device)
        self.frame = 0
        self.use_surrogate = True
        self.last_error = None

    def check(self, pipe: EnvPipeline, env, stream=None) -> float:
        G.glint_surrogate_samples(self.sur.ctx, env, pipe.ind_j, pipe.ind_t, pipe.R, pipe.K, pipe.fp, pipe.filt_ws,
                                  self.dirs, self.ax, self.ay, self.x, self.t, stream)
        G.glint_surrogate_forward(self.sur.ctx, self.sur.K, self.sur.w, self.sur.wb, self.x, self.y, stream)
        err = float((self.y - self.t).abs().mean().item())
        self.last_error = err
        self.use_surrogate = err <= self.threshold
        return err

    @property
    def radiance(self):
        return self.sur_sh.radiance if self.use_surrogate else self.plain_sh.radiance

    def run(self, pipe: EnvPipeline, env, stream=None):
        if self.frame % self.every == 0:
            self.check(pipe, env, stream)
        self.frame += 1
        if self.use_surrogate:
            self.sur_sh.run(pipe.env_struct(), stream)
        else:
            self.plain_sh.run(pipe.env_struct(), stream)
