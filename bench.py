"""Benchmark of the glint hot path on one MI355X.

A step is one frame of the whole per-frame path on the frame workload:
environment partition (luminance min/max, radiance levels, fuzzy
indicators), source mip chain, NDF prefilter of the K indicator channels and
RGB into the roughness pyramid, then glint shading of the 1920x1080 G-buffer
(N_P, reflection probabilities, dual-gated multinomial, radiance).  The
lookup tables are built once per BRDF model before timing (not per frame).
Inputs are synthetic and resident in HBM before the timed region.

Forms: ``plain`` (the paper's method), ``surrogate`` (the indicator lookup
replaced by the learned network; trained before the timed region, its
training step timed separately).  ``--dtype`` selects the indicator
pyramid's storage type.  ``--workload batched`` times the 64-view graph.

Frames run back to back with the environment work of frame f+1 overlapping
the shading of frame f (two buffer sets, two streams; `--no-overlap` runs
them serially); every frame does the whole path.

Prints one JSON line: value = glint-shaded Mpix/s (pixels that ran the glint
shader, per second of wall time over the timed frames), prefilter ms/frame
and per-kernel durations from a serial pass, per-kernel average durations of
the roofline kernels inside the timed region (HIP events carried by their
dispatches), the roofline record of the dominant kernel and the CPU-oracle
baseline.  The cost model (algorithmic operations and bytes per unit of
work) is in the functions below.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

METRIC = "glint-shaded Mpix/s + env prefilter ms/frame; surrogate/FP16 vs plain, 1 GPU"
HBM_PEAK_GBS = 8000.0
# Peak VALU lane-operations per second: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
# (one wave64 VALU instruction per SIMD every 4 cycles).  Double FMA issues at
# this rate on this part, as does non-packed float.
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
BF16_MFMA_PEAK_TFLOPS = 2500.0
STORAGE_BYTES = {"f32": 4, "f16": 2, "bf16": 2, "unorm16": 2}


# --- cost model ---------------------------------------------------------------------

def filter_taps(R, M, T, alpha):
    """(weight > 0, lod) of the T taps of the filter at roughness alpha (the
    quadrature's tap table: GGX half vectors from a Hammersley set, weight
    <r, l>+, filtered-importance-sampling lod)."""
    j = np.arange(T)
    rev = np.array([int(format(int(i), "032b")[::-1], 2) for i in j], dtype=np.float64) / 2.0 ** 32
    a2 = alpha * alpha
    c2 = (1.0 - rev) / (1.0 + (a2 - 1.0) * rev)
    w = np.maximum(0.0, 2.0 * c2 - 1.0)
    den = 1.0 + (a2 - 1.0) * c2
    D = a2 / (math.pi * den * den)
    with np.errstate(divide="ignore"):
        lod = 0.5 * np.log2((4.0 / (T * D)) / (4.0 * math.pi / (6.0 * R * R))) + 1.0
    return w > 0, np.clip(lod, 0.0, M - 1)


# Per tap: rotate the half vector into the texel's frame (9 FMA), mirror
# (6), face select and projection (~12), bilinear coordinates and weights
# (~12 per level).
TAP_FIXED_OPS = 27
TAP_LEVEL_OPS = 12


def prefilter_cost(R, M, T, K, dtype_bytes=4):
    """Algorithmic VALU lane-ops and HBM bytes of one k_prefilter launch
    (mips 1..M-1): per output texel and effective tap (weight > 0), a
    weighted sum of the C = K+3 channels of 4 texels on each of the one or
    two chain levels the tap's lod touches (one FMA per channel and texel),
    plus the tap's direction work; then C normalisations.  Bytes: the
    pyramid written (K indicator values of the stored type + 4 RGB floats
    per texel) and the stored source chain (levels >= 1 with their border
    rings, 16-byte-padded records) read once."""
    C = K + 3
    ops = 0.0
    texels = 0
    for m in range(1, M):
        n = R >> m
        eff, lod = filter_taps(R, M, T, (m / (M - 1)) ** 2)
        levels = np.where(lod > np.floor(lod), 2, 1)[eff]
        per_texel = float(np.sum(levels * (4 * C + TAP_LEVEL_OPS) + TAP_FIXED_OPS)) + C
        ops += 6 * n * n * per_texel
        texels += 6 * n * n
    chain_records = sum(6 * ((R >> s) + 2) ** 2 for s in range(1, M))
    bytes_ = texels * (K * dtype_bytes + 16) + chain_records * 4 * ((C + 3) // 4 * 4)
    return ops, bytes_, texels


def shade_ops_per_pixel(K, V=1):
    """Algorithmic VALU lane-ops per glint pixel (transcendentals weighted 4,
    their issue cost at quarter rate):
      set-up: N_P, reflection, lod, lattice level ~ 25;
      lookup: 2 levels x 4 texels x (K+3) channel FMAs + addressing ~ 40;
      p_k and three LUT bilinears: 2K + 30;
      per lattice vertex and tree node: hash 16 + xi 4, gating thresholds
        15 + 2 pow (2 transcendentals each), AS 241 quantile ~ 30 (one
        division), Gaussian and masks 15 -> 80 + 5 transcendentals;
      combine: 2K + 15 per vertex, radiance 10."""
    node = 80 + 4 * 5
    return float(25 + 8 * (K + 3) + 40 + 2 * K + 30 + V * ((K - 1) * node + 2 * K + 15) + 10)


SHADE_BYTES_PER_PIXEL = 16 * 4 + 12  # G-buffer fields + radiance


def mlp_flops_per_row(K, padded=False):
    """Matrix-core flops of one network evaluation: 2 x (5x64 + 64x64 + 64x64
    + 64xK) multiply-adds (unpadded), or the padded tiles the kernel issues
    (16-wide input, 32-wide output)."""
    if padded:
        return 2.0 * (16 * 64 + 2 * 64 * 64 + 64 * 32)
    return 2.0 * (5 * 64 + 2 * 64 * 64 + 64 * K)


# --- measured HBM traffic ---------------------------------------------------------

ROOT = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = {"k_prefilter": ("prefilter.hip", "device.hpp"), "k_shade": ("shade.hip", "device.hpp"),
                  "k_shade_surrogate": ("shade.hip", "device.hpp"), "k_mlp_lookup": ("mlp.hip", "device.hpp")}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "frame_hbm_counters.md")


def kernel_source_hash(kernel):
    """Short hash of the sources a kernel is built from (to tell whether
    recorded counters still describe the built kernel)."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel]:
        with open(os.path.join(ROOT, "paper_2507_02674_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def recorded_traffic(kernel, config_tag):
    """HBM bytes per launch of `kernel` on configuration `config_tag` from the
    counter summary (FETCH_SIZE and WRITE_SIZE, scaled by a plain copy of
    known size), or None if absent or recorded for other kernel sources."""
    import re
    try:
        text = open(TRAFFIC_FILE).read()
    except OSError:
        return None
    for m in re.finditer(r"^traffic (\S+) (\S+) bytes=(\d+) sources=([0-9a-f]+)$", text, re.M):
        if m.group(1) == kernel and m.group(2) == config_tag and m.group(4) == kernel_source_hash(kernel):
            return int(m.group(3))
    return None


# --- helpers -------------------------------------------------------------------------

SAMPLERS = {"dual": 0, "single": 1, "single-floor": 2}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=100,
                    help="untimed frames first (the GPU reaches its steady clocks after ~50 ms of work)")
    ap.add_argument("--workload", default="frame")
    ap.add_argument("--form", default="plain", choices=["plain", "surrogate"])
    ap.add_argument("--dtype", default="f32", choices=["f32", "f16", "bf16", "unorm16"])
    ap.add_argument("--vertices", type=int, default=1, choices=[1, 6, 12],
                    help="lattice vertices per pixel: 1, 6 (uv triangle x 2 scales) or 12 (footprint grid)")
    ap.add_argument("--sampler", default="dual", choices=list(SAMPLERS),
                    help="binomial approximation at every tree node (dual-gated is the paper's method)")
    ap.add_argument("--probs", default="env", choices=["env", "constant"],
                    help="reflection probabilities from the map (the paper) or one constant for every facet")
    ap.add_argument("--gamma", type=float, default=0.05, help="the constant probability of --probs constant")
    ap.add_argument("--lobe-taps", type=int, default=0, choices=[0, 2, 4, 8],
                    help="anisotropic lookup with this many taps along the lobe (0: one lookup)")
    ap.add_argument("--visibility", default="none", choices=["none", "contact"],
                    help="occlusion that attenuates the probabilities (contact: the scene's AO-like field)")
    ap.add_argument("--train-epochs", type=int, default=20,
                    help="surrogate training epochs over 2^22 filter samples (batch 4096) before timing")
    ap.add_argument("--rotate-frames", type=int, default=8,
                    help="surrogate form: frames of the rotating-sun study after the timed region (frozen, "
                         "fine-tuned and retrained network against the plain filter)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--env", default="dynamic", choices=["dynamic", "static"],
                    help="dynamic: the map is partitioned and prefiltered every frame (the headline); static: "
                         "prefiltered once, frames shade only (the paper's two runtime scenarios)")
    ap.add_argument("--buffers", type=int, default=3,
                    help="environment buffer sets of the overlapped frame pipeline (the environment work runs "
                         "up to buffers - 1 frames ahead of the shading)")
    ap.add_argument("--no-overlap", action="store_true",
                    help="run frames back to back on one stream (no environment/shading overlap)")
    ap.add_argument("--cpu-sample", type=float, default=1.0 / 48.0,
                    help="fraction of pyramid texels and glint pixels the oracle times")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (calibrates HBM byte counters)")
    return ap.parse_args()


def copy_probe(mib: int) -> None:
    """A plain device-to-device copy of known size, to scale the FETCH_SIZE /
    WRITE_SIZE counters of the same profiler pass."""
    import torch
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_mib": mib, "launches": 3}), flush=True)


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_share() -> int:
    """Host threads this process may use: OMP_NUM_THREADS when set (the
    process's CPU share), else the visible CPUs."""
    try:
        n = int(os.environ.get("OMP_NUM_THREADS", "0"))
    except ValueError:
        n = 0
    if n <= 0:
        try:
            n = len(os.sched_getaffinity(0))
        except AttributeError:
            n = os.cpu_count() or 1
    return max(1, n)


def cpu_baseline(w, env, gbuf, glint_pixels, frac, shade_inputs):
    """Times the oracle (as it stands) on a stratified sample of the same
    frame, once on one thread and once on every thread of the process's CPU
    share, and scales to Mpix/s of whole frames.  shade_inputs: the frame's
    pyramid, levels and LUTs (host copies), so the sampled pixels shade real
    values."""
    share = cpu_share()
    multi = cpu_baseline_leg(w, env, gbuf, glint_pixels, frac, shade_inputs, share)
    single = cpu_baseline_leg(w, env, gbuf, glint_pixels, frac, shade_inputs, 1)
    multi["single_thread"] = {k: single[k] for k in ("value", "cores", "prefilter_s_per_frame",
                                                      "shade_s_per_frame")}
    multi["cpu_model"] = cpu_model()
    multi["host_cpus_visible"] = os.cpu_count()
    return multi


def cpu_baseline_leg(w, env, gbuf, glint_pixels, frac, shade_inputs, threads, reps=3):
    """One leg of the CPU baseline: each timed stage is the best of `reps`
    runs (the first call of a stage pays one-off costs: thread start-up,
    first touch of the inputs, which the sample's scaling would multiply)."""
    import oracle

    def best(fn):
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            r = fn()
            ts.append(time.perf_counter() - t0)
        return min(ts), r

    t_part, (levels, ij, it, chain) = best(lambda: (lambda l, j, t: (l, j, t, oracle.mipchain(env, j, t, w.K, w.M)))(
        *oracle.partition(env, w.K, w.ell)))
    n_tex = oracle.pyramid_texels(w.R, w.M)
    step = max(1, int(round(1.0 / frac)))
    tex = np.arange(0, n_tex, step, dtype=np.int64)
    t_pre, _ = best(lambda: oracle.prefilter(env, ij, it, chain, w.K, w.M, w.T, texel_ids=tex, threads=threads))
    t_pre *= n_tex / len(tex)
    ind, rgb, lv, lut_S, lut_E = shade_inputs
    hit = np.nonzero(gbuf["surf_id"] != 0xFFFFFFFF)[0]
    pix = hit[::step]
    t_sh, _ = best(lambda: oracle.shade(gbuf, ind, rgb, lv, lut_S, lut_E, w.R, w.K, w.M, w.hash_seed, 1, pixels=pix,
                                        threads=threads))
    t_sh *= len(hit) / len(pix)
    frame_s = t_part + t_pre + t_sh
    return {"value": glint_pixels / frame_s / 1e6, "unit": "Mpix/s", "cores": threads, "kind": "oracle",
            "sample": f"full partition + mip chain; every {step}th pyramid texel ({len(tex)}) and every {step}th "
                      f"glint pixel ({len(pix)}) timed (best of {reps} runs per stage), scaled to the whole "
                      f"frame; oracle frame time {frame_s:.2f} s (prefilter {t_part + t_pre:.2f} s, shade "
                      f"{t_sh:.2f} s)",
            "prefilter_s_per_frame": t_part + t_pre, "shade_s_per_frame": t_sh}


WARMUP_MIN_S = 0.1


def warm_up(step, frames, torch):
    """Untimed frames before the timed region: the requested number, and
    more until WARMUP_MIN_S of wall time has passed (the GPU needs ~50 ms
    of work to reach its steady clocks; a few frames of a fraction of a
    millisecond leave the timed region at ramping clocks).  Returns the
    number of frames run."""
    t0 = time.perf_counter()
    n = 0
    while n < frames or time.perf_counter() - t0 < WARMUP_MIN_S:
        step()
        n += 1
        if n >= frames and n % 8 == 0:
            torch.cuda.synchronize()  # the wall clock then measures finished work
    torch.cuda.synchronize()
    return n


def kernel_table(G, ctx, steps):
    prof = G.glint_profile_collect(ctx)
    return {k: {"avg_ms": round(ms / n, 5), "launches_per_step": n / steps} for k, (ms, n) in prof.items()}


def alu_record(kernel, ops, avg_ms, extra=None, config_tag=None):
    achieved = ops / (avg_ms * 1e-3) / 1e12
    r = {"bound": "alu", "kernel": kernel, "achieved": round(achieved, 3), "peak": round(VALU_PEAK_TOPS, 4),
         "unit": "TOP/s (VALU lane-ops)", "frac": round(achieved / VALU_PEAK_TOPS, 4),
         "traffic": recorded_traffic(kernel, config_tag) if config_tag else None, "ops_per_launch": ops}
    if extra:
        r.update(extra)
    return r


def batched(a):
    """64 views of uneven size over 4 maps (K = 4, 8, 16, 8), one graph
    launch per frame (glint_frame_batched)."""
    import torch

    import synth
    from paper_2507_02674_amd import glint as G
    from paper_2507_02674_amd.pipeline import BatchedFrame

    views = synth.batched_views(64)
    envs = [(torch.from_numpy(synth.make_env(256, seed)).cuda(), K, 8, 64) for (seed, K) in synth.BATCHED_ENVS]
    ctx = G.glint_create(0)
    surrogates, train_info = None, None
    if a.form == "surrogate":
        from paper_2507_02674_amd.pipeline import EnvPipeline
        surrogates, train_info = [], []
        for (env, K, M, T) in envs:
            pipe = EnvPipeline(ctx, int(env.shape[1]), K, M, T)
            pipe.build_luts()
            pipe.run(env)
            sur, info = train_surrogate(G, ctx, pipe, env, K, a.train_epochs)
            surrogates.append(sur)
            train_info.append(info)
    bf = BatchedFrame(ctx, envs, views, surrogates=surrogates)
    glint_pixels = sum(int((gb["surf_id"] != 0xFFFFFFFF).sum()) for (gb, _, _, _) in views)
    bf.run()  # set-up call (autotune + capture)
    torch.cuda.synchronize()
    warm = warm_up(bf.run, a.warmup, torch)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    for _ in range(a.steps):
        bf.run()
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = max(e0.elapsed_time(e1) / a.steps, 1e3 * wall / a.steps)
    out = {"metric": METRIC, "value": round(glint_pixels / (ms * 1e-3) / 1e6, 3), "unit": "Mpix/s", "n_gpus": 1,
           "steps": a.steps, "warmup": a.warmup, "warmup_frames_run": warm, "ms_per_step": round(ms, 4),
           "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "batched: 64 views (256^2..1920x1080, log-uniform pixels), 4 cube maps "
                                  "6x256x256 with K=4,8,16,8, M=8, T=64; one graph launch per frame",
                      "form": a.form, "views": len(views), "total_pixels": bf.total_pixels,
                      "glint_pixels": glint_pixels, "tile_px": G.glint_batched_tile_px(ctx)}}
    if train_info is not None:
        out["surrogate"] = train_info
    G.glint_destroy(ctx)
    print(json.dumps(out), flush=True)


def train_surrogate(G, ctx, pipe, env, K, epochs, batch=4096):
    """Trains the surrogate on the plain filter of the current map with the
    workload's schedule (2^22 samples, `epochs` epochs, not timed as part of
    a frame); then times training steps on their own."""
    import torch
    from paper_2507_02674_amd.pipeline import Surrogate
    sur = Surrogate(ctx, K)
    sur.init(seed=7)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    curve = sur.train(pipe, env, epochs=epochs, log_every=2048)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    steps = sur.step
    xv, tv = sur.samples(pipe, env, 1 << 14, seed=2)
    loss = float(sur.gradient(xv, tv, pipe.levels, Surrogate.TRAIN["lam"])[1].item())
    err = float((sur.forward(xv) - tv).abs().mean().item())
    # training-step throughput (b7): 50 steps at the training batch
    xs, ts = xv[:batch].contiguous(), tv[:batch].contiguous()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(50):
        sur.train_step(xs, ts, 1e-5, pipe.levels, Surrogate.TRAIN["lam"])
    e1.record()
    torch.cuda.synchronize()
    step_ms = e0.elapsed_time(e1) / 50
    flops = 3.0 * mlp_flops_per_row(K) * batch
    info = {"train_steps": steps, "batch": batch, "schedule": dict(Surrogate.TRAIN, epochs=epochs),
            "train_s": round(train_s, 3), "loss_curve": [(st, round(l, 5)) for st, l in curve],
            "heldout_loss": round(loss, 5), "heldout_mean_abs_F_err": err,
            "train_step_ms": round(step_ms, 4), "train_samples_per_s": round(batch / (step_ms * 1e-3), 1),
            "train_tflops_algorithmic": round(flops / (step_ms * 1e-3) / 1e12, 3)}
    return sur, info


ACCURACY_METRIC = ("mean relative radiance error: sum |L - L_ref| / sum |L_ref| over the glint pixels and the RGB "
                   "channels, same hash draws; L_ref shaded with the plain filter evaluated at each pixel's "
                   "lookup (glint_filter_pixels, no mip interpolation)")


def filter_accuracy(G, ctx, w, pipe, env, gbuf_np, shader, envs):
    """The form under test and the plain f32 pyramid, each against shading
    with the plain filter at every pixel's lookup."""
    import torch
    from paper_2507_02674_amd.pipeline import EnvPipeline, FilterShader, Shader, relative_l1
    g = {k: v for k, v in gbuf_np.items() if k not in G.GBUF_OPTIONAL}
    ref = FilterShader(ctx, g, w.K, seed=w.hash_seed)
    f32 = EnvPipeline(ctx, w.R, w.K, w.M, w.T, G.GLINT_F32, w.ell)
    f32.build_luts()
    f32.run(env)
    ref.run(f32, env)
    pyr = Shader(ctx, g, seed=w.hash_seed)
    pyr.run(f32.env_struct())
    shader.run(envs)
    torch.cuda.synchronize()
    hit = torch.from_numpy(gbuf_np["surf_id"] != 0xFFFFFFFF).cuda()
    return {"metric": ACCURACY_METRIC,
            "form_vs_filter": relative_l1(shader.radiance, ref.radiance, hit),
            "pyramid_f32_vs_filter": relative_l1(pyr.radiance, ref.radiance, hit),
            "form_vs_pyramid_f32": relative_l1(shader.radiance, pyr.radiance, hit)}


def rotating_study(G, ctx, w, env_np, gbuf_np, sur, frames, epochs):
    """Rotating suns (sun s's azimuth +2 (s+1) degrees per frame): per
    frame, the network trained on frame 0 (frozen), the same network
    fine-tuned frame after frame (200 steps on 2^18 fresh samples of each
    frame's filter) and the f32 pyramid, each against the plain filter of
    that frame; at the last frame also a network retrained from scratch."""
    import torch
    import synth
    from paper_2507_02674_amd.pipeline import (EnvPipeline, FilterShader, Shader, Surrogate, SurrogateShader,
                                               relative_l1)
    g = {k: v for k, v in gbuf_np.items() if k not in G.GBUF_OPTIONAL}
    hit = torch.from_numpy(gbuf_np["surf_id"] != 0xFFFFFFFF).cuda()
    frozen = Surrogate(ctx, w.K)
    frozen.restore(sur.state())
    tuned = Surrogate(ctx, w.K)
    tuned.restore(sur.state())
    pipe = EnvPipeline(ctx, w.R, w.K, w.M, w.T, G.GLINT_F32, w.ell)
    pipe.build_luts()
    ref = FilterShader(ctx, g, w.K, seed=w.hash_seed)
    pyr = Shader(ctx, g, seed=w.hash_seed)
    sh_frozen = SurrogateShader(ctx, g, frozen, seed=w.hash_seed)
    sh_tuned = SurrogateShader(ctx, g, tuned, seed=w.hash_seed)
    rows, tune_ms = [], []
    for f in range(1, frames + 1):
        env = torch.from_numpy(synth.make_env(w.R, w.env_seed, frame=f)).cuda()
        pipe.run(env)
        ref.run(pipe, env)
        pyr.run(pipe.env_struct())
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        tuned.fine_tune(pipe, env, seed=100 + f)
        torch.cuda.synchronize()
        tune_ms.append(1e3 * (time.perf_counter() - t0))
        sh_frozen.run(pipe.env_struct())
        sh_tuned.run(pipe.env_struct())
        torch.cuda.synchronize()
        rows.append({"frame": f, "frozen": relative_l1(sh_frozen.radiance, ref.radiance, hit),
                     "fine_tuned": relative_l1(sh_tuned.radiance, ref.radiance, hit),
                     "pyramid_f32": relative_l1(pyr.radiance, ref.radiance, hit)})
    fresh = Surrogate(ctx, w.K)
    fresh.init(seed=7)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fresh.train(pipe, env, epochs=epochs)
    torch.cuda.synchronize()
    retrain_s = time.perf_counter() - t0
    sh_fresh = SurrogateShader(ctx, g, fresh, seed=w.hash_seed)
    sh_fresh.run(pipe.env_struct())
    torch.cuda.synchronize()
    mean = lambda k: float(np.mean([r[k] for r in rows]))
    return {"metric": ACCURACY_METRIC, "frames": rows,
            "mean": {k: mean(k) for k in ("frozen", "fine_tuned", "pyramid_f32")},
            "fine_tune": dict(Surrogate.FINE_TUNE, ms_per_frame=round(float(np.mean(tune_ms)), 2)),
            "retrained_last_frame": {"vs_filter": relative_l1(sh_fresh.radiance, ref.radiance, hit),
                                     "train_s": round(retrain_s, 3), "epochs": epochs}}


def roofline_records(kernels, w, a, shader, glint_pixels, config_tag):
    """Roofline record per timed kernel (cost model of this file over the
    kernel's average launch duration)."""
    pf_ops, pf_bytes, pf_texels = prefilter_cost(w.R, w.M, w.T, w.K, STORAGE_BYTES[a.dtype])
    records = {}
    if "k_prefilter" in kernels:
        ms = kernels["k_prefilter"]["avg_ms"]
        records["k_prefilter"] = alu_record("k_prefilter", pf_ops, ms, {
            "ops_per_texel": round(pf_ops / pf_texels, 1), "output_texels": pf_texels,
            "algorithmic_bytes": pf_bytes, "hbm_gbs": round(pf_bytes / (ms * 1e-3) / 1e9, 1),
            "hbm_frac": round(pf_bytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}, config_tag)
    shade_kernel = "k_shade_surrogate" if a.form == "surrogate" else "k_shade"
    if shade_kernel in kernels:
        ms = kernels[shade_kernel]["avg_ms"]
        opp = shade_ops_per_pixel(w.K, a.vertices)
        records[shade_kernel] = alu_record(shade_kernel, opp * glint_pixels, ms, {
            "ops_per_pixel": opp, "algorithmic_bytes": SHADE_BYTES_PER_PIXEL * shader.P,
            "hbm_gbs": round(SHADE_BYTES_PER_PIXEL * shader.P / (ms * 1e-3) / 1e9, 1),
            "hbm_frac": round(SHADE_BYTES_PER_PIXEL * shader.P / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}, config_tag)
    if "k_mlp_lookup" in kernels:
        ms = kernels["k_mlp_lookup"]["avg_ms"]
        fl = mlp_flops_per_row(w.K) * shader.P
        ach = fl / (ms * 1e-3) / 1e12
        records["k_mlp_lookup"] = {"bound": "mfma", "kernel": "k_mlp_lookup", "achieved": round(ach, 3),
                                   "peak": BF16_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                                   "traffic": recorded_traffic("k_mlp_lookup", config_tag),
                                   "frac": round(ach / BF16_MFMA_PEAK_TFLOPS, 4), "flops_per_launch": fl,
                                   "padded_flops_per_launch": mlp_flops_per_row(w.K, True) * shader.P}
    return records


def main():
    a = parse()
    if a.copy_probe:
        copy_probe(a.copy_probe)
        return
    if a.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; multi-GPU runs are not part of it",
                          "n_gpus": a.gpus}))
        sys.exit(2)
    import torch

    import synth
    from paper_2507_02674_amd import glint as G
    from paper_2507_02674_amd.pipeline import EnvPipeline, FramePipeline, Shader, SurrogateShader

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(1)
    if a.workload == "batched":
        batched(a)
        return
    dtypes = {"f32": G.GLINT_F32, "f16": G.GLINT_F16, "bf16": G.GLINT_BF16, "unorm16": G.GLINT_UNORM16}
    w = synth.WORKLOADS[a.workload]
    env_np, gbuf_np = w.env(), w.gbuf()
    if a.visibility == "contact":
        gbuf_np["visibility"] = synth.contact_visibility(gbuf_np)
    if a.lobe_taps:
        gbuf_np["tx"], gbuf_np["ty"], gbuf_np["tz"] = synth.surface_tangents(gbuf_np)
    if a.vertices == 12:
        gbuf_np["dudx"], gbuf_np["dudy"], gbuf_np["dvdx"], gbuf_np["dvdy"] = synth.uv_jacobian(gbuf_np, w.W, w.H)
    prob_mode = G.GLINT_PROBS_CONSTANT if a.probs == "constant" else G.GLINT_PROBS_ENV
    default_path = a.sampler == "dual" and a.probs == "env" and a.visibility == "none" and a.lobe_taps == 0
    glint_pixels = int((gbuf_np["surf_id"] != 0xFFFFFFFF).sum())
    ctx = G.glint_create(0)
    env = torch.from_numpy(env_np).cuda()

    def new_env(dtype=a.dtype):
        return EnvPipeline(ctx, w.R, w.K, w.M, w.T, dtypes[dtype], w.ell)

    pipe = new_env()  # the serial pass's buffers (also the surrogate's training source)
    pipe.build_luts()
    pipe.run(env)
    extra = {}
    if a.form == "surrogate":
        sur, extra["surrogate"] = train_surrogate(G, ctx, pipe, env, w.K, a.train_epochs)
        shader = SurrogateShader(ctx, gbuf_np, sur, seed=w.hash_seed, vertices=a.vertices,
                                 sampler=SAMPLERS[a.sampler])
    else:
        shader = Shader(ctx, gbuf_np, seed=w.hash_seed, vertices=a.vertices, sampler=SAMPLERS[a.sampler],
                        prob_mode=prob_mode, gamma=a.gamma, lobe_taps=a.lobe_taps)
    if a.env == "static":
        # the map is prefiltered once (above); a frame is the shading launch
        class _Static:
            def step(self, _env):
                shader.run(pipe.env_struct())
        frames = _Static()
    else:
        frames = FramePipeline(new_env, shader, overlap=not a.no_overlap, buffers=a.buffers)
        frames.build_luts()
    warm = warm_up(lambda: frames.step(env), a.warmup, torch)

    # timed region: K frames, each the whole per-frame path; with overlap the
    # environment work of frame f+1 runs beside the shading of frame f.  The
    # roofline kernels carry HIP events in their dispatches.
    timed = ["k_prefilter", "k_mlp_lookup", "k_shade_surrogate"] if a.form == "surrogate" else ["k_prefilter", "k_shade"]
    G.glint_profile_select(ctx, timed)
    G.glint_profile_enable(ctx, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        frames.step(env)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kernels = kernel_table(G, ctx, a.steps)
    G.glint_profile_enable(ctx, False)
    ms_per_step = 1e3 * wall / a.steps
    value = glint_pixels / (ms_per_step * 1e-3) / 1e6

    # serial reference pass (not the timed region): one stream, every kernel
    # timed, environment and shading bracketed separately
    G.glint_profile_select(ctx, None)
    G.glint_profile_enable(ctx, True)
    envs = pipe.env_struct()
    n_ser = max(5, min(a.steps, 20))
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(n_ser)]
    torch.cuda.synchronize()
    for s in range(n_ser):
        ev[s][0].record()
        pipe.run(env)
        ev[s][1].record()
        shader.run(envs)
        ev[s][2].record()
    torch.cuda.synchronize()
    kernels_serial = kernel_table(G, ctx, n_ser)
    G.glint_profile_enable(ctx, False)
    pre_ms = float(np.mean([e[0].elapsed_time(e[1]) for e in ev]))
    sh_ms = float(np.mean([e[1].elapsed_time(e[2]) for e in ev]))
    serial_ms = float(ev[0][0].elapsed_time(ev[-1][2])) / n_ser

    config_tag = f"{w.name}-{a.form}-{a.dtype}-v{a.vertices}" + (
        "" if default_path else f"-{a.sampler}-{a.probs}-{a.visibility}-t{a.lobe_taps}")
    records = roofline_records(kernels, w, a, shader, glint_pixels, config_tag)
    dominant = max(records, key=lambda k: kernels[k]["avg_ms"] * kernels[k]["launches_per_step"])
    roofline = dict(records[dominant])
    others = {k: v for k, v in records.items() if k != dominant}
    serial_records = roofline_records(kernels_serial, w, a, shader, glint_pixels, config_tag)

    out = {"metric": METRIC, "value": round(value, 3), "unit": "Mpix/s", "n_gpus": 1, "steps": a.steps,
           "warmup": a.warmup, "warmup_frames_run": warm, "ms_per_step": round(ms_per_step, 4),
           "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"{w.name}: {w.W}x{w.H} sphere+plane G-buffer, cube map 6x{w.R}x{w.R}, "
                                  f"{w.M} mips, K={w.K}, T={w.T} taps, " +
                                  ("per-frame partition+prefilter+shade" if a.env == "dynamic"
                                   else "map prefiltered once, per-frame shade"),
                      "env": a.env,
                      "form": a.form, "pyramid_dtype": a.dtype, "vertices": a.vertices, "sampler": a.sampler,
                      "probs": a.probs if a.probs == "env" else f"constant gamma={a.gamma}",
                      "visibility": a.visibility, "lobe_taps": a.lobe_taps,
                      "glint_pixels": glint_pixels, "total_pixels": shader.P,
                      "frames_overlapped": a.env == "dynamic" and not a.no_overlap},
           "prefilter_ms_per_frame": round(pre_ms, 4), "shade_ms_per_frame": round(sh_ms, 4),
           "serial_ms_per_step": round(serial_ms, 4),
           "kernels": kernels, "roofline": roofline, "other_rooflines": others,
           "serial_pass": {"kernels": kernels_serial,
                           "rooflines": {k: {"achieved": v["achieved"], "frac": v["frac"], "unit": v["unit"]}
                                         for k, v in serial_records.items()}}}
    out.update(extra)
    if a.dtype != "f32" or a.form != "plain" or not default_path:
        # against the plain f32 path on the same frame (itself checked against the oracle): reflection
        # probabilities p_k, per-pixel radiance, and the frame's mean radiance
        ref_pipe = new_env("f32")
        ref_pipe.build_luts()
        ref_pipe.run(env)
        ref_sh = Shader(ctx, {k: v for k, v in gbuf_np.items() if k not in G.GBUF_OPTIONAL}, seed=w.hash_seed,
                        vertices=a.vertices)
        P = shader.P
        dbg0 = {"probs": torch.empty((P, w.K), dtype=torch.float64, device="cuda")}
        Kd = 2 if prob_mode == G.GLINT_PROBS_CONSTANT else w.K  # constant probabilities: two bins
        dbg1 = {"probs": torch.empty((P, Kd), dtype=torch.float64, device="cuda")}
        ref_sh.run(ref_pipe.env_struct(), debug=dbg0)
        shader.run(envs, debug=dbg1)
        torch.cuda.synchronize()
        hit = torch.from_numpy(gbuf_np["surf_id"] != 0xFFFFFFFF).cuda()
        r0 = ref_sh.radiance[hit].double().sum(1)
        r1 = shader.radiance[hit].double().sum(1)
        rel = ((r1 - r0).abs() / r0.abs().clamp_min(1e-12))
        lit = r0 > 1e-6 * r0.max()
        out["vs_plain_f32"] = {
            "probs_mean_abs_err": float((dbg1["probs"][hit] - dbg0["probs"][hit]).abs().mean().item())
            if Kd == w.K else None,
            "radiance_mean_rel_err": float(rel[lit].mean().item()),
            "frame_mean_radiance_ratio": float((r1.mean() / r0.mean()).item())}
    if a.form == "surrogate" or (a.dtype != "f32" and default_path):
        out["vs_plain_filter"] = filter_accuracy(G, ctx, w, pipe, env, gbuf_np, shader, envs)
    if a.form == "surrogate" and a.rotate_frames > 0:
        out["rotating_suns"] = rotating_study(G, ctx, w, env_np, gbuf_np, sur, a.rotate_frames, a.train_epochs)
    if not a.no_cpu_baseline and a.form == "plain" and default_path:
        if a.dtype == "f32":
            ind_h = pipe.ind_pyr.cpu().numpy()
        else:
            ind_h = np.full((pipe.texels, w.K), 1.0 / w.K, np.float32)
        inputs = (ind_h, pipe.rgb_pyr.cpu().numpy(), pipe.levels.cpu().numpy(), pipe.lut_S.cpu().numpy(),
                  pipe.lut_E.cpu().numpy())
        out["cpu_baseline"] = cpu_baseline(w, env_np, gbuf_np, glint_pixels, a.cpu_sample, inputs)
    G.glint_destroy(ctx)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
