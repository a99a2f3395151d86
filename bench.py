"""Benchmark of the glint hot path on one MI355X.

A step is one frame of the whole per-frame path on the frame workload:
environment partition (luminance min/max, radiance levels, fuzzy
indicators), source mip chain, NDF prefilter of the K indicator channels and
RGB into the roughness pyramid, then glint shading of the 1920x1080 G-buffer
(N_P, reflection probabilities, dual-gated multinomial, radiance).  The
lookup tables are built once per BRDF model before timing (not per frame).
Inputs are synthetic and resident in HBM before the timed region.

Prints one JSON line: value = glint-shaded Mpix/s (pixels that ran the glint
shader, per second of whole-frame time), plus prefilter ms/frame, the
roofline record of the dominant kernel and the CPU-oracle baseline.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

METRIC = "glint-shaded Mpix/s + env prefilter ms/frame; surrogate/FP16 vs plain, 1 GPU"
HBM_PEAK_GBS = 8000.0
# Peak VALU lane-operations per second: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
# (one wave64 VALU instruction per SIMD every 4 cycles); double FMA issues at
# the same rate as non-packed float on this part.
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12


def shade_ops_per_pixel(K: int) -> float:
    """VALU lane-ops per pixel the algorithm needs:
    lookup (8 texels x (K+3) channels, double FMA + convert) + per tree node
    (hash, float gating with two powf, double Gaussian with AS 241) + combine."""
    lookup = 8 * (K + 3) * 2 + 120
    node = 22 + 2 * 40 + 30 + 140
    combine = 6 * K + 40
    return float(lookup + (K - 1) * node + combine)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="frame")
    ap.add_argument("--dtype", default="f32", choices=["f32", "f16", "bf16", "unorm16"])
    ap.add_argument("--vertices", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
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


def cpu_baseline(w, env, gbuf, glint_pixels, frac, shade_inputs):
    """Times the oracle (as it stands) on a stratified sample of the same frame
    and scales to Mpix/s of whole frames.  shade_inputs: the frame's pyramid,
    levels and LUTs (host copies), so the sampled pixels shade real values."""
    import oracle
    threads = min(os.cpu_count() or 1, 16)
    t0 = time.perf_counter()
    levels, ij, it = oracle.partition(env, w.K, w.ell)
    chain = oracle.mipchain(env, ij, it, w.K, w.M)
    t_part = time.perf_counter() - t0
    n_tex = oracle.pyramid_texels(w.R, w.M)
    step = max(1, int(round(1.0 / frac)))
    tex = np.arange(0, n_tex, step, dtype=np.int64)
    t0 = time.perf_counter()
    oracle.prefilter(env, ij, it, chain, w.K, w.M, w.T, texel_ids=tex, threads=threads)
    t_pre = (time.perf_counter() - t0) * (n_tex / len(tex))
    ind, rgb, lv, lut_S, lut_E = shade_inputs
    hit = np.nonzero(gbuf["surf_id"] != 0xFFFFFFFF)[0]
    pix = hit[::step]
    t0 = time.perf_counter()
    oracle.shade(gbuf, ind, rgb, lv, lut_S, lut_E, w.R, w.K, w.M, w.hash_seed, 1, pixels=pix, threads=threads)
    t_sh = (time.perf_counter() - t0) * (len(hit) / len(pix))
    frame_s = t_part + t_pre + t_sh
    return {"value": glint_pixels / frame_s / 1e6, "unit": "Mpix/s", "cores": threads, "kind": "oracle",
            "sample": f"full partition + mip chain; every {step}th pyramid texel ({len(tex)}) and every {step}th "
                      f"glint pixel ({len(pix)}) timed, scaled to the whole frame; oracle frame time "
                      f"{frame_s:.2f} s (prefilter {t_part + t_pre:.2f} s, shade {t_sh:.2f} s)",
            "prefilter_s_per_frame": t_part + t_pre, "shade_s_per_frame": t_sh}


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
    bf = BatchedFrame(ctx, envs, views)
    glint_pixels = sum(int((gb["surf_id"] != 0xFFFFFFFF).sum()) for (gb, _, _, _) in views)
    bf.run()  # set-up call (autotune + capture)
    torch.cuda.synchronize()
    for _ in range(a.warmup):
        bf.run()
    torch.cuda.synchronize()
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
           "steps": a.steps, "warmup": a.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "batched: 64 views (256^2..1920x1080, log-uniform pixels), 4 cube maps "
                                  "6x256x256 with K=4,8,16,8, M=8, T=64; one graph launch per frame",
                      "views": len(views), "total_pixels": bf.total_pixels, "glint_pixels": glint_pixels,
                      "tile_px": G.glint_batched_tile_px(ctx)}}
    G.glint_destroy(ctx)
    print(json.dumps(out), flush=True)


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
    from paper_2507_02674_amd.pipeline import EnvPipeline, Shader

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(1)
    if a.workload == "batched":
        batched(a)
        return
    dtypes = {"f32": G.GLINT_F32, "f16": G.GLINT_F16, "bf16": G.GLINT_BF16, "unorm16": G.GLINT_UNORM16}
    w = synth.WORKLOADS[a.workload]
    env_np, gbuf_np = w.env(), w.gbuf()
    glint_pixels = int((gbuf_np["surf_id"] != 0xFFFFFFFF).sum())
    ctx = G.glint_create(0)
    env = torch.from_numpy(env_np).cuda()
    pipe = EnvPipeline(ctx, w.R, w.K, w.M, w.T, dtypes[a.dtype], w.ell)
    shader = Shader(ctx, gbuf_np, seed=w.hash_seed, vertices=a.vertices)
    pipe.build_luts()
    torch.cuda.synchronize()
    envs = pipe.env_struct()
    for _ in range(a.warmup):
        pipe.run(env)
        shader.run(envs)
    torch.cuda.synchronize()

    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(a.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(a.steps):
        ev[s][0].record()
        pipe.run(env)
        ev[s][1].record()
        shader.run(envs)
        ev[s][2].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    pre_ms = float(np.mean([e[0].elapsed_time(e[1]) for e in ev]))
    sh_ms = float(np.mean([e[1].elapsed_time(e[2]) for e in ev]))
    frame_ms = float(ev[0][0].elapsed_time(ev[-1][2])) / a.steps
    ms_per_step = max(frame_ms, 1e3 * wall / a.steps)
    value = glint_pixels / (ms_per_step * 1e-3) / 1e6

    ops = shade_ops_per_pixel(w.K) * glint_pixels * a.vertices
    achieved = ops / (sh_ms * 1e-3) / 1e12
    roofline = {"bound": "alu", "kernel": "k_shade", "achieved": round(achieved, 3), "peak": VALU_PEAK_TOPS,
                "unit": "TOP/s (VALU lane-ops)", "frac": round(achieved / VALU_PEAK_TOPS, 4), "traffic": None,
                "ops_per_pixel": shade_ops_per_pixel(w.K), "hbm_gbs": round(76.0 * glint_pixels / (sh_ms * 1e-3) / 1e9, 1),
                "hbm_frac": round(76.0 * glint_pixels / (sh_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    out = {"metric": METRIC, "value": round(value, 3), "unit": "Mpix/s", "n_gpus": 1, "steps": a.steps,
           "warmup": a.warmup, "ms_per_step": round(ms_per_step, 4), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"{w.name}: {w.W}x{w.H} sphere+plane G-buffer, cube map 6x{w.R}x{w.R}, "
                                  f"{w.M} mips, K={w.K}, T={w.T} taps, per-frame partition+prefilter+shade",
                      "pyramid_dtype": a.dtype, "vertices": a.vertices, "glint_pixels": glint_pixels},
           "prefilter_ms_per_frame": round(pre_ms, 4), "shade_ms_per_frame": round(sh_ms, 4),
           "roofline": roofline}
    if not a.no_cpu_baseline:
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
