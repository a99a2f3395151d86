"""Thin Python binding of libglint.so (the C ABI in include/glint.h).

Argument marshalling only: torch tensors are passed as device pointers and
torch's current HIP stream as the stream; every step of the hot path runs in
the library's HIP kernels.  There is no CPU fallback: if the library is
missing or no GPU is present, calls raise.
"""
from __future__ import annotations

import ctypes as C
import os

from . import build as _build

GLINT_OK, GLINT_EINVAL, GLINT_EUNSUPPORTED, GLINT_EDEVICE, GLINT_ENOMEM, GLINT_ENOTTRAINED = 0, 1, 2, 3, 4, 5
GLINT_F32, GLINT_F16, GLINT_BF16, GLINT_UNORM16 = 0, 1, 2, 3
GLINT_SAMPLER_DUAL, GLINT_SAMPLER_SINGLE, GLINT_SAMPLER_SINGLE_FLOOR, GLINT_SAMPLER_DUAL_SYMMETRIC = 0, 1, 2, 3
GLINT_PROBS_ENV, GLINT_PROBS_CONSTANT = 0, 1
GLINT_TREE_BALANCED, GLINT_TREE_CHAIN = 0, 1
GLINT_NO_SURFACE = 0xFFFFFFFF
LUT_N = 64

GBUF_FIELDS = ("nx", "ny", "nz", "vx", "vy", "vz", "u", "v", "area", "ax", "ay", "density",
               "f0r", "f0g", "f0b", "surf_id")
GBUF_OPTIONAL = ("visibility", "tx", "ty", "tz", "dudx", "dudy", "dvdx", "dvdy")  # float32, may be absent


class GlintError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"glint error {code}: {msg}")
        self.code = code


class PartitionParams(C.Structure):
    _fields_ = [("K", C.c_int), ("ell", C.c_double), ("level_mode", C.c_int), ("weight_space", C.c_int)]


class PrefilterParams(C.Structure):
    _fields_ = [("num_mips", C.c_int), ("taps", C.c_int), ("dtype", C.c_int)]


class GBuffer(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in GBUF_FIELDS] + [(k, C.c_void_p) for k in GBUF_OPTIONAL]


class Env(C.Structure):
    _fields_ = [("ind_pyr", C.c_void_p), ("rgb_pyr", C.c_void_p), ("levels", C.c_void_p),
                ("lut_S", C.c_void_p), ("lut_E", C.c_void_p), ("R", C.c_int), ("K", C.c_int),
                ("num_mips", C.c_int), ("dtype", C.c_int), ("quantile_tail", C.c_void_p)]


class ShadeParams(C.Structure):
    _fields_ = [("seed", C.c_uint32), ("vertices", C.c_int), ("exact_gating", C.c_int), ("sampler", C.c_int),
                ("prob_mode", C.c_int), ("gamma", C.c_float), ("lobe_taps", C.c_int), ("tree", C.c_int)]


class ShadeDebug(C.Structure):
    _fields_ = [("counts", C.c_void_p), ("codes", C.c_void_p), ("probs", C.c_void_p)]


class EnvTask(C.Structure):
    _fields_ = [("env", C.c_void_p), ("R", C.c_int), ("partition", PartitionParams), ("prefilter", PrefilterParams),
                ("partition_workspace", C.c_void_p), ("prefilter_workspace", C.c_void_p), ("levels", C.c_void_p),
                ("ind_j", C.c_void_p), ("ind_t", C.c_void_p), ("ind_pyr", C.c_void_p), ("rgb_pyr", C.c_void_p),
                ("lut_S", C.c_void_p), ("lut_E", C.c_void_p), ("quantile_tail", C.c_void_p),
                ("surrogate_w", C.c_void_p), ("surrogate_w_bf16", C.c_void_p)]


class View(C.Structure):
    _fields_ = [("gbuf", GBuffer), ("num_pixels", C.c_int64), ("env_index", C.c_int), ("shade", ShadeParams),
                ("radiance", C.c_void_p), ("surrogate_F", C.c_void_p)]


_LIB = None

EXPORTS = {
    "glint_version": ([], C.c_int),
    "glint_last_error": ([C.c_void_p], C.c_char_p),
    "glint_create": ([C.c_int, C.POINTER(C.c_void_p)], C.c_int),
    "glint_destroy": ([C.c_void_p], None),
    "glint_sync": ([C.c_void_p], C.c_int),
    "glint_partition_workspace_bytes": ([C.c_int], C.c_size_t),
    "glint_partition_env": ([C.c_void_p, C.c_void_p, C.c_int, C.POINTER(PartitionParams), C.c_void_p, C.c_void_p,
                             C.c_void_p, C.c_void_p, C.c_void_p], C.c_int),
    "glint_partition_env_noalloc": ([C.c_void_p, C.c_void_p, C.c_int, C.POINTER(PartitionParams), C.c_void_p,
                                     C.c_void_p, C.c_void_p, C.c_void_p], C.c_int),
    "glint_pyramid_texels": ([C.c_int, C.c_int], C.c_int64),
    "glint_prefilter_workspace_bytes": ([C.c_int, C.c_int, C.POINTER(PrefilterParams)], C.c_size_t),
    "glint_prefilter": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_int,
                         C.POINTER(PrefilterParams), C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p], C.c_int),
    "glint_build_luts": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p], C.c_int),
    "glint_quantile_table_bytes": ([], C.c_size_t),
    "glint_build_quantile_table": ([C.c_void_p, C.c_void_p, C.c_void_p], C.c_int),
    "glint_sample_binomial": ([C.c_void_p, C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                               C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p], C.c_int),
    "glint_shade": ([C.c_void_p, C.POINTER(GBuffer), C.c_int64, C.POINTER(Env), C.POINTER(ShadeParams),
                     C.c_void_p, C.POINTER(ShadeDebug), C.c_void_p], C.c_int),
    "glint_sample_filter": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_int,
                             C.POINTER(PrefilterParams), C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p,
                             C.c_void_p], C.c_int),
    "glint_surrogate_samples": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_int,
                                 C.POINTER(PrefilterParams), C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                 C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p], C.c_int),
    "glint_filter_pixels": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_int,
                             C.POINTER(PrefilterParams), C.c_void_p, C.POINTER(GBuffer), C.c_int64, C.c_void_p,
                             C.c_void_p], C.c_int),
    "glint_surrogate_params": ([], C.c_int),
    "glint_surrogate_workspace_bytes": ([C.c_int], C.c_size_t),
    "glint_surrogate_prepare": ([C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p], C.c_int),
    "glint_surrogate_forward": ([C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p,
                                 C.c_void_p], C.c_int),
    "glint_surrogate_gradient": ([C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                  C.c_float, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p], C.c_int),
    "glint_surrogate_train_step": ([C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int,
                                    C.c_float, C.c_void_p, C.c_void_p, C.c_void_p, C.c_float, C.c_int, C.c_void_p,
                                    C.c_void_p, C.c_void_p], C.c_int),
    "glint_shade_surrogate_workspace_bytes": ([C.c_int64, C.c_int], C.c_size_t),
    "glint_shade_surrogate": ([C.c_void_p, C.POINTER(GBuffer), C.c_int64, C.POINTER(Env), C.c_void_p, C.c_void_p,
                               C.POINTER(ShadeParams), C.c_void_p, C.c_void_p, C.POINTER(ShadeDebug), C.c_void_p],
                              C.c_int),
    "glint_shade_given_F": ([C.c_void_p, C.POINTER(GBuffer), C.c_int64, C.POINTER(Env), C.c_void_p,
                             C.POINTER(ShadeParams), C.c_void_p, C.POINTER(ShadeDebug), C.c_void_p], C.c_int),
    "glint_batched_workspace_bytes": ([C.c_int], C.c_size_t),
    "glint_frame_batched": ([C.c_void_p, C.POINTER(EnvTask), C.c_int, C.POINTER(View), C.c_int, C.c_void_p,
                             C.c_void_p], C.c_int),
    "glint_batched_tile_px": ([C.c_void_p], C.c_int),
    "glint_profile_enable": ([C.c_void_p, C.c_int], C.c_int),
    "glint_profile_select": ([C.c_void_p, C.c_char_p], C.c_int),
    "glint_profile_collect": ([C.c_void_p, C.POINTER(C.c_int)], C.c_int),
    "glint_profile_entry": ([C.c_void_p, C.c_int, C.POINTER(C.c_char_p), C.POINTER(C.c_double),
                             C.POINTER(C.c_int64)], C.c_int),
}


def lib():
    """Loads the in-tree libglint.so (building it once if it was never built)."""
    global _LIB
    if _LIB is None:
        path = _build.library_path()
        if not os.path.exists(path):
            _build.build_library()
        L = C.CDLL(path)
        for name, (args, res) in EXPORTS.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _LIB = L
    return _LIB


def library_path() -> str:
    return _build.library_path()


def _check(rc):
    if rc != GLINT_OK:
        raise GlintError(rc, lib().glint_last_error(None).decode())


def _ptr(t):
    if t is None:
        return None
    return C.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(stream.cuda_stream)


def _require_cuda(*tensors):
    for t in tensors:
        if t is not None and not t.is_cuda:
            raise GlintError(GLINT_EINVAL, "tensor arguments must live on the GPU")


# --- C ABI, one function per entry point ------------------------------------------

def glint_version() -> int:
    return lib().glint_version()


def glint_last_error(ctx=None) -> str:
    return lib().glint_last_error(ctx).decode()


def glint_create(device: int = 0) -> C.c_void_p:
    h = C.c_void_p()
    _check(lib().glint_create(device, C.byref(h)))
    return h


def glint_destroy(ctx) -> None:
    lib().glint_destroy(ctx)


def glint_sync(ctx) -> None:
    _check(lib().glint_sync(ctx))


def glint_partition_workspace_bytes(R: int) -> int:
    return lib().glint_partition_workspace_bytes(R)


def glint_partition_env(ctx, env, R, params: PartitionParams, workspace, levels, ind_j, ind_t, stream=None):
    _require_cuda(env, workspace, levels, ind_j, ind_t)
    _check(lib().glint_partition_env(ctx, _ptr(env), R, C.byref(params), _ptr(workspace), _ptr(levels),
                                     _ptr(ind_j), _ptr(ind_t), _stream(stream)))


def glint_partition_env_noalloc(ctx, env, R, params: PartitionParams, levels, ind_j, ind_t, stream=None):
    _require_cuda(env, levels, ind_j, ind_t)
    _check(lib().glint_partition_env_noalloc(ctx, _ptr(env), R, C.byref(params), _ptr(levels), _ptr(ind_j),
                                             _ptr(ind_t), _stream(stream)))


def glint_pyramid_texels(R: int, num_mips: int) -> int:
    return lib().glint_pyramid_texels(R, num_mips)


def glint_prefilter_workspace_bytes(R: int, K: int, params: PrefilterParams) -> int:
    return lib().glint_prefilter_workspace_bytes(R, K, C.byref(params))


def glint_prefilter(ctx, env, ind_j, ind_t, R, K, params: PrefilterParams, workspace, ind_pyr, rgb_pyr,
                    stream=None):
    _require_cuda(env, ind_j, ind_t, workspace, ind_pyr, rgb_pyr)
    _check(lib().glint_prefilter(ctx, _ptr(env), _ptr(ind_j), _ptr(ind_t), R, K, C.byref(params),
                                 _ptr(workspace), _ptr(ind_pyr), _ptr(rgb_pyr), _stream(stream)))


def glint_build_luts(ctx, lut_S, lut_E, stream=None):
    _require_cuda(lut_S, lut_E)
    _check(lib().glint_build_luts(ctx, _ptr(lut_S), _ptr(lut_E), _stream(stream)))


def glint_quantile_table_bytes() -> int:
    return lib().glint_quantile_table_bytes()


def glint_build_quantile_table(ctx, table, stream=None):
    _require_cuda(table)
    _check(lib().glint_build_quantile_table(ctx, _ptr(table), _stream(stream)))


def glint_sample_binomial(ctx, sampler, N, p, h1, h2, n, nbar, code, quantile_tail=None, exact_gating=0,
                          stream=None):
    """N, p: float64; h1, h2: 32-bit words (int32 or uint32 storage); n, nbar:
    float64 outputs; code: uint8 output; all device tensors of one length."""
    _require_cuda(N, p, h1, h2, n, nbar, code, quantile_tail)
    count = N.numel()
    if any(t.numel() != count for t in (p, h1, h2, n, nbar, code)):
        raise ValueError("all arrays must have the same length")
    _check(lib().glint_sample_binomial(ctx, sampler, exact_gating, _ptr(N), _ptr(p), _ptr(h1), _ptr(h2), count,
                                       _ptr(quantile_tail), _ptr(n), _ptr(nbar), _ptr(code), _stream(stream)))


def make_gbuffer(fields: dict) -> GBuffer:
    """Maps a dict of device tensors (one per G-buffer field, plus the optional
    float32 fields of GBUF_OPTIONAL) to the C struct."""
    _require_cuda(*fields.values())
    opt = [fields.get(k) for k in GBUF_OPTIONAL]
    g = GBuffer(*[fields[k].data_ptr() for k in GBUF_FIELDS], *[t.data_ptr() if t is not None else None for t in opt])
    g._keep = dict(fields)  # the struct holds raw pointers: keep the tensors alive with it
    return g


def make_env(ind_pyr, rgb_pyr, levels, lut_S, lut_E, R, K, num_mips, dtype, quantile_tail=None) -> Env:
    _require_cuda(ind_pyr, rgb_pyr, levels, lut_S, lut_E, quantile_tail)
    def ptr(t):
        return t.data_ptr() if t is not None else None
    e = Env(ptr(ind_pyr), ptr(rgb_pyr), ptr(levels), ptr(lut_S), ptr(lut_E), R, K, num_mips, dtype,
            ptr(quantile_tail))
    e._keep = (ind_pyr, rgb_pyr, levels, lut_S, lut_E, quantile_tail)  # keeps the tensors alive with the struct
    return e


def glint_shade(ctx, gbuf: GBuffer, num_pixels: int, env: Env, params: ShadeParams, radiance, debug=None,
                stream=None):
    _require_cuda(radiance)
    dbg = None
    if debug is not None:
        _require_cuda(*[t for t in debug.values() if t is not None])
        dbg = ShadeDebug(*[debug.get(k).data_ptr() if debug.get(k) is not None else None
                           for k in ("counts", "codes", "probs")])
    _check(lib().glint_shade(ctx, C.byref(gbuf), num_pixels, C.byref(env), C.byref(params), _ptr(radiance),
                             C.byref(dbg) if dbg is not None else None, _stream(stream)))


def _debug(debug):
    if debug is None:
        return None
    _require_cuda(*[t for t in debug.values() if t is not None])
    return ShadeDebug(*[debug.get(k).data_ptr() if debug.get(k) is not None else None
                        for k in ("counts", "codes", "probs")])


def glint_sample_filter(ctx, env, ind_j, ind_t, R, K, params: PrefilterParams, workspace, dirs, alphas, out,
                        stream=None):
    _require_cuda(env, ind_j, ind_t, workspace, dirs, alphas, out)
    n = int(alphas.numel())
    _check(lib().glint_sample_filter(ctx, _ptr(env), _ptr(ind_j), _ptr(ind_t), R, K, C.byref(params),
                                     _ptr(workspace), _ptr(dirs), _ptr(alphas), n, _ptr(out), _stream(stream)))


def glint_surrogate_samples(ctx, env, ind_j, ind_t, R, K, params: PrefilterParams, workspace, dirs, ax, ay, x,
                            target, stream=None):
    _require_cuda(env, ind_j, ind_t, workspace, dirs, ax, ay, x, target)
    n = int(ax.numel())
    _check(lib().glint_surrogate_samples(ctx, _ptr(env), _ptr(ind_j), _ptr(ind_t), R, K, C.byref(params),
                                         _ptr(workspace), _ptr(dirs), _ptr(ax), _ptr(ay), n, _ptr(x), _ptr(target),
                                         _stream(stream)))


def glint_filter_pixels(ctx, env, ind_j, ind_t, R, K, params: PrefilterParams, workspace, gbuf: GBuffer,
                        num_pixels: int, F, stream=None):
    _require_cuda(env, ind_j, ind_t, workspace, F)
    _check(lib().glint_filter_pixels(ctx, _ptr(env), _ptr(ind_j), _ptr(ind_t), R, K, C.byref(params),
                                     _ptr(workspace), C.byref(gbuf), num_pixels, _ptr(F), _stream(stream)))


def glint_surrogate_params() -> int:
    return lib().glint_surrogate_params()


def glint_surrogate_workspace_bytes(batch: int) -> int:
    return lib().glint_surrogate_workspace_bytes(batch)


def glint_surrogate_prepare(ctx, K, w, w_bf16, stream=None):
    _require_cuda(w, w_bf16)
    _check(lib().glint_surrogate_prepare(ctx, K, _ptr(w), _ptr(w_bf16), _stream(stream)))


def glint_surrogate_forward(ctx, K, w, w_bf16, x, probs, stream=None):
    _require_cuda(w, w_bf16, x, probs)
    B = int(x.shape[0])
    _check(lib().glint_surrogate_forward(ctx, K, _ptr(w), _ptr(w_bf16), _ptr(x), B, _ptr(probs), _stream(stream)))


def glint_surrogate_gradient(ctx, K, w, w_bf16, x, target, workspace, grad, loss, stream=None, levels=None,
                             radiance_weight=0.0):
    _require_cuda(w, w_bf16, x, target, workspace, grad, loss, levels)
    B = int(x.shape[0])
    _check(lib().glint_surrogate_gradient(ctx, K, _ptr(w), _ptr(w_bf16), _ptr(x), _ptr(target), _ptr(levels),
                                          radiance_weight, B, _ptr(workspace), _ptr(grad), _ptr(loss),
                                          _stream(stream)))


def glint_surrogate_train_step(ctx, K, w, w_bf16, m, v, step, lr, x, target, workspace, loss, stream=None,
                               levels=None, radiance_weight=0.0):
    _require_cuda(w, w_bf16, m, v, x, target, workspace, loss, levels)
    B = int(x.shape[0])
    _check(lib().glint_surrogate_train_step(ctx, K, _ptr(w), _ptr(w_bf16), _ptr(m), _ptr(v), step, lr, _ptr(x),
                                            _ptr(target), _ptr(levels), radiance_weight, B, _ptr(workspace),
                                            _ptr(loss), _stream(stream)))


def glint_shade_surrogate_workspace_bytes(num_pixels: int, K: int) -> int:
    return lib().glint_shade_surrogate_workspace_bytes(num_pixels, K)


def glint_shade_surrogate(ctx, gbuf: GBuffer, num_pixels: int, env: Env, w, w_bf16, params: ShadeParams, workspace,
                          radiance, debug=None, stream=None):
    _require_cuda(w, w_bf16, workspace, radiance)
    dbg = _debug(debug)
    _check(lib().glint_shade_surrogate(ctx, C.byref(gbuf), num_pixels, C.byref(env), _ptr(w), _ptr(w_bf16),
                                       C.byref(params), _ptr(workspace), _ptr(radiance),
                                       C.byref(dbg) if dbg is not None else None, _stream(stream)))


def glint_shade_given_F(ctx, gbuf: GBuffer, num_pixels: int, env: Env, F, params: ShadeParams, radiance,
                        debug=None, stream=None):
    _require_cuda(F, radiance)
    dbg = _debug(debug)
    _check(lib().glint_shade_given_F(ctx, C.byref(gbuf), num_pixels, C.byref(env), _ptr(F), C.byref(params),
                                     _ptr(radiance), C.byref(dbg) if dbg is not None else None, _stream(stream)))


def glint_batched_workspace_bytes(n_views: int) -> int:
    return lib().glint_batched_workspace_bytes(n_views)


def glint_frame_batched(ctx, envs, views, workspace, stream=None):
    """envs: sequence of EnvTask, views: sequence of View (C structs)."""
    _require_cuda(workspace)
    ea = (EnvTask * len(envs))(*envs)
    va = (View * len(views))(*views)
    _check(lib().glint_frame_batched(ctx, ea, len(envs), va, len(views), _ptr(workspace), _stream(stream)))


def glint_batched_tile_px(ctx) -> int:
    return lib().glint_batched_tile_px(ctx)


def glint_profile_enable(ctx, enable: bool = True) -> None:
    _check(lib().glint_profile_enable(ctx, 1 if enable else 0))


def glint_profile_select(ctx, kernels=None) -> None:
    """Times only the named kernels (iterable of names; None: all)."""
    _check(lib().glint_profile_select(ctx, ",".join(kernels).encode() if kernels else None))


def glint_profile_collect(ctx) -> dict:
    """Per-kernel totals so far: {name: (total_ms, launches)} (cumulative)."""
    n = C.c_int()
    _check(lib().glint_profile_collect(ctx, C.byref(n)))
    out = {}
    for i in range(n.value):
        name, ms, cnt = C.c_char_p(), C.c_double(), C.c_int64()
        _check(lib().glint_profile_entry(ctx, i, C.byref(name), C.byref(ms), C.byref(cnt)))
        out[name.value.decode()] = (ms.value, cnt.value)
    return out
