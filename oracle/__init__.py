"""FP64 CPU oracle for image-based glint lighting (Kneiphof & Klein, EGSR 2025).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py``, never by the product path.  It
shares no code with the HIP library.  The arithmetic lives in
``glint_oracle.c`` (plain loops, double precision); this module only marshals
numpy arrays into it and chains its steps in the paper's order:

* Sec. 5, "Discrete Radiance Levels" / "Fuzzy Indicator Functions"
  -> :func:`partition`
* Sec. 5, "Integrated NDF", Eq. (rtiblndf) with the kernel of Sec. 3.4
  -> :func:`mipchain`, :func:`prefilter`
* Sec. 5 (visible reflecting facet area) and Sec. 3.4 (split sum)
  -> :func:`luts`
* Sec. 3.2 (N_P), Sec. 4 Eq. (probhk) and Eq. (iblglints:fin), Sec. 6 and
  Alg. "Dual-gated Gaussian" -> :func:`shade`
* Sec. 6 "Single-Gated Gaussians" / "Gating Generalization", Eq. (gated),
  Eq. (oldgated) -> :func:`sample_binomial`, ``shade(sampler=...)``
* Sec. 3.3 footprint grid -> :func:`footprint_grid`, ``shade(vertices=12)``;
  Sec. 8 anisotropic lookup and occlusion, Sec. 7 comparison method ->
  ``shade(lobe_taps=..., prob_mode=..., gbuf["visibility"])``

Pins (tests/test_oracle_*.py): every step is checked against closed forms,
invariants, library routines or brute force.  The per-footprint hash (pcg4d,
Jarzynski & Olano 2020) has no published output values to compare with; it
is pinned by the properties the method relies on (tests/test_oracle_hash.py:
avalanche of the upper output bits, the carry structure of its multiply-add
and xorshift steps, 2-D chi^2 independence of a node's two uniforms, of the
two nodes sharing one hash and of neighbouring vertices), which reject the
plausible slips in its definition; the GPU path implements the same
published definition independently.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from .build import build_oracle, library_path

_LIB = None
LUT_N = 64


def lib():
    global _LIB
    if _LIB is None:
        path = library_path()
        if not os.path.exists(path):
            build_oracle()
        _LIB = C.CDLL(path)
        _declare(_LIB)
    return _LIB


def _p(a, ctype):
    return a.ctypes.data_as(C.POINTER(ctype))


def _declare(L):
    f32p, f64p = C.POINTER(C.c_float), C.POINTER(C.c_double)
    u8p, i64p = C.POINTER(C.c_uint8), C.POINTER(C.c_int64)
    L.orc_partition.argtypes = [f32p, C.c_int, C.c_int, C.c_double, C.c_int, C.c_int, f64p, u8p, f32p]
    L.orc_mipchain.argtypes = [f32p, u8p, f32p, C.c_int, C.c_int, C.c_int, f32p]
    L.orc_prefilter_texels.argtypes = [f32p, u8p, f32p, f32p, C.c_int, C.c_int, C.c_int, C.c_int, i64p,
                                       C.c_int64, f64p, C.c_int]
    L.orc_lut_cells.argtypes = [C.POINTER(C.c_int), C.c_int64, f64p, f64p, f64p, C.c_int]
    L.orc_ppnd16.argtypes = [C.c_double]
    L.orc_ppnd16.restype = C.c_double
    L.orc_hash_xi.argtypes = [C.c_uint32, C.c_uint32, C.c_int32, C.c_int64, C.c_int64, C.c_int,
                              f32p, f32p]
    L.orc_quantile_levels.argtypes = [f32p, C.c_int, C.c_int, C.c_double, f64p, f64p]
    L.orc_pcg4d.argtypes = [C.POINTER(C.c_uint32), C.POINTER(C.c_uint32), C.c_int64]
    L.orc_shade_pixels.argtypes = [C.POINTER(f32p), f32p, f32p, f64p, f32p, f32p, C.c_int, C.c_int, C.c_int,
                                   C.c_uint32, C.c_int, C.c_int, C.c_int, C.c_int, C.c_double, C.c_int, i64p,
                                   C.c_int64, f64p, f64p, u8p, f64p, u8p, C.c_int]
    L.orc_shade_pixels_given_F.argtypes = [C.POINTER(f32p), f64p, f32p, f64p, f32p, f32p, C.c_int, C.c_int,
                                           C.c_int, C.c_uint32, C.c_int, C.c_int, C.c_int, i64p, C.c_int64, f64p,
                                           f64p, u8p, f64p, u8p, C.c_int]
    u32p = C.POINTER(C.c_uint32)
    L.orc_footprint_grid.argtypes = [C.c_double] * 6 + [f64p, f64p, u32p, i64p, i64p]
    L.orc_footprint_grid.restype = C.c_int
    L.orc_sample_binomial.argtypes = [C.c_int, f64p, f64p, u32p, u32p, C.c_int64, f64p, f64p, u8p, u8p, C.c_int]
    L.orc_gate_probs.argtypes = [C.c_float, C.c_float, f32p]
    L.orc_gate_probs_symmetric.argtypes = [C.c_float, C.c_float, C.c_float, f32p]
    L.orc_dual_gated.argtypes = [C.c_double, C.c_double, C.c_float, C.c_float, f64p, f64p, u8p]
    L.orc_multinomial.argtypes = [C.c_int, C.c_int, C.c_double, f64p, C.c_int, C.c_uint32, C.c_uint32, C.c_int32,
                                  C.c_int64, C.c_int64, f64p, u8p]
    L.orc_multinomial.restype = C.c_int
    L.orc_face_dir.argtypes = [C.c_int, C.c_double, C.c_double, f64p]
    L.orc_dir_face.argtypes = [f64p, f64p]
    L.orc_dir_face.restype = C.c_int
    L.orc_lattice_level.argtypes = [C.c_double, f64p]
    L.orc_lattice_level.restype = C.c_int
    L.orc_taps.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, f64p]
    L.orc_pyramid_lookup.argtypes = [f32p, C.c_int, C.c_int, C.c_int, f64p, f64p, C.c_int64, f64p]
    L.orc_sample_filter.argtypes = [f32p, u8p, f32p, f32p, C.c_int, C.c_int, C.c_int, C.c_int, f64p, f64p,
                                    C.c_int64, f64p, C.c_int]


def threads_default():
    return int(os.environ.get("GLINT_ORACLE_THREADS", os.cpu_count() or 1))


def pyramid_texels(R: int, M: int) -> int:
    return sum(6 * (R >> m) ** 2 for m in range(M))


def level_offset(R: int, m: int) -> int:
    return sum(6 * (R >> s) ** 2 for s in range(m))


def partition(env: np.ndarray, K: int, ell: float = 1e-3, level_mode: int = 0, weight_space: int = 0):
    """Radiance levels and fuzzy indicators (Sec. 5).  env: [6,R,R,3] float32.

    Returns (levels [K] f64, ind_j [6,R,R] u8, ind_t [6,R,R] f32).
    Pinned by closed forms in tests/test_oracle_env.py.
    """
    env = np.ascontiguousarray(env, dtype=np.float32)
    R = env.shape[1]
    levels = np.zeros(K, np.float64)
    ind_j = np.zeros((6, R, R), np.uint8)
    ind_t = np.zeros((6, R, R), np.float32)
    rc = lib().orc_partition(_p(env, C.c_float), R, K, ell, level_mode, weight_space, _p(levels, C.c_double),
                             _p(ind_j, C.c_uint8), _p(ind_t, C.c_float))
    if rc:
        raise ValueError("orc_partition rejected its arguments")
    return levels, ind_j, ind_t


def mipchain(env, ind_j, ind_t, K: int, M: int) -> np.ndarray:
    """Source mip chain levels 1..M-1, float32, flat [texels, K+3]."""
    R = env.shape[1]
    n = level_offset(R, M) - 6 * R * R
    chain = np.zeros((max(n, 1), K + 3), np.float32)
    rc = lib().orc_mipchain(_p(env, C.c_float), _p(ind_j, C.c_uint8), _p(ind_t, C.c_float), R, K, M,
                            _p(chain, C.c_float))
    if rc:
        raise ValueError("orc_mipchain rejected its arguments")
    return chain


def prefilter(env, ind_j, ind_t, chain, K: int, M: int, T: int = 64, texel_ids=None, threads=None):
    """Prefiltered pyramid values (double) [n, K+3] for the given mip-major texel
    ids (all texels when None).  Channels: K indicators, then RGB."""
    env = np.ascontiguousarray(env, dtype=np.float32)
    R = env.shape[1]
    if texel_ids is None:
        texel_ids = np.arange(pyramid_texels(R, M), dtype=np.int64)
    texel_ids = np.ascontiguousarray(texel_ids, dtype=np.int64)
    out = np.zeros((len(texel_ids), K + 3), np.float64)
    rc = lib().orc_prefilter_texels(_p(env, C.c_float), _p(ind_j, C.c_uint8), _p(ind_t, C.c_float),
                                    _p(chain, C.c_float), R, K, M, T, _p(texel_ids, C.c_int64),
                                    len(texel_ids), _p(out, C.c_double), threads or threads_default())
    if rc:
        raise ValueError("orc_prefilter_texels rejected its arguments")
    return out


def split_pyramid(values: np.ndarray, K: int):
    """[n, K+3] double -> (ind [n,K] float32, rgb [n,4] float32) as stored."""
    ind = values[:, :K].astype(np.float32)
    rgb = np.zeros((len(values), 4), np.float32)
    rgb[:, :3] = values[:, K:K + 3].astype(np.float32)
    return ind, rgb


def luts(cells=None, threads=None):
    """S = E_D / D_H and split-sum (A, B) on the 64x64 (sqrt(alpha), mu) grid.

    Returns (S [n] f64, A [n], B [n]) for cells = ia*64+im (all when None)."""
    if cells is None:
        cells = np.arange(LUT_N * LUT_N, dtype=np.int32)
    cells = np.ascontiguousarray(cells, dtype=np.int32)
    S = np.zeros(len(cells)); A = np.zeros(len(cells)); B = np.zeros(len(cells))
    rc = lib().orc_lut_cells(_p(cells, C.c_int), len(cells), _p(S, C.c_double), _p(A, C.c_double),
                             _p(B, C.c_double), threads or threads_default())
    if rc:
        raise ValueError("orc_lut_cells rejected its arguments")
    return S, A, B


def lut_tables(threads=None):
    """Full LUTs as stored (float32): S [64,64], E [64,64,2]."""
    S, A, B = luts(threads=threads)
    lut_S = S.astype(np.float32).reshape(LUT_N, LUT_N)
    lut_E = np.stack([A, B], axis=-1).astype(np.float32).reshape(LUT_N, LUT_N, 2)
    return lut_S, lut_E


GBUF_FIELDS = ("nx", "ny", "nz", "vx", "vy", "vz", "u", "v", "area", "ax", "ay", "density",
               "f0r", "f0g", "f0b", "surf_id")


SAMPLERS = {"dual": 0, "single": 1, "single-floor": 2, "dual-symmetric": 3}


def shade(gbuf: dict, ind_pyr, rgb_pyr, levels, lut_S, lut_E, R: int, K: int, M: int, seed: int,
          vertices: int = 1, pixels=None, threads=None, F=None, sampler: int = 0, prob_mode: int = 0,
          gamma: float = 1.0, lobe_taps: int = 0, tree: int = 0):
    """Glint radiance of the requested pixels (all when None).

    sampler: binomial approximation of every tree node, 0 dual-gated (Sec. 6
    Alg. "Dual-gated Gaussian"), 1 single-gated Eq. (gated), 2 the prior
    single-gated form Eq. (oldgated), 3 dual-gated with the bias of
    "Numeric Gating Issues" on both powers (the node's right-side
    probability computed on its own).
    tree: shape of the hierarchical multinomial, 0 balanced binary tree,
    1 sequential chain (bin i against the bins after it).
    prob_mode 1: one reflection probability gamma for every facet (the
    comparison method of Sec. 7), outputs laid out for K = 2.
    gbuf may carry "visibility" (float32 in [0, 1]) to attenuate the
    reflection probabilities.
    lobe_taps in {2, 4, 8}: anisotropic lookup along the lobe's major axis
    (gbuf must carry the tangent "tx", "ty", "tz").
    vertices 12: the footprint grid (gbuf must carry the uv Jacobian
    "dudx", "dudy", "dvdx", "dvdy").

    gbuf: dict of flat float32 arrays (surf_id uint32).  ind_pyr [texels,K]
    float32 and rgb_pyr [texels,4] float32 are the stored pyramids.  With F
    ([n,K], one row per requested pixel) the filtered indicator values are
    taken from F instead of the indicator pyramid (ind_pyr is then unused).
    Returns dict(radiance [n,3] f64, counts [n,V,K] f64, codes [n,V,K-1] u8,
    probs [n,K] f64, flags [n] u8).
    """
    fields = [np.ascontiguousarray(gbuf[k], dtype=np.uint32 if k == "surf_id" else np.float32)
              for k in GBUF_FIELDS]
    P = len(fields[0])
    if pixels is None:
        pixels = np.arange(P, dtype=np.int64)
    pixels = np.ascontiguousarray(pixels, dtype=np.int64)
    n = len(pixels)
    extra = [gbuf.get(k) for k in ("visibility", "tx", "ty", "tz", "dudx", "dudy", "dvdx", "dvdy")]
    extra = [None if a is None else np.ascontiguousarray(a, dtype=np.float32) for a in extra]
    keep = fields + [a for a in extra if a is not None]
    ptrs = [f.ctypes.data_as(C.POINTER(C.c_float)) for f in fields] + \
        [a.ctypes.data_as(C.POINTER(C.c_float)) if a is not None else C.POINTER(C.c_float)() for a in extra]
    arr = (C.POINTER(C.c_float) * 24)(*ptrs)
    if prob_mode == 1:
        K = 2
    gamma = float(np.float32(gamma))  # a float parameter, as in the C interface
    ind_pyr = np.ascontiguousarray(ind_pyr if F is None else np.zeros(1), dtype=np.float32)
    rgb_pyr = np.ascontiguousarray(rgb_pyr, dtype=np.float32)
    levels = np.ascontiguousarray(levels, dtype=np.float64)
    lut_S = np.ascontiguousarray(lut_S, dtype=np.float32)
    lut_E = np.ascontiguousarray(lut_E, dtype=np.float32)
    out = dict(radiance=np.zeros((n, 3)), counts=np.zeros((n, vertices, K)),
               codes=np.zeros((n, vertices, K - 1), np.uint8), probs=np.zeros((n, K)),
               flags=np.zeros(n, np.uint8))
    if F is not None:
        F = np.ascontiguousarray(F, dtype=np.float64).reshape(n, K)
        rc = lib().orc_shade_pixels_given_F(arr, _p(F, C.c_double), _p(rgb_pyr, C.c_float), _p(levels, C.c_double),
                                            _p(lut_S, C.c_float), _p(lut_E, C.c_float), R, K, M, seed, vertices,
                                            sampler, tree, _p(pixels, C.c_int64), n,
                                            _p(out["radiance"], C.c_double),
                                            _p(out["counts"], C.c_double), _p(out["codes"], C.c_uint8),
                                            _p(out["probs"], C.c_double), _p(out["flags"], C.c_uint8),
                                            threads or threads_default())
        if rc:
            raise ValueError("orc_shade_pixels_given_F rejected its arguments")
        return out
    rc = lib().orc_shade_pixels(arr, _p(ind_pyr, C.c_float), _p(rgb_pyr, C.c_float), _p(levels, C.c_double),
                                _p(lut_S, C.c_float), _p(lut_E, C.c_float), R, K, M, seed, vertices,
                                sampler, tree, prob_mode, gamma, lobe_taps, _p(pixels, C.c_int64), n,
                                _p(out["radiance"], C.c_double),
                                _p(out["counts"], C.c_double), _p(out["codes"], C.c_uint8),
                                _p(out["probs"], C.c_double), _p(out["flags"], C.c_uint8),
                                threads or threads_default())
    if rc:
        raise ValueError("orc_shade_pixels rejected its arguments")
    return out


def quantile_levels(env: np.ndarray, K: int, ell: float = 1e-3):
    """Quantile levels (level_mode 1) and, per level, the margin of its
    weighted distribution function to q W, over W."""
    env = np.ascontiguousarray(env, dtype=np.float32)
    R = env.shape[1]
    levels = np.zeros(K, np.float64)
    margin = np.zeros(K, np.float64)
    if lib().orc_quantile_levels(_p(env, C.c_float), R, K, ell, _p(levels, C.c_double), _p(margin, C.c_double)):
        raise ValueError("orc_quantile_levels rejected its arguments")
    return levels, margin


def frame(env, gbuf, K, M, T=64, ell=1e-3, seed=1, vertices=1, level_mode=0, weight_space=0, pixels=None,
          threads=None, lut=None):
    """Whole hot path on the CPU: partition -> mip chain -> prefilter -> LUTs ->
    shade.  Returns a dict with every intermediate."""
    levels, ind_j, ind_t = partition(env, K, ell, level_mode, weight_space)
    chain = mipchain(env, ind_j, ind_t, K, M)
    pyr = prefilter(env, ind_j, ind_t, chain, K, M, T, threads=threads)
    ind_pyr, rgb_pyr = split_pyramid(pyr, K)
    lut_S, lut_E = lut if lut is not None else lut_tables(threads)
    R = env.shape[1]
    sh = shade(gbuf, ind_pyr, rgb_pyr, levels, lut_S, lut_E, R, K, M, seed, vertices, pixels, threads)
    return dict(levels=levels, ind_j=ind_j, ind_t=ind_t, chain=chain, pyramid=pyr, ind_pyr=ind_pyr,
                rgb_pyr=rgb_pyr, lut_S=lut_S, lut_E=lut_E, **sh)


# --- small pieces, exposed for the definition tests --------------------------

def ppnd16(p: float) -> float:
    return lib().orc_ppnd16(float(p))


def hash_xi(seed, surf, level, a, b, node):
    x1, x2 = C.c_float(), C.c_float()
    lib().orc_hash_xi(seed, surf, level, a, b, node, C.byref(x1), C.byref(x2))
    return x1.value, x2.value


def pcg4d(words):
    """The per-footprint hash on an [n, 4] array of 32-bit words."""
    a = np.ascontiguousarray(words, dtype=np.uint32).reshape(-1, 4)
    out = np.empty_like(a)
    lib().orc_pcg4d(_p(a, C.c_uint32), _p(out, C.c_uint32), a.shape[0])
    return out


def gate_probs(N: float, p: float):
    out = np.zeros(4, np.float32)
    lib().orc_gate_probs(N, p, _p(out, C.c_float))
    return out  # P(n=N), P(n=1), P(nb=N), P(nb=1)


def gate_probs_symmetric(N: float, p: float, q: float):
    """Gating probabilities with the bias on both powers (q = 1 - p computed
    on its own): P(n=N), P(n=1), P(nb=N), P(nb=1)."""
    out = np.zeros(4, np.float32)
    lib().orc_gate_probs_symmetric(N, p, q, _p(out, C.c_float))
    return out


def dual_gated(N: float, p: float, xi1: float, xi2: float):
    n, nb, code = C.c_double(), C.c_double(), C.c_uint8()
    lib().orc_dual_gated(N, p, xi1, xi2, C.byref(n), C.byref(nb), C.byref(code))
    return n.value, nb.value, code.value


def multinomial(sampler: int, NP: float, p, seed: int, surf: int, level: int, a: int, b: int, tree: int = 0):
    """One hierarchical multinomial draw (Sec. 6) of N_P facets over the
    given probabilities, hashed as a V = 1 shading draw at lattice vertex
    (a, b) of `level`; tree 0 balanced binary tree, 1 sequential chain.
    Returns (counts [K], codes [K-1], flags)."""
    p = np.ascontiguousarray(p, dtype=np.float64)
    K = len(p)
    M = np.zeros(K)
    codes = np.zeros(K - 1, np.uint8)
    fl = lib().orc_multinomial(sampler, tree, float(NP), _p(p, C.c_double), K, seed, surf, level, a, b,
                               _p(M, C.c_double), _p(codes, C.c_uint8))
    if fl < 0:
        raise ValueError("orc_multinomial rejected its arguments")
    return M, codes, fl


def sample_binomial(sampler: int, N, p, h1, h2, threads=None):
    """Binomial approximation of Sec. 6 for each element (sampler as in
    shade), with the random words h1 (gate) and h2 (Gaussian) mapped to
    (0,1) as the hash outputs are.  Returns dict(n, nb, code, flags)."""
    N = np.ascontiguousarray(N, dtype=np.float64)
    p = np.ascontiguousarray(p, dtype=np.float64)
    h1 = np.ascontiguousarray(h1, dtype=np.uint32)
    h2 = np.ascontiguousarray(h2, dtype=np.uint32)
    m = len(N)
    if not (len(p) == len(h1) == len(h2) == m):
        raise ValueError("length mismatch")
    out = dict(n=np.zeros(m), nb=np.zeros(m), code=np.zeros(m, np.uint8), flags=np.zeros(m, np.uint8))
    rc = lib().orc_sample_binomial(sampler, _p(N, C.c_double), _p(p, C.c_double), _p(h1, C.c_uint32),
                                   _p(h2, C.c_uint32), m, _p(out["n"], C.c_double), _p(out["nb"], C.c_double),
                                   _p(out["code"], C.c_uint8), _p(out["flags"], C.c_uint8),
                                   threads or threads_default())
    if rc:
        raise ValueError("orc_sample_binomial rejected its arguments")
    return out


def footprint_grid(u, v, dudx, dudy, dvdx, dvdy):
    """The footprint grid's 12 draws of one pixel: dict(w, r, key, a, b,
    flag), or None for a degenerate Jacobian."""
    w, r = np.zeros(12), np.zeros(12)
    key = np.zeros(12, np.uint32)
    a, b = np.zeros(12, np.int64), np.zeros(12, np.int64)
    rc = lib().orc_footprint_grid(u, v, dudx, dudy, dvdx, dvdy, _p(w, C.c_double), _p(r, C.c_double),
                                  _p(key, C.c_uint32), _p(a, C.c_int64), _p(b, C.c_int64))
    if rc < 0:
        return None
    return dict(w=w, r=r, key=key, a=a, b=b, flag=rc)


def face_dir(face, s, t):
    d = np.zeros(3)
    lib().orc_face_dir(face, s, t, _p(d, C.c_double))
    return d


def dir_face(d):
    d = np.ascontiguousarray(d, dtype=np.float64)
    st = np.zeros(2)
    f = lib().orc_dir_face(_p(d, C.c_double), _p(st, C.c_double))
    return f, st[0], st[1]


def lattice_level(area):
    fr = C.c_double()
    l0 = lib().orc_lattice_level(float(area), C.byref(fr))
    return l0, fr.value


def taps(m, M, T, R):
    out = np.zeros((T, 5))
    lib().orc_taps(m, M, T, R, _p(out, C.c_double))
    return out


def pyramid_lookup(pyr, R, M, dirs, lods):
    """Trilinear seamless lookup of a float pyramid [texels, C] at dirs [n,3]."""
    pyr = np.ascontiguousarray(pyr, dtype=np.float32)
    dirs = np.ascontiguousarray(dirs, dtype=np.float64).reshape(-1, 3)
    lods = np.ascontiguousarray(np.broadcast_to(lods, (len(dirs),)), dtype=np.float64)
    Cn = pyr.shape[1]
    out = np.zeros((len(dirs), Cn))
    lib().orc_pyramid_lookup(_p(pyr, C.c_float), R, M, Cn, _p(dirs, C.c_double), _p(lods, C.c_double), len(dirs),
                             _p(out, C.c_double))
    return out


def sample_filter(env, ind_j, ind_t, chain, K, M, T, dirs, alphas, threads=None):
    """The prefilter's quadrature at arbitrary (direction, alpha): [n, K+3] double."""
    env = np.ascontiguousarray(env, dtype=np.float32)
    R = env.shape[1]
    dirs = np.ascontiguousarray(dirs, dtype=np.float64).reshape(-1, 3)
    alphas = np.ascontiguousarray(np.broadcast_to(alphas, (len(dirs),)), dtype=np.float64)
    out = np.zeros((len(dirs), K + 3))
    rc = lib().orc_sample_filter(_p(env, C.c_float), _p(ind_j, C.c_uint8), _p(ind_t, C.c_float),
                                 _p(chain, C.c_float), R, K, M, T, _p(dirs, C.c_double), _p(alphas, C.c_double),
                                 len(dirs), _p(out, C.c_double), threads or threads_default())
    if rc:
        raise ValueError("orc_sample_filter rejected its arguments")
    return out
