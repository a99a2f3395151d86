"""Seeded synthetic inputs for the glint hot path (shared by tests, smoke and bench).

This module synthesises *inputs only*: environment cube maps and G-buffers
(surface normal, view vector, uv, footprint area, material).  It holds none of
the method's arithmetic (no partition, filtering, probabilities or sampling).
The paper's environment maps and scenes are not available, so these stand in
for them:

* environment: sky gradient + ground + 3 seeded Gaussian sun lobes of
  radiance 10-1000 (high dynamic range, as the paper's HDR captures);
* ``tiny``: orthographic unit sphere, 128x128, isotropic GGX alpha = 0.1,
  density 1e4 per unit area;
* ``frame``: pinhole camera, unit sphere + bounded ground plane, seeded value
  noise for anisotropic alpha in [0.02, 0.5] and log-uniform density.

Cube-map layout (a storage format shared with the library's documentation):
``env[face][y][x][rgb]`` float32, faces +X,-X,+Y,-Y,+Z,-Z, texel centre
s = 2(x+1/2)/R - 1, t = 2(y+1/2)/R - 1, direction +X:(1,-t,-s) -X:(-1,-t,s)
+Y:(s,1,t) -Y:(s,-1,-t) +Z:(s,-t,1) -Z:(-s,-t,-1).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

GBUF_FIELDS = ("nx", "ny", "nz", "vx", "vy", "vz", "u", "v", "area", "ax", "ay", "density",
               "f0r", "f0g", "f0b", "surf_id")
NO_SURFACE = 0xFFFFFFFF


def _face_dirs(R: int) -> np.ndarray:
    c = (np.arange(R) + 0.5) * (2.0 / R) - 1.0
    t, s = np.meshgrid(c, c, indexing="ij")  # t along rows (y), s along columns (x)
    one = np.ones_like(s)
    faces = [
        (one, -t, -s), (-one, -t, s), (s, one, t), (s, -one, -t), (s, -t, one), (-s, -t, -one),
    ]
    d = np.stack([np.stack(f, axis=-1) for f in faces])  # [6,R,R,3]
    return d / np.linalg.norm(d, axis=-1, keepdims=True)


def make_env(R: int, seed: int, suns: int = 3, frame: int = 0) -> np.ndarray:
    """Sky gradient + ground + seeded sun lobes; returns [6,R,R,3] float32.

    frame > 0: the rotating-sun sequence of the surrogate workload, sun s's
    azimuth advanced by 2 (s + 1) degrees per frame (each sun at its own
    rate, so the map changes non-rigidly); frame 0 is the static map."""
    rng = np.random.default_rng(seed)
    d = _face_dirs(R)
    y = d[..., 1]
    sky = np.array([0.20, 0.35, 0.80]) * (0.25 + 0.75 * np.clip(y, 0.0, 1.0))[..., None]
    ground = np.broadcast_to(np.array([0.04, 0.035, 0.03]), d.shape)
    env = np.where((y >= 0.0)[..., None], sky, ground).astype(np.float64)
    for sun in range(suns):
        amp = 10.0 ** rng.uniform(1.0, 3.0)
        el = math.radians(rng.uniform(10.0, 70.0))
        az = math.radians(rng.uniform(0.0, 360.0) + 2.0 * (sun + 1) * frame)
        sigma = rng.uniform(1.5, 4.0) * (math.pi / 2.0) / R
        sd = np.array([math.cos(el) * math.sin(az), math.sin(el), math.cos(el) * math.cos(az)])
        cos_t = d @ sd
        lobe = amp * np.exp((cos_t - 1.0) / (sigma * sigma))
        env += lobe[..., None] * np.array([1.0, 0.95, 0.85])
    return np.ascontiguousarray(env.astype(np.float32))


def uniform_env(R: int, value: float = 1.0) -> np.ndarray:
    return np.full((6, R, R, 3), value, np.float32)


def disc_env(R: int, lights, background: float = 0.05) -> np.ndarray:
    """Grey map of constant background luminance with constant-luminance
    discs: lights = [(elevation_deg, azimuth_deg, radius_deg, luminance)];
    a texel belongs to the first disc containing its centre direction."""
    d = _face_dirs(R)
    env = np.full(d.shape[:3], background, np.float64)
    done = np.zeros(d.shape[:3], bool)
    for (el, az, rad, lum) in lights:
        e, a = math.radians(el), math.radians(az)
        c = np.array([math.cos(e) * math.sin(a), math.sin(e), math.cos(e) * math.cos(a)])
        inside = (d @ c >= math.cos(math.radians(rad))) & ~done
        env[inside] = lum
        done |= inside
    return np.ascontiguousarray(np.repeat(env[..., None], 3, axis=-1).astype(np.float32))


def sweep_plane(elevations_deg, np_rows, alpha: float, azimuth_deg: float = 0.0, area: float = 1e-4,
                f0: float = 0.9) -> dict:
    """A flat surface (normal +y) seen so that column c reflects towards
    elevation elevations_deg[c] (azimuth azimuth_deg) and row r holds
    np_rows[r] facets per footprint; isotropic roughness alpha, footprint
    area `area`, uv spaced so that every pixel draws at its own lattice
    vertex."""
    el = np.radians(np.asarray(elevations_deg, np.float64))
    NP = np.asarray(np_rows, np.float64)
    W, H = len(el), len(NP)
    a = math.radians(azimuth_deg)
    wr = np.stack([np.cos(el) * math.sin(a), np.sin(el), np.cos(el) * math.cos(a)], -1)  # [W,3]
    n = np.array([0.0, 1.0, 0.0])
    v = 2.0 * (wr @ n)[:, None] * n[None] - wr
    P = W * H
    g = _empty_gbuf(P)
    cols = np.tile(np.arange(W), H)
    rows = np.repeat(np.arange(H), W)
    g["nx"][:], g["ny"][:], g["nz"][:] = 0.0, 1.0, 0.0
    g["vx"][:], g["vy"][:], g["vz"][:] = v[cols, 0], v[cols, 1], v[cols, 2]
    step = 4.0 * math.sqrt(area)  # a few lattice spacings apart
    g["u"][:], g["v"][:] = cols * step, rows * step
    g["area"][:] = area
    g["ax"][:] = alpha
    g["ay"][:] = alpha
    g["density"][:] = NP[rows] / area
    g["f0r"][:] = g["f0g"][:] = g["f0b"][:] = f0
    g["surf_id"][:] = 3
    return _finish(g)


# --- value noise ---------------------------------------------------------------

def _splitmix64(x: np.ndarray) -> np.ndarray:
    x = x.astype(np.uint64)
    with np.errstate(over="ignore"):
        x = x + np.uint64(0x9E3779B97F4A7C15)
        z = x
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return z


def value_noise(u: np.ndarray, v: np.ndarray, seed: int, channel: int, cells_per_unit: float = 8.0):
    """Smooth value noise in [0,1] on a square lattice (seeded hash per vertex)."""
    x = u * cells_per_unit
    y = v * cells_per_unit
    ix = np.floor(x)
    iy = np.floor(y)
    fx = x - ix
    fy = y - iy

    def lat(i, j):
        key = ((i.astype(np.int64) & 0xFFFFFF).astype(np.uint64) << np.uint64(24)) | \
              (j.astype(np.int64) & 0xFFFFFF).astype(np.uint64)
        key = key ^ (np.uint64(seed & 0xFFFF) << np.uint64(48)) ^ (np.uint64(channel & 0xFF) << np.uint64(56))
        return (_splitmix64(key) >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)

    sx = fx * fx * (3.0 - 2.0 * fx)
    sy = fy * fy * (3.0 - 2.0 * fy)
    a = lat(ix, iy); b = lat(ix + 1, iy); c = lat(ix, iy + 1); d = lat(ix + 1, iy + 1)
    return (a * (1 - sx) + b * sx) * (1 - sy) + (c * (1 - sx) + d * sx) * sy


# --- G-buffers -----------------------------------------------------------------

def _empty_gbuf(P: int) -> dict:
    g = {k: np.zeros(P, np.float64) for k in GBUF_FIELDS if k != "surf_id"}
    g["surf_id"] = np.full(P, NO_SURFACE, np.uint32)
    return g


def _finish(g: dict) -> dict:
    out = {}
    for k in GBUF_FIELDS:
        out[k] = np.ascontiguousarray(g[k].astype(np.uint32 if k == "surf_id" else np.float32))
    return out


def _sphere_uv(n):
    u = np.arctan2(n[:, 0], n[:, 2]) / (2.0 * np.pi) + 0.5
    v = np.arccos(np.clip(n[:, 1], -1.0, 1.0)) / np.pi
    return u, v


def scene_tiny(W: int = 128, H: int = 128, alpha: float = 0.1, density: float = 1e4, f0: float = 0.9) -> dict:
    """Orthographic view along -Z of the unit sphere over [-1,1]^2."""
    j, i = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    x = (-1.0 + (i + 0.5) * 2.0 / W).ravel()
    y = (1.0 - (j + 0.5) * 2.0 / H).ravel()
    P = W * H
    g = _empty_gbuf(P)
    hit = x * x + y * y < 1.0
    z = np.sqrt(np.clip(1.0 - x * x - y * y, 0.0, None))
    n = np.stack([x, y, z], -1)[hit]
    g["nx"][hit], g["ny"][hit], g["nz"][hit] = n[:, 0], n[:, 1], n[:, 2]
    g["vz"][hit] = 1.0
    g["area"][hit] = (2.0 / W) * (2.0 / H) / n[:, 2]
    u, v = _sphere_uv(n)
    g["u"][hit], g["v"][hit] = u, v
    g["ax"][hit] = alpha
    g["ay"][hit] = alpha
    g["density"][hit] = density
    g["f0r"][hit] = g["f0g"][hit] = g["f0b"][hit] = f0
    g["surf_id"][hit] = 1
    return _finish(g)


def scene_frame(W: int, H: int, seed: int = 7, density_decades=(6.0, 9.0), eye=(0.0, 0.6, 4.0),
                target=(0.0, -0.2, 0.0), vfov_deg: float = 40.0, plane_half: float = 20.0) -> dict:
    """Pinhole view of the unit sphere and the bounded plane y = -1.

    Footprint area from the pixel's solid angle: |P| = t^2 dOmega / |<d,n>|.
    Materials from seeded value noise: alpha_x, alpha_y = 0.02 * 25^eta,
    density = 10^(lo + (hi-lo) eta)."""
    eye = np.array(eye, np.float64)
    fwd = np.array(target, np.float64) - eye
    fwd /= np.linalg.norm(fwd)
    right = np.cross(fwd, np.array([0.0, 1.0, 0.0]))
    right /= np.linalg.norm(right)
    up = np.cross(right, fwd)
    th = math.tan(math.radians(vfov_deg) * 0.5)
    j, i = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    xs = ((2.0 * (i + 0.5) / W - 1.0) * th * W / H).ravel()
    ys = ((1.0 - 2.0 * (j + 0.5) / H) * th).ravel()
    d = fwd[None] + xs[:, None] * right[None] + ys[:, None] * up[None]
    dlen = np.linalg.norm(d, axis=1)
    d /= dlen[:, None]
    pix = 2.0 * th / H
    cos_cam = d @ fwd
    domega = pix * pix * cos_cam ** 3
    P = W * H
    # sphere
    b = d @ eye
    c = eye @ eye - 1.0
    disc = b * b - c
    ts = np.where(disc > 0.0, -b - np.sqrt(np.clip(disc, 0.0, None)), np.inf)
    ts = np.where(ts > 1e-6, ts, np.inf)
    # plane y = -1
    with np.errstate(divide="ignore", invalid="ignore"):
        tp = np.where(d[:, 1] < 0.0, (-1.0 - eye[1]) / d[:, 1], np.inf)
    hp = eye[None] + np.where(np.isfinite(tp), tp, 0.0)[:, None] * d
    inside = (np.abs(hp[:, 0]) <= plane_half) & (np.abs(hp[:, 2]) <= plane_half) & np.isfinite(tp)
    tp = np.where(inside, tp, np.inf)
    g = _empty_gbuf(P)
    on_s = np.isfinite(ts) & (ts <= tp)
    on_p = np.isfinite(tp) & ~on_s
    lo, hi = density_decades
    for mask, t, sid in ((on_s, ts, 1), (on_p, tp, 2)):
        if not mask.any():
            continue
        dd = d[mask]
        hitp = eye[None] + t[mask][:, None] * dd
        if sid == 1:
            n = hitp / np.linalg.norm(hitp, axis=1, keepdims=True)
            u, v = _sphere_uv(n)
            f0 = np.array([0.95, 0.95, 0.95])
        else:
            n = np.tile(np.array([0.0, 1.0, 0.0]), (len(dd), 1))
            u, v = hitp[:, 0], hitp[:, 2]
            f0 = np.array([0.9, 0.7, 0.4])
        cosn = np.abs(np.sum(dd * n, axis=1))
        g["nx"][mask], g["ny"][mask], g["nz"][mask] = n[:, 0], n[:, 1], n[:, 2]
        g["vx"][mask], g["vy"][mask], g["vz"][mask] = -dd[:, 0], -dd[:, 1], -dd[:, 2]
        g["u"][mask], g["v"][mask] = u, v
        g["area"][mask] = t[mask] ** 2 * domega[mask] / np.maximum(cosn, 1e-6)
        e1 = value_noise(u, v, seed, 1)
        e2 = value_noise(u, v, seed, 2)
        e3 = value_noise(u, v, seed, 3)
        g["ax"][mask] = 0.02 * 25.0 ** e1
        g["ay"][mask] = 0.02 * 25.0 ** e2
        g["density"][mask] = 10.0 ** (lo + (hi - lo) * e3)
        g["f0r"][mask], g["f0g"][mask], g["f0b"][mask] = f0[0], f0[1], f0[2]
        g["surf_id"][mask] = sid
    return _finish(g)


def contact_visibility(g: dict) -> np.ndarray:
    """Occlusion stand-in for the sphere-and-plane scene (an ambient-occlusion
    like field, float32 in [0, 1]): on the plane (surface 2) it falls to 0.2
    towards the sphere's contact point at the uv origin, on the sphere
    (surface 1) from 1 at the top to 0.6 at the bottom; 1 elsewhere."""
    vis = np.ones(len(g["nx"]), np.float32)
    sphere = g["surf_id"] == 1
    plane = g["surf_id"] == 2
    vis[sphere] = 0.6 + 0.4 * np.clip(0.5 * g["ny"][sphere] + 0.5, 0.0, 1.0)
    r = np.hypot(g["u"][plane].astype(np.float64), g["v"][plane].astype(np.float64))
    vis[plane] = np.clip(0.2 + 0.8 * (r - 0.2) / 1.3, 0.2, 1.0)
    return vis


def _camera_rays(W, H, px, py, eye, target, vfov_deg):
    """Unit ray directions through image positions (px, py) in pixels."""
    eye = np.array(eye, np.float64)
    fwd = np.array(target, np.float64) - eye
    fwd /= np.linalg.norm(fwd)
    right = np.cross(fwd, np.array([0.0, 1.0, 0.0]))
    right /= np.linalg.norm(right)
    up = np.cross(right, fwd)
    th = math.tan(math.radians(vfov_deg) * 0.5)
    xs = (2.0 * px / W - 1.0) * th * W / H
    ys = (1.0 - 2.0 * py / H) * th
    d = fwd[None] + xs[:, None] * right[None] + ys[:, None] * up[None]
    return d / np.linalg.norm(d, axis=1, keepdims=True)


def _scene_uv(d, eye, plane_half):
    """Surface id (1 sphere, 2 plane, 0 none) and uv of the first hit."""
    eye = np.array(eye, np.float64)
    b = d @ eye
    disc = b * b - (eye @ eye - 1.0)
    ts = np.where(disc > 0.0, -b - np.sqrt(np.clip(disc, 0.0, None)), np.inf)
    ts = np.where(ts > 1e-6, ts, np.inf)
    with np.errstate(divide="ignore", invalid="ignore"):
        tp = np.where(d[:, 1] < 0.0, (-1.0 - eye[1]) / d[:, 1], np.inf)
    hp = eye[None] + np.where(np.isfinite(tp), tp, 0.0)[:, None] * d
    inside = (np.abs(hp[:, 0]) <= plane_half) & (np.abs(hp[:, 2]) <= plane_half) & np.isfinite(tp)
    tp = np.where(inside, tp, np.inf)
    sid = np.zeros(len(d), np.int64)
    on_s = np.isfinite(ts) & (ts <= tp)
    on_p = np.isfinite(tp) & ~on_s
    sid[on_s], sid[on_p] = 1, 2
    uv = np.zeros((len(d), 2))
    hs = eye[None] + ts[on_s][:, None] * d[on_s]
    uv[on_s] = np.stack(_sphere_uv(hs / np.linalg.norm(hs, axis=1, keepdims=True)), -1)
    hq = eye[None] + tp[on_p][:, None] * d[on_p]
    uv[on_p] = hq[:, [0, 2]]
    return sid, uv


def uv_jacobian(g: dict, W: int, H: int, eye=(0.0, 0.6, 4.0), target=(0.0, -0.2, 0.0), vfov_deg: float = 40.0,
                plane_half: float = 20.0):
    """Pixel footprint of scene_frame's camera as the uv Jacobian (float32
    dudx, dudy, dvdx, dvdy): differences of the uv hit by rays half a pixel
    to either side (one-sided where a side leaves the surface, longitude
    wrapped), zero where both sides do."""
    j, i = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    i, j = i.ravel().astype(np.float64) + 0.5, j.ravel().astype(np.float64) + 0.5
    sid0 = g["surf_id"].astype(np.int64)
    sid0 = np.where(sid0 == NO_SURFACE, 0, sid0)
    _, uv0 = _scene_uv(_camera_rays(W, H, i, j, eye, target, vfov_deg), eye, plane_half)
    out = []
    for dx, dy in ((0.5, 0.0), (0.0, 0.5)):
        sp, uvp = _scene_uv(_camera_rays(W, H, i + dx, j + dy, eye, target, vfov_deg), eye, plane_half)
        sm, uvm = _scene_uv(_camera_rays(W, H, i - dx, j - dy, eye, target, vfov_deg), eye, plane_half)
        okp, okm = (sp == sid0) & (sid0 > 0), (sm == sid0) & (sid0 > 0)
        dp, dm = uvp - uv0, uv0 - uvm
        for dd in (dp, dm):
            dd[:, 0] = np.where(sid0 == 1, (dd[:, 0] + 0.5) % 1.0 - 0.5, dd[:, 0])
        deriv = np.where((okp & okm)[:, None], dp + dm, np.where(okp[:, None], 2 * dp, np.where(okm[:, None], 2 * dm, 0.0)))
        out.append(deriv)
    ddx, ddy = out
    return (ddx[:, 0].astype(np.float32), ddy[:, 0].astype(np.float32), ddx[:, 1].astype(np.float32),
            ddy[:, 1].astype(np.float32))


def surface_tangents(g: dict):
    """Tangent of the alpha_x axis for the sphere-and-plane scene (float32
    tx, ty, tz): on the sphere the direction of increasing longitude u
    (normalised (n_z, 0, -n_x), (1, 0, 0) at the poles), on the plane +x
    (the u axis); (1, 0, 0) elsewhere."""
    P = len(g["nx"])
    t = np.zeros((P, 3))
    t[:, 0] = 1.0
    sphere = g["surf_id"] == 1
    nx, nz = g["nx"][sphere].astype(np.float64), g["nz"][sphere].astype(np.float64)
    ln = np.hypot(nx, nz)
    ok = ln > 1e-9
    ts = np.zeros((sphere.sum(), 3))
    ts[:, 0] = 1.0
    ts[ok, 0] = nz[ok] / ln[ok]
    ts[ok, 2] = -nx[ok] / ln[ok]
    t[sphere] = ts
    return t[:, 0].astype(np.float32), t[:, 1].astype(np.float32), t[:, 2].astype(np.float32)


def n_sweep(W: int = 512, rows: int = 64, max_decades: float = 12.0, seed: int = 5) -> dict:
    """Counts sweep: row r has N_P = 10^(max_decades r / (rows-1)) (1 .. 1e12,
    the range where float counts lose integers); along a row the normal tilts
    and the roughness runs log-uniformly over [0.02, 0.5], so each row sees a
    fixed pattern of reflection probabilities.  Footprint area 1e-4."""
    j, i = np.meshgrid(np.arange(rows), np.arange(W), indexing="ij")
    j, i = j.ravel(), i.ravel()
    P = W * rows
    g = _empty_gbuf(P)
    rng = np.random.default_rng(seed)
    phi = 2.0 * np.pi * i / W
    tilt = 0.25 + 0.5 * ((i * 7) % W) / W
    n = np.stack([np.sin(tilt) * np.cos(phi), np.cos(tilt), np.sin(tilt) * np.sin(phi)], -1)
    g["nx"][:], g["ny"][:], g["nz"][:] = n[:, 0], n[:, 1], n[:, 2]
    v = np.stack([np.zeros(P), np.ones(P), np.zeros(P)], -1)
    g["vx"][:], g["vy"][:], g["vz"][:] = v[:, 0], v[:, 1], v[:, 2]
    g["u"][:] = rng.uniform(-40.0, 40.0, P)
    g["v"][:] = rng.uniform(-40.0, 40.0, P)
    g["area"][:] = 1e-4
    a = 0.02 * 25.0 ** (((i * 13) % W) / (W - 1.0))
    g["ax"][:] = a
    g["ay"][:] = a * (0.5 + ((i * 5) % W) / W)
    g["density"][:] = 10.0 ** (max_decades * j / (rows - 1.0)) / 1e-4
    g["f0r"][:] = g["f0g"][:] = g["f0b"][:] = 0.9
    g["surf_id"][:] = 1 + j
    return _finish(g)


def subsample_gbuf(g: dict, pixels: np.ndarray) -> dict:
    return {k: np.ascontiguousarray(v[pixels]) for k, v in g.items()}


# --- workloads -----------------------------------------------------------------

@dataclass(frozen=True)
class Workload:
    name: str
    R: int
    M: int
    K: int
    T: int
    W: int
    H: int
    env_seed: int
    scene: str
    ell: float = 1e-3
    hash_seed: int = 1
    density_decades: tuple = (6.0, 9.0)
    vertices: int = 1
    extra: dict = field(default_factory=dict)

    def env(self) -> np.ndarray:
        key = ("env", self.name)
        if key not in _CACHE:
            _CACHE[key] = make_env(self.R, self.env_seed)
        return _CACHE[key].copy()

    def gbuf(self) -> dict:
        """The workload's G-buffer (generated once per process; every call
        returns fresh copies of the arrays)."""
        key = ("gbuf", self.name)
        if key not in _CACHE:
            if self.scene == "tiny":
                _CACHE[key] = scene_tiny(self.W, self.H)
            else:
                _CACHE[key] = scene_frame(self.W, self.H, seed=self.env_seed + 5,
                                          density_decades=self.density_decades)
        return {k: v.copy() for k, v in _CACHE[key].items()}


_CACHE = {}


WORKLOADS = {
    # small case the oracle finishes in seconds
    "tiny": Workload("tiny", R=32, M=6, K=4, T=64, W=128, H=128, env_seed=1, scene="tiny"),
    # per-frame prefilter + shade at frame size (the headline workload)
    "frame": Workload("frame", R=256, M=8, K=8, T=64, W=1920, H=1080, env_seed=2, scene="frame"),
    # larger map and frame, density up to 1e10
    "precision": Workload("precision", R=512, M=9, K=8, T=64, W=2560, H=1440, env_seed=3, scene="frame",
                          density_decades=(6.0, 10.0)),
}


def batched_views(n_views: int = 64, seed: int = 11, max_pixels: int = 1920 * 1080, min_pixels: int = 256 * 256,
                  n_env: int = 4):
    """Views of uneven size for the batched frame: pixel counts log-uniform in
    [min_pixels, max_pixels], aspect ratios 1, 4:3 or 16:9, cameras on seeded
    orbits around the sphere+plane scene, per-view density decades.
    Returns a list of (gbuf, env_index, hash_seed, vertices)."""
    rng = np.random.default_rng(seed)
    out = []
    for v in range(n_views):
        px = math.exp(rng.uniform(math.log(min_pixels), math.log(max_pixels)))
        aspect = [1.0, 4.0 / 3.0, 16.0 / 9.0][rng.integers(3)]
        H = max(16, int(round(math.sqrt(px / aspect))))
        W = max(16, int(round(H * aspect)))
        az = rng.uniform(0, 2 * math.pi)
        dist = rng.uniform(3.0, 6.0)
        eye = (dist * math.sin(az), rng.uniform(0.2, 1.5), dist * math.cos(az))
        lo = rng.uniform(4.0, 7.0)
        gb = scene_frame(W, H, seed=100 + v, density_decades=(lo, lo + rng.uniform(1.0, 3.0)), eye=eye,
                         target=(0.0, -0.3, 0.0))
        out.append((gb, v % n_env, 1000 + v, 1))
    return out


BATCHED_ENVS = ((101, 4), (102, 8), (103, 16), (104, 8))  # (seed, K); each map 6x256x256, 8 mips
