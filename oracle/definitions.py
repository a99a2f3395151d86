"""Plain definitions (numpy/scipy) that pin the step-by-step oracle.

TEST INFRASTRUCTURE ONLY.  These evaluate what the paper *defines* rather than
how the method approximates it, so the distance between the two is measured:

* GGX NDF and its total microfacet area D_H (Sec. 3.2: D_H = integral of D
  over the hemisphere, >= 1), closed form;
* the IBL filtering kernel written as a direct sum over every environment
  texel (Sec. 3.4, Eq. (rtibl), kernel assumed n = v = r), with exact texel
  solid angles -- the brute-force counterpart of the importance-sampled
  quadrature;
* the visible reflecting facet area E_D and the split-sum albedo E_rho as
  integrals over incident directions (a parameterisation different from the
  oracle's half-vector quadrature);
* explicit microfacets (Sec. 3.2, Eq. (discrete_ndf)): N_P facets with
  normals distributed as D/D_H, each reflecting from the region its mirror
  direction falls in.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import integrate


def ggx_D(cos_h: np.ndarray, alpha: float) -> np.ndarray:
    """Isotropic GGX (Trowbridge-Reitz) NDF."""
    a2 = alpha * alpha
    c2 = cos_h * cos_h
    den = c2 * (a2 - 1.0) + 1.0
    return np.where(cos_h > 0, a2 / (math.pi * den * den), 0.0)


def total_facet_area(alpha: float) -> float:
    """D_H = integral of D over the hemisphere (closed form, derived by
    substituting y = cos(theta)): 1 + alpha^2 atanh(b)/b, b = sqrt(1-alpha^2)."""
    if alpha >= 1.0:
        return 2.0 if alpha == 1.0 else 1.0 + alpha * alpha * math.atan(math.sqrt(alpha * alpha - 1)) / math.sqrt(alpha * alpha - 1)
    b = math.sqrt(1.0 - alpha * alpha)
    return 1.0 + alpha * alpha * math.atanh(b) / b


def smith_lambda(mu, alpha):
    mu = np.asarray(mu, dtype=np.float64)
    t2 = (1.0 - mu * mu) / (mu * mu)
    return 0.5 * (-1.0 + np.sqrt(1.0 + alpha * alpha * t2))


def visible_facet_area(mu_o: float, alpha: float) -> float:
    """E_D(w_o) = integral over incident directions l (upper hemisphere) of
    D(h)/(4<h,l>), h the half vector of w_o and l (Sec. 5 "Integrated NDF")."""
    so = math.sqrt(1.0 - mu_o * mu_o)
    wo = np.array([so, 0.0, mu_o])

    def f(phi, th):
        l = np.array([math.sin(th) * math.cos(phi), math.sin(th) * math.sin(phi), math.cos(th)])
        h = wo + l
        nh = np.linalg.norm(h)
        if nh == 0:
            return 0.0
        h /= nh
        hl = float(h @ l)
        if hl <= 0:
            return 0.0
        return float(ggx_D(np.array(h[2]), alpha)) / (4.0 * hl) * math.sin(th)

    val, _ = integrate.dblquad(f, 0.0, math.pi / 2, 0.0, 2 * math.pi, epsabs=1e-10, epsrel=1e-8)
    return val


def split_sum_albedo(mu_o: float, alpha: float):
    """E_rho = F0 A + B: integral of Schlick F x height-correlated Smith G2 x D
    / (4 mu_o mu_i) x mu_i over incident directions."""
    so = math.sqrt(1.0 - mu_o * mu_o)
    wo = np.array([so, 0.0, mu_o])
    lam_o = float(smith_lambda(mu_o, alpha))

    def integrand(phi, th, which):
        l = np.array([math.sin(th) * math.cos(phi), math.sin(th) * math.sin(phi), math.cos(th)])
        mu_i = l[2]
        if mu_i <= 0:
            return 0.0
        h = wo + l
        h /= np.linalg.norm(h)
        vh = float(h @ wo)
        if vh <= 0:
            return 0.0
        g2 = 1.0 / (1.0 + lam_o + float(smith_lambda(mu_i, alpha)))
        fc = (1.0 - vh) ** 5
        d = float(ggx_D(np.array(h[2]), alpha))
        base = g2 * d / (4.0 * mu_o) * math.sin(th)
        return (1.0 - fc) * base if which == 0 else fc * base

    A, _ = integrate.dblquad(lambda p, t: integrand(p, t, 0), 0.0, math.pi / 2, 0.0, 2 * math.pi,
                             epsabs=1e-9, epsrel=1e-7)
    B, _ = integrate.dblquad(lambda p, t: integrand(p, t, 1), 0.0, math.pi / 2, 0.0, 2 * math.pi,
                             epsabs=1e-9, epsrel=1e-7)
    return A, B


# --- cube map helpers (independent numpy implementation) ----------------------

def face_dirs(R: int) -> np.ndarray:
    c = (np.arange(R) + 0.5) * (2.0 / R) - 1.0
    t, s = np.meshgrid(c, c, indexing="ij")
    one = np.ones_like(s)
    faces = [(one, -t, -s), (-one, -t, s), (s, one, t), (s, -one, -t), (s, -t, one), (-s, -t, -one)]
    d = np.stack([np.stack(f, axis=-1) for f in faces])
    return d / np.linalg.norm(d, axis=-1, keepdims=True)


def texel_solid_angles(R: int) -> np.ndarray:
    """Exact solid angle of every cube texel: the area element of the unit
    cube face projected on the sphere, integrated over the texel via
    F(x,y) = atan2(xy, sqrt(x^2+y^2+1))."""
    e = np.linspace(-1.0, 1.0, R + 1)

    def F(x, y):
        return np.arctan2(x * y, np.sqrt(x * x + y * y + 1.0))

    y0, x0 = np.meshgrid(e[:-1], e[:-1], indexing="ij")
    y1, x1 = np.meshgrid(e[1:], e[1:], indexing="ij")
    w = F(x1, y1) - F(x0, y1) - F(x1, y0) + F(x0, y0)
    return np.broadcast_to(w, (6, R, R)).copy()


def dense_level0(ind_j, ind_t, env, K):
    """Dense indicator weights (Eq. (wkdefpractice)) + RGB per texel: [6,R,R,K+3]."""
    R = ind_j.shape[1]
    out = np.zeros((6, R, R, K + 3))
    t = ind_t.astype(np.float64)
    j = ind_j.astype(np.int64)
    np.put_along_axis(out, j[..., None], (1.0 - t)[..., None], axis=-1)
    np.put_along_axis(out, (j + 1)[..., None], t[..., None], axis=-1)
    e = env.astype(np.float64)
    e = np.where(np.isfinite(e) & (e > 0), e, 0.0)
    out[..., K:] = e
    return out


def brute_force_filter(values: np.ndarray, r: np.ndarray, alpha: float) -> np.ndarray:
    """Direct sum of the IBL kernel over every texel: K(l) ~ D(h) <r,l>+ (the
    importance-sampled kernel of the quadrature, pdf_l = D/4 with n = v = r,
    weighted by <r,l>+), times the texel solid angle, normalised."""
    R = values.shape[1]
    d = face_dirs(R).reshape(-1, 3)
    om = texel_solid_angles(R).reshape(-1)
    v = values.reshape(-1, values.shape[-1])
    r = r / np.linalg.norm(r)
    cos_rl = d @ r
    h = d + r[None]
    h /= np.linalg.norm(h, axis=1, keepdims=True)
    w = np.where(cos_rl > 0, ggx_D(h @ r, alpha) * cos_rl, 0.0) * om
    return (w[:, None] * v).sum(0) / w.sum()


# --- explicit microfacets --------------------------------------------------------

def sample_ggx_normals(rng, n: int, alpha: float) -> np.ndarray:
    """n facet normals with density D(h)/D_H over the hemisphere (identically
    sized facets distributed as the unprojected facet area, Sec. 3.2): the
    marginal of cos(theta) is inverted numerically, azimuth uniform."""
    a2 = alpha * alpha
    # marginal of y = cos(theta) under D dw / D_H: 2 pi D(y) dy / D_H
    ys = np.linspace(0.0, 1.0, 200001)
    pdf = 2.0 * math.pi * a2 / (math.pi * (1.0 + (a2 - 1.0) * ys * ys) ** 2)
    cdf = np.concatenate([[0.0], np.cumsum(0.5 * (pdf[1:] + pdf[:-1]) * np.diff(ys))])
    cdf /= cdf[-1]
    u = rng.random(n)
    y = np.interp(u, cdf, ys)
    phi = rng.random(n) * 2.0 * math.pi
    s = np.sqrt(np.clip(1.0 - y * y, 0.0, None))
    return np.stack([s * np.cos(phi), s * np.sin(phi), y], -1)


def explicit_counts(rng, NP: int, n: np.ndarray, wo: np.ndarray, alpha: float, region_of_dir, K: int):
    """Counts of NP explicit facets per region (bin 0 also takes facets that do
    not reflect w_o into the upper hemisphere).  region_of_dir(l) returns the
    fuzzy weights [m, K] of world directions l; each facet draws its region
    from them."""
    loc = sample_ggx_normals(rng, NP, alpha)
    # tangent frame around n
    n = n / np.linalg.norm(n)
    a = np.array([1.0, 0.0, 0.0]) if abs(n[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
    t1 = np.cross(n, a); t1 /= np.linalg.norm(t1)
    t2 = np.cross(n, t1)
    h = loc[:, :1] * t1 + loc[:, 1:2] * t2 + loc[:, 2:3] * n
    vh = h @ wo
    l = 2.0 * vh[:, None] * h - wo[None]
    valid = (vh > 0) & (l @ n > 0)
    counts = np.zeros(K)
    if valid.any():
        w = region_of_dir(l[valid])
        u = rng.random(int(valid.sum()))
        k = (np.cumsum(w, axis=1) < u[:, None]).sum(1)
        k = np.minimum(k, K - 1)
        counts += np.bincount(k, minlength=K)
    counts[0] += (~valid).sum()
    return counts
