"""Element-wise tolerances of the surrogate's bfloat16 evaluation against its
plain FP64 definition (oracle/mlp.py, bf=False), for the GPU parity tests of
the forward pass, the gradient and the Adam step.

The matrix cores take bfloat16 operands and accumulate in float32;
activations and error signals are rounded to bfloat16 between layers.  A
worst-case (absolute-value) bound of those roundings grows by sum_j |W_ij|
(~10) per layer and says nothing after three layers, so the tolerance is the
standard deviation of a rounding-error model instead: each bfloat16 rounding
of a value v adds an error of variance (u v)^2 / 3 (uniform within half a
unit in the last place, u = 2^-8), propagated to first order through the
FP64 network:

* errors that differ from sample to sample (input and activation roundings)
  are independent: their variances add through every sum;
* errors of the rounded weights are shared by all samples of a batch: a sum
  over the batch adds their standard deviations (Minkowski's inequality,
  valid whatever the correlation), a sum over a sample's inputs adds their
  variances (different weights round independently);
* SiLU and its derivative scale errors by silu'(z) and silu''(z); softmax
  maps dz to y_k (dz_k - sum_j y_j dz_j).

float32 accumulation (n 2^-24 relative, n <= 4096) is two orders below u and
enters as 1e-6 of each element's magnitude.  tests/test_oracle_mlp.py checks
on the CPU that the bfloat16 mirror of the kernels (bf=True), which rounds
exactly where they round, deviates from FP64 by the order of this sigma and
never beyond the factor the GPU tests allow.
"""
import numpy as np

from oracle import mlp

U = 2.0 ** -8    # bfloat16 unit roundoff
Q = U * U / 3.0  # variance of one rounding, relative to the value squared
FREL = 1e-6      # float32 accumulation and transcendentals, relative


def _sig(z):
    return 1.0 / (1.0 + np.exp(-z))


def _silu(z):
    return z * _sig(z)


def _dsilu(z):
    s = _sig(z)
    return s * (1.0 + z * (1.0 - s))


def _d2silu(z):
    s = _sig(z)
    return s * (1.0 - s) * (2.0 + z * (1.0 - 2.0 * s))


def _dense(a, Vi, Vs, W, b):
    """z = a W^T + b with its independent and shared error variances."""
    W2 = W * W
    z = a @ W.T + b
    return z, Vi @ W2.T, Vs @ W2.T + Q * ((a * a) @ W2.T)


def forward_sigma(w, x, K):
    """(y64, sigma_y, cache): the FP64 outputs and the model's standard
    deviation of a bfloat16 evaluation's deviation from them."""
    p = mlp.unpack(np.asarray(w, dtype=np.float64), K)
    a = np.asarray(x, dtype=np.float64)
    Vi, Vs = Q * a * a, np.zeros_like(a)
    cache = dict(p=p, a=[a], Vi=[Vi], Vs=[Vs], z=[], Vzi=[], Vzs=[])
    for l in (1, 2, 3):
        z, Vzi, Vzs = _dense(a, Vi, Vs, p[f"W{l}"], p[f"b{l}"])
        d1 = _dsilu(z) ** 2
        h = _silu(z)
        a, Vi, Vs = h, d1 * Vzi + Q * h * h, d1 * Vzs
        for k, v in (("a", a), ("Vi", Vi), ("Vs", Vs), ("z", z), ("Vzi", Vzi), ("Vzs", Vzs)):
            cache[k].append(v)
    z4, Vzi, Vzs = _dense(a, Vi, Vs, p["W4"], p["b4"])
    zz = z4 - z4.max(axis=1, keepdims=True)
    y = np.exp(zz)
    y /= y.sum(axis=1, keepdims=True)

    Vyi, Vys = _soft_var(y, Vzi), _soft_var(y, Vzs)
    cache.update(y=y, Vyi=Vyi, Vys=Vys, Vz4i=Vzi, Vz4s=Vzs)
    return y, np.sqrt(Vyi + Vys) + FREL * y, cache


def _soft_var(y, V):
    """Variance of softmax outputs y for independent logit errors of variance V."""
    y2 = y * y
    return y2 * ((1.0 - y) ** 2 * V + (y2 * V).sum(axis=1, keepdims=True) - y2 * V)


def gradient_sigma(w, x, t, K, levels=None, lam=0.0):
    """(g64, sigma_g): the FP64 gradient of the mean loss (flat padded
    layout; with levels and lam the radiance-weighted term of
    mlp.loss_and_grad) and the model's standard deviation of a bfloat16
    evaluation's deviation from it, per element.  The two terms' errors
    are correlated: their standard deviations add."""
    y, _, c = forward_sigma(w, x, K)
    p = c["p"]
    B = len(x)
    t = np.asarray(t, dtype=np.float64)
    d = (y - t) / B
    sdi, sds = np.sqrt(c["Vyi"]) / B, np.sqrt(c["Vys"]) / B
    if levels is not None and lam > 0:
        yp, tp, ok = mlp.radiance_weighted(y, t, levels)
        d = d.copy()
        d[ok, 1:] += lam * (yp[ok] - tp[ok]) / B
        for sd, V in ((sdi, c["Vz4i"]), (sds, c["Vz4s"])):
            add = lam * np.sqrt(_soft_var(yp, V[:, 1:])) / B
            sd[ok, 1:] += add[ok]
    Vi = sdi * sdi + Q * d * d
    Vs = sds * sds
    g, S = {}, {}
    for l in (4, 3, 2, 1):
        a, Vai, Vas = c["a"][l - 1], c["Vi"][l - 1], c["Vs"][l - 1]
        g[f"W{l}"] = d.T @ a
        ind = (d * d).T @ Vai + Vi.T @ (a * a)
        sh = np.zeros_like(g[f"W{l}"])
        for b0 in range(0, B, 256):  # sum over the batch of per-sample standard deviations
            db, ab = d[b0:b0 + 256], a[b0:b0 + 256]
            sh += np.sqrt((db * db)[:, :, None] * Vas[b0:b0 + 256][:, None, :] +
                          Vs[b0:b0 + 256][:, :, None] * (ab * ab)[:, None, :]).sum(axis=0)
        S[f"W{l}"] = np.sqrt(ind) + sh + FREL * (np.abs(d).T @ np.abs(a))
        g[f"b{l}"] = d.sum(axis=0)
        S[f"b{l}"] = np.sqrt(Vi.sum(axis=0)) + np.sqrt(Vs).sum(axis=0) + FREL * np.abs(d).sum(axis=0)
        if l == 1:
            break
        W = p[f"W{l}"]
        W2 = W * W
        back = d @ W
        Vbi, Vbs = Vi @ W2, Vs @ W2 + Q * ((d * d) @ W2)
        z, Vzi, Vzs = c["z"][l - 2], c["Vzi"][l - 2], c["Vzs"][l - 2]
        ds, dds = _dsilu(z), _d2silu(z)
        dn = back * ds
        Vi = ds ** 2 * Vbi + (back * dds) ** 2 * Vzi + Q * dn * dn
        Vs = ds ** 2 * Vbs + (back * dds) ** 2 * Vzs
        d = dn
    return mlp.pack(g, K), mlp.pack(S, K)
