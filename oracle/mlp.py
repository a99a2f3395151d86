"""Plain FP64 definition of the learned surrogate (numpy).  TEST INFRASTRUCTURE ONLY.

The surrogate maps a lookup (reflection direction w, alpha_x, alpha_y) to the
K normalised filtered indicator values F_k / sum F that the roughness pyramid
would otherwise provide (Sec. 5, Eq. (rtiblndf) feeds p_k = S F_k / sum F).
Not from the paper: the network, its inputs and its training are the
project's own.

Network: x (5) -> 64 -> 64 -> 64 -> K, SiLU hidden units, softmax output,
soft-label cross-entropy against the filter's normalised outputs, plus an
optional cross-entropy of the radiance-weighted distributions (the glint
radiance of Eq. (iblglints:fin) weights each bin's error by its level).
Inputs: (w_x, w_y, w_z, (ln alpha_x - c)/h, (ln alpha_y - c)/h) with c, h
mapping [ln 0.02, ln 0.5] to [-1, 1].

Storage layout (flat float32, padded for 32x32x16 matrix-core tiles): W1
[64][16] (inputs 5..15 zero), b1 [64], W2 [64][64], b2 [64], W3 [64][64],
b3 [64], W4 [32][64] (rows K..31 zero), b4 [32].  The GPU feeds the matrix
cores bfloat16 weights and activations and accumulates in float32; with
``bf16=True`` this module rounds at exactly those points (inputs, weights,
hidden activations, and the error signals of the backward pass), so its
results differ from the GPU's only by accumulation order.
"""
from __future__ import annotations

import math

import numpy as np

HIDDEN = 64
IN_PAD = 16
OUT_PAD = 32
LN_LO, LN_HI = math.log(0.02), math.log(0.5)
ALPHA_C = 0.5 * (LN_LO + LN_HI)
ALPHA_H = 0.5 * (LN_HI - LN_LO)

OFF = {}
_o = 0
for _name, _n in (("W1", HIDDEN * IN_PAD), ("b1", HIDDEN), ("W2", HIDDEN * HIDDEN), ("b2", HIDDEN),
                  ("W3", HIDDEN * HIDDEN), ("b3", HIDDEN), ("W4", OUT_PAD * HIDDEN), ("b4", OUT_PAD)):
    OFF[_name] = (_o, _n)
    _o += _n
N_PARAMS = _o  # 11488 stored entries


def real_params(K: int) -> int:
    """Parameters of the unpadded network."""
    return 5 * HIDDEN + HIDDEN + 2 * (HIDDEN * HIDDEN + HIDDEN) + HIDDEN * K + K


def bf16(a):
    """Round to bfloat16 (nearest even), returned as float64."""
    a = np.asarray(a, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def features(dirs, ax, ay):
    """Network inputs [n, 5] from unit directions and alpha_x, alpha_y."""
    dirs = np.asarray(dirs, dtype=np.float64)
    ux = (np.log(np.asarray(ax, dtype=np.float64)) - ALPHA_C) / ALPHA_H
    uy = (np.log(np.asarray(ay, dtype=np.float64)) - ALPHA_C) / ALPHA_H
    return np.concatenate([dirs, ux[:, None], uy[:, None]], axis=1)


def unpack(w, K):
    w = np.asarray(w, dtype=np.float64)
    g = lambda n: w[OFF[n][0]:OFF[n][0] + OFF[n][1]]
    return dict(W1=g("W1").reshape(HIDDEN, IN_PAD)[:, :5], b1=g("b1"), W2=g("W2").reshape(HIDDEN, HIDDEN),
                b2=g("b2"), W3=g("W3").reshape(HIDDEN, HIDDEN), b3=g("b3"),
                W4=g("W4").reshape(OUT_PAD, HIDDEN)[:K], b4=g("b4")[:K])


def pack(p, K):
    w = np.zeros(N_PARAMS)
    for n in ("b1", "b2", "b3"):
        w[OFF[n][0]:OFF[n][0] + OFF[n][1]] = p[n]
    w1 = np.zeros((HIDDEN, IN_PAD)); w1[:, :5] = p["W1"]
    w[OFF["W1"][0]:OFF["W1"][0] + OFF["W1"][1]] = w1.ravel()
    w[OFF["W2"][0]:OFF["W2"][0] + OFF["W2"][1]] = np.asarray(p["W2"]).ravel()
    w[OFF["W3"][0]:OFF["W3"][0] + OFF["W3"][1]] = np.asarray(p["W3"]).ravel()
    w4 = np.zeros((OUT_PAD, HIDDEN)); w4[:K] = p["W4"]
    w[OFF["W4"][0]:OFF["W4"][0] + OFF["W4"][1]] = w4.ravel()
    b4 = np.zeros(OUT_PAD); b4[:K] = p["b4"]
    w[OFF["b4"][0]:OFF["b4"][0] + OFF["b4"][1]] = b4
    return w


def init(K, seed=7):
    """He-style uniform initialisation (seeded), biases zero; flat float32."""
    rng = np.random.default_rng(seed)
    p = {}
    for n, (fo, fi) in (("W1", (HIDDEN, 5)), ("W2", (HIDDEN, HIDDEN)), ("W3", (HIDDEN, HIDDEN)), ("W4", (K, HIDDEN))):
        lim = math.sqrt(6.0 / fi)
        p[n] = rng.uniform(-lim, lim, (fo, fi))
    p["b1"], p["b2"], p["b3"], p["b4"] = np.zeros(HIDDEN), np.zeros(HIDDEN), np.zeros(HIDDEN), np.zeros(K)
    return pack(p, K).astype(np.float32)


def _sig(z):
    return 1.0 / (1.0 + np.exp(-z))


def silu(z):
    return z * _sig(z)


def dsilu(z):
    s = _sig(z)
    return s * (1.0 + z * (1.0 - s))


def forward(w, x, K, bf=False):
    """Returns (probs [n,K], cache).  bf: round as the matrix cores are fed."""
    r = bf16 if bf else (lambda a: np.asarray(a, dtype=np.float64))
    p = unpack(w, K)
    W = {n: r(p[n]) for n in ("W1", "W2", "W3", "W4")}
    a0 = r(x)
    z1 = a0 @ W["W1"].T + p["b1"]
    h1 = r(silu(z1))
    z2 = h1 @ W["W2"].T + p["b2"]
    h2 = r(silu(z2))
    z3 = h2 @ W["W3"].T + p["b3"]
    h3 = r(silu(z3))
    z4 = h3 @ W["W4"].T + p["b4"]
    z4 = z4 - z4.max(axis=1, keepdims=True)
    e = np.exp(z4)
    y = e / e.sum(axis=1, keepdims=True)
    return y, dict(a0=a0, z1=z1, h1=h1, z2=z2, h2=h2, z3=z3, h3=h3, W=W, y=y)


def radiance_weighted(y, t, levels):
    """The radiance-weighted distributions over the bins k >= 1:
    y'_k = L_k y_k / sum_{j>=1} L_j y_j and t' likewise, and the mask of the
    samples for which both sums are positive (the others get no term)."""
    L = np.asarray(levels, dtype=np.float64)[1:]
    yw, tw = y[:, 1:] * L, t[:, 1:] * L
    ys, ts = yw.sum(1, keepdims=True), tw.sum(1, keepdims=True)
    ok = (ys[:, 0] > 0) & (ts[:, 0] > 0)
    return yw / np.where(ys > 0, ys, 1.0), tw / np.where(ts > 0, ts, 1.0), ok


def loss_and_grad(w, x, t, K, bf=False, levels=None, lam=0.0):
    """Mean loss over the batch and its gradient (flat, padded layout; pad
    entries 0).  The loss is the soft-label cross-entropy -sum_k t_k ln y_k
    plus, with levels and lam > 0, lam times the cross-entropy of the
    radiance-weighted distributions, -sum_{k>=1} t'_k ln y'_k (see
    radiance_weighted).  Its gradient with respect to the logits is
    (y - t) + lam (y' - t') on the bins k >= 1: y' is the softmax of
    z_k + ln L_k over those bins."""
    r = bf16 if bf else (lambda a: np.asarray(a, dtype=np.float64))
    y, c = forward(w, x, K, bf)
    B = len(x)
    t = np.asarray(t, dtype=np.float64)
    loss = -np.sum(t * np.log(np.maximum(y, 1e-300))) / B
    dz = y - t
    if levels is not None and lam > 0:
        yp, tp, ok = radiance_weighted(y, t, levels)
        loss += lam * -np.sum(tp[ok] * np.log(np.maximum(yp[ok], 1e-300))) / B
        dz = dz.copy()
        dz[ok, 1:] += lam * (yp[ok] - tp[ok])
    dz4 = r(dz / B)
    g = {}
    g["W4"] = dz4.T @ c["h3"]
    g["b4"] = dz4.sum(0)
    dz3 = r((dz4 @ c["W"]["W4"]) * dsilu(c["z3"]))
    g["W3"] = dz3.T @ c["h2"]
    g["b3"] = dz3.sum(0)
    dz2 = r((dz3 @ c["W"]["W3"]) * dsilu(c["z2"]))
    g["W2"] = dz2.T @ c["h1"]
    g["b2"] = dz2.sum(0)
    dz1 = r((dz2 @ c["W"]["W2"]) * dsilu(c["z1"]))
    g["W1"] = dz1.T @ c["a0"]
    g["b1"] = dz1.sum(0)
    return loss, pack(g, K)


def adam(w, m, v, g, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (step counts from 1); returns new (w, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v
