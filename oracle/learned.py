"""Float64 oracle for the learned position model over prefix-table boundaries.

TEST INFRASTRUCTURE ONLY (see the package header).  The learned index is not
in the paper: it is a faster way to find the elementary interval that holds
an address, and the interval it must find is fixed by the paper's matching
definition (Algorithm 1 applied to the whole CIDR list).  This module states,
in float64 numpy, what the GPU's model, training step and error measure
compute, so their float32 results can be checked against it.

Notation.  B[0..m) are the sorted interval boundaries (``oracle.endpoints``);
the position of address a is pos(a) = j with B[j] <= a < B[j+1].
The models see x = a / 2^32 and are trained to y = j / m.

MLP 1-16-1 (49 parameters, vector order w1[16], b1[16], w2[16], b2):
    z_k = w1_k x + b1_k,  h_k = max(z_k, 0),  f(x) = sum_k w2_k h_k + b2,
    loss = mean_i (f(x_i) - y_i)^2.
PLA with S <= 256 segments at equal-count knots: segment s holds boundaries
    k_s <= j < k_{s+1}, k_s = floor(s m / S), knot_s = B[k_s]; its line
    j ~ c_s + g_s (B[j] - knot_s) is the least-squares fit over the segment.
"""
from __future__ import annotations

import numpy as np

H = 16
N_PARAMS = 3 * H + 1


def split(params):
    p = np.asarray(params, dtype=np.float64)
    return p[0:H], p[H:2 * H], p[2 * H:3 * H], p[3 * H]


def positions(B: np.ndarray, a: np.ndarray) -> np.ndarray:
    """pos(a): index of the last boundary <= a (a sorted search)."""
    return np.searchsorted(B, np.asarray(a, dtype=np.uint32), side="right").astype(np.int64) - 1


def training_set(B: np.ndarray):
    """Inputs x = B[j] / 2^32 and targets y = j / m for every boundary."""
    m = B.shape[0]
    x = B.astype(np.float64) / 4294967296.0
    y = np.arange(m, dtype=np.float64) / m
    return x, y


def mlp_forward(params, x):
    w1, b1, w2, b2 = split(params)
    x = np.asarray(x, dtype=np.float64)
    z = x[:, None] * w1[None, :] + b1[None, :]
    h = np.maximum(z, 0.0)
    return h @ w2 + b2


def mlp_loss_grad(params, x, y):
    """Mean squared error and its exact gradient (back-propagation written
    out by hand: dL/df = 2 (f - y) / n, then through w2, the ReLU and w1)."""
    w1, b1, w2, b2 = split(params)
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    n = x.shape[0]
    z = x[:, None] * w1[None, :] + b1[None, :]
    h = np.maximum(z, 0.0)
    f = h @ w2 + b2
    r = f - y
    loss = float(np.mean(r * r))
    d = 2.0 * r / n
    g_w2 = h.T @ d
    g_b2 = d.sum()
    dz = (d[:, None] * w2[None, :]) * (z > 0.0)
    g_w1 = dz.T @ x
    g_b1 = dz.sum(axis=0)
    return loss, np.concatenate([g_w1, g_b1, g_w2, [g_b2]])


def mlp_init_hinges():
    """Deterministic start: hinges at x = k/16 (w1 = 1, b1 = -k/16), w2 = b2 = 0."""
    p = np.zeros(N_PARAMS)
    p[0:H] = 1.0
    p[H:2 * H] = -np.arange(H) / H
    return p


def adam_steps(params, x, y, steps, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """Full-batch Adam (Kingma and Ba, 2015) in float64: the update rule the
    GPU trainer applies, for a trajectory check over a few steps."""
    p = np.asarray(params, dtype=np.float64).copy()
    m1 = np.zeros_like(p)
    m2 = np.zeros_like(p)
    for t in range(1, steps + 1):
        _, g = mlp_loss_grad(p, x, y)
        m1 = beta1 * m1 + (1 - beta1) * g
        m2 = beta2 * m2 + (1 - beta2) * g * g
        mh = m1 / (1 - beta1 ** t)
        vh = m2 / (1 - beta2 ** t)
        p = p - lr * mh / (np.sqrt(vh) + eps)
    return p


def pla_fit(B: np.ndarray, S: int = 256):
    """Equal-count segments and their least-squares lines (float64).
    Returns (knot[S] uint32, first[S+1] int64, c[S], g[S])."""
    m = B.shape[0]
    S = min(S, m)
    k = (np.arange(S + 1, dtype=np.int64) * m) // S
    knot = B[k[:S]].astype(np.uint32)
    c = np.zeros(S)
    g = np.zeros(S)
    for s in range(S):
        j = np.arange(k[s], k[s + 1], dtype=np.float64)
        u = B[k[s]:k[s + 1]].astype(np.float64) - float(knot[s])
        if j.shape[0] < 2 or np.all(u == u[0]):
            c[s] = j.mean()
            g[s] = 0.0
            continue
        um, jm = u.mean(), j.mean()
        g[s] = np.sum((u - um) * (j - jm)) / np.sum((u - um) ** 2)
        c[s] = jm - g[s] * um
    return knot, k, c, g


def pla_predict(knot, c, g, a):
    """Float64 PLA prediction of pos(a)."""
    a = np.asarray(a, dtype=np.uint32)
    s = np.searchsorted(knot, a, side="right") - 1
    return c[s] + g[s] * (a.astype(np.float64) - knot[s].astype(np.float64))


def max_error(pred_fn, B: np.ndarray) -> float:
    """max over intervals j of |pred - j| at both ends B[j] and B[j+1]-1 (for
    a prediction monotone inside each interval this bounds every address)."""
    m = B.shape[0]
    j = np.arange(m, dtype=np.float64)
    lo = B.astype(np.uint32)
    hi = np.empty(m, np.uint32)
    hi[:-1] = B[1:] - 1
    hi[-1] = 0xFFFFFFFF
    return float(max(np.max(np.abs(pred_fn(lo) - j)), np.max(np.abs(pred_fn(hi) - j))))


def mlp_grad_abs_sum(params, x, y):
    """Per-parameter sum of |per-sample gradient terms| (the magnitude that a
    float32 sum of those terms is accurate relative to)."""
    w1, b1, w2, b2 = split(params)
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    n = x.shape[0]
    z = x[:, None] * w1[None, :] + b1[None, :]
    h = np.maximum(z, 0.0)
    r = h @ w2 + b2 - y
    a = 2.0 * np.abs(r) / n
    dz = (a[:, None] * np.abs(w2)[None, :]) * (z > 0.0)
    return np.concatenate([dz.T @ np.abs(x), dz.sum(axis=0), h.T @ a, [a.sum()]])


# ---------------------------------------------------------------------------
# Rounded positions in float32.  A model's prediction becomes an integer
# position (the start of the bounded search), so the measured bound depends on
# the precision the prediction is taken in; these functions take it in the
# float32 arithmetic of the lookups, one IEEE rounding per operation and no
# fused multiply-add, then clamp to [0, m - 1] and round to the nearest
# integer (ties to even).
# ---------------------------------------------------------------------------
def _clamp_round(p, m):
    p = np.fmin(np.fmax(p, np.float32(0.0)), np.float32(m - 1))   # NaN -> 0
    return np.rint(p).astype(np.int64)


def pla_position_f32(knot, c, g, a, m):
    """Rounded PLA position of addresses a: the last knot <= a picks the
    segment s, then p = c_s + g_s * float32(a - knot_s)."""
    knot = np.asarray(knot, dtype=np.uint32)
    a = np.asarray(a, dtype=np.uint32)
    s = np.searchsorted(knot, a, side="right") - 1
    d = (a - knot[s]).astype(np.float32)                 # a - knot_s < 2^32, rounded once
    p = np.asarray(c, np.float32)[s] + np.asarray(g, np.float32)[s] * d
    return _clamp_round(p.astype(np.float32), m)


def mlp_position_f32(params, a, m):
    """Rounded MLP position: x = float32(a) * 2^-32, f = b2 + sum_k w2_k
    relu(w1_k x + b1_k) accumulated in k order, p = f * float32(m)."""
    w = np.asarray(params, dtype=np.float32)
    x = np.asarray(a, dtype=np.uint32).astype(np.float32) * np.float32(2.0 ** -32)
    f = np.full(x.shape, w[48], dtype=np.float32)
    for k in range(H):
        z = w[k] * x + w[H + k]
        f = f + w[2 * H + k] * np.maximum(z, np.float32(0.0))
    return _clamp_round(f * np.float32(m), m)


def max_error_rounded(pos_fn, B: np.ndarray) -> int:
    """max over intervals j of |pos_fn(a) - j| at a = B[j] and a = B[j+1] - 1
    (the last interval ends at 2^32 - 1): the bound a lookup's search window
    must cover, for a prediction monotone inside every interval."""
    m = B.shape[0]
    j = np.arange(m, dtype=np.int64)
    lo = B.astype(np.uint32)
    hi = np.empty(m, np.uint32)
    hi[:-1] = B[1:] - 1
    hi[-1] = 0xFFFFFFFF
    return int(max(np.max(np.abs(pos_fn(lo) - j)), np.max(np.abs(pos_fn(hi) - j))))
