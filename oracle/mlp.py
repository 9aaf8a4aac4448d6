"""CPU reference for the learned importance-sampling part -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this module.  It shares no code with the GPU library.

The learned part is not in the paper: it picks the vertex-sampling
probabilities of the VSamp estimator (Alg. 4, made weighted as a
Hansen-Hurwitz estimator with single-draw term B_v / (4 q_v)).  The network
never changes a count, so the estimator stays unbiased whatever it predicts.

Everything here is plain numpy in float64:

* ``features``: the eight per-vertex features from the edge list.
* ``forward`` / ``grad``: the MLP 8 -> 64 -> 64 -> 1 with ReLU and its
  gradient by back-propagation written out layer by layer.  With
  ``emulate=True`` the values are rounded where the matrix-core kernels
  round them (BF16 weights and features, BF16 hidden layer 1, BF16 dZ2 and
  dZ1 for the products that use them); with ``emulate=False`` it is the plain
  float64 network.
* ``adam``: one Adam step.
* ``probs_from_predictions``, ``vsamp_weights``, ``single_draw_variance``,
  ``draws_for``: the sampling side (uniform floor, integer weights as VSamp
  quantises them, the closed-form variance of one draw, the draws needed for a
  relative error at a confidence level).

Pins (tests/test_oracle_mlp.py): BF16 rounding against torch's conversion;
the plain forward against torch.nn in float64; the plain gradient against
central finite differences and torch.autograd; features against closed forms
on complete bipartite graphs and stars; the variance against enumeration of
every pair of draws on a small graph.
"""
from __future__ import annotations

import math

import numpy as np

NFEAT = 8
HID = 64
# parameter layout (float offsets), shared by the FP32 master copy, the
# Adam moments and the gradient
P_W1, P_B1, P_W2, P_B2, P_W3, P_B3, P_N = 0, 512, 576, 4672, 4736, 4800, 4801


def unpack(params):
    """Views (W1[8][64], b1[64], W2[64][64], b2[64], w3[64], b3) of a flat array."""
    p = np.asarray(params)
    return (p[P_W1:P_B1].reshape(NFEAT, HID), p[P_B1:P_W2], p[P_W2:P_B2].reshape(HID, HID),
            p[P_B2:P_W3], p[P_W3:P_B3], p[P_B3])


def pack(W1, b1, W2, b2, w3, b3):
    out = np.zeros(P_N, np.float64)
    out[P_W1:P_B1] = np.ravel(W1)
    out[P_B1:P_W2] = b1
    out[P_W2:P_B2] = np.ravel(W2)
    out[P_B2:P_W3] = b2
    out[P_W3:P_B3] = w3
    out[P_B3] = b3
    return out


# ------------------------------------------------------------------ bfloat16
def bf16_bits(x):
    """float -> float32 -> bfloat16 bit pattern, round to nearest even."""
    f = np.ascontiguousarray(np.asarray(x, np.float64).astype(np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    nan = (u & 0x7F800000) == 0x7F800000
    nan &= (u & 0x007FFFFF) != 0
    r = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    r = np.where(nan, (u >> 16) | 0x40, r)
    return r.astype(np.uint16)


def bf16_value(bits):
    b = np.asarray(bits, np.uint16).astype(np.uint32) << 16
    return b.view(np.float32).astype(np.float64)


def bf16(x):
    return bf16_value(bf16_bits(x))


def f32(x):
    return np.asarray(x, np.float64).astype(np.float32).astype(np.float64)


# ------------------------------------------------------------------ features
def raw_features(nl, nr, l, r):
    """Unrounded features, rows by global id (L ids, then nl + R id).

    For vertex v with neighbours u: side, then divided by 8: log1p d_v,
    log1p sum d_u, log1p sum d_u^2, log1p max d_u, log1p sum (d_u - 1) (the
    wedges with v at an end), log1p C(d_v, 2) (wedges with v in the middle),
    log1p(sum d_u / d_v).  Isolated vertices get 0 for the neighbour terms.
    """
    l = np.asarray(l, np.int64)
    r = np.asarray(r, np.int64)
    dl = np.bincount(l, minlength=nl).astype(np.float64)
    dr = np.bincount(r, minlength=nr).astype(np.float64)
    out = np.zeros((nl + nr, NFEAT), np.float64)
    for side, (src, dst, dsrc, ddst, n, row0) in enumerate(
            [(l, r, dl, dr, nl, 0), (r, l, dr, dl, nr, nl)]):
        du = ddst[dst]                       # degree of the far endpoint of each edge
        s1 = np.bincount(src, weights=du, minlength=n)
        s2 = np.bincount(src, weights=du * du, minlength=n)
        s3 = np.bincount(src, weights=du - 1.0, minlength=n)
        mx = np.zeros(n, np.float64)
        np.maximum.at(mx, src, du)
        dv = dsrc
        ratio = np.divide(s1, dv, out=np.zeros(n), where=dv > 0)
        f = out[row0:row0 + n]
        f[:, 0] = float(side)
        f[:, 1] = np.log1p(dv) / 8
        f[:, 2] = np.log1p(s1) / 8
        f[:, 3] = np.log1p(s2) / 8
        f[:, 4] = np.log1p(mx) / 8
        f[:, 5] = np.log1p(s3) / 8
        f[:, 6] = np.log1p(np.where(dv > 1, dv * (dv - 1.0) / 2, 0.0)) / 8   # C(d, 2), +0 below 2
        f[:, 7] = np.log1p(ratio) / 8
    return out


def features(nl, nr, l, r):
    """BF16 bit patterns of the features, shape (nl + nr, 8), uint16."""
    return bf16_bits(raw_features(nl, nr, l, r))


def targets(counts):
    """Training target log1p(B_v) / 8, rounded to float32 as the kernels store it."""
    return f32(np.log1p(np.asarray(counts, np.float64)) / 8)


# ------------------------------------------------------------------ network
def _relu(z):
    return np.maximum(z, 0.0)


def forward(params, X, emulate=True):
    """Returns (y, cache).  X: features (uint16 BF16 bits if emulate, else floats)."""
    W1, b1, W2, b2, w3, b3 = unpack(np.asarray(params, np.float64))
    if emulate:
        x = bf16_value(X)
        W1, W2, w3 = bf16(W1), bf16(W2), bf16(w3)
        b1, b2, b3 = f32(b1), f32(b2), float(f32(b3))
    else:
        x = np.asarray(X, np.float64)
    z1 = x @ W1 + b1
    h1 = _relu(z1)
    if emulate:
        h1 = bf16(h1)                        # hidden layer 1 feeds the matrix cores in BF16
    z2 = h1 @ W2 + b2
    h2 = _relu(z2)
    y = h2 @ w3 + b3
    return y, dict(x=x, W1=W1, W2=W2, w3=w3, z1=z1, h1=h1, z2=z2, h2=h2)


def loss_value(params, X, t, emulate=False):
    y, _ = forward(params, X, emulate)
    e = y - np.asarray(t, np.float64)
    return float(np.dot(e, e)) / len(e)


def grad(params, X, t, emulate=True):
    """Gradient of mean squared error over the rows, and the sum of squared errors.

    Back-propagation through y = relu(relu(x W1 + b1) W2 + b2) w3 + b3:
    dy = 2 (y - t) / rows; db3 = sum dy; dw3 = h2^T dy; dZ2 = [z2 > 0] w3 dy;
    db2 = sum dZ2; dW2 = h1^T dZ2; dZ1 = [z1 > 0] (dZ2 W2^T); db1 = sum dZ1;
    dW1 = x^T dZ1.
    """
    y, c = forward(params, X, emulate)
    t = np.asarray(t, np.float64)
    rows = len(t)
    err = y - t
    dy = 2.0 * err / rows
    db3 = dy.sum()
    dw3 = c["h2"].T @ dy
    dz2 = (c["z2"] > 0) * np.outer(dy, c["w3"])
    db2 = dz2.sum(axis=0)
    dz2m = bf16(dz2) if emulate else dz2     # operand of the two products below
    dW2 = c["h1"].T @ dz2m
    dh1 = dz2m @ c["W2"].T
    dz1 = (c["z1"] > 0) * dh1
    db1 = dz1.sum(axis=0)
    dz1m = bf16(dz1) if emulate else dz1
    dW1 = c["x"].T @ dz1m
    return pack(dW1, db1, dW2, db2, dw3, db3), float(np.dot(err, err))


def adam(params, m1, m2, g, lr, beta1, beta2, eps, step):
    """One Adam step (Kingma and Ba) with bias correction; returns new (params, m1, m2)."""
    m1 = beta1 * m1 + (1 - beta1) * g
    m2 = beta2 * m2 + (1 - beta2) * g * g
    c1 = 1 - beta1 ** step
    c2 = 1 - beta2 ** step
    return params - lr * (m1 / c1) / (np.sqrt(m2 / c2) + eps), m1, m2


# ------------------------------------------------------------------ sampling side
def probs_from_predictions(y, floor_frac):
    """q_v = max(expm1(8 y_v), floor_frac * mean_v max(expm1(8 y_v), 0)).

    floor_frac > 0 keeps every q_v positive, so the Hansen-Hurwitz estimate
    is unbiased whatever the network predicts; with no positive prediction
    (mean 0) the floor is empty and uniform sampling (q_v = 1) is used.
    """
    if not floor_frac > 0:
        raise ValueError("floor_frac must be positive")
    v = np.expm1(8.0 * np.asarray(y, np.float64))
    mean = np.maximum(v, 0.0).sum() / len(v)
    if mean == 0:
        return np.ones_like(v), mean
    return np.maximum(v, floor_frac * mean), mean


def vsamp_weights(probs):
    """Integer draw weights of weighted VSamp: max(1, floor(p / max p * (2^32 - 1))) for p > 0."""
    p = np.asarray(probs, np.float64)
    mx = p.max()
    w = np.floor(p / mx * 4294967295.0)
    return np.where(p > 0, np.maximum(w, 1.0), 0.0)


def single_draw_variance(counts, weights=None, exact=True):
    """Variance of one draw's term B_v / (4 q_v) with q_v = w_v / sum w (uniform if None).

    Equals sum_v B_v^2 / (16 q_v) - B^2 with B = sum_v B_v / 4; infinite if a
    vertex with B_v > 0 has weight 0 (the estimator would be biased).  With
    exact=True it is computed in rationals up to the final division (Python
    integers, for small graphs); otherwise in float64.
    """
    if not exact:
        bf = np.asarray(counts, np.float64)
        B = bf.sum() / 4
        if weights is None:
            return float(len(bf) * np.dot(bf, bf) / 16 - B * B)
        w = np.asarray(weights, np.float64)
        nz = bf > 0
        if np.any(w[nz] == 0):
            return math.inf
        q = w[nz] / w.sum()
        return float(np.sum(bf[nz] ** 2 / (16 * q)) - B * B)
    b = [int(x) for x in np.asarray(counts, np.uint64)]
    total4 = sum(b)                          # = 4 B
    if weights is None:
        n = len(b)
        num = n * sum(x * x for x in b) - total4 * total4      # 16 Var
        return num / 16.0
    w = [int(x) for x in np.asarray(weights, np.float64)]
    W = sum(w)
    from fractions import Fraction
    acc = Fraction(0)
    for bv, wv in zip(b, w):
        if bv == 0:
            continue
        if wv == 0:
            return math.inf
        acc += Fraction(bv * bv * W, wv)
    return float((acc - total4 * total4) / 16)


def draws_for(sigma1, total, rel=0.01, z=1.959963984540054):
    """Smallest k with z sigma1 / sqrt(k) <= rel * total (normal approximation)."""
    if total <= 0:
        return math.inf
    return max(1, math.ceil((z * sigma1 / (rel * total)) ** 2))
