"""Oracle of the learned warm start (not part of the paper; a build extension).

The warm start predicts each level's CG solution from its right-hand side
with a small per-point network whose inputs are local: for point i of level
l, its 16 nearest same-level points n_1..n_16 (squared FP64 distance, ties
by global input index, the point itself excluded; a level with fewer than 17
points pads the list with i itself) and

    s_i      = sqrt(mean of b^2 over {i, n_1..n_16})
    features = [b_i/s, (b_{n_m}/s, (x_{n_m} - x_i)/delta_l  for m = 1..16)]
               (1 + 16 (1 + d) values, zero-padded to a multiple of 8)
    x0_i     = s * (w2 . relu(W1 feat + b1) + b2)      (0 where s = 0)

with 64 hidden units. On the GPU the first layer runs with BF16 weights and
BF16 features (round to nearest even) and FP32 accumulation; the reference
below rounds the same operands and accumulates in FP64.

Pins: the kNN lists against scipy's KD-tree query (an independent library
routine) and brute force; bf16 rounding against hand-worked bit patterns; the
forward pass against an explicit per-sample loop.
"""
from __future__ import annotations

import numpy as np

HIDDEN = 64
KNN = 16


def feature_count(dim: int) -> int:
    """Features per point, padded to a multiple of 8."""
    f = 1 + KNN * (1 + dim)
    return (f + 7) // 8 * 8


def knn16(X: np.ndarray, input_index: np.ndarray | None = None) -> np.ndarray:
    """16 nearest other points of every point of one level (indices into X).

    Brute force on squared FP64 distances dx*dx + dy*dy (+ dz*dz); ties by
    input_index (default: position in X). Fewer than 17 points: padded with
    the point itself.
    """
    n, d = X.shape
    idx = np.arange(n) if input_index is None else np.asarray(input_index)
    out = np.empty((n, KNN), dtype=np.int64)
    for s in range(0, n, 2048):
        a = X[s:s + 2048]
        d2 = None
        for ax in range(d):
            dx = a[:, None, ax] - X[None, :, ax]
            d2 = dx * dx if d2 is None else d2 + dx * dx
        rows = np.arange(a.shape[0])
        d2[rows, s + rows] = np.inf  # exclude self
        for r in range(a.shape[0]):
            order = np.lexsort((idx, d2[r]))[: min(KNN, n - 1)]
            lst = list(order)
            while len(lst) < KNN:
                lst.append(s + r)
            out[s + r] = lst
    return out


def bf16(x: np.ndarray) -> np.ndarray:
    """Round float32 values to bfloat16 (round to nearest, ties to even),
    returned as float32 (NaN inputs are not expected here)."""
    b = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    lsb = (b >> np.uint64(16)) & np.uint64(1)
    r = ((b + np.uint64(0x7FFF) + lsb) >> np.uint64(16)) << np.uint64(16)
    return r.astype(np.uint32).view(np.float32)


def features(X: np.ndarray, b: np.ndarray, nb: np.ndarray, delta: float):
    """(features [n][F] float32, s [n]) of one level, as defined above."""
    n, d = X.shape
    F = feature_count(d)
    ss = b * b  # sum of squares in stencil order: i, n_1, ..., n_16
    for m in range(KNN):
        ss = ss + b[nb[:, m]] * b[nb[:, m]]
    s = np.sqrt(ss / float(KNN + 1))
    safe = np.where(s > 0, s, 1.0)
    feat = np.zeros((n, F), dtype=np.float64)
    feat[:, 0] = b / safe
    for m in range(KNN):
        j = nb[:, m]
        base = 1 + m * (1 + d)
        feat[:, base] = b[j] / safe
        for ax in range(d):
            feat[:, base + 1 + ax] = (X[j, ax] - X[:, ax]) / delta
    feat[s == 0] = 0.0
    return feat.astype(np.float32), s


def forward(W1, b1, w2, b2, feat, s, bf16_first_layer: bool = True) -> np.ndarray:
    """x0 = s * (w2 . relu(W1 feat + b1) + b2); FP64 accumulation."""
    A = bf16(feat).astype(np.float64) if bf16_first_layer else feat.astype(np.float64)
    W = bf16(W1).astype(np.float64) if bf16_first_layer else W1.astype(np.float64)
    hdn = np.maximum(A @ W.T + b1.astype(np.float64), 0.0)
    y = hdn @ w2.astype(np.float64) + float(b2)
    return np.where(s > 0, s * y, 0.0)


def forward_loop(W1, b1, w2, b2, feat_row, s_i) -> float:
    """The same network for one point, written as plain loops (FP64)."""
    if s_i == 0:
        return 0.0
    fr = bf16(feat_row)
    Wb = bf16(W1)
    out = float(b2)
    for h in range(W1.shape[0]):
        acc = float(b1[h])
        for k in range(W1.shape[1]):
            acc += float(Wb[h, k]) * float(fr[k])
        out += float(w2[h]) * max(acc, 0.0)
    return s_i * out
