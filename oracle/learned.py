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

Training (below): mean squared error against alpha_i / s_i, its gradient by
the chain rule, Adam steps from zero moments on fixed mini-batches.

Pins (tests/test_oracle_learned.py): the kNN lists against scipy's KD-tree
query (an independent library routine); bf16 rounding against hand-worked bit
patterns; the features and s of a 3-point level worked by hand (padding with
the point itself, the divisor 17); the forward pass of a 2-unit network worked
by hand (ReLU active and clipped, BF16 rounding of a feature); the gradient of
a 2-unit network worked by hand and against central finite differences of the
FP64 loss; Adam's first steps against their closed form (a step of -lr g /
(|g| + eps) under a constant gradient); the mini-batch schedule by listing.
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


# ------------------------------------------------------------------ training
#
# The network is trained on (features, target) samples, target = alpha_i / s_i
# (the correction the level's solve produced, in the units of the stencil
# scale), by minimising the mean squared error of the network output over
# mini-batches with Adam (Kingma and Ba, "Adam: a method for stochastic
# optimization", ICLR 2015, Algorithm 1: first and second moment estimates
# with bias correction). The first layer sees the same BF16-rounded weights
# and features as inference; its gradient is taken with respect to those
# rounded values and applied to the unrounded weights (straight-through).

ADAM_BETA1 = 0.9
ADAM_BETA2 = 0.999
ADAM_EPS = 1e-8
TRAIN_BATCH = 128


def pack(W1, b1, w2, b2) -> np.ndarray:
    """Flat parameter vector in the library's order: W1 [H][F], b1 [H], w2 [H], b2."""
    return np.concatenate([np.ravel(W1), np.ravel(b1), np.ravel(w2), [float(b2)]]).astype(np.float64)


def unpack(p: np.ndarray, F: int, hidden: int = HIDDEN):
    """(W1 [H][F], b1 [H], w2 [H], b2) views of a flat parameter vector."""
    H = hidden
    W1 = p[: H * F].reshape(H, F)
    b1 = p[H * F: H * F + H]
    w2 = p[H * F + H: H * F + 2 * H]
    return W1, b1, w2, p[H * F + 2 * H]


def loss_and_grads(W1, b1, w2, b2, X, y, bf16_first_layer: bool = True):
    """Mean over the rows of X of (net(x) - y)^2, net(x) = w2 . relu(W1 x + b1) + b2,
    and its gradient with respect to (W1, b1, w2, b2), all in FP64.

    Chain rule, with B rows, e = net(x) - y and a = W1 x + b1:
      d/d b2 = sum_q 2 e_q / B,   d/d w2 = sum_q (2 e_q / B) relu(a_q),
      d/d b1 = sum_q (2 e_q / B) w2 * [a_q > 0],   d/d W1 = (that term) outer x_q.
    """
    A = bf16(X).astype(np.float64) if bf16_first_layer else np.asarray(X, dtype=np.float64)
    W = bf16(W1).astype(np.float64) if bf16_first_layer else np.asarray(W1, dtype=np.float64)
    b1 = np.asarray(b1, dtype=np.float64)
    w2 = np.asarray(w2, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    B = A.shape[0]
    pre = A @ W.T + b1
    hdn = np.maximum(pre, 0.0)
    err = hdn @ w2 + float(b2) - y
    loss = float(np.mean(err * err))
    d_out = 2.0 * err / B
    g_b2 = float(np.sum(d_out))
    g_w2 = hdn.T @ d_out
    d_pre = np.outer(d_out, w2) * (pre > 0.0)
    g_b1 = d_pre.sum(axis=0)
    g_W1 = d_pre.T @ A
    return loss, (g_W1, g_b1, g_w2, g_b2)


def adam_update(p, g, m, v, t: int, lr: float, beta1: float = ADAM_BETA1, beta2: float = ADAM_BETA2,
                eps: float = ADAM_EPS):
    """One Adam step t (t = 1, 2, ...) on parameters p with gradient g and
    moment estimates m, v; returns the new (p, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def batch_rows(step: int, ns: int, batch: int = TRAIN_BATCH) -> np.ndarray:
    """Sample rows of mini-batch `step` (0-based): (step * batch + q) mod ns, q < batch."""
    return (step * batch + np.arange(batch)) % ns


def train(p0: np.ndarray, X: np.ndarray, y: np.ndarray, steps: int, lr: float, F: int | None = None,
          batch: int = TRAIN_BATCH, bf16_first_layer: bool = True):
    """Adam from fresh (zero) moments on the mini-batches of `batch_rows`;
    returns (parameters after `steps` steps, loss of each mini-batch before
    its update)."""
    F = X.shape[1] if F is None else F
    p = np.array(p0, dtype=np.float64)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    losses = []
    for step in range(steps):
        rows = batch_rows(step, X.shape[0], batch)
        W1, b1, w2, b2 = unpack(p, F)
        loss, g = loss_and_grads(W1, b1, w2, b2, X[rows], y[rows], bf16_first_layer)
        losses.append(loss)
        p, m, v = adam_update(p, pack(*g), m, v, step + 1, lr)
    return p, np.array(losses)


def grad_error_bound(W1, b1, w2, b2, X, y, lam: float = 8.0) -> np.ndarray:
    """Probabilistic bound on the error of an FP32 evaluation of
    `loss_and_grads` (BF16 first layer, any summation order), per parameter
    in the flat order. Rounding errors are modelled as independent (Higham
    and Mary, "A new approach to probabilistic rounding error analysis",
    SIAM J. Sci. Comput. 2019): a sum of n terms has an error scale of
    sqrt(n) u sum|terms| (u = 2^-24); scales carried from earlier stages add
    as a root sum of squares; the bound is lam times the final scale. A
    sample whose pre-activation lies within lam times its own error scale of
    zero contributes its whole term (its ReLU mask may flip)."""
    u = 2.0 ** -24
    A = bf16(X).astype(np.float64)
    W = bf16(W1).astype(np.float64)
    b1 = np.asarray(b1, dtype=np.float64)
    w2 = np.asarray(w2, dtype=np.float64)
    B, F = A.shape
    H = W.shape[0]
    pre = A @ W.T + b1
    hdn = np.maximum(pre, 0.0)
    err = hdn @ w2 + float(b2) - np.asarray(y, dtype=np.float64)
    s_pre = np.sqrt(F + 1) * u * (np.abs(A) @ np.abs(W).T + np.abs(b1))                 # [B][H]
    s_out = np.sqrt((np.sqrt(H + 1) * u * (np.abs(hdn) @ np.abs(w2) + abs(float(b2)))) ** 2
                    + (s_pre * s_pre) @ (w2 * w2) + (u * (np.abs(y) + np.abs(err))) ** 2)  # [B]
    d_out = 2.0 * err / B
    s_dout = 2.0 * s_out / B + u * np.abs(d_out)                                         # [B]
    flip = np.abs(pre) <= lam * s_pre                                                    # [B][H]
    live = (pre > 0.0) | flip
    t_pre = np.abs(np.outer(d_out, w2)) * live            # |d loss / d pre| where it may count
    sp = np.outer(s_dout, np.abs(w2)) * live + u * t_pre   # error scale of d loss / d pre
    fl = t_pre * flip                                      # terms that may be missing or extra
    sq = np.sqrt(B + 1) * u
    g_W1 = lam * np.sqrt((sq * (t_pre.T @ np.abs(A))) ** 2 + (sp * sp).T @ (A * A)) + fl.T @ np.abs(A)
    g_b1 = lam * np.sqrt((sq * t_pre.sum(axis=0)) ** 2 + (sp * sp).sum(axis=0)) + fl.sum(axis=0)
    g_w2 = lam * np.sqrt((sq * (hdn.T @ np.abs(d_out))) ** 2 + (hdn * hdn).T @ (s_dout * s_dout)
                         + (s_pre * s_pre).T @ (d_out * d_out))
    g_b2 = lam * np.sqrt((sq * np.abs(d_out).sum()) ** 2 + (s_dout * s_dout).sum())
    return pack(g_W1, g_b1, g_w2, g_b2)
