"""Pins of the learned warm start's reference (CPU only): exact kNN lists
against scipy's KD-tree (an independent library routine), bfloat16 rounding
against hand-worked bit patterns, the vectorised forward pass against plain
loops, and the feature layout against its definition."""
import numpy as np
import pytest
from scipy.spatial import cKDTree

from oracle import learned as ol


@pytest.mark.parametrize("d,n", [(2, 700), (3, 500), (2, 10)])
def test_knn_matches_kdtree(d, n):
    X = np.random.default_rng(d * 100 + n).random((n, d))
    nb = ol.knn16(X)
    k = min(16, n - 1)
    dist, idx = cKDTree(X).query(X, k=k + 1)
    for i in range(n):
        ref = [j for j in idx[i] if j != i][:k]
        assert sorted(nb[i, :k]) == sorted(ref)
        d2 = ((X[nb[i, :k]] - X[i]) ** 2).sum(axis=1)
        assert np.all(np.diff(d2) >= 0)  # ascending distance
        assert np.all(nb[i, k:] == i)  # padding with self on tiny levels


def test_knn_ties_by_index():
    # points on a grid: many exact distance ties; order (d2, index)
    t = np.arange(6) * 0.125
    X = np.stack(np.meshgrid(t, t, indexing="ij"), -1).reshape(-1, 2)
    nb = ol.knn16(X)
    for i in range(len(X)):
        d2 = ((X[nb[i]] - X[i]) ** 2).sum(axis=1)
        for a in range(15):
            assert d2[a] < d2[a + 1] or (d2[a] == d2[a + 1] and nb[i, a] < nb[i, a + 1])


def test_bf16_rounding_hand_values():
    x = np.array([1.0, 1.0 / 3.0, -2.5, 1.00390625, 1.005859375, 65504.0], dtype=np.float32)
    # 1/3 = 0x3EAAAAAB -> 0x3EAB; 1+2^-8 is a tie -> even (1.0); 1+3*2^-9 rounds up to 1+2^-7
    got = ol.bf16(x).view(np.uint32) >> 16
    assert got.tolist() == [0x3F80, 0x3EAB, 0xC020, 0x3F80, 0x3F81, 0x4780]


def test_forward_matches_loops_and_features():
    rng = np.random.default_rng(4)
    X = rng.random((200, 2))
    b = rng.standard_normal(200)
    nb = ol.knn16(X)
    feat, s = ol.features(X, b, nb, delta=0.1)
    assert feat.shape == (200, ol.feature_count(2)) and ol.feature_count(2) == 56 and ol.feature_count(3) == 72
    i = 17
    assert feat[i, 0] == pytest.approx(b[i] / s[i], rel=1e-6)
    assert feat[i, 1 + 3 * 2] == pytest.approx(b[nb[i, 2]] / s[i], rel=1e-6)
    assert feat[i, 2 + 3 * 2] == pytest.approx((X[nb[i, 2], 0] - X[i, 0]) / 0.1, rel=1e-6)
    assert np.all(feat[:, 49:] == 0)
    W1 = rng.standard_normal((64, 56)).astype(np.float32) * 0.2
    b1 = rng.standard_normal(64).astype(np.float32) * 0.1
    w2 = rng.standard_normal(64).astype(np.float32) * 0.2
    out = ol.forward(W1, b1, w2, 0.05, feat, s)
    for i in (0, 50, 199):
        assert out[i] == pytest.approx(ol.forward_loop(W1, b1, w2, 0.05, feat[i], s[i]), rel=1e-12, abs=1e-14)


def test_features_three_point_level_by_hand():
    # level of 3 points: the kNN list is the two others by distance, then the
    # point itself 14 times; s^2 = (b_i^2 + b_1^2 + b_2^2 + 14 b_i^2) / 17
    X = np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 2.0]])
    b = np.array([1.0, 2.0, 3.0])
    nb = ol.knn16(X)
    assert nb[0].tolist() == [1, 2] + [0] * 14
    assert nb[2].tolist() == [0, 1] + [2] * 14  # d^2 = 4 and 5
    feat, s = ol.features(X, b, nb, delta=0.5)
    assert s[0] == np.sqrt(28.0 / 17.0)
    assert s[2] == np.sqrt((9.0 + 1.0 + 4.0 + 14 * 9.0) / 17.0)
    sc = np.sqrt(28.0 / 17.0)
    want = [1 / sc, 2 / sc, 2.0, 0.0, 3 / sc, 0.0, 4.0] + [1 / sc, 0.0, 0.0] * 14
    want = np.array(want + [0.0] * (56 - len(want)), dtype=np.float32)
    assert np.array_equal(feat[0], want)


def test_forward_by_hand():
    F = 56
    W1 = np.zeros((2, F), dtype=np.float32)
    W1[0, 0], W1[0, 1], W1[1, 0] = 1.0, -1.0, 0.5
    b1 = np.array([0.0, 0.25], dtype=np.float32)
    w2 = np.array([2.0, -4.0], dtype=np.float32)
    feat = np.zeros((3, F), dtype=np.float32)
    feat[0, :2] = [3.0, 1.0]        # hidden (2, 1.75): y = 4 - 7 + 0.5 = -2.5, x0 = s y
    feat[1, :2] = [-1.0, 1.0]       # hidden (0, 0) after the ReLU: y = b2
    feat[2, 1] = np.float32(-1 / 3)  # bf16(-1/3) = -0.333984375: hidden (0.333984375, 0.25)
    s = np.array([2.0, 1.0, 1.0])
    out = ol.forward(W1, b1, w2, 0.5, feat, s)
    assert out[0] == -5.0 and out[1] == 0.5
    assert out[2] == 2.0 * 0.333984375 - 4.0 * 0.25 + 0.5
    assert ol.forward(W1, b1, w2, 0.5, feat, s, bf16_first_layer=False)[2] == \
        2.0 * float(np.float32(1 / 3)) - 4.0 * 0.25 + 0.5


def test_gradient_by_hand():
    # 2 hidden units, 2 features, one sample: a = (3.5, -2.5), h = (3.5, 0),
    # out = 10.75, e = 8.75, loss = 76.5625, d out = 17.5
    W1 = np.array([[1.0, 2.0], [-1.0, 0.5]])
    b1 = np.array([0.5, -2.0])
    w2 = np.array([3.0, -1.0])
    loss, (gW1, gb1, gw2, gb2) = ol.loss_and_grads(W1, b1, w2, 0.25, np.array([[1.0, 1.0]]), np.array([2.0]))
    assert loss == 76.5625
    assert gb2 == 17.5
    assert gw2.tolist() == [61.25, 0.0]
    assert gb1.tolist() == [52.5, 0.0]
    assert gW1.tolist() == [[52.5, 52.5], [0.0, 0.0]]


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(7)
    B, F, H = 9, 6, 5
    X = rng.standard_normal((B, F))
    y = rng.standard_normal(B)
    p = ol.pack(rng.standard_normal((H, F)), rng.standard_normal(H), rng.standard_normal(H), 0.3)

    def loss(q):
        W1, b1, w2, b2 = ol.unpack(q, F, H)
        return ol.loss_and_grads(W1, b1, w2, b2, X, y, bf16_first_layer=False)[0]

    W1, b1, w2, b2 = ol.unpack(p, F, H)
    g = ol.pack(*ol.loss_and_grads(W1, b1, w2, b2, X, y, bf16_first_layer=False)[1])
    h = 1e-6
    fd = np.array([(loss(p + h * e) - loss(p - h * e)) / (2 * h) for e in np.eye(len(p))])
    assert np.allclose(g, fd, rtol=1e-6, atol=1e-7)


def test_bf16_gradient_is_taken_at_the_rounded_values():
    # straight-through: the gradient equals the FP64 gradient at bf16(W1), bf16(X)
    rng = np.random.default_rng(8)
    X = rng.standard_normal((7, 8)).astype(np.float32)
    W1 = rng.standard_normal((3, 8)).astype(np.float32)
    b1, w2, y = rng.standard_normal(3), rng.standard_normal(3), rng.standard_normal(7)
    a = ol.loss_and_grads(W1, b1, w2, 0.1, X, y, bf16_first_layer=True)
    b = ol.loss_and_grads(ol.bf16(W1), b1, w2, 0.1, ol.bf16(X), y, bf16_first_layer=False)
    assert a[0] == b[0]
    for ga, gb in zip(a[1], b[1]):
        assert np.array_equal(ga, gb)
    assert not np.array_equal(ol.bf16(W1), W1)


def test_adam_closed_form_under_constant_gradient():
    # with m0 = v0 = 0 the bias-corrected moments of a constant gradient are g
    # and g^2 at every step, so each step moves by -lr g / (|g| + eps)
    g = np.array([3.0, -2e-3, 0.0, 1e-9])
    p, m, v = np.zeros(4), np.zeros(4), np.zeros(4)
    for t in range(1, 6):
        p_new, m, v = ol.adam_update(p, g, m, v, t, lr=1e-2)
        assert np.allclose(p_new - p, -1e-2 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-18)
        p = p_new
    # a gradient that flips sign after one step: m_2 = 0.1 (0.9 g - g) ...
    p, m, v = ol.adam_update(np.zeros(1), np.array([1.0]), np.zeros(1), np.zeros(1), 1, lr=1.0)
    p2, m2, v2 = ol.adam_update(p, np.array([-1.0]), m, v, 2, lr=1.0)
    mh = (0.9 * 0.1 - 0.1) / (1 - 0.81)
    vh = (0.999 * 0.001 + 0.001) / (1 - 0.999 ** 2)
    assert p2[0] - p[0] == pytest.approx(-mh / (np.sqrt(vh) + 1e-8), rel=1e-12)


def test_batch_schedule_by_listing():
    assert ol.batch_rows(0, 5, batch=3).tolist() == [0, 1, 2]
    assert ol.batch_rows(1, 5, batch=3).tolist() == [3, 4, 0]
    assert ol.batch_rows(2, 5, batch=3).tolist() == [1, 2, 3]


def test_train_lowers_the_loss_of_a_learnable_target():
    # a target that the network class contains (a teacher network of the same
    # shape): Adam drives the mini-batch loss far down
    rng = np.random.default_rng(9)
    F, ns = 56, 1024
    X = rng.standard_normal((ns, F)).astype(np.float32)
    teacher = ol.pack(rng.standard_normal((64, F)) * 0.2, rng.standard_normal(64) * 0.1,
                      rng.standard_normal(64) * 0.2, 0.05)
    W1, b1, w2, b2 = ol.unpack(teacher, F)
    y = ol.forward(W1, b1, w2, b2, X, np.ones(ns))
    p0 = ol.pack(rng.standard_normal((64, F)) * 0.1, np.zeros(64), rng.standard_normal(64) * 0.1, 0.0)
    _, losses = ol.train(p0, X, y, steps=400, lr=3e-3)
    assert losses[-8:].mean() < 0.1 * losses[:8].mean()


def test_grad_error_bound_covers_fp32_evaluation():
    # an FP32 evaluation of the same gradient stays within the bound
    rng = np.random.default_rng(10)
    B, F, H = 128, 56, 64
    X = rng.standard_normal((B, F)).astype(np.float32)
    y = rng.standard_normal(B).astype(np.float32)
    W1 = (rng.standard_normal((H, F)) * 0.2).astype(np.float32)
    b1 = (rng.standard_normal(H) * 0.1).astype(np.float32)
    w2 = (rng.standard_normal(H) * 0.2).astype(np.float32)
    _, g = ol.loss_and_grads(W1, b1, w2, 0.05, X, y)
    g = ol.pack(*g)
    A, W = ol.bf16(X), ol.bf16(W1)
    pre = (A @ W.T + b1).astype(np.float32)
    hdn = np.maximum(pre, np.float32(0))
    d_out = (np.float32(2) * ((hdn @ w2 + np.float32(0.05)) - y) / np.float32(B)).astype(np.float32)
    d_pre = (np.outer(d_out, w2) * (pre > 0)).astype(np.float32)
    g32 = ol.pack(d_pre.T @ A, d_pre.sum(axis=0), hdn.T @ d_out, d_out.sum())
    bound = ol.grad_error_bound(W1, b1, w2, 0.05, X, y)
    assert np.all(np.abs(g32 - g) <= bound)
    assert np.median(bound / np.maximum(np.abs(g), 1e-30)) < 1e-3  # and is not vacuous
