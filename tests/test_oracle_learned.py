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
