"""Pins of the oracle's kernel and block assembly (CPU only).

Each test ties the oracle to something other than itself: closed-form values
of phi_{3,1} worked out by hand, lattice-point counts, brute force, symmetry
and nesting properties of the blocks defined in Section 3, and the input
recipe of Table 1.
"""
import math
import os

import numpy as np
import pytest

import oracle
import synth
from oracle import multiscale as ms
from oracle.wendland import phi31

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# --- phi_{3,1} (Section 5) ------------------------------------------------------------

def test_phi_special_values():
    # phi(0) = 1 (unit peak), phi(1/2) = (1/2)^4 * 3 = 3/16, zero on and beyond r = 1
    assert phi31(0.0) == 1.0
    assert phi31(0.5) == 0.1875
    assert phi31(1.0) == 0.0
    assert np.all(phi31(np.array([1.0 + 1e-12, 1.5, 7.0])) == 0.0)
    # hand-computed fractions: phi(3/7) = (4/7)^4 (19/7) = 4864/16807,
    # phi(6/7) = (1/7)^4 (31/7) = 31/16807
    assert phi31(3.0 / 7.0) == pytest.approx(4864.0 / 16807.0, rel=1e-15)
    assert phi31(6.0 / 7.0) == pytest.approx(31.0 / 16807.0, rel=1e-13)


def test_phi_smoothness_at_support_edge_and_origin():
    # C^2 contact with zero at r = 1: phi(1-h) / h^4 -> 5 ; flat top: (1-phi(h))/h^2 -> 10
    for h in (1e-2, 1e-3):
        assert phi31(1.0 - h) / h ** 4 == pytest.approx(5.0 - 4.0 * h, rel=1e-6)
        assert (1.0 - phi31(h)) / h ** 2 == pytest.approx(10.0, rel=0.05)
    r = np.linspace(0.0, 1.0, 1001)
    assert np.all(np.diff(phi31(r)) <= 0.0)  # monotone decreasing on [0, 1]


@pytest.mark.parametrize("d", [1, 2, 3])
def test_phi_positive_definite(d):
    # Wendland phi_{3,1} is positive definite on R^d for d <= 3 (the paper's A_l are SPD)
    rng = np.random.default_rng(7 + d)
    X = rng.random((300, d))
    A = ms.kernel_matrix_dense(X, delta=0.35)
    ev = np.linalg.eigvalsh(A)
    assert ev.min() > 0.0
    assert np.allclose(A, A.T, rtol=0, atol=0)


# --- blocks B_{k,j} (Section 3) ---------------------------------------------------------

def test_tiny_block_by_hand():
    # points 0, 0.3, 0.9 on a line (embedded in 2-D), delta = 0.7: pairs at 0.3 and 0.6 are in
    X = np.array([[0.0, 0.0], [0.3, 0.0], [0.9, 0.0]])
    rp, col, val = oracle.block_bruteforce(X, X, 0.7)
    assert rp.tolist() == [0, 2, 5, 7]
    assert col.tolist() == [0, 1, 0, 1, 2, 1, 2]
    a, b = 4864.0 / 16807.0, 31.0 / 16807.0  # phi(3/7), phi(6/7)
    np.testing.assert_allclose(val, [1, a, a, 1, b, b, 1], rtol=1e-12)


def test_grid_counts_strict_support():
    # spacing s, delta = 4 s: interior rows hold the lattice points with i^2 + j^2 < 16
    # (45 of them); the 4 points with i^2+j^2 = 16 sit exactly at distance delta and are
    # excluded by the strict support. A corner holds the quarter disc: 15 points.
    h = synth.grid_hierarchy()
    blk = ms.assemble(h.points, h.offsets, h.delta)
    rp = blk.csr[(3, 3)][0]
    cnt = np.diff(rp)
    n = 65
    ij = np.arange(n * n)
    ix, iy = ij % n, ij // n
    interior = (ix >= 4) & (ix <= n - 5) & (iy >= 4) & (iy <= n - 5)
    assert np.all(cnt[interior] == 45)
    assert cnt[0] == 15 and cnt[n - 1] == 15 and cnt[n * n - 1] == 15
    assert cnt.max() == 45


def _assert_same_csr(a, b):
    assert np.array_equal(a[0], b[0])
    assert np.array_equal(a[1], b[1])
    assert np.array_equal(a[2], b[2])


@pytest.mark.parametrize("case", ["grid", "halton", "uniform3d", "random2d_off", "scattered_rows"])
def test_cells_equal_bruteforce(case):
    rng = np.random.default_rng(11)
    if case == "grid":
        h = synth.grid_hierarchy()
        pairs = [(h.level_points(3), h.level_points(1), h.delta[1]), (h.level_points(3), h.level_points(3), h.delta[3])]
    elif case == "halton":
        h = synth.halton_hierarchy(5)
        pairs = [(h.level_points(4), h.level_points(j), h.delta[j]) for j in range(5)]
    elif case == "uniform3d":
        h = synth.uniform3d_hierarchy(3, n0=64)
        pairs = [(h.level_points(2), h.level_points(j), h.delta[j]) for j in range(3)]
    elif case == "random2d_off":
        # rows outside the centres' bounding box, negative coordinates
        pairs = [(rng.random((2000, 2)) * 3 - 1, rng.random((700, 2)), 0.11)]
    else:
        pairs = [(rng.random((3000, 2)), rng.random((2500, 2)) * 0.5, 0.05)]
    for rows, cols, dl in pairs:
        _assert_same_csr(oracle.block_bruteforce(rows, cols, dl), oracle.block_cells(rows, cols, dl))


def test_blocks_symmetric_and_nested():
    h = synth.halton_hierarchy(5)
    blk = ms.assemble(h.points, h.offsets, h.delta)
    for l in range(5):
        A = blk.mat(l, l)
        D = (A - A.T)
        assert D.nnz == 0 or abs(D).max() == 0.0  # bitwise symmetric values and structure
        assert np.all(A.diagonal() == 1.0)
    # prefix nesting: the first N_j points of level k are level j's points, so those rows of
    # B_{k,j} (centre radius delta_j) are the rows of A_j
    for k in range(1, 5):
        for j in range(k):
            Bk = blk.mat(k, j)[: blk.sizes[j]]
            assert (Bk != blk.mat(j, j)).nnz == 0


def test_nnz_per_row_matches_density():
    # nu = sqrt(40/pi): about 40 same-level points inside delta for interior points
    h = synth.halton_hierarchy(6)
    blk = ms.assemble(h.points, h.offsets, h.delta)
    cnt = np.diff(blk.csr[(5, 5)][0])
    assert 38.0 < cnt.mean() < 41.0
    h3 = synth.uniform3d_hierarchy(3)
    blk3 = ms.assemble(h3.points, h3.offsets, h3.delta)
    c3 = np.diff(blk3.csr[(2, 2)][0]).mean()
    assert 50.0 < c3 < 61.0


# --- inputs -----------------------------------------------------------------------------

def test_table1_recipe_matches_paper():
    rows = np.loadtxt(os.path.join(GOLDEN, "table1_sizes.txt"))
    for l, n, hl, ql in rows:
        l = int(l)
        s = 2.0 ** -l
        assert (2 ** l + 1) ** 2 == int(n)
        # printed to three significant digits
        assert s / math.sqrt(2) == pytest.approx(hl, rel=2e-3)
        assert s / 2 == pytest.approx(ql, rel=2e-3)
    h = synth.table1_hierarchy(4)
    assert h.sizes() == [9, 25, 81, 289]
    assert h.delta[0] == pytest.approx(4 * 0.5 / math.sqrt(2))


def test_generators_published_values():
    # SplitMix64 seeded with 0: the published first outputs
    z = synth.splitmix64(0, 0, 3)
    assert [int(v) for v in z] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    # Halton (2,3) from index 1
    np.testing.assert_allclose(synth.halton(3), [[0.5, 1 / 3], [0.25, 2 / 3], [0.75, 1 / 9]], rtol=1e-15)
    h = synth.halton_hierarchy(8)
    assert h.sizes() == [64 * 4 ** j for j in range(8)] and h.n_total == 1398080
