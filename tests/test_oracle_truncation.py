"""Pins of the truncation oracle (Section 4, Thresholding; Section 5.2).

* Figures 2 and 3: the normalised norm difference and the nonzero ratio of
  M~_L(T) for L = 3..6 and T = 1..6 on the Table 1 grids equal the printed
  five-decimal values (tests/golden/fig2_truncation_norm.txt,
  fig3_truncation_nnz.txt); L = 7 runs in the slow set.
* Separation distances of the Table 1 grids equal the printed q_l.
* Lagrange property: X_{jj} = B_jj A_j^-1 = I, and on nested grids the rows
  of X_{kj} at points of level k that are also points of level j are unit
  vectors (chi_l^(j)(x_n^(j)) = delta_ln).
* Limits: T beyond the domain's diameter keeps M (ratio 0, nonzeros 1);
  T = 0 removes every entry (ratio 1, nonzeros 0).
* The perturbed solve: with untruncated blocks it reproduces the sequential
  solution; with truncated blocks its beta~ solves (I - M~) beta~ = f as a
  dense linear system, and alpha~ = D^-1 beta~.
"""
import os

import numpy as np
import pytest

import oracle
import synth
from oracle import multiscale as ms
from oracle import truncation as tr

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    t = np.loadtxt(os.path.join(GOLDEN, name))
    return {(int(L), int(T)): v for L, T, v in t}


@pytest.fixture(scope="module")
def fig_values():
    out = {}
    for L in (3, 4, 5, 6):
        h = synth.table1_hierarchy(L)
        blk = ms.assemble(h.points, h.offsets, h.delta)
        for T, v in tr.figure_quantities(blk, h.points, h.offsets, [1, 2, 3, 4, 5, 6]).items():
            out[(L, T)] = v
    return out


def test_fig2_norm_difference(fig_values):
    g = _golden("fig2_truncation_norm.txt")
    for key, (norm_ratio, _) in fig_values.items():
        assert round(norm_ratio, 5) == pytest.approx(g[key], abs=1.5e-5), key


def test_fig3_nonzero_ratio(fig_values):
    g = _golden("fig3_truncation_nnz.txt")
    for key, (_, nnz_ratio) in fig_values.items():
        assert round(nnz_ratio, 5) == pytest.approx(g[key], abs=1.5e-5), key


@pytest.mark.slow
def test_fig2_fig3_seven_levels():
    g2, g3 = _golden("fig2_truncation_norm.txt"), _golden("fig3_truncation_nnz.txt")
    h = synth.table1_hierarchy(7)
    blk = ms.assemble(h.points, h.offsets, h.delta)
    for T, (a, b) in tr.figure_quantities(blk, h.points, h.offsets, [1, 2, 3, 4, 5, 6]).items():
        assert round(a, 5) == pytest.approx(g2[(7, T)], abs=1.5e-5), T
        assert round(b, 5) == pytest.approx(g3[(7, T)], abs=1.5e-5), T


def test_separation_distance_table1():
    t = np.loadtxt(os.path.join(GOLDEN, "table1_sizes.txt"))
    for l, _, _, q in t:
        if l > 6:
            continue
        q_or = tr.separation_distance(synth.grid_points(int(l)))
        assert q_or == 2.0 ** -(l + 1), l  # half the spacing 2^-l, exactly
        assert q_or == pytest.approx(q, rel=2e-3), l  # the printed three digits
    # two points at distance 0.3 plus a far one: q = 0.15
    X = np.array([[0.0, 0.0], [0.3, 0.0], [5.0, 5.0]])
    assert tr.separation_distance(X) == pytest.approx(0.15, rel=1e-15)


def test_lagrange_property():
    h = synth.table1_hierarchy(4)
    blk = ms.assemble(h.points, h.offsets, h.delta)
    for j in range(4):
        assert np.allclose(tr.lagrange_block(blk, j, j), np.eye(blk.sizes[j]), atol=1e-10)
    # nested grids: point n of level j sits on level k as well
    for k in range(1, 4):
        Xk = h.points[h.offsets[k]:h.offsets[k + 1]]
        for j in range(k):
            Xj = h.points[h.offsets[j]:h.offsets[j + 1]]
            Xkj = tr.lagrange_block(blk, k, j)
            hits = 0
            for n, x in enumerate(Xj):
                i = np.flatnonzero(np.all(Xk == x, axis=1))
                assert i.size == 1
                e = np.zeros(blk.sizes[j])
                e[n] = 1.0
                assert np.allclose(Xkj[i[0]], e, atol=1e-10)
                hits += 1
            assert hits == blk.sizes[j]


def test_truncation_limits():
    h = synth.table1_hierarchy(3)
    blk = ms.assemble(h.points, h.offsets, h.delta)
    q = [tr.separation_distance(h.points[h.offsets[l]:h.offsets[l + 1]]) for l in range(3)]
    big = 10.0 / min(q)  # radius T q_j beyond the unit square's diameter for every j
    r = tr.figure_quantities(blk, h.points, h.offsets, [0.0, big])
    assert r[0.0] == (1.0, 0.0)
    assert r[big][0] == 0.0 and r[big][1] == 1.0


def test_truncated_solve_exact_and_perturbed():
    h = synth.table1_hierarchy(4)
    f = synth.franke(h.points)
    blk = ms.assemble(h.points, h.offsets, h.delta)
    blocks = tr.m_blocks(blk)
    # no truncation: the sequential (exact) coefficients
    a_full = tr.truncated_solve(blk, f, blocks)
    a_seq = oracle.sequential_solve(blk, f)
    assert np.linalg.norm(a_full - a_seq) <= 1e-10 * np.linalg.norm(a_seq)
    # truncated at T = 3: (I - M~) beta~ = f as one dense solve, M~ = -X~
    q = [tr.separation_distance(h.points[h.offsets[l]:h.offsets[l + 1]]) for l in range(4)]
    tb = tr.truncate(blocks, h.points, h.offsets, q, 3.0)
    a_t, b_t = tr.truncated_solve(blk, f, tb, return_beta=True)
    N = h.n_total
    Mt = np.zeros((N, N))
    Mt[:, :h.offsets[-2]] = -tr.assemble_dense(tb, blk.sizes)
    b_dense = np.linalg.solve(np.eye(N) - Mt, f)
    assert np.linalg.norm(b_t - b_dense) <= 1e-12 * np.linalg.norm(b_dense)
    # alpha~ = D^-1 beta~ level by level
    for l in range(4):
        s = slice(h.offsets[l], h.offsets[l + 1])
        assert np.allclose(blk.mat(l, l) @ a_t[s], b_t[s], rtol=0, atol=1e-11 * np.abs(b_t).max())
    # and the truncation changed the answer (T = 3 drops entries)
    assert np.linalg.norm(a_t - a_seq) > 1e-6 * np.linalg.norm(a_seq)
