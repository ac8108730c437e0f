"""Pins of the oracle's solvers (CPU only).

* CG against dense Cholesky; Cholesky against its own residual.
* One level: plain RBF interpolation (the approximant reproduces f on X_1).
* Sequential (eq. (mas)) and monolithic (eq. (split) + Theorem jacobi)
  forms give the same coefficients.
* Nilpotency: from beta_0 = f, block k of beta is exact after k-1 sweeps;
  from an arbitrary beta_0 exactly L sweeps are needed (Theorem jacobi).
* The multiscale approximant interpolates f on the finest set and every
  partial sum f_l interpolates f on X_l (Section 2: e_l vanishes on X_l).
* Figure 1's printed values of ||M_L||_2.
"""
import os

import numpy as np
import pytest

import oracle
import synth
from oracle import multiscale as ms

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _hier(name):
    if name == "grid4":
        h = synth.grid_hierarchy()
        return h, synth.gauss_sine(h.points)
    if name == "halton5":
        h = synth.halton_hierarchy(5)
        return h, synth.fourier_target(1000)(h.points)
    if name == "uniform3d3":
        h = synth.uniform3d_hierarchy(3, n0=64)
        return h, synth.fourier_target(2001, 3)(h.points)
    if name == "table1_4":
        h = synth.table1_hierarchy(4)
        return h, synth.franke(h.points)
    raise KeyError(name)


@pytest.fixture(scope="module", params=["grid4", "halton5", "uniform3d3", "table1_4"])
def case(request):
    h, f = _hier(request.param)
    blk = ms.assemble(h.points, h.offsets, h.delta)
    return h, f, blk


def test_cg_matches_cholesky():
    h = synth.halton_hierarchy(4)
    blk = ms.assemble(h.points, h.offsets, h.delta)
    A = blk.mat(3, 3)
    b = np.random.default_rng(1).standard_normal(A.shape[0])
    xc = oracle.cholesky_solve(A, b)
    assert np.linalg.norm(A @ xc - b) <= 1e-13 * np.linalg.norm(b)
    xg, it = oracle.cg(A, b, 1e-14)
    assert 5 < it < 1000
    assert np.linalg.norm(xg - xc) <= 1e-12 * np.linalg.norm(xc)
    # warm start at the solution needs no iteration
    assert oracle.cg(A, b, 1e-10, x0=xc)[1] == 0


def test_single_level_is_rbf_interpolation():
    rng = np.random.default_rng(3)
    X = rng.random((400, 2))
    delta = np.array([0.2])
    off = np.array([0, 400])
    f = np.sin(3 * X[:, 0]) + X[:, 1] ** 2
    blk = ms.assemble(X, off, delta)
    a = oracle.sequential_solve(blk, f, solver="cholesky")
    # dense kernel matrix built pair by pair, independently of the CSR assembly
    Ad = ms.kernel_matrix_dense(X, 0.2)
    np.testing.assert_allclose(Ad @ a, f, rtol=0, atol=1e-12)
    np.testing.assert_allclose(oracle.evaluate(X, off, delta, a, X), f, rtol=0, atol=1e-12)


def test_sequential_equals_monolithic(case):
    h, f, blk = case
    a_seq = oracle.sequential_solve(blk, f)
    a_mono = oracle.monolithic_solve(blk, f)
    assert np.linalg.norm(a_mono - a_seq) <= 1e-11 * np.linalg.norm(a_seq)
    rel, per, _ = oracle.residual(blk, a_seq, f)
    assert rel <= 1e-12


def test_nilpotency_staircase(case):
    h, f, blk = case
    L = blk.levels
    a_seq = oracle.sequential_solve(blk, f)
    # exact beta of T' beta = f is D alpha
    beta_star = np.concatenate([blk.mat(l, l) @ a_seq[h.offsets[l]:h.offsets[l + 1]] for l in range(L)])
    _, hist = oracle.monolithic_solve(blk, f, sweeps=L, return_beta=True)
    for m, beta in enumerate(hist):
        for k in range(L):
            sl = slice(h.offsets[k], h.offsets[k + 1])
            err = np.linalg.norm(beta[sl] - beta_star[sl]) / np.linalg.norm(beta_star[sl])
            if k <= m:  # 0-based level k is exact after k sweeps
                assert err <= 1e-11, (m, k, err)
            elif m == 0 and k >= 1:
                assert err > 1e-6
    # from an arbitrary start: L sweeps are exact, L-1 are not (in general)
    beta0 = np.random.default_rng(5).standard_normal(h.n_total)
    _, hist0 = oracle.monolithic_solve(blk, f, sweeps=L, beta0=beta0, return_beta=True)
    top = slice(h.offsets[L - 1], h.offsets[L])
    e = lambda b: np.linalg.norm(b[top] - beta_star[top]) / np.linalg.norm(beta_star[top])
    assert e(hist0[L]) <= 1e-11
    assert e(hist0[L - 1]) > 1e-8


def test_partial_sums_interpolate(case):
    h, f, blk = case
    a = oracle.sequential_solve(blk, f)
    for l in range(blk.levels):
        X = h.level_points(l)
        fl = oracle.evaluate(h.points, h.offsets, h.delta, a, X, upto=l + 1)
        np.testing.assert_allclose(fl, f[h.offsets[l]:h.offsets[l + 1]], rtol=0,
                                   atol=1e-11 * np.abs(f).max())


def test_residual_detects_wrong_coefficients(case):
    h, f, blk = case
    a = oracle.sequential_solve(blk, f)
    bad = a.copy()
    sl = slice(h.offsets[1], h.offsets[2])
    bad[sl] *= -1.0
    assert oracle.residual(blk, bad, f)[0] > 1e-3
    bad2 = a.copy()
    bad2[-1] += 1e-3
    assert oracle.residual(blk, bad2, f)[0] > 1e-8


def test_evaluate_brute_equals_cells():
    h, f = _hier("halton5")
    blk = ms.assemble(h.points, h.offsets, h.delta)
    a = oracle.sequential_solve(blk, f)
    q = np.random.default_rng(9).random((1500, 2))
    e1 = oracle.evaluate(h.points, h.offsets, h.delta, a, q, method="brute")
    e2 = oracle.evaluate(h.points, h.offsets, h.delta, a, q, method="cells")
    np.testing.assert_array_equal(e1, e2)


def test_coefficient_scaling_convention():
    # with the paper's scaled kernel delta^-d phi(./delta) every block B_{k,j} is multiplied
    # by delta_j^-d, so its coefficients are delta_l^d times the unit-peak ones while the
    # approximant is unchanged
    h, f = _hier("halton5")
    blk = ms.assemble(h.points, h.offsets, h.delta)
    a = oracle.sequential_solve(blk, f)
    sc = ms.Blocks(blk.sizes)
    for (k, j), (rp, col, val) in blk.csr.items():
        sc.csr[(k, j)] = (rp, col, val * h.delta[j] ** -2)
    a_paper = oracle.sequential_solve(sc, f)
    scale = np.concatenate([np.full(n, h.delta[l] ** 2) for l, n in enumerate(h.sizes())])
    np.testing.assert_allclose(a_paper, scale * a, rtol=1e-9, atol=1e-12 * np.abs(a_paper).max())


def test_condition_numbers_level_independent():
    # Lemma condA: on quasi-uniform sets (here the Table 1 grids) kappa(A_l) is bounded
    # independently of the level
    h = synth.table1_hierarchy(5)
    blk = ms.assemble(h.points, h.offsets, h.delta)
    kap = [np.linalg.cond(blk.mat(l, l).toarray()) for l in range(2, 5)]
    assert max(kap) < 40.0 and max(kap) / min(kap) < 1.3


@pytest.mark.parametrize("L", [2, 3, 4, 5, 6, 7])
def test_fig1_spectral_norm_of_M(L):
    golden = dict(np.loadtxt(os.path.join(GOLDEN, "fig1_mnorm.txt")))
    h = synth.table1_hierarchy(L)
    blk = ms.assemble(h.points, h.offsets, h.delta)
    assert round(oracle.m_norm(blk), 3) == pytest.approx(golden[L], abs=1.5e-3)


def test_fig1_convention_distinguishes_spacing_delta():
    # the same grids with delta = 4 * spacing (not 4 * fill distance) do NOT give Figure 1
    golden = dict(np.loadtxt(os.path.join(GOLDEN, "fig1_mnorm.txt")))
    h = synth.table1_hierarchy(2, nu=4.0 * np.sqrt(2.0))
    blk = ms.assemble(h.points, h.offsets, h.delta)
    assert abs(oracle.m_norm(blk) - golden[2]) > 0.02
