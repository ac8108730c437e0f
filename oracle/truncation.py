"""Thresholded Jacobi of Section 4 (truncated Lagrange blocks) in plain FP64.

TEST INFRASTRUCTURE ONLY (see the package header): nothing in the GPU library
imports this module.

Definitions followed (Section 4, "Thresholding"):

* the Lagrange functions of level j, chi_l^(j) = sum_m c_m phi_j(. - x_m^(j))
  with A_j c = e_l, so chi_l^(j)(x_n^(j)) = delta_{ln};
* the blocks of M = I - T'_L (eq. (M)): block (k, j), k > j, has entry (i, l)
  = chi_l^(j)(x_i^(k)), i.e. the matrix frak X_{kj} = B_{kj} A_j^-1 (the
  sign of the Jacobi update is carried by the solver below, reading R5);
* the truncated blocks frak X~_{kj}(T): the entry (i, l) is kept iff the
  distance between the evaluation point x_i^(k) and the centre x_l^(j) is
  strictly below T max(q_k, q_j) = T q_j, q the separation distance of a
  level (half the smallest distance between two of its points); all other
  entries are zero (the printed definition swaps the indices of the two
  points; read as row point against centre, as everywhere else);
* M~(T) (eq. (perturbedmatrix)) has these blocks, and the perturbed split
  (eq. (perturbed_split)) is D alpha~ = beta~, (I - M~(T)) beta~ = f.

Section 5.2 reports two quantities per (L, T) on the Table 1 grids:
||M - M~(T)||_2 / ||M||_2 (Figure 2) and nnz(M~(T)) / nnz(M) (Figure 3). The
count of nonzeros ignores entries of magnitude <= 1e-8 (M is dense in exact
arithmetic; entries at rounding level are not counted) - a reading, since
the paper does not say how it counted.

Library primitives used as single steps: dense Cholesky factorisation and
triangular solves (numpy/scipy), the dense spectral norm (numpy SVD) and
ARPACK's largest singular value for large matrices. Everything else is
written out here.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse.linalg as spla

from .multiscale import Blocks, split_levels, _level_solver

NNZ_EPS = 1e-8  # magnitude at or below which an entry of M is not counted


def separation_distance(X: np.ndarray, chunk: int = 2048) -> float:
    """q = half the smallest distance between two distinct points of X (all
    pairs, in row chunks)."""
    X = np.ascontiguousarray(X, dtype=np.float64)
    n = X.shape[0]
    if n < 2:
        return float("inf")
    best = np.inf
    for a in range(0, n, chunk):
        b = min(n, a + chunk)
        d2 = None
        for ax in range(X.shape[1]):
            dx = X[a:b, None, ax] - X[None, :, ax]
            d2 = dx * dx if d2 is None else d2 + dx * dx
        idx = np.arange(a, b)
        d2[idx - a, idx] = np.inf  # a point against itself
        best = min(best, float(d2.min()))
    return 0.5 * float(np.sqrt(best))


def lagrange_block(blk: Blocks, k: int, j: int) -> np.ndarray:
    """frak X_{kj} = B_{kj} A_j^-1 as a dense N(k) x N(j) array: column l holds
    the Lagrange function chi_l^(j) at the points of level k. A_j^-1 is
    applied through its Cholesky factor (A_j is SPD)."""
    Aj = blk.mat(j, j).toarray()
    C = np.linalg.cholesky(Aj)
    Bt = blk.mat(k, j).toarray().T  # N(j) x N(k)
    # X^T = A_j^-1 B_kj^T (A_j symmetric)
    Y = sla.solve_triangular(C, Bt, lower=True)
    Xt = sla.solve_triangular(C.T, Y, lower=False)
    return np.ascontiguousarray(Xt.T)


def distance_mask(Xk: np.ndarray, Xj: np.ndarray, radius: float) -> np.ndarray:
    """Boolean N(k) x N(j): ||x_i^(k) - x_l^(j)|| < radius (squared distances
    compared with radius^2, left to right, no fusion)."""
    d2 = None
    for ax in range(Xk.shape[1]):
        dx = Xk[:, None, ax] - Xj[None, :, ax]
        d2 = dx * dx if d2 is None else d2 + dx * dx
    return d2 < radius * radius


def m_blocks(blk: Blocks) -> dict:
    """All blocks frak X_{kj}, k > j, of M (dense)."""
    return {(k, j): lagrange_block(blk, k, j) for k in range(blk.levels) for j in range(k)}


def truncate(blocks: dict, points: np.ndarray, offsets, q, T: float) -> dict:
    """frak X~_{kj}(T): entries with ||x_i^(k) - x_l^(j)|| >= T q_j set to 0."""
    out = {}
    for (k, j), X in blocks.items():
        Xk = points[offsets[k]:offsets[k + 1]]
        Xj = points[offsets[j]:offsets[j + 1]]
        out[(k, j)] = np.where(distance_mask(Xk, Xj, T * q[j]), X, 0.0)
    return out


def assemble_dense(blocks: dict, sizes) -> np.ndarray:
    """The strictly block-lower matrix with the given blocks, N rows and the
    columns of levels < L only (the last level's columns are zero; the sign
    of M does not change any norm or count below)."""
    off = np.concatenate(([0], np.cumsum(sizes)))
    M = np.zeros((int(off[-1]), int(off[-2])))
    for (k, j), X in blocks.items():
        M[off[k]:off[k + 1], off[j]:off[j + 1]] = X
    return M


def spectral_norm(M: np.ndarray) -> float:
    """Largest singular value: dense SVD up to 4096 columns, ARPACK above."""
    if min(M.shape) <= 4096:
        return float(np.linalg.norm(M, 2))
    s = spla.svds(M, k=1, return_singular_vectors=False, tol=1e-12, random_state=0)
    return float(s[0])


def figure_quantities(blk: Blocks, points: np.ndarray, offsets, Ts) -> dict:
    """For each T: (||M - M~(T)||_2 / ||M||_2, nnz(M~(T)) / nnz(M)), the
    quantities of Figures 2 and 3. Only the columns of levels < L carry
    nonzeros, so the matrices hold those columns only."""
    sizes = blk.sizes
    L = len(sizes)
    q = [separation_distance(points[offsets[l]:offsets[l + 1]]) for l in range(L)]
    blocks = m_blocks(blk)
    M = assemble_dense(blocks, sizes)
    nM = spectral_norm(M)
    nnzM = int(np.count_nonzero(np.abs(M) > NNZ_EPS))
    out = {}
    for T in Ts:
        Mt = assemble_dense(truncate(blocks, points, offsets, q, T), sizes)
        nnz_ratio = int(np.count_nonzero(np.abs(Mt) > NNZ_EPS)) / nnzM
        np.subtract(M, Mt, out=Mt)  # M - M~(T), in place
        out[T] = (spectral_norm(Mt) / nM, nnz_ratio)
    return out


def truncated_solve(blk: Blocks, f: np.ndarray, tblocks: dict, solver: str = "auto", rtol: float = 1e-14,
                    sweeps: int | None = None, return_beta: bool = False):
    """Solution of the perturbed split (eq. (perturbed_split)).

    Jacobi on (I - M~) beta~ = f with M~ = -frak X~ (reading R5): starting
    from beta~ = f, each sweep sets beta~^(k) = f^(k) - sum_{j<k} X~_{kj}
    beta~^(j); the truncated matrix is still strictly block lower, so L-1
    sweeps give the exact solution of the perturbed system. Then
    alpha~_l = A_l^-1 beta~^(l) on every level.
    """
    L = blk.levels
    S = L - 1 if sweeps is None else sweeps
    fl = split_levels(f, blk.sizes)
    beta = [b.copy() for b in fl]
    for _ in range(S):
        new = [fl[0].copy()]
        for k in range(1, L):
            acc = fl[k].copy()
            for j in range(k):
                acc -= tblocks[(k, j)] @ beta[j]
            new.append(acc)
        beta = new
    solve = _level_solver(solver, rtol)
    alpha = np.concatenate([solve(blk.mat(l, l), beta[l]) for l in range(L)])
    if return_beta:
        return alpha, np.concatenate(beta)
    return alpha
