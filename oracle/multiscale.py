"""Solvers of the multiscale method in plain FP64 (Sections 2-3, 5).

Notation follows the paper: levels l = 1..L (0-based in code), blocks
B_{k,j} (rows: level k, columns: level j, radius delta_j), A_l = B_{l,l},
the block-lower-triangular T_L of eq. (bigt), its factorisation
T_L = T'_L D_L (eq. (matrix_decomposition)) and the split
D alpha = beta, T' beta = f (eq. (split)).

Library primitives used as single steps: scipy CSR matrix-vector products,
numpy dense Cholesky, scipy triangular solves, scipy sparse LU and ARPACK
(for the spectral norm only). Everything else is written out here.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .neighbours import block_bruteforce, block_cells
from .wendland import phi31

BRUTE_FORCE_MAX_PAIRS = 20_000_000


@dataclass
class Blocks:
    """All blocks B_{k,j}, k >= j, of one hierarchy in canonical CSR."""

    sizes: list
    csr: dict = field(default_factory=dict)  # (k, j) -> (rowptr, col, val)

    @property
    def levels(self) -> int:
        return len(self.sizes)

    def mat(self, k: int, j: int) -> sp.csr_matrix:
        rp, col, val = self.csr[(k, j)]
        return sp.csr_matrix((val, col, rp), shape=(self.sizes[k], self.sizes[j]))

    def nnz(self, k: int, j: int) -> int:
        return int(self.csr[(k, j)][0][-1])


def assemble(points: np.ndarray, offsets: np.ndarray, delta: np.ndarray, method: str = "auto") -> Blocks:
    """Every block B_{k,j} (k >= j) of the hierarchy (Section 3).

    ``method``: "brute" (all pairs), "cells" (bucket search) or "auto"
    (brute force for blocks up to 2e7 pairs, cells above).
    """
    L = len(delta)
    sizes = [int(offsets[l + 1] - offsets[l]) for l in range(L)]
    blk = Blocks(sizes)
    for k in range(L):
        Xk = points[offsets[k]:offsets[k + 1]]
        for j in range(k + 1):
            Xj = points[offsets[j]:offsets[j + 1]]
            use_brute = method == "brute" or (method == "auto" and sizes[k] * sizes[j] <= BRUTE_FORCE_MAX_PAIRS)
            f = block_bruteforce if use_brute else block_cells
            blk.csr[(k, j)] = f(Xk, Xj, float(delta[j]))
    return blk


def split_levels(v: np.ndarray, sizes) -> list:
    out, s = [], 0
    for n in sizes:
        out.append(v[s:s + n])
        s += n
    return out


def cg(A, b: np.ndarray, rtol: float, x0: np.ndarray | None = None, maxiter: int = 100000):
    """Textbook conjugate gradients (Hestenes-Stiefel) for SPD A.

    Starts from x0 (zero by default, as Algorithm 1 does) and stops once
    ||r||_2 <= rtol * ||b||_2. Returns (x, iterations).
    """
    b = np.asarray(b, dtype=np.float64)
    if b.shape[0] == 0:
        return np.zeros(0), 0
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    r = b - A @ x if x0 is not None else b.copy()
    bnorm = np.linalg.norm(b)
    rr = float(r @ r)
    if np.sqrt(rr) <= rtol * bnorm:
        return x, 0
    p = r.copy()
    it = 0
    while it < maxiter:
        q = A @ p
        alpha = rr / float(p @ q)
        x += alpha * p
        r -= alpha * q
        rr_new = float(r @ r)
        it += 1
        if np.sqrt(rr_new) <= rtol * bnorm:
            break
        p = r + (rr_new / rr) * p
        rr = rr_new
    return x, it


def cholesky_solve(A, b: np.ndarray) -> np.ndarray:
    """Direct solve of the SPD system A x = b by dense Cholesky A = C C^T."""
    Ad = A.toarray() if sp.issparse(A) else np.asarray(A)
    if Ad.shape[0] == 0:
        return np.zeros(0)
    C = np.linalg.cholesky(Ad)
    y = sla.solve_triangular(C, b, lower=True)
    return sla.solve_triangular(C.T, y, lower=False)


def _level_solver(kind: str, rtol: float):
    if kind == "cholesky":
        return lambda A, b: cholesky_solve(A, b)
    if kind == "cg":
        return lambda A, b: cg(A, b, rtol)[0]
    if kind == "auto":  # exact-ish: Cholesky on small levels, tight CG above
        return lambda A, b: cholesky_solve(A, b) if A.shape[0] <= 4096 else cg(A, b, min(rtol, 1e-14))[0]
    raise ValueError(kind)


def sequential_solve(blk: Blocks, f: np.ndarray, solver: str = "auto", rtol: float = 1e-14) -> np.ndarray:
    """Coefficients of the sequential multiscale algorithm, eq. (mas).

    For l = 1..L: A_l alpha^(l) = f^(l) - sum_{k<l} B_{l,k} alpha^(k), i.e.
    block forward substitution with the block-lower-triangular T_L.
    """
    solve = _level_solver(solver, rtol)
    fl = split_levels(f, blk.sizes)
    alpha = []
    for l in range(blk.levels):
        rhs = fl[l].copy()
        for k in range(l):
            rhs -= blk.mat(l, k) @ alpha[k]
        alpha.append(solve(blk.mat(l, l), rhs))
    return np.concatenate(alpha)


def monolithic_solve(blk: Blocks, f: np.ndarray, sweeps: int | None = None, solver: str = "auto",
                     rtol: float = 1e-14, beta0: np.ndarray | None = None, return_beta: bool = False):
    """Coefficients from the split D alpha = beta, T' beta = f (eq. (split)).

    Jacobi on T' beta = f (Theorem jacobi): starting from beta_0 (= f by
    default), each sweep solves t_j = A_j^-1 beta^(j) on the levels j < L
    (Theorem cg) and sets beta^(k) = f^(k) - sum_{j<k} B_{k,j} t_j. From any
    start L sweeps are exact (I - T' is nilpotent of order L); from beta_0 = f,
    block k is exact after k-1 sweeps, so L-1 sweeps (the default) suffice.
    Then alpha_l = A_l^-1 beta^(l) on every level.
    """
    solve = _level_solver(solver, rtol)
    L = blk.levels
    S = L - 1 if sweeps is None else sweeps
    fl = split_levels(f, blk.sizes)
    beta = [b.copy() for b in (split_levels(beta0, blk.sizes) if beta0 is not None else fl)]
    history = [np.concatenate(beta)]
    for _ in range(S):
        t = [solve(blk.mat(j, j), beta[j]) for j in range(L - 1)]
        new = [fl[0].copy()]
        for k in range(1, L):
            acc = fl[k].copy()
            for j in range(k):
                acc -= blk.mat(k, j) @ t[j]
            new.append(acc)
        beta = new
        history.append(np.concatenate(beta))
    alpha = np.concatenate([solve(blk.mat(l, l), beta[l]) for l in range(L)])
    if return_beta:
        return alpha, history
    return alpha


def residual(blk: Blocks, alpha: np.ndarray, f: np.ndarray):
    """r = f - T_L alpha (eq. (bigt)).

    Returns (||r||_2 / ||f||_2, per-level ||r_l||_2 / ||f_l||_2, r).
    """
    al = split_levels(alpha, blk.sizes)
    fl = split_levels(f, blk.sizes)
    r = []
    for k in range(blk.levels):
        acc = fl[k].copy()
        for j in range(k + 1):
            acc -= blk.mat(k, j) @ al[j]
        r.append(acc)
    rv = np.concatenate(r)
    per = [float(np.linalg.norm(r[k]) / max(np.linalg.norm(fl[k]), 1e-300)) for k in range(blk.levels)]
    return float(np.linalg.norm(rv) / np.linalg.norm(f)), per, rv


def evaluate(points: np.ndarray, offsets: np.ndarray, delta: np.ndarray, alpha: np.ndarray,
             query: np.ndarray, upto: int | None = None, method: str = "auto") -> np.ndarray:
    """The approximant f_L(y) = sum_l sum_n alpha_n^(l) phi(||y - x_n^(l)|| / delta_l).

    eq. (fapproximation), in the unit-peak kernel scaling. ``upto`` limits the
    sum to the first levels (the partial sums f_l of Section 2).
    """
    L = len(delta) if upto is None else upto
    out = np.zeros(query.shape[0], dtype=np.float64)
    for l in range(L):
        X = points[offsets[l]:offsets[l + 1]]
        a = alpha[offsets[l]:offsets[l + 1]]
        brute = method == "brute" or (method == "auto" and query.shape[0] * X.shape[0] <= BRUTE_FORCE_MAX_PAIRS)
        rp, col, val = (block_bruteforce if brute else block_cells)(query, X, float(delta[l]))
        out += sp.csr_matrix((val, col, rp), shape=(query.shape[0], X.shape[0])) @ a
    return out


def lower_matrix(blk: Blocks) -> sp.csr_matrix:
    """The strictly lower part T_L - D_L as one N x N sparse matrix."""
    off = np.concatenate(([0], np.cumsum(blk.sizes)))
    R, C, V = [], [], []
    for k in range(blk.levels):
        for j in range(k):
            m = blk.mat(k, j).tocoo()
            R.append(m.row + off[k])
            C.append(m.col + off[j])
            V.append(m.data)
    N = int(off[-1])
    if not R:
        return sp.csr_matrix((N, N))
    return sp.csr_matrix((np.concatenate(V), (np.concatenate(R), np.concatenate(C))), shape=(N, N))


def m_norm(blk: Blocks) -> float:
    """Spectral norm of M = I - T'_L (Section 4; Figure 1 plots it).

    M is strictly block lower triangular with blocks -B_{k,j} A_j^-1, so
    M v = -B_low D^-1 v and M^T u = -D^-1 B_low^T u (A_j symmetric). The
    largest singular value comes from ARPACK on that operator pair, with
    sparse LU factors of each A_j.
    """
    L, sizes = blk.levels, blk.sizes
    N = sum(sizes)
    off = np.concatenate(([0], np.cumsum(sizes)))
    lu = [spla.splu(blk.mat(j, j).tocsc()) for j in range(L)]
    low = lower_matrix(blk)
    lowT = low.T.tocsr()

    def dinv(v):
        return np.concatenate([lu[j].solve(np.ascontiguousarray(v[off[j]:off[j + 1]])) for j in range(L)])

    op = spla.LinearOperator((N, N), matvec=lambda v: -(low @ dinv(np.ravel(v))),
                             rmatvec=lambda u: -dinv(lowT @ np.ravel(u)), dtype=np.float64)
    s = spla.svds(op, k=1, return_singular_vectors=False, tol=1e-10, random_state=0)
    return float(s[0])


def kernel_matrix_dense(X: np.ndarray, delta: float) -> np.ndarray:
    """Dense A = (phi(||x_i - x_l|| / delta)) by direct evaluation of all pairs."""
    d2 = None
    for ax in range(X.shape[1]):
        dx = X[:, None, ax] - X[None, :, ax]
        d2 = dx * dx if d2 is None else d2 + dx * dx
    return phi31(np.sqrt(d2) / delta)
