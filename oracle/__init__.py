"""Plain FP64 CPU oracle of the monolithic kernel-based multiscale method.

TEST INFRASTRUCTURE ONLY. This package exists to check the GPU library; it is
not part of the product path. Only the test suite, the smoke check of the
package entry file and the CPU-baseline leg of the benchmark may import it.
The GPU library never imports, links or calls anything here, and nothing here
imports the GPU library: the two share no code. Inputs come from the separate
``synth`` generator module, which holds no arithmetic of the method.

What it computes (paper: Lot & Rieger, "Efficiently parallelizable
kernel-based multi-scale algorithm", arXiv 2503.04914):

* ``wendland``   -- the Wendland function phi_{3,1}(r) = (1-r)_+^4 (4r+1)
                    (Section 5) in the unit-peak scaling phi(||x-y||/delta).
* ``neighbours`` -- the compactly supported blocks B_{k,j} (Section 3):
                    entry (i, l) = phi(||x_i^(k) - x_l^(j)||/delta_j) whenever
                    the squared distance is strictly below delta_j^2. Brute
                    force and an independent cell-bucket search.
* ``multiscale`` -- the sequential level-by-level residual algorithm
                    (Section 2, in matrix form eq. (mas)), the monolithic
                    split D alpha = beta, T' beta = f (eq. (split)) solved by
                    Jacobi sweeps with per-level CG (Theorems cg and jacobi),
                    the monolithic residual f - T alpha (eq. (bigt)), the
                    multiscale approximant (eq. (fapproximation)), and the
                    spectral norm of M = I - T' (Section 5.1, Figure 1).
* ``truncation`` -- the thresholded Jacobi of Section 4: the Lagrange blocks
                    X_{kj} = B_{kj} A_j^-1 of M, their truncation X~_{kj}(T)
                    (entries with distance >= T q_j dropped, eq.
                    (perturbedmatrix)), the quantities of Figures 2-3 and the
                    solution of the perturbed split (eq. (perturbed_split)).

Conventions (readings of the paper, listed with reasons in the design notes):

* unit-peak kernel: the delta^-d prefactor of eq. (kernelscaling) is left
  out, so coefficients here equal the paper's divided by delta_l^d; the
  approximant, B A^-1 and ||M|| do not change;
* strict support: a pair is a structural nonzero iff d^2 < delta^2, where
  d^2 = dx*dx + dy*dy (+ dz*dz) is evaluated left to right in FP64 with every
  operation separately rounded (numpy elementwise ops never fuse) and
  delta^2 = delta*delta in FP64;
* Jacobi update beta^(k) <- f^(k) - sum_{j<k} B_kj A_j^-1 beta^(j): the sign
  follows from eq. (mas) with beta = D alpha.

Parity status: every function is pinned by a test in tests/test_oracle_*.py
against closed forms, brute force, dense Cholesky, the paper's invariants or
values printed in the paper; none is "parity unpinned".
"""
from . import wendland, neighbours, multiscale, truncation  # noqa: F401
from .wendland import phi31  # noqa: F401
from .neighbours import block_bruteforce, block_cells, sqdist_pairs  # noqa: F401
from .multiscale import (  # noqa: F401
    Blocks,
    assemble,
    cg,
    cholesky_solve,
    sequential_solve,
    monolithic_solve,
    residual,
    evaluate,
    m_norm,
)
