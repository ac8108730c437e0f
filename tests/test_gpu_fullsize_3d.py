"""GPU parity on the full 3-D mixed-precision workload (5 prefix-nested
levels of a seeded uniform stream, 512 .. 2,097,152 points, 2,396,672 in
total, ~614M nonzeros), in the benchmark's launch configuration (a
hierarchy that stores FP32 values and their remainders only, block-Jacobi
preconditioned sequential mixed solve).

Checks the oracle can make at this size:

* structure and values of sampled rows of every block B_{4,j} and B_{2,j}
  against the oracle's brute-force neighbour lists (bit-exact structure,
  values within one FP32 rounding: the hierarchy stores FP32 values);
* block-triangular locality: levels 0..2 of the full solve equal the
  oracle's exact solve of the 3-level prefix hierarchy (1e-8 after
  refinement to 1e-12);
* sampled rows of f - T alpha recomputed by the oracle from the GPU's
  coefficients, and the GPU's FP64 relative residual <= 1e-8;
* the approximant at sampled query points against the oracle's sum.
"""
import numpy as np
import pytest

import oracle
import synth
from oracle import multiscale as ms
from oracle.wendland import phi31

pytestmark = pytest.mark.gpu

LEVELS = 5
PREFIX = 3


@pytest.fixture(scope="module")
def setup():
    import paper_2503_04914_amd as m

    print("[fullsize3d] building the 5-level 3-D hierarchy", flush=True)
    h = synth.uniform3d_hierarchy(LEVELS)
    f = synth.fourier_target(2001, dim=3)(h.points)
    ctx = m.mskm_create(0)
    hd = m.mskm_hier_create(ctx, h.points, h.offsets, h.delta, fp64=False, fp32=True)
    m.mskm_autotune(ctx, hd, repeats=2)
    hp = synth.uniform3d_hierarchy(PREFIX)
    assert np.array_equal(hp.points, h.points[: hp.n_total])
    blk = ms.assemble(hp.points, hp.offsets, hp.delta)
    a_prefix = oracle.sequential_solve(blk, f[: hp.n_total])
    yield m, ctx, h, f, hd, hp, a_prefix
    m.mskm_hier_destroy(hd)
    m.mskm_destroy(ctx)


@pytest.mark.parametrize("k", [4, 2])
def test_sampled_rows_bit_exact(setup, k):
    m, ctx, h, f, hd, *_ = setup
    n = h.sizes()[k]
    rows = np.random.default_rng(300 + k).choice(n, size=min(n, 300), replace=False)
    rows = np.concatenate([rows, [0, n - 1]])
    Xr = h.level_points(k)[rows]
    for j in range(k + 1):
        rp, col, val = m.mskm_export_rows(ctx, hd, k, j, rows)
        orp, ocol, oval = oracle.block_bruteforce(Xr, h.level_points(j), float(h.delta[j]))
        assert np.array_equal(rp, orp), (k, j)
        assert np.array_equal(col, ocol), (k, j)
        # an FP32-only hierarchy exports its values widened from FP32 (one FP32 rounding)
        np.testing.assert_allclose(val, oval, rtol=6e-8, atol=0)


def test_fast_form_solve(setup):
    m, ctx, h, f, hd, hp, a_prefix = setup
    alpha = np.zeros_like(f)
    o = m.solve_opts(precision=m.MSKM_PREC_FP32, algorithm=m.MSKM_ALG_SEQUENTIAL, cg_rtol=1e-4,
                     target_rel_residual=1e-12, max_refine=16, precond=m.MSKM_PRECOND_BLOCK_JACOBI)
    print("[fullsize3d] fast-form solve", flush=True)
    res = m.mskm_solve(ctx, hd, f, alpha, o)
    assert res.status == m.MSKM_OK, res.report
    rel = m.mskm_residual(ctx, hd, alpha, f)[0]
    assert rel <= 1e-12
    for l in range(PREFIX):
        sl = slice(hp.offsets[l], hp.offsets[l + 1])
        err = np.linalg.norm(alpha[sl] - a_prefix[sl]) / np.linalg.norm(a_prefix[sl])
        print(f"[fullsize3d] level {l}: {err:.2e}", flush=True)
        assert err <= 1e-8, (l, err)
    # sampled residual rows of the finest level, recomputed by the oracle
    top = LEVELS - 1
    rows = np.random.default_rng(9).choice(h.sizes()[top], size=200, replace=False)
    Xr = h.level_points(top)[rows]
    r = f[h.offsets[top] + rows].copy()
    for j in range(LEVELS):
        rp, col, val = oracle.block_bruteforce(Xr, h.level_points(j), float(h.delta[j]))
        B = ms.sp.csr_matrix((val, col, rp), shape=(len(rows), h.sizes()[j]))
        r -= B @ alpha[h.offsets[j]:h.offsets[j + 1]]
    assert np.sqrt(np.mean(r ** 2)) <= 1e-10 * np.sqrt(np.mean(f ** 2))
    # approximant at sampled query points
    q = np.random.default_rng(10).random((100, 3))
    out = np.zeros(len(q))
    m.mskm_evaluate(ctx, hd, alpha, q, out)
    ref = np.zeros(len(q))
    for j in range(LEVELS):
        X = h.level_points(j)
        if j < 3:
            d2 = ((q[:, None, 0] - X[None, :, 0]) ** 2 + (q[:, None, 1] - X[None, :, 1]) ** 2
                  + (q[:, None, 2] - X[None, :, 2]) ** 2)
            ref += (phi31(np.sqrt(d2) / h.delta[j]) * (d2 < h.delta[j] ** 2)) @ alpha[h.offsets[j]:h.offsets[j + 1]]
        else:
            rp, col, val = oracle.block_bruteforce(q, X, float(h.delta[j]))
            ref += ms.sp.csr_matrix((val, col, rp), shape=(len(q), len(X))) @ alpha[h.offsets[j]:h.offsets[j + 1]]
    assert np.abs(out - ref).max() <= 1e-12 * np.abs(ref).max()
