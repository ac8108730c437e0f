"""GPU parity at the benchmark's full size (2-D Halton, 8 levels, 1,398,080
points, ~389M nonzeros), in the benchmark's launch configuration.

The oracle cannot assemble and solve this hierarchy in seconds, so the
checks use outputs it can compute one by one and properties that hold at any
size:

* structure: sampled rows of every block B_{7,j} and B_{3,j} against the
  oracle's brute-force neighbour lists of those rows (bit-exact);
* block-triangular locality: levels 0..5 of the full solve depend only on
  levels 0..5, so they must equal the oracle's exact solve of the 6-level
  prefix hierarchy (eq. (mas) / block forward substitution);
* residual: sampled rows of f - T alpha recomputed by the oracle from the
  GPU coefficients, and the GPU's own FP64 relative residual <= 1e-8;
* approximant at sampled query points against the oracle's brute-force sum.
"""
import numpy as np
import pytest

import oracle
import synth
from oracle import multiscale as ms
from oracle.wendland import phi31

pytestmark = pytest.mark.gpu

LEVELS = 8
PREFIX = 6


@pytest.fixture(scope="module")
def setup():
    import paper_2503_04914_amd as m

    print("[fullsize] building the 8-level Halton hierarchy", flush=True)
    h = synth.halton_hierarchy(LEVELS)
    f = synth.fourier_target(1000)(h.points)
    ctx = m.mskm_create(0)
    hd = m.mskm_hier_create(ctx, h.points, h.offsets, h.delta, fp64=True, fp32=True)
    m.mskm_autotune(ctx, hd, repeats=2)
    hp = synth.halton_hierarchy(PREFIX)
    blk = ms.assemble(hp.points, hp.offsets, hp.delta)
    a_prefix = oracle.sequential_solve(blk, f[: hp.n_total])
    yield m, ctx, h, f, hd, hp, a_prefix
    m.mskm_hier_destroy(hd)
    m.mskm_destroy(ctx)


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("k", [7, 3])
def test_sampled_rows_bit_exact(setup, k):
    m, ctx, h, f, hd, *_ = setup
    n = h.sizes()[k]
    rows = np.random.default_rng(100 + k).choice(n, size=min(n, 400), replace=False)
    rows = np.concatenate([rows, [0, n - 1]])  # plus the first and last row
    Xr = h.level_points(k)[rows]
    for j in range(k + 1):
        rp, col, val = m.mskm_export_rows(ctx, hd, k, j, rows)
        orp, ocol, oval = oracle.block_bruteforce(Xr, h.level_points(j), float(h.delta[j]))
        assert np.array_equal(rp, orp), (k, j)
        assert np.array_equal(col, ocol), (k, j)
        np.testing.assert_allclose(val, oval, rtol=1e-15, atol=0)


@pytest.mark.parametrize("form", ["plain_fp64", "mixed_sequential", "fast_form"])
def test_full_solve(setup, form):
    """fast_form: the timed configuration of the benchmark (a hierarchy that
    stores FP32 values and their remainders only, 16-bit sliced products,
    block-Jacobi preconditioned sequential mixed solve, one workgroup per
    small level), run to a tighter target so that the coefficients can be
    compared with the oracle's."""
    m, ctx, h, f, hd, hp, a_prefix = setup
    alpha = np.zeros_like(f)
    hs = hd
    if form == "plain_fp64":
        o = m.solve_opts(cg_rtol=1e-13, max_cg_iters=20000)
        bar = 1e-10
    elif form == "mixed_sequential":
        o = m.solve_opts(precision=m.MSKM_PREC_FP32, algorithm=m.MSKM_ALG_SEQUENTIAL, cg_rtol=1e-4,
                         target_rel_residual=1e-12, max_refine=12)
        bar = 1e-8
    else:
        hs = m.mskm_hier_create(ctx, h.points, h.offsets, h.delta, fp64=False, fp32=True)
        assert m.mskm_hier_stats_get(hs)["sell_col16"] == 1
        o = m.solve_opts(precision=m.MSKM_PREC_FP32, algorithm=m.MSKM_ALG_SEQUENTIAL, cg_rtol=1e-4,
                         target_rel_residual=1e-12, max_refine=12, precond=m.MSKM_PRECOND_BLOCK_JACOBI)
        bar = 1e-8
    print(f"[fullsize] solve {form}", flush=True)
    try:
        res = m.mskm_solve(ctx, hs, f, alpha, o)
        assert res.status == m.MSKM_OK, res.report
        rel = m.mskm_residual(ctx, hs, alpha, f)[0]
    finally:
        if hs is not hd:
            m.mskm_hier_destroy(hs)
    assert rel <= 1e-8
    # the residual of the FP32-only hierarchy (FP32 values + remainders) against the FP64 one
    rel64 = m.mskm_residual(ctx, hd, alpha, f)[0]
    assert rel64 <= 1e-8 and abs(rel64 - rel) <= 1e-11, (rel64, rel)
    # levels 0..PREFIX-1 against the oracle's exact prefix solve
    for l in range(PREFIX):
        sl = slice(hp.offsets[l], hp.offsets[l + 1])
        assert _rel(alpha[sl], a_prefix[sl]) <= bar, (l, _rel(alpha[sl], a_prefix[sl]))
    # sampled rows of the residual, recomputed by the oracle from the GPU alpha
    top = LEVELS - 1
    rows = np.random.default_rng(7).choice(h.sizes()[top], size=300, replace=False)
    Xr = h.level_points(top)[rows]
    r = f[h.offsets[top] + rows].copy()
    for j in range(LEVELS):
        rp, col, val = oracle.block_bruteforce(Xr, h.level_points(j), float(h.delta[j]))
        B = ms.sp.csr_matrix((val, col, rp), shape=(len(rows), h.sizes()[j]))
        r -= B @ alpha[h.offsets[j]:h.offsets[j + 1]]
    assert np.sqrt(np.mean(r ** 2)) <= 1e-7 * np.sqrt(np.mean(f ** 2))
    # approximant at sampled query points
    q = np.random.default_rng(8).random((200, 2))
    out = np.zeros(len(q))
    m.mskm_evaluate(ctx, hd, alpha, q, out)
    ref = np.zeros(len(q))
    for j in range(LEVELS):
        X = h.level_points(j)
        d2 = ((q[:, None, 0] - X[None, :, 0]) ** 2 + (q[:, None, 1] - X[None, :, 1]) ** 2) if j < 6 else None
        if d2 is not None:
            ref += (phi31(np.sqrt(d2) / h.delta[j]) * (d2 < h.delta[j] ** 2)) @ alpha[h.offsets[j]:h.offsets[j + 1]]
        else:
            rp, col, val = oracle.block_bruteforce(q, X, float(h.delta[j]))
            ref += ms.sp.csr_matrix((val, col, rp), shape=(len(q), len(X))) @ alpha[h.offsets[j]:h.offsets[j + 1]]
    assert np.abs(out - ref).max() <= 1e-12 * np.abs(ref).max()
