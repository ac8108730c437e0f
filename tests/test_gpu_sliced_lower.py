"""GPU parity of the sliced copy of the strictly-lower blocks
(MSKM_SLICED_LOWER): the products (T - D) x and T x through it, the FP64
residual f - T alpha over it (FP64 values, or FP32 values plus remainders),
and solves that use it, against the oracle.

* products: FP64 within 1e-14 of the oracle's (summation order only), FP32
  within 1e-5 (FP32 values and accumulation), on Halton, Table 1 grids
  (levels of 9..1089 points, ragged last slices) and a batch object;
* every product through the copy equals the CSR product of the same
  precision to rounding (same entries);
* residual: the oracle's FP64 residual of the same alpha within 1e-6
  relative (the residual itself is small; its absolute error is ~1e-16 of
  ||f||);
* solves: the fast form (FP32-only hierarchy, sequential, block-Jacobi,
  refinement to 1e-12) and the plain FP64 form match the oracle's
  coefficients (1e-8 / 1e-10 per level).
"""
import numpy as np
import pytest

import oracle
import synth
from oracle import multiscale as ms

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def m():
    import paper_2503_04914_amd as mod

    return mod


@pytest.fixture(scope="module")
def ctx(m):
    c = m.mskm_create(0)
    yield c
    m.mskm_destroy(c)


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _hier(name):
    return {"halton5": lambda: synth.halton_hierarchy(5), "table1_6": lambda: synth.table1_hierarchy(6),
            "uniform3d3": lambda: synth.uniform3d_hierarchy(3, n0=64)}[name]()


@pytest.mark.parametrize("name", ["halton5", "table1_6", "uniform3d3"])
def test_products_through_the_sliced_copy(m, ctx, name):
    h = _hier(name)
    print(f"[sliced] products {name}", flush=True)
    blk = ms.assemble(h.points, h.offsets, h.delta)
    x = np.random.default_rng(21).standard_normal(h.n_total)
    off = h.offsets
    yd = np.concatenate([blk.mat(l, l) @ x[off[l]:off[l + 1]] for l in range(h.levels)])
    yl = ms.lower_matrix(blk) @ x
    hd = m.mskm_hier_create(ctx, h.points, h.offsets, h.delta, fp64=True, fp32=True, sliced_lower=True)
    try:
        st = m.mskm_hier_stats_get(hd)
        assert st["lower_sliced"] == 1 and st["lower_sliced_entries"] >= st["nnz_lower"]
        for op, ref in ((m.MSKM_OP_LOWER, yl), (m.MSKM_OP_FULL, yd + yl)):
            for pr, tol in ((m.MSKM_PREC_FP64, 1e-14), (m.MSKM_PREC_FP32, 1e-5)):
                m.mskm_set_spmv_width(hd, op, pr, m.SELL_CODE)
                y = np.zeros_like(x)
                m.mskm_apply(ctx, hd, op, x, y, prec=pr)
                assert _rel(y, ref) <= tol, (op, pr, _rel(y, ref))
                m.mskm_set_spmv_width(hd, op, pr, 1016)  # the CSR product of the same entries
                y2 = np.zeros_like(x)
                m.mskm_apply(ctx, hd, op, x, y2, prec=pr)
                assert _rel(y, y2) <= (1e-15 if pr == m.MSKM_PREC_FP64 else 1e-6), (op, pr)
    finally:
        m.mskm_hier_destroy(hd)


@pytest.mark.parametrize("store", ["fp64", "fp32_only"])
def test_residual_through_the_sliced_copy(m, ctx, store):
    h = synth.halton_hierarchy(5)
    f = synth.fourier_target(1000)(h.points)
    blk = ms.assemble(h.points, h.offsets, h.delta)
    a = oracle.sequential_solve(blk, f)
    a = a + 1e-6 * np.random.default_rng(22).standard_normal(a.shape)
    ref = oracle.residual(blk, a, f)[0]
    fp64 = store == "fp64"
    hd = m.mskm_hier_create(ctx, h.points, h.offsets, h.delta, fp64=fp64, fp32=True, sliced_lower=True)
    hc = m.mskm_hier_create(ctx, h.points, h.offsets, h.delta, fp64=fp64, fp32=True)
    try:
        rel = m.mskm_residual(ctx, hd, a, f)[0]
        rel_csr = m.mskm_residual(ctx, hc, a, f)[0]
        assert rel == pytest.approx(ref, rel=1e-6), (rel, ref)
        assert rel == pytest.approx(rel_csr, rel=1e-9), (rel, rel_csr)
    finally:
        m.mskm_hier_destroy(hd)
        m.mskm_hier_destroy(hc)


@pytest.mark.parametrize("form", ["fast", "plain_fp64"])
def test_solves_through_the_sliced_copy(m, ctx, form):
    h = synth.halton_hierarchy(5)
    f = synth.fourier_target(1001)(h.points)
    blk = ms.assemble(h.points, h.offsets, h.delta)
    ref = oracle.sequential_solve(blk, f)
    if form == "fast":
        hd = m.mskm_hier_create(ctx, h.points, h.offsets, h.delta, fp64=False, fp32=True, sliced_lower=True)
        o = m.solve_opts(precision=m.MSKM_PREC_FP32, algorithm=m.MSKM_ALG_SEQUENTIAL, cg_rtol=1e-4,
                         target_rel_residual=1e-12, max_refine=16, precond=m.MSKM_PRECOND_BLOCK_JACOBI)
        bar, pr = 1e-8, m.MSKM_PREC_FP32
    else:
        hd = m.mskm_hier_create(ctx, h.points, h.offsets, h.delta, fp64=True, sliced_lower=True)
        o = m.solve_opts(cg_rtol=1e-14)
        bar, pr = 1e-10, m.MSKM_PREC_FP64
    try:
        m.mskm_set_spmv_width(hd, m.MSKM_OP_LOWER, pr, m.SELL_CODE)  # lower products through the copy
        a = np.zeros_like(f)
        res = m.mskm_solve(ctx, hd, f, a, o)
        assert res.status == m.MSKM_OK, res.report
        for l in range(h.levels):
            sl = slice(h.offsets[l], h.offsets[l + 1])
            assert _rel(a[sl], ref[sl]) <= bar, (l, _rel(a[sl], ref[sl]))
    finally:
        m.mskm_hier_destroy(hd)


def test_batch_object_with_sliced_copy(m, ctx):
    hs = synth.batch_hierarchies(count=4, n_min=300, n_max=5000, levels_choice=(1, 3, 4), seed=4300)
    hb = m.mskm_hier_create_batch(ctx, [(x.points, x.offsets, x.delta) for x, _ in hs], fp64=True, fp32=True,
                                  sliced_lower=True)
    try:
        assert m.mskm_hier_stats_get(hb)["lower_sliced"] == 1
        f = np.concatenate([fb for _, fb in hs])
        m.mskm_set_spmv_width(hb, m.MSKM_OP_LOWER, m.MSKM_PREC_FP64, m.SELL_CODE)
        a = np.zeros_like(f)
        res = m.mskm_solve(ctx, hb, f, a, m.solve_opts(cg_rtol=1e-14, algorithm=m.MSKM_ALG_SEQUENTIAL))
        assert res.status == m.MSKM_OK
        o = 0
        rel = m.mskm_residual(ctx, hb, a, f)
        for g, (x, fx) in enumerate(hs):
            bx = ms.assemble(x.points, x.offsets, x.delta)
            ref = oracle.sequential_solve(bx, fx)
            assert _rel(a[o:o + x.n_total], ref) <= 1e-10, g
            assert rel[g] == pytest.approx(oracle.residual(bx, a[o:o + x.n_total], fx)[0], rel=1e-6, abs=1e-15)
            o += x.n_total
    finally:
        m.mskm_hier_destroy(hb)
