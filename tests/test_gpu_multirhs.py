"""GPU parity of the many-right-hand-side path: all right-hand sides of one
solve share the launches (CG per level and right-hand side, multi-vector
SpMM). Each right-hand side must match the oracle's solution for it alone.
Widths cover R < 64 (several rows per wave), R = 64 and ragged R > 64.
"""
import numpy as np
import pytest

import oracle
import synth
from oracle import multiscale as ms

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import paper_2503_04914_amd as m

    ctx = m.mskm_create(0)
    cache = {}

    def get(name):
        if name not in cache:
            if name == "halton5":
                h = synth.halton_hierarchy(5)
            elif name == "uniform3d3":
                h = synth.uniform3d_hierarchy(3, n0=64)
            else:
                h = synth.grid_hierarchy()
            blk = ms.assemble(h.points, h.offsets, h.delta)
            hd = m.mskm_hier_create(ctx, h.points, h.offsets, h.delta, fp64=True, fp32=True)
            cache[name] = (h, blk, hd)
        return cache[name]

    yield m, ctx, get
    for _, _, hd in cache.values():
        m.mskm_hier_destroy(hd)
    m.mskm_destroy(ctx)


def _targets(h, R, seed0):
    return np.ascontiguousarray(np.stack([synth.fourier_target(seed0 + r, h.dim)(h.points) for r in range(R)], axis=1))


@pytest.mark.parametrize("name,R", [("halton5", 3), ("grid4", 64), ("uniform3d3", 130)])
@pytest.mark.parametrize("alg", ["sequential", "monolithic"])
def test_multi_rhs_fp64(env, name, R, alg):
    m, ctx, get = env
    h, blk, hd = get(name)
    F = _targets(h, R, 3000)
    A = np.zeros_like(F)
    o = m.solve_opts(cg_rtol=1e-14, algorithm=m.MSKM_ALG_SEQUENTIAL if alg == "sequential" else m.MSKM_ALG_MONOLITHIC)
    res = m.mskm_solve(ctx, hd, F, A, o, nrhs=R)
    assert res.status == m.MSKM_OK, res.report
    rels = m.mskm_residual(ctx, hd, A, F, nrhs=R)
    for r in list(range(min(R, 4))) + [R - 1]:
        ref = oracle.sequential_solve(blk, F[:, r])
        for l in range(h.levels):
            sl = slice(h.offsets[l], h.offsets[l + 1])
            err = np.linalg.norm(A[sl, r] - ref[sl]) / np.linalg.norm(ref[sl])
            assert err <= 1e-10, (r, l, err)
        assert rels[r] == pytest.approx(oracle.residual(blk, A[:, r], F[:, r])[0], rel=1e-6, abs=1e-15)


@pytest.mark.parametrize("name,R", [("halton5", 3), ("uniform3d3", 130)])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_multi_rhs_block_jacobi(env, name, R, prec):
    """Many right-hand sides with the cell block-Jacobi preconditioner: each
    matches the oracle, in fewer iterations than plain CG."""
    m, ctx, get = env
    h, blk, hd = get(name)
    F = _targets(h, R, 3200)
    if prec == "fp64":
        o = dict(cg_rtol=1e-14, algorithm=m.MSKM_ALG_SEQUENTIAL)
        bar = 1e-10
    else:
        o = dict(precision=m.MSKM_PREC_FP32, algorithm=m.MSKM_ALG_SEQUENTIAL, cg_rtol=1e-5,
                 target_rel_residual=1e-13, max_refine=20)
        bar = 1e-8
    iters = {}
    for pc in (m.MSKM_PRECOND_NONE, m.MSKM_PRECOND_BLOCK_JACOBI):
        A = np.zeros_like(F)
        res = m.mskm_solve(ctx, hd, F, A, m.solve_opts(precond=pc, **o), nrhs=R)
        assert res.status == m.MSKM_OK, res.report
        iters[pc] = res.report["cg_iters_total"]
    for r in list(range(min(R, 3))) + [R - 1]:
        ref = oracle.sequential_solve(blk, F[:, r])
        for l in range(h.levels):
            sl = slice(h.offsets[l], h.offsets[l + 1])
            err = np.linalg.norm(A[sl, r] - ref[sl]) / np.linalg.norm(ref[sl])
            assert err <= bar, (r, l, err)
    assert iters[m.MSKM_PRECOND_BLOCK_JACOBI] < iters[m.MSKM_PRECOND_NONE], iters


@pytest.mark.parametrize("R", [64, 100, 128, 192])
def test_multi_rhs_mixed_wide_2d(env, R):
    """Mixed precision, block-Jacobi preconditioned, with R >= 64 (several
    right-hand sides per lane) on a 2-D hierarchy; multiples of 64 take the
    one-wave-per-row kernels (lanes own 1, 2 or 3 consecutive right-hand
    sides; R = 192 has the strided lower product and block-Jacobi apply),
    R = 100 the strided forms throughout."""
    m, ctx, get = env
    h, blk, hd = get("halton5")
    F = _targets(h, R, 3400)
    A = np.zeros_like(F)
    o = m.solve_opts(precision=m.MSKM_PREC_FP32, algorithm=m.MSKM_ALG_SEQUENTIAL, cg_rtol=1e-5,
                     target_rel_residual=1e-13, max_refine=20, precond=m.MSKM_PRECOND_BLOCK_JACOBI)
    res = m.mskm_solve(ctx, hd, F, A, o, nrhs=R)
    assert res.status == m.MSKM_OK, res.report
    for r in (0, 1, R // 2, R - 1):
        ref = oracle.sequential_solve(blk, F[:, r])
        for l in range(h.levels):
            sl = slice(h.offsets[l], h.offsets[l + 1])
            err = np.linalg.norm(A[sl, r] - ref[sl]) / np.linalg.norm(ref[sl])
            assert err <= 1e-8, (r, l, err)


def test_multi_rhs_mixed_matches_single(env):
    m, ctx, get = env
    h, blk, hd = get("halton5")
    R = 5
    F = _targets(h, R, 3100)
    A = np.zeros_like(F)
    o = m.solve_opts(precision=m.MSKM_PREC_FP32, algorithm=m.MSKM_ALG_SEQUENTIAL, cg_rtol=1e-5,
                     target_rel_residual=1e-13, max_refine=20)
    res = m.mskm_solve(ctx, hd, F, A, o, nrhs=R)
    assert res.status == m.MSKM_OK, res.report
    for r in range(R):
        ref = oracle.sequential_solve(blk, F[:, r])
        assert np.linalg.norm(A[:, r] - ref) / np.linalg.norm(ref) <= 1e-8
        single = np.zeros(h.n_total)
        m.mskm_solve(ctx, hd, np.ascontiguousarray(F[:, r]), single, o)
        assert np.linalg.norm(A[:, r] - single) / np.linalg.norm(single) <= 1e-8


def test_batch_and_multi_rhs_together(env):
    m, ctx, _ = env
    hs = synth.batch_hierarchies(count=3, n_min=500, n_max=3000, levels_choice=(2, 3))
    hd = m.mskm_hier_create_batch(ctx, [(h.points, h.offsets, h.delta) for h, _ in hs])
    try:
        R = 2
        F = np.concatenate([_targets(h, R, 5000 + 10 * g) for g, (h, _) in enumerate(hs)])
        A = np.zeros_like(F)
        res = m.mskm_solve(ctx, hd, F, A, m.solve_opts(cg_rtol=1e-14, algorithm=m.MSKM_ALG_SEQUENTIAL), nrhs=R)
        assert res.status == m.MSKM_OK
        base = 0
        for g, (h, _) in enumerate(hs):
            blk = ms.assemble(h.points, h.offsets, h.delta)
            for r in range(R):
                ref = oracle.sequential_solve(blk, F[base:base + h.n_total, r])
                got = A[base:base + h.n_total, r]
                assert np.linalg.norm(got - ref) / np.linalg.norm(ref) <= 1e-10
            base += h.n_total
        rels = m.mskm_residual(ctx, hd, A, F, nrhs=R)
        assert rels.shape == (R * len(hs),) and rels.max() < 1e-12
    finally:
        m.mskm_hier_destroy(hd)


@pytest.mark.parametrize("name,R", [("halton5", 3), ("uniform3d3", 70)])
def test_multi_rhs_fp32_only_hierarchy(env, name, R):
    """A hierarchy that stores only FP32 values (and their FP32 remainders,
    which its FP64 residuals use): mixed many-right-hand-side solves still
    reach the oracle's coefficients, and the residuals match the oracle's."""
    m, ctx, get = env
    h, blk, _ = get(name)
    hd = m.mskm_hier_create(ctx, h.points, h.offsets, h.delta, fp64=False, fp32=True)
    try:
        F = _targets(h, R, 3400)
        A = np.zeros_like(F)
        o = m.solve_opts(precision=m.MSKM_PREC_FP32, algorithm=m.MSKM_ALG_SEQUENTIAL, cg_rtol=1e-5,
                         target_rel_residual=1e-13, max_refine=20, precond=m.MSKM_PRECOND_BLOCK_JACOBI)
        res = m.mskm_solve(ctx, hd, F, A, o, nrhs=R)
        assert res.status == m.MSKM_OK, res.report
        rels = m.mskm_residual(ctx, hd, A, F, nrhs=R)
        for r in (0, R - 1):
            ref = oracle.sequential_solve(blk, F[:, r])
            for l in range(h.levels):
                sl = slice(h.offsets[l], h.offsets[l + 1])
                err = np.linalg.norm(A[sl, r] - ref[sl]) / np.linalg.norm(ref[sl])
                assert err <= 1e-8, (r, l, err)
            assert rels[r] == pytest.approx(oracle.residual(blk, A[:, r], F[:, r])[0], rel=1e-6, abs=1e-15)
    finally:
        m.mskm_hier_destroy(hd)


def test_many_rhs_product_timing(env):
    """The timing entry point of the many-right-hand-side CG product runs the
    solver's kernel on one level and rejects widths outside [2, 512]."""
    m, ctx, get = env
    h, blk, hd = get("halton5")
    for R in (2, 64, 256):
        ms = m.mskm_mr_product_time(ctx, hd, h.levels - 1, R, repeats=3)
        assert 0.0 < ms < 1e3
    for bad in (1, 513):
        with pytest.raises(m.MskmError):
            m.mskm_mr_product_time(ctx, hd, 0, bad)
    with pytest.raises(m.MskmError):
        m.mskm_mr_product_time(ctx, hd, h.levels, 64)


@pytest.mark.parametrize("name", ["halton5", "uniform3d3"])
@pytest.mark.parametrize("chunk", [64, 128])
def test_multi_rhs_product_layouts(env, name, chunk):
    """Each CG-product layout of the many-rhs solve, pinned (slices of 64 or
    128 right-hand sides): each right-hand side matches the oracle."""
    m, ctx, get = env
    h, blk, hd = get(name)
    R = 128
    m.mskm_set_mr_chunk(hd, R, m.MSKM_PREC_FP32, chunk)
    F = _targets(h, R, 3600 + chunk)
    A = np.zeros_like(F)
    o = m.solve_opts(precision=m.MSKM_PREC_FP32, algorithm=m.MSKM_ALG_SEQUENTIAL, cg_rtol=1e-5,
                     target_rel_residual=1e-13, max_refine=20, precond=m.MSKM_PRECOND_BLOCK_JACOBI)
    res = m.mskm_solve(ctx, hd, F, A, o, nrhs=R)
    assert res.status == m.MSKM_OK, res.report
    for r in (0, R // 3, R - 1):
        ref = oracle.sequential_solve(blk, F[:, r])
        for l in range(h.levels):
            sl = slice(h.offsets[l], h.offsets[l + 1])
            err = np.linalg.norm(A[sl, r] - ref[sl]) / np.linalg.norm(ref[sl])
            assert err <= 1e-8, (chunk, r, l, err)


def test_multi_rhs_layout_pin_rejects_bad_values(env):
    m, ctx, get = env
    h, blk, hd = get("halton5")
    for args in ((100, m.MSKM_PREC_FP32, 64), (128, m.MSKM_PREC_FP32, 256), (128, m.MSKM_PREC_FP32, 32),
                 (128, m.MSKM_PREC_FP32, 1), (128, m.MSKM_PREC_FP64, 96), (1024, m.MSKM_PREC_FP32, 64)):
        with pytest.raises(m.MskmError):
            m.mskm_set_mr_chunk(hd, *args)
