"""GPU parity: the HIP library (through the C ABI) against the FP64 oracle.

Bars:
* neighbour lists / CSR structure: bit-exact (rowptr and columns of every
  block B_{k,j} in canonical order);
* block values: <= 4 ulp-ish (1e-15 relative; the same FP64 formula on both sides);
* FP64 SpMV: <= 1e-14 relative; FP64 solve: coefficients <= 1e-10 relative
  per level against the oracle's exact sequential solve;
* mixed path (FP32 values inside, FP64 refinement): <= 1e-8 relative;
* approximant values at query points: same bars, relative to max |f_L|.
Sizes span many 256-row tiles and ragged tails (levels of 81..32768 points).
"""
import numpy as np
import pytest

import oracle
import synth
from oracle import multiscale as ms

pytestmark = pytest.mark.gpu

CASES = ["grid4", "halton5", "uniform3d3", "table1_5"]


def _case(name):
    if name == "grid4":
        h = synth.grid_hierarchy()
        return h, synth.gauss_sine(h.points)
    if name == "halton5":
        h = synth.halton_hierarchy(5)
        return h, synth.fourier_target(1000)(h.points)
    if name == "uniform3d3":
        h = synth.uniform3d_hierarchy(3)
        return h, synth.fourier_target(2001, 3)(h.points)
    if name == "table1_5":
        h = synth.table1_hierarchy(5)
        return h, synth.franke(h.points)
    raise KeyError(name)


@pytest.fixture(scope="module")
def mod():
    import paper_2503_04914_amd as m

    return m


@pytest.fixture(scope="module")
def ctx(mod):
    c = mod.mskm_create(0)
    yield c
    for entry in _cache.values():  # hierarchies go before their context
        mod.mskm_hier_destroy(entry[3])
    _cache.clear()
    mod.mskm_destroy(c)


_cache = {}


def _setup(mod, ctx, name):
    if name not in _cache:
        print(f"[parity] case {name}", flush=True)
        h, f = _case(name)
        blk = ms.assemble(h.points, h.offsets, h.delta)
        hd = mod.mskm_hier_create(ctx, h.points, h.offsets, h.delta, fp64=True, fp32=True)
        a_ref = oracle.sequential_solve(blk, f)
        _cache[name] = (h, f, blk, hd, a_ref)
    return _cache[name]


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


@pytest.mark.parametrize("name", CASES)
def test_structure_bit_exact(mod, ctx, name):
    h, f, blk, hd, _ = _setup(mod, ctx, name)
    st = mod.mskm_hier_stats_get(hd)
    assert st["nnz_diag"] == sum(blk.nnz(l, l) for l in range(h.levels))
    assert st["nnz_lower"] == sum(blk.nnz(k, j) for k in range(h.levels) for j in range(k))
    for k in range(h.levels):
        for j in range(k + 1):
            rp, col, val = mod.mskm_export_block(ctx, hd, k, j)
            orp, ocol, oval = blk.csr[(k, j)]
            assert np.array_equal(rp, orp), (k, j)
            assert np.array_equal(col, ocol), (k, j)
            np.testing.assert_allclose(val, oval, rtol=1e-15, atol=0)


@pytest.mark.parametrize("name", CASES)
def test_spmv_fp64_and_fp32(mod, ctx, name):
    h, f, blk, hd, _ = _setup(mod, ctx, name)
    x = np.random.default_rng(3).standard_normal(h.n_total)
    D = [blk.mat(l, l) for l in range(h.levels)]
    off = h.offsets
    yd = np.concatenate([D[l] @ x[off[l]:off[l + 1]] for l in range(h.levels)])
    yl = ms.lower_matrix(blk) @ x
    for op, ref in ((mod.MSKM_OP_DIAG, yd), (mod.MSKM_OP_LOWER, yl), (mod.MSKM_OP_FULL, yd + yl)):
        y = np.zeros_like(x)
        mod.mskm_apply(ctx, hd, op, x, y, prec=mod.MSKM_PREC_FP64)
        assert _rel(y, ref) <= 1e-14, op
        y32 = np.zeros_like(x)
        mod.mskm_apply(ctx, hd, op, x, y32, prec=mod.MSKM_PREC_FP32)
        assert _rel(y32, ref) <= 1e-5, op  # FP32 values, FP32 accumulation


@pytest.mark.parametrize("name", ["halton5", "uniform3d3"])
def test_every_spmv_variant(mod, ctx, name):
    """Each of the autotuner's SpMV variants, pinned explicitly, against the
    oracle's products (the variants differ only in summation order)."""
    h, f, blk, hd, _ = _setup(mod, ctx, name)
    x = np.random.default_rng(4).standard_normal(h.n_total)
    D = [blk.mat(l, l) for l in range(h.levels)]
    off = h.offsets
    yd = np.concatenate([D[l] @ x[off[l]:off[l + 1]] for l in range(h.levels)])
    yl = ms.lower_matrix(blk) @ x
    saved = {(op, pr): mod.mskm_spmv_width(hd, op, pr) for op in range(3) for pr in range(2)}
    try:
        for code in mod.TUNE_VARIANTS:
            for op, ref in ((mod.MSKM_OP_DIAG, yd), (mod.MSKM_OP_LOWER, yl), (mod.MSKM_OP_FULL, yd + yl)):
                if code in (mod.SELL_CODE, mod.SELL32_CODE) and op != mod.MSKM_OP_DIAG:
                    with pytest.raises(mod.MskmError):  # the sliced copy holds the diagonal blocks only
                        mod.mskm_set_spmv_width(hd, op, 0, code)
                    continue
                for pr, tol in ((mod.MSKM_PREC_FP64, 1e-14), (mod.MSKM_PREC_FP32, 1e-5)):
                    mod.mskm_set_spmv_width(hd, op, pr, code)
                    y = np.zeros_like(x)
                    mod.mskm_apply(ctx, hd, op, x, y, prec=pr)
                    assert _rel(y, ref) <= tol, (code, op, pr)
        for bad in (0, 3, 65, 1005, 4004, -4):
            with pytest.raises(mod.MskmError):
                mod.mskm_set_spmv_width(hd, 0, 0, bad)
    finally:
        for (op, pr), w in saved.items():
            mod.mskm_set_spmv_width(hd, op, pr, w)


def test_sell_column_offsets(mod, ctx):
    """The sliced copy stores 16-bit column offsets when every 64-row slice's
    columns span at most 65536 rows, and its 16-bit product equals the 32-bit
    one bit for bit (same entries, same order). A lattice of 8 planes of
    320 x 320 points whose cell layers hold over 65536 rows each has slices
    coupled across layers: there the copy keeps 32-bit columns only and code
    4064 runs the 32-bit kernel."""
    h, f, blk, hd, _ = _setup(mod, ctx, "halton5")
    assert mod.mskm_hier_stats_get(hd)["sell_col16"] == 1
    g = (np.arange(320) + 0.5) / 320
    X, Y, Z = np.meshgrid(g, g, (np.arange(8) + 0.5) / 320, indexing="ij")
    pts = np.ascontiguousarray(np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1))
    wide = mod.mskm_hier_create(ctx, pts, np.array([0, len(pts)], dtype=np.int64), np.array([1.5 / 320]),
                                fp64=True, fp32=True)
    try:
        assert mod.mskm_hier_stats_get(wide)["sell_col16"] == 0
        for hh, n in ((hd, h.n_total), (wide, len(pts))):
            x = np.random.default_rng(6).standard_normal(n)
            out = {}
            for code in (mod.SELL_CODE, mod.SELL32_CODE):
                for pr in (mod.MSKM_PREC_FP64, mod.MSKM_PREC_FP32):
                    mod.mskm_set_spmv_width(hh, mod.MSKM_OP_DIAG, pr, code)
                    y = np.zeros_like(x)
                    mod.mskm_apply(ctx, hh, mod.MSKM_OP_DIAG, x, y, prec=pr)
                    out[code, pr] = y
            for pr in (mod.MSKM_PREC_FP64, mod.MSKM_PREC_FP32):
                assert np.array_equal(out[mod.SELL_CODE, pr], out[mod.SELL32_CODE, pr])
                y8 = np.zeros_like(x)
                mod.mskm_set_spmv_width(hh, mod.MSKM_OP_DIAG, pr, 1008)
                mod.mskm_apply(ctx, hh, mod.MSKM_OP_DIAG, x, y8, prec=pr)
                assert _rel(out[mod.SELL_CODE, pr], y8) <= (1e-14 if pr == mod.MSKM_PREC_FP64 else 1e-5)
    finally:
        mod.mskm_hier_destroy(wide)


@pytest.mark.parametrize("name", ["halton5", "uniform3d3"])
@pytest.mark.parametrize("code", [3008, 3016, 4064, 4032])
def test_solve_with_variant(mod, ctx, name, code):
    """Solves whose CG products run on the recomputed-value or the sliced
    (SELL) variant, and whose lower-block products recompute the values,
    still match the oracle (FP64 and mixed)."""
    h, f, blk, hd, a_ref = _setup(mod, ctx, name)
    saved = {(op, pr): mod.mskm_spmv_width(hd, op, pr) for op in range(3) for pr in range(2)}
    try:
        for op in range(3):
            for pr in range(2):
                mod.mskm_set_spmv_width(hd, op, pr, code if op == 0 or code < mod.SELL32_CODE else 3016)
        for prec, bar in ((mod.MSKM_PREC_FP64, 1e-10), (mod.MSKM_PREC_FP32, 1e-8)):
            alpha = np.zeros_like(f)
            o = mod.solve_opts(precision=prec, cg_rtol=1e-14 if prec == mod.MSKM_PREC_FP64 else 1e-5,
                               target_rel_residual=1e-13, max_refine=20, max_cg_iters=20000)
            res = mod.mskm_solve(ctx, hd, f, alpha, o)
            assert res.status == mod.MSKM_OK, res.report
            for l in range(h.levels):
                sl = slice(h.offsets[l], h.offsets[l + 1])
                assert _rel(alpha[sl], a_ref[sl]) <= bar, (prec, l, _rel(alpha[sl], a_ref[sl]))
    finally:
        for (op, pr), w in saved.items():
            mod.mskm_set_spmv_width(hd, op, pr, w)


@pytest.mark.parametrize("name", CASES)
@pytest.mark.parametrize("alg", ["monolithic", "sequential", "monolithic_warm"])
def test_solve_fp64(mod, ctx, name, alg):
    h, f, blk, hd, a_ref = _setup(mod, ctx, name)
    alpha = np.zeros_like(f)
    o = mod.solve_opts(cg_rtol=1e-14, max_cg_iters=20000,
                       algorithm=mod.MSKM_ALG_SEQUENTIAL if alg == "sequential" else mod.MSKM_ALG_MONOLITHIC,
                       warm_start=1 if alg == "monolithic_warm" else 0)
    res = mod.mskm_solve(ctx, hd, f, alpha, o)
    assert res.status == mod.MSKM_OK
    for l in range(h.levels):
        sl = slice(h.offsets[l], h.offsets[l + 1])
        assert _rel(alpha[sl], a_ref[sl]) <= 1e-10, (l, _rel(alpha[sl], a_ref[sl]))
    rel_o, _, _ = oracle.residual(blk, alpha, f)
    assert rel_o <= 1e-12
    assert res.report["rel_residual"] == pytest.approx(rel_o, rel=1e-3, abs=1e-15)


@pytest.mark.parametrize("name", ["halton5", "uniform3d3"])
def test_solve_mixed_refined(mod, ctx, name):
    h, f, blk, hd, a_ref = _setup(mod, ctx, name)
    alpha = np.zeros_like(f)
    o = mod.solve_opts(precision=mod.MSKM_PREC_FP32, cg_rtol=1e-6, target_rel_residual=1e-13, max_refine=20)
    res = mod.mskm_solve(ctx, hd, f, alpha, o)
    assert res.status == mod.MSKM_OK, res.report
    assert res.report["refine_steps"] >= 2
    for l in range(h.levels):
        sl = slice(h.offsets[l], h.offsets[l + 1])
        assert _rel(alpha[sl], a_ref[sl]) <= 1e-8, (l, _rel(alpha[sl], a_ref[sl]))
    assert oracle.residual(blk, alpha, f)[0] <= 1e-12


@pytest.mark.parametrize("name", CASES)
@pytest.mark.parametrize("alg", ["monolithic", "sequential"])
@pytest.mark.parametrize("diag", ["csr", "sell"])
def test_solve_block_jacobi(mod, ctx, name, alg, diag):
    """CG preconditioned by the cell block-Jacobi inverses reaches the
    oracle's coefficients (FP64 <= 1e-10; mixed <= 1e-8 after refinement),
    with the CSR or the sliced product."""
    h, f, blk, hd, a_ref = _setup(mod, ctx, name)
    saved = mod.mskm_spmv_width(hd, mod.MSKM_OP_DIAG, 0), mod.mskm_spmv_width(hd, mod.MSKM_OP_DIAG, 1)
    code = mod.SELL_CODE if diag == "sell" else 1008
    try:
        for pr in range(2):
            mod.mskm_set_spmv_width(hd, mod.MSKM_OP_DIAG, pr, code)
        algo = mod.MSKM_ALG_SEQUENTIAL if alg == "sequential" else mod.MSKM_ALG_MONOLITHIC
        for prec, bar in ((mod.MSKM_PREC_FP64, 1e-10), (mod.MSKM_PREC_FP32, 1e-8)):
            alpha = np.zeros_like(f)
            o = mod.solve_opts(precision=prec, algorithm=algo, precond=mod.MSKM_PRECOND_BLOCK_JACOBI,
                               cg_rtol=1e-14 if prec == mod.MSKM_PREC_FP64 else 1e-5,
                               target_rel_residual=1e-13, max_refine=20, max_cg_iters=20000)
            res = mod.mskm_solve(ctx, hd, f, alpha, o)
            assert res.status == mod.MSKM_OK, res.report
            for l in range(h.levels):
                sl = slice(h.offsets[l], h.offsets[l + 1])
                assert _rel(alpha[sl], a_ref[sl]) <= bar, (prec, l, _rel(alpha[sl], a_ref[sl]))
    finally:
        mod.mskm_set_spmv_width(hd, mod.MSKM_OP_DIAG, 0, saved[0])
        mod.mskm_set_spmv_width(hd, mod.MSKM_OP_DIAG, 1, saved[1])


def test_level_size_boundaries(mod, ctx):
    """Level sizes at the edges of the launch shapes: 64 / 257 / 1024 rows
    (solved by one workgroup each, with the three product layouts), 1025 rows
    (the first chunked size), 2017 = 2 x 993 + 31 rows (the last window of
    preconditioner blocks merged into the one before) and 2018 rows (not
    merged). Plain and preconditioned, FP64 and mixed, both algorithms. The
    near-duplicate level pairs make some levels' right-hand sides tiny and
    their coefficients sensitive, so every solve is checked by the oracle's
    monolithic residual of the GPU coefficients (and the coefficients are
    checked against the oracle's loosely)."""
    h = synth.halton_hierarchy(sizes=[64, 257, 1024, 1025, 2017, 2018, 3000])
    f = synth.fourier_target(77)(h.points)
    blk = ms.assemble(h.points, h.offsets, h.delta)
    a_ref = oracle.sequential_solve(blk, f)
    hd = mod.mskm_hier_create(ctx, h.points, h.offsets, h.delta, fp64=True, fp32=True)
    try:
        for pc in (mod.MSKM_PRECOND_NONE, mod.MSKM_PRECOND_BLOCK_JACOBI):
            for algo in (mod.MSKM_ALG_SEQUENTIAL, mod.MSKM_ALG_MONOLITHIC):
                for prec, bar in ((mod.MSKM_PREC_FP64, 1e-11), (mod.MSKM_PREC_FP32, 1e-12)):
                    alpha = np.zeros_like(f)
                    o = mod.solve_opts(precision=prec, algorithm=algo, precond=pc,
                                       cg_rtol=1e-14 if prec == mod.MSKM_PREC_FP64 else 1e-5,
                                       target_rel_residual=1e-13, max_refine=20, max_cg_iters=20000)
                    res = mod.mskm_solve(ctx, hd, f, alpha, o)
                    assert res.status == mod.MSKM_OK, (pc, algo, prec, res.report)
                    rel = oracle.residual(blk, alpha, f)[0]
                    assert rel <= bar, (pc, algo, prec, rel)
                    for l in range(h.levels):
                        sl = slice(h.offsets[l], h.offsets[l + 1])
                        err = _rel(alpha[sl], a_ref[sl])
                        assert err <= 1e-5, (pc, algo, prec, l, err)
                    assert all(0 < it < 20000 for it in res.report["cg_iters_last"][:h.levels])
    finally:
        mod.mskm_hier_destroy(hd)


def test_block_jacobi_needs_fewer_iterations(mod, ctx):
    """On the 3-D case the preconditioned solves take clearly fewer CG
    iterations than the plain ones to the same tolerance."""
    h, f, blk, hd, a_ref = _setup(mod, ctx, "uniform3d3")
    its = {}
    for pc in (mod.MSKM_PRECOND_NONE, mod.MSKM_PRECOND_BLOCK_JACOBI):
        alpha = np.zeros_like(f)
        res = mod.mskm_solve(ctx, hd, f, alpha, mod.solve_opts(algorithm=mod.MSKM_ALG_SEQUENTIAL, cg_rtol=1e-10,
                                                               precond=pc))
        assert res.status == mod.MSKM_OK
        its[pc] = res.report["cg_iters_total"]
    assert its[mod.MSKM_PRECOND_BLOCK_JACOBI] < 0.7 * its[mod.MSKM_PRECOND_NONE], its


def test_several_rhs_reject_learned_warm_start(mod, ctx):
    h, f, blk, hd, _ = _setup(mod, ctx, "grid4")
    F = np.ascontiguousarray(np.stack([f, 2 * f], axis=1))
    A = np.zeros_like(F)
    with pytest.raises(mod.MskmError):  # no network given either: rejected before anything runs
        mod.mskm_solve(ctx, hd, F, A, mod.solve_opts(precond=mod.MSKM_PRECOND_LEARNED), nrhs=2)


@pytest.mark.parametrize("name", ["grid4", "halton5", "uniform3d3"])
def test_fp32_only_hierarchy(mod, ctx, name):
    """A hierarchy that stores only FP32 values: its FP64 residual takes each
    entry as the FP32 value plus its stored FP32 remainder, and the mixed
    solve still reaches the oracle's coefficients."""
    h, f, blk, _, a_ref = _setup(mod, ctx, name)
    hd = mod.mskm_hier_create(ctx, h.points, h.offsets, h.delta, fp64=False, fp32=True)
    try:
        a = a_ref + 1e-6 * np.random.default_rng(21).standard_normal(a_ref.shape)
        rel = mod.mskm_residual(ctx, hd, a, f)[0]
        assert rel == pytest.approx(oracle.residual(blk, a, f)[0], rel=1e-9)
        assert mod.mskm_residual(ctx, hd, np.zeros_like(f), f)[0] == pytest.approx(1.0, rel=1e-14)
        alpha = np.zeros_like(f)
        res = mod.mskm_solve(ctx, hd, f, alpha, mod.solve_opts(precision=mod.MSKM_PREC_FP32, cg_rtol=1e-6,
                                                               target_rel_residual=1e-13, max_refine=20))
        assert res.status == mod.MSKM_OK, res.report
        for l in range(h.levels):
            sl = slice(h.offsets[l], h.offsets[l + 1])
            assert _rel(alpha[sl], a_ref[sl]) <= 1e-8, (l, _rel(alpha[sl], a_ref[sl]))
        with pytest.raises(mod.MskmError):  # FP64 solves need the FP64 values
            mod.mskm_solve(ctx, hd, f, alpha, mod.solve_opts(precision=mod.MSKM_PREC_FP64))
    finally:
        mod.mskm_hier_destroy(hd)


@pytest.mark.parametrize("name", CASES)
def test_residual_and_evaluate(mod, ctx, name):
    h, f, blk, hd, a_ref = _setup(mod, ctx, name)
    rng = np.random.default_rng(17)
    a = a_ref + 1e-6 * rng.standard_normal(a_ref.shape)  # not the solution: nonzero residual
    rel = mod.mskm_residual(ctx, hd, a, f)[0]
    assert rel == pytest.approx(oracle.residual(blk, a, f)[0], rel=1e-10)
    q = rng.random((3000, h.dim)) * 1.2 - 0.1  # includes points outside the hull
    q = np.concatenate([q, h.level_points(h.levels - 1)[:500]])
    out = np.zeros(len(q))
    mod.mskm_evaluate(ctx, hd, a_ref, q, out)
    ref = oracle.evaluate(h.points, h.offsets, h.delta, a_ref, q)
    assert np.abs(out - ref).max() <= 1e-12 * np.abs(ref).max()


def test_bad_arguments_fail_cleanly(mod, ctx):
    with pytest.raises(mod.MskmError) as e:
        mod.mskm_hier_create(ctx, np.zeros((4, 2)), np.array([0, 4]), np.array([-1.0]))
    assert e.value.status == mod.MSKM_EINVAL
    pts = np.zeros((4, 2))
    pts[2, 1] = np.nan
    with pytest.raises(mod.MskmError):
        mod.mskm_hier_create(ctx, pts, np.array([0, 4]), np.array([0.5]))
    h, f, blk, hd, _ = _setup(mod, ctx, "grid4")
    with pytest.raises(mod.MskmError):
        mod.mskm_export_block(ctx, hd, 1, 2)  # column level above row level
    # iteration cap hit: warning status with outputs written
    alpha = np.zeros_like(f)
    res = mod.mskm_solve(ctx, hd, f, alpha, mod.solve_opts(max_cg_iters=2))
    assert res.status == mod.MSKM_ENOCONV
    assert np.all(np.isfinite(alpha))


def test_degenerate_hierarchies(mod, ctx):
    # single level, single point; empty middle level; coincident coarse/fine points
    for pts, off, dl in [
        (np.array([[0.3, 0.4]]), [0, 1], [0.1]),
        (np.array([[0.1, 0.1], [0.9, 0.9], [0.5, 0.5], [0.2, 0.7]]), [0, 2, 2, 4], [0.8, 0.5, 0.6]),
        (np.random.default_rng(1).random((700, 2)), [0, 100, 100, 700], [0.3, 0.2, 0.08]),
    ]:
        pts = np.ascontiguousarray(pts)
        off = np.array(off, dtype=np.int64)
        dl = np.array(dl)
        blk = ms.assemble(pts, off, dl)
        f = np.sin(pts[:, 0] * 3) + pts[:, 1]
        hd = mod.mskm_hier_create(ctx, pts, off, dl)
        try:
            for k in range(len(dl)):
                for j in range(k + 1):
                    rp, col, _ = mod.mskm_export_block(ctx, hd, k, j)
                    assert np.array_equal(rp, blk.csr[(k, j)][0]) and np.array_equal(col, blk.csr[(k, j)][1])
            alpha = np.zeros_like(f)
            mod.mskm_solve(ctx, hd, f, alpha, mod.solve_opts(cg_rtol=1e-14))
            ref = oracle.sequential_solve(blk, f, solver="cholesky")
            assert _rel(alpha, ref) <= 1e-10
        finally:
            mod.mskm_hier_destroy(hd)


def test_deterministic_repeat(mod, ctx):
    h, f, blk, hd, _ = _setup(mod, ctx, "halton5")
    a1, a2 = np.zeros_like(f), np.zeros_like(f)
    o = mod.solve_opts(cg_rtol=1e-12)
    mod.mskm_solve(ctx, hd, f, a1, o)
    mod.mskm_solve(ctx, hd, f, a2, o)
    assert np.array_equal(a1, a2)


@pytest.mark.parametrize("check_every", [1, 3, 8, 64])
def test_result_independent_of_poll_interval(mod, ctx, check_every):
    # levels stop at different iterations while the host keeps launching
    # iterations for the slower ones: a stopped level must stay stopped
    h, f, blk, hd, a_ref = _setup(mod, ctx, "halton5")
    for alg in (mod.MSKM_ALG_MONOLITHIC, mod.MSKM_ALG_SEQUENTIAL):
        for rt in (1e-8, 1e-11):
            alpha = np.zeros_like(f)
            res = mod.mskm_solve(ctx, hd, f, alpha, mod.solve_opts(cg_rtol=rt, algorithm=alg, check_every=check_every))
            assert res.status == mod.MSKM_OK
            assert res.report["rel_residual"] < 1e3 * rt
            assert max(res.report["cg_iters_last"]) < 2000


def test_autotune_keeps_results(mod, ctx):
    h, f, blk, hd, a_ref = _setup(mod, ctx, "uniform3d3")
    x = np.random.default_rng(5).standard_normal(h.n_total)
    y0 = np.zeros_like(x)
    mod.mskm_apply(ctx, hd, mod.MSKM_OP_FULL, x, y0)
    t = mod.mskm_autotune(ctx, hd, repeats=2)
    assert t.shape == (3, 2, len(mod.TUNE_VARIANTS))
    sell = [mod.TUNE_VARIANTS.index(mod.SELL_CODE), mod.TUNE_VARIANTS.index(mod.SELL32_CODE)]
    assert np.all(np.delete(t, sell, axis=2) > 0) and np.all(t[0][:, sell] > 0) and np.all(t[1:][:, :, sell] == 0)
    for op in range(3):
        for pr in range(2):
            assert mod.mskm_spmv_width(hd, op, pr) in mod.TUNE_VARIANTS
    y1 = np.zeros_like(x)
    mod.mskm_apply(ctx, hd, mod.MSKM_OP_FULL, x, y1)
    assert _rel(y1, y0) <= 1e-14
    # a hierarchy of the same shape created on this context inherits the widths
    hd2 = mod.mskm_hier_create(ctx, h.points, h.offsets, h.delta, fp64=True, fp32=True)
    try:
        for op in range(3):
            assert mod.mskm_spmv_width(hd2, op, 0) == mod.mskm_spmv_width(hd, op, 0)
    finally:
        mod.mskm_hier_destroy(hd2)
