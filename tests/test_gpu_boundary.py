"""GPU tests of the boundary's composite calls, through the C ABI, against
the FP64 oracle:

* mskm_solve_batch: separately created uneven hierarchies with different
  numbers of right-hand sides solved in the same launches; every
  hierarchy's coefficients against the oracle's sequential solve of that
  hierarchy alone (FP64 <= 1e-10, mixed <= 1e-8 relative per level), reports
  against the oracle's residuals; the internal batch object is reused and
  released with its members;
* MSKM_PREFIX_NESTED: a hierarchy given by its largest level only has the
  same blocks (bit-exact) and coefficients as the one given level by level;
* the learned start combined with the block-Jacobi preconditioner: same
  coefficients (CG decides convergence);
* the sliced copy keeps 16-bit column offsets on levels whose size is not a
  multiple of 64 (the Table 1 grids, an uneven batch).
"""
import numpy as np
import pytest

import oracle
import synth
from oracle import learned as ol
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


@pytest.fixture(scope="module")
def members(m, ctx):
    print("[boundary] building separate hierarchies", flush=True)
    hs = synth.batch_hierarchies(count=3, n_min=300, n_max=5000, levels_choice=(1, 3, 4), seed=4100)
    nrhs = [1, 3, 2]
    out = []
    for g, ((h, f0), R) in enumerate(zip(hs, nrhs)):
        F = np.stack([f0] + [synth.fourier_target(4200 + 10 * g + r)(h.points) for r in range(1, R)], axis=1)
        blk = ms.assemble(h.points, h.offsets, h.delta)
        refs = np.stack([oracle.sequential_solve(blk, F[:, r]) for r in range(R)], axis=1)
        hd = m.mskm_hier_create(ctx, h.points, h.offsets, h.delta, fp64=True, fp32=True)
        out.append((h, np.ascontiguousarray(F), blk, refs, hd))
    yield out
    for *_, hd in out:
        m.mskm_hier_destroy(hd)


def _check_member(h, alpha, refs, bar):
    for r in range(refs.shape[1]):
        for l in range(h.levels):
            sl = slice(h.offsets[l], h.offsets[l + 1])
            err = np.linalg.norm(alpha[sl, r] - refs[sl, r]) / np.linalg.norm(refs[sl, r])
            assert err <= bar, (r, l, err)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("alg", ["sequential", "monolithic"])
def test_solve_batch_matches_oracle(m, ctx, members, prec, alg):
    kw = dict(algorithm=m.MSKM_ALG_SEQUENTIAL if alg == "sequential" else m.MSKM_ALG_MONOLITHIC,
              precond=m.MSKM_PRECOND_BLOCK_JACOBI)
    if prec == "fp64":
        kw.update(cg_rtol=1e-14)
        bar = 1e-10
    else:
        kw.update(precision=m.MSKM_PREC_FP32, cg_rtol=1e-5, target_rel_residual=1e-13, max_refine=20)
        bar = 1e-8
    hds = [mb[4] for mb in members]
    Fs = [mb[1] for mb in members]
    As = [np.zeros_like(F) for F in Fs]
    st, reps = m.mskm_solve_batch(ctx, hds, Fs, As, m.solve_opts(**kw), nrhs=[F.shape[1] for F in Fs])
    assert st == m.MSKM_OK, reps
    for (h, F, blk, refs, hd), a, rep in zip(members, As, reps):
        _check_member(h, a, refs, bar)
        assert rep["levels"] == h.levels
        ro = max(oracle.residual(blk, a[:, r], F[:, r])[0] for r in range(F.shape[1]))
        assert rep["rel_residual"] == pytest.approx(ro, rel=1e-6, abs=1e-15)
        assert all(it > 0 for it in rep["cg_iters_last"])


def test_solve_batch_single_rhs_and_device_io(m, ctx, members):
    import torch

    hds = [mb[4] for mb in members]
    Fs = [torch.from_numpy(np.ascontiguousarray(mb[1][:, 0])).cuda() for mb in members]
    As = [torch.zeros_like(F) for F in Fs]
    st, reps = m.mskm_solve_batch(ctx, hds, Fs, As, m.solve_opts(cg_rtol=1e-14, algorithm=m.MSKM_ALG_SEQUENTIAL))
    assert st == m.MSKM_OK
    for (h, F, blk, refs, hd), a in zip(members, As):
        _check_member(h, a.cpu().numpy()[:, None], refs[:, :1], 1e-10)
    # the same as each hierarchy solved on its own
    for (h, F, blk, refs, hd), a in zip(members, As):
        b = np.zeros(h.n_total)
        m.mskm_solve(ctx, hd, np.ascontiguousarray(F[:, 0]), b, m.solve_opts(cg_rtol=1e-14,
                                                                           algorithm=m.MSKM_ALG_SEQUENTIAL))
        assert np.linalg.norm(a.cpu().numpy() - b) <= 1e-10 * np.linalg.norm(b)


def test_solve_batch_cache_follows_members(m, ctx):
    hs = synth.batch_hierarchies(count=2, n_min=500, n_max=2000, levels_choice=(2, 3), seed=4300)
    hds = [m.mskm_hier_create(ctx, h.points, h.offsets, h.delta) for h, _ in hs]
    try:
        fs = [f.copy() for _, f in hs]
        a1 = [np.zeros_like(f) for f in fs]
        a2 = [np.zeros_like(f) for f in fs]
        o = m.solve_opts(cg_rtol=1e-14, algorithm=m.MSKM_ALG_SEQUENTIAL)
        assert m.mskm_solve_batch(ctx, hds, fs, a1, o)[0] == m.MSKM_OK
        assert m.mskm_solve_batch(ctx, hds, fs, a2, o)[0] == m.MSKM_OK  # reuses the batch object
        for x, y in zip(a1, a2):
            assert np.array_equal(x, y)
        # a member is destroyed and a new hierarchy takes part: rebuilt, still right
        m.mskm_hier_destroy(hds[1])
        h, f = hs[1]
        hds[1] = m.mskm_hier_create(ctx, h.points, h.offsets, h.delta)
        a3 = [np.zeros_like(f) for f in fs]
        assert m.mskm_solve_batch(ctx, hds, fs, a3, o)[0] == m.MSKM_OK
        for x, y in zip(a1, a3):
            assert np.linalg.norm(x - y) <= 1e-12 * np.linalg.norm(x)
        # the same hierarchy twice, and a batch object as a member, are rejected
        with pytest.raises(m.MskmError):
            m.mskm_solve_batch(ctx, [hds[0], hds[0]], [fs[0], fs[0]], [a3[0], a3[1]], o)
    finally:
        for hd in hds:
            m.mskm_hier_destroy(hd)


@pytest.mark.parametrize("name", ["halton4", "uniform3d3"])
def test_prefix_nested_equals_level_by_level(m, ctx, name):
    h = synth.halton_hierarchy(4) if name == "halton4" else synth.uniform3d_hierarchy(3, n0=64)
    top = h.level_points(h.levels - 1)
    for l in range(h.levels):  # these hierarchies are prefix-nested
        assert np.array_equal(h.level_points(l), top[: h.sizes()[l]])
    hd = m.mskm_hier_create(ctx, h.points, h.offsets, h.delta)
    hp = m.mskm_hier_create(ctx, np.ascontiguousarray(top), h.offsets, h.delta, prefix_nested=True)
    try:
        for k in range(h.levels):
            for j in range(k + 1):
                a = m.mskm_export_block(ctx, hd, k, j)
                b = m.mskm_export_block(ctx, hp, k, j)
                assert all(np.array_equal(x, y) for x, y in zip(a, b)), (k, j)
        f = synth.fourier_target(1000, dim=h.dim)(h.points)
        x, y = np.zeros_like(f), np.zeros_like(f)
        o = m.solve_opts(cg_rtol=1e-14)
        m.mskm_solve(ctx, hd, f, x, o)
        m.mskm_solve(ctx, hp, f, y, o)
        assert np.array_equal(x, y)
        ref = oracle.sequential_solve(ms.assemble(h.points, h.offsets, h.delta), f)
        assert np.linalg.norm(y - ref) <= 1e-10 * np.linalg.norm(ref)
    finally:
        m.mskm_hier_destroy(hd)
        m.mskm_hier_destroy(hp)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_learned_start_with_block_jacobi(m, ctx, prec):
    h = synth.halton_hierarchy(4)
    f = synth.fourier_target(6001)(h.points)
    ref = oracle.sequential_solve(ms.assemble(h.points, h.offsets, h.delta), f)
    rng = np.random.default_rng(5)
    F = ol.feature_count(2)
    net = m.mskm_mlp_load(ctx, m.mlp_blob(2, (rng.standard_normal((64, F)) * 0.05).astype(np.float32),
                                          np.zeros(64, np.float32), (rng.standard_normal(64) * 0.05).astype(np.float32),
                                          0.0))
    hd = m.mskm_hier_create(ctx, h.points, h.offsets, h.delta, fp64=True, fp32=True)
    try:
        kw = dict(algorithm=m.MSKM_ALG_SEQUENTIAL, precond=m.MSKM_PRECOND_BLOCK_JACOBI,
                  warm_start=m.MSKM_START_LEARNED, mlp=net.value)
        if prec == "fp64":
            kw.update(cg_rtol=1e-14)
            bar = 1e-10
        else:
            kw.update(precision=m.MSKM_PREC_FP32, cg_rtol=1e-5, target_rel_residual=1e-13, max_refine=20)
            bar = 1e-8
        a = np.zeros_like(f)
        res = m.mskm_solve(ctx, hd, f, a, m.solve_opts(**kw))
        assert res.status == m.MSKM_OK
        assert np.linalg.norm(a - ref) <= bar * np.linalg.norm(ref)
        # the learned start needs a network, and takes a single right-hand side
        with pytest.raises(m.MskmError):
            m.mskm_solve(ctx, hd, f, a, m.solve_opts(warm_start=m.MSKM_START_LEARNED))
        F2 = np.ascontiguousarray(np.stack([f, f], axis=1))
        with pytest.raises(m.MskmError):
            m.mskm_solve(ctx, hd, F2, np.zeros_like(F2), m.solve_opts(**kw), nrhs=2)
    finally:
        m.mskm_hier_destroy(hd)
        m.mskm_mlp_destroy(net)


def test_sliced_copy_keeps_16bit_columns_on_ragged_levels(m, ctx):
    h = synth.table1_hierarchy(9)  # top level (2^9+1)^2 = 263,169 rows: not a multiple of 64
    assert h.sizes()[-1] % 64 != 0 and h.n_total > 65536
    hd = m.mskm_hier_create(ctx, h.points, h.offsets, h.delta, fp64=False, fp32=True)
    try:
        assert m.mskm_hier_stats_get(hd)["sell_col16"] == 1
    finally:
        m.mskm_hier_destroy(hd)
    hs = synth.batch_hierarchies(count=6, n_min=20_000, n_max=60_000, levels_choice=(3, 4), seed=4400)
    assert any(n % 64 for hh, _ in hs for n in hh.sizes())
    hb = m.mskm_hier_create_batch(ctx, [(hh.points, hh.offsets, hh.delta) for hh, _ in hs], fp64=False, fp32=True)
    try:
        assert m.mskm_hier_stats_get(hb)["n_total"] > 65536
        assert m.mskm_hier_stats_get(hb)["sell_col16"] == 1
    finally:
        m.mskm_hier_destroy(hb)
