"""GPU parity of batched solves: several independent uneven hierarchies in
one hierarchy object (levels of equal depth solved in the same launches).

Each hierarchy's blocks and coefficients must equal the oracle's for that
hierarchy alone (structure bit-exact, FP64 coefficients <= 1e-10 relative),
and the per-group residuals must match the oracle's.
"""
import numpy as np
import pytest

import oracle
import synth
from oracle import multiscale as ms

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def batch():
    import paper_2503_04914_amd as m

    print("[batch] building", flush=True)
    hs = synth.batch_hierarchies(count=5, n_min=300, n_max=5000, levels_choice=(1, 3, 4))
    ctx = m.mskm_create(0)
    hd = m.mskm_hier_create_batch(ctx, [(h.points, h.offsets, h.delta) for h, _ in hs], fp64=True, fp32=True)
    refs = []
    for h, f in hs:
        blk = ms.assemble(h.points, h.offsets, h.delta)
        refs.append((blk, oracle.sequential_solve(blk, f)))
    yield m, ctx, hs, hd, refs
    m.mskm_hier_destroy(hd)
    m.mskm_destroy(ctx)


def test_batch_layout_and_structure(batch):
    m, ctx, hs, hd, refs = batch
    st = m.mskm_hier_stats_get(hd)
    assert st["ngroups"] == len(hs)
    assert st["levels"] == sum(h.levels for h, _ in hs)
    base = 0
    seen = {}
    for lev in range(st["levels"]):
        info = m.mskm_hier_level_info(hd, lev)
        seen[(info["group"], info["depth"])] = lev
    for g, (h, _) in enumerate(hs):
        for d in range(h.levels):
            info = m.mskm_hier_level_info(hd, seen[(g, d)])
            assert info["n"] == h.sizes()[d]
            assert info["input_offset"] == base + h.offsets[d]
        base += h.n_total
    for g, (h, _) in enumerate(hs):
        blk = refs[g][0]
        for k in range(h.levels):
            for j in range(k + 1):
                rp, col, val = m.mskm_export_block(ctx, hd, seen[(g, k)], seen[(g, j)])
                assert np.array_equal(rp, blk.csr[(k, j)][0]) and np.array_equal(col, blk.csr[(k, j)][1])
                np.testing.assert_allclose(val, blk.csr[(k, j)][2], rtol=1e-15, atol=0)
    # a block between two different hierarchies does not exist
    with pytest.raises(m.MskmError):
        m.mskm_export_block(ctx, hd, seen[(0, 1)], seen[(1, 0)])


@pytest.mark.parametrize("alg", ["sequential", "monolithic"])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("pc", ["plain", "block_jacobi"])
def test_batch_solve(batch, alg, prec, pc):
    m, ctx, hs, hd, refs = batch
    f = np.concatenate([f for _, f in hs])
    alpha = np.zeros_like(f)
    kw = dict(algorithm=m.MSKM_ALG_SEQUENTIAL if alg == "sequential" else m.MSKM_ALG_MONOLITHIC,
              precond=m.MSKM_PRECOND_BLOCK_JACOBI if pc == "block_jacobi" else m.MSKM_PRECOND_NONE)
    if prec == "fp64":
        kw.update(cg_rtol=1e-14)
        bar = 1e-10
    else:
        kw.update(precision=m.MSKM_PREC_FP32, cg_rtol=1e-5, target_rel_residual=1e-13, max_refine=20)
        bar = 1e-8
    res = m.mskm_solve(ctx, hd, f, alpha, m.solve_opts(**kw))
    assert res.status == m.MSKM_OK, res.report
    rels = m.mskm_residual(ctx, hd, alpha, f)
    base = 0
    for g, (h, fg) in enumerate(hs):
        ag = alpha[base:base + h.n_total]
        blk, ref = refs[g]
        for l in range(h.levels):
            sl = slice(h.offsets[l], h.offsets[l + 1])
            err = np.linalg.norm(ag[sl] - ref[sl]) / np.linalg.norm(ref[sl])
            assert err <= bar, (g, l, err)
        ro = oracle.residual(blk, ag, fg)[0]
        assert rels[g] == pytest.approx(ro, rel=1e-6, abs=1e-15)
        base += h.n_total
