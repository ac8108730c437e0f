"""The context's block cache: a destroyed hierarchy's device blocks serve
later allocations of the same size, so they come back holding stale data.
Rebuilding a hierarchy on them (same shape, after a different hierarchy
used them too) must give bit-identical structure and coefficients, and
match the oracle."""
import numpy as np
import pytest

import oracle
import synth
from oracle import multiscale as ms

pytestmark = pytest.mark.gpu


def _solve(m, ctx, h, f, fp32_only):
    hd = m.mskm_hier_create(ctx, h.points, h.offsets, h.delta, fp64=not fp32_only, fp32=True,
                            sliced_lower=True)
    try:
        if fp32_only:
            o = m.solve_opts(precision=m.MSKM_PREC_FP32, algorithm=m.MSKM_ALG_SEQUENTIAL, cg_rtol=1e-4,
                             target_rel_residual=1e-12, max_refine=16, precond=m.MSKM_PRECOND_BLOCK_JACOBI)
        else:
            o = m.solve_opts(cg_rtol=1e-14, algorithm=m.MSKM_ALG_SEQUENTIAL)
        a = np.zeros_like(f)
        res = m.mskm_solve(ctx, hd, f, a, o)
        assert res.status == m.MSKM_OK, res.report
        rp, col, val = m.mskm_export_block(ctx, hd, h.levels - 1, h.levels - 2)
        return a, (rp, col, val), m.mskm_residual(ctx, hd, a, f)[0]
    finally:
        m.mskm_hier_destroy(hd)


@pytest.mark.parametrize("fp32_only", [True, False])
def test_rebuild_on_cached_blocks_is_bit_identical(fp32_only):
    import paper_2503_04914_amd as m

    h = synth.halton_hierarchy(5)
    other = synth.uniform3d_hierarchy(3, n0=64)
    f = synth.fourier_target(1200)(h.points)
    fo = synth.fourier_target(1201, dim=3)(other.points)
    ctx = m.mskm_create(0)
    try:
        a1, blk1, rel1 = _solve(m, ctx, h, f, fp32_only)
        _solve(m, ctx, other, fo, fp32_only)  # a different hierarchy takes and returns blocks
        a2, blk2, rel2 = _solve(m, ctx, h, f, fp32_only)  # same shape: the cached blocks again
        a3, blk3, rel3 = _solve(m, ctx, h, f, fp32_only)
        for a, blk, rel in ((a2, blk2, rel2), (a3, blk3, rel3)):
            assert np.array_equal(a, a1)
            assert rel == rel1
            for x, y in zip(blk, blk1):
                assert np.array_equal(x, y)
        ref = oracle.sequential_solve(ms.assemble(h.points, h.offsets, h.delta), f)
        for l in range(h.levels):
            sl = slice(h.offsets[l], h.offsets[l + 1])
            assert np.linalg.norm(a1[sl] - ref[sl]) / np.linalg.norm(ref[sl]) <= (1e-8 if fp32_only else 1e-10)
    finally:
        m.mskm_destroy(ctx)


def test_creation_returns_before_its_last_passes():
    """mskm_hier_create returns once the last assembly passes are queued: a
    destroy right after it (which waits for the stream) and creations in a
    row on the same blocks and pinned staging must leave every later
    hierarchy intact; the assembly time is read at the first statistics
    query."""
    import paper_2503_04914_amd as m

    h = synth.halton_hierarchy(5)
    ctx = m.mskm_create(0)
    try:
        print("[cache] create / destroy at once", flush=True)
        for _ in range(3):  # destroyed while its sliced copies may still be written
            m.mskm_hier_destroy(m.mskm_hier_create(ctx, h.points, h.offsets, h.delta, fp64=True, fp32=True,
                                                   sliced_lower=True))
        hs = [m.mskm_hier_create(ctx, h.points, h.offsets, h.delta, fp64=True, fp32=True, sliced_lower=True)
              for _ in range(3)]
        try:
            st = [m.mskm_hier_stats_get(x) for x in hs]
            assert all(s["assemble_ms"] > 0.0 for s in st)
            assert m.mskm_hier_stats_get(hs[0])["assemble_ms"] == st[0]["assemble_ms"]  # read once, kept
            blks = [m.mskm_export_block(ctx, x, h.levels - 1, h.levels - 3) for x in hs]
            for b in blks[1:]:
                for u, v in zip(b, blks[0]):
                    assert np.array_equal(u, v)
            orp, ocol, oval = ms.assemble(h.points, h.offsets, h.delta).csr[(h.levels - 1, h.levels - 3)]
            rp, col, val = blks[0]
            assert np.array_equal(rp, orp) and np.array_equal(col, ocol)
            np.testing.assert_allclose(val, oval, rtol=1e-15, atol=0)
        finally:
            for x in hs:
                m.mskm_hier_destroy(x)
    finally:
        m.mskm_destroy(ctx)
