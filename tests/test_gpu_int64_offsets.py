"""GPU structure and solve past 2^31 stored entries: the paper's Table 1
grids at L = 12 (22.4M points, about 5e9 nonzeros; FP32 values and their
remainders only, about 80 GB), so that the strictly-lower CSR's offsets of
the finest level's rows exceed 2^31 and every product, export and residual
takes its 64-bit offset path (the paper notes that 32-bit indices limit its
own implementation, Section 5.3).

* sampled rows of the finest level (stored last: most of their lower-block
  entries sit past entry 2^31, the last row's near entry 5e9), against the
  oracle's brute-force neighbour lists of those rows
  (bit-exact structure, values within one FP32 rounding); candidates are
  preselected by a box of side 2 delta_j around each row point, a filter
  that drops no point closer than delta_j;
* the fast form's solve reaches a 1e-8 FP64 relative residual, checked on
  sampled rows of the finest level by the oracle from the GPU coefficients.
"""
import numpy as np
import pytest

import oracle
import synth
from oracle import multiscale as ms

pytestmark = pytest.mark.gpu

L = 12


def _rows_bruteforce(Xr, Xj, delta):
    """Canonical CSR of the listed row points against Xj (oracle brute force
    over the points of a 2 delta box around each row point)."""
    rps, cols, vals = [0], [], []
    for p in Xr:
        cand = np.nonzero((np.abs(Xj[:, 0] - p[0]) < delta) & (np.abs(Xj[:, 1] - p[1]) < delta))[0]
        rp, col, val = oracle.block_bruteforce(p[None, :], Xj[cand], float(delta))
        cols.append(cand[col])
        vals.append(val)
        rps.append(rps[-1] + len(col))
    return np.array(rps, dtype=np.int64), np.concatenate(cols).astype(np.int32), np.concatenate(vals)


def test_past_two_to_the_31_entries():
    import paper_2503_04914_amd as m

    h = synth.table1_hierarchy(L)
    f = synth.franke(h.points)
    print(f"[int64] Table 1 L={L}: {h.n_total} points", flush=True)
    ctx = m.mskm_create(0)
    hd = m.mskm_hier_create(ctx, h.points, h.offsets, h.delta, fp64=False, fp32=True)
    try:
        st = m.mskm_hier_stats_get(hd)
        print(f"[int64] nnz diag {st['nnz_diag']} lower {st['nnz_lower']}", flush=True)
        assert st["nnz_lower"] > 2 ** 31 + 2 ** 28
        k = L - 1
        n = h.sizes()[k]
        rows = np.concatenate([np.random.default_rng(1200).choice(n, size=40, replace=False), [0, n - 1]])
        Xr = h.level_points(k)[rows]
        for j in (0, 4, 8, 10, 11):
            rp, col, val = m.mskm_export_rows(ctx, hd, k, j, rows)
            orp, ocol, oval = _rows_bruteforce(Xr, h.level_points(j), h.delta[j])
            assert np.array_equal(rp, orp) and np.array_equal(col, ocol), j
            np.testing.assert_allclose(val, oval, rtol=6e-8, atol=0)
        a = np.zeros_like(f)
        o = m.solve_opts(precision=m.MSKM_PREC_FP32, algorithm=m.MSKM_ALG_SEQUENTIAL, cg_rtol=1e-4,
                         target_rel_residual=1e-8, max_refine=12, precond=m.MSKM_PRECOND_BLOCK_JACOBI)
        res = m.mskm_solve(ctx, hd, f, a, o)
        print(f"[int64] solve {res.report['solve_ms']:.1f} ms, rel {res.report['rel_residual']:.2e}", flush=True)
        assert res.status == m.MSKM_OK
        rel = m.mskm_residual(ctx, hd, a, f)[0]
        assert rel <= 1e-8
        # sampled residual rows of the finest level, recomputed by the oracle
        r = f[h.offsets[k] + rows].copy()
        for j in range(L):
            rp, col, val = _rows_bruteforce(Xr, h.level_points(j), h.delta[j])
            B = ms.sp.csr_matrix((val, col, rp), shape=(len(rows), h.sizes()[j]))
            r -= B @ a[h.offsets[j]:h.offsets[j + 1]]
        assert np.sqrt(np.mean(r ** 2)) <= 1e-6 * np.sqrt(np.mean(f ** 2))
    finally:
        m.mskm_hier_destroy(hd)
        m.mskm_destroy(ctx)
