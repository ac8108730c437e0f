"""GPU test of the allocation-free residual (mskm_residual_noalloc), through
the C ABI, against mskm_residual on the same inputs.

The two compute the same sums (eq. (bigt): ||f - T_L alpha|| / ||f|| per
right-hand side and group) in a different order, so they agree to a few
units of rounding: 1e-12 relative. Two calls in a row, the second on a
smaller input (fewer points and right-hand sides), check that the shared
static scratch array carries nothing from one call to the next. Host
pointers are rejected by the library before any launch.
"""
import ctypes as C

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

TOL = 1e-12


@pytest.fixture(scope="module")
def m():
    import paper_2503_04914_amd as mod

    return mod


@pytest.fixture(scope="module")
def ctx(m):
    c = m.mskm_create(0)
    yield c
    m.mskm_destroy(c)


def _case(m, ctx, h, nrhs, seed, fp64, fp32, batch=None):
    import torch

    print(f"[no_alloc] case N={h.n_total if batch is None else sum(x.n_total for x, _ in batch)} "
          f"nrhs={nrhs} fp64={fp64} fp32={fp32} batch={batch is not None}", flush=True)
    if batch is None:
        hd = m.mskm_hier_create(ctx, h.points, h.offsets, h.delta, fp64=fp64, fp32=fp32)
        pts = h.points
    else:
        hd = m.mskm_hier_create_batch(ctx, [(x.points, x.offsets, x.delta) for x, _ in batch], fp64=fp64, fp32=fp32)
        pts = None
    st = m.mskm_hier_stats_get(hd)
    N, G = st["n_total"], st["ngroups"]
    rng = np.random.default_rng(seed)
    if pts is not None:
        F = np.stack([synth.fourier_target(seed + r, dim=pts.shape[1])(pts) for r in range(nrhs)], axis=1)
    else:
        F = rng.standard_normal((N, nrhs))
    F = np.ascontiguousarray(F)
    # a solve gives residuals of about 1e-6; a random alpha gives O(1) ones
    A = np.zeros_like(F)
    if nrhs == 1:
        a1 = np.zeros(N)
        o = m.solve_opts(cg_rtol=1e-6) if fp64 else m.solve_opts(precision=m.MSKM_PREC_FP32, cg_rtol=1e-4,
                                                                  target_rel_residual=1e-6)
        m.mskm_solve(ctx, hd, np.ascontiguousarray(F[:, 0]), a1, o)
        A[:, 0] = a1
    A = np.ascontiguousarray(A + 1e-3 * rng.standard_normal(A.shape))
    want = m.mskm_residual(ctx, hd, A.reshape(-1) if nrhs == 1 else A, F.reshape(-1) if nrhs == 1 else F, nrhs=nrhs)
    dev = torch.device("cuda:0")
    A_d = torch.from_numpy(A).to(dev)
    F_d = torch.from_numpy(F).to(dev)
    out = torch.full((nrhs * G,), -1.0, dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    m.mskm_residual_noalloc(ctx, hd, A_d, F_d, out, nrhs=nrhs)
    # the call only enqueues: wait for the library's stream (all streams)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    assert np.all(np.isfinite(got)) and np.all(got >= 0.0), got
    np.testing.assert_allclose(got, want, rtol=TOL, atol=0.0)
    m.mskm_hier_destroy(hd)
    return got


def test_noalloc_matches_residual_twice_smaller_second(m, ctx):
    big = synth.halton_hierarchy(5)
    small = synth.halton_hierarchy(3)
    _case(m, ctx, big, 3, 7100, fp64=True, fp32=True)
    _case(m, ctx, small, 1, 7200, fp64=True, fp32=True)


def test_noalloc_fp32_only_hierarchy_split_values(m, ctx):
    # FP32-only storage: the residual reads FP32 values plus their remainders
    _case(m, ctx, synth.uniform3d_hierarchy(3), 2, 7300, fp64=False, fp32=True)
    _case(m, ctx, synth.grid_hierarchy(), 1, 7400, fp64=False, fp32=True)


def test_noalloc_batch_per_group(m, ctx):
    hs = synth.batch_hierarchies(count=4, n_min=300, n_max=4000, levels_choice=(1, 2, 3), seed=7500)
    _case(m, ctx, None, 2, 7600, fp64=True, fp32=False, batch=hs)
    _case(m, ctx, None, 1, 7700, fp64=False, fp32=True, batch=hs[:2])


def test_noalloc_rejects_host_memory(m, ctx):
    h = synth.halton_hierarchy(2)
    hd = m.mskm_hier_create(ctx, h.points, h.offsets, h.delta)
    try:
        a = np.zeros(h.n_total)
        out = np.zeros(1)
        p = lambda x: C.c_void_p(x.ctypes.data)  # noqa: E731
        st = m.lib().mskm_residual_noalloc(ctx, hd, p(a), p(a), 1, p(out))
        assert st == m.MSKM_EINVAL, st
        assert "device memory" in m.mskm_last_error()
    finally:
        m.mskm_hier_destroy(hd)
