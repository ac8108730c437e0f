"""GPU parity of the learned warm start.

* kNN-16 lists: bit-exact against the oracle's brute force;
* network inference (BF16 MFMA, FP32 accumulation) against the oracle's
  forward pass with the same BF16 rounding (FP64 accumulation);
* training: one Adam step on fixed samples against the oracle's FP64
  gradient and Adam step, parameter by parameter, within the FP32 error
  bound of the gradient; a 100-step loss trajectory against the oracle's
  FP64 training run; determinism; the loss falls on pairs from the solver;
  save/load round trip;
* solves with the warm start, and with the network as a preconditioner inside
  flexible CG: coefficients still match the oracle (the true residual decides
  convergence), FP64 <= 1e-10, mixed <= 1e-8; with a zero network flexible CG is
  block-Jacobi PCG (same coefficients, about the same iterations).
"""
import numpy as np
import pytest

import oracle
import synth
from oracle import learned as ol
from oracle import multiscale as ms

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import paper_2503_04914_amd as m

    ctx = m.mskm_create(0)
    h = synth.halton_hierarchy(5)
    hd = m.mskm_hier_create(ctx, h.points, h.offsets, h.delta, fp64=True, fp32=True)
    h3 = synth.uniform3d_hierarchy(3, n0=64)
    hd3 = m.mskm_hier_create(ctx, h3.points, h3.offsets, h3.delta)
    yield m, ctx, (h, hd), (h3, hd3)
    m.mskm_hier_destroy(hd)
    m.mskm_hier_destroy(hd3)
    m.mskm_destroy(ctx)


def test_knn_bit_exact(env):
    m, ctx, (h, hd), (h3, hd3) = env
    for hh, hdd in ((h, hd), (h3, hd3)):
        for l in range(hh.levels):
            got = m.mskm_knn_export(ctx, hdd, l)
            ref = ol.knn16(hh.level_points(l))
            assert np.array_equal(got, ref), l


def _random_net(dim, seed):
    rng = np.random.default_rng(seed)
    F = ol.feature_count(dim)
    W1 = (rng.standard_normal((64, F)) * 0.3).astype(np.float32)
    b1 = (rng.standard_normal(64) * 0.1).astype(np.float32)
    w2 = (rng.standard_normal(64) * 0.3).astype(np.float32)
    return W1, b1, w2, np.float32(0.02)


@pytest.mark.parametrize("which", ["2d", "3d"])
def test_inference_matches_reference(env, which):
    m, ctx, (h, hd), (h3, hd3) = env
    hh, hdd = (h, hd) if which == "2d" else (h3, hd3)
    W1, b1, w2, b2 = _random_net(hh.dim, 11)
    net = m.mskm_mlp_load(ctx, m.mlp_blob(hh.dim, W1, b1, w2, float(b2)))
    try:
        b = np.random.default_rng(3).standard_normal(hh.n_total)
        b[hh.offsets[1]:hh.offsets[1] + 5] = 0.0
        x0 = np.zeros_like(b)
        m.mskm_mlp_predict(ctx, hdd, net, b, x0)
        for l in range(hh.levels):
            X = hh.level_points(l)
            bl = b[hh.offsets[l]:hh.offsets[l + 1]]
            feat, s = ol.features(X, bl, ol.knn16(X), float(hh.delta[l]))
            ref = ol.forward(W1, b1, w2, b2, feat, s)
            got = x0[hh.offsets[l]:hh.offsets[l + 1]]
            assert np.linalg.norm(got - ref) <= 2e-6 * np.linalg.norm(ref), l
        # save / load round trip gives the same predictions
        net2 = m.mskm_mlp_load(ctx, m.mskm_mlp_save(net))
        x1 = np.zeros_like(b)
        m.mskm_mlp_predict(ctx, hdd, net2, b, x1)
        assert np.array_equal(x0, x1)
        m.mskm_mlp_destroy(net2)
    finally:
        m.mskm_mlp_destroy(net)


def test_train_and_solve(env):
    m, ctx, (h, hd), _ = env
    Ftr = np.ascontiguousarray(np.stack([synth.fourier_target(5000 + r)(h.points) for r in range(8)], axis=1))
    net, log = m.mskm_mlp_train(ctx, hd, Ftr, nrhs=8, samples=20000, steps=1500, lr=1e-3, seed=1, cg_rtol=1e-10)
    try:
        assert len(log) == 30 and np.all(np.isfinite(log)) and np.all(log > 0)  # every entry written
        # mini-batch losses are noisy and the local features explain only part of
        # the target's variance: ask for a clear drop of the late average
        assert np.mean(log[-5:]) < 0.75 * log[0]
        # held-out target: the warm start lowers the level residuals, the solve stays exact
        f = synth.fourier_target(6000)(h.points)
        blk = ms.assemble(h.points, h.offsets, h.delta)
        ref = oracle.sequential_solve(blk, f)
        a = np.zeros_like(f)
        res = m.mskm_solve(ctx, hd, f, a, m.solve_opts(cg_rtol=1e-14, algorithm=m.MSKM_ALG_SEQUENTIAL,
                                                        precond=m.MSKM_PRECOND_LEARNED, mlp=net.value))
        assert res.status == m.MSKM_OK
        assert np.linalg.norm(a - ref) / np.linalg.norm(ref) <= 1e-10
        assert res.report["warm_fallbacks"] <= h.levels
        # the same for the monolithic form and the mixed path
        a2 = np.zeros_like(f)
        res2 = m.mskm_solve(ctx, hd, f, a2, m.solve_opts(precision=m.MSKM_PREC_FP32, cg_rtol=1e-5,
                                                          target_rel_residual=1e-13, max_refine=20,
                                                          precond=m.MSKM_PRECOND_LEARNED, mlp=net.value))
        assert res2.status == m.MSKM_OK
        assert np.linalg.norm(a2 - ref) / np.linalg.norm(ref) <= 1e-8
        # the network as a preconditioner at every iteration (flexible CG), FP64 and mixed
        for prec, kw, bar in ((m.MSKM_PREC_FP64, dict(cg_rtol=1e-14), 1e-10),
                              (m.MSKM_PREC_FP32, dict(cg_rtol=1e-5, target_rel_residual=1e-13, max_refine=20), 1e-8)):
            a3 = np.zeros_like(f)
            res3 = m.mskm_solve(ctx, hd, f, a3, m.solve_opts(precision=prec, algorithm=m.MSKM_ALG_SEQUENTIAL,
                                                              precond=m.MSKM_PRECOND_FLEX_LEARNED, mlp=net.value,
                                                              **kw))
            assert res3.status == m.MSKM_OK, res3.report
            assert np.linalg.norm(a3 - ref) / np.linalg.norm(ref) <= bar, prec
        # the flexible form takes the sequential algorithm and one right-hand side only
        with pytest.raises(m.MskmError):
            m.mskm_solve(ctx, hd, f, a3, m.solve_opts(precond=m.MSKM_PRECOND_FLEX_LEARNED, mlp=net.value))
    finally:
        m.mskm_mlp_destroy(net)


def test_flexible_cg_with_zero_network_is_block_jacobi_pcg(env):
    """A network whose output layer is zero gives z = M_BJ^-1 r at every
    iteration, a fixed SPD preconditioner: flexible CG then takes the
    iterates of block-Jacobi PCG (to rounding), so it meets the oracle's
    coefficients and needs about the same iterations per level (the two
    recurrences round differently, and a window of slow progress restarts
    the flexible form's direction once)."""
    m, ctx, (h, hd), _ = env
    F = ol.feature_count(h.dim)
    rng = np.random.default_rng(77)
    W1 = (rng.standard_normal((64, F)) * 0.3).astype(np.float32)
    b1 = (rng.standard_normal(64) * 0.1).astype(np.float32)
    net = m.mskm_mlp_load(ctx, m.mlp_blob(h.dim, W1, b1, np.zeros(64, np.float32), 0.0))
    try:
        f = synth.fourier_target(6001)(h.points)
        ref = oracle.sequential_solve(ms.assemble(h.points, h.offsets, h.delta), f)
        common = dict(cg_rtol=1e-12, algorithm=m.MSKM_ALG_SEQUENTIAL)
        a_bj = np.zeros_like(f)
        r_bj = m.mskm_solve(ctx, hd, f, a_bj, m.solve_opts(precond=m.MSKM_PRECOND_BLOCK_JACOBI, **common))
        a_fx = np.zeros_like(f)
        r_fx = m.mskm_solve(ctx, hd, f, a_fx, m.solve_opts(precond=m.MSKM_PRECOND_FLEX_LEARNED, mlp=net.value,
                                                            **common))
        assert r_bj.status == m.MSKM_OK and r_fx.status == m.MSKM_OK, r_fx.report
        for a in (a_bj, a_fx):
            assert np.linalg.norm(a - ref) / np.linalg.norm(ref) <= 1e-10
        it_bj, it_fx = r_bj.report["cg_iters_last"], r_fx.report["cg_iters_last"]
        print("[flex-zero] iterations per level", it_bj, it_fx, flush=True)
        for l in range(h.levels):
            assert abs(it_fx[l] - it_bj[l]) <= max(3, it_bj[l] // 10), (l, it_bj, it_fx)
    finally:
        m.mskm_mlp_destroy(net)


def _fit_case(dim, seed, ns):
    """Random features and a target from a teacher network of the same shape
    (so the loss can fall far), a random student."""
    rng = np.random.default_rng(seed)
    F = ol.feature_count(dim)
    X = rng.standard_normal((ns, F)).astype(np.float32)
    T1 = (rng.standard_normal((64, F)) * 0.2).astype(np.float32)
    t1 = (rng.standard_normal(64) * 0.1).astype(np.float32)
    t2 = (rng.standard_normal(64) * 0.2).astype(np.float32)
    y = ol.forward(T1, t1, t2, 0.05, X, np.ones(ns)).astype(np.float32)
    W1 = (rng.standard_normal((64, F)) * 0.1).astype(np.float32)
    b1 = (rng.standard_normal(64) * 0.05).astype(np.float32)
    w2 = (rng.standard_normal(64) * 0.1).astype(np.float32)
    return X, y, (W1, b1, w2, np.float32(0.01))


@pytest.mark.parametrize("dim", [2, 3])
def test_fit_one_step_matches_oracle(env, dim):
    m, ctx, _, _ = env
    X, y, (W1, b1, w2, b2) = _fit_case(dim, 20 + dim, 300)
    lr = 1e-3
    net = m.mskm_mlp_load(ctx, m.mlp_blob(dim, W1, b1, w2, float(b2)))
    try:
        log = m.mskm_mlp_fit(ctx, net, X, y, steps=1, lr=lr)
        got = m.mlp_params(net).astype(np.float64)
    finally:
        m.mskm_mlp_destroy(net)
    rows = ol.batch_rows(0, len(y))
    loss, g = ol.loss_and_grads(W1, b1, w2, b2, X[rows], y[rows])
    g = ol.pack(*g)
    p0 = ol.pack(W1, b1, w2, b2)
    want, _, _ = ol.adam_update(p0, g, np.zeros_like(p0), np.zeros_like(p0), 1, lr)
    # first Adam step: -lr g / (|g| + eps); an FP32 gradient within E of g
    # moves it by at most lr min(2, 2 E / (|g| + eps)); plus the FP32
    # rounding of the Adam arithmetic and of the updated parameter
    E = ol.grad_error_bound(W1, b1, w2, b2, X[rows], y[rows])
    ulp = np.spacing(np.maximum(np.abs(p0), np.abs(want)).astype(np.float32)).astype(np.float64)
    tol = lr * np.minimum(2.0, 2.0 * E / (np.abs(g) + 1e-8)) + 1e-5 * lr + 2.0 * ulp
    bad = np.flatnonzero(np.abs(got - want) > tol)
    assert bad.size == 0, (bad[:10], got[bad[:10]], want[bad[:10]], tol[bad[:10]])
    assert np.mean(np.abs(got - p0) > 0.5 * lr) > 0.9  # the step is a real one
    assert log[0] == pytest.approx(loss, rel=1e-5)


def test_fit_trajectory_matches_oracle(env):
    m, ctx, _, _ = env
    X, y, (W1, b1, w2, b2) = _fit_case(2, 31, 2000)
    steps, lr = 100, 1e-3
    net = m.mskm_mlp_load(ctx, m.mlp_blob(2, W1, b1, w2, float(b2)))
    net2 = m.mskm_mlp_load(ctx, m.mlp_blob(2, W1, b1, w2, float(b2)))
    try:
        log = m.mskm_mlp_fit(ctx, net, X, y, steps=steps, lr=lr)
        log2 = m.mskm_mlp_fit(ctx, net2, X, y, steps=steps, lr=lr)
        assert np.array_equal(log, log2) and np.array_equal(m.mlp_params(net), m.mlp_params(net2))  # deterministic
        got = m.mlp_params(net).astype(np.float64)
    finally:
        m.mskm_mlp_destroy(net)
        m.mskm_mlp_destroy(net2)
    want, ref_log = ol.train(ol.pack(W1, b1, w2, b2), X, y, steps, lr)
    # FP32 and FP64 runs separate slowly: an FP32 emulation of this loop
    # (numpy, another summation order) stays within 1.1e-4 of the FP64 losses
    # and within 6e-7 in median parameter over these 100 steps
    assert np.all(np.abs(log - ref_log) <= 1e-3 * ref_log), np.max(np.abs(log - ref_log) / ref_log)
    assert np.mean(ref_log[-10:]) < 0.5 * np.mean(ref_log[:10])
    assert np.median(np.abs(got - want)) < 1e-2 * lr
