#!/usr/bin/env python3
"""Benchmark: time to 1e-8 relative residual and SpMV bandwidth on one MI355X.

Workload (default): the 2-D Halton hierarchy of 8 levels, level j = first
64*4^j Halton points (bases 2, 3), 1,398,080 points in total, Wendland
phi_{3,1} with delta_j = sqrt(40/pi) * N_j^(-1/2) (about 40 neighbours per
row), target = seeded sum of 32 random Fourier modes. Inputs are generated on
the host and placed in HBM before anything is timed.

One step = one pass of the whole path over that input (each phase timed by
HIP events on the one stream that torch and the library share):
  assembly (cell lists, neighbour search, Wendland blocks into CSR and the
  sliced copies) ->
  solve to ||f - T alpha|| / ||f|| <= 1e-8 with the fast form (FP32 values
  and accumulation inside, FP64 dots and FP64 residual refinement, block
  forward substitution) -> independent FP64 residual check -> evaluation of
  the approximant at 65,536 query points.
After the timed steps: the plain FP64 baseline (Jacobi sweeps on T' with CG
on D, as the paper's algorithms do) to the same 1e-8, the standalone SpMV
kernels (bandwidth against the 8 TB/s HBM peak), and the CPU oracle on a
bounded sample.

Prints one JSON line. ``--gpus`` above 1 is not supported (one GPU).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3  # MI355X vector FP32
# HBM bytes per launch of the roofline kernel (the CG product on the finest
# level): rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE (KiB per dispatch) of
# `bench.py --spmv-only --spmv-op cg --spmv-prec fp32 --spmv-variant 4064`,
# each scaled by the factor that makes the same counter read 1 GiB for the
# 1 GiB streaming copy kernel of those runs. Only valid for that kernel, at
# that launch, on that workload, as built when the counters were taken.
PMC_TRAFFIC = {
    ("halton2d_L8", "k_cg_spmv1_sell<float,float,true>", "level 7"): {
        "fetch_kib": 146135.97, "fetch_scale": 1048576 / 524300.42,
        "write_kib": 4192.75, "write_scale": 1048576 / 1048628.35},
    # `bench.py --spmv-only --spmv-op mr --spmv-prec fp32 --spmv-rhs 256 --spmv-variant 4064`
    ("halton2d_L8", "k_mr_cg_spmm_w<1,float,float> R=256", "level 7"): {
        "fetch_kib": 3607406.5, "fetch_scale": 1048576 / 524300.8,
        "write_kib": 1081344.0, "write_scale": 1048576 / 1048604.3},
}
TARGET = 1e-8
RTOL_LADDER = [3e-3, 1e-3, 3e-4, 1e-4, 3e-5, 1e-5, 1e-6, 1e-7, 1e-8, 1e-9, 1e-10, 1e-11, 1e-12]


def pmc_traffic(key):
    """HBM bytes per launch from the counter runs recorded for `key`, or None."""
    pmc = PMC_TRAFFIC.get(key)
    if pmc is None:
        return None
    return int(pmc["fetch_kib"] * pmc["fetch_scale"] * 1024 + pmc["write_kib"] * pmc["write_scale"] * 1024)


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def build_inputs(levels: int):
    import synth

    h = synth.halton_hierarchy(levels)
    f = synth.fourier_target(1000)(h.points)
    return h, f


def spmv_bytes(nnz: int, n: int, nrowptr: int, sval: int, sx: int, scol: int = 4) -> int:
    """Algorithmic bytes of one SpMV: values + columns (int32, or 16-bit
    offsets in the sliced copy), 8 bytes of row metadata per row and matrix
    (nrowptr), x read once, y written once."""
    return nnz * (sval + scol) + nrowptr * (n + 1) * 8 + n * sx + n * sx


def diag_col_bytes(code: int, stats: dict) -> int:
    """Column bytes per entry of the diagonal-block variant `code`: 2 for the
    sliced copy with 16-bit column offsets, else 4."""
    return 2 if code == 4064 and stats.get("sell_col16") else 4


def spmv_kernel_name(code: int, t: str, col16: bool = False) -> str:
    """Kernel that a SpMV variant code launches (lanes per row + 1000 for
    16-byte loads, + 2000 for non-temporal 16-byte loads, + 3000 for
    recomputed values; 4064 / 4032 the sliced copy, 16-bit / 32-bit columns)."""
    g, kind = code % 1000, code // 1000
    if kind == 0:
        return f"k_spmv<{g},{t}>"
    if kind == 3:
        return f"k_spmv_rec<{g},{t}>"
    if kind == 4:
        return f"k_spmv_sell<{t},{'true' if code == 4064 and col16 else 'false'}>"
    return f"k_spmv_v<{g},{t}{',nontemporal' if kind == 2 else ''}>"


def cg_product_kernel_name(code: int, col16: bool) -> str:
    """Product kernel of the preconditioned CG iteration for diagonal variant
    `code` (FP32 values and vectors): the sliced copy's for 4064 / 4032, else
    the CSR one with `code % 1000` lanes per row."""
    if code in (4064, 4032):
        return f"k_cg_spmv1_sell<float,float,{'true' if code == 4064 and col16 else 'false'}>"
    return f"k_cg_spmv1<{code % 1000},{'true' if code // 1000 else 'false'},float,float>"


def calibrate(m, ctx, hd, f_dev, alpha_dev, base_opts: dict, label: str):
    """Fastest inner CG tolerance of the ladder whose solution verifies the
    target by the independent FP64 residual, with a 5% margin (the timed
    steps' FP32-only hierarchies compute that residual by another kernel,
    rounding differently in the last digits). The time is not monotone in
    the tolerance (a looser one can need another refinement round), so up
    to four passing tolerances are timed, from the loosest."""
    passing = []
    for rt in RTOL_LADDER:
        o = m.solve_opts(cg_rtol=rt, **base_opts)
        m.mskm_solve(ctx, hd, f_dev, alpha_dev, o)  # first call: graphs and preconditioner set up
        res = m.mskm_solve(ctx, hd, f_dev, alpha_dev, o)
        rel = float(m.mskm_residual(ctx, hd, alpha_dev, f_dev)[0])
        log(f"calibrate {label}: rtol={rt:g} rel={rel:.3e} ms={res.report['solve_ms']:.1f} status={res.status}")
        if res.status >= 0 and rel <= 0.95 * TARGET:
            passing.append((res.report["solve_ms"], rt))
            if len(passing) == 4:
                break
    if not passing:
        raise RuntimeError(f"{label}: no tolerance in the ladder reaches {TARGET}")
    return min(passing)[1]


def host_cpu() -> dict:
    """Host facts for the CPU baseline record: logical CPUs and model name."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "cpu_model": model}


def cpu_baseline(levels_sample: int, levels_full: int, nnz_full_diag: list, nnz_full_lower: list):
    """The oracle as it stands, single-threaded, on the first `levels_sample`
    levels of the bench hierarchy: its assembly, then the block forward
    substitution (eq. (mas)) level by level, each level's right-hand side by
    the oracle's sparse products and its solve by the oracle's textbook CG from
    zero, at the loosest tolerance of a short ladder whose result verifies the
    1e-8 relative residual by the oracle's own FP64 residual.

    The full workload's time is estimated from this sample level by level:
    each measured level contributes its measured time; a missing finer level
    takes the last measured level's time per CG iteration per diagonal
    nonzero times its own diagonal nonzeros, times an iteration count grown
    from the last measured level by the measured growth ratio of the last two
    levels; its right-hand side product and assembly scale with its lower /
    all nonzeros at the sample's measured rates."""
    import oracle
    import synth
    from oracle import multiscale as ms

    try:
        from threadpoolctl import threadpool_limits
    except ImportError:  # pragma: no cover
        threadpool_limits = None
    h = synth.halton_hierarchy(levels_sample)
    f = synth.fourier_target(1000)(h.points)
    lim = threadpool_limits(1) if threadpool_limits else None
    try:
        t0 = time.perf_counter()
        blk = ms.assemble(h.points, h.offsets, h.delta)
        t_asm = time.perf_counter() - t0
        fl = ms.split_levels(f, blk.sizes)
        chosen = None
        for rtol in (1e-6, 1e-7, 1e-8, 1e-9, 1e-10, 1e-11):
            alphas, rows = [], []
            for l in range(h.levels):
                t1 = time.perf_counter()
                b = fl[l].copy()
                for k in range(l):
                    b -= blk.mat(l, k) @ alphas[k]
                t2 = time.perf_counter()
                a, it = ms.cg(blk.mat(l, l), b, rtol)
                t3 = time.perf_counter()
                alphas.append(a)
                rows.append({"level": l, "rhs_s": t2 - t1, "cg_s": t3 - t2, "cg_iters": it,
                             "nnz_diag": blk.nnz(l, l), "nnz_lower": sum(blk.nnz(l, k) for k in range(l))})
            rel = float(oracle.residual(blk, np.concatenate(alphas), f)[0])
            log(f"cpu baseline: oracle rtol {rtol:g} -> rel. residual {rel:.3e}")
            if rel <= TARGET:
                chosen = rtol
                break
    finally:
        if lim is not None:
            lim.__exit__(None, None, None)
    if chosen is None:
        raise RuntimeError("cpu baseline: no oracle tolerance reached 1e-8")
    nnz_sample = sum(blk.nnz(k, j) for k in range(h.levels) for j in range(k + 1))
    last, prev = rows[-1], rows[-2]
    growth = last["cg_iters"] / max(prev["cg_iters"], 1)
    s_per_iter_nnz = last["cg_s"] / max(last["cg_iters"] * last["nnz_diag"], 1)
    s_per_lower_nnz = last["rhs_s"] / max(last["nnz_lower"], 1)
    est = [r["rhs_s"] + r["cg_s"] for r in rows]
    iters = last["cg_iters"]
    for l in range(levels_sample, levels_full):
        iters *= growth
        est.append(iters * nnz_full_diag[l] * s_per_iter_nnz + nnz_full_lower[l] * s_per_lower_nnz)
    nnz_full = sum(nnz_full_diag) + sum(nnz_full_lower)
    return {"solve_ms_est": sum(est) * 1e3, "assemble_ms_est": t_asm * nnz_full / nnz_sample * 1e3,
            "sample_solve_ms": sum(r["rhs_s"] + r["cg_s"] for r in rows) * 1e3, "sample_assemble_ms": t_asm * 1e3,
            "rel_residual": rel, "cg_rtol": chosen, "levels": rows, "iter_growth": growth,
            "n_points": h.n_total, "nnz": nnz_sample}


def batched(m, ctx, hd, h, pts_dev, dev, fast_opts, rt_fast, nrhs, count):
    """Many right-hand sides on the bench hierarchy and many independent
    uneven hierarchies, each solved in shared launches (fast form)."""
    import torch

    import synth

    out = {}
    if nrhs > 1:
        log(f"batched: {nrhs} right-hand sides")
        F = torch.stack([synth.fourier_target(3000 + r).torch_eval(pts_dev) for r in range(nrhs)], dim=1).contiguous()
        A = torch.zeros_like(F)
        # several right-hand sides per launch (block-Jacobi preconditioned CG, no learned warm start)
        o = m.solve_opts(cg_rtol=rt_fast, **dict(fast_opts, precond=m.MSKM_PRECOND_BLOCK_JACOBI, mlp=None))
        m.mskm_solve(ctx, hd, F, A, o, nrhs=nrhs)  # warm-up (allocations, code objects)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = m.mskm_solve(ctx, hd, F, A, o, nrhs=nrhs)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) * 1e3
        rel = m.mskm_residual(ctx, hd, A, F, nrhs=nrhs)
        out["multi_rhs"] = {"nrhs": nrhs, "time_to_1e-8_ms": round(wall, 2), "ms_per_rhs": round(wall / nrhs, 3),
                            "max_rel_residual": float(rel.max()), "status": res.status,
                            "cg_iters_total": res.report["cg_iters_total"], "refine": res.report["refine_steps"]}
        log("multi_rhs", out["multi_rhs"])
        # roofline of the solve's dominant kernel: its CG product on the finest level
        top = h.levels - 1
        ms_p = m.mskm_mr_product_time(ctx, hd, top, nrhs, prec=m.MSKM_PREC_FP32, repeats=5)
        nnz_t, n_t = m.block_nnz(ctx, hd, top, top), int(h.sizes()[top])
        byt = nnz_t * 8 + (n_t + 1) * 8 + 2 * n_t * nrhs * 4  # values + columns, row pointers, P read once, Q written
        flop = 2.0 * nnz_t * nrhs
        t_hbm, t_alu = byt / (HBM_PEAK_GBS * 1e9), flop / (FP32_PEAK_TFLOPS * 1e12)
        bound = "hbm" if t_hbm >= t_alu else "alu"
        achieved = byt / (ms_p * 1e-3) / 1e9 if bound == "hbm" else flop / (ms_p * 1e-3) / 1e12
        peak = HBM_PEAK_GBS if bound == "hbm" else FP32_PEAK_TFLOPS
        out["multi_rhs"]["roofline"] = {
            "bound": bound, "achieved": round(achieved, 1), "peak": peak, "unit": "GB/s" if bound == "hbm" else "TFLOP/s",
            "frac": round(achieved / peak, 4), "traffic": pmc_traffic(("halton2d_L8", "k_mr_cg_spmm_w<1,float,float> R=256",
                                                                         "level 7")) if (nrhs == 256 and h.levels == 8) else None,
            "kernel": f"k_mr_cg_spmm_w<1,float,float> (CG product Q = A_l P for {nrhs} right-hand sides in chunks "
                      f"of 64, level {top}: {n_t} rows, {nnz_t} nonzeros, FP32)",
            "ms": round(ms_p, 4), "algorithmic_bytes": byt, "flop": flop,
            "tflops": round(flop / (ms_p * 1e-3) / 1e12, 2),
            "gathered_bytes": nnz_t * nrhs * 4}  # the rows of P read through the caches, one per nonzero
        log("multi_rhs roofline", out["multi_rhs"]["roofline"])
        del F, A
        torch.cuda.empty_cache()
    if count > 0:
        log(f"batched: {count} hierarchies")
        hs = synth.batch_hierarchies(count)
        f = np.concatenate([fb for _, fb in hs])
        f_dev = torch.from_numpy(f).to(dev)
        a_dev = torch.zeros_like(f_dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        hb = m.mskm_hier_create_batch(ctx, [(hh.points, hh.offsets, hh.delta) for hh, _ in hs], fp64=False, fp32=True)
        torch.cuda.synchronize()
        t_asm = (time.perf_counter() - t0) * 1e3
        st = m.mskm_hier_stats_get(hb)
        o = m.solve_opts(cg_rtol=rt_fast, **fast_opts)
        m.mskm_solve(ctx, hb, f_dev, a_dev, o)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = m.mskm_solve(ctx, hb, f_dev, a_dev, o)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) * 1e3
        rel = m.mskm_residual(ctx, hb, a_dev, f_dev)
        out["multi_hierarchy"] = {"hierarchies": count, "n_points": st["n_total"], "levels": st["levels"],
                                  "nnz": st["nnz_diag"] + st["nnz_lower"], "assemble_ms": round(t_asm, 2),
                                  "time_to_1e-8_ms": round(wall, 2), "max_rel_residual": float(rel.max()),
                                  "status": res.status, "cg_iters_total": res.report["cg_iters_total"]}
        log("multi_hierarchy", out["multi_hierarchy"])
        m.mskm_hier_destroy(hb)
    return out


def uniform3d(m, ctx, dev, args):
    """The 3-D mixed-precision workload: 5 prefix-nested levels of a seeded
    uniform stream (512 .. 2,097,152 points, about 60 neighbours per row).
    Fast form (FP32 values and accumulation, FP64 dots and residual
    refinement) against the plain FP64 Jacobi+CG baseline, both to 1e-8, the
    fast form's coefficient error against a tight FP64 solve, and the FP32
    full-T SpMV bandwidth."""
    import torch

    import synth

    h3 = synth.uniform3d_hierarchy(5)
    f3 = torch.from_numpy(synth.fourier_target(2001, dim=3)(h3.points)).to(dev)
    p3 = torch.from_numpy(h3.points).to(dev)
    a3 = torch.zeros_like(f3)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hd3 = m.mskm_hier_create(ctx, p3, h3.offsets, h3.delta, fp64=True, fp32=True, sliced_lower=True)
    torch.cuda.synchronize()
    t_asm = (time.perf_counter() - t0) * 1e3
    st = m.mskm_hier_stats_get(hd3)
    log("uniform3d hierarchy", st)
    m.mskm_autotune(ctx, hd3, repeats=3)
    fast_opts = dict(precision=m.MSKM_PREC_FP32, algorithm=m.MSKM_ALG_SEQUENTIAL, target_rel_residual=TARGET,
                     max_refine=8, precond=m.MSKM_PRECOND_BLOCK_JACOBI)
    plain_opts = dict(precision=m.MSKM_PREC_FP64, algorithm=m.MSKM_ALG_MONOLITHIC)
    out = {"workload": "uniform3d_L5", "n_points": st["n_total"], "nnz": st["nnz_diag"] + st["nnz_lower"],
           "assemble_fp64_fp32_ms": round(t_asm, 2)}
    for label, opts in (("fast", fast_opts), ("plain_fp64_jacobi", plain_opts)):
        rt = calibrate(m, ctx, hd3, f3, a3, opts, f"uniform3d {label}")
        o = m.solve_opts(cg_rtol=rt, **opts)
        ts = []
        for _ in range(3):
            r = m.mskm_solve(ctx, hd3, f3, a3, o)
            ts.append(r.report["solve_ms"])
        rel = float(m.mskm_residual(ctx, hd3, a3, f3)[0])
        out[label] = {"cg_rtol": rt, "time_to_1e-8_ms": round(float(np.median(ts)), 3), "rel_residual": rel,
                      "cg_iters_total": r.report["cg_iters_total"], "status": r.status}
        if label == "fast":
            a_fast = a3.clone()
    # coefficient error of the fast form against a tight FP64 solve
    a_ref = torch.zeros_like(f3)
    m.mskm_solve(ctx, hd3, f3, a_ref, m.solve_opts(cg_rtol=1e-13, precision=m.MSKM_PREC_FP64,
                                                   algorithm=m.MSKM_ALG_SEQUENTIAL))
    errs = []
    for l in range(h3.levels):
        sl = slice(int(h3.offsets[l]), int(h3.offsets[l + 1]))
        errs.append(float(torch.linalg.norm(a_fast[sl] - a_ref[sl]) / torch.linalg.norm(a_ref[sl])))
    out["fast"]["coef_rel_err_vs_fp64_per_level"] = errs
    out["speedup_vs_plain_fp64"] = round(out["plain_fp64_jacobi"]["time_to_1e-8_ms"] / out["fast"]["time_to_1e-8_ms"],
                                         3)
    N3 = st["n_total"]
    x32 = torch.randn(N3, dtype=torch.float32, device=dev)
    y32 = torch.empty_like(x32)
    m.mskm_apply_internal(ctx, hd3, m.MSKM_OP_FULL, x32, y32, prec=m.MSKM_PREC_FP32, repeats=2)
    ms = m.mskm_apply_internal(ctx, hd3, m.MSKM_OP_FULL, x32, y32, prec=m.MSKM_PREC_FP32, repeats=args.spmv_repeats)
    b = spmv_bytes(out["nnz"], N3, 2, 4, 4)
    out["spmv_full_fp32"] = {"ms": round(ms, 4), "bytes": b, "GBps": round(b / ms / 1e6, 1),
                             "variant": m.mskm_spmv_width(hd3, m.MSKM_OP_FULL, m.MSKM_PREC_FP32)}
    log("uniform3d", out)
    m.mskm_hier_destroy(hd3)
    del p3, f3, a3, a_ref, a_fast, x32, y32
    torch.cuda.empty_cache()
    return out


# The paper's own timings for solving its system on the Table 1 grids with the
# Franke target (Figure 4, A100, 3456 warps, seconds): context, not a target
# (other hardware, and the paper does not state its CG tolerance).
PAPER_FIG4_A100_S = {7: 0.974, 8: 1.485, 9: 4.479, 10: 20.111, 11: 92.642}


def paper_workload(m, ctx, dev, levels_list):
    """The paper's own workload: Table 1 grids (spacing 2^-l, l = 1..L,
    delta_l = 4 * fill distance), Franke target, solved to 1e-8 by the plain
    FP64 method (Jacobi sweeps + CG, the paper's algorithm) and by the fast
    form; the paper's A100 times alongside."""
    import torch

    import synth

    out = []
    for L in levels_list:
        h = synth.table1_hierarchy(L)
        f = torch.from_numpy(synth.franke(h.points)).to(dev)
        pts = torch.from_numpy(h.points).to(dev)
        a = torch.zeros_like(f)
        hd = m.mskm_hier_create(ctx, pts, h.offsets, h.delta, fp64=True, fp32=True)
        st = m.mskm_hier_stats_get(hd)
        m.mskm_autotune(ctx, hd, repeats=2)
        row = {"levels": L, "n_points": st["n_total"], "nnz": st["nnz_diag"] + st["nnz_lower"],
               "assemble_ms": round(st["assemble_ms"], 2), "paper_a100_s": PAPER_FIG4_A100_S.get(L)}
        forms = (("fast", dict(precision=m.MSKM_PREC_FP32, algorithm=m.MSKM_ALG_SEQUENTIAL, target_rel_residual=TARGET,
                               max_refine=8, precond=m.MSKM_PRECOND_BLOCK_JACOBI), (1e-4, 1e-5, 1e-6)),
                 ("plain_fp64_jacobi", dict(precision=m.MSKM_PREC_FP64, algorithm=m.MSKM_ALG_MONOLITHIC),
                  (1e-6, 1e-7, 1e-8, 1e-9, 1e-10)))
        for label, opts, ladder in forms:
            for rt in ladder:
                o = m.solve_opts(cg_rtol=rt, **opts)
                m.mskm_solve(ctx, hd, f, a, o)
                r = m.mskm_solve(ctx, hd, f, a, o)
                rel = float(m.mskm_residual(ctx, hd, a, f)[0])
                if rel <= TARGET:
                    row[label] = {"cg_rtol": rt, "time_to_1e-8_ms": round(r.report["solve_ms"], 3),
                                  "rel_residual": rel, "cg_iters_total": r.report["cg_iters_total"]}
                    break
        log("paper workload", row)
        out.append(row)
        m.mskm_hier_destroy(hd)
        del f, pts, a
        torch.cuda.empty_cache()
    return out


def thresholded(m, ctx, dev, L: int, Ts):
    """Section 4's thresholded Jacobi on the Table 1 grids (Franke target):
    the truncated Lagrange blocks X~(T) built on the device (Lagrange
    coefficients by many-right-hand-side CG), then the perturbed split as the
    inner solve of an FP64 residual refinement to 1e-8 (Jacobi sweeps = one
    product with X~ each, then block-Jacobi preconditioned CG on every
    level)."""
    import torch

    import synth

    h = synth.table1_hierarchy(L)
    f = torch.from_numpy(synth.franke(h.points)).to(dev)
    pts = torch.from_numpy(h.points).to(dev)
    a = torch.zeros_like(f)
    hd = m.mskm_hier_create(ctx, pts, h.offsets, h.delta, fp64=True, fp32=False)
    st = m.mskm_hier_stats_get(hd)
    out = {"workload": f"table1_L{L}_franke", "n_points": st["n_total"], "nnz_lower_T": st["nnz_lower"], "rows": []}
    for T in Ts:
        status, t = m.mskm_trunc_create(ctx, hd, float(T))
        info = m.mskm_trunc_info(t, L)
        o = m.solve_opts(cg_rtol=1e-6, target_rel_residual=TARGET, max_refine=40,
                         precond=m.MSKM_PRECOND_BLOCK_JACOBI)
        m.mskm_trunc_solve(ctx, t, f, a, o)
        ts = []
        for _ in range(3):
            r = m.mskm_trunc_solve(ctx, t, f, a, o)
            ts.append(r.report["solve_ms"])
        rel = float(m.mskm_residual(ctx, hd, a, f)[0])
        out["rows"].append({"T": T, "status": status, "build_ms": round(info["build_ms"], 2), "nnz": info["nnz"],
                            "lagrange_cg_iters": info["cg_iters"], "time_to_1e-8_ms": round(float(np.median(ts)), 3),
                            "rounds": r.report["refine_steps"], "cg_iters_total": r.report["cg_iters_total"],
                            "rel_residual": rel, "solve_status": r.status})
        m.mskm_trunc_destroy(t)
    log("thresholded", out)
    m.mskm_hier_destroy(hd)
    del f, pts, a
    torch.cuda.empty_cache()
    return out


def train_warm_start(m, ctx, args):
    """Train the warm-start network on (rhs -> correction) pairs from plain
    solves of a 6-level Halton hierarchy with random Fourier targets."""
    import synth

    h6 = synth.halton_hierarchy(6)
    ntr = args.train_rhs
    F = np.ascontiguousarray(np.stack([synth.fourier_target(5000 + r)(h6.points) for r in range(ntr)], axis=1))
    h6d = m.mskm_hier_create(ctx, h6.points, h6.offsets, h6.delta, fp64=True, fp32=False)
    t0 = time.perf_counter()
    net, loss = m.mskm_mlp_train(ctx, h6d, F, nrhs=ntr, samples=args.train_samples, steps=args.train_steps, lr=1e-3,
                                 seed=5000, cg_rtol=1e-10)
    train_ms = (time.perf_counter() - t0) * 1e3
    m.mskm_hier_destroy(h6d)
    info = {"train_hierarchy": f"halton2d_L6 ({h6.n_total} points)", "train_rhs": ntr,
            "samples": args.train_samples, "steps": args.train_steps, "train_ms": round(train_ms, 1),
            "loss_first": float(loss[0]), "loss_last": float(loss[-1])}
    log("warm start trained", info)
    return net, info


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--levels", type=int, default=8)
    ap.add_argument("--spmv-repeats", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-levels", type=int, default=7)
    ap.add_argument("--nq", type=int, default=65536)
    ap.add_argument("--rhs", type=int, default=256, help="right-hand sides of the batched solve (0: skip)")
    ap.add_argument("--train-rhs", type=int, default=16)
    ap.add_argument("--train-samples", type=int, default=10000)
    ap.add_argument("--train-steps", type=int, default=3000)
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--fast-rtol", type=float, default=0.0,
                    help="inner CG tolerance of the fast form (default: calibrated, the fastest that verifies 1e-8)")
    ap.add_argument("--no-3d", action="store_true", help="skip the 3-D mixed-precision workload")
    ap.add_argument("--paper-levels", default="7,8,9,10,11",
                    help="Table 1 grid hierarchies (comma-separated L) of the paper's own workload ('' to skip)")
    ap.add_argument("--trunc-levels", type=int, default=7,
                    help="Table 1 levels of the thresholded-Jacobi workload (0: skip)")
    ap.add_argument("--spmv-only", action="store_true",
                    help="assemble, autotune, then only time one SpMV operator and a 1 GiB streaming copy kernel "
                         "(the counter-collection runs)")
    ap.add_argument("--spmv-variant", type=int, default=0,
                    help="with --spmv-only: pin this SpMV variant code instead of autotuning")
    ap.add_argument("--spmv-op", choices=("diag", "lower", "full", "cg", "mr"), default="diag",
                    help="with --spmv-only (cg: the CG product kernel on the finest level; mr: its many-rhs form)")
    ap.add_argument("--spmv-prec", choices=("fp32", "fp64"), default="fp32", help="with --spmv-only")
    ap.add_argument("--spmv-rhs", type=int, default=256, help="with --spmv-only --spmv-op mr: right-hand sides")
    ap.add_argument("--batch-count", type=int, default=64, help="hierarchies of the batched solve (0: skip)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)

    import torch

    import paper_2503_04914_amd as m

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    log("generating inputs")
    h, f = build_inputs(args.levels)
    N = h.n_total
    pts_dev = torch.from_numpy(h.points).to(dev)
    f_dev = torch.from_numpy(f).to(dev)
    alpha_dev = torch.zeros(N, dtype=torch.float64, device=dev)
    q_host = np.random.default_rng(12345).random((args.nq, 2))
    q_dev = torch.from_numpy(q_host).to(dev)
    ev_out = torch.zeros(args.nq, dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    # one stream for torch's work, the library's launches and the timing
    # events, so that an event recorded after a call is ordered after its kernels
    work_stream = torch.cuda.Stream(device=dev)
    torch.cuda.set_stream(work_stream)
    ctx = m.mskm_create(0, stream="torch")

    # ---- calibration of the tolerances (untimed)
    hd = m.mskm_hier_create(ctx, pts_dev, h.offsets, h.delta, fp64=True, fp32=True, sliced_lower=True)
    if args.spmv_only:
        st = m.mskm_hier_stats_get(hd)
        op = {"diag": m.MSKM_OP_DIAG, "lower": m.MSKM_OP_LOWER, "full": m.MSKM_OP_FULL, "cg": m.MSKM_OP_DIAG,
              "mr": m.MSKM_OP_DIAG}[args.spmv_op]
        prec = m.MSKM_PREC_FP32 if args.spmv_prec == "fp32" else m.MSKM_PREC_FP64
        if args.spmv_variant:
            m.mskm_set_spmv_width(hd, op, prec, args.spmv_variant)
        else:
            m.mskm_autotune(ctx, hd, repeats=3)
        dt = torch.float32 if prec == m.MSKM_PREC_FP32 else torch.float64
        x = torch.randn(N, dtype=dt, device=dev)
        y = torch.empty_like(x)
        if args.spmv_op == "cg":  # the CG product kernel on the finest level
            top = args.levels - 1
            m.mskm_cg_product_time(ctx, hd, top, prec, repeats=2)
            ms = m.mskm_cg_product_time(ctx, hd, top, prec, repeats=args.spmv_repeats)
        elif args.spmv_op == "mr":  # the many-rhs CG product on the finest level
            top = args.levels - 1
            m.mskm_mr_product_time(ctx, hd, top, args.spmv_rhs, prec=prec, repeats=2)
            ms = m.mskm_mr_product_time(ctx, hd, top, args.spmv_rhs, prec=prec, repeats=args.spmv_repeats)
        else:
            m.mskm_apply_internal(ctx, hd, op, x, y, prec=prec, repeats=2)
            ms = m.mskm_apply_internal(ctx, hd, op, x, y, prec=prec, repeats=args.spmv_repeats)
        src = torch.ones(1 << 27, dtype=torch.float64, device=dev)  # 1 GiB
        dst = torch.empty_like(src)
        torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.spmv_repeats):
            torch.mul(src, 1.0, out=dst)  # a plain streaming kernel: reads 1 GiB, writes 1 GiB
        e1.record()
        torch.cuda.synchronize()
        sv = 4 if prec == m.MSKM_PREC_FP32 else 8
        code = m.mskm_spmv_width(hd, op, prec)
        if args.spmv_op == "cg":
            top = args.levels - 1
            n_top = int(h.offsets[top + 1] - h.offsets[top])
            b = spmv_bytes(m.block_nnz(ctx, hd, top, top), n_top, 1, sv, sv) + n_top * sv
            kname = cg_product_kernel_name(code, bool(st["sell_col16"]))
        elif args.spmv_op == "mr":
            top = args.levels - 1
            n_top = int(h.offsets[top + 1] - h.offsets[top])
            b = m.block_nnz(ctx, hd, top, top) * (sv + 4) + (n_top + 1) * 8 + 2 * n_top * args.spmv_rhs * sv
            tname = "float" if sv == 4 else "double"
            kname = f"mskm::k_mr_cg_spmm_w<1, {tname}, {tname}> (or the chunk width timed fastest)"
        else:
            nnz = {"diag": st["nnz_diag"], "lower": st["nnz_lower"], "full": st["nnz_diag"] + st["nnz_lower"]}[args.spmv_op]
            sc = diag_col_bytes(code, st) if args.spmv_op == "diag" else 4
            b = spmv_bytes(nnz, N, 2 if args.spmv_op == "full" else 1, sv, sv, sc)
            kname = spmv_kernel_name(code, "float" if sv == 4 else "double", st["sell_col16"])
        print(json.dumps({"op": args.spmv_op, "prec": args.spmv_prec, "ms": ms, "bytes": b, "GBps": b / ms / 1e6,
                          "variant": code, "sell_col16": st["sell_col16"], "kernel": kname,
                          "copy_bytes_each_way": 1 << 30, "copy_ms": e0.elapsed_time(e1) / args.spmv_repeats}))
        m.mskm_hier_destroy(hd)
        m.mskm_destroy(ctx)
        return
    stats = m.mskm_hier_stats_get(hd)
    log("hierarchy", stats)
    nnz_levels = {"diag": [m.block_nnz(ctx, hd, l, l) for l in range(args.levels)],
                  "lower": [sum(m.block_nnz(ctx, hd, l, j) for j in range(l)) for l in range(args.levels)]}
    tune = m.mskm_autotune(ctx, hd, repeats=5)
    widths = {f"{op}_{pr}": m.mskm_spmv_width(hd, i, j) for i, op in enumerate(("diag", "lower", "full"))
              for j, pr in enumerate(("fp64", "fp32"))}
    log("autotune ms [op][prec][variant]", m.TUNE_VARIANTS, np.round(tune, 3).tolist(), "chosen", widths)
    fast_opts = dict(precision=m.MSKM_PREC_FP32, algorithm=m.MSKM_ALG_SEQUENTIAL, target_rel_residual=TARGET,
                     max_refine=8, precond=m.MSKM_PRECOND_BLOCK_JACOBI)
    plain_opts = dict(precision=m.MSKM_PREC_FP64, algorithm=m.MSKM_ALG_MONOLITHIC)
    rt_fast = args.fast_rtol or calibrate(m, ctx, hd, f_dev, alpha_dev, fast_opts, "fast")
    learned = None
    if not args.no_learned:
        net, tinfo = train_warm_start(m, ctx, args)
        # held-out target (seed 6000) on the bench hierarchy: with vs without warm start
        import synth

        f_ho = torch.from_numpy(synth.fourier_target(6000)(h.points)).to(dev)
        cmp = {}
        # the warm start replaces the preconditioner: compare it with plain CG from zero
        for label, extra in (("zero_start", {"precond": m.MSKM_PRECOND_NONE}),
                             ("learned_start", {"precond": m.MSKM_PRECOND_LEARNED, "mlp": net.value}),
                             ("learned_start_block_jacobi", {"warm_start": m.MSKM_START_LEARNED, "mlp": net.value}),
                             ("flexible_cg_learned_preconditioner",
                              {"precond": m.MSKM_PRECOND_FLEX_LEARNED, "mlp": net.value})):
            o = m.solve_opts(cg_rtol=rt_fast, **dict(fast_opts, **extra))
            m.mskm_solve(ctx, hd, f_ho, alpha_dev, o)
            ts = []
            for _ in range(2):
                r = m.mskm_solve(ctx, hd, f_ho, alpha_dev, o)
                ts.append(r.report["solve_ms"])
            rel = float(m.mskm_residual(ctx, hd, alpha_dev, f_ho)[0])
            cmp[label] = {"time_to_1e-8_ms": round(float(np.median(ts)), 3), "rel_residual": rel,
                          "cg_iters_total": r.report["cg_iters_total"], "warm_fallbacks": r.report["warm_fallbacks"],
                          "status": r.status}
        learned = {**tinfo, "held_out_seed": 6000, **cmp}
        log("learned", learned)
        learned["block_jacobi_fast_form_ms"] = None
        o = m.solve_opts(cg_rtol=rt_fast, **fast_opts)
        m.mskm_solve(ctx, hd, f_ho, alpha_dev, o)
        learned["block_jacobi_fast_form_ms"] = round(m.mskm_solve(ctx, hd, f_ho, alpha_dev, o).report["solve_ms"], 3)
        # the fastest learned form that verifies the target replaces the fast form if it beats it
        best = min(("learned_start", "learned_start_block_jacobi", "flexible_cg_learned_preconditioner"),
                   key=lambda k: cmp[k]["time_to_1e-8_ms"] if cmp[k]["rel_residual"] <= TARGET else float("inf"))
        use = (cmp[best]["time_to_1e-8_ms"] < learned["block_jacobi_fast_form_ms"]
               and cmp[best]["rel_residual"] <= TARGET)
        learned["used_in_fast_form"] = best if use else None
        if use:
            extra = {"learned_start": {"precond": m.MSKM_PRECOND_LEARNED},
                     "learned_start_block_jacobi": {"warm_start": m.MSKM_START_LEARNED},
                     "flexible_cg_learned_preconditioner": {"precond": m.MSKM_PRECOND_FLEX_LEARNED}}[best]
            fast_opts = dict(fast_opts, mlp=net.value, **extra)
    fast = m.solve_opts(cg_rtol=rt_fast, **fast_opts)

    def step():
        e = [torch.cuda.Event(enable_timing=True) for _ in range(5)]
        e[0].record()
        hs = m.mskm_hier_create(ctx, pts_dev, h.offsets, h.delta, fp64=False, fp32=True, sliced_lower=True)
        e[1].record()
        res = m.mskm_solve(ctx, hs, f_dev, alpha_dev, fast)
        e[2].record()
        rel = float(m.mskm_residual(ctx, hs, alpha_dev, f_dev)[0])
        e[3].record()
        m.mskm_evaluate(ctx, hs, alpha_dev, q_dev, ev_out)
        e[4].record()
        m.mskm_hier_destroy(hs)
        torch.cuda.synchronize()
        ph = [e[i].elapsed_time(e[i + 1]) for i in range(4)]
        return {"assemble_ms": ph[0], "solve_ms": ph[1], "residual_ms": ph[2], "evaluate_ms": ph[3],
                "rel_residual": rel, "status": res.status, "cg_iters": res.report["cg_iters_total"],
                "refine": res.report["refine_steps"]}

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    steps = [step() for _ in range(args.steps)]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = wall * 1e3 / args.steps
    for s in steps:
        if s["rel_residual"] > TARGET or s["status"] < 0:
            raise RuntimeError(f"fast solve missed the target: {s}")
    fast_ms = float(np.median([s["solve_ms"] for s in steps]))
    log("steps", steps)

    # ---- plain FP64 baseline (Jacobi + CG, L sweeps), same target
    rt_plain = calibrate(m, ctx, hd, f_dev, alpha_dev, plain_opts, "plain")
    plain = m.solve_opts(cg_rtol=rt_plain, **plain_opts)
    pt = []
    for _ in range(2):
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        pr = m.mskm_solve(ctx, hd, f_dev, alpha_dev, plain)
        e1.record()
        torch.cuda.synchronize()
        pt.append(e0.elapsed_time(e1))
    plain_rel = float(m.mskm_residual(ctx, hd, alpha_dev, f_dev)[0])
    plain_ms = float(np.median(pt))
    seq64 = m.solve_opts(cg_rtol=rt_plain, precision=m.MSKM_PREC_FP64, algorithm=m.MSKM_ALG_SEQUENTIAL)
    sr = m.mskm_solve(ctx, hd, f_dev, alpha_dev, seq64)
    seq64_ms = sr.report["solve_ms"]

    # ---- standalone SpMV kernels (internal order, HIP events around the launches)
    x64 = torch.randn(N, dtype=torch.float64, device=dev)
    y64 = torch.empty_like(x64)
    x32, y32 = x64.float(), torch.empty(N, dtype=torch.float32, device=dev)
    nnz_d, nnz_l = stats["nnz_diag"], stats["nnz_lower"]
    spmv = {}
    for name, op, prec, x, y, nnz, nrp, sval, sx in [
        ("full_fp64", m.MSKM_OP_FULL, m.MSKM_PREC_FP64, x64, y64, nnz_d + nnz_l, 2, 8, 8),
        ("full_fp32", m.MSKM_OP_FULL, m.MSKM_PREC_FP32, x32, y32, nnz_d + nnz_l, 2, 4, 4),
        ("diag_fp64", m.MSKM_OP_DIAG, m.MSKM_PREC_FP64, x64, y64, nnz_d, 1, 8, 8),
        ("diag_fp32", m.MSKM_OP_DIAG, m.MSKM_PREC_FP32, x32, y32, nnz_d, 1, 4, 4),
        ("lower_fp64", m.MSKM_OP_LOWER, m.MSKM_PREC_FP64, x64, y64, nnz_l, 1, 8, 8),
    ]:
        m.mskm_apply_internal(ctx, hd, op, x, y, prec=prec, repeats=2)
        ms = m.mskm_apply_internal(ctx, hd, op, x, y, prec=prec, repeats=args.spmv_repeats)
        sc = diag_col_bytes(m.mskm_spmv_width(hd, op, prec), stats) if op == m.MSKM_OP_DIAG else 4
        b = spmv_bytes(nnz, N, nrp, sval, sx, sc)
        spmv[name] = {"ms": ms, "bytes": b, "GBps": b / ms / 1e6, "variant": m.mskm_spmv_width(hd, op, prec)}
    log("spmv", spmv)
    # the dominant kernel of the timed step: the CG product on the diagonal
    # blocks, FP32, at the launch shape of the finest level (its largest launch)
    top = args.levels - 1
    n_top = int(h.offsets[top + 1] - h.offsets[top])
    m.mskm_cg_product_time(ctx, hd, top, m.MSKM_PREC_FP32, repeats=3)
    cg_ms = m.mskm_cg_product_time(ctx, hd, top, m.MSKM_PREC_FP32, repeats=args.spmv_repeats)
    # SpMV bytes of the level (values + int32 columns, row metadata, x read, q
    # written) + the second vector its dot partials read (r)
    cg_bytes = spmv_bytes(nnz_levels["diag"][top], n_top, 1, 4, 4) + n_top * 4
    cg_stored = spmv_bytes(nnz_levels["diag"][top], n_top, 1, 4, 4, diag_col_bytes(widths["diag_fp32"], stats)) + n_top * 4
    cg_kernel = cg_product_kernel_name(widths["diag_fp32"], bool(stats["sell_col16"]))
    log("cg product", cg_kernel, cg_ms, cg_bytes / cg_ms / 1e6)
    bt = batched(m, ctx, hd, h, pts_dev, dev, fast_opts, rt_fast, args.rhs, args.batch_count)
    m.mskm_hier_destroy(hd)
    u3 = None if args.no_3d else uniform3d(m, ctx, dev, args)
    pw = paper_workload(m, ctx, dev, [int(x) for x in args.paper_levels.split(",") if x]) if args.paper_levels else None
    thr = thresholded(m, ctx, dev, args.trunc_levels, (2, 4, 6)) if args.trunc_levels > 0 else None
    m.mskm_destroy(ctx)

    traffic = pmc_traffic((f"halton2d_L{args.levels}", cg_kernel, f"level {top}"))
    cg_gbps = cg_bytes / cg_ms / 1e6
    out = {
        "metric": "time-to-1e-8 rel. residual + kernel SpMV GB/s, plain FP64 vs mixed/learned",
        "value": round(fast_ms, 3),
        "unit": "ms",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32/f64",
        "data": "synthetic",
        "config": {"workload": f"halton2d_L{args.levels}", "n_points": N, "levels": args.levels,
                   "nnz": nnz_d + nnz_l, "kernel": "wendland_3_1", "neighbours_per_row": 40,
                   "target": "fourier32_seed1000", "parallelism": "single_gpu"},
        "fast_form": {"name": "mixed FP32/FP64-refined, block forward substitution, "
                      + (learned["used_in_fast_form"].replace("_", " ") if learned and learned.get("used_in_fast_form")
                         else "cell block-Jacobi preconditioned CG"),
                      "cg_rtol": rt_fast,
                      "time_to_1e-8_ms": round(fast_ms, 3), "steps": steps},
        "plain_fp64_jacobi": {"cg_rtol": rt_plain, "time_to_1e-8_ms": round(plain_ms, 3),
                              "rel_residual": plain_rel, "sweeps": h.levels,
                              "cg_iters_total": pr.report["cg_iters_total"]},
        "plain_fp64_sequential_ms": round(seq64_ms, 3),
        "speedup_vs_plain_fp64": round(plain_ms / fast_ms, 3),
        "spmv": {k: {kk: round(vv, 4) if isinstance(vv, float) else vv for kk, vv in v.items()}
                 for k, v in spmv.items()},
        "batched": bt,
        "learned": learned,
        "uniform3d_mixed": u3,
        "paper_table1_franke": pw,
        "thresholded_jacobi": thr,
        "spmv_GBps": round(spmv["diag_fp32"]["GBps"], 1),
        "spmv_widths": widths,
        "roofline": {"bound": "hbm", "achieved": round(cg_gbps, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(cg_gbps / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "kernel": cg_kernel + f" (CG product q = A_l z with its dot partials, level {top}: "
                               f"{n_top} rows, {nnz_levels['diag'][top]} nonzeros, FP32)",
                     "algorithmic_bytes": cg_bytes, "ms": round(cg_ms, 5),
                     "stored_bytes": cg_stored, "frac_stored_bytes": round(cg_stored / cg_ms / 1e6 / HBM_PEAK_GBS, 4)},
    }
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle, 1 thread)")
        cb = cpu_baseline(args.cpu_levels, args.levels, nnz_levels["diag"], nnz_levels["lower"])
        out["cpu_baseline"] = {
            "value": round(cb["solve_ms_est"], 1), "unit": "ms", "cores": 1, "kind": "oracle",
            "sample": f"first {len(cb['levels'])} of the {args.levels} Halton levels ({cb['n_points']} points, "
                      f"{cb['nnz']} nonzeros), the oracle's block forward substitution with textbook CG from zero "
                      f"(rtol {cb['cg_rtol']:g}) to rel. residual {cb['rel_residual']:.2e}, single thread, measured "
                      f"per level; value = measured levels + each missing finer level estimated from the last "
                      f"measured one (time per CG iteration per diagonal nonzero, iterations x "
                      f"{cb['iter_growth']:.2f} per level, the measured growth of the last two levels)",
            "sample_solve_ms": round(cb["sample_solve_ms"], 1), "sample_assemble_ms": round(cb["sample_assemble_ms"], 1),
            "assemble_ms_est": round(cb["assemble_ms_est"], 1),
            "per_level": [{k: (round(v, 4) if isinstance(v, float) else v) for k, v in r.items()} for r in cb["levels"]],
            **host_cpu()}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
