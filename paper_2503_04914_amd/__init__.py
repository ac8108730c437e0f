"""MI355X (gfx950) multiscale kernel solver: thin Python binding of ``libmskm.so``.

The functions here carry the C ABI's names (see ``include/mskm.h``) and only
marshal arguments: every step of assembly, solve, residual and evaluation runs
in the library's HIP kernels. Host arrays are numpy; device arrays are torch
tensors on the GPU (the call then passes ``MSKM_IO_DEVICE`` and uses the
tensor's memory directly, on torch's current stream when the context was
created with ``stream="torch"``).

The library must be built first (``python -m paper_2503_04914_amd.build``);
importing the functions without it raises ``MskmLibraryMissing`` -- there is
no fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmskm.so")

# status codes (mskm.h)
MSKM_OK, MSKM_ENOCONV = 0, 1
MSKM_EINVAL, MSKM_ENOMEM, MSKM_EDEVICE, MSKM_ELIMIT, MSKM_ESTATE = -1, -2, -3, -4, -5
MSKM_WENDLAND_3_1 = 31
MSKM_POINTS_ON_DEVICE, MSKM_STORE_FP64, MSKM_STORE_FP32, MSKM_PREFIX_NESTED, MSKM_SLICED_LOWER = 1, 2, 4, 8, 16
MSKM_IO_DEVICE = 1
MSKM_OP_DIAG, MSKM_OP_LOWER, MSKM_OP_FULL = 0, 1, 2
MSKM_PREC_FP64, MSKM_PREC_FP32 = 0, 1
MSKM_ALG_MONOLITHIC, MSKM_ALG_SEQUENTIAL = 0, 1
MSKM_PRECOND_NONE, MSKM_PRECOND_LEARNED, MSKM_PRECOND_BLOCK_JACOBI, MSKM_PRECOND_FLEX_LEARNED = 0, 1, 2, 3
MSKM_START_ZERO, MSKM_START_PREVIOUS, MSKM_START_LEARNED = 0, 1, 2

EXPORTED = [
    "mskm_create", "mskm_destroy", "mskm_last_error", "mskm_abi_version",
    "mskm_hier_create", "mskm_hier_create_batch", "mskm_hier_destroy", "mskm_hier_stats_get", "mskm_hier_offsets",
    "mskm_hier_level_info",
    "mskm_export_block", "mskm_export_rows", "mskm_export_perm", "mskm_apply", "mskm_apply_internal",
    "mskm_autotune", "mskm_spmv_width", "mskm_set_spmv_width", "mskm_cg_product_time", "mskm_mr_product_time",
    "mskm_set_mr_chunk",
    "mskm_solve_opts_default", "mskm_solve", "mskm_solve_batch", "mskm_residual", "mskm_residual_noalloc",
    "mskm_evaluate",
    "mskm_trunc_create", "mskm_trunc_destroy", "mskm_trunc_info", "mskm_trunc_export_block", "mskm_trunc_solve",
    "mskm_mlp_train", "mskm_mlp_fit", "mskm_mlp_destroy", "mskm_mlp_save", "mskm_mlp_load", "mskm_mlp_predict", "mskm_knn_export",
]


class MskmLibraryMissing(RuntimeError):
    pass


class MskmError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"mskm status {status}: {msg}")
        self.status = status


class HierDesc(C.Structure):
    _fields_ = [("dim", C.c_int32), ("levels", C.c_int32), ("level_offsets", C.POINTER(C.c_int64)),
                ("points", C.c_void_p), ("delta", C.POINTER(C.c_double)), ("kernel", C.c_int32),
                ("flags", C.c_int32)]


class HierStats(C.Structure):
    _fields_ = [("dim", C.c_int32), ("levels", C.c_int32), ("n_total", C.c_int64), ("nnz_diag", C.c_int64),
                ("nnz_lower", C.c_int64), ("has_fp64", C.c_int32), ("has_fp32", C.c_int32),
                ("device_bytes", C.c_int64), ("assemble_ms", C.c_double), ("ngroups", C.c_int32),
                ("sell_col16", C.c_int32), ("sell_entries", C.c_int64), ("lower_sliced", C.c_int32),
                ("lower_sliced_entries", C.c_int64)]


class LevelInfo(C.Structure):
    _fields_ = [("group", C.c_int32), ("depth", C.c_int32), ("n", C.c_int64), ("input_offset", C.c_int64),
                ("delta", C.c_double)]


class SolveOpts(C.Structure):
    _fields_ = [("precision", C.c_int32), ("algorithm", C.c_int32), ("cg_rtol", C.c_double), ("sweeps", C.c_int32),
                ("max_cg_iters", C.c_int32), ("warm_start", C.c_int32), ("target_rel_residual", C.c_double),
                ("max_refine", C.c_int32), ("precond", C.c_int32), ("mlp", C.c_void_p), ("check_every", C.c_int32),
                ("flags", C.c_int32)]


class Report(C.Structure):
    _fields_ = [("levels", C.c_int32), ("sweeps_done", C.c_int32), ("refine_steps", C.c_int32),
                ("cg_iters_total", C.c_int64), ("cg_iters_last", C.c_int32 * 64), ("rel_residual", C.c_double),
                ("solve_ms", C.c_double), ("warm_fallbacks", C.c_int32)]


class TrainDesc(C.Structure):
    _fields_ = [("h", C.c_void_p), ("f", C.c_void_p), ("nrhs", C.c_int32), ("samples", C.c_int64),
                ("steps", C.c_int32), ("lr", C.c_float), ("seed", C.c_uint64), ("cg_rtol", C.c_double),
                ("flags", C.c_int32)]


_lib = None


def lib():
    """The loaded library (raises MskmLibraryMissing if it was not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise MskmLibraryMissing(f"{LIB_PATH} not found: build it with python -m paper_2503_04914_amd.build")
    # torch ships its own HIP runtime under the same soname. Loading torch
    # first makes the library bind to that runtime, so device pointers and
    # streams are shared and only one runtime opens the GPU; loaded the other
    # way round, the process holds two runtimes and torch's finds no device.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, dp = C.c_void_p, C.c_int32, C.c_int64, C.POINTER(C.c_double)
    L.mskm_create.argtypes = [i32, vp, C.POINTER(vp)]
    L.mskm_destroy.argtypes = [vp]
    L.mskm_last_error.restype = C.c_char_p
    L.mskm_abi_version.restype = i32
    L.mskm_hier_create.argtypes = [vp, C.POINTER(HierDesc), C.POINTER(vp)]
    L.mskm_hier_destroy.argtypes = [vp]
    L.mskm_hier_stats_get.argtypes = [vp, C.POINTER(HierStats)]
    L.mskm_hier_offsets.argtypes = [vp, C.POINTER(i64)]
    L.mskm_hier_create_batch.argtypes = [vp, C.POINTER(HierDesc), i32, C.POINTER(vp)]
    L.mskm_hier_level_info.argtypes = [vp, i32, C.POINTER(LevelInfo)]
    L.mskm_export_block.argtypes = [vp, vp, i32, i32, vp, vp, vp, C.POINTER(i64)]
    L.mskm_export_perm.argtypes = [vp, vp, vp]
    L.mskm_export_rows.argtypes = [vp, vp, i32, i32, vp, i64, vp, vp, vp, C.POINTER(i64)]
    L.mskm_apply.argtypes = [vp, vp, i32, i32, vp, i32, vp, i32]
    L.mskm_apply_internal.argtypes = [vp, vp, i32, i32, vp, vp, i32, C.POINTER(C.c_float)]
    L.mskm_autotune.argtypes = [vp, vp, i32, C.POINTER(C.c_float)]
    L.mskm_spmv_width.argtypes = [vp, i32, i32, C.POINTER(i32)]
    L.mskm_set_spmv_width.argtypes = [vp, i32, i32, i32]
    L.mskm_cg_product_time.argtypes = [vp, vp, i32, i32, i32, C.POINTER(C.c_float)]
    L.mskm_mr_product_time.argtypes = [vp, vp, i32, i32, i32, i32, C.POINTER(C.c_float)]
    L.mskm_set_mr_chunk.argtypes = [vp, i32, i32, i32]
    L.mskm_solve_opts_default.argtypes = [C.POINTER(SolveOpts)]
    L.mskm_solve_opts_default.restype = None
    L.mskm_solve.argtypes = [vp, vp, vp, i32, C.POINTER(SolveOpts), vp, C.POINTER(Report)]
    L.mskm_solve_batch.argtypes = [vp, C.POINTER(vp), i32, C.POINTER(vp), C.POINTER(i32), C.POINTER(SolveOpts),
                                   C.POINTER(vp), C.POINTER(Report)]
    L.mskm_residual.argtypes = [vp, vp, vp, vp, i32, dp, i32]
    L.mskm_residual_noalloc.argtypes = [vp, vp, vp, vp, i32, vp]
    L.mskm_evaluate.argtypes = [vp, vp, vp, i32, vp, i64, vp, i32]
    L.mskm_trunc_create.argtypes = [vp, vp, C.c_double, C.c_double, C.POINTER(vp)]
    L.mskm_trunc_destroy.argtypes = [vp]
    L.mskm_trunc_info.argtypes = [vp, vp, C.POINTER(i64), C.POINTER(i64), C.POINTER(C.c_double)]
    L.mskm_trunc_export_block.argtypes = [vp, vp, i32, i32, vp, vp, vp, C.POINTER(i64)]
    L.mskm_trunc_solve.argtypes = [vp, vp, vp, C.POINTER(SolveOpts), vp, C.POINTER(Report)]
    L.mskm_mlp_train.argtypes = [vp, C.POINTER(TrainDesc), C.POINTER(vp), C.POINTER(C.c_float)]
    L.mskm_mlp_fit.argtypes = [vp, vp, vp, vp, i64, i32, C.c_float, i32, C.POINTER(C.c_float)]
    L.mskm_mlp_destroy.argtypes = [vp]
    L.mskm_mlp_save.argtypes = [vp, vp, C.POINTER(C.c_size_t)]
    L.mskm_mlp_load.argtypes = [vp, vp, C.c_size_t, C.POINTER(vp)]
    L.mskm_mlp_predict.argtypes = [vp, vp, vp, vp, vp, i32]
    L.mskm_knn_export.argtypes = [vp, vp, i32, vp]
    for name in EXPORTED:
        if name not in ("mskm_last_error", "mskm_abi_version", "mskm_solve_opts_default"):
            getattr(L, name).restype = i32
    _lib = L
    return L


def _check(st: int, what: str) -> int:
    if st < 0:
        msg = lib().mskm_last_error().decode(errors="replace")
        raise MskmError(st, f"{what}: {msg}")
    return st


def _is_torch(a) -> bool:
    return type(a).__module__.startswith("torch")


def _ptr(a, dtype):
    """(pointer, on_device) of a C-contiguous array of the given numpy dtype."""
    if _is_torch(a):
        import torch

        want = {np.float64: torch.float64, np.int64: torch.int64, np.int32: torch.int32}[dtype]
        if a.dtype != want or not a.is_contiguous():
            raise TypeError(f"tensor must be contiguous {want}")
        return C.c_void_p(a.data_ptr()), a.is_cuda
    if not (isinstance(a, np.ndarray) and a.dtype == dtype and a.flags.c_contiguous):
        raise TypeError(f"array must be a C-contiguous numpy {np.dtype(dtype).name} array")
    return C.c_void_p(a.ctypes.data), False


# ----------------------------------------------------------------- context

def mskm_abi_version() -> int:
    return int(lib().mskm_abi_version())


def mskm_last_error() -> str:
    return lib().mskm_last_error().decode(errors="replace")


def mskm_create(device: int = 0, stream=None):
    """Context on `device`. stream: None (library stream), "torch" (torch's
    current stream, which must not be the default stream: a null handle asks
    the library for a stream of its own, unordered with torch's work) or a
    raw hipStream_t integer."""
    if stream == "torch":
        import torch

        stream = torch.cuda.current_stream(device).cuda_stream
        if not stream:
            raise ValueError("torch's current stream is the default stream; set a torch.cuda.Stream first")
    out = C.c_void_p()
    _check(lib().mskm_create(int(device), C.c_void_p(stream) if stream else None, C.byref(out)), "mskm_create")
    return out


def mskm_destroy(ctx) -> None:
    lib().mskm_destroy(ctx)


# --------------------------------------------------------------- hierarchy

def mskm_hier_create(ctx, points, offsets, delta, dim: int | None = None, fp64: bool = True, fp32: bool = False,
                     prefix_nested: bool = False, sliced_lower: bool = False):
    """Assemble all blocks of a hierarchy. points: [N][dim] float64 (numpy, or
    a CUDA tensor), offsets: [L+1] int64, delta: [L] float64 (host). With
    prefix_nested, points holds only the largest level and level l is its
    first offsets[l+1] - offsets[l] points; sliced_lower also keeps the
    sliced copy of the lower blocks."""
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    delta = np.ascontiguousarray(delta, dtype=np.float64)
    if dim is None:
        dim = int(points.shape[1])
    pp, pdev = _ptr(points, np.float64)
    flags = (MSKM_POINTS_ON_DEVICE if pdev else 0) | (MSKM_STORE_FP64 if fp64 else 0) | \
        (MSKM_STORE_FP32 if fp32 else 0) | (MSKM_PREFIX_NESTED if prefix_nested else 0) | \
        (MSKM_SLICED_LOWER if sliced_lower else 0)
    d = HierDesc(dim, len(delta), offsets.ctypes.data_as(C.POINTER(C.c_int64)), pp,
                 delta.ctypes.data_as(C.POINTER(C.c_double)), MSKM_WENDLAND_3_1, flags)
    out = C.c_void_p()
    _check(lib().mskm_hier_create(ctx, C.byref(d), C.byref(out)), "mskm_hier_create")
    return out


def mskm_hier_create_batch(ctx, hierarchies, fp64: bool = True, fp32: bool = False, sliced_lower: bool = False):
    """One object holding several independent hierarchies; `hierarchies` is a
    list of (points [N_g][dim], offsets [L_g+1], delta [L_g]) host arrays."""
    keep = []
    descs = (HierDesc * len(hierarchies))()
    for g, (points, offsets, delta) in enumerate(hierarchies):
        offsets = np.ascontiguousarray(offsets, dtype=np.int64)
        delta = np.ascontiguousarray(delta, dtype=np.float64)
        pp, pdev = _ptr(points, np.float64)
        keep += [offsets, delta, points]
        flags = (MSKM_POINTS_ON_DEVICE if pdev else 0) | (MSKM_STORE_FP64 if fp64 else 0) | \
                (MSKM_STORE_FP32 if fp32 else 0) | (MSKM_SLICED_LOWER if sliced_lower else 0)
        descs[g] = HierDesc(int(points.shape[1]), len(delta), offsets.ctypes.data_as(C.POINTER(C.c_int64)), pp,
                            delta.ctypes.data_as(C.POINTER(C.c_double)), MSKM_WENDLAND_3_1, flags)
    out = C.c_void_p()
    _check(lib().mskm_hier_create_batch(ctx, descs, len(hierarchies), C.byref(out)), "mskm_hier_create_batch")
    return out


def mskm_hier_level_info(h, level: int) -> dict:
    i = LevelInfo()
    _check(lib().mskm_hier_level_info(h, level, C.byref(i)), "mskm_hier_level_info")
    return {k: getattr(i, k) for k, _ in LevelInfo._fields_}


def mskm_hier_destroy(h) -> None:
    lib().mskm_hier_destroy(h)


def mskm_hier_stats_get(h) -> dict:
    s = HierStats()
    _check(lib().mskm_hier_stats_get(h, C.byref(s)), "mskm_hier_stats_get")
    return {k: getattr(s, k) for k, _ in HierStats._fields_}


def mskm_export_block(ctx, h, row_level: int, col_level: int, values: bool = True):
    """Canonical CSR (rowptr int64, col int32, val float64 or None) of B_{row,col}."""
    nnz = C.c_int64()
    _check(lib().mskm_export_block(ctx, h, row_level, col_level, None, None, None, C.byref(nnz)), "export (size)")
    n = nnz.value
    off = mskm_hier_offsets(h)
    rowptr = np.zeros(int(off[row_level + 1] - off[row_level]) + 1, dtype=np.int64)
    col = np.zeros(max(n, 1), dtype=np.int32)
    val = np.zeros(max(n, 1), dtype=np.float64) if values else None
    _check(lib().mskm_export_block(ctx, h, row_level, col_level, C.c_void_p(rowptr.ctypes.data),
                                   C.c_void_p(col.ctypes.data), C.c_void_p(val.ctypes.data) if values else None,
                                   C.byref(nnz)), "mskm_export_block")
    return rowptr, col[:n], (val[:n] if values else None)


def block_nnz(ctx, h, row_level: int, col_level: int) -> int:
    """Stored entries of B_{row,col} (mskm_export_block's size query)."""
    nnz = C.c_int64()
    _check(lib().mskm_export_block(ctx, h, row_level, col_level, None, None, None, C.byref(nnz)), "export (size)")
    return int(nnz.value)


def mskm_export_rows(ctx, h, row_level: int, col_level: int, rows, values: bool = True):
    """Canonical CSR of the listed rows (indices within row_level) of B_{row,col}."""
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    nnz = C.c_int64()
    _check(lib().mskm_export_rows(ctx, h, row_level, col_level, C.c_void_p(rows.ctypes.data), len(rows), None, None,
                                  None, C.byref(nnz)), "export_rows (size)")
    n = nnz.value
    rowptr = np.zeros(len(rows) + 1, dtype=np.int64)
    col = np.zeros(max(n, 1), dtype=np.int32)
    val = np.zeros(max(n, 1), dtype=np.float64) if values else None
    _check(lib().mskm_export_rows(ctx, h, row_level, col_level, C.c_void_p(rows.ctypes.data), len(rows),
                                  C.c_void_p(rowptr.ctypes.data), C.c_void_p(col.ctypes.data),
                                  C.c_void_p(val.ctypes.data) if values else None, C.byref(nnz)), "mskm_export_rows")
    return rowptr, col[:n], (val[:n] if values else None)


def mskm_hier_offsets(h) -> np.ndarray:
    L = mskm_hier_stats_get(h)["levels"]
    off = np.zeros(L + 1, dtype=np.int64)
    _check(lib().mskm_hier_offsets(h, off.ctypes.data_as(C.POINTER(C.c_int64))), "mskm_hier_offsets")
    return off


def mskm_export_perm(ctx, h, n_total: int) -> np.ndarray:
    perm = np.zeros(n_total, dtype=np.int32)
    _check(lib().mskm_export_perm(ctx, h, C.c_void_p(perm.ctypes.data)), "mskm_export_perm")
    return perm


# ------------------------------------------------------------------- solve

def mskm_apply(ctx, h, op: int, x, y, prec: int = MSKM_PREC_FP64, nrhs: int = 1) -> None:
    xp, xd = _ptr(x, np.float64)
    yp, yd = _ptr(y, np.float64)
    if xd != yd:
        raise ValueError("x and y must both be host or both be device arrays")
    _check(lib().mskm_apply(ctx, h, op, prec, xp, nrhs, yp, MSKM_IO_DEVICE if xd else 0), "mskm_apply")


def mskm_apply_internal(ctx, h, op: int, x, y, prec: int = MSKM_PREC_FP64, repeats: int = 1) -> float:
    """y = op x on CUDA tensors in the internal order; returns mean ms per launch."""
    if not (_is_torch(x) and _is_torch(y) and x.is_cuda and y.is_cuda):
        raise TypeError("mskm_apply_internal takes CUDA tensors")
    ms = C.c_float()
    _check(lib().mskm_apply_internal(ctx, h, op, prec, C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()), repeats,
                                     C.byref(ms)), "mskm_apply_internal")
    return float(ms.value)


TUNE_VARIANTS = [4, 8, 16, 32, 64, 1004, 1008, 1016, 1032, 1064, 2004, 2008, 2016, 2032, 2064,
                 3004, 3008, 3016, 3032, 3064, 4064, 4032]
SELL_CODE = 4064  # sliced copies (the diagonal blocks; the lower blocks too with sliced_lower), 16-bit offsets
SELL32_CODE = 4032  # the same copy with 32-bit columns (MSKM_OP_DIAG only)


def mskm_autotune(ctx, h, repeats: int = 5) -> np.ndarray:
    """Pick the fastest SpMV variant per operator/precision; returns the
    [3][2][len(TUNE_VARIANTS)] table of mean ms per launch (op, precision, variant)."""
    t = np.zeros(3 * 2 * len(TUNE_VARIANTS), dtype=np.float32)
    _check(lib().mskm_autotune(ctx, h, repeats, t.ctypes.data_as(C.POINTER(C.c_float))), "mskm_autotune")
    return t.reshape(3, 2, len(TUNE_VARIANTS))


def mskm_spmv_width(h, op: int, prec: int = MSKM_PREC_FP64) -> int:
    w = C.c_int32()
    _check(lib().mskm_spmv_width(h, op, prec, C.byref(w)), "mskm_spmv_width")
    return int(w.value)


def mskm_cg_product_time(ctx, h, level: int, prec: int = MSKM_PREC_FP32, repeats: int = 20) -> float:
    """Mean ms per launch of the CG product kernel on one level."""
    ms = C.c_float()
    _check(lib().mskm_cg_product_time(ctx, h, level, prec, repeats, C.byref(ms)), "mskm_cg_product_time")
    return float(ms.value)


def mskm_mr_product_time(ctx, h, level: int, nrhs: int, prec: int = MSKM_PREC_FP32, repeats: int = 10) -> float:
    """Mean ms per launch of the many-right-hand-side CG product on one level."""
    ms = C.c_float()
    _check(lib().mskm_mr_product_time(ctx, h, level, prec, nrhs, repeats, C.byref(ms)), "mskm_mr_product_time")
    return float(ms.value)


def mskm_set_mr_chunk(h, nrhs: int, prec: int, chunk: int) -> None:
    """Pins the many-rhs CG-product chunk width (64, 128, 256 or 512 dividing nrhs)."""
    _check(lib().mskm_set_mr_chunk(h, nrhs, prec, chunk), "mskm_set_mr_chunk")


def mskm_set_spmv_width(h, op: int, prec: int, width: int) -> None:
    _check(lib().mskm_set_spmv_width(h, op, prec, width), "mskm_set_spmv_width")


def mskm_solve_opts_default() -> SolveOpts:
    o = SolveOpts()
    lib().mskm_solve_opts_default(C.byref(o))
    return o


def solve_opts(**kw) -> SolveOpts:
    o = mskm_solve_opts_default()
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


@dataclass
class SolveResult:
    status: int
    report: dict


def mskm_solve(ctx, h, f, alpha, opts: SolveOpts | None = None, nrhs: int = 1) -> SolveResult:
    """alpha = T_L^-1 f. Returns the status (0 or MSKM_ENOCONV) and the report."""
    opts = opts or mskm_solve_opts_default()
    fp, fd = _ptr(f, np.float64)
    ap, ad = _ptr(alpha, np.float64)
    if fd != ad:
        raise ValueError("f and alpha must both be host or both be device arrays")
    o = SolveOpts()
    C.pointer(o)[0] = opts
    o.flags = (o.flags | MSKM_IO_DEVICE) if fd else (o.flags & ~MSKM_IO_DEVICE)
    rep = Report()
    st = _check(lib().mskm_solve(ctx, h, fp, nrhs, C.byref(o), ap, C.byref(rep)), "mskm_solve")
    r = {k: getattr(rep, k) for k, _ in Report._fields_}
    r["cg_iters_last"] = list(rep.cg_iters_last)[: rep.levels]
    return SolveResult(st, r)


def mskm_solve_batch(ctx, hs, fs, alphas, opts: SolveOpts | None = None, nrhs=None):
    """Separately created hierarchies hs solved in the same launches; fs /
    alphas: one [N_g][nrhs_g] array per hierarchy (all host or all device).
    Returns (status, one report dict per hierarchy)."""
    nh = len(hs)
    nrhs = [1] * nh if nrhs is None else list(nrhs)
    opts = opts or mskm_solve_opts_default()
    fps, aps, devs = [], [], set()
    for f, a in zip(fs, alphas):
        fp, fd = _ptr(f, np.float64)
        ap, ad = _ptr(a, np.float64)
        fps.append(fp.value)
        aps.append(ap.value)
        devs |= {fd, ad}
    if len(devs) != 1:
        raise ValueError("f and alpha arrays must all be host or all be device arrays")
    o = SolveOpts()
    C.pointer(o)[0] = opts
    o.flags = (o.flags | MSKM_IO_DEVICE) if devs.pop() else (o.flags & ~MSKM_IO_DEVICE)
    reps = (Report * nh)()
    hv = (C.c_void_p * nh)(*[h.value if isinstance(h, C.c_void_p) else h for h in hs])
    st = _check(lib().mskm_solve_batch(ctx, hv, nh, (C.c_void_p * nh)(*fps), (C.c_int32 * nh)(*nrhs), C.byref(o),
                                       (C.c_void_p * nh)(*aps), reps), "mskm_solve_batch")
    out = []
    for g in range(nh):
        r = {k: getattr(reps[g], k) for k, _ in Report._fields_}
        r["cg_iters_last"] = list(reps[g].cg_iters_last)[: reps[g].levels]
        out.append(r)
    return st, out


def mskm_residual(ctx, h, alpha, f, nrhs: int = 1) -> np.ndarray:
    """Relative FP64 residual per right-hand side and group: [nrhs * ngroups]."""
    ap, ad = _ptr(alpha, np.float64)
    fp, fd = _ptr(f, np.float64)
    if fd != ad:
        raise ValueError("alpha and f must both be host or both be device arrays")
    out = np.zeros(nrhs * mskm_hier_stats_get(h)["ngroups"], dtype=np.float64)
    _check(lib().mskm_residual(ctx, h, ap, fp, nrhs, out.ctypes.data_as(C.POINTER(C.c_double)),
                               MSKM_IO_DEVICE if ad else 0), "mskm_residual")
    return out


def mskm_residual_noalloc(ctx, h, alpha, f, rel_out, nrhs: int = 1) -> None:
    """Allocation-free residual: alpha, f [N][nrhs] and rel_out [nrhs * ngroups]
    are device tensors; enqueued on the context's stream (no host wait)."""
    ap, ad = _ptr(alpha, np.float64)
    fp, fd = _ptr(f, np.float64)
    op, od = _ptr(rel_out, np.float64)
    if not (ad and fd and od):
        raise ValueError("alpha, f and rel_out must be device tensors")
    _check(lib().mskm_residual_noalloc(ctx, h, ap, fp, nrhs, op), "mskm_residual_noalloc")


# ------------------------------------------------------- thresholded Jacobi

def mskm_trunc_create(ctx, h, T: float, cg_rtol: float = 1e-13):
    """Truncated Lagrange blocks X~_kj(T) of hierarchy h (status, handle)."""
    out = C.c_void_p()
    st = _check(lib().mskm_trunc_create(ctx, h, float(T), float(cg_rtol), C.byref(out)), "mskm_trunc_create")
    return st, out


def mskm_trunc_destroy(t) -> None:
    _check(lib().mskm_trunc_destroy(t), "mskm_trunc_destroy")


def mskm_trunc_info(t, levels: int) -> dict:
    q = np.zeros(levels, dtype=np.float64)
    nnz, it, ms = C.c_int64(), C.c_int64(), C.c_double()
    _check(lib().mskm_trunc_info(t, C.c_void_p(q.ctypes.data), C.byref(nnz), C.byref(it), C.byref(ms)),
           "mskm_trunc_info")
    return {"q": q, "nnz": int(nnz.value), "cg_iters": int(it.value), "build_ms": float(ms.value)}


def mskm_trunc_export_block(ctx, t, row_level: int, col_level: int, n_rows: int):
    """Canonical CSR (rowptr, col, val) of X~_{row,col}; n_rows = points of row_level."""
    nnz = C.c_int64()
    _check(lib().mskm_trunc_export_block(ctx, t, row_level, col_level, None, None, None, C.byref(nnz)),
           "trunc export (size)")
    n = nnz.value
    rowptr = np.zeros(n_rows + 1, dtype=np.int64)
    col = np.zeros(max(n, 1), dtype=np.int32)
    val = np.zeros(max(n, 1), dtype=np.float64)
    _check(lib().mskm_trunc_export_block(ctx, t, row_level, col_level, C.c_void_p(rowptr.ctypes.data),
                                         C.c_void_p(col.ctypes.data), C.c_void_p(val.ctypes.data), C.byref(nnz)),
           "mskm_trunc_export_block")
    return rowptr, col[:n], val[:n]


def mskm_trunc_solve(ctx, t, f, alpha, opts: SolveOpts | None = None) -> SolveResult:
    """alpha~ of the perturbed split (with refinement when opts.target_rel_residual > 0)."""
    opts = opts or mskm_solve_opts_default()
    fp, fd = _ptr(f, np.float64)
    ap, ad = _ptr(alpha, np.float64)
    if fd != ad:
        raise ValueError("f and alpha must both be host or both be device arrays")
    o = SolveOpts()
    C.pointer(o)[0] = opts
    o.flags = (o.flags | MSKM_IO_DEVICE) if fd else (o.flags & ~MSKM_IO_DEVICE)
    rep = Report()
    st = _check(lib().mskm_trunc_solve(ctx, t, fp, C.byref(o), ap, C.byref(rep)), "mskm_trunc_solve")
    r = {k: getattr(rep, k) for k, _ in Report._fields_}
    r["cg_iters_last"] = list(rep.cg_iters_last)[: rep.levels]
    return SolveResult(st, r)


def mskm_evaluate(ctx, h, alpha, query, out, nrhs: int = 1) -> None:
    ap, ad = _ptr(alpha, np.float64)
    qp, qd = _ptr(query, np.float64)
    op, od = _ptr(out, np.float64)
    if not (ad == qd == od):
        raise ValueError("alpha, query and out must all be host or all be device arrays")
    nq = int(query.shape[0])
    _check(lib().mskm_evaluate(ctx, h, ap, nrhs, qp, nq, op, MSKM_IO_DEVICE if ad else 0), "mskm_evaluate")


# ------------------------------------------------------- learned warm start

def mskm_mlp_train(ctx, h, f, nrhs: int, samples: int = 20000, steps: int = 2000, lr: float = 1e-3,
                   seed: int = 5000, cg_rtol: float = 1e-10):
    """Train the warm-start network on pairs from plain solves of f [N][nrhs];
    returns (mlp handle, loss log every 50 steps)."""
    fp, fd = _ptr(f, np.float64)
    d = TrainDesc(h.value if isinstance(h, C.c_void_p) else h, fp.value, nrhs, samples, steps, lr, seed, cg_rtol,
                  MSKM_IO_DEVICE if fd else 0)
    out = C.c_void_p()
    log = np.zeros((steps + 49) // 50, dtype=np.float32)
    _check(lib().mskm_mlp_train(ctx, C.byref(d), C.byref(out), log.ctypes.data_as(C.POINTER(C.c_float))),
           "mskm_mlp_train")
    return out, log


def mskm_mlp_fit(ctx, m, X, y, steps: int, lr: float = 1e-3) -> np.ndarray:
    """Adam on caller-given samples (X [ns][F] float32, y [ns] float32, numpy
    or CUDA tensors); updates the network in place and returns the loss of
    every mini-batch."""
    if _is_torch(X):
        import torch

        if X.dtype != torch.float32 or y.dtype != torch.float32 or not (X.is_contiguous() and y.is_contiguous()):
            raise TypeError("X and y must be contiguous float32 tensors")
        xp, yp, dev = C.c_void_p(X.data_ptr()), C.c_void_p(y.data_ptr()), X.is_cuda
        if y.is_cuda != dev:
            raise ValueError("X and y must both be host or both be device arrays")
    else:
        X = np.ascontiguousarray(X, dtype=np.float32)
        y = np.ascontiguousarray(y, dtype=np.float32)
        xp, yp, dev = C.c_void_p(X.ctypes.data), C.c_void_p(y.ctypes.data), False
    log = np.zeros(steps, dtype=np.float32)
    _check(lib().mskm_mlp_fit(ctx, m, xp, yp, int(X.shape[0]), steps, lr, MSKM_IO_DEVICE if dev else 0,
                              log.ctypes.data_as(C.POINTER(C.c_float))), "mskm_mlp_fit")
    return log


def mlp_params(m) -> np.ndarray:
    """Flat FP32 parameters (W1, b1, w2, b2) of a network, from its saved blob."""
    return np.frombuffer(mskm_mlp_save(m)[20:], dtype=np.float32).copy()


def mskm_mlp_destroy(m) -> None:
    lib().mskm_mlp_destroy(m)


def mskm_mlp_save(m) -> bytes:
    n = C.c_size_t()
    _check(lib().mskm_mlp_save(m, None, C.byref(n)), "mskm_mlp_save (size)")
    buf = C.create_string_buffer(n.value)
    _check(lib().mskm_mlp_save(m, buf, C.byref(n)), "mskm_mlp_save")
    return buf.raw[: n.value]


def mskm_mlp_load(ctx, blob: bytes):
    out = C.c_void_p()
    buf = C.create_string_buffer(blob, len(blob))
    _check(lib().mskm_mlp_load(ctx, buf, len(blob), C.byref(out)), "mskm_mlp_load")
    return out


def mlp_blob(dim: int, W1: np.ndarray, b1: np.ndarray, w2: np.ndarray, b2: float) -> bytes:
    """Weight blob in the library's MSKMMLP1 layout."""
    F = W1.shape[1]
    hdr = np.array([dim, F, W1.shape[0]], dtype=np.int32).tobytes()
    body = np.concatenate([W1.ravel(), b1, w2, [b2]]).astype(np.float32).tobytes()
    return b"MSKMMLP1" + hdr + body


def mskm_mlp_predict(ctx, h, m, b, x0) -> None:
    bp, bd = _ptr(b, np.float64)
    xp, xd = _ptr(x0, np.float64)
    if bd != xd:
        raise ValueError("b and x0 must both be host or both be device arrays")
    _check(lib().mskm_mlp_predict(ctx, h, m, bp, xp, MSKM_IO_DEVICE if bd else 0), "mskm_mlp_predict")


def mskm_knn_export(ctx, h, level: int) -> np.ndarray:
    n = int(mskm_hier_level_info(h, level)["n"])
    out = np.zeros((max(n, 1), 16), dtype=np.int32)
    _check(lib().mskm_knn_export(ctx, h, level, C.c_void_p(out.ctypes.data)), "mskm_knn_export")
    return out[:n]
