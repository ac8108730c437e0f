"""The compactly supported blocks B_{k,j} of Section 3 as canonical CSR.

B_{k,j} has one row per point of level k (the evaluation level) and one
column per point of level j (the centre level); entry (i, l) is
phi(||x_i^(k) - x_l^(j)|| / delta_j) with the support radius of the *centre*
level. A pair is a structural nonzero iff its squared distance is strictly
below delta_j^2 (closed ball vs open ball does not change values since
phi(1) = 0, but it fixes the structure when exact ties occur, as on grids).

Canonical CSR: rows in input order, columns ascending within a row,
``rowptr`` int64, ``col`` int32 (column index within level j), ``val`` FP64.

Two independent searches produce it: ``block_bruteforce`` tests every pair;
``block_cells`` buckets the centres into cells of side slightly above delta
and tests only the 3^d cells around each row point. The tests require the two
to agree bit for bit.
"""
from __future__ import annotations

import numpy as np

from .wendland import phi31


def sqdist_pairs(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Squared distances of matched rows a[i], b[i]: left to right, no fusion."""
    d2 = None
    for ax in range(a.shape[1]):
        dx = a[:, ax] - b[:, ax]
        sq = dx * dx
        d2 = sq if d2 is None else d2 + sq
    return d2


def _sqdist_dense(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """All squared distances a[i] to b[l], same operation order as sqdist_pairs."""
    d2 = None
    for ax in range(a.shape[1]):
        dx = a[:, None, ax] - b[None, :, ax]
        sq = dx * dx
        d2 = sq if d2 is None else d2 + sq
    return d2


def _to_csr(nrows: int, ri: np.ndarray, ci: np.ndarray, d2: np.ndarray, delta: float):
    """Sort pairs by (row, col) and build canonical CSR with phi values."""
    order = np.lexsort((ci, ri))
    ri, ci, d2 = ri[order], ci[order], d2[order]
    rowptr = np.zeros(nrows + 1, dtype=np.int64)
    np.cumsum(np.bincount(ri, minlength=nrows), out=rowptr[1:])
    val = phi31(np.sqrt(d2) / delta)
    return rowptr, ci.astype(np.int32), val


def block_bruteforce(rows: np.ndarray, cols: np.ndarray, delta: float, chunk_pairs: int = 1 << 22):
    """Canonical CSR of one block by testing every (row, column) pair."""
    rows = np.ascontiguousarray(rows, dtype=np.float64)
    cols = np.ascontiguousarray(cols, dtype=np.float64)
    d2max = delta * delta
    nr, nc = rows.shape[0], cols.shape[0]
    step = max(1, chunk_pairs // max(nc, 1))
    RI, CI, D2 = [], [], []
    for s in range(0, nr, step):
        d2 = _sqdist_dense(rows[s:s + step], cols)
        i, l = np.nonzero(d2 < d2max)
        RI.append(i + s)
        CI.append(l)
        D2.append(d2[i, l])
    if nr == 0:
        return np.zeros(1, np.int64), np.zeros(0, np.int32), np.zeros(0)
    return _to_csr(nr, np.concatenate(RI), np.concatenate(CI), np.concatenate(D2), delta)


def block_cells(rows: np.ndarray, cols: np.ndarray, delta: float, chunk_rows: int = 1 << 15):
    """Canonical CSR of one block through a cell-bucket search.

    Centres are bucketed into cells of side c = delta*(1 + 1e-6). For two
    points closer than delta the computed cell coordinates floor((x-lo)/c)
    differ by at most one on every axis: the real quotients differ by less
    than 1/(1+1e-6) and the rounding of (x-lo)/c is below 1e-12 for
    coordinates of moderate size. So the 3^d cells around a row point's cell
    contain every centre within delta of it.
    """
    rows = np.ascontiguousarray(rows, dtype=np.float64)
    cols = np.ascontiguousarray(cols, dtype=np.float64)
    nr, nc, d = rows.shape[0], cols.shape[0], cols.shape[1]
    if nr == 0 or nc == 0:
        return np.zeros(nr + 1, np.int64), np.zeros(0, np.int32), np.zeros(0)
    d2max = delta * delta
    c = delta * (1.0 + 1e-6)
    lo = cols.min(axis=0)
    ncell = np.floor((cols.max(axis=0) - lo) / c).astype(np.int64) + 1
    ccell = np.floor((cols - lo) / c).astype(np.int64)
    stride = np.ones(d, dtype=np.int64)
    for ax in range(1, d):
        stride[ax] = stride[ax - 1] * ncell[ax - 1]
    key = (ccell * stride).sum(axis=1)
    order = np.argsort(key, kind="stable")
    skey = key[order]
    total = int(np.prod(ncell))
    start = np.searchsorted(skey, np.arange(total + 1))
    offsets = np.stack(np.meshgrid(*([np.arange(-1, 2)] * d), indexing="ij"), -1).reshape(-1, d)
    RI, CI, D2 = [], [], []
    for s in range(0, nr, chunk_rows):
        pr = rows[s:s + chunk_rows]
        rcell = np.floor((pr - lo) / c).astype(np.int64)
        for off in offsets:
            nb = rcell + off
            ok = np.all((nb >= 0) & (nb < ncell), axis=1)
            ridx = np.nonzero(ok)[0]
            if ridx.size == 0:
                continue
            k = (nb[ridx] * stride).sum(axis=1)
            a, b = start[k], start[k + 1]
            cnt = b - a
            tot = int(cnt.sum())
            if tot == 0:
                continue
            rr = np.repeat(ridx, cnt)
            first = np.repeat(a - np.concatenate(([0], np.cumsum(cnt)[:-1])), cnt)
            cc = order[first + np.arange(tot)]
            d2 = sqdist_pairs(pr[rr], cols[cc])
            keep = d2 < d2max
            RI.append(rr[keep] + s)
            CI.append(cc[keep])
            D2.append(d2[keep])
    if not RI:
        return np.zeros(nr + 1, np.int64), np.zeros(0, np.int32), np.zeros(0)
    return _to_csr(nr, np.concatenate(RI), np.concatenate(CI), np.concatenate(D2), delta)
