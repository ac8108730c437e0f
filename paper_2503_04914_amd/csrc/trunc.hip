// Thresholded Jacobi on gfx950 (Section 4, "Thresholding"): the explicit,
// truncated blocks of M = I - T' and the perturbed split they define.
//
// For levels k > j of one hierarchy the block of T' is frak X_{kj} =
// B_{kj} A_j^-1: entry (i, n) is chi_n^(j)(x_i^(k)), the Lagrange function of
// centre n of level j (coefficients A_j^-1 e_n) evaluated at point i of level
// k. The truncated block frak X~_{kj}(T) keeps the entries whose points lie
// closer than T q_j, q_j = the separation distance of level j (half the
// smallest distance between two of its points), and drops the rest
// (eq. (perturbedmatrix)); the perturbed split (eq. (perturbed_split)) then
// needs one product with these blocks per Jacobi sweep and no inner solve.
//
// Construction, all on the device:
//   1. q_j from the diagonal block's pairs (every pair closer than delta_j is
//      stored there); a level whose points are all further apart than
//      delta_j falls back to a test of all pairs;
//   2. the pattern: for every row point, the level-j points within T q_j,
//      searched over a window of cells of level j's grid (a count pass, a
//      scan, a fill pass; columns ascending, rows like the lower CSR: level
//      0's columns first, then level 1's, ...);
//   3. the values: A_j^-1 e_n for chunks of up to 512 centres n by CG with
//      many right-hand sides, then chi_n(x_i) = sum_m B_kj[i][m] (A_j^-1
//      e_n)[m] for every kept entry (i, n) whose centre lies in the chunk.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>

#include "device_common.h"

namespace mskm {

// ---------------------------------------------------- separation distance

// Smallest squared distance of a row point to the other points of its own
// row of the diagonal block, reduced per level by an atomic minimum on the
// FP64 bit pattern (non-negative doubles order like their bits).
__global__ void __launch_bounds__(kBlock)
    k_sep_min(int dim, int64_t r0, int64_t r1, const double* __restrict__ xs, int64_t N,
              const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
              unsigned long long* __restrict__ out) {
  const int64_t i = r0 + (int64_t)blockIdx.x * kBlock + threadIdx.x;
  double m = std::numeric_limits<double>::infinity();
  if (i < r1) {
    const double px = xs[i], py = xs[N + i], pz = dim == 3 ? xs[2 * N + i] : 0.0;
    for (int64_t k = rp[i]; k < rp[i + 1]; ++k) {
      const int64_t c = col[k];
      if (c == i) continue;
      const double d2 = sqdist(dim, px, py, pz, xs[c], xs[N + c], dim == 3 ? xs[2 * N + c] : 0.0);
      m = d2 < m ? d2 : m;
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const double u = __shfl_xor(m, o, kWave);
    m = u < m ? u : m;
  }
  if (threadIdx.x % kWave == 0 && m < std::numeric_limits<double>::infinity())
    atomicMin(out, (unsigned long long)__double_as_longlong(m));
}

// The same over all pairs of one level (levels whose diagonal block has no
// off-diagonal entry).
__global__ void __launch_bounds__(kBlock)
    k_sep_all_pairs(int dim, int64_t off, int64_t n, const double* __restrict__ xs, int64_t N,
                    unsigned long long* __restrict__ out) {
  const int64_t i = off + (int64_t)blockIdx.x * kBlock + threadIdx.x;
  double m = std::numeric_limits<double>::infinity();
  if (i < off + n) {
    const double px = xs[i], py = xs[N + i], pz = dim == 3 ? xs[2 * N + i] : 0.0;
    for (int64_t c = off; c < off + n; ++c) {
      if (c == i) continue;
      const double d2 = sqdist(dim, px, py, pz, xs[c], xs[N + c], dim == 3 ? xs[2 * N + c] : 0.0);
      m = d2 < m ? d2 : m;
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const double u = __shfl_xor(m, o, kWave);
    m = u < m ? u : m;
  }
  if (threadIdx.x % kWave == 0 && m < std::numeric_limits<double>::infinity())
    atomicMin(out, (unsigned long long)__double_as_longlong(m));
}

// ------------------------------------------------------------- pattern

// Per centre level: the squared truncation radius (T q_j)^2 (infinite: keep
// every point) and the half-width of the window of cells that holds every
// point within T q_j of a cell.
struct TruncLev {
  double r2;
  int32_t w;
  int32_t pad;
};

// Visits the points of level j within sqrt(r2) of (px, py, pz) in ascending
// internal index: cell rows of the window in key order, each one contiguous
// range of points.
template <typename F>
__device__ __forceinline__ void for_each_in_radius(int dim, const DevLevel& Lj, const TruncLev& tj,
                                                   const int32_t* __restrict__ cs_all, const double* __restrict__ xs,
                                                   int64_t N, double px, double py, double pz, F&& f) {
  if (Lj.n == 0) return;
  const int cx = cell_coord(px, Lj.lo[0], Lj.inv_cell, Lj.nc[0]);
  const int cy = cell_coord(py, Lj.lo[1], Lj.inv_cell, Lj.nc[1]);
  const int cz = dim == 3 ? cell_coord(pz, Lj.lo[2], Lj.inv_cell, Lj.nc[2]) : 0;
  const int w = tj.w;
  const int x0 = max(cx - w, 0), x1 = min(cx + w, Lj.nc[0] - 1);
  const int y0 = max(cy - w, 0), y1 = min(cy + w, Lj.nc[1] - 1);
  const int z0 = dim == 3 ? max(cz - w, 0) : 0, z1 = dim == 3 ? min(cz + w, Lj.nc[2] - 1) : 0;
  const int32_t* cs = cs_all + Lj.cs_off;
  for (int z = z0; z <= z1; ++z)
    for (int y = y0; y <= y1; ++y) {
      const int rk = (z * Lj.nc[1] + y) * Lj.nc[0];
      for (int64_t t = cs[rk + x0]; t < cs[rk + x1 + 1]; ++t) {
        const double d2 = sqdist(dim, px, py, pz, xs[t], xs[N + t], dim == 3 ? xs[2 * N + t] : 0.0);
        if (d2 < tj.r2) f(t);
      }
    }
}

// COUNT (out == nullptr): cnt[i - r0] = kept entries of row i over every
// coarser level of its hierarchy. FILL: their columns at rp[i].
__global__ void __launch_bounds__(kBlock)
    k_trunc_rows(int dim, int k, int64_t r0, int64_t r1, const DevLevel* __restrict__ lev,
                 const TruncLev* __restrict__ tl, const int32_t* __restrict__ cs_all, const double* __restrict__ xs,
                 int64_t N, int64_t* __restrict__ cnt, const int64_t* __restrict__ rp, int32_t* __restrict__ out) {
  const int64_t i = r0 + (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= r1) return;
  const double px = xs[i], py = xs[N + i], pz = dim == 3 ? xs[2 * N + i] : 0.0;
  int64_t c = 0;
  int64_t pos = out ? rp[i] : 0;
  for (int j = lev[k].first; j != k && j >= 0; j = lev[j].next) {
    const DevLevel Lj = lev[j];
    const TruncLev tj = tl[j];
    if (out)
      for_each_in_radius(dim, Lj, tj, cs_all, xs, N, px, py, pz, [&](int64_t t) { out[pos++] = (int32_t)t; });
    else
      for_each_in_radius(dim, Lj, tj, cs_all, xs, N, px, py, pz, [&](int64_t) { ++c; });
  }
  if (!out) cnt[i - r0] = c;
}

// -------------------------------------------------------------- values

// First position in [a, e) of the ascending array col whose value is >= v.
__device__ __forceinline__ int64_t lower_bound_col(const int32_t* __restrict__ col, int64_t a, int64_t e, int64_t v) {
  while (a < e) {
    const int64_t m = a + (e - a) / 2;
    if ((int64_t)col[m] < v) a = m + 1;
    else e = m;
  }
  return a;
}

// For rows i of level k: every kept entry (i, n) with centre n in the chunk
// [c0, c0 + R) of level j's internal indices gets
//   X[i][n] = sum over the lower CSR's level-j entries (m, b) of row i of
//             b * Z[m][n - c0],
// Z [N][R] holding A_j^-1 e_n for the chunk's centres (rows of level j).
__global__ void __launch_bounds__(kBlock)
    k_trunc_values(int64_t r0, int64_t r1, int64_t j0, int64_t j1, int64_t c0, int R,
                   const int64_t* __restrict__ lrp, const int32_t* __restrict__ lcol, const double* __restrict__ lval,
                   const double* __restrict__ Z, const int64_t* __restrict__ xrp, const int32_t* __restrict__ xcol,
                   double* __restrict__ xval) {
  const int64_t i = r0 + (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= r1) return;
  // kept entries of row i in the chunk
  const int64_t xa = xrp[i], xe = xrp[i + 1];
  if (xa == xe || (int64_t)xcol[xe - 1] < c0 || (int64_t)xcol[xa] >= c0 + R) return;
  const int64_t ea = lower_bound_col(xcol, xa, xe, c0);
  const int64_t ee = lower_bound_col(xcol, ea, xe, c0 + R);
  if (ea == ee) return;
  // row i's entries of B_kj in the lower CSR
  const int64_t la = lower_bound_col(lcol, lrp[i], lrp[i + 1], j0);
  const int64_t le = lower_bound_col(lcol, la, lrp[i + 1], j1);
  for (int64_t e = ea; e < ee; ++e) {
    const int64_t r = (int64_t)xcol[e] - c0;
    double acc = 0.0;
    for (int64_t k = la; k < le; ++k) acc += lval[k] * Z[(int64_t)lcol[k] * R + r];
    xval[e] = acc;
  }
}

namespace {

unsigned grid_rows(int64_t n) { return (unsigned)std::max<int64_t>(1, (n + kBlock - 1) / kBlock); }

struct Scratch {
  std::vector<void*> p;
  ~Scratch() {
    for (void* q : p) (void)hipFree(q);
  }
  template <typename T>
  mskm_status get(T** out, size_t count) {
    MSKM_TRY(dalloc(out, count));
    p.push_back(*out);
    return MSKM_OK;
  }
};

}  // namespace

mskm_status trunc_build(mskm_hier* h, double T, double cg_rtol, mskm_trunc* tr) {
  hipStream_t s = h->ctx->stream;
  const int L = h->L;
  const int64_t N = h->N;
  const int dim = h->dim;
  if (!h->lower.val || !h->diag.val) return fail(MSKM_ESTATE, "thresholded blocks need the FP64 block values");
  Scratch sc;
  MSKM_HIP_TRY(hipEventRecord(h->ctx->ev0, s));
  // 1. separation distances
  unsigned long long* dmin = nullptr;
  MSKM_TRY(sc.get(&dmin, L));
  const double inf = std::numeric_limits<double>::infinity();
  unsigned long long inf_bits = 0;
  std::memcpy(&inf_bits, &inf, 8);
  std::vector<unsigned long long> hmin(L, inf_bits);
  auto as_double = [](unsigned long long b) {
    double d;
    std::memcpy(&d, &b, 8);
    return d;
  };
  MSKM_HIP_TRY(hipMemcpyAsync(dmin, hmin.data(), L * 8, hipMemcpyHostToDevice, s));
  for (int l = 0; l < L; ++l) {
    const int64_t n = h->h_off[l + 1] - h->h_off[l];
    if (n >= 2)
      hipLaunchKernelGGL(k_sep_min, dim3(grid_rows(n)), dim3(kBlock), 0, s, dim, h->h_off[l], h->h_off[l + 1], h->xs, N,
                         h->diag.rowptr, h->diag.col, dmin + l);
  }
  MSKM_HIP_TRY(hipMemcpyAsync(hmin.data(), dmin, L * 8, hipMemcpyDeviceToHost, s));
  MSKM_HIP_TRY(hipStreamSynchronize(s));
  bool again = false;
  for (int l = 0; l < L; ++l) {
    const int64_t n = h->h_off[l + 1] - h->h_off[l];
    if (n >= 2 && as_double(hmin[l]) == inf) {
      if (n > (1 << 16))
        return fail(MSKM_ELIMIT, "level " + std::to_string(l) +
                                     ": no two points closer than its support radius, and too many points (> 65536) "
                                     "to search all pairs for the separation distance");
      hipLaunchKernelGGL(k_sep_all_pairs, dim3(grid_rows(n)), dim3(kBlock), 0, s, dim, h->h_off[l], n, h->xs, N, dmin + l);
      again = true;
    }
  }
  if (again) {
    MSKM_HIP_TRY(hipMemcpyAsync(hmin.data(), dmin, L * 8, hipMemcpyDeviceToHost, s));
    MSKM_HIP_TRY(hipStreamSynchronize(s));
  }
  tr->q.assign(L, inf);
  tr->r2.assign(L, inf);
  std::vector<TruncLev> ht(L);
  for (int l = 0; l < L; ++l) {
    const int64_t n = h->h_off[l + 1] - h->h_off[l];
    const DevLevel& D = h->h_lev[l];
    int32_t wmax = std::max(std::max(D.nc[0], D.nc[1]), D.nc[2]);
    if (n >= 2) tr->q[l] = 0.5 * std::sqrt(as_double(hmin[l]));
    const double R = T * tr->q[l];
    tr->r2[l] = R * R;
    ht[l].r2 = tr->r2[l];
    // every point within R lies at most floor(R / cell) + 1 cells away
    const double wc = std::floor(R * D.inv_cell) + 1.0;
    ht[l].w = std::isfinite(wc) && wc < (double)wmax ? (int32_t)wc : wmax;
  }
  TruncLev* dtl = nullptr;
  MSKM_TRY(sc.get(&dtl, L));
  MSKM_HIP_TRY(hipMemcpyAsync(dtl, ht.data(), L * sizeof(TruncLev), hipMemcpyHostToDevice, s));

  // 2. pattern: count, scan, fill
  int64_t *cnt = nullptr, *part = nullptr;
  MSKM_TRY(sc.get(&cnt, N + 1));
  MSKM_TRY(sc.get(&part, scan_parts(N + 1)));
  MSKM_HIP_TRY(hipMemsetAsync(cnt, 0, (N + 1) * 8, s));
  for (int l = 0; l < L; ++l) {
    const int64_t n = h->h_off[l + 1] - h->h_off[l];
    if (n == 0 || h->h_depth[l] == 0) continue;
    hipLaunchKernelGGL(k_trunc_rows, dim3(grid_rows(n)), dim3(kBlock), 0, s, dim, l, h->h_off[l], h->h_off[l + 1],
                       h->d_lev, dtl, h->cell_start, h->xs, N, cnt + h->h_off[l], nullptr, nullptr);
  }
  MSKM_TRY(tr_alloc(tr, &tr->X.rowptr, N + 1));
  MSKM_TRY(exclusive_scan_i64(s, cnt, tr->X.rowptr, N + 1, part));
  int64_t nnz = 0;
  MSKM_HIP_TRY(hipMemcpyAsync(&nnz, tr->X.rowptr + N, 8, hipMemcpyDeviceToHost, s));
  MSKM_HIP_TRY(hipStreamSynchronize(s));
  if (nnz >= ((int64_t)1 << 40)) return fail(MSKM_ELIMIT, "truncated blocks too large");
  tr->X.nnz = nnz;
  MSKM_TRY(tr_alloc(tr, &tr->X.col, (size_t)nnz + kCsrPad));
  MSKM_TRY(tr_alloc(tr, &tr->X.val, (size_t)nnz + kCsrPad));
  MSKM_HIP_TRY(hipMemsetAsync(tr->X.col, 0, ((size_t)nnz + kCsrPad) * 4, s));
  MSKM_HIP_TRY(hipMemsetAsync(tr->X.val, 0, ((size_t)nnz + kCsrPad) * 8, s));
  for (int l = 0; l < L; ++l) {
    const int64_t n = h->h_off[l + 1] - h->h_off[l];
    if (n == 0 || h->h_depth[l] == 0) continue;
    hipLaunchKernelGGL(k_trunc_rows, dim3(grid_rows(n)), dim3(kBlock), 0, s, dim, l, h->h_off[l], h->h_off[l + 1],
                       h->d_lev, dtl, h->cell_start, h->xs, N, nullptr, tr->X.rowptr, tr->X.col);
  }

  // 3. values, centre level by centre level, chunks of up to 512 centres
  constexpr int kChunk = 512;
  double* Z = nullptr;
  const int64_t maxn = [&] {
    int64_t m = 0;
    for (int l = 0; l < L; ++l)
      if (h->h_next[l] >= 0) m = std::max(m, h->h_off[l + 1] - h->h_off[l]);
    return m;
  }();
  const int R = (int)std::max<int64_t>(1, std::min<int64_t>(kChunk, maxn));
  if (nnz > 0 && maxn > 0) MSKM_TRY(sc.get(&Z, (size_t)N * R));
  tr->cg_iters = 0;
  tr->capped = false;
  for (int j = 0; j < L && nnz > 0; ++j) {
    if (h->h_next[j] < 0) continue;  // no finer level: no block has centres here
    const int64_t nj = h->h_off[j + 1] - h->h_off[j];
    for (int64_t n0 = 0; n0 < nj; n0 += R) {
      int64_t it = 0;
      bool capped = false;
      MSKM_TRY(lagrange_columns(h, j, n0, R, cg_rtol, 20000, Z, &it, &capped));
      tr->cg_iters += it;
      tr->capped |= capped;
      for (int k = h->h_next[j]; k >= 0; k = h->h_next[k]) {
        const int64_t nk = h->h_off[k + 1] - h->h_off[k];
        if (nk == 0) continue;
        hipLaunchKernelGGL(k_trunc_values, dim3(grid_rows(nk)), dim3(kBlock), 0, s, h->h_off[k], h->h_off[k + 1],
                           h->h_off[j], h->h_off[j + 1], h->h_off[j] + n0, R, h->lower.rowptr, h->lower.col,
                           h->lower.val, Z, tr->X.rowptr, tr->X.col, tr->X.val);
      }
    }
  }
  MSKM_HIP_TRY(hipEventRecord(h->ctx->ev1, s));
  MSKM_HIP_TRY(hipStreamSynchronize(s));
  float ms = 0.f;
  MSKM_HIP_TRY(hipEventElapsedTime(&ms, h->ctx->ev0, h->ctx->ev1));
  tr->build_ms = ms;
  MSKM_HIP_TRY(hipGetLastError());
  return MSKM_OK;
}

}  // namespace mskm
