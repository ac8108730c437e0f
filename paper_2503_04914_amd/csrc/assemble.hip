// Hierarchy assembly on gfx950: cell lists per level, neighbour search for
// every level pair k >= j and evaluation of the Wendland blocks
// B_{k,j}[i][n] = phi(||x_i^(k) - x_n^(j)|| / delta_j) (Section 3) into CSR.
//
// Pipeline (all on the context stream):
//   bbox per level -> cell key per point -> histogram -> scan -> scatter ->
//   in-cell rank by input index (deterministic order) -> SoA coordinates ->
//   count pass (one wave per row, lanes over candidate cells) -> int64 scan ->
//   fill pass (same traversal; ballot/popcount gives each hit its slot, so
//   columns come out ascending and writes are contiguous per row).
#include <algorithm>
#include <cmath>

#include "device_common.h"

namespace mskm {

// ------------------------------------------------------------------ scans

// Exclusive scan of int64, three passes. Block b scans kScanTile items.
constexpr int kScanItems = 8;
constexpr int kScanTile = kBlock * kScanItems;

__global__ void __launch_bounds__(kBlock) k_scan_partials(const int64_t* __restrict__ in, int64_t n,
                                                          int64_t* __restrict__ part) {
  __shared__ int64_t sm[kBlock / kWave];
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  int64_t s = 0;
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t i = base + (int64_t)k * kBlock + threadIdx.x;
    if (i < n) s += in[i];
  }
  s = block_sum(s, sm);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// Single block: exclusive scan of the partials in place (sequential chunks).
__global__ void __launch_bounds__(kBlock) k_scan_partials_scan(int64_t* __restrict__ part, int64_t nparts) {
  __shared__ int64_t sm[kBlock];
  __shared__ int64_t carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int64_t base = 0; base < nparts; base += kBlock) {
    const int64_t i = base + threadIdx.x;
    const int64_t v = i < nparts ? part[i] : 0;
    sm[threadIdx.x] = v;
    __syncthreads();
    // Hillis-Steele inclusive scan in LDS
    for (int o = 1; o < kBlock; o <<= 1) {
      int64_t t = threadIdx.x >= o ? sm[threadIdx.x - o] : 0;
      __syncthreads();
      sm[threadIdx.x] += t;
      __syncthreads();
    }
    if (i < nparts) part[i] = carry + sm[threadIdx.x] - v;
    __syncthreads();
    if (threadIdx.x == 0) carry += sm[kBlock - 1];
    __syncthreads();
  }
}

__global__ void __launch_bounds__(kBlock) k_scan_final(const int64_t* __restrict__ in, int64_t n,
                                                       const int64_t* __restrict__ part, int64_t* __restrict__ out) {
  __shared__ int64_t sm[kBlock];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  int64_t v[kScanItems];
  int64_t s = 0;
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t i = base + k;
    v[k] = i < n ? in[i] : 0;
    s += v[k];
  }
  sm[threadIdx.x] = s;
  __syncthreads();
  for (int o = 1; o < kBlock; o <<= 1) {
    int64_t t = threadIdx.x >= o ? sm[threadIdx.x - o] : 0;
    __syncthreads();
    sm[threadIdx.x] += t;
    __syncthreads();
  }
  int64_t run = part[blockIdx.x] + sm[threadIdx.x] - s;
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t i = base + k;
    if (i < n) out[i] = run;
    run += v[k];
  }
}

int64_t scan_parts(int64_t n) { return std::max<int64_t>(1, (n + kScanTile - 1) / kScanTile); }

// out[0..n) = exclusive scan of in[0..n), stream-ordered (no host
// synchronisation). in and out may not alias; part is scratch of
// scan_parts(n) entries, free again once the scan's kernels have run.
mskm_status exclusive_scan_i64(hipStream_t s, const int64_t* in, int64_t* out, int64_t n, int64_t* part) {
  if (n <= 0) return MSKM_OK;
  const int64_t nb = scan_parts(n);
  if (nb > (int64_t)INT32_MAX) return fail(MSKM_ELIMIT, "scan too large");
  hipLaunchKernelGGL(k_scan_partials, dim3((unsigned)nb), dim3(kBlock), 0, s, in, n, part);
  hipLaunchKernelGGL(k_scan_partials_scan, dim3(1), dim3(kBlock), 0, s, part, nb);
  hipLaunchKernelGGL(k_scan_final, dim3((unsigned)nb), dim3(kBlock), 0, s, in, n, part, out);
  MSKM_HIP_TRY(hipGetLastError());
  return MSKM_OK;
}


// ------------------------------------------------------------- cell lists

__global__ void __launch_bounds__(kBlock) k_widen(const int32_t* __restrict__ a, int64_t* __restrict__ b, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) b[i] = a[i];
}

__global__ void __launch_bounds__(kBlock) k_narrow(const int64_t* __restrict__ a, int32_t* __restrict__ b, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) b[i] = (int32_t)a[i];
}

constexpr int kBboxBlocks = 128;

// Per-level bounding box of the input points (AoS); level l spans input
// points [rng[2l], rng[2l+1]). Grid (kBboxBlocks, L).
__global__ void __launch_bounds__(kBlock) k_bbox_partial(const double* __restrict__ pts, const int64_t* __restrict__ rng,
                                                         int dim, double* __restrict__ part) {
  __shared__ double smn[3][kBlock], smx[3][kBlock];
  const int l = blockIdx.y;
  const int64_t a = rng[2 * l], b = rng[2 * l + 1];
  double mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int64_t i = a + (int64_t)blockIdx.x * kBlock + threadIdx.x; i < b; i += (int64_t)gridDim.x * kBlock) {
    for (int d = 0; d < dim; ++d) {
      const double v = pts[i * dim + d];
      // NaN propagates into the box (fmin/fmax would drop it): the host rejects it
      mn[d] = (v < mn[d] || v != v) ? v : mn[d];
      mx[d] = (v > mx[d] || v != v) ? v : mx[d];
    }
  }
  for (int d = 0; d < 3; ++d) {
    smn[d][threadIdx.x] = mn[d];
    smx[d][threadIdx.x] = mx[d];
  }
  __syncthreads();
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      for (int d = 0; d < 3; ++d) {
        const double u = smn[d][threadIdx.x + s], w = smx[d][threadIdx.x + s];
        smn[d][threadIdx.x] = (u < smn[d][threadIdx.x] || u != u) ? u : smn[d][threadIdx.x];
        smx[d][threadIdx.x] = (w > smx[d][threadIdx.x] || w != w) ? w : smx[d][threadIdx.x];
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double* o = part + ((size_t)l * gridDim.x + blockIdx.x) * 6;
    for (int d = 0; d < 3; ++d) {
      o[d] = smn[d][0];
      o[3 + d] = smx[d][0];
    }
  }
}

// Cell key of every point of level l (row-major, axis 0 fastest).
__global__ void __launch_bounds__(kBlock) k_cell_key(const double* __restrict__ pts, int dim,
                                                     const DevLevel* __restrict__ lev, int l, int64_t off, int64_t n,
                                                     int32_t* __restrict__ key, int32_t* __restrict__ count) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const DevLevel L = lev[l];
  const int64_t g = off + i;
  int k = 0, stride = 1;
  for (int d = 0; d < dim; ++d) {
    const int c = cell_coord(pts[g * dim + d], L.lo[d], L.inv_cell, L.nc[d]);
    k += c * stride;
    stride *= L.nc[d];
  }
  key[g] = k;
  atomicAdd(&count[L.cs_off + k], 1);
}

// Unordered placement of each point into its cell's slot range.
__global__ void __launch_bounds__(kBlock) k_cell_scatter(const DevLevel* __restrict__ lev, int l, int64_t off,
                                                         int64_t n, const int32_t* __restrict__ key,
                                                         const int64_t* __restrict__ cs, int32_t* __restrict__ cursor,
                                                         int32_t* __restrict__ tmp) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const int64_t g = off + i;
  const int c = lev[l].cs_off + key[g];
  const int pos = atomicAdd(&cursor[c], 1);
  tmp[cs[c] + pos] = (int32_t)g;
}

// Final position = cell start + rank of the input index among the cell's
// points: the in-cell order is ascending input index, independent of the
// order in which the scatter's atomics landed.
__global__ void __launch_bounds__(kBlock) k_cell_rank(const DevLevel* __restrict__ lev, int l, int64_t off,
                                                      int64_t n, int dim, const double* __restrict__ pts,
                                                      const int32_t* __restrict__ key, const int64_t* __restrict__ cs,
                                                      const int32_t* __restrict__ tmp, int32_t* __restrict__ perm,
                                                      int32_t* __restrict__ iperm, double* __restrict__ xs,
                                                      int64_t N) {
  const int64_t s = off + (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (s >= off + n) return;
  const int32_t g = tmp[s];
  const int c = lev[l].cs_off + key[g];
  const int64_t a = cs[c], b = cs[c + 1];
  int64_t rank = 0;
  for (int64_t t = a; t < b; ++t) rank += tmp[t] < g;
  const int64_t p = a + rank;
  perm[p] = g;
  iperm[g] = (int32_t)p;
  for (int d = 0; d < dim; ++d) xs[(size_t)d * N + p] = pts[(size_t)g * dim + d];
}

// ------------------------------------------------------- neighbour search

// Visit every candidate of row point (px, py, pz) in level j's grid: the 3^d
// cells around its cell. With a row-major key the three cells along axis 0
// are one contiguous slot range, so there are 3 ranges in 2-D and 9 in 3-D.
// The callback gets (range begin, range end) in internal global indices.
template <typename F>
__device__ __forceinline__ void for_each_range(int dim, const DevLevel& L, const int32_t* __restrict__ cs_all,
                                               double px, double py, double pz, F&& f) {
  const int cx = cell_coord(px, L.lo[0], L.inv_cell, L.nc[0]);
  const int cy = cell_coord(py, L.lo[1], L.inv_cell, L.nc[1]);
  const int cz = dim == 3 ? cell_coord(pz, L.lo[2], L.inv_cell, L.nc[2]) : 0;
  const int x0 = cx > 0 ? cx - 1 : 0;
  const int x1 = cx < L.nc[0] - 1 ? cx + 1 : L.nc[0] - 1;
  const int z0 = dim == 3 ? (cz > 0 ? cz - 1 : 0) : 0;
  const int z1 = dim == 3 ? (cz < L.nc[2] - 1 ? cz + 1 : L.nc[2] - 1) : 0;
  const int y0 = cy > 0 ? cy - 1 : 0;
  const int y1 = cy < L.nc[1] - 1 ? cy + 1 : L.nc[1] - 1;
  const int32_t* cs = cs_all + L.cs_off;
  for (int z = z0; z <= z1; ++z) {
    for (int y = y0; y <= y1; ++y) {
      const int rowkey = (z * L.nc[1] + y) * L.nc[0];
      f((int64_t)cs[rowkey + x0], (int64_t)cs[rowkey + x1 + 1]);
    }
  }
}

// Neighbour search on LDS-staged cell tiles: a tile is 64 consecutive rows
// of level k; rows in the internal (cell) order are spatial neighbours. For
// every level j of the rows' hierarchy, from the coarsest up to k:
//   * the union of the rows' 3^d neighbour cells in level j's grid is
//     bounded by a box of cell rows; each box row is one contiguous range of
//     level j's points;
//   * when the box holds at most kTileCap points they are staged in LDS
//     (coalesced copies) and the candidates are read from there, else from
//     global memory (same arithmetic, same order);
//   * a row's candidates are its own 3^d cells' points in ascending index
//     order, so its columns come out ascending (canonical CSR).
// COUNT (one row per lane, no writes but the two counts): cnt_d[i] = hits on
// level k, cnt_l[i] = hits on the coarser levels. FILL (one row per wave
// step, ballot compaction): the hits with their phi values at the row's
// CSR positions, as contiguous runs.
constexpr int kTileCap = 768;    // staged points per level
constexpr int kMaxBoxRows = 64;  // cell rows of a stageable box (one lane each)

template <typename T>
__device__ __forceinline__ T wave_min(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const T u = __shfl_xor(v, o, kWave);
    v = u < v ? u : v;
  }
  return v;
}
template <typename T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const T u = __shfl_xor(v, o, kWave);
    v = u > v ? u : v;
  }
  return v;
}

template <int DIM>
__global__ void __launch_bounds__(kWave)
    k_nbr_tile_count(int k, const DevLevel* __restrict__ lev, const int32_t* __restrict__ cs_all,
                     const double* __restrict__ xs, int64_t N, int64_t* __restrict__ cnt_d,
                     int64_t* __restrict__ cnt_l, int32_t* __restrict__ cnt_lv) {
  __shared__ double sx[kTileCap], sy[kTileCap], sz[DIM == 3 ? kTileCap : 1];
  __shared__ int64_t box_a[kMaxBoxRows];
  __shared__ int32_t box_o[kMaxBoxRows];
  const DevLevel Lk = lev[k];
  const int lane = threadIdx.x;
  const int64_t r = (int64_t)blockIdx.x * kWave + lane;
  const bool act = r < Lk.n;
  const int64_t i = Lk.off + (act ? r : 0);
  const double* X = xs;
  const double* Y = xs + N;
  const double* Z = xs + 2 * N;
  const double px = X[i], py = Y[i], pz = DIM == 3 ? Z[i] : 0.0;
  int64_t nd = 0, nl = 0;
  int seg = 0;  // position of level j in the row's hierarchy (the lower segment index)
  for (int j = Lk.first;; j = lev[j].next, ++seg) {
    const DevLevel Lj = lev[j];
    const bool is_diag = j == k;
    const int cx = cell_coord(px, Lj.lo[0], Lj.inv_cell, Lj.nc[0]);
    const int cy = cell_coord(py, Lj.lo[1], Lj.inv_cell, Lj.nc[1]);
    const int cz = DIM == 3 ? cell_coord(pz, Lj.lo[2], Lj.inv_cell, Lj.nc[2]) : 0;
    const int x0 = max(cx - 1, 0), x1 = min(cx + 1, Lj.nc[0] - 1);
    const int y0 = max(cy - 1, 0), y1 = min(cy + 1, Lj.nc[1] - 1);
    const int z0 = DIM == 3 ? max(cz - 1, 0) : 0, z1 = DIM == 3 ? min(cz + 1, Lj.nc[2] - 1) : 0;
    // the tile's box of cell rows (inactive lanes do not widen it)
    const int BX0 = wave_min(act ? x0 : INT32_MAX), BX1 = wave_max(act ? x1 : -1);
    const int BY0 = wave_min(act ? y0 : INT32_MAX), BY1 = wave_max(act ? y1 : -1);
    const int BZ0 = wave_min(act ? z0 : INT32_MAX), BZ1 = wave_max(act ? z1 : -1);
    const int ny = BY1 - BY0 + 1;
    const int nrows = ny * (BZ1 - BZ0 + 1);
    const int32_t* cs = cs_all + Lj.cs_off;
    const bool boxed = nrows >= 1 && nrows <= kMaxBoxRows;
    bool staged = false;
    if (boxed) {
      int64_t a = 0, len = 0;
      if (lane < nrows) {
        const int yy = BY0 + lane % ny, zz = BZ0 + lane / ny;
        const int rk = (zz * Lj.nc[1] + yy) * Lj.nc[0];
        a = cs[rk + BX0];
        len = cs[rk + BX1 + 1] - a;
      }
      // exclusive scan of the box rows' lengths
      int64_t incl = len;
#pragma unroll
      for (int o = 1; o < kWave; o <<= 1) {
        const int64_t u = __shfl_up(incl, o, kWave);
        if (lane >= o) incl += u;
      }
      const int64_t total = __shfl(incl, kWave - 1, kWave);
      if (lane < nrows) {
        box_a[lane] = a;
        box_o[lane] = (int32_t)(incl - len);
      }
      staged = total <= kTileCap;
      __syncthreads();
      if (staged) {
        for (int q = 0; q < nrows; ++q) {
          const int64_t qa = box_a[q];
          const int32_t qo = box_o[q];
          const int32_t qn = (q + 1 < nrows ? box_o[q + 1] : (int32_t)total) - qo;
          for (int t = lane; t < qn; t += kWave) {
            sx[qo + t] = X[qa + t];
            sy[qo + t] = Y[qa + t];
            if (DIM == 3) sz[qo + t] = Z[qa + t];
          }
        }
      }
      __syncthreads();
    }
    if (act) {
      int64_t hits = 0;
      for (int zz = z0; zz <= z1; ++zz)
        for (int yy = y0; yy <= y1; ++yy) {
          const int rk = (zz * Lj.nc[1] + yy) * Lj.nc[0];
          const int64_t a = cs[rk + x0], b = cs[rk + x1 + 1];
          // LDS slot of point t: its box row starts at box_a with offset box_o
          int64_t shift = 0;
          if (staged) {
            const int q = (zz - BZ0) * ny + (yy - BY0);
            shift = (int64_t)box_o[q] - box_a[q];
          }
          for (int64_t t = a; t < b; ++t) {
            double qx, qy, qz = 0.0;
            if (staged) {
              qx = sx[t + shift];
              qy = sy[t + shift];
              if (DIM == 3) qz = sz[t + shift];
            } else {
              qx = X[t];
              qy = Y[t];
              if (DIM == 3) qz = Z[t];
            }
            hits += sqdist(DIM, px, py, pz, qx, qy, qz) < Lj.d2max;
          }
        }
      if (is_diag) {
        nd = hits;
      } else {
        nl += hits;
        if (cnt_lv) cnt_lv[seg * N + i] = (int32_t)hits;  // per-level counts for the sliced lower copy
      }
    }
    if (boxed) __syncthreads();  // before the next level reuses the LDS
    if (is_diag) break;
  }
  if (act) {
    cnt_d[i] = nd;
    cnt_l[i] = nl;
  }
}

// Fill pass on the same staged tiles, four waves per tile: wave w fills rows
// w, w + 4, ... of the tile, one row at a time (the row's quantities are
// wave-uniform). For each level the lanes test 64 candidates per step (in
// 2-D the row's three cell-row ranges taken as one list); the hits' squared
// distances and columns are appended in order to the wave's LDS queue (ballot
// prefix count), which is flushed 64 entries at a time and at the end of the
// row's run: every lane then evaluates one phi value, and the stores of a
// flush are one contiguous run per array, in ascending column order. So the
// FP64 square root and division run on full waves instead of on the ~third
// of the lanes that hit in a step. The first wave computes the box.
constexpr int kFillWaves = 4;
constexpr int kBoxCols = 16;     // cell starts of a box row staged in LDS (boxes of up to 15 cells in x)
constexpr int kQueue = 2 * kWave;  // hit queue of a wave: up to 63 carried + 64 appended

// Orders a wave's LDS accesses before and after this point (the queue is
// written and read by different lanes of the same wave).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int DIM>
__global__ void __launch_bounds__(kFillWaves * kWave)
    k_nbr_tile_fill(int k, const DevLevel* __restrict__ lev, const int32_t* __restrict__ cs_all,
                    const double* __restrict__ xs, int64_t N, const int64_t* __restrict__ dptr,
                    int32_t* __restrict__ dcol, double* __restrict__ dval, float* __restrict__ dval32,
                    const int64_t* __restrict__ lptr, int32_t* __restrict__ lcol, double* __restrict__ lval,
                    float* __restrict__ lval32, float* __restrict__ dlo, float* __restrict__ llo) {
  __shared__ double2 sxy[kTileCap];
  __shared__ double sz[DIM == 3 ? kTileCap : 1];
  __shared__ int64_t box_a[kMaxBoxRows];
  __shared__ int32_t box_o[kMaxBoxRows];
  __shared__ double q_d2[kFillWaves][kQueue];
  __shared__ int32_t q_col[kFillWaves][kQueue];
  // the box's cell starts, cs[row key + BX0 + c] for c <= BX1 - BX0 + 1, when
  // the box is at most kBoxCols - 1 cells wide (box[7] = 1): a row's candidate
  // ranges are then read from LDS, not from the cell table in global memory
  __shared__ int32_t box_cs[kMaxBoxRows * kBoxCols];
  __shared__ int box[8];         // X0, X1, Y0, Y1, Z0, Z1, staged, cell starts staged
  __shared__ int64_t lpos_s[kWave];  // next lower-block position of each row of the tile
  const DevLevel Lk = lev[k];
  const int lane = threadIdx.x % kWave;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
  const int64_t tile0 = (int64_t)blockIdx.x * kWave;
  const int nrow_tile = (int)min<int64_t>(kWave, Lk.n - tile0);
  double* const qd = q_d2[w];
  int32_t* const qc = q_col[w];
  const double* X = xs;
  const double* Y = xs + N;
  const double* Z = xs + 2 * N;
  if (threadIdx.x < nrow_tile) lpos_s[threadIdx.x] = lptr[Lk.off + tile0 + threadIdx.x];
  for (int j = Lk.first;; j = lev[j].next) {
    const DevLevel Lj = lev[j];
    const bool is_diag = j == k;
    const int32_t* cs = cs_all + Lj.cs_off;
    if (w == 0) {  // the tile's box of cell rows, and its candidate count
      const bool act = lane < nrow_tile;
      const int64_t i = Lk.off + tile0 + (act ? lane : 0);
      const double px = X[i], py = Y[i], pz = DIM == 3 ? Z[i] : 0.0;
      const int cx = cell_coord(px, Lj.lo[0], Lj.inv_cell, Lj.nc[0]);
      const int cy = cell_coord(py, Lj.lo[1], Lj.inv_cell, Lj.nc[1]);
      const int cz = DIM == 3 ? cell_coord(pz, Lj.lo[2], Lj.inv_cell, Lj.nc[2]) : 0;
      const int BX0 = wave_min(act ? max(cx - 1, 0) : INT32_MAX);
      const int BX1 = wave_max(act ? min(cx + 1, Lj.nc[0] - 1) : -1);
      const int BY0 = wave_min(act ? max(cy - 1, 0) : INT32_MAX);
      const int BY1 = wave_max(act ? min(cy + 1, Lj.nc[1] - 1) : -1);
      const int BZ0 = DIM == 3 ? wave_min(act ? max(cz - 1, 0) : INT32_MAX) : 0;
      const int BZ1 = DIM == 3 ? wave_max(act ? min(cz + 1, Lj.nc[2] - 1) : -1) : 0;
      const int ny = BY1 - BY0 + 1;
      const int nrows = ny * (BZ1 - BZ0 + 1);
      int staged = 0;
      if (nrows >= 1 && nrows <= kMaxBoxRows) {
        int64_t a = 0, len = 0;
        if (lane < nrows) {
          const int yy = BY0 + lane % ny, zz = BZ0 + lane / ny;
          const int rk = (zz * Lj.nc[1] + yy) * Lj.nc[0];
          a = cs[rk + BX0];
          len = cs[rk + BX1 + 1] - a;
        }
        int64_t incl = len;
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) {
          const int64_t u = __shfl_up(incl, o, kWave);
          if (lane >= o) incl += u;
        }
        const int64_t total = __shfl(incl, kWave - 1, kWave);
        if (lane < nrows) {
          box_a[lane] = a;
          box_o[lane] = (int32_t)(incl - len);
        }
        staged = total <= kTileCap ? (int)total + 1 : 0;  // total + 1 when staged
      }
      const int wcs = BX1 - BX0 + 2;  // cell starts of one box row
      const int cs_staged = nrows >= 1 && nrows <= kMaxBoxRows && wcs <= kBoxCols;
      if (cs_staged && lane < nrows) {
        const int yy = BY0 + lane % ny, zz = BZ0 + lane / ny;
        const int rk = (zz * Lj.nc[1] + yy) * Lj.nc[0];
        for (int c = 0; c < wcs; ++c) box_cs[lane * kBoxCols + c] = cs[rk + BX0 + c];
      }
      if (lane == 0) {
        box[0] = BX0;
        box[1] = BX1;
        box[2] = BY0;
        box[3] = BY1;
        box[4] = BZ0;
        box[5] = BZ1;
        box[6] = staged;
        box[7] = cs_staged;
      }
    }
    __syncthreads();
    const int BX0 = box[0], BY0 = box[2], BZ0 = box[4];
    const int ny = box[3] - BY0 + 1;
    const int nrows = ny * (box[5] - BZ0 + 1);
    const bool staged = box[6] > 0;
    const bool cs_staged = box[7] != 0;
    if (staged) {
      const int32_t total = box[6] - 1;
      for (int q = 0; q < nrows; ++q) {
        const int64_t qa = box_a[q];
        const int32_t qo = box_o[q];
        const int32_t qn = (q + 1 < nrows ? box_o[q + 1] : total) - qo;
        for (int t = threadIdx.x; t < qn; t += kFillWaves * kWave) {
          sxy[qo + t] = make_double2(X[qa + t], Y[qa + t]);
          if (DIM == 3) sz[qo + t] = Z[qa + t];
        }
      }
    }
    __syncthreads();
    int32_t* col = is_diag ? dcol : lcol;
    double* val = is_diag ? dval : lval;
    float* val32 = is_diag ? dval32 : lval32;
    float* vlo = is_diag ? dlo : llo;
    for (int q = w; q < nrow_tile; q += kFillWaves) {
      const int64_t i = Lk.off + tile0 + q;
      const double qx = X[i], qy = Y[i], qz = DIM == 3 ? Z[i] : 0.0;
      const int cx = cell_coord(qx, Lj.lo[0], Lj.inv_cell, Lj.nc[0]);
      const int cy = cell_coord(qy, Lj.lo[1], Lj.inv_cell, Lj.nc[1]);
      const int cz = DIM == 3 ? cell_coord(qz, Lj.lo[2], Lj.inv_cell, Lj.nc[2]) : 0;
      const int qx0 = max(cx - 1, 0), qx1 = min(cx + 1, Lj.nc[0] - 1);
      const int qy0 = max(cy - 1, 0), qy1 = min(cy + 1, Lj.nc[1] - 1);
      const int qz0 = DIM == 3 ? max(cz - 1, 0) : 0, qz1 = DIM == 3 ? min(cz + 1, Lj.nc[2] - 1) : 0;
      const int64_t pos = is_diag ? dptr[i] : lpos_s[q];
      int64_t nh = 0;  // the row's entries written so far
      int qn = 0;      // queued hits
      // write queue entries 0 .. m-1 at the row's next m positions
      auto flush = [&](int m) {
        wave_lds_sync();
        if (lane < m) {
          const double d2 = qd[lane];
          const int64_t pp = pos + nh + lane;
          col[pp] = qc[lane];
          const double v = phi31_d2(d2, Lj.delta);
          if (val) val[pp] = v;
          if (val32) val32[pp] = (float)v;
          if (vlo) vlo[pp] = (float)(v - (double)(float)v);
        }
        nh += m;
      };
      // one candidate step: 64 lanes test candidates, hits appended in order
      auto step = [&](int32_t t, double cxv, double cyv, double czv, bool valid) {
        const double d2 = valid ? sqdist(DIM, qx, qy, qz, cxv, cyv, czv) : Lj.d2max;
        const bool hit = d2 < Lj.d2max;
        const uint64_t m = __ballot(hit);
        if (hit) {
          const int o = qn + __popcll(m & below);
          qd[o] = d2;
          qc[o] = t;
        }
        qn += __popcll(m);
        if (qn >= kWave) {
          flush(kWave);
          const int rest = qn - kWave;
          double dr = 0.0;
          int32_t cr = 0;
          if (lane < rest) {
            dr = qd[kWave + lane];
            cr = qc[kWave + lane];
          }
          wave_lds_sync();
          if (lane < rest) {
            qd[lane] = dr;
            qc[lane] = cr;
          }
          qn = rest;
        }
      };
      if constexpr (DIM == 2) {
        // the row's cell-row ranges as one list: candidate c of range r is
        // point c + gb[r] (LDS slot c + lb[r] when staged)
        int32_t cnt[3], gb[3], lb[3];
        int32_t pre = 0;
#pragma unroll
        for (int r = 0; r < 3; ++r) {
          const int yy = qy0 + r;
          int32_t a = 0, b = 0, sh = 0;
          if (yy <= qy1) {
            if (cs_staged) {  // the row's cells lie inside the box: qx0 >= BX0, qx1 + 1 <= BX1 + 1
              const int32_t* bc = box_cs + (yy - BY0) * kBoxCols;
              a = bc[qx0 - BX0];
              b = bc[qx1 + 1 - BX0];
            } else {
              const int rk = yy * Lj.nc[0];
              a = cs[rk + qx0];
              b = cs[rk + qx1 + 1];
            }
            if (staged) sh = box_o[yy - BY0] - (int32_t)box_a[yy - BY0];
          }
          cnt[r] = b - a;
          gb[r] = a - pre;
          lb[r] = a + sh - pre;
          pre += b - a;
        }
        const int32_t total = pre, e1 = cnt[0], e2 = cnt[0] + cnt[1];
        for (int32_t c0 = 0; c0 < total; c0 += kWave) {
          const int32_t c = c0 + lane;
          const bool valid = c < total;
          const int32_t t = c + (c < e1 ? gb[0] : c < e2 ? gb[1] : gb[2]);
          double cxv = 0.0, cyv = 0.0;
          if (staged) {
            if (valid) {
              const double2 p = sxy[c + (c < e1 ? lb[0] : c < e2 ? lb[1] : lb[2])];
              cxv = p.x;
              cyv = p.y;
            }
          } else if (valid) {
            cxv = X[t];
            cyv = Y[t];
          }
          step(t, cxv, cyv, 0.0, valid);
        }
      } else {
        for (int zz = qz0; zz <= qz1; ++zz)
          for (int yy = qy0; yy <= qy1; ++yy) {
            int32_t a, b;
            if (cs_staged) {
              const int32_t* bc = box_cs + ((zz - BZ0) * ny + (yy - BY0)) * kBoxCols;
              a = bc[qx0 - BX0];
              b = bc[qx1 + 1 - BX0];
            } else {
              const int rk = (zz * Lj.nc[1] + yy) * Lj.nc[0];
              a = cs[rk + qx0];
              b = cs[rk + qx1 + 1];
            }
            int32_t sh = 0;
            if (staged) {
              const int bq = (zz - BZ0) * ny + (yy - BY0);
              sh = box_o[bq] - (int32_t)box_a[bq];
            }
            for (int32_t t0 = a; t0 < b; t0 += kWave) {
              const int32_t t = t0 + lane;
              const bool valid = t < b;
              double cxv = 0.0, cyv = 0.0, czv = 0.0;
              if (valid) {
                if (staged) {
                  const double2 p = sxy[t + sh];
                  cxv = p.x;
                  cyv = p.y;
                  czv = sz[t + sh];
                } else {
                  cxv = X[t];
                  cyv = Y[t];
                  czv = Z[t];
                }
              }
              step(t, cxv, cyv, czv, valid);
            }
          }
      }
      if (qn > 0) flush(qn);
      wave_lds_sync();  // the queue's reads are done before the next row appends
      if (!is_diag && lane == 0) lpos_s[q] = pos + nh;
    }
    __syncthreads();  // before the next level reuses the LDS and the box
    if (is_diag) break;
  }
}

// ------------------------------------------------------------- work table

mskm_status build_work_table(mskm_hier* h, WorkTable* wt, int min_rows, int max_blocks_per_level) {
  std::vector<int32_t> lev;
  std::vector<int64_t> r0, r1;
  wt->h_lev_begin.assign(h->L + 1, 0);
  for (int l = 0; l < h->L; ++l) {
    wt->h_lev_begin[l] = (int32_t)lev.size();
    const int64_t n = h->h_off[l + 1] - h->h_off[l];
    const int64_t rpb = std::max<int64_t>(min_rows, (n + max_blocks_per_level - 1) / max_blocks_per_level);
    for (int64_t a = h->h_off[l]; a < h->h_off[l + 1]; a += rpb) {
      lev.push_back(l);
      r0.push_back(a);
      r1.push_back(std::min<int64_t>(a + rpb, h->h_off[l + 1]));
    }
  }
  wt->h_lev_begin[h->L] = (int32_t)lev.size();
  if (lev.size() > (size_t)INT32_MAX) return fail(MSKM_ELIMIT, "work table too large");
  wt->nblocks = (int32_t)lev.size();
  wt->rows_per_block = min_rows;
  MSKM_TRY(halloc(h, &wt->lev, lev.size()));
  MSKM_TRY(halloc(h, &wt->row0, r0.size()));
  MSKM_TRY(halloc(h, &wt->row1, r1.size()));
  MSKM_TRY(halloc(h, &wt->lev_begin, wt->h_lev_begin.size()));
  MSKM_TRY(upload_async(h, wt->lev, lev.data(), lev.size() * 4));
  MSKM_TRY(upload_async(h, wt->row0, r0.data(), r0.size() * 8));
  MSKM_TRY(upload_async(h, wt->row1, r1.data(), r1.size() * 8));
  MSKM_TRY(upload_async(h, wt->lev_begin, wt->h_lev_begin.data(), wt->h_lev_begin.size() * 4));
  return MSKM_OK;
}

// ------------------------------------------------------------- assembly

static unsigned grid_for(int64_t n, int per_block) {
  int64_t g = (n + per_block - 1) / per_block;
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(g, 1 << 30));
}

// Record of internal point i: {x, y, z (0 in 2-D), 1/delta of its level};
// the level is found by binary search over the level offsets.
__global__ void __launch_bounds__(kBlock) k_point_records(int dim, int L, const DevLevel* __restrict__ lev,
                                                          const double* __restrict__ xs, int64_t N,
                                                          double* __restrict__ rec) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= N) return;
  int lo = 0, hi = L - 1;  // last level with off <= i
  while (lo < hi) {
    const int mid = (lo + hi + 1) / 2;
    if (lev[mid].off <= i) lo = mid;
    else hi = mid - 1;
  }
  double4 r;
  r.x = xs[i];
  r.y = xs[N + i];
  r.z = dim == 3 ? xs[2 * N + i] : 0.0;
  r.w = lev[lo].inv_delta;
  reinterpret_cast<double4*>(rec)[i] = r;
}

static mskm_status build_sell(mskm_hier* h, bool want64, bool want32, bool with_lo);

mskm_status assemble_hierarchy(mskm_hier* h, const double* pts, bool want64, bool want32, bool want_lsell) {
  hipStream_t s = h->ctx->stream;
  const int L = h->L, dim = h->dim;
  const int64_t N = h->N;
  for (hipEvent_t* e : {&h->ev_asm[0], &h->ev_asm[1]})
    if (!*e) MSKM_HIP_TRY(hipEventCreate(e));
  MSKM_HIP_TRY(hipEventRecord(h->ev_asm[0], s));

  std::vector<int64_t> rng(2 * (size_t)L);
  for (int l = 0; l < L; ++l) {
    rng[2 * l] = h->h_in_off[l];
    rng[2 * l + 1] = h->h_in_off[l] + (h->h_off[l + 1] - h->h_off[l]);
  }
  // 1. bounding boxes
  std::vector<double> bbox((size_t)L * kBboxBlocks * 6);
  {
    int64_t* d_off = nullptr;
    double* d_part = nullptr;
    void* bb = nullptr;
    Carve cv;
    cv.add(&d_off, 2 * (size_t)L);
    cv.add(&d_part, bbox.size());
    MSKM_TRY(cv.alloc(h->ctx, &bb));
    CtxScratch free_bb{h->ctx, bb, cv.bytes};
    MSKM_HIP_TRY(hipMemcpyAsync(d_off, rng.data(), rng.size() * 8, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_bbox_partial, dim3(kBboxBlocks, L), dim3(kBlock), 0, s, pts, d_off, dim, d_part);
    MSKM_HIP_TRY(hipMemcpyAsync(bbox.data(), d_part, bbox.size() * 8, hipMemcpyDeviceToHost, s));
    MSKM_HIP_TRY(hipStreamSynchronize(s));
  }

  // 2. level grids (host): cell side delta*(1+1e-6), enlarged if the grid
  //    would exceed max(4n, 64) cells
  h->h_lev.resize(L);
  int64_t cs_total = 0;
  for (int l = 0; l < L; ++l) {
    DevLevel& D = h->h_lev[l];
    D.off = h->h_off[l];
    D.n = (int32_t)(h->h_off[l + 1] - h->h_off[l]);
    D.first = h->h_first[l];
    D.next = h->h_next[l];
    D.delta = h->h_delta[l];
    D.d2max = D.delta * D.delta;
    D.inv_delta = 1.0 / D.delta;
    double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    for (int d = 0; d < 3; ++d) {
      lo[d] = INFINITY;
      hi[d] = -INFINITY;
    }
    for (int b = 0; b < kBboxBlocks; ++b) {
      const double* o = &bbox[((size_t)l * kBboxBlocks + b) * 6];
      for (int d = 0; d < dim; ++d) {
        if (std::isnan(o[d]) || std::isnan(o[3 + d])) return fail(MSKM_EINVAL, "non-finite point coordinate");
        lo[d] = std::min(lo[d], o[d]);
        hi[d] = std::max(hi[d], o[3 + d]);
      }
    }
    for (int d = 0; d < dim; ++d) {
      if (D.n > 0 && (!std::isfinite(lo[d]) || !std::isfinite(hi[d])))
        return fail(MSKM_EINVAL, "non-finite point coordinate");
      if (D.n == 0) lo[d] = hi[d] = 0.0;
    }
    double cell = D.delta * (1.0 + 1e-6);
    const double maxcells = std::max<double>(64.0, 4.0 * (double)D.n);
    for (;;) {
      double tot = 1.0;
      for (int d = 0; d < dim; ++d) tot *= std::floor((hi[d] - lo[d]) / cell) + 1.0;
      if (tot <= maxcells) break;
      cell *= 1.25;
    }
    D.inv_cell = 1.0 / cell;
    int64_t ncell = 1;
    for (int d = 0; d < 3; ++d) {
      D.lo[d] = d < dim ? lo[d] : 0.0;
      D.nc[d] = d < dim ? (int32_t)std::floor((hi[d] - lo[d]) * D.inv_cell) + 1 : 1;
      if (D.nc[d] < 1) D.nc[d] = 1;
      ncell *= D.nc[d];
    }
    D.ncell_tot = (int32_t)ncell;
    D.cs_off = (int32_t)cs_total;
    cs_total += ncell + 1;
  }
  if (cs_total >= INT32_MAX) return fail(MSKM_ELIMIT, "cell tables too large");
  MSKM_TRY(halloc(h, &h->d_lev, L));
  MSKM_TRY(upload_async(h, h->d_lev, h->h_lev.data(), L * sizeof(DevLevel)));

  // 3. counting sort into cells. Scratch of the sort, the counts and the
  //    scans: one allocation, freed once the fill pass is queued (a free
  //    between kernels would synchronise the device)
  int32_t *key = nullptr, *count = nullptr, *tmp = nullptr;
  int64_t *count64 = nullptr, *cs64 = nullptr, *cnt_d = nullptr, *cnt_l = nullptr, *part = nullptr;
  int32_t* cnt_lv = nullptr;  // [coarser level][N] per-level lower counts (sliced lower copy only)
  int max_depth = 1;
  for (int g = 0; g < h->ngroups; ++g) max_depth = std::max(max_depth, (int)h->h_group_levels[g] - 1);
  void* scratch = nullptr;
  size_t scratch_bytes = 0;
  {
    Carve cv;
    if (want_lsell) cv.add(&cnt_lv, (size_t)N * max_depth);
    cv.add(&key, N);
    cv.add(&count, cs_total);
    cv.add(&count64, cs_total);
    cv.add(&cs64, cs_total);
    cv.add(&tmp, N);
    cv.add(&cnt_d, N + 1);
    cv.add(&cnt_l, N + 1);
    cv.add(&part, std::max(scan_parts(cs_total), scan_parts(N + 1)));
    MSKM_TRY(cv.alloc(h->ctx, &scratch));
    scratch_bytes = cv.bytes;
  }
  CtxScratch free_scratch{h->ctx, scratch, scratch_bytes};
  MSKM_HIP_TRY(hipMemsetAsync(count, 0, cs_total * 4, s));
  for (int l = 0; l < L; ++l) {
    const int64_t n = h->h_lev[l].n;
    if (n == 0) continue;
    hipLaunchKernelGGL(k_cell_key, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, s, pts, dim, h->d_lev, l, h->h_in_off[l],
                       n, key, count);
  }
  // widen counts and scan over all levels' tables at once: since every
  // point lands in exactly one cell of its level, the scan value at a
  // level's first cell equals that level's offset, so cs64 holds internal
  // global indices directly.
  MSKM_TRY(halloc(h, &h->cell_start, cs_total));
  hipLaunchKernelGGL(k_widen, dim3(grid_for(cs_total, kBlock)), dim3(kBlock), 0, s, count, count64, cs_total);
  MSKM_TRY(exclusive_scan_i64(s, count64, cs64, cs_total, part));
  hipLaunchKernelGGL(k_narrow, dim3(grid_for(cs_total, kBlock)), dim3(kBlock), 0, s, cs64, h->cell_start, cs_total);
  MSKM_HIP_TRY(hipMemsetAsync(count, 0, cs_total * 4, s));  // reuse as cursors
  MSKM_TRY(halloc(h, &h->perm, N));
  MSKM_TRY(halloc(h, &h->iperm, N));
  MSKM_TRY(halloc(h, &h->xs, (size_t)dim * N));
  for (int l = 0; l < L; ++l) {
    const int64_t n = h->h_lev[l].n;
    if (n == 0) continue;
    hipLaunchKernelGGL(k_cell_scatter, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, s, h->d_lev, l, h->h_in_off[l], n, key,
                       cs64, count, tmp);
  }
  for (int l = 0; l < L; ++l) {
    const int64_t n = h->h_lev[l].n;
    if (n == 0) continue;
    hipLaunchKernelGGL(k_cell_rank, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, s, h->d_lev, l, h->h_off[l], n, dim, pts,
                       key, cs64, tmp, h->perm, h->iperm, h->xs, N);
  }

  // point records for the SpMV variants that recompute entry values
  MSKM_TRY(halloc(h, &h->prec, (size_t)4 * N));
  hipLaunchKernelGGL(k_point_records, dim3(grid_for(N, kBlock)), dim3(kBlock), 0, s, dim, L, h->d_lev, h->xs, N,
                     h->prec);

  // 4. count pass
  MSKM_HIP_TRY(hipMemsetAsync(cnt_d + N, 0, 8, s));
  MSKM_HIP_TRY(hipMemsetAsync(cnt_l + N, 0, 8, s));
  for (int k = 0; k < L; ++k) {
    const int64_t n = h->h_lev[k].n;
    if (n == 0) continue;
    if (dim == 3)
      hipLaunchKernelGGL(k_nbr_tile_count<3>, dim3(grid_for(n, kWave)), dim3(kWave), 0, s, k, h->d_lev, h->cell_start,
                         h->xs, N, cnt_d, cnt_l, cnt_lv);
    else
      hipLaunchKernelGGL(k_nbr_tile_count<2>, dim3(grid_for(n, kWave)), dim3(kWave), 0, s, k, h->d_lev, h->cell_start,
                         h->xs, N, cnt_d, cnt_l, cnt_lv);
  }
  MSKM_TRY(halloc(h, &h->diag.rowptr, N + 1));
  MSKM_TRY(halloc(h, &h->lower.rowptr, N + 1));
  MSKM_TRY(exclusive_scan_i64(s, cnt_d, h->diag.rowptr, N + 1, part));
  MSKM_TRY(exclusive_scan_i64(s, cnt_l, h->lower.rowptr, N + 1, part));
  MSKM_HIP_TRY(hipMemcpyAsync(&h->diag.nnz, h->diag.rowptr + N, 8, hipMemcpyDeviceToHost, s));
  MSKM_HIP_TRY(hipMemcpyAsync(&h->lower.nnz, h->lower.rowptr + N, 8, hipMemcpyDeviceToHost, s));
  MSKM_HIP_TRY(hipStreamSynchronize(s));

  // 5. fill pass (FP32-only hierarchies also keep the FP32 rounding remainders)
  const bool want_lo = want32 && !want64;
  for (Csr* c : {&h->diag, &h->lower}) {
    MSKM_TRY(halloc(h, &c->col, (size_t)c->nnz + kCsrPad));
    if (want64) MSKM_TRY(halloc(h, &c->val, (size_t)c->nnz + kCsrPad));
    if (want32) MSKM_TRY(halloc(h, &c->val32, (size_t)c->nnz + kCsrPad));
    if (want_lo) MSKM_TRY(halloc(h, &c->val32lo, (size_t)c->nnz + kCsrPad));
    // pads hold finite values (never used: the loads that reach them are masked)
    MSKM_HIP_TRY(hipMemsetAsync(c->col + c->nnz, 0, kCsrPad * 4, s));
    if (want64) MSKM_HIP_TRY(hipMemsetAsync(c->val + c->nnz, 0, kCsrPad * 8, s));
    if (want32) MSKM_HIP_TRY(hipMemsetAsync(c->val32 + c->nnz, 0, kCsrPad * 4, s));
    if (want_lo) MSKM_HIP_TRY(hipMemsetAsync(c->val32lo + c->nnz, 0, kCsrPad * 4, s));
  }
  for (int k = 0; k < L; ++k) {
    const int64_t n = h->h_lev[k].n;
    if (n == 0) continue;
    if (dim == 3)
      hipLaunchKernelGGL(k_nbr_tile_fill<3>, dim3(grid_for(n, kWave)), dim3(kFillWaves * kWave), 0, s, k, h->d_lev,
                         h->cell_start, h->xs, N, h->diag.rowptr, h->diag.col, h->diag.val, h->diag.val32, h->lower.rowptr,
                         h->lower.col, h->lower.val, h->lower.val32, h->diag.val32lo, h->lower.val32lo);
    else
      hipLaunchKernelGGL(k_nbr_tile_fill<2>, dim3(grid_for(n, kWave)), dim3(kFillWaves * kWave), 0, s, k, h->d_lev,
                         h->cell_start, h->xs, N, h->diag.rowptr, h->diag.col, h->diag.val, h->diag.val32, h->lower.rowptr,
                         h->lower.col, h->lower.val, h->lower.val32, h->diag.val32lo, h->lower.val32lo);
  }
  MSKM_TRY(build_sell(h, want64, want32, want_lsell));
  if (want_lsell) MSKM_TRY(build_lsell(h, want64, want32, cnt_lv));
  MSKM_HIP_TRY(hipEventRecord(h->ev_asm[1], s));
  h->asm_pending = true;  // assemble_ms is read at the first statistics query
  MSKM_HIP_TRY(hipGetLastError());
  return MSKM_OK;
}

// ------------------------------------------------------------------ SELL

// Row of every slot: slot t of the level's slices holds row off + t, or -1
// past the level's last row.
__global__ void __launch_bounds__(kBlock) k_sell_rows(int64_t off, int64_t n, int64_t slot0, int64_t nslots,
                                                      int32_t* __restrict__ rows) {
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (t >= nslots) return;
  rows[slot0 + t] = t < n ? (int32_t)(off + t) : -1;
}

// Width (in entries, w_s * kSellC) of every slice: its longest row rounded
// up to a multiple of 4, times kSellC. Entry nslices is 0 (scan sentinel).
__global__ void __launch_bounds__(kBlock) k_sell_width(int64_t nslices, const int32_t* __restrict__ rows,
                                                       const int64_t* __restrict__ rp, int64_t* __restrict__ w) {
  const int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (s > nslices) return;
  if (s == nslices) {
    w[s] = 0;
    return;
  }
  int64_t m = 0;
  for (int t = 0; t < kSellC; ++t) {
    const int32_t r = rows[s * kSellC + t];
    if (r >= 0) m = max(m, rp[r + 1] - rp[r]);
  }
  w[s] = (m + 3) / 4 * 4 * kSellC;
}

// Copy the CSR rows into the slot-interleaved layout (groups of four
// consecutive entries per slot: entry k of slot t at e0 + (k / 4) 4 kSellC +
// 4 t + k % 4). One workgroup of kSellFillWaves waves per slice; wave w copies
// slots 16w .. 16w + 15, lane i taking slot 16w + i % 16 and the groups
// g = i / 16, i / 16 + 4, ...: it loads entries 4g .. 4g + 3 of its row (one
// 16-byte load when all four lie inside the row) and stores them as one
// 4-wide vector. Per instruction the loads read 64 consecutive bytes of each
// of 16 rows and the stores write 4 runs of 16 consecutive slots. No LDS and
// no barriers.
constexpr int kSellFillWaves = 4;
constexpr int kSellFillRows = kSellC / kSellFillWaves;
constexpr int kSellFillGroups = kSellC / kSellFillRows;
__global__ void __launch_bounds__(kSellFillWaves * kSellC)
    k_sell_fill(int64_t nslices, const int32_t* __restrict__ rows, const int64_t* __restrict__ sptr,
                const int64_t* __restrict__ rp, const int32_t* __restrict__ col, const double* __restrict__ val,
                const float* __restrict__ val32, const float* __restrict__ lo32, int32_t* __restrict__ scol,
                double* __restrict__ sval, float* __restrict__ sval32, float* __restrict__ slo) {
  const int64_t s = blockIdx.x;
  const int lane = threadIdx.x % kSellC, w = threadIdx.x / kSellC;
  const int t = w * kSellFillRows + lane % kSellFillRows, gl = lane / kSellFillRows;
  const int32_t row = rows[s * kSellC + t];
  // pad column: the slot's own row, or for an empty slot (past the level's
  // last row) the slice's first row, so that it stays inside the slice's span
  const int32_t pad = row >= 0 ? row : rows[s * kSellC];
  const int64_t b = row >= 0 ? rp[row] : 0;
  const int64_t len = row >= 0 ? rp[row + 1] - b : 0;
  const int64_t e0 = sptr[s], groups = (sptr[s + 1] - e0) / (4 * kSellC);
  for (int64_t g = gl; g < groups; g += kSellFillGroups) {
    const int64_t d = e0 + g * (4 * kSellC) + 4 * t;
    const int64_t k = 4 * g, src = b + k;
    int4 c;
    float4 v32 = make_float4(0.f, 0.f, 0.f, 0.f), vlo = v32;
    double2 v64a = make_double2(0.0, 0.0), v64b = v64a;
    if (k + 4 <= len) {  // the whole group inside the row: 16-byte loads (4-byte aligned)
      __builtin_memcpy(&c, col + src, 16);
      if (sval32) __builtin_memcpy(&v32, val32 + src, 16);
      if (slo) __builtin_memcpy(&vlo, lo32 + src, 16);
      if (sval) {
        __builtin_memcpy(&v64a, val + src, 16);
        __builtin_memcpy(&v64b, val + src + 2, 16);
      }
    } else {
      const bool in0 = k < len, in1 = k + 1 < len, in2 = k + 2 < len;  // k + 3 < len is false here
      c = make_int4(in0 ? col[src] : pad, in1 ? col[src + 1] : pad, in2 ? col[src + 2] : pad, pad);
      if (sval32) v32 = make_float4(in0 ? val32[src] : 0.f, in1 ? val32[src + 1] : 0.f, in2 ? val32[src + 2] : 0.f, 0.f);
      if (slo) vlo = make_float4(in0 ? lo32[src] : 0.f, in1 ? lo32[src + 1] : 0.f, in2 ? lo32[src + 2] : 0.f, 0.f);
      if (sval) {
        v64a = make_double2(in0 ? val[src] : 0.0, in1 ? val[src + 1] : 0.0);
        v64b = make_double2(in2 ? val[src + 2] : 0.0, 0.0);
      }
    }
    *reinterpret_cast<int4*>(scol + d) = c;
    if (sval) {
      *reinterpret_cast<double2*>(sval + d) = v64a;
      *reinterpret_cast<double2*>(sval + d + 2) = v64b;
    }
    if (sval32) *reinterpret_cast<float4*>(sval32 + d) = v32;
    if (slo) *reinterpret_cast<float4*>(slo + d) = vlo;
  }
}

// Smallest column of each slice (one wave per slice); the slices whose
// columns span more than 65536 rows are counted in *wide.
__global__ void __launch_bounds__(kSellC)
    k_sell_span(const int64_t* __restrict__ sptr, const int32_t* __restrict__ scol, int32_t* __restrict__ cbase,
                int32_t* __restrict__ wide) {
  const int64_t s = blockIdx.x;
  int32_t lo = INT32_MAX, hi = -1;
  for (int64_t d = sptr[s] + threadIdx.x; d < sptr[s + 1]; d += kSellC) {
    const int32_t c = scol[d];
    lo = min(lo, c);
    hi = max(hi, c);
  }
#pragma unroll
  for (int o = kSellC / 2; o > 0; o >>= 1) {
    lo = min(lo, __shfl_xor(lo, o, kSellC));
    hi = max(hi, __shfl_xor(hi, o, kSellC));
  }
  if (threadIdx.x == 0) {
    cbase[s] = hi >= 0 ? lo : 0;
    if (hi >= 0 && hi - lo > 65535) atomicAdd(wide, 1);
  }
}

// col16 = col - cbase[slice] (one workgroup per slice).
__global__ void __launch_bounds__(kSellC)
    k_sell_narrow(const int64_t* __restrict__ sptr, const int32_t* __restrict__ scol,
                  const int32_t* __restrict__ cbase, uint16_t* __restrict__ col16) {
  const int64_t s = blockIdx.x;
  const int32_t b = cbase[s];
  for (int64_t d = sptr[s] + threadIdx.x; d < sptr[s + 1]; d += kSellC) col16[d] = (uint16_t)(scol[d] - b);
}

static mskm_status build_sell(mskm_hier* h, bool want64, bool want32, bool with_lo) {
  hipStream_t s = h->ctx->stream;
  Sell& S = h->sell;
  const int L = h->L;
  S.h_slice_begin.assign(L + 1, 0);
  for (int l = 0; l < L; ++l)
    S.h_slice_begin[l + 1] = S.h_slice_begin[l] + (h->h_off[l + 1] - h->h_off[l] + kSellC - 1) / kSellC;
  S.nslices = S.h_slice_begin[L];
  MSKM_TRY(halloc(h, &S.rows, (size_t)S.nslices * kSellC));
  MSKM_TRY(halloc(h, &S.sptr, (size_t)S.nslices + 1));
  for (int l = 0; l < L; ++l) {
    const int64_t nslots = (S.h_slice_begin[l + 1] - S.h_slice_begin[l]) * kSellC;
    if (nslots > 0)
      hipLaunchKernelGGL(k_sell_rows, dim3(grid_for(nslots, kBlock)), dim3(kBlock), 0, s, h->h_off[l],
                         h->h_off[l + 1] - h->h_off[l], S.h_slice_begin[l] * kSellC, nslots, S.rows);
  }
  // scratch: slice widths, scan partials, the wide-slice counter
  int64_t *d_w = nullptr, *part = nullptr;
  int32_t* d_wide = nullptr;
  void* scratch = nullptr;
  size_t scratch_bytes = 0;
  {
    Carve cv;
    cv.add(&d_w, (size_t)S.nslices + 1);
    cv.add(&part, scan_parts(S.nslices + 1));
    cv.add(&d_wide, 1);
    MSKM_TRY(cv.alloc(h->ctx, &scratch));
    scratch_bytes = cv.bytes;
  }
  CtxScratch free_scratch{h->ctx, scratch, scratch_bytes};
  hipLaunchKernelGGL(k_sell_width, dim3(grid_for(S.nslices + 1, kBlock)), dim3(kBlock), 0, s, S.nslices, S.rows,
                     h->diag.rowptr, d_w);
  MSKM_TRY(exclusive_scan_i64(s, d_w, S.sptr, S.nslices + 1, part));
  MSKM_HIP_TRY(hipMemcpyAsync(&S.entries, S.sptr + S.nslices, 8, hipMemcpyDeviceToHost, s));
  MSKM_HIP_TRY(hipStreamSynchronize(s));
  MSKM_TRY(halloc(h, &S.col, (size_t)S.entries));
  if (want64) MSKM_TRY(halloc(h, &S.val, (size_t)S.entries));
  if (want32) MSKM_TRY(halloc(h, &S.val32, (size_t)S.entries));
  // the FP32 remainders too when the residual will run over the sliced copies
  const float* lo_src = with_lo ? h->diag.val32lo : nullptr;
  if (lo_src) MSKM_TRY(halloc(h, &S.lo, (size_t)S.entries));
  if (S.nslices > 0)
    hipLaunchKernelGGL(k_sell_fill, dim3((unsigned)S.nslices), dim3(kSellFillWaves * kSellC), 0, s, S.nslices,
                       S.rows, S.sptr, h->diag.rowptr, h->diag.col, h->diag.val, h->diag.val32, lo_src, S.col, S.val,
                       S.val32, S.lo);
  // 16-bit column offsets when every slice's columns span at most 65536 rows
  if (S.nslices > 0) {
    int32_t* cbase = nullptr;
    int32_t wide = 0;
    {
      void* q = nullptr;
      MSKM_TRY(ctx_alloc(h->ctx, (size_t)S.nslices * 4, &q));
      cbase = static_cast<int32_t*>(q);
    }
    mskm_status st = MSKM_OK;
    if (hipMemsetAsync(d_wide, 0, 4, s) != hipSuccess) st = fail(MSKM_EDEVICE, "memset");
    if (st == MSKM_OK) {
      hipLaunchKernelGGL(k_sell_span, dim3((unsigned)S.nslices), dim3(kSellC), 0, s, S.sptr, S.col, cbase, d_wide);
      if (hipMemcpyAsync(&wide, d_wide, 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
          hipStreamSynchronize(s) != hipSuccess)
        st = fail(MSKM_EDEVICE, "SELL column span");
    }
    if (st == MSKM_OK && wide == 0) {
      h->allocs.push_back(cbase);
      h->alloc_bytes.push_back((size_t)S.nslices * 4);
      h->device_bytes += S.nslices * 4;
      S.cbase = cbase;
      st = halloc(h, &S.col16, (size_t)S.entries);
      if (st == MSKM_OK)
        hipLaunchKernelGGL(k_sell_narrow, dim3((unsigned)S.nslices), dim3(kSellC), 0, s, S.sptr, S.col, S.cbase,
                           S.col16);
    } else {
      ctx_release(h->ctx, cbase, (size_t)S.nslices * 4);
    }
    MSKM_TRY(st);
  }
  // launch table: blocks of 4 slices (one wave each) within each level
  WorkTable& wt = h->wt_sell;
  std::vector<int32_t> lev;
  std::vector<int64_t> r0, r1;
  wt.h_lev_begin.assign(L + 1, 0);
  const int per = kBlock / kSellC;
  for (int l = 0; l < L; ++l) {
    wt.h_lev_begin[l] = (int32_t)lev.size();
    for (int64_t a = S.h_slice_begin[l]; a < S.h_slice_begin[l + 1]; a += per) {
      lev.push_back(l);
      r0.push_back(a);
      r1.push_back(std::min<int64_t>(a + per, S.h_slice_begin[l + 1]));
    }
  }
  wt.h_lev_begin[L] = (int32_t)lev.size();
  if (lev.size() > (size_t)INT32_MAX) return fail(MSKM_ELIMIT, "SELL table too large");
  wt.nblocks = (int32_t)lev.size();
  wt.rows_per_block = per;
  MSKM_TRY(halloc(h, &wt.lev, lev.size()));
  MSKM_TRY(halloc(h, &wt.row0, r0.size()));
  MSKM_TRY(halloc(h, &wt.row1, r1.size()));
  MSKM_TRY(halloc(h, &wt.lev_begin, wt.h_lev_begin.size()));
  MSKM_TRY(upload_async(h, wt.lev, lev.data(), lev.size() * 4));
  MSKM_TRY(upload_async(h, wt.row0, r0.data(), r0.size() * 8));
  MSKM_TRY(upload_async(h, wt.row1, r1.data(), r1.size() * 8));
  MSKM_TRY(upload_async(h, wt.lev_begin, wt.h_lev_begin.data(), wt.h_lev_begin.size() * 4));
  MSKM_HIP_TRY(hipGetLastError());
  return MSKM_OK;
}

// ------------------------------------------------------------------ export

// pts[perm[i]][a] = xs[a][i]: the points back in the input order (AoS).
__global__ void __launch_bounds__(kBlock) k_points_to_input(int dim, const double* __restrict__ xs, int64_t N,
                                                            const int32_t* __restrict__ perm,
                                                            double* __restrict__ pts) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= N) return;
  const int64_t o = (int64_t)perm[i] * dim;
  for (int a = 0; a < dim; ++a) pts[o + a] = xs[a * N + i];
}

mskm_status export_points_device(mskm_hier* h, double* pts_dev) {
  hipLaunchKernelGGL(k_points_to_input, dim3(grid_for(h->N, kBlock)), dim3(kBlock), 0, h->ctx->stream, h->dim, h->xs,
                     h->N, h->perm, pts_dev);
  MSKM_HIP_TRY(hipGetLastError());
  return MSKM_OK;
}

// Entries of block (k, j) in canonical row r (or in row rows[r] of level k
// when a row list is given): count pass.
__global__ void __launch_bounds__(kBlock) k_export_count(const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                                                         const int32_t* __restrict__ iperm, int64_t row_off,
                                                         int64_t nrows, int64_t c0, int64_t c1,
                                                         const int64_t* __restrict__ rows, int64_t* __restrict__ cnt) {
  const int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (r >= nrows) return;
  const int64_t i = iperm[row_off + (rows ? rows[r] : r)];
  int64_t c = 0;
  for (int64_t t = rp[i]; t < rp[i + 1]; ++t) c += (col[t] >= c0 && col[t] < c1);
  cnt[r] = c;
}

// Fill pass: canonical column = input index within level j; insertion sort
// of the row (rows are short: tens to a few hundred entries).
template <typename TV>
__global__ void __launch_bounds__(kBlock) k_export_fill(const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                                                        const TV* __restrict__ val, const int32_t* __restrict__ iperm,
                                                        const int32_t* __restrict__ perm, int64_t row_off,
                                                        int64_t nrows, int64_t c0, int64_t c1, int64_t cin,
                                                        const int64_t* __restrict__ rows,
                                                        const int64_t* __restrict__ optr, int32_t* __restrict__ ocol,
                                                        double* __restrict__ oval) {
  const int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (r >= nrows) return;
  const int64_t i = iperm[row_off + (rows ? rows[r] : r)];
  const int64_t o = optr[r];
  int64_t n = 0;
  for (int64_t t = rp[i]; t < rp[i + 1]; ++t) {
    const int32_t c = col[t];
    if (c < c0 || c >= c1) continue;
    const int32_t cc = (int32_t)(perm[c] - cin);
    const double v = val ? (double)val[t] : 0.0;
    int64_t p = n;
    while (p > 0 && ocol[o + p - 1] > cc) {
      ocol[o + p] = ocol[o + p - 1];
      if (oval) oval[o + p] = oval[o + p - 1];
      --p;
    }
    ocol[o + p] = cc;
    if (oval) oval[o + p] = v;
    ++n;
  }
}

mskm_status export_block(mskm_hier* h, int k, int j, int64_t* rowptr, int32_t* col, double* val, int64_t* nnz_out,
                         const int64_t* rows_host, int64_t nrows_sel, const Csr* csr) {
  hipStream_t s = h->ctx->stream;
  const Csr& C = csr ? *csr : (k == j) ? h->diag : h->lower;
  const int64_t row_off = h->h_in_off[k];
  const int64_t nrows = rows_host ? nrows_sel : h->h_off[k + 1] - h->h_off[k];
  const int64_t c0 = h->h_off[j], c1 = h->h_off[j + 1];
  const int64_t cin = h->h_in_off[j];
  int64_t* rows = nullptr;
  if (rows_host) {
    MSKM_TRY(dalloc(&rows, nrows));
    MSKM_HIP_TRY(hipMemcpy(rows, rows_host, nrows * 8, hipMemcpyHostToDevice));
  }
  struct FreeRows {
    int64_t* p;
    ~FreeRows() { (void)hipFree(p); }
  } free_rows{rows};
  int64_t *cnt = nullptr, *optr = nullptr, *part = nullptr;
  MSKM_TRY(dalloc(&cnt, nrows + 1));
  MSKM_TRY(dalloc(&optr, nrows + 1));
  MSKM_TRY(dalloc(&part, scan_parts(nrows + 1)));
  MSKM_HIP_TRY(hipMemsetAsync(cnt + nrows, 0, 8, s));
  if (nrows > 0)
    hipLaunchKernelGGL(k_export_count, dim3(grid_for(nrows, kBlock)), dim3(kBlock), 0, s, C.rowptr, C.col, h->iperm,
                       row_off, nrows, c0, c1, rows, cnt);
  mskm_status st = exclusive_scan_i64(s, cnt, optr, nrows + 1, part);
  if (st == MSKM_OK && hipStreamSynchronize(s) != hipSuccess) st = fail(MSKM_EDEVICE, "export scan");
  (void)hipFree(part);
  int64_t nnz = 0;
  if (st == MSKM_OK) {
    (void)hipMemcpy(&nnz, optr + nrows, 8, hipMemcpyDeviceToHost);
    if (nnz_out) *nnz_out = nnz;
  }
  if (st == MSKM_OK && col != nullptr) {
    int32_t* ocol = nullptr;
    double* oval = nullptr;
    st = dalloc(&ocol, nnz);
    if (st == MSKM_OK && val) st = dalloc(&oval, nnz);
    if (st == MSKM_OK && nrows > 0) {
      if (C.val || !C.val32)
        hipLaunchKernelGGL(k_export_fill<double>, dim3(grid_for(nrows, kBlock)), dim3(kBlock), 0, s, C.rowptr, C.col,
                           C.val, h->iperm, h->perm, row_off, nrows, c0, c1, cin, rows, optr, ocol, oval);
      else
        hipLaunchKernelGGL(k_export_fill<float>, dim3(grid_for(nrows, kBlock)), dim3(kBlock), 0, s, C.rowptr, C.col,
                           C.val32, h->iperm, h->perm, row_off, nrows, c0, c1, cin, rows, optr, ocol, oval);
    }
    if (st == MSKM_OK) {
      hipError_t e = hipMemcpyAsync(rowptr, optr, (nrows + 1) * 8, hipMemcpyDeviceToHost, s);
      if (e == hipSuccess) e = hipMemcpyAsync(col, ocol, nnz * 4, hipMemcpyDeviceToHost, s);
      if (e == hipSuccess && val) e = hipMemcpyAsync(val, oval, nnz * 8, hipMemcpyDeviceToHost, s);
      if (e == hipSuccess) e = hipStreamSynchronize(s);
      if (e != hipSuccess) st = fail(MSKM_EDEVICE, std::string("export copy: ") + hipGetErrorString(e));
    }
    (void)hipFree(ocol);
    (void)hipFree(oval);
  } else if (st == MSKM_OK && rowptr) {
    (void)hipMemcpy(rowptr, optr, (nrows + 1) * 8, hipMemcpyDeviceToHost);
  }
  (void)hipFree(cnt);
  (void)hipFree(optr);
  return st;
}

}  // namespace mskm
