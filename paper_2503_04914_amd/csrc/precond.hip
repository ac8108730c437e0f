// Cell block-Jacobi preconditioner for the per-level CG solves (a build
// extension; the paper's CG is unpreconditioned). The blocks are the cells of
// each level's grid: a cell's points are consecutive internal rows and
// interact strongly (the cell side is about delta), so the dense inverses of
// these small diagonal blocks remove much of the local ill-conditioning of
// A_l at the cost of about m reads per row (m = rows of the row's block).
#include <vector>

#include "device_common.h"

namespace mskm {

// Lane `lane`'s value of v (a wave-uniform lane), for every lane.
__device__ __forceinline__ double readlane_d(double v, int lane) {
  const int64_t u = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(u & 0xffffffff), lane);
  const int hi = __builtin_amdgcn_readlane((int)(u >> 32), lane);
  return __longlong_as_double(((int64_t)hi << 32) | (uint32_t)lo);
}

// One 64-thread workgroup per block: the dense m x m principal submatrix of
// the block's rows, gathered from the diagonal CSR rows (the block's rows are
// consecutive, so their entries form one contiguous run that the wave reads
// coalesced; each entry finds its row among the block's m + 1 row pointers),
// inverted in place by Gauss-Jordan elimination without pivoting (the block
// is SPD), in FP64, then symmetrized and stored. Lane t keeps column t in
// registers during the elimination; the pivot row is each lane's own entry
// and the pivot column is read lane by lane. A non-positive or non-finite
// pivot (a block too ill-conditioned for this) stores the identity: that
// block is then left unpreconditioned.
__global__ void __launch_bounds__(kWave)
    k_bj_invert(int64_t b0, const int64_t* __restrict__ start, const int64_t* __restrict__ off,
                const int64_t* __restrict__ rp, const int32_t* __restrict__ col, const double* __restrict__ val,
                const float* __restrict__ val32, double* __restrict__ inv, float* __restrict__ inv32) {
  __shared__ double M[kBjMax][kBjMax + 1];
  __shared__ int64_t rps[kBjMax + 1];
  const int64_t b = b0 + blockIdx.x;
  const int64_t a = start[b];
  const int m = (int)(start[b + 1] - a);
  const int t = threadIdx.x;
  for (int k = t; k < kBjMax * (kBjMax + 1); k += kWave) (&M[0][0])[k] = 0.0;
  if (t <= m) rps[t] = rp[a + t];
  __syncthreads();
  // the run of entries in batches of 4 per lane, loads of a batch issued together
  constexpr int kU = 4;
  const int64_t k1 = rps[m];
  for (int64_t kk = rps[0] + t; kk < k1; kk += kU * kWave) {
    int64_t c[kU];
    double v[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int64_t k = kk + u * kWave;
      c[u] = k < k1 ? col[k] : -1;
      v[u] = k < k1 ? (val ? val[k] : (double)val32[k]) : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kU; ++u)
      if (c[u] >= a && c[u] < a + m) {
        const int64_t k = kk + u * kWave;
        int lo = 0, hi = m - 1;  // the row of entry k: the last i with rps[i] <= k
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (rps[mid] <= k)
            lo = mid;
          else
            hi = mid - 1;
        }
        M[lo][c[u] - a] = v[u];
      }
  }
  __syncthreads();
  double cc[kBjMax];  // column t
#pragma unroll
  for (int i = 0; i < kBjMax; ++i) cc[i] = M[i][t < kBjMax ? t : 0];
  bool bad = false;
#pragma unroll
  for (int k = 0; k < kBjMax; ++k) {
    if (k < m) {
      const double piv = readlane_d(cc[k], k);
      bad = bad || !(piv > 0.0) || !isfinite(piv);
      const double rk = (t == k ? 1.0 : cc[k]) / piv;  // row k of the new matrix, entry t
#pragma unroll
      for (int i = 0; i < kBjMax; ++i)
        if (i < m) {
          const double fi = readlane_d(cc[i], k);  // entry i of the pivot column
          cc[i] = i == k ? rk : (t == k ? 0.0 : cc[i]) - fi * rk;
        }
    }
  }
  __syncthreads();
  if (t < m)
#pragma unroll
    for (int i = 0; i < kBjMax; ++i)
      if (i < m) M[i][t] = cc[i];
  __syncthreads();
  const int64_t o = off[b];
  for (int q = t; q < m * m; q += kWave) {
    const int i = q / m, j = q - i * m;
    double v = 0.5 * (M[i][j] + M[j][i]);
    if (bad || !isfinite(v)) v = i == j ? 1.0 : 0.0;
    if (inv) inv[o + q] = v;
    if (inv32) inv32[o + q] = (float)v;
  }
}

// Blocks of cell-table slot k: the cell's rows cut into ceil(count / kBjMax)
// near-equal chunks. cell_start is one array over all levels; each level's
// table ends in the level's end row, which is also the next level's first
// row, so those closing slots count zero rows. nch[nslots] = 0 closes the
// scan.
__global__ void __launch_bounds__(kBlock)
    k_bj_cell_chunks(const int32_t* __restrict__ cs, int64_t nslots, int64_t* __restrict__ nch) {
  const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (k > nslots) return;
  nch[k] = k < nslots ? (cs[k + 1] - cs[k] + kBjMax - 1) / kBjMax : 0;
}

// Block tables from the exclusive scan bbase of the chunk counts: the first
// row of each block, its m^2 (scanned next into the inverse offsets) and the
// block of every row; the closing entries start[nb] = N and msq[nb] = 0.
__global__ void __launch_bounds__(kBlock)
    k_bj_blocks(const int32_t* __restrict__ cs, int64_t nslots, const int64_t* __restrict__ bbase,
                int64_t* __restrict__ start, int64_t* __restrict__ msq, int32_t* __restrict__ of_row) {
  const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (k > nslots) return;
  if (k == nslots) {
    start[bbase[k]] = cs[k];
    msq[bbase[k]] = 0;
    return;
  }
  const int64_t a = cs[k], e = cs[k + 1], nc = bbase[k + 1] - bbase[k];
  for (int64_t q = 0; q < nc; ++q) {
    const int64_t ca = a + (e - a) * q / nc, ce = a + (e - a) * (q + 1) / nc;
    const int64_t b = bbase[k] + q;
    start[b] = ca;
    msq[b] = (ce - ca) * (ce - ca);
    for (int64_t r = ca; r < ce; ++r) of_row[r] = (int32_t)b;
  }
}

// Workgroups of whole blocks: within a level, the blocks whose first row
// falls in one window of step = bj_group_step(n) rows (windows counted from
// the level's first row) form one group, so a group spans at most step - 1 +
// kBjMax <= kBjGroupRows rows. Any window of at least kBjMax rows holds a
// block start (blocks have at most kBjMax rows); a shorter last window is
// merged into the one before it (at most step + kBjMax - 1 rows).
// gbase = first group of each level, its window count gbase[l+1] - gbase[l].
__global__ void __launch_bounds__(kBlock)
    k_bj_groups(int64_t nb, const int64_t* __restrict__ start, const DevLevel* __restrict__ lev, int L,
                const int32_t* __restrict__ gbase, int32_t* __restrict__ glev, int64_t* __restrict__ row0,
                int64_t* __restrict__ row1) {
  const int64_t b = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (b >= nb) return;
  const int64_t s = start[b], e = start[b + 1];
  int lo = 0, hi = L - 1;  // the level holding row s: the last with off <= s (an empty level shares its
                          // offset with the next level, so the last such level is never empty)
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (lev[mid].off <= s)
      lo = mid;
    else
      hi = mid - 1;
  }
  const int64_t l0 = lev[lo].off, l1 = l0 + lev[lo].n;
  const int64_t nw = gbase[lo + 1] - gbase[lo];
  const int64_t step = bj_group_step(lev[lo].n);
  const int64_t w = min((s - l0) / step, nw - 1);
  const int64_t w0 = l0 + w * step, w1 = w == nw - 1 ? l1 : w0 + step;
  const int g = gbase[lo] + (int)w;
  if (b == 0 || start[b - 1] < w0) {
    row0[g] = s;
    glev[g] = lo;
  }
  if (e >= w1 || e == l1) row1[g] = e;
}

// u = M^-1 r over workgroups of whole blocks (r staged in LDS).
template <typename TX>
__global__ void __launch_bounds__(kBlock)
    k_bj_apply(const WorkTable wt, int base, const int64_t* __restrict__ start, const int32_t* __restrict__ of_row,
               const int64_t* __restrict__ off, const TX* __restrict__ inv, const TX* __restrict__ r,
               TX* __restrict__ u) {
  __shared__ TX rs[kBjGroupRows];
  const int blk = base + xcd_block_id(gridDim.x);
  const int64_t row0 = wt.row0[blk], row1 = wt.row1[blk];
  for (int64_t i = row0 + threadIdx.x; i < row1; i += kBlock) rs[i - row0] = r[i];
  __syncthreads();
  for (int64_t i = row0 + threadIdx.x; i < row1; i += kBlock) u[i] = bj_row<TX>(i, row0, rs, start, of_row, off, inv);
}

template <typename TX>
void launch_bj_apply(mskm_hier* h, int lo, int hi, const TX* r, TX* u) {
  const BlockJacobi& B = h->bj;
  const int b0 = B.wt.h_lev_begin[lo], nb = B.wt.h_lev_begin[hi + 1] - b0;
  if (nb <= 0) return;
  const TX* inv;
  if constexpr (sizeof(TX) == 8)
    inv = B.inv;
  else
    inv = B.inv32;
  hipLaunchKernelGGL(k_bj_apply<TX>, dim3(nb), dim3(kBlock), 0, h->ctx->stream, B.wt, b0, B.start, B.of_row, B.off,
                     inv, r, u);
}
template void launch_bj_apply<double>(mskm_hier*, int, int, const double*, double*);
template void launch_bj_apply<float>(mskm_hier*, int, int, const float*, float*);

mskm_status build_block_jacobi(mskm_hier* h) {
  BlockJacobi& B = h->bj;
  if (B.built) return MSKM_OK;
  hipStream_t s = h->ctx->stream;
  const int L = h->L;
  const DevLevel& last = h->h_lev[L - 1];
  // blocks = cells cut into near-equal chunks of <= kBjMax rows, built on the
  // device from the cell tables; sized first by an upper bound (one block per
  // cell slot plus one per kBjMax rows), the exact counts read back once
  const int64_t nslots = (int64_t)last.cs_off + last.ncell_tot;
  const int64_t nb_max = nslots + h->N / kBjMax + 1;
  // scratch (one allocation): chunk counts, block bases, block sizes, scan partials
  int64_t *nch = nullptr, *bbase = nullptr, *msq = nullptr, *part = nullptr;
  const size_t a1 = ((size_t)nslots + 1 + 31) / 32 * 32, a2 = ((size_t)nb_max + 1 + 31) / 32 * 32;
  int64_t* scratch = nullptr;
  const size_t scratch_bytes = 8 * (2 * a1 + a2 + (size_t)std::max(scan_parts(nslots + 1), scan_parts(nb_max + 1)));
  void* sq = nullptr;
  mskm_status st = ctx_alloc(h->ctx, scratch_bytes, &sq);  // used on the main stream only (synchronized below)
  scratch = static_cast<int64_t*>(sq);
  if (st == MSKM_OK) {
    nch = scratch;
    bbase = scratch + a1;
    msq = scratch + 2 * a1;
    part = scratch + 2 * a1 + a2;
  }
  if (st == MSKM_OK) st = halloc(h, &B.start, (size_t)nb_max + 1);
  if (st == MSKM_OK) st = halloc(h, &B.off, (size_t)nb_max + 1);
  if (st == MSKM_OK) st = halloc(h, &B.of_row, (size_t)h->N);
  // the finest depth's blocks are inverted on the side stream (when there are
  // coarser levels); blocks are numbered level by level, levels depth by depth
  const int D = (int)h->h_depth_begin.size() - 1;
  const int side0 = D >= 2 ? h->h_depth_begin[D - 1] : INT32_MAX;
  int64_t counts[3] = {0, 0, 0};
  if (st == MSKM_OK) {
    const unsigned gs = (unsigned)((nslots + kBlock) / kBlock);
    hipLaunchKernelGGL(k_bj_cell_chunks, dim3(gs), dim3(kBlock), 0, s, h->cell_start, nslots, nch);
    st = exclusive_scan_i64(s, nch, bbase, nslots + 1, part);
    if (st == MSKM_OK) {
      if (hipMemsetAsync(msq, 0, ((size_t)nb_max + 1) * 8, s) != hipSuccess) st = fail(MSKM_EDEVICE, "memset");
      hipLaunchKernelGGL(k_bj_blocks, dim3(gs), dim3(kBlock), 0, s, h->cell_start, nslots, bbase, B.start, msq,
                         B.of_row);
    }
    if (st == MSKM_OK) st = exclusive_scan_i64(s, msq, B.off, nb_max + 1, part);
    if (st == MSKM_OK && (hipMemcpyAsync(&counts[0], bbase + nslots, 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
                          hipMemcpyAsync(&counts[1], B.off + nb_max, 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
                          (side0 < L && hipMemcpyAsync(&counts[2], bbase + h->h_lev[side0].cs_off, 8,
                                                       hipMemcpyDeviceToHost, s) != hipSuccess) ||
                          hipStreamSynchronize(s) != hipSuccess))
      st = fail(MSKM_EDEVICE, "block-Jacobi counts");
  }
  ctx_release(h->ctx, scratch, scratch_bytes);
  MSKM_TRY(st);
  B.nblocks = counts[0];
  B.nvals = counts[1];
  if (B.nblocks > (int64_t)INT32_MAX) return fail(MSKM_ELIMIT, "block-Jacobi tables too large");
  if (h->diag.val) MSKM_TRY(halloc(h, &B.inv, (size_t)B.nvals));
  if (h->diag.val32) MSKM_TRY(halloc(h, &B.inv32, (size_t)B.nvals));
  // blocks [0, nb_main) on the main stream, then [nb_main, nblocks) (the
  // finest depth's levels) on the side stream
  const int64_t nb_main = side0 < L ? counts[2] : B.nblocks;
  if (nb_main > 0)
    hipLaunchKernelGGL(k_bj_invert, dim3((unsigned)nb_main), dim3(kWave), 0, s, (int64_t)0, B.start, B.off,
                       h->diag.rowptr, h->diag.col, h->diag.val, h->diag.val32, B.inv, B.inv32);
  if (nb_main < B.nblocks) {  // started by bj_start_side
    B.side_b0 = nb_main;
    B.side_level0 = side0;
    B.side_pending = true;
    B.side_started = false;
  }
  // workgroups of whole blocks: one per window of bj_group_step rows, a last
  // window shorter than kBjMax merged into the one before
  WorkTable& wt = B.wt;
  wt.h_lev_begin.assign(L + 1, 0);
  int64_t ng = 0;
  for (int l = 0; l < L; ++l) {
    wt.h_lev_begin[l] = (int32_t)ng;
    const int64_t n = h->h_lev[l].n;
    const int64_t step = bj_group_step(n);
    int64_t nw = (n + step - 1) / step;
    if (nw > 1 && n - (nw - 1) * step < kBjMax) --nw;
    ng += nw;
    if (ng > (int64_t)INT32_MAX) return fail(MSKM_ELIMIT, "block-Jacobi tables too large");
  }
  wt.h_lev_begin[L] = (int32_t)ng;
  wt.nblocks = (int32_t)ng;
  wt.rows_per_block = kBjGroupRows;
  MSKM_TRY(halloc(h, &wt.lev, (size_t)ng));
  MSKM_TRY(halloc(h, &wt.row0, (size_t)ng));
  MSKM_TRY(halloc(h, &wt.row1, (size_t)ng));
  MSKM_TRY(halloc(h, &wt.lev_begin, wt.h_lev_begin.size()));
  MSKM_TRY(upload_async(h, wt.lev_begin, wt.h_lev_begin.data(), wt.h_lev_begin.size() * 4));
  if (B.nblocks > 0)
    hipLaunchKernelGGL(k_bj_groups, dim3((unsigned)((B.nblocks + kBlock - 1) / kBlock)), dim3(kBlock), 0, s,
                       B.nblocks, B.start, h->d_lev, L, wt.lev_begin, wt.lev, wt.row0, wt.row1);
  MSKM_HIP_TRY(hipGetLastError());
  B.built = true;
  return MSKM_OK;
}

mskm_status bj_start_side(mskm_hier* h) {
  BlockJacobi& B = h->bj;
  if (!B.side_pending || B.side_started) return MSKM_OK;
  hipStream_t s = h->ctx->stream;
  if (!B.ev_tables) MSKM_HIP_TRY(hipEventCreateWithFlags(&B.ev_tables, hipEventDisableTiming));
  if (!B.ev_side) MSKM_HIP_TRY(hipEventCreateWithFlags(&B.ev_side, hipEventDisableTiming));
  MSKM_HIP_TRY(hipEventRecord(B.ev_tables, s));
  MSKM_HIP_TRY(hipStreamWaitEvent(h->ctx->side, B.ev_tables, 0));
  hipLaunchKernelGGL(k_bj_invert, dim3((unsigned)(B.nblocks - B.side_b0)), dim3(kWave), 0, h->ctx->side, B.side_b0,
                     B.start, B.off, h->diag.rowptr, h->diag.col, h->diag.val, h->diag.val32, B.inv, B.inv32);
  MSKM_HIP_TRY(hipEventRecord(B.ev_side, h->ctx->side));
  B.side_started = true;
  return MSKM_OK;
}

mskm_status bj_wait(mskm_hier* h, int hi) {
  BlockJacobi& B = h->bj;
  if (!B.side_pending || hi < B.side_level0) return MSKM_OK;
  MSKM_TRY(bj_start_side(h));
  MSKM_HIP_TRY(hipStreamWaitEvent(h->ctx->stream, B.ev_side, 0));
  B.side_pending = false;
  return MSKM_OK;
}

}  // namespace mskm
