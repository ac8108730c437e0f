// Cell block-Jacobi preconditioner for the per-level CG solves (a build
// extension; the paper's CG is unpreconditioned). The blocks are the cells of
// each level's grid: a cell's points are consecutive internal rows and
// interact strongly (the cell side is about delta), so the dense inverses of
// these small diagonal blocks remove much of the local ill-conditioning of
// A_l at the cost of about m reads per row (m = rows of the row's block).
#include <algorithm>
#include <vector>

#include "device_common.h"

namespace mskm {

// One 64-thread workgroup per block: the dense m x m principal submatrix of
// the block's rows from the diagonal CSR rows, inverted in place by
// Gauss-Jordan elimination without pivoting (the block is SPD), in FP64,
// then symmetrized and stored. A non-positive or non-finite pivot (a block
// too ill-conditioned for this) stores the identity: that block is then left
// unpreconditioned.
__global__ void __launch_bounds__(kWave)
    k_bj_invert(const int64_t* __restrict__ start, const int64_t* __restrict__ off, const int64_t* __restrict__ rp,
                const int32_t* __restrict__ col, const double* __restrict__ val, const float* __restrict__ val32,
                double* __restrict__ inv, float* __restrict__ inv32) {
  __shared__ double M[kBjMax][kBjMax + 1];
  __shared__ double F[kBjMax];
  const int64_t b = blockIdx.x;
  const int64_t a = start[b];
  const int m = (int)(start[b + 1] - a);
  const int t = threadIdx.x;
  if (t < m)
    for (int i = 0; i < m; ++i) M[i][t] = 0.0;
  __syncthreads();
  if (t < m) {
    for (int64_t k = rp[a + t]; k < rp[a + t + 1]; ++k) {
      const int64_t c = col[k];
      if (c >= a && c < a + m) M[t][c - a] = val ? val[k] : (double)val32[k];
    }
  }
  __syncthreads();
  bool bad = false;
  for (int k = 0; k < m; ++k) {
    const double piv = M[k][k];
    bad = bad || !(piv > 0.0) || !isfinite(piv);
    double rk = 0.0;
    if (t < m) {
      rk = (t == k ? 1.0 : M[k][t]) / piv;
      F[t] = t == k ? 0.0 : M[t][k];
    }
    __syncthreads();
    if (t < m) {
      for (int i = 0; i < m; ++i) M[i][t] = i == k ? rk : (t == k ? 0.0 : M[i][t]) - F[i] * rk;
    }
    __syncthreads();
  }
  const int64_t o = off[b];
  if (t < m) {
    for (int j = 0; j < m; ++j) {
      double v = 0.5 * (M[t][j] + M[j][t]);
      if (bad || !isfinite(v)) v = t == j ? 1.0 : 0.0;
      if (inv) inv[o + (int64_t)t * m + j] = v;
      if (inv32) inv32[o + (int64_t)t * m + j] = (float)v;
    }
  }
}

// of_row[r] = b for the rows of block b.
__global__ void __launch_bounds__(kBlock) k_bj_rows(int64_t nb, const int64_t* __restrict__ start,
                                                    int32_t* __restrict__ of_row) {
  const int64_t b = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (b >= nb) return;
  for (int64_t r = start[b]; r < start[b + 1]; ++r) of_row[r] = (int32_t)b;
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
  const int64_t cs_total = (int64_t)last.cs_off + last.ncell_tot + 1;
  std::vector<int32_t> cs((size_t)cs_total);
  MSKM_HIP_TRY(hipMemcpyAsync(cs.data(), h->cell_start, cs.size() * 4, hipMemcpyDeviceToHost, s));
  MSKM_HIP_TRY(hipStreamSynchronize(s));
  // blocks = cells (cut into near-equal chunks of <= kBjMax rows); groups =
  // runs of whole blocks of one level with <= kBjGroupRows rows
  std::vector<int64_t> start, off;
  std::vector<int32_t> glev;
  std::vector<int64_t> g0, g1;
  B.wt.h_lev_begin.assign(L + 1, 0);
  int64_t nv = 0;
  for (int l = 0; l < L; ++l) {
    B.wt.h_lev_begin[l] = (int32_t)glev.size();
    const DevLevel& D = h->h_lev[l];
    int64_t ga = -1, ge = -1;
    for (int c = 0; c < D.ncell_tot; ++c) {
      const int64_t a = cs[(size_t)D.cs_off + c], e = cs[(size_t)D.cs_off + c + 1];
      if (e <= a) continue;
      const int64_t nch = (e - a + kBjMax - 1) / kBjMax;
      for (int64_t q = 0; q < nch; ++q) {
        const int64_t ca = a + (e - a) * q / nch, ce = a + (e - a) * (q + 1) / nch;
        start.push_back(ca);
        off.push_back(nv);
        nv += (ce - ca) * (ce - ca);
        if (ga >= 0 && ce - ga > kBjGroupRows) {
          glev.push_back(l);
          g0.push_back(ga);
          g1.push_back(ge);
          ga = -1;
        }
        if (ga < 0) ga = ca;
        ge = ce;
      }
    }
    if (ga >= 0) {
      glev.push_back(l);
      g0.push_back(ga);
      g1.push_back(ge);
    }
    if (ge >= 0 && ge != h->h_off[l + 1]) return fail(MSKM_EDEVICE, "block-Jacobi blocks do not tile a level");
  }
  B.wt.h_lev_begin[L] = (int32_t)glev.size();
  start.push_back(h->N);
  off.push_back(nv);
  B.nblocks = (int64_t)start.size() - 1;
  B.nvals = nv;
  if (glev.size() > (size_t)INT32_MAX || B.nblocks > (int64_t)INT32_MAX)
    return fail(MSKM_ELIMIT, "block-Jacobi tables too large");
  MSKM_TRY(halloc(h, &B.start, start.size()));
  MSKM_TRY(halloc(h, &B.off, off.size()));
  MSKM_TRY(halloc(h, &B.of_row, (size_t)h->N));
  MSKM_HIP_TRY(hipMemcpyAsync(B.start, start.data(), start.size() * 8, hipMemcpyHostToDevice, s));
  MSKM_HIP_TRY(hipMemcpyAsync(B.off, off.data(), off.size() * 8, hipMemcpyHostToDevice, s));
  if (h->diag.val) MSKM_TRY(halloc(h, &B.inv, (size_t)nv));
  if (h->diag.val32) MSKM_TRY(halloc(h, &B.inv32, (size_t)nv));
  if (B.nblocks > 0) {
    hipLaunchKernelGGL(k_bj_rows, dim3((unsigned)((B.nblocks + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, B.nblocks,
                       B.start, B.of_row);
    hipLaunchKernelGGL(k_bj_invert, dim3((unsigned)B.nblocks), dim3(kWave), 0, s, B.start, B.off, h->diag.rowptr,
                       h->diag.col, h->diag.val, h->diag.val32, B.inv, B.inv32);
  }
  WorkTable& wt = B.wt;
  wt.nblocks = (int32_t)glev.size();
  wt.rows_per_block = kBjGroupRows;
  MSKM_TRY(halloc(h, &wt.lev, glev.size()));
  MSKM_TRY(halloc(h, &wt.row0, g0.size()));
  MSKM_TRY(halloc(h, &wt.row1, g1.size()));
  MSKM_TRY(halloc(h, &wt.lev_begin, wt.h_lev_begin.size()));
  if (!glev.empty()) {
    MSKM_HIP_TRY(hipMemcpyAsync(wt.lev, glev.data(), glev.size() * 4, hipMemcpyHostToDevice, s));
    MSKM_HIP_TRY(hipMemcpyAsync(wt.row0, g0.data(), g0.size() * 8, hipMemcpyHostToDevice, s));
    MSKM_HIP_TRY(hipMemcpyAsync(wt.row1, g1.data(), g1.size() * 8, hipMemcpyHostToDevice, s));
  }
  MSKM_HIP_TRY(hipMemcpyAsync(wt.lev_begin, wt.h_lev_begin.data(), wt.h_lev_begin.size() * 4, hipMemcpyHostToDevice,
                              s));
  MSKM_HIP_TRY(hipStreamSynchronize(s));
  MSKM_HIP_TRY(hipGetLastError());
  B.built = true;
  return MSKM_OK;
}

}  // namespace mskm
