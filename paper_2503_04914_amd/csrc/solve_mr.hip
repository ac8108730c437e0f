// Many right-hand sides in the same launches: CG on A_l X_l = B_l for every
// (level, right-hand side) pair, Jacobi sweeps / forward substitution with a
// multi-vector SpMM, FP64 residuals per right-hand side. Vectors are
// point-major [N][R] in the internal order, so the R values gathered for one
// column are contiguous and a group of lanes reads them in one coalesced
// access; every matrix entry is loaded once per SpMM and applied to all R
// right-hand sides.
//
// Lane mapping: a group of LR lanes (LR = 64 for R >= 64, else the power of
// two >= R) handles one row; lane t of the group owns right-hand sides
// t, t + LR, ... (at most kMaxRPerLane of them).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>

#include "device_common.h"

namespace mskm {

constexpr int kMaxRPerLane = 8;  // R <= 64 * 8 = 512

struct MrCfg {
  int R, LR, RM;  // right-hand sides, lanes per row, right-hand sides per lane
};

static MrCfg mr_cfg(int R) {
  int LR = 1;
  while (LR < R && LR < 64) LR <<= 1;
  return MrCfg{R, LR, (R + LR - 1) / LR};
}

// Per-(level, rhs) CG state (index l * R + r).
struct MrState {
  double rtol2, bb, rr, alpha, beta;
  double rz;  // r.z with z = M^-1 r (preconditioned), else r.r
  int32_t maxit, on, iters, done, capped, pad;
};

static unsigned mr_nblk(int64_t n, int per) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + per - 1) / per, 1 << 30));
}

// out[i*R + r] = in[perm[i]*R + r] (input -> internal), or the inverse.
template <typename TO>
__global__ void __launch_bounds__(kBlock) k_mr_to_internal(const double* __restrict__ in, const int32_t* __restrict__ perm,
                                                           TO* __restrict__ out, int64_t n, int R) {
  const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (e >= n * R) return;
  const int64_t i = e / R, r = e % R;
  out[e] = (TO)in[(int64_t)perm[i] * R + r];
}

template <typename TI>
__global__ void __launch_bounds__(kBlock) k_mr_to_input(const TI* __restrict__ in, const int32_t* __restrict__ perm,
                                                        double* __restrict__ out, int64_t n, int R) {
  const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (e >= n * R) return;
  const int64_t i = e / R, r = e % R;
  out[(int64_t)perm[i] * R + r] = (double)in[e];
}

// Y[i][:] = b[i][:] + sign * (A X)[i][:] for rows [r0, r1) (b nullable).
template <typename TV, typename TX>
__global__ void __launch_bounds__(kBlock)
    k_mr_spmm(const int64_t* __restrict__ rp, const int32_t* __restrict__ col, const TV* __restrict__ val,
              const TX* __restrict__ x, const TX* __restrict__ b, TX* __restrict__ y, TX sign, int64_t r0, int64_t r1,
              MrCfg c) {
  const int gl = threadIdx.x % c.LR;
  const int groups_per_block = kBlock / c.LR;
  const int64_t groups = (int64_t)gridDim.x * groups_per_block;
  for (int64_t i = r0 + (int64_t)blockIdx.x * groups_per_block + threadIdx.x / c.LR; i < r1; i += groups) {
    TX acc[kMaxRPerLane];
#pragma unroll
    for (int m = 0; m < kMaxRPerLane; ++m) acc[m] = 0;
    const int64_t ke = rp[i + 1];
    for (int64_t k = rp[i]; k < ke; ++k) {
      const TX v = (TX)val[k];
      const TX* xr = x + (int64_t)col[k] * c.R;
#pragma unroll
      for (int m = 0; m < kMaxRPerLane; ++m) {
        const int r = gl + m * c.LR;
        if (m < c.RM && r < c.R) acc[m] += v * xr[r];
      }
    }
#pragma unroll
    for (int m = 0; m < kMaxRPerLane; ++m) {
      const int r = gl + m * c.LR;
      if (m < c.RM && r < c.R) y[i * c.R + r] = (b ? b[i * c.R + r] : (TX)0) + sign * acc[m];
    }
  }
}

// Block partials of per-rhs sums: each lane holds acc[m] for rhs gl + m*LR;
// the block's row groups are combined in LDS; part[blk*R + r].
__device__ __forceinline__ void mr_block_partial(const double* acc, const MrCfg& c, double* sm, double* part,
                                                 int blk) {
  const int gl = threadIdx.x % c.LR, grp = threadIdx.x / c.LR, ngrp = kBlock / c.LR;
  for (int m = 0; m < c.RM; ++m) {
    const int r = gl + m * c.LR;
    if (r < c.R) sm[grp * c.R + r] = acc[m];
  }
  __syncthreads();
  for (int r = threadIdx.x; r < c.R; r += kBlock) {
    double s = 0.0;
    for (int g = 0; g < ngrp; ++g) s += sm[g * c.R + r];
    part[(size_t)blk * c.R + r] = s;
  }
  __syncthreads();
}

constexpr int kMrLds = kBlock * kMaxRPerLane;  // doubles of LDS for block partials

// ---------------------------------------------------------------- wave rows
// Fast path for R a multiple of 64: one wave per row, lane gl owns RM
// consecutive right-hand sides gl RM .. gl RM + RM - 1 of a chunk, so a
// gathered row of X is one RM-wide load per lane. A row's entries are read
// 64 at a time by the lanes and broadcast with readlane, and gathered in
// batches of eight, two batches in flight (mr_row_acc), instead of one
// dependent chain of index load -> gather per entry. The CG product takes
// the right-hand sides in chunks (blockIdx.y, the slowest launch dimension):
// in chunks of 64 the rows of X the running workgroups gather are 256 bytes
// (FP32) wide, a working set the L2 holds better. On the 1M-row Halton level,
// 256 right-hand sides, it takes 2.70 ms in chunks of 64, 3.14 ms in chunks
// of 128 and 3.22 ms unchunked. The lower products and the
// residual read rows with entries in every coarser level, whose re-reading
// per chunk costs more than the narrower gathers save (the top level's lower
// product 1.6 ms unchunked, 2.3 ms in chunks of 64): one chunk of all R.
inline bool mr_wave_rows(const MrCfg& c) { return c.LR == 64 && c.R == 64 * c.RM; }

template <int RM, typename T>
__device__ __forceinline__ void ld_rm(const T* __restrict__ p, T (&v)[RM]) {
  typedef T vec __attribute__((ext_vector_type(RM)));
  const vec u = *reinterpret_cast<const vec*>(p);
#pragma unroll
  for (int m = 0; m < RM; ++m) v[m] = u[m];
}
template <int RM, typename T>
__device__ __forceinline__ void st_rm(T* __restrict__ p, const T (&v)[RM]) {
  typedef T vec __attribute__((ext_vector_type(RM)));
  vec u;
#pragma unroll
  for (int m = 0; m < RM; ++m) u[m] = v[m];
  *reinterpret_cast<vec*>(p) = u;
}
template <>
__device__ __forceinline__ void ld_rm<1, float>(const float* __restrict__ p, float (&v)[1]) { v[0] = *p; }
template <>
__device__ __forceinline__ void ld_rm<1, double>(const double* __restrict__ p, double (&v)[1]) { v[0] = *p; }
template <>
__device__ __forceinline__ void st_rm<1, float>(float* __restrict__ p, const float (&v)[1]) { *p = v[0]; }
template <>
__device__ __forceinline__ void st_rm<1, double>(double* __restrict__ p, const double (&v)[1]) { *p = v[0]; }

__device__ __forceinline__ int32_t lane_bcast(int32_t v, int l) { return __builtin_amdgcn_readlane(v, l); }
__device__ __forceinline__ float lane_bcast(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ __forceinline__ double lane_bcast(double v, int l) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
  return __hiloint2double(hi, lo);
}

// acc[m] += sum over the entries k in [s, e) of value(k) * X[col[k]][gl RM + m],
// in entry order. value(k) returns the entry's value in the accumulation type TA.
// The entries of a 64-entry run are taken in batches of eight gathers; the
// next batch's gathers are issued before the current batch's products, so
// two batches are in flight. Entry j of the run is lane j's: lanes past the
// run's end hold value 0 and the run's last column, so no batch needs a
// bounds branch (a batch starts below the run's end and ends at lane 63 at
// most).
template <int RM, typename TA, typename TX>
__device__ __forceinline__ void mr_gather8(const TX* __restrict__ x, int64_t ldx, int gl, int32_t cl, int u,
                                           TX (&xv)[8][RM]) {
#pragma unroll
  for (int q = 0; q < 8; ++q) ld_rm<RM>(x + (int64_t)lane_bcast(cl, u + q) * ldx + gl * RM, xv[q]);
}
template <int RM, typename TA, typename TX>
__device__ __forceinline__ void mr_fma8(TA vl, int u, const TX (&xv)[8][RM], TA (&acc)[RM]) {
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const TA v = lane_bcast(vl, u + q);
#pragma unroll
    for (int m = 0; m < RM; ++m) acc[m] += v * (TA)xv[q][m];
  }
}
template <int RM, typename TA, typename TX, typename ValueOf>
__device__ __forceinline__ void mr_row_acc(int64_t s, int64_t e, const int32_t* __restrict__ col, ValueOf value,
                                           const TX* __restrict__ x, int64_t ldx, int gl, TA (&acc)[RM]) {
  const int lane = threadIdx.x % 64;
  for (int64_t k0 = s; k0 < e; k0 += 64) {
    const int n = (int)min<int64_t>(64, e - k0);
    const int64_t k = k0 + min(lane, n - 1);
    const int32_t cl = col[k];
    const TA vl = lane < n ? value(k) : (TA)0;
    const int nb = (n + 7) / 8;
    TX xa[8][RM], xb[8][RM];
    mr_gather8<RM, TA, TX>(x, ldx, gl, cl, 0, xa);
    for (int b = 0; b < nb; b += 2) {
      if (b + 1 < nb) mr_gather8<RM, TA, TX>(x, ldx, gl, cl, 8 * (b + 1), xb);
      mr_fma8<RM, TA, TX>(vl, 8 * b, xa, acc);
      if (b + 2 < nb) mr_gather8<RM, TA, TX>(x, ldx, gl, cl, 8 * (b + 2), xa);
      if (b + 1 < nb) mr_fma8<RM, TA, TX>(vl, 8 * (b + 1), xb, acc);
    }
  }
}

// Block partials for the wave-row mapping: acc[m] belongs to rhs c0 + gl RM
// + m of the chunk of 64 RM right-hand sides starting at c0; part[blk][ldr].
template <int RM>
__device__ __forceinline__ void mr_block_partial_w(const double (&acc)[RM], double* sm, double* part, int blk,
                                                   int ldr = 64 * RM, int c0 = 0) {
  constexpr int R = 64 * RM, ngrp = kBlock / 64;
  const int gl = threadIdx.x % 64, grp = threadIdx.x / 64;
#pragma unroll
  for (int m = 0; m < RM; ++m) sm[grp * R + gl * RM + m] = acc[m];
  __syncthreads();
  for (int r = threadIdx.x; r < R; r += kBlock) {
    double t = 0.0;
    for (int g = 0; g < ngrp; ++g) t += sm[g * R + r];
    part[(size_t)blk * ldr + c0 + r] = t;
  }
  __syncthreads();
}

// Reductions over a level's per-block partials part[b][R]: one block of
// kMrRedThreads threads per (level, chunk of 64 right-hand sides); thread
// (k, r) sums the partials b = lev_begin + k, k + kMrRedLanes, ... of rhs r,
// then the kMrRedLanes sums of each rhs are added in LDS in a fixed order
// (deterministic).
constexpr int kMrRedLanes = 16;
constexpr int kMrRedThreads = 64 * kMrRedLanes;

__device__ __forceinline__ double mr_level_sum(const double* __restrict__ part, int b0, int b1, int R, int r,
                                               double* sm) {
  const int k = threadIdx.x / 64, rl = threadIdx.x % 64;
  double v = 0.0;
  if (r < R)
    for (int b = b0 + k; b < b1; b += kMrRedLanes) v += part[(size_t)b * R + r];
  sm[k * 64 + rl] = v;
  __syncthreads();
  double t = 0.0;
  if (k == 0)
    for (int q = 0; q < kMrRedLanes; ++q) t += sm[q * 64 + rl];
  __syncthreads();
  return t;  // valid in the threads with k == 0
}

// init: X = 0, Rv = B, P = 0; partials of b.b and r.r per rhs.
template <typename TX>
__global__ void __launch_bounds__(kBlock)
    k_mr_init(const WorkTable wt, int base, const TX* __restrict__ b, TX* __restrict__ x, TX* __restrict__ r,
              TX* __restrict__ p, const MrState* __restrict__ st, double* __restrict__ bbp, MrCfg c) {
  __shared__ double sm[kMrLds];
  const int blk = base + xcd_block_id(gridDim.x);
  const int l = wt.lev[blk];
  const int gl = threadIdx.x % c.LR;
  double acc[kMaxRPerLane];
  for (int m = 0; m < kMaxRPerLane; ++m) acc[m] = 0.0;
  for (int64_t i = wt.row0[blk] + threadIdx.x / c.LR; i < wt.row1[blk]; i += kBlock / c.LR) {
    for (int m = 0; m < c.RM; ++m) {
      const int rr = gl + m * c.LR;
      if (rr >= c.R || !st[(size_t)l * c.R + rr].on) continue;
      const int64_t e = i * c.R + rr;
      const TX bi = b[e];
      x[e] = (TX)0;
      r[e] = bi;
      p[e] = (TX)0;
      acc[m] += (double)bi * (double)bi;
    }
  }
  mr_block_partial(acc, c, sm, bbp, blk);
}

// Initial state (r = b, so rr = bb); grid (levels, rhs chunks of 64). The
// level's done flag is set by the host-visible all-stopped test of red_b.
__global__ void __launch_bounds__(kMrRedThreads) k_mr_red_init(int lev0, const int32_t* __restrict__ lev_begin,
                                                               const double* __restrict__ bbp,
                                                               const int32_t* __restrict__ zlev_begin,
                                                               const double* __restrict__ rzp,
                                                               MrState* __restrict__ st, MrCfg c) {
  __shared__ double sm[kMrRedThreads];
  const int l = lev0 + blockIdx.x;
  const int r = blockIdx.y * 64 + (int)(threadIdx.x % 64);
  const double bb = mr_level_sum(bbp, lev_begin[l], lev_begin[l + 1], c.R, r, sm);
  const double rz = rzp ? mr_level_sum(rzp, zlev_begin[l], zlev_begin[l + 1], c.R, r, sm) : bb;
  if (threadIdx.x < 64 && r < c.R) {
    MrState& S = st[(size_t)l * c.R + r];
    S.bb = bb;
    S.rr = bb;
    S.rz = rz;
    S.alpha = S.beta = 0.0;
    S.iters = 0;
    const bool finite = isfinite(bb);
    const bool conv = finite && !(bb > S.rtol2 * bb);
    S.capped = S.on && !conv && (!finite || S.maxit <= 0);
    S.done = !S.on || conv || S.capped;
  }
}

// lev_done[l] = every system of level l has stopped (one block per level).
__global__ void __launch_bounds__(kBlock) k_mr_lev_done(int lev0, const MrState* __restrict__ st,
                                                        int32_t* __restrict__ lev_done, MrCfg c) {
  __shared__ int any;
  const int l = lev0 + blockIdx.x;
  if (threadIdx.x == 0) any = 0;
  __syncthreads();
  for (int r = threadIdx.x; r < c.R; r += kBlock)
    if (!st[(size_t)l * c.R + r].done) any = 1;
  __syncthreads();
  if (threadIdx.x == 0) lev_done[l] = !any;
}

// p = r + beta p (per element of not-stopped systems).
template <typename TX>
__global__ void __launch_bounds__(kBlock)
    k_mr_dir(const WorkTable wt, int base, const TX* __restrict__ r, TX* __restrict__ p,
             const MrState* __restrict__ st, const int32_t* __restrict__ lev_done, MrCfg c) {
  // r here is the direction's source: the residual, or z = M^-1 r when
  // preconditioned. Lane gl of a row group owns right-hand sides gl + m LR:
  // their state is read once, then the group's rows are streamed (a group's
  // lanes touch consecutive entries of a row).
  const int blk = base + xcd_block_id(gridDim.x);
  const int l = wt.lev[blk];
  if (lev_done[l]) return;
  const int gl = threadIdx.x % c.LR;
  TX beta[kMaxRPerLane];
  bool run[kMaxRPerLane];
#pragma unroll
  for (int m = 0; m < kMaxRPerLane; ++m) {
    const int rr = gl + m * c.LR;
    run[m] = m < c.RM && rr < c.R && !st[(size_t)l * c.R + rr].done;
    beta[m] = run[m] ? (TX)st[(size_t)l * c.R + rr].beta : (TX)0;
  }
  for (int64_t i = wt.row0[blk] + threadIdx.x / c.LR; i < wt.row1[blk]; i += kBlock / c.LR) {
#pragma unroll
    for (int m = 0; m < kMaxRPerLane; ++m) {
      if (!run[m]) continue;
      const int64_t e = i * c.R + gl + m * c.LR;
      p[e] = r[e] + beta[m] * p[e];
    }
  }
}

// Q = A P on the block's rows; partial p.q per rhs.
template <typename TV, typename TX>
__global__ void __launch_bounds__(kBlock)
    k_mr_cg_spmm(const WorkTable wt, int base, const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                 const TV* __restrict__ val, const TX* __restrict__ p, TX* __restrict__ q,
                 const int32_t* __restrict__ lev_done, double* __restrict__ pqp, MrCfg c) {
  __shared__ double sm[kMrLds];
  const int blk = base + xcd_block_id(gridDim.x);
  const int l = wt.lev[blk];
  if (lev_done[l]) return;
  const int gl = threadIdx.x % c.LR;
  double part[kMaxRPerLane];
#pragma unroll
  for (int m = 0; m < kMaxRPerLane; ++m) part[m] = 0.0;
  for (int64_t i = wt.row0[blk] + threadIdx.x / c.LR; i < wt.row1[blk]; i += kBlock / c.LR) {
    TX acc[kMaxRPerLane];
#pragma unroll
    for (int m = 0; m < kMaxRPerLane; ++m) acc[m] = 0;
    const int64_t ke = rp[i + 1];
    for (int64_t k = rp[i]; k < ke; ++k) {
      const TX v = (TX)val[k];
      const TX* pr = p + (int64_t)col[k] * c.R;
#pragma unroll
      for (int m = 0; m < kMaxRPerLane; ++m) {
        const int r = gl + m * c.LR;
        if (m < c.RM && r < c.R) acc[m] += v * pr[r];
      }
    }
#pragma unroll
    for (int m = 0; m < kMaxRPerLane; ++m) {
      const int r = gl + m * c.LR;
      if (m < c.RM && r < c.R) {
        q[i * c.R + r] = acc[m];
        part[m] += (double)p[i * c.R + r] * (double)acc[m];
      }
    }
  }
  mr_block_partial(part, c, sm, pqp, blk);
}

// alpha = rr / p.q per system; grid (levels, rhs chunks of 64).
__global__ void __launch_bounds__(kMrRedThreads) k_mr_red_a(int lev0, const int32_t* __restrict__ lev_begin,
                                                            const double* __restrict__ pqp, MrState* __restrict__ st,
                                                            const int32_t* __restrict__ lev_done, MrCfg c) {
  __shared__ double sm[kMrRedThreads];
  const int l = lev0 + blockIdx.x;
  if (lev_done[l]) return;
  const int r = blockIdx.y * 64 + (int)(threadIdx.x % 64);
  const double pq = mr_level_sum(pqp, lev_begin[l], lev_begin[l + 1], c.R, r, sm);
  if (threadIdx.x < 64 && r < c.R) {
    MrState& S = st[(size_t)l * c.R + r];
    if (S.done) return;
    if (pq > 0.0 && isfinite(pq)) {
      S.alpha = S.rz / pq;
    } else {
      S.alpha = 0.0;
      S.done = 1;
      S.capped = !(S.rr <= S.rtol2 * S.bb);
    }
  }
}

// X += alpha P; R -= alpha Q; partial r.r per rhs.
template <typename TX>
__global__ void __launch_bounds__(kBlock)
    k_mr_update(const WorkTable wt, int base, TX* __restrict__ x, TX* __restrict__ r, const TX* __restrict__ p,
                const TX* __restrict__ q, const MrState* __restrict__ st, const int32_t* __restrict__ lev_done,
                double* __restrict__ rrp, MrCfg c) {
  __shared__ double sm[kMrLds];
  const int blk = base + xcd_block_id(gridDim.x);
  const int l = wt.lev[blk];
  if (lev_done[l]) return;
  const int gl = threadIdx.x % c.LR;
  double acc[kMaxRPerLane], alpha[kMaxRPerLane];
  bool has[kMaxRPerLane], run[kMaxRPerLane];
#pragma unroll
  for (int m = 0; m < kMaxRPerLane; ++m) {  // the lane's systems: state read once
    const int rr = gl + m * c.LR;
    acc[m] = 0.0;
    has[m] = m < c.RM && rr < c.R;
    run[m] = has[m] && !st[(size_t)l * c.R + rr].done;
    alpha[m] = run[m] ? st[(size_t)l * c.R + rr].alpha : 0.0;
  }
  for (int64_t i = wt.row0[blk] + threadIdx.x / c.LR; i < wt.row1[blk]; i += kBlock / c.LR) {
#pragma unroll
    for (int m = 0; m < kMaxRPerLane; ++m) {
      if (!has[m]) continue;
      const int64_t e = i * c.R + gl + m * c.LR;
      if (run[m]) {
        x[e] = (TX)((double)x[e] + alpha[m] * (double)p[e]);
        r[e] = (TX)((double)r[e] - alpha[m] * (double)q[e]);
      }
      acc[m] += (double)r[e] * (double)r[e];
    }
  }
  mr_block_partial(acc, c, sm, rrp, blk);
}

// rr_new, stop test, beta per system; grid (levels, rhs chunks of 64).
__global__ void __launch_bounds__(kMrRedThreads) k_mr_red_b(int lev0, const int32_t* __restrict__ lev_begin,
                                                            const double* __restrict__ rrp,
                                                            const int32_t* __restrict__ zlev_begin,
                                                            const double* __restrict__ rzp, MrState* __restrict__ st,
                                                            const int32_t* __restrict__ lev_done, MrCfg c) {
  __shared__ double sm[kMrRedThreads];
  const int l = lev0 + blockIdx.x;
  if (lev_done[l]) return;
  const int r = blockIdx.y * 64 + (int)(threadIdx.x % 64);
  const double rr = mr_level_sum(rrp, lev_begin[l], lev_begin[l + 1], c.R, r, sm);
  const double rz = rzp ? mr_level_sum(rzp, zlev_begin[l], zlev_begin[l + 1], c.R, r, sm) : rr;
  if (threadIdx.x < 64 && r < c.R) {
    MrState& S = st[(size_t)l * c.R + r];
    if (S.done) return;
    S.iters += 1;
    const double old = S.rz;
    S.rr = rr;
    S.rz = rz;
    if (isfinite(rr) && !(rr > S.rtol2 * S.bb)) {
      S.done = 1;
    } else if (!isfinite(rr) || !isfinite(rz) || S.iters >= S.maxit) {
      S.done = 1;
      S.capped = 1;
    } else {
      S.beta = rz / old;
    }
  }
}

// Block-Jacobi product for many right-hand sides: z[i][:] = M^-1 r over the
// workgroups of whole blocks (grid: groups x chunks of 64 rhs). Wave w of a
// workgroup takes blocks w, w + 4, ... of its group; lane t holds rhs
// chunk*64 + t, keeps the block's m entries of r in registers and forms its
// m entries of z (each r value is read once per block). Partial r.z per
// (group, rhs).
template <typename TX>
__global__ void __launch_bounds__(kBlock)
    k_mr_bj_apply(const WorkTable wt, int base, const int64_t* __restrict__ start, const int32_t* __restrict__ of_row,
                  const int64_t* __restrict__ off, const TX* __restrict__ inv, const TX* __restrict__ rv,
                  TX* __restrict__ z, const int32_t* __restrict__ lev_done, double* __restrict__ rzp, MrCfg c) {
  __shared__ double sm[kBlock];
  const int blk = base + xcd_block_id(gridDim.x);
  const int l = wt.lev[blk];
  if (lev_done && lev_done[l]) return;
  const int t = threadIdx.x % 64, w = threadIdx.x / 64;
  const int rr = blockIdx.y * 64 + t;
  const bool on = rr < c.R;
  const int64_t row0 = wt.row0[blk], row1 = wt.row1[blk];
  const int32_t bfirst = of_row[row0], blast = of_row[row1 - 1];
  double acc = 0.0;
  for (int32_t b = bfirst + w; b <= blast; b += kBlock / 64) {
    const int64_t a = start[b];
    const int m = (int)(start[b + 1] - a);
    const TX* Mb = inv + off[b];
    TX x[kBjMax];
#pragma unroll
    for (int j = 0; j < kBjMax; ++j) x[j] = (on && j < m) ? rv[(a + j) * c.R + rr] : (TX)0;
    for (int i = 0; i < m; ++i) {
      TX zi = 0;
#pragma unroll
      for (int j = 0; j < kBjMax; ++j)
        if (j < m) zi += Mb[(int64_t)i * m + j] * x[j];
      if (on) z[(a + i) * c.R + rr] = zi;
      TX xi = 0;
#pragma unroll
      for (int j = 0; j < kBjMax; ++j)
        if (j == i) xi = x[j];
      acc += (double)xi * (double)zi;
    }
  }
  sm[w * 64 + t] = acc;
  __syncthreads();
  if (w == 0 && on) {
    double s = 0.0;
    for (int q = 0; q < kBlock / 64; ++q) s += sm[q * 64 + t];
    rzp[(size_t)blk * c.R + rr] = s;
  }
}

// Wave-row forms of the CG product, the SpMM and the FP64 residual (R = 64 RM).
// The CG product takes the right-hand sides in chunks of 64 RM (blockIdx.y,
// the slowest launch dimension): the rows of P that the running workgroups
// gather are then 64 RM wide, a working set the L2 holds.
template <int RM, typename TV, typename TX>
__global__ void __launch_bounds__(kBlock)
    k_mr_cg_spmm_w(const WorkTable wt, int base, const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                   const TV* __restrict__ val, const TX* __restrict__ p, TX* __restrict__ q,
                   const int32_t* __restrict__ lev_done, double* __restrict__ pqp, int ldr) {
  __shared__ double sm[kMrLds];
  const int blk = base + xcd_block_id(gridDim.x);
  const int l = wt.lev[blk];
  if (lev_done[l]) return;
  const int gl = threadIdx.x % 64;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);
  const int c0 = (int)blockIdx.y * 64 * RM;
  double part[RM];
#pragma unroll
  for (int m = 0; m < RM; ++m) part[m] = 0.0;
  for (int64_t i = wt.row0[blk] + w; i < wt.row1[blk]; i += kBlock / 64) {
    TX acc[RM];
#pragma unroll
    for (int m = 0; m < RM; ++m) acc[m] = 0;
    mr_row_acc<RM, TX, TX>(rp[i], rp[i + 1], col, [&](int64_t k) { return (TX)val[k]; }, p + c0, ldr, gl, acc);
    TX pi[RM];
    ld_rm<RM>(p + i * ldr + c0 + gl * RM, pi);
    st_rm<RM>(q + i * ldr + c0 + gl * RM, acc);
#pragma unroll
    for (int m = 0; m < RM; ++m) part[m] += (double)pi[m] * (double)acc[m];
  }
  mr_block_partial_w<RM>(part, sm, pqp, blk, ldr, c0);
}

// Y[i][:] = b[i][:] + sign (A X)[i][:] for rows [r0, r1) (b nullable), one
// wave per row, the right-hand sides in chunks of 64 RM (blockIdx.y; the
// caller launches one chunk of all R).
template <int RM, typename TV, typename TX>
__global__ void __launch_bounds__(kBlock)
    k_mr_spmm_w(const int64_t* __restrict__ rp, const int32_t* __restrict__ col, const TV* __restrict__ val,
                const TX* __restrict__ x, const TX* __restrict__ b, TX* __restrict__ y, TX sign, int64_t r0,
                int64_t r1, int ldr) {
  const int gl = threadIdx.x % 64;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);
  const int c0 = (int)blockIdx.y * 64 * RM;
  const int64_t waves = (int64_t)gridDim.x * (kBlock / 64);
  for (int64_t i = r0 + (int64_t)blockIdx.x * (kBlock / 64) + w; i < r1; i += waves) {
    TX acc[RM];
#pragma unroll
    for (int m = 0; m < RM; ++m) acc[m] = 0;
    mr_row_acc<RM, TX, TX>(rp[i], rp[i + 1], col, [&](int64_t k) { return (TX)val[k]; }, x + c0, ldr, gl, acc);
    const int64_t o = i * ldr + c0 + gl * RM;
    TX bi[RM];
    if (b) ld_rm<RM>(b + o, bi);
#pragma unroll
    for (int m = 0; m < RM; ++m) acc[m] = (b ? bi[m] : (TX)0) + sign * acc[m];
    st_rm<RM>(y + o, acc);
  }
}

// FP64 residual, one wave per row, the right-hand sides in chunks of 64 RM
// (blockIdx.y): values stored FP64, else FP32 plus the FP32 remainder;
// partials rr[blk][r], ff[blk][r].
template <int RM>
__global__ void __launch_bounds__(kBlock)
    k_mr_residual_w(const WorkTable wt, const int64_t* __restrict__ drp, const int32_t* __restrict__ dc,
                    const double* __restrict__ dv, const int64_t* __restrict__ lrp, const int32_t* __restrict__ lc,
                    const double* __restrict__ lv, const float* __restrict__ dh, const float* __restrict__ dl,
                    const float* __restrict__ lh, const float* __restrict__ ll, const double* __restrict__ a,
                    const double* __restrict__ f, double* __restrict__ rout, double* __restrict__ rrp,
                    double* __restrict__ ffp, int ldr) {
  __shared__ double sm[kMrLds];
  const int blk = xcd_block_id(gridDim.x);
  const int gl = threadIdx.x % 64;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);
  const int c0 = (int)blockIdx.y * 64 * RM;
  double prr[RM], pff[RM];
#pragma unroll
  for (int m = 0; m < RM; ++m) prr[m] = pff[m] = 0.0;
  for (int64_t i = wt.row0[blk] + w; i < wt.row1[blk]; i += kBlock / 64) {
    double acc[RM];
#pragma unroll
    for (int m = 0; m < RM; ++m) acc[m] = 0.0;
    const double* ac = a + c0;
    if (dv)
      mr_row_acc<RM, double, double>(drp[i], drp[i + 1], dc, [&](int64_t k) { return dv[k]; }, ac, ldr, gl, acc);
    else
      mr_row_acc<RM, double, double>(drp[i], drp[i + 1], dc,
                                     [&](int64_t k) { return (double)dh[k] + (double)dl[k]; }, ac, ldr, gl, acc);
    if (lv)
      mr_row_acc<RM, double, double>(lrp[i], lrp[i + 1], lc, [&](int64_t k) { return lv[k]; }, ac, ldr, gl, acc);
    else
      mr_row_acc<RM, double, double>(lrp[i], lrp[i + 1], lc,
                                     [&](int64_t k) { return (double)lh[k] + (double)ll[k]; }, ac, ldr, gl, acc);
    const int64_t o = i * ldr + c0 + gl * RM;
    double fi[RM];
    ld_rm<RM>(f + o, fi);
#pragma unroll
    for (int m = 0; m < RM; ++m) {
      acc[m] = fi[m] - acc[m];
      prr[m] += acc[m] * acc[m];
      pff[m] += fi[m] * fi[m];
    }
    if (rout) st_rm<RM>(rout + o, acc);
  }
  mr_block_partial_w<RM>(prr, sm, rrp, blk, ldr, c0);
  mr_block_partial_w<RM>(pff, sm, ffp, blk, ldr, c0);
}

// Per-level sums of block partials part[b][R] -> out[l][R] (grid: levels x
// chunks of 64 right-hand sides; fixed order).
__global__ void __launch_bounds__(kMrRedThreads) k_mr_level_sums(const int32_t* __restrict__ lev_begin,
                                                                 const double* __restrict__ part,
                                                                 double* __restrict__ out, int R) {
  __shared__ double sm[kMrRedThreads];
  const int l = blockIdx.x;
  const int r = blockIdx.y * 64 + (int)(threadIdx.x % 64);
  const double v = mr_level_sum(part, lev_begin[l], lev_begin[l + 1], R, r, sm);
  if (threadIdx.x < 64 && r < R) out[(size_t)l * R + r] = v;
}

// Block-Jacobi product in the wave-row mapping (FP32 vectors, R = 64 RM,
// RM <= 4): wave w of a workgroup takes blocks w, w + 4, ... of its group;
// lane gl holds the block's m rows of r for its RM right-hand sides (one
// RM-wide load per row), and the block's inverse entries are wave-uniform
// (scalar loads), each applied to RM right-hand sides. MB bounds the block
// size at compile time (8, 16 or 32 by the block's m). Partial r.z per
// (group, rhs).
template <int RM, int MB>
__device__ __forceinline__ void mr_bj_block(int64_t a, int m, const float* __restrict__ Mb,
                                            const float* __restrict__ rv, float* __restrict__ z, int gl,
                                            double (&acc)[RM]) {
  constexpr int R = 64 * RM;
  float x[MB][RM];
#pragma unroll
  for (int j = 0; j < MB; ++j) {
    if (j < m) {
      ld_rm<RM>(rv + (a + j) * R + gl * RM, x[j]);
    } else {
#pragma unroll
      for (int q = 0; q < RM; ++q) x[j][q] = 0.0f;
    }
  }
#pragma unroll
  for (int i = 0; i < MB; ++i) {
    if (i < m) {
      float zi[RM];
#pragma unroll
      for (int q = 0; q < RM; ++q) zi[q] = 0.0f;
#pragma unroll
      for (int j = 0; j < MB; ++j) {
        const float mij = j < m ? Mb[(int64_t)i * m + j] : 0.0f;
#pragma unroll
        for (int q = 0; q < RM; ++q) zi[q] += mij * x[j][q];
      }
      st_rm<RM>(z + (a + i) * R + gl * RM, zi);
#pragma unroll
      for (int q = 0; q < RM; ++q) acc[q] += (double)x[i][q] * (double)zi[q];
    }
  }
}

// Blocks of more than 16 rows (rare): one right-hand side of the lane at a time.
template <int RM>
__device__ __forceinline__ void mr_bj_block_big(int64_t a, int m, const float* __restrict__ Mb,
                                                const float* __restrict__ rv, float* __restrict__ z, int gl,
                                                double (&acc)[RM]) {
  constexpr int R = 64 * RM;
#pragma unroll
  for (int q = 0; q < RM; ++q) {
    float x[kBjMax];
#pragma unroll
    for (int j = 0; j < kBjMax; ++j) x[j] = j < m ? rv[(a + j) * R + gl * RM + q] : 0.0f;
    for (int i = 0; i < m; ++i) {
      float zi = 0.0f, xi = 0.0f;
#pragma unroll
      for (int j = 0; j < kBjMax; ++j) {
        zi += (j < m ? Mb[(int64_t)i * m + j] : 0.0f) * x[j];
        if (j == i) xi = x[j];
      }
      z[(a + i) * R + gl * RM + q] = zi;
      acc[q] += (double)xi * (double)zi;
    }
  }
}

template <int RM>
__global__ void __launch_bounds__(kBlock)
    k_mr_bj_apply_w(const WorkTable wt, int base, const int64_t* __restrict__ start, const int32_t* __restrict__ of_row,
                    const int64_t* __restrict__ off, const float* __restrict__ inv, const float* __restrict__ rv,
                    float* __restrict__ z, const int32_t* __restrict__ lev_done, double* __restrict__ rzp) {
  __shared__ double sm[kMrLds];
  const int blk = base + xcd_block_id(gridDim.x);
  const int l = wt.lev[blk];
  if (lev_done && lev_done[l]) return;
  const int gl = threadIdx.x % 64;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);
  const int64_t row0 = wt.row0[blk], row1 = wt.row1[blk];
  const int32_t bfirst = of_row[row0], blast = of_row[row1 - 1];
  double acc[RM];
#pragma unroll
  for (int q = 0; q < RM; ++q) acc[q] = 0.0;
  for (int32_t b = bfirst + w; b <= blast; b += kBlock / 64) {
    const int64_t a = start[b];
    const int m = (int)(start[b + 1] - a);
    const float* Mb = inv + off[b];
    if (m <= 8)
      mr_bj_block<RM, 8>(a, m, Mb, rv, z, gl, acc);
    else if (m <= 16)
      mr_bj_block<RM, 16>(a, m, Mb, rv, z, gl, acc);
    else
      mr_bj_block_big<RM>(a, m, Mb, rv, z, gl, acc);
  }
  mr_block_partial_w<RM>(acc, sm, rzp, blk);
}

// FP64 residual per rhs over the level-aligned SpMV table: partials
// rr[blk][r], ff[blk][r]. Values: stored FP64, else the split FP32 values
// (hi + remainder; an FP32-only hierarchy stores the remainders).
__global__ void __launch_bounds__(kBlock)
    k_mr_residual(const WorkTable wt, const int64_t* __restrict__ drp, const int32_t* __restrict__ dc,
                  const double* __restrict__ dv, const int64_t* __restrict__ lrp, const int32_t* __restrict__ lc,
                  const double* __restrict__ lv, const float* __restrict__ dh, const float* __restrict__ dl,
                  const float* __restrict__ lh, const float* __restrict__ ll, const double* __restrict__ a,
                  const double* __restrict__ f, double* __restrict__ rout, double* __restrict__ rrp,
                  double* __restrict__ ffp, MrCfg c) {
  __shared__ double sm[kMrLds];
  const int blk = xcd_block_id(gridDim.x);
  const int gl = threadIdx.x % c.LR;
  double prr[kMaxRPerLane], pff[kMaxRPerLane];
  for (int m = 0; m < kMaxRPerLane; ++m) prr[m] = pff[m] = 0.0;
  for (int64_t i = wt.row0[blk] + threadIdx.x / c.LR; i < wt.row1[blk]; i += kBlock / c.LR) {
    double acc[kMaxRPerLane];
    for (int m = 0; m < kMaxRPerLane; ++m) acc[m] = 0.0;
    for (int pass = 0; pass < 2; ++pass) {
      const int64_t* rp = pass == 0 ? drp : lrp;
      const int32_t* col = pass == 0 ? dc : lc;
      const double* val = pass == 0 ? dv : lv;
      const float* vh = pass == 0 ? dh : lh;
      const float* vl = pass == 0 ? dl : ll;
      for (int64_t k = rp[i]; k < rp[i + 1]; ++k) {
        const int64_t cc = col[k];
        const double v = val ? val[k] : (double)vh[k] + (double)vl[k];
        const double* ar = a + cc * c.R;
        for (int m = 0; m < c.RM; ++m) {
          const int r = gl + m * c.LR;
          if (r < c.R) acc[m] += v * ar[r];
        }
      }
    }
    for (int m = 0; m < c.RM; ++m) {
      const int r = gl + m * c.LR;
      if (r >= c.R) continue;
      const double fi = f[i * c.R + r];
      const double ri = fi - acc[m];
      if (rout) rout[i * c.R + r] = ri;
      prr[m] += ri * ri;
      pff[m] += fi * fi;
    }
  }
  mr_block_partial(prr, c, sm, rrp, blk);
  mr_block_partial(pff, c, sm, ffp, blk);
}

// Residual of a = 0 (r = f): partials of f.f for both sums.
__global__ void __launch_bounds__(kBlock)
    k_mr_residual_zero(const WorkTable wt, const double* __restrict__ f, double* __restrict__ rout,
                       double* __restrict__ rrp, double* __restrict__ ffp, MrCfg c) {
  __shared__ double sm[kMrLds];
  const int blk = xcd_block_id(gridDim.x);
  const int gl = threadIdx.x % c.LR;
  double pff[kMaxRPerLane];
  for (int m = 0; m < kMaxRPerLane; ++m) pff[m] = 0.0;
  for (int64_t i = wt.row0[blk] + threadIdx.x / c.LR; i < wt.row1[blk]; i += kBlock / c.LR) {
    for (int m = 0; m < c.RM; ++m) {
      const int r = gl + m * c.LR;
      if (r >= c.R) continue;
      const double fi = f[i * c.R + r];
      if (rout) rout[i * c.R + r] = fi;
      pff[m] += fi * fi;
    }
  }
  mr_block_partial(pff, c, sm, rrp, blk);
  mr_block_partial(pff, c, sm, ffp, blk);
}

__global__ void __launch_bounds__(kBlock) k_mr_axpy(const float* __restrict__ d, double* __restrict__ a, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) a[i] += (double)d[i];
}

__global__ void __launch_bounds__(kBlock) k_mr_to_f32(const double* __restrict__ in, float* __restrict__ out,
                                                      int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) out[i] = (float)in[i];
}

// ------------------------------------------------------------------ driver

namespace {

struct MrWS {
  MrCfg c{};
  size_t NR = 0;
  double *fi = nullptr, *ai = nullptr, *res = nullptr;
  void *beta = nullptr, *t = nullptr, *r = nullptr, *p = nullptr, *q = nullptr, *f32 = nullptr, *a32 = nullptr;
  void* z = nullptr;  // M^-1 r (block-Jacobi form)
  double *part_s = nullptr, *part_v = nullptr, *part_v2 = nullptr, *part_z = nullptr;
  bool pc = false;
  MrState* st = nullptr;
  int32_t* lev_done = nullptr;
  int32_t* h_lev_done = nullptr;
  ~MrWS() {
    for (void* v : {(void*)fi, (void*)ai, (void*)res, beta, t, r, p, q, f32, a32, z, (void*)part_s, (void*)part_v,
                    (void*)part_v2, (void*)part_z, (void*)st, (void*)lev_done})
      (void)hipFree(v);
    if (h_lev_done) (void)hipHostFree(h_lev_done);
  }
};

struct MrStats {
  int64_t iters_total = 0;
  std::vector<int32_t> last_iters;
  bool capped = false;
};

template <typename T>
__global__ void __launch_bounds__(kBlock) k_mr_fill(T* __restrict__ v, int64_t n, T x) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) v[i] = x;
}

// q = A p with the partials p.q per (block, rhs) over the blocks [b0, b0 + nb)
// of the SpMV work table (the CG product of every running level). For R a
// multiple of 64 the right-hand sides go in chunks of `chunk` (64, 128, 256
// or 512, dividing R).
template <typename TV, typename TX>
static void launch_mr_cg_product(mskm_hier* h, const MrCfg& c, int chunk, int b0, int nb, const TV* dval,
                                 const TX* p, TX* q, const int32_t* lev_done, double* part) {
  hipStream_t s = h->ctx->stream;
  const WorkTable& ws = h->wt_spmv;
  const int64_t* drp = h->diag.rowptr;
  const int32_t* dcl = h->diag.col;
  if (!mr_wave_rows(c)) {
    hipLaunchKernelGGL((k_mr_cg_spmm<TV, TX>), dim3(nb), dim3(kBlock), 0, s, ws, b0, drp, dcl, dval, p, q, lev_done,
                       part, c);
    return;
  }
  const dim3 grid(nb, c.R / chunk);
  switch (chunk / 64) {
#define MSKM_MR_CGP_W(RMV)                                                                                      \
  case RMV:                                                                                                    \
    hipLaunchKernelGGL((k_mr_cg_spmm_w<RMV, TV, TX>), grid, dim3(kBlock), 0, s, ws, b0, drp, dcl, dval, p, q,  \
                       lev_done, part, c.R);                                                                   \
    break;
    MSKM_MR_CGP_W(2)
    MSKM_MR_CGP_W(4)
    MSKM_MR_CGP_W(8)
#undef MSKM_MR_CGP_W
    default:
      hipLaunchKernelGGL((k_mr_cg_spmm_w<1, TV, TX>), dim3(nb, c.R / 64), dim3(kBlock), 0, s, ws, b0, drp, dcl, dval,
                         p, q, lev_done, part, c.R);
  }
}

// Chunk width of the CG product for this R: the fastest of the candidates
// (64, 128, 256, 512 dividing R) timed once per hierarchy, R and precision on
// its largest level, then kept (the timing overwrites q and the partials,
// which the solve rewrites). Staging each 64-row block's distinct columns of
// P in LDS instead (sorted lists, one byte per entry for its position) ran
// at half the speed of the chunked gathers: the 48-64 KB of LDS per
// workgroup leave two or three workgroups per CU.
template <typename TV, typename TX>
static int mr_chunk_for(mskm_hier* h, const MrCfg& c, const TV* dval, const TX* p, TX* q, double* part,
                        const int32_t* zeros) {
  if (!mr_wave_rows(c) || c.R / 64 > 8) return 64;
  int32_t& slot = h->mr_chunk[c.R / 64 - 1][sizeof(TX) == 4 ? 1 : 0];
  if (slot > 0) return slot;
  int big = 0;  // the largest level (a solve's first call may run only the coarsest)
  for (int l = 1; l < h->L; ++l)
    if (h->h_lev[l].n > h->h_lev[big].n) big = l;
  const WorkTable& ws = h->wt_spmv;
  const int b0 = ws.h_lev_begin[big], nb = ws.h_lev_begin[big + 1] - b0;
  hipStream_t s = h->ctx->stream;
  int best = 64;
  float best_ms = 0.f;
  for (int ch = 64; ch <= std::min(c.R, 512); ch *= 2) {
    if (c.R % ch) continue;
    launch_mr_cg_product<TV, TX>(h, c, ch, b0, nb, dval, p, q, zeros, part);  // warm
    float ms = 0.f;
    if (hipEventRecord(h->ctx->ev0, s) != hipSuccess) return 64;
    for (int k = 0; k < 2; ++k) launch_mr_cg_product<TV, TX>(h, c, ch, b0, nb, dval, p, q, zeros, part);
    if (hipEventRecord(h->ctx->ev1, s) != hipSuccess || hipEventSynchronize(h->ctx->ev1) != hipSuccess ||
        hipEventElapsedTime(&ms, h->ctx->ev0, h->ctx->ev1) != hipSuccess)
      return 64;
    if (ch == 64 || ms < best_ms) {
      best = ch;
      best_ms = ms;
    }
  }
  slot = best;
  return best;
}

template <typename TV, typename TX>
mskm_status mr_cg(mskm_hier* h, MrWS& W, const TV* dval, const std::vector<char>& on, const TX* b, TX* x, double rtol,
                  int maxit, int K, MrStats* ms) {
  hipStream_t s = h->ctx->stream;
  const MrCfg c = W.c;
  const WorkTable& ws = h->wt_spmv;
  // vector phases: 64-row blocks when each row carries 16 or more right-hand
  // sides (a 1024-row block of 512 right-hand sides left small levels to a
  // handful of workgroups), else the 1024-row streaming table
  const WorkTable& wv = c.R >= 16 ? h->wt_spmv : h->wt_vec;
  int lo = 0, hi = h->L - 1;
  while (lo < h->L && !on[lo]) ++lo;
  while (hi >= 0 && !on[hi]) --hi;
  if (lo > hi) return MSKM_OK;
  std::vector<MrState> hs((size_t)h->L * c.R);
  for (int l = 0; l < h->L; ++l)
    for (int r = 0; r < c.R; ++r) {
      MrState& S = hs[(size_t)l * c.R + r];
      std::memset(&S, 0, sizeof(S));
      S.rtol2 = rtol * rtol;
      S.maxit = maxit;
      S.on = on[l] ? 1 : 0;
      S.done = 1;
    }
  MSKM_HIP_TRY(hipMemcpyAsync(W.st, hs.data(), hs.size() * sizeof(MrState), hipMemcpyHostToDevice, s));
  std::vector<int32_t> ld(h->L, 1);
  MSKM_HIP_TRY(hipMemcpyAsync(W.lev_done, ld.data(), h->L * 4, hipMemcpyHostToDevice, s));
  const int nlev = hi - lo + 1;
  const int sb0 = ws.h_lev_begin[lo], sbn = ws.h_lev_begin[hi + 1] - sb0;
  const int vb0 = wv.h_lev_begin[lo], vbn = wv.h_lev_begin[hi + 1] - vb0;
  TX* r = (TX*)W.r;
  TX* p = (TX*)W.p;
  TX* q = (TX*)W.q;
  TX* z = (TX*)W.z;
  const bool pc = W.pc;
  const BlockJacobi& B = h->bj;
  const int zb0 = pc ? B.wt.h_lev_begin[lo] : 0, zbn = pc ? B.wt.h_lev_begin[hi + 1] - zb0 : 0;
  const TX* inv = nullptr;
  if (pc) {
    if constexpr (sizeof(TX) == 8)
      inv = B.inv;
    else
      inv = B.inv32;
  }
  const dim3 zgrid(std::max(zbn, 1), (c.R + 63) / 64);
  auto bj_apply = [&](const int32_t* ld) {
    if (zbn <= 0) return;
    if constexpr (sizeof(TX) == 4) {
      if (mr_wave_rows(c) && (c.RM == 1 || c.RM == 2 || c.RM == 4)) {
        const dim3 g1(zbn);
        const float *iv = (const float*)inv, *rr = (const float*)r;
        float* zz = (float*)z;
        if (c.RM == 1)
          hipLaunchKernelGGL(k_mr_bj_apply_w<1>, g1, dim3(kBlock), 0, s, B.wt, zb0, B.start, B.of_row, B.off, iv, rr,
                             zz, ld, W.part_z);
        else if (c.RM == 2)
          hipLaunchKernelGGL(k_mr_bj_apply_w<2>, g1, dim3(kBlock), 0, s, B.wt, zb0, B.start, B.of_row, B.off, iv, rr,
                             zz, ld, W.part_z);
        else
          hipLaunchKernelGGL(k_mr_bj_apply_w<4>, g1, dim3(kBlock), 0, s, B.wt, zb0, B.start, B.of_row, B.off, iv, rr,
                             zz, ld, W.part_z);
        return;
      }
    }
    hipLaunchKernelGGL(k_mr_bj_apply<TX>, zgrid, dim3(kBlock), 0, s, B.wt, zb0, B.start, B.of_row, B.off, inv,
                       (const TX*)r, z, ld, W.part_z, c);
  };
  const int32_t* zlb = pc ? B.wt.lev_begin : nullptr;
  double* rzp = pc ? W.part_z : nullptr;
  // chunk width of the product (timed at the first solve with this R; levels all running)
  hipLaunchKernelGGL(k_mr_fill<int32_t>, dim3(mr_nblk(h->L, kBlock)), dim3(kBlock), 0, s, W.lev_done, (int64_t)h->L, 0);
  const int chunk = mr_chunk_for<TV, TX>(h, c, dval, p, q, W.part_s, W.lev_done);
  if (vbn > 0)
    hipLaunchKernelGGL(k_mr_init<TX>, dim3(vbn), dim3(kBlock), 0, s, wv, vb0, b, x, r, p, W.st, W.part_v, c);
  if (pc) bj_apply(nullptr);
  const dim3 rgrid(nlev, (c.R + 63) / 64);
  hipLaunchKernelGGL(k_mr_red_init, rgrid, dim3(kMrRedThreads), 0, s, lo, wv.lev_begin, W.part_v, zlb, rzp, W.st, c);
  hipLaunchKernelGGL(k_mr_lev_done, dim3(nlev), dim3(kBlock), 0, s, lo, W.st, W.lev_done, c);
  // K iterations of every running system, captured once into a graph: its
  // kernels read and update the per-system state, so each replay continues
  // the solve; the host polls the per-level stop flags between replays.
  auto enqueue_chunk = [&]() {
    for (int kk = 0; kk < K; ++kk) {
      if (vbn > 0)
        hipLaunchKernelGGL(k_mr_dir<TX>, dim3(vbn), dim3(kBlock), 0, s, wv, vb0, pc ? (const TX*)z : (const TX*)r, p,
                           W.st, W.lev_done, c);
      if (sbn > 0) launch_mr_cg_product<TV, TX>(h, c, chunk, sb0, sbn, dval, p, q, W.lev_done, W.part_s);
      hipLaunchKernelGGL(k_mr_red_a, rgrid, dim3(kMrRedThreads), 0, s, lo, ws.lev_begin, W.part_s, W.st, W.lev_done,
                         c);
      if (vbn > 0)
        hipLaunchKernelGGL(k_mr_update<TX>, dim3(vbn), dim3(kBlock), 0, s, wv, vb0, x, r, p, q, W.st, W.lev_done,
                           W.part_v, c);
      if (pc) bj_apply(W.lev_done);
      hipLaunchKernelGGL(k_mr_red_b, rgrid, dim3(kMrRedThreads), 0, s, lo, wv.lev_begin, W.part_v, zlb, rzp, W.st,
                         W.lev_done, c);
      hipLaunchKernelGGL(k_mr_lev_done, dim3(nlev), dim3(kBlock), 0, s, lo, W.st, W.lev_done, c);
    }
  };
  hipGraphExec_t exec = nullptr;
  {
    hipGraph_t graph = nullptr;
    MSKM_HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    enqueue_chunk();
    MSKM_HIP_TRY(hipStreamEndCapture(s, &graph));
    const hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return fail(MSKM_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
  }
  struct ExecGuard {
    hipGraphExec_t e;
    ~ExecGuard() { (void)hipGraphExecDestroy(e); }
  } exec_guard{exec};
  for (int it = 0; it < maxit; it += K) {
    MSKM_HIP_TRY(hipGraphLaunch(exec, s));
    MSKM_HIP_TRY(hipMemcpyAsync(W.h_lev_done, W.lev_done, h->L * 4, hipMemcpyDeviceToHost, s));
    MSKM_HIP_TRY(hipStreamSynchronize(s));
    bool any = false;
    for (int l = lo; l <= hi; ++l) any |= on[l] && !W.h_lev_done[l];
    if (!any) break;
  }
  MSKM_HIP_TRY(hipGetLastError());
  MSKM_HIP_TRY(hipMemcpy(hs.data(), W.st, hs.size() * sizeof(MrState), hipMemcpyDeviceToHost));
  for (int l = lo; l <= hi; ++l) {
    if (!on[l]) continue;
    int32_t mx = 0;
    for (int r2 = 0; r2 < c.R; ++r2) {
      const MrState& S = hs[(size_t)l * c.R + r2];
      ms->iters_total += S.iters;
      mx = std::max(mx, S.iters);
      if (S.capped || !S.done) ms->capped = true;
    }
    ms->last_iters[l] = mx;
  }
  return MSKM_OK;
}

template <typename TV, typename TX>
void mr_lower(mskm_hier* h, const TV* lval, const TX* t, const TX* f, TX* y, int64_t r0, int64_t r1, const MrCfg& c) {
  if (r1 <= r0) return;
  const dim3 grid(mr_nblk(r1 - r0, kBlock / c.LR));
  hipStream_t s = h->ctx->stream;
  const int64_t* rp = h->lower.rowptr;
  const int32_t* cl = h->lower.col;
  // all right-hand sides in one chunk: the lower rows are long (all coarser
  // levels), and re-reading them per chunk of 64 costs more than it saves
  switch (mr_wave_rows(c) && c.RM <= 8 && (c.RM & (c.RM - 1)) == 0 ? c.RM : 0) {
#define MSKM_MR_SPMM_W(RMV)                                                                                       \
  case RMV:                                                                                                      \
    hipLaunchKernelGGL((k_mr_spmm_w<RMV, TV, TX>), grid, dim3(kBlock), 0, s, rp, cl, lval, t, f, y, (TX)-1, r0, r1, \
                       c.R);                                                                                     \
    break;
    MSKM_MR_SPMM_W(1)
    MSKM_MR_SPMM_W(2)
    MSKM_MR_SPMM_W(4)
    MSKM_MR_SPMM_W(8)
#undef MSKM_MR_SPMM_W
    default:
      hipLaunchKernelGGL((k_mr_spmm<TV, TX>), grid, dim3(kBlock), 0, s, rp, cl, lval, t, f, y, (TX)-1, r0, r1, c);
  }
}

template <typename TV, typename TX>
mskm_status mr_solve_internal(mskm_hier* h, MrWS& W, const TV* dval, const TV* lval, const TX* f, TX* alpha,
                              const mskm_solve_opts* o, int* sweeps_done, MrStats* ms) {
  hipStream_t s = h->ctx->stream;
  const MrCfg c = W.c;
  const int L = h->L;
  TX* beta = (TX*)W.beta;
  TX* t = (TX*)W.t;
  const size_t NR = W.NR;
  const int maxit = o->max_cg_iters > 0 ? o->max_cg_iters : 20000;
  const int K = o->check_every > 0 ? o->check_every : 8;
  std::vector<char> on(L, 0);
  if (o->algorithm == MSKM_ALG_SEQUENTIAL) {
    MSKM_HIP_TRY(hipMemsetAsync(alpha, 0, NR * sizeof(TX), s));
    const int D = (int)h->h_depth_begin.size() - 1;
    for (int d = 0; d < D; ++d) {
      const int l0 = h->h_depth_begin[d], l1 = h->h_depth_begin[d + 1];
      mr_lower<TV, TX>(h, lval, alpha, f, beta, h->h_off[l0], h->h_off[l1], c);
      std::fill(on.begin(), on.end(), 0);
      for (int l = l0; l < l1; ++l) on[l] = 1;
      MSKM_TRY((mr_cg<TV, TX>(h, W, dval, on, beta, alpha, o->cg_rtol, maxit, K, ms)));
    }
    *sweeps_done = 0;
    return MSKM_OK;
  }
  int Lmax = 0;
  for (int g = 0; g < h->ngroups; ++g) Lmax = std::max(Lmax, (int)h->h_group_levels[g]);
  const int S = o->sweeps > 0 ? o->sweeps : Lmax;
  MSKM_HIP_TRY(hipMemcpyAsync(beta, f, NR * sizeof(TX), hipMemcpyDeviceToDevice, s));
  for (int l = 0; l < L; ++l) on[l] = h->h_next[l] >= 0;
  for (int sw = 0; sw < S && Lmax > 1; ++sw) {
    MSKM_TRY((mr_cg<TV, TX>(h, W, dval, on, beta, t, o->cg_rtol, maxit, K, ms)));
    mr_lower<TV, TX>(h, lval, t, f, beta, 0, h->N, c);
    *sweeps_done = sw + 1;
  }
  std::fill(on.begin(), on.end(), 1);
  MSKM_TRY((mr_cg<TV, TX>(h, W, dval, on, beta, alpha, o->cg_rtol, maxit, K, ms)));
  return MSKM_OK;
}

// Per-rhs, per-group relative residuals (host rel[R][ngroups]); rout nullable.
mskm_status mr_residual(mskm_hier* h, MrWS& W, const double* a, const double* f, double* rout, std::vector<double>& rel,
                        bool a_zero = false) {
  hipStream_t s = h->ctx->stream;
  const MrCfg c = W.c;
  const WorkTable& wt = h->wt_spmv;
  const dim3 grid(wt.nblocks);
  const Csr &D = h->diag, &Lw = h->lower;
  if (a_zero) {
    hipLaunchKernelGGL(k_mr_residual_zero, grid, dim3(kBlock), 0, s, wt, f, rout, W.part_s, W.part_v2, c);
  } else {
    // one chunk (the rows span every level; see mr_lower)
    switch (mr_wave_rows(c) && c.RM <= 8 && (c.RM & (c.RM - 1)) == 0 ? c.RM : 0) {
#define MSKM_MR_RES_W(RMV)                                                                                          \
  case RMV:                                                                                                        \
    hipLaunchKernelGGL(k_mr_residual_w<RMV>, grid, dim3(kBlock), 0, s, wt, D.rowptr, D.col, D.val, Lw.rowptr,      \
                       Lw.col, Lw.val, D.val32, D.val32lo, Lw.val32, Lw.val32lo, a, f, rout, W.part_s, W.part_v2,  \
                       c.R);                                                                                       \
    break;
      MSKM_MR_RES_W(1)
      MSKM_MR_RES_W(2)
      MSKM_MR_RES_W(4)
      MSKM_MR_RES_W(8)
#undef MSKM_MR_RES_W
      default:
        hipLaunchKernelGGL(k_mr_residual, grid, dim3(kBlock), 0, s, wt, D.rowptr, D.col, D.val, Lw.rowptr, Lw.col,
                           Lw.val, D.val32, D.val32lo, Lw.val32, Lw.val32lo, a, f, rout, W.part_s, W.part_v2, c);
    }
  }
  // per-level sums on the device (part_v holds 2 L R doubles), then per group on the host
  const size_t LR = (size_t)h->L * c.R;
  const dim3 lgrid(h->L, (c.R + 63) / 64);
  hipLaunchKernelGGL(k_mr_level_sums, lgrid, dim3(kMrRedThreads), 0, s, wt.lev_begin, W.part_s, W.part_v, c.R);
  hipLaunchKernelGGL(k_mr_level_sums, lgrid, dim3(kMrRedThreads), 0, s, wt.lev_begin, W.part_v2, W.part_v + LR, c.R);
  std::vector<double> sums(2 * LR);
  MSKM_HIP_TRY(hipMemcpyAsync(sums.data(), W.part_v, sums.size() * 8, hipMemcpyDeviceToHost, s));
  MSKM_HIP_TRY(hipStreamSynchronize(s));
  rel.assign((size_t)c.R * h->ngroups, 0.0);
  std::vector<double> rr((size_t)c.R * h->ngroups, 0.0), ff((size_t)c.R * h->ngroups, 0.0);
  for (int l = 0; l < h->L; ++l) {
    const int g = h->h_group[l];
    for (int r = 0; r < c.R; ++r) {
      rr[(size_t)r * h->ngroups + g] += sums[(size_t)l * c.R + r];
      ff[(size_t)r * h->ngroups + g] += sums[LR + (size_t)l * c.R + r];
    }
  }
  for (size_t i = 0; i < rel.size(); ++i) rel[i] = ff[i] > 0.0 ? std::sqrt(rr[i] / ff[i]) : std::sqrt(rr[i]);
  return MSKM_OK;
}

}  // namespace

bool mr_supported(int nrhs) { return nrhs >= 2 && nrhs <= 64 * kMaxRPerLane; }

mskm_status set_mr_chunk(mskm_hier* h, int R, int prec, int chunk) {
  if (!mr_supported(R) || R % 64) return fail(MSKM_EINVAL, "nrhs must be a multiple of 64 in [64, 512]");
  const bool fp32 = prec == MSKM_PREC_FP32;
  if (chunk < 64 || chunk > 512 || (chunk & (chunk - 1)) || R % chunk)
    return fail(MSKM_EINVAL, "chunk must be a power of two in [64, 512] dividing nrhs");
  h->mr_chunk[R / 64 - 1][fp32 ? 1 : 0] = chunk;
  return MSKM_OK;
}

// Mean device time of the many-right-hand-side CG product (q = A_l p for R
// right-hand sides with the partials p.q) on level `level` alone, in the
// chunk width the solver uses for R (tuned here if no solve has), launched
// `repeats` times between two events; vectors of the precision the solve
// uses for prec (FP32 values and vectors, or FP64), allocated here.
template <typename TV, typename TX>
static mskm_status time_mr_product_t(mskm_hier* h, const TV* dval, int level, int R, int repeats, float* avg_ms) {
  hipStream_t s = h->ctx->stream;
  const MrCfg c = mr_cfg(R);
  const WorkTable& ws = h->wt_spmv;
  const int b0 = ws.h_lev_begin[level], nb = ws.h_lev_begin[level + 1] - b0;
  const size_t NR = (size_t)h->N * R;
  TX *p = nullptr, *q = nullptr;
  double* part = nullptr;
  int32_t* done = nullptr;
  mskm_status st = dalloc(&p, NR);
  if (st == MSKM_OK) st = dalloc(&q, NR);
  if (st == MSKM_OK) st = dalloc(&part, (size_t)std::max(ws.nblocks, 1) * R);
  if (st == MSKM_OK) st = dalloc(&done, (size_t)h->L);
  if (st == MSKM_OK) {
    hipLaunchKernelGGL(k_mr_fill<TX>, dim3(mr_nblk((int64_t)NR, kBlock)), dim3(kBlock), 0, s, p, (int64_t)NR, (TX)1);
    hipLaunchKernelGGL(k_mr_fill<int32_t>, dim3(mr_nblk(h->L, kBlock)), dim3(kBlock), 0, s, done, (int64_t)h->L, 0);
    const int chunk = mr_chunk_for<TV, TX>(h, c, dval, (const TX*)p, q, part, done);
    float ms = 0.f;
    if (hipEventRecord(h->ctx->ev0, s) != hipSuccess) st = fail(MSKM_EDEVICE, "event record");
    for (int k = 0; st == MSKM_OK && k < repeats; ++k)
      if (nb > 0) launch_mr_cg_product<TV, TX>(h, c, chunk, b0, nb, dval, p, q, done, part);
    if (st == MSKM_OK && (hipEventRecord(h->ctx->ev1, s) != hipSuccess || hipEventSynchronize(h->ctx->ev1) != hipSuccess ||
                          hipEventElapsedTime(&ms, h->ctx->ev0, h->ctx->ev1) != hipSuccess))
      st = fail(MSKM_EDEVICE, "event timing");
    if (st == MSKM_OK && hipGetLastError() != hipSuccess) st = fail(MSKM_EDEVICE, "many-rhs product launch");
    if (st == MSKM_OK) *avg_ms = ms / (float)repeats;
  }
  (void)hipFree(p);
  (void)hipFree(q);
  (void)hipFree(part);
  (void)hipFree(done);
  return st;
}

mskm_status time_mr_product(mskm_hier* h, int level, int prec, int R, int repeats, float* avg_ms) {
  if (!mr_supported(R)) return fail(MSKM_EINVAL, "nrhs out of range for the many-right-hand-side product");
  if (prec == MSKM_PREC_FP32) {
    if (!h->diag.val32) return fail(MSKM_ESTATE, "FP32 values are not stored");
    return time_mr_product_t<float, float>(h, h->diag.val32, level, R, repeats, avg_ms);
  }
  if (!h->diag.val) return fail(MSKM_ESTATE, "FP64 values are not stored");
  return time_mr_product_t<double, double>(h, h->diag.val, level, R, repeats, avg_ms);
}

// Unit right-hand sides of level l: E[i][r] = 1 for i = off + n0 + r (r < nr).
__global__ void __launch_bounds__(kBlock) k_mr_unit(double* __restrict__ E, int64_t off, int64_t n0, int nr, int R) {
  const int r = blockIdx.x * kBlock + threadIdx.x;
  if (r < nr) E[(off + n0 + r) * R + r] = 1.0;
}

mskm_status lagrange_columns(mskm_hier* h, int l, int64_t n0, int R, double rtol, int maxit, double* Z,
                             int64_t* iters, bool* capped) {
  if (R < 1 || R > 64 * kMaxRPerLane) return fail(MSKM_EINVAL, "lagrange_columns: R out of range");
  if (!h->diag.val) return fail(MSKM_ESTATE, "lagrange_columns: FP64 values are not stored");
  hipStream_t s = h->ctx->stream;
  const int64_t nl = h->h_off[l + 1] - h->h_off[l];
  const int nr = (int)std::max<int64_t>(0, std::min<int64_t>(R, nl - n0));
  MrWS W;
  W.c = mr_cfg(R);
  W.NR = (size_t)h->N * R;
  const size_t NR = W.NR;
  MSKM_TRY(dalloc(&W.fi, NR));
  for (void** v : {&W.r, &W.p, &W.q}) MSKM_TRY(dalloc(reinterpret_cast<char**>(v), NR * 8));
  const size_t nbp = (size_t)std::max(h->wt_spmv.nblocks, h->wt_vec.nblocks) * R;
  MSKM_TRY(dalloc(&W.part_s, nbp));
  MSKM_TRY(dalloc(&W.part_v, std::max(nbp, (size_t)2 * h->L * R)));
  MSKM_TRY(dalloc(&W.part_v2, nbp));
  MSKM_TRY(dalloc(&W.st, (size_t)h->L * R));
  MSKM_TRY(dalloc(&W.lev_done, h->L));
  MSKM_HIP_TRY(hipHostMalloc(reinterpret_cast<void**>(&W.h_lev_done), h->L * 4, hipHostMallocDefault));
  MSKM_HIP_TRY(hipMemsetAsync(W.fi, 0, NR * 8, s));
  if (nr > 0)
    hipLaunchKernelGGL(k_mr_unit, dim3((nr + kBlock - 1) / kBlock), dim3(kBlock), 0, s, W.fi, h->h_off[l], n0, nr, R);
  std::vector<char> on(h->L, 0);
  on[l] = 1;
  MrStats ms;
  ms.last_iters.assign(h->L, 0);
  MSKM_TRY((mr_cg<double, double>(h, W, h->diag.val, on, W.fi, Z, rtol, maxit, 8, &ms)));
  MSKM_HIP_TRY(hipStreamSynchronize(s));
  if (iters) *iters = ms.iters_total;
  if (capped) *capped = ms.capped;
  return MSKM_OK;
}

// Multi-rhs solve: f, alpha [N][nrhs] (input order; device if io_dev).
mskm_status solve_multi(mskm_hier* h, const double* f_in, int nrhs, const mskm_solve_opts* o, double* alpha_out,
                        mskm_report* rep) {
  hipStream_t s = h->ctx->stream;
  const bool io_dev = (o->flags & MSKM_IO_DEVICE) != 0;
  const bool mixed = o->precision == MSKM_PREC_FP32;
  if (mixed ? !h->diag.val32 : !h->diag.val) return fail(MSKM_ESTATE, "requested precision's values are not stored");
  MrWS W;
  W.c = mr_cfg(nrhs);
  W.NR = (size_t)h->N * nrhs;
  const size_t NR = W.NR;
  for (double** v : {&W.fi, &W.ai}) MSKM_TRY(dalloc(v, NR));
  if (mixed) MSKM_TRY(dalloc(&W.res, NR));
  const size_t xs = mixed ? 4 : 8;
  W.pc = o->precond == MSKM_PRECOND_BLOCK_JACOBI;
  if (W.pc) {
    MSKM_TRY(build_block_jacobi(h));
    MSKM_TRY(bj_wait(h, h->L - 1));
  }
  for (void** v : {&W.beta, &W.t, &W.r, &W.p, &W.q}) MSKM_TRY(dalloc(reinterpret_cast<char**>(v), NR * xs));
  if (W.pc) MSKM_TRY(dalloc(reinterpret_cast<char**>(&W.z), NR * xs));
  if (mixed) {
    MSKM_TRY(dalloc(reinterpret_cast<float**>(&W.f32), NR));
    MSKM_TRY(dalloc(reinterpret_cast<float**>(&W.a32), NR));
  }
  const size_t nbp = (size_t)std::max(h->wt_spmv.nblocks, h->wt_vec.nblocks) * nrhs;
  MSKM_TRY(dalloc(&W.part_s, nbp));
  MSKM_TRY(dalloc(&W.part_v, std::max(nbp, (size_t)2 * h->L * nrhs)));  // also the residual's level sums
  MSKM_TRY(dalloc(&W.part_v2, nbp));
  if (W.pc) MSKM_TRY(dalloc(&W.part_z, (size_t)std::max(h->bj.wt.nblocks, 1) * nrhs));
  MSKM_TRY(dalloc(&W.st, (size_t)h->L * nrhs));
  MSKM_TRY(dalloc(&W.lev_done, h->L));
  MSKM_HIP_TRY(hipHostMalloc(reinterpret_cast<void**>(&W.h_lev_done), h->L * 4, hipHostMallocDefault));
  const double* fdev = f_in;
  double* fstage = nullptr;
  if (!io_dev) {
    MSKM_TRY(dalloc(&fstage, NR));
    MSKM_HIP_TRY(hipMemcpyAsync(fstage, f_in, NR * 8, hipMemcpyHostToDevice, s));
    fdev = fstage;
  }
  MrStats ms;
  ms.last_iters.assign(h->L, 0);
  int sweeps_done = 0, refine = 0;
  std::vector<double> rel;
  MSKM_HIP_TRY(hipEventRecord(h->ctx->ev0, s));
  hipLaunchKernelGGL(k_mr_to_internal<double>, dim3(mr_nblk(NR, kBlock)), dim3(kBlock), 0, s, fdev, h->perm, W.fi, h->N,
                     nrhs);
  mskm_status st = MSKM_OK;
  if (!mixed) {
    st = mr_solve_internal<double, double>(h, W, h->diag.val, h->lower.val, W.fi, W.ai, o, &sweeps_done, &ms);
    if (st == MSKM_OK) st = mr_residual(h, W, W.ai, W.fi, nullptr, rel);
  } else {
    const int maxref = o->max_refine > 0 ? o->max_refine : 10;
    MSKM_HIP_TRY(hipMemsetAsync(W.ai, 0, NR * 8, s));
    for (;;) {
      st = mr_residual(h, W, W.ai, W.fi, W.res, rel, refine == 0);  // alpha = 0 at the start
      if (st != MSKM_OK) break;
      const double worst = *std::max_element(rel.begin(), rel.end());
      if (worst <= o->target_rel_residual || refine >= maxref) break;
      hipLaunchKernelGGL(k_mr_to_f32, dim3(mr_nblk(NR, kBlock)), dim3(kBlock), 0, s, W.res, (float*)W.f32, (int64_t)NR);
      mskm_solve_opts oi = *o;
      if (refine > 0) oi.cg_rtol = std::min(0.1, std::max(o->cg_rtol, 0.5 * o->target_rel_residual / worst));
      st = mr_solve_internal<float, float>(h, W, h->diag.val32, h->lower.val32, (const float*)W.f32, (float*)W.a32, &oi,
                                           &sweeps_done, &ms);
      if (st != MSKM_OK) break;
      hipLaunchKernelGGL(k_mr_axpy, dim3(mr_nblk(NR, kBlock)), dim3(kBlock), 0, s, (const float*)W.a32, W.ai,
                         (int64_t)NR);
      ++refine;
    }
  }
  if (st == MSKM_OK) {
    double* adev = alpha_out;
    double* astage = nullptr;
    if (!io_dev) st = dalloc(&astage, NR), adev = astage;
    if (st == MSKM_OK) {
      hipLaunchKernelGGL(k_mr_to_input<double>, dim3(mr_nblk(NR, kBlock)), dim3(kBlock), 0, s, (const double*)W.ai,
                         h->perm, adev, h->N, nrhs);
      if (hipEventRecord(h->ctx->ev1, s) != hipSuccess) st = fail(MSKM_EDEVICE, "event");
      if (st == MSKM_OK && !io_dev &&
          hipMemcpyAsync(alpha_out, astage, NR * 8, hipMemcpyDeviceToHost, s) != hipSuccess)
        st = fail(MSKM_EDEVICE, "alpha copy");
      if (st == MSKM_OK && hipStreamSynchronize(s) != hipSuccess) st = fail(MSKM_EDEVICE, "sync");
    }
    (void)hipFree(astage);
  }
  (void)hipFree(fstage);
  MSKM_TRY(st);
  float msec = 0.f;
  MSKM_HIP_TRY(hipEventElapsedTime(&msec, h->ctx->ev0, h->ctx->ev1));
  const double worst = rel.empty() ? 0.0 : *std::max_element(rel.begin(), rel.end());
  const bool enoconv = mixed ? worst > o->target_rel_residual : ms.capped;
  if (rep) {
    std::memset(rep, 0, sizeof(*rep));
    rep->levels = h->L;
    rep->sweeps_done = sweeps_done;
    rep->refine_steps = refine;
    rep->cg_iters_total = ms.iters_total;
    for (int l = 0; l < std::min(h->L, 64); ++l) rep->cg_iters_last[l] = ms.last_iters[l];
    rep->rel_residual = worst;
    rep->solve_ms = msec;
  }
  MSKM_HIP_TRY(hipGetLastError());
  return enoconv ? MSKM_ENOCONV : MSKM_OK;
}

}  // namespace mskm
