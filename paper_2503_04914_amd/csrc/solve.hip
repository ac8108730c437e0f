// Solve path on gfx950: CSR SpMV with the stored blocks, per-level conjugate
// gradients on the SPD diagonal blocks A_l for all levels in one launch
// (Theorem cg), Jacobi sweeps on T' (Theorem jacobi, eq. (split)), block
// forward substitution (eq. (mas)), the monolithic residual f - T alpha
// (eq. (bigt)) and the approximant at query points (eq. (fapproximation)).
//
// All vectors live in the internal (cell-sorted) order; the entry points
// permute inputs in and outputs out. Reductions are deterministic: each block
// reduces in a fixed tree, the last block of a level to arrive sums the
// per-block partials in block order (agent-scope fences + an arrival ticket).
#include <mutex>
#include <algorithm>
#include <cmath>
#include <cstring>
#include <type_traits>

#include "device_common.h"

namespace mskm {

// ------------------------------------------------------------ permutations

// out[i] = in[perm[i]]: input order -> internal order (nrhs interleaved)
template <typename TO>
__global__ void __launch_bounds__(kBlock) k_to_internal(const double* __restrict__ in, const int32_t* __restrict__ perm,
                                                        TO* __restrict__ out, int64_t n, int nrhs, int r) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) out[i] = (TO)in[(int64_t)perm[i] * nrhs + r];
}

// out[perm[i]] = in[i]: internal order -> input order
template <typename TI>
__global__ void __launch_bounds__(kBlock) k_to_input(const TI* __restrict__ in, const int32_t* __restrict__ perm,
                                                     double* __restrict__ out, int64_t n, int nrhs, int r) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) out[(int64_t)perm[i] * nrhs + r] = (double)in[i];
}

template <typename TI, typename TO>
__global__ void __launch_bounds__(kBlock) k_convert(const TI* __restrict__ in, TO* __restrict__ out, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) out[i] = (TO)in[i];
}

// a += d (FP32 correction accumulated into the FP64 iterate)
__global__ void __launch_bounds__(kBlock) k_axpy_f32(const float* __restrict__ d, double* __restrict__ a, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) a[i] += (double)d[i];
}

static unsigned nblk(int64_t n, int per = kBlock) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + per - 1) / per, 1 << 30));
}

// ------------------------------------------------------------------- SpMV

// Dot of CSR row `row` with x by a group of G lanes (lane gl of the group),
// accumulated in TA; the group sum is returned in every lane of the group.
template <int G, typename TV, typename TX, typename TA>
__device__ __forceinline__ TA csr_row_dot(const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                                          const TV* __restrict__ val, const TX* __restrict__ x, int64_t row, int gl) {
  const int64_t e = rp[row + 1];
  TA acc = 0;
  for (int64_t k = rp[row] + gl; k < e; k += G) acc += (TA)val[k] * (TA)x[col[k]];
  return group_sum<G>(acc);
}

// V = 16 / sizeof(TV) consecutive values and columns of a CSR row from
// entry k, one 16-byte value load and one 8- or 16-byte column load (NT: the
// matrix streams are read once per SpMV; non-temporal loads keep them from
// displacing the gathered x entries in the caches).
template <typename TV, bool NT>
__device__ __forceinline__ void csr_load_v(const int32_t* __restrict__ col, const TV* __restrict__ val, int64_t k,
                                           TV* v, int32_t* c) {
  if constexpr (sizeof(TV) == 8) {
    typedef double nd2 __attribute__((ext_vector_type(2)));
    typedef int ni2 __attribute__((ext_vector_type(2)));
    nd2 a;
    ni2 b;
    if constexpr (NT) {
      a = __builtin_nontemporal_load(reinterpret_cast<const nd2*>(val + k));
      b = __builtin_nontemporal_load(reinterpret_cast<const ni2*>(col + k));
    } else {
      a = *reinterpret_cast<const nd2*>(val + k);
      b = *reinterpret_cast<const ni2*>(col + k);
    }
    v[0] = a.x; v[1] = a.y; c[0] = b.x; c[1] = b.y;
  } else {
    typedef float nf4 __attribute__((ext_vector_type(4)));
    typedef int ni4 __attribute__((ext_vector_type(4)));
    nf4 a;
    ni4 b;
    if constexpr (NT) {
      a = __builtin_nontemporal_load(reinterpret_cast<const nf4*>(val + k));
      b = __builtin_nontemporal_load(reinterpret_cast<const ni4*>(col + k));
    } else {
      a = *reinterpret_cast<const nf4*>(val + k);
      b = *reinterpret_cast<const ni4*>(col + k);
    }
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
    c[0] = b.x; c[1] = b.y; c[2] = b.z; c[3] = b.w;
  }
}

// Same dot with 16-byte loads: each lane takes V = 16/sizeof(TV) consecutive
// entries starting from the row start rounded down to a multiple of V;
// entries outside the row are masked. Two such chunks (G V entries apart)
// are loaded before either is used, so each lane keeps two loads of each
// stream in flight. Value and column arrays carry a tail pad of kCsrPad
// entries, so the rounded loads never leave their allocation.
template <int G, typename TV, typename TX, typename TA, bool NT = false>
__device__ __forceinline__ TA csr_row_dot_v(const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                                            const TV* __restrict__ val, const TX* __restrict__ x, int64_t row,
                                            int gl) {
  constexpr int V = 16 / sizeof(TV);
  constexpr int64_t step = (int64_t)G * V;
  const int64_t s = rp[row], e = rp[row + 1];
  TA acc = 0;
  int64_t k = (s & ~(int64_t)(V - 1)) + (int64_t)gl * V;
  for (; k + step < e; k += 2 * step) {
    TV v[2 * V];
    int32_t c[2 * V];
    csr_load_v<TV, NT>(col, val, k, v, c);
    csr_load_v<TV, NT>(col, val, k + step, v + V, c + V);
#pragma unroll
    for (int u = 0; u < V; ++u)
      if (k + u >= s) acc += (TA)v[u] * (TA)x[c[u]];
#pragma unroll
    for (int u = 0; u < V; ++u)
      if (k + step + u < e) acc += (TA)v[V + u] * (TA)x[c[V + u]];
  }
  if (k < e) {
    TV v[V];
    int32_t c[V];
    csr_load_v<TV, NT>(col, val, k, v, c);
#pragma unroll
    for (int u = 0; u < V; ++u)
      if (k + u >= s && k + u < e) acc += (TA)v[u] * (TA)x[c[u]];
  }
  return group_sum<G>(acc);
}

// y[i] = beta_b * b[i] + sign * (A1 x)[i] + sign * (A2 x)[i]  for i in [0, n)
// (A2 optional). G lanes per row, grid-stride over rows.
template <int G, typename TV, typename TX, typename TA>
__global__ void __launch_bounds__(kBlock)
    k_spmv(const int64_t* __restrict__ rp1, const int32_t* __restrict__ c1, const TV* __restrict__ v1,
           const int64_t* __restrict__ rp2, const int32_t* __restrict__ c2, const TV* __restrict__ v2,
           const TX* __restrict__ x, const TX* __restrict__ b, TX* __restrict__ y, TA sign, int64_t r0, int64_t r1) {
  const int gl = threadIdx.x % G;
  const int64_t groups = (int64_t)gridDim.x * (kBlock / G);
  for (int64_t i = r0 + (int64_t)blockIdx.x * (kBlock / G) + threadIdx.x / G; i < r1; i += groups) {
    TA acc = csr_row_dot<G, TV, TX, TA>(rp1, c1, v1, x, i, gl);
    if (rp2) acc += csr_row_dot<G, TV, TX, TA>(rp2, c2, v2, x, i, gl);
    if (gl == 0) y[i] = (TX)((b ? (TA)b[i] : (TA)0) + sign * acc);
  }
}

template <int G, typename TV, typename TX, typename TA, bool NT = false>
__global__ void __launch_bounds__(kBlock)
    k_spmv_v(const int64_t* __restrict__ rp1, const int32_t* __restrict__ c1, const TV* __restrict__ v1,
             const int64_t* __restrict__ rp2, const int32_t* __restrict__ c2, const TV* __restrict__ v2,
             const TX* __restrict__ x, const TX* __restrict__ b, TX* __restrict__ y, TA sign, int64_t r0, int64_t r1) {
  const int gl = threadIdx.x % G;
  const int64_t groups = (int64_t)gridDim.x * (kBlock / G);
  for (int64_t i = r0 + (int64_t)blockIdx.x * (kBlock / G) + threadIdx.x / G; i < r1; i += groups) {
    TA acc = csr_row_dot_v<G, TV, TX, TA, NT>(rp1, c1, v1, x, i, gl);
    if (rp2) acc += csr_row_dot_v<G, TV, TX, TA, NT>(rp2, c2, v2, x, i, gl);
    if (gl == 0) y[i] = (TX)((b ? (TA)b[i] : (TA)0) + sign * acc);
  }
}

// Entry value recomputed from the point records: phi_{3,1}(sqrt(d2) / delta)
// with 1/delta of the column point's level. The FP64 form differs from the
// stored value only by the rounding of the reciprocal; the FP32 form takes
// the root and the polynomial in single precision (for FP32 operators).
template <typename TA>
__device__ __forceinline__ TA phi_rec(double d2, double inv_delta);
template <>
__device__ __forceinline__ double phi_rec<double>(double d2, double inv_delta) {
  const double r = sqrt(d2) * inv_delta;
  double t = 1.0 - r;
  t = t > 0.0 ? t : 0.0;
  const double t2 = t * t;
  return t2 * t2 * (4.0 * r + 1.0);
}
template <>
__device__ __forceinline__ float phi_rec<float>(double d2, double inv_delta) {
  return phi31_f(sqrtf((float)d2) * (float)inv_delta);
}

// Row dot with values recomputed from the records: only the column stream
// is read from HBM (16-byte loads of 4 columns from the row start rounded
// down to a multiple of 4, entries outside the row masked; the column array
// carries a tail pad of kCsrPad entries); the records and x are gathered
// through the caches. The structure is the stored one, so it stays exact.
template <int G, int DIM, typename TX, typename TA>
__device__ __forceinline__ TA rec_row_dot(const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                                          const double4* __restrict__ rec, const TX* __restrict__ x, int64_t row,
                                          int gl, const double4 me) {
  const int64_t s = rp[row], e = rp[row + 1];
  TA acc = 0;
  for (int64_t k = (s & ~(int64_t)3) + (int64_t)gl * 4; k < e; k += (int64_t)G * 4) {
    const int4 cc = *reinterpret_cast<const int4*>(col + k);
    const int32_t c[4] = {cc.x, cc.y, cc.z, cc.w};
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (k + u >= s && k + u < e) {
        const double4 q = rec[c[u]];
        const double d2 = sqdist(DIM, me.x, me.y, me.z, q.x, q.y, q.z);
        acc += phi_rec<TA>(d2, q.w) * (TA)x[c[u]];
      }
  }
  return group_sum<G>(acc);
}

// y = b + sign * (A1 + A2) x with recomputed values (variant code G + 3000).
template <int G, int DIM, typename T>
__global__ void __launch_bounds__(kBlock)
    k_spmv_rec(const int64_t* __restrict__ rp1, const int32_t* __restrict__ c1, const int64_t* __restrict__ rp2,
               const int32_t* __restrict__ c2, const double4* __restrict__ rec, const T* __restrict__ x,
               const T* __restrict__ b, T* __restrict__ y, T sign, int64_t r0, int64_t r1) {
  const int gl = threadIdx.x % G;
  const int64_t groups = (int64_t)gridDim.x * (kBlock / G);
  for (int64_t i = r0 + (int64_t)blockIdx.x * (kBlock / G) + threadIdx.x / G; i < r1; i += groups) {
    const double4 me = rec[i];
    T acc = rec_row_dot<G, DIM, T, T>(rp1, c1, rec, x, i, gl, me);
    if (rp2) acc += rec_row_dot<G, DIM, T, T>(rp2, c2, rec, x, i, gl, me);
    if (gl == 0) y[i] = (b ? b[i] : (T)0) + sign * acc;
  }
}

// The sliced copy stores each slot's entries in groups of four consecutive
// entries (entry k of slot t at e0 + (k / 4) * 4 kSellC + 4 t + k % 4), so a
// lane reads four values and four columns with one load each.
typedef float sf4 __attribute__((ext_vector_type(4)));
typedef double sd2 __attribute__((ext_vector_type(2)));
typedef int si4 __attribute__((ext_vector_type(4)));
typedef unsigned short su4 __attribute__((ext_vector_type(4)));

// Four values of one slot (non-temporal: the stream is read once per product
// and should not evict the gathered x entries).
__device__ __forceinline__ void sell_vals4(const float* p, float v[4]) {
  const sf4 a = __builtin_nontemporal_load(reinterpret_cast<const sf4*>(p));
  v[0] = a.x;
  v[1] = a.y;
  v[2] = a.z;
  v[3] = a.w;
}
__device__ __forceinline__ void sell_vals4(const double* p, double v[4]) {
  const sd2 a = __builtin_nontemporal_load(reinterpret_cast<const sd2*>(p));
  const sd2 b = __builtin_nontemporal_load(reinterpret_cast<const sd2*>(p + 2));
  v[0] = a.x;
  v[1] = a.y;
  v[2] = b.x;
  v[3] = b.y;
}

// Columns of the sliced copy: 32-bit, or 16-bit offsets from the slice's
// smallest column.
template <bool C16>
struct SellCols;
template <>
struct SellCols<false> {
  const int32_t* col;
  __device__ __forceinline__ void at4(int64_t, int64_t d, int32_t c[4]) const {
    const si4 b = __builtin_nontemporal_load(reinterpret_cast<const si4*>(col + d));
    c[0] = b.x;
    c[1] = b.y;
    c[2] = b.z;
    c[3] = b.w;
  }
};
template <>
struct SellCols<true> {
  const uint16_t* col16;
  const int32_t* cbase;
  __device__ __forceinline__ void at4(int64_t sl, int64_t d, int32_t c[4]) const {
    const su4 b = __builtin_nontemporal_load(reinterpret_cast<const su4*>(col16 + d));
    const int32_t o = cbase[sl];
    c[0] = o + (int32_t)b.x;
    c[1] = o + (int32_t)b.y;
    c[2] = o + (int32_t)b.z;
    c[3] = o + (int32_t)b.w;
  }
};

// Dot of slot t of slice sl with x: entries in order, four per load.
template <typename TV, typename TX, bool C16>
__device__ __forceinline__ TX sell_slot_dot(int64_t sl, int t, int64_t e0, int64_t e1, const SellCols<C16>& cols,
                                            const TV* __restrict__ val, const TX* __restrict__ x) {
  TX acc = 0;
#pragma unroll 2
  for (int64_t d = e0 + 4 * t; d < e1; d += 4 * kSellC) {
    TV v[4];
    int32_t c[4];
    sell_vals4(val + d, v);
    cols.at4(sl, d, c);
#pragma unroll
    for (int u = 0; u < 4; ++u) acc += (TX)v[u] * x[c[u]];
  }
  return acc;
}

// y = b + sign * A_diag x from the sliced copy: one wave per slice, one row
// per lane, the slice's entries read slot-interleaved (fully coalesced).
template <typename T, bool C16>
__global__ void __launch_bounds__(kBlock)
    k_spmv_sell(int64_t nslices, const int64_t* __restrict__ sptr, const int32_t* __restrict__ rows,
                const SellCols<C16> cols, const T* __restrict__ val, const T* __restrict__ x,
                const T* __restrict__ b, T* __restrict__ y, T sign) {
  const int64_t sl = (int64_t)xcd_block_id(gridDim.x) * (kBlock / kSellC) + threadIdx.x / kSellC;
  if (sl >= nslices) return;
  const int t = threadIdx.x % kSellC;
  const T acc = sell_slot_dot<T, T, C16>(sl, t, sptr[sl], sptr[sl + 1], cols, val, x);
  const int32_t row = rows[sl * kSellC + t];
  if (row >= 0) y[row] = (b ? b[row] : (T)0) + sign * acc;
}

// ------------------------------------------------- sliced lower blocks
//
// Products over the sliced copy of the strictly-lower blocks (lsell.hip):
// one wave per slice, one row per lane; the slice's segments (one per coarser
// level) in order, four entries per vector load, 16-bit column offsets from
// each segment's smallest column.

// Dot of slot t of one segment with x (entries in order, four per load).
template <typename TV, typename TX>
__device__ __forceinline__ TX lsell_seg_dot(int32_t base, int t, int64_t e0, int64_t e1,
                                            const uint16_t* __restrict__ col16, const TV* __restrict__ val,
                                            const TX* __restrict__ x) {
  TX acc = 0;
#pragma unroll 2
  for (int64_t d = e0 + 4 * t; d < e1; d += 4 * kSellC) {
    TV v[4];
    sell_vals4(val + d, v);
    const su4 c = __builtin_nontemporal_load(reinterpret_cast<const su4*>(col16 + d));
    acc += (TX)v[0] * x[base + (int32_t)c.x];
    acc += (TX)v[1] * x[base + (int32_t)c.y];
    acc += (TX)v[2] * x[base + (int32_t)c.z];
    acc += (TX)v[3] * x[base + (int32_t)c.w];
  }
  return acc;
}

// The same with split values (FP32 value + FP32 remainder), FP64 accumulation.
template <typename VA>
__device__ __forceinline__ double lsell_seg_dot_split(int32_t base, int t, int64_t e0, int64_t e1,
                                                      const uint16_t* __restrict__ col16, const float* __restrict__ hi,
                                                      const float* __restrict__ lo, const VA& x) {
  double acc = 0.0;
#pragma unroll 2
  for (int64_t d = e0 + 4 * t; d < e1; d += 4 * kSellC) {
    const sf4 h = __builtin_nontemporal_load(reinterpret_cast<const sf4*>(hi + d));
    const sf4 l = __builtin_nontemporal_load(reinterpret_cast<const sf4*>(lo + d));
    const su4 c = __builtin_nontemporal_load(reinterpret_cast<const su4*>(col16 + d));
    acc += ((double)h.x + (double)l.x) * x(base + (int32_t)c.x);
    acc += ((double)h.y + (double)l.y) * x(base + (int32_t)c.y);
    acc += ((double)h.z + (double)l.z) * x(base + (int32_t)c.z);
    acc += ((double)h.w + (double)l.w) * x(base + (int32_t)c.w);
  }
  return acc;
}

// Diagonal copy's slot dot with split values (FP64 accumulation).
template <bool C16, typename VA>
__device__ __forceinline__ double sell_slot_dot_split(int64_t sl, int t, int64_t e0, int64_t e1,
                                                      const SellCols<C16>& cols, const float* __restrict__ hi,
                                                      const float* __restrict__ lo, const VA& x) {
  double acc = 0.0;
#pragma unroll 2
  for (int64_t d = e0 + 4 * t; d < e1; d += 4 * kSellC) {
    const sf4 h = __builtin_nontemporal_load(reinterpret_cast<const sf4*>(hi + d));
    const sf4 l = __builtin_nontemporal_load(reinterpret_cast<const sf4*>(lo + d));
    int32_t c[4];
    cols.at4(sl, d, c);
    acc += ((double)h.x + (double)l.x) * x(c[0]);
    acc += ((double)h.y + (double)l.y) * x(c[1]);
    acc += ((double)h.z + (double)l.z) * x(c[2]);
    acc += ((double)h.w + (double)l.w) * x(c[3]);
  }
  return acc;
}

// y = b + sign * (T - D) x, or (FULL) b + sign * T x, on slices [s0, s1).
template <typename T, bool FULL, bool C16>
__global__ void __launch_bounds__(kBlock)
    k_spmv_lsell(int64_t s0, int64_t s1, const int64_t* __restrict__ sptr, const int32_t* __restrict__ rows,
                 const SellCols<C16> dcols, const T* __restrict__ dval, const int64_t* __restrict__ slice_seg,
                 const int64_t* __restrict__ seg_ptr, const int32_t* __restrict__ seg_base,
                 const uint16_t* __restrict__ lcol, const T* __restrict__ lval, const T* __restrict__ x,
                 const T* __restrict__ b, T* __restrict__ y, T sign) {
  const int64_t sl = s0 + (int64_t)xcd_block_id(gridDim.x) * (kBlock / kSellC) + threadIdx.x / kSellC;
  if (sl >= s1) return;
  const int t = threadIdx.x % kSellC;
  T acc = 0;
  for (int64_t g = slice_seg[sl]; g < slice_seg[sl + 1]; ++g)
    acc += lsell_seg_dot<T, T>(seg_base[g], t, seg_ptr[g], seg_ptr[g + 1], lcol, lval, x);
  if constexpr (FULL) acc += sell_slot_dot<T, T, C16>(sl, t, sptr[sl], sptr[sl + 1], dcols, dval, x);
  const int32_t row = rows[sl * kSellC + t];
  if (row >= 0) y[row] = (b ? b[row] : (T)0) + sign * acc;
}

// FP64 residual r = f - T a over the sliced copies (blocks of 4 slices of the
// sliced table, level-aligned): FP64 values when stored (SPLIT false), else
// the FP32 values plus their remainders; partials r.r and f.f per block.
template <bool SPLIT, bool C16, typename VA>
__global__ void __launch_bounds__(kBlock)
    k_residual_sell(const WorkTable wt, const int64_t* __restrict__ sptr, const int32_t* __restrict__ rows,
                    const SellCols<C16> dcols, const double* __restrict__ dv, const float* __restrict__ dhi,
                    const float* __restrict__ dlo, const int64_t* __restrict__ slice_seg,
                    const int64_t* __restrict__ seg_ptr, const int32_t* __restrict__ seg_base,
                    const uint16_t* __restrict__ lcol, const double* __restrict__ lv, const float* __restrict__ lhi,
                    const float* __restrict__ llo, const VA a, const VA f, double* __restrict__ part,
                    double* __restrict__ rout) {
  __shared__ double sm[kBlock / kWave];
  const int blk = xcd_block_id(gridDim.x);
  const int64_t sl = wt.row0[blk] + threadIdx.x / kSellC;
  const int t = threadIdx.x % kSellC;
  double srr = 0.0, sff = 0.0;
  if (sl < wt.row1[blk]) {
    double acc = 0.0;
    for (int64_t g = slice_seg[sl]; g < slice_seg[sl + 1]; ++g) {
      if constexpr (SPLIT)
        acc += lsell_seg_dot_split(seg_base[g], t, seg_ptr[g], seg_ptr[g + 1], lcol, lhi, llo, a);
      else {
        const int32_t base = seg_base[g];
        for (int64_t d = seg_ptr[g] + 4 * t; d < seg_ptr[g + 1]; d += 4 * kSellC) {
          double v[4];
          sell_vals4(lv + d, v);
          const su4 c = __builtin_nontemporal_load(reinterpret_cast<const su4*>(lcol + d));
          acc += v[0] * a(base + (int32_t)c.x) + v[1] * a(base + (int32_t)c.y) + v[2] * a(base + (int32_t)c.z) +
                 v[3] * a(base + (int32_t)c.w);
        }
      }
    }
    if constexpr (SPLIT) {
      acc += sell_slot_dot_split(sl, t, sptr[sl], sptr[sl + 1], dcols, dhi, dlo, a);
    } else {
      for (int64_t d = sptr[sl] + 4 * t; d < sptr[sl + 1]; d += 4 * kSellC) {
        double v[4];
        int32_t c[4];
        sell_vals4(dv + d, v);
        dcols.at4(sl, d, c);
        acc += v[0] * a(c[0]) + v[1] * a(c[1]) + v[2] * a(c[2]) + v[3] * a(c[3]);
      }
    }
    const int32_t row = rows[sl * kSellC + t];
    if (row >= 0) {
      const double fi = f(row);
      const double ri = fi - acc;
      if (rout) rout[row] = ri;
      srr = ri * ri;
      sff = fi * fi;
    }
  }
  srr = block_sum(srr, sm);
  sff = block_sum(sff, sm);
  if (threadIdx.x == 0) {
    part[2 * blk] = srr;
    part[2 * blk + 1] = sff;
  }
}

// --------------------------------------------------------------------- CG
//
// Conjugate gradients on A_l x_l = b_l for every participating level l, all
// levels in each launch, no grid-wide fences. Textbook form (Theorem cg),
// five kernels per iteration:
//   dir    p = r + beta p
//   spmv   q = A p; partial p.q per block
//   red_a  one block per level: alpha = rr / sum(partials)
//   update x += alpha p; r -= alpha q; partial r.r per block
//   red_b  one block per level: rr_new, stop test ||r|| <= rtol ||b|| or the
//          iteration cap, beta = rr_new / rr.
// Single-reduction form (Chronopoulos and Gear's rearrangement, the same
// iterates in exact arithmetic), three kernels per iteration, used for the
// FP32 inner solves of the mixed path (the FP64 outer refinement bounds the
// effect of its different rounding):
//   spmv   q = A r; partials r.q and r.r per block
//   red    one block per level: gamma = r.r, stop test, beta = gamma /
//          gamma_prev, alpha = gamma / (r.q - beta gamma / alpha_prev)
//   update p = r + beta p; s = q + beta s (= A p); x += alpha p; r -= alpha s.
// The per-level scalars are written only by the reduce kernels and read by the
// big kernels of the next phase; the kernel boundaries order and publish them.
// Partial sums are reduced in block order: the result is deterministic.

// Per-level solve control and state (one struct per level).
struct CgLevel {
  double rtol2;   // rtol^2 (host)
  double bb;      // b.b
  double rr;      // r.r of the current iterate
  double alpha;   // step of the current iteration
  double beta;    // direction coefficient for the next spmv
  int32_t maxit;  // iteration cap (host)
  int32_t on;     // participates (host)
  int32_t iters;  // iterations done
  int32_t done;   // stopped (converged, capped or broken down)
  int32_t capped; // stopped by the cap or by non-finite data
  int32_t fallback; // flexible CG: 0 network in use, 2 just dropped (restart), 1 dropped
  double rr_prev;   // single-reduction form: r.r and step of the previous iteration
  double alpha_prev;
};

constexpr int kRedBlock = 1024;  // threads of the per-level reduce kernels

// Fixed-order block sum of part[a..e), result in thread 0.
__device__ __forceinline__ double block_range_sum(const double* __restrict__ part, int a, int e, double* sm) {
  double s = 0.0;
  for (int i = a + (int)threadIdx.x; i < e; i += (int)blockDim.x) s += part[i];
  return block_sum(s, sm);
}

// Block sum written to part[slot] by thread 0.
__device__ __forceinline__ void block_partial(double v, double* sm, double* __restrict__ part, int slot) {
  v = block_sum(v, sm);
  if (threadIdx.x == 0) part[slot] = v;
}

// Init: x = x0 (warm) or 0; r = b - A x; p_old = 0; partials b.b and r.r
// (over the SpMV table's blocks).
template <int G, typename TV, typename TX>
__global__ void __launch_bounds__(kBlock)
    k_cg_init(const WorkTable wt, const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
              const TV* __restrict__ val, const TX* __restrict__ b, TX* __restrict__ x, TX* __restrict__ r,
              TX* __restrict__ p0, const CgLevel* __restrict__ st, int warm, double* __restrict__ bbp,
              double* __restrict__ rrp, int base, TX* __restrict__ s0) {
  __shared__ double sm[kBlock / kWave];
  const int blk = base + xcd_block_id(gridDim.x);
  const int l = wt.lev[blk];
  const bool on = st[l].on != 0;
  const int64_t row0 = wt.row0[blk], row1 = wt.row1[blk];
  double sb = 0.0, sr = 0.0;
  if (on) {
    const int gl = threadIdx.x % G;
    for (int64_t i = row0 + threadIdx.x / G; i < row1; i += kBlock / G) {
      double ri = (double)b[i];
      if (warm) ri -= csr_row_dot<G, TV, TX, double>(rp, col, val, x, i, gl);
      if (gl == 0) {
        const double bi = (double)b[i];
        if (!warm) x[i] = (TX)0;
        r[i] = (TX)ri;
        p0[i] = (TX)0;
        if (s0) s0[i] = (TX)0;
        sb += bi * bi;
        sr += (double)(TX)ri * (double)(TX)ri;
      }
    }
  }
  block_partial(sb, sm, bbp, blk);
  block_partial(sr, sm, rrp, blk);
}

// One block per level: initial b.b, r.r and stop test.
__global__ void __launch_bounds__(kRedBlock) k_cg_red_init(int lev0, const int32_t* __restrict__ lev_begin,
                                                        const double* __restrict__ bbp, const double* __restrict__ rrp,
                                                        CgLevel* __restrict__ st) {
  __shared__ double sm[kRedBlock / kWave];
  const int l = lev0 + blockIdx.x;
  const double bb = block_range_sum(bbp, lev_begin[l], lev_begin[l + 1], sm);
  const double rr = block_range_sum(rrp, lev_begin[l], lev_begin[l + 1], sm);
  if (threadIdx.x == 0) {
    CgLevel& S = st[l];
    S.bb = bb;
    S.rr = rr;
    S.alpha = 0.0;
    S.beta = 0.0;
    S.iters = 0;
    S.capped = 0;
    S.rr_prev = 0.0;
    S.alpha_prev = 0.0;
    const bool finite = isfinite(bb) && isfinite(rr);
    const bool conv = finite && !(rr > S.rtol2 * bb);
    S.capped = S.on && !conv && (!finite || S.maxit <= 0);
    S.done = !S.on || conv || S.capped;
  }
}

// direction phase: p = r + beta p on the rows of not-stopped levels.
template <typename TX>
__global__ void __launch_bounds__(kBlock) k_cg_dir(const WorkTable wt, int base, const TX* __restrict__ r,
                                                   TX* __restrict__ p, const CgLevel* __restrict__ st) {
  const int blk = base + xcd_block_id(gridDim.x);
  const int l = wt.lev[blk];
  if (st[l].done) return;
  const TX beta = (TX)st[l].beta;
  const int64_t row0 = wt.row0[blk], row1 = wt.row1[blk];
  for (int64_t i = row0 + threadIdx.x; i < row1; i += kBlock) p[i] = r[i] + beta * p[i];
}

// Product phase: q = A p with per-block partials p.q (pqp) and, when given,
// p.rv (ppp; p.p without rv) and rv.rv (p3).
template <int G, bool VEC, typename TV, typename TX>
__global__ void __launch_bounds__(kBlock)
    k_cg_spmv1(const WorkTable wt, int base, const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
               const TV* __restrict__ val, const TX* __restrict__ p, TX* __restrict__ q,
               const CgLevel* __restrict__ st, double* __restrict__ pqp, double* __restrict__ ppp,
               const TX* __restrict__ rv, double* __restrict__ p3) {
  __shared__ double sm[kBlock / kWave];
  const int blk = base + xcd_block_id(gridDim.x);
  const int l = wt.lev[blk];
  if (st[l].done) return;
  const int64_t row0 = wt.row0[blk], row1 = wt.row1[blk];
  const int gl = threadIdx.x % G;
  double s = 0.0, s2 = 0.0, s3 = 0.0;
  for (int64_t i = row0 + threadIdx.x / G; i < row1; i += kBlock / G) {
    TX acc;
    if constexpr (VEC)
      acc = csr_row_dot_v<G, TV, TX, TX>(rp, col, val, p, i, gl);
    else
      acc = csr_row_dot<G, TV, TX, TX>(rp, col, val, p, i, gl);
    if (gl == 0) {
      q[i] = acc;
      const double vi = (double)p[i], wi = rv ? (double)rv[i] : vi;
      s += vi * (double)acc;
      s2 += vi * wi;
      s3 += wi * wi;
    }
  }
  block_partial(s, sm, pqp, blk);
  if (ppp) block_partial(s2, sm, ppp, blk);
  if (p3) block_partial(s3, sm, p3, blk);
}

// The same with recomputed values (variant code G + 3000).
template <int G, int DIM, typename TX>
__global__ void __launch_bounds__(kBlock)
    k_cg_spmv1_rec(const WorkTable wt, int base, const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                   const double4* __restrict__ rec, const TX* __restrict__ p, TX* __restrict__ q,
                       const CgLevel* __restrict__ st, double* __restrict__ pqp, double* __restrict__ ppp,
                   const TX* __restrict__ rv, double* __restrict__ p3) {
  __shared__ double sm[kBlock / kWave];
  const int blk = base + xcd_block_id(gridDim.x);
  const int l = wt.lev[blk];
  if (st[l].done) return;
  const int64_t row0 = wt.row0[blk], row1 = wt.row1[blk];
  const int gl = threadIdx.x % G;
  double s = 0.0, s2 = 0.0, s3 = 0.0;
  for (int64_t i = row0 + threadIdx.x / G; i < row1; i += kBlock / G) {
    const TX acc = rec_row_dot<G, DIM, TX, TX>(rp, col, rec, p, i, gl, rec[i]);
    if (gl == 0) {
      q[i] = acc;
      const double vi = (double)p[i], wi = rv ? (double)rv[i] : vi;
      s += vi * (double)acc;
      s2 += vi * wi;
      s3 += wi * wi;
    }
  }
  block_partial(s, sm, pqp, blk);
  if (ppp) block_partial(s2, sm, ppp, blk);
  if (p3) block_partial(s3, sm, p3, blk);
}

// Slot t's share of slice sl with x for one of two waves per slice: the
// 4-entry groups of parity par (entries in order within the share), with
// ordinary loads, so a small level's entries stay in L2 between iterations.
template <typename TV, typename TX>
__device__ __forceinline__ TX sell_slot_dot_half(int64_t sl, int t, int par, int64_t e0, int64_t e1,
                                                 const SellCols<true>& cols, const TV* __restrict__ val,
                                                 const TX* __restrict__ x) {
  TX acc = 0;
  const int32_t o = cols.cbase[sl];
#pragma unroll 2
  for (int64_t d = e0 + 4 * t + 4 * kSellC * par; d < e1; d += 8 * kSellC) {
    TV v[4];
    if constexpr (sizeof(TV) == 4) {
      const sf4 a = *reinterpret_cast<const sf4*>(val + d);
      v[0] = a.x;
      v[1] = a.y;
      v[2] = a.z;
      v[3] = a.w;
    } else {
      const sd2 a = *reinterpret_cast<const sd2*>(val + d);
      const sd2 b = *reinterpret_cast<const sd2*>(val + d + 2);
      v[0] = a.x;
      v[1] = a.y;
      v[2] = b.x;
      v[3] = b.y;
    }
    const su4 c = *reinterpret_cast<const su4*>(cols.col16 + d);
    acc += (TX)v[0] * x[o + (int32_t)c.x];
    acc += (TX)v[1] * x[o + (int32_t)c.y];
    acc += (TX)v[2] * x[o + (int32_t)c.z];
    acc += (TX)v[3] * x[o + (int32_t)c.w];
  }
  return acc;
}

// The product below for levels of few rows, whose launches are bound by the
// latency of each lane's chain of dependent loads: two waves per slice (the
// same blocks of 4 slices, 512 threads), each taking every other 4-entry
// group of its slots, the halves added through LDS.
template <typename TV, typename TX>
__global__ void __launch_bounds__(2 * kBlock)
    k_cg_spmv1_sell2(const WorkTable wt, int base, const int64_t* __restrict__ sptr, const int32_t* __restrict__ rows,
                     const SellCols<true> cols, const TV* __restrict__ val, const TX* __restrict__ p,
                     TX* __restrict__ q, const CgLevel* __restrict__ st, double* __restrict__ pqp,
                     double* __restrict__ ppp, const TX* __restrict__ rv, double* __restrict__ p3) {
  __shared__ double sm[2 * kBlock / kWave];
  __shared__ TX half[kBlock];  // the odd groups' share of each slot
  const int blk = base + xcd_block_id(gridDim.x);
  const int l = wt.lev[blk];
  if (st[l].done) return;  // uniform over the block
  const int w = threadIdx.x / kWave, t = threadIdx.x % kSellC;
  const int ls = w >> 1, par = w & 1;  // slice of the block, group parity
  const int64_t sl = wt.row0[blk] + ls;
  const bool on = sl < wt.row1[blk];
  TX acc = 0;
  if (on) acc = sell_slot_dot_half<TV, TX>(sl, t, par, sptr[sl], sptr[sl + 1], cols, val, p);
  if (par) half[ls * kSellC + t] = acc;
  __syncthreads();
  double s = 0.0, s2 = 0.0, s3 = 0.0;
  if (on && !par) {
    acc += half[ls * kSellC + t];
    const int32_t row = rows[sl * kSellC + t];
    if (row >= 0) {
      q[row] = acc;
      const double vi = (double)p[row], wi = rv ? (double)rv[row] : vi;
      s = vi * (double)acc;
      s2 = vi * wi;
      s3 = wi * wi;
    }
  }
  block_partial(s, sm, pqp, blk);
  if (ppp) block_partial(s2, sm, ppp, blk);
  if (p3) block_partial(s3, sm, p3, blk);
}

// The same from the sliced copy (variant kSellCode): blocks of 4 slices of
// one level.
template <typename TV, typename TX, bool C16>
__global__ void __launch_bounds__(kBlock)
    k_cg_spmv1_sell(const WorkTable wt, int base, const int64_t* __restrict__ sptr, const int32_t* __restrict__ rows,
                    const SellCols<C16> cols, const TV* __restrict__ val, const TX* __restrict__ p,
                    TX* __restrict__ q, const CgLevel* __restrict__ st, double* __restrict__ pqp,
                    double* __restrict__ ppp, const TX* __restrict__ rv, double* __restrict__ p3) {
  __shared__ double sm[kBlock / kWave];
  const int blk = base + xcd_block_id(gridDim.x);
  const int l = wt.lev[blk];
  if (st[l].done) return;
  const int64_t sl = wt.row0[blk] + threadIdx.x / kSellC;
  const int t = threadIdx.x % kSellC;
  double s = 0.0, s2 = 0.0, s3 = 0.0;
  if (sl < wt.row1[blk]) {
    const TX acc = sell_slot_dot<TV, TX, C16>(sl, t, sptr[sl], sptr[sl + 1], cols, val, p);
    const int32_t row = rows[sl * kSellC + t];
    if (row >= 0) {
      q[row] = acc;
      const double vi = (double)p[row], wi = rv ? (double)rv[row] : vi;
      s = vi * (double)acc;
      s2 = vi * wi;
      s3 = wi * wi;
    }
  }
  block_partial(s, sm, pqp, blk);
  if (ppp) block_partial(s2, sm, ppp, blk);
  if (p3) block_partial(s3, sm, p3, blk);
}

// One block per level: alpha = rr / p.q.
__global__ void __launch_bounds__(kRedBlock) k_cg_red_a(int lev0, const int32_t* __restrict__ lev_begin,
                                                     const double* __restrict__ pqp, CgLevel* __restrict__ st) {
  __shared__ double sm[kRedBlock / kWave];
  const int l = lev0 + blockIdx.x;
  if (st[l].done) return;
  const double pq = block_range_sum(pqp, lev_begin[l], lev_begin[l + 1], sm);
  if (threadIdx.x == 0) {
    CgLevel& S = st[l];
    if (pq > 0.0 && isfinite(pq)) {
      S.alpha = S.rr / pq;
    } else {  // p.q <= 0 cannot happen for SPD A and p != 0: stop this level
      S.alpha = 0.0;
      S.done = 1;
      S.capped = !(S.rr <= S.rtol2 * S.bb);
    }
  }
}

// update phase: x += alpha p; r -= alpha q; partial r.r.
template <typename TX>
__global__ void __launch_bounds__(kBlock)
    k_cg_update(const WorkTable wt, int base, TX* __restrict__ x, TX* __restrict__ r, const TX* __restrict__ p,
                const TX* __restrict__ q, const CgLevel* __restrict__ st, double* __restrict__ rrp) {
  __shared__ double sm[kBlock / kWave];
  const int blk = base + xcd_block_id(gridDim.x);
  const int l = wt.lev[blk];
  if (st[l].done) return;
  const double alpha = st[l].alpha;
  const int64_t row0 = wt.row0[blk], row1 = wt.row1[blk];
  double s = 0.0;
  for (int64_t i = row0 + threadIdx.x; i < row1; i += kBlock) {
    x[i] = (TX)((double)x[i] + alpha * (double)p[i]);
    const TX ri = (TX)((double)r[i] - alpha * (double)q[i]);
    r[i] = ri;
    s += (double)ri * (double)ri;
  }
  block_partial(s, sm, rrp, blk);
}

// One block per level: rr_new, stop test, beta.
__global__ void __launch_bounds__(kRedBlock) k_cg_red_b(int lev0, const int32_t* __restrict__ lev_begin,
                                                     const double* __restrict__ rrp, CgLevel* __restrict__ st) {
  __shared__ double sm[kRedBlock / kWave];
  const int l = lev0 + blockIdx.x;
  if (st[l].done) return;
  const double rr = block_range_sum(rrp, lev_begin[l], lev_begin[l + 1], sm);
  if (threadIdx.x == 0) {
    CgLevel& S = st[l];
    S.iters += 1;
    const double old = S.rr;
    S.rr = rr;
    const bool finite = isfinite(rr);
    if (finite && !(rr > S.rtol2 * S.bb)) {
      S.done = 1;
    } else if (!finite || S.iters >= S.maxit) {
      S.done = 1;
      S.capped = 1;
    } else {
      S.beta = rr / old;
    }
  }
}

// Single-reduction step decision on the level's sums: gamma = r.z (z = r, or
// M^-1 r when preconditioned), delta = z.A z, rr = r.r. Stops on rr before
// the update; else beta = gamma / gamma_prev, alpha = gamma / (delta - beta
// gamma / alpha_prev). Returns true when the update is to be applied.
__device__ __forceinline__ bool cg1_decide(CgLevel& S, double gamma, double delta, double rr) {
  S.rr = rr;
  const bool finite = isfinite(rr) && isfinite(gamma) && isfinite(delta);
  if (finite && !(rr > S.rtol2 * S.bb)) {
    S.done = 1;
    return false;
  }
  if (!finite || S.iters >= S.maxit) {
    S.done = 1;
    S.capped = 1;
    return false;
  }
  const double beta = S.iters == 0 ? 0.0 : gamma / S.rr_prev;
  const double den = S.iters == 0 ? delta : delta - beta * gamma / S.alpha_prev;
  if (!(den > 0.0) || !isfinite(den) || !(gamma > 0.0)) {  // cannot happen for SPD A (and M) and r != 0
    S.done = 1;
    S.capped = 1;
    return false;
  }
  S.beta = beta;
  S.alpha = gamma / den;
  S.rr_prev = gamma;
  S.alpha_prev = S.alpha;
  S.iters += 1;
  return true;
}

// Single-reduction form, one block per level: the sums of the product's
// partials (dq: z.A z, gp: r.z, rp: r.r, null when z = r) and the decision.
__global__ void __launch_bounds__(kRedBlock) k_cg1_red(int lev0, const int32_t* __restrict__ lev_begin,
                                                    const double* __restrict__ dq, const double* __restrict__ gp,
                                                    const double* __restrict__ rp, CgLevel* __restrict__ st) {
  __shared__ double sm[kRedBlock / kWave];
  const int l = lev0 + blockIdx.x;
  if (st[l].done) return;
  const double delta = block_range_sum(dq, lev_begin[l], lev_begin[l + 1], sm);
  const double gamma = block_range_sum(gp, lev_begin[l], lev_begin[l + 1], sm);
  const double rr = rp ? block_range_sum(rp, lev_begin[l], lev_begin[l + 1], sm) : gamma;
  if (threadIdx.x == 0) cg1_decide(st[l], gamma, delta, rr);
}

// Preconditioner arguments of the single-reduction update (PC form).
template <typename TX>
struct PcArgs {
  const int64_t* start;
  const int32_t* of_row;
  const int64_t* off;
  const TX* inv;
  TX* z;  // z = M^-1 r
};

// Single-reduction update on the block's rows: p = z + beta p; s = q + beta s
// (= A p); x += alpha p; r -= alpha s; then (PC) z = M^-1 r for the block's
// rows, the block being a workgroup of whole preconditioner blocks.
template <typename TX, bool PC>
__device__ __forceinline__ void cg1_rows(int64_t row0, int64_t row1, double alpha, TX beta, TX* __restrict__ x,
                                         TX* __restrict__ r, TX* __restrict__ p, TX* __restrict__ sv,
                                         const TX* __restrict__ q, const PcArgs<TX>& pc, TX* rs) {
  for (int64_t i = row0 + threadIdx.x; i < row1; i += kBlock) {
    const TX zi = PC ? pc.z[i] : r[i];
    const TX pi = zi + beta * p[i];
    const TX si = q[i] + beta * sv[i];
    p[i] = pi;
    sv[i] = si;
    x[i] = (TX)((double)x[i] + alpha * (double)pi);
    const TX ri = (TX)((double)r[i] - alpha * (double)si);
    r[i] = ri;
    if constexpr (PC) rs[i - row0] = ri;
  }
  if constexpr (PC) {
    __syncthreads();
    for (int64_t i = row0 + threadIdx.x; i < row1; i += kBlock)
      pc.z[i] = bj_row<TX>(i, row0, rs, pc.start, pc.of_row, pc.off, pc.inv);
  }
}

// Single-reduction update with the decision taken by k_cg1_red.
template <typename TX, bool PC>
__global__ void __launch_bounds__(kBlock)
    k_cg1_update(const WorkTable wt, int base, TX* __restrict__ x, TX* __restrict__ r, TX* __restrict__ p,
                 TX* __restrict__ sv, const TX* __restrict__ q, const CgLevel* __restrict__ st, const PcArgs<TX> pc) {
  __shared__ TX rs[PC ? kBjGroupRows : 1];
  const int blk = base + xcd_block_id(gridDim.x);
  const int l = wt.lev[blk];
  if (st[l].done) return;
  cg1_rows<TX, PC>(wt.row0[blk], wt.row1[blk], st[l].alpha, (TX)st[l].beta, x, r, p, sv, q, pc, rs);
}

// Single-reduction form with the reduction folded into the update: every
// block of a level sums that level's partials itself (same order in every
// block, so all blocks take the same decision), thread 0 of the level's first
// block publishes the new state. The state is double-buffered by iteration
// parity (read cur, write next), so no block reads a state another block of
// the same launch writes.
constexpr int kFusedMaxPartials = 1024;  // larger levels use the separate reduce kernel

template <typename TX, bool PC>
__global__ void __launch_bounds__(kBlock)
    k_cg1_step(const WorkTable wt, int base, const int32_t* __restrict__ qlev_begin, const double* __restrict__ dq,
               const double* __restrict__ gp, const double* __restrict__ rp, TX* __restrict__ x, TX* __restrict__ r,
               TX* __restrict__ p, TX* __restrict__ sv, const TX* __restrict__ q, const CgLevel* __restrict__ cur,
               CgLevel* __restrict__ next, const PcArgs<TX> pc) {
  __shared__ double sm[kBlock / kWave];
  __shared__ double coef[2];
  __shared__ int go;
  __shared__ TX rs[PC ? kBjGroupRows : 1];
  const int blk = base + xcd_block_id(gridDim.x);
  const int l = wt.lev[blk];
  const bool writer = blk == wt.lev_begin[l];
  if (cur[l].done) {
    if (writer && threadIdx.x == 0) next[l] = cur[l];
    return;
  }
  const double delta = block_range_sum(dq, qlev_begin[l], qlev_begin[l + 1], sm);
  const double gamma = block_range_sum(gp, qlev_begin[l], qlev_begin[l + 1], sm);
  const double rr = rp ? block_range_sum(rp, qlev_begin[l], qlev_begin[l + 1], sm) : gamma;
  if (threadIdx.x == 0) {
    CgLevel S = cur[l];
    go = cg1_decide(S, gamma, delta, rr) ? 1 : 0;
    if (writer) next[l] = S;
    coef[0] = S.alpha;
    coef[1] = S.beta;
  }
  __syncthreads();
  if (!go) return;
  cg1_rows<TX, PC>(wt.row0[blk], wt.row1[blk], coef[0], (TX)coef[1], x, r, p, sv, q, pc, rs);
}

// Small levels: the whole CG solve of a level in one workgroup (one
// workgroup per level, levels lev0 + blockIdx.x), in the single-reduction
// form and with the decision rule of the kernels above (cg1_decide), so a
// level stops after the same test. The phases are separated by workgroup
// barriers instead of launches, so no launch and no host check sits between
// iterations. The level's vectors live in LDS (its diagonal block couples
// only rows of the level); thread t owns row t (n <= kWgThreads) in the
// vector phases, the product spreads each row over a group of lanes, and the
// row bounds and preconditioner block of each row are read once, so an
// iteration reads from memory only the matrix entries and the inverse rows.
// x0 = 0; the final state goes to st[l], the solution to x.
constexpr int kWgSolveRows = 1024;  // largest level solved by one workgroup
constexpr int kWgThreads = 1024;

// G lanes per row in the product, R rows per group of G lanes (R kWgThreads / G >= n).
template <typename TV, typename TX, bool PC, int G, int R>
__global__ void __launch_bounds__(kWgThreads)
    k_cg_level_wg(int lev0, const DevLevel* __restrict__ lev, const int64_t* __restrict__ rp,
                  const int32_t* __restrict__ col, const TV* __restrict__ val, const TX* __restrict__ b,
                  TX* __restrict__ x, CgLevel* __restrict__ st, double rtol2, int maxit, const PcArgs<TX> pc) {
  constexpr int kW = kWgThreads / kWave;
  __shared__ double sm[3 * kW];
  __shared__ double coef[2];
  __shared__ int go;
  __shared__ TX xs[kWgSolveRows], rs[kWgSolveRows], ps[kWgSolveRows], ss[kWgSolveRows], qs[kWgSolveRows];
  __shared__ TX zs[PC ? kWgSolveRows : 1];
  const int l = lev0 + blockIdx.x;
  const int64_t r0 = lev[l].off;
  const int n = lev[l].n;
  const int t = threadIdx.x, w = t / kWave, lane = t % kWave;
  const bool mine = t < n;
  // sum of three per-thread values over the workgroup, fixed order, in thread 0
  auto sum3 = [&](double& a, double& c, double& d) {
    a = wave_sum(a);
    c = wave_sum(c);
    d = wave_sum(d);
    if (lane == 0) {
      sm[w] = a;
      sm[kW + w] = c;
      sm[2 * kW + w] = d;
    }
    __syncthreads();
    if (t == 0) {
      a = c = d = 0.0;
      for (int k = 0; k < kW; ++k) {
        a += sm[k];
        c += sm[kW + k];
        d += sm[2 * kW + k];
      }
    }
  };
  // product layout: group gi of G lanes takes rows gi, gi + ng, ... (at
  // most R); step j of a row is its entry gl + j G, and one step of all the
  // group's rows is issued together
  constexpr int ng = kWgThreads / G;
  const int gi = t / G, gl = t % G;
  const int64_t e0 = rp[r0];  // entries of the level's rows relative to its first (fewer than 2^31)
  const int32_t* cl = col + e0;
  const TV* vl = val + e0;
  int kb[R], len[R];
  int steps = 0;
#pragma unroll
  for (int u = 0; u < R; ++u) {
    const int i = gi + u * ng;
    kb[u] = 0;
    len[u] = 0;
    if (i < n) {
      kb[u] = (int)(rp[r0 + i] - e0) + gl;
      const int e = (int)(rp[r0 + i + 1] - e0);
      len[u] = e > kb[u] ? (e - kb[u] + G - 1) / G : 0;
    }
    steps = max(steps, len[u]);
  }
  // preconditioner row of row t: its block's first row (level-relative), size and inverse row
  int ba = 0, bm = 0;
  const TX* Mi = nullptr;
  if (PC && mine) {
    const int32_t bk = pc.of_row[r0 + t];
    const int64_t a = pc.start[bk];
    bm = (int)(pc.start[bk + 1] - a);
    ba = (int)(a - r0);
    Mi = pc.inv + pc.off[bk] + (r0 + t - a) * bm;
  }
  auto bj = [&]() {
    TX acc = 0;
    for (int j = 0; j < bm; ++j) acc += Mi[j] * rs[ba + j];
    return acc;
  };
  // r = b, x = p = s = 0; b.b (= r.r)
  double sb = 0.0, u1 = 0.0, u2 = 0.0;
  if (mine) {
    const TX bi = b[r0 + t];
    xs[t] = (TX)0;
    rs[t] = bi;
    ps[t] = (TX)0;
    ss[t] = (TX)0;
    sb = (double)bi * (double)bi;
  }
  sum3(sb, u1, u2);
  CgLevel S{};
  if (t == 0) {
    S.rtol2 = rtol2;
    S.maxit = maxit;
    S.on = 1;
    S.bb = sb;
    S.rr = sb;
    const bool finite = isfinite(sb);
    const bool conv = finite && !(sb > rtol2 * sb);
    S.capped = !conv && (!finite || maxit <= 0);
    S.done = conv || S.capped;
    go = S.done ? 0 : 1;
  }
  __syncthreads();
  if constexpr (PC) {
    if (mine) zs[t] = bj();
    __syncthreads();
  }
  const TX* zv = PC ? zs : rs;
  while (go) {
    // q = A z with z.q, r.z and r.r
    TX acc[R];
#pragma unroll
    for (int u = 0; u < R; ++u) acc[u] = 0;
    for (int j = 0; j < steps; ++j) {
#pragma unroll
      for (int u = 0; u < R; ++u)
        if (j < len[u]) {
          const int k = kb[u] + j * G;
          acc[u] += (TX)vl[k] * zv[cl[k] - r0];
        }
    }
    double s1 = 0.0, s2 = 0.0, s3 = 0.0;
#pragma unroll
    for (int u = 0; u < R; ++u) {
      TX a = acc[u];
#pragma unroll
      for (int o = G >> 1; o > 0; o >>= 1) a += __shfl_xor(a, o, G);
      const int i = gi + u * ng;
      if (gl == 0 && i < n) {
        qs[i] = a;
        const double vi = (double)zv[i], wi = (double)rs[i];
        s1 += vi * (double)a;
        s2 += vi * wi;
        s3 += wi * wi;
      }
    }
    sum3(s1, s2, s3);
    if (t == 0) {
      go = cg1_decide(S, s2, s1, PC ? s3 : s2) ? 1 : 0;
      coef[0] = S.alpha;
      coef[1] = S.beta;
    }
    __syncthreads();
    if (!go) break;
    const double alpha = coef[0];
    const TX beta = (TX)coef[1];
    if (mine) {
      const TX zi = zv[t];
      const TX pi = zi + beta * ps[t];
      const TX si = qs[t] + beta * ss[t];
      ps[t] = pi;
      ss[t] = si;
      xs[t] = (TX)((double)xs[t] + alpha * (double)pi);
      rs[t] = (TX)((double)rs[t] - alpha * (double)si);
    }
    __syncthreads();
    if constexpr (PC) {
      if (mine) zs[t] = bj();
      __syncthreads();
    }
  }
  if (mine) x[r0 + t] = xs[t];
  if (t == 0) st[l] = S;
}

// ---------------------------------------------------------- solver driver

constexpr int kGDiag = 8;  // lanes per row of the CG init kernel (diagonal rows hold 40-60 entries)

template <typename TV, typename TX>
static void launch_cg_spmv1(hipStream_t s, int code, const WorkTable& wt, int base, int nb, const Csr& A,
                            const TV* val, const TX* p, TX* q, const CgLevel* st, double* pqp, const double* rec,
                            int dim, double* ppp, const TX* rv, double* p3) {
  if (code >= 3 * kVecFlag) {
    const double4* r4 = reinterpret_cast<const double4*>(rec);
#define MSKM_CGREC_CASE(GG)                                                                                   \
  case GG:                                                                                                   \
    if (dim == 3)                                                                                            \
      hipLaunchKernelGGL((k_cg_spmv1_rec<GG, 3, TX>), dim3(nb), dim3(kBlock), 0, s, wt, base, A.rowptr, A.col, \
                         r4, p, q, st, pqp, ppp, rv, p3);                                                                 \
    else                                                                                                     \
      hipLaunchKernelGGL((k_cg_spmv1_rec<GG, 2, TX>), dim3(nb), dim3(kBlock), 0, s, wt, base, A.rowptr, A.col, \
                         r4, p, q, st, pqp, ppp, rv, p3);                                                                 \
    return;
    switch (code - 3 * kVecFlag) {
      MSKM_CGREC_CASE(4)
      MSKM_CGREC_CASE(8)
      MSKM_CGREC_CASE(16)
      MSKM_CGREC_CASE(32)
      default:
        MSKM_CGREC_CASE(64)
    }
#undef MSKM_CGREC_CASE
  }
#define MSKM_CGSPMV1_CASE(GG)                                                                                    \
  case GG:                                                                                                      \
    hipLaunchKernelGGL((k_cg_spmv1<GG, false, TV, TX>), dim3(nb), dim3(kBlock), 0, s, wt, base, A.rowptr, A.col, \
                       val, p, q, st, pqp, ppp, rv, p3);                                                                     \
    break;                                                                                                      \
  case GG + kVecFlag:                                                                                           \
    hipLaunchKernelGGL((k_cg_spmv1<GG, true, TV, TX>), dim3(nb), dim3(kBlock), 0, s, wt, base, A.rowptr, A.col,  \
                       val, p, q, st, pqp, ppp, rv, p3);                                                                     \
    break;
  switch (code) {
    MSKM_CGSPMV1_CASE(4)
    MSKM_CGSPMV1_CASE(8)
    MSKM_CGSPMV1_CASE(16)
    MSKM_CGSPMV1_CASE(32)
    default:
      hipLaunchKernelGGL((k_cg_spmv1<8, false, TV, TX>), dim3(nb), dim3(kBlock), 0, s, wt, base, A.rowptr, A.col,
                         val, p, q, st, pqp, ppp, rv, p3);
  }
#undef MSKM_CGSPMV1_CASE
}

// Persistent solver workspace of one hierarchy, created at its first solve:
// vectors in the internal order (sized for N doubles; the FP32 path uses the
// same memory as float), reduction partials, per-level CG state, and the
// cache of instantiated CG chunk graphs. Stable pointers let a chunk of CG
// iterations be captured once and replayed by every later solve.
struct SolveWS {
  double *beta = nullptr, *t = nullptr, *r = nullptr, *p0 = nullptr, *p1 = nullptr, *q = nullptr;
  double *fi = nullptr, *ai = nullptr, *res = nullptr;  // FP64 f, alpha, residual (internal order)
  float *f32 = nullptr, *a32 = nullptr;                 // FP32 rhs and correction (mixed path)
  double *part_s = nullptr, *part_s2 = nullptr, *part_s3 = nullptr, *part_v = nullptr;
  double* z = nullptr;  // preconditioned residual M^-1 r (block-Jacobi form)
  CgLevel* st = nullptr;
  CgLevel* h_st = nullptr;  // pinned
  CgLevel* h_chk[2] = {nullptr, nullptr};  // pinned state copies of the two chunks in flight
  CgLevel* h_defer = nullptr;  // pinned final states of levels solved by one workgroup, read at the next flush
  std::vector<char> deferred;  // levels whose final state waits in h_defer
  hipEvent_t ev_defer = nullptr;  // after the last copy into h_defer
  hipEvent_t ev_chk[2] = {nullptr, nullptr};
  hipEvent_t pending = nullptr;  // copy of a speculative chunk still in flight (null: none)
  struct Graph {
    int tx;
    const void* val;
    int lo, hi;
    const void* x;
    int K, G;
    hipGraphExec_t exec;
  };
  std::vector<Graph> graphs;
  void* arena = nullptr;     // every device buffer above, carved from one allocation
  double* part_res = nullptr;    // residual partials (r.r, f.f per block of the SpMV table)
  double* h_part_res = nullptr;  // pinned copy of them
  void* pinned = nullptr;  // h_st, the two h_chk copies, h_defer and h_part_res, one pinned allocation
  mskm_ctx* ctx = nullptr;  // arena and pinned blocks go back to its caches
  size_t arena_bytes = 0, pinned_bytes = 0;
  ~SolveWS() {
    if (pending) (void)hipEventSynchronize(pending);
    for (auto& g : graphs) (void)hipGraphExecDestroy(g.exec);
    mskm::ctx_release(ctx, arena, arena_bytes);
    for (hipEvent_t e : ev_chk)
      if (e) (void)hipEventDestroy(e);
    if (ev_defer) (void)hipEventDestroy(ev_defer);
    mskm::ctx_host_release(ctx, pinned, pinned_bytes);
  }
};

static void free_solve_ws(void* p) { delete static_cast<SolveWS*>(p); }

static mskm_status get_ws(mskm_hier* h, SolveWS** out) {
  if (h->solve_ws) {
    *out = static_cast<SolveWS*>(h->solve_ws);
    return MSKM_OK;
  }
  auto* w = new (std::nothrow) SolveWS();
  if (!w) return fail(MSKM_ENOMEM, "workspace allocation");
  const size_t N = (size_t)h->N;
  const size_t np = (size_t)std::max(std::max(h->wt_spmv.nblocks, h->wt_sell.nblocks), 1);
  // one device allocation for all vectors (each 256-byte aligned), one
  // pinned allocation for the host copies of the level states
  size_t bytes = 0;
  auto carve = [&](auto** p, size_t count, char* base) {
    const size_t sz = (std::max(count, (size_t)1) * sizeof(**p) + 255) & ~(size_t)255;
    if (base) *p = reinterpret_cast<std::remove_reference_t<decltype(*p)>>(base + bytes);
    bytes += sz;
  };
  auto layout = [&](char* base) {
    bytes = 0;
    for (double** v : {&w->beta, &w->t, &w->r, &w->p0, &w->p1, &w->q, &w->fi, &w->ai, &w->res, &w->z})
      carve(v, N, base);
    carve(&w->f32, N, base);
    carve(&w->a32, N, base);
    for (double** v : {&w->part_s, &w->part_s2, &w->part_s3}) carve(v, np, base);
    carve(&w->part_v, (size_t)h->wt_vec.nblocks, base);
    carve(&w->part_res, 2 * (size_t)h->wt_spmv.nblocks, base);
    carve(&w->st, 2 * (size_t)h->L, base);  // two parities (fused single-reduction form)
  };
  layout(nullptr);
  w->ctx = h->ctx;
  mskm_status st = MSKM_OK;
  void* base = nullptr;
  const size_t arena_bytes = bytes;
  st = mskm::ctx_alloc(h->ctx, arena_bytes, &base);
  if (st == MSKM_OK) {
    w->arena = base;
    w->arena_bytes = arena_bytes;
    layout(static_cast<char*>(base));
  }
  const size_t pin_states = 4 * (size_t)h->L * sizeof(CgLevel);  // a multiple of 8 bytes
  const size_t pin_bytes = pin_states + 2 * (size_t)h->wt_spmv.nblocks * sizeof(double);
  if (st == MSKM_OK) st = mskm::ctx_host_alloc(h->ctx, pin_bytes, &w->pinned);
  if (st == MSKM_OK) w->pinned_bytes = pin_bytes;
  if (st == MSKM_OK) {
    CgLevel* ps = static_cast<CgLevel*>(w->pinned);
    w->h_st = ps;
    w->h_chk[0] = ps + h->L;
    w->h_chk[1] = ps + 2 * h->L;
    w->h_defer = ps + 3 * h->L;
    w->h_part_res = reinterpret_cast<double*>(static_cast<char*>(w->pinned) + pin_states);
    w->deferred.assign(h->L, 0);
  }
  for (hipEvent_t* e : {&w->ev_chk[0], &w->ev_chk[1], &w->ev_defer})
    if (st == MSKM_OK && hipEventCreateWithFlags(e, hipEventDisableTiming) != hipSuccess)
      st = fail(MSKM_EDEVICE, "event creation");
  if (st != MSKM_OK) {
    delete w;
    return st;
  }
  h->solve_ws = w;
  h->solve_ws_free = free_solve_ws;
  *out = w;
  return MSKM_OK;
}

template <typename TV>
static const TV* sell_values(const Sell& S);
template <>
const double* sell_values<double>(const Sell& S) {
  return S.val;
}
template <>
const float* sell_values<float>(const Sell& S) {
  return S.val32;
}

struct CgStats {
  int64_t iters_total = 0;
  int32_t last_iters[kMaxLevels] = {};
  bool capped = false;
  int32_t warm_fallbacks = 0;
};

// CG forms: textbook (five kernels per iteration), single-reduction (two or
// three), single-reduction with the cell block-Jacobi preconditioner.
enum CgForm { kCgTextbook = 0, kCgOneRed = 1, kCgOneRedBj = 2 };

template <typename TX>
static PcArgs<TX> pc_args(mskm_hier* h, SolveWS& W) {
  PcArgs<TX> a{h->bj.start, h->bj.of_row, h->bj.off, nullptr, (TX*)W.z};
  if constexpr (sizeof(TX) == 8)
    a.inv = h->bj.inv;
  else
    a.inv = h->bj.inv32;
  return a;
}

// The CG product q = A v over blocks [qb0, qb0 + qbn) of the product's launch
// table (the sliced copy's for variants kSellCode / kSell32Code, else the
// CSR table), with the per-block partials v.q into W.part_s and, when given,
// v.rv (v.v without rv) into pp and rv.rv into p3.
// Levels of at most this many rows take the two-waves-per-slice product.
constexpr int64_t kSplitProductRows = 65536;

template <typename TV, typename TX>
static void launch_cg_product(mskm_hier* h, SolveWS& W, const TV* dval, int G, int qb0, int qbn, const TX* v, TX* q,
                              double* pp, const TX* rv, double* p3, const CgLevel* st, bool split) {
  if (qbn <= 0) return;
  hipStream_t s = h->ctx->stream;
  const bool sell = G == kSellCode || G == kSell32Code;
  if (split && sell && G == kSellCode && h->sell.col16)
    hipLaunchKernelGGL((k_cg_spmv1_sell2<TV, TX>), dim3(qbn), dim3(2 * kBlock), 0, s, h->wt_sell, qb0, h->sell.sptr,
                       h->sell.rows, SellCols<true>{h->sell.col16, h->sell.cbase}, sell_values<TV>(h->sell), v, q, st,
                       W.part_s, pp, rv, p3);
  else if (sell && G == kSellCode && h->sell.col16)
    hipLaunchKernelGGL((k_cg_spmv1_sell<TV, TX, true>), dim3(qbn), dim3(kBlock), 0, s, h->wt_sell, qb0, h->sell.sptr,
                       h->sell.rows, SellCols<true>{h->sell.col16, h->sell.cbase}, sell_values<TV>(h->sell), v, q, st,
                       W.part_s, pp, rv, p3);
  else if (sell)
    hipLaunchKernelGGL((k_cg_spmv1_sell<TV, TX, false>), dim3(qbn), dim3(kBlock), 0, s, h->wt_sell, qb0, h->sell.sptr,
                       h->sell.rows, SellCols<false>{h->sell.col}, sell_values<TV>(h->sell), v, q, st, W.part_s, pp, rv,
                       p3);
  else
    launch_cg_spmv1<TV, TX>(s, G, h->wt_spmv, qb0, qbn, h->diag, dval, v, q, st, W.part_s, h->prec, h->dim, pp, rv,
                            p3);
}

// K CG iterations of the given form on levels lo..hi.
template <typename TV, typename TX>
static void enqueue_chunk(mskm_hier* h, SolveWS& W, const TV* dval, int lo, int hi, TX* x, int K, int G, int form) {
  hipStream_t s = h->ctx->stream;
  const WorkTable& ws = h->wt_spmv;
  const bool pcf = form == kCgOneRedBj;
  const WorkTable& wv = pcf ? h->bj.wt : h->wt_vec;  // vector table (whole preconditioner blocks when pcf)
  const WorkTable& wc = h->wt_sell;
  const bool sell = G == kSellCode || G == kSell32Code;
  const bool c16 = G == kSellCode && h->sell.col16;
  const WorkTable& wq = sell ? wc : ws;  // table of the product kernel (and of its partials)
  const int nlev = hi - lo + 1;
  const int qb0 = wq.h_lev_begin[lo], qbn = wq.h_lev_begin[hi + 1] - qb0;
  const int vb0 = wv.h_lev_begin[lo], vbn = wv.h_lev_begin[hi + 1] - vb0;
  TX* p = (TX*)W.p0;
  TX* sv = (TX*)W.p1;
  TX* r = (TX*)W.r;
  TX* q = (TX*)W.q;
  const PcArgs<TX> pc = pc_args<TX>(h, W);
  // q = A v with partials v.q, v.rv (v.v without rv) when pp, rv.rv when p3
  const bool split = h->h_off[hi + 1] - h->h_off[lo] <= kSplitProductRows;
  auto product = [&](const TX* v, double* pp, const TX* rv, double* p3, const CgLevel* st) {
    launch_cg_product<TV, TX>(h, W, dval, G, qb0, qbn, v, q, pp, rv, p3, st, split);
  };
  // fold the reduction into the update when every level's partials are few
  int maxpart = 0;
  for (int l = lo; l <= hi; ++l) maxpart = std::max(maxpart, wq.h_lev_begin[l + 1] - wq.h_lev_begin[l]);
  const bool fused = form != kCgTextbook && maxpart <= kFusedMaxPartials;
  // single-reduction product: of z (= M^-1 r) with r.z and r.r partials, or of r with r.r
  const TX* zv = pcf ? pc.z : r;
  const TX* rv = pcf ? r : nullptr;
  double* p3 = pcf ? W.part_s3 : nullptr;
  for (int it = 0; it < K; ++it) {
    if (form != kCgTextbook && fused) {
      CgLevel* cur = W.st + (size_t)(it & 1) * h->L;
      CgLevel* nxt = W.st + (size_t)((it + 1) & 1) * h->L;
      product(zv, W.part_s2, rv, p3, cur);
      if (vbn > 0) {
        if (pcf)
          hipLaunchKernelGGL((k_cg1_step<TX, true>), dim3(vbn), dim3(kBlock), 0, s, wv, vb0, wq.lev_begin, W.part_s,
                             W.part_s2, p3, x, r, p, sv, q, cur, nxt, pc);
        else
          hipLaunchKernelGGL((k_cg1_step<TX, false>), dim3(vbn), dim3(kBlock), 0, s, wv, vb0, wq.lev_begin, W.part_s,
                             W.part_s2, p3, x, r, p, sv, q, cur, nxt, pc);
      }
    } else if (form != kCgTextbook) {
      product(zv, W.part_s2, rv, p3, W.st);
      hipLaunchKernelGGL(k_cg1_red, dim3(nlev), dim3(kRedBlock), 0, s, lo, wq.lev_begin, W.part_s, W.part_s2, p3,
                         W.st);
      if (vbn > 0) {
        if (pcf)
          hipLaunchKernelGGL((k_cg1_update<TX, true>), dim3(vbn), dim3(kBlock), 0, s, wv, vb0, x, r, p, sv, q, W.st,
                             pc);
        else
          hipLaunchKernelGGL((k_cg1_update<TX, false>), dim3(vbn), dim3(kBlock), 0, s, wv, vb0, x, r, p, sv, q, W.st,
                             pc);
      }
    } else {
      // direction update (beta = 0 on the first iteration after the init, p = 0 there)
      if (vbn > 0) hipLaunchKernelGGL(k_cg_dir<TX>, dim3(vbn), dim3(kBlock), 0, s, wv, vb0, r, p, W.st);
      product(p, nullptr, nullptr, nullptr, W.st);
      hipLaunchKernelGGL(k_cg_red_a, dim3(nlev), dim3(kRedBlock), 0, s, lo, wq.lev_begin, W.part_s, W.st);
      if (vbn > 0)
        hipLaunchKernelGGL(k_cg_update<TX>, dim3(vbn), dim3(kBlock), 0, s, wv, vb0, x, r, p, q, W.st, W.part_v);
      hipLaunchKernelGGL(k_cg_red_b, dim3(nlev), dim3(kRedBlock), 0, s, lo, wv.lev_begin, W.part_v, W.st);
    }
  }
}

// Instantiated graph of one chunk (captured on first use).
template <typename TV, typename TX>
static mskm_status chunk_graph(mskm_hier* h, SolveWS& W, const TV* dval, int lo, int hi, TX* x, int K, int G,
                               int form, hipGraphExec_t* out) {
  const int tx = (int)sizeof(TX) + 100 * form;
  for (const auto& g : W.graphs)
    if (g.tx == tx && g.val == dval && g.lo == lo && g.hi == hi && g.x == x && g.K == K && g.G == G) {
      *out = g.exec;
      return MSKM_OK;
    }
  hipStream_t s = h->ctx->stream;
  hipGraph_t graph = nullptr;
  MSKM_HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
  enqueue_chunk<TV, TX>(h, W, dval, lo, hi, x, K, G, form);
  MSKM_HIP_TRY(hipStreamEndCapture(s, &graph));
  hipGraphExec_t exec = nullptr;
  const hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) return fail(MSKM_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
  W.graphs.push_back(SolveWS::Graph{tx, dval, lo, hi, x, K, G, exec});
  *out = exec;
  return MSKM_OK;
}

// Adds the final states of the levels solved by one workgroup (copied into
// h_defer behind their launch) to the statistics; waits for that copy.
static mskm_status flush_deferred(mskm_hier* h, SolveWS& W, CgStats* cs) {
  bool any = false;
  for (char d : W.deferred) any = any || d != 0;
  if (!any) return MSKM_OK;
  MSKM_HIP_TRY(hipEventSynchronize(W.ev_defer));
  for (int l = 0; l < h->L; ++l) {
    if (!W.deferred[l]) continue;
    W.deferred[l] = 0;
    const CgLevel& o = W.h_defer[l];
    cs->iters_total += o.iters;
    if (l < kMaxLevels) cs->last_iters[l] = o.iters;
    if (o.capped || !o.done) cs->capped = true;
  }
  return MSKM_OK;
}

// Per-level CG on A_l x_l = b_l for the levels in `mask` (contiguous bits).
// x holds x0 if warm, else it is overwritten. Iterations run as replays of a
// captured chunk of K iterations; the host reads the per-level state after
// each chunk and stops when every level has stopped.
template <typename TV, typename TX>
static mskm_status cg_run(mskm_hier* h, SolveWS& W, const TV* dval, const std::vector<char>& on, const TX* b, TX* x,
                          double rtol, int maxit, bool warm, int K, CgStats* cs, const mskm_mlp* mlp, bool bj,
                          const std::vector<char>* next_on = nullptr) {
  hipStream_t s = h->ctx->stream;
  const WorkTable& ws = h->wt_spmv;
  int lo = 0, hi = h->L - 1;
  while (lo < h->L && !on[lo]) ++lo;
  while (hi >= 0 && !on[hi]) --hi;
  if (lo > hi) return MSKM_OK;
  if (bj) MSKM_TRY(bj_wait(h, hi));  // the finest levels' inverses may still be forming on the side stream
  // form: preconditioned single-reduction when asked; the single-reduction
  // form for the FP32 inner solves; the textbook form otherwise
  const int form = bj ? kCgOneRedBj : sizeof(TX) == 4 ? kCgOneRed : kCgTextbook;
  // levels lo..hi all small enough for one workgroup each (and all on)
  auto all_small = [&](const std::vector<char>& m, int a, int e) {
    bool ok = form != kCgTextbook && !mlp && !warm;
    for (int l = a; l <= e && ok; ++l) ok = m[l] && h->h_lev[l].n <= kWgSolveRows;
    return ok;
  };
  if (all_small(on, lo, hi)) {  // one workgroup per level, all iterations in one launch, no host check
    for (int l = lo; l <= hi; ++l)
      if (W.deferred[l]) {  // a state of this level still waits in h_defer
        MSKM_TRY(flush_deferred(h, W, cs));
        break;
      }
    const PcArgs<TX> pc = pc_args<TX>(h, W);
    int nmax = 0;
    for (int l = lo; l <= hi; ++l) nmax = std::max(nmax, (int)h->h_lev[l].n);
    // lanes and rows per product group by level size (measured on 64-, 256- and 1024-row levels)
    const int shape = nmax <= 64 ? 0 : nmax <= 256 ? 1 : 2;
#define MSKM_WG_LAUNCH(PCF, GG, RR)                                                                              \
  hipLaunchKernelGGL((k_cg_level_wg<TV, TX, PCF, GG, RR>), dim3(hi - lo + 1), dim3(kWgThreads), 0, s, lo, h->d_lev, \
                     h->diag.rowptr, h->diag.col, dval, b, x, W.st, rtol * rtol, maxit, pc)
    if (bj) {
      if (shape == 0)
        MSKM_WG_LAUNCH(true, 16, 1);
      else if (shape == 1)
        MSKM_WG_LAUNCH(true, 4, 1);
      else
        MSKM_WG_LAUNCH(true, 8, 8);
    } else {
      if (shape == 0)
        MSKM_WG_LAUNCH(false, 16, 1);
      else if (shape == 1)
        MSKM_WG_LAUNCH(false, 4, 1);
      else
        MSKM_WG_LAUNCH(false, 8, 8);
    }
#undef MSKM_WG_LAUNCH
    MSKM_HIP_TRY(hipMemcpyAsync(W.h_defer + lo, W.st + lo, (hi - lo + 1) * sizeof(CgLevel), hipMemcpyDeviceToHost, s));
    MSKM_HIP_TRY(hipEventRecord(W.ev_defer, s));
    for (int l = lo; l <= hi; ++l) W.deferred[l] = 1;
    // capture the next levels' chunk while the workgroups run (when they are chunked)
    if (next_on) {
      int nlo = 0, nhi = h->L - 1;
      while (nlo < h->L && !(*next_on)[nlo]) ++nlo;
      while (nhi >= 0 && !(*next_on)[nhi]) --nhi;
      if (nlo <= nhi && !all_small(*next_on, nlo, nhi)) {
        int Gn = h->spmv_g[MSKM_OP_DIAG][sizeof(TX) == 4 ? 1 : 0];
        if (Gn >= 2 * kVecFlag && Gn < 3 * kVecFlag) Gn -= kVecFlag;
        hipGraphExec_t next_exec = nullptr;
        MSKM_TRY((chunk_graph<TV, TX>(h, W, dval, nlo, nhi, x, K, Gn, form, &next_exec)));
      }
    }
    return MSKM_OK;
  }
  // the first chunked level starts the side-stream inversion of the finest
  // depth's blocks (its few-block launches leave most of the GPU free)
  if (bj) MSKM_TRY(bj_start_side(h));
  if (W.pending) {  // the previous run's speculative chunk copy lands in h_chk
    MSKM_HIP_TRY(hipEventSynchronize(W.pending));
    W.pending = nullptr;
  }
  for (int l = 0; l < h->L; ++l) {
    CgLevel& S = W.h_st[l];
    std::memset(&S, 0, sizeof(S));
    S.rtol2 = rtol * rtol;
    S.maxit = maxit;
    S.on = on[l] ? 1 : 0;
    S.done = 1;
  }
  MSKM_HIP_TRY(hipMemcpyAsync(W.st, W.h_st, h->L * sizeof(CgLevel), hipMemcpyHostToDevice, s));
  const int nlev = hi - lo + 1;
  const int sb0 = ws.h_lev_begin[lo], sbn = ws.h_lev_begin[hi + 1] - sb0;
  int G = h->spmv_g[MSKM_OP_DIAG][sizeof(TX) == 4 ? 1 : 0];
  if (G >= 2 * kVecFlag && G < 3 * kVecFlag) G -= kVecFlag;  // CG SpMV: 16-byte loads (no non-temporal variant)
  if (mlp) {  // learned warm start x0 = MLP(b) on every participating level
    for (int l = lo; l <= hi; ++l)
      if (on[l]) MSKM_TRY(mlp_predict_rows<TX>(h, mlp, l, b, x));
    warm = true;
  }
  if (sbn > 0)
    hipLaunchKernelGGL((k_cg_init<kGDiag, TV, TX>), dim3(sbn), dim3(kBlock), 0, s, ws, h->diag.rowptr, h->diag.col,
                       dval, b, x, (TX*)W.r, (TX*)W.p0, W.st, warm ? 1 : 0, W.part_s, W.part_s2, sb0, (TX*)W.p1);
  hipLaunchKernelGGL(k_cg_red_init, dim3(nlev), dim3(kRedBlock), 0, s, lo, ws.lev_begin, W.part_s, W.part_s2, W.st);
  if (bj) launch_bj_apply<TX>(h, lo, hi, (const TX*)W.r, (TX*)W.z);
  if (mlp) {  // CG checks the warm start: ||b - A x0|| >= ||b|| restarts that level from zero
    MSKM_HIP_TRY(hipMemcpyAsync(W.h_st, W.st, h->L * sizeof(CgLevel), hipMemcpyDeviceToHost, s));
    MSKM_HIP_TRY(hipStreamSynchronize(s));
    bool again = false;
    for (int l = lo; l <= hi; ++l) {
      const CgLevel& S = W.h_st[l];
      if (on[l] && S.bb > 0.0 && !(S.rr < S.bb)) {
        MSKM_HIP_TRY(hipMemsetAsync(x + h->h_off[l], 0, (h->h_off[l + 1] - h->h_off[l]) * sizeof(TX), s));
        cs->warm_fallbacks += 1;
        again = true;
      }
    }
    if (again) {
      for (int l = 0; l < h->L; ++l) {
        W.h_st[l].done = 1;
        W.h_st[l].iters = 0;
      }
      MSKM_HIP_TRY(hipMemcpyAsync(W.st, W.h_st, h->L * sizeof(CgLevel), hipMemcpyHostToDevice, s));
      if (sbn > 0)
        hipLaunchKernelGGL((k_cg_init<kGDiag, TV, TX>), dim3(sbn), dim3(kBlock), 0, s, ws, h->diag.rowptr, h->diag.col,
                           dval, b, x, (TX*)W.r, (TX*)W.p0, W.st, 1, W.part_s, W.part_s2, sb0, (TX*)W.p1);
      hipLaunchKernelGGL(k_cg_red_init, dim3(nlev), dim3(kRedBlock), 0, s, lo, ws.lev_begin, W.part_s, W.part_s2,
                         W.st);
      if (bj) launch_bj_apply<TX>(h, lo, hi, (const TX*)W.r, (TX*)W.z);
    }
  }
  hipGraphExec_t exec = nullptr;
  MSKM_TRY((chunk_graph<TV, TX>(h, W, dval, lo, hi, x, K, G, form, &exec)));
  // Two chunks in flight: chunk k+1 is queued before the host reads chunk
  // k's state, so the device does not idle during the check. Iterations of
  // stopped levels are no-ops, so a speculative chunk changes nothing.
  const int max_chunks = (maxit + K - 1) / K;
  int launched = 0, checked = 0;
  auto launch = [&]() -> mskm_status {
    const int slot = launched & 1;
    MSKM_HIP_TRY(hipGraphLaunch(exec, s));
    MSKM_HIP_TRY(hipMemcpyAsync(W.h_chk[slot], W.st, h->L * sizeof(CgLevel), hipMemcpyDeviceToHost, s));
    MSKM_HIP_TRY(hipEventRecord(W.ev_chk[slot], s));
    ++launched;
    return MSKM_OK;
  };
  MSKM_TRY(launch());
  bool prepared = next_on == nullptr;
  while (checked < launched) {
    if (launched < max_chunks) MSKM_TRY(launch());
    if (!prepared) {  // capture the next levels' chunk while this one's two chunks run
      prepared = true;
      int nlo = 0, nhi = h->L - 1;
      while (nlo < h->L && !(*next_on)[nlo]) ++nlo;
      while (nhi >= 0 && !(*next_on)[nhi]) --nhi;
      hipGraphExec_t next_exec = nullptr;
      if (nlo <= nhi && !all_small(*next_on, nlo, nhi))
        MSKM_TRY((chunk_graph<TV, TX>(h, W, dval, nlo, nhi, x, K, G, form, &next_exec)));
    }
    MSKM_HIP_TRY(hipEventSynchronize(W.ev_chk[checked & 1]));
    const CgLevel* c = W.h_chk[checked & 1];
    ++checked;
    bool any = false;
    for (int l = lo; l <= hi; ++l) any |= c[l].done == 0;
    if (!any) break;
  }
  if (launched > checked) W.pending = W.ev_chk[(launched - 1) & 1];
  const CgLevel* fin = W.h_chk[(checked - 1) & 1];
  MSKM_HIP_TRY(hipGetLastError());
  for (int l = lo; l <= hi; ++l) {
    if (!on[l]) continue;
    const CgLevel& o = fin[l];
    cs->iters_total += o.iters;
    if (l < kMaxLevels) cs->last_iters[l] = o.iters;
    if (o.capped || !o.done) cs->capped = true;
  }
  return MSKM_OK;
}

// ------------------------------------------------- flexible CG (learned)
//
// Flexible conjugate gradients with one previous direction kept (Notay's
// FCG(1); with a fixed SPD preconditioner the iterates are those of PCG):
// the preconditioner may change from one iteration to the next, as a
// nonlinear learned one does. With z = P(r):
//   q = A p; alpha = p.r / p.q; x += alpha p; r -= alpha q;
//   z = P(r); beta = -z.q / p.q; p = z + beta p,
// from p = z = P(b), x = 0. Here P(r) = M^-1 r + net(r): the cell
// block-Jacobi inverse plus the learned network's prediction of A^-1 r from
// r's 17-point stencils. CG decides convergence: the stopping test is the true
// residual ||r|| <= rtol ||b||; and plain preconditioned CG is the fallback:
// a level whose r.r has not fallen by the factor kFcgWindowDrop over a window
// of kFcgWindow iterations drops the network for the rest of its solve
// (z = M^-1 r, direction restarted: FCG with a fixed SPD preconditioner is
// PCG). State per level in CgLevel: bb, rr, alpha, beta, fallback; rr_prev
// holds p.q of the current iteration, alpha_prev r.r at the start of the
// window.
constexpr int kFcgWindow = 8;
constexpr double kFcgWindowDrop = 0.25;

// x = 0, r = b, partial b.b per block of the vector table.
template <typename TX>
__global__ void __launch_bounds__(kBlock)
    k_fcg_init(const WorkTable wt, int base, const TX* __restrict__ b, TX* __restrict__ x, TX* __restrict__ r,
               double* __restrict__ part) {
  __shared__ double sm[kBlock / kWave];
  const int blk = base + xcd_block_id(gridDim.x);
  double acc = 0.0;
  for (int64_t i = wt.row0[blk] + threadIdx.x; i < wt.row1[blk]; i += kBlock) {
    const TX bi = b[i];
    x[i] = (TX)0;
    r[i] = bi;
    acc += (double)bi * (double)bi;
  }
  block_partial(acc, sm, part, blk);
}

// z = u (+ w) on running levels (u: block-Jacobi part or null, w: network
// part or null; levels that fell back take u only)
template <typename TX>
__global__ void __launch_bounds__(kBlock)
    k_fcg_precond(const WorkTable wt, int base, const TX* __restrict__ u, const TX* __restrict__ w, TX* __restrict__ z,
                  const CgLevel* __restrict__ st) {
  const int blk = base + xcd_block_id(gridDim.x);
  const CgLevel& S = st[wt.lev[blk]];
  if (S.done) return;
  const TX* wn = S.fallback ? nullptr : w;
  for (int64_t i = wt.row0[blk] + threadIdx.x; i < wt.row1[blk]; i += kBlock)
    z[i] = (u ? u[i] : (TX)0) + (wn ? wn[i] : (TX)0);
}

// x += alpha p; r -= alpha q; partial r.r (running levels).
template <typename TX>
__global__ void __launch_bounds__(kBlock)
    k_fcg_update(const WorkTable wt, int base, TX* __restrict__ x, TX* __restrict__ r, const TX* __restrict__ p,
                 const TX* __restrict__ q, const CgLevel* __restrict__ st, double* __restrict__ part) {
  __shared__ double sm[kBlock / kWave];
  const int blk = base + xcd_block_id(gridDim.x);
  const int l = wt.lev[blk];
  double acc = 0.0;
  if (!st[l].done) {
    const TX a = (TX)st[l].alpha;
    for (int64_t i = wt.row0[blk] + threadIdx.x; i < wt.row1[blk]; i += kBlock) {
      x[i] += a * p[i];
      const TX ri = r[i] - a * q[i];
      r[i] = ri;
      acc += (double)ri * (double)ri;
    }
  }
  block_partial(acc, sm, part, blk);
}

// partial z.q (running levels)
template <typename TX>
__global__ void __launch_bounds__(kBlock)
    k_fcg_dot(const WorkTable wt, int base, const TX* __restrict__ z, const TX* __restrict__ q,
              const CgLevel* __restrict__ st, double* __restrict__ part) {
  __shared__ double sm[kBlock / kWave];
  const int blk = base + xcd_block_id(gridDim.x);
  double acc = 0.0;
  if (!st[wt.lev[blk]].done)
    for (int64_t i = wt.row0[blk] + threadIdx.x; i < wt.row1[blk]; i += kBlock) acc += (double)z[i] * (double)q[i];
  block_partial(acc, sm, part, blk);
}

// p = z + beta p (first: p = z)
template <typename TX>
__global__ void __launch_bounds__(kBlock)
    k_fcg_dir(const WorkTable wt, int base, const TX* __restrict__ z, TX* __restrict__ p,
              const CgLevel* __restrict__ st, int first) {
  const int blk = base + xcd_block_id(gridDim.x);
  const int l = wt.lev[blk];
  if (st[l].done) return;
  const TX beta = (TX)st[l].beta;
  for (int64_t i = wt.row0[blk] + threadIdx.x; i < wt.row1[blk]; i += kBlock) p[i] = first ? z[i] : z[i] + beta * p[i];
}

// Per-level scalar steps of FCG (one block per level, fixed-order sums):
//   phase 0 (init):  bb = rr = sum(part_v); stop if bb = 0
//   phase 1 (alpha): pq = sum(part_q), alpha = sum(part_q2) / pq (p.r / p.q)
//   phase 2 (stop):  rr = sum(part_v); iters++; stop on rr <= rtol^2 bb or the cap
//   phase 3 (beta):  beta = -sum(part_v) / pq (z.q / p.q)
__global__ void __launch_bounds__(kRedBlock)
    k_fcg_red(int phase, int lev0, const int32_t* __restrict__ qbeg, const double* __restrict__ part_q,
              const double* __restrict__ part_q2, const int32_t* __restrict__ vbeg, const double* __restrict__ part_v,
              CgLevel* __restrict__ st) {
  __shared__ double sm[kRedBlock / kWave];
  const int l = lev0 + blockIdx.x;
  CgLevel& S = st[l];
  if (phase > 0 && S.done) return;
  if (phase == 1) {
    const double pq = block_range_sum(part_q, qbeg[l], qbeg[l + 1], sm);
    const double pr = block_range_sum(part_q2, qbeg[l], qbeg[l + 1], sm);
    if (threadIdx.x == 0) {
      if (pq > 0.0 && isfinite(pq) && isfinite(pr)) {
        S.rr_prev = pq;
        S.alpha = pr / pq;
      } else {  // breakdown: stop the level (reported as capped unless converged)
        S.alpha = 0.0;
        S.done = 1;
        S.capped = 1;
      }
    }
    return;
  }
  const double v = block_range_sum(part_v, vbeg[l], vbeg[l + 1], sm);
  if (threadIdx.x != 0) return;
  if (phase == 0) {
    S.bb = v;
    S.rr = v;
    S.iters = 0;
    S.alpha = S.beta = 0.0;
    S.alpha_prev = v;  // r.r at the start of the first window
    S.fallback = 0;
    const bool finite = isfinite(v);
    const bool conv = finite && !(v > S.rtol2 * v);
    S.capped = S.on && !conv && (!finite || S.maxit <= 0);
    S.done = !S.on || conv || S.capped;
  } else if (phase == 2) {
    S.rr = v;
    S.iters += 1;
    const bool conv = isfinite(v) && v <= S.rtol2 * S.bb;
    if (conv) S.done = 1;
    else if (!isfinite(v) || S.iters >= S.maxit) S.done = S.capped = 1;
    else if (S.iters % kFcgWindow == 0) {
      if (!S.fallback && v > kFcgWindowDrop * S.alpha_prev) S.fallback = 2;  // restart at the next direction
      S.alpha_prev = v;
    }
  } else {
    if (S.fallback == 2) {  // first direction of the fallback: p = z = M^-1 r
      S.beta = 0.0;
      S.fallback = 1;
    } else {
      S.beta = -v / S.rr_prev;
    }
  }
}

template <typename TV, typename TX>
static mskm_status fcg_run(mskm_hier* h, SolveWS& W, const TV* dval, const std::vector<char>& on, const TX* b, TX* x,
                           double rtol, int maxit, int K, CgStats* cs, const mskm_mlp* mlp, bool bj) {
  hipStream_t s = h->ctx->stream;
  int lo = 0, hi = h->L - 1;
  while (lo < h->L && !on[lo]) ++lo;
  while (hi >= 0 && !on[hi]) --hi;
  if (lo > hi) return MSKM_OK;
  MSKM_TRY(flush_deferred(h, W, cs));
  if (bj) MSKM_TRY(bj_wait(h, hi));
  int G = h->spmv_g[MSKM_OP_DIAG][sizeof(TX) == 4 ? 1 : 0];
  if (G >= 2 * kVecFlag && G < 3 * kVecFlag) G -= kVecFlag;
  const bool sell = G == kSellCode || G == kSell32Code;
  const WorkTable& wq = sell ? h->wt_sell : h->wt_spmv;
  const WorkTable& wv = h->wt_vec;
  const int nlev = hi - lo + 1;
  const int qb0 = wq.h_lev_begin[lo], qbn = wq.h_lev_begin[hi + 1] - qb0;
  const int vb0 = wv.h_lev_begin[lo], vbn = wv.h_lev_begin[hi + 1] - vb0;
  TX* r = (TX*)W.r;
  TX* p = (TX*)W.p0;
  TX* q = (TX*)W.q;
  TX* z = (TX*)W.z;
  TX* tz = (TX*)W.p1;  // network part of z
  TX* bz = (TX*)W.t;   // block-Jacobi part of z (W.t is free in the sequential algorithm)
  for (int l = 0; l < h->L; ++l) {
    CgLevel& S = W.h_st[l];
    std::memset(&S, 0, sizeof(S));
    S.rtol2 = rtol * rtol;
    S.maxit = maxit;
    S.on = on[l] ? 1 : 0;
    S.done = 1;
  }
  MSKM_HIP_TRY(hipMemcpyAsync(W.st, W.h_st, h->L * sizeof(CgLevel), hipMemcpyHostToDevice, s));
  auto precond = [&]() -> mskm_status {
    if (bj) launch_bj_apply<TX>(h, lo, hi, (const TX*)r, bz);
    if (mlp)
      for (int l = lo; l <= hi; ++l)
        if (on[l]) MSKM_TRY(mlp_predict_rows<TX>(h, mlp, l, (const TX*)r, tz));
    if (vbn > 0)
      hipLaunchKernelGGL(k_fcg_precond<TX>, dim3(vbn), dim3(kBlock), 0, s, wv, vb0, bj ? (const TX*)bz : nullptr,
                         mlp ? (const TX*)tz : nullptr, z, W.st);
    return MSKM_OK;
  };
  if (vbn > 0) hipLaunchKernelGGL(k_fcg_init<TX>, dim3(vbn), dim3(kBlock), 0, s, wv, vb0, b, x, r, W.part_v);
  hipLaunchKernelGGL(k_fcg_red, dim3(nlev), dim3(kRedBlock), 0, s, 0, lo, wq.lev_begin, W.part_s, W.part_s2,
                     wv.lev_begin, W.part_v, W.st);
  MSKM_TRY(precond());
  if (vbn > 0) hipLaunchKernelGGL(k_fcg_dir<TX>, dim3(vbn), dim3(kBlock), 0, s, wv, vb0, (const TX*)z, p, W.st, 1);
  std::vector<CgLevel> fin(h->L);
  for (int it = 0; it < maxit; it += K) {
    for (int kk = 0; kk < K; ++kk) {
      launch_cg_product<TV, TX>(h, W, dval, G, qb0, qbn, (const TX*)p, q, W.part_s2, (const TX*)r, nullptr, W.st,
                                h->h_off[hi + 1] - h->h_off[lo] <= kSplitProductRows);
      hipLaunchKernelGGL(k_fcg_red, dim3(nlev), dim3(kRedBlock), 0, s, 1, lo, wq.lev_begin, W.part_s, W.part_s2,
                         wv.lev_begin, W.part_v, W.st);
      if (vbn > 0)
        hipLaunchKernelGGL(k_fcg_update<TX>, dim3(vbn), dim3(kBlock), 0, s, wv, vb0, x, r, (const TX*)p, (const TX*)q,
                           W.st, W.part_v);
      hipLaunchKernelGGL(k_fcg_red, dim3(nlev), dim3(kRedBlock), 0, s, 2, lo, wq.lev_begin, W.part_s, W.part_s2,
                         wv.lev_begin, W.part_v, W.st);
      MSKM_TRY(precond());
      if (vbn > 0)
        hipLaunchKernelGGL(k_fcg_dot<TX>, dim3(vbn), dim3(kBlock), 0, s, wv, vb0, (const TX*)z, (const TX*)q, W.st,
                           W.part_v);
      hipLaunchKernelGGL(k_fcg_red, dim3(nlev), dim3(kRedBlock), 0, s, 3, lo, wq.lev_begin, W.part_s, W.part_s2,
                         wv.lev_begin, W.part_v, W.st);
      if (vbn > 0) hipLaunchKernelGGL(k_fcg_dir<TX>, dim3(vbn), dim3(kBlock), 0, s, wv, vb0, (const TX*)z, p, W.st, 0);
    }
    MSKM_HIP_TRY(hipMemcpyAsync(fin.data(), W.st, h->L * sizeof(CgLevel), hipMemcpyDeviceToHost, s));
    MSKM_HIP_TRY(hipStreamSynchronize(s));
    bool any = false;
    for (int l = lo; l <= hi; ++l) any |= on[l] && !fin[l].done;
    if (!any) break;
  }
  MSKM_HIP_TRY(hipGetLastError());
  for (int l = lo; l <= hi; ++l) {
    if (!on[l]) continue;
    cs->iters_total += fin[l].iters;
    if (l < kMaxLevels) cs->last_iters[l] = fin[l].iters;
    if (fin[l].capped || !fin[l].done) cs->capped = true;
    if (fin[l].fallback) cs->warm_fallbacks += 1;  // the network was dropped on this level
  }
  return MSKM_OK;
}

template <typename T>
static void spmv_launch(hipStream_t s, int G, const Csr* A1, const T* v1, const Csr* A2, const T* v2, const T* x,
                        const T* b, T* y, T sign, int64_t r0, int64_t r1);

// beta = f - (T - D) t on rows [r0, r1): the Jacobi update, or one level's
// right-hand side of the forward substitution.
// y = b + sign * (T - D) x, or (full) b + sign * T x, on rows [r0, r1) from
// the sliced copies; false (nothing launched) when the lower copy is not
// built, the precision's values are not stored there, or the rows are not
// whole levels.
template <typename T>
static bool launch_lsell(mskm_hier* h, bool full, const T* x, const T* b, T* y, T sign, int64_t r0, int64_t r1) {
  const LSell& X = h->lsell;
  const Sell& S = h->sell;
  if (!X.built) return false;
  const T* lv;
  const T* dv;
  if constexpr (sizeof(T) == 8) {
    lv = X.val;
    dv = S.val;
  } else {
    lv = X.val32;
    dv = S.val32;
  }
  if (!lv || (full && !dv)) return false;
  const auto a = std::lower_bound(h->h_off.begin(), h->h_off.end(), r0);
  const auto e = std::lower_bound(h->h_off.begin(), h->h_off.end(), r1);
  if (a == h->h_off.end() || e == h->h_off.end() || *a != r0 || *e != r1) return false;
  const int64_t s0 = S.h_slice_begin[a - h->h_off.begin()], s1 = S.h_slice_begin[e - h->h_off.begin()];
  if (s1 <= s0) return true;
  const dim3 grid(nblk(s1 - s0, kBlock / kSellC));
  hipStream_t st = h->ctx->stream;
  if (full && !S.col16)
    hipLaunchKernelGGL((k_spmv_lsell<T, true, false>), grid, dim3(kBlock), 0, st, s0, s1, S.sptr, S.rows,
                       SellCols<false>{S.col}, dv, X.slice_seg, X.seg_ptr, X.seg_base, X.col16, lv, x, b, y, sign);
  else if (full)
    hipLaunchKernelGGL((k_spmv_lsell<T, true, true>), grid, dim3(kBlock), 0, st, s0, s1, S.sptr, S.rows,
                       SellCols<true>{S.col16, S.cbase}, dv, X.slice_seg, X.seg_ptr, X.seg_base, X.col16, lv, x, b, y,
                       sign);
  else
    hipLaunchKernelGGL((k_spmv_lsell<T, false, true>), grid, dim3(kBlock), 0, st, s0, s1, S.sptr, S.rows,
                       SellCols<true>{S.col16, S.cbase}, dv, X.slice_seg, X.seg_ptr, X.seg_base, X.col16, lv, x, b, y,
                       sign);
  return true;
}

template <typename TV, typename TX>
static void lower_update(mskm_hier* h, const TV* lval, const TX* t, const TX* f, TX* beta, int64_t r0, int64_t r1) {
  const int G = h->spmv_g[MSKM_OP_LOWER][sizeof(TX) == 4 ? 1 : 0];
  if constexpr (sizeof(TV) == sizeof(TX))
    if (G == kSellCode && launch_lsell<TX>(h, false, t, f, beta, (TX)-1, r0, r1)) return;
  spmv_launch<TX>(h->ctx->stream, G == kSellCode ? 16 + kVecFlag : G, &h->lower, lval, nullptr, nullptr, t, f, beta,
                  (TX)-1, r0, r1, h->prec, h->dim);
}

// alpha = T^-1 f in the internal order: monolithic (Jacobi sweeps on T' with
// CG on the levels below the top, then CG on D) or sequential (block forward
// substitution, one CG per level).
template <typename TV, typename TX>
static mskm_status solve_internal(mskm_hier* h, SolveWS& W, const TV* dval, const TV* lval, const TX* f, TX* alpha,
                                  const mskm_solve_opts* o, int* sweeps_done, CgStats* cs) {
  hipStream_t s = h->ctx->stream;
  const int64_t N = h->N;
  const int L = h->L;
  TX* beta = (TX*)W.beta;
  TX* t = (TX*)W.t;
  // learned start (with or without the block-Jacobi preconditioner), or the
  // previous sweep's solution as the start of the monolithic sweeps
  const bool learned = o->precond == MSKM_PRECOND_LEARNED || o->warm_start == MSKM_START_LEARNED;
  const mskm_mlp* mlp = learned ? o->mlp : nullptr;
  const bool prev = o->warm_start == MSKM_START_PREVIOUS;
  const bool bj = o->precond == MSKM_PRECOND_BLOCK_JACOBI;
  const bool flex = o->precond == MSKM_PRECOND_FLEX_LEARNED;  // sequential algorithm only (checked by the caller)
  const int maxit = o->max_cg_iters > 0 ? o->max_cg_iters : 20000;
  int K = o->check_every > 0 ? o->check_every : 8;
  K += K & 1;  // even chunk length
  std::vector<char> on(L, 0);
  if (o->algorithm == MSKM_ALG_SEQUENTIAL) {
    // block forward substitution, depth by depth (every group's level of
    // that depth in the same launches): rhs_l = f_l - sum_{k<l} B_{l,k} alpha_k
    MSKM_HIP_TRY(hipMemsetAsync(alpha, 0, N * sizeof(TX), s));
    const int D = (int)h->h_depth_begin.size() - 1;
    std::vector<char> next(L, 0);
    for (int d = 0; d < D; ++d) {
      const int l0 = h->h_depth_begin[d], l1 = h->h_depth_begin[d + 1];
      lower_update<TV, TX>(h, lval, alpha, f, beta, h->h_off[l0], h->h_off[l1]);
      std::fill(on.begin(), on.end(), 0);
      for (int l = l0; l < l1; ++l) on[l] = 1;
      std::fill(next.begin(), next.end(), 0);
      if (d + 1 < D)
        for (int l = l1; l < h->h_depth_begin[d + 2]; ++l) next[l] = 1;
      if (flex)
        MSKM_TRY((fcg_run<TV, TX>(h, W, dval, on, beta, alpha, o->cg_rtol, maxit, K, cs, o->mlp, true)));
      else
        MSKM_TRY((cg_run<TV, TX>(h, W, dval, on, beta, alpha, o->cg_rtol, maxit, false, K, cs, mlp, bj,
                                 d + 1 < D ? &next : nullptr)));
    }
    *sweeps_done = 0;
    return flush_deferred(h, W, cs);
  }
  // monolithic: Jacobi on T' beta = f from beta_0 = f, then D alpha = beta
  int Lmax = 0;
  for (int g = 0; g < h->ngroups; ++g) Lmax = std::max(Lmax, (int)h->h_group_levels[g]);
  const int S = o->sweeps > 0 ? o->sweeps : Lmax;
  MSKM_HIP_TRY(hipMemcpyAsync(beta, f, N * sizeof(TX), hipMemcpyDeviceToDevice, s));
  MSKM_HIP_TRY(hipMemsetAsync(t, 0, N * sizeof(TX), s));
  for (int l = 0; l < L; ++l) on[l] = h->h_next[l] >= 0;  // every level below its hierarchy's top
  for (int sw = 0; sw < S && Lmax > 1; ++sw) {
    MSKM_TRY((cg_run<TV, TX>(h, W, dval, on, beta, t, o->cg_rtol, maxit, prev && sw > 0, K, cs, nullptr, bj)));
    lower_update<TV, TX>(h, lval, t, f, beta, 0, N);
    *sweeps_done = sw + 1;
  }
  if (prev) MSKM_HIP_TRY(hipMemcpyAsync(alpha, t, N * sizeof(TX), hipMemcpyDeviceToDevice, s));
  std::fill(on.begin(), on.end(), 1);
  MSKM_TRY((cg_run<TV, TX>(h, W, dval, on, beta, alpha, o->cg_rtol, maxit, prev, K, cs, prev ? nullptr : mlp, bj)));
  return flush_deferred(h, W, cs);
}

// ------------------------------------------------------------- residual
//
// r = f - (D + Lo) alpha over the level-aligned blocks of the SpMV table,
// with per-block partials of r.r and f.f (summed per level, then per group,
// on the host in block order).

// Vector access of the residual kernels: an internal-order device vector, or
// an input-order [N][nrhs] vector read through the permutation (used by the
// allocation-free residual, which keeps no internal-order copies).
struct VecDirect {
  const double* v;
  __device__ __forceinline__ double operator()(int64_t i) const { return v[i]; }
};
struct VecPerm {
  const double* v;
  const int32_t* perm;
  int32_t nrhs, r;
  __device__ __forceinline__ double operator()(int64_t i) const { return v[(int64_t)perm[i] * nrhs + r]; }
};

// Lane gl's share of CSR row `row` dotted with x (FP64 values).
template <int G, typename VA>
__device__ __forceinline__ double res_row_part(const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                                               const double* __restrict__ val, const VA& x, int64_t row, int gl) {
  const int64_t e = rp[row + 1];
  double acc = 0.0;
  for (int64_t k = rp[row] + gl; k < e; k += G) acc += val[k] * x(col[k]);
  return acc;
}

template <typename VA>
__global__ void __launch_bounds__(kBlock)
    k_residual64(const WorkTable wt, const int64_t* __restrict__ drp, const int32_t* __restrict__ dc,
                 const double* __restrict__ dv, const int64_t* __restrict__ lrp, const int32_t* __restrict__ lc,
                 const double* __restrict__ lv, const VA a, const VA f, double* __restrict__ part,
                 double* __restrict__ rout) {
  constexpr int G = 16;
  __shared__ double sm[kBlock / kWave];
  const int blk = xcd_block_id(gridDim.x);
  const int64_t row0 = wt.row0[blk], row1 = wt.row1[blk];
  const int gl = threadIdx.x % G;
  double srr = 0.0, sff = 0.0;
  for (int64_t i = row0 + threadIdx.x / G; i < row1; i += kBlock / G) {
    double acc = group_sum<G>(res_row_part<G>(drp, dc, dv, a, i, gl));
    acc += group_sum<G>(res_row_part<G>(lrp, lc, lv, a, i, gl));
    if (gl == 0) {
      const double fi = f(i);
      const double ri = fi - acc;
      if (rout) rout[i] = ri;
      srr += ri * ri;
      sff += fi * fi;
    }
  }
  srr = block_sum(srr, sm);
  sff = block_sum(sff, sm);
  if (threadIdx.x == 0) {
    part[2 * blk] = srr;
    part[2 * blk + 1] = sff;
  }
}

// Same with split values (FP32-only hierarchies): v = (double)hi + (double)lo,
// the FP32 value and its stored FP32 remainder. Each lane reads four
// consecutive entries per (non-temporal, 16-byte) load from the row start
// rounded down to a multiple of 4, entries outside the row masked; the arrays
// carry a tail pad of kCsrPad entries. Lane gl's share of the row's dot (the
// caller sums over the G lanes).
template <int G, typename VA>
__device__ __forceinline__ double split_row_part(const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                                                 const float* __restrict__ hi, const float* __restrict__ lo,
                                                 const VA& x, int64_t row, int gl) {
  // one chunk of four entries per lane and step: two chunks in flight (as in
  // the CSR product) measured slower here (1.29 -> 1.59 ms on 389M nonzeros),
  // the three streams per chunk already keep enough loads outstanding
  const int64_t s = rp[row], e = rp[row + 1];
  double acc = 0.0;
  for (int64_t k = (s & ~(int64_t)3) + (int64_t)gl * 4; k < e; k += (int64_t)G * 4) {
    const sf4 h = __builtin_nontemporal_load(reinterpret_cast<const sf4*>(hi + k));
    const sf4 l = __builtin_nontemporal_load(reinterpret_cast<const sf4*>(lo + k));
    const si4 c = __builtin_nontemporal_load(reinterpret_cast<const si4*>(col + k));
    const float hv[4] = {h.x, h.y, h.z, h.w}, lv[4] = {l.x, l.y, l.z, l.w};
    const int32_t cv[4] = {c.x, c.y, c.z, c.w};
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (k + u >= s && k + u < e) acc += ((double)hv[u] + (double)lv[u]) * x(cv[u]);
  }
  return acc;
}

constexpr int kSplitG = 16;  // lanes per row of the split-value residual

template <typename VA>
__global__ void __launch_bounds__(kBlock)
    k_residual_split(const WorkTable wt, const int64_t* __restrict__ drp, const int32_t* __restrict__ dc,
                     const float* __restrict__ dh, const float* __restrict__ dl, const int64_t* __restrict__ lrp,
                     const int32_t* __restrict__ lc, const float* __restrict__ lh, const float* __restrict__ ll,
                     const VA a, const VA f, double* __restrict__ part, double* __restrict__ rout) {
  constexpr int G = kSplitG;
  __shared__ double sm[kBlock / kWave];
  const int blk = xcd_block_id(gridDim.x);
  const int64_t row0 = wt.row0[blk], row1 = wt.row1[blk];
  const int gl = threadIdx.x % G;
  double srr = 0.0, sff = 0.0;
  for (int64_t i = row0 + threadIdx.x / G; i < row1; i += kBlock / G) {
    double acc = split_row_part<G>(lrp, lc, lh, ll, a, i, gl) + split_row_part<G>(drp, dc, dh, dl, a, i, gl);
    acc = group_sum<G>(acc);
    if (gl == 0) {
      const double fi = f(i);
      const double ri = fi - acc;
      if (rout) rout[i] = ri;
      srr += ri * ri;
      sff += fi * fi;
    }
  }
  srr = block_sum(srr, sm);
  sff = block_sum(sff, sm);
  if (threadIdx.x == 0) {
    part[2 * blk] = srr;
    part[2 * blk + 1] = sff;
  }
}

// The residual product over the SpMV table's blocks: FP64 values when
// stored, else the split FP32 values (an FP32-only hierarchy stores the
// remainders). Partials r.r, f.f per block into part[2 b], part[2 b + 1].
template <typename VA>
static void launch_residual(mskm_hier* h, const VA& a, const VA& f, double* part, double* rout) {
  hipStream_t s = h->ctx->stream;
  const WorkTable& wt = h->wt_spmv;
  if (h->diag.val && h->lower.val) {
    hipLaunchKernelGGL(k_residual64<VA>, dim3(wt.nblocks), dim3(kBlock), 0, s, wt, h->diag.rowptr, h->diag.col,
                       h->diag.val, h->lower.rowptr, h->lower.col, h->lower.val, a, f, part, rout);
  } else {
    hipLaunchKernelGGL(k_residual_split<VA>, dim3(wt.nblocks), dim3(kBlock), 0, s, wt, h->diag.rowptr, h->diag.col,
                       h->diag.val32, h->diag.val32lo, h->lower.rowptr, h->lower.col, h->lower.val32,
                       h->lower.val32lo, a, f, part, rout);
  }
}

// The residual over the sliced copies (partials per block of the sliced
// table); false when the lower copy or the needed values are missing.
template <typename VA>
static bool launch_residual_sell(mskm_hier* h, const VA& a, const VA& f, double* part, double* rout) {
  const LSell& X = h->lsell;
  const Sell& S = h->sell;
  const WorkTable& wt = h->wt_sell;
  if (!X.built || wt.nblocks <= 0) return false;
  hipStream_t s = h->ctx->stream;
  const dim3 grid(wt.nblocks);
  if (X.val && S.val) {
    if (S.col16)
      hipLaunchKernelGGL((k_residual_sell<false, true, VA>), grid, dim3(kBlock), 0, s, wt, S.sptr, S.rows,
                         SellCols<true>{S.col16, S.cbase}, S.val, nullptr, nullptr, X.slice_seg, X.seg_ptr, X.seg_base,
                         X.col16, X.val, nullptr, nullptr, a, f, part, rout);
    else
      hipLaunchKernelGGL((k_residual_sell<false, false, VA>), grid, dim3(kBlock), 0, s, wt, S.sptr, S.rows,
                         SellCols<false>{S.col}, S.val, nullptr, nullptr, X.slice_seg, X.seg_ptr, X.seg_base, X.col16,
                         X.val, nullptr, nullptr, a, f, part, rout);
    return true;
  }
  if (X.val32 && X.lo && S.val32 && S.lo) {
    if (S.col16)
      hipLaunchKernelGGL((k_residual_sell<true, true, VA>), grid, dim3(kBlock), 0, s, wt, S.sptr, S.rows,
                         SellCols<true>{S.col16, S.cbase}, nullptr, S.val32, S.lo, X.slice_seg, X.seg_ptr, X.seg_base,
                         X.col16, nullptr, X.val32, X.lo, a, f, part, rout);
    else
      hipLaunchKernelGGL((k_residual_sell<true, false, VA>), grid, dim3(kBlock), 0, s, wt, S.sptr, S.rows,
                         SellCols<false>{S.col}, nullptr, S.val32, S.lo, X.slice_seg, X.seg_ptr, X.seg_base, X.col16,
                         nullptr, X.val32, X.lo, a, f, part, rout);
    return true;
  }
  return false;
}

// Residual of a = 0: r = f (partials of f.f twice).
__global__ void __launch_bounds__(kBlock)
    k_residual_zero(const WorkTable wt, const double* __restrict__ f, double* __restrict__ part,
                    double* __restrict__ rout) {
  __shared__ double sm[kBlock / kWave];
  const int blk = xcd_block_id(gridDim.x);
  const int64_t row0 = wt.row0[blk], row1 = wt.row1[blk];
  double sff = 0.0;
  for (int64_t i = row0 + threadIdx.x; i < row1; i += kBlock) {
    const double fi = f[i];
    if (rout) rout[i] = fi;
    sff += fi * fi;
  }
  sff = block_sum(sff, sm);
  if (threadIdx.x == 0) {
    part[2 * blk] = sff;
    part[2 * blk + 1] = sff;
  }
}

// ||f - T a|| / ||f|| per group (rel_groups, host [ngroups]) and the maximum
// over groups (*rel), internal order device vectors. rout (nullable)
// receives r. FP64 values are used when stored, else the split FP32 values
// (an FP32-only hierarchy stores the remainders).
static mskm_status residual_internal(mskm_hier* h, SolveWS& W, const double* a, const double* f, double* rel,
                                     double* rout, double* rel_groups = nullptr, bool a_zero = false) {
  hipStream_t s = h->ctx->stream;
  const WorkTable& wt = h->wt_spmv;
  const WorkTable* tab = &wt;  // the table whose blocks wrote the partials
  double* part = W.part_res;
  if (a_zero)
    hipLaunchKernelGGL(k_residual_zero, dim3(wt.nblocks), dim3(kBlock), 0, s, wt, f, part, rout);
  else if (!launch_residual_sell(h, VecDirect{a}, VecDirect{f}, part, rout))
    launch_residual(h, VecDirect{a}, VecDirect{f}, part, rout);
  else
    tab = &h->wt_sell;  // partials per block of the sliced table
  const double* hp = W.h_part_res;
  hipError_t e = hipMemcpyAsync(W.h_part_res, part, 2 * (size_t)tab->nblocks * 8, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail(MSKM_EDEVICE, std::string("residual: ") + hipGetErrorString(e));
  std::vector<double> rr(h->ngroups, 0.0), ff(h->ngroups, 0.0);
  for (int l = 0; l < h->L; ++l) {
    const int g = h->h_group[l];
    for (int b = tab->h_lev_begin[l]; b < tab->h_lev_begin[l + 1]; ++b) {
      rr[g] += hp[2 * b];
      ff[g] += hp[2 * b + 1];
    }
  }
  *rel = 0.0;
  for (int g = 0; g < h->ngroups; ++g) {
    const double rg = ff[g] > 0.0 ? std::sqrt(rr[g] / ff[g]) : std::sqrt(rr[g]);
    if (rel_groups) rel_groups[g] = rg;
    *rel = std::max(*rel, rg);
  }
  return MSKM_OK;
}

// ---------------------------------------------------------------- evaluate

// One wave per query point: f_L(y) = sum_l sum_{n in cells} alpha_n phi.
__global__ void __launch_bounds__(kBlock)
    k_evaluate(int dim, int L, const DevLevel* __restrict__ lev, const int32_t* __restrict__ cs_all,
               const double* __restrict__ xs, int64_t N, const double* __restrict__ a, const double* __restrict__ qy,
               int64_t nq, double* __restrict__ out, int nrhs, int rhs) {
  const int lane = threadIdx.x % kWave;
  const int64_t waves = (int64_t)gridDim.x * (kBlock / kWave);
  const double* X = xs;
  const double* Y = xs + N;
  const double* Z = xs + 2 * N;
  for (int64_t qi = (int64_t)blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave; qi < nq; qi += waves) {
    const double px = qy[qi * dim], py = qy[qi * dim + 1], pz = dim == 3 ? qy[qi * dim + 2] : 0.0;
    double acc = 0.0;
    for (int j = 0; j < L; ++j) {
      const DevLevel Lj = lev[j];
      if (Lj.n == 0) continue;
      const int cx = cell_coord(px, Lj.lo[0], Lj.inv_cell, Lj.nc[0]);
      const int cy = cell_coord(py, Lj.lo[1], Lj.inv_cell, Lj.nc[1]);
      const int cz = dim == 3 ? cell_coord(pz, Lj.lo[2], Lj.inv_cell, Lj.nc[2]) : 0;
      const int x0 = cx > 0 ? cx - 1 : 0, x1 = cx < Lj.nc[0] - 1 ? cx + 1 : Lj.nc[0] - 1;
      const int y0 = cy > 0 ? cy - 1 : 0, y1 = cy < Lj.nc[1] - 1 ? cy + 1 : Lj.nc[1] - 1;
      const int z0 = dim == 3 ? (cz > 0 ? cz - 1 : 0) : 0;
      const int z1 = dim == 3 ? (cz < Lj.nc[2] - 1 ? cz + 1 : Lj.nc[2] - 1) : 0;
      const int32_t* cs = cs_all + Lj.cs_off;
      for (int z = z0; z <= z1; ++z)
        for (int y = y0; y <= y1; ++y) {
          const int rk = (z * Lj.nc[1] + y) * Lj.nc[0];
          const int64_t b0 = cs[rk + x0], b1 = cs[rk + x1 + 1];
          for (int64_t t = b0 + lane; t < b1; t += kWave) {
            const double d2 = sqdist(dim, px, py, pz, X[t], Y[t], dim == 3 ? Z[t] : 0.0);
            if (d2 < Lj.d2max) acc += a[t] * phi31_d2(d2, Lj.delta);
          }
        }
    }
    acc = wave_sum(acc);
    if (lane == 0) out[qi * nrhs + rhs] = acc;
  }
}

// ------------------------------------------------------------ entry points

namespace {
// Device buffer: adopts a device pointer or stages a host array.
struct DevBuf {
  double* p = nullptr;
  bool own = false;
  ~DevBuf() {
    if (own) (void)hipFree(p);
  }
};

mskm_status stage_in(hipStream_t s, const double* src, size_t n, bool io_dev, DevBuf& b) {
  if (io_dev) {
    b.p = const_cast<double*>(src);
    return MSKM_OK;
  }
  MSKM_TRY(dalloc(&b.p, n));
  b.own = true;
  MSKM_HIP_TRY(hipMemcpyAsync(b.p, src, n * 8, hipMemcpyHostToDevice, s));
  return MSKM_OK;
}

mskm_status stage_out_alloc(double* dst, size_t n, bool io_dev, DevBuf& b) {
  if (io_dev) {
    b.p = dst;
    return MSKM_OK;
  }
  MSKM_TRY(dalloc(&b.p, n));
  b.own = true;
  return MSKM_OK;
}

mskm_status stage_out_copy(hipStream_t s, double* dst, size_t n, bool io_dev, DevBuf& b) {
  if (!io_dev) MSKM_HIP_TRY(hipMemcpyAsync(dst, b.p, n * 8, hipMemcpyDeviceToHost, s));
  MSKM_HIP_TRY(hipStreamSynchronize(s));
  return MSKM_OK;
}
}  // namespace

// y = bsign_b + sign * (A1 + A2) x over rows [r0, r1) with G lanes per row,
// G chosen at run time among the compiled widths.
template <typename T>
static void spmv_launch(hipStream_t s, int G, const Csr* A1, const T* v1, const Csr* A2, const T* v2, const T* x,
                        const T* b, T* y, T sign, int64_t r0, int64_t r1, const double* rec, int dim) {
  if (r1 <= r0) return;
  const int64_t* rp2 = A2 ? A2->rowptr : nullptr;
  const int32_t* c2 = A2 ? A2->col : nullptr;
  if (G >= 3 * kVecFlag) {
    const double4* r4 = reinterpret_cast<const double4*>(rec);
#define MSKM_REC_CASE(GG)                                                                                          \
  case GG:                                                                                                        \
    if (dim == 3)                                                                                                 \
      hipLaunchKernelGGL((k_spmv_rec<GG, 3, T>), dim3(nblk(r1 - r0, kBlock / GG)), dim3(kBlock), 0, s, A1->rowptr, \
                         A1->col, rp2, c2, r4, x, b, y, sign, r0, r1);                                            \
    else                                                                                                          \
      hipLaunchKernelGGL((k_spmv_rec<GG, 2, T>), dim3(nblk(r1 - r0, kBlock / GG)), dim3(kBlock), 0, s, A1->rowptr, \
                         A1->col, rp2, c2, r4, x, b, y, sign, r0, r1);                                            \
    return;
    switch (G - 3 * kVecFlag) {
      MSKM_REC_CASE(4)
      MSKM_REC_CASE(8)
      MSKM_REC_CASE(16)
      MSKM_REC_CASE(32)
      default:
        MSKM_REC_CASE(64)
    }
#undef MSKM_REC_CASE
  }
#define MSKM_SPMV_CASE(GG)                                                                                      \
  case GG:                                                                                                     \
    hipLaunchKernelGGL((k_spmv<GG, T, T, T>), dim3(nblk(r1 - r0, kBlock / GG)), dim3(kBlock), 0, s, A1->rowptr, \
                       A1->col, v1, rp2, c2, v2, x, b, y, sign, r0, r1);                                        \
    break;                                                                                                     \
  case GG + kVecFlag:                                                                                          \
    hipLaunchKernelGGL((k_spmv_v<GG, T, T, T>), dim3(nblk(r1 - r0, kBlock / GG)), dim3(kBlock), 0, s,          \
                       A1->rowptr, A1->col, v1, rp2, c2, v2, x, b, y, sign, r0, r1);                            \
    break;                                                                                                     \
  case GG + 2 * kVecFlag:                                                                                      \
    hipLaunchKernelGGL((k_spmv_v<GG, T, T, T, true>), dim3(nblk(r1 - r0, kBlock / GG)), dim3(kBlock), 0, s,    \
                       A1->rowptr, A1->col, v1, rp2, c2, v2, x, b, y, sign, r0, r1);                            \
    break;
  switch (G) {
    MSKM_SPMV_CASE(4)
    MSKM_SPMV_CASE(8)
    MSKM_SPMV_CASE(16)
    MSKM_SPMV_CASE(32)
    MSKM_SPMV_CASE(64)
    default:
      hipLaunchKernelGGL((k_spmv<32, T, T, T>), dim3(nblk(r1 - r0, kBlock / 32)), dim3(kBlock), 0, s, A1->rowptr,
                         A1->col, v1, rp2, c2, v2, x, b, y, sign, r0, r1);
  }
#undef MSKM_SPMV_CASE
}

// One SpMV launch of op in internal order (no permutation).
template <typename T>
static void launch_apply(mskm_hier* h, int op, const T* v1, const T* v2, const T* x, T* y) {
  const Csr* A1 = op == MSKM_OP_LOWER ? &h->lower : &h->diag;
  const Csr* A2 = op == MSKM_OP_FULL ? &h->lower : nullptr;
  const int G = h->spmv_g[op][sizeof(T) == 4 ? 1 : 0];
  if (G == kSellCode && op != MSKM_OP_DIAG) {  // the sliced copies of the lower (and diagonal) blocks
    if (!launch_lsell<T>(h, op == MSKM_OP_FULL, x, (const T*)nullptr, y, (T)1, 0, h->N))
      spmv_launch<T>(h->ctx->stream, 16 + kVecFlag, A1, v1, A2, v2, x, (const T*)nullptr, y, (T)1, 0, h->N, h->prec,
                     h->dim);
    return;
  }
  if (G == kSellCode || G == kSell32Code) {  // diagonal operator
    const dim3 grid(nblk(h->sell.nslices, kBlock / kSellC));
    if (h->sell.nslices <= 0) return;
    if (G == kSellCode && h->sell.col16)
      hipLaunchKernelGGL((k_spmv_sell<T, true>), grid, dim3(kBlock), 0, h->ctx->stream, h->sell.nslices, h->sell.sptr,
                         h->sell.rows, SellCols<true>{h->sell.col16, h->sell.cbase}, sell_values<T>(h->sell), x,
                         (const T*)nullptr, y, (T)1);
    else
      hipLaunchKernelGGL((k_spmv_sell<T, false>), grid, dim3(kBlock), 0, h->ctx->stream, h->sell.nslices,
                         h->sell.sptr, h->sell.rows, SellCols<false>{h->sell.col}, sell_values<T>(h->sell), x,
                         (const T*)nullptr, y, (T)1);
    return;
  }
  spmv_launch<T>(h->ctx->stream, G, A1, v1, A2, v2, x, (const T*)nullptr, y, (T)1, 0, h->N, h->prec, h->dim);
}

mskm_status apply_internal(mskm_hier* h, int op, int prec, const void* x, void* y, int repeats, float* avg_ms) {
  const bool f32 = prec == MSKM_PREC_FP32;
  if (f32 ? !h->diag.val32 : !h->diag.val) return fail(MSKM_ESTATE, "requested precision's values are not stored");
  hipStream_t s = h->ctx->stream;
  const Csr* A1 = op == MSKM_OP_LOWER ? &h->lower : &h->diag;
  MSKM_HIP_TRY(hipEventRecord(h->ctx->ev0, s));
  for (int k = 0; k < repeats; ++k) {
    if (f32)
      launch_apply<float>(h, op, A1->val32, h->lower.val32, (const float*)x, (float*)y);
    else
      launch_apply<double>(h, op, A1->val, h->lower.val, (const double*)x, (double*)y);
  }
  MSKM_HIP_TRY(hipEventRecord(h->ctx->ev1, s));
  MSKM_HIP_TRY(hipEventSynchronize(h->ctx->ev1));
  MSKM_HIP_TRY(hipGetLastError());
  float ms = 0.f;
  MSKM_HIP_TRY(hipEventElapsedTime(&ms, h->ctx->ev0, h->ctx->ev1));
  if (avg_ms) *avg_ms = ms / repeats;
  return MSKM_OK;
}

// Autotuner: for every operator and stored precision, time each lanes-per-row
// width on the hierarchy's own matrices (scratch vectors, `repeats` launches
// each after one warm-up) and keep the fastest.
mskm_status autotune(mskm_hier* h, int repeats, float* times_out) {
  static const int widths[kTuneVariants] = {4,    8,    16,   32,   64,   1004, 1008, 1016, 1032, 1064, 2004,
                                            2008, 2016, 2032, 2064, 3004, 3008, 3016, 3032, 3064, kSellCode,
                                            kSell32Code};
  double* x = nullptr;
  double* y = nullptr;
  MSKM_TRY(dalloc(&x, h->N));
  MSKM_TRY(dalloc(&y, h->N));
  hipStream_t s = h->ctx->stream;
  mskm_status st = MSKM_OK;
  if (hipMemsetAsync(x, 0, h->N * 8, s) != hipSuccess) st = fail(MSKM_EDEVICE, "memset");
  for (int op = 0; op < 3 && st == MSKM_OK; ++op) {
    for (int prec = 0; prec < 2 && st == MSKM_OK; ++prec) {
      if (prec == 0 ? !h->diag.val : !h->diag.val32) continue;
      float best = 1e30f;
      int bestg = h->spmv_g[op][prec];
      for (int wi = 0; wi < kTuneVariants && st == MSKM_OK; ++wi) {
        // lower and full operators: the sliced copies when the lower one is built (16-bit columns only)
        const bool lsell_ok = h->lsell.built && (prec == 0 ? h->lsell.val != nullptr : h->lsell.val32 != nullptr);
        if (widths[wi] >= kSell32Code && op != MSKM_OP_DIAG && !(widths[wi] == kSellCode && lsell_ok)) {
          if (times_out) times_out[(op * 2 + prec) * kTuneVariants + wi] = 0.f;
          continue;
        }
        h->spmv_g[op][prec] = widths[wi];
        float ms = 0.f;
        st = apply_internal(h, op, prec, x, y, 1, nullptr);
        if (st == MSKM_OK) st = apply_internal(h, op, prec, x, y, repeats, &ms);
        if (times_out) times_out[(op * 2 + prec) * kTuneVariants + wi] = ms;
        if (st == MSKM_OK && ms < best) {
          best = ms;
          bestg = widths[wi];
        }
      }
      h->spmv_g[op][prec] = bestg;
    }
  }
  (void)hipFree(x);
  (void)hipFree(y);
  if (st == MSKM_OK) {  // remember for hierarchies of the same shape on this context
    TuneEntry e{h->dim, h->L, h->N, h->diag.nnz, h->lower.nnz, {}};
    std::memcpy(e.g, h->spmv_g, sizeof(e.g));
    auto& c = h->ctx->tune_cache;
    bool found = false;
    for (auto& t : c)
      if (t.dim == e.dim && t.L == e.L && t.N == e.N && t.nnz_diag == e.nnz_diag && t.nnz_lower == e.nnz_lower) {
        t = e;
        found = true;
      }
    if (!found) c.push_back(e);
  }
  return st;
}

mskm_status apply_op(mskm_hier* h, int op, int prec, const double* x_in, int nrhs, double* y_in, bool io_dev) {
  hipStream_t s = h->ctx->stream;
  const int64_t N = h->N;
  const bool f32 = prec == MSKM_PREC_FP32;
  if (f32 ? !h->diag.val32 : !h->diag.val) return fail(MSKM_ESTATE, "requested precision's values are not stored");
  DevBuf X, Y;
  MSKM_TRY(stage_in(s, x_in, (size_t)N * nrhs, io_dev, X));
  MSKM_TRY(stage_out_alloc(y_in, (size_t)N * nrhs, io_dev, Y));
  void *xi = nullptr, *yi = nullptr;
  MSKM_TRY(dalloc(reinterpret_cast<double**>(&xi), N));
  MSKM_TRY(dalloc(reinterpret_cast<double**>(&yi), N));
  const Csr* A1 = op == MSKM_OP_LOWER ? &h->lower : &h->diag;
  for (int r = 0; r < nrhs; ++r) {
    if (f32) {
      hipLaunchKernelGGL(k_to_internal<float>, dim3(nblk(N)), dim3(kBlock), 0, s, X.p, h->perm, (float*)xi, N, nrhs, r);
      launch_apply<float>(h, op, A1->val32, h->lower.val32, (const float*)xi, (float*)yi);
      hipLaunchKernelGGL(k_to_input<float>, dim3(nblk(N)), dim3(kBlock), 0, s, (const float*)yi, h->perm, Y.p, N, nrhs,
                         r);
    } else {
      hipLaunchKernelGGL(k_to_internal<double>, dim3(nblk(N)), dim3(kBlock), 0, s, X.p, h->perm, (double*)xi, N, nrhs,
                         r);
      launch_apply<double>(h, op, A1->val, h->lower.val, (const double*)xi, (double*)yi);
      hipLaunchKernelGGL(k_to_input<double>, dim3(nblk(N)), dim3(kBlock), 0, s, (const double*)yi, h->perm, Y.p, N,
                         nrhs, r);
    }
  }
  mskm_status st = stage_out_copy(s, y_in, (size_t)N * nrhs, io_dev, Y);
  (void)hipFree(xi);
  (void)hipFree(yi);
  MSKM_HIP_TRY(hipGetLastError());
  return st;
}

mskm_status solve(mskm_hier* h, const double* f_in, int nrhs, const mskm_solve_opts* o, double* alpha_out,
                  mskm_report* rep) {
  if (nrhs > 1 && mr_supported(nrhs)) return solve_multi(h, f_in, nrhs, o, alpha_out, rep);
  hipStream_t s = h->ctx->stream;
  const int64_t N = h->N;
  const bool io_dev = (o->flags & MSKM_IO_DEVICE) != 0;
  const bool mixed = o->precision == MSKM_PREC_FP32;
  if (mixed ? !h->diag.val32 : !h->diag.val) return fail(MSKM_ESTATE, "requested precision's values are not stored");
  if (o->precond == MSKM_PRECOND_BLOCK_JACOBI || o->precond == MSKM_PRECOND_FLEX_LEARNED)
    MSKM_TRY(build_block_jacobi(h));
  DevBuf F, A;
  MSKM_TRY(stage_in(s, f_in, (size_t)N * nrhs, io_dev, F));
  MSKM_TRY(stage_out_alloc(alpha_out, (size_t)N * nrhs, io_dev, A));
  SolveWS* Wp = nullptr;
  MSKM_TRY(get_ws(h, &Wp));
  SolveWS& W = *Wp;
  double* fi = W.fi;
  double* ai = W.ai;
  CgStats cs;
  int sweeps_done = 0, refine = 0;
  double worst_rel = 0.0;
  MSKM_HIP_TRY(hipEventRecord(h->ctx->ev0, s));
  for (int r = 0; r < nrhs; ++r) {
    hipLaunchKernelGGL(k_to_internal<double>, dim3(nblk(N)), dim3(kBlock), 0, s, F.p, h->perm, fi, N, nrhs, r);
    double rel = 0.0;
    if (!mixed) {
      MSKM_TRY((solve_internal<double, double>(h, W, h->diag.val, h->lower.val, fi, ai, o, &sweeps_done, &cs)));
      MSKM_TRY(residual_internal(h, W, ai, fi, &rel, nullptr));
    } else {
      // FP64 residual refinement around FP32 inner solves (values, vectors and
      // SpMV accumulation in FP32, dots in FP64)
      const int maxref = o->max_refine > 0 ? o->max_refine : 10;
      MSKM_HIP_TRY(hipMemsetAsync(ai, 0, N * 8, s));
      refine = 0;
      for (;;) {
        MSKM_TRY(residual_internal(h, W, ai, fi, &rel, W.res, nullptr, refine == 0));  // alpha = 0 at the start
        if (rel <= o->target_rel_residual || refine >= maxref) break;
        hipLaunchKernelGGL((k_convert<double, float>), dim3(nblk(N)), dim3(kBlock), 0, s, (const double*)W.res, W.f32,
                           N);
        // inner tolerance: cg_rtol for the first round; later rounds only
        // need to shrink the current residual to the target (with margin)
        mskm_solve_opts oi = *o;
        if (refine > 0) oi.cg_rtol = std::min(0.1, std::max(o->cg_rtol, 0.5 * o->target_rel_residual / rel));
        MSKM_TRY((solve_internal<float, float>(h, W, h->diag.val32, h->lower.val32, W.f32, W.a32, &oi, &sweeps_done,
                                               &cs)));
        hipLaunchKernelGGL(k_axpy_f32, dim3(nblk(N)), dim3(kBlock), 0, s, W.a32, ai, N);
        ++refine;
      }
    }
    worst_rel = std::max(worst_rel, rel);
    hipLaunchKernelGGL(k_to_input<double>, dim3(nblk(N)), dim3(kBlock), 0, s, (const double*)ai, h->perm, A.p, N, nrhs,
                       r);
  }
  MSKM_HIP_TRY(hipEventRecord(h->ctx->ev1, s));
  MSKM_TRY(stage_out_copy(s, alpha_out, (size_t)N * nrhs, io_dev, A));
  float ms = 0.f;
  MSKM_HIP_TRY(hipEventElapsedTime(&ms, h->ctx->ev0, h->ctx->ev1));
  // the mixed path is decided by its FP64 outer residual alone (its FP32 inner
  // solves stop at their attainable accuracy by design)
  const bool enoconv = mixed ? worst_rel > o->target_rel_residual : cs.capped;
  if (rep) {
    std::memset(rep, 0, sizeof(*rep));
    rep->levels = h->L;
    rep->sweeps_done = sweeps_done;
    rep->refine_steps = refine;
    rep->cg_iters_total = cs.iters_total;
    for (int l = 0; l < std::min(h->L, 64); ++l) rep->cg_iters_last[l] = cs.last_iters[l];  // first 64 levels
    rep->rel_residual = worst_rel;
    rep->solve_ms = ms;
    rep->warm_fallbacks = cs.warm_fallbacks;
  }
  MSKM_HIP_TRY(hipGetLastError());
  return enoconv ? MSKM_ENOCONV : MSKM_OK;
}

__global__ void __launch_bounds__(kBlock) k_axpy64(const double* __restrict__ d, double* __restrict__ a, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) a[i] += d[i];
}

// Thresholded solve (Section 4, eq. (perturbed_split)): Jacobi sweeps on
// (I - M~) beta~ = r, each one product with the truncated blocks X~
// (beta~ <- r - X~ beta~, from beta~ = r), then alpha~ = D^-1 beta~ by CG on
// every level. With a target residual the perturbed solve is the inner
// solve of an FP64 residual refinement: alpha += alpha~(f - T alpha) until
// ||f - T alpha|| / ||f|| <= target (the refinement converges when the
// truncation is small, ||M - M~|| < 1 in effect).
mskm_status trunc_solve(mskm_hier* h, const Csr& X, const double* f_in, const mskm_solve_opts* o, double* alpha_out,
                        mskm_report* rep) {
  hipStream_t s = h->ctx->stream;
  const int64_t N = h->N;
  const bool io_dev = (o->flags & MSKM_IO_DEVICE) != 0;
  if (o->precision != MSKM_PREC_FP64) return fail(MSKM_EINVAL, "the thresholded solve runs in FP64");
  if (!h->diag.val) return fail(MSKM_ESTATE, "FP64 values are not stored");
  const bool bj = o->precond == MSKM_PRECOND_BLOCK_JACOBI;
  if (bj) MSKM_TRY(build_block_jacobi(h));
  DevBuf F, A;
  MSKM_TRY(stage_in(s, f_in, (size_t)N, io_dev, F));
  MSKM_TRY(stage_out_alloc(alpha_out, (size_t)N, io_dev, A));
  SolveWS* Wp = nullptr;
  MSKM_TRY(get_ws(h, &Wp));
  SolveWS& W = *Wp;
  int Lmax = 0;
  for (int g = 0; g < h->ngroups; ++g) Lmax = std::max(Lmax, (int)h->h_group_levels[g]);
  const int S = o->sweeps > 0 ? o->sweeps : Lmax - 1;
  const int maxit = o->max_cg_iters > 0 ? o->max_cg_iters : 20000;
  int K = o->check_every > 0 ? o->check_every : 8;
  K += K & 1;
  const bool refine_on = o->target_rel_residual > 0.0;
  const int maxref = refine_on ? (o->max_refine > 0 ? o->max_refine : 10) : 1;
  CgStats cs;
  std::vector<char> on(h->L, 1);
  double rel = 0.0;
  int rounds = 0;
  MSKM_HIP_TRY(hipEventRecord(h->ctx->ev0, s));
  hipLaunchKernelGGL(k_to_internal<double>, dim3(nblk(N)), dim3(kBlock), 0, s, F.p, h->perm, W.fi, N, 1, 0);
  MSKM_HIP_TRY(hipMemsetAsync(W.ai, 0, N * 8, s));
  MSKM_TRY(residual_internal(h, W, W.ai, W.fi, &rel, W.res, nullptr, true));  // r = f
  while (rounds < maxref && !(refine_on && rel <= o->target_rel_residual)) {
    double* b = W.beta;
    double* nb = W.t;
    MSKM_HIP_TRY(hipMemcpyAsync(b, W.res, N * 8, hipMemcpyDeviceToDevice, s));
    for (int sw = 0; sw < S; ++sw) {
      spmv_launch<double>(s, 16 + kVecFlag, &X, X.val, nullptr, nullptr, b, W.res, nb, -1.0, 0, N, h->prec, h->dim);
      std::swap(b, nb);
    }
    double rtol = o->cg_rtol;
    if (refine_on && rounds > 0) rtol = std::min(0.1, std::max(o->cg_rtol, 0.5 * o->target_rel_residual / rel));
    MSKM_TRY((cg_run<double, double>(h, W, h->diag.val, on, b, nb, rtol, maxit, false, K, &cs, nullptr, bj)));
    MSKM_TRY(flush_deferred(h, W, &cs));
    hipLaunchKernelGGL(k_axpy64, dim3(nblk(N)), dim3(kBlock), 0, s, (const double*)nb, W.ai, N);
    ++rounds;
    MSKM_TRY(residual_internal(h, W, W.ai, W.fi, &rel, W.res));
  }
  hipLaunchKernelGGL(k_to_input<double>, dim3(nblk(N)), dim3(kBlock), 0, s, (const double*)W.ai, h->perm, A.p, N, 1, 0);
  MSKM_HIP_TRY(hipEventRecord(h->ctx->ev1, s));
  MSKM_TRY(stage_out_copy(s, alpha_out, (size_t)N, io_dev, A));
  float ms = 0.f;
  MSKM_HIP_TRY(hipEventElapsedTime(&ms, h->ctx->ev0, h->ctx->ev1));
  if (rep) {
    std::memset(rep, 0, sizeof(*rep));
    rep->levels = h->L;
    rep->sweeps_done = S;
    rep->refine_steps = rounds;
    rep->cg_iters_total = cs.iters_total;
    for (int l = 0; l < std::min(h->L, 64); ++l) rep->cg_iters_last[l] = cs.last_iters[l];
    rep->rel_residual = rel;
    rep->solve_ms = ms;
  }
  MSKM_HIP_TRY(hipGetLastError());
  const bool enoconv = refine_on ? rel > o->target_rel_residual : cs.capped;
  return enoconv ? MSKM_ENOCONV : MSKM_OK;
}

// Training pairs for the learned warm start: for each right-hand side a
// plain FP64 sequential solve gives alpha; each level's own rhs is then
// beta = f - (T - D) alpha (the residual the sequential algorithm hands to
// that level), so (beta_l, alpha_l) is one (rhs -> correction) pair per level.
mskm_status train_pairs(mskm_hier* h, const double* f, int nrhs, bool io_dev, double cg_rtol,
                        std::vector<double*>* rhs_int, std::vector<double*>* alpha_int) {
  hipStream_t s = h->ctx->stream;
  const int64_t N = h->N;
  DevBuf F;
  MSKM_TRY(stage_in(s, f, (size_t)N * nrhs, io_dev, F));
  SolveWS* Wp = nullptr;
  MSKM_TRY(get_ws(h, &Wp));
  mskm_solve_opts o;
  mskm_solve_opts_default(&o);
  o.algorithm = MSKM_ALG_SEQUENTIAL;
  o.cg_rtol = cg_rtol;
  for (int r = 0; r < nrhs; ++r) {
    double *bi = nullptr, *ai = nullptr;
    MSKM_TRY(dalloc(&bi, N));
    rhs_int->push_back(bi);
    MSKM_TRY(dalloc(&ai, N));
    alpha_int->push_back(ai);
    hipLaunchKernelGGL(k_to_internal<double>, dim3(nblk(N)), dim3(kBlock), 0, s, F.p, h->perm, Wp->fi, N, nrhs, r);
    CgStats cs;
    int sw = 0;
    MSKM_TRY((solve_internal<double, double>(h, *Wp, h->diag.val, h->lower.val, Wp->fi, ai, &o, &sw, &cs)));
    lower_update<double, double>(h, h->lower.val, ai, Wp->fi, bi, 0, N);
  }
  MSKM_HIP_TRY(hipStreamSynchronize(s));
  return MSKM_OK;
}

mskm_status residual(mskm_hier* h, const double* alpha, const double* f, int nrhs, double* rel_out, bool io_dev) {
  hipStream_t s = h->ctx->stream;
  const int64_t N = h->N;
  DevBuf A, F;
  MSKM_TRY(stage_in(s, alpha, (size_t)N * nrhs, io_dev, A));
  MSKM_TRY(stage_in(s, f, (size_t)N * nrhs, io_dev, F));
  SolveWS* Wp = nullptr;  // the solver workspace's internal-order vectors and residual partials
  MSKM_TRY(get_ws(h, &Wp));
  double* ai = Wp->ai;
  double* fi = Wp->fi;
  mskm_status st = MSKM_OK;
  for (int r = 0; r < nrhs && st == MSKM_OK; ++r) {
    hipLaunchKernelGGL(k_to_internal<double>, dim3(nblk(N)), dim3(kBlock), 0, s, A.p, h->perm, ai, N, nrhs, r);
    hipLaunchKernelGGL(k_to_internal<double>, dim3(nblk(N)), dim3(kBlock), 0, s, F.p, h->perm, fi, N, nrhs, r);
    double worst = 0.0;
    st = residual_internal(h, *Wp, ai, fi, &worst, nullptr, rel_out + (size_t)r * h->ngroups);
  }
  return st;
}

mskm_status evaluate(mskm_hier* h, const double* alpha, int nrhs, const double* query, int64_t nq, double* out,
                     bool io_dev) {
  hipStream_t s = h->ctx->stream;
  const int64_t N = h->N;
  DevBuf A, Q, O;
  MSKM_TRY(stage_in(s, alpha, (size_t)N * nrhs, io_dev, A));
  MSKM_TRY(stage_in(s, query, (size_t)nq * h->dim, io_dev, Q));
  MSKM_TRY(stage_out_alloc(out, (size_t)nq * nrhs, io_dev, O));
  // internal-order coefficients: the solver workspace's vector when one exists
  // (no allocation, no implicit device synchronisation), else a scratch vector
  double* ai = h->solve_ws ? static_cast<SolveWS*>(h->solve_ws)->ai : nullptr;
  const bool own = ai == nullptr;
  if (own) MSKM_TRY(dalloc(&ai, N));
  for (int r = 0; r < nrhs; ++r) {
    hipLaunchKernelGGL(k_to_internal<double>, dim3(nblk(N)), dim3(kBlock), 0, s, A.p, h->perm, ai, N, nrhs, r);
    if (nq > 0)
      hipLaunchKernelGGL(k_evaluate, dim3(nblk(nq, kBlock / kWave)), dim3(kBlock), 0, s, h->dim, h->L, h->d_lev,
                         h->cell_start, h->xs, N, ai, Q.p, nq, O.p, nrhs, r);
  }
  mskm_status st = stage_out_copy(s, out, (size_t)nq * nrhs, io_dev, O);
  if (own) (void)hipFree(ai);
  MSKM_HIP_TRY(hipGetLastError());
  return st;
}


// ------------------------------------------------------------- timing

template <typename T>
__global__ void __launch_bounds__(kBlock) k_fill(T* __restrict__ v, int64_t n, T x) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) v[i] = x;
}

// Mean device time of the CG product kernel that the preconditioned
// single-reduction CG launches for one level (q = A_l z with the partials
// z.q, z.r and r.r), in the hierarchy's current diagonal variant and the
// given precision, launched `repeats` times between two events.
template <typename TV, typename TX>
static mskm_status time_cg_product_t(mskm_hier* h, const TV* dval, int level, int repeats, float* avg_ms) {
  hipStream_t s = h->ctx->stream;
  SolveWS* Wp = nullptr;
  MSKM_TRY(get_ws(h, &Wp));
  SolveWS& W = *Wp;
  const int G = h->spmv_g[MSKM_OP_DIAG][sizeof(TV) == 4 ? 1 : 0];
  const bool sell = G == kSellCode || G == kSell32Code;
  const WorkTable& wq = sell ? h->wt_sell : h->wt_spmv;
  const int qb0 = wq.h_lev_begin[level], qbn = wq.h_lev_begin[level + 1] - qb0;
  const int64_t N = h->N;
  TX* z = (TX*)W.z;
  TX* r = (TX*)W.r;
  hipLaunchKernelGGL(k_fill<TX>, dim3(nblk(N)), dim3(kBlock), 0, s, z, N, (TX)1);
  hipLaunchKernelGGL(k_fill<TX>, dim3(nblk(N)), dim3(kBlock), 0, s, r, N, (TX)1);
  MSKM_HIP_TRY(hipMemsetAsync(W.st, 0, 2 * (size_t)h->L * sizeof(CgLevel), s));  // every level running
  MSKM_HIP_TRY(hipEventRecord(h->ctx->ev0, s));
  const bool split = h->h_off[level + 1] - h->h_off[level] <= kSplitProductRows;  // as the solver launches it
  for (int k = 0; k < repeats; ++k)
    launch_cg_product<TV, TX>(h, W, dval, G, qb0, qbn, z, (TX*)W.q, W.part_s2, r, W.part_s3, W.st, split);
  MSKM_HIP_TRY(hipEventRecord(h->ctx->ev1, s));
  MSKM_HIP_TRY(hipEventSynchronize(h->ctx->ev1));
  float ms = 0.f;
  MSKM_HIP_TRY(hipEventElapsedTime(&ms, h->ctx->ev0, h->ctx->ev1));
  if (avg_ms) *avg_ms = ms / (float)repeats;
  MSKM_HIP_TRY(hipGetLastError());
  return MSKM_OK;
}

mskm_status time_cg_product(mskm_hier* h, int level, int prec, int repeats, float* avg_ms) {
  if (prec == MSKM_PREC_FP32) {
    if (!h->diag.val32) return fail(MSKM_ESTATE, "FP32 values are not stored");
    return time_cg_product_t<float, float>(h, h->diag.val32, level, repeats, avg_ms);
  }
  if (!h->diag.val) return fail(MSKM_ESTATE, "FP64 values are not stored");
  return time_cg_product_t<double, double>(h, h->diag.val, level, repeats, avg_ms);
}

// ------------------------------------------------ allocation-free residual
//
// mskm_residual_noalloc takes the per-block partials of the residual product
// from `scratch`, a static device array (one copy per device, held until the
// process ends), instead of the solver workspace, and reduces them per
// group on the device: nothing is allocated and the host never waits. The
// partials are fully rewritten by every product, so nothing needs clearing.
// Calls that overlap on one device share the array and race.
constexpr size_t kNoallocDoubles = (size_t)1 << 18;  // 2 MiB: r.r and f.f of up to 131072 blocks
static __device__ __align__(256) double scratch[kNoallocDoubles];
constexpr int kNoallocDevices = 64;
static double* g_scratch[kNoallocDevices] = {};
static std::mutex g_scratch_mu;

// Device address of this device's `scratch` (the symbol's name is a host
// stand-in and must not reach a kernel). Called with `device` current.
mskm_status noalloc_init(int device) {
  if (device < 0 || device >= kNoallocDevices) return fail(MSKM_ELIMIT, "device index beyond 63");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch[device]) return MSKM_OK;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p) return fail(MSKM_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
  g_scratch[device] = static_cast<double*>(p);
  return MSKM_OK;
}

// rel[g] = sqrt(rr_g / ff_g) (sqrt(rr_g) when ff_g = 0), rr_g and ff_g the
// sums of the partials of group g's levels; one workgroup per group, a
// fixed-order sum (deterministic). A group's first level is its group index
// (depth 0 of every group comes first, in group order).
__global__ void __launch_bounds__(kBlock)
    k_residual_rel(int L, const DevLevel* __restrict__ lev, const int32_t* __restrict__ lev_begin,
                   const double* __restrict__ part, double* __restrict__ rel) {
  __shared__ double sm[kBlock / kWave];
  const int g = blockIdx.x;
  double rr = 0.0, ff = 0.0;
  for (int l = 0; l < L; ++l) {
    if (lev[l].first != g) continue;
    for (int b = lev_begin[l] + (int)threadIdx.x; b < lev_begin[l + 1]; b += kBlock) {
      rr += part[2 * b];
      ff += part[2 * b + 1];
    }
  }
  rr = block_sum(rr, sm);
  ff = block_sum(ff, sm);
  if (threadIdx.x == 0) rel[g] = ff > 0.0 ? sqrt(rr / ff) : sqrt(rr);
}

mskm_status residual_noalloc(mskm_hier* h, const double* alpha, const double* f, int nrhs, double* rel_out) {
  const WorkTable& wt = h->wt_spmv;
  if (2 * (size_t)wt.nblocks > kNoallocDoubles)
    return fail(MSKM_ELIMIT, "mskm_residual_noalloc: " + std::to_string(wt.nblocks) +
                                 " row blocks exceed the scratch limit of 131072 (about 8.4M points)");
  double* part = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    part = h->ctx->device < kNoallocDevices ? g_scratch[h->ctx->device] : nullptr;
  }
  if (!part) return fail(MSKM_ESTATE, "mskm_residual_noalloc: scratch not initialised for this device");
  hipStream_t s = h->ctx->stream;
  for (int r = 0; r < nrhs; ++r) {
    launch_residual(h, VecPerm{alpha, h->perm, nrhs, r}, VecPerm{f, h->perm, nrhs, r}, part, nullptr);
    hipLaunchKernelGGL(k_residual_rel, dim3(h->ngroups), dim3(kBlock), 0, s, h->L, h->d_lev, wt.lev_begin, part,
                       rel_out + (size_t)r * h->ngroups);
  }
  MSKM_HIP_TRY(hipGetLastError());
  return MSKM_OK;
}

}  // namespace mskm
