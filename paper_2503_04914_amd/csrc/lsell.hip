// Sliced copy of the strictly-lower blocks (the B_{k,j}, j < k, of eq.
// (bigt)) for bandwidth-bound products: y = b + sign (T - D) x, y = b + sign
// T x, and the FP64 residual f - T alpha.
//
// Layout: the rows of every level in the slices of the diagonal copy (64
// consecutive internal rows, one row per lane). Within a slice of level k,
// one segment per coarser level j of the hierarchy (coarsest first, the
// order of a lower CSR row), each laid out like a diagonal slice: its width
// is the slice's largest count of level-j entries in a row, rounded up to 4,
// and entry e of slot t sits at seg_ptr + (e / 4) 4 kSellC + 4 t + e % 4 (four
// consecutive entries of a row side by side, a wave's load one contiguous
// 1 KiB run). Columns are 16-bit offsets from the segment's smallest column:
// a row's level-j neighbours lie within a few cell rows of level j, so every
// segment spans far fewer than 65536 points in 2-D and 3-D (the copy is not
// built otherwise). Rows shorter than the width are padded with value 0 and
// the segment's smallest column.
#include <algorithm>
#include <cmath>

#include "device_common.h"

namespace mskm {

// One wave per slice: for each of the slice's segments (level j, the q-th
// coarser level), the width in entries x kSellC and the smallest column; a
// segment whose columns span more than 65536 points raises *wide. A row's
// level-j entries are the run of cnt_lv[row][q] entries after those of the
// coarser levels (columns ascend, coarsest level first); cnt_lv is
// level-major, cnt_lv[q N + row].
__global__ void __launch_bounds__(kSellC)
    k_lsell_count(int64_t s0, int64_t ns, int64_t seg0, int nseg_per_slice, const int32_t* __restrict__ rows,
                  const int64_t* __restrict__ rp, const int32_t* __restrict__ col, const int32_t* __restrict__ cnt_lv,
                  int64_t N, int64_t* __restrict__ w, int32_t* __restrict__ base, int32_t* __restrict__ wide) {
  if (blockIdx.x >= ns) return;
  const int64_t sl = s0 + blockIdx.x;
  const int t = threadIdx.x;
  const int32_t row = rows[sl * kSellC + t];
  int64_t a = row >= 0 ? rp[row] : 0;
  for (int q = 0; q < nseg_per_slice; ++q) {
    const int64_t n = row >= 0 ? cnt_lv[q * N + row] : 0;
    int64_t cnt = n;
    int32_t lo = n > 0 ? col[a] : INT32_MAX, hi = n > 0 ? col[a + n - 1] : -1;
#pragma unroll
    for (int o = kSellC / 2; o > 0; o >>= 1) {
      cnt = max(cnt, (int64_t)__shfl_xor(cnt, o, kSellC));
      lo = min(lo, __shfl_xor(lo, o, kSellC));
      hi = max(hi, __shfl_xor(hi, o, kSellC));
    }
    if (t == 0) {
      const int64_t sg = seg0 + (int64_t)blockIdx.x * nseg_per_slice + q;
      w[sg] = (cnt + 3) / 4 * 4 * kSellC;
      base[sg] = hi >= 0 ? lo : 0;
      if (hi >= 0 && hi - lo > 65535) atomicAdd(wide, 1);
    }
    a += n;
  }
}

// One workgroup of kLsWaves waves per slice. Wave w copies slots 16w ..
// 16w + 15; lane i of the wave takes slot 16w + i % 16 and, of each segment,
// the 4-entry groups g = i / 16, i / 16 + 4, ...: it loads entries 4g ..
// 4g + 3 of its row's level-j run (one 16-byte load when all four lie inside
// the run, zero past the row's count) and stores them as one 4-wide vector.
// Per instruction the loads read 64 consecutive bytes of each of 16 rows and
// the stores write 4 runs of 16 consecutive slots (256 bytes of FP32 values
// each). No LDS and no barriers.
constexpr int kLsWaves = 4;
constexpr int kLsRows = kSellC / kLsWaves;   // slots per wave
constexpr int kLsGroups = kSellC / kLsRows;  // groups per wave step
__global__ void __launch_bounds__(kLsWaves * kSellC)
    k_lsell_fill(int64_t s0, int64_t ns, int64_t seg0, int nseg_per_slice, const int32_t* __restrict__ rows,
                 const int64_t* __restrict__ rp, const int32_t* __restrict__ col, const double* __restrict__ val,
                 const float* __restrict__ val32, const float* __restrict__ lo32, const int32_t* __restrict__ cnt_lv,
                 int64_t N, const int64_t* __restrict__ seg_ptr, const int32_t* __restrict__ base,
                 uint16_t* __restrict__ scol, double* __restrict__ sval, float* __restrict__ sval32,
                 float* __restrict__ slo) {
  if (blockIdx.x >= ns) return;
  const int64_t sl = s0 + blockIdx.x;
  const int lane = threadIdx.x % kSellC, w = threadIdx.x / kSellC;
  const int t = w * kLsRows + lane % kLsRows, gl = lane / kLsRows;
  const int32_t row = rows[sl * kSellC + t];
  int64_t a = row >= 0 ? rp[row] : 0;
  typedef unsigned short us4 __attribute__((ext_vector_type(4)));
  for (int q = 0; q < nseg_per_slice; ++q) {
    const int64_t n = row >= 0 ? cnt_lv[q * N + row] : 0;
    const int64_t sg = seg0 + (int64_t)blockIdx.x * nseg_per_slice + q;
    const int64_t e0 = seg_ptr[sg], groups = (seg_ptr[sg + 1] - e0) / (4 * kSellC);
    const int32_t cb = base[sg];
    for (int64_t g = gl; g < groups; g += kLsGroups) {
      const int64_t d = e0 + g * (4 * kSellC) + 4 * t;
      const int64_t k = 4 * g, src = a + k;
      int4 c;
      float4 v32 = make_float4(0.f, 0.f, 0.f, 0.f), vlo = v32;
      double2 v64a = make_double2(0.0, 0.0), v64b = v64a;
      if (k + 4 <= n) {  // the whole group inside the run: 16-byte loads (4-byte aligned)
        __builtin_memcpy(&c, col + src, 16);
        if (sval32) __builtin_memcpy(&v32, val32 + src, 16);
        if (slo) __builtin_memcpy(&vlo, lo32 + src, 16);
        if (sval) {
          __builtin_memcpy(&v64a, val + src, 16);
          __builtin_memcpy(&v64b, val + src + 2, 16);
        }
      } else {
        const bool in0 = k < n, in1 = k + 1 < n, in2 = k + 2 < n;  // k + 3 < n is false here
        c = make_int4(in0 ? col[src] : cb, in1 ? col[src + 1] : cb, in2 ? col[src + 2] : cb, cb);
        if (sval32) v32 = make_float4(in0 ? val32[src] : 0.f, in1 ? val32[src + 1] : 0.f, in2 ? val32[src + 2] : 0.f, 0.f);
        if (slo) vlo = make_float4(in0 ? lo32[src] : 0.f, in1 ? lo32[src + 1] : 0.f, in2 ? lo32[src + 2] : 0.f, 0.f);
        if (sval) {
          v64a = make_double2(in0 ? val[src] : 0.0, in1 ? val[src + 1] : 0.0);
          v64b = make_double2(in2 ? val[src + 2] : 0.0, 0.0);
        }
      }
      us4 c4;
      c4.x = (uint16_t)(c.x - cb);
      c4.y = (uint16_t)(c.y - cb);
      c4.z = (uint16_t)(c.z - cb);
      c4.w = (uint16_t)(c.w - cb);
      *reinterpret_cast<us4*>(scol + d) = c4;
      if (sval) {
        *reinterpret_cast<double2*>(sval + d) = v64a;
        *reinterpret_cast<double2*>(sval + d + 2) = v64b;
      }
      if (sval32) *reinterpret_cast<float4*>(sval32 + d) = v32;
      if (slo) *reinterpret_cast<float4*>(slo + d) = vlo;
    }
    a += n;
  }
}

mskm_status build_lsell(mskm_hier* h, bool want64, bool want32, const int32_t* cnt_lv) {
  hipStream_t s = h->ctx->stream;
  const Sell& S = h->sell;
  LSell& X = h->lsell;
  const int L = h->L;
  if (S.nslices == 0 || h->lower.nnz == 0) return MSKM_OK;
  // segments: every slice of level l has depth(l) of them
  std::vector<int64_t> seg0(L + 1, 0);
  for (int l = 0; l < L; ++l) seg0[l + 1] = seg0[l] + (S.h_slice_begin[l + 1] - S.h_slice_begin[l]) * h->h_depth[l];
  X.nseg = seg0[L];
  if (X.nseg == 0) return MSKM_OK;
  int64_t *w = nullptr, *part = nullptr;
  int32_t* wide = nullptr;
  void* scratch = nullptr;
  size_t scratch_bytes = 0;
  {
    Carve cv;
    cv.add(&w, (size_t)X.nseg + 1);
    cv.add(&part, scan_parts(X.nseg + 1));
    cv.add(&wide, 1);
    MSKM_TRY(cv.alloc(h->ctx, &scratch));
    scratch_bytes = cv.bytes;
  }
  CtxScratch free_scratch{h->ctx, scratch, scratch_bytes};
  int32_t* base = nullptr;
  {
    void* q = nullptr;
    MSKM_TRY(ctx_alloc(h->ctx, (size_t)X.nseg * 4, &q));
    base = static_cast<int32_t*>(q);
  }
  struct FreeBase {  // back to the cache unless the copy is built (then the hierarchy owns it)
    mskm_ctx* c;
    int32_t** p;
    size_t bytes;
    ~FreeBase() {
      if (*p) ctx_release(c, *p, bytes);
    }
  } free_base{h->ctx, &base, (size_t)X.nseg * 4};
  MSKM_HIP_TRY(hipMemsetAsync(wide, 0, 4, s));
  MSKM_HIP_TRY(hipMemsetAsync(w + X.nseg, 0, 8, s));
  for (int l = 0; l < L; ++l) {
    const int64_t ns = S.h_slice_begin[l + 1] - S.h_slice_begin[l];
    if (ns == 0 || h->h_depth[l] == 0) continue;
    hipLaunchKernelGGL(k_lsell_count, dim3((unsigned)ns), dim3(kSellC), 0, s, S.h_slice_begin[l], ns, seg0[l],
                       h->h_depth[l], S.rows, h->lower.rowptr, h->lower.col, cnt_lv, h->N, w, base, wide);
  }
  int32_t hwide = 0;
  MSKM_HIP_TRY(hipMemcpyAsync(&hwide, wide, 4, hipMemcpyDeviceToHost, s));
  MSKM_HIP_TRY(hipStreamSynchronize(s));
  if (hwide > 0) return MSKM_OK;  // some segment too wide for 16-bit offsets: products stay on the CSR
  MSKM_TRY(halloc(h, &X.seg_ptr, (size_t)X.nseg + 1));
  MSKM_TRY(exclusive_scan_i64(s, w, X.seg_ptr, X.nseg + 1, part));
  MSKM_HIP_TRY(hipMemcpyAsync(&X.entries, X.seg_ptr + X.nseg, 8, hipMemcpyDeviceToHost, s));
  MSKM_HIP_TRY(hipStreamSynchronize(s));
  MSKM_TRY(halloc(h, &X.col16, (size_t)X.entries));
  if (want64) MSKM_TRY(halloc(h, &X.val, (size_t)X.entries));
  if (want32) MSKM_TRY(halloc(h, &X.val32, (size_t)X.entries));
  if (h->lower.val32lo) MSKM_TRY(halloc(h, &X.lo, (size_t)X.entries));
  for (int l = 0; l < L; ++l) {
    const int64_t ns = S.h_slice_begin[l + 1] - S.h_slice_begin[l];
    if (ns == 0 || h->h_depth[l] == 0) continue;
    hipLaunchKernelGGL(k_lsell_fill, dim3((unsigned)ns), dim3(kLsWaves * kSellC), 0, s, S.h_slice_begin[l], ns, seg0[l],
                       h->h_depth[l], S.rows, h->lower.rowptr, h->lower.col, h->lower.val, h->lower.val32,
                       h->lower.val32lo, cnt_lv, h->N, X.seg_ptr, base, X.col16, X.val, X.val32, X.lo);
  }
  h->allocs.push_back(base);
  h->alloc_bytes.push_back((size_t)X.nseg * 4);
  h->device_bytes += X.nseg * 4;
  X.seg_base = base;
  base = nullptr;
  // the first segment of every slice (host table, then device)
  std::vector<int64_t> ss((size_t)S.nslices + 1, 0);
  for (int l = 0; l < L; ++l)
    for (int64_t sl = S.h_slice_begin[l]; sl < S.h_slice_begin[l + 1]; ++sl)
      ss[sl] = seg0[l] + (sl - S.h_slice_begin[l]) * h->h_depth[l];
  ss[S.nslices] = X.nseg;
  MSKM_TRY(halloc(h, &X.slice_seg, ss.size()));
  MSKM_TRY(upload_async(h, X.slice_seg, ss.data(), ss.size() * 8));
  X.built = true;
  MSKM_HIP_TRY(hipGetLastError());
  return MSKM_OK;
}

}  // namespace mskm
