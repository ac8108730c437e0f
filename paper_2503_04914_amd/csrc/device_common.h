// Device helpers shared by the gfx950 kernels: wave64 reductions, the exact
// pair test, the Wendland phi_{3,1} and cell-grid lookups.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "mskm_internal.h"

namespace mskm {

constexpr int kWave = 64;

// XCD-aware block id: the hardware hands block b to XCD (b % 8). Remapping
// gives every XCD one contiguous range of logical blocks, so neighbouring
// rows (which share most of their gathered x entries) stay in one L2.
__device__ __forceinline__ int xcd_block_id(int nblocks) {
  const int b = blockIdx.x;
  // blocks are dispatched round-robin over the 8 XCDs
  const int per = nblocks / 8;
  const int rem = nblocks % 8;
  const int xcd = b % 8;
  const int k = b / 8;
  // XCDs 0..rem-1 own per+1 blocks, the others per.
  const int base = xcd < rem ? xcd * (per + 1) : rem * (per + 1) + (xcd - rem) * per;
  return base + k;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

// Sum over a group of G consecutive lanes (G a power of two <= 64), result in
// every lane of the group. Fixed butterfly order: deterministic.
template <int G, typename T>
__device__ __forceinline__ T group_sum(T v) {
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, G);
  return v;
}

// Block-wide sum of one value per thread, deterministic for a fixed block size.
// Returns the total in thread 0 (others: unspecified). Needs kBlock/64 slots.
template <typename T>
__device__ __forceinline__ T block_sum(T v, T* smem) {
  v = wave_sum(v);
  const int w = threadIdx.x / kWave, l = threadIdx.x % kWave;
  if (l == 0) smem[w] = v;
  __syncthreads();
  T t = 0;
  if (threadIdx.x == 0) {
    for (int i = 0; i < (int)(blockDim.x / kWave); ++i) t += smem[i];
  }
  __syncthreads();
  return t;
}

// Squared distance evaluated as dx*dx + dy*dy (+ dz*dz), left to right, with
// every operation rounded separately: no contraction into fused multiply-add,
// so the host-side definition and this one agree bit for bit.
__device__ __forceinline__ double sqdist(int dim, double ax, double ay, double az, double bx, double by, double bz) {
#pragma clang fp contract(off)
  const double dx = ax - bx;
  const double dy = ay - by;
  double d2 = dx * dx;
  d2 = d2 + dy * dy;
  if (dim == 3) {
    const double dz = az - bz;
    d2 = d2 + dz * dz;
  }
  return d2;
}

// phi_{3,1}(r) = (1-r)_+^4 (4r+1) with r = sqrt(d2) / delta (FP64).
__device__ __forceinline__ double phi31_d2(double d2, double delta) {
  const double r = sqrt(d2) / delta;
  double t = 1.0 - r;
  t = t > 0.0 ? t : 0.0;
  const double t2 = t * t;
  return t2 * t2 * (4.0 * r + 1.0);
}

// FP32 variant (values applied in single precision): r from FP32 distance.
__device__ __forceinline__ float phi31_f(float r) {
  float t = 1.0f - r;
  t = t > 0.0f ? t : 0.0f;
  const float t2 = t * t;
  return t2 * t2 * (4.0f * r + 1.0f);
}

// Cell coordinate of x on one axis of a level grid, clamped into the grid.
// Clamping is monotone and 1-Lipschitz, so points closer than the cell side
// still land in equal or adjacent cells.
__device__ __forceinline__ int cell_coord(double x, double lo, double inv_cell, int nc) {
  double q = floor((x - lo) * inv_cell);
  q = q < 0.0 ? 0.0 : q;
  const double hi = (double)(nc - 1);
  q = q > hi ? hi : q;
  return (int)q;
}

// Row i of the block-Jacobi product u = M^-1 r: the row of its block's
// dense inverse times the block's entries of r, which the caller staged in
// rs (rs[k] = r[row0 + k] for the rows of its workgroup of whole blocks).
template <typename TX>
__device__ __forceinline__ TX bj_row(int64_t i, int64_t row0, const TX* rs, const int64_t* __restrict__ start,
                                     const int32_t* __restrict__ of_row, const int64_t* __restrict__ off,
                                     const TX* __restrict__ inv) {
  const int32_t b = of_row[i];
  const int64_t a = start[b];
  const int m = (int)(start[b + 1] - a);
  const TX* Mi = inv + off[b] + (i - a) * m;
  const TX* rb = rs + (a - row0);
  TX acc = 0;
  for (int j = 0; j < m; ++j) acc += Mi[j] * rb[j];
  return acc;
}

}  // namespace mskm
