// Learned warm start for the per-level CG solves (a build extension; the
// paper's CG starts from zero). For point i of level l the network sees its
// 16 nearest same-level points n_1..n_16 (exact kNN on squared FP64
// distances, ties by input index, self excluded, padded with i when the
// level is smaller than 17) and predicts
//     x0_i = s * (w2 . relu(W1 feat + b1) + b2),
//     s = sqrt(mean of b^2 over the stencil {i, n_1..n_16}),
//     feat = [b_i/s, (b_{n_m}/s, (x_{n_m} - x_i)/delta_l) for m = 1..16].
// Inference: the first layer on MFMA (v_mfma_f32_32x32x8_bf16: 32 points x 32
// hidden units x 8 features per instruction, BF16 operands, FP32
// accumulation), 32 points per wave. Training: one deterministic block (FP32
// Adam on the mean squared error, the first layer with the same BF16-rounded
// weights and features as inference) on (rhs stencil -> correction / s)
// samples drawn from the solver's own sequential solves, or on samples the
// caller gives. CG checks the result: a level whose warm start does
// not reduce ||b - A x0|| below ||b|| restarts from zero.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "device_common.h"

namespace mskm {

constexpr int kKnn = 16;
constexpr int kHidden = 64;
constexpr int kMaxF = 72;  // 1 + 16 (1 + 3), padded to a multiple of 8

static int feature_count(int dim) { return ((1 + kKnn * (1 + dim)) + 7) / 8 * 8; }

// ------------------------------------------------------------------ kNN-16

// One thread per point: scan the (2w+1)^d cells around the point, keep the 16
// smallest (d2, input index) in a sorted register list; widen w until the
// 16th distance is below the scanned radius (w cells from any point of the
// centre cell), so the result is the exact kNN. At most w = 4, then the whole
// level is scanned.
__global__ void __launch_bounds__(kBlock) k_knn16(int dim, int l, const DevLevel* __restrict__ lev,
                                                  const int32_t* __restrict__ cs_all, const double* __restrict__ xs,
                                                  int64_t N, const int32_t* __restrict__ perm,
                                                  int32_t* __restrict__ knn) {
  const DevLevel L = lev[l];
  const int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (r >= L.n) return;
  const int64_t i = L.off + r;
  const double px = xs[i], py = xs[N + i], pz = dim == 3 ? xs[2 * N + i] : 0.0;
  const int cx = cell_coord(px, L.lo[0], L.inv_cell, L.nc[0]);
  const int cy = cell_coord(py, L.lo[1], L.inv_cell, L.nc[1]);
  const int cz = dim == 3 ? cell_coord(pz, L.lo[2], L.inv_cell, L.nc[2]) : 0;
  const double cell = 1.0 / L.inv_cell;
  double bd[kKnn];
  int32_t bi[kKnn], bk[kKnn];
  int found = 0;
  for (int w = 1;; ++w) {
    const bool all = w > 4;
    found = 0;
    const int x0 = all ? 0 : max(cx - w, 0), x1 = all ? L.nc[0] - 1 : min(cx + w, L.nc[0] - 1);
    const int y0 = all ? 0 : max(cy - w, 0), y1 = all ? L.nc[1] - 1 : min(cy + w, L.nc[1] - 1);
    const int z0 = dim == 3 ? (all ? 0 : max(cz - w, 0)) : 0;
    const int z1 = dim == 3 ? (all ? L.nc[2] - 1 : min(cz + w, L.nc[2] - 1)) : 0;
    const int32_t* cs = cs_all + L.cs_off;
    for (int z = z0; z <= z1; ++z)
      for (int y = y0; y <= y1; ++y) {
        const int rk = (z * L.nc[1] + y) * L.nc[0];
        for (int64_t t = cs[rk + x0]; t < cs[rk + x1 + 1]; ++t) {
          if (t == i) continue;
          const double d2 = sqdist(dim, px, py, pz, xs[t], xs[N + t], dim == 3 ? xs[2 * N + t] : 0.0);
          const int32_t key = perm[t];
          if (found == kKnn && !(d2 < bd[kKnn - 1] || (d2 == bd[kKnn - 1] && key < bk[kKnn - 1]))) continue;
          int p = found < kKnn ? found++ : kKnn - 1;
          while (p > 0 && (d2 < bd[p - 1] || (d2 == bd[p - 1] && key < bk[p - 1]))) {
            bd[p] = bd[p - 1];
            bi[p] = bi[p - 1];
            bk[p] = bk[p - 1];
            --p;
          }
          bd[p] = d2;
          bi[p] = (int32_t)t;
          bk[p] = key;
        }
      }
    if (all) break;
    // exact if the 16th neighbour is closer than any unscanned point can be
    const double reach = w * cell * (1.0 - 1e-9);
    if (found == kKnn && bd[kKnn - 1] < reach * reach) break;
    if (found < kKnn && (int64_t)found == (int64_t)L.n - 1) break;  // the level has no more points
  }
  for (int m = 0; m < kKnn; ++m) knn[i * kKnn + m] = m < found ? bi[m] : (int32_t)i;
}

// ---------------------------------------------------------------- features

// Features of point i from rhs b (internal order) into f[0..F), returns s.
// Evaluated in FP64 in the definition's order with every operation rounded
// separately (no contraction), so the FP32 features agree bit for bit with a
// host evaluation of the same expressions.
template <typename TX>
__device__ __forceinline__ double point_features(int dim, int F, int64_t i, double delta,
                                                 const int32_t* __restrict__ knn, const double* __restrict__ xs,
                                                 int64_t N, const TX* __restrict__ b, float* f) {
#pragma clang fp contract(off)
  const double bi = (double)b[i];
  double ss = bi * bi;
  for (int m = 0; m < kKnn; ++m) {
    const double bn = (double)b[knn[i * kKnn + m]];
    ss += bn * bn;
  }
  const double s = sqrt(ss / (double)(kKnn + 1));
  for (int k = 0; k < F; ++k) f[k] = 0.0f;
  if (!(s > 0.0)) return 0.0;
  f[0] = (float)(bi / s);
  for (int m = 0; m < kKnn; ++m) {
    const int64_t j = knn[i * kKnn + m];
    const int base = 1 + m * (1 + dim);
    f[base] = (float)((double)b[j] / s);
    for (int a = 0; a < dim; ++a) f[base + 1 + a] = (float)((xs[a * N + j] - xs[a * N + i]) / delta);
  }
  return s;
}

// ------------------------------------------------------ inference (MFMA)

typedef short v4i16 __attribute__((ext_vector_type(4)));
typedef float v16f __attribute__((ext_vector_type(16)));

// float -> bfloat16 bits, round to nearest even (finite inputs)
__device__ __forceinline__ short to_bf16(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (short)(u >> 16);
}

constexpr int kInferWaves = 4;  // waves per block, 32 points per wave

// x0[i] = s_i * MLP(features_i) for rows [r0, r1) of one level.
// w1b: BF16 first layer [64][F]; b1, w2: FP32 [64]; b2: FP32.
template <typename TX>
__global__ void __launch_bounds__(kInferWaves * kWave)
    k_mlp_infer(int dim, int F, int64_t r0, int64_t r1, double delta, const int32_t* __restrict__ knn,
                const double* __restrict__ xs, int64_t N, const TX* __restrict__ b, const short* __restrict__ w1b,
                const float* __restrict__ b1, const float* __restrict__ w2, const float* __restrict__ b2p,
                TX* __restrict__ x0) {
  __shared__ float feat[kInferWaves][32][kMaxF + 1];
  __shared__ double sval[kInferWaves][32];
  const int wv = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const int64_t base = r0 + ((int64_t)blockIdx.x * kInferWaves + wv) * 32;
  // lanes 0..31 compute the features of their point (FP64 arithmetic, stored FP32)
  if (lane < 32) {
    const int64_t i = base + lane;
    float f[kMaxF];
    double s = 0.0;
    if (i < r1) s = point_features<TX>(dim, F, i, delta, knn, xs, N, b, f);
    else
      for (int k = 0; k < F; ++k) f[k] = 0.0f;
    for (int k = 0; k < F; ++k) feat[wv][lane][k] = f[k];
    sval[wv][lane] = s;
  }
  __syncthreads();
  const int p = lane % 32, half = lane / 32;
  float vsum[16];
#pragma unroll
  for (int e = 0; e < 16; ++e) vsum[e] = 0.0f;
  for (int tile = 0; tile < 2; ++tile) {
    const int n = tile * 32 + p;  // hidden unit of this lane's B column
    v16f acc = {};
    for (int ks = 0; ks < F / 8; ++ks) {
      const int k = ks * 8 + half * 4;
      v4i16 a, bb;
      a[0] = to_bf16(feat[wv][p][k]);
      a[1] = to_bf16(feat[wv][p][k + 1]);
      a[2] = to_bf16(feat[wv][p][k + 2]);
      a[3] = to_bf16(feat[wv][p][k + 3]);
      bb[0] = w1b[n * F + k];
      bb[1] = w1b[n * F + k + 1];
      bb[2] = w1b[n * F + k + 2];
      bb[3] = w1b[n * F + k + 3];
      acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, bb, acc, 0, 0, 0);
    }
    const float bn = b1[n], wn = w2[n];
#pragma unroll
    for (int e = 0; e < 16; ++e) vsum[e] += wn * fmaxf(acc[e] + bn, 0.0f);
  }
  // sum over the 32 hidden units held by the lanes of this half
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    float v = vsum[e];
    for (int o = 1; o < 32; o <<= 1) v += __shfl_xor(v, o, kWave);
    vsum[e] = v;
  }
  if (p == 0) {
    const float bias2 = b2p[0];
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int row = 8 * (e / 4) + 4 * half + (e % 4);  // point of accumulator element e
      const int64_t i = base + row;
      if (i < r1) x0[i] = (TX)(sval[wv][row] * (double)(vsum[e] + bias2));
    }
  }
}

// ------------------------------------------------------------- training

constexpr int kTrainB = 128;  // mini-batch = threads of the training block

// Sample k: point idx[k] (internal), features from rhs b, target alpha/s.
template <typename TX>
__global__ void __launch_bounds__(kBlock)
    k_mlp_samples(int dim, int F, int L, const DevLevel* __restrict__ lev, const int32_t* __restrict__ knn,
                  const double* __restrict__ xs, int64_t N, const TX* __restrict__ b, const TX* __restrict__ alpha,
                  const int64_t* __restrict__ idx, int64_t ns, float* __restrict__ X, float* __restrict__ y) {
  const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (k >= ns) return;
  const int64_t i = idx[k];
  int l = 0;
  while (l + 1 < L && i >= lev[l + 1].off) ++l;
  float f[kMaxF];
  const double s = point_features<TX>(dim, F, i, lev[l].delta, knn, xs, N, b, f);
  for (int j = 0; j < F; ++j) X[k * F + j] = f[j];
  y[k] = s > 0.0 ? (float)((double)alpha[i] / s) : 0.0f;
}

// float rounded to the nearest bfloat16 (ties to even) and widened back.
__device__ __forceinline__ float bf16_round(float x) { return __uint_as_float((uint32_t)(uint16_t)to_bf16(x) << 16); }

// Parameters in one FP32 array: W1 [64][F], b1 [64], w2 [64], b2 [1].
// One block of kTrainB threads runs `steps` Adam steps on mini-batches
// (sample (step*B + t) mod ns). The first layer computes with BF16-rounded
// weights and features, as inference on MFMA does; its gradient (taken at
// the rounded values) updates the FP32 weights. Every parameter is owned by
// one thread, every gradient is a fixed-order sum over the batch: the run is
// deterministic.
__global__ void __launch_bounds__(kTrainB)
    k_mlp_train(int F, const float* __restrict__ X, const float* __restrict__ y, int64_t ns, int steps, float lr,
                float* __restrict__ params, float* __restrict__ adam_m, float* __restrict__ adam_v,
                float* __restrict__ loss_log, int log_every) {
  extern __shared__ float smem[];
  const int P = kHidden * F + 2 * kHidden + 1;
  const int XS = F + 1;  // padded row stride
  float* W = smem;                      // [P]
  float* Xs = W + P;                    // [B][F+1]
  float* Hs = Xs + kTrainB * XS;        // [B][65]
  float* dH = Hs + kTrainB * (kHidden + 1);  // [B][65]
  float* dy = dH + kTrainB * (kHidden + 1);  // [B]
  float* red = dy + kTrainB;                 // [B]
  const int t = threadIdx.x;
  for (int p = t; p < P; p += kTrainB) W[p] = params[p];
  const float beta1 = 0.9f, beta2 = 0.999f, eps = 1e-8f;
  float b1t = 1.0f, b2t = 1.0f;
  __syncthreads();
  for (int step = 0; step < steps; ++step) {
    const int64_t k = ((int64_t)step * kTrainB + t) % ns;
    for (int j = 0; j < F; ++j) Xs[t * XS + j] = bf16_round(X[k * F + j]);
    const float target = y[k];
    __syncthreads();
    // forward
    const float* W1 = W;
    const float* b1 = W + kHidden * F;
    const float* w2 = b1 + kHidden;
    const float b2 = w2[kHidden];
    float out = b2;
    for (int h = 0; h < kHidden; ++h) {
      float a = b1[h];
      for (int j = 0; j < F; ++j) a += bf16_round(W1[h * F + j]) * Xs[t * XS + j];
      a = fmaxf(a, 0.0f);
      Hs[t * (kHidden + 1) + h] = a;
      out += w2[h] * a;
    }
    const float err = out - target;
    const float g = 2.0f * err / (float)kTrainB;
    dy[t] = g;
    red[t] = err * err;
    for (int h = 0; h < kHidden; ++h)
      dH[t * (kHidden + 1) + h] = Hs[t * (kHidden + 1) + h] > 0.0f ? g * w2[h] : 0.0f;
    __syncthreads();
    if (log_every > 0 && step % log_every == 0 && t == 0) {
      float s = 0.0f;
      for (int q = 0; q < kTrainB; ++q) s += red[q];
      loss_log[step / log_every] = s / (float)kTrainB;
    }
    // gradients + Adam, one owner thread per parameter
    b1t *= beta1;
    b2t *= beta2;
    for (int p = t; p < P; p += kTrainB) {
      float gr = 0.0f;
      if (p < kHidden * F) {
        const int h = p / F, j = p % F;
        for (int q = 0; q < kTrainB; ++q) gr += dH[q * (kHidden + 1) + h] * Xs[q * XS + j];
      } else if (p < kHidden * F + kHidden) {
        const int h = p - kHidden * F;
        for (int q = 0; q < kTrainB; ++q) gr += dH[q * (kHidden + 1) + h];
      } else if (p < kHidden * F + 2 * kHidden) {
        const int h = p - kHidden * F - kHidden;
        for (int q = 0; q < kTrainB; ++q) gr += dy[q] * Hs[q * (kHidden + 1) + h];
      } else {
        for (int q = 0; q < kTrainB; ++q) gr += dy[q];
      }
      const float m = beta1 * adam_m[p] + (1.0f - beta1) * gr;
      const float v = beta2 * adam_v[p] + (1.0f - beta2) * gr * gr;
      adam_m[p] = m;
      adam_v[p] = v;
      const float mh = m / (1.0f - b1t), vh = v / (1.0f - b2t);
      W[p] -= lr * mh / (sqrtf(vh) + eps);
    }
    __syncthreads();
  }
  for (int p = t; p < P; p += kTrainB) params[p] = W[p];
}

__global__ void __launch_bounds__(kBlock) k_to_bf16(const float* __restrict__ in, short* __restrict__ out, int n) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i < n) out[i] = to_bf16(in[i]);
}

// Sample positions: idx[k] = SplitMix64(seed, k) mod N (counter based).
__global__ void __launch_bounds__(kBlock) k_sample_points(uint64_t seed, int64_t base, int64_t ns, int64_t N,
                                                          int64_t* __restrict__ idx) {
  const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (k >= ns) return;
  uint64_t z = seed + (uint64_t)(base + k + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  idx[base + k] = (int64_t)(z % (uint64_t)N);
}

// ------------------------------------------------------------------- host

mskm_status ensure_knn(mskm_hier* h) {
  if (h->knn) return MSKM_OK;
  MSKM_TRY(halloc(h, &h->knn, (size_t)h->N * kKnn));
  hipStream_t s = h->ctx->stream;
  for (int l = 0; l < h->L; ++l) {
    const int64_t n = h->h_off[l + 1] - h->h_off[l];
    if (n == 0) continue;
    hipLaunchKernelGGL(k_knn16, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, h->dim, l, h->d_lev,
                       h->cell_start, h->xs, h->N, h->perm, h->knn);
  }
  MSKM_HIP_TRY(hipGetLastError());
  return MSKM_OK;
}

mskm_status mlp_upload(mskm_mlp* m) {
  const int P = kHidden * m->F + 2 * kHidden + 1;
  if (!m->d_params) {
    MSKM_TRY(dalloc(&m->d_params, P));
    MSKM_TRY(dalloc(&m->d_w1b, (size_t)kHidden * m->F));
  }
  MSKM_HIP_TRY(hipMemcpy(m->d_params, m->params.data(), P * 4, hipMemcpyHostToDevice));
  hipLaunchKernelGGL(k_to_bf16, dim3((kHidden * m->F + kBlock - 1) / kBlock), dim3(kBlock), 0, 0, m->d_params, m->d_w1b,
                     kHidden * m->F);
  MSKM_HIP_TRY(hipDeviceSynchronize());
  return MSKM_OK;
}

// x0 = MLP warm start for rows [r0, r1) of level l (internal order vectors).
template <typename TX>
mskm_status mlp_predict_rows(mskm_hier* h, const mskm_mlp* m, int l, const TX* b, TX* x0) {
  MSKM_TRY(ensure_knn(h));
  const int64_t r0 = h->h_off[l], r1 = h->h_off[l + 1];
  if (r1 <= r0) return MSKM_OK;
  const int64_t pts_per_block = 32 * kInferWaves;
  const float* b1 = m->d_params + kHidden * m->F;
  hipLaunchKernelGGL(k_mlp_infer<TX>, dim3((unsigned)((r1 - r0 + pts_per_block - 1) / pts_per_block)),
                     dim3(kInferWaves * kWave), 0, h->ctx->stream, h->dim, m->F, r0, r1, h->h_delta[l], h->knn,
                     h->xs, h->N, b, m->d_w1b, b1, b1 + kHidden, b1 + 2 * kHidden, x0);
  MSKM_HIP_TRY(hipGetLastError());
  return MSKM_OK;
}

template mskm_status mlp_predict_rows<double>(mskm_hier*, const mskm_mlp*, int, const double*, double*);

__global__ void __launch_bounds__(kBlock) k_perm_gather(const double* __restrict__ in, const int32_t* __restrict__ perm,
                                                        double* __restrict__ out, int64_t n, int dir) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  if (dir == 0) out[i] = in[perm[i]];  // input -> internal
  else out[perm[i]] = in[i];           // internal -> input
}

mskm_status mlp_predict_all(mskm_hier* h, const mskm_mlp* m, const double* b, double* x0, bool io_dev) {
  hipStream_t s = h->ctx->stream;
  const int64_t N = h->N;
  double *bd = nullptr, *bi = nullptr, *xi = nullptr, *xd = nullptr;
  MSKM_TRY(dalloc(&bi, N));
  MSKM_TRY(dalloc(&xi, N));
  if (!io_dev) {
    MSKM_TRY(dalloc(&bd, N));
    MSKM_TRY(dalloc(&xd, N));
    MSKM_HIP_TRY(hipMemcpyAsync(bd, b, N * 8, hipMemcpyHostToDevice, s));
  }
  const unsigned g = (unsigned)((N + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_perm_gather, dim3(g), dim3(kBlock), 0, s, io_dev ? b : bd, h->perm, bi, N, 0);
  MSKM_HIP_TRY(hipMemsetAsync(xi, 0, N * 8, s));
  mskm_status st = MSKM_OK;
  for (int l = 0; l < h->L && st == MSKM_OK; ++l) st = mlp_predict_rows<double>(h, m, l, bi, xi);
  if (st == MSKM_OK) {
    hipLaunchKernelGGL(k_perm_gather, dim3(g), dim3(kBlock), 0, s, xi, h->perm, io_dev ? x0 : xd, N, 1);
    if (!io_dev && hipMemcpyAsync(x0, xd, N * 8, hipMemcpyDeviceToHost, s) != hipSuccess)
      st = fail(MSKM_EDEVICE, "copy");
    if (st == MSKM_OK && hipStreamSynchronize(s) != hipSuccess) st = fail(MSKM_EDEVICE, "sync");
  }
  for (double* p : {bd, bi, xi, xd}) (void)hipFree(p);
  return st;
}

__global__ void __launch_bounds__(kBlock) k_knn_canon(const int32_t* __restrict__ knn, const int32_t* __restrict__ iperm,
                                                      const int32_t* __restrict__ perm, int64_t in_off, int64_t n,
                                                      int32_t* __restrict__ out) {
  const int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (r >= n) return;
  const int64_t i = iperm[in_off + r];
  for (int m = 0; m < kKnn; ++m) out[r * kKnn + m] = (int32_t)(perm[knn[i * kKnn + m]] - in_off);
}

mskm_status knn_export(mskm_hier* h, int level, int32_t* out) {
  MSKM_TRY(ensure_knn(h));
  const int64_t n = h->h_off[level + 1] - h->h_off[level];
  if (n == 0) return MSKM_OK;
  int32_t* d = nullptr;
  MSKM_TRY(dalloc(&d, (size_t)n * kKnn));
  hipStream_t s = h->ctx->stream;
  hipLaunchKernelGGL(k_knn_canon, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, h->knn, h->iperm,
                     h->perm, h->h_in_off[level], n, d);
  hipError_t e = hipMemcpyAsync(out, d, (size_t)n * kKnn * 4, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(d);
  if (e != hipSuccess) return fail(MSKM_EDEVICE, std::string("knn export: ") + hipGetErrorString(e));
  return MSKM_OK;
}
template mskm_status mlp_predict_rows<float>(mskm_hier*, const mskm_mlp*, int, const float*, float*);

mskm_status mlp_new(int dim, uint64_t seed, mskm_mlp** out) {
  auto* m = new (std::nothrow) mskm_mlp();
  if (!m) return fail(MSKM_ENOMEM, "mlp allocation");
  m->dim = dim;
  m->F = feature_count(dim);
  const int P = kHidden * m->F + 2 * kHidden + 1;
  m->params.assign(P, 0.0f);
  // uniform(-a, a) initial weights, a = sqrt(6 / (fan_in + fan_out)), from SplitMix64
  uint64_t st = seed;
  auto next = [&]() {
    st += 0x9E3779B97F4A7C15ull;
    uint64_t z = st;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return (double)((z ^ (z >> 31)) >> 11) * (1.0 / 9007199254740992.0);
  };
  const double a1 = std::sqrt(6.0 / (m->F + kHidden)), a2 = std::sqrt(6.0 / (kHidden + 1));
  for (int p = 0; p < kHidden * m->F; ++p) m->params[p] = (float)((2.0 * next() - 1.0) * a1);
  for (int p = 0; p < kHidden; ++p) m->params[kHidden * m->F + kHidden + p] = (float)((2.0 * next() - 1.0) * a2);
  *out = m;
  return MSKM_OK;
}

// `steps` Adam steps of k_mlp_train on device samples (X [ns][F], y [ns])
// from the moments in am / av; the network's host and device parameters
// (and its BF16 copy of W1) are updated; the mini-batch loss of steps 0,
// log_every, ... goes to lg.
static mskm_status run_train(hipStream_t s, mskm_mlp* m, const float* X, const float* y, int64_t ns, int steps,
                             float lr, float* am, float* av, float* lg, int log_every) {
  const int F = m->F;
  const int P = kHidden * F + 2 * kHidden + 1;
  if (!m->d_params) MSKM_TRY(mlp_upload(m));
  const size_t lds = sizeof(float) * (P + kTrainB * (F + 1) + 2 * kTrainB * (kHidden + 1) + 2 * kTrainB);
  MSKM_HIP_TRY(hipFuncSetAttribute((const void*)k_mlp_train, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  hipLaunchKernelGGL(k_mlp_train, dim3(1), dim3(kTrainB), lds, s, F, X, y, ns, steps, lr, m->d_params, am, av, lg,
                     log_every);
  MSKM_HIP_TRY(hipGetLastError());
  MSKM_HIP_TRY(hipStreamSynchronize(s));
  MSKM_HIP_TRY(hipMemcpy(m->params.data(), m->d_params, P * 4, hipMemcpyDeviceToHost));
  return mlp_upload(m);
}

// Train on samples of (level rhs -> correction) pairs from plain FP64
// sequential solves of the given right-hand sides (internal order rhs in fi).
mskm_status mlp_train_device(mskm_hier* h, mskm_mlp* m, const std::vector<double*>& rhs_int,
                             const std::vector<double*>& alpha_int, int64_t samples, int steps, float lr, uint64_t seed,
                             std::vector<float>* loss_log) {
  hipStream_t s = h->ctx->stream;
  MSKM_TRY(ensure_knn(h));
  const int nr = (int)rhs_int.size();
  const int64_t per = std::max<int64_t>(1, samples / std::max(nr, 1));
  const int64_t ns = per * nr;
  const int F = m->F;
  int64_t* idx = nullptr;
  float *X = nullptr, *y = nullptr, *am = nullptr, *av = nullptr, *lg = nullptr;
  MSKM_TRY(dalloc(&idx, ns));
  MSKM_TRY(dalloc(&X, (size_t)ns * F));
  MSKM_TRY(dalloc(&y, ns));
  const int P = kHidden * F + 2 * kHidden + 1;
  MSKM_TRY(dalloc(&am, P));
  MSKM_TRY(dalloc(&av, P));
  const int log_every = 50;
  const int nlog = (steps + log_every - 1) / log_every;  // steps 0, 50, ..., < steps
  MSKM_TRY(dalloc(&lg, nlog));
  struct Free {
    void* v[6];
    ~Free() {
      for (void* p : v) (void)hipFree(p);
    }
  } fr{{idx, X, y, am, av, lg}};
  MSKM_HIP_TRY(hipMemsetAsync(am, 0, P * 4, s));
  MSKM_HIP_TRY(hipMemsetAsync(av, 0, P * 4, s));
  MSKM_HIP_TRY(hipMemsetAsync(lg, 0, nlog * 4, s));
  for (int r = 0; r < nr; ++r) {
    hipLaunchKernelGGL(k_sample_points, dim3((unsigned)((per + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, seed,
                       (int64_t)r * per, per, h->N, idx);
    hipLaunchKernelGGL(k_mlp_samples<double>, dim3((unsigned)((per + kBlock - 1) / kBlock)), dim3(kBlock), 0, s,
                       h->dim, F, h->L, h->d_lev, h->knn, h->xs, h->N, rhs_int[r], alpha_int[r], idx + (int64_t)r * per,
                       per, X + (int64_t)r * per * F, y + (int64_t)r * per);
  }
  MSKM_TRY(run_train(s, m, X, y, ns, steps, lr, am, av, lg, log_every));
  if (loss_log) {
    loss_log->resize(nlog);
    MSKM_HIP_TRY(hipMemcpy(loss_log->data(), lg, nlog * 4, hipMemcpyDeviceToHost));
  }
  m->samples = ns;
  return MSKM_OK;
}

// Adam on caller-given samples: X [ns][F], y [ns] (FP32, host or device).
mskm_status mlp_fit(mskm_ctx* ctx, mskm_mlp* m, const float* X, const float* y, int64_t ns, int steps, float lr,
                    bool io_dev, float* loss_log) {
  hipStream_t s = ctx->stream;
  const int F = m->F;
  const int P = kHidden * F + 2 * kHidden + 1;
  float *Xd = nullptr, *yd = nullptr, *am = nullptr, *av = nullptr, *lg = nullptr;
  if (!io_dev) {
    MSKM_TRY(dalloc(&Xd, (size_t)ns * F));
    MSKM_TRY(dalloc(&yd, ns));
  }
  MSKM_TRY(dalloc(&am, P));
  MSKM_TRY(dalloc(&av, P));
  MSKM_TRY(dalloc(&lg, steps));
  struct Free {
    void* v[5];
    ~Free() {
      for (void* p : v) (void)hipFree(p);
    }
  } fr{{Xd, yd, am, av, lg}};
  if (!io_dev) {
    MSKM_HIP_TRY(hipMemcpyAsync(Xd, X, (size_t)ns * F * 4, hipMemcpyHostToDevice, s));
    MSKM_HIP_TRY(hipMemcpyAsync(yd, y, (size_t)ns * 4, hipMemcpyHostToDevice, s));
  }
  MSKM_HIP_TRY(hipMemsetAsync(am, 0, P * 4, s));
  MSKM_HIP_TRY(hipMemsetAsync(av, 0, P * 4, s));
  MSKM_TRY(run_train(s, m, io_dev ? X : Xd, io_dev ? y : yd, ns, steps, lr, am, av, lg, 1));
  if (loss_log) MSKM_HIP_TRY(hipMemcpy(loss_log, lg, (size_t)steps * 4, hipMemcpyDeviceToHost));
  return MSKM_OK;
}

}  // namespace mskm
