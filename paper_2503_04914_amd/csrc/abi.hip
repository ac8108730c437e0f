// C ABI entry points: argument validation, context and handle lifetime,
// thread-local error text. The numerical work lives in assemble.hip and
// solve.hip.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "mskm_internal.h"

namespace {
thread_local std::string g_last_error;
std::atomic<uint64_t> g_serial{0};

bool valid_ctx(const mskm_ctx* c) { return c != nullptr; }

// B_{k,j} exists for levels k, j of one hierarchy with depth(j) <= depth(k)
bool valid_block(const mskm_hier* h, int k, int j) {
  return k >= 0 && k < h->L && j >= 0 && j < h->L && h->h_group[k] == h->h_group[j] && h->h_depth[j] <= h->h_depth[k];
}
}  // namespace

namespace mskm {
void set_error(const std::string& msg) { g_last_error = msg; }
mskm_status fail(mskm_status st, const std::string& msg) {
  g_last_error = msg;
  return st;
}
}  // namespace mskm

using mskm::fail;

namespace mskm {

constexpr size_t kBlockCacheCap = (size_t)32 << 30;

mskm_status ctx_alloc(mskm_ctx* c, size_t bytes, void** out) {
  *out = nullptr;
  if (c) {
    std::lock_guard<std::mutex> lock(c->cache_mu);
    auto it = c->cache.find(bytes);
    if (it != c->cache.end()) {
      *out = it->second;
      c->cache_bytes -= bytes;
      c->cache.erase(it);
      return MSKM_OK;
    }
  }
  hipError_t e = hipMalloc(out, bytes);
  if (e != hipSuccess && c && c->cache_bytes > 0) {  // give the cached blocks back and try once more
    (void)hipGetLastError();
    ctx_trim(c);
    e = hipMalloc(out, bytes);
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();
    *out = nullptr;
    return fail(MSKM_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
  }
  return MSKM_OK;
}

void ctx_release(mskm_ctx* c, void* p, size_t bytes) {
  if (!p) return;
  if (c) {
    std::lock_guard<std::mutex> lock(c->cache_mu);
    if (c->cache_bytes + bytes <= kBlockCacheCap) {
      c->cache.emplace(bytes, p);
      c->cache_bytes += bytes;
      return;
    }
  }
  (void)hipFree(p);
}

void ctx_trim(mskm_ctx* c) {
  if (!c) return;
  std::lock_guard<std::mutex> lock(c->cache_mu);
  for (auto& kv : c->cache) (void)hipFree(kv.second);
  c->cache.clear();
  c->cache_bytes = 0;
  for (auto& kv : c->host_cache) (void)hipHostFree(kv.second);
  c->host_cache.clear();
}

mskm_status ctx_host_alloc(mskm_ctx* c, size_t bytes, void** out) {
  *out = nullptr;
  if (c) {
    std::lock_guard<std::mutex> lock(c->cache_mu);
    auto it = c->host_cache.find(bytes);
    if (it != c->host_cache.end()) {
      *out = it->second;
      c->host_cache.erase(it);
      return MSKM_OK;
    }
  }
  if (hipHostMalloc(out, bytes, hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    *out = nullptr;
    return fail(MSKM_ENOMEM, "pinned allocation of " + std::to_string(bytes) + " bytes failed");
  }
  return MSKM_OK;
}

mskm_status upload_async(mskm_hier* h, void* dst, const void* src, size_t bytes) {
  if (bytes == 0) return MSKM_OK;
  constexpr size_t kStageChunk = size_t(1) << 20;  // one cached size for the tables of most hierarchies
  const size_t need = (bytes + 255) / 256 * 256;
  if (h->stage_blocks.empty() || h->stage_used + need > h->stage_bytes.back()) {
    const size_t cap = (need + kStageChunk - 1) / kStageChunk * kStageChunk;
    void* p = nullptr;
    MSKM_TRY(ctx_host_alloc(h->ctx, cap, &p));
    h->stage_blocks.push_back(p);
    h->stage_bytes.push_back(cap);
    h->stage_used = 0;
  }
  char* p = static_cast<char*>(h->stage_blocks.back()) + h->stage_used;
  h->stage_used += need;
  std::memcpy(p, src, bytes);
  MSKM_HIP_TRY(hipMemcpyAsync(dst, p, bytes, hipMemcpyHostToDevice, h->ctx->stream));
  return MSKM_OK;
}

void ctx_host_release(mskm_ctx* c, void* p, size_t bytes) {
  if (!p) return;
  if (c) {
    std::lock_guard<std::mutex> lock(c->cache_mu);
    if (c->host_cache.size() < 64) {
      c->host_cache.emplace(bytes, p);
      return;
    }
  }
  (void)hipHostFree(p);
}

}  // namespace mskm

extern "C" {

const char* mskm_last_error(void) { return g_last_error.c_str(); }

int32_t mskm_abi_version(void) { return MSKM_ABI_VERSION; }

mskm_status mskm_create(int32_t device, void* hip_stream, mskm_ctx** out) {
  if (!out) return fail(MSKM_EINVAL, "mskm_create: out is NULL");
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return fail(MSKM_EDEVICE, "no HIP device");
  if (device < 0 || device >= ndev) return fail(MSKM_EINVAL, "device index out of range");
  if (hipSetDevice(device) != hipSuccess) return fail(MSKM_EDEVICE, "hipSetDevice failed");
  // device address of the allocation-free residual's static scratch array
  MSKM_TRY(mskm::noalloc_init(device));
  auto* c = new (std::nothrow) mskm_ctx();
  if (!c) return fail(MSKM_ENOMEM, "context allocation");
  c->device = device;
  if (hip_stream) {
    c->stream = static_cast<hipStream_t>(hip_stream);
  } else {
    if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
      delete c;
      return fail(MSKM_EDEVICE, "hipStreamCreate failed");
    }
    c->own_stream = true;
  }
  if (hipEventCreate(&c->ev0) != hipSuccess || hipEventCreate(&c->ev1) != hipSuccess ||
      hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking) != hipSuccess) {
    if (c->ev0) (void)hipEventDestroy(c->ev0);
    if (c->ev1) (void)hipEventDestroy(c->ev1);
    mskm::ctx_trim(c);
  if (c->own_stream) (void)hipStreamDestroy(c->stream);
    delete c;
    return fail(MSKM_EDEVICE, "hipEventCreate / hipStreamCreate failed");
  }
  *out = c;
  return MSKM_OK;
}

mskm_status mskm_destroy(mskm_ctx* c) {
  if (!c) return MSKM_OK;
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  for (auto& b : c->batch_cache) {
    b.merged->ctx = nullptr;  // the cache is being torn down: no lookup in it
    mskm_hier_destroy(b.merged);
  }
  c->batch_cache.clear();
  (void)hipEventDestroy(c->ev0);
  (void)hipEventDestroy(c->ev1);
  if (c->side) {
    (void)hipStreamSynchronize(c->side);
    (void)hipStreamDestroy(c->side);
  }
  mskm::ctx_trim(c);  // the cached device and pinned blocks of destroyed hierarchies
  if (c->own_stream) (void)hipStreamDestroy(c->stream);
  delete c;
  return MSKM_OK;
}

namespace {

// Validation of one descriptor; returns its point count in *n.
mskm_status check_desc(const mskm_hier_desc* d, int64_t* n) {
  if (d->dim != 2 && d->dim != 3) return fail(MSKM_EINVAL, "dim must be 2 or 3");
  if (d->levels < 1 || d->levels > mskm::kMaxLevels) return fail(MSKM_EINVAL, "levels out of range");
  if (d->kernel != MSKM_WENDLAND_3_1) return fail(MSKM_EINVAL, "unsupported kernel");
  if (!d->level_offsets || !d->points || !d->delta) return fail(MSKM_EINVAL, "NULL array in descriptor");
  if (d->level_offsets[0] != 0) return fail(MSKM_EINVAL, "level_offsets[0] must be 0");
  int64_t largest = 0;
  for (int l = 0; l < d->levels; ++l) {
    if (d->level_offsets[l + 1] < d->level_offsets[l]) return fail(MSKM_EINVAL, "level_offsets must not decrease");
    if (!(d->delta[l] > 0.0) || !std::isfinite(d->delta[l])) return fail(MSKM_EINVAL, "delta must be finite and > 0");
    largest = std::max(largest, d->level_offsets[l + 1] - d->level_offsets[l]);
  }
  *n = d->level_offsets[d->levels];
  // points passed: all levels concatenated, or only the largest level of a prefix-nested hierarchy
  const int64_t np = (d->flags & MSKM_PREFIX_NESTED) ? largest : *n;
  if (!(d->flags & MSKM_POINTS_ON_DEVICE)) {
    for (int64_t i = 0; i < np * d->dim; ++i)
      if (!std::isfinite(d->points[i])) return fail(MSKM_EINVAL, "non-finite point coordinate");
  }
  return MSKM_OK;
}

// One hierarchy object from `count` independent hierarchies (groups). Levels
// are ordered depth-major; inputs (points, and later f / alpha) are the
// groups' arrays concatenated in descriptor order.
mskm_status create_groups(mskm_ctx* ctx, const mskm_hier_desc* ds, int32_t count, mskm_hier** out) {
  if (!valid_ctx(ctx) || !ds || !out || count < 1) return fail(MSKM_EINVAL, "hierarchy create: NULL argument");
  *out = nullptr;
  std::vector<int64_t> gn(count);
  int64_t N = 0;
  int Ltot = 0, Dmax = 0;
  for (int g = 0; g < count; ++g) {
    MSKM_TRY(check_desc(&ds[g], &gn[g]));
    if (ds[g].dim != ds[0].dim) return fail(MSKM_EINVAL, "all hierarchies of a batch need the same dim");
    const int32_t store = MSKM_STORE_FP64 | MSKM_STORE_FP32 | MSKM_SLICED_LOWER;
    if ((ds[g].flags & store) != (ds[0].flags & store))
      return fail(MSKM_EINVAL, "all hierarchies of a batch need the same storage flags");
    N += gn[g];
    Ltot += ds[g].levels;
    Dmax = std::max(Dmax, (int)ds[g].levels);
    if (Ltot > mskm::kMaxLevels) return fail(MSKM_ELIMIT, "more than 4096 levels in one hierarchy object");
  }
  if (N <= 0) return fail(MSKM_EINVAL, "hierarchy has no points");
  if (N >= (int64_t)INT32_MAX) return fail(MSKM_ELIMIT, "more than 2^31-1 points");
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(MSKM_EDEVICE, "hipSetDevice failed");
  bool want64 = (ds[0].flags & MSKM_STORE_FP64) != 0, want32 = (ds[0].flags & MSKM_STORE_FP32) != 0;
  if (!want64 && !want32) want64 = true;

  auto* h = new (std::nothrow) mskm_hier();
  if (!h) return fail(MSKM_ENOMEM, "hierarchy allocation");
  h->ctx = ctx;
  h->serial = ++g_serial;
  h->dim = ds[0].dim;
  h->L = Ltot;
  h->N = N;
  h->ngroups = count;
  h->h_group_in_off.assign(count + 1, 0);
  for (int g = 0; g < count; ++g) {
    h->h_group_in_off[g + 1] = h->h_group_in_off[g] + gn[g];
    h->h_group_levels.push_back(ds[g].levels);
  }
  // depth-major level order
  std::vector<std::vector<int32_t>> idx(count, std::vector<int32_t>(Dmax, -1));
  h->h_off.assign(1, 0);
  for (int d = 0; d < Dmax; ++d) {
    h->h_depth_begin.push_back((int32_t)h->h_delta.size());
    for (int g = 0; g < count; ++g) {
      if (d >= ds[g].levels) continue;
      idx[g][d] = (int32_t)h->h_delta.size();
      const int64_t n = ds[g].level_offsets[d + 1] - ds[g].level_offsets[d];
      h->h_off.push_back(h->h_off.back() + n);
      h->h_in_off.push_back(h->h_group_in_off[g] + ds[g].level_offsets[d]);
      h->h_delta.push_back(ds[g].delta[d]);
      h->h_group.push_back(g);
      h->h_depth.push_back(d);
    }
  }
  h->h_depth_begin.push_back(Ltot);
  h->h_first.assign(Ltot, 0);
  h->h_next.assign(Ltot, -1);
  for (int l = 0; l < Ltot; ++l) {
    const int g = h->h_group[l], d = h->h_depth[l];
    h->h_first[l] = idx[g][0];
    h->h_next[l] = d + 1 < ds[g].levels ? idx[g][d + 1] : -1;
  }
  // the input-order points, read by the assembly kernels only (the block
  // goes back to the context's cache behind them, stream-ordered)
  double* pts = nullptr;
  const size_t pts_bytes = (size_t)N * h->dim * sizeof(double);
  void* pv = nullptr;
  mskm_status st = mskm::ctx_alloc(ctx, pts_bytes, &pv);
  pts = static_cast<double*>(pv);
  for (int g = 0; g < count && st == MSKM_OK; ++g) {
    const bool dev = (ds[g].flags & MSKM_POINTS_ON_DEVICE) != 0;
    const hipMemcpyKind kind = dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    double* dst = pts + h->h_group_in_off[g] * h->dim;
    if (ds[g].flags & MSKM_PREFIX_NESTED) {  // level l = the first n_l points of the largest level
      for (int l = 0; l < ds[g].levels && st == MSKM_OK; ++l) {
        const int64_t nl = ds[g].level_offsets[l + 1] - ds[g].level_offsets[l];
        if (nl > 0 && hipMemcpyAsync(dst + ds[g].level_offsets[l] * h->dim, ds[g].points, (size_t)nl * h->dim * 8, kind,
                                     ctx->stream) != hipSuccess)
          st = fail(MSKM_EDEVICE, "point upload failed");
      }
    } else if (gn[g] > 0 &&
               hipMemcpyAsync(dst, ds[g].points, (size_t)gn[g] * h->dim * 8, kind, ctx->stream) != hipSuccess) {
      st = fail(MSKM_EDEVICE, "point upload failed");
    }
  }
  if (st == MSKM_OK) st = mskm::assemble_hierarchy(h, pts, want64, want32, (ds[0].flags & MSKM_SLICED_LOWER) != 0);
  if (st == MSKM_OK) {  // widths tuned earlier on this context for the same shape
    for (const auto& t : ctx->tune_cache)
      if (t.dim == h->dim && t.L == h->L && t.N == h->N && t.nnz_diag == h->diag.nnz && t.nnz_lower == h->lower.nnz)
        std::memcpy(h->spmv_g, t.g, sizeof(t.g));
  }
  // SpMV phase: 64 rows per block (one to four passes depending on the
  // lanes per row); streaming phase: 1024 rows per block (4 per thread)
  if (st == MSKM_OK) st = mskm::build_work_table(h, &h->wt_spmv, 64, 1 << 30);
  if (st == MSKM_OK) st = mskm::build_work_table(h, &h->wt_vec, 4 * mskm::kBlock, 1 << 30);
  mskm::ctx_release(ctx, pts, pts_bytes);
  if (st != MSKM_OK) {
    mskm_hier_destroy(h);
    return st;
  }
  *out = h;
  return MSKM_OK;
}

}  // namespace

mskm_status mskm_hier_create(mskm_ctx* ctx, const mskm_hier_desc* d, mskm_hier** out) {
  if (!d) return fail(MSKM_EINVAL, "mskm_hier_create: NULL descriptor");
  return create_groups(ctx, d, 1, out);
}

mskm_status mskm_hier_create_batch(mskm_ctx* ctx, const mskm_hier_desc* descs, int32_t count, mskm_hier** out) {
  return create_groups(ctx, descs, count, out);
}

mskm_status mskm_hier_destroy(mskm_hier* h) {
  if (!h) return MSKM_OK;
  if (h->ctx) {  // internal batch objects built from this hierarchy go with it
    auto& bc = h->ctx->batch_cache;
    for (size_t i = 0; i < bc.size();) {
      if (std::find(bc[i].members.begin(), bc[i].members.end(), h) != bc[i].members.end()) {
        mskm_hier* m = bc[i].merged;
        bc.erase(bc.begin() + (long)i);
        mskm_hier_destroy(m);
      } else {
        ++i;
      }
    }
  }
  if (h->ctx) {
    (void)hipSetDevice(h->ctx->device);
    (void)hipStreamSynchronize(h->ctx->stream);
  }
  for (hipEvent_t e : {h->bj.ev_tables, h->bj.ev_side, h->ev_asm[0], h->ev_asm[1]})
    if (e) {
      (void)hipEventSynchronize(e);
      (void)hipEventDestroy(e);
    }
  if (h->solve_ws_free) h->solve_ws_free(h->solve_ws);
  for (mskm_trunc* t : h->truncs) t->h = nullptr;  // they keep their own memory until destroyed
  for (size_t i = 0; i < h->allocs.size(); ++i) mskm::ctx_release(h->ctx, h->allocs[i], h->alloc_bytes[i]);
  for (size_t i = 0; i < h->stage_blocks.size(); ++i)
    mskm::ctx_host_release(h->ctx, h->stage_blocks[i], h->stage_bytes[i]);
  delete h;
  return MSKM_OK;
}

mskm_status mskm_hier_stats_get(const mskm_hier* h, mskm_hier_stats* o) {
  if (!h || !o) return fail(MSKM_EINVAL, "mskm_hier_stats_get: NULL argument");
  std::memset(o, 0, sizeof(*o));
  o->dim = h->dim;
  o->levels = h->L;
  o->n_total = h->N;
  o->nnz_diag = h->diag.nnz;
  o->nnz_lower = h->lower.nnz;
  o->has_fp64 = h->diag.val != nullptr;
  o->has_fp32 = h->diag.val32 != nullptr;
  o->device_bytes = h->device_bytes;
  if (h->asm_pending) {  // the assembly's last kernels may still have been running at creation's return
    float ms = 0.f;
    if (hipEventSynchronize(h->ev_asm[1]) != hipSuccess ||
        hipEventElapsedTime(&ms, h->ev_asm[0], h->ev_asm[1]) != hipSuccess)
      return fail(MSKM_EDEVICE, "assembly timing events");
    h->assemble_ms = ms;
    h->asm_pending = false;
  }
  o->assemble_ms = h->assemble_ms;
  o->ngroups = h->ngroups;
  o->sell_col16 = h->sell.col16 ? 1 : 0;
  o->sell_entries = h->sell.entries;
  o->lower_sliced = h->lsell.built ? 1 : 0;
  o->lower_sliced_entries = h->lsell.entries;
  return MSKM_OK;
}

mskm_status mskm_hier_level_info(const mskm_hier* h, int32_t level, mskm_level_info* info) {
  if (!h || !info) return fail(MSKM_EINVAL, "mskm_hier_level_info: NULL argument");
  if (level < 0 || level >= h->L) return fail(MSKM_EINVAL, "level out of range");
  info->group = h->h_group[level];
  info->depth = h->h_depth[level];
  info->n = h->h_off[level + 1] - h->h_off[level];
  info->input_offset = h->h_in_off[level];
  info->delta = h->h_delta[level];
  return MSKM_OK;
}

mskm_status mskm_hier_offsets(const mskm_hier* h, int64_t* off) {
  if (!h || !off) return fail(MSKM_EINVAL, "mskm_hier_offsets: NULL argument");
  for (int l = 0; l <= h->L; ++l) off[l] = h->h_off[l];
  return MSKM_OK;
}

mskm_status mskm_export_block(mskm_ctx* ctx, const mskm_hier* h, int32_t row_level, int32_t col_level, int64_t* rowptr,
                              int32_t* col, double* val, int64_t* nnz_out) {
  if (!valid_ctx(ctx) || !h) return fail(MSKM_EINVAL, "mskm_export_block: NULL handle");
  if (!valid_block(h, row_level, col_level))
    return fail(MSKM_EINVAL, "no such block: need levels of one hierarchy with depth(col) <= depth(row)");
  if (col && !rowptr) return fail(MSKM_EINVAL, "rowptr required with col");
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(MSKM_EDEVICE, "hipSetDevice failed");
  return mskm::export_block(const_cast<mskm_hier*>(h), row_level, col_level, rowptr, col, val, nnz_out);
}

mskm_status mskm_export_rows(mskm_ctx* ctx, const mskm_hier* h, int32_t row_level, int32_t col_level,
                             const int64_t* rows, int64_t nrows, int64_t* rowptr, int32_t* col, double* val,
                             int64_t* nnz_out) {
  if (!valid_ctx(ctx) || !h || !rows || nrows < 0) return fail(MSKM_EINVAL, "mskm_export_rows: NULL argument");
  if (!valid_block(h, row_level, col_level))
    return fail(MSKM_EINVAL, "no such block: need levels of one hierarchy with depth(col) <= depth(row)");
  if (col && !rowptr) return fail(MSKM_EINVAL, "rowptr required with col");
  const int64_t n = h->h_off[row_level + 1] - h->h_off[row_level];
  for (int64_t i = 0; i < nrows; ++i)
    if (rows[i] < 0 || rows[i] >= n) return fail(MSKM_EINVAL, "row index outside the row level");
  if (nrows == 0) {
    if (rowptr) rowptr[0] = 0;
    if (nnz_out) *nnz_out = 0;
    return MSKM_OK;
  }
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(MSKM_EDEVICE, "hipSetDevice failed");
  return mskm::export_block(const_cast<mskm_hier*>(h), row_level, col_level, rowptr, col, val, nnz_out, rows, nrows);
}

mskm_status mskm_export_perm(mskm_ctx* ctx, const mskm_hier* h, int32_t* perm) {
  if (!valid_ctx(ctx) || !h || !perm) return fail(MSKM_EINVAL, "mskm_export_perm: NULL argument");
  if (hipMemcpy(perm, h->perm, h->N * 4, hipMemcpyDeviceToHost) != hipSuccess)
    return fail(MSKM_EDEVICE, "perm copy failed");
  return MSKM_OK;
}

mskm_status mskm_apply(mskm_ctx* ctx, const mskm_hier* h, int32_t op, int32_t prec, const double* x, int32_t nrhs,
                       double* y, int32_t flags) {
  if (!valid_ctx(ctx) || !h || !x || !y) return fail(MSKM_EINVAL, "mskm_apply: NULL argument");
  if (op < MSKM_OP_DIAG || op > MSKM_OP_FULL) return fail(MSKM_EINVAL, "unknown op");
  if (prec != MSKM_PREC_FP64 && prec != MSKM_PREC_FP32) return fail(MSKM_EINVAL, "unknown precision");
  if (nrhs < 1) return fail(MSKM_EINVAL, "nrhs must be >= 1");
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(MSKM_EDEVICE, "hipSetDevice failed");
  return mskm::apply_op(const_cast<mskm_hier*>(h), op, prec, x, nrhs, y, (flags & MSKM_IO_DEVICE) != 0);
}

mskm_status mskm_apply_internal(mskm_ctx* ctx, const mskm_hier* h, int32_t op, int32_t prec, const void* x, void* y,
                                int32_t repeats, float* avg_ms) {
  if (!valid_ctx(ctx) || !h || !x || !y) return fail(MSKM_EINVAL, "mskm_apply_internal: NULL argument");
  if (x == y) return fail(MSKM_EINVAL, "mskm_apply_internal: y aliases x");
  if (op < MSKM_OP_DIAG || op > MSKM_OP_FULL) return fail(MSKM_EINVAL, "unknown op");
  if (prec != MSKM_PREC_FP64 && prec != MSKM_PREC_FP32) return fail(MSKM_EINVAL, "unknown precision");
  if (repeats < 1) return fail(MSKM_EINVAL, "repeats must be >= 1");
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(MSKM_EDEVICE, "hipSetDevice failed");
  return mskm::apply_internal(const_cast<mskm_hier*>(h), op, prec, x, y, repeats, avg_ms);
}

mskm_status mskm_autotune(mskm_ctx* ctx, mskm_hier* h, int32_t repeats, float* times_ms) {
  if (!valid_ctx(ctx) || !h) return fail(MSKM_EINVAL, "mskm_autotune: NULL argument");
  if (repeats < 1) return fail(MSKM_EINVAL, "repeats must be >= 1");
  if (times_ms) std::memset(times_ms, 0, sizeof(float) * 3 * 2 * mskm::kTuneVariants);
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(MSKM_EDEVICE, "hipSetDevice failed");
  return mskm::autotune(h, repeats, times_ms);
}

mskm_status mskm_spmv_width(const mskm_hier* h, int32_t op, int32_t prec, int32_t* width) {
  if (!h || !width) return fail(MSKM_EINVAL, "mskm_spmv_width: NULL argument");
  if (op < MSKM_OP_DIAG || op > MSKM_OP_FULL || (prec != MSKM_PREC_FP64 && prec != MSKM_PREC_FP32))
    return fail(MSKM_EINVAL, "unknown op or precision");
  *width = h->spmv_g[op][prec];
  return MSKM_OK;
}

mskm_status mskm_set_spmv_width(mskm_hier* h, int32_t op, int32_t prec, int32_t width) {
  if (!h) return fail(MSKM_EINVAL, "mskm_set_spmv_width: NULL hierarchy");
  if (op < MSKM_OP_DIAG || op > MSKM_OP_FULL || (prec != MSKM_PREC_FP64 && prec != MSKM_PREC_FP32))
    return fail(MSKM_EINVAL, "unknown op or precision");
  const int g = width % mskm::kVecFlag, kind = width / mskm::kVecFlag;
  if (width == mskm::kSellCode || width == mskm::kSell32Code) {
    // lower and full operators: the sliced copies, when the lower one was built
    const bool lower_ok = width == mskm::kSellCode && h->lsell.built &&
                          (prec == MSKM_PREC_FP64 ? h->lsell.val != nullptr : h->lsell.val32 != nullptr);
    if (op != MSKM_OP_DIAG && !lower_ok)
      return fail(MSKM_EINVAL, "mskm_set_spmv_width: the SELL variants serve MSKM_OP_DIAG, and 4064 the lower and "
                               "full operators of a hierarchy created with MSKM_SLICED_LOWER");
  } else if (width < 0 || kind > 3 || (g != 4 && g != 8 && g != 16 && g != 32 && g != 64)) {
    return fail(MSKM_EINVAL, "mskm_set_spmv_width: unknown variant code " + std::to_string(width));
  }
  h->spmv_g[op][prec] = width;
  return MSKM_OK;
}

void mskm_solve_opts_default(mskm_solve_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->precision = MSKM_PREC_FP64;
  o->algorithm = MSKM_ALG_MONOLITHIC;
  o->cg_rtol = 1e-12;
  o->sweeps = 0;
  o->max_cg_iters = 20000;
  o->warm_start = 0;
  o->target_rel_residual = 1e-8;
  o->max_refine = 10;
  o->precond = MSKM_PRECOND_NONE;
  o->mlp = nullptr;
  o->check_every = 8;
  o->flags = 0;
}

namespace {
// Option checks shared by mskm_solve and mskm_solve_batch.
mskm_status check_opts(const mskm_solve_opts& o, const mskm_hier* h, int nrhs) {
  if (o.precision != MSKM_PREC_FP64 && o.precision != MSKM_PREC_FP32) return fail(MSKM_EINVAL, "unknown precision");
  if (o.algorithm != MSKM_ALG_MONOLITHIC && o.algorithm != MSKM_ALG_SEQUENTIAL)
    return fail(MSKM_EINVAL, "unknown algorithm");
  if (!(o.cg_rtol > 0.0) || !(o.cg_rtol < 1.0)) return fail(MSKM_EINVAL, "cg_rtol must be in (0, 1)");
  if (o.precision == MSKM_PREC_FP32 && !(o.target_rel_residual > 0.0))
    return fail(MSKM_EINVAL, "target_rel_residual must be > 0 on the mixed path");
  if (o.precond != MSKM_PRECOND_NONE && o.precond != MSKM_PRECOND_LEARNED && o.precond != MSKM_PRECOND_BLOCK_JACOBI &&
      o.precond != MSKM_PRECOND_FLEX_LEARNED)
    return fail(MSKM_EINVAL, "unknown precond");
  if (o.precond == MSKM_PRECOND_FLEX_LEARNED) {
    if (!o.mlp) return fail(MSKM_EINVAL, "the flexible learned preconditioner needs an mlp");
    if (o.mlp->dim != h->dim) return fail(MSKM_EINVAL, "network and hierarchy dimensions differ");
    if (o.algorithm != MSKM_ALG_SEQUENTIAL)
      return fail(MSKM_EINVAL, "the flexible learned preconditioner runs with the sequential algorithm");
    if (nrhs > 1) return fail(MSKM_EINVAL, "the flexible learned preconditioner takes one right-hand side");
    if (o.warm_start != MSKM_START_ZERO) return fail(MSKM_EINVAL, "the flexible learned preconditioner starts from zero");
  }
  if (o.warm_start != MSKM_START_ZERO && o.warm_start != MSKM_START_PREVIOUS && o.warm_start != MSKM_START_LEARNED)
    return fail(MSKM_EINVAL, "unknown warm_start");
  const bool learned = o.precond == MSKM_PRECOND_LEARNED || o.warm_start == MSKM_START_LEARNED;
  if (learned && !o.mlp) return fail(MSKM_EINVAL, "learned warm start needs an mlp");
  if (learned && o.mlp->dim != h->dim) return fail(MSKM_EINVAL, "network and hierarchy dimensions differ");
  if (nrhs > 1 && learned) return fail(MSKM_EINVAL, "solves of several right-hand sides take no learned warm start");
  return MSKM_OK;
}
}  // namespace

mskm_status mskm_solve(mskm_ctx* ctx, const mskm_hier* h, const double* f, int32_t nrhs, const mskm_solve_opts* opts,
                       double* alpha, mskm_report* rep) {
  if (!valid_ctx(ctx) || !h || !f || !alpha) return fail(MSKM_EINVAL, "mskm_solve: NULL argument");
  if (nrhs < 1) return fail(MSKM_EINVAL, "nrhs must be >= 1");
  mskm_solve_opts o;
  if (opts) o = *opts;
  else mskm_solve_opts_default(&o);
  MSKM_TRY(check_opts(o, h, nrhs));
  if (!(o.flags & MSKM_IO_DEVICE)) {
    for (int64_t i = 0; i < h->N * (int64_t)nrhs; ++i)
      if (!std::isfinite(f[i])) return fail(MSKM_EINVAL, "non-finite right-hand side");
  }
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(MSKM_EDEVICE, "hipSetDevice failed");
  return mskm::solve(const_cast<mskm_hier*>(h), f, nrhs, &o, alpha, rep);
}

namespace {
// The context's batch object for exactly these hierarchies (in this order),
// assembled from their points at the first request.
mskm_status merged_batch(mskm_ctx* ctx, const mskm_hier* const* hs, int nh, mskm_hier** out) {
  for (const auto& b : ctx->batch_cache) {
    if ((int)b.members.size() != nh) continue;
    bool same = true;
    for (int g = 0; g < nh && same; ++g) same = b.members[g] == hs[g] && b.serials[g] == hs[g]->serial;
    if (same) {
      *out = b.merged;
      return MSKM_OK;
    }
  }
  // points back in each hierarchy's input order, then one batch assembly
  int64_t total = 0;
  for (int g = 0; g < nh; ++g) total += hs[g]->N;
  double* pts = nullptr;
  MSKM_TRY(mskm::dalloc(&pts, (size_t)total * hs[0]->dim));
  struct FreePts {
    double* p;
    ~FreePts() { (void)hipFree(p); }
  } free_pts{pts};
  std::vector<mskm_hier_desc> ds(nh);
  int64_t o = 0;
  for (int g = 0; g < nh; ++g) {
    mskm_hier* hg = const_cast<mskm_hier*>(hs[g]);
    MSKM_TRY(mskm::export_points_device(hg, pts + o * hg->dim));
    ds[g].dim = hg->dim;
    ds[g].levels = hg->L;
    ds[g].level_offsets = hg->h_off.data();
    ds[g].points = pts + o * hg->dim;
    ds[g].delta = hg->h_delta.data();
    ds[g].kernel = MSKM_WENDLAND_3_1;
    ds[g].flags = MSKM_POINTS_ON_DEVICE | (hg->diag.val ? MSKM_STORE_FP64 : 0) | (hg->diag.val32 ? MSKM_STORE_FP32 : 0);
    o += hg->N;
  }
  mskm_hier* m = nullptr;
  MSKM_TRY(create_groups(ctx, ds.data(), nh, &m));
  std::memcpy(m->spmv_g, hs[0]->spmv_g, sizeof(m->spmv_g));  // the members' SpMV choices
  mskm::MergedBatch b;
  b.members.assign(hs, hs + nh);
  for (int g = 0; g < nh; ++g) b.serials.push_back(hs[g]->serial);
  b.merged = m;
  ctx->batch_cache.push_back(b);
  *out = m;
  return MSKM_OK;
}
}  // namespace

mskm_status mskm_solve_batch(mskm_ctx* ctx, const mskm_hier* const* h, int32_t nh, const double* const* f,
                             const int32_t* nrhs, const mskm_solve_opts* opts, double* const* alpha,
                             mskm_report* reps) {
  if (!valid_ctx(ctx) || !h || !f || !nrhs || !alpha || nh < 1)
    return fail(MSKM_EINVAL, "mskm_solve_batch: NULL argument");
  mskm_solve_opts o;
  if (opts) o = *opts;
  else mskm_solve_opts_default(&o);
  int R = 0;
  for (int g = 0; g < nh; ++g) {
    if (!h[g] || !f[g] || !alpha[g]) return fail(MSKM_EINVAL, "mskm_solve_batch: NULL hierarchy or vector");
    if (h[g]->ngroups != 1) return fail(MSKM_EINVAL, "mskm_solve_batch: a batch object cannot be a member");
    if (h[g]->ctx != ctx) return fail(MSKM_EINVAL, "mskm_solve_batch: hierarchy of another context");
    if (h[g]->dim != h[0]->dim || (h[g]->diag.val != nullptr) != (h[0]->diag.val != nullptr) ||
        (h[g]->diag.val32 != nullptr) != (h[0]->diag.val32 != nullptr))
      return fail(MSKM_EINVAL, "mskm_solve_batch: hierarchies need the same dim and stored precisions");
    for (int k = 0; k < g; ++k)
      if (h[k] == h[g]) return fail(MSKM_EINVAL, "mskm_solve_batch: a hierarchy appears twice");
    if (nrhs[g] < 1 || nrhs[g] > 512) return fail(MSKM_EINVAL, "mskm_solve_batch: nrhs must be in [1, 512]");
    R = std::max(R, (int)nrhs[g]);
  }
  MSKM_TRY(check_opts(o, h[0], R));
  const bool io_dev = (o.flags & MSKM_IO_DEVICE) != 0;
  if (!io_dev) {
    for (int g = 0; g < nh; ++g)
      for (int64_t i = 0; i < h[g]->N * (int64_t)nrhs[g]; ++i)
        if (!std::isfinite(f[g][i])) return fail(MSKM_EINVAL, "non-finite right-hand side");
  }
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(MSKM_EDEVICE, "hipSetDevice failed");
  mskm_hier* m = nullptr;
  MSKM_TRY(merged_batch(ctx, h, nh, &m));
  // concatenated [N][R] right-hand sides (zero columns past a hierarchy's own nrhs)
  hipStream_t s = ctx->stream;
  const int64_t N = m->N;
  double *F = nullptr, *A = nullptr;
  MSKM_TRY(mskm::dalloc(&F, (size_t)N * R));
  MSKM_TRY(mskm::dalloc(&A, (size_t)N * R));
  struct FreeFA {
    double *a, *b;
    ~FreeFA() {
      (void)hipFree(a);
      (void)hipFree(b);
    }
  } free_fa{F, A};
  const hipMemcpyKind in_kind = io_dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  const hipMemcpyKind out_kind = io_dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  MSKM_HIP_TRY(hipMemsetAsync(F, 0, (size_t)N * R * 8, s));
  for (int g = 0; g < nh; ++g)
    if (h[g]->N > 0)
      MSKM_HIP_TRY(hipMemcpy2DAsync(F + m->h_group_in_off[g] * R, (size_t)R * 8, f[g], (size_t)nrhs[g] * 8,
                                    (size_t)nrhs[g] * 8, (size_t)h[g]->N, in_kind, s));
  o.flags |= MSKM_IO_DEVICE;
  mskm_report all;
  const mskm_status st = mskm::solve(m, F, R, &o, A, &all);
  MSKM_TRY(st);
  for (int g = 0; g < nh; ++g)
    if (h[g]->N > 0)
      MSKM_HIP_TRY(hipMemcpy2DAsync(alpha[g], (size_t)nrhs[g] * 8, A + m->h_group_in_off[g] * R, (size_t)R * 8,
                                    (size_t)nrhs[g] * 8, (size_t)h[g]->N, out_kind, s));
  std::vector<double> rel((size_t)R * nh, 0.0);
  MSKM_TRY(mskm::residual(m, A, F, R, rel.data(), true));
  bool missed = false;
  for (int g = 0; g < nh; ++g) {
    double worst = 0.0;
    for (int r = 0; r < nrhs[g]; ++r) worst = std::max(worst, rel[(size_t)r * nh + g]);
    if (o.precision == MSKM_PREC_FP32 && worst > o.target_rel_residual) missed = true;
    if (!reps) continue;
    mskm_report& rp = reps[g];
    std::memset(&rp, 0, sizeof(rp));
    rp.levels = h[g]->L;
    rp.sweeps_done = all.sweeps_done;
    rp.refine_steps = all.refine_steps;
    rp.cg_iters_total = all.cg_iters_total;
    for (int l = 0; l < m->L && l < 64; ++l)
      if (m->h_group[l] == g && m->h_depth[l] < 64) rp.cg_iters_last[m->h_depth[l]] = all.cg_iters_last[l];
    rp.rel_residual = worst;
    rp.solve_ms = all.solve_ms;
    rp.warm_fallbacks = all.warm_fallbacks;
  }
  MSKM_HIP_TRY(hipStreamSynchronize(s));
  return (st == MSKM_ENOCONV || missed) ? MSKM_ENOCONV : MSKM_OK;
}

mskm_status mskm_residual(mskm_ctx* ctx, const mskm_hier* h, const double* alpha, const double* f, int32_t nrhs,
                          double* rel_out, int32_t flags) {
  if (!valid_ctx(ctx) || !h || !alpha || !f || !rel_out) return fail(MSKM_EINVAL, "mskm_residual: NULL argument");
  if (nrhs < 1) return fail(MSKM_EINVAL, "nrhs must be >= 1");
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(MSKM_EDEVICE, "hipSetDevice failed");
  return mskm::residual(const_cast<mskm_hier*>(h), alpha, f, nrhs, rel_out, (flags & MSKM_IO_DEVICE) != 0);
}

mskm_status mskm_cg_product_time(mskm_ctx* ctx, mskm_hier* h, int32_t level, int32_t prec, int32_t repeats,
                                 float* avg_ms) {
  if (!valid_ctx(ctx) || !h || !avg_ms) return fail(MSKM_EINVAL, "mskm_cg_product_time: NULL argument");
  if (level < 0 || level >= h->L) return fail(MSKM_EINVAL, "level out of range");
  if (prec != MSKM_PREC_FP64 && prec != MSKM_PREC_FP32) return fail(MSKM_EINVAL, "unknown precision");
  if (repeats < 1) return fail(MSKM_EINVAL, "repeats must be >= 1");
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(MSKM_EDEVICE, "hipSetDevice failed");
  return mskm::time_cg_product(h, level, prec, repeats, avg_ms);
}

mskm_status mskm_mr_product_time(mskm_ctx* ctx, mskm_hier* h, int32_t level, int32_t prec, int32_t nrhs,
                                 int32_t repeats, float* avg_ms) {
  if (!valid_ctx(ctx) || !h || !avg_ms) return fail(MSKM_EINVAL, "mskm_mr_product_time: NULL argument");
  if (level < 0 || level >= h->L) return fail(MSKM_EINVAL, "level out of range");
  if (prec != MSKM_PREC_FP64 && prec != MSKM_PREC_FP32) return fail(MSKM_EINVAL, "unknown precision");
  if (repeats < 1) return fail(MSKM_EINVAL, "repeats must be >= 1");
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(MSKM_EDEVICE, "hipSetDevice failed");
  return mskm::time_mr_product(h, level, prec, nrhs, repeats, avg_ms);
}

mskm_status mskm_set_mr_chunk(mskm_hier* h, int32_t nrhs, int32_t prec, int32_t chunk) {
  if (!h) return fail(MSKM_EINVAL, "mskm_set_mr_chunk: NULL hierarchy");
  if (prec != MSKM_PREC_FP64 && prec != MSKM_PREC_FP32) return fail(MSKM_EINVAL, "unknown precision");
  if (hipSetDevice(h->ctx->device) != hipSuccess) return fail(MSKM_EDEVICE, "hipSetDevice failed");
  return mskm::set_mr_chunk(h, nrhs, prec, chunk);
}

// ------------------------------------------------------- thresholded Jacobi

mskm_status mskm_trunc_create(mskm_ctx* ctx, mskm_hier* h, double T, double cg_rtol, mskm_trunc** out) {
  if (!valid_ctx(ctx) || !h || !out) return fail(MSKM_EINVAL, "mskm_trunc_create: NULL argument");
  *out = nullptr;
  if (!(T > 0.0) || std::isnan(T)) return fail(MSKM_EINVAL, "T must be > 0 (INFINITY keeps every entry)");
  if (!(cg_rtol > 0.0 && cg_rtol < 1.0)) return fail(MSKM_EINVAL, "cg_rtol must lie in (0, 1)");
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(MSKM_EDEVICE, "hipSetDevice failed");
  auto* t = new (std::nothrow) mskm_trunc();
  if (!t) return fail(MSKM_ENOMEM, "truncated-block object allocation");
  t->h = h;
  t->T = T;
  const mskm_status st = mskm::trunc_build(h, T, cg_rtol, t);
  if (st < 0) {
    delete t;
    return st;
  }
  h->truncs.push_back(t);
  *out = t;
  return t->capped ? MSKM_ENOCONV : MSKM_OK;
}

mskm_status mskm_trunc_destroy(mskm_trunc* t) {
  if (!t) return MSKM_OK;
  if (t->h) {
    auto& v = t->h->truncs;
    v.erase(std::remove(v.begin(), v.end(), t), v.end());
    if (t->h->ctx) {
      (void)hipSetDevice(t->h->ctx->device);
      (void)hipStreamSynchronize(t->h->ctx->stream);
    }
  }
  delete t;
  return MSKM_OK;
}

mskm_status mskm_trunc_info(const mskm_trunc* t, double* q, int64_t* nnz, int64_t* cg_iters, double* build_ms) {
  if (!t) return fail(MSKM_EINVAL, "mskm_trunc_info: NULL handle");
  if (q) std::copy(t->q.begin(), t->q.end(), q);
  if (nnz) *nnz = t->X.nnz;
  if (cg_iters) *cg_iters = t->cg_iters;
  if (build_ms) *build_ms = t->build_ms;
  return MSKM_OK;
}

mskm_status mskm_trunc_export_block(mskm_ctx* ctx, const mskm_trunc* t, int32_t row_level, int32_t col_level,
                                    int64_t* rowptr, int32_t* col, double* val, int64_t* nnz_out) {
  if (!valid_ctx(ctx) || !t) return fail(MSKM_EINVAL, "mskm_trunc_export_block: NULL handle");
  if (!t->h) return fail(MSKM_ESTATE, "the hierarchy of these blocks was destroyed");
  if (!valid_block(t->h, row_level, col_level) || row_level == col_level)
    return fail(MSKM_EINVAL, "no such block: need levels of one hierarchy with depth(col) < depth(row)");
  if (col && !rowptr) return fail(MSKM_EINVAL, "rowptr required with col");
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(MSKM_EDEVICE, "hipSetDevice failed");
  return mskm::export_block(t->h, row_level, col_level, rowptr, col, val, nnz_out, nullptr, 0, &t->X);
}

mskm_status mskm_trunc_solve(mskm_ctx* ctx, const mskm_trunc* t, const double* f, const mskm_solve_opts* opts,
                             double* alpha, mskm_report* rep) {
  if (!valid_ctx(ctx) || !t || !f || !opts || !alpha) return fail(MSKM_EINVAL, "mskm_trunc_solve: NULL argument");
  if (!t->h) return fail(MSKM_ESTATE, "the hierarchy of these blocks was destroyed");
  if (!(opts->cg_rtol > 0.0)) return fail(MSKM_EINVAL, "cg_rtol must be > 0");
  if (opts->precond != MSKM_PRECOND_NONE && opts->precond != MSKM_PRECOND_BLOCK_JACOBI)
    return fail(MSKM_EINVAL, "the thresholded solve takes no learned start");
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(MSKM_EDEVICE, "hipSetDevice failed");
  return mskm::trunc_solve(t->h, t->X, f, opts, alpha, rep);
}

namespace {
// True when p is device memory of `device` (hipMalloc'd or managed).
bool on_device(const void* p, int device) {
  hipPointerAttribute_t a{};
  if (hipPointerGetAttributes(&a, p) != hipSuccess) {
    (void)hipGetLastError();  // host memory the runtime does not know: clear the error
    return false;
  }
  return (a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged) && a.device == device;
}
}  // namespace

mskm_status mskm_residual_noalloc(mskm_ctx* ctx, const mskm_hier* h, const double* alpha, const double* f,
                                  int32_t nrhs, double* rel_out) {
  if (!valid_ctx(ctx) || !h || !alpha || !f || !rel_out)
    return fail(MSKM_EINVAL, "mskm_residual_noalloc: NULL argument");
  if (nrhs < 1) return fail(MSKM_EINVAL, "nrhs must be >= 1");
  if (!h->ctx || h->ctx->device != ctx->device)
    return fail(MSKM_EINVAL, "mskm_residual_noalloc: hierarchy lives on another device");
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(MSKM_EDEVICE, "hipSetDevice failed");
  if (!on_device(alpha, ctx->device) || !on_device(f, ctx->device) || !on_device(rel_out, ctx->device))
    return fail(MSKM_EINVAL, "mskm_residual_noalloc: alpha, f and rel_out must be device memory of the context's device");
  return mskm::residual_noalloc(const_cast<mskm_hier*>(h), alpha, f, nrhs, rel_out);
}

mskm_status mskm_evaluate(mskm_ctx* ctx, const mskm_hier* h, const double* alpha, int32_t nrhs, const double* query,
                          int64_t nq, double* out, int32_t flags) {
  if (!valid_ctx(ctx) || !h || !alpha || (nq > 0 && (!query || !out)))
    return fail(MSKM_EINVAL, "mskm_evaluate: NULL argument");
  if (nrhs < 1 || nq < 0) return fail(MSKM_EINVAL, "nrhs must be >= 1 and nq >= 0");
  if (nq == 0) return MSKM_OK;
  if (h->ngroups != 1) return fail(MSKM_EINVAL, "mskm_evaluate takes a single hierarchy, not a batch");
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(MSKM_EDEVICE, "hipSetDevice failed");
  return mskm::evaluate(const_cast<mskm_hier*>(h), alpha, nrhs, query, nq, out, (flags & MSKM_IO_DEVICE) != 0);
}

mskm_status mskm_mlp_train(mskm_ctx* ctx, const mskm_train_desc* d, mskm_mlp** out, float* loss_log) {
  if (!valid_ctx(ctx) || !d || !out || !d->h || !d->f) return fail(MSKM_EINVAL, "mskm_mlp_train: NULL argument");
  *out = nullptr;
  if (d->nrhs < 1 || d->samples < 1 || d->steps < 1 || !(d->lr > 0.0f) || !(d->cg_rtol > 0.0 && d->cg_rtol < 1.0))
    return fail(MSKM_EINVAL, "mskm_mlp_train: nrhs, samples, steps, lr and cg_rtol must be positive");
  mskm_hier* h = const_cast<mskm_hier*>(d->h);
  if (!h->diag.val) return fail(MSKM_ESTATE, "training pairs need FP64 values (MSKM_STORE_FP64)");
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(MSKM_EDEVICE, "hipSetDevice failed");
  mskm_mlp* m = nullptr;
  MSKM_TRY(mskm::mlp_new(h->dim, d->seed, &m));
  std::vector<double*> rhs, alpha;
  mskm_status st = mskm::train_pairs(h, d->f, d->nrhs, (d->flags & MSKM_IO_DEVICE) != 0, d->cg_rtol, &rhs, &alpha);
  std::vector<float> log;
  if (st == MSKM_OK) st = mskm::mlp_train_device(h, m, rhs, alpha, d->samples, d->steps, d->lr, d->seed, &log);
  for (double* p : rhs) (void)hipFree(p);
  for (double* p : alpha) (void)hipFree(p);
  if (st != MSKM_OK) {
    delete m;
    return st;
  }
  if (loss_log) std::memcpy(loss_log, log.data(), log.size() * sizeof(float));
  *out = m;
  return MSKM_OK;
}

mskm_status mskm_mlp_fit(mskm_ctx* ctx, mskm_mlp* m, const float* X, const float* y, int64_t ns, int32_t steps,
                         float lr, int32_t flags, float* loss_log) {
  if (!valid_ctx(ctx) || !m || !X || !y) return fail(MSKM_EINVAL, "mskm_mlp_fit: NULL argument");
  if (ns < 1 || steps < 1 || !(lr > 0.0f) || !std::isfinite(lr))
    return fail(MSKM_EINVAL, "mskm_mlp_fit: ns, steps and lr must be positive");
  if (!(flags & MSKM_IO_DEVICE)) {
    for (int64_t i = 0; i < ns * (int64_t)m->F; ++i)
      if (!std::isfinite(X[i])) return fail(MSKM_EINVAL, "mskm_mlp_fit: non-finite feature");
    for (int64_t i = 0; i < ns; ++i)
      if (!std::isfinite(y[i])) return fail(MSKM_EINVAL, "mskm_mlp_fit: non-finite target");
  }
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(MSKM_EDEVICE, "hipSetDevice failed");
  return mskm::mlp_fit(ctx, m, X, y, ns, steps, lr, (flags & MSKM_IO_DEVICE) != 0, loss_log);
}

mskm_status mskm_mlp_destroy(mskm_mlp* m) {
  delete m;
  return MSKM_OK;
}

mskm_status mskm_mlp_save(const mskm_mlp* m, void* blob, size_t* size) {
  if (!m || !size) return fail(MSKM_EINVAL, "mskm_mlp_save: NULL argument");
  const size_t need = 8 + 3 * 4 + m->params.size() * 4;
  if (!blob) {
    *size = need;
    return MSKM_OK;
  }
  if (*size < need) return fail(MSKM_EINVAL, "mskm_mlp_save: blob too small");
  char* p = static_cast<char*>(blob);
  std::memcpy(p, "MSKMMLP1", 8);
  const int32_t hdr[3] = {m->dim, m->F, 64};
  std::memcpy(p + 8, hdr, 12);
  std::memcpy(p + 20, m->params.data(), m->params.size() * 4);
  *size = need;
  return MSKM_OK;
}

mskm_status mskm_mlp_load(mskm_ctx* ctx, const void* blob, size_t size, mskm_mlp** out) {
  if (!valid_ctx(ctx) || !blob || !out) return fail(MSKM_EINVAL, "mskm_mlp_load: NULL argument");
  *out = nullptr;
  const char* p = static_cast<const char*>(blob);
  if (size < 20 || std::memcmp(p, "MSKMMLP1", 8) != 0) return fail(MSKM_EINVAL, "not an MSKMMLP1 blob");
  int32_t hdr[3];
  std::memcpy(hdr, p + 8, 12);
  if ((hdr[0] != 2 && hdr[0] != 3) || hdr[2] != 64 || hdr[1] != ((1 + 16 * (1 + hdr[0])) + 7) / 8 * 8)
    return fail(MSKM_EINVAL, "unsupported network shape");
  const size_t P = (size_t)64 * hdr[1] + 2 * 64 + 1;
  if (size < 20 + P * 4) return fail(MSKM_EINVAL, "truncated blob");
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(MSKM_EDEVICE, "hipSetDevice failed");
  mskm_mlp* m = nullptr;
  MSKM_TRY(mskm::mlp_new(hdr[0], 0, &m));
  std::memcpy(m->params.data(), p + 20, P * 4);
  for (float v : m->params)
    if (!std::isfinite(v)) {
      delete m;
      return fail(MSKM_EINVAL, "non-finite weight");
    }
  mskm_status st = mskm::mlp_upload(m);
  if (st != MSKM_OK) {
    delete m;
    return st;
  }
  *out = m;
  return MSKM_OK;
}

mskm_status mskm_mlp_predict(mskm_ctx* ctx, const mskm_hier* hc, const mskm_mlp* m, const double* b, double* x0,
                             int32_t flags) {
  if (!valid_ctx(ctx) || !hc || !m || !b || !x0) return fail(MSKM_EINVAL, "mskm_mlp_predict: NULL argument");
  mskm_hier* h = const_cast<mskm_hier*>(hc);
  if (m->dim != h->dim) return fail(MSKM_EINVAL, "network and hierarchy dimensions differ");
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(MSKM_EDEVICE, "hipSetDevice failed");
  return mskm::mlp_predict_all(h, m, b, x0, (flags & MSKM_IO_DEVICE) != 0);
}

mskm_status mskm_knn_export(mskm_ctx* ctx, const mskm_hier* hc, int32_t level, int32_t* out) {
  if (!valid_ctx(ctx) || !hc || !out) return fail(MSKM_EINVAL, "mskm_knn_export: NULL argument");
  if (level < 0 || level >= hc->L) return fail(MSKM_EINVAL, "level out of range");
  mskm_hier* h = const_cast<mskm_hier*>(hc);
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(MSKM_EDEVICE, "hipSetDevice failed");
  return mskm::knn_export(h, level, out);
}

}  // extern "C"
