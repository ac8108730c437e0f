// Internal declarations of the gfx950 multiscale kernel library.
//
// Device data layout (one hierarchy):
//   * internal order: every level's points are sorted by the row-major key of
//     their cell in that level's own cell grid (cell side >= delta_l), ties by
//     input index. Level l occupies internal rows [off_l, off_l + n_l). A
//     hierarchy object holds one or more independent hierarchies ("groups");
//     its levels are ordered depth-major (depth 0 of every group, then depth
//     1, ...), so the levels of one depth are contiguous. perm[i] = global
//     input index of internal i (inputs are group-major, coarse to fine).
//   * coordinates: SoA FP64, xs[a][i] for axis a, internal order.
//   * blocks: CSR over internal rows. "diag" holds A_l = B_{l,l} for every l,
//     "lower" holds B_{k,j}, j < k. Column = internal global index (int32),
//     row pointers int64; columns ascend within a row (a row of "lower" lists
//     level 0's neighbours first, then level 1's, ...).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/mskm.h"

namespace mskm {

constexpr int kMaxLevels = 4096;  // levels of one hierarchy object (all groups of a batch)
constexpr int kBlock = 256;  // threads per block of every streaming / SpMV kernel
constexpr int kCsrPad = 16;  // tail pad (entries) of CSR column and value arrays
// SpMV variant code: lanes per row G, plus 1000: 16-byte value/column loads,
// 2000: the same non-temporal, 3000: values recomputed from point records;
// kSellCode: the sliced copy of the diagonal blocks (one row per lane), with
// 16-bit column offsets when every slice allows them; kSell32Code: the same
// copy with its 32-bit columns
constexpr int kVecFlag = 1000;
constexpr int kSellCode = 4064;
constexpr int kSell32Code = 4032;
constexpr int kTuneVariants = 22;  // widths 4..64 x the four kinds, then the two SELL codes (diagonal operator only)
constexpr int kSellC = 64;         // SELL slice height: one wave, one row per lane

// Per-level descriptor read by the kernels (all fields uniform per wave).
struct DevLevel {
  int64_t off;       // first internal row
  int32_t n;         // points of the level
  int32_t ncell_tot; // cells of the level's grid
  double delta;      // support radius
  double d2max;      // delta * delta (FP64, round to nearest)
  double inv_delta;  // 1 / delta
  double lo[3];      // grid origin
  double inv_cell;   // 1 / cell side
  int32_t nc[3];     // cells per axis
  int32_t cs_off;    // offset of this level's cell_start table in the shared array
  int32_t first;     // first (coarsest) level of this level's hierarchy
  int32_t next;      // next finer level of the same hierarchy (-1 at its top)
};

// A launch table: block b works on rows [row0[b], row1[b]) of level lev[b].
// Blocks of one level are contiguous: [lev_begin[l], lev_begin[l+1]).
struct WorkTable {
  int32_t nblocks = 0;
  int32_t rows_per_block = 0;
  int32_t* lev = nullptr;     // device [nblocks]
  int64_t* row0 = nullptr;    // device [nblocks]
  int64_t* row1 = nullptr;    // device [nblocks]
  int32_t* lev_begin = nullptr;  // device [L+1]
  std::vector<int32_t> h_lev_begin;
};

// Sliced-ELL copy of the diagonal blocks. Each level's rows, in the internal
// (cell) order, are cut into slices of kSellC consecutive rows from the level
// start; slice s stores its width w_s = longest row of the slice rounded up
// to a multiple of 4, and entry k of slot t at
// sptr[s] + (k / 4) * 4 kSellC + 4 t + k % 4 (four consecutive entries of a
// slot side by side, one vector load each; shorter rows padded with value 0
// and their own row as column). Rows are not reordered by length: keeping
// neighbouring rows together keeps the gathers of one load instruction on
// few cache lines, which measures faster than the padding it saves.
struct Sell {
  int64_t nslices = 0, entries = 0;
  int64_t* sptr = nullptr;   // [nslices + 1]
  int32_t* rows = nullptr;   // [nslices * kSellC] internal row of each slot, -1 for an empty slot
  int32_t* col = nullptr;    // [entries]
  // 16-bit copy of the columns, col = cbase[slice] + col16 (null when some
  // slice's columns span more than 65536 rows)
  uint16_t* col16 = nullptr;  // [entries]
  int32_t* cbase = nullptr;   // [nslices] smallest column of each slice
  double* val = nullptr;     // [entries] FP64 values (null when not stored)
  float* val32 = nullptr;    // [entries] FP32 values (null when not stored)
  float* lo = nullptr;       // [entries] FP32 remainders (FP32-only hierarchies with the lower copy)
  std::vector<int64_t> h_slice_begin;  // [L+1] first slice of each level
};

// Sliced copy of the strictly-lower blocks (lsell.hip): the rows of each
// level in the diagonal copy's slices; within a slice of level k one segment
// per coarser level j of its hierarchy (coarsest first), laid out like a
// diagonal slice with 16-bit column offsets from the segment's smallest
// column (seg_base). Not built (built = false) when some segment spans more
// than 65536 points.
struct LSell {
  bool built = false;
  int64_t nseg = 0, entries = 0;
  int64_t* slice_seg = nullptr;  // [nslices + 1] first segment of each slice
  int64_t* seg_ptr = nullptr;    // [nseg + 1] first entry of each segment
  int32_t* seg_base = nullptr;   // [nseg] smallest column of each segment
  uint16_t* col16 = nullptr;     // [entries]
  double* val = nullptr;         // [entries] FP64 values (when stored)
  float* val32 = nullptr;        // [entries] FP32 values (when stored)
  float* lo = nullptr;           // [entries] FP32 remainders (FP32-only hierarchies)
};

// Block-Jacobi preconditioner: the diagonal blocks of A_l restricted to each
// cell of the level's grid (cells hold consecutive internal rows; cells of
// more than kBjMax rows are cut into near-equal chunks), inverted densely.
constexpr int kBjMax = 32;         // largest block
// Rows of one workgroup of whole blocks (at most): 1024 on levels of more
// than 524288 rows (at least 512 workgroups, two per CU, each thread walking
// four rows), 256 below, so that the latency-bound preconditioned updates of
// the smaller levels spread over many CUs with one row per thread (1024-row
// groups there made the fast solve 4% slower; 256-row groups on a 1M-row
// level made its update 13% slower).
constexpr int kBjGroupRows = 1024;
constexpr int kBjSmallGroupRows = 256;
constexpr int64_t kBjLargeLevelRows = 524288;
// Window of block starts of one workgroup on a level of n rows.
__host__ __device__ inline int64_t bj_group_step(int64_t n) {
  return (n > kBjLargeLevelRows ? kBjGroupRows : kBjSmallGroupRows) - kBjMax + 1;
}
struct BlockJacobi {
  bool built = false;
  int64_t nblocks = 0, nvals = 0;
  int64_t* start = nullptr;   // [nblocks + 1] first internal row of each block (blocks tile every level)
  int64_t* off = nullptr;     // [nblocks + 1] offset of each block's m x m inverse (row-major)
  int32_t* of_row = nullptr;  // [N] block of each internal row
  double* inv = nullptr;      // [nvals] FP64 inverses
  float* inv32 = nullptr;     // [nvals] FP32 copies
  WorkTable wt;               // per-level workgroups of whole blocks (<= kBjGroupRows rows)
  // the inverses of the finest depth (blocks from side_b0, levels >=
  // side_level0) are formed on the context's side stream, started once the
  // solve reaches its first chunked (many-workgroup) level, so that they
  // overlap the latency-bound middle levels rather than the one-workgroup
  // ones; ev_side marks their end and the main stream waits for it before
  // their first use (side_pending)
  int side_level0 = INT32_MAX;
  int64_t side_b0 = 0;
  bool side_pending = false, side_started = false;
  hipEvent_t ev_tables = nullptr, ev_side = nullptr;
};

struct Csr {
  int64_t nnz = 0;
  int64_t* rowptr = nullptr;  // [N+1]
  int32_t* col = nullptr;     // [nnz]
  double* val = nullptr;      // [nnz] FP64 values (optional)
  float* val32 = nullptr;     // [nnz] FP32 values (optional)
  // [nnz] FP32 remainders v - (double)(float)v, stored with FP32 values when
  // FP64 values are not: (double)val32 + (double)val32lo reproduces v to
  // about 2^-48 relative, for the FP64 residual of an FP32-only hierarchy
  float* val32lo = nullptr;
};

}  // namespace mskm

namespace mskm {
// Autotuner result remembered by the context for hierarchies of one shape.
struct TuneEntry {
  int32_t dim, L;
  int64_t N, nnz_diag, nnz_lower;
  int32_t g[3][2];
};
}  // namespace mskm

namespace mskm {
// Internal batch object assembled for mskm_solve_batch from separately
// created hierarchies (identified by handle and creation serial).
struct MergedBatch {
  std::vector<const mskm_hier*> members;
  std::vector<uint64_t> serials;
  mskm_hier* merged = nullptr;
};
}  // namespace mskm

struct mskm_ctx {
  std::vector<mskm::TuneEntry> tune_cache;  // shape -> SpMV widths
  std::vector<mskm::MergedBatch> batch_cache;  // mskm_solve_batch objects
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  // second stream (default priority): block-Jacobi inverses of a
  // hierarchy's finest levels are formed there while the main stream solves
  // the coarser levels
  hipStream_t side = nullptr;
  // device blocks of destroyed hierarchies, kept for the next allocation of
  // the same size (a hierarchy rebuilt with the same shape reuses all of
  // them without hipMalloc); at most kBlockCacheCap bytes, freed by
  // mskm_destroy or when an allocation would otherwise fail
  std::mutex cache_mu;
  std::multimap<size_t, void*> cache;
  size_t cache_bytes = 0;
  std::multimap<size_t, void*> host_cache;  // pinned host blocks, likewise (solver workspaces)
};

// Truncated Lagrange blocks frak X~_{kj}(T) of one hierarchy (trunc.hip):
// one CSR over its internal rows whose row i (level k) holds the kept
// entries of every block (k, j), j < k, level 0's columns first (columns =
// internal global indices, ascending), FP64 values, arrays padded by
// kCsrPad entries for the 16-byte-load product.
struct mskm_trunc {
  mskm_hier* h = nullptr;         // null once the hierarchy was destroyed
  double T = 0.0;
  std::vector<double> q, r2;      // [L] separation distance, (T q)^2 (inf: keep all)
  mskm::Csr X;
  std::vector<void*> allocs;
  int64_t cg_iters = 0;           // CG iterations of the Lagrange coefficient solves
  bool capped = false;            // a coefficient solve hit its iteration cap
  double build_ms = 0.0;
  ~mskm_trunc() {
    for (void* p : allocs) (void)hipFree(p);
  }
};

// Learned warm start network (learned.hip).
struct mskm_mlp {
  int32_t dim = 2, F = 56;         // point dimension, padded feature count
  std::vector<float> params;       // W1 [64][F], b1 [64], w2 [64], b2
  float* d_params = nullptr;       // device copy (FP32)
  short* d_w1b = nullptr;          // device W1 in bfloat16
  int64_t samples = 0;             // training samples used
  ~mskm_mlp() {
    (void)hipFree(d_params);
    (void)hipFree(d_w1b);
  }
};

struct mskm_hier {
  mskm_ctx* ctx = nullptr;
  uint64_t serial = 0;                  // creation number (unique per process)
  int32_t dim = 0, L = 0;
  int64_t N = 0;
  std::vector<int64_t> h_off;           // [L+1] internal offsets (level order)
  std::vector<int64_t> h_in_off;        // [L] input offset of each level
  std::vector<int32_t> h_group, h_depth, h_first, h_next;  // [L] level graph
  int32_t ngroups = 1;
  std::vector<int32_t> h_group_levels;  // [ngroups] levels per group
  std::vector<int64_t> h_group_in_off;  // [ngroups+1] input offsets of the groups
  std::vector<int32_t> h_depth_begin;   // [Dmax+1] level range of each depth
  std::vector<double> h_delta;          // [L]
  std::vector<mskm::DevLevel> h_lev;    // [L]
  mskm::DevLevel* d_lev = nullptr;      // device [L]
  double* xs = nullptr;                 // device [dim][N] SoA, internal order
  double* prec = nullptr;               // device [N][4] point records {x, y, z or 0, 1/delta of its level}
  int32_t* perm = nullptr;              // device [N] internal -> input
  int32_t* iperm = nullptr;             // device [N] input -> internal
  int32_t* cell_start = nullptr;        // device, all levels' tables
  mskm::Csr diag, lower;
  mskm::WorkTable wt_spmv;              // per-level one-pass SpMV blocks (CG phase 1)
  mskm::WorkTable wt_vec;               // per-level streaming blocks (CG phase 3)
  mskm::Sell sell;                      // sliced copy of the diagonal blocks
  mskm::LSell lsell;                    // sliced copy of the strictly-lower blocks
  mskm::WorkTable wt_sell;              // per-level blocks of 4 slices ("rows" are slices)
  mskm::BlockJacobi bj;                 // cell block-Jacobi preconditioner (built at its first use)
  int32_t spmv_g[3][2] = {{8, 8}, {32, 32}, {32, 32}};  // lanes per row [op][FP64, FP32]
  // right-hand sides per chunk of the many-rhs CG product, by R / 64 - 1 and
  // [FP64, FP32] (0: not tuned yet; set by timing at the first solve with R)
  int32_t mr_chunk[8][2] = {};
  int64_t device_bytes = 0;
  // assembly timing: events around the assembly's launches, read at the first
  // statistics query (creation returns without waiting for its last kernels)
  mutable double assemble_ms = 0.0;
  hipEvent_t ev_asm[2] = {nullptr, nullptr};
  mutable bool asm_pending = false;
  std::vector<void*> allocs;            // everything to free (given back to the context's block cache)
  std::vector<size_t> alloc_bytes;      // their sizes
  // pinned staging of host-built tables (upload_async); released at destroy,
  // after the stream has drained, so no upload waits on its copy
  std::vector<void*> stage_blocks;
  std::vector<size_t> stage_bytes;
  size_t stage_used = 0;                // bytes taken from the last staging block
  int32_t* knn = nullptr;               // [N][16] same-level nearest neighbours (learned warm start)
  std::vector<mskm_trunc*> truncs;      // thresholded blocks built on this hierarchy (detached at destroy)
  void* solve_ws = nullptr;             // solver workspace (solve.hip), created on first solve
  void (*solve_ws_free)(void*) = nullptr;
};

namespace mskm {

// error helpers (abi.hip)
void set_error(const std::string& msg);
mskm_status fail(mskm_status st, const std::string& msg);

#define MSKM_HIP_TRY(...)                                                                    \
  do {                                                                                       \
    hipError_t _e = (__VA_ARGS__);                                                           \
    if (_e != hipSuccess)                                                                    \
      return ::mskm::fail(_e == hipErrorOutOfMemory ? MSKM_ENOMEM : MSKM_EDEVICE,            \
                          std::string(#__VA_ARGS__) + ": " + hipGetErrorString(_e));         \
  } while (0)

#define MSKM_TRY(...)               \
  do {                              \
    mskm_status _s = (__VA_ARGS__); \
    if (_s < 0) return _s;          \
  } while (0)

// Context block cache (abi.hip): a block of exactly `bytes` from the cache,
// else hipMalloc (after emptying the cache if the first attempt fails).
mskm_status ctx_alloc(mskm_ctx* c, size_t bytes, void** out);
// Gives a block back to the cache (hipFree beyond the cap or without a context).
void ctx_release(mskm_ctx* c, void* p, size_t bytes);
// Frees every cached block.
void ctx_trim(mskm_ctx* c);
// Pinned host blocks: from the cache, else hipHostMalloc; given back likewise.
mskm_status ctx_host_alloc(mskm_ctx* c, size_t bytes, void** out);
void ctx_host_release(mskm_ctx* c, void* p, size_t bytes);
// Queues a host-to-device copy of `bytes` from host memory src to device dst
// on the context stream through the hierarchy's pinned staging blocks: src
// may be reused at once, and the host does not wait for the copy.
mskm_status upload_async(mskm_hier* h, void* dst, const void* src, size_t bytes);


// device allocation tracked by the hierarchy
template <typename T>
mskm_status halloc(mskm_hier* h, T** p, size_t count) {
  *p = nullptr;
  if (count == 0) count = 1;
  const size_t bytes = count * sizeof(T);
  void* q = nullptr;
  MSKM_TRY(ctx_alloc(h->ctx, bytes, &q));
  *p = static_cast<T*>(q);
  h->allocs.push_back(q);
  h->alloc_bytes.push_back(bytes);
  h->device_bytes += static_cast<int64_t>(bytes);
  return MSKM_OK;
}

// scratch allocation owned by the caller (freed with hipFree)
template <typename T>
mskm_status dalloc(T** p, size_t count) {
  *p = nullptr;
  if (count == 0) count = 1;
  hipError_t e = hipMalloc(reinterpret_cast<void**>(p), count * sizeof(T));
  if (e != hipSuccess) return fail(MSKM_ENOMEM, "hipMalloc of " + std::to_string(count * sizeof(T)) + " bytes failed");
  return MSKM_OK;
}

// Pieces of one device allocation, each aligned to 256 bytes.
struct Carve {
  size_t bytes = 0;
  std::vector<std::pair<void**, size_t>> want;
  template <typename T>
  void add(T** p, size_t count) {
    want.push_back({reinterpret_cast<void**>(p), std::max<size_t>(count, 1) * sizeof(T)});
    bytes += (std::max<size_t>(count, 1) * sizeof(T) + 255) / 256 * 256;
  }
  // one hipMalloc for all pieces; *base receives it (freed by the caller)
  mskm_status alloc(void** base) {
    char* b = nullptr;
    MSKM_TRY(dalloc(&b, bytes));
    *base = b;
    place(b);
    return MSKM_OK;
  }
  // one block from the context's cache for all pieces (given back by the caller)
  mskm_status alloc(mskm_ctx* c, void** base);
  void place(char* b) {
    size_t o = 0;
    for (auto& w : want) {
      *w.first = b + o;
      o += (w.second + 255) / 256 * 256;
    }
  }
};

// A scratch block of the context's cache, given back when it goes out of
// scope (work on the context stream that uses it stays ordered before any
// later use of the same block).
struct CtxScratch {
  mskm_ctx* c;
  void* p;
  size_t bytes;
  ~CtxScratch();
};
inline mskm_status Carve::alloc(mskm_ctx* c, void** base) {
  MSKM_TRY(ctx_alloc(c, bytes, base));
  place(static_cast<char*>(*base));
  return MSKM_OK;
}
inline CtxScratch::~CtxScratch() { ctx_release(c, p, bytes); }

// assemble.hip
mskm_status assemble_hierarchy(mskm_hier* h, const double* points_dev, bool want64, bool want32,
                               bool want_lsell);
// The hierarchy's points in its input order, AoS [N][dim], into device memory.
mskm_status export_points_device(mskm_hier* h, double* pts_dev);
// rows_host == nullptr: every row of the level; else the listed rows (indices
// within the row level, host array of nrows_sel entries).
// csr: another CSR over the hierarchy's rows with the same column
// convention (the truncated blocks) instead of its own blocks.
mskm_status export_block(mskm_hier* h, int row_level, int col_level, int64_t* rowptr, int32_t* col, double* val,
                         int64_t* nnz_out, const int64_t* rows_host = nullptr, int64_t nrows_sel = 0,
                         const Csr* csr = nullptr);
// lsell.hip: the sliced copy of the lower blocks
// cnt_lv: [q][N] each row's entry count in the q-th coarser level of its
// hierarchy (from the neighbour count pass).
mskm_status build_lsell(mskm_hier* h, bool want64, bool want32, const int32_t* cnt_lv);
// Stream-ordered exclusive scan; part: scratch of scan_parts(n) entries.
int64_t scan_parts(int64_t n);
mskm_status exclusive_scan_i64(hipStream_t s, const int64_t* in, int64_t* out, int64_t n, int64_t* part);
// Rows of each level split into blocks of max(min_rows, n_l / max_blocks) rows,
// so that no level has more than max_blocks blocks.
mskm_status build_work_table(mskm_hier* h, WorkTable* wt, int min_rows, int max_blocks_per_level);
// precond.hip
mskm_status build_block_jacobi(mskm_hier* h);
// Orders the main stream after the inverses of levels up to `hi` (a no-op
// once they are known to be formed).
mskm_status bj_wait(mskm_hier* h, int hi);
// Starts the side-stream inversion of the finest depth's blocks (once).
mskm_status bj_start_side(mskm_hier* h);
template <typename TX>
void launch_bj_apply(mskm_hier* h, int lo, int hi, const TX* r, TX* u);

// solve.hip
mskm_status apply_op(mskm_hier* h, int op, int prec, const double* x_in, int nrhs, double* y_in, bool io_dev);
mskm_status apply_internal(mskm_hier* h, int op, int prec, const void* x, void* y, int repeats, float* avg_ms);
mskm_status autotune(mskm_hier* h, int repeats, float* times_out);
mskm_status time_cg_product(mskm_hier* h, int level, int prec, int repeats, float* avg_ms);
mskm_status time_mr_product(mskm_hier* h, int level, int prec, int R, int repeats, float* avg_ms);
mskm_status set_mr_chunk(mskm_hier* h, int R, int prec, int chunk);
mskm_status solve(mskm_hier* h, const double* f, int nrhs, const mskm_solve_opts* o, double* alpha,
                  mskm_report* rep);
// trunc.hip: q per level, pattern and values of the truncated blocks
mskm_status trunc_build(mskm_hier* h, double T, double cg_rtol, mskm_trunc* tr);
// allocation owned by a truncated-block object
template <typename T>
mskm_status tr_alloc(mskm_trunc* tr, T** p, size_t count) {
  MSKM_TRY(dalloc(p, count));
  tr->allocs.push_back(*p);
  return MSKM_OK;
}
// solve.hip: the perturbed split with the truncated blocks (one right-hand side)
mskm_status trunc_solve(mskm_hier* h, const Csr& X, const double* f, const mskm_solve_opts* o, double* alpha,
                        mskm_report* rep);
// learned.hip
mskm_status ensure_knn(mskm_hier* h);
mskm_status mlp_new(int dim, uint64_t seed, mskm_mlp** out);
mskm_status mlp_upload(mskm_mlp* m);
template <typename TX>
mskm_status mlp_predict_rows(mskm_hier* h, const mskm_mlp* m, int l, const TX* b, TX* x0);
mskm_status mlp_train_device(mskm_hier* h, mskm_mlp* m, const std::vector<double*>& rhs_int,
                             const std::vector<double*>& alpha_int, int64_t samples, int steps, float lr, uint64_t seed,
                             std::vector<float>* loss_log);
mskm_status mlp_fit(mskm_ctx* ctx, mskm_mlp* m, const float* X, const float* y, int64_t ns, int steps, float lr,
                    bool io_dev, float* loss_log);
mskm_status mlp_predict_all(mskm_hier* h, const mskm_mlp* m, const double* b, double* x0, bool io_dev);
mskm_status knn_export(mskm_hier* h, int level, int32_t* out);
mskm_status train_pairs(mskm_hier* h, const double* f, int nrhs, bool io_dev, double cg_rtol,
                        std::vector<double*>* rhs_int, std::vector<double*>* alpha_int);

// solve_mr.hip: many right-hand sides in the same launches (2 <= nrhs <= 512)
bool mr_supported(int nrhs);
// Columns n0 .. n0+R-1 of A_l^-1 (the coefficient vectors of level l's
// Lagrange functions, Section 4) by CG from zero on A_l with unit right-hand
// sides: Z [N][R] FP64 device, internal order, rows of level l written
// (columns past the level's end are zero). The CG iterations (sum over the
// R systems) and whether a cap stopped one are returned.
mskm_status lagrange_columns(mskm_hier* h, int l, int64_t n0, int R, double rtol, int maxit, double* Z,
                             int64_t* iters, bool* capped);
mskm_status solve_multi(mskm_hier* h, const double* f, int nrhs, const mskm_solve_opts* o, double* alpha,
                        mskm_report* rep);
mskm_status residual(mskm_hier* h, const double* alpha, const double* f, int nrhs, double* rel_out, bool io_dev);
// Allocation-free residual: device vectors in input order, partials in the
// static scratch array (noalloc_init at context creation), stream-ordered.
mskm_status noalloc_init(int device);
mskm_status residual_noalloc(mskm_hier* h, const double* alpha, const double* f, int nrhs, double* rel_out);
mskm_status evaluate(mskm_hier* h, const double* alpha, int nrhs, const double* query, int64_t nq, double* out,
                     bool io_dev);

}  // namespace mskm
