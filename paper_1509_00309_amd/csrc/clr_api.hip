// Host side of the C ABI declared in include/clr.h: contexts, CLR matrices in
// blocks of an arena, and the drivers of the product, the blockwise combination and
// the Newton-Schulz square-root inverse (Sec. 4.1 and 4.2 of Calvin, Lewis &
// Valeev, IA^3 2015).
//
// Storage of a CLR matrix with blocking m_0..m_{R-1} x n_0..n_{C-1}: one FP64
// arena and a table of block offsets; block (I, J) starts at arena +
// boff[I * C + J].  A dense block is m x n column-major (ld m); a factored
// block stores U (m x r) then V (n x r).  Three layouts share that form:
//  * packed: a block takes exactly what it stores (inputs from clr_create,
//    compressed inputs, the identity, clr_compact), so memory follows ranks;
//  * planned: a product or combination reserves, per block, the most its
//    result can store (m n when accumulated densely, since a truncation keeps
//    2 r <= min(m, n) and (m + n) r <= m n; (m + n) R for a concatenation of
//    rank R) and writes the offsets on the device before it runs;
//  * dense slots (m n for every block): the fixed iterates of a captured
//    Newton-Schulz iteration, whose results change rank from replay to replay.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <cstdarg>
#include <mutex>
#include <string>
#include <memory>
#include <vector>

#include "clr.h"
#include "clr_internal.h"

using namespace clr;

// ---------------------------------------------------------------------------
// Context and buffers
// ---------------------------------------------------------------------------

// A caller's device allocator (clr_set_allocator); alloc == null is hipMalloc.
struct Allocator {
  clr_alloc_fn alloc = nullptr;
  clr_release_fn release = nullptr;
  void* user = nullptr;
  void* stream = nullptr;
};

// A growable device buffer.  src (optional) names the allocator to grow from;
// owner is the allocator that made p, and the one that releases it.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  const Allocator* src = nullptr;
  Allocator owner;
};

// Workspace of the product and combination pipelines: per-block counts and
// offsets, the work lists, the thin-product pool, recompression scratch, the
// dense accumulators and the device-resident list lengths.  The context holds
// one set for its calls; a captured iteration owns another, whose buffers
// must not move once a graph has recorded their addresses.
struct Work {
  DevBuf cnt, off, st, flags, totals, seg_dense, items_dense, seg_thin1, items_thin1, seg_thin2,
      items_thin2, pieces, rec, pool, scratch, acc, terms, comb_dense, recg, order, order_thin,
      sortw, live, flops, lists;
  clr::Caps seen{};   // largest list lengths of the runs sized on the host
  double host_flops = 0.0;   // product flops of those runs (their symbolic statistics)
};

struct clr_context {
  int device = 0;
  hipStream_t stream = nullptr;
  Allocator alloc;   // device memory of matrices and work lists (default hipMalloc)
  std::string last_error;
  Work w;
  Work gw;   // work lists of graph-replayed iterations (kept between calls, only grown)
  DevBuf status, ptrs;
  hipEvent_t ev[10] = {};
  // grouped-GEMM item edges per precision (0: the kernel's largest tile), set
  // explicitly or by clr_autotune
  // per precision (0: FP64 and OZAKI, 1: MIXED) and shape class; 0 is the
  // kernel's full tile
  clr::EdgeTable tiles[2] = {};
  // dense certificate before the truncated SVD of dense-accumulated blocks
  int dense_cert = 1;
  // clr_compress truncates by column-pivoted QR instead of the SVD
  int compress_rrqr = 0;
  // Stream-ordered cache of freed matrix allocations: a matrix released on the
  // context stream can back the next matrix of a similar size without a
  // hipMalloc (all users are ordered on the same stream).
  std::vector<std::pair<void*, size_t>> cache;
  size_t cache_bytes = 0;
};

struct clr_matrix {
  clr_context* ctx = nullptr;
  Allocator owner;   // the allocator of block (alloc == null: the context's hipMalloc cache)
  int nrb = 0, ncb = 0;
  std::vector<int> rs, cs, roff, coff;
  int64_t rows = 0, cols = 0;
  int* d_roff = nullptr;
  int* d_coff = nullptr;
  int* d_kind = nullptr;
  int* d_rank = nullptr;
  double* d_norm = nullptr;
  int64_t* d_boff = nullptr;   // block offsets into the arena (doubles)
  double* arena = nullptr;
  int64_t cap = 0;             // arena capacity (doubles)
  std::vector<int64_t> boff;   // host copy of d_boff when host_boff
  bool host_boff = false;      // false: offsets planned on the device
  void* block = nullptr;   // one allocation holding the arena and the metadata
  size_t block_bytes = 0;

  MatView view() const {
    MatView v;
    v.kind = d_kind;
    v.rank = d_rank;
    v.norm = d_norm;
    v.roff = d_roff;
    v.coff = d_coff;
    v.arena = arena;
    v.boff = d_boff;
    v.nrb = nrb;
    v.ncb = ncb;
    return v;
  }
  bool square_blocked() const { return rs == cs; }
};

namespace {

constexpr int kMaxBlockEdge = 512;

// Device memory of clr_identity_residual_noalloc: the per-block terms of the
// residual, at most kNoAllocMaxBlocks of them.  Every device the library runs
// on holds its own copy for the life of the process.  Host code never uses the
// array's name as an address: its device address is looked up once per device
// (noalloc_setup, at context creation) and kept in noalloc_ptr.
constexpr int64_t kNoAllocMaxBlocks = 65536;
static __device__ __align__(256) double noalloc_scratch[kNoAllocMaxBlocks];
constexpr int kMaxDevices = 256;
std::mutex noalloc_mu;
double* noalloc_ptr[kMaxDevices] = {};

// With `device` current: record the device address of noalloc_scratch.
hipError_t noalloc_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(noalloc_mu);
  if (noalloc_ptr[device]) return hipSuccess;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(noalloc_scratch));
  if (e != hipSuccess) return e;
  noalloc_ptr[device] = static_cast<double*>(p);
  return hipSuccess;
}

double* noalloc_terms(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(noalloc_mu);
  return noalloc_ptr[device];
}

clr_status fail(clr_context* ctx, clr_status s, const char* fmt, ...) {
  if (ctx) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    ctx->last_error = buf;
  }
  return s;
}

#define HIP_TRY(ctx, expr)                                                              \
  do {                                                                                  \
    hipError_t _e = (expr);                                                             \
    if (_e != hipSuccess)                                                               \
      return fail((ctx), CLR_ERR_HIP, "%s failed: %s", #expr, hipGetErrorString(_e)); \
  } while (0)

// Memory from an allocator (hipMalloc when it has no alloc function).
void* dev_alloc(const Allocator& a, size_t bytes) {
  void* p = nullptr;
  if (a.alloc) return a.alloc(bytes, a.stream, a.user);
  return hipMalloc(&p, bytes) == hipSuccess ? p : nullptr;
}
void dev_release(const Allocator& a, void* p, size_t bytes) {
  if (!p) return;
  if (a.alloc) {
    if (a.release) a.release(p, bytes, a.stream, a.user);
  } else {
    (void)hipFree(p);
  }
}

void free_buf(DevBuf& b) {
  dev_release(b.owner, b.p, b.bytes);
  b.p = nullptr;
  b.bytes = 0;
  b.owner = Allocator{};
}

hipError_t ensure(DevBuf& b, size_t bytes) {
  if (bytes == 0) bytes = 8;
  if (b.bytes >= bytes) return hipSuccess;
  const size_t want = std::max(bytes, b.bytes + b.bytes / 2);
  free_buf(b);
  const Allocator a = b.src ? *b.src : Allocator{};
  (void)hipGetLastError();
  b.p = dev_alloc(a, want);
  b.bytes = want;
  if (!b.p) {
    (void)hipGetLastError();
    b.p = dev_alloc(a, bytes);
    b.bytes = bytes;
  }
  if (!b.p) {
    b.bytes = 0;
    return hipErrorOutOfMemory;
  }
  b.owner = a;
  return hipSuccess;
}

template <typename F>
void each_buf(Work& w, F f) {
  for (DevBuf* b : {&w.cnt, &w.off, &w.st, &w.flags, &w.totals, &w.seg_dense, &w.items_dense,
                    &w.seg_thin1, &w.items_thin1, &w.seg_thin2, &w.items_thin2, &w.pieces, &w.rec,
                    &w.pool, &w.scratch, &w.acc, &w.terms, &w.comb_dense, &w.recg, &w.order,
                    &w.order_thin, &w.sortw, &w.live, &w.flops, &w.lists})
    f(*b);
}
void free_work(Work& w) {
  each_buf(w, [](DevBuf& b) { free_buf(b); });
}
// Grow the buffers of w from allocator a from now on.
void bind_work(Work& w, const Allocator* a) {
  each_buf(w, [a](DevBuf& b) { b.src = a; });
}

template <typename T>
T* as(DevBuf& b) {
  return static_cast<T*>(b.p);
}

constexpr size_t kCacheLimit = (size_t)96 << 30;

hipError_t ctx_malloc(clr_context* ctx, size_t bytes, void** p, size_t* got) {
  if (ctx->alloc.alloc) {   // the caller's allocator: no cache of our own
    *p = ctx->alloc.alloc(bytes, ctx->alloc.stream, ctx->alloc.user);
    *got = bytes;
    return *p ? hipSuccess : hipErrorOutOfMemory;
  }
  int best = -1;
  for (int i = 0; i < (int)ctx->cache.size(); ++i) {
    const size_t b = ctx->cache[i].second;
    if (b >= bytes && b <= bytes + bytes / 4 + 65536 &&
        (best < 0 || b < ctx->cache[best].second))
      best = i;
  }
  if (best >= 0) {
    *p = ctx->cache[best].first;
    *got = ctx->cache[best].second;
    ctx->cache_bytes -= *got;
    ctx->cache.erase(ctx->cache.begin() + best);
    return hipSuccess;
  }
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess && !ctx->cache.empty()) {
    (void)hipGetLastError();
    (void)hipStreamSynchronize(ctx->stream);
    for (auto& c : ctx->cache) (void)hipFree(c.first);
    ctx->cache.clear();
    ctx->cache_bytes = 0;
    e = hipMalloc(p, bytes);
  }
  *got = bytes;
  return e;
}

void ctx_release(clr_context* ctx, void* p, size_t bytes) {
  if (!p) return;
  ctx->cache.emplace_back(p, bytes);
  ctx->cache_bytes += bytes;
  while (ctx->cache_bytes > kCacheLimit && !ctx->cache.empty()) {
    (void)hipStreamSynchronize(ctx->stream);
    ctx->cache_bytes -= ctx->cache.front().second;
    (void)hipFree(ctx->cache.front().first);
    ctx->cache.erase(ctx->cache.begin());
  }
}

void free_matrix(clr_matrix* m) {
  if (!m) return;
  if (m->owner.alloc)
    dev_release(m->owner, m->block, m->block_bytes);
  else
    ctx_release(m->ctx, m->block, m->block_bytes);
  delete m;
}

// Dense-slot offset of block (I, J): room for every block stored dense.
int64_t dense_slot(const std::vector<int>& roff, const std::vector<int>& coff, int64_t cols, int I,
                   int J) {
  return (int64_t)roff[I] * cols + (int64_t)(roff[I + 1] - roff[I]) * coff[J];
}

// Allocate a matrix with the given blocking; metadata set to "all zero blocks".
// Layout: offsets given on the host (with the arena capacity cap), or none and
// cap < 0 for dense slots, or none and cap >= 0 for offsets that a kernel
// writes before the matrix is read (zero until then).
clr_status alloc_matrix(clr_context* ctx, const std::vector<int>& rs, const std::vector<int>& cs,
                        clr_matrix** out, const std::vector<int64_t>* offsets = nullptr,
                        int64_t cap = -1) {
  *out = nullptr;
  if (rs.empty() || cs.empty()) return fail(ctx, CLR_ERR_INVALID_ARG, "empty blocking");
  for (int v : rs)
    if (v < 1) return fail(ctx, CLR_ERR_INVALID_ARG, "block size %d < 1", v);
  for (int v : cs)
    if (v < 1) return fail(ctx, CLR_ERR_INVALID_ARG, "block size %d < 1", v);
  for (int v : rs)
    if (v > kMaxBlockEdge)
      return fail(ctx, CLR_ERR_CAPACITY, "block size %d exceeds %d", v, kMaxBlockEdge);
  for (int v : cs)
    if (v > kMaxBlockEdge)
      return fail(ctx, CLR_ERR_CAPACITY, "block size %d exceeds %d", v, kMaxBlockEdge);
  clr_matrix* m = new clr_matrix();
  m->ctx = ctx;
  m->nrb = (int)rs.size();
  m->ncb = (int)cs.size();
  m->rs = rs;
  m->cs = cs;
  m->roff.assign(m->nrb + 1, 0);
  m->coff.assign(m->ncb + 1, 0);
  for (int i = 0; i < m->nrb; ++i) m->roff[i + 1] = m->roff[i] + rs[i];
  for (int j = 0; j < m->ncb; ++j) m->coff[j + 1] = m->coff[j] + cs[j];
  m->rows = m->roff.back();
  m->cols = m->coff.back();
  const int64_t nb = (int64_t)m->nrb * m->ncb;
  if (nb > (int64_t)1 << 30) {
    free_matrix(m);
    return fail(ctx, CLR_ERR_CAPACITY, "too many blocks");
  }
  if (offsets) {
    if ((int64_t)offsets->size() != nb || cap < 0) {
      delete m;
      return fail(ctx, CLR_ERR_INTERNAL, "block offsets do not match the blocking");
    }
    m->boff = *offsets;
    m->cap = cap;
    m->host_boff = true;
  } else if (cap < 0) {
    m->boff.resize(nb);
    for (int I = 0; I < m->nrb; ++I)
      for (int J = 0; J < m->ncb; ++J)
        m->boff[(size_t)I * m->ncb + J] = dense_slot(m->roff, m->coff, m->cols, I, J);
    m->cap = m->rows * m->cols;
    m->host_boff = true;
  } else {
    m->cap = cap;
  }
  auto up = [](size_t b) { return (b + 255) / 256 * 256; };
  const size_t b_arena = up(sizeof(double) * (size_t)std::max<int64_t>(m->cap, 1));
  const size_t b_norm = up(sizeof(double) * nb);
  const size_t b_boff = up(sizeof(int64_t) * nb);
  const size_t b_kind = up(sizeof(int) * nb);
  const size_t b_roff = up(sizeof(int) * (m->nrb + 1));
  const size_t b_coff = up(sizeof(int) * (m->ncb + 1));
  const size_t total = b_arena + b_norm + b_boff + 2 * b_kind + b_roff + b_coff;
  m->owner = ctx->alloc;
  hipError_t e = ctx_malloc(ctx, total, &m->block, &m->block_bytes);
  if (e == hipSuccess) {
    char* base = static_cast<char*>(m->block);
    m->arena = reinterpret_cast<double*>(base);
    base += b_arena;
    m->d_norm = reinterpret_cast<double*>(base);
    base += b_norm;
    m->d_boff = reinterpret_cast<int64_t*>(base);
    base += b_boff;
    m->d_kind = reinterpret_cast<int*>(base);
    m->d_rank = reinterpret_cast<int*>(base + b_kind);
    m->d_roff = reinterpret_cast<int*>(base + 2 * b_kind);
    m->d_coff = reinterpret_cast<int*>(base + 2 * b_kind + b_roff);
  }
  if (e == hipSuccess)
    e = hipMemcpyAsync(m->d_roff, m->roff.data(), sizeof(int) * (m->nrb + 1),
                       hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(m->d_coff, m->coff.data(), sizeof(int) * (m->ncb + 1),
                       hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess) {
    if (m->host_boff)
      e = hipMemcpyAsync(m->d_boff, m->boff.data(), sizeof(int64_t) * nb, hipMemcpyHostToDevice,
                         ctx->stream);
    else
      e = launch_fill_i32(reinterpret_cast<int*>(m->d_boff), 0, 2 * nb, ctx->stream);
  }
  if (e == hipSuccess) e = launch_fill_i32(m->d_kind, 0, nb, ctx->stream);
  if (e == hipSuccess) e = launch_fill_i32(m->d_rank, 0, nb, ctx->stream);
  if (e == hipSuccess) e = launch_fill_f64(m->d_norm, 0.0, nb, ctx->stream);
  // host vectors roff/coff outlive the copies: they belong to the matrix
  if (e != hipSuccess) {
    free_matrix(m);
    return fail(ctx, CLR_ERR_HIP, "matrix allocation failed: %s", hipGetErrorString(e));
  }
  *out = m;
  return CLR_OK;
}

clr_status check_opts(clr_context* ctx, const clr_gemm_opts* o) {
  if (!o) return fail(ctx, CLR_ERR_INVALID_ARG, "null options");
  if (!(o->tol >= 0.0) || !(o->tol < 1.0)) return fail(ctx, CLR_ERR_INVALID_ARG, "tol must be in [0, 1)");
  if (!(o->eps_sp >= 0.0)) return fail(ctx, CLR_ERR_INVALID_ARG, "eps_sp must be >= 0");
  if (o->screen != CLR_SCREEN_ABS && o->screen != CLR_SCREEN_AREA)
    return fail(ctx, CLR_ERR_INVALID_ARG, "bad screen mode");
  if (o->precision != CLR_FP64 && o->precision != CLR_MIXED && o->precision != CLR_OZAKI)
    return fail(ctx, CLR_ERR_INVALID_ARG, "bad precision");
  if (o->precision == CLR_OZAKI && o->split != 0 && (o->split < 2 || o->split > kOzMaxSlices))
    return fail(ctx, CLR_ERR_INVALID_ARG, "OZAKI digits must be 2..%d (0: %d)", kOzMaxSlices,
                kOzMaxSlices);
  if (!std::isfinite(o->alpha)) return fail(ctx, CLR_ERR_INVALID_ARG, "alpha must be finite");
  return CLR_OK;
}

// live: optional device-resident item count (n is then the launch's capacity).
hipError_t run_ggemm(const clr_gemm_opts* o, const GemmItem* items, const Seg* segs, int n,
                     hipStream_t s, bool dense = false, const int* order = nullptr,
                     const int64_t* live = nullptr) {
  if (o->precision == CLR_MIXED)
    return launch_ggemm_f32(items, segs, n, o->split, s, dense, order, live);
  if (o->precision == CLR_OZAKI && dense) {
    if (live) return hipErrorNotSupported;   // the INT8 form sizes its launch on the host
    return launch_ggemm_ozaki(items, segs, n, o->split ? o->split : kOzMaxSlices, s, order);
  }
  return launch_ggemm_f64(items, segs, n, s, dense, order, live);
}

// The dense accumulation of a product: the longest-first list `order` (n
// slots, followed by one int of room for the counter) on a persistent launch
// of the LDS kernel (the INT8 form keeps its own launch).
hipError_t run_dense(const clr_gemm_opts* o, const GemmItem* items, const Seg* segs, int n,
                     int* order, hipStream_t s, const int64_t* live) {
  if (n <= 0) return hipSuccess;
  if (o->precision == CLR_OZAKI) return run_ggemm(o, items, segs, n, s, true, order, live);
  int* next = order + n;
  hipError_t e = launch_fill_i32(next, 0, 1, s);
  if (e != hipSuccess) return e;
  if (o->precision == CLR_MIXED)
    return launch_ggemm_f32(items, segs, n, o->split, s, true, order, live, next);
  return launch_ggemm_f64(items, segs, n, s, true, order, live, next);
}

int max_item(const clr_gemm_opts* o) {
  if (o->precision == CLR_OZAKI) return kMaxItemOzaki;
  if (o->precision == CLR_MIXED) return o->split ? kMaxItemF32Split : kMaxItemF32;
  return kMaxItemF64;
}

// Factor products (one side a rank) run on the wave-per-item kernel.
hipError_t run_wgemm(const clr_gemm_opts* o, const GemmItem* items, const Seg* segs, int n,
                     hipStream_t s, const int* order = nullptr, const int64_t* live = nullptr) {
  if (o->precision == CLR_MIXED) return launch_wgemm_f32(items, segs, n, o->split, s, order, live);
  return launch_wgemm_f64(items, segs, n, s, order, live);
}

// Item edges of one call: the context's table for the precision (OZAKI shares
// the FP64 one), unset classes at the kernel's full tile, capped to it.
EdgeTable edge_table(const clr_context* ctx, const clr_gemm_opts* o) {
  const int pi = o->precision == CLR_MIXED ? 1 : 0;
  const EdgeTable& t = ctx->tiles[pi];
  const int top = max_item(o);
  EdgeTable e;
  for (int c = 0; c < kDenseClasses; ++c) e.dense[c] = t.dense[c] > 0 ? std::min(t.dense[c], top) : top;
  for (int c = 0; c < kThinClasses; ++c)
    e.thin[c] = t.thin[c] > 0 ? std::min(t.thin[c], kMaxItemThin) : kMaxItemThin;
  return e;
}

// Read and clear the device status word; map it to a status code.
clr_status check_status(clr_context* ctx) {
  int h = 0;
  HIP_TRY(ctx, hipMemcpyAsync(&h, ctx->status.p, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  if (h == 0) return CLR_OK;
  HIP_TRY(ctx, launch_fill_i32(as<int>(ctx->status), 0, 1, ctx->stream));
  if (h & 2) return fail(ctx, CLR_ERR_NONFINITE, "non-finite block norm");
  if (h & (4 | 8)) return fail(ctx, CLR_ERR_INTERNAL, "recompression working set mis-planned");
  if (h & 1) return fail(ctx, CLR_ERR_INTERNAL, "Jacobi SVD did not converge");
  return fail(ctx, CLR_ERR_INTERNAL, "device status %d", h);
}

float elapsed(hipEvent_t a, hipEvent_t b) {
  float ms = 0.f;
  if (hipEventElapsedTime(&ms, a, b) != hipSuccess) return 0.f;
  return ms;
}

struct HostMeta {
  std::vector<int> kind, rank;
  std::vector<double> norm;
};

clr_status fetch_meta(clr_context* ctx, const clr_matrix* m, HostMeta& h) {
  const size_t nb = (size_t)m->nrb * m->ncb;
  h.kind.resize(nb);
  h.rank.resize(nb);
  h.norm.resize(nb);
  HIP_TRY(ctx, hipMemcpyAsync(h.kind.data(), m->d_kind, nb * sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
  HIP_TRY(ctx, hipMemcpyAsync(h.rank.data(), m->d_rank, nb * sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
  HIP_TRY(ctx, hipMemcpyAsync(h.norm.data(), m->d_norm, nb * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  return CLR_OK;
}

double stored_elements(const clr_matrix* m, const HostMeta& h) {
  double s = 0.0;
  for (int I = 0; I < m->nrb; ++I)
    for (int J = 0; J < m->ncb; ++J) {
      const int k = h.kind[(size_t)I * m->ncb + J];
      if (k == 1) s += (double)m->rs[I] * m->cs[J];
      if (k == 2) s += (double)(m->rs[I] + m->cs[J]) * h.rank[(size_t)I * m->ncb + J];
    }
  return s;
}

// Packed offsets of the blocks described by h (each takes what it stores);
// returns the arena capacity.
int64_t packed_offsets(const clr_matrix* m, const HostMeta& h, std::vector<int64_t>& offs) {
  offs.assign((size_t)m->nrb * m->ncb, 0);
  int64_t cap = 0;
  for (int I = 0; I < m->nrb; ++I)
    for (int J = 0; J < m->ncb; ++J) {
      const size_t b = (size_t)I * m->ncb + J;
      offs[b] = cap;
      cap += stored_size(h.kind[b], m->rs[I], m->cs[J], h.rank[b]);
    }
  return cap;
}

// A copy of src in another layout: offsets given on the host with the arena
// capacity, or dense slots (offs null).  Metadata is copied; every block's
// stored elements move to their new place.
clr_status relayout_matrix(clr_context* ctx, const clr_matrix* src, const std::vector<int64_t>* offs,
                           int64_t cap, clr_matrix** out) {
  clr_matrix* m = nullptr;
  clr_status s = offs ? alloc_matrix(ctx, src->rs, src->cs, &m, offs, cap)
                      : alloc_matrix(ctx, src->rs, src->cs, &m);
  if (s != CLR_OK) return s;
  const size_t nb = (size_t)src->nrb * src->ncb;
  hipError_t e = hipMemcpyAsync(m->d_kind, src->d_kind, nb * sizeof(int), hipMemcpyDeviceToDevice, ctx->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(m->d_rank, src->d_rank, nb * sizeof(int), hipMemcpyDeviceToDevice, ctx->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(m->d_norm, src->d_norm, nb * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream);
  if (e == hipSuccess) e = launch_relayout(src->view(), m->arena, m->d_boff, ctx->stream);
  if (e != hipSuccess) {
    free_matrix(m);
    return fail(ctx, CLR_ERR_HIP, "relayout: %s", hipGetErrorString(e));
  }
  *out = m;
  return CLR_OK;
}

// m takes t's storage and t m's old one, which is released with t.  Same
// blocking; the release is ordered on the context stream after the work that
// read it.
void adopt_storage(clr_matrix* m, clr_matrix* t) {
  std::swap(m->owner, t->owner);
  std::swap(m->block, t->block);
  std::swap(m->block_bytes, t->block_bytes);
  std::swap(m->arena, t->arena);
  std::swap(m->cap, t->cap);
  std::swap(m->d_boff, t->d_boff);
  std::swap(m->boff, t->boff);
  std::swap(m->host_boff, t->host_boff);
  std::swap(m->d_kind, t->d_kind);
  std::swap(m->d_rank, t->d_rank);
  std::swap(m->d_norm, t->d_norm);
  std::swap(m->d_roff, t->d_roff);
  std::swap(m->d_coff, t->d_coff);
  free_matrix(t);
}

// Repack m in place so that its arena holds exactly the stored elements.
clr_status compact_matrix(clr_context* ctx, clr_matrix* m) {
  HostMeta h;
  clr_status s = fetch_meta(ctx, m, h);
  if (s != CLR_OK) return s;
  std::vector<int64_t> offs;
  const int64_t cap = packed_offsets(m, h, offs);
  if (m->host_boff && cap == m->cap && offs == m->boff) return CLR_OK;   // already packed
  clr_matrix* t = nullptr;
  s = relayout_matrix(ctx, m, &offs, cap, &t);
  if (s != CLR_OK) return s;
  adopt_storage(m, t);
  return CLR_OK;
}

// Upload a host vector into a growable device buffer (synchronous with the stream).
template <typename T>
clr_status upload(clr_context* ctx, DevBuf& b, const std::vector<T>& v) {
  HIP_TRY(ctx, ensure(b, sizeof(T) * v.size()));
  if (!v.empty())
    HIP_TRY(ctx, hipMemcpyAsync(b.p, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice, ctx->stream));
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  return CLR_OK;
}

// Output-product slots of the recompression launch (one GEMM item and one
// term per recompressed block).
// Recompression workspace of n items: the emitted G * basis products (items
// and segments), the launch order of the register engine, the dense
// certificates and the launch's counters.
struct RecWork {
  GemmItem* gi;
  Seg* gs;
  int* order;
  int* cert;
  RecCounters* ctr;
};
inline size_t align256(size_t b) { return (b + 255) / 256 * 256; }
size_t rec_work_bytes(int64_t nitems) {
  const size_t n = (size_t)std::max<int64_t>(nitems, 1);
  return align256(sizeof(GemmItem) * n) + align256(sizeof(Seg) * n) +
         align256(sizeof(int) * (n + 1)) + align256(sizeof(int) * (n + 3)) + sizeof(RecCounters);
}
RecWork rec_work(void* base, int64_t nitems) {
  const size_t n = (size_t)std::max<int64_t>(nitems, 1);
  char* p = static_cast<char*>(base);
  RecWork w;
  w.gi = reinterpret_cast<GemmItem*>(p);
  p += align256(sizeof(GemmItem) * n);
  w.gs = reinterpret_cast<Seg*>(p);
  p += align256(sizeof(Seg) * n);
  w.order = reinterpret_cast<int*>(p);   // the launch order and the persistent counter
  p += align256(sizeof(int) * (n + 1));
  w.cert = reinterpret_cast<int*>(p);   // the proofs and three persistent counters
  p += align256(sizeof(int) * (n + 3));
  w.ctr = reinterpret_cast<RecCounters*>(p);
  return w;
}

// Recompression of nitems result blocks with workspace W.  With live (a
// device-resident count), nitems is the capacity and W.recg must already
// hold it: nothing is allocated.
hipError_t launch_recompress_work(clr_context* ctx, Work& W, const RecItem* items,
                                  const Piece* pieces, int nitems, double tol, bool timed = false,
                                  const int64_t* live = nullptr) {
  if (live) {
    if (W.recg.bytes < rec_work_bytes(nitems)) return hipErrorInvalidValue;
  } else {
    hipError_t e = ensure(W.recg, rec_work_bytes(nitems));
    if (e != hipSuccess) return e;
  }
  const RecWork w = rec_work(W.recg.p, nitems);
  return launch_recompress(items, pieces, nitems, tol, as<int>(ctx->status), w.gi, w.gs, w.order,
                           ctx->dense_cert ? w.cert : nullptr, live ? nullptr : w.ctr, ctx->stream,
                           timed ? ctx->ev[8] : nullptr, timed ? ctx->ev[9] : nullptr, live);
}

hipError_t launch_recompress_ctx(clr_context* ctx, const RecItem* items, const Piece* pieces,
                                 int nitems, double tol, bool timed = false) {
  return launch_recompress_work(ctx, ctx->w, items, pieces, nitems, tol, timed);
}

// Buffer sizes of a pipeline run over npairs result blocks whose work lists
// hold at most caps.c[*] entries (the output room, kCntOut, is the output
// matrix's own arena).
// Counters of doubles (arena room, pools), which may exceed int32.
inline bool counts_doubles(int c) {
  return c == kCntPool || c == kCntScratch || c == kCntOut || c == kCntAcc;
}
struct WorkSizes {
  std::vector<std::pair<DevBuf Work::*, size_t>> bufs;
};
WorkSizes work_sizes(int64_t npairs, const Caps& caps, int64_t list_ints = 0) {
  auto n = [&](int c) { return (size_t)std::max<int64_t>(caps.c[c], 0); };
  WorkSizes w;
  w.bufs = {
      {&Work::cnt, sizeof(int64_t) * kNumCounters * (size_t)npairs},
      {&Work::off, sizeof(int64_t) * kNumCounters * (size_t)npairs},
      {&Work::st, sizeof(double) * kNumStats * (size_t)npairs},
      {&Work::flags, sizeof(int) * (size_t)npairs},
      {&Work::totals, sizeof(int64_t) * kNumCounters + sizeof(double) * kNumStats},
      {&Work::seg_dense, sizeof(Seg) * n(kCntSegDense)},
      {&Work::items_dense, sizeof(GemmItem) * n(kCntGemmItems)},
      {&Work::order, sizeof(int) * (n(kCntGemmItems) + 1)},   // list and the persistent counter
      {&Work::order_thin, sizeof(int) * n(kCntThin1)},
      {&Work::seg_thin1, sizeof(Seg) * n(kCntThin1)},
      {&Work::items_thin1, sizeof(GemmItem) * n(kCntThin1)},
      {&Work::seg_thin2, sizeof(Seg) * n(kCntThin2)},
      {&Work::items_thin2, sizeof(GemmItem) * n(kCntThin2)},
      {&Work::pieces, sizeof(Piece) * n(kCntPieces)},
      {&Work::rec, sizeof(RecItem) * n(kCntComputed)},
      {&Work::pool, sizeof(double) * n(kCntPool)},
      {&Work::scratch, sizeof(double) * n(kCntScratch)},
      {&Work::comb_dense, sizeof(AxpbyDenseItem) * n(kCntCombDense)},
      {&Work::acc, sizeof(double) * n(kCntAcc)},
      {&Work::recg, rec_work_bytes(caps.c[kCntComputed])},
      {&Work::terms, sizeof(double) * (size_t)npairs},
      {&Work::live, sizeof(int64_t) * kNumLive},
      {&Work::flops, sizeof(double)},
      {&Work::lists, sizeof(int) * (size_t)list_ints},
  };
  return w;
}
hipError_t reserve_work(Work& W, const WorkSizes& ws) {
  for (const auto& b : ws.bufs) {
    hipError_t e = ensure(W.*(b.first), b.second);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}
bool work_fits(const Work& W, const WorkSizes& ws) {
  for (const auto& b : ws.bufs)
    if ((W.*(b.first)).bytes < std::max<size_t>(b.second, 8)) return false;
  return true;
}

// A run whose work-list lengths stay on the device: every list has the
// capacity caps and the launches read their lengths from W.live (see Caps).
struct DevRun {
  Caps caps;
};

// Zero kinds, ranks and norms of a matrix about to be rewritten in place.
hipError_t reset_meta(clr_context* ctx, clr_matrix* m) {
  const int64_t nb = (int64_t)m->nrb * m->ncb;
  hipError_t e = launch_fill_i32(m->d_kind, 0, nb, ctx->stream);
  if (e == hipSuccess) e = launch_fill_i32(m->d_rank, 0, nb, ctx->stream);
  if (e == hipSuccess) e = launch_fill_f64(m->d_norm, 0.0, nb, ctx->stream);
  return e;
}

// A copy with the same layout (offsets and arena copied as they are).
clr_status copy_matrix(clr_context* ctx, const clr_matrix* src, clr_matrix** out) {
  clr_matrix* m = nullptr;
  clr_status s = src->host_boff ? alloc_matrix(ctx, src->rs, src->cs, &m, &src->boff, src->cap)
                                : alloc_matrix(ctx, src->rs, src->cs, &m, nullptr, src->cap);
  if (s != CLR_OK) return s;
  const size_t nb = (size_t)src->nrb * src->ncb;
  hipError_t e = hipMemcpyAsync(m->d_kind, src->d_kind, nb * sizeof(int), hipMemcpyDeviceToDevice, ctx->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(m->d_rank, src->d_rank, nb * sizeof(int), hipMemcpyDeviceToDevice, ctx->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(m->d_norm, src->d_norm, nb * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(m->d_boff, src->d_boff, nb * sizeof(int64_t), hipMemcpyDeviceToDevice, ctx->stream);
  if (e == hipSuccess && src->cap > 0)
    e = hipMemcpyAsync(m->arena, src->arena, sizeof(double) * (size_t)src->cap,
                       hipMemcpyDeviceToDevice, ctx->stream);
  if (e != hipSuccess) {
    free_matrix(m);
    return fail(ctx, CLR_ERR_HIP, "copy failed: %s", hipGetErrorString(e));
  }
  *out = m;
  return CLR_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// Context
// ---------------------------------------------------------------------------

extern "C" clr_status clr_context_create(clr_context** ctx, void* stream) {
  if (!ctx) return CLR_ERR_INVALID_ARG;
  *ctx = nullptr;
  clr_context* c = new clr_context();
  if (hipGetDevice(&c->device) != hipSuccess || noalloc_setup(c->device) != hipSuccess) {
    delete c;
    return CLR_ERR_HIP;
  }
  c->stream = (hipStream_t)stream;
  c->alloc.stream = stream;
  bind_work(c->w, &c->alloc);
  bind_work(c->gw, &c->alloc);
  c->ptrs.src = &c->alloc;
  for (auto& e : c->ev)
    if (hipEventCreate(&e) != hipSuccess) {
      delete c;
      return CLR_ERR_HIP;
    }
  if (ensure(c->status, sizeof(int)) != hipSuccess ||
      launch_fill_i32(as<int>(c->status), 0, 1, c->stream) != hipSuccess) {
    delete c;
    return CLR_ERR_HIP;
  }
  *ctx = c;
  return CLR_OK;
}

// The caller's device allocator for this context's matrices and work lists.
// Blocks of the context's own hipMalloc cache are released now; buffers keep
// the allocator that made them until they are released or regrown.
extern "C" clr_status clr_set_allocator(clr_context* ctx, clr_alloc_fn alloc,
                                        clr_release_fn release, void* user) {
  if (!ctx) return CLR_ERR_INVALID_ARG;
  if ((alloc == nullptr) != (release == nullptr))
    return fail(ctx, CLR_ERR_INVALID_ARG, "alloc and release must be given together");
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  for (auto& c : ctx->cache) (void)hipFree(c.first);
  ctx->cache.clear();
  ctx->cache_bytes = 0;
  ctx->alloc.alloc = alloc;
  ctx->alloc.release = release;
  ctx->alloc.user = user;
  return CLR_OK;
}

extern "C" clr_status clr_context_destroy(clr_context* ctx) {
  if (!ctx) return CLR_ERR_INVALID_ARG;
  (void)hipStreamSynchronize(ctx->stream);
  free_work(ctx->w);
  free_work(ctx->gw);
  free_buf(ctx->status);
  free_buf(ctx->ptrs);
  for (auto& c : ctx->cache) (void)hipFree(c.first);
  ctx->cache.clear();
  for (auto& e : ctx->ev)
    if (e) (void)hipEventDestroy(e);
  delete ctx;
  return CLR_OK;
}

extern "C" const char* clr_last_error(const clr_context* ctx) {
  return ctx ? ctx->last_error.c_str() : "";
}

extern "C" const char* clr_status_string(clr_status s) {
  switch (s) {
    case CLR_OK: return "ok";
    case CLR_ERR_INVALID_ARG: return "invalid argument";
    case CLR_ERR_SHAPE: return "blockings do not conform";
    case CLR_ERR_CAPACITY: return "capacity exceeded";
    case CLR_ERR_NONFINITE: return "non-finite value";
    case CLR_ERR_NOT_CONVERGED: return "not converged";
    case CLR_ERR_HIP: return "HIP runtime error";
    case CLR_ERR_NORM_MISMATCH: return "norms disagree with the factors";
    case CLR_ERR_DIVERGED: return "iteration diverged";
    case CLR_ERR_INTERNAL: return "internal error";
  }
  return "unknown status";
}

// ---------------------------------------------------------------------------
// Matrices
// ---------------------------------------------------------------------------

extern "C" clr_status clr_create(clr_context* ctx, int nrb, const int* row_sizes, int ncb,
                                 const int* col_sizes, const int8_t* kind, const int* rank,
                                 const double* norms, const double* const* f0,
                                 const double* const* f1, clr_matrix** out) {
  if (!ctx || !out) return CLR_ERR_INVALID_ARG;
  *out = nullptr;
  if (nrb < 1 || ncb < 1 || !row_sizes || !col_sizes || !kind || !f0)
    return fail(ctx, CLR_ERR_INVALID_ARG, "clr_create: missing blocking, kinds or factors");
  std::vector<int> rs(row_sizes, row_sizes + nrb), cs(col_sizes, col_sizes + ncb);
  const size_t nb = (size_t)nrb * ncb;
  std::vector<int> k(nb), r(nb, 0);
  std::vector<const double*> p0(nb, nullptr), p1(nb, nullptr);
  for (int I = 0; I < nrb; ++I)
    for (int J = 0; J < ncb; ++J) {
      const size_t b = (size_t)I * ncb + J;
      k[b] = kind[b];
      if (k[b] < 0 || k[b] > 2) return fail(ctx, CLR_ERR_INVALID_ARG, "block (%d,%d): bad kind", I, J);
      if (k[b] == 0) continue;
      if (I < 0 || rs[I] < 1 || cs[J] < 1) return fail(ctx, CLR_ERR_INVALID_ARG, "bad block size");
      p0[b] = f0[b];
      if (!p0[b]) return fail(ctx, CLR_ERR_INVALID_ARG, "block (%d,%d): null factor", I, J);
      if (k[b] == 2) {
        if (!rank || !f1 || !f1[b])
          return fail(ctx, CLR_ERR_INVALID_ARG, "block (%d,%d): low-rank block needs rank and V", I, J);
        r[b] = rank[b];
        const int64_t m = rs[I], n = cs[J];
        if (r[b] < 1 || (m + n) * r[b] > m * n)
          return fail(ctx, CLR_ERR_CAPACITY, "block (%d,%d): rank %d does not fit the %lldx%lld slot",
                      I, J, r[b], (long long)m, (long long)n);
        p1[b] = f1[b];
      } else {
        r[b] = std::min(rs[I], cs[J]);
      }
    }
  // packed: every block takes what it stores
  std::vector<int64_t> offs(nb, 0);
  int64_t cap = 0;
  for (int I = 0; I < nrb; ++I)
    for (int J = 0; J < ncb; ++J) {
      const size_t b = (size_t)I * ncb + J;
      offs[b] = cap;
      cap += stored_size(k[b], rs[I], cs[J], r[b]);
    }
  clr_matrix* m = nullptr;
  clr_status s = alloc_matrix(ctx, rs, cs, &m, &offs, cap);
  if (s != CLR_OK) return s;
  std::vector<const double*> tab(2 * nb);
  std::copy(p0.begin(), p0.end(), tab.begin());
  std::copy(p1.begin(), p1.end(), tab.begin() + nb);
  hipError_t e = hipMemcpyAsync(m->d_kind, k.data(), nb * sizeof(int), hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(m->d_rank, r.data(), nb * sizeof(int), hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess) e = ensure(ctx->ptrs, tab.size() * sizeof(double*));
  if (e == hipSuccess)
    e = hipMemcpyAsync(ctx->ptrs.p, tab.data(), tab.size() * sizeof(double*), hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess) {
    const double* const* d0 = as<const double*>(ctx->ptrs);
    e = launch_ingest(m->view(), m->arena, d0, d0 + nb, m->d_norm, ctx->stream);
  }
  std::vector<double> got(nb);
  if (e == hipSuccess)
    e = hipMemcpyAsync(got.data(), m->d_norm, nb * sizeof(double), hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) {
    free_matrix(m);
    return fail(ctx, CLR_ERR_HIP, "clr_create: %s", hipGetErrorString(e));
  }
  for (size_t b = 0; b < nb; ++b) {
    if (!std::isfinite(got[b])) {
      free_matrix(m);
      return fail(ctx, CLR_ERR_NONFINITE, "block %zu has a non-finite norm", b);
    }
    if (norms && k[b] != 0) {
      const double ref = norms[b];
      if (!(fabs(ref - got[b]) <= 1e-10 * std::max(fabs(got[b]), 1e-300))) {
        free_matrix(m);
        return fail(ctx, CLR_ERR_NORM_MISMATCH, "block %zu: norm %.17g given, %.17g computed", b,
                    ref, got[b]);
      }
    }
  }
  *out = m;
  return CLR_OK;
}

// Recompression of every block of a dense matrix (compression of an input).
extern "C" clr_status clr_compress(clr_context* ctx, const double* dense, int64_t ld, int nrb,
                                   const int* row_sizes, int ncb, const int* col_sizes,
                                   double tol, double drop, clr_matrix** out) {
  if (!ctx || !out) return CLR_ERR_INVALID_ARG;
  *out = nullptr;
  if (!dense || nrb < 1 || ncb < 1 || !row_sizes || !col_sizes)
    return fail(ctx, CLR_ERR_INVALID_ARG, "clr_compress: missing input");
  if (!(tol >= 0.0 && tol < 1.0) || !(drop >= 0.0))
    return fail(ctx, CLR_ERR_INVALID_ARG, "clr_compress: bad tol or drop");
  std::vector<int> rs(row_sizes, row_sizes + nrb), cs(col_sizes, col_sizes + ncb);
  clr_matrix* m = nullptr;
  clr_status s = alloc_matrix(ctx, rs, cs, &m);
  if (s != CLR_OK) return s;
  if (ld < m->rows) {
    free_matrix(m);
    return fail(ctx, CLR_ERR_INVALID_ARG, "clr_compress: ld < rows");
  }
  const bool square = m->square_blocked();
  std::vector<RecItem> items;
  int64_t scratch_total = 0;
  std::vector<int64_t> scratch_off;
  for (int I = 0; I < nrb; ++I)
    for (int J = 0; J < ncb; ++J) {
      RecItem r{};
      r.path = (square && I == J) ? kPathForceDense : kPathDense;
      r.cert_hint = 1;
      r.rrqr = ctx->compress_rrqr;
      r.m = rs[I];
      r.n = cs[J];
      r.R = 0;
      r.D = dense + m->roff[I] + (int64_t)m->coff[J] * ld;
      r.ldd = ld;
      r.tau = drop;
      r.out = m->arena + m->boff[(size_t)I * ncb + J];   // dense slots until compacted
      const int64_t need = rec_scratch_doubles(r.path, r.m, r.n, 0, tol);
      scratch_off.push_back(need > 0 ? scratch_total : -1);
      scratch_total += need;
      const size_t b = (size_t)I * ncb + J;
      r.kind_out = m->d_kind + b;
      r.rank_out = m->d_rank + b;
      r.norm_out = m->d_norm + b;
      items.push_back(r);
    }
  hipError_t e = ensure(ctx->w.scratch, sizeof(double) * std::max<int64_t>(scratch_total, 1));
  if (e != hipSuccess) {
    free_matrix(m);
    return fail(ctx, CLR_ERR_HIP, "scratch allocation: %s", hipGetErrorString(e));
  }
  for (size_t i = 0; i < items.size(); ++i)
    items[i].scratch = scratch_off[i] >= 0 ? as<double>(ctx->w.scratch) + scratch_off[i] : nullptr;
  s = upload(ctx, ctx->w.rec, items);
  if (s != CLR_OK) {
    free_matrix(m);
    return s;
  }
  e = launch_recompress_ctx(ctx, as<RecItem>(ctx->w.rec), nullptr, (int)items.size(), tol);
  if (e != hipSuccess) {
    free_matrix(m);
    return fail(ctx, CLR_ERR_HIP, "recompress launch: %s", hipGetErrorString(e));
  }
  s = check_status(ctx);
  // the result is packed: memory follows the ranks found
  if (s == CLR_OK) s = compact_matrix(ctx, m);
  if (s != CLR_OK) {
    free_matrix(m);
    return s;
  }
  *out = m;
  return CLR_OK;
}

extern "C" clr_status clr_destroy(clr_matrix* m) {
  if (!m) return CLR_ERR_INVALID_ARG;
  (void)hipStreamSynchronize(m->ctx->stream);
  free_matrix(m);
  return CLR_OK;
}

extern "C" clr_status clr_matrix_arena(const clr_matrix* m, int64_t* capacity, size_t* bytes) {
  if (!m) return CLR_ERR_INVALID_ARG;
  if (capacity) *capacity = m->cap;
  if (bytes) *bytes = m->block_bytes;
  return CLR_OK;
}

extern "C" clr_status clr_compact(clr_context* ctx, clr_matrix* m) {
  if (!ctx || !m) return CLR_ERR_INVALID_ARG;
  if (m->ctx != ctx) return fail(ctx, CLR_ERR_INVALID_ARG, "clr_compact: matrix of another context");
  return compact_matrix(ctx, m);
}

extern "C" clr_status clr_matrix_info(const clr_matrix* m, int* nrb, int* ncb, int64_t* rows,
                                      int64_t* cols, int64_t* stored) {
  if (!m) return CLR_ERR_INVALID_ARG;
  if (nrb) *nrb = m->nrb;
  if (ncb) *ncb = m->ncb;
  if (rows) *rows = m->rows;
  if (cols) *cols = m->cols;
  if (stored) {
    HostMeta h;
    clr_status s = fetch_meta(m->ctx, m, h);
    if (s != CLR_OK) return s;
    *stored = (int64_t)stored_elements(m, h);
  }
  return CLR_OK;
}

extern "C" clr_status clr_get_meta(clr_context* ctx, const clr_matrix* m, int8_t* kind, int* rank,
                                   double* norms) {
  if (!ctx || !m) return CLR_ERR_INVALID_ARG;
  HostMeta h;
  clr_status s = fetch_meta(ctx, m, h);
  if (s != CLR_OK) return s;
  const size_t nb = (size_t)m->nrb * m->ncb;
  for (size_t b = 0; b < nb; ++b) {
    if (kind) kind[b] = (int8_t)h.kind[b];
    if (rank) rank[b] = h.kind[b] == 0 ? 0 : h.rank[b];
    if (norms) norms[b] = h.norm[b];
  }
  return CLR_OK;
}

extern "C" clr_status clr_get_block(clr_context* ctx, const clr_matrix* m, int I, int J,
                                    double* f0, double* f1) {
  if (!ctx || !m || !f0) return CLR_ERR_INVALID_ARG;
  if (I < 0 || J < 0 || I >= m->nrb || J >= m->ncb)
    return fail(ctx, CLR_ERR_INVALID_ARG, "block index out of range");
  const size_t b = (size_t)I * m->ncb + J;
  int k = 0, r = 0;
  int64_t at = m->host_boff ? m->boff[b] : 0;
  HIP_TRY(ctx, hipMemcpyAsync(&k, m->d_kind + b, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
  HIP_TRY(ctx, hipMemcpyAsync(&r, m->d_rank + b, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
  if (!m->host_boff)
    HIP_TRY(ctx, hipMemcpyAsync(&at, m->d_boff + b, sizeof(int64_t), hipMemcpyDeviceToHost, ctx->stream));
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  const int64_t rows = m->rs[I], cols = m->cs[J];
  const double* src = m->arena + at;
  if (k == 0) return fail(ctx, CLR_ERR_INVALID_ARG, "block (%d,%d) is zero", I, J);
  if (k == 1) {
    HIP_TRY(ctx, hipMemcpyAsync(f0, src, sizeof(double) * rows * cols, hipMemcpyDeviceToDevice, ctx->stream));
  } else {
    if (!f1) return fail(ctx, CLR_ERR_INVALID_ARG, "low-rank block needs f1");
    HIP_TRY(ctx, hipMemcpyAsync(f0, src, sizeof(double) * rows * r, hipMemcpyDeviceToDevice, ctx->stream));
    HIP_TRY(ctx, hipMemcpyAsync(f1, src + rows * r, sizeof(double) * cols * r, hipMemcpyDeviceToDevice, ctx->stream));
  }
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  return CLR_OK;
}

extern "C" clr_status clr_to_dense(clr_context* ctx, const clr_matrix* m, double* out, int64_t ld) {
  if (!ctx || !m || !out) return CLR_ERR_INVALID_ARG;
  if (ld < m->rows) return fail(ctx, CLR_ERR_INVALID_ARG, "ld < rows");
  HIP_TRY(ctx, launch_to_dense(m->view(), out, ld, ctx->stream));
  return CLR_OK;
}

// ---------------------------------------------------------------------------
// The product
// ---------------------------------------------------------------------------

namespace {

// The product C = alpha A B with workspace W.  C is a new matrix, or Cinto
// (same blocking) rewritten in place.  With dev, the work lists have the
// capacities dev->caps and their lengths stay on the device: no host
// read-back, allocation or synchronisation, so the call can be recorded into
// a graph (W must already hold the capacities; statistics and the status
// word are then read by the caller after the run).
clr_status gemm_impl(clr_context* ctx, Work& W, const clr_matrix* A, const clr_matrix* B,
                     const clr_gemm_opts* o, clr_matrix** Cout, clr_gemm_stats* st,
                     const clr_matrix* mask = nullptr, clr_matrix* Cinto = nullptr,
                     const DevRun* dev = nullptr) {
  *Cout = nullptr;
  if (A->cs != B->rs)
    return fail(ctx, CLR_ERR_SHAPE, "column blocking of A differs from row blocking of B");
  if (dev && (st || o->precision == CLR_OZAKI || !Cinto))
    return fail(ctx, CLR_ERR_INVALID_ARG, "device-sized product: in place, FP64 or mixed, no statistics");
  // the output: Cinto, or allocated once the symbolic phase has sized its room
  clr_matrix* C = Cinto;
  if (C) {
    if (C->rs != A->rs || C->cs != B->cs)
      return fail(ctx, CLR_ERR_SHAPE, "output blocking differs from the product's");
    HIP_TRY(ctx, reset_meta(ctx, C));
  }
  auto bail = [&](clr_status code) {
    if (!Cinto && C) free_matrix(C);
    return code;
  };
  hipStream_t stream = ctx->stream;
  PlanParams P{};
  P.A = A->view();
  P.B = B->view();
  P.nrb = A->nrb;
  P.ncb = B->ncb;
  P.nkb = A->ncb;
  P.eps_sp = o->eps_sp;
  P.screen = o->screen;
  P.alpha = o->alpha;
  P.tol = o->tol;
  P.square = (A->rs == B->cs) ? 1 : 0;
  P.edges = edge_table(ctx, o);
  P.mask_kind = mask ? mask->d_kind : nullptr;
  const int64_t npairs = (int64_t)P.nrb * P.ncb;
  const int64_t list_ints = block_list_ints(P.nrb, P.ncb, P.nkb);
  hipError_t e = hipSuccess;
  if (dev) {
    if (!work_fits(W, work_sizes(npairs, dev->caps, list_ints)))
      return bail(fail(ctx, CLR_ERR_CAPACITY, "workspace smaller than the run's capacities"));
  } else {
    if (e == hipSuccess) e = ensure(W.lists, sizeof(int) * list_ints);
    if (e == hipSuccess) e = ensure(W.cnt, sizeof(int64_t) * kNumCounters * npairs);
    if (e == hipSuccess) e = ensure(W.off, sizeof(int64_t) * kNumCounters * npairs);
    if (e == hipSuccess) e = ensure(W.st, sizeof(double) * kNumStats * npairs);
    if (e == hipSuccess) e = ensure(W.flags, sizeof(int) * npairs);
    if (e == hipSuccess) e = ensure(W.totals, sizeof(int64_t) * kNumCounters + sizeof(double) * kNumStats);
    if (e != hipSuccess) {
      fail(ctx, CLR_ERR_HIP, "workspace: %s", hipGetErrorString(e));
      return bail(CLR_ERR_HIP);
    }
  }
  int64_t* tot_cnt = as<int64_t>(W.totals);
  double* tot_st = reinterpret_cast<double*>(tot_cnt + kNumCounters);
  if (!dev && e == hipSuccess) e = hipEventRecord(ctx->ev[0], stream);
  bind_block_lists(P, as<int>(W.lists));
  if (e == hipSuccess) e = launch_block_lists(P, as<int>(W.lists), stream);
  if (e == hipSuccess) e = launch_symbolic(P, as<int64_t>(W.cnt), as<double>(W.st), as<int>(W.flags), stream);
  if (e == hipSuccess) e = launch_scan(as<int64_t>(W.cnt), as<int64_t>(W.off), npairs, kNumCounters, tot_cnt, stream);
  // n[c]: length (eager) or capacity (device-sized) of list c; live: the
  // device-resident lengths of a device-sized run
  int64_t n[kNumCounters];
  double hs[kNumStats];
  int64_t* live = nullptr;
  if (dev) {
    live = as<int64_t>(W.live);
    Caps caps = dev->caps;
    caps.c[kCntOut] = C->cap;   // the output's arena bounds its room
    if (e == hipSuccess) e = launch_caps(tot_cnt, caps, live, stream);
    if (e == hipSuccess) e = launch_reduce(as<double>(W.st), npairs, kNumStats, tot_st, stream);
    if (e == hipSuccess) e = launch_add_flops(tot_st, as<double>(W.flops), stream);
    for (int i = 0; i < kNumCounters; ++i) n[i] = caps.c[i];
  } else {
    if (e == hipSuccess) e = launch_reduce(as<double>(W.st), npairs, kNumStats, tot_st, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(n, tot_cnt, sizeof(n), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(hs, tot_st, sizeof(hs), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
  }
  if (e != hipSuccess) {
    fail(ctx, CLR_ERR_HIP, "symbolic phase: %s", hipGetErrorString(e));
    return bail(CLR_ERR_HIP);
  }
  for (int i = 0; i < kNumCounters; ++i)
    if (n[i] < 0 || (!counts_doubles(i) && n[i] > INT32_MAX))
      return bail(fail(ctx, CLR_ERR_CAPACITY, "work list %d too long (%lld)", i, (long long)n[i]));
  if (!dev) {
    for (int i = 0; i < kNumCounters; ++i) W.seen.c[i] = std::max(W.seen.c[i], n[i]);
    W.host_flops += hs[kStFlopsDD] + hs[kStFlopsLD] + hs[kStFlopsDL] + hs[kStFlopsLL] +
                    hs[kStFlopsDensify];
    if (C) {
      if (n[kCntOut] > C->cap)
        return bail(fail(ctx, CLR_ERR_CAPACITY, "output arena of %lld doubles, %lld needed",
                         (long long)C->cap, (long long)n[kCntOut]));
    } else {
      clr_status s = alloc_matrix(ctx, A->rs, B->cs, &C, nullptr, n[kCntOut]);
      if (s != CLR_OK) return s;
    }
    Caps exact;
    for (int i = 0; i < kNumCounters; ++i) exact.c[i] = n[i];
    e = reserve_work(W, work_sizes(npairs, exact));
    if (e == hipSuccess) e = ensure(W.order_thin, sizeof(int) * n[kCntThin1]);
    if (e == hipSuccess) e = ensure(W.sortw, operand_order_bytes((int)n[kCntThin1]));
    if (e != hipSuccess) {
      fail(ctx, CLR_ERR_HIP, "work lists: %s", hipGetErrorString(e));
      return bail(CLR_ERR_HIP);
    }
  }
  auto lv = [&](int c) { return live ? live + c : nullptr; };
  FillParams F{};
  F.off = as<int64_t>(W.off);
  F.cnt = as<int64_t>(W.cnt);
  F.flags = as<int>(W.flags);
  F.seg_dense = as<Seg>(W.seg_dense);
  F.items_dense = as<GemmItem>(W.items_dense);
  F.seg_thin1 = as<Seg>(W.seg_thin1);
  F.items_thin1 = as<GemmItem>(W.items_thin1);
  F.seg_thin2 = as<Seg>(W.seg_thin2);
  F.items_thin2 = as<GemmItem>(W.items_thin2);
  F.pieces = as<Piece>(W.pieces);
  F.rec = as<RecItem>(W.rec);
  F.pool = as<double>(W.pool);
  F.scratch = as<double>(W.scratch);
  F.acc = as<double>(W.acc);
  F.c_arena = C->arena;
  F.c_boff = C->d_boff;
  F.c_kind = C->d_kind;
  F.c_rank = C->d_rank;
  F.c_norm = C->d_norm;
  F.abort = lv(kLiveOverflow);
  // the offsets are planned on the device from here on (the host copy is stale)
  C->host_boff = false;
  // The operand-grouped order of the factor products only improves L2 reuse
  // (each item is computed on its own).  A device-sized run groups them with
  // the hashed counting sort, which a graph can record.
  const int* order_thin = as<int>(W.order_thin);
  if (e == hipSuccess) e = launch_fill(P, F, stream);
  if (e == hipSuccess)
    e = launch_item_order(F.items_dense, (int)n[kCntGemmItems], as<int>(W.order), stream,
                          lv(kCntGemmItems));
  if (e == hipSuccess && !dev)
    e = launch_operand_order(F.items_thin1, F.seg_thin1, (int)n[kCntThin1], W.sortw.p,
                             as<int>(W.order_thin), stream);
  if (e == hipSuccess && dev)
    e = launch_operand_group(F.items_thin1, F.seg_thin1, (int)n[kCntThin1], as<int>(W.order_thin),
                             stream, lv(kCntThin1));
  if (e == hipSuccess && !dev) e = hipEventRecord(ctx->ev[1], stream);
  if (e == hipSuccess)
    e = run_wgemm(o, F.items_thin1, F.seg_thin1, (int)n[kCntThin1], stream, order_thin,
                  lv(kCntThin1));
  if (e == hipSuccess)
    e = run_wgemm(o, F.items_thin2, F.seg_thin2, (int)n[kCntThin2], stream, nullptr, lv(kCntThin2));
  if (e == hipSuccess && !dev) e = hipEventRecord(ctx->ev[6], stream);
  if (e == hipSuccess)
    e = run_dense(o, F.items_dense, F.seg_dense, (int)n[kCntGemmItems], as<int>(W.order), stream,
                  lv(kCntGemmItems));
  if (e == hipSuccess && !dev) e = hipEventRecord(ctx->ev[2], stream);
  if (e == hipSuccess)
    e = launch_recompress_work(ctx, W, F.rec, F.pieces, (int)n[kCntComputed], o->tol,
                               st != nullptr, lv(kCntComputed));
  if (e == hipSuccess && !dev) e = hipEventRecord(ctx->ev[3], stream);
  if (e != hipSuccess) {
    fail(ctx, CLR_ERR_HIP, "product launch: %s", hipGetErrorString(e));
    return bail(CLR_ERR_HIP);
  }
  if (dev) {
    *Cout = C;
    return CLR_OK;
  }
  clr_status s = check_status(ctx);
  if (s != CLR_OK) return bail(s);
  if (st) {
    const int64_t* hc = n;
    memset(st, 0, sizeof(*st));
    st->candidates = (int64_t)hs[kStCandidate];
    st->computed = hc[kCntComputed];
    st->n_dd = (int64_t)hs[kStNDD];
    st->n_ld = (int64_t)hs[kStNLD];
    st->n_dl = (int64_t)hs[kStNDL];
    st->n_ll = (int64_t)hs[kStNLL];
    st->triples = st->n_dd + st->n_ld + st->n_dl + st->n_ll;
    st->flops_dd = hs[kStFlopsDD];
    st->flops_ld = hs[kStFlopsLD];
    st->flops_dl = hs[kStFlopsDL];
    st->flops_ll = hs[kStFlopsLL];
    st->flops_densify = hs[kStFlopsDensify];
    st->flops_products = st->flops_dd + st->flops_ld + st->flops_dl + st->flops_ll + st->flops_densify;
    st->ms_symbolic = elapsed(ctx->ev[0], ctx->ev[1]);
    st->ms_products = elapsed(ctx->ev[1], ctx->ev[2]);
    st->ms_recompress = elapsed(ctx->ev[2], ctx->ev[3]);
    st->ms_total = elapsed(ctx->ev[0], ctx->ev[3]);
    st->ms_thin = elapsed(ctx->ev[1], ctx->ev[6]);
    st->ms_dense = elapsed(ctx->ev[6], ctx->ev[2]);
    st->ms_rec_engine = hc[kCntComputed] > 0 ? elapsed(ctx->ev[8], ctx->ev[9]) : 0.0;
    if (hc[kCntComputed] > 0) {
      RecCounters rc;
      HIP_TRY(ctx, hipMemcpy(&rc, rec_work(W.recg.p, hc[kCntComputed]).ctr, sizeof(rc),
                             hipMemcpyDeviceToHost));
      st->flops_rec_engine = rc.flops_bidiag;
      st->certified_dense = (int64_t)rc.certified;
    }
    HostMeta ha, hb, hcm;
    if ((s = fetch_meta(ctx, A, ha)) != CLR_OK) return bail(s);
    if ((s = fetch_meta(ctx, B, hb)) != CLR_OK) return bail(s);
    if ((s = fetch_meta(ctx, C, hcm)) != CLR_OK) return bail(s);
    st->bytes_compulsory = 8.0 * (stored_elements(A, ha) + stored_elements(B, hb) + stored_elements(C, hcm));
    std::vector<int> fl(npairs);
    HIP_TRY(ctx, hipMemcpy(fl.data(), W.flags.p, sizeof(int) * npairs, hipMemcpyDeviceToHost));
    for (int64_t b = 0; b < npairs; ++b) {
      if (!(fl[b] & kFlagComputed)) continue;
      if (fl[b] & kFlagDensify) st->densified++;
      if (hcm.kind[b] == 0) st->dropped++;
      if (hcm.kind[b] == 1) st->out_dense++;
      if (hcm.kind[b] == 2) st->out_lowrank++;
    }
  }
  *Cout = C;
  return CLR_OK;
}

}  // namespace

extern "C" clr_status clr_gemm(clr_context* ctx, const clr_matrix* A, const clr_matrix* B,
                               const clr_gemm_opts* opts, clr_matrix** C, clr_gemm_stats* st) {
  if (!ctx || !A || !B || !C) return CLR_ERR_INVALID_ARG;
  *C = nullptr;
  clr_status s = check_opts(ctx, opts);
  if (s != CLR_OK) return s;
  return gemm_impl(ctx, ctx->w, A, B, opts, C, st);
}

// ---------------------------------------------------------------------------
// Tile edges of the grouped GEMM and their autotuner
// ---------------------------------------------------------------------------

extern "C" clr_status clr_set_tile_edges(clr_context* ctx, int precision, int dense_edge,
                                         int thin_edge) {
  if (!ctx) return CLR_ERR_INVALID_ARG;
  if (precision != CLR_FP64 && precision != CLR_MIXED)
    return fail(ctx, CLR_ERR_INVALID_ARG, "bad precision");
  const int top = precision == CLR_MIXED ? kMaxItemF32 : kMaxItemF64;
  if (dense_edge != 0 && (dense_edge < 16 || dense_edge > top || dense_edge % 16 != 0))
    return fail(ctx, CLR_ERR_INVALID_ARG, "dense tile edge %d: 0 or a multiple of 16 in [16, %d]",
                dense_edge, top);
  if (thin_edge != 0 && (thin_edge < 16 || thin_edge > kMaxItemThin || thin_edge % 16 != 0))
    return fail(ctx, CLR_ERR_INVALID_ARG, "thin tile edge %d: 0 or a multiple of 16 in [16, %d]",
                thin_edge, kMaxItemThin);
  EdgeTable& t = ctx->tiles[precision == CLR_MIXED ? 1 : 0];
  for (int c = 0; c < kDenseClasses; ++c) t.dense[c] = dense_edge;
  for (int c = 0; c < kThinClasses; ++c) t.thin[c] = thin_edge;
  return CLR_OK;
}

extern "C" clr_status clr_set_tile_classes(clr_context* ctx, int precision, const int* dense_edges,
                                           const int* thin_edges) {
  if (!ctx || !dense_edges || !thin_edges) return CLR_ERR_INVALID_ARG;
  if (precision != CLR_FP64 && precision != CLR_MIXED)
    return fail(ctx, CLR_ERR_INVALID_ARG, "bad precision");
  const int top = precision == CLR_MIXED ? kMaxItemF32 : kMaxItemF64;
  for (int c = 0; c < kDenseClasses; ++c) {
    const int v = dense_edges[c];
    if (v != 0 && (v < 16 || v > top || v % 16 != 0))
      return fail(ctx, CLR_ERR_INVALID_ARG, "dense class %d edge %d: 0 or a multiple of 16 in [16, %d]",
                  c, v, top);
  }
  for (int c = 0; c < kThinClasses; ++c) {
    const int v = thin_edges[c];
    if (v != 0 && (v < 16 || v > kMaxItemThin || v % 16 != 0))
      return fail(ctx, CLR_ERR_INVALID_ARG, "thin class %d edge %d: 0 or a multiple of 16 in [16, %d]",
                  c, v, kMaxItemThin);
  }
  EdgeTable& t = ctx->tiles[precision == CLR_MIXED ? 1 : 0];
  for (int c = 0; c < kDenseClasses; ++c) t.dense[c] = dense_edges[c];
  for (int c = 0; c < kThinClasses; ++c) t.thin[c] = thin_edges[c];
  return CLR_OK;
}

extern "C" clr_status clr_get_tile_classes(const clr_context* ctx, int precision, int* dense_edges,
                                           int* thin_edges) {
  if (!ctx || !dense_edges || !thin_edges) return CLR_ERR_INVALID_ARG;
  if (precision != CLR_FP64 && precision != CLR_MIXED) return CLR_ERR_INVALID_ARG;
  const EdgeTable& t = ctx->tiles[precision == CLR_MIXED ? 1 : 0];
  for (int c = 0; c < kDenseClasses; ++c) dense_edges[c] = t.dense[c];
  for (int c = 0; c < kThinClasses; ++c) thin_edges[c] = t.thin[c];
  return CLR_OK;
}

// Dense certificate (a proof from the Gram matrix that a dense-accumulated
// block keeps more than half its rank, Sec. 4.1 rank rule) before the SVD.
extern "C" clr_status clr_set_dense_certificate(clr_context* ctx, int enable) {
  if (!ctx) return CLR_ERR_INVALID_ARG;
  ctx->dense_cert = enable ? 1 : 0;
  return CLR_OK;
}

// Dense overlap-like or Coulomb-like kernel matrix on the device: the input
// that clr_compress turns into a CLR matrix.
extern "C" clr_status clr_kernel_matrix(clr_context* ctx, const double* row_points,
                                        int64_t nrows, const double* col_points, int64_t ncols,
                                        int dim, int kernel, double a, double diag, double* out,
                                        int64_t ld) {
  if (!ctx) return CLR_ERR_INVALID_ARG;
  if (!row_points || !col_points || !out) return fail(ctx, CLR_ERR_INVALID_ARG, "null pointer");
  if (nrows < 1 || ncols < 1 || ld < nrows)
    return fail(ctx, CLR_ERR_INVALID_ARG, "bad sizes (%lld x %lld, ld %lld)", (long long)nrows,
                (long long)ncols, (long long)ld);
  if ((ncols + 31) / 32 > 65535 || (nrows + 255) / 256 > INT32_MAX)
    return fail(ctx, CLR_ERR_CAPACITY, "kernel matrix too large");
  if (dim < 1 || dim > 3) return fail(ctx, CLR_ERR_INVALID_ARG, "dim must be 1, 2 or 3");
  if (kernel != CLR_KERNEL_GAUSSIAN && kernel != CLR_KERNEL_COULOMB)
    return fail(ctx, CLR_ERR_INVALID_ARG, "kernel %d", kernel);
  if (!std::isfinite(a) || !std::isfinite(diag) || a < 0.0 ||
      (kernel == CLR_KERNEL_COULOMB && !(a > 0.0)))
    return fail(ctx, CLR_ERR_INVALID_ARG, "bad kernel parameters");
  HIP_TRY(ctx, launch_kernel_matrix(row_points, nrows, col_points, ncols, dim, kernel, a, diag,
                                    out, ld, ctx->stream));
  return CLR_OK;
}

// Measured FP64 MFMA rate and copy bandwidth (best of several timed runs).
extern "C" clr_status clr_measure_peaks(clr_context* ctx, double* mfma_f64_tflops,
                                        double* copy_gbps) {
  if (!ctx) return CLR_ERR_INVALID_ARG;
  int ncu = 0;
  HIP_TRY(ctx, hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, ctx->device));
  const int blocks = 4 * std::max(ncu, 1);   // 16 waves per CU: four per SIMD
  const int iters = 4096;
  const size_t bytes = (size_t)1 << 30;     // per buffer, far above L2 and the last-level cache
  double* buf = nullptr;
  HIP_TRY(ctx, hipMalloc(&buf, 2 * bytes + 256));
  auto run = [&]() -> clr_status {
    float best_mfma = 1e30f, best_copy = 1e30f;
    for (int rep = 0; rep < 4; ++rep) {
      HIP_TRY(ctx, hipEventRecord(ctx->ev[0], ctx->stream));
      HIP_TRY(ctx, launch_mfma_loop(blocks, iters, buf, ctx->stream));
      HIP_TRY(ctx, hipEventRecord(ctx->ev[1], ctx->stream));
      HIP_TRY(ctx, launch_copy(buf + 32, buf + 32 + bytes / 8, (int64_t)(bytes / 8), ctx->stream));
      HIP_TRY(ctx, hipEventRecord(ctx->ev[2], ctx->stream));
      HIP_TRY(ctx, hipEventSynchronize(ctx->ev[2]));
      if (rep == 0) continue;   // the first round warms up
      best_mfma = std::min(best_mfma, elapsed(ctx->ev[0], ctx->ev[1]));
      best_copy = std::min(best_copy, elapsed(ctx->ev[1], ctx->ev[2]));
    }
    if (mfma_f64_tflops) *mfma_f64_tflops = mfma_loop_flops(blocks, iters) / (best_mfma * 1e-3) / 1e12;
    if (copy_gbps) *copy_gbps = 2.0 * (double)bytes / (best_copy * 1e-3) / 1e9;
    return CLR_OK;
  };
  HIP_TRY(ctx, launch_fill_f64(buf, 0.0, (int64_t)((2 * bytes + 256) / 8), ctx->stream));
  const clr_status s = run();
  (void)hipStreamSynchronize(ctx->stream);
  (void)hipFree(buf);
  return s;
}

// Factorisation used by clr_compress (the paper builds its input blocks by
// rank-revealing QR, Sec. 4.1; products keep the truncated SVD).
extern "C" clr_status clr_set_compression(clr_context* ctx, int method) {
  if (!ctx) return CLR_ERR_INVALID_ARG;
  if (method != CLR_COMPRESS_SVD && method != CLR_COMPRESS_RRQR)
    return fail(ctx, CLR_ERR_INVALID_ARG, "compression method %d", method);
  ctx->compress_rrqr = method == CLR_COMPRESS_RRQR ? 1 : 0;
  return CLR_OK;
}

// Empirical choice, on the caller's own product, of the item edges of the
// dense-accumulation launch and of the factor-product launches: first one edge
// per launch class (every multiple of 32 up to the kernel's tile), then each
// shape class of items on its own (coordinate descent from that choice), each
// candidate timed on the product (best of two runs, device events around each
// launch class).  The numerical result does not depend on the edges: every
// output element is accumulated over the same inner sequence whatever the
// tiling.
extern "C" clr_status clr_autotune(clr_context* ctx, const clr_matrix* A, const clr_matrix* B,
                                   const clr_gemm_opts* opts, int* dense_edge, int* thin_edge,
                                   double* ms_dense, double* ms_thin) {
  if (!ctx || !A || !B) return CLR_ERR_INVALID_ARG;
  clr_status s = check_opts(ctx, opts);
  if (s != CLR_OK) return s;
  if (opts->precision == CLR_OZAKI)
    return fail(ctx, CLR_ERR_INVALID_ARG, "autotune covers the FP64 and MIXED forms");
  const int pi = opts->precision == CLR_MIXED ? 1 : 0;
  const int top = max_item(opts);
  EdgeTable& T = ctx->tiles[pi];
  const EdgeTable saved = T;
  // launch times of the product with the current table (best of two runs)
  auto measure = [&](double* td, double* tt) -> clr_status {
    *td = *tt = 1e300;
    for (int rep = 0; rep < 2; ++rep) {
      clr_matrix* C = nullptr;
      clr_gemm_stats st{};
      clr_status r = gemm_impl(ctx, ctx->w, A, B, opts, &C, &st);
      free_matrix(C);
      if (r != CLR_OK) return r;
      *td = std::min(*td, (double)st.ms_dense);
      *tt = std::min(*tt, (double)st.ms_thin);
    }
    return CLR_OK;
  };
  auto set_all = [&](int de, int te) {
    for (int c = 0; c < kDenseClasses; ++c) T.dense[c] = de;
    for (int c = 0; c < kThinClasses; ++c) T.thin[c] = te;
  };
  // 1. one edge per launch class: multiples of 32 up to the full tile
  double best_d = 1e300, best_t = 1e300;
  int arg_d = top, arg_t = std::min(top, kMaxItemThin);
  for (int edge = 32; edge <= top; edge += 32) {
    set_all(edge, std::min(edge, kMaxItemThin));
    double td, tt;
    if ((s = measure(&td, &tt)) != CLR_OK) {
      T = saved;
      return s;
    }
    if (td < best_d) {
      best_d = td;
      arg_d = edge;
    }
    if (tt < best_t) {
      best_t = tt;
      arg_t = std::min(edge, kMaxItemThin);
    }
  }
  set_all(arg_d, arg_t);
  // 2. per shape class, one class at a time from that choice: an edge is kept
  // only if it shortens its launch by more than 2 % (classes absent from the
  // product change nothing and keep the launch-class edge)
  for (int c = 0; c < kDenseClasses; ++c) {
    const int cur = T.dense[c];
    int best = cur;
    double bt = best_d;
    for (int edge = 32; edge <= top; edge += 32) {
      if (edge == cur) continue;
      T.dense[c] = edge;
      double td, tt;
      if ((s = measure(&td, &tt)) != CLR_OK) {
        T = saved;
        return s;
      }
      if (td < 0.98 * bt) {
        bt = td;
        best = edge;
      }
    }
    T.dense[c] = best;
    best_d = bt;
  }
  for (int c = 0; c < kThinClasses; ++c) {
    const int cur = T.thin[c];
    int best = cur;
    double bt = best_t;
    for (int edge = 16; edge <= kMaxItemThin; edge += 16) {
      if (edge == cur) continue;
      T.thin[c] = edge;
      double td, tt;
      if ((s = measure(&td, &tt)) != CLR_OK) {
        T = saved;
        return s;
      }
      if (tt < 0.98 * bt) {
        bt = tt;
        best = edge;
      }
    }
    T.thin[c] = best;
    best_t = bt;
  }
  if (dense_edge) *dense_edge = arg_d;
  if (thin_edge) *thin_edge = arg_t;
  if (ms_dense) *ms_dense = best_d;
  if (ms_thin) *ms_thin = best_t;
  return CLR_OK;
}

// ---------------------------------------------------------------------------
// Batches of products: one plan, one launch per phase for the whole batch
// ---------------------------------------------------------------------------

struct clr_plan {
  clr_context* ctx = nullptr;
  int nprod = 0;
  clr_gemm_opts o{};
  std::vector<const clr_matrix*> A, B;
  std::vector<clr_matrix*> C;
  // execution buffers owned by the plan (a captured graph keeps their addresses)
  DevBuf seg_dense, items_dense, seg_thin1, items_thin1, seg_thin2, items_thin2, pieces, rec,
      pool, scratch, acc, recg, status, bases, order, order_thin;
  int64_t n_thin1 = 0, n_thin2 = 0, n_dense = 0, n_rec = 0;
  int dense_cert = 1;
  double flops[kNumStats] = {};
  int64_t counts[kNumCounters] = {};
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

void plan_free(clr_plan* pl) {
  if (!pl) return;
  if (pl->exec) (void)hipGraphExecDestroy(pl->exec);
  if (pl->graph) (void)hipGraphDestroy(pl->graph);
  for (DevBuf* b : {&pl->seg_dense, &pl->items_dense, &pl->seg_thin1, &pl->items_thin1,
                    &pl->seg_thin2, &pl->items_thin2, &pl->pieces, &pl->rec, &pl->pool,
                    &pl->scratch, &pl->acc, &pl->recg, &pl->status, &pl->bases, &pl->order,
                    &pl->order_thin})
    free_buf(*b);
  delete pl;
}

// The execution phase of a planned batch: factor products, dense accumulation,
// recompression (with its output products).  Only kernel launches on the
// context stream, so it can be recorded into a graph.
hipError_t plan_launch(clr_plan* pl, hipStream_t s) {
  const clr_gemm_opts* o = &pl->o;
  hipError_t e = run_wgemm(o, as<GemmItem>(pl->items_thin1), as<Seg>(pl->seg_thin1),
                           (int)pl->n_thin1, s, as<int>(pl->order_thin));
  if (e == hipSuccess)
    e = run_wgemm(o, as<GemmItem>(pl->items_thin2), as<Seg>(pl->seg_thin2), (int)pl->n_thin2, s);
  if (e == hipSuccess)
    e = run_dense(o, as<GemmItem>(pl->items_dense), as<Seg>(pl->seg_dense), (int)pl->n_dense,
                  as<int>(pl->order), s, nullptr);
  if (e == hipSuccess && pl->n_rec > 0) {
    const RecWork w = rec_work(pl->recg.p, pl->n_rec);
    e = launch_recompress(as<RecItem>(pl->rec), as<Piece>(pl->pieces), (int)pl->n_rec, o->tol,
                          as<int>(pl->status), w.gi, w.gs, w.order,
                          pl->dense_cert ? w.cert : nullptr, w.ctr, s);
  }
  return e;
}

clr_status plan_status(clr_context* ctx, clr_plan* pl) {
  int h = 0;
  HIP_TRY(ctx, hipMemcpyAsync(&h, pl->status.p, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  if (h == 0) return CLR_OK;
  HIP_TRY(ctx, launch_fill_i32(as<int>(pl->status), 0, 1, ctx->stream));
  if (h & 2) return fail(ctx, CLR_ERR_NONFINITE, "non-finite block norm");
  if (h & (4 | 8)) return fail(ctx, CLR_ERR_INTERNAL, "recompression working set mis-planned");
  return fail(ctx, CLR_ERR_INTERNAL, "Jacobi SVD did not converge");
}

// Screening and work lists of every product (device symbolic phase per product,
// one read-back of all totals), output matrices, and the filled lists.
clr_status plan_build(clr_context* ctx, clr_plan* pl) {
  const int np = pl->nprod;
  hipStream_t stream = ctx->stream;
  std::vector<PlanParams> P(np);
  std::vector<int64_t> pb(np + 1, 0);
  pl->C.assign(np, nullptr);
  for (int p = 0; p < np; ++p) {
    const clr_matrix* A = pl->A[p];
    const clr_matrix* B = pl->B[p];
    if (A->cs != B->rs)
      return fail(ctx, CLR_ERR_SHAPE, "product %d: column blocking of A differs from row blocking of B", p);
    PlanParams& q = P[p];
    q = PlanParams{};
    q.A = A->view();
    q.B = B->view();
    q.nrb = A->nrb;
    q.ncb = B->ncb;
    q.nkb = A->ncb;
    q.eps_sp = pl->o.eps_sp;
    q.screen = pl->o.screen;
    q.alpha = pl->o.alpha;
    q.tol = pl->o.tol;
    q.square = (A->rs == B->cs) ? 1 : 0;
    q.edges = edge_table(ctx, &pl->o);
    q.mask_kind = nullptr;
    pb[p + 1] = pb[p] + (int64_t)q.nrb * q.ncb;
  }
  const int64_t tp = pb[np];
  // every product's block lists (read by its symbolic and fill kernels)
  std::vector<int64_t> lb(np + 1, 0);
  for (int p = 0; p < np; ++p) lb[p + 1] = lb[p] + block_list_ints(P[p].nrb, P[p].ncb, P[p].nkb);
  HIP_TRY(ctx, ensure(ctx->w.lists, sizeof(int) * lb[np]));
  for (int p = 0; p < np; ++p) bind_block_lists(P[p], as<int>(ctx->w.lists) + lb[p]);
  const size_t tot_bytes = (size_t)np * (sizeof(int64_t) * kNumCounters + sizeof(double) * kNumStats);
  HIP_TRY(ctx, ensure(ctx->w.cnt, sizeof(int64_t) * kNumCounters * tp));
  HIP_TRY(ctx, ensure(ctx->w.off, sizeof(int64_t) * kNumCounters * tp));
  HIP_TRY(ctx, ensure(ctx->w.st, sizeof(double) * kNumStats * tp));
  HIP_TRY(ctx, ensure(ctx->w.flags, sizeof(int) * tp));
  HIP_TRY(ctx, ensure(ctx->w.totals, tot_bytes));
  int64_t* tc = as<int64_t>(ctx->w.totals);
  double* ts = reinterpret_cast<double*>(tc + (size_t)np * kNumCounters);
  for (int p = 0; p < np; ++p) {
    const int64_t npairs = pb[p + 1] - pb[p];
    int64_t* cnt = as<int64_t>(ctx->w.cnt) + kNumCounters * pb[p];
    int64_t* off = as<int64_t>(ctx->w.off) + kNumCounters * pb[p];
    double* st = as<double>(ctx->w.st) + kNumStats * pb[p];
    HIP_TRY(ctx, launch_block_lists(P[p], as<int>(ctx->w.lists) + lb[p], stream));
    HIP_TRY(ctx, launch_symbolic(P[p], cnt, st, as<int>(ctx->w.flags) + pb[p], stream));
    HIP_TRY(ctx, launch_scan(cnt, off, npairs, kNumCounters, tc + (size_t)p * kNumCounters, stream));
    HIP_TRY(ctx, launch_reduce(st, npairs, kNumStats, ts + (size_t)p * kNumStats, stream));
  }
  std::vector<int64_t> hc((size_t)np * kNumCounters);
  std::vector<double> hs((size_t)np * kNumStats);
  HIP_TRY(ctx, hipMemcpyAsync(hc.data(), tc, sizeof(int64_t) * hc.size(), hipMemcpyDeviceToHost, stream));
  HIP_TRY(ctx, hipMemcpyAsync(hs.data(), ts, sizeof(double) * hs.size(), hipMemcpyDeviceToHost, stream));
  HIP_TRY(ctx, hipStreamSynchronize(stream));
  // place of every product in the concatenated lists (the output room is
  // per product: each output has an arena of its own)
  std::vector<int64_t> base((size_t)np * kNumCounters);
  int64_t sum[kNumCounters] = {};
  for (int p = 0; p < np; ++p)
    for (int c = 0; c < kNumCounters; ++c) {
      const int64_t v = hc[(size_t)p * kNumCounters + c];
      if (v < 0) return fail(ctx, CLR_ERR_INTERNAL, "negative work count");
      base[(size_t)p * kNumCounters + c] = c == kCntOut ? 0 : sum[c];
      sum[c] += v;
    }
  for (int c = 0; c < kNumCounters; ++c) {
    if (!counts_doubles(c) && sum[c] > INT32_MAX)
      return fail(ctx, CLR_ERR_CAPACITY, "batch work list %d too long (%lld)", c, (long long)sum[c]);
    pl->counts[c] = sum[c];
  }
  for (int p = 0; p < np; ++p) {
    clr_status s = alloc_matrix(ctx, pl->A[p]->rs, pl->B[p]->cs, &pl->C[p], nullptr,
                                hc[(size_t)p * kNumCounters + kCntOut]);
    if (s != CLR_OK) return s;
  }
  for (int p = 0; p < np; ++p)
    for (int k = 0; k < kNumStats; ++k) pl->flops[k] += hs[(size_t)p * kNumStats + k];
  pl->n_thin1 = sum[kCntThin1];
  pl->n_thin2 = sum[kCntThin2];
  pl->n_dense = sum[kCntGemmItems];
  pl->n_rec = sum[kCntComputed];
  hipError_t e = hipSuccess;
  if (e == hipSuccess) e = ensure(pl->seg_dense, sizeof(Seg) * sum[kCntSegDense]);
  if (e == hipSuccess) e = ensure(pl->items_dense, sizeof(GemmItem) * sum[kCntGemmItems]);
  if (e == hipSuccess) e = ensure(pl->order, sizeof(int) * (sum[kCntGemmItems] + 1));
  if (e == hipSuccess) e = ensure(pl->seg_thin1, sizeof(Seg) * sum[kCntThin1]);
  if (e == hipSuccess) e = ensure(pl->items_thin1, sizeof(GemmItem) * sum[kCntThin1]);
  if (e == hipSuccess) e = ensure(pl->seg_thin2, sizeof(Seg) * sum[kCntThin2]);
  if (e == hipSuccess) e = ensure(pl->items_thin2, sizeof(GemmItem) * sum[kCntThin2]);
  if (e == hipSuccess) e = ensure(pl->pieces, sizeof(Piece) * sum[kCntPieces]);
  if (e == hipSuccess) e = ensure(pl->rec, sizeof(RecItem) * sum[kCntComputed]);
  if (e == hipSuccess) e = ensure(pl->pool, sizeof(double) * sum[kCntPool]);
  if (e == hipSuccess) e = ensure(pl->scratch, sizeof(double) * sum[kCntScratch]);
  if (e == hipSuccess && sum[kCntAcc] > 0) e = ensure(pl->acc, sizeof(double) * (size_t)sum[kCntAcc]);
  if (e == hipSuccess) e = ensure(pl->recg, rec_work_bytes(sum[kCntComputed]));
  if (e == hipSuccess) e = ensure(pl->status, sizeof(int));
  if (e == hipSuccess) e = launch_fill_i32(as<int>(pl->status), 0, 1, stream);
  if (e != hipSuccess) return fail(ctx, CLR_ERR_HIP, "batch work lists: %s", hipGetErrorString(e));
  clr_status s = CLR_OK;
  {
    // the bases must stay valid until the shift kernels have run
    HIP_TRY(ctx, ensure(pl->bases, sizeof(int64_t) * base.size()));
    HIP_TRY(ctx, hipMemcpyAsync(pl->bases.p, base.data(), sizeof(int64_t) * base.size(),
                                hipMemcpyHostToDevice, stream));
  }
  for (int p = 0; p < np; ++p) {
    const int64_t npairs = pb[p + 1] - pb[p];
    int64_t* off = as<int64_t>(ctx->w.off) + kNumCounters * pb[p];
    HIP_TRY(ctx, launch_add_base(off, npairs, kNumCounters, as<int64_t>(pl->bases) + (size_t)p * kNumCounters, stream));
    FillParams F{};
    F.off = off;
    F.cnt = as<int64_t>(ctx->w.cnt) + kNumCounters * pb[p];
    F.flags = as<int>(ctx->w.flags) + pb[p];
    F.seg_dense = as<Seg>(pl->seg_dense);
    F.items_dense = as<GemmItem>(pl->items_dense);
    F.seg_thin1 = as<Seg>(pl->seg_thin1);
    F.items_thin1 = as<GemmItem>(pl->items_thin1);
    F.seg_thin2 = as<Seg>(pl->seg_thin2);
    F.items_thin2 = as<GemmItem>(pl->items_thin2);
    F.pieces = as<Piece>(pl->pieces);
    F.rec = as<RecItem>(pl->rec);
    F.pool = as<double>(pl->pool);
    F.scratch = as<double>(pl->scratch);
    F.acc = as<double>(pl->acc);
    F.c_arena = pl->C[p]->arena;
    F.c_boff = pl->C[p]->d_boff;
    F.c_kind = pl->C[p]->d_kind;
    F.c_rank = pl->C[p]->d_rank;
    F.c_norm = pl->C[p]->d_norm;
    HIP_TRY(ctx, launch_fill(P[p], F, stream));
  }
  HIP_TRY(ctx, launch_item_order(as<GemmItem>(pl->items_dense), (int)sum[kCntGemmItems],
                                 as<int>(pl->order), stream));
  HIP_TRY(ctx, ensure(pl->order_thin, sizeof(int) * sum[kCntThin1]));
  HIP_TRY(ctx, ensure(ctx->w.sortw, operand_order_bytes((int)sum[kCntThin1])));
  HIP_TRY(ctx, launch_operand_order(as<GemmItem>(pl->items_thin1), as<Seg>(pl->seg_thin1),
                                    (int)sum[kCntThin1], ctx->w.sortw.p, as<int>(pl->order_thin),
                                    stream));
  HIP_TRY(ctx, hipStreamSynchronize(stream));
  return s;
}

clr_status plan_stats(clr_context* ctx, const clr_plan* pl, clr_gemm_stats* st) {
  memset(st, 0, sizeof(*st));
  st->candidates = (int64_t)pl->flops[kStCandidate];
  st->computed = pl->counts[kCntComputed];
  st->n_dd = (int64_t)pl->flops[kStNDD];
  st->n_ld = (int64_t)pl->flops[kStNLD];
  st->n_dl = (int64_t)pl->flops[kStNDL];
  st->n_ll = (int64_t)pl->flops[kStNLL];
  st->triples = st->n_dd + st->n_ld + st->n_dl + st->n_ll;
  st->flops_dd = pl->flops[kStFlopsDD];
  st->flops_ld = pl->flops[kStFlopsLD];
  st->flops_dl = pl->flops[kStFlopsDL];
  st->flops_ll = pl->flops[kStFlopsLL];
  st->flops_densify = pl->flops[kStFlopsDensify];
  st->flops_products = st->flops_dd + st->flops_ld + st->flops_dl + st->flops_ll + st->flops_densify;
  if (pl->n_rec > 0) {
    RecCounters rc;
    HIP_TRY(ctx, hipMemcpy(&rc, rec_work(pl->recg.p, pl->n_rec).ctr, sizeof(rc),
                           hipMemcpyDeviceToHost));
    st->flops_rec_engine = rc.flops_bidiag;
    st->certified_dense = (int64_t)rc.certified;
  }
  return CLR_OK;
}

}  // namespace

extern "C" clr_status clr_plan_create(clr_context* ctx, int nprod, const clr_matrix* const* A,
                                      const clr_matrix* const* B, const clr_gemm_opts* opts,
                                      int use_graph, clr_plan** plan, clr_matrix** C) {
  if (!ctx || !A || !B || !plan || !C || nprod < 1) return CLR_ERR_INVALID_ARG;
  *plan = nullptr;
  for (int p = 0; p < nprod; ++p) {
    C[p] = nullptr;
    if (!A[p] || !B[p]) return fail(ctx, CLR_ERR_INVALID_ARG, "null operand in product %d", p);
  }
  clr_status s = check_opts(ctx, opts);
  if (s != CLR_OK) return s;
  clr_plan* pl = new clr_plan();
  pl->ctx = ctx;
  for (DevBuf* b : {&pl->seg_dense, &pl->items_dense, &pl->seg_thin1, &pl->items_thin1,
                    &pl->seg_thin2, &pl->items_thin2, &pl->pieces, &pl->rec, &pl->pool,
                    &pl->scratch, &pl->acc, &pl->recg, &pl->status, &pl->bases, &pl->order,
                    &pl->order_thin})
    b->src = &ctx->alloc;
  pl->dense_cert = ctx->dense_cert;
  pl->nprod = nprod;
  pl->o = *opts;
  pl->A.assign(A, A + nprod);
  pl->B.assign(B, B + nprod);
  auto bail = [&](clr_status code) {
    for (auto* m : pl->C) free_matrix(m);
    plan_free(pl);
    return code;
  };
  if ((s = plan_build(ctx, pl)) != CLR_OK) return bail(s);
  if (use_graph) {
    // Record the execution phase once on a capture stream of its own (the
    // context stream may be the legacy default stream, which cannot be
    // captured); executing the plan replays the graph on the context stream.
    HIP_TRY(ctx, prepare_recompress());
    hipStream_t cs = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      hipError_t le = plan_launch(pl, cs);
      e = hipStreamEndCapture(cs, &pl->graph);
      if (e == hipSuccess) e = le;
    }
    if (cs) (void)hipStreamDestroy(cs);
    if (e == hipSuccess) e = hipGraphInstantiate(&pl->exec, pl->graph, nullptr, nullptr, 0);
    if (e != hipSuccess)
      return bail(fail(ctx, CLR_ERR_HIP, "graph capture: %s", hipGetErrorString(e)));
  }
  for (int p = 0; p < nprod; ++p) C[p] = pl->C[p];
  *plan = pl;
  return CLR_OK;
}

extern "C" clr_status clr_plan_execute(clr_context* ctx, clr_plan* pl, clr_gemm_stats* st) {
  if (!ctx || !pl || pl->ctx != ctx) return CLR_ERR_INVALID_ARG;
  HIP_TRY(ctx, hipEventRecord(ctx->ev[0], ctx->stream));
  if (pl->exec) {
    HIP_TRY(ctx, hipGraphLaunch(pl->exec, ctx->stream));
  } else {
    HIP_TRY(ctx, plan_launch(pl, ctx->stream));
  }
  HIP_TRY(ctx, hipEventRecord(ctx->ev[3], ctx->stream));
  clr_status s = plan_status(ctx, pl);
  if (s != CLR_OK) return s;
  if (st) {
    s = plan_stats(ctx, pl, st);
    if (s != CLR_OK) return s;
    st->ms_total = elapsed(ctx->ev[0], ctx->ev[3]);
    st->ms_products = st->ms_total;
  }
  return CLR_OK;
}

extern "C" clr_status clr_plan_destroy(clr_plan* pl) {
  if (!pl) return CLR_ERR_INVALID_ARG;
  (void)hipStreamSynchronize(pl->ctx->stream);
  plan_free(pl);
  return CLR_OK;
}

extern "C" clr_status clr_gemm_batch(clr_context* ctx, int nprod, const clr_matrix* const* A,
                                     const clr_matrix* const* B, const clr_gemm_opts* opts,
                                     clr_matrix** C, clr_gemm_stats* st) {
  clr_plan* pl = nullptr;
  clr_status s = clr_plan_create(ctx, nprod, A, B, opts, 0, &pl, C);
  if (s != CLR_OK) return s;
  s = clr_plan_execute(ctx, pl, st);
  clr_plan_destroy(pl);
  if (s != CLR_OK) {
    for (int p = 0; p < nprod; ++p) {
      free_matrix(C[p]);
      C[p] = nullptr;
    }
  }
  return s;
}

// ---------------------------------------------------------------------------
// Blockwise combination a X + b Y + c I
// ---------------------------------------------------------------------------

namespace {

// T = a X + b Y + c I with workspace W, planned on the device (k_comb_count,
// scan, k_comb_fill): dense parts summed elementwise, low-rank operands of
// densified blocks added by the grouped GEMM, then every computed block
// recompressed.  T is new or Tinto rewritten in place; dev as in gemm_impl.
clr_status axpby_impl(clr_context* ctx, Work& W, double a, const clr_matrix* X, double b,
                      const clr_matrix* Y, double c, const clr_gemm_opts* o, clr_matrix** Tout,
                      clr_matrix* Tinto = nullptr, const DevRun* dev = nullptr) {
  *Tout = nullptr;
  if (Y && (Y->rs != X->rs || Y->cs != X->cs))
    return fail(ctx, CLR_ERR_SHAPE, "clr_axpby: blockings differ");
  if (dev && !Tinto) return fail(ctx, CLR_ERR_INVALID_ARG, "device-sized combination: in place only");
  // the output: Tinto, or allocated once the plan has sized its room
  clr_matrix* T = Tinto;
  if (T) {
    if (T->rs != X->rs || T->cs != X->cs) return fail(ctx, CLR_ERR_SHAPE, "clr_axpby: output blocking");
    HIP_TRY(ctx, reset_meta(ctx, T));
  }
  auto bail = [&](clr_status code) {
    if (!Tinto && T) free_matrix(T);
    return code;
  };
  hipStream_t stream = ctx->stream;
  const int64_t nb = (int64_t)X->nrb * X->ncb;
  hipError_t e = hipSuccess;
  if (dev) {
    if (!work_fits(W, work_sizes(nb, dev->caps)))
      return bail(fail(ctx, CLR_ERR_CAPACITY, "workspace smaller than the run's capacities"));
  } else {
    if (e == hipSuccess) e = ensure(W.cnt, sizeof(int64_t) * kNumCounters * nb);
    if (e == hipSuccess) e = ensure(W.off, sizeof(int64_t) * kNumCounters * nb);
    if (e == hipSuccess) e = ensure(W.totals, sizeof(int64_t) * kNumCounters + sizeof(double) * kNumStats);
    if (e != hipSuccess) return bail(fail(ctx, CLR_ERR_HIP, "workspace: %s", hipGetErrorString(e)));
  }
  CombParams P{};
  P.X = X->view();
  if (Y) P.Y = Y->view();
  P.a = a;
  P.b = b;
  P.c = c;
  P.square = X->square_blocked() ? 1 : 0;
  P.eps_sp = o->eps_sp;
  P.screen = o->screen;
  P.tol = o->tol;
  P.edges = edge_table(ctx, o);
  int64_t* tot = as<int64_t>(W.totals);
  if (e == hipSuccess) e = launch_comb_count(P, as<int64_t>(W.cnt), stream);
  if (e == hipSuccess) e = launch_scan(as<int64_t>(W.cnt), as<int64_t>(W.off), nb, kNumCounters, tot, stream);
  int64_t n[kNumCounters];
  int64_t* live = nullptr;
  if (dev) {
    live = as<int64_t>(W.live);
    Caps caps = dev->caps;
    caps.c[kCntOut] = T->cap;   // the output's arena bounds its room
    if (e == hipSuccess) e = launch_caps(tot, caps, live, stream);
    for (int i = 0; i < kNumCounters; ++i) n[i] = caps.c[i];
  } else {
    if (e == hipSuccess) e = hipMemcpyAsync(n, tot, sizeof(n), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e == hipSuccess) {
      for (int i = 0; i < kNumCounters; ++i) W.seen.c[i] = std::max(W.seen.c[i], n[i]);
      Caps exact;
      for (int i = 0; i < kNumCounters; ++i) exact.c[i] = n[i];
      e = reserve_work(W, work_sizes(nb, exact));
    }
  }
  if (e != hipSuccess) return bail(fail(ctx, CLR_ERR_HIP, "combination plan: %s", hipGetErrorString(e)));
  for (int i = 0; i < kNumCounters; ++i)
    if (n[i] < 0 || (!counts_doubles(i) && n[i] > INT32_MAX))
      return bail(fail(ctx, CLR_ERR_CAPACITY, "work list %d too long (%lld)", i, (long long)n[i]));
  if (!dev) {
    if (T) {
      if (n[kCntOut] > T->cap)
        return bail(fail(ctx, CLR_ERR_CAPACITY, "output arena of %lld doubles, %lld needed",
                         (long long)T->cap, (long long)n[kCntOut]));
    } else {
      clr_status s = alloc_matrix(ctx, X->rs, X->cs, &T, nullptr, n[kCntOut]);
      if (s != CLR_OK) return s;
    }
  }
  P.t_arena = T->arena;
  P.t_boff = T->d_boff;
  P.t_kind = T->d_kind;
  P.t_rank = T->d_rank;
  P.t_norm = T->d_norm;
  T->host_boff = false;   // offsets planned on the device from here on
  auto lv = [&](int k) { return live ? live + k : nullptr; };
  P.acc = as<double>(W.acc);
  CombLists L{};
  L.off = as<int64_t>(W.off);
  L.cnt = as<int64_t>(W.cnt);
  L.dense = as<AxpbyDenseItem>(W.comb_dense);
  L.segs = as<Seg>(W.seg_dense);
  L.items = as<GemmItem>(W.items_dense);
  L.pieces = as<Piece>(W.pieces);
  L.rec = as<RecItem>(W.rec);
  L.scratch = as<double>(W.scratch);
  L.abort = lv(kLiveOverflow);
  if (e == hipSuccess) e = launch_comb_fill(P, L, stream);
  if (e == hipSuccess)
    e = launch_axpby_dense(L.dense, (int)n[kCntCombDense], stream, lv(kCntCombDense));
  if (e == hipSuccess)
    e = run_ggemm(o, L.items, L.segs, (int)n[kCntGemmItems], stream, false, nullptr,
                  lv(kCntGemmItems));
  if (e == hipSuccess)
    e = launch_recompress_work(ctx, W, L.rec, L.pieces, (int)n[kCntComputed], o->tol, false,
                               lv(kCntComputed));
  if (e != hipSuccess) return bail(fail(ctx, CLR_ERR_HIP, "axpby launch: %s", hipGetErrorString(e)));
  if (!dev) {
    clr_status s = check_status(ctx);
    if (s != CLR_OK) return bail(s);
  }
  *Tout = T;
  return CLR_OK;
}

}  // namespace

extern "C" clr_status clr_axpby(clr_context* ctx, double a, const clr_matrix* X, double b,
                                const clr_matrix* Y, double c, const clr_gemm_opts* o,
                                clr_matrix** Tout) {
  if (!ctx || !X || !Tout) return CLR_ERR_INVALID_ARG;
  *Tout = nullptr;
  clr_status s = check_opts(ctx, o);
  if (s != CLR_OK) return s;
  return axpby_impl(ctx, ctx->w, a, X, b, Y, c, o, Tout);
}

// ---------------------------------------------------------------------------
// Residuals and the square-root inverse
// ---------------------------------------------------------------------------

extern "C" clr_status clr_identity_residual(clr_context* ctx, const clr_matrix* X, double* out) {
  if (!ctx || !X || !out) return CLR_ERR_INVALID_ARG;
  if (!X->square_blocked()) return fail(ctx, CLR_ERR_SHAPE, "identity residual needs a square blocking");
  const int64_t nb = (int64_t)X->nrb * X->ncb;
  HIP_TRY(ctx, ensure(ctx->w.terms, sizeof(double) * nb));
  HIP_TRY(ctx, launch_identity_terms(X->view(), as<double>(ctx->w.terms), ctx->stream));
  std::vector<double> t(nb);
  HIP_TRY(ctx, hipMemcpyAsync(t.data(), ctx->w.terms.p, sizeof(double) * nb, hipMemcpyDeviceToHost, ctx->stream));
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  double s = 0.0;
  for (double v : t) s += v;
  *out = sqrt(s) / sqrt((double)X->rows);
  return CLR_OK;
}

// Allocation-free form of the above: the per-block terms go to the device's
// fixed array and the sum is taken on the device, so nothing is allocated and
// the host does not wait.
extern "C" clr_status clr_identity_residual_noalloc(clr_context* ctx, const clr_matrix* X,
                                                   double* out) {
  if (!ctx || !X || !out) return CLR_ERR_INVALID_ARG;
  if (!X->square_blocked()) return fail(ctx, CLR_ERR_SHAPE, "identity residual needs a square blocking");
  const int64_t nb = (int64_t)X->nrb * X->ncb;
  if (nb > kNoAllocMaxBlocks)
    return fail(ctx, CLR_ERR_CAPACITY, "%lld blocks exceed the %lld of the fixed array",
                (long long)nb, (long long)kNoAllocMaxBlocks);
  double* terms = noalloc_terms(ctx->device);
  if (!terms) return fail(ctx, CLR_ERR_HIP, "fixed array not set up on device %d", ctx->device);
  HIP_TRY(ctx, launch_identity_terms(X->view(), terms, ctx->stream));
  HIP_TRY(ctx, launch_residual_finish(terms, nb, (double)X->rows, out, ctx->stream));
  return CLR_OK;
}

namespace {

clr_status scaled_copy(clr_context* ctx, const clr_matrix* src, double sc, clr_matrix** out) {
  clr_status s = copy_matrix(ctx, src, out);
  if (s != CLR_OK) return s;
  HIP_TRY(ctx, launch_scale((*out)->view(), (*out)->arena, (*out)->d_norm, sc, ctx->stream));
  return CLR_OK;
}

clr_status identity_matrix(clr_context* ctx, const std::vector<int>& sizes, clr_matrix** out) {
  clr_matrix* Z = nullptr;
  // packed: the diagonal blocks one after another
  const size_t nbl = sizes.size();
  std::vector<int64_t> offs(nbl * nbl, 0);
  int64_t cap = 0;
  for (size_t I = 0; I < nbl; ++I) {
    offs[I * nbl + I] = cap;
    cap += (int64_t)sizes[I] * sizes[I];
  }
  clr_status s = alloc_matrix(ctx, sizes, sizes, &Z, &offs, cap);
  if (s != CLR_OK) return s;
  // Z = 0 * (nothing) + 1 * I through the dense combination path
  const int nb = Z->nrb;
  std::vector<AxpbyDenseItem> items;
  std::vector<int> kind(nb * nb, 0), rank(nb * nb, 0);
  std::vector<double> norm(nb * nb, 0.0);
  for (int I = 0; I < nb; ++I) {
    AxpbyDenseItem d{};
    d.D = Z->arena + Z->boff[(size_t)I * nb + I];
    d.c = 1.0;
    d.m = d.n = sizes[I];
    items.push_back(d);
    kind[I * nb + I] = 1;
    rank[I * nb + I] = sizes[I];
    norm[I * nb + I] = sqrt((double)sizes[I]);
  }
  if ((s = upload(ctx, ctx->w.comb_dense, items)) != CLR_OK) {
    free_matrix(Z);
    return s;
  }
  hipError_t e = launch_axpby_dense(ctx->w.comb_dense.p, nb, ctx->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(Z->d_kind, kind.data(), sizeof(int) * nb * nb, hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(Z->d_rank, rank.data(), sizeof(int) * nb * nb, hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(Z->d_norm, norm.data(), sizeof(double) * nb * nb, hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) {
    free_matrix(Z);
    return fail(ctx, CLR_ERR_HIP, "identity: %s", hipGetErrorString(e));
  }
  *out = Z;
  return CLR_OK;
}

// ||W S W - I||_F / sqrt(N) with untruncated, unscreened FP64 products.
clr_status explicit_residual(clr_context* ctx, const clr_matrix* W, const clr_matrix* S,
                             double* out, double* flops) {
  clr_gemm_opts ex{};
  ex.tol = 0.0;
  ex.eps_sp = 0.0;
  ex.screen = CLR_SCREEN_ABS;
  ex.precision = CLR_FP64;
  ex.alpha = 1.0;
  clr_matrix *WS = nullptr, *WSW = nullptr;
  clr_gemm_stats g1{}, g2{};
  clr_status s = gemm_impl(ctx, ctx->w, W, S, &ex, &WS, &g1);
  if (s != CLR_OK) return s;
  s = gemm_impl(ctx, ctx->w, WS, W, &ex, &WSW, &g2);
  free_matrix(WS);
  if (s != CLR_OK) return s;
  s = clr_identity_residual(ctx, WSW, out);
  free_matrix(WSW);
  if (flops) *flops += g1.flops_products + g2.flops_products;
  return s;
}

}  // namespace

namespace {

// One iteration of Eqs. (8)-(11) recorded as a HIP graph and replayed.
//
// The iterates live in two fixed pairs (Z, Y)[0..1] (ping-pong) next to fixed
// X_n, X_n^2 and T_n, and every product and the combination run with their
// work-list lengths left on the device (gemm_impl / axpby_impl with a DevRun),
// so a replay needs no host read-back: the host reads the residual's block
// terms and the overflow flag after it.  graph[p] reads pair p and writes pair
// 1 - p.  Capacities come from the lengths of the iteration run directly
// (times the margin); a replay that would exceed one leaves its inputs intact,
// so that iteration is redone directly and both graphs are recorded again.
constexpr double kGraphMargin = 2.0;    // default capacity over the lengths seen

struct IterGraph {
  clr_context* ctx;
  Work& W;   // the context's graph workspace: buffers persist (and only grow) between calls
  clr_matrix* Zb[2] = {};
  clr_matrix* Yb[2] = {};
  clr_matrix *X = nullptr, *Q = nullptr, *T = nullptr;
  hipGraph_t graph[2] = {};
  hipGraphExec_t exec[2] = {};
  DevRun run{};
  double margin = kGraphMargin;
  int cur = 0;        // the pair holding the current iterates
  int captures = 0, replays = 0;
  double flops = 0.0;

  explicit IterGraph(clr_context* c) : ctx(c), W(c->gw) {
    W.seen = Caps{};
  }
  ~IterGraph() {
    drop_graphs();
    for (clr_matrix* m : {Zb[0], Zb[1], Yb[0], Yb[1], X, Q, T}) free_matrix(m);
  }
  void drop_graphs() {
    for (int p = 0; p < 2; ++p) {
      if (exec[p]) (void)hipGraphExecDestroy(exec[p]);
      if (graph[p]) (void)hipGraphDestroy(graph[p]);
      exec[p] = nullptr;
      graph[p] = nullptr;
    }
  }
  // X_n, X_n^2, T_n and the next pair from pair p; the block terms of
  // ||X_n - I|| go to W.terms.  dev: device-sized (recordable) or direct.
  clr_status iterate(int p, const clr_gemm_opts* gx, const clr_gemm_opts* gr,
                     const clr_gemm_opts* g64, const DevRun* dev) {
    clr_matrix* out = nullptr;
    clr_status s = gemm_impl(ctx, W, Yb[p], Zb[p], gx, &out, nullptr, nullptr, X, dev);  // Eq. (8)
    if (s == CLR_OK) s = gemm_impl(ctx, W, X, X, gr, &out, nullptr, nullptr, Q, dev);
    if (s == CLR_OK)
      s = axpby_impl(ctx, W, -10.0 / 8.0, X, 3.0 / 8.0, Q, 15.0 / 8.0, g64, &out, T, dev);  // Eq. (9)
    if (s == CLR_OK) s = gemm_impl(ctx, W, Zb[p], T, gr, &out, nullptr, nullptr, Zb[1 - p], dev);
    if (s == CLR_OK) s = gemm_impl(ctx, W, T, Yb[p], gr, &out, nullptr, nullptr, Yb[1 - p], dev);
    if (s == CLR_OK) HIP_TRY(ctx, launch_identity_terms(X->view(), as<double>(W.terms), ctx->stream));
    return s;
  }

  // Record graph[p] on a capture stream of its own (the context stream may be
  // the legacy default stream, which cannot be captured).
  clr_status capture(int p, const clr_gemm_opts* gx, const clr_gemm_opts* gr,
                     const clr_gemm_opts* g64) {
    hipStream_t cs = nullptr;
    HIP_TRY(ctx, hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    hipStream_t saved = ctx->stream;
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    clr_status s = CLR_OK;
    if (e == hipSuccess) {
      ctx->stream = cs;
      // the overflow flag starts clear on every replay (a kernel, not a memset)
      hipError_t le = launch_fill_i32(reinterpret_cast<int*>(as<int64_t>(W.live) + kLiveOverflow), 0,
                                      2, cs);
      if (le == hipSuccess)
        le = launch_fill_f64(as<double>(W.flops), 0.0, 1, cs);
      s = le == hipSuccess ? iterate(p, gx, gr, g64, &run) : fail(ctx, CLR_ERR_HIP, "capture: %s", hipGetErrorString(le));
      ctx->stream = saved;
      e = hipStreamEndCapture(cs, &graph[p]);
    }
    (void)hipStreamDestroy(cs);
    if (s != CLR_OK) return s;
    if (e == hipSuccess) e = hipGraphInstantiate(&exec[p], graph[p], nullptr, nullptr, 0);
    if (e != hipSuccess) return fail(ctx, CLR_ERR_HIP, "iteration graph: %s", hipGetErrorString(e));
    ++captures;
    return CLR_OK;
  }

  // Capacities from the lengths seen (times m) and both graphs.
  clr_status prepare(double m, const clr_gemm_opts* gx, const clr_gemm_opts* gr,
                     const clr_gemm_opts* g64) {
    drop_graphs();
    for (int c = 0; c < kNumCounters; ++c)
      run.caps.c[c] = std::max<int64_t>(run.caps.c[c],
                                        (int64_t)std::ceil(m * (double)W.seen.c[c]) + 16);
    const int64_t nb = (int64_t)X->nrb * X->ncb;
    HIP_TRY(ctx, reserve_work(W, work_sizes(nb, run.caps, block_list_ints(X->nrb, X->ncb, X->ncb))));
    HIP_TRY(ctx, launch_fill_i32(reinterpret_cast<int*>(as<int64_t>(W.live)), 0, 2 * kNumLive,
                                 ctx->stream));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    for (int p = 0; p < 2; ++p) {
      clr_status s = capture(p, gx, gr, g64);
      if (s != CLR_OK) return s;
    }
    return CLR_OK;
  }

  // ||X_n - I||_F / sqrt(N) from the block terms in W.terms, summed on the
  // host in block order (as clr_identity_residual does).
  clr_status residual(double* r) {
    const int64_t nb = (int64_t)X->nrb * X->ncb;
    std::vector<double> t(nb);
    HIP_TRY(ctx, hipMemcpyAsync(t.data(), W.terms.p, sizeof(double) * nb, hipMemcpyDeviceToHost,
                                ctx->stream));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    double sum = 0.0;
    for (double v : t) sum += v;
    *r = sqrt(sum) / sqrt((double)X->rows);
    return CLR_OK;
  }

  // One iteration from the current pair: directly the first time (which sizes
  // the graphs), replayed afterwards.
  clr_status step(const clr_gemm_opts* gx, const clr_gemm_opts* gr, const clr_gemm_opts* g64,
                  double* r) {
    clr_status s;
    if (!exec[0]) {
      s = direct(gx, gr, g64);
      if (s == CLR_OK) s = prepare(margin, gx, gr, g64);
    } else {
      HIP_TRY(ctx, hipGraphLaunch(exec[cur], ctx->stream));
      int64_t flag = 0;
      double f = 0.0;
      HIP_TRY(ctx, hipMemcpyAsync(&flag, as<int64_t>(W.live) + kLiveOverflow, sizeof(flag),
                                  hipMemcpyDeviceToHost, ctx->stream));
      HIP_TRY(ctx, hipMemcpyAsync(&f, W.flops.p, sizeof(f), hipMemcpyDeviceToHost, ctx->stream));
      HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
      s = check_status(ctx);
      if (s != CLR_OK) return s;
      if (flag) {
        // a list outgrew its capacity: the inputs are intact, so redo the
        // iteration directly and record the graphs for the lengths seen
        Caps need;
        HIP_TRY(ctx, hipMemcpy(need.c, as<int64_t>(W.live) + kLiveNeed, sizeof(need.c),
                               hipMemcpyDeviceToHost));
        for (int c = 0; c < kNumCounters; ++c) W.seen.c[c] = std::max(W.seen.c[c], need.c[c]);
        s = direct(gx, gr, g64);
        if (s == CLR_OK) s = prepare(std::max(margin, kGraphMargin), gx, gr, g64);
      } else {
        flops += f;
        ++replays;
        s = CLR_OK;
      }
    }
    if (s != CLR_OK) return s;
    s = residual(r);
    cur = 1 - cur;
    return s;
  }

  // The iteration from the current pair with every list sized on the host
  // (which also records the lengths in W.seen and the flops).
  clr_status direct(const clr_gemm_opts* gx, const clr_gemm_opts* gr, const clr_gemm_opts* g64) {
    const double f0 = W.host_flops;
    clr_status s = iterate(cur, gx, gr, g64, nullptr);
    if (s == CLR_OK) s = check_status(ctx);
    flops += W.host_flops - f0;
    return s;
  }
};

}  // namespace

extern "C" clr_status clr_sqrt_inv(clr_context* ctx, const clr_matrix* S, const clr_sqrtinv_opts* o,
                                   clr_matrix** Wout, clr_sqrtinv_stats* st) {
  if (!ctx || !S || !o || !Wout) return CLR_ERR_INVALID_ARG;
  *Wout = nullptr;
  clr_status s = check_opts(ctx, &o->g);
  if (s != CLR_OK) return s;
  if (!S->square_blocked()) return fail(ctx, CLR_ERR_SHAPE, "S must be square-blocked");
  if (!(o->conv_tol >= 0.0) || o->max_iter < 1 || o->fixed_iters < 0 || !(o->alpha >= 0.0) ||
      !(o->reduced_below >= 0.0) || !(o->graph_margin >= 0.0))
    return fail(ctx, CLR_ERR_INVALID_ARG, "bad iteration options");
  if (o->graph && (o->reduced_below > 0.0 || o->g.precision == CLR_OZAKI))
    return fail(ctx, CLR_ERR_INVALID_ARG,
                "graph replay needs reduced_below == 0 and the FP64 or MIXED form");
  HIP_TRY(ctx, hipEventRecord(ctx->ev[4], ctx->stream));
  double alpha = o->alpha;
  if (alpha == 0.0) {
    HostMeta h;
    if ((s = fetch_meta(ctx, S, h)) != CLR_OK) return s;
    double worst = 0.0;
    for (int I = 0; I < S->nrb; ++I) {
      double row = 0.0;
      for (int J = 0; J < S->ncb; ++J)
        if (h.kind[(size_t)I * S->ncb + J]) row += h.norm[(size_t)I * S->ncb + J];
      worst = std::max(worst, row);
    }
    if (!(worst > 0.0)) return fail(ctx, CLR_ERR_INVALID_ARG, "S has no nonzero blocks");
    alpha = 1.0 / worst;
  }
  clr_gemm_opts g = o->g;
  g.alpha = 1.0;
  clr_gemm_opts ga = g;
  ga.alpha = alpha;
  // the FP64 options of the precision schedule's early iterations and of X_n
  clr_gemm_opts g64 = g, ga64 = ga;
  g64.precision = ga64.precision = CLR_FP64;
  g64.split = ga64.split = 0;
  const bool scheduled = o->g.precision != CLR_FP64 && o->reduced_below > 0.0;
  clr_matrix *Z = nullptr, *Y = nullptr;
  if (o->graph) {
    // the graph's fixed pairs hold results of any rank: dense slots
    if ((s = identity_matrix(ctx, S->rs, &Y)) != CLR_OK) return s;
    s = relayout_matrix(ctx, Y, nullptr, -1, &Z);
    free_matrix(Y);
    Y = nullptr;
    if (s != CLR_OK) return s;
    if ((s = relayout_matrix(ctx, S, nullptr, -1, &Y)) != CLR_OK) {
      free_matrix(Z);
      return s;
    }
  } else {
    if ((s = identity_matrix(ctx, S->rs, &Z)) != CLR_OK) return s;
    if ((s = copy_matrix(ctx, S, &Y)) != CLR_OK) {
      free_matrix(Z);
      return s;
    }
  }
  // graph replay: the iterates move into the graph's fixed pairs, which it owns
  std::unique_ptr<IterGraph> G;
  if (o->graph) {
    G.reset(new IterGraph(ctx));
    G->margin = o->graph_margin > 0.0 ? o->graph_margin : kGraphMargin;
    G->Zb[0] = Z;
    G->Yb[0] = Y;
    for (clr_matrix** m : {&G->Zb[1], &G->Yb[1], &G->X, &G->Q, &G->T})
      if ((s = alloc_matrix(ctx, S->rs, S->rs, m)) != CLR_OK) return s;
  }
  auto release = [&]() {
    if (G) {
      G.reset();
    } else {
      free_matrix(Z);
      free_matrix(Y);
    }
    Z = Y = nullptr;
  };
  std::vector<double> internal;
  std::vector<double> expl;
  double flops = 0.0;
  int n_gemms = 0;
  int it = 0;
  clr_status result = CLR_ERR_NOT_CONVERGED;
  bool converged = false;
  double last_explicit = -1.0;
  const int n_iter = o->fixed_iters > 0 ? o->fixed_iters : o->max_iter;
  for (it = 0; it < n_iter; ++it) {
    double r = 0.0;
    if (G) {
      s = G->step(&ga, &g, &g64, &r);
      n_gemms += 4;
      if (s != CLR_OK) {
        release();
        return s;
      }
      Z = G->Zb[G->cur];
      Y = G->Yb[G->cur];
    } else {
      clr_matrix *X = nullptr, *Q = nullptr, *T = nullptr, *Zn = nullptr, *Yn = nullptr;
      clr_gemm_stats gs{};
      // precision of this iteration's products: everything in g.precision, or (the
      // schedule) FP64 until the residual has fallen to reduced_below, then X_n in
      // FP64 and the other products in g.precision
      const bool reduced = !scheduled || (!internal.empty() && internal.back() <= o->reduced_below);
      const clr_gemm_opts* gx = scheduled ? &ga64 : &ga;
      const clr_gemm_opts* gr = reduced ? &g : &g64;
      s = gemm_impl(ctx, ctx->w, Y, Z, gx, &X, &gs);                  // X_n = alpha Y_n Z_n   (Eq. (8))
      flops += gs.flops_products;
      if (scheduled && reduced && o->correction) {
        // T_n = I + D_n, D_n = -E_n/2 + 3 E_n^2/8 with E_n = X_n - I (Eq. (9) expanded)
        clr_matrix *E = nullptr, *E2 = nullptr, *P = nullptr, *R = nullptr;
        if (s == CLR_OK) s = clr_axpby(ctx, 1.0, X, 0.0, nullptr, -1.0, &g64, &E);
        if (s == CLR_OK) s = gemm_impl(ctx, ctx->w, E, E, gr, &E2, &gs);
        flops += gs.flops_products;
        if (s == CLR_OK) s = clr_axpby(ctx, -0.5, E, 3.0 / 8.0, E2, 0.0, &g64, &T);   // T holds D_n
        if (s == CLR_OK) s = gemm_impl(ctx, ctx->w, Z, T, gr, &P, &gs);                        // Z_n D_n
        flops += gs.flops_products;
        if (s == CLR_OK) s = clr_axpby(ctx, 1.0, Z, 1.0, P, 0.0, &g64, &Zn);          // Eq. (10)
        if (s == CLR_OK) s = gemm_impl(ctx, ctx->w, T, Y, gr, &R, &gs);                        // D_n Y_n
        flops += gs.flops_products;
        if (s == CLR_OK) s = clr_axpby(ctx, 1.0, Y, 1.0, R, 0.0, &g64, &Yn);          // Eq. (11)
        free_matrix(E);
        free_matrix(E2);
        free_matrix(P);
        free_matrix(R);
      } else {
        if (s == CLR_OK) s = gemm_impl(ctx, ctx->w, X, X, gr, &Q, &gs);  // X_n^2
        flops += gs.flops_products;
        if (s == CLR_OK) s = clr_axpby(ctx, -10.0 / 8.0, X, 3.0 / 8.0, Q, 15.0 / 8.0, &g64, &T);  // Eq. (9)
        if (s == CLR_OK) s = gemm_impl(ctx, ctx->w, Z, T, gr, &Zn, &gs);  // Z_{n+1} = Z_n T_n     (Eq. (10))
        flops += gs.flops_products;
        if (s == CLR_OK) s = gemm_impl(ctx, ctx->w, T, Y, gr, &Yn, &gs);  // Y_{n+1} = T_n Y_n     (Eq. (11))
        flops += gs.flops_products;
      }
      if (s == CLR_OK) s = clr_identity_residual(ctx, X, &r);
      n_gemms += 4;
      free_matrix(X);
      free_matrix(Q);
      free_matrix(T);
      if (s != CLR_OK) {
        free_matrix(Zn);
        free_matrix(Yn);
        release();
        return s;
      }
      free_matrix(Z);
      free_matrix(Y);
      Z = Zn;
      Y = Yn;
    }
    internal.push_back(r);
    if (o->fixed_iters > 0) continue;
    if (r <= o->conv_tol) {
      clr_matrix* W = nullptr;
      if ((s = scaled_copy(ctx, Z, sqrt(alpha), &W)) != CLR_OK) break;
      double e = 0.0;
      s = explicit_residual(ctx, W, S, &e, &flops);
      n_gemms += 2;
      free_matrix(W);
      if (s != CLR_OK) break;
      expl.push_back(e);
      if (e <= o->conv_tol) {
        converged = true;
        result = CLR_OK;
        ++it;
        break;
      }
      if (last_explicit >= 0.0 && e > 0.5 * last_explicit) {
        result = CLR_ERR_NOT_CONVERGED;
        ++it;
        break;
      }
      last_explicit = e;
    } else if (internal.size() >= 3 && internal[internal.size() - 1] > internal[internal.size() - 2] &&
               internal[internal.size() - 2] > internal[internal.size() - 3]) {
      // the residual falls monotonically in exact arithmetic once
      // ||alpha S - I||_2 < 1 (Sec. 4.2): growth while it is small is the
      // truncation / precision floor (stalled), growth beyond 0.5 divergence
      if (internal.back() > 0.5) {
        release();
        return fail(ctx, CLR_ERR_DIVERGED, "||X_n - I|| grew in two consecutive iterations");
      }
      result = CLR_ERR_NOT_CONVERGED;
      ++it;
      break;
    }
  }
  if (s != CLR_OK) {
    release();
    return s;
  }
  if (o->fixed_iters > 0) result = CLR_OK;
  clr_matrix* W = nullptr;
  s = scaled_copy(ctx, Z, sqrt(alpha), &W);
  const int replays = G ? G->replays : 0, captures = G ? G->captures : 0;
  if (G) flops += G->flops;
  release();
  if (s != CLR_OK) return s;
  HIP_TRY(ctx, hipEventRecord(ctx->ev[5], ctx->stream));
  HIP_TRY(ctx, hipEventSynchronize(ctx->ev[5]));
  if (st) {
    memset(st, 0, sizeof(*st));
    st->iterations = o->fixed_iters > 0 ? o->fixed_iters : it;
    st->converged = converged ? 1 : 0;
    st->alpha = alpha;
    st->internal_residual = internal.empty() ? -1.0 : internal.back();
    st->explicit_residual = expl.empty() ? -1.0 : expl.back();
    st->n_gemms = n_gemms;
    st->flops_products = flops;
    st->ms_total = elapsed(ctx->ev[4], ctx->ev[5]);
    st->graph_replays = replays;
    st->graph_captures = captures;
  }
  *Wout = W;
  if (result != CLR_OK)
    fail(ctx, result, "stopped after %d iterations without meeting conv_tol", it);
  return result;
}

// ---------------------------------------------------------------------------
// Adjoints
// ---------------------------------------------------------------------------

namespace {

// All-dense CLR matrix from a dense device matrix (ld); blocks outside `mask`
// (if given) and exactly-zero blocks become zero blocks.
clr_status dense_to_clr(clr_context* ctx, const double* D, int64_t ld, const std::vector<int>& rs,
                        const std::vector<int>& cs, const clr_matrix* mask, clr_matrix** out) {
  clr_matrix* M = nullptr;
  clr_status s = alloc_matrix(ctx, rs, cs, &M);
  if (s != CLR_OK) return s;
  hipError_t e = launch_from_dense(M->view(), M->arena, M->d_kind, M->d_rank, M->d_norm, D, ld,
                                   mask ? mask->d_kind : nullptr, ctx->stream);
  if (e != hipSuccess) {
    free_matrix(M);
    return fail(ctx, CLR_ERR_HIP, "dense ingest: %s", hipGetErrorString(e));
  }
  *out = M;
  return CLR_OK;
}

clr_status transpose_clr(clr_context* ctx, const clr_matrix* A, clr_matrix** out) {
  // block (J, I) of T stores as many elements as block (I, J) of A: same offsets
  const size_t nb = (size_t)A->nrb * A->ncb;
  std::vector<int64_t> ab = A->boff;
  if (!A->host_boff) {
    ab.resize(nb);
    HIP_TRY(ctx, hipMemcpyAsync(ab.data(), A->d_boff, sizeof(int64_t) * nb, hipMemcpyDeviceToHost,
                                ctx->stream));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  }
  std::vector<int64_t> tb(nb);
  for (int I = 0; I < A->nrb; ++I)
    for (int J = 0; J < A->ncb; ++J) tb[(size_t)J * A->nrb + I] = ab[(size_t)I * A->ncb + J];
  clr_matrix* T = nullptr;
  clr_status s = alloc_matrix(ctx, A->cs, A->rs, &T, &tb, A->cap);
  if (s != CLR_OK) return s;
  hipError_t e = launch_transpose(A->view(), T->view(), T->arena, T->d_kind, T->d_rank, T->d_norm,
                                  ctx->stream);
  if (e != hipSuccess) {
    free_matrix(T);
    return fail(ctx, CLR_ERR_HIP, "transpose: %s", hipGetErrorString(e));
  }
  *out = T;
  return CLR_OK;
}

// Exact (untruncated, unscreened) products and sums for cotangents.
clr_gemm_opts exact_opts(const clr_gemm_opts* g, double alpha) {
  clr_gemm_opts o{};
  o.tol = 0.0;
  o.eps_sp = 0.0;
  o.screen = CLR_SCREEN_ABS;
  o.precision = g ? g->precision : CLR_FP64;
  o.split = g ? g->split : 0;
  o.alpha = alpha;
  return o;
}

// Owning handle list: frees every matrix on scope exit.
struct Owned {
  std::vector<clr_matrix*> v;
  clr_matrix* keep(clr_matrix* m) {
    v.push_back(m);
    return m;
  }
  void drop(clr_matrix* m) {
    for (auto& x : v)
      if (x == m) {
        free_matrix(x);
        x = nullptr;
      }
  }
  ~Owned() {
    for (auto* m : v) free_matrix(m);
  }
};

// P = a X + b Y exactly, where either operand may be absent (NULL = zero).
clr_status exact_sum(clr_context* ctx, double a, const clr_matrix* X, double b, const clr_matrix* Y,
                     const clr_gemm_opts* g, clr_matrix** out) {
  *out = nullptr;
  const clr_gemm_opts o = exact_opts(g, 1.0);
  if (!X && !Y) return CLR_OK;
  if (!X) return clr_axpby(ctx, b, Y, 0.0, nullptr, 0.0, &o, out);
  return clr_axpby(ctx, a, X, Y ? b : 0.0, Y, 0.0, &o, out);
}

// alpha * L * R exactly (NULL operand = zero product).
clr_status exact_product(clr_context* ctx, const clr_matrix* L, const clr_matrix* R, double alpha,
                         const clr_gemm_opts* g, clr_matrix** out, double* flops,
                         const clr_matrix* mask = nullptr) {
  *out = nullptr;
  if (!L || !R) return CLR_OK;
  const clr_gemm_opts o = exact_opts(g, alpha);
  clr_gemm_stats gs{};
  clr_status s = gemm_impl(ctx, ctx->w, L, R, &o, out, &gs, mask);
  if (flops) *flops += gs.flops_products;
  return s;
}

clr_status write_dense(clr_context* ctx, const clr_matrix* M, const std::vector<int>& rs,
                       const std::vector<int>& cs, double* out, int64_t ld) {
  if (M) {
    HIP_TRY(ctx, launch_to_dense(M->view(), out, ld, ctx->stream));
  } else {
    int64_t rows = 0, cols = 0;
    for (int v : rs) rows += v;
    for (int v : cs) cols += v;
    HIP_TRY(ctx, hipMemset2DAsync(out, sizeof(double) * ld, 0, sizeof(double) * rows, cols, ctx->stream));
  }
  return CLR_OK;
}

}  // namespace

extern "C" clr_status clr_gemm_backward(clr_context* ctx, const clr_matrix* A, const clr_matrix* B,
                                        double alpha, const double* dC, int64_t ldc, double* dA,
                                        int64_t lda, double* dB, int64_t ldb) {
  if (!ctx || !A || !B || !dC) return CLR_ERR_INVALID_ARG;
  if (A->cs != B->rs)
    return fail(ctx, CLR_ERR_SHAPE, "column blocking of A differs from row blocking of B");
  if (!std::isfinite(alpha)) return fail(ctx, CLR_ERR_INVALID_ARG, "alpha must be finite");
  if (ldc < A->rows || (dA && lda < A->rows) || (dB && ldb < B->rows))
    return fail(ctx, CLR_ERR_INVALID_ARG, "leading dimension smaller than the row count");
  Owned own;
  clr_matrix* G = nullptr;
  clr_status s = dense_to_clr(ctx, dC, ldc, A->rs, B->cs, nullptr, &G);
  if (s != CLR_OK) return s;
  own.keep(G);
  const clr_gemm_opts g = exact_opts(nullptr, alpha);
  if (dA) {
    // dA = alpha dC B^T on A's stored blocks
    clr_matrix *Bt = nullptr, *P = nullptr;
    if ((s = transpose_clr(ctx, B, &Bt)) != CLR_OK) return s;
    own.keep(Bt);
    if ((s = exact_product(ctx, G, Bt, alpha, &g, &P, nullptr, A)) != CLR_OK) return s;
    own.keep(P);
    if ((s = write_dense(ctx, P, A->rs, A->cs, dA, lda)) != CLR_OK) return s;
  }
  if (dB) {
    // dB = alpha A^T dC on B's stored blocks
    clr_matrix *At = nullptr, *P = nullptr;
    if ((s = transpose_clr(ctx, A, &At)) != CLR_OK) return s;
    own.keep(At);
    if ((s = exact_product(ctx, At, G, alpha, &g, &P, nullptr, B)) != CLR_OK) return s;
    own.keep(P);
    if ((s = write_dense(ctx, P, B->rs, B->cs, dB, ldb)) != CLR_OK) return s;
  }
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  return CLR_OK;
}

// Reverse of the iteration of Sec. 4.2, Eqs. (8)-(11), with alpha held
// constant and truncation treated as the identity (straight-through):
//   Zb_K = sqrt(alpha) Wbar, Yb_K = 0; for n = K-1 .. 0:
//   Tb = Z_n^T Zb + Yb Y_n^T
//   Xb = -(10/8) Tb + (3/8)(Tb X_n^T + X_n^T Tb)
//   Zb <- Zb T_n^T + alpha Y_n^T Xb,   Yb <- T_n^T Yb + alpha Xb Z_n^T
// dS = Yb_0 on S's stored blocks.  Forward iterates are kept at checkpoints
// and recomputed one segment at a time.
extern "C" clr_status clr_sqrt_inv_backward(clr_context* ctx, const clr_matrix* S,
                                            const clr_sqrtinv_opts* o, int iters,
                                            int checkpoint_every, const double* Wbar, double* dS,
                                            int64_t ld, clr_matrix** Wout) {
  if (!ctx || !S || !o || !Wbar || !dS) return CLR_ERR_INVALID_ARG;
  if (Wout) *Wout = nullptr;
  clr_status s = check_opts(ctx, &o->g);
  if (s != CLR_OK) return s;
  if (!S->square_blocked()) return fail(ctx, CLR_ERR_SHAPE, "S must be square-blocked");
  if (iters < 1 || checkpoint_every < 1 || !(o->alpha >= 0.0))
    return fail(ctx, CLR_ERR_INVALID_ARG, "bad iteration options");
  if (o->reduced_below != 0.0 || o->correction != 0)
    return fail(ctx, CLR_ERR_INVALID_ARG, "the adjoint unrolls the iteration as printed (no precision schedule)");
  if (ld < S->rows) return fail(ctx, CLR_ERR_INVALID_ARG, "ld < N");
  double alpha = o->alpha;
  if (alpha == 0.0) {
    HostMeta h;
    if ((s = fetch_meta(ctx, S, h)) != CLR_OK) return s;
    double worst = 0.0;
    for (int I = 0; I < S->nrb; ++I) {
      double row = 0.0;
      for (int J = 0; J < S->ncb; ++J)
        if (h.kind[(size_t)I * S->ncb + J]) row += h.norm[(size_t)I * S->ncb + J];
      worst = std::max(worst, row);
    }
    if (!(worst > 0.0)) return fail(ctx, CLR_ERR_INVALID_ARG, "S has no nonzero blocks");
    alpha = 1.0 / worst;
  }
  clr_gemm_opts g = o->g;
  g.alpha = 1.0;
  clr_gemm_opts ga = g;
  ga.alpha = alpha;
  // one forward step from (Y, Z): X, T, and the next pair
  auto step = [&](const clr_matrix* Y, const clr_matrix* Z, clr_matrix** X, clr_matrix** T,
                  clr_matrix** Yn, clr_matrix** Zn) -> clr_status {
    clr_matrix* Q = nullptr;
    clr_status r = gemm_impl(ctx, ctx->w, Y, Z, &ga, X, nullptr);
    if (r == CLR_OK) r = gemm_impl(ctx, ctx->w, *X, *X, &g, &Q, nullptr);
    if (r == CLR_OK) r = clr_axpby(ctx, -10.0 / 8.0, *X, 3.0 / 8.0, Q, 15.0 / 8.0, &g, T);
    free_matrix(Q);
    if (r == CLR_OK) r = gemm_impl(ctx, ctx->w, Z, *T, &g, Zn, nullptr);
    if (r == CLR_OK) r = gemm_impl(ctx, ctx->w, *T, Y, &g, Yn, nullptr);
    return r;
  };
  Owned own;
  // forward with checkpoints of (Y_n, Z_n) at n = 0, c, 2c, ...
  const int K = iters, c = checkpoint_every;
  std::vector<clr_matrix*> ckY((K + c - 1) / c, nullptr), ckZ((K + c - 1) / c, nullptr);
  clr_matrix *Z = nullptr, *Y = nullptr;
  if ((s = identity_matrix(ctx, S->rs, &Z)) != CLR_OK) return s;
  own.keep(Z);
  if ((s = copy_matrix(ctx, S, &Y)) != CLR_OK) return s;
  own.keep(Y);
  for (int n = 0; n < K; ++n) {
    if (n % c == 0) {
      ckY[n / c] = Y;
      ckZ[n / c] = Z;
    }
    clr_matrix *X = nullptr, *T = nullptr, *Yn = nullptr, *Zn = nullptr;
    s = step(Y, Z, &X, &T, &Yn, &Zn);
    free_matrix(X);
    free_matrix(T);
    if (Yn) own.keep(Yn);
    if (Zn) own.keep(Zn);
    if (s != CLR_OK) return s;
    if (n % c != 0) {   // not a checkpoint: the previous pair is no longer needed
      own.drop(Y);
      own.drop(Z);
    }
    Y = Yn;
    Z = Zn;
  }
  if (Wout) {
    clr_matrix* W = nullptr;
    if ((s = scaled_copy(ctx, Z, sqrt(alpha), &W)) != CLR_OK) return s;
    *Wout = W;
  }
  own.drop(Y);
  own.drop(Z);
  auto fail_out = [&](clr_status code) {
    if (Wout && *Wout) {
      free_matrix(*Wout);
      *Wout = nullptr;
    }
    return code;
  };
  // cotangents (NULL = zero)
  clr_matrix* Zb = nullptr;
  clr_matrix* Yb = nullptr;
  {
    clr_matrix* Wb = nullptr;
    if ((s = dense_to_clr(ctx, Wbar, ld, S->rs, S->cs, nullptr, &Wb)) != CLR_OK) return fail_out(s);
    HIP_TRY(ctx, launch_scale(Wb->view(), Wb->arena, Wb->d_norm, sqrt(alpha), ctx->stream));
    Zb = Wb;
  }
  Owned cot;
  cot.keep(Zb);
  for (int seg = (K - 1) / c; seg >= 0; --seg) {
    const int n0 = seg * c, n1 = std::min(K, n0 + c);
    // recompute the segment's iterates
    Owned segown;
    std::vector<clr_matrix*> Ys, Zs, Xs, Ts;
    const clr_matrix* Yc = ckY[seg];
    const clr_matrix* Zc = ckZ[seg];
    for (int n = n0; n < n1; ++n) {
      clr_matrix *X = nullptr, *T = nullptr, *Yn = nullptr, *Zn = nullptr;
      s = step(Yc, Zc, &X, &T, &Yn, &Zn);
      for (clr_matrix* mm : {X, T, Yn, Zn})
        if (mm) segown.keep(mm);
      if (s != CLR_OK) return fail_out(s);
      Ys.push_back(const_cast<clr_matrix*>(Yc));
      Zs.push_back(const_cast<clr_matrix*>(Zc));
      Xs.push_back(X);
      Ts.push_back(T);
      Yc = Yn;
      Zc = Zn;
    }
    for (int n = n1 - 1; n >= n0; --n) {
      const int i = n - n0;
      Owned tmp;
      clr_matrix *Zt = nullptr, *Yt = nullptr, *Xt = nullptr, *Tt = nullptr;
      if ((s = transpose_clr(ctx, Zs[i], &Zt)) != CLR_OK) return fail_out(s);
      tmp.keep(Zt);
      if ((s = transpose_clr(ctx, Ys[i], &Yt)) != CLR_OK) return fail_out(s);
      tmp.keep(Yt);
      if ((s = transpose_clr(ctx, Xs[i], &Xt)) != CLR_OK) return fail_out(s);
      tmp.keep(Xt);
      if ((s = transpose_clr(ctx, Ts[i], &Tt)) != CLR_OK) return fail_out(s);
      tmp.keep(Tt);
      clr_matrix *P1 = nullptr, *P2 = nullptr, *Tb = nullptr;
      if ((s = exact_product(ctx, Zt, Zb, 1.0, &g, &P1, nullptr)) != CLR_OK) return fail_out(s);
      if (P1) tmp.keep(P1);
      if ((s = exact_product(ctx, Yb, Yt, 1.0, &g, &P2, nullptr)) != CLR_OK) return fail_out(s);
      if (P2) tmp.keep(P2);
      if ((s = exact_sum(ctx, 1.0, P1, 1.0, P2, &g, &Tb)) != CLR_OK) return fail_out(s);
      if (Tb) tmp.keep(Tb);
      clr_matrix *Q1 = nullptr, *Q2 = nullptr, *Q = nullptr, *Xb = nullptr;
      if ((s = exact_product(ctx, Tb, Xt, 1.0, &g, &Q1, nullptr)) != CLR_OK) return fail_out(s);
      if (Q1) tmp.keep(Q1);
      if ((s = exact_product(ctx, Xt, Tb, 1.0, &g, &Q2, nullptr)) != CLR_OK) return fail_out(s);
      if (Q2) tmp.keep(Q2);
      if ((s = exact_sum(ctx, 1.0, Q1, 1.0, Q2, &g, &Q)) != CLR_OK) return fail_out(s);
      if (Q) tmp.keep(Q);
      if ((s = exact_sum(ctx, -10.0 / 8.0, Tb, 3.0 / 8.0, Q, &g, &Xb)) != CLR_OK) return fail_out(s);
      if (Xb) tmp.keep(Xb);
      clr_matrix *Z1 = nullptr, *Z2 = nullptr, *Zbn = nullptr;
      if ((s = exact_product(ctx, Zb, Tt, 1.0, &g, &Z1, nullptr)) != CLR_OK) return fail_out(s);
      if (Z1) tmp.keep(Z1);
      if ((s = exact_product(ctx, Yt, Xb, alpha, &g, &Z2, nullptr)) != CLR_OK) return fail_out(s);
      if (Z2) tmp.keep(Z2);
      if ((s = exact_sum(ctx, 1.0, Z1, 1.0, Z2, &g, &Zbn)) != CLR_OK) return fail_out(s);
      clr_matrix *Y1 = nullptr, *Y2 = nullptr, *Ybn = nullptr;
      if ((s = exact_product(ctx, Tt, Yb, 1.0, &g, &Y1, nullptr)) != CLR_OK) return fail_out(s);
      if (Y1) tmp.keep(Y1);
      if ((s = exact_product(ctx, Xb, Zt, alpha, &g, &Y2, nullptr)) != CLR_OK) return fail_out(s);
      if (Y2) tmp.keep(Y2);
      if ((s = exact_sum(ctx, 1.0, Y1, 1.0, Y2, &g, &Ybn)) != CLR_OK) {
        free_matrix(Zbn);
        return fail_out(s);
      }
      if (Zb) cot.drop(Zb);
      if (Yb) cot.drop(Yb);
      Zb = Zbn;
      Yb = Ybn;
      if (Zb) cot.keep(Zb);
      if (Yb) cot.keep(Yb);
    }
  }
  if ((s = write_dense(ctx, Yb, S->rs, S->cs, dS, ld)) != CLR_OK) return fail_out(s);
  HIP_TRY(ctx, launch_mask_dense(S->view(), dS, ld, ctx->stream));
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  return CLR_OK;
}
