// Internal declarations shared by the HIP kernels and the host driver of the
// CLR block-product library (gfx950).  Nothing here is part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace clr {

// ---------------------------------------------------------------------------
// Tunables
// ---------------------------------------------------------------------------
constexpr int kSlabK = 16;            // inner indices staged in LDS per pipeline step
constexpr int kGemmThreads = 256;     // 4 waves, arranged 2 x 2 over the output tile
constexpr int kF64WaveTiles = 5;      // 16x16 MFMA tiles per wave and dimension (FP64 form)
constexpr int kF32WaveTiles = 4;      // same for the FP32-MFMA (mixed) form
constexpr int kMaxItemF64 = 32 * kF64WaveTiles;   // 160: largest output tile edge per item
constexpr int kMaxItemF32 = kMaxItemF64;          // 160: the FP32-MFMA form without correction
constexpr int kMaxItemF32Split = 32 * kF32WaveTiles;   // 128: with the hi*lo + lo*hi products
constexpr int kMaxItemOzaki = 64;                  // item edge of the INT8 (operand-split) form
constexpr int kOzMaxSlices = 7;                    // digits per operand in that form
constexpr int kRecThreads = 512;      // recompression workgroup (32 groups of 16 lanes)
constexpr int kRecLdsBytes = 140 * 1024;  // dynamic LDS for the working set (160 KiB minus bookkeeping)
constexpr int kJacobiMaxSweeps = 60;
constexpr int kCertEdge = 160;        // most columns the dense certificate examines
constexpr int kCertMaxShort = 2 * kCertEdge - 1;   // largest short edge of the column-subset form
constexpr int kCertMaxEdge = 512;    // largest block edge of the left-looking form beyond that

// The thread index, opaque to loop-invariant code motion.  Kernels that run
// one work unit after another in a persistent loop would otherwise have the
// values derived from threadIdx.x hoisted out of that loop, live across every
// phase of every unit, and spilled.  Reading the index through an empty asm
// statement makes each read a new value, so its uses stay where they are.
__device__ __forceinline__ int opaque_tid() {
  int t = threadIdx.x;
  asm volatile("" : "+v"(t));
  return t;
}

// ---------------------------------------------------------------------------
// XCD-blocked workgroup mapping: the dispatcher deals workgroups to the 8 XCDs
// round-robin, so workgroup b runs on XCD b % 8; unit u = (b % 8) * per + b / 8
// gives each XCD a contiguous run of `per` units (neighbouring units share an
// L2).  per comes from the grid, or, for a launch sized by a capacity, from the
// live count n: workgroups past the runs get -1.
__device__ inline int xcd_unit(int n, bool from_count) {
  const int per = from_count ? (n + 7) / 8 : (int)gridDim.x / 8;
  const int l = (int)blockIdx.x / 8;
  if (l >= per) return -1;
  return (int)(blockIdx.x % 8) * per + l;
}

// Work descriptors (device resident, built by the planning kernels)
// ---------------------------------------------------------------------------

// One term of a grouped GEMM item:  scale * L (m x k) * R (k x n) where
// L(i, kk) = L[i*sLi + kk*sLk] and R(kk, j) = R[kk*sRk + j*sRj].  Strides are
// block-local (at most the largest block edge), so the GEMM kernel forms
// i * sLi and j * sRj in 32 bits.
struct Seg {
  const double* L;
  const double* R;
  int64_t sLi, sLk, sRk, sRj;
  int k;          // inner length of this term
  int kbase;      // inner offset of this term inside its item's concatenated inner range
  double scale;
};

// One output tile: C[row0.., col0..] (m x n, column-major, ldc) =
//   (accumulate ? C : 0) + alpha * sum_s scale_s * L_s * R_s,
// where every term's L is offset by row0 rows and R by col0 columns.
struct GemmItem {
  double* C;
  int64_t ldc;
  int row0, col0, m, n;
  int seg0, nseg;
  int ktotal;
  int accumulate;
  double alpha;
};

// A low-rank term scale * U V^T of a result block kept in factored form.
struct Piece {
  const double* U;
  const double* V;
  int64_t ldu, ldv;
  int r;
  int pad;
  double scale;
};

enum RecPath : int { kPathSkip = -1, kPathDense = 0, kPathLowRank = 1, kPathForceDense = 2 };

// Recompression of one result block (Sec. 4.1, Eqs. (5)-(7) and the rank rule).
struct RecItem {
  int path;
  int m, n;
  int piece0, npieces, R;     // low-rank path: concatenated factors
  int cert_hint;              // dense path: 1 to try the dense certificate first
  int rrqr;                   // dense path: truncate by column-pivoted QR instead of the SVD
  const double* D;            // dense path: accumulated block
  int64_t ldd;
  double tau;                 // drop threshold
  double* out;                // result slot (dense m*n, or U m*r followed by V n*r)
  double* scratch;            // global working memory when the LDS budget is exceeded
  int* kind_out;
  int* rank_out;
  double* norm_out;
};

// Doubles of working memory the recompression of one block needs, and how much
// of it must come from global scratch (when it exceeds the LDS budget).
__host__ __device__ inline int64_t rec_work_doubles(int path, int m, int n, int R) {
  if (path == kPathLowRank) return (int64_t)(m + n) * R + 2 * (int64_t)R * R + 2 * (int64_t)R;
  return (int64_t)m * n;
}
__host__ __device__ inline int64_t rec_scratch_doubles(int path, int m, int n, int R, double tol) {
  if (path == kPathSkip || path == kPathForceDense) return 0;
  if (path == kPathDense && tol == 0.0) return 0;
  const int64_t w = rec_work_doubles(path, m, n, R);
  return w * 8 > (int64_t)kRecLdsBytes ? w : 0;
}

// Per-block plan produced by the symbolic phase of a product.
enum PlanCounter : int {
  kCntSegDense = 0,   // terms of the dense accumulation GEMM (densified blocks)
  kCntPieces,         // low-rank pieces (blocks kept in factored form)
  kCntThin1,          // thin factor products, first launch
  kCntThin2,          // thin factor products that consume a core Z (second launch)
  kCntPool,           // doubles of thin-product output
  kCntScratch,        // doubles of recompression scratch
  kCntComputed,       // 1 if the block passed screening
  kCntGemmItems,      // output tiles of the dense accumulation GEMM
  kCntCombDense,      // dense parts of a combination a X + b Y + c I (zero in a product)
  kCntOut,            // doubles of the output block's room (its largest possible storage)
  kCntAcc,            // doubles of the dense accumulator of a densified block
  kNumCounters
};

// Work-list lengths that stay on the device (a captured graph replays the
// pipeline without reading them back).  live[0 .. kNumCounters) are the
// lengths the launches use, live[kLiveOverflow] is set once a length exceeded
// its capacity (from then on every length reads 0, so nothing runs past a
// list's end), and live[kLiveNeed + c] keeps the largest length of counter c
// seen, for growing the capacities.
constexpr int kLiveOverflow = kNumCounters;
constexpr int kLiveNeed = kNumCounters + 1;
constexpr int kNumLive = 2 * kNumCounters + 1;
struct Caps {
  int64_t c[kNumCounters];
};

// Floating-point per-block statistics of the symbolic phase.
enum PlanStat : int {
  kStEst = 0, kStFlopsDD, kStFlopsLD, kStFlopsDL, kStFlopsLL, kStFlopsDensify,
  kStNDD, kStNLD, kStNDL, kStNLL, kStCandidate, kNumStats
};

// Device view of a CLR matrix's metadata and arena.
// Block b = I * ncb + J of a matrix is stored at arena + boff[b]: a dense
// block as m x n column-major, a factored block as U (m x r) followed by
// V (n x r).  The offsets are free: packed (a block takes exactly what it
// stores), dense-slot (every block has room for m x n) or upper bounds
// planned on the device before a product runs.
struct MatView {
  const int* kind;      // nrb*ncb
  const int* rank;
  const double* norm;
  const int* roff;      // nrb+1
  const int* coff;      // ncb+1
  const double* arena;
  const int64_t* boff;  // nrb*ncb block offsets into arena (doubles)
  int nrb, ncb;
};

__device__ inline const double* block_at(const MatView& M, int b) { return M.arena + M.boff[b]; }

// Elements a block of the given kind stores.
__host__ __device__ inline int64_t stored_size(int kind, int m, int n, int r) {
  return kind == 1 ? (int64_t)m * n : kind == 2 ? (int64_t)(m + n) * r : 0;
}

// Split `extent` into at most ceil(extent/maxe) parts on 16-element boundaries.
__host__ __device__ inline int num_parts(int extent, int maxe) {
  return (extent + maxe - 1) / maxe;
}
__host__ __device__ inline void part_range(int extent, int parts, int p, int* start, int* len) {
  const int tiles = (extent + 15) / 16;
  const int base = tiles / parts, extra = tiles % parts;
  const int t0 = p * base + (p < extra ? p : extra);
  const int tn = base + (p < extra ? 1 : 0);
  int s = t0 * 16, e = (t0 + tn) * 16;
  if (e > extent) e = extent;
  *start = s;
  *len = e - s;
}

// Item edges per shape class.  Dense-accumulation items are classed by the
// block's longer edge: (0, 32], (32, 64], (64, 96], (96, 128], (128, 160],
// above 160; factor-product (thin) items by the narrow extent of their output,
// which is a rank: (0, 8], (8, 16], (16, 32], (32, 64], above 64.  A block is
// split into items of at most its class's edge on 16-element boundaries.
constexpr int kDenseClasses = 6;
constexpr int kThinClasses = 5;
struct EdgeTable {
  int dense[kDenseClasses];
  int thin[kThinClasses];
};
__host__ __device__ inline int dense_class(int m, int n) {
  const int e = m > n ? m : n;
  return e <= 32 ? 0 : e <= 64 ? 1 : e <= 96 ? 2 : e <= 128 ? 3 : e <= 160 ? 4 : 5;
}
__host__ __device__ inline int thin_class(int rows, int cols) {
  const int r = rows < cols ? rows : cols;
  return r <= 8 ? 0 : r <= 16 ? 1 : r <= 32 ? 2 : r <= 64 ? 3 : 4;
}
__host__ __device__ inline int dense_edge(const EdgeTable& E, int m, int n) {
  return E.dense[dense_class(m, n)];
}
__host__ __device__ inline int thin_edge(const EdgeTable& E, int rows, int cols) {
  return E.thin[thin_class(rows, cols)];
}

struct PlanParams {
  MatView A, B;
  int nrb, ncb, nkb;
  double eps_sp;
  int screen;     // 0 absolute, 1 per area
  double alpha;
  double tol;
  int square;     // C's row and column blockings are identical
  EdgeTable edges;    // item edges of the dense-accumulation and factor-product launches
  const int* mask_kind;   // optional: only blocks stored in this kind table are computed
  // nonzero blocks of A's block rows and B's block columns, inner index K
  // ascending: row I's at a_idx + I * nkb (a_cnt[I] of them), column J's at
  // b_idx + J * nkb (b_cnt[J]); built by launch_block_lists
  const int* a_cnt;
  const int* a_idx;
  const int* b_cnt;
  const int* b_idx;
};

// Ints of the block lists of a product with nrb x nkb and nkb x ncb blockings.
inline int64_t block_list_ints(int nrb, int ncb, int nkb) {
  return (int64_t)(nrb + ncb) * (1 + (int64_t)nkb);
}
// The lists inside a buffer of block_list_ints ints.
inline void bind_block_lists(PlanParams& P, int* base) {
  int* a_cnt = base;
  int* b_cnt = a_cnt + P.nrb;
  int* a_idx = b_cnt + P.ncb;
  int* b_idx = a_idx + (int64_t)P.nrb * P.nkb;
  P.a_cnt = a_cnt;
  P.b_cnt = b_cnt;
  P.a_idx = a_idx;
  P.b_idx = b_idx;
}

struct FillParams {
  const int64_t* off;     // [kNumCounters][npairs]
  const int64_t* cnt;
  const int* flags;
  Seg* seg_dense;
  GemmItem* items_dense;
  Seg* seg_thin1;
  GemmItem* items_thin1;
  Seg* seg_thin2;
  GemmItem* items_thin2;
  Piece* pieces;
  RecItem* rec;
  double* pool;
  double* scratch;
  double* acc;            // dense accumulators (a block's at its kCntAcc offset)
  double* c_arena;        // output room (a block's at its kCntOut offset)
  int64_t* c_boff;        // output block offsets, written for every block
  int* c_kind;
  int* c_rank;
  double* c_norm;
  const int64_t* abort;   // optional: nothing is written while *abort != 0
};

enum : int { kFlagComputed = 1, kFlagDensify = 2, kFlagForce = 4 };

// Dense part of one block of a X + b Y + c I.
struct AxpbyDenseItem {
  double* D;
  const double* X;   // dense block of X or null
  const double* Y;   // dense block of Y or null
  double a, b, c;
  int m, n;
};

// Blockwise combination T = a X + b Y + c I planned on the device: one thread
// per block decides screening and path and counts its work (k_comb_count);
// after the scan, k_comb_fill writes the lists at the offsets.
struct CombParams {
  MatView X, Y;           // Y.kind null when there is no Y
  double a, b, c;
  int square;             // X is square-blocked (the identity term lives on diagonal blocks)
  double eps_sp;
  int screen;
  double tol;
  EdgeTable edges;        // item edges of the low-rank-term GEMM items (dense classes)
  double* acc;            // dense accumulators (a block's at its kCntAcc offset)
  double* t_arena;        // output room (a block's at its kCntOut offset)
  int64_t* t_boff;        // output block offsets, written for every block
  int* t_kind;
  int* t_rank;
  double* t_norm;
};
struct CombLists {
  const int64_t* off;     // [kNumCounters][nblocks]
  const int64_t* cnt;
  AxpbyDenseItem* dense;
  Seg* segs;
  GemmItem* items;
  Piece* pieces;
  RecItem* rec;
  double* scratch;
  const int64_t* abort;   // optional, as in FillParams
};

// ---------------------------------------------------------------------------
// Kernel launchers (defined in the .hip files)
// ---------------------------------------------------------------------------
// order: optional item permutation (workgroup b runs item order[b]), e.g.
// from launch_item_order; null keeps the XCD-blocked order.
// live: optional device-resident item count; the launch covers nitems
// items (its capacity) and the kernels stop at min(nitems, *live).
// next: optional device counter, zero at launch: the LDS kernel runs
// persistent (one workgroup per CU taking list slots from it).
hipError_t launch_ggemm_f64(const GemmItem* items, const Seg* segs, int nitems, hipStream_t s,
                            bool dense = false, const int* order = nullptr,
                            const int64_t* live = nullptr, int* next = nullptr);
hipError_t launch_wgemm_f64(const GemmItem* items, const Seg* segs, int nitems, hipStream_t s,
                            const int* order = nullptr, const int64_t* live = nullptr);
hipError_t launch_wgemm_f32(const GemmItem* items, const Seg* segs, int nitems, int split,
                            hipStream_t s, const int* order = nullptr,
                            const int64_t* live = nullptr);
constexpr int kMaxItemThin = 64;   // largest edge of a wave-per-item (thin) GEMM item
hipError_t launch_ggemm_f32(const GemmItem* items, const Seg* segs, int nitems, int split,
                            hipStream_t s, bool dense = false, const int* order = nullptr,
                            const int64_t* live = nullptr, int* next = nullptr);
// Workgroups of a persistent launch over nitems items: per_cu per CU.
int persistent_grid(int nitems, int per_cu = 1);
// Items of the LDS grouped GEMM by decreasing estimated cost (slabs times the
// busiest wave's tiles, in quarter-octave classes) into order[0 .. nitems).
hipError_t launch_item_order(const GemmItem* items, int nitems, int* order, hipStream_t s,
                             const int64_t* live = nullptr);
// Dense accumulation on INT8 MFMA with `slices` digits per operand (2..7);
// items of at most kMaxItemOzaki x kMaxItemOzaki.
hipError_t launch_ggemm_ozaki(const GemmItem* items, const Seg* segs, int nitems, int slices,
                              hipStream_t s, const int* order = nullptr);
// Items of the wave-per-item GEMM grouped by their first term's left operand
// (the dense block of a low-rank x dense product), so that the items reading
// one block run next to each other: a radix sort of the operand addresses.
// work must hold operand_order_bytes(nitems) bytes.
size_t operand_order_bytes(int nitems);
// Dense kernel matrix (clr_kernel_matrix): kind 0 exp(-a r^2), 1 1/sqrt(r^2 + a^2).
hipError_t launch_kernel_matrix(const double* xr, int64_t nr, const double* xc, int64_t nc,
                                int dim, int kind, double a, double diag, double* out,
                                int64_t ld, hipStream_t s);
hipError_t launch_operand_order(const GemmItem* items, const Seg* segs, int nitems, void* work,
                                int* order, hipStream_t s);
// The same grouping by a hashed counting sort in one workgroup (no library
// call, no workspace): order[0 .. min(nitems, *live)) for recorded launches.
hipError_t launch_operand_group(const GemmItem* items, const Seg* segs, int nitems, int* order,
                                hipStream_t s, const int64_t* live = nullptr);
// Per item, 1 if a dense-path block is proved to stay dense (kept rank above
// half its short edge), else 0; count (optional) is incremented per proof.
hipError_t launch_dense_cert(const RecItem* items, int nitems, double tol, int* cert,
                             unsigned long long* count, hipStream_t s,
                             const int64_t* live = nullptr);
// Device-side statistics of one recompression launch (zeroed by the caller).
struct RecCounters {
  double flops_bidiag;              // 4 p q^2 - 4 q^3 / 3 per block the register engine reduces
  unsigned long long certified;     // blocks proved dense without an SVD
};
// order: workspace of nitems + 1 ints; when given, the register engine runs
// its blocks in decreasing order of estimated cost, persistent (one workgroup
// per CU taking list slots from the counter in the last int); null: one
// workgroup per block in the XCD-blocked order.
// cert: workspace of nitems + 3 ints; when given, dense-path blocks are
// first tested by the dense certificate (persistent launches, their counters
// in the last three ints) and the proved ones are copied out without an SVD.  ctr (optional) receives the launch's counters.
hipError_t launch_recompress(const RecItem* items, const Piece* pieces, int nitems, double tol,
                             int* status, GemmItem* gout, Seg* gseg, int* order, int* cert,
                             RecCounters* ctr, hipStream_t s, hipEvent_t engine_begin = nullptr,
                             hipEvent_t engine_end = nullptr, const int64_t* live = nullptr);
// Sparse block lists of A's rows and B's columns into `base`, the buffer
// bind_block_lists bound P's list pointers to.
hipError_t launch_block_lists(const PlanParams& P, int* base, hipStream_t s);
hipError_t launch_symbolic(const PlanParams& P, int64_t* cnt, double* st, int* flags,
                           hipStream_t s);
hipError_t launch_scan(const int64_t* in, int64_t* out, int64_t n, int narrays, int64_t* totals,
                       hipStream_t s);
hipError_t launch_reduce(const double* in, int64_t n, int narrays, double* totals, hipStream_t s);
hipError_t launch_fill(const PlanParams& P, const FillParams& F, hipStream_t s);
hipError_t launch_add_base(int64_t* off, int64_t n, int narrays, const int64_t* base,
                           hipStream_t s);
// Capacity check of one pipeline run (after the scan wrote totals): the live
// lengths become the totals, or 0 once any total exceeds its capacity.
hipError_t launch_caps(const int64_t* totals, const Caps& caps, int64_t* live, hipStream_t s);
// acc[0] += the flop totals (kStFlops*) of one product, on the device.
hipError_t launch_add_flops(const double* tot_st, double* acc, hipStream_t s);
hipError_t launch_comb_count(const CombParams& P, int64_t* cnt, hipStream_t s);
hipError_t launch_comb_fill(const CombParams& P, const CombLists& L, hipStream_t s);
hipError_t prepare_recompress();
hipError_t launch_ingest(const MatView& M, double* arena, const double* const* f0,
                         const double* const* f1, double* norm_out, hipStream_t s);
hipError_t launch_to_dense(const MatView& M, double* out, int64_t ld, hipStream_t s);
hipError_t launch_scale(const MatView& M, double* arena, double* norm, double sc, hipStream_t s);
hipError_t launch_identity_terms(const MatView& M, double* out, hipStream_t s);
hipError_t launch_axpby_dense(const void* items, int n, hipStream_t s,
                              const int64_t* live = nullptr);
// out[0] = sqrt(sum of n terms) / sqrt(rows) on the device (one workgroup).
hipError_t launch_residual_finish(const double* terms, int64_t n, double rows, double* out,
                                  hipStream_t s);
hipError_t launch_fill_i32(int* p, int v, int64_t n, hipStream_t s);
hipError_t launch_from_dense(const MatView& M, double* arena, int* kind, int* rank, double* norm,
                             const double* D, int64_t ld, const int* mask_kind, hipStream_t s);
hipError_t launch_transpose(const MatView& A, const MatView& T, double* tarena, int* tkind,
                            int* trank, double* tnorm, hipStream_t s);
hipError_t launch_mask_dense(const MatView& M, double* out, int64_t ld, hipStream_t s);
// Copy every block's stored elements from src to dst_arena + dst_boff[b]
// (same blocking, kinds and ranks; the two layouts must not overlap).
hipError_t launch_relayout(const MatView& src, double* dst_arena, const int64_t* dst_boff,
                           hipStream_t s);
hipError_t launch_fill_f64(double* p, double v, int64_t n, hipStream_t s);
// Measurement kernels (k_peaks.hip): a chain of FP64 MFMAs per wave (4 waves
// per workgroup) and a plain copy of n_doubles (even) doubles.
double mfma_loop_flops(int blocks, int iters);
hipError_t launch_mfma_loop(int blocks, int iters, double* sink, hipStream_t s);
hipError_t launch_copy(const double* src, double* dst, int64_t n_doubles, hipStream_t s);

}  // namespace clr
