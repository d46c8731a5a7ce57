/*
 * clr.h - C ABI of the MI355X (gfx950) library for products of clustered
 * low-rank (CLR) block-rank-sparse matrices and the Newton-Schulz square-root
 * inverse built on them.
 *
 * Method: Calvin, Lewis & Valeev, "Scalable Task-Based Algorithm for
 * Multiplication of Block-Rank-Sparse Matrices" (IA^3 2015), Sec. 4.1 (CLR
 * representation, Eqs. (4)-(7), screening) and Sec. 4.2 (Eqs. (8)-(11)).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - All numeric payload is IEEE double, column-major.  A dense block of an
 *   m x n block is m x n with leading dimension m; a low-rank block is a pair
 *   U (m x r, ld m) and V (n x r, ld n) with value U V^T.
 * - Block metadata arrays (kind, rank, norm) are row-major over the block grid:
 *   entry I * ncb + J describes block (I, J).  kind: 0 zero, 1 dense, 2 low rank.
 * - Pointers documented as "device" must point to memory of the device that
 *   was current when the context was created; "host" pointers are plain CPU
 *   memory.  The library never retains caller pointers after a call returns.
 * - Every call is enqueued on the context's stream.  Calls that return host
 *   data, and calls whose output sizes depend on results (clr_gemm,
 *   clr_compress, clr_sqrt_inv and the backward calls), synchronise that
 *   stream.
 * - A failing call returns a status other than CLR_OK, leaves any output
 *   handle set to NULL, and records a message retrievable by clr_last_error().
 *   No C++ exception crosses this interface.
 * - A context and the matrices created from it are used by one host thread at
 *   a time.
 */
#ifndef CLR_H
#define CLR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct clr_context clr_context;
typedef struct clr_matrix clr_matrix;
typedef struct clr_plan clr_plan;

typedef enum {
  CLR_OK = 0,
  CLR_ERR_INVALID_ARG = 1,   /* null handle, negative size, bad option value        */
  CLR_ERR_SHAPE = 2,         /* inner blockings of a product differ                 */
  CLR_ERR_CAPACITY = 3,      /* a size exceeds what the library supports            */
  CLR_ERR_NONFINITE = 4,     /* a block norm is NaN or infinite                     */
  CLR_ERR_NOT_CONVERGED = 5, /* S^-1/2: stopped without meeting conv_tol            */
  CLR_ERR_HIP = 6,           /* a HIP runtime call failed                           */
  CLR_ERR_NORM_MISMATCH = 7, /* caller norms disagree with the recomputed ones      */
  CLR_ERR_DIVERGED = 8,      /* S^-1/2: ||X_n - I|| grew in two consecutive steps   */
  CLR_ERR_INTERNAL = 9       /* a kernel reported an inconsistent state             */
} clr_status;

/* Block products in FP64 MFMA; FP32 MFMA with FP64 accumulation (MIXED); or
 * the dense accumulation on INT8 MFMA by operand splitting (OZAKI: every
 * 64-deep chunk of an operand row / column scaled by a power of two and cut
 * into `split` signed 7-bit digits, digit products summed exactly in int32,
 * groups added in FP64; factor products stay FP64).  Recompression and
 * convergence checks are FP64 in every form.                                */
typedef enum { CLR_FP64 = 0, CLR_MIXED = 1, CLR_OZAKI = 2 } clr_precision;

/* Truncating factorisation of clr_compress (Sec. 4.1): the truncated SVD
 * (default) or the paper's rank-revealing QR with column pivoting.          */
typedef enum { CLR_COMPRESS_SVD = 0, CLR_COMPRESS_RRQR = 1 } clr_compression;

/* Kernels of clr_kernel_matrix: the overlap-like exp(-a r^2) and the
 * Coulomb-like 1 / sqrt(r^2 + a^2) stand-ins for the paper's test matrices
 * (Sec. 4.2: overlap and Coulomb matrices of water clusters).                */
typedef enum { CLR_KERNEL_GAUSSIAN = 0, CLR_KERNEL_COULOMB = 1 } clr_kernel;

/* Screening threshold tau of a result block (I, J) of size m x n (Sec. 4.1,
 * last paragraph): ABS uses tau = eps_sp, AREA uses tau = eps_sp * m * n.    */
typedef enum { CLR_SCREEN_ABS = 0, CLR_SCREEN_AREA = 1 } clr_screen_mode;

typedef struct {
  double tol;      /* relative truncation tolerance per block; 0 = no truncation       */
  double eps_sp;   /* screening threshold (see clr_screen_mode)                        */
  int screen;      /* clr_screen_mode                                                  */
  int precision;   /* clr_precision: block products in FP64, or FP32 MFMA with the
                      FP32 partials added into FP64 every 32 inner indices of the dense
                      accumulation (every 8 of the factor products) (MIXED)            */
  int split;       /* MIXED: 1 adds the hi*lo and lo*hi correction products, 0 uses
                      the FP32-rounded operands alone.  OZAKI: digits per operand,
                      2..7 (0 selects 7, near FP64 accuracy)                           */
  double alpha;    /* result is alpha * A * B (screening estimate scaled by |alpha|)   */
} clr_gemm_opts;

typedef struct {
  clr_gemm_opts g;     /* options of every product of the iteration                    */
  double alpha;        /* scaling of Eq. (8); 0 selects 1 / max_I sum_J ||S_IJ||_F      */
  double conv_tol;     /* target of ||X_n - I||_F/sqrt(N) and of ||W S W - I||_F/sqrt(N) */
  int max_iter;        /* iteration cap when fixed_iters == 0                          */
  int fixed_iters;     /* > 0: run exactly this many iterations, no stopping test       */
  /* Precision schedule of the reduced-precision forms (g.precision != CLR_FP64).
   * reduced_below == 0: every product in g.precision.  reduced_below > 0: the
   * products run in FP64 until an iteration ends with ||X_n - I||_F/sqrt(N) <=
   * reduced_below; from the next iteration on, X_n = alpha Y_n Z_n stays FP64
   * and the other three products run in g.precision.                          */
  double reduced_below;
  /* With reduced_below > 0 and correction != 0, those later iterations form
   * Eqs. (9)-(11) through D_n = T_n - I = -E_n / 2 + 3 E_n^2 / 8, E_n = X_n - I
   * (the same T_n in exact arithmetic): Z_{n+1} = Z_n + Z_n D_n and
   * Y_{n+1} = Y_n + D_n Y_n, the sums and E_n, D_n recompressed in FP64.  The
   * reduced-precision products E_n^2, Z_n D_n, D_n Y_n then carry the small
   * D_n, so their rounding scales with ||X_n - I|| instead of ||T_n||.        */
  int correction;
  /* graph != 0: one iteration (the four products of Eqs. (8)-(11), the
   * combination of Eq. (9) and the block terms of ||X_n - I||) is recorded
   * once as a HIP graph and replayed, each replay with no host read-back or
   * allocation inside.  The first iteration runs directly and measures its
   * work-list lengths; the lists of the graph get graph_margin (0 selects 2)
   * times those lengths.  A replay whose lists would exceed their capacity is
   * detected on the device (nothing runs past a list's end); that iteration
   * is redone directly and the graph recorded again with capacities of at
   * least twice the lengths seen (stats: graph_replays + graph_captures / 2
   * equals the iteration count).  The results equal those with
   * graph == 0 bit for bit.  Needs
   * reduced_below == 0 and g.precision FP64 or MIXED.  The graph's fixed
   * iterates are allocated for the call; its work lists stay with the context
   * (grown as needed, released by clr_context_destroy).                      */
  int graph;
  double graph_margin;
} clr_sqrtinv_opts;

typedef struct {
  int64_t candidates;   /* result blocks with at least one nonzero pair              */
  int64_t computed;     /* of those, passed the screening test                        */
  int64_t dropped;      /* computed but below tau after accumulation                  */
  int64_t triples;      /* block products formed                                      */
  int64_t n_dd, n_ld, n_dl, n_ll;
  int64_t out_dense, out_lowrank;
  int64_t densified;    /* result blocks accumulated densely                          */
  double flops_dd, flops_ld, flops_dl, flops_ll; /* 2mkn, 2r k n, 2 m k r, 2k rA rB + 2 side rA rB */
  double flops_densify; /* 2 m n r for low-rank terms added into dense accumulators   */
  double flops_products;/* sum of the five above                                      */
  double bytes_compulsory; /* stored elements of A, B and C, 8 bytes each             */
  double ms_symbolic, ms_products, ms_recompress, ms_total; /* device time per phase */
  double ms_thin;       /* launches of the thin factor products (LD, DL, LL terms)     */
  double ms_dense;      /* launch of the dense accumulation GEMM (DD + densified terms) */
  double flops_rec_engine; /* Golub-Van Loan bidiagonalisation count 4 p q^2 - 4 q^3 / 3
                              (p >= q the block edges) of the blocks the register-resident
                              SVD kernel bidiagonalises                                 */
  double ms_rec_engine; /* device time of that kernel                                   */
  int64_t certified_dense; /* dense-accumulated blocks proved dense without an SVD      */
} clr_gemm_stats;

typedef struct {
  int iterations;
  int converged;            /* 1 when ||W S W - I||_F/sqrt(N) <= conv_tol              */
  double alpha;
  double internal_residual; /* last ||X_n - I||_F / sqrt(N)                            */
  double explicit_residual; /* ||W S W - I||_F / sqrt(N) at exit (untruncated products) */
  int n_gemms;
  double flops_products;    /* sum over every product of clr_gemm_stats.flops_products  */
  double ms_total;
  int graph_replays;        /* iterations replayed from a graph (opts.graph)            */
  int graph_captures;       /* graphs recorded (two per capacity: ping and pong)        */
} clr_sqrtinv_stats;

/* ---- context ------------------------------------------------------------ */

/* Create a context bound to the current HIP device and to `stream` (a
 * hipStream_t; NULL selects the default stream).  Owns all workspace. */
clr_status clr_context_create(clr_context** ctx, void* stream);
clr_status clr_context_destroy(clr_context* ctx);

/* The caller's device allocator for this context (for instance a framework's
 * caching allocator): alloc(bytes, stream, user) returns device memory usable
 * on `stream` (the context's stream, as given to clr_context_create) or NULL
 * when out of memory; release(ptr, bytes, stream, user) gives it back, in
 * stream order (work already queued on the stream may still read it).  Both
 * NULL restores hipMalloc.  Matrices created afterwards and the work lists
 * grown afterwards use it; memory is always released through the allocator
 * that made it, so existing matrices stay valid.  The status word, the
 * allocation-free residual's fixed array and clr_measure_peaks' buffer stay
 * on hipMalloc.  Synchronises the context stream. */
typedef void* (*clr_alloc_fn)(size_t bytes, void* stream, void* user);
typedef void (*clr_release_fn)(void* ptr, size_t bytes, void* stream, void* user);
clr_status clr_set_allocator(clr_context* ctx, clr_alloc_fn alloc, clr_release_fn release,
                             void* user);
/* Message of the last failing call on this context ("" if none).  Valid until
 * the next call on the context. */
const char* clr_last_error(const clr_context* ctx);
const char* clr_status_string(clr_status s);

/* ---- matrices (Sec. 4.1: the CLR representation) ------------------------- */

/* Build a CLR matrix from given factors, copied into a library-owned arena.
 *   row_sizes[nrb], col_sizes[ncb] (host): the nonuniform blocking.
 *   kind[nrb*ncb] (host): 0 zero, 1 dense, 2 low rank.
 *   rank[nrb*ncb] (host): r of low-rank blocks, 1 <= r and (m + n) r <= m n (a factored
 *     block never stores more than its dense form, else CLR_ERR_CAPACITY); ignored otherwise.
 *   norms[nrb*ncb] (host, nullable): ||block||_F; when given they are checked
 *     against the recomputed values (relative 1e-10, else CLR_ERR_NORM_MISMATCH).
 *   f0[nrb*ncb], f1[nrb*ncb] (host arrays of device pointers): dense block or U;
 *     V for low-rank blocks.  Entries of zero blocks are ignored.
 * Sizes must be >= 1.  The stored norms are recomputed on the device.  The
 * arena is packed: it holds exactly the stored elements (m n per dense block,
 * (m + n) r per low-rank block). */
clr_status clr_create(clr_context* ctx, int nrb, const int* row_sizes, int ncb,
                      const int* col_sizes, const int8_t* kind, const int* rank,
                      const double* norms, const double* const* f0,
                      const double* const* f1, clr_matrix** out);

/* CLR form of a dense matrix (device, column-major, leading dimension ld >=
 * rows): blocks with ||block||_F < drop become zero, diagonal blocks of a
 * square blocking stay dense, every other block is truncated to relative
 * `tol` and stored dense iff its rank exceeds half of min(m, n).  The
 * truncation is the SVD's, or with CLR_COMPRESS_RRQR (clr_set_compression)
 * the paper's rank-revealing QR (Sec. 4.1): M P = Q R with column pivoting,
 * U = Q_r, V^T = R_r P^T, r the smallest rank with ||M - U V^T||_F <= tol
 * ||M||_F (the dropped rows of R). */
clr_status clr_compress(clr_context* ctx, const double* dense, int64_t ld, int nrb,
                        const int* row_sizes, int ncb, const int* col_sizes, double tol,
                        double drop, clr_matrix** out);

/* Dense kernel matrix generated on the device, the input of clr_compress
 * (the step before the product, Sec. 4.1: a matrix whose blocks are then
 * truncated).  For i < nrows, j < ncols:
 *   r2 = sum_c (x_i[c] - y_j[c])^2   (c = 0 .. dim-1, each step rounded, no FMA;
 *        sqrt and the division correctly rounded, exp within one unit in the
 *        last place)
 *   out[i + j*ld] = exp(-a r2)            (CLR_KERNEL_GAUSSIAN)
 *                 = 1 / sqrt(r2 + a^2)    (CLR_KERNEL_COULOMB, r2 starts at a^2)
 *                 + diag where i == j.
 * row_points (nrows x dim) and col_points (ncols x dim) are device, row-major;
 * pass the same pointer twice for a symmetric matrix.  out is device,
 * column-major, ld >= nrows, caller-owned.  dim is 1, 2 or 3; a must be
 * finite, >= 0 for GAUSSIAN and > 0 for COULOMB.  Enqueued on the context
 * stream; returns CLR_ERR_INVALID_ARG for a bad argument. */
clr_status clr_kernel_matrix(clr_context* ctx, const double* row_points, int64_t nrows,
                             const double* col_points, int64_t ncols, int dim, int kernel,
                             double a, double diag, double* out, int64_t ld);

clr_status clr_destroy(clr_matrix* m);

/* Device storage of m (host outputs, nullable): the arena's capacity in
 * doubles and the bytes of its one allocation (arena and block metadata).
 * Inputs from clr_create and clr_compress are packed (capacity = stored
 * elements); a product or combination reserves per block the most its result
 * can store (m n for a block accumulated densely, (m + n) R for a
 * concatenation of rank R), which clr_compact gives back. */
clr_status clr_matrix_arena(const clr_matrix* m, int64_t* capacity, size_t* bytes);

/* Repack m in place so that its arena holds exactly its stored elements
 * (Sec. 4.1: m n per dense block, (m + n) r per low-rank block).  Values,
 * kinds, ranks and norms are unchanged; the handle stays valid.  Synchronises
 * the context stream (the kinds and ranks are read back); returns
 * CLR_ERR_INVALID_ARG for a matrix of another context. */
clr_status clr_compact(clr_context* ctx, clr_matrix* m);

/* Blocking and storage summary (host outputs, all nullable). */
clr_status clr_matrix_info(const clr_matrix* m, int* nrb, int* ncb, int64_t* rows,
                           int64_t* cols, int64_t* stored_elements);
/* Block metadata copied to host arrays of nrb*ncb entries (each nullable). */
clr_status clr_get_meta(clr_context* ctx, const clr_matrix* m, int8_t* kind, int* rank,
                        double* norms);
/* Copy the factors of block (I, J) to device buffers: f0 receives the dense
 * block (m*n) or U (m*r); f1 receives V (n*r) and may be NULL for dense blocks. */
clr_status clr_get_block(clr_context* ctx, const clr_matrix* m, int I, int J, double* f0,
                         double* f1);
/* Expand to a dense device matrix (column-major, leading dimension ld >= rows). */
clr_status clr_to_dense(clr_context* ctx, const clr_matrix* m, double* out, int64_t ld);

/* ---- the product (Sec. 4.1, Eqs. (4)-(7) and the screening rule) ---------- */

/* C = alpha * A * B in CLR arithmetic: screening by norm estimates, dense x
 * dense / low-rank x dense / dense x low-rank / low-rank x low-rank block
 * products, accumulation (dense sum or factor concatenation), FP64
 * recompression by truncated SVD, and C's norm table.  A's column blocking
 * must equal B's row blocking.  `st` (nullable) receives counts and times. */
clr_status clr_gemm(clr_context* ctx, const clr_matrix* A, const clr_matrix* B,
                    const clr_gemm_opts* opts, clr_matrix** C, clr_gemm_stats* st);

/* T = a * X + b * Y + c * I blockwise with the same accumulation and
 * recompression rules (Y nullable; c applies to diagonal blocks of a square
 * blocking).  With a = -10/8, b = 3/8, c = 15/8 and Y = X*X this is Eq. (9). */
clr_status clr_axpby(clr_context* ctx, double a, const clr_matrix* X, double b,
                     const clr_matrix* Y, double c, const clr_gemm_opts* opts,
                     clr_matrix** T);

/* ---- the square-root inverse (Sec. 4.2, Eqs. (8)-(11)) -------------------- */

/* W = S^-1/2 by the coupled third-order Newton-Schulz iteration: X = alpha Y Z,
 * T = (-10 X + 3 X^2 + 15 I)/8, Z <- Z T, Y <- T Y, W = sqrt(alpha) Z.  S must be
 * square-blocked.  Stops when ||X_n - I||_F/sqrt(N) <= conv_tol and the explicit
 * residual of W is <= conv_tol, or when the explicit residual stops halving
 * (CLR_ERR_NOT_CONVERGED, W still returned), or at max_iter
 * (CLR_ERR_NOT_CONVERGED, W returned), or on growth of ||X_n - I|| in two
 * consecutive iterations (CLR_ERR_DIVERGED, no W). */
clr_status clr_sqrt_inv(clr_context* ctx, const clr_matrix* S, const clr_sqrtinv_opts* opts,
                        clr_matrix** W, clr_sqrtinv_stats* st);

/* ||X - I||_F / sqrt(N) of a square-blocked matrix (host result). */
clr_status clr_identity_residual(clr_context* ctx, const clr_matrix* X, double* out);

/* The same residual for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation):
 * writes ||X - I||_F / sqrt(N) to out[0] (device, one double, caller-owned) on
 * the context stream, without allocating and without synchronising.  The
 * per-block terms go to a fixed device array of 65536 doubles (512 KiB) that
 * every device the library runs on keeps until the process ends; X may have at
 * most 65536 blocks (else CLR_ERR_CAPACITY, nothing launched).  All calls on one
 * device share that array and overwrite it: calls that overlap on a device
 * (different streams or contexts without ordering between them) race, and the
 * caller must order them.  Errors as clr_identity_residual. */
clr_status clr_identity_residual_noalloc(clr_context* ctx, const clr_matrix* X, double* out);

/* ---- adjoints (truncation treated as the identity) ------------------------ */

/* Given dC (device, dense rows(A) x cols(B), column-major, leading dimension
 * ldc), write dA = alpha dC B^T and dB = alpha A^T dC restricted to the stored
 * blocks of A and B (entries of zero blocks are set to 0), dense column-major
 * with leading dimensions lda, ldb.  Either output may be NULL. */
clr_status clr_gemm_backward(clr_context* ctx, const clr_matrix* A, const clr_matrix* B,
                             double alpha, const double* dC, int64_t ldc, double* dA,
                             int64_t lda, double* dB, int64_t ldb);

/* Largest output-tile edge of the grouped-GEMM items of the dense-accumulation
 * launch and of the factor-product launches, per precision (CLR_FP64 or
 * CLR_MIXED) for this context: 0 (default) is the kernel's full tile (dense:
 * 160, or 128 in the mixed form with split = 1; factor products: 64, one wave
 * per item), otherwise a multiple of 16 up to 160 (a larger edge than the
 * kernel's tile is capped to it).  Sets the edge of every shape class (below).
 * Results do not depend on these edges, only the launch shapes do. */
clr_status clr_set_tile_edges(clr_context* ctx, int precision, int dense_edge, int thin_edge);

/* The same edges per shape class.  Dense-accumulation items are classed by
 * their block's longer edge: dense_edges[0..5] for (0, 32], (32, 64], (64, 96],
 * (96, 128], (128, 160] and above 160; factor-product items by the narrow
 * extent of their output (a rank): thin_edges[0..4] for (0, 8], (8, 16],
 * (16, 32], (32, 64] and above 64.  Host arrays; values as for
 * clr_set_tile_edges (0 = full tile).  clr_get_tile_classes reads them back. */
clr_status clr_set_tile_classes(clr_context* ctx, int precision, const int* dense_edges,
                                const int* thin_edges);
clr_status clr_get_tile_classes(const clr_context* ctx, int precision, int* dense_edges,
                                int* thin_edges);

/* Dense certificate (on by default).  A dense-accumulated block D (m x n,
 * q = min(m, n), h = floor(q / 2)) is stored dense when its kept rank exceeds
 * q / 2 (Sec. 4.1 rank rule), which holds as soon as s_h(D) > tol ||D||_F.
 * Before the truncated SVD, a Cholesky factorisation with diagonal pivoting of
 * D^T D (or D D^T) shifted by a rounding-safe multiple of tol^2 ||D||_F^2 tries
 * to prove s_h(D) above that bound with h + 1 columns; proved blocks are
 * copied out dense without the SVD.  Results are the same either way (the
 * proof's margin exceeds the SVD's rounding error); only the work differs.
 * Applies to products and plans created afterwards on this context. */
clr_status clr_set_dense_certificate(clr_context* ctx, int enable);

/* Measurement helper: the sustained FP64 MFMA rate of a long chain of
 * independent v_mfma_f64_16x16x4 per wave (16 waves per compute unit, operands
 * in registers), in TFLOP/s, and the bandwidth of a plain device copy of
 * 1 GiB (read + write bytes over time), in GB/s; best of three timed runs each
 * after one warm-up run.  Allocates and frees 2 GiB of device memory and
 * synchronises the context stream.  Either output may be NULL. */
clr_status clr_measure_peaks(clr_context* ctx, double* mfma_f64_tflops, double* copy_gbps);

/* Truncating factorisation of clr_compress on this context (CLR_COMPRESS_SVD,
 * the default, or CLR_COMPRESS_RRQR); products always recompress by SVD. */
clr_status clr_set_compression(clr_context* ctx, int method);

/* Autotuner: times the product A B (options as for clr_gemm; output discarded),
 * best of two runs per candidate.  First one edge per launch class (multiples
 * of 32 up to the full tile), then each shape class on its own from that choice
 * (dense classes: multiples of 32; factor-product classes: multiples of 16 up
 * to 64), keeping an edge only when it shortens its launch by more than 2 %.
 * The table stays set for this context and precision (clr_get_tile_classes).
 * Returns the launch-class edges of the first stage and the launch times (ms)
 * after the second; any output pointer may be NULL. */
clr_status clr_autotune(clr_context* ctx, const clr_matrix* A, const clr_matrix* B,
                        const clr_gemm_opts* opts, int* dense_edge, int* thin_edge,
                        double* ms_dense, double* ms_thin);

/* Batched products C_p = A_p B_p (p < nprod), each with the semantics of
 * clr_gemm (Sec. 4.1).  Planning screens every product on the device and
 * reads back all work totals once; execution runs one launch per phase for the
 * whole batch (factor products, dense accumulation, recompression), so blocks
 * of all products share each launch.
 *
 * clr_plan_create allocates the nprod outputs C[p] (owned by the caller, freed
 * with clr_destroy) and the plan's own work buffers.  A, B and C must stay
 * alive, with unchanged block structure (kinds and ranks), while the plan is
 * executed.  Screening, the block products and the accumulation paths are
 * fixed at planning time from the block norms the operands have then: an
 * execution computes the values of the planned blocks from the operands'
 * current factors (recompression and truncation are redone from those
 * values), so it equals clr_gemm of the current operands whenever their block
 * norms are the planning-time ones, for instance after the factors are
 * rewritten with values of the same norms.  Operands whose norms changed
 * need a new plan.  With use_graph != 0
 * the execution phase is recorded once as a HIP graph on the context stream
 * and clr_plan_execute replays it.  clr_plan_execute writes C and, if st is
 * given, aggregated counts and flops and the device time of the execution
 * (ms_total).  On error the outputs are NULL (create) or unspecified
 * (execute).  clr_gemm_batch = create (no graph) + execute + destroy. */
clr_status clr_plan_create(clr_context* ctx, int nprod, const clr_matrix* const* A,
                           const clr_matrix* const* B, const clr_gemm_opts* opts, int use_graph,
                           clr_plan** plan, clr_matrix** C);
clr_status clr_plan_execute(clr_context* ctx, clr_plan* plan, clr_gemm_stats* st);
clr_status clr_plan_destroy(clr_plan* plan);
clr_status clr_gemm_batch(clr_context* ctx, int nprod, const clr_matrix* const* A,
                          const clr_matrix* const* B, const clr_gemm_opts* opts, clr_matrix** C,
                          clr_gemm_stats* st);

/* dS of L = sum(Wbar .* W) for W from `iters` unrolled iterations (alpha held
 * constant, truncation treated as the identity), restricted to S's stored
 * blocks.  Wbar and dS are dense device matrices N x N with leading dimension
 * ld.  Iterates are re-computed from checkpoints kept every
 * `checkpoint_every` iterations.  W (nullable) receives the forward result.
 * The iteration is unrolled as printed: opts->reduced_below and
 * opts->correction must be 0 (CLR_ERR_INVALID_ARG otherwise). */
clr_status clr_sqrt_inv_backward(clr_context* ctx, const clr_matrix* S,
                                 const clr_sqrtinv_opts* opts, int iters,
                                 int checkpoint_every, const double* Wbar, double* dS,
                                 int64_t ld, clr_matrix** W);

#ifdef __cplusplus
}
#endif
#endif /* CLR_H */
