// Elementwise and per-block helper kernels of the CLR library: ingest of
// caller factors into the slot arena with exact block norms, expansion to a
// dense matrix, scaling, the blockwise terms of ||X - I||_F, the dense part of
// the blockwise combination a X + b Y + c I, and the blockwise transpose,
// dense ingest and structure masking used by the adjoints.
#include <hipcub/hipcub.hpp>

#include "clr_internal.h"

namespace clr {

__device__ double wg_sum(double v, double* red) {
  const int tid = threadIdx.x;
  red[tid] = v;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (tid < s) red[tid] += red[tid + s];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

// Copy caller factors into the arena and compute exact block norms
// (dense: sqrt(sum d^2); low rank: sqrt(sum (U V^T)_ij^2)).
__global__ __launch_bounds__(256) void k_ingest(MatView M, double* arena, const double* const* f0,
                                                const double* const* f1, double* norm_out) {
  __shared__ double red[256];
  const int blk = blockIdx.x;
  const int I = blk / M.ncb, J = blk % M.ncb;
  const int kind = M.kind[blk];
  if (kind == 0) {
    if (threadIdx.x == 0) norm_out[blk] = 0.0;
    return;
  }
  const int m = M.roff[I + 1] - M.roff[I];
  const int n = M.coff[J + 1] - M.coff[J];
  double* dst = arena + M.boff[blk];
  double part = 0.0;
  if (kind == 1) {
    const double* src = f0[blk];
    for (int64_t e = threadIdx.x; e < (int64_t)m * n; e += 256) {
      const double v = src[e];
      dst[e] = v;
      part += v * v;
    }
  } else {
    const int r = M.rank[blk];
    const double* u = f0[blk];
    const double* v = f1[blk];
    for (int64_t e = threadIdx.x; e < (int64_t)m * r; e += 256) dst[e] = u[e];
    for (int64_t e = threadIdx.x; e < (int64_t)n * r; e += 256) dst[(int64_t)m * r + e] = v[e];
    for (int64_t e = threadIdx.x; e < (int64_t)m * n; e += 256) {
      const int i = (int)(e % m), j = (int)(e / m);
      double s = 0.0;
      for (int c = 0; c < r; ++c) s += u[i + (int64_t)c * m] * v[j + (int64_t)c * n];
      part += s * s;
    }
  }
  const double tot = wg_sum(part, red);
  if (threadIdx.x == 0) norm_out[blk] = sqrt(tot);
}

// out (rows x cols, column-major, ld) = dense expansion of M.
__global__ __launch_bounds__(256) void k_to_dense(MatView M, double* out, int64_t ld) {
  const int blk = blockIdx.x;
  const int I = blk / M.ncb, J = blk % M.ncb;
  const int m = M.roff[I + 1] - M.roff[I];
  const int n = M.coff[J + 1] - M.coff[J];
  const int kind = M.kind[blk];
  const double* src = block_at(M, blk);
  double* dst = out + M.roff[I] + (int64_t)M.coff[J] * ld;
  const int r = kind == 2 ? M.rank[blk] : 0;
  for (int64_t e = threadIdx.x; e < (int64_t)m * n; e += 256) {
    const int i = (int)(e % m), j = (int)(e / m);
    double v = 0.0;
    if (kind == 1) {
      v = src[e];
    } else if (kind == 2) {
      const double* u = src;
      const double* w = src + (int64_t)m * r;
      for (int c = 0; c < r; ++c) v += u[i + (int64_t)c * m] * w[j + (int64_t)c * n];
    }
    dst[i + (int64_t)j * ld] = v;
  }
}

// M <- s * M  (dense blocks and U factors scaled; norms by |s|).
__global__ __launch_bounds__(256) void k_scale(MatView M, double* arena, double* norm, double s) {
  const int blk = blockIdx.x;
  const int kind = M.kind[blk];
  if (kind == 0) return;
  const int I = blk / M.ncb, J = blk % M.ncb;
  const int m = M.roff[I + 1] - M.roff[I];
  const int n = M.coff[J + 1] - M.coff[J];
  double* dst = arena + M.boff[blk];
  const int64_t cnt = kind == 1 ? (int64_t)m * n : (int64_t)m * M.rank[blk];
  for (int64_t e = threadIdx.x; e < cnt; e += 256) dst[e] *= s;
  if (threadIdx.x == 0) norm[blk] = fabs(s) * norm[blk];
}

// Per-block term of ||X - I||_F^2: diagonal blocks exactly, others by their stored norm.
__global__ __launch_bounds__(256) void k_identity_terms(MatView M, double* out) {
  __shared__ double red[256];
  const int blk = blockIdx.x;
  const int I = blk / M.ncb, J = blk % M.ncb;
  const int kind = M.kind[blk];
  const int m = M.roff[I + 1] - M.roff[I];
  const int n = M.coff[J + 1] - M.coff[J];
  if (I != J) {
    if (threadIdx.x == 0) out[blk] = kind == 0 ? 0.0 : M.norm[blk] * M.norm[blk];
    return;
  }
  const double* src = block_at(M, blk);
  const int r = kind == 2 ? M.rank[blk] : 0;
  double part = 0.0;
  for (int64_t e = threadIdx.x; e < (int64_t)m * n; e += 256) {
    const int i = (int)(e % m), j = (int)(e / m);
    double v = 0.0;
    if (kind == 1) {
      v = src[e];
    } else if (kind == 2) {
      for (int c = 0; c < r; ++c) v += src[i + (int64_t)c * m] * src[(int64_t)m * r + j + (int64_t)c * n];
    }
    if (i == j) v -= 1.0;
    part += v * v;
  }
  const double tot = wg_sum(part, red);
  if (threadIdx.x == 0) out[blk] = tot;
}

// out[0] = sqrt(sum_b terms[b]) / sqrt(rows): the identity residual from the
// per-block terms of k_identity_terms, summed on the device by one workgroup
// (each thread a strided subset in index order, then a fixed tree).
__global__ __launch_bounds__(256) void k_residual_finish(const double* __restrict__ terms,
                                                         int64_t n, double rows,
                                                         double* __restrict__ out) {
  __shared__ double red[256];
  double part = 0.0;
  for (int64_t b = threadIdx.x; b < n; b += 256) part += terms[b];
  const double tot = wg_sum(part, red);
  if (threadIdx.x == 0) out[0] = sqrt(tot) / sqrt(rows);
}

// D = a X + b Y + c I over the dense parts of one block.
__global__ __launch_bounds__(256) void k_axpby_dense(const AxpbyDenseItem* items,
                                                     const int64_t* __restrict__ live) {
  if (live && (int64_t)blockIdx.x >= *live) return;
  const AxpbyDenseItem it = items[blockIdx.x];
  for (int64_t e = threadIdx.x; e < (int64_t)it.m * it.n; e += 256) {
    const int i = (int)(e % it.m), j = (int)(e / it.m);
    double v = 0.0;
    if (it.X) v += it.a * it.X[e];
    if (it.Y) v += it.b * it.Y[e];
    if (i == j) v += it.c;
    it.D[e] = v;
  }
}

__global__ void k_fill_i32(int* p, int v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}
__global__ void k_fill_f64(double* p, double v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// ---------------------------------------------------------------------------
// Adjoint helpers ------------------------------------------------------------

// Dense device matrix D (column-major, ld) -> CLR matrix with all blocks dense:
// kind 1 where the block is nonzero (and, if mask_kind is given, the mask block
// is stored), kind 0 otherwise; exact block norms.
__global__ __launch_bounds__(256) void k_from_dense(MatView M, double* arena, int* kind, int* rank,
                                                    double* norm, const double* D, int64_t ld,
                                                    const int* mask_kind) {
  __shared__ double red[256];
  const int blk = blockIdx.x;
  const int I = blk / M.ncb, J = blk % M.ncb;
  const int m = M.roff[I + 1] - M.roff[I];
  const int n = M.coff[J + 1] - M.coff[J];
  const bool keep = mask_kind == nullptr || mask_kind[blk] != 0;
  double* dst = arena + M.boff[blk];
  const double* src = D + M.roff[I] + (int64_t)M.coff[J] * ld;
  double part = 0.0;
  if (keep) {
    for (int64_t e = threadIdx.x; e < (int64_t)m * n; e += 256) {
      const int i = (int)(e % m), j = (int)(e / m);
      const double v = src[i + (int64_t)j * ld];
      dst[e] = v;
      part += v * v;
    }
  }
  const double s = wg_sum(part, red);
  if (threadIdx.x == 0) {
    const bool nz = keep && s > 0.0;
    kind[blk] = nz ? 1 : 0;
    rank[blk] = nz ? (m < n ? m : n) : 0;
    norm[blk] = nz ? sqrt(s) : 0.0;
  }
}

// T = A^T blockwise: block (J, I) of T is (A_IJ)^T; a dense block is
// transposed, a factored block U V^T becomes V U^T (factors swapped).
__global__ __launch_bounds__(256) void k_transpose(MatView A, MatView T, double* tarena, int* tkind,
                                                   int* trank, double* tnorm) {
  const int blk = blockIdx.x;
  const int I = blk / A.ncb, J = blk % A.ncb;
  const int tb = J * A.nrb + I;
  const int m = A.roff[I + 1] - A.roff[I];
  const int n = A.coff[J + 1] - A.coff[J];
  const int kind = A.kind[blk];
  if (threadIdx.x == 0) {
    tkind[tb] = kind;
    trank[tb] = A.rank[blk];
    tnorm[tb] = A.norm[blk];
  }
  if (kind == 0) return;
  const double* src = block_at(A, blk);
  double* dst = tarena + T.boff[tb];
  if (kind == 1) {
    for (int64_t e = threadIdx.x; e < (int64_t)m * n; e += 256) {
      const int j = (int)(e % n), i = (int)(e / n);   // dst is n x m, ld n
      dst[e] = src[i + (int64_t)j * m];
    }
  } else {
    const int r = A.rank[blk];
    const double* u = src;                      // m x r
    const double* v = src + (int64_t)m * r;     // n x r
    for (int64_t e = threadIdx.x; e < (int64_t)n * r; e += 256) dst[e] = v[e];
    for (int64_t e = threadIdx.x; e < (int64_t)m * r; e += 256) dst[(int64_t)n * r + e] = u[e];
  }
}

// Zero the blocks of a dense matrix (ld) whose block in the mask is not stored.
__global__ __launch_bounds__(256) void k_mask_dense(MatView M, double* out, int64_t ld) {
  const int blk = blockIdx.x;
  if (M.kind[blk] != 0) return;
  const int I = blk / M.ncb, J = blk % M.ncb;
  const int m = M.roff[I + 1] - M.roff[I];
  const int n = M.coff[J + 1] - M.coff[J];
  double* dst = out + M.roff[I] + (int64_t)M.coff[J] * ld;
  for (int64_t e = threadIdx.x; e < (int64_t)m * n; e += 256) {
    const int i = (int)(e % m), j = (int)(e / m);
    dst[i + (int64_t)j * ld] = 0.0;
  }
}

hipError_t launch_from_dense(const MatView& M, double* arena, int* kind, int* rank, double* norm,
                             const double* D, int64_t ld, const int* mask_kind, hipStream_t s) {
  const int nb = M.nrb * M.ncb;
  if (nb == 0) return hipSuccess;
  hipLaunchKernelGGL(k_from_dense, dim3(nb), dim3(256), 0, s, M, arena, kind, rank, norm, D, ld,
                     mask_kind);
  return hipGetLastError();
}
hipError_t launch_transpose(const MatView& A, const MatView& T, double* tarena, int* tkind,
                            int* trank, double* tnorm, hipStream_t s) {
  const int nb = A.nrb * A.ncb;
  if (nb == 0) return hipSuccess;
  hipLaunchKernelGGL(k_transpose, dim3(nb), dim3(256), 0, s, A, T, tarena, tkind, trank, tnorm);
  return hipGetLastError();
}
// Block b's stored elements (m n dense, (m + n) r factored) from its place in
// src to dst + dst_boff[b].
__global__ __launch_bounds__(256) void k_relayout(MatView M, double* __restrict__ dst,
                                                  const int64_t* __restrict__ dst_boff) {
  const int blk = blockIdx.x;
  const int kind = M.kind[blk];
  if (kind == 0) return;
  const int I = blk / M.ncb, J = blk % M.ncb;
  const int m = M.roff[I + 1] - M.roff[I];
  const int n = M.coff[J + 1] - M.coff[J];
  const int64_t cnt = stored_size(kind, m, n, kind == 2 ? M.rank[blk] : 0);
  const double* __restrict__ src = block_at(M, blk);
  double* __restrict__ out = dst + dst_boff[blk];
  for (int64_t e = threadIdx.x; e < cnt; e += 256) out[e] = src[e];
}

hipError_t launch_relayout(const MatView& src, double* dst_arena, const int64_t* dst_boff,
                           hipStream_t s) {
  const int nb = src.nrb * src.ncb;
  if (nb == 0) return hipSuccess;
  hipLaunchKernelGGL(k_relayout, dim3(nb), dim3(256), 0, s, src, dst_arena, dst_boff);
  return hipGetLastError();
}

hipError_t launch_mask_dense(const MatView& M, double* out, int64_t ld, hipStream_t s) {
  const int nb = M.nrb * M.ncb;
  if (nb == 0) return hipSuccess;
  hipLaunchKernelGGL(k_mask_dense, dim3(nb), dim3(256), 0, s, M, out, ld);
  return hipGetLastError();
}

hipError_t launch_ingest(const MatView& M, double* arena, const double* const* f0,
                         const double* const* f1, double* norm_out, hipStream_t s) {
  const int nb = M.nrb * M.ncb;
  if (nb == 0) return hipSuccess;
  hipLaunchKernelGGL(k_ingest, dim3(nb), dim3(256), 0, s, M, arena, f0, f1, norm_out);
  return hipGetLastError();
}
hipError_t launch_to_dense(const MatView& M, double* out, int64_t ld, hipStream_t s) {
  const int nb = M.nrb * M.ncb;
  if (nb == 0) return hipSuccess;
  hipLaunchKernelGGL(k_to_dense, dim3(nb), dim3(256), 0, s, M, out, ld);
  return hipGetLastError();
}
hipError_t launch_scale(const MatView& M, double* arena, double* norm, double sc, hipStream_t s) {
  const int nb = M.nrb * M.ncb;
  if (nb == 0) return hipSuccess;
  hipLaunchKernelGGL(k_scale, dim3(nb), dim3(256), 0, s, M, arena, norm, sc);
  return hipGetLastError();
}
hipError_t launch_identity_terms(const MatView& M, double* out, hipStream_t s) {
  const int nb = M.nrb * M.ncb;
  if (nb == 0) return hipSuccess;
  hipLaunchKernelGGL(k_identity_terms, dim3(nb), dim3(256), 0, s, M, out);
  return hipGetLastError();
}
hipError_t launch_residual_finish(const double* terms, int64_t n, double rows, double* out,
                                  hipStream_t s) {
  hipLaunchKernelGGL(k_residual_finish, dim3(1), dim3(256), 0, s, terms, n, rows, out);
  return hipGetLastError();
}
hipError_t launch_axpby_dense(const void* items, int n, hipStream_t s, const int64_t* live) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_axpby_dense, dim3(n), dim3(256), 0, s, (const AxpbyDenseItem*)items, live);
  return hipGetLastError();
}
hipError_t launch_fill_i32(int* p, int v, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}
hipError_t launch_fill_f64(double* p, double v, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_f64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Longest-first order of grouped-GEMM items.  One workgroup: a histogram of
// the items' cost classes, an exclusive scan from the most expensive class
// down, and a scatter.  The order inside a class is whatever the atomics give,
// which changes no result: every item is computed on its own.
// ---------------------------------------------------------------------------
constexpr int kOrderThreads = 1024;
constexpr int kOrderClasses = 64;

__device__ inline int item_cost_class(const GemmItem& it) {
  // slabs of 16 inner indices times (1 + tiles of the busiest wave of the
  // 2 x 4 wave grid), the per-slab overhead counted as one tile
  const int mt = (it.m + 15) >> 4, nt = (it.n + 15) >> 4;
  const int worst = min(5, (mt + 1) >> 1) * min(3, (nt + 3) >> 2);
  const double cost = (double)((it.ktotal + 15) >> 4) * (double)(worst + 1);
  const int c = cost > 1.0 ? (int)(4.0 * log2(cost)) : 0;
  return min(c, kOrderClasses - 1);
}

__global__ __launch_bounds__(kOrderThreads) void k_item_order(const GemmItem* __restrict__ items,
                                                             int n, int* __restrict__ order,
                                                             const int64_t* __restrict__ live) {
  __shared__ int cnt[kOrderClasses];
  const int tid = threadIdx.x;
  if (live) n = (int)min((int64_t)n, *live);
  if (tid < kOrderClasses) cnt[tid] = 0;
  __syncthreads();
  for (int i = tid; i < n; i += kOrderThreads) atomicAdd(&cnt[item_cost_class(items[i])], 1);
  __syncthreads();
  if (tid == 0) {
    int run = 0;
    for (int c = kOrderClasses - 1; c >= 0; --c) {
      const int k = cnt[c];
      cnt[c] = run;
      run += k;
    }
  }
  __syncthreads();
  for (int i = tid; i < n; i += kOrderThreads) order[atomicAdd(&cnt[item_cost_class(items[i])], 1)] = i;
}

hipError_t launch_item_order(const GemmItem* items, int nitems, int* order, hipStream_t s,
                             const int64_t* live) {
  if (nitems <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_item_order, dim3(1), dim3(kOrderThreads), 0, s, items, nitems, order, live);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Operand-grouped order of the wave-per-item items.  A low-rank x dense term
// reads a whole dense block for a thin result, and the same dense block
// serves every low-rank partner on the other side, so in pair order those
// reads miss L2.  Sorting the items by the address of their left operand (the
// dense block of LD and DL terms, V_A of LL cores) puts the readers of one
// block next to each other; the key is the element index of that address
// (low 32 bits: two distinct blocks sharing a key only costs locality).
// ---------------------------------------------------------------------------
namespace {
constexpr size_t align256(size_t b) { return (b + 255) & ~size_t(255); }
size_t sort_temp_bytes(int n) {
  size_t t = 0;
  (void)hipcub::DeviceRadixSort::SortPairs(nullptr, t, (const uint32_t*)nullptr, (uint32_t*)nullptr,
                                           (const int*)nullptr, (int*)nullptr, n, 0, 32);
  return t;
}
}  // namespace

__global__ __launch_bounds__(256) void k_operand_keys(const GemmItem* __restrict__ items,
                                                      const Seg* __restrict__ segs, int n,
                                                      uint32_t* __restrict__ keys,
                                                      int* __restrict__ vals) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  keys[i] = (uint32_t)((uintptr_t)segs[items[i].seg0].L >> 3);
  vals[i] = i;
}

// ---------------------------------------------------------------------------
// Kernel-generated dense matrix.  Thread i of a workgroup column owns row i
// and walks kKmCols columns, so the column-major stores are coalesced and
// the column points are read as uniform (scalar) loads.  Every step of r^2
// is rounded on its own (no contraction: plain operators under the pragma,
// since the *_rn helpers are inline functions the pragma does not reach), so
// with correctly rounded sqrt and division the Coulomb-like kernel equals a
// host evaluation of the same formula bit for bit; exp may differ in the
// last bit.
// ---------------------------------------------------------------------------
constexpr int kKmCols = 32;

__global__ __launch_bounds__(256) void k_kernel_matrix(const double* __restrict__ xr, int64_t nr,
                                                       const double* __restrict__ xc, int64_t nc,
                                                       int dim, int kind, double a, double diag,
                                                       double* __restrict__ out, int64_t ld) {
#pragma clang fp contract(off)
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= nr) return;
  double xi[3] = {0.0, 0.0, 0.0};
  for (int c = 0; c < dim; ++c) xi[c] = xr[i * dim + c];
  const double r0 = kind == 1 ? a * a : 0.0;
  const int64_t j0 = (int64_t)blockIdx.y * kKmCols;
  const int64_t j1 = j0 + kKmCols < nc ? j0 + kKmCols : nc;
  for (int64_t j = j0; j < j1; ++j) {
    double r2 = r0;
    for (int c = 0; c < dim; ++c) {
      const double d = xi[c] - xc[j * dim + c];
      const double sq = d * d;
      r2 = r2 + sq;
    }
    double v = kind == 1 ? 1.0 / sqrt(r2) : exp(-a * r2);
    if (i == j) v = v + diag;
    out[i + j * ld] = v;
  }
}

hipError_t launch_kernel_matrix(const double* xr, int64_t nr, const double* xc, int64_t nc,
                                int dim, int kind, double a, double diag, double* out,
                                int64_t ld, hipStream_t s) {
  if (nr <= 0 || nc <= 0) return hipSuccess;
  const dim3 grid((unsigned)((nr + 255) / 256), (unsigned)((nc + kKmCols - 1) / kKmCols));
  hipLaunchKernelGGL(k_kernel_matrix, grid, dim3(256), 0, s, xr, nr, xc, nc, dim, kind, a, diag,
                     out, ld);
  return hipGetLastError();
}

// Operand grouping without a library sort (recordable in a graph): a
// counting sort of the items into kGroupBuckets buckets by a multiplicative
// hash of their first term's left-operand address, in one workgroup.  Items
// that read the same operand block share the address, hence the bucket, so
// they run next to each other; the order inside a bucket (atomics) and of the
// buckets changes no result.
constexpr int kGroupBuckets = 4096;

__device__ inline int operand_bucket(const GemmItem* items, const Seg* segs, int i) {
  const uint64_t a = (uint64_t)(uintptr_t)segs[items[i].seg0].L >> 3;
  return (int)((a * 0x9E3779B97F4A7C15ull) >> (64 - 12));
}

__global__ __launch_bounds__(kOrderThreads) void k_operand_group(const GemmItem* __restrict__ items,
                                                                const Seg* __restrict__ segs, int n,
                                                                int* __restrict__ order,
                                                                const int64_t* __restrict__ live) {
  static_assert(kGroupBuckets == 1 << 12, "the hash keeps 12 bits");
  __shared__ int cnt[kGroupBuckets];
  __shared__ int part[kOrderThreads];
  const int tid = threadIdx.x;
  if (live) n = (int)min((int64_t)n, *live);
  for (int b = tid; b < kGroupBuckets; b += kOrderThreads) cnt[b] = 0;
  __syncthreads();
  for (int i = tid; i < n; i += kOrderThreads) atomicAdd(&cnt[operand_bucket(items, segs, i)], 1);
  __syncthreads();
  // exclusive scan of the buckets: each thread owns kGroupBuckets / kOrderThreads
  // consecutive buckets; the per-thread totals are scanned in LDS
  constexpr int per = kGroupBuckets / kOrderThreads;
  int own = 0;
  for (int t = 0; t < per; ++t) own += cnt[tid * per + t];
  part[tid] = own;
  __syncthreads();
  for (int o = 1; o < kOrderThreads; o <<= 1) {
    const int v = tid >= o ? part[tid - o] : 0;
    __syncthreads();
    part[tid] += v;
    __syncthreads();
  }
  int run = part[tid] - own;
  for (int t = 0; t < per; ++t) {
    const int c = cnt[tid * per + t];
    cnt[tid * per + t] = run;
    run += c;
  }
  __syncthreads();
  for (int i = tid; i < n; i += kOrderThreads)
    order[atomicAdd(&cnt[operand_bucket(items, segs, i)], 1)] = i;
}

hipError_t launch_operand_group(const GemmItem* items, const Seg* segs, int nitems, int* order,
                                hipStream_t s, const int64_t* live) {
  if (nitems <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_operand_group, dim3(1), dim3(kOrderThreads), 0, s, items, segs, nitems,
                     order, live);
  return hipGetLastError();
}

size_t operand_order_bytes(int nitems) {
  if (nitems <= 0) return 0;
  return 3 * align256(sizeof(uint32_t) * (size_t)nitems) + align256(sort_temp_bytes(nitems));
}

hipError_t launch_operand_order(const GemmItem* items, const Seg* segs, int nitems, void* work,
                                int* order, hipStream_t s) {
  if (nitems <= 0) return hipSuccess;
  const size_t a = align256(sizeof(uint32_t) * (size_t)nitems);
  char* w = static_cast<char*>(work);
  uint32_t* kin = reinterpret_cast<uint32_t*>(w);
  uint32_t* kout = reinterpret_cast<uint32_t*>(w + a);
  int* vin = reinterpret_cast<int*>(w + 2 * a);
  void* temp = w + 3 * a;
  size_t tb = sort_temp_bytes(nitems);
  hipLaunchKernelGGL(k_operand_keys, dim3((unsigned)((nitems + 255) / 256)), dim3(256), 0, s, items,
                     segs, nitems, kin, vin);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return hipcub::DeviceRadixSort::SortPairs(temp, tb, kin, kout, vin, order, nitems, 0, 32, s);
}

}  // namespace clr
