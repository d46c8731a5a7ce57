// Grouped block-product GEMM for gfx950.
//
// Every heavy product of the CLR method runs through this one kernel: the
// dense x dense block products, the thin factor products of the low-rank
// terms (Sec. 4.1, Eq. (4): V_A^T B, A U_B, the core Z = V_A^T U_B and its
// contraction with the smaller side), and the dense accumulation of all terms
// of a result block.  A launch processes a list of output tiles ("items") of
// uneven shapes; each item walks its list of terms ("segments") as one
// concatenated inner dimension, staged through LDS 16 inner indices at a time
// with a two-deep pipeline, and multiplies on MFMA:
//   FP64 form:  v_mfma_f64_16x16x4_f64, FP64 accumulation in registers.
//   Mixed form: v_mfma_f32_16x16x4_f32 on FP32-rounded operands, the FP32
//               partial of every 16 inner indices is added into FP64
//               accumulators; optionally the hi*lo + lo*hi correction terms
//               (lo = fp32(x - hi)) go to a second FP32 partial.
//
// Workgroup: 256 threads = 4 waves in a 2 x 2 arrangement; wave (wr, wc)
// owns the 16 x 16 output tiles (wr + 2a, wc + 2b), a, b < WT.
//
// MFMA operand layout for the 16x16x4 shapes (64 lanes, lane = l):
//   A(i, k): i = l % 16, k = l / 16;   B(k, j): j = l % 16, k = l / 16;
//   D(i, j) is held by lane l = j + 16*g, element v, with
//     f32: i = 4*g + v        f64: i = g + 4*v   (the f64 shape interleaves rows).
#include "clr_internal.h"

namespace clr {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
// Operand pointers are read back from LDS as generic pointers; loads through
// them would compile to flat instructions, which count against the LDS wait
// counter too and so serialise the MFMA operand reads behind the next slab's
// global prefetch.  Casting to the global address space keeps them on the
// vector-memory counter only.
typedef const double __attribute__((address_space(1))) gdouble;
typedef double __attribute__((address_space(1))) gdouble_mut;
__device__ inline gdouble* as_global(const double* p) { return (gdouble*)p; }
__device__ inline gdouble_mut* as_global_mut(double* p) { return (gdouble_mut*)p; }

template <int WT, bool F32>
struct GemmLds {
  static constexpr int TM = 32 * WT;
  static constexpr int LD = TM + 1;  // odd stride: k-fast stores hit distinct banks
  using T = typename std::conditional<F32, float, double>::type;
  T a[2][kSlabK][LD];
  T b[2][kSlabK][LD];
  T alo[F32 ? 2 : 1][F32 ? kSlabK : 1][F32 ? LD : 1];
  T blo[F32 ? 2 : 1][F32 ? kSlabK : 1][F32 ? LD : 1];
  // per inner-row source descriptors of the slab being loaded next
  const double* lp[2][kSlabK];
  const double* rp[2][kSlabK];
  int64_t sli[2][kSlabK];
  int64_t srj[2][kSlabK];
  double scale[2][kSlabK];
};

// Thread t < 16 resolves inner row t of slab `slab`: which segment it falls in
// and where its L column / R row start.  `cur` is that thread's segment cursor
// (monotone over slabs).
__device__ inline void resolve_row(const GemmItem& it, const Seg* __restrict__ segs, int slab,
                                   int t, int& cur, const double*& lp, const double*& rp,
                                   int64_t& sli, int64_t& srj, double& sc) {
  const int g = slab * kSlabK + t;
  lp = nullptr;
  rp = nullptr;
  sli = 0;
  srj = 0;
  sc = 0.0;
  if (g >= it.ktotal) return;
  while (cur < it.nseg) {
    const Seg& s = segs[it.seg0 + cur];
    if (g < s.kbase + s.k) break;
    ++cur;
  }
  if (cur >= it.nseg) return;
  const Seg& s = segs[it.seg0 + cur];
  const int kl = g - s.kbase;
  lp = s.L + (int64_t)it.row0 * s.sLi + (int64_t)kl * s.sLk;
  rp = s.R + (int64_t)it.col0 * s.sRj + (int64_t)kl * s.sRk;
  sli = s.sLi;
  srj = s.sRj;
  sc = s.scale;
}

template <int WT, bool F32, bool SPLIT>
__global__ __launch_bounds__(kGemmThreads, 1) void k_ggemm(const GemmItem* __restrict__ items,
                                                           const Seg* __restrict__ segs,
                                                           int nitems) {
  using L = GemmLds<WT, F32>;
  constexpr int TM = L::TM;
  constexpr int NE = (kSlabK * TM) / kGemmThreads;  // staged elements per thread and operand
  static_assert((kSlabK * TM) % kGemmThreads == 0, "tile/thread mismatch");
  __shared__ L sh;

  // XCD-aware order: consecutive items (tiles of one block row) share an XCD's L2.
  const int per = gridDim.x / 8;
  const int item = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
  if (item >= nitems) return;
  const GemmItem it = items[item];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int mt = (it.m + 15) >> 4, nt = (it.n + 15) >> 4;
  const int nslab = (it.ktotal + kSlabK - 1) / kSlabK;

  d4 acc[WT][WT];
#pragma unroll
  for (int a = 0; a < WT; ++a)
#pragma unroll
    for (int b = 0; b < WT; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};

  int cursor = 0;  // meaningful for tid < 16 only
  double ra[NE], rb[NE];

  auto resolve = [&](int slab, int buf) {
    if (tid < kSlabK) {
      const double* lp;
      const double* rp;
      int64_t sli, srj;
      double sc;
      resolve_row(it, segs, slab, tid, cursor, lp, rp, sli, srj, sc);
      sh.lp[buf][tid] = lp;
      sh.rp[buf][tid] = rp;
      sh.sli[buf][tid] = sli;
      sh.srj[buf][tid] = srj;
      sh.scale[buf][tid] = sc;
    }
  };
  // global -> registers; the thread->element map is chosen from inner row 0:
  // rows contiguous in memory are read row-fast, otherwise inner-fast.
  auto load = [&](int buf) {
    const bool arow = sh.sli[buf][0] == 1;
    const bool brow = sh.srj[buf][0] == 1;
#pragma unroll
    for (int u = 0; u < NE; ++u) {
      const int e = tid + u * kGemmThreads;
      int t, i;
      if (arow) { t = e / TM; i = e % TM; } else { t = e % kSlabK; i = e / kSlabK; }
      const double* p = sh.lp[buf][t];
      double v = 0.0;
      if (p != nullptr && i < it.m) v = as_global(p)[(int64_t)i * sh.sli[buf][t]] * sh.scale[buf][t];
      ra[u] = v;
      if (brow) { t = e / TM; i = e % TM; } else { t = e % kSlabK; i = e / kSlabK; }
      const double* q = sh.rp[buf][t];
      double w = 0.0;
      if (q != nullptr && i < it.n) w = as_global(q)[(int64_t)i * sh.srj[buf][t]];
      rb[u] = w;
    }
  };
  auto store = [&](int buf, int pbuf) {
    const bool arow = sh.sli[pbuf][0] == 1;
    const bool brow = sh.srj[pbuf][0] == 1;
#pragma unroll
    for (int u = 0; u < NE; ++u) {
      const int e = tid + u * kGemmThreads;
      int t, i;
      if (arow) { t = e / TM; i = e % TM; } else { t = e % kSlabK; i = e / kSlabK; }
      if constexpr (F32) {
        const float hi = (float)ra[u];
        sh.a[buf][t][i] = hi;
        if constexpr (SPLIT) sh.alo[buf][t][i] = (float)(ra[u] - (double)hi);
      } else {
        sh.a[buf][t][i] = ra[u];
      }
      if (brow) { t = e / TM; i = e % TM; } else { t = e % kSlabK; i = e / kSlabK; }
      if constexpr (F32) {
        const float hi = (float)rb[u];
        sh.b[buf][t][i] = hi;
        if constexpr (SPLIT) sh.blo[buf][t][i] = (float)(rb[u] - (double)hi);
      } else {
        sh.b[buf][t][i] = rb[u];
      }
    }
  };

  if (nslab > 0) {
    resolve(0, 0);
    __syncthreads();
    load(0);
    store(0, 0);
    if (nslab > 1) resolve(1, 1);
    __syncthreads();
  }

  const int kr = lane >> 4;   // inner row within a 4-step
  const int lc = lane & 15;   // row (A) / column (B) within a tile
  for (int s = 0; s < nslab; ++s) {
    const int cur = s & 1, nxt = cur ^ 1;
    if (s + 1 < nslab) load(nxt);
    if constexpr (!F32) {
#pragma unroll
      for (int q = 0; q < kSlabK / 4; ++q) {
        double av[WT], bv[WT];
#pragma unroll
        for (int a = 0; a < WT; ++a) av[a] = sh.a[cur][4 * q + kr][16 * (wr + 2 * a) + lc];
#pragma unroll
        for (int b = 0; b < WT; ++b) bv[b] = sh.b[cur][4 * q + kr][16 * (wc + 2 * b) + lc];
#pragma unroll
        for (int a = 0; a < WT; ++a) {
          if (wr + 2 * a >= mt) continue;
#pragma unroll
          for (int b = 0; b < WT; ++b) {
            if (wc + 2 * b >= nt) continue;
            acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
          }
        }
      }
    } else {
#pragma unroll
      for (int a = 0; a < WT; ++a) {
        if (wr + 2 * a >= mt) continue;
#pragma unroll
        for (int b = 0; b < WT; ++b) {
          if (wc + 2 * b >= nt) continue;
          f4 p = f4{0.f, 0.f, 0.f, 0.f};
          f4 pl = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int q = 0; q < kSlabK / 4; ++q) {
            const float av = sh.a[cur][4 * q + kr][16 * (wr + 2 * a) + lc];
            const float bv = sh.b[cur][4 * q + kr][16 * (wc + 2 * b) + lc];
            p = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, p, 0, 0, 0);
            if constexpr (SPLIT) {
              const float al = sh.alo[cur][4 * q + kr][16 * (wr + 2 * a) + lc];
              const float bl = sh.blo[cur][4 * q + kr][16 * (wc + 2 * b) + lc];
              pl = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bl, pl, 0, 0, 0);
              pl = __builtin_amdgcn_mfma_f32_16x16x4f32(al, bv, pl, 0, 0, 0);
            }
          }
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            acc[a][b][v] += (double)p[v];
            if constexpr (SPLIT) acc[a][b][v] += (double)pl[v];
          }
        }
      }
    }
    if (s + 1 < nslab) store(nxt, nxt);
    if (s + 2 < nslab) resolve(s + 2, cur);
    __syncthreads();
  }

  // epilogue (output layout per precision, see the header comment)
#pragma unroll
  for (int a = 0; a < WT; ++a) {
    if (wr + 2 * a >= mt) continue;
#pragma unroll
    for (int b = 0; b < WT; ++b) {
      if (wc + 2 * b >= nt) continue;
      const int j = 16 * (wc + 2 * b) + lc;
      if (j >= it.n) continue;
      gdouble_mut* col = as_global_mut(it.C) + (int64_t)(it.col0 + j) * it.ldc + it.row0;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        // f64 16x16x4: row (lane/16) + 4v;  f32 16x16x4: row 4*(lane/16) + v
        const int i = 16 * (wr + 2 * a) + (F32 ? 4 * kr + v : kr + 4 * v);
        if (i < it.m) {
          const double val = it.alpha * acc[a][b][v];
          col[i] = it.accumulate ? col[i] + val : val;
        }
      }
    }
  }
}

static inline int xcd_grid(int n) { return ((n + 7) / 8) * 8; }

hipError_t launch_ggemm_f64(const GemmItem* items, const Seg* segs, int nitems, hipStream_t s) {
  if (nitems <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_ggemm<kF64WaveTiles, false, false>), dim3(xcd_grid(nitems)),
                     dim3(kGemmThreads), 0, s, items, segs, nitems);
  return hipGetLastError();
}

hipError_t launch_ggemm_f32(const GemmItem* items, const Seg* segs, int nitems, int split,
                            hipStream_t s) {
  if (nitems <= 0) return hipSuccess;
  if (split)
    hipLaunchKernelGGL((k_ggemm<kF32WaveTiles, true, true>), dim3(xcd_grid(nitems)),
                       dim3(kGemmThreads), 0, s, items, segs, nitems);
  else
    hipLaunchKernelGGL((k_ggemm<kF32WaveTiles, true, false>), dim3(xcd_grid(nitems)),
                       dim3(kGemmThreads), 0, s, items, segs, nitems);
  return hipGetLastError();
}

}  // namespace clr
