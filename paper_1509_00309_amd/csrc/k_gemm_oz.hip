// Dense accumulation of the CLR product on INT8 MFMA by operand splitting
// (Ozaki, Ogita, Oishi and Rump's error-free splitting, with the integer-unit
// products of Ootomo, Ozaki and Yokota), v_mfma_i32_16x16x64_i8 on gfx950.
//
// Same work lists as the FP64 dense accumulation launch: an item is an output
// tile of at most 64 x 64 and its terms form one concatenated inner range,
// walked 64 inner indices (one MFMA k-extent) at a time.  In a chunk, every
// row i of the left operand and every column j of the right one is scaled by
// a power of two so that its entries lie in (-1, 1), and expanded into S
// signed 7-bit digits:
//   x = 2^e (sum_{p<S} d_p 2^(-7(p+1)) + r),   |d_p| <= 127,  |r| < 2^(-7S).
// The digit products with p + q < S are summed exactly by the MFMA in int32
// (a group g = p + q holds at most 7 * 64 * 127^2 < 2^23 in magnitude) and
// each group is added into FP64 accumulators with the exact weight
// 2^(e_i + e_j - 7(g + 2)).  The only roundings are the FP64 additions and
// the dropped digit products and remainders, of relative size about
// (S + 3) 2^(-7S) against the chunk's largest |x_ik| |y_kj|; S = 7 keeps the
// product near FP64 accuracy.
//
// Workgroup: 256 threads = 4 waves in a 2 x 2 arrangement, a wave owns the
// 2 x 2 tiles of 16 x 16 of one 32 x 32 quadrant; two workgroups per CU, so
// one's digit expansion and barriers overlap the other's MFMA work.  Per chunk: resolve the
// inner rows' terms, load and take per-row / per-column maxima, exponents,
// digit expansion into LDS (16 consecutive inner indices of one row per
// thread, one 16-byte store per digit), then the MFMA groups.
#include "k_gemm.h"

namespace clr {

namespace {

constexpr int kOzEdge = kMaxItemOzaki;   // item rows and columns
constexpr int kOzK = 64;                 // inner indices per chunk
constexpr int kOzThreads = 256;
constexpr int kOzRow = kOzK + 16;        // bytes per digit row in LDS (16-byte aligned, skewed banks)
static_assert(kOzEdge == 64 && kOzThreads == 4 * kOzEdge, "one thread per (row, inner quarter)");

typedef int i4v __attribute__((ext_vector_type(4)));

struct OzLds {
  int8_t la[kOzMaxSlices][kOzEdge][kOzRow];   // digits of L: [p][row i][inner k]
  int8_t rb[kOzMaxSlices][kOzEdge][kOzRow];   // digits of R: [q][column j][inner k]
  double pml[4][kOzEdge];                     // per inner quarter, max |x| of a row of L
  double pmr[4][kOzEdge];                     // per inner quarter, max |y| of a column of R
  int el[kOzEdge], er[kOzEdge];               // chunk exponents
  double wl[kOzEdge], wr[kOzEdge];            // 2^e
  const double* lp[kOzK];
  const double* rp[kOzK];
  int64_t sli[kOzK], srj[kOzK];
  double scale[kOzK], bok[kOzK];
};
// two workgroups per CU (the term descriptors are read through L2, not cached in LDS)
static_assert(sizeof(OzLds) <= 160 * 1024 / 2, "two workgroups per CU");

// Smallest e with m < 2^e for m > 0; a zero row or column gets 0 (its digits
// are all zero whatever the exponent).
__device__ inline int chunk_exponent(double m) {
  if (!(m > 0.0)) return 0;
  int e;
  (void)frexp(m, &e);   // m = f 2^e, f in [0.5, 1)
  return e;
}

// Digits of the 16 values x[u] (one row's inner quarter) under exponent e,
// packed 4 per dword in inner order, one 16-byte group per digit.
__device__ inline void expand(const double (&x)[16], int e, int S, uint32_t (&w)[kOzMaxSlices][4]) {
#pragma unroll
  for (int p = 0; p < kOzMaxSlices; ++p)
#pragma unroll
    for (int c = 0; c < 4; ++c) w[p][c] = 0u;
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    double y = ldexp(x[u], -e);   // |y| < 1
#pragma unroll
    for (int p = 0; p < kOzMaxSlices; ++p) {
      if (p < S) {
        y *= 128.0;               // exact
        const double d = trunc(y);
        y -= d;                   // exact
        w[p][u >> 2] |= (uint32_t)(uint8_t)(int8_t)(int)d << (8 * (u & 3));
      }
    }
  }
}

}  // namespace

__global__ __launch_bounds__(kOzThreads, 2) void k_ggemm_ozaki(const GemmItem* __restrict__ items,
                                                           const Seg* __restrict__ segs,
                                                           int nitems,
                                                           const int* __restrict__ order,
                                                           int S) {
  __shared__ OzLds sh;
  int item;
  if (order) {
    if ((int)blockIdx.x >= nitems) return;
    item = order[blockIdx.x];
  } else {
    const int per = gridDim.x / 8;
    item = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
    if (item >= nitems) return;
  }
  GemmItem it = items[item];
  // the planner caps items at kOzEdge; the clamp only keeps every access in bounds
  it.m = uni(min(it.m, kOzEdge));
  it.n = uni(min(it.n, kOzEdge));
  it.row0 = uni(it.row0);
  it.col0 = uni(it.col0);
  it.seg0 = uni(it.seg0);
  it.nseg = uni(it.nseg);
  it.ktotal = uni(it.ktotal);
  it.accumulate = uni(it.accumulate);
  it.ldc = uni64(it.ldc);
  S = uni(S);
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = uni(tid >> 6);
  const int wr = wave >> 1, wc = wave & 1;

  const Seg* terms = segs + it.seg0;   // resolve_row's cache, here in global memory

  // this thread's operand share: row (L) / column (R) `own`, inner quarter kq
  const int own = tid & 63, kq = tid >> 6;
  int cursor = 0;   // term cursor of inner row tid (tid < 64)

  typedef double d4 __attribute__((ext_vector_type(4)));
  d4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};

  const int lr = lane & 15;          // tile row (A) / column (B) of this lane
  const int lk = (lane >> 4) * 16;   // first inner byte of this lane's 16
  const int nchunk = (it.ktotal + kOzK - 1) / kOzK;
  for (int c = 0; c < nchunk; ++c) {
    __syncthreads();   // previous chunk's MFMA reads are done
    if (tid < kOzK) {
      const double* lp;
      const double* rp;
      int64_t sli, srj;
      double sc, bok;
      resolve_row(it, segs, terms, c * (kOzK / kSlabK) + (tid >> 4), tid & 15, cursor, lp, rp,
                  sli, srj, sc, bok);
      sh.lp[tid] = lp;
      sh.rp[tid] = rp;
      sh.sli[tid] = sli;
      sh.srj[tid] = srj;
      sh.scale[tid] = sc;
      sh.bok[tid] = bok;
    }
    __syncthreads();
    double xl[16], xr[16];
    double ml = 0.0, mr = 0.0;
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int k = kq * 16 + u;
      const double sc = sh.scale[k];   // 0 past the item's inner range
      const double bk = sh.bok[k];
      const double* lp = sh.lp[k];
      const double* rp = sh.rp[k];
      const int il = own < it.m ? own : 0;
      const int jr = own < it.n ? own : 0;
      const double a = *as_global(lp + (int64_t)il * sh.sli[k]);
      const double b = *as_global(rp + (int64_t)jr * sh.srj[k]);
      xl[u] = (own < it.m && sc != 0.0) ? a * sc : 0.0;
      xr[u] = (own < it.n && bk != 0.0) ? b : 0.0;
      ml = fmax(ml, fabs(xl[u]));
      mr = fmax(mr, fabs(xr[u]));
    }
    sh.pml[kq][own] = ml;
    sh.pmr[kq][own] = mr;
    __syncthreads();
    if (tid < kOzEdge) {
      const double m = fmax(fmax(sh.pml[0][tid], sh.pml[1][tid]), fmax(sh.pml[2][tid], sh.pml[3][tid]));
      const int e = chunk_exponent(m);
      sh.el[tid] = e;
      sh.wl[tid] = ldexp(1.0, e);
    } else if (tid < 2 * kOzEdge) {
      const int j = tid - kOzEdge;
      const double m = fmax(fmax(sh.pmr[0][j], sh.pmr[1][j]), fmax(sh.pmr[2][j], sh.pmr[3][j]));
      const int e = chunk_exponent(m);
      sh.er[j] = e;
      sh.wr[j] = ldexp(1.0, e);
    }
    __syncthreads();
    {
      uint32_t w[kOzMaxSlices][4];
      expand(xl, sh.el[own], S, w);
#pragma unroll
      for (int p = 0; p < kOzMaxSlices; ++p)
        if (p < S) *(i4v*)&sh.la[p][own][kq * 16] = i4v{(int)w[p][0], (int)w[p][1], (int)w[p][2], (int)w[p][3]};
      expand(xr, sh.er[own], S, w);
#pragma unroll
      for (int q = 0; q < kOzMaxSlices; ++q)
        if (q < S) *(i4v*)&sh.rb[q][own][kq * 16] = i4v{(int)w[q][0], (int)w[q][1], (int)w[q][2], (int)w[q][3]};
    }
    __syncthreads();

    // MFMA groups g = p + q < S of this wave's tiles; tiles outside the item
    // compute on zero digits and are never stored.  The left digits stay in
    // registers, the right ones are read per product.
    i4v da[kOzMaxSlices][2];
#pragma unroll
    for (int p = 0; p < kOzMaxSlices; ++p) {
      if (p < S) {
#pragma unroll
        for (int a = 0; a < 2; ++a) da[p][a] = *(const i4v*)&sh.la[p][32 * wr + 16 * a + lr][lk];
      }
    }
    // output (row 4 (lane / 16) + v, column lane % 16) of each tile: its weight
    double rs[2][4], cs[2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int v = 0; v < 4; ++v) rs[a][v] = sh.wl[32 * wr + 16 * a + 4 * (lane >> 4) + v];
#pragma unroll
    for (int b = 0; b < 2; ++b) cs[b] = sh.wr[32 * wc + 16 * b + lr];
#pragma unroll
    for (int g = 0; g < kOzMaxSlices; ++g) {
      if (g < S) {
        i4v s[2][2];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int b = 0; b < 2; ++b) s[a][b] = i4v{0, 0, 0, 0};
#pragma unroll
        for (int p = 0; p <= g; ++p) {
          i4v db[2];
#pragma unroll
          for (int b = 0; b < 2; ++b) db[b] = *(const i4v*)&sh.rb[g - p][32 * wc + 16 * b + lr][lk];
#pragma unroll
          for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
              s[a][b] = __builtin_amdgcn_mfma_i32_16x16x64_i8(da[p][a], db[b], s[a][b], 0, 0, 0);
        }
        const double wg = ldexp(1.0, -7 * (g + 2));
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int b = 0; b < 2; ++b) {
            const double cw = cs[b] * wg;
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[a][b][v] += (double)s[a][b][v] * (rs[a][v] * cw);
          }
      }
    }
  }

  const double alpha = it.alpha;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int j = 32 * wc + 16 * b + lr;
      if (j >= it.n) continue;
      gdouble_mut* col = as_global_mut(it.C) + (int64_t)(it.col0 + j) * it.ldc + it.row0;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = 32 * wr + 16 * a + 4 * (lane >> 4) + v;
        if (i < it.m) {
          const double val = alpha * acc[a][b][v];
          col[i] = it.accumulate ? col[i] + val : val;
        }
      }
    }
}

hipError_t launch_ggemm_ozaki(const GemmItem* items, const Seg* segs, int nitems, int slices,
                              hipStream_t s, const int* order) {
  if (nitems <= 0) return hipSuccess;
  if (slices < 2 || slices > kOzMaxSlices) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_ggemm_ozaki, dim3(xcd_grid(nitems)), dim3(kOzThreads), 0, s, items, segs,
                     nitems, order, slices);
  return hipGetLastError();
}

}  // namespace clr
