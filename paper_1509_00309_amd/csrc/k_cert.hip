// Certificate that a dense-accumulated result block stays dense under the
// rank rule of Sec. 4.1, so that its truncated SVD can be skipped.
//
// A block D (m x n) is stored dense when its kept rank r satisfies
// 2 r > min(m, n), where r is the smallest rank whose discarded tail
// sqrt(sum_{i >= r} s_i^2) is at most tol ||D||_F.  With q = min(m, n),
// p = max(m, n) and h = floor(q / 2), the block is dense as soon as
// s_h > tol ||D||_F (singular values in decreasing order, s_0 the largest).
//
// Orient D so that its q columns are the short side (D or D^T, p x q).  By
// the Courant-Fischer minimax characterisation, s_h(D) >= s_min(D_S) for any
// h + 1 of those columns S.  The columns are chosen greedily: Cholesky with
// diagonal pivoting of the Gram matrix D^T D - c I takes at every step the
// column of largest residual norm (the Gram-matrix form of QR with column
// pivoting).  If h + 1 steps complete with positive pivots, D_S^T D_S - c I is
// positive definite up to rounding, and the rounding is bounded by
//  * the Gram matrix's error, at most gamma_p ||D||_F^2 in the 2-norm
//    (gamma_k = k u / (1 - k u), u = 2^-53);
//  * the Cholesky backward error: a factorisation R^T R of A that completes in
//    floating point satisfies R^T R = A + E with ||E||_2 <= gamma_{q+1}
//    trace(A) (Higham, Accuracy and Stability of Numerical Algorithms,
//    Thm. 10.3), and trace(A) <= ||D||_F^2;
//  * the subtraction of c from the diagonal, at most u ||D||_F^2.
// The shift c = ||D||_F^2 (9/8 tol^2 + 4 (p + q + 2) u) covers the three
// terms twice, so success proves s_h(D)^2 > (9/8 tol^2 + 2 (p + q + 2) u)
// ||D||_F^2.  The margin this leaves between s_h and tol ||D||_F is at least
// about 7e-9 ||D||_F for every tol, two orders of magnitude above the
// worst-case error bound of a Householder-based SVD of a block of edge <= 512,
// so the SVD path reaches the same decision: the certificate changes no
// result (a certified block is copied out exactly as a block the SVD finds
// dense), it only skips work.
//
// Short edges q in (319, 512], and those in (160, 319] whose column subset
// fails (h + 1 pivots out of 160 columns leave little choice near 319): every
// column takes part and the Gram matrix is not held at all.  A left-looking pivoted Cholesky
// forms, at step k, the pivot's Gram column g_j = <d_j, d_piv> (a dot product
// of length p, each entry computed once: the symmetric matrix with those
// entries differs from D^T D by at most gamma_p |D|^T |D|, so by at most
// gamma_p ||D||_F^2 in the 2-norm, as above), subtracts L(j, 0:k) L(piv, 0:k)^T
// and keeps column k of L in the block's recompression scratch (q x (h + 1)
// doubles, which the block's SVD working set m n exceeds).  The Cholesky error
// bound holds for any order of the inner products, so the proof is unchanged.
//
// Short edges q in (160, 319]: the columns examined are a subset T of
// qs = 160 of the q, evenly spread (column floor(a q / qs) for a < qs).
// Deleting columns can only lower singular values (interlacing), so
// s_h(D) >= s_h(D_T), and h + 1 <= qs pivots fit in the subset.  Every error
// term above is bounded through ||D_T||_F <= ||D||_F and qs <= q, and the
// shift takes the full ||D||_F^2 (summed separately, its own rounding far
// inside the factor-two cover), so the same proof holds for the whole block.
//
// One workgroup per block.  The Gram matrix (q x q) is computed on FP64 MFMA
// (v_mfma_f64_16x16x4) from 16-deep slabs of D staged in LDS, with the next
// slab's loads in flight, and stays in the MFMA output registers: the waves
// form a WR x WC grid, wave (wr, wc) owns the 16 x 16 tiles (wr + WR u,
// wc + WC w) for u < TU, w < TW, T = ceil(q / 16) <= WR TU, WC TW.  One
// kernel per size class of q: q <= 128 on 512 threads (2 x 4 waves of 4 x 2
// tiles, two workgroups per CU), q <= 160 on 1024 threads (4 x 4 waves of
// 3 x 3 tiles).  The right-looking pivoted Cholesky then updates those
// registers in place.  Every wave keeps its own copy of the residual
// diagonal in registers and updates it from the published pivot column with
// the same arithmetic, so every wave picks the same pivot without a barrier;
// with the pivot column double-buffered in LDS a step costs one barrier.
#include "clr_internal.h"

namespace clr {
namespace {

typedef const double __attribute__((address_space(1))) cgdbl;
typedef double __attribute__((address_space(1))) gdbl;

constexpr int kCertSlab = 16;               // inner indices staged per slab
constexpr int kCertLd = kCertEdge + 1;
constexpr int kCertDiag = (kCertEdge + 63) / 64;   // residual diagonal entries per lane
constexpr int kCertColLd = 64 * kCertDiag;          // pivot column, zero beyond q

struct CertLds {
  double slab[kCertSlab][kCertLd];
  double col[2][kCertColLd];
  double dg[kCertEdge];
};

// Lane permutations inside a DPP row of 16 (vector ALU, no LDS round trip).
template <int CTRL>
__device__ __attribute__((always_inline)) inline int dpp_i(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __attribute__((always_inline)) inline double dpp_d(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = dpp_i<CTRL>((int)(b & 0xffffffffLL));
  const int hi = dpp_i<CTRL>((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
// The value of the partner row: lanes 16 apart (permlane16 swap) or 32 apart
// (permlane32 swap).  With both operands the same register the two results
// are the even-row and odd-row values; the lane's partner value is the one
// that is not its own.
__device__ __attribute__((always_inline)) inline double other_d16(double v, bool odd) {
  const long long b = __double_as_longlong(v);
  const unsigned lo = (unsigned)(b & 0xffffffffLL), hi = (unsigned)(b >> 32);
  const auto l = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
  const auto h = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
  const unsigned rl = odd ? l[0] : l[1], rh = odd ? h[0] : h[1];
  return __longlong_as_double((long long)(((unsigned long long)rh << 32) | rl));
}
__device__ __attribute__((always_inline)) inline double other_d32(double v, bool upper) {
  const long long b = __double_as_longlong(v);
  const unsigned lo = (unsigned)(b & 0xffffffffLL), hi = (unsigned)(b >> 32);
  const auto l = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
  const auto h = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
  const unsigned rl = upper ? l[0] : l[1], rh = upper ? h[0] : h[1];
  return __longlong_as_double((long long)(((unsigned long long)rh << 32) | rl));
}
__device__ __attribute__((always_inline)) inline int other_i16(int v, bool odd) {
  const auto r = __builtin_amdgcn_permlane16_swap((unsigned)v, (unsigned)v, false, false);
  return (int)(odd ? r[0] : r[1]);
}
__device__ __attribute__((always_inline)) inline int other_i32(int v, bool upper) {
  const auto r = __builtin_amdgcn_permlane32_swap((unsigned)v, (unsigned)v, false, false);
  return (int)(upper ? r[0] : r[1]);
}

// Largest value over the wave and, among the lanes holding it, the smallest
// index: max is exact, so every lane (and every wave given the same values)
// ends with the same pair.
__device__ __attribute__((always_inline)) inline void wave_argmax(double& v, int& i, int lane) {
  const bool odd = (lane >> 4) & 1, upper = lane >= 32;
  double m = v;
  m = fmax(m, dpp_d<0xB1>(m));    // quad_perm [1,0,3,2]
  m = fmax(m, dpp_d<0x4E>(m));    // quad_perm [2,3,0,1]
  m = fmax(m, dpp_d<0x141>(m));   // row_half_mirror
  m = fmax(m, dpp_d<0x140>(m));   // row_mirror
  m = fmax(m, other_d16(m, odd));
  m = fmax(m, other_d32(m, upper));
  int k = v == m ? i : 0x7fffffff;
  k = min(k, dpp_i<0xB1>(k));
  k = min(k, dpp_i<0x4E>(k));
  k = min(k, dpp_i<0x141>(k));
  k = min(k, dpp_i<0x140>(k));
  k = min(k, other_i16(k, odd));
  k = min(k, other_i32(k, upper));
  v = m;
  i = k;
}

typedef double d4 __attribute__((ext_vector_type(4)));

template <int WR, int WC, int TU, int TW>
__device__ __attribute__((always_inline)) inline bool cert_block(const RecItem& it, double tol,
                                                                 CertLds& L) {
  constexpr int NT = 64 * WR * WC;
  const int tid = opaque_tid();
  const int m = it.m, n = it.n;
  const int q = m < n ? m : n, p = m < n ? n : m;
  const int qs = q < kCertEdge ? q : kCertEdge;   // columns examined (all of them up to 160)
  const int T = (qs + 15) >> 4;  // 16 x 16 tiles per dimension
  const bool trans = m < n;      // columns of D^T are the short side
  cgdbl* D = (cgdbl*)it.D;
  const int64_t ldd = it.ldd;
  const int lane = tid & 63, wave = tid >> 6;
  const int wr = wave % WR, wc = wave / WR;
  // ||D||_F^2 of the whole block when only a column subset is examined: per-thread
  // partials in a fixed assignment, lane 0's butterfly sum per wave, the wave sums
  // added in wave order by every thread (one value in every wave)
  double full = 0.0;
  if (q > qs) {
    double part = 0.0;
    for (int j = wave; j < n; j += NT / 64)
      for (int i = lane; i < m; i += 64) {
        const double v = D[i + (int64_t)j * ldd];
        part = fma(v, v, part);
      }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) part += __shfl_xor(part, o, 64);
    if (lane == 0) L.dg[wave] = part;
    __syncthreads();
    for (int w = 0; w < NT / 64; ++w) full += L.dg[w];
    __syncthreads();
  }
  static_assert(16 * (WR - 1) + 3 + 16 * WR * (TU - 1) + 12 < kCertColLd &&
                    16 * (WC - 1) + 15 + 16 * WC * (TW - 1) < kCertColLd,
                "pivot-column reads stay inside the zero-padded column");
  // MFMA f64 16x16x4 lanes: operand row/column lc, inner index kr; output
  // rows kr + 4 v (v < 4) of column lc
  const int lc = lane & 15, kr = lane >> 4;

  // ---- Gram matrix G^T G of the p x q orientation G
  d4 acc[TU][TW];
#pragma unroll
  for (int u = 0; u < TU; ++u)
#pragma unroll
    for (int w = 0; w < TW; ++w) acc[u][w] = d4{0.0, 0.0, 0.0, 0.0};
  for (int e = tid; e < kCertSlab * kCertLd; e += NT) {
    const int a = e % kCertLd;
    if (a >= qs) L.slab[e / kCertLd][a] = 0.0;
  }
  // pivot-column entries beyond qs stay zero: reads need no clamping, so their
  // addresses are one base register plus constant offsets
  for (int e = tid; e < 2 * kCertColLd; e += NT)
    if (e % kCertColLd >= qs) L.col[e / kCertColLd][e % kCertColLd] = 0.0;
  // staging slots of this thread (16 qs <= 16 * 16 WR TU elements per slab):
  // consecutive threads read consecutive addresses of D; slot = (kk << 8) | a,
  // src = the column of the p x q orientation that subset column a stands for
  constexpr int PRE = (kCertSlab * 16 * WR * TU + NT - 1) / NT;
  int slot[PRE], src[PRE];
#pragma unroll
  for (int u = 0; u < PRE; ++u) {
    const int e = tid + NT * u;
    const int kk = trans ? e / qs : e % kCertSlab;
    const int a = trans ? e % qs : e / kCertSlab;
    slot[u] = e < kCertSlab * qs ? (kk << 8) | a : -1;
    src[u] = (int)(((int64_t)a * q) / qs);
  }
  double pre[PRE];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int u = 0; u < PRE; ++u) {
      const int k = k0 + (slot[u] >> 8), a = src[u];
      pre[u] = 0.0;
      if (slot[u] >= 0 && k < p) pre[u] = trans ? D[a + (int64_t)k * ldd] : D[k + (int64_t)a * ldd];
    }
  };
  fetch(0);
  for (int k0 = 0; k0 < p; k0 += kCertSlab) {
    __syncthreads();   // previous slab consumed
#pragma unroll
    for (int u = 0; u < PRE; ++u)
      if (slot[u] >= 0) L.slab[slot[u] >> 8][slot[u] & 255] = pre[u];
    __syncthreads();
    if (k0 + kCertSlab < p) fetch(k0 + kCertSlab);
#pragma unroll 2
    for (int s4 = 0; s4 < kCertSlab / 4; ++s4) {
      double av[TU], bv[TW];
#pragma unroll
      for (int u = 0; u < TU; ++u)
        av[u] = L.slab[4 * s4 + kr][min(16 * (wr + WR * u) + lc, kCertEdge - 1)];
#pragma unroll
      for (int w = 0; w < TW; ++w)
        bv[w] = L.slab[4 * s4 + kr][min(16 * (wc + WC * w) + lc, kCertEdge - 1)];
#pragma unroll
      for (int u = 0; u < TU; ++u)
#pragma unroll
        for (int w = 0; w < TW; ++w)
          if (wr + WR * u < T && wc + WC * w < T)   // wave-uniform
            acc[u][w] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u], bv[w], acc[u][w], 0, 0, 0);
    }
  }

  // ---- residual diagonal (every wave's own copy), ||D||_F^2, the shift
#pragma unroll
  for (int u = 0; u < TU; ++u)
#pragma unroll
    for (int w = 0; w < TW; ++w)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int a = 16 * (wr + WR * u) + kr + 4 * v, b = 16 * (wc + WC * w) + lc;
        if (a == b && a < qs) L.dg[a] = acc[u][w][v];
      }
  __syncthreads();
  double dgr[kCertDiag];
  bool cb[kCertDiag];
  double s = 0.0;
#pragma unroll
  for (int t = 0; t < kCertDiag; ++t) {
    const int a = lane + 64 * t;
    dgr[t] = a < qs ? L.dg[a] : 0.0;
    cb[t] = a >= qs;
    s += dgr[t];
  }
  // every wave sums the same values in the same order, then takes lane 0's sum
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o, 64);
  s = __shfl(s, 0, 64);
  // no underflow in the Gram matrix and no overflow
  if (!(s > 0x1p-600 && s < 0x1p+1000)) return false;
  // the shift scales with ||D||_F^2 of the whole block (never below the subset's)
  if (q > qs) {
    if (!(full < 0x1p+1000)) return false;
    s = fmax(s, full);
  }
  const double c = s * (1.125 * tol * tol + 4.0 * (double)(p + q + 2) * 0x1p-53);
#pragma unroll
  for (int t = 0; t < kCertDiag; ++t) dgr[t] -= c;

  // ---- h + 1 steps of Cholesky with diagonal pivoting (h + 1 <= qs)
  const int h = q / 2;
  int buf = 0;
  for (int step = 0; step <= h; ++step) {
    double bv = -__builtin_huge_val();
    int bi = 0x7fffffff;
#pragma unroll
    for (int t = 0; t < kCertDiag; ++t)
      if (!cb[t] && dgr[t] > bv) {
        bv = dgr[t];
        bi = lane + 64 * t;
      }
    wave_argmax(bv, bi, lane);
    // identical in every wave: the whole workgroup leaves together
    if (!(bv > 0.0)) return false;
    const int piv = __builtin_amdgcn_readfirstlane(bi);
    const double inv = 1.0 / sqrt(bv);
    double* colb = L.col[buf];
    const int tp = piv >> 4;   // tile column of the pivot
    if (wc == tp % WC && lc == (piv & 15)) {
      // one branch per register tile column (uniform in the wave), so acc is
      // only ever indexed by constants and stays in registers
#pragma unroll
      for (int w = 0; w < TW; ++w) {
        if (w == tp / WC) {
#pragma unroll
          for (int u = 0; u < TU; ++u)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const int a = 16 * (wr + WR * u) + kr + 4 * v;
              if (a < qs) colb[a] = acc[u][w][v];
            }
        }
      }
    }
    __syncthreads();
    const double* xcol = colb + 16 * wr + kr;
    const double* ycol = colb + 16 * wc + lc;
    double y[TW];
#pragma unroll
    for (int w = 0; w < TW; ++w) y[w] = ycol[16 * WC * w] * inv;
#pragma unroll
    for (int u = 0; u < TU; ++u) {
      double x[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) x[v] = xcol[16 * WR * u + 4 * v] * inv;
#pragma unroll
      for (int w = 0; w < TW; ++w)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][w][v] = fma(-x[v], y[w], acc[u][w][v]);
      // one tile row at a time: keeps the live operands within the register
      // budget of two workgroups per CU
      __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int t = 0; t < kCertDiag; ++t) {
      const double l = colb[lane + 64 * t] * inv;
      const bool done = cb[t] || lane + 64 * t == piv;
      dgr[t] = done ? dgr[t] : fma(-l, l, dgr[t]);
      cb[t] = done;
    }
    buf ^= 1;
  }
  return true;
}

// Size class (qlo, qhi] of the short edge: WR x WC waves of TU x TW tiles of
// 16 x 16 holding the Gram matrix of min(q, 160) columns; four waves per SIMD
// (two 512-thread or one 1024-thread workgroup per CU).
// Item of the next iteration of a certificate kernel: with `next` (a counter,
// zero at launch) the launch is persistent and its workgroups take the items
// in index order from it; otherwise every workgroup takes its own item once.
// -1: nothing left.  Uniform in the workgroup.
__device__ inline int cert_next(int* next, int* slot_sh, bool first, int nitems, bool live) {
  if (next) {
    if (!first) __syncthreads();   // slot_sh and the LDS of the last item free
    if (threadIdx.x == 0) *slot_sh = atomicAdd(next, 1);
    __syncthreads();
    const int slot = __builtin_amdgcn_readfirstlane(*slot_sh);
    return slot < nitems ? slot : -1;
  }
  if (!first) return -1;
  const int item = xcd_unit(nitems, live);
  return item >= 0 && item < nitems ? item : -1;
}

template <int WR, int WC, int TU, int TW>
__global__ __launch_bounds__(64 * WR * WC, 4) void k_dense_cert(
    const RecItem* __restrict__ items, int nitems, double tol, int qlo, int qhi,
    int* __restrict__ cert, unsigned long long* __restrict__ count,
    const int64_t* __restrict__ live, int* __restrict__ next) {
  __shared__ CertLds L;
  __shared__ int slot_sh;
  if (live) nitems = (int)min((int64_t)nitems, *live);
  for (bool first = true;; first = false) {
    const int item = cert_next(next, &slot_sh, first, nitems, live != nullptr);
    if (item < 0) return;
    const RecItem it = items[item];
    const int q = it.m < it.n ? it.m : it.n;
    if (!(it.path == kPathDense && it.cert_hint && tol > 0.0 && q > qlo && q <= qhi &&
          min(q, kCertEdge) <= 16 * WR * TU && q / 2 < kCertEdge && it.D != nullptr))
      continue;
    const bool ok = cert_block<WR, WC, TU, TW>(it, tol, L);
    if (ok && threadIdx.x == 0) {
      cert[item] = 1;
      if (count) atomicAdd(count, 1ull);
    }
  }
}

// All 16 lanes of a DPP row end with the row's sum: each step adds the
// lane's value and its partner's (the same two numbers in both lanes).
__device__ __attribute__((always_inline)) inline double row_sum16(double v) {
  v += dpp_d<0xB1>(v);    // quad_perm [1,0,3,2]
  v += dpp_d<0x4E>(v);    // quad_perm [2,3,0,1]
  v += dpp_d<0x141>(v);   // row_half_mirror
  v += dpp_d<0x140>(v);   // row_mirror
  return v;
}

constexpr int kBigThreads = 512;
struct BigCertLds {
  double dg[kCertMaxEdge];     // residual diagonal of D^T D - c I
  double colp[kCertMaxEdge];   // the pivot column of G (p entries)
  double gcol[kCertMaxEdge];   // its Gram column
  double lrow[kCertMaxEdge / 2 + 1];   // the pivot's row of L
  int taken[kCertMaxEdge];
  double wv[kBigThreads / 64];
  int wi[kBigThreads / 64];
};

// Short edges in (kCertEdge, kCertMaxEdge] not proved by the column subset:
// G (p x q) is D or D^T, thread t owns column t of G (q <= 512 = the
// workgroup).
__device__ bool cert_big(const RecItem& it, double tol, BigCertLds& L) {
  const int tid = opaque_tid();
  const int lane = tid & 63, wave = tid >> 6;
  const int m = it.m, n = it.n;
  const bool trans = m < n;
  const int q = trans ? m : n, p = trans ? n : m;
  cgdbl* D = (cgdbl*)it.D;
  const int64_t ldd = it.ldd;
  gdbl* __restrict__ Lf = (gdbl*)it.scratch;   // column k of L at Lf + k q
  // G(i, j) = D(i, j), or D(j, i) when the columns of D^T are the short side
  auto g_at = [&](int i, int j) -> double { return trans ? D[j + (int64_t)i * ldd] : D[i + (int64_t)j * ldd]; };
  // squared column norms (thread t sums column t in index order)
  double own = 0.0;
  if (tid < q)
    for (int i = 0; i < p; ++i) {
      const double v = g_at(i, tid);
      own = fma(v, v, own);
    }
  // ||D||_F^2: lane 0's butterfly sum per wave, the wave sums in wave order
  double part = own;
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) part += __shfl_xor(part, o, 64);
  if (lane == 0) L.wv[wave] = part;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < kBigThreads / 64; ++w) s += L.wv[w];
  if (!(s > 0x1p-600 && s < 0x1p+1000)) return false;   // uniform
  const double c = s * (1.125 * tol * tol + 4.0 * (double)(p + q + 2) * 0x1p-53);
  if (tid < q) {
    L.dg[tid] = own - c;
    L.taken[tid] = 0;
  }
  __syncthreads();
  const int h = q / 2;
  for (int k = 0; k <= h; ++k) {
    // pivot: the largest residual diagonal entry, the smallest index among ties
    double bv = -__builtin_huge_val();
    int bi = 0x7fffffff;
    if (tid < q && !L.taken[tid]) {
      bv = L.dg[tid];
      bi = tid;
    }
    wave_argmax(bv, bi, lane);
    if (lane == 0) {
      L.wv[wave] = bv;
      L.wi[wave] = bi;
    }
    __syncthreads();
    bv = L.wv[0];
    bi = L.wi[0];
    for (int w = 1; w < kBigThreads / 64; ++w)
      if (L.wv[w] > bv || (L.wv[w] == bv && L.wi[w] < bi)) {
        bv = L.wv[w];
        bi = L.wi[w];
      }
    if (!(bv > 0.0)) return false;   // the same decision in every thread
    const int piv = bi;
    const double inv = 1.0 / sqrt(bv);
    for (int i = tid; i < p; i += kBigThreads) L.colp[i] = g_at(i, piv);
    for (int j = tid; j < k; j += kBigThreads) L.lrow[j] = Lf[piv + (int64_t)j * q];
    __syncthreads();
    // Gram column of the pivot over the columns not yet taken
    if (trans) {
      // G(i, j) = D(j, i): consecutive threads read consecutive addresses
      if (tid < q && !L.taken[tid] && tid != piv) {
        double g = 0.0;
#pragma unroll 8
        for (int i = 0; i < p; ++i) g = fma(D[tid + (int64_t)i * ldd], L.colp[i], g);
        L.gcol[tid] = g;
      }
    } else {
      // 32 groups of 16 lanes, one column per group at a time
      const int grp = tid >> 4, gl = tid & 15;
      for (int j = grp; j < q; j += kBigThreads / 16) {
        if (L.taken[j] || j == piv) continue;   // uniform in the group
        cgdbl* __restrict__ col = D + (int64_t)j * ldd;
        double g = 0.0;
        for (int i = gl; i < p; i += 16) g = fma(col[i], L.colp[i], g);
        g = row_sum16(g);
        if (gl == 0) L.gcol[j] = g;
      }
    }
    __syncthreads();
    if (tid < q && !L.taken[tid] && tid != piv) {
      double v = L.gcol[tid];
      for (int j = 0; j < k; ++j) v = fma(-Lf[tid + (int64_t)j * q], L.lrow[j], v);
      const double l = v * inv;
      Lf[tid + (int64_t)k * q] = l;
      L.dg[tid] = fma(-l, l, L.dg[tid]);
    }
    if (tid == piv) L.taken[tid] = 1;
    __syncthreads();
  }
  return true;
}

__global__ __launch_bounds__(kBigThreads) void k_dense_cert_big(
    const RecItem* __restrict__ items, int nitems, double tol, int* __restrict__ cert,
    unsigned long long* __restrict__ count, const int64_t* __restrict__ live,
    int* __restrict__ next) {
  __shared__ BigCertLds L;
  __shared__ int slot_sh;
  if (live) nitems = (int)min((int64_t)nitems, *live);
  for (bool first = true;; first = false) {
    const int item = cert_next(next, &slot_sh, first, nitems, live != nullptr);
    if (item < 0) return;
    const RecItem it = items[item];
    const int q = it.m < it.n ? it.m : it.n, p = it.m < it.n ? it.n : it.m;
    // short edges beyond 319, and those in (160, 319] that the column subset
    // did not prove (its h + 1 pivots use up to all 160 columns); the factor L
    // (q x (h + 1)) lives in the block's scratch, which holds m n
    if (!(it.path == kPathDense && it.cert_hint && tol > 0.0 && q > kCertEdge &&
          p <= kCertMaxEdge && cert[item] == 0 && it.D != nullptr && it.scratch != nullptr))
      continue;
    const bool ok = cert_big(it, tol, L);
    if (ok && threadIdx.x == 0) {
      cert[item] = 1;
      if (count) atomicAdd(count, 1ull);
    }
  }
}

}  // namespace

hipError_t launch_dense_cert(const RecItem* items, int nitems, double tol, int* cert,
                             unsigned long long* count, hipStream_t s, const int64_t* live) {
  static_assert(16 * 4 * 3 >= kCertEdge, "the largest size class covers kCertEdge");
  if (nitems <= 0) return hipSuccess;
  // the proofs and the three launches' counters start at zero
  hipError_t e = launch_fill_i32(cert, 0, nitems + 3, s);
  if (e != hipSuccess) return e;
  int* next = cert + nitems;
  // persistent: two 512-thread, one 1024-thread or two big-form workgroups per CU
  hipLaunchKernelGGL((k_dense_cert<2, 4, 4, 2>), dim3(persistent_grid(nitems, 2)), dim3(512), 0, s,
                     items, nitems, tol, 0, 128, cert, count, live, next);
  hipLaunchKernelGGL((k_dense_cert<4, 4, 3, 3>), dim3(persistent_grid(nitems, 1)), dim3(1024), 0,
                     s, items, nitems, tol, 128, kCertMaxShort, cert, count, live, next + 1);
  hipLaunchKernelGGL(k_dense_cert_big, dim3(persistent_grid(nitems, 2)), dim3(kBigThreads), 0, s,
                     items, nitems, tol, cert, count, live, next + 2);
  return hipGetLastError();
}

}  // namespace clr
