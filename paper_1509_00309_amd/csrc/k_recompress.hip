// Recompression of accumulated result blocks, FP64 (Sec. 4.1, Eqs. (5)-(7)).
//
// One workgroup (512 threads) per result block.  Two paths:
//  * dense path: the block D (m x n) was accumulated densely.  ||D||_F
//    decides the drop; the singular values decide the kept rank r (smallest r
//    whose discarded tail sqrt(sum_{i>=r} s_i^2) is <= tol * ||D||_F).  If
//    2r > min(m, n) the block stays dense and untruncated; otherwise it is
//    stored as a pair whose one factor is the orthonormal top-r singular basis
//    of the shorter side and whose other factor is D (or D^T) times that basis.
//  * low-rank path: the block is the concatenation U_cat V_cat^T of R columns
//    (Eq. (5)).  Householder QR of both factors, core M = R_U R_V^T (Eq. (6)),
//    SVD of M, then U' = Q_U [u_M] and V' = Q_V [M^T u_M] (= Q_V V_M Sigma,
//    Eq. (7)).
//
// Singular values and vectors of a working matrix G (p x q, p >= q) come from
// one-sided Jacobi preconditioned by QR with column pivoting: G P = Q R, the
// factorisation stops once the trailing part is below 1e-19 of ||G||_F (the
// numerical rank k), and Jacobi rotations orthogonalise the columns of
// R(0:k, :)^T, whose column norms are the singular values and whose normalised
// columns, permuted by P, are the right singular vectors of G.  The
// pivoted-QR preconditioning cuts the number of Jacobi sweeps by about 3x on
// kernel-matrix blocks with decaying spectra.  Working sets live in LDS when
// they fit, otherwise in a global scratch area.
//
// Lanes are organised in groups of 16; a group owns one column (pair) at a
// time and reduces with xor-shuffles inside the group.
#include <float.h>

#include "clr_internal.h"

namespace clr {

// Working matrices live either in LDS or in global scratch.  The routines that
// touch them are templates over the pointer's address space so that each use
// compiles to ds_* or global_* instructions; generic (flat) accesses would
// couple the LDS and vector-memory wait counters and defeat latency hiding.
typedef double __attribute__((address_space(3))) ldbl;
typedef double __attribute__((address_space(1))) gdbl;
typedef const double __attribute__((address_space(1))) cgdbl;
#define CLR_INLINE __device__ __attribute__((always_inline)) inline

constexpr int kMaxDim = 512;            // largest block edge of the recompression kernel
constexpr double kNegligible2 = 1e-40;  // Jacobi ignores columns below this squared (relative) norm
constexpr double kRankFloor2 = 1e-38;   // pivoted QR stops at this squared (relative) trailing norm
constexpr int kGroups = kRecThreads / 16;



struct RecShared {
  double sigma[kMaxDim];      // pivoted QR: partial column norms^2; then singular values
  double tails[kMaxDim + 1];  // pivoted QR: reference norms^2; then tail sums
  int order[kMaxDim];
  int perm[kMaxDim];
  double red[kRecThreads];
  int flag, rank, piv;
  double drop2, tau;
};

// Cross-lane sums.  Within a row of 16 lanes the butterfly uses DPP lane
// permutations, which stay in the vector ALU (quad_perm [1,0,3,2], quad_perm
// [2,3,0,1], row_half_mirror, row_mirror): after the four steps every lane of
// the row holds the row's sum.  Crossing rows (32 and 64 lanes) uses the lane
// swaps below.
template <int CTRL>
__device__ inline double dpp_move(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffLL), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ inline double group_sum16(double v) {
  v += dpp_move<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_move<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_move<0x141>(v);  // row_half_mirror
  v += dpp_move<0x140>(v);  // row_mirror
  return v;
}

// x[l] + x[l ^ 16] and x[l] + x[l ^ 32] in every lane with the gfx950 lane
// swaps (v_permlane16_swap / v_permlane32_swap: vector ALU, no LDS round
// trip).  With both operands the same register, the two results of a swap
// are the even-row (lower-half) value and the odd-row (upper-half) value of
// the lane's pair, so every lane adds the same two numbers in the same order.
__device__ inline double xor16_sum(double v) {
  const long long b = __double_as_longlong(v);
  const unsigned lo = (unsigned)(b & 0xffffffffLL), hi = (unsigned)(b >> 32);
  const auto l = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
  const auto h = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
  const double e = __longlong_as_double((long long)(((unsigned long long)h[0] << 32) | l[0]));
  const double o = __longlong_as_double((long long)(((unsigned long long)h[1] << 32) | l[1]));
  return e + o;
}

__device__ inline double xor32_sum(double v) {
  const long long b = __double_as_longlong(v);
  const unsigned lo = (unsigned)(b & 0xffffffffLL), hi = (unsigned)(b >> 32);
  const auto l = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
  const auto h = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
  const double e = __longlong_as_double((long long)(((unsigned long long)h[0] << 32) | l[0]));
  const double o = __longlong_as_double((long long)(((unsigned long long)h[1] << 32) | l[1]));
  return e + o;
}

// Reduce-scatter steps over lane pairs 16 and 32 apart.  A swap exchanges the
// odd rows of its first operand with the even rows of its second, so with
// (a, b) a lane of an even row ends up with a + a' (a' its partner's a) and a
// lane of an odd row with b' + b: two values are summed over the pair in one
// swap each instead of two all-reduces.  The 32-lane form pairs the lower
// and upper halves of the wave the same way.
__device__ inline double swap16_sum(double a, double b) {
  const long long ab = __double_as_longlong(a), bb = __double_as_longlong(b);
  const auto l = __builtin_amdgcn_permlane16_swap((unsigned)(ab & 0xffffffffLL),
                                                  (unsigned)(bb & 0xffffffffLL), false, false);
  const auto h = __builtin_amdgcn_permlane16_swap((unsigned)(ab >> 32), (unsigned)(bb >> 32), false,
                                                  false);
  const double x = __longlong_as_double((long long)(((unsigned long long)h[0] << 32) | l[0]));
  const double y = __longlong_as_double((long long)(((unsigned long long)h[1] << 32) | l[1]));
  return x + y;
}

__device__ inline double swap32_sum(double a, double b) {
  const long long ab = __double_as_longlong(a), bb = __double_as_longlong(b);
  const auto l = __builtin_amdgcn_permlane32_swap((unsigned)(ab & 0xffffffffLL),
                                                  (unsigned)(bb & 0xffffffffLL), false, false);
  const auto h = __builtin_amdgcn_permlane32_swap((unsigned)(ab >> 32), (unsigned)(bb >> 32), false,
                                                  false);
  const double x = __longlong_as_double((long long)(((unsigned long long)h[0] << 32) | l[0]));
  const double y = __longlong_as_double((long long)(((unsigned long long)h[1] << 32) | l[1]));
  return x + y;
}

__device__ inline double hw_sum(double v) { return xor16_sum(group_sum16(v)); }

__device__ inline double wave_sum(double v) { return xor32_sum(hw_sum(v)); }

// Deterministic workgroup sum: per-thread partials, tree over LDS.
CLR_INLINE double block_sum(double v, RecShared& sh) {
  const int tid = opaque_tid();
  sh.red[tid] = v;
  __syncthreads();
  for (int s = kRecThreads / 2; s > 0; s >>= 1) {
    if (tid < s) sh.red[tid] += sh.red[tid + s];
    __syncthreads();
  }
  const double r = sh.red[0];
  __syncthreads();
  return r;
}

// Circle-method tournament: round r (0..P-2) pairs positions into P/2 disjoint pairs.
__device__ inline void tournament(int round, int k, int P, int& a, int& b) {
  if (k == 0) {
    a = P - 1;
    b = round;
  } else {
    a = (round + k) % (P - 1);
    b = (round - k + (P - 1)) % (P - 1);
  }
}

// QR with column pivoting of G (p x q, leading dimension ld, scaled to unit
// Frobenius norm), in place.  Stops when the trailing submatrix falls below
// kRankFloor2; returns the number of steps k.  sh.perm holds the column
// permutation (G P = Q R), sh.drop2 the squared norm of what was left out.
// Only R is kept: the reflector tails below the diagonal are dead afterwards.
// stop2: the factorisation stops once the squared norm of the remaining
// columns is at most stop2 (relative to a unit-norm G).  keep_tau: the
// reflector scalars are kept in sh.sigma[0 .. k) (each slot is free once its
// column has been chosen).
template <typename PT>
CLR_INLINE int pivoted_qr(PT* G, int p, int q, int64_t ld, RecShared& sh,
                          double stop2 = kRankFloor2, bool keep_tau = false) {
  const int tid = opaque_tid();
  const int lane = tid & 63, wave = tid >> 6;
  const int g = tid >> 4, gl = tid & 15;
  for (int j = g; j < q; j += kGroups) {
    const PT* c = G + (int64_t)j * ld;
    double s = 0.0;
    for (int i = gl; i < p; i += 16) s += c[i] * c[i];
    s = group_sum16(s);
    if (gl == 0) {
      sh.sigma[j] = s;
      sh.tails[j] = s;
      sh.perm[j] = j;
    }
  }
  __syncthreads();
  const int kmax = p < q ? p : q;
  int k = 0;
  for (; k < kmax; ++k) {
    if (wave == 0) {
      double best = -1.0, tot = 0.0;
      int bj = q;
      for (int j = k + lane; j < q; j += 64) {
        const double v = sh.sigma[j];
        tot += v;
        if (v > best || (v == best && j < bj)) {
          best = v;
          bj = j;
        }
      }
      for (int o = 32; o >= 1; o >>= 1) {
        const double ob = __shfl_xor(best, o, 64);
        const int oj = __shfl_xor(bj, o, 64);
        if (ob > best || (ob == best && oj < bj)) {
          best = ob;
          bj = oj;
        }
      }
      tot = wave_sum(tot);
      if (lane == 0) {
        sh.piv = bj;
        sh.drop2 = tot;
      }
    }
    __syncthreads();
    if (sh.drop2 <= stop2) break;
    const int piv = sh.piv;
    if (piv != k) {
      PT* a = G + (int64_t)k * ld;
      PT* b = G + (int64_t)piv * ld;
      for (int i = tid; i < p; i += kRecThreads) {
        const double t = a[i];
        a[i] = b[i];
        b[i] = t;
      }
      if (tid == 0) {
        double t = sh.sigma[k]; sh.sigma[k] = sh.sigma[piv]; sh.sigma[piv] = t;
        t = sh.tails[k]; sh.tails[k] = sh.tails[piv]; sh.tails[piv] = t;
        const int pi = sh.perm[k]; sh.perm[k] = sh.perm[piv]; sh.perm[piv] = pi;
      }
    }
    __syncthreads();
    PT* col = G + (int64_t)k * ld;
    if (wave == 0) {
      double s2 = 0.0;
      for (int i = k + 1 + lane; i < p; i += 64) s2 += col[i] * col[i];
      s2 = wave_sum(s2);
      const double x0 = col[k];
      double t = 0.0, beta = x0;
      if (s2 > 0.0) {
        beta = -copysign(sqrt(x0 * x0 + s2), x0);
        t = (beta - x0) / beta;
        const double scal = 1.0 / (x0 - beta);
        for (int i = k + 1 + lane; i < p; i += 64) col[i] *= scal;
      }
      if (lane == 0) {
        col[k] = beta;
        sh.tau = t;
        if (keep_tau) sh.sigma[k] = t;
      }
    }
    __syncthreads();
    const double t = sh.tau;
    for (int j = k + 1 + g; j < q; j += kGroups) {
      PT* cj = G + (int64_t)j * ld;
      double rkj = cj[k];
      if (t != 0.0) {
        double w = 0.0;
        for (int i = k + gl; i < p; i += 16) w += (i == k ? 1.0 : col[i]) * cj[i];
        w = group_sum16(w);
        double mine = 0.0;
        for (int i = k + gl; i < p; i += 16) {
          const double v = cj[i] - t * (i == k ? 1.0 : col[i]) * w;
          cj[i] = v;
          if (i == k) mine = v;   // the new R(k, j), held by one lane of the group
        }
        rkj = group_sum16(mine);
      }
      // partial column norm downdate with recomputation on cancellation
      const double nd = sh.sigma[j] - rkj * rkj;
      double nv;
      if (nd <= 1e-8 * sh.tails[j]) {
        double s = 0.0;
        for (int i = k + 1 + gl; i < p; i += 16) s += cj[i] * cj[i];
        nv = group_sum16(s);
        if (gl == 0) sh.tails[j] = nv;
      } else {
        nv = nd;
      }
      if (gl == 0) sh.sigma[j] = nv;
    }
    __syncthreads();
  }
  if (k == kmax && tid == 0) sh.drop2 = 0.0;
  __syncthreads();
  return k;
}

// Overwrite the leading q x k part of G with R(0:k, 0:q)^T (lower triangular).
template <typename PT>
CLR_INLINE void transpose_r(PT* G, int q, int k, int64_t ld) {
  // pairs (i, j), i < j < q, i < k: X(j, i) = R(i, j); X(i, j) = R(j, i) = 0 when j < k
  const int64_t total = (int64_t)k * q;
  for (int64_t e = opaque_tid(); e < total; e += kRecThreads) {
    const int i = (int)(e / q), j = (int)(e % q);
    if (j <= i) continue;
    const double v = G[i + (int64_t)j * ld];
    G[j + (int64_t)i * ld] = v;
    if (j < k) G[i + (int64_t)j * ld] = 0.0;
  }
  __syncthreads();
}

// One-sided Jacobi on the kc columns (length rows, leading dimension ld) of X.
// X has unit Frobenius norm; columns below kNegligible2 are left alone (they
// lie far below any truncation threshold and rotating them only chases
// rounding noise).  Each 16-lane group reads its column pair once into
// registers (rows <= 16 NR), forms the three inner products, and writes the
// pair back only when it rotates: one LDS pass per pair instead of three.
// Returns false if it did not converge.
template <int NR, typename PT>
CLR_INLINE bool jacobi_columns_t(PT* X, int rows, int kc, int64_t ld, RecShared& sh) {
  const int tid = opaque_tid();
  const int g = tid >> 4, gl = tid & 15;
  const int P = kc + (kc & 1);
  const double tolj = (double)rows * DBL_EPSILON;
  for (int sweep = 0; sweep < kJacobiMaxSweeps; ++sweep) {
    if (tid == 0) sh.flag = 0;
    __syncthreads();
    for (int round = 0; round < P - 1; ++round) {
      for (int pr = g; pr < P / 2; pr += kGroups) {
        int a, b;
        tournament(round, pr, P, a, b);
        if (a >= kc || b >= kc) continue;
        PT* wa = X + (int64_t)a * ld;
        PT* wb = X + (int64_t)b * ld;
        double xa[NR], xb[NR];
        double al = 0.0, be = 0.0, ga = 0.0;
#pragma unroll
        for (int t = 0; t < NR; ++t) {
          const int i = gl + 16 * t;
          xa[t] = i < rows ? wa[i] : 0.0;
          xb[t] = i < rows ? wb[i] : 0.0;
          al += xa[t] * xa[t];
          be += xb[t] * xb[t];
          ga += xa[t] * xb[t];
        }
        al = group_sum16(al);
        be = group_sum16(be);
        ga = group_sum16(ga);
        if (al > kNegligible2 && be > kNegligible2 && fabs(ga) > tolj * sqrt(al) * sqrt(be)) {
          const double zeta = (be - al) / (2.0 * ga);
          const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + hypot(1.0, zeta));
          const double c = 1.0 / sqrt(1.0 + t * t);
          const double s = c * t;
#pragma unroll
          for (int u = 0; u < NR; ++u) {
            const int i = gl + 16 * u;
            if (i < rows) {
              wa[i] = c * xa[u] - s * xb[u];
              wb[i] = s * xa[u] + c * xb[u];
            }
          }
          if (gl == 0) sh.flag = 1;
        }
      }
      __syncthreads();
    }
    const int rotated = sh.flag;
    __syncthreads();
    if (!rotated) return true;
  }
  return false;
}

// Two-pass variant for columns longer than 160 (blocks beyond the register engine).
template <typename PT>
CLR_INLINE bool jacobi_columns_long(PT* X, int rows, int kc, int64_t ld, RecShared& sh) {
  const int tid = opaque_tid();
  const int g = tid >> 4, gl = tid & 15;
  const int P = kc + (kc & 1);
  const double tolj = (double)rows * DBL_EPSILON;
  for (int sweep = 0; sweep < kJacobiMaxSweeps; ++sweep) {
    if (tid == 0) sh.flag = 0;
    __syncthreads();
    for (int round = 0; round < P - 1; ++round) {
      for (int pr = g; pr < P / 2; pr += kGroups) {
        int a, b;
        tournament(round, pr, P, a, b);
        if (a >= kc || b >= kc) continue;
        PT* wa = X + (int64_t)a * ld;
        PT* wb = X + (int64_t)b * ld;
        double al = 0.0, be = 0.0, ga = 0.0;
        for (int i = gl; i < rows; i += 16) {
          const double x = wa[i], y = wb[i];
          al += x * x;
          be += y * y;
          ga += x * y;
        }
        al = group_sum16(al);
        be = group_sum16(be);
        ga = group_sum16(ga);
        if (al > kNegligible2 && be > kNegligible2 && fabs(ga) > tolj * sqrt(al) * sqrt(be)) {
          const double zeta = (be - al) / (2.0 * ga);
          const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + hypot(1.0, zeta));
          const double c = 1.0 / sqrt(1.0 + t * t);
          const double s = c * t;
          for (int i = gl; i < rows; i += 16) {
            const double x = wa[i], y = wb[i];
            wa[i] = c * x - s * y;
            wb[i] = s * x + c * y;
          }
          if (gl == 0) sh.flag = 1;
        }
      }
      __syncthreads();
    }
    const int rotated = sh.flag;
    __syncthreads();
    if (!rotated) return true;
  }
  return false;
}

template <typename PT>
CLR_INLINE bool jacobi_columns(PT* X, int rows, int kc, int64_t ld, RecShared& sh) {
  if (rows <= 160) return jacobi_columns_t<10>(X, rows, kc, ld, sh);
  return jacobi_columns_long(X, rows, kc, ld, sh);
}

// Singular values (column norms of X, rows x kc), descending order (ties by
// index), tails including the part left out by the pivoted QR, and the kept
// rank for relative tolerance tol (the working matrix has unit norm).
template <typename PT>
CLR_INLINE int rank_from_columns(const PT* X, int rows, int kc, int64_t ld, double tol,
                                 RecShared& sh) {
  const int tid = opaque_tid();
  const int g = tid >> 4, gl = tid & 15;
  for (int j = g; j < kc; j += kGroups) {
    const PT* w = X + (int64_t)j * ld;
    double s = 0.0;
    for (int i = gl; i < rows; i += 16) s += w[i] * w[i];
    s = group_sum16(s);
    if (gl == 0) sh.sigma[j] = sqrt(s);
  }
  __syncthreads();
  for (int j = tid; j < kc; j += kRecThreads) {
    const double sj = sh.sigma[j];
    int pos = 0;
    for (int i = 0; i < kc; ++i) {
      const double si = sh.sigma[i];
      pos += (si > sj) || (si == sj && i < j);
    }
    sh.order[pos] = j;
  }
  __syncthreads();
  if (tid == 0) {
    double acc = sh.drop2;
    sh.tails[kc] = acc;
    for (int i = kc - 1; i >= 0; --i) {
      const double s = sh.sigma[sh.order[i]];
      acc += s * s;
      sh.tails[i] = acc;
    }
    int r = kc;
    for (int i = 0; i <= kc; ++i)
      if (sqrt(sh.tails[i]) <= tol) {
        r = i;
        break;
      }
    sh.rank = r;
  }
  __syncthreads();
  return sh.rank;
}

// Top-r right singular basis of G (q-long vectors): basis(:, c) = P x_{order[c]} / sigma.
template <typename PT, typename BT>
CLR_INLINE void write_basis(const PT* X, int64_t ld, int q, int r, BT* basis, int64_t ldb,
                            RecShared& sh) {
  for (int64_t e = opaque_tid(); e < (int64_t)q * r; e += kRecThreads) {
    const int j = (int)(e % q), c = (int)(e / q);
    const int src = sh.order[c];
    basis[sh.perm[j] + (int64_t)c * ldb] = X[j + (int64_t)src * ld] / sh.sigma[src];
  }
  __syncthreads();
}

// Pivoted QR + Jacobi on G (p x q, p >= q, unit norm): returns the kept rank;
// the Jacobi columns stay in G's leading q x k part for write_basis.
template <typename PT>
CLR_INLINE int svd_rank(PT* G, int p, int q, int64_t ld, double tol, int* status,
                        RecShared& sh) {
  const int kc = pivoted_qr(G, p, q, ld, sh);
  transpose_r(G, q, kc, ld);
  if (!jacobi_columns(G, q, kc, ld, sh)) {
    if (opaque_tid() == 0) atomicOr(status, 1);
  }
  return rank_from_columns(G, q, kc, ld, tol, sh);
}


// ---------------------------------------------------------------------------
// Register-resident engine for blocks with both edges <= 160.
//
// The working matrix G (p x q, p >= q, unit Frobenius norm) is spread over the
// 512 threads as a 16 x 32 grid: thread (tr, tc) = (tid % 16, tid / 16) holds
// G(i, j) for i = tr + 16 a, j = tc + 32 b (a < 10, b < 5).  A column lives in
// one 16-lane DPP row, so column reductions stay in the vector ALU; rows are
// reduced inside each wave with two lane exchanges and across the 8 waves
// through LDS.  This keeps 160 x 160 FP64 blocks (200 KiB) on chip, beyond the
// LDS capacity.
//
//  * Householder bidiagonalisation G = U_B B V_B^T.  Every wave computes each
//    reflector itself from the column or row published in LDS (identical
//    inputs and reduction order give bitwise identical reflectors), so a step
//    costs three workgroup barriers.  The right reflectors stay in LDS.
//  * Singular values of B by multisection on the Golub-Kahan tridiagonal
//    (zero diagonal, off-diagonals d_0, e_0, d_1, ...; eigenvalues +-sigma_i)
//    with Sturm counts.  A first round probes 512 log-spaced points, later
//    rounds split only the brackets that can still move the kept rank.
//  * Truncated blocks: the top-r values are refined to full precision and
//    each singular vector of B comes from one twisted factorisation of
//    T_GK - sigma I (one thread per vector); the right reflectors map them to
//    singular vectors of G.  Vectors of values closer than 1e-3 (relative)
//    are re-orthogonalised; if that collapses a vector (an unresolved
//    multiple value) the block falls back to pivoted QR + Jacobi.
// ---------------------------------------------------------------------------
constexpr int kRegEdge = 160;
constexpr int kRowCls = kRecThreads / 32;      // 16 row classes (one DPP row per column class)
constexpr int kRR = kRegEdge / kRowCls;        // 10 rows per thread
constexpr int kRC = kRegEdge / 32;             // 5 columns per thread
constexpr int kWaves = kRecThreads / 64;
constexpr int kVStore = kRegEdge * (kRegEdge - 1) / 2;
constexpr int kSeg = 32;                               // twisted-factorisation checkpoint interval
constexpr int kMaxSeg = (2 * kRegEdge + kSeg - 1) / kSeg;
constexpr int kMaxVec = kRegEdge / 2;                  // truncated ranks satisfy 2 r <= q
constexpr int kVecPerGroup = (kMaxVec + kGroups - 1) / kGroups;
constexpr double kProbeFloor = 1e-20;                  // brackets narrower than this are settled
static_assert(kWaves == 8 && kRecThreads == 512, "register engine layout assumes 512 threads");

struct RegLds {
  double vstore[kVStore];     // right reflector of step k at vs_off(k, q), length q - k - 1
  double tauR[kRegEdge];
  double d[kRegEdge];
  double e[kRegEdge];
  double colk[kRegEdge];      // pivoted QR: vector of the next left reflector
  double rowk[kRegEdge + 192];  // row of the next right reflector; zero tail for unmasked loads
  double tauL;
  int flag;
  union {
    struct {
      double part[kWaves][kRegEdge + 1];
      double wrow[kRegEdge];
      double colb[2][kRegEdge];  // published column of the next left reflector, by parity
    } bd;
    struct {
      double b2[2 * kRegEdge];
      double lo[kRegEdge];
      double hi[kRegEdge];
      int cnt[kRecThreads];
      int act[kRegEdge];
      int nact, rlo, rhi, rmid;
    } st;
    struct {
      double ckf[kMaxVec][kMaxSeg];
      double ckb[kMaxVec][kMaxSeg];
    } tw;
    struct {
      double colA[kRegEdge];
      double colB[kRegEdge];
    } qr;
  } u;
};
static_assert(sizeof(RegLds) <= (size_t)kRecLdsBytes, "register engine bookkeeping exceeds LDS");

typedef double RegTile[kRR][kRC];

CLR_INLINE void write_meta(const RecItem& it, int kind, int rank, double norm) {
  if (opaque_tid() == 0) {
    *it.kind_out = kind;
    *it.rank_out = rank;
    *it.norm_out = norm;
  }
}

CLR_INLINE int vs_off(int k, int q) { return k * (2 * q - k - 1) / 2; }

CLR_INLINE void reg_load(RegTile& a, const double* D, int64_t ldd, bool trans, double scale,
                         int p, int q) {
  const int tr = opaque_tid() & 15, tc = opaque_tid() >> 4;
#pragma unroll
  for (int ir = 0; ir < kRR; ++ir)
#pragma unroll
    for (int jc = 0; jc < kRC; ++jc) {
      const int i = tr + 16 * ir, j = tc + 32 * jc;
      double v = 0.0;
      const cgdbl* gD = (const cgdbl*)D;
      if (i < p && j < q) v = (trans ? gD[j + (int64_t)i * ldd] : gD[i + (int64_t)j * ldd]) * scale;
      a[ir][jc] = v;
    }
}

// Householder reflector (I - tau v v^T) x = beta e_1, v = (1, x[1:] * scal),
// from x0 = x[0] and s2 = |x[1:]|^2.  Each quotient has operands of
// comparable size, so columns whose norm is near the bottom of the exponent
// range (trailing columns of rapidly decaying spectra) stay finite; s2 = 0
// gives the identity (tau = 0), selected without a branch.
CLR_INLINE void house_from(double x0, double s2, double& beta, double& tau, double& scal) {
  const double bt = -copysign(sqrt(fma(x0, x0, s2)), x0);
  const double ta = (bt - x0) / bt;
  const double sc = 1.0 / (x0 - bt);
  const bool refl = s2 > 0.0;
  beta = refl ? bt : x0;
  tau = refl ? ta : 0.0;
  scal = refl ? sc : 0.0;
}

// Sum over the 16 lanes of a DPP row for code where every lane is active:
// the same butterfly as group_sum16 without a fill value for the moves.
template <int CTRL>
__device__ inline double dpp_move_full(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffLL), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ inline double row_sum16(double v) {
  v += dpp_move_full<0xB1>(v);
  v += dpp_move_full<0x4E>(v);
  v += dpp_move_full<0x141>(v);
  v += dpp_move_full<0x140>(v);
  return v;
}

__device__ inline double row_sum64(double v) { return xor32_sum(xor16_sum(row_sum16(v))); }

// Householder bidiagonalisation (Golub-Kahan) of the register-resident G:
// d, e, the right reflectors (vstore, tauR) in LDS.  The tile is left in an
// unspecified state.
//
// Layout: thread (tr, tc) = (tid & 15, tid >> 4) holds rows tr + 16 ir and
// columns tc + 32 jc.  A DPP row of 16 lanes therefore holds a whole column
// class, so sums over rows stay inside one wave; sums over columns cross the
// 8 waves and go through LDS.  Rows >= p and columns >= q of the tile are zero
// and stay zero (every weight built from them is zero).
//
// Phases: the steps k in [16 P, 16 P + 16) form phase P, compiled once per P.
// In phase P the row blocks ir < P hold only finished rows (< k) and the
// column blocks jc < P / 2 only finished columns (<= k), so the loops over
// the register tile start at P and P / 2 at compile time: the arithmetic
// follows the shrinking trailing matrix with no guards, and only the boundary
// blocks ir = P and jc = P / 2 (P / 2 + 1 for the pivot column of the right
// reflector at the end of an odd phase) carry element masks.  The finished
// entries of every published row and column are written as zeros, and the
// right-update row sums are stored with zeros on the rows they do not touch,
// so the reflector vectors need no masks beyond the one pivot element.
//
// Three barriers per step.  The owners of column k + 1 publish it after the
// left update of step k and before that step's right update; every thread
// loads it right after the first barrier, loads the right-update row sums w
// after the third, and rebuilds the updated column as published - tau w for
// itself, so the column norm of the next left reflector is a row-local DPP
// sum with no LDS round trip or barrier of its own.  The published column
// alternates between two buffers so the next publish cannot overwrite a
// column another wave is still reading.  Every LDS load is unconditional and
// issued in a batch ahead of its use.  Every wave derives the reflectors from
// bitwise identical sums (the butterflies add the same operands in the same
// order in every lane), so the tau != 0 tests are uniform in the workgroup.
struct BdCarry {
  double cbn[kRR];   // published column of the step, this thread's rows
  double wr[kRR];    // previous right-update row sums, this thread's rows
  double x0c, x0w;   // the same two at the step's diagonal row
  double tprev;      // tau of the previous right reflector (0 before the first)
};

// row_sum16 of v[B .. N), level by level so the chains interleave.
template <int B, int N>
__device__ inline void row_sum16_from(double (&v)[N]) {
#pragma unroll
  for (int i = B; i < N; ++i) v[i] += dpp_move_full<0xB1>(v[i]);
#pragma unroll
  for (int i = B; i < N; ++i) v[i] += dpp_move_full<0x4E>(v[i]);
#pragma unroll
  for (int i = B; i < N; ++i) v[i] += dpp_move_full<0x141>(v[i]);
#pragma unroll
  for (int i = B; i < N; ++i) v[i] += dpp_move_full<0x140>(v[i]);
}

// One step; returns false after the last column (left reflector only).
template <int P>
CLR_INLINE bool bd_step(RegTile& a, int k, int p, int q, RegLds& L, BdCarry& S) {
  constexpr int JB = P >> 1;   // first column block with unfinished columns
  const int tid = opaque_tid();
  const int tr = tid & 15, tc = tid >> 4;
  const int lane = tid & 63, wave = tid >> 6;
  const int kk = k - 16 * P;   // the diagonal row within block P
  // ---- left reflector on column k (rows < k of the column are zero)
  double c[kRR];
  double s2 = 0.0;
#pragma unroll
  for (int ir = P; ir < kRR; ++ir) c[ir] = S.cbn[ir] - S.tprev * S.wr[ir];
#pragma unroll
  for (int ir = P + 1; ir < kRR; ++ir) s2 += c[ir] * c[ir];
  s2 += (tr != kk) ? c[P] * c[P] : 0.0;
  s2 = row_sum16(s2);
  double beta, tau, scal;
  house_from(S.x0c - S.tprev * S.x0w, s2, beta, tau, scal);
  if (tid == 0) L.d[k] = beta;
  if (tau != 0.0) {
    double vr[kRR], w[kRC];
#pragma unroll
    for (int ir = P; ir < kRR; ++ir) vr[ir] = c[ir] * scal;
    vr[P] = (tr == kk) ? 1.0 : vr[P];
#pragma unroll
    for (int jc = JB; jc < kRC; ++jc) {
      w[jc] = 0.0;
#pragma unroll
      for (int ir = P; ir < kRR; ++ir) w[jc] += vr[ir] * a[ir][jc];
    }
    row_sum16_from<JB>(w);
    w[JB] *= (tc + 32 * JB > k) ? tau : 0.0;
#pragma unroll
    for (int jc = JB + 1; jc < kRC; ++jc) w[jc] *= tau;
#pragma unroll
    for (int ir = P; ir < kRR; ++ir)
#pragma unroll
      for (int jc = JB; jc < kRC; ++jc) a[ir][jc] -= vr[ir] * w[jc];
  }
  if (k == q - 1) return false;
  // ---- publish column k + 1 (before the right update) and row k, with their
  // finished entries as zeros
  const int k1 = k + 1;
  double* const nb = L.u.bd.colb[k1 & 1];
  if (tc == (k1 & 31)) {
    // column k + 1 lies in block JB, or in JB + 1 at the end of an odd phase
    if ((k1 >> 5) == JB) {
      nb[tr + 16 * P] = (tr > kk) ? a[P][JB] : 0.0;
#pragma unroll
      for (int ir = P + 1; ir < kRR; ++ir) nb[tr + 16 * ir] = a[ir][JB];
    } else if (JB + 1 < kRC) {
      nb[tr + 16 * P] = (tr > kk) ? a[P][JB + 1 < kRC ? JB + 1 : JB] : 0.0;
#pragma unroll
      for (int ir = P + 1; ir < kRR; ++ir) nb[tr + 16 * ir] = a[ir][JB + 1 < kRC ? JB + 1 : JB];
    }
  }
  if (tr == kk) {
    L.rowk[tc + 32 * JB] = (tc + 32 * JB > k) ? a[P][JB] : 0.0;
#pragma unroll
    for (int jc = JB + 1; jc < kRC; ++jc) L.rowk[tc + 32 * jc] = a[P][jc];
  }
  __syncthreads();
  // ---- everything published before the barrier, loaded at once: row k for
  // the right reflector, and column k + 1 for the next step
  double rv[3], rr[kRC];
#pragma unroll
  for (int t = 0; t < 3; ++t) rv[t] = L.rowk[k + 2 + lane + 64 * t];
  const double rx0 = L.rowk[k1];
#pragma unroll
  for (int jc = JB; jc < kRC; ++jc) rr[jc] = L.rowk[tc + 32 * jc];
#pragma unroll
  for (int ir = P; ir < kRR; ++ir) S.cbn[ir] = nb[tr + 16 * ir];
  S.x0c = nb[k1];
  // ---- right reflector on row k, elements k + 1 .. q - 1 (entries >= q are
  // zero), applied to rows > k
  s2 = 0.0;
#pragma unroll
  for (int t = 0; t < 3; ++t) s2 += rv[t] * rv[t];
  s2 = row_sum64(s2);
  house_from(rx0, s2, beta, tau, scal);
  if (tid == 0) {
    L.e[k] = beta;
    L.tauR[k] = tau;
  }
  if (wave == 0) {
    double* vs = L.vstore + vs_off(k, q);
    if (lane == 0) vs[0] = 1.0;
#pragma unroll
    for (int t = 0; t < 3; ++t) {
      const int j = k + 2 + lane + 64 * t;
      if (j < q) vs[j - k - 1] = rv[t] * scal;
    }
  }
  double vc[kRC];
#pragma unroll
  for (int jc = JB; jc < kRC; ++jc) vc[jc] = rr[jc] * scal;
  {
    const bool piv = tc == (k1 & 31);
    if ((k1 >> 5) == JB) {
      vc[JB] = piv ? 1.0 : vc[JB];
    } else if (JB + 1 < kRC) {
      vc[JB + 1 < kRC ? JB + 1 : JB] = piv ? 1.0 : vc[JB + 1 < kRC ? JB + 1 : JB];
    }
  }
  if (tau != 0.0) {
    double w[kRR];
#pragma unroll
    for (int ir = 0; ir < kRR; ++ir) {
      w[ir] = 0.0;
      if (ir >= P) {
#pragma unroll
        for (int jc = JB; jc < kRC; ++jc) w[ir] += a[ir][jc] * vc[jc];
      }
    }
    // sum over the 4 column classes of this wave (lanes 16 and 32 apart) as
    // a reduce-scatter: row pair (0, 1) of lanes keeps blocks 0-4 vs 5-9,
    // then halves (0-1, 2-3) keep blocks {0, 1} vs {3, 4}; block 2 (+5) is
    // summed over the halves in both.  Lane row rw = lane >> 4 ends with the
    // full sums of blocks b + {0, 1, 2} (rw = 0, 1) or b + {3, 4, 2} (rw = 2,
    // 3), b = 5 on odd rw.
    double u[5];
#pragma unroll
    for (int i = 0; i < 5; ++i) u[i] = swap16_sum(w[i], w[i + 5]);
    const double t0 = swap32_sum(u[0], u[3]);
    const double t1 = swap32_sum(u[1], u[4]);
    const double t2 = xor32_sum(u[2]);
    const int rw = lane >> 4;
    const int b = (rw & 1) ? 5 : 0, hi = (rw & 2) ? 3 : 0;
    double* const pw = L.u.bd.part[wave];
    pw[tr + 16 * (b + hi)] = t0;
    pw[tr + 16 * (b + hi + 1)] = t1;
    if (rw < 2) pw[tr + 16 * (b + 2)] = t2;
  }
  __syncthreads();
  if (tau != 0.0 && tid < kRegEdge) {
    double pw[kWaves];
#pragma unroll
    for (int w = 0; w < kWaves; ++w) pw[w] = L.u.bd.part[w][tid];
    const double s = ((pw[0] + pw[1]) + (pw[2] + pw[3])) + ((pw[4] + pw[5]) + (pw[6] + pw[7]));
    L.u.bd.wrow[tid] = (tid > k && tid < p) ? s : 0.0;
  }
  __syncthreads();
  if (tau != 0.0) {
#pragma unroll
    for (int ir = P; ir < kRR; ++ir) S.wr[ir] = L.u.bd.wrow[tr + 16 * ir];
    S.x0w = L.u.bd.wrow[k1];
#pragma unroll
    for (int ir = P; ir < kRR; ++ir) {
      const double w = tau * S.wr[ir];
#pragma unroll
      for (int jc = JB; jc < kRC; ++jc) a[ir][jc] -= w * vc[jc];
    }
  }
  S.tprev = tau;
  return true;
}

template <int P>
CLR_INLINE bool bd_phase(RegTile& a, int p, int q, RegLds& L, BdCarry& S) {
  const int ke = min(16 * P + 16, q);
  for (int k = 16 * P; k < ke; ++k)
    if (!bd_step<P>(a, k, p, q, L, S)) return false;
  return true;
}

CLR_INLINE void reg_bidiag(RegTile& a, int p_in, int q_in, RegLds& L) {
  static_assert(kRR == 10 && kRC == 5, "phase dispatch below assumes a 160 x 160 frame");
  // uniform in the workgroup; made explicit so loop bounds are scalar
  const int p = __builtin_amdgcn_readfirstlane(p_in), q = __builtin_amdgcn_readfirstlane(q_in);
  const int tid = opaque_tid();
  const int tr = tid & 15, tc = tid >> 4;
  if (tc == 0) {
#pragma unroll
    for (int ir = 0; ir < kRR; ++ir) L.u.bd.colb[0][tr + 16 * ir] = a[ir][0];
  }
  if (tid < 192) L.rowk[kRegEdge + tid] = 0.0;
  __syncthreads();
  BdCarry S;
#pragma unroll
  for (int ir = 0; ir < kRR; ++ir) {
    S.cbn[ir] = L.u.bd.colb[0][tr + 16 * ir];
    S.wr[ir] = 0.0;
  }
  S.x0c = L.u.bd.colb[0][0];
  S.x0w = 0.0;
  S.tprev = 0.0;
  bool go = true;
  if (go) go = bd_phase<0>(a, p, q, L, S);
  if (go && q > 16) go = bd_phase<1>(a, p, q, L, S);
  if (go && q > 32) go = bd_phase<2>(a, p, q, L, S);
  if (go && q > 48) go = bd_phase<3>(a, p, q, L, S);
  if (go && q > 64) go = bd_phase<4>(a, p, q, L, S);
  if (go && q > 80) go = bd_phase<5>(a, p, q, L, S);
  if (go && q > 96) go = bd_phase<6>(a, p, q, L, S);
  if (go && q > 112) go = bd_phase<7>(a, p, q, L, S);
  if (go && q > 128) go = bd_phase<8>(a, p, q, L, S);
  if (go && q > 144) go = bd_phase<9>(a, p, q, L, S);
}

// #{sigma_i > x} for the bidiagonal whose Golub-Kahan off-diagonals squared
// (d_0^2, e_0^2, d_1^2, ..., d_{q-1}^2) are in b2; x > 0.  Sylvester inertia of
// T - x I through its leading principal minors d_k = -x d_{k-1} - b_{k-1}^2 d_{k-2}
// (no divisions): every sign change is a negative pivot, i.e. an eigenvalue
// below x.  The pair (d_{k-1}, d_k) is rescaled by a power of two every 8 steps
// (growth per step is at most the golden ratio for a unit-norm matrix).  An
// exact zero minor needs no special case: it counts as non-negative, and since
// every b2 is positive (floored at 2^-600 where the off-diagonal vanishes) the
// next minor is -b2 d_{k-1}, of the opposite sign to d_{k-1}, so the two steps
// together add one sign change, as the pivot-floor rule of the quotient form
// does (a zero minor cannot be followed by another).  Only a zero last minor
// (x exactly an eigenvalue) may count either way.
CLR_INLINE int sturm_greater(const double* b2, int q, double x) {
  double dm = 1.0, d = -x;
  int neg = 1;
  if (d == 0.0) d = -1e-300;
  const int n = 2 * q - 1;
  auto step = [&](double bb) {
    const double dn = fma(-x, d, -bb * dm);
    neg += (dn < 0.0) != (d < 0.0);
    dm = d;
    d = dn;
  };
  int s = 0;
  // eight squared off-diagonals at a time: the LDS reads of a chunk are issued
  // together instead of one per dependent step
  for (; s + 8 <= n; s += 8) {
    double bb[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) bb[t] = b2[s + t];
#pragma unroll
    for (int t = 0; t < 8; ++t) step(bb[t]);
    int e;
    (void)frexp(d, &e);
    d = ldexp(d, -e);
    dm = ldexp(dm, -e);
  }
  for (; s < n; ++s) step(b2[s]);
  return 2 * q - neg;
}

CLR_INLINE double probe_point(int t) { return exp2(-0.125 * (double)t); }

CLR_INLINE bool bracket_settled(double lo, double hi) {
  return hi - lo <= fmax(0x1p-50 * hi, kProbeFloor);
}

CLR_INLINE int wave_isum(int v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Wave 0: kept-rank bounds from the brackets.  With T(r) = sum_{i>=r} s_i^2
// the kept rank is #{r < q : T(r) > tol^2}; evaluated with the lower ends,
// the upper ends and the midpoints of the brackets.
CLR_INLINE void rank_counts(const RegLds& L, int q, double bound, int& rlo, int& rhi, int& rmid) {
  const int lane = opaque_tid() & 63;
  double sl[3], shh[3], sm[3];
  double cl = 0.0, ch = 0.0, cm = 0.0;
#pragma unroll
  for (int t = 2; t >= 0; --t) {
    const int i = 3 * lane + t;
    if (i < q) {
      const double lo = L.u.st.lo[i], hi = L.u.st.hi[i], mid = 0.5 * (lo + hi);
      cl += lo * lo;
      ch += hi * hi;
      cm += mid * mid;
    }
    sl[t] = cl;
    shh[t] = ch;
    sm[t] = cm;
  }
  // sums over the chunks of the lanes above this one
  double xl = cl, xh = ch, xm = cm;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const double tl = __shfl_down(xl, o, 64), th = __shfl_down(xh, o, 64), tm = __shfl_down(xm, o, 64);
    if (lane + o < 64) {
      xl += tl;
      xh += th;
      xm += tm;
    }
  }
  const double el = xl - cl, eh = xh - ch, em = xm - cm;
  int nl = 0, nh = 0, nm = 0;
#pragma unroll
  for (int t = 0; t < 3; ++t) {
    const int i = 3 * lane + t;
    if (i < q) {
      nl += (sl[t] + el > bound);
      nh += (shh[t] + eh > bound);
      nm += (sm[t] + em > bound);
    }
  }
  rlo = wave_isum(nl);
  rhi = wave_isum(nh);
  rmid = wave_isum(nm);
}

// One multisection round over the active brackets (S.act[0 .. nact)).
CLR_INLINE void multisect_round(int q, int nact, RegLds& L) {
  auto& S = L.u.st;
  const int tid = opaque_tid();
  const int ts = kRecThreads / nact;
  const int a = tid / ts, sub = tid % ts;
  // probe points lo + (s + 1) w, w = (hi - lo) / (ts + 1), computed the same
  // way by the probing threads and by the bracket update
  if (a < nact) {
    const int i = S.act[a];
    const double lo = S.lo[i], w = (S.hi[i] - lo) / (double)(ts + 1);
    const double x = lo + (double)(sub + 1) * w;
    S.cnt[tid] = sturm_greater(S.b2, q, x);
  }
  __syncthreads();
  if (a < nact && sub == 0) {
    const int i = S.act[a];
    const double lo = S.lo[i], hi = S.hi[i], w = (hi - lo) / (double)(ts + 1);
    double nlo = lo, nhi = hi;
    for (int s2 = 0; s2 < ts; ++s2) {
      const double x = lo + (double)(s2 + 1) * w;
      if (S.cnt[a * ts + s2] > i) {
        nlo = x;
      } else {
        nhi = x;
        break;
      }
    }
    S.lo[i] = nlo;
    S.hi[i] = nhi;
  }
  __syncthreads();
}

// Wave 0: active list of the unsettled brackets with index in [from, to).
CLR_INLINE int collect_active(RegLds& L, int from, int to) {
  auto& S = L.u.st;
  const int lane = opaque_tid() & 63;
  int base = 0;
  for (int c0 = 0; c0 < to; c0 += 64) {
    const int i = c0 + lane;
    const bool act = i >= from && i < to && !bracket_settled(S.lo[i], S.hi[i]);
    const unsigned long long msk = __ballot(act);
    if (act) S.act[base + __popcll(msk & ((1ull << lane) - 1ull))] = i;
    base += __popcll(msk);
  }
  return base;
}

// Singular values of the bidiagonal (d, e in LDS) and the kept rank for tol.
// Brackets end in L.u.st.lo / hi; sh.sigma receives the midpoints.
CLR_INLINE int reg_decide(int q, double tol, RegLds& L, RecShared& sh) {
  auto& S = L.u.st;
  const int tid = opaque_tid(), wave = tid >> 6, lane = tid & 63;
  if (tid < 2 * q - 1) {
    const double b = (tid & 1) ? L.e[tid >> 1] : L.d[tid >> 1];
    S.b2[tid] = fmax(b * b, 0x1p-600);   // positive: see sturm_greater
  }
  __syncthreads();
  S.cnt[tid] = sturm_greater(S.b2, q, probe_point(tid));
  __syncthreads();
  if (tid < q) {
    int lo_t = 0, hi_t = kRecThreads;   // first probe with more than tid values above it
    while (lo_t < hi_t) {
      const int mid = (lo_t + hi_t) >> 1;
      if (S.cnt[mid] > tid)
        hi_t = mid;
      else
        lo_t = mid + 1;
    }
    if (lo_t == kRecThreads) {
      S.lo[tid] = 0.0;
      S.hi[tid] = probe_point(kRecThreads - 1);
    } else {
      S.lo[tid] = probe_point(lo_t);
      S.hi[tid] = lo_t == 0 ? 1.0 + 1e-12 : probe_point(lo_t - 1);
    }
  }
  __syncthreads();
  const double bound = tol * tol;
  for (int round = 0; round < 256; ++round) {
    if (wave == 0) {
      int rlo, rhi, rmid;
      rank_counts(L, q, bound, rlo, rhi, rmid);
      const bool settled = rlo == rhi || 2 * rlo > q;
      const int nact = settled ? 0 : collect_active(L, rlo, q);
      if (lane == 0) {
        S.nact = nact;
        S.rlo = rlo;
        S.rmid = rmid;
        sh.flag = settled ? 1 : 0;
      }
    }
    __syncthreads();
    if (sh.flag || S.nact == 0) break;
    multisect_round(q, S.nact, L);
  }
  const int r = sh.flag ? S.rlo : S.rmid;
  __syncthreads();
  return r;
}

// Full-precision brackets for values 0 .. r-1; midpoints into sh.sigma.
CLR_INLINE void reg_refine_top(int q, int r, RegLds& L, RecShared& sh) {
  auto& S = L.u.st;
  const int tid = opaque_tid(), wave = tid >> 6, lane = tid & 63;
  for (int round = 0; round < 256; ++round) {
    if (wave == 0) {
      const int nact = collect_active(L, 0, r);
      if (lane == 0) S.nact = nact;
    }
    __syncthreads();
    if (S.nact == 0) break;
    multisect_round(q, S.nact, L);
  }
  if (tid < q) sh.sigma[tid] = 0.5 * (S.lo[tid] + S.hi[tid]);
  __syncthreads();
}

// Golub-Kahan off-diagonal c_i (i < 2q - 1): d_0, e_0, d_1, e_1, ...
#define GK_C(L, i) (((i) & 1) ? (L).e[(i) >> 1] : (L).d[(i) >> 1])
CLR_INLINE double pivot_floor(double x) { return x != 0.0 ? x : -1e-300; }

// 1 / x by the hardware reciprocal estimate and two Newton-Raphson steps
// r <- r + r (1 - x r) (each step squares the relative error, ending within
// about one unit in the last place): five dependent operations instead of the
// correctly rounded division's ten, on the serial pivot chains below.  x is a
// pivot: nonzero, finite.
CLR_INLINE double recip_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}
// Next pivot of a twisted factorisation: -lam - c^2 / d.
CLR_INLINE double next_pivot(double lam, double c, double d) {
  return pivot_floor(fma(-(c * c), recip_nr(d), -lam));
}

// Right singular vector of the bidiagonal for the singular value lam, as the
// even entries of the eigenvector z of T_GK (size n = 2q) for +lam, from the
// twisted factorisation of T_GK - lam I: top-down pivots D+ (L D+ L^T) and
// bottom-up pivots D- (U D- U^T) meet at the index k where
// |gamma_k| = |D+_k + D-_k + lam| is smallest; z_k = 1 and the other entries
// follow from the two bidiagonal factors.  Pivots are kept only every kSeg
// entries (ckf, ckb) and recomputed segment by segment.  Writes the q entries
// (unnormalised) to v; returns false on a non-finite result.
CLR_INLINE bool twisted_vector(const RegLds& L, double* ckf, double* ckb, int q, double lam,
                               gdbl* v) {
  const int n = 2 * q;
  const int nseg = (n + kSeg - 1) / kSeg;
  // forward pivots; ckf[s] = D+_{32 s - 1}
  {
    double dp = pivot_floor(-lam);
    for (int s = 0; s < nseg; ++s) {
      if (s > 0) ckf[s] = dp;
#pragma unroll
      for (int t = 0; t < kSeg; ++t) {
        const int i = kSeg * s + t;
        if (i > 0 && i < n) {
          dp = next_pivot(lam, GK_C(L, i - 1), dp);
        }
      }
    }
  }
  // backward pivots with the twist search; ckb[s] = D-_{32 s + 32}
  double best = 1e300;
  int kst = n - 1;
  {
    double dm = pivot_floor(-lam);
    for (int s = nseg - 1; s >= 0; --s) {
      double seg[kSeg];
      double x = s > 0 ? ckf[s] : 0.0;
#pragma unroll
      for (int t = 0; t < kSeg; ++t) {
        const int i = kSeg * s + t;
        if (i < n) {
          if (i == 0) {
            x = pivot_floor(-lam);
          } else {
            x = next_pivot(lam, GK_C(L, i - 1), x);
          }
        }
        seg[t] = x;
      }
      if (s < nseg - 1) ckb[s] = dm;
#pragma unroll
      for (int t = kSeg - 1; t >= 0; --t) {
        const int i = kSeg * s + t;
        if (i < n) {
          if (i < n - 1) dm = next_pivot(lam, GK_C(L, i), dm);
          const double g = fabs(seg[t] + dm + lam);
          if (g < best) {
            best = g;
            kst = i;
          }
        }
      }
    }
  }
  double nrm2 = 0.0;
  if ((kst & 1) == 0) {
    v[kst >> 1] = 1.0;
    nrm2 = 1.0;
  }
  // entries above the twist: z_i = -(c_i / D+_i) z_{i+1}
  {
    double z = 1.0;
    for (int s = (kst - 1) / kSeg; kst > 0 && s >= 0; --s) {
      double seg[kSeg];
      double x = s > 0 ? ckf[s] : 0.0;
#pragma unroll
      for (int t = 0; t < kSeg; ++t) {
        const int i = kSeg * s + t;
        if (i < n) {
          if (i == 0) {
            x = pivot_floor(-lam);
          } else {
            x = next_pivot(lam, GK_C(L, i - 1), x);
          }
        }
        seg[t] = x;
      }
#pragma unroll
      for (int t = kSeg - 1; t >= 0; --t) {
        const int i = kSeg * s + t;
        if (i < kst) {
          z = -(GK_C(L, i) * recip_nr(seg[t])) * z;
          if ((t & 1) == 0) {
            v[i >> 1] = z;
            nrm2 += z * z;
          }
        }
      }
    }
  }
  // entries below the twist: z_i = -(c_{i-1} / D-_i) z_{i-1}
  {
    double z = 1.0;
    for (int s = (kst + 1) / kSeg; s < nseg; ++s) {
      double seg[kSeg];
      double y = s < nseg - 1 ? ckb[s] : 0.0;
#pragma unroll
      for (int t = kSeg - 1; t >= 0; --t) {
        const int i = kSeg * s + t;
        if (i < n) {
          if (i == n - 1) {
            y = pivot_floor(-lam);
          } else {
            y = next_pivot(lam, GK_C(L, i), y);
          }
        }
        seg[t] = y;
      }
#pragma unroll
      for (int t = 0; t < kSeg; ++t) {
        const int i = kSeg * s + t;
        if (i > kst && i < n) {
          z = -(GK_C(L, i - 1) * recip_nr(seg[t])) * z;
          if ((t & 1) == 0) {
            v[i >> 1] = z;
            nrm2 += z * z;
          }
        }
      }
    }
  }
  return nrm2 > 0.0 && nrm2 < 1e300;
}
#undef GK_C

// Values c - 1 and c belong to one cluster (vectors re-orthogonalised).
CLR_INLINE bool close_values(const RecShared& sh, int c) {
  return sh.sigma[c - 1] - sh.sigma[c] < 1e-3 * sh.sigma[c - 1];
}

// Top-r right singular basis of G (q-long, orthonormal) into basis (ld q) and
// the other factor G_orig * basis, from the bidiagonal in LDS.  Returns false
// (nothing final written) when a vector cannot be resolved this way.
CLR_INLINE bool reg_vectors(const RecItem& it, int p, int q, bool trans, int r, double normc,
                            RegLds& L, RecShared& sh, GemmItem* gout, Seg* gseg, int gidx) {
  const int tid = opaque_tid();
  const int g = tid >> 4, gl = tid & 15;
  const int m = it.m;
  gdbl* Uo = (gdbl*)it.out;
  gdbl* Vo = Uo + (int64_t)m * r;
  gdbl* basis = trans ? Uo : Vo;
  gdbl* other = trans ? Vo : Uo;   // p x r >= q x r: staging for the raw vectors
  reg_refine_top(q, r, L, sh);
  if (tid == 0) L.flag = 0;
  __syncthreads();
  if (tid < r) {
    if (!twisted_vector(L, L.u.tw.ckf[tid], L.u.tw.ckb[tid], q, sh.sigma[tid],
                        other + (int64_t)tid * q))
      L.flag = 1;
  }
  __syncthreads();
  if (L.flag) return false;
  // normalise and map through the right reflectors: vectors c = g + 32 u,
  // lane gl holds entries j = gl + 16 t
  double vv[kVecPerGroup][kRR];
#pragma unroll
  for (int u = 0; u < kVecPerGroup; ++u) {
    const int c = g + kGroups * u;
    double s = 0.0;
#pragma unroll
    for (int t = 0; t < kRR; ++t) {
      const int j = gl + 16 * t;
      vv[u][t] = (c < r && j < q) ? other[j + (int64_t)c * q] : 0.0;
      s += vv[u][t] * vv[u][t];
    }
    s = group_sum16(s);
    const double inv = s > 0.0 ? 1.0 / sqrt(s) : 0.0;
#pragma unroll
    for (int t = 0; t < kRR; ++t) vv[u][t] *= inv;
  }
  if (g < r) {
    for (int k = q - 2; k >= 0; --k) {
      const double tau = L.tauR[k];
      if (tau == 0.0) continue;
      const double* vs = L.vstore + vs_off(k, q);
      double w[kRR];
#pragma unroll
      for (int t = 0; t < kRR; ++t) {
        const int j = gl + 16 * t;
        w[t] = (j > k && j < q) ? vs[j - k - 1] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < kVecPerGroup; ++u) {
        if (g + kGroups * u < r) {
          double dot = 0.0;
#pragma unroll
          for (int t = 0; t < kRR; ++t) dot += w[t] * vv[u][t];
          dot = tau * group_sum16(dot);
#pragma unroll
          for (int t = 0; t < kRR; ++t) vv[u][t] -= w[t] * dot;
        }
      }
    }
  }
  __syncthreads();   // reflectors consumed: vstore becomes the vector store X (q x r)
  double* X = L.vstore;
#pragma unroll
  for (int u = 0; u < kVecPerGroup; ++u) {
    const int c = g + kGroups * u;
    if (c < r) {
#pragma unroll
      for (int t = 0; t < kRR; ++t) {
        const int j = gl + 16 * t;
        if (j < q) X[j + c * q] = vv[u][t];
      }
    }
  }
  __syncthreads();
  // re-orthogonalise within clusters of close values (one vector at a time)
  for (int c = 1; c < r; ++c) {
    int c0 = c;
    while (c0 > 0 && close_values(sh, c0)) --c0;
    if (c0 == c) continue;
    if (g == 0) {
      double* xc = X + c * q;
      for (int b = c0; b < c; ++b) {
        const double* xb = X + b * q;
        double dot = 0.0;
        for (int j = gl; j < q; j += 16) dot += xb[j] * xc[j];
        dot = group_sum16(dot);
        for (int j = gl; j < q; j += 16) xc[j] -= dot * xb[j];
      }
      double s = 0.0;
      for (int j = gl; j < q; j += 16) s += xc[j] * xc[j];
      s = group_sum16(s);
      if (!(s > 1e-2)) {
        if (gl == 0) L.flag = 1;
      } else {
        const double inv = 1.0 / sqrt(s);
        for (int j = gl; j < q; j += 16) xc[j] *= inv;
      }
    }
    __syncthreads();
  }
  if (L.flag) return false;
  for (int e = tid; e < q * r; e += kRecThreads) basis[e] = X[e];
  // The other factor, G_orig * basis (G_orig = D for m >= n, D^T otherwise),
  // is an ordinary dense product: it is emitted as one grouped-GEMM item and
  // computed on MFMA by the launch that follows this kernel.
  if (tid == 0) {
    Seg sg{};
    sg.L = it.D;
    sg.sLi = trans ? it.ldd : 1;
    sg.sLk = trans ? 1 : it.ldd;
    sg.R = (const double*)basis;
    sg.sRk = 1;
    sg.sRj = q;
    sg.k = q;
    sg.kbase = 0;
    sg.scale = 1.0;
    gseg[gidx] = sg;
    GemmItem g{};
    g.C = (double*)other;
    g.ldc = p;
    g.row0 = 0;
    g.col0 = 0;
    g.m = p;
    g.n = r;
    g.seg0 = gidx;   // this item's term sits at the same index of the term array
    g.nseg = 1;
    g.ktotal = q;
    g.accumulate = 0;
    g.alpha = 1.0;
    gout[gidx] = g;
  }
  double kept = 0.0;
  for (int c = 0; c < r; ++c) kept += sh.sigma[c] * sh.sigma[c];
  write_meta(it, 2, r, normc * sqrt(kept));
  return true;
}

// Left reflector of the pivoted QR on column k of the tile (vector in colk).
CLR_INLINE void reg_left(RegTile& a, int k, int p, int q, RegLds& L) {
  const int tr = opaque_tid() & 15, tc = opaque_tid() >> 4;
  const int kj = k >> 5;
  if (tc == (k & 31)) {
    double s2 = 0.0, x0p = 0.0;
#pragma unroll
    for (int ir = 0; ir < kRR; ++ir)
#pragma unroll
      for (int jc = 0; jc < kRC; ++jc)
        if (jc == kj) {
          const int i = tr + 16 * ir;
          const double x = a[ir][jc];
          if (i > k && i < p) s2 += x * x;
          if (i == k) x0p = x;
        }
    s2 = group_sum16(s2);
    const double x0 = group_sum16(x0p);
    double t = 0.0, beta = x0, scal = 0.0;
    if (s2 > 0.0) {
      beta = -copysign(sqrt(x0 * x0 + s2), x0);
      t = (beta - x0) / beta;
      scal = 1.0 / (x0 - beta);
    }
#pragma unroll
    for (int ir = 0; ir < kRR; ++ir)
#pragma unroll
      for (int jc = 0; jc < kRC; ++jc)
        if (jc == kj) {
          const int i = tr + 16 * ir;
          if (i >= k && i < p) {
            L.colk[i] = (i == k) ? 1.0 : a[ir][jc] * scal;
            a[ir][jc] = (i == k) ? beta : 0.0;
          }
        }
    if (tr == 0) L.tauL = t;
  }
  __syncthreads();
  const double t = L.tauL;
  if (t == 0.0) return;
  double vr[kRR];
#pragma unroll
  for (int ir = 0; ir < kRR; ++ir) {
    const int i = tr + 16 * ir;
    vr[ir] = (i >= k && i < p) ? L.colk[i] : 0.0;
  }
#pragma unroll
  for (int jc = 0; jc < kRC; ++jc) {
    const int j = tc + 32 * jc;
    if (j > k && j < q) {
      double w = 0.0;
#pragma unroll
      for (int ir = 0; ir < kRR; ++ir) w += vr[ir] * a[ir][jc];
      w = group_sum16(w);
#pragma unroll
      for (int ir = 0; ir < kRR; ++ir) a[ir][jc] -= t * vr[ir] * w;
    }
  }
}

// Pivoted Householder QR of the register-resident G; stops at the numerical
// rank (trailing squared norm <= kRankFloor2).  Returns the number of steps k;
// R(0:k, :) stays in the registers, sh.perm holds the permutation.
CLR_INLINE int reg_pivoted_qr(RegTile& a, int p, int q, RegLds& L, RecShared& sh) {
  const int tid = opaque_tid();
  const int tr = tid & 15, tc = tid >> 4;
  const int lane = tid & 63, wave = tid >> 6;
  auto column_norms = [&](int from_row, int from_col) {
#pragma unroll
    for (int jc = 0; jc < kRC; ++jc) {
      const int j = tc + 32 * jc;
      if (j >= from_col && j < q) {
        double s = 0.0;
#pragma unroll
        for (int ir = 0; ir < kRR; ++ir) {
          const int i = tr + 16 * ir;
          if (i >= from_row && i < p) s += a[ir][jc] * a[ir][jc];
        }
        s = group_sum16(s);
        if (tr == 0) sh.sigma[j] = s;
      }
    }
  };
  column_norms(0, 0);
  if (tid < q) sh.perm[tid] = tid;
  __syncthreads();
  int k = 0;
  for (; k < q; ++k) {
    if (wave == 0) {
      double best = -1.0, tot = 0.0;
      int bj = q;
      for (int j = k + lane; j < q; j += 64) {
        const double v = sh.sigma[j];
        tot += v;
        if (v > best || (v == best && j < bj)) {
          best = v;
          bj = j;
        }
      }
      for (int o = 32; o >= 1; o >>= 1) {
        const double ob = __shfl_xor(best, o, 64);
        const int oj = __shfl_xor(bj, o, 64);
        if (ob > best || (ob == best && oj < bj)) {
          best = ob;
          bj = oj;
        }
      }
      tot = wave_sum(tot);
      if (lane == 0) {
        sh.piv = bj;
        sh.drop2 = tot;
      }
    }
    __syncthreads();
    if (sh.drop2 <= kRankFloor2) break;
    const int piv = sh.piv;
    if (piv != k) {
      const int kj = k >> 5, pj = piv >> 5;
#pragma unroll
      for (int ir = 0; ir < kRR; ++ir)
#pragma unroll
        for (int jc = 0; jc < kRC; ++jc) {
          const int i = tr + 16 * ir;
          if (i < p) {
            if (tc == (k & 31) && jc == kj) L.u.qr.colA[i] = a[ir][jc];
            if (tc == (piv & 31) && jc == pj) L.u.qr.colB[i] = a[ir][jc];
          }
        }
      __syncthreads();
#pragma unroll
      for (int ir = 0; ir < kRR; ++ir)
#pragma unroll
        for (int jc = 0; jc < kRC; ++jc) {
          const int i = tr + 16 * ir;
          if (i < p) {
            if (tc == (k & 31) && jc == kj) a[ir][jc] = L.u.qr.colB[i];
            if (tc == (piv & 31) && jc == pj) a[ir][jc] = L.u.qr.colA[i];
          }
        }
      if (tid == 0) {
        const double t = sh.sigma[k];
        sh.sigma[k] = sh.sigma[piv];
        sh.sigma[piv] = t;
        const int pi = sh.perm[k];
        sh.perm[k] = sh.perm[piv];
        sh.perm[piv] = pi;
      }
      __syncthreads();
    }
    reg_left(a, k, p, q, L);
    column_norms(k + 1, k + 1);
    __syncthreads();
  }
  if (k == q && tid == 0) sh.drop2 = 0.0;
  __syncthreads();
  return k;
}

// X (q x kq, leading dimension ldx) = R(0:kq, 0:q)^T from the registers.
template <typename PT>
CLR_INLINE void reg_store_rt(const RegTile& a, int q, int kq, PT* X, int64_t ldx) {
  const int tr = opaque_tid() & 15, tc = opaque_tid() >> 4;
#pragma unroll
  for (int ir = 0; ir < kRR; ++ir)
#pragma unroll
    for (int jc = 0; jc < kRC; ++jc) {
      const int i = tr + 16 * ir, j = tc + 32 * jc;
      if (i < kq && j < q) X[j + (int64_t)i * ldx] = (j >= i) ? a[ir][jc] : 0.0;
    }
  __syncthreads();
}

CLR_INLINE void copy_dense_out(const RecItem& it) {
  const int64_t total = (int64_t)it.m * it.n;
  const cgdbl* D = (const cgdbl*)it.D;
  gdbl* out = (gdbl*)it.out;
  for (int64_t e = opaque_tid(); e < total; e += kRecThreads) {
    const int i = (int)(e % it.m), j = (int)(e / it.m);
    out[e] = D[i + (int64_t)j * it.ldd];
  }
}

// Householder QR of W (rows x cols, ld rows) in place: R in the upper
// triangle, reflector tails below the diagonal, tau[k] alongside
// (H_k = I - tau_k v_k v_k^T, v_k = (1, W[k+1:, k])).
template <typename PT>
CLR_INLINE void householder_qr(PT* W, int rows, int cols, PT* tau) {
  const int tid = opaque_tid();
  const int lane = tid & 63, wave = tid >> 6;
  const int g = tid >> 4, gl = tid & 15;
  for (int k = 0; k < cols && k < rows; ++k) {
    PT* col = W + (int64_t)k * rows;
    if (wave == 0) {
      double s2 = 0.0;
      for (int i = k + 1 + lane; i < rows; i += 64) s2 += col[i] * col[i];
      s2 = wave_sum(s2);
      const double x0 = col[k];
      double t = 0.0, beta = x0;
      if (s2 > 0.0) {
        beta = -copysign(sqrt(x0 * x0 + s2), x0);
        t = (beta - x0) / beta;
        const double scal = 1.0 / (x0 - beta);
        for (int i = k + 1 + lane; i < rows; i += 64) col[i] *= scal;
      }
      if (lane == 0) {
        col[k] = beta;
        tau[k] = t;
      }
    }
    __syncthreads();
    const double t = tau[k];
    if (t != 0.0) {
      for (int j = k + 1 + g; j < cols; j += kGroups) {
        PT* cj = W + (int64_t)j * rows;
        double w = 0.0;
        for (int i = k + gl; i < rows; i += 16) w += (i == k ? 1.0 : col[i]) * cj[i];
        w = group_sum16(w);
        for (int i = k + gl; i < rows; i += 16) cj[i] -= t * (i == k ? 1.0 : col[i]) * w;
      }
    }
    __syncthreads();
  }
}

// X (rows x ncol, ld ldx, global) <- Q X with Q = H_0 H_1 ... H_{kk-1} from householder_qr.
template <typename PT, typename TT = PT>
CLR_INLINE void apply_q(const PT* W, int rows, int kk, const TT* tau, gdbl* X, int64_t ldx,
                        int ncol) {
  const int tid = opaque_tid();
  const int g = tid >> 4, gl = tid & 15;
  for (int c = g; c < ncol; c += kGroups) {
    gdbl* x = X + (int64_t)c * ldx;
    for (int k = kk - 1; k >= 0; --k) {
      const double t = tau[k];
      if (t == 0.0) continue;
      const PT* v = W + (int64_t)k * rows;
      double w = 0.0;
      for (int i = k + gl; i < rows; i += 16) w += (i == k ? 1.0 : v[i]) * x[i];
      w = group_sum16(w);
      for (int i = k + gl; i < rows; i += 16) x[i] -= t * (i == k ? 1.0 : v[i]) * w;
    }
  }
  __syncthreads();
}

// Factored output of a truncated dense-path block from the sorted Jacobi
// columns X (q rows, leading dimension ldx) of the working matrix G:
//   basis = right singular vectors of G (q-long), other = G_orig * basis;
//   m >= n: V' = basis (n x r), U' = D basis (m x r)
//   m <  n: U' = basis (m x r), V' = D^T basis (n x r)
template <typename PT>
CLR_INLINE void dense_truncated_out(const RecItem& it, const PT* X, int64_t ldx, int p, int q,
                                    bool trans, int r, double normc, RecShared& sh) {
  const int m = it.m, n = it.n;
  double kept = 0.0;
  for (int c = 0; c < r; ++c) {
    const double s = sh.sigma[sh.order[c]];
    kept += s * s;
  }
  kept *= normc * normc;
  gdbl* Uo = (gdbl*)it.out;
  gdbl* Vo = Uo + (int64_t)m * r;
  gdbl* basis = trans ? Uo : Vo;
  gdbl* other = trans ? Vo : Uo;
  write_basis(X, ldx, q, r, basis, q, sh);
  const cgdbl* D = (const cgdbl*)it.D;
  const int g = opaque_tid() >> 4, gl = opaque_tid() & 15;
  for (int o = g; o < p * r; o += kGroups) {
    const int i = o % p, c = o / p;
    const gdbl* b = basis + (int64_t)c * q;
    double s = 0.0;
    if (!trans) {
      for (int j = gl; j < n; j += 16) s += D[i + (int64_t)j * it.ldd] * b[j];
    } else {
      const cgdbl* dcol = D + (int64_t)i * it.ldd;   // column i of D (m long)
      for (int j = gl; j < m; j += 16) s += dcol[j] * b[j];
    }
    s = group_sum16(s);
    if (gl == 0) other[i + (int64_t)c * p] = s;
  }
  write_meta(it, 2, r, sqrt(kept));
}

// Jacobi on the register engine's R^T, then the factored output.
template <typename PT>
CLR_INLINE void reg_truncated(const RecItem& it, const RegTile& a, PT* X, int64_t ldx, int p,
                              int q, int kc, bool trans, int r, double tol, double normc,
                              int* status, RecShared& sh) {
  reg_store_rt(a, q, kc, X, ldx);
  if (!jacobi_columns(X, q, kc, ldx, sh)) {
    if (opaque_tid() == 0) atomicOr(status, 1);
  }
  // sorted Jacobi columns give the vectors; the rank decided from the bidiagonal stands
  (void)rank_from_columns(X, q, kc, ldx, tol, sh);
  dense_truncated_out(it, X, ldx, p, q, trans, r < kc ? r : kc, normc, sh);
}

// Dense path on a working matrix in LDS or global scratch (blocks beyond the
// register engine): pivoted QR + Jacobi decide the rank and give the vectors.
template <typename PT>
CLR_INLINE void dense_general(const RecItem& it, PT* G, int p, int q, bool trans, double tol,
                              double normc, int* status, RecShared& sh) {
  const int m = it.m, n = it.n;
  const double inv_norm = 1.0 / normc;
  const cgdbl* D = (const cgdbl*)it.D;
  for (int64_t e = opaque_tid(); e < (int64_t)m * n; e += kRecThreads) {
    const int i = (int)(e % m), j = (int)(e / m);
    const double v = D[i + (int64_t)j * it.ldd] * inv_norm;
    if (!trans)
      G[i + (int64_t)j * p] = v;
    else
      G[j + (int64_t)i * p] = v;
  }
  __syncthreads();
  const int r = svd_rank(G, p, q, p, tol, status, sh);
  if (r == 0) {
    write_meta(it, 0, 0, 0.0);
    return;
  }
  if (2 * r > q) {
    copy_dense_out(it);
    write_meta(it, 1, q, normc);
    return;
  }
  dense_truncated_out(it, G, p, p, q, trans, r, normc, sh);
}

// Truncation of a dense block by the paper's rank-revealing QR (Sec. 4.1):
// column-pivoted Householder QR of G = D / ||D||_F (m x n, columns of D
// pivoted), stopped at the first k whose remaining columns have squared norm
// <= tol^2, i.e. ||D - Q_k R_k P^T||_F <= tol ||D||_F.  r = k; dense iff
// 2 r > min(m, n); otherwise U = Q_r (Q applied to [I_r; 0]) and
// V = ||D||_F (R_r P^T)^T, the pivoted rows of R.
template <typename PT>
CLR_INLINE void dense_rrqr(const RecItem& it, PT* G, double tol, double normc, RecShared& sh) {
  const int m = it.m, n = it.n, q = m < n ? m : n;
  const double inv_norm = 1.0 / normc;
  const cgdbl* D = (const cgdbl*)it.D;
  for (int64_t e = opaque_tid(); e < (int64_t)m * n; e += kRecThreads) {
    const int i = (int)(e % m), j = (int)(e / m);
    G[i + (int64_t)j * m] = D[i + (int64_t)j * it.ldd] * inv_norm;
  }
  __syncthreads();
  const int r = pivoted_qr(G, m, n, m, sh, tol * tol, true);
  if (r == 0) {
    write_meta(it, 0, 0, 0.0);
    return;
  }
  if (2 * r > q) {
    copy_dense_out(it);
    write_meta(it, 1, q, normc);
    return;
  }
  gdbl* Uo = (gdbl*)it.out;
  gdbl* Vo = Uo + (int64_t)m * r;
  for (int64_t e = opaque_tid(); e < (int64_t)m * r; e += kRecThreads) {
    const int i = (int)(e % m), c = (int)(e / m);
    Uo[e] = i == c ? 1.0 : 0.0;
  }
  __syncthreads();
  apply_q(G, m, r, sh.sigma, Uo, m, r);
  double part = 0.0;
  for (int64_t e = opaque_tid(); e < (int64_t)n * r; e += kRecThreads) {
    const int j = (int)(e % n), i = (int)(e / n);
    const double v = j >= i ? G[i + (int64_t)j * m] : 0.0;
    part += v * v;
    Vo[sh.perm[j] + (int64_t)i * n] = normc * v;
  }
  const double kept = block_sum(part, sh);
  write_meta(it, 2, r, normc * sqrt(kept));
}

// certified: the dense certificate proved the kept rank above q / 2, so the
// block is copied out without the SVD (the SVD would reach the same result).
template <bool REG>
CLR_INLINE void dense_path(const RecItem& it, double tol, double* lds, int* status,
                           RecShared& sh, bool certified, GemmItem* gout = nullptr,
                           Seg* gseg = nullptr, int gidx = 0, double* flops_bidiag = nullptr) {
  const int m = it.m, n = it.n;
  const cgdbl* D = (const cgdbl*)it.D;
  double part = 0.0;
  for (int64_t e = opaque_tid(); e < (int64_t)m * n; e += kRecThreads) {
    const double v = D[(e % m) + (e / m) * it.ldd];
    part += v * v;
  }
  const double normc = sqrt(block_sum(part, sh));
  if (!(normc == normc) || normc > DBL_MAX) {
    if (opaque_tid() == 0) atomicOr(status, 2);
  }
  if (normc < it.tau || (normc == 0.0 && it.tau == 0.0)) {
    write_meta(it, 0, 0, 0.0);
    return;
  }
  const int q = m < n ? m : n;
  if (it.path == kPathForceDense || tol == 0.0 || certified) {
    copy_dense_out(it);
    write_meta(it, 1, q, normc);
    return;
  }
  // working matrix G = D / ||D|| (m >= n) or D^T / ||D|| (m < n): p x q, p >= q
  const bool trans = m < n;
  const int p = trans ? n : m;
  if constexpr (REG) {
    RegLds& L = *reinterpret_cast<RegLds*>(lds);
    RegTile a;
    reg_load(a, it.D, it.ldd, trans, 1.0 / normc, p, q);
    reg_bidiag(a, p, q, L);
    if (flops_bidiag && opaque_tid() == 0)
      atomicAdd(flops_bidiag, 4.0 * p * (double)q * q - 4.0 * (double)q * q * q / 3.0);
    const int r = reg_decide(q, tol, L, sh);
    if (r == 0) {
      write_meta(it, 0, 0, 0.0);
      return;
    }
    if (2 * r > q) {
      copy_dense_out(it);
      write_meta(it, 1, q, normc);
      return;
    }
    // truncated: singular vectors from the bidiagonal, else pivoted QR + Jacobi on R^T
    if (reg_vectors(it, p, q, trans, r, normc, L, sh, gout, gseg, gidx)) return;
    reg_load(a, it.D, it.ldd, trans, 1.0 / normc, p, q);
    const int kc = reg_pivoted_qr(a, p, q, L, sh);
    // odd leading dimension: the columns of one wave start in different LDS banks
    const int64_t ldx = q + 1 - (q & 1);
    if (ldx * kc * 8 <= (int64_t)kRecLdsBytes) {
      reg_truncated(it, a, (ldbl*)lds, ldx, p, q, kc, trans, r, tol, normc, status, sh);
    } else if (it.scratch != nullptr) {
      reg_truncated(it, a, (gdbl*)it.scratch, ldx, p, q, kc, trans, r, tol, normc, status, sh);
    } else if (opaque_tid() == 0) {
      atomicOr(status, 4);   // cannot happen with the planner's scratch rule
    }
  } else if (it.rrqr) {
    if (it.scratch != nullptr)
      dense_rrqr(it, (gdbl*)it.scratch, tol, normc, sh);
    else
      dense_rrqr(it, (ldbl*)lds, tol, normc, sh);
  } else {
    if (it.scratch != nullptr)
      dense_general(it, (gdbl*)it.scratch, p, q, trans, tol, normc, status, sh);
    else
      dense_general(it, (ldbl*)lds, p, q, trans, tol, normc, status, sh);
  }
}

template <typename PT>
CLR_INLINE void lowrank_body(const RecItem& it, const Piece* __restrict__ pieces, double tol,
                             PT* W, int* status, RecShared& sh) {
  const int m = it.m, n = it.n, R = it.R;
  PT* Uc = W;
  PT* Vc = Uc + (int64_t)m * R;
  PT* G = Vc + (int64_t)n * R;     // working copy of M^T / ||M||
  PT* Mc = G + (int64_t)R * R;     // M itself
  PT* tauU = Mc + (int64_t)R * R;
  PT* tauV = tauU + R;
  gdbl* out = (gdbl*)it.out;
  // gather the concatenation (Eq. (5)); the scale rides on U
  int off = 0;
  for (int pc = 0; pc < it.npieces; ++pc) {
    const Piece pz = pieces[it.piece0 + pc];
    const cgdbl* pu = (const cgdbl*)pz.U;
    const cgdbl* pv = (const cgdbl*)pz.V;
    for (int64_t e = opaque_tid(); e < (int64_t)m * pz.r; e += kRecThreads) {
      const int i = (int)(e % m), c = (int)(e / m);
      Uc[i + (int64_t)(off + c) * m] = pz.scale * pu[i + (int64_t)c * pz.ldu];
    }
    for (int64_t e = opaque_tid(); e < (int64_t)n * pz.r; e += kRecThreads) {
      const int i = (int)(e % n), c = (int)(e / n);
      Vc[i + (int64_t)(off + c) * n] = pv[i + (int64_t)c * pz.ldv];
    }
    off += pz.r;
  }
  __syncthreads();
  if (tol == 0.0) {
    // no truncation: the concatenation itself is the result; keep a copy in the
    // output slot before the QR below overwrites the working factors
    for (int64_t e = opaque_tid(); e < (int64_t)(m + n) * R; e += kRecThreads) out[e] = W[e];
    __syncthreads();
  }
  householder_qr(Uc, m, R, tauU);
  householder_qr(Vc, n, R, tauV);
  // core M = R_U R_V^T (Eq. (6)), both factors upper triangular;
  // ||U V^T||_F = ||M||_F keeps its accuracy when the concatenated terms cancel
  double part = 0.0;
  for (int e = opaque_tid(); e < R * R; e += kRecThreads) {
    const int i = e % R, j = e / R;
    double s = 0.0;
    for (int k = (i > j ? i : j); k < R; ++k) s += Uc[i + (int64_t)k * m] * Vc[j + (int64_t)k * n];
    Mc[e] = s;
    part += s * s;
  }
  const double normc = sqrt(block_sum(part, sh));
  if (!(normc == normc) || normc > DBL_MAX) {
    if (opaque_tid() == 0) atomicOr(status, 2);
  }
  if (normc < it.tau || (normc == 0.0 && it.tau == 0.0)) {
    write_meta(it, 0, 0, 0.0);
    return;
  }
  if (tol == 0.0) {
    write_meta(it, 2, R, normc);
    return;
  }
  const double inv_norm = 1.0 / normc;
  for (int e = opaque_tid(); e < R * R; e += kRecThreads) {
    const int i = e % R, j = e / R;
    G[j + (int64_t)i * R] = Mc[e] * inv_norm;   // G = M^T / ||M||
  }
  __syncthreads();
  const int r = svd_rank(G, R, R, R, tol, status, sh);
  if (r == 0) {
    write_meta(it, 0, 0, 0.0);
    return;
  }
  double kept = 0.0;
  for (int c = 0; c < r; ++c) {
    const double s = sh.sigma[sh.order[c]];
    kept += s * s;
  }
  kept *= normc * normc;
  gdbl* Uo = out;
  gdbl* Vo = out + (int64_t)m * r;
  // left singular vectors of M (right ones of M^T) into the top of U'
  for (int64_t e = opaque_tid(); e < (int64_t)m * r; e += kRecThreads) Uo[e] = 0.0;
  __syncthreads();
  write_basis(G, R, R, r, Uo, m, sh);
  // V' top rows = M^T u_M (= V_M Sigma)
  for (int64_t e = opaque_tid(); e < (int64_t)n * r; e += kRecThreads) {
    const int i = (int)(e % n), c = (int)(e / n);
    double s = 0.0;
    if (i < R)
      for (int a = 0; a < R; ++a) s += Mc[a + (int64_t)i * R] * Uo[a + (int64_t)c * m];
    Vo[e] = s;
  }
  __syncthreads();
  apply_q(Uc, m, R, tauU, Uo, m, r);
  apply_q(Vc, n, R, tauV, Vo, n, r);
  write_meta(it, 2, r, sqrt(kept));
}

CLR_INLINE void lowrank_path(const RecItem& it, const Piece* __restrict__ pieces, double tol,
                             double* lds, int* status, RecShared& sh) {
  if (it.scratch != nullptr)
    lowrank_body(it, pieces, tol, (gdbl*)it.scratch, status, sh);
  else
    lowrank_body(it, pieces, tol, (ldbl*)lds, status, sh);
}

// Dense-path blocks whose edges are both <= 160 (and tol > 0) go to the
// register-resident kernel; everything else to the general one.
__device__ inline bool register_item(const RecItem& it, double tol) {
  return it.path == kPathDense && !it.rrqr && tol != 0.0 && it.m <= kRegEdge && it.n <= kRegEdge;
}

__device__ inline bool item_guard(const RecItem& it, double tol, int* status) {
  // the planner gives scratch to every block whose working set exceeds the LDS budget
  if (it.scratch == nullptr && rec_scratch_doubles(it.path, it.m, it.n, it.R, tol) > 0) {
    if (opaque_tid() == 0) atomicOr(status, 4);
    return false;
  }
  if (it.m > kMaxDim || it.n > kMaxDim) {
    if (opaque_tid() == 0) atomicOr(status, 8);
    return false;
  }
  return true;
}

__global__ __launch_bounds__(kRecThreads) void k_recompress(const RecItem* __restrict__ items,
                                                            const Piece* __restrict__ pieces,
                                                            int nitems, double tol, int* status,
                                                            const int* __restrict__ cert,
                                                            const int64_t* __restrict__ live) {
  extern __shared__ double lds[];
  __shared__ RecShared sh;
  if (live) nitems = (int)min((int64_t)nitems, *live);
  const int item = xcd_unit(nitems, live != nullptr);
  if (item < 0 || item >= nitems) return;
  const RecItem it = items[item];
  if (it.path == kPathSkip || register_item(it, tol)) return;
  if (!item_guard(it, tol, status)) return;
  if (it.path == kPathLowRank)
    lowrank_path(it, pieces, tol, lds, status, sh);
  else
    dense_path<false>(it, tol, lds, status, sh, cert != nullptr && cert[item] != 0);
}

// Longest-first launch order of the register engine's blocks (one workgroup
// per block, so a long block started last sets the end of the launch).  The
// bidiagonalisation dominates and costs about q steps of a fixed overhead
// plus the trailing-matrix work, so the class is 4 log2(q (q + p + 64));
// blocks off the register path exit at once and, with the blocks proved dense
// (a copy), go last.  Histogram, scan
// from the most expensive class down, scatter (the order inside a class does
// not change any result).
constexpr int kRecOrderClasses = 64;

__device__ inline int rec_cost_class(const RecItem& it, double tol, bool certified) {
  if (!register_item(it, tol) || certified) return 0;
  const int q = min(it.m, it.n), p = max(it.m, it.n);
  const double cost = (double)q * (double)(q + p + 64);
  return min(kRecOrderClasses - 1, max(1, (int)(4.0 * log2(cost)) - 40));
}

__global__ __launch_bounds__(1024) void k_rec_order(const RecItem* __restrict__ items, int n,
                                                    double tol, const int* __restrict__ cert,
                                                    int* __restrict__ order,
                                                    const int64_t* __restrict__ live) {
  __shared__ int cnt[kRecOrderClasses];
  const int tid = threadIdx.x;
  if (live) n = (int)min((int64_t)n, *live);
  if (tid < kRecOrderClasses) cnt[tid] = 0;
  __syncthreads();
  for (int i = tid; i < n; i += 1024)
    atomicAdd(&cnt[rec_cost_class(items[i], tol, cert != nullptr && cert[i] != 0)], 1);
  __syncthreads();
  if (tid == 0) {
    int run = 0;
    for (int c = kRecOrderClasses - 1; c >= 0; --c) {
      const int k = cnt[c];
      cnt[c] = run;
      run += k;
    }
  }
  __syncthreads();
  for (int i = tid; i < n; i += 1024)
    order[atomicAdd(&cnt[rec_cost_class(items[i], tol, cert != nullptr && cert[i] != 0)], 1)] = i;
}

// With `next` (a counter, zero at launch) the launch is persistent: one
// workgroup per CU takes the slots of the longest-first order from it, so a
// long block goes to whichever CU frees first.
__global__ __launch_bounds__(kRecThreads) void k_recompress_reg(const RecItem* __restrict__ items,
                                                                int nitems, double tol,
                                                                int* status, GemmItem* gout,
                                                                Seg* gseg,
                                                                const int* __restrict__ order,
                                                                const int* __restrict__ cert,
                                                                double* flops_bidiag,
                                                                const int64_t* __restrict__ live,
                                                                int* __restrict__ next) {
  extern __shared__ double lds[];
  __shared__ RecShared sh;
  __shared__ int slot_sh;
  if (live) nitems = (int)min((int64_t)nitems, *live);
  auto run = [&](int item) {
    const RecItem it = items[item];
    if (!register_item(it, tol)) return;
    if (!item_guard(it, tol, status)) return;
    dense_path<true>(it, tol, lds, status, sh, cert != nullptr && cert[item] != 0, gout, gseg, item,
                     flops_bidiag);
  };
  // one call site of the block body (it is inlined): persistent slots, or the
  // workgroup's own block once
  for (bool first = true;; first = false) {
    int item;
    if (next) {
      if (!first) __syncthreads();   // LDS and slot_sh free for the next block
      if (threadIdx.x == 0) slot_sh = atomicAdd(next, 1);
      __syncthreads();
      const int slot = __builtin_amdgcn_readfirstlane(slot_sh);
      if (slot >= nitems) return;   // the same value in every thread
      item = order[slot];
    } else {
      if (!first) return;
      if (order) {
        if ((int)blockIdx.x >= nitems) return;
        item = order[blockIdx.x];
      } else {
        item = xcd_unit(nitems, live != nullptr);
        if (item < 0 || item >= nitems) return;
      }
    }
    run(item);
  }
}

// Dynamic-LDS limits of the recompression kernels; done once, before any
// launch (and before any stream capture that records one).
hipError_t prepare_recompress() {
  static bool attr_set = false;
  if (attr_set) return hipSuccess;
  hipError_t e = hipFuncSetAttribute((const void*)k_recompress,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, kRecLdsBytes);
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)k_recompress_reg,
                            hipFuncAttributeMaxDynamicSharedMemorySize, kRecLdsBytes);
  if (e == hipSuccess) attr_set = true;
  return e;
}

hipError_t launch_recompress(const RecItem* items, const Piece* pieces, int nitems, double tol,
                             int* status, GemmItem* gout, Seg* gseg, int* order, int* cert,
                             RecCounters* ctr, hipStream_t s, hipEvent_t engine_begin,
                             hipEvent_t engine_end, const int64_t* live) {
  if (nitems <= 0) return hipSuccess;
  {
    hipError_t e = prepare_recompress();
    if (e != hipSuccess) return e;
  }
  const int grid = ((nitems + 7) / 8) * 8;
  // every item's output-product slot starts empty (m = 0: nothing to compute)
  static_assert(sizeof(GemmItem) % sizeof(int) == 0, "GemmItem is filled as int words");
  hipError_t e = launch_fill_i32(reinterpret_cast<int*>(gout), 0,
                                 (int64_t)nitems * (int64_t)(sizeof(GemmItem) / sizeof(int)), s);
  if (e != hipSuccess) return e;
  if (ctr) {
    static_assert(sizeof(RecCounters) % sizeof(double) == 0, "counters are cleared as doubles");
    e = launch_fill_f64(reinterpret_cast<double*>(ctr), 0.0,
                        (int64_t)(sizeof(RecCounters) / sizeof(double)), s);
    if (e != hipSuccess) return e;
  }
  if (cert && tol > 0.0) {
    e = launch_dense_cert(items, nitems, tol, cert, ctr ? &ctr->certified : nullptr, s, live);
    if (e != hipSuccess) return e;
  } else {
    cert = nullptr;
  }
  if (order) {
    hipLaunchKernelGGL(k_rec_order, dim3(1), dim3(1024), 0, s, items, nitems, tol, cert, order,
                       live);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (engine_begin) {
    e = hipEventRecord(engine_begin, s);
    if (e != hipSuccess) return e;
  }
  // with an order, persistent: one workgroup per CU over the list (counter after it)
  int* next = order ? order + nitems : nullptr;
  if (next) {
    e = launch_fill_i32(next, 0, 1, s);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_recompress_reg, dim3(next ? persistent_grid(nitems) : grid), dim3(kRecThreads),
                     kRecLdsBytes, s, items, nitems, tol, status, gout, gseg, order, cert,
                     ctr ? &ctr->flops_bidiag : nullptr, live, next);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (engine_end) {
    e = hipEventRecord(engine_end, s);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_recompress, dim3(grid), dim3(kRecThreads), kRecLdsBytes, s, items, pieces,
                     nitems, tol, status, cert, live);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  // other factors of the truncated register-engine blocks: G_orig * basis on FP64 MFMA
  return launch_ggemm_f64(gout, gseg, nitems, s);
}

}  // namespace clr
