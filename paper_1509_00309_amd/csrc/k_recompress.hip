// Recompression of accumulated result blocks, FP64 (Sec. 4.1, Eqs. (5)-(7)).
//
// One workgroup per result block.  Two paths:
//  * dense path: the block was accumulated densely (m x n).  Its Frobenius
//    norm decides the drop; otherwise its singular values decide the kept
//    rank r (smallest r whose discarded tail sqrt(sum_{i>=r} s_i^2) is
//    <= tol * ||C||_F).  If 2r > min(m, n) the block stays dense and
//    untruncated; else it is stored as U (orthonormal) and V = D^T U, or the
//    mirror image when m < n.  Singular values come from one-sided Jacobi
//    (Hestenes) rotations on the columns of D or D^T, held in LDS when they
//    fit, otherwise in a global scratch area.
//  * low-rank path: the block is the concatenation U_cat V_cat^T of R
//    columns (Eq. (5)).  Householder QR of both factors, core
//    M = R_U R_V^T, one-sided Jacobi on M, rank rule, then
//    U' = Q_U [u_M] and V' = Q_V [M^T u_M]  (= Q_V V_M Sigma, Eq. (7)).
//
// Lanes are organised in groups of 16; a group owns one column (pair) at a
// time and reduces with xor-shuffles inside the group.
#include <float.h>

#include "clr_internal.h"

namespace clr {

constexpr int kMaxDim = 512;  // largest block edge handled by the recompression kernel
constexpr double kNegligible2 = 1e-40;  // squared column norm, relative to the block's

struct RecShared {
  double sigma[kMaxDim];
  double tails[kMaxDim + 1];
  int order[kMaxDim];
  double red[kRecThreads];
  int flag;
  int rank;
  double normc;
};

__device__ inline double group_sum16(double v) {
  v += __shfl_xor(v, 8, 16);
  v += __shfl_xor(v, 4, 16);
  v += __shfl_xor(v, 2, 16);
  v += __shfl_xor(v, 1, 16);
  return v;
}

__device__ inline double wave_sum(double v) {
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Deterministic workgroup sum: per-thread partials, tree over LDS.
__device__ double block_sum(double v, RecShared& sh) {
  const int tid = threadIdx.x;
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

// One-sided Jacobi on the q columns (length p, leading dimension ldw) of W.
// W is scaled to unit Frobenius norm by the callers; columns whose squared
// norm is below kNegligible2 (1e-20 of the block norm) are left alone: they
// lie far below any truncation threshold and rotating them only chases
// rounding noise (in the subnormal range for strongly decaying kernels).
// Returns false if it did not converge within kJacobiMaxSweeps sweeps.
__device__ bool jacobi_columns(double* W, int p, int q, int64_t ldw, RecShared& sh) {
  const int tid = threadIdx.x;
  const int g = tid >> 4, gl = tid & 15;
  constexpr int ngroups = kRecThreads / 16;
  const int P = q + (q & 1);
  const double tolj = (double)p * DBL_EPSILON;
  bool converged = false;
  for (int sweep = 0; sweep < kJacobiMaxSweeps; ++sweep) {
    if (tid == 0) sh.flag = 0;
    __syncthreads();
    for (int round = 0; round < P - 1; ++round) {
      for (int k = g; k < P / 2; k += ngroups) {
        int a, b;
        tournament(round, k, P, a, b);
        if (a >= q || b >= q) continue;
        double* wa = W + (int64_t)a * ldw;
        double* wb = W + (int64_t)b * ldw;
        double al = 0.0, be = 0.0, ga = 0.0;
        for (int i = gl; i < p; i += 16) {
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
          for (int i = gl; i < p; i += 16) {
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
    if (!rotated) {
      converged = true;
      break;
    }
  }
  return converged;
}

// Column norms, descending order (ties by index) and the kept rank for `tol`.
__device__ int rank_from_columns(const double* W, int p, int q, int64_t ldw, double tol,
                                 double normc, RecShared& sh) {
  const int tid = threadIdx.x;
  const int g = tid >> 4, gl = tid & 15;
  for (int j = g; j < q; j += kRecThreads / 16) {
    const double* w = W + (int64_t)j * ldw;
    double s = 0.0;
    for (int i = gl; i < p; i += 16) s += w[i] * w[i];
    s = group_sum16(s);
    if (gl == 0) sh.sigma[j] = sqrt(s);
  }
  __syncthreads();
  for (int j = tid; j < q; j += kRecThreads) {
    const double sj = sh.sigma[j];
    int pos = 0;
    for (int i = 0; i < q; ++i) {
      const double si = sh.sigma[i];
      pos += (si > sj) || (si == sj && i < j);
    }
    sh.order[pos] = j;
  }
  __syncthreads();
  if (tid == 0) {
    double acc = 0.0;
    sh.tails[q] = 0.0;
    for (int i = q - 1; i >= 0; --i) {
      const double s = sh.sigma[sh.order[i]];
      acc += s * s;
      sh.tails[i] = acc;
    }
    const double bound = tol * normc;
    int r = q;
    for (int i = 0; i <= q; ++i)
      if (sqrt(sh.tails[i]) <= bound) {
        r = i;
        break;
      }
    sh.rank = r;
  }
  __syncthreads();
  return sh.rank;
}

__device__ void write_meta(const RecItem& it, int kind, int rank, double norm) {
  if (threadIdx.x == 0) {
    *it.kind_out = kind;
    *it.rank_out = rank;
    *it.norm_out = norm;
  }
}

__device__ void copy_dense_out(const RecItem& it) {
  const int64_t total = (int64_t)it.m * it.n;
  for (int64_t e = threadIdx.x; e < total; e += kRecThreads) {
    const int i = (int)(e % it.m), j = (int)(e / it.m);
    it.out[e] = it.D[i + (int64_t)j * it.ldd];
  }
}

// Householder QR of W (rows x cols, ld rows) in place: R in the upper
// triangle, reflector tails below the diagonal, tau[k] alongside
// (H_k = I - tau_k v_k v_k^T, v_k = (1, W[k+1:, k])).
__device__ void householder_qr(double* W, int rows, int cols, double* tau, RecShared& sh) {
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int g = tid >> 4, gl = tid & 15;
  for (int k = 0; k < cols && k < rows; ++k) {
    double* col = W + (int64_t)k * rows;
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
      for (int j = k + 1 + g; j < cols; j += kRecThreads / 16) {
        double* cj = W + (int64_t)j * rows;
        double w = 0.0;
        for (int i = k + gl; i < rows; i += 16) w += (i == k ? 1.0 : col[i]) * cj[i];
        w = group_sum16(w);
        for (int i = k + gl; i < rows; i += 16) cj[i] -= t * (i == k ? 1.0 : col[i]) * w;
      }
    }
    __syncthreads();
  }
  (void)sh;
}

// X (rows x ncol, ld ldx, global) <- Q X with Q = H_0 H_1 ... H_{kk-1} from householder_qr.
__device__ void apply_q(const double* W, int rows, int kk, const double* tau, double* X,
                        int64_t ldx, int ncol) {
  const int tid = threadIdx.x;
  const int g = tid >> 4, gl = tid & 15;
  for (int c = g; c < ncol; c += kRecThreads / 16) {
    double* x = X + (int64_t)c * ldx;
    for (int k = kk - 1; k >= 0; --k) {
      const double t = tau[k];
      if (t == 0.0) continue;
      const double* v = W + (int64_t)k * rows;
      double w = 0.0;
      for (int i = k + gl; i < rows; i += 16) w += (i == k ? 1.0 : v[i]) * x[i];
      w = group_sum16(w);
      for (int i = k + gl; i < rows; i += 16) x[i] -= t * (i == k ? 1.0 : v[i]) * w;
    }
  }
  __syncthreads();
}

__device__ void dense_path(const RecItem& it, double tol, double* lds, int* status,
                           RecShared& sh) {
  const int m = it.m, n = it.n;
  double part = 0.0;
  for (int64_t e = threadIdx.x; e < (int64_t)m * n; e += kRecThreads) {
    const double v = it.D[(e % m) + (e / m) * it.ldd];
    part += v * v;
  }
  const double normc = sqrt(block_sum(part, sh));
  if (!(normc == normc) || normc > DBL_MAX) {
    if (threadIdx.x == 0) atomicOr(status, 2);
  }
  if (normc < it.tau || (normc == 0.0 && it.tau == 0.0)) {
    write_meta(it, 0, 0, 0.0);
    return;
  }
  const int q = m < n ? m : n;
  if (it.path == kPathForceDense || tol == 0.0) {
    copy_dense_out(it);
    write_meta(it, 1, q, normc);
    return;
  }
  const bool trans = m < n;
  const int p = trans ? n : m;
  double* W = it.scratch != nullptr ? it.scratch : lds;
  const double inv_norm = 1.0 / normc;
  for (int64_t e = threadIdx.x; e < (int64_t)m * n; e += kRecThreads) {
    const int i = (int)(e % m), j = (int)(e / m);
    const double v = it.D[i + (int64_t)j * it.ldd] * inv_norm;
    if (!trans)
      W[i + (int64_t)j * p] = v;
    else
      W[j + (int64_t)i * p] = v;
  }
  __syncthreads();
  if (!jacobi_columns(W, p, q, p, sh)) {
    if (threadIdx.x == 0) atomicOr(status, 1);
  }
  const int r = rank_from_columns(W, p, q, p, tol, 1.0, sh);
  if (r == 0) {
    write_meta(it, 0, 0, 0.0);
    return;
  }
  if (2 * r > q) {
    copy_dense_out(it);
    write_meta(it, 1, q, normc);
    return;
  }
  double kept = 0.0;
  for (int k = 0; k < r; ++k) {
    const double s = sh.sigma[sh.order[k]];
    kept += s * s;
  }
  kept *= normc * normc;
  // basis side: the orthonormal factor from the Jacobi columns
  double* basis = trans ? it.out + (int64_t)m * r : it.out;  // V' (n x r) or U' (m x r)
  double* other = trans ? it.out : it.out + (int64_t)m * r;  // U' (m x r) or V' (n x r)
  const int bl = p;                 // rows of the basis factor
  const int ol = trans ? m : n;     // rows of the other factor
  for (int64_t e = threadIdx.x; e < (int64_t)bl * r; e += kRecThreads) {
    const int i = (int)(e % bl), k = (int)(e / bl);
    const int j = sh.order[k];
    basis[e] = W[i + (int64_t)j * p] / sh.sigma[j];
  }
  // other = D^T basis (no transpose) or D basis (transpose): dot over the p-long side
  const int g = threadIdx.x >> 4, gl = threadIdx.x & 15;
  for (int o = g; o < ol * r; o += kRecThreads / 16) {
    const int j = o % ol, k = o / ol;
    const int src = sh.order[k];
    const double inv = 1.0 / sh.sigma[src];
    double s = 0.0;
    if (!trans) {
      const double* dcol = it.D + (int64_t)j * it.ldd;   // column j of D (m long)
      for (int i = gl; i < m; i += 16) s += dcol[i] * W[i + (int64_t)src * p];
    } else {
      for (int i = gl; i < n; i += 16) s += it.D[j + (int64_t)i * it.ldd] * W[i + (int64_t)src * p];
    }
    s = group_sum16(s) * inv;
    if (gl == 0) other[j + (int64_t)k * ol] = s;
  }
  write_meta(it, 2, r, sqrt(kept));
}

__device__ void lowrank_path(const RecItem& it, const Piece* __restrict__ pieces, double tol,
                             double* lds, int* status, RecShared& sh) {
  const int m = it.m, n = it.n, R = it.R;
  double* W = it.scratch != nullptr ? it.scratch : lds;
  double* Uc = W;
  double* Vc = Uc + (int64_t)m * R;
  double* M = Vc + (int64_t)n * R;
  double* Mc = M + (int64_t)R * R;
  double* tauU = Mc + (int64_t)R * R;
  double* tauV = tauU + R;
  // gather the concatenation (Eq. (5)); the scale rides on U
  int off = 0;
  for (int pc = 0; pc < it.npieces; ++pc) {
    const Piece pz = pieces[it.piece0 + pc];
    for (int64_t e = threadIdx.x; e < (int64_t)m * pz.r; e += kRecThreads) {
      const int i = (int)(e % m), c = (int)(e / m);
      Uc[i + (int64_t)(off + c) * m] = pz.scale * pz.U[i + (int64_t)c * pz.ldu];
    }
    for (int64_t e = threadIdx.x; e < (int64_t)n * pz.r; e += kRecThreads) {
      const int i = (int)(e % n), c = (int)(e / n);
      Vc[i + (int64_t)(off + c) * n] = pz.V[i + (int64_t)c * pz.ldv];
    }
    off += pz.r;
  }
  __syncthreads();
  if (tol == 0.0) {
    // no truncation: the concatenation itself is the result; keep a copy in the
    // output slot before the QR below overwrites the working factors
    for (int64_t e = threadIdx.x; e < (int64_t)(m + n) * R; e += kRecThreads) it.out[e] = W[e];
    __syncthreads();
  }
  householder_qr(Uc, m, R, tauU, sh);
  householder_qr(Vc, n, R, tauV, sh);
  // core M = R_U R_V^T (Eq. (6)), both factors upper triangular
  double part = 0.0;
  for (int e = threadIdx.x; e < R * R; e += kRecThreads) {
    const int i = e % R, j = e / R;
    double s = 0.0;
    for (int k = (i > j ? i : j); k < R; ++k) s += Uc[i + (int64_t)k * m] * Vc[j + (int64_t)k * n];
    M[e] = s;
    Mc[e] = s;
    part += s * s;
  }
  // ||U V^T||_F = ||R_U R_V^T||_F: the QR route keeps its accuracy when the
  // concatenated terms cancel (a Gram-matrix formula would not)
  const double normc = sqrt(block_sum(part, sh));
  if (!(normc == normc) || normc > DBL_MAX) {
    if (threadIdx.x == 0) atomicOr(status, 2);
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
  for (int e = threadIdx.x; e < R * R; e += kRecThreads) M[e] *= inv_norm;
  __syncthreads();
  if (!jacobi_columns(M, R, R, R, sh)) {
    if (threadIdx.x == 0) atomicOr(status, 1);
  }
  const int r = rank_from_columns(M, R, R, R, tol, 1.0, sh);
  if (r == 0) {
    write_meta(it, 0, 0, 0.0);
    return;
  }
  double kept = 0.0;
  for (int k = 0; k < r; ++k) {
    const double s = sh.sigma[sh.order[k]];
    kept += s * s;
  }
  kept *= normc * normc;
  double* Uo = it.out;
  double* Vo = it.out + (int64_t)m * r;
  // U' = Q_U [u_M ; 0]
  for (int64_t e = threadIdx.x; e < (int64_t)m * r; e += kRecThreads) {
    const int i = (int)(e % m), k = (int)(e / m);
    const int j = sh.order[k];
    Uo[e] = i < R ? M[i + (int64_t)j * R] / sh.sigma[j] : 0.0;
  }
  // V' = Q_V [M^T u_M ; 0]   (M^T u_M = V_M Sigma)
  for (int64_t e = threadIdx.x; e < (int64_t)n * r; e += kRecThreads) {
    const int i = (int)(e % n), k = (int)(e / n);
    double s = 0.0;
    if (i < R) {
      const int j = sh.order[k];
      for (int a = 0; a < R; ++a) s += Mc[a + (int64_t)i * R] * M[a + (int64_t)j * R];
      s /= sh.sigma[j];
    }
    Vo[e] = s;
  }
  __syncthreads();
  apply_q(Uc, m, R, tauU, Uo, m, r);
  apply_q(Vc, n, R, tauV, Vo, n, r);
  write_meta(it, 2, r, sqrt(kept));
}

__global__ __launch_bounds__(kRecThreads) void k_recompress(const RecItem* __restrict__ items,
                                                            const Piece* __restrict__ pieces,
                                                            int nitems, double tol, int* status) {
  extern __shared__ double lds[];
  __shared__ RecShared sh;
  const int per = gridDim.x / 8;
  const int item = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
  if (item >= nitems) return;
  const RecItem it = items[item];
  if (it.path == kPathSkip) return;
  // the planner gives scratch to every block whose working set exceeds the LDS budget
  if (it.scratch == nullptr && rec_scratch_doubles(it.path, it.m, it.n, it.R, tol) > 0) {
    if (threadIdx.x == 0) atomicOr(status, 4);
    return;
  }
  if (it.m > kMaxDim || it.n > kMaxDim) {
    if (threadIdx.x == 0) atomicOr(status, 8);
    return;
  }
  if (it.path == kPathLowRank)
    lowrank_path(it, pieces, tol, lds, status, sh);
  else
    dense_path(it, tol, lds, status, sh);
}

hipError_t launch_recompress(const RecItem* items, const Piece* pieces, int nitems, double tol,
                             int* status, hipStream_t s) {
  if (nitems <= 0) return hipSuccess;
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute((const void*)k_recompress,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, kRecLdsBytes);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  const int grid = ((nitems + 7) / 8) * 8;
  hipLaunchKernelGGL(k_recompress, dim3(grid), dim3(kRecThreads), kRecLdsBytes, s, items, pieces,
                     nitems, tol, status);
  return hipGetLastError();
}

}  // namespace clr
