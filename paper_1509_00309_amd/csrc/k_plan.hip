// Symbolic phase of the CLR product C = alpha A B on the device.
//
// k_block_lists: the nonzero blocks of every block row of A and block column
//   of B as lists of inner indices K, ascending (one wave per row or column,
//   compacted with ballots).
// k_symbolic: one wave per candidate result block (I, J).  It walks the
//   shorter of row I's list and column J's list and keeps, in ascending K,
//   the pairs where both A_IK and B_KJ are nonzero (work proportional to the
//   shorter list, not to the number of inner blocks), accumulates the norm
//   estimate
//   est_IJ = |alpha| sum_K ||A_IK||_F ||B_KJ||_F (triangle inequality and
//   submultiplicativity, Sec. 4.1), applies the screening test est >= tau,
//   decides dense or factored accumulation, and counts the work and memory
//   every later phase needs.
// k_scan:     exclusive prefix sums of those counts (a workgroup per array).
// k_reduce:   deterministic totals of the per-block statistics (one per array).
// k_fill:     writes the work lists at the scanned offsets: thin factor
//   products (Eq. (4)), terms of the dense accumulation GEMM, low-rank pieces
//   of factored blocks (Eq. (5)) and one recompression item per block.
#include "clr_internal.h"

namespace clr {

__device__ inline int64_t parts2(int rows, int cols, int maxe) {
  return (int64_t)num_parts(rows, maxe) * num_parts(cols, maxe);
}
// items of a thin (factor-product) output and of a dense-accumulated block
__device__ inline int64_t thin_parts(const EdgeTable& E, int rows, int cols) {
  return parts2(rows, cols, thin_edge(E, rows, cols));
}
__device__ inline int64_t dense_parts(const EdgeTable& E, int m, int n) {
  return parts2(m, n, dense_edge(E, m, n));
}

// Wave w < nrb lists row w of A, wave nrb + J column J of B, into the
// buffer `base` that bind_block_lists laid out (counts of the rows, counts of
// the columns, then the row lists and the column lists, nkb ints each).
__global__ __launch_bounds__(256) void k_block_lists(PlanParams P, int* __restrict__ base) {
  const int wave = (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
  const int lane = threadIdx.x & 63;
  if (wave >= P.nrb + P.ncb) return;
  const bool row = wave < P.nrb;
  const int r = row ? wave : wave - P.nrb;
  int* const a_cnt = base;
  int* const b_cnt = a_cnt + P.nrb;
  int* const a_idx = b_cnt + P.ncb;
  int* const b_idx = a_idx + (int64_t)P.nrb * P.nkb;
  int* out = (row ? a_idx : b_idx) + (int64_t)r * P.nkb;
  int n = 0;
  for (int k0 = 0; k0 < P.nkb; k0 += 64) {
    const int K = k0 + lane;
    bool nz = false;
    if (K < P.nkb) nz = (row ? P.A.kind[(int64_t)r * P.nkb + K] : P.B.kind[(int64_t)K * P.ncb + r]) != 0;
    const unsigned long long m = __ballot(nz);
    if (nz) out[n + __popcll(m & ((1ull << lane) - 1ull))] = K;
    n += __popcll(m);
  }
  if (lane == 0) (row ? a_cnt : b_cnt)[r] = n;
}

hipError_t launch_block_lists(const PlanParams& P, int* base, hipStream_t s) {
  const int waves = P.nrb + P.ncb;
  if (waves == 0) return hipSuccess;
  hipLaunchKernelGGL(k_block_lists, dim3((waves + 3) / 4), dim3(256), 0, s, P, base);
  return hipGetLastError();
}


// The candidate inner indices of result block (I, J): the shorter of A's
// row-I list and B's column-J list (K ascending); the other side's kind table
// then says whether K is a term.
struct TermList {
  const int* k;
  int n;
};
__device__ inline TermList term_list(const PlanParams& P, int I, int J) {
  const int na = P.a_cnt[I], nb = P.b_cnt[J];
  if (nb < na) return TermList{P.b_idx + (int64_t)J * P.nkb, nb};
  return TermList{P.a_idx + (int64_t)I * P.nkb, na};
}

// Sum over the wave of a per-lane value (exact for the integer-valued
// quantities it is used on: counts and flop counts below 2^53).
template <typename T>
__device__ inline T wave_sum_all(T v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// One wave per candidate result block.  The lanes take the candidate terms of
// 64-entry chunks of the block's term list (a term where both A_IK and B_KJ
// are nonzero); the
// norm estimate is summed in ascending K as a term-by-term walk would (lane
// by lane, a lane without a term adding +0), every other per-block quantity
// is a count or an integer-valued flop count and is summed over the wave.
constexpr int kSymThreads = 256;
__global__ __launch_bounds__(kSymThreads) void k_symbolic(PlanParams P, int64_t* __restrict__ cnt,
                                                          double* __restrict__ st,
                                                          int* __restrict__ flags) {
  const int npairs = P.nrb * P.ncb;
  const int lane = threadIdx.x & 63;
  const int pair = (int)((blockIdx.x * (unsigned)kSymThreads + threadIdx.x) >> 6);
  if (pair >= npairs) return;
  const int I = pair / P.ncb, J = pair % P.ncb;
  const int m = P.A.roff[I + 1] - P.A.roff[I];
  const int n = P.B.coff[J + 1] - P.B.coff[J];
  double est = 0.0, fdd = 0.0, fld = 0.0, fdl = 0.0, fll = 0.0, fden = 0.0;
  int nseg = 0, ndd = 0, nld = 0, ndl = 0, nll = 0;
  int64_t rcat = 0, pool = 0, thin1 = 0, thin2 = 0;
  bool anydd = false;
  // low-rank contributions that a densified block adds with rank r cost 2 m n r
  int64_t lr_rank_sum = 0;
  const TermList tl = term_list(P, I, J);
  for (int c0 = 0; c0 < tl.n; c0 += 64) {
    const int K = c0 + lane < tl.n ? tl.k[c0 + lane] : -1;
    const int ka = K >= 0 ? P.A.kind[I * P.nkb + K] : 0;
    const int kb = K >= 0 ? P.B.kind[K * P.ncb + J] : 0;
    const bool term = ka != 0 && kb != 0;
    double prod = 0.0, ldd = 0.0, lld = 0.0, ldl = 0.0, lll = 0.0;
    int64_t lrc = 0, lpool = 0, lt1 = 0, lt2 = 0;
    if (term) {
      const int k = P.A.coff[K + 1] - P.A.coff[K];
      prod = P.A.norm[I * P.nkb + K] * P.B.norm[K * P.ncb + J];
      if (ka == 1 && kb == 1) {
        ldd = 2.0 * m * (double)k * n;
      } else if (ka == 2 && kb == 1) {
        const int ra = P.A.rank[I * P.nkb + K];
        lrc = ra;
        lpool = (int64_t)n * ra;
        lt1 = thin_parts(P.edges, n, ra);
        lld = 2.0 * ra * (double)k * n;
      } else if (ka == 1 && kb == 2) {
        const int rb = P.B.rank[K * P.ncb + J];
        lrc = rb;
        lpool = (int64_t)m * rb;
        lt1 = thin_parts(P.edges, m, rb);
        ldl = 2.0 * m * (double)k * rb;
      } else {
        const int ra = P.A.rank[I * P.nkb + K];
        const int rb = P.B.rank[K * P.ncb + J];
        lpool = (int64_t)ra * rb;
        lt1 = thin_parts(P.edges, ra, rb);
        if (rb < ra) {
          lrc = rb;
          lpool += (int64_t)m * rb;
          lt2 = thin_parts(P.edges, m, rb);
          lll = 2.0 * k * (double)ra * rb + 2.0 * m * (double)ra * rb;
        } else {
          lrc = ra;
          lpool += (int64_t)n * ra;
          lt2 = thin_parts(P.edges, n, ra);
          lll = 2.0 * k * (double)ra * rb + 2.0 * n * (double)ra * rb;
        }
      }
    }
    // the estimate in K order: the chunk's lanes one after another
    {
      const long long bits = __double_as_longlong(prod);
      const int lo = (int)(bits & 0xffffffffLL), hi = (int)(bits >> 32);
      for (int l = 0; l < 64; ++l) {
        const unsigned blo = (unsigned)__builtin_amdgcn_readlane(lo, l);
        const unsigned bhi = (unsigned)__builtin_amdgcn_readlane(hi, l);
        est += __longlong_as_double((long long)(((unsigned long long)bhi << 32) | blo));
      }
    }
    nseg += wave_sum_all<int>(term ? 1 : 0);
    ndd += wave_sum_all<int>(term && ka == 1 && kb == 1 ? 1 : 0);
    nld += wave_sum_all<int>(term && ka == 2 && kb == 1 ? 1 : 0);
    ndl += wave_sum_all<int>(term && ka == 1 && kb == 2 ? 1 : 0);
    nll += wave_sum_all<int>(term && ka == 2 && kb == 2 ? 1 : 0);
    fdd += wave_sum_all<double>(ldd);
    fld += wave_sum_all<double>(lld);
    fdl += wave_sum_all<double>(ldl);
    fll += wave_sum_all<double>(lll);
    rcat += wave_sum_all<long long>(lrc);
    pool += wave_sum_all<long long>(lpool);
    thin1 += wave_sum_all<long long>(lt1);
    thin2 += wave_sum_all<long long>(lt2);
  }
  anydd = ndd > 0;
  if (lane != 0) return;
  lr_rank_sum = rcat;
  est *= fabs(P.alpha);
  const double tau = P.screen ? P.eps_sp * m * (double)n : P.eps_sp;
  const bool candidate = nseg > 0 && (P.mask_kind == nullptr || P.mask_kind[pair] != 0);
  const bool computed = candidate && est >= tau;
  const bool force = P.square && I == J;
  const int mn = m < n ? m : n;
  const bool densify = force || anydd || 2 * rcat >= mn;
  int64_t c[kNumCounters];
  for (int i = 0; i < kNumCounters; ++i) c[i] = 0;
  if (computed) {
    c[kCntSegDense] = densify ? nseg : 0;
    c[kCntPieces] = densify ? 0 : nseg;
    c[kCntThin1] = thin1;
    c[kCntThin2] = thin2;
    c[kCntPool] = pool;
    const int path = force ? kPathForceDense : (densify ? kPathDense : kPathLowRank);
    c[kCntScratch] = rec_scratch_doubles(path, m, n, (int)rcat, P.tol);
    c[kCntComputed] = 1;
    c[kCntGemmItems] = densify ? dense_parts(P.edges, m, n) : 0;
    // room of the result: dense, or truncated to rank r with 2 r <= min(m, n)
    // ((m + n) r <= m n); a factored block keeps rank <= rcat
    c[kCntOut] = densify ? (int64_t)m * n : (int64_t)(m + n) * rcat;
    c[kCntAcc] = densify ? (int64_t)m * n : 0;
    if (densify) fden = 2.0 * m * (double)n * (double)lr_rank_sum;
  }
  for (int i = 0; i < kNumCounters; ++i) cnt[(int64_t)i * npairs + pair] = c[i];
  const double s[kNumStats] = {est,
                               computed ? fdd : 0.0,
                               computed ? fld : 0.0,
                               computed ? fdl : 0.0,
                               computed ? fll : 0.0,
                               computed ? fden : 0.0,
                               computed ? (double)ndd : 0.0,
                               computed ? (double)nld : 0.0,
                               computed ? (double)ndl : 0.0,
                               computed ? (double)nll : 0.0,
                               candidate ? 1.0 : 0.0};
  for (int i = 0; i < kNumStats; ++i) st[(int64_t)i * npairs + pair] = s[i];
  flags[pair] = (computed ? kFlagComputed : 0) | (densify ? kFlagDensify : 0) |
                (force ? kFlagForce : 0);
}

// Exclusive prefix sums of `narrays` arrays of length n (a workgroup of 1024 per array).
__global__ __launch_bounds__(1024) void k_scan(const int64_t* __restrict__ in,
                                               int64_t* __restrict__ out, int64_t n,
                                               int narrays, int64_t* __restrict__ totals) {
  __shared__ int64_t part[1024];
  const int tid = threadIdx.x;
  const int64_t chunk = (n + 1023) / 1024;
  // workgroup a scans array a (the grid covers the arrays)
  for (int a = blockIdx.x; a < narrays; a += gridDim.x) {
    const int64_t* x = in + (int64_t)a * n;
    int64_t* y = out + (int64_t)a * n;
    const int64_t b0 = tid * chunk;
    const int64_t b1 = b0 + chunk < n ? b0 + chunk : n;
    int64_t s = 0;
    for (int64_t i = b0; i < b1; ++i) s += x[i];
    part[tid] = s;
    __syncthreads();
    // Hillis-Steele inclusive scan over the 1024 partials
    for (int o = 1; o < 1024; o <<= 1) {
      const int64_t v = tid >= o ? part[tid - o] : 0;
      __syncthreads();
      part[tid] += v;
      __syncthreads();
    }
    int64_t run = part[tid] - s;
    for (int64_t i = b0; i < b1; ++i) {
      y[i] = run;
      run += x[i];
    }
    if (tid == 1023) totals[a] = part[1023];
    __syncthreads();
  }
}

// Totals of `narrays` double arrays of length n in a fixed order (a workgroup of 256 per array).
__global__ __launch_bounds__(256) void k_reduce(const double* __restrict__ in, int64_t n,
                                                int narrays, double* __restrict__ totals) {
  __shared__ double part[256];
  const int tid = threadIdx.x;
  // workgroup a sums array a (the grid covers the arrays)
  for (int a = blockIdx.x; a < narrays; a += gridDim.x) {
    double s = 0.0;
    for (int64_t i = tid; i < n; i += 256) s += in[(int64_t)a * n + i];
    part[tid] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if (tid < o) part[tid] += part[tid + o];
      __syncthreads();
    }
    if (tid == 0) totals[a] = part[0];
    __syncthreads();
  }
}

// Emit the sub-items of one thin product job (single term) into a list.
__device__ void emit_thin(Seg* segs, GemmItem* items, int64_t& cursor, const Seg& s, double* C,
                          int64_t ldc, int rows, int cols, const EdgeTable& E) {
  const int max_item = thin_edge(E, rows, cols);
  const int pr = num_parts(rows, max_item), pc = num_parts(cols, max_item);
  for (int a = 0; a < pr; ++a) {
    int r0, rl;
    part_range(rows, pr, a, &r0, &rl);
    for (int b = 0; b < pc; ++b) {
      int c0, cl;
      part_range(cols, pc, b, &c0, &cl);
      Seg sc = s;
      sc.kbase = 0;
      segs[cursor] = sc;
      GemmItem it;
      it.C = C;
      it.ldc = ldc;
      it.row0 = r0;
      it.col0 = c0;
      it.m = rl;
      it.n = cl;
      it.seg0 = (int)cursor;
      it.nseg = 1;
      it.ktotal = s.k;
      it.accumulate = 0;
      it.alpha = 1.0;
      items[cursor] = it;
      ++cursor;
    }
  }
}

__device__ inline Seg make_seg(const double* L, int64_t sLi, int64_t sLk, const double* R,
                               int64_t sRk, int64_t sRj, int k, double scale) {
  Seg s;
  s.L = L;
  s.R = R;
  s.sLi = sLi;
  s.sLk = sLk;
  s.sRk = sRk;
  s.sRj = sRj;
  s.k = k;
  s.kbase = 0;
  s.scale = scale;
  return s;
}

// Inclusive sum over the lanes 0..lane of the wave.
template <typename T>
__device__ inline T wave_incl_scan(T v, int lane) {
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const T u = __shfl_up(v, d, 64);
    if (lane >= d) v += u;
  }
  return v;
}

// One wave per result block.  The lanes take the candidate terms of a chunk
// of 64 entries of the block's term list (the shorter of A's row list and B's
// column list), so the terms of a chunk are the lanes with both blocks nonzero,
// in ascending K; every list
// offset (terms, factor-product items, pool doubles, inner ranges) is an
// exclusive prefix sum over the terms before, plus the running totals of the
// earlier chunks: the lists are the ones a walk term by term would write.
constexpr int kFillThreads = 256;
__global__ __launch_bounds__(kFillThreads) void k_fill(PlanParams P, FillParams F) {
  const int npairs = P.nrb * P.ncb;
  const int lane = threadIdx.x & 63;
  const int pair = (int)((blockIdx.x * (unsigned)kFillThreads + threadIdx.x) >> 6);
  if (pair >= npairs) return;
  if (F.abort && *F.abort) return;   // a list would overflow its capacity
  // every block's offset (a zero block's is never read)
  if (lane == 0) F.c_boff[pair] = F.off[(int64_t)kCntOut * npairs + pair];
  const int fl = F.flags[pair];
  if (!(fl & kFlagComputed)) return;
  const bool densify = fl & kFlagDensify;
  const bool force = fl & kFlagForce;
  const int I = pair / P.ncb, J = pair % P.ncb;
  const int m = P.A.roff[I + 1] - P.A.roff[I];
  const int n = P.B.coff[J + 1] - P.B.coff[J];
  auto off = [&](int c) { return F.off[(int64_t)c * npairs + pair]; };
  // running totals of the earlier chunks (uniform in the wave)
  int64_t po = off(kCntPool);
  int64_t so = off(kCntSegDense);
  const int64_t so0 = so;
  int64_t pi = off(kCntPieces);
  const int64_t pi0 = pi;
  int64_t t1 = off(kCntThin1);
  int64_t t2 = off(kCntThin2);
  const int64_t cslot = off(kCntOut);
  double* accb = F.acc + off(kCntAcc);
  int kb = 0;
  int rcat = 0;
  bool anydd = false;
  const TermList tl = term_list(P, I, J);
  for (int c0 = 0; c0 < tl.n; c0 += 64) {
    const int K = c0 + lane < tl.n ? tl.k[c0 + lane] : -1;
    const int ka = K >= 0 ? P.A.kind[I * P.nkb + K] : 0;
    const int kbk = K >= 0 ? P.B.kind[K * P.ncb + J] : 0;
    const bool term = ka != 0 && kbk != 0;
    // this lane's term: its counts
    int k = 0, ra = 0, rb = 0, rk = 0;   // rk: rank (inner extent) of the term's dense form
    int64_t npool = 0, nt1 = 0, nt2 = 0;
    if (term) {
      k = P.A.coff[K + 1] - P.A.coff[K];
      ra = ka == 2 ? P.A.rank[I * P.nkb + K] : 0;
      rb = kbk == 2 ? P.B.rank[K * P.ncb + J] : 0;
      if (ka == 1 && kbk == 1) {
        rk = k;
      } else if (ka == 2 && kbk == 1) {
        rk = ra;
        npool = (int64_t)n * ra;
        nt1 = thin_parts(P.edges, n, ra);
      } else if (ka == 1 && kbk == 2) {
        rk = rb;
        npool = (int64_t)m * rb;
        nt1 = thin_parts(P.edges, m, rb);
      } else {
        nt1 = thin_parts(P.edges, ra, rb);
        if (rb < ra) {
          rk = rb;
          npool = (int64_t)ra * rb + (int64_t)m * rb;
          nt2 = thin_parts(P.edges, m, rb);
        } else {
          rk = ra;
          npool = (int64_t)ra * rb + (int64_t)n * ra;
          nt2 = thin_parts(P.edges, n, ra);
        }
      }
    }
    const int one = term ? 1 : 0;
    // exclusive prefixes over the chunk's terms
    const int64_t xpool = wave_incl_scan<long long>(npool, lane) - npool;
    const int64_t xt1 = wave_incl_scan<long long>(nt1, lane) - nt1;
    const int64_t xt2 = wave_incl_scan<long long>(nt2, lane) - nt2;
    const int xone = wave_incl_scan<int>(one, lane) - one;
    const int xrk = wave_incl_scan<int>(term ? rk : 0, lane) - (term ? rk : 0);
    if (term) {
      const double* a = block_at(P.A, I * P.nkb + K);
      const double* b = block_at(P.B, K * P.ncb + J);
      int64_t my_po = po + xpool;
      int64_t my_t1 = t1 + xt1;
      int64_t my_t2 = t2 + xt2;
      Seg dense_term;
      Piece pc;
      pc.pad = 0;
      pc.scale = P.alpha;
      if (ka == 1 && kbk == 1) {
        dense_term = make_seg(a, 1, m, b, 1, k, k, 1.0);
      } else if (ka == 2 && kbk == 1) {
        // LD: U_A (B^T V_A)^T; T = B^T V_A is n x rA
        const double* Ua = a;
        const double* Va = a + (int64_t)m * ra;
        double* T = F.pool + my_po;
        emit_thin(F.seg_thin1, F.items_thin1, my_t1, make_seg(b, k, 1, Va, 1, k, k, 1.0), T, n, n,
                  ra, P.edges);
        dense_term = make_seg(Ua, 1, m, T, n, 1, ra, 1.0);
        pc.U = Ua; pc.ldu = m; pc.V = T; pc.ldv = n; pc.r = ra;
      } else if (ka == 1 && kbk == 2) {
        // DL: (A U_B) V_B^T; T = A U_B is m x rB
        const double* Ub = b;
        const double* Vb = b + (int64_t)k * rb;
        double* T = F.pool + my_po;
        emit_thin(F.seg_thin1, F.items_thin1, my_t1, make_seg(a, 1, m, Ub, 1, k, k, 1.0), T, m, m,
                  rb, P.edges);
        dense_term = make_seg(T, 1, m, Vb, n, 1, rb, 1.0);
        pc.U = T; pc.ldu = m; pc.V = Vb; pc.ldv = n; pc.r = rb;
      } else {
        // LL: core Z = V_A^T U_B (rA x rB), absorbed on the side giving the smaller rank (Eq. (4))
        const double* Ua = a;
        const double* Va = a + (int64_t)m * ra;
        const double* Ub = b;
        const double* Vb = b + (int64_t)k * rb;
        double* Z = F.pool + my_po;
        emit_thin(F.seg_thin1, F.items_thin1, my_t1, make_seg(Va, k, 1, Ub, 1, k, k, 1.0), Z, ra,
                  ra, rb, P.edges);
        double* T = Z + (int64_t)ra * rb;
        if (rb < ra) {
          // T = U_A Z (m x rB)
          emit_thin(F.seg_thin2, F.items_thin2, my_t2, make_seg(Ua, 1, m, Z, 1, ra, ra, 1.0), T, m,
                    m, rb, P.edges);
          dense_term = make_seg(T, 1, m, Vb, n, 1, rb, 1.0);
          pc.U = T; pc.ldu = m; pc.V = Vb; pc.ldv = n; pc.r = rb;
        } else {
          // T = V_B Z^T (n x rA)
          emit_thin(F.seg_thin2, F.items_thin2, my_t2, make_seg(Vb, 1, n, Z, ra, 1, rb, 1.0), T, n,
                    n, ra, P.edges);
          dense_term = make_seg(Ua, 1, m, T, n, 1, ra, 1.0);
          pc.U = Ua; pc.ldu = m; pc.V = T; pc.ldv = n; pc.r = ra;
        }
      }
      if (densify) {
        dense_term.kbase = kb + xrk;
        F.seg_dense[so + xone] = dense_term;
      } else {
        F.pieces[pi + xone] = pc;
      }
    }
    // advance the running totals by the chunk's sums (read from the last lane)
    const int64_t spool = __shfl(xpool + npool, 63, 64);
    const int64_t st1 = __shfl(xt1 + nt1, 63, 64);
    const int64_t st2 = __shfl(xt2 + nt2, 63, 64);
    const int sone = __shfl(xone + one, 63, 64);
    const int srk = __shfl(xrk + (term ? rk : 0), 63, 64);
    po += spool;
    t1 += st1;
    t2 += st2;
    if (densify) {
      so += sone;
      kb += srk;
    } else {
      pi += sone;
      rcat += srk;
    }
    anydd = anydd || __ballot(term && ka == 1 && kbk == 1) != 0ull;
  }
  if (lane != 0) return;
  const double tau = P.screen ? P.eps_sp * m * (double)n : P.eps_sp;
  if (densify) {
    int64_t gi = off(kCntGemmItems);
    const int de = dense_edge(P.edges, m, n);
    const int pr = num_parts(m, de), pcn = num_parts(n, de);
    for (int a = 0; a < pr; ++a) {
      int r0, rl;
      part_range(m, pr, a, &r0, &rl);
      for (int b = 0; b < pcn; ++b) {
        int c0, cl;
        part_range(n, pcn, b, &c0, &cl);
        GemmItem it;
        it.C = accb;
        it.ldc = m;
        it.row0 = r0;
        it.col0 = c0;
        it.m = rl;
        it.n = cl;
        it.seg0 = (int)so0;
        it.nseg = (int)(so - so0);
        it.ktotal = kb;
        it.accumulate = 0;
        it.alpha = P.alpha;
        F.items_dense[gi++] = it;
      }
    }
  }
  RecItem r{};   // every field defined (rrqr = 0: products truncate by the SVD)
  r.path = force ? kPathForceDense : (densify ? kPathDense : kPathLowRank);
  r.m = m;
  r.n = n;
  r.piece0 = (int)pi0;
  r.npieces = (int)(pi - pi0);
  r.R = rcat;
  // blocks with a dense x dense term are the ones that tend to stay dense;
  // blocks densified only by the number of low-rank terms mostly end low-rank
  r.cert_hint = anydd ? 1 : 0;
  r.D = accb;
  r.ldd = m;
  r.tau = tau;
  r.out = F.c_arena + cslot;
  r.scratch = F.cnt[(int64_t)kCntScratch * npairs + pair] > 0 ? F.scratch + off(kCntScratch)
                                                               : nullptr;
  r.kind_out = F.c_kind + pair;
  r.rank_out = F.c_rank + pair;
  r.norm_out = F.c_norm + pair;
  F.rec[off(kCntComputed)] = r;
}

hipError_t launch_symbolic(const PlanParams& P, int64_t* cnt, double* st, int* flags,
                           hipStream_t s) {
  const int npairs = P.nrb * P.ncb;
  if (npairs == 0) return hipSuccess;
  constexpr int per = kSymThreads / 64;   // result blocks (waves) per workgroup
  hipLaunchKernelGGL(k_symbolic, dim3((npairs + per - 1) / per), dim3(kSymThreads), 0, s, P, cnt,
                     st, flags);
  return hipGetLastError();
}

hipError_t launch_scan(const int64_t* in, int64_t* out, int64_t n, int narrays, int64_t* totals,
                       hipStream_t s) {
  if (narrays <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_scan, dim3(narrays), dim3(1024), 0, s, in, out, n, narrays, totals);
  return hipGetLastError();
}

hipError_t launch_reduce(const double* in, int64_t n, int narrays, double* totals,
                         hipStream_t s) {
  if (narrays <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_reduce, dim3(narrays), dim3(256), 0, s, in, n, narrays, totals);
  return hipGetLastError();
}

// Shift the exclusive prefix sums of one product of a batch by that product's
// place in the batch's concatenated work lists (base[a] for array a).
__global__ void k_add_base(int64_t* __restrict__ off, int64_t n, int narrays,
                           const int64_t* __restrict__ base) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int a = 0; a < narrays; ++a) off[(int64_t)a * n + i] += base[a];
}

hipError_t launch_add_base(int64_t* off, int64_t n, int narrays, const int64_t* base,
                           hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_add_base, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, off, n,
                     narrays, base);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Capacity check of a run whose list lengths stay on the device (one thread).
// ---------------------------------------------------------------------------
__global__ void k_caps(const int64_t* __restrict__ totals, Caps caps, int64_t* __restrict__ live) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  bool over = live[kLiveOverflow] != 0;
  for (int c = 0; c < kNumCounters; ++c) {
    const int64_t t = totals[c];
    if (t > caps.c[c]) over = true;
    if (t > live[kLiveNeed + c]) live[kLiveNeed + c] = t;
  }
  for (int c = 0; c < kNumCounters; ++c) live[c] = over ? 0 : totals[c];
  if (over) live[kLiveOverflow] = 1;
}

// acc[0] += the flop totals of one product (DD, LD, DL, LL and densify terms).
__global__ void k_add_flops(const double* __restrict__ tot_st, double* __restrict__ acc) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  acc[0] += tot_st[kStFlopsDD] + tot_st[kStFlopsLD] + tot_st[kStFlopsDL] + tot_st[kStFlopsLL] +
            tot_st[kStFlopsDensify];
}

hipError_t launch_add_flops(const double* tot_st, double* acc, hipStream_t s) {
  hipLaunchKernelGGL(k_add_flops, dim3(1), dim3(64), 0, s, tot_st, acc);
  return hipGetLastError();
}

hipError_t launch_caps(const int64_t* totals, const Caps& caps, int64_t* live, hipStream_t s) {
  hipLaunchKernelGGL(k_caps, dim3(1), dim3(64), 0, s, totals, caps, live);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Blockwise combination T = a X + b Y + c I.  Per block: the estimate
// |a| ||X_IJ|| + |b| ||Y_IJ|| + |c| sqrt(m) (the identity on diagonal blocks)
// screened against tau; the block is summed densely (and then recompressed
// by the dense path) if it is diagonal, has a dense operand, or its
// concatenated rank reaches half its short edge; otherwise the factors are
// concatenated (Eq. (5)) and recompressed by the low-rank path.
// ---------------------------------------------------------------------------
struct CombDecision {
  bool computed, densify, diag;
  int m, n, kx, ky, rx, ry, R;
  double tau;
};

__device__ inline CombDecision comb_decide(const CombParams& P, int I, int J) {
  CombDecision d{};
  const int b = I * P.X.ncb + J;
  d.m = P.X.roff[I + 1] - P.X.roff[I];
  d.n = P.X.coff[J + 1] - P.X.coff[J];
  d.kx = P.X.kind[b];
  d.ky = P.Y.kind ? P.Y.kind[b] : 0;
  d.rx = d.kx == 2 ? P.X.rank[b] : 0;
  d.ry = d.ky == 2 ? P.Y.rank[b] : 0;
  d.diag = P.square && I == J;
  const bool has_i = d.diag && P.c != 0.0;
  double est = 0.0;
  if (d.kx) est += fabs(P.a) * P.X.norm[b];
  if (d.ky) est += fabs(P.b) * P.Y.norm[b];
  if (has_i) est += fabs(P.c) * sqrt((double)d.m);
  d.tau = P.screen ? P.eps_sp * d.m * (double)d.n : P.eps_sp;
  d.computed = (d.kx || d.ky || has_i) && est >= d.tau;
  d.R = d.rx + d.ry;
  const bool any_dense = d.kx == 1 || d.ky == 1 || has_i;
  d.densify = d.diag || any_dense || 2 * d.R >= min(d.m, d.n);
  return d;
}

__global__ void k_comb_count(CombParams P, int64_t* __restrict__ cnt) {
  const int nb = P.X.nrb * P.X.ncb;
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  const CombDecision d = comb_decide(P, b / P.X.ncb, b % P.X.ncb);
  int64_t c[kNumCounters];
  for (int i = 0; i < kNumCounters; ++i) c[i] = 0;
  if (d.computed) {
    const int nlr = (d.kx == 2) + (d.ky == 2);
    c[kCntComputed] = 1;
    if (d.densify) {
      c[kCntCombDense] = 1;
      c[kCntSegDense] = nlr;
      c[kCntGemmItems] = nlr ? dense_parts(P.edges, d.m, d.n) : 0;
      c[kCntScratch] =
          rec_scratch_doubles(d.diag ? kPathForceDense : kPathDense, d.m, d.n, 0, P.tol);
      c[kCntOut] = (int64_t)d.m * d.n;
      c[kCntAcc] = (int64_t)d.m * d.n;
    } else {
      c[kCntPieces] = nlr;
      c[kCntScratch] = rec_scratch_doubles(kPathLowRank, d.m, d.n, d.R, P.tol);
      c[kCntOut] = (int64_t)(d.m + d.n) * d.R;
    }
  }
  for (int i = 0; i < kNumCounters; ++i) cnt[(int64_t)i * nb + b] = c[i];
}

__global__ void k_comb_fill(CombParams P, CombLists L) {
  const int nb = P.X.nrb * P.X.ncb;
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  if (L.abort && *L.abort) return;
  auto off = [&](int c) { return L.off[(int64_t)c * nb + b]; };
  P.t_boff[b] = off(kCntOut);   // every block's (a zero block's is never read)
  const int I = b / P.X.ncb, J = b % P.X.ncb;
  const CombDecision d = comb_decide(P, I, J);
  if (!d.computed) return;
  const int m = d.m, n = d.n;
  const double* xs = block_at(P.X, b);
  const double* ys = P.Y.kind ? block_at(P.Y, b) : nullptr;
  double* accb = P.acc + off(kCntAcc);
  RecItem r{};
  r.m = m;
  r.n = n;
  r.tau = d.tau;
  r.out = P.t_arena + off(kCntOut);
  r.kind_out = P.t_kind + b;
  r.rank_out = P.t_rank + b;
  r.norm_out = P.t_norm + b;
  if (d.densify) {
    r.path = d.diag ? kPathForceDense : kPathDense;
    r.cert_hint = 1;
    r.D = accb;
    r.ldd = m;
    AxpbyDenseItem di;
    di.D = accb;
    di.X = d.kx == 1 ? xs : nullptr;
    di.Y = d.ky == 1 ? ys : nullptr;
    di.a = P.a;
    di.b = P.b;
    di.c = d.diag ? P.c : 0.0;
    di.m = m;
    di.n = n;
    L.dense[off(kCntCombDense)] = di;
    // low-rank operands enter the dense sum as U V^T products (scale a or b)
    const int64_t s0 = off(kCntSegDense);
    int64_t sc = s0;
    int kb = 0;
    auto add_lr = [&](const double* f, int rk, double scale) {
      Seg sg;
      sg.L = f;                     // U (m x r)
      sg.sLi = 1;
      sg.sLk = m;
      sg.R = f + (int64_t)m * rk;   // V (n x r) used transposed
      sg.sRk = n;
      sg.sRj = 1;
      sg.k = rk;
      sg.kbase = kb;
      sg.scale = scale;
      kb += rk;
      L.segs[sc++] = sg;
    };
    if (d.kx == 2) add_lr(xs, d.rx, P.a);
    if (d.ky == 2) add_lr(ys, d.ry, P.b);
    if (kb > 0) {
      int64_t gi = off(kCntGemmItems);
      const int de = dense_edge(P.edges, m, n);
      const int pr = num_parts(m, de), pc = num_parts(n, de);
      for (int pa = 0; pa < pr; ++pa)
        for (int pb = 0; pb < pc; ++pb) {
          GemmItem g;
          part_range(m, pr, pa, &g.row0, &g.m);
          part_range(n, pc, pb, &g.col0, &g.n);
          g.C = accb;
          g.ldc = m;
          g.seg0 = (int)s0;
          g.nseg = (int)(sc - s0);
          g.ktotal = kb;
          g.accumulate = 1;
          g.alpha = 1.0;
          L.items[gi++] = g;
        }
    }
  } else {
    r.path = kPathLowRank;
    r.piece0 = (int)off(kCntPieces);
    r.R = d.R;
    int64_t pi = off(kCntPieces);
    auto add_piece = [&](const double* f, int rk, double scale) {
      Piece p{};
      p.U = f;
      p.ldu = m;
      p.V = f + (int64_t)m * rk;
      p.ldv = n;
      p.r = rk;
      p.scale = scale;
      L.pieces[pi++] = p;
    };
    if (d.kx == 2) add_piece(xs, d.rx, P.a);
    if (d.ky == 2) add_piece(ys, d.ry, P.b);
    r.npieces = (int)(pi - r.piece0);
  }
  r.scratch = L.cnt[(int64_t)kCntScratch * nb + b] > 0 ? L.scratch + off(kCntScratch) : nullptr;
  L.rec[off(kCntComputed)] = r;
}

hipError_t launch_comb_count(const CombParams& P, int64_t* cnt, hipStream_t s) {
  const int nb = P.X.nrb * P.X.ncb;
  if (nb == 0) return hipSuccess;
  hipLaunchKernelGGL(k_comb_count, dim3((nb + 255) / 256), dim3(256), 0, s, P, cnt);
  return hipGetLastError();
}

hipError_t launch_comb_fill(const CombParams& P, const CombLists& L, hipStream_t s) {
  const int nb = P.X.nrb * P.X.ncb;
  if (nb == 0) return hipSuccess;
  hipLaunchKernelGGL(k_comb_fill, dim3((nb + 255) / 256), dim3(256), 0, s, P, L);
  return hipGetLastError();
}

hipError_t launch_fill(const PlanParams& P, const FillParams& F, hipStream_t s) {
  const int npairs = P.nrb * P.ncb;
  if (npairs == 0) return hipSuccess;
  constexpr int per = kFillThreads / 64;   // result blocks (waves) per workgroup
  hipLaunchKernelGGL(k_fill, dim3((npairs + per - 1) / per), dim3(kFillThreads), 0, s, P, F);
  return hipGetLastError();
}

}  // namespace clr
