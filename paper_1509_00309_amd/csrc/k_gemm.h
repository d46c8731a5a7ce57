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
//               partial of every 32 inner indices is added into FP64
//               accumulators; optionally the hi*lo + lo*hi correction terms
//               (lo = fp32(x - hi)) go to a second FP32 partial.
//
// Workgroup: 512 threads = 8 waves in a 2 x 4 arrangement (two waves per
// SIMD, so one computes while the other stages operands or waits at the slab
// barrier); wave (wr, wc) owns the 16 x 16 output tiles (wr + 2a, wc + 4b),
// a < NA, b < NB, where NA, NB are the item's valid tile counts for that wave
// (at most 5 x 3 of the 10 x 10 tiles of the FP64 form and of the plain
// FP32 form, 4 x 2 of the 8 x 8 tiles of the corrected FP32 form).  The item loop is instantiated per (NA, NB) and
// selected once per item by a scalar switch, so no MFMA sits behind a
// per-tile branch and each variant keeps only its own accumulators live.
//
// MFMA operand layout for the 16x16x4 shapes (64 lanes, lane = l):
//   A(i, k): i = l % 16, k = l / 16;   B(k, j): j = l % 16, k = l / 16;
//   D(i, j) is held by lane l = j + 16*g, element v, with
//     f32: i = 4*g + v        f64: i = g + 4*v   (the f64 shape interleaves rows).
#pragma once
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

__device__ inline int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ inline int64_t uni64(int64_t v) {
  const int lo = __builtin_amdgcn_readfirstlane((int)(v & 0xffffffffLL));
  const int hi = __builtin_amdgcn_readfirstlane((int)(v >> 32));
  return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

constexpr int kSegCache = 96;  // segment descriptors of an item kept in LDS (operand-split kernel)
constexpr int kSegCacheLds = 256;  // same in the LDS GEMM kernel
typedef const Seg __attribute__((address_space(1))) gseg;   // descriptors in global memory
typedef const Seg __attribute__((address_space(3))) lseg;   // descriptors cached in LDS

// Wave grid and tiles of the LDS kernel per form: WR x WC waves, a wave owns
// up to TA x TB of the TILES x TILES tiles of 16 x 16.  The FP64 form and the
// FP32-MFMA form without correction products take items of up to 160 x 160
// (every block of the 96..160 workloads in one item); the corrected FP32 form
// holds a second FP32 partial per tile and keeps to 128 x 128.
template <bool F32, bool SPLIT>
struct GemmCfg {
  static constexpr int WR = 2, WC = 4, TA = 5, TB = 3, TILES = 10;   // 160 x 160
};
template <>
struct GemmCfg<true, true> {
  static constexpr int WR = 2, WC = 4, TA = 4, TB = 2, TILES = 8;    // 128 x 128
};
constexpr int kLdsGemmThreads = 512;
// s_waitcnt operand (gfx9 encoding) that waits for vmcnt 0 and leaves the
// expcnt and lgkmcnt limits at their maxima.
constexpr int kWaitVmAll = 0x0F70;
// FP32 partials of the mixed form are added into the FP64 accumulators every
// kF32FlushSlabs slabs (32 inner indices).
constexpr int kF32FlushSlabs = 2;

template <bool F32, bool SPLIT>
struct GemmLds {
  static constexpr int TM = 16 * GemmCfg<F32, SPLIT>::TILES;
  static constexpr int LD = TM + 1;  // odd stride: k-fast stores hit distinct banks
  using T = typename std::conditional<F32, float, double>::type;
  T a[2][kSlabK][LD];
  T b[2][kSlabK][LD];
  T alo[SPLIT ? 2 : 1][SPLIT ? kSlabK : 1][SPLIT ? LD : 1];
  T blo[SPLIT ? 2 : 1][SPLIT ? kSlabK : 1][SPLIT ? LD : 1];
  // per inner-row source descriptors of the slabs in flight
  const double* lp[2][kSlabK];
  const double* rp[2][kSlabK];
  int64_t sli[2][kSlabK];
  int64_t srj[2][kSlabK];
  double scale[2][kSlabK];   // L scale of the row; 0 for rows past the item
  Seg segs[kSegCacheLds];
};

// Thread t < 16 resolves inner row t of slab `slab`: which segment it falls in
// and where its L column / R row start.  `cur` is that thread's segment cursor
// (monotone over slabs).  With kAll, `cache` holds every descriptor of the
// item; otherwise the first kSegCache come from it and the rest from `segs`.
// A row past the item gets the first segment's operands with zero strides and
// zero weights, so every address the loader forms is valid.
// CacheP is the type of the cached-descriptor pointer: an LDS-qualified
// pointer in the LDS kernel (so its loads stay LDS loads), a plain pointer
// where the "cache" is global memory.
template <typename CacheP, bool kAll = false>
__device__ inline void resolve_row(const GemmItem& it, const Seg* __restrict__ segs,
                                   CacheP cache, int slab, int t, int& cur,
                                   const double*& lp, const double*& rp, int64_t& sli,
                                   int64_t& srj, double& sc, double& bok) {
  const int g = slab * kSlabK + t;
  lp = cache[0].L;
  rp = cache[0].R;
  sli = 0;
  srj = 0;
  sc = 0.0;
  bok = 0.0;
  if (g >= it.ktotal) return;
  // The cached descriptors and the global ones are read on separate paths, so
  // each load keeps its own address space (a pointer selected between the two
  // would be generic, and flat loads also wait on the global-load counter).
  while (cur < it.nseg) {
    int kend;
    if (kAll || cur < kSegCache) {
      kend = cache[cur].kbase + cache[cur].k;
    } else {
      const gseg* sg = (const gseg*)(segs + it.seg0 + cur);
      kend = sg->kbase + sg->k;
    }
    if (g < kend) break;
    ++cur;
  }
  if (cur >= it.nseg) return;
  const double* L;
  const double* R;
  int64_t sLi, sLk, sRk, sRj;
  int kbase;
  double scale;
  if (kAll || cur < kSegCache) {
    const auto& s = cache[cur];
    L = s.L; R = s.R; sLi = s.sLi; sLk = s.sLk; sRk = s.sRk; sRj = s.sRj; kbase = s.kbase;
    scale = s.scale;
  } else {
    const gseg& s = *(const gseg*)(segs + it.seg0 + cur);
    L = s.L; R = s.R; sLi = s.sLi; sLk = s.sLk; sRk = s.sRk; sRj = s.sRj; kbase = s.kbase;
    scale = s.scale;
  }
  const int kl = g - kbase;
  lp = L + (int64_t)it.row0 * sLi + (int64_t)kl * sLk;
  rp = R + (int64_t)it.col0 * sRj + (int64_t)kl * sRk;
  sli = sLi;
  srj = sRj;
  sc = scale;
  bok = 1.0;
}

// MFMA work of one LDS slab for a wave that owns NA x NB valid tiles
// (tile rows wr + WR a, tile columns wc + WC b).  The tile counts are
// template constants so the body is straight-line code.  `mid(q)` runs after
// the MFMAs of 4-step q are issued: the staging stores of the next slab go
// there, so they execute while the matrix pipe works through those MFMAs
// (the scheduling barriers keep the compiler from moving them back behind the
// whole chain).
template <bool F32, bool SPLIT, int NA, int NB, typename Mid>
__device__ __attribute__((always_inline)) inline void slab_mfma(
    GemmLds<F32, SPLIT>& sh, int cur, int wr, int wc, int kr, int lc,
    d4 (&acc)[GemmCfg<F32, SPLIT>::TA][GemmCfg<F32, SPLIT>::TB],
    f4 (&p)[GemmCfg<F32, SPLIT>::TA][GemmCfg<F32, SPLIT>::TB],
    f4 (&pl)[SPLIT ? GemmCfg<F32, SPLIT>::TA : 1][SPLIT ? GemmCfg<F32, SPLIT>::TB : 1], bool flush,
    Mid&& mid) {
  constexpr int WR = GemmCfg<F32, SPLIT>::WR, WC = GemmCfg<F32, SPLIT>::WC;
  if constexpr (!F32) {
    // operands of 4-step q + 1 are read from LDS while the MFMAs of q run
    // (two operand sets instead of the whole slab's)
    double av[2][NA], bv[2][NB];
#pragma unroll
    for (int a = 0; a < NA; ++a) av[0][a] = sh.a[cur][kr][16 * (wr + WR * a) + lc];
#pragma unroll
    for (int b = 0; b < NB; ++b) bv[0][b] = sh.b[cur][kr][16 * (wc + WC * b) + lc];
#pragma unroll
    for (int q = 0; q < kSlabK / 4; ++q) {
      if (q + 1 < kSlabK / 4) {
#pragma unroll
        for (int a = 0; a < NA; ++a)
          av[(q + 1) & 1][a] = sh.a[cur][4 * (q + 1) + kr][16 * (wr + WR * a) + lc];
#pragma unroll
        for (int b = 0; b < NB; ++b)
          bv[(q + 1) & 1][b] = sh.b[cur][4 * (q + 1) + kr][16 * (wc + WC * b) + lc];
      }
#pragma unroll
      for (int a = 0; a < NA; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[q & 1][a], bv[q & 1][b], acc[a][b], 0,
                                                             0, 0);
      __builtin_amdgcn_sched_barrier(0);
      mid(q);
      __builtin_amdgcn_sched_barrier(0);
    }
  } else {
#pragma unroll
    for (int q = 0; q < kSlabK / 4; ++q) {
      float av[NA], bv[NB];
#pragma unroll
      for (int a = 0; a < NA; ++a) av[a] = sh.a[cur][4 * q + kr][16 * (wr + WR * a) + lc];
#pragma unroll
      for (int b = 0; b < NB; ++b) bv[b] = sh.b[cur][4 * q + kr][16 * (wc + WC * b) + lc];
#pragma unroll
      for (int a = 0; a < NA; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b)
          p[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a], bv[b], p[a][b], 0, 0, 0);
      if constexpr (SPLIT) {
        float al[NA], bl[NB];
#pragma unroll
        for (int a = 0; a < NA; ++a) al[a] = sh.alo[cur][4 * q + kr][16 * (wr + WR * a) + lc];
#pragma unroll
        for (int b = 0; b < NB; ++b) bl[b] = sh.blo[cur][4 * q + kr][16 * (wc + WC * b) + lc];
#pragma unroll
        for (int a = 0; a < NA; ++a)
#pragma unroll
          for (int b = 0; b < NB; ++b) {
            pl[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a], bl[b], pl[a][b], 0, 0, 0);
            pl[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(al[a], bv[b], pl[a][b], 0, 0, 0);
          }
      }
      __builtin_amdgcn_sched_barrier(0);
      mid(q);
      __builtin_amdgcn_sched_barrier(0);
    }
    // FP64 flush of the FP32 partials (every kF32FlushSlabs slabs and after the last)
    if (flush) {
#pragma unroll
      for (int a = 0; a < NA; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b) {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            double add = (double)p[a][b][v];
            if constexpr (SPLIT) add += (double)pl[a][b][v];
            acc[a][b][v] += add;
          }
          p[a][b] = f4{0.f, 0.f, 0.f, 0.f};
          if constexpr (SPLIT) pl[a][b] = f4{0.f, 0.f, 0.f, 0.f};
        }
    }
  }
}

// Main loop and epilogue of one item for a wave that owns NA x NB valid
// tiles (0 x 0 for waves with nothing to compute; they still stage operands).
//
// Pipeline over 16-deep slabs with one barrier per slab.  While the MFMAs of
// slab s read LDS buffer s & 1, the staging registers, which hold slab s + 1
// (loaded during slab s - 1), are written to the other buffer between the
// MFMA steps: the L values after the first 4-step, the R values after the
// second.  Right after each store the same registers receive the global loads
// of slab s + 2.  Every load thus has a whole slab of MFMA work to land, and
// the staging stores run while the matrix pipe is busy instead of after it.
template <bool F32, bool SPLIT, int NA, int NB>
__device__ __attribute__((always_inline)) inline void run_item(GemmLds<F32, SPLIT>& sh,
                                                                const GemmItem& it,
                                                                const Seg* __restrict__ segs,
                                                                int wr, int wc) {
  using CF = GemmCfg<F32, SPLIT>;
  constexpr int WR = CF::WR, WC = CF::WC;
  constexpr int TM = GemmLds<F32, SPLIT>::TM;
  constexpr int LD = GemmLds<F32, SPLIT>::LD;
  constexpr int NE = TM / 32;  // staged elements per thread and operand
  static_assert(kSlabK == 16 && kLdsGemmThreads == 512, "staging map assumes 16 x 32 threads");
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int nslab = (it.ktotal + kSlabK - 1) / kSlabK;

  d4 acc[CF::TA][CF::TB];
  // FP32 partials of the mixed form (unused in the FP64 form)
  f4 p[CF::TA][CF::TB];
  f4 pl[SPLIT ? CF::TA : 1][SPLIT ? CF::TB : 1];
#pragma unroll
  for (int a = 0; a < NA; ++a)
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};
      if constexpr (F32) p[a][b] = f4{0.f, 0.f, 0.f, 0.f};
      if constexpr (SPLIT) pl[a][b] = f4{0.f, 0.f, 0.f, 0.f};
    }

  int cursor = 0;  // meaningful for tid < 16 only
  // Inner row `tid` of slab `slab`: its operand pointers, strides and scale
  // go to descriptor buffer `d` (two buffers, by slab parity).
  // Every term descriptor comes from the LDS cache when the item has at most
  // kSegCacheLds terms (the choice is uniform over the item), else from global
  // memory: a lane-by-lane mix of the two would make each lookup wait for all of
  // the wave's global loads, the operand prefetch included.
  auto resolve = [&](int slab, int d) {
    if (tid < kSlabK) {
      const double* lp;
      const double* rp;
      int64_t sli, srj;
      double sc, bok;
      if (it.nseg <= kSegCacheLds)
        resolve_row<lseg*, true>(it, segs, (lseg*)sh.segs, slab, tid, cursor, lp, rp, sli, srj, sc,
                                 bok);
      else {
        resolve_row<gseg*, true>(it, segs, (gseg*)(segs + it.seg0), slab, tid, cursor, lp, rp, sli,
                                 srj, sc, bok);
        // Nothing of this path stays in flight: otherwise the compiler, which
        // cannot tell the paths apart where they join, waits for every global
        // load at the top of each slab (the operand prefetch included) before
        // it reuses the registers these descriptor loads wrote.
        __builtin_amdgcn_s_waitcnt(kWaitVmAll);
      }
      sh.lp[d][tid] = lp;
      sh.rp[d][tid] = rp;
      sh.sli[d][tid] = sli;
      sh.srj[d][tid] = srj;
      sh.scale[d][tid] = sc;
    }
  };
  // Staging map: every thread serves one inner row t of the slab and the
  // elements i0 + 32u of that row.  Rows contiguous in memory (unit stride
  // along i) are read row-fast: t = tid / 32, i0 = tid % 32, so 32 lanes read
  // 256 contiguous bytes; otherwise inner-fast: t = tid % 16, i0 = tid / 16,
  // so 16 lanes read 16 consecutive inner indices.  The map is fixed per slab
  // from row 0 and a thread needs one descriptor per operand and slab.
  //
  // Global -> registers without branches or selects: an element past the
  // item's m rows (n columns) reads row m - 1 (column n - 1) instead.  Such an
  // element only enters output rows (columns) that are never stored, so its
  // value does not matter.  An inner row past the item's last term reads the
  // first term's operands with zero strides and scale 0, so its L values
  // become exact zeros (the R values are finite) and it adds nothing.
  double ra[NE], rb[NE];
  int aoff = 0, boff = 0;   // LDS offsets (inner row * LD + first element) of the staged values
  double sc = 0.0;          // term scale of the thread's L row
  // Descriptors of the slab to load next, read at the top of a slab so their
  // LDS latency passes under its first MFMA step.  Both candidate rows of the
  // staging map (row-fast: tid / 32, inner-fast: tid % 16) are read
  // unconditionally, so no read waits for another; the map is chosen when
  // the loads are issued.
  struct Desc {
    int64_t s0;                 // stride of inner row 0 (selects the map)
    const double* p[2];         // operand pointers of the two candidate rows
    int64_t st[2];              // their strides along the tile
    double sc[2];               // their term scales (L only)
  };
  Desc da, db;
  const int t_row = tid >> 5, i_row = tid & 31;   // row-fast map
  const int t_inn = tid & 15, i_inn = tid >> 4;   // inner-fast map
  auto prep = [&](int d) {
    da.s0 = sh.sli[d][0];
    da.p[0] = sh.lp[d][t_row];
    da.p[1] = sh.lp[d][t_inn];
    da.st[0] = sh.sli[d][t_row];
    da.st[1] = sh.sli[d][t_inn];
    da.sc[0] = sh.scale[d][t_row];
    da.sc[1] = sh.scale[d][t_inn];
    db.s0 = sh.srj[d][0];
    db.p[0] = sh.rp[d][t_row];
    db.p[1] = sh.rp[d][t_inn];
    db.st[0] = sh.srj[d][t_row];
    db.st[1] = sh.srj[d][t_inn];
  };
  auto load_a = [&]() {
    const bool arow = da.s0 == 1;
    const int ta = arow ? t_row : t_inn;
    const int ia0 = arow ? i_row : i_inn;
    gdouble* pa = as_global(arow ? da.p[0] : da.p[1]);
    const int sa = (int)(arow ? da.st[0] : da.st[1]);
    const int mlast = it.m - 1;
#pragma unroll
    for (int u = 0; u < NE; ++u) ra[u] = pa[min(ia0 + 32 * u, mlast) * sa];
    aoff = ta * LD + ia0;
    sc = arow ? da.sc[0] : da.sc[1];
  };
  auto load_b = [&]() {
    const bool brow = db.s0 == 1;
    const int tb = brow ? t_row : t_inn;
    const int ib0 = brow ? i_row : i_inn;
    gdouble* pb = as_global(brow ? db.p[0] : db.p[1]);
    const int sb = (int)(brow ? db.st[0] : db.st[1]);
    const int nlast = it.n - 1;
#pragma unroll
    for (int u = 0; u < NE; ++u) rb[u] = pb[min(ib0 + 32 * u, nlast) * sb];
    boff = tb * LD + ib0;
  };
  auto store_a = [&](int buf) {
    auto* dst = &sh.a[buf][0][0] + aoff;
#pragma unroll
    for (int u = 0; u < NE; ++u) {
      const double xa = ra[u] * sc;
      if constexpr (F32) {
        const float ha = (float)xa;
        dst[32 * u] = ha;
        if constexpr (SPLIT) (&sh.alo[buf][0][0] + aoff)[32 * u] = (float)(xa - (double)ha);
      } else {
        dst[32 * u] = xa;
      }
    }
  };
  auto store_b = [&](int buf) {
    auto* dst = &sh.b[buf][0][0] + boff;
#pragma unroll
    for (int u = 0; u < NE; ++u) {
      const double xb = rb[u];
      if constexpr (F32) {
        const float hb = (float)xb;
        dst[32 * u] = hb;
        if constexpr (SPLIT) (&sh.blo[buf][0][0] + boff)[32 * u] = (float)(xb - (double)hb);
      } else {
        dst[32 * u] = xb;
      }
    }
  };

  const int kr = lane >> 4;   // inner row within a 4-step
  const int lc = lane & 15;   // row (A) / column (B) within a tile
  if (nslab > 0) {
    resolve(0, 0);
    if (nslab > 1) resolve(1, 1);
    __syncthreads();
    prep(0);
    load_a();
    load_b();
    store_a(0);
    store_b(0);
    if (nslab > 1) {
      prep(1);
      load_a();
      load_b();
    }
    __syncthreads();                 // buffer 0 holds slab 0; descriptors 0 and 1 consumed
    if (nslab > 2) resolve(2, 0);
    __syncthreads();
    for (int s = 0; s < nslab; ++s) {
      const int cur = s & 1, nxt = cur ^ 1;
      // descriptors of slab s + 2 sit in buffer s & 1, those of s + 1 were consumed
      // The staging stores and loads run in every slab, also where there is
      // no next slab to stage (they then store into the idle buffer and
      // reload the last prepared descriptors, whose addresses are valid).
      // With one path through the loop, the compiler's wait before each
      // store counts only the loads that precede it; a skipped load on one
      // path would make it wait for the newest prefetch on every path.
      if (s + 2 < nslab) prep(cur);
      if (s + 3 < nslab) resolve(s + 3, nxt);
      auto mid = [&](int q) {
        if (q == 0) {
          store_a(nxt);
          load_a();
        }
        if (q == 1) {
          store_b(nxt);
          load_b();
        }
      };
      if constexpr (NA > 0 && NB > 0) {
        const bool flush = (s % kF32FlushSlabs) == kF32FlushSlabs - 1 || s + 1 == nslab;
        slab_mfma<F32, SPLIT, NA, NB>(sh, cur, wr, wc, kr, lc, acc, p, pl, flush, mid);
      } else {
        mid(0);
        mid(1);
      }
      __syncthreads();
    }
  }

  // epilogue (output layout per precision, see the header comment).  The
  // accumulators leave through one more MFMA (+ 0 * 0): with only MFMA users
  // inside and after the loop, the compiler keeps them in accumulation
  // registers for the whole loop instead of copying them out every slab.
  const double alpha = it.alpha;
#pragma unroll
  for (int a = 0; a < NA; ++a) {
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const d4 fin = __builtin_amdgcn_mfma_f64_16x16x4f64(0.0, 0.0, acc[a][b], 0, 0, 0);
      const int j = 16 * (wc + WC * b) + lc;
      if (j >= it.n) continue;
      gdouble_mut* col = as_global_mut(it.C) + (int64_t)(it.col0 + j) * it.ldc + it.row0;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        // f64 16x16x4: row (lane/16) + 4v;  f32 16x16x4: row 4*(lane/16) + v
        const int i = 16 * (wr + WR * a) + (F32 ? 4 * kr + v : kr + 4 * v);
        if (i < it.m) {
          const double val = alpha * fin[v];
          col[i] = it.accumulate ? col[i] + val : val;
        }
      }
    }
  }
}

template <bool F32, bool SPLIT, int NA>
__device__ __attribute__((always_inline)) inline void run_nb(GemmLds<F32, SPLIT>& sh,
                                                              const GemmItem& it,
                                                              const Seg* __restrict__ segs,
                                                              int wr, int wc, int nb) {
  constexpr int TB = GemmCfg<F32, SPLIT>::TB;
  static_assert(TB >= 2 && TB <= 3, "column dispatch covers 2 or 3 tiles per wave");
  switch (nb) {
    case 0: run_item<F32, SPLIT, NA, 0>(sh, it, segs, wr, wc); break;
    case 1: run_item<F32, SPLIT, NA, 1>(sh, it, segs, wr, wc); break;
    case 2: run_item<F32, SPLIT, NA, 2>(sh, it, segs, wr, wc); break;
    default: run_item<F32, SPLIT, NA, TB>(sh, it, segs, wr, wc); break;
  }
}

// One item of the LDS kernel, start to finish (every thread of the workgroup).
template <bool F32, bool SPLIT>
__device__ __attribute__((always_inline)) inline void ggemm_item(GemmLds<F32, SPLIT>& sh,
                                                                  const GemmItem* __restrict__ items,
                                                                  const Seg* __restrict__ segs,
                                                                  int item) {
  using CF = GemmCfg<F32, SPLIT>;
  // Item fields are the same for every lane; readfirstlane lets the compiler
  // keep them (and all control flow derived from them) in scalar registers.
  GemmItem it = items[item];
  it.m = uni(it.m);
  it.n = uni(it.n);
  it.row0 = uni(it.row0);
  it.col0 = uni(it.col0);
  it.seg0 = uni(it.seg0);
  it.nseg = uni(it.nseg);
  it.ktotal = uni(it.ktotal);
  it.accumulate = uni(it.accumulate);
  it.ldc = uni64(it.ldc);
  const int tid = threadIdx.x;
  // Wave w runs on SIMD w % 4.  The two waves sharing a SIMD get tile-column
  // classes WC/2 apart, so every SIMD carries a wide and a narrow class.
  const int wave = uni(tid >> 6);
  const int wr = wave / CF::WC;
  const int wc = (wave % CF::WC + wr * (CF::WC / 2)) % CF::WC;
  const int mt = (it.m + 15) >> 4, nt = (it.n + 15) >> 4;
  // valid tiles of this wave: a with wr + WR a < mt, b with wc + WC b < nt
  const int na = min(CF::TA, max(0, (mt - wr + CF::WR - 1) / CF::WR));
  const int nb = min(CF::TB, max(0, (nt - wc + CF::WC - 1) / CF::WC));

  const int ncache = it.nseg <= kSegCacheLds ? it.nseg : 0;
  for (int s = tid; s < ncache; s += kLdsGemmThreads) sh.segs[s] = segs[it.seg0 + s];
  __syncthreads();

  // Every wave runs the same slab loop (the barriers are shared); only the
  // MFMA body and epilogue differ with the wave's tile counts.
  switch (na) {
    case 0: run_item<F32, SPLIT, 0, 0>(sh, it, segs, wr, wc); break;
    case 1: run_nb<F32, SPLIT, 1>(sh, it, segs, wr, wc, nb); break;
    case 2: run_nb<F32, SPLIT, 2>(sh, it, segs, wr, wc, nb); break;
    case 3: run_nb<F32, SPLIT, 3>(sh, it, segs, wr, wc, nb); break;
    case 4: run_nb<F32, SPLIT, 4>(sh, it, segs, wr, wc, nb); break;
    default: run_nb<F32, SPLIT, CF::TA>(sh, it, segs, wr, wc, nb); break;
  }
}

// DENSE only names the instantiation: the dense-accumulation launch of a
// product gets its own kernel symbol, so profiles separate it from the other
// launches that share the code.
//
// With `next` (a device counter, zero at launch), the launch is persistent:
// one workgroup per CU takes list slots from the counter until the list is
// exhausted, so the items of the longest-first order go to whichever CU of
// whichever XCD frees up first (list scheduling, no static XCD deal).
template <bool F32, bool SPLIT, bool DENSE>
__global__ __launch_bounds__(kLdsGemmThreads, 1) void k_ggemm(const GemmItem* __restrict__ items,
                                                              const Seg* __restrict__ segs,
                                                              int nitems,
                                                              const int* __restrict__ order,
                                                              const int64_t* __restrict__ live,
                                                              int* __restrict__ next) {
  __shared__ GemmLds<F32, SPLIT> sh;
  __shared__ int slot_sh;
  // a device-resident count (captured launches) caps the grid's capacity
  if (live) nitems = uni((int)min((int64_t)nitems, *live));

  if (next) {
    for (;;) {
      if (threadIdx.x == 0) slot_sh = atomicAdd(next, 1);
      __syncthreads();
      const int slot = uni(slot_sh);
      if (slot >= nitems) return;   // the same value in every thread
      ggemm_item<F32, SPLIT>(sh, items, segs, order ? order[slot] : slot);
      __syncthreads();   // LDS and slot_sh free for the next item
    }
  }

  // With an order (items by decreasing cost), workgroup b runs item order[b]:
  // the dispatcher deals workgroups to the 8 XCDs round-robin, so the long
  // items start first on every XCD and the short ones fill the tail.
  // Without one, the XCD-aware order: consecutive items (tiles of one block
  // row) share an XCD's L2.
  int item;
  if (order) {
    if ((int)blockIdx.x >= nitems) return;
    item = order[blockIdx.x];
  } else {
    item = xcd_unit(nitems, live != nullptr);
    if (item < 0 || item >= nitems) return;
  }
  ggemm_item<F32, SPLIT>(sh, items, segs, item);
}

static inline int xcd_grid(int n) { return ((n + 7) / 8) * 8; }

// ---------------------------------------------------------------------------
// Wave-per-item grouped GEMM for narrow items (the factor products of Eq. (4):
// one side is a rank).  Each wave computes one item of at most 4 x 4 tiles of
// 16 x 16, reading its MFMA operands straight from global memory (lane l takes
// row l % 16 and inner index l / 16 of each 16 x 4 fragment): no LDS and no
// barriers, so many items are in flight per CU and their load latencies
// overlap.  Terms of the item are walked in order, 16 inner indices per
// unrolled group (FP32 partials of the mixed form are flushed per group).
// ---------------------------------------------------------------------------
constexpr int kWaveTiles = 4;
constexpr int kWaveKSteps = 2;   // MFMA k-steps (of 4) per operand group; two groups in flight
static_assert(kMaxItemThin == 16 * kWaveTiles, "thin item edge = wave kernel tiles");
constexpr int kWaveItemsPerBlock = 4;

template <bool F32, bool SPLIT, int NA, int NB>
__device__ __attribute__((always_inline)) inline void wave_item(const GemmItem& it,
                                                                const Seg* __restrict__ segs,
                                                                int lane) {
  const int kr = lane >> 4, lc = lane & 15;
  d4 acc[NA][NB];
#pragma unroll
  for (int a = 0; a < NA; ++a)
#pragma unroll
    for (int b = 0; b < NB; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};
  for (int sgi = 0; sgi < it.nseg; ++sgi) {
    const Seg& sg = segs[it.seg0 + sgi];
    const int64_t sLi = uni64(sg.sLi), sLk = uni64(sg.sLk), sRk = uni64(sg.sRk), sRj = uni64(sg.sRj);
    const int K = uni(sg.k);
    const double scale = sg.scale;
    gdouble* L = as_global(sg.L) + (int64_t)it.row0 * sLi;
    gdouble* R = as_global(sg.R) + (int64_t)it.col0 * sRj;
    // per-lane fixed parts of the fragment addresses (rows / columns clamped
    // into the item; out-of-range entries are zeroed by selects)
    int64_t aoff[NA], boff[NB];
    bool aval[NA], bval[NB];
#pragma unroll
    for (int a = 0; a < NA; ++a) {
      const int i = 16 * a + lc;
      aval[a] = i < it.m;
      aoff[a] = (int64_t)(aval[a] ? i : 0) * sLi;
    }
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int j = 16 * b + lc;
      bval[b] = j < it.n;
      boff[b] = (int64_t)(bval[b] ? j : 0) * sRj;
    }
    // Two operand groups in flight: the raw loads of group g + 1 are issued
    // before the MFMAs of group g, so their latency hides behind that work.
    // Loads are unconditional; validity and the segment scale are applied by
    // selects right before the MFMAs, so no load result is consumed early.
    //
    // Inner-index order: the two k-steps of a group starting at k0 give lane
    // row kr the inner indices kp = k0 + 2 kr and kp + 1 (a fixed permutation
    // of the group's 8 indices, the same for A and B and for every item and
    // tiling).  An operand contiguous along the inner index then loads both
    // of a lane's values with one 16-byte load, starting at min(kp, K - 2) so
    // the pair stays inside the segment; the other operands load the two
    // values separately (an index past K reads index 0).
    constexpr int G = 4 * kWaveKSteps;
    static_assert(kWaveKSteps == 2, "inner pairs: two k-steps per group");
    typedef double d2 __attribute__((ext_vector_type(2)));
    typedef const d2 __attribute__((address_space(1), aligned(8))) gd2;
    const bool apair = sLk == 1 && K >= 2;   // A contiguous along the inner index
    const bool bpair = sRk == 1 && K >= 2;
    double ra0[kWaveKSteps][NA], rb0[kWaveKSteps][NB], ra1[kWaveKSteps][NA], rb1[kWaveKSteps][NB];
    auto load = [&](double (&ra)[kWaveKSteps][NA], double (&rb)[kWaveKSteps][NB], int k0) {
      const int kp = k0 + 2 * kr;
      if (apair) {
        const int s0 = min(kp, K - 2);
#pragma unroll
        for (int a = 0; a < NA; ++a) {
          const d2 v = *(gd2*)(L + aoff[a] + s0);
          ra[0][a] = v.x;
          ra[1][a] = v.y;
        }
      } else {
#pragma unroll
        for (int q = 0; q < kWaveKSteps; ++q) {
          const int kc = kp + q < K ? kp + q : 0;
#pragma unroll
          for (int a = 0; a < NA; ++a) ra[q][a] = L[aoff[a] + (int64_t)kc * sLk];
        }
      }
      if (bpair) {
        const int s0 = min(kp, K - 2);
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          const d2 v = *(gd2*)(R + boff[b] + s0);
          rb[0][b] = v.x;
          rb[1][b] = v.y;
        }
      } else {
#pragma unroll
        for (int q = 0; q < kWaveKSteps; ++q) {
          const int kc = kp + q < K ? kp + q : 0;
#pragma unroll
          for (int b = 0; b < NB; ++b) rb[q][b] = R[(int64_t)kc * sRk + boff[b]];
        }
      }
    };
    auto compute = [&](const double (&ra)[kWaveKSteps][NA], const double (&rb)[kWaveKSteps][NB],
                       int k0) {
      double av[kWaveKSteps][NA], bv[kWaveKSteps][NB];
      const int kp = k0 + 2 * kr;
      // a pair clamped to start at K - 2 holds the wanted index K - 1 second
      const bool shifted = kp == K - 1;
#pragma unroll
      for (int q = 0; q < kWaveKSteps; ++q) {
        const bool kv = kp + q < K;
#pragma unroll
        for (int a = 0; a < NA; ++a) {
          const double x = (q == 0 && apair && shifted) ? ra[1][a] : ra[q][a];
          av[q][a] = (kv & aval[a]) ? x * scale : 0.0;
        }
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          const double y = (q == 0 && bpair && shifted) ? rb[1][b] : rb[q][b];
          bv[q][b] = (kv & bval[b]) ? y : 0.0;
        }
      }
      if constexpr (!F32) {
#pragma unroll
        for (int q = 0; q < kWaveKSteps; ++q)
#pragma unroll
          for (int a = 0; a < NA; ++a)
#pragma unroll
            for (int b = 0; b < NB; ++b)
              acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[q][a], bv[q][b], acc[a][b], 0, 0, 0);
      } else {
        f4 p[NA][NB];
#pragma unroll
        for (int a = 0; a < NA; ++a)
#pragma unroll
          for (int b = 0; b < NB; ++b) p[a][b] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int q = 0; q < kWaveKSteps; ++q) {
          float ah[NA], bh[NB];
#pragma unroll
          for (int a = 0; a < NA; ++a) ah[a] = (float)av[q][a];
#pragma unroll
          for (int b = 0; b < NB; ++b) bh[b] = (float)bv[q][b];
#pragma unroll
          for (int a = 0; a < NA; ++a)
#pragma unroll
            for (int b = 0; b < NB; ++b) {
              p[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(ah[a], bh[b], p[a][b], 0, 0, 0);
              if constexpr (SPLIT) {
                const float al = (float)(av[q][a] - (double)ah[a]);
                const float bl = (float)(bv[q][b] - (double)bh[b]);
                p[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(ah[a], bl, p[a][b], 0, 0, 0);
                p[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(al, bh[b], p[a][b], 0, 0, 0);
              }
            }
        }
#pragma unroll
        for (int a = 0; a < NA; ++a)
#pragma unroll
          for (int b = 0; b < NB; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[a][b][v] += (double)p[a][b][v];
      }
    };
    // (the scheduling barriers keep the compiler from sinking the prefetch
    // next to its use, which it otherwise does under register pressure)
    if (K > 0) {
      load(ra0, rb0, 0);
      for (int k0 = 0;;) {
        load(ra1, rb1, k0 + G);
        __builtin_amdgcn_sched_barrier(0);
        compute(ra0, rb0, k0);
        k0 += G;
        if (k0 >= K) break;
        load(ra0, rb0, k0 + G);
        __builtin_amdgcn_sched_barrier(0);
        compute(ra1, rb1, k0);
        k0 += G;
        if (k0 >= K) break;
      }
    }
  }
  const double alpha = it.alpha;
#pragma unroll
  for (int a = 0; a < NA; ++a)
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const d4 fin = acc[a][b];
      const int j = 16 * b + lc;
      if (j >= it.n) continue;
      gdouble_mut* col = as_global_mut(it.C) + (int64_t)(it.col0 + j) * it.ldc + it.row0;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = 16 * a + (F32 ? 4 * kr + v : kr + 4 * v);
        if (i < it.m) {
          const double val = alpha * fin[v];
          col[i] = it.accumulate ? col[i] + val : val;
        }
      }
    }
}

template <bool F32, bool SPLIT, int NA>
__device__ __attribute__((always_inline)) inline void wave_nb(const GemmItem& it,
                                                              const Seg* __restrict__ segs,
                                                              int lane, int nb) {
  switch (nb) {
    case 1: wave_item<F32, SPLIT, NA, 1>(it, segs, lane); break;
    case 2: wave_item<F32, SPLIT, NA, 2>(it, segs, lane); break;
    case 3: wave_item<F32, SPLIT, NA, 3>(it, segs, lane); break;
    default: wave_item<F32, SPLIT, NA, 4>(it, segs, lane); break;
  }
}

template <bool F32, bool SPLIT>
__global__ __launch_bounds__(64 * kWaveItemsPerBlock, 2) void k_wgemm(const GemmItem* __restrict__ items,
                                                                  const Seg* __restrict__ segs,
                                                                  int nitems,
                                                                  const int* __restrict__ order,
                                                                  const int64_t* __restrict__ live) {
  if (live) nitems = uni((int)min((int64_t)nitems, *live));
  // Workgroups are dealt to the 8 XCDs round-robin; blk numbers the
  // workgroups of one XCD consecutively, so neighbouring slots (items that
  // share an operand block once ordered by it) run on one XCD's L2.
  const int blk = xcd_unit((nitems + kWaveItemsPerBlock - 1) / kWaveItemsPerBlock, live != nullptr);
  if (blk < 0) return;
  const int slot = blk * kWaveItemsPerBlock + uni((int)threadIdx.x >> 6);
  if (slot >= nitems) return;
  const int item = order ? uni(order[slot]) : slot;
  GemmItem it = items[item];
  it.m = uni(it.m);
  it.n = uni(it.n);
  it.row0 = uni(it.row0);
  it.col0 = uni(it.col0);
  it.seg0 = uni(it.seg0);
  it.nseg = uni(it.nseg);
  it.accumulate = uni(it.accumulate);
  it.ldc = uni64(it.ldc);
  if (it.m <= 0 || it.n <= 0) return;
  const int lane = threadIdx.x & 63;
  const int na = (it.m + 15) >> 4, nb = (it.n + 15) >> 4;   // <= kWaveTiles (planner)
  switch (na) {
    case 1: wave_nb<F32, SPLIT, 1>(it, segs, lane, nb); break;
    case 2: wave_nb<F32, SPLIT, 2>(it, segs, lane, nb); break;
    case 3: wave_nb<F32, SPLIT, 3>(it, segs, lane, nb); break;
    default: wave_nb<F32, SPLIT, 4>(it, segs, lane, nb); break;
  }
}

static inline int wave_grid(int nitems) {
  return xcd_grid((nitems + kWaveItemsPerBlock - 1) / kWaveItemsPerBlock);
}

}  // namespace clr
