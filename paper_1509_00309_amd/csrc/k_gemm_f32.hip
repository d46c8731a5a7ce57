// Mixed-form (FP32 MFMA, FP64 accumulation) instantiations of the grouped
// block-product GEMM (k_gemm.h).
#include "k_gemm.h"

namespace clr {

hipError_t launch_ggemm_f32(const GemmItem* items, const Seg* segs, int nitems, int split,
                            hipStream_t s, bool dense, const int* order, const int64_t* live,
                            int* next) {
  if (nitems <= 0) return hipSuccess;
  const dim3 grid(next ? persistent_grid(nitems) : xcd_grid(nitems)), block(kLdsGemmThreads);
  if (split && dense)
    hipLaunchKernelGGL((k_ggemm<true, true, true>), grid, block, 0, s, items, segs, nitems, order,
                       live, next);
  else if (split)
    hipLaunchKernelGGL((k_ggemm<true, true, false>), grid, block, 0, s, items, segs, nitems, order,
                       live, next);
  else if (dense)
    hipLaunchKernelGGL((k_ggemm<true, false, true>), grid, block, 0, s, items, segs, nitems, order,
                       live, next);
  else
    hipLaunchKernelGGL((k_ggemm<true, false, false>), grid, block, 0, s, items, segs, nitems, order,
                       live, next);
  return hipGetLastError();
}

hipError_t launch_wgemm_f32(const GemmItem* items, const Seg* segs, int nitems, int split,
                            hipStream_t s, const int* order, const int64_t* live) {
  if (nitems <= 0) return hipSuccess;
  const dim3 grid(wave_grid(nitems)), block(64 * kWaveItemsPerBlock);
  if (split)
    hipLaunchKernelGGL((k_wgemm<true, true>), grid, block, 0, s, items, segs, nitems, order, live);
  else
    hipLaunchKernelGGL((k_wgemm<true, false>), grid, block, 0, s, items, segs, nitems, order, live);
  return hipGetLastError();
}

}  // namespace clr
