// FP64 instantiations of the grouped block-product GEMM (k_gemm.h).
#include "k_gemm.h"

namespace clr {

hipError_t launch_ggemm_f64(const GemmItem* items, const Seg* segs, int nitems, hipStream_t s,
                            bool dense, const int* order, const int64_t* live) {
  if (nitems <= 0) return hipSuccess;
  if (dense)
    hipLaunchKernelGGL((k_ggemm<false, false, true>), dim3(xcd_grid(nitems)),
                       dim3(kLdsGemmThreads), 0, s, items, segs, nitems, order, live);
  else
    hipLaunchKernelGGL((k_ggemm<false, false, false>), dim3(xcd_grid(nitems)),
                       dim3(kLdsGemmThreads), 0, s, items, segs, nitems, order, live);
  return hipGetLastError();
}

hipError_t launch_wgemm_f64(const GemmItem* items, const Seg* segs, int nitems, hipStream_t s,
                            const int* order, const int64_t* live) {
  if (nitems <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_wgemm<false, false>), dim3(wave_grid(nitems)),
                     dim3(64 * kWaveItemsPerBlock), 0, s, items, segs, nitems, order, live);
  return hipGetLastError();
}

}  // namespace clr
