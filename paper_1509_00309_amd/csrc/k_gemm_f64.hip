// FP64 instantiations of the grouped block-product GEMM (k_gemm.h).
#include "k_gemm.h"

namespace clr {

int persistent_grid(int nitems, int per_cu) {
  static int cus = 0;
  if (cus == 0) {
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && n > 0)
      cus = n;
    else
      cus = 256;
  }
  const int64_t g = (int64_t)cus * per_cu;
  return nitems < g ? nitems : (int)g;
}

hipError_t launch_ggemm_f64(const GemmItem* items, const Seg* segs, int nitems, hipStream_t s,
                            bool dense, const int* order, const int64_t* live, int* next) {
  if (nitems <= 0) return hipSuccess;
  const dim3 grid(next ? persistent_grid(nitems) : xcd_grid(nitems));
  if (dense)
    hipLaunchKernelGGL((k_ggemm<false, false, true>), grid, dim3(kLdsGemmThreads), 0, s, items,
                       segs, nitems, order, live, next);
  else
    hipLaunchKernelGGL((k_ggemm<false, false, false>), grid, dim3(kLdsGemmThreads), 0, s, items,
                       segs, nitems, order, live, next);
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
