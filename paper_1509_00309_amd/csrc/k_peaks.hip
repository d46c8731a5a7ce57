// Measured ceilings of the two resources the product's kernels are bound by:
// the FP64 matrix pipe (a long chain of independent v_mfma_f64_16x16x4 per
// wave, operands in registers) and HBM (a device-to-device copy of a buffer
// far larger than the caches).  They are quoted next to the datasheet peaks
// so that roofline fractions can be read against what the chip sustains.
#include "clr_internal.h"

namespace clr {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
constexpr int kPeakAcc = 8;   // independent accumulators per wave (hides the MFMA latency)

__global__ __launch_bounds__(256) void k_mfma_f64_loop(int iters, double* __restrict__ sink) {
  const int lane = threadIdx.x & 63;
  double a = 1.0 + 1e-3 * lane, b = 1.0 - 1e-3 * lane;
  d4 acc[kPeakAcc];
#pragma unroll
  for (int t = 0; t < kPeakAcc; ++t) acc[t] = d4{0.0, 0.0, 0.0, 0.0};
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int t = 0; t < kPeakAcc; ++t) acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[t], 0, 0, 0);
  }
  // The accumulators leave through one more MFMA (+ 0 * 0): with only MFMA
  // users, the compiler keeps them in accumulation registers for the whole
  // loop instead of copying them between register files every iteration.
  double s = 0.0;
#pragma unroll
  for (int t = 0; t < kPeakAcc; ++t) {
    const d4 fin = __builtin_amdgcn_mfma_f64_16x16x4f64(0.0, 0.0, acc[t], 0, 0, 0);
    s += fin[0] + fin[1] + fin[2] + fin[3];
  }
  // a value the compiler cannot drop; written by one lane of one wave only
  if (blockIdx.x == 0 && threadIdx.x == 0) sink[0] = s;
}

__global__ __launch_bounds__(256) void k_copy_d2(const double2* __restrict__ src,
                                                 double2* __restrict__ dst, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    dst[i] = src[i];
}

}  // namespace

// flops of one k_mfma_f64_loop launch: waves * iters * kPeakAcc * 2 * 16 * 16 * 4
double mfma_loop_flops(int blocks, int iters) {
  return (double)blocks * 4.0 * iters * kPeakAcc * 2.0 * 16 * 16 * 4;
}

hipError_t launch_mfma_loop(int blocks, int iters, double* sink, hipStream_t s) {
  hipLaunchKernelGGL(k_mfma_f64_loop, dim3(blocks), dim3(256), 0, s, iters, sink);
  return hipGetLastError();
}

hipError_t launch_copy(const double* src, double* dst, int64_t n_doubles, hipStream_t s) {
  const int64_t n2 = n_doubles / 2;
  hipLaunchKernelGGL(k_copy_d2, dim3(8192), dim3(256), 0, s, (const double2*)src, (double2*)dst, n2);
  return hipGetLastError();
}

}  // namespace clr
