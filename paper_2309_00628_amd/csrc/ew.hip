// Element-wise block kernels: one launch processes an array of parts
// (blocks of possibly different shape and recipe, ew_body.h); the block
// index selects the part.
#include <hip/hip_runtime.h>

#include "desc.h"
#include "ew_body.h"
#include "kernels.h"

namespace mm {

namespace {

using namespace ew_detail;

template <typename T>
__global__ __launch_bounds__(kThreads) void ew_kernel(KernelBases kb, const EwPart* __restrict__ parts,
                                                      int nparts) {
  const int b = blockIdx.x;
  int lo = 0, hi = nparts - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (parts[mid].blk_start <= b) lo = mid; else hi = mid - 1;
  }
  ew_block<T>(kb, parts[lo], b - parts[lo].blk_start, threadIdx.x);
}

}  // namespace

int ew_blocks(int rows, int cols, int dtype) {
  const int V = dtype == DT_F64 ? 2 : 4;
  const int64_t cpr = (cols + V - 1) / V;
  const int64_t chunks = (int64_t)rows * cpr;
  return (int)((chunks + kThreads * kItems - 1) / (kThreads * kItems));
}

hipError_t launch_ew(int dtype, const KernelBases& kb, const EwPart* dparts, int nparts, int blocks,
                     hipStream_t s) {
  if (blocks <= 0) return hipSuccess;
  if (dtype == DT_F64)
    hipLaunchKernelGGL(ew_kernel<double>, dim3(blocks), dim3(kThreads), 0, s, kb, dparts, nparts);
  else
    hipLaunchKernelGGL(ew_kernel<float>, dim3(blocks), dim3(kThreads), 0, s, kb, dparts, nparts);
  return hipGetLastError();
}

}  // namespace mm
