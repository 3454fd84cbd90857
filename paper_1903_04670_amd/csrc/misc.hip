// Small utility kernels: NaN/Inf check.
#include <hip/hip_runtime.h>

#include "pipeline.hpp"

namespace dgfs {

__global__ void k_count_nonfinite(const double *x, int64_t n_nodes, int64_t n3, int64_t stride, unsigned int *count) {
  unsigned int bad = 0;
  const int64_t total = n_nodes * n3;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const double v = x[(i / n3) * stride + i % n3];
    bad += isfinite(v) ? 0u : 1u;
  }
  if (bad) atomicAdd(count, bad);
}

__global__ void k_zero_u32(unsigned int *p) { *p = 0u; }

dgfs_status check_finite(const double *x, int64_t n_nodes, int64_t n3, int64_t stride, hipStream_t st) {
  unsigned int *d = nullptr, h = 0;
  hipError_t e = hipMallocAsync((void **)&d, sizeof(unsigned int), st);
  if (e != hipSuccess) return hip_status(e, "DGFS_CHECK allocation");
  hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(1), 0, st, d);
  hipLaunchKernelGGL(k_count_nonfinite, dim3(1024), dim3(256), 0, st, x, n_nodes, n3, stride, d);
  e = hipMemcpyAsync(&h, d, sizeof(h), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  (void)hipFreeAsync(d, st);
  if (e != hipSuccess) return hip_status(e, "DGFS_CHECK");
  if (h) {
    set_error("DGFS_CHECK: %u non-finite values in the output", h);
    return DGFS_ENONFINITE;
  }
  return DGFS_OK;
}

}  // namespace dgfs
