// Small utility kernels: fills (used instead of hipMemsetAsync so that every
// stage stays safe to capture in a HIP graph), control-block reset and the
// status clear.
#include "dcm_internal.hpp"

namespace dcm {

__global__ void k_fill_u32(uint32_t *p, uint32_t v, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void k_fill_i32(int32_t *p, int32_t v, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void k_fill_u64(unsigned long long *p, unsigned long long v, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void k_reset_ctl(Ctl *ctl) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    Ctl c = {};
    *ctl = c;
  }
}

__global__ void k_clear_status(uint32_t *st) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *st = 0u;
}

static int fill_grid(int64_t n) {
  int64_t b = ceil_div(n, 256);
  if (b < 1) b = 1;
  if (b > 4096) b = 4096;
  return (int)b;
}

void launch_fill_u32(hipStream_t s, uint32_t *p, uint32_t v, int64_t n) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill_u32, dim3(fill_grid(n)), dim3(256), 0, s, p, v, n);
}

void launch_fill_i32(hipStream_t s, int32_t *p, int32_t v, int64_t n) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill_i32, dim3(fill_grid(n)), dim3(256), 0, s, p, v, n);
}

void launch_fill_u64(hipStream_t s, unsigned long long *p, unsigned long long v, int64_t n) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill_u64, dim3(fill_grid(n)), dim3(256), 0, s, p, v, n);
}

void launch_reset_ctl(hipStream_t s, Ctl *ctl) {
  hipLaunchKernelGGL(k_reset_ctl, dim3(1), dim3(64), 0, s, ctl);
}

void launch_clear_status(hipStream_t s, uint32_t *st) {
  hipLaunchKernelGGL(k_clear_status, dim3(1), dim3(64), 0, s, st);
}

}  // namespace dcm
