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

__global__ void k_zero2_i32(int32_t *p, int32_t *q, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    p[i] = 0;
    q[i] = 0;
  }
}

__global__ void k_zero2_u32(uint32_t *p, int64_t np, uint32_t *q, int64_t nq) {
  const int64_t n = np > nq ? np : nq;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    if (i < np) p[i] = 0u;
    if (i < nq) q[i] = 0u;
  }
}

void launch_zero2_u32(hipStream_t s, uint32_t *p, int64_t np, uint32_t *q, int64_t nq) {
  const int64_t n = np > nq ? np : nq;
  if (n <= 0) return;
  hipLaunchKernelGGL(k_zero2_u32, dim3(fill_grid(n)), dim3(256), 0, s, p, np, q, nq);
}

void launch_zero2_i32(hipStream_t s, int32_t *p, int32_t *q, int64_t n) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_zero2_i32, dim3(fill_grid(n)), dim3(256), 0, s, p, q, n);
}

void launch_fill_i32(hipStream_t s, int32_t *p, int32_t v, int64_t n) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill_i32, dim3(fill_grid(n)), dim3(256), 0, s, p, v, n);
}

void launch_fill_u64(hipStream_t s, unsigned long long *p, unsigned long long v, int64_t n) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill_u64, dim3(fill_grid(n)), dim3(256), 0, s, p, v, n);
}

// Smallest finite non-negative value of v[0..n) into *out (+inf if none):
// one workgroup, for the one-off reductions of the cell-edge tuner.
__global__ __launch_bounds__(1024) void k_min_f64(const double *__restrict__ v, int64_t n,
                                                  double *out) {
  __shared__ double wmin[16];
  double m = __builtin_huge_val();
  for (int64_t i = threadIdx.x; i < n; i += 1024) {
    const double x = v[i];
    if (x >= 0.0 && x < m) m = x;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const double o = __shfl_xor(m, off, 64);
    m = o < m ? o : m;
  }
  if ((threadIdx.x & 63) == 0) wmin[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < 16; ++w) m = wmin[w] < m ? wmin[w] : m;
    m = wmin[0] < m ? wmin[0] : m;
    *out = m;
  }
}

void launch_min_f64(hipStream_t s, const double *v, int64_t n, double *out) {
  hipLaunchKernelGGL(k_min_f64, dim3(1), dim3(1024), 0, s, v, n, out);
}

void launch_reset_ctl(hipStream_t s, Ctl *ctl) {
  hipLaunchKernelGGL(k_reset_ctl, dim3(1), dim3(64), 0, s, ctl);
}

void launch_clear_status(hipStream_t s, uint32_t *st) {
  hipLaunchKernelGGL(k_clear_status, dim3(1), dim3(64), 0, s, st);
}

}  // namespace dcm
