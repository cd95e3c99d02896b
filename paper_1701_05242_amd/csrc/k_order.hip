// Particle-order kernels for the stepping loop: dcm_step keeps its working
// copies of positions, velocities, forces and cutoffs in cell order (so every
// per-particle kernel reads memory nearly sequentially) and maps them back to
// the caller's order only when it returns.
#include "dcm_device.hpp"
#include "dcm_internal.hpp"

namespace dcm {

__global__ __launch_bounds__(256) void k_iota(int32_t *__restrict__ p, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = (int32_t)i;
}

// dst_k[s] = src_k[perm[s]] for every field, and the caller index carried
// along: owner_dst[s] = owner_src[perm[s]].
__global__ __launch_bounds__(256) void k_permute_gather(PermFields f,
                                                        const int32_t *__restrict__ perm,
                                                        const int32_t *__restrict__ owner_src,
                                                        int32_t *__restrict__ owner_dst,
                                                        int64_t n) {
  for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < n;
       s += (int64_t)gridDim.x * blockDim.x) {
    const int32_t p = perm[s];
#pragma unroll
    for (int k = 0; k < kPermFields; ++k)
      if (k < f.nf) f.dst[k][s] = f.src[k][p];
    owner_dst[s] = owner_src[p];
  }
}

// dst_k[owner[s]] = src_k[s]: back to the caller's order.
__global__ __launch_bounds__(256) void k_permute_scatter(PermFields f,
                                                         const int32_t *__restrict__ owner,
                                                         int64_t n) {
  for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < n;
       s += (int64_t)gridDim.x * blockDim.x) {
    const int32_t q = owner[s];
#pragma unroll
    for (int k = 0; k < kPermFields; ++k)
      if (k < f.nf) f.dst[k][q] = f.src[k][s];
  }
}

static unsigned grid_for(int64_t n) {
  int64_t b = ceil_div(n, 256);
  if (b < 1) b = 1;
  if (b > 16384) b = 16384;
  return (unsigned)b;
}

void launch_iota(hipStream_t s, int32_t *p, int64_t n) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_iota, dim3(grid_for(n)), dim3(256), 0, s, p, n);
}

void launch_permute_gather(hipStream_t s, const PermFields &f, const int32_t *perm,
                           const int32_t *owner_src, int32_t *owner_dst, int64_t n) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_permute_gather, dim3(grid_for(n)), dim3(256), 0, s, f, perm, owner_src,
                     owner_dst, n);
}

void launch_permute_scatter(hipStream_t s, const PermFields &f, const int32_t *owner,
                            int64_t n) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_permute_scatter, dim3(grid_for(n)), dim3(256), 0, s, f, owner, n);
}

}  // namespace dcm
