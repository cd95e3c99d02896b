// Bubble filter of the interface detection (Section 2.1): connected
// components of either phase smaller than a given volume take the other
// phase.  Components are 6-connected with periodic neighbours.
//
// Labels come from a lock-free union-find over voxel indices: every voxel
// starts as its own root, each voxel unites with its +x, +y and +z neighbour
// of the same phase (a root is hooked under the smaller of the two roots
// with a compare-and-swap), and a last pass points every voxel at its root,
// the smallest voxel index of its component.  Parent indices only ever
// point to smaller indices, so every walk up the tree ends, and a failed
// hook always continues from a smaller root.
#include "dcm_device.hpp"
#include "dcm_internal.hpp"

namespace dcm {

// Root of x, halving the path on the way (a non-root is pointed at its
// grandparent, still an ancestor in the same set).
__device__ __forceinline__ int ccl_find(int32_t *lab, int x) {
  int p = lab[x];
  while (p != x) {
    const int gp = lab[p];
    if (gp != p) lab[x] = gp;
    x = p;
    p = gp;
  }
  return x;
}

__device__ __forceinline__ void ccl_unite(int32_t *lab, int a, int b, uint32_t *status) {
  int ra = ccl_find(lab, a), rb = ccl_find(lab, b);
  // every failed hook moves to a strictly smaller root, so this ends long
  // before the bound; the bound only guards the invariant
  for (int it = 0; ra != rb; ++it) {
    if (it > (1 << 30)) {
      atomicOr(status, ST_NOT_CONVERGED);
      return;
    }
    if (ra < rb) {
      const int t = ra;
      ra = rb;
      rb = t;
    }
    const int old = atomicCAS(&lab[ra], ra, rb);
    if (old == ra) return;
    ra = ccl_find(lab, old);
    rb = ccl_find(lab, rb);
  }
}

__global__ __launch_bounds__(256) void k_ccl_init(int32_t *__restrict__ lab, int nvox) {
  for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < nvox; v += gridDim.x * blockDim.x)
    lab[v] = v;
}

__global__ __launch_bounds__(256) void k_ccl_union(const uint8_t *__restrict__ seg, int32_t *lab,
                                                   int nx, int ny, int nz, uint32_t *status) {
  const int nvox = nx * ny * nz;
  for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < nvox; v += gridDim.x * blockDim.x) {
    const int x = v % nx, r = v / nx;
    const int y = r % ny, z = r / ny;
    const uint8_t p = seg[v];
    const int ux = (x + 1 == nx ? 0 : x + 1) + r * nx;
    const int uy = ((z * ny) + (y + 1 == ny ? 0 : y + 1)) * nx + x;
    const int uz = (((z + 1 == nz ? 0 : z + 1) * ny) + y) * nx + x;
    if (ux != v && seg[ux] == p) ccl_unite(lab, v, ux, status);
    if (uy != v && seg[uy] == p) ccl_unite(lab, v, uy, status);
    if (uz != v && seg[uz] == p) ccl_unite(lab, v, uz, status);
  }
}

// Root of x without writing on the way: once no hooks happen, a walk that
// reads a parent, or a root another thread has just stored, still ends at
// the root.  (Halving here would race with those stores: a walk through x
// could overwrite x's stored root with an older ancestor.)
__device__ __forceinline__ int ccl_root(const int32_t *lab, int x) {
  int p = lab[x];
  while (p != x) {
    x = p;
    p = lab[x];
  }
  return x;
}

__global__ __launch_bounds__(256) void k_ccl_flatten(int32_t *lab, int nvox) {
  for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < nvox; v += gridDim.x * blockDim.x)
    lab[v] = ccl_root(lab, v);
}

// Voxels per component, counted only up to min_volume: runs of equal labels
// in a wavefront add their length with one atomic, and a run whose component
// already has min_volume voxels adds nothing (the count can only grow, so a
// component reaches min_volume exactly when it has that many voxels).
__global__ __launch_bounds__(256) void k_ccl_sizes(const int32_t *__restrict__ lab, int nvox,
                                                   int32_t *size, int32_t min_volume) {
  const int stride = gridDim.x * blockDim.x;
  for (int base = blockIdx.x * blockDim.x; base < nvox; base += stride) {
    const int v = base + threadIdx.x;
    const bool valid = v < nvox;
    const uint32_t key = valid ? (uint32_t)lab[v] : 0u;
    const int lane = threadIdx.x & 63;
    unsigned long long vmask;
    const unsigned long long heads = wave_run_heads(key, valid, vmask);
    if ((heads >> lane) & 1ull) {
      if (*(volatile int32_t *)&size[key] < min_volume)
        atomicAdd(&size[key], wave_run_len(lane, heads, vmask));
    }
  }
}

// Flip the voxels of small components; then the interface of the new map.
__global__ __launch_bounds__(256) void k_ccl_flip(const int32_t *__restrict__ lab,
                                                  const int32_t *__restrict__ size, int nvox,
                                                  int32_t min_volume, uint8_t *seg) {
  for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < nvox; v += gridDim.x * blockDim.x)
    if (size[lab[v]] < min_volume) seg[v] = (uint8_t)(1 - seg[v]);
}

__global__ __launch_bounds__(256) void k_iface_bytes(const uint8_t *__restrict__ seg, int nx,
                                                     int ny, int nz, uint8_t *__restrict__ iface) {
  const int nvox = nx * ny * nz;
  for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < nvox; v += gridDim.x * blockDim.x) {
    const int x = v % nx, r = v / nx;
    const int y = r % ny, z = r / ny;
    uint8_t f = 0;
    if (seg[v]) {
      const int xm = x == 0 ? nx - 1 : x - 1, xp = x + 1 == nx ? 0 : x + 1;
      const int ym = y == 0 ? ny - 1 : y - 1, yp = y + 1 == ny ? 0 : y + 1;
      const int zm = z == 0 ? nz - 1 : z - 1, zp = z + 1 == nz ? 0 : z + 1;
      f = !seg[r * nx + xm] || !seg[r * nx + xp] || !seg[(z * ny + ym) * nx + x] ||
          !seg[(z * ny + yp) * nx + x] || !seg[(zm * ny + y) * nx + x] ||
          !seg[(zp * ny + y) * nx + x];
    }
    iface[v] = f;
  }
}

static unsigned ccl_grid(int64_t nvox) {
  int64_t b = ceil_div(nvox, 256);
  if (b < 1) b = 1;
  if (b > 16384) b = 16384;
  return (unsigned)b;
}

void launch_bubble_filter(hipStream_t s, const int32_t nv[3], int64_t min_volume, uint8_t *seg,
                          uint8_t *iface, int32_t *label, int32_t *size, uint32_t *status) {
  const int64_t nvox = (int64_t)nv[0] * nv[1] * nv[2];
  const unsigned g = ccl_grid(nvox);
  const int32_t mv = (int32_t)min_volume;
  hipLaunchKernelGGL(k_ccl_init, dim3(g), dim3(256), 0, s, label, (int)nvox);
  hipLaunchKernelGGL(k_ccl_union, dim3(g), dim3(256), 0, s, seg, label, nv[0], nv[1], nv[2],
                     status);
  hipLaunchKernelGGL(k_ccl_flatten, dim3(g), dim3(256), 0, s, label, (int)nvox);
  launch_fill_i32(s, size, 0, nvox);
  hipLaunchKernelGGL(k_ccl_sizes, dim3(g), dim3(256), 0, s, label, (int)nvox, size, mv);
  hipLaunchKernelGGL(k_ccl_flip, dim3(g), dim3(256), 0, s, label, size, (int)nvox, mv, seg);
  hipLaunchKernelGGL(k_iface_bytes, dim3(g), dim3(256), 0, s, seg, nv[0], nv[1], nv[2], iface);
}

}  // namespace dcm
