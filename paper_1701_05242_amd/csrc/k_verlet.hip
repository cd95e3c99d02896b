// Velocity Verlet in FP64 (Section 2, Fig. 3 box 5):
//   kick  v += dt/(2m) F,   drift  x <- wrap(x + dt v),   kick again after F.
#include "dcm_device.hpp"
#include "dcm_internal.hpp"

namespace dcm {

__global__ __launch_bounds__(256) void k_kick(double *__restrict__ vx, double *__restrict__ vy,
                                              double *__restrict__ vz,
                                              const double *__restrict__ fx,
                                              const double *__restrict__ fy,
                                              const double *__restrict__ fz, int64_t n,
                                              double c) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    vx[i] = vx[i] + c * fx[i];
    vy[i] = vy[i] + c * fy[i];
    vz[i] = vz[i] + c * fz[i];
  }
}

__global__ __launch_bounds__(256) void k_kick_drift(
    double *__restrict__ x, double *__restrict__ y, double *__restrict__ z,
    double *__restrict__ vx, double *__restrict__ vy, double *__restrict__ vz,
    const double *__restrict__ fx, const double *__restrict__ fy, const double *__restrict__ fz,
    int64_t n, double c, double dt, double Lx, double Ly, double Lz) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    double a = vx[i] + c * fx[i];
    double b = vy[i] + c * fy[i];
    double d = vz[i] + c * fz[i];
    vx[i] = a;
    vy[i] = b;
    vz[i] = d;
    x[i] = wrap_coord(x[i] + dt * a, Lx);
    y[i] = wrap_coord(y[i] + dt * b, Ly);
    z[i] = wrap_coord(z[i] + dt * d, Lz);
  }
}

// The closing kick of one step and the opening kick and drift of the next
// in one pass over the particles: the same operations in the same order as
// k_kick followed by k_kick_drift, without the round trip of v through HBM.
__global__ __launch_bounds__(256) void k_kick_kick_drift(
    double *__restrict__ x, double *__restrict__ y, double *__restrict__ z,
    double *__restrict__ vx, double *__restrict__ vy, double *__restrict__ vz,
    const double *__restrict__ fx, const double *__restrict__ fy, const double *__restrict__ fz,
    int64_t n, double c, double dt, double Lx, double Ly, double Lz) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double gx = c * fx[i], gy = c * fy[i], gz = c * fz[i];
    const double a = (vx[i] + gx) + gx;
    const double b = (vy[i] + gy) + gy;
    const double d = (vz[i] + gz) + gz;
    vx[i] = a;
    vy[i] = b;
    vz[i] = d;
    x[i] = wrap_coord(x[i] + dt * a, Lx);
    y[i] = wrap_coord(y[i] + dt * b, Ly);
    z[i] = wrap_coord(z[i] + dt * d, Lz);
  }
}

// The same, and the density binning of the next step's detection (Section
// 2.1) from the new positions while they are in registers: counts[v] += 1
// for the voxel v of each particle, as the binning pass computes it (the
// positions written here are wrapped already, and wrapping them again gives
// them back unchanged).  A non-finite position is flagged and not binned.
// Uniform trip count: every lane of a wavefront reaches the aggregated add.
__global__ __launch_bounds__(256) void k_kick_kick_drift_bin(
    double *__restrict__ x, double *__restrict__ y, double *__restrict__ z,
    double *__restrict__ vx, double *__restrict__ vy, double *__restrict__ vz,
    const double *__restrict__ fx, const double *__restrict__ fy, const double *__restrict__ fz,
    int64_t n, double c, double dt, double Lx, double Ly, double Lz, int nx, int ny, int nz,
    double sx, double sy, double sz, uint32_t *counts, uint32_t *status) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t base = blockIdx.x * (int64_t)blockDim.x; base < n; base += stride) {
    const int64_t i = base + threadIdx.x;
    bool valid = i < n;
    uint32_t vox = 0;
    if (valid) {
      const double gx = c * fx[i], gy = c * fy[i], gz = c * fz[i];
      const double a = (vx[i] + gx) + gx;
      const double b = (vy[i] + gy) + gy;
      const double d = (vz[i] + gz) + gz;
      vx[i] = a;
      vy[i] = b;
      vz[i] = d;
      const double px = wrap_coord(x[i] + dt * a, Lx);
      const double py = wrap_coord(y[i] + dt * b, Ly);
      const double pz = wrap_coord(z[i] + dt * d, Lz);
      x[i] = px;
      y[i] = py;
      z[i] = pz;
      if (!finite3(px, py, pz)) {
        atomicOr(status, ST_NONFINITE_POS);
        valid = false;
      } else {
        const int cx = slab_index(wrap_coord(px, Lx), sx, nx);
        const int cy = slab_index(wrap_coord(py, Ly), sy, ny);
        const int cz = slab_index(wrap_coord(pz, Lz), sz, nz);
        vox = (uint32_t)(((int64_t)cz * ny + cy) * nx + cx);
      }
    }
    wave_run_add(counts, vox, valid);
  }
}

static unsigned grid_for(int64_t n) {
  int64_t b = ceil_div(n, 256);
  if (b < 1) b = 1;
  if (b > 16384) b = 16384;
  return (unsigned)b;
}

void launch_kick(hipStream_t s, double *vx, double *vy, double *vz, const double *fx,
                 const double *fy, const double *fz, int64_t n, double c) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_kick, dim3(grid_for(n)), dim3(256), 0, s, vx, vy, vz, fx, fy, fz, n, c);
}

void launch_kick_drift(hipStream_t s, double *x, double *y, double *z, double *vx, double *vy,
                       double *vz, const double *fx, const double *fy, const double *fz,
                       int64_t n, double c, double dt, const double L[3]) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_kick_drift, dim3(grid_for(n)), dim3(256), 0, s, x, y, z, vx, vy, vz, fx,
                     fy, fz, n, c, dt, L[0], L[1], L[2]);
}

void launch_kick_kick_drift(hipStream_t s, double *x, double *y, double *z, double *vx,
                            double *vy, double *vz, const double *fx, const double *fy,
                            const double *fz, int64_t n, double c, double dt, const double L[3]) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_kick_kick_drift, dim3(grid_for(n)), dim3(256), 0, s, x, y, z, vx, vy, vz,
                     fx, fy, fz, n, c, dt, L[0], L[1], L[2]);
}

void launch_kick_kick_drift_bin(hipStream_t s, double *x, double *y, double *z, double *vx,
                                double *vy, double *vz, const double *fx, const double *fy,
                                const double *fz, int64_t n, double c, double dt,
                                const double L[3], const int32_t nv[3], const double sc[3],
                                uint32_t *counts, uint32_t *status) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_kick_kick_drift_bin, dim3(grid_for(n)), dim3(256), 0, s, x, y, z, vx, vy,
                     vz, fx, fy, fz, n, c, dt, L[0], L[1], L[2], nv[0], nv[1], nv[2], sc[0],
                     sc[1], sc[2], counts, status);
}

// Kinetic energy sum_i m v_i^2 / 2: fixed-size grid of block partials, then
// one workgroup sums them in a fixed order.
constexpr int kKeBlocks = 1024;
int64_t kinetic_blocks(int64_t n) {
  (void)n;
  return kKeBlocks;
}

__global__ __launch_bounds__(256) void k_kinetic_partial(const double *__restrict__ vx,
                                                         const double *__restrict__ vy,
                                                         const double *__restrict__ vz,
                                                         int64_t n, double *partials) {
  double acc = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    acc += (vx[i] * vx[i] + vy[i] * vy[i]) + vz[i] * vz[i];
  __shared__ double red[4];
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) partials[blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
}

__global__ __launch_bounds__(256) void k_kinetic_final(const double *__restrict__ partials,
                                                       int64_t blocks, double half_m,
                                                       double *out) {
  double acc = 0.0;
  for (int64_t b = threadIdx.x; b < blocks; b += 256) acc += partials[b];
  __shared__ double red[4];
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) *out = half_m * (((red[0] + red[1]) + red[2]) + red[3]);
}

void launch_kinetic(hipStream_t s, const double *vx, const double *vy, const double *vz,
                    int64_t n, double mass, double *partials, int64_t blocks, double *out) {
  hipLaunchKernelGGL(k_kinetic_partial, dim3((unsigned)blocks), dim3(256), 0, s, vx, vy, vz, n,
                     partials);
  hipLaunchKernelGGL(k_kinetic_final, dim3(1), dim3(256), 0, s, partials, blocks, 0.5 * mass,
                     out);
}

}  // namespace dcm
