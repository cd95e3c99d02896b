// Cutoff assignment (Section 2.2) and linked-cell binning (Section 2.3).
#include "dcm_device.hpp"
#include "dcm_internal.hpp"

namespace dcm {

// ----------------------------------------------------- cutoff assignment
// delta_i: periodic trilinear interpolation of the voxel-centred distances at
// the particle; rc_i = rc_max - (rc_max - rc_min) * min(delta_i/ramp, 1).
__global__ __launch_bounds__(256) void k_assign_cutoffs(
    const double *__restrict__ x, const double *__restrict__ y, const double *__restrict__ z,
    int64_t n, double Lx, double Ly, double Lz, int nx, int ny, int nz, double sx, double sy,
    double sz, const double *__restrict__ D, double rc_min, double rc_max, double ramp,
    double *__restrict__ delta, double *__restrict__ rc) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n;
       p += (int64_t)gridDim.x * blockDim.x) {
    double px = x[p], py = y[p], pz = z[p];
    if (!finite3(px, py, pz)) {
      if (delta) delta[p] = __builtin_nan("");
      rc[p] = rc_max;
      continue;
    }
    const double pos[3] = {wrap_coord(px, Lx), wrap_coord(py, Ly), wrap_coord(pz, Lz)};
    const double sc[3] = {sx, sy, sz};
    const int nn[3] = {nx, ny, nz};
    int i0[3], i1[3];
    double t[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      double u = pos[a] * sc[a] - 0.5;
      double f = floor(u);
      t[a] = u - f;
      int ia = (int)f;  // f lies in [-1, n)
      i0[a] = wrap_index(ia, nn[a]);
      i1[a] = wrap_index(ia + 1, nn[a]);
    }
    auto DV = [&](int i, int j, int k) { return D[((int64_t)k * ny + j) * nx + i]; };
    double wx0 = 1.0 - t[0], wx1 = t[0];
    double wy0 = 1.0 - t[1], wy1 = t[1];
    double wz0 = 1.0 - t[2], wz1 = t[2];
    double c00 = DV(i0[0], i0[1], i0[2]) * wx0 + DV(i1[0], i0[1], i0[2]) * wx1;
    double c10 = DV(i0[0], i1[1], i0[2]) * wx0 + DV(i1[0], i1[1], i0[2]) * wx1;
    double c01 = DV(i0[0], i0[1], i1[2]) * wx0 + DV(i1[0], i0[1], i1[2]) * wx1;
    double c11 = DV(i0[0], i1[1], i1[2]) * wx0 + DV(i1[0], i1[1], i1[2]) * wx1;
    double c0 = c00 * wy0 + c10 * wy1;
    double c1 = c01 * wy0 + c11 * wy1;
    double d = c0 * wz0 + c1 * wz1;
    if (delta) delta[p] = d;
    double q = d / ramp;
    if (q > 1.0) q = 1.0;
    rc[p] = rc_max - (rc_max - rc_min) * q;
  }
}

void launch_assign_cutoffs(hipStream_t s, const double *x, const double *y, const double *z,
                           int64_t n, const double L[3], const int32_t nv[3],
                           const double sc[3], const double *dist, dcm_rule rule,
                           double *delta, double *rc) {
  if (n <= 0) return;
  int64_t b = ceil_div(n, 256);
  if (b > 16384) b = 16384;
  hipLaunchKernelGGL(k_assign_cutoffs, dim3((unsigned)b), dim3(256), 0, s, x, y, z, n, L[0],
                     L[1], L[2], nv[0], nv[1], nv[2], sc[0], sc[1], sc[2], dist, rule.rc_min,
                     rule.rc_max, rule.ramp, delta, rc);
}

// ------------------------------------------------------------ cell count
__global__ __launch_bounds__(256) void k_cell_count(
    const double *__restrict__ x, const double *__restrict__ y, const double *__restrict__ z,
    const double *__restrict__ rc, int64_t n, double Lx, double Ly, double Lz, int nx, int ny,
    int nz, double sx, double sy, double sz, double rc_cap, int32_t *__restrict__ cell_of,
    int32_t *count, Ctl *ctl, uint32_t *status) {
  unsigned long long rmax = 0;
  // uniform trip count: every lane reaches the run-aggregated atomic
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t base = blockIdx.x * (int64_t)blockDim.x; base < n; base += stride) {
    const int64_t i = base + threadIdx.x;
    const bool valid = i < n;
    int c = 0;
    if (valid) {
      double px = x[i], py = y[i], pz = z[i], r = rc[i];
      if (finite3(px, py, pz)) {
        int cx = slab_index(wrap_coord(px, Lx), sx, nx);
        int cy = slab_index(wrap_coord(py, Ly), sy, ny);
        int cz = slab_index(wrap_coord(pz, Lz), sz, nz);
        c = (cz * ny + cy) * nx + cx;
      } else {
        atomicOr(status, ST_NONFINITE_POS);
      }
      // rc_cap: the build's bound on every cutoff (inclusive, below L/2)
      if (!(r >= 0.0) || r > rc_cap) {
        atomicOr(status, ST_RC_RANGE);
        r = (r > rc_cap) ? rc_cap : 0.0;
      }
      unsigned long long bits = (unsigned long long)__double_as_longlong(r);
      rmax = bits > rmax ? bits : rmax;
      cell_of[i] = c;
    }
    wave_run_add(count, (uint32_t)c, valid);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    unsigned long long o = __shfl_xor(rmax, off, 64);
    rmax = o > rmax ? o : rmax;
  }
  // most waves hold no new maximum: look before taking the atomic
  if ((threadIdx.x & 63) == 0 && rmax > *(volatile unsigned long long *)&ctl->rc_max_bits)
    atomicMax(&ctl->rc_max_bits, rmax);
}

__global__ void k_reset_rcmax(Ctl *ctl) {
  if (threadIdx.x == 0 && blockIdx.x == 0) ctl->rc_max_bits = 0ull;
}

void launch_cell_count(hipStream_t s, const double *x, const double *y, const double *z,
                       const double *rc, int64_t n, const double L[3], const int32_t nc[3],
                       const double sc[3], double rc_cap, int32_t *cell_of, int32_t *cell_count,
                       Ctl *ctl, uint32_t *status) {
  hipLaunchKernelGGL(k_reset_rcmax, dim3(1), dim3(64), 0, s, ctl);
  if (n <= 0) return;
  int64_t b = ceil_div(n, 256);
  if (b > 16384) b = 16384;
  hipLaunchKernelGGL(k_cell_count, dim3((unsigned)b), dim3(256), 0, s, x, y, z, rc, n, L[0],
                     L[1], L[2], nc[0], nc[1], nc[2], sc[0], sc[1], sc[2], rc_cap, cell_of,
                     cell_count, ctl, status);
}

// ------------------------------------------------------- exclusive scan
// Three phases over tiles of kScanTile elements: tile totals, a single-block
// scan of the totals, then each tile's local scan plus its offset.
constexpr int kScanThreads = 256;
constexpr int kScanPer = 8;
constexpr int kScanTile = kScanThreads * kScanPer;

int64_t scan_tmp_elems(int64_t n) { return ceil_div(n, kScanTile) + 1; }

__device__ __forceinline__ int32_t block_exclusive_scan(int32_t v, int32_t *lds, int32_t *total) {
  // lds: kScanThreads entries; Hillis-Steele inclusive scan, then shift
  const int tid = threadIdx.x;
  lds[tid] = v;
  __syncthreads();
  for (int off = 1; off < kScanThreads; off <<= 1) {
    int32_t o = tid >= off ? lds[tid - off] : 0;
    __syncthreads();
    lds[tid] += o;
    __syncthreads();
  }
  int32_t incl = lds[tid];
  *total = lds[kScanThreads - 1];
  __syncthreads();
  return incl - v;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_tiles(const int32_t *__restrict__ in,
                                                             int64_t n, int32_t *tile_sum) {
  __shared__ int32_t lds[kScanThreads];
  const int64_t base = blockIdx.x * (int64_t)kScanTile + threadIdx.x * kScanPer;
  int32_t s = 0;
#pragma unroll
  for (int q = 0; q < kScanPer; ++q)
    if (base + q < n) s += in[base + q];
  int32_t total;
  block_exclusive_scan(s, lds, &total);
  if (threadIdx.x == 0) tile_sum[blockIdx.x] = total;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_totals(int32_t *tile_sum, int64_t ntiles,
                                                              int32_t *out_last) {
  __shared__ int32_t lds[kScanThreads];
  int32_t carry = 0;
  for (int64_t b0 = 0; b0 < ntiles; b0 += kScanThreads) {
    int64_t t = b0 + threadIdx.x;
    int32_t v = t < ntiles ? tile_sum[t] : 0;
    int32_t total;
    int32_t ex = block_exclusive_scan(v, lds, &total);
    if (t < ntiles) tile_sum[t] = ex + carry;
    carry += total;
  }
  if (threadIdx.x == 0) *out_last = carry;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_apply(const int32_t *__restrict__ in,
                                                             int64_t n,
                                                             const int32_t *__restrict__ tile_off,
                                                             int32_t *__restrict__ out) {
  __shared__ int32_t lds[kScanThreads];
  const int64_t base = blockIdx.x * (int64_t)kScanTile + threadIdx.x * kScanPer;
  int32_t v[kScanPer];
  int32_t s = 0;
#pragma unroll
  for (int q = 0; q < kScanPer; ++q) {
    v[q] = (base + q < n) ? in[base + q] : 0;
    s += v[q];
  }
  int32_t total;
  int32_t run = block_exclusive_scan(s, lds, &total) + tile_off[blockIdx.x];
#pragma unroll
  for (int q = 0; q < kScanPer; ++q) {
    if (base + q < n) out[base + q] = run;
    run += v[q];
  }
}

void launch_exclusive_scan(hipStream_t s, const int32_t *in, int32_t *out, int64_t n,
                           int32_t *tmp) {
  // out has n + 1 entries; out[n] = total
  int64_t ntiles = ceil_div(n, kScanTile);
  if (ntiles < 1) ntiles = 1;
  hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)ntiles), dim3(kScanThreads), 0, s, in, n, tmp);
  hipLaunchKernelGGL(k_scan_totals, dim3(1), dim3(kScanThreads), 0, s, tmp, ntiles, out + n);
  hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)ntiles), dim3(kScanThreads), 0, s, in, n, tmp,
                     out);
}

// ------------------------------------------------ scatter + stable order
__global__ __launch_bounds__(256) void k_cell_scatter(const int32_t *__restrict__ cell_of,
                                                      int64_t n,
                                                      const int32_t *__restrict__ cell_start,
                                                      int32_t *fill, int32_t *__restrict__ perm) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t base = blockIdx.x * (int64_t)blockDim.x; base < n; base += stride) {
    const int64_t i = base + threadIdx.x;
    const bool valid = i < n;
    const int c = valid ? cell_of[i] : 0;
    const int slot = wave_run_slot(fill, (uint32_t)c, valid);
    if (valid) perm[cell_start[c] + slot] = (int32_t)i;
  }
}

void launch_cell_scatter(hipStream_t s, const int32_t *cell_of, int64_t n,
                         const int32_t *cell_start, int32_t *cell_fill, int32_t *perm) {
  if (n <= 0) return;
  int64_t b = ceil_div(n, 256);
  if (b > 16384) b = 16384;
  hipLaunchKernelGGL(k_cell_scatter, dim3((unsigned)b), dim3(256), 0, s, cell_of, n, cell_start,
                     cell_fill, perm);
}

// Atomic slots give an arbitrary order inside a cell; sort each cell's
// entries by caller index so the layout (and every FP sum) is reproducible.
__global__ __launch_bounds__(256) void k_cell_sort(const int32_t *__restrict__ cell_start,
                                                   int64_t ncell, int32_t *perm) {
  for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < ncell;
       c += (int64_t)gridDim.x * blockDim.x) {
    int a = cell_start[c], b = cell_start[c + 1];
    for (int p = a + 1; p < b; ++p) {
      int key = perm[p];
      int q = p - 1;
      while (q >= a && perm[q] > key) {
        perm[q + 1] = perm[q];
        --q;
      }
      perm[q + 1] = key;
    }
  }
}

void launch_cell_sort(hipStream_t s, const int32_t *cell_start, int64_t ncell, int32_t *perm) {
  int64_t b = ceil_div(ncell, 256);
  if (b < 1) b = 1;
  if (b > 16384) b = 16384;
  hipLaunchKernelGGL(k_cell_sort, dim3((unsigned)b), dim3(256), 0, s, cell_start, ncell, perm);
}

// Sorted copy (x, y, z, rc) with positions wrapped into the box.
__global__ __launch_bounds__(256) void k_gather(const double *__restrict__ x,
                                                const double *__restrict__ y,
                                                const double *__restrict__ z,
                                                const double *__restrict__ rc,
                                                const int32_t *__restrict__ perm, int64_t n,
                                                double Lx, double Ly, double Lz, double rc_cap,
                                                double4 *__restrict__ sorted) {
  for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < n;
       s += (int64_t)gridDim.x * blockDim.x) {
    int i = perm[s];
    double px = x[i], py = y[i], pz = z[i];
    double4 o;
    if (finite3(px, py, pz)) {
      o.x = wrap_coord(px, Lx);
      o.y = wrap_coord(py, Ly);
      o.z = wrap_coord(pz, Lz);
    } else {
      o.x = o.y = o.z = 0.0;
    }
    double r = rc[i];
    o.w = (r >= 0.0) ? (r < rc_cap ? r : rc_cap) : 0.0;  // NaN -> 0
    sorted[s] = o;
  }
}

void launch_gather(hipStream_t s, const double *x, const double *y, const double *z,
                   const double *rc, const int32_t *perm, int64_t n, const double L[3],
                   double rc_cap, double4 *sorted) {
  if (n <= 0) return;
  int64_t b = ceil_div(n, 256);
  if (b > 16384) b = 16384;
  hipLaunchKernelGGL(k_gather, dim3((unsigned)b), dim3(256), 0, s, x, y, z, rc, perm, n, L[0],
                     L[1], L[2], rc_cap, sorted);
}

// ------------------------------------------------ periodic ghost images
// The extended grid (ExtGeom) lets a lane walk any row of cells around its
// particle as one contiguous range of the extended array, without
// wrap-around or image shifts.
__global__ __launch_bounds__(256) void k_ext_count(const int32_t *__restrict__ cell_start,
                                                   ExtGeom g, int64_t next,
                                                   int32_t *__restrict__ ext_count) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < next;
       e += (int64_t)gridDim.x * blockDim.x) {
    int rc, p[3];
    ext_to_real(g, e, rc, p);
    ext_count[e] = cell_start[rc + 1] - cell_start[rc];
  }
}

// Writes stop at the buffer's capacity; running past it flags an overflow
// (the pair kernel then refuses to read ghost ranges beyond the capacity).
__global__ __launch_bounds__(256) void k_ext_fill(const int32_t *__restrict__ cell_start,
                                                  const int32_t *__restrict__ ext_start,
                                                  const double4 *__restrict__ sorted, ExtGeom g,
                                                  int64_t next, int64_t cap,
                                                  double4 *__restrict__ ext_pos,
                                                  float4 *__restrict__ ext_rel,
                                                  uint32_t *status) {
  const double len[3] = {g.L[0] / (double)g.nc[0], g.L[1] / (double)g.nc[1],
                         g.L[2] / (double)g.nc[2]};
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < next;
       e += (int64_t)gridDim.x * blockDim.x) {
    int rc, p[3];
    ext_to_real(g, e, rc, p);
    const double sx = (double)p[0] * g.L[0], sy = (double)p[1] * g.L[1],
                 sz = (double)p[2] * g.L[2];
    const int a = cell_start[rc], b = cell_start[rc + 1];
    int64_t o = ext_start[e];
    if (o + (b - a) > cap) {
      atomicOr(status, ST_GHOST_OVERFLOW);
      continue;
    }
    // extended cell coordinates, relative to the real grid
    const int ex = (int)(e % g.ne[0]) - g.h[0];
    const int ey = (int)((e / g.ne[0]) % g.ne[1]) - g.h[1];
    const int ez = (int)(e / ((int64_t)g.ne[0] * g.ne[1])) - g.h[2];
    for (int k = a; k < b; ++k, ++o) {
      double4 q = sorted[k];
      q.x = q.x + sx;
      q.y = q.y + sy;
      q.z = q.z + sz;
      ext_pos[o] = q;
      if (ext_rel) ext_rel[o] = rel_record(q, ex, ey, ez, len);
    }
  }
}

void launch_ext_build(hipStream_t s, const int32_t *cell_start, const double4 *sorted,
                      const int32_t nc[3], const int32_t h[3], const double L[3],
                      int64_t ext_cap, int32_t *ext_count, int32_t *ext_start,
                      int32_t *scan_tmp, double4 *ext_pos, float4 *ext_rel, uint32_t *status) {
  ExtGeom g;
  int64_t next = 1;
  for (int a = 0; a < 3; ++a) {
    g.nc[a] = nc[a];
    g.h[a] = h[a];
    g.ne[a] = nc[a] + 2 * h[a];
    g.L[a] = L[a];
    next *= g.ne[a];
  }
  int64_t b = ceil_div(next, 256);
  if (b > 16384) b = 16384;
  hipLaunchKernelGGL(k_ext_count, dim3((unsigned)b), dim3(256), 0, s, cell_start, g, next,
                     ext_count);
  launch_exclusive_scan(s, ext_count, ext_start, next, scan_tmp);
  hipLaunchKernelGGL(k_ext_fill, dim3((unsigned)b), dim3(256), 0, s, cell_start, ext_start,
                     sorted, g, next, ext_cap, ext_pos, ext_rel, status);
}

}  // namespace dcm
