// Verlet neighbour list with a skin (Section 2.3, Algorithm 2.2) and the
// force pass over it (Algorithm 2.3), on the ghost-extended cells of the
// last cell build.
//
// Particle i's list holds every extended slot j != i with
// r_ij^2 < (r_c(i) + skin)^2, found by the pair kernel's row walk and kept in
// the walk's order, so a force pass over the list sums exactly the pairs, in
// exactly the order, of the cell-walk force kernel.  Lists are stored per
// wavefront, entry k of lane l at wave_base + 64 k + l (wave_base: 64 times
// the sum of the longest lists of the earlier wavefronts), so a force pass
// reads each entry with one coalesced load.
#include "dcm_device.hpp"
#include "dcm_internal.hpp"

namespace dcm {

constexpr int kListBlock = 256;

__device__ __forceinline__ int clampl(int v, int lo, int hi) {
  return v < lo ? lo : (v > hi ? hi : v);
}

// Walk the rows of sorted particle s within radius R (x, y, z, self slot
// given) and call f(j) for every extended slot j != self with r^2 < R^2, in
// row order (z planes, then y rows, then x).
template <typename F>
__device__ __forceinline__ void walk_within(const ListArgs &a, double xi, double yi, double zi,
                                            double R, int self, F &&f) {
  const int nx = a.nc[0], ny = a.nc[1], nz = a.nc[2];
  const int hx = a.h[0], hy = a.h[1], hz = a.h[2];
  const int nex = a.ne[0], ney = a.ne[1];
  const double guard = 1e-9 * (a.len[0] + a.len[1] + a.len[2]);
  const double Rg = R + guard, R2 = Rg * Rg, Rt2 = R * R;
  const int cy = slab_index(yi, a.sc[1], ny), cz = slab_index(zi, a.sc[2], nz);
  const int zlo = clampl((int)floor((zi - Rg) * a.sc[2]), -hz, nz + hz - 1);
  const int zhi = clampl((int)floor((zi + Rg) * a.sc[2]), -hz, nz + hz - 1);
  for (int z = zlo; z <= zhi; ++z) {
    double ez = 0.0;
    if (z < cz) ez = zi - (double)(z + 1) * a.len[2];
    else if (z > cz) ez = (double)z * a.len[2] - zi;
    ez = ez > guard ? ez - guard : 0.0;
    const double remz = R2 - ez * ez;
    if (remz < 0.0) continue;
    const double wy = (double)(sqrtf((float)remz) * 1.00001f) + guard;
    const int ylo = clampl((int)floor((yi - wy) * a.sc[1]), -hy, ny + hy - 1);
    const int yhi = clampl((int)floor((yi + wy) * a.sc[1]), -hy, ny + hy - 1);
    for (int y = ylo; y <= yhi; ++y) {
      double ey = 0.0;
      if (y < cy) ey = yi - (double)(y + 1) * a.len[1];
      else if (y > cy) ey = (double)y * a.len[1] - yi;
      ey = ey > guard ? ey - guard : 0.0;
      const double rem = remz - ey * ey;
      if (rem < 0.0) continue;
      const double w = (double)(sqrtf((float)rem) * 1.00001f) + guard;
      const int xlo = clampl((int)floor((xi - w) * a.sc[0]), -hx, nx + hx - 1);
      const int xhi = clampl((int)floor((xi + w) * a.sc[0]), -hx, nx + hx - 1);
      const int32_t *es = a.ext_start + ((int64_t)(z + hz) * ney + (y + hy)) * nex + hx;
      const int j0 = es[xlo];
      int j1 = es[xhi + 1];
      if (j1 > a.ext_cap) j1 = (int)a.ext_cap;
      for (int j = j0; j < j1; ++j) {
        if (j == self) continue;
        const double4 q = a.ext_pos[j];
        const double dx = xi - q.x, dy = yi - q.y, dz = zi - q.z;
        if ((dx * dx + dy * dy) + dz * dz < Rt2) f(j);
      }
    }
  }
}

// particle s: position, list radius and own extended slot
__device__ __forceinline__ bool list_lane(const ListArgs &a, int64_t s, double &xi, double &yi,
                                          double &zi, double &R, int &self) {
  if (s >= a.n) return false;
  const double4 p = a.pos[s];
  xi = p.x;
  yi = p.y;
  zi = p.z;
  R = (p.w < a.rc_bound ? p.w : a.rc_bound) + a.skin;
  const int cx = slab_index(xi, a.sc[0], a.nc[0]);
  const int cy = slab_index(yi, a.sc[1], a.nc[1]), cz = slab_index(zi, a.sc[2], a.nc[2]);
  const int real = (cz * a.nc[1] + cy) * a.nc[0] + cx;
  const int ext = ((cz + a.h[2]) * a.ne[1] + (cy + a.h[1])) * a.ne[0] + (cx + a.h[0]);
  self = a.ext_start[ext] + (int)(s - a.cell_start[real]);
  return true;
}

// Pass 1: list lengths; the longest of each wavefront into wave_len.
__global__ __launch_bounds__(kListBlock) void k_list_count(ListArgs a) {
  const int64_t s = blockIdx.x * (int64_t)kListBlock + threadIdx.x;
  double xi, yi, zi, R;
  int self = -1, cnt = 0;
  if (list_lane(a, s, xi, yi, zi, R, self)) walk_within(a, xi, yi, zi, R, self, [&](int) { ++cnt; });
  if (s < a.n) {
    a.count[s] = cnt;
    a.ref[s] = make_double4(xi, yi, zi, R);  // where the list was built, and its radius
  }
  int m = cnt;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const int o = __shfl_xor(m, off, 64);
    m = o > m ? o : m;
  }
  if ((threadIdx.x & 63) == 0 && (s >> 6) < a.n_waves) a.wave_len[s >> 6] = m;
}

// Pass 2: the entries, at wave_base + 64 k + lane.
__global__ __launch_bounds__(kListBlock) void k_list_fill(ListArgs a) {
  const int64_t s = blockIdx.x * (int64_t)kListBlock + threadIdx.x;
  double xi, yi, zi, R;
  int self = -1;
  if (!list_lane(a, s, xi, yi, zi, R, self)) return;
  const int64_t base = 64 * (int64_t)a.wave_start[s >> 6] + (s & 63);
  if (64 * (int64_t)a.wave_start[a.n_waves] > a.list_cap) {
    atomicOr(a.status, ST_GHOST_OVERFLOW);
    return;
  }
  int k = 0;
  walk_within(a, xi, yi, zi, R, self, [&](int j) {
    a.list[base + 64 * (int64_t)k] = j;
    ++k;
  });
}

// Reuse over steps: sorted particle s takes its new position and cutoff.  It
// moves by the minimum image of its displacement from where the list was
// built, so the ghost images refilled from it move with it whether or not
// the caller wrapped it back into the box.  Per workgroup: the largest
// squared displacement and the smallest slack R_s - r_c(s).
__global__ __launch_bounds__(kListBlock) void k_list_update(
    const double *__restrict__ x, const double *__restrict__ y, const double *__restrict__ z,
    const double *__restrict__ rc, const int32_t *__restrict__ perm,
    const double4 *__restrict__ ref, int64_t n, double Lx, double Ly, double Lz, double rc_cap,
    double4 *__restrict__ sorted, double2 *__restrict__ part, uint32_t *status) {
  __shared__ double2 red[kListBlock / 64];
  const int64_t s = blockIdx.x * (int64_t)kListBlock + threadIdx.x;
  double d2 = 0.0, slack = INFINITY;
  if (s < n) {
    const int i = perm[s];
    const double4 r0 = ref[s];
    const double px = x[i], py = y[i], pz = z[i];
    double c = rc[i];
    double4 o = r0;
    if (finite3(px, py, pz)) {
      double dx = px - r0.x, dy = py - r0.y, dz = pz - r0.z;
      dx -= Lx * rint(dx / Lx);
      dy -= Ly * rint(dy / Ly);
      dz -= Lz * rint(dz / Lz);
      o.x = r0.x + dx;
      o.y = r0.y + dy;
      o.z = r0.z + dz;
      d2 = (dx * dx + dy * dy) + dz * dz;
    } else {
      atomicOr(status, ST_NONFINITE_POS);
      d2 = INFINITY;
    }
    if (!(c >= 0.0) || c > rc_cap) {
      atomicOr(status, ST_RC_RANGE);
      c = (c > rc_cap) ? rc_cap : 0.0;
    }
    o.w = c;
    sorted[s] = o;
    slack = r0.w - c;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const double od = __shfl_xor(d2, off, 64), os = __shfl_xor(slack, off, 64);
    d2 = od > d2 ? od : d2;
    slack = os < slack ? os : slack;
  }
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = make_double2(d2, slack);
  __syncthreads();
  if (threadIdx.x == 0) {
    double2 m = red[0];
#pragma unroll
    for (int w = 1; w < kListBlock / 64; ++w) {
      m.x = red[w].x > m.x ? red[w].x : m.x;
      m.y = red[w].y < m.y ? red[w].y : m.y;
    }
    part[blockIdx.x] = m;
  }
}

// One workgroup: out = (largest displacement, smallest slack) over the parts.
__global__ __launch_bounds__(kListBlock) void k_list_verdict(const double2 *__restrict__ part,
                                                             int64_t nparts, double *out) {
  __shared__ double2 red[kListBlock / 64];
  double d2 = 0.0, slack = INFINITY;
  for (int64_t b = threadIdx.x; b < nparts; b += kListBlock) {
    const double2 m = part[b];
    d2 = m.x > d2 ? m.x : d2;
    slack = m.y < slack ? m.y : slack;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const double od = __shfl_xor(d2, off, 64), os = __shfl_xor(slack, off, 64);
    d2 = od > d2 ? od : d2;
    slack = os < slack ? os : slack;
  }
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = make_double2(d2, slack);
  __syncthreads();
  if (threadIdx.x == 0) {
    double2 m = red[0];
    for (int w = 1; w < kListBlock / 64; ++w) {
      m.x = red[w].x > m.x ? red[w].x : m.x;
      m.y = red[w].y < m.y ? red[w].y : m.y;
    }
    out[0] = sqrt(m.x);
    out[1] = m.y;
  }
}

int64_t list_update_blocks(int64_t n) { return ceil_div(n, kListBlock) > 0 ? ceil_div(n, kListBlock) : 1; }

void launch_list_update(hipStream_t s, const double *x, const double *y, const double *z,
                        const double *rc, const int32_t *perm, const double4 *ref, int64_t n,
                        const double L[3], double rc_cap, double4 *sorted, double2 *part,
                        double *out, uint32_t *status) {
  const int64_t blocks = list_update_blocks(n);
  hipLaunchKernelGGL(k_list_update, dim3((unsigned)blocks), dim3(kListBlock), 0, s, x, y, z, rc,
                     perm, ref, n, L[0], L[1], L[2], rc_cap, sorted, part, status);
  hipLaunchKernelGGL(k_list_verdict, dim3(1), dim3(kListBlock), 0, s, part, blocks, out);
}

int64_t list_waves(int64_t n) { return ceil_div(n, 64); }

void launch_list_count(hipStream_t s, const ListArgs &a) {
  const int64_t blocks = ceil_div(a.n, kListBlock) > 0 ? ceil_div(a.n, kListBlock) : 1;
  hipLaunchKernelGGL(k_list_count, dim3((unsigned)blocks), dim3(kListBlock), 0, s, a);
}

void launch_list_fill(hipStream_t s, const ListArgs &a) {
  const int64_t blocks = ceil_div(a.n, kListBlock) > 0 ? ceil_div(a.n, kListBlock) : 1;
  hipLaunchKernelGGL(k_list_fill, dim3((unsigned)blocks), dim3(kListBlock), 0, s, a);
}

}  // namespace dcm
