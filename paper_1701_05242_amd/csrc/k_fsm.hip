// Cutoff-limited fast-sweeping distances (Section 2.2, Algorithm 2.1).
//
// Every voxel applies the first-order Godunov upwind update of |grad d| = 1,
// d <- min(d, G(neighbours)), accepting only values <= rc_grid, until nothing
// changes.  The update is monotone, so any order of updates reaches the same
// fixed point as the paper's sweeps; source voxels (interface and
// low-density phase) hold 0 and are never rewritten.
//
// Grids at least two voxels larger than a tile on every axis use temporal
// blocking: a launch stages 16 x 8 x 8 voxel tiles (plus a one-voxel halo)
// in LDS and iterates synchronous sub-waves inside each tile until it stops
// changing, with the halo frozen.  Like the paper's queue of boxes next to
// updated boxes, a tile only runs again when it or one of its 26 neighbour
// tiles changed in the previous launch; a launch in which no tile changes
// ends the sweep.  Launches read one global buffer and write the other, so
// the result does not depend on scheduling.  Thinner grids use plain
// synchronous waves over all voxels.
#include "dcm_device.hpp"
#include "dcm_internal.hpp"

namespace dcm {

constexpr int TX = 16, TY = 8, TZ = 8;                 // tile interior
constexpr int QX = TX + 2, QY = TY + 2, QZ = TZ + 2;   // with halo
constexpr int kTileThreads = 256;
constexpr int kMaxSubWaves = 64;

bool fsm_tiled(const int32_t nv[3]) {
  return nv[0] >= TX + 2 && nv[1] >= TY + 2 && nv[2] >= TZ + 2;
}

int64_t fsm_tile_count(const int32_t nv[3]) {
  return ceil_div(nv[0], TX) * ceil_div(nv[1], TY) * ceil_div(nv[2], TZ);
}

__global__ void k_fsm_clear(uint8_t *chg0, int ntiles, uint32_t *flags, int nflags) {
  for (int t = threadIdx.x; t < ntiles; t += blockDim.x) chg0[t] = 0;
  for (int f = threadIdx.x; f < nflags; f += blockDim.x) flags[f] = 0u;
}

// Sources (low-density phase and interface) start at 0, the rest at +inf.
// With tiles, every tile holding an interface voxel is flagged as changed
// before the first pass: only next to an interface can a pass change
// anything at first (a liquid voxel with a source face neighbour is itself
// an interface voxel).
__global__ __launch_bounds__(256) void k_fsm_init(const uint8_t *__restrict__ seg,
                                                  const uint8_t *__restrict__ iface,
                                                  int64_t nvox, int nx, int ny, double *dA,
                                                  double *dB, uint8_t *chg0, int ntx, int nty) {
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < nvox;
       v += (int64_t)gridDim.x * blockDim.x) {
    const bool fc = iface[v] != 0;
    double d = (seg[v] == 0 || fc) ? 0.0 : __builtin_huge_val();
    dA[v] = d;
    dB[v] = d;
    if (fc && chg0) {
      const int64_t row = v / nx;
      const int x = (int)(v - row * nx), y = (int)(row % ny), z = (int)(row / ny);
      chg0[((z / TZ) * nty + y / TY) * ntx + x / TX] = 1;
    }
  }
}

// The same from the bit-packed phase maps of the regularisation passes
// (final_phase_map), without the byte maps: a voxel starts at +inf iff it
// and its six face neighbours (periodic) are all high density -- otherwise
// it is low density or an interface voxel, a source.
__global__ __launch_bounds__(256) void k_fsm_init_bits(const uint32_t *b0, const uint32_t *b1,
                                                       const Ctl *ctl, int nx, int ny, int nz,
                                                       double *dA, double *dB, uint8_t *chg0,
                                                       int ntx, int nty) {
  const uint32_t *__restrict__ s =
      final_phase_map(ctl->maj_chg1, ctl->maj_chg2, kMajorityMaxPasses, b0, b1);
  const int W = (nx + 31) >> 5;
  const int64_t nvox = (int64_t)nx * ny * nz;
  auto bit = [&](int x, int y, int z) -> uint32_t {
    return (s[((int64_t)z * ny + y) * W + (x >> 5)] >> (x & 31)) & 1u;
  };
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < nvox;
       v += (int64_t)gridDim.x * blockDim.x) {
    const int64_t row = v / nx;
    const int x = (int)(v - row * nx), y = (int)(row % ny), z = (int)(row / ny);
    const uint32_t sv = bit(x, y, z);
    bool fc = false;
    if (sv) {
      const int xm = x == 0 ? nx - 1 : x - 1, xp = x + 1 == nx ? 0 : x + 1;
      const int ym = y == 0 ? ny - 1 : y - 1, yp = y + 1 == ny ? 0 : y + 1;
      const int zm = z == 0 ? nz - 1 : z - 1, zp = z + 1 == nz ? 0 : z + 1;
      fc = (bit(xm, y, z) & bit(xp, y, z) & bit(x, ym, z) & bit(x, yp, z) & bit(x, y, zm) &
            bit(x, y, zp)) == 0u;
    }
    const double d = (sv == 0u || fc) ? 0.0 : __builtin_huge_val();
    dA[v] = d;
    dB[v] = d;
    if (fc && chg0) chg0[((z / TZ) * nty + y / TY) * ntx + x / TX] = 1;
  }
}

// Godunov solve: with the smaller face neighbour a_k and spacing h_k per axis
// (w_k = 1/h_k^2), d solves sum over the m smallest a_k of w_k (d - a_k)^2 = 1
// for the largest m whose root does not pass the next a_k; written relative
// to the smallest a.
// ISO: equal spacings on every axis (h0 = h1 = h2, w0 = w1 = w2), so only
// the a's need ordering: the same arithmetic on the same values.
template <bool ISO = false>
__device__ __forceinline__ double godunov(double a0, double a1, double a2, double h0,
                                          double h1, double h2, double w0, double w1,
                                          double w2) {
  // order (a, h, w) by a, ascending, keeping axis order on ties
  if (a1 < a0) {
    double t = a0; a0 = a1; a1 = t;
    if constexpr (!ISO) {
      t = h0; h0 = h1; h1 = t;
      t = w0; w0 = w1; w1 = t;
    }
  }
  if (a2 < a1) {
    double t = a1; a1 = a2; a2 = t;
    if constexpr (!ISO) {
      t = h1; h1 = h2; h2 = t;
      t = w1; w1 = w2; w2 = t;
    }
    if (a1 < a0) {
      t = a0; a0 = a1; a1 = t;
      if constexpr (!ISO) {
        t = h0; h0 = h1; h1 = t;
        t = w0; w0 = w1; w1 = t;
      }
    }
  }
  if (isinf(a0)) return a0;
  double d = a0 + h0;
  if (d <= a1) return d;
  double b1 = a1 - a0;
  double A = w0 + w1;
  double B = w1 * b1;
  double C = w1 * b1 * b1 - 1.0;
  double disc = B * B - A * C;
  if (disc < 0.0) disc = 0.0;
  d = a0 + (B + sqrt(disc)) / A;
  if (d <= a2) return d;
  double b2 = a2 - a0;
  A = (w0 + w1) + w2;
  B = w1 * b1 + w2 * b2;
  C = (w1 * b1 * b1 + w2 * b2 * b2) - 1.0;
  disc = B * B - A * C;
  if (disc < 0.0) disc = 0.0;
  return a0 + (B + sqrt(disc)) / A;
}

struct SweepGeom {
  int nx, ny, nz;
  double hx, hy, hz, wx, wy, wz;
  double rc_grid;
};

// ------------------------------------------------------------- tiled sweep
// Launch L reads buf[(L-1)&1] and tile flags chg[(L-1)&1]; writes buf[L&1]
// for its active tiles and chg[L&1] for every tile.
template <bool ISO>
__global__ __launch_bounds__(kTileThreads) void k_fsm_tiles(double *dA, double *dB,
                                                            uint8_t *chg0, uint8_t *chg1,
                                                            SweepGeom g, int ntx, int nty,
                                                            int ntz, int launch,
                                                            uint32_t *flags) {
  // a pass runs only while the previous one changed something
  if (launch > 1 && flags[launch - 1] == 0u) return;
  __shared__ double A[QZ][QY][QX];
  __shared__ double B[QZ][QY][QX];
  __shared__ int act;
  const double *__restrict__ src = (launch & 1) ? dA : dB;
  double *__restrict__ dst = (launch & 1) ? dB : dA;
  const uint8_t *chg_prev = (launch & 1) ? chg0 : chg1;
  uint8_t *chg_cur = (launch & 1) ? chg1 : chg0;
  const int tid = threadIdx.x;
  const int ntiles = ntx * nty * ntz;
  unsigned long long tiles_changed = 0;
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const int tx = t % ntx;
    const int tr = t / ntx;
    const int ty = tr % nty;
    const int tz = tr / nty;
    // active: this tile or a neighbour changed in the last launch (before
    // the first, the tiles holding interface voxels count as changed)
    if (tid == 0) act = 0;
    __syncthreads();
    if (tid < 27) {
      const int dx = tid % 3 - 1, dy = (tid / 3) % 3 - 1, dz = tid / 9 - 1;
      const int nxp = wrap_index(tx + dx, ntx), nyp = wrap_index(ty + dy, nty),
                nzp = wrap_index(tz + dz, ntz);
      if (chg_prev[(nzp * nty + nyp) * ntx + nxp]) act = 1;
    }
    __syncthreads();
    if (!act) {
      if (tid == 0) chg_cur[t] = 0;
      __syncthreads();
      continue;
    }
    const int x0 = tx * TX, y0 = ty * TY, z0 = tz * TZ;
    // stage the tile and its halo (periodic); the grid is at least two voxels
    // wider than the tile, so no voxel appears twice
    for (int e = tid; e < QZ * QY * QX; e += kTileThreads) {
      const int lz = e / (QY * QX);
      const int r = e - lz * (QY * QX);
      const int ly = r / QX;
      const int lx = r - ly * QX;
      int gx = x0 + lx - 1, gy = y0 + ly - 1, gz = z0 + lz - 1;
      gx = gx < 0 ? gx + g.nx : (gx >= g.nx ? gx - g.nx : gx);
      gy = gy < 0 ? gy + g.ny : (gy >= g.ny ? gy - g.ny : gy);
      gz = gz < 0 ? gz + g.nz : (gz >= g.nz ? gz - g.nz : gz);
      const double d = src[((int64_t)gz * g.ny + gy) * g.nx + gx];
      A[lz][ly][lx] = d;
      B[lz][ly][lx] = d;
    }
    __syncthreads();
    // sub-waves: each thread owns 4 interior voxels (fixed x, y; z = q*2+...)
    bool tile_changed = false;
    for (int sub = 0; sub < kMaxSubWaves; ++sub) {
      bool mine = false;
      double (*in)[QY][QX] = (sub & 1) ? B : A;
      double (*out)[QY][QX] = (sub & 1) ? A : B;
#pragma unroll
      for (int q = 0; q < (TX * TY * TZ) / kTileThreads; ++q) {
        const int e = tid + q * kTileThreads;
        const int lx = e % TX + 1;
        const int ly = (e / TX) % TY + 1;
        const int lz = e / (TX * TY) + 1;
        const bool owned = (x0 + lx - 1 < g.nx) && (y0 + ly - 1 < g.ny) && (z0 + lz - 1 < g.nz);
        const double d = in[lz][ly][lx];
        double nd = d;
        if (owned && d != 0.0) {
          const double ax = fmin(in[lz][ly][lx - 1], in[lz][ly][lx + 1]);
          const double ay = fmin(in[lz][ly - 1][lx], in[lz][ly + 1][lx]);
          const double az = fmin(in[lz - 1][ly][lx], in[lz + 1][ly][lx]);
          const double gv = godunov<ISO>(ax, ay, az, g.hx, g.hy, g.hz, g.wx, g.wy, g.wz);
          if (gv < d && gv <= g.rc_grid) nd = gv;
        }
        out[lz][ly][lx] = nd;
        mine |= (nd != d);
      }
      const int changed = __syncthreads_or(mine ? 1 : 0);
      if (!changed) break;
      tile_changed = true;
    }
    // A holds the latest state: a loop that stops on a sub-wave with no
    // change wrote identical values into both buffers, and a loop that runs
    // out ends on an odd sub-wave, which writes A (kMaxSubWaves is even).
    // A tile that has not settled is marked changed and runs again.
    static_assert(kMaxSubWaves % 2 == 0, "the last sub-wave must write A");
#pragma unroll
    for (int q = 0; q < (TX * TY * TZ) / kTileThreads; ++q) {
      const int e = tid + q * kTileThreads;
      const int lx = e % TX + 1;
      const int ly = (e / TX) % TY + 1;
      const int lz = e / (TX * TY) + 1;
      const int gx = x0 + lx - 1, gy = y0 + ly - 1, gz = z0 + lz - 1;
      if (gx < g.nx && gy < g.ny && gz < g.nz)
        dst[((int64_t)gz * g.ny + gy) * g.nx + gx] = A[lz][ly][lx];
    }
    if (tid == 0) chg_cur[t] = tile_changed ? 1 : 0;
    tiles_changed += tile_changed ? 1 : 0;
    __syncthreads();
  }
  if (tid == 0 && tiles_changed) flags[launch] = 1u;
}

// ------------------------------------------------------------- plain waves
// Wave w reads state w-1 from buf[(w-1)&1] and writes state w to buf[w&1].
__global__ __launch_bounds__(256) void k_fsm_wave(double *dA, double *dB, SweepGeom g, int wave,
                                                  uint32_t *flags) {
  if (wave > 1 && flags[wave - 1] == 0u) return;
  const double *__restrict__ src = (wave & 1) ? dA : dB;
  double *__restrict__ dst = (wave & 1) ? dB : dA;
  const int i = blockIdx.x * 64 + (threadIdx.x & 63);
  const int j = blockIdx.y * 4 + (threadIdx.x >> 6);
  bool chg = false;
  if (i < g.nx && j < g.ny) {
    const int im = i == 0 ? g.nx - 1 : i - 1, ip = i + 1 == g.nx ? 0 : i + 1;
    const int jm = j == 0 ? g.ny - 1 : j - 1, jp = j + 1 == g.ny ? 0 : j + 1;
    for (int k = blockIdx.z; k < g.nz; k += gridDim.z) {
      const int km = k == 0 ? g.nz - 1 : k - 1, kp = k + 1 == g.nz ? 0 : k + 1;
      const int64_t rowk = (int64_t)k * g.ny;
      const int64_t v = (rowk + j) * g.nx + i;
      const double d = src[v];
      if (d == 0.0) continue;
      const double ax = fmin(src[(rowk + j) * g.nx + im], src[(rowk + j) * g.nx + ip]);
      const double ay = fmin(src[(rowk + jm) * g.nx + i], src[(rowk + jp) * g.nx + i]);
      const double az = fmin(src[((int64_t)km * g.ny + j) * g.nx + i],
                             src[((int64_t)kp * g.ny + j) * g.nx + i]);
      const double gv = godunov(ax, ay, az, g.hx, g.hy, g.hz, g.wx, g.wy, g.wz);
      const double nd = (gv < d && gv <= g.rc_grid) ? gv : d;
      dst[v] = nd;
      chg |= (nd != d);
    }
  }
  if (__syncthreads_or(chg ? 1 : 0) && threadIdx.x == 0) flags[wave] = 1u;
}

// The last pass is the first one that changed nothing (its output equals its
// input); if every pass changed something the sweep did not converge.
__global__ __launch_bounds__(256) void k_fsm_final(const double *dA, const double *dB,
                                                   int64_t nvox, double rc_grid,
                                                   const uint32_t *flags, int max_steps,
                                                   double *__restrict__ dist, int32_t *waves_out,
                                                   uint32_t *status) {
  int last = max_steps;
  for (int p = 1; p <= max_steps; ++p)
    if (flags[p] == 0u) {
      last = p;
      break;
    }
  const double *__restrict__ D = (last & 1) ? dB : dA;
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < nvox;
       v += (int64_t)gridDim.x * blockDim.x) {
    double d = D[v];
    dist[v] = d > rc_grid ? rc_grid : d;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (waves_out) *waves_out = (int32_t)last;
    if (flags[max_steps] != 0u) atomicOr(status, ST_NOT_CONVERGED);
  }
}

static unsigned flat_grid(int64_t nvox) {
  int64_t b = ceil_div(nvox, 256 * 4);
  if (b < 1) b = 1;
  if (b > 4096) b = 4096;
  return (unsigned)b;
}

static SweepGeom geom(const int32_t nv[3], const double h[3], double rc_grid) {
  SweepGeom g;
  g.nx = nv[0];
  g.ny = nv[1];
  g.nz = nv[2];
  g.hx = h[0];
  g.hy = h[1];
  g.hz = h[2];
  g.wx = 1.0 / (h[0] * h[0]);
  g.wy = 1.0 / (h[1] * h[1]);
  g.wz = 1.0 / (h[2] * h[2]);
  g.rc_grid = rc_grid;
  return g;
}

void launch_fsm_init(hipStream_t s, const uint8_t *seg, const uint8_t *iface, const int32_t nv[3],
                     double *dA, double *dB, uint8_t *chg0, uint32_t *flags, int max_steps) {
  const int64_t nvox = (int64_t)nv[0] * nv[1] * nv[2];
  const bool tiled = fsm_tiled(nv);
  const int ntx = (int)ceil_div(nv[0], TX), nty = (int)ceil_div(nv[1], TY);
  const int ntiles = tiled ? (int)fsm_tile_count(nv) : 0;
  hipLaunchKernelGGL(k_fsm_clear, dim3(1), dim3(1024), 0, s, chg0, ntiles, flags, max_steps + 2);
  hipLaunchKernelGGL(k_fsm_init, dim3(flat_grid(nvox)), dim3(256), 0, s, seg, iface, nvox, nv[0],
                     nv[1], dA, dB, tiled ? chg0 : nullptr, ntx, nty);
}

void launch_fsm_init_bits(hipStream_t s, const uint32_t *const maps[2], const Ctl *ctl,
                          const int32_t nv[3], double *dA, double *dB, uint8_t *chg0,
                          uint32_t *flags, int max_steps) {
  const int64_t nvox = (int64_t)nv[0] * nv[1] * nv[2];
  const bool tiled = fsm_tiled(nv);
  const int ntx = (int)ceil_div(nv[0], TX), nty = (int)ceil_div(nv[1], TY);
  const int ntiles = tiled ? (int)fsm_tile_count(nv) : 0;
  hipLaunchKernelGGL(k_fsm_clear, dim3(1), dim3(1024), 0, s, chg0, ntiles, flags, max_steps + 2);
  hipLaunchKernelGGL(k_fsm_init_bits, dim3(flat_grid(nvox)), dim3(256), 0, s, maps[0], maps[1],
                     ctl, nv[0], nv[1], nv[2], dA, dB, tiled ? chg0 : nullptr, ntx, nty);
}

// workgroups of a tiled pass, each walking tiles in turn (measured on the
// 160 x 160 x 400 grid: 2048 the same, 4096 3% slower over the sweep)
constexpr int64_t kFsmTileBlocks = 1024;

void launch_fsm_step(hipStream_t s, double *dA, double *dB, uint8_t *chg0, uint8_t *chg1,
                     const int32_t nv[3], const double h[3], double rc_grid, int step,
                     uint32_t *flags) {
  const SweepGeom g = geom(nv, h, rc_grid);
  if (fsm_tiled(nv)) {
    const int ntx = (int)ceil_div(nv[0], TX), nty = (int)ceil_div(nv[1], TY),
              ntz = (int)ceil_div(nv[2], TZ);
    int64_t blocks = (int64_t)ntx * nty * ntz;
    if (blocks > kFsmTileBlocks) blocks = kFsmTileBlocks;  // passes after convergence stay cheap
    if (h[0] == h[1] && h[1] == h[2])
      hipLaunchKernelGGL(k_fsm_tiles<true>, dim3((unsigned)blocks), dim3(kTileThreads), 0, s, dA,
                         dB, chg0, chg1, g, ntx, nty, ntz, step, flags);
    else
      hipLaunchKernelGGL(k_fsm_tiles<false>, dim3((unsigned)blocks), dim3(kTileThreads), 0, s, dA,
                         dB, chg0, chg1, g, ntx, nty, ntz, step, flags);
  } else {
    int zb = nv[2] < 64 ? nv[2] : 64;
    hipLaunchKernelGGL(k_fsm_wave,
                       dim3((unsigned)ceil_div(nv[0], 64), (unsigned)ceil_div(nv[1], 4),
                            (unsigned)zb),
                       dim3(256), 0, s, dA, dB, g, step, flags);
  }
}

void launch_fsm_final(hipStream_t s, const double *dA, const double *dB, int64_t nvox,
                      double rc_grid, const uint32_t *flags, int max_steps, double *dist,
                      int32_t *waves_out, uint32_t *status) {
  hipLaunchKernelGGL(k_fsm_final, dim3(flat_grid(nvox)), dim3(256), 0, s, dA, dB, nvox,
                     rc_grid, flags, max_steps, dist, waves_out, status);
}

}  // namespace dcm
