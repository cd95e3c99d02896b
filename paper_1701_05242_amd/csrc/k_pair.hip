// Dynamic-cutoff Lennard-Jones force, energy and virial (Section 2.4,
// Algorithm 2.3, Eqs. 2-3) over the linked cells of Section 2.3.
//
// One lane owns one particle i (particles in cell order, so a wavefront
// covers neighbouring particles with similar cutoffs).  Instead of storing
// the neighbour list of Algorithm 2.2, each lane enumerates the cell rows
// (fixed y and z cell; consecutive x cells are consecutive in the sorted
// arrays) that can hold a j within its search radius, trims each row to the
// chord of the search sphere -- the small-cell traversal of Section 2.3 -- and
// writes the resulting index segments into a private LDS list.  It then runs
// one flat loop over all candidates of those segments, so lanes with
// different row lengths never wait for each other row by row.  The periodic
// image shift is constant per segment.  No Newton-3 update is made
// (Section 2.4): a lane writes only its own particle.
#include "dcm_device.hpp"
#include "dcm_internal.hpp"

namespace dcm {

constexpr int kPairBlock = 256;
constexpr int kSegCap = 16;  // segments per lane per chunk (LDS: 8 B each)
int pair_block_size() { return kPairBlock; }

// Per-lane accumulators.
template <int PREC>
struct Acc;

template <>
struct Acc<DCM_FP64> {
  double fx = 0, fy = 0, fz = 0, e = 0, w[6] = {0, 0, 0, 0, 0, 0};
};

template <>
struct Acc<DCM_FP32_MIXED> {
  double fx = 0, fy = 0, fz = 0;
  float e = 0, w[6] = {0, 0, 0, 0, 0, 0};
};

// 1/r2 from the hardware reciprocal estimate refined by Newton steps
// y <- y + y (1 - r2 y): two steps for FP64, one before rounding to FP32.
__device__ __forceinline__ double recip_newton2(double r2) {
  double y = __builtin_amdgcn_rcp(r2);
  double e = fma(-r2, y, 1.0);
  y = fma(y, e, y);
  e = fma(-r2, y, 1.0);
  return fma(y, e, y);
}

__device__ __forceinline__ float recip_to_f32(double r2) {
  double y = __builtin_amdgcn_rcp(r2);
  double e = fma(-r2, y, 1.0);
  return (float)fma(y, e, y);
}

// One interacting pair with separation d (FP64) and r2.  The force factor
// excludes 24 eps, the energy 4 eps / 2, the virial 24 eps / 2; they are
// applied once per particle.
template <int PREC, int EVM>
__device__ __forceinline__ void interact(Acc<PREC> &acc, double dx, double dy, double dz,
                                         double r2, double sig2) {
  if constexpr (PREC == DCM_FP64) {
    double r2i = recip_newton2(r2);
    double s2 = sig2 * r2i;
    double s6 = s2 * s2 * s2;
    double fp = s6 * fma(2.0, s6, -1.0) * r2i;
    acc.fx = fma(fp, dx, acc.fx);
    acc.fy = fma(fp, dy, acc.fy);
    acc.fz = fma(fp, dz, acc.fz);
    if constexpr ((EVM & 1) != 0) acc.e = fma(s6, s6 - 1.0, acc.e);
    if constexpr ((EVM & 2) != 0) {
      double fdx = fp * dx, fdy = fp * dy, fdz = fp * dz;
      acc.w[0] = fma(fdx, dx, acc.w[0]);
      acc.w[1] = fma(fdy, dy, acc.w[1]);
      acc.w[2] = fma(fdz, dz, acc.w[2]);
      acc.w[3] = fma(fdy, dx, acc.w[3]);
      acc.w[4] = fma(fdz, dx, acc.w[4]);
      acc.w[5] = fma(fdz, dy, acc.w[5]);
    }
  } else {
    float r2i = recip_to_f32(r2);
    float s2 = (float)sig2 * r2i;
    float s6 = s2 * s2 * s2;
    float fp = s6 * fmaf(2.0f, s6, -1.0f) * r2i;
    double fpd = (double)fp;
    acc.fx = fma(fpd, dx, acc.fx);
    acc.fy = fma(fpd, dy, acc.fy);
    acc.fz = fma(fpd, dz, acc.fz);
    if constexpr ((EVM & 1) != 0) acc.e = fmaf(s6, s6 - 1.0f, acc.e);
    if constexpr ((EVM & 2) != 0) {
      float dxf = (float)dx, dyf = (float)dy, dzf = (float)dz;
      float fdx = fp * dxf, fdy = fp * dyf, fdz = fp * dzf;
      acc.w[0] = fmaf(fdx, dxf, acc.w[0]);
      acc.w[1] = fmaf(fdy, dyf, acc.w[1]);
      acc.w[2] = fmaf(fdz, dzf, acc.w[2]);
      acc.w[3] = fmaf(fdy, dxf, acc.w[3]);
      acc.w[4] = fmaf(fdz, dxf, acc.w[4]);
      acc.w[5] = fmaf(fdz, dyf, acc.w[5]);
    }
  }
}

// Segment encoding in LDS: .x = first sorted index, .y = count (low 24 bits)
// | shift code << 24.  Shift code bits: x (2 bits), y (2 bits), z (2 bits),
// each 0 = none, 1 = +L, 2 = -L; bit 6 = take the image per pair instead.
constexpr uint32_t kPerPairImage = 1u << 6;

__device__ __forceinline__ double code_shift(uint32_t c, double L) {
  return c == 1u ? L : (c == 2u ? -L : 0.0);
}

template <int RULE, int PREC, int EVM>
__global__ __launch_bounds__(kPairBlock) void k_pair(PairArgs a) {
  __shared__ uint2 segs[kSegCap][kPairBlock];
  const int lane_id = threadIdx.x;
  const int64_t s = blockIdx.x * (int64_t)kPairBlock + threadIdx.x;
  const bool active = s < a.n;
  Acc<PREC> acc;
  int cnt = 0;
  const double Lx = a.L[0], Ly = a.L[1], Lz = a.L[2];
  const int nx = a.nc[0], ny = a.nc[1], nz = a.nc[2];
  const double sig2 = a.sigma * a.sigma;
  double xi = 0, yi = 0, zi = 0, rci = 0, rci2 = 0;
  // row enumeration state
  int zlo = 0, zhi = -1, ylo = 0, yhi = -1, zc = 0, yc = 0, cy = 0, cz = 0;
  bool fully = false, fullz = false;
  double R2 = 0, guard = 0;
  if (active) {
    const double4 pi = a.pos[s];
    xi = pi.x;
    yi = pi.y;
    zi = pi.z;
    rci = pi.w;
    double R = rci;
    if constexpr (RULE == DCM_PAIR_MAX) {
      double rall = __longlong_as_double((long long)a.ctl->rc_max_bits);
      R = rall > R ? rall : R;
    }
    rci2 = rci * rci;
    // search radius widened by a hair: rounding in the cell geometry can
    // only add candidates, never drop one
    guard = 1e-9 * (a.len[0] + a.len[1] + a.len[2]);
    const double Rg = R + guard;
    R2 = Rg * Rg;
    cy = slab_index(yi, a.sc[1], ny);
    cz = slab_index(zi, a.sc[2], nz);
    zlo = (int)floor((zi - Rg) * a.sc[2]);
    zhi = (int)floor((zi + Rg) * a.sc[2]);
    ylo = (int)floor((yi - Rg) * a.sc[1]);
    yhi = (int)floor((yi + Rg) * a.sc[1]);
    fullz = (zhi - zlo + 1) >= nz;
    fully = (yhi - ylo + 1) >= ny;
    if (fullz) { zlo = 0; zhi = nz - 1; }
    if (fully) { ylo = 0; yhi = ny - 1; }
    zc = zlo;
    yc = ylo;
  }
  bool rows_left = active;
  while (rows_left) {
    // ---- fill: append the segments of the next rows to this lane's list
    int nseg = 0;
    while (rows_left && nseg <= kSegCap - 2) {
      const int zcur = zc, ycur = yc;
      if (++yc > yhi) {
        yc = ylo;
        if (++zc > zhi) rows_left = false;
      }
      int zw = zcur, yw = ycur;
      uint32_t cz_code = 0, cy_code = 0;
      double ez = 0.0, ey = 0.0;
      if (!fullz) {
        if (zcur < 0) { zw = zcur + nz; cz_code = 1; }
        else if (zcur >= nz) { zw = zcur - nz; cz_code = 2; }
        if (zcur < cz) ez = zi - (double)(zcur + 1) * a.len[2];
        else if (zcur > cz) ez = (double)zcur * a.len[2] - zi;
        ez = ez > guard ? ez - guard : 0.0;
      }
      if (!fully) {
        if (ycur < 0) { yw = ycur + ny; cy_code = 1; }
        else if (ycur >= ny) { yw = ycur - ny; cy_code = 2; }
        if (ycur < cy) ey = yi - (double)(ycur + 1) * a.len[1];
        else if (ycur > cy) ey = (double)ycur * a.len[1] - yi;
        ey = ey > guard ? ey - guard : 0.0;
      }
      const double rem = R2 - ez * ez - ey * ey;
      if (rem < 0.0) continue;
      // chord half-width, rounded up generously (it only selects cells)
      const double w = (double)(sqrtf((float)rem) * 1.00001f) + guard;
      const int xlo = (int)floor((xi - w) * a.sc[0]);
      const int xhi = (int)floor((xi + w) * a.sc[0]);
      const int32_t *cs = a.cell_start + (zw * ny + yw) * nx;
      const uint32_t yz = (cy_code << 2) | (cz_code << 4);
      auto push = [&](int c0, int c1, uint32_t code) {  // cells [c0, c1)
        int j0 = cs[c0], j1 = cs[c1];
        if (j1 > j0) {
          segs[nseg][lane_id] = make_uint2((uint32_t)j0, (uint32_t)(j1 - j0) | (code << 24));
          ++nseg;
        }
      };
      if (xhi - xlo + 1 >= nx) {
        push(0, nx, kPerPairImage);
      } else if (fully || fullz) {
        int lo = xlo, hi = xhi;
        if (lo < 0) { push(lo + nx, nx, kPerPairImage); lo = 0; }
        if (hi >= nx) { push(0, hi - nx + 1, kPerPairImage); hi = nx - 1; }
        push(lo, hi + 1, kPerPairImage);
      } else {
        int lo = xlo, hi = xhi;
        if (lo < 0) { push(lo + nx, nx, yz | 1u); lo = 0; }
        if (hi >= nx) { push(0, hi - nx + 1, yz | 2u); hi = nx - 1; }
        push(lo, hi + 1, yz);
      }
    }
    // ---- scan: one flat loop over every candidate of the listed segments
    int sidx = 0, j = 0, jend = 0;
    double shx = 0.0, shy = 0.0, shz = 0.0;
    bool per_pair = false;
    while (true) {
      if (j >= jend) {
        if (sidx >= nseg) break;
        const uint2 sg = segs[sidx][lane_id];
        ++sidx;
        j = (int)sg.x;
        jend = j + (int)(sg.y & 0xffffffu);
        const uint32_t code = sg.y >> 24;
        per_pair = (code & kPerPairImage) != 0;
        shx = code_shift(code & 3u, Lx);
        shy = code_shift((code >> 2) & 3u, Ly);
        shz = code_shift((code >> 4) & 3u, Lz);
      }
      const double4 pj = a.pos[j];
      double dx = xi - pj.x, dy = yi - pj.y, dz = zi - pj.z;
      if (per_pair) {
        dx = dx - Lx * rint(dx / Lx);
        dy = dy - Ly * rint(dy / Ly);
        dz = dz - Lz * rint(dz / Lz);
      } else {
        dx = dx + shx;
        dy = dy + shy;
        dz = dz + shz;
      }
      const double r2 = (dx * dx + dy * dy) + dz * dz;
      bool inc;
      if constexpr (RULE == DCM_PAIR_OWN) {
        inc = r2 < rci2;
      } else {
        double m = rci > pj.w ? rci : pj.w;
        inc = r2 <= m * m;
      }
      if (inc && j != (int)s) {
        interact<PREC, EVM>(acc, dx, dy, dz, r2, sig2);
        ++cnt;
      }
      ++j;
    }
  }
  if (active) {
    const double c24 = 24.0 * a.eps;
    const double Fx = c24 * acc.fx, Fy = c24 * acc.fy, Fz = c24 * acc.fz;
    const int32_t i = a.perm[s];
    a.fx[i] = Fx;
    a.fy[i] = Fy;
    a.fz[i] = Fz;
    if (a.nnbr) a.nnbr[i] = cnt;
    if (!finite3(Fx, Fy, Fz)) atomicOr(a.status, ST_NONFINITE_FORCE);
  }
  // deterministic block partials: E, W[6], pair count
  double v[kPartialSlots];
  v[0] = (double)acc.e * (2.0 * a.eps);
#pragma unroll
  for (int k = 0; k < 6; ++k) v[1 + k] = (double)acc.w[k] * (12.0 * a.eps);
  v[7] = (double)cnt;
  __shared__ double red[kPairBlock / 64][kPartialSlots];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < kPartialSlots; ++k) {
    double t = wave_sum(v[k]);
    if (lane == 0) red[wid][k] = t;
  }
  __syncthreads();
  if (threadIdx.x < kPartialSlots) {
    double t = 0.0;
#pragma unroll
    for (int q = 0; q < kPairBlock / 64; ++q) t += red[q][threadIdx.x];
    a.partials[blockIdx.x * (int64_t)kPartialSlots + threadIdx.x] = t;
  }
}

template <int RULE, int PREC>
static void launch_pair_ev(hipStream_t s, const PairArgs &a, dim3 g, dim3 b) {
  const int evm = ((a.ev_flags & DCM_EV_ENERGY) ? 1 : 0) | ((a.ev_flags & DCM_EV_VIRIAL) ? 2 : 0);
  switch (evm) {
    case 0: hipLaunchKernelGGL((k_pair<RULE, PREC, 0>), g, b, 0, s, a); break;
    case 1: hipLaunchKernelGGL((k_pair<RULE, PREC, 1>), g, b, 0, s, a); break;
    case 2: hipLaunchKernelGGL((k_pair<RULE, PREC, 2>), g, b, 0, s, a); break;
    default: hipLaunchKernelGGL((k_pair<RULE, PREC, 3>), g, b, 0, s, a); break;
  }
}

void launch_pair(hipStream_t s, const PairArgs &a, int rule, int prec) {
  const int64_t blocks = ceil_div(a.n, kPairBlock) > 0 ? ceil_div(a.n, kPairBlock) : 1;
  dim3 g((unsigned)blocks), b(kPairBlock);
  if (rule == DCM_PAIR_OWN) {
    if (prec == DCM_FP64) launch_pair_ev<DCM_PAIR_OWN, DCM_FP64>(s, a, g, b);
    else launch_pair_ev<DCM_PAIR_OWN, DCM_FP32_MIXED>(s, a, g, b);
  } else {
    if (prec == DCM_FP64) launch_pair_ev<DCM_PAIR_MAX, DCM_FP64>(s, a, g, b);
    else launch_pair_ev<DCM_PAIR_MAX, DCM_FP32_MIXED>(s, a, g, b);
  }
}

// Sum the block partials in a fixed order (one workgroup), so the energy,
// virial and pair count do not depend on scheduling.
__global__ __launch_bounds__(256) void k_reduce_partials(const double *__restrict__ partials,
                                                         int64_t blocks, int ev_flags,
                                                         double *energy, double *virial,
                                                         uint64_t *npairs) {
  __shared__ double red[4][kPartialSlots];
  double v[kPartialSlots];
#pragma unroll
  for (int k = 0; k < kPartialSlots; ++k) v[k] = 0.0;
  for (int64_t b = threadIdx.x; b < blocks; b += 256)
#pragma unroll
    for (int k = 0; k < kPartialSlots; ++k) v[k] += partials[b * kPartialSlots + k];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < kPartialSlots; ++k) {
    double t = wave_sum(v[k]);
    if (lane == 0) red[wid][k] = t;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double t[kPartialSlots];
    for (int k = 0; k < kPartialSlots; ++k)
      t[k] = ((red[0][k] + red[1][k]) + red[2][k]) + red[3][k];
    if (energy && (ev_flags & DCM_EV_ENERGY)) *energy = t[0];
    if (virial && (ev_flags & DCM_EV_VIRIAL))
      for (int k = 0; k < 6; ++k) virial[k] = t[1 + k];
    if (npairs && (ev_flags & DCM_EV_COUNTS)) *npairs = (uint64_t)t[7];
  }
}

void launch_reduce_partials(hipStream_t s, const double *partials, int64_t blocks, double eps,
                            int ev_flags, double *energy, double *virial, uint64_t *npairs) {
  (void)eps;
  hipLaunchKernelGGL(k_reduce_partials, dim3(1), dim3(256), 0, s, partials, blocks, ev_flags,
                     energy, virial, npairs);
}

}  // namespace dcm
