// Dynamic-cutoff Lennard-Jones force, energy and virial (Section 2.4,
// Algorithm 2.3, Eqs. 2-3) over the linked cells of Section 2.3.
//
// One lane owns one particle i (particles in cell order, so a wavefront
// covers neighbouring particles with similar cutoffs).  Instead of storing
// the neighbour list of Algorithm 2.2, each lane enumerates the cell rows
// (fixed y and z cell; consecutive x cells are consecutive in memory) that can
// hold a j within its search radius and trims each row to the chord of the
// search sphere -- the small-cell traversal of Section 2.3.  The rows are
// walked in the ghost-extended cell grid, where periodic images sit in halo
// cells with their coordinates already shifted, so every row is one
// contiguous index range and a separation is a plain difference.  A lane
// writes its rows' ranges into a private LDS list, then runs one flat loop
// over all their candidates, so lanes with different row lengths never wait
// for each other row by row.  No Newton-3 update is made (Section 2.4): a
// lane writes only its own particle.
#include "dcm_device.hpp"
#include "dcm_internal.hpp"

namespace dcm {

constexpr int kPairBlock = 256;
#ifndef DCM_PAIR_SEGCAP
#define DCM_PAIR_SEGCAP 24
#endif
constexpr int kSegCap = DCM_PAIR_SEGCAP;  // row ranges per lane per chunk (LDS: 8 B each)
#ifndef DCM_PAIR_XCD_GROUP
#define DCM_PAIR_XCD_GROUP 16
#endif
constexpr int kXcdGroup = DCM_PAIR_XCD_GROUP;
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

// Test candidate j (position pj) against lane particle i and accumulate it.
template <int RULE, int PREC, int EVM>
__device__ __forceinline__ void candidate(const double4 &pj, int j, int self, double xi,
                                          double yi, double zi, double rci, double rci2,
                                          double sig2, Acc<PREC> &acc, int &cnt) {
  const double dx = xi - pj.x, dy = yi - pj.y, dz = zi - pj.z;
  const double r2 = (dx * dx + dy * dy) + dz * dz;
  bool inc;
  if constexpr (RULE == DCM_PAIR_OWN) {
    inc = r2 < rci2;
  } else {
    double m = rci > pj.w ? rci : pj.w;
    inc = r2 <= m * m;
  }
  if (inc && j != self) {
    interact<PREC, EVM>(acc, dx, dy, dz, r2, sig2);
    ++cnt;
  }
}

// One flat loop over every candidate j of this lane's first nseg listed
// ranges [seg.x, seg.y) of the extended array, two candidates per trip with
// two register sets: each candidate's position is loaded a full candidate
// ahead of its use, without copying registers between trips.
template <int RULE, int PREC, int EVM>
__device__ __forceinline__ void scan_ranges(const uint2 (*segs)[kPairBlock], int nseg,
                                            const double4 *__restrict__ pos, int self, double xi,
                                            double yi, double zi, double rci, double rci2,
                                            double sig2, Acc<PREC> &acc, int &cnt) {
  const int lane_id = threadIdx.x;
  int sidx = 1;
  uint2 sg = segs[0][lane_id];
  int jend = (int)sg.y;
  // next candidate after j, or -1 when the list is exhausted
  auto advance = [&](int j) -> int {
    int jn = j + 1;
    if (jn >= jend) {
      if (sidx < nseg) {
        sg = segs[sidx][lane_id];
        ++sidx;
        jn = (int)sg.x;
        jend = (int)sg.y;
      } else {
        jn = -1;
      }
    }
    return jn;
  };
  int ja = (int)sg.x;
  double4 A = pos[ja];
  int jb = advance(ja);
  while (true) {
    double4 B;
    if (jb >= 0) B = pos[jb];
    const int jc = jb >= 0 ? advance(jb) : -1;
    candidate<RULE, PREC, EVM>(A, ja, self, xi, yi, zi, rci, rci2, sig2, acc, cnt);
    if (jb < 0) break;
    if (jc >= 0) A = pos[jc];
    const int jd = jc >= 0 ? advance(jc) : -1;
    candidate<RULE, PREC, EVM>(B, jb, self, xi, yi, zi, rci, rci2, sig2, acc, cnt);
    if (jc < 0) break;
    ja = jc;
    jb = jd;
  }
}

__device__ __forceinline__ int clampi(int v, int lo, int hi) {
  return v < lo ? lo : (v > hi ? hi : v);
}

template <int RULE, int PREC, int EVM>
__global__ __launch_bounds__(kPairBlock) void k_pair(PairArgs a) {
  __shared__ uint2 segs[kSegCap][kPairBlock];
  const int lane_id = threadIdx.x;
  const int64_t lblock = xcd_block(blockIdx.x, gridDim.x, kXcdGroup);
  const int64_t s = lblock * kPairBlock + threadIdx.x;
  const bool active = s < a.n;
  Acc<PREC> acc;
  int cnt = 0;
  const int nx = a.nc[0], ny = a.nc[1], nz = a.nc[2];
  const int hx = a.h[0], hy = a.h[1], hz = a.h[2];
  const int nex = a.ne[0], ney = a.ne[1];
  const double sig2 = a.sigma * a.sigma;
  double xi = 0, yi = 0, zi = 0, rci = 0, rci2 = 0, R2 = 0, guard = 0;
  int zlo = 0, zhi = -1, ylo = 0, yhi = -1, zc = 0, yc = 0, cy = 0, cz = 0, self = -1;
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
    R = R < a.rc_bound ? R : a.rc_bound;
    rci2 = rci * rci;
    // search radius widened by a hair: rounding in the cell geometry can
    // only add candidates, never drop one
    guard = 1e-9 * (a.len[0] + a.len[1] + a.len[2]);
    const double Rg = R + guard;
    R2 = Rg * Rg;
    const int cx = slab_index(xi, a.sc[0], nx);
    cy = slab_index(yi, a.sc[1], ny);
    cz = slab_index(zi, a.sc[2], nz);
    // the halo holds ceil(rc_bound/len) + 1 cells, so these stay inside it
    zlo = clampi((int)floor((zi - Rg) * a.sc[2]), -hz, nz + hz - 1);
    zhi = clampi((int)floor((zi + Rg) * a.sc[2]), -hz, nz + hz - 1);
    ylo = clampi((int)floor((yi - Rg) * a.sc[1]), -hy, ny + hy - 1);
    yhi = clampi((int)floor((yi + Rg) * a.sc[1]), -hy, ny + hy - 1);
    zc = zlo;
    yc = ylo;
    // this particle's own copy in the extended array
    const int real_cell = (cz * ny + cy) * nx + cx;
    const int ext_cell = ((cz + hz) * ney + (cy + hy)) * nex + (cx + hx);
    self = a.ext_start[ext_cell] + (int)(s - a.cell_start[real_cell]);
  }
  bool rows_left = active;
  while (rows_left) {
    // ---- fill: append the ranges of the next rows to this lane's list
    int nseg = 0;
    while (rows_left && nseg < kSegCap) {
      const int zcur = zc, ycur = yc;
      if (++yc > yhi) {
        yc = ylo;
        if (++zc > zhi) rows_left = false;
      }
      double ez = 0.0, ey = 0.0;
      if (zcur < cz) ez = zi - (double)(zcur + 1) * a.len[2];
      else if (zcur > cz) ez = (double)zcur * a.len[2] - zi;
      ez = ez > guard ? ez - guard : 0.0;
      if (ycur < cy) ey = yi - (double)(ycur + 1) * a.len[1];
      else if (ycur > cy) ey = (double)ycur * a.len[1] - yi;
      ey = ey > guard ? ey - guard : 0.0;
      const double rem = R2 - ez * ez - ey * ey;
      if (rem < 0.0) continue;
      // chord half-width, rounded up generously (it only selects cells)
      const double w = (double)(sqrtf((float)rem) * 1.00001f) + guard;
      const int xlo = clampi((int)floor((xi - w) * a.sc[0]), -hx, nx + hx - 1);
      const int xhi = clampi((int)floor((xi + w) * a.sc[0]), -hx, nx + hx - 1);
      const int32_t *es = a.ext_start + ((int64_t)(zcur + hz) * ney + (ycur + hy)) * nex + hx;
      int j0 = es[xlo], j1 = es[xhi + 1];
      if (j1 > a.ext_cap) j1 = (int)a.ext_cap;  // overflowed ghosts (flagged at build)
      if (j1 > j0) {
        segs[nseg][lane_id] = make_uint2((uint32_t)j0, (uint32_t)j1);
        ++nseg;
      }
    }
    if (nseg > 0)
      scan_ranges<RULE, PREC, EVM>(segs, nseg, a.ext_pos, self, xi, yi, zi, rci, rci2, sig2, acc,
                                   cnt);
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
    a.partials[lblock * kPartialSlots + threadIdx.x] = t;
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
