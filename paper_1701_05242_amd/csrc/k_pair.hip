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

// Everything one lane needs to find and sum its particle's neighbours; the
// single-system kernel fills it from its arguments, the batched kernel from
// the table entry of the system a work item belongs to.
struct PairView {
  const double4 *pos;            // sorted particles (x, y, z, rc)
  const int32_t *cell_start;     // this system's real cells -> sorted slots
  const int32_t *perm;           // sorted slot -> particle id
  int64_t id0;                   // particle id of the system's first caller index
  const double4 *ext_pos;        // extended (ghost) array
  const int32_t *ext_start;      // this system's extended cells -> extended slots
  int64_t ext_cap;
  int nc[3], h[3], ne[3];
  double len[3], sc[3];
  double rc_bound;
  const unsigned long long *rc_all_bits;  // largest cutoff of the system (rule MAX)
  double *fx, *fy, *fz;
  int32_t *nnbr;
};

// One block of kPairBlock particles: sorted slot s for this lane (active if
// it holds a particle).  Writes the forces and, from lanes 0..7, the block's
// partial sums E, W[6], pair count to partial_out.
template <int RULE, int PREC, int EVM>
__device__ __forceinline__ void pair_block(const PairView &v, int64_t s, bool active, double eps,
                                           double sig2, uint2 (*segs)[kPairBlock],
                                           double (*red)[kPartialSlots], uint32_t *status,
                                           double *partial_out) {
  const int lane_id = threadIdx.x;
  Acc<PREC> acc;
  int cnt = 0;
  const int nx = v.nc[0], ny = v.nc[1], nz = v.nc[2];
  const int hx = v.h[0], hy = v.h[1], hz = v.h[2];
  const int nex = v.ne[0], ney = v.ne[1];
  double xi = 0, yi = 0, zi = 0, rci = 0, rci2 = 0, R2 = 0, guard = 0;
  int zlo = 0, zhi = -1, ylo = 0, yhi = -1, zc = 0, yc = 0, cy = 0, cz = 0, self = -1;
  if (active) {
    const double4 pi = v.pos[s];
    xi = pi.x;
    yi = pi.y;
    zi = pi.z;
    rci = pi.w;
    double R = rci;
    if constexpr (RULE == DCM_PAIR_MAX) {
      double rall = __longlong_as_double((long long)*v.rc_all_bits);
      R = rall > R ? rall : R;
    }
    R = R < v.rc_bound ? R : v.rc_bound;
    rci2 = rci * rci;
    // search radius widened by a hair: rounding in the cell geometry can
    // only add candidates, never drop one
    guard = 1e-9 * (v.len[0] + v.len[1] + v.len[2]);
    const double Rg = R + guard;
    R2 = Rg * Rg;
    const int cx = slab_index(xi, v.sc[0], nx);
    cy = slab_index(yi, v.sc[1], ny);
    cz = slab_index(zi, v.sc[2], nz);
    // the halo holds ceil(rc_bound/len) + 1 cells, so these stay inside it
    zlo = clampi((int)floor((zi - Rg) * v.sc[2]), -hz, nz + hz - 1);
    zhi = clampi((int)floor((zi + Rg) * v.sc[2]), -hz, nz + hz - 1);
    ylo = clampi((int)floor((yi - Rg) * v.sc[1]), -hy, ny + hy - 1);
    yhi = clampi((int)floor((yi + Rg) * v.sc[1]), -hy, ny + hy - 1);
    zc = zlo;
    yc = ylo;
    // this particle's own copy in the extended array
    const int real_cell = (cz * ny + cy) * nx + cx;
    const int ext_cell = ((cz + hz) * ney + (cy + hy)) * nex + (cx + hx);
    self = v.ext_start[ext_cell] + (int)(s - v.cell_start[real_cell]);
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
      if (zcur < cz) ez = zi - (double)(zcur + 1) * v.len[2];
      else if (zcur > cz) ez = (double)zcur * v.len[2] - zi;
      ez = ez > guard ? ez - guard : 0.0;
      if (ycur < cy) ey = yi - (double)(ycur + 1) * v.len[1];
      else if (ycur > cy) ey = (double)ycur * v.len[1] - yi;
      ey = ey > guard ? ey - guard : 0.0;
      const double rem = R2 - ez * ez - ey * ey;
      if (rem < 0.0) continue;
      // chord half-width, rounded up generously (it only selects cells)
      const double w = (double)(sqrtf((float)rem) * 1.00001f) + guard;
      const int xlo = clampi((int)floor((xi - w) * v.sc[0]), -hx, nx + hx - 1);
      const int xhi = clampi((int)floor((xi + w) * v.sc[0]), -hx, nx + hx - 1);
      const int32_t *es = v.ext_start + ((int64_t)(zcur + hz) * ney + (ycur + hy)) * nex + hx;
      int j0 = es[xlo], j1 = es[xhi + 1];
      if (j1 > v.ext_cap) j1 = (int)v.ext_cap;  // overflowed ghosts (flagged at build)
      if (j1 > j0) {
        segs[nseg][lane_id] = make_uint2((uint32_t)j0, (uint32_t)j1);
        ++nseg;
      }
    }
    if (nseg > 0)
      scan_ranges<RULE, PREC, EVM>(segs, nseg, v.ext_pos, self, xi, yi, zi, rci, rci2, sig2, acc,
                                   cnt);
  }
  if (active) {
    const double c24 = 24.0 * eps;
    const double Fx = c24 * acc.fx, Fy = c24 * acc.fy, Fz = c24 * acc.fz;
    const int64_t i = v.perm[s] - v.id0;
    v.fx[i] = Fx;
    v.fy[i] = Fy;
    v.fz[i] = Fz;
    if (v.nnbr) v.nnbr[i] = cnt;
    if (!finite3(Fx, Fy, Fz)) atomicOr(status, ST_NONFINITE_FORCE);
  }
  // deterministic block partials: E, W[6], pair count
  double pv[kPartialSlots];
  pv[0] = (double)acc.e * (2.0 * eps);
#pragma unroll
  for (int k = 0; k < 6; ++k) pv[1 + k] = (double)acc.w[k] * (12.0 * eps);
  pv[7] = (double)cnt;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < kPartialSlots; ++k) {
    double t = wave_sum(pv[k]);
    if (lane == 0) red[wid][k] = t;
  }
  __syncthreads();
  if (threadIdx.x < kPartialSlots) {
    double t = 0.0;
#pragma unroll
    for (int q = 0; q < kPairBlock / 64; ++q) t += red[q][threadIdx.x];
    partial_out[threadIdx.x] = t;
  }
}

template <int RULE, int PREC, int EVM>
__global__ __launch_bounds__(kPairBlock) void k_pair(PairArgs a) {
  __shared__ uint2 segs[kSegCap][kPairBlock];
  __shared__ double red[kPairBlock / 64][kPartialSlots];
  const int64_t lblock = xcd_block(blockIdx.x, gridDim.x, kXcdGroup);
  const int64_t s = lblock * kPairBlock + threadIdx.x;
  PairView v;
  v.pos = a.pos;
  v.cell_start = a.cell_start;
  v.perm = a.perm;
  v.id0 = 0;
  v.ext_pos = a.ext_pos;
  v.ext_start = a.ext_start;
  v.ext_cap = a.ext_cap;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    v.nc[k] = a.nc[k];
    v.h[k] = a.h[k];
    v.ne[k] = a.ne[k];
    v.len[k] = a.len[k];
    v.sc[k] = a.sc[k];
  }
  v.rc_bound = a.rc_bound;
  v.rc_all_bits = &a.ctl->rc_max_bits;
  v.fx = a.fx;
  v.fy = a.fy;
  v.fz = a.fz;
  v.nnbr = a.nnbr;
  pair_block<RULE, PREC, EVM>(v, s, s < a.n, a.eps, a.sigma * a.sigma, segs, red, a.status,
                              a.partials + lblock * kPartialSlots);
}

// Batched form: a persistent grid takes work items (blocks of kPairBlock
// particles of one system) from a queue ordered by estimated cost.  Every
// workgroup leaves the loop once the queue head passes the item count.
template <int RULE, int PREC, int EVM>
__global__ __launch_bounds__(kPairBlock) void k_pair_batched(BatchPairArgs a) {
  __shared__ uint2 segs[kSegCap][kPairBlock];
  __shared__ double red[kPairBlock / 64][kPartialSlots];
  __shared__ int32_t next_item;
  const double sig2 = a.sigma * a.sigma;
  while (true) {
    if (threadIdx.x == 0) next_item = (int32_t)atomicAdd(a.head, 1u);
    __syncthreads();
    const int32_t qi = next_item;
    __syncthreads();
    if (qi >= a.nitems) break;
    const int32_t item = __builtin_amdgcn_readfirstlane(a.queue[qi]);
    const int2 w = a.items[item];
    const int b = __builtin_amdgcn_readfirstlane(w.x);
    const int64_t first = __builtin_amdgcn_readfirstlane(w.y);
    const SysGeom &g = a.sys[b];
    PairView v;
    v.pos = a.pos;
    v.cell_start = a.cell_start + g.cell0;
    v.perm = a.perm;
    v.id0 = g.p0;
    v.ext_pos = a.ext_pos;
    v.ext_start = a.ext_start + g.ext_cell0;
    v.ext_cap = a.ext_cap;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      v.nc[k] = g.nc[k];
      v.h[k] = g.h[k];
      v.ne[k] = g.ne[k];
      v.len[k] = g.len[k];
      v.sc[k] = g.sc[k];
    }
    v.rc_bound = g.rc_cap;
    v.rc_all_bits = a.rc_max_bits + b;
    v.fx = g.fx;
    v.fy = g.fy;
    v.fz = g.fz;
    v.nnbr = g.nnbr;
    const int64_t local = first + threadIdx.x;
    pair_block<RULE, PREC, EVM>(v, g.p0 + local, local < g.n, a.eps, sig2, segs, red, a.status,
                                a.partials + (int64_t)item * kPartialSlots);
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

template <int RULE, int PREC>
static void launch_pair_batched_ev(hipStream_t s, const BatchPairArgs &a, dim3 g, dim3 b) {
  const int evm = ((a.ev_flags & DCM_EV_ENERGY) ? 1 : 0) | ((a.ev_flags & DCM_EV_VIRIAL) ? 2 : 0);
  switch (evm) {
    case 0: hipLaunchKernelGGL((k_pair_batched<RULE, PREC, 0>), g, b, 0, s, a); break;
    case 1: hipLaunchKernelGGL((k_pair_batched<RULE, PREC, 1>), g, b, 0, s, a); break;
    case 2: hipLaunchKernelGGL((k_pair_batched<RULE, PREC, 2>), g, b, 0, s, a); break;
    default: hipLaunchKernelGGL((k_pair_batched<RULE, PREC, 3>), g, b, 0, s, a); break;
  }
}

// Resident workgroups of the persistent kernel: what the occupancy allows on
// every compute unit, never more than the number of items.
static int64_t persistent_grid(int rule, int prec, int64_t nitems) {
  static int cached[2][2] = {{0, 0}, {0, 0}};
  int &per_cu = cached[rule][prec];
  if (per_cu == 0) {
    const void *fn;
    if (rule == DCM_PAIR_OWN)
      fn = prec == DCM_FP64 ? (const void *)k_pair_batched<DCM_PAIR_OWN, DCM_FP64, 3>
                            : (const void *)k_pair_batched<DCM_PAIR_OWN, DCM_FP32_MIXED, 3>;
    else
      fn = prec == DCM_FP64 ? (const void *)k_pair_batched<DCM_PAIR_MAX, DCM_FP64, 3>
                            : (const void *)k_pair_batched<DCM_PAIR_MAX, DCM_FP32_MIXED, 3>;
    int blocks = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, fn, kPairBlock, 0) != hipSuccess ||
        blocks < 1)
      blocks = 1;
    per_cu = blocks;
  }
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      cus < 1)
    cus = 1;
  int64_t g = (int64_t)per_cu * cus;
  return g < nitems ? g : (nitems > 0 ? nitems : 1);
}

void launch_pair_batched(hipStream_t s, const BatchPairArgs &a, int rule, int prec) {
  if (a.nitems <= 0) return;
  dim3 g((unsigned)persistent_grid(rule, prec, a.nitems)), b(kPairBlock);
  if (rule == DCM_PAIR_OWN) {
    if (prec == DCM_FP64) launch_pair_batched_ev<DCM_PAIR_OWN, DCM_FP64>(s, a, g, b);
    else launch_pair_batched_ev<DCM_PAIR_OWN, DCM_FP32_MIXED>(s, a, g, b);
  } else {
    if (prec == DCM_FP64) launch_pair_batched_ev<DCM_PAIR_MAX, DCM_FP64>(s, a, g, b);
    else launch_pair_batched_ev<DCM_PAIR_MAX, DCM_FP32_MIXED>(s, a, g, b);
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
