// Cutoff assignment (Section 2.2) and linked-cell binning (Section 2.3).
#include "dcm_device.hpp"
#include "dcm_internal.hpp"

namespace dcm {

// ----------------------------------------------------- cutoff assignment
// delta_i: periodic trilinear interpolation of the voxel-centred distances at
// the particle; rc_i = rc_max - (rc_max - rc_min) * min(delta_i/ramp, 1).
// SWEEP: D is the sweep's own pair of buffers (D, D2) and its pass flags,
// read as the sweep's final pass would write the field: the buffer of the
// first pass that changed nothing, each value capped at `cap`; a sweep that
// ran out of passes is flagged here.
// SLOTS: cells built before the cutoffs were known (their records carry no
// cutoff): the threads walk the sorted slots, particle p = perm[slot], and
// each record takes its particle's cutoff, clamped to [0, rc_cap] as the
// cell build's gather clamps it (a value outside is flagged).
template <bool SWEEP, bool SLOTS>
__global__ __launch_bounds__(256) void k_assign_cutoffs(
    const double *__restrict__ x, const double *__restrict__ y, const double *__restrict__ z,
    int64_t n, double Lx, double Ly, double Lz, int nx, int ny, int nz, double sx, double sy,
    double sz, const double *__restrict__ D, double rc_min, double rc_max, double ramp,
    double *__restrict__ delta, double *__restrict__ rc, const double *__restrict__ D2,
    const uint32_t *__restrict__ flags, int max_steps, double cap, uint32_t *status,
    const int32_t *__restrict__ perm, double4 *__restrict__ sorted, double rc_cap) {
  if constexpr (SWEEP) {
    int last = max_steps;
    for (int q = 1; q <= max_steps; ++q)
      if (flags[q] == 0u) {
        last = q;
        break;
      }
    if (last & 1) D = D2;
    if (blockIdx.x == 0 && threadIdx.x == 0 && flags[max_steps] != 0u)
      atomicOr(status, ST_NOT_CONVERGED);
  }
  // the record's cutoff as the gather writes it
  auto record = [&](int64_t slot, double r) {
    if constexpr (SLOTS) {
      if (!(r >= 0.0) || r > rc_cap) atomicOr(status, ST_RC_RANGE);
      sorted[slot].w = (r >= 0.0) ? (r < rc_cap ? r : rc_cap) : 0.0;  // NaN -> 0
    }
  };
  for (int64_t it = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; it < n;
       it += (int64_t)gridDim.x * blockDim.x) {
    int64_t p = it;
    if constexpr (SLOTS) p = perm[it];
    double px = x[p], py = y[p], pz = z[p];
    if (!finite3(px, py, pz)) {
      if (delta) delta[p] = __builtin_nan("");
      rc[p] = rc_max;
      record(it, rc_max);
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
    auto DV = [&](int i, int j, int k) {
      const double v = D[((int64_t)k * ny + j) * nx + i];
      if constexpr (SWEEP) return v > cap ? cap : v;
      else return v;
    };
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
    const double r = rc_max - (rc_max - rc_min) * q;
    rc[p] = r;
    record(it, r);
  }
}

void launch_assign_cutoffs(hipStream_t s, const double *x, const double *y, const double *z,
                           int64_t n, const double L[3], const int32_t nv[3],
                           const double sc[3], const double *dist, dcm_rule rule,
                           double *delta, double *rc) {
  if (n <= 0) return;
  int64_t b = ceil_div(n, 256);
  if (b > 16384) b = 16384;
  hipLaunchKernelGGL((k_assign_cutoffs<false, false>), dim3((unsigned)b), dim3(256), 0, s, x, y,
                     z, n, L[0], L[1], L[2], nv[0], nv[1], nv[2], sc[0], sc[1], sc[2], dist,
                     rule.rc_min, rule.rc_max, rule.ramp, delta, rc, nullptr, nullptr, 0, 0.0,
                     nullptr, nullptr, nullptr, 0.0);
}

void launch_assign_cutoffs_sweep(hipStream_t s, const double *x, const double *y,
                                 const double *z, int64_t n, const double L[3],
                                 const int32_t nv[3], const double sc[3], const double *dA,
                                 const double *dB, const uint32_t *flags, int max_steps,
                                 double rc_grid, dcm_rule rule, double *delta, double *rc,
                                 uint32_t *status, const int32_t *perm, double4 *sorted,
                                 double rc_cap) {
  if (n <= 0) return;
  int64_t b = ceil_div(n, 256);
  if (b > 16384) b = 16384;
  if (perm)
    hipLaunchKernelGGL((k_assign_cutoffs<true, true>), dim3((unsigned)b), dim3(256), 0, s, x, y,
                       z, n, L[0], L[1], L[2], nv[0], nv[1], nv[2], sc[0], sc[1], sc[2], dA,
                       rule.rc_min, rule.rc_max, rule.ramp, delta, rc, dB, flags, max_steps,
                       rc_grid, status, perm, sorted, rc_cap);
  else
    hipLaunchKernelGGL((k_assign_cutoffs<true, false>), dim3((unsigned)b), dim3(256), 0, s, x, y,
                       z, n, L[0], L[1], L[2], nv[0], nv[1], nv[2], sc[0], sc[1], sc[2], dA,
                       rule.rc_min, rule.rc_max, rule.ramp, delta, rc, dB, flags, max_steps,
                       rc_grid, status, nullptr, nullptr, 0.0);
}

// ------------------------------------------------------------ cell count
__global__ __launch_bounds__(256) void k_cell_count(
    const double *__restrict__ x, const double *__restrict__ y, const double *__restrict__ z,
    const double *__restrict__ rc, int64_t n, double Lx, double Ly, double Lz, int nx, int ny,
    int nz, double sx, double sy, double sz, double rc_cap, int32_t *__restrict__ cell_of,
    int32_t *count, unsigned long long *__restrict__ block_max, uint32_t *__restrict__ xq,
    uint32_t *status) {
  unsigned long long rmax = 0;
  // uniform trip count: every lane reaches the run-aggregated atomic
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t base = blockIdx.x * (int64_t)blockDim.x; base < n; base += stride) {
    const int64_t i = base + threadIdx.x;
    const bool valid = i < n;
    int c = 0;
    if (valid) {
      // rc null: the cutoffs are not known yet (the cutoff assignment adds them)
      double px = x[i], py = y[i], pz = z[i], r = rc ? rc[i] : 0.0;
      uint32_t q = 0;
      if (finite3(px, py, pz)) {
        const double wx = wrap_coord(px, Lx);
        int cx = slab_index(wx, sx, nx);
        int cy = slab_index(wrap_coord(py, Ly), sy, ny);
        int cz = slab_index(wrap_coord(pz, Lz), sz, nz);
        c = (cz * ny + cy) * nx + cx;
        q = x_key(wx, sx, cx);
      } else {
        atomicOr(status, ST_NONFINITE_POS);
      }
      if (xq) xq[i] = q;
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
  // the workgroup's largest cutoff, stored without atomics (one address
  // shared by every workgroup would serialise them)
  __shared__ unsigned long long wmax[4];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    unsigned long long o = __shfl_xor(rmax, off, 64);
    rmax = o > rmax ? o : rmax;
  }
  if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = rmax;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long m = wmax[0];
    for (int w = 1; w < 4; ++w) m = wmax[w] > m ? wmax[w] : m;
    block_max[blockIdx.x] = m;
  }
}

// Largest of the workgroup maxima into the control block.
__global__ __launch_bounds__(1024) void k_reduce_rcmax(const unsigned long long *__restrict__ bm,
                                                       int64_t nb, Ctl *ctl) {
  __shared__ unsigned long long wmax[16];
  unsigned long long m = 0;
  for (int64_t b = threadIdx.x; b < nb; b += 1024) m = bm[b] > m ? bm[b] : m;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    unsigned long long o = __shfl_xor(m, off, 64);
    m = o > m ? o : m;
  }
  if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < 16; ++w) m = wmax[w] > m ? wmax[w] : m;
    m = wmax[0] > m ? wmax[0] : m;
    ctl->rc_max_bits = m;
    ctl->big_cells = 0u;  // for the cell sort that follows
  }
}

int64_t cell_count_blocks(int64_t n) {
  int64_t b = ceil_div(n, 256);
  if (b > 16384) b = 16384;
  return b < 1 ? 1 : b;
}

void launch_cell_count(hipStream_t s, const double *x, const double *y, const double *z,
                       const double *rc, int64_t n, const double L[3], const int32_t nc[3],
                       const double sc[3], double rc_cap, int32_t *cell_of, int32_t *cell_count,
                       unsigned long long *block_max, uint32_t *xq, Ctl *ctl, uint32_t *status) {
  const int64_t b = cell_count_blocks(n);
  if (n > 0)
    hipLaunchKernelGGL(k_cell_count, dim3((unsigned)b), dim3(256), 0, s, x, y, z, rc, n, L[0],
                       L[1], L[2], nc[0], nc[1], nc[2], sc[0], sc[1], sc[2], rc_cap, cell_of,
                       cell_count, block_max, xq, status);
  hipLaunchKernelGGL(k_reduce_rcmax, dim3(1), dim3(1024), 0, s, block_max, n > 0 ? b : 0, ctl);
}

// ------------------------------------------------------- exclusive scan
// Three phases over tiles of kScanTile elements: tile totals, one workgroup
// scanning the totals, then each tile's local scan plus its offset.  A thread
// owns kScanPer consecutive elements, read and written as int4.
constexpr int kScanThreads = 256;
constexpr int kScanPer = 16;
constexpr int kScanTile = kScanThreads * kScanPer;
constexpr int kTotalsThreads = 1024;
constexpr int64_t kScanSumTiles = 4096;  // up to this many tiles: no pass over the totals

int64_t scan_tmp_elems(int64_t n) { return ceil_div(n, kScanTile) + 1; }

// Inclusive scan over the 64 lanes of a wavefront.
__device__ __forceinline__ int32_t wave_inclusive_scan(int32_t v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int32_t o = __shfl_up(v, off, 64);
    if (lane >= off) v += o;
  }
  return v;
}

// Exclusive scan over the workgroup (NW wavefronts); lds holds NW entries.
template <int NW>
__device__ __forceinline__ int32_t block_exclusive_scan(int32_t v, int32_t *lds, int32_t *total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int32_t incl = wave_inclusive_scan(v);
  if (lane == 63) lds[w] = incl;
  __syncthreads();
  int32_t before = 0, all = 0;
#pragma unroll
  for (int k = 0; k < NW; ++k) {
    const int32_t t = lds[k];
    before += k < w ? t : 0;
    all += t;
  }
  __syncthreads();  // lds may be reused after this
  *total = all;
  return before + incl - v;
}

// this thread's kScanPer elements starting at base (zeros past n)
__device__ __forceinline__ void load_run(const int32_t *__restrict__ in, int64_t base, int64_t n,
                                         int32_t (&v)[kScanPer]) {
  if (base + kScanPer <= n) {
    const int4 *p = reinterpret_cast<const int4 *>(in + base);
#pragma unroll
    for (int q = 0; q < kScanPer / 4; ++q) {
      const int4 t = p[q];
      v[4 * q] = t.x;
      v[4 * q + 1] = t.y;
      v[4 * q + 2] = t.z;
      v[4 * q + 3] = t.w;
    }
  } else {
#pragma unroll
    for (int q = 0; q < kScanPer; ++q) v[q] = base + q < n ? in[base + q] : 0;
  }
}

__global__ __launch_bounds__(kScanThreads) void k_scan_tiles(const int32_t *__restrict__ in,
                                                             int64_t n, int32_t *tile_sum) {
  __shared__ int32_t lds[kScanThreads / 64];
  const int64_t base = blockIdx.x * (int64_t)kScanTile + threadIdx.x * kScanPer;
  int32_t v[kScanPer];
  load_run(in, base, n, v);
  int32_t s = 0;
#pragma unroll
  for (int q = 0; q < kScanPer; ++q) s += v[q];
  int32_t total;
  block_exclusive_scan<kScanThreads / 64>(s, lds, &total);
  if (threadIdx.x == 0) tile_sum[blockIdx.x] = total;
}

// Exclusive scan of the tile totals in place; each thread owns a run of
// consecutive tiles.
__global__ __launch_bounds__(kTotalsThreads) void k_scan_totals(int32_t *tile_sum, int64_t ntiles,
                                                                int32_t *out_last) {
  __shared__ int32_t lds[kTotalsThreads / 64];
  const int64_t per = (ntiles + kTotalsThreads - 1) / kTotalsThreads;
  const int64_t t0 = threadIdx.x * per;
  const int64_t t1 = t0 + per < ntiles ? t0 + per : ntiles;
  int32_t s = 0;
  for (int64_t t = t0; t < t1; ++t) s += tile_sum[t];
  int32_t total;
  int32_t run = block_exclusive_scan<kTotalsThreads / 64>(s, lds, &total);
  for (int64_t t = t0; t < t1; ++t) {
    const int32_t v = tile_sum[t];
    tile_sum[t] = run;
    run += v;
  }
  if (threadIdx.x == 0) *out_last = total;
}

// Each tile's local scan plus its offset: the scanned tile totals (SUM
// false), or the sum of the raw totals of the tiles before it (SUM true: no
// separate pass over the totals; the last tile also writes out[n]).
template <bool SUM>
__global__ __launch_bounds__(kScanThreads) void k_scan_apply(const int32_t *__restrict__ in,
                                                             int64_t n,
                                                             const int32_t *__restrict__ tile_off,
                                                             int32_t *__restrict__ out) {
  __shared__ int32_t lds[kScanThreads / 64];
  int32_t off;
  if constexpr (SUM) {
    int32_t pre = 0;
    for (int64_t t = threadIdx.x; t < (int64_t)blockIdx.x; t += kScanThreads) pre += tile_off[t];
    block_exclusive_scan<kScanThreads / 64>(pre, lds, &off);
  } else {
    off = tile_off[blockIdx.x];
  }
  const int64_t base = blockIdx.x * (int64_t)kScanTile + threadIdx.x * kScanPer;
  int32_t v[kScanPer];
  load_run(in, base, n, v);
  int32_t s = 0;
#pragma unroll
  for (int q = 0; q < kScanPer; ++q) s += v[q];
  int32_t total;
  int32_t run = block_exclusive_scan<kScanThreads / 64>(s, lds, &total) + off;
  if (SUM && blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) out[n] = off + total;
  int32_t o[kScanPer];
#pragma unroll
  for (int q = 0; q < kScanPer; ++q) {
    o[q] = run;
    run += v[q];
  }
  if (base + kScanPer <= n) {
    int4 *p = reinterpret_cast<int4 *>(out + base);
#pragma unroll
    for (int q = 0; q < kScanPer / 4; ++q)
      p[q] = make_int4(o[4 * q], o[4 * q + 1], o[4 * q + 2], o[4 * q + 3]);
  } else {
#pragma unroll
    for (int q = 0; q < kScanPer; ++q)
      if (base + q < n) out[base + q] = o[q];
  }
}

void launch_exclusive_scan(hipStream_t s, const int32_t *in, int32_t *out, int64_t n,
                           int32_t *tmp) {
  // out has n + 1 entries; out[n] = total.  in and out are 16-byte aligned.
  int64_t ntiles = ceil_div(n, kScanTile);
  if (ntiles < 1) ntiles = 1;
  hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)ntiles), dim3(kScanThreads), 0, s, in, n, tmp);
  if (ntiles <= kScanSumTiles) {
    // each tile sums the totals before it (at most kScanSumTiles / 256 reads
    // per thread): two launches
    hipLaunchKernelGGL(k_scan_apply<true>, dim3((unsigned)ntiles), dim3(kScanThreads), 0, s, in,
                       n, tmp, out);
    return;
  }
  hipLaunchKernelGGL(k_scan_totals, dim3(1), dim3(kTotalsThreads), 0, s, tmp, ntiles, out + n);
  hipLaunchKernelGGL(k_scan_apply<false>, dim3((unsigned)ntiles), dim3(kScanThreads), 0, s, in, n,
                     tmp, out);
}

// ------------------------------------------------ scatter + stable order
// Slot of every particle inside its cell: perm[slot] = id, skey[slot] = its
// x key.
__global__ __launch_bounds__(256) void k_cell_scatter(const int32_t *__restrict__ cell_of,
                                                      int64_t n,
                                                      const int32_t *__restrict__ cell_start,
                                                      int32_t *fill, int32_t *__restrict__ perm,
                                                      const uint32_t *__restrict__ xq,
                                                      uint32_t *__restrict__ skey) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t base = blockIdx.x * (int64_t)blockDim.x; base < n; base += stride) {
    const int64_t i = base + threadIdx.x;
    const bool valid = i < n;
    const int c = valid ? cell_of[i] : 0;
    const int slot = wave_run_slot(fill, (uint32_t)c, valid);
    if (valid) {
      const int64_t p = cell_start[c] + slot;
      perm[p] = (int32_t)i;
      skey[p] = xq[i];
    }
  }
}

void launch_cell_scatter(hipStream_t s, const int32_t *cell_of, int64_t n,
                         const int32_t *cell_start, int32_t *cell_fill, int32_t *perm,
                         const uint32_t *xq, uint32_t *skey) {
  if (n <= 0) return;
  int64_t b = ceil_div(n, 256);
  if (b > 16384) b = 16384;
  hipLaunchKernelGGL(k_cell_scatter, dim3((unsigned)b), dim3(256), 0, s, cell_of, n, cell_start,
                     cell_fill, perm, xq, skey);
}

// Atomic slots give an arbitrary order inside a cell; sort each cell's
// entries by (x key, caller index) so the layout (and every FP sum) is
// reproducible and each cell's particles are in x order.  Cells of at most
// kSmallCell entries are ranked one thread per particle (k_cell_rank);
// larger cells go to a list that whole workgroups sort (k_cell_sort_big).
constexpr int kSmallCell = 32;
constexpr int kSortChunk = 4096;  // entries a workgroup sorts at once in LDS
constexpr int kBigSortBlocks = 256;

// Order of two particles of one cell: by x key, then by caller index (the
// keys are x positions quantised to 2^-20 of the cell, so a cell's particles
// end up in x order and every extended row is x-sorted).
__device__ __forceinline__ uint64_t sort_key(const uint32_t *__restrict__ xq, int i) {
  return ((uint64_t)xq[i] << 32) | (uint32_t)i;
}

// A cell's sub-cell word from the x keys of its slots [a, b): nibble k
// (k = 0..6) counts its particles with x keys below (k + 1)/8 of the cell --
// with the particles in key order, the first slot of sub-cell k + 1 is the
// cell's first plus that count -- and nibble 7 counts them all; 0 (no
// sub-cells) for a cell of more than 15.  A nibble histogram of the
// sub-cells times 0x11111111 is its prefix sums.
__device__ __forceinline__ uint32_t sub_word(const uint32_t *__restrict__ skey, int a, int b) {
  if (b - a > 15) return 0u;
  uint32_t hist = 0;
  for (int p = a; p < b; ++p) hist += 1u << (4 * (skey[p] >> (20 - kXSubLog)));
  return hist * 0x11111111u;
}

// One thread per cell: its sub-cell word, and a cell of more than
// kSmallCell particles goes to the list that whole workgroups sort
// (k_cell_sort_big).
__global__ __launch_bounds__(256) void k_cell_small(const int32_t *__restrict__ cell_start,
                                                    int64_t ncell,
                                                    const uint32_t *__restrict__ skey,
                                                    uint32_t *__restrict__ qword,
                                                    int32_t *__restrict__ big_list,
                                                    uint32_t *big_count) {
  for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < ncell;
       c += (int64_t)gridDim.x * blockDim.x) {
    const int a = cell_start[c], b = cell_start[c + 1];
    if (qword) qword[c] = sub_word(skey, a, b);
    if (b - a > kSmallCell) big_list[atomicAdd(big_count, 1u)] = (int32_t)c;
  }
}

// One thread per slot of the cell-scattered order perm (x keys skey): a
// particle of a small cell moves to its cell's start plus its rank there
// (the count of the cell's particles with smaller (x key, id)); a particle
// of a large cell keeps its slot.  out receives the result; no thread waits
// on another.
// The sorted record of particle i: (x, y, z) wrapped into the box (0 when
// not finite) and rc clamped to [0, rc_cap] (NaN -> 0).
__device__ __forceinline__ double4 gather_record(const GatherOut &go, double px, double py,
                                                 double pz, double r) {
  double4 o;
  if (finite3(px, py, pz)) {
    o.x = wrap_coord(px, go.L[0]);
    o.y = wrap_coord(py, go.L[1]);
    o.z = wrap_coord(pz, go.L[2]);
  } else {
    o.x = o.y = o.z = 0.0;
  }
  o.w = (r >= 0.0) ? (r < go.rc_cap ? r : go.rc_cap) : 0.0;
  return o;
}

__device__ __forceinline__ double4 gather_record(const GatherOut &go, int i) {
  return gather_record(go, go.x[i], go.y[i], go.z[i], go.rc ? go.rc[i] : 0.0);
}

// GATHER: a particle of a small cell also writes its sorted record at its
// final slot (the gather of the sorted copy done here, not in a pass of its
// own); out is then the final order.
template <bool GATHER>
__global__ __launch_bounds__(256) void k_cell_rank(const int32_t *__restrict__ cell_start,
                                                   const int32_t *__restrict__ cell_of,
                                                   const int32_t *__restrict__ perm, int64_t n,
                                                   const uint32_t *__restrict__ skey,
                                                   int32_t *__restrict__ out, GatherOut go) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n;
       p += (int64_t)gridDim.x * blockDim.x) {
    const int i = perm[p];
    // the record's inputs are read while the cell's keys are counted
    double px = 0.0, py = 0.0, pz = 0.0, pr = 0.0;
    if constexpr (GATHER) {
      px = go.x[i];
      py = go.y[i];
      pz = go.z[i];
      pr = go.rc ? go.rc[i] : 0.0;
    }
    const int c = cell_of[i];
    const int a = cell_start[c], b = cell_start[c + 1];
    if (b - a > kSmallCell) {
      out[p] = i;
      continue;
    }
    const uint32_t ki = skey[p];
    int r = 0;
    // four keys per round, all read before they are compared
    for (int q0 = a; q0 < b; q0 += 4) {
      uint32_t kj[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) kj[u] = q0 + u < b ? skey[q0 + u] : 0xffffffffu;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if (q0 + u >= b) continue;
        r += kj[u] < ki ? 1 : 0;
        if (kj[u] == ki) r += perm[q0 + u] < i ? 1 : 0;  // equal keys (rare): by id
      }
    }
    out[a + r] = i;
    if constexpr (GATHER) go.sorted[a + r] = gather_record(go, px, py, pz, pr);
  }
}

// One workgroup per listed cell: chunks of kSortChunk entries are sorted in
// LDS (bitonic), then runs are merged pairwise, each entry moving to its own
// offset in its run plus the count of smaller keys in the partner run (keys
// are distinct: they end in the caller index), ping-ponging between perm and
// tmp.  Entries are caller indices; their keys are looked up (sort_key).
template <bool GATHER>
__global__ __launch_bounds__(256) void k_cell_sort_big(const int32_t *__restrict__ cell_start,
                                                       int32_t *perm, int32_t *tmp,
                                                       const uint32_t *__restrict__ xq,
                                                       const int32_t *__restrict__ big_list,
                                                       const uint32_t *big_count, GatherOut go) {
  __shared__ int32_t buf[kSortChunk];
  const int tid = threadIdx.x;
  const uint32_t nbig = *big_count;
  for (uint32_t q = blockIdx.x; q < nbig; q += gridDim.x) {
    const int64_t c = big_list[q];
    const int a = cell_start[c], n = cell_start[c + 1] - a;
    for (int c0 = 0; c0 < n; c0 += kSortChunk) {
      const int len = n - c0 < kSortChunk ? n - c0 : kSortChunk;
      int P = 1;
      while (P < len) P <<= 1;
      // padding entries (-1) sort after every particle
      for (int i = tid; i < P; i += 256) buf[i] = i < len ? perm[a + c0 + i] : -1;
      __syncthreads();
      auto key = [&](int v) -> uint64_t { return v < 0 ? ~uint64_t(0) : sort_key(xq, v); };
      for (int k = 2; k <= P; k <<= 1)
        for (int j = k >> 1; j > 0; j >>= 1) {
          for (int i = tid; i < P; i += 256) {
            const int l = i ^ j;
            if (l > i) {
              const int u = buf[i], w = buf[l];
              if ((key(u) > key(w)) == ((i & k) == 0)) {
                buf[i] = w;
                buf[l] = u;
              }
            }
          }
          __syncthreads();
        }
      for (int i = tid; i < len; i += 256) perm[a + c0 + i] = buf[i];
      __syncthreads();
    }
    int32_t *src = perm + a, *dst = tmp + a;
    for (int L = kSortChunk; L < n; L <<= 1) {
      for (int p = tid; p < n; p += 256) {
        const int r = p / L, off = p - r * L;
        const int x = src[p];
        const uint64_t kx = sort_key(xq, x);
        const int o = (r ^ 1) * L;  // partner run
        int lo = 0, hi = 0;
        if (o < n) {
          hi = n - o < L ? n - o : L;
          while (lo < hi) {  // count of partner keys below x's
            const int m = (lo + hi) >> 1;
            if (sort_key(xq, src[o + m]) < kx) lo = m + 1;
            else hi = m;
          }
        }
        dst[(r & ~1) * L + off + lo] = x;
      }
      __syncthreads();
      int32_t *t = src;
      src = dst;
      dst = t;
    }
    if (src != perm + a) {
      for (int p = tid; p < n; p += 256) perm[a + p] = src[p];
      __syncthreads();
    }
    if constexpr (GATHER)
      for (int p = tid; p < n; p += 256) go.sorted[a + p] = gather_record(go, perm[a + p]);
  }
}

void launch_cell_sort(hipStream_t s, const int32_t *cell_start, int64_t ncell,
                      const int32_t *cell_of, int64_t n, int32_t *perm, const uint32_t *xq,
                      const uint32_t *skey, uint32_t *qword, int32_t *sorted_perm,
                      int32_t *big_list, uint32_t *big_count, const GatherOut *go) {
  int64_t b = ceil_div(ncell, 256);
  if (b < 1) b = 1;
  if (b > 16384) b = 16384;
  hipLaunchKernelGGL(k_cell_small, dim3((unsigned)b), dim3(256), 0, s, cell_start, ncell, skey,
                     qword, big_list, big_count);
  const GatherOut g = go ? *go : GatherOut{};
  if (n > 0) {
    int64_t bn = ceil_div(n, 256);
    if (bn > 16384) bn = 16384;
    if (go)
      hipLaunchKernelGGL(k_cell_rank<true>, dim3((unsigned)bn), dim3(256), 0, s, cell_start,
                         cell_of, perm, n, skey, sorted_perm, g);
    else
      hipLaunchKernelGGL(k_cell_rank<false>, dim3((unsigned)bn), dim3(256), 0, s, cell_start,
                         cell_of, perm, n, skey, sorted_perm, g);
  }
  // the large cells, in place in sorted_perm with perm as scratch
  if (go)
    hipLaunchKernelGGL(k_cell_sort_big<true>, dim3(kBigSortBlocks), dim3(256), 0, s, cell_start,
                       sorted_perm, perm, xq, big_list, big_count, g);
  else
    hipLaunchKernelGGL(k_cell_sort_big<false>, dim3(kBigSortBlocks), dim3(256), 0, s, cell_start,
                       sorted_perm, perm, xq, big_list, big_count, g);
}

int64_t cell_sort_list_elems(int64_t n) { return n / (kSmallCell + 1) + 1; }

// ------------------------------------------------ periodic ghost images
// The extended grid (ExtGeom) lets a lane walk any row of cells around its
// particle as one contiguous range of the extended array, without
// wrap-around or image shifts.
//
// It is built row by row.  An extended row (ey, ez) repeats real row
// (ry, rz) periodically along x.  With S(r) the particles of the real row in
// its cells [0, r) and T its total, the particles in unwrapped cells [0, u)
// number F(u) = p T + S(r) for u = p n_x + r, 0 <= r < n_x, and the extended
// row holds unwrapped cells [-h_x, n_x + h_x): its k-th particle is the
// unwrapped particle P = F(-h_x) + k, i.e. particle P mod T of the real row
// shifted by floor(P / T) periods.

// Per extended row: its particle count and F(-h_x).
__global__ __launch_bounds__(256) void k_ext_rows(const int32_t *__restrict__ cell_start,
                                                  ExtGeom g, int64_t nrows,
                                                  int32_t *__restrict__ row_count,
                                                  int32_t *__restrict__ row_lo) {
  for (int row = blockIdx.x * blockDim.x + threadIdx.x; row < (int)nrows;
       row += gridDim.x * blockDim.x) {
    const ExtRow r = ext_row(g, row);
    const int64_t T = cell_start[r.r0 + g.nc[0]] - cell_start[r.r0];
    const int64_t lo = row_prefix(cell_start, r.r0, g.nc[0], T, -g.h[0]);
    const int64_t hi = row_prefix(cell_start, r.r0, g.nc[0], T, g.nc[0] + g.h[0]);
    row_count[row] = (int32_t)(hi - lo);
    row_lo[row] = (int32_t)lo;
  }
}

// ext_start of every extended cell (and of one past the last) from the row
// starts, one wavefront per extended row with the row's values uniform.  Cell
// u of the unwrapped row lies p = floor(u / n_x) periods away; with a halo of
// at most n_x cells, u is in [-n_x, 2 n_x) and p in {-1, 0, 1}.
__global__ __launch_bounds__(256) void k_ext_starts(const int32_t *__restrict__ cell_start,
                                                    const int32_t *__restrict__ row_start,
                                                    const int32_t *__restrict__ row_lo,
                                                    ExtGeom g, int64_t next, int64_t nrows,
                                                    int32_t *__restrict__ ext_start,
                                                    const uint32_t *__restrict__ qword,
                                                    int2 *__restrict__ ext_sq) {
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(
      (int)((blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6));
  const int nwaves = (int)(((int64_t)gridDim.x * blockDim.x) >> 6);
  if (wave == 0 && lane == 0) {
    ext_start[next] = row_start[nrows];
    if (ext_sq) ext_sq[next] = make_int2(row_start[nrows], 0);
  }
  const int nx = g.nc[0], hx = g.h[0], nex = g.ne[0];
  const bool near = hx <= nx;
  // next < 2^30 (checked at build), so 32-bit cell indices suffice
  for (int row = wave; row < (int)nrows; row += nwaves) {
    const ExtRow r = ext_row(g, row);
    const int c0 = cell_start[r.r0];
    const int64_t T = cell_start[r.r0 + nx] - c0;
    const int64_t base = (int64_t)row_start[row] - row_lo[row];
    int32_t *__restrict__ out = ext_start + (int64_t)row * nex;
    for (int ex = lane; ex < nex; ex += 64) {
      const int u = ex - hx;
      const int p = near ? (u < 0 ? -1 : (u >= nx ? 1 : 0)) : floor_div(u, nx);
      const int rc = r.r0 + (u - p * nx);
      const int32_t st = (int32_t)(base + p * T + (cell_start[rc] - c0));
      out[ex] = st;
      if (ext_sq) ext_sq[(int64_t)row * nex + ex] = make_int2(st, (int)qword[rc]);
    }
  }
}

// Copy of every extended row, one wavefront per row.  Writes stop at the
// buffer's capacity; running past it flags an overflow (the pair kernel then
// refuses to read ghost ranges beyond the capacity).  Each of ext_pos,
// ext_rel and ext_src (the source's sorted slot) is written when not null.
__global__ __launch_bounds__(256) void k_ext_fill(const int32_t *__restrict__ cell_start,
                                                  const int32_t *__restrict__ row_start,
                                                  const int32_t *__restrict__ row_lo,
                                                  const double4 *__restrict__ sorted, ExtGeom g,
                                                  int64_t nrows, int64_t cap,
                                                  double4 *__restrict__ ext_pos,
                                                  float4 *__restrict__ ext_rel,
                                                  int32_t *__restrict__ ext_src,
                                                  uint32_t *status) {
  const double len[3] = {g.L[0] / (double)g.nc[0], g.L[1] / (double)g.nc[1],
                         g.L[2] / (double)g.nc[2]};
  const double sc0 = (double)g.nc[0] / g.L[0];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(
      (int)((blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6));
  const int nwaves = (int)(((int64_t)gridDim.x * blockDim.x) >> 6);
  // with a halo of at most n_x cells a row's unwrapped prefixes P lie in
  // [-T, 2T), so the period floor(P / T) is -1, 0 or 1
  const bool near = g.h[0] <= g.nc[0];
  for (int row = wave; row < (int)nrows; row += nwaves) {
    const ExtRow r = ext_row(g, row);
    const int first = cell_start[r.r0];
    const int T = cell_start[r.r0 + g.nc[0]] - first;
    const int64_t o0 = row_start[row], cnt = row_start[row + 1] - o0;
    const int lo = row_lo[row];
    const double sy = (double)r.py * g.L[1], sz = (double)r.pz * g.L[2];
    bool over = false;
    // kFillUnroll slots per lane at a time: their source reads are all
    // issued before the first is used
    constexpr int kFillUnroll = 4;
    for (int k0 = lane; k0 < cnt; k0 += 64 * kFillUnroll) {
      double4 q[kFillUnroll];
      int pk[kFillUnroll];
      bool ok[kFillUnroll];
#pragma unroll
      for (int u = 0; u < kFillUnroll; ++u) {
        const int k = k0 + 64 * u;
        const int P = lo + k;
        // cnt > 0 implies T > 0
        const int p = near ? (P < 0 ? -1 : (P >= T ? 1 : 0)) : floor_div(P, T);
        const int64_t o = o0 + k;
        pk[u] = p;
        ok[u] = k < cnt;
        if (ok[u] && o >= cap) {
          over = true;
          ok[u] = false;
        }
        const int src = first + (P - p * T);
        if (ok[u] && ext_src) ext_src[o] = src;
        if (ok[u] && ext_pos) q[u] = sorted[src];
      }
      if (!ext_pos) continue;
#pragma unroll
      for (int u = 0; u < kFillUnroll; ++u) {
        if (!ok[u]) continue;
        const int64_t o = o0 + k0 + 64 * u;
        const int p = pk[u];
        double4 w = q[u];
        const int ex = slab_index(w.x, sc0, g.nc[0]) + p * g.nc[0];
        w.x = w.x + (double)p * g.L[0];
        w.y = w.y + sy;
        w.z = w.z + sz;
        ext_pos[o] = w;
        if (ext_rel) ext_rel[o] = rel_record(w, ex, r.ey, r.ez, len);
      }
    }
    if (over) atomicOr(status, ST_GHOST_OVERFLOW);
  }
}

int64_t ext_row_scratch_elems(const int32_t nc[3], const int32_t h[3]) {
  return (int64_t)(nc[1] + 2 * h[1]) * (nc[2] + 2 * h[2]) + 1;
}

static ExtGeom ext_geom(const int32_t nc[3], const int32_t h[3], const double L[3]) {
  ExtGeom g;
  for (int a = 0; a < 3; ++a) {
    g.nc[a] = nc[a];
    g.h[a] = h[a];
    g.ne[a] = nc[a] + 2 * h[a];
    g.L[a] = L[a];
  }
  return g;
}

static void launch_ext_fill(hipStream_t s, const int32_t *cell_start, const int32_t *row_start,
                            const int32_t *row_lo, const double4 *sorted, const ExtGeom &g,
                            int64_t ext_cap, double4 *ext_pos, float4 *ext_rel,
                            int32_t *ext_src, uint32_t *status) {
  const int64_t nrows = (int64_t)g.ne[1] * g.ne[2];
  int64_t b = ceil_div(nrows, 4);  // four rows per workgroup of 256
  if (b > 16384) b = 16384;
  hipLaunchKernelGGL(k_ext_fill, dim3((unsigned)b), dim3(256), 0, s, cell_start, row_start,
                     row_lo, sorted, g, nrows, ext_cap, ext_pos, ext_rel, ext_src, status);
}

void launch_ext_src(hipStream_t s, const int32_t *cell_start, const int32_t *row_start,
                    const int32_t *row_lo, const int32_t nc[3], const int32_t h[3],
                    const double L[3], int64_t ext_cap, int32_t *ext_src, uint32_t *status) {
  launch_ext_fill(s, cell_start, row_start, row_lo, nullptr, ext_geom(nc, h, L), ext_cap, nullptr,
                  nullptr, ext_src, status);
}

void launch_ext_refill(hipStream_t s, const int32_t *cell_start, const int32_t *row_start,
                       const int32_t *row_lo, const double4 *sorted, const int32_t nc[3],
                       const int32_t h[3], const double L[3], int64_t ext_cap, double4 *ext_pos,
                       uint32_t *status) {
  launch_ext_fill(s, cell_start, row_start, row_lo, sorted, ext_geom(nc, h, L), ext_cap, ext_pos,
                  nullptr, nullptr, status);
}

void launch_ext_count(hipStream_t s, const int32_t *cell_start, const int32_t nc[3],
                      const int32_t h[3], const double L[3], int32_t *row_count,
                      int32_t *row_start, int32_t *row_lo, int32_t *ext_start,
                      int32_t *scan_tmp, const uint32_t *qword, int2 *ext_sq) {
  const ExtGeom g = ext_geom(nc, h, L);
  const int64_t next = (int64_t)g.ne[0] * g.ne[1] * g.ne[2];
  const int64_t nrows = (int64_t)g.ne[1] * g.ne[2];
  int64_t b = ceil_div(nrows, 256);
  if (b > 16384) b = 16384;
  hipLaunchKernelGGL(k_ext_rows, dim3((unsigned)b), dim3(256), 0, s, cell_start, g, nrows,
                     row_count, row_lo);
  launch_exclusive_scan(s, row_count, row_start, nrows, scan_tmp);
  b = ceil_div(nrows, 4);  // four rows per workgroup of 256
  if (b < 1) b = 1;
  if (b > 16384) b = 16384;
  hipLaunchKernelGGL(k_ext_starts, dim3((unsigned)b), dim3(256), 0, s, cell_start, row_start,
                     row_lo, g, next, nrows, ext_start, qword, ext_sq);
}

void launch_ext_images(hipStream_t s, const int32_t *cell_start, const int32_t *row_start,
                       const int32_t *row_lo, const double4 *sorted, const int32_t nc[3],
                       const int32_t h[3], const double L[3], int64_t ext_cap, double4 *ext_pos,
                       float4 *ext_rel, uint32_t *status) {
  launch_ext_fill(s, cell_start, row_start, row_lo, sorted, ext_geom(nc, h, L), ext_cap, ext_pos,
                  ext_rel, nullptr, status);
}

}  // namespace dcm
