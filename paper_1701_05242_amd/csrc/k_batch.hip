// Build kernels of the batched form: linked cells (Section 2.3) and ghost
// images for many independent systems, one launch per stage.  The systems'
// particles, cells and extended cells are concatenated in system order, so a
// single exclusive scan over all cells yields every system's cell starts and
// keeps each system's sorted particles in its own contiguous slice.  A block
// of 256 threads always works inside one system: the host lists one
// (system, first index) entry per block.
#include "dcm_device.hpp"
#include "dcm_internal.hpp"

namespace dcm {

constexpr int kBatchBlock = 256;

__device__ __forceinline__ int block_system(const int2 *tab, int64_t &first) {
  const int2 w = tab[blockIdx.x];
  first = __builtin_amdgcn_readfirstlane(w.y);
  return __builtin_amdgcn_readfirstlane(w.x);
}

__device__ __forceinline__ ExtGeom ext_geom(const SysGeom &g) {
  ExtGeom e;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    e.nc[a] = g.nc[a];
    e.h[a] = g.h[a];
    e.ne[a] = g.ne[a];
    e.L[a] = g.L[a];
  }
  return e;
}

// Cell of every particle (concatenated cell index), its x key, per-cell
// counts, and the largest cutoff of each workgroup (reduced per system by
// kb_reduce_rcmax).
__global__ __launch_bounds__(kBatchBlock) void kb_cell_count(
    const SysGeom *__restrict__ sys, const int2 *__restrict__ pblk, int32_t *__restrict__ cell_of,
    int32_t *count, unsigned long long *__restrict__ block_max, uint32_t *__restrict__ xq,
    uint32_t *status) {
  int64_t first;
  const int b = block_system(pblk, first);
  const SysGeom &g = sys[b];
  const int64_t i = first + threadIdx.x;
  const bool valid = i < g.n;
  int c = 0;
  unsigned long long bits = 0;
  if (valid) {
    const double px = g.x[i], py = g.y[i], pz = g.z[i];
    double r = g.rc[i];
    int lc = 0;
    uint32_t q = 0;
    if (finite3(px, py, pz)) {
      const double wx = wrap_coord(px, g.L[0]);
      const int cx = slab_index(wx, g.sc[0], g.nc[0]);
      const int cy = slab_index(wrap_coord(py, g.L[1]), g.sc[1], g.nc[1]);
      const int cz = slab_index(wrap_coord(pz, g.L[2]), g.sc[2], g.nc[2]);
      lc = (cz * g.nc[1] + cy) * g.nc[0] + cx;
      q = x_key(wx, g.sc[0], cx);
    } else {
      atomicOr(status, ST_NONFINITE_POS);
    }
    xq[g.p0 + i] = q;
    if (!(r >= 0.0) || r > g.rc_cap) {
      atomicOr(status, ST_RC_RANGE);
      r = (r > g.rc_cap) ? g.rc_cap : 0.0;
    }
    bits = (unsigned long long)__double_as_longlong(r);
    c = (int)g.cell0 + lc;
    cell_of[g.p0 + i] = c;
  }
  wave_run_add(count, (uint32_t)c, valid);
  __shared__ unsigned long long wmax[kBatchBlock / 64];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    unsigned long long o = __shfl_xor(bits, off, 64);
    bits = o > bits ? o : bits;
  }
  if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = bits;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long m = wmax[0];
    for (int w = 1; w < kBatchBlock / 64; ++w) m = wmax[w] > m ? wmax[w] : m;
    block_max[blockIdx.x] = m;
  }
}

// Largest cutoff of each system from its workgroups' maxima (a system's
// workgroups are items [item0, item0 + nitems) of the block table).
__global__ __launch_bounds__(256) void kb_reduce_rcmax(const SysGeom *__restrict__ sys,
                                                       const unsigned long long *__restrict__ bm,
                                                       unsigned long long *rc_max_bits) {
  const SysGeom &g = sys[blockIdx.x];
  __shared__ unsigned long long wmax[4];
  unsigned long long m = 0;
  for (int64_t t = threadIdx.x; t < g.nitems; t += 256) {
    const unsigned long long v = bm[g.item0 + t];
    m = v > m ? v : m;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    unsigned long long o = __shfl_xor(m, off, 64);
    m = o > m ? o : m;
  }
  if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 0; w < 4; ++w) m = wmax[w] > m ? wmax[w] : m;
    rc_max_bits[blockIdx.x] = m;
  }
}

// Slot of every particle inside its cell; perm[slot] = concatenated id,
// skey[slot] = its x key.
__global__ __launch_bounds__(kBatchBlock) void kb_cell_scatter(
    const SysGeom *__restrict__ sys, const int2 *__restrict__ pblk,
    const int32_t *__restrict__ cell_of, const int32_t *__restrict__ cell_start, int32_t *fill,
    int32_t *__restrict__ perm, const uint32_t *__restrict__ xq, uint32_t *__restrict__ skey) {
  int64_t first;
  const int b = block_system(pblk, first);
  const SysGeom &g = sys[b];
  const int64_t i = first + threadIdx.x;
  const bool valid = i < g.n;
  const int c = valid ? cell_of[g.p0 + i] : 0;
  const int slot = wave_run_slot(fill, (uint32_t)c, valid);
  if (valid) {
    const int64_t p = cell_start[c] + slot;
    perm[p] = (int32_t)(g.p0 + i);
    skey[p] = xq[g.p0 + i];
  }
}

// Sorted copy (x, y, z, rc) in the order order[] (concatenated ids, copied
// to perm) with positions wrapped into each system's box.
__global__ __launch_bounds__(kBatchBlock) void kb_gather(const SysGeom *__restrict__ sys,
                                                         const int2 *__restrict__ pblk,
                                                         const int32_t *__restrict__ order,
                                                         double4 *__restrict__ sorted,
                                                         int32_t *__restrict__ perm) {
  int64_t first;
  const int b = block_system(pblk, first);
  const SysGeom &g = sys[b];
  const int64_t k = first + threadIdx.x;
  if (k >= g.n) return;
  const int64_t s = g.p0 + k;
  const int32_t id = order[s];
  perm[s] = id;
  const int64_t i = id - g.p0;
  const double px = g.x[i], py = g.y[i], pz = g.z[i];
  double4 o;
  if (finite3(px, py, pz)) {
    o.x = wrap_coord(px, g.L[0]);
    o.y = wrap_coord(py, g.L[1]);
    o.z = wrap_coord(pz, g.L[2]);
  } else {
    o.x = o.y = o.z = 0.0;
  }
  const double r = g.rc[i];
  o.w = (r >= 0.0) ? (r < g.rc_cap ? r : g.rc_cap) : 0.0;  // NaN -> 0
  sorted[s] = o;
}

__device__ __forceinline__ int64_t ext_cells_of(const SysGeom &g) {
  return (int64_t)g.ne[0] * g.ne[1] * g.ne[2];
}

// Ghost images row by row (the scheme of k_cells.hip): per extended row of a
// system its particle count and F(-h_x), one scan over the rows of all
// systems, the extended-cell starts from the row starts, and one wavefront
// copying each row.  rblk lists (system, first row) per group of kBatchBlock
// rows; row indices are local to a system, g.row0 its first row overall.
__device__ __forceinline__ int64_t ext_rows_of(const SysGeom &g) {
  return (int64_t)g.ne[1] * g.ne[2];
}

__global__ __launch_bounds__(kBatchBlock) void kb_ext_rows(const SysGeom *__restrict__ sys,
                                                           const int2 *__restrict__ rblk,
                                                           const int32_t *__restrict__ cell_start,
                                                           int32_t *__restrict__ row_count,
                                                           int32_t *__restrict__ row_lo) {
  int64_t first;
  const int b = block_system(rblk, first);
  const SysGeom &g = sys[b];
  const int64_t row = first + threadIdx.x;
  if (row >= ext_rows_of(g)) return;
  const ExtGeom eg = ext_geom(g);
  const ExtRow r = ext_row(eg, (int)row);
  const int32_t *cs = cell_start + g.cell0;
  const int64_t T = cs[r.r0 + g.nc[0]] - cs[r.r0];
  const int64_t lo = row_prefix(cs, r.r0, g.nc[0], T, -g.h[0]);
  const int64_t hi = row_prefix(cs, r.r0, g.nc[0], T, g.nc[0] + g.h[0]);
  row_count[g.row0 + row] = (int32_t)(hi - lo);
  row_lo[g.row0 + row] = (int32_t)lo;
}

__global__ __launch_bounds__(kBatchBlock) void kb_ext_starts(
    const SysGeom *__restrict__ sys, const int2 *__restrict__ eblk,
    const int32_t *__restrict__ cell_start, const int32_t *__restrict__ row_start,
    const int32_t *__restrict__ row_lo, int64_t next_total, int64_t nrows_total,
    int32_t *__restrict__ ext_start, const uint32_t *__restrict__ qword,
    int2 *__restrict__ ext_sq) {
  int64_t first;
  const int b = block_system(eblk, first);
  const SysGeom &g = sys[b];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ext_start[next_total] = row_start[nrows_total];
    if (ext_sq) ext_sq[next_total] = make_int2(row_start[nrows_total], 0);
  }
  const int64_t e = first + threadIdx.x;
  if (e >= ext_cells_of(g)) return;
  const int row = (int)(e / g.ne[0]);
  const int ex = (int)(e - (int64_t)row * g.ne[0]);
  const ExtRow r = ext_row(ext_geom(g), row);
  const int32_t *cs = cell_start + g.cell0;
  const int64_t T = cs[r.r0 + g.nc[0]] - cs[r.r0];
  const int64_t f = row_prefix(cs, r.r0, g.nc[0], T, ex - g.h[0]);
  const int32_t st = (int32_t)(row_start[g.row0 + row] + (f - row_lo[g.row0 + row]));
  ext_start[g.ext_cell0 + e] = st;
  if (ext_sq)
    ext_sq[g.ext_cell0 + e] =
        make_int2(st, (int)qword[g.cell0 + r.r0 + wrap_index(ex - g.h[0], g.nc[0])]);
}

// One wavefront per row: workgroup w takes rows 4 (w mod 64) .. + 3 of row
// group w / 64.  Writes stop at the buffer's capacity; running past it flags
// an overflow.
constexpr int kFillGroups = kBatchBlock / (kBatchBlock / 64);  // workgroups per row group

__global__ __launch_bounds__(kBatchBlock) void kb_ext_fill(
    const SysGeom *__restrict__ sys, const int2 *__restrict__ rblk,
    const int32_t *__restrict__ cell_start, const int32_t *__restrict__ row_start,
    const int32_t *__restrict__ row_lo, const double4 *__restrict__ sorted, int64_t cap,
    double4 *__restrict__ ext_pos, float4 *__restrict__ ext_rel, uint32_t *status) {
  const int2 w = rblk[blockIdx.x / kFillGroups];
  const int b = __builtin_amdgcn_readfirstlane(w.x);
  const int64_t first = __builtin_amdgcn_readfirstlane(w.y);
  const SysGeom &g = sys[b];
  const ExtGeom eg = ext_geom(g);
  const int64_t nrows = ext_rows_of(g);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const double sc0 = (double)g.nc[0] / g.L[0];
  bool over = false;
  const int64_t row = first + (int64_t)(blockIdx.x % kFillGroups) * (kBatchBlock / 64) + wave;
  if (row < nrows) {
    const ExtRow r = ext_row(eg, (int)row);
    const int32_t *cs = cell_start + g.cell0;
    const int start = cs[r.r0];
    const int T = cs[r.r0 + g.nc[0]] - start;
    const int64_t o0 = row_start[g.row0 + row];
    const int64_t cnt = row_start[g.row0 + row + 1] - o0;
    const int lo = row_lo[g.row0 + row];
    const double sy = (double)r.py * g.L[1], sz = (double)r.pz * g.L[2];
    for (int k = lane; k < cnt; k += 64) {
      const int P = lo + k;
      const int p = floor_div(P, T);  // cnt > 0 implies T > 0
      const int64_t o = o0 + k;
      if (o >= cap) {
        over = true;
        continue;
      }
      double4 q = sorted[start + (P - p * T)];
      const int ex = slab_index(q.x, sc0, g.nc[0]) + p * g.nc[0];
      q.x = q.x + (double)p * g.L[0];
      q.y = q.y + sy;
      q.z = q.z + sz;
      ext_pos[o] = q;
      if (ext_rel) ext_rel[o] = rel_record(q, ex, r.ey, r.ez, g.len);
    }
  }
  if (over) atomicOr(status, ST_GHOST_OVERFLOW);
}

// One workgroup per system sums the system's work-item partials in a fixed
// order (the same order as the single-system reduction over its blocks).
// (the same summation as the single-system reduction, so a system's sums
// are bit for bit those of dcm_forces on the same cells)
__global__ __launch_bounds__(kReduceThreads) void kb_reduce(const SysGeom *__restrict__ sys,
                                                            const double *__restrict__ partials,
                                                            int ev_flags) {
  const SysGeom &g = sys[blockIdx.x];
  __shared__ double red[kReduceThreads / 64][kPartialSlots];
  double t[kPartialSlots];
  sum_rows<kReduceThreads, kPartialSlots>(partials + g.item0 * kPartialSlots, g.nitems, red, t);
  if (threadIdx.x == 0) {
    if (g.energy && (ev_flags & DCM_EV_ENERGY)) *g.energy = t[0];
    if (g.virial && (ev_flags & DCM_EV_VIRIAL))
      for (int k = 0; k < 6; ++k) g.virial[k] = t[1 + k];
    if (g.npairs && (ev_flags & DCM_EV_COUNTS)) *g.npairs = (uint64_t)t[7];
  }
}

void launch_batch_cell_count(hipStream_t s, const SysGeom *sys, int32_t nsys, const int2 *pblk,
                             int64_t npblk, int32_t *cell_of, int32_t *cell_count,
                             unsigned long long *block_max, unsigned long long *rc_max_bits,
                             uint32_t *xq, uint32_t *status) {
  if (npblk > 0)
    hipLaunchKernelGGL(kb_cell_count, dim3((unsigned)npblk), dim3(kBatchBlock), 0, s, sys, pblk,
                       cell_of, cell_count, block_max, xq, status);
  if (nsys > 0)
    hipLaunchKernelGGL(kb_reduce_rcmax, dim3((unsigned)nsys), dim3(256), 0, s, sys, block_max,
                       rc_max_bits);
}

void launch_batch_cell_scatter(hipStream_t s, const SysGeom *sys, const int2 *pblk,
                               int64_t npblk, const int32_t *cell_of, const int32_t *cell_start,
                               int32_t *cell_fill, int32_t *perm, const uint32_t *xq,
                               uint32_t *skey) {
  if (npblk <= 0) return;
  hipLaunchKernelGGL(kb_cell_scatter, dim3((unsigned)npblk), dim3(kBatchBlock), 0, s, sys, pblk,
                     cell_of, cell_start, cell_fill, perm, xq, skey);
}

void launch_batch_gather(hipStream_t s, const SysGeom *sys, const int2 *pblk, int64_t npblk,
                         const int32_t *order, double4 *sorted, int32_t *perm) {
  if (npblk <= 0) return;
  hipLaunchKernelGGL(kb_gather, dim3((unsigned)npblk), dim3(kBatchBlock), 0, s, sys, pblk, order,
                     sorted, perm);
}

void launch_batch_ext(hipStream_t s, const SysGeom *sys, const int2 *eblk, int64_t neblk,
                      const int2 *rblk, int64_t nrblk, const int32_t *cell_start,
                      const double4 *sorted, int64_t next_total, int64_t nrows_total,
                      int64_t ext_cap, int32_t *row_count, int32_t *row_start, int32_t *row_lo,
                      int32_t *ext_start, int32_t *scan_tmp, double4 *ext_pos, float4 *ext_rel,
                      const uint32_t *qword, int2 *ext_sq, uint32_t *status) {
  if (nrblk <= 0 || neblk <= 0) return;
  hipLaunchKernelGGL(kb_ext_rows, dim3((unsigned)nrblk), dim3(kBatchBlock), 0, s, sys, rblk,
                     cell_start, row_count, row_lo);
  launch_exclusive_scan(s, row_count, row_start, nrows_total, scan_tmp);
  hipLaunchKernelGGL(kb_ext_starts, dim3((unsigned)neblk), dim3(kBatchBlock), 0, s, sys, eblk,
                     cell_start, row_start, row_lo, next_total, nrows_total, ext_start, qword,
                     ext_sq);
  hipLaunchKernelGGL(kb_ext_fill, dim3((unsigned)(nrblk * kFillGroups)), dim3(kBatchBlock), 0, s,
                     sys, rblk, cell_start, row_start, row_lo, sorted, ext_cap, ext_pos, ext_rel,
                     status);
}

void launch_batch_reduce(hipStream_t s, const SysGeom *sys, int32_t nsys,
                         const double *partials, int ev_flags) {
  if (nsys <= 0) return;
  hipLaunchKernelGGL(kb_reduce, dim3((unsigned)nsys), dim3(kReduceThreads), 0, s, sys, partials,
                     ev_flags);
}

}  // namespace dcm
