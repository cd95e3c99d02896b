// Device-side helpers shared by the library's kernels.  Every operation whose
// bits matter for an exact comparison (wrap, voxel/cell index, trilinear
// weights) is written as one fixed sequence of correctly rounded IEEE
// operations; the library is compiled with -ffp-contract=off so nothing is
// fused unless fma() is written explicitly.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace dcm {

// Periodic wrap into [0, L): w = x - L*floor(x/L), folding a result that
// rounds below 0 or up to L.
__device__ __forceinline__ double wrap_coord(double x, double L) {
  double q = floor(x / L);
  double w = x - L * q;
  if (w < 0.0) w = w + L;
  if (w >= L) w = 0.0;
  return w;
}

// Index of the slab [c*L/n, (c+1)*L/n) holding a wrapped coordinate;
// scale = n/L (computed once on the host).  Clamped so that a NaN or an
// out-of-range input can never index outside [0, n).
__device__ __forceinline__ int slab_index(double w, double scale, int n) {
  double f = floor(w * scale);
  int c = (f >= 0.0) ? ((f < (double)n) ? (int)f : n - 1) : 0;
  return c;
}

// x key of a particle in cell c of the slab grid (scale = n/L): its offset
// into the cell, (w scale - c), in units of 2^-20 of the cell, clamped to
// [0, 2^20).  Cells keep their particles in key order; sub-cell q (of
// kXSub along x) of a cell holds the keys [q, q + 1) 2^20 / kXSub.
constexpr uint32_t kXKeyOne = 1u << 20;
constexpr int kXSubLog = 3;
constexpr int kXSub = 1 << kXSubLog;
__device__ __forceinline__ uint32_t x_key(double w, double scale, int c) {
  const double f = (w * scale - (double)c) * (double)kXKeyOne;
  return f > 0.0 ? (f < (double)(kXKeyOne - 1) ? (uint32_t)f : kXKeyOne - 1) : 0u;
}

// The regularisation passes of the phase map (majority vote or length term):
// pass q ended the iteration if it changed nothing (chg1[q] = 0: fixed point)
// or, from the second pass on, reproduced state q-2 (chg2[q] = 0: 2-cycle).
// A pass that did not run left both at 0, so the test holds after the end.
__device__ __forceinline__ bool phase_pass_stopped(const uint32_t *chg1, const uint32_t *chg2,
                                                   int q) {
  return chg1[q] == 0u || (q >= 2 && chg2[q] == 0u);
}

// The map holding the final phase: state p lives in b[p & 1]; the last pass
// is the first that stopped (max_passes if none did).
__device__ __forceinline__ const uint32_t *final_phase_map(const uint32_t *chg1,
                                                           const uint32_t *chg2, int max_passes,
                                                           const uint32_t *b0,
                                                           const uint32_t *b1) {
  int last = max_passes;
  for (int p = 1; p <= max_passes; ++p)
    if (phase_pass_stopped(chg1, chg2, p)) {
      last = p;
      break;
    }
  return (last & 1) ? b1 : b0;
}

__device__ __forceinline__ int wrap_index(int i, int n) {
  int r = i % n;
  return r < 0 ? r + n : r;
}

__device__ __forceinline__ bool finite3(double a, double b, double c) {
  return isfinite(a) && isfinite(b) && isfinite(c);
}

// Compact candidate record of the FP32-mixed pair kernel (16 bytes instead of
// 32): the position relative to the centre of its extended cell (ex, ey, ez)
// in FP32 -- each component lies within half a cell edge of 0, so it keeps
// a few 1e-8 of absolute precision -- and ex + 1/2 (exact in FP32) in the
// last word.  A lane rebuilds the separation in FP64 from its own position
// and the cell centre.
__device__ __forceinline__ float4 rel_record(const double4 &q, int ex, int ey, int ez,
                                             const double len[3]) {
  float4 r;
  r.x = (float)(q.x - ((double)ex + 0.5) * len[0]);
  r.y = (float)(q.y - ((double)ey + 0.5) * len[1]);
  r.z = (float)(q.z - ((double)ez + 0.5) * len[2]);
  r.w = (float)ex + 0.5f;
  return r;
}

// Ghost-extended cell grid: the cell grid grown by h[a] cells on both sides
// of every axis.  Extended cell (ex, ey, ez) holds a copy of real cell
// (ex - h[0], ey - h[1], ez - h[2]) wrapped into the box, with positions
// shifted by the matching multiple of the box length.
struct ExtGeom {
  int nc[3];
  int h[3];
  int ne[3];
  double L[3];
};

// Real cell rc behind extended cell e, and the periods p[a] crossed.
__device__ __forceinline__ void ext_to_real(const ExtGeom &g, int64_t e, int &rc, int p[3]) {
  const int ex = (int)(e % g.ne[0]);
  const int64_t t = e / g.ne[0];
  const int ey = (int)(t % g.ne[1]);
  const int ez = (int)(t / g.ne[1]);
  const int u[3] = {ex - g.h[0], ey - g.h[1], ez - g.h[2]};
  int r[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    r[a] = wrap_index(u[a], g.nc[a]);
    p[a] = (u[a] - r[a]) / g.nc[a];  // periods crossed: exact division
  }
  rc = (r[2] * g.nc[1] + r[1]) * g.nc[0] + r[0];
}

// floor(a / b) for b > 0
__device__ __forceinline__ int floor_div(int a, int b) {
  const int q = a / b;
  return (a % b != 0 && a < 0) ? q - 1 : q;
}

// Real row behind extended row (ey, ez): its first cell, and the y and z
// periods crossed.
struct ExtRow {
  int r0;     // first real cell of the row
  int py, pz;
  int ey, ez;  // extended cell coordinates relative to the real grid
};

__device__ __forceinline__ ExtRow ext_row(const ExtGeom &g, int row) {
  ExtRow r;
  const int ez0 = row / g.ne[1];
  const int ey = row - ez0 * g.ne[1] - g.h[1];
  const int ez = ez0 - g.h[2];
  const int ry = wrap_index(ey, g.nc[1]), rz = wrap_index(ez, g.nc[2]);
  r.py = (ey - ry) / g.nc[1];
  r.pz = (ez - rz) / g.nc[2];
  r.r0 = (rz * g.nc[1] + ry) * g.nc[0];
  r.ey = ey;
  r.ez = ez;
  return r;
}

// F(u) of the row starting at real cell r0 (T: the row's total)
__device__ __forceinline__ int64_t row_prefix(const int32_t *__restrict__ cell_start, int r0,
                                              int nx, int64_t T, int u) {
  const int p = floor_div(u, nx);
  const int r = u - p * nx;
  return (int64_t)p * T + (cell_start[r0 + r] - cell_start[r0]);
}

// MI355X has 8 XCDs, each with its own L2; consecutive workgroups are
// dispatched round-robin across them.  xcd_block(b, n, G) remaps workgroup b
// so that each XCD receives runs of G consecutive logical blocks (spatially
// neighbouring work, which shares cell data, then shares an L2) while the
// runs still interleave across XCDs (work that clusters in space stays
// spread over all of them).  G = 0 keeps the hardware order; blocks past the
// last whole group of 8 G keep it too.
constexpr int kXcds = 8;
__device__ __forceinline__ int64_t xcd_block(int64_t b, int64_t nblocks, int group) {
  if (group <= 0) return b;
  const int64_t span = (int64_t)kXcds * group;
  if (b >= (nblocks / span) * span) return b;
  const int64_t x = b % kXcds, k = b / kXcds;
  return ((k / group) * kXcds + x) * group + k % group;
}

// Sum of a value over the 64 lanes of a wavefront (fixed butterfly order).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sums of the first S columns of `rows` rows of STRIDE doubles (row r at
// p + r STRIDE) by one workgroup of NT threads, in a fixed order: thread t
// adds rows t, t + NT, ... in turn, each wavefront sums its lanes with
// shuffles, and thread 0 adds the wavefronts in order.  A column's sum does
// not depend on S.  Every thread must call it; thread 0 gets out[].
template <int NT, int S, int STRIDE = S>
__device__ __forceinline__ void sum_rows(const double *__restrict__ p, int64_t rows,
                                         double (*red)[S], double *out) {
  double v[S];
#pragma unroll
  for (int k = 0; k < S; ++k) v[k] = 0.0;
  for (int64_t r = threadIdx.x; r < rows; r += NT)
#pragma unroll
    for (int k = 0; k < S; ++k) v[k] += p[r * STRIDE + k];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < S; ++k) {
    const double t = wave_sum(v[k]);
    if (lane == 0) red[wid][k] = t;
  }
  __syncthreads();
  if (threadIdx.x == 0)
    for (int k = 0; k < S; ++k) {
      double t = red[0][k];
      for (int w = 1; w < NT / 64; ++w) t += red[w][k];
      out[k] = t;
    }
}

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Add 1 to hist[key] for every valid lane with one atomic per distinct key in
// the wavefront.  Must be reached by all lanes of the wavefront together.
template <typename Counter>
__device__ __forceinline__ void wave_aggregated_add(Counter *hist, uint32_t key, bool valid) {
  unsigned long long pending = __ballot(valid);
  while (pending) {
    const int leader = __ffsll((long long)pending) - 1;
    const uint32_t k = __shfl(key, leader, 64);
    const unsigned long long same = __ballot(valid && key == k);
    if ((int)(threadIdx.x & 63) == leader) atomicAdd(&hist[k], (Counter)__popcll(same));
    pending &= ~same;
  }
}

// Run-aggregated counters for key-ordered input (cell-sorted particles): the
// lanes of a wavefront are cut into runs of consecutive valid lanes with equal
// keys, and the first lane of every run issues one atomic for its run -- all
// runs in the same instruction, however many distinct keys the wavefront
// holds.  Equal keys in separate runs take separate atomics, so any input
// order gives the same totals.
__device__ __forceinline__ unsigned long long wave_run_heads(uint32_t key, bool valid,
                                                             unsigned long long &vmask) {
  const int lane = (int)(threadIdx.x & 63);
  const uint32_t prev = __shfl_up(key, 1, 64);
  const int prev_valid = __shfl_up(valid ? 1 : 0, 1, 64);
  const bool head = valid && (lane == 0 || !prev_valid || prev != key);
  vmask = __ballot(valid);
  return __ballot(head);
}

// length of the run starting at head lane `lane`
__device__ __forceinline__ int wave_run_len(int lane, unsigned long long heads,
                                            unsigned long long vmask) {
  const unsigned long long stops =
      lane == 63 ? 0ull : (heads | ~vmask) & (~0ull << (lane + 1));
  return (stops ? __ffsll((long long)stops) - 1 : 64) - lane;
}

template <typename Counter>
__device__ __forceinline__ void wave_run_add(Counter *hist, uint32_t key, bool valid) {
  const int lane = (int)(threadIdx.x & 63);
  unsigned long long vmask;
  const unsigned long long heads = wave_run_heads(key, valid, vmask);
  if ((heads >> lane) & 1ull) atomicAdd(&hist[key], (Counter)wave_run_len(lane, heads, vmask));
}

// One slot per valid lane in fill[key]: the run's first lane reserves the
// run's slots, the run's lanes take them in lane order.
__device__ __forceinline__ int wave_run_slot(int32_t *fill, uint32_t key, bool valid) {
  const int lane = (int)(threadIdx.x & 63);
  unsigned long long vmask;
  const unsigned long long heads = wave_run_heads(key, valid, vmask);
  int base = 0;
  if ((heads >> lane) & 1ull)
    base = atomicAdd(&fill[key], (int32_t)wave_run_len(lane, heads, vmask));
  const unsigned long long upto = heads & (lane == 63 ? ~0ull : ((2ull << lane) - 1ull));
  const int hl = upto ? 63 - __clzll((long long)upto) : lane;
  return __shfl(base, hl, 64) + (lane - hl);
}

// Reserve one slot per valid lane in fill[key] (lanes with equal keys share
// one atomic and take consecutive slots in lane order); returns the slot.
__device__ __forceinline__ int wave_aggregated_slot(int32_t *fill, uint32_t key, bool valid) {
  const int lane = (int)(threadIdx.x & 63);
  unsigned long long pending = __ballot(valid);
  int slot = 0;
  while (pending) {
    const int leader = __ffsll((long long)pending) - 1;
    const uint32_t k = __shfl(key, leader, 64);
    const unsigned long long same = __ballot(valid && key == k);
    int base = 0;
    if (lane == leader) base = atomicAdd(&fill[k], (int32_t)__popcll(same));
    base = __shfl(base, leader, 64);
    if (valid && key == k)
      slot = base + (int)__popcll(same & ((1ull << lane) - 1ull));
    pending &= ~same;
  }
  return slot;
}

}  // namespace dcm
