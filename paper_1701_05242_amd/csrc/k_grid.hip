// Interface detection on the density grid (Section 2.1, Fig. 4, Eq. 4):
// binning -> gray value -> histogram -> two-phase threshold -> majority
// regularisation -> interface marking.  All stages are integer stencils or
// exact integer sums, so their results are bit-for-bit deterministic.
//
// The gray value's 27-point window runs on 64 x 4 columns of (x, y) outputs
// that march through z with the (x, y) halo of each plane staged in LDS; the
// interface marking reads 64 x 4 x 4 tiles.
#include "dcm_device.hpp"
#include "dcm_internal.hpp"

namespace dcm {

constexpr int SX = 64, SY = 4, SZ = 4;                 // stencil tile (outputs)
constexpr int HX = SX + 2, HY = SY + 2;                // with halo

// periodic index for a coordinate within one period of [0, n)
__device__ __forceinline__ int wrap_near(int i, int n) {
  if (i < 0) i += n;
  if (i >= n) i -= n;
  if (i < 0 || i >= n) i = wrap_index(i, n);  // grids thinner than the halo
  return i;
}

// ------------------------------------------------------------ binning (Fig. 4a)
__global__ __launch_bounds__(256) void k_bin_density(const double *__restrict__ x,
                                                     const double *__restrict__ y,
                                                     const double *__restrict__ z, int64_t n,
                                                     double Lx, double Ly, double Lz, int nx,
                                                     int ny, int nz, double sx, double sy,
                                                     double sz, uint32_t *counts,
                                                     uint32_t *status) {
  // grid-stride loop with a uniform trip count so every lane reaches the
  // run-aggregated atomic together
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t base = blockIdx.x * (int64_t)blockDim.x; base < n; base += stride) {
    const int64_t i = base + threadIdx.x;
    bool valid = i < n;
    uint32_t v = 0;
    if (valid) {
      double px = x[i], py = y[i], pz = z[i];
      if (!finite3(px, py, pz)) {
        atomicOr(status, ST_NONFINITE_POS);
        valid = false;
      } else {
        int vx = slab_index(wrap_coord(px, Lx), sx, nx);
        int vy = slab_index(wrap_coord(py, Ly), sy, ny);
        int vz = slab_index(wrap_coord(pz, Lz), sz, nz);
        v = (uint32_t)(((int64_t)vz * ny + vy) * nx + vx);
      }
    }
    wave_run_add(counts, v, valid);
  }
}

void launch_bin_density(hipStream_t s, const double *x, const double *y, const double *z,
                        int64_t n, const double L[3], const int32_t nv[3], const double sc[3],
                        uint32_t *counts, uint32_t *status) {
  if (n <= 0) return;
  int64_t b = ceil_div(n, 256);
  if (b > 8192) b = 8192;
  hipLaunchKernelGGL(k_bin_density, dim3((unsigned)b), dim3(256), 0, s, x, y, z, n, L[0], L[1],
                     L[2], nv[0], nv[1], nv[2], sc[0], sc[1], sc[2], counts, status);
}

static dim3 stencil_grid(const int32_t nv[3]) {
  return dim3((unsigned)ceil_div(nv[0], SX), (unsigned)ceil_div(nv[1], SY),
              (unsigned)ceil_div(nv[2], SZ));
}

// --------------------------------------- gray value and histogram (Fig. 4b)
// gray[v] = sum of counts over the periodic 3x3x3 window of v, and the
// histogram of the gray values, in one pass.  A workgroup owns a 64 x 4
// column of (x, y) outputs and marches through kGrayZ planes of z (32: fewer
// workgroups merge fewer private histograms, measured 41 us against 50 us
// for 16 and 47 us for 64 on the 160 x 160 x 400 grid): each plane
// of counts is staged in LDS with its one-voxel (x, y) halo and summed over
// the 3 x 3 window of each output, and the sums of three consecutive planes
// give the gray value of the middle one.  A plane is read once per column
// (1.55 words per output with the halo) instead of three times.
//
// Histogram: a private LDS histogram per workgroup, merged once into one of
// kHistCopies global copies (the split sums them).  The low-density phase puts most voxels into the first few
// bins: a lane counts those in registers and adds them to the LDS histogram
// at the end; every other voxel takes one LDS atomic (lanes that hit the same
// bin are serialised by the LDS itself).  Counts are exact integers, so the
// histogram does not depend on the order of the additions.
#ifndef DCM_GRAY_Z
#define DCM_GRAY_Z 32
#endif
constexpr int kGrayZ = DCM_GRAY_Z;
constexpr int kHistLow = 3;

__global__ __launch_bounds__(SX * SY) void k_gray_hist(const uint32_t *__restrict__ counts,
                                                     uint32_t *__restrict__ gray, int nx, int ny,
                                                     int nz, uint32_t *hist, uint32_t *status) {
  __shared__ uint32_t plane[HY][HX];
  __shared__ uint32_t lh[kHistBins];
  const int tid = threadIdx.y * SX + threadIdx.x;
  for (int b = tid; b < kHistBins; b += SX * SY) lh[b] = 0u;
  const int x0 = blockIdx.x * SX, y0 = blockIdx.y * SY, z0 = blockIdx.z * kGrayZ;
  const int lx = threadIdx.x, ly = threadIdx.y;
  const int gx = x0 + lx, gy = y0 + ly;
  const bool mine = gx < nx && gy < ny;
  const int zend = z0 + kGrayZ < nz ? z0 + kGrayZ : nz;
  uint32_t low[kHistLow] = {0u, 0u, 0u};
  bool over = false;
  uint32_t s0 = 0u, s1 = 0u;  // 3 x 3 sums of the two planes before plane z
  // this thread's (at most two) elements of a haloed plane; the next plane's
  // are read while the current one is summed
  static_assert(HY * HX <= 2 * SX * SY, "two elements per thread cover a plane");
  const int e1 = tid + SX * SY;
  const int py0 = tid / HX, px0 = tid - py0 * HX, py1 = e1 / HX, px1 = e1 - py1 * HX;
  const bool has0 = tid < HY * HX, has1 = e1 < HY * HX;
  const int64_t off0 = has0 ? (int64_t)wrap_near(y0 + py0 - 1, ny) * nx + wrap_near(x0 + px0 - 1, nx) : 0;
  const int64_t off1 = has1 ? (int64_t)wrap_near(y0 + py1 - 1, ny) * nx + wrap_near(x0 + px1 - 1, nx) : 0;
  const int64_t pstride = (int64_t)ny * nx;
  auto fetch = [&](int z, uint32_t &v0, uint32_t &v1) {
    const uint32_t *src = counts + wrap_near(z, nz) * pstride;
    v0 = has0 ? src[off0] : 0u;
    v1 = has1 ? src[off1] : 0u;
  };
  uint32_t n0, n1;
  fetch(z0 - 1, n0, n1);
  // plane z is read for z = z0 - 1 .. zend; output plane z - 1 once three
  // planes are summed
  for (int z = z0 - 1; z <= zend; ++z) {
    __syncthreads();  // the previous plane has been summed (and lh cleared)
    if (has0) plane[py0][px0] = n0;
    if (has1) plane[py1][px1] = n1;
    __syncthreads();
    if (z < zend) fetch(z + 1, n0, n1);
    uint32_t s2 = 0u;
#pragma unroll
    for (int dy = 0; dy < 3; ++dy)
#pragma unroll
      for (int dx = 0; dx < 3; ++dx) s2 += plane[ly + dy][lx + dx];
    if (z > z0 && mine) {
      const uint32_t g = s0 + s1 + s2;
      gray[((int64_t)(z - 1) * ny + gy) * nx + gx] = g;
#pragma unroll
      for (int k = 0; k < kHistLow; ++k) low[k] += g == (uint32_t)k ? 1u : 0u;
      if (g >= (uint32_t)kHistLow) {
        if (g < (uint32_t)kHistBins) atomicAdd(&lh[g], 1u);
        else over = true;
      }
    }
    s0 = s1;
    s1 = s2;
  }
  if (over) atomicOr(status, ST_HIST_RANGE);
#pragma unroll
  for (int k = 0; k < kHistLow; ++k)
    if (low[k]) atomicAdd(&lh[k], low[k]);
  __syncthreads();
  // workgroups spread their merges over kHistCopies copies of the histogram,
  // so the few bins of the liquid are not all added into one address
  const int64_t bid = ((int64_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
  uint32_t *dst = hist + (bid % kHistCopies) * kHistBins;
  for (int b = tid; b < kHistBins; b += SX * SY)
    if (lh[b]) atomicAdd(&dst[b], lh[b]);
}

void launch_gray_hist(hipStream_t s, const uint32_t *counts, uint32_t *gray, const int32_t nv[3],
                      uint32_t *hist, uint32_t *status) {
  const dim3 g((unsigned)ceil_div(nv[0], SX), (unsigned)ceil_div(nv[1], SY),
               (unsigned)ceil_div(nv[2], kGrayZ));
  hipLaunchKernelGGL(k_gray_hist, g, dim3(SX, SY), 0, s, counts, gray, nv[0], nv[1], nv[2], hist,
                     status);
}

// ------------------------------ two-phase split of the gray values (Eq. 4)
// For threshold t the phases are {g >= t} and {g < t}.  The piecewise-
// constant two-phase energy with no length term is smallest where
// S0^2/n0 + S1^2/n1 is largest (S, n: exact integer sum and count of each
// phase); ties go to the smallest t.  One workgroup of 1024 threads owns 4
// consecutive histogram bins each (summed over the histogram's copies).
__global__ __launch_bounds__(1024) void k_otsu(const uint32_t *__restrict__ hist, Ctl *ctl,
                                               int32_t *t_out, uint32_t *status) {
  __shared__ long long sc[1024];
  __shared__ long long ss[1024];
  __shared__ double bscore[1024];
  __shared__ int bt[1024];
  __shared__ long long best_n1, best_s1;
  const int tid = threadIdx.x;
  const int t0 = tid * 4;
  long long c[4], sm[4];
  long long lc = 0, ls = 0;
  // this thread's 4 bins summed over the copies (16-byte loads; a bin holds
  // at most the voxel count, below 2^31)
  // (eight copies' loads in flight at a time: one workgroup reads the whole
  // set, so the loads' latency, not bandwidth, sets the time; 14 us with
  // one at a time, 11.8 with eight, 12.7 with sixteen)
  static_assert(kHistCopies % 8 == 0, "copies are read eight at a time");
  uint4 h = make_uint4(0u, 0u, 0u, 0u);
  for (int k0 = 0; k0 < kHistCopies; k0 += 8) {
    uint4 v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k)
      v[k] = *reinterpret_cast<const uint4 *>(hist + (k0 + k) * kHistBins + t0);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      h.x += v[k].x;
      h.y += v[k].y;
      h.z += v[k].z;
      h.w += v[k].w;
    }
  }
  const uint32_t hv[4] = {h.x, h.y, h.z, h.w};
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    c[q] = (long long)hv[q];
    sm[q] = c[q] * (long long)(t0 + q);
    lc += c[q];
    ls += sm[q];
  }
  sc[tid] = lc;
  ss[tid] = ls;
  __syncthreads();
  // inclusive suffix scan over threads: sc[tid] = sum over threads u >= tid
  for (int off = 1; off < 1024; off <<= 1) {
    long long vc = (tid + off < 1024) ? sc[tid + off] : 0;
    long long vs = (tid + off < 1024) ? ss[tid + off] : 0;
    __syncthreads();
    sc[tid] += vc;
    ss[tid] += vs;
    __syncthreads();
  }
  const long long total_n = sc[0], total_s = ss[0];
  long long above_n = (tid + 1 < 1024) ? sc[tid + 1] : 0;
  long long above_s = (tid + 1 < 1024) ? ss[tid + 1] : 0;
  double best = -1.0;
  int best_t = -1;
  long long n1q[4], s1q[4];
  // n1/S1 at t = t0+q: every bin >= t
  for (int q = 3; q >= 0; --q) {
    above_n += c[q];
    above_s += sm[q];
    n1q[q] = above_n;
    s1q[q] = above_s;
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    int t = t0 + q;
    if (t < 1) continue;
    long long nn1 = n1q[q], ss1 = s1q[q];
    long long nn0 = total_n - nn1, ss0 = total_s - ss1;
    if (nn0 == 0 || nn1 == 0) continue;
    double S0 = (double)ss0, S1 = (double)ss1;
    double score = (S0 * S0) / (double)nn0 + (S1 * S1) / (double)nn1;
    if (score > best) {
      best = score;
      best_t = t;
    }
  }
  bscore[tid] = best;
  bt[tid] = best_t;
  __syncthreads();
  for (int off = 512; off > 0; off >>= 1) {
    if (tid < off) {
      double o = bscore[tid + off];
      int ot = bt[tid + off];
      bool take = (ot >= 0) && (bt[tid] < 0 || o > bscore[tid] ||
                                (o == bscore[tid] && ot < bt[tid]));
      if (take) {
        bscore[tid] = o;
        bt[tid] = ot;
      }
    }
    __syncthreads();
  }
  const int T = bt[0];
  if (T >= 0 && T >= t0 && T < t0 + 4) {
    best_n1 = n1q[T - t0];
    best_s1 = s1q[T - t0];
  }
  __syncthreads();
  if (tid == 0) {
    int degenerate = 1;
    double c0 = 0.0, c1 = 0.0;
    if (T >= 0) {
      long long nn1 = best_n1, ss1 = best_s1;
      long long nn0 = total_n - nn1, ss0 = total_s - ss1;
      c0 = (double)ss0 / (double)nn0;
      c1 = (double)ss1 / (double)nn1;
      degenerate = ((c1 + 3.0) / (c0 + 3.0) < 2.0) ? 1 : 0;
    }
    ctl->threshold = T;
    ctl->degenerate = degenerate;
    ctl->c0 = c0;
    ctl->c1 = c1;
    if (degenerate) atomicOr(status, ST_DEGENERATE);
    if (t_out) *t_out = T;
  }
}

void launch_otsu(hipStream_t s, const uint32_t *hist, int64_t nvox, Ctl *ctl, int32_t *t_out,
                 uint32_t *status) {
  (void)nvox;
  hipLaunchKernelGGL(k_otsu, dim3(1), dim3(1024), 0, s, hist, ctl, t_out, status);
}

// ------------------------------- bit-packed phase maps (majority filter)
// The phase map of every majority pass is stored one bit per voxel: each
// x-row is W = ceil(nx/32) 32-bit words, bit b of word k holding voxel
// x = 32k + b; bits at x >= nx are always 0.  A pass then evaluates 32
// voxels per lane with bitwise arithmetic instead of byte stencils.
__host__ __device__ __forceinline__ int row_words(int nx) { return (nx + 31) >> 5; }

// Initial phase map s0 = [g >= T] (or [g >= split] for a fixed split); a
// single-phase volume is all high density.  One lane per (row, bit) slot of
// the padded rows; a ballot packs 32 lanes into a word.  Also resets the
// majority-pass state for the passes that follow.
constexpr int kThreshUnroll = 4;
__global__ __launch_bounds__(256) void k_threshold(const uint32_t *__restrict__ gray, int nx,
                                                   int64_t rows, double split, Ctl *ctl,
                                                   uint32_t *__restrict__ bits0,
                                                   int32_t *t_out) {
  const bool fixed = split > 0.0;
  const int T = ctl->threshold;
  const bool deg = !fixed && ctl->degenerate;
  const int W = row_words(nx);
  const int64_t slots = rows * W * 32;
  const int lane = threadIdx.x & 63;
  // uniform trip count: whole wavefronts reach every ballot.  A lane reads
  // kThreshUnroll slots a grid stride apart before testing any of them, so
  // that many loads are in flight per wavefront (one at a time left the
  // pass bound by load latency at a quarter of the bandwidth: 20 us against
  // 15 with four; eight, 19 us, leave most lanes idle in the last round on
  // the 160 x 160 x 400 grid).  A word index is below the voxel count, so
  // below 2^31.
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t base = blockIdx.x * (int64_t)blockDim.x; base < slots;
       base += kThreshUnroll * stride) {
    uint32_t g[kThreshUnroll];
    bool ok[kThreshUnroll];
#pragma unroll
    for (int u = 0; u < kThreshUnroll; ++u) {
      const int64_t t = base + u * stride + threadIdx.x;
      const uint32_t word = (uint32_t)(t >> 5);
      const uint32_t row = word / (uint32_t)W;
      const int x = (int)(word - row * (uint32_t)W) * 32 + (int)(t & 31);
      ok[u] = t < slots && x < nx;
      g[u] = ok[u] ? gray[(int64_t)row * nx + x] : 0u;
    }
#pragma unroll
    for (int u = 0; u < kThreshUnroll; ++u) {
      const int64_t t = base + u * stride + threadIdx.x;
      bool s = false;
      if (ok[u]) {
        if (fixed)
          s = (double)g[u] >= split;
        else
          s = deg || (int64_t)g[u] >= (int64_t)T;
      }
      const unsigned long long m = __ballot(s);
      if ((lane & 31) == 0 && t < slots) bits0[t >> 5] = (uint32_t)(m >> (lane & 32));
    }
  }
  if (blockIdx.x == 0 && threadIdx.x < kMajorityMaxPasses + 2) {
    ctl->maj_chg1[threadIdx.x] = 0u;
    ctl->maj_chg2[threadIdx.x] = 0u;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (fixed) {
      ctl->threshold = (int32_t)ceil(split);
      ctl->degenerate = 0;
      if (t_out) *t_out = (int32_t)ceil(split);
    }
  }
}

static unsigned flat_grid(int64_t n) {
  int64_t b = ceil_div(n, 256 * 4);
  if (b < 1) b = 1;
  if (b > 4096) b = 4096;
  return (unsigned)b;
}

void launch_threshold(hipStream_t s, const uint32_t *gray, const int32_t nv[3], double split,
                      const Ctl *ctl, uint32_t *bits0, int32_t *t_out) {
  const int64_t rows = (int64_t)nv[1] * nv[2];
  hipLaunchKernelGGL(k_threshold, dim3(flat_grid(rows * row_words(nv[0]) * 32)), dim3(256), 0, s,
                     gray, nv[0], rows, split, const_cast<Ctl *>(ctl), bits0, t_out);
}

// ---------------------------------------- majority regularisation (4b)
// Pass p reads state p-1 from buf[(p-1)&1] and writes state p to buf[p&1],
// noting whether any voxel differs from state p-1 (none: fixed point) and
// from the overwritten state p-2 (none: 2-cycle).
// Pass q ended the iteration if it changed nothing (fixed point) or, from the
// second pass on, reproduced state q-2 (2-cycle).  A pass that did not run
// left both flags at 0, so the test also holds for every pass after the end.
__device__ __forceinline__ bool majority_stopped(const Ctl *ctl, int q) {
  return phase_pass_stopped(ctl->maj_chg1, ctl->maj_chg2, q);
}

// Word k of a row with its periodic x-neighbours: a holds bit x-1 and c bit
// x+1 at the position of x.  lw / rw are the row's words k-1 and k+1
// (cyclically); `top` is the bit position of x = nx - 1 in the last word.
__device__ __forceinline__ void x_neighbours(uint32_t lw, uint32_t w, uint32_t rw, bool first,
                                             bool lastw, int top, uint32_t &a, uint32_t &c) {
  a = (w << 1) | (first ? ((lw >> top) & 1u) : (lw >> 31));
  c = (w >> 1) | (lastw ? ((rw & 1u) << top) : (rw << 31));
}

// Add the x-window sums (a + w + c per bit) of one row into the bit-sliced
// 5-bit counters c0..c4 of a 27-window count.
__device__ __forceinline__ void add_row_window(uint32_t a, uint32_t w, uint32_t c, uint32_t &c0,
                                               uint32_t &c1, uint32_t &c2, uint32_t &c3,
                                               uint32_t &c4) {
  // x-window sum a + w + c as two bit slices
  const uint32_t h0 = a ^ w ^ c;
  const uint32_t h1 = (a & w) | (c & (a ^ w));
  // add the 2-bit number (h1 h0) into the 5-bit counter
  const uint32_t k0 = c0 & h0;
  c0 ^= h0;
  const uint32_t t1 = c1 ^ h1;
  const uint32_t k1 = (c1 & h1) | (k0 & t1);
  c1 = t1 ^ k0;
  const uint32_t k2 = c2 & k1;
  c2 ^= k1;
  const uint32_t k3 = c3 & k2;
  c3 ^= k2;
  c4 ^= k3;
}

// One lane per word: the 27-window count of each of its 32 voxels as a
// bit-sliced 5-bit number (c0..c4), then [count >= 14].
__global__ __launch_bounds__(256) void k_majority(uint32_t *buf0, uint32_t *buf1, int nx, int ny,
                                                  int nz, int pass, Ctl *ctl) {
  if (pass > 1 && majority_stopped(ctl, pass - 1)) return;
  const uint32_t *__restrict__ src = (pass & 1) ? buf0 : buf1;
  uint32_t *__restrict__ dst = (pass & 1) ? buf1 : buf0;
  const int W = row_words(nx);
  const int top = (nx - 1) & 31;
  const uint32_t last_mask = (nx & 31) ? ((1u << (nx & 31)) - 1u) : 0xffffffffu;
  const int64_t words = (int64_t)ny * nz * W;
  bool ch1 = false, ch2 = false;
  for (int64_t wi = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; wi < words;
       wi += (int64_t)gridDim.x * blockDim.x) {
    const int64_t row = wi / W;
    const int k = (int)(wi - row * W);
    const int y = (int)(row % ny), z = (int)(row / ny);
    const int kl = k == 0 ? W - 1 : k - 1, kr = k == W - 1 ? 0 : k + 1;
    const bool first = k == 0, lastw = k == W - 1;
    uint32_t c0 = 0, c1 = 0, c2 = 0, c3 = 0, c4 = 0, prev = 0;
#pragma unroll
    for (int dz = -1; dz <= 1; ++dz) {
      int zz = z + dz;
      zz = zz < 0 ? zz + nz : (zz >= nz ? zz - nz : zz);
#pragma unroll
      for (int dy = -1; dy <= 1; ++dy) {
        int yy = y + dy;
        yy = yy < 0 ? yy + ny : (yy >= ny ? yy - ny : yy);
        const uint32_t *r = src + ((int64_t)zz * ny + yy) * W;
        const uint32_t w = r[k];
        if (dz == 0 && dy == 0) prev = w;
        uint32_t a, c;
        x_neighbours(r[kl], w, r[kr], first, lastw, top, a, c);
        add_row_window(a, w, c, c0, c1, c2, c3, c4);
      }
    }
    // count >= 14: 16..27 have c4 set, 14 and 15 are 0111x
    uint32_t nw = c4 | (c3 & c2 & c1);
    if (lastw) nw &= last_mask;
    const uint32_t old = dst[wi];
    dst[wi] = nw;
    ch1 |= nw != prev;
    ch2 |= nw != old;
  }
  // any change in this workgroup: store the pass's flag (same value from
  // every writer, so no atomic is needed)
  const int any1 = __syncthreads_or(ch1 ? 1 : 0);
  const int any2 = __syncthreads_or(ch2 ? 1 : 0);
  if (threadIdx.x == 0) {
    if (any1) ctl->maj_chg1[pass] = 1u;
    if (any2) ctl->maj_chg2[pass] = 1u;
  }
}

// ------------------------------ length-term regularisation (4b', Eq. 4)
// The two-phase piecewise-constant energy with a length term of weight nu,
// sum_v (g_v - c_{s_v})^2 + nu * (differing 26-neighbour pairs), lowered by
// synchronous iterated conditional modes with the phase means of the split
// held fixed: d = ((g - c1)^2 - (g - c0)^2) + nu * (26 - 2 n1) for the n1
// high-density neighbours; phase 1 if d < 0, 0 if d > 0, unchanged if d = 0.
// Same buffers, pass numbering and stop flags as the majority vote.  A
// single-phase volume is left as it is.
__global__ __launch_bounds__(256) void k_potts(uint32_t *buf0, uint32_t *buf1,
                                               const uint32_t *__restrict__ gray, int nx, int ny,
                                               int nz, double nu, int pass, Ctl *ctl) {
  if (pass > 1 && majority_stopped(ctl, pass - 1)) return;
  const uint32_t *__restrict__ src = (pass & 1) ? buf0 : buf1;
  uint32_t *__restrict__ dst = (pass & 1) ? buf1 : buf0;
  const bool keep = ctl->degenerate != 0;
  const double c0 = ctl->c0, c1 = ctl->c1;
  const int W = row_words(nx);
  const int top = (nx - 1) & 31;
  const int64_t words = (int64_t)ny * nz * W;
  bool ch1 = false, ch2 = false;
  for (int64_t wi = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; wi < words;
       wi += (int64_t)gridDim.x * blockDim.x) {
    const int64_t row = wi / W;
    const int k = (int)(wi - row * W);
    const int y = (int)(row % ny), z = (int)(row / ny);
    const int kl = k == 0 ? W - 1 : k - 1, kr = k == W - 1 ? 0 : k + 1;
    const bool first = k == 0, lastw = k == W - 1;
    uint32_t q0 = 0, q1 = 0, q2 = 0, q3 = 0, q4 = 0, prev = 0;
#pragma unroll
    for (int dz = -1; dz <= 1; ++dz) {
      int zz = z + dz;
      zz = zz < 0 ? zz + nz : (zz >= nz ? zz - nz : zz);
#pragma unroll
      for (int dy = -1; dy <= 1; ++dy) {
        int yy = y + dy;
        yy = yy < 0 ? yy + ny : (yy >= ny ? yy - ny : yy);
        const uint32_t *r = src + ((int64_t)zz * ny + yy) * W;
        const uint32_t w = r[k];
        if (dz == 0 && dy == 0) prev = w;
        uint32_t a, c;
        x_neighbours(r[kl], w, r[kr], first, lastw, top, a, c);
        const uint32_t h0 = a ^ w ^ c;
        const uint32_t h1 = (a & w) | (c & (a ^ w));
        const uint32_t k0 = q0 & h0;
        q0 ^= h0;
        const uint32_t t1 = q1 ^ h1;
        const uint32_t k1 = (q1 & h1) | (k0 & t1);
        q1 = t1 ^ k0;
        const uint32_t k2 = q2 & k1;
        q2 ^= k1;
        const uint32_t k3 = q3 & k2;
        q3 ^= k2;
        q4 ^= k3;
      }
    }
    uint32_t nw = prev;
    if (!keep) {
      nw = 0u;
      const int nb = lastw ? top + 1 : 32;
      const uint32_t *grow = gray + row * nx + k * 32;
      for (int b = 0; b < nb; ++b) {
        const uint32_t self = (prev >> b) & 1u;
        const int n1 = (int)(((q0 >> b) & 1u) + 2u * ((q1 >> b) & 1u) + 4u * ((q2 >> b) & 1u) +
                             8u * ((q3 >> b) & 1u) + 16u * ((q4 >> b) & 1u) - self);
        const double ga = (double)grow[b] - c1, gb = (double)grow[b] - c0;
        const double d = (ga * ga - gb * gb) + nu * (double)(26 - 2 * n1);
        const uint32_t bit = d < 0.0 ? 1u : (d > 0.0 ? 0u : self);
        nw |= bit << b;
      }
    }
    const uint32_t old = dst[wi];
    dst[wi] = nw;
    ch1 |= nw != prev;
    ch2 |= nw != old;
  }
  const int any1 = __syncthreads_or(ch1 ? 1 : 0);
  const int any2 = __syncthreads_or(ch2 ? 1 : 0);
  if (threadIdx.x == 0) {
    if (any1) ctl->maj_chg1[pass] = 1u;
    if (any2) ctl->maj_chg2[pass] = 1u;
  }
}

void launch_potts_pass(hipStream_t s, uint32_t *buf0, uint32_t *buf1, const uint32_t *gray,
                       const int32_t nv[3], double nu, int pass, Ctl *ctl) {
  int64_t b = ceil_div(phase_bits_words(nv), 256);
  if (b < 1) b = 1;
  if (b > 2048) b = 2048;
  hipLaunchKernelGGL(k_potts, dim3((unsigned)b), dim3(256), 0, s, buf0, buf1, gray, nv[0], nv[1],
                     nv[2], nu, pass, ctl);
}

int64_t phase_bits_words(const int32_t nv[3]) {
  return (int64_t)nv[1] * nv[2] * row_words(nv[0]);
}

void launch_majority_pass(hipStream_t s, uint32_t *buf0, uint32_t *buf1, const int32_t nv[3],
                          int pass, int max_passes, Ctl *ctl) {
  (void)max_passes;
  int64_t b = ceil_div(phase_bits_words(nv), 256);
  if (b < 1) b = 1;
  if (b > 2048) b = 2048;
  hipLaunchKernelGGL(k_majority, dim3((unsigned)b), dim3(256), 0, s, buf0, buf1, nv[0], nv[1],
                     nv[2], pass, ctl);
}

// ------------------------------------------- interface marking (Fig. 4c)
// seg[v] = final phase; iface[v] = 1 for a high-density voxel with a
// low-density face neighbour.
__device__ __forceinline__ uint32_t phase_bit(const uint32_t *s, int W, int nx, int ny, int x,
                                              int y, int z) {
  (void)nx;
  return (s[((int64_t)z * ny + y) * W + (x >> 5)] >> (x & 31)) & 1u;
}

__global__ __launch_bounds__(256) void k_interface(const uint32_t *buf0, const uint32_t *buf1,
                                                   int nx, int ny, int nz, const Ctl *ctl,
                                                   uint8_t *__restrict__ seg,
                                                   uint8_t *__restrict__ iface) {
  const uint32_t *__restrict__ s =
      final_phase_map(ctl->maj_chg1, ctl->maj_chg2, kMajorityMaxPasses, buf0, buf1);
  const int W = row_words(nx);
  const int i = blockIdx.x * SX + threadIdx.x;
  const int j = blockIdx.y * SY + threadIdx.y;
  if (i >= nx || j >= ny) return;
  const int im = i == 0 ? nx - 1 : i - 1, ip = i + 1 == nx ? 0 : i + 1;
  const int jm = j == 0 ? ny - 1 : j - 1, jp = j + 1 == ny ? 0 : j + 1;
#pragma unroll
  for (int q = 0; q < SZ; ++q) {
    const int k = blockIdx.z * SZ + q;
    if (k >= nz) break;
    const int km = k == 0 ? nz - 1 : k - 1, kp = k + 1 == nz ? 0 : k + 1;
    const int64_t v = ((int64_t)k * ny + j) * nx + i;
    const uint32_t sv = phase_bit(s, W, nx, ny, i, j, k);
    uint32_t f = 0;
    if (sv)
      f = (phase_bit(s, W, nx, ny, im, j, k) & phase_bit(s, W, nx, ny, ip, j, k) &
           phase_bit(s, W, nx, ny, i, jm, k) & phase_bit(s, W, nx, ny, i, jp, k) &
           phase_bit(s, W, nx, ny, i, j, km) & phase_bit(s, W, nx, ny, i, j, kp)) ^ 1u;
    seg[v] = (uint8_t)sv;
    iface[v] = (uint8_t)f;
  }
}

void launch_interface(hipStream_t s, const uint32_t *buf0, const uint32_t *buf1,
                      const int32_t nv[3], const Ctl *ctl, uint8_t *seg, uint8_t *iface) {
  hipLaunchKernelGGL(k_interface, stencil_grid(nv), dim3(SX, SY), 0, s, buf0, buf1, nv[0], nv[1],
                     nv[2], ctl, seg, iface);
}

}  // namespace dcm
