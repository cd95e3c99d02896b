// Dynamic-cutoff Lennard-Jones force, energy and virial (Section 2.4,
// Algorithm 2.3, Eqs. 2-3) over the linked cells of Section 2.3.
//
// One lane owns one particle i (particles in cell order, so a wavefront
// covers neighbouring particles with similar cutoffs).  Instead of storing
// the neighbour list of Algorithm 2.2, each lane enumerates the cell rows
// (fixed y and z cell; consecutive x cells are consecutive in memory) that can
// hold a j within its search radius and trims each row to the chord of the
// search sphere -- the small-cell traversal of Section 2.3.  Cells keep their
// particles in x order with a table of where each eighth of the cell (along
// x) starts, so a row's two end cells are trimmed to the eighths the chord
// reaches: the walk sees about the candidates of cells an eighth as wide
// along x while reading two table entries per row.  The rows are
// walked in the ghost-extended cell grid, where periodic images sit in halo
// cells with their coordinates already shifted, so every row is one
// contiguous index range and a separation is a plain difference.  A lane
// writes its rows' ranges into a private LDS list, then runs one flat loop
// over all their candidates, so lanes with different row lengths never wait
// for each other row by row.
//
// Rules: own cutoff (Algorithm 2.3) and the symmetric max(rc_i, rc_j), both
// without a Newton-3 update (Section 2.4), so a lane writes only its own
// particle; and the symmetric rule with Newton's third law, where each pair
// is evaluated once and the partner's reaction is added with atomics.
// Precisions: FP64 records (32 B per candidate); for FP32-mixed own-cutoff
// forces on narrow cells, 16-byte cell-relative records with FP32
// separations, the pairs inside a proven error band of the cutoff decided
// from the FP64 record.  FP32-mixed evaluates close pairs (r < 1.1 sigma)
// in FP64 from the FP64 record: their forces are the largest and the
// r^-14 dependence multiplies every relative rounding of r^2 and 1/r^2
// by about 7, so in FP32 they alone would set the worst particle's error.
// Also here: forces over a stored Verlet list, the persistent batched form,
// and the fixed-order reduction of block partials.
#include "dcm_device.hpp"
#include "dcm_internal.hpp"

namespace dcm {

constexpr int kPairBlock = 256;
// Row ranges per lane per chunk (LDS: 8 B each), for the kernels reading FP64
// records and for those reading compact records.  A smaller list allows more
// resident workgroups: the compact-record kernels, with cheaper candidates,
// gain from that, while the FP64 kernels, bound by their gathers, lose
// (measured on the large slab).  The compact-record kernels also hold their
// close-pair queue (kNearCap + 1 entries of 4 B); with 14 row entries both
// fit in the 40 KB of LDS that keeps four workgroups on a compute unit.
#ifndef DCM_PAIR_SEGCAP
#define DCM_PAIR_SEGCAP 24
#endif
#ifndef DCM_PAIR_SEGCAP_REL
#define DCM_PAIR_SEGCAP_REL 14
#endif
constexpr int kSegCap = DCM_PAIR_SEGCAP;
constexpr int kSegCapRel = DCM_PAIR_SEGCAP_REL;
// The batched compact-record kernel also exists with a wider list (fewer
// chunks per particle, one workgroup fewer per compute unit); its tuner
// times both (16 entries won on a 64-system batch, 14 on the large slab).
constexpr int kSegCapRelWide = 16;
template <bool REL>
constexpr int seg_cap() {
  return REL ? kSegCapRel : kSegCap;
}
#ifndef DCM_PAIR_XCD_GROUP
#define DCM_PAIR_XCD_GROUP 16
#endif
constexpr int kXcdGroup = DCM_PAIR_XCD_GROUP;
#ifndef DCM_PAIR_FILL
#define DCM_PAIR_FILL 2
#endif
constexpr int kFillRows = DCM_PAIR_FILL;  // cell rows whose starts are read together
static_assert(kSegCap >= kFillRows + 4 && kSegCapRel >= kFillRows + 4,
              "a chunk holds a batch of rows, a sentinel and a look-ahead entry");
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
  // the compact-record loop's FP32 force sums, added into fx, fy, fz after
  // each chunk of rows (they collect only pairs beyond the close range,
  // each below ~2.5 eps/sigma, so FP32 sums of a chunk lose nothing that
  // the FP32 pair terms themselves keep)
  float px = 0, py = 0, pz = 0;
};

// FP32-mixed evaluates a pair with r^2 < kNear2 sigma^2 in FP64.  A relative
// error e of an FP32 separation or of 1/r^2 becomes ~13 e or ~7 e in the pair
// force, and at r < 1.1 sigma that force is up to ~60 times the RMS particle
// force of a dense liquid (F(0.85 sigma) ~ 320 eps/sigma), so FP32 rounding
// of these few pairs (well under 1% of the interacting pairs) would dominate
// the largest per-particle error measured in units of the RMS force.
constexpr double kNear2 = 1.21;
// The compact-record loop queues its close pairs (their extended slots) in a
// per-lane LDS list of kNearCap entries and evaluates them from the FP64
// records after each chunk of rows, so the wavefront never waits on a record
// gather inside the candidate loop.  The lane's own slot passes through the
// queue too.  A lane with more queued pairs in one chunk starts over on the
// FP64 records: an equilibrated LJ liquid at density 0.8 has 3.3 neighbours
// within 1.1 sigma on average and at most 9 or 10 (measured).
constexpr int kNearCap = 10;

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

// A close pair of the FP32-mixed kernels in FP64 arithmetic (from an FP64
// separation): FP64 force sums, the energy and virial terms rounded once into
// the FP32 accumulators.  Returns the force factor.
template <int EVM>
__device__ __forceinline__ double interact_exact(Acc<DCM_FP32_MIXED> &acc, double dx, double dy,
                                                 double dz, double r2, double sig2) {
  const double r2i = recip_newton2(r2);
  const double s2 = sig2 * r2i;
  const double s6 = s2 * s2 * s2;
  const double fp = s6 * fma(2.0, s6, -1.0) * r2i;
  acc.fx = fma(fp, dx, acc.fx);
  acc.fy = fma(fp, dy, acc.fy);
  acc.fz = fma(fp, dz, acc.fz);
  if constexpr ((EVM & 1) != 0) acc.e += (float)(s6 * (s6 - 1.0));
  if constexpr ((EVM & 2) != 0) {
    const double fdx = fp * dx, fdy = fp * dy, fdz = fp * dz;
    acc.w[0] += (float)(fdx * dx);
    acc.w[1] += (float)(fdy * dy);
    acc.w[2] += (float)(fdz * dz);
    acc.w[3] += (float)(fdy * dx);
    acc.w[4] += (float)(fdz * dx);
    acc.w[5] += (float)(fdz * dy);
  }
  return fp;
}

// One interacting pair with separation d (FP64) and r2.  The force factor
// excludes 24 eps, the energy 4 eps / 2, the virial 24 eps / 2; they are
// applied once per particle.  Returns the force factor (for a reaction).
template <int PREC, int EVM>
__device__ __forceinline__ double interact(Acc<PREC> &acc, double dx, double dy, double dz,
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
    return fp;
  } else {
    if (r2 < kNear2 * sig2) return interact_exact<EVM>(acc, dx, dy, dz, r2, sig2);
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
    return fpd;
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

// Kernels that count the walk's candidates and rows (for dcm_walk_stats):
// the compact-record ones in their pair-count instance, the others (which
// always count pairs) whenever a counter buffer is passed.
template <bool REL, int EVM>
constexpr bool walk_counts() {
  return !REL || (EVM & 4) != 0;
}

__device__ __forceinline__ int clampi(int v, int lo, int hi) {
  return min(max(v, lo), hi);  // one v_med3_i32 (lo <= hi)
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
  const float4 *ext_rel;         // its compact cell-relative copy (FP32-mixed builds)
  double rel_delta;              // bound on the per-coordinate error of ext_rel
  const int32_t *ext_start;      // this system's extended cells -> extended slots
  // (first slot, sub-cell word) of every extended cell and (extended count,
  // 0) past the last; the word's nibbles k = 0..6 count the cell's particles
  // (in x order) below (k + 1)/8 of the cell, nibble 7 all of them; 0 for a
  // cell without sub-cells.  Null: rows take whole end cells.
  const int2 *ext_sq;
  int64_t ext_cap;
  // pair-count passes: candidates tested and cell rows visited, summed over
  // the particles (null: not collected)
  unsigned long long *walk;
  int nc[3], h[3], ne[3];
  double len[3], sc[3];
  double rc_bound;
  const unsigned long long *rc_all_bits;  // largest cutoff of the system (rule MAX)
  double *fx, *fy, *fz;
  int32_t *nnbr;
  const int32_t *ext_src;        // rule DCM_PAIR_MAX_N3: source slot of each extended slot
  double4 *n3_f;                 // ... and the sorted-order force and count sums
  int32_t *n3_cnt;
};

// One lane's particle and search window.
struct LaneGeo {
  double xi, yi, zi, rci, rci2;
  // FP32 geometry: the lane's position relative to the centre of its own
  // cell (a0), the cell edges and their inverses, the squared search radius
  // with the row-selection guard fguard added (fR2); for compact records also
  // the cell's x index + 1/2 (wc), rc^2 and the band around it within which
  // an FP32 r^2 cannot decide a pair
  float a0x, a0y, a0z, lenf[3], invf[3], fR2, fguard, wc, rc2f, margin, hi2f;
  uint32_t incw;  // FP32 bits of the inside range's width (compact records)
  // per axis: the distances (plus the guard) from the lane to the far faces
  // of its cell's positive (gp) and negative (gm) neighbours less one cell,
  // 0.5 len +- a0 + guard, and the lane's offset in cell units, a0/len + 1/2
  float gp[3], gm[3], ac[3];
  // kXSub invf[0] and kXSub ac[0]: the sub-cell offsets along x, and the
  // extended grid's first and last sub-cell relative to the lane's cell
  float qinv, qac;
  int qmin, qmax;
  // compact records: FP32 r^2 below which a pair is evaluated in FP64, and
  // sigma^2 for that evaluation
  float near2f;
  double sig2;
  int zlo, zhi, cx, cy, cz, self;
  int slot;  // sorted slot of the lane's particle
};

// Newton's third law (rule MAX): a pair belongs to the endpoint with the
// larger cutoff (ties: the smaller sorted slot), whose own cutoff is then the
// pair's max(rc_i, rc_j), so the lane's own search radius finds every pair
// it owns and each interacting pair is evaluated exactly once.  The partner's
// reaction goes to the sorted-order sums with atomics.  A lane's own copy has
// its own slot as source and is never owned.
template <int PREC, int EVM>
__device__ __forceinline__ void scan_n3(const uint2 (*segs)[kPairBlock], int nseg,
                                        const PairView &v, const LaneGeo &g, double sig2,
                                        Acc<PREC> &acc, int &cnt) {
  const int lane_id = threadIdx.x;
  for (int q = 0; q < nseg; ++q) {
    const uint2 sg = segs[q][lane_id];
    for (int j = (int)sg.x; j < (int)sg.y; ++j) {
      const double4 pj = v.ext_pos[j];
      const int src = v.ext_src[j];
      const double dx = g.xi - pj.x, dy = g.yi - pj.y, dz = g.zi - pj.z;
      const double r2 = (dx * dx + dy * dy) + dz * dz;
      const bool owned = pj.w < g.rci || (pj.w == g.rci && src > g.slot);
      if (owned && r2 <= g.rci2) {
        const double fp = interact<PREC, EVM>(acc, dx, dy, dz, r2, sig2);
        double *f = &v.n3_f[src].x;
        unsafeAtomicAdd(f, -fp * dx);
        unsafeAtomicAdd(f + 1, -fp * dy);
        unsafeAtomicAdd(f + 2, -fp * dz);
        if (v.n3_cnt) atomicAdd(&v.n3_cnt[src], 1);
        ++cnt;
      }
    }
  }
}

// One pair of the own-cutoff FP32-mixed kernel on compact records, evaluated
// for every lane with the result kept only where inc is set: the force of a
// lane without an interaction in this step is computed and discarded instead
// of branched around (the wavefront executes it anyway whenever any lane
// interacts).  FP32 separations, r^2 and force sums (added into the FP64 sums
// after each chunk of rows).  The mask is applied once, to 1/r^2:
// a masked pair then has s6 = 0 and adds exactly zero force, energy and
// virial, whatever its r^2 (an unmasked pair at r = 0 stays non-finite).
template <int EVM>
__device__ __forceinline__ void interact_rel(Acc<DCM_FP32_MIXED> &acc, float dx, float dy, float dz,
                                             float r2, float sig2, bool inc) {
  const float r2i = inc ? __builtin_amdgcn_rcpf(r2) : 0.0f;
  const float s2 = sig2 * r2i;
  const float s6 = s2 * s2 * s2;
  // the pair energy's s6^2 - s6 and the force factor's 2 s6^2 - s6 share
  // one product: two fused ops where the energy would take a third
  const float e = fmaf(s6, s6, -s6);
  const float fp = fmaf(s6, s6, e) * r2i;
  acc.px = fmaf(fp, dx, acc.px);
  acc.py = fmaf(fp, dy, acc.py);
  acc.pz = fmaf(fp, dz, acc.pz);
  if constexpr ((EVM & 1) != 0) acc.e += e;
  if constexpr ((EVM & 2) != 0) {
    const float fdx = fp * dx, fdy = fp * dy, fdz = fp * dz;
    acc.w[0] = fmaf(fdx, dx, acc.w[0]);
    acc.w[1] = fmaf(fdy, dy, acc.w[1]);
    acc.w[2] = fmaf(fdz, dz, acc.w[2]);
    acc.w[3] = fmaf(fdy, dx, acc.w[3]);
    acc.w[4] = fmaf(fdz, dx, acc.w[4]);
    acc.w[5] = fmaf(fdz, dy, acc.w[5]);
  }
}

// Compact records are read through a buffer resource: 32-bit offsets, and a
// read past the resource's size returns zeros instead of touching memory.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
constexpr int kBufferWord3 = 0x00020000;  // raw 32-bit dword access (gfx9 family)

// Flat loop over the compact-record candidates of this lane's first nseg
// listed rows, two candidates of one row per step (steps in all: the sum of
// the rows' halved lengths, rounded up; the second candidate of a row's last
// step is masked when the row's length is odd).  The order of evaluation,
// and so every sum, is that of one candidate at a time.  A list entry is
// (first slot, length | (row y - cy) << 16 | (row z - cz) << 24), the
// offsets as signed bytes, the length at least 1; the lane's own slot is
// never listed.  Entry nseg is a sentinel (slot 0, length 65535) and entry
// nseg + 1 exists, so the stream needs no bounds: it moves at most one entry
// past the last row (into the sentinel) before the step count ends it.
// Separations are formed in FP32 between the two cell-centre-relative
// positions, the candidate's cell k cells away: d = (a0 - k len) - rel.  A
// close pair, and a pair whose FP32 r^2 lies within the lane's proven error
// band around rc^2, is queued in nearq (nq entries; row kNearCap takes the
// overflow) for flush_near, which decides and evaluates it in FP64.  The
// stream advances with selects, and two register sets take turns so that
// every pair of records is loaded a full step before its use.
template <int EVM>
__device__ __forceinline__ void scan_rel(const uint2 (*segs)[kPairBlock], int steps,
                                         __amdgpu_buffer_rsrc_t rs, const LaneGeo &g,
                                         float sig2, Acc<DCM_FP32_MIXED> &acc, int &cnt,
                                         int32_t (*nearq)[kPairBlock], int &nq) {
  const int lane_id = threadIdx.x;
  const uint2 s0 = segs[0][lane_id];
  int j = (int)s0.x, jend = (int)s0.x + (int)(s0.y & 0xffffu), sidx = 1;
  uint32_t tag = s0.y;
  uint2 nx = segs[1][lane_id];
  // move to the next step of the stream (past the last row: slots of the
  // sentinel, never evaluated)
  auto advance = [&]() {
    const int jn = j + 2;
    const bool sw = jn >= jend;
    j = sw ? (int)nx.x : jn;
    jend = sw ? (int)nx.x + (int)(nx.y & 0xffffu) : jend;
    tag = sw ? nx.y : tag;
    sidx += sw ? 1 : 0;
    nx = segs[sidx][lane_id];
  };
  auto one = [&](const float4 &r, float ay, float az, int jr, bool valid) {
    const float dx = fmaf(-(r.w - g.wc), g.lenf[0], g.a0x) - r.x;
    const float dy = ay - r.y, dz = az - r.z;
    float r2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
    // a masked slot (past the row's end) takes part in nothing
    r2 = valid ? r2 : 3.0e38f;
    // inside: near^2 <= r^2 < rc^2 - margin, one unsigned comparison of the
    // bits of r^2 - near^2 (a negative difference has its sign bit set, so
    // it compares above every positive width).  A close pair, or one too
    // near rc^2 for the FP32 test (rare: the band is 3e-5 to 2e-4 sigma^2
    // wide), is neither inside nor beyond rc^2 + margin and waits for
    // flush_near; the queue's next entry is written whatever the test says
    // and kept only if it holds
    const bool inc = __float_as_uint(r2 - g.near2f) < g.incw;
    const bool exact = !inc && r2 <= g.hi2f;
    nearq[nq < kNearCap ? nq : kNearCap][lane_id] = jr;
    nq += exact ? 1 : 0;
    interact_rel<EVM>(acc, dx, dy, dz, r2, sig2, inc);
    if constexpr ((EVM & 4) != 0) cnt += inc ? 1 : 0;
  };
  auto eval = [&](const float4 &r0, const float4 &r1, uint32_t t, int jr, bool v2) {
    const int dyc = (int)(t << 8) >> 24, dzc = (int)t >> 24;
    const float ay = fmaf(-(float)dyc, g.lenf[1], g.a0y);
    const float az = fmaf(-(float)dzc, g.lenf[2], g.a0z);
    one(r0, ay, az, jr, true);
    one(r1, ay, az, jr + 1, v2);
  };
  // records jr and jr + 1 (one address, the second at an immediate offset;
  // a slot past the records reads zeros)
  auto load2 = [&](int jr, float4 &r0, float4 &r1) {
    const u32x4 a = __builtin_amdgcn_raw_buffer_load_b128(rs, jr << 4, 0, 0);
    const u32x4 b = __builtin_amdgcn_raw_buffer_load_b128(rs, jr << 4, 16, 0);
    r0 = make_float4(__uint_as_float(a.x), __uint_as_float(a.y), __uint_as_float(a.z),
                     __uint_as_float(a.w));
    r1 = make_float4(__uint_as_float(b.x), __uint_as_float(b.y), __uint_as_float(b.z),
                     __uint_as_float(b.w));
  };
  int left = steps;
  int ja = j;
  uint32_t ta = tag;
  bool va = j + 1 < jend;
  float4 A0, A1, B0, B1;
  load2(ja, A0, A1);
  advance();
  while (true) {
    const int jb = j;
    const uint32_t tb = tag;
    const bool vb = j + 1 < jend;
    load2(jb, B0, B1);
    advance();
    eval(A0, A1, ta, ja, va);
    if (--left == 0) break;
    ja = j;
    ta = tag;
    va = j + 1 < jend;
    load2(ja, A0, A1);
    advance();
    eval(B0, B1, tb, jb, vb);
    if (--left == 0) break;
  }
}

// The queued pairs of the lane (the first min(nq, kNearCap)), decided and
// evaluated in FP64 from their FP64 records, two records in flight.
template <int EVM>
__device__ __forceinline__ void flush_near(const int32_t (*nearq)[kPairBlock], int nq,
                                           const double4 *__restrict__ ext_pos, const LaneGeo &g,
                                           Acc<DCM_FP32_MIXED> &acc, int &cnt) {
  const int lane_id = threadIdx.x;
  const int m = nq < kNearCap ? nq : kNearCap;
  auto one = [&](const double4 &q) {
    const double ex = g.xi - q.x, ey = g.yi - q.y, ez = g.zi - q.z;
    const double e2 = (ex * ex + ey * ey) + ez * ez;
    const bool in64 = e2 < g.rci2;
    if (in64) interact_exact<EVM>(acc, ex, ey, ez, e2, g.sig2);
    if constexpr ((EVM & 4) != 0) cnt += in64 ? 1 : 0;
  };
  for (int k = 0; k < m; k += 2) {
    // the lane's own slot (queued at separation 0) is skipped unread
    const int j0 = nearq[k][lane_id];
    const int j1 = k + 1 < m ? nearq[k + 1][lane_id] : g.self;
    const bool u0 = j0 != g.self, u1 = j1 != g.self;
    double4 q0, q1;
    if (u0) q0 = ext_pos[j0];
    if (u1) q1 = ext_pos[j1];
    if (u0) one(q0);
    if (u1) one(q1);
  }
}

// Distance from the lane to the near face of the cell d cells away along axis
// a, less the guard; 0 for its own cell (gp, gm > 0 make that value negative).
__device__ __forceinline__ float face_gap(int d, const LaneGeo &g, int a) {
  const float e = fmaf(fabsf((float)d), g.lenf[a], -(d > 0 ? g.gp[a] : g.gm[a]));
  return fmaxf(e, 0.0f);
}

// Offset from the lane's cell of the cell holding the point a0 + p along
// axis a.
__device__ __forceinline__ int cell_off(float p, const LaneGeo &g, int a) {
  return (int)floorf(fmaf(p, g.invf[a], g.ac[a]));
}

// The same along x in sub-cells: q >> kXSubLog is cell_off(p, g, 0) (scaling
// by a power of 2 is exact in FP32), q & (kXSub - 1) the sub-cell of that
// cell holding a0 + p.
__device__ __forceinline__ int sub_off(float p, const LaneGeo &g) {
  return (int)floorf(fmaf(p, g.qinv, g.qac));
}

// Walk this lane's rows (fill a list, scan it, repeat) for a lane with run
// set.  REL: compact records (FP32-mixed, own-cutoff rule); else the FP64
// records.  CAP: the row capacity of segs.
template <int RULE, int PREC, int EVM, bool REL, int CAP>
__device__ __forceinline__ void sweep_rows(const PairView &v, bool run, const LaneGeo &g,
                                           double sig2, uint2 (*segs)[kPairBlock],
                                           int32_t (*nearq)[kPairBlock], Acc<PREC> &acc,
                                           int &cnt, bool &redo, int &wcand, int &wrows) {
  const int lane_id = threadIdx.x;
  const int hx = v.h[0], hy = v.h[1], hz = v.h[2];
  const int nex = v.ne[0], ney = v.ne[1];
  const int ny = v.nc[1];
  // rows are walked plane by plane (z), each plane's rows limited to the
  // y range its circle of radius sqrt(R^2 - ez^2) can reach
  // (row selection in FP32 relative to the lane's cell: the guard outweighs
  // every rounding, so rows and cells are only ever added, never dropped)
  int zc = g.zlo, yc = 0, ylo_c = 0, yhi_c = -1;
  float remz_c = 0.0f;
  // extended-cell index of row (y, z) at x = 0 is rowbase(z) + y nex; the
  // extended grid has fewer than 2^30 cells, so 32-bit indices suffice
  int rowbase_c = 0;
  const int own_row = ((g.cz + hz) * ney + (g.cy + hy)) * nex + hx;
  auto plane = [&](int z) -> bool {
    const float ez = face_gap(z - g.cz, g, 2);
    const float remz = fmaf(-ez, ez, g.fR2);
    if (remz < 0.0f) return false;
    const float w = __builtin_amdgcn_sqrtf(remz) + g.fguard;
    ylo_c = clampi(g.cy + cell_off(-w, g, 1), -hy, ny + hy - 1);
    yhi_c = clampi(g.cy + cell_off(w, g, 1), -hy, ny + hy - 1);
    remz_c = remz;
    rowbase_c = ((z + hz) * ney + hy) * nex + hx;
    return true;
  };
  bool rows_left = false;
  if (run)
    for (; zc <= g.zhi; ++zc)
      if (plane(zc)) {
        rows_left = true;
        break;
      }
  yc = ylo_c;
  // cell starts through a buffer resource: 32-bit offsets, and an offset past
  // the array reads 0 instead of touching memory
  // (sizes and offsets are unsigned 32-bit: up to 2^30 cells of 4 bytes)
  const int64_t start_bytes = ((int64_t)v.ne[0] * v.ne[1] * v.ne[2] + 1) * 4;
  const __amdgpu_buffer_rsrc_t rs_start = __builtin_amdgcn_make_buffer_rsrc(
      (void *)v.ext_start, (short)0,
      (int)(start_bytes > 0xffffffffll ? 0xffffffffu : (uint32_t)start_bytes), kBufferWord3);
  auto load_start = [&](int idx) -> int {
    return (int)__builtin_amdgcn_raw_buffer_load_b32(rs_start, (int)((uint32_t)idx << 2), 0, 0);
  };
  // the trimming table, (next + 1) entries of 8 bytes (it exists for fewer
  // than 2^28 extended cells, so its byte offsets fit in 32 bits); the
  // compact-record walk is only chosen with it
  const bool trim = REL || v.ext_sq != nullptr;
  // the extended records' capacity, as a 32-bit clamp of the row ends
  const int cap32 = v.ext_cap < 0x7fffffff ? (int)v.ext_cap : 0x7fffffff;
  const __amdgpu_buffer_rsrc_t rs_sq = __builtin_amdgcn_make_buffer_rsrc(
      (void *)v.ext_sq, (short)0, trim ? (int)(uint32_t)(2 * start_bytes) : 0, kBufferWord3);
  __amdgpu_buffer_rsrc_t rs;
  if constexpr (REL)
    rs = __builtin_amdgcn_make_buffer_rsrc((void *)v.ext_rel, (short)0,
                                           (int)(v.ext_cap * (int64_t)sizeof(float4)),
                                           kBufferWord3);
  while (rows_left) {
    // ---- fill: append the ranges of the next rows to this lane's list,
    // kFillRows rows at a time: the two ext_start reads of all of them are
    // issued before the first is used, so their latencies overlap
    int nseg = 0, steps = 0;
    // a row adds at most one entry (compact records: two entries stay free
    // for the sentinel and the look-ahead)
    while (rows_left && nseg <= CAP - kFillRows - (REL ? 2 : 1)) {
      int j0[kFillRows], j1[kFillRows], rz[kFillRows], ry[kFillRows], sl[kFillRows],
          sh[kFillRows];
      u32x2 tl[kFillRows], th[kFillRows];
      bool ok[kFillRows];
#pragma unroll
      for (int k = 0; k < kFillRows; ++k) {
        const int zcur = zc, ycur = yc, rowbase = rowbase_c;
        const float remz = remz_c;
        bool in = rows_left;
        if (rows_left && ++yc > yhi_c) {
          bool more = false;
          while (++zc <= g.zhi)
            if (plane(zc)) {
              more = true;
              break;
            }
          if (more) yc = ylo_c;
          else rows_left = false;
        }
        const float ey = face_gap(ycur - g.cy, g, 1);
        const float rem = fmaf(-ey, ey, remz);
        in = in && rem >= 0.0f;
        // chord half-width, widened by the guard (it only selects cells and
        // sub-cells)
        const float w = in ? __builtin_amdgcn_sqrtf(rem) + g.fguard : 0.0f;
        // the chord's ends in sub-cells from the lane's cell, within the
        // extended grid (-w <= 0 <= w: the lower end can only leave it below,
        // the upper above)
        const int qlo = max(sub_off(-w, g), g.qmin);
        const int qhi = min(sub_off(w, g), g.qmax);
        // a row that is not taken still reads (its own cell row's) starts
        const int row = in ? rowbase + __mul24(ycur, nex) : own_row;
        const int e0 = row + g.cx + (qlo >> kXSubLog), e1 = row + g.cx + (qhi >> kXSubLog) + 1;
        if (trim) {
          // from the start of sub-cell qlo & 7 of cell e0 to the end of
          // sub-cell qhi & 7 of cell e1 - 1 (the end cells' sub-cells beyond
          // the chord are skipped): (start, word) of e0, and (word of e1 - 1,
          // start of e1), 8 bytes each from one table
          tl[k] = __builtin_amdgcn_raw_buffer_load_b64(rs_sq, (int)((uint32_t)e0 << 3), 0, 0);
          th[k] = __builtin_amdgcn_raw_buffer_load_b64(rs_sq, (int)(((uint32_t)e1 << 3) - 4), 0, 0);
          sl[k] = (qlo & (kXSub - 1)) << 2;
          sh[k] = (qhi & (kXSub - 1)) << 2;
        } else {
          j0[k] = load_start(e0);
          j1[k] = load_start(e1);
        }
        rz[k] = zcur;
        ry[k] = ycur;
        ok[k] = in;
      }
#pragma unroll
      for (int k = 0; k < kFillRows; ++k) {
        if (!ok[k]) continue;
        if (trim) {
          // start of sub-cell ql: nibble ql - 1 (0 for ql = 0); end of
          // sub-cell qh: n less nibble qh (0 for qh = 7)
          j0[k] = (int)(tl[k].x + (((tl[k].y << 4) >> sl[k]) & 0xfu));
          j1[k] = (int)(th[k].y - ((th[k].x >> 28) - ((th[k].x >> sh[k]) & 0xfu)));
        }
        const int a0 = j0[k];
        const int a1 = j1[k] > cap32 ? cap32 : j1[k];  // overflow (flagged at build)
        if constexpr (walk_counts<REL, EVM>()) {
          ++wrows;
          wcand += a1 > a0 ? a1 - a0 : 0;
        }
        if constexpr (REL) {
          // the lane's own slot stays in its row: at separation 0 it is
          // queued like a close pair, and flush_near drops it
          const uint32_t rowtag = ((uint32_t)(uint8_t)(ry[k] - g.cy) << 16) |
                                  ((uint32_t)(uint8_t)(rz[k] - g.cz) << 24);
          const int len = a1 - a0;
          // entries hold at most 65535 slots; a longer row goes to the exact pass
          if (len > 65535) {
            redo = true;
            continue;
          }
          if (len > 0) {
            segs[nseg][lane_id] = make_uint2((uint32_t)a0, (uint32_t)len | rowtag);
            ++nseg;
            steps += (len + 1) >> 1;
          }
        } else {
          if (a1 > a0) {
            segs[nseg][lane_id] = make_uint2((uint32_t)a0, (uint32_t)a1);
            ++nseg;
          }
        }
      }
    }
    if (nseg > 0) {
      if constexpr (REL) {
        segs[nseg][lane_id] = make_uint2(0u, 0xffffu);
        int nq = 0;
        scan_rel<EVM>(segs, steps, rs, g, (float)sig2, acc, cnt, nearq, nq);
        if (nq > kNearCap) redo = true;  // more close pairs than the queue holds
        flush_near<EVM>(nearq, nq, v.ext_pos, g, acc, cnt);
        acc.fx += (double)acc.px;
        acc.fy += (double)acc.py;
        acc.fz += (double)acc.pz;
        acc.px = acc.py = acc.pz = 0.0f;
      } else if constexpr (RULE == DCM_PAIR_MAX_N3)
        scan_n3<PREC, EVM>(segs, nseg, v, g, sig2, acc, cnt);
      else
        scan_ranges<RULE, PREC, EVM>(segs, nseg, v.ext_pos, g.self, g.xi, g.yi, g.zi, g.rci,
                                     g.rci2, sig2, acc, cnt);
    }
  }
}

// The block's deterministic partial sums: E = e_scale * sum of the lanes'
// energy terms, W = w_scale * virial terms, and the pair count.
template <int PREC>
__device__ __forceinline__ void block_partials(const Acc<PREC> &acc, int64_t cnt, double e_scale,
                                               double w_scale, double (*red)[kPartialSlots],
                                               double *partial_out) {
  double pv[kPartialSlots];
  pv[0] = (double)acc.e * e_scale;
#pragma unroll
  for (int k = 0; k < 6; ++k) pv[1 + k] = (double)acc.w[k] * w_scale;
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

// Lane order of a workgroup's particles for the own-cutoff walk on compact
// records.  A particle's walk grows with the cube of its cutoff, and near an
// interface the cutoffs of neighbouring cells differ by up to the whole
// ramp, so the 64 consecutive slots of a wavefront hold walks of very
// different lengths and the short ones idle until the longest ends.  The
// workgroup's particles are ranked by cutoff bin (kRcBins bins of rc_bound /
// kRcBins, the largest first; slot order within a bin; empty slots last) and
// lane t takes the particle of rank t, so each wavefront holds similar
// cutoffs.  The rank depends only on the workgroup's records: the same
// particles in the same slots give the same lanes in every kernel using it.
// scratch: kPairBlock + (kPairBlock / 64) * (kRcBins + 1) ints of LDS, free
// on entry and on return.  Returns the slot offset (0 .. kPairBlock - 1)
// this lane takes.
constexpr int kRcBins = 8;
static_assert((kNearCap + 1) * kPairBlock >= kPairBlock + (kPairBlock / 64) * (kRcBins + 1),
              "the lane order borrows the close-pair queue's LDS");
__device__ __forceinline__ int rc_lane_order(const double4 *pos, int64_t base, int64_t count,
                                             double rc_bound, int32_t *scratch) {
  constexpr int kKeys = kRcBins + 1;
  const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
  int key = kRcBins;  // empty slot
  if (t < count) {
    const double r = pos[base + t].w;
    const double q = rc_bound > 0.0 ? r * ((double)kRcBins / rc_bound) : 0.0;
    int b = q >= 0.0 ? (int)q : 0;  // NaN: bin 0
    b = b > kRcBins - 1 ? kRcBins - 1 : b;
    key = kRcBins - 1 - b;
  }
  int32_t *start = scratch + kPairBlock;  // [wave][key]
  unsigned long long mine = 0;
#pragma unroll
  for (int k = 0; k < kKeys; ++k) {
    const unsigned long long m = __ballot(key == k);
    mine = key == k ? m : mine;
    if (lane == 0) start[wave * kKeys + k] = __popcll(m);
  }
  __syncthreads();
  if (t == 0) {  // exclusive prefix over (key, wave)
    int acc = 0;
    for (int k = 0; k < kKeys; ++k)
      for (int w = 0; w < kPairBlock / 64; ++w) {
        const int c = start[w * kKeys + k];
        start[w * kKeys + k] = acc;
        acc += c;
      }
  }
  __syncthreads();
  const int rank = start[wave * kKeys + key] + __popcll(mine & ((1ull << lane) - 1ull));
  scratch[rank] = t;
  __syncthreads();
  const int mine_t = scratch[t];
  __syncthreads();
  return mine_t;
}

// Forces of the lane's particle to caller order (24 eps applied), its pair
// count, and the block's deterministic partial sums E, W[6], pair count.
template <int PREC>
__device__ __forceinline__ void finish_block(const int32_t *perm, int64_t id0, double *fx,
                                             double *fy, double *fz, int32_t *nnbr, int64_t s,
                                             bool active, double eps, const Acc<PREC> &acc,
                                             int cnt, double (*red)[kPartialSlots],
                                             uint32_t *status, double *partial_out) {
  if (active) {
    const double c24 = 24.0 * eps;
    const double Fx = c24 * acc.fx, Fy = c24 * acc.fy, Fz = c24 * acc.fz;
    const int64_t i = perm[s] - id0;
    fx[i] = Fx;
    fy[i] = Fy;
    fz[i] = Fz;
    if (nnbr) nnbr[i] = cnt;
    if (!finite3(Fx, Fy, Fz)) atomicOr(status, ST_NONFINITE_FORCE);
  }
  block_partials<PREC>(acc, cnt, 2.0 * eps, 12.0 * eps, red, partial_out);
}

// One block of kPairBlock particles: sorted slot s for this lane (active if
// it holds a particle).  Writes the forces and, from lanes 0..7, the block's
// partial sums E, W[6], pair count to partial_out.  REL: FP32-mixed
// own-cutoff evaluation on compact records, then the lanes that met an
// undecidable pair are recomputed from the FP64 records.  segs holds
// seg_cap<REL>() rows.
template <int RULE, int PREC, int EVM, bool REL, int CAP = seg_cap<REL>()>
__device__ __forceinline__ void pair_block(const PairView &v, int64_t s, bool active, double eps,
                                           double sig2, uint2 (*segs)[kPairBlock],
                                           int32_t (*nearq)[kPairBlock],
                                           double (*red)[kPartialSlots], uint32_t *status,
                                           double *partial_out) {
  Acc<PREC> acc;
  int cnt = 0;
  const int nx = v.nc[0], ny = v.nc[1], nz = v.nc[2];
  const int hx = v.h[0], hy = v.h[1], hz = v.h[2];
  const int nex = v.ne[0], ney = v.ne[1];
  LaneGeo g;
  g.xi = g.yi = g.zi = g.rci = g.rci2 = 0.0;
  g.a0x = g.a0y = g.a0z = g.wc = g.rc2f = g.margin = g.fR2 = g.fguard = g.hi2f = 0.0f;
  g.incw = 0u;
  // the FP32 r^2 of a pair at most a few ulps off: evaluating a pair just
  // past the threshold in FP64 as well costs nothing in accuracy
  g.near2f = (float)(kNear2 * sig2);
  g.sig2 = sig2;
  g.lenf[0] = g.lenf[1] = g.lenf[2] = 0.0f;
  g.invf[0] = g.invf[1] = g.invf[2] = 0.0f;
  for (int k = 0; k < 3; ++k) g.gp[k] = g.gm[k] = g.ac[k] = 0.0f;
  g.qinv = g.qac = 0.0f;
  g.qmin = g.qmax = 0;
  g.cx = 0;
  g.zlo = 0;
  g.zhi = -1;
  g.cy = g.cz = 0;
  g.self = -1;
  g.slot = (int)s;
  if (active) {
    const double4 pi = v.pos[s];
    g.xi = pi.x;
    g.yi = pi.y;
    g.zi = pi.z;
    g.rci = pi.w;
    double R = g.rci;
    if constexpr (RULE == DCM_PAIR_MAX) {
      double rall = __longlong_as_double((long long)*v.rc_all_bits);
      R = rall > R ? rall : R;
    }
    R = R < v.rc_bound ? R : v.rc_bound;
    g.rci2 = g.rci * g.rci;
    // search radius widened by a hair: rounding in the cell geometry can
    // only add candidates, never drop one
    const double Rg = R + 1e-9 * (v.len[0] + v.len[1] + v.len[2]);
    const int cx = slab_index(g.xi, v.sc[0], nx);
    g.cx = cx;
    g.cy = slab_index(g.yi, v.sc[1], ny);
    g.cz = slab_index(g.zi, v.sc[2], nz);
    g.a0x = (float)(g.xi - ((double)cx + 0.5) * v.len[0]);
    g.a0y = (float)(g.yi - ((double)g.cy + 0.5) * v.len[1]);
    g.a0z = (float)(g.zi - ((double)g.cz + 0.5) * v.len[2]);
    double lmax = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      g.lenf[k] = (float)v.len[k];
      g.invf[k] = (float)v.sc[k];
      lmax = v.len[k] > lmax ? v.len[k] : lmax;
    }
    // FP32 row selection: every quantity it forms is below ~Rg + 2 len, so its
    // roundings (and the hardware square root's ulp) stay below ~1e-6 (Rg + len);
    // the guard, 4e-6 (Rg + len), widens
    // every face distance and chord beyond them, and raises R^2 by
    // 2 Rg fguard, far above the ~4 u R^2 rounding of R^2 - ez^2 - ey^2
    g.fguard = (float)(4e-6 * (Rg + lmax));
    const float a0[3] = {g.a0x, g.a0y, g.a0z};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      g.gp[k] = fmaf(0.5f, g.lenf[k], a0[k]) + g.fguard;
      g.gm[k] = fmaf(0.5f, g.lenf[k], -a0[k]) + g.fguard;
      g.ac[k] = fmaf(a0[k], g.invf[k], 0.5f);
    }
    g.qinv = (float)kXSub * g.invf[0];
    g.qac = (float)kXSub * g.ac[0];
    g.qmin = kXSub * (-hx - cx);
    g.qmax = kXSub * (nx + hx - 1 - cx) + (kXSub - 1);
    const double Rf = Rg + (double)g.fguard;
    g.fR2 = (float)(Rf * Rf) * (1.0f + 0x1p-20f);
    if constexpr (REL) {
      g.wc = (float)cx + 0.5f;
      g.rc2f = (float)g.rci2;
      // Error of an FP32 separation component against the exact one, with
      // u = 2^-24 and a candidate at most k cells away (|k| len <= Rg + len):
      // a0 rounded (u len), len rounded (u |k| len), a0 - k len rounded
      // (u (Rg + 2 len)), the final difference rounded (u (Rg + 3 len)), and
      // the record's own error rel_delta; so del <= u (3 Rg + 7 len) + rel_delta.
      // For a pair within rc + 1 (the only ones whose side of rc^2 is in
      // question), |FP32 r^2 - FP64 r^2| <= E = 2 sqrt(3) (rc+1) del + 3 del^2
      // + 3 u (rc+1)^2 (the three roundings of r^2).  Outside a band of
      // E + u rc^2 (rc^2's own rounding) around the FP32 rc^2 the FP32 test
      // decides as the FP64 one; the band kept is twice that.
      const double u = 0x1p-24, rr = g.rci + 1.0;
      const double del = u * (3.0 * Rg + 7.0 * lmax) + v.rel_delta + 1e-12;
      const double E = 3.4641016151377548 * rr * del + 3.0 * del * del + 3.01 * u * rr * rr +
                       1e-12 * rr * rr;
      g.margin = (float)(2.0 * (E + u * g.rci2)) * (1.0f + 0x1p-20f);
      // the band's two edges as the FP32 tests use them, each moved outward
      // past the roundings of forming it and of r^2 - near^2 (relative
      // 2^-24 each): a pair these move only changes from the FP32 decision
      // to the FP64 one
      g.hi2f = (float)(((double)g.rc2f + (double)g.margin) * (1.0 + 0x1p-22));
      const double lo = ((double)g.rc2f - (double)g.margin - (double)g.near2f) * (1.0 - 0x1p-20);
      g.incw = lo > 0.0 ? __float_as_uint((float)lo) : 0u;
    }
    // the halo holds ceil(rc_bound/len) + 1 cells, so these stay inside it
    g.zlo = clampi((int)floor((g.zi - Rg) * v.sc[2]), -hz, nz + hz - 1);
    g.zhi = clampi((int)floor((g.zi + Rg) * v.sc[2]), -hz, nz + hz - 1);
    // this particle's own copy in the extended array
    const int real_cell = (g.cz * ny + g.cy) * nx + cx;
    const int ext_cell = ((g.cz + hz) * ney + (g.cy + hy)) * nex + (cx + hx);
    g.self = v.ext_start[ext_cell] + (int)(s - v.cell_start[real_cell]);
  }
  bool redo = false;
  int wcand = 0, wrows = 0;
  sweep_rows<RULE, PREC, EVM, REL, CAP>(v, active, g, sig2, segs, nearq, acc, cnt, redo, wcand,
                                        wrows);
  if constexpr (REL) {
    // rare: lanes with a row longer than a list entry can describe, or with
    // more close pairs in one chunk than their queue holds, start over on
    // the FP64 records
    if (__syncthreads_or(redo ? 1 : 0)) {
      if (redo) {
        acc = Acc<PREC>();
        cnt = 0;
      }
      bool unused = false;
      sweep_rows<RULE, PREC, EVM, false, CAP>(v, active && redo, g, sig2, segs, nearq, acc, cnt,
                                              unused, wcand, wrows);
    }
  }
  if constexpr (walk_counts<REL, EVM>()) {
    if (v.walk) {  // the lane's own slot lies in its rows but is no candidate
      const unsigned long long c = wave_sum_u64((unsigned long long)(wcand - (active ? 1 : 0)));
      const unsigned long long r = wave_sum_u64((unsigned long long)wrows);
      if ((threadIdx.x & 63) == 0) {
        atomicAdd(&v.walk[0], c);
        atomicAdd(&v.walk[1], r);
      }
    }
  }
  if constexpr (RULE == DCM_PAIR_MAX_N3) {
    // partners add to this particle's sums too; each pair counts for both
    // endpoints and carries its whole energy and virial
    if (active) {
      double *f = &v.n3_f[s].x;
      unsafeAtomicAdd(f, acc.fx);
      unsafeAtomicAdd(f + 1, acc.fy);
      unsafeAtomicAdd(f + 2, acc.fz);
      if (v.n3_cnt) atomicAdd(&v.n3_cnt[s], cnt);
    }
    block_partials<PREC>(acc, 2 * (int64_t)cnt, 4.0 * eps, 24.0 * eps, red, partial_out);
  } else {
    finish_block<PREC>(v.perm, v.id0, v.fx, v.fy, v.fz, v.nnbr, s, active, eps, acc, cnt, red,
                       status, partial_out);
  }
}

template <int RULE, int PREC, int EVM, bool REL>
__global__ __launch_bounds__(kPairBlock) void k_pair(PairArgs a) {
  __shared__ uint2 segs[seg_cap<REL>()][kPairBlock];
  __shared__ int32_t nearq[REL ? kNearCap + 1 : 1][kPairBlock];
  __shared__ double red[kPairBlock / 64][kPartialSlots];
  const int64_t lblock = xcd_block(blockIdx.x, gridDim.x, kXcdGroup);
  int64_t s = lblock * kPairBlock + threadIdx.x;
  if constexpr (REL)
    s = lblock * kPairBlock + rc_lane_order(a.pos, lblock * kPairBlock,
                                            a.n - lblock * kPairBlock, a.rc_bound, &nearq[0][0]);
  PairView v;
  v.pos = a.pos;
  v.cell_start = a.cell_start;
  v.perm = a.perm;
  v.id0 = 0;
  v.ext_pos = a.ext_pos;
  v.ext_rel = a.ext_rel;
  v.rel_delta = a.rel_delta;
  v.ext_start = a.ext_start;
  v.ext_sq = a.ext_sq;
  v.walk = a.walk;
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
  v.ext_src = a.ext_src;
  v.n3_f = a.n3_f;
  v.n3_cnt = a.n3_cnt;
  pair_block<RULE, PREC, EVM, REL>(v, s, s < a.n, a.eps, a.sigma * a.sigma, segs, nearq, red,
                                   a.status,
                              a.partials + lblock * kPartialSlots);
}

// Forces from a Verlet list (Algorithm 2.3, own-cutoff rule): the lane's
// list, entry k at wave_base + 64 k + lane, holds the candidates in the order
// of the cell walk, so the included pairs and their order are those of
// k_pair.
template <int PREC, int EVM>
__global__ __launch_bounds__(kPairBlock) void k_pair_list(PairArgs a, const int32_t *count,
                                                          const int32_t *wave_start,
                                                          const int32_t *list) {
  __shared__ double red[kPairBlock / 64][kPartialSlots];
  const int64_t s = blockIdx.x * (int64_t)kPairBlock + threadIdx.x;
  const bool active = s < a.n;
  Acc<PREC> acc;
  int cnt = 0;
  double xi = 0.0, yi = 0.0, zi = 0.0, rci = 0.0;
  int len = 0;
  if (active) {
    const double4 pi = a.pos[s];
    xi = pi.x;
    yi = pi.y;
    zi = pi.z;
    rci = pi.w;
    len = count[s];
  }
  const double rci2 = rci * rci, sig2 = a.sigma * a.sigma;
  int wmax = len;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const int o = __shfl_xor(wmax, off, 64);
    wmax = o > wmax ? o : wmax;
  }
  // wavefronts past the last particle read the first list (their lanes are idle)
  const int64_t w = (s >> 6) < ((a.n + 63) >> 6) ? (s >> 6) : 0;
  const int32_t *mine = list + 64 * (int64_t)wave_start[w] + (s & 63);
  // two entries per trip, each loaded a trip ahead of its use
  int k = 0;
  int ja = 0 < len ? mine[0] : 0;
  double4 A = a.ext_pos[ja];
  while (k < wmax) {
    const int jb = k + 1 < len ? mine[64 * (int64_t)(k + 1)] : ja;
    const double4 B = a.ext_pos[jb];
    if (k < len) candidate<DCM_PAIR_OWN, PREC, EVM>(A, ja, -1, xi, yi, zi, rci, rci2, sig2, acc, cnt);
    if (k + 1 >= wmax) break;
    const int jc = k + 2 < len ? mine[64 * (int64_t)(k + 2)] : jb;
    A = a.ext_pos[jc];
    if (k + 1 < len)
      candidate<DCM_PAIR_OWN, PREC, EVM>(B, jb, -1, xi, yi, zi, rci, rci2, sig2, acc, cnt);
    ja = jc;
    k += 2;
  }
  finish_block<PREC>(a.perm, 0, a.fx, a.fy, a.fz, a.nnbr, s, active, a.eps, acc, cnt, red,
                     a.status, a.partials + blockIdx.x * kPartialSlots);
}

template <int PREC>
static void launch_pair_list_ev(hipStream_t s, const PairArgs &a, const int32_t *count,
                                const int32_t *wave_start, const int32_t *list, dim3 g, dim3 b) {
  const int evm = ((a.ev_flags & DCM_EV_ENERGY) ? 1 : 0) | ((a.ev_flags & DCM_EV_VIRIAL) ? 2 : 0);
  switch (evm) {
    case 0: hipLaunchKernelGGL((k_pair_list<PREC, 0>), g, b, 0, s, a, count, wave_start, list); break;
    case 1: hipLaunchKernelGGL((k_pair_list<PREC, 1>), g, b, 0, s, a, count, wave_start, list); break;
    case 2: hipLaunchKernelGGL((k_pair_list<PREC, 2>), g, b, 0, s, a, count, wave_start, list); break;
    default: hipLaunchKernelGGL((k_pair_list<PREC, 3>), g, b, 0, s, a, count, wave_start, list); break;
  }
}

void launch_pair_list(hipStream_t s, const PairArgs &a, int prec, const int32_t *count,
                      const int32_t *wave_start, const int32_t *list) {
  const int64_t blocks = ceil_div(a.n, kPairBlock) > 0 ? ceil_div(a.n, kPairBlock) : 1;
  dim3 g((unsigned)blocks), b(kPairBlock);
  if (prec == DCM_FP64) launch_pair_list_ev<DCM_FP64>(s, a, count, wave_start, list, g, b);
  else launch_pair_list_ev<DCM_FP32_MIXED>(s, a, count, wave_start, list, g, b);
}

// Batched form: a persistent grid takes work items (blocks of kPairBlock
// particles of one system) from a queue in segments: one, ordered by
// estimated cost, or one per XCD holding whole systems, so that a system's
// records are read through one L2.  A workgroup drains its home segment
// (workgroup b runs on XCD b mod kXcds) and then the others in turn; it
// leaves the loop once every segment's position has passed its end.
template <int RULE, int PREC, int EVM, bool REL, int CAP = seg_cap<REL>()>
__global__ __launch_bounds__(kPairBlock) void k_pair_batched(BatchPairArgs a) {
  static_assert(CAP >= kFillRows + 4, "a chunk holds a batch of rows, a sentinel and a look-ahead");
  __shared__ uint2 segs[CAP][kPairBlock];
  __shared__ int32_t nearq[REL ? kNearCap + 1 : 1][kPairBlock];
  __shared__ double red[kPairBlock / 64][kPartialSlots];
  __shared__ int32_t next_item;
  const double sig2 = a.sigma * a.sigma;
  const int home = a.nqueues > 1 ? (int)(blockIdx.x % (unsigned)a.nqueues) : 0;
  int tried = 0;  // segments found empty
  while (true) {
    if (threadIdx.x == 0) {
      int32_t got = -1;
      while (tried < a.nqueues) {
        const int q = (home + tried) % a.nqueues;
        const int32_t pos = a.qseg[q] + (int32_t)atomicAdd(&a.head[q], 1u);
        if (pos < a.qseg[q + 1]) {
          got = pos;
          break;
        }
        ++tried;
      }
      next_item = got;
    }
    __syncthreads();
    const int32_t qi = next_item;
    __syncthreads();
    if (qi < 0) break;
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
    v.ext_rel = a.ext_rel;
    v.rel_delta = g.rel_delta;
    v.ext_start = a.ext_start + g.ext_cell0;
    v.ext_sq = a.ext_sq && (int64_t)g.ne[0] * g.ne[1] * g.ne[2] < kQStartMaxCells
                   ? a.ext_sq + g.ext_cell0
                   : nullptr;
    v.walk = nullptr;
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
    v.ext_src = nullptr;
    v.n3_f = nullptr;
    v.n3_cnt = nullptr;
    int64_t local = first + threadIdx.x;
    if constexpr (REL)
      local = first + rc_lane_order(a.pos, g.p0 + first, g.n - first, g.rc_cap, &nearq[0][0]);
    pair_block<RULE, PREC, EVM, REL, CAP>(v, g.p0 + local, local < g.n, a.eps, sig2, segs, nearq,
                                          red,
                                     a.status,
                                a.partials + (int64_t)item * kPartialSlots);
  }
}

// Evaluation-mode bits of the kernels: 1 energy, 2 virial, 4 pair counts.
// The compact-record kernels count only when asked (bit 4); the others always
// count, so their modes stop at 3.
static int ev_mode(int ev_flags, bool rel) {
  return ((ev_flags & DCM_EV_ENERGY) ? 1 : 0) | ((ev_flags & DCM_EV_VIRIAL) ? 2 : 0) |
         ((rel && (ev_flags & DCM_EV_COUNTS)) ? 4 : 0);
}

template <int RULE, int PREC, bool REL, int E = 0>
static void launch_pair_ev(hipStream_t s, const PairArgs &a, dim3 g, dim3 b, int evm) {
  if constexpr (E < (REL ? 8 : 4)) {
    if (evm == E) hipLaunchKernelGGL((k_pair<RULE, PREC, E, REL>), g, b, 0, s, a);
    else launch_pair_ev<RULE, PREC, REL, E + 1>(s, a, g, b, evm);
  }
}

void launch_pair(hipStream_t s, const PairArgs &a, int rule, int prec) {
  const int64_t blocks = ceil_div(a.n, kPairBlock) > 0 ? ceil_div(a.n, kPairBlock) : 1;
  dim3 g((unsigned)blocks), b(kPairBlock);
  const int evm = ev_mode(a.ev_flags, false);
  if (rule == DCM_PAIR_OWN) {
    if (prec == DCM_FP64) launch_pair_ev<DCM_PAIR_OWN, DCM_FP64, false>(s, a, g, b, evm);
    else if (a.ext_rel)
      launch_pair_ev<DCM_PAIR_OWN, DCM_FP32_MIXED, true>(s, a, g, b, ev_mode(a.ev_flags, true));
    else launch_pair_ev<DCM_PAIR_OWN, DCM_FP32_MIXED, false>(s, a, g, b, evm);
  } else if (rule == DCM_PAIR_MAX) {
    if (prec == DCM_FP64) launch_pair_ev<DCM_PAIR_MAX, DCM_FP64, false>(s, a, g, b, evm);
    else launch_pair_ev<DCM_PAIR_MAX, DCM_FP32_MIXED, false>(s, a, g, b, evm);
  } else {
    if (prec == DCM_FP64) launch_pair_ev<DCM_PAIR_MAX_N3, DCM_FP64, false>(s, a, g, b, evm);
    else launch_pair_ev<DCM_PAIR_MAX_N3, DCM_FP32_MIXED, false>(s, a, g, b, evm);
  }
}

// Rule DCM_PAIR_MAX_N3: the sorted-order sums (complete once the pair kernel
// has finished) to caller order.
__global__ __launch_bounds__(256) void k_n3_out(const double4 *__restrict__ f,
                                                const int32_t *__restrict__ cnt,
                                                const int32_t *__restrict__ perm, int64_t n,
                                                double c24, double *__restrict__ fx,
                                                double *__restrict__ fy, double *__restrict__ fz,
                                                int32_t *__restrict__ nnbr, uint32_t *status) {
  for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < n;
       s += (int64_t)gridDim.x * blockDim.x) {
    const double4 F = f[s];
    const double Fx = c24 * F.x, Fy = c24 * F.y, Fz = c24 * F.z;
    const int i = perm[s];
    fx[i] = Fx;
    fy[i] = Fy;
    fz[i] = Fz;
    if (nnbr) nnbr[i] = cnt[s];
    if (!finite3(Fx, Fy, Fz)) atomicOr(status, ST_NONFINITE_FORCE);
  }
}

void launch_n3_out(hipStream_t s, const double4 *f, const int32_t *cnt, const int32_t *perm,
                   int64_t n, double eps, double *fx, double *fy, double *fz, int32_t *nnbr,
                   uint32_t *status) {
  if (n <= 0) return;
  int64_t b = ceil_div(n, 256);
  if (b > 16384) b = 16384;
  hipLaunchKernelGGL(k_n3_out, dim3((unsigned)b), dim3(256), 0, s, f, cnt, perm, n, 24.0 * eps,
                     fx, fy, fz, nnbr, status);
}

template <int RULE, int PREC, bool REL, int CAP, int E = 0>
static void launch_pair_batched_ev(hipStream_t s, const BatchPairArgs &a, dim3 g, dim3 b,
                                   int evm) {
  if constexpr (E < (REL ? 8 : 4)) {
    if (evm == E) hipLaunchKernelGGL((k_pair_batched<RULE, PREC, E, REL, CAP>), g, b, 0, s, a);
    else launch_pair_batched_ev<RULE, PREC, REL, CAP, E + 1>(s, a, g, b, evm);
  }
}

int batched_row_lists(int k) { return k == 1 ? kSegCapRelWide : kSegCapRel; }

// Resident workgroups of the persistent kernel: what the occupancy allows on
// every compute unit, never more than the number of items.
static int64_t persistent_grid(int rule, int prec, bool wide, int64_t nitems) {
  static int cached[2][2][2] = {{{0, 0}, {0, 0}}, {{0, 0}, {0, 0}}};
  int &per_cu = cached[rule][prec][wide ? 1 : 0];
  if (per_cu == 0) {
    const void *fn;
    if (rule == DCM_PAIR_OWN)
      fn = prec == DCM_FP64
               ? (const void *)k_pair_batched<DCM_PAIR_OWN, DCM_FP64, 3, false>
               : (wide ? (const void *)k_pair_batched<DCM_PAIR_OWN, DCM_FP32_MIXED, 7, true,
                                                     kSegCapRelWide>
                       : (const void *)k_pair_batched<DCM_PAIR_OWN, DCM_FP32_MIXED, 7, true>);
    else
      fn = prec == DCM_FP64 ? (const void *)k_pair_batched<DCM_PAIR_MAX, DCM_FP64, 3, false>
                            : (const void *)k_pair_batched<DCM_PAIR_MAX, DCM_FP32_MIXED, 3, false>;
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

void launch_pair_batched(hipStream_t s, const BatchPairArgs &a, int rule, int prec,
                         int row_lists) {
  if (a.nitems <= 0) return;
  constexpr int kF = seg_cap<false>(), kR = kSegCapRel, kW = kSegCapRelWide;
  // the row-list capacity is a choice of the compact-record kernel only
  const bool wide = rule == DCM_PAIR_OWN && prec != DCM_FP64 && a.ext_rel && row_lists == 1;
  dim3 g((unsigned)persistent_grid(rule, prec, wide, a.nitems)), b(kPairBlock);
  const int evm = ev_mode(a.ev_flags, false);
  if (rule == DCM_PAIR_OWN) {
    if (prec == DCM_FP64)
      launch_pair_batched_ev<DCM_PAIR_OWN, DCM_FP64, false, kF>(s, a, g, b, evm);
    else if (a.ext_rel && wide)
      launch_pair_batched_ev<DCM_PAIR_OWN, DCM_FP32_MIXED, true, kW>(s, a, g, b,
                                                                     ev_mode(a.ev_flags, true));
    else if (a.ext_rel)
      launch_pair_batched_ev<DCM_PAIR_OWN, DCM_FP32_MIXED, true, kR>(s, a, g, b,
                                                                     ev_mode(a.ev_flags, true));
    else
      launch_pair_batched_ev<DCM_PAIR_OWN, DCM_FP32_MIXED, false, kF>(s, a, g, b, evm);
  } else {
    if (prec == DCM_FP64)
      launch_pair_batched_ev<DCM_PAIR_MAX, DCM_FP64, false, kF>(s, a, g, b, evm);
    else
      launch_pair_batched_ev<DCM_PAIR_MAX, DCM_FP32_MIXED, false, kF>(s, a, g, b, evm);
  }
}

// Sum the block partials in a fixed order (one workgroup), so the energy,
// virial and pair count do not depend on scheduling.  ONLY_E: the energy
// alone (slot 0 of each block), the same sum as in the full reduction.
template <bool ONLY_E>
__global__ __launch_bounds__(kReduceThreads) void k_reduce_partials(
    const double *__restrict__ partials, int64_t blocks, int ev_flags, double *energy,
    double *virial, uint64_t *npairs) {
  constexpr int S = ONLY_E ? 1 : kPartialSlots;
  __shared__ double red[kReduceThreads / 64][S];
  double t[S];
  sum_rows<kReduceThreads, S, kPartialSlots>(partials, blocks, red, t);
  if (threadIdx.x == 0) {
    if (energy && (ev_flags & DCM_EV_ENERGY)) *energy = t[0];
    if constexpr (!ONLY_E) {
      if (virial && (ev_flags & DCM_EV_VIRIAL))
        for (int k = 0; k < 6; ++k) virial[k] = t[1 + k];
      if (npairs && (ev_flags & DCM_EV_COUNTS)) *npairs = (uint64_t)t[7];
    }
  }
}

void launch_reduce_partials(hipStream_t s, const double *partials, int64_t blocks, double eps,
                            int ev_flags, double *energy, double *virial, uint64_t *npairs) {
  (void)eps;
  const bool only_e = !(ev_flags & (DCM_EV_VIRIAL | DCM_EV_COUNTS)) || (!virial && !npairs);
  if (only_e)
    hipLaunchKernelGGL(k_reduce_partials<true>, dim3(1), dim3(kReduceThreads), 0, s, partials,
                       blocks, ev_flags, energy, virial, npairs);
  else
    hipLaunchKernelGGL(k_reduce_partials<false>, dim3(1), dim3(kReduceThreads), 0, s, partials,
                       blocks, ev_flags, energy, virial, npairs);
}

}  // namespace dcm
