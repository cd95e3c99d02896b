// Internal declarations of the gfx950 DCM library: the context, device
// control block, status bits and the host-side launchers of every kernel.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstdint>
#include <map>
#include <string>
#include <vector>

#include "../../include/dcm.h"

namespace dcm {

// Sticky device status bits (OR-ed by kernels, read by dcm_sync_status).
enum : uint32_t {
  ST_NONFINITE_POS = 1u << 0,
  ST_HIST_RANGE = 1u << 1,
  ST_DEGENERATE = 1u << 2,
  ST_NOT_CONVERGED = 1u << 3,
  ST_NONFINITE_FORCE = 1u << 4,
  ST_RC_RANGE = 1u << 5,
  ST_GHOST_OVERFLOW = 1u << 6,
};

constexpr int kHistBins = 4096;       // gray values (27-window counts) must stay below this
constexpr int kHistCopies = 32;      // histogram copies the gray-value workgroups add into
constexpr int kMajorityMaxPasses = 16;
constexpr int kBatchQueues = 8;  // work-queue segments of the XCD-affine batched plan (one per XCD)
constexpr int kPartialSlots = 8;      // per-block partial sums: E, W[6], pair count
constexpr int kReduceThreads = 1024;  // workgroup that sums the block partials
constexpr int kReorderEvery = 8;      // dcm_step re-sorts its working copies this often
// the pair kernel addresses the ghost-extended array with 32-bit byte offsets
constexpr int64_t kMaxExtSlots = (int64_t(1) << 27) - 1;

// Bound on the per-coordinate error of a separation rebuilt from the compact
// (cell-centre-relative FP32) candidate records: half an FP32 ulp of the
// largest offset from a cell centre (half the largest cell edge, widened a
// hair for particles binned across a rounded cell boundary), plus the FP64
// rounding of forming the offset and of rebuilding, each at most a few units
// of 2^-53 of the largest extended-grid coordinate `span`.
inline double rel_record_delta(const double len[3], double span) {
  const double m = std::max(len[0], std::max(len[1], len[2]));
  int e = 0;
  std::frexp(0.5 * m * (1.0 + 1e-9), &e);  // in [2^(e-1), 2^e): ulp 2^(e-24)
  return std::ldexp(1.0, e - 25) + 1e-15 * (span + 1.0);
}
// the compact-record path packs a row's cell offset from the lane's cell in
// 8 bits, so it needs halos of at most this many cells
constexpr int kRelMaxHalo = 127;
// Compact records only for cells at most this many LJ sigma wide: their FP32
// positions relative to cell centres err by up to ~2^-24 times the edge, and
// the force of a close pair amplifies a separation error ~14-fold, so wider
// cells would push FP32-mixed forces past 1e-5; those read the FP64 records.
constexpr double kRelMaxEdgeSigma = 2.0;

// Device-resident control block: scalars produced and consumed on the device
// so that no stage needs a host round trip.
// Iterated stages (majority passes, sweep passes) keep one "changed" flag per
// pass instead of counters: every workgroup that saw a change stores 1 into
// its pass's slot (no atomics), and pass p+1 runs only if pass p changed
// something.  The stage's final kernel finds the last pass from the flags.
struct Ctl {
  // interface detection
  int32_t threshold;
  int32_t degenerate;
  double c0, c1;
  // majority pass p stores into maj_chg1[p] (differs from state p-1) and
  // maj_chg2[p] (differs from state p-2)
  uint32_t maj_chg1[kMajorityMaxPasses + 2];
  uint32_t maj_chg2[kMajorityMaxPasses + 2];
  // cells: largest cutoff seen (bit pattern of a non-negative double), and
  // the number of cells too large for a one-thread sort (zeroed with it)
  unsigned long long rc_max_bits;
  uint32_t big_cells;
};

// Device allocation owned by its holder (freed when the holder goes).
struct DevBuf {
  void *p = nullptr;
  size_t cap = 0;
  DevBuf() = default;
  DevBuf(const DevBuf &) = delete;
  DevBuf &operator=(const DevBuf &) = delete;
  ~DevBuf() {
    if (p) (void)hipFree(p);  // nothing to report from a destructor
  }
};

struct Timer {
  double ms = 0.0;
  int64_t launches = 0;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pending;
};

// One system of a batch as the device sees it: the caller's arrays, its
// slices of the concatenated particle, cell and extended-cell orders, and
// its cell geometry.
struct SysGeom {
  const double *x, *y, *z, *rc;
  double *fx, *fy, *fz;
  int32_t *nnbr;
  double *energy, *virial;
  uint64_t *npairs;
  int64_t n;
  int64_t p0;         // first slot of the system in the concatenated particle order
  int64_t cell0;      // first real cell
  int64_t ext_cell0;  // first extended cell
  int64_t row0;       // first extended row (rows: ne[1] * ne[2] per system)
  int64_t item0;      // first pair work item (blocks of 256 particles)
  int64_t nitems;
  double rel_delta;   // error bound of the compact records (rel_record_delta)
  int32_t nc[3], h[3], ne[3];
  double len[3], sc[3], L[3];
  double rc_cap;
};

struct BatchState;  // dcm_batch.cpp

}  // namespace dcm

struct dcm_ctx {
  hipStream_t stream = nullptr;
  int device = 0;
  std::string err;
  uint32_t *d_status = nullptr;
  uint32_t *h_status = nullptr;  // pinned
  dcm::Ctl *ctl = nullptr;       // device control block
  // grid scratch
  dcm::DevBuf counts, gray, hist, seg_a, seg_b, dA, dB, fsm_chg,
      fsm_flags;
  dcm::DevBuf ccl_label, ccl_size;  // bubble filter
  // Verlet list of the last cell build
  dcm::DevBuf list_count, list_wave_len, list_wave_start, list;
  dcm::DevBuf list_ref, list_part, list_out;
  int64_t list_n = -1;  // particles of the list (-1: none built)
  double list_skin = 0.0;
  int32_t *h_list_total = nullptr;  // pinned: entries / 64 of the last build
  double *h_list_verdict = nullptr; // pinned: [displacement, slack] of the last update
  bool cells_moved = false;  // positions replaced by dcm_update_list since the build
  // particle scratch
  dcm::DevBuf delta, rc, partials, ke, scalars;
  dcm::DevBuf tune_f;  // forces of the cell-edge tuner's trial passes (dcm_build_cells)
  // cells
  dcm::DevBuf cell_of, cell_count, cell_start, cell_fill, perm, sorted, scan_tmp, rcmax_part;
  // x key of every particle (within-cell order), sub-cell word of every real
  // cell and (start, sub-cell word) of every extended cell (the pair walk's
  // x trimming)
  dcm::DevBuf xkey, skey, qword, ext_sq;
  // candidates tested and rows visited by the last DCM_EV_COUNTS cell walk
  dcm::DevBuf walk;
  bool walk_valid = false;
  dcm::DevBuf sort_tmp, sort_list;  // large-cell sort: scratch entries and the cells' list
  dcm::DevBuf ext_row_count, ext_row_start, ext_row_lo, ext_start, ext_pos;
  dcm::DevBuf ext_rel;  // FP32-mixed builds: compact cell-relative copy of ext_pos
  dcm::DevBuf ext_src;  // sorted slot of each extended slot's particle (on demand)
  bool ext_src_ok = false;  // ext_src belongs to the current cell build
  dcm::DevBuf n3_f, n3_cnt;  // Newton's-third-law forces and counts in sorted order
  int64_t ext_cap = 0;             // particles ext_pos can hold
  int32_t *h_ext_total = nullptr;  // pinned: ghost-extended count of the last build
  // the copy into h_ext_total completes with ext_event; the count is kept for
  // the next build of the same cell geometry (ext_key: cells, halo, n)
  hipEvent_t ext_event = nullptr;
  bool ext_copy_pending = false;
  int64_t ext_key[7] = {-1, -1, -1, -1, -1, -1, -1};
  int64_t ext_exact = -1;  // synchronised count of the last build with ext_key
  int32_t nc[3] = {0, 0, 0};
  int32_t halo[3] = {0, 0, 0};
  double rc_bound = 0.0;
  double cell_len[3] = {0, 0, 0};
  double cell_scale[3] = {0, 0, 0};
  dcm_box cell_box = {{0, 0, 0}};
  int64_t cell_n = -1;
  int cell_prec = 0;
  bool cell_rel = false;  // the last build wrote ext_rel
  bool cell_qtab = false; // ... and the trimming table ext_sq
  // dcm_step's working copies in cell order: two sets of 11 fields (x y z,
  // vx vy vz, fx fy fz, delta, rc) and the caller index of each slot
  dcm::DevBuf ws[2], ws_owner[2];
  // last distance field kept for dcm_step, with what it was computed for
  bool have_field = false;
  int32_t field_n[3] = {0, 0, 0};
  double field_h[3] = {0, 0, 0}, field_L[3] = {0, 0, 0};
  double field_rc_grid = 0.0;
  int64_t field_particles = -1;
  int32_t field_waves = 0;  // pass limit of the sweep whose buffers hold the field
  // batched form: plan, buffers and recorded graph
  dcm::BatchState *batch = nullptr;
  int batch_queues = 0;  // work-queue layout asked for (0: tuned)
  // dcm_step: a second stream on which the cell build of a step runs beside
  // the sweep, with its fork and join events; while that build is enqueued,
  // stream is the second stream and forked_from the context's own
  hipStream_t side = nullptr;
  hipEvent_t fork_ev = nullptr, join_ev = nullptr;
  hipStream_t forked_from = nullptr;
  // set for the next cell build: build without the cutoffs (the sorted
  // records' rc comes later, from the cutoff assignment); consumed by that build
  bool build_no_rc = false;
  int batch_lists = 0;   // row-list variant asked for (0: tuned, 1: 14 entries, 2: 16)
  // profiling
  bool profile = false;
  std::string profile_only;  // record only this family ("" = every family)
  std::map<std::string, dcm::Timer> timers;
};

namespace dcm {

// ---- interface detection in parts (dcm_api.cpp): argument checks, and the
// launches on given scratch buffers (counts, gray values, histogram copies,
// the two bit-packed phase maps; the bubble filter's labels and sizes when
// opts.min_volume > 0)
struct DetectScratch {
  uint32_t *counts = nullptr, *gray = nullptr, *hist = nullptr, *seg_a = nullptr,
           *seg_b = nullptr;
  int32_t *ccl_label = nullptr, *ccl_size = nullptr;
};
// the context's detection scratch for a grid of nvox voxels (counts: the
// caller's, or null for the context's own)
dcm_status detect_scratch(dcm_ctx *ctx, const dcm_grid &grid, int64_t nvox,
                          const dcm_detect_opts &opts, uint32_t *counts, DetectScratch *out);
dcm_status detect_check(dcm_ctx *ctx, const double *x, const double *y, const double *z,
                        int64_t n, const dcm_box &box, const dcm_grid &grid,
                        const dcm_detect_opts *opts, const uint8_t *seg, const uint8_t *iface,
                        int64_t *nvox);
// binned: the counts (and the zeroed histogram) are in sc already
dcm_status detect_enqueue(dcm_ctx *ctx, const double *x, const double *y, const double *z,
                          int64_t n, const dcm_box &box, const dcm_grid &grid,
                          const dcm_detect_opts &opts, const DetectScratch &sc, uint8_t *seg,
                          uint8_t *iface, int32_t *threshold_out, bool timed,
                          bool binned = false);
// dcm_noalloc.hip: look up (once per device) the device address of the
// static scratch array of dcm_detect_interface_noalloc
dcm_status noalloc_scratch_setup(int device, std::string *err);

// ---- context helpers (dcm_api.cpp)
dcm_status fail(dcm_ctx *ctx, dcm_status code, const std::string &msg);
dcm_status ensure(dcm_ctx *ctx, DevBuf &b, size_t bytes);
dcm_status check_launch(dcm_ctx *ctx, const char *what);
void timer_begin(dcm_ctx *ctx, const char *family, hipEvent_t *ev);
void timer_end(dcm_ctx *ctx, const char *family, hipEvent_t ev);
void batch_free(dcm_ctx *ctx);  // dcm_batch.cpp

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// ---- launchers (one per kernel family; all enqueue on ctx->stream)
// k_common.hip
void launch_fill_u32(hipStream_t s, uint32_t *p, uint32_t v, int64_t n);
void launch_fill_i32(hipStream_t s, int32_t *p, int32_t v, int64_t n);
// p[0..n) = q[0..n) = 0 in one launch
void launch_zero2_i32(hipStream_t s, int32_t *p, int32_t *q, int64_t n);
// p[0..np) = 0 and q[0..nq) = 0 in one launch
void launch_zero2_u32(hipStream_t s, uint32_t *p, int64_t np, uint32_t *q, int64_t nq);
void launch_reset_ctl(hipStream_t s, Ctl *ctl);
void launch_min_f64(hipStream_t s, const double *v, int64_t n, double *out);
void launch_clear_status(hipStream_t s, uint32_t *st);

// k_grid.hip
void launch_bin_density(hipStream_t s, const double *x, const double *y, const double *z,
                        int64_t n, const double L[3], const int32_t nv[3], const double sc[3],
                        uint32_t *counts, uint32_t *status);
void launch_gray_hist(hipStream_t s, const uint32_t *counts, uint32_t *gray, const int32_t nv[3],
                      uint32_t *hist, uint32_t *status);
void launch_otsu(hipStream_t s, const uint32_t *hist, int64_t nvox, Ctl *ctl, int32_t *t_out,
                 uint32_t *status);
// phase maps of the majority passes are bit-packed: ceil(nx/32) words per
// x-row; phase_bits_words gives the words of one map
int64_t phase_bits_words(const int32_t nv[3]);
// one length-term pass (same buffers and flags as launch_majority_pass)
void launch_potts_pass(hipStream_t s, uint32_t *buf0, uint32_t *buf1, const uint32_t *gray,
                       const int32_t nv[3], double nu, int pass, Ctl *ctl);
// k_ccl.hip: bubble filter on the byte phase map, then its interface
void launch_bubble_filter(hipStream_t s, const int32_t nv[3], int64_t min_volume, uint8_t *seg,
                          uint8_t *iface, int32_t *label, int32_t *size, uint32_t *status);
void launch_threshold(hipStream_t s, const uint32_t *gray, const int32_t nv[3], double split,
                      const Ctl *ctl, uint32_t *bits0, int32_t *t_out);
void launch_majority_pass(hipStream_t s, uint32_t *buf0, uint32_t *buf1, const int32_t nv[3],
                          int pass, int max_passes, Ctl *ctl);
// byte maps of the final phase and the interface
void launch_interface(hipStream_t s, const uint32_t *buf0, const uint32_t *buf1,
                      const int32_t nv[3], const Ctl *ctl, uint8_t *seg, uint8_t *iface);

// k_fsm.hip
// initial distances; with tiles also the first pass's tile flags in chg0
// the same from the regularisation passes' two bit-packed phase maps (the
// final one chosen from the pass flags, as launch_interface does)
void launch_fsm_init_bits(hipStream_t s, const uint32_t *const maps[2], const Ctl *ctl,
                          const int32_t nv[3], double *dA, double *dB, uint8_t *chg0,
                          uint32_t *flags, int max_steps);
void launch_fsm_init(hipStream_t s, const uint8_t *seg, const uint8_t *iface, const int32_t nv[3],
                     double *dA, double *dB, uint8_t *chg0, uint32_t *flags, int max_steps);
// one launch of the sweep: a temporally blocked tile pass when fsm_tiled(nv),
// else one synchronous wave; chg0/chg1 hold one flag per tile
bool fsm_tiled(const int32_t nv[3]);
int64_t fsm_tile_count(const int32_t nv[3]);
void launch_fsm_step(hipStream_t s, double *dA, double *dB, uint8_t *chg0, uint8_t *chg1,
                     const int32_t nv[3], const double h[3], double rc_grid, int step,
                     uint32_t *flags);
void launch_fsm_final(hipStream_t s, const double *dA, const double *dB, int64_t nvox,
                      double rc_grid, const uint32_t *flags, int max_steps, double *dist,
                      int32_t *waves_out, uint32_t *status);

// k_cells.hip
// the same from the distance sweep's buffers (dA, dB) and pass flags, as
// its final pass would have written the field (see launch_fsm_final); with
// perm, for cells built without the cutoffs: the threads walk the sorted
// slots and sorted[slot].w takes rc[perm[slot]] clamped to [0, rc_cap]
// (out of range flagged)
void launch_assign_cutoffs_sweep(hipStream_t s, const double *x, const double *y,
                                 const double *z, int64_t n, const double L[3],
                                 const int32_t nv[3], const double sc[3], const double *dA,
                                 const double *dB, const uint32_t *flags, int max_steps,
                                 double rc_grid, dcm_rule rule, double *delta, double *rc,
                                 uint32_t *status, const int32_t *perm = nullptr,
                                 double4 *sorted = nullptr, double rc_cap = 0.0);
void launch_assign_cutoffs(hipStream_t s, const double *x, const double *y, const double *z,
                           int64_t n, const double L[3], const int32_t nv[3],
                           const double sc[3], const double *dist, dcm_rule rule,
                           double *delta, double *rc);
// workgroups of the cell-count kernel: the size of its block_max scratch
int64_t cell_count_blocks(int64_t n);
void launch_cell_count(hipStream_t s, const double *x, const double *y, const double *z,
                       const double *rc, int64_t n, const double L[3], const int32_t nc[3],
                       const double sc[3], double rc_cap, int32_t *cell_of, int32_t *cell_count,
                       unsigned long long *block_max, uint32_t *xq, Ctl *ctl, uint32_t *status);
void launch_exclusive_scan(hipStream_t s, const int32_t *in, int32_t *out, int64_t n,
                           int32_t *tmp);
int64_t scan_tmp_elems(int64_t n);
// perm[slot] = id and skey[slot] = xq[id] for every particle's slot in its cell
void launch_cell_scatter(hipStream_t s, const int32_t *cell_of, int64_t n,
                         const int32_t *cell_start, int32_t *cell_fill, int32_t *perm,
                         const uint32_t *xq, uint32_t *skey);
// The sorted copy written by the cell sort itself (launch_cell_sort with go
// not null): sorted[slot] = (x, y, z, rc) of the particle sorted_perm[slot],
// positions wrapped into the box (0 when not finite), rc clamped to
// [0, rc_cap] (NaN -> 0).
struct GatherOut {
  const double *x, *y, *z, *rc;
  double L[3];
  double rc_cap;
  double4 *sorted;
};
// sorted_perm receives the entries of perm (particle ids in cell order, cell
// c of particle id holding cell_of[id], x keys xq by id and skey by slot)
// with each cell's sorted by (x key, id); perm is left as scratch.  qword (null: none) receives the
// cells' sub-cell words (sub_word: prefix counts of each cell's eighths
// along x, 0 for cells of more than 15).  big_list holds
// cell_sort_list_elems(n) entries; big_count must be 0 on entry.
void launch_cell_sort(hipStream_t s, const int32_t *cell_start, int64_t ncell,
                      const int32_t *cell_of, int64_t n, int32_t *perm, const uint32_t *xq,
                      const uint32_t *skey, uint32_t *qword, int32_t *sorted_perm,
                      int32_t *big_list, uint32_t *big_count, const GatherOut *go = nullptr);
int64_t cell_sort_list_elems(int64_t n);
// rows of the extended grid + 1: the size of each per-row scratch array
int64_t ext_row_scratch_elems(const int32_t nc[3], const int32_t h[3]);
// ghost-extended cells in two parts: the per-row tables and the extended
// cell starts (ext_start[next] then holds the extended particle count), and
// the images themselves into buffers of ext_cap slots.  ext_sq (null: none;
// int2 [next + 1]) receives (ext_start, sub-cell word of the real cell) of
// every extended cell and (extended count, 0) past the last.
void launch_ext_count(hipStream_t s, const int32_t *cell_start, const int32_t nc[3],
                      const int32_t h[3], const double L[3], int32_t *row_count,
                      int32_t *row_start, int32_t *row_lo, int32_t *ext_start,
                      int32_t *scan_tmp, const uint32_t *qword, int2 *ext_sq);
void launch_ext_images(hipStream_t s, const int32_t *cell_start, const int32_t *row_start,
                       const int32_t *row_lo, const double4 *sorted, const int32_t nc[3],
                       const int32_t h[3], const double L[3], int64_t ext_cap, double4 *ext_pos,
                       float4 *ext_rel, uint32_t *status);
// source sorted slot of every extended slot of the last build (row tables)
void launch_ext_src(hipStream_t s, const int32_t *cell_start, const int32_t *row_start,
                    const int32_t *row_lo, const int32_t nc[3], const int32_t h[3],
                    const double L[3], int64_t ext_cap, int32_t *ext_src, uint32_t *status);
// ghost images again from new positions of the same cells (the row tables of
// the last build), without compact records
void launch_ext_refill(hipStream_t s, const int32_t *cell_start, const int32_t *row_start,
                       const int32_t *row_lo, const double4 *sorted, const int32_t nc[3],
                       const int32_t h[3], const double L[3], int64_t ext_cap, double4 *ext_pos,
                       uint32_t *status);

// Extended grids of at least this many cells get no trimming table (its
// 32-bit byte offsets would overflow): their pair walks take whole end cells.
constexpr int64_t kQStartMaxCells = int64_t(1) << 28;

// k_pair.hip
struct PairArgs {
  const double4 *pos;        // sorted real particles (x, y, z, rc), wrapped into the box
  const int32_t *cell_start; // real cells [ncell + 1]
  const int32_t *perm;       // sorted -> caller index
  const double4 *ext_pos;    // real cells plus periodic ghost images, by extended cell
  const float4 *ext_rel;     // compact cell-relative copy of ext_pos, or null
  double rel_delta;          // its per-coordinate error bound
  const int32_t *ext_start;  // extended cells [next + 1]
  const int2 *ext_sq;        // (start, sub-cell word) of the extended cells [next + 1], or null
  unsigned long long *walk;  // DCM_EV_COUNTS cell walks: candidates, rows (zeroed), or null
  int64_t n;
  int64_t ext_cap;           // capacity of ext_pos
  int32_t nc[3];
  int32_t h[3];              // ghost cells on each side
  int32_t ne[3];             // extended cells per axis = nc + 2h
  double len[3];             // cell edge per axis = L/n
  double sc[3];              // n/L
  double L[3];
  double rc_bound;
  double eps, sigma;
  int ev_flags;
  const Ctl *ctl;
  double *fx, *fy, *fz;
  int32_t *nnbr;
  double *partials;          // [blocks * kPartialSlots]
  uint32_t *status;
  // rule DCM_PAIR_MAX_N3: source slots of ext_pos, and the sorted-order
  // force and count sums the pairs' both endpoints are added to (zeroed)
  const int32_t *ext_src;
  double4 *n3_f;
  int32_t *n3_cnt;           // null without DCM_EV_COUNTS
};
int pair_block_size();
void launch_pair(hipStream_t s, const PairArgs &a, int rule, int prec);
// rule DCM_PAIR_MAX_N3: sorted-order sums to caller order (24 eps applied)
void launch_n3_out(hipStream_t s, const double4 *f, const int32_t *cnt, const int32_t *perm,
                   int64_t n, double eps, double *fx, double *fy, double *fz, int32_t *nnbr,
                   uint32_t *status);
// forces over a Verlet list (k_list.hip layout), own-cutoff rule
void launch_pair_list(hipStream_t s, const PairArgs &a, int prec, const int32_t *count,
                      const int32_t *wave_start, const int32_t *list);

// k_list.hip: Verlet list with a skin on the cells of the last build
struct ListArgs {
  const double4 *pos;        // sorted particles (x, y, z, rc)
  const int32_t *cell_start;
  const double4 *ext_pos;
  const int32_t *ext_start;
  int64_t n, ext_cap;
  int32_t nc[3], h[3], ne[3];
  double len[3], sc[3];
  double rc_bound, skin;
  int32_t *count;            // [n] list lengths
  int32_t *wave_len;         // [n_waves] longest list of each wavefront
  const int32_t *wave_start; // [n_waves + 1] exclusive scan of wave_len
  int64_t n_waves;
  int32_t *list;             // [list_cap]
  int64_t list_cap;
  double4 *ref;              // [n] build position and list radius R (count pass)
  uint32_t *status;
};
int64_t list_waves(int64_t n);
int64_t list_update_blocks(int64_t n);
// new positions and cutoffs for the cells of the list's build (sorted order),
// out[0] = largest displacement from the build, out[1] = smallest R - r_c
void launch_list_update(hipStream_t s, const double *x, const double *y, const double *z,
                        const double *rc, const int32_t *perm, const double4 *ref, int64_t n,
                        const double L[3], double rc_cap, double4 *sorted, double2 *part,
                        double *out, uint32_t *status);
void launch_list_count(hipStream_t s, const ListArgs &a);
void launch_list_fill(hipStream_t s, const ListArgs &a);

struct BatchPairArgs {
  const SysGeom *sys;
  const int2 *items;          // work item -> (system, first local particle)
  const int32_t *queue;       // items in the order they are handed out, in nqueues segments
  const int32_t *qseg;        // [nqueues + 1] segment starts in queue
  int32_t nqueues;            // 1, or kXcds: segment x first serves workgroups on XCD x
  int32_t nitems;
  uint32_t *head;             // [nqueues] positions in the segments, zero before the launch
  const double4 *pos;         // sorted particles, concatenated
  const int32_t *cell_start;  // concatenated real cells
  const int32_t *perm;        // sorted slot -> concatenated particle id
  const float4 *ext_rel;      // compact cell-relative copy of ext_pos, or null
  const double4 *ext_pos;
  const int32_t *ext_start;   // concatenated extended cells
  const int2 *ext_sq;         // their (start, sub-cell word) [cells + 1], or null
  int64_t ext_cap;
  const unsigned long long *rc_max_bits;  // per system
  double eps, sigma;
  int ev_flags;
  double *partials;           // [nitems * kPartialSlots], by item
  uint32_t *status;
};
// row_lists: 0 or 1, the compact-record kernel's row-list variant (entries
// per lane: batched_row_lists(row_lists)); other kernels have one
void launch_pair_batched(hipStream_t s, const BatchPairArgs &a, int rule, int prec,
                         int row_lists);
int batched_row_lists(int k);

// k_batch.hip: build kernels of the batched form.  pblk holds one (system,
// first local particle) entry per block of 256 particles, eblk one (system,
// first local extended cell) entry per block of 256 extended cells.
void launch_batch_cell_count(hipStream_t s, const SysGeom *sys, int32_t nsys, const int2 *pblk,
                             int64_t npblk, int32_t *cell_of, int32_t *cell_count,
                             unsigned long long *block_max, unsigned long long *rc_max_bits,
                             uint32_t *xq, uint32_t *status);
void launch_batch_cell_scatter(hipStream_t s, const SysGeom *sys, const int2 *pblk,
                               int64_t npblk, const int32_t *cell_of, const int32_t *cell_start,
                               int32_t *cell_fill, int32_t *perm, const uint32_t *xq,
                               uint32_t *skey);
void launch_batch_gather(hipStream_t s, const SysGeom *sys, const int2 *pblk, int64_t npblk,
                         const int32_t *order, double4 *sorted, int32_t *perm);
void launch_batch_ext(hipStream_t s, const SysGeom *sys, const int2 *eblk, int64_t neblk,
                      const int2 *rblk, int64_t nrblk, const int32_t *cell_start,
                      const double4 *sorted, int64_t next_total, int64_t nrows_total,
                      int64_t ext_cap, int32_t *row_count, int32_t *row_start, int32_t *row_lo,
                      int32_t *ext_start, int32_t *scan_tmp, double4 *ext_pos, float4 *ext_rel,
                      const uint32_t *qword, int2 *ext_sq, uint32_t *status);
void launch_batch_reduce(hipStream_t s, const SysGeom *sys, int32_t nsys,
                         const double *partials, int ev_flags);
void launch_fill_u64(hipStream_t s, unsigned long long *p, unsigned long long v, int64_t n);
void launch_reduce_partials(hipStream_t s, const double *partials, int64_t blocks, double eps,
                            int ev_flags, double *energy, double *virial, uint64_t *npairs);

// k_order.hip
constexpr int kPermFields = 11;
struct PermFields {
  const double *src[kPermFields];
  double *dst[kPermFields];
  int nf;
};
void launch_iota(hipStream_t s, int32_t *p, int64_t n);
void launch_permute_gather(hipStream_t s, const PermFields &f, const int32_t *perm,
                           const int32_t *owner_src, int32_t *owner_dst, int64_t n);
void launch_permute_scatter(hipStream_t s, const PermFields &f, const int32_t *owner,
                            int64_t n);

// k_verlet.hip
void launch_kick(hipStream_t s, double *vx, double *vy, double *vz, const double *fx,
                 const double *fy, const double *fz, int64_t n, double c);
void launch_kick_kick_drift(hipStream_t s, double *x, double *y, double *z, double *vx,
                            double *vy, double *vz, const double *fx, const double *fy,
                            const double *fz, int64_t n, double c, double dt, const double L[3]);
void launch_kick_drift(hipStream_t s, double *x, double *y, double *z, double *vx, double *vy,
                       double *vz, const double *fx, const double *fy, const double *fz,
                       int64_t n, double c, double dt, const double L[3]);
// the same as launch_kick_kick_drift, and the next detection's density
// counts of the new positions (counts zeroed beforehand)
void launch_kick_kick_drift_bin(hipStream_t s, double *x, double *y, double *z, double *vx,
                                double *vy, double *vz, const double *fx, const double *fy,
                                const double *fz, int64_t n, double c, double dt,
                                const double L[3], const int32_t nv[3], const double sc[3],
                                uint32_t *counts, uint32_t *status);
void launch_kinetic(hipStream_t s, const double *vx, const double *vy, const double *vz,
                    int64_t n, double mass, double *partials, int64_t blocks, double *out);
int64_t kinetic_blocks(int64_t n);

}  // namespace dcm
