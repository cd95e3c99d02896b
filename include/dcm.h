/*
 * dcm.h -- C ABI of the MI355X (gfx950) dynamic cutoff method library.
 *
 * The library runs the per-step hot path of the dynamic cutoff method (DCM)
 * of Springer, Ismail and Bientinesi, "A Scalable, Linear-Time Dynamic
 * Cutoff Algorithm for Molecular Dynamics":
 *
 *   interface detection on a density grid      (Section 2.1, Fig. 4, Eq. 4)
 *   cutoff-limited fast-sweeping distances     (Section 2.2, Algorithm 2.1)
 *   per-particle cutoffs from the distances    (Section 2.2)
 *   linked-cell binning with small cells       (Section 2.3, Algorithm 2.2)
 *   Verlet lists with a skin, reused over steps (Section 2.3, Algorithm 2.2)
 *   dynamic-cutoff Lennard-Jones forces        (Section 2.4, Algorithm 2.3, Eqs. 2-3),
 *     optionally with Newton's third law       (Section 2.4)
 *   many independent systems in one pass       (Section 2.4, dynamic scheduling)
 *   velocity Verlet integration                (Section 2, Fig. 3 box 5)
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Array arguments are DEVICE pointers owned by the caller, contiguous,
 *   structure-of-arrays, in the caller's particle order (outputs too: the
 *   library undoes its internal spatial ordering).  Positions are in the
 *   periodic box [0, L_a); inputs outside it are wrapped on the fly.
 * - Every call is asynchronous on the context's HIP stream.  Scalar outputs
 *   (energies, virials, counters) are device scalars.  No call synchronises
 *   the stream except dcm_sync_status, dcm_create, dcm_destroy,
 *   dcm_build_list and dcm_update_list (they read a size or a verdict back),
 *   dcm_forces_batched when it tunes the cell edge of a new batch,
 *   dcm_build_cells with cell_edge < 0 and dcm_step when they tune the cell
 *   edge of a new system shape, and dcm_build_cells (and dcm_step through it)
 *   the first time it meets a cell geometry, when it reads its ghost-image
 *   count back to size the image buffer; a later build of the same geometry
 *   waits only for the previous build's count.
 * - Scratch memory (grid buffers, cells, sorted copies, partial sums) is owned
 *   by the context and grown on demand; growing it allocates device memory,
 *   so call each entry point once with its largest sizes before capturing it
 *   in a HIP graph.
 * - Return value: DCM_OK, or an error detected on the host (bad arguments,
 *   HIP launch failure) -- then nothing was enqueued.  Conditions only the
 *   device can see (non-finite input or output, a distance sweep that did not
 *   converge, a single-phase density field) raise a sticky device flag that
 *   dcm_sync_status reports and clears.
 * - A context is not thread-safe; separate contexts are independent.
 */
#ifndef DCM_H
#define DCM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t dcm_status;
#define DCM_OK 0
#define DCM_ERR_INVALID 1       /* null pointer, negative size, non-positive length ... */
#define DCM_ERR_RANGE 2         /* rc_max >= L_a/2 (breaks the minimum image), size limits */
#define DCM_ERR_NOT_CONVERGED 3 /* distance sweep hit its wave limit */
#define DCM_ERR_DEGENERATE 4    /* the density field holds a single phase */
#define DCM_ERR_NONFINITE 5     /* NaN/Inf position or force */
#define DCM_ERR_HIP 6           /* HIP runtime error */
#define DCM_ERR_NOMEM 7         /* device allocation failed */

typedef struct dcm_ctx dcm_ctx;

/* Orthorhombic periodic box, edges L[0..2] > 0 (Section 2: the domain
 * L = L_x x L_y x L_z). */
typedef struct { double L[3]; } dcm_box;

/* Lennard-Jones 12-6 parameters, truncated and unshifted (Eq. 3). */
typedef struct { double epsilon, sigma; } dcm_lj;

/* Cutoff as a function of the particle-interface distance delta
 * (Section 2.2): rc = rc_max - (rc_max - rc_min) * min(delta/ramp, 1), i.e.
 * rc_max at the interface and in the low-density phase, rc_min at distance
 * >= ramp inside the high-density phase.  Requires 0 < rc_min <= rc_max,
 * ramp > 0. */
typedef struct { double rc_min, rc_max, ramp; } dcm_rule;

/* Density grid (Section 2.1, footnote 2): n[a] voxels of edge h[a] = L_a/n[a]
 * along each axis; voxel v = (k*n[1] + j)*n[0] + i. */
typedef struct { int32_t n[3]; double h[3]; } dcm_grid;

/* Arithmetic of the pair kernel.
 * DCM_FP64: all FP64.
 * DCM_FP32_MIXED: the Lennard-Jones terms in FP32, per-particle force sums
 * and the global energy/virial in FP64.  Under DCM_PAIR_OWN with cells at
 * most 2 sigma wide, separations and r^2 are FP32 too, from 16-byte
 * cell-relative records; a pair whose FP32 r^2 lies within a proven error
 * band of rc^2 is decided in FP64, so the pairs included are exactly those
 * of DCM_FP64.  Otherwise the separations and r^2 are FP64.  Close pairs
 * (r < 1.1 sigma), whose large forces would carry most of the FP32 rounding,
 * are evaluated in FP64 throughout. */
enum { DCM_FP64 = 0, DCM_FP32_MIXED = 1 };

/* Which pairs interact.
 * DCM_PAIR_OWN (Algorithm 2.3): j acts on i iff r_ij < rc_i; Newton's third
 * law is not applied (Section 2.4), so sum_i F_i need not vanish.
 * DCM_PAIR_MAX: j and i interact iff r_ij <= max(rc_i, rc_j) (symmetric).
 * DCM_PAIR_MAX_N3: the pairs of DCM_PAIR_MAX, each evaluated once with
 * Newton's third law (Section 2.4 and its footnotes on the trade-off): the
 * endpoint with the larger cutoff (ties: the one sorted first) searches its
 * own cutoff and adds the partner's reaction with atomics.  Results equal
 * DCM_PAIR_MAX's up to FP64 summation order; the forces are not bitwise
 * reproducible (atomic order), energy, virial and counts are.  dcm_forces
 * and dcm_step only. */
enum { DCM_PAIR_OWN = 0, DCM_PAIR_MAX = 1, DCM_PAIR_MAX_N3 = 2 };

/* Optional outputs of dcm_forces. */
enum { DCM_EV_ENERGY = 1, DCM_EV_VIRIAL = 2, DCM_EV_COUNTS = 4 };

/* ---------------------------------------------------------------- context */

/* Create a context bound to `hip_stream` (a hipStream_t; NULL = the default
 * stream) on the current device.  *out receives the context. */
dcm_status dcm_create(dcm_ctx **out, void *hip_stream);

/* Synchronise and free the context and all of its scratch memory. */
dcm_status dcm_destroy(dcm_ctx *ctx);

/* Rebind the context to another stream of the same device. */
dcm_status dcm_set_stream(dcm_ctx *ctx, void *hip_stream);

/* Synchronise the stream, then return (and clear) the sticky device status:
 * DCM_ERR_NONFINITE, DCM_ERR_NOT_CONVERGED, DCM_ERR_RANGE or
 * DCM_ERR_DEGENERATE in that priority order, else DCM_OK. */
dcm_status dcm_sync_status(dcm_ctx *ctx);

/* Text of the last error raised on this context ("" if none).  The string is
 * owned by the context and valid until the next call on it. */
const char *dcm_last_error(const dcm_ctx *ctx);

/* Host helper: grid with n[a] = max(1, round(L_a/h)) and h[a] = L_a/n[a]
 * (the voxel edge h is chosen once per run, Section 2.1 footnote 2). */
dcm_status dcm_make_grid(dcm_box box, double h, dcm_grid *out);

/* Host helper: the distance r_c^grid up to which dcm_sweep_distance should
 * propagate (Section 2.2, Algorithm 2.1 and its footnote on r_c^grid): the
 * cutoff ramp plus three of the largest voxel edges, rule.ramp + 3 max_a
 * grid.h[a].  Beyond `ramp` every particle gets rc_min whatever its distance,
 * and the discrete distance changes by at most one voxel edge per face step,
 * so capping the field there leaves every cutoff unchanged.  *out receives
 * it; DCM_ERR_INVALID for a null out, a non-positive or non-finite ramp or
 * voxel edge. */
dcm_status dcm_rc_grid(dcm_rule rule, dcm_grid grid, double *out);

/* ------------------------------------------------------------- hot path */

/* Interface detection (Section 2.1, Fig. 4, Eq. 4).
 * Bins the n particles (x, y, z) into the grid (counts, optional, uint32
 * [N_v]), takes each voxel's gray value as the particle count of its periodic
 * 3x3x3 window, splits the volume into high (1) and low (0) density phases
 * and regularises the split, then marks interface voxels: high-density voxels
 * with a low-density face neighbour.
 *   split <= 0: the threshold minimises the two-phase piecewise-constant
 *               energy with no length term (the 2-means split of the gray
 *               values); a density contrast below 2 flags DCM_ERR_DEGENERATE
 *               and classifies the whole volume as high density.
 *   split  > 0: fixed threshold, phase 1 iff gray value >= split.
 * Regularisation: synchronous 27-neighbour majority vote (>= 14 of 27),
 * repeated to a fixed point or a 2-cycle, at most 16 passes.
 * seg (uint8 [N_v], S of Eq. 4) and iface (uint8 [N_v]) are required;
 * threshold_out (int32 device scalar) is optional.
 * Limits: N_v < 2^31; gray values must stay below 4096 (else DCM_ERR_RANGE
 * via dcm_sync_status). */
dcm_status dcm_detect_interface(dcm_ctx *ctx, const double *x, const double *y,
                                const double *z, int64_t n, dcm_box box, dcm_grid grid,
                                double split, uint32_t *counts, uint8_t *seg,
                                uint8_t *iface, int32_t *threshold_out);

/* Segmentation options of dcm_detect_interface_opts (Section 2.1, Eq. 4). */
typedef struct {
  double split;        /* as in dcm_detect_interface */
  double nu;           /* < 0: majority-vote regularisation, as in dcm_detect_interface;
                          >= 0: length term of weight nu (needs split <= 0) */
  int64_t min_volume;  /* > 0: bubble filter with this volume in voxels; 0: none */
} dcm_detect_opts;

/* Interface detection with the length term of the two-phase piecewise-
 * constant Mumford-Shah energy and the bubble filter (Section 2.1).
 * With nu >= 0 the split is regularised by synchronous iterated conditional
 * modes on sum_v (g_v - c_{s_v})^2 + nu * (pairs of periodic 26-neighbours in
 * different phases), the phase means c0, c1 of the two-phase split held
 * fixed: a voxel takes phase 1 if ((g - c1)^2 - (g - c0)^2) + nu (26 - 2 n1)
 * < 0, phase 0 if > 0, and keeps its phase if = 0 (n1: its neighbours in
 * phase 1); passes stop as the majority vote's do (fixed point, 2-cycle, 16
 * passes).  nu = 0 leaves the split as it is; a single-phase volume is not
 * regularised.  With min_volume > 0, every periodic 6-connected component of
 * either phase with fewer than min_volume voxels then takes the other phase
 * (all on the same map), and the interface is marked on the result.
 * Arguments and outputs as in dcm_detect_interface; opts is a host pointer.
 * Errors: DCM_ERR_INVALID for a null opts, a non-finite nu, nu >= 0 with
 * split > 0, or min_volume < 0 or >= 2^31. */
dcm_status dcm_detect_interface_opts(dcm_ctx *ctx, const double *x, const double *y,
                                     const double *z, int64_t n, dcm_box box, dcm_grid grid,
                                     const dcm_detect_opts *opts, uint32_t *counts,
                                     uint8_t *seg, uint8_t *iface, int32_t *threshold_out);

/* Interface detection that allocates nothing, for callers that cannot
 * allocate device memory: code being captured into a HIP graph, tight serving
 * loops, harnesses that forbid allocation.  Arguments, outputs and results
 * are those of dcm_detect_interface (bit for bit).  Its scratch -- the
 * gray-value histogram copies (512 KiB), the gray values (4 N_v bytes), two
 * bit-packed phase maps (N_y N_z ceil(N_x/32) words each) and, when counts is
 * NULL, the voxel counts (4 N_v bytes) -- lives in one static 32 MiB device
 * array per GPU, which the library holds until the process ends (its address
 * is looked up when the first context is created on that GPU).  That bounds
 * the grid: about 7.7 M voxels with a caller counts array, 4.0 M without
 * (fewer when N_x is far below a multiple of 32); larger grids return
 * DCM_ERR_RANGE before anything is enqueued.  Every call
 * on a GPU shares that one array and leaves its contents behind (the call
 * clears what must start at zero itself): calls that overlap on one GPU --
 * from other streams, contexts or threads -- race and must be serialised by
 * the caller. */
dcm_status dcm_detect_interface_noalloc(dcm_ctx *ctx, const double *x, const double *y,
                                        const double *z, int64_t n, dcm_box box, dcm_grid grid,
                                        double split, uint32_t *counts, uint8_t *seg,
                                        uint8_t *iface, int32_t *threshold_out);

/* Box-interface distances (Section 2.2, Algorithm 2.1).  Interface and
 * low-density voxels start at 0, the rest at +infinity; the first-order
 * Godunov upwind update of |grad d| = 1 is applied to every voxel in
 * synchronous waves, accepting only values <= rc_grid, until a wave changes
 * nothing (at most max_waves waves, else DCM_ERR_NOT_CONVERGED via
 * dcm_sync_status).  dist (double [N_v]) receives min(D, rc_grid);
 * waves_out (int32 device scalar, optional) the number of waves run. */
dcm_status dcm_sweep_distance(dcm_ctx *ctx, const uint8_t *seg, const uint8_t *iface,
                              dcm_grid grid, double rc_grid, int32_t max_waves,
                              double *dist, int32_t *waves_out);

/* Cutoff assignment (Section 2.2): delta_i = periodic trilinear interpolation
 * of the voxel-centred distances at x_i; rc_i from the rule.  delta (double
 * [n]) is optional, rc (double [n]) required. */
dcm_status dcm_assign_cutoffs(dcm_ctx *ctx, const double *x, const double *y,
                              const double *z, int64_t n, dcm_box box, dcm_grid grid,
                              const double *dist, dcm_rule rule, double *delta,
                              double *rc);

/* Linked cells (Section 2.3).  Cells of edge L_a/n_a with
 * n_a = floor(L_a/cell_edge), cell c = (c_z*n_y + c_y)*n_x + c_x.
 * cell_edge == 0: a default of about two particles per cell at the mean
 * density.  cell_edge < 0: a measured choice among 1/3, 0.4, 1/2, 0.6, 0.7
 * and 0.8 of the smallest cutoff (for DCM_FP32_MIXED at most the widest edge
 * whose cells stay within 2, the widest cell its compact records serve at
 * sigma = 1): the first such call for a system
 * shape (device, n, box, smallest cutoff, rc_bound, prec) times a cell build
 * and a force pass (own rule, eps = sigma = 1) at each and synchronises; the
 * choice is kept for the rest of the process.
 * Particles are sorted by cell and, within a cell, by x (positions quantised
 * to 2^-20 of the cell; ties in ascending caller index) into context-owned
 * copies of (x, y, z, rc) that dcm_forces reads, together
 * with periodic ghost images of the cells within rc_bound of the box faces.
 * rc_bound is an upper bound on every cutoff (<= 0: half the shortest box
 * edge); larger cutoffs are clamped to it and flag DCM_ERR_RANGE, and so do
 * cutoffs >= half a box edge (minimum image).  cell_of (int32 [n]) and
 * cell_start (int32 [n_cells + 1], exclusive prefix of per-cell counts) are
 * optional copies for the caller; dcm_cell_dims gives n_cells.  prec selects
 * the layout of the sorted copy for the later dcm_forces call.  The positions
 * and cutoffs are read during this call only.  n must be below 2^24. */
dcm_status dcm_build_cells(dcm_ctx *ctx, const double *x, const double *y, const double *z,
                           const double *rc, int64_t n, dcm_box box, double cell_edge,
                           double rc_bound, int prec, int32_t *cell_of, int32_t *cell_start);

/* Host query: cell counts per axis and cell edge lengths of the last
 * dcm_build_cells call on this context. */
dcm_status dcm_cell_dims(const dcm_ctx *ctx, int32_t n_cells[3], double cell_len[3]);

/* Dynamic-cutoff Lennard-Jones forces (Algorithm 2.3, Eqs. 2-3) on the cells
 * of the last dcm_build_cells call.  For every i, F_i sums
 * f_ij = 24 eps s6 (2 s6 - 1) / r^2 * (x_i - x_j), s6 = (sigma/r)^6, over the
 * interacting j (pair_rule), with minimum-image separations.
 * fx, fy, fz (double [n], caller order) are required.  With ev_flags:
 *   DCM_EV_ENERGY: *energy = sum over interacting ordered pairs of U/2,
 *                  U = 4 eps s6 (s6 - 1);
 *   DCM_EV_VIRIAL: virial[6] = xx yy zz xy xz yz of sum of d_a f_b / 2;
 *   DCM_EV_COUNTS: nnbr[i] = number of j acting on i (int32 [n]), *npairs =
 *                  number of interacting ordered pairs (uint64).
 * Pointers for unrequested outputs may be NULL.  energy/virial/npairs are
 * device scalars.  The energy and virial sums are deterministic; so are the
 * forces, except under DCM_PAIR_MAX_N3 (atomic reactions).
 * Errors: DCM_ERR_INVALID before a cell build, after dcm_update_list, or for
 * an unknown rule or precision. */
dcm_status dcm_forces(dcm_ctx *ctx, dcm_lj lj, int pair_rule, int prec, int ev_flags,
                      double *fx, double *fy, double *fz, double *energy, double *virial,
                      int32_t *nnbr, uint64_t *npairs);

/* Work of the cell walk (the small-bin traversal of Section 2.3) in the last
 * dcm_forces call on this context made with DCM_EV_COUNTS: stats[0] = the
 * candidate pairs it tested (each particle's trimmed rows, its own slot
 * excluded), stats[1] = the cell rows it visited, both summed over the
 * particles (host uint64 [2]).  Candidates per interacting pair, stats[0] /
 * npairs, is the overhead of the search over the pairs the rule accepts.
 * Synchronises the context's stream.
 * Errors: DCM_ERR_INVALID if the last dcm_forces call had no DCM_EV_COUNTS. */
dcm_status dcm_walk_stats(dcm_ctx *ctx, uint64_t stats[2]);

/* Verlet neighbour list with a skin (Section 2.3, Algorithm 2.2) on the cells
 * of the last dcm_build_cells: particle i's list holds every other particle or
 * periodic image j with r_ij^2 < R_i^2, R_i = min(r_c(i), rc_bound) + skin,
 * in the order in which dcm_forces visits its candidates.  skin in
 * [0, smallest cell edge].  The list belongs to that cell build; a new build
 * discards it.  Synchronises the context's stream (the list's size is read
 * back to size its buffer).
 * Errors: DCM_ERR_INVALID before a cell build, after dcm_update_list, or for
 * a skin out of range. */
dcm_status dcm_build_list(dcm_ctx *ctx, double skin);

/* Reuse of the list over steps (Section 2.3): new positions x, y, z and
 * cutoffs rc (double [n], caller order, n as in the cell build) replace those
 * of the build; dcm_forces_list then evaluates them.  Each particle moves by
 * the minimum image of its displacement from its position at the list build,
 * so wrapped and unwrapped coordinates give the same result.
 * *valid (host int32, required) is set to 1 when the list still holds every
 * pair that interacts now: with D the largest displacement since the list
 * build and S the smallest R_i - r_c(i) (new cutoffs), when S - 2 D exceeds a
 * rounding margin of 1e-12 (rc_bound + skin), or D = 0 and S >= 0.
 * Otherwise 0: build the cells and the list again.  max_disp and min_slack
 * (host doubles, optional) receive D and S.  Cutoffs are clamped to
 * [0, rc_bound] and flag DCM_ERR_RANGE at dcm_sync_status as in the cell
 * build.  After this call dcm_forces (the cell walk) and dcm_build_list
 * refuse until the cells are built again.  Synchronises the stream.
 * Errors: DCM_ERR_INVALID without a list for the current cell build, for
 * another n, or for a null pointer. */
dcm_status dcm_update_list(dcm_ctx *ctx, const double *x, const double *y, const double *z,
                           const double *rc, int64_t n, double *max_disp, double *min_slack,
                           int32_t *valid);

/* Own-cutoff forces (Algorithm 2.3) over the list of the current cell build:
 * arguments and results as dcm_forces with DCM_PAIR_OWN.  Until an update,
 * the pairs and their summation order are those of dcm_forces, so both give
 * identical results.
 * Errors: DCM_ERR_INVALID without a list for the current cell build. */
dcm_status dcm_forces_list(dcm_ctx *ctx, dcm_lj lj, int prec, int ev_flags, double *fx,
                           double *fy, double *fz, double *energy, double *virial, int32_t *nnbr,
                           uint64_t *npairs);

/* Velocity-Verlet MD with the whole DCM pipeline (Fig. 3).
 * nsteps == 0: compute forces at the current positions (detection, distances,
 * cutoffs, cells, forces) into fx, fy, fz.
 * nsteps  > 0: fx, fy, fz must hold the forces at the current positions; each
 * step does v += dt/(2m) F; x += dt v (wrapped); re-detect the interface and
 * re-sweep the distances when (step0 + s + 1) % redetect_every == 0 or no
 * distance field exists yet; re-assign cutoffs and rebuild cells (every
 * step); recompute F; v += dt/(2m) F.  The cell edge is a measured choice
 * among 1/3, 0.4, 1/2, 0.6, 0.7 and 0.8 of rc_min (for DCM_FP32_MIXED at most
 * the widest edge whose cells stay within 2 sigma, so that the compact
 * records apply): the first call for a system shape
 * (device, n, box, rc_min, rc_max, prec, pair_rule, sigma) in the process
 * times a cell build and a force pass at each, synchronising once; later
 * calls and contexts reuse the choice (dcm_cell_dims reports it).
 * energy_series (double [2*nsteps], optional): potential and kinetic energy
 * after each step.  delta/rc (double [n], optional) receive the last
 * distances and cutoffs.  The context keeps the last distance field between
 * calls; a call with nsteps > 0 reuses it until its first re-detection only
 * when n, box, grid and rc_grid equal those it was computed for (continue a
 * run with step0 = the steps done so far).
 * On a step with re-detection, for DCM_PAIR_OWN and a cell edge already
 * chosen, the cell build runs on a second stream that the context creates
 * (non-blocking, default priority) beside the distance sweep, and the
 * context's stream waits for it before the cutoffs are assigned; every
 * launch of the call is complete once the context's stream is.  A stream
 * being captured into a graph keeps the build on the context's stream. */
dcm_status dcm_step(dcm_ctx *ctx, double *x, double *y, double *z, double *vx, double *vy,
                    double *vz, double *fx, double *fy, double *fz, int64_t n, double mass,
                    dcm_box box, dcm_lj lj, dcm_rule rule, dcm_grid grid, double rc_grid,
                    int pair_rule, int prec, double dt, int32_t nsteps,
                    int32_t redetect_every, int64_t step0, double *energy_series,
                    double *delta, double *rc);

/* ---------------------------------------------------------- batched form */

/* One system of a batch: the caller's device arrays and periodic box. */
typedef struct {
  const double *x, *y, *z, *rc; /* double [n], caller order; required when n > 0 */
  double *fx, *fy, *fz;         /* double [n], caller order; required when n > 0 */
  int32_t *nnbr;                /* int32 [n]; written with DCM_EV_COUNTS if not NULL */
  double *energy;               /* device scalar; required with DCM_EV_ENERGY */
  double *virial;               /* device double [6]; required with DCM_EV_VIRIAL */
  uint64_t *npairs;             /* device scalar; written with DCM_EV_COUNTS if not NULL */
  int64_t n;                    /* particles, >= 0 */
  dcm_box box;
  double cell_edge;             /* as in dcm_build_cells; <= 0: picked by the tuner */
  double rc_bound;              /* as in dcm_build_cells (<= 0: half the shortest edge) */
} dcm_system;

/* Linked cells and dynamic-cutoff forces (Sections 2.3-2.4, Algorithm 2.3)
 * of nsys independent systems in one pass.  For every system the outputs are
 * those of dcm_build_cells(x, y, z, rc, n, box, cell_edge, rc_bound) followed
 * by dcm_forces(lj, pair_rule, prec, ev_flags) -- bit for bit when the cell
 * edge is the same -- but all systems share one launch of each build kernel
 * and one persistent pair kernel that takes blocks of 256 particles from a
 * work queue ordered by estimated cost (largest first), or from one such
 * queue per XCD (dcm_set_batched_queues), so systems of very different size
 * and cutoff balance across the GPU (the dynamic scheduling of Section 2.4).
 * sys: host array of nsys descriptors (nsys = 0 is a no-op).  Systems whose
 * cell_edge is <= 0 share one edge chosen, together with the work-queue
 * layout and the pair kernel's row-list size, by timing a few candidates the
 * first time a batch is seen (this call synchronises the stream); the choice
 * is kept for later calls with the same descriptors.
 * use_graph != 0: the first call for a given set of descriptors and
 * parameters records the launches in a HIP graph; later identical calls
 * replay it (the arrays' contents may change between calls, their addresses
 * and sizes may not).  Work is ordered after earlier work on the context's
 * stream and before later work on it.
 * Limits: sum of n below 2^24; pair_rule DCM_PAIR_OWN or DCM_PAIR_MAX.
 * Device-detected conditions (non-finite input or force, cutoffs above
 * rc_bound) as for the single-system calls. */
dcm_status dcm_forces_batched(dcm_ctx *ctx, int32_t nsys, const dcm_system *sys, dcm_lj lj,
                              int pair_rule, int prec, int ev_flags, int use_graph);


/* Cell edge the tuner chose for the last batch (0 if none was needed). */
dcm_status dcm_batched_edge(const dcm_ctx *ctx, double *edge);

/* Work-queue layout of the batched pair kernel for later dcm_forces_batched
 * calls on this context: queues = 1, one queue with the costliest work first;
 * 8, one queue per XCD of the MI355X, each holding whole systems (balanced by
 * estimated cost, so a system's records are read through one L2), drained by
 * that XCD's workgroups before they help the others; 0 (the default), timed
 * together with the cell edge when a batch needs tuning, else 1.  The
 * results do not depend on the layout.  A change re-plans (and re-tunes) the
 * next batch.  Errors: DCM_ERR_INVALID for other values. */
dcm_status dcm_set_batched_queues(dcm_ctx *ctx, int32_t queues);

/* The work-queue layout (1 or 8) of the last batch, 0 before any. */
dcm_status dcm_batched_queues(const dcm_ctx *ctx, int32_t *queues);

/* Row-list entries per lane (14 or 16) of the FP32-mixed own-cutoff batched
 * pair kernel for the last batch, 0 before any: a batch whose cell edge is
 * tuned also times both and keeps the faster (more entries: fewer chunks per
 * particle, fewer resident workgroups); otherwise 14.  Other kernels have one
 * list size. */
dcm_status dcm_batched_row_lists(const dcm_ctx *ctx, int32_t *entries);

/* Row-list entries for later dcm_forces_batched calls on this context: 14 or
 * 16, or 0 (the default) for the tuner's choice.  A change re-tunes the next
 * batch that tunes.  Results differ between the two in the last bits of the
 * forces (the FP32 chunk sums end at other rows), not in the pair counts.
 * Errors: DCM_ERR_INVALID for other values. */
dcm_status dcm_set_batched_row_lists(dcm_ctx *ctx, int32_t entries);

/* ------------------------------------------------------------ profiling */

/* Record HIP events around every launch of the named kernel family
 * ("pair", "cells", "detect", "sweep", "cutoffs", "verlet"; "batch_cells",
 * "batch_pair" for the batched form, "batch_graph" for a replayed graph)
 * when enabled. */
dcm_status dcm_set_profiling(dcm_ctx *ctx, int enable);

/* While profiling, record events only around the launches of one kernel
 * family (family NULL or "": every family, the default), so that timing one
 * kernel adds two events per launch of it and none elsewhere.  The name is
 * copied.  Errors: DCM_ERR_INVALID for a null context. */
dcm_status dcm_set_profiling_only(dcm_ctx *ctx, const char *family);

/* Synchronise, then return the summed event time (ms) and launch count of a
 * kernel family since profiling was enabled, and reset them. */
dcm_status dcm_kernel_time(dcm_ctx *ctx, const char *family, double *total_ms,
                           int64_t *launches);

#ifdef __cplusplus
}
#endif

#endif /* DCM_H */
