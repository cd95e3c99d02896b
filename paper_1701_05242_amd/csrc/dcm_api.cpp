// Host side of the C ABI declared in include/dcm.h: argument validation,
// context-owned scratch memory, and the order in which each entry point
// enqueues its kernels on the context's stream.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <vector>

#include "dcm_internal.hpp"

using namespace dcm;

namespace dcm {

dcm_status fail(dcm_ctx *ctx, dcm_status code, const std::string &msg) {
  if (ctx) ctx->err = msg;
  return code;
}

dcm_status ensure(dcm_ctx *ctx, DevBuf &b, size_t bytes) {
  if (bytes < 256) bytes = 256;
  if (b.cap >= bytes) return DCM_OK;
  if (b.p) {
    // work queued on the context's streams may still use the old buffer:
    // its stream, dcm_step's second stream, and the stream that one was
    // forked from while it builds cells
    hipError_t e = hipStreamSynchronize(ctx->stream);
    if (e == hipSuccess && ctx->side && ctx->side != ctx->stream)
      e = hipStreamSynchronize(ctx->side);
    if (e == hipSuccess && ctx->forked_from) e = hipStreamSynchronize(ctx->forked_from);
    if (e != hipSuccess)
      return fail(ctx, DCM_ERR_HIP, "buffer growth: stream synchronisation failed");
    (void)hipFree(b.p);
    b.p = nullptr;
    b.cap = 0;
  }
  size_t sz = (bytes + 4095) & ~size_t(4095);
  hipError_t e = hipMalloc(&b.p, sz);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    b.p = nullptr;
    return fail(ctx, DCM_ERR_NOMEM,
                std::string("device allocation of ") + std::to_string(sz) + " bytes failed");
  }
  b.cap = sz;
  return DCM_OK;
}

dcm_status check_launch(dcm_ctx *ctx, const char *what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess)
    return fail(ctx, DCM_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
  return DCM_OK;
}

void timer_begin(dcm_ctx *ctx, const char *family, hipEvent_t *ev) {
  *ev = nullptr;
  if (!ctx->profile) return;
  if (!ctx->profile_only.empty() && ctx->profile_only != family) return;
  if (hipEventCreate(ev) != hipSuccess) {
    *ev = nullptr;
    return;
  }
  (void)hipEventRecord(*ev, ctx->stream);  // a failed record only loses this timing
}

void timer_end(dcm_ctx *ctx, const char *family, hipEvent_t ev) {
  if (!ev) return;
  hipEvent_t e2;
  if (hipEventCreate(&e2) != hipSuccess) return;
  (void)hipEventRecord(e2, ctx->stream);
  ctx->timers[family].pending.push_back({ev, e2});
}

dcm_status detect_check(dcm_ctx *ctx, const double *x, const double *y, const double *z,
                        int64_t n, const dcm_box &box, const dcm_grid &grid,
                        const dcm_detect_opts *opts, const uint8_t *seg, const uint8_t *iface,
                        int64_t *nvox) {
  if (!ctx) return DCM_ERR_INVALID;
  if (!opts) return fail(ctx, DCM_ERR_INVALID, "dcm_detect_interface_opts: null opts");
  const double split = opts->split, nu = opts->nu;
  if (!std::isfinite(nu)) return fail(ctx, DCM_ERR_INVALID, "nu must be finite");
  if (nu >= 0.0 && split > 0.0)
    return fail(ctx, DCM_ERR_INVALID, "a length-term weight needs the two-phase split (split <= 0)");
  if (opts->min_volume < 0 || opts->min_volume >= (int64_t(1) << 31))
    return fail(ctx, DCM_ERR_INVALID, "min_volume must be in [0, 2^31)");
  if (n < 0) return fail(ctx, DCM_ERR_INVALID, "particle count must be >= 0");
  if (n >= (int64_t(1) << 31) - 1) return fail(ctx, DCM_ERR_RANGE, "particle count >= 2^31 - 1");
  for (int a = 0; a < 3; ++a)
    if (!(std::isfinite(box.L[a]) && box.L[a] > 0.0))
      return fail(ctx, DCM_ERR_INVALID, "box lengths must be > 0");
  int64_t v = 1;
  for (int a = 0; a < 3; ++a) {
    if (grid.n[a] < 1 || !(std::isfinite(grid.h[a]) && grid.h[a] > 0.0))
      return fail(ctx, DCM_ERR_INVALID, "grid needs n >= 1 and h > 0 on every axis");
    v *= grid.n[a];
    if (v >= (int64_t(1) << 31)) return fail(ctx, DCM_ERR_RANGE, "grid has 2^31 or more voxels");
  }
  *nvox = v;
  if ((n > 0 && (!x || !y || !z)) || !seg || !iface)
    return fail(ctx, DCM_ERR_INVALID, "dcm_detect_interface: null pointer");
  if (!std::isfinite(split)) return fail(ctx, DCM_ERR_INVALID, "split must be finite");
  return DCM_OK;
}

dcm_status detect_enqueue(dcm_ctx *ctx, const double *x, const double *y, const double *z,
                          int64_t n, const dcm_box &box, const dcm_grid &grid,
                          const dcm_detect_opts &opts, const DetectScratch &sc, uint8_t *seg,
                          uint8_t *iface, int32_t *threshold_out, bool timed, bool binned) {
  const int64_t nvox = (int64_t)grid.n[0] * grid.n[1] * grid.n[2];
  const double sc3[3] = {(double)grid.n[0] / box.L[0], (double)grid.n[1] / box.L[1],
                         (double)grid.n[2] / box.L[2]};
  hipStream_t s = ctx->stream;
  hipEvent_t ev = nullptr;
  if (timed) timer_begin(ctx, "detect", &ev);
  if (!binned) {
    launch_zero2_u32(s, sc.counts, nvox, sc.hist, (int64_t)kHistCopies * kHistBins);
    launch_bin_density(s, x, y, z, n, box.L, grid.n, sc3, sc.counts, ctx->d_status);
  }
  launch_gray_hist(s, sc.counts, sc.gray, grid.n, sc.hist, ctx->d_status);
  if (opts.split <= 0.0) launch_otsu(s, sc.hist, nvox, ctx->ctl, threshold_out, ctx->d_status);
  launch_threshold(s, sc.gray, grid.n, opts.split, ctx->ctl, sc.seg_a, threshold_out);
  for (int p = 1; p <= kMajorityMaxPasses; ++p) {
    if (opts.nu < 0.0)
      launch_majority_pass(s, sc.seg_a, sc.seg_b, grid.n, p, kMajorityMaxPasses, ctx->ctl);
    else
      launch_potts_pass(s, sc.seg_a, sc.seg_b, sc.gray, grid.n, opts.nu, p, ctx->ctl);
  }
  // seg null (dcm_step): the phase maps feed the distance sweep directly
  if (seg) launch_interface(s, sc.seg_a, sc.seg_b, grid.n, ctx->ctl, seg, iface);
  if (opts.min_volume > 0)
    launch_bubble_filter(s, grid.n, opts.min_volume, seg, iface, sc.ccl_label, sc.ccl_size,
                         ctx->d_status);
  if (timed) timer_end(ctx, "detect", ev);
  return check_launch(ctx, "dcm_detect_interface");
}


}  // namespace dcm

namespace {

template <typename T>
T *ptr(const DevBuf &b) {
  return static_cast<T *>(b.p);
}

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

dcm_status check_box(dcm_ctx *ctx, const dcm_box &box) {
  for (int a = 0; a < 3; ++a)
    if (!finite_pos(box.L[a])) return fail(ctx, DCM_ERR_INVALID, "box lengths must be > 0");
  return DCM_OK;
}

dcm_status check_grid(dcm_ctx *ctx, const dcm_grid &g, int64_t *nvox) {
  int64_t v = 1;
  for (int a = 0; a < 3; ++a) {
    if (g.n[a] < 1 || !finite_pos(g.h[a]))
      return fail(ctx, DCM_ERR_INVALID, "grid needs n >= 1 and h > 0 on every axis");
    v *= g.n[a];
    if (v >= (int64_t(1) << 31)) return fail(ctx, DCM_ERR_RANGE, "grid has 2^31 or more voxels");
  }
  *nvox = v;
  return DCM_OK;
}

dcm_status check_n(dcm_ctx *ctx, int64_t n) {
  if (n < 0) return fail(ctx, DCM_ERR_INVALID, "particle count must be >= 0");
  if (n >= (int64_t(1) << 31) - 1) return fail(ctx, DCM_ERR_RANGE, "particle count >= 2^31 - 1");
  return DCM_OK;
}

#define DCM_TRY(expr)                  \
  do {                                 \
    dcm_status st_ = (expr);           \
    if (st_ != DCM_OK) return st_;     \
  } while (0)

// ---- cell-edge tuner (Section 2.3, small cells): the edge of the linked
// cells is chosen among fractions of a reference cutoff r_ref (the smallest
// cutoff) by timing a cell build plus a force pass at each, and remembered
// for the rest of the process per system shape (device, particle count, box,
// cutoff range, precision, rule, sigma), so that every context of a process
// makes the same choice for the same system.
std::mutex g_edge_mu;
std::map<std::vector<double>, double> g_edge_cache;

// f r_ref for f = 1/3, 0.4, 1/2, 0.6, 0.7, 0.8, each at most the widest
// edge whose cells (of length L_a / floor(L_a / edge) >= edge) stay within
// cap (the widest cell the compact FP32 records serve, for FP32-mixed
// forces); repeats dropped
std::vector<double> edge_candidates(double r_ref, double cap, const double L[3]) {
  double top = cap;
  if (std::isfinite(cap))
    for (int a = 0; a < 3; ++a) top = std::min(top, L[a] / std::ceil(L[a] / cap));
  std::vector<double> c;
  for (double f : {1.0 / 3.0, 0.4, 0.5, 0.6, 0.7, 0.8}) {
    const double e = std::min(f * r_ref, top);
    if (c.empty() || std::fabs(e - c.back()) > 1e-12 * e) c.push_back(e);
  }
  return c;
}

bool edge_cached(const std::vector<double> &key, double *edge) {
  std::lock_guard<std::mutex> lock(g_edge_mu);
  auto it = g_edge_cache.find(key);
  if (it == g_edge_cache.end()) return false;
  *edge = it->second;
  return true;
}

// Times run(edge) (a cell build plus a force pass, enqueued on the context's
// stream) once untimed and twice timed per candidate; synchronises.
dcm_status tune_edge(dcm_ctx *ctx, const std::vector<double> &key,
                     const std::vector<double> &cands,
                     const std::function<dcm_status(double)> &run, double *best) {
  if (edge_cached(key, best)) return DCM_OK;
  double pick = cands.front();
  if (cands.size() > 1) {
    const bool prof = ctx->profile;
    ctx->profile = false;  // the trials are not part of any kernel family's time
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
      (void)hipGetLastError();
      if (e0) (void)hipEventDestroy(e0);
      ctx->profile = prof;
      return fail(ctx, DCM_ERR_HIP, "cell-edge tuner: event creation failed");
    }
    float best_ms = INFINITY;
    dcm_status st = DCM_OK;
    for (double e : cands) {
      if ((st = run(e)) != DCM_OK) break;  // first run: buffers grow, caches warm
      const hipError_t r0 = hipEventRecord(e0, ctx->stream);
      if ((st = run(e)) != DCM_OK || (st = run(e)) != DCM_OK) break;
      const hipError_t r1 = hipEventRecord(e1, ctx->stream);
      float ms = 0.0f;
      if (r0 != hipSuccess || r1 != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
          hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
        st = fail(ctx, DCM_ERR_HIP, "cell-edge tuner: timing failed");
        break;
      }
      if (ms < best_ms) {
        best_ms = ms;
        pick = e;
      }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    ctx->profile = prof;
    if (st != DCM_OK) return st;
  }
  std::lock_guard<std::mutex> lock(g_edge_mu);
  auto it = g_edge_cache.emplace(key, pick).first;  // a concurrent tuning may have won
  *best = it->second;
  return DCM_OK;
}

}  // namespace

namespace dcm {
dcm_status detect_scratch(dcm_ctx *ctx, const dcm_grid &grid, int64_t nvox,
                          const dcm_detect_opts &o, uint32_t *counts, DetectScratch *out) {
  const dcm_detect_opts *opts = &o;
  DetectScratch &sc = *out;
  DCM_TRY(ensure(ctx, ctx->gray, nvox * sizeof(uint32_t)));
  DCM_TRY(ensure(ctx, ctx->hist, (size_t)kHistCopies * kHistBins * sizeof(uint32_t)));
  DCM_TRY(ensure(ctx, ctx->seg_a, phase_bits_words(grid.n) * sizeof(uint32_t)));
  DCM_TRY(ensure(ctx, ctx->seg_b, phase_bits_words(grid.n) * sizeof(uint32_t)));
  if (opts->min_volume > 0) {
    DCM_TRY(ensure(ctx, ctx->ccl_label, nvox * sizeof(int32_t)));
    DCM_TRY(ensure(ctx, ctx->ccl_size, nvox * sizeof(int32_t)));
    sc.ccl_label = ptr<int32_t>(ctx->ccl_label);
    sc.ccl_size = ptr<int32_t>(ctx->ccl_size);
  }
  if (!counts) {
    DCM_TRY(ensure(ctx, ctx->counts, nvox * sizeof(uint32_t)));
    counts = ptr<uint32_t>(ctx->counts);
  }
  sc.counts = counts;
  sc.gray = ptr<uint32_t>(ctx->gray);
  sc.hist = ptr<uint32_t>(ctx->hist);
  sc.seg_a = ptr<uint32_t>(ctx->seg_a);
  sc.seg_b = ptr<uint32_t>(ctx->seg_b);
  return DCM_OK;
}
}  // namespace dcm

extern "C" {

dcm_status dcm_create(dcm_ctx **out, void *hip_stream) {
  if (!out) return DCM_ERR_INVALID;
  *out = nullptr;
  dcm_ctx *ctx = new (std::nothrow) dcm_ctx();
  if (!ctx) return DCM_ERR_NOMEM;
  ctx->stream = static_cast<hipStream_t>(hip_stream);
  if (hipGetDevice(&ctx->device) != hipSuccess) {
    (void)hipGetLastError();
    delete ctx;
    return DCM_ERR_HIP;
  }
  void *p = nullptr;
  if (hipMalloc(&p, 256) != hipSuccess) {
    (void)hipGetLastError();
    delete ctx;
    return DCM_ERR_NOMEM;
  }
  ctx->d_status = static_cast<uint32_t *>(p);
  if (hipMalloc(&p, sizeof(Ctl)) != hipSuccess) {
    (void)hipGetLastError();
    (void)hipFree(ctx->d_status);
    delete ctx;
    return DCM_ERR_NOMEM;
  }
  ctx->ctl = static_cast<Ctl *>(p);
  if (hipHostMalloc(&p, 64, hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    (void)hipFree(ctx->d_status);
    (void)hipFree(ctx->ctl);
    delete ctx;
    return DCM_ERR_NOMEM;
  }
  ctx->h_status = static_cast<uint32_t *>(p);
  if (hipEventCreateWithFlags(&ctx->ext_event, hipEventDisableTiming) != hipSuccess) {
    (void)hipGetLastError();
    (void)hipFree(ctx->d_status);
    (void)hipFree(ctx->ctl);
    (void)hipHostFree(ctx->h_status);
    delete ctx;
    return DCM_ERR_HIP;
  }
  ctx->h_ext_total = reinterpret_cast<int32_t *>(static_cast<char *>(p) + 8);
  *ctx->h_ext_total = 0;
  ctx->h_list_total = reinterpret_cast<int32_t *>(static_cast<char *>(p) + 16);
  ctx->h_list_verdict = reinterpret_cast<double *>(static_cast<char *>(p) + 24);
  launch_clear_status(ctx->stream, ctx->d_status);
  launch_reset_ctl(ctx->stream, ctx->ctl);
  dcm_status st = check_launch(ctx, "dcm_create");
  // the device address of this GPU's no-allocation scratch array, once per
  // device (dcm_noalloc.hip)
  if (st == DCM_OK) st = noalloc_scratch_setup(ctx->device, &ctx->err);
  if (st == DCM_OK && hipStreamSynchronize(ctx->stream) != hipSuccess) st = DCM_ERR_HIP;
  if (st != DCM_OK) {
    (void)hipEventDestroy(ctx->ext_event);
    (void)hipFree(ctx->d_status);
    (void)hipFree(ctx->ctl);
    (void)hipHostFree(ctx->h_status);
    delete ctx;
    return st;
  }
  *out = ctx;
  return DCM_OK;
}

dcm_status dcm_destroy(dcm_ctx *ctx) {
  if (!ctx) return DCM_ERR_INVALID;
  (void)hipStreamSynchronize(ctx->stream);  // freed below whatever its status
  if (ctx->side) {
    (void)hipStreamSynchronize(ctx->side);
    (void)hipStreamDestroy(ctx->side);
  }
  if (ctx->fork_ev) (void)hipEventDestroy(ctx->fork_ev);
  if (ctx->join_ev) (void)hipEventDestroy(ctx->join_ev);
  // the context's device buffers go with it
  batch_free(ctx);
  for (auto &kv : ctx->timers)
    for (auto &pr : kv.second.pending) {
      (void)hipEventDestroy(pr.first);
      (void)hipEventDestroy(pr.second);
    }
  (void)hipEventDestroy(ctx->ext_event);
  (void)hipFree(ctx->d_status);
  (void)hipFree(ctx->ctl);
  (void)hipHostFree(ctx->h_status);
  delete ctx;
  return DCM_OK;
}

dcm_status dcm_set_stream(dcm_ctx *ctx, void *hip_stream) {
  if (!ctx) return DCM_ERR_INVALID;
  ctx->stream = static_cast<hipStream_t>(hip_stream);
  return DCM_OK;
}

dcm_status dcm_sync_status(dcm_ctx *ctx) {
  if (!ctx) return DCM_ERR_INVALID;
  if (hipStreamSynchronize(ctx->stream) != hipSuccess)
    return fail(ctx, DCM_ERR_HIP, std::string("stream error: ") +
                                      hipGetErrorString(hipGetLastError()));
  if (hipMemcpy(ctx->h_status, ctx->d_status, sizeof(uint32_t), hipMemcpyDeviceToHost) !=
      hipSuccess)
    return fail(ctx, DCM_ERR_HIP, "status read failed");
  uint32_t st = *ctx->h_status;
  launch_clear_status(ctx->stream, ctx->d_status);
  if (hipStreamSynchronize(ctx->stream) != hipSuccess) return DCM_ERR_HIP;
  if (st & (ST_NONFINITE_POS | ST_NONFINITE_FORCE))
    return fail(ctx, DCM_ERR_NONFINITE, "non-finite position or force");
  if (st & ST_NOT_CONVERGED)
    return fail(ctx, DCM_ERR_NOT_CONVERGED, "distance sweep reached its wave limit");
  if (st & ST_GHOST_OVERFLOW)
    return fail(ctx, DCM_ERR_RANGE, "ghost images exceeded their buffer; build the cells again");
  if (st & (ST_HIST_RANGE | ST_RC_RANGE))
    return fail(ctx, DCM_ERR_RANGE, "gray value >= 4096 or cutoff outside [0, rc_bound]");
  if (st & ST_DEGENERATE)
    return fail(ctx, DCM_ERR_DEGENERATE, "density field holds a single phase");
  return DCM_OK;
}

const char *dcm_last_error(const dcm_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

dcm_status dcm_make_grid(dcm_box box, double h, dcm_grid *out) {
  if (!out || !finite_pos(h)) return DCM_ERR_INVALID;
  for (int a = 0; a < 3; ++a)
    if (!finite_pos(box.L[a])) return DCM_ERR_INVALID;
  for (int a = 0; a < 3; ++a) {
    double r = std::round(box.L[a] / h);
    if (r > 2147483647.0) return DCM_ERR_RANGE;
    int32_t k = (int32_t)r;
    if (k < 1) k = 1;
    out->n[a] = k;
    out->h[a] = box.L[a] / (double)k;
  }
  return DCM_OK;
}

dcm_status dcm_rc_grid(dcm_rule rule, dcm_grid grid, double *out) {
  if (!out || !finite_pos(rule.ramp)) return DCM_ERR_INVALID;
  double hmax = 0.0;
  for (int a = 0; a < 3; ++a) {
    if (!finite_pos(grid.h[a])) return DCM_ERR_INVALID;
    hmax = std::max(hmax, grid.h[a]);
  }
  *out = rule.ramp + 3.0 * hmax;
  return DCM_OK;
}

dcm_status dcm_detect_interface(dcm_ctx *ctx, const double *x, const double *y, const double *z,
                                int64_t n, dcm_box box, dcm_grid grid, double split,
                                uint32_t *counts, uint8_t *seg, uint8_t *iface,
                                int32_t *threshold_out) {
  const dcm_detect_opts opts = {split, -1.0, 0};
  return dcm_detect_interface_opts(ctx, x, y, z, n, box, grid, &opts, counts, seg, iface,
                                   threshold_out);
}

dcm_status dcm_detect_interface_opts(dcm_ctx *ctx, const double *x, const double *y,
                                     const double *z, int64_t n, dcm_box box, dcm_grid grid,
                                     const dcm_detect_opts *opts, uint32_t *counts,
                                     uint8_t *seg, uint8_t *iface, int32_t *threshold_out) {
  int64_t nvox = 0;
  DCM_TRY(detect_check(ctx, x, y, z, n, box, grid, opts, seg, iface, &nvox));
  DetectScratch sc;
  DCM_TRY(detect_scratch(ctx, grid, nvox, *opts, counts, &sc));
  return detect_enqueue(ctx, x, y, z, n, box, grid, *opts, sc, seg, iface, threshold_out, true);
}


namespace {
// The sweep on the context's buffers; dist null: no final pass (the field
// stays in dA / dB with the pass flags, as dcm_step reads it).
// maps set: sources from the regularisation passes' bit-packed phase maps
// (launch_fsm_init_bits) instead of the byte maps seg / iface.
dcm_status sweep_enqueue(dcm_ctx *ctx, const uint8_t *seg, const uint8_t *iface,
                         const dcm_grid &grid, int64_t nvox, double rc_grid, int32_t max_waves,
                         double *dist, int32_t *waves_out, const uint32_t *const *maps = nullptr) {
  DCM_TRY(ensure(ctx, ctx->dA, nvox * sizeof(double)));
  DCM_TRY(ensure(ctx, ctx->dB, nvox * sizeof(double)));
  const int64_t ntiles = fsm_tile_count(grid.n);
  DCM_TRY(ensure(ctx, ctx->fsm_chg, 2 * ntiles));
  uint8_t *chg0 = ptr<uint8_t>(ctx->fsm_chg), *chg1 = chg0 + ntiles;
  DCM_TRY(ensure(ctx, ctx->fsm_flags, (size_t)(max_waves + 2) * sizeof(uint32_t)));
  uint32_t *flags = ptr<uint32_t>(ctx->fsm_flags);
  hipStream_t s = ctx->stream;
  hipEvent_t ev;
  timer_begin(ctx, "sweep", &ev);
  if (maps)
    launch_fsm_init_bits(s, maps, ctx->ctl, grid.n, ptr<double>(ctx->dA), ptr<double>(ctx->dB),
                         chg0, flags, max_waves);
  else
    launch_fsm_init(s, seg, iface, grid.n, ptr<double>(ctx->dA), ptr<double>(ctx->dB), chg0,
                    flags, max_waves);
  for (int w = 1; w <= max_waves; ++w)
    launch_fsm_step(s, ptr<double>(ctx->dA), ptr<double>(ctx->dB), chg0, chg1, grid.n, grid.h,
                    rc_grid, w, flags);
  if (dist)
    launch_fsm_final(s, ptr<double>(ctx->dA), ptr<double>(ctx->dB), nvox, rc_grid, flags,
                     max_waves, dist, waves_out, ctx->d_status);
  timer_end(ctx, "sweep", ev);
  return check_launch(ctx, "dcm_sweep_distance");
}
}  // namespace

dcm_status dcm_sweep_distance(dcm_ctx *ctx, const uint8_t *seg, const uint8_t *iface,
                              dcm_grid grid, double rc_grid, int32_t max_waves, double *dist,
                              int32_t *waves_out) {
  if (!ctx) return DCM_ERR_INVALID;
  int64_t nvox = 0;
  DCM_TRY(check_grid(ctx, grid, &nvox));
  if (!seg || !iface || !dist) return fail(ctx, DCM_ERR_INVALID, "dcm_sweep_distance: null pointer");
  if (!finite_pos(rc_grid)) return fail(ctx, DCM_ERR_INVALID, "rc_grid must be > 0");
  if (max_waves < 1 || max_waves > 100000)
    return fail(ctx, DCM_ERR_INVALID, "max_waves must be in [1, 100000]");
  ctx->have_field = false;  // dcm_step's field lives in the sweep buffers this call reuses
  return sweep_enqueue(ctx, seg, iface, grid, nvox, rc_grid, max_waves, dist, waves_out);
}

dcm_status dcm_assign_cutoffs(dcm_ctx *ctx, const double *x, const double *y, const double *z,
                              int64_t n, dcm_box box, dcm_grid grid, const double *dist,
                              dcm_rule rule, double *delta, double *rc) {
  if (!ctx) return DCM_ERR_INVALID;
  int64_t nvox = 0;
  DCM_TRY(check_n(ctx, n));
  DCM_TRY(check_box(ctx, box));
  DCM_TRY(check_grid(ctx, grid, &nvox));
  if (n > 0 && (!x || !y || !z || !dist || !rc))
    return fail(ctx, DCM_ERR_INVALID, "dcm_assign_cutoffs: null pointer");
  if (!finite_pos(rule.rc_min) || !finite_pos(rule.rc_max) || !finite_pos(rule.ramp) ||
      rule.rc_min > rule.rc_max)
    return fail(ctx, DCM_ERR_INVALID, "rule needs 0 < rc_min <= rc_max and ramp > 0");
  const double sc[3] = {(double)grid.n[0] / box.L[0], (double)grid.n[1] / box.L[1],
                        (double)grid.n[2] / box.L[2]};
  hipEvent_t ev;
  timer_begin(ctx, "cutoffs", &ev);
  launch_assign_cutoffs(ctx->stream, x, y, z, n, box.L, grid.n, sc, dist, rule, delta, rc);
  timer_end(ctx, "cutoffs", ev);
  return check_launch(ctx, "dcm_assign_cutoffs");
}

dcm_status dcm_build_cells(dcm_ctx *ctx, const double *x, const double *y, const double *z,
                           const double *rc, int64_t n, dcm_box box, double cell_edge,
                           double rc_bound, int prec, int32_t *cell_of, int32_t *cell_start) {
  if (!ctx) return DCM_ERR_INVALID;
  // dcm_step's build beside the sweep: rc is not read (the
  // sorted records' cutoffs are written by the cutoff assignment)
  const bool no_rc = ctx->build_no_rc;
  ctx->build_no_rc = false;
  ctx->list_n = -1;
  ctx->ext_src_ok = false;
  DCM_TRY(check_n(ctx, n));
  DCM_TRY(check_box(ctx, box));
  if (n > 0 && (!x || !y || !z || !rc))
    return fail(ctx, DCM_ERR_INVALID, "dcm_build_cells: null pointer");
  if (prec != DCM_FP64 && prec != DCM_FP32_MIXED)
    return fail(ctx, DCM_ERR_INVALID, "unknown precision");
  if (!std::isfinite(cell_edge)) return fail(ctx, DCM_ERR_INVALID, "cell_edge must be finite");
  if (!std::isfinite(rc_bound)) return fail(ctx, DCM_ERR_INVALID, "rc_bound must be finite");
  double edge = cell_edge;
  if (edge == 0.0) {
    // about two particles per cell at the mean density
    double vol = box.L[0] * box.L[1] * box.L[2];
    edge = std::cbrt(2.0 * vol / (double)std::max<int64_t>(n, 1));
  } else if (edge < 0.0) {
    // measured choice among fractions of the smallest cutoff
    DCM_TRY(ensure(ctx, ctx->scalars, 16 * sizeof(double)));
    double *d_min = ptr<double>(ctx->scalars) + 15;
    launch_min_f64(ctx->stream, rc, n, d_min);
    double r_ref = 0.0;
    if (hipMemcpyAsync(&r_ref, d_min, sizeof(double), hipMemcpyDeviceToHost, ctx->stream) !=
            hipSuccess ||
        hipStreamSynchronize(ctx->stream) != hipSuccess)
      return fail(ctx, DCM_ERR_HIP, "dcm_build_cells: cutoff read-back failed");
    const double half = 0.5 * std::min(box.L[0], std::min(box.L[1], box.L[2]));
    if (!(r_ref > 0.0) || !std::isfinite(r_ref)) r_ref = rc_bound > 0.0 ? rc_bound : half;
    const std::vector<double> key = {(double)ctx->device, (double)n, box.L[0], box.L[1],
                                     box.L[2], r_ref, rc_bound, (double)prec, 1.0};
    const double cap = prec == DCM_FP32_MIXED ? kRelMaxEdgeSigma : INFINITY;
    const int64_t nn = std::max<int64_t>(n, 1);
    DCM_TRY(ensure(ctx, ctx->tune_f, 3 * nn * sizeof(double)));
    double *f = ptr<double>(ctx->tune_f);
    auto run = [&](double e) -> dcm_status {
      DCM_TRY(dcm_build_cells(ctx, x, y, z, rc, n, box, e, rc_bound, prec, nullptr, nullptr));
      // forces only: the trials run a kernel instance of their own, so a
      // kernel trace keeps them apart from the caller's energy passes
      return dcm_forces(ctx, dcm_lj{1.0, 1.0}, DCM_PAIR_OWN, prec, 0, f, f + nn, f + 2 * nn,
                        nullptr, nullptr, nullptr, nullptr);
    };
    DCM_TRY(tune_edge(ctx, key, edge_candidates(r_ref, cap, box.L), run, &edge));
  }
  int32_t nc[3];
  int64_t ncell = 1;
  for (int a = 0; a < 3; ++a) {
    double k = std::floor(box.L[a] / edge);
    if (k < 1.0) k = 1.0;
    if (k > 65536.0) return fail(ctx, DCM_ERR_RANGE, "more than 65536 cells along an axis");
    nc[a] = (int32_t)k;
    ncell *= nc[a];
  }
  if (ncell >= (int64_t(1) << 30)) return fail(ctx, DCM_ERR_RANGE, "too many cells");
  DCM_TRY(ensure(ctx, ctx->cell_count, ncell * sizeof(int32_t)));
  DCM_TRY(ensure(ctx, ctx->cell_fill, ncell * sizeof(int32_t)));
  DCM_TRY(ensure(ctx, ctx->cell_start, (ncell + 1) * sizeof(int32_t)));
  DCM_TRY(ensure(ctx, ctx->scan_tmp, scan_tmp_elems(ncell) * sizeof(int32_t)));
  if (n >= (int64_t(1) << 24))
    return fail(ctx, DCM_ERR_RANGE, "the pair kernel supports fewer than 2^24 particles");
  DCM_TRY(ensure(ctx, ctx->perm, n * sizeof(int32_t)));
  DCM_TRY(ensure(ctx, ctx->sort_tmp, std::max<int64_t>(n, 1) * sizeof(int32_t)));
  DCM_TRY(ensure(ctx, ctx->sort_list, cell_sort_list_elems(n) * sizeof(int32_t)));
  DCM_TRY(ensure(ctx, ctx->sorted, n * sizeof(double4)));
  int32_t *cof = cell_of;
  if (!cof) {
    DCM_TRY(ensure(ctx, ctx->cell_of, n * sizeof(int32_t)));
    cof = ptr<int32_t>(ctx->cell_of);
  }
  const double sc[3] = {(double)nc[0] / box.L[0], (double)nc[1] / box.L[1],
                        (double)nc[2] / box.L[2]};
  // every cutoff is clamped to rc_cap, strictly below half the shortest edge
  // so that at most one periodic image of a pair can interact
  const double half = 0.5 * std::min(box.L[0], std::min(box.L[1], box.L[2]));
  const double below_half = std::nextafter(half, 0.0);
  const double rc_cap = rc_bound > 0.0 ? std::min(rc_bound, below_half) : below_half;
  // ghost halo: enough cells on each side for any search radius <= rc_cap
  int32_t halo[3];
  int64_t next = 1;
  double uniform = 1.0, hard = 1.0;
  for (int a = 0; a < 3; ++a) {
    const double len = box.L[a] / (double)nc[a];
    halo[a] = (int32_t)std::ceil(rc_cap / len) + 1;
    const int64_t ne = nc[a] + 2 * (int64_t)halo[a];
    next *= ne;
    if (next >= (int64_t(1) << 30)) return fail(ctx, DCM_ERR_RANGE, "too many ghost cells");
    uniform *= (double)ne / (double)nc[a];
    hard *= 1.0 + 2.0 * std::ceil((double)halo[a] / (double)nc[a]);
  }
  // ghost-extended particle capacity, sized from a synchronised count: the
  // exact count of the previous build of the same cell geometry (its copy
  // has completed once ext_event has, so a caller queuing many builds waits
  // for at most the previous one) with 25% headroom for particles moving
  // between builds, else this build's own count, read back before the
  // images are written.  A stream being captured into a graph cannot wait:
  // it keeps the uniform-density estimate, the overflow is flagged.
  hipStreamCaptureStatus capture = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(ctx->stream, &capture) != hipSuccess) {
    (void)hipGetLastError();
    capture = hipStreamCaptureStatusNone;
  }
  const bool capturing = capture != hipStreamCaptureStatusNone;
  const int64_t key[7] = {nc[0], nc[1], nc[2], halo[0], halo[1], halo[2], n};
  const bool same_geom = std::equal(key, key + 7, ctx->ext_key);
  if (ctx->ext_copy_pending && !capturing) {
    if (hipEventSynchronize(ctx->ext_event) != hipSuccess)
      return fail(ctx, DCM_ERR_HIP, "dcm_build_cells: ghost count read-back failed");
    ctx->ext_copy_pending = false;
    ctx->ext_exact = *ctx->h_ext_total;
  }
  const double max_need = hard * (double)n + 64.0;  // the most any arrangement needs
  const bool known = same_geom && ctx->ext_exact >= 0 && !ctx->ext_copy_pending;
  // the buffer grows to 1.25 x the exact count (+4096) only when it holds
  // less than 1.1 x (+1024), so a count creeping up between builds does not
  // reallocate it every time
  auto sizes = [&](double exact, double *need, double *want) {
    *need = std::min(std::min(1.1 * exact + 1024.0, max_need), (double)kMaxExtSlots);
    *want = std::min(std::min(1.25 * exact + 4096.0, max_need), (double)kMaxExtSlots);
  };
  double need = 0.0, want = 0.0;
  if (known) sizes((double)ctx->ext_exact, &need, &want);
  else need = want = std::min(std::min(1.5 * uniform * (double)n + 4096.0, max_need),
                              (double)kMaxExtSlots);
  DCM_TRY(ensure(ctx, ctx->rcmax_part, cell_count_blocks(n) * sizeof(unsigned long long)));
  const int64_t nrow1 = ext_row_scratch_elems(nc, halo);
  DCM_TRY(ensure(ctx, ctx->ext_row_count, nrow1 * sizeof(int32_t)));
  DCM_TRY(ensure(ctx, ctx->ext_row_start, nrow1 * sizeof(int32_t)));
  DCM_TRY(ensure(ctx, ctx->ext_row_lo, nrow1 * sizeof(int32_t)));
  DCM_TRY(ensure(ctx, ctx->ext_start, (next + 1) * sizeof(int32_t)));
  // the trimming table (the pair walk's x trimming), unless the extended
  // grid is too large for it
  const bool qtab = next < kQStartMaxCells;
  if (qtab) {
    DCM_TRY(ensure(ctx, ctx->ext_sq, (next + 1) * sizeof(int2)));
    DCM_TRY(ensure(ctx, ctx->qword, std::max<int64_t>(ncell, 1) * sizeof(uint32_t)));
  }
  DCM_TRY(ensure(ctx, ctx->xkey, std::max<int64_t>(n, 1) * sizeof(uint32_t)));
  DCM_TRY(ensure(ctx, ctx->skey, std::max<int64_t>(n, 1) * sizeof(uint32_t)));
  DCM_TRY(ensure(ctx, ctx->scan_tmp, scan_tmp_elems(std::max(ncell, nrow1)) * sizeof(int32_t)));
  // FP32-mixed builds also write the compact records the pair kernel reads
  const bool rel = prec == DCM_FP32_MIXED && halo[1] <= kRelMaxHalo && halo[2] <= kRelMaxHalo;
  hipStream_t s = ctx->stream;
  hipEvent_t ev;
  timer_begin(ctx, "cells", &ev);
  launch_zero2_i32(s, ptr<int32_t>(ctx->cell_count), ptr<int32_t>(ctx->cell_fill), ncell);
  const double *rc_in = no_rc ? nullptr : rc;
  launch_cell_count(s, x, y, z, rc_in, n, box.L, nc, sc, rc_cap, cof, ptr<int32_t>(ctx->cell_count),
                    ptr<unsigned long long>(ctx->rcmax_part), ptr<uint32_t>(ctx->xkey), ctx->ctl,
                    ctx->d_status);
  launch_exclusive_scan(s, ptr<int32_t>(ctx->cell_count), ptr<int32_t>(ctx->cell_start), ncell,
                        ptr<int32_t>(ctx->scan_tmp));
  // the scatter's order (arbitrary within a cell) goes to sort_tmp; the sort
  // writes the final order into perm and the sorted copy beside it
  launch_cell_scatter(s, cof, n, ptr<int32_t>(ctx->cell_start), ptr<int32_t>(ctx->cell_fill),
                      ptr<int32_t>(ctx->sort_tmp), ptr<uint32_t>(ctx->xkey),
                      ptr<uint32_t>(ctx->skey));
  const GatherOut go = {x, y, z, rc_in, {box.L[0], box.L[1], box.L[2]}, rc_cap,
                        ptr<double4>(ctx->sorted)};
  launch_cell_sort(s, ptr<int32_t>(ctx->cell_start), ncell, cof, n, ptr<int32_t>(ctx->sort_tmp),
                   ptr<uint32_t>(ctx->xkey), ptr<uint32_t>(ctx->skey),
                   qtab ? ptr<uint32_t>(ctx->qword) : nullptr, ptr<int32_t>(ctx->perm),
                   ptr<int32_t>(ctx->sort_list), &ctx->ctl->big_cells, &go);
  launch_ext_count(s, ptr<int32_t>(ctx->cell_start), nc, halo, box.L,
                   ptr<int32_t>(ctx->ext_row_count), ptr<int32_t>(ctx->ext_row_start),
                   ptr<int32_t>(ctx->ext_row_lo), ptr<int32_t>(ctx->ext_start),
                   ptr<int32_t>(ctx->scan_tmp), qtab ? ptr<uint32_t>(ctx->qword) : nullptr,
                   qtab ? ptr<int2>(ctx->ext_sq) : nullptr);
  if (!known && !capturing) {
    // a new geometry: this build's exact count sizes the buffers
    if (hipMemcpyAsync(ctx->h_ext_total, ptr<int32_t>(ctx->ext_start) + next, sizeof(int32_t),
                       hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return fail(ctx, DCM_ERR_HIP, "dcm_build_cells: ghost count read-back failed");
    ctx->ext_exact = *ctx->h_ext_total;
    sizes((double)ctx->ext_exact, &need, &want);
  }
  if (!capturing && ctx->ext_exact > kMaxExtSlots)
    return fail(ctx, DCM_ERR_RANGE, "ghost-extended system too large");
  const int64_t ext_cap = (double)ctx->ext_cap >= need ? ctx->ext_cap : (int64_t)want;
  DCM_TRY(ensure(ctx, ctx->ext_pos, ext_cap * sizeof(double4)));
  if (rel) DCM_TRY(ensure(ctx, ctx->ext_rel, ext_cap * sizeof(float4)));
  ctx->ext_cap = ext_cap;
  launch_ext_images(s, ptr<int32_t>(ctx->cell_start), ptr<int32_t>(ctx->ext_row_start),
                    ptr<int32_t>(ctx->ext_row_lo), ptr<double4>(ctx->sorted), nc, halo, box.L,
                    ext_cap, ptr<double4>(ctx->ext_pos), rel ? ptr<float4>(ctx->ext_rel) : nullptr,
                    ctx->d_status);
  // exact ghost-extended count, read by the next build of this geometry
  std::copy(key, key + 7, ctx->ext_key);
  if (!capturing) {
    if (hipMemcpyAsync(ctx->h_ext_total, ptr<int32_t>(ctx->ext_start) + next, sizeof(int32_t),
                       hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipEventRecord(ctx->ext_event, s) != hipSuccess)
      return fail(ctx, DCM_ERR_HIP, "dcm_build_cells: ghost count read-back failed");
    ctx->ext_copy_pending = true;
  }
  if (cell_start && hipMemcpyAsync(cell_start, ctx->cell_start.p, (ncell + 1) * sizeof(int32_t),
                                   hipMemcpyDeviceToDevice, s) != hipSuccess)
    return fail(ctx, DCM_ERR_HIP, "dcm_build_cells: cell_start copy failed");
  timer_end(ctx, "cells", ev);
  for (int a = 0; a < 3; ++a) {
    ctx->halo[a] = halo[a];
    ctx->nc[a] = nc[a];
    ctx->cell_len[a] = box.L[a] / (double)nc[a];
    ctx->cell_scale[a] = sc[a];
    ctx->cell_box.L[a] = box.L[a];
  }
  ctx->cell_n = n;
  ctx->list_n = -1;  // a list belongs to the build it was made on
  ctx->cells_moved = false;
  ctx->ext_src_ok = false;
  ctx->cell_prec = prec;
  ctx->cell_rel = rel;
  ctx->cell_qtab = qtab;
  ctx->rc_bound = rc_cap;
  return check_launch(ctx, "dcm_build_cells");
}

dcm_status dcm_walk_stats(dcm_ctx *ctx, uint64_t stats[2]) {
  if (!ctx || !stats) return DCM_ERR_INVALID;
  if (!ctx->walk_valid)
    return fail(ctx, DCM_ERR_INVALID, "dcm_walk_stats: no dcm_forces call with DCM_EV_COUNTS");
  unsigned long long h[2] = {0, 0};
  if (hipMemcpyAsync(h, ctx->walk.p, sizeof(h), hipMemcpyDeviceToHost, ctx->stream) != hipSuccess ||
      hipStreamSynchronize(ctx->stream) != hipSuccess)
    return fail(ctx, DCM_ERR_HIP, "dcm_walk_stats: read-back failed");
  stats[0] = h[0];
  stats[1] = h[1];
  return DCM_OK;
}

dcm_status dcm_cell_dims(const dcm_ctx *ctx, int32_t n_cells[3], double cell_len[3]) {
  if (!ctx || !n_cells) return DCM_ERR_INVALID;
  if (ctx->cell_n < 0) return DCM_ERR_INVALID;
  for (int a = 0; a < 3; ++a) {
    n_cells[a] = ctx->nc[a];
    if (cell_len) cell_len[a] = ctx->cell_len[a];
  }
  return DCM_OK;
}

namespace {
// dcm_forces and dcm_forces_list: the cell walk, or the Verlet list of the
// current cell build
dcm_status forces_impl(dcm_ctx *ctx, dcm_lj lj, int pair_rule, int prec, int ev_flags, double *fx,
                       double *fy, double *fz, double *energy, double *virial, int32_t *nnbr,
                       uint64_t *npairs, bool use_list) {
  if (!ctx) return DCM_ERR_INVALID;
  if (ctx->cell_n < 0) return fail(ctx, DCM_ERR_INVALID, "dcm_forces before dcm_build_cells");
  if (use_list && ctx->list_n != ctx->cell_n)
    return fail(ctx, DCM_ERR_INVALID, "dcm_forces_list needs dcm_build_list after the cell build");
  if (!use_list && ctx->cells_moved)
    return fail(ctx, DCM_ERR_INVALID,
                "dcm_forces after dcm_update_list: the particles have left their cells; build "
                "the cells again");
  const int64_t n = ctx->cell_n;
  if (n > 0 && (!fx || !fy || !fz)) return fail(ctx, DCM_ERR_INVALID, "dcm_forces: null force");
  if (pair_rule != DCM_PAIR_OWN && pair_rule != DCM_PAIR_MAX && pair_rule != DCM_PAIR_MAX_N3)
    return fail(ctx, DCM_ERR_INVALID, "unknown pair rule");
  if (prec != DCM_FP64 && prec != DCM_FP32_MIXED)
    return fail(ctx, DCM_ERR_INVALID, "unknown precision");
  if (!finite_pos(lj.epsilon) || !finite_pos(lj.sigma))
    return fail(ctx, DCM_ERR_INVALID, "LJ epsilon and sigma must be > 0");
  if ((ev_flags & DCM_EV_ENERGY) && !energy)
    return fail(ctx, DCM_ERR_INVALID, "energy requested without a pointer");
  if ((ev_flags & DCM_EV_VIRIAL) && !virial)
    return fail(ctx, DCM_ERR_INVALID, "virial requested without a pointer");
  const int64_t blocks = std::max<int64_t>(1, ceil_div(n, pair_block_size()));
  DCM_TRY(ensure(ctx, ctx->partials, blocks * kPartialSlots * sizeof(double)));
  PairArgs a;
  a.pos = ptr<double4>(ctx->sorted);
  a.cell_start = ptr<int32_t>(ctx->cell_start);
  a.perm = ptr<int32_t>(ctx->perm);
  a.ext_pos = ptr<double4>(ctx->ext_pos);
  // FP32-mixed own-cutoff forces on an FP32-mixed build read the compact
  // records, if the cells are narrow enough for their precision
  const double max_len =
      std::max(ctx->cell_len[0], std::max(ctx->cell_len[1], ctx->cell_len[2]));
  // (the compact-record walk always trims rows with the sub-cell table)
  const bool rel = ctx->cell_rel && ctx->cell_qtab && prec == DCM_FP32_MIXED &&
                   pair_rule == DCM_PAIR_OWN && max_len <= kRelMaxEdgeSigma * lj.sigma;
  a.ext_rel = rel ? ptr<float4>(ctx->ext_rel) : nullptr;
  double span = 0.0;  // largest coordinate magnitude in the extended grid
  for (int k = 0; k < 3; ++k)
    span = std::max(span, ctx->cell_box.L[k] + 2.0 * ctx->halo[k] * ctx->cell_len[k]);
  a.rel_delta = rel_record_delta(ctx->cell_len, span);
  a.ext_start = ptr<int32_t>(ctx->ext_start);
  a.ext_sq = ctx->cell_qtab ? ptr<int2>(ctx->ext_sq) : nullptr;
  a.n = n;
  a.ext_cap = ctx->ext_cap;
  for (int k = 0; k < 3; ++k) {
    a.nc[k] = ctx->nc[k];
    a.h[k] = ctx->halo[k];
    a.ne[k] = ctx->nc[k] + 2 * ctx->halo[k];
    a.len[k] = ctx->cell_len[k];
    a.sc[k] = ctx->cell_scale[k];
    a.L[k] = ctx->cell_box.L[k];
  }
  a.rc_bound = ctx->rc_bound;
  a.eps = lj.epsilon;
  a.sigma = lj.sigma;
  a.ev_flags = ev_flags;
  a.ctl = ctx->ctl;
  a.fx = fx;
  a.fy = fy;
  a.fz = fz;
  a.nnbr = (ev_flags & DCM_EV_COUNTS) ? nnbr : nullptr;
  a.partials = ptr<double>(ctx->partials);
  a.status = ctx->d_status;
  const bool n3 = pair_rule == DCM_PAIR_MAX_N3;
  a.ext_src = nullptr;
  a.n3_f = nullptr;
  a.n3_cnt = nullptr;
  if (n3) {
    // the ghosts' source slots, made once per cell build
    if (!ctx->ext_src_ok) {
      DCM_TRY(ensure(ctx, ctx->ext_src, ctx->ext_cap * sizeof(int32_t)));
      launch_ext_src(ctx->stream, ptr<int32_t>(ctx->cell_start), ptr<int32_t>(ctx->ext_row_start),
                     ptr<int32_t>(ctx->ext_row_lo), ctx->nc, ctx->halo, ctx->cell_box.L,
                     ctx->ext_cap, ptr<int32_t>(ctx->ext_src), ctx->d_status);
      ctx->ext_src_ok = true;
    }
    a.ext_src = ptr<int32_t>(ctx->ext_src);
    DCM_TRY(ensure(ctx, ctx->n3_f, std::max<int64_t>(n, 1) * sizeof(double4)));
    DCM_TRY(ensure(ctx, ctx->n3_cnt, std::max<int64_t>(n, 1) * sizeof(int32_t)));
    a.n3_f = ptr<double4>(ctx->n3_f);
    a.n3_cnt = (ev_flags & DCM_EV_COUNTS) ? ptr<int32_t>(ctx->n3_cnt) : nullptr;
    // zero sums (fill kernels, not memsets, so the calls stay capturable)
    launch_fill_u32(ctx->stream, ptr<uint32_t>(ctx->n3_f), 0u, 8 * n);
    if (a.n3_cnt) launch_fill_i32(ctx->stream, a.n3_cnt, 0, n);
  }
  // a pair-count pass over the cells also counts the walk's candidates and rows
  a.walk = nullptr;
  ctx->walk_valid = false;
  if ((ev_flags & DCM_EV_COUNTS) && !use_list) {
    DCM_TRY(ensure(ctx, ctx->walk, 2 * sizeof(unsigned long long)));
    a.walk = ptr<unsigned long long>(ctx->walk);
    launch_fill_u64(ctx->stream, a.walk, 0ull, 2);
    ctx->walk_valid = true;
  }
  hipEvent_t ev;
  timer_begin(ctx, "pair", &ev);
  if (use_list)
    launch_pair_list(ctx->stream, a, prec, ptr<int32_t>(ctx->list_count),
                     ptr<int32_t>(ctx->list_wave_start), ptr<int32_t>(ctx->list));
  else
    launch_pair(ctx->stream, a, pair_rule, prec);
  timer_end(ctx, "pair", ev);
  if (n3)
    launch_n3_out(ctx->stream, a.n3_f, a.n3_cnt, a.perm, n, lj.epsilon, fx, fy, fz, a.nnbr,
                  ctx->d_status);
  if (ev_flags & (DCM_EV_ENERGY | DCM_EV_VIRIAL | DCM_EV_COUNTS))
    launch_reduce_partials(ctx->stream, a.partials, blocks, lj.epsilon, ev_flags, energy, virial,
                           npairs);
  return check_launch(ctx, use_list ? "dcm_forces_list" : "dcm_forces");
}
}  // namespace

dcm_status dcm_forces(dcm_ctx *ctx, dcm_lj lj, int pair_rule, int prec, int ev_flags,
                      double *fx, double *fy, double *fz, double *energy, double *virial,
                      int32_t *nnbr, uint64_t *npairs) {
  return forces_impl(ctx, lj, pair_rule, prec, ev_flags, fx, fy, fz, energy, virial, nnbr, npairs,
                     false);
}

dcm_status dcm_build_list(dcm_ctx *ctx, double skin) {
  if (!ctx) return DCM_ERR_INVALID;
  if (ctx->cell_n < 0) return fail(ctx, DCM_ERR_INVALID, "dcm_build_list before dcm_build_cells");
  const double edge = std::min(ctx->cell_len[0], std::min(ctx->cell_len[1], ctx->cell_len[2]));
  if (!std::isfinite(skin) || skin < 0.0 || skin > edge)
    return fail(ctx, DCM_ERR_INVALID, "skin must be in [0, cell edge]");
  if (ctx->cells_moved)
    return fail(ctx, DCM_ERR_INVALID,
                "dcm_build_list after dcm_update_list: build the cells again first");
  const int64_t n = ctx->cell_n, nw = list_waves(n);
  DCM_TRY(ensure(ctx, ctx->list_count, std::max<int64_t>(n, 1) * sizeof(int32_t)));
  DCM_TRY(ensure(ctx, ctx->list_wave_len, std::max<int64_t>(nw, 1) * sizeof(int32_t)));
  DCM_TRY(ensure(ctx, ctx->list_wave_start, (nw + 1) * sizeof(int32_t)));
  DCM_TRY(ensure(ctx, ctx->list_ref, std::max<int64_t>(n, 1) * sizeof(double4)));
  DCM_TRY(ensure(ctx, ctx->scan_tmp, scan_tmp_elems(std::max<int64_t>(nw, 1)) * sizeof(int32_t)));
  ListArgs a;
  a.pos = ptr<double4>(ctx->sorted);
  a.cell_start = ptr<int32_t>(ctx->cell_start);
  a.ext_pos = ptr<double4>(ctx->ext_pos);
  a.ext_start = ptr<int32_t>(ctx->ext_start);
  a.n = n;
  a.ext_cap = ctx->ext_cap;
  for (int k = 0; k < 3; ++k) {
    a.nc[k] = ctx->nc[k];
    a.h[k] = ctx->halo[k];
    a.ne[k] = ctx->nc[k] + 2 * ctx->halo[k];
    a.len[k] = ctx->cell_len[k];
    a.sc[k] = ctx->cell_scale[k];
  }
  a.rc_bound = ctx->rc_bound;
  a.skin = skin;
  a.count = ptr<int32_t>(ctx->list_count);
  a.wave_len = ptr<int32_t>(ctx->list_wave_len);
  a.wave_start = ptr<int32_t>(ctx->list_wave_start);
  a.n_waves = nw;
  a.list = nullptr;
  a.list_cap = 0;
  a.ref = ptr<double4>(ctx->list_ref);
  a.status = ctx->d_status;
  hipStream_t s = ctx->stream;
  hipEvent_t ev;
  timer_begin(ctx, "list", &ev);
  ctx->list_n = -1;
  if (n > 0) {
    launch_list_count(s, a);
    launch_exclusive_scan(s, ptr<int32_t>(ctx->list_wave_len), ptr<int32_t>(ctx->list_wave_start),
                          nw, ptr<int32_t>(ctx->scan_tmp));
    // the list's size, read back to size its buffer
    if (hipMemcpyAsync(ctx->h_list_total, ptr<int32_t>(ctx->list_wave_start) + nw, sizeof(int32_t),
                       hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return fail(ctx, DCM_ERR_HIP, "dcm_build_list: size read-back failed");
    const int64_t entries = 64 * (int64_t)*ctx->h_list_total;
    DCM_TRY(ensure(ctx, ctx->list, std::max<int64_t>(entries, 1) * sizeof(int32_t)));
    a.list = ptr<int32_t>(ctx->list);
    a.list_cap = entries;
    launch_list_fill(s, a);
  }
  timer_end(ctx, "list", ev);
  DCM_TRY(check_launch(ctx, "dcm_build_list"));
  ctx->list_n = n;
  ctx->list_skin = skin;
  return DCM_OK;
}

dcm_status dcm_update_list(dcm_ctx *ctx, const double *x, const double *y, const double *z,
                           const double *rc, int64_t n, double *max_disp, double *min_slack,
                           int32_t *valid) {
  if (!ctx) return DCM_ERR_INVALID;
  if (!valid) return fail(ctx, DCM_ERR_INVALID, "dcm_update_list: null valid");
  *valid = 0;
  if (ctx->cell_n < 0 || ctx->list_n != ctx->cell_n)
    return fail(ctx, DCM_ERR_INVALID, "dcm_update_list needs dcm_build_list after the cell build");
  if (n != ctx->cell_n)
    return fail(ctx, DCM_ERR_INVALID, "dcm_update_list: n differs from the cell build");
  if (n > 0 && (!x || !y || !z || !rc))
    return fail(ctx, DCM_ERR_INVALID, "dcm_update_list: null pointer");
  const int64_t blocks = list_update_blocks(n);
  DCM_TRY(ensure(ctx, ctx->list_part, blocks * sizeof(double2)));
  DCM_TRY(ensure(ctx, ctx->list_out, 2 * sizeof(double)));
  hipStream_t s = ctx->stream;
  hipEvent_t ev;
  timer_begin(ctx, "list", &ev);
  ctx->cells_moved = true;
  double dmax = 0.0, slack = INFINITY;
  if (n > 0) {
    launch_list_update(s, x, y, z, rc, ptr<int32_t>(ctx->perm), ptr<double4>(ctx->list_ref), n,
                       ctx->cell_box.L, ctx->rc_bound, ptr<double4>(ctx->sorted),
                       ptr<double2>(ctx->list_part), ptr<double>(ctx->list_out), ctx->d_status);
    launch_ext_refill(s, ptr<int32_t>(ctx->cell_start), ptr<int32_t>(ctx->ext_row_start),
                      ptr<int32_t>(ctx->ext_row_lo), ptr<double4>(ctx->sorted), ctx->nc,
                      ctx->halo, ctx->cell_box.L, ctx->ext_cap, ptr<double4>(ctx->ext_pos),
                      ctx->d_status);
  }
  timer_end(ctx, "list", ev);
  if (n > 0) {
    if (hipMemcpyAsync(ctx->h_list_verdict, ptr<double>(ctx->list_out), 2 * sizeof(double),
                       hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return fail(ctx, DCM_ERR_HIP, "dcm_update_list: read-back failed");
    dmax = ctx->h_list_verdict[0];
    slack = ctx->h_list_verdict[1];
  }
  DCM_TRY(check_launch(ctx, "dcm_update_list"));
  // every pair within r_c(i) now was within r_c(i) + 2 dmax <= R_i at the
  // build; the margin covers the rounding of the distance tests
  const double guard = 1e-12 * (ctx->rc_bound + ctx->list_skin);
  const bool ok = (dmax == 0.0 && slack >= 0.0) || (slack - 2.0 * dmax >= guard);
  *valid = ok ? 1 : 0;
  if (max_disp) *max_disp = dmax;
  if (min_slack) *min_slack = slack;
  return DCM_OK;
}

dcm_status dcm_forces_list(dcm_ctx *ctx, dcm_lj lj, int prec, int ev_flags, double *fx,
                           double *fy, double *fz, double *energy, double *virial, int32_t *nnbr,
                           uint64_t *npairs) {
  return forces_impl(ctx, lj, DCM_PAIR_OWN, prec, ev_flags, fx, fy, fz, energy, virial, nnbr,
                     npairs, true);
}

dcm_status dcm_step(dcm_ctx *ctx, double *x, double *y, double *z, double *vx, double *vy,
                    double *vz, double *fx, double *fy, double *fz, int64_t n, double mass,
                    dcm_box box, dcm_lj lj, dcm_rule rule, dcm_grid grid, double rc_grid,
                    int pair_rule, int prec, double dt, int32_t nsteps, int32_t redetect_every,
                    int64_t step0, double *energy_series, double *delta, double *rc) {
  if (!ctx) return DCM_ERR_INVALID;
  int64_t nvox = 0;
  DCM_TRY(check_n(ctx, n));
  DCM_TRY(check_box(ctx, box));
  DCM_TRY(check_grid(ctx, grid, &nvox));
  if (n > 0 && (!x || !y || !z || !fx || !fy || !fz))
    return fail(ctx, DCM_ERR_INVALID, "dcm_step: null pointer");
  if (nsteps > 0 && n > 0 && (!vx || !vy || !vz))
    return fail(ctx, DCM_ERR_INVALID, "dcm_step: null velocity");
  if (nsteps < 0 || redetect_every < 1 || !finite_pos(mass) || !std::isfinite(dt) ||
      !finite_pos(rc_grid))
    return fail(ctx, DCM_ERR_INVALID, "dcm_step: bad nsteps/redetect_every/mass/dt/rc_grid");
  if (!finite_pos(rule.rc_min) || !finite_pos(rule.rc_max) || !finite_pos(rule.ramp) ||
      rule.rc_min > rule.rc_max)
    return fail(ctx, DCM_ERR_INVALID, "rule needs 0 < rc_min <= rc_max and ramp > 0");
  for (int a = 0; a < 3; ++a)
    if (!(rule.rc_max < 0.5 * box.L[a]))
      return fail(ctx, DCM_ERR_RANGE, "rc_max must be below half of every box length");
  DCM_TRY(ensure(ctx, ctx->scalars, 16 * sizeof(double)));
  DCM_TRY(ensure(ctx, ctx->ke, kinetic_blocks(n) * sizeof(double)));
  // working copies: fields x y z, vx vy vz, fx fy fz, delta, rc of every
  // particle, kept in cell order between cell builds
  enum { WX = 0, WY, WZ, WVX, WVY, WVZ, WFX, WFY, WFZ, WDELTA, WRC, WFIELDS };
  static_assert(WFIELDS == kPermFields, "one permute pass moves every field");
  const int64_t nn = std::max<int64_t>(n, 1);
  for (int b = 0; b < 2; ++b) {
    DCM_TRY(ensure(ctx, ctx->ws[b], (size_t)WFIELDS * nn * sizeof(double)));
    DCM_TRY(ensure(ctx, ctx->ws_owner[b], nn * sizeof(int32_t)));
  }
  // a distance field from an earlier call is reused only for the same grid,
  // box, sweep limit and particle count
  for (int a = 0; a < 3; ++a)
    if (ctx->field_n[a] != grid.n[a] || ctx->field_h[a] != grid.h[a] ||
        ctx->field_L[a] != box.L[a])
      ctx->have_field = false;
  if (ctx->field_rc_grid != rc_grid || ctx->field_particles != n) ctx->have_field = false;
  hipStream_t s = ctx->stream;
  int cur = 0;
  auto field = [&](int set, int k) { return ptr<double>(ctx->ws[set]) + (int64_t)k * nn; };
  auto owner = [&](int set) { return ptr<int32_t>(ctx->ws_owner[set]); };
  {
    double *src[] = {x, y, z, vx, vy, vz, fx, fy, fz};
    const int nload = nsteps > 0 ? 9 : 3;
    for (int k = 0; k < nload; ++k)
      if (n > 0 && src[k] &&
          hipMemcpyAsync(field(0, k), src[k], n * sizeof(double), hipMemcpyDeviceToDevice,
                         s) != hipSuccess)
        return fail(ctx, DCM_ERR_HIP, "dcm_step: copy into the working arrays failed");
    launch_iota(s, owner(0), n);
  }
  double *W[WFIELDS];
  auto bind = [&]() {
    for (int k = 0; k < WFIELDS; ++k) W[k] = field(cur, k);
  };
  bind();
  // reorder the working copies into the order of the last cell build.  Only
  // the fields read before the next force pass rewrites them move: positions
  // and velocities, and the forces when the next step opens with its own kick
  // (an energy series is recorded); delta and rc are always recomputed.
  auto reorder = [&]() {
    PermFields f;
    f.nf = 0;
    for (int k = 0; k < WFIELDS; ++k) {
      const bool force = k == WFX || k == WFY || k == WFZ;
      if (k == WDELTA || k == WRC || (force && !energy_series)) continue;
      f.src[f.nf] = field(cur, k);
      f.dst[f.nf] = field(1 - cur, k);
      ++f.nf;
    }
    launch_permute_gather(s, f, ptr<int32_t>(ctx->perm), owner(cur), owner(1 - cur), n);
    cur = 1 - cur;
    bind();
  };
  // results back to the caller's order
  auto unload = [&]() -> dcm_status {
    PermFields f;
    f.nf = 0;
    double *dst[] = {x, y, z, vx, vy, vz, fx, fy, fz, delta, rc};
    const bool want[] = {nsteps > 0, nsteps > 0, nsteps > 0, nsteps > 0, nsteps > 0,
                         nsteps > 0, true,       true,       true,       delta != nullptr,
                         rc != nullptr};
    for (int k = 0; k < WFIELDS; ++k)
      if (want[k] && dst[k]) {
        f.src[f.nf] = W[k];
        f.dst[f.nf] = dst[k];
        ++f.nf;
      }
    launch_permute_scatter(s, f, owner(cur), n);
    return check_launch(ctx, "dcm_step");
  };
  // sweep passes stop early once one changes nothing; the cap only bounds
  // the launches.  A tiled pass settles whole 16x8x8 tiles, so a front
  // crosses at least a tile per pass; a plain pass advances one voxel.
  double hmin = std::min(grid.h[0], std::min(grid.h[1], grid.h[2]));
  int32_t max_waves = fsm_tiled(grid.n)
                          ? std::max<int32_t>(12, (int32_t)std::ceil(2.0 * rc_grid / (8.0 * hmin)) + 8)
                          : std::max<int32_t>(64, (int32_t)std::ceil(4.0 * rc_grid / hmin) + 8);
  double *scal = ptr<double>(ctx->scalars);
  const dcm_detect_opts dopts = {0.0, -1.0, 0};
  // the cell build beside the sweep (set below; a no-op where it does not apply)
  std::function<dcm_status()> build_beside;
  // the previous step's integrator pass binned the density counts already
  bool binned = false;
  auto detect = [&]() -> dcm_status {
    // detection (Section 2.1) without the byte maps: the sweep takes its
    // sources from the phase maps, and the field stays in the sweep's
    // buffers, where the cutoffs read it
    DetectScratch sc;
    DCM_TRY(detect_scratch(ctx, grid, nvox, dopts, nullptr, &sc));
    DCM_TRY(detect_enqueue(ctx, W[WX], W[WY], W[WZ], n, box, grid, dopts, sc, nullptr, nullptr,
                           nullptr, true, binned));
    binned = false;
    const uint32_t *const maps[2] = {sc.seg_a, sc.seg_b};
    if (build_beside) DCM_TRY(build_beside());
    DCM_TRY(sweep_enqueue(ctx, nullptr, nullptr, grid, nvox, rc_grid, max_waves, nullptr, nullptr,
                          maps));
    ctx->have_field = true;
    ctx->field_waves = max_waves;
    for (int a = 0; a < 3; ++a) {
      ctx->field_n[a] = grid.n[a];
      ctx->field_h[a] = grid.h[a];
      ctx->field_L[a] = box.L[a];
    }
    ctx->field_rc_grid = rc_grid;
    ctx->field_particles = n;
    return DCM_OK;
  };
  // small cells (Section 2.3): a measured choice between a third and 0.8 of
  // the smallest cutoff, for FP32-mixed forces at most the widest cell the
  // compact records serve (tuned on the first cell build of this system
  // shape in the process, then remembered)
  double step_cell_edge = 0.0;
  const std::vector<double> edge_key = {
      (double)ctx->device, (double)n,  box.L[0],        box.L[1],          box.L[2],
      rule.rc_min,         rule.rc_max, (double)prec,   (double)pair_rule, lj.sigma};
  const std::vector<double> edge_cands = edge_candidates(
      rule.rc_min, prec == DCM_FP32_MIXED ? kRelMaxEdgeSigma * lj.sigma : INFINITY, box.L);
  // an edge tuned by an earlier call serves from the first step on
  (void)edge_cached(edge_key, &step_cell_edge);
  // cutoffs, cells and forces of the working copies; the forces land in the
  // working order (the cells map sorted slots back to it)
  const double vsc[3] = {(double)grid.n[0] / box.L[0], (double)grid.n[1] / box.L[1],
                         (double)grid.n[2] / box.L[2]};
  // the cells of this step were built beside the sweep (prebuild), and only
  // their records' cutoffs are missing
  bool prebuilt = false;
  auto forces = [&](double *e_out) -> dcm_status {
    // cells built on the second stream: complete before their records
    // take the cutoffs
    if (prebuilt && hipStreamWaitEvent(s, ctx->join_ev, 0) != hipSuccess)
      return fail(ctx, DCM_ERR_HIP, "dcm_step: stream join failed");
    {  // cutoffs (Section 2.2) from the field in the sweep's buffers; the
       // distances are kept only when the caller asks for them
      hipEvent_t cev;
      timer_begin(ctx, "cutoffs", &cev);
      launch_assign_cutoffs_sweep(s, W[WX], W[WY], W[WZ], n, box.L, grid.n, vsc,
                                  ptr<double>(ctx->dA), ptr<double>(ctx->dB),
                                  ptr<uint32_t>(ctx->fsm_flags), ctx->field_waves,
                                  ctx->field_rc_grid, rule, delta ? W[WDELTA] : nullptr, W[WRC],
                                  ctx->d_status,
                                  prebuilt ? ptr<int32_t>(ctx->perm) : nullptr,
                                  ptr<double4>(ctx->sorted), ctx->rc_bound);
      timer_end(ctx, "cutoffs", cev);
      DCM_TRY(check_launch(ctx, "dcm_step cutoffs"));
    }
    if (prebuilt) {
      prebuilt = false;
      return dcm_forces(ctx, lj, pair_rule, prec, DCM_EV_ENERGY, W[WFX], W[WFY], W[WFZ],
                        e_out ? e_out : scal, nullptr, nullptr, nullptr);
    }
    if (step_cell_edge <= 0.0) {
      auto run = [&](double e) -> dcm_status {
        DCM_TRY(dcm_build_cells(ctx, W[WX], W[WY], W[WZ], W[WRC], n, box, e, rule.rc_max, prec,
                                nullptr, nullptr));
        // forces only (a kernel instance apart from the steps' energy passes)
        return dcm_forces(ctx, lj, pair_rule, prec, 0, W[WFX], W[WFY], W[WFZ], nullptr,
                          nullptr, nullptr, nullptr);
      };
      DCM_TRY(tune_edge(ctx, edge_key, edge_cands, run, &step_cell_edge));
    }
    DCM_TRY(dcm_build_cells(ctx, W[WX], W[WY], W[WZ], W[WRC], n, box, step_cell_edge,
                            rule.rc_max, prec, nullptr, nullptr));
    return dcm_forces(ctx, lj, pair_rule, prec, DCM_EV_ENERGY, W[WFX], W[WFY], W[WFZ],
                      e_out ? e_out : scal, nullptr, nullptr, nullptr);
  };
  // Build the cells of a step on a second stream while the sweep runs on the
  // context's stream: the build reads only the positions, and the
  // own-cutoff walk reads only each particle's own cutoff, which the cutoff
  // assignment writes into its sorted record once the cells are complete.
  // The sweep's passes are bound by latency and leave the memory system to
  // the build (the detection before it is bound by HBM bandwidth, as the
  // build is).  Taken once the cell edge is tuned, for the own-cutoff rule,
  // outside stream capture.
  auto prebuild = [&]() -> dcm_status {
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (pair_rule != DCM_PAIR_OWN || step_cell_edge <= 0.0 ||
        hipStreamIsCapturing(s, &cap) != hipSuccess || cap != hipStreamCaptureStatusNone)
      return DCM_OK;
    if (!ctx->side) {
      // on the context's device, whichever is current
      int cur = ctx->device;
      if (hipGetDevice(&cur) != hipSuccess ||
          (cur != ctx->device && hipSetDevice(ctx->device) != hipSuccess))
        return fail(ctx, DCM_ERR_HIP, "dcm_step: device selection failed");
      hipStream_t side = nullptr;
      hipEvent_t fork = nullptr, join = nullptr;
      hipError_t e = hipStreamCreateWithFlags(&side, hipStreamNonBlocking);
      if (e == hipSuccess) e = hipEventCreateWithFlags(&fork, hipEventDisableTiming);
      if (e == hipSuccess) e = hipEventCreateWithFlags(&join, hipEventDisableTiming);
      if (e != hipSuccess) {  // nothing is kept: a later step tries again
        if (join) (void)hipEventDestroy(join);
        if (fork) (void)hipEventDestroy(fork);
        if (side) (void)hipStreamDestroy(side);
      }
      if (cur != ctx->device) (void)hipSetDevice(cur);
      if (e != hipSuccess) return fail(ctx, DCM_ERR_HIP, "dcm_step: stream creation failed");
      ctx->side = side;
      ctx->fork_ev = fork;
      ctx->join_ev = join;
    }
    if (hipEventRecord(ctx->fork_ev, s) != hipSuccess ||
        hipStreamWaitEvent(ctx->side, ctx->fork_ev, 0) != hipSuccess)
      return fail(ctx, DCM_ERR_HIP, "dcm_step: stream fork failed");
    ctx->stream = ctx->side;
    ctx->forked_from = s;
    ctx->build_no_rc = true;
    const dcm_status st = dcm_build_cells(ctx, W[WX], W[WY], W[WZ], W[WRC], n, box,
                                          step_cell_edge, rule.rc_max, prec, nullptr, nullptr);
    ctx->stream = s;
    ctx->forked_from = nullptr;
    ctx->build_no_rc = false;
    if (st != DCM_OK) return st;
    if (hipEventRecord(ctx->join_ev, ctx->side) != hipSuccess)
      return fail(ctx, DCM_ERR_HIP, "dcm_step: stream join failed");
    prebuilt = true;
    return DCM_OK;
  };
  build_beside = prebuild;
  if (nsteps == 0) {
    DCM_TRY(detect());
    DCM_TRY(forces(nullptr));
    return unload();
  }
  const double c = (0.5 * dt) / mass;
  bool drifted = false;  // this step's opening kick and drift are done
  for (int32_t st = 0; st < nsteps; ++st) {
    hipEvent_t ev;
    if (!drifted) {
      timer_begin(ctx, "verlet", &ev);
      launch_kick_drift(s, W[WX], W[WY], W[WZ], W[WVX], W[WVY], W[WVZ], W[WFX], W[WFY], W[WFZ],
                        n, c, dt, box.L);
      timer_end(ctx, "verlet", ev);
    }
    // (a step without detection builds its cells in line: nothing to overlap)
    if (!ctx->have_field || (step0 + st + 1) % redetect_every == 0)
      DCM_TRY(detect());
    else
      binned = false;  // (never set for such a step)
    DCM_TRY(forces(energy_series ? energy_series + 2 * (int64_t)st : nullptr));
    timer_begin(ctx, "verlet", &ev);
    // without an energy series to record in between, the closing kick and
    // the next step's opening kick and drift share one pass
    drifted = !energy_series && st + 1 < nsteps;
    // a next step with detection has its density counts binned here, from
    // the new positions (the field exists from this step on)
    const bool bin_next = drifted && (step0 + st + 2) % redetect_every == 0;
    if (bin_next) {
      DetectScratch sc;
      DCM_TRY(detect_scratch(ctx, grid, nvox, dopts, nullptr, &sc));
      launch_zero2_u32(s, sc.counts, nvox, sc.hist, (int64_t)kHistCopies * kHistBins);
      launch_kick_kick_drift_bin(s, W[WX], W[WY], W[WZ], W[WVX], W[WVY], W[WVZ], W[WFX], W[WFY],
                                 W[WFZ], n, c, dt, box.L, grid.n, vsc, sc.counts, ctx->d_status);
      binned = true;
    } else if (drifted) {
      launch_kick_kick_drift(s, W[WX], W[WY], W[WZ], W[WVX], W[WVY], W[WVZ], W[WFX], W[WFY],
                             W[WFZ], n, c, dt, box.L);
    } else {
      launch_kick(s, W[WVX], W[WVY], W[WVZ], W[WFX], W[WFY], W[WFZ], n, c);
    }
    timer_end(ctx, "verlet", ev);
    if (energy_series)
      launch_kinetic(s, W[WVX], W[WVY], W[WVZ], n, mass, ptr<double>(ctx->ke), kinetic_blocks(n),
                     energy_series + 2 * (int64_t)st + 1);
    // keep the working copies in cell order: after the first build, then
    // every few steps (particles move little between steps)
    if (st + 1 < nsteps && (st == 0 || (st + 1) % kReorderEvery == 0)) {
      timer_begin(ctx, "verlet", &ev);
      reorder();
      timer_end(ctx, "verlet", ev);
    }
    DCM_TRY(check_launch(ctx, "dcm_step"));
  }
  return unload();
}

dcm_status dcm_set_profiling(dcm_ctx *ctx, int enable) {
  if (!ctx) return DCM_ERR_INVALID;
  ctx->profile = enable != 0;
  return DCM_OK;
}

dcm_status dcm_set_profiling_only(dcm_ctx *ctx, const char *family) {
  if (!ctx) return DCM_ERR_INVALID;
  ctx->profile_only = family ? family : "";
  return DCM_OK;
}

dcm_status dcm_kernel_time(dcm_ctx *ctx, const char *family, double *total_ms,
                           int64_t *launches) {
  if (!ctx || !family) return DCM_ERR_INVALID;
  if (hipStreamSynchronize(ctx->stream) != hipSuccess) return DCM_ERR_HIP;
  Timer &t = ctx->timers[family];
  for (auto &pr : t.pending) {
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, pr.first, pr.second) == hipSuccess) {
      t.ms += ms;
      t.launches += 1;
    }
    (void)hipEventDestroy(pr.first);
    (void)hipEventDestroy(pr.second);
  }
  t.pending.clear();
  if (total_ms) *total_ms = t.ms;
  if (launches) *launches = t.launches;
  t.ms = 0.0;
  t.launches = 0;
  return DCM_OK;
}

}  // extern "C"
