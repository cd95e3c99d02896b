// Host side of dcm_forces_batched: the plan (per-system cell geometry, the
// concatenated layout, block tables and the cost-ordered work queue), the
// cell-edge tuner, and the HIP graph that replays a recorded batch.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>

#include "dcm_internal.hpp"

namespace dcm {

namespace {

constexpr int kItem = 256;  // particles per work item = pair kernel block
// cell edges the tuner tries for systems that leave the edge to the library
constexpr double kTuneEdges[] = {1.0, 1.15, 1.3, 1.5, 1.75};

template <typename T>
T *dptr(const DevBuf &b, size_t byte_off = 0) {
  return reinterpret_cast<T *>(static_cast<char *>(b.p) + byte_off);
}

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

}  // namespace

struct BatchState {
  // descriptors of the batch the plan was made for
  std::vector<dcm_system> desc;
  bool have_plan = false;
  double plan_edge = 0.0;  // edge used for systems with cell_edge <= 0
  bool tuned = false;
  double tuned_edge = 0.0;
  int tuned_queues = 1;
  int tuned_lists = 0;  // row-list variant of the compact-record pair kernel
  int row_lists = 0;    // the variant the next launches use
  bool needs_tuning = false;
  int plan_queues = 1;  // work-queue segments of the plan: 1 or kXcds
  // plan
  std::vector<SysGeom> geo;
  std::vector<int2> items;  // natural order: system-major, also the particle block table
  std::vector<int2> eblk;
  std::vector<int2> rblk;  // (system, first extended row) per group of 256 rows
  std::vector<int32_t> queue;
  std::vector<int32_t> qseg;  // segment starts in queue [plan_queues + 1]
  int64_t n_total = 0, cells_total = 0, ext_cells_total = 0, ext_rows_total = 0, ext_cap = 0;
  bool rel_ok = true;  // every system's halos fit the compact records
  double max_len = 0.0;  // widest cell edge of any system
  size_t off_geo = 0, off_items = 0, off_eblk = 0, off_rblk = 0, off_queue = 0, off_qseg = 0,
         table_bytes = 0;
  std::vector<unsigned char> table_host;
  // device memory
  DevBuf tables, cell_of, cell_count, cell_fill, cell_start, perm, sorted, scan_tmp, row_count,
      row_start, row_lo, ext_start, ext_pos, ext_rel, partials, rcmax, rcmax_part, head,
      sort_tmp, sort_list, xkey, skey, qword, ext_sq;
  // recorded graph
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<unsigned char> graph_key;

  void drop_graph() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
    graph_key.clear();
  }
};

namespace {

bool same_desc(const std::vector<dcm_system> &a, int32_t nsys, const dcm_system *b) {
  return (int64_t)a.size() == nsys &&
         (nsys == 0 || std::memcmp(a.data(), b, sizeof(dcm_system) * nsys) == 0);
}

dcm_status check_system(dcm_ctx *ctx, const dcm_system &s, int32_t b, int ev_flags) {
  auto bad = [&](const char *what) {
    return fail(ctx, DCM_ERR_INVALID,
                std::string("dcm_forces_batched: system ") + std::to_string(b) + ": " + what);
  };
  if (s.n < 0) return bad("particle count must be >= 0");
  for (int a = 0; a < 3; ++a)
    if (!std::isfinite(s.box.L[a]) || !(s.box.L[a] > 0.0)) return bad("box lengths must be > 0");
  if (!std::isfinite(s.cell_edge)) return bad("cell_edge must be finite");
  if (!std::isfinite(s.rc_bound)) return bad("rc_bound must be finite");
  if (s.n > 0 && (!s.x || !s.y || !s.z || !s.rc || !s.fx || !s.fy || !s.fz))
    return bad("null array");
  if ((ev_flags & DCM_EV_ENERGY) && !s.energy) return bad("energy requested without a pointer");
  if ((ev_flags & DCM_EV_VIRIAL) && !s.virial) return bad("virial requested without a pointer");
  return DCM_OK;
}

// Cell geometry, concatenated layout, block tables and work queue for the
// batch, with `edge` for the systems that leave the cell edge to the tuner,
// and `queues` work-queue segments (1 or kBatchQueues).
dcm_status make_plan(dcm_ctx *ctx, BatchState &B, double edge, int queues) {
  const int32_t nsys = (int32_t)B.desc.size();
  B.geo.assign(nsys, SysGeom{});
  B.items.clear();
  B.eblk.clear();
  B.rblk.clear();
  std::vector<double> cost_pp(nsys, 0.0);
  int64_t p0 = 0, cell0 = 0, ext_cell0 = 0, row0 = 0;
  double ext_bound = 0.0;
  B.rel_ok = true;
  B.max_len = 0.0;
  for (int32_t b = 0; b < nsys; ++b) {
    const dcm_system &d = B.desc[b];
    SysGeom &g = B.geo[b];
    g.x = d.x;
    g.y = d.y;
    g.z = d.z;
    g.rc = d.rc;
    g.fx = d.fx;
    g.fy = d.fy;
    g.fz = d.fz;
    g.nnbr = d.nnbr;
    g.energy = d.energy;
    g.virial = d.virial;
    g.npairs = d.npairs;
    g.n = d.n;
    const double e = d.cell_edge > 0.0 ? d.cell_edge : edge;
    const double half = 0.5 * std::min(d.box.L[0], std::min(d.box.L[1], d.box.L[2]));
    const double below_half = std::nextafter(half, 0.0);
    g.rc_cap = d.rc_bound > 0.0 ? std::min(d.rc_bound, below_half) : below_half;
    int64_t cells = 1, next = 1;
    double mult = 1.0;
    for (int a = 0; a < 3; ++a) {
      double k = std::floor(d.box.L[a] / e);
      if (k < 1.0) k = 1.0;
      if (k > 65536.0)
        return fail(ctx, DCM_ERR_RANGE, "dcm_forces_batched: more than 65536 cells along an axis");
      g.nc[a] = (int32_t)k;
      g.L[a] = d.box.L[a];
      g.len[a] = d.box.L[a] / (double)g.nc[a];
      g.sc[a] = (double)g.nc[a] / d.box.L[a];
      g.h[a] = (int32_t)std::ceil(g.rc_cap / g.len[a]) + 1;
      g.ne[a] = g.nc[a] + 2 * g.h[a];
      cells *= g.nc[a];
      next *= g.ne[a];
      // copies of one real cell in the extended grid along this axis
      mult *= std::ceil((double)g.ne[a] / (double)g.nc[a]);
      if (cells >= (int64_t(1) << 30) || next >= (int64_t(1) << 30))
        return fail(ctx, DCM_ERR_RANGE, "dcm_forces_batched: too many cells");
    }
    double span = 0.0;  // largest coordinate magnitude in the extended grid
    for (int a = 0; a < 3; ++a) span = std::max(span, g.L[a] + 2.0 * g.h[a] * g.len[a]);
    g.rel_delta = rel_record_delta(g.len, span);
    if (g.h[1] > kRelMaxHalo || g.h[2] > kRelMaxHalo) B.rel_ok = false;
    for (int a = 0; a < 3; ++a) B.max_len = std::max(B.max_len, g.len[a]);
    g.p0 = p0;
    g.cell0 = cell0;
    g.ext_cell0 = ext_cell0;
    g.row0 = row0;
    const int64_t rows = (int64_t)g.ne[1] * g.ne[2];
    for (int64_t k = 0; k < rows; k += 256) B.rblk.push_back(make_int2(b, (int)k));
    row0 += rows;
    g.item0 = (int64_t)B.items.size();
    g.nitems = (d.n + kItem - 1) / kItem;
    for (int64_t k = 0; k < g.nitems; ++k) B.items.push_back(make_int2(b, (int)(k * kItem)));
    for (int64_t k = 0; k < next; k += 256) B.eblk.push_back(make_int2(b, (int)k));
    p0 += d.n;
    cell0 += cells;
    ext_cell0 += next;
    ext_bound += mult * (double)d.n;
    // candidates per particle grow with the density and the search volume
    const double vol = d.box.L[0] * d.box.L[1] * d.box.L[2];
    cost_pp[b] = ((double)d.n / vol) * g.rc_cap * g.rc_cap * g.rc_cap;
    if (p0 >= (int64_t(1) << 24))
      return fail(ctx, DCM_ERR_RANGE, "dcm_forces_batched: 2^24 or more particles in total");
    if (cell0 >= (int64_t(1) << 30) || ext_cell0 >= (int64_t(1) << 30))
      return fail(ctx, DCM_ERR_RANGE, "dcm_forces_batched: too many cells");
  }
  // beyond the addressable size the build flags an overflow instead
  if (ext_bound > (double)kMaxExtSlots) ext_bound = (double)kMaxExtSlots;
  B.n_total = p0;
  B.cells_total = cell0;
  B.ext_cells_total = ext_cell0;
  B.ext_rows_total = row0;
  // the most ghost copies any arrangement of the particles can need
  // (capped at what the pair kernel can address)
  B.ext_cap = std::max<int64_t>((int64_t)ext_bound, 1);
  // work queue: largest estimated cost first, ties in natural order
  const int64_t nitems = (int64_t)B.items.size();
  std::vector<double> cost(nitems);
  for (int64_t k = 0; k < nitems; ++k) {
    const int b = B.items[k].x;
    const int64_t cnt = std::min<int64_t>(kItem, B.desc[b].n - B.items[k].y);
    cost[k] = cost_pp[b] * (double)cnt;
  }
  B.plan_queues = queues;
  B.queue.resize(nitems);
  B.qseg.assign(queues + 1, 0);
  if (queues == 1) {
    std::iota(B.queue.begin(), B.queue.end(), 0);
    std::stable_sort(B.queue.begin(), B.queue.end(),
                     [&](int32_t a, int32_t b) { return cost[a] > cost[b]; });
    B.qseg[1] = (int32_t)nitems;
  } else {
    // whole systems to segments, the costliest first onto the least loaded
    // one; a segment lists its systems' items in natural order
    std::vector<double> scost(nsys, 0.0);
    for (int64_t k = 0; k < nitems; ++k) scost[B.items[k].x] += cost[k];
    std::vector<int32_t> order(nsys);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(),
                     [&](int32_t a, int32_t b) { return scost[a] > scost[b]; });
    std::vector<double> load(queues, 0.0);
    std::vector<int32_t> seg_of(nsys, 0);
    for (int32_t b : order) {
      const int q = (int)(std::min_element(load.begin(), load.end()) - load.begin());
      seg_of[b] = q;
      load[q] += scost[b];
    }
    int64_t pos = 0;
    for (int q = 0; q < queues; ++q) {
      B.qseg[q] = (int32_t)pos;
      for (int64_t k = 0; k < nitems; ++k)
        if (seg_of[B.items[k].x] == q) B.queue[pos++] = (int32_t)k;
    }
    B.qseg[queues] = (int32_t)pos;
  }
  // device tables, uploaded once per plan
  B.off_geo = 0;
  B.off_items = align256(sizeof(SysGeom) * nsys);
  B.off_eblk = B.off_items + align256(sizeof(int2) * std::max<int64_t>(nitems, 1));
  B.off_rblk = B.off_eblk + align256(sizeof(int2) * std::max<size_t>(B.eblk.size(), 1));
  B.off_queue = B.off_rblk + align256(sizeof(int2) * std::max<size_t>(B.rblk.size(), 1));
  B.off_qseg = B.off_queue + align256(sizeof(int32_t) * std::max<int64_t>(nitems, 1));
  B.table_bytes = B.off_qseg + align256(sizeof(int32_t) * (queues + 1));
  B.table_host.assign(B.table_bytes, 0);
  std::memcpy(B.table_host.data() + B.off_geo, B.geo.data(), sizeof(SysGeom) * nsys);
  if (nitems) {
    std::memcpy(B.table_host.data() + B.off_items, B.items.data(), sizeof(int2) * nitems);
    std::memcpy(B.table_host.data() + B.off_queue, B.queue.data(), sizeof(int32_t) * nitems);
  }
  std::memcpy(B.table_host.data() + B.off_qseg, B.qseg.data(), sizeof(int32_t) * (queues + 1));
  if (!B.eblk.empty())
    std::memcpy(B.table_host.data() + B.off_eblk, B.eblk.data(), sizeof(int2) * B.eblk.size());
  if (!B.rblk.empty())
    std::memcpy(B.table_host.data() + B.off_rblk, B.rblk.data(), sizeof(int2) * B.rblk.size());
  // growing a buffer moves it: a recorded graph would hold stale addresses
  B.drop_graph();
  dcm_status st;
  if ((st = ensure(ctx, B.tables, B.table_bytes)) != DCM_OK) return st;
  if ((st = ensure(ctx, B.cell_of, sizeof(int32_t) * std::max<int64_t>(B.n_total, 1))) != DCM_OK)
    return st;
  if ((st = ensure(ctx, B.cell_count, sizeof(int32_t) * B.cells_total)) != DCM_OK) return st;
  if ((st = ensure(ctx, B.cell_fill, sizeof(int32_t) * B.cells_total)) != DCM_OK) return st;
  if ((st = ensure(ctx, B.cell_start, sizeof(int32_t) * (B.cells_total + 1))) != DCM_OK) return st;
  if ((st = ensure(ctx, B.sort_tmp, sizeof(int32_t) * std::max<int64_t>(B.n_total, 1))) != DCM_OK)
    return st;
  if ((st = ensure(ctx, B.sort_list, sizeof(int32_t) * cell_sort_list_elems(B.n_total))) != DCM_OK)
    return st;
  if ((st = ensure(ctx, B.perm, sizeof(int32_t) * std::max<int64_t>(B.n_total, 1))) != DCM_OK)
    return st;
  if ((st = ensure(ctx, B.xkey, sizeof(uint32_t) * std::max<int64_t>(B.n_total, 1))) != DCM_OK)
    return st;
  if ((st = ensure(ctx, B.skey, sizeof(uint32_t) * std::max<int64_t>(B.n_total, 1))) != DCM_OK)
    return st;
  if ((st = ensure(ctx, B.qword, sizeof(uint32_t) * std::max<int64_t>(B.cells_total, 1))) !=
      DCM_OK)
    return st;
  if ((st = ensure(ctx, B.sorted, sizeof(double4) * std::max<int64_t>(B.n_total, 1))) != DCM_OK)
    return st;
  if ((st = ensure(ctx, B.scan_tmp,
                   sizeof(int32_t) * scan_tmp_elems(std::max(B.cells_total, B.ext_rows_total)))) !=
      DCM_OK)
    return st;
  if ((st = ensure(ctx, B.row_count, sizeof(int32_t) * (B.ext_rows_total + 1))) != DCM_OK) return st;
  if ((st = ensure(ctx, B.row_start, sizeof(int32_t) * (B.ext_rows_total + 1))) != DCM_OK) return st;
  if ((st = ensure(ctx, B.row_lo, sizeof(int32_t) * (B.ext_rows_total + 1))) != DCM_OK) return st;
  if ((st = ensure(ctx, B.ext_start, sizeof(int32_t) * (B.ext_cells_total + 1))) != DCM_OK)
    return st;
  if ((st = ensure(ctx, B.ext_sq, sizeof(int2) * (B.ext_cells_total + 1))) != DCM_OK) return st;
  if ((st = ensure(ctx, B.ext_pos, sizeof(double4) * B.ext_cap)) != DCM_OK) return st;
  if (B.rel_ok && (st = ensure(ctx, B.ext_rel, sizeof(float4) * B.ext_cap)) != DCM_OK) return st;
  if ((st = ensure(ctx, B.partials,
                   sizeof(double) * kPartialSlots * std::max<int64_t>(nitems, 1))) != DCM_OK)
    return st;
  if ((st = ensure(ctx, B.rcmax, sizeof(unsigned long long) * nsys)) != DCM_OK) return st;
  if ((st = ensure(ctx, B.rcmax_part, sizeof(unsigned long long) * std::max<int64_t>(nitems, 1))) !=
      DCM_OK)
    return st;
  // work-queue positions and the cell sort's count of large cells
  if ((st = ensure(ctx, B.head, (kBatchQueues + 1) * sizeof(uint32_t))) != DCM_OK) return st;
  // plans change rarely: a synchronous upload keeps the host copy free to
  // change as soon as this returns
  if (hipMemcpyAsync(B.tables.p, B.table_host.data(), B.table_bytes, hipMemcpyHostToDevice,
                     ctx->stream) != hipSuccess ||
      hipStreamSynchronize(ctx->stream) != hipSuccess)
    return fail(ctx, DCM_ERR_HIP, "dcm_forces_batched: table upload failed");
  B.have_plan = true;
  B.plan_edge = edge;
  return DCM_OK;
}

// Enqueue the whole batch on stream s (no allocation, no host sync).
void enqueue(dcm_ctx *ctx, BatchState &B, hipStream_t s, dcm_lj lj, int rule, int prec,
             int ev_flags, bool timed) {
  const int32_t nsys = (int32_t)B.desc.size();
  const SysGeom *geo = dptr<SysGeom>(B.tables, B.off_geo);
  const int2 *items = dptr<int2>(B.tables, B.off_items);
  const int2 *eblk = dptr<int2>(B.tables, B.off_eblk);
  const int32_t *queue = dptr<int32_t>(B.tables, B.off_queue);
  const int64_t nitems = (int64_t)B.items.size();
  // FP32-mixed own-cutoff forces read the compact records
  float4 *rel = (B.rel_ok && prec == DCM_FP32_MIXED && rule == DCM_PAIR_OWN &&
                 B.max_len <= kRelMaxEdgeSigma * lj.sigma)
                    ? dptr<float4>(B.ext_rel)
                    : nullptr;
  hipEvent_t ev = nullptr;
  if (timed) timer_begin(ctx, "batch_cells", &ev);
  launch_zero2_i32(s, dptr<int32_t>(B.cell_count), dptr<int32_t>(B.cell_fill), B.cells_total);
  launch_fill_u32(s, dptr<uint32_t>(B.head), 0u, kBatchQueues + 1);
  launch_batch_cell_count(s, geo, nsys, items, nitems, dptr<int32_t>(B.cell_of),
                          dptr<int32_t>(B.cell_count), dptr<unsigned long long>(B.rcmax_part),
                          dptr<unsigned long long>(B.rcmax), dptr<uint32_t>(B.xkey),
                          ctx->d_status);
  launch_exclusive_scan(s, dptr<int32_t>(B.cell_count), dptr<int32_t>(B.cell_start),
                        B.cells_total, dptr<int32_t>(B.scan_tmp));
  launch_batch_cell_scatter(s, geo, items, nitems, dptr<int32_t>(B.cell_of),
                            dptr<int32_t>(B.cell_start), dptr<int32_t>(B.cell_fill),
                            dptr<int32_t>(B.perm), dptr<uint32_t>(B.xkey), dptr<uint32_t>(B.skey));
  launch_cell_sort(s, dptr<int32_t>(B.cell_start), B.cells_total, dptr<int32_t>(B.cell_of),
                   B.n_total, dptr<int32_t>(B.perm), dptr<uint32_t>(B.xkey),
                   dptr<uint32_t>(B.skey), dptr<uint32_t>(B.qword), dptr<int32_t>(B.sort_tmp),
                   dptr<int32_t>(B.sort_list), dptr<uint32_t>(B.head) + kBatchQueues);
  launch_batch_gather(s, geo, items, nitems, dptr<int32_t>(B.sort_tmp), dptr<double4>(B.sorted),
                      dptr<int32_t>(B.perm));
  launch_batch_ext(s, geo, eblk, (int64_t)B.eblk.size(), dptr<int2>(B.tables, B.off_rblk),
                   (int64_t)B.rblk.size(), dptr<int32_t>(B.cell_start), dptr<double4>(B.sorted),
                   B.ext_cells_total, B.ext_rows_total, B.ext_cap, dptr<int32_t>(B.row_count),
                   dptr<int32_t>(B.row_start), dptr<int32_t>(B.row_lo), dptr<int32_t>(B.ext_start),
                   dptr<int32_t>(B.scan_tmp), dptr<double4>(B.ext_pos), rel,
                   dptr<uint32_t>(B.qword), dptr<int2>(B.ext_sq), ctx->d_status);
  if (timed) timer_end(ctx, "batch_cells", ev);
  BatchPairArgs a;
  a.sys = geo;
  a.items = items;
  a.queue = queue;
  a.qseg = dptr<int32_t>(B.tables, B.off_qseg);
  a.nqueues = B.plan_queues;
  a.nitems = (int32_t)nitems;
  a.head = dptr<uint32_t>(B.head);
  a.pos = dptr<double4>(B.sorted);
  a.cell_start = dptr<int32_t>(B.cell_start);
  a.perm = dptr<int32_t>(B.perm);
  a.ext_pos = dptr<double4>(B.ext_pos);
  a.ext_rel = rel;
  a.ext_start = dptr<int32_t>(B.ext_start);
  a.ext_sq = dptr<int2>(B.ext_sq);
  a.ext_cap = B.ext_cap;
  a.rc_max_bits = dptr<unsigned long long>(B.rcmax);
  a.eps = lj.epsilon;
  a.sigma = lj.sigma;
  a.ev_flags = ev_flags;
  a.partials = dptr<double>(B.partials);
  a.status = ctx->d_status;
  if (timed) timer_begin(ctx, "batch_pair", &ev);
  launch_pair_batched(s, a, rule, prec, B.row_lists);
  launch_batch_reduce(s, geo, nsys, dptr<double>(B.partials), ev_flags);
  if (timed) timer_end(ctx, "batch_pair", ev);
}

// Time the batch at each candidate edge, work-queue layout (one queue in
// cost order, or one per XCD) and, for the compact-record kernel, row-list
// variant (second of two runs each) and keep the fastest.  Synchronises the
// stream.
dcm_status tune(dcm_ctx *ctx, BatchState &B, dcm_lj lj, int rule, int prec, int ev_flags) {
  double best_ms = 0.0, best_edge = kTuneEdges[0];
  int best_queues = 1, best_lists = 0;
  bool first = true;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return fail(ctx, DCM_ERR_HIP, "event create failed");
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(ctx, DCM_ERR_HIP, "event create failed");
  }
  dcm_status st = DCM_OK;
  const int nedges = (int)(sizeof(kTuneEdges) / sizeof(kTuneEdges[0]));
  const int nlayouts = ctx->batch_queues ? 1 : 2;  // a fixed layout: edges only
  const int nlists =
      (prec == DCM_FP32_MIXED && rule == DCM_PAIR_OWN && ctx->batch_lists == 0) ? 2 : 1;
  for (int trial = 0; trial < nedges * nlayouts * nlists && st == DCM_OK; ++trial) {
    const int il = trial % nlists, iq = (trial / nlists) % nlayouts;
    const double edge = kTuneEdges[trial / (nlists * nlayouts)];
    const int queues = ctx->batch_queues ? ctx->batch_queues : (iq ? kBatchQueues : 1);
    if (il == 0 && (st = make_plan(ctx, B, edge, queues)) != DCM_OK) break;
    B.row_lists = ctx->batch_lists ? ctx->batch_lists - 1 : il;
    enqueue(ctx, B, ctx->stream, lj, rule, prec, ev_flags, false);
    const hipError_t r0 = hipEventRecord(e0, ctx->stream);
    enqueue(ctx, B, ctx->stream, lj, rule, prec, ev_flags, false);
    const hipError_t r1 = hipEventRecord(e1, ctx->stream);
    if ((st = check_launch(ctx, "dcm_forces_batched (tuning)")) != DCM_OK) break;
    float ms = 0.0f;
    if (r0 != hipSuccess || r1 != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
      st = fail(ctx, DCM_ERR_HIP, "dcm_forces_batched: tuning run failed");
      break;
    }
    if (first || ms < best_ms) {
      best_ms = ms;
      best_edge = edge;
      best_queues = queues;
      best_lists = B.row_lists;
      first = false;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != DCM_OK) return st;
  B.tuned = true;
  B.tuned_edge = best_edge;
  B.tuned_queues = best_queues;
  B.tuned_lists = best_lists;
  return DCM_OK;
}

std::vector<unsigned char> graph_key(const BatchState &B, dcm_lj lj, int rule, int prec,
                                     int ev_flags) {
  std::vector<unsigned char> k(sizeof(dcm_system) * B.desc.size() + 64);
  std::memcpy(k.data(), B.desc.data(), sizeof(dcm_system) * B.desc.size());
  unsigned char *t = k.data() + sizeof(dcm_system) * B.desc.size();
  std::memcpy(t, &lj, sizeof(lj));
  std::memcpy(t + 16, &rule, sizeof(int));
  std::memcpy(t + 20, &prec, sizeof(int));
  std::memcpy(t + 24, &ev_flags, sizeof(int));
  std::memcpy(t + 28, &B.plan_edge, sizeof(double));
  std::memcpy(t + 36, &B.plan_queues, sizeof(int));
  std::memcpy(t + 40, &B.row_lists, sizeof(int));
  return k;
}

}  // namespace

void batch_free(dcm_ctx *ctx) {
  BatchState *B = ctx->batch;
  if (!B) return;
  B->drop_graph();
  if (B->cap) (void)hipStreamDestroy(B->cap);
  delete B;
  ctx->batch = nullptr;
}

}  // namespace dcm

using namespace dcm;

extern "C" {

dcm_status dcm_forces_batched(dcm_ctx *ctx, int32_t nsys, const dcm_system *sys, dcm_lj lj,
                              int pair_rule, int prec, int ev_flags, int use_graph) {
  if (!ctx) return DCM_ERR_INVALID;
  if (nsys < 0) return fail(ctx, DCM_ERR_INVALID, "dcm_forces_batched: nsys must be >= 0");
  if (nsys > 0 && !sys) return fail(ctx, DCM_ERR_INVALID, "dcm_forces_batched: null systems");
  if (pair_rule != DCM_PAIR_OWN && pair_rule != DCM_PAIR_MAX)
    return fail(ctx, DCM_ERR_INVALID, "unknown pair rule");
  if (prec != DCM_FP64 && prec != DCM_FP32_MIXED)
    return fail(ctx, DCM_ERR_INVALID, "unknown precision");
  if (!std::isfinite(lj.epsilon) || !(lj.epsilon > 0.0) || !std::isfinite(lj.sigma) ||
      !(lj.sigma > 0.0))
    return fail(ctx, DCM_ERR_INVALID, "LJ epsilon and sigma must be > 0");
  if (nsys == 0) return DCM_OK;
  for (int32_t b = 0; b < nsys; ++b) {
    dcm_status st = check_system(ctx, sys[b], b, ev_flags);
    if (st != DCM_OK) return st;
  }
  if (!ctx->batch) {
    ctx->batch = new (std::nothrow) BatchState();
    if (!ctx->batch) return DCM_ERR_NOMEM;
  }
  BatchState &B = *ctx->batch;
  dcm_status st;
  if (!same_desc(B.desc, nsys, sys)) {
    B.desc.assign(sys, sys + nsys);
    B.have_plan = false;
    B.tuned = false;
    B.drop_graph();
    B.needs_tuning = false;
    for (int32_t b = 0; b < nsys; ++b)
      if (!(sys[b].cell_edge > 0.0)) B.needs_tuning = true;
  }
  if (B.needs_tuning && !B.tuned) {
    if ((st = tune(ctx, B, lj, pair_rule, prec, ev_flags)) != DCM_OK) {
      B.have_plan = false;
      return st;
    }
  }
  const double edge = B.needs_tuning ? B.tuned_edge : 0.0;
  const int queues =
      ctx->batch_queues ? ctx->batch_queues : (B.needs_tuning ? B.tuned_queues : 1);
  B.row_lists = ctx->batch_lists ? ctx->batch_lists - 1 : (B.needs_tuning ? B.tuned_lists : 0);
  if (!B.have_plan || B.plan_edge != edge || B.plan_queues != queues) {
    if ((st = make_plan(ctx, B, edge, queues)) != DCM_OK) {
      B.have_plan = false;
      return st;
    }
  }
  if (!use_graph) {
    enqueue(ctx, B, ctx->stream, lj, pair_rule, prec, ev_flags, ctx->profile);
    return check_launch(ctx, "dcm_forces_batched");
  }
  std::vector<unsigned char> key = graph_key(B, lj, pair_rule, prec, ev_flags);
  if (!B.exec || key != B.graph_key) {
    B.drop_graph();
    if (!B.cap && hipStreamCreateWithFlags(&B.cap, hipStreamNonBlocking) != hipSuccess) {
      B.cap = nullptr;
      return fail(ctx, DCM_ERR_HIP, "dcm_forces_batched: stream create failed");
    }
    // recorded on a stream of our own (the context's stream may be the
    // default stream, which cannot be captured), replayed on the context's
    if (hipStreamBeginCapture(B.cap, hipStreamCaptureModeThreadLocal) != hipSuccess)
      return fail(ctx, DCM_ERR_HIP, "dcm_forces_batched: begin capture failed");
    enqueue(ctx, B, B.cap, lj, pair_rule, prec, ev_flags, false);
    hipError_t ce = hipStreamEndCapture(B.cap, &B.graph);
    if (ce != hipSuccess || !B.graph) {
      (void)hipGetLastError();
      B.graph = nullptr;
      return fail(ctx, DCM_ERR_HIP, "dcm_forces_batched: capture failed");
    }
    if (hipGraphInstantiate(&B.exec, B.graph, nullptr, nullptr, 0) != hipSuccess) {
      (void)hipGetLastError();
      B.drop_graph();
      return fail(ctx, DCM_ERR_HIP, "dcm_forces_batched: graph instantiation failed");
    }
    B.graph_key = key;
  }
  hipEvent_t ev = nullptr;
  timer_begin(ctx, "batch_graph", &ev);
  if (hipGraphLaunch(B.exec, ctx->stream) != hipSuccess) {
    (void)hipGetLastError();
    return fail(ctx, DCM_ERR_HIP, "dcm_forces_batched: graph launch failed");
  }
  timer_end(ctx, "batch_graph", ev);
  return check_launch(ctx, "dcm_forces_batched");
}

dcm_status dcm_batched_edge(const dcm_ctx *ctx, double *edge) {
  if (!ctx || !edge) return DCM_ERR_INVALID;
  *edge = (ctx->batch && ctx->batch->needs_tuning) ? ctx->batch->tuned_edge : 0.0;
  return DCM_OK;
}

dcm_status dcm_batched_queues(const dcm_ctx *ctx, int32_t *queues) {
  if (!ctx || !queues) return DCM_ERR_INVALID;
  *queues = ctx->batch && ctx->batch->have_plan ? ctx->batch->plan_queues : 0;
  return DCM_OK;
}

dcm_status dcm_batched_row_lists(const dcm_ctx *ctx, int32_t *entries) {
  if (!ctx || !entries) return DCM_ERR_INVALID;
  *entries = ctx->batch && ctx->batch->have_plan ? batched_row_lists(ctx->batch->row_lists) : 0;
  return DCM_OK;
}

dcm_status dcm_set_batched_row_lists(dcm_ctx *ctx, int32_t entries) {
  if (!ctx) return DCM_ERR_INVALID;
  int v = -1;
  for (int k = 0; k < 2; ++k)
    if (entries == batched_row_lists(k)) v = k + 1;
  if (entries == 0) v = 0;
  if (v < 0)
    return fail(ctx, DCM_ERR_INVALID, "dcm_set_batched_row_lists: entries must be 0, 14 or 16");
  if (v != ctx->batch_lists && ctx->batch) ctx->batch->tuned = false;  // tune again
  ctx->batch_lists = v;
  return DCM_OK;
}

dcm_status dcm_set_batched_queues(dcm_ctx *ctx, int32_t queues) {
  if (!ctx) return DCM_ERR_INVALID;
  if (queues != 0 && queues != 1 && queues != kBatchQueues)
    return fail(ctx, DCM_ERR_INVALID, "dcm_set_batched_queues: queues must be 0, 1 or 8");
  if (queues != ctx->batch_queues && ctx->batch) {
    ctx->batch->tuned = false;  // tune again (and re-plan) under the new layout
    ctx->batch->have_plan = false;
  }
  ctx->batch_queues = queues;
  return DCM_OK;
}

}  // extern "C"
