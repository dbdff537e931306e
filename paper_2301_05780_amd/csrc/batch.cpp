// Batched assembly of many BVP instances in one persistent launch, HIP graph
// capture/replay, and the launch-shape autotuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>

#include "context.h"

namespace pdd {

namespace {

pdd_status bad(pdd_ctx* ctx, pdd_status st, const std::string& msg) {
  ctx->err = msg;
  return st;
}

bool same_inst_tables(const BatchCache& bc, int32_t n, const pdd_instance* in, int32_t per_ticket,
                      const std::vector<std::vector<int32_t>>& npk) {
  if ((int32_t)bc.parts.size() != n || bc.per_ticket != per_ticket) return false;
  for (int32_t i = 0; i < n; ++i) {
    const pdd_partition& a = bc.parts[i];
    const pdd_partition& b = in[i].part;
    if (a.x0 != b.x0 || a.x1 != b.x1 || a.y0 != b.y0 || a.y1 != b.y1 || a.H != b.H) return false;
    if (bc.knots[i].m != in[i].knots.m || bc.knots[i].ext != in[i].knots.ext) return false;
    if (bc.h[i] != in[i].run.h || bc.a[i] != in[i].coeffs.param[0] || bc.inst_ids[i] != in[i].run.instance) return false;
    if (bc.npk[i] != npk[i]) return false;
  }
  return true;
}

bool is_capturing(hipStream_t s) {
  hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &st) != hipSuccess) return false;
  return st == hipStreamCaptureStatusActive;
}

}  // namespace

pdd_status run_assemble_batch(pdd_ctx* ctx, int32_t n, const pdd_instance* in) {
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return check_hip(ctx, e, "hipSetDevice");
  const pdd_instance& i0 = in[0];
  for (int32_t i = 0; i < n; ++i) {
    const pdd_instance& q = in[i];
    pdd_status st = validate_run(ctx, q.coeffs, q.run);
    if (st != PDD_OK) return st;
    if (!q.row_ptr || !q.col_idx || !q.val || !q.b) return bad(ctx, PDD_EINVAL, "pdd_assemble_batch: null output");
    if (q.run.precision != i0.run.precision || q.run.exit_rule != i0.run.exit_rule ||
        q.coeffs.kind != i0.coeffs.kind || q.run.seed != i0.run.seed)
      return bad(ctx, PDD_EINVAL, "pdd_assemble_batch: instances must share precision, exit rule, family and seed");
    if (q.run.u_ref || q.run.dump_paths)
      return bad(ctx, PDD_EUNSUPPORTED, "pdd_assemble_batch: no u_ref or dump in batches");
    if (q.run.interp != PDD_INTERP_HAT)
      return bad(ctx, PDD_EUNSUPPORTED, "pdd_assemble_batch: batches use the hat interpolation");
    if (q.run.h_per_knot)
      return bad(ctx, PDD_EUNSUPPORTED, "pdd_assemble_batch: one time step per instance (run.h_per_knot unset)");
    // a control variate is shared: the same mode and table or network for
    // every instance, on one domain (the gradient table spans it)
    const int qcv = q.run.cv ? q.run.cv->mode : PDD_CV_NONE;
    const int cv0 = i0.run.cv ? i0.run.cv->mode : PDD_CV_NONE;
    if (qcv != cv0) return bad(ctx, PDD_EINVAL, "pdd_assemble_batch: instances must share the control variate");
    if (cv0 != PDD_CV_NONE) {
      const pdd_cv& a = *q.run.cv;
      const pdd_cv& b0 = *i0.run.cv;
      if (a.params != b0.params || a.grad_lut != b0.grad_lut || a.lut_n != b0.lut_n)
        return bad(ctx, PDD_EINVAL, "pdd_assemble_batch: instances must share the control variate");
      if (q.part.x0 != i0.part.x0 || q.part.x1 != i0.part.x1 || q.part.y0 != i0.part.y0 || q.part.y1 != i0.part.y1)
        return bad(ctx, PDD_EINVAL, "pdd_assemble_batch: with a control variate the instances share the domain");
      if (cv0 == PDD_CV_NETWORK && q.run.precision == PDD_FP64_SAME_STREAM)
        return bad(ctx, PDD_EUNSUPPORTED, "pdd_assemble_batch: the network control variate is float32 only in batches");
    }
  }
  const int cv_mode = i0.run.cv ? i0.run.cv->mode : PDD_CV_NONE;
  const int kind = i0.coeffs.kind;
  if (kind != PDD_COEF_POISSON && kind != PDD_COEF_VARCOEF && kind != PDD_COEF_AMPLITUDE)
    return bad(ctx, PDD_EUNSUPPORTED, "pdd_assemble_batch: families POISSON, VARCOEF and AMPLITUDE only");
  const int precision = i0.run.precision;

  // paths per knot of every instance (validated while building)
  std::vector<std::vector<int32_t>> npk(n);
  int64_t total_paths = 0;
  std::vector<int64_t> n_knots(n);
  for (int32_t i = 0; i < n; ++i) {
    // knot count without building the pattern
    const int64_t H = in[i].part.H, m = in[i].knots.m;
    if (H < 2 || m < 1) return bad(ctx, PDD_EINVAL, "pdd_assemble_batch: invalid partition");
    n_knots[i] = knot_count((int32_t)H, (int32_t)m);
    npk[i].resize(n_knots[i]);
    for (int64_t k = 0; k < n_knots[i]; ++k) {
      const int64_t v = in[i].run.n_paths_per_knot ? in[i].run.n_paths_per_knot[k] : in[i].run.n_paths;
      if (v < 1 || v > INT32_MAX) return bad(ctx, PDD_EINVAL, "pdd_assemble_batch: path counts must be >= 1");
      npk[i][k] = (int32_t)v;
      total_paths += v;
    }
  }

  // launch shape (slot length known only after the geometry: use the cached one if any)
  int block = ctx->force_block ? ctx->force_block : 256;
  BatchCache* bc = ctx->batch.get();
  const bool capturing = is_capturing(ctx->stream);

  // ticket size from the occupancy of a provisional shape
  auto shape = [&](int slot_len, int& blk, size_t& lds, int64_t& grid) -> pdd_status {
    const int row_len = 4 * slot_len + EX_COUNT;
    blk = block;
    lds = assemble_lds_bytes(precision, kind, row_len, blk, cv_mode, true, pool_rows_for(ctx, blk));
    while (lds > 65536 && blk > 64) {
      blk /= 2;
      lds = assemble_lds_bytes(precision, kind, row_len, blk, cv_mode, true, pool_rows_for(ctx, blk));
    }
    if (lds > 65536) return bad(ctx, PDD_EUNSUPPORTED, "tally rows exceed the LDS of one workgroup");
    int per_cu = 0;
    hipError_t ee = assemble_occupancy(precision, kind, cv_mode, true, blk, lds, &per_cu);
    if (ee != hipSuccess) return check_hip(ctx, ee, "occupancy query");
    grid = ctx->force_grid ? ctx->force_grid : (int64_t)ctx->cu_count * std::max(per_cu, 1);
    return PDD_OK;
  };

  int slot_guess = bc ? bc->slot_len : 0;
  if (!slot_guess) {
    for (int32_t i = 0; i < n; ++i)
      slot_guess = std::max(slot_guess, 2 * in[i].knots.m + 2 * in[i].knots.ext + 1);
  }
  int blk;
  size_t lds;
  int64_t grid;
  pdd_status st = shape(slot_guess, blk, lds, grid);
  if (st != PDD_OK) return st;
  const int64_t waves = grid * (blk / 64);
  int64_t per_ticket = ctx->force_per_ticket;
  if (per_ticket <= 0) per_ticket = std::max<int64_t>(256, (total_paths + 7 * waves - 1) / (7 * waves));

  if (!bc || !same_inst_tables(*bc, n, in, (int32_t)per_ticket, npk)) {
    if (capturing) return bad(ctx, PDD_EINVAL, "pdd_assemble_batch: tables not cached; run the batch once before capturing");
    auto fresh = std::make_unique<BatchCache>();
    fresh->per_ticket = (int32_t)per_ticket;
    fresh->npk = npk;
    int slot_len = 1;
    int64_t knots_total = 0;
    for (int32_t i = 0; i < n; ++i) {
      fresh->parts.push_back(in[i].part);
      fresh->knots.push_back(in[i].knots);
      fresh->h.push_back(in[i].run.h);
      fresh->a.push_back(in[i].coeffs.param[0]);
      fresh->inst_ids.push_back(in[i].run.instance);
      std::unique_ptr<GeoCache> g;
      st = build_geo_cache(ctx, in[i].part, in[i].knots, g);
      if (st != PDD_OK) return st;
      slot_len = std::max(slot_len, g->g.slot_len);
      fresh->knot_off.push_back(knots_total);
      knots_total += g->g.n;
      fresh->geos.push_back(std::move(g));
    }
    fresh->slot_len = slot_len;
    // concatenated knot descriptors
    if ((e = fresh->desc.reserve((size_t)knots_total * sizeof(KnotDesc))) != hipSuccess) return check_hip(ctx, e, "hipMalloc(batch desc)");
    for (int32_t i = 0; i < n; ++i) {
      const GeoCache& g = *fresh->geos[i];
      if ((e = hipMemcpy(fresh->desc.as<KnotDesc>() + fresh->knot_off[i], g.desc.ptr, (size_t)g.g.n * sizeof(KnotDesc),
                         hipMemcpyDeviceToDevice)) != hipSuccess)
        return check_hip(ctx, e, "copy batch desc");
    }
    // instance table
    std::vector<InstDesc> idesc(n);
    for (int32_t i = 0; i < n; ++i) {
      const Geometry& g = fresh->geos[i]->g;
      InstDesc d;
      std::memset(&d, 0, sizeof(d));
      d.x0 = g.x0; d.x1 = g.x1; d.y0 = g.y0; d.y1 = g.y1; d.dx = g.dx; d.dy = g.dy;
      d.h = in[i].run.h;
      d.sqrt_h = std::sqrt(in[i].run.h);
      d.a = in[i].coeffs.param[0];
      d.inv_dx = (float)(1.0 / g.dx);
      d.inv_dy = (float)(1.0 / g.dy);
      d.L = g.L;
      d.inst_id = in[i].run.instance;
      idesc[i] = d;
    }
    if ((e = fresh->insts.reserve(idesc.size() * sizeof(InstDesc))) != hipSuccess) return check_hip(ctx, e, "hipMalloc(insts)");
    if ((e = hipMemcpy(fresh->insts.ptr, idesc.data(), idesc.size() * sizeof(InstDesc), hipMemcpyHostToDevice)) != hipSuccess)
      return check_hip(ctx, e, "upload insts");
    // tickets of all instances (instance-major), cost = paths x patch area / h
    std::vector<Ticket> tk;
    std::vector<double> cost;
    for (int32_t i = 0; i < n; ++i) {
      const Geometry& g = fresh->geos[i]->g;
      fresh->ticket_off.push_back((int64_t)tk.size());
      std::vector<int32_t> tb(g.n + 1, 0);
      for (int64_t k = 0; k < g.n; ++k) {
        const int64_t N = npk[i][k];
        const int64_t c = (N + per_ticket - 1) / per_ticket;
        const double area = (double)(g.box[4 * k + 1] - g.box[4 * k]) * g.dx *
                            (double)(g.box[4 * k + 3] - g.box[4 * k + 2]) * g.dy;
        for (int64_t q = 0; q < c; ++q) {
          Ticket t;
          t.knot = (int32_t)(fresh->knot_off[i] + k);
          t.p0 = (int32_t)(N * q / c);
          t.p1 = (int32_t)(N * (q + 1) / c);
          t.inst = (uint32_t)i;
          tk.push_back(t);
          cost.push_back(area / in[i].run.h * (double)(t.p1 - t.p0));
        }
        tb[k + 1] = (int32_t)(tk.size() - fresh->ticket_off[i]);
      }
      if ((int64_t)tk.size() > INT32_MAX) return bad(ctx, PDD_EUNSUPPORTED, "too many tickets");
      fresh->n_tickets.push_back((int64_t)tk.size() - fresh->ticket_off[i]);
      auto tbd = std::make_unique<DeviceBuffer>();
      auto npd = std::make_unique<DeviceBuffer>();
      if ((e = tbd->reserve(tb.size() * 4)) != hipSuccess) return check_hip(ctx, e, "hipMalloc(ticket_begin)");
      if ((e = npd->reserve(npk[i].size() * 4)) != hipSuccess) return check_hip(ctx, e, "hipMalloc(n_paths)");
      if ((e = hipMemcpy(tbd->ptr, tb.data(), tb.size() * 4, hipMemcpyHostToDevice)) != hipSuccess) return check_hip(ctx, e, "upload ticket_begin");
      if ((e = hipMemcpy(npd->ptr, npk[i].data(), npk[i].size() * 4, hipMemcpyHostToDevice)) != hipSuccess) return check_hip(ctx, e, "upload n_paths");
      fresh->ticket_begin.push_back(std::move(tbd));
      fresh->n_paths.push_back(std::move(npd));
    }
    fresh->total_tickets = (int64_t)tk.size();
    std::vector<int32_t> order(tk.size());
    for (size_t q = 0; q < order.size(); ++q) order[q] = (int32_t)q;
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return cost[a] > cost[b]; });
    if ((e = fresh->tickets.reserve(tk.size() * sizeof(Ticket))) != hipSuccess) return check_hip(ctx, e, "hipMalloc(tickets)");
    if ((e = fresh->order.reserve(order.size() * 4)) != hipSuccess) return check_hip(ctx, e, "hipMalloc(order)");
    if ((e = hipStreamSynchronize(ctx->stream)) != hipSuccess) return check_hip(ctx, e, "hipStreamSynchronize");
    if ((e = hipMemcpy(fresh->tickets.ptr, tk.data(), tk.size() * sizeof(Ticket), hipMemcpyHostToDevice)) != hipSuccess) return check_hip(ctx, e, "upload tickets");
    if ((e = hipMemcpy(fresh->order.ptr, order.data(), order.size() * 4, hipMemcpyHostToDevice)) != hipSuccess) return check_hip(ctx, e, "upload order");
    ctx->batch = std::move(fresh);
    bc = ctx->batch.get();
  }

  st = shape(bc->slot_len, blk, lds, grid);
  if (st != PDD_OK) return st;
  const int slot_len = bc->slot_len;
  const int row_len = 4 * slot_len + EX_COUNT;
  grid = std::min<int64_t>(grid, (bc->total_tickets + blk / 64 - 1) / (blk / 64));
  grid = std::max<int64_t>(grid, 1);
  const size_t partial_bytes = (size_t)bc->total_tickets * row_len * sizeof(double);
  if (partial_bytes > ctx->partial.bytes) {
    if (capturing) return bad(ctx, PDD_EINVAL, "pdd_assemble_batch: scratch not sized; run the batch once before capturing");
    if ((e = hipStreamSynchronize(ctx->stream)) != hipSuccess) return check_hip(ctx, e, "hipStreamSynchronize");
    if ((e = ctx->partial.reserve(partial_bytes)) != hipSuccess) return check_hip(ctx, e, "hipMalloc(partial)");
  }
  if (ctx->schedule == PDD_SCHEDULE_DYNAMIC && !ctx->ticket_counter.ptr) {
    if (capturing) return bad(ctx, PDD_EINVAL, "pdd_assemble_batch: counter not allocated; run once before capturing");
    if ((e = ctx->ticket_counter.reserve(8 * sizeof(uint32_t))) != hipSuccess) return check_hip(ctx, e, "hipMalloc(counter)");
    if ((e = hipMemset(ctx->ticket_counter.ptr, 0, 8 * sizeof(uint32_t))) != hipSuccess) return check_hip(ctx, e, "hipMemset(counter)");
  }

  // patterns into the caller's arrays
  for (int32_t i = 0; i < n; ++i) {
    const GeoCache& g = *bc->geos[i];
    if ((e = hipMemcpyAsync(in[i].row_ptr, g.row_ptr.ptr, (g.g.n + 1) * 4, hipMemcpyDeviceToDevice, ctx->stream)) != hipSuccess)
      return check_hip(ctx, e, "copy row_ptr");
    if (g.g.nnz > 0 && (e = hipMemcpyAsync(in[i].col_idx, g.col_idx.ptr, g.g.nnz * 4, hipMemcpyDeviceToDevice, ctx->stream)) != hipSuccess)
      return check_hip(ctx, e, "copy col_idx");
  }

  AsmParams P;
  fill_asm_params(*bc->geos[0], i0.coeffs, i0.run, P);
  P.desc = bc->desc.as<KnotDesc>();
  P.insts = bc->insts.as<InstDesc>();
  P.tickets = bc->tickets.as<Ticket>();
  P.order = bc->order.as<int32_t>();
  P.n_tickets = (int32_t)bc->total_tickets;
  P.row_len = row_len;
  P.slot_len = slot_len;
  P.partial = ctx->partial.as<double>();
  P.u_ref = nullptr;
  P.lattice = nullptr;
  P.ticket_counter = ctx->schedule == PDD_SCHEDULE_DYNAMIC ? ctx->ticket_counter.as<uint32_t>() : nullptr;
  P.refill_min = ctx->refill_min;
  P.pool_rows = pool_rows_for(ctx, blk);

  hipEvent_t t0 = nullptr, t1 = nullptr;
  if (ctx->timing && !capturing && ctx->ev_used < 4096) {
    while ((int)ctx->ev_pool.size() < 2 * (ctx->ev_used + 1)) {
      hipEvent_t ev;
      if ((e = hipEventCreate(&ev)) != hipSuccess) return check_hip(ctx, e, "hipEventCreate");
      ctx->ev_pool.push_back(ev);
    }
    t0 = ctx->ev_pool[2 * ctx->ev_used];
    t1 = ctx->ev_pool[2 * ctx->ev_used + 1];
    if ((e = hipEventRecord(t0, ctx->stream)) != hipSuccess) return check_hip(ctx, e, "hipEventRecord");
  }
  e = launch_assemble(P, precision, (int)grid, blk, lds, ctx->stream);
  if (e != hipSuccess) return check_hip(ctx, e, "launch batched assemble");
  if (t1 && !ctx->timing_with_finalize) {
    if ((e = hipEventRecord(t1, ctx->stream)) != hipSuccess) return check_hip(ctx, e, "hipEventRecord");
    ctx->ev_used += 1;
  }

  for (int32_t i = 0; i < n; ++i) {
    const GeoCache& g = *bc->geos[i];
    FinalizeParams F{};
    F.partial = P.partial + (size_t)bc->ticket_off[i] * row_len;
    F.ticket_begin = bc->ticket_begin[i]->as<int32_t>();
    F.desc = P.desc + bc->knot_off[i];
    F.knot_ij = g.knot_ij.as<int32_t>();
    F.row_ptr = g.row_ptr.as<int32_t>();
    F.col_idx = g.col_idx.as<int32_t>();
    F.n_paths = bc->n_paths[i]->as<int32_t>();
    F.row_len = row_len;
    F.slot_len = slot_len;
    F.n = g.g.n;
    F.val = in[i].val;
    F.b = in[i].b;
    F.diag = in[i].diag;
    F.ticket_counter = (i == 0) ? P.ticket_counter : nullptr;
    e = launch_finalize(F, ctx->stream);
    if (e != hipSuccess) return check_hip(ctx, e, "launch finalize");
  }
  if (t1 && ctx->timing_with_finalize) {
    if ((e = hipEventRecord(t1, ctx->stream)) != hipSuccess) return check_hip(ctx, e, "hipEventRecord");
    ctx->ev_used += 1;
  }
  ctx->last_grid = (int)grid;
  ctx->last_block = blk;
  ctx->last_tickets = bc->total_tickets;
  return PDD_OK;
}

}  // namespace pdd

using namespace pdd;

extern "C" {

pdd_status pdd_assemble_batch(pdd_ctx* ctx, int32_t n_inst, const pdd_instance* inst) {
  if (!ctx) return PDD_EINVAL;
  if (n_inst < 1 || !inst) return bad(ctx, PDD_EINVAL, "pdd_assemble_batch: need n_inst >= 1 instances");
  return run_assemble_batch(ctx, n_inst, inst);
}

pdd_status pdd_graph_begin(pdd_ctx* ctx) {
  if (!ctx) return PDD_EINVAL;
  if (ctx->capturing) return bad(ctx, PDD_EINVAL, "pdd_graph_begin: already capturing");
  if (!ctx->stream) return bad(ctx, PDD_EINVAL, "pdd_graph_begin: capture needs a non-null stream");
  hipError_t e = hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return check_hip(ctx, e, "hipStreamBeginCapture");
  ctx->capturing = true;
  return PDD_OK;
}

pdd_status pdd_graph_end(pdd_ctx* ctx, int32_t* n_nodes) {
  if (!ctx) return PDD_EINVAL;
  if (!ctx->capturing) return bad(ctx, PDD_EINVAL, "pdd_graph_end: not capturing");
  ctx->capturing = false;
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(ctx->stream, &g);
  if (e != hipSuccess) return check_hip(ctx, e, "hipStreamEndCapture");
  if (ctx->graph_exec) { (void)hipGraphExecDestroy(ctx->graph_exec); ctx->graph_exec = nullptr; }
  if (ctx->graph) { (void)hipGraphDestroy(ctx->graph); ctx->graph = nullptr; }
  ctx->graph = g;
  if ((e = hipGraphInstantiate(&ctx->graph_exec, g, nullptr, nullptr, 0)) != hipSuccess)
    return check_hip(ctx, e, "hipGraphInstantiate");
  if (n_nodes) {
    size_t cnt = 0;
    if ((e = hipGraphGetNodes(g, nullptr, &cnt)) != hipSuccess) return check_hip(ctx, e, "hipGraphGetNodes");
    *n_nodes = (int32_t)cnt;
  }
  return PDD_OK;
}

pdd_status pdd_graph_launch(pdd_ctx* ctx) {
  if (!ctx) return PDD_EINVAL;
  if (!ctx->graph_exec) return bad(ctx, PDD_EINVAL, "pdd_graph_launch: no captured graph");
  return check_hip(ctx, hipGraphLaunch(ctx->graph_exec, ctx->stream), "hipGraphLaunch");
}

pdd_status pdd_autotune(pdd_ctx* ctx, int32_t n_inst, const pdd_instance* inst, int32_t reps, double* best_ms,
                        char* report, int32_t report_len) {
  if (!ctx) return PDD_EINVAL;
  if (n_inst < 1 || !inst || reps < 1 || !best_ms) return bad(ctx, PDD_EINVAL, "pdd_autotune: bad arguments");
  // signature of the workload: instance geometries, path counts and options
  std::string sig;
  char buf[384];
  // FNV-1a over a host array (per-knot path counts or steps)
  auto fnv = [](const void* p, size_t bytes) -> unsigned long long {
    unsigned long long hsh = 1469598103934665603ull;
    const unsigned char* c = static_cast<const unsigned char*>(p);
    for (size_t i = 0; i < bytes; ++i) hsh = (hsh ^ c[i]) * 1099511628211ull;
    return hsh;
  };
  for (int32_t i = 0; i < n_inst; ++i) {
    const pdd_instance& q = inst[i];
    unsigned long long hn = 0, hh = 0;
    if (q.run.n_paths_per_knot || q.run.h_per_knot) {
      GeoCache* gc = nullptr;
      if (get_geometry(ctx, q.part, q.knots, &gc) == PDD_OK) {
        const size_t n = (size_t)gc->g.n;
        if (q.run.n_paths_per_knot) hn = fnv(q.run.n_paths_per_knot, n * sizeof(int32_t));
        if (q.run.h_per_knot) hh = fnv(q.run.h_per_knot, n * sizeof(double));
      }
    }
    snprintf(buf, sizeof(buf), "%d:%d:%d:%d:%d:%.17g:%lld:%d:%d:%.17g:%.17g:%.17g:%.17g:%.17g:%d:%d:%.17g:%llx:%llx;",
             q.coeffs.kind, q.coeffs.lut_n, q.part.H, q.knots.m, q.knots.ext, q.run.h, (long long)q.run.n_paths,
             q.run.precision, q.run.exit_rule, q.coeffs.param[0], q.part.x0, q.part.x1, q.part.y0, q.part.y1,
             q.run.cv ? q.run.cv->mode : PDD_CV_NONE, q.run.interp, q.run.rbf_c, hn, hh);
    sig += buf;
  }
  sig += ctx->table_read_all ? "|table:all" : "|table:scan";
  auto run_once = [&]() -> pdd_status {
    if (n_inst == 1) {
      const pdd_instance& q = inst[0];
      return pdd_assemble(ctx, &q.coeffs, &q.part, &q.knots, &q.run, q.row_ptr, q.col_idx, q.val, q.b, q.diag);
    }
    return run_assemble_batch(ctx, n_inst, inst);
  };
  for (const auto& c : ctx->tune_cache) {
    if (c.sig == sig) {
      ctx->force_block = c.block; ctx->force_grid = c.grid; ctx->force_per_ticket = c.per_ticket;
      ctx->schedule = c.schedule; ctx->refill_min = c.refill; ctx->spare_rows = c.spare;
      *best_ms = c.ms;
      if (report && report_len > 0) snprintf(report, report_len, "cached: %s", c.report.c_str());
      return run_once();              // tables for the cached shape, and pdd_last_launch
    }
  }
  std::string rep;
  double best = 1e300;
  int bb = 0, bg = 0, bt = 0, bs = 0, br = 1;
  // mean device time of `reps` launches with the context's current shape:
  // the assembly kernel and the row sums after it, whose cost grows with
  // the ticket count
  auto time_shape = [&](double* ms_out) -> pdd_status {
    hipError_t e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return check_hip(ctx, e, "hipStreamSynchronize");
    const bool was = ctx->timing;
    ctx->timing = true;
    ctx->timing_with_finalize = true;
    ctx->ev_used = 0;
    pdd_status st = PDD_OK;
    for (int r = 0; r < reps && st == PDD_OK; ++r) st = run_once();
    double ms = 0.0;
    for (int r = 0; r < ctx->ev_used && st == PDD_OK; ++r) {
      float t = 0.0f;
      if ((e = hipEventSynchronize(ctx->ev_pool[2 * r + 1])) != hipSuccess)
        st = check_hip(ctx, e, "hipEventSynchronize");
      else if ((e = hipEventElapsedTime(&t, ctx->ev_pool[2 * r], ctx->ev_pool[2 * r + 1])) != hipSuccess)
        st = check_hip(ctx, e, "hipEventElapsedTime");
      ms += t;
    }
    *ms_out = ms / std::max(ctx->ev_used, 1);
    ctx->timing = was;
    ctx->timing_with_finalize = false;
    ctx->ev_used = 0;
    return st;
  };
  const int blocks[] = {256, 128};
  const int tickets[] = {256, 384, 512, 768, 1024};
  ctx->refill_min = 1;
  ctx->spare_rows = -1;
  for (int blk : blocks) {
    for (int per_cu_sub = 0; per_cu_sub < 2; ++per_cu_sub) {
      for (int ppt : tickets) {
        for (int sched = 0; sched < 2; ++sched) {
          ctx->force_block = blk;
          ctx->force_grid = 0;
          ctx->force_per_ticket = ppt;
          ctx->schedule = sched;
          pdd_status st = run_once();   // builds tables, reports the automatic grid
          if (st != PDD_OK) return st;
          int grid = ctx->last_grid;
          if (per_cu_sub) {
            // one workgroup per CU fewer than the occupancy limit
            const int per_cu = std::max(1, grid / std::max(ctx->cu_count, 1) - 1);
            grid = per_cu * ctx->cu_count;
            ctx->force_grid = grid;
            if ((st = run_once()) != PDD_OK) return st;
          }
          double ms = 0.0;
          if ((st = time_shape(&ms)) != PDD_OK) return st;
          snprintf(buf, sizeof(buf), "block %3d grid %5d tickets %7lld ppt %5d %s refill  1: %.4f ms\n",
                   ctx->last_block, ctx->last_grid, (long long)ctx->last_tickets, ppt,
                   sched ? "dynamic" : "static ", ms);
          rep += buf;
          if (ms < best) {
            best = ms;
            bb = blk; bg = ctx->force_grid; bt = ppt; bs = sched;
          }
        }
      }
    }
  }
  // deferred refill on the best shape: a wave waits until this many of its lanes are idle
  ctx->force_block = bb; ctx->force_grid = bg; ctx->force_per_ticket = bt; ctx->schedule = bs;
  for (int refill : {8, 16, 32}) {
    ctx->refill_min = refill;
    double ms = 0.0;
    pdd_status st = run_once();
    if (st != PDD_OK) return st;
    if ((st = time_shape(&ms)) != PDD_OK) return st;
    snprintf(buf, sizeof(buf), "best shape, refill %2d: %.4f ms\n", refill, ms);
    rep += buf;
    if (ms < best) { best = ms; br = refill; }
  }
  ctx->refill_min = br;
  int bt2 = bt;
  // fewer tally rows per workgroup on the best schedule, with the grid the
  // smaller LDS allows (more resident waves, which sometimes wait for a row)
  // and larger tickets, which make those waits rarer.  Both block sizes: the
  // waves the smaller LDS admits depend on the block size, and the two can
  // tie within the timing noise in the sweep above
  int bsp = -1, bb2 = bb;
  // (single-instance assemblies share rows only with tabulated coefficients)
  const bool pooled = n_inst > 1 || inst[0].coeffs.kind == PDD_COEF_LUT;
  for (int blk : {bb, bb == 256 ? 128 : 256}) {
    for (int spare : {2, 1, 0}) {
      if (!pooled) break;
      // the sweep's ticket size and the larger ones, each once
      int cands[4], nc = 0;
      cands[nc++] = bt;
      for (int p : {1024, 2048, 4096})
        if (p > bt) cands[nc++] = p;
      for (int c = 0; c < nc; ++c) {
        const int ppt = cands[c];
        ctx->force_block = blk;
        ctx->spare_rows = spare;
        ctx->force_grid = 0;
        ctx->force_per_ticket = ppt;
        double ms = 0.0;
        pdd_status st = run_once();
        if (st != PDD_OK) return st;
        if ((st = time_shape(&ms)) != PDD_OK) return st;
        snprintf(buf, sizeof(buf), "block %3d, %d spare rows, ppt %5d, grid %5d: %.4f ms\n", blk, spare, ppt,
                 ctx->last_grid, ms);
        rep += buf;
        if (ms < best) { best = ms; bsp = spare; bg = 0; bt2 = ppt; bb2 = blk; }
      }
    }
  }
  bb = bb2;
  bt = bt2;
  ctx->force_block = bb;
  ctx->force_per_ticket = bt;
  ctx->spare_rows = bsp;
  ctx->force_grid = bg;
  // one launch with the chosen settings: its tables are the cached ones (a
  // graph captured next replays them) and pdd_last_launch reports its shape
  if (pdd_status st = run_once(); st != PDD_OK) return st;
  *best_ms = best;
  TuneEntry te;
  te.sig = sig; te.block = bb; te.grid = bg; te.per_ticket = bt; te.schedule = bs; te.refill = br; te.spare = bsp;
  te.ms = best;
  te.report = rep;
  ctx->tune_cache.push_back(te);
  if (report && report_len > 0) snprintf(report, report_len, "%s", rep.c_str());
  return PDD_OK;
}

}  // extern "C"
