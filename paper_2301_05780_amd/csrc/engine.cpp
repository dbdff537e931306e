// Host engine of the assembly: run validation, ticket construction, launch
// shape, and the enqueue of the assembly and finalize kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>

#include "context.h"
#include "plan.h"
#include "rbf.h"

namespace pdd {

namespace {

pdd_status bad(pdd_ctx* ctx, pdd_status st, const char* msg) {
  ctx->err = msg;
  return st;
}

}  // namespace

pdd_status validate_run(pdd_ctx* ctx, const pdd_coeffs& c, const pdd_run& r) {
  if (c.kind < PDD_COEF_POISSON || c.kind > PDD_COEF_EQ43)
    return bad(ctx, PDD_EINVAL, "coeffs.kind: unknown coefficient family");
  if (c.kind == PDD_COEF_AMPLITUDE && !(c.param[0] >= 0.0 && c.param[0] < 1.0))
    return bad(ctx, PDD_EINVAL, "coeffs.param[0]: amplitude must lie in [0, 1)");
  if (c.kind == PDD_COEF_LUT && (!c.lut || c.lut_n < 2 || c.lut_n > 65536))
    return bad(ctx, PDD_EINVAL, "coeffs: LUT kind needs a device table and 2 <= lut_n <= 65536");
  if (c.kind == PDD_COEF_LUT && (reinterpret_cast<uintptr_t>(c.lut) & 15u) != 0)
    return bad(ctx, PDD_EINVAL, "coeffs: the LUT must be 16-byte aligned");
  if (r.precision != PDD_FP64_SAME_STREAM && r.precision != PDD_FP32_PRODUCTION)
    return bad(ctx, PDD_EINVAL, "run.precision: unknown precision mode");
  if (r.exit_rule != PDD_EXIT_NAIVE && r.exit_rule != PDD_EXIT_GM)
    return bad(ctx, PDD_EINVAL, "run.exit_rule: unknown exit rule");
  if (!(r.h > 0.0) || !std::isfinite(r.h)) return bad(ctx, PDD_EINVAL, "run.h: need a finite h > 0");
  if (!r.n_paths_per_knot && (r.n_paths < 1 || r.n_paths > INT32_MAX))
    return bad(ctx, PDD_EINVAL, "run.n_paths: need 1 <= n_paths <= 2^31 - 1");
  if (r.dump_paths < 0 || (r.dump_paths > 0 && !r.dump))
    return bad(ctx, PDD_EINVAL, "run.dump_paths: need dump_paths >= 0 and a dump buffer when > 0");
  if (r.interp != PDD_INTERP_HAT && r.interp != PDD_INTERP_RBF_IMQ)
    return bad(ctx, PDD_EINVAL, "run.interp: unknown interpolation");
  if (r.interp == PDD_INTERP_RBF_IMQ) {
    if (!(r.rbf_c > 0.0) || !std::isfinite(r.rbf_c)) return bad(ctx, PDD_EINVAL, "run.rbf_c: need a finite shape parameter > 0");
    if (r.u_ref) return bad(ctx, PDD_EUNSUPPORTED, "run.u_ref: not available with RBF interpolation");
    if (r.cv && r.cv->mode == PDD_CV_NETWORK)
      return bad(ctx, PDD_EUNSUPPORTED, "run.cv: RBF interpolation takes no control variate or the gradient table");
  }
  if (r.cv) {
    const pdd_cv& cv = *r.cv;
    if (cv.mode < PDD_CV_NONE || cv.mode > PDD_CV_GRAD_LUT) return bad(ctx, PDD_EINVAL, "run.cv.mode: unknown mode");
    if (cv.mode == PDD_CV_NETWORK && !cv.params) return bad(ctx, PDD_EINVAL, "run.cv: network mode needs params");
    if (cv.mode == PDD_CV_GRAD_LUT && (!cv.grad_lut || cv.lut_n < 2 || cv.lut_n > 65536))
      return bad(ctx, PDD_EINVAL, "run.cv: grad-table mode needs a table and 2 <= lut_n <= 65536");
    if (cv.mode == PDD_CV_GRAD_LUT && (reinterpret_cast<uintptr_t>(cv.grad_lut) & 7u) != 0)
      return bad(ctx, PDD_EINVAL, "run.cv: the gradient table must be 8-byte aligned");
    if (cv.mode == PDD_CV_GRAD_LUT && r.precision == PDD_FP32_PRODUCTION && cv.lut_n > 23170)
      return bad(ctx, PDD_EUNSUPPORTED, "run.cv: float32 runs read the gradient table with 32-bit offsets (lut_n <= 23170)");
    if (cv.mode != PDD_CV_NONE && (c.kind == PDD_COEF_CONSTSOL || c.kind == PDD_COEF_EXITTIME))
      return bad(ctx, PDD_EUNSUPPORTED, "run.cv: control variates are built for the poisson, varcoef, amplitude, LUT and eq43 families");
  }
  return PDD_OK;
}

// The table-wide sigma maxima of the Gobet-Menozzi bound; `scanned`: the
// table scan of prepare_lut_cells has gathered them already (the float32
// table assembly).
pdd_status prepare_lut_bound(pdd_ctx* ctx, const pdd_coeffs& co, const pdd_run& run, AsmParams& P, bool capturing,
                             bool scanned) {
  if (co.kind != PDD_COEF_LUT || run.exit_rule != PDD_EXIT_GM) return PDD_OK;
  hipError_t e;
  if (!ctx->lut_max.ptr) {
    if (capturing) return bad(ctx, PDD_EINVAL, "LUT bound scratch not allocated; run the same call once before capturing");
    if ((e = ctx->lut_max.reserve(4 * sizeof(uint32_t))) != hipSuccess) return check_hip(ctx, e, "hipMalloc(lut bound)");
  }
  if (!scanned && (e = launch_lut_bound(co.lut, co.lut_n, ctx->lut_max.as<uint32_t>(), ctx->stream)) != hipSuccess)
    return check_hip(ctx, e, "launch LUT bound");
  P.coef.lut_max = ctx->lut_max.as<uint32_t>();
  return PDD_OK;
}

bool uses_lut_cells(const pdd_coeffs& co, const pdd_run& run) {
  if (co.kind != PDD_COEF_LUT || run.precision != PDD_FP32_PRODUCTION) return false;
  return !(run.cv && run.cv->mode == PDD_CV_NETWORK);     // that kernel reads the node table per lane
}

// The cell-major copy of the table and its layout word.  *lane_layout tells
// whether the copy holds only the varying fields: read back from the device
// (waiting for the stream) on eager calls, the last eager call's answer
// while a graph is captured (the kernels read the layout word themselves,
// so a stale answer picks the slower kernel, never a wrong result).
pdd_status prepare_lut_cells(pdd_ctx* ctx, const pdd_coeffs& co, const pdd_run& run, bool capturing, bool* lane_layout) {
  *lane_layout = false;
  if (!uses_lut_cells(co, run)) return PDD_OK;
  const size_t bytes = (size_t)(co.lut_n - 1) * (size_t)(co.lut_n - 1) * 128;
  // the float32 kernels address the copy with 32-bit byte offsets
  if (bytes >= ((size_t)1 << 32))
    return bad(ctx, PDD_EUNSUPPORTED, "LUT too large for the float32 cell-major copy (below 4 GiB, lut_n <= 5793)");
  hipError_t e;
  if (ctx->lut_cells.bytes < bytes) {
    if (capturing) return bad(ctx, PDD_EINVAL, "LUT cell table not allocated; run the same call once before capturing");
    if ((e = hipStreamSynchronize(ctx->stream)) != hipSuccess) return check_hip(ctx, e, "hipStreamSynchronize");
    if ((e = ctx->lut_cells.reserve(bytes)) != hipSuccess) return check_hip(ctx, e, "hipMalloc(lut cells)");
  }
  if (!ctx->lut_info.ptr) {
    if (capturing) return bad(ctx, PDD_EINVAL, "LUT layout word not allocated; run the same call once before capturing");
    if ((e = ctx->lut_info.reserve(16 * sizeof(uint32_t))) != hipSuccess) return check_hip(ctx, e, "hipMalloc(lut info)");
  }
  const bool gm = run.exit_rule == PDD_EXIT_GM;
  if (gm && !ctx->lut_max.ptr) {
    if (capturing) return bad(ctx, PDD_EINVAL, "LUT bound scratch not allocated; run the same call once before capturing");
    if ((e = ctx->lut_max.reserve(4 * sizeof(uint32_t))) != hipSuccess) return check_hip(ctx, e, "hipMalloc(lut bound)");
  }
  if ((e = launch_lut_cells(co.lut, co.lut_n, ctx->table_read_all, ctx->lut_info.as<uint32_t>(),
                            gm ? ctx->lut_max.as<uint32_t>() : nullptr, ctx->lut_cells.as<float4>(), ctx->stream)) !=
      hipSuccess)
    return check_hip(ctx, e, "launch LUT cells");
  if (!capturing) {
    uint32_t lay = 0u;
    if ((e = hipMemcpyAsync(&lay, ctx->lut_info.as<uint32_t>() + 1, sizeof(lay), hipMemcpyDeviceToHost, ctx->stream)) !=
        hipSuccess)
      return check_hip(ctx, e, "read LUT layout");
    if ((e = hipStreamSynchronize(ctx->stream)) != hipSuccess) return check_hip(ctx, e, "hipStreamSynchronize");
    ctx->lut_lane = (lay & LUT_LANE_READ) != 0u;
  }
  *lane_layout = ctx->lut_lane;
  return PDD_OK;
}

void fill_asm_params(const GeoCache& gcr, const pdd_coeffs& co, const pdd_run& run, AsmParams& P) {
  const Geometry& g = gcr.g;
  std::memset(&P, 0, sizeof(P));
  P.desc = gcr.desc.as<KnotDesc>();
  P.L = g.L;
  P.key0 = (uint32_t)(run.seed & 0xFFFFFFFFu);
  P.key1 = (uint32_t)(run.seed >> 32);
  P.exit_rule = run.exit_rule;
  P.h = run.h;
  P.sqrt_h = std::sqrt(run.h);
  P.x0 = g.x0; P.x1 = g.x1; P.y0 = g.y0; P.y1 = g.y1; P.dx = g.dx; P.dy = g.dy;
  P.inv_dx = (float)(1.0 / g.dx);
  P.inv_dy = (float)(1.0 / g.dy);
  P.coef.kind = co.kind;
  P.coef.lut_n = co.lut_n;
  P.coef.a = co.param[0];
  P.coef.lut = co.lut;
  P.coef.x0 = g.x0; P.coef.x1 = g.x1; P.coef.y0 = g.y0; P.coef.y1 = g.y1;
  P.coef.x0f = (float)g.x0;
  P.coef.y0f = (float)g.y0;
  if (co.kind == PDD_COEF_LUT) {
    P.coef.lut_sx = (float)((co.lut_n - 1) / (g.x1 - g.x0));
    P.coef.lut_sy = (float)((co.lut_n - 1) / (g.y1 - g.y0));
  }
  P.u_ref = run.u_ref;
  P.lattice = gcr.lattice.as<int32_t>();
  P.cv_mode = run.cv ? run.cv->mode : PDD_CV_NONE;
  if (P.cv_mode == PDD_CV_NETWORK) P.cv_params = run.cv->params;
  if (P.cv_mode == PDD_CV_GRAD_LUT) {
    P.cv_lut = run.cv->grad_lut;
    P.cv_lut_n = run.cv->lut_n;
    P.cv_lut_sx = (float)((run.cv->lut_n - 1) / (g.x1 - g.x0));
    P.cv_lut_sy = (float)((run.cv->lut_n - 1) / (g.y1 - g.y0));
  }
}

// The inverse table of the RBF stencil matrices for this geometry and shape
// parameter (built on the host and uploaded once per combination).
pdd_status prepare_rbf(pdd_ctx* ctx, const Geometry& g, const pdd_run& run, AsmParams& P, bool capturing) {
  RbfCache* rc = ctx->rbf.get();
  if (!rc || rc->slot_len != g.slot_len || rc->dx != g.dx || rc->dy != g.dy || rc->c != run.rbf_c) {
    if (capturing) return bad(ctx, PDD_EINVAL, "pdd_assemble: RBF table not cached; run the same call once before capturing");
    auto fresh = std::make_unique<RbfCache>();
    fresh->slot_len = g.slot_len;
    fresh->dx = g.dx;
    fresh->dy = g.dy;
    fresh->c = run.rbf_c;
    std::vector<double> tab;
    if (!rbf_inverse_table(g.slot_len, g.dx, g.dy, run.rbf_c, tab, fresh->half))
      return bad(ctx, PDD_EINVAL, "run.rbf_c: a stencil's interpolation matrix is not positive definite in float64 "
                                  "(shape parameter too large for the stencil)");
    hipError_t e;
    if ((e = fresh->tab.reserve(tab.size() * sizeof(double))) != hipSuccess) return check_hip(ctx, e, "hipMalloc(rbf table)");
    if ((e = hipStreamSynchronize(ctx->stream)) != hipSuccess) return check_hip(ctx, e, "hipStreamSynchronize");
    if ((e = hipMemcpy(fresh->tab.ptr, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice)) != hipSuccess)
      return check_hip(ctx, e, "upload rbf table");
    ctx->rbf = std::move(fresh);
    rc = ctx->rbf.get();
  }
  P.rbf_inv = rc->tab.as<double>();
  P.rbf_half = rc->half;
  P.rbf_c2 = run.rbf_c * run.rbf_c;
  return PDD_OK;
}

pdd_status run_assemble(pdd_ctx* ctx, const AssembleJob& job) {
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return check_hip(ctx, e, "hipSetDevice");
  GeoCache* gc = nullptr;
  pdd_status st = get_geometry(ctx, job.part, job.knots, &gc);
  if (st != PDD_OK) return st;
  const Geometry& g = gc->g;
  const pdd_run& run = job.run;
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  const bool capturing = hipStreamIsCapturing(ctx->stream, &cap) == hipSuccess && cap == hipStreamCaptureStatusActive;

  // paths per knot
  std::vector<int32_t> npk(g.n);
  int64_t total = 0;
  for (int64_t k = 0; k < g.n; ++k) {
    const int64_t v = run.n_paths_per_knot ? run.n_paths_per_knot[k] : run.n_paths;
    if (v < 1 || v > INT32_MAX) return bad(ctx, PDD_EINVAL, "run.n_paths_per_knot: entries must be >= 1");
    npk[k] = (int32_t)v;
    total += v;
  }
  // per-knot time steps (eq. 40)
  std::vector<double> hk;
  if (run.h_per_knot) {
    hk.assign(run.h_per_knot, run.h_per_knot + g.n);
    for (double v : hk)
      if (!(v > 0.0) || !std::isfinite(v)) return bad(ctx, PDD_EINVAL, "run.h_per_knot: entries must be finite and > 0");
  }
  if (run.u_ref) {
    if (!gc->lattice.ptr && capturing) return bad(ctx, PDD_EINVAL, "pdd_assemble: lattice table not cached before capture");
    st = get_lattice(ctx, gc);
    if (st != PDD_OK) return st;
  }

  // float32 table: its cell copy first, whose layout picks the kernel
  bool lane_layout = false;
  if ((st = prepare_lut_cells(ctx, job.coeffs, run, capturing, &lane_layout)) != PDD_OK) return st;
  const bool rbf = run.interp == PDD_INTERP_RBF_IMQ;
  const bool lane_kernel = lane_layout && !rbf && hk.empty();

  // launch shape
  const int slot_len = g.slot_len;
  const int row_len = 4 * slot_len + EX_COUNT;
  const int cv_mode = run.cv ? run.cv->mode : PDD_CV_NONE;
  int block = ctx->force_block ? ctx->force_block : 256;
  // the tally rows of a workgroup: a shared pool for the table family (spare
  // rows as set on the context), two per wave otherwise
  auto rows_for = [&](int blk) { return job.coeffs.kind == PDD_COEF_LUT ? pool_rows_for(ctx, blk) : 2 * (blk / 64); };
  size_t lds = assemble_lds_bytes(run.precision, job.coeffs.kind, row_len, block, cv_mode, false, rows_for(block),
                                  lane_kernel);
  while (lds > 65536 && block > 64) {
    block /= 2;
    lds = assemble_lds_bytes(run.precision, job.coeffs.kind, row_len, block, cv_mode, false, rows_for(block),
                             lane_kernel);
  }
  if (lds > 65536) return bad(ctx, PDD_EUNSUPPORTED, "tally rows exceed the LDS of one workgroup");
  int per_cu = 0;
  e = rbf ? assemble_occupancy_rbf(run.precision, job.coeffs.kind, cv_mode, block, lds, &per_cu)
          : assemble_occupancy(run.precision, job.coeffs.kind, cv_mode, false, block, lds, &per_cu, !hk.empty(),
                               lane_kernel);
  if (e != hipSuccess) return check_hip(ctx, e, "occupancy query");
  per_cu = std::max(per_cu, 1);
  int64_t grid = ctx->force_grid ? ctx->force_grid : (int64_t)ctx->cu_count * per_cu;
  const int64_t waves = grid * (block / 64);

  // Tabulated coefficients make the path memory-bound on table gathers: order
  // the tickets spatially (subdomains in Morton order) and give each XCD a
  // contiguous share, so the workgroups that share an L2 gather from one
  // neighbourhood; cut knots into more tickets so that the share in flight on
  // one XCD covers few knots.  Otherwise: about seven tickets per wave, longest
  // expected first (the static stride stays balanced); at least 256 paths each.
  const bool spatial = job.coeffs.kind == PDD_COEF_LUT;
  int64_t per_ticket = ctx->force_per_ticket;
  if (per_ticket <= 0) {
    const int64_t per_wave = spatial ? 256 : 7;
    per_ticket = std::max<int64_t>(256, (total + per_wave * waves - 1) / (per_wave * waves));
  }

  // tickets (cached while geometry, path counts, ticket size and order repeat)
  TicketCache* tc = ctx->tickets.get();
  if (!tc || tc->geo != gc || tc->per_ticket != per_ticket || tc->npk != npk || tc->inst != run.instance ||
      tc->spatial != spatial || tc->hk != hk) {
    if (capturing) return bad(ctx, PDD_EINVAL, "pdd_assemble: tables not cached; run the same call once before capturing");
    auto fresh = std::make_unique<TicketCache>();
    fresh->geo = gc;
    fresh->npk = npk;
    fresh->per_ticket = (int32_t)per_ticket;
    fresh->inst = run.instance;
    TicketPlan plan;
    std::string err;
    fresh->hk = hk;
    if ((st = plan_tickets(g, npk, per_ticket, spatial, run.instance, plan, err, hk.empty() ? nullptr : hk.data())) !=
        PDD_OK)
      return bad(ctx, st, err.c_str());
    const std::vector<Ticket>& tk = plan.tickets;
    const std::vector<int32_t>& tb = plan.begin;
    const std::vector<int32_t>& order = plan.order;
    fresh->cum_cost = plan.cum_cost;
    fresh->spatial = spatial;
    fresh->n_tickets = (int64_t)tk.size();
    if ((e = fresh->tickets.reserve(tk.size() * sizeof(Ticket))) != hipSuccess) return check_hip(ctx, e, "hipMalloc(tickets)");
    if ((e = fresh->order.reserve(order.size() * 4)) != hipSuccess) return check_hip(ctx, e, "hipMalloc(order)");
    if ((e = fresh->ticket_begin.reserve(tb.size() * 4)) != hipSuccess) return check_hip(ctx, e, "hipMalloc(ticket_begin)");
    if ((e = fresh->n_paths.reserve(npk.size() * 4)) != hipSuccess) return check_hip(ctx, e, "hipMalloc(n_paths)");
    // the stream may still read the previous cache's arrays
    if ((e = hipStreamSynchronize(ctx->stream)) != hipSuccess) return check_hip(ctx, e, "hipStreamSynchronize");
    if ((e = hipMemcpy(fresh->tickets.ptr, tk.data(), tk.size() * sizeof(Ticket), hipMemcpyHostToDevice)) != hipSuccess) return check_hip(ctx, e, "upload tickets");
    if ((e = hipMemcpy(fresh->order.ptr, order.data(), order.size() * 4, hipMemcpyHostToDevice)) != hipSuccess) return check_hip(ctx, e, "upload order");
    if ((e = hipMemcpy(fresh->ticket_begin.ptr, tb.data(), tb.size() * 4, hipMemcpyHostToDevice)) != hipSuccess) return check_hip(ctx, e, "upload ticket_begin");
    if ((e = hipMemcpy(fresh->n_paths.ptr, npk.data(), npk.size() * 4, hipMemcpyHostToDevice)) != hipSuccess) return check_hip(ctx, e, "upload n_paths");
    if (!hk.empty()) {
      if ((e = fresh->h_knot.reserve(hk.size() * sizeof(double))) != hipSuccess) return check_hip(ctx, e, "hipMalloc(h_knot)");
      if ((e = hipMemcpy(fresh->h_knot.ptr, hk.data(), hk.size() * sizeof(double), hipMemcpyHostToDevice)) != hipSuccess)
        return check_hip(ctx, e, "upload h_knot");
    }
    ctx->tickets = std::move(fresh);
    tc = ctx->tickets.get();
  }
  const int64_t need_waves = tc->n_tickets;
  grid = std::min<int64_t>(grid, (need_waves + block / 64 - 1) / (block / 64));
  grid = std::max<int64_t>(grid, 1);

  // XCD split of the spatial order (at least one workgroup per XCD): XCD x,
  // holding ceil((grid - x) / 8) of the workgroups, gets a contiguous share
  // of the order with the same fraction of the expected cost; its waves take
  // the share in a fixed stride (static) or from the XCD's own counter
  // (dynamic)
  const bool split_xcd = tc->spatial && grid >= 8;
  if (split_xcd && tc->xcd_grid != (int32_t)grid) {
    if (capturing) return bad(ctx, PDD_EINVAL, "pdd_assemble: XCD split not cached for this grid; run once before capturing");
    int32_t xb[9];
    xcd_split(tc->cum_cost, tc->n_tickets, grid, xb);
    if ((e = tc->xcd_begin.reserve(sizeof(xb))) != hipSuccess) return check_hip(ctx, e, "hipMalloc(xcd split)");
    if ((e = hipStreamSynchronize(ctx->stream)) != hipSuccess) return check_hip(ctx, e, "hipStreamSynchronize");
    if ((e = hipMemcpy(tc->xcd_begin.ptr, xb, sizeof(xb), hipMemcpyHostToDevice)) != hipSuccess)
      return check_hip(ctx, e, "upload xcd split");
    tc->xcd_grid = (int32_t)grid;
  }

  const size_t partial_bytes = (size_t)tc->n_tickets * row_len * sizeof(double);
  if (partial_bytes > ctx->partial.bytes) {
    if (capturing) return bad(ctx, PDD_EINVAL, "pdd_assemble: scratch not sized; run the same call once before capturing");
    if ((e = hipStreamSynchronize(ctx->stream)) != hipSuccess) return check_hip(ctx, e, "hipStreamSynchronize");
    if ((e = ctx->partial.reserve(partial_bytes)) != hipSuccess) return check_hip(ctx, e, "hipMalloc(partial)");
  }

  // pattern into the caller's arrays
  if ((e = hipMemcpyAsync(job.row_ptr, gc->row_ptr.ptr, (g.n + 1) * 4, hipMemcpyDeviceToDevice, ctx->stream)) != hipSuccess)
    return check_hip(ctx, e, "copy row_ptr");
  if (g.nnz > 0 && (e = hipMemcpyAsync(job.col_idx, gc->col_idx.ptr, g.nnz * 4, hipMemcpyDeviceToDevice, ctx->stream)) != hipSuccess)
    return check_hip(ctx, e, "copy col_idx");

  AsmParams P;
  fill_asm_params(*gc, job.coeffs, run, P);
  P.tickets = tc->tickets.as<Ticket>();
  P.order = tc->order.as<int32_t>();
  P.h_knot = hk.empty() ? nullptr : tc->h_knot.as<double>();
  P.n_tickets = (int32_t)tc->n_tickets;
  P.xcd_begin = split_xcd ? tc->xcd_begin.as<int32_t>() : nullptr;
  P.refill_min = ctx->refill_min;
  P.pool_rows = rows_for(block);
  P.row_len = row_len;
  P.slot_len = slot_len;
  P.partial = ctx->partial.as<double>();
  P.dump_paths = run.dump_paths;
  P.dump = run.dump_paths > 0 ? run.dump : nullptr;
  P.ticket_counter = nullptr;
  if ((st = prepare_lut_bound(ctx, job.coeffs, run, P, capturing, uses_lut_cells(job.coeffs, run))) != PDD_OK)
    return st;
  if (uses_lut_cells(job.coeffs, run)) {
    P.coef.cells = ctx->lut_cells.as<float4>();
    P.coef.lut_info = ctx->lut_info.as<uint32_t>();
  }
  P.table_lane = lane_kernel ? 1 : 0;
  if (rbf && (st = prepare_rbf(ctx, g, run, P, capturing)) != PDD_OK) return st;
  if (ctx->schedule == PDD_SCHEDULE_DYNAMIC) {
    if (!ctx->ticket_counter.ptr) {
      if (capturing) return bad(ctx, PDD_EINVAL, "pdd_assemble: counter not allocated; run once before capturing");
      if ((e = ctx->ticket_counter.reserve(8 * sizeof(uint32_t))) != hipSuccess) return check_hip(ctx, e, "hipMalloc(counter)");
      if ((e = hipMemset(ctx->ticket_counter.ptr, 0, 8 * sizeof(uint32_t))) != hipSuccess) return check_hip(ctx, e, "hipMemset(counter)");
    }
    P.ticket_counter = ctx->ticket_counter.as<uint32_t>();
  }

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
  e = rbf ? launch_assemble_rbf(P, run.precision, (int)grid, block, lds, ctx->stream)
          : launch_assemble(P, run.precision, (int)grid, block, lds, ctx->stream);
  if (e != hipSuccess) return check_hip(ctx, e, "launch assemble");
  if (t1 && !ctx->timing_with_finalize) {
    if ((e = hipEventRecord(t1, ctx->stream)) != hipSuccess) return check_hip(ctx, e, "hipEventRecord");
    ctx->ev_used += 1;
  }

  FinalizeParams F{};
  F.partial = P.partial;
  F.ticket_begin = tc->ticket_begin.as<int32_t>();
  F.desc = P.desc;
  F.knot_ij = gc->knot_ij.as<int32_t>();
  F.row_ptr = gc->row_ptr.as<int32_t>();
  F.col_idx = gc->col_idx.as<int32_t>();
  F.n_paths = tc->n_paths.as<int32_t>();
  F.row_len = row_len;
  F.slot_len = slot_len;
  F.n = g.n;
  F.val = job.val;
  F.b = job.b;
  F.diag = job.diag;
  F.ticket_counter = P.ticket_counter;
  F.rbf_inv = P.rbf_inv;
  F.rbf_half = P.rbf_half;
  e = launch_finalize(F, ctx->stream);
  if (e != hipSuccess) return check_hip(ctx, e, "launch finalize");
  if (t1 && ctx->timing_with_finalize) {
    if ((e = hipEventRecord(t1, ctx->stream)) != hipSuccess) return check_hip(ctx, e, "hipEventRecord");
    ctx->ev_used += 1;
  }
  ctx->last_grid = (int)grid;
  ctx->last_block = block;
  ctx->last_tickets = tc->n_tickets;
  return PDD_OK;
}

}  // namespace pdd
