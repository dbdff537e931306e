// C ABI of libpdd: context, validation, geometry/ticket caches and launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "context.h"
#include "geometry.h"
#include "spectral.h"
#include "kernels.h"
#include "mlp.h"
#include "plan.h"
#include "rbf.h"

using namespace pdd;

namespace {

thread_local std::string g_err;   // message of calls that have no context

pdd_status fail(pdd_ctx* ctx, pdd_status st, const std::string& msg) {
  if (ctx) ctx->err = msg; else g_err = msg;
  return st;
}

bool same_part(const pdd_partition& a, const pdd_partition& b) {
  return a.x0 == b.x0 && a.x1 == b.x1 && a.y0 == b.y0 && a.y1 == b.y1 && a.H == b.H;
}

}  // namespace

namespace pdd {

DeviceBuffer::~DeviceBuffer() { release(); }
void DeviceBuffer::release() {
  if (ptr) (void)hipFree(ptr);
  ptr = nullptr;
  bytes = 0;
}
hipError_t DeviceBuffer::reserve(size_t want) {
  if (want <= bytes) return hipSuccess;
  release();
  hipError_t e = hipMalloc(&ptr, want);
  if (e != hipSuccess) { ptr = nullptr; return e; }
  bytes = want;
  return hipSuccess;
}

pdd_status check_hip(pdd_ctx* ctx, hipError_t e, const char* what) {
  if (e == hipSuccess) return PDD_OK;
  ctx->err = std::string(what) + ": " + hipGetErrorString(e);
  return (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) ? PDD_ENOMEM : PDD_EDEVICE;
}

// Geometry of (part, knots), built on the host and uploaded.
pdd_status build_geo_cache(pdd_ctx* ctx, const pdd_partition& part, const pdd_knots& kn,
                           std::unique_ptr<GeoCache>& out) {
  auto gc = std::make_unique<GeoCache>();
  gc->part = part;
  gc->kn = kn;
  std::string err;
  pdd_status st = build_geometry(part, kn, gc->g, err);
  if (st != PDD_OK) return fail(ctx, st, err);
  const Geometry& g = gc->g;
  if ((int64_t)g.slot_len * 4 + EX_COUNT > 8000)
    return fail(ctx, PDD_EUNSUPPORTED, "stencils too long for the LDS tally row (reduce m or ext)");

  std::vector<KnotDesc> desc(g.n);
  std::vector<int32_t> ij(2 * g.n);
  for (int64_t k = 0; k < g.n; ++k) {
    KnotDesc d;
    std::memset(&d, 0, sizeof(d));
    d.sx = g.x0 + (double)g.ix[k] * g.dx;
    d.sy = g.y0 + (double)g.iy[k] * g.dy;
    d.bmask = 0;
    for (int o = 0; o < 4; ++o) {
      SideInfo s = g.side(k, o);
      d.line[o] = s.vertical ? g.x0 + (double)s.at * g.dx : g.y0 + (double)s.at * g.dy;
      d.at[o] = s.at;
      d.clo[o] = s.clo;
      d.chi[o] = s.chi;
      if (s.boundary) d.bmask |= 1 << o;
    }
    d.knot = (int32_t)k;
    desc[k] = d;
    ij[2 * k] = g.ix[k];
    ij[2 * k + 1] = g.iy[k];
  }
  hipError_t e;
  if ((e = gc->desc.reserve(desc.size() * sizeof(KnotDesc))) != hipSuccess) return check_hip(ctx, e, "hipMalloc(desc)");
  if ((e = gc->knot_ij.reserve(ij.size() * 4)) != hipSuccess) return check_hip(ctx, e, "hipMalloc(knot_ij)");
  if ((e = gc->row_ptr.reserve(g.row_ptr.size() * 4)) != hipSuccess) return check_hip(ctx, e, "hipMalloc(row_ptr)");
  if ((e = gc->col_idx.reserve(std::max<size_t>(1, g.col_idx.size()) * 4)) != hipSuccess) return check_hip(ctx, e, "hipMalloc(col_idx)");
  // synchronous uploads: the host vectors die at the end of this function
  if ((e = hipMemcpy(gc->desc.ptr, desc.data(), desc.size() * sizeof(KnotDesc), hipMemcpyHostToDevice)) != hipSuccess) return check_hip(ctx, e, "upload desc");
  if ((e = hipMemcpy(gc->knot_ij.ptr, ij.data(), ij.size() * 4, hipMemcpyHostToDevice)) != hipSuccess) return check_hip(ctx, e, "upload knot_ij");
  if ((e = hipMemcpy(gc->row_ptr.ptr, g.row_ptr.data(), g.row_ptr.size() * 4, hipMemcpyHostToDevice)) != hipSuccess) return check_hip(ctx, e, "upload row_ptr");
  if (!g.col_idx.empty() && (e = hipMemcpy(gc->col_idx.ptr, g.col_idx.data(), g.col_idx.size() * 4, hipMemcpyHostToDevice)) != hipSuccess) return check_hip(ctx, e, "upload col_idx");
  out = std::move(gc);
  return PDD_OK;
}

bool same_geometry(const GeoCache& gc, const pdd_partition& part, const pdd_knots& kn) {
  return same_part(gc.part, part) && gc.kn.m == kn.m && gc.kn.ext == kn.ext;
}

// Cached geometry of (part, knots) for single-instance calls (up to 8 kept).
pdd_status get_geometry(pdd_ctx* ctx, const pdd_partition& part, const pdd_knots& kn, GeoCache** out) {
  for (auto& gc : ctx->geo) {
    if (same_geometry(*gc, part, kn)) {
      *out = gc.get();
      return PDD_OK;
    }
  }
  std::unique_ptr<GeoCache> gc;
  pdd_status st = build_geo_cache(ctx, part, kn, gc);
  if (st != PDD_OK) return st;
  if (ctx->geo.size() >= 8) {
    // the stream may still read the evicted arrays
    hipError_t e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return check_hip(ctx, e, "hipStreamSynchronize");
    ctx->geo.erase(ctx->geo.begin());
  }
  ctx->geo.push_back(std::move(gc));
  *out = ctx->geo.back().get();
  return PDD_OK;
}

pdd_status get_lattice(pdd_ctx* ctx, GeoCache* gc) {
  if (gc->lattice.ptr) return PDD_OK;
  hipError_t e = gc->lattice.reserve(gc->g.index.size() * 4);
  if (e != hipSuccess) return check_hip(ctx, e, "hipMalloc(lattice)");
  e = hipMemcpy(gc->lattice.ptr, gc->g.index.data(), gc->g.index.size() * 4, hipMemcpyHostToDevice);
  return check_hip(ctx, e, "upload lattice");
}

}  // namespace pdd

extern "C" {

pdd_status pdd_create(pdd_ctx** out, int32_t device, void* stream) {
  if (!out) return fail(nullptr, PDD_EINVAL, "pdd_create: null output pointer");
  *out = nullptr;
  int count = 0;
  hipError_t e = hipGetDeviceCount(&count);
  if (e != hipSuccess || count == 0) return fail(nullptr, PDD_EDEVICE, "pdd_create: no HIP device");
  if (device < 0 || device >= count) return fail(nullptr, PDD_EINVAL, "pdd_create: device index out of range");
  e = hipSetDevice(device);
  if (e != hipSuccess) return fail(nullptr, PDD_EDEVICE, std::string("hipSetDevice: ") + hipGetErrorString(e));
  hipDeviceProp_t prop;
  e = hipGetDeviceProperties(&prop, device);
  if (e != hipSuccess) return fail(nullptr, PDD_EDEVICE, std::string("hipGetDeviceProperties: ") + hipGetErrorString(e));
  // the device's copy of pdd_solve_noalloc's static scratch (once per device)
  e = solve_noalloc_setup(device);
  if (e != hipSuccess) return fail(nullptr, PDD_EDEVICE, std::string("hipGetSymbolAddress(solve scratch): ") + hipGetErrorString(e));
  pdd_ctx* ctx = new (std::nothrow) pdd_ctx();
  if (!ctx) return fail(nullptr, PDD_ENOMEM, "pdd_create: out of host memory");
  ctx->device = device;
  ctx->stream = reinterpret_cast<hipStream_t>(stream);
  ctx->cu_count = prop.multiProcessorCount;
  ctx->arch = prop.gcnArchName;
  *out = ctx;
  return PDD_OK;
}

void pdd_destroy(pdd_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  delete ctx;
}

pdd_status pdd_set_stream(pdd_ctx* ctx, void* stream) {
  if (!ctx) return fail(nullptr, PDD_EINVAL, "pdd_set_stream: null context");
  ctx->stream = reinterpret_cast<hipStream_t>(stream);
  return PDD_OK;
}

pdd_status pdd_sync(pdd_ctx* ctx) {
  if (!ctx) return fail(nullptr, PDD_EINVAL, "pdd_sync: null context");
  return check_hip(ctx, hipStreamSynchronize(ctx->stream), "hipStreamSynchronize");
}

const char* pdd_last_error(const pdd_ctx* ctx) {
  return ctx ? ctx->err.c_str() : g_err.c_str();
}

pdd_status pdd_pattern(const pdd_partition* part, const pdd_knots* knots, int64_t* n, int64_t* nnz,
                       int32_t* row_ptr, int32_t* col_idx) {
  if (!part || !knots || !n || !nnz) return fail(nullptr, PDD_EINVAL, "pdd_pattern: null argument");
  Geometry g;
  std::string err;
  pdd_status st = build_geometry(*part, *knots, g, err);
  if (st != PDD_OK) return fail(nullptr, st, err);
  *n = g.n;
  *nnz = g.nnz;
  if (row_ptr) std::copy(g.row_ptr.begin(), g.row_ptr.end(), row_ptr);
  if (col_idx) std::copy(g.col_idx.begin(), g.col_idx.end(), col_idx);
  return PDD_OK;
}

pdd_status pdd_plan_tickets(const pdd_partition* part, const pdd_knots* knots, const int32_t* n_paths_per_knot,
                            int32_t paths_per_ticket, int32_t spatial, int32_t grid, int64_t* n_tickets,
                            int32_t* tickets, int32_t* order, int32_t* xcd_begin) {
  if (!part || !knots || !n_paths_per_knot || !n_tickets) return fail(nullptr, PDD_EINVAL, "pdd_plan_tickets: null argument");
  if (paths_per_ticket < 1) return fail(nullptr, PDD_EINVAL, "pdd_plan_tickets: paths_per_ticket must be >= 1");
  if (xcd_begin && (!spatial || grid < 8))
    return fail(nullptr, PDD_EINVAL, "pdd_plan_tickets: the XCD split needs the spatial order and grid >= 8");
  Geometry g;
  std::string err;
  pdd_status st = build_geometry(*part, *knots, g, err, false);
  if (st != PDD_OK) return fail(nullptr, st, err);
  std::vector<int32_t> npk(n_paths_per_knot, n_paths_per_knot + g.n);
  TicketPlan plan;
  if ((st = plan_tickets(g, npk, paths_per_ticket, spatial != 0, 0u, plan, err)) != PDD_OK) return fail(nullptr, st, err);
  *n_tickets = (int64_t)plan.tickets.size();
  if (tickets) {
    for (size_t i = 0; i < plan.tickets.size(); ++i) {
      tickets[3 * i] = plan.tickets[i].knot;
      tickets[3 * i + 1] = plan.tickets[i].p0;
      tickets[3 * i + 2] = plan.tickets[i].p1;
    }
  }
  if (order) std::copy(plan.order.begin(), plan.order.end(), order);
  if (xcd_begin) xcd_split(plan.cum_cost, (int64_t)plan.tickets.size(), grid, xcd_begin);
  return PDD_OK;
}

pdd_status pdd_knot_xy(const pdd_partition* part, const pdd_knots* knots, double* xy) {
  if (!part || !knots || !xy) return fail(nullptr, PDD_EINVAL, "pdd_knot_xy: null argument");
  Geometry g;
  std::string err;
  pdd_status st = build_geometry(*part, *knots, g, err, false);
  if (st != PDD_OK) return fail(nullptr, st, err);
  for (int64_t k = 0; k < g.n; ++k) {
    xy[2 * k] = g.x0 + (double)g.ix[k] * g.dx;
    xy[2 * k + 1] = g.y0 + (double)g.iy[k] * g.dy;
  }
  return PDD_OK;
}

pdd_status pdd_assemble(pdd_ctx* ctx, const pdd_coeffs* coeffs, const pdd_partition* part,
                        const pdd_knots* knots, const pdd_run* run, int32_t* row_ptr,
                        int32_t* col_idx, double* val, double* b, double* diag) {
  if (!ctx) return fail(nullptr, PDD_EINVAL, "pdd_assemble: null context");
  if (!coeffs || !part || !knots || !run) return fail(ctx, PDD_EINVAL, "pdd_assemble: null argument");
  if (!row_ptr || !col_idx || !val || !b) return fail(ctx, PDD_EINVAL, "pdd_assemble: null output");
  pdd_status st = validate_run(ctx, *coeffs, *run);
  if (st != PDD_OK) return st;
  AssembleJob job;
  job.coeffs = *coeffs;
  job.part = *part;
  job.knots = *knots;
  job.run = *run;
  job.row_ptr = row_ptr;
  job.col_idx = col_idx;
  job.val = val;
  job.b = b;
  job.diag = diag;
  return run_assemble(ctx, job);
}

pdd_status pdd_solve(pdd_ctx* ctx, int64_t n, const int32_t* row_ptr, const int32_t* col_idx,
                     const double* val, const double* b, double* u, double tol, int32_t max_iter,
                     int32_t* iters, double* relres) {
  if (!ctx) return fail(nullptr, PDD_EINVAL, "pdd_solve: null context");
  if (n < 1 || !row_ptr || !col_idx || !val || !b || !u || !iters || !relres)
    return fail(ctx, PDD_EINVAL, "pdd_solve: need n >= 1 and non-null arrays");
  if (!(tol > 0.0) || max_iter < 1) return fail(ctx, PDD_EINVAL, "pdd_solve: need tol > 0 and max_iter >= 1");
  return run_solve(ctx, n, row_ptr, col_idx, val, b, u, tol, max_iter, iters, relres);
}

pdd_status pdd_solve_noalloc(pdd_ctx* ctx, int64_t n, const int32_t* row_ptr, const int32_t* col_idx,
                             const double* val, const double* b, double* u, double tol, int32_t max_iter,
                             int32_t* iters, double* relres) {
  if (!ctx) return fail(nullptr, PDD_EINVAL, "pdd_solve_noalloc: null context");
  if (n < 1 || !row_ptr || !col_idx || !val || !b || !u || !iters || !relres || !(tol > 0.0) || max_iter < 1)
    return fail(ctx, PDD_EINVAL, "pdd_solve_noalloc: bad arguments");
  if (n > INT32_MAX) return fail(ctx, PDD_EINVAL, "pdd_solve_noalloc: n must fit int32");
  return run_solve_noalloc(ctx, n, row_ptr, col_idx, val, b, u, tol, max_iter, iters, relres);
}

pdd_status pdd_eval_subdomain(pdd_ctx* ctx, const pdd_coeffs* coeffs, const pdd_partition* part,
                              const pdd_knots* knots, const double* u_knots, int64_t n_pts, const double* xy,
                              const pdd_run* run, double* u, double* se) {
  if (!ctx) return fail(nullptr, PDD_EINVAL, "pdd_eval_subdomain: null context");
  if (!coeffs || !part || !knots || !run || !u_knots || n_pts < 0 || (n_pts > 0 && (!xy || !u)))
    return fail(ctx, PDD_EINVAL, "pdd_eval_subdomain: bad arguments");
  if (run->cv && run->cv->mode != PDD_CV_NONE)
    return fail(ctx, PDD_EINVAL, "pdd_eval_subdomain: run.cv must be NULL");
  if (run->n_paths_per_knot || run->dump_paths != 0)
    return fail(ctx, PDD_EINVAL, "pdd_eval_subdomain: run.n_paths_per_knot must be NULL and run.dump_paths 0");
  if (run->instance >= 0x80000000u)
    return fail(ctx, PDD_EINVAL, "pdd_eval_subdomain: run.instance must be below 2^31");
  if (run->interp != PDD_INTERP_HAT)
    return fail(ctx, PDD_EUNSUPPORTED, "pdd_eval_subdomain: boundary values use the hat interpolation (run.interp 0)");
  if (run->h_per_knot) return fail(ctx, PDD_EUNSUPPORTED, "pdd_eval_subdomain: run.h_per_knot must be NULL");
  if (n_pts > INT32_MAX) return fail(ctx, PDD_EINVAL, "pdd_eval_subdomain: at most 2^31 - 1 points");
  pdd_status st = validate_run(ctx, *coeffs, *run);
  if (st != PDD_OK) return st;
  if (n_pts == 0) return PDD_OK;
  return run_eval_subdomain(ctx, *coeffs, *part, *knots, u_knots, n_pts, xy, *run, u, se);
}

namespace {

// Collocation tables of degree p on the context's device (built once per p).
pdd_status get_spec(pdd_ctx* ctx, int32_t p, SpecCache** out) {
  SpecCache* sc = ctx->spec.get();
  if (!sc || sc->p != p) {
    SpectralTables t;
    std::string err;
    if (!spectral_tables(p, t, err)) return fail(ctx, PDD_EINVAL, err);
    auto fresh = std::make_unique<SpecCache>();
    fresh->p = p;
    fresh->decomp_residual = t.decomp_residual;
    fresh->inverse_residual = t.inverse_residual;
    const size_t nn = (size_t)SPEC_T * SPEC_T;
    std::vector<double> all;
    all.reserve(2 * SPEC_T + 2 * SPEC_T + 3 * nn + SPEC_T);
    auto put = [&](const std::vector<double>& v, size_t len) {
      const size_t off = all.size();
      all.insert(all.end(), v.begin(), v.end());
      all.resize(off + len, 0.0);
      return off;
    };
    const size_t o_nodes = put(t.nodes, SPEC_T), o_bw = put(t.bw, SPEC_T), o_D = put(t.D, nn),
                 o_D2b = put(t.D2b, 2 * SPEC_T), o_V = put(t.V, nn), o_Vi = put(t.Vinv, nn), o_lam = put(t.lam, SPEC_T);
    hipError_t e = fresh->buf.reserve(all.size() * sizeof(double));
    if (e != hipSuccess) return check_hip(ctx, e, "hipMalloc(spectral tables)");
    if ((e = hipMemcpy(fresh->buf.ptr, all.data(), all.size() * sizeof(double), hipMemcpyHostToDevice)) != hipSuccess)
      return check_hip(ctx, e, "upload spectral tables");
    const double* b = fresh->buf.as<double>();
    fresh->dev = SpecDev{b + o_nodes, b + o_bw, b + o_D, b + o_D2b, b + o_V, b + o_Vi, b + o_lam};
    ctx->spec = std::move(fresh);
    sc = ctx->spec.get();
  }
  *out = sc;
  return PDD_OK;
}

bool bad_domain(const pdd_partition& part) {
  return !(part.x1 > part.x0) || !(part.y1 > part.y0) || part.H < 2 || !std::isfinite(part.x0) ||
         !std::isfinite(part.x1) || !std::isfinite(part.y0) || !std::isfinite(part.y1);
}

}  // namespace

pdd_status pdd_spectral_solve(pdd_ctx* ctx, const pdd_coeffs* coeffs, const pdd_partition* part,
                              const pdd_knots* knots, int32_t p, int32_t interp, double rbf_c, const double* u_knots,
                              double* grid) {
  if (!ctx) return fail(nullptr, PDD_EINVAL, "pdd_spectral_solve: null context");
  if (!coeffs || !part || !knots || !u_knots || !grid || bad_domain(*part))
    return fail(ctx, PDD_EINVAL, "pdd_spectral_solve: bad arguments");
  if (p < 2 || p > SPEC_MAX_P) return fail(ctx, PDD_EINVAL, "pdd_spectral_solve: need 2 <= p <= 63");
  if (interp != PDD_INTERP_HAT && interp != PDD_INTERP_RBF_IMQ)
    return fail(ctx, PDD_EINVAL, "pdd_spectral_solve: unknown interpolation");
  if (interp == PDD_INTERP_RBF_IMQ && (!(rbf_c > 0.0) || !std::isfinite(rbf_c)))
    return fail(ctx, PDD_EINVAL, "pdd_spectral_solve: RBF side values need a finite shape parameter > 0");
  const int kind = coeffs->kind;
  if (kind != PDD_COEF_POISSON && kind != PDD_COEF_EXITTIME && kind != PDD_COEF_EQ43 && kind != PDD_COEF_LUT)
    return fail(ctx, PDD_EUNSUPPORTED,
                "pdd_spectral_solve: constant-coefficient operators only (POISSON, EXITTIME, EQ43, or a LUT with "
                "constant sigma, zero drift and constant reaction)");
  pdd_run run{};
  run.precision = PDD_FP64_SAME_STREAM;
  run.exit_rule = PDD_EXIT_NAIVE;
  run.n_paths = 1;
  run.h = 1.0;
  run.interp = interp;
  run.rbf_c = interp == PDD_INTERP_RBF_IMQ ? rbf_c : 0.0;
  pdd_status st = validate_run(ctx, *coeffs, run);
  if (st != PDD_OK) return st;
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return check_hip(ctx, e, "hipSetDevice");
  const double Sx = (part->x1 - part->x0) / part->H, Sy = (part->y1 - part->y0) / part->H;
  double axx = 2.0, ayy = 2.0, cr = 0.0;           // a_xx, a_yy of sigma = sqrt(2) I
  if (kind == PDD_COEF_LUT) {
    // the operator must be constant over the table: read every field's range
    const int64_t nodes = (int64_t)coeffs->lut_n * coeffs->lut_n;
    if ((e = ctx->spec_range.reserve((12 + 1024 * 12) * sizeof(double))) != hipSuccess)
      return check_hip(ctx, e, "hipMalloc(spectral range)");
    if ((e = launch_lut_field_range(coeffs->lut, nodes, ctx->spec_range.as<double>(), ctx->stream)) != hipSuccess)
      return check_hip(ctx, e, "launch lut range");
    double r[12];
    if ((e = hipMemcpyAsync(r, ctx->spec_range.ptr, sizeof(r), hipMemcpyDeviceToHost, ctx->stream)) != hipSuccess)
      return check_hip(ctx, e, "read lut range");
    if ((e = hipStreamSynchronize(ctx->stream)) != hipSuccess) return check_hip(ctx, e, "hipStreamSynchronize");
    // fields: 0 sxx, 1 sxy, 2 syy, 3 dx, 4 dy, 5 c; r[q] = min, r[6 + q] = max
    for (int q = 0; q < 6; ++q)
      if (r[q] != r[6 + q])
        return fail(ctx, PDD_EUNSUPPORTED, "pdd_spectral_solve: the table's sigma, drift and reaction must be constant");
    if (r[1] != 0.0 || r[3] != 0.0 || r[4] != 0.0)
      return fail(ctx, PDD_EUNSUPPORTED, "pdd_spectral_solve: the table needs a diagonal sigma and zero drift");
    axx = r[0] * r[0];
    ayy = r[2] * r[2];
    cr = r[5];
    if (cr > 0.0) return fail(ctx, PDD_EINVAL, "pdd_spectral_solve: the reaction must be <= 0");
  }
  GeoCache* gc = nullptr;
  if ((st = get_geometry(ctx, *part, *knots, &gc)) != PDD_OK) return st;
  if ((st = get_lattice(ctx, gc)) != PDD_OK) return st;
  SpecCache* sc = nullptr;
  if ((st = get_spec(ctx, p, &sc)) != PDD_OK) return st;
  SpecArgs A;
  fill_asm_params(*gc, *coeffs, run, A.P);
  if (interp == PDD_INTERP_RBF_IMQ) {
    if (std::min(knots->m + 2 * knots->ext, (int32_t)gc->g.L) + 1 > gc->g.slot_len)
      return fail(ctx, PDD_EINVAL, "pdd_spectral_solve: side stencil longer than the stencil table");
    if ((st = prepare_rbf(ctx, gc->g, run, A.P, false)) != PDD_OK) return st;
  }
  A.T = sc->dev;
  A.p = p;
  A.H = part->H;
  A.m = knots->m;
  A.ext = knots->ext;
  A.rbf = interp == PDD_INTERP_RBF_IMQ;
  A.ax = 0.5 * axx * (2.0 / Sx) * (2.0 / Sx);
  A.ay = 0.5 * ayy * (2.0 / Sy) * (2.0 / Sy);
  A.c = cr;
  A.u_knots = u_knots;
  A.grid = grid;
  return check_hip(ctx, launch_spectral_solve(A, ctx->stream), "launch spectral solve");
}

pdd_status pdd_spectral_eval(pdd_ctx* ctx, const pdd_partition* part, int32_t p, const double* grid, int64_t n_pts,
                             const double* xy, double* u, double* grad) {
  if (!ctx) return fail(nullptr, PDD_EINVAL, "pdd_spectral_eval: null context");
  if (!part || !grid || bad_domain(*part) || n_pts < 0 || (n_pts > 0 && (!xy || (!u && !grad))))
    return fail(ctx, PDD_EINVAL, "pdd_spectral_eval: bad arguments");
  if (p < 2 || p > SPEC_MAX_P) return fail(ctx, PDD_EINVAL, "pdd_spectral_eval: need 2 <= p <= 63");
  if (n_pts == 0) return PDD_OK;
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return check_hip(ctx, e, "hipSetDevice");
  SpecCache* sc = nullptr;
  pdd_status st = get_spec(ctx, p, &sc);
  if (st != PDD_OK) return st;
  return check_hip(ctx, launch_spectral_eval(sc->dev, p, part->H, part->x0, part->x1, part->y0, part->y1, grid, n_pts,
                                             xy, 0, u, grad, nullptr, ctx->stream),
                   "launch spectral eval");
}

pdd_status pdd_spectral_grad_lut(pdd_ctx* ctx, const pdd_partition* part, int32_t p, const double* grid, int32_t lut_n,
                                 float* grad_lut) {
  if (!ctx) return fail(nullptr, PDD_EINVAL, "pdd_spectral_grad_lut: null context");
  if (!part || !grid || !grad_lut || bad_domain(*part) || lut_n < 2 || lut_n > 65536)
    return fail(ctx, PDD_EINVAL, "pdd_spectral_grad_lut: bad arguments");
  if (p < 2 || p > SPEC_MAX_P) return fail(ctx, PDD_EINVAL, "pdd_spectral_grad_lut: need 2 <= p <= 63");
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return check_hip(ctx, e, "hipSetDevice");
  SpecCache* sc = nullptr;
  pdd_status st = get_spec(ctx, p, &sc);
  if (st != PDD_OK) return st;
  return check_hip(ctx, launch_spectral_eval(sc->dev, p, part->H, part->x0, part->x1, part->y0, part->y1, grid, 0,
                                             nullptr, lut_n, nullptr, nullptr, grad_lut, ctx->stream),
                   "launch spectral grad table");
}

pdd_status pdd_spectral_tables(int32_t p, double* decomp_residual, double* inverse_residual) {
  SpectralTables t;
  std::string err;
  if (!spectral_tables(p, t, err)) return fail(nullptr, PDD_EINVAL, "pdd_spectral_tables: " + err);
  if (decomp_residual) *decomp_residual = t.decomp_residual;
  if (inverse_residual) *inverse_residual = t.inverse_residual;
  return PDD_OK;
}

pdd_status pdd_calibrate(pdd_ctx* ctx, const pdd_coeffs* coeffs, const pdd_partition* part, const pdd_knots* knots,
                         const pdd_run* run, const double* u_knots, double* stats) {
  if (!ctx) return fail(nullptr, PDD_EINVAL, "pdd_calibrate: null context");
  if (!coeffs || !part || !knots || !run || !u_knots || !stats)
    return fail(ctx, PDD_EINVAL, "pdd_calibrate: bad arguments");
  if (run->n_paths < 1 || run->n_paths > INT32_MAX) return fail(ctx, PDD_EINVAL, "pdd_calibrate: need 1 <= n_paths < 2^31");
  if (run->cv && run->cv->mode == PDD_CV_NETWORK)
    return fail(ctx, PDD_EINVAL, "pdd_calibrate: xi is drawn with the gradient table (run.cv mode GRAD_LUT) or not at all");
  if (run->h_per_knot) return fail(ctx, PDD_EUNSUPPORTED, "pdd_calibrate: one time step h0 (run.h_per_knot NULL)");
  pdd_run r = *run;
  r.exit_rule = PDD_EXIT_GM;
  r.n_paths_per_knot = nullptr;
  r.dump = nullptr;
  r.dump_paths = 0;
  pdd_status st = validate_run(ctx, *coeffs, r);
  if (st != PDD_OK) return st;
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return check_hip(ctx, e, "hipSetDevice");
  GeoCache* gc = nullptr;
  if ((st = get_geometry(ctx, *part, *knots, &gc)) != PDD_OK) return st;
  if ((st = get_lattice(ctx, gc)) != PDD_OK) return st;
  const size_t bytes = calibrate_scratch_bytes(gc->g.n, (int32_t)r.n_paths);
  if (bytes > ((size_t)16 << 30)) return fail(ctx, PDD_EINVAL, "pdd_calibrate: n * n_paths too large (16 GiB scratch)");
  if ((e = ctx->calib_scratch.reserve(bytes)) != hipSuccess) return check_hip(ctx, e, "hipMalloc(calibration scratch)");
  AsmParams P;
  fill_asm_params(*gc, *coeffs, r, P);
  if ((st = prepare_lut_bound(ctx, *coeffs, r, P, false)) != PDD_OK) return st;
  double* alpha = nullptr;
  if (r.interp == PDD_INTERP_RBF_IMQ) {
    // the stencil inverses, and scratch for the per-side RBF coefficients of u0
    if ((st = prepare_rbf(ctx, gc->g, r, P, false)) != PDD_OK) return st;
    const size_t abytes = (size_t)gc->g.n * 4 * gc->g.slot_len * sizeof(double);
    if ((e = ctx->calib_alpha.reserve(abytes)) != hipSuccess) return check_hip(ctx, e, "hipMalloc(rbf coefficients)");
    alpha = ctx->calib_alpha.as<double>();
  }
  e = launch_calibrate(P, r.precision, gc->g.n, (int32_t)r.n_paths, r.instance, u_knots, ctx->calib_scratch.as<double>(),
                       stats, ctx->stream, alpha, gc->g.slot_len);
  return check_hip(ctx, e, "launch calibrate");
}

pdd_status pdd_calibration_plan(int64_t n, const double* stats, int64_t n_paths, double h0_cal, double h0, double eps,
                                int32_t n_job, double* h, int32_t* paths, double* bias, double* var, double* rho2) {
  if (n < 0 || (n > 0 && (!stats || !h || !paths)) || n_paths < 1 || !(h0 > 0.0) || !(h0_cal >= h0) ||
      !std::isfinite(h0_cal) || !(eps > 0.0) || n_job < 1)
    return fail(nullptr, PDD_EINVAL, "pdd_calibration_plan: bad arguments (need 0 < h0 <= h0_cal, eps > 0, n_job >= 1)");
  const double N = (double)n_paths;
  for (int64_t i = 0; i < n; ++i) {
    const double* s = stats + i * PDD_CAL_WIDTH;
    const double mdiff = s[0] / N, mphi = s[1] / N, mxi = s[3] / N;
    const double vphi = std::max(s[2] / N - mphi * mphi, 0.0);
    const double vxi = std::max(s[4] / N - mxi * mxi, 0.0);
    const double cov = s[5] / N - mphi * mxi;
    const double den = vphi * vxi;
    const double r2 = den > 0.0 ? std::min(cov * cov / den, 1.0) : 0.0;
    h[i] = mdiff != 0.0 ? std::min(h0, 2.0 * h0_cal * eps / (3.0 * std::fabs(mdiff))) : h0;
    const double nraw = 9.0 * vphi * (1.0 - r2) / (eps * eps);
    const double k = std::max(std::floor(nraw / n_job + 0.5), 1.0);
    if (k * n_job > (double)INT32_MAX) return fail(nullptr, PDD_EINVAL, "pdd_calibration_plan: path count overflows int32");
    paths[i] = (int32_t)(k * n_job);
    if (bias) bias[i] = 0.5 * std::fabs(mdiff);
    if (var) var[i] = vphi;
    if (rho2) rho2[i] = r2;
  }
  return PDD_OK;
}

pdd_status pdd_rbf_shape(int32_t n_nodes, double spacing, double target_cond, double* c) {
  const pdd_status st = rbf_shape(n_nodes, spacing, target_cond, c);
  if (st != PDD_OK) return fail(nullptr, st, "pdd_rbf_shape: need 2 <= n_nodes <= 256, spacing > 0 and 1 < target_cond <= 1e14 in reach");
  return PDD_OK;
}

pdd_status pdd_mlp_init(pdd_ctx* ctx, float* params, uint64_t seed) {
  if (!ctx) return fail(nullptr, PDD_EINVAL, "pdd_mlp_init: null context");
  if (!params) return fail(ctx, PDD_EINVAL, "pdd_mlp_init: null params");
  return run_mlp_init(ctx, params, seed);
}

pdd_status pdd_mlp_eval(pdd_ctx* ctx, const float* params, int64_t n, const float* xy, float* v, float* grad) {
  if (!ctx) return fail(nullptr, PDD_EINVAL, "pdd_mlp_eval: null context");
  if (!params || n < 0 || (n > 0 && (!xy || (!v && !grad)))) return fail(ctx, PDD_EINVAL, "pdd_mlp_eval: bad arguments");
  if (n == 0) return PDD_OK;
  return run_mlp_eval(ctx, params, n, xy, v, grad);
}

pdd_status pdd_mlp_grad_bf16(pdd_ctx* ctx, const float* params, int64_t n, const float* xy, float* grad) {
  if (!ctx) return fail(nullptr, PDD_EINVAL, "pdd_mlp_grad_bf16: null context");
  if (!params || n < 0 || (n > 0 && (!xy || !grad))) return fail(ctx, PDD_EINVAL, "pdd_mlp_grad_bf16: bad arguments");
  if (n == 0) return PDD_OK;
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return check_hip(ctx, e, "hipSetDevice");
  return run_mlp_grad_bf16(ctx, params, n, xy, grad);
}

pdd_status pdd_mlp_grad(pdd_ctx* ctx, const float* params, int64_t n, const float* xy, const float* target,
                        float* grad, float* loss) {
  if (!ctx) return fail(nullptr, PDD_EINVAL, "pdd_mlp_grad: null context");
  if (!params || !xy || !target || !grad || n < 1 || n > INT32_MAX)
    return fail(ctx, PDD_EINVAL, "pdd_mlp_grad: bad arguments");
  // identity order over the n points, one batch of n
  hipError_t e = ctx->mlp_scratch.reserve((size_t)n * sizeof(int32_t));
  if (e != hipSuccess) return check_hip(ctx, e, "hipMalloc(mlp scratch)");
  std::vector<int32_t> order(n);
  for (int64_t i = 0; i < n; ++i) order[i] = (int32_t)i;
  e = hipMemcpy(ctx->mlp_scratch.ptr, order.data(), (size_t)n * sizeof(int32_t), hipMemcpyHostToDevice);
  if (e != hipSuccess) return check_hip(ctx, e, "upload order");
  return run_mlp_train(ctx, const_cast<float*>(params), nullptr, nullptr, n, xy, target, ctx->mlp_scratch.as<int32_t>(),
                       n, (int32_t)n, 1, 0, 0.0f, loss, grad);
}

pdd_status pdd_mlp_train(pdd_ctx* ctx, float* params, float* adam_m, float* adam_s, int64_t n_points,
                         const float* xy, const float* target, const int32_t* order, int64_t n_order, int32_t batch,
                         int32_t steps, int32_t step0, float lr, float* losses) {
  if (!ctx) return fail(nullptr, PDD_EINVAL, "pdd_mlp_train: null context");
  if (!params || !adam_m || !adam_s || !xy || !target || !order || n_points < 1 || n_order < 1 || batch < 1 ||
      steps < 0 || step0 < 0 || !(lr > 0.0f))
    return fail(ctx, PDD_EINVAL, "pdd_mlp_train: bad arguments");
  if (steps == 0) return PDD_OK;
  return run_mlp_train(ctx, params, adam_m, adam_s, n_points, xy, target, order, n_order, batch, steps, step0, lr,
                       losses, nullptr);
}

pdd_status pdd_mlp_bake_grad_lut(pdd_ctx* ctx, const float* params, const pdd_partition* part, int32_t lut_n,
                                 float* grad_lut) {
  if (!ctx) return fail(nullptr, PDD_EINVAL, "pdd_mlp_bake_grad_lut: null context");
  if (!params || !part || !grad_lut || lut_n < 2 || lut_n > 65536 || !(part->x1 > part->x0) || !(part->y1 > part->y0))
    return fail(ctx, PDD_EINVAL, "pdd_mlp_bake_grad_lut: bad arguments");
  return run_mlp_bake(ctx, params, *part, lut_n, grad_lut);
}

pdd_status pdd_collect_training(pdd_ctx* ctx, const pdd_coeffs* coeffs, const pdd_partition* part,
                                const pdd_knots* knots, const pdd_run* run, const double* u0, int32_t paths_per_knot,
                                int32_t points_per_path, float* xy, float* target) {
  if (!ctx) return fail(nullptr, PDD_EINVAL, "pdd_collect_training: null context");
  if (!coeffs || !part || !knots || !run || !u0 || !xy || !target || paths_per_knot < 1 || points_per_path < 1)
    return fail(ctx, PDD_EINVAL, "pdd_collect_training: bad arguments");
  if (run->cv && run->cv->mode != PDD_CV_NONE)
    return fail(ctx, PDD_EINVAL, "pdd_collect_training: collect from plain paths (run.cv must be NULL)");
  if (run->interp != PDD_INTERP_HAT)
    return fail(ctx, PDD_EUNSUPPORTED, "pdd_collect_training: targets use the hat interpolation (run.interp 0)");
  if (run->h_per_knot) return fail(ctx, PDD_EUNSUPPORTED, "pdd_collect_training: run.h_per_knot must be NULL");
  if (run->instance >= PDD_COLLECT_STREAM)
    return fail(ctx, PDD_EINVAL, "pdd_collect_training: run.instance must be below 2^30");
  pdd_status st = validate_run(ctx, *coeffs, *run);
  if (st != PDD_OK) return st;
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return check_hip(ctx, e, "hipSetDevice");
  GeoCache* gc = nullptr;
  if ((st = get_geometry(ctx, *part, *knots, &gc)) != PDD_OK) return st;
  if ((st = get_lattice(ctx, gc)) != PDD_OK) return st;
  const int64_t slots = gc->g.n * (int64_t)paths_per_knot * points_per_path;
  if (slots > ((int64_t)1 << 31)) return fail(ctx, PDD_EINVAL, "pdd_collect_training: too many record slots");
  if ((e = ctx->collect_scratch.reserve((size_t)slots * 2 * sizeof(float))) != hipSuccess)
    return check_hip(ctx, e, "hipMalloc(collect scratch)");
  AsmParams P;
  fill_asm_params(*gc, *coeffs, *run, P);
  if ((st = prepare_lut_bound(ctx, *coeffs, *run, P, false)) != PDD_OK) return st;
  // the pairs draw from their own stream class (instance word + 2^30), so
  // no assembly with instance < 2^30 reuses the paths the network was fitted on
  e = launch_collect(P, gc->g.n, paths_per_knot, points_per_path, run->instance + PDD_COLLECT_STREAM, u0, xy,
                     ctx->collect_scratch.as<float>(), target, ctx->stream);
  return check_hip(ctx, e, "launch collect");
}

pdd_status pdd_set_launch(pdd_ctx* ctx, int32_t block, int32_t grid, int32_t paths_per_ticket,
                          int32_t schedule) {
  if (!ctx) return fail(nullptr, PDD_EINVAL, "pdd_set_launch: null context");
  if (block < 0 || block > 256 || block % 64 != 0 || grid < 0 || paths_per_ticket < 0)
    return fail(ctx, PDD_EINVAL, "pdd_set_launch: block must be 0 or a multiple of 64 up to 256; grid, paths_per_ticket >= 0");
  if (schedule != PDD_SCHEDULE_STATIC && schedule != PDD_SCHEDULE_DYNAMIC)
    return fail(ctx, PDD_EINVAL, "pdd_set_launch: unknown schedule");
  ctx->force_block = block;
  ctx->force_grid = grid;
  ctx->force_per_ticket = paths_per_ticket;
  ctx->schedule = schedule;
  return PDD_OK;
}

pdd_status pdd_set_refill(pdd_ctx* ctx, int32_t min_idle) {
  if (!ctx) return fail(nullptr, PDD_EINVAL, "pdd_set_refill: null context");
  if (min_idle < 1 || min_idle > 64) return fail(ctx, PDD_EINVAL, "pdd_set_refill: need 1 <= min_idle <= 64");
  ctx->refill_min = min_idle;
  return PDD_OK;
}

pdd_status pdd_set_spare_rows(pdd_ctx* ctx, int32_t spare) {
  if (!ctx) return fail(nullptr, PDD_EINVAL, "pdd_set_spare_rows: null context");
  if (spare < -1) return fail(ctx, PDD_EINVAL, "pdd_set_spare_rows: need spare >= 0, or -1 for one per wave");
  ctx->spare_rows = spare;
  return PDD_OK;
}

pdd_status pdd_set_table_read(pdd_ctx* ctx, int32_t read_all) {
  if (!ctx) return fail(nullptr, PDD_EINVAL, "pdd_set_table_read: null context");
  if (read_all != 0 && read_all != 1) return fail(ctx, PDD_EINVAL, "pdd_set_table_read: read_all must be 0 or 1");
  ctx->table_read_all = read_all;
  return PDD_OK;
}

pdd_status pdd_table_fields(pdd_ctx* ctx, uint32_t* varying, int32_t* lane_read) {
  if (!ctx) return fail(nullptr, PDD_EINVAL, "pdd_table_fields: null context");
  if (!varying || !lane_read) return fail(ctx, PDD_EINVAL, "pdd_table_fields: null output");
  if (!ctx->lut_info.ptr) return fail(ctx, PDD_EINVAL, "pdd_table_fields: no float32 LUT assembly has run");
  uint32_t w[2];
  hipError_t e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return check_hip(ctx, e, "hipStreamSynchronize");
  if ((e = hipMemcpy(w, ctx->lut_info.ptr, sizeof(w), hipMemcpyDeviceToHost)) != hipSuccess)
    return check_hip(ctx, e, "read LUT layout");
  *varying = w[0];
  *lane_read = (w[1] & LUT_LANE_READ) ? 1 : 0;
  return PDD_OK;
}

pdd_status pdd_get_spare_rows(const pdd_ctx* ctx, int32_t* spare) {
  if (!ctx || !spare) return PDD_EINVAL;
  *spare = ctx->spare_rows;
  return PDD_OK;
}

pdd_status pdd_get_refill(const pdd_ctx* ctx, int32_t* min_idle) {
  if (!ctx || !min_idle) return PDD_EINVAL;
  *min_idle = ctx->refill_min;
  return PDD_OK;
}

pdd_status pdd_last_launch(const pdd_ctx* ctx, int32_t* grid, int32_t* block, int64_t* tickets) {
  if (!ctx || !grid || !block || !tickets) return fail(nullptr, PDD_EINVAL, "pdd_last_launch: null argument");
  *grid = ctx->last_grid;
  *block = ctx->last_block;
  *tickets = ctx->last_tickets;
  return PDD_OK;
}

pdd_status pdd_set_timing(pdd_ctx* ctx, int32_t enable) {
  if (!ctx) return fail(nullptr, PDD_EINVAL, "pdd_set_timing: null context");
  hipError_t e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return check_hip(ctx, e, "hipStreamSynchronize");
  ctx->timing = enable != 0;
  ctx->ev_used = 0;
  return PDD_OK;
}

pdd_status pdd_kernel_ms(pdd_ctx* ctx, double* total_ms, int32_t* launches) {
  if (!ctx || !total_ms || !launches) return fail(ctx, PDD_EINVAL, "pdd_kernel_ms: null argument");
  double sum = 0.0;
  for (int i = 0; i < ctx->ev_used; ++i) {
    float ms = 0.0f;
    hipError_t e = hipEventSynchronize(ctx->ev_pool[2 * i + 1]);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, ctx->ev_pool[2 * i], ctx->ev_pool[2 * i + 1]);
    if (e != hipSuccess) return check_hip(ctx, e, "hipEventElapsedTime");
    sum += ms;
  }
  *total_ms = sum;
  *launches = ctx->ev_used;
  return PDD_OK;
}

}  // extern "C"
