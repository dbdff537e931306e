// Library context: device, stream, caches and scratch owned by one pdd_ctx.
#pragma once

#include <algorithm>

#include <hip/hip_runtime.h>

#include <memory>
#include <string>
#include <vector>

#include "geometry.h"
#include "kernels.h"
#include "pdd.h"
#include "spectral.h"

namespace pdd {

// Owning device allocation that only grows.
struct DeviceBuffer {
  void* ptr = nullptr;
  size_t bytes = 0;
  DeviceBuffer() = default;
  DeviceBuffer(const DeviceBuffer&) = delete;
  DeviceBuffer& operator=(const DeviceBuffer&) = delete;
  ~DeviceBuffer();
  hipError_t reserve(size_t want);
  void release();
  template <typename T> T* as() const { return static_cast<T*>(ptr); }
};

// Host geometry of one (partition, knots) pair and its device copies.
struct GeoCache {
  pdd_partition part{};
  pdd_knots kn{};
  Geometry g;
  DeviceBuffer desc, knot_ij, row_ptr, col_idx, lattice;
};

// Tickets of one (geometry, path counts, ticket size) combination.
struct TicketCache {
  const GeoCache* geo = nullptr;
  std::vector<int32_t> npk;       // paths per knot
  std::vector<double> hk;         // per-knot time steps (empty: the launch's h)
  DeviceBuffer h_knot;            // device copy of hk
  int32_t per_ticket = 0;
  uint32_t inst = 0;
  bool spatial = false;           // spatial order (tabulated coefficients) instead of longest-first
  int64_t n_tickets = 0;
  DeviceBuffer tickets, ticket_begin, n_paths, order;
  // spatial order: cumulative expected cost along the order, and the XCD
  // split of the order for the grid it was last computed for
  std::vector<double> cum_cost;
  int32_t xcd_grid = -1;
  DeviceBuffer xcd_begin;
};

// Device-side tables of one batch of instances (rebuilt when the batch changes).
struct BatchCache {
  std::vector<pdd_partition> parts;
  std::vector<pdd_knots> knots;
  std::vector<std::vector<int32_t>> npk;
  std::vector<double> h, a;
  std::vector<uint32_t> inst_ids;
  int32_t per_ticket = 0;
  std::vector<std::unique_ptr<GeoCache>> geos;
  std::vector<int64_t> knot_off, ticket_off, n_tickets;
  int64_t total_tickets = 0;
  int slot_len = 0;
  DeviceBuffer desc, insts, tickets, order;
  std::vector<std::unique_ptr<DeviceBuffer>> ticket_begin, n_paths;
};

struct TuneEntry {
  std::string sig;
  int block, grid, per_ticket, schedule, refill, spare;
  double ms;
  std::string report;
};

struct AssembleJob {
  pdd_coeffs coeffs;
  pdd_partition part;
  pdd_knots knots;
  pdd_run run;
  int32_t* row_ptr;
  int32_t* col_idx;
  double* val;
  double* b;
  double* diag;
};

}  // namespace pdd

namespace pdd {
// Collocation tables of one spectral degree p on the device.
struct SpecCache {
  int32_t p = 0;
  DeviceBuffer buf;
  SpecDev dev{};
  double decomp_residual = 0, inverse_residual = 0;
};
// Inverses of the RBF stencil matrices for one (slot length, spacing, c).
struct RbfCache {
  int32_t slot_len = 0;
  double dx = 0, dy = 0, c = 0;
  int64_t half = 0;
  DeviceBuffer tab;
};
}  // namespace pdd

struct pdd_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  int cu_count = 0;
  std::string arch;
  std::string err;
  std::vector<std::unique_ptr<pdd::GeoCache>> geo;
  std::unique_ptr<pdd::TicketCache> tickets;
  std::unique_ptr<pdd::BatchCache> batch;
  std::unique_ptr<pdd::RbfCache> rbf;
  std::unique_ptr<pdd::SpecCache> spec;
  pdd::DeviceBuffer spec_range;      // LUT field ranges of the spectral solve (12 + 1024 * 12 doubles)
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  bool capturing = false;
  std::vector<pdd::TuneEntry> tune_cache;
  pdd::DeviceBuffer partial;
  pdd::DeviceBuffer solve_scratch, solve_flag;
  pdd::DeviceBuffer collect_scratch, mlp_scratch, calib_scratch, calib_alpha;
  pdd::DeviceBuffer mlp_wide;        // per-workgroup gradients of the multi-workgroup Adam step
  // launch overrides (0 = automatic), set by the tuner
  int force_block = 0, force_grid = 0, force_per_ticket = 0;
  int schedule = PDD_SCHEDULE_STATIC;
  int refill_min = 1;                // refill idle lanes once at least this many are idle
  int spare_rows = -1;               // tally rows per workgroup beyond one per wave (-1: one per wave)
  pdd::DeviceBuffer ticket_counter;
  pdd::DeviceBuffer lut_max;         // LUT + GM: table-wide |sigma| maxima
  pdd::DeviceBuffer lut_cells;       // float32 LUT assembly: cell-major copy of the table
  pdd::DeviceBuffer lut_info;        // its varying fields, layout and constant fields (16 words)
  int32_t table_read_all = 0;        // 1: the full cooperative read even for constant fields
  bool lut_lane = false;             // the last eager float32 table assembly found the lane-read layout
  // shape of the last assembly launch (reported by pdd_last_launch)
  int last_grid = 0, last_block = 0;
  int64_t last_tickets = 0;
  // optional event pairs around the assembly kernels
  bool timing = false;
  bool timing_with_finalize = false;  // the autotuner's pairs also cover the row sums
  std::vector<hipEvent_t> ev_pool;   // 2 per timed launch, reused
  int ev_used = 0;                   // pairs recorded since pdd_set_timing
  ~pdd_ctx() {
    for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
    if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
    if (graph) (void)hipGraphDestroy(graph);
  }
};

namespace pdd {

pdd_status check_hip(pdd_ctx* ctx, hipError_t e, const char* what);
pdd_status get_geometry(pdd_ctx* ctx, const pdd_partition& part, const pdd_knots& kn, GeoCache** out);
pdd_status get_lattice(pdd_ctx* ctx, GeoCache* gc);
pdd_status build_geo_cache(pdd_ctx* ctx, const pdd_partition& part, const pdd_knots& kn,
                           std::unique_ptr<GeoCache>& out);
bool same_geometry(const GeoCache& gc, const pdd_partition& part, const pdd_knots& kn);
pdd_status run_assemble_batch(pdd_ctx* ctx, int32_t n_inst, const pdd_instance* inst);
pdd_status validate_run(pdd_ctx* ctx, const pdd_coeffs& c, const pdd_run& r);
void fill_asm_params(const GeoCache& gc, const pdd_coeffs& co, const pdd_run& run, AsmParams& P);
pdd_status run_assemble(pdd_ctx* ctx, const AssembleJob& job);
// LUT family under the GM rule: enqueue the table-bound kernels and point
// P.coef.lut_max at their result (no-op otherwise).
pdd_status prepare_lut_bound(pdd_ctx* ctx, const pdd_coeffs& co, const pdd_run& run, AsmParams& P, bool capturing,
                             bool scanned = false);
// LUT family in float32: enqueue the cell-major copy of the table and point
// P.coef.cells at it (no-op otherwise).
bool uses_lut_cells(const pdd_coeffs& co, const pdd_run& run);
pdd_status prepare_lut_cells(pdd_ctx* ctx, const pdd_coeffs& co, const pdd_run& run, bool capturing, bool* lane_layout);
// RBF interpolation: build (once per geometry and shape parameter) and
// upload the inverses of the stencil matrices; point P.rbf_inv at them.
pdd_status prepare_rbf(pdd_ctx* ctx, const Geometry& g, const pdd_run& run, AsmParams& P, bool capturing);
pdd_status run_eval_subdomain(pdd_ctx* ctx, const pdd_coeffs& co, const pdd_partition& part, const pdd_knots& kn,
                              const double* u_knots, int64_t n_pts, const double* xy, const pdd_run& run, double* u,
                              double* se);
pdd_status run_solve(pdd_ctx* ctx, int64_t n, const int32_t* rp, const int32_t* ci, const double* val,
                     const double* b, double* u, double tol, int32_t max_iter, int32_t* iters, double* relres);
// pdd_solve_noalloc: the same solve on the library's static device scratch
// (SOLVE_NOALLOC_BYTES per GPU); solve_noalloc_setup(device) looks up that
// device's copy once (the device current).
constexpr size_t SOLVE_NOALLOC_BYTES = (size_t)128 << 20;
hipError_t solve_noalloc_setup(int device);
pdd_status run_solve_noalloc(pdd_ctx* ctx, int64_t n, const int32_t* rp, const int32_t* ci, const double* val,
                             const double* b, double* u, double tol, int32_t max_iter, int32_t* iters,
                             double* relres);

// Tally rows in an assembly workgroup's pool: one per wave plus the context's
// spare rows (at most one more per wave).
inline int pool_rows_for(const pdd_ctx* ctx, int block) {
  const int w = block / 64;
  return ctx->spare_rows < 0 ? 2 * w : w + std::min(ctx->spare_rows, w);
}

}  // namespace pdd
