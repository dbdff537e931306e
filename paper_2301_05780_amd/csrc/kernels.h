// Parameter blocks shared by the host engine and the HIP kernels, and the
// host-callable launchers.  Plain structs only; no torch types anywhere.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

#include "pdd.h"

namespace pdd {

// Offset of the S x S block in one orientation's half of the RBF inverse
// table: blocks for S = 1, 2, ... are stored back to back, so S starts at
// 1^2 + ... + (S-1)^2.
__host__ __device__ inline int64_t rbf_block_offset(int64_t S) { return (S - 1) * S * (2 * S - 1) / 6; }

// Per-knot descriptor read by the assembly kernels (one per unknown).
struct KnotDesc {
  double sx, sy;          // start point x_k
  double line[4];         // physical coordinate of the line of side E, N, W, S
  int32_t at[4];          // lattice coordinate of the line of side E, N, W, S
  int32_t clo[4], chi[4]; // clamp range of each side along its line (lattice units)
  int32_t bmask;          // bit o set: side o lies on the domain boundary
  int32_t knot;           // canonical index
  int32_t pad[6];
};
static_assert(sizeof(KnotDesc) == 128, "KnotDesc must stay 128 bytes");

// Per-instance parameters of a batched launch (one BVP instance each).
struct InstDesc {
  double x0, x1, y0, y1, dx, dy;   // domain and lattice spacing
  double h, sqrt_h;                // time step
  double a;                        // AMPLITUDE family parameter
  float inv_dx, inv_dy;
  int32_t L;                       // lattice intervals per direction
  uint32_t inst_id;                // fourth Philox counter word
  int32_t pad[2];
};
static_assert(sizeof(InstDesc) == 96, "InstDesc must stay 96 bytes");

// A unit of work: paths [p0, p1) of one knot of one instance.
struct Ticket {
  int32_t knot;
  int32_t p0, p1;
  uint32_t inst;
};

struct CoefParams {
  int32_t kind;
  int32_t lut_n;
  double a;                   // AMPLITUDE parameter
  const float* lut;           // LUT kind
  double x0, x1, y0, y1;      // domain (LUT node grid spans it)
  float lut_sx, lut_sy;       // (n-1)/(x1-x0), (n-1)/(y1-y0)
  float x0f, y0f;             // (float)x0, (float)y0 for the float32 table reads
  // LUT kind under the Gobet-Menozzi rule: max |sxx|, |sxy|, |syy| over the
  // table's nodes as float bit patterns (device, written by launch_lut_bound)
  const uint32_t* lut_max;
  // float32 LUT kernels: the table re-laid cell by cell (launch_lut_cells):
  // cell (i, j) holds 8 float4, float4 q = the bilinear form of field q on
  // the cell, (v00, v10 - v00, v01 - v00, v11 - v10 - v01 + v00) of its
  // corners (i, j), (i+1, j), (i, j+1), (i+1, j+1); q = 7 is zero padding
  // (128 B per cell).  When at most two of the seven fields vary over the
  // table (launch_lut_cells decides, see lut_info), the copy holds only the
  // varying fields' forms, 16 B each per cell, and the kernels read it one
  // lane per path.
  const float4* cells;
  // float32 LUT kernels (device, written by launch_lut_cells):
  // [0] bit q set when field q varies over the table (or is not finite);
  // [1] layout of `cells`: 0 = all eight forms per cell, else
  //     LUT_LANE_READ | k1 | k2 << 4 | count << 8 (the count <= 2 varying
  //     fields k1, k2 in that order, 15 for none; count 0 reads field k1 = 6);
  // [8 + q] the float bits of field q at node 0, plus 0 (16 words in all)
  const uint32_t* lut_info;
};
constexpr uint32_t LUT_LANE_READ = 0x80000000u;

struct AsmParams {
  const KnotDesc* desc;
  const Ticket* tickets;      // batched: Ticket.inst indexes `insts`, Ticket.knot the concatenated descs
  const InstDesc* insts;      // batched launches only (nullptr otherwise)
  const int32_t* order;       // schedule: ticket ids in the order they are handed out
  int32_t n_tickets;
  // static schedule split by XCD (nullable): the waves of the workgroups with
  // blockIdx % 8 == x take order[xcd_begin[x] .. xcd_begin[x+1]) among
  // themselves, in a fixed stride
  const int32_t* xcd_begin;
  int32_t refill_min;         // refill a wave's idle lanes once at least this many are idle (>= 1)
  int32_t pool_rows;          // tally rows per workgroup, shared by its waves (0: two per wave)
  int32_t row_len;            // doubles per partial row: 4 slot_len + 8
  int32_t slot_len;           // G slots per side
  int32_t L;                  // lattice intervals per direction
  double* partial;            // n_tickets * row_len
  uint32_t key0, key1;
  int32_t exit_rule;
  int32_t dump_paths;
  double h, sqrt_h;
  double x0, x1, y0, y1, dx, dy;
  float inv_dx, inv_dy;       // 1/dx, 1/dy in float32 (production mode)
  CoefParams coef;
  const double* u_ref;        // nullable
  const int32_t* lattice;     // (L+1)^2 lattice -> knot index (for u_ref)
  double* dump;               // nullable
  uint32_t* ticket_counter;   // dynamic schedule: 8 zeroed work counters (one per XCD share when
                              // xcd_begin is set, else the first); nullptr: static stride
  // control variate
  int32_t cv_mode;            // PDD_CV_*
  int32_t cv_lut_n;
  const float* cv_params;     // network parameters (float32, PDD_MLP_PARAMS)
  const float* cv_lut;        // grad v table [n][n][2]
  float cv_lut_sx, cv_lut_sy; // (n-1)/(x1-x0), (n-1)/(y1-y0)
  // RBF interpolation (kernels built for it only): inverses of the stencil
  // interpolation matrices, S x S row-major at rbf_inv[vert * rbf_half +
  // rbf_block_offset(S)] (vert: sides on lines x = const, spacing dy)
  const double* rbf_inv;
  int64_t rbf_half;
  double rbf_c2;              // c^2
  // per-knot time steps h_i (eq. 40), device, nullable: the launch's h
  // (single launches of the generic and RBF kernels)
  const double* h_knot;
  // host only: launch the lane-per-path table kernel (the copy of the table
  // was found in the lane-read layout)
  int32_t table_lane;
};

// Extras stored after the 4 slot_len G slots of a partial row.
enum { EX_B = 0, EX_S = 1, EX_S2 = 2, EX_K = 3, EX_E = 4, EX_N = 5, EX_W = 6, EX_S_SIDE = 7, EX_COUNT = 8 };

struct FinalizeParams {
  const double* partial;
  const int32_t* ticket_begin;   // n + 1, tickets of knot k are [tb[k], tb[k+1])
  const KnotDesc* desc;
  const int32_t* knot_ij;        // 2 per knot: lattice ix, iy
  const int32_t* row_ptr;
  const int32_t* col_idx;
  const int32_t* n_paths;        // per knot
  int32_t row_len, slot_len;
  int64_t n;
  double* val;
  double* b;
  double* diag;                  // nullable
  uint32_t* ticket_counter;      // 8 counters reset to zero for the next assembly (nullable)
  // RBF interpolation (nullable: hat weights): the slots of an interface side
  // hold sums of Y phi_c(|z - z_q|); the weights are Phi^{-1} times them
  const double* rbf_inv;
  int64_t rbf_half;
};

// Launchers (defined in assemble.hip).  Return hipSuccess or the launch error.
hipError_t launch_assemble(const AsmParams& p, int precision, int grid, int block,
                           size_t lds_bytes, hipStream_t stream);
// RBF interpolation: the same launch with the kernels built for it (single
// launches; control variate none or gradient table)
hipError_t launch_assemble_rbf(const AsmParams& p, int precision, int grid, int block, size_t lds_bytes,
                               hipStream_t stream);
hipError_t assemble_occupancy_rbf(int precision, int kind, int cv_mode, int block, size_t lds_bytes,
                                  int* blocks_per_cu);
hipError_t launch_finalize(const FinalizeParams& p, hipStream_t stream);
// Training-pair collection (collect.hip).
hipError_t launch_collect(const AsmParams& P, int64_t n, int32_t paths_per_knot, int32_t points_per_path,
                          uint32_t inst, const double* u0, float* xy, float* yz, float* target, hipStream_t stream);
// Table-wide maxima of |sxx|, |sxy|, |syy| of a LUT (lut.hip): out[0..2]
// as float bit patterns, out[3] unused.  Two kernels, no memset.
// Phase II calibration: per-path records (scratch of calibrate_scratch_bytes)
// and their per-knot sums, stats[n * PDD_CAL_WIDTH]
size_t calibrate_scratch_bytes(int64_t n, int32_t n_paths);
// alpha (nullable): RBF interpolation of u0, scratch of 4 n slot_len doubles
// for the per-side coefficients (P.rbf_inv and P.rbf_c2 set)
hipError_t launch_calibrate(const AsmParams& P, int precision, int64_t n, int32_t n_paths, uint32_t inst,
                            const double* u0, double* rec, double* stats, hipStream_t stream,
                            double* alpha = nullptr, int32_t slot_len = 0);
hipError_t launch_lut_bound(const float* lut, int32_t lut_n, uint32_t* out, hipStream_t stream);
// Cell-major copy of a LUT (lut.hip): the varying fields of the table
// (info[0]) and, for read_all == 0 and at most two of them, their forms
// only (count float4 per cell, count >= 1), else all eight per cell,
// cells[(j (n-1) + i) 8 + q]; the layout goes to info[1], node 0's values
// to info[8..14].  `cells` holds (n-1)^2 cells of 128 B; info 16 words.
// bmax (nullable, 4 words): the same pass writes launch_lut_bound's maxima.
hipError_t launch_lut_cells(const float* lut, int32_t lut_n, int32_t read_all, uint32_t* info, uint32_t* bmax,
                            float4* cells, hipStream_t stream);
// Dynamic LDS bytes per workgroup for a precision, row length, block size and CV mode.
// LDS bytes of an assembly workgroup; pool_rows tally rows shared by its
// waves (0: two per wave)
size_t assemble_lds_bytes(int precision, int kind, int row_len, int block, int cv_mode, bool batch, int pool_rows,
                          bool lane = false);
// Kernel attribute query for occupancy-based grid sizing.
hipError_t assemble_occupancy(int precision, int kind, int cv_mode, bool batch, int block, size_t lds_bytes,
                              int* blocks_per_cu, bool per_knot_h = false, bool lane = false);

}  // namespace pdd
