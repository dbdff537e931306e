// Phase II calibration (Sec. 4.1-4.2, eqs. 32-39): mixed Gobet-Menozzi /
// Euler-Maruyama trajectories scored with the warm-up solution.
//
// One lane per path (knot k, path p < N0'), the assembly's random stream,
// step and exit rules; waves are persistent and claim path ids from a
// device counter as their lanes fall idle.  A path runs until it leaves the
// closed patch (the naive exit); on the way, the first step whose iterate
// is not strictly inside the Gobet-Menozzi-shrunk patch is its GM exit.
// Each exit is
// resolved as in the assembly (side choice, projection, hat weights) and
// scored with u0: phi = Z_K + Y_K u0(P_K), u0 interpolated from the warm-up
// knot values on interface sides and the boundary datum g on the domain
// boundary.  xi is the control variate (eq. 37, with the gradient table) at
// the GM exit.  Each path writes (phi_EM - phi_GM, phi_GM, xi, K_GM, K_EM);
// a second kernel sums a knot's paths in a fixed order into
//   sum(phi_EM - phi_GM), sum phi_GM, sum phi_GM^2, sum xi, sum xi^2,
//   sum phi_GM xi, sum K_GM, sum K_EM.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <type_traits>

#include "context.h"
#include "device_common.h"
#include "net_grad.h"

namespace pdd {

namespace {

constexpr int BLK = 256;
constexpr int REC = 5;               // per-path record width

struct CalArgs {
  AsmParams P;                       // geometry, coefficients, step, stream, gradient table
  int64_t n;                         // knots
  int32_t n_paths;                   // N0' paths per knot
  const double* u0;                  // warm-up knot values
  uint32_t inst;                     // fourth Philox counter word
  double* rec;                       // REC doubles per path
  unsigned long long* counter;       // next path id (zeroed before the launch)
  // RBF interpolation of u0 (nullable: hat weights): per knot and side the
  // coefficients alpha = Phi^{-1} v of the interpolant of the stencil values
  // v (knot values, g at boundary lattice points), slot_len per side
  const double* alpha;
  int32_t slot_len;
};

// u0 at the exit point resolved from the flagged sides `fl` (bit o: side o)
template <int KIND, typename R, bool F64>
__device__ R exit_value(const AsmParams& P, const KnotDesc& d, const double* u0, const double* alpha, int SL, R x,
                        R y, uint32_t fl) {
  const bool fE = fl & 1u, fN = (fl >> 1) & 1u, fW = (fl >> 2) & 1u, fS = (fl >> 3) & 1u;
  const int o = choose_side<R>(x, y, fE, fN, fW, fS, d.line);
  const bool vert = (o == 0 || o == 2);
  const R along = vert ? y : x;
  const R lpos = (R)d.line[o];
  if ((d.bmask >> o) & 1) {
    const R a0 = vert ? (R)P.y0 : (R)P.x0, a1 = vert ? (R)P.y1 : (R)P.x1;
    const R pa = fmin(fmax(along, a0), a1);
    return vert ? g_at<KIND>(lpos, pa) : g_at<KIND>(pa, lpos);
  }
  if (alpha) {
    // RBF: u0(z) = sum_i alpha_i phi_c(|z - z_i|) over the side's stencil,
    // z the exit point clamped to the stencil, in float64
    const double da = vert ? P.dy : P.dx;
    const double a0 = vert ? P.y0 : P.x0;
    const int clo = d.clo[o], S = d.chi[o] - clo + 1;
    const double zd = fmin(fmax(((double)along - a0) / da, (double)clo), (double)d.chi[o]) * da;
    const double* a = alpha + ((size_t)d.knot * 4 + o) * SL;
    double acc = 0.0;
    for (int i = 0; i < S; ++i) {
      const double rr = zd - (double)(clo + i) * da;
      acc = fma(a[i], rsqrt_f64(fma(rr, rr, P.rbf_c2)), acc);
    }
    return (R)acc;
  }
  int q0;
  R w;
  hat_weights<R, F64>(along, vert ? (R)P.y0 : (R)P.x0, vert ? P.dy : P.dx, vert ? P.inv_dy : P.inv_dx, d.clo[o],
                      d.chi[o], q0, w);
  R val = 0;
  for (int e = 0; e < 2; ++e) {
    const int q = q0 + e;
    R v;
    if (q == 0 || q == P.L) {
      const R qc = vert ? (R)P.y0 + (R)q * (R)P.dy : (R)P.x0 + (R)q * (R)P.dx;
      v = vert ? g_at<KIND>(lpos, qc) : g_at<KIND>(qc, lpos);
    } else {
      const int lx = vert ? d.at[o] : q, ly = vert ? q : d.at[o];
      v = (R)u0[P.lattice[(size_t)ly * (P.L + 1) + lx]];
    }
    {
#pragma clang fp contract(off)
      val = val + (e == 0 ? (R)1 - w : w) * v;
    }
  }
  return val;
}

// Persistent: each wave takes path ids from a device counter, a batch for
// its idle lanes at a time (once at least REFILL lanes are idle, or all of
// them), so a lane whose path ended starts the next one instead of waiting
// for the longest path of its wave.  A path's arithmetic is independent of
// which lane runs it, so the records do not depend on the schedule.
constexpr int REFILL = 16;
constexpr int EXIT_BATCH = 16;       // waiting exits that trigger their evaluation

template <int KIND, bool F64, bool CVON>
__global__ __launch_bounds__(BLK) void k_calibrate(CalArgs C) {
  using R = typename std::conditional<F64, double, float>::type;
  const AsmParams& P = C.P;
  const int lane = threadIdx.x & 63;
  const int64_t total = C.n * C.n_paths;
  const R h = (R)P.h, sq = (R)P.sqrt_h;
  bool active = false, exhausted = false;
  int64_t gid = 0, k = 0;
  uint32_t p = 0;
  R egm[4], env[4];
  const double* line = nullptr;      // the knot's side lines (global; read by the table family's GM test)
  R x = 0, y = 0, Y = 0, Z = 0, Xi = 0;
  R phi_gm = 0, xi_gm = 0, phi_em = 0;
  uint32_t K = 0, K_gm = 0, j = 0;
  bool gm_done = false;
  // exits waiting for their u0 value: the GM exit's state, and the naive
  // exit (the path's final state, the lane stepping no further)
  bool pgm = false, pem = false;
  R gmx = 0, gmy = 0, gmY = 0, gmZ = 0;
  uint32_t gmfl = 0, emfl = 0;
  while (true) {
    // ---- refill idle lanes with the next path ids -----------------------
    const uint64_t idle = __ballot(!active);
    const int n_idle = __popcll(idle);
    if (!exhausted && idle != 0 && (n_idle >= REFILL || idle == ~0ull)) {
      unsigned long long base = 0;
      if (lane == 0) base = atomicAdd(C.counter, (unsigned long long)n_idle);
      base = ((unsigned long long)__builtin_amdgcn_readfirstlane((int)(base >> 32)) << 32) |
             (unsigned)__builtin_amdgcn_readfirstlane((int)(base & 0xffffffffull));
      if ((int64_t)(base + n_idle) >= total) exhausted = true;
      if (!active) {
        const int64_t g = (int64_t)base + __popcll(idle & ((1ull << lane) - 1ull));
        if (g < total) {
          gid = g;
          k = g / C.n_paths;
          p = (uint32_t)(g % C.n_paths);
          const KnotDesc d = P.desc[k];
          for (int o = 0; o < 4; ++o) {
            egm[o] = exit_threshold<KIND, R>(P.coef, PDD_EXIT_GM, P.sqrt_h, d, o);
            env[o] = exit_threshold<KIND, R>(P.coef, PDD_EXIT_NAIVE, P.sqrt_h, d, o);
          }
          line = P.desc[k].line;
          x = (R)d.sx; y = (R)d.sy; Y = 1; Z = 0; Xi = 0;
          phi_gm = 0; xi_gm = 0; phi_em = 0;
          K = 0; K_gm = 0; j = 0;
          gm_done = false;
          active = true;
        }
      }
    }
    if (__ballot(active) == 0) {
      if (exhausted) break;
      continue;
    }
    // ---- one draw, up to two steps (lanes whose path has not ended) ------
    if (active && !pem) {
      const U4 r = philox10(j, p, (uint32_t)k, C.inst, P.key0, P.key1);
      for (int half = 0; half < 2 && !pem; ++half) {
        R z0, z1;
        if constexpr (F64) box_muller(uniform64(half ? r.c : r.a), uniform64(half ? r.d : r.b), z0, z1);
        else box_muller(uniform32(half ? r.c : r.a), uniform32(half ? r.d : r.b), z0, z1);
        R gx = 0, gy = 0;
        if constexpr (CVON) grad_lut(P, x, y, gx, gy);
        em_step<KIND, R, CVON>(P.coef, h, sq, z0, z1, x, y, Y, Z, gx, gy, &Xi);
        ++K;
        if (!gm_done) {
          const uint32_t fl = exit_sides<KIND, R>(P.coef, PDD_EXIT_GM, sq, line, egm, x, y);
          if (fl) {
            gmx = x; gmy = y; gmY = Y; gmZ = Z; gmfl = fl;
            xi_gm = Xi;
            K_gm = K;
            gm_done = true;
            pgm = true;
          }
        }
        const uint32_t fl = exit_sides<KIND, R>(P.coef, PDD_EXIT_NAIVE, sq, line, env, x, y);
        if (fl) {
          emfl = fl;
          pem = true;
        }
      }
      ++j;
      if (!pem && 2 * j >= (1u << 24) - 2) {      // step cap: every side flagged
        if (!gm_done) {
          gmx = x; gmy = y; gmY = Y; gmZ = Z; gmfl = 15u;
          xi_gm = Xi;
          K_gm = K;
          gm_done = true;
          pgm = true;
        }
        emfl = 15u;
        pem = true;
      }
    }
    // ---- exit values, for the waiting exits together -----------------------
    // u0 at an exit (a loop over the stencil with RBF weights) runs once
    // enough lanes wait for it, or when no lane can step any more, so that
    // the wave does not take that loop for every single exit.
    const uint64_t waiting = __ballot(pgm || pem);
    if (waiting != 0 && (__popcll(waiting) >= EXIT_BATCH || __ballot(active && !pem) == 0)) {
      if (pgm) {
        const KnotDesc d = P.desc[k];
        phi_gm = gmZ + gmY * exit_value<KIND, R, F64>(P, d, C.u0, C.alpha, C.slot_len, gmx, gmy, gmfl);
        pgm = false;
      }
      if (pem) {
        const KnotDesc d = P.desc[k];
        phi_em = Z + Y * exit_value<KIND, R, F64>(P, d, C.u0, C.alpha, C.slot_len, x, y, emfl);
        double* out = C.rec + gid * REC;
        out[0] = (double)phi_em - (double)phi_gm;
        out[1] = (double)phi_gm;
        out[2] = (double)xi_gm;
        out[3] = (double)K_gm;
        out[4] = (double)K;
        pem = false;
        active = false;
      }
    }
  }
}

// The RBF coefficients of u0 on every interface side: one wave per (knot,
// side); the stencil values in LDS, then alpha_i = sum_j (Phi^{-1})_ji v_j
// (Phi^{-1} symmetric: lane i reads column i).
template <int KIND>
__global__ __launch_bounds__(256) void k_calib_alpha(AsmParams P, int64_t n, int32_t SL, const double* u0,
                                                     double* alpha) {
  extern __shared__ double vs[];
  const int lane = threadIdx.x & 63;
  const int64_t w = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (w >= 4 * n) return;
  const int64_t k = w >> 2;
  const int o = (int)(w & 3);
  const KnotDesc& d = P.desc[k];
  if ((d.bmask >> o) & 1) return;
  double* v = vs + (size_t)(threadIdx.x >> 6) * SL;
  const bool vert = (o == 0 || o == 2);
  const int clo = d.clo[o], S = d.chi[o] - clo + 1;
  for (int i = lane; i < S; i += 64) {
    const int q = clo + i;
    if (q == 0 || q == P.L) {
      const double qc = vert ? P.y0 + (double)q * P.dy : P.x0 + (double)q * P.dx;
      v[i] = vert ? g_at<KIND>(d.line[o], qc) : g_at<KIND>(qc, d.line[o]);
    } else {
      const int lx = vert ? d.at[o] : q, ly = vert ? q : d.at[o];
      v[i] = u0[P.lattice[(size_t)ly * (P.L + 1) + lx]];
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
  const double* Mi = P.rbf_inv + (vert ? P.rbf_half : 0) + rbf_block_offset(S);
  for (int i = lane; i < S; i += 64) {
    double acc = 0.0;
    for (int j = 0; j < S; ++j) acc = fma(Mi[(size_t)j * S + i], v[j], acc);
    alpha[(size_t)w * SL + i] = acc;
  }
}

template <int KIND>
hipError_t launch_alpha_kind(const AsmParams& P, int64_t n, int32_t SL, const double* u0, double* alpha,
                             hipStream_t stream) {
  const int64_t waves = 4 * n;
  const unsigned grid = (unsigned)((waves + 3) / 4);
  const size_t lds = (size_t)4 * SL * sizeof(double);
  hipLaunchKernelGGL((k_calib_alpha<KIND>), dim3(grid), dim3(256), lds, stream, P, n, SL, u0, alpha);
  return hipGetLastError();
}

hipError_t launch_alpha(const AsmParams& P, int64_t n, int32_t SL, const double* u0, double* alpha,
                        hipStream_t stream) {
  switch (P.coef.kind) {
    case PDD_COEF_POISSON: return launch_alpha_kind<PDD_COEF_POISSON>(P, n, SL, u0, alpha, stream);
    case PDD_COEF_VARCOEF: return launch_alpha_kind<PDD_COEF_VARCOEF>(P, n, SL, u0, alpha, stream);
    case PDD_COEF_AMPLITUDE: return launch_alpha_kind<PDD_COEF_AMPLITUDE>(P, n, SL, u0, alpha, stream);
    case PDD_COEF_LUT: return launch_alpha_kind<PDD_COEF_LUT>(P, n, SL, u0, alpha, stream);
    case PDD_COEF_CONSTSOL: return launch_alpha_kind<PDD_COEF_CONSTSOL>(P, n, SL, u0, alpha, stream);
    case PDD_COEF_EQ43: return launch_alpha_kind<PDD_COEF_EQ43>(P, n, SL, u0, alpha, stream);
    default: return launch_alpha_kind<PDD_COEF_EXITTIME>(P, n, SL, u0, alpha, stream);
  }
}

__global__ void k_zero_counter(unsigned long long* c) {
  if (threadIdx.x == 0) *c = 0ull;
}

// Per-knot sums of the path records: one wave per knot, lane l takes paths
// l, l + 64, ... in order, then a fixed butterfly across the lanes.
__global__ __launch_bounds__(BLK) void k_calibrate_sum(const double* __restrict__ rec, int64_t n, int32_t n_paths,
                                                       double* __restrict__ stats) {
  const int lane = threadIdx.x & 63;
  const int64_t k = (int64_t)blockIdx.x * (BLK / 64) + (threadIdx.x >> 6);
  if (k >= n) return;
  double s[PDD_CAL_WIDTH] = {};
  for (int32_t p = lane; p < n_paths; p += 64) {
    const double* r = rec + ((size_t)k * n_paths + p) * REC;
    s[0] += r[0];
    s[1] += r[1];
    s[2] += r[1] * r[1];
    s[3] += r[2];
    s[4] += r[2] * r[2];
    s[5] += r[1] * r[2];
    s[6] += r[3];
    s[7] += r[4];
  }
#pragma unroll
  for (int i = 0; i < PDD_CAL_WIDTH; ++i) {
    for (int off = 32; off > 0; off >>= 1) s[i] += __shfl_xor(s[i], off, 64);
  }
  if (lane < PDD_CAL_WIDTH) {
    double v = s[0];
#pragma unroll
    for (int i = 1; i < PDD_CAL_WIDTH; ++i) if (lane == i) v = s[i];
    stats[k * PDD_CAL_WIDTH + lane] = v;
  }
}

template <int KIND, bool F64>
hipError_t launch_kind(const CalArgs& C, bool cv, hipStream_t stream) {
  // persistent grid: enough workgroups to fill the device, fewer for small runs
  const int64_t threads = C.n * C.n_paths;
  const unsigned grid = (unsigned)std::min<int64_t>((threads + BLK - 1) / BLK, 2048);
  if (cv) hipLaunchKernelGGL((k_calibrate<KIND, F64, true>), dim3(grid), dim3(BLK), 0, stream, C);
  else hipLaunchKernelGGL((k_calibrate<KIND, F64, false>), dim3(grid), dim3(BLK), 0, stream, C);
  return hipGetLastError();
}

template <bool F64>
hipError_t launch_prec(const CalArgs& C, bool cv, hipStream_t stream) {
  switch (C.P.coef.kind) {
    case PDD_COEF_POISSON: return launch_kind<PDD_COEF_POISSON, F64>(C, cv, stream);
    case PDD_COEF_VARCOEF: return launch_kind<PDD_COEF_VARCOEF, F64>(C, cv, stream);
    case PDD_COEF_AMPLITUDE: return launch_kind<PDD_COEF_AMPLITUDE, F64>(C, cv, stream);
    case PDD_COEF_LUT: return launch_kind<PDD_COEF_LUT, F64>(C, cv, stream);
    case PDD_COEF_CONSTSOL: return launch_kind<PDD_COEF_CONSTSOL, F64>(C, cv, stream);
    case PDD_COEF_EQ43: return launch_kind<PDD_COEF_EQ43, F64>(C, cv, stream);
    default: return launch_kind<PDD_COEF_EXITTIME, F64>(C, cv, stream);
  }
}

}  // namespace

// the path records, then the path counter (256-byte aligned)
size_t calibrate_scratch_bytes(int64_t n, int32_t n_paths) {
  return ((size_t)n * n_paths * REC * sizeof(double) + 255) / 256 * 256 + 256;
}

hipError_t launch_calibrate(const AsmParams& P, int precision, int64_t n, int32_t n_paths, uint32_t inst,
                            const double* u0, double* rec, double* stats, hipStream_t stream, double* alpha,
                            int32_t slot_len) {
  CalArgs C;
  C.alpha = alpha;
  C.slot_len = slot_len;
  if (alpha) {
    const hipError_t e = launch_alpha(P, n, slot_len, u0, alpha, stream);
    if (e != hipSuccess) return e;
  }
  C.P = P;
  C.n = n;
  C.n_paths = n_paths;
  C.u0 = u0;
  C.inst = inst;
  C.rec = rec;
  C.counter = reinterpret_cast<unsigned long long*>(reinterpret_cast<char*>(rec) +
                                                    ((size_t)n * n_paths * REC * sizeof(double) + 255) / 256 * 256);
  hipLaunchKernelGGL(k_zero_counter, dim3(1), dim3(64), 0, stream, C.counter);
  const bool cv = P.cv_mode == PDD_CV_GRAD_LUT;
  hipError_t e = precision == PDD_FP64_SAME_STREAM ? launch_prec<true>(C, cv, stream) : launch_prec<false>(C, cv, stream);
  if (e != hipSuccess) return e;
  const unsigned grid = (unsigned)((n + BLK / 64 - 1) / (BLK / 64));
  hipLaunchKernelGGL(k_calibrate_sum, dim3(grid), dim3(BLK), 0, stream, rec, n, n_paths, stats);
  return hipGetLastError();
}

}  // namespace pdd
