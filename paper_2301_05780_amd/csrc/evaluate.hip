// Point values inside the subdomains once the knot values are known.
//
// Each subdomain square is an independent Dirichlet problem for (6) whose
// sides carry u: the solved knot values interpolated along the grid lines on
// interfaces, g on the domain boundary (Sec. 3.3).  The value at a point is
// the Feynman-Kac expectation of eq. (8) over paths started there and
// absorbed at the square's boundary, with the assembly's Euler-Maruyama step,
// exit rules and side choice; the exit value is g at the projection on a
// boundary side, else the hat interpolation of the side line's lattice values
// with the along-side coordinate clamped to the side.
//
// One wave per point: lane l integrates paths l, l + 64, ... of the point in
// turn and keeps float64 sums of the score and its square; a fixed butterfly
// combines the lanes (deterministic).  Stream: counter (draw, path, point,
// instance + 2^31).
#include <hip/hip_runtime.h>

#include <cmath>
#include <type_traits>

#include "context.h"
#include "device_common.h"

namespace pdd {

namespace {

constexpr int BLK = 256;
constexpr uint32_t MAX_STEPS = (1u << 24) - 2;
constexpr uint32_t POINT_STREAM = 1u << 31;

struct EvalArgs {
  AsmParams P;                 // geometry, coefficients, step and stream parameters
  int32_t H, m;                // subdomains per direction, lattice intervals per side
  int64_t n_pts;
  int64_t n_paths;
  uint32_t inst;               // fourth counter word (POINT_STREAM already added)
  const double* xy;
  const double* u_knots;
  double* u;
  double* se;
};

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// u on the grid line of side o of the square: g on a boundary line, else hat
// interpolation of the lattice values (points of the domain boundary take g).
template <int KIND, typename R, bool F64>
__device__ __forceinline__ R line_value(const EvalArgs& A, const KnotDesc& d, int o, R along) {
  const AsmParams& P = A.P;
  const bool vert = (o == 0 || o == 2);
  const R lpos = (R)d.line[o];
  const int lo = d.clo[o], hi = d.chi[o];
  if ((d.bmask >> o) & 1) {
    const R a_lo = vert ? (R)(P.y0 + (double)lo * P.dy) : (R)(P.x0 + (double)lo * P.dx);
    const R a_hi = vert ? (R)(P.y0 + (double)hi * P.dy) : (R)(P.x0 + (double)hi * P.dx);
    const R pa = fmin(fmax(along, a_lo), a_hi);
    return vert ? g_at<KIND>(lpos, pa) : g_at<KIND>(pa, lpos);
  }
  int q0;
  R w;
  hat_weights<R, F64>(along, vert ? (R)P.y0 : (R)P.x0, vert ? P.dy : P.dx, vert ? P.inv_dy : P.inv_dx, lo, hi, q0, w);
  R v[2];
#pragma unroll
  for (int e = 0; e < 2; ++e) {
    const int q = q0 + e;
    if (q == 0 || q == P.L) {
      const R qc = vert ? (R)P.y0 + (R)q * (R)P.dy : (R)P.x0 + (R)q * (R)P.dx;
      v[e] = vert ? g_at<KIND>(lpos, qc) : g_at<KIND>(qc, lpos);
    } else {
      const int at = d.at[o];
      const int lx = vert ? at : q, ly = vert ? q : at;
      v[e] = (R)A.u_knots[P.lattice[(size_t)ly * (P.L + 1) + lx]];
    }
  }
  R out;
  {
#pragma clang fp contract(off)
    out = ((R)1 - w) * v[0] + w * v[1];
  }
  return out;
}

template <int KIND, bool F64>
__global__ __launch_bounds__(BLK) void k_eval(EvalArgs A) {
  using R = typename std::conditional<F64, double, float>::type;
  const AsmParams& P = A.P;
  const int lane = threadIdx.x & 63;
  const int64_t pt = (int64_t)blockIdx.x * (BLK / 64) + (threadIdx.x >> 6);
  if (pt >= A.n_pts) return;
  const double px = A.xy[2 * pt], py = A.xy[2 * pt + 1];
  if (!(px >= P.x0 && px <= P.x1 && py >= P.y0 && py <= P.y1)) {
    if (lane == 0) {
      A.u[pt] = NAN;
      if (A.se) A.se[pt] = NAN;
    }
    return;
  }
  // the square holding the point and its description as a "patch"
  const int m = A.m, H = A.H, L = P.L;
  const int a = max(min((int)floor((px - P.x0) / (P.dx * (double)m)), H - 1), 0);
  const int c = max(min((int)floor((py - P.y0) / (P.dy * (double)m)), H - 1), 0);
  const int xlo = a * m, xhi = xlo + m, ylo = c * m, yhi = ylo + m;
  KnotDesc d;
  d.sx = px;
  d.sy = py;
  d.line[0] = P.x0 + (double)xhi * P.dx;
  d.line[1] = P.y0 + (double)yhi * P.dy;
  d.line[2] = P.x0 + (double)xlo * P.dx;
  d.line[3] = P.y0 + (double)ylo * P.dy;
  d.at[0] = xhi; d.at[1] = yhi; d.at[2] = xlo; d.at[3] = ylo;
  d.clo[0] = d.clo[2] = ylo; d.chi[0] = d.chi[2] = yhi;
  d.clo[1] = d.clo[3] = xlo; d.chi[1] = d.chi[3] = xhi;
  d.bmask = (xhi == L ? 1 : 0) | (yhi == L ? 2 : 0) | (xlo == 0 ? 4 : 0) | (ylo == 0 ? 8 : 0);
  d.knot = (int32_t)pt;

  // a point on the square's boundary takes the line value directly
  const bool on_v = px == d.line[2] || px == d.line[0];
  const bool on_h = py == d.line[3] || py == d.line[1];
  if (on_v || on_h) {
    if (lane == 0) {
      const int o = on_v ? (px == d.line[2] ? 2 : 0) : (py == d.line[3] ? 3 : 1);
      A.u[pt] = (double)line_value<KIND, R, F64>(A, d, o, on_v ? (R)py : (R)px);
      if (A.se) A.se[pt] = 0.0;
    }
    return;
  }

  R e[4];
#pragma unroll
  for (int o = 0; o < 4; ++o) e[o] = exit_threshold<KIND, R>(P.coef, P.exit_rule, P.sqrt_h, d, o);
  const R h = (R)P.h, sq = (R)P.sqrt_h;
  double s1 = 0.0, s2 = 0.0;
  for (int64_t p = lane; p < A.n_paths; p += 64) {
    R x = (R)px, y = (R)py, Y = (R)1, Z = (R)0;
    uint32_t j = 0, fl = 0;
    while (fl == 0) {
      const U4 r = philox10(j, (uint32_t)p, (uint32_t)pt, A.inst, P.key0, P.key1);
      R z0, z1;
      if constexpr (F64) box_muller(uniform64(r.a), uniform64(r.b), z0, z1);
      else box_muller(uniform32(r.a), uniform32(r.b), z0, z1);
      em_step<KIND, R>(P.coef, h, sq, z0, z1, x, y, Y, Z);
      fl = exit_sides<KIND, R>(P.coef, P.exit_rule, sq, d.line, e, x, y);
      if (fl == 0) {
        if constexpr (F64) box_muller(uniform64(r.c), uniform64(r.d), z0, z1);
        else box_muller(uniform32(r.c), uniform32(r.d), z0, z1);
        em_step<KIND, R>(P.coef, h, sq, z0, z1, x, y, Y, Z);
        fl = exit_sides<KIND, R>(P.coef, P.exit_rule, sq, d.line, e, x, y);
      }
      ++j;
      if (fl == 0 && 2 * j >= MAX_STEPS) fl = 15u;
    }
    const int o = choose_side<R>(x, y, fl & 1u, (fl >> 1) & 1u, (fl >> 2) & 1u, (fl >> 3) & 1u, d.line);
    const bool vert = (o == 0 || o == 2);
    R s;
    if (isnan(x) || isnan(y)) {
      s = (R)NAN;
    } else {
      const R val = line_value<KIND, R, F64>(A, d, o, vert ? y : x);
      {
#pragma clang fp contract(off)
        s = Z + Y * val;
      }
    }
    s1 += (double)s;
    s2 += (double)s * (double)s;
  }
  s1 = wave_sum(s1);
  s2 = wave_sum(s2);
  if (lane == 0) {
    const double N = (double)A.n_paths;
    const double mean = s1 / N;
    A.u[pt] = mean;
    if (A.se) A.se[pt] = sqrt(fmax(s2 / N - mean * mean, 0.0) / N);
  }
}

template <bool F64>
hipError_t launch_kind(const EvalArgs& A, unsigned grid, hipStream_t stream) {
  switch (A.P.coef.kind) {
    case PDD_COEF_POISSON: hipLaunchKernelGGL((k_eval<PDD_COEF_POISSON, F64>), dim3(grid), dim3(BLK), 0, stream, A); break;
    case PDD_COEF_VARCOEF: hipLaunchKernelGGL((k_eval<PDD_COEF_VARCOEF, F64>), dim3(grid), dim3(BLK), 0, stream, A); break;
    case PDD_COEF_AMPLITUDE: hipLaunchKernelGGL((k_eval<PDD_COEF_AMPLITUDE, F64>), dim3(grid), dim3(BLK), 0, stream, A); break;
    case PDD_COEF_LUT: hipLaunchKernelGGL((k_eval<PDD_COEF_LUT, F64>), dim3(grid), dim3(BLK), 0, stream, A); break;
    case PDD_COEF_CONSTSOL: hipLaunchKernelGGL((k_eval<PDD_COEF_CONSTSOL, F64>), dim3(grid), dim3(BLK), 0, stream, A); break;
    case PDD_COEF_EQ43: hipLaunchKernelGGL((k_eval<PDD_COEF_EQ43, F64>), dim3(grid), dim3(BLK), 0, stream, A); break;
    default: hipLaunchKernelGGL((k_eval<PDD_COEF_EXITTIME, F64>), dim3(grid), dim3(BLK), 0, stream, A); break;
  }
  return hipGetLastError();
}

}  // namespace

pdd_status run_eval_subdomain(pdd_ctx* ctx, const pdd_coeffs& co, const pdd_partition& part, const pdd_knots& kn,
                              const double* u_knots, int64_t n_pts, const double* xy, const pdd_run& run, double* u,
                              double* se) {
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return check_hip(ctx, e, "hipSetDevice");
  GeoCache* gc = nullptr;
  pdd_status st = get_geometry(ctx, part, kn, &gc);
  if (st != PDD_OK) return st;
  if ((st = get_lattice(ctx, gc)) != PDD_OK) return st;
  EvalArgs A;
  fill_asm_params(*gc, co, run, A.P);
  if ((st = prepare_lut_bound(ctx, co, run, A.P, false)) != PDD_OK) return st;
  A.H = part.H;
  A.m = kn.m;
  A.n_pts = n_pts;
  A.n_paths = run.n_paths;
  A.inst = run.instance + POINT_STREAM;
  A.xy = xy;
  A.u_knots = u_knots;
  A.u = u;
  A.se = se;
  const unsigned grid = (unsigned)((n_pts + BLK / 64 - 1) / (BLK / 64));
  e = run.precision == PDD_FP64_SAME_STREAM ? launch_kind<true>(A, grid, ctx->stream)
                                            : launch_kind<false>(A, grid, ctx->stream);
  return check_hip(ctx, e, "launch eval_subdomain");
}

}  // namespace pdd
