// Training pairs for the control-variate network from the method's own paths.
//
// One thread per path (knot k, path p < paths_per_knot), float32, the same
// random stream and step as the production assembly, so the recorded points
// lie on the paths that build G and b.  The first `points_per_path` iterates
// X_n of each path are recorded with Y_n and Z_n; when the path exits at step
// K the value carried out of the patch is Z_K + Y_K u(exit), with u at the
// exit interpolated from the solved knot values u0 (hat weights on the exit
// line) or taken from the boundary datum, and each recorded point gets the
// tail score (Z_K + Y_K u(exit) - Z_n) / Y_n, whose conditional mean given
// X_n is u(X_n).  Unused record slots get a NaN target.
#include <hip/hip_runtime.h>

#include <cmath>

#include "context.h"
#include "device_common.h"

namespace pdd {

namespace {

constexpr int BLK = 256;

struct CollectArgs {
  AsmParams P;               // geometry, coefficients, step and stream parameters
  int64_t n;                 // knots
  int32_t paths_per_knot;
  int32_t points_per_path;
  const double* u0;          // solved knot values
  uint32_t inst;             // fourth Philox counter word
  float* xy;                 // 2 per record slot
  float* yz;                 // scratch: Y_n, Z_n per record slot
  float* target;             // per record slot
};

template <int KIND>
__global__ __launch_bounds__(BLK) void k_collect(CollectArgs C) {
  const AsmParams& P = C.P;
  const int64_t gid = (int64_t)blockIdx.x * BLK + threadIdx.x;
  if (gid >= C.n * C.paths_per_knot) return;
  const int64_t k = gid / C.paths_per_knot;
  const uint32_t p = (uint32_t)(gid % C.paths_per_knot);
  const KnotDesc& d = P.desc[k];
  float eb[4];
  for (int o = 0; o < 4; ++o) eb[o] = exit_threshold<KIND, float>(P.coef, P.exit_rule, P.sqrt_h, d, o);
  const int S = C.points_per_path;
  const int64_t slot0 = gid * S;
  float x = (float)d.sx, y = (float)d.sy, Y = 1.0f, Z = 0.0f;
  uint32_t j = 0;
  int recorded = 0;
  bool ex = false;
  uint32_t fl = 0;
  while (!ex) {
    const U4 r = philox10(j, p, (uint32_t)k, C.inst, P.key0, P.key1);
    float z0, z1;
    for (int half = 0; half < 2 && !ex; ++half) {
      if (half == 0) box_muller(uniform32(r.a), uniform32(r.b), z0, z1);
      else box_muller(uniform32(r.c), uniform32(r.d), z0, z1);
      if (recorded < S) {
        // the network's input: the point in the domain's unit coordinates
        C.xy[2 * (slot0 + recorded)] = (x - (float)P.x0) * (float)(1.0 / (P.x1 - P.x0));
        C.xy[2 * (slot0 + recorded) + 1] = (y - (float)P.y0) * (float)(1.0 / (P.y1 - P.y0));
        C.yz[2 * (slot0 + recorded)] = Y;
        C.yz[2 * (slot0 + recorded) + 1] = Z;
        ++recorded;
      }
      em_step<KIND, float>(P.coef, (float)P.h, (float)P.sqrt_h, z0, z1, x, y, Y, Z);
      fl = exit_sides<KIND, float>(P.coef, P.exit_rule, (float)P.sqrt_h, d.line, eb, x, y);
      ex = fl != 0;
    }
    ++j;
    if (!ex && 2 * j >= (1u << 24) - 2) break;   // safety cap (forced exit below)
  }
  if (!ex) fl = 15u;
  const bool fE = fl & 1u, fN = (fl >> 1) & 1u, fW = (fl >> 2) & 1u, fS = (fl >> 3) & 1u;
  const int o = choose_side<float>(x, y, fE, fN, fW, fS, d.line);
  const bool vert = (o == 0 || o == 2);
  const float along = vert ? y : x;
  const float lpos = (float)d.line[o];
  float uex;
  if ((d.bmask >> o) & 1) {
    const float a0 = vert ? (float)P.y0 : (float)P.x0, a1 = vert ? (float)P.y1 : (float)P.x1;
    const float pa = fminf(fmaxf(along, a0), a1);
    uex = vert ? g_at<KIND>(lpos, pa) : g_at<KIND>(pa, lpos);
  } else {
    int q0;
    float w;
    hat_weights<float, false>(along, vert ? (float)P.y0 : (float)P.x0, vert ? P.dy : P.dx,
                              vert ? P.inv_dy : P.inv_dx, d.clo[o], d.chi[o], q0, w);
    uex = 0.0f;
    for (int e = 0; e < 2; ++e) {
      const int q = q0 + e;
      const float wq = e == 0 ? 1.0f - w : w;
      float val;
      if (q == 0 || q == P.L) {
        const float qc = vert ? (float)P.y0 + (float)q * (float)P.dy : (float)P.x0 + (float)q * (float)P.dx;
        val = vert ? g_at<KIND>(lpos, qc) : g_at<KIND>(qc, lpos);
      } else {
        const int lx = vert ? d.at[o] : q, ly = vert ? q : d.at[o];
        val = (float)C.u0[P.lattice[(size_t)ly * (P.L + 1) + lx]];
      }
      uex += wq * val;
    }
  }
  const float vout = (isnan(x) || isnan(y)) ? NAN : Z + Y * uex;
  for (int n = 0; n < S; ++n) {
    const int64_t sl = slot0 + n;
    if (n < recorded) {
      const float Yn = C.yz[2 * sl], Zn = C.yz[2 * sl + 1];
      C.target[sl] = (vout - Zn) / Yn;
    } else {
      C.target[sl] = NAN;
      C.xy[2 * sl] = 0.0f;
      C.xy[2 * sl + 1] = 0.0f;
    }
  }
}

}  // namespace

hipError_t launch_collect(const AsmParams& P, int64_t n, int32_t paths_per_knot, int32_t points_per_path,
                          uint32_t inst, const double* u0, float* xy, float* yz, float* target, hipStream_t stream) {
  CollectArgs C;
  C.inst = inst;
  C.P = P;
  C.n = n;
  C.paths_per_knot = paths_per_knot;
  C.points_per_path = points_per_path;
  C.u0 = u0;
  C.xy = xy;
  C.yz = yz;
  C.target = target;
  const int64_t threads = n * paths_per_knot;
  const unsigned grid = (unsigned)((threads + BLK - 1) / BLK);
  switch (P.coef.kind) {
    case PDD_COEF_POISSON: hipLaunchKernelGGL(k_collect<PDD_COEF_POISSON>, dim3(grid), dim3(BLK), 0, stream, C); break;
    case PDD_COEF_VARCOEF: hipLaunchKernelGGL(k_collect<PDD_COEF_VARCOEF>, dim3(grid), dim3(BLK), 0, stream, C); break;
    case PDD_COEF_AMPLITUDE: hipLaunchKernelGGL(k_collect<PDD_COEF_AMPLITUDE>, dim3(grid), dim3(BLK), 0, stream, C); break;
    case PDD_COEF_LUT: hipLaunchKernelGGL(k_collect<PDD_COEF_LUT>, dim3(grid), dim3(BLK), 0, stream, C); break;
    case PDD_COEF_CONSTSOL: hipLaunchKernelGGL(k_collect<PDD_COEF_CONSTSOL>, dim3(grid), dim3(BLK), 0, stream, C); break;
    case PDD_COEF_EQ43: hipLaunchKernelGGL(k_collect<PDD_COEF_EQ43>, dim3(grid), dim3(BLK), 0, stream, C); break;
    default: hipLaunchKernelGGL(k_collect<PDD_COEF_EXITTIME>, dim3(grid), dim3(BLK), 0, stream, C); break;
  }
  return hipGetLastError();
}

}  // namespace pdd
