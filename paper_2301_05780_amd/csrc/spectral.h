// Pseudospectral subdomain solves (Sec. 3.3, Sec. 5.1): host tables and
// kernel launchers.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include <hip/hip_runtime.h>

#include "kernels.h"
#include "pdd.h"

namespace pdd {

constexpr int SPEC_T = 64;          // tile edge of the dense products (p + 1 <= 64)
constexpr int SPEC_MAX_P = 63;

// Collocation tables of degree p on the reference interval [-1, 1], float64,
// matrices row-major and zero-padded to SPEC_T x SPEC_T:
//   nodes[p+1]  t_j = -cos(pi j / p);  bw[p+1] barycentric weights
//   D           first-derivative matrix
//   D2b[2 (p-1)] the boundary columns D2[i][0], D2[i][p] of D2 = D D for the
//               interior rows i = 1 .. p-1
//   V, Vinv, lam  D2[1..p-1][1..p-1] = V diag(lam) Vinv (lam padded with -1)
struct SpectralTables {
  int32_t p = 0;
  std::vector<double> nodes, bw, D, D2b, V, Vinv, lam;
  double decomp_residual = 0, inverse_residual = 0;
};

bool spectral_tables(int32_t p, SpectralTables& t, std::string& err);

// Device copies of the tables of one p.
struct SpecDev {
  const double* nodes;
  const double* bw;
  const double* D;
  const double* D2b;
  const double* V;
  const double* Vinv;
  const double* lam;
};

// One subdomain-solve launch: AsmParams supplies the geometry (lattice map,
// spacings, domain), the coefficients and, with RBF side values, the stencil
// inverses.
struct SpecArgs {
  AsmParams P;
  SpecDev T;
  int32_t p;
  int32_t H;
  int32_t m;
  int32_t ext;
  int32_t rbf;                 // 0: hat side values, 1: RBF cardinal side values
  double ax, ay, c;            // 1/2 a_xx (2/S)^2, 1/2 a_yy (2/S)^2, reaction
  const double* u_knots;
  double* grid;                // [H^2][3][p+1][p+1]
};

hipError_t launch_spectral_solve(const SpecArgs& A, hipStream_t stream);
hipError_t launch_spectral_eval(const SpecDev& T, int32_t p, int32_t H, double x0, double x1, double y0, double y1,
                                const double* grid, int64_t n_pts, const double* xy, int32_t lut_n, double* u,
                                double* grad, float* grad_lut, hipStream_t stream);
hipError_t launch_lut_field_range(const float* lut, int64_t nodes, double* out, hipStream_t stream);

}  // namespace pdd
