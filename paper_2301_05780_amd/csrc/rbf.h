// Host side of the RBF cardinal interpolation (Sec. 2.1, eqs. 1-5; Sec. 5.1
// for the shape parameter): inverse-multiquadric interpolation matrices of
// equispaced side stencils, their inverses, and the shape parameter that
// reaches a given condition number.
#pragma once

#include <cstdint>
#include <vector>

#include "kernels.h"
#include "pdd.h"

namespace pdd {

// Inverses of Phi_ij = 1 / sqrt(((i - j) d)^2 + c^2) for S = 1 .. slot_len
// points, d = dx in the first half of `tab` (horizontal sides, along x) and
// d = dy in the second (vertical sides, along y); each block row-major and
// exactly symmetric.  `half` receives the length of one half.  False when a
// matrix is not positive definite to float64 working accuracy (a squared
// Cholesky pivot below 1e-14 of its diagonal entry).
bool rbf_inverse_table(int32_t slot_len, double dx, double dy, double c, std::vector<double>& tab, int64_t& half);

// Spectral condition number of Phi for n equispaced points (cyclic Jacobi);
// +inf once the smallest eigenvalue is not positive in float64.
double rbf_condition(int32_t n, double spacing, double c);

// pdd_rbf_shape's search (bisection on log c).
pdd_status rbf_shape(int32_t n, double spacing, double target, double* c);

}  // namespace pdd
