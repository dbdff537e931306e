// Inverse-multiquadric interpolation matrices of equispaced stencils
// (eqs. 2-3), their inverses by Cholesky factorisation, and the shape
// parameter search of Sec. 5.1.  Host only, float64.
#include "rbf.h"

#include <cmath>
#include <limits>

namespace pdd {

namespace {

// Phi of n equispaced points, row-major
void imq_matrix(int n, double d, double c, std::vector<double>& A) {
  A.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      const double r = (double)(i - j) * d;
      A[(size_t)i * n + j] = 1.0 / std::sqrt(r * r + c * c);
    }
}

// In-place lower Cholesky factor of the SPD matrix A (n x n, row-major).
// False when a squared pivot falls below 1e-14 of its diagonal entry: the
// matrix is then singular to float64 working accuracy (condition number
// beyond about 1e14) and its inverse meaningless.
bool cholesky(int n, std::vector<double>& A) {
  for (int j = 0; j < n; ++j) {
    const double ajj = A[(size_t)j * n + j];
    double s = ajj;
    for (int k = 0; k < j; ++k) s -= A[(size_t)j * n + k] * A[(size_t)j * n + k];
    if (!(s > 1e-14 * ajj)) return false;
    const double ljj = std::sqrt(s);
    A[(size_t)j * n + j] = ljj;
    for (int i = j + 1; i < n; ++i) {
      double t = A[(size_t)i * n + j];
      for (int k = 0; k < j; ++k) t -= A[(size_t)i * n + k] * A[(size_t)j * n + k];
      A[(size_t)i * n + j] = t / ljj;
    }
  }
  return true;
}

// Phi^{-1} from its Cholesky factor L: column j solves L L^T x = e_j
void inverse_from_cholesky(int n, const std::vector<double>& L, double* out) {
  std::vector<double> y(n);
  for (int j = 0; j < n; ++j) {
    for (int i = 0; i < n; ++i) {
      double t = i == j ? 1.0 : 0.0;
      for (int k = 0; k < i; ++k) t -= L[(size_t)i * n + k] * y[k];
      y[i] = t / L[(size_t)i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {
      double t = y[i];
      for (int k = i + 1; k < n; ++k) t -= L[(size_t)k * n + i] * y[k];
      y[i] = t / L[(size_t)i * n + i];
    }
    for (int i = 0; i < n; ++i) out[(size_t)i * n + j] = y[i];
  }
  // exact symmetry, so that column reads equal row reads
  for (int i = 0; i < n; ++i)
    for (int j = i + 1; j < n; ++j) {
      const double m = 0.5 * (out[(size_t)i * n + j] + out[(size_t)j * n + i]);
      out[(size_t)i * n + j] = m;
      out[(size_t)j * n + i] = m;
    }
}

// Eigenvalues of a symmetric matrix by cyclic Jacobi rotations
// (Golub and Van Loan, Sec. 8.5), returned unsorted in `ev`.
void jacobi_eigenvalues(int n, std::vector<double> A, std::vector<double>& ev) {
  auto a = [&](int i, int j) -> double& { return A[(size_t)i * n + j]; };
  for (int sweep = 0; sweep < 100; ++sweep) {
    bool rotated = false;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = a(p, q);
        // skip entries already negligible relative to their diagonal pair
        if (std::fabs(apq) <= 0x1p-53 * std::sqrt(std::fabs(a(p, p) * a(q, q)))) {
          a(p, q) = a(q, p) = 0.0;
          continue;
        }
        rotated = true;
        const double theta = (a(q, q) - a(p, p)) / (2.0 * apq);
        const double t = (theta >= 0.0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double cs = 1.0 / std::sqrt(t * t + 1.0), sn = t * cs;
        for (int k = 0; k < n; ++k) {          // columns p, q
          const double akp = a(k, p), akq = a(k, q);
          a(k, p) = cs * akp - sn * akq;
          a(k, q) = sn * akp + cs * akq;
        }
        for (int k = 0; k < n; ++k) {          // rows p, q
          const double apk = a(p, k), aqk = a(q, k);
          a(p, k) = cs * apk - sn * aqk;
          a(q, k) = sn * apk + cs * aqk;
        }
        a(p, q) = a(q, p) = 0.0;
      }
    if (!rotated) break;
  }
  ev.resize(n);
  for (int i = 0; i < n; ++i) ev[i] = a(i, i);
}

}  // namespace

bool rbf_inverse_table(int32_t slot_len, double dx, double dy, double c, std::vector<double>& tab, int64_t& half) {
  half = rbf_block_offset((int64_t)slot_len + 1);
  tab.assign((size_t)(2 * half), 0.0);
  std::vector<double> A;
  for (int side = 0; side < 2; ++side) {
    const double d = side ? dy : dx;
    for (int S = 1; S <= slot_len; ++S) {
      imq_matrix(S, d, c, A);
      if (!cholesky(S, A)) return false;
      inverse_from_cholesky(S, A, tab.data() + side * half + rbf_block_offset(S));
    }
  }
  return true;
}

double rbf_condition(int32_t n, double spacing, double c) {
  std::vector<double> A, ev;
  imq_matrix(n, spacing, c, A);
  jacobi_eigenvalues(n, A, ev);
  double lo = ev[0], hi = ev[0];
  for (double v : ev) {
    lo = std::fmin(lo, v);
    hi = std::fmax(hi, v);
  }
  return lo > 0.0 ? hi / lo : std::numeric_limits<double>::infinity();
}

pdd_status rbf_shape(int32_t n, double spacing, double target, double* c) {
  if (n < 2 || n > 256 || !(spacing > 0.0) || !std::isfinite(spacing) || !(target > 1.0) || !(target <= 1e14) || !c)
    return PDD_EINVAL;
  double lo = 1e-3 * spacing, hi = 1e3 * spacing;
  if (!(rbf_condition(n, spacing, lo) < target && target < rbf_condition(n, spacing, hi))) return PDD_EINVAL;
  for (int it = 0; it < 200 && hi / lo - 1.0 >= 1e-12; ++it) {
    const double mid = std::sqrt(lo * hi);
    if (rbf_condition(n, spacing, mid) < target) lo = mid;
    else hi = mid;
  }
  *c = std::sqrt(lo * hi);
  return PDD_OK;
}

}  // namespace pdd
