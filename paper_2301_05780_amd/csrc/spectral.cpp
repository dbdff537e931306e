// Host side of the pseudospectral subdomain solves (Sec. 3.3, Sec. 5.1):
// the Chebyshev-Gauss-Lobatto collocation matrices of one polynomial degree
// p and the eigen-decomposition of the interior block of the second
// derivative, which turns every constant-coefficient subdomain solve into
// four dense products (fast diagonalisation).  Computed once per p in long
// double and rounded to float64.
#include "spectral.h"

#include <cmath>
#include <vector>

namespace pdd {

namespace {

using ld = long double;

struct Mat {
  int n = 0;
  std::vector<ld> a;
  explicit Mat(int n_) : n(n_), a((size_t)n_ * n_, 0.0L) {}
  ld& operator()(int i, int j) { return a[(size_t)i * n + j]; }
  ld operator()(int i, int j) const { return a[(size_t)i * n + j]; }
};

// Reduce A to upper Hessenberg form H = Q^T A Q by Householder reflections;
// Q accumulates the reflections.
void hessenberg(Mat& A, Mat& Q) {
  const int n = A.n;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) Q(i, j) = i == j ? 1.0L : 0.0L;
  std::vector<ld> v(n);
  for (int k = 0; k + 2 < n; ++k) {
    ld alpha = 0.0L;
    for (int i = k + 1; i < n; ++i) alpha += A(i, k) * A(i, k);
    alpha = std::sqrt(alpha);
    if (alpha == 0.0L) continue;
    if (A(k + 1, k) > 0) alpha = -alpha;
    ld vn = 0.0L;
    for (int i = 0; i < n; ++i) v[i] = 0.0L;
    v[k + 1] = A(k + 1, k) - alpha;
    for (int i = k + 2; i < n; ++i) v[i] = A(i, k);
    for (int i = k + 1; i < n; ++i) vn += v[i] * v[i];
    if (vn == 0.0L) continue;
    // A <- (I - 2 v v^T / vn) A (I - 2 v v^T / vn), Q <- Q (I - 2 v v^T / vn)
    for (int j = 0; j < n; ++j) {
      ld s = 0.0L;
      for (int i = k + 1; i < n; ++i) s += v[i] * A(i, j);
      s *= 2.0L / vn;
      for (int i = k + 1; i < n; ++i) A(i, j) -= s * v[i];
    }
    for (int i = 0; i < n; ++i) {
      ld s = 0.0L, t = 0.0L;
      for (int j = k + 1; j < n; ++j) {
        s += A(i, j) * v[j];
        t += Q(i, j) * v[j];
      }
      s *= 2.0L / vn;
      t *= 2.0L / vn;
      for (int j = k + 1; j < n; ++j) {
        A(i, j) -= s * v[j];
        Q(i, j) -= t * v[j];
      }
    }
    for (int i = k + 2; i < n; ++i) A(i, k) = 0.0L;
  }
}

// Shifted QR iteration on the Hessenberg matrix H (Wilkinson shifts, Givens
// rotations applied to the whole matrix and accumulated in Q) until H is
// upper triangular: the real Schur form of a matrix with real eigenvalues.
// False if a 2 x 2 block keeps complex eigenvalues or the iteration stalls.
bool schur_real(Mat& H, Mat& Q) {
  const int n = H.n;
  const ld eps = 4.0L * std::numeric_limits<ld>::epsilon();
  int hi = n - 1;
  int iter = 0;
  while (hi > 0) {
    if (++iter > 100 * n) return false;
    // deflate a negligible subdiagonal entry at the bottom of the window
    int lo = hi;
    while (lo > 0) {
      const ld s = std::fabs(H(lo - 1, lo - 1)) + std::fabs(H(lo, lo));
      if (std::fabs(H(lo, lo - 1)) <= eps * s) {
        H(lo, lo - 1) = 0.0L;
        break;
      }
      --lo;
    }
    if (lo == hi) {
      --hi;
      iter = 0;
      continue;
    }
    // Wilkinson shift from the trailing 2 x 2 block
    const ld a = H(hi - 1, hi - 1), b = H(hi - 1, hi), c = H(hi, hi - 1), d = H(hi, hi);
    const ld tr = 0.5L * (a - d);
    const ld disc = tr * tr + b * c;
    ld mu;
    if (disc >= 0.0L) {
      const ld r = std::sqrt(disc);
      mu = d - b * c / (tr + (tr >= 0.0L ? r : -r) + (tr == 0.0L && r == 0.0L ? 1e-300L : 0.0L));
    } else {
      if (hi - lo == 1) return false;      // an isolated complex pair
      mu = d;
    }
    if (iter % 11 == 10) mu = d + std::fabs(H(hi, hi - 1));   // exceptional shift
    // explicit QR step on the window [lo, hi]: H - mu I = R by Givens from the
    // left, then H = R G^T + mu I; the rotations also act on the rows/columns
    // outside the window and on Q
    std::vector<ld> cs(hi - lo), sn(hi - lo);
    for (int i = lo; i <= hi; ++i) H(i, i) -= mu;
    for (int k = lo; k < hi; ++k) {
      const ld x = H(k, k), y = H(k + 1, k);
      const ld r = std::hypot(x, y);
      const ld cc = r == 0.0L ? 1.0L : x / r, ss = r == 0.0L ? 0.0L : y / r;
      cs[k - lo] = cc;
      sn[k - lo] = ss;
      for (int j = k; j < n; ++j) {
        const ld t1 = H(k, j), t2 = H(k + 1, j);
        H(k, j) = cc * t1 + ss * t2;
        H(k + 1, j) = -ss * t1 + cc * t2;
      }
    }
    for (int k = lo; k < hi; ++k) {
      const ld cc = cs[k - lo], ss = sn[k - lo];
      const int top = 0;
      for (int i = top; i <= std::min(k + 2, hi); ++i) {
        const ld t1 = H(i, k), t2 = H(i, k + 1);
        H(i, k) = cc * t1 + ss * t2;
        H(i, k + 1) = -ss * t1 + cc * t2;
      }
      for (int i = 0; i < n; ++i) {
        const ld t1 = Q(i, k), t2 = Q(i, k + 1);
        Q(i, k) = cc * t1 + ss * t2;
        Q(i, k + 1) = -ss * t1 + cc * t2;
      }
    }
    for (int i = lo; i <= hi; ++i) H(i, i) += mu;
  }
  return true;
}

// Inverse by Gaussian elimination with partial pivoting; false if singular.
bool invert(const Mat& A, Mat& X) {
  const int n = A.n;
  Mat M = A;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) X(i, j) = i == j ? 1.0L : 0.0L;
  for (int k = 0; k < n; ++k) {
    int piv = k;
    for (int i = k + 1; i < n; ++i)
      if (std::fabs(M(i, k)) > std::fabs(M(piv, k))) piv = i;
    if (M(piv, k) == 0.0L) return false;
    if (piv != k)
      for (int j = 0; j < n; ++j) {
        std::swap(M(k, j), M(piv, j));
        std::swap(X(k, j), X(piv, j));
      }
    const ld inv = 1.0L / M(k, k);
    for (int i = 0; i < n; ++i) {
      if (i == k) continue;
      const ld f = M(i, k) * inv;
      if (f == 0.0L) continue;
      for (int j = 0; j < n; ++j) {
        M(i, j) -= f * M(k, j);
        X(i, j) -= f * X(k, j);
      }
    }
    for (int j = 0; j < n; ++j) {
      M(k, j) *= inv;
      X(k, j) *= inv;
    }
  }
  return true;
}

}  // namespace

bool spectral_tables(int32_t p, SpectralTables& t, std::string& err) {
  if (p < 2 || p > SPEC_MAX_P) {
    err = "spectral degree p must lie in [2, 63]";
    return false;
  }
  const int N = p + 1, n = p - 1;
  // nodes t_j = -cos(pi j / p), barycentric weights (-1)^j halved at the ends
  std::vector<ld> tn(N), w(N);
  const ld pi = 3.141592653589793238462643383279502884L;
  for (int j = 0; j < N; ++j) {
    tn[j] = -std::cos(pi * (ld)j / (ld)p);
    w[j] = (j % 2 ? -1.0L : 1.0L) * ((j == 0 || j == p) ? 0.5L : 1.0L);
  }
  tn[0] = -1.0L;
  tn[p] = 1.0L;
  // D_ij = (w_j / w_i) / (t_i - t_j), D_ii = -sum_{j != i} D_ij
  Mat D(N);
  for (int i = 0; i < N; ++i) {
    ld s = 0.0L;
    for (int j = 0; j < N; ++j) {
      if (j == i) continue;
      D(i, j) = (w[j] / w[i]) / (tn[i] - tn[j]);
      s += D(i, j);
    }
    D(i, i) = -s;
  }
  Mat D2(N);
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) {
      ld s = 0.0L;
      for (int k = 0; k < N; ++k) s += D(i, k) * D(k, j);
      D2(i, j) = s;
    }
  // interior block E = D2[1..p-1][1..p-1] = V diag(lambda) V^{-1}
  Mat E(n), Q(n), V(n), Vi(n);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) E(i, j) = D2(i + 1, j + 1);
  Mat H = E;
  hessenberg(H, Q);
  if (!schur_real(H, Q)) {
    err = "spectral tables: the interior second-derivative block did not reduce to real Schur form";
    return false;
  }
  // eigenvectors of the triangular Schur factor by back-substitution, then Q y
  std::vector<ld> lam(n), y(n);
  for (int k = 0; k < n; ++k) lam[k] = H(k, k);
  const ld tiny = std::numeric_limits<ld>::epsilon();
  for (int k = 0; k < n; ++k) {
    for (int i = 0; i < n; ++i) y[i] = 0.0L;
    y[k] = 1.0L;
    for (int i = k - 1; i >= 0; --i) {
      ld s = 0.0L;
      for (int j = i + 1; j <= k; ++j) s += H(i, j) * y[j];
      ld den = H(i, i) - lam[k];
      if (std::fabs(den) < tiny * std::fabs(lam[k])) den = (den < 0 ? -1.0L : 1.0L) * tiny * std::fabs(lam[k]);
      y[i] = -s / den;
    }
    ld nrm = 0.0L;
    for (int i = 0; i < n; ++i) {
      ld s = 0.0L;
      for (int j = 0; j <= k; ++j) s += Q(i, j) * y[j];
      V(i, k) = s;
      nrm += s * s;
    }
    nrm = std::sqrt(nrm);
    for (int i = 0; i < n; ++i) V(i, k) /= nrm;
  }
  if (!invert(V, Vi)) {
    err = "spectral tables: singular eigenvector matrix";
    return false;
  }
  // accuracy checks of the decomposition (relative to the matrix size)
  ld emax = 0.0L, res = 0.0L, idr = 0.0L;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      emax = std::max(emax, std::fabs(E(i, j)));
      ld r = -V(i, j) * lam[j], id = (i == j ? -1.0L : 0.0L);
      for (int k = 0; k < n; ++k) {
        r += E(i, k) * V(k, j);
        id += V(i, k) * Vi(k, j);
      }
      res = std::max(res, std::fabs(r));
      idr = std::max(idr, std::fabs(id));
    }
  for (int k = 0; k < n; ++k)
    if (!(lam[k] < 0.0L)) {
      err = "spectral tables: an eigenvalue of the interior second derivative is not negative";
      return false;
    }
  t.decomp_residual = (double)(res / emax);
  t.inverse_residual = (double)idr;
  if (!(t.decomp_residual < 1e-11) || !(t.inverse_residual < 1e-9)) {
    err = "spectral tables: the eigen-decomposition is not accurate to float64";
    return false;
  }
  // round to float64, zero-padded to SPEC_T x SPEC_T
  t.p = p;
  t.nodes.assign(N, 0.0);
  t.bw.assign(N, 0.0);
  t.D.assign((size_t)SPEC_T * SPEC_T, 0.0);
  t.D2b.assign((size_t)2 * SPEC_T, 0.0);
  t.V.assign((size_t)SPEC_T * SPEC_T, 0.0);
  t.Vinv.assign((size_t)SPEC_T * SPEC_T, 0.0);
  t.lam.assign(SPEC_T, -1.0);
  for (int j = 0; j < N; ++j) {
    t.nodes[j] = (double)tn[j];
    t.bw[j] = (double)w[j];
  }
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) t.D[(size_t)i * SPEC_T + j] = (double)D(i, j);
  for (int i = 0; i < n; ++i) {
    t.D2b[(size_t)i * 2] = (double)D2(i + 1, 0);
    t.D2b[(size_t)i * 2 + 1] = (double)D2(i + 1, p);
    t.lam[i] = (double)lam[i];
    for (int j = 0; j < n; ++j) {
      t.V[(size_t)i * SPEC_T + j] = (double)V(i, j);
      t.Vinv[(size_t)i * SPEC_T + j] = (double)Vi(i, j);
    }
  }
  return true;
}

}  // namespace pdd
