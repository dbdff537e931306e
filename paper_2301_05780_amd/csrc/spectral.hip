// Pseudospectral subdomain solves (Sec. 3.3, Sec. 5.1) and the global u0(x)
// they define (Sec. 4.3, Phase I), for constant-coefficient operators
// 1/2 a_xx u_xx + 1/2 a_yy u_yy + c u = f.
//
// Every square of the partition carries the tensor grid of the p + 1
// Chebyshev-Gauss-Lobatto points per direction.  Its side values come from
// the knot values (hat or inverse-multiquadric cardinal interpolation along
// the grid line over the side's extended stencil) or from g on the domain
// boundary; the interior values solve the collocation system
//   ax E U + ay U E^T + c U = F,   E = D2[1..p-1][1..p-1],
// F the source at the interior points minus the boundary columns of D2
// applied to the side values.  With E = V diag(lam) V^{-1} (host, once per
// p) the solve is four dense products and a pointwise division:
//   U = V [(V^{-1} F V^{-T}) / (ax lam_i + ay lam_j + c)] V^T,
// run per square by one workgroup on the float64 matrix cores
// (v_mfma_f64_16x16x4_f64) with 64 x 64 tiles in LDS.  Two more products
// give the grid derivatives (2/S) D U and U ((2/S) D)^T.
//
// Grid layout (device, float64): grid[s][f][i][j], square s = a + H c (a
// along x), field f = 0 (u), 1 (du/dx), 2 (du/dy), i the x index and j the y
// index of the point (x_a + S (t_i + 1) / 2, y_c + S (t_j + 1) / 2).
#include <hip/hip_runtime.h>

#include "device_common.h"
#include "spectral.h"

namespace pdd {

namespace {

constexpr int LDT = SPEC_T + 1;     // LDS row stride (doubles): spreads a fragment over the banks
typedef double v4d __attribute__((ext_vector_type(4)));

__device__ __forceinline__ double* gfield(const SpecArgs& A, int64_t s, int f) {
  const int N = A.p + 1;
  return A.grid + ((size_t)s * 3 + f) * (size_t)N * N;
}

// lattice value of the line at lattice coordinate `at` (vertical: x = const)
// at along-line lattice point q: g on the domain boundary, else the knot value
template <int KIND>
__device__ __forceinline__ double lattice_value(const SpecArgs& A, bool vert, int at, int q) {
  const AsmParams& P = A.P;
  if (q == 0 || q == P.L) {
    const double lx = vert ? P.x0 + (double)at * P.dx : P.x0 + (double)q * P.dx;
    const double ly = vert ? P.y0 + (double)q * P.dy : P.y0 + (double)at * P.dy;
    return g_at<KIND>(lx, ly);
  }
  const int ix = vert ? at : q, iy = vert ? q : at;
  return A.u_knots[P.lattice[(size_t)iy * (P.L + 1) + ix]];
}

// Side values: one wave per (square, side); side o = 0 (S), 1 (N), 2 (W),
// 3 (E).  The horizontal sides take all p + 1 points (the corners included),
// the vertical sides the p - 1 interior ones.
template <int KIND>
__global__ __launch_bounds__(256) void k_spec_sides(SpecArgs A, int32_t smax) {
  extern __shared__ double sv[];
  const AsmParams& P = A.P;
  const int lane = threadIdx.x & 63;
  const int64_t w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (w >= 4LL * A.H * A.H) return;
  const int64_t s = w >> 2;
  const int o = (int)(w & 3);
  const int a = (int)(s % A.H), c = (int)(s / A.H);
  const int p = A.p, N = p + 1, m = A.m, L = P.L;
  const bool vert = o >= 2;
  const int at = vert ? (o == 2 ? a * m : (a + 1) * m) : (o == 0 ? c * m : (c + 1) * m);
  const int lo = vert ? c * m : a * m, hi = lo + m;
  const double Sx = (P.x1 - P.x0) / A.H, Sy = (P.y1 - P.y0) / A.H;
  const double xa = P.x0 + a * Sx, ya = P.y0 + c * Sy;
  double* U = gfield(A, s, 0);
  const bool bnd = at == 0 || at == L;
  const int clo = max(0, lo - A.ext), chi = min(L, hi + A.ext);
  const double a0 = vert ? P.y0 : P.x0, d = vert ? P.dy : P.dx;
  double* v = sv + (size_t)(threadIdx.x >> 6) * 2 * smax;
  double* al = v + smax;
  const int S = chi - clo + 1;
  if (!bnd && A.rbf) {
    // alpha = Phi^{-1} v over the side's stencil
    for (int i = lane; i < S; i += 64) v[i] = lattice_value<KIND>(A, vert, at, clo + i);
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    const double* Mi = P.rbf_inv + (vert ? P.rbf_half : 0) + rbf_block_offset(S);
    for (int i = lane; i < S; i += 64) {
      double acc = 0.0;
      for (int j = 0; j < S; ++j) acc = fma(Mi[(size_t)j * S + i], v[j], acc);
      al[i] = acc;
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
  }
  const int first = vert ? 1 : 0, last = vert ? p - 1 : p;
  for (int k = first + lane; k <= last; k += 64) {
    const double t = A.T.nodes[k];
    const double xk = vert ? (o == 2 ? xa : xa + Sx) : xa + Sx * (t + 1.0) * 0.5;
    const double yk = vert ? ya + Sy * (t + 1.0) * 0.5 : (o == 0 ? ya : ya + Sy);
    double val;
    if (bnd) {
      val = g_at<KIND>(xk, yk);
    } else {
      const double z = vert ? yk : xk;
      if (A.rbf) {
        double acc = 0.0;
        for (int q = 0; q < S; ++q) {
          const double r = z - (a0 + (double)(clo + q) * d);
          acc = fma(al[q], 1.0 / sqrt(fma(r, r, P.rbf_c2)), acc);
        }
        val = acc;
      } else {
        double tt = (z - a0) / d;
        tt = fmin(fmax(tt, (double)clo), (double)chi);
        const double i0 = fmin(floor(tt), (double)(chi - 1));
        const double wt = tt - i0;
        const int q0 = (int)i0;
        val = (1.0 - wt) * lattice_value<KIND>(A, vert, at, q0) + wt * lattice_value<KIND>(A, vert, at, q0 + 1);
      }
    }
    const int i = vert ? (o == 2 ? 0 : p) : k, j = vert ? k : (o == 0 ? 0 : p);
    U[(size_t)i * N + j] = val;
  }
}

// C strip of wave w (rows 16 w .. 16 w + 15) of C = A B for 64 x 64
// operands: acc[ct] holds the 16 x 16 tile of columns 16 ct .. 16 ct + 15.
// Operands per lane l and K step: A[16 w + l % 16][k0 + l / 16] and
// B[k0 + l / 16][16 ct + l % 16]; the float64 accumulator holds element q of
// lane l at row 16 w + l / 16 + 4 q, column 16 ct + l % 16.
template <class FA, class FB>
__device__ __forceinline__ void mfma_strip(FA fa, FB fb, v4d acc[4]) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int r = lane & 15, kq = lane >> 4;
#pragma unroll
  for (int ct = 0; ct < 4; ++ct) acc[ct] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
  for (int k0 = 0; k0 < SPEC_T; k0 += 4) {
    const double av = fa(16 * w + r, k0 + kq);
#pragma unroll
    for (int ct = 0; ct < 4; ++ct)
      acc[ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, fb(k0 + kq, 16 * ct + r), acc[ct], 0, 0, 0);
  }
}

template <class F>
__device__ __forceinline__ void strip_for_each(const v4d acc[4], F f) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int ct = 0; ct < 4; ++ct)
#pragma unroll
    for (int q = 0; q < 4; ++q) f(16 * w + (lane >> 4) + 4 * q, 16 * ct + (lane & 15), acc[ct][q]);
}

// Interior solve and grid derivatives of one square per workgroup (4 waves).
template <int KIND>
__global__ __launch_bounds__(256) void k_spec_solve(SpecArgs A) {
  __shared__ double B[SPEC_T * LDT];
  const AsmParams& P = A.P;
  const int64_t s = blockIdx.x;
  const int a = (int)(s % A.H), c = (int)(s / A.H);
  const int p = A.p, N = p + 1, n = p - 1;
  const double Sx = (P.x1 - P.x0) / A.H, Sy = (P.y1 - P.y0) / A.H;
  const double xa = P.x0 + a * Sx, ya = P.y0 + c * Sy;
  double* U = gfield(A, s, 0);
  const double* nodes = A.T.nodes;
  const double* D2b = A.T.D2b;
  // F: source at the interior points minus the boundary columns of the operator
  for (int e = threadIdx.x; e < SPEC_T * SPEC_T; e += blockDim.x) {
    const int i = e / SPEC_T, j = e % SPEC_T;
    double f = 0.0;
    if (i < n && j < n) {
      const double x = xa + Sx * (nodes[i + 1] + 1.0) * 0.5;
      const double y = ya + Sy * (nodes[j + 1] + 1.0) * 0.5;
      Coef<double> cf;
      coef_at<KIND>(P.coef, x, y, cf);
      f = cf.f - A.ax * (D2b[2 * i] * U[(size_t)0 * N + j + 1] + D2b[2 * i + 1] * U[(size_t)p * N + j + 1]) -
          A.ay * (D2b[2 * j] * U[(size_t)(i + 1) * N] + D2b[2 * j + 1] * U[(size_t)(i + 1) * N + p]);
    }
    B[i * LDT + j] = f;
  }
  __syncthreads();
  const double* V = A.T.V;
  const double* Vi = A.T.Vinv;
  v4d acc[4];
  auto lds = [&](int i, int k) { return B[i * LDT + k]; };
  // V^{-1} F
  mfma_strip([&](int i, int k) { return Vi[i * SPEC_T + k]; }, lds, acc);
  __syncthreads();
  strip_for_each(acc, [&](int i, int j, double v) { B[i * LDT + j] = v; });
  __syncthreads();
  // (V^{-1} F) V^{-T}, divided by ax lam_i + ay lam_j + c
  mfma_strip(lds, [&](int k, int j) { return Vi[j * SPEC_T + k]; }, acc);
  __syncthreads();
  const double* lam = A.T.lam;
  strip_for_each(acc, [&](int i, int j, double v) { B[i * LDT + j] = v / (A.ax * lam[i] + A.ay * lam[j] + A.c); });
  __syncthreads();
  // V (.)
  mfma_strip([&](int i, int k) { return V[i * SPEC_T + k]; }, lds, acc);
  __syncthreads();
  strip_for_each(acc, [&](int i, int j, double v) { B[i * LDT + j] = v; });
  __syncthreads();
  // (.) V^T: the interior values
  mfma_strip(lds, [&](int k, int j) { return V[j * SPEC_T + k]; }, acc);
  __syncthreads();
  // the whole grid into LDS (zero-padded): interior from the product, sides from global
  strip_for_each(acc, [&](int i, int j, double v) {
    if (i < n && j < n) {
      B[(i + 1) * LDT + j + 1] = v;
      U[(size_t)(i + 1) * N + j + 1] = v;
    }
  });
  for (int e = threadIdx.x; e < SPEC_T * SPEC_T; e += blockDim.x) {
    const int i = e / SPEC_T, j = e % SPEC_T;
    if (i >= N || j >= N) B[i * LDT + j] = 0.0;
    else if (i == 0 || i == p || j == 0 || j == p) B[i * LDT + j] = U[(size_t)i * N + j];
  }
  __syncthreads();
  const double* Dm = A.T.D;
  const double sx = 2.0 / Sx, sy = 2.0 / Sy;
  double* Gx = gfield(A, s, 1);
  double* Gy = gfield(A, s, 2);
  // du/dx = (2/S) D U
  mfma_strip([&](int i, int k) { return Dm[i * SPEC_T + k]; }, lds, acc);
  strip_for_each(acc, [&](int i, int j, double v) {
    if (i < N && j < N) Gx[(size_t)i * N + j] = sx * v;
  });
  // du/dy = U ((2/S) D)^T
  mfma_strip(lds, [&](int k, int j) { return Dm[j * SPEC_T + k]; }, acc);
  strip_for_each(acc, [&](int i, int j, double v) {
    if (i < N && j < N) Gy[(size_t)i * N + j] = sy * v;
  });
}

template <int KIND>
hipError_t launch_kind(const SpecArgs& A, hipStream_t stream) {
  const int64_t waves = 4LL * A.H * A.H;
  const int smax = min(A.m + 2 * A.ext, A.P.L) + 1;
  const size_t lds = (size_t)4 * 2 * smax * sizeof(double);
  hipLaunchKernelGGL((k_spec_sides<KIND>), dim3((unsigned)((waves + 3) / 4)), dim3(256), lds, stream, A, smax);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_spec_solve<KIND>), dim3((unsigned)(A.H * A.H)), dim3(256), 0, stream, A);
  return hipGetLastError();
}

// wave sum, every lane receiving it
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// barycentric basis value of node `lane` at reference coordinate z (exact at a node)
__device__ __forceinline__ double bary_basis(const double* nodes, const double* bw, int p, double z) {
  const int lane = threadIdx.x & 63;
  const bool mine = lane <= p;
  const double dz = mine ? z - nodes[lane] : 1.0;
  const uint64_t hit = __ballot(mine && dz == 0.0);
  if (hit) return (int)__builtin_ctzll(hit) == lane ? 1.0 : 0.0;
  const double r = mine ? bw[lane] / dz : 0.0;
  return r / wave_sum(r);
}

// One wave per point: 2-D barycentric interpolation of u, du/dx, du/dy on the
// point's square.  Points are either xy[2 n] (outputs u[n], grad[2 n], each
// nullable) or, with lut_n > 0, the lut_n^2 nodes of the domain's node grid
// (output grad_lut[(j lut_n + i) 2 + d] in float32).
__global__ __launch_bounds__(256) void k_spec_eval(SpecDev T, int32_t p, int32_t H, double x0, double x1, double y0,
                                                   double y1, const double* __restrict__ grid, int64_t n_pts,
                                                   const double* __restrict__ xy, int32_t lut_n, double* u,
                                                   double* grad, float* grad_lut) {
  __shared__ double lys[4][64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int N = p + 1;
  const double Sx = (x1 - x0) / H, Sy = (y1 - y0) / H;
  for (int64_t q = (int64_t)blockIdx.x * 4 + wv; q < n_pts; q += (int64_t)gridDim.x * 4) {
    double x, y;
    if (lut_n > 0) {
      const int i = (int)(q % lut_n), j = (int)(q / lut_n);
      x = x0 + (x1 - x0) * (double)i / (double)(lut_n - 1);
      y = y0 + (y1 - y0) * (double)j / (double)(lut_n - 1);
    } else {
      x = xy[2 * q];
      y = xy[2 * q + 1];
    }
    const int a = min(max((int)floor((x - x0) / Sx), 0), H - 1);
    const int c = min(max((int)floor((y - y0) / Sy), 0), H - 1);
    const double zx = 2.0 * (x - (x0 + a * Sx)) / Sx - 1.0;
    const double zy = 2.0 * (y - (y0 + c * Sy)) / Sy - 1.0;
    const double lx = bary_basis(T.nodes, T.bw, p, zx);
    const double ly = bary_basis(T.nodes, T.bw, p, zy);
    lys[wv][lane] = ly;
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    const size_t sq = (size_t)(a + (int64_t)H * c) * 3 * N * N;
    double out[3];
#pragma unroll
    for (int f = 0; f < 3; ++f) {
      double r = 0.0;
      if (lane < N && lx != 0.0) {
        const double* row = grid + sq + (size_t)f * N * N + (size_t)lane * N;
        for (int j = 0; j < N; ++j) r = fma(lys[wv][j], row[j], r);
      }
      out[f] = wave_sum(lx * r);
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    if (lane == 0) {
      if (lut_n > 0) {
        grad_lut[2 * q] = (float)out[1];
        grad_lut[2 * q + 1] = (float)out[2];
      } else {
        if (u) u[q] = out[0];
        if (grad) {
          grad[2 * q] = out[1];
          grad[2 * q + 1] = out[2];
        }
      }
    }
  }
}

// Range of the fields 0..5 (sxx, sxy, syy, dx, dy, c) of a LUT: per-block
// minima and maxima, then one block combines them into out[12] (min, max).
constexpr int RANGE_BLOCKS = 1024;
__global__ __launch_bounds__(256) void k_lut_range_part(const float* __restrict__ lut, int64_t nodes,
                                                        double* __restrict__ part) {
  __shared__ double red[256][12];
  double mn[6], mx[6];
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    mn[q] = INFINITY;
    mx[q] = -INFINITY;
  }
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < nodes; i += (int64_t)gridDim.x * 256) {
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      const double v = lut[(size_t)i * PDD_LUT_STRIDE + q];
      mn[q] = fmin(mn[q], v);
      mx[q] = fmax(mx[q], v);
    }
  }
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    red[threadIdx.x][q] = mn[q];
    red[threadIdx.x][6 + q] = mx[q];
  }
  __syncthreads();
  if (threadIdx.x < 12) {
    const int q = threadIdx.x;
    double v = red[0][q];
    for (int t = 1; t < 256; ++t) v = q < 6 ? fmin(v, red[t][q]) : fmax(v, red[t][q]);
    part[(size_t)blockIdx.x * 12 + q] = v;
  }
}

__global__ void k_lut_range_final(const double* __restrict__ part, int blocks, double* __restrict__ out) {
  if (threadIdx.x < 12) {
    const int q = threadIdx.x;
    double v = part[q];
    for (int b = 1; b < blocks; ++b) v = q < 6 ? fmin(v, part[(size_t)b * 12 + q]) : fmax(v, part[(size_t)b * 12 + q]);
    out[q] = v;
  }
}

}  // namespace

hipError_t launch_spectral_solve(const SpecArgs& A, hipStream_t stream) {
  switch (A.P.coef.kind) {
    case PDD_COEF_POISSON: return launch_kind<PDD_COEF_POISSON>(A, stream);
    case PDD_COEF_EXITTIME: return launch_kind<PDD_COEF_EXITTIME>(A, stream);
    case PDD_COEF_EQ43: return launch_kind<PDD_COEF_EQ43>(A, stream);
    case PDD_COEF_LUT: return launch_kind<PDD_COEF_LUT>(A, stream);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_spectral_eval(const SpecDev& T, int32_t p, int32_t H, double x0, double x1, double y0, double y1,
                                const double* grid, int64_t n_pts, const double* xy, int32_t lut_n, double* u,
                                double* grad, float* grad_lut, hipStream_t stream) {
  const int64_t pts = lut_n > 0 ? (int64_t)lut_n * lut_n : n_pts;
  const unsigned blocks = (unsigned)std::min<int64_t>((pts + 3) / 4, 65536);
  hipLaunchKernelGGL(k_spec_eval, dim3(std::max(blocks, 1u)), dim3(256), 0, stream, T, p, H, x0, x1, y0, y1, grid, pts,
                     xy, lut_n, u, grad, grad_lut);
  return hipGetLastError();
}

hipError_t launch_lut_field_range(const float* lut, int64_t nodes, double* out, hipStream_t stream) {
  // out[0..11] = min, max of fields 0..5; out + 12 holds RANGE_BLOCKS * 12 partials
  double* part = out + 12;
  hipLaunchKernelGGL(k_lut_range_part, dim3(RANGE_BLOCKS), dim3(256), 0, stream, lut, nodes, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_lut_range_final, dim3(1), dim3(64), 0, stream, part, RANGE_BLOCKS, out);
  return hipGetLastError();
}

}  // namespace pdd
