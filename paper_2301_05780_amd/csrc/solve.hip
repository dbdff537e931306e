// Solution of the assembled system G u = b (eq. 23): mixed-precision
// iterative refinement.  The outer loop keeps u and the residual
// r = b - G u in float64; each correction G d = r is solved by BiCGStab
// (van der Vorst, 1992) on float32 vectors and a float32 copy of G, with
// float64 dot products.  Scalars of the recurrence live on the device; the
// host reads the residual norm only every few iterations.
//
// Kernels: CSR SpMV with one wave per row (rows hold 1 to a few hundred
// entries), fused vector updates that also produce per-block partial dot
// products, and a one-block reduction that finishes the dots and advances
// the scalars.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>

#include "context.h"

namespace pdd {

namespace {

constexpr int RED_BLOCKS = 256;     // partial-dot blocks
constexpr int BLK = 256;
constexpr int MAX_DEVICES = 64;

// Scratch of pdd_solve_noalloc: a file-scope device array, one copy per GPU
// that runs the library, held until the process ends.  Host code uses only
// its per-device address from hipGetSymbolAddress (solve_noalloc_setup); the
// array's name on the host is a stand-in, not a device address.
__device__ __align__(256) char scratch[SOLVE_NOALLOC_BYTES];
void* g_scratch_ptr[MAX_DEVICES] = {};
std::mutex g_scratch_mu;

// Scalars of one BiCGStab recurrence (device).
struct Scal {
  double rho, rho_new, alpha, omega;
  double rv, ts, tt, rr;
  int32_t broke;                    // breakdown flag
  int32_t pad;
};

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// block-level sum of up to 3 values into partial[q * RED_BLOCKS + blockIdx.x]
template <int NQ>
__device__ __forceinline__ void block_partials(double (&v)[NQ], double* partial) {
  __shared__ double sh[NQ][BLK / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const double s = wave_sum(v[q]);
    if (lane == 0) sh[q][wid] = s;
  }
  __syncthreads();
  if (threadIdx.x < NQ) {
    double s = 0.0;
    for (int w = 0; w < BLK / 64; ++w) s += sh[threadIdx.x][w];
    partial[threadIdx.x * RED_BLOCKS + blockIdx.x] = s;
  }
}

// y = A x (one wave per row); optional fused dot d0 = <w, y>
template <typename TA, typename TX>
__global__ __launch_bounds__(BLK) void k_spmv(int64_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                              const TA* __restrict__ val, const TX* __restrict__ x, TX* __restrict__ y) {
  const int lane = threadIdx.x & 63;
  const int64_t row = (int64_t)blockIdx.x * (BLK / 64) + (threadIdx.x >> 6);
  if (row >= n) return;
  double s = 0.0;
  for (int p = rp[row] + lane; p < rp[row + 1]; p += 64) s += (double)val[p] * (double)x[ci[p]];
  s = wave_sum(s);
  if (lane == 0) y[row] = (TX)s;
}

// r = b - A u (float64) and partial ||r||^2
__global__ __launch_bounds__(BLK) void k_residual(int64_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                                  const double* __restrict__ val, const double* __restrict__ u,
                                                  const double* __restrict__ b, double* __restrict__ r) {
  const int lane = threadIdx.x & 63;
  const int64_t row = (int64_t)blockIdx.x * (BLK / 64) + (threadIdx.x >> 6);
  if (row >= n) return;
  double s = 0.0;
  for (int p = rp[row] + lane; p < rp[row + 1]; p += 64) s += val[p] * u[ci[p]];
  s = wave_sum(s);
  if (lane == 0) r[row] = b[row] - s;
}

// grid-stride helpers over n with RED_BLOCKS blocks
#define GRID_LOOP(i) for (int64_t i = (int64_t)blockIdx.x * BLK + threadIdx.x; i < n; i += (int64_t)RED_BLOCKS * BLK)

__global__ __launch_bounds__(BLK) void k_norm2(int64_t n, const double* __restrict__ a, double* partial) {
  double v[1] = {0.0};
  GRID_LOOP(i) v[0] += a[i] * a[i];
  block_partials<1>(v, partial);
}

// inner start: x = 0, r = rhat = p = float(r64), v = 0; partials <rhat, r>, <r, r>
__global__ __launch_bounds__(BLK) void k_init(int64_t n, const double* __restrict__ r64, float* x, float* r, float* rhat,
                                              float* p, float* v, double* partial) {
  double acc[2] = {0.0, 0.0};
  GRID_LOOP(i) {
    const float ri = (float)r64[i];
    x[i] = 0.0f; r[i] = ri; rhat[i] = ri; p[i] = ri; v[i] = 0.0f;
    acc[0] += (double)ri * ri;
    acc[1] += (double)ri * ri;
  }
  block_partials<2>(acc, partial);
}

// finish partial sums: which = 0: rho_new, rr (start) | 1: rv | 2: ts, tt | 3: rho_next, rr
__global__ __launch_bounds__(BLK) void k_reduce(const double* __restrict__ partial, int nq, int which, Scal* S) {
  __shared__ double sh[3][BLK / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int q = 0; q < nq; ++q) {
    double s = 0.0;
    for (int i = threadIdx.x; i < RED_BLOCKS; i += BLK) s += partial[q * RED_BLOCKS + i];
    s = wave_sum(s);
    if (lane == 0) sh[q][wid] = s;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  double t[3] = {0, 0, 0};
  for (int q = 0; q < nq; ++q)
    for (int w = 0; w < BLK / 64; ++w) t[q] += sh[q][w];
  if (which == 0) {
    S->rho = 1.0; S->alpha = 1.0; S->omega = 1.0; S->rho_new = t[0]; S->rr = t[1]; S->broke = 0;
  } else if (which == 1) {
    S->rv = t[0];
    if (!(t[0] != 0.0) || !isfinite(t[0])) S->broke = 1;
  } else if (which == 2) {
    S->ts = t[0]; S->tt = t[1];
    if (!isfinite(t[0]) || !isfinite(t[1])) S->broke = 1;
  } else {
    // an exact half-step solution (s = 0, omega = 0) ends the recurrence here
    S->rho = S->rho_new; S->rho_new = t[0]; S->rr = t[1];
    if (!(t[0] != 0.0) || !isfinite(t[0]) || S->omega == 0.0) S->broke = 1;
  }
}

// p = r + beta (p - omega v), beta = (rho_new / rho) (alpha / omega); first iteration p = r
__global__ __launch_bounds__(BLK) void k_update_p(int64_t n, int first, const Scal* S, const float* r, const float* v, float* p) {
  if (S->broke) return;
  const double beta = first ? 0.0 : (S->rho_new / S->rho) * (S->alpha / S->omega);
  const float fb = (float)beta, fo = (float)S->omega;
  GRID_LOOP(i) p[i] = r[i] + fb * (p[i] - fo * v[i]);
}

// alpha = rho_new / <rhat, v>; s = r - alpha v
__global__ __launch_bounds__(BLK) void k_update_s(int64_t n, Scal* S, const float* r, const float* v, float* s) {
  if (S->broke) return;
  const double alpha = S->rho_new / S->rv;
  if (blockIdx.x == 0 && threadIdx.x == 0) S->alpha = alpha;
  const float fa = (float)alpha;
  GRID_LOOP(i) s[i] = r[i] - fa * v[i];
}

// partial <t, s>, <t, t>
__global__ __launch_bounds__(BLK) void k_dots_ts(int64_t n, const float* t, const float* s, double* partial) {
  double acc[2] = {0.0, 0.0};
  GRID_LOOP(i) { acc[0] += (double)t[i] * s[i]; acc[1] += (double)t[i] * t[i]; }
  block_partials<2>(acc, partial);
}

// partial <rhat, v>
__global__ __launch_bounds__(BLK) void k_dot_rv(int64_t n, const float* rhat, const float* v, double* partial) {
  double acc[1] = {0.0};
  GRID_LOOP(i) acc[0] += (double)rhat[i] * v[i];
  block_partials<1>(acc, partial);
}

// omega = <t,s>/<t,t>; x += alpha p + omega s; r = s - omega t; partials <rhat, r>, <r, r>
__global__ __launch_bounds__(BLK) void k_update_xr(int64_t n, Scal* S, const float* p, const float* s, const float* t,
                                                   const float* rhat, float* x, float* r, double* partial) {
  double acc[2] = {0.0, 0.0};
  if (!S->broke) {
    const double omega = S->tt > 0.0 ? S->ts / S->tt : 0.0;
    if (blockIdx.x == 0 && threadIdx.x == 0) S->omega = omega;
    const float fa = (float)S->alpha, fo = (float)omega;
    GRID_LOOP(i) {
      x[i] = x[i] + fa * p[i] + fo * s[i];
      const float ri = s[i] - fo * t[i];
      r[i] = ri;
      acc[0] += (double)rhat[i] * ri;
      acc[1] += (double)ri * ri;
    }
  }
  block_partials<2>(acc, partial);
}

// u += x (float64)
__global__ __launch_bounds__(BLK) void k_accumulate(int64_t n, const float* x, double* u) {
  GRID_LOOP(i) u[i] += (double)x[i];
}

__global__ __launch_bounds__(BLK) void k_to_f32(int64_t nnz, const double* a, float* b) {
  for (int64_t i = (int64_t)blockIdx.x * BLK + threadIdx.x; i < nnz; i += (int64_t)gridDim.x * BLK) b[i] = (float)a[i];
}

// CSR sanity: row_ptr[0] = 0, non-decreasing, column indices in [0, n)
__global__ __launch_bounds__(BLK) void k_check_csr(int64_t n, const int32_t* rp, const int32_t* ci, int32_t* bad) {
  for (int64_t i = (int64_t)blockIdx.x * BLK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BLK) {
    const int32_t a = rp[i], e = rp[i + 1];
    if ((i == 0 && a != 0) || e < a) { *bad = 1; continue; }
    for (int32_t p = a; p < e; ++p)
      if (ci[p] < 0 || ci[p] >= n) { *bad = 1; break; }
  }
}

__global__ __launch_bounds__(BLK) void k_zero(int64_t n, double* u) {
  GRID_LOOP(i) u[i] = 0.0;
}

__global__ void k_zero_flag(int32_t* flag) {
  if (threadIdx.x == 0) *flag = 0;
}

// Bytes of solver scratch for n unknowns and nnz entries: float32 matrix,
// 7 float32 vectors, float64 residual, partials, scalars (and padding).
size_t solve_bytes(int64_t n, int64_t nnz) {
  return ((size_t)nnz + 7 * (size_t)n) * sizeof(float) + ((size_t)n + 3 * RED_BLOCKS) * sizeof(double) +
         sizeof(Scal) + 256;
}

// nnz = row_ptr[n] (synchronises the stream)
pdd_status read_nnz(pdd_ctx* ctx, int64_t n, const int32_t* rp, int32_t* nnz) {
  hipError_t e;
  if ((e = hipMemcpyAsync(nnz, rp + n, sizeof(int32_t), hipMemcpyDeviceToHost, ctx->stream)) != hipSuccess)
    return check_hip(ctx, e, "read nnz");
  if ((e = hipStreamSynchronize(ctx->stream)) != hipSuccess) return check_hip(ctx, e, "hipStreamSynchronize");
  if (*nnz < 1) {
    ctx->err = "pdd_solve: empty matrix (row_ptr[n] < 1)";
    return PDD_EINVAL;
  }
  return PDD_OK;
}

// Validate the CSR structure on the device before any kernel indexes with it
// (flag: one device int32, cleared here by a kernel).
pdd_status check_csr(pdd_ctx* ctx, int64_t n, const int32_t* rp, const int32_t* ci, int32_t* flag) {
  hipStream_t st = ctx->stream;
  hipLaunchKernelGGL(k_zero_flag, dim3(1), dim3(64), 0, st, flag);
  hipLaunchKernelGGL(k_check_csr, dim3((unsigned)std::min<int64_t>(1024, (n + BLK - 1) / BLK)), dim3(BLK), 0, st, n, rp, ci, flag);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return check_hip(ctx, e, "launch csr check");
  int32_t hbad = 0;
  if ((e = hipMemcpyAsync(&hbad, flag, sizeof(int32_t), hipMemcpyDeviceToHost, st)) != hipSuccess) return check_hip(ctx, e, "read flag");
  if ((e = hipStreamSynchronize(st)) != hipSuccess) return check_hip(ctx, e, "hipStreamSynchronize");
  if (hbad) {
    ctx->err = "pdd_solve: malformed CSR (row_ptr not monotone from 0, or a column outside [0, n))";
    return PDD_EINVAL;
  }
  return PDD_OK;
}

// The refinement loop on caller-provided scratch of solve_bytes(n, nnz) bytes
// (256-byte aligned); allocates nothing.
pdd_status solve_body(pdd_ctx* ctx, int64_t n, int32_t nnz, const int32_t* rp, const int32_t* ci, const double* val,
                      const double* b, double* u, double tol, int32_t max_iter, int32_t* iters, double* relres,
                      char* base) {
  hipError_t e;
  hipStream_t st = ctx->stream;
  double* r64 = reinterpret_cast<double*>(base);
  double* partial = r64 + n;
  Scal* S = reinterpret_cast<Scal*>(partial + 3 * RED_BLOCKS);
  float* val32 = reinterpret_cast<float*>(reinterpret_cast<char*>(S) + 128);
  float* x = val32 + nnz;
  float* r = x + n;
  float* rhat = r + n;
  float* p = rhat + n;
  float* v = p + n;
  float* s = v + n;
  float* t = s + n;

  const unsigned rows_grid = (unsigned)((n + BLK / 64 - 1) / (BLK / 64));
  auto L = [&](const char* what) -> pdd_status { return check_hip(ctx, hipGetLastError(), what); };
  pdd_status ps;

  hipLaunchKernelGGL(k_to_f32, dim3(1024), dim3(BLK), 0, st, (int64_t)nnz, val, val32);
  hipLaunchKernelGGL(k_zero, dim3(RED_BLOCKS), dim3(BLK), 0, st, n, u);
  hipLaunchKernelGGL(k_norm2, dim3(RED_BLOCKS), dim3(BLK), 0, st, n, b, partial);
  if ((ps = L("solve setup")) != PDD_OK) return ps;
  double hp[RED_BLOCKS];
  if ((e = hipMemcpyAsync(hp, partial, RED_BLOCKS * sizeof(double), hipMemcpyDeviceToHost, st)) != hipSuccess) return check_hip(ctx, e, "read |b|");
  if ((e = hipStreamSynchronize(st)) != hipSuccess) return check_hip(ctx, e, "hipStreamSynchronize");
  double bb = 0.0;
  for (double q : hp) bb += q;
  const double bnorm = std::sqrt(bb);
  if (bnorm == 0.0) {
    *iters = 0;
    *relres = 0.0;
    return PDD_OK;   // u = 0 solves G u = 0
  }

  const int inner_max = 400;
  const double inner_tol = 1e-5;
  int total = 0;
  double rel = 1.0;
  for (int outer = 0; outer < 50; ++outer) {
    // float64 residual of the current iterate
    hipLaunchKernelGGL(k_residual, dim3(rows_grid), dim3(BLK), 0, st, n, rp, ci, val, u, b, r64);
    hipLaunchKernelGGL(k_norm2, dim3(RED_BLOCKS), dim3(BLK), 0, st, n, r64, partial);
    if ((ps = L("residual")) != PDD_OK) return ps;
    if ((e = hipMemcpyAsync(hp, partial, RED_BLOCKS * sizeof(double), hipMemcpyDeviceToHost, st)) != hipSuccess) return check_hip(ctx, e, "read residual");
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return check_hip(ctx, e, "hipStreamSynchronize");
    double rr = 0.0;
    for (double q : hp) rr += q;
    rel = std::sqrt(rr) / bnorm;
    if (!(rel > tol) || total >= max_iter) break;

    // BiCGStab on G d = r (float32 vectors), d accumulated into u
    hipLaunchKernelGGL(k_init, dim3(RED_BLOCKS), dim3(BLK), 0, st, n, r64, x, r, rhat, p, v, partial);
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(BLK), 0, st, partial, 2, 0, S);
    const double r0 = std::sqrt(rr);
    for (int it = 0; it < inner_max && total < max_iter; ++it, ++total) {
      hipLaunchKernelGGL(k_update_p, dim3(RED_BLOCKS), dim3(BLK), 0, st, n, it == 0 ? 1 : 0, S, r, v, p);
      hipLaunchKernelGGL((k_spmv<float, float>), dim3(rows_grid), dim3(BLK), 0, st, n, rp, ci, val32, p, v);
      hipLaunchKernelGGL(k_dot_rv, dim3(RED_BLOCKS), dim3(BLK), 0, st, n, rhat, v, partial);
      hipLaunchKernelGGL(k_reduce, dim3(1), dim3(BLK), 0, st, partial, 1, 1, S);
      hipLaunchKernelGGL(k_update_s, dim3(RED_BLOCKS), dim3(BLK), 0, st, n, S, r, v, s);
      hipLaunchKernelGGL((k_spmv<float, float>), dim3(rows_grid), dim3(BLK), 0, st, n, rp, ci, val32, s, t);
      hipLaunchKernelGGL(k_dots_ts, dim3(RED_BLOCKS), dim3(BLK), 0, st, n, t, s, partial);
      hipLaunchKernelGGL(k_reduce, dim3(1), dim3(BLK), 0, st, partial, 2, 2, S);
      hipLaunchKernelGGL(k_update_xr, dim3(RED_BLOCKS), dim3(BLK), 0, st, n, S, p, s, t, rhat, x, r, partial);
      hipLaunchKernelGGL(k_reduce, dim3(1), dim3(BLK), 0, st, partial, 2, 3, S);
      if ((ps = L("bicgstab")) != PDD_OK) return ps;
      if ((it & 3) == 3) {
        Scal hs;
        if ((e = hipMemcpyAsync(&hs, S, sizeof(Scal), hipMemcpyDeviceToHost, st)) != hipSuccess) return check_hip(ctx, e, "read scalars");
        if ((e = hipStreamSynchronize(st)) != hipSuccess) return check_hip(ctx, e, "hipStreamSynchronize");
        if (hs.broke || std::sqrt(hs.rr) <= inner_tol * r0) { ++total; break; }
      }
    }
    hipLaunchKernelGGL(k_accumulate, dim3(RED_BLOCKS), dim3(BLK), 0, st, n, x, u);
    if ((ps = L("accumulate")) != PDD_OK) return ps;
  }
  *iters = total;
  *relres = rel;
  if (!(rel <= tol)) {
    ctx->err = "pdd_solve: tolerance not reached within max_iter";
    return PDD_ENOTCONV;
  }
  return PDD_OK;
}

}  // namespace

pdd_status run_solve(pdd_ctx* ctx, int64_t n, const int32_t* rp, const int32_t* ci, const double* val,
                     const double* b, double* u, double tol, int32_t max_iter, int32_t* iters, double* relres) {
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return check_hip(ctx, e, "hipSetDevice");
  int32_t nnz = 0;
  pdd_status ps = read_nnz(ctx, n, rp, &nnz);
  if (ps != PDD_OK) return ps;
  if ((e = ctx->solve_flag.reserve(sizeof(int32_t))) != hipSuccess) return check_hip(ctx, e, "hipMalloc(flag)");
  if ((ps = check_csr(ctx, n, rp, ci, ctx->solve_flag.as<int32_t>())) != PDD_OK) return ps;
  if ((e = ctx->solve_scratch.reserve(solve_bytes(n, nnz))) != hipSuccess) return check_hip(ctx, e, "hipMalloc(solve scratch)");
  return solve_body(ctx, n, nnz, rp, ci, val, b, u, tol, max_iter, iters, relres, ctx->solve_scratch.as<char>());
}

hipError_t solve_noalloc_setup(int device) {
  if (device < 0 || device >= MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device]) return hipSuccess;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch_ptr[device] = ptr;
  return hipSuccess;
}

pdd_status run_solve_noalloc(pdd_ctx* ctx, int64_t n, const int32_t* rp, const int32_t* ci, const double* val,
                             const double* b, double* u, double tol, int32_t max_iter, int32_t* iters,
                             double* relres) {
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return check_hip(ctx, e, "hipSetDevice");
  if ((e = solve_noalloc_setup(ctx->device)) != hipSuccess) return check_hip(ctx, e, "hipGetSymbolAddress(solve scratch)");
  char* base = static_cast<char*>(g_scratch_ptr[ctx->device]);
  int32_t nnz = 0;
  pdd_status ps = read_nnz(ctx, n, rp, &nnz);
  if (ps != PDD_OK) return ps;
  // the first 256 bytes hold the CSR flag, the solver's scratch follows
  if (solve_bytes(n, nnz) + 256 > SOLVE_NOALLOC_BYTES) {
    ctx->err = "pdd_solve_noalloc: n and nnz need more than the static 128 MiB of scratch "
               "(4 (nnz + 7 n) + 8 n bytes plus 7 KiB)";
    return PDD_EINVAL;
  }
  if ((ps = check_csr(ctx, n, rp, ci, reinterpret_cast<int32_t*>(base))) != PDD_OK) return ps;
  return solve_body(ctx, n, nnz, rp, ci, val, b, u, tol, max_iter, iters, relres, base + 256);
}

}  // namespace pdd
