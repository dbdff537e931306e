// The control-variate network v(x) = w3 . tanh(W2 tanh(W1 x + b1) + b2) + b3
// (2 -> 64 -> 64 -> 1) on the GPU: pointwise evaluation with input gradient,
// the single-workgroup Adam trainer, the grad-v table bake, and the kernel
// that collects (path point, tail score) training pairs from the method's own
// paths.
//
// Any adapted F keeps the mean of the Feynman-Kac score (eq. 38); F = sigma^T
// grad u would remove the variance (eq. 11).  The network is fitted to
// pathwise estimates of u: for a point X_n of a path that exits at step K,
// E[(Z_K + Y_K u(X_K) - Z_n) / Y_n | X_n] = u(X_n), with u at the exit taken
// from the solved knot values (hat interpolation) or the boundary datum.
//
// Parameter layout (4417 float32): W1[64][2], b1[64], W2[64][64] (out, in),
// b2[64], w3[64], b3.
#include <hip/hip_runtime.h>

#include <cmath>

#include "context.h"
#include "device_common.h"
#include "mlp.h"

namespace pdd {

namespace {

constexpr int BLK = 256;

__device__ __forceinline__ float tanh_f(float z) {
  // 1 - 2 / (exp(2z) + 1): exact limits +-1, one exp and one reciprocal
  const float e = __builtin_amdgcn_exp2f(z * 2.8853900817779268f);
  return 1.0f - 2.0f * __builtin_amdgcn_rcpf(e + 1.0f);
}

// v and grad v at one point, float32 throughout, parameters from `th`
__device__ __forceinline__ void net_eval_f32(const float* __restrict__ th, float x, float y, float& v, float& gx,
                                             float& gy) {
  float h1[MLP_W];
#pragma unroll
  for (int k = 0; k < MLP_W; ++k)
    h1[k] = tanhf(th[OW1 + 2 * k] * x + th[OW1 + 2 * k + 1] * y + th[OB1 + k]);
  float g1[MLP_W];
#pragma unroll
  for (int k = 0; k < MLP_W; ++k) g1[k] = 0.0f;
  float vv = th[OB3];
  for (int j = 0; j < MLP_W; ++j) {
    float z = th[OB2 + j];
#pragma unroll
    for (int k = 0; k < MLP_W; ++k) z += th[OW2 + j * MLP_W + k] * h1[k];
    const float h2 = tanhf(z);
    vv += th[OW3 + j] * h2;
    const float g2 = (1.0f - h2 * h2) * th[OW3 + j];
#pragma unroll
    for (int k = 0; k < MLP_W; ++k) g1[k] += th[OW2 + j * MLP_W + k] * g2;
  }
  float ax = 0.0f, ay = 0.0f;
#pragma unroll
  for (int k = 0; k < MLP_W; ++k) {
    const float d = (1.0f - h1[k] * h1[k]) * g1[k];
    ax += th[OW1 + 2 * k] * d;
    ay += th[OW1 + 2 * k + 1] * d;
  }
  v = vv;
  gx = ax;
  gy = ay;
}

__global__ __launch_bounds__(BLK) void k_mlp_eval(const float* __restrict__ params, int64_t n, const float* __restrict__ xy,
                                                  float* __restrict__ v, float* __restrict__ g) {
  __shared__ float th[MLP_PARAMS];
  for (int i = threadIdx.x; i < MLP_PARAMS; i += BLK) th[i] = params[i];
  __syncthreads();
  for (int64_t i = (int64_t)blockIdx.x * BLK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BLK) {
    float vv, gx, gy;
    net_eval_f32(th, xy[2 * i], xy[2 * i + 1], vv, gx, gy);
    if (v) v[i] = vv;
    if (g) { g[2 * i] = gx; g[2 * i + 1] = gy; }
  }
}

// grad v on the node-centred grid of the domain: grad_lut[(j n + i) 2 + d]
__global__ __launch_bounds__(BLK) void k_mlp_bake(const float* __restrict__ params, int lut_n, double x0, double x1,
                                                  double y0, double y1, float* __restrict__ out) {
  __shared__ float th[MLP_PARAMS];
  for (int i = threadIdx.x; i < MLP_PARAMS; i += BLK) th[i] = params[i];
  __syncthreads();
  const int64_t total = (int64_t)lut_n * lut_n;
  for (int64_t q = (int64_t)blockIdx.x * BLK + threadIdx.x; q < total; q += (int64_t)gridDim.x * BLK) {
    const int i = (int)(q % lut_n), j = (int)(q / lut_n);
    const float x = (float)(x0 + (double)i * (x1 - x0) / (double)(lut_n - 1));
    const float y = (float)(y0 + (double)j * (y1 - y0) / (double)(lut_n - 1));
    float vv, gx, gy;
    net_eval_f32(th, x, y, vv, gx, gy);
    out[2 * q] = gx;
    out[2 * q + 1] = gy;
  }
}

// ---- single-workgroup trainer ---------------------------------------------
// One workgroup runs every Adam step (the steps are sequential).  The batch is
// processed in chunks of 32 points by 256 threads, 8 per point, each owning 8
// hidden units; per-point vectors are staged in LDS and every thread then
// accumulates the gradient entries it owns (parameter q = tid + 256 i) over
// the chunk.  Parameters stay in LDS; Adam moments live in global memory and
// are touched once per step.
struct TrainArgs {
  float* params;
  float* m;
  float* s;
  const float* xy;
  const float* target;
  const int32_t* order;
  int64_t n_order;
  int64_t n_points;       // order entries outside [0, n_points) are skipped
  int32_t batch;
  int32_t steps;
  int32_t step0;          // Adam step counter before this call
  float lr;
  int32_t update;         // 0: write the gradient of the first batch to grad_out only
  float* grad_out;
  float* losses;          // per step, nullable
};

constexpr int OWN = (MLP_PARAMS + BLK - 1) / BLK;   // 18

__global__ __launch_bounds__(BLK) void k_mlp_train(TrainArgs A) {
  __shared__ float th[MLP_PARAMS];
  __shared__ float sh1[32][MLP_W + 1], sh2[32][MLP_W + 1], sdz2[32][MLP_W + 1], sdz1[32][MLP_W + 1];
  __shared__ float sx[32][2], sdv[32];
  __shared__ float sred[BLK / 64];
  const int tid = threadIdx.x;
  const int pt = tid >> 3, part = tid & 7;      // point within the chunk, hidden-unit slice
  for (int i = tid; i < MLP_PARAMS; i += BLK) th[i] = A.params[i];
  __syncthreads();
  const float inv_b = 1.0f / (float)A.batch;

  for (int step = 0; step < A.steps; ++step) {
    float g[OWN];
#pragma unroll
    for (int i = 0; i < OWN; ++i) g[i] = 0.0f;
    float loss = 0.0f;
    for (int c0 = 0; c0 < A.batch; c0 += 32) {
      const int p = c0 + pt;
      const int64_t oi = ((int64_t)step * A.batch + p) % A.n_order;
      const int32_t oidx = p < A.batch ? A.order[oi] : -1;
      const bool valid = oidx >= 0 && (int64_t)oidx < A.n_points;
      const int32_t idx = valid ? oidx : 0;
      const float x = valid ? A.xy[2 * (int64_t)idx] : 0.0f;
      const float y = valid ? A.xy[2 * (int64_t)idx + 1] : 0.0f;
      if (part == 0) { sx[pt][0] = x; sx[pt][1] = y; }
      // layer 1 (8 units per thread)
      for (int u = 0; u < 8; ++u) {
        const int k = part * 8 + u;
        sh1[pt][k] = tanhf(th[OW1 + 2 * k] * x + th[OW1 + 2 * k + 1] * y + th[OB1 + k]);
      }
      __syncthreads();
      // layer 2 and output
      float vpart = 0.0f;
      float h2v[8];
      for (int u = 0; u < 8; ++u) {
        const int j = part * 8 + u;
        float z = th[OB2 + j];
        for (int k = 0; k < MLP_W; ++k) z += th[OW2 + j * MLP_W + k] * sh1[pt][k];
        h2v[u] = tanhf(z);
        sh2[pt][j] = h2v[u];
        vpart += th[OW3 + j] * h2v[u];
      }
      // sum the 8 slices of a point (adjacent lanes)
      vpart += __shfl_xor(vpart, 1, 64);
      vpart += __shfl_xor(vpart, 2, 64);
      vpart += __shfl_xor(vpart, 4, 64);
      const float v = vpart + th[OB3];
      const float t = valid ? A.target[idx] : v;
      const float r = valid ? (v - t) : 0.0f;
      const float dv = r * inv_b;
      if (part == 0) { sdv[pt] = dv; loss += 0.5f * r * r * inv_b; }
      for (int u = 0; u < 8; ++u) {
        const int j = part * 8 + u;
        sdz2[pt][j] = dv * th[OW3 + j] * (1.0f - h2v[u] * h2v[u]);
      }
      __syncthreads();
      // back to layer 1
      for (int u = 0; u < 8; ++u) {
        const int k = part * 8 + u;
        float d = 0.0f;
        for (int j = 0; j < MLP_W; ++j) d += th[OW2 + j * MLP_W + k] * sdz2[pt][j];
        const float h = sh1[pt][k];
        sdz1[pt][k] = d * (1.0f - h * h);
      }
      __syncthreads();
      // accumulate owned gradient entries over the chunk
#pragma unroll
      for (int i = 0; i < OWN; ++i) {
        const int q = tid + BLK * i;
        if (q >= MLP_PARAMS) break;
        float acc = 0.0f;
        if (q < OB1) {
          const int k = q >> 1, dd = q & 1;
          for (int pp = 0; pp < 32; ++pp) acc += sdz1[pp][k] * sx[pp][dd];
        } else if (q < OW2) {
          const int k = q - OB1;
          for (int pp = 0; pp < 32; ++pp) acc += sdz1[pp][k];
        } else if (q < OB2) {
          const int j = (q - OW2) / MLP_W, k = (q - OW2) % MLP_W;
          for (int pp = 0; pp < 32; ++pp) acc += sdz2[pp][j] * sh1[pp][k];
        } else if (q < OW3) {
          const int j = q - OB2;
          for (int pp = 0; pp < 32; ++pp) acc += sdz2[pp][j];
        } else if (q < OB3) {
          const int j = q - OW3;
          for (int pp = 0; pp < 32; ++pp) acc += sdv[pp] * sh2[pp][j];
        } else {
          for (int pp = 0; pp < 32; ++pp) acc += sdv[pp];
        }
        g[i] += acc;
      }
      __syncthreads();
    }
    // loss of the step (block reduction)
    float lw = loss;
    for (int off = 32; off > 0; off >>= 1) lw += __shfl_xor(lw, off, 64);
    if ((tid & 63) == 0) sred[tid >> 6] = lw;
    __syncthreads();
    if (tid == 0 && A.losses) A.losses[step] = sred[0] + sred[1] + sred[2] + sred[3];
    if (!A.update) {
#pragma unroll
      for (int i = 0; i < OWN; ++i) {
        const int q = tid + BLK * i;
        if (q < MLP_PARAMS) A.grad_out[q] = g[i];
      }
      return;
    }
    // Adam (bias-corrected), beta1 = 0.9, beta2 = 0.999, eps = 1e-8
    const int tstep = A.step0 + step + 1;
    const float c1 = 1.0f - powf(0.9f, (float)tstep);
    const float c2 = 1.0f - powf(0.999f, (float)tstep);
#pragma unroll
    for (int i = 0; i < OWN; ++i) {
      const int q = tid + BLK * i;
      if (q >= MLP_PARAMS) break;
      const float mq = 0.9f * A.m[q] + 0.1f * g[i];
      const float sq = 0.999f * A.s[q] + 0.001f * g[i] * g[i];
      A.m[q] = mq;
      A.s[q] = sq;
      th[q] -= A.lr * (mq / c1) / (sqrtf(sq / c2) + 1e-8f);
    }
    __syncthreads();
  }
  for (int i = tid; i < MLP_PARAMS; i += BLK) A.params[i] = th[i];
}

}  // namespace

pdd_status run_mlp_eval(pdd_ctx* ctx, const float* params, int64_t n, const float* xy, float* v, float* g) {
  const int grid = (int)std::min<int64_t>(4096, (n + BLK - 1) / BLK);
  hipLaunchKernelGGL(k_mlp_eval, dim3(std::max(grid, 1)), dim3(BLK), 0, ctx->stream, params, n, xy, v, g);
  return check_hip(ctx, hipGetLastError(), "launch mlp_eval");
}

pdd_status run_mlp_bake(pdd_ctx* ctx, const float* params, const pdd_partition& part, int32_t lut_n, float* out) {
  const int64_t total = (int64_t)lut_n * lut_n;
  const int grid = (int)std::min<int64_t>(8192, (total + BLK - 1) / BLK);
  hipLaunchKernelGGL(k_mlp_bake, dim3(grid), dim3(BLK), 0, ctx->stream, params, lut_n, part.x0, part.x1, part.y0,
                     part.y1, out);
  return check_hip(ctx, hipGetLastError(), "launch mlp_bake");
}

pdd_status run_mlp_train(pdd_ctx* ctx, float* params, float* m, float* s, int64_t n_points, const float* xy,
                         const float* target, const int32_t* order, int64_t n_order, int32_t batch, int32_t steps,
                         int32_t step0, float lr, float* losses, float* grad_out) {
  TrainArgs A;
  A.n_points = n_points;
  A.params = params; A.m = m; A.s = s; A.xy = xy; A.target = target; A.order = order;
  A.n_order = n_order; A.batch = batch; A.steps = steps; A.step0 = step0; A.lr = lr;
  A.update = grad_out ? 0 : 1;
  A.grad_out = grad_out;
  A.losses = losses;
  hipLaunchKernelGGL(k_mlp_train, dim3(1), dim3(BLK), 0, ctx->stream, A);
  return check_hip(ctx, hipGetLastError(), "launch mlp_train");
}

}  // namespace pdd
