// The control-variate network v(x) = w3 . tanh(W2 tanh(W1 x + b1) + b2) + b3
// (2 -> 64 -> 64 -> 1) on the GPU: pointwise evaluation with input gradient,
// the single-workgroup Adam trainer (float32 MFMA), the grad-v table bake, and the kernel
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
#include "net_grad.h"

namespace pdd {

namespace {

constexpr int BLK = 256;

// tanh for the trainer: 1 - 2 / (exp(2z) + 1) (one exp, one reciprocal,
// exact limits +-1, absolute error about 1e-7), and for |z| < 1/16 the odd
// Taylor polynomial z - z^3/3 + 2 z^5/15 (relative error below 1e-8), where
// the first form would lose relative accuracy
__device__ __forceinline__ float tanh_f(float z) {
  const float e = __builtin_amdgcn_exp2f(z * 2.8853900817779268f);
  const float t = 1.0f - 2.0f * __builtin_amdgcn_rcpf(e + 1.0f);
  const float z2 = z * z;
  const float p = z * __builtin_fmaf(z2, __builtin_fmaf(z2, 0.13333333f, -0.33333333f), 1.0f);
  return __builtin_fabsf(z) < 0.0625f ? p : t;
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

// grad v through net_grad_mfma, the routine the float32 network control
// variate runs at every Euler step of the assembly: each wave takes 64
// consecutive points per pass.  Lanes past the end repeat the last point, so
// every lane of the wave takes part in the MFMA products, and store nothing.
__global__ __launch_bounds__(BLK) void k_mlp_grad_bf16(const float* __restrict__ params, int64_t n,
                                                       const float* __restrict__ xy, float* __restrict__ g) {
  __shared__ NetLds N;
  net_stage(&N, params);
  __syncthreads();
  const int lane = (int)(threadIdx.x & 63);
  const int64_t waves = (int64_t)gridDim.x * (BLK / 64);
  const int64_t wave = (int64_t)blockIdx.x * (BLK / 64) + (threadIdx.x >> 6);
  for (int64_t base = wave * 64; base < n; base += waves * 64) {      // wave-uniform bound
    const int64_t i = base + lane;
    const int64_t r = i < n ? i : n - 1;
    float gx, gy;
    net_grad_mfma(&N, xy[2 * r], xy[2 * r + 1], gx, gy);
    if (i < n) {
      g[2 * i] = gx;
      g[2 * i + 1] = gy;
    }
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
    // the network's input: the node in the domain's unit coordinates; the
    // gradient scaled back to the domain's
    const float x = (float)((double)i / (double)(lut_n - 1));
    const float y = (float)((double)j / (double)(lut_n - 1));
    float vv, gx, gy;
    net_eval_f32(th, x, y, vv, gx, gy);
    out[2 * q] = gx * (float)(1.0 / (x1 - x0));
    out[2 * q + 1] = gy * (float)(1.0 / (y1 - y0));
  }
}

// ---- single-workgroup trainer (float32 MFMA) ---------------------------------
// One workgroup of four waves runs every Adam step (the steps are
// sequential).  A step's minibatch is processed in rounds of 128 points, 32
// per wave.  Per wave and round, with points as the columns c = lane % 32 and
// the two half-waves h = lane / 32 splitting the contraction index:
//   h1 = tanh(W1 x + b1)                          VALU, 32 values per lane
//   z2^T = W2 h1^T                                v_mfma_f32_32x32x2_f32, K = 64
//   h2 = tanh(z2 + b2), v = w3 . h2 + b3, dv = (v - t) / B
//   dz2^T = dv (1 - h2^2) w3                      in registers
//   gW2 += dz2^T h1                               MFMA, K = the 32 points
//   dh1^T = W2^T dz2^T, dz1 = dh1 (1 - h1^2)      MFMA, K = 64
//   gW1, gb1, gb2, gw3, gb3                       VALU sums over the points
// The contraction order of z2 and dh1 follows the accumulator's row order
// (row = 8 (r / 4) + 4 h + r % 4 of register r), so h1 and dz2 serve as
// operands straight from registers; the batch contractions read the wave's
// LDS copies.  The four waves' gradients are summed in wave order (fixed,
// reproducible), then every thread applies Adam to the parameters it owns.
// Parameters stay in LDS; each thread keeps the Adam moments of the
// parameters it owns in registers for the whole call.
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
  // wide steps (update == 0, one step per launch): workgroup g takes the
  // points [g slice, (g + 1) slice) of the batch of order step `order_step`
  // and writes its gradient sum (and loss) to grad_out + g GPAD
  int32_t slice;          // 0: the whole batch in one workgroup
  int32_t order_step;
};

typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;

constexpr int TW = 4;                 // waves per workgroup
constexpr int WIDE_BATCH = 1024;      // larger batches take the multi-workgroup step
constexpr int H1S = 68;               // row stride of the h1 copy [point][unit] (16-byte aligned rows)
constexpr int DZS = 36;               // row stride of the [unit][point] copies
constexpr int PARAM_PAD = ((MLP_PARAMS + 3) / 4) * 4;

struct TrainWaveLds {
  float h1[32 * H1S];                 // h1[c][k]
  float dz[64 * DZS];                 // dz2^T[j][c], later dz1^T[k][c]
  float dh[64 * DZS];                 // dv_c h2[j][c]
  float xy[32][2];
};

constexpr size_t train_lds_bytes() { return PARAM_PAD * sizeof(float) + TW * sizeof(TrainWaveLds); }
constexpr int OWN = (MLP_PARAMS + TW * 64 - 1) / (TW * 64);   // parameters per thread in Adam
constexpr int GSTRIDE = PARAM_PAD + 4;                         // one wave's gradient slice (+ loss)
constexpr int GPAD = PARAM_PAD + 4;                            // one workgroup's gradient (+ loss), wide steps
static_assert(TW * GSTRIDE * sizeof(float) <= TW * sizeof(TrainWaveLds), "gradient slices fit the wave buffers");

// accumulator register r of a 32 x 32 tile holds row 8 (r / 4) + 4 h + r % 4
__device__ __forceinline__ int acc_row(int r, int h) { return 8 * (r >> 2) + 4 * h + (r & 3); }

__global__ __launch_bounds__(TW * 64) void k_mlp_train(TrainArgs A) {
  extern __shared__ float tlds[];
  float* th = tlds;
  TrainWaveLds* WL = reinterpret_cast<TrainWaveLds*>(tlds + PARAM_PAD);
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, h = lane >> 5, c = lane & 31;
  TrainWaveLds& L = WL[w];
  for (int i = tid; i < MLP_PARAMS; i += TW * 64) th[i] = A.params[i];
  float mown[OWN], sown[OWN];           // Adam moments of parameters tid + i TW 64
#pragma unroll
  for (int i = 0; i < OWN; ++i) {
    const int q = tid + i * TW * 64;
    mown[i] = (q < MLP_PARAMS && A.update) ? A.m[q] : 0.0f;
    sown[i] = (q < MLP_PARAMS && A.update) ? A.s[q] : 0.0f;
  }
  __syncthreads();
  const float inv_b = 1.0f / (float)A.batch;
  // this workgroup's points of each batch: all of them, or one slice
  const int pbase = A.slice > 0 ? (int)blockIdx.x * A.slice : 0;
  const int pend = A.slice > 0 ? min(A.batch, pbase + A.slice) : A.batch;
  const int rounds = (pend - pbase + 32 * TW - 1) / (32 * TW);

  for (int step = 0; step < A.steps; ++step) {
    f32x16 gw2[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) gw2[a][b] = f32x16{};
    float g_b2 = 0.0f, g_w3 = 0.0f, g_w1x = 0.0f, g_w1y = 0.0f, g_b1 = 0.0f, g_b3 = 0.0f, loss = 0.0f;

    for (int rd = 0; rd < rounds; ++rd) {
      const int p = pbase + rd * 32 * TW + 32 * w + c;
      const bool inb = p < pend;
      const int64_t oi = ((int64_t)(step + A.order_step) * A.batch + p) % A.n_order;
      const int32_t oidx = inb ? A.order[oi] : -1;
      const bool valid = oidx >= 0 && (int64_t)oidx < A.n_points;
      const int32_t idx = valid ? oidx : 0;
      const float x = valid ? A.xy[2 * (int64_t)idx] : 0.0f;
      const float y = valid ? A.xy[2 * (int64_t)idx + 1] : 0.0f;
      const float t = valid ? A.target[idx] : 0.0f;
      if (h == 0) { L.xy[c][0] = x; L.xy[c][1] = y; }
      // layer 1: units k = 32 kb + acc_row(r, h) of point c
      float h1r[2][16];
#pragma unroll
      for (int kb = 0; kb < 2; ++kb)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int k = 32 * kb + acc_row(r, h);
          const float v = tanh_f(th[OW1 + 2 * k] * x + th[OW1 + 2 * k + 1] * y + th[OB1 + k]);
          h1r[kb][r] = v;
          L.h1[c * H1S + k] = v;
        }
      // layer 2: z2^T[j][c], contraction k(s, h) = 32 (s / 16) + acc_row(s % 16, h)
      f32x16 z[2];
#pragma unroll
      for (int jb = 0; jb < 2; ++jb) {
        z[jb] = f32x16{};
        const float* wrow = th + OW2 + (32 * jb + c) * MLP_W;
#pragma unroll
        for (int q = 0; q < 8; ++q) {          // four steps s = 4q .. 4q+3 read four consecutive k
          const float4 a4 = *reinterpret_cast<const float4*>(wrow + 32 * (q >> 2) + 8 * (q & 3) + 4 * h);
          const float av[4] = {a4.x, a4.y, a4.z, a4.w};
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int s2 = 4 * q + e;
            z[jb] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[e], h1r[s2 >> 4][s2 & 15], z[jb], 0, 0, 0);
          }
        }
      }
      // output, residual and dz2 (registers: rows j = 32 jb + acc_row(r, h) of column c)
      float vpart = 0.0f;
      float dz2r[2][16];
#pragma unroll
      for (int jb = 0; jb < 2; ++jb)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int j = 32 * jb + acc_row(r, h);
          const float h2 = tanh_f(z[jb][r] + th[OB2 + j]);
          vpart += th[OW3 + j] * h2;
          z[jb][r] = h2;
          dz2r[jb][r] = (1.0f - h2 * h2) * th[OW3 + j];
        }
      const float v = vpart + __shfl_xor(vpart, 32, 64) + th[OB3];
      const float res = valid ? v - t : 0.0f;
      const float dv = res * inv_b;
      if (h == 0) { loss += 0.5f * res * res * inv_b; g_b3 += dv; }
#pragma unroll
      for (int jb = 0; jb < 2; ++jb)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int j = 32 * jb + acc_row(r, h);
          dz2r[jb][r] *= dv;
          L.dz[j * DZS + c] = dz2r[jb][r];
          L.dh[j * DZS + c] = dv * z[jb][r];
        }
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      __builtin_amdgcn_wave_barrier();
      // gb2[j], gw3[j] for j = lane: sums over the 32 points
      {
        const float4* dzr = reinterpret_cast<const float4*>(L.dz + lane * DZS);
        const float4* dhr = reinterpret_cast<const float4*>(L.dh + lane * DZS);
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const float4 a4 = dzr[q], b4 = dhr[q];
          g_b2 += (a4.x + a4.y) + (a4.z + a4.w);
          g_w3 += (b4.x + b4.y) + (b4.z + b4.w);
        }
      }
      // gW2[j][k] += sum_c dz2^T[j][c] h1[c][k]; contraction c(s, h) = 16 h + s
#pragma unroll
      for (int jb = 0; jb < 2; ++jb) {
        const float* arow = L.dz + (32 * jb + c) * DZS + 16 * h;
        float av[16];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const float4 a4 = *reinterpret_cast<const float4*>(arow + 4 * q);
          av[4 * q] = a4.x; av[4 * q + 1] = a4.y; av[4 * q + 2] = a4.z; av[4 * q + 3] = a4.w;
        }
#pragma unroll
        for (int kb = 0; kb < 2; ++kb)
#pragma unroll
          for (int s2 = 0; s2 < 16; ++s2)
            gw2[jb][kb] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[s2], L.h1[(16 * h + s2) * H1S + 32 * kb + c],
                                                               gw2[jb][kb], 0, 0, 0);
      }
      // backward: dh1^T[k][c] = sum_j W2[j][k] dz2^T[j][c], contraction j(s, h) = 32 (s / 16) + acc_row(s % 16, h)
      float dz1r[2][16];
#pragma unroll
      for (int kb = 0; kb < 2; ++kb) {
        f32x16 d = f32x16{};
#pragma unroll
        for (int s2 = 0; s2 < 32; ++s2) {
          const int j = 32 * (s2 >> 4) + acc_row(s2 & 15, h);
          d = __builtin_amdgcn_mfma_f32_32x32x2f32(th[OW2 + j * MLP_W + 32 * kb + c], dz2r[s2 >> 4][s2 & 15], d, 0, 0, 0);
        }
#pragma unroll
        for (int r = 0; r < 16; ++r) dz1r[kb][r] = d[r] * (1.0f - h1r[kb][r] * h1r[kb][r]);
      }
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      __builtin_amdgcn_wave_barrier();
#pragma unroll
      for (int kb = 0; kb < 2; ++kb)
#pragma unroll
        for (int r = 0; r < 16; ++r) L.dz[(32 * kb + acc_row(r, h)) * DZS + c] = dz1r[kb][r];
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      __builtin_amdgcn_wave_barrier();
      // gW1[k][.], gb1[k] for k = lane: sums over the 32 points
      {
        const float4* dzr = reinterpret_cast<const float4*>(L.dz + lane * DZS);
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const float4 a4 = dzr[q];
          const float av[4] = {a4.x, a4.y, a4.z, a4.w};
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int cc = 4 * q + e;
            g_w1x += av[e] * L.xy[cc][0];
            g_w1y += av[e] * L.xy[cc][1];
            g_b1 += av[e];
          }
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      __builtin_amdgcn_wave_barrier();
    }
    // loss and gb3 of the wave (lanes with h == 0 hold one point each)
    for (int off = 32; off > 0; off >>= 1) {
      loss += __shfl_xor(loss, off, 64);
      g_b3 += __shfl_xor(g_b3, off, 64);
    }
    // the four waves' gradients into four slices of the (now free) wave
    // buffers, then summed per parameter in wave order (fixed, reproducible)
    __syncthreads();
    float* Gw = reinterpret_cast<float*>(WL) + w * GSTRIDE;
#pragma unroll
    for (int jb = 0; jb < 2; ++jb)
#pragma unroll
      for (int kb = 0; kb < 2; ++kb)
#pragma unroll
        for (int r = 0; r < 16; ++r) Gw[OW2 + (32 * jb + acc_row(r, h)) * MLP_W + 32 * kb + c] = gw2[jb][kb][r];
    Gw[OW1 + 2 * lane] = g_w1x;
    Gw[OW1 + 2 * lane + 1] = g_w1y;
    Gw[OB1 + lane] = g_b1;
    Gw[OB2 + lane] = g_b2;
    Gw[OW3 + lane] = g_w3;
    if (lane == 0) { Gw[OB3] = g_b3; Gw[MLP_PARAMS] = loss; }
    __syncthreads();
    const float* G0 = reinterpret_cast<const float*>(WL);
    auto gsum = [&](int q) __attribute__((always_inline)) {
      return ((G0[q] + G0[GSTRIDE + q]) + G0[2 * GSTRIDE + q]) + G0[3 * GSTRIDE + q];
    };
    if (!A.update) {
      if (A.slice > 0) {
        float* out = A.grad_out + (size_t)blockIdx.x * GPAD;
        for (int q = tid; q <= MLP_PARAMS; q += TW * 64) out[q] = gsum(q);
        return;
      }
      if (tid == 0 && A.losses) A.losses[step] = gsum(MLP_PARAMS);
      for (int q = tid; q < MLP_PARAMS; q += TW * 64) A.grad_out[q] = gsum(q);
      return;
    }
    if (tid == 0 && A.losses) A.losses[step] = gsum(MLP_PARAMS);
    // Adam (bias-corrected), beta1 = 0.9, beta2 = 0.999, eps = 1e-8; each
    // thread keeps the moments of the parameters it owns in registers
    const int tstep = A.step0 + step + 1;
    const float c1 = 1.0f - powf(0.9f, (float)tstep);
    const float c2 = 1.0f - powf(0.999f, (float)tstep);
#pragma unroll
    for (int i = 0; i < OWN; ++i) {
      const int q = tid + i * TW * 64;
      if (q < MLP_PARAMS) {
        const float g = gsum(q);
        const float mq = 0.9f * mown[i] + 0.1f * g;
        const float sq = 0.999f * sown[i] + 0.001f * g * g;
        mown[i] = mq;
        sown[i] = sq;
        th[q] -= A.lr * (mq / c1) / (sqrtf(sq / c2) + 1e-8f);
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < OWN; ++i) {
    const int q = tid + i * TW * 64;
    if (q < MLP_PARAMS && A.update) {
      A.m[q] = mown[i];
      A.s[q] = sown[i];
    }
  }
  for (int i = tid; i < MLP_PARAMS; i += TW * 64) A.params[i] = th[i];
}


// Glorot-uniform weights, zero biases: parameter i of a weight matrix with
// fan sum F is lim (2u - 1), lim = sqrt(6 / F), u the float64 uniform of the
// first word of Philox4x32-10 at counter (i, 0, 0, 0), key (seed lo, seed hi)
__global__ __launch_bounds__(BLK) void k_mlp_init(float* __restrict__ params, uint32_t k0, uint32_t k1) {
  const int i = blockIdx.x * BLK + threadIdx.x;
  if (i >= MLP_PARAMS) return;
  int fan = 0;
  if (i < OB1) fan = MLP_W + 2;
  else if (i >= OW2 && i < OB2) fan = 2 * MLP_W;
  else if (i >= OW3 && i < OB3) fan = MLP_W + 1;
  float w = 0.0f;
  if (fan) {
    const double u = uniform64(philox10((uint32_t)i, 0u, 0u, 0u, k0, k1).a);
    w = (float)(sqrt(6.0 / fan) * (2.0 * u - 1.0));
  }
  params[i] = w;
}

}  // namespace

pdd_status run_mlp_init(pdd_ctx* ctx, float* params, uint64_t seed) {
  hipLaunchKernelGGL(k_mlp_init, dim3((MLP_PARAMS + BLK - 1) / BLK), dim3(BLK), 0, ctx->stream, params,
                     (uint32_t)seed, (uint32_t)(seed >> 32));
  return check_hip(ctx, hipGetLastError(), "launch mlp_init");
}

pdd_status run_mlp_eval(pdd_ctx* ctx, const float* params, int64_t n, const float* xy, float* v, float* g) {
  const int grid = (int)std::min<int64_t>(4096, (n + BLK - 1) / BLK);
  hipLaunchKernelGGL(k_mlp_eval, dim3(std::max(grid, 1)), dim3(BLK), 0, ctx->stream, params, n, xy, v, g);
  return check_hip(ctx, hipGetLastError(), "launch mlp_eval");
}

pdd_status run_mlp_grad_bf16(pdd_ctx* ctx, const float* params, int64_t n, const float* xy, float* g) {
  const int64_t waves = (n + 63) / 64;
  const int grid = (int)std::min<int64_t>(2048, (waves + BLK / 64 - 1) / (BLK / 64));
  hipLaunchKernelGGL(k_mlp_grad_bf16, dim3(std::max(grid, 1)), dim3(BLK), 0, ctx->stream, params, n, xy, g);
  return check_hip(ctx, hipGetLastError(), "launch mlp_grad_bf16");
}

pdd_status run_mlp_bake(pdd_ctx* ctx, const float* params, const pdd_partition& part, int32_t lut_n, float* out) {
  const int64_t total = (int64_t)lut_n * lut_n;
  const int grid = (int)std::min<int64_t>(8192, (total + BLK - 1) / BLK);
  hipLaunchKernelGGL(k_mlp_bake, dim3(grid), dim3(BLK), 0, ctx->stream, params, lut_n, part.x0, part.x1, part.y0,
                     part.y1, out);
  return check_hip(ctx, hipGetLastError(), "launch mlp_bake");
}

// Adam step of a wide step: the workgroups' gradients summed in workgroup
// order (fixed), then the same bias-corrected update as the trainer, with the
// moments in global memory.
__global__ __launch_bounds__(256) void k_mlp_adam(float* __restrict__ params, float* __restrict__ m,
                                                  float* __restrict__ s, const float* __restrict__ part, int groups,
                                                  int tstep, float lr, float* losses) {
  const float c1 = 1.0f - powf(0.9f, (float)tstep);
  const float c2 = 1.0f - powf(0.999f, (float)tstep);
  for (int q = threadIdx.x; q <= MLP_PARAMS; q += 256) {
    float g = 0.0f;
    for (int b = 0; b < groups; ++b) g += part[(size_t)b * GPAD + q];
    if (q == MLP_PARAMS) {
      if (losses) *losses = g;
      continue;
    }
    const float mq = 0.9f * m[q] + 0.1f * g;
    const float sq = 0.999f * s[q] + 0.001f * g * g;
    m[q] = mq;
    s[q] = sq;
    params[q] -= lr * (mq / c1) / (sqrtf(sq / c2) + 1e-8f);
  }
}

pdd_status run_mlp_train(pdd_ctx* ctx, float* params, float* m, float* s, int64_t n_points, const float* xy,
                         const float* target, const int32_t* order, int64_t n_order, int32_t batch, int32_t steps,
                         int32_t step0, float lr, float* losses, float* grad_out) {
  // batches above WIDE_BATCH: every step spread over workgroups of 256 points
  if (grad_out == nullptr && batch > WIDE_BATCH) {
    const int groups = (batch + 255) / 256;
    hipError_t e = ctx->mlp_wide.reserve((size_t)groups * GPAD * sizeof(float));
    if (e != hipSuccess) return check_hip(ctx, e, "hipMalloc(mlp wide)");
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_mlp_train), hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)train_lds_bytes());
    if (e != hipSuccess) return check_hip(ctx, e, "hipFuncSetAttribute(mlp_train)");
    TrainArgs A;
    A.n_points = n_points;
    A.params = params; A.m = m; A.s = s; A.xy = xy; A.target = target; A.order = order;
    A.n_order = n_order; A.batch = batch; A.steps = 1; A.step0 = 0; A.lr = lr;
    A.update = 0;
    A.grad_out = ctx->mlp_wide.as<float>();
    A.losses = nullptr;
    A.slice = 256;
    for (int32_t st = 0; st < steps; ++st) {
      A.order_step = st;
      hipLaunchKernelGGL(k_mlp_train, dim3(groups), dim3(TW * 64), train_lds_bytes(), ctx->stream, A);
      hipLaunchKernelGGL(k_mlp_adam, dim3(1), dim3(256), 0, ctx->stream, params, m, s, A.grad_out, groups,
                         step0 + st + 1, lr, losses ? losses + st : nullptr);
    }
    return check_hip(ctx, hipGetLastError(), "launch mlp_train (wide)");
  }
  TrainArgs A;
  A.n_points = n_points;
  A.params = params; A.m = m; A.s = s; A.xy = xy; A.target = target; A.order = order;
  A.n_order = n_order; A.batch = batch; A.steps = steps; A.step0 = step0; A.lr = lr;
  A.update = grad_out ? 0 : 1;
  A.grad_out = grad_out;
  A.losses = losses;
  A.slice = 0;
  A.order_step = 0;
  // more than 64 KiB of LDS for one workgroup (gfx950 allows 160 KiB)
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_mlp_train),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)train_lds_bytes());
  if (e != hipSuccess) return check_hip(ctx, e, "hipFuncSetAttribute(mlp_train)");
  hipLaunchKernelGGL(k_mlp_train, dim3(1), dim3(TW * 64), train_lds_bytes(), ctx->stream, A);
  return check_hip(ctx, hipGetLastError(), "launch mlp_train");
}

}  // namespace pdd
