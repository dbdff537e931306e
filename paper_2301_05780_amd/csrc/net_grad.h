// grad v of the control-variate network inside the path kernels.
//
// float32 production: one wave evaluates grad v at its 64 lanes' points at
// once with bf16 MFMA (v_mfma_f32_32x32x16_bf16, float32 accumulation), in the
// transposed form z2^T = W2 h1^T and dh1^T = W2^T g2^T with points as matrix
// columns.  The reduction index of both products is visited in the row order
// of the MFMA accumulator layout (row = 8 (r / 4) + 4 (lane / 32) + r % 4 for
// accumulator register r), so the accumulator of the first product is, after
// the elementwise tanh step, already the B operand of the second, and its rows
// line up with the layer-1 activations that the backward step multiplies by
// 1 - h1^2: no LDS transposes.  tanh runs on the VALU.  Must be called with
// every lane of the wave active.
//
// float64 same stream: each lane evaluates the network in float64 with plain
// loops (mirrors the CPU definition to rounding).
#pragma once

#include <hip/hip_runtime.h>

#include "device_common.h"
#include "mlp.h"

namespace pdd {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(__bf16)))) __bf16 bf16x4;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;

// Network operands staged in LDS for the MFMA path.
struct NetLds {
  __bf16 W2b[MLP_W * MLP_W];    // W2 [out][in]
  __bf16 W2Tb[MLP_W * MLP_W];   // W2^T [in][out]
  float W1[2 * MLP_W], b1[MLP_W], b2[MLP_W], w3[MLP_W];
};

__device__ __forceinline__ float tanh_fast(float z) {
  const float e = __builtin_amdgcn_exp2f(z * 2.8853900817779268f);   // exp(2z)
  return 1.0f - 2.0f * __builtin_amdgcn_rcpf(e + 1.0f);
}

// Fill NetLds from the float32 parameter vector (all threads of the block).
__device__ __forceinline__ void net_stage(NetLds* N, const float* __restrict__ th) {
  for (int i = threadIdx.x; i < MLP_W * MLP_W; i += blockDim.x) {
    const int o = i / MLP_W, k = i % MLP_W;
    const float w = th[OW2 + i];
    N->W2b[i] = (__bf16)w;
    N->W2Tb[k * MLP_W + o] = (__bf16)w;
  }
  for (int i = threadIdx.x; i < 2 * MLP_W; i += blockDim.x) N->W1[i] = th[OW1 + i];
  for (int i = threadIdx.x; i < MLP_W; i += blockDim.x) {
    N->b1[i] = th[OB1 + i];
    N->b2[i] = th[OB2 + i];
    N->w3[i] = th[OW3 + i];
  }
}

__device__ __forceinline__ bf16x8 load_frag(const __bf16* row, int base) {
  // elements base .. base+3 and base+8 .. base+11 of a row
  const bf16x4 lo = *reinterpret_cast<const bf16x4*>(row + base);
  const bf16x4 hi = *reinterpret_cast<const bf16x4*>(row + base + 8);
  return bf16x8{lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
}

// grad v at every lane's (x, y); all 64 lanes must be active.  The two
// 32-point column blocks are processed one after the other to bound the live
// operand fragments.
__device__ __forceinline__ void net_grad_mfma(const NetLds* __restrict__ N, float x, float y, float& gx, float& gy) {
  const int lane = (int)(threadIdx.x & 63);
  const int g = lane >> 5, c = lane & 31;
  const float xo = __shfl_xor(x, 32, 64), yo = __shfl_xor(y, 32, 64);
  float own_x = 0.0f, own_y = 0.0f, oth_x = 0.0f, oth_y = 0.0f;
#pragma unroll 1
  for (int pb = 0; pb < 2; ++pb) {
    // the network operands are loop-invariant LDS data: keep the compiler
    // from hoisting ~200 of them into registers for the whole kernel
    __asm__ __volatile__("" ::: "memory");
    const bool mine = (pb == g);
    const float xp = mine ? x : xo, yp = mine ? y : yo;
    // layer 1: h1^T as B operands; chunk (kb, h) slot i holds k1 = 32 kb + 16 h + 8 (i / 4) + 4 g + i % 4
    bf16x8 Bf[2][2];
#pragma unroll
    for (int kb = 0; kb < 2; ++kb)
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const int k1 = 32 * kb + 16 * h + 8 * (i >> 2) + 4 * g + (i & 3);
          Bf[kb][h][i] = (__bf16)tanh_fast(N->W1[2 * k1] * xp + N->W1[2 * k1 + 1] * yp + N->b1[k1]);
          // bound the scheduler's look-ahead so operand loads are not all issued up front
          if ((i & 3) == 3) __builtin_amdgcn_sched_barrier(0);
        }
    // layer 2: z2^T tile (ob) = sum over chunks W2[out rows][chunk] h1^T[chunk][points]
    bf16x8 G2[2][2];
#pragma unroll
    for (int ob = 0; ob < 2; ++ob) {
      const __bf16* wrow = N->W2b + (32 * ob + c) * MLP_W;
      f32x16 acc = {};
#pragma unroll
      for (int kb = 0; kb < 2; ++kb)
#pragma unroll
        for (int h = 0; h < 2; ++h)
          acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(load_frag(wrow, 32 * kb + 16 * h + 4 * g), Bf[kb][h], acc, 0, 0,
                                                        0);
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int out = 32 * ob + 8 * (r >> 2) + 4 * g + (r & 3);
        const float h2 = tanh_fast(acc[r] + N->b2[out]);
        G2[ob][r >> 3][r & 7] = (__bf16)((1.0f - h2 * h2) * N->w3[out]);
        if ((r & 3) == 3) __builtin_amdgcn_sched_barrier(0);
      }
    }
    // backward: dh1^T tile (kb) = W2^T[k1 rows][chunk] g2^T[chunk][points]; chunk (ob, h)
    float px = 0.0f, py = 0.0f;
#pragma unroll
    for (int kb = 0; kb < 2; ++kb) {
      const __bf16* wrow = N->W2Tb + (32 * kb + c) * MLP_W;
      f32x16 acc = {};
#pragma unroll
      for (int ob = 0; ob < 2; ++ob)
#pragma unroll
        for (int h = 0; h < 2; ++h)
          acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(load_frag(wrow, 32 * ob + 16 * h + 4 * g), G2[ob][h], acc, 0, 0,
                                                        0);
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int k1 = 32 * kb + 8 * (r >> 2) + 4 * g + (r & 3);
        const float h1 = (float)Bf[kb][r >> 3][r & 7];
        const float d = acc[r] * (1.0f - h1 * h1);
        px += N->W1[2 * k1] * d;
        py += N->W1[2 * k1 + 1] * d;
        if ((r & 3) == 3) __builtin_amdgcn_sched_barrier(0);
      }
    }
    if (mine) { own_x = px; own_y = py; } else { oth_x = px; oth_y = py; }
  }
  // a point's k1 rows are split between lanes c and c + 32
  gx = own_x + __shfl_xor(oth_x, 32, 64);
  gy = own_y + __shfl_xor(oth_y, 32, 64);
}

// float64 grad v of one point from float32 parameters (staged in LDS).
// grad v = sum_j g2_j c_j with g2_j = (1 - h2_j^2) w3_j and
// c_j = sum_k W2[j][k] (1 - h1_k^2) W1[k]: the same sum as
// W1^T [(1 - h1^2) * (W2^T g2)] taken in another order, which keeps only h1
// live across the loop over j (64 doubles instead of 128).
__device__ __forceinline__ void net_grad_f64(const float* th, double x, double y, double& gx, double& gy) {
  double h1[MLP_W];
#pragma unroll
  for (int k = 0; k < MLP_W; ++k)
    h1[k] = tanh((double)th[OW1 + 2 * k] * x + (double)th[OW1 + 2 * k + 1] * y + (double)th[OB1 + k]);
  double ax = 0.0, ay = 0.0;
#pragma unroll 1
  for (int j = 0; j < MLP_W; ++j) {
    double z = (double)th[OB2 + j], cx = 0.0, cy = 0.0;
#pragma unroll
    for (int k = 0; k < MLP_W; ++k) {
      const double w = (double)th[OW2 + j * MLP_W + k];
      z += w * h1[k];
      const double s = w * (1.0 - h1[k] * h1[k]);
      cx += s * (double)th[OW1 + 2 * k];
      cy += s * (double)th[OW1 + 2 * k + 1];
    }
    const double h2 = tanh(z);
    const double g2 = (1.0 - h2 * h2) * (double)th[OW3 + j];
    ax += g2 * cx;
    ay += g2 * cy;
  }
  gx = ax;
  gy = ay;
}

// grad v from the node-centred float32 table [n][n][2] (bilinear; same cell
// and weight rules as the coefficient table).
__device__ __forceinline__ void grad_lut(const AsmParams& P, double x, double y, double& gx, double& gy) {
#pragma clang fp contract(off)
  const int n = P.cv_lut_n;
  double fx = (x - P.x0) / (P.x1 - P.x0) * (double)(n - 1);
  double fy = (y - P.y0) / (P.y1 - P.y0) * (double)(n - 1);
  fx = fmin(fmax(fx, 0.0), (double)(n - 1));
  fy = fmin(fmax(fy, 0.0), (double)(n - 1));
  const int i = (int)fmin(floor(fx), (double)(n - 2));
  const int j = (int)fmin(floor(fy), (double)(n - 2));
  const double tx = fx - (double)i, ty = fy - (double)j;
  const float* p00 = P.cv_lut + ((size_t)j * n + i) * 2;
  const float* p01 = p00 + (size_t)n * 2;
  double v[2];
#pragma unroll
  for (int q = 0; q < 2; ++q)
    v[q] = (1.0 - ty) * ((1.0 - tx) * (double)p00[q] + tx * (double)p00[2 + q]) +
           ty * ((1.0 - tx) * (double)p01[q] + tx * (double)p01[2 + q]);
  gx = v[0];
  gy = v[1];
}

__device__ __forceinline__ void grad_lut(const AsmParams& P, float x, float y, float& gx, float& gy) {
  const int n = P.cv_lut_n;
  float fx = fminf(fmaxf((x - (float)P.x0) * P.cv_lut_sx, 0.0f), (float)(n - 1));
  float fy = fminf(fmaxf((y - (float)P.y0) * P.cv_lut_sy, 0.0f), (float)(n - 1));
  const int i = min((int)fx, n - 2), j = min((int)fy, n - 2);
  const float tx = fx - (float)i, ty = fy - (float)j;
  const float2* row0 = reinterpret_cast<const float2*>(P.cv_lut) + (size_t)j * n + i;
  const float2* row1 = row0 + n;
  const float2 a0 = row0[0], a1 = row0[1], b0 = row1[0], b1 = row1[1];
  const float lx = a0.x + tx * (a1.x - a0.x), hx = b0.x + tx * (b1.x - b0.x);
  const float ly = a0.y + tx * (a1.y - a0.y), hy = b0.y + tx * (b1.y - b0.y);
  gx = lx + ty * (hx - lx);
  gy = ly + ty * (hy - ly);
}

}  // namespace pdd
