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

// Network operands staged in LDS for the MFMA path (bf16).
//   W1x: layer 1 as an MFMA with K = 8 used columns: for unit k,
//        (W1x_hi, W1x_hi, W1x_lo, W1y_hi, W1y_hi, W1y_lo, b1_hi, b1_lo) against the
//        point column (x_hi, x_lo, x_hi, y_hi, y_lo, y_hi, 1, 1): the hi/lo
//        bf16 splits recover W1 x + b1 to about 2^-16 relative.
//   W2b:  W2 [out][in].
//   W2Tb: W2^T [in][out] scaled by 4 w3[out] (folds the output weight and the
//         factor 4 of 1 - tanh^2 = 4 r (1 - r) into the backward product).
//   W1x, W2b and b2 carry the factor S = 2 log2(e), so that the accumulators
//   hold S z and tanh z = 1 - 2 r with r = 1 / (2^(S z) + 1).
//   Both matrices are stored with a row stride of NW = 72 elements (144 B):
//   the 32 lanes of a fragment read read 32 different rows at one column, and
//   a 128-byte stride would put every row on the same LDS banks.
//   Afin: the final contraction grad v = W1^T d as an MFMA: rows 0..3 are
//         W1x_hi, W1y_hi, W1x_lo, W1y_lo, stored per (chunk, row, half) in the
//         contraction order of the chunk.
constexpr int NW = MLP_W + 8;
constexpr float NET_S = 2.8853900817779268f;   // 2 log2(e)
struct NetLds {
  __bf16 W1x[MLP_W * 8];
  __bf16 W2b[MLP_W * NW];
  __bf16 W2Tb[MLP_W * NW];
  __bf16 Afin[4 * 4 * 2 * 8];
  float b2[MLP_W];
};

// r = 1 / (2^u + 1) for an accumulator holding u = S z: tanh z = 1 - 2 r and
// 1 - tanh^2 z = 4 r (1 - r); exact limits at +-infinity
__device__ __forceinline__ float net_r(float u) {
  return __builtin_amdgcn_rcpf(__builtin_amdgcn_exp2f(u) + 1.0f);
}

__device__ __forceinline__ void split_bf16(float v, __bf16& hi, __bf16& lo) {
  hi = (__bf16)v;
  lo = (__bf16)(v - (float)hi);
}

// unit of contraction slot i in chunk (kb, h) for lane half g: the row order
// of the 32 x 32 accumulator
__device__ __forceinline__ int chunk_unit(int kb, int h, int g, int i) {
  return 32 * kb + 16 * h + 8 * (i >> 2) + 4 * g + (i & 3);
}

// Fill NetLds from the float32 parameter vector (all threads of the block).
__device__ __forceinline__ void net_stage(NetLds* N, const float* __restrict__ th) {
  for (int i = threadIdx.x; i < MLP_W * MLP_W; i += blockDim.x) {
    const int o = i / MLP_W, k = i % MLP_W;
    const float w = th[OW2 + i];
    N->W2b[o * NW + k] = (__bf16)(NET_S * w);
    N->W2Tb[k * NW + o] = (__bf16)(4.0f * w * th[OW3 + o]);
  }
  for (int k = threadIdx.x; k < MLP_W; k += blockDim.x) {
    __bf16 xh, xl, yh, yl, bh, bl;
    split_bf16(NET_S * th[OW1 + 2 * k], xh, xl);
    split_bf16(NET_S * th[OW1 + 2 * k + 1], yh, yl);
    split_bf16(NET_S * th[OB1 + k], bh, bl);
    __bf16* r = N->W1x + 8 * k;
    r[0] = xh; r[1] = xh; r[2] = xl; r[3] = yh; r[4] = yh; r[5] = yl; r[6] = bh; r[7] = bl;
    N->b2[k] = NET_S * th[OB2 + k];
  }
  for (int e = threadIdx.x; e < 4 * 4 * 2 * 8; e += blockDim.x) {
    const int i = e & 7, g = (e >> 3) & 1, m = (e >> 4) & 3, ch = e >> 6;
    const int unit = chunk_unit(ch >> 1, ch & 1, g, i);
    __bf16 xh, xl, yh, yl;
    split_bf16(th[OW1 + 2 * unit], xh, xl);
    split_bf16(th[OW1 + 2 * unit + 1], yh, yl);
    N->Afin[e] = (m == 0) ? xh : (m == 1) ? yh : (m == 2) ? xl : yl;
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
// operand fragments.  Per block: layer 1, layer 2, the backward product and
// the final contraction are four MFMA stages; tanh and the elementwise
// factors run on the VALU.
__device__ __forceinline__ void net_grad_mfma(const NetLds* __restrict__ N, float x, float y, float& gx, float& gy) {
  const int lane = (int)(threadIdx.x & 63);
  const int g = lane >> 5, c = lane & 31;
  const float xo = __shfl_xor(x, 32, 64), yo = __shfl_xor(y, 32, 64);
  const bf16x8 zero8 = {};
  float res_x[2], res_y[2];
#pragma unroll 1
  for (int pb = 0; pb < 2; ++pb) {
    // the network operands are loop-invariant LDS data: keep the compiler
    // from hoisting them into registers for the whole kernel
    __asm__ __volatile__("" ::: "memory");
    const bool mine = (pb == g);
    const float xp = mine ? x : xo, yp = mine ? y : yo;
    // layer 1: z1^T = W1x (32 units x 16) . X (16 x 32 points); only lanes of half 0 carry the 8 used rows
    bf16x8 B1 = zero8;
    if (g == 0) {
      __bf16 xh, xl, yh, yl;
      split_bf16(xp, xh, xl);
      split_bf16(yp, yh, yl);
      const __bf16 one = (__bf16)1.0f;
      B1 = bf16x8{xh, xl, xh, yh, yl, yh, one, one};
    }
    bf16x8 Bf[2][2];
    {
      const bf16x8 A10 = (g == 0) ? *reinterpret_cast<const bf16x8*>(N->W1x + 8 * c) : zero8;
      const bf16x8 A11 = (g == 0) ? *reinterpret_cast<const bf16x8*>(N->W1x + 8 * (32 + c)) : zero8;
      const f32x16 z10 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A10, B1, f32x16{}, 0, 0, 0);
      const f32x16 z11 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A11, B1, f32x16{}, 0, 0, 0);
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        Bf[0][r >> 3][r & 7] = (__bf16)__builtin_fmaf(-2.0f, net_r(z10[r]), 1.0f);
        if ((r & 3) == 3) __builtin_amdgcn_sched_barrier(0);
      }
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        Bf[1][r >> 3][r & 7] = (__bf16)__builtin_fmaf(-2.0f, net_r(z11[r]), 1.0f);
        if ((r & 3) == 3) __builtin_amdgcn_sched_barrier(0);
      }
    }
    // layer 2: z2^T tile (ob) = b2 + W2[out rows][chunk] h1^T[chunk][points]; the two
    // output tiles' MFMA chains are interleaved, then G2/4 = r (1 - r)
    bf16x8 G2[2][2];
    {
      const __bf16* w0 = N->W2b + c * NW;
      const __bf16* w1 = N->W2b + (32 + c) * NW;
      f32x16 acc0, acc1;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        acc0[r] = N->b2[8 * (r >> 2) + 4 * g + (r & 3)];
        acc1[r] = N->b2[32 + 8 * (r >> 2) + 4 * g + (r & 3)];
      }
#pragma unroll
      for (int kb = 0; kb < 2; ++kb)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(load_frag(w0, 32 * kb + 16 * h + 4 * g), Bf[kb][h], acc0,
                                                         0, 0, 0);
          acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(load_frag(w1, 32 * kb + 16 * h + 4 * g), Bf[kb][h], acc1,
                                                         0, 0, 0);
        }
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const float q = net_r(acc0[r]);
        G2[0][r >> 3][r & 7] = (__bf16)__builtin_fmaf(-q, q, q);
        if ((r & 3) == 3) __builtin_amdgcn_sched_barrier(0);
      }
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const float q = net_r(acc1[r]);
        G2[1][r >> 3][r & 7] = (__bf16)__builtin_fmaf(-q, q, q);
        if ((r & 3) == 3) __builtin_amdgcn_sched_barrier(0);
      }
    }
    // backward: dh1^T tile (kb) = (4 W2^T w3)[k1 rows][chunk] (g2/4)^T[chunk][points], the two
    // tiles' chains interleaved; d = dh1 (1 - h1^2); then the final contraction
    f32x16 fin = f32x16{};
    {
      const __bf16* w0 = N->W2Tb + c * NW;
      const __bf16* w1 = N->W2Tb + (32 + c) * NW;
      f32x16 acc0 = f32x16{}, acc1 = f32x16{};
#pragma unroll
      for (int ob = 0; ob < 2; ++ob)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(load_frag(w0, 32 * ob + 16 * h + 4 * g), G2[ob][h], acc0,
                                                         0, 0, 0);
          acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(load_frag(w1, 32 * ob + 16 * h + 4 * g), G2[ob][h], acc1,
                                                         0, 0, 0);
        }
#pragma unroll
      for (int kb = 0; kb < 2; ++kb) {
        bf16x8 D[2];
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const float h1 = (float)Bf[kb][r >> 3][r & 7];
          D[r >> 3][r & 7] = (__bf16)((kb ? acc1[r] : acc0[r]) * (1.0f - h1 * h1));
        }
        // final contraction: rows 0..3 of W1^T (hi/lo splits) against d
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const bf16x8 Af = (c < 4) ? *reinterpret_cast<const bf16x8*>(N->Afin + (((2 * kb + h) * 4 + c) * 2 + g) * 8)
                                    : zero8;
          fin = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Af, D[h], fin, 0, 0, 0);
        }
      }
    }
    // rows 0..3 sit in registers 0..3 of the lanes of half 0
    res_x[pb] = fin[0] + fin[2];
    res_y[pb] = fin[1] + fin[3];
  }
  // block 0 holds the points of lanes 0..31, block 1 those of lanes 32..63 (in lanes 0..31)
  const float tx = __shfl_xor(res_x[1], 32, 64), ty = __shfl_xor(res_y[1], 32, 64);
  gx = g ? tx : res_x[0];
  gy = g ? ty : res_y[0];
}

// float64 grad v of one point from float32 parameters (staged in LDS), the
// parity form, in chunks of NG_J output units j so that few values
// are live: for each chunk, one pass over the hidden units k (h1_k =
// tanh(W1_k x + b1_k) recomputed per chunk) accumulates
//   z_j = b2_j + sum_k W2_jk h1_k   and   c_j = sum_k W2_jk (1 - h1_k^2) W1_k,
// then grad v += (1 - tanh(z_j)^2) w3_j c_j in j order.
constexpr int NG_J = 8;
__device__ __forceinline__ void net_grad_f64(const float* th, double x, double y, double& gx, double& gy) {
  double ax = 0.0, ay = 0.0;
#pragma unroll 1
  for (int j0 = 0; j0 < MLP_W; j0 += NG_J) {
    double z[NG_J], cx[NG_J], cy[NG_J];
#pragma unroll
    for (int jj = 0; jj < NG_J; ++jj) {
      z[jj] = (double)th[OB2 + j0 + jj];
      cx[jj] = 0.0;
      cy[jj] = 0.0;
    }
#pragma unroll 1
    for (int k = 0; k < MLP_W; ++k) {
      const double w1x = (double)th[OW1 + 2 * k], w1y = (double)th[OW1 + 2 * k + 1];
      const double h = tanh(w1x * x + w1y * y + (double)th[OB1 + k]);
      const double sk = 1.0 - h * h;
#pragma unroll
      for (int jj = 0; jj < NG_J; ++jj) {
        const double w = (double)th[OW2 + (j0 + jj) * MLP_W + k];
        z[jj] += w * h;
        const double t = w * sk;
        cx[jj] += t * w1x;
        cy[jj] += t * w1y;
      }
    }
#pragma unroll
    for (int jj = 0; jj < NG_J; ++jj) {
      const double h2 = tanh(z[jj]);
      const double g2 = (1.0 - h2 * h2) * (double)th[OW3 + j0 + jj];
      ax += g2 * cx[jj];
      ay += g2 * cy[jj];
    }
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
  const float fx = clamp_node((x - P.coef.x0f) * P.cv_lut_sx, (float)(n - 1));
  const float fy = clamp_node((y - P.coef.y0f) * P.cv_lut_sy, (float)(n - 1));
  const int i = min((int)fx, n - 2), j = min((int)fy, n - 2);
  const float tx = fx - (float)i, ty = fy - (float)j;
  // 32-bit byte offsets from the table's base (the host keeps float32 runs'
  // tables below 4 GiB, lut_n <= 23170), so the loads take the base from
  // scalar registers
  // (nodes i and i + 1 of a row are 16 contiguous bytes, 8-byte aligned)
  struct __attribute__((aligned(8))) Pair { float2 lo, hi; };
  const char* base = reinterpret_cast<const char*>(P.cv_lut);
  const uint32_t o0 = (__umul24((uint32_t)j, (uint32_t)n) + (uint32_t)i) * 8u;
  const Pair r0 = *reinterpret_cast<const Pair*>(base + o0);
  const Pair r1 = *reinterpret_cast<const Pair*>(base + (o0 + (uint32_t)n * 8u));
  const float2 a0 = r0.lo, a1 = r0.hi, b0 = r1.lo, b1 = r1.hi;
  const float lx = a0.x + tx * (a1.x - a0.x), hx = b0.x + tx * (b1.x - b0.x);
  const float ly = a0.y + tx * (a1.y - a0.y), hy = b0.y + tx * (b1.y - b0.y);
  gx = lx + ty * (hx - lx);
  gy = ly + ty * (hy - ly);
}

}  // namespace pdd
