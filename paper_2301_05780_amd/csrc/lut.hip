// Table-wide bounds of a coefficient look-up table, and its cell-major copy.
//
// The float32 assembly reads the table cooperatively (eight lanes fetch one
// path's cell as one 128-byte line), so it reads a copy laid out cell by
// cell: the four corners of each field contiguous, the seven fields of a cell
// in one line.
//
// Tables often hold fields that do not vary at all (a constant diffusion
// matrix, no drift, no reaction).  Such a field's bilinear form on every cell
// is (v, 0, 0, 0), whose value is v itself, so the copy leaves it out when at
// most two fields vary: each cell then holds only the varying fields' forms
// (16 or 32 B), read by one lane per path, and the constant fields come from
// the table's first node.  The values are the same bits the full read gives.
//
// The Gobet-Menozzi test of the LUT family (Sec. 2.3) shifts each side
// inwards by c_GM sqrt(a_nn(P)) sqrt(h) with a_nn taken at the projection P,
// which varies along the side.  The assembly first tests against a shift
// built from a bound on a_nn over the whole table and evaluates the exact
// shift only for the iterates that pass it (the float32 kernels use exact
// thresholds instead when sigma is constant).  These kernels produce the
// bound's ingredients,
// max |sxx|, |sxy|, |syy| over the table's nodes, as
// float bit patterns (non-negative floats order like their bit patterns, so
// an unsigned max is a float max).  A NaN anywhere yields a NaN-pattern
// maximum, which the threshold code treats as "no bound" (every iterate is
// then tested exactly).
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace pdd {

namespace {

constexpr int BLK = 256;

__global__ void k_lut_zero(uint32_t* out) {
  if (threadIdx.x < 4) out[threadIdx.x] = 0u;
}

__global__ __launch_bounds__(BLK) void k_lut_bound(const float4* lut, int64_t nodes, uint32_t* out) {
  uint32_t m0 = 0u, m1 = 0u, m2 = 0u;
  const int64_t stride = (int64_t)gridDim.x * BLK;
  for (int64_t i = (int64_t)blockIdx.x * BLK + threadIdx.x; i < nodes; i += stride) {
    const float4 v = lut[i * (PDD_LUT_STRIDE / 4)];      // fields sxx, sxy, syy, dx of node i
    m0 = max(m0, __float_as_uint(fabsf(v.x)));
    m1 = max(m1, __float_as_uint(fabsf(v.y)));
    m2 = max(m2, __float_as_uint(fabsf(v.z)));
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    m0 = max(m0, (uint32_t)__shfl_xor((int)m0, off, 64));
    m1 = max(m1, (uint32_t)__shfl_xor((int)m1, off, 64));
    m2 = max(m2, (uint32_t)__shfl_xor((int)m2, off, 64));
  }
  __shared__ uint32_t part[BLK / 64][3];
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    part[w][0] = m0; part[w][1] = m1; part[w][2] = m2;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 1; k < BLK / 64; ++k) {
      m0 = max(m0, part[k][0]);
      m1 = max(m1, part[k][1]);
      m2 = max(m2, part[k][2]);
    }
    atomicMax(out + 0, m0);
    atomicMax(out + 1, m1);
    atomicMax(out + 2, m2);
  }
}

// Field q counts as varying when any node's value differs from node 0's in
// its bits, or when node 0's value is not finite (an infinite constant would
// turn into NaN differences in the full copy; such fields keep the full read).
// Also keeps node 0's values + 0 (a constant field's value in the full read,
// which turns -0 into +0) in info[8 + q], and clears the sigma maxima (bmax,
// nullable) that the scan gathers for the Gobet-Menozzi bound.
__global__ void k_lut_vary_init(const float* lut, uint32_t* info, uint32_t* bmax) {
  if (bmax && threadIdx.x < 4) bmax[threadIdx.x] = 0u;
  if (threadIdx.x == 0) {
    uint32_t m = 0u;
    for (int q = 0; q < 7; ++q) {
      if (!isfinite(lut[q])) m |= 1u << q;
      info[8 + q] = __float_as_uint(lut[q] + 0.0f);
    }
    info[15] = 0u;
    info[0] = m;
    info[1] = 0u;
  }
}

// With bmax, the same pass gathers max |sxx|, |sxy|, |syy| as k_lut_bound does.
__global__ __launch_bounds__(BLK) void k_lut_vary(const float4* lut, int64_t nodes, uint32_t* info, uint32_t* bmax) {
  const float4 r0 = lut[0], r1 = lut[1];
  uint32_t m = 0u, m0 = 0u, m1 = 0u, m2 = 0u;
  const int64_t stride = (int64_t)gridDim.x * BLK;
  for (int64_t i = (int64_t)blockIdx.x * BLK + threadIdx.x; i < nodes; i += stride) {
    const float4 a = lut[2 * i], b = lut[2 * i + 1];
    m0 = max(m0, __float_as_uint(fabsf(a.x)));
    m1 = max(m1, __float_as_uint(fabsf(a.y)));
    m2 = max(m2, __float_as_uint(fabsf(a.z)));
    m |= (__float_as_uint(a.x) != __float_as_uint(r0.x) ? 1u : 0u) |
         (__float_as_uint(a.y) != __float_as_uint(r0.y) ? 2u : 0u) |
         (__float_as_uint(a.z) != __float_as_uint(r0.z) ? 4u : 0u) |
         (__float_as_uint(a.w) != __float_as_uint(r0.w) ? 8u : 0u) |
         (__float_as_uint(b.x) != __float_as_uint(r1.x) ? 16u : 0u) |
         (__float_as_uint(b.y) != __float_as_uint(r1.y) ? 32u : 0u) |
         (__float_as_uint(b.z) != __float_as_uint(r1.z) ? 64u : 0u);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    m |= (uint32_t)__shfl_xor((int)m, off, 64);
    m0 = max(m0, (uint32_t)__shfl_xor((int)m0, off, 64));
    m1 = max(m1, (uint32_t)__shfl_xor((int)m1, off, 64));
    m2 = max(m2, (uint32_t)__shfl_xor((int)m2, off, 64));
  }
  // the block's waves combine in LDS, then one thread updates the words
  // (same-address atomics from every wave serialise in the L2)
  __shared__ uint32_t part[BLK / 64][4];
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    part[w][0] = m; part[w][1] = m0; part[w][2] = m1; part[w][3] = m2;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 1; k < BLK / 64; ++k) {
      m |= part[k][0];
      m0 = max(m0, part[k][1]);
      m1 = max(m1, part[k][2]);
      m2 = max(m2, part[k][3]);
    }
    if (m) atomicOr(info, m);
    if (bmax) {
      atomicMax(bmax + 0, m0);
      atomicMax(bmax + 1, m1);
      atomicMax(bmax + 2, m2);
    }
  }
}

// One thread per output float4, holding the bilinear form of a field on a
// cell, (v00, v10 - v00, v01 - v00, v11 - v10 - v01 + v00), so that
// v(tx, ty) = a + tx b + ty (c + tx d) is three fused multiply-adds.  Full
// layout: cell c = j (n-1) + i holds the forms of fields 0..6 and a zero
// float4; lane-read layout: the forms of the varying fields k1 (, k2).
__global__ __launch_bounds__(BLK) void k_lut_cells(const float* __restrict__ lut, int32_t n, int32_t read_all,
                                                   uint32_t* info, float4* __restrict__ cells) {
  const uint32_t vm = info[0] & 0x7Fu;
  const int cnt = __popc(vm);
  uint32_t layout = 0u;
  int k1 = 6, k2 = 15, shift = 3;              // shift: log2 of the float4 per cell
  if (!read_all && cnt <= 2) {
    if (cnt >= 1) k1 = __ffs(vm) - 1;
    if (cnt == 2) k2 = 31 - __clz(vm);
    layout = LUT_LANE_READ | (uint32_t)k1 | ((uint32_t)k2 << 4) | ((uint32_t)cnt << 8);
    shift = cnt == 2 ? 1 : 0;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) info[1] = layout;
  const int64_t m = n - 1;
  const int64_t total = (m * m) << shift;
  const int64_t stride = (int64_t)gridDim.x * BLK;
  for (int64_t t = (int64_t)blockIdx.x * BLK + threadIdx.x; t < total; t += stride) {
    const int s = (int)(t & ((1 << shift) - 1));
    const int q = layout ? (s == 0 ? k1 : k2) : s;
    const int64_t c = t >> shift;
    const int64_t j = c / m, i = c - j * m;
    float4 v = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    if (q < 7) {
      const float* p00 = lut + (j * n + i) * PDD_LUT_STRIDE + q;
      const float* p01 = p00 + (int64_t)n * PDD_LUT_STRIDE;
      const float v00 = p00[0], v10 = p00[PDD_LUT_STRIDE], v01 = p01[0], v11 = p01[PDD_LUT_STRIDE];
      v = make_float4(v00, v10 - v00, v01 - v00, (v11 - v10) - (v01 - v00));
    }
    cells[t] = v;
  }
}

}  // namespace

hipError_t launch_lut_cells(const float* lut, int32_t lut_n, int32_t read_all, uint32_t* info, uint32_t* bmax,
                            float4* cells, hipStream_t stream) {
  const int64_t nodes = (int64_t)lut_n * lut_n;
  const int64_t want_v = (nodes + BLK - 1) / BLK;
  hipLaunchKernelGGL(k_lut_vary_init, dim3(1), dim3(64), 0, stream, lut, info, bmax);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_lut_vary, dim3((unsigned)(want_v < 1024 ? want_v : 1024)), dim3(BLK), 0, stream,
                     reinterpret_cast<const float4*>(lut), nodes, info, bmax);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const int64_t total = (int64_t)(lut_n - 1) * (lut_n - 1) * 8;
  const int64_t want = (total + BLK - 1) / BLK;
  const unsigned grid = (unsigned)(want < 16384 ? want : 16384);
  hipLaunchKernelGGL(k_lut_cells, dim3(grid), dim3(BLK), 0, stream, lut, lut_n, read_all, info, cells);
  return hipGetLastError();
}

hipError_t launch_lut_bound(const float* lut, int32_t lut_n, uint32_t* out, hipStream_t stream) {
  const int64_t nodes = (int64_t)lut_n * lut_n;
  const int64_t want = (nodes + BLK - 1) / BLK;
  const unsigned grid = (unsigned)(want < 1024 ? want : 1024);
  hipLaunchKernelGGL(k_lut_zero, dim3(1), dim3(64), 0, stream, out);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_lut_bound, dim3(grid), dim3(BLK), 0, stream, reinterpret_cast<const float4*>(lut), nodes, out);
  return hipGetLastError();
}

}  // namespace pdd
