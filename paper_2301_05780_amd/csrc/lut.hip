// Table-wide bounds of a coefficient look-up table, and its cell-major copy.
//
// The float32 assembly reads the table cooperatively (eight lanes fetch one
// path's cell as one 128-byte line), so it reads a copy laid out cell by
// cell: the four corners of each field contiguous, the seven fields of a cell
// in one line.
//
// The Gobet-Menozzi test of the LUT family (Sec. 2.3) shifts each side
// inwards by c_GM sqrt(a_nn(P)) sqrt(h) with a_nn taken at the projection P,
// which varies along the side.  The assembly first tests against a shift
// built from a bound on a_nn over the whole table and evaluates the exact
// shift only for the rare iterates that pass it.  These kernels produce the
// bound's ingredients, max |sxx|, |sxy|, |syy| over the table's nodes, as
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
  if ((threadIdx.x & 63) == 0) {
    atomicMax(out + 0, m0);
    atomicMax(out + 1, m1);
    atomicMax(out + 2, m2);
  }
}

// One thread per output float4: cell c = j (n-1) + i, field q, holding the
// bilinear form of the field on the cell, (v00, v10 - v00, v01 - v00,
// v11 - v10 - v01 + v00), so that v(tx, ty) = a + tx b + ty (c + tx d) is
// three fused multiply-adds.
__global__ __launch_bounds__(BLK) void k_lut_cells(const float* __restrict__ lut, int32_t n, float4* __restrict__ cells) {
  const int64_t m = n - 1;
  const int64_t total = m * m * 8;
  const int64_t stride = (int64_t)gridDim.x * BLK;
  for (int64_t t = (int64_t)blockIdx.x * BLK + threadIdx.x; t < total; t += stride) {
    const int q = (int)(t & 7);
    const int64_t c = t >> 3;
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

hipError_t launch_lut_cells(const float* lut, int32_t lut_n, float4* cells, hipStream_t stream) {
  const int64_t total = (int64_t)(lut_n - 1) * (lut_n - 1) * 8;
  const int64_t want = (total + BLK - 1) / BLK;
  const unsigned grid = (unsigned)(want < 16384 ? want : 16384);
  hipLaunchKernelGGL(k_lut_cells, dim3(grid), dim3(BLK), 0, stream, lut, lut_n, cells);
  return hipGetLastError();
}

hipError_t launch_lut_bound(const float* lut, int32_t lut_n, uint32_t* out, hipStream_t stream) {
  const int64_t nodes = (int64_t)lut_n * lut_n;
  const int64_t want = (nodes + BLK - 1) / BLK;
  const unsigned grid = (unsigned)(want < 2048 ? want : 2048);
  hipLaunchKernelGGL(k_lut_zero, dim3(1), dim3(64), 0, stream, out);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_lut_bound, dim3(grid), dim3(BLK), 0, stream, reinterpret_cast<const float4*>(lut), nodes, out);
  return hipGetLastError();
}

}  // namespace pdd
