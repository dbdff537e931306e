// Table-wide bounds of a coefficient look-up table.
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

}  // namespace

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
