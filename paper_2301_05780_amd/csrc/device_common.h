// Device helpers of the assembly kernels: the Philox4x32-10 stream, the
// uniform and Box-Muller maps, and the coefficient families of problem (6).
//
// Two numeric flavours share one code base:
//   FP64 "same stream": float64 throughout, library transcendentals, FMA
//     contraction switched off in the arithmetic that mirrors the CPU
//     definition, so results agree with it to rounding;
//   FP32 "production": float32 paths with the CDNA transcendental units
//     (v_sin/v_cos take revolutions, v_log/v_exp are base 2, v_sqrt).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

#include <type_traits>

#include "kernels.h"

namespace pdd {

constexpr double kPi = 3.141592653589793;
constexpr double kGM = 0.5825971579390106;  // -zeta(1/2)/sqrt(2 pi), Gobet-Menozzi

// ---- Philox4x32-10 (Salmon et al., SC'11) ---------------------------------
// Round: (hi0, lo0) = M0 c0, (hi1, lo1) = M1 c2 as full 64-bit products;
// c <- (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0); key bumped by the Weyl
// constants between rounds.
struct U4 { uint32_t a, b, c, d; };

__device__ __forceinline__ U4 philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                       uint32_t k0, uint32_t k1) {
  // The keys are uniform (kernel arguments).  Marking them as redefined here
  // makes each call derive its round keys with scalar adds, instead of the
  // twenty loop-invariant round keys being hoisted into scalar registers,
  // spilled, and read back with one vector lane read each per draw.
  __asm__ volatile("" : "+s"(k0), "+s"(k1));
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    // three-input XOR in one VALU op (truth table 0x96 = a ^ b ^ c)
    const uint32_t n0 = __builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), c1, k0, 0x96);
    const uint32_t n2 = __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), c3, k1, 0x96);
    c1 = (uint32_t)p1;
    c3 = (uint32_t)p0;
    c0 = n0;
    c2 = n2;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return U4{c0, c1, c2, c3};
}

// ---- uniforms ---------------------------------------------------------------
// float64: u = (r + 1/2) 2^-32, exact, in (0, 1).
__device__ __forceinline__ double uniform64(uint32_t r) {
  return ((double)r + 0.5) * 0x1p-32;
}
// float32: the top 23 bits, u = (r >> 9) 2^-23 + 2^-24 = (2 (r >> 9) + 1) 2^-24,
// exact, in (0, 1).
__device__ __forceinline__ float uniform32(uint32_t r) {
  return __builtin_fmaf((float)(r >> 9), 0x1p-23f, 0x1p-24f);
}

// ---- CDNA transcendental units (float32) ------------------------------------
// v_sin/v_cos take the angle in revolutions and accept |r| <= 256; the host
// rejects domains with a coordinate beyond 128 in absolute value, which keeps
// every argument below (at most 2 |x| revolutions) in range.
__device__ __forceinline__ float sin_rev(float r) {   // sin(2 pi r)
  return __builtin_amdgcn_sinf(r);
}
__device__ __forceinline__ float cos_rev(float r) {   // cos(2 pi r)
  return __builtin_amdgcn_cosf(r);
}
__device__ __forceinline__ float fsqrt(float v) { return __builtin_amdgcn_sqrtf(v); }
__device__ __forceinline__ float fexp(float v) { return __builtin_amdgcn_exp2f(v * 1.4426950408889634f); }
__device__ __forceinline__ float flog2(float v) { return __builtin_amdgcn_logf(v); }

// 1 / sqrt(x) for x >= c^2 > 0 in float64: the hardware estimate (relative
// error about 2^-23) refined by one Halley step for the reciprocal square
// root, y <- y (1 + e/2 + 3 e^2/8) with e = 1 - x y^2, which cubes the
// relative error (below the float64 rounding of the final step).
__device__ __forceinline__ double rsqrt_f64(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  const double e = fma(-x * y, y, 1.0);
  return fma(y * e, fma(0.375, e, 0.5), y);
}

// Box-Muller: two N(0,1) from two uniforms, rho = sqrt(-2 ln u0), theta = 2 pi u1.
__device__ __forceinline__ void box_muller(float u0, float u1, float& z0, float& z1) {
  const float rho = fsqrt(-1.3862943611198906f * flog2(u0));   // -2 ln 2 log2(u0)
  z0 = rho * cos_rev(u1);
  z1 = rho * sin_rev(u1);
}
__device__ __forceinline__ void box_muller(double u0, double u1, double& z0, double& z1) {
#pragma clang fp contract(off)
  const double rho = sqrt(-2.0 * log(u0));
  const double th = 2.0 * kPi * u1;
  z0 = rho * cos(th);
  z1 = rho * sin(th);
}

// ---- coefficients -----------------------------------------------------------
template <typename R>
struct Coef {
  R sxx, sxy, syy, dx, dy, c, f;
};

// Which terms of eq. (9) a family has (lets the step skip structural zeros;
// skipping an exact zero never changes a result).
template <int KIND> struct Traits {
  static constexpr bool drift = (KIND == PDD_COEF_VARCOEF || KIND == PDD_COEF_CONSTSOL || KIND == PDD_COEF_LUT);
  static constexpr bool reaction = drift;
  static constexpr bool offdiag = (KIND == PDD_COEF_LUT);
};

// Float32 node coordinate clamped to [0, hi] in one instruction (the median
// of v, 0 and hi; fmaxf/fminf take three with the IEEE-mode quieting of hi).
// For a finite or infinite v it is the two-sided clamp; a NaN yields 0 or
// NaN, and the index conversion turns either into node 0, so every address
// stays in the table.
__device__ __forceinline__ float clamp_node(float v, float hi) { return __builtin_amdgcn_fmed3f(v, 0.0f, hi); }

// Bilinear read of the node-centred LUT (seven fields).  Position -> node
// coordinate clamped to [0, n-1], cell index clamped to n-2.
__device__ __forceinline__ void lut_fetch(const CoefParams& cp, double x, double y, Coef<double>& o) {
#pragma clang fp contract(off)
  const int n = cp.lut_n;
  double fx = (x - cp.x0) / (cp.x1 - cp.x0) * (double)(n - 1);
  double fy = (y - cp.y0) / (cp.y1 - cp.y0) * (double)(n - 1);
  fx = fmin(fmax(fx, 0.0), (double)(n - 1));
  fy = fmin(fmax(fy, 0.0), (double)(n - 1));
  const int i = (int)fmin(floor(fx), (double)(n - 2));
  const int j = (int)fmin(floor(fy), (double)(n - 2));
  const double tx = fx - (double)i, ty = fy - (double)j;
  const float* p00 = cp.lut + ((size_t)j * n + i) * PDD_LUT_STRIDE;
  const float* p01 = p00 + (size_t)n * PDD_LUT_STRIDE;
  double v[7];
#pragma unroll
  for (int q = 0; q < 7; ++q) {
    const double v00 = p00[q], v10 = p00[PDD_LUT_STRIDE + q];
    const double v01 = p01[q], v11 = p01[PDD_LUT_STRIDE + q];
    v[q] = (1.0 - ty) * ((1.0 - tx) * v00 + tx * v10) + ty * ((1.0 - tx) * v01 + tx * v11);
  }
  o.sxx = v[0]; o.sxy = v[1]; o.syy = v[2]; o.dx = v[3]; o.dy = v[4]; o.c = v[5]; o.f = v[6];
}

__device__ __forceinline__ void lut_fetch(const CoefParams& cp, float x, float y, Coef<float>& o) {
  const int n = cp.lut_n;
  float fx = (x - cp.x0f) * cp.lut_sx;
  float fy = (y - cp.y0f) * cp.lut_sy;
  fx = clamp_node(fx, (float)(n - 1));
  fy = clamp_node(fy, (float)(n - 1));
  const int i = min((int)fx, n - 2);
  const int j = min((int)fy, n - 2);
  const float tx = fx - (float)i, ty = fy - (float)j;
  const float4* p00 = reinterpret_cast<const float4*>(cp.lut + ((size_t)j * n + i) * PDD_LUT_STRIDE);
  const float4* p01 = p00 + (size_t)n * (PDD_LUT_STRIDE / 4);
  const float4 a0 = p00[0], a1 = p00[1], b0 = p00[2], b1 = p00[3];
  const float4 c0 = p01[0], c1 = p01[1], d0 = p01[2], d1 = p01[3];
  auto bl = [&](float v00, float v10, float v01, float v11) {
    const float lo = v00 + tx * (v10 - v00);
    const float hi = v01 + tx * (v11 - v01);
    return lo + ty * (hi - lo);
  };
  o.sxx = bl(a0.x, b0.x, c0.x, d0.x);
  o.sxy = bl(a0.y, b0.y, c0.y, d0.y);
  o.syy = bl(a0.z, b0.z, c0.z, d0.z);
  o.dx = bl(a0.w, b0.w, c0.w, d0.w);
  o.dy = bl(a1.x, b1.x, c1.x, d1.x);
  o.c = bl(a1.y, b1.y, c1.y, d1.y);
  o.f = bl(a1.z, b1.z, c1.z, d1.z);
}

// The manufactured solution of the Sec. 5 experiment (eq. 43),
//   u = 3 + sin(r) / 3 + tanh(s) / 3,  r = sqrt(1 + x^2/100 + y^2/50),
//   s = sin(3x/25 + y/20) + sin(x/20 - 3y/25),
// and its Laplacian, the source of eq. 42: with T = tanh s,
//   Lap sin(r) = cos(r) Lap r - sin(r) |grad r|^2,
//   Lap r = 1/(100 r) + 1/(50 r) - (x/100)^2/r^3 - (y/50)^2/r^3,
//   Lap tanh(s) = (1 - T^2) (Lap s - 2 T |grad s|^2),  Lap s = -(9/625 + 1/400) s.
template <typename R>
__device__ __forceinline__ R eq43_u(R x, R y) {
#pragma clang fp contract(off)
  const R r = sqrt((R)1 + x * x / (R)100 + y * y / (R)50);
  const R s = sin((R)3 * x / (R)25 + y / (R)20) + sin(x / (R)20 - (R)3 * y / (R)25);
  return (R)3 + sin(r) / (R)3 + tanh(s) / (R)3;
}

template <typename R>
__device__ __forceinline__ R eq43_laplacian(R x, R y) {
#pragma clang fp contract(off)
  const R r = sqrt((R)1 + x * x / (R)100 + y * y / (R)50);
  const R rx = x / ((R)100 * r), ry = y / ((R)50 * r);
  const R lap_r = (R)1 / ((R)100 * r) + (R)1 / ((R)50 * r) - (rx * rx + ry * ry) / r;
  const R lap_a = cos(r) * lap_r - sin(r) * (rx * rx + ry * ry);
  const R al = (R)3 * x / (R)25 + y / (R)20, be = x / (R)20 - (R)3 * y / (R)25;
  const R sa = sin(al), sb = sin(be), ca = cos(al), cb = cos(be);
  const R s = sa + sb;
  const R sx = (R)3 / (R)25 * ca + cb / (R)20, sy = ca / (R)20 - (R)3 / (R)25 * cb;
  const R lap_s = -((R)9 / (R)625 + (R)1 / (R)400) * s;
  const R T = tanh(s);
  const R lap_b = ((R)1 - T * T) * (lap_s - (R)2 * T * (sx * sx + sy * sy));
  return (lap_a + lap_b) / (R)3;
}

// float32 form of the same Laplacian on the transcendental units: angles in
// revolutions, 1/r from the reciprocal square root, tanh from exp2, and
// multiplications by reciprocal constants instead of divisions.
__device__ __forceinline__ float eq43_laplacian(float x, float y) {
  constexpr float inv2pi = 0.15915494309189535f;
  const float q = 1.0f + x * x * 0.01f + y * y * 0.02f;
  const float ir = __builtin_amdgcn_rsqf(q), r = q * ir;
  const float rx = x * 0.01f * ir, ry = y * 0.02f * ir;
  const float g2 = rx * rx + ry * ry;
  const float lap_r = (0.03f - g2) * ir;
  const float lap_a = cos_rev(r * inv2pi) * lap_r - sin_rev(r * inv2pi) * g2;
  const float al = (0.12f * x + 0.05f * y) * inv2pi, be = (0.05f * x - 0.12f * y) * inv2pi;
  const float sa = sin_rev(al), sb = sin_rev(be), ca = cos_rev(al), cb = cos_rev(be);
  const float s = sa + sb;
  const float sx = 0.12f * ca + 0.05f * cb, sy = 0.05f * ca - 0.12f * cb;
  // tanh s = 1 - 2 / (e^{2s} + 1), e^{2s} = 2^{2s log2 e}; |s| <= 2 keeps it finite
  const float T = 1.0f - 2.0f * __builtin_amdgcn_rcpf(__builtin_amdgcn_exp2f(s * 2.8853900817779268f) + 1.0f);
  const float lap_b = (1.0f - T * T) * (-0.0169f * s - 2.0f * T * (sx * sx + sy * sy));
  return (lap_a + lap_b) * 0.3333333333333333f;
}

// Coefficients at (x, y).  float64 versions mirror the CPU definition's
// expression order; float32 versions use the transcendental units.
template <int KIND>
__device__ __forceinline__ void coef_at(const CoefParams& cp, double x, double y, Coef<double>& o) {
#pragma clang fp contract(off)
  if constexpr (KIND == PDD_COEF_POISSON || KIND == PDD_COEF_EXITTIME) {
    o.sxx = sqrt(2.0); o.sxy = 0.0; o.syy = sqrt(2.0);
    o.dx = 0.0; o.dy = 0.0; o.c = 0.0;
    if constexpr (KIND == PDD_COEF_POISSON)
      o.f = -2.0 * kPi * kPi * sin(kPi * x) * sin(kPi * y) + 2.0 * y;
    else
      o.f = -1.0;
  } else if constexpr (KIND == PDD_COEF_VARCOEF || KIND == PDD_COEF_CONSTSOL) {
    const double s2px = sin(2.0 * kPi * x), c2px = cos(2.0 * kPi * x);
    const double s2py = sin(2.0 * kPi * y), c2py = cos(2.0 * kPi * y);
    o.sxx = sqrt(2.0 * (1.0 + 0.5 * s2px));
    o.sxy = 0.0;
    o.syy = sqrt(2.0 * (1.0 + 0.5 * c2py));
    o.dx = s2py;
    o.dy = c2px;
    o.c = -(1.0 + x * x);
    if constexpr (KIND == PDD_COEF_VARCOEF) {
      const double ex = exp(x), c2y = cos(2.0 * y), s2y = sin(2.0 * y);
      o.f = ex * ((1.0 + 0.5 * s2px) * c2y - 4.0 * (1.0 + 0.5 * c2py) * c2y + s2py * c2y -
                  2.0 * c2px * s2y - (1.0 + x * x) * c2y);
    } else {
      o.f = -(1.0 + x * x);
    }
  } else if constexpr (KIND == PDD_COEF_EQ43) {
    o.sxx = sqrt(2.0); o.sxy = 0.0; o.syy = sqrt(2.0);
    o.dx = 0.0; o.dy = 0.0; o.c = 0.0;
    o.f = eq43_laplacian(x, y);
  } else if constexpr (KIND == PDD_COEF_AMPLITUDE) {
    const double a = cp.a;
    const double s2px = sin(2.0 * kPi * x), c2py = cos(2.0 * kPi * y);
    o.sxx = sqrt(2.0 * (1.0 + a * s2px));
    o.sxy = 0.0;
    o.syy = sqrt(2.0 * (1.0 + a * c2py));
    o.dx = 0.0; o.dy = 0.0; o.c = 0.0;
    const double ss = sin(kPi * x) * sin(kPi * y);
    o.f = (1.0 + a * s2px) * (-kPi * kPi * ss + 2.0 * y) + (1.0 + a * c2py) * (-kPi * kPi * ss);
  } else {
    lut_fetch(cp, x, y, o);
  }
}

template <int KIND>
__device__ __forceinline__ void coef_at(const CoefParams& cp, float x, float y, Coef<float>& o) {
  constexpr float kPiF = 3.14159265358979f;
  if constexpr (KIND == PDD_COEF_POISSON || KIND == PDD_COEF_EXITTIME) {
    o.sxx = 1.41421356237f; o.sxy = 0.0f; o.syy = 1.41421356237f;
    o.dx = 0.0f; o.dy = 0.0f; o.c = 0.0f;
    if constexpr (KIND == PDD_COEF_POISSON)
      o.f = -2.0f * kPiF * kPiF * sin_rev(0.5f * x) * sin_rev(0.5f * y) + 2.0f * y;
    else
      o.f = -1.0f;
  } else if constexpr (KIND == PDD_COEF_VARCOEF || KIND == PDD_COEF_CONSTSOL) {
    const float s2px = sin_rev(x), c2px = cos_rev(x);
    const float s2py = sin_rev(y), c2py = cos_rev(y);
    o.sxx = fsqrt(2.0f + s2px);
    o.sxy = 0.0f;
    o.syy = fsqrt(2.0f + c2py);
    o.dx = s2py;
    o.dy = c2px;
    o.c = -(1.0f + x * x);
    if constexpr (KIND == PDD_COEF_VARCOEF) {
      const float r = y * 0.3183098861837907f;       // 2y in revolutions
      const float ex = fexp(x), c2y = cos_rev(r), s2y = sin_rev(r);
      o.f = ex * ((1.0f + 0.5f * s2px - 4.0f - 2.0f * c2py + s2py - 1.0f - x * x) * c2y -
                  2.0f * c2px * s2y);
    } else {
      o.f = -(1.0f + x * x);
    }
  } else if constexpr (KIND == PDD_COEF_EQ43) {
    o.sxx = 1.41421356237f; o.sxy = 0.0f; o.syy = 1.41421356237f;
    o.dx = 0.0f; o.dy = 0.0f; o.c = 0.0f;
    o.f = eq43_laplacian(x, y);
  } else if constexpr (KIND == PDD_COEF_AMPLITUDE) {
    const float a = (float)cp.a;
    const float s2px = sin_rev(x), c2py = cos_rev(y);
    const float ax = 1.0f + a * s2px, ay = 1.0f + a * c2py;
    o.sxx = fsqrt(2.0f * ax);
    o.sxy = 0.0f;
    o.syy = fsqrt(2.0f * ay);
    o.dx = 0.0f; o.dy = 0.0f; o.c = 0.0f;
    const float ss = sin_rev(0.5f * x) * sin_rev(0.5f * y);
    o.f = -kPiF * kPiF * ss * (ax + ay) + 2.0f * y * ax;
  } else {
    lut_fetch(cp, x, y, o);
  }
}

// Dirichlet datum g at (x, y).
template <int KIND>
__device__ __forceinline__ double g_at(double x, double y) {
#pragma clang fp contract(off)
  if constexpr (KIND == PDD_COEF_EQ43) return eq43_u(x, y);
  else if constexpr (KIND == PDD_COEF_VARCOEF) return exp(x) * cos(2.0 * y);
  else if constexpr (KIND == PDD_COEF_CONSTSOL) return 1.0;
  else if constexpr (KIND == PDD_COEF_EXITTIME) return 0.0;
  else return sin(kPi * x) * sin(kPi * y) + x * x * y;
}
template <int KIND>
__device__ __forceinline__ float g_at(float x, float y) {
  if constexpr (KIND == PDD_COEF_EQ43) return eq43_u(x, y);
  else if constexpr (KIND == PDD_COEF_VARCOEF) return fexp(x) * cos_rev(y * 0.3183098861837907f);
  else if constexpr (KIND == PDD_COEF_CONSTSOL) return 1.0f;
  else if constexpr (KIND == PDD_COEF_EXITTIME) return 0.0f;
  else return sin_rev(0.5f * x) * sin_rev(0.5f * y) + x * x * y;
}

// ---- path step and exit rules (shared by the assembly, collection and
// point-evaluation kernels) ------------------------------------------------

// One Euler-Maruyama step of eq. (9) with coefficients frozen at the left
// point.  With the control variate (CVON), Xi gains -Y (sigma^T grad v) . dW
// (eq. 37), grad v = (gx, gy) taken at the same left point.
// The step with the coefficients at the left point already in `c`.
template <int KIND, typename R, bool CVON = false>
__device__ __forceinline__ void em_step_c(const Coef<R>& c, R h, R sq, R z0, R z1, R& x, R& y, R& Y, R& Z,
                                          R gx = 0, R gy = 0, R* Xi = nullptr) {
  using T = Traits<KIND>;
  if constexpr (std::is_same<R, double>::value) {
#pragma clang fp contract(off)
    const double dWx = sq * z0, dWy = sq * z1;
    if constexpr (CVON) {
      double Fx, Fy;
      if constexpr (T::offdiag) {
        Fx = c.sxx * gx + c.sxy * gy;
        Fy = c.sxy * gx + c.syy * gy;
      } else {
        Fx = c.sxx * gx;
        Fy = c.syy * gy;
      }
      *Xi = *Xi - Y * (Fx * dWx + Fy * dWy);
    }
    double nx = x, ny = y;
    if constexpr (T::drift) { nx = nx + c.dx * h; ny = ny + c.dy * h; }
    if constexpr (T::offdiag) {
      nx = nx + (c.sxx * dWx + c.sxy * dWy);
      ny = ny + (c.sxy * dWx + c.syy * dWy);
    } else {
      nx = nx + c.sxx * dWx;
      ny = ny + c.syy * dWy;
    }
    const double nZ = Z - c.f * Y * h;
    if constexpr (T::reaction) Y = Y * (1.0 + c.c * h);
    x = nx; y = ny; Z = nZ;
  } else {
    const float dWx = sq * z0, dWy = sq * z1;
    if constexpr (CVON) {
      float Fx, Fy;
      if constexpr (T::offdiag) {
        Fx = c.sxx * gx + c.sxy * gy;
        Fy = c.sxy * gx + c.syy * gy;
      } else {
        Fx = c.sxx * gx;
        Fy = c.syy * gy;
      }
      *Xi = *Xi - Y * (Fx * dWx + Fy * dWy);
    }
    float nx = x, ny = y;
    if constexpr (T::drift) { nx = nx + c.dx * h; ny = ny + c.dy * h; }
    if constexpr (T::offdiag) {
      nx = nx + (c.sxx * dWx + c.sxy * dWy);
      ny = ny + (c.sxy * dWx + c.syy * dWy);
    } else {
      nx = nx + c.sxx * dWx;
      ny = ny + c.syy * dWy;
    }
    const float nZ = Z - c.f * Y * h;
    if constexpr (T::reaction) Y = Y * (1.0f + c.c * h);
    x = nx; y = ny; Z = nZ;
  }
}

template <int KIND, typename R, bool CVON = false>
__device__ __forceinline__ void em_step(const CoefParams& cp, R h, R sq, R z0, R z1, R& x, R& y, R& Y, R& Z,
                                        R gx = 0, R gy = 0, R* Xi = nullptr) {
  Coef<R> c;
  coef_at<KIND>(cp, x, y, c);
  em_step_c<KIND, R, CVON>(c, h, sq, z0, z1, x, y, Y, Z, gx, gy, Xi);
}

// Exit threshold of side o for the knot in `d` (NAIVE: the side line; GM: the
// line shifted inwards by c_GM sqrt(a_nn) sqrt(h), a_nn = N^T A N evaluated on
// the side at the knot's along-line coordinate; for every analytic family a_nn
// of a vertical side depends on x only and of a horizontal side on y only).
// Returned as the strict threshold of the test that flags side o.
//
// The LUT family's a_nn varies along a side, so under GM its threshold is a
// candidate one: the shift uses a bound on a_nn over the whole table (a
// bilinear value never exceeds its largest node in magnitude, so
// sxx(P)^2 + sxy(P)^2 <= max|sxx|^2 + max|sxy|^2), widened by 1e-5 to absorb
// rounding.  Every point the exact test flags passes the candidate test; the
// exact decision, with a_nn at the projection, is lut_gm_refine's.
template <int KIND, typename R>
__device__ __forceinline__ R exit_threshold(const CoefParams& cp, int exit_rule, double sqrt_h, const KnotDesc& d,
                                            int o) {
  const double line = d.line[o];
  if (exit_rule == PDD_EXIT_NAIVE) return (R)line;
  const bool vert = (o == 0 || o == 2);
  R thr;
  if constexpr (KIND == PDD_COEF_LUT) {
    const double mxx = (double)__uint_as_float(cp.lut_max[0]);
    const double mxy = (double)__uint_as_float(cp.lut_max[1]);
    const double myy = (double)__uint_as_float(cp.lut_max[2]);
    const double bound = (vert ? mxx * mxx + mxy * mxy : mxy * mxy + myy * myy) * (1.0 + 1e-5);
    // no finite bound (a NaN in the table): every iterate becomes a candidate
    const R delta = isfinite(bound) ? (R)(kGM * sqrt(bound) * sqrt_h * (1.0 + 1e-5)) : (R)INFINITY;
    thr = (o < 2) ? (R)line - delta : (R)line + delta;
  } else {
    Coef<R> c;
    const R px = vert ? (R)line : (R)d.sx;
    const R py = vert ? (R)d.sy : (R)line;
    coef_at<KIND>(cp, px, py, c);
    {
#pragma clang fp contract(off)
      const R ann = vert ? (c.sxx * c.sxx + c.sxy * c.sxy) : (c.sxy * c.sxy + c.syy * c.syy);
      const R delta = (R)kGM * sqrt(ann) * (R)sqrt_h;
      thr = (o < 2) ? (R)line - delta : (R)line + delta;
    }
  }
  // x >= thr  <=>  x > nextafter(thr, -inf);  x <= thr  <=>  x < nextafter(thr, +inf)
  return (o < 2) ? nextafter(thr, (R)-INFINITY) : nextafter(thr, (R)INFINITY);
}

// sigma entries (sxx, sxy, syy) of the LUT at (x, y): the first three fields
// of lut_fetch, computed the same way.
__device__ __forceinline__ void lut_sigma(const CoefParams& cp, double x, double y, double& sxx, double& sxy,
                                          double& syy) {
#pragma clang fp contract(off)
  const int n = cp.lut_n;
  double fx = (x - cp.x0) / (cp.x1 - cp.x0) * (double)(n - 1);
  double fy = (y - cp.y0) / (cp.y1 - cp.y0) * (double)(n - 1);
  fx = fmin(fmax(fx, 0.0), (double)(n - 1));
  fy = fmin(fmax(fy, 0.0), (double)(n - 1));
  const int i = (int)fmin(floor(fx), (double)(n - 2));
  const int j = (int)fmin(floor(fy), (double)(n - 2));
  const double tx = fx - (double)i, ty = fy - (double)j;
  const float* p00 = cp.lut + ((size_t)j * n + i) * PDD_LUT_STRIDE;
  const float* p01 = p00 + (size_t)n * PDD_LUT_STRIDE;
  double v[3];
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    const double v00 = p00[q], v10 = p00[PDD_LUT_STRIDE + q];
    const double v01 = p01[q], v11 = p01[PDD_LUT_STRIDE + q];
    v[q] = (1.0 - ty) * ((1.0 - tx) * v00 + tx * v10) + ty * ((1.0 - tx) * v01 + tx * v11);
  }
  sxx = v[0]; sxy = v[1]; syy = v[2];
}

__device__ __forceinline__ void lut_sigma(const CoefParams& cp, float x, float y, float& sxx, float& sxy,
                                          float& syy) {
  const int n = cp.lut_n;
  float fx = (x - cp.x0f) * cp.lut_sx;
  float fy = (y - cp.y0f) * cp.lut_sy;
  fx = clamp_node(fx, (float)(n - 1));
  fy = clamp_node(fy, (float)(n - 1));
  const int i = min((int)fx, n - 2);
  const int j = min((int)fy, n - 2);
  const float tx = fx - (float)i, ty = fy - (float)j;
  const float4* p00 = reinterpret_cast<const float4*>(cp.lut + ((size_t)j * n + i) * PDD_LUT_STRIDE);
  const float4* p01 = p00 + (size_t)n * (PDD_LUT_STRIDE / 4);
  const float4 a0 = p00[0], b0 = p00[2], c0 = p01[0], d0 = p01[2];
  auto bl = [&](float v00, float v10, float v01, float v11) {
    const float lo = v00 + tx * (v10 - v00);
    const float hi = v01 + tx * (v11 - v01);
    return lo + ty * (hi - lo);
  };
  sxx = bl(a0.x, b0.x, c0.x, d0.x);
  sxy = bl(a0.y, b0.y, c0.y, d0.y);
  syy = bl(a0.z, b0.z, c0.z, d0.z);
}

// Exact Gobet-Menozzi decision for the LUT family on the candidate sides
// `cand` (bit o: side o passed the candidate test): side o is flagged iff the
// point lies on or beyond the line shifted inwards by c_GM sqrt(a_nn(P_o))
// sqrt(h), P_o the projection onto side o with its along-side coordinate
// clamped to the side.  `line` holds the lines of E, N, W, S.  Returns the
// flagged sides as a bit mask.
template <typename R>
__device__ __forceinline__ uint32_t lut_gm_refine(const CoefParams& cp, R sqrt_h, const double* line, R x, R y,
                                                  uint32_t cand) {
  const R xE = (R)line[0], yN = (R)line[1], xW = (R)line[2], yS = (R)line[3];
  uint32_t fl = 0;
  // one candidate side per pass (lowest first): a wave makes as many passes
  // as its lanes have candidates at most, almost always one
  uint32_t rest = cand;
  while (rest != 0u) {
    const int o = __builtin_ctz(rest);
    rest &= rest - 1u;
    const bool vert = (o & 1) == 0;                 // E (0) and W (2)
    const R lpos = (o == 0) ? xE : (o == 1) ? yN : (o == 2) ? xW : yS;
    const R px = vert ? lpos : fmin(fmax(x, xW), xE);
    const R py = vert ? fmin(fmax(y, yS), yN) : lpos;
    R sxx, sxy, syy;
    lut_sigma(cp, px, py, sxx, sxy, syy);
    bool hit;
    {
#pragma clang fp contract(off)
      const R ann = vert ? (sxx * sxx + sxy * sxy) : (sxy * sxy + syy * syy);
      const R delta = (R)kGM * sqrt(ann) * sqrt_h;
      const R c = vert ? x : y;
      hit = (o < 2) ? (c >= lpos - delta) : (c <= lpos + delta);
    }
    if (hit) fl |= 1u << o;
  }
  return fl;
}

// Sides flagged at (x, y) against the strict thresholds e[] of
// exit_threshold (x > e[0], y > e[1], x < e[2], y < e[3]) as a bit mask; 0
// while the point is strictly inside.  A NaN iterate flags every side, so it
// exits instead of running to the step cap.  For the LUT family under GM a
// candidate hit is decided exactly by lut_gm_refine.
template <int KIND, typename R>
__device__ __forceinline__ uint32_t exit_sides(const CoefParams& cp, int exit_rule, R sqrt_h, const double* line,
                                               const R* e, R x, R y) {
  const bool inside = (x <= e[0]) & (y <= e[1]) & (x >= e[2]) & (y >= e[3]);
  if (inside) return 0u;
  const uint32_t cand = (uint32_t)(x > e[0]) | ((uint32_t)(y > e[1]) << 1) | ((uint32_t)(x < e[2]) << 2) |
                        ((uint32_t)(y < e[3]) << 3);
  if (cand == 0) return 15u;
  if constexpr (KIND == PDD_COEF_LUT) {
    if (exit_rule == PDD_EXIT_GM) return lut_gm_refine<R>(cp, sqrt_h, line, x, y, cand);
  }
  return cand;
}

// Side chosen at an exit: among the tripped sides, the one whose grid line is
// closest to the exit iterate; ties go to the first of E, N, W, S.  `line`
// holds the physical coordinate of each side's line.
template <typename R>
__device__ __forceinline__ int choose_side(R x, R y, bool fE, bool fN, bool fW, bool fS, const double* line) {
  int o = -1;
  R best = 0;
  if (fE) { o = 0; best = fabs(x - (R)line[0]); }
  if (fN) { const R v = fabs(y - (R)line[1]); if (o < 0 || v < best) { o = 1; best = v; } }
  if (fW) { const R v = fabs(x - (R)line[2]); if (o < 0 || v < best) { o = 2; best = v; } }
  if (fS) { const R v = fabs(y - (R)line[3]); if (o < 0 || v < best) { o = 3; best = v; } }
  return o;
}

// Hat-function interpolation on an interface line: lattice coordinate t of the
// exit point clamped to [clo, chi], i0 = min(floor t, chi - 1), w = t - i0;
// lattice points i0 and i0 + 1 carry 1 - w and w.
template <typename R, bool F64>
__device__ __forceinline__ void hat_weights(R along, R a0, double d, float inv_d, int clo, int chi, int& q0, R& w) {
  R t;
  if constexpr (F64) t = (along - a0) / (R)d;
  else t = (along - a0) * (R)inv_d;
  t = fmin(fmax(t, (R)clo), (R)chi);
  const R i0 = fmin(floor(t), (R)(chi - 1));
  w = t - i0;
  q0 = (int)i0;
}

}  // namespace pdd
