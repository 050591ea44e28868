// Noise generation and spectral filter, device side.
//
// * Philox-4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): the counter-based
//   generator that plays the role of the paper's R() (Section 3, Input 4 of
//   each algorithm).  Field b uses key seed+b; the block with counter
//   (q, row, tag, 0) supplies the four normals of slots 4q..4q+3 of that row.
// * Box & Muller (1958) turns the four uniforms (x + 1/2) 2^-32 into four
//   independent N(0,1) values.
// * The filter h_k = sqrt(S(p_k)/|D|) with the spectral densities of the
//   supported covariance families (Section 2: C is the Fourier transform of
//   gamma = S); its parameters arrive as a per-field record computed in
//   float64 (FieldRec, grf_common.hpp).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "grf_common.hpp"
#include "grf_fft.hpp"

namespace grf {

// One round's "hi ^ c ^ k" with the key in a scalar register: a single
// three-input VALU op (gfx950 bitop3 with the xor truth table; the compiler
// splits it into two xors otherwise).  Pure ALU.
__device__ __forceinline__ uint32_t xor3_sk(uint32_t a, uint32_t b, uint32_t k) {
  uint32_t r;
  asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x96" : "=v"(r) : "s"(k), "v"(a), "v"(b));   // 0x96 = a ^ b ^ c
  return r;
}

// UNIFORM_KEY: the key (k0, k1) is the same for every lane of the wave (one
// field per workgroup); then it lives in scalar registers.
template <bool UNIFORM_KEY = false>
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
  if constexpr (UNIFORM_KEY) {
    k0 = __builtin_amdgcn_readfirstlane(k0);
    k1 = __builtin_amdgcn_readfirstlane(k1);
  }
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    if constexpr (UNIFORM_KEY)
      c = make_uint4(xor3_sk(hi1, c.y, k0), lo1, xor3_sk(hi0, c.w, k1), lo0);
    else
      c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return c;
}

// Box-Muller on one pair of 32-bit outputs, float32 arithmetic.
// r^2 = -2 ln u is taken from the hardware log2, whose result carries the
// rounding of u to float32: an absolute error of at most 2^-24 in r^2, i.e.
// 2^-25 / r in r.  In the top 2^-13 of the interval (d = 1 - u < 2^-13,
// r < 2^-6) that would exceed 2e-6, so there the series
// -2 ln(1-d) = 2d + d^2 + 2d^3/3 (+ O(d^4) < 2^-40 relative) is used with d
// formed exactly from x read as a signed integer (d = (-x - 1/2) 2^-32).
// A wavefront takes that branch in fewer than 1% of calls.
__device__ __forceinline__ void box_muller(uint32_t xa, uint32_t xb, float& n0, float& n1) {
  const float u = fmaf((float)xa, 0x1p-32f, 0x1p-33f);
  float r2 = __builtin_amdgcn_logf(u) * -1.38629436111989061883f;   // log2(u) * (-2 ln 2)
  if (__builtin_expect(xa >= 0xFFF80000u, 0)) {
    const float d = fmaf((float)(int32_t)xa, -0x1p-32f, -0x1p-33f);
    r2 = d * fmaf(d, fmaf(d, 0.666666687f, 1.0f), 2.0f);
  }
  const float r = __builtin_amdgcn_sqrtf(r2);
  const float t = fmaf((float)xb, 0x1p-32f, 0x1p-33f);   // revolutions
  n0 = r * __builtin_amdgcn_cosf(t);
  n1 = r * __builtin_amdgcn_sinf(t);
}

// float64 version: the uniforms are exact in float64.
__device__ __forceinline__ void box_muller(uint32_t xa, uint32_t xb, double& n0, double& n1) {
  const double u = ((double)xa + 0.5) * 0x1p-32;
  const double t = ((double)xb + 0.5) * 0x1p-32;
  const double r = sqrt(-2.0 * log(u));
  double s, c;
  sincospi(2.0 * t, &s, &c);
  n0 = r * c;
  n1 = r * s;
}

template <typename T, bool UNIFORM_KEY = false>
__device__ __forceinline__ void normals4(uint32_t q, uint32_t row, uint32_t tag, uint32_t k0, uint32_t k1, T* z) {
  const uint4 x = philox4x32_10<UNIFORM_KEY>(make_uint4(q, row, tag, 0u), k0, k1);
  box_muller(x.x, x.y, z[0], z[1]);
  box_muller(x.z, x.w, z[2], z[3]);
}

// Per-field filter constants converted once to the working precision.
template <typename T> struct Filt {
  int kind;
  T c0, a, b, e;
};

template <typename T>
__device__ __forceinline__ Filt<T> load_filt(const FieldRec& r, double extra_scale) {
  Filt<T> f;
  f.kind = r.kind;
  f.c0 = (T)(r.c0 * extra_scale);
  f.a = (T)r.a;
  f.b = (T)r.b;
  f.e = (T)r.e;
  if (r.kind == COV_GAUSSIAN && sizeof(T) == 4) f.e = (T)(r.e * 1.4426950408889634);  // exp -> exp2
  return f;
}

// h at squared frequency p2 (cycles^2).
__device__ __forceinline__ float filt_h(const Filt<float>& f, float p2) {
  if (f.kind == COV_GAUSSIAN) return f.c0 * __builtin_amdgcn_exp2f(f.e * p2);
  const float u = fmaf(f.b, p2, f.a);
  return f.c0 * __builtin_amdgcn_exp2f(f.e * __builtin_amdgcn_logf(u));
}
__device__ __forceinline__ double filt_h(const Filt<double>& f, double p2) {
  if (f.kind == COV_GAUSSIAN) return f.c0 * exp(f.e * p2);
  const double u = fma(f.b, p2, f.a);
  return f.c0 * exp(f.e * log(u));
}

// wrapped frequency index kappa(k) = k (k < n/2), k - n (k >= n/2)
__device__ __forceinline__ int wrapk(int k, int n) { return (2 * k < n) ? k : k - n; }

}  // namespace grf
