// Workgroup-level Stockham FFT building blocks for gfx950 (wave64).
//
// The fast transform the sampler needs (Section 3: "each FFT is done in
// O(N log N)") is written here from the textbook Stockham autosort recursion:
// a length-L transform, L = R_0 R_1 ... R_{s-1}, runs s stages; stage t with
// radix R and stride Ns = R_0 ... R_{t-1} maps butterfly j (0 <= j < L/R) to
//   inputs   x[j + m L/R]                         m = 0..R-1
//   twiddle  x_m *= w^{m (j mod Ns)},  w = exp(DIR 2 pi i / (Ns R))
//   outputs  y[(j div Ns) Ns R + (j mod Ns) + m Ns] = DFT_R(x)_m
// so every stage reads with unit stride across threads and the last stage
// writes in natural order.  Data live in registers during a butterfly and in
// LDS between stages; twiddles come from a per-length table W_L[i] =
// exp(2 pi i i/L) computed in float64 on the host and rounded once.
//
// DIR = +1 is the unnormalised inverse transform (e^{+2 pi i k j / L}),
// DIR = -1 the forward one.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace grf {

// ----------------------------------------------------------------------------
// complex helpers (float2 / double2)
template <typename T> struct cvec;
template <> struct cvec<float> { using type = float2; };
template <> struct cvec<double> { using type = double2; };
template <typename T> using C = typename cvec<T>::type;

template <typename T> __device__ __forceinline__ C<T> mk(T x, T y) { C<T> r; r.x = x; r.y = y; return r; }
template <typename V> __device__ __forceinline__ V cadd(V a, V b) { a.x += b.x; a.y += b.y; return a; }
template <typename V> __device__ __forceinline__ V csub(V a, V b) { a.x -= b.x; a.y -= b.y; return a; }
// Fused multiply-add.  The library is compiled without automatic
// contraction (-ffp-contract=off): every fma is written out, so that the
// rounding of each value is fixed by the source and identical on every code
// path that computes it (plans, batches, fused launches).
__device__ __forceinline__ float fmat(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmat(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <typename V> __device__ __forceinline__ V cmul(V a, V b) {
  V r; r.x = fmat(a.x, b.x, -(a.y * b.y)); r.y = fmat(a.x, b.y, a.y * b.x); return r;
}
template <typename V> __device__ __forceinline__ V cconj(V a) { a.y = -a.y; return a; }
template <typename V, typename T> __device__ __forceinline__ V cscale(V a, T s) { a.x *= s; a.y *= s; return a; }
// multiply by DIR * i
template <int DIR, typename V> __device__ __forceinline__ V cmuli(V a) {
  V r;
  if (DIR > 0) { r.x = -a.y; r.y = a.x; } else { r.x = a.y; r.y = -a.x; }
  return r;
}
// multiply by twiddle w (DIR=+1) or conj(w) (DIR=-1)
template <int DIR, typename V> __device__ __forceinline__ V ctw(V a, V w) {
  V r;
  if (DIR > 0) { r.x = fmat(a.x, w.x, -(a.y * w.y)); r.y = fmat(a.x, w.y, a.y * w.x); }
  else         { r.x = fmat(a.x, w.x, a.y * w.y);    r.y = fmat(a.y, w.x, -(a.x * w.y)); }
  return r;
}

// ----------------------------------------------------------------------------
// compile-time cos/sin of 2 pi n / R (Taylor series, exact to ~1 ulp in float64)
constexpr double ct_pi = 3.141592653589793238462643383279502884;
constexpr double ct_sin_red(double x) {  // |x| <= pi/4
  double t = x, s = x;
  for (int k = 1; k < 14; ++k) { t *= -x * x / ((2 * k) * (2 * k + 1)); s += t; }
  return s;
}
constexpr double ct_cos_red(double x) {
  double t = 1, s = 1;
  for (int k = 1; k < 14; ++k) { t *= -x * x / ((2 * k - 1) * (2 * k)); s += t; }
  return s;
}
// cos / sin of 2 pi n / R via octant reduction on the rational n/R
constexpr double ct_cos2pi(long n, long R) {
  n %= R; if (n < 0) n += R;
  // reduce to angle in [0, 2pi): use exact symmetries on the rational
  long n8 = 8 * n;                      // octant index = floor(8n/R)
  long oct = n8 / R;
  double f = 2 * ct_pi * (double)n / (double)R;
  switch (oct) {
    case 0: return ct_cos_red(f);
    case 1: return ct_sin_red(ct_pi / 2 - f);
    case 2: return -ct_sin_red(f - ct_pi / 2);
    case 3: return -ct_cos_red(ct_pi - f);
    case 4: return -ct_cos_red(f - ct_pi);
    case 5: return -ct_sin_red(3 * ct_pi / 2 - f);
    case 6: return ct_sin_red(f - 3 * ct_pi / 2);
    default: return ct_cos_red(2 * ct_pi - f);
  }
}
// sin(2 pi n / R) = cos(2 pi (4n - R) / (4R))
constexpr double ct_sin2pi(long n, long R) { return ct_cos2pi(4 * n - R, 4 * R); }

// ----------------------------------------------------------------------------
// small DFTs in registers: y_k = sum_n x_n exp(DIR 2 pi i n k / R)
template <int R, int DIR, typename V> struct Dft;

template <int DIR, typename V> struct Dft<1, DIR, V> {
  __device__ __forceinline__ static void run(V*) {}
};
template <int DIR, typename V> struct Dft<2, DIR, V> {
  __device__ __forceinline__ static void run(V* x) {
    V a = x[0], b = x[1];
    x[0] = cadd(a, b); x[1] = csub(a, b);
  }
};
template <int DIR, typename V> struct Dft<3, DIR, V> {
  __device__ __forceinline__ static void run(V* x) {
    using T = decltype(x[0].x);
    const T c = (T)0.86602540378443864676;   // sqrt(3)/2
    V s = cadd(x[1], x[2]);
    V d = csub(x[1], x[2]);
    V y0 = cadd(x[0], s);
    V t; t.x = fmat((T)-0.5, s.x, x[0].x); t.y = fmat((T)-0.5, s.y, x[0].y);
    V u = cmuli<DIR>(cscale(d, c));
    x[0] = y0; x[1] = cadd(t, u); x[2] = csub(t, u);
  }
};
template <int DIR, typename V> struct Dft<4, DIR, V> {
  __device__ __forceinline__ static void run(V* x) {
    V a = cadd(x[0], x[2]), b = csub(x[0], x[2]);
    V c = cadd(x[1], x[3]), d = cmuli<DIR>(csub(x[1], x[3]));
    x[0] = cadd(a, c); x[2] = csub(a, c);
    x[1] = cadd(b, d); x[3] = csub(b, d);
  }
};
template <int DIR, typename V> struct Dft<5, DIR, V> {
  __device__ __forceinline__ static void run(V* x) {
    using T = decltype(x[0].x);
    const T c1 = (T)0.30901699437494742410, c2 = (T)-0.80901699437494742410;
    const T s1 = (T)0.95105651629515357212, s2 = (T)0.58778525229247312917;
    V p14 = cadd(x[1], x[4]), m14 = csub(x[1], x[4]);
    V p23 = cadd(x[2], x[3]), m23 = csub(x[2], x[3]);
    V y0 = cadd(x[0], cadd(p14, p23));
    V a1, a2, b1, b2;
    a1.x = fmat(c2, p23.x, fmat(c1, p14.x, x[0].x)); a1.y = fmat(c2, p23.y, fmat(c1, p14.y, x[0].y));
    a2.x = fmat(c1, p23.x, fmat(c2, p14.x, x[0].x)); a2.y = fmat(c1, p23.y, fmat(c2, p14.y, x[0].y));
    V t1, t2;
    t1.x = fmat(s1, m14.x, s2 * m23.x); t1.y = fmat(s1, m14.y, s2 * m23.y);
    t2.x = fmat(s2, m14.x, -(s1 * m23.x)); t2.y = fmat(s2, m14.y, -(s1 * m23.y));
    b1 = cmuli<DIR>(t1); b2 = cmuli<DIR>(t2);
    x[0] = y0; x[1] = cadd(a1, b1); x[4] = csub(a1, b1); x[2] = cadd(a2, b2); x[3] = csub(a2, b2);
  }
};

// Composite radix R = A * B in registers (Cooley-Tukey with n = n1 + A n2,
// k = B k1 + k2): B-point DFTs on the decimated subsequences, constant
// twiddles w_R^{n1 k2}, then A-point DFTs.
template <int A, int B, int DIR, typename V>
__device__ __forceinline__ void dft_composite(V* x) {
  using T = decltype(x[0].x);
  constexpr int R = A * B;
  V sub[A][B];
#pragma unroll
  for (int n1 = 0; n1 < A; ++n1) {
#pragma unroll
    for (int n2 = 0; n2 < B; ++n2) sub[n1][n2] = x[n1 + A * n2];
    Dft<B, DIR, V>::run(sub[n1]);
  }
#pragma unroll
  for (int n1 = 1; n1 < A; ++n1) {
#pragma unroll
    for (int k2 = 1; k2 < B; ++k2) {
      const int e = (n1 * k2) % R;
      if (4 * e == R) { sub[n1][k2] = cmuli<DIR>(sub[n1][k2]); }
      else if (2 * e == R) { sub[n1][k2].x = -sub[n1][k2].x; sub[n1][k2].y = -sub[n1][k2].y; }
      else if (4 * e == 3 * R) { sub[n1][k2] = cmuli<-DIR>(sub[n1][k2]); }
      else {
        V w; w.x = (T)ct_cos2pi(e, R); w.y = (T)ct_sin2pi(e, R);
        sub[n1][k2] = ctw<DIR>(sub[n1][k2], w);
      }
    }
  }
#pragma unroll
  for (int k2 = 0; k2 < B; ++k2) {
    V col[A];
#pragma unroll
    for (int n1 = 0; n1 < A; ++n1) col[n1] = sub[n1][k2];
    Dft<A, DIR, V>::run(col);
#pragma unroll
    for (int k1 = 0; k1 < A; ++k1) x[B * k1 + k2] = col[k1];
  }
}
template <int DIR, typename V> struct Dft<6, DIR, V> {
  __device__ __forceinline__ static void run(V* x) { dft_composite<2, 3, DIR>(x); }
};
template <int DIR, typename V> struct Dft<8, DIR, V> {
  __device__ __forceinline__ static void run(V* x) { dft_composite<2, 4, DIR>(x); }
};
template <int DIR, typename V> struct Dft<9, DIR, V> {
  __device__ __forceinline__ static void run(V* x) { dft_composite<3, 3, DIR>(x); }
};
template <int DIR, typename V> struct Dft<10, DIR, V> {
  __device__ __forceinline__ static void run(V* x) { dft_composite<2, 5, DIR>(x); }
};
template <int DIR, typename V> struct Dft<12, DIR, V> {
  __device__ __forceinline__ static void run(V* x) { dft_composite<4, 3, DIR>(x); }
};
template <int DIR, typename V> struct Dft<16, DIR, V> {
  __device__ __forceinline__ static void run(V* x) { dft_composite<4, 4, DIR>(x); }
};

// ----------------------------------------------------------------------------
// Compile-time factor list
template <int... Rs> struct Radices {
  static constexpr int count = sizeof...(Rs);
  static constexpr int get(int i) {
    constexpr int a[] = {Rs...};
    return a[i];
  }
  static constexpr int prod() {
    int p = 1;
    constexpr int a[] = {Rs...};
    for (int i = 0; i < (int)sizeof...(Rs); ++i) p *= a[i];
    return p;
  }
  static constexpr int ns(int i) {  // product of radices before stage i
    int p = 1;
    constexpr int a[] = {Rs...};
    for (int k = 0; k < i; ++k) p *= a[k];
    return p;
  }
};

}  // namespace grf
