// Host/device shared definitions: per-field covariance constants.
//
// The spectral densities (cycles convention, C(x) = int S(p) e^{-2 pi i p.x} dp,
// Section 2) of the supported families, written so that the filter
// h = sqrt(S / |D|) and the log-derivatives needed by the adjoint are cheap:
//
//   Matern (Rasmussen & Williams 2006, eq. 4.15):
//     S = sigma^2 K u^{-(nu + d/2)},  u = 2 nu / ell^2 + 4 pi^2 |p|^2,
//     K = 2^d pi^{d/2} Gamma(nu + d/2) (2 nu)^nu / (Gamma(nu) ell^{2 nu})
//     h = c0 u^e,  c0 = sigma sqrt(K / |D|),  e = -(nu + d/2)/2
//     dlogS/dsigma = 2/sigma
//     dlogS/dell   = -2 nu/ell + (nu + d/2) 4 nu / (ell^3 u)
//     dlogS/dnu    = psi(nu + d/2) - psi(nu) + ln(2 nu) + 1 - 2 ln ell - ln u
//                    - (nu + d/2)(2 / ell^2) / u
//   Exponential: the Matern case nu = 1/2 (nu is not a parameter: dnu = 0).
//   Gaussian:  S = sigma^2 (2 pi ell^2)^{d/2} exp(-2 pi^2 ell^2 |p|^2)
//     h = c0 exp(e |p|^2),  c0 = sigma (2 pi ell^2)^{d/4} / sqrt|D|,  e = -pi^2 ell^2
//     dlogS/dell = d/ell - 4 pi^2 ell |p|^2,  dnu = 0.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace grf {

enum { COV_GAUSSIAN = 0, COV_MATERN = 1, COV_EXPONENTIAL = 2 };

struct FieldRec {
  int32_t kind;
  int32_t has_nu;      // 1 if nu is a parameter (Matern)
  double sigma, ell, nu;
  double c0, a, b, e;  // filter: Matern h = c0 (a + b p2)^e ; Gaussian h = c0 exp(e p2)
  // gradient: dlogS/dsigma = gs
  //           dlogS/dell   = gl0 + gl1 * q   (q = 1/u Matern, q = p2 Gaussian)
  //           dlogS/dnu    = gn0 - ln u - gn1 / u   (Matern only)
  double gs, gl0, gl1, gn0, gn1;
};

// Digamma for x > 0: upward recurrence psi(x) = psi(x+1) - 1/x to x >= 10, then
// the asymptotic series ln x - 1/(2x) - sum B_2k / (2k x^2k) (Bernardo 1976,
// Applied Statistics algorithm AS 103, with more terms).
__host__ __device__ inline double digamma_pos(double x) {
  double acc = 0.0;
  while (x < 10.0) { acc -= 1.0 / x; x += 1.0; }
  const double r = 1.0 / (x * x);
  const double s = r * (1.0 / 12 - r * (1.0 / 120 - r * (1.0 / 252 - r * (1.0 / 240 - r * (1.0 / 132 - r * (691.0 / 32760 - r / 12.0))))));
  return acc + log(x) - 0.5 / x - s;
}

// Record of a family whose filter exists only as a table (the family of
// Section 4, eq. (5), or a tabulated density): sigma is the one parameter
// (dlogS/dsigma = 2/sigma); the filter constant is NaN, so that a pass that
// evaluated h from the record instead of the table would produce NaN.
__host__ __device__ inline void make_table_rec(double sigma, FieldRec* r) {
  r->kind = COV_GAUSSIAN;
  r->has_nu = 0;
  r->sigma = sigma;
  r->ell = 0.0;
  r->nu = 0.0;
  r->c0 = __builtin_nan("");
  r->a = r->b = r->e = 0.0;
  r->gs = 2.0 / sigma;
  r->gl0 = r->gl1 = r->gn0 = r->gn1 = 0.0;
}

// Fills a record from (kind, d, |D|, sigma, ell, nu).  Returns 0 on success,
// -1 on invalid parameters.
__host__ __device__ inline int make_field_rec(int kind, int d, double vol, double sigma, double ell,
                                              double nu, FieldRec* r) {
  const double pi = 3.141592653589793238462643383279502884;
  if (!(sigma > 0) || !(ell > 0) || !(vol > 0)) return -1;
  r->kind = kind;
  r->sigma = sigma;
  r->ell = ell;
  r->has_nu = 0;
  r->gs = 2.0 / sigma;
  if (kind == COV_GAUSSIAN) {
    r->nu = nu;
    r->c0 = sigma * pow(2 * pi * ell * ell, 0.25 * d) / sqrt(vol);
    r->a = 0.0;
    r->b = 0.0;
    r->e = -pi * pi * ell * ell;
    r->gl0 = d / ell;
    r->gl1 = -4 * pi * pi * ell;
    r->gn0 = 0.0;
    r->gn1 = 0.0;
    return 0;
  }
  if (kind == COV_EXPONENTIAL) nu = 0.5;
  else if (kind != COV_MATERN) return -1;
  if (!(nu > 0)) return -1;
  const double ad = nu + 0.5 * d;
  const double logK = d * log(2.0) + 0.5 * d * log(pi) + lgamma(ad) + nu * log(2 * nu)
                      - lgamma(nu) - 2 * nu * log(ell);
  r->nu = nu;
  r->c0 = sigma * exp(0.5 * (logK - log(vol)));
  r->a = 2 * nu / (ell * ell);
  r->b = 4 * pi * pi;
  r->e = -0.5 * ad;
  r->gl0 = -2 * nu / ell;
  r->gl1 = ad * 4 * nu / (ell * ell * ell);
  if (kind == COV_MATERN) {
    r->has_nu = 1;
    r->gn0 = digamma_pos(ad) - digamma_pos(nu) + log(2 * nu) + 1.0 - 2 * log(ell);
    r->gn1 = ad * 2.0 / (ell * ell);
  } else {
    r->gn0 = 0.0;
    r->gn1 = 0.0;
  }
  return 0;
}

}  // namespace grf
