// Device evaluation of the kernel functions of Table 1 (r = ||x - y||_2)
// and of the two test kernels, in double precision.
#pragma once

#include <hip/hip_runtime.h>

#include "tt_kernel.h"
#include "ttk_wave.h"

namespace ttk {

// z^nu K_nu(z) for z > 0, from the integral K_nu(z) = int_0^inf exp(-z cosh t)
// cosh(nu t) dt (Abramowitz & Stegun 9.6.24) by the trapezoidal rule, which
// converges exponentially for this analytic, doubly-exponentially decaying
// integrand (Trefethen & Weideman, SIAM Review 2014).  The step shrinks like
// 1/sqrt(z) because the integrand's width does; terms are summed as
// exp(nu (ln z + t) - z cosh t) (1 + exp(-2 nu t)) / 2 so that z^nu never
// overflows.  All terms are positive: no cancellation.
__device__ inline double zpow_besselk(double nu, double z) {
  const double h = fmin(0.1, 0.5 / sqrt(z));
  const double lz = log(z);
  double s = 0.5 * exp(nu * lz - z);
  const double tstar = asinh(nu / z);   // the integrand peaks at sinh t = nu / z
  for (int j = 1; j < 20000; ++j) {
    const double t = j * h;
    const double term = exp(nu * (lz + t) - z * cosh(t)) * 0.5 * (1.0 + exp(-2.0 * nu * t));
    s += term;
    if (t > tstar && term < 1e-18 * s) break;
  }
  return h * s;
}

// The same sum with the 16 lanes of a DPP row sharing it: lane l takes the
// terms j = 1 + l, 17 + l, ... (lane 0 also the half-weight j = 0 term) and
// stops by the same rule on its own partial sum, which lies within a few
// orders of the whole near the peak, so no term above 1e-18 of the sum is
// dropped; the row reduction then gives every lane the same total.  All 16
// lanes of the row must call it with the same (nu, z).  The value agrees with
// zpow_besselk to rounding; the cross evaluates every entry this way, so an
// entry it evaluates twice has one value.
__device__ inline double zpow_besselk_row16(double nu, double z, int l16) {
  const double h = fmin(0.1, 0.5 / sqrt(z));
  const double lz = log(z);
  double s = l16 == 0 ? 0.5 * exp(nu * lz - z) : 0.0;
  const double tstar = asinh(nu / z);
  for (int j = 1 + l16; j < 20000; j += 16) {
    const double t = j * h;
    const double term = exp(nu * (lz + t) - z * cosh(t)) * 0.5 * (1.0 + exp(-2.0 * nu * t));
    s += term;
    if (t > tstar && term < 1e-18 * s) break;
  }
  return h * row16_sum(s);
}

// Matern with smoothness nu and length scale ell: 2^(1-nu)/Gamma(nu) z^nu K_nu(z),
// z = sqrt(2 nu) r / ell; the r -> 0 limit is 1.  ROW16: the 16 lanes of a
// row share the Bessel sum (zpow_besselk_row16), l16 = the lane in the row.
template <bool ROW16>
__device__ inline double matern_general(double r, double ell, double nu, int l16) {
  if (r <= 0.0) return 1.0;
  const double z = sqrt(2.0 * nu) * r / ell;
  return exp2(1.0 - nu) / tgamma(nu) * (ROW16 ? zpow_besselk_row16(nu, z, l16) : zpow_besselk(nu, z));
}

// kappa(x, y; theta) for the kind in tt_kernel_kind, at the coordinates
// c = (x_1..x_d, theta_1..theta_dt, y_1..y_d).  d and dt are compile-time so
// that c stays in registers (every index below is a constant).  With dt = 0
// a kind that has parameters takes them from tf0, tf1 (fixed theta: the
// non-parametric TTK method).  The general Matern kinds (Bessel integral) are
// compiled in only when G is set, so the closed-form kinds keep a small
// register footprint.  ROW16: the call is made by all 16 lanes of a DPP row
// for one entry (the same c in every lane), which share the general Matern
// sum; l16 = the lane's index in its row.  The closed forms are evaluated by
// every lane alike.
template <int d, int dt, bool G, bool ROW16 = false>
__device__ inline double kappa_eval(int kind, double kconst, double tf0, double tf1,
                                    const double (&c)[2 * d + dt], int l16 = 0) {
  const double th0 = dt > 0 ? c[dt > 0 ? d : 0] : tf0;
  const double th1 = dt > 1 ? c[dt > 1 ? d + 1 : 0] : tf1;
  if (kind == TTK_TEST_POLY) {
    double dot = 0.0;
#pragma unroll
    for (int j = 0; j < d; ++j) dot += c[j] * c[d + dt + j];
    const double u = 1.0 + th0 * dot;
    return u * u * u;
  }
  if (kind == TTK_TEST_SEP) {
    double sx = 0.0, sy = 0.0;
#pragma unroll
    for (int j = 0; j < d; ++j) { sx += c[j]; sy += c[d + dt + j]; }
    return exp(sx) * th0 * exp(-sy);
  }
  double r2 = 0.0;
#pragma unroll
  for (int j = 0; j < d; ++j) { const double t = c[j] - c[d + dt + j]; r2 += t * t; }
  const double r = sqrt(r2);
  switch (kind) {
    case TTK_SE: { const double u = r / th0; return exp(-u * u); }
    case TTK_EXPONENTIAL: return exp(-r / th0);
    case TTK_MATERN32: { const double a = 1.7320508075688772 * r / th0; return (1.0 + a) * exp(-a); }
    case TTK_MATERN52: {
      const double a = 2.23606797749979 * r / th0;
      return (1.0 + a + a * a / 3.0) * exp(-a);
    }
    case TTK_MATERN_NU: return G ? matern_general<ROW16>(r, th0, kconst, l16) : __builtin_nan("");
    case TTK_MATERN: return G ? matern_general<ROW16>(r, th0, th1, l16) : __builtin_nan("");
    case TTK_MULTIQUADRIC: { const double u = r / th0; return sqrt(1.0 + u * u); }
    case TTK_TPS: { const double u = r2 / (th0 * th0); return u > 0.0 ? u * log(u) : 0.0; }
    case TTK_LAPLACE3D: return 1.0 / r;
    case TTK_LAPLACE2D: return -log(r);
    case TTK_BIHARMONIC: return 1.0 / r2;
    case TTK_THINPLATE: return r2 * log(r);
    default: return __builtin_nan("");
  }
}

}  // namespace ttk
