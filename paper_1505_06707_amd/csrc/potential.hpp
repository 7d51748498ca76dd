// Potential and ECS-strip helpers shared by the propagation and the
// stationary solver (device code).
#pragma once
#include "cx.hpp"

namespace sofft {

// ---------------------------------------------------------------- potential phase
// exp(-i a) exp(b) for real a, b.  Small arguments (the usual case: U dt/2 of
// a few hundredths) use Taylor polynomials, which reach the FP64 rounding level
// for |a|, |b| < 0.3; larger ones go to the math library out of line.
static __device__ __noinline__ cx<double> expi_libm(double a, double b) {
  double sn, c;
  sincos(a, &sn, &c);
  const double e = exp(b);
  return {e * c, -e * sn};
}

__device__ __forceinline__ cx<double> expi(double a, double b) {
  if (!(fabs(a) < 0.3 && fabs(b) < 0.3)) return expi_libm(a, b);
  const double a2 = a * a;
  const double sn = a * (1.0 - a2 * (1.0 / 6) * (1.0 - a2 * (1.0 / 20) * (1.0 - a2 * (1.0 / 42) *
                    (1.0 - a2 * (1.0 / 72) * (1.0 - a2 * (1.0 / 110) * (1.0 - a2 * (1.0 / 156) *
                    (1.0 - a2 * (1.0 / 210))))))));
  const double c = 1.0 - a2 * 0.5 * (1.0 - a2 * (1.0 / 12) * (1.0 - a2 * (1.0 / 30) * (1.0 - a2 * (1.0 / 56) *
                   (1.0 - a2 * (1.0 / 90) * (1.0 - a2 * (1.0 / 132) * (1.0 - a2 * (1.0 / 182)))))));
  double e = 1.0;
  if (b != 0.0) {
    e = 1.0 + b * (1.0 / 15);
#pragma unroll
    for (int k = 14; k >= 1; --k) e = 1.0 + b * (1.0 / k) * e;
  }
  return {e * c, -e * sn};
}

// U = -charge/sqrt(s) + f x with s = sum z^2 + a2 (principal branch), in FP64:
// the soft-core potential on the complex contour plus the dipole term at the
// real coordinate.
__device__ __forceinline__ cx<double> potential_value(cx<double> s, double charge, double fx) {
  double ure = fx, uim = 0.0;
  if (charge != 0.0) {
    if (s.im == 0.0 && s.re > 0.0) {
      ure -= charge / sqrt(s.re);
    } else {
      // sqrt(s) = wr + i wi; -charge/sqrt(s) = -charge (wr - i wi)/|s|
      const double r = sqrt(fma(s.re, s.re, s.im * s.im));
      double wr, wi;
      if (s.re >= 0.0) {
        wr = sqrt(0.5 * (r + s.re));
        wi = 0.5 * s.im / wr;
      } else {
        wi = copysign(sqrt(0.5 * (r - s.re)), s.im);
        wr = 0.5 * s.im / wi;
      }
      const double q = charge / r;
      ure -= q * wr;
      uim += q * wi;
    }
  }
  return {ure, uim};
}

// exp(-i U dt/2) for the potential above.
__device__ __forceinline__ cx<double> potential_phase(cx<double> s, double charge, double fx, double ht) {
  const cx<double> u = potential_value(s, charge, fx);
  return expi(u.re * ht, u.im * ht);
}

__device__ __forceinline__ int strip_pos_rt(int e, int j0, int n) {
  int p = e - j0;
  return p < 0 ? p + n : p;
}

// Position of element e on the ECS strip of its axis (>= m when outside).
template <int N>
__device__ __forceinline__ int strip_pos(int e, int j0) {
  int p = e - j0;
  return p < 0 ? p + N : p;
}

}  // namespace sofft
