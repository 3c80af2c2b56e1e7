// The fits' unconstrained coordinates psi and the map theta = T(psi), elementwise (device).
#pragma once

#include <math.h>

namespace celeste {
namespace {

// Elementwise map theta_i = t_i(psi_i): scaled logistic on boxes, exp on variances.
struct Box {
  double lo, hi;
  int kind;   // 0 identity, 1 logistic on [lo, hi], 2 exp
};

__device__ inline Box box_of(int i, const double* u0, double u_box) {
  if (i == 0 || i == 1) return {u0[i] - u_box, u0[i] + u_box, 1};
  if (i == 2 || i == 3) return {1e-4, 1.0 - 1e-4, 1};
  if (i == 4) return {0.01, 0.99, 1};
  if (i == 6) return {0.2, 15.0, 1};
  if (i == 9 || i == 10 || i >= 19) return {0.0, 0.0, 2};
  return {0.0, 0.0, 0};
}

__device__ inline double to_psi1(double th, Box b) {
  if (b.kind == 0) return th;
  if (b.kind == 2) return log(th);
  const double span = b.hi - b.lo;
  const double x = fmin(fmax(th, b.lo + 1e-9 * span), b.hi - 1e-9 * span);
  const double f = (x - b.lo) / span;
  return log(f) - log1p(-f);
}

__device__ inline double to_theta1(double psi, Box b, double* d1, double* d2) {
  if (b.kind == 0) {
    *d1 = 1.0;
    *d2 = 0.0;
    return psi;
  }
  if (b.kind == 2) {
    const double e = exp(psi);
    *d1 = e;
    *d2 = e;
    return e;
  }
  const double span = b.hi - b.lo;
  const double s = 1.0 / (1.0 + exp(-psi));
  *d1 = span * s * (1.0 - s);
  *d2 = span * s * (1.0 - s) * (1.0 - 2.0 * s);
  return b.lo + span * s;
}

}  // namespace
}  // namespace celeste
