// Per-sample omega-bar prox of the node-level loop (Sec. 3.1), shared by the
// one-problem and the batched streaming passes.
#pragma once
#include "bca_internal.h"

namespace bca {

// Per-sample omega-bar prox (Sec. 3.1, omega-bar step): with q = M w and
// beta = rho_l / M minimise l(q; b) + (beta/2)(q - M c)^2 and return w = q / M.
// w_prev (the previous omega-bar of the sample) only seeds the Newton iteration.
__device__ __forceinline__ double prox_scalar(int loss, double c, double b, int M, double rho_l, double w_prev) {
  if (loss == BCA_LOSS_SQUARED) return (2.0 * b + rho_l * c) / (2.0 * M + rho_l);
  if (loss == BCA_LOSS_HINGE) {
    // Hinge max(0, 1 - b q), b = +-1: with s = b q and d = b M c the problem is
    // max(0, 1 - s) + (beta/2)(s - d)^2, minimised at s = d when d >= 1 (loss
    // inactive), at s = d + 1/beta when that is <= 1 (linear piece), else at the
    // kink s = 1.
    const double ib = 1.0 / (rho_l / M);  // 1 / beta
    const double d = b * M * c;
    const double s = d >= 1.0 ? d : (d + ib <= 1.0 ? d + ib : 1.0);
    return b * s / M;
  }
  // Logistic: root of -b sigmoid(-b q) + beta (q - Mc), bracketed in
  // [Mc - 1/beta, Mc + 1/beta]; Newton steps kept inside the bracket by bisection,
  // until the step is below the rounding level of the derivative, a few ulp of
  // |q| + |Mc| + 1/beta (a tolerance relative to |q| alone is unreachable when
  // |q| is much smaller than |q - Mc|).
  const double beta = rho_l / M;
  const double q0 = M * c;
  double lo = q0 - 1.0 / beta, hi = q0 + 1.0 / beta;
  double q = M * w_prev;
  if (!(q > lo && q < hi)) q = q0;
  const double tol = 4.0 * 2.220446049250313e-16 * (fabs(q0) + 1.0 / beta);
  for (int it = 0; it < 100; ++it) {
    const double sg = 1.0 / (1.0 + exp(b * q));  // sigmoid(-b q)
    const double g = -b * sg + beta * (q - q0);
    if (g == 0.0) break;
    if (g < 0.0) lo = q; else hi = q;
    const double h = sg * (1.0 - sg) + beta;
    const double step = g / h;
    const double t = tol + 4.0 * 2.220446049250313e-16 * fabs(q);
    // A converged step is taken as is: near the root q - step can round to q
    // itself (the bracket end just set), which the bracket test below would
    // misread as an overshoot and answer with bisection steps.
    if (fabs(step) <= t) {
      q -= step;
      break;
    }
    double qn = q - step;
    if (!(qn > lo && qn < hi)) qn = 0.5 * (lo + hi);
    const bool done = (hi - lo) <= t;
    q = qn;
    if (done) break;
  }
  return q / M;
}

}  // namespace bca
