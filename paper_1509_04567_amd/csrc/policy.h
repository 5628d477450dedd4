// Decision rules of the restarted block Krylov march, written once and used by the device
// kernels and the host step control alike.  They are pure functions of a few numbers, so
// the host-only entry points of paraexp_policy.h expose them for CPU tests.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

namespace pe {

// ---- second Gram-Schmidt pass of a block Arnoldi step ------------------------------
// After the first block classical Gram-Schmidt pass, W' = W - V S1 keeps a component along
// the basis V of rounding size: |V^T w'_a| <~ c eps |w_a| for each column a, |w_a| its norm
// before the projection.  The in-block QR W' = Q1 R1 gives Q1 = W' R1^{-1}, so
//     |V^T q_b| <~ c eps sum_a |w_a| |(R1^{-1})_{ab}| = c eps rho_b,
// where the sum runs over the columns the QR kept (a deflated column is a zero column of
// Q1 with a zero row and diagonal in R1).  Column b is orthogonal enough without a second
// pass when rho_b <= 1 / kappa: its loss of orthogonality is then at most c eps / kappa.
// R1 is bw x bw upper triangular, row-major; Rn[a] = |w_a|.  z: caller storage of bw
// doubles (device code passes LDS, so no per-thread array is indexed at run time).
__host__ __device__ inline bool reorth_column_ok(const double* R, const double* Rn, int bw, int b, double kappa,
                                                 double* z) {
  const double rbb = R[b * bw + b];
  if (rbb == 0.0) return true;  // deflated: contributes no direction
  // z = R1^{-1} e_b on the kept columns, by back substitution from row b upwards
  double rho = Rn[b] * fabs(1.0 / rbb);
  z[b] = 1.0 / rbb;
  for (int a = b - 1; a >= 0; --a) {
    const double raa = R[a * bw + a];
    if (raa == 0.0) {
      z[a] = 0.0;
      continue;
    }
    double acc = 0.0;
    for (int k = a + 1; k <= b; ++k) acc += R[a * bw + k] * z[k];
    z[a] = -acc / raa;
    rho += Rn[a] * fabs(z[a]);
  }
  return rho * kappa <= 1.0;  // false as well when rho is not finite
}

// ---- step-size decision of one restart trial ---------------------------------------
// A trial evaluates the projected exponential at the squaring levels k = 0..nsq, i.e. at
// the steps alpha 2^k, and returns per level the error estimate (a residual norm of the
// Krylov approximation) and |y_k|.  The largest level whose estimate is within
//     lim_k = tol max(ref, |y_k|) / tspan
// is accepted.  Rules, in order:
//   * a non-finite estimate or |y| at level 0 (the smallest step of the trial, whose
//     Taylor argument is below 1 in norm) can only come from non-finite entries of the
//     projected matrix: the march cannot recover and stops (kStepStop);
//   * the largest passing level is accepted; an exact zero estimate with |y| > 0 at the
//     top level flags an invariant Krylov space (happy breakdown);
//   * when no level passes and the level-0 step is already at the minimum dmin, the
//     tolerance is out of reach: the march stops as well (kStepStop), rather than
//     crawling on at the minimum step;
//   * otherwise the step is reduced by a factor in [0.05, 0.5] from the error ratio at
//     level 0 and the order of a Krylov space of l steps (kStepReject).
// The local order p of the estimate (err ~ step^p) is measured from two consecutive
// levels well above rounding; it sets the growth of the next step (step_growth).
enum { kStepAccept = 0, kStepReject = 1, kStepStop = 2 };
constexpr int kFlagNotConverged = 1;
constexpr int kFlagBreakdown = 2;

struct StepIn {
  int nsq;             // levels 0..nsq evaluated
  const double* est;   // 2 (nsq + 1): est[2k] error estimate, est[2k + 1] |y_k|
  double alpha;        // step of level 0
  double tol, ref, tspan, dmin;
  int krylov_steps;
  double pexp;         // local order from earlier trials, 0 = unknown
};

struct StepOut {
  int action, level, flags;
  double step;         // accepted step, or the step of the next trial
  double rho;          // accepted estimate / its limit
  double pexp;         // updated local order
  double err;          // accepted estimate
};

inline StepOut step_decide(const StepIn& in) {
  StepOut o{};
  o.pexp = in.pexp;
  o.level = -1;
  const double e0 = in.est[0], y0 = in.est[1];
  if (!std::isfinite(e0) || !std::isfinite(y0)) {
    o.action = kStepStop;
    o.flags = kFlagNotConverged;
    return o;
  }
  int best = -1;
  double best_err = 0.0, best_lim = 1.0;
  for (int k = in.nsq; k >= 0; --k) {
    const double err = in.est[2 * k], yn = in.est[2 * k + 1];
    const double lim = in.tol * std::fmax(in.ref, yn) / in.tspan;
    if (std::isfinite(err) && std::isfinite(yn) && err <= lim) {
      best = k;
      best_err = err;
      best_lim = lim;
      break;
    }
  }
  if (best < 0 && in.alpha <= in.dmin) {
    o.action = kStepStop;
    o.flags = kFlagNotConverged;
    return o;
  }
  if (best >= 0) {
    const int ns = in.nsq;
    if (in.est[2 * ns] == 0.0 && in.est[2 * ns + 1] > 0.0) o.flags |= kFlagBreakdown;
    const int lo = best < ns ? best : best - 1;
    if (lo >= 0) {
      const double e_lo = in.est[2 * lo], e_hi = in.est[2 * (lo + 1)];
      if (std::isfinite(e_hi) && e_lo > 1e-6 * best_lim && e_hi > 2.0 * e_lo)
        o.pexp = std::fmin(40.0, std::fmax(2.0, std::log2(e_hi / e_lo)));
    }
    o.action = kStepAccept;
    o.level = best;
    o.err = best_err;
    o.rho = best_lim > 0.0 ? best_err / best_lim : 0.0;
    o.step = std::ldexp(in.alpha, best);
    return o;
  }
  const double lim0 = in.tol * std::fmax(in.ref, y0) / in.tspan;
  const double rho = e0 / lim0;
  const double ex = 1.0 / std::fmax(2.0, in.krylov_steps / 3.0);
  o.action = kStepReject;
  o.step = std::fmax(in.dmin, in.alpha * std::fmin(0.5, std::fmax(0.05, 0.9 * std::pow(rho, -ex))));
  o.rho = rho;
  return o;
}

// growth factor of the next step after an accepted one: aim at 0.95 of the limit with
// err ~ step^p, p measured (or, unknown, the order of a Krylov space of l steps)
inline double step_growth(double rho, double pexp, int krylov_steps) {
  const double ex = pexp > 0.0 ? 1.0 / pexp : 1.0 / std::fmax(2.0, krylov_steps / 3.0);
  return std::fmin(4.0, std::fmax(0.5, 0.95 * std::pow(std::fmax(rho, 1e-30), -ex)));
}

}  // namespace pe
