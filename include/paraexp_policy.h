/*
 * paraexp_policy.h -- host-only entry points of the step-size and reorthogonalisation
 * rules of the gfx950 Paraexp library (libparaexp.so).
 *
 * The restarted block Krylov march of Sec. 2.1 (eq. 2.4 with time sub-steps; the paper
 * restarts its block Krylov process and leaves the stopping test to the EBK method it
 * builds on) takes two decisions that do not depend on the data layout: how large a
 * sub-step a trial of the projected exponential may take, and whether a block Arnoldi
 * step needs a second Gram-Schmidt pass.  The library makes them with the functions
 * below -- the same code that runs in the march (host) and in the update kernel
 * (device).  They are exported so that tests can drive them on the CPU with synthetic
 * inputs.  Pure functions: no context, no device, no allocation; all pointers are host
 * pointers owned by the caller; they never fail (invalid sizes give the documented
 * neutral result).
 */
#ifndef PARAEXP_POLICY_H
#define PARAEXP_POLICY_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Input of one step-size trial: the projected exponential was evaluated at the squaring
 * levels k = 0..nsq, i.e. at the steps alpha 2^k.
 *   est   host, 2 (nsq + 1) doubles: est[2k] = error estimate at level k (a residual norm
 *         of the Krylov approximation), est[2k + 1] = |y_k| (norm of the projected state)
 *   tol, ref, tspan   the limit at level k is tol max(ref, |y_k|) / tspan
 *   dmin  smallest step the march may take
 *   krylov_steps      block steps per restart cycle (order of the step-reduction rule)
 *   pexp  local order of the estimate measured by earlier trials, 0 = unknown */
typedef struct {
  int32_t nsq;
  const double* est;
  double alpha, tol, ref, tspan, dmin;
  int32_t krylov_steps;
  double pexp;
} pe_step_trial;

enum { PE_STEP_ACCEPT = 0, PE_STEP_REJECT = 1, PE_STEP_STOP = 2 };

/* Result: action PE_STEP_ACCEPT (level = the accepted level, step = alpha 2^level, rho =
 * estimate / limit there), PE_STEP_REJECT (step = the next trial's step) or PE_STEP_STOP
 * (the march of this problem ends: a non-finite estimate or |y| at level 0, or no level
 * within the limit at the minimum step; flags carries PE_FLAG_NOT_CONVERGED).  flags may
 * also carry PE_FLAG_BREAKDOWN (exact zero estimate at the top level).  pexp is the
 * updated local order. */
typedef struct {
  int32_t action, level, flags;
  double step, rho, pexp, err;
} pe_step_decision;

/* Decide one trial.  A null t or out does nothing. */
void pe_policy_step(const pe_step_trial* t, pe_step_decision* out);

/* Growth factor of the next step after an accepted one, in [0.5, 4]: aims at 0.95 of the
 * limit with err ~ step^p (p = pexp, or krylov_steps / 3 when pexp = 0). */
double pe_policy_step_growth(double rho, double pexp, int32_t krylov_steps);

/* Second Gram-Schmidt pass of a block Arnoldi step.  R: host, bw x bw upper triangular,
 * row-major -- the triangular factor of the block after the first projection (a zero
 * diagonal marks a deflated column); Rn: host, bw norms of the block's columns before the
 * projection.  Returns 1 when every column b satisfies kappa sum_a Rn[a] |(R^{-1})_{ab}|
 * <= 1 over the kept columns a (the first pass alone leaves the new basis block
 * orthogonal to the old basis to ~eps / kappa), else 0.  bw outside [1, 32] gives 0. */
int32_t pe_policy_reorth_skip(const double* R, const double* Rn, int32_t bw, double kappa);

#ifdef __cplusplus
}
#endif

#endif /* PARAEXP_POLICY_H */
