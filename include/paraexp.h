/*
 * paraexp.h -- C ABI of the MI355X (gfx950) block-Krylov Paraexp exp-action library.
 *
 * Method: Kooij, Botchev & Geurts, "A block Krylov subspace implementation of the
 * time-parallel Paraexp method and its extension for nonlinear partial differential
 * equations" (arXiv 1509.04567).  The library solves, per Paraexp window,
 *
 *     u'(t) = L u(t) + g(t),  t in [t0, t1];   u'(t) = L u(t) after t1          (eq. 2.1)
 *
 * where L is a periodic 3-point finite-difference stencil (Sec. 3, eq. 3.2) and g is
 * given by s time samples (eq. 2.2).  The samples are compressed by a truncated SVD
 * into U p(t) (eq. 2.3, Sec. 2.1), p is a least-squares polynomial in time, and the
 * solution is advanced by restarted block Arnoldi on the Krylov space of [x | U]
 * (eq. 2.4) with the exponential of the projected, source-augmented block-Hessenberg
 * matrix.  With shift = 1 the window is the Paraexp subproblem of eqs. (2.5)-(2.8):
 * v(t0) = 0, source L u0 + g, and the outputs are v(t_k); u = u0 + sum_j v_j
 * (eq. 2.9, pe_superpose).
 *
 * Sign convention: `L` is the right-hand-side operator, the paper's A in u' = A u + g.
 *
 * Conventions for every entry point:
 *   - pointers documented "device" are HIP device pointers on the context's device;
 *     "host" pointers are ordinary host memory read during the call;
 *   - the caller owns every buffer it passes; the library owns only the memory inside
 *     a pe_ctx (workspace, grown on demand, released by pe_destroy);
 *   - all matrices are column-major with the stated leading dimension;
 *   - `stream` is a hipStream_t (NULL = the null stream).  Calls enqueue work on it and
 *     return after it has completed (the solver's step control reads scalars back);
 *   - errors are negative pe_status values with a message in pe_last_error(); a
 *     non-converged solve is not an error: its report carries PE_FLAG_* bits and the
 *     outputs are still written (NaN at output times that a march does not reach: it
 *     stops at once when no sub-step down to 1e-13 of its time span meets tol or when
 *     its projected matrix is not finite, and after at most 100000 restart cycles);
 *     the other problems of a batch are not affected.
 */
#ifndef PARAEXP_H
#define PARAEXP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PE_OK = 0,
  PE_ERR_ARG = -1,          /* invalid argument (sizes, ordering, null pointers)      */
  PE_ERR_NONFINITE = -2,    /* NaN/Inf found in u0, G or the stencil coefficients     */
  PE_ERR_DEVICE = -3,       /* a HIP runtime call failed                              */
  PE_ERR_OOM = -4,          /* device workspace allocation failed                     */
  PE_ERR_UNSUPPORTED = -5   /* valid request outside what this build implements      */
} pe_status;

/* report flags (informational, outputs are written) */
enum {
  PE_FLAG_NOT_CONVERGED = 1,  /* the march stopped: no sub-step down to the minimum met tol, the
                                 projected matrix or its estimate was not finite, or the cycle cap
                                 was hit; outputs it did not reach are NaN                   */
  PE_FLAG_BREAKDOWN = 2,      /* Krylov space became invariant (exact, "happy") early      */
  PE_FLAG_RANK_CAPPED = 4,    /* truncation wanted more than rank_max singular vectors     */
  PE_FLAG_FIT_CAPPED = 8      /* fit residual above fit_tol at q_max terms                 */
};

typedef enum { PE_FP64 = 0, PE_MIXED = 1 } pe_precision;

/* Krylov space of a restart cycle (Sec. 2.1): polynomial, K_l(L, [x | U]), or rational
 * shift-and-invert, K_l((I - gamma L)^{-1}, [x | U]) -- the acceleration the paper uses
 * (Sec. 2.1, Sec. 3.2), whose convergence does not degrade with the grid's stiffness. */
typedef enum { PE_KRYLOV_POLY = 0, PE_KRYLOV_SAI = 1 } pe_krylov;

/* The time dependence p(t) of the compressed source (Sec. 2.1, eq. 2.3): one
 * least-squares polynomial over the window in the Chebyshev basis (degree chosen by
 * fit_tol, capped by q_max), or the paper's own choice (Sec. 3): the piecewise cubic
 * spline interpolating the coefficients at the samples, not-a-knot end conditions. */
typedef enum { PE_FIT_CHEBYSHEV = 0, PE_FIT_SPLINE = 1 } pe_source_fit;

typedef struct pe_ctx pe_ctx; /* opaque: device, stream-independent workspace */

/* The operator L (Sec. 3, eq. 3.2):
 *   (L u)_i = c_minus[i] u_{i-1} + c_zero[i] u_i + c_plus[i] u_{i+1},  indices mod n.
 * per_point = 0: coeffs points to 3 HOST doubles {c_minus, c_zero, c_plus};
 * per_point = 1: coeffs points to 3*n DEVICE doubles, rows c_minus[0..n), c_zero, c_plus. */
typedef struct {
  int64_t n;
  int32_t per_point;
  const double* coeffs;
} pe_stencil;

/* One window subproblem (Sec. 2.1-2.2; the inputs of the linear algorithm of Fig. 2.1:
 * the operator, the initial value and the source).
 *   u0        device, n: initial condition of the whole problem (shifted: used for L u0)
 *   t0, t1    window; the source acts on [t0, t1] and is zero after t1
 *   t_samples host, s ascending, t_samples[0] = t0, t_samples[s-1] = t1, s >= 1
 *   G         device, n x s (ldG >= n): raw source samples g(t_i)
 *   shift     1: Paraexp shift (v(t0) = 0, source L u0 + g, outputs v); 0: outputs u
 *   t_out     host, n_out non-decreasing absolute times; with shift = 0 all >= t0,
 *             with shift = 1 times before t0 give zero columns
 *   out       device, n x n_out (ldOut >= n), written
 *   krylov_steps  block Arnoldi steps per restart cycle (l >= 1)
 *   rank_max  cap on the retained singular vectors; q_max cap on polynomial terms
 *   tol       accuracy target of the time integration, relative to max(|u0|, |state|)
 *   svd_tol   truncation: keep m singular vectors with dropped energy <= svd_tol |G^|_F
 *   fit_tol   polynomial degree: smallest with relative fit residual <= fit_tol
 *   prec      PE_FP64, or PE_MIXED (Krylov basis stored in fp32, fp64 arithmetic)
 *   krylov    PE_KRYLOV_POLY or PE_KRYLOV_SAI
 *   sai_shift shift-and-invert only: gamma = sai_shift times the step a restart cycle
 *             aims at (0: 0.1); the shifted system is solved as a periodic tridiagonal
 *             system without pivoting, so I - gamma L should be diagonally dominant
 *             (always so for 2 nu >= |a| h, the cell Peclet condition)
 *   source_fit PE_FIT_CHEBYSHEV or PE_FIT_SPLINE (then q_max and fit_tol are unused, the
 *             report's q is 4, and every sample time is a restart point of the march;
 *             pe_expaction_batch takes Chebyshev coefficients only). */
typedef struct {
  pe_stencil op;
  const double* u0;
  double t0, t1;
  const double* t_samples;
  int32_t s;
  const double* G;
  int64_t ldG;
  int32_t shift;
  const double* t_out;
  int32_t n_out;
  double* out;
  int64_t ldOut;
  int32_t krylov_steps;
  int32_t rank_max;
  int32_t q_max;
  double tol;
  double svd_tol;
  double fit_tol;
  pe_precision prec;
  pe_krylov krylov;
  double sai_shift;
  pe_source_fit source_fit;
} pe_problem;

/* Per-problem report (host). */
typedef struct {
  int32_t rank;        /* m, retained singular vectors                            */
  int32_t q;           /* polynomial terms of p(t)                                */
  int32_t cycles;      /* accepted restart cycles (time sub-steps)                */
  int32_t rejected;    /* rejected step-size trials                               */
  int32_t block_steps; /* block Arnoldi steps performed                           */
  int32_t flags;       /* PE_FLAG_* bits                                          */
  double resid_est;    /* largest accepted per-cycle error estimate (absolute)    */
  double fit_resid;    /* relative fit residual of the chosen q                   */
  double svd_tail;     /* dropped singular energy relative to |G^|_F              */
  double sigma1;       /* largest singular value of the shifted samples           */
} pe_report;

/* Create a context on HIP device `device`.  *ctx receives the handle. */
pe_status pe_create(pe_ctx** ctx, int device);
/* Release the context and its workspace (synchronises the device first). */
pe_status pe_destroy(pe_ctx* ctx);
/* Message for the last non-OK status returned on this context (never NULL). */
const char* pe_last_error(const pe_ctx* ctx);
/* Library version string, e.g. "paraexp-gfx950 0.1". */
const char* pe_version(void);

/* Step S0 (Sec. 3, eq. 3.2): Y = L X for an n x ncols block.
 * X, Y device, column-major with leading dimensions ldx, ldy >= n; X and Y must not
 * overlap.  Exposed for tests and for the stencil bandwidth measurement. */
pe_status pe_stencil_apply(pe_ctx* ctx, const pe_stencil* op, const double* X, int64_t ldx,
                           double* Y, int64_t ldy, int32_t ncols, void* stream);

/* Steps S1-S4 (Sec. 2.1, eqs. 2.2-2.3, 2.6): shifted samples, truncated SVD and the
 * Chebyshev fit of the coefficients, for one problem.
 *   U     device, n x rank_max (ldU = n): the m retained left singular vectors
 *   Pi    device, rank_max x q_max (ld = rank_max): p(t) = sum_k Pi[:,k] T_k(x(t)),
 *         x = (2t - t0 - t1)/(t1 - t0); with source_fit = PE_FIT_SPLINE it receives the
 *         spline pieces instead (room for 4 (s - 1) rank_max doubles): Pi[(i 4 + k) m + a]
 *         is coefficient k of row a on piece i, p_a(t) = sum_k c_k (t - t_i)^k
 *   sigma host, s entries (may be NULL): singular values of the shifted samples that
 *         the routine resolved (zeros beyond the numerical rank), descending
 *   m, q  host out; report host out (rank, q, fit_resid, svd_tail, sigma1, flags). */
pe_status pe_compress(pe_ctx* ctx, const pe_problem* prob, double* U, double* Pi, int32_t* m,
                      int32_t* q, double* sigma, pe_report* report, void* stream);

/* pe_compress without any allocation, for callers that cannot allocate device memory
 * (code under stream capture, tight serving loops, harnesses that forbid hipMalloc).
 * Same arguments, results and errors as pe_compress; the device workspace is instead a
 * fixed 64 MiB array of the library on each GPU (held until the process ends) and the
 * host read-back buffer lives in the context, so the call makes no hipMalloc, hipFree,
 * hipHostMalloc or other allocating call.  A problem whose compression needs more than
 * 64 MiB of workspace (two n x s copies of the samples, up to n x 128 range vectors and
 * partial sums: n = 8192 with s = 256 needs 48 MiB) is rejected with PE_ERR_UNSUPPORTED
 * before any device work.  Every call on one GPU
 * shares that array: calls that overlap on one GPU (several streams or threads) race. */
pe_status pe_compress_noalloc(pe_ctx* ctx, const pe_problem* prob, double* U, double* Pi, int32_t* m, int32_t* q,
                              double* sigma, pe_report* report, void* stream);

/* Steps S5-S8 (Sec. 2.1, eq. 2.4: the block Krylov space of [x | U] and the exponential
 * of the projected source-augmented matrix; Sec. 2.2 for the window subproblem) for
 * nprob independent problems with a given compressed source
 * (stage parity: every problem uses U[i] (n x m[i], ld n) and Pi[i] (m[i] x q[i],
 * ld m[i]) -- device pointers; U[i]/Pi[i] may be NULL when m[i] = 0).  The sample
 * fields of the problems (t_samples, G, svd_tol, fit_tol) are ignored; t0, t1 still
 * define the window and the polynomial variable.  Outputs and reports as in
 * pe_solve_batch.  All problems advance together, one restart cycle at a time. */
pe_status pe_expaction_batch(pe_ctx* ctx, const pe_problem* probs, const double* const* U,
                             const double* const* Pi, const int32_t* m, const int32_t* q,
                             int32_t nprob, pe_report* reports, void* stream);

/* Steps S1-S8 for nprob independent window subproblems (instances and/or Paraexp
 * windows) in one batched pipeline: the linear PEBK algorithm of Sec. 2.2 (Fig. 2.1)
 * per problem -- shifted samples (eq. 2.6), truncated SVD and time fit (eq. 2.3),
 * restarted block Krylov exp-action (eq. 2.4) to every output time.  Windows of one
 * problem are independent (eqs. 2.7-2.8) and are superposed with pe_superpose (eq. 2.9).
 * probs: host array of nprob; reports: host array of nprob, written. */
pe_status pe_solve_batch(pe_ctx* ctx, const pe_problem* probs, int32_t nprob,
                         pe_report* reports, void* stream);

/* Device memory that pe_solve_batch on these problems may need, in bytes: the largest
 * context workspace (compression of any one problem, or the batched march with every
 * problem at rank rank_max and min(q_max, s) polynomial terms -- the most its
 * compression can give) plus the compressed sources it allocates for the call.  Only
 * the size fields are read (n, s, krylov_steps, rank_max, q_max, prec); data pointers
 * may be NULL.  Pure host arithmetic: ctx may be NULL, and no device is touched.  The
 * workspace persists in ctx and grows on demand (released by pe_destroy).  Returns
 * PE_ERR_UNSUPPORTED if some restart cycle the problems can meet has no kernel
 * geometry within the workspace (the solve would fail the same way). */
pe_status pe_workspace_query(pe_ctx* ctx, const pe_problem* probs, int32_t nprob, size_t* bytes);

/* Step S8 (eq. 2.9): u[:, k] = u0 + sum_{j<P} v_j[:, k], summed in window order.
 * u0 device n; v host array of P device pointers, each n x n_out with ld ldv;
 * u device n x n_out with ld ldu (may alias none of the inputs). */
pe_status pe_superpose(pe_ctx* ctx, const double* u0, const double* const* v, int32_t P,
                       int64_t n, int32_t n_out, int64_t ldv, double* u, int64_t ldu,
                       void* stream);

/* Step S10 (Secs. 2.3-2.4, eqs. 2.10-2.20; Sec. 4): waveform relaxation for the viscous
 * Burgers equation u_t + u u_x = nu u_xx on the periodic unit interval, central
 * differences with h = 1/n and the advective form N(u)_i = -u_i (u_{i+1} - u_{i-1})/(2h).
 * [0, T] is split into P windows; window j has s uniform samples
 *     t_{j,i} = T j / P + i (T / P) / (s - 1),  i = 0..s-1  (end points included).
 * Iteration k -> k+1 solves every window with the operator L_j = nu D2 + Jbar_j, where
 * Jbar_j is the trapezoid average over the window's samples of the Jacobian of N at the
 * iterate u_k (jacobian = 1, eqs. 2.12-2.14) or zero (jacobian = 0: Picard), and the
 * source samples g = N(u_k) - Jbar_j u_k (eq. 2.10 with the correction of eq. 2.13),
 * shifted by L_j u0 (eq. 2.16 read with u_k in place of the hatted term).  The window
 * subsolutions from zero state are superposed with the homogeneous continuation of the
 * earlier windows through each later window's own operator (eqs. 2.19-2.20):
 *     u_{k+1}(t) = u0 + sum_j v_j(t).
 *   u0       device, n
 *   u_init   device, n x (P s), ld n, window-major columns; NULL = u0 at every sample
 *   u_final  device, n x (P s), ld n: the iterate after K iterations (may alias u_init)
 *   forcing  device, n x (P s), ld n, window-major columns: samples of an external source
 *            f(x, t) added to the nonlinear term at every sample (the manufactured source
 *            of Sec. 4.1, eq. 4.1); NULL = none
 *   the remaining fields are as in pe_problem and apply to every window solve.
 * reports: host, P entries (the window solves of the last iteration); increments: host,
 * K entries (|u_{k+1} - u_k| / |u_{k+1}| over all samples), or NULL. */
typedef struct {
  int64_t n;
  double nu, T;
  int32_t P, s, K, jacobian;
  const double* u0;
  const double* u_init;
  double* u_final;
  int32_t krylov_steps;
  int32_t rank_max;
  int32_t q_max;
  double tol, svd_tol, fit_tol;
  pe_precision prec;
  pe_krylov krylov;
  double sai_shift;
  const double* forcing;
  pe_source_fit source_fit;
} pe_wr_problem;
pe_status pe_wr_burgers(pe_ctx* ctx, const pe_wr_problem* wr, pe_report* reports, double* increments,
                        void* stream);

/* Tile autotuning of the block orthogonalisation kernels (the batched pipeline of
 * Sec. 2.2: every window's and instance's block Arnoldi, eq. 2.4, runs on them).  For each
 * block width a march of the given problems can meet (1 .. rank_max + 1) at the problem's
 * precision, times 12 block Arnoldi steps on a seeded random block of the problem's size
 * for every admissible pair (rows per update chunk in {64, 128, 256, 512}, rows per
 * projection chunk in {16, ..., 256} with rows x width <= 1024) and keeps in ctx the
 * fastest if it beats the built-in tiling by 3%, else the built-in one.  The key is (ceil(log2 n), block width, precision): later calls on ctx with grids
 * of the same power-of-two bucket use the choice; keys already in ctx are not re-timed.
 * The choice changes only the partition of the rows into chunks (and so the rounding
 * order of the reductions), never the method.
 *   probs       host array of nprob; only op.n, rank_max and prec are read
 *   cache_path  text file of lines "log2n width mixed rows_u rows_p", or NULL; read before
 *               tuning (its entries are taken as tuned; lines whose chunk heights are not
 *               powers of two in [64, 4096] and [16, 1024] are skipped) and, when this call
 *               timed a new key, rewritten after with every entry of ctx
 *   tuned       host, or NULL: the number of keys timed by this call
 * Uses the context workspace (grown on demand) and synchronises the stream; each key
 * costs up to 20 timed runs, seconds per key on grids of 10^6 points.  Errors:
 * PE_ERR_ARG for n < 64, rank_max outside [0, 31] or an unwritable cache file. */
pe_status pe_autotune(pe_ctx* ctx, const pe_problem* probs, int32_t nprob, const char* cache_path,
                      int32_t* tuned, void* stream);
/* The tuning table of ctx: writes up to max_rows rows of five int32 (log2n, width, mixed,
 * rows_u, rows_p) to rows (host, may be NULL) and returns the number of entries. */
int32_t pe_autotune_table(const pe_ctx* ctx, int32_t* rows, int32_t max_rows);

/* Kernel timing for roofline measurements.  Enables HIP-event timing, on the stream of
 * each call, of one kernel family: "block_update" (block Gram-Schmidt update + chunk QR
 * + TSQR combine) or "block_proj" (block projections) -- the first orthogonalisation
 * pass of every block Arnoldi step, which always runs in full -- or "gemm" (the f64 MFMA
 * products of the projected exponential, 2 N^3 flops per problem multiplied) or "stencil"
 * (pe_stencil_apply), or NULL to switch timing off.  Resets the accumulators.  Timing
 * adds two event records per timed launch; within a march every restart cycle is timed
 * (all of its block steps). */
pe_status pe_profile_enable(pe_ctx* ctx, const char* family);
/* Read and reset the accumulators: timed launches, their summed duration (ms), and the
 * algorithmic traffic (bytes, each datum read or written once per launch) and flops of
 * those launches.  All pointers are host pointers. */
pe_status pe_profile_read(pe_ctx* ctx, int64_t* launches, double* ms, double* bytes, double* flops);

#ifdef __cplusplus
}
#endif

#endif /* PARAEXP_H */
