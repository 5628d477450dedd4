// Shared device/host definitions of the gfx950 Paraexp library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#define PE_WAVE 64

// ---------------------------------------------------------------------------------
// Per-problem descriptor, resident in device memory and rewritten by the host at the
// start of each restart cycle.  All device pointers belong to the context workspace
// except u0 / G / out / coef which belong to the caller.
// ---------------------------------------------------------------------------------
struct ProbDev {
  // operator (paper Sec. 3, eq. 3.2): (L u)_i = cm[i] u_{i-1} + cz[i] u_i + cp[i] u_{i+1}
  int64_t n;
  int32_t per_point;
  double c3[3];            // constant coefficients when per_point == 0
  const double* coef;      // 3*n rows when per_point == 1

  // Krylov basis: (lmax+1) blocks of n*bw, row-major inside a block; fp64 or fp32 storage
  double* V;               // fp64 basis; with mixed storage only block 0, in fp64
  float* V32;              // fp32 basis (mixed storage)
  int32_t mixed;           // 1: basis stored in fp32 (V32), arithmetic in fp64
  double* Qloc1;           // n*bw local Q factors of the two TSQR passes
  double* Qloc2;
  double* Rloc;            // Cu*bw*bw local R factors (reused by both passes)
  double* Cn;              // Cu*bw squared column norms of the chunks before projection
  double* Qs1;             // Cu*bw*bw combine factors
  double* Qs2;
  double* Rf;              // 3 * bw*bw: final R of pass 1, pass 2, init
  double* Part;            // 2 * Cp*(nbmax)*bw*bw projection partials (pass 1, pass 2)
  double* S;               // 2 * nbmax*bw*bw reduced projection coefficients
  double* H;               // ((l+1)*bw) x (l*bw) column-major, ldH = (l+1)*bw
  int64_t ldH;
  unsigned* cnt;           // counters: [0..nbmax) pass-1 slots, [nbmax..2nbmax) pass 2, [2nbmax] update
  int32_t nbmax;           // capacity of slots (lmax + 1)

  // sources used by the first block of a cycle / by given-block mode
  const double* U;         // n x m column-major (ld n)
  const double* x;         // current state, n
  int32_t m;               // source columns in the first block
  int32_t with_x;          // 1: the state is the last column of the first block
  const double* Xg;        // given-block mode: column-major source matrix
  int64_t ldXg;

  double* xstate;          // writable state (same buffer as x)
  const double* yacc;      // accepted projected solution y (l*bw entries used)
  double* outcol;          // output column to receive the new state, or null
  int32_t proj;            // 1: project the state with this cycle's accepted y

  // cycle geometry
  int32_t bw;              // block width this cycle
  int32_t l;               // block steps this cycle
  int32_t active;          // 1: participates in this cycle's kernels
  int32_t rows_u;          // rows per update chunk (>= bw); last chunk takes the remainder
  int32_t rows_u_log2;     // rows_u is a power of two
  int32_t Cu;              // number of update chunks
  int32_t comb_global;     // 1: the TSQR combine works on the stacked factors in global memory
  int32_t comb_tree;       // 1: two-level register combine (blocks of 17..32 columns)
  double dep_tol;          // a column whose remainder after projection is <= dep_tol times its
                           // norm before projection is deflated (dependent)
  int32_t rows_p;          // rows per projection chunk
  int32_t Cp;              // number of projection chunks

  // shift-and-invert Arnoldi: the input block W = (I - gamma L)^{-1} V_j of a step,
  // row-major n x bw (fp64), written by the tridiagonal solve
  const double* Wb;
};

// ---------------------------------------------------------------------------------
// Shift-and-invert operator (I - gamma L)^{-1} of one problem: a periodic tridiagonal
// matrix T = I - gamma L solved by partition: the rows are cut into C chunks of R rows
// (C a power of two; the last chunk takes the remainder, R..2R-1 rows); each chunk is
// eliminated on its own (Thomas), its coupling to the neighbouring chunks' end rows
// enters through two spike vectors, and the 2C interface values solve a periodic
// block-tridiagonal system by cyclic reduction.
// ---------------------------------------------------------------------------------
struct TriDev {
  int64_t n;
  int32_t per_point;
  double c3[3];            // constant coefficients of L (per_point == 0)
  const double* coef;      // 3 n coefficients of L (per_point == 1)
  double gamma;            // shift: T = I - gamma L
  int32_t R, C;            // rows per chunk, chunks
  int32_t bw;              // columns of the current block
  int32_t active;
  double* ta;              // n: sub-diagonal of T
  double* tinv;            // n: inverse pivots of the chunk eliminations
  double* tc;              // n: eliminated super-diagonal
  double* vL;              // n: left spikes  T_c^{-1} (a_s e_first)
  double* vR;              // n: right spikes T_c^{-1} (b_e e_last)
  double* red;             // cyclic-reduction coefficients of the interface system (sai.hip)
  double* rrhs;            // 2 C x bw: interface values of the chunk solutions
  double* ru;              // 2 C x bw: interface values of the solution
  double* W;               // n x bw row-major: the solution block
  double* GW;              // bw x bw: Gram of (I - gamma L) V_l (residual estimate)
  int32_t* piv;            // row interchanges of the projected matrix's LU
  unsigned* cnt;           // 2 counters ([1]: the Gram's last-workgroup hand-off; [0] unused)
  double* LU;              // N0 x N0 (ld N0) work: LU factors of the projected matrix
  double* Kinv;            // N0 x N0 (ld N0): its inverse
  const double* H;         // projected matrix (Arnoldi Hessenberg of the shifted inverse)
  int64_t ldH;
  int32_t N0;              // l bw
};

// squaring levels whose exponential actions are evaluated in one trial
#define PE_MAX_LEVELS 40

struct ExpmDev {
  int32_t N;               // dimension of the augmented projected matrix (l*bw + q)
  int32_t active;          // 1: this problem runs the current trial
  int32_t nsq;             // squarings for this trial
  int32_t l, bw, m, q, with_x;
  int32_t lbw;             // l*bw: start of the polynomial block
  int32_t ldPi;
  double alpha;            // delta / 2^nsq
  double kscale;           // 2 / (t1 - t0): time derivative of the Chebyshev variable
  double* Ht;              // N x N column-major (unscaled augmented matrix)
  double* A;               // work matrices, N x N each
  double* A2;
  double* A3;
  double* A4;
  double* P;
  double* T;
  double* b;               // N: initial projected vector
  double* y;               // (kMaxLevels+1) x N: exp(alpha 2^k Ht) b for squaring level k
  double* out;             // 2 (kMaxLevels+1): per level error estimate, |y[0:lbw]|
  const double* H;         // Arnoldi Hessenberg, column-major, ldH
  int64_t ldH;
  const double* R0;        // bw x bw row-major: [U | x] = V_0 R0
  const double* Pi;        // m x q column-major (ldPi): Chebyshev coefficients of p(t)
  const double* w;         // q: T_k(x(tau)) at the start of the cycle
  const double* Dm;        // qmax x qmax row-major Chebyshev derivative matrix
  int32_t qmax;
  // shift-and-invert: the projected operator is (I - K^{-1}) / gamma with K the Arnoldi
  // matrix of (I - gamma L)^{-1}; the residual estimate needs the Gram of
  // (I - gamma L) V_l
  int32_t sai;
  double gamma;
  const double* Kinv;      // lbw x lbw (ld lbw)
  const double* GW;        // bw x bw
  // dense output by propagation: Eprop = exp(delta Ht) for an output spacing delta and
  // ycur the projected solution at the last output; a pass with prop = 1 forms
  // y_0 = Eprop ycur (level 0, no squarings) instead of evaluating a trial
  int32_t prop;
  double* Eprop;           // N x N column-major
  double* ycur;            // N
  // piecewise-cubic source: q = 4 m, the polynomial part holds the Taylor coefficients
  // z_j = p^(j)(t) / j! (blocks of m, z_j' = (j + 1) z_{j+1}); Pw[(i 4 + k) m + a] is
  // coefficient k of piece i of row a; piece / pdelta locate the current time
  int32_t spline;
  const double* Pw;
  int32_t piece;
  double pdelta;
  int32_t zreset;          // 1: k_spline_reset rewrites ycur's z part
};

// Host-visible helpers ---------------------------------------------------------
#define PE_CHECK_HIP(expr)                                                        \
  do {                                                                            \
    hipError_t _e = (expr);                                                       \
    if (_e != hipSuccess) return pe_fail(ctx, PE_ERR_DEVICE, #expr, _e);         \
  } while (0)
