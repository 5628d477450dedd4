// HIP kernels (gfx950) of the block-Krylov Paraexp exp-action path.
//
// Steps covered here (Kooij, Botchev & Geurts, arXiv 1509.04567):
//   S0  stencil operator (Sec. 3, eq. 3.2)                       k_stencil_cols, fused in k_block_*
//   S3  QR of the source samples (Sec. 2.1, eq. 2.2-2.3)         k_block_* in MODE_GIVEN
//   S5  block Arnoldi on K_l(A, [x|U]) (eq. 2.4)                 k_block_* in MODE_ARNOLDI / MODE_INIT
//   S6  exponential of the projected augmented matrix            k_build_aug, k_gemm (MFMA f64),
//                                                                k_elementwise, k_expm_apply
//   S7  state/output projection V y                              k_project
//   S8  superposition u = u0 + sum_j v_j (eq. 2.9)               k_superpose
//
// Block orthogonalisation = block classical Gram-Schmidt, a second pass only where the
// first leaves the new block insufficiently orthogonal to the basis, each pass followed
// by a tall-skinny QR (TSQR: a register-resident classical Gram-Schmidt QR of each row
// chunk, with a second in-chunk pass where needed, then a QR of the stacked chunk R
// factors by the last workgroup to finish).  Dependent columns are deflated (zero
// column, zero row of R) rather than replaced.
#include "devutil.h"
#include "kernels.h"
#include "policy.h"

#include <type_traits>

#include <cmath>

namespace pe {

// ------------------------------------------------------------------------------------
// reductions and helpers
// ------------------------------------------------------------------------------------
// Modified Gram-Schmidt applied twice, column by column, by the whole workgroup on a
// row-major rows x bw array X (leading dimension ld, any bw); thread t handles rows t,
// t + blockDim.x, ...  A column whose remainder is <= dep_tol times its norm as given is
// dependent and deflated: a zero column with a zero diagonal in R.  R (bw x bw,
// row-major, pre-zeroed) receives the triangular factor; `red` holds >= 16 doubles.
__device__ void mgs2_qr_block(double* X, int rows, int ld, int bw, double* R, double dep_tol, double* red) {
  const int T = (int)blockDim.x, t = (int)threadIdx.x;
  for (int b = 0; b < bw; ++b) {
    double s0 = 0.0;
    for (int r = t; r < rows; r += T) s0 += X[(int64_t)r * ld + b] * X[(int64_t)r * ld + b];
    const double n0 = sqrt(block_sum(s0, red));
    for (int pass = 0; pass < 2; ++pass)
      for (int a = 0; a < b; ++a) {
        double s = 0.0;
        for (int r = t; r < rows; r += T) s += X[(int64_t)r * ld + a] * X[(int64_t)r * ld + b];
        const double d = block_sum(s, red);
        for (int r = t; r < rows; r += T) X[(int64_t)r * ld + b] -= d * X[(int64_t)r * ld + a];
        if (t == 0) R[a * bw + b] += d;
      }
    double s1 = 0.0;
    for (int r = t; r < rows; r += T) s1 += X[(int64_t)r * ld + b] * X[(int64_t)r * ld + b];
    const double nr = sqrt(block_sum(s1, red));
    const bool dep = !(nr > dep_tol * n0 && nr > 1e-300);
    const double inv = dep ? 0.0 : 1.0 / nr;
    for (int r = t; r < rows; r += T) X[(int64_t)r * ld + b] *= inv;
    if (t == 0) R[b * bw + b] = dep ? 0.0 : nr;
  }
}

// Classical Gram-Schmidt applied twice, column by column, by a team of NW waves (NW = 1:
// one wave, no barriers; NW > 1: the whole workgroup, barriers inside) on a rows x bw
// array X with leading dimension ld, in LDS or global memory (thread t owns rows t,
// t + 64 NW, ..., so no row is touched by two threads).  The dot products of a column
// with the previous columns are reduced eight at a time within each wave (independent
// reductions overlap); one wave keeps dot a in lane a, a team exchanges the per-wave sums
// through the LDS scratch `red` (32 NW doubles) with one barrier pair per pass.  No
// per-thread array is indexed at run time.  A column whose remainder is <= dep_tol times
// its reference norm ref[b] is dependent: it becomes a zero column with a zero row in R
// (deflation), so it adds no direction and later columns do not couple to it.  R (bw x
// bw, row-major, pre-zeroed) receives the triangular factor.
__device__ __forceinline__ double lane_value(double v, int src) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), src);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), src);
  return __hiloint2double(hi, lo);
}
template <int NW>
__device__ __forceinline__ void cgs2_qr_team(double* X, int rows, int ld, int bw, double* R, const double* ref,
                                             double dep_tol, double* red) {
  const int t = (NW == 1) ? (int)(threadIdx.x & 63) : (int)threadIdx.x;
  const int w = t >> 6, lane = t & 63;
  constexpr int T = 64 * NW;
  double mydot = 0.0;  // NW == 1: lane a holds the dot product with column a
  auto team = [&](int a) -> double {
    if (NW == 1) return lane_value(mydot, a);
    double v = 0.0;
    for (int ww = 0; ww < NW; ++ww) v += red[ww * 32 + a];
    return v;
  };
  for (int b = 0; b < bw; ++b) {
    for (int pass = 0; pass < 2; ++pass) {
      for (int a0 = 0; a0 < b; a0 += 8) {
        double sd[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) sd[k] = 0.0;
        for (int r = t; r < rows; r += T) {
          const double xb = X[(int64_t)r * ld + b];
#pragma unroll
          for (int k = 0; k < 8; ++k)
            if (a0 + k < b) sd[k] += X[(int64_t)r * ld + a0 + k] * xb;
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) sd[k] = wave_sum(sd[k]);
        if (NW == 1) {
#pragma unroll
          for (int k = 0; k < 8; ++k)
            if (lane == a0 + k) mydot = sd[k];
        } else if (lane == 0) {
#pragma unroll
          for (int k = 0; k < 8; ++k)
            if (a0 + k < b) red[w * 32 + a0 + k] = sd[k];
        }
      }
      if (NW > 1) __syncthreads();
      for (int r = t; r < rows; r += T) {
        double acc = X[(int64_t)r * ld + b];
        for (int a = 0; a < b; ++a) acc -= team(a) * X[(int64_t)r * ld + a];
        X[(int64_t)r * ld + b] = acc;
      }
      for (int a = 0; a < b; ++a) {
        const double v = team(a);
        if (t == 0) R[a * bw + b] += v;
      }
      if (NW > 1) __syncthreads();
    }
    double s1 = 0.0;
    for (int r = t; r < rows; r += T) s1 += X[(int64_t)r * ld + b] * X[(int64_t)r * ld + b];
    s1 = wave_sum(s1);
    double nsq = s1;
    if (NW > 1) {
      if (lane == 0) red[w * 32] = s1;
      __syncthreads();
      nsq = team(0);
      __syncthreads();
    }
    const double nr = sqrt(nsq);
    const bool dep = !(nr > dep_tol * ref[b] && nr > 1e-300);
    const double inv = dep ? 0.0 : 1.0 / nr;
    for (int r = t; r < rows; r += T) X[(int64_t)r * ld + b] *= inv;
    if (t == 0) R[b * bw + b] = dep ? 0.0 : nr;
  }
}

// Register-resident Gram-Schmidt QR (classical, second pass where needed) of a rows x bw
// array (LDS, leading dimension ld) by a team
// of NW waves (NW = 1: no barriers; NW > 1: the whole workgroup, barriers inside).
// Thread t of the team keeps rows t + 64 NW q, q < RPL, in registers; column loops are
// unrolled to BWM >= bw so register indices are compile-time constants.  Dependent
// columns are deflated as in cgs2_qr_team.  `red` is LDS scratch of NW * BWM doubles.
template <int BWM, int RPL, int NW>
__device__ __forceinline__ void cgs2_team(const double* Xi, int ldi, double* X, int ld, int rows, int bw, double* R,
                                          const double* ref, double dep_tol, double* red) {
  const int t = (NW == 1) ? (int)(threadIdx.x & 63) : (int)threadIdx.x;
  const int w = t >> 6;
  constexpr int T = 64 * NW;
  double xr[RPL][BWM];
#pragma unroll
  for (int q = 0; q < RPL; ++q) {
    const int r = t + T * q;
#pragma unroll
    for (int a = 0; a < BWM; ++a) {
      // unconditional load from a clamped address, then select: a guarded load would
      // be compiled to a branch that waits for it, serialising the loads
      const double v = Xi[(r < rows ? r : rows - 1) * ldi + (a < bw ? a : bw - 1)];
      xr[q][a] = (a < bw && r < rows) ? v : 0.0;
    }
  }
  // sum over the team of NA values (NA known at compile time); result in sd[]
  auto team_sums = [&](double* sd, int NA) {
#pragma unroll
    for (int a = 0; a < BWM; ++a)
      if (a < NA) sd[a] = wave_sum(sd[a]);
    if (NW > 1) {
      __syncthreads();
      if ((t & 63) == 0)
#pragma unroll
        for (int a = 0; a < BWM; ++a)
          if (a < NA) red[w * BWM + a] = sd[a];
      __syncthreads();
#pragma unroll
      for (int a = 0; a < BWM; ++a)
        if (a < NA) {
          double v = 0.0;
          for (int ww = 0; ww < NW; ++ww) v += red[ww * BWM + a];
          sd[a] = v;
        }
    }
  };
#pragma unroll
  for (int b = 0; b < BWM; ++b) {
    if (b < bw) {
      const double n0 = ref[b];
      // First pass: the projections on the previous columns and the squared norm are
      // reduced together; the norm after the pass follows by Pythagoras.  A second pass
      // runs only when the first removed more than half of the squared norm ("twice is
      // enough", Kahan and Parlett): otherwise the remainder is already orthogonal to
      // working precision.  A column thus costs one team reduction, or two.
      double nsq, s2sum = 0.0;
      {
        double sd[BWM];
#pragma unroll
        for (int a = 0; a < BWM; ++a) sd[a] = 0.0;
#pragma unroll
        for (int q = 0; q < RPL; ++q) {
#pragma unroll
          for (int a = 0; a < b; ++a) sd[a] += xr[q][a] * xr[q][b];
          sd[b] += xr[q][b] * xr[q][b];
        }
        team_sums(sd, b + 1);
#pragma unroll
        for (int q = 0; q < RPL; ++q)
#pragma unroll
          for (int a = 0; a < b; ++a) xr[q][b] -= sd[a] * xr[q][a];
        if (t == 0)
#pragma unroll
          for (int a = 0; a < b; ++a) R[a * bw + b] += sd[a];
        nsq = sd[b];
#pragma unroll
        for (int a = 0; a < b; ++a) s2sum += sd[a] * sd[a];
      }
      if (b > 0 && nsq - s2sum < 0.5 * nsq) {
        double sd[BWM];
#pragma unroll
        for (int a = 0; a < BWM; ++a) sd[a] = 0.0;
#pragma unroll
        for (int q = 0; q < RPL; ++q) {
#pragma unroll
          for (int a = 0; a < b; ++a) sd[a] += xr[q][a] * xr[q][b];
          sd[b] += xr[q][b] * xr[q][b];
        }
        team_sums(sd, b + 1);
#pragma unroll
        for (int q = 0; q < RPL; ++q)
#pragma unroll
          for (int a = 0; a < b; ++a) xr[q][b] -= sd[a] * xr[q][a];
        if (t == 0)
#pragma unroll
          for (int a = 0; a < b; ++a) R[a * bw + b] += sd[a];
        nsq = sd[b];
        s2sum = 0.0;
#pragma unroll
        for (int a = 0; a < b; ++a) s2sum += sd[a] * sd[a];
      }
      const double nr = sqrt(nsq > s2sum ? nsq - s2sum : 0.0);
      const bool dep = !(nr > dep_tol * n0 && nr > 1e-300);
      const double inv = dep ? 0.0 : 1.0 / nr;
#pragma unroll
      for (int q = 0; q < RPL; ++q) xr[q][b] *= inv;
      if (t == 0) R[b * bw + b] = dep ? 0.0 : nr;
    }
  }
#pragma unroll
  for (int q = 0; q < RPL; ++q) {
    const int r = t + T * q;
    if (r < rows)
#pragma unroll
      for (int a = 0; a < BWM; ++a)
        if (a < bw) X[r * ld + a] = xr[q][a];
  }
}

// dispatch of the register-resident QR over block-width buckets and rows per thread;
// Xi (ld ldi) is read once, the Q factor written to X (ld ld), which may alias Xi
template <int NW>
__device__ __forceinline__ bool cgs2_dispatch(const double* Xi, int ldi, double* X, int ld, int rows, int bw, double* R,
                                              const double* ref, double dep_tol, double* red) {
  const int rpl = (rows + 64 * NW - 1) / (64 * NW);
  if (bw <= 8) {
    if (rpl <= 1) { cgs2_team<8, 1, NW>(Xi, ldi, X, ld, rows, bw, R, ref, dep_tol, red); return true; }
    if (rpl <= 2) { cgs2_team<8, 2, NW>(Xi, ldi, X, ld, rows, bw, R, ref, dep_tol, red); return true; }
    if (rpl <= 4) { cgs2_team<8, 4, NW>(Xi, ldi, X, ld, rows, bw, R, ref, dep_tol, red); return true; }
  } else if (bw <= 16) {
    if (rpl <= 1) { cgs2_team<16, 1, NW>(Xi, ldi, X, ld, rows, bw, R, ref, dep_tol, red); return true; }
  }
  return false;  // wider blocks or more rows: cgs2_qr_team on an LDS or global array
}


// ------------------------------------------------------------------------------------
// S0: Y = L X, column-major blocks
// ------------------------------------------------------------------------------------
__global__ void k_stencil_cols(int64_t n, int per_point, double c0, double c1, double c2, const double* coef,
                               const double* __restrict__ X, int64_t ldx, double* __restrict__ Y, int64_t ldy) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (r >= n) return;
  const double* x = X + (int64_t)c * ldx;
  const int64_t rm = r == 0 ? n - 1 : r - 1;
  const int64_t rp = r == n - 1 ? 0 : r + 1;
  double cm = c0, cz = c1, cp = c2;
  if (per_point) {
    cm = coef[r];
    cz = coef[n + r];
    cp = coef[2 * n + r];
  }
  Y[(int64_t)c * ldy + r] = cm * x[rm] + cz * x[r] + cp * x[rp];
}

void launch_stencil_cols(int64_t n, int per_point, const double* c3, const double* coef, const double* X,
                         int64_t ldx, double* Y, int64_t ldy, int ncols, hipStream_t st) {
  if (n <= 0 || ncols <= 0) return;
  dim3 grid((unsigned)((n + 255) / 256), (unsigned)ncols);
  double a = per_point ? 0.0 : c3[0], b = per_point ? 0.0 : c3[1], c = per_point ? 0.0 : c3[2];
  hipLaunchKernelGGL(k_stencil_cols, grid, dim3(256), 0, st, n, per_point, a, b, c, coef, X, ldx, Y, ldy);
}

__global__ void k_add_column(int64_t n, const double* __restrict__ G, int64_t ldG, const double* __restrict__ add,
                             double* __restrict__ Gh, int64_t ldGh) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (r >= n) return;
  Gh[(int64_t)c * ldGh + r] = G[(int64_t)c * ldG + r] + (add ? add[r] : 0.0);
}

void launch_add_column(int64_t n, int s, const double* G, int64_t ldG, const double* add, double* Gh,
                       int64_t ldGh, hipStream_t st) {
  dim3 grid((unsigned)((n + 255) / 256), (unsigned)s);
  hipLaunchKernelGGL(k_add_column, grid, dim3(256), 0, st, n, G, ldG, add, Gh, ldGh);
}

// ------------------------------------------------------------------------------------
// Block orthogonalisation.  Per block step and pass:
//   k_block_proj:   S_i = V_i^T X over row chunks, for a group of GS slots per workgroup;
//                   the last workgroup of a group reduces the chunk partials into S.
//   k_block_update: X -= sum_i V_i S_i on one row chunk, wave-level QR of the chunk,
//                   and the TSQR combine by the last workgroup.
// The input block X of a pass is
//   pass 0, MODE_ARNOLDI: W = L V_j, V_j given by the previous TSQR (Qloc2, Qs2);
//                         the projection kernel commits V_j to the basis
//   pass 0, MODE_GIVEN:   columns [j*bw, j*bw + bw) of the given matrix
//   pass 0, MODE_INIT:    [U | x]
//   pass 1:               Q1 of the pass-0 TSQR (Qloc1, Qs1)
// ------------------------------------------------------------------------------------


// Bulk global -> LDS copy: cnt elements, element e read by src(e) and stored by
// put(e, v).  Each thread keeps kBulkDepth loads in flight, so a phase costs one or two
// memory round trips however many elements a thread handles (data written by other
// workgroups comes from other XCDs with microsecond latency).
__device__ __forceinline__ int64_t wrap_row(int64_t g, int64_t n) { return g < 0 ? g + n : (g >= n ? g - n : g); }

// Input block X (rows x bw, leading dimension ld, LDS) of the update kernel's chunk
// [r0, r0 + rows) (one TSQR chunk).  Qrow: LDS staging of (rows + 2) x bw doubles, Qsl
// of one bw x bw combine block.  Row/column walks are per thread (col = t % bw fixed) so
// no division sits in the loops.
template <typename TS>
__device__ __forceinline__ void form_block(const ProbDev& p, int mode, int pass, int j, int64_t r0, int rows, double* X,
                                           int ld, double* Qrow, double* Qsl) {
  const int bw = p.bw, bw2 = bw * bw;
  const int t = threadIdx.x, T = blockDim.x;
  const int64_t n = p.n;
  const TS* V = basis_ptr<TS>(p);
  const int64_t blk = n * bw;
  const int col = t % bw, rstep = T / bw, rr0 = t / bw;
  const bool act = rr0 < rstep;
  if (mode == MODE_INIT) {  // [U | x], column-major sources: coalesce along rows
    bulk_load(
        (int64_t)rows * bw,
        [&](int64_t e) -> double {
          const int c = (int)(e / rows);
          const int64_t g = r0 + e % rows;
          const double* ptr = c < p.m ? p.U + (int64_t)c * n + g : p.x + g;
          return *ptr;
        },
        [&](int64_t e, double v) { X[(e % rows) * ld + e / rows] = v; });
  } else if (pass == 0 && mode == MODE_GIVEN) {
    bulk_load(
        (int64_t)rows * bw,
        [&](int64_t e) -> double {
          const int gc = j * bw + (int)(e / rows);
          const double v = p.Xg[(int64_t)(gc < p.m ? gc : p.m - 1) * p.ldXg + r0 + e % rows];
          return gc < p.m ? v : 0.0;
        },
        [&](int64_t e, double v) { X[(e % rows) * ld + e / rows] = v; });
  } else if (pass == 0 && mode == MODE_SAI) {  // W = (I - gamma L)^{-1} V_j, solved beforehand
    bulk_load(
        (int64_t)rows * bw, [&](int64_t e) -> double { return p.Wb[r0 * bw + e]; },
        [&](int64_t e, double v) { X[(e / bw) * ld + e % bw] = v; });
  } else if (pass == 0) {  // MODE_ARNOLDI: W = L V_j, V_j read from the basis
    const TS* vj = V + (int64_t)j * blk;
    const int64_t gm = wrap_row(r0 - 1, n), gp = wrap_row(r0 + rows, n);
    const int64_t top = (int64_t)(rows + 1) * bw;
    bulk_load(
        top + bw,
        [&](int64_t e) -> double {  // rows r0-1 .. r0+rows, the halo rows wrapped
          return (double)vj[e < bw ? gm * bw + e : (e >= top ? gp * bw + (e - top) : (r0 - 1) * bw + e)];
        },
        [&](int64_t e, double v) { Qrow[e] = v; });
    __syncthreads();
    if (act)
      for (int rr = rr0; rr < rows; rr += rstep) {
        double cm, cz, cp;
        stencil_coefs(p, r0 + rr, cm, cz, cp);
        X[rr * ld + col] = cm * Qrow[rr * bw + col] + cz * Qrow[(rr + 1) * bw + col] + cp * Qrow[(rr + 2) * bw + col];
      }
  } else {  // pass 1: X = Q1 = Qloc1 Qs1 on this chunk
    const int64_t nr = (int64_t)rows * bw;
    const double* qs = p.Qs1 + (int64_t)chunk_of(p, r0) * bw2 - nr;
    bulk_load(
        nr + bw2,
        [&](int64_t e) -> double {
          const double* ptr = e < nr ? p.Qloc1 + r0 * bw + e : qs + e;  // select, then one load
          return *ptr;
        },
        [&](int64_t e, double v) {
          if (e < nr) Qrow[e] = v;
          else Qsl[e - nr] = v;
        });
    __syncthreads();
    if (act)
      for (int rr = rr0; rr < rows; rr += rstep) {
        double v = 0.0;
        for (int k = 0; k < bw; ++k) v += Qrow[rr * bw + k] * Qsl[k * bw + col];
        X[rr * ld + col] = v;
      }
  }
  __syncthreads();
}

// Projections S_i = V_i^T X, i in the workgroup's slot group, on one row chunk.  One
// bulk phase stages everything the chunk needs (TSQR factors of the input block and the
// basis rows of the group's slots); the input block is formed in LDS (in MODE_ARNOLDI
// pass 0: V_j = Qloc2 Qs2 with its halo, committed to the basis by slot group 0, then
// W = L V_j); each thread then owns one output of one slot over all rows of the chunk.
// The last workgroup of a slot group reduces the Cp chunk partials into S.
template <typename TS>
__global__ __launch_bounds__(256) void k_block_proj(const ProbDev* __restrict__ probs, int j, int nb, int pass, int mode) {
  const ProbDev p = probs[blockIdx.y];  // by value: uniform, loaded once
  if (!p.active || j >= p.l) return;
  const int bw = p.bw, nout = bw * bw, bw2 = nout;
  const int grp = blockIdx.x / p.Cp;
  const int c = blockIdx.x % p.Cp;
  const int ngroups = (nb + kSlotGroup - 1) / kSlotGroup;
  if (grp >= ngroups) return;
  if (arnoldi_mode(mode) && pass == 1 && p.cnt[2 * p.nbmax + 1]) return;  // reorthogonalisation not needed
  const int64_t n = p.n;
  const int64_t r0 = (int64_t)c * p.rows_p;
  if (r0 >= n) return;
  const int rows = (int)(r0 + p.rows_p < n ? p.rows_p : n - r0);
  const int t = threadIdx.x;
  extern __shared__ double smem[];
  // unpadded row-major tiles: every access below is a broadcast or walks consecutive rows
  double* Xs = smem;                                           // rows_p * bw
  double* Vh = Xs + (int64_t)p.rows_p * bw;                    // (rows_p + 2) * bw
  double* Vs = Vh + (int64_t)(p.rows_p + 2) * bw;              // kSlotGroup * rows_p * bw
  double* red = Vs + (int64_t)kSlotGroup * p.rows_p * bw;      // 256
  double* Qrow = red + 256;                                    // (rows_p + 2) * bw
  double* Qsl = Qrow + (int64_t)(p.rows_p + 2) * bw;           // (rows_p / rows_u + 4) * bw^2
  __shared__ int is_last;
  TS* V = basis_ptr<TS>(p);
  const int64_t blk = n * bw;
  const bool arn0 = (mode == MODE_ARNOLDI && pass == 0);
  const bool given0 = (mode == MODE_GIVEN && pass == 0);
  const bool sai0 = (mode == MODE_SAI && pass == 0);  // input block W from Wb, V_j committed
  const int i_lo = grp * kSlotGroup, i_hi = min(nb, i_lo + kSlotGroup);
  const int col = t % bw, rstep = 256 / bw, rr0 = t / bw;
  const bool act = rr0 < rstep;

  // ---- one bulk phase: every global load of the chunk is issued before any is
  // consumed, with plain per-thread strides (rows_p * bw <= 1024, checked on the host)
  const int u_lo = chunk_of(p, r0), u_hi = chunk_of(p, r0 + rows - 1);
  const int nm = u_hi - u_lo + 1;
  {
    const int per_slot = rows * bw;
    double vv[kSlotGroup][4];
#pragma unroll
    for (int kk = 0; kk < kSlotGroup; ++kk) {
      const int i = i_lo + kk < nb ? i_lo + kk : nb - 1;
      const TS* base = V + (int64_t)i * blk + r0 * bw;
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const int e = t + 256 * m;
        vv[kk][m] = (double)base[e < per_slot ? e : per_slot - 1];
      }
    }
    // V_j is the last pass's TSQR output: the first pass's when the previous step
    // skipped its second pass
    const bool first = !arn0 || p.cnt[2 * p.nbmax + 1] != 0;
    const double* Ql = first ? p.Qloc1 : p.Qloc2;
    const double* Qsb = first ? p.Qs1 : p.Qs2;
    const int64_t gm = wrap_row(r0 - 1, n), gp = wrap_row(r0 + rows, n);
    const int nqr = (arn0 ? rows + 2 : rows) * bw;
    double qv[5];
#pragma unroll
    for (int m = 0; m < 5; ++m) {
      const int e0 = t + 256 * m;
      const int e = e0 < nqr ? e0 : nqr - 1;
      int64_t a;
      if (arn0)  // halo rows wrap around the periodic grid
        a = e < bw ? gm * bw + e : (e >= (rows + 1) * bw ? gp * bw + (e - (rows + 1) * bw) : (r0 - 1) * bw + e);
      else
        a = r0 * bw + e;
      qv[m] = Ql[a];
    }
    const int ua = chunk_of(p, gm), ub = chunk_of(p, gp);
    const int nqs = (nm + (arn0 ? 2 : 0)) * bw2;
    const float inv_bw2 = 1.0f / (float)bw2;
    auto qs_addr = [&](int e) -> int64_t {
      const int b = (int)(((float)e + 0.5f) * inv_bw2);
      const int u = b < nm ? u_lo + b : (b == nm ? ua : ub);
      return (int64_t)u * bw2 + (e - b * bw2);
    };
    double sq[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const int e0 = t + 256 * m;
      sq[m] = Qsb[qs_addr(e0 < nqs ? e0 : nqs - 1)];
    }
#pragma unroll
    for (int kk = 0; kk < kSlotGroup; ++kk) {
      const int i = i_lo + kk;
      if (i < i_hi && !(arn0 && i == j))
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          const int e = t + 256 * m;
          if (e < per_slot) Vs[(int64_t)kk * p.rows_p * bw + e] = vv[kk][m];
        }
    }
    if (!given0 && !sai0) {
#pragma unroll
      for (int m = 0; m < 5; ++m)
        if (t + 256 * m < nqr) Qrow[t + 256 * m] = qv[m];
#pragma unroll
      for (int m = 0; m < 4; ++m)
        if (t + 256 * m < nqs) Qsl[t + 256 * m] = sq[m];
      for (int e = t + 1024; e < nqs; e += 256) Qsl[e] = Qsb[qs_addr(e)];  // wide blocks only
    }
  }
  if (given0)
    bulk_load(
        (int64_t)rows * bw,
        [&](int64_t e) -> double {
          const int gc = j * bw + (int)(e / rows);
          const double v = p.Xg[(int64_t)(gc < p.m ? gc : p.m - 1) * p.ldXg + r0 + e % rows];
          return gc < p.m ? v : 0.0;
        },
        [&](int64_t e, double v) { Xs[(e % rows) * bw + e / rows] = v; });
  else if (sai0)
    bulk_load(
        (int64_t)rows * bw, [&](int64_t e) -> double { return p.Wb[r0 * bw + e]; },
        [&](int64_t e, double v) { Xs[e] = v; });
  __syncthreads();
  // ---- form the input block
  if (arn0) {
    const bool commit = (grp == 0);
    if (act)
      for (int rr = rr0; rr < rows + 2; rr += rstep) {
        const int slot = rr == 0 ? nm : (rr == rows + 1 ? nm + 1 : chunk_of(p, r0 - 1 + rr) - u_lo);
        const double* q = Qrow + rr * bw;
        const double* sq = Qsl + slot * bw2 + col;
        double v = 0.0;
        for (int k = 0; k < bw; ++k) v += q[k] * sq[k * bw];
        const TS vs = (TS)v;
        Vh[rr * bw + col] = (double)vs;
        if (commit && rr >= 1 && rr <= rows) {
          V[(int64_t)j * blk + (r0 - 1 + rr) * bw + col] = vs;
          // fp32 storage: block 0 is also kept unrounded for the state projection
          if (!std::is_same<TS, double>::value && j == 0) p.V[(r0 - 1 + rr) * bw + col] = v;
        }
      }
    __syncthreads();
    if (act)
      for (int rr = rr0; rr < rows; rr += rstep) {
        double cm, cz, cp;
        stencil_coefs(p, r0 + rr, cm, cz, cp);
        Xs[rr * bw + col] = cm * Vh[rr * bw + col] + cz * Vh[(rr + 1) * bw + col] + cp * Vh[(rr + 2) * bw + col];
      }
    if (j >= i_lo && j < i_hi) {  // slot j is V_j itself
      double* dst = Vs + (int64_t)(j - i_lo) * p.rows_p * bw;
      for (int e = t; e < rows * bw; e += 256) dst[e] = Vh[bw + e];
    }
  } else if (!given0 && !sai0) {  // pass 1: X = Q1 = Qloc1 Qs1
    if (act)
      for (int rr = rr0; rr < rows; rr += rstep) {
        const double* q = Qrow + rr * bw;
        const double* sq = Qsl + (int64_t)(chunk_of(p, r0 + rr) - u_lo) * bw2 + col;
        double v = 0.0;
        for (int k = 0; k < bw; ++k) v += q[k] * sq[k * bw];
        Xs[rr * bw + col] = v;
      }
  }
  __syncthreads();
  // ---- chunk partials: one output of one slot per thread, all rows
  double* part = p.Part + (int64_t)pass * p.Cp * p.nbmax * nout;
  for (int e = t; e < (i_hi - i_lo) * nout; e += 256) {
    const int kk = e / nout, o = e - kk * nout, a = o / bw, b = o - a * bw;
    const double* Vi = Vs + (int64_t)kk * p.rows_p * bw;
    double acc0 = 0.0, acc1 = 0.0;
    int rr = 0;
    for (; rr + 1 < rows; rr += 2) {
      acc0 += Vi[rr * bw + a] * Xs[rr * bw + b];
      acc1 += Vi[(rr + 1) * bw + a] * Xs[(rr + 1) * bw + b];
    }
    if (rr < rows) acc0 += Vi[rr * bw + a] * Xs[rr * bw + b];
    st_agent(part + ((int64_t)(i_lo + kk) * p.Cp + c) * nout + o, acc0 + acc1);
  }
  // ---- the last workgroup of this slot group reduces the Cp partials of its slots
  if (!arrive_last(p.cnt + pass * p.nbmax + grp, (unsigned)p.Cp, &is_last)) return;
  double* Sout = p.S + (int64_t)pass * p.nbmax * nout;
  // G threads per output, each summing a strided subset of the partials with 32 loads
  // in flight
  const int total = (i_hi - i_lo) * nout;
  const int G = total >= 256 ? 1 : 256 / total;
  const int per = 256 / G;
  for (int e0 = 0; e0 < total; e0 += per) {
    const int e = e0 + t / G, g = t % G;
    double acc = 0.0;
    if (t < per * G && e < total) {
      const double* ps = part + (int64_t)(i_lo + e / nout) * p.Cp * nout + (e % nout);
      for (int cc = g; cc < p.Cp; cc += 32 * G) {
        double v[32];
#pragma unroll
        for (int k = 0; k < 32; ++k) {
          const int c2 = cc + k * G;
          const double x = ps[(int64_t)(c2 < p.Cp ? c2 : p.Cp - 1) * nout];
          v[k] = c2 < p.Cp ? x : 0.0;
        }
#pragma unroll
        for (int k = 0; k < 32; ++k) acc += v[k];
      }
    }
    red[t] = acc;
    __syncthreads();
    if (g == 0 && t < per * G && e < total) {
      double sacc = 0.0;
      for (int gg = 0; gg < G; ++gg) sacc += red[t + gg];
      Sout[(int64_t)(i_lo + e / nout) * nout + (e % nout)] = sacc;
    }
    __syncthreads();
  }
  if (t == 0) atomicExch(p.cnt + pass * p.nbmax + grp, 0u);
}

typedef double dbl4 __attribute__((ext_vector_type(4)));

// X (rows x bw, LDS, ld) -= sum_{i < nb} V_i[rows] S_i on f64 MFMA (16x16x4): wave w takes
// 16-row tiles w, w+4, ...; the A operand (-V rows) streams from global memory with PF
// slots of loads in flight, the B operand (S_i, row-major bw x bw) from LDS, staged in
// batches of kSb doubles.  Accumulator layout: row = lane/16 + 4v, column = lane%16.
template <int BWM, typename TS>
__device__ __forceinline__ void subtract_proj_mfma(const TS* V, int64_t blk, const double* Sp, int nb, int64_t r0,
                                                   int rows, int bw, double* X, int ld, double* Sb) {
  constexpr int KT = BWM / 4;                   // k-steps per slot
  constexpr int NT = (BWM + 15) / 16;           // 16-column tiles
  constexpr int PF = BWM <= 8 ? 8 : (BWM <= 16 ? 4 : 2);
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int nout = bw * bw;
  const int ksb = max(1, kSb / nout);
  const int RT = (rows + 15) / 16;
  const int li = lane & 15, lk = lane >> 4;
  for (int i0 = 0; i0 < nb; i0 += ksb) {
    const int k = min(ksb, nb - i0);
    __syncthreads();
    bulk_load(
        (int64_t)k * nout, [&](int64_t e) -> double { return Sp[(int64_t)i0 * nout + e]; },
        [&](int64_t e, double v) { Sb[e] = v; });
    __syncthreads();
    for (int rt = w; rt < RT; rt += 4) {
      const int row = rt * 16 + li;  // A-operand row of this lane
      const bool rok = row < rows;
      dbl4 acc[NT];
#pragma unroll
      for (int nt = 0; nt < NT; ++nt)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int rr = rt * 16 + lk + 4 * v, cc = nt * 16 + li;
          acc[nt][v] = (rr < rows && cc < bw) ? X[rr * ld + cc] : 0.0;
        }
      for (int kk0 = 0; kk0 < k; kk0 += PF) {
        double a[PF][KT];
#pragma unroll
        for (int f = 0; f < PF; ++f) {
          // clamped addresses and unconditional loads keep all PF * KT loads in flight
          const bool fok = kk0 + f < k;
          const TS* vr = V + (int64_t)(i0 + (fok ? kk0 + f : k - 1)) * blk + (r0 + (rok ? row : rows - 1)) * bw;
#pragma unroll
          for (int kt = 0; kt < KT; ++kt) {
            const int ka = kt * 4 + lk;
            const double x = (double)vr[ka < bw ? ka : bw - 1];
            a[f][kt] = (fok && rok && ka < bw) ? -x : 0.0;
          }
        }
#pragma unroll
        for (int f = 0; f < PF; ++f) {
          if (kk0 + f >= k) break;
          const double* sb = Sb + (kk0 + f) * nout;
#pragma unroll
          for (int kt = 0; kt < KT; ++kt) {
            const int ka = kt * 4 + lk;
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) {
              const int cc = nt * 16 + li;
              const double b = (ka < bw && cc < bw) ? sb[ka * bw + cc] : 0.0;
              acc[nt] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[f][kt], b, acc[nt], 0, 0, 0);
            }
          }
        }
      }
#pragma unroll
      for (int nt = 0; nt < NT; ++nt)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int rr = rt * 16 + lk + 4 * v, cc = nt * 16 + li;
          if (rr < rows && cc < bw) X[rr * ld + cc] = acc[nt][v];
        }
    }
  }
  __syncthreads();
}

// the second Gram-Schmidt pass of an Arnoldi step is skipped when every column of the
// first pass's Q1 is orthogonal to the basis to ~eps / kReorthSkip (reorth_column_ok)
constexpr double kReorthSkip = 0.3;

template <typename TS>
__global__ __launch_bounds__(256) void k_block_update(const ProbDev* __restrict__ probs, int j, int nb, int pass, int mode) {
  const ProbDev p = probs[blockIdx.y];  // by value: uniform, loaded once
  if (!p.active || (mode != MODE_INIT && j >= p.l)) return;
  const int bw = p.bw, nout = bw * bw;
  const int u = blockIdx.x;
  if (u >= p.Cu) return;
  const int64_t n = p.n;
  const int64_t r0 = (int64_t)u * p.rows_u;
  const int64_t r1 = (u == p.Cu - 1) ? n : r0 + p.rows_u;
  const int rows = (int)(r1 - r0);
  const int rmax = 2 * p.rows_u;
  const int ld = bw + 1;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const bool reg_comb = combine_in_registers(bw, p.Cu);
  extern __shared__ double smem[];
  const int64_t xs_cap =
      p.comb_tree ? (int64_t)ld * max(rmax, max(kTreeFan, (p.Cu + kTreeFan - 1) / kTreeFan) * bw)
                  : (int64_t)ld * (reg_comb || p.comb_global || rmax > p.Cu * bw ? rmax : p.Cu * bw);
  double* X = smem;                               // xs_cap
  // the input rows staged for form_block are dead once the block is formed: the
  // projection coefficients of the subtraction reuse that space
  double* Qrow = X + xs_cap;                      // (rmax + 2) * bw
  double* Sb = Qrow;                              // kSb
  double* Rl = Qrow + max((int64_t)kSb, (int64_t)(rmax + 2) * bw);  // bw^2
  double* Rn = Rl + nout;                         // bw
  double* Qsl = Rn + bw;                          // max(bw^2, 128)
  __shared__ int is_last;
  const TS* V = basis_ptr<TS>(p);
  const int64_t blk = n * bw;
  const bool hcol = (mode != MODE_INIT && pass == 1);

  // Arnoldi steps whose first pass kept enough of every column skip the second pass
  // (decided, and column block j of H written, by the first pass's last workgroup)
  if (arnoldi_mode(mode) && pass == 1 && p.cnt[2 * p.nbmax + 1]) return;

  // 0. pass 1: blocks i < nb of column block j of H (of R in MODE_GIVEN), one block per
  //    workgroup: H_ij = S1_i + S2_i Rf1 (the block nb needs the combine below)
  if (hcol) {
    const double* R1 = p.Rf;
    const double* S1 = p.S;
    const double* S2 = p.S + (int64_t)p.nbmax * nout;
    for (int i = u; i < nb; i += p.Cu)
      for (int o = t; o < nout; o += 256) {
        const int a = o / bw, b = o % bw;
        double v = S1[(int64_t)i * nout + o];
#pragma unroll 8
        for (int k = 0; k < bw; ++k) v += S2[(int64_t)i * nout + a * bw + k] * R1[k * bw + b];
        p.H[(int64_t)(i * bw + a) + p.ldH * (int64_t)(j * bw + b)] = v;
      }
    // blocks below the subdiagonal block are never written: readers take them as zero
  }
  // 1. input block of this chunk
  form_block<TS>(p, mode, pass, j, r0, rows, X, ld, Qrow, Qsl);
  // reference column norms before the projections
  for (int b = w; b < bw; b += 4) {
    double s0 = 0.0;
    for (int rr = lane; rr < rows; rr += 64) s0 += X[rr * ld + b] * X[rr * ld + b];
    s0 = wave_sum(s0);
    if (lane == 0) {
      Rn[b] = sqrt(s0);
      st_agent(p.Cn + (int64_t)u * bw + b, s0);
    }
  }
  // 2. X -= sum_i V_i S_i
  if (mode != MODE_INIT) {
    const double* Sp = p.S + (int64_t)pass * p.nbmax * nout;
    if (bw <= 8)
      subtract_proj_mfma<8, TS>(V, blk, Sp, nb, r0, rows, bw, X, ld, Sb);
    else if (bw <= 16)
      subtract_proj_mfma<16, TS>(V, blk, Sp, nb, r0, rows, bw, X, ld, Sb);
    else
      subtract_proj_mfma<32, TS>(V, blk, Sp, nb, r0, rows, bw, X, ld, Sb);
  }
  // 3. local QR of the chunk (wave 0)
  for (int o = t; o < nout; o += 256) Rl[o] = 0.0;
  __syncthreads();
  // Q of the chunk goes straight from registers to Qloc (row-major, ld bw)
  double* Qloc = (pass == 0 ? p.Qloc1 : p.Qloc2) + r0 * bw;
  __shared__ int reg_qr;
  if (t == 0) reg_qr = 1;
  __syncthreads();
  if (w == 0) {
    if (!cgs2_dispatch<1>(X, ld, Qloc, bw, rows, bw, Rl, Rn, p.dep_tol, nullptr)) {
      cgs2_qr_team<1>(X, rows, ld, bw, Rl, Rn, p.dep_tol, Qsl);
      if (lane == 0) reg_qr = 0;
    }
  }
  __syncthreads();
  if (!reg_qr) {
    const int col = t % bw, rstep = 256 / bw;
    if (t / bw < rstep)
      for (int rr = t / bw; rr < rows; rr += rstep) Qloc[rr * bw + col] = X[rr * ld + col];
  }
  for (int o = t; o < nout; o += 256) st_agent(p.Rloc + (int64_t)u * nout + o, Rl[o]);
  double* Qs = pass == 0 ? p.Qs1 : p.Qs2;
  int ngroups = 0;
  if (p.comb_tree) {
    // 4a. two-level combine (stacks too tall for one workgroup's LDS): the last workgroup
    // of each group of kTreeFan chunks factors the group's stacked factors (one wave, from
    // LDS; dependence judged against the group's column norms), writes the group's Q
    // blocks to Qs and its R factor over the first chunk's slot of Rloc
    ngroups = (p.Cu + kTreeFan - 1) / kTreeFan;
    const int g = u / kTreeFan, ua = g * kTreeFan, ub = min(p.Cu, ua + kTreeFan);
    if (!arrive_last(p.cnt + 2 * p.nbmax + 2 + g, (unsigned)(ub - ua), &is_last)) return;
    const int rg = (ub - ua) * bw;
    bulk_load(
        (int64_t)rg * bw, [&](int64_t e) -> double { return p.Rloc[(int64_t)ua * nout + e]; },
        [&](int64_t e, double v) { X[(e / bw) * ld + (e % bw)] = v; });
    for (int o = t; o < nout; o += 256) Rl[o] = 0.0;
    {
      const int per = 256 / bw, b = t % bw, k = t / bw;
      double acc = 0.0;
      if (k < per)
        for (int uu = ua + k; uu < ub; uu += per) acc += p.Cn[(int64_t)uu * bw + b];
      Sb[t] = acc;
    }
    __syncthreads();
    for (int b = t; b < bw; b += 256) {
      double s0 = 0.0;
      for (int k = 0; k < 256 / bw; ++k) s0 += Sb[k * bw + b];
      Rn[b] = sqrt(s0);
    }
    __syncthreads();
    if (w == 0) cgs2_qr_team<1>(X, rg, ld, bw, Rl, Rn, p.dep_tol, Qsl);
    __syncthreads();
    for (int e = t; e < rg * bw; e += 256) st_agent(Qs + (int64_t)ua * nout + e, X[(e / bw) * ld + (e % bw)]);
    for (int o = t; o < nout; o += 256) st_agent(p.Rloc + (int64_t)ua * nout + o, Rl[o]);
    if (t == 0) atomicExch(p.cnt + 2 * p.nbmax + 2 + g, 0u);
  }
  // 4. TSQR combine by the last workgroup (of all chunks, or of all groups)
  if (!arrive_last(p.cnt + 2 * p.nbmax, (unsigned)(p.comb_tree ? ngroups : p.Cu), &is_last)) return;
  const int srows = (p.comb_tree ? ngroups : p.Cu) * bw;
  for (int o = t; o < nout; o += 256) Rl[o] = 0.0;
  {
    // global reference norms: 256 / bw threads per column, eight loads in flight each
    const int per = 256 / bw, b = t % bw, k = t / bw;
    double acc = 0.0;
    if (k < per)
      for (int uu = k; uu < p.Cu; uu += 8 * per) {
        double v[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const int u2 = uu + q * per;
          const double x = p.Cn[(int64_t)(u2 < p.Cu ? u2 : p.Cu - 1) * bw + b];
          v[q] = u2 < p.Cu ? x : 0.0;
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) acc += v[q];
      }
    Sb[t] = acc;  // the coefficient buffer is free after the subtraction
  }
  __syncthreads();
  for (int b = t; b < bw; b += 256) {
    double s0 = 0.0;
    for (int k = 0; k < 256 / bw; ++k) s0 += Sb[k * bw + b];
    Rn[b] = sqrt(s0);
  }
  __syncthreads();
  if (p.comb_tree) {
    // 4b. the group factors (each in its group's first chunk slot of Rloc) stacked and
    // factored by one wave
    bulk_load(
        (int64_t)srows * bw,
        [&](int64_t e) -> double {
          const int gg = (int)(e / nout);
          return p.Rloc[(int64_t)gg * kTreeFan * nout + (e - (int64_t)gg * nout)];
        },
        [&](int64_t e, double v) { X[(e / bw) * ld + (e % bw)] = v; });
    __syncthreads();
    if (w == 0) cgs2_qr_team<1>(X, srows, ld, bw, Rl, Rn, p.dep_tol, Qsl);
    __syncthreads();
    // the group blocks of the second-level Q replace the group factors in Rloc;
    // k_tree_assemble multiplies them into the chunks' Q blocks
    for (int e = t; e < srows * bw; e += 256) {
      const int gg = e / nout, o = e - gg * nout;
      p.Rloc[(int64_t)gg * kTreeFan * nout + o] = X[(int64_t)(gg * bw + o / bw) * ld + (o % bw)];
    }
    __syncthreads();
  } else if (reg_comb) {
    // stacked chunk factors read straight from global memory into registers
    cgs2_dispatch<4>(p.Rloc, bw, Qs, bw, srows, bw, Rl, Rn, p.dep_tol, Qsl);
    __syncthreads();
  } else if (!p.comb_global) {
    bulk_load(
        (int64_t)srows * bw, [&](int64_t e) -> double { return p.Rloc[e]; },
        [&](int64_t e, double v) { X[(e / bw) * ld + (e % bw)] = v; });
    __syncthreads();
    cgs2_qr_team<4>(X, srows, ld, bw, Rl, Rn, p.dep_tol, Qsl);
    __syncthreads();
    for (int e = t; e < srows * bw; e += 256) Qs[e] = X[(e / bw) * ld + (e % bw)];
  } else {
    // stack too tall for LDS: QR in place in Qs (global); each row is copied and then
    // worked on by the one thread that owns it, so no fence is needed inside
    for (int r = t; r < srows; r += 256)
      for (int b = 0; b < bw; ++b) Qs[(int64_t)r * bw + b] = p.Rloc[(int64_t)r * bw + b];
    cgs2_qr_team<4>(Qs, srows, bw, bw, Rl, Rn, p.dep_tol, Qsl);
    __syncthreads();
  }
  double* Rout = p.Rf + (mode == MODE_INIT ? 2 : pass) * nout;
  for (int o = t; o < nout; o += 256) Rout[o] = Rl[o];
  if (mode == MODE_INIT && t == 0) p.cnt[2 * p.nbmax + 1] = 0u;
  if (arnoldi_mode(mode) && pass == 0) {
    // the loss of orthogonality of each column of Q1 = W' R1^{-1} to the basis is bounded
    // through R1^{-1} and the pre-projection norms (reorth_column_ok); when every column
    // passes, the second pass is skipped: V_{j+1} = Q1, H column = S1 and subdiagonal
    // block Rf1 (W = V S1 + Q1 Rf1 exactly)
    __shared__ int skip;
    if (w == 0) {
      bool ok = true;  // lane b: column b of Q1 orthogonal enough
      if (lane < bw) ok = reorth_column_ok(Rl, Rn, bw, lane, kReorthSkip, Sb + lane * 32);
      const bool all_ok = __all(ok);
      if (lane == 0) {
        skip = all_ok ? 1 : 0;
        p.cnt[2 * p.nbmax + 1] = (unsigned)skip;
      }
    }
    __syncthreads();
    if (skip) {
      const double* S1 = p.S;
      for (int e = t; e < nb * nout; e += 256) {
        const int i = e / nout, o = e - i * nout;
        p.H[(int64_t)(i * bw + o / bw) + p.ldH * (int64_t)(j * bw + o % bw)] = S1[e];
      }
      for (int o = t; o < nout; o += 256)
        p.H[(int64_t)(nb * bw + o / bw) + p.ldH * (int64_t)(j * bw + o % bw)] = Rl[o];
    }
  }
  if (hcol) {
    // W = V (S1 + S2 Rf1) + Q2 (Rf2 Rf1): the subdiagonal block of column block j
    const double* R1 = p.Rf;
    for (int o = t; o < nout; o += 256) {
      const int a = o / bw, b = o % bw;
      double v = 0.0;
      for (int k = 0; k < bw; ++k) v += Rl[a * bw + k] * R1[k * bw + b];
      p.H[(int64_t)(nb * bw + a) + p.ldH * (int64_t)(j * bw + b)] = v;
    }
  }
  if (t == 0) atomicExch(p.cnt + 2 * p.nbmax, 0u);
}

// V_j = Qloc2 . Qs2 committed to basis block j
template <typename TS>
__global__ void k_block_commit(const ProbDev* __restrict__ probs, int j) {
  const ProbDev p = probs[blockIdx.y];  // by value: uniform, loaded once
  if (!p.active) return;
  const int bw = p.bw;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= p.n * bw) return;
  const int64_t r = e / bw;
  const int col = (int)(e % bw);
  basis_ptr<TS>(p)[(int64_t)j * p.n * bw + e] = (TS)tsqr_entry(p, p.Qloc2, p.Qs2, r, col);
}

void init_block_kernels() {
  static bool done = false;
  if (done) return;
  // opt in to large dynamic LDS (gfx950 has 160 KiB per CU); a refusal leaves the 64 KiB
  // default, which the host-side geometry check then enforces
  const void* fns[4] = {(const void*)k_block_proj<double>, (const void*)k_block_proj<float>,
                        (const void*)k_block_update<double>, (const void*)k_block_update<float>};
  for (const void* f : fns)
    if (hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, kUpdateLdsMax) != hipSuccess)
      (void)hipGetLastError();
  done = true;
}

void launch_block_proj(ProbDev* d, int nprob, int grid_x, size_t smem, int j, int nb, int pass, int mode,
                       int mixed, hipStream_t st) {
  if (grid_x <= 0 || nprob <= 0 || nb <= 0) return;
  init_block_kernels();
  dim3 grid((unsigned)grid_x, (unsigned)nprob);
  if (mixed)
    hipLaunchKernelGGL(k_block_proj<float>, grid, dim3(256), smem, st, d, j, nb, pass, mode);
  else
    hipLaunchKernelGGL(k_block_proj<double>, grid, dim3(256), smem, st, d, j, nb, pass, mode);
}

// Two-level combine, last step: the Q block of chunk u becomes its group-level block
// times its group's block of the second-level Q (left in the group's first Rloc slot).
__global__ __launch_bounds__(256) void k_tree_assemble(const ProbDev* __restrict__ probs, int j, int pass, int mode) {
  const ProbDev p = probs[blockIdx.y];  // by value: uniform, loaded once
  if (!p.active || !p.comb_tree || (mode != MODE_INIT && j >= p.l)) return;
  if (arnoldi_mode(mode) && pass == 1 && p.cnt[2 * p.nbmax + 1]) return;  // second pass skipped
  const int u = blockIdx.x;
  if (u >= p.Cu) return;
  const int bw = p.bw, nout = bw * bw;
  double* Qs = (pass == 0 ? p.Qs1 : p.Qs2) + (int64_t)u * nout;
  const double* Q2 = p.Rloc + (int64_t)(u / kTreeFan) * kTreeFan * nout;
  __shared__ double qa[1024], qb[1024];
  for (int e = threadIdx.x; e < nout; e += 256) {
    qa[e] = Qs[e];
    qb[e] = Q2[e];
  }
  __syncthreads();
  for (int e = threadIdx.x; e < nout; e += 256) {
    const int r = e / bw, c = e - r * bw;
    double acc = 0.0;
    for (int k = 0; k < bw; ++k) acc += qa[r * bw + k] * qb[k * bw + c];
    Qs[e] = acc;
  }
}

void launch_block_update(ProbDev* d, int nprob, int grid_x, size_t smem, int j, int nb, int pass, int mode,
                         int mixed, int tree, hipStream_t st) {
  if (grid_x <= 0 || nprob <= 0) return;
  init_block_kernels();
  dim3 grid((unsigned)grid_x, (unsigned)nprob);
  if (mixed)
    hipLaunchKernelGGL(k_block_update<float>, grid, dim3(256), smem, st, d, j, nb, pass, mode);
  else
    hipLaunchKernelGGL(k_block_update<double>, grid, dim3(256), smem, st, d, j, nb, pass, mode);
  if (tree) hipLaunchKernelGGL(k_tree_assemble, grid, dim3(256), 0, st, d, j, pass, mode);
}

void launch_block_commit(ProbDev* d, int nprob, int grid_x, int j, int mixed, hipStream_t st) {
  if (grid_x <= 0 || nprob <= 0) return;
  dim3 grid((unsigned)grid_x, (unsigned)nprob);
  if (mixed)
    hipLaunchKernelGGL(k_block_commit<float>, grid, dim3(256), 0, st, d, j);
  else
    hipLaunchKernelGGL(k_block_commit<double>, grid, dim3(256), 0, st, d, j);
}

// ------------------------------------------------------------------------------------
// S6: exponential of the projected, source-augmented matrix
//   Ht = [[H_l, E_1 R0[:, :m] Pi], [0, kscale * D]],  b = [R0[:, m] (state) ; 0 ; w(tau)]
// Taylor polynomial of degree 16 (Paterson-Stockmeyer with A^2, A^3, A^4) on
// A = (delta / 2^s) Ht, then s squarings; y = exp(delta Ht) b.
// ------------------------------------------------------------------------------------
// Taylor coefficient z_j (entry idx = j m + a) of the piecewise-cubic source at offset
// pdelta into piece `piece`: z_j = sum_{k >= j} C(k, j) c_k pdelta^(k - j)
__device__ __forceinline__ double spline_z(const ExpmDev& e, int idx) {
  const int j = idx / e.m, a = idx - j * e.m;
  const double* c = e.Pw + (int64_t)e.piece * 4 * e.m + a;
  const double d = e.pdelta;
  const double c0 = c[0], c1 = c[e.m], c2 = c[2 * e.m], c3 = c[3 * e.m];
  switch (j) {
    case 0: return c0 + d * (c1 + d * (c2 + d * c3));
    case 1: return c1 + d * (2.0 * c2 + 3.0 * d * c3);
    case 2: return c2 + 3.0 * d * c3;
    default: return c3;
  }
}

__global__ void k_build_aug(const ExpmDev* __restrict__ E) {
  const ExpmDev e = E[blockIdx.y];  // by value: uniform, loaded once
  if (!e.active) return;
  const int N = e.N;
  const int64_t NN = (int64_t)N * N;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int lbw = e.lbw, bw = e.bw;
  if (idx < NN) {
    const int r = (int)(idx % N), c = (int)(idx / N);
    double v = 0.0;
    if (r < lbw && c < lbw) {
      if (e.sai)  // shift-and-invert: H_L = (I - K^{-1}) / gamma
        v = ((r == c ? 1.0 : 0.0) - e.Kinv[(int64_t)r + (int64_t)lbw * c]) / e.gamma;
      // block upper Hessenberg: blocks below the subdiagonal are zero (never written)
      else if (r / bw <= c / bw + 1)
        v = e.H[(int64_t)r + e.ldH * c];
    } else if (r < bw && c >= lbw) {
      const int k = c - lbw;
      if (e.spline)  // the source U z_0 in Krylov coordinates: E_1 R0[:, :m]
        v = k < e.m ? e.R0[r * bw + k] : 0.0;
      else
        for (int cc = 0; cc < e.m; ++cc) v += e.R0[r * bw + cc] * e.Pi[cc + (int64_t)e.ldPi * k];
    } else if (r >= lbw && c >= lbw) {
      if (e.spline) {  // z_j' = (j + 1) z_{j+1}, blocks of m
        const int rr = r - lbw, cc = c - lbw;
        v = (cc == rr + e.m && rr < 3 * e.m) ? (double)(rr / e.m + 1) : 0.0;
      } else {
        v = e.kscale * e.Dm[(r - lbw) * e.qmax + (c - lbw)];
      }
    }
    e.Ht[idx] = v;
  }
  if (idx < N) {
    const int r = (int)idx;
    double v = 0.0;
    if (r < bw) v = e.with_x ? e.R0[r * bw + e.m] : 0.0;
    else if (r >= lbw) v = e.spline ? spline_z(e, r - lbw) : e.w[r - lbw];
    e.b[r] = v;
  }
}

// piecewise source: the z part of the held solution ycur restarts from the Taylor
// coefficients of the current piece at the current time (problems with zreset set)
__global__ void k_spline_reset(const ExpmDev* __restrict__ E) {
  const ExpmDev e = E[blockIdx.y];  // by value: uniform, loaded once
  if (!e.zreset) return;
  for (int i = threadIdx.x; i < 4 * e.m; i += blockDim.x) e.ycur[e.lbw + i] = spline_z(e, i);
}

void launch_spline_reset(ExpmDev* e, int nprob, hipStream_t st) {
  hipLaunchKernelGGL(k_spline_reset, dim3(1, (unsigned)nprob), dim3(128), 0, st, e);
}

void launch_build_aug(ExpmDev* e, int nprob, int64_t maxNN, hipStream_t st) {
  dim3 grid((unsigned)((maxNN + 255) / 256), (unsigned)nprob);
  hipLaunchKernelGGL(k_build_aug, grid, dim3(256), 0, st, e);
}

// out[p] = ||Ht||_1 (largest absolute column sum); one wave per column, grid over column
// groups; non-negative doubles order like their bit patterns, so the maximum is an
// integer atomic max (out[] zeroed by the host)
__global__ __launch_bounds__(256) void k_norm1(const ExpmDev* __restrict__ E, double* out) {
  const ExpmDev e = E[blockIdx.y];  // by value: uniform, loaded once
  if (!e.active) return;
  const int N = e.N;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int c = blockIdx.x * 4 + w;
  if (c >= N) return;
  double s = 0.0;
  for (int r = lane; r < N; r += 64) s += fabs(e.Ht[(int64_t)r + (int64_t)N * c]);
  s = wave_sum(s);
  if (lane == 0) atomicMax((unsigned long long*)(out + blockIdx.y), (unsigned long long)__double_as_longlong(s));
}

void launch_norm1(ExpmDev* e, double* out, int nprob, int maxN, hipStream_t st) {
  hipLaunchKernelGGL(k_norm1, dim3((unsigned)((maxN + 3) / 4), (unsigned)nprob), dim3(256), 0, st, e, out);
}

__device__ __constant__ double c_taylor[17] = {
    1.0, 1.0, 1.0 / 2, 1.0 / 6, 1.0 / 24, 1.0 / 120, 1.0 / 720, 1.0 / 5040, 1.0 / 40320, 1.0 / 362880,
    1.0 / 3628800, 1.0 / 39916800, 1.0 / 479001600, 1.0 / 6227020800.0, 1.0 / 87178291200.0,
    1.0 / 1307674368000.0, 1.0 / 20922789888000.0};

// A = alpha Ht (op 0) or P = c16 A4 + c15 A3 + c14 A2 + c13 A + c12 I (op 1)
__global__ void k_elementwise(const ExpmDev* __restrict__ E, int op) {
  const ExpmDev e = E[blockIdx.y];  // by value: uniform, loaded once
  if (!e.active || e.prop) return;
  const int N = e.N;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)N * N) return;
  if (op == 0) {
    e.A[idx] = e.alpha * e.Ht[idx];
  } else {
    const int r = (int)(idx % N), c = (int)(idx / N);
    e.P[idx] = c_taylor[16] * e.A4[idx] + c_taylor[15] * e.A3[idx] + c_taylor[14] * e.A2[idx] +
               c_taylor[13] * e.A[idx] + (r == c ? c_taylor[12] : 0.0);
  }
}

void launch_elementwise(ExpmDev* e, int op, int nprob, int64_t maxNN, hipStream_t st) {
  dim3 grid((unsigned)((maxNN + 255) / 256), (unsigned)nprob);
  hipLaunchKernelGGL(k_elementwise, grid, dim3(256), 0, st, e, op);
}


// C = A B (+ Taylor epilogue), 32 x 32 tile per workgroup, 4 waves of 16 x 16 MFMA f64.
//   op 0: A2 = A A      op 1: A3 = A2 A      op 2: A4 = A2 A2
//   op 3: T = P A4 + c11 A3 + c10 A2 + c9 A + c8 I
//   op 4: P = T A4 + c7 A3 + c6 A2 + c5 A + c4 I
//   op 5: T = P A4 + c3 A3 + c2 A2 + c1 A + c0 I
//   op 6: squaring number k: (k even) P = T T, (k odd) T = P P; skipped when k >= nsq
constexpr int kGemmPf = 4;  // k-steps of fragment loads in flight per wave
__global__ __launch_bounds__(256) void k_gemm(const ExpmDev* __restrict__ E, int op, int k) {
  const ExpmDev e = E[blockIdx.y];  // by value: uniform, loaded once
  if (!e.active || e.prop) return;
  if (op == 6 && k >= e.nsq) return;
  const int N = e.N;
  const int nt = (N + 31) / 32;
  const int tile = blockIdx.x;
  if (tile >= nt * nt) return;
  const int i0 = 32 * (tile % nt), j0 = 32 * (tile / nt);
  const double *A, *B;
  double* C;
  int ep = -1;  // epilogue base index (c[ep+3] A3 + c[ep+2] A2 + c[ep+1] A + c[ep] I)
  switch (op) {
    case 0: A = e.A; B = e.A; C = e.A2; break;
    case 1: A = e.A2; B = e.A; C = e.A3; break;
    case 2: A = e.A2; B = e.A2; C = e.A4; break;
    case 3: A = e.P; B = e.A4; C = e.T; ep = 8; break;
    case 4: A = e.T; B = e.A4; C = e.P; ep = 4; break;
    case 5: A = e.P; B = e.A4; C = e.T; ep = 0; break;
    default:
      if (k & 1) { A = e.P; B = e.P; C = e.T; }
      else { A = e.T; B = e.T; C = e.P; }
      break;
  }
  // Every wave computes the whole 32 x 32 tile over the k-steps (of 4) w, w + 4, ...:
  // four 16 x 16 f64 MFMA accumulators, fragments loaded straight from memory (the
  // matrices are L2-resident) with kGemmPf k-steps in flight and no barrier in the loop.
  // The four partial tiles are then summed through LDS, wave w finishing 16 x 16 block w.
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int nks = (N + 3) / 4;
  const int r0 = i0 + li, r1 = i0 + 16 + li, c0 = j0 + li, c1 = j0 + 16 + li;
  const bool r0ok = r0 < N, r1ok = r1 < N, c0ok = c0 < N, c1ok = c1 < N;
  const double* pa0 = A + (r0ok ? r0 : N - 1);  // clamped: every load is in bounds
  const double* pa1 = A + (r1ok ? r1 : N - 1);
  const double* pb0 = B + (int64_t)N * (c0ok ? c0 : N - 1);
  const double* pb1 = B + (int64_t)N * (c1ok ? c1 : N - 1);
  dbl4 acc[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) acc[q] = dbl4{0.0, 0.0, 0.0, 0.0};
  for (int ks0 = w; ks0 < nks; ks0 += 4 * kGemmPf) {
    double a0[kGemmPf], a1[kGemmPf], b0[kGemmPf], b1[kGemmPf];
#pragma unroll
    for (int f = 0; f < kGemmPf; ++f) {
      const int kq = 4 * (ks0 + 4 * f) + lk;
      const bool kok = kq < N;
      const int64_t kc = kok ? kq : N - 1;
      const double x0 = pa0[(int64_t)N * kc], x1 = pa1[(int64_t)N * kc];
      const double y0 = pb0[kc], y1 = pb1[kc];
      a0[f] = (kok && r0ok) ? x0 : 0.0;
      a1[f] = (kok && r1ok) ? x1 : 0.0;
      b0[f] = (kok && c0ok) ? y0 : 0.0;
      b1[f] = (kok && c1ok) ? y1 : 0.0;
    }
#pragma unroll
    for (int f = 0; f < kGemmPf; ++f) {
      acc[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0[f], b0[f], acc[0], 0, 0, 0);
      acc[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0[f], b1[f], acc[1], 0, 0, 0);
      acc[2] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1[f], b0[f], acc[2], 0, 0, 0);
      acc[3] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1[f], b1[f], acc[3], 0, 0, 0);
    }
  }
  // red[src wave][block][v * 64 + lane]: every wave holds the same fragment layout
  __shared__ double red[4][4][256];
#pragma unroll
  for (int q = 0; q < 4; ++q)
    if (q != w)
#pragma unroll
      for (int v = 0; v < 4; ++v) red[w][q][v * 64 + lane] = acc[q][v];
  __syncthreads();
  dbl4 sum = acc[0];
#pragma unroll
  for (int q = 1; q < 4; ++q)
    if (q == w) sum = acc[q];  // compile-time register indices: select, no run-time index
#pragma unroll
  for (int q = 0; q < 4; ++q)
    if (q != w)
#pragma unroll
      for (int v = 0; v < 4; ++v) sum[v] += red[q][w][v * 64 + lane];
  const int bi = w >> 1, bj = w & 1;  // block w: rows 16 bi.., columns 16 bj..
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    // accumulator layout of the f64 16x16x4 MFMA: row = lane/16 + 4 v, column = lane % 16
    const int i = i0 + bi * 16 + lk + 4 * v;
    const int j = j0 + bj * 16 + li;
    if (i < N && j < N) {
      const int64_t o = (int64_t)i + (int64_t)N * j;
      double val = sum[v];
      if (ep >= 0)
        val += c_taylor[ep + 3] * e.A3[o] + c_taylor[ep + 2] * e.A2[o] + c_taylor[ep + 1] * e.A[o] +
               (i == j ? c_taylor[ep] : 0.0);
      C[o] = val;
    }
  }
}

void launch_gemm(ExpmDev* e, int op, int k, int nprob, int tiles_max, hipStream_t st) {
  dim3 grid((unsigned)tiles_max, (unsigned)nprob);
  hipLaunchKernelGGL(k_gemm, grid, dim3(256), 0, st, e, op, k);
}

// y_k = exp(alpha 2^k Ht) b after k squarings (T for even k, P for odd k); rows spread
// over workgroups.  Problems with fewer squarings than k skip.  A propagation pass
// (prop = 1) forms y_0 = Eprop ycur.
// A workgroup takes 64 rows; its 16 column groups (of 64 lanes each, one row per lane)
// sum strided columns with eight loads in flight and reduce through LDS.
constexpr int kApplySplit = 16;
__global__ __launch_bounds__(1024) void k_expm_apply(const ExpmDev* __restrict__ E, int level) {
  const ExpmDev e = E[blockIdx.y];  // by value: uniform, loaded once
  if (!e.active || level > e.nsq) return;
  const int N = e.N;
  const int lane = threadIdx.x & 63, cs = threadIdx.x >> 6;
  const int r0 = blockIdx.x * 64;
  if (r0 >= N) return;
  const int r = r0 + lane;
  __shared__ double red[kApplySplit * 64];
  const double* M = e.prop ? e.Eprop : (level & 1) ? e.P : e.T;
  const double* bvec = e.prop ? e.ycur : e.b;
  double acc = 0.0;
  if (r < N)
    for (int c = cs; c < N; c += 8 * kApplySplit) {
      double v[8], bb[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const int c2 = c + k * kApplySplit;
        const int cc = c2 < N ? c2 : N - 1;
        const double mv = M[(int64_t)r + (int64_t)N * cc], bv = bvec[cc];
        v[k] = c2 < N ? mv : 0.0;
        bb[k] = c2 < N ? bv : 0.0;
      }
#pragma unroll
      for (int k = 0; k < 8; ++k) acc += v[k] * bb[k];
    }
  red[cs * 64 + lane] = acc;
  __syncthreads();
  if (cs == 0 && r < N) {
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < kApplySplit; ++k) s += red[k * 64 + lane];
    e.y[(int64_t)level * N + r] = s;
  }
}

// out[2k] = residual norm of the Krylov solution at the end of the step of level k,
// out[2k+1] = |y_k[0 : l bw]|.  Polynomial Krylov: |H_{l+1,l} y_k[(l-1)bw : l bw]|.
// Shift-and-invert: |(I - gamma L) V_{l+1} K_{l+1,l} E_l^T K^{-1} y_k| / gamma, with
// E_l^T K^{-1} y = E_l^T (I - gamma H_L) y and the norm from the Gram GW.
__global__ __launch_bounds__(256) void k_expm_resid(const ExpmDev* __restrict__ E, int level) {
  const ExpmDev e = E[blockIdx.x];  // by value: uniform, loaded once
  if (!e.active || level > e.nsq) return;
  __shared__ double red[16];
  __shared__ double zs[32];
  const double* y = e.y + (int64_t)level * e.N;
  double yn = 0.0;
  for (int r = threadIdx.x; r < e.lbw; r += blockDim.x) yn += y[r] * y[r];
  yn = block_sum(yn, red);
  double rr = 0.0;
  const int bw = e.bw, l = e.l;
  if (e.sai) {
    // z = E_l^T (I - gamma H_L) y (one wave per row), c = K_{l+1,l} z, |r|^2 = c^T GW c
    const int lbw = e.lbw, N = e.N, lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __shared__ double cvs[32];
    for (int a = w; a < bw; a += 4) {
      double sa = 0.0;
      for (int c = lane; c < lbw; c += 64) sa += e.Ht[(int64_t)(lbw - bw + a) + (int64_t)N * c] * y[c];
      sa = wave_sum(sa);
      if (lane == 0) zs[a] = y[lbw - bw + a] - e.gamma * sa;
    }
    __syncthreads();
    if ((int)threadIdx.x < bw) {
      const int a = threadIdx.x;
      double acc = 0.0;
      for (int b = 0; b < bw; ++b) acc += e.H[(int64_t)(l * bw + a) + e.ldH * (int64_t)((l - 1) * bw + b)] * zs[b];
      cvs[a] = acc;
    }
    __syncthreads();
    double q = 0.0;
    if ((int)threadIdx.x < bw) {
      const int a = threadIdx.x;
      double acc = 0.0;
      for (int b = 0; b < bw; ++b) acc += e.GW[a * bw + b] * cvs[b];
      q = cvs[a] * acc;
    }
    q = block_sum(q, red);
    if (threadIdx.x == 0) {
      e.out[2 * level] = sqrt(fmax(q, 0.0)) / e.gamma;
      e.out[2 * level + 1] = sqrt(yn);
    }
    return;
  }
  if ((int)threadIdx.x < bw) {
    const int a = threadIdx.x;
    double sacc = 0.0;
    for (int c = 0; c < bw; ++c)
      sacc += e.H[(int64_t)(l * bw + a) + e.ldH * (int64_t)((l - 1) * bw + c)] * y[(l - 1) * bw + c];
    rr = sacc * sacc;
  }
  rr = block_sum(rr, red);
  if (threadIdx.x == 0) {
    e.out[2 * level] = sqrt(rr);
    e.out[2 * level + 1] = sqrt(yn);
  }
}

void launch_expm_apply(ExpmDev* e, int level, int nprob, int maxN, hipStream_t st) {
  hipLaunchKernelGGL(k_expm_apply, dim3((unsigned)((maxN + 63) / 64), (unsigned)nprob), dim3(64 * kApplySplit), 0,
                     st, e, level);
  hipLaunchKernelGGL(k_expm_resid, dim3((unsigned)nprob), dim3(256), 0, st, e, level);
}

// ------------------------------------------------------------------------------------
// S7: x = V_{0..l-1} y[0:l*bw]  (and the output column)
// ------------------------------------------------------------------------------------
template <typename TS>
__global__ __launch_bounds__(256) void k_project(const ProbDev* __restrict__ probs, const ExpmDev* __restrict__ E) {
  const ProbDev p = probs[blockIdx.y];  // by value: uniform, loaded once
  if (!p.active || !p.proj) return;
  (void)E;
  extern __shared__ double ys[];
  const int lbw = p.l * p.bw;
  for (int c = threadIdx.x; c < lbw; c += blockDim.x) ys[c] = p.yacc[c];
  __syncthreads();
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= p.n) return;
  const int bw = p.bw;
  const TS* V = basis_ptr<TS>(p);
  const int64_t blk = p.n * bw;
  double acc = 0.0;
  // block 0 (the orthonormalised [U | x]) carries most of the state: with fp32 storage
  // it is read from its fp64 copy, so short steps do not re-round the state
  if (!std::is_same<TS, double>::value) {
    const double* row = p.V + r * bw;
    for (int c = 0; c < bw; ++c) acc += row[c] * ys[c];
  }
  for (int i = std::is_same<TS, double>::value ? 0 : 1; i < p.l; ++i) {
    const TS* row = V + (int64_t)i * blk + r * bw;
    for (int c = 0; c < bw; ++c) acc += (double)row[c] * ys[i * bw + c];
  }
  p.xstate[r] = acc;
  if (p.outcol) p.outcol[r] = acc;
}

void launch_project(ProbDev* d, ExpmDev* e, int nprob, int64_t maxn, int max_lbw, int mixed, hipStream_t st) {
  dim3 grid((unsigned)((maxn + 255) / 256), (unsigned)nprob);
  size_t smem = sizeof(double) * (size_t)max_lbw + 16;
  if (mixed)
    hipLaunchKernelGGL(k_project<float>, grid, dim3(256), smem, st, d, e);
  else
    hipLaunchKernelGGL(k_project<double>, grid, dim3(256), smem, st, d, e);
}

// ------------------------------------------------------------------------------------
// Compression (S3, S4): singular values of the QR factor R of the samples, left vectors,
// truncation is decided on the host, then U = Q W_m and the Chebyshev fit of C.
// ------------------------------------------------------------------------------------
__global__ void k_row_norms(const double* R, int64_t ldR, int rows, int cols, double* rn) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= rows) return;
  double s = 0.0;
  for (int c = 0; c < cols; ++c) {
    const double v = R[(int64_t)i + ldR * c];
    s += v * v;
  }
  rn[i] = sqrt(s);
}

void launch_row_norms(const double* R, int64_t ldR, int rows, int cols, double* rn, hipStream_t st) {
  hipLaunchKernelGGL(k_row_norms, dim3((unsigned)((rows + 255) / 256)), dim3(256), 0, st, R, ldR, rows, cols, rn);
}

// out = |x|_2 of a vector of n entries, one workgroup (fixed summation order)
__global__ __launch_bounds__(1024) void k_vec_norm(const double* __restrict__ x, int64_t n, double* out) {
  __shared__ double red[16];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) s += x[i] * x[i];
  s = block_sum(s, red);
  if (threadIdx.x == 0) *out = sqrt(s);
}

// deterministic pseudo-random fill in [-1/2, 1/2) (splitmix64 of the index), for tuning runs
__global__ void k_fill_hash(double* x, int64_t n, uint64_t seed) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint64_t z = (uint64_t)i + seed * 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  z ^= z >> 31;
  x[i] = (double)(z >> 11) * (1.0 / 9007199254740992.0) - 0.5;
}

void launch_fill_hash(double* x, int64_t n, uint64_t seed, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill_hash, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, x, n, seed);
}

void launch_vec_norm(const double* x, int64_t n, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_vec_norm, dim3(1), dim3(1024), 0, st, x, n, out);
}

// One-sided (Hestenes) Jacobi on A = R[sel, 0:s]^T (s x r): A J has orthogonal columns.
// Singular values are the column norms; J (r x r, column-major) holds the left singular
// vectors of R[sel, :].  Round-robin ordering, one wave per pair, one workgroup.
__global__ __launch_bounds__(256) void k_jacobi_svd(const double* R, int64_t ldR, const int* sel, int s, int r,
                                                    double* A, double* J, double* sig, int* perm, int* info) {
  __shared__ double red[16];
  __shared__ double wmax[4];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  for (int64_t e = t; e < (int64_t)s * r; e += blockDim.x) {
    const int k = (int)(e % s), i = (int)(e / s);
    A[e] = R[(int64_t)sel[i] + ldR * k];
  }
  for (int64_t e = t; e < (int64_t)r * r; e += blockDim.x) J[e] = ((e % r) == (e / r)) ? 1.0 : 0.0;
  __syncthreads();
  // A pair counts as orthogonal when its coupling is below tol times the geometric mean
  // of the two squared norms, tol = sqrt(s) eps (the one-sided Jacobi test of Demmel and
  // Veselic, as in LAPACK's dgesvj).  A test relative to each pair keeps the small
  // singular values accurate; the rows passed in are the non-deflated rows of R.
  const double tol = sqrt((double)s) * 2.220446049250313e-16;
  const int r2 = r + (r & 1);
  int sweep = 0;
  for (; sweep < 30 && r > 1; ++sweep) {
    double off = 0.0;
    for (int round = 0; round < r2 - 1; ++round) {
      for (int pi = w; pi < r2 / 2; pi += 4) {
        int pp, qq;
        if (pi == 0) {
          pp = 0;
          qq = (round % (r2 - 1)) + 1;
        } else {
          pp = ((round + pi) % (r2 - 1)) + 1;
          qq = ((round - pi + r2 - 1) % (r2 - 1)) + 1;
        }
        if (pp >= r || qq >= r) continue;
        double* ap = A + (int64_t)pp * s;
        double* aq = A + (int64_t)qq * s;
        double al = 0.0, be = 0.0, ga = 0.0;
        for (int k = lane; k < s; k += 64) {
          al += ap[k] * ap[k];
          be += aq[k] * aq[k];
          ga += ap[k] * aq[k];
        }
        al = wave_sum(al);
        be = wave_sum(be);
        ga = wave_sum(ga);
        if (ga == 0.0 || al == 0.0 || be == 0.0) continue;
        const double rel = fabs(ga) / sqrt(al * be);
        off = fmax(off, rel);
        if (rel <= tol) continue;
        const double zeta = (be - al) / (2.0 * ga);
        const double tt = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        const double cs = 1.0 / sqrt(1.0 + tt * tt), sn = cs * tt;
        for (int k = lane; k < s; k += 64) {
          const double x = ap[k], y = aq[k];
          ap[k] = cs * x - sn * y;
          aq[k] = sn * x + cs * y;
        }
        double* jp = J + (int64_t)pp * r;
        double* jq = J + (int64_t)qq * r;
        for (int k = lane; k < r; k += 64) {
          const double x = jp[k], y = jq[k];
          jp[k] = cs * x - sn * y;
          jq[k] = sn * x + cs * y;
        }
      }
      __threadfence_block();
      __syncthreads();
    }
    if (lane == 0) wmax[w] = off;
    __syncthreads();
    const double o = fmax(fmax(wmax[0], wmax[1]), fmax(wmax[2], wmax[3]));
    __syncthreads();
    if (o <= tol) {
      ++sweep;
      break;
    }
  }
  for (int i = w; i < r; i += 4) {
    double q = 0.0;
    for (int k = lane; k < s; k += 64) q += A[(int64_t)i * s + k] * A[(int64_t)i * s + k];
    q = wave_sum(q);
    if (lane == 0) sig[i] = sqrt(q);
  }
  __threadfence_block();
  __syncthreads();
  if (t == 0) {
    for (int i = 0; i < r; ++i) perm[i] = i;
    for (int i = 0; i < r; ++i) {  // selection sort, descending
      int b = i;
      for (int k = i + 1; k < r; ++k)
        if (sig[perm[k]] > sig[perm[b]]) b = k;
      const int tmp = perm[i];
      perm[i] = perm[b];
      perm[b] = tmp;
    }
    info[0] = sweep;
  }
}

void launch_jacobi_svd(const double* R, int64_t ldR, const int* sel, int s, int r, double* A, double* J,
                       double* sig, int* perm, int* info, hipStream_t st) {
  hipLaunchKernelGGL(k_jacobi_svd, dim3(1), dim3(256), 0, st, R, ldR, sel, s, r, A, J, sig, perm, info);
}

// U[:, k] = sum_i Q[:, sel_i] J[i, perm_k], Q stored as blocks of n x bwc (row-major)
__global__ void k_form_u(const double* Q, int bwc, int64_t n, const int* sel, int r, const double* J,
                         const int* perm, int m, double* U, int64_t ldU) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  for (int k = 0; k < m; ++k) {
    const double* jc = J + (int64_t)perm[k] * r;
    double acc = 0.0;
    for (int i = 0; i < r; ++i) {
      const int col = sel[i];
      acc += Q[(int64_t)(col / bwc) * n * bwc + g * bwc + (col % bwc)] * jc[i];
    }
    U[g + ldU * k] = acc;
  }
}

void launch_form_u(const double* Q, int bwc, int64_t n, const int* sel, int r, const double* J, const int* perm,
                   int m, double* U, int64_t ldU, hipStream_t st) {
  hipLaunchKernelGGL(k_form_u, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, Q, bwc, n, sel, r, J, perm, m,
                     U, ldU);
}

// Least-squares Chebyshev fit of the rows of C = (A J)[:, perm[0:m]]^T over the samples:
// smallest q with relative residual <= fit_tol (q <= qcap); Pi (m x q, column-major).
// work: qcap*s + qcap*qcap + m*qcap + m*s doubles.  info: [q, residual, capped].
__global__ __launch_bounds__(256) void k_fit(const double* A, int s, const int* perm, int m, const double* ts,
                                             double t0, double t1, int qcap, double fit_tol, double* Pi, int ldPi,
                                             double* work, double* info) {
  __shared__ double red[16];
  __shared__ int qsel_s;
  __shared__ double res_s;
  const int t = threadIdx.x;
  double* Tq = work;                              // s x qcap row-major
  double* Rt = Tq + (int64_t)s * qcap;            // qcap x qcap
  double* Ch = Rt + (int64_t)qcap * qcap;         // m x qcap
  double* Em = Ch + (int64_t)m * qcap;            // m x s
  double cn = 0.0;
  for (int64_t e = t; e < (int64_t)m * s; e += blockDim.x) {
    const int a = (int)(e / s), i = (int)(e % s);
    const double v = A[(int64_t)perm[a] * s + i];
    Em[e] = v;
    cn += v * v;
  }
  cn = sqrt(block_sum(cn, red));
  for (int i = t; i < s; i += blockDim.x) {
    const double x = (2.0 * ts[i] - t0 - t1) / (t1 - t0);
    double a = 1.0, b = x;
    for (int k = 0; k < qcap; ++k) {
      double v;
      if (k == 0) v = 1.0;
      else if (k == 1) v = x;
      else {
        v = 2.0 * x * b - a;
        a = b;
        b = v;
      }
      Tq[(int64_t)i * qcap + k] = v;
    }
  }
  for (int e = t; e < qcap * qcap; e += blockDim.x) Rt[e] = 0.0;
  __threadfence_block();
  __syncthreads();
  mgs2_qr_block(Tq, s, qcap, qcap, Rt, 1e-12, red);
  __threadfence_block();
  __syncthreads();
  for (int e = t; e < m * qcap; e += blockDim.x) {
    const int a = e / qcap, k = e % qcap;
    double acc = 0.0;
    for (int i = 0; i < s; ++i) acc += Em[(int64_t)a * s + i] * Tq[(int64_t)i * qcap + k];
    Ch[e] = acc;
  }
  __threadfence_block();
  __syncthreads();
  int qsel = qcap;
  double res = 0.0;
  for (int q = 1; q <= qcap; ++q) {
    double ss = 0.0;
    for (int64_t e = t; e < (int64_t)m * s; e += blockDim.x) {
      const int a = (int)(e / s), i = (int)(e % s);
      const double v = Em[e] - Ch[a * qcap + q - 1] * Tq[(int64_t)i * qcap + q - 1];
      Em[e] = v;
      ss += v * v;
    }
    res = cn > 0.0 ? sqrt(block_sum(ss, red)) / cn : 0.0;
    if (res <= fit_tol) {
      qsel = q;
      break;
    }
  }
  if (t == 0) {
    qsel_s = qsel;
    res_s = res;
  }
  __syncthreads();
  qsel = qsel_s;
  for (int a = t; a < m; a += blockDim.x) {
    for (int k = qsel - 1; k >= 0; --k) {
      double v = Ch[a * qcap + k];
      for (int kk = k + 1; kk < qsel; ++kk) v -= Rt[k * qcap + kk] * Pi[a + (int64_t)ldPi * kk];
      const double d = Rt[k * qcap + k];
      Pi[a + (int64_t)ldPi * k] = d != 0.0 ? v / d : 0.0;
    }
  }
  if (t == 0) {
    info[0] = (double)qsel;
    info[1] = res_s;
    info[2] = (res_s > fit_tol) ? 1.0 : 0.0;
  }
}

void launch_fit(const double* A, int s, const int* perm, int m, const double* ts, double t0, double t1, int qcap,
                double fit_tol, double* Pi, int ldPi, double* work, double* info, hipStream_t st) {
  hipLaunchKernelGGL(k_fit, dim3(1), dim3(256), 0, st, A, s, perm, m, ts, t0, t1, qcap, fit_tol, Pi, ldPi, work,
                     info);
}

// S4, piecewise: the not-a-knot cubic spline through each coefficient row (one thread per
// row).  Unknowns are the second derivatives M_i at the samples; the not-a-knot
// conditions (third derivative continuous at the second and the second-to-last sample)
// give M_0 = (1 + h0/h1) M_1 - (h0/h1) M_2 and the mirror for M_{s-1}, which turn the
// first and last interior continuity equations into rows of a diagonally dominant
// tridiagonal system for M_1..M_{s-2}, solved by elimination without pivoting.  Three
// samples give one parabola, two a straight line.  Output: Pw[(i 4 + k) m + a] = c_k of
// piece i of row a, p(t) = sum_k c_k (t - t_i)^k on [t_i, t_{i+1}].
// work: 3 s doubles per row.
__global__ void k_spline(const double* A, int s, const int* perm, int m, const double* ts, double* Pw,
                         double* work) {
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= m) return;
  const double* y = A + (int64_t)perm[a] * s;
  double* M = work + (int64_t)a * 3 * s;
  double* cp = M + s;  // eliminated super-diagonal
  double* dp = cp + s; // eliminated right-hand side
  auto hh = [&](int i) { return ts[i + 1] - ts[i]; };
  auto slope = [&](int i) { return (y[i + 1] - y[i]) / hh(i); };
  for (int i = 0; i < s; ++i) M[i] = 0.0;
  if (s == 3) {
    const double dd = (slope(1) - slope(0)) / (ts[2] - ts[0]);
    M[0] = M[1] = M[2] = 2.0 * dd;
  } else if (s >= 4) {
    // rows i = 1..s-2 of the reduced system: sub[i] M_{i-1} + dia[i] M_i + sup[i] M_{i+1} = rhs[i]
    for (int i = 1; i <= s - 2; ++i) {
      const double h0 = hh(i - 1), h1 = hh(i);
      double sub = h0, dia = 2.0 * (h0 + h1), sup = h1;
      const double rhs = 6.0 * (slope(i) - slope(i - 1));
      if (i == 1) {  // M_0 eliminated
        dia += h0 + h0 * h0 / h1;
        sup -= h0 * h0 / h1;
        sub = 0.0;
      }
      if (i == s - 2) {  // M_{s-1} eliminated
        dia += h1 + h1 * h1 / h0;
        sub -= h1 * h1 / h0;
        sup = 0.0;
      }
      if (i == 1) {
        cp[i] = sup / dia;
        dp[i] = rhs / dia;
      } else {
        const double den = dia - sub * cp[i - 1];
        cp[i] = sup / den;
        dp[i] = (rhs - sub * dp[i - 1]) / den;
      }
    }
    M[s - 2] = dp[s - 2];
    for (int i = s - 3; i >= 1; --i) M[i] = dp[i] - cp[i] * M[i + 1];
    const double g0 = hh(0) / hh(1), g1 = hh(s - 2) / hh(s - 3);
    M[0] = (1.0 + g0) * M[1] - g0 * M[2];
    M[s - 1] = (1.0 + g1) * M[s - 2] - g1 * M[s - 3];
  }
  for (int i = 0; i + 1 < s; ++i) {
    const double h = hh(i);
    double* c = Pw + (int64_t)i * 4 * m + a;
    c[0] = y[i];
    c[m] = slope(i) - h * (2.0 * M[i] + M[i + 1]) / 6.0;
    c[2 * m] = 0.5 * M[i];
    c[3 * m] = (M[i + 1] - M[i]) / (6.0 * h);
  }
}

void launch_spline(const double* A, int s, const int* perm, int m, const double* ts, double* Pw, double* work,
                   hipStream_t st) {
  if (m <= 0 || s < 2) return;
  hipLaunchKernelGGL(k_spline, dim3(1), dim3(64), 0, st, A, s, perm, m, ts, Pw, work);
}

// ------------------------------------------------------------------------------------
// S8 and utilities
// ------------------------------------------------------------------------------------
struct PtrList {
  const double* v[64];
};

__global__ void k_superpose(const double* u0, PtrList vl, int P, int64_t n, int64_t ldv, double* u, int64_t ldu,
                            int accumulate) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int k = blockIdx.y;
  if (r >= n) return;
  double acc = accumulate ? u[r + ldu * k] : u0[r];
  for (int j = 0; j < P; ++j) acc += vl.v[j][r + ldv * k];
  u[r + ldu * k] = acc;
}

void launch_superpose(const double* u0, const double* const* v, int P, int64_t n, int n_out, int64_t ldv, double* u,
                      int64_t ldu, hipStream_t st) {
  dim3 grid((unsigned)((n + 255) / 256), (unsigned)n_out);
  if (P == 0) {  // u = u0 in every column
    PtrList pl;
    hipLaunchKernelGGL(k_superpose, grid, dim3(256), 0, st, u0, pl, 0, n, ldv, u, ldu, 0);
    return;
  }
  for (int j0 = 0; j0 < P; j0 += 64) {
    PtrList pl;
    const int cnt = (P - j0) < 64 ? (P - j0) : 64;
    for (int i = 0; i < cnt; ++i) pl.v[i] = v[j0 + i];
    hipLaunchKernelGGL(k_superpose, grid, dim3(256), 0, st, u0, pl, cnt, n, ldv, u, ldu, j0 > 0 ? 1 : 0);
  }
}

// ------------------------------------------------------------------------------------
// S10: waveform-relaxation sources for viscous Burgers on one window.
// For iterate u_k at the window's s samples (n x s, ld n):
//   Jbar = sum_i w_i dN/du(u_k(t_i)), stencil rows [u/(2h), -(u_{+}-u_{-})/(2h), -u/(2h)]
//   coef = nu D2 + Jbar (per-point stencil, rows c_minus, c_zero, c_plus)
//   G[:, i] = N(u_k(t_i)) - Jbar u_k(t_i),  N(u) = -u (u_{+} - u_{-}) / (2h)
// with trapezoid weights w (end weight w_end, interior w_in).  Without the Jacobian
// Jbar = 0 (Picard iteration).  One thread per grid point.
// ------------------------------------------------------------------------------------
__global__ void k_wr_source(int64_t n, int s, double h, double nu, const double* __restrict__ U, int jacobian,
                            double w_end, double w_in, const double* __restrict__ F, double* __restrict__ coef,
                            double* __restrict__ G) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  const int64_t rm = r == 0 ? n - 1 : r - 1, rp = r == n - 1 ? 0 : r + 1;
  const double i2h = 1.0 / (2.0 * h);
  double j0 = 0.0, j1 = 0.0, j2 = 0.0;
  if (jacobian)
    for (int i = 0; i < s; ++i) {
      const double* u = U + (int64_t)i * n;
      const double w = (i == 0 || i == s - 1) ? w_end : w_in;
      const double ur = u[r];
      j0 += w * (ur * i2h);
      j1 += w * (-(u[rp] - u[rm]) * i2h);
      j2 += w * (-ur * i2h);
    }
  const double d2 = nu / (h * h);
  coef[r] = d2 + j0;
  coef[n + r] = -2.0 * d2 + j1;
  coef[2 * n + r] = d2 + j2;
  for (int i = 0; i < s; ++i) {
    const double* u = U + (int64_t)i * n;
    const double um = u[rm], uz = u[r], up = u[rp];
    G[(int64_t)i * n + r] = -uz * (up - um) * i2h - (j0 * um + j1 * uz + j2 * up) + (F ? F[(int64_t)i * n + r] : 0.0);
  }
}

void launch_wr_source(int64_t n, int s, double h, double nu, const double* U, int jacobian, double w_end, double w_in,
                      const double* F, double* coef, double* G, hipStream_t st) {
  hipLaunchKernelGGL(k_wr_source, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, s, h, nu, U, jacobian,
                     w_end, w_in, F, coef, G);
}

// per-block partial sums of |a - b|^2 and |a|^2 over cnt contiguous doubles
__global__ __launch_bounds__(256) void k_diff_norms(const double* a, const double* b, int64_t cnt, double* part) {
  __shared__ double red[16];
  double d2 = 0.0, a2 = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < cnt; e += (int64_t)gridDim.x * 256) {
    const double x = a[e], y = b[e];
    d2 += (x - y) * (x - y);
    a2 += x * x;
  }
  d2 = block_sum(d2, red);
  a2 = block_sum(a2, red);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = d2;
    part[2 * blockIdx.x + 1] = a2;
  }
}

void launch_diff_norms(const double* a, const double* b, int64_t cnt, double* part, int blocks, hipStream_t st) {
  hipLaunchKernelGGL(k_diff_norms, dim3((unsigned)blocks), dim3(256), 0, st, a, b, cnt, part);
}

__global__ void k_check_finite(const double* x, int64_t n, int64_t ld, int* flag) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (r >= n) return;
  const double v = x[r + ld * c];
  if (!isfinite(v)) atomicOr(flag, 1);
}

void launch_check_finite(const double* x, int64_t n, int cols, int64_t ld, int* flag, hipStream_t st) {
  if (n <= 0 || cols <= 0) return;
  dim3 grid((unsigned)((n + 255) / 256), (unsigned)cols);
  hipLaunchKernelGGL(k_check_finite, grid, dim3(256), 0, st, x, n, ld, flag);
}

__global__ void k_zero_u32(unsigned* x, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = 0u;
}

void launch_zero_u32(unsigned* x, int64_t n, hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(k_zero_u32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, x, n);
}

__global__ void k_fill(double* x, int64_t n, int64_t ld, double v) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (r < n) x[r + ld * c] = v;
}

void launch_fill(double* x, int64_t n, int cols, int64_t ld, double v, hipStream_t st) {
  if (n <= 0 || cols <= 0) return;
  dim3 grid((unsigned)((n + 255) / 256), (unsigned)cols);
  hipLaunchKernelGGL(k_fill, grid, dim3(256), 0, st, x, n, ld, v);
}

__global__ void k_copy(const double* a, double* b, int64_t n) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r < n) b[r] = a[r];
}

void launch_copy(const double* a, double* b, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_copy, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, a, b, n);
}

}  // namespace pe
