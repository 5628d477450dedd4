// Shift-and-invert (rational) block Krylov on gfx950: the block Arnoldi process of the
// shifted inverse (I - gamma L)^{-1} instead of L (the acceleration of Sec. 2.1 and
// Sec. 3.2, after the EBK method the paper builds on).  With
//     (I - gamma L)^{-1} V_l = V_l K_l + V_{l+1} K_{l+1,l} E_l^T
// the projected operator is H_L = (I - K_l^{-1}) / gamma and the residual of the Krylov
// solution V_l y(t) of u' = L u + U p(t) is
//     r(t) = (1/gamma) (I - gamma L) V_{l+1} K_{l+1,l} E_l^T K_l^{-1} y(t).
//
// Kernels here:
//   k_tri_factor / k_tri_reduce_factor  factor T = I - gamma L (periodic tridiagonal) by
//                                        partition: per-chunk elimination, spikes, and the
//                                        periodic block-tridiagonal interface system
//   k_sai_solve / k_sai_recon           W = T^{-1} V_j for the Arnoldi step j (V_j formed
//                                        from its TSQR factors and committed to the basis)
//   k_sai_gram                          Gram of (I - gamma L) V_l for the residual estimate
//   k_hess_lu / k_hess_inv              K_l^{-1} by LU with row interchanges
#include <type_traits>

#include "devutil.h"
#include "kernels.h"

namespace pe {

namespace {

__device__ __forceinline__ void tri_coefs(const TriDev& t, int64_t r, double& a, double& d, double& b) {
  double cm, cz, cp;
  if (t.per_point) {
    cm = t.coef[r];
    cz = t.coef[t.n + r];
    cp = t.coef[2 * t.n + r];
  } else {
    cm = t.c3[0];
    cz = t.c3[1];
    cp = t.c3[2];
  }
  a = -t.gamma * cm;
  d = 1.0 - t.gamma * cz;
  b = -t.gamma * cp;
}

__device__ __forceinline__ int64_t chunk_start(const TriDev& t, int c) { return (int64_t)c * t.R; }
__device__ __forceinline__ int64_t chunk_end(const TriDev& t, int c) {
  return c == t.C - 1 ? t.n : (int64_t)(c + 1) * t.R;
}
__device__ __forceinline__ int tri_chunk_of(const TriDev& t, int64_t r) {
  const int64_t c = r / t.R;
  return (int)(c < t.C - 1 ? c : t.C - 1);
}

// 2 x 2 helpers, row-major [m00 m01 m10 m11]
__device__ __forceinline__ void inv2(const double* m, double* o) {
  const double det = m[0] * m[3] - m[1] * m[2];
  const double id = 1.0 / det;
  o[0] = m[3] * id;
  o[1] = -m[1] * id;
  o[2] = -m[2] * id;
  o[3] = m[0] * id;
}

// reduced-system layout inside TriDev::red (per chunk c, then 4 trailing doubles):
//   Dinv[4c..4c+4)          inverse of the eliminated diagonal block
//   Lm  [4C + 4c ..)        forward multiplier A_c Dinv_{c-1}
//   Cc  [8C + 2c ..)        (vR_c[first], vR_c[last]): the coupling to F_{c+1}
//   Z   [10C + 4c ..)       rows 2c, 2c+1 of Z = M0^{-1} P (two columns, row-major pairs)
//   Sinv[14C ..14C+4)       (I + Q^T Z)^{-1}
// For C = 1 the whole 2 x 2 system's inverse sits in Sinv.

}  // namespace

// ---- factorisation --------------------------------------------------------------------
// one thread per chunk: elimination coefficients and the two spikes
__global__ __launch_bounds__(256) void k_tri_factor(const TriDev* __restrict__ tds) {
  const TriDev t = tds[blockIdx.y];
  if (!t.active) return;
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= t.C) return;
  const int64_t s = chunk_start(t, c), e = chunk_end(t, c);
  double prev_tc = 0.0;
  double yl = 0.0, yr = 0.0;  // forward sweeps of the two spike right-hand sides
  for (int64_t i = s; i < e; ++i) {
    double a, d, b;
    tri_coefs(t, i, a, d, b);
    const double den = (i == s) ? d : d - a * prev_tc;
    const double inv = 1.0 / den;
    const double tc = b * inv;
    t.ta[i] = a;
    t.tinv[i] = inv;
    t.tc[i] = tc;
    prev_tc = tc;
    // spike right-hand sides: a_s at the first row, b_{e-1} at the last row
    const double fl = (i == s) ? a : 0.0;
    double fr = 0.0;
    if (i == e - 1) fr = b;
    yl = (i == s) ? fl * inv : (fl - a * yl) * inv;
    yr = (i == s) ? fr * inv : (fr - a * yr) * inv;
    t.vL[i] = yl;
    t.vR[i] = yr;
  }
  // back substitution of both spikes
  double xl = t.vL[e - 1], xr = t.vR[e - 1];
  for (int64_t i = e - 2; i >= s; --i) {
    const double tc = t.tc[i];
    xl = t.vL[i] - tc * xl;
    xr = t.vR[i] - tc * xr;
    t.vL[i] = xl;
    t.vR[i] = xr;
  }
}

// one thread per problem: block elimination of the periodic interface system
//   F_c + vL_c[0] G_{c-1} + vR_c[0] F_{c+1} = y_c[0],  G_c + vL_c[e] G_{c-1} + vR_c[e] F_{c+1} = y_c[e]
// (chunk indices mod C): block tridiagonal M0 plus the two wrap-around couplings, which
// enter by the Sherman-Morrison-Woodbury formula
__global__ void k_tri_reduce_factor(const TriDev* __restrict__ tds) {
  const TriDev t = tds[blockIdx.x];
  if (!t.active || threadIdx.x != 0) return;
  const int C = t.C;
  double* Dinv = t.red;
  double* Lm = t.red + 4 * (int64_t)C;
  double* Cc = t.red + 8 * (int64_t)C;
  double* Z = t.red + 10 * (int64_t)C;
  double* Sinv = t.red + 14 * (int64_t)C;
  auto vLf = [&](int c) { return t.vL[chunk_start(t, c)]; };
  auto vLe = [&](int c) { return t.vL[chunk_end(t, c) - 1]; };
  auto vRf = [&](int c) { return t.vR[chunk_start(t, c)]; };
  auto vRe = [&](int c) { return t.vR[chunk_end(t, c) - 1]; };
  if (C == 1) {
    // F = x_0, G = x_{n-1}: x_{s-1} = G and x_e = F within the single chunk
    const double m[4] = {1.0 + vRf(0), vLf(0), vRe(0), 1.0 + vLe(0)};
    inv2(m, Sinv);
    return;
  }
  for (int c = 0; c < C; ++c) {
    Cc[2 * c] = vRf(c);
    Cc[2 * c + 1] = vRe(c);
  }
  // M0: D_0 = I; D_c = I - A_c Dinv_{c-1} C_{c-1}, with A_c = [[0, vLf],[0, vLe]] and
  // C_c = [[vRf, 0],[vRe, 0]]
  Dinv[0] = 1.0;
  Dinv[1] = 0.0;
  Dinv[2] = 0.0;
  Dinv[3] = 1.0;
  Lm[0] = Lm[1] = Lm[2] = Lm[3] = 0.0;
  for (int c = 1; c < C; ++c) {
    const double* Dp = Dinv + 4 * (c - 1);
    // A_c Dp: A_c has only its second column (vLf(c), vLe(c))
    const double l0 = vLf(c), l1 = vLe(c);
    double L4[4] = {l0 * Dp[2], l0 * Dp[3], l1 * Dp[2], l1 * Dp[3]};
    for (int k = 0; k < 4; ++k) Lm[4 * c + k] = L4[k];
    // D = I - L4 C_{c-1}, C_{c-1} has only its first column (Cc[2(c-1)], Cc[2(c-1)+1])
    const double c0 = Cc[2 * (c - 1)], c1 = Cc[2 * (c - 1) + 1];
    const double D[4] = {1.0 - (L4[0] * c0 + L4[1] * c1), 0.0, -(L4[2] * c0 + L4[3] * c1), 1.0};
    inv2(D, Dinv + 4 * c);
  }
  // Z = M0^{-1} P: P's columns are the wrap-around couplings, (vLf(0), vLe(0)) in block
  // row 0 (coefficient of G_{C-1}) and (vRf(C-1), vRe(C-1)) in block row C-1
  // (coefficient of F_0); forward sweep then back sweep, both columns at once
  for (int col = 0; col < 2; ++col) {
    // g_c = p_c - Lm_c g_{c-1}, stored in Z temporarily
    for (int c = 0; c < C; ++c) {
      double p0 = 0.0, p1 = 0.0;
      if (col == 0 && c == 0) {
        p0 = vLf(0);
        p1 = vLe(0);
      }
      if (col == 1 && c == C - 1) {
        p0 = vRf(C - 1);
        p1 = vRe(C - 1);
      }
      if (c > 0) {
        const double* L4 = Lm + 4 * c;
        const double g0 = Z[4 * (c - 1) + col], g1 = Z[4 * (c - 1) + 2 + col];
        p0 -= L4[0] * g0 + L4[1] * g1;
        p1 -= L4[2] * g0 + L4[3] * g1;
      }
      Z[4 * c + col] = p0;
      Z[4 * c + 2 + col] = p1;
    }
    for (int c = C - 1; c >= 0; --c) {
      double g0 = Z[4 * c + col], g1 = Z[4 * c + 2 + col];
      if (c < C - 1) {  // g -= C_c y_{c+1}: C_c picks F_{c+1}
        const double f1 = Z[4 * (c + 1) + col];
        g0 -= Cc[2 * c] * f1;
        g1 -= Cc[2 * c + 1] * f1;
      }
      const double* Di = Dinv + 4 * c;
      Z[4 * c + col] = Di[0] * g0 + Di[1] * g1;
      Z[4 * c + 2 + col] = Di[2] * g0 + Di[3] * g1;
    }
  }
  // S = I + Q^T Z, Q^T picks the entries G_{C-1} (row 2C-1) and F_0 (row 0)
  const double S[4] = {1.0 + Z[4 * (C - 1) + 2 + 0], Z[4 * (C - 1) + 2 + 1], Z[0], 1.0 + Z[1]};
  inv2(S, Sinv);
}

// ---- the solve of one Arnoldi step ----------------------------------------------------
// W = T^{-1} V_j.  One thread per (chunk, column): V_j's rows of the chunk are formed from
// the step's TSQR factors (first-pass factors when the previous step skipped its second
// pass) and committed to basis block j in the storage precision; the chunk solution y is
// written to W and its end values to rrhs.  The last workgroup of the problem solves the
// interface system, one thread per column.
template <typename TS>
__global__ __launch_bounds__(256) void k_sai_solve(const ProbDev* __restrict__ pds, const TriDev* __restrict__ tds,
                                                   int j) {
  const ProbDev p = pds[blockIdx.y];
  const TriDev t = tds[blockIdx.y];
  if (!p.active || !t.active || j >= p.l) return;
  __shared__ int flag;
  const int bw = p.bw;
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  const bool first = p.cnt[2 * p.nbmax + 1] != 0;
  const double* Ql = first ? p.Qloc1 : p.Qloc2;
  const double* Qs = first ? p.Qs1 : p.Qs2;
  TS* V = basis_ptr<TS>(p);
  const int64_t blk = p.n * bw;
  if (g < t.C * bw) {
    const int c = g / bw, col = g % bw;
    const int64_t s = chunk_start(t, c), e = chunk_end(t, c);
    double y = 0.0;
    for (int64_t i = s; i < e; ++i) {
      const double v = tsqr_entry(p, Ql, Qs, i, col);
      const TS vs = (TS)v;
      V[(int64_t)j * blk + i * bw + col] = vs;
      if (!std::is_same<TS, double>::value && j == 0) p.V[i * bw + col] = v;
      const double f = (double)vs;
      y = (i == s) ? f * t.tinv[i] : (f - t.ta[i] * y) * t.tinv[i];
      t.W[i * bw + col] = y;
    }
    double x = y;
    st_agent(t.rrhs + (int64_t)(2 * c + 1) * bw + col, x);
    for (int64_t i = e - 2; i >= s; --i) {
      x = t.W[i * bw + col] - t.tc[i] * x;
      t.W[i * bw + col] = x;
    }
    st_agent(t.rrhs + (int64_t)(2 * c) * bw + col, x);
  }
  if (!arrive_last(t.cnt, gridDim.x, &flag)) return;
  if (threadIdx.x == 0) atomicExch(t.cnt, 0u);
  const int col = threadIdx.x;
  if (col >= bw) return;
  const int C = t.C;
  const double* Dinv = t.red;
  const double* Lm = t.red + 4 * (int64_t)C;
  const double* Cc = t.red + 8 * (int64_t)C;
  const double* Z = t.red + 10 * (int64_t)C;
  const double* Sinv = t.red + 14 * (int64_t)C;
  const double* f = t.rrhs;
  double* u = t.ru;
  auto F = [&](int c) -> double& { return u[(int64_t)(2 * c) * bw + col]; };
  auto G = [&](int c) -> double& { return u[(int64_t)(2 * c + 1) * bw + col]; };
  if (C == 1) {
    const double f0 = f[col], f1 = f[bw + col];
    F(0) = Sinv[0] * f0 + Sinv[1] * f1;
    G(0) = Sinv[2] * f0 + Sinv[3] * f1;
    return;
  }
  // y = M0^{-1} f (forward sweep into u, then back sweep)
  double g0 = 0.0, g1 = 0.0;
  for (int c = 0; c < C; ++c) {
    double a0 = f[(int64_t)(2 * c) * bw + col], a1 = f[(int64_t)(2 * c + 1) * bw + col];
    if (c > 0) {
      const double* L4 = Lm + 4 * c;
      a0 -= L4[0] * g0 + L4[1] * g1;
      a1 -= L4[2] * g0 + L4[3] * g1;
    }
    F(c) = a0;
    G(c) = a1;
    g0 = a0;
    g1 = a1;
  }
  double fnext = 0.0;
  for (int c = C - 1; c >= 0; --c) {
    double a0 = F(c), a1 = G(c);
    if (c < C - 1) {
      a0 -= Cc[2 * c] * fnext;
      a1 -= Cc[2 * c + 1] * fnext;
    }
    const double* Di = Dinv + 4 * c;
    const double y0 = Di[0] * a0 + Di[1] * a1, y1 = Di[2] * a0 + Di[3] * a1;
    F(c) = y0;
    G(c) = y1;
    fnext = y0;
  }
  // Woodbury: u = y - Z Sinv (y[G_{C-1}], y[F_0])
  const double q0 = G(C - 1), q1 = F(0);
  const double w0 = Sinv[0] * q0 + Sinv[1] * q1, w1 = Sinv[2] * q0 + Sinv[3] * q1;
  for (int c = 0; c < C; ++c) {
    F(c) -= Z[4 * c] * w0 + Z[4 * c + 1] * w1;
    G(c) -= Z[4 * c + 2] * w0 + Z[4 * c + 3] * w1;
  }
}

// W[r, col] -= G_{c-1} vL[r] + F_{c+1} vR[r]: the chunk solutions coupled to the
// neighbouring chunks' end values (chunk indices mod C)
__global__ __launch_bounds__(256) void k_sai_recon(const TriDev* __restrict__ tds) {
  const TriDev t = tds[blockIdx.y];
  if (!t.active) return;
  const int bw = t.bw;
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= t.n * bw) return;
  const int64_t r = g / bw;
  const int col = (int)(g % bw);
  const int c = tri_chunk_of(t, r);
  const int cm = c == 0 ? t.C - 1 : c - 1, cp = c == t.C - 1 ? 0 : c + 1;
  const double Gm = t.ru[(int64_t)(2 * cm + 1) * bw + col];
  const double Fp = t.ru[(int64_t)(2 * cp) * bw + col];
  t.W[g] -= Gm * t.vL[r] + Fp * t.vR[r];
}

// ---- residual Gram ----------------------------------------------------------------------
// GW = W^T W for W = (I - gamma L) V_l, V_l the last step's TSQR output (formed from its
// factors, with the periodic neighbour rows for the stencil).  One row per thread; the
// workgroup sums its rows' outer products, the last workgroup sums the partials.
constexpr int kGramRows = 128;  // rows (and threads) per workgroup of k_sai_gram
__global__ __launch_bounds__(kGramRows) void k_sai_gram(const ProbDev* __restrict__ pds,
                                                        const TriDev* __restrict__ tds, double* part) {
  const ProbDev p = pds[blockIdx.y];
  const TriDev t = tds[blockIdx.y];
  if (!p.active || !t.active) return;
  __shared__ int flag;
  __shared__ double wrow[kGramRows * 33];
  const int bw = p.bw, tid = threadIdx.x;
  const bool first = p.cnt[2 * p.nbmax + 1] != 0;
  const double* Ql = first ? p.Qloc1 : p.Qloc2;
  const double* Qs = first ? p.Qs1 : p.Qs2;
  const int64_t r = (int64_t)blockIdx.x * kGramRows + tid;
  if (r < p.n) {
    const int64_t rm = r == 0 ? p.n - 1 : r - 1, rp = r == p.n - 1 ? 0 : r + 1;
    double cm, cz, cp;
    stencil_coefs(p, r, cm, cz, cp);
    for (int a = 0; a < bw; ++a) {
      const double v = tsqr_entry(p, Ql, Qs, r, a);
      const double lv = cm * tsqr_entry(p, Ql, Qs, rm, a) + cz * v + cp * tsqr_entry(p, Ql, Qs, rp, a);
      wrow[tid * 33 + a] = v - t.gamma * lv;
    }
  } else {
    for (int a = 0; a < bw; ++a) wrow[tid * 33 + a] = 0.0;
  }
  __syncthreads();
  double* mine = part + ((int64_t)blockIdx.y * gridDim.x + blockIdx.x) * 1024;
  for (int o = tid; o < bw * bw; o += kGramRows) {
    const int a = o / bw, b = o % bw;
    double s = 0.0;
    for (int k = 0; k < kGramRows; ++k) s += wrow[k * 33 + a] * wrow[k * 33 + b];
    st_agent(mine + o, s);
  }
  if (!arrive_last(t.cnt + 1, gridDim.x, &flag)) return;
  if (tid == 0) atomicExch(t.cnt + 1, 0u);
  for (int o = tid; o < bw * bw; o += kGramRows) {
    double s = 0.0;
    for (unsigned k = 0; k < gridDim.x; ++k) s += part[((int64_t)blockIdx.y * gridDim.x + k) * 1024 + o];
    t.GW[o] = s;
  }
}

// ---- inverse of the projected matrix --------------------------------------------------
// LU with row interchanges of the block upper Hessenberg K (N0 = l bw, blocks of bw; the
// blocks below the subdiagonal are zero and are never read from H).  Column k can only
// have nonzeros down to row (k / bw + 2) bw - 1, so the pivot search and the elimination
// stay in that band.  One workgroup per problem, factors in place in LU (ld N0).  A
// deflated basis column gives a zero row and column and a unit pivot; any other zero
// pivot makes the inverse NaN (the march then stops on the non-finite projected matrix).
__global__ __launch_bounds__(256) void k_hess_lu(const TriDev* __restrict__ tds) {
  const TriDev t = tds[blockIdx.x];
  if (!t.active) return;
  const int N0 = t.N0, bw = t.bw, tid = threadIdx.x;
  double* A = t.LU;
  __shared__ int piv_s;
  __shared__ int bad;
  if (tid == 0) bad = 0;
  for (int64_t e = tid; e < (int64_t)N0 * N0; e += 256) {
    const int r = (int)(e % N0), c = (int)(e / N0);
    A[e] = (r / bw <= c / bw + 1) ? t.H[(int64_t)r + t.ldH * c] : 0.0;
  }
  __syncthreads();
  for (int k = 0; k < N0; ++k) {
    const int rlim = min(N0, (k / bw + 2) * bw);
    if (tid < 64) {
      double best = -1.0;
      int bi = k;
      for (int i = k + tid; i < rlim; i += 64) {
        const double v = fabs(A[i + (int64_t)N0 * k]);
        if (v > best) {
          best = v;
          bi = i;
        }
      }
      // wave argmax (largest value, smallest row among equals)
      for (int off = 32; off > 0; off >>= 1) {
        const double ob = __shfl_down(best, off);
        const int oi = __shfl_down(bi, off);
        if (ob > best || (ob == best && oi < bi)) {
          best = ob;
          bi = oi;
        }
      }
      if (tid == 0) {
        piv_s = (best > 0.0) ? bi : -1;
        t.piv[k] = (best > 0.0) ? bi : k;
      }
    }
    __syncthreads();
    if (piv_s < 0) {
      // A zero column: the Arnoldi process deflated basis column k (a zero vector), which
      // leaves row and column k of K zero.  That direction carries nothing, so it gets a
      // unit pivot (K^{-1} = 1 there, the projected operator 0).  A zero column with a
      // nonzero row would be a singular K: the inverse is then flagged NaN.
      int nz = 0;
      for (int c = k + 1 + tid; c < N0; c += 256) nz |= (A[k + (int64_t)N0 * c] != 0.0);
      if (__syncthreads_or(nz)) {
        if (tid == 0) bad = 1;
      } else if (tid == 0) {
        A[k + (int64_t)N0 * k] = 1.0;
      }
      __syncthreads();
      continue;
    }
    const int pr = piv_s;
    if (pr != k)
      for (int c = tid; c < N0; c += 256) {
        const double x = A[k + (int64_t)N0 * c];
        A[k + (int64_t)N0 * c] = A[pr + (int64_t)N0 * c];
        A[pr + (int64_t)N0 * c] = x;
      }
    __syncthreads();
    const double dinv = 1.0 / A[k + (int64_t)N0 * k];
    for (int i = k + 1 + tid; i < rlim; i += 256) A[i + (int64_t)N0 * k] *= dinv;
    __syncthreads();
    const int nr = rlim - k - 1;
    for (int e = tid; e < nr * (N0 - k - 1); e += 256) {
      const int i = k + 1 + e % nr, c = k + 1 + e / nr;
      A[i + (int64_t)N0 * c] -= A[i + (int64_t)N0 * k] * A[k + (int64_t)N0 * c];
    }
    __syncthreads();
  }
  if (bad && tid == 0) A[0] = __longlong_as_double(0x7ff8000000000000LL);
}

// Kinv = K^{-1}: one wave per column of the identity: row interchanges, unit lower
// forward substitution, upper back substitution; the column lives in LDS
__global__ __launch_bounds__(256) void k_hess_inv(const TriDev* __restrict__ tds) {
  const TriDev t = tds[blockIdx.y];
  if (!t.active) return;
  extern __shared__ double xs[];
  const int N0 = t.N0, lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int col = blockIdx.x * 4 + w;
  if (col >= N0) return;
  double* x = xs + (int64_t)w * N0;
  const double* A = t.LU;
  for (int i = lane; i < N0; i += 64) x[i] = (i == col) ? 1.0 : 0.0;
  __builtin_amdgcn_wave_barrier();
  if (lane == 0)
    for (int k = 0; k < N0; ++k) {
      const int p = t.piv[k];
      if (p != k) {
        const double v = x[k];
        x[k] = x[p];
        x[p] = v;
      }
    }
  __builtin_amdgcn_wave_barrier();
  for (int k = 0; k < N0 - 1; ++k) {
    const double xk = x[k];
    if (xk != 0.0)
      for (int i = k + 1 + lane; i < N0; i += 64) x[i] -= A[i + (int64_t)N0 * k] * xk;
    __builtin_amdgcn_wave_barrier();
  }
  for (int k = N0 - 1; k >= 0; --k) {
    const double xk = x[k] / A[k + (int64_t)N0 * k];
    __builtin_amdgcn_wave_barrier();
    if (lane == 0) x[k] = xk;
    if (xk != 0.0)
      for (int i = lane; i < k; i += 64) x[i] -= A[i + (int64_t)N0 * k] * xk;
    __builtin_amdgcn_wave_barrier();
  }
  for (int i = lane; i < N0; i += 64) t.Kinv[i + (int64_t)N0 * col] = x[i];
}

// ---- launchers ----------------------------------------------------------------------------
void launch_tri_factor(TriDev* td, int nprob, int maxC, hipStream_t st) {
  hipLaunchKernelGGL(k_tri_factor, dim3((unsigned)((maxC + 255) / 256), (unsigned)nprob), dim3(256), 0, st, td);
  hipLaunchKernelGGL(k_tri_reduce_factor, dim3((unsigned)nprob), dim3(64), 0, st, td);
}

void launch_sai_solve(ProbDev* d, TriDev* td, int nprob, int maxCbw, int64_t maxnbw, int j, int mixed,
                      hipStream_t st) {
  const dim3 gs((unsigned)((maxCbw + 255) / 256), (unsigned)nprob);
  if (mixed)
    hipLaunchKernelGGL(k_sai_solve<float>, gs, dim3(256), 0, st, d, td, j);
  else
    hipLaunchKernelGGL(k_sai_solve<double>, gs, dim3(256), 0, st, d, td, j);
  hipLaunchKernelGGL(k_sai_recon, dim3((unsigned)((maxnbw + 255) / 256), (unsigned)nprob), dim3(256), 0, st, td);
}

void launch_sai_gram(ProbDev* d, TriDev* td, int nprob, int64_t maxn, double* part, hipStream_t st) {
  hipLaunchKernelGGL(k_sai_gram, dim3((unsigned)((maxn + kGramRows - 1) / kGramRows), (unsigned)nprob),
                     dim3(kGramRows), 0, st, d, td, part);
}

void launch_hess_inverse(TriDev* td, int nprob, int maxN0, hipStream_t st) {
  hipLaunchKernelGGL(k_hess_lu, dim3((unsigned)nprob), dim3(256), 0, st, td);
  const size_t lds = sizeof(double) * 4 * (size_t)maxN0;
  static bool attr = false;
  if (!attr) {
    if (hipFuncSetAttribute((const void*)k_hess_inv, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024) !=
        hipSuccess)
      (void)hipGetLastError();
    attr = true;
  }
  hipLaunchKernelGGL(k_hess_inv, dim3((unsigned)((maxN0 + 3) / 4), (unsigned)nprob), dim3(256), lds, st, td);
}

}  // namespace pe
