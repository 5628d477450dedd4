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
//   k_sai_solve / k_sai_pcr / k_sai_recon   W = T^{-1} V_j for the Arnoldi step j (V_j formed
//                                        from its TSQR factors and committed to the basis)
//   k_sai_gram                          Gram of (I - gamma L) V_l for the residual estimate
//   k_lu_panel / k_lu_trail / k_hess_inv   K_l^{-1} by LU with row interchanges
#include <algorithm>
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

// The interface system (two unknowns per chunk: F_c, the first row, and G_c, the last)
//   A_c u_{c-1} + u_c + C_c u_{c+1} = f_c,   u_c = (F_c, G_c), indices mod C,
//   A_c = [[0, vL_c(first)], [0, vL_c(last)]],   C_c = [[vR_c(first), 0], [vR_c(last), 0]],
// is solved by parallel cyclic reduction: C is a power of two, and level k (stride
// s = 2^k) replaces row c by row c minus alpha_c row (c - s) minus beta_c row (c + s),
// alpha_c = A_c D_{c-s}^{-1}, beta_c = C_c D_{c+s}^{-1}, which couples it to rows c -+ 2s;
// after log2(C) levels both couplings land on row c itself and u_c = E_c f_c with
// E_c = (A_c + D_c + C_c)^{-1}.  TriDev::red holds, per level, alpha_c and beta_c
// (8 doubles per chunk), then E_c (4 per chunk).
__device__ __forceinline__ int sai_levels(int C) {
  int k = 0;
  while ((1 << k) < C) ++k;
  return k;
}

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

// one workgroup per problem: the cyclic-reduction coefficients of the interface system,
// one thread per chunk, the blocks of the current level in LDS
__device__ __forceinline__ void mul2(const double* a, const double* b, double* o) {
  o[0] = a[0] * b[0] + a[1] * b[2];
  o[1] = a[0] * b[1] + a[1] * b[3];
  o[2] = a[2] * b[0] + a[3] * b[2];
  o[3] = a[2] * b[1] + a[3] * b[3];
}
__global__ __launch_bounds__(256) void k_tri_reduce_factor(const TriDev* __restrict__ tds) {
  const TriDev t = tds[blockIdx.x];
  if (!t.active) return;
  __shared__ double sA[4 * 256], sC[4 * 256], sD[4 * 256];
  const int C = t.C, c = threadIdx.x;
  const int nlev = sai_levels(C);
  double A[4] = {0, 0, 0, 0}, Cm[4] = {0, 0, 0, 0}, D[4] = {1, 0, 0, 1};
  if (c < C) {
    A[1] = t.vL[chunk_start(t, c)];
    A[3] = t.vL[chunk_end(t, c) - 1];
    Cm[0] = t.vR[chunk_start(t, c)];
    Cm[2] = t.vR[chunk_end(t, c) - 1];
  }
  for (int lev = 0; lev < nlev; ++lev) {
    const int s = 1 << lev;
    if (c < C)
      for (int k = 0; k < 4; ++k) {
        sA[4 * c + k] = A[k];
        sC[4 * c + k] = Cm[k];
        sD[4 * c + k] = D[k];
      }
    __syncthreads();
    if (c < C) {
      const int m = (c - s + C) % C, p = (c + s) % C;
      double Dm[4], Dp[4], al[4], be[4], t1[4], t2[4];
      inv2(sD + 4 * m, Dm);
      inv2(sD + 4 * p, Dp);
      mul2(A, Dm, al);
      mul2(Cm, Dp, be);
      double* out = t.red + ((int64_t)lev * C + c) * 8;
      for (int k = 0; k < 4; ++k) {
        out[k] = al[k];
        out[4 + k] = be[k];
      }
      // D' = D - al C_{c-s} - be A_{c+s};  A' = -al A_{c-s};  C' = -be C_{c+s}
      mul2(al, sC + 4 * m, t1);
      mul2(be, sA + 4 * p, t2);
      for (int k = 0; k < 4; ++k) D[k] -= t1[k] + t2[k];
      mul2(al, sA + 4 * m, t1);
      mul2(be, sC + 4 * p, t2);
      for (int k = 0; k < 4; ++k) {
        A[k] = -t1[k];
        Cm[k] = -t2[k];
      }
    }
    __syncthreads();
  }
  if (c < C) {
    // after the last level both couplings refer to row c itself
    const double S[4] = {A[0] + D[0] + Cm[0], A[1] + D[1] + Cm[1], A[2] + D[2] + Cm[2], A[3] + D[3] + Cm[3]};
    inv2(S, t.red + ((int64_t)nlev * C) * 8 + 4 * (int64_t)c);
  }
}

// ---- the solve of one Arnoldi step ----------------------------------------------------
// V_j = Qloc Qs (the step's TSQR factors; first-pass factors when the previous step
// skipped its second pass), committed to basis block j in the storage precision (and in
// fp64 for block 0 of an fp32 basis).  One thread per entry.
template <typename TS>
__global__ __launch_bounds__(256) void k_sai_commit(const ProbDev* __restrict__ pds, int j) {
  const ProbDev p = pds[blockIdx.y];
  if (!p.active || j >= p.l) return;
  const int bw = p.bw;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= p.n * bw) return;
  const bool first = p.cnt[2 * p.nbmax + 1] != 0;
  const int64_t r = e / bw;
  const int col = (int)(e - r * bw);
  const double v = tsqr_entry(p, first ? p.Qloc1 : p.Qloc2, first ? p.Qs1 : p.Qs2, r, col);
  basis_ptr<TS>(p)[(int64_t)j * p.n * bw + e] = (TS)v;
  if (!std::is_same<TS, double>::value && j == 0) p.V[e] = v;
}

// The interface system by cyclic reduction (k_sai_pcr, one workgroup per column): f, g are LDS
// ping-pong buffers of bw interface vectors, column-major (entry (2c + k) of column col at
// col 2C + 2c + k: F_c for k = 0, G_c for k = 1; consecutive chunks are consecutive in
// memory, so a wave's accesses spread over the LDS banks); the result goes to u (same
// layout).  Thread c < C takes chunk c for every column; every level's coefficients are
// loaded up front.  The workgroup barrier orders the levels.
__device__ void pcr_solve(int C, int bw, const double* __restrict__ red, double* f, double* g, double* u) {
  constexpr int kMaxLev = 8;  // C <= 256 chunks
  const int nlev = sai_levels(C);
  const int c = threadIdx.x;
  const bool act = c < C;
  const int64_t ld = 2 * (int64_t)C;
  // the chunk's coefficients of every level and its final 2 x 2 block, all loads issued
  // at once (clamped indices); the levels then wait only on LDS
  double abl[kMaxLev][8], fin[4];
#pragma unroll
  for (int lev = 0; lev < kMaxLev; ++lev)
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const bool ok = act && lev < nlev;
      const double v = red[ok ? ((int64_t)lev * C + c) * 8 + k : 0];
      abl[lev][k] = ok ? v : 0.0;
    }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const double v = red[act ? (int64_t)nlev * C * 8 + 4 * (int64_t)c + k : 0];
    fin[k] = act ? v : 0.0;
  }
#pragma unroll
  for (int lev = 0; lev < kMaxLev; ++lev) {
    if (lev >= nlev) break;
    const int s = 1 << lev;
    const double* ab = abl[lev];
    if (act) {
      const int m = (c - s) & (C - 1), p = (c + s) & (C - 1);  // C is a power of two
#pragma unroll 4
      for (int col = 0; col < bw; ++col) {
        const double* fc = f + col * ld;
        const double f0 = fc[2 * c], f1 = fc[2 * c + 1];
        const double m0 = fc[2 * m], m1 = fc[2 * m + 1];
        const double p0 = fc[2 * p], p1 = fc[2 * p + 1];
        g[col * ld + 2 * c] = f0 - (ab[0] * m0 + ab[1] * m1) - (ab[4] * p0 + ab[5] * p1);
        g[col * ld + 2 * c + 1] = f1 - (ab[2] * m0 + ab[3] * m1) - (ab[6] * p0 + ab[7] * p1);
      }
    }
    lds_barrier();
    double* tmp = f;
    f = g;
    g = tmp;
  }
  if (act)
    for (int col = 0; col < bw; ++col) {  // u_c = E_c f_c, E_c the final block
      const double f0 = f[col * ld + 2 * c], f1 = f[col * ld + 2 * c + 1];
      u[col * ld + 2 * c] = fin[0] * f0 + fin[1] * f1;
      u[col * ld + 2 * c + 1] = fin[2] * f0 + fin[3] * f1;
    }
}

// W = T^{-1} V_j (V_j committed): a workgroup takes cpw consecutive chunks (cpw bw <= 64
// threads); when their rows of V_j fit in LDS they are staged there -- each chunk in its
// own region, padded by two doubles so that the chunks a wave works on start in different
// LDS banks -- and thread (chunk, column) eliminates its chunk in LDS, otherwise it works
// on W in global memory.  The chunk solutions y go to W and their end values to rrhs
// (column-major interface vectors, see pcr_solve); k_sai_pcr then solves the interface
// system, one workgroup per column.
template <typename TS>
__global__ __launch_bounds__(256) void k_sai_solve(const ProbDev* __restrict__ pds, const TriDev* __restrict__ tds,
                                                   int j) {
  const ProbDev p = pds[blockIdx.y];
  const TriDev t = tds[blockIdx.y];
  if (!p.active || !t.active || j >= p.l) return;
  extern __shared__ double xs[];
  const int bw = p.bw, tid = threadIdx.x, R = t.R;
  const int cpw = sai_chunks_per_group(R, bw);
  const bool lds = sai_stage_in_lds(R, bw);
  const int c0 = blockIdx.x * cpw;
  const int64_t ld = 2 * (int64_t)t.C;
  const TS* V = basis_ptr<TS>(p) + (int64_t)j * p.n * bw;
  if (c0 < t.C) {
    const int c1 = min(t.C, c0 + cpw);
    const int cl = tid / bw, col = tid - (tid / bw) * bw;
    const int c = c0 + cl;
    const bool mine = cl < cpw && c < c1;
    if (lds) {
      // chunk k of the group: values at xv(k) (rows x bw), coefficients at xa(k), xi(k),
      // xc(k) (rows each); regions padded by 2 doubles, the group's last chunk may be long
      const int xstr = R * bw + 2, cstr = R + 2;
      const int rows_last = (int)(chunk_end(t, c1 - 1) - chunk_start(t, c1 - 1));
      double* xv0 = xs;
      double* xa0 = xs + (int64_t)(c1 - c0 - 1) * xstr + rows_last * bw + 2;
      const int cspan = (c1 - c0 - 1) * cstr + rows_last + 2;
      double* xi0 = xa0 + cspan;
      double* xc0 = xi0 + cspan;
      // one bulk phase for all of the group's values and coefficients; chunk k of the
      // group is min(row / R, nch - 1) (its last chunk may be long)
      const int nch = c1 - c0;
      const int64_t rs = chunk_start(t, c0);
      const int nrows = (int)(chunk_end(t, c1 - 1) - rs);
      const int rbw = R * bw;
      bulk_load<16>(
          (int64_t)nrows * bw, [=](int64_t q) -> double { return (double)V[rs * bw + q]; },
          [=](int64_t q, double v) {
            const int k = min((int)q / rbw, nch - 1);
            xv0[q + 2 * k] = v;
          });
      // the three coefficient rows as offsets from the first (arithmetic selection: a
      // select among pointers compiles to a table in scratch memory)
      const double* ta = t.ta;
      const int64_t o1 = t.tinv - t.ta, o2 = t.tc - t.ta;
      const int64_t x1 = xi0 - xa0, x2 = xc0 - xa0;
      bulk_load<16>(
          3 * (int64_t)nrows,
          [=](int64_t q) -> double {
            const int a = (int)q / nrows, r = (int)q - a * nrows;
            return ta[(a == 1 ? o1 : 0) + (a == 2 ? o2 : 0) + rs + r];
          },
          [=](int64_t q, double v) {
            const int a = (int)q / nrows, r = (int)q - a * nrows;
            const int k = min(r / R, nch - 1);
            xa0[(a == 1 ? x1 : 0) + (a == 2 ? x2 : 0) + r + 2 * k] = v;
          });
      lds_barrier();
      if (mine) {
        const int e0 = (int)(chunk_end(t, c) - chunk_start(t, c));
        double* __restrict__ x = xv0 + (int64_t)cl * xstr + col;
        const double* __restrict__ cta_ = xa0 + (int64_t)cl * cstr;
        const double* __restrict__ cti_ = xi0 + (int64_t)cl * cstr;
        const double* __restrict__ ctc_ = xc0 + (int64_t)cl * cstr;
        // both sweeps in batches of 8 rows: the batch's operands are read before any
        // of its results is written, so the loads overlap and only the recurrence waits
        constexpr int B = 8;
        double y = 0.0;
        for (int i0 = 0; i0 < e0; i0 += B) {
          double xq[B], av[B], iv[B];
#pragma unroll
          for (int q = 0; q < B; ++q) {
            const int i = i0 + q < e0 ? i0 + q : e0 - 1;
            xq[q] = x[i * bw];
            av[q] = cta_[i];
            iv[q] = cti_[i];
          }
#pragma unroll
          for (int q = 0; q < B; ++q) {
            if (i0 + q >= e0) break;
            y = (i0 + q == 0) ? xq[q] * iv[q] : (xq[q] - av[q] * y) * iv[q];
            xq[q] = y;
          }
#pragma unroll
          for (int q = 0; q < B; ++q)
            if (i0 + q < e0) x[(i0 + q) * bw] = xq[q];
        }
        st_agent(t.rrhs + col * ld + 2 * c + 1, y);
        for (int i1 = e0 - 2; i1 >= 0; i1 -= B) {  // rows i1, i1 - 1, ..., down to 0
          double xq[B], cv[B];
#pragma unroll
          for (int q = 0; q < B; ++q) {
            const int i = i1 - q >= 0 ? i1 - q : 0;
            xq[q] = x[i * bw];
            cv[q] = ctc_[i];
          }
#pragma unroll
          for (int q = 0; q < B; ++q) {
            if (i1 - q < 0) break;
            y = xq[q] - cv[q] * y;
            xq[q] = y;
          }
#pragma unroll
          for (int q = 0; q < B; ++q)
            if (i1 - q >= 0) x[(i1 - q) * bw] = xq[q];
        }
        st_agent(t.rrhs + col * ld + 2 * c, y);
      }
      lds_barrier();  // the interface values' stores stay in flight
      for (int q = tid; q < nrows * bw; q += 256) t.W[rs * bw + q] = xv0[q + 2 * min(q / rbw, nch - 1)];
    } else if (mine) {
      const int64_t s = chunk_start(t, c), e = chunk_end(t, c);
      double* x = t.W + s * bw + col;
      const TS* v = V + s * bw + col;
      double y = 0.0;
      for (int64_t i = s; i < e; ++i) {
        const double f = (double)v[(i - s) * bw];
        y = (i == s) ? f * t.tinv[i] : (f - t.ta[i] * y) * t.tinv[i];
        x[(i - s) * bw] = y;
      }
      st_agent(t.rrhs + col * ld + 2 * c + 1, y);
      for (int64_t i = e - 2; i >= s; --i) {
        y = x[(i - s) * bw] - t.tc[i] * y;
        x[(i - s) * bw] = y;
      }
      st_agent(t.rrhs + col * ld + 2 * c, y);
    }
  }
}

// launch bounds of the interface solve: chunks (sai_chunking) and block width
constexpr int kSaiMaxC = 256;
constexpr int kSaiMaxBw = 32;

// The interface system of one column (k_sai_solve wrote its right-hand sides): one
// workgroup per (column, problem), thread c for chunk c, ping-pong buffers in LDS.
// Per column the arithmetic is that of a multi-column sweep, in the same order.
__global__ __launch_bounds__(256) void k_sai_pcr(const TriDev* __restrict__ tds) {
  const TriDev t = tds[blockIdx.y];
  const int col = blockIdx.x;
  if (!t.active || col >= t.bw) return;
  extern __shared__ double xs[];
  const int64_t ld = 2 * (int64_t)t.C;
  double* f = xs;
  double* g = xs + ld;
  const double* src = t.rrhs + col * ld;
  bulk_load(ld, [=](int64_t e) -> double { return src[e]; }, [=](int64_t e, double v) { f[e] = v; });
  __syncthreads();
  pcr_solve(t.C, 1, t.red, f, g, t.ru + col * ld);
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
  const double Gm = t.ru[(int64_t)col * 2 * t.C + 2 * cm + 1];
  const double Fp = t.ru[(int64_t)col * 2 * t.C + 2 * cp];
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
// K (N0 = l bw) is block upper Hessenberg with blocks of bw: column k has nonzeros down
// to row pe(k) = min(N0, (k / bw + 2) bw) - 1 only.  LU with row interchanges, one block
// column (panel) at a time, K in place in global memory:
//   (a) one wave factors the panel in LDS: for each of its columns k the pivot is the
//       largest entry of column k in rows [k, pe) (NaN entries never chosen), rows k and
//       pivot are exchanged in the panel columns >= k only (LINPACK storage: multipliers
//       stay where they were computed), the multipliers are formed and the rest of the
//       panel updated;
//   (b) one wave per trailing column applies the panel's interchanges and eliminations
//       to the column's 2 bw band entries (one per lane), in order.
// A deflated basis column (a zero vector) leaves row and column k of K zero: it gets a
// unit pivot (K^{-1} = 1 there, the projected operator 0).  A zero pivot column with a
// nonzero row (a singular K) makes the result NaN, and the march stops on the non-finite
// projected matrix.
__device__ __forceinline__ void lds_order() {
  __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0): this wave's LDS operations are done
  __builtin_amdgcn_wave_barrier();
}

// One launch pair per block column: the panel (one wave, in LDS) and the trailing update
// (one wave per trailing column, the column's band rows one per lane), so the trailing
// sweeps run over the whole chip.
__global__ void k_lu_init(const TriDev* __restrict__ tds) {
  const TriDev t = tds[blockIdx.y];
  if (!t.active) return;
  const int N0 = t.N0, bw = t.bw;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < (int64_t)N0 * N0;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(e % N0), c = (int)(e / N0);
    t.LU[e] = c >= (r / bw - 1) * bw ? t.H[(int64_t)r + t.ldH * c] : 0.0;
  }
}

__device__ __forceinline__ double lane_bcast(double v, int src) {
  const int s = __builtin_amdgcn_readfirstlane(src);
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), s);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), s);
  return __hiloint2double(hi, lo);
}

// (value, index) maximum over the wave, the smallest index among equal values, returned
// to every lane: the DPP pattern of wave_sum (rows of 16 lanes, then the row broadcasts
// into lane 63) with a compare-select in place of the add; lanes outside a stage's
// row mask keep their own pair
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ void argmax_stage(double& best, int& bi) {
  const int lo = __builtin_amdgcn_update_dpp(__double2loint(best), __double2loint(best), CTRL, ROW_MASK, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(__double2hiint(best), __double2hiint(best), CTRL, ROW_MASK, 0xF, false);
  const int oi = __builtin_amdgcn_update_dpp(bi, bi, CTRL, ROW_MASK, 0xF, false);
  const double ob = __hiloint2double(hi, lo);
  if (ob > best || (ob == best && oi < bi)) {
    best = ob;
    bi = oi;
  }
}
__device__ __forceinline__ void wave_argmax(double& best, int& bi) {
  argmax_stage<0xB1, 0xF>(best, bi);
  argmax_stage<0x4E, 0xF>(best, bi);
  argmax_stage<0x124, 0xF>(best, bi);
  argmax_stage<0x128, 0xF>(best, bi);
  argmax_stage<0x142, 0xA>(best, bi);
  argmax_stage<0x143, 0xC>(best, bi);
  const int lo = __builtin_amdgcn_readlane(__double2loint(best), 63);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(best), 63);
  bi = __builtin_amdgcn_readlane(bi, 63);
  best = __hiloint2double(hi, lo);
}

// panel jb: rows [k0, pe) (at most 2 bw <= 64), columns [k0, k1); lane q holds row k0 + q
// in registers (BWM >= bw columns, compile-time register indices), the pivot row and the
// interchanged rows broadcast by readlane
template <int BWM>
__device__ __forceinline__ void lu_panel_regs(const TriDev& t, int jb, int lane) {
  const int N0 = t.N0, bw = t.bw;
  double* A = t.LU;
  const int k0 = jb * bw, k1 = k0 + bw, pe = min(N0, k1 + bw), nb = pe - k0, nc = bw;
  double xr[BWM];
#pragma unroll
  for (int c = 0; c < BWM; ++c) {
    const double v = A[(int64_t)(k0 + (lane < nb ? lane : nb - 1)) + (int64_t)N0 * (k0 + (c < nc ? c : nc - 1))];
    xr[c] = (lane < nb && c < nc) ? v : 0.0;
  }
  int bad = 0;
#pragma unroll
  for (int kq = 0; kq < BWM; ++kq) {
    if (kq >= nc) break;
    // pivot: the largest |entry| of column kq in rows kq..nb-1, the smallest row among equals
    double best = (lane >= kq && lane < nb) ? fabs(xr[kq]) : -1.0;
    if (!(best >= 0.0)) best = -1.0;
    int bi = lane;
    wave_argmax(best, bi);
    if (!(best > 0.0)) {
      // zero column: a deflated basis direction when row kq is zero as well (unit pivot)
      int nz = 0;
#pragma unroll
      for (int c = kq + 1; c < BWM; ++c)
        if (c < nc) nz |= (lane_bcast(xr[c], kq) != 0.0);
      for (int c = k1 + lane; c < N0; c += 64) nz |= (A[(int64_t)(k0 + kq) + (int64_t)N0 * c] != 0.0);
      bad |= __any(nz);
      if (lane == kq) xr[kq] = 1.0;
      if (lane == 0) t.piv[k0 + kq] = k0 + kq;
      continue;
    }
    if (lane == 0) t.piv[k0 + kq] = k0 + bi;
    if (bi != kq) {  // exchange rows kq and bi in columns >= kq (multipliers stay in place)
#pragma unroll
      for (int c = kq; c < BWM; ++c) {
        const double a = lane_bcast(xr[c], kq), b = lane_bcast(xr[c], bi);
        if (lane == kq) xr[c] = b;
        else if (lane == bi) xr[c] = a;
      }
    }
    double prow[BWM];
#pragma unroll
    for (int c = kq; c < BWM; ++c) prow[c] = lane_bcast(xr[c], kq);
    if (lane > kq && lane < nb) {
      const double m = xr[kq] / prow[kq];
      xr[kq] = m;
#pragma unroll
      for (int c = kq + 1; c < BWM; ++c) xr[c] -= m * prow[c];
    }
  }
#pragma unroll
  for (int c = 0; c < BWM; ++c)
    if (lane < nb && c < nc) A[(int64_t)(k0 + lane) + (int64_t)N0 * (k0 + c)] = xr[c];
  // a zero pivot column with a nonzero row: K is singular (row 0 is final by now)
  if (lane == 0 && bad) A[0] = __longlong_as_double(0x7ff8000000000000LL);
}

// wider panels (bw > 16): the panel in LDS, one lane per row
__device__ __forceinline__ void lu_panel_lds(const TriDev& t, int jb, int lane) {
  const int N0 = t.N0, bw = t.bw;
  constexpr int LD = 33;
  __shared__ double P[64 * LD];
  double* A = t.LU;
  const int k0 = jb * bw, k1 = k0 + bw, pe = min(N0, k1 + bw), nb = pe - k0, nc = bw;
  for (int c = 0; c < nc; ++c) P[lane * LD + c] = lane < nb ? A[(int64_t)(k0 + lane) + (int64_t)N0 * (k0 + c)] : 0.0;
  lds_order();
  int bad = 0;
  for (int kq = 0; kq < nc; ++kq) {
    // pivot: the largest |entry| of column kq in rows kq..nb-1, the smallest row among equals
    double best = (lane >= kq && lane < nb) ? fabs(P[lane * LD + kq]) : -1.0;
    if (!(best >= 0.0)) best = -1.0;
    int bi = lane;
    wave_argmax(best, bi);
    if (!(best > 0.0)) {
      // zero column: a deflated basis direction when row kq is zero as well (unit pivot)
      int nz = 0;
      for (int c = kq + 1 + lane; c < nc; c += 64) nz |= (P[kq * LD + c] != 0.0);
      for (int c = k1 + lane; c < N0; c += 64) nz |= (A[(int64_t)(k0 + kq) + (int64_t)N0 * c] != 0.0);
      bad |= __any(nz);
      lds_order();
      if (lane == kq) P[kq * LD + kq] = 1.0;
      if (lane == 0) t.piv[k0 + kq] = k0 + kq;
      lds_order();
      continue;
    }
    if (lane == 0) t.piv[k0 + kq] = k0 + bi;
    if (bi != kq) {  // exchange rows kq and bi in columns >= kq (multipliers stay in place)
      for (int c = kq + lane; c < nc; c += 64) {
        const double a = P[kq * LD + c], b = P[bi * LD + c];
        P[kq * LD + c] = b;
        P[bi * LD + c] = a;
      }
      lds_order();
    }
    const double piv = P[kq * LD + kq];
    if (lane > kq && lane < nb) {
      const double m = P[lane * LD + kq] / piv;
      P[lane * LD + kq] = m;
      for (int c = kq + 1; c < nc; ++c) P[lane * LD + c] -= m * P[kq * LD + c];
    }
    lds_order();
  }
  for (int c = 0; c < nc; ++c)
    if (lane < nb) A[(int64_t)(k0 + lane) + (int64_t)N0 * (k0 + c)] = P[lane * LD + c];
  // a zero pivot column with a nonzero row: K is singular (row 0 is final by now)
  if (lane == 0 && bad) A[0] = __longlong_as_double(0x7ff8000000000000LL);
}

__global__ __launch_bounds__(64) void k_lu_panel(const TriDev* __restrict__ tds, int jb) {
  const TriDev t = tds[blockIdx.x];
  if (!t.active) return;
  if (jb >= t.N0 / t.bw) return;
  const int lane = threadIdx.x;
  if (t.bw <= 8)
    lu_panel_regs<8>(t, jb, lane);
  else if (t.bw <= 16)
    lu_panel_regs<16>(t, jb, lane);
  else
    lu_panel_lds(t, jb, lane);
}

// trailing columns of panel jb: the interchanges and eliminations in order
__global__ __launch_bounds__(256) void k_lu_trail(const TriDev* __restrict__ tds, int jb) {
  const TriDev t = tds[blockIdx.y];
  if (!t.active) return;
  const int N0 = t.N0, bw = t.bw;
  if (jb >= N0 / bw) return;
  const int k0 = jb * bw, k1 = k0 + bw, pe = min(N0, k1 + bw), nb = pe - k0;
  __shared__ double mul[32 * 64];  // mul[kq * 64 + q] = L(k0 + q, k0 + kq)
  __shared__ int pv[32];
  const double* A = t.LU;
  for (int e = threadIdx.x; e < nb * bw; e += 256) {
    const int q = e % nb, kq = e / nb;
    mul[kq * 64 + q] = A[(int64_t)(k0 + q) + (int64_t)N0 * (k0 + kq)];
  }
  if (threadIdx.x < bw) pv[threadIdx.x] = t.piv[k0 + threadIdx.x] - k0;
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int c = k1 + blockIdx.x * 4 + (threadIdx.x >> 6);
  if (c >= N0) return;
  double* col = t.LU + (int64_t)N0 * c + k0;
  double x = lane < nb ? col[lane] : 0.0;
  for (int kq = 0; kq < bw; ++kq) {
    const int pq = pv[kq];
    const double xk = lane_bcast(x, pq), xo = lane_bcast(x, kq);
    if (lane == kq) x = xk;
    else if (lane == pq) x = xo;
    if (xk != 0.0 && lane > kq && lane < nb) x -= mul[kq * 64 + lane] * xk;
  }
  if (lane < nb) col[lane] = x;
}

// Kinv = K^{-1}: one wave per column of the identity, the column in LDS: forward sweep
// with the interchanges and multipliers in the order they were made (LINPACK storage; the
// multipliers of column k sit in rows (k, pe(k)) and are staged in LDS for the
// workgroup when they fit), then back substitution with U, whose columns are staged in
// LDS a block at a time by the whole workgroup.
template <bool kStageL>
__global__ __launch_bounds__(256) void k_hess_inv(const TriDev* __restrict__ tds) {
  const TriDev t = tds[blockIdx.y];
  if (!t.active) return;
  extern __shared__ double xs[];
  const int N0 = t.N0, bw = t.bw, tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  if (blockIdx.x * 4 >= N0) return;
  const double* A = t.LU;
  const int col = blockIdx.x * 4 + w;
  const bool act = col < N0;  // every wave stays for the workgroup barriers
  double* x = xs + (int64_t)w * N0;
  double* work = xs + 4 * (int64_t)N0;
  // multipliers: Lb[k * 2bw + (i - k - 1)] = L[i][k], i in (k, pe(k))
  const int lw = 2 * bw;
  if (kStageL) {
    bulk_load(
        (int64_t)N0 * lw,
        [&](int64_t e) -> double {
          const int k = (int)(e / lw), i = k + 1 + (int)(e % lw);
          return A[(i < N0 ? i : N0 - 1) + (int64_t)N0 * k];
        },
        [&](int64_t e, double v) {
          const int k = (int)(e / lw), i = k + 1 + (int)(e % lw);
          work[e] = (i < min(N0, (k / bw + 2) * bw)) ? v : 0.0;
        });
  }
  for (int i = lane; i < N0; i += 64) x[i] = (i == col) ? 1.0 : 0.0;
  __syncthreads();
  if (act)
    for (int k = 0; k < N0 - 1; ++k) {
      const int pr = t.piv[k];
      const double xk = x[pr];
      const double xkk = x[k];
      lds_order();
      if (lane == 0 && pr != k) {
        x[pr] = xkk;
        x[k] = xk;
      }
      lds_order();
      if (xk != 0.0 && lane < lw - 1) {
        const int i = k + 1 + lane;
        if (i < min(N0, (k / bw + 2) * bw)) x[i] -= (kStageL ? work[(int64_t)k * lw + lane] : A[i + (int64_t)N0 * k]) * xk;
      }
      lds_order();
    }
  // back substitution: columns [klo, khi] of U (rows 0..khi) staged per block
  const int room = kSaiLdsDoubles - 4 * N0;
  const int CB = max(1, min(64, room / N0));
  for (int khi = N0 - 1; khi >= 0; khi -= CB) {
    const int klo = max(0, khi - CB + 1), nr = khi + 1;
    __syncthreads();
    bulk_load(
        (int64_t)(khi - klo + 1) * nr, [&](int64_t e) -> double { return A[(e % nr) + (int64_t)N0 * (klo + e / nr)]; },
        [&](int64_t e, double v) { work[e] = v; });
    __syncthreads();
    if (act)
      for (int k = khi; k >= klo; --k) {
        const double* uc = work + (int64_t)(k - klo) * nr;
        const double xk = x[k] / uc[k];
        lds_order();
        if (lane == 0) x[k] = xk;
        if (xk != 0.0)
          for (int i = lane; i < k; i += 64) x[i] -= uc[i] * xk;
        lds_order();
      }
  }
  __syncthreads();
  if (act)
    for (int i = lane; i < N0; i += 64) t.Kinv[i + (int64_t)N0 * col] = x[i];
}

// ---- launchers ----------------------------------------------------------------------------
void launch_tri_factor(TriDev* td, int nprob, int maxC, hipStream_t st) {
  hipLaunchKernelGGL(k_tri_factor, dim3((unsigned)((maxC + 255) / 256), (unsigned)nprob), dim3(256), 0, st, td);
  hipLaunchKernelGGL(k_tri_reduce_factor, dim3((unsigned)nprob), dim3(256), 0, st, td);
}

// groups: workgroups per problem (the most that any problem's chunks need,
// sai_solve_groups)
void launch_sai_solve(ProbDev* d, TriDev* td, int nprob, int groups, int64_t maxnbw, int j, int mixed,
                      hipStream_t st) {
  static bool attr = false;
  if (!attr) {
    const void* fns[2] = {(const void*)k_sai_solve<double>, (const void*)k_sai_solve<float>};
    for (const void* f : fns)
      if (hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, kSaiLdsDoubles * 8) != hipSuccess)
        (void)hipGetLastError();
    attr = true;
  }
  const dim3 ge((unsigned)((maxnbw + 255) / 256), (unsigned)nprob);
  if (mixed)
    hipLaunchKernelGGL(k_sai_commit<float>, ge, dim3(256), 0, st, d, j);
  else
    hipLaunchKernelGGL(k_sai_commit<double>, ge, dim3(256), 0, st, d, j);
  const dim3 gs((unsigned)groups, (unsigned)nprob);
  const size_t lds = sizeof(double) * kSaiLdsDoubles;
  if (mixed)
    hipLaunchKernelGGL(k_sai_solve<float>, gs, dim3(256), lds, st, d, td, j);
  else
    hipLaunchKernelGGL(k_sai_solve<double>, gs, dim3(256), lds, st, d, td, j);
  hipLaunchKernelGGL(k_sai_pcr, dim3((unsigned)kSaiMaxBw, (unsigned)nprob), dim3(256),
                     sizeof(double) * 4 * kSaiMaxC, st, td);
  hipLaunchKernelGGL(k_sai_recon, ge, dim3(256), 0, st, td);
}

int sai_solve_groups(int C, int R, int bw) {
  const int cpw = sai_chunks_per_group(R, bw);
  return (C + cpw - 1) / cpw;
}

void launch_sai_gram(ProbDev* d, TriDev* td, int nprob, int64_t maxn, double* part, hipStream_t st) {
  hipLaunchKernelGGL(k_sai_gram, dim3((unsigned)((maxn + kGramRows - 1) / kGramRows), (unsigned)nprob),
                     dim3(kGramRows), 0, st, d, td, part);
}

void launch_hess_inverse(TriDev* td, int nprob, int maxN0, int maxbw, int maxl, hipStream_t st) {
  static bool attr = false;
  if (!attr) {
    const void* fns[2] = {(const void*)k_hess_inv<true>, (const void*)k_hess_inv<false>};
    for (const void* f : fns)
      if (hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024) != hipSuccess)
        (void)hipGetLastError();
    attr = true;
  }
  {
    const unsigned gi = (unsigned)std::min<int64_t>(1024, ((int64_t)maxN0 * maxN0 + 255) / 256);
    hipLaunchKernelGGL(k_lu_init, dim3(gi, (unsigned)nprob), dim3(256), 0, st, td);
    const dim3 gt((unsigned)((maxN0 + 3) / 4), (unsigned)nprob);
    for (int jb = 0; jb < maxl; ++jb) {
      hipLaunchKernelGGL(k_lu_panel, dim3((unsigned)nprob), dim3(64), 0, st, td, jb);
      hipLaunchKernelGGL(k_lu_trail, gt, dim3(256), 0, st, td, jb);
    }
  }
  // four columns in LDS plus a work region (the staged multipliers, N0 x 2 bw, when they
  // fit -- else read in place -- then blocks of U's columns)
  const size_t ldsfull = sizeof(double) * kSaiLdsDoubles;
  const bool stage = (size_t)4 * maxN0 + (size_t)2 * maxbw * maxN0 <= (size_t)kSaiLdsDoubles;
  if (stage)
    hipLaunchKernelGGL(k_hess_inv<true>, dim3((unsigned)((maxN0 + 3) / 4), (unsigned)nprob), dim3(256), ldsfull, st,
                       td);
  else
    hipLaunchKernelGGL(k_hess_inv<false>, dim3((unsigned)((maxN0 + 3) / 4), (unsigned)nprob), dim3(256), ldsfull, st,
                       td);
}

}  // namespace pe
