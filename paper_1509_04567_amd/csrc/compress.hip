// Truncated SVD of the shifted source samples (Sec. 2.1, eqs. 2.2-2.3) on gfx950:
// a column-pivoted Gram-Schmidt range finder.
//
// The samples G^ (n x s, one column per sample time) are strongly correlated in time, so
// an unpivoted QR meets nearly parallel columns early and keeps rounding noise as new
// directions.  Here each step instead takes the column of the residual A = (I - Q Q^T) G^
// with the largest norm (Businger-Golub pivoting), orthogonalises it against Q twice
// (classical Gram-Schmidt with one reorthogonalisation), appends it to Q and removes its
// direction from every residual column.  The loop stops when the residual's Frobenius
// norm is below max(1e-15, 2 k eps) |G^|_F (k columns taken: the residual's rounding
// level) or at a column cap.  R = Q^T G^ is then formed from the samples
// themselves (not from the residual), so directions taken from rounding noise carry
// rounding-size rows only; the singular values of G^ are those of R (the SVD of R is
// done by the one-sided Jacobi kernel), and the residual energy counts towards the
// dropped tail.
//
// Every kernel works on a 2-D grid of (row chunk, 64-column group) tiles; reductions
// over row chunks go through per-workgroup partials and the last workgroup to arrive
// (write-through stores at agent scope, atomic counter), in a fixed order, so results
// do not depend on scheduling.
#include "devutil.h"
#include "kernels.h"

namespace pe {

namespace {

constexpr int kCpCols = 64;  // columns per column group (one per lane of a 64-wide tile)

// state of the range finder (device memory)
struct CpState {
  int k;         // columns of Q so far
  int done;      // 1: stop (residual below the floor, column cap, or exact rank found)
  int piv;       // pivot column of the current step
  int kcap;      // column cap
  double gfro2;  // |G^|_F^2
  double thr2;   // residual floor (squared) of the last stop test
  double qnorm;  // norm of the reorthogonalised pivot column
  double res2;   // |A|_F^2 after the last step
  double c[kCpMaxK];  // projections of the pivot column on Q (both passes)
};

struct CpArgs {
  int64_t n;
  int s, rw, P, CG;   // rows per chunk, row chunks, column groups
  const double* G;    // n x s (ld n): shifted samples
  double* A;          // n x s (ld n): residual
  double* Q;          // n x kcap (ld n)
  double* R;          // kcap x s (ld kcap)
  double* part;       // partials
  double* cn2;        // s: squared residual column norms
  double* rrow;       // s: q^T A of the current step
  unsigned* cnt;      // counters: [0] second level, [1 + g] per column group
  CpState* st;
};

// The last workgroup of column group g to finish (over the P row chunks) returns true; the
// caller then reduces that group's partials.  cnt[1 + g] is reset by that workgroup.
__device__ __forceinline__ bool group_last(const CpArgs& a, int g, int* flag) {
  if (!arrive_last(a.cnt + 1 + g, (unsigned)a.P, flag)) return false;
  if (threadIdx.x == 0) atomicExch(a.cnt + 1 + g, 0u);
  return true;
}

// the last of the column-group reducers (second level); resets cnt[0]
__device__ __forceinline__ bool all_last(const CpArgs& a, int* flag) {
  if (!arrive_last(a.cnt, (unsigned)a.CG, flag)) return false;
  if (threadIdx.x == 0) atomicExch(a.cnt, 0u);
  return true;
}

// column partial sums of this tile (rows [r0, r1), columns of group g): wave w takes
// columns w, w + 4, ... of the group; f(r, j) gives the term of row r, column j
template <typename F>
__device__ __forceinline__ void tile_col_partials(const CpArgs& a, int64_t r0, int64_t r1, int g, F f) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int jj = w; jj < kCpCols; jj += 4) {
    const int j = g * kCpCols + jj;
    if (j >= a.s) break;
    double acc = 0.0;
    for (int64_t r = r0 + lane; r < r1; r += 64) acc += f(r, j);
    acc = wave_sum(acc);
    if (lane == 0) st_agent(a.part + (int64_t)blockIdx.x * a.s + j, acc);
  }
}

// the group's last workgroup: out[j] = sum over row chunks of the partials, j in group g
__device__ __forceinline__ void reduce_group(const CpArgs& a, int g, double* out) {
  for (int jj = threadIdx.x; jj < kCpCols; jj += blockDim.x) {
    const int j = g * kCpCols + jj;
    if (j >= a.s) break;
    double acc = 0.0;
    for (int p = 0; p < a.P; ++p) acc += a.part[(int64_t)p * a.s + j];
    st_agent(out + j, acc);
  }
}

// second level: residual energy, stop test and the next pivot (largest column norm,
// the smallest index among equals)
__device__ void pick_pivot(const CpArgs& a, bool first) {
  __shared__ double rv[256];
  __shared__ int ri[256];
  __shared__ double rs[256];
  const int t = threadIdx.x;
  double best = -1.0, tot = 0.0;
  int bi = 0;
  for (int j = t; j < a.s; j += 256) {
    const double v = a.cn2[j];
    tot += v;
    if (v > best) {
      best = v;
      bi = j;
    }
  }
  rv[t] = best;
  ri[t] = bi;
  rs[t] = tot;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (t < h) {
      const double v2 = rv[t + h];
      const int i2 = ri[t + h];
      if (v2 > rv[t] || (v2 == rv[t] && i2 < ri[t])) {
        rv[t] = v2;
        ri[t] = i2;
      }
      rs[t] += rs[t + h];
    }
    __syncthreads();
  }
  if (t == 0) {
    CpState& S = *a.st;
    if (first) {
      S.gfro2 = rs[0];
      S.k = 0;
      S.done = 0;
    } else {
      S.k += 1;
    }
    // the residual's own rounding grows with the columns taken (~k eps |G^|_F): below
    // that level it carries no direction, so the loop stops there as well
    const double fl = fmax(kCpFloor, 2.0 * S.k * 2.220446049250313e-16);
    S.thr2 = fl * fl * S.gfro2;
    S.res2 = rs[0];
    S.piv = ri[0];
    if (!(rs[0] > S.thr2) || !(rv[0] > 0.0) || S.k >= S.kcap) S.done = 1;
  }
}

// zero counters, fresh state
__global__ void k_cp_reset(CpArgs a, int kcap) {
  for (int i = threadIdx.x; i < 1 + a.CG; i += blockDim.x) a.cnt[i] = 0u;
  if (threadIdx.x == 0) {
    CpState& S = *a.st;
    S.k = 0;
    S.done = 0;
    S.piv = 0;
    S.kcap = kcap;
    S.gfro2 = S.thr2 = S.qnorm = S.res2 = 0.0;
  }
}

// A = G^ and its squared column norms; first pivot
__global__ __launch_bounds__(256) void k_cp_init(CpArgs a) {
  __shared__ int flag;
  const int g = blockIdx.y;
  const int64_t r0 = (int64_t)blockIdx.x * a.rw, r1 = min(a.n, r0 + a.rw);
  tile_col_partials(a, r0, r1, g, [&](int64_t r, int j) {
    const double v = a.G[(int64_t)j * a.n + r];
    a.A[(int64_t)j * a.n + r] = v;
    return v * v;
  });
  if (!group_last(a, g, &flag)) return;
  reduce_group(a, g, a.cn2);
  if (!all_last(a, &flag)) return;
  pick_pivot(a, true);
}

// pass = 0: c = Q[:, :k]^T a_piv; pass = 1: c += Q^T a1 with a1 = a_piv - Q c, and the
// norm of a1 - Q (Q^T a1) (Pythagoras, a1 being orthogonal to Q up to the first pass's
// rounding).  One row chunk per workgroup, wave w takes columns w, w + 4, ... of Q.
__global__ __launch_bounds__(256) void k_cp_qdots(CpArgs a, int pass) {
  __shared__ int flag;
  __shared__ double v[kCpMaxRw];
  const CpState& S = *a.st;
  if (S.done) return;
  const int k = S.k, piv = S.piv;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int64_t r0 = (int64_t)blockIdx.x * a.rw, r1 = min(a.n, r0 + a.rw);
  const int rows = (int)(r1 - r0);
  const int stride = kCpMaxK + 1;
  for (int rr = t; rr < rows; rr += 256) {
    double x = a.A[(int64_t)piv * a.n + r0 + rr];
    if (pass == 1)
      for (int i = 0; i < k; ++i) x -= a.Q[(int64_t)i * a.n + r0 + rr] * S.c[i];
    v[rr] = x;
  }
  __syncthreads();
  for (int i = w; i < k; i += 4) {
    double acc = 0.0;
    for (int rr = lane; rr < rows; rr += 64) acc += a.Q[(int64_t)i * a.n + r0 + rr] * v[rr];
    acc = wave_sum(acc);
    if (lane == 0) st_agent(a.part + (int64_t)blockIdx.x * stride + i, acc);
  }
  if (pass == 1 && w == 0) {
    double acc = 0.0;
    for (int rr = lane; rr < rows; rr += 64) acc += v[rr] * v[rr];
    acc = wave_sum(acc);
    if (lane == 0) st_agent(a.part + (int64_t)blockIdx.x * stride + kCpMaxK, acc);
  }
  if (!arrive_last(a.cnt, (unsigned)a.P, &flag)) return;
  if (t == 0) atomicExch(a.cnt, 0u);
  CpState& Sw = *a.st;
  __shared__ double c2[kCpMaxK + 1];
  for (int i = t; i < (pass == 1 ? kCpMaxK + 1 : k); i += 256) {
    if (i < k || i == kCpMaxK) {
      double acc = 0.0;
      for (int p = 0; p < a.P; ++p) acc += a.part[(int64_t)p * stride + i];
      c2[i] = acc;
    }
  }
  __syncthreads();
  if (t == 0) {
    if (pass == 0) {
      for (int i = 0; i < k; ++i) Sw.c[i] = c2[i];
    } else {
      double s2 = 0.0;
      for (int i = 0; i < k; ++i) {
        Sw.c[i] += c2[i];
        s2 += c2[i] * c2[i];
      }
      const double q2 = c2[kCpMaxK] - s2;
      Sw.qnorm = q2 > 0.0 ? sqrt(q2) : 0.0;
      if (!(Sw.qnorm > 0.0)) Sw.done = 1;  // the pivot column lies in span(Q): rank found
    }
  }
}

// q = (a_piv - Q c) / qnorm into Q[:, k] (written by column group 0), and the partials of
// r = q^T A over this tile; the group's last workgroup reduces r for its columns
__global__ __launch_bounds__(256) void k_cp_qform(CpArgs a) {
  __shared__ int flag;
  __shared__ double q[kCpMaxRw];
  const CpState& S = *a.st;
  if (S.done) return;
  const int k = S.k, piv = S.piv, g = blockIdx.y;
  const double inv = 1.0 / S.qnorm;
  const int t = threadIdx.x;
  const int64_t r0 = (int64_t)blockIdx.x * a.rw, r1 = min(a.n, r0 + a.rw);
  const int rows = (int)(r1 - r0);
  for (int rr = t; rr < rows; rr += 256) {
    double x = a.A[(int64_t)piv * a.n + r0 + rr];
    for (int i = 0; i < k; ++i) x -= a.Q[(int64_t)i * a.n + r0 + rr] * S.c[i];
    x *= inv;
    q[rr] = x;
    if (g == 0) a.Q[(int64_t)k * a.n + r0 + rr] = x;
  }
  __syncthreads();
  tile_col_partials(a, r0, r1, g, [&](int64_t r, int j) { return q[r - r0] * a.A[(int64_t)j * a.n + r]; });
  if (!group_last(a, g, &flag)) return;
  reduce_group(a, g, a.rrow);
}

// A -= q r^T on this tile and the new squared column norms; second level: residual
// energy, stop test, next pivot
__global__ __launch_bounds__(256) void k_cp_update(CpArgs a) {
  __shared__ int flag;
  const CpState& S = *a.st;
  if (S.done) return;
  const int k = S.k, g = blockIdx.y;
  const int64_t r0 = (int64_t)blockIdx.x * a.rw, r1 = min(a.n, r0 + a.rw);
  const double* q = a.Q + (int64_t)k * a.n;
  tile_col_partials(a, r0, r1, g, [&](int64_t r, int j) {
    const double x = a.A[(int64_t)j * a.n + r] - q[r] * a.rrow[j];
    a.A[(int64_t)j * a.n + r] = x;
    return x * x;
  });
  if (!group_last(a, g, &flag)) return;
  reduce_group(a, g, a.cn2);
  if (!all_last(a, &flag)) return;
  pick_pivot(a, false);
}

// R = Q[:, :k]^T G^ (k x s, ld kcap): each tile stages 32-row slices of Q and of its
// column group of G^ in LDS; thread t accumulates outputs (i, jj) = t, t + 256, ...; the
// group's last workgroup reduces over row chunks.
__global__ __launch_bounds__(256) void k_cp_rfinal(CpArgs a) {
  constexpr int kSl = 32;  // rows per LDS slice
  __shared__ int flag;
  __shared__ double qs[kSl * kCpMaxK];
  __shared__ double gs[kSl * kCpCols];
  const int k = a.st->k, g = blockIdx.y, t = threadIdx.x;
  if (k == 0) return;
  const int64_t r0 = (int64_t)blockIdx.x * a.rw, r1 = min(a.n, r0 + a.rw);
  const int ncol = min(kCpCols, a.s - g * kCpCols);
  const int nout = k * ncol;
  constexpr int kOut = (kCpMaxK * kCpCols + 255) / 256;
  double acc[kOut];
#pragma unroll
  for (int o = 0; o < kOut; ++o) acc[o] = 0.0;
  for (int64_t b0 = r0; b0 < r1; b0 += kSl) {
    const int rows = (int)min<int64_t>(kSl, r1 - b0);
    __syncthreads();
    for (int e = t; e < kSl * k; e += 256) {
      const int i = e / kSl, rr = e % kSl;
      qs[rr * kCpMaxK + i] = rr < rows ? a.Q[(int64_t)i * a.n + b0 + rr] : 0.0;
    }
    for (int e = t; e < kSl * ncol; e += 256) {
      const int jj = e / kSl, rr = e % kSl;
      gs[rr * kCpCols + jj] = rr < rows ? a.G[(int64_t)(g * kCpCols + jj) * a.n + b0 + rr] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int o = 0; o < kOut; ++o) {
      const int e = t + 256 * o;
      if (e < nout) {
        const int i = e / ncol, jj = e % ncol;
        double s = 0.0;
        for (int rr = 0; rr < rows; ++rr) s += qs[rr * kCpMaxK + i] * gs[rr * kCpCols + jj];
        acc[o] += s;
      }
    }
  }
  // partials: k x ncol per tile, at part[(chunk * CG + g) * kCpMaxK * kCpCols + e]
  double* mine = a.part + ((int64_t)blockIdx.x * a.CG + g) * (kCpMaxK * kCpCols);
#pragma unroll
  for (int o = 0; o < kOut; ++o) {
    const int e = t + 256 * o;
    if (e < nout) st_agent(mine + e, acc[o]);
  }
  if (!group_last(a, g, &flag)) return;
  for (int e = t; e < nout; e += 256) {
    double s = 0.0;
    for (int p = 0; p < a.P; ++p) s += a.part[((int64_t)p * a.CG + g) * (kCpMaxK * kCpCols) + e];
    const int i = e / ncol, jj = e % ncol;
    a.R[(int64_t)i + (int64_t)a.st->kcap * (g * kCpCols + jj)] = s;
  }
}

}  // namespace

// geometry: rows per chunk (a multiple of 64, at most kCpMaxRw) and the counts
void cp_geometry(int64_t n, int s, int& rw, int& P, int& CG) {
  int64_t r = 256;
  while ((n + r - 1) / r > 512 && r < kCpMaxRw) r *= 2;
  rw = (int)r;
  P = (int)((n + r - 1) / r);
  CG = (s + kCpCols - 1) / kCpCols;
}

size_t cp_part_doubles(int64_t n, int s) {
  int rw, P, CG;
  cp_geometry(n, s, rw, P, CG);
  const size_t a = (size_t)P * s;
  const size_t b = (size_t)P * (kCpMaxK + 1);
  const size_t c = (size_t)P * CG * kCpMaxK * kCpCols;
  return std::max(a, std::max(b, c));
}

size_t cp_state_bytes() { return sizeof(CpState); }

void launch_cp_range(int64_t n, int s, int kcap, const double* G, double* A, double* Q, double* R, double* part,
                     double* cn2, double* rrow, unsigned* cnt, void* state, hipStream_t st) {
  CpArgs a;
  a.n = n;
  a.s = s;
  cp_geometry(n, s, a.rw, a.P, a.CG);
  a.G = G;
  a.A = A;
  a.Q = Q;
  a.R = R;
  a.part = part;
  a.cn2 = cn2;
  a.rrow = rrow;
  a.cnt = cnt;
  a.st = (CpState*)state;
  // counters and state are set by a kernel (no memset or host copy in the launch sequence)
  hipLaunchKernelGGL(k_cp_reset, dim3(1), dim3(256), 0, st, a, kcap);
  const dim3 g2((unsigned)a.P, (unsigned)a.CG), g1((unsigned)a.P);
  hipLaunchKernelGGL(k_cp_init, g2, dim3(256), 0, st, a);
  for (int it = 0; it < kcap; ++it) {
    hipLaunchKernelGGL(k_cp_qdots, g1, dim3(256), 0, st, a, 0);
    hipLaunchKernelGGL(k_cp_qdots, g1, dim3(256), 0, st, a, 1);
    hipLaunchKernelGGL(k_cp_qform, g2, dim3(256), 0, st, a);
    hipLaunchKernelGGL(k_cp_update, g2, dim3(256), 0, st, a);
  }
  hipLaunchKernelGGL(k_cp_rfinal, g2, dim3(256), 0, st, a);
}

void read_cp_state(const void* host_copy, int* k, double* gfro2, double* res2) {
  const CpState* S = (const CpState*)host_copy;
  *k = S->k;
  *gfro2 = S->gfro2;
  *res2 = S->res2;
}

}  // namespace pe
