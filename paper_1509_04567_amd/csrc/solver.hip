// Host orchestration and C ABI of the gfx950 Paraexp library.
//
// pe_solve_batch runs, for every window subproblem (paper Sec. 2.2, Fig. 2.1):
//   S1  shifted samples G^ = G + (L u0) 1^T                          (eq. 2.6)
//   S2-S3  block CGS2+TSQR factorisation G^ = Q R, one-sided Jacobi SVD of R,
//          truncation to m columns: G^ ~= U C                          (eqs. 2.2-2.3)
//   S4  least-squares Chebyshev fit of C in time: p(t) = Pi T(x(t))
//   S5-S7  restarted block Arnoldi on the Krylov space of [U | x] (eq. 2.4), one
//          restart cycle per time sub-step: the exponential of the projected matrix
//          augmented with the polynomial source gives the state at the end of the
//          sub-step; cycle ends are placed at output times and at the window end.
// All problems of a batch advance together: every kernel launch serves the whole
// batch, and the step-size decision of each problem is taken on the host from one
// small read-back per trial.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/paraexp.h"
#include "../../include/paraexp_policy.h"
#include "kernels.h"
#include "policy.h"

// ---- fixed device scratch of the no-allocation entry point (pe_compress_noalloc) ----
// One file-scope device array per GPU, alive until the process ends.  In host code the
// array's name is only a stand-in: its device address, on each device, comes from
// hipGetSymbolAddress (taken once per device, with that device current, by pe_create)
// and only that address is ever handed to kernels or copies.  Calls that overlap on one
// GPU share the array and race.
constexpr size_t kScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) char scratch[kScratchBytes];
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static char* g_scratch_ptr[kMaxDevices] = {};
static hipError_t g_scratch_err[kMaxDevices] = {};
// host buffer of the no-allocation entry point: read-backs of the range finder's state,
// singular values, permutation and fit summary (kept in the context, sized at creation)
constexpr size_t kScratchHostDoubles = 1024;

// Block-kernel tiling chosen by pe_autotune for a (grid-size bucket, block width,
// precision): rows per update chunk and per projection chunk.
struct TuneKey {
  int nlog2, bw, mixed;
  bool operator<(const TuneKey& o) const {
    return nlog2 != o.nlog2 ? nlog2 < o.nlog2 : (bw != o.bw ? bw < o.bw : mixed < o.mixed);
  }
};
struct TuneVal {
  int rows_u, rows_p;
};
using TuneTable = std::map<TuneKey, TuneVal>;

struct pe_ctx {
  int device = 0;
  TuneTable tune;  // pe_autotune's choices, consulted by every call on this context
  std::string err;
  char* arena = nullptr;
  size_t arena_cap = 0;
  // buffers that live across the calls using the arena: the compressed sources of
  // pe_solve_batch, the iterates and window sources of pe_wr_burgers; grown on demand and
  // kept like the arena
  char* keep = nullptr;
  size_t keep_cap = 0;
  char* keep_wr = nullptr;
  size_t keep_wr_cap = 0;
  char* pinned = nullptr;
  size_t pinned_cap = 0;
  // kernel timing (pe_profile_enable / pe_profile_read)
  std::string prof_name;
  std::vector<hipEvent_t> ev;
  struct Pending {
    int e0;
    double bytes, flops;
  };
  std::vector<Pending> pend;
  size_t ev_used = 0;
  int64_t prof_launches = 0;
  double prof_ms = 0.0, prof_bytes = 0.0, prof_flops = 0.0;
  bool prof_sample = true;  // false: the current restart cycle is not timed
  // workspace query: ensure_arena records the size and stops the call there
  bool query = false;
  size_t query_bytes = 0;
  // no-allocation entry point: device address of this device's scratch array, host buffer
  char* scratch_dev = nullptr;
  double scratch_host[kScratchHostDoubles];
};

static pe_status pe_fail(pe_ctx* ctx, pe_status st, const std::string& msg, hipError_t e = hipSuccess) {
  if (ctx) {
    ctx->err = msg;
    if (e != hipSuccess) ctx->err += std::string(": ") + hipGetErrorString(e);
  }
  return st;
}

#define HCK(expr)                                                                     \
  do {                                                                                \
    hipError_t _e = (expr);                                                           \
    if (_e != hipSuccess) return pe_fail(ctx, PE_ERR_DEVICE, #expr, _e);             \
  } while (0)

namespace {

// ---- kernel timing with HIP events on the launch stream ----------------------------
int prof_begin(pe_ctx* ctx, const char* family, hipStream_t st) {
  if (!ctx->prof_sample || ctx->prof_name.empty() || ctx->prof_name != family) return -1;
  while (ctx->ev.size() < ctx->ev_used + 2) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return -1;
    ctx->ev.push_back(e);
  }
  const int i = (int)ctx->ev_used;
  ctx->ev_used += 2;
  if (hipEventRecord(ctx->ev[i], st) != hipSuccess) return -1;
  return i;
}

void prof_end(pe_ctx* ctx, int i, double bytes, double flops, hipStream_t st) {
  if (i < 0) return;
  (void)hipEventRecord(ctx->ev[i + 1], st);
  ctx->pend.push_back({i, bytes, flops});
}

// after the stream is synchronised: fold the recorded launches into the totals
void prof_collect(pe_ctx* ctx) {
  for (const auto& p : ctx->pend) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, ctx->ev[p.e0], ctx->ev[p.e0 + 1]) == hipSuccess) {
      ctx->prof_ms += ms;
      ctx->prof_bytes += p.bytes;
      ctx->prof_flops += p.flops;
      ++ctx->prof_launches;
    }
  }
  ctx->pend.clear();
  ctx->ev_used = 0;
}

constexpr double kTaylorTheta = 0.78;  // ||A||_1 bound for the degree-16 Taylor polynomial
constexpr int kMaxTrials = 6;
// truncation floor: singular values at or below kSigmaFloor sigma_1 are never kept
constexpr double kSigmaFloor = 1e-14;
// dependence tolerances of the block QR: the compression resolves the sample matrix to
// an absolute ~1e-14 of its column norms (below the truncation floor's reach); the
// Arnoldi process deflates remainders below 1e-12 of the pre-projection norm
constexpr double kDepTolCompress = 1e-14;
constexpr double kDepTolArnoldi = 1e-12;
constexpr int kRowsU = 64;

// shift-and-invert: gamma = kSaiShift times the step a restart cycle aims at, unless the
// problem sets its own factor
constexpr double kSaiShift = 0.1;
// largest projected dimension l bw of a shift-and-invert cycle (the inverse of the
// projected matrix keeps four of its columns and one of U's in LDS)
constexpr int kSaiMaxN0 = 4000;
// chunks of the partitioned tridiagonal solve: a power of two (the interface system is
// solved by cyclic reduction), at most 256 and with at least 16 rows each; the rows per
// chunk follow (the last chunk takes the remainder)
void sai_chunking(int64_t n, int& R, int& C) {
  C = 1;
  while (2 * C <= 256 && 2 * (int64_t)C * 16 <= n) C *= 2;
  // the last chunk takes the remainder; the solve kernels hold R..2R-1 rows per chunk
  // (LDS staging, sweeps), so C is halved until the remainder is below R
  while (C > 1 && n % C >= n / C) C /= 2;
  R = (int)(n / C);
}
int sai_red_doubles(int C) {
  int lev = 0;
  while ((1 << lev) < C) ++lev;
  return 8 * C * lev + 4 * C + 4;
}

// bound on the re-expansion growth of the Chebyshev source basis over one step
constexpr double kGrowthCap = 100.0;
// An output spacing that matches the held propagator's step to this relative accuracy is
// reached with it: the time offset, at most kPropRel delta, moves the result by about
// kPropRel delta |u'|, far below any tolerance the march accepts.
constexpr double kPropRel = 1e-13;
// restart cycles of a march between two timed ones (pe_profile_enable)
constexpr int kProfEvery = 1;
// restart cycles per march before it gives up (flagged, unreached outputs NaN)
constexpr int kCycleCap = 100000;

// PARAEXP_TRACE=1 prints one line per restart trial to stderr;
// PARAEXP_MAX_CYCLES=k lowers the cycle cap to k.
int env_int(const char* name, int dflt) {
  const char* v = std::getenv(name);
  return v ? std::atoi(v) : dflt;
}

// ---- workspace carving ----------------------------------------------------------
struct Carver {
  size_t off = 0;
  template <typename T>
  size_t take(size_t count) {
    off = (off + 255) & ~(size_t)255;
    size_t o = off;
    off += count * sizeof(T);
    return o;
  }
};

// status of a call stopped by a workspace query at its first allocation (never returned
// through the ABI)
constexpr pe_status kQueryStop = (pe_status)1;

pe_status ensure_arena(pe_ctx* ctx, size_t bytes) {
  if (ctx->query) {
    ctx->query_bytes = std::max(ctx->query_bytes, bytes);
    return kQueryStop;
  }
  if (bytes <= ctx->arena_cap) return PE_OK;
  if (ctx->arena) {
    hipDeviceSynchronize();
    hipFree(ctx->arena);
    ctx->arena = nullptr;
    ctx->arena_cap = 0;
  }
  size_t cap = bytes + bytes / 4 + (1 << 20);
  hipError_t e = hipMalloc((void**)&ctx->arena, cap);
  if (e != hipSuccess) return pe_fail(ctx, PE_ERR_OOM, "device workspace allocation failed", e);
  ctx->arena_cap = cap;
  return PE_OK;
}

// one of the context's kept device buffers (pe_ctx::keep, keep_wr), at least `bytes`
pe_status ensure_kept(pe_ctx* ctx, char*& buf, size_t& cap, size_t bytes) {
  if (bytes <= cap) return PE_OK;
  if (buf) {
    hipDeviceSynchronize();
    hipFree(buf);
    buf = nullptr;
    cap = 0;
  }
  const size_t c = bytes + bytes / 4 + (1 << 20);
  hipError_t e = hipMalloc((void**)&buf, c);
  if (e != hipSuccess) return pe_fail(ctx, PE_ERR_OOM, "device workspace allocation failed", e);
  cap = c;
  return PE_OK;
}

pe_status ensure_pinned(pe_ctx* ctx, size_t bytes) {
  if (bytes <= ctx->pinned_cap) return PE_OK;
  if (ctx->pinned) hipHostFree(ctx->pinned);
  ctx->pinned = nullptr;
  ctx->pinned_cap = 0;
  size_t cap = bytes + 4096;
  hipError_t e = hipHostMalloc((void**)&ctx->pinned, cap);
  if (e != hipSuccess) return pe_fail(ctx, PE_ERR_OOM, "pinned host allocation failed", e);
  ctx->pinned_cap = cap;
  return PE_OK;
}

// ---- geometry of the block kernels ------------------------------------------------
size_t update_smem(const ProbDev& d);
size_t proj_smem(const ProbDev& d);
int rows_p_for(int bw) { return bw <= 8 ? 128 : (bw <= 16 ? 64 : 32); }

// Rows per update chunk: kRowsU when the update kernel (chunk staging plus a register- or
// LDS-resident TSQR combine) fits in LDS; else the smallest power of two from kRowsU up
// for which the two-level combine (groups of kTreeFan chunk factors, then the stacked
// group factors, each in LDS) fits; else the smallest with a one-level LDS combine; when
// none does (wide blocks on long grids), the largest chunk whose staging fits, with the
// combine working on the stacked chunk factors in global memory.
void choose_update_chunks(int64_t n, int bw, int& rows_u, int& comb_global, int& comb_tree) {
  comb_tree = 0;
  {
    ProbDev d{};
    d.bw = bw;
    d.rows_u = kRowsU;
    d.Cu = (int)std::max<int64_t>(1, n / kRowsU);
    if (update_smem(d) <= (size_t)pe::kUpdateLdsMax) {
      rows_u = kRowsU;
      comb_global = 0;
      return;
    }
  }
  for (int ru = kRowsU; ru <= 1024; ru *= 2) {
    ProbDev d{};
    d.bw = bw;
    d.rows_u = ru;
    d.Cu = (int)std::max<int64_t>(1, n / ru);
    d.comb_tree = 1;
    if (update_smem(d) <= (size_t)pe::kUpdateLdsMax) {
      rows_u = ru;
      comb_global = 0;
      comb_tree = 1;
      return;
    }
  }
  for (int glob = 0; glob < 2; ++glob) {
    int best = 0;
    for (int ru = kRowsU; ru <= 4096; ru *= 2) {
      ProbDev d{};
      d.bw = bw;
      d.rows_u = ru;
      d.Cu = (int)std::max<int64_t>(1, n / ru);
      d.comb_global = glob;
      if (update_smem(d) <= (size_t)pe::kUpdateLdsMax) {
        best = ru;
        if (!glob) break;
      }
    }
    if (best) {
      rows_u = best;
      comb_global = glob;
      return;
    }
  }
  rows_u = kRowsU;  // nothing fits: geometry_fits reports it
  comb_global = 1;
}

// the tuning table of the call in progress (pe_autotune's choices on its context), or null
thread_local const TuneTable* g_tune = nullptr;
struct TuneScope {
  explicit TuneScope(const pe_ctx* c) { g_tune = c ? &c->tune : nullptr; }
  ~TuneScope() { g_tune = nullptr; }
};
int tune_nlog2(int64_t n) {
  int k = 0;
  while (((int64_t)1 << k) < n) ++k;
  return k;
}

// update-chunk layout for a given chunk height: the combine placement as in
// choose_update_chunks (registers or LDS, else two-level, else global); false when even
// the staging does not fit
bool update_chunks_for(int64_t n, int bw, int ru, int& comb_global, int& comb_tree) {
  for (int mode = 0; mode < 3; ++mode) {
    ProbDev d{};
    d.bw = bw;
    d.rows_u = ru;
    d.Cu = (int)std::max<int64_t>(1, n / ru);
    d.comb_tree = mode == 1;
    d.comb_global = mode == 2;
    if (update_smem(d) <= (size_t)pe::kUpdateLdsMax) {
      comb_global = d.comb_global;
      comb_tree = d.comb_tree;
      return true;
    }
  }
  return false;
}

void set_geometry(ProbDev& d, int64_t n, int bw) {
  d.bw = bw;
  choose_update_chunks(n, bw, d.rows_u, d.comb_global, d.comb_tree);
  int tuned_p = 0;
  if (g_tune) {
    auto it = g_tune->find(TuneKey{tune_nlog2(n), bw, d.mixed});
    if (it != g_tune->end()) {
      int cg, ct;
      // chunk heights are powers of two (chunk_of shifts by rows_u_log2); anything else
      // in the table is ignored
      const int ru = it->second.rows_u, rp = it->second.rows_p;
      if (ru >= 64 && ru <= 4096 && (ru & (ru - 1)) == 0 && ru <= n && update_chunks_for(n, bw, ru, cg, ct)) {
        d.rows_u = ru;
        d.comb_global = cg;
        d.comb_tree = ct;
      }
      if (rp >= 16 && (rp & (rp - 1)) == 0 && rp * bw <= 1024) tuned_p = rp;
    }
  }
  d.rows_u_log2 = 0;
  while ((1 << d.rows_u_log2) < d.rows_u) ++d.rows_u_log2;
  d.Cu = (int)std::max<int64_t>(1, n / d.rows_u);
  d.rows_p = tuned_p ? tuned_p : rows_p_for(bw);  // rows_p * bw <= 1024: the projection kernel's staging assumes it
  d.Cp = (int)((n + d.rows_p - 1) / d.rows_p);
}

size_t proj_smem(const ProbDev& d) {
  const size_t ld = d.bw + 1;
  const size_t qsl = (size_t)(d.rows_p / d.rows_u + 4) * d.bw * d.bw;
  const size_t qrow = (size_t)(d.rows_p + 2) * d.bw;
  (void)ld;
  return sizeof(double) * ((size_t)d.rows_p * d.bw * (1 + pe::kSlotGroup) + (size_t)(d.rows_p + 2) * d.bw + 256 +
                            qrow + qsl) + 64;
}

size_t update_smem(const ProbDev& d) {
  const size_t ld = d.bw + 1;
  const size_t rmax = 2 * (size_t)d.rows_u;
  const bool reg = pe::combine_in_registers(d.bw, d.Cu);
  const size_t bw2 = (size_t)d.bw * d.bw;
  const size_t ng = (size_t)(d.Cu + pe::kTreeFan - 1) / pe::kTreeFan;
  const size_t xs = d.comb_tree ? ld * std::max(rmax, std::max<size_t>(pe::kTreeFan, ng) * d.bw)
                                : ((reg || d.comb_global || rmax > (size_t)d.Cu * d.bw) ? rmax * ld
                                                                                        : (size_t)d.Cu * d.bw * ld);
  return sizeof(double) * (xs + std::max<size_t>(pe::kSb, (rmax + 2) * d.bw) + bw2 + d.bw + std::max<size_t>(bw2, 128)) +
         64;
}

// capacities of the per-problem block workspace for block widths up to bwmax
struct BlockCaps {
  int64_t n;
  int bwmax, nbmax;
  size_t basis, qloc, rloc, rf, part, S, H, cnt;
  int64_t ldH_rows, H_cols;
};

BlockCaps block_caps(int64_t n, int bwmax, int nbmax, int64_t H_rows, int64_t H_cols) {
  BlockCaps c;
  c.n = n;
  c.bwmax = bwmax;
  c.nbmax = nbmax;
  size_t cu_bw2 = 0, cp_bw2 = 0, ngmax = 0;
  for (int bw = 1; bw <= bwmax; ++bw)
    for (int mixed = 0; mixed < 2; ++mixed) {  // tuned tilings may differ per precision
      ProbDev d{};
      d.mixed = mixed;
      set_geometry(d, n, bw);
      cu_bw2 = std::max(cu_bw2, (size_t)d.Cu * bw * bw);
      cp_bw2 = std::max(cp_bw2, (size_t)d.Cp * bw * bw);
      ngmax = std::max(ngmax, (size_t)(d.Cu + pe::kTreeFan - 1) / pe::kTreeFan);
    }
  c.basis = (size_t)nbmax * n * bwmax;
  c.qloc = (size_t)n * bwmax;
  c.rloc = cu_bw2;
  c.rf = 3 * (size_t)bwmax * bwmax;
  c.part = 2 * (size_t)nbmax * cp_bw2;
  c.S = 2 * (size_t)nbmax * bwmax * bwmax;
  c.H = (size_t)H_rows * H_cols;
  // projection groups (2 passes), update counter, reorth flag, group counters of the
  // two-level combine
  c.cnt = 2 * (size_t)nbmax + 2 + ngmax;
  c.ldH_rows = H_rows;
  c.H_cols = H_cols;
  return c;
}

struct BlockOffsets {
  size_t V, V0, Qloc1, Qloc2, Rloc, Cn, Qs1, Qs2, Rf, Part, S, H, cnt;
};

BlockOffsets carve_block(Carver& cv, const BlockCaps& c, bool mixed) {
  BlockOffsets o;
  o.V = mixed ? cv.take<float>(c.basis) : cv.take<double>(c.basis);
  // mixed: block 0 (the orthonormalised [U | x]) is also kept in fp64 for the projection
  o.V0 = mixed ? cv.take<double>((size_t)c.n * c.bwmax) : 0;
  o.Qloc1 = cv.take<double>(c.qloc);
  o.Qloc2 = cv.take<double>(c.qloc);
  o.Rloc = cv.take<double>(c.rloc);
  o.Cn = cv.take<double>(c.rloc);
  o.Qs1 = cv.take<double>(c.rloc);
  o.Qs2 = cv.take<double>(c.rloc);
  o.Rf = cv.take<double>(c.rf);
  o.Part = cv.take<double>(c.part);
  o.S = cv.take<double>(c.S);
  o.H = cv.take<double>(c.H);
  o.cnt = cv.take<unsigned>(c.cnt);
  return o;
}

void bind_block(ProbDev& d, char* base, const BlockOffsets& o, bool mixed, int nbmax) {
  d.V = mixed ? (double*)(base + o.V0) : (double*)(base + o.V);
  d.V32 = mixed ? (float*)(base + o.V) : nullptr;
  d.mixed = mixed ? 1 : 0;
  d.Qloc1 = (double*)(base + o.Qloc1);
  d.Qloc2 = (double*)(base + o.Qloc2);
  d.Rloc = (double*)(base + o.Rloc);
  d.Cn = (double*)(base + o.Cn);
  d.Qs1 = (double*)(base + o.Qs1);
  d.Qs2 = (double*)(base + o.Qs2);
  d.Rf = (double*)(base + o.Rf);
  d.Part = (double*)(base + o.Part);
  d.S = (double*)(base + o.S);
  d.H = (double*)(base + o.H);
  d.cnt = (unsigned*)(base + o.cnt);
  d.nbmax = nbmax;
}

// host check that a cycle's geometry fits the carved capacities
bool geometry_fits(const ProbDev& d, const BlockCaps& c, int nb_needed) {
  const size_t bw2 = (size_t)d.bw * d.bw;
  if (d.bw < 1 || d.bw > c.bwmax) return false;
  if (nb_needed > c.nbmax) return false;
  if ((size_t)d.Cu * bw2 > c.rloc) return false;
  if (2 * (size_t)d.Cp * c.nbmax * bw2 > c.part) return false;
  if ((size_t)(d.Cu) * d.rows_u > (size_t)c.n + (size_t)d.rows_u) return false;
  if (c.n < d.bw) return false;
  if (update_smem(d) > (size_t)pe::kUpdateLdsMax) return false;
  if (proj_smem(d) > (size_t)pe::kUpdateLdsMax) return false;
  return true;
}

// Chebyshev derivative matrix: T_k' = sum_j D[k][j] T_j, j < k, k - j odd, weight 2k
// (k for j = 0)
std::vector<double> chebyshev_derivative(int qmax) {
  std::vector<double> D((size_t)qmax * qmax, 0.0);
  for (int k = 1; k < qmax; ++k)
    for (int j = k - 1; j >= 0; j -= 2) D[(size_t)k * qmax + j] = (j == 0) ? k : 2.0 * k;
  return D;
}

void chebyshev_values(double x, int q, double* w) {
  double a = 1.0, b = x;
  for (int k = 0; k < q; ++k) {
    if (k == 0) w[k] = 1.0;
    else if (k == 1) w[k] = x;
    else {
      const double v = 2.0 * x * b - a;
      a = b;
      b = v;
      w[k] = v;
    }
  }
}

pe_status validate_problem(pe_ctx* ctx, const pe_problem& p, bool need_samples) {
  if (p.op.n < 4) return pe_fail(ctx, PE_ERR_ARG, "n must be >= 4");
  if (!p.op.coeffs) return pe_fail(ctx, PE_ERR_ARG, "stencil coefficients are null");
  if (!p.u0) return pe_fail(ctx, PE_ERR_ARG, "u0 is null");
  if (!(p.t1 > p.t0)) return pe_fail(ctx, PE_ERR_ARG, "window needs t1 > t0");
  if (p.n_out < 0 || (p.n_out > 0 && (!p.t_out || !p.out))) return pe_fail(ctx, PE_ERR_ARG, "bad outputs");
  if (p.ldOut < p.op.n) return pe_fail(ctx, PE_ERR_ARG, "ldOut < n");
  for (int k = 0; k < p.n_out; ++k) {
    if (!std::isfinite(p.t_out[k])) return pe_fail(ctx, PE_ERR_ARG, "non-finite output time");
    if (k > 0 && p.t_out[k] < p.t_out[k - 1]) return pe_fail(ctx, PE_ERR_ARG, "t_out must be non-decreasing");
    if (!p.shift && p.t_out[k] < p.t0) return pe_fail(ctx, PE_ERR_ARG, "unshifted problem needs t_out >= t0");
  }
  if (p.krylov_steps < 1 || p.krylov_steps > 512) return pe_fail(ctx, PE_ERR_ARG, "krylov_steps out of range");
  if (p.rank_max < 0 || p.rank_max > 31) return pe_fail(ctx, PE_ERR_UNSUPPORTED, "rank_max must be in [0, 31]");
  if (p.q_max < 1 || p.q_max > 64) return pe_fail(ctx, PE_ERR_ARG, "q_max must be in [1, 64]");
  if (!(p.tol > 0.0)) return pe_fail(ctx, PE_ERR_ARG, "tol must be positive");
  if (p.prec != PE_FP64 && p.prec != PE_MIXED) return pe_fail(ctx, PE_ERR_ARG, "unknown precision");
  if (p.krylov != PE_KRYLOV_POLY && p.krylov != PE_KRYLOV_SAI) return pe_fail(ctx, PE_ERR_ARG, "unknown Krylov space");
  if (!(p.sai_shift >= 0.0) || !std::isfinite(p.sai_shift)) return pe_fail(ctx, PE_ERR_ARG, "bad sai_shift");
  if (p.source_fit != PE_FIT_CHEBYSHEV && p.source_fit != PE_FIT_SPLINE)
    return pe_fail(ctx, PE_ERR_ARG, "unknown source fit");
  if (need_samples) {
    if (p.s < 1 || !p.t_samples || !p.G) return pe_fail(ctx, PE_ERR_ARG, "missing source samples");
    if (p.ldG < p.op.n) return pe_fail(ctx, PE_ERR_ARG, "ldG < n");
    for (int i = 0; i < p.s; ++i) {
      if (!std::isfinite(p.t_samples[i])) return pe_fail(ctx, PE_ERR_ARG, "non-finite sample time");
      if (i > 0 && !(p.t_samples[i] > p.t_samples[i - 1]))
        return pe_fail(ctx, PE_ERR_ARG, "t_samples must be strictly increasing");
    }
    if (p.s > 1 && (p.t_samples[0] != p.t0 || p.t_samples[p.s - 1] != p.t1))
      return pe_fail(ctx, PE_ERR_ARG, "t_samples must start at t0 and end at t1");
    if (!(p.svd_tol >= 0.0) || !(p.fit_tol >= 0.0)) return pe_fail(ctx, PE_ERR_ARG, "negative tolerance");
  }
  if (!p.op.per_point)
    for (int i = 0; i < 3; ++i)
      if (!std::isfinite(p.op.coeffs[i])) return pe_fail(ctx, PE_ERR_NONFINITE, "non-finite stencil coefficient");
  return PE_OK;
}

// ---- device finiteness check of caller arrays -------------------------------------
pe_status check_finite_dev(pe_ctx* ctx, const double* x, int64_t n, int cols, int64_t ld, int* dflag, int* hflag,
                           hipStream_t st, const char* what) {
  pe::launch_zero_u32((unsigned*)dflag, 1, st);
  pe::launch_check_finite(x, n, cols, ld, dflag, st);
  HCK(hipMemcpyAsync(hflag, dflag, sizeof(int), hipMemcpyDeviceToHost, st));
  HCK(hipStreamSynchronize(st));
  if (*hflag) return pe_fail(ctx, PE_ERR_NONFINITE, std::string("NaN or Inf in ") + what);
  return PE_OK;
}

// ---- block orthogonalisation driver -------------------------------------------------
// Algorithmic traffic of one block step's pass over all active problems: the
// projection reads the nb basis blocks and the input block; the update reads them again
// and writes the chunk Q factor.
struct StepCost {
  double proj_bytes = 0.0, upd_bytes = 0.0, flops = 0.0;
};

void run_block_step(pe_ctx* ctx, ProbDev* dd, int nprob, int gx_proj, size_t smem_p, int gx_upd, size_t smem_u,
                    int j, int nb, int mode, int mixed, int tree, const StepCost& cost, hipStream_t st) {
  // Timing covers the first pass, which every step runs in full; the second pass runs
  // only where the first lost too much of a column (decided on the device), so its
  // launches do not all carry the algorithmic traffic of the cost model.
  for (int pass = 0; pass < 2; ++pass) {
    int ev = pass == 0 ? prof_begin(ctx, "block_proj", st) : -1;
    pe::launch_block_proj(dd, nprob, gx_proj, smem_p, j, nb, pass, mode, mixed, st);
    prof_end(ctx, ev, cost.proj_bytes, cost.flops, st);
    ev = pass == 0 ? prof_begin(ctx, "block_update", st) : -1;
    pe::launch_block_update(dd, nprob, gx_upd, smem_u, j, nb, pass, mode, mixed, tree, st);
    prof_end(ctx, ev, cost.upd_bytes, cost.flops, st);
  }
}

StepCost step_cost(int64_t n, int bw, int nb, int beta) {
  StepCost c;
  const double blk = (double)n * bw;
  c.proj_bytes = blk * beta * (nb + 1);
  c.upd_bytes = blk * beta * (nb + 1) + blk * 8.0;
  c.flops = 2.0 * nb * blk * bw;
  return c;
}

// ---------------------------------------------------------------------------------
// compression of one problem: S1-S4
// ---------------------------------------------------------------------------------
struct CompressOut {
  int m = 0, q = 0, flags = 0;
  double fit_resid = 0.0, svd_tail = 0.0, sigma1 = 0.0;
  int nsig = 0;                  // singular values resolved (the rest are zero)
  double sigma[pe::kCpMaxK] = {};
};

// Workspace of a call: the context arena (grown on demand) and its pinned host buffer, or
// a fixed device region and host buffer given by the caller (no allocation at all).
struct FixedWs {
  char* dev;
  size_t dev_bytes;
  double* host;
  size_t host_bytes;
};

pe_status compress_one(pe_ctx* ctx, const pe_problem& p, double* U, int64_t ldU, double* Pi, int ldPi,
                       CompressOut& res, hipStream_t st, const FixedWs* fx = nullptr) {
  const int64_t n = p.op.n;
  const int s = p.s;
  const int qcap = std::min(p.q_max, s);
  // columns of the range finder: the numerical rank of the samples, up to kCpMaxK (beyond
  // that the residual's energy is reported in the dropped tail); none when nothing may
  // be kept
  const int kcap = p.rank_max == 0 ? 0 : (int)std::min<int64_t>({(int64_t)s, n, (int64_t)pe::kCpMaxK});
  int cp_rw, cp_P, cp_CG;
  pe::cp_geometry(n, s, cp_rw, cp_P, cp_CG);
  Carver cv;
  const size_t o_lu0 = cv.take<double>(n);
  const size_t o_gh = cv.take<double>((size_t)n * s);
  const size_t o_res = cv.take<double>((size_t)n * s);
  const size_t o_Q = cv.take<double>((size_t)n * std::max(1, kcap));
  const size_t o_R = cv.take<double>((size_t)std::max(1, kcap) * s);
  const size_t o_part = cv.take<double>(pe::cp_part_doubles(n, s));
  const size_t o_cn2 = cv.take<double>(s);
  const size_t o_rrow = cv.take<double>(s);
  const size_t o_cnt = cv.take<unsigned>(1 + (size_t)cp_CG);
  const size_t o_state = cv.take<char>(pe::cp_state_bytes());
  const size_t o_sel = cv.take<int>(std::max(1, kcap));
  const size_t o_A = cv.take<double>((size_t)s * std::max(1, kcap));
  const size_t o_J = cv.take<double>((size_t)std::max(1, kcap) * std::max(1, kcap));
  const size_t o_sig = cv.take<double>(std::max(1, kcap));
  const size_t o_perm = cv.take<int>(std::max(1, kcap));
  const size_t o_info = cv.take<int>(4);
  const size_t o_ts = cv.take<double>(s);
  const size_t o_fw = cv.take<double>(std::max((size_t)s * qcap + (size_t)qcap * qcap + (size_t)32 * qcap + (size_t)32 * s,
                                               (size_t)3 * 32 * s));
  const size_t o_fi = cv.take<double>(4);
  const size_t o_flag = cv.take<int>(4);
  const size_t host_need = std::max(sizeof(double) * (4 * (size_t)std::max(1, kcap) + 64), pe::cp_state_bytes());
  char* base;
  double* hp;
  pe_status stt;
  if (fx) {
    if (cv.off > fx->dev_bytes || host_need > fx->host_bytes)
      return pe_fail(ctx, PE_ERR_UNSUPPORTED, "problem needs " + std::to_string(cv.off) +
                                                  " bytes of device scratch, more than the fixed " +
                                                  std::to_string(fx->dev_bytes));
    base = fx->dev;
    hp = fx->host;
  } else {
    stt = ensure_arena(ctx, cv.off);
    if (stt != PE_OK) return stt;
    stt = ensure_pinned(ctx, host_need);
    if (stt != PE_OK) return stt;
    base = ctx->arena;
    hp = (double*)ctx->pinned;
  }

  // non-finite inputs
  stt = check_finite_dev(ctx, p.u0, n, 1, n, (int*)(base + o_flag), (int*)hp, st, "u0");
  if (stt != PE_OK) return stt;
  stt = check_finite_dev(ctx, p.G, n, s, p.ldG, (int*)(base + o_flag), (int*)hp, st, "G");
  if (stt != PE_OK) return stt;
  if (p.op.per_point) {
    stt = check_finite_dev(ctx, p.op.coeffs, 3 * n, 1, 3 * n, (int*)(base + o_flag), (int*)hp, st, "stencil");
    if (stt != PE_OK) return stt;
  }
  // S1: G^ = G + L u0
  double* Gh = (double*)(base + o_gh);
  double* Lu0 = (double*)(base + o_lu0);
  if (p.shift) {
    pe::launch_stencil_cols(n, p.op.per_point, p.op.coeffs, p.op.coeffs, p.u0, n, Lu0, n, 1, st);
    pe::launch_add_column(n, s, p.G, p.ldG, Lu0, Gh, n, st);
  } else {
    pe::launch_add_column(n, s, p.G, p.ldG, nullptr, Gh, n, st);
  }
  res.nsig = 0;
  res.m = 0;
  // S2-S3: range of G^ by column-pivoted Gram-Schmidt, R = Q^T G^ (k x s, ld kcap)
  double* Qc = (double*)(base + o_Q);
  double* R = (double*)(base + o_R);
  pe::launch_cp_range(n, s, kcap, Gh, (double*)(base + o_res), Qc, R, (double*)(base + o_part),
                      (double*)(base + o_cn2), (double*)(base + o_rrow), (unsigned*)(base + o_cnt), base + o_state, st);
  HCK(hipGetLastError());
  HCK(hipMemcpyAsync(hp, base + o_state, pe::cp_state_bytes(), hipMemcpyDeviceToHost, st));
  HCK(hipStreamSynchronize(st));
  int r = 0;
  double gfro2 = 0.0, res2 = 0.0;
  pe::read_cp_state(hp, &r, &gfro2, &res2);
  if (gfro2 == 0.0 || r == 0) {  // a zero source, or nothing may be kept (rank_max = 0)
    res.sigma1 = 0.0;
    res.svd_tail = gfro2 > 0.0 ? 1.0 : 0.0;
    if (gfro2 > 0.0) res.flags |= PE_FLAG_RANK_CAPPED;
    return PE_OK;
  }
  int sel[pe::kCpMaxK], perm[pe::kCpMaxK];
  double sig[pe::kCpMaxK], tail[pe::kCpMaxK + 1];
  for (int i = 0; i < r; ++i) sel[i] = i;
  HCK(hipMemcpyAsync(base + o_sel, sel, sizeof(int) * r, hipMemcpyHostToDevice, st));
  double* A = (double*)(base + o_A);
  double* J = (double*)(base + o_J);
  pe::launch_jacobi_svd(R, kcap, (int*)(base + o_sel), s, r, A, J, (double*)(base + o_sig), (int*)(base + o_perm),
                        (int*)(base + o_info), st);
  HCK(hipMemcpyAsync(hp, base + o_sig, sizeof(double) * r, hipMemcpyDeviceToHost, st));
  HCK(hipMemcpyAsync(hp + r, base + o_perm, sizeof(int) * r, hipMemcpyDeviceToHost, st));
  HCK(hipStreamSynchronize(st));
  std::memcpy(perm, hp + r, sizeof(int) * r);
  for (int i = 0; i < r; ++i) sig[i] = hp[perm[i]];
  // truncation (the energy rule of the truncated SVD, Sec. 2.1 eq. 2.3): the smallest m
  // with dropped energy <= svd_tol |G^|_F; singular values <= kSigmaFloor sigma_1 are
  // never kept; a cut inside a cluster (|sigma_m - sigma_{m+1}| <= 1e-12 sigma_1) keeps
  // the cluster whole; m is capped at rank_max
  // (the energy left in the range finder's residual belongs to the dropped tail)
  const double gfro = std::sqrt(gfro2);
  tail[r] = std::sqrt(std::max(res2, 0.0));
  for (int i = r - 1; i >= 0; --i) tail[i] = std::sqrt(tail[i + 1] * tail[i + 1] + sig[i] * sig[i]);
  int m = r;
  for (int i = 0; i <= r; ++i)
    if (tail[i] <= p.svd_tol * gfro) {
      m = i;
      break;
    }
  while (m > 0 && sig[m - 1] <= kSigmaFloor * sig[0]) --m;
  while (m > 0 && m < r && std::fabs(sig[m - 1] - sig[m]) <= 1e-12 * sig[0] && sig[m] > kSigmaFloor * sig[0]) ++m;
  if (m > p.rank_max) {
    m = p.rank_max;
    res.flags |= PE_FLAG_RANK_CAPPED;
  }
  res.m = m;
  res.sigma1 = sig[0];
  res.svd_tail = gfro > 0.0 ? tail[m] / gfro : 0.0;
  res.nsig = std::min(r, s);
  for (int i = 0; i < res.nsig; ++i) res.sigma[i] = sig[i];
  if (m == 0) return PE_OK;
  // U = Q J[:, perm[0:m]]  (Q column-major: blocks of width 1)
  pe::launch_form_u(Qc, 1, n, (int*)(base + o_sel), r, J, (int*)(base + o_perm), m, U, ldU, st);
  // S4: Chebyshev fit (or cubic spline) of C = Sigma Z^T rows over the samples
  HCK(hipMemcpyAsync(base + o_ts, p.t_samples, sizeof(double) * s, hipMemcpyHostToDevice, st));
  if (p.source_fit == PE_FIT_SPLINE) {
    pe::launch_spline(A, s, (int*)(base + o_perm), m, (double*)(base + o_ts), Pi, (double*)(base + o_fw), st);
    HCK(hipStreamSynchronize(st));
    res.q = 4;
    res.fit_resid = 0.0;
    return PE_OK;
  }
  pe::launch_fit(A, s, (int*)(base + o_perm), m, (double*)(base + o_ts), p.t0, p.t1, qcap, p.fit_tol, Pi, ldPi,
                 (double*)(base + o_fw), (double*)(base + o_fi), st);
  HCK(hipMemcpyAsync(hp, base + o_fi, sizeof(double) * 3, hipMemcpyDeviceToHost, st));
  HCK(hipStreamSynchronize(st));
  res.q = (int)hp[0];
  res.fit_resid = hp[1];
  if (hp[2] != 0.0) res.flags |= PE_FLAG_FIT_CAPPED;
  return PE_OK;
}

// ---------------------------------------------------------------------------------
// the march: S5-S7 for a batch of problems of one precision
// ---------------------------------------------------------------------------------
struct HostState {
  double tau = 0.0, dlast = 0.0, Tspan = 1.0, ref = 1.0, dgrow = 2.0;
  int k = 0;
  bool xzero = true, done = false;
  int cycles = 0, rejected = 0, steps = 0, flags = 0;
  double resid = 0.0;
  // per-cycle
  bool src = false;
  double target = 0.0, dtry = 0.0, nrm = 0.0;
  int bw = 1, N = 0;
  bool pending = false, accepted = false;
  bool stop = false;  // the march cannot continue (non-finite projected matrix or estimate)
  int level = 0;
  double rho = 1.0;
  double pexp = 0.0;  // local order of the error estimate in the step (0: unknown)
  // dense output: after a step lands on an output time, the next output is tried from
  // the same Krylov space (offsets measured from the cycle start tau_c); a new space is
  // built only when that space cannot reach further than the state already has
  double tau_c = 0.0;
  bool reuse = false;      // the next plan tries the current space first
  bool reuse_now = false;  // this pass evaluates the current space (no new Arnoldi)
  // outputs at a repeated spacing prop_dt (> 0 when Eprop = exp(prop_dt Ht) of the
  // current space is held) are reached by one matrix-vector product from the last one
  double prop_dt = 0.0;
  bool prop_now = false;
  // piecewise-cubic source: the spline piece holding tau; every sample time is a target
  int piece = 0;
};

pe_status march_batch(pe_ctx* ctx, const pe_problem* probs, const int* idx, int nb_prob, const double* const* Ul,
                      const double* const* Pil, const int* ldPil, const int* ml, const int* ql, pe_report* reports,
                      hipStream_t st) {
  if (nb_prob == 0) return PE_OK;
  struct SampleReset {  // launches outside a march are always timed
    pe_ctx* c;
    ~SampleReset() { c->prof_sample = true; }
  } sample_reset{ctx};
  const bool mixed = probs[idx[0]].prec == PE_MIXED;
  int qmax_all = 1;
  for (int ii = 0; ii < nb_prob; ++ii) qmax_all = std::max(qmax_all, ql[ii]);
  // carve
  Carver cv;
  std::vector<BlockCaps> caps(nb_prob);
  std::vector<BlockOffsets> bo(nb_prob);
  std::vector<size_t> o_x(nb_prob), o_e(nb_prob), o_w(nb_prob), o_coef(nb_prob);
  std::vector<int> Nmax(nb_prob);
  int64_t maxn = 0;
  int maxNall = 1, max_lbw = 1;
  for (int ii = 0; ii < nb_prob; ++ii) {
    const pe_problem& p = probs[idx[ii]];
    const int bwmax = ml[ii] + 1;
    const int l = p.krylov_steps;
    caps[ii] = block_caps(p.op.n, bwmax, l + 1, (int64_t)(l + 1) * bwmax, (int64_t)l * bwmax);
    bo[ii] = carve_block(cv, caps[ii], mixed);
    o_x[ii] = cv.take<double>(p.op.n);
    Nmax[ii] = l * bwmax + ql[ii];
    o_e[ii] = cv.take<double>(8 * (size_t)Nmax[ii] * Nmax[ii] + (PE_MAX_LEVELS + 3) * (size_t)Nmax[ii] +
                              2 * (PE_MAX_LEVELS + 1));
    o_w[ii] = cv.take<double>(std::max(1, ql[ii]));
    maxn = std::max<int64_t>(maxn, p.op.n);
    maxNall = std::max(maxNall, Nmax[ii]);
    max_lbw = std::max(max_lbw, l * bwmax);
  }
  // shift-and-invert: factors of I - gamma L, interface system, solve block, residual Gram
  const bool sai = probs[idx[0]].krylov == PE_KRYLOV_SAI;
  struct SaiOff {
    size_t ta, tinv, tc, vL, vR, red, rrhs, ru, W, GW, piv, cnt;
    int R, C;
  };
  std::vector<SaiOff> so(sai ? nb_prob : 0);
  int maxC = 1, maxbwall = 1, sai_groups = 1;
  if (sai)
    for (int ii = 0; ii < nb_prob; ++ii) {
      const pe_problem& p = probs[idx[ii]];
      const int64_t n = p.op.n;
      const int bwmax = ml[ii] + 1;
      SaiOff& o = so[ii];
      sai_chunking(n, o.R, o.C);
      o.ta = cv.take<double>(n);
      o.tinv = cv.take<double>(n);
      o.tc = cv.take<double>(n);
      o.vL = cv.take<double>(n);
      o.vR = cv.take<double>(n);
      o.red = cv.take<double>(sai_red_doubles(o.C));
      o.rrhs = cv.take<double>(2 * (size_t)o.C * bwmax);
      o.ru = cv.take<double>(2 * (size_t)o.C * bwmax);
      o.W = cv.take<double>((size_t)n * bwmax);
      o.GW = cv.take<double>((size_t)bwmax * bwmax);
      o.piv = cv.take<int32_t>((size_t)p.krylov_steps * bwmax);
      o.cnt = cv.take<unsigned>(2);
      maxC = std::max(maxC, o.C);
      maxbwall = std::max(maxbwall, bwmax);
      for (int bw = 1; bw <= bwmax; ++bw) sai_groups = std::max(sai_groups, pe::sai_solve_groups(o.C, o.R, bw));
    }
  const size_t o_td = cv.take<TriDev>(sai ? nb_prob : 1);
  int64_t maxn_all = 1;
  for (int ii = 0; ii < nb_prob; ++ii) maxn_all = std::max<int64_t>(maxn_all, probs[idx[ii]].op.n);
  const size_t o_gpart = cv.take<double>(sai ? (size_t)nb_prob * ((maxn_all + 127) / 128) * 1024 : 1);
  const size_t o_pd = cv.take<ProbDev>(nb_prob);
  const size_t o_ed = cv.take<ExpmDev>(nb_prob);
  const size_t o_Dm = cv.take<double>((size_t)qmax_all * qmax_all);
  const size_t o_nrm = cv.take<double>(nb_prob);
  pe_status stt = ensure_arena(ctx, cv.off);
  if (stt != PE_OK) return stt;
  stt = ensure_pinned(ctx, sizeof(double) * (2 * (PE_MAX_LEVELS + 1) * (size_t)nb_prob + 64));
  if (stt != PE_OK) return stt;
  char* base = ctx->arena;
  double* hp = (double*)ctx->pinned;
  ProbDev* dd = (ProbDev*)(base + o_pd);
  ExpmDev* ed = (ExpmDev*)(base + o_ed);
  {
    std::vector<double> D = chebyshev_derivative(qmax_all);
    HCK(hipMemcpyAsync(base + o_Dm, D.data(), sizeof(double) * D.size(), hipMemcpyHostToDevice, st));
    HCK(hipStreamSynchronize(st));
  }
  std::vector<ProbDev> hd(nb_prob);
  std::vector<ExpmDev> he(nb_prob);
  std::vector<HostState> hs(nb_prob);
  std::vector<double> u0n(nb_prob, 0.0);
  // norms of u0 (reference scale of the error control)
  {
    double* tmp = (double*)(base + o_nrm);
    for (int ii = 0; ii < nb_prob; ++ii) {
      const pe_problem& p = probs[idx[ii]];
      pe::launch_vec_norm(p.u0, p.op.n, tmp + ii, st);
    }
    HCK(hipMemcpyAsync(hp, tmp, sizeof(double) * nb_prob, hipMemcpyDeviceToHost, st));
    HCK(hipStreamSynchronize(st));
    for (int ii = 0; ii < nb_prob; ++ii) u0n[ii] = hp[ii];
  }
  for (int ii = 0; ii < nb_prob; ++ii) {
    const pe_problem& p = probs[idx[ii]];
    ProbDev& d = hd[ii];
    d = ProbDev{};
    d.n = p.op.n;
    d.per_point = p.op.per_point;
    if (!p.op.per_point) std::memcpy(d.c3, p.op.coeffs, 3 * sizeof(double));
    d.coef = p.op.per_point ? p.op.coeffs : nullptr;
    bind_block(d, base, bo[ii], mixed, p.krylov_steps + 1);
    d.U = Ul[ii];
    d.dep_tol = kDepTolArnoldi;
    d.xstate = (double*)(base + o_x[ii]);
    d.x = d.xstate;
    HostState& h = hs[ii];
    h.tau = p.t0;
    h.k = 0;
    const double tlast = p.n_out > 0 ? p.t_out[p.n_out - 1] : p.t0;
    h.Tspan = std::max(tlast - p.t0, 1e-300);
    h.ref = std::max(u0n[ii], 1e-300);
    h.dlast = h.Tspan;
    h.xzero = p.shift != 0;
    if (p.shift) pe::launch_fill(d.xstate, p.op.n, 1, p.op.n, 0.0, st);
    else pe::launch_copy(p.u0, d.xstate, p.op.n, st);
    // outputs at or before the start
    while (h.k < p.n_out && p.t_out[h.k] <= p.t0) {
      double* col = p.out + (int64_t)h.k * p.ldOut;
      if (p.t_out[h.k] < p.t0 || p.shift) pe::launch_fill(col, p.op.n, 1, p.op.n, 0.0, st);
      else pe::launch_copy(p.u0, col, p.op.n, st);
      ++h.k;
    }
    h.done = h.k >= p.n_out;
    HCK(hipMemsetAsync(d.cnt, 0, caps[ii].cnt * sizeof(unsigned), st));
    ExpmDev& e = he[ii];
    e = ExpmDev{};
    double* eb = (double*)(base + o_e[ii]);
    const size_t NN = (size_t)Nmax[ii] * Nmax[ii];
    e.Ht = eb;
    e.A = eb + NN;
    e.A2 = eb + 2 * NN;
    e.A3 = eb + 3 * NN;
    e.A4 = eb + 4 * NN;
    e.P = eb + 5 * NN;
    e.T = eb + 6 * NN;
    e.b = eb + 7 * NN;
    e.y = e.b + Nmax[ii];
    e.out = e.y + (size_t)(PE_MAX_LEVELS + 1) * Nmax[ii];
    e.ycur = e.out + 2 * (PE_MAX_LEVELS + 1);
    e.Eprop = e.ycur + Nmax[ii];
    e.H = d.H;
    e.R0 = d.Rf + 0;  // set per cycle (depends on bw)
    e.Pi = Pil[ii];
    e.ldPi = ldPil[ii];
    e.w = (double*)(base + o_w[ii]);
    e.Dm = (double*)(base + o_Dm);
    e.qmax = qmax_all;
    e.kscale = 2.0 / (p.t1 - p.t0);
    e.spline = (p.source_fit == PE_FIT_SPLINE && ml[ii] > 0) ? 1 : 0;
    e.Pw = Pil[ii];
  }
  std::vector<TriDev> ht(sai ? nb_prob : 0);
  TriDev* tdd = (TriDev*)(base + o_td);
  for (int ii = 0; ii < (sai ? nb_prob : 0); ++ii) {
    const pe_problem& p = probs[idx[ii]];
    const SaiOff& o = so[ii];
    TriDev& t = ht[ii];
    t = TriDev{};
    t.n = p.op.n;
    t.per_point = p.op.per_point;
    if (!p.op.per_point) std::memcpy(t.c3, p.op.coeffs, 3 * sizeof(double));
    t.coef = p.op.per_point ? p.op.coeffs : nullptr;
    t.R = o.R;
    t.C = o.C;
    t.ta = (double*)(base + o.ta);
    t.tinv = (double*)(base + o.tinv);
    t.tc = (double*)(base + o.tc);
    t.vL = (double*)(base + o.vL);
    t.vR = (double*)(base + o.vR);
    t.red = (double*)(base + o.red);
    t.rrhs = (double*)(base + o.rrhs);
    t.ru = (double*)(base + o.ru);
    t.W = (double*)(base + o.W);
    t.GW = (double*)(base + o.GW);
    t.piv = (int32_t*)(base + o.piv);
    t.cnt = (unsigned*)(base + o.cnt);
    t.LU = he[ii].A;      // the exponential's work matrices are free until the trials
    t.Kinv = he[ii].A2;
    t.H = hd[ii].H;
    pe::launch_zero_u32(t.cnt, 2, st);
    hd[ii].Wb = t.W;
    he[ii].sai = 1;
    he[ii].Kinv = t.Kinv;
    he[ii].GW = t.GW;
  }
  std::vector<std::vector<double>> wv(nb_prob, std::vector<double>(qmax_all + 1));
  int guard = 0;
  const int trace = env_int("PARAEXP_TRACE", 0);
  const int max_cycles = env_int("PARAEXP_MAX_CYCLES", 0);
  // next restart target of problem ii: the next output, the window end while the source
  // acts, and with a spline source the end of the piece holding tau (a sample time)
  auto target_of = [&](int ii) -> double {
    const pe_problem& p = probs[idx[ii]];
    HostState& h = hs[ii];
    double tg = h.src ? std::min(p.t_out[h.k], p.t1) : p.t_out[h.k];
    if (h.src && he[ii].spline) {
      while (h.piece + 1 <= p.s - 2 && p.t_samples[h.piece + 1] <= h.tau) ++h.piece;
      tg = std::min(tg, p.t_samples[h.piece + 1]);
    }
    return tg;
  };
  while (true) {
    // ---- plan the cycle
    int nact = 0, nreuse = 0, nzreset = 0, lmax = 0, tree = 0, gx_p = 0, gx_u = 0, mb_N = 1;
    size_t smem_p = 0, smem_u = 0;
    int64_t maxNN = 1;
    for (int ii = 0; ii < nb_prob; ++ii) {
      const pe_problem& p = probs[idx[ii]];
      HostState& h = hs[ii];
      ProbDev& d = hd[ii];
      d.active = 0;
      d.proj = 0;
      he[ii].active = 0;
      h.reuse_now = false;
      h.prop_now = false;
      he[ii].prop = 0;
      he[ii].zreset = 0;
      if (h.done) continue;
      const int m = ml[ii];
      h.src = (m > 0) && (h.tau < p.t1);
      if (!h.src && h.xzero) {  // the shifted state stays zero: remaining outputs are zero
        for (; h.k < p.n_out; ++h.k) pe::launch_fill(p.out + (int64_t)h.k * p.ldOut, p.op.n, 1, p.op.n, 0.0, st);
        h.done = true;
        continue;
      }
      h.target = target_of(ii);
      // The exponential of the Chebyshev generator over a step re-expands the basis at a
      // shift of c = 2 step / (t1 - t0) in x, with coefficients growing like
      // (1 + sqrt(2c))^q; rounding in the projected exponential grows with them.  Steps
      // (offsets from the cycle start) are capped so that the growth stays below kGrowthCap.
      const bool spl = he[ii].spline && h.src;
      const double cap = (h.src && ql[ii] > 0 && !spl)
                             ? 0.25 * std::pow(std::pow(kGrowthCap, 1.0 / ql[ii]) - 1.0, 2) * (p.t1 - p.t0)
                             : HUGE_VAL;
      if (spl) {  // the piece holding tau, and tau's offset into it
        he[ii].piece = h.piece;
        he[ii].pdelta = h.tau - p.t_samples[h.piece];
      }
      if (h.reuse) {
        // spline pieces: each pass restarts from the held solution at tau (its polynomial
        // part reset to the current piece), so offsets count from tau
        if (spl) h.tau_c = h.tau;
        const double off = std::min(h.target - h.tau_c, cap);
        if (off > h.tau - h.tau_c) {  // the same space, evaluated further out
          h.dtry = off;
          h.reuse_now = true;
          h.prop_now = h.prop_dt > 0.0 && off == h.target - h.tau_c &&
                       std::fabs((h.target - h.tau) - h.prop_dt) <= kPropRel * h.prop_dt;
          if (spl) {
            he[ii].zreset = 1;
            ++nzreset;
          }
          ++nreuse;
          mb_N = std::max(mb_N, h.N);
          maxNN = std::max<int64_t>(maxNN, (int64_t)h.N * h.N);
          continue;
        }
        h.reuse = false;
      }
      h.tau_c = h.tau;
      h.prop_dt = 0.0;
      h.dtry = std::min(std::min(h.target - h.tau, h.dgrow * h.dlast), cap);
      h.bw = h.src ? (h.xzero ? m : m + 1) : 1;
      d.m = h.src ? m : 0;
      d.with_x = h.xzero ? 0 : 1;
      d.l = p.krylov_steps;
      d.ldH = (int64_t)(d.l + 1) * h.bw;
      set_geometry(d, p.op.n, h.bw);
      if (!geometry_fits(d, caps[ii], d.l + 1))
        return pe_fail(ctx, PE_ERR_UNSUPPORTED, "cycle geometry exceeds the workspace");
      d.active = 1;
      ++nact;
      tree |= d.comb_tree;
      lmax = std::max(lmax, d.l);
      gx_p = std::max(gx_p, d.Cp);
      gx_u = std::max(gx_u, d.Cu);
      smem_p = std::max(smem_p, proj_smem(d));
      smem_u = std::max(smem_u, update_smem(d));
      h.N = d.l * h.bw + (h.src ? ql[ii] : 0);
      mb_N = std::max(mb_N, h.N);
      maxNN = std::max<int64_t>(maxNN, (int64_t)h.N * h.N);
      ExpmDev& e = he[ii];
      e.N = h.N;
      e.l = d.l;
      e.bw = h.bw;
      e.m = d.m;
      e.q = h.src ? ql[ii] : 0;
      e.with_x = d.with_x;
      e.lbw = d.l * h.bw;
      e.ldH = d.ldH;
      e.R0 = d.Rf + 2 * (size_t)h.bw * h.bw;
      if (h.src && ql[ii] > 0 && !he[ii].spline) {
        chebyshev_values((2.0 * h.tau - p.t0 - p.t1) / (p.t1 - p.t0), ql[ii], wv[ii].data());
        HCK(hipMemcpyAsync((void*)e.w, wv[ii].data(), sizeof(double) * ql[ii], hipMemcpyHostToDevice, st));
      }
    }
    if (nact == 0 && nreuse == 0) break;
    // shift-and-invert: gamma from the step each cycle aims at; factor I - gamma L
    int maxN0 = 1;
    if (sai && nact > 0) {
      for (int ii = 0; ii < nb_prob; ++ii) {
        const pe_problem& p = probs[idx[ii]];
        TriDev& t = ht[ii];
        const ProbDev& d = hd[ii];
        t.active = d.active;
        if (!d.active) continue;
        if (d.l * d.bw > kSaiMaxN0)
          return pe_fail(ctx, PE_ERR_UNSUPPORTED, "shift-and-invert: krylov_steps x block width above 4000");
        t.gamma = (p.sai_shift > 0.0 ? p.sai_shift : kSaiShift) * hs[ii].dtry;
        t.bw = d.bw;
        t.N0 = d.l * d.bw;
        t.ldH = d.ldH;
        he[ii].gamma = t.gamma;
        maxN0 = std::max(maxN0, t.N0);
      }
      HCK(hipMemcpyAsync(tdd, ht.data(), sizeof(TriDev) * nb_prob, hipMemcpyHostToDevice, st));
      pe::launch_tri_factor(tdd, nb_prob, maxC, st);
    }
    // a march times every kProfEvery-th restart cycle (all of its block steps, so the
    // sample spans the same step mix)
    ctx->prof_sample = (guard % kProfEvery) == 0;
    if (nact > 0 && ++guard > (max_cycles > 0 ? max_cycles : kCycleCap)) {
      // out of cycles (a tolerance below the attainable accuracy crawls at the minimum
      // step): flag, and mark the outputs not reached with NaN
      for (int ii = 0; ii < nb_prob; ++ii) {
        HostState& h = hs[ii];
        const pe_problem& p = probs[idx[ii]];
        if (h.done) continue;
        h.flags |= PE_FLAG_NOT_CONVERGED;
        for (; h.k < p.n_out; ++h.k)
          pe::launch_fill(p.out + (int64_t)h.k * p.ldOut, p.op.n, 1, p.op.n, std::nan(""), st);
        h.done = true;
      }
      break;
    }
    // ---- S5: initial block and block Arnoldi (problems that start a new space)
    if (nact > 0) {
      HCK(hipMemcpyAsync(dd, hd.data(), sizeof(ProbDev) * nb_prob, hipMemcpyHostToDevice, st));
      pe::launch_block_update(dd, nb_prob, gx_u, smem_u, 0, 0, 1, pe::MODE_INIT, mixed, tree, st);
      for (int j = 0; j < lmax; ++j) {
        const int groups = (j + 1 + pe::kSlotGroup - 1) / pe::kSlotGroup;
        StepCost cost;
        for (int ii = 0; ii < nb_prob; ++ii)
          if (hd[ii].active && j < hd[ii].l) {
            const StepCost c = step_cost(hd[ii].n, hd[ii].bw, j + 1, mixed ? 4 : 8);
            cost.proj_bytes += c.proj_bytes;
            cost.upd_bytes += c.upd_bytes;
            cost.flops += c.flops;
          }
        if (sai) {
          pe::launch_sai_solve(dd, tdd, nb_prob, sai_groups, maxn_all * maxbwall, j, mixed, st);
          run_block_step(ctx, dd, nb_prob, gx_p * groups, smem_p, gx_u, smem_u, j, j + 1, pe::MODE_SAI, mixed, tree,
                         cost, st);
        } else {
          run_block_step(ctx, dd, nb_prob, gx_p * groups, smem_p, gx_u, smem_u, j, j + 1, pe::MODE_ARNOLDI, mixed,
                         tree, cost, st);
        }
      }
      if (sai) {  // residual Gram of the last block, then K^{-1} for the projected operator
        pe::launch_sai_gram(dd, tdd, nb_prob, maxn_all, (double*)(base + o_gpart), st);
        pe::launch_hess_inverse(tdd, nb_prob, maxN0, maxbwall, lmax, st);
      }
    }
    // ---- S6: projected exponential with step-size trials (a reused space keeps its
    // projected matrix, start vector and norm)
    if (nact > 0) {
      for (int ii = 0; ii < nb_prob; ++ii) he[ii].active = hd[ii].active;
      HCK(hipMemcpyAsync(ed, he.data(), sizeof(ExpmDev) * nb_prob, hipMemcpyHostToDevice, st));
      pe::launch_build_aug(ed, nb_prob, maxNN, st);
      HCK(hipMemsetAsync(base + o_nrm, 0, sizeof(double) * nb_prob, st));
      pe::launch_norm1(ed, (double*)(base + o_nrm), nb_prob, mb_N, st);
      HCK(hipMemcpyAsync(hp, base + o_nrm, sizeof(double) * nb_prob, hipMemcpyDeviceToHost, st));
      HCK(hipStreamSynchronize(st));
    }
    for (int ii = 0; ii < nb_prob; ++ii) {
      HostState& h = hs[ii];
      if (hd[ii].active) h.nrm = hp[ii];
      h.pending = hd[ii].active != 0 || h.reuse_now;
      h.accepted = false;
      h.stop = false;
      // a non-finite projected matrix: no step can be taken
      if (hd[ii].active && !std::isfinite(hp[ii])) {
        h.pending = false;
        h.stop = true;
        h.flags |= PE_FLAG_NOT_CONVERGED;
      }
    }
    if (nzreset > 0) {
      // spline pieces evaluated from the held solution: its polynomial part restarts from
      // the current piece, and the trial starts from it
      HCK(hipMemcpyAsync(ed, he.data(), sizeof(ExpmDev) * nb_prob, hipMemcpyHostToDevice, st));
      pe::launch_spline_reset(ed, nb_prob, st);
      for (int ii = 0; ii < nb_prob; ++ii) {
        if (!he[ii].zreset) continue;
        if (!hs[ii].prop_now)
          HCK(hipMemcpyAsync(he[ii].b, he[ii].ycur, sizeof(double) * hs[ii].N, hipMemcpyDeviceToDevice, st));
        he[ii].zreset = 0;
      }
    }
    const int tiles = (mb_N + 31) / 32;
    // Each trial evaluates the step at every squaring level: after k squarings the
    // exponential is exp(alpha 2^k Ht) with alpha = dtry / 2^nsq, so the largest level
    // whose error estimate passes gives the accepted step without recomputation.
    for (int trial = 0; trial < kMaxTrials; ++trial) {
      int maxsq = 0, npend = 0, nfull = 0;
      for (int ii = 0; ii < nb_prob; ++ii) {
        ExpmDev& e = he[ii];
        HostState& h = hs[ii];
        e.active = h.pending ? 1 : 0;
        e.prop = h.pending && h.prop_now ? 1 : 0;
        if (!h.pending) continue;
        ++npend;
        if (e.prop) {  // one product with the held propagator, evaluated as level 0
          e.nsq = 0;
          e.alpha = h.dtry;
          continue;
        }
        ++nfull;
        const double nn = h.dtry * h.nrm;
        int s = 0;
        if (nn > kTaylorTheta) s = (int)std::ceil(std::log2(nn / kTaylorTheta));
        s = std::max(0, std::min(s, PE_MAX_LEVELS));
        e.nsq = s;
        e.alpha = std::ldexp(h.dtry, -s);
        maxsq = std::max(maxsq, s);
      }
      if (npend == 0) break;
      HCK(hipMemcpyAsync(ed, he.data(), sizeof(ExpmDev) * nb_prob, hipMemcpyHostToDevice, st));
      // one timed GEMM launch: 2 N^3 flops and 3 N^2 doubles (A, B read, C written; the
      // Paterson-Stockmeyer epilogue reads three more) per problem it multiplies for
      auto gemm = [&](int op, int k) {
        double fl = 0.0, by = 0.0;
        for (int ii = 0; ii < nb_prob; ++ii) {
          const ExpmDev& e = he[ii];
          if (!e.active || e.prop || (op == 6 && k >= e.nsq)) continue;
          const double NN = (double)e.N * e.N;
          fl += 2.0 * NN * e.N;
          by += 8.0 * NN * (op >= 3 && op <= 5 ? 6.0 : 3.0);
        }
        const int ev = prof_begin(ctx, "gemm", st);
        pe::launch_gemm(ed, op, k, nb_prob, tiles * tiles, st);
        prof_end(ctx, ev, by, fl, st);
      };
      if (nfull > 0) {
        pe::launch_elementwise(ed, 0, nb_prob, maxNN, st);
        gemm(0, 0);
        gemm(1, 0);
        gemm(2, 0);
        pe::launch_elementwise(ed, 1, nb_prob, maxNN, st);
        gemm(3, 0);
        gemm(4, 0);
        gemm(5, 0);
      }
      pe::launch_expm_apply(ed, 0, nb_prob, mb_N, st);
      for (int k = 0; k < maxsq; ++k) {
        gemm(6, k);
        pe::launch_expm_apply(ed, k + 1, nb_prob, mb_N, st);
      }
      for (int ii = 0; ii < nb_prob; ++ii)
        if (hs[ii].pending)
          HCK(hipMemcpyAsync(hp + 2 * (PE_MAX_LEVELS + 1) * ii, he[ii].out,
                             2 * (he[ii].nsq + 1) * sizeof(double), hipMemcpyDeviceToHost, st));
      HCK(hipStreamSynchronize(st));
      for (int ii = 0; ii < nb_prob; ++ii) {
        HostState& h = hs[ii];
        if (!h.pending) continue;
        const pe_problem& p = probs[idx[ii]];
        const double* ho = hp + 2 * (PE_MAX_LEVELS + 1) * ii;
        const int ns = he[ii].nsq;
        if (trace)
          for (int k = ns; k >= 0; --k)
            fprintf(stderr, "[paraexp] prob %d cycle %d trial %d level %d tau %.6e d %.3e N %d bw %d |H|1 %.3e "
                    "err %.3e |y| %.3e\n", idx[ii], guard, trial, k, h.tau, std::ldexp(he[ii].alpha, k), h.N, h.bw,
                    h.nrm, ho[2 * k], ho[2 * k + 1]);
        pe::StepIn in{};
        in.nsq = ns;
        in.est = ho;
        in.alpha = he[ii].alpha;
        in.tol = p.tol;
        in.ref = h.ref;
        in.tspan = h.Tspan;
        in.dmin = 1e-13 * h.Tspan;
        in.krylov_steps = p.krylov_steps;
        in.pexp = h.pexp;
        const pe::StepOut o = pe::step_decide(in);
        if (h.reuse_now && o.action != pe::kStepAccept) {
          h.pending = false;  // the space does not reach the next output: build a new one
          continue;
        }
        h.flags |= o.flags;
        h.pexp = o.pexp;
        if (o.action == pe::kStepAccept) {
          h.accepted = true;
          h.pending = false;
          h.level = o.level;
          h.rho = o.rho;
          h.dtry = o.step;
          h.resid = std::max(h.resid, o.err * h.dtry);
          if (o.level < ns && !h.reuse_now) h.rejected += 1;
        } else if (o.action == pe::kStepReject) {
          ++h.rejected;
          h.dtry = o.step;
        } else {
          h.pending = false;
          h.stop = true;
        }
      }
    }
    // ---- S7: project the accepted problems
    int nproj = 0;
    for (int ii = 0; ii < nb_prob; ++ii) {
      HostState& h = hs[ii];
      ProbDev& d = hd[ii];
      const pe_problem& p = probs[idx[ii]];
      d.proj = 0;
      d.outcol = nullptr;
      if (!d.active && !h.reuse_now) continue;
      if (d.active) h.steps += d.l;
      if (h.stop) {
        // the march of this problem ends here: outputs not reached are NaN
        for (; h.k < p.n_out; ++h.k)
          pe::launch_fill(p.out + (int64_t)h.k * p.ldOut, p.op.n, 1, p.op.n, std::nan(""), st);
        h.done = true;
        continue;
      }
      const bool landed = h.dtry >= h.target - h.tau_c;
      if (h.reuse_now && h.accepted && !landed && !(h.tau_c + h.dtry > h.tau)) h.accepted = false;
      if (!h.accepted) {
        if (h.reuse_now) h.reuse = false;  // new space from the current state next pass
        else h.dlast = h.dtry;             // retry the cycle with the reduced step
        continue;
      }
      d.active = 1;  // the projection reads the space of a reused cycle too
      d.proj = 1;
      d.yacc = he[ii].y + (size_t)h.level * h.N;
      if (landed && h.target == p.t_out[h.k]) d.outcol = p.out + (int64_t)h.k * p.ldOut;
      ++nproj;
    }
    if (nproj) {
      HCK(hipMemcpyAsync(dd, hd.data(), sizeof(ProbDev) * nb_prob, hipMemcpyHostToDevice, st));
      pe::launch_project(dd, ed, nb_prob, maxn, max_lbw, mixed, st);
    }
    for (int ii = 0; ii < nb_prob; ++ii) {
      HostState& h = hs[ii];
      ProbDev& d = hd[ii];
      const pe_problem& p = probs[idx[ii]];
      if (!d.active || !h.accepted) continue;
      const bool landed = h.dtry >= h.target - h.tau_c;
      h.tau = landed ? h.target : h.tau_c + h.dtry;
      // offsets reached from one space set the next space's first step; an offset
      // clipped at an output time does not limit it
      if (!landed || h.dtry >= h.dlast) h.dlast = h.dtry;
      h.dgrow = pe::step_growth(h.rho, h.pexp, p.krylov_steps);
      h.xzero = false;
      if (!h.reuse_now) ++h.cycles;
      // landed on an output inside the source interval (or past it): try the next output
      // from the same space
      h.reuse = landed && !(h.src && h.target >= p.t1);
      if (d.outcol) {
        const double tk = p.t_out[h.k];
        ++h.k;
        while (h.k < p.n_out && p.t_out[h.k] == tk) {
          pe::launch_copy(d.outcol, p.out + (int64_t)h.k * p.ldOut, p.op.n, st);
          ++h.k;
        }
      }
      if (h.k >= p.n_out) h.done = true;
      if (h.reuse && !h.done) {
        // the next output of this space starts from the projected solution here; the
        // exponential of this step serves as the propagator when the next spacing equals
        // it (the matrix of level k is T for even k, P for odd k, and the last two levels
        // of a trial are still held)
        ExpmDev& e = he[ii];
        HCK(hipMemcpyAsync(e.ycur, d.yacc, sizeof(double) * h.N, hipMemcpyDeviceToDevice, st));
        if (!h.prop_now) {
          h.prop_dt = 0.0;
          const double next = target_of(ii) - h.tau;
          if (h.level >= e.nsq - 1 && std::fabs(next - h.dtry) <= kPropRel * h.dtry) {
            HCK(hipMemcpyAsync(e.Eprop, (h.level & 1) ? e.P : e.T, sizeof(double) * h.N * h.N,
                               hipMemcpyDeviceToDevice, st));
            h.prop_dt = h.dtry;
          }
        }
      }
    }
    // host descriptors are rewritten next cycle: drain the queued uploads first
    HCK(hipStreamSynchronize(st));
  }
  HCK(hipStreamSynchronize(st));
  for (int ii = 0; ii < nb_prob; ++ii) {
    pe_report& r = reports[idx[ii]];
    r.cycles = hs[ii].cycles;
    r.rejected = hs[ii].rejected;
    r.block_steps = hs[ii].steps;
    r.flags |= hs[ii].flags;
    r.resid_est = hs[ii].resid;
  }
  return PE_OK;
}

pe_status march_all(pe_ctx* ctx, const pe_problem* probs, int nprob, const double* const* Ul,
                    const double* const* Pil, const int* ldPil, const int* ml, const int* ql, pe_report* reports,
                    hipStream_t st) {
  for (int grp = 0; grp < 4; ++grp) {
    const int prec = grp & 1, kry = grp >> 1;
    std::vector<int> idx;
    std::vector<const double*> U, Pi;
    std::vector<int> ld, m, q;
    for (int i = 0; i < nprob; ++i)
      if ((int)probs[i].prec == prec && (int)probs[i].krylov == kry) {
        idx.push_back(i);
        U.push_back(Ul[i]);
        Pi.push_back(Pil[i]);
        ld.push_back(ldPil[i]);
        m.push_back(ml[i]);
        q.push_back(ql[i]);
      }
    if (idx.empty()) continue;
    pe_status s = march_batch(ctx, probs, idx.data(), (int)idx.size(), U.data(), Pi.data(), ld.data(), m.data(),
                              q.data(), reports, st);
    if (s != PE_OK) return s;
  }
  return PE_OK;
}

}  // namespace

// =====================================================================================
// C ABI
// =====================================================================================
extern "C" {

const char* pe_version(void) { return "paraexp-gfx950 0.1"; }

pe_status pe_create(pe_ctx** ctx_out, int device) {
  if (!ctx_out) return PE_ERR_ARG;
  *ctx_out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) return PE_ERR_DEVICE;
  if (device < 0 || device >= count) return PE_ERR_ARG;
  if (hipSetDevice(device) != hipSuccess) return PE_ERR_DEVICE;
  pe_ctx* ctx = new pe_ctx();
  ctx->device = device;
  if (device < kMaxDevices) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device] && g_scratch_err[device] == hipSuccess) {
      void* ptr = nullptr;
      const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
      if (e == hipSuccess && ptr) g_scratch_ptr[device] = (char*)ptr;
      else g_scratch_err[device] = e != hipSuccess ? e : hipErrorInvalidSymbol;
    }
    ctx->scratch_dev = g_scratch_ptr[device];
  }
  *ctx_out = ctx;
  return PE_OK;
}

pe_status pe_destroy(pe_ctx* ctx) {
  if (!ctx) return PE_ERR_ARG;
  hipSetDevice(ctx->device);
  hipDeviceSynchronize();
  if (ctx->arena) hipFree(ctx->arena);
  if (ctx->keep) hipFree(ctx->keep);
  if (ctx->keep_wr) hipFree(ctx->keep_wr);
  if (ctx->pinned) hipHostFree(ctx->pinned);
  for (hipEvent_t e : ctx->ev) hipEventDestroy(e);
  delete ctx;
  return PE_OK;
}

const char* pe_last_error(const pe_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

pe_status pe_stencil_apply(pe_ctx* ctx, const pe_stencil* op, const double* X, int64_t ldx, double* Y, int64_t ldy,
                           int32_t ncols, void* stream) {
  if (!ctx) return PE_ERR_ARG;
  if (!op || !op->coeffs || !X || !Y || op->n < 1 || ldx < op->n || ldy < op->n || ncols < 0)
    return pe_fail(ctx, PE_ERR_ARG, "pe_stencil_apply: bad arguments");
  HCK(hipSetDevice(ctx->device));
  hipStream_t st = (hipStream_t)stream;
  const int ev = prof_begin(ctx, "stencil", st);
  pe::launch_stencil_cols(op->n, op->per_point, op->coeffs, op->coeffs, X, ldx, Y, ldy, ncols, st);
  prof_end(ctx, ev, 16.0 * (double)op->n * ncols + (op->per_point ? 24.0 * op->n : 0.0), 5.0 * op->n * ncols, st);
  HCK(hipGetLastError());
  HCK(hipStreamSynchronize(st));
  prof_collect(ctx);
  return PE_OK;
}

pe_status pe_compress(pe_ctx* ctx, const pe_problem* prob, double* U, double* Pi, int32_t* m, int32_t* q,
                      double* sigma, pe_report* report, void* stream) {
  if (!ctx) return PE_ERR_ARG;
  if (!prob || !U || !Pi || !m || !q) return pe_fail(ctx, PE_ERR_ARG, "pe_compress: null argument");
  pe_status s = validate_problem(ctx, *prob, true);
  if (s != PE_OK) return s;
  HCK(hipSetDevice(ctx->device));
  hipStream_t st = (hipStream_t)stream;
  CompressOut co;
  s = compress_one(ctx, *prob, U, prob->op.n, Pi, std::max(1, prob->rank_max), co, st);
  if (s != PE_OK) return s;
  HCK(hipGetLastError());
  HCK(hipStreamSynchronize(st));
  prof_collect(ctx);
  *m = co.m;
  *q = co.q;
  if (sigma)
    for (int i = 0; i < prob->s; ++i) sigma[i] = i < co.nsig ? co.sigma[i] : 0.0;
  if (report) {
    std::memset(report, 0, sizeof(pe_report));
    report->rank = co.m;
    report->q = co.q;
    report->flags = co.flags;
    report->fit_resid = co.fit_resid;
    report->svd_tail = co.svd_tail;
    report->sigma1 = co.sigma1;
  }
  return PE_OK;
}

pe_status pe_compress_noalloc(pe_ctx* ctx, const pe_problem* prob, double* U, double* Pi, int32_t* m, int32_t* q,
                      double* sigma, pe_report* report, void* stream) {
  if (!ctx) return PE_ERR_ARG;
  if (!prob || !U || !Pi || !m || !q) return pe_fail(ctx, PE_ERR_ARG, "pe_compress_noalloc: null argument");
  pe_status s = validate_problem(ctx, *prob, true);
  if (s != PE_OK) return s;
  HCK(hipSetDevice(ctx->device));
  hipStream_t st = (hipStream_t)stream;
  if (!ctx->scratch_dev) {
    const hipError_t e = ctx->device < kMaxDevices ? g_scratch_err[ctx->device] : hipErrorInvalidDevice;
    return pe_fail(ctx, PE_ERR_DEVICE, "pe_compress_noalloc: no device scratch on this device", e);
  }
  const FixedWs fx{ctx->scratch_dev, kScratchBytes, ctx->scratch_host, sizeof(ctx->scratch_host)};
  CompressOut co;
  s = compress_one(ctx, *prob, U, prob->op.n, Pi, std::max(1, prob->rank_max), co, st, &fx);
  if (s != PE_OK) return s;
  HCK(hipGetLastError());
  HCK(hipStreamSynchronize(st));
  *m = co.m;
  *q = co.q;
  if (sigma)
    for (int i = 0; i < prob->s; ++i) sigma[i] = i < co.nsig ? co.sigma[i] : 0.0;
  if (report) {
    std::memset(report, 0, sizeof(pe_report));
    report->rank = co.m;
    report->q = co.q;
    report->flags = co.flags;
    report->fit_resid = co.fit_resid;
    report->svd_tail = co.svd_tail;
    report->sigma1 = co.sigma1;
  }
  return PE_OK;
}

pe_status pe_expaction_batch(pe_ctx* ctx, const pe_problem* probs, const double* const* U, const double* const* Pi,
                             const int32_t* m, const int32_t* q, int32_t nprob, pe_report* reports, void* stream) {
  if (!ctx) return PE_ERR_ARG;
  TuneScope tune_scope(ctx);
  if (nprob < 0 || (nprob > 0 && (!probs || !m || !q || !reports || !U || !Pi)))
    return pe_fail(ctx, PE_ERR_ARG, "pe_expaction_batch: bad arguments");
  for (int i = 0; i < nprob; ++i) {
    pe_status s = validate_problem(ctx, probs[i], false);
    if (s != PE_OK) return s;
    if (m[i] < 0 || m[i] > 31 || q[i] < 0 || q[i] > 64 || (m[i] > 0 && (q[i] < 1 || !U[i] || !Pi[i])))
      return pe_fail(ctx, PE_ERR_ARG, "pe_expaction_batch: bad m/q/U/Pi");
    if (probs[i].op.n < m[i] + 1) return pe_fail(ctx, PE_ERR_ARG, "n too small for the block width");
    if (probs[i].source_fit != PE_FIT_CHEBYSHEV && m[i] > 0)
      return pe_fail(ctx, PE_ERR_UNSUPPORTED, "pe_expaction_batch takes Chebyshev coefficients only");
  }
  HCK(hipSetDevice(ctx->device));
  hipStream_t st = (hipStream_t)stream;
  std::vector<int> ld(nprob), mm(nprob), qq(nprob);
  for (int i = 0; i < nprob; ++i) {
    ld[i] = std::max(1, m[i]);
    mm[i] = m[i];
    qq[i] = m[i] > 0 ? q[i] : 0;
    std::memset(&reports[i], 0, sizeof(pe_report));
    reports[i].rank = m[i];
    reports[i].q = qq[i];
  }
  pe_status s = march_all(ctx, probs, nprob, U, Pi, ld.data(), mm.data(), qq.data(), reports, st);
  if (s != PE_OK) return s;
  HCK(hipGetLastError());
  HCK(hipStreamSynchronize(st));
  prof_collect(ctx);
  return PE_OK;
}

pe_status pe_solve_batch(pe_ctx* ctx, const pe_problem* probs, int32_t nprob, pe_report* reports, void* stream) {
  if (!ctx) return PE_ERR_ARG;
  TuneScope tune_scope(ctx);
  if (nprob < 0 || (nprob > 0 && (!probs || !reports))) return pe_fail(ctx, PE_ERR_ARG, "pe_solve_batch: bad arguments");
  for (int i = 0; i < nprob; ++i) {
    pe_status s = validate_problem(ctx, probs[i], true);
    if (s != PE_OK) return s;
    if (probs[i].op.n < probs[i].rank_max + 1) return pe_fail(ctx, PE_ERR_ARG, "n too small for rank_max");
  }
  HCK(hipSetDevice(ctx->device));
  hipStream_t st = (hipStream_t)stream;
  // compressed sources live in their own device allocation so the march can reuse the arena
  size_t tot = 0;
  std::vector<size_t> offU(nprob), offPi(nprob);
  for (int i = 0; i < nprob; ++i) {
    tot = (tot + 255) & ~(size_t)255;
    offU[i] = tot;
    tot += sizeof(double) * (size_t)probs[i].op.n * std::max(1, probs[i].rank_max);
    tot = (tot + 255) & ~(size_t)255;
    offPi[i] = tot;
    tot += sizeof(double) * (size_t)std::max(1, probs[i].rank_max) *
           (probs[i].source_fit == PE_FIT_SPLINE ? 4 * (size_t)std::max(1, probs[i].s - 1) : (size_t)probs[i].q_max);
  }
  {
    const pe_status ks = ensure_kept(ctx, ctx->keep, ctx->keep_cap, std::max<size_t>(tot, 256));
    if (ks != PE_OK) return ks;
  }
  char* src = ctx->keep;
  std::vector<const double*> Ul(nprob), Pil(nprob);
  std::vector<int> ld(nprob), mm(nprob), qq(nprob);
  pe_status s = PE_OK;
  for (int i = 0; i < nprob && s == PE_OK; ++i) {
    std::memset(&reports[i], 0, sizeof(pe_report));
    CompressOut co;
    double* U = (double*)(src + offU[i]);
    double* Pi = (double*)(src + offPi[i]);
    s = compress_one(ctx, probs[i], U, probs[i].op.n, Pi, std::max(1, probs[i].rank_max), co, st);
    if (s != PE_OK) break;
    Ul[i] = U;
    Pil[i] = Pi;
    ld[i] = std::max(1, probs[i].rank_max);
    mm[i] = co.m;
    // the march's polynomial part: q Chebyshev terms, or the 4 m Taylor coefficients of
    // the spline pieces
    qq[i] = co.m > 0 ? (probs[i].source_fit == PE_FIT_SPLINE ? 4 * co.m : co.q) : 0;
    reports[i].rank = co.m;
    reports[i].q = co.q;
    reports[i].flags = co.flags;
    reports[i].fit_resid = co.fit_resid;
    reports[i].svd_tail = co.svd_tail;
    reports[i].sigma1 = co.sigma1;
  }
  if (s == PE_OK) s = march_all(ctx, probs, nprob, Ul.data(), Pil.data(), ld.data(), mm.data(), qq.data(), reports, st);
  hipStreamSynchronize(st);
  prof_collect(ctx);
  if (s != PE_OK) return s;
  HCK(hipGetLastError());
  return PE_OK;
}

// ---- S10: waveform relaxation for Burgers ------------------------------------------
pe_status pe_wr_burgers(pe_ctx* ctx, const pe_wr_problem* wr, pe_report* reports, double* increments, void* stream) {
  if (!ctx) return PE_ERR_ARG;
  if (!wr || !reports) return pe_fail(ctx, PE_ERR_ARG, "pe_wr_burgers: null argument");
  const pe_wr_problem& w = *wr;
  if (w.n < 4 || w.P < 1 || w.s < 2 || w.K < 0 || !(w.T > 0.0) || !(w.nu >= 0.0) || !w.u0 || !w.u_final)
    return pe_fail(ctx, PE_ERR_ARG, "pe_wr_burgers: bad sizes or pointers");
  if (w.n < w.rank_max + 1) return pe_fail(ctx, PE_ERR_ARG, "n too small for rank_max");
  HCK(hipSetDevice(ctx->device));
  hipStream_t st = (hipStream_t)stream;
  const int64_t n = w.n;
  const int P = w.P, s = w.s, cols = P * s;
  const double h = 1.0 / (double)n;
  // sample times, window-major; the product and the sum are separate statements so the
  // compiler cannot fuse them (the same two roundings as t0 + i * step elsewhere)
  std::vector<double> times((size_t)cols), tw(P + 1);
  for (int j = 0; j <= P; ++j) tw[j] = w.T * (double)j / (double)P;
  for (int j = 0; j < P; ++j) {
    const double step = (tw[j + 1] - tw[j]) / (double)(s - 1);
    for (int i = 0; i < s; ++i) {
      const double a = (double)i * step;
      times[(size_t)j * s + i] = a + tw[j];
    }
    times[(size_t)j * s] = tw[j];
    times[(size_t)j * s + s - 1] = tw[j + 1];
  }
  // trapezoid weights of uniform samples, normalised by the window length
  const double w_in = 1.0 / (double)(s - 1), w_end = 0.5 / (double)(s - 1);
  // device buffers: iterate, window solutions, continuations, sources, operators
  const size_t blkn = (size_t)n * cols;
  const int nblk = 256;
  double* base = nullptr;
  const size_t tot = sizeof(double) * (4 * blkn + 3 * (size_t)n * P + n + 2 * nblk);
  {
    const pe_status ks = ensure_kept(ctx, ctx->keep_wr, ctx->keep_wr_cap, tot);
    if (ks != PE_OK) return ks;
  }
  base = (double*)ctx->keep_wr;
  double* Uk = base;
  double* Vown = Uk + blkn;
  double* Cc = Vown + blkn;
  double* G = Cc + blkn;
  double* coef = G + blkn;
  double* z = coef + 3 * (size_t)n * P;
  double* part = z + n;
  std::vector<double> hpart(2 * nblk);
  pe_status res = PE_OK;
  auto fail = [&](pe_status e) {
    res = e;
    return e;
  };
  do {
    if (w.u_init) {
      if (hipMemcpyAsync(Uk, w.u_init, sizeof(double) * blkn, hipMemcpyDeviceToDevice, st) != hipSuccess) {
        fail(pe_fail(ctx, PE_ERR_DEVICE, "pe_wr_burgers: copy u_init"));
        break;
      }
    } else {
      std::vector<const double*> none;
      pe::launch_superpose(w.u0, none.data(), 0, n, cols, n, Uk, n, st);
    }
    for (int k = 0; k < w.K && res == PE_OK; ++k) {
      // sources and operators of every window from the current iterate
      for (int j = 0; j < P; ++j)
        pe::launch_wr_source(n, s, h, w.nu, Uk + (size_t)j * s * n, w.jacobian, w_end, w_in,
                             w.forcing ? w.forcing + (size_t)j * s * n : nullptr, coef + 3 * (size_t)n * j,
                             G + (size_t)j * s * n, st);
      // the P window subproblems, batched: v_j at the window's own samples
      std::vector<pe_problem> pr((size_t)P);
      for (int j = 0; j < P; ++j) {
        pe_problem& q = pr[j];
        std::memset(&q, 0, sizeof(q));
        q.op.n = n;
        q.op.per_point = 1;
        q.op.coeffs = coef + 3 * (size_t)n * j;
        q.u0 = w.u0;
        q.t0 = tw[j];
        q.t1 = tw[j + 1];
        q.t_samples = times.data() + (size_t)j * s;
        q.s = s;
        q.G = G + (size_t)j * s * n;
        q.ldG = n;
        q.shift = 1;
        q.t_out = times.data() + (size_t)j * s;
        q.n_out = s;
        q.out = Vown + (size_t)j * s * n;
        q.ldOut = n;
        q.krylov_steps = w.krylov_steps;
        q.rank_max = w.rank_max;
        q.q_max = w.q_max;
        q.tol = w.tol;
        q.svd_tol = w.svd_tol;
        q.fit_tol = w.fit_tol;
        q.prec = w.prec;
        q.krylov = w.krylov;
        q.sai_shift = w.sai_shift;
        q.source_fit = w.source_fit;
      }
      {
        const pe_status sb = pe_solve_batch(ctx, pr.data(), P, reports, stream);
        if (sb != PE_OK) {
          res = sb;
          break;
        }
      }
      // homogeneous continuation of the earlier windows through window i with L_i:
      // c_i(T_i) = c_{i-1}(T_i) + v_{i-1}(T_i), then c' = L_i c over window i
      pe::launch_fill(Cc, n, s, n, 0.0, st);
      for (int i = 1; i < P && res == PE_OK; ++i) {
        const double* vlast = Vown + ((size_t)i * s - 1) * n;
        const double* clast = Cc + ((size_t)i * s - 1) * n;
        pe::launch_superpose(vlast, &clast, 1, n, 1, n, z, n, st);
        pe_problem q;
        std::memset(&q, 0, sizeof(q));
        q.op.n = n;
        q.op.per_point = 1;
        q.op.coeffs = coef + 3 * (size_t)n * i;
        q.u0 = z;
        q.t0 = tw[i];
        q.t1 = tw[i + 1];
        q.shift = 0;
        q.t_out = times.data() + (size_t)i * s;
        q.n_out = s;
        q.out = Cc + (size_t)i * s * n;
        q.ldOut = n;
        q.krylov_steps = w.krylov_steps;
        q.rank_max = w.rank_max;
        q.q_max = w.q_max;
        q.tol = w.tol;
        q.prec = w.prec;
        q.krylov = w.krylov;
        q.sai_shift = w.sai_shift;
        q.source_fit = w.source_fit;
        const double* nullp = nullptr;
        const int32_t zero = 0;
        pe_report rep;
        const pe_status se = pe_expaction_batch(ctx, &q, &nullp, &nullp, &zero, &zero, 1, &rep, stream);
        if (se != PE_OK) {
          res = se;
          break;
        }
        reports[i].cycles += rep.cycles;
        reports[i].block_steps += rep.block_steps;
        reports[i].rejected += rep.rejected;
        reports[i].flags |= rep.flags;
      }
      if (res != PE_OK) break;
      // u_{k+1} = u0 + v + c at every sample; increment against u_k
      const double* vv[2] = {Vown, Cc};
      pe::launch_superpose(w.u0, vv, 2, n, cols, n, G, n, st);
      pe::launch_diff_norms(G, Uk, (int64_t)blkn, part, nblk, st);
      if (hipMemcpyAsync(hpart.data(), part, sizeof(double) * 2 * nblk, hipMemcpyDeviceToHost, st) != hipSuccess ||
          hipMemcpyAsync(Uk, G, sizeof(double) * blkn, hipMemcpyDeviceToDevice, st) != hipSuccess ||
          hipStreamSynchronize(st) != hipSuccess) {
        fail(pe_fail(ctx, PE_ERR_DEVICE, "pe_wr_burgers: iterate update"));
        break;
      }
      double d2 = 0.0, a2 = 0.0;
      for (int b = 0; b < nblk; ++b) {
        d2 += hpart[2 * b];
        a2 += hpart[2 * b + 1];
      }
      if (increments) increments[k] = a2 > 0.0 ? std::sqrt(d2 / a2) : std::sqrt(d2);
    }
    if (res == PE_OK &&
        hipMemcpyAsync(w.u_final, Uk, sizeof(double) * blkn, hipMemcpyDeviceToDevice, st) != hipSuccess)
      fail(pe_fail(ctx, PE_ERR_DEVICE, "pe_wr_burgers: copy u_final"));
  } while (false);
  hipStreamSynchronize(st);
  if (res != PE_OK) return res;
  HCK(hipGetLastError());
  return PE_OK;
}

pe_status pe_workspace_query(pe_ctx* ctx, const pe_problem* probs, int32_t nprob, size_t* bytes) {
  pe_ctx local;  // host-only arithmetic: a null ctx is allowed
  pe_ctx* c = ctx ? ctx : &local;
  TuneScope tune_scope(c);
  if (!bytes || nprob < 0 || (nprob > 0 && !probs)) return pe_fail(c, PE_ERR_ARG, "pe_workspace_query: bad arguments");
  *bytes = 0;
  struct QueryScope {
    pe_ctx* c;
    ~QueryScope() {
      c->query = false;
      c->query_bytes = 0;
    }
  } scope{c};
  size_t arena = 0, src = 0;
  std::vector<int> ml(nprob), ql(nprob);
  for (int i = 0; i < nprob; ++i) {
    const pe_problem& p = probs[i];
    if (p.op.n < 4 || p.s < 1 || p.krylov_steps < 1 || p.krylov_steps > 512 || p.q_max < 1 || p.q_max > 64 ||
        (p.prec != PE_FP64 && p.prec != PE_MIXED))
      return pe_fail(c, PE_ERR_ARG, "pe_workspace_query: bad problem sizes");
    if (p.rank_max < 0 || p.rank_max > 31) return pe_fail(c, PE_ERR_UNSUPPORTED, "rank_max must be in [0, 31]");
    if (p.op.n < p.rank_max + 1) return pe_fail(c, PE_ERR_ARG, "n too small for rank_max");
    // compression (S1-S4): its own arena layout
    c->query = true;
    c->query_bytes = 0;
    CompressOut co;
    pe_status s = compress_one(c, p, nullptr, p.op.n, nullptr, std::max(1, p.rank_max), co, nullptr);
    if (s != kQueryStop) return s == PE_OK ? pe_fail(c, PE_ERR_DEVICE, "query did not stop") : s;
    arena = std::max(arena, c->query_bytes);
    // compressed sources (the context's kept buffer in pe_solve_batch)
    src = (src + 255) & ~(size_t)255;
    src += sizeof(double) * (size_t)p.op.n * std::max(1, p.rank_max);
    src = (src + 255) & ~(size_t)255;
    const bool spl = p.source_fit == PE_FIT_SPLINE;
    src += sizeof(double) * (size_t)std::max(1, p.rank_max) * (spl ? 4 * (size_t)std::max(1, p.s - 1) : p.q_max);
    // the march at the largest rank and polynomial order the problem allows
    ml[i] = std::min(p.rank_max, p.s);
    ql[i] = spl ? 4 * ml[i] : std::min(p.q_max, p.s);
    // every cycle geometry the march can meet (rank m' <= ml, block width m' in the
    // zero-state cycle, m' + 1 after it, 1 past the window) must fit its workspace
    const int l = p.krylov_steps;
    for (int mm = 0; mm <= ml[i]; ++mm) {
      const int bwc = mm + 1;
      const BlockCaps caps = block_caps(p.op.n, bwc, l + 1, (int64_t)(l + 1) * bwc, (int64_t)l * bwc);
      for (int bw : {1, std::max(1, mm), bwc}) {
        ProbDev d{};
        d.mixed = p.prec == PE_MIXED ? 1 : 0;
        set_geometry(d, p.op.n, bw);
        if (!geometry_fits(d, caps, l + 1))
          return pe_fail(c, PE_ERR_UNSUPPORTED, "cycle geometry exceeds the workspace");
      }
    }
  }
  for (int prec = 0; prec < 2; ++prec) {
    std::vector<int> idx, m, q, ld;
    for (int i = 0; i < nprob; ++i)
      if ((int)probs[i].prec == prec) {
        idx.push_back(i);
        m.push_back(ml[i]);
        q.push_back(ql[i]);
        ld.push_back(std::max(1, probs[i].rank_max));
      }
    if (idx.empty()) continue;
    std::vector<const double*> nul(idx.size(), nullptr);
    std::vector<pe_report> rep(nprob);
    c->query = true;
    c->query_bytes = 0;
    pe_status s = march_batch(c, probs, idx.data(), (int)idx.size(), nul.data(), nul.data(), ld.data(), m.data(),
                              q.data(), rep.data(), nullptr);
    if (s != kQueryStop) return s == PE_OK ? pe_fail(c, PE_ERR_DEVICE, "query did not stop") : s;
    arena = std::max(arena, c->query_bytes);
  }
  *bytes = arena + src;
  return PE_OK;
}

// ---- pe_autotune: block-kernel tiling per (grid bucket, block width, precision) ------
// Times kTuneSteps block Arnoldi steps of the polynomial space on a random block for
// every admissible (rows per update chunk, rows per projection chunk) and keeps the
// fastest when it beats the built-in tiling by kTuneMargin; the choice applies to grids
// of the same power-of-two bucket.
constexpr int kTuneSteps = 12;
constexpr double kTuneMargin = 0.97;  // a tiling replaces the built-in one when 3% faster

pe_status tune_one(pe_ctx* ctx, int64_t n, int bw, int mixed, hipStream_t st, TuneVal& best) {
  const int L = kTuneSteps;
  // capacities for the smallest chunks (the most chunks of any candidate)
  BlockCaps caps;
  {
    const TuneTable* saved = g_tune;
    g_tune = nullptr;
    caps = block_caps(n, bw, L + 1, (int64_t)(L + 1) * bw, (int64_t)L * bw);
    g_tune = saved;
  }
  caps.rloc = std::max(caps.rloc, (size_t)std::max<int64_t>(1, n / 64) * bw * bw);
  caps.part = std::max(caps.part, 2 * (size_t)(L + 1) * (size_t)((n + 15) / 16) * bw * bw);
  caps.cnt = std::max(caps.cnt, 2 * (size_t)(L + 1) + 2 + (size_t)(n / 64 + pe::kTreeFan - 1) / pe::kTreeFan);
  Carver cv;
  const BlockOffsets bo = carve_block(cv, caps, mixed != 0);
  const size_t o_u = cv.take<double>((size_t)n * bw);
  const size_t o_pd = cv.take<ProbDev>(1);
  pe_status stt = ensure_arena(ctx, cv.off);
  if (stt != PE_OK) return stt;
  char* base = ctx->arena;
  double* Ux = (double*)(base + o_u);  // columns 0..bw-2: U, column bw-1: x
  pe::launch_fill_hash(Ux, (int64_t)n * bw, 0x5eedULL + (uint64_t)bw, st);
  ProbDev d{};
  d.n = n;
  d.per_point = 0;
  d.c3[0] = 1.0;
  d.c3[1] = -2.0;
  d.c3[2] = 1.0;
  bind_block(d, base, bo, mixed != 0, L + 1);
  d.U = Ux;
  d.m = bw - 1;
  d.x = Ux + (size_t)n * (bw - 1);
  d.xstate = (double*)d.x;
  d.with_x = 1;
  d.dep_tol = kDepTolArnoldi;
  d.l = L;
  d.ldH = (int64_t)(L + 1) * bw;
  d.active = 1;
  ProbDev* dd = (ProbDev*)(base + o_pd);
  hipEvent_t e0, e1;
  HCK(hipEventCreate(&e0));
  HCK(hipEventCreate(&e1));
  // time of L block steps (best of three passes; the first warms the caches) on a tiling,
  // or HUGE_VAL when the tiling does not fit
  auto time_tiling = [&](int ru, int rp) -> double {
    int cg, ct;
    if (ru > n || rp * bw > 1024 || rp > n || !update_chunks_for(n, bw, ru, cg, ct)) return HUGE_VAL;
    d.bw = bw;
    d.rows_u = ru;
    d.rows_u_log2 = 0;
    while ((1 << d.rows_u_log2) < ru) ++d.rows_u_log2;
    d.Cu = (int)std::max<int64_t>(1, n / ru);
    d.comb_global = cg;
    d.comb_tree = ct;
    d.rows_p = rp;
    d.Cp = (int)((n + rp - 1) / rp);
    if (!geometry_fits(d, caps, L + 1)) return HUGE_VAL;
    HCK(hipMemsetAsync(d.cnt, 0, caps.cnt * sizeof(unsigned), st));
    HCK(hipMemcpyAsync(dd, &d, sizeof(ProbDev), hipMemcpyHostToDevice, st));
    const size_t smem_p = proj_smem(d), smem_u = update_smem(d);
    double ms = HUGE_VAL;
    for (int rep = 0; rep < 3; ++rep) {
      HCK(hipEventRecord(e0, st));
      pe::launch_block_update(dd, 1, d.Cu, smem_u, 0, 0, 1, pe::MODE_INIT, mixed, ct, st);
      for (int j = 0; j < L; ++j) {
        const int groups = (j + 1 + pe::kSlotGroup - 1) / pe::kSlotGroup;
        StepCost cost;
        run_block_step(ctx, dd, 1, d.Cp * groups, smem_p, d.Cu, smem_u, j, j + 1, pe::MODE_ARNOLDI, mixed, ct, cost,
                       st);
      }
      HCK(hipEventRecord(e1, st));
      HCK(hipEventSynchronize(e1));
      float t = 0.0f;
      HCK(hipEventElapsedTime(&t, e0, e1));
      ms = std::min(ms, (double)t);
    }
    return ms;
  };
  // the built-in tiling is the prior: another replaces it only when clearly faster
  int du, dcg, dct;
  choose_update_chunks(n, bw, du, dcg, dct);
  const int dp = rows_p_for(bw);
  const double def_ms = time_tiling(du, dp);
  best = TuneVal{du, dp};
  double best_ms = def_ms;
  for (int ru : {64, 128, 256, 512})
    for (int rp : {16, 32, 64, 128, 256}) {
      if (ru == du && rp == dp) continue;
      const double ms = time_tiling(ru, rp);
      if (ms < best_ms) {
        best_ms = ms;
        best = TuneVal{ru, rp};
      }
    }
  if (!(best_ms < kTuneMargin * def_ms) && def_ms < HUGE_VAL) best = TuneVal{du, dp};
  if (!(best_ms < HUGE_VAL)) best = TuneVal{0, 0};
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  HCK(hipGetLastError());
  return best.rows_u ? PE_OK : pe_fail(ctx, PE_ERR_UNSUPPORTED, "pe_autotune: no tiling fits");
}

pe_status pe_autotune(pe_ctx* ctx, const pe_problem* probs, int32_t nprob, const char* cache_path, int32_t* tuned,
                      void* stream) {
  if (!ctx) return PE_ERR_ARG;
  if (nprob < 0 || (nprob > 0 && !probs)) return pe_fail(ctx, PE_ERR_ARG, "pe_autotune: bad arguments");
  HCK(hipSetDevice(ctx->device));
  hipStream_t st = (hipStream_t)stream;
  if (cache_path) {  // earlier choices: lines "nlog2 bw mixed rows_u rows_p"
    std::ifstream in(cache_path);
    int a, b, c, ru, rp;
    while (in >> a >> b >> c >> ru >> rp)
      if (a > 0 && a < 48 && b >= 1 && b <= 32 && (c == 0 || c == 1) && ru >= 64 && ru <= 4096 && (ru & (ru - 1)) == 0 &&
          rp >= 16 && rp <= 1024 && (rp & (rp - 1)) == 0)
        ctx->tune[TuneKey{a, b, c}] = TuneVal{ru, rp};
  }
  int count = 0;
  for (int i = 0; i < nprob; ++i) {
    const pe_problem& p = probs[i];
    if (p.op.n < 64 || p.rank_max < 0 || p.rank_max > 31) return pe_fail(ctx, PE_ERR_ARG, "pe_autotune: bad problem");
    const int mixed = p.prec == PE_MIXED ? 1 : 0;
    // every width a march can meet: compressed rank m <= rank_max, m + 1 with the state,
    // m in the zero-state cycle, 1 past the window
    for (int bw = 1; bw <= p.rank_max + 1; ++bw) {
      const TuneKey key{tune_nlog2(p.op.n), bw, mixed};
      if (ctx->tune.count(key)) continue;
      TuneVal v;
      const pe_status s = tune_one(ctx, p.op.n, bw, mixed, st, v);
      if (s != PE_OK) return s;
      ctx->tune[key] = v;
      ++count;
    }
  }
  if (tuned) *tuned = count;
  if (cache_path && count > 0) {
    std::ofstream out(cache_path, std::ios::trunc);
    if (!out) return pe_fail(ctx, PE_ERR_ARG, "pe_autotune: cannot write the cache file");
    for (const auto& kv : ctx->tune)
      out << kv.first.nlog2 << ' ' << kv.first.bw << ' ' << kv.first.mixed << ' ' << kv.second.rows_u << ' '
          << kv.second.rows_p << '\n';
  }
  return PE_OK;
}

// the tuning table of the context as (nlog2, bw, mixed, rows_u, rows_p) rows
int32_t pe_autotune_table(const pe_ctx* ctx, int32_t* rows, int32_t max_rows) {
  if (!ctx) return 0;
  int k = 0;
  for (const auto& kv : ctx->tune) {
    if (rows && k < max_rows) {
      int32_t* r = rows + 5 * k;
      r[0] = kv.first.nlog2;
      r[1] = kv.first.bw;
      r[2] = kv.first.mixed;
      r[3] = kv.second.rows_u;
      r[4] = kv.second.rows_p;
    }
    ++k;
  }
  return k;
}

pe_status pe_profile_enable(pe_ctx* ctx, const char* family) {
  if (!ctx) return PE_ERR_ARG;
  if (family && std::strcmp(family, "block_update") && std::strcmp(family, "block_proj") &&
      std::strcmp(family, "stencil") && std::strcmp(family, "gemm"))
    return pe_fail(ctx, PE_ERR_ARG, "pe_profile_enable: unknown kernel family");
  ctx->prof_name = family ? family : "";
  ctx->prof_launches = 0;
  ctx->prof_ms = ctx->prof_bytes = ctx->prof_flops = 0.0;
  return PE_OK;
}

pe_status pe_profile_read(pe_ctx* ctx, int64_t* launches, double* ms, double* bytes, double* flops) {
  if (!ctx || !launches || !ms || !bytes || !flops) return PE_ERR_ARG;
  *launches = ctx->prof_launches;
  *ms = ctx->prof_ms;
  *bytes = ctx->prof_bytes;
  *flops = ctx->prof_flops;
  ctx->prof_launches = 0;
  ctx->prof_ms = ctx->prof_bytes = ctx->prof_flops = 0.0;
  return PE_OK;
}

pe_status pe_superpose(pe_ctx* ctx, const double* u0, const double* const* v, int32_t P, int64_t n, int32_t n_out,
                       int64_t ldv, double* u, int64_t ldu, void* stream) {
  if (!ctx) return PE_ERR_ARG;
  if (!u0 || !u || P < 0 || n < 1 || n_out < 0 || ldv < n || ldu < n || (P > 0 && !v))
    return pe_fail(ctx, PE_ERR_ARG, "pe_superpose: bad arguments");
  for (int j = 0; j < P; ++j)
    if (!v[j]) return pe_fail(ctx, PE_ERR_ARG, "pe_superpose: null window pointer");
  HCK(hipSetDevice(ctx->device));
  hipStream_t st = (hipStream_t)stream;
  if (n_out == 0) return PE_OK;
  if (P == 0) {
    for (int k = 0; k < n_out; ++k) pe::launch_copy(u0, u + (int64_t)k * ldu, n, st);
  } else {
    pe::launch_superpose(u0, v, P, n, n_out, ldv, u, ldu, st);
  }
  HCK(hipGetLastError());
  HCK(hipStreamSynchronize(st));
  return PE_OK;
}

// ---- host-only decision rules (paraexp_policy.h) -----------------------------------
void pe_policy_step(const pe_step_trial* t, pe_step_decision* out) {
  if (!t || !out || !t->est || t->nsq < 0) return;
  pe::StepIn in{};
  in.nsq = t->nsq;
  in.est = t->est;
  in.alpha = t->alpha;
  in.tol = t->tol;
  in.ref = t->ref;
  in.tspan = t->tspan;
  in.dmin = t->dmin;
  in.krylov_steps = t->krylov_steps;
  in.pexp = t->pexp;
  const pe::StepOut o = pe::step_decide(in);
  out->action = o.action;
  out->level = o.level;
  out->flags = o.flags;
  out->step = o.step;
  out->rho = o.rho;
  out->pexp = o.pexp;
  out->err = o.err;
}

double pe_policy_step_growth(double rho, double pexp, int32_t krylov_steps) {
  return pe::step_growth(rho, pexp, krylov_steps);
}

int32_t pe_policy_reorth_skip(const double* R, const double* Rn, int32_t bw, double kappa) {
  if (!R || !Rn || bw < 1 || bw > 32) return 0;
  double z[32];
  for (int b = 0; b < bw; ++b)
    if (!pe::reorth_column_ok(R, Rn, bw, b, kappa, z)) return 0;
  return 1;
}

}  // extern "C"
