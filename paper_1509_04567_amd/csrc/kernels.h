// Kernel launchers of the gfx950 Paraexp library (host-callable, defined in kernels.hip).
#pragma once

#include "common.h"

namespace pe {

// modes of the block orthogonalisation kernels: Arnoldi step of L (the input block is
// formed on the fly as L V_j), of the shifted inverse (I - gamma L)^{-1} (input block read
// from ProbDev::Wb, V_j already committed), a given block (columns of ProbDev::Xg), or
// the initial block [U | x]
enum BlockMode : int { MODE_ARNOLDI = 0, MODE_GIVEN = 1, MODE_INIT = 2, MODE_SAI = 3 };
__host__ __device__ inline bool arnoldi_mode(int mode) { return mode == MODE_ARNOLDI || mode == MODE_SAI; }

// dynamic LDS requested by the update kernel at most (bytes)
constexpr int kUpdateLdsMax = 150 * 1024;
// slot group handled by one projection workgroup
constexpr int kSlotGroup = 4;
// LDS doubles for the projection coefficients staged by the update kernel
constexpr int kSb = 4096;
// chunks per group of the two-level TSQR combine
constexpr int kTreeFan = 8;

// The TSQR combine of Cu stacked bw x bw factors runs register-resident (four waves)
// when it fits; otherwise from LDS.
__host__ __device__ inline bool combine_in_registers(int bw, int Cu) {
  const int rpl = (Cu * bw + 255) / 256;
  return (bw <= 8 && rpl <= 4) || (bw <= 16 && rpl <= 1);
}

// Y[:, c] = L X[:, c]
void launch_stencil_cols(int64_t n, int per_point, const double* c3, const double* coef, const double* X,
                         int64_t ldx, double* Y, int64_t ldy, int ncols, hipStream_t st);
// Gh[:, i] = G[:, i] + add[:]   (add may be null)
void launch_add_column(int64_t n, int s, const double* G, int64_t ldG, const double* add, double* Gh,
                       int64_t ldGh, hipStream_t st);

// block orthogonalisation (batched over problems; basis storage fp32 when `mixed`);
// init_block_kernels sets their launch attributes once (also called by the launchers)
void init_block_kernels();
void launch_block_proj(ProbDev* d, int nprob, int grid_x, size_t smem, int j, int nb, int pass, int mode,
                       int mixed, hipStream_t st);
// tree: some problem of the batch uses the two-level combine (k_tree_assemble follows)
void launch_block_update(ProbDev* d, int nprob, int grid_x, size_t smem, int j, int nb, int pass, int mode,
                         int mixed, int tree, hipStream_t st);
void launch_block_commit(ProbDev* d, int nprob, int grid_x, int j, int mixed, hipStream_t st);

// exponential of the projected augmented matrix
void launch_build_aug(ExpmDev* e, int nprob, int64_t maxNN, hipStream_t st);
void launch_norm1(ExpmDev* e, double* out, int nprob, int maxN, hipStream_t st);
void launch_elementwise(ExpmDev* e, int op, int nprob, int64_t maxNN, hipStream_t st);
void launch_gemm(ExpmDev* e, int op, int k, int nprob, int tiles_max, hipStream_t st);
void launch_expm_apply(ExpmDev* e, int level, int nprob, int maxN, hipStream_t st);

// shift-and-invert operator (sai.hip): factorisation of I - gamma L, the solve of an
// Arnoldi step (V_j committed, W = (I - gamma L)^{-1} V_j into TriDev::W), the Gram of
// (I - gamma L) V_l (part: nprob x ceil(n / 128) x 1024 doubles), inverse of the
// projected matrix
// LDS of the solve kernel (doubles, within gfx950's 160 KiB per workgroup); chunks per
// workgroup of the solve and whether their rows are staged in LDS
constexpr int kSaiLdsDoubles = 20000;
// (64 sweeping threads per workgroup: more workgroups share the staging loads, which
// dominate the solve at one problem)
__host__ __device__ inline int sai_chunks_per_group(int R, int bw) {
  const int by_threads = bw <= 64 ? 64 / bw : 1, by_lds = kSaiLdsDoubles / ((R + 2) * (bw + 3)) - 1;
  const int c = by_threads < by_lds ? by_threads : by_lds;
  return c < 1 ? 1 : c;
}
// staged: the group's rows of V_j and the three elimination coefficients per row
__host__ __device__ inline bool sai_stage_in_lds(int R, int bw) {
  return (int64_t)(sai_chunks_per_group(R, bw) + 1) * (R + 2) * (bw + 3) <= kSaiLdsDoubles;
}
int sai_solve_groups(int C, int R, int bw);
void launch_tri_factor(TriDev* td, int nprob, int maxC, hipStream_t st);
void launch_sai_solve(ProbDev* d, TriDev* td, int nprob, int groups, int64_t maxnbw, int j, int mixed,
                      hipStream_t st);
void launch_sai_gram(ProbDev* d, TriDev* td, int nprob, int64_t maxn, double* part, hipStream_t st);
void launch_hess_inverse(TriDev* td, int nprob, int maxN0, int maxbw, int maxl, hipStream_t st);

// x = V y (+ output column)
void launch_project(ProbDev* d, ExpmDev* e, int nprob, int64_t maxn, int max_lbw, int mixed, hipStream_t st);

// compression helpers (single problem)
void launch_row_norms(const double* R, int64_t ldR, int rows, int cols, double* rn, hipStream_t st);
void launch_vec_norm(const double* x, int64_t n, double* out, hipStream_t st);
void launch_fill_hash(double* x, int64_t n, uint64_t seed, hipStream_t st);
void launch_jacobi_svd(const double* R, int64_t ldR, const int* sel, int s, int r, double* A, double* J,
                       double* sig, int* perm, int* info, hipStream_t st);
void launch_form_u(const double* Q, int bwc, int64_t n, const int* sel, int r, const double* J, const int* perm,
                   int m, double* U, int64_t ldU, hipStream_t st);
void launch_fit(const double* A, int s, const int* perm, int m, const double* ts, double t0, double t1, int qcap,
                double fit_tol, double* Pi, int ldPi, double* work, double* info, hipStream_t st);
// piecewise-cubic p(t): not-a-knot spline coefficients of the m rows (work: 3 s m doubles)
void launch_spline(const double* A, int s, const int* perm, int m, const double* ts, double* Pw, double* work,
                   hipStream_t st);
void launch_spline_reset(ExpmDev* e, int nprob, hipStream_t st);

// column-pivoted Gram-Schmidt range finder of the shifted samples (compress.hip):
// Q (n x k, ld n) orthonormal, R = Q^T G (k x s, ld kcap); k and the squared norms of G
// and of the residual are in the state block (read back with read_cp_state)
constexpr int kCpMaxK = 128;     // column cap of the range finder
constexpr int kCpMaxRw = 4096;   // rows per chunk at most
constexpr double kCpFloor = 1e-15;  // stop when |residual|_F <= max(kCpFloor, 2 k eps) |G|_F
void cp_geometry(int64_t n, int s, int& rw, int& P, int& CG);
size_t cp_part_doubles(int64_t n, int s);
size_t cp_state_bytes();
void launch_cp_range(int64_t n, int s, int kcap, const double* G, double* A, double* Q, double* R, double* part,
                     double* cn2, double* rrow, unsigned* cnt, void* state, hipStream_t st);
void read_cp_state(const void* host_copy, int* k, double* gfro2, double* res2);

// waveform relaxation (Burgers): per-point operator and source samples of one window
// F: forcing samples of the window (n x s, ld n) added to the source, or null
void launch_wr_source(int64_t n, int s, double h, double nu, const double* U, int jacobian, double w_end, double w_in,
                      const double* F, double* coef, double* G, hipStream_t st);
void launch_diff_norms(const double* a, const double* b, int64_t cnt, double* part, int blocks, hipStream_t st);

// utilities
void launch_superpose(const double* u0, const double* const* v, int P, int64_t n, int n_out, int64_t ldv,
                      double* u, int64_t ldu, hipStream_t st);
void launch_check_finite(const double* x, int64_t n, int cols, int64_t ld, int* flag, hipStream_t st);
void launch_zero_u32(unsigned* x, int64_t n, hipStream_t st);
void launch_fill(double* x, int64_t n, int cols, int64_t ld, double v, hipStream_t st);
void launch_copy(const double* a, double* b, int64_t n, hipStream_t st);

}  // namespace pe
