// Wave and workgroup reductions and the cross-workgroup hand-off shared by the gfx950
// kernels of the Paraexp library.
#pragma once

#include <hip/hip_runtime.h>

#include "common.h"

namespace pe {

// DPP data movement of a double (both 32-bit halves); rows outside row_mask receive 0
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_move(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROW_MASK, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROW_MASK, 0xF, false);
  return __hiloint2double(hi, lo);
}

// Sum over the 64 lanes of a wave, returned to every lane.  Within each row of 16 lanes:
// quad_perm [1,0,3,2], quad_perm [2,3,0,1], row_ror 4, row_ror 8; then row_bcast 15 into
// rows 1 and 3 and row_bcast 31 into rows 2 and 3, which leaves the total in lane 63.
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_move<0xB1, 0xF>(v);
  v += dpp_move<0x4E, 0xF>(v);
  v += dpp_move<0x124, 0xF>(v);
  v += dpp_move<0x128, 0xF>(v);
  v += dpp_move<0x142, 0xA>(v);
  v += dpp_move<0x143, 0xC>(v);
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
  return __hiloint2double(hi, lo);
}

// sum over a workgroup whose size is a multiple of 64; `red` holds >= 16 doubles of LDS
__device__ __forceinline__ double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) red[w] = v;
  __syncthreads();
  double t = 0.0;
  const int nw = blockDim.x >> 6;
  for (int i = 0; i < nw; ++i) t += red[i];
  return t;
}

// Cross-workgroup hand-off inside a kernel: data for the last workgroup is stored
// write-through at agent scope, every thread waits for its stores, then thread 0 bumps
// the counter.  The last workgroup invalidates its L2 view (agent-scope acquire) before
// reading.  No L2 write-back is needed, unlike a full __threadfence per workgroup.
__device__ __forceinline__ void st_agent(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ bool arrive_last(unsigned* counter, unsigned expected, int* flag) {
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) *flag = (atomicAdd(counter, 1u) == expected - 1);
  __syncthreads();
  const bool last = *flag != 0;
  if (last) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  return last;
}

// Bulk copy: element e of [0, cnt) is read with src(e) and stored with put(e, v); each
// thread keeps kBulkDepth loads in flight (clamped addresses, unconditional loads)
constexpr int kBulkDepth = 8;
template <int D = kBulkDepth, typename Src, typename Put>
__device__ __forceinline__ void bulk_load(int64_t cnt, Src src, Put put) {
  const int T = blockDim.x;
  for (int64_t e0 = threadIdx.x; e0 < cnt; e0 += D * (int64_t)T) {
    double v[D];
#pragma unroll
    for (int k = 0; k < D; ++k) {
      const int64_t e = e0 + (int64_t)k * T;
      const double x = src(e < cnt ? e : cnt - 1);  // clamped, unconditional: loads stay in flight
      v[k] = e < cnt ? x : 0.0;
    }
#pragma unroll
    for (int k = 0; k < D; ++k) {
      const int64_t e = e0 + (int64_t)k * T;
      if (e < cnt) put(e, v[k]);
    }
  }
}

// Workgroup barrier that orders LDS accesses only: outstanding global loads and stores
// stay in flight across it (a __syncthreads waits for them as well)
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}


// ---- access to the per-problem block workspace (ProbDev) ----------------------------
template <typename TS>
__device__ __forceinline__ TS* basis_ptr(const ProbDev& p);
template <>
__device__ __forceinline__ double* basis_ptr<double>(const ProbDev& p) { return p.V; }
template <>
__device__ __forceinline__ float* basis_ptr<float>(const ProbDev& p) { return p.V32; }

__device__ __forceinline__ void stencil_coefs(const ProbDev& p, int64_t r, double& cm, double& cz, double& cp) {
  if (p.per_point) {
    cm = p.coef[r];
    cz = p.coef[p.n + r];
    cp = p.coef[2 * p.n + r];
  } else {
    cm = p.c3[0];
    cz = p.c3[1];
    cp = p.c3[2];
  }
}

// chunk of a row for the update (TSQR) partition: the last chunk takes the remainder
__device__ __forceinline__ int chunk_of(const ProbDev& p, int64_t r) {
  int64_t u = r >> p.rows_u_log2;
  return (int)(u < p.Cu - 1 ? u : p.Cu - 1);
}

// entry (r, col) of a TSQR output block: Qloc[r, :] . Qs[u(r)][:, col]
__device__ __forceinline__ double tsqr_entry(const ProbDev& p, const double* Qloc, const double* Qs, int64_t r,
                                             int col) {
  const int bw = p.bw;
  const int u = chunk_of(p, r);
  const double* q = Qloc + r * bw;
  const double* s = Qs + (int64_t)u * bw * bw + col;
  double acc = 0.0;
  for (int k = 0; k < bw; ++k) acc += q[k] * s[k * bw];
  return acc;
}

}  // namespace pe
