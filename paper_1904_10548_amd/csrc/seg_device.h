// Device helpers shared by the sweep kernels (segment and scan forms).
#pragma once

#include <cmath>

#include "kernels.h"

namespace tapg {

namespace {

// Control state of a backward launch's tree: read from ctl, or, in the first
// backward launch of an iteration that closes the previous one, advanced from
// ctl_prev by every workgroup alike and written (with the residual history
// entry) by the tree's first workgroup (wg: index among the level's) of the
// launch.
template <typename T>
__device__ inline DevCtl bwd_ctl(const SegArgs<T>& a, int tree, int wg) {
  if (!a.close) return a.ctl[tree];
  const DevCtl p = a.ctl_prev[tree];
  bool record;
  double res = 0.0;
  const DevCtl n = ctl_advance(p, &record, &res);
  const bool writer = wg == 0 || (a.wgtree && a.wgtree[wg - 1] != tree);
  if (writer && threadIdx.x == 0) {
    a.ctl[tree] = n;
    if (record) a.hist[(size_t)tree * a.hist_stride + p.iter] = res;
  }
  return n;
}

// The state of a tree's first backward launch as every workgroup advances it
// (bwd_ctl without the write: for workgroups that are not the tree's first).
template <typename T>
__device__ inline DevCtl bwd_ctl_peek(const SegArgs<T>& a, int tree) {
  bool record;
  double res = 0.0;
  return ctl_advance(a.ctl_prev[tree], &record, &res);
}

template <typename T>
__device__ __forceinline__ T wext(T y, T yp, T beta) {
  return y + beta * (y - yp);
}

// Wait until every vector memory operation of the wave has completed:
// s_waitcnt vmcnt(0), expcnt and lgkmcnt left at their maxima (gfx9 encoding:
// vmcnt [3:0] and [15:14], expcnt [6:4], lgkmcnt [11:8]).
__device__ __forceinline__ void vm_wait_all() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// Load from a clamped index (element 0 when !ok), NOT masked: a select right
// after the load would make the compiler wait for it there.  Prefetched values
// are masked where they are consumed, one stage later.
template <typename T>
__device__ __forceinline__ T ldc(const T* __restrict__ p, size_t idx, bool ok) {
  return p[ok ? idx : 0];
}

// Load from a clamped index, masked at once (stage-invariant data only).
template <typename T>
__device__ __forceinline__ T ldm(const T* __restrict__ p, size_t idx, bool ok) {
  const T v = p[ok ? idx : 0];
  return ok ? v : T(0);
}

// A double moved across lanes by a DPP pattern (each 32-bit half separately).
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

// Sum over the 64 lanes of a wave (all lanes active), every lane getting the
// same value: each step adds to a lane the value of a partner lane in the
// other half of its current group, and both partners form the same sum (a + b
// = b + a), so the result is identical in every lane and from run to run.
// Steps: xor 1 and xor 2 inside a quad, mirror inside 8 and 16 lanes (DPP),
// then rows 16 apart and halves 32 apart (gfx950 permlane swaps: with both
// operands equal to v, the pair returned holds v of the lower and of the
// upper partner in the same order in every lane).
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_f64<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_f64<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_f64<0x141>(v);  // row_half_mirror
  v += dpp_f64<0x140>(v);  // row_mirror
  {
    const auto lo = __builtin_amdgcn_permlane16_swap(__double2loint(v), __double2loint(v), false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap(__double2hiint(v), __double2hiint(v), false, false);
    v = __hiloint2double((int)hi[0], (int)lo[0]) + __hiloint2double((int)hi[1], (int)lo[1]);
  }
  {
    const auto lo = __builtin_amdgcn_permlane32_swap(__double2loint(v), __double2loint(v), false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap(__double2hiint(v), __double2hiint(v), false, false);
    v = __hiloint2double((int)hi[0], (int)lo[0]) + __hiloint2double((int)hi[1], (int)lo[1]);
  }
  return v;
}

__device__ __forceinline__ double block_max512(double v, double* s) {
  s[threadIdx.x] = v;
  __syncthreads();
  for (int st = kSegThreads / 2; st > 0; st >>= 1) {
    if (threadIdx.x < st) s[threadIdx.x] = fmax(s[threadIdx.x], s[threadIdx.x + st]);
    __syncthreads();
  }
  const double r = s[0];
  __syncthreads();
  return r;
}

__device__ __forceinline__ double block_sum512(double v, double* s) {
  s[threadIdx.x] = v;
  __syncthreads();
  for (int st = kSegThreads / 2; st > 0; st >>= 1) {
    if (threadIdx.x < st) s[threadIdx.x] += s[threadIdx.x + st];
    __syncthreads();
  }
  const double r = s[0];
  __syncthreads();
  return r;
}

// The first K entries of one CSR row held in registers (the row is the same
// at every stage), the rest of the row, rare in a flow network whose rows have
// a few entries each, read from LDS.  apply() adds the row's products in CSR
// order; the register entries' loads are independent of each other.
template <typename T, int K>
struct RegRow {
  int col[K];
  T val[K];
  int n, xb, xe;  // entries in registers; LDS range [xb, xe) of the others
  __device__ __forceinline__ void load(const int* srow, const int* scol, const T* sval, int i,
                                       bool ok) {
    const int p0 = ok ? srow[i] : 0, p1 = ok ? srow[i + 1] : 0;
    n = min(p1 - p0, K);
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int p = k < n ? p0 + k : 0;
      col[k] = k < n ? scol[p] : 0;
      val[k] = k < n ? sval[p] : T(0);
    }
    xb = p0 + n;
    xe = p1;
  }
  __device__ __forceinline__ T apply(T acc, const T* X, const int* scol, const T* sval) const {
    T t[K];
#pragma unroll
    for (int k = 0; k < K; ++k) t[k] = X[col[k]];
#pragma unroll
    for (int k = 0; k < K; ++k)
      if (k < n) acc += val[k] * t[k];
    for (int p = xb; p < xe; ++p) acc += sval[p] * X[scol[p]];
    return acc;
  }
};

// Copy of a CSR matrix into LDS (row pointers, columns, values).
template <typename T>
__device__ __forceinline__ void csr_to_lds(const int* row, const int* col, const T* val, int nrows,
                                           int nnz, int* srow, int* scol, T* sval) {
  for (int i = threadIdx.x; i <= nrows; i += kSegThreads) srow[i] = row[i];
  for (int i = threadIdx.x; i < nnz; i += kSegThreads) {
    scol[i] = col[i];
    sval[i] = val[i];
  }
}

}  // namespace


}  // namespace tapg
