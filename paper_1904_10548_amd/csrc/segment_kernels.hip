// Segment sweep kernels for gfx950.
//
// The tree is cut into levels of consecutive stages.  In a level, workgroup w
// owns a group of consecutive nodes at the level's first stage and all their
// descendants down to the level's last stage; by the breadth-first numbering
// these are one contiguous node range per stage.  A workgroup therefore walks
// all stages of its level without any grid-wide synchronisation: children
// (backward) and parents (forward) of its nodes are its own nodes of the
// neighbouring stage, kept in LDS.  Only level boundaries go through global
// memory, between launches.
//
// Latency is the enemy of a stage-by-stage walk, so nothing inside the stage
// loop waits on a global load that could have been issued earlier:
//  * stage-invariant data (the workgroup's node ranges, the CSR of B / B',
//    the bounds) is loaded once per launch into LDS or registers;
//  * the stage factor Fbar_s (nu x nu, u-dimension padded to 128) is held in
//    registers: thread t owns row t % 128 and the 32-column slice t / 128.
//    It is reloaded only when the next stage is served by another factor
//    block (stages whose factors agree to rounding share one; with W_u = w I
//    every Fbar_s is Z Z' / w, so a launch loads it once);
//  * every per-node input of the next stage (duals, tree indices, kappa / j,
//    1/p, g) is loaded while the current stage computes;
//  * a stage's global stores are issued at the start of the next stage, so
//    the one wait per stage (at its start) finds them long completed.
//
// Structure used: W_u = w I gives Kbar_s = w Fbar_s, so one matrix per stage
// serves both sweeps (general W_u: Kbar_s v = Fbar_s (W_u v), W_u streamed);
// A = I skips the A products (general A: streamed); B and B' are applied from
// their CSR (a flow network's incidence has a few entries per row).
#include <cmath>

#include "kernels.h"

namespace tapg {

namespace {

constexpr int kRT = 128;   // rows per slice of a register-resident GEMV
constexpr int kKS = kSegThreads / kRT;
constexpr int kKC = 32;    // columns per slice
constexpr int kLDU = 128;  // padded u-dimension of the segment layout

template <typename T>
__device__ __forceinline__ T wext(T y, T yp, T beta) {
  return y + beta * (y - yp);
}

// m[j] = Fbar_s(r, kb + j); the padded stage block makes all 32 loads valid
// and unconditional, so they issue back to back.
template <typename T>
__device__ __forceinline__ void load_factor(const T* __restrict__ F, int r, int kb,
                                            T (&m)[kKC]) {
  const T* base = F + (size_t)kb * kLDU + r;
#pragma unroll
  for (int j = 0; j < kKC; ++j) m[j] = base[j * kLDU];
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

// Streamed GEMV partials for a general matrix (A, A' or W_u), used only when
// A != I or W_u is not a multiple of I: red[(ks*NB + b)*128 + r] =
// sum_{k in slice ks} M(r, k) X[b][k].
template <typename T, int NB>
__device__ __noinline__ void stream_partials(const T* __restrict__ M, int ldm_, int R, int K,
                                             const T* X, int ldx, int ncols, T* red) {
  const int r = threadIdx.x % kRT;
  const int ks = __builtin_amdgcn_readfirstlane(threadIdx.x / kRT);
  const int kc = (K + kKS - 1) / kKS;
  const int kb = ks * kc, ke = min(K, kb + kc);
  for (int b = 0; b < ncols && b < NB; ++b) {
    T acc = T(0);
    if (r < R) {
#pragma unroll 8
      for (int k = kb; k < ke; ++k) acc += M[(size_t)k * ldm_ + r] * X[b * ldx + k];
    }
    red[(ks * NB + b) * kRT + r] = acc;
  }
}

template <typename T, int NB>
__device__ __forceinline__ T sum_partials(const T* red, int b, int r) {
  T s = red[(0 * NB + b) * kRT + r];
#pragma unroll
  for (int q = 1; q < kKS; ++q) s += red[(q * NB + b) * kRT + r];
  return s;
}

// Sum over the 64 lanes of a wave by a xor butterfly: every lane gets the
// same, run-to-run identical value (each pairwise sum is commutative).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
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

// Bytes of dynamic LDS of a segment launch: iterate buffers, GEMV partials,
// the workgroup's node ranges and one CSR (B or B').
template <typename T, int NB>
size_t seg_lds_bytes(const SegArgs<T>& a) {
  const int nrows = a.nu > a.nx ? a.nu : a.nx;
  const int cb = a.nch > NB ? a.nch : NB;  // child buffers also hold the boundary children
  size_t b = (size_t)(2 * cb * a.LDX + 2 * cb * a.LDU + 4 * NB * kRT) * sizeof(T);
  b += (size_t)a.nst * sizeof(int2) + (size_t)(a.nst + 1) * sizeof(int);  // ranges, factor ids
  b += (size_t)(nrows + 2 + a.nnzB) * sizeof(int);
  b += (size_t)a.nnzB * sizeof(T);
  return (b + 15) & ~(size_t)15;
}

// ---------------------------------------------------------------------------
// Backward sweep over one level, stages s_end down to s_begin.  Per node:
//   lambda_n = a_n + A' sum_{c} lambda_c                 (a_n = w1_n + w2_n)
//   v_n      = -(w3_n + B' lambda_n)/2 + W_u sum_{c} j_c
//   j_n      = kappa_n + Fbar_s v_n
// ---------------------------------------------------------------------------
template <typename T, int NB>
__global__ __launch_bounds__(kSegThreads) void seg_bwd_kernel(SegArgs<T> a) {
  const DevCtl* ctl = a.ctl;
  if (ctl->done) return;
  constexpr int QX = NB * 128 / kSegThreads > 0 ? NB * 128 / kSegThreads : 1;
  const int tid = threadIdx.x;
  const int it = ctl->iter;
  const bool power = a.mode == 1;
  const T* Yc = (it & 1) ? a.Y1 : a.Y0;
  const T* Yo = (it & 1) ? a.Y0 : a.Y1;
  const T beta = (T)ctl->beta;
  const T scale = (T)ctl->pw_scale;
  const int nx = a.nx, nu = a.nu, LDX = a.LDX, LDU = a.LDU, LDY = a.LDY;

  const int CB = a.nch > NB ? a.nch : NB;  // capacity of the child buffers
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* sL0 = reinterpret_cast<T*>(smem_raw);  // lambda ping-pong
  T* sL1 = sL0 + CB * LDX;
  T* sJ = sL1 + CB * LDX;  // children's j, then this stage's j
  T* sV = sJ + CB * LDU;   // GEMV input
  T* red = sV + CB * LDU;  // 4 * NB * 128 partials
  int2* sRg = reinterpret_cast<int2*>(red + 4 * NB * kRT);
  int* sFid = reinterpret_cast<int*>(sRg + a.nst);   // factor block of each stage
  int* sRow = sFid + a.nst + (a.nst & 1);            // CSR of B' (nu rows), 8-byte aligned
  int* sCol = sRow + nu + 1;
  T* sVal = reinterpret_cast<T*>(sCol + a.nnzB + ((nu + 1 + a.nnzB) & 1));  // 8-byte aligned
  {
    const int2* rg = a.ranges + (size_t)blockIdx.x * a.nst;
    for (int i = tid; i < a.nst; i += kSegThreads) {
      sRg[i] = rg[i];
      sFid[i] = a.fid[a.s_begin + i];
    }
    csr_to_lds<T>(a.Btrow, a.Btcol, a.Btval, nu, a.nnzB, sRow, sCol, sVal);
    __syncthreads();
  }

  const int r = tid % kRT;
  const int ks = __builtin_amdgcn_readfirstlane(tid / kRT);  // wave-uniform slice
  const int kb = ks * kKC;

  // Per-node inputs of a stage from global memory: per x-slot (y1, y1o, y2,
  // y2o, first/last child) and u-slot (y3, y3o, kappa, first/last child).  Two
  // sets alternate between stages, so the loads for stage s-1 fly while stage
  // s computes and no register is copied.
  struct Pre {
    T px[QX][4], pu[QX][3];
    int cx[QX][2], cu[QX][2];
  };
  Pre PA, PB;
  // The stage factor lives in registers and is reloaded only when the next
  // stage is served by another block (right after the GEMV that consumed it).
  T mreg[kKC];
  int f_cur = __builtin_amdgcn_readfirstlane(sFid[a.s_end - a.s_begin]);
  load_factor<T>(a.F + (size_t)f_cur * kLDU * kLDU, r, kb, mreg);
  auto load_stage = [&](int s_, Pre& P) {

    const int2 rr_ = sRg[s_ - a.s_begin];
    const int lo_ = rr_.x, nb_ = rr_.y - rr_.x;
    #pragma unroll
    for (int q = 0; q < QX; ++q) {
      const int idx = tid + q * kSegThreads;
      const int b = idx / LDX, i = idx - b * LDX;
      const bool ok = idx < NB * LDX && b < nb_ && i < nx;
      const size_t o = (size_t)(lo_ + b) * LDY + i;
      P.px[q][0] = ldc(Yc, o, ok);
      P.px[q][1] = ldc(Yo, o, ok);
      P.px[q][2] = ldc(Yc, o + LDX, ok);
      P.px[q][3] = ldc(Yo, o + LDX, ok);
      P.cx[q][0] = ldc(a.cbeg, lo_ + b, ok);
      P.cx[q][1] = ldc(a.cend, lo_ + b, ok);
    }
    #pragma unroll
    for (int q = 0; q < QX; ++q) {
      const int idx = tid + q * kSegThreads;
      const int b = idx / LDU, i = idx - b * LDU;
      const bool ok = idx < NB * LDU && b < nb_ && i < nu;
      const size_t n = (size_t)(lo_ + b);
      P.pu[q][0] = ldc(Yc, n * LDY + 2 * LDX + i, ok);
      P.pu[q][1] = ldc(Yo, n * LDY + 2 * LDX + i, ok);
      P.pu[q][2] = ldc(a.kappa, n * LDU + i, ok);
      P.cu[q][0] = ldc(a.cbeg, n, ok);
      P.cu[q][1] = ldc(a.cend, n, ok);
    }
  };

  int s = a.s_end;
  load_stage(s, PA);
  T* sLc = sL0;  // children's lambda (stage s+1)
  T* sLn = sL1;  // this stage's lambda
  int lo_c = 0;  // first child node held in LDS
  if (s + 1 < a.N) {  // children of the level's last stage: written by the level below
    const int2 rr = sRg[s - a.s_begin];
    lo_c = a.cbeg[rr.x];
    const int nc = a.cend[rr.y - 1] - lo_c;
    for (int idx = tid; idx < nc * LDX; idx += kSegThreads) {
      const int b = idx / LDX, i = idx - b * LDX;
      sLc[idx] = i < nx ? a.lam[(size_t)(lo_c + b) * LDX + i] : T(0);
    }
    for (int idx = tid; idx < nc * LDU; idx += kSegThreads) {
      const int b = idx / LDU, i = idx - b * LDU;
      sJ[idx] = i < nu ? a.jv[(size_t)(lo_c + b) * LDU + i] : T(0);
    }
  }
  const bool has_kids_last = s + 1 < a.N;
  __syncthreads();

  // A stage's global stores (j) are issued at the start of the next stage,
  // after its wait for the prefetched loads.  Loads and stores in flight
  // together complete out of order, so that wait has to count both: stores
  // issued at the very end of a stage would make the next stage wait for
  // their acknowledgement, delayed ones were issued a stage earlier.
  T dj[QX];
  int dn[QX];  // element offset into j, -1: nothing pending
#pragma unroll
  for (int q = 0; q < QX; ++q) dn[q] = -1;
  auto flush = [&]() {
#pragma unroll
    for (int q = 0; q < QX; ++q)
      if (dn[q] >= 0) a.jv[dn[q]] = dj[q];
  };

  auto stage = [&](int s, Pre& C, Pre& Nx) {
    vm_wait_all();  // this stage's prefetch and the previous stage's stores
    const int2 rr = sRg[s - a.s_begin];
    const int lo = rr.x, nb = rr.y - rr.x;
    const bool kids = s < a.s_end || has_kids_last;  // children are in LDS

    // consume the prefetched inputs of this stage
    T aval[QX], w3v[QX], sig[QX], kap[QX], lsum[QX];
#pragma unroll
    for (int q = 0; q < QX; ++q) {
      const int idx = tid + q * kSegThreads;
      const int b = idx / LDX, i = idx - b * LDX;
      const bool ok = idx < NB * LDX && b < nb && i < nx;
      const T av = power ? scale * (C.px[q][0] + C.px[q][2])
                         : wext(C.px[q][0], C.px[q][1], beta) + wext(C.px[q][2], C.px[q][3], beta);
      aval[q] = ok ? av : T(0);
      T ls = T(0);
      if (ok && kids) {
        for (int c = C.cx[q][0]; c < C.cx[q][1]; ++c) ls += sLc[(c - lo_c) * LDX + i];
      }
      lsum[q] = ls;
    }
#pragma unroll
    for (int q = 0; q < QX; ++q) {
      const int idx = tid + q * kSegThreads;
      const int b = idx / LDU, i = idx - b * LDU;
      const bool ok = idx < NB * LDU && b < nb && i < nu;
      w3v[q] = power ? scale * C.pu[q][0] : wext(C.pu[q][0], C.pu[q][1], beta);
      kap[q] = power ? T(0) : C.pu[q][2];
      T sg = T(0);
      if (ok && kids) {
        for (int c = C.cu[q][0]; c < C.cu[q][1]; ++c) sg += sJ[(c - lo_c) * LDU + i];
      }
      sig[q] = ok ? sg : T(0);
    }
    flush();
    // the next stage's factor and inputs load while this stage computes.  The
    // load is unconditional (the level's first stage reloads itself): under a
    // branch the compiler's wait counting merges both paths and would wait for
    // these loads right here.
    load_stage(s > a.s_begin ? s - 1 : s, Nx);
#pragma unroll
    for (int q = 0; q < QX; ++q) {
      const int idx = tid + q * kSegThreads;
      if (idx < NB * LDX) sLn[idx] = a.a_ident ? (aval[q] + lsum[q]) : lsum[q];
    }
    __syncthreads();
    if (!a.a_ident) {  // lambda = a + A' lambda_sum
      stream_partials<T, NB>(a.At, LDX, nx, nx, sLn, LDX, nb, red);
      __syncthreads();
#pragma unroll
      for (int q = 0; q < QX; ++q) {
        const int idx = tid + q * kSegThreads;
        const int b = idx / LDX, i = idx - b * LDX;
        if (idx < NB * LDX) {
          const bool ok = b < nb && i < nx;
          sLn[idx] = ok ? aval[q] + sum_partials<T, NB>(red, b, i) : T(0);
        }
      }
      __syncthreads();
    }
    // v = -(w3 + B' lambda)/2 + W_u sigma
    T vv[QX];
#pragma unroll
    for (int q = 0; q < QX; ++q) {
      const int idx = tid + q * kSegThreads;
      const int b = idx / LDU, i = idx - b * LDU;
      const bool ok = idx < NB * LDU && b < nb && i < nu;
      T e = w3v[q];
      if (ok) {
        const int pe = sRow[i + 1];
        for (int p = sRow[i]; p < pe; ++p) e += sVal[p] * sLn[b * LDX + sCol[p]];
      }
      vv[q] = ok ? T(-0.5) * e + (a.wu_scalar ? a.wu * sig[q] : T(0)) : T(0);
      if (idx < NB * LDU) sV[idx] = a.wu_scalar ? vv[q] : sig[q];
    }
    __syncthreads();
    if (!a.wu_scalar) {  // v += W_u sigma
      stream_partials<T, NB>(a.Wu, LDU, nu, nu, sV, LDU, nb, red);
      __syncthreads();
#pragma unroll
      for (int q = 0; q < QX; ++q) {
        const int idx = tid + q * kSegThreads;
        const int b = idx / LDU, i = idx - b * LDU;
        if (idx < NB * LDU) {
          const bool ok = b < nb && i < nu;
          sV[idx] = ok ? vv[q] + sum_partials<T, NB>(red, b, i) : T(0);
        }
      }
      __syncthreads();
    }
    // j = kappa + Fbar_s v   (register-resident Fbar_s)
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      if (b < nb) {
        T acc = T(0);
#pragma unroll
        for (int j = 0; j < kKC; ++j) acc += mreg[j] * sV[b * kLDU + kb + j];
        red[(ks * NB + b) * kRT + r] = acc;
      }
    }
    if (s > a.s_begin) {
      const int fn = __builtin_amdgcn_readfirstlane(sFid[s - 1 - a.s_begin]);
      if (fn != f_cur) {
        f_cur = fn;
        load_factor<T>(a.F + (size_t)fn * kLDU * kLDU, r, kb, mreg);
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < QX; ++q) {
      const int idx = tid + q * kSegThreads;
      const int b = idx / LDU, i = idx - b * LDU;
      dn[q] = -1;
      if (idx < NB * LDU && b < nb && i < nu) {
        const T jn = kap[q] + sum_partials<T, NB>(red, b, i);
        sJ[b * LDU + i] = jn;
        dj[q] = jn;
        dn[q] = (lo + b) * LDU + i;
      }
    }
    if (s == a.s_begin && s > 0) {  // the parent level reads this stage's lambda
#pragma unroll
      for (int q = 0; q < QX; ++q) {
        const int idx = tid + q * kSegThreads;
        const int b = idx / LDX, i = idx - b * LDX;
        if (idx < NB * LDX && b < nb && i < nx) a.lam[(size_t)(lo + b) * LDX + i] = sLn[idx];
      }
    }
    __syncthreads();
    T* t = sLc;
    sLc = sLn;
    sLn = t;
    lo_c = lo;
  };
  while (true) {
    stage(s, PA, PB);
    if (--s < a.s_begin) break;
    stage(s, PB, PA);
    if (--s < a.s_begin) break;
  }
  flush();
}

// ---------------------------------------------------------------------------
// Forward sweep over one level, stages s_begin up to s_end, with the fused
// prox / dual update.  Per node:
//   u_n = Fbar_s (W_u u_anc) + j_n / p_n       (= Kbar_s u_anc + k_n)
//   x_n = A x_anc + B u_n + g_n
//   v = w + gamma (x_n, x_n, u_n);  blocks 1, 2: r = v - gamma P_C(v/gamma),
//   y+ = r min(1, W / |r|);  block 3: y+ = v - gamma P_U(v/gamma)
// The product Fbar_s (W_u u_anc) is formed once per parent.  The launch of
// the last level ends the iteration in its last workgroup to finish.
// ---------------------------------------------------------------------------
template <typename T, int NB>
__global__ __launch_bounds__(kSegThreads) void seg_fwd_kernel(SegArgs<T> a) {
  DevCtl* ctl = a.ctl;
  if (ctl->done) return;
  constexpr int QX = NB * 128 / kSegThreads > 0 ? NB * 128 / kSegThreads : 1;
  const int tid = threadIdx.x;
  const int it = ctl->iter;
  const bool power = a.mode == 1;
  const T* Yc = (it & 1) ? a.Y1 : a.Y0;
  T* Yn = (it & 1) ? a.Y0 : a.Y1;  // y^{nu-1} in, y^{nu+1} out
  const T beta = (T)ctl->beta;
  const double gam64 = ctl->gamma;
  const T gam = (T)gam64;
  const int nx = a.nx, nu = a.nu, LDX = a.LDX, LDU = a.LDU, LDY = a.LDY;

  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* sU0 = reinterpret_cast<T*>(smem_raw);
  T* sU1 = sU0 + NB * LDU;
  T* sX0 = sU1 + NB * LDU;
  T* sX1 = sX0 + NB * LDX;
  T* red = sX1 + NB * LDX;  // 4 * NB * 128 partials; reused for the norms
  int2* sRg = reinterpret_cast<int2*>(red + 4 * NB * kRT);
  int* sFid = reinterpret_cast<int*>(sRg + a.nst);   // factor block of each stage
  int* sRow = sFid + a.nst + (a.nst & 1);            // CSR of B (nx rows), 8-byte aligned
  int* sCol = sRow + nx + 1;
  T* sVal = reinterpret_cast<T*>(sCol + a.nnzB + ((nx + 1 + a.nnzB) & 1));  // 8-byte aligned
  __shared__ double sred[kSegThreads];
  __shared__ int s_last;
  {
    const int2* rg = a.ranges + (size_t)blockIdx.x * a.nst;
    for (int i = tid; i < a.nst; i += kSegThreads) {
      sRg[i] = rg[i];
      sFid[i] = a.fid[a.s_begin + i];
    }
    csr_to_lds<T>(a.Brow, a.Bcol, a.Bval, nx, a.nnzB, sRow, sCol, sVal);
  }

  const int r = tid % kRT;
  const int ks = __builtin_amdgcn_readfirstlane(tid / kRT);
  const int kb = ks * kKC;
  // stage-invariant bounds of this thread's slots
  T bxlo[QX], bxhi[QX], bxs[QX], bulo[QX], buhi[QX];
#pragma unroll
  for (int q = 0; q < QX; ++q) {
    const int ix = (tid + q * kSegThreads) % LDX, iu = (tid + q * kSegThreads) % LDU;
    bxlo[q] = ldm(a.xmin, ix, ix < nx);
    bxhi[q] = ldm(a.xmax, ix, ix < nx);
    bxs[q] = ldm(a.xs, ix, ix < nx);
    bulo[q] = ldm(a.umin, iu, iu < nu);
    buhi[q] = ldm(a.umax, iu, iu < nu);
  }
  // Per-node inputs of a stage: u-slots (j, 1/p, parent, y3, y3o), x-slots
  // (g, parent, y1, y1o, y2, y2o).  Two sets alternate between stages, so the
  // loads for stage s+1 fly while stage s computes and no register is copied.
  struct Pre {
    T pj[QX], pp[QX], py3[QX][2], pg[QX], py12[QX][4];
    int pau[QX], pax[QX];
  };
  Pre PA, PB;
  T mreg[kKC];  // reloaded right after a GEMV when the next stage has another factor block
  auto load_stage = [&](int s_, Pre& P) {

    const int2 rr_ = sRg[s_ - a.s_begin];
    const int lo_ = rr_.x, nb_ = rr_.y - rr_.x;
    #pragma unroll
    for (int q = 0; q < QX; ++q) {
      const int idx = tid + q * kSegThreads;
      const int b = idx / LDU, i = idx - b * LDU;
      const bool ok = idx < NB * LDU && b < nb_ && i < nu;
      const size_t n = (size_t)(lo_ + b);
      P.pj[q] = ldc(a.jv, n * LDU + i, ok);
      P.pp[q] = ldc(a.invp, n, ok);
      P.pau[q] = ldc(a.anc, n, ok);
      P.py3[q][0] = ldc(Yc, n * LDY + 2 * LDX + i, ok);
      P.py3[q][1] = ldc((const T*)Yn, n * LDY + 2 * LDX + i, ok);
    }
    #pragma unroll
    for (int q = 0; q < QX; ++q) {
      const int idx = tid + q * kSegThreads;
      const int b = idx / LDX, i = idx - b * LDX;
      const bool ok = idx < NB * LDX && b < nb_ && i < nx;
      const size_t n = (size_t)(lo_ + b);
      P.pg[q] = ldc(a.g, n * LDX + i, ok);
      P.pax[q] = ldc(a.anc, n, ok);
      P.py12[q][0] = ldc(Yc, n * LDY + i, ok);
      P.py12[q][1] = ldc((const T*)Yn, n * LDY + i, ok);
      P.py12[q][2] = ldc(Yc, n * LDY + LDX + i, ok);
      P.py12[q][3] = ldc((const T*)Yn, n * LDY + LDX + i, ok);
    }
  };

  int s = a.s_begin;
  __syncthreads();  // sRg, sFid ready
  int f_cur = __builtin_amdgcn_readfirstlane(sFid[0]);
  load_factor<T>(a.F + (size_t)f_cur * kLDU * kLDU, r, kb, mreg);
  load_stage(s, PA);
  T* sUp = sU0;  // parents (stage s-1)
  T* sUn = sU1;
  T* sXp = sX0;
  T* sXn = sX1;
  int lo_p = 0, np = 0;
  {  // parents of the first stage come from global memory (or p, q at the root)
    const int2 rr = sRg[0];
    const int par0 = a.anc[rr.x];
    lo_p = par0 >= 0 ? par0 : 0;
    np = par0 >= 0 ? a.anc[rr.y - 1] - par0 + 1 : 1;
    for (int idx = tid; idx < NB * LDU; idx += kSegThreads) {
      const int b = idx / LDU, i = idx - b * LDU;
      T v = T(0);
      if (b < np && i < nu)
        v = par0 >= 0 ? a.u[(size_t)(lo_p + b) * LDU + i] : (power ? T(0) : a.pq[LDX + i]);
      sUp[idx] = v;
    }
    for (int idx = tid; idx < NB * LDX; idx += kSegThreads) {
      const int b = idx / LDX, i = idx - b * LDX;
      T v = T(0);
      if (b < np && i < nx)
        v = par0 >= 0 ? a.x[(size_t)(lo_p + b) * LDX + i] : (power ? T(0) : a.pq[i]);
      sXp[idx] = v;
    }
  }
  double rmax = 0.0, zsq = 0.0;
  const bool wave_norm = LDX == 64;  // one node's x-block is exactly one wave

  // A stage's global stores (u, x, y+) are issued at the start of the next
  // stage, after its wait for the prefetched loads (as in the backward sweep).
  T du[QX], dy3[QX], dxv[QX], dy1[QX], dy2[QX];
  int dnu[QX], dnx[QX];  // node of the pending u-slot / x-slot values, -1: none
#pragma unroll
  for (int q = 0; q < QX; ++q) dnu[q] = dnx[q] = -1;
  auto flush = [&]() {
#pragma unroll
    for (int q = 0; q < QX; ++q) {
      const int iu = (tid + q * kSegThreads) % LDU;
      if (dnu[q] >= 0) {
        a.u[(size_t)dnu[q] * LDU + iu] = du[q];
        Yn[(size_t)dnu[q] * LDY + 2 * LDX + iu] = dy3[q];
      }
      const int ix = (tid + q * kSegThreads) % LDX;
      if (dnx[q] >= 0) {
        a.x[(size_t)dnx[q] * LDX + ix] = dxv[q];
        Yn[(size_t)dnx[q] * LDY + ix] = dy1[q];
        Yn[(size_t)dnx[q] * LDY + LDX + ix] = dy2[q];
      }
    }
  };

  auto stage = [&](int s, Pre& C, Pre& Nx) {
    vm_wait_all();  // this stage's prefetch and factor, the previous stage's stores
    const int2 rr = sRg[s - a.s_begin];
    const int lo = rr.x, nb = rr.y - rr.x;
    // consume the prefetched inputs (the extrapolation w is formed at once)
    T w3c[QX], w1c[QX], w2c[QX];
#pragma unroll
    for (int q = 0; q < QX; ++q) {
      w3c[q] = wext(C.py3[q][0], C.py3[q][1], beta);
      w1c[q] = wext(C.py12[q][0], C.py12[q][1], beta);
      w2c[q] = wext(C.py12[q][2], C.py12[q][3], beta);
    }
    flush();
    load_stage(s < a.s_end ? s + 1 : s, Nx);  // unconditional, as in the backward sweep
    __syncthreads();
    const T* V = sUp;
    if (!a.wu_scalar) {  // W_u u_anc per parent, into sUn
      stream_partials<T, NB>(a.Wu, LDU, nu, nu, sUp, LDU, np, red);
      __syncthreads();
      for (int idx = tid; idx < NB * LDU; idx += kSegThreads) {
        const int b = idx / LDU, i = idx - b * LDU;
        sUn[idx] = (b < np && i < nu) ? sum_partials<T, NB>(red, b, i) : T(0);
      }
      __syncthreads();
      V = sUn;
    }
    // Fbar_s (W_u u_anc), one column per parent
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      if (b < np) {
        T acc = T(0);
#pragma unroll
        for (int j = 0; j < kKC; ++j) acc += mreg[j] * V[b * kLDU + kb + j];
        red[(ks * NB + b) * kRT + r] = acc;
      }
    }
    // this stage's factor is consumed: load the next stage's into the same
    // registers if it is another block
    if (s < a.s_end) {
      const int fn = __builtin_amdgcn_readfirstlane(sFid[s + 1 - a.s_begin]);
      if (fn != f_cur) {
        f_cur = fn;
        load_factor<T>(a.F + (size_t)fn * kLDU * kLDU, r, kb, mreg);
      }
    }
    __syncthreads();
    const T wsc = a.wu_scalar ? a.wu : T(1);
    T uv[QX];
#pragma unroll
    for (int q = 0; q < QX; ++q) {
      const int idx = tid + q * kSegThreads;
      const int b = idx / LDU, i = idx - b * LDU;
      T un = T(0);
      dnu[q] = -1;
      if (idx < NB * LDU && b < nb && i < nu) {
        const int pb = C.pau[q] >= 0 ? C.pau[q] - lo_p : 0;
        un = wsc * sum_partials<T, NB>(red, pb, i) + C.pj[q] * C.pp[q];
        dnu[q] = lo + b;
      }
      du[q] = un;
      uv[q] = un;
      if (idx < NB * LDU) sUn[idx] = un;
    }
    __syncthreads();
    // x = A x_anc + B u + g
    if (!a.a_ident) {
      stream_partials<T, NB>(a.A, LDX, nx, nx, sXp, LDX, np, red);
      __syncthreads();
    }
    T xv[QX];
#pragma unroll
    for (int q = 0; q < QX; ++q) {
      const int idx = tid + q * kSegThreads;
      const int b = idx / LDX, i = idx - b * LDX;
      T xn = T(0);
      dnx[q] = -1;
      if (idx < NB * LDX && b < nb && i < nx) {
        const int pb = C.pax[q] >= 0 ? C.pax[q] - lo_p : 0;
        xn = a.a_ident ? sXp[pb * LDX + i] : sum_partials<T, NB>(red, pb, i);
        const int pe = sRow[i + 1];
        for (int p = sRow[i]; p < pe; ++p) xn += sVal[p] * sUn[b * LDU + sCol[p]];
        if (!power) xn += C.pg[q];
        dnx[q] = lo + b;
      }
      dxv[q] = xn;
      xv[q] = xn;
      if (idx < NB * LDX) sXn[idx] = xn;
    }

    // ---- prox / dual update ----
    if (power) {
#pragma unroll
      for (int q = 0; q < QX; ++q) {
        const int idx = tid + q * kSegThreads;
        const int b = idx / LDX, i = idx - b * LDX;
        dy1[q] = -xv[q];
        dy2[q] = -xv[q];
        if (idx < NB * LDX && b < nb && i < nx) zsq += 2.0 * (double)xv[q] * (double)xv[q];
      }
#pragma unroll
      for (int q = 0; q < QX; ++q) {
        const int idx = tid + q * kSegThreads;
        const int b = idx / LDU, i = idx - b * LDU;
        dy3[q] = -uv[q];
        if (idx < NB * LDU && b < nb && i < nu) zsq += (double)uv[q] * (double)uv[q];
      }
    } else {
      // block 3: box projection, elementwise
#pragma unroll
      for (int q = 0; q < QX; ++q) {
        const int idx = tid + q * kSegThreads;
        const int b = idx / LDU, i = idx - b * LDU;
        if (idx < NB * LDU && b < nb && i < nu) {
          const T w = w3c[q];
          const T v = w + gam * uv[q];
          const T y = v - gam * fmin(fmax(v / gam, bulo[q]), buhi[q]);
          dy3[q] = y;
          double d = fabs((double)y - (double)w) / gam64;
          if (!(d <= 1.0e308)) d = INFINITY;
          rmax = fmax(rmax, d);
        }
      }
      // blocks 1, 2: distance prox, needs the Euclidean norm of each node's block
      T r1v[QX], r2v[QX], w1v[QX], w2v[QX];
      double q1v[QX], q2v[QX];
#pragma unroll
      for (int q = 0; q < QX; ++q) {
        const int idx = tid + q * kSegThreads;
        const int b = idx / LDX, i = idx - b * LDX;
        const bool ok = idx < NB * LDX && b < nb && i < nx;
        const T w1 = w1c[q];
        const T w2 = w2c[q];
        const T v1 = w1 + gam * xv[q], v2 = w2 + gam * xv[q];
        const T rr1 = v1 - gam * fmin(fmax(v1 / gam, bxlo[q]), bxhi[q]);
        const T rr2 = v2 - gam * fmax(v2 / gam, bxs[q]);
        r1v[q] = ok ? rr1 : T(0);
        r2v[q] = ok ? rr2 : T(0);
        w1v[q] = w1;
        w2v[q] = w2;
        q1v[q] = (double)r1v[q] * (double)r1v[q];
        q2v[q] = (double)r2v[q] * (double)r2v[q];
      }
      double n1v[QX], n2v[QX];
      if (wave_norm) {
#pragma unroll
        for (int q = 0; q < QX; ++q) {
          n1v[q] = wave_sum(q1v[q]);
          n2v[q] = wave_sum(q2v[q]);
        }
      } else {
        __syncthreads();  // red is free: the x update has read it
        double* sq = reinterpret_cast<double*>(red);  // [2][NB][LDX]
#pragma unroll
        for (int q = 0; q < QX; ++q) {
          const int idx = tid + q * kSegThreads;
          if (idx < NB * LDX) {
            sq[idx] = q1v[q];
            sq[NB * LDX + idx] = q2v[q];
          }
        }
        __syncthreads();
        for (int st = a.LDXR / 2; st > 0; st >>= 1) {
          for (int idx = tid; idx < 2 * NB * st; idx += kSegThreads) {
            const int h = idx / (NB * st), rem = idx - h * NB * st;
            const int b = rem / st, i = rem - b * st;
            if (i + st < LDX)
              sq[h * NB * LDX + b * LDX + i] += sq[h * NB * LDX + b * LDX + i + st];
          }
          __syncthreads();
        }
#pragma unroll
        for (int q = 0; q < QX; ++q) {
          const int idx = tid + q * kSegThreads;
          const int b = min(idx / LDX, NB - 1);
          n1v[q] = sq[b * LDX];
          n2v[q] = sq[NB * LDX + b * LDX];
        }
      }
#pragma unroll
      for (int q = 0; q < QX; ++q) {
        const int idx = tid + q * kSegThreads;
        const int b = idx / LDX, i = idx - b * LDX;
        if (idx < NB * LDX && b < nb && i < nx) {
          const double n1 = sqrt(n1v[q]), n2 = sqrt(n2v[q]);
          const T sc1 = n1 > (double)a.Wx ? (T)((double)a.Wx / n1) : T(1);
          const T sc2 = n2 > (double)a.Ws ? (T)((double)a.Ws / n2) : T(1);
          const T y1 = r1v[q] * sc1, y2 = r2v[q] * sc2;
          dy1[q] = y1;
          dy2[q] = y2;
          double d1 = fabs((double)y1 - (double)w1v[q]) / gam64;
          double d2 = fabs((double)y2 - (double)w2v[q]) / gam64;
          if (!(d1 <= 1.0e308)) d1 = INFINITY;
          if (!(d2 <= 1.0e308)) d2 = INFINITY;
          rmax = fmax(rmax, fmax(d1, d2));
        }
      }
    }
    __syncthreads();
    // this stage's nodes are the next stage's parents
    T* t = sUp;
    sUp = sUn;
    sUn = t;
    t = sXp;
    sXp = sXn;
    sXn = t;
    lo_p = lo;
    np = nb;
  };
  while (true) {
    stage(s, PA, PB);
    if (++s > a.s_end) break;
    stage(s, PB, PA);
    if (++s > a.s_end) break;
  }
  flush();

  // ---- end of the launch: residual / power partials, end of iteration ----
  if (power) {
    const double tot = block_sum512(zsq, sred);
    if (tid == 0) a.part[a.part_base + blockIdx.x] = tot;
  } else {
    const double m = block_max512(rmax, sred);
    if (tid == 0) atomicMax(&ctl->res_bits, (unsigned long long)__double_as_longlong(m));
  }
  if (!a.last_level) return;
  __threadfence();
  if (tid == 0) {
    const unsigned prev = atomicAdd(&ctl->wg_done, 1u);
    s_last = prev == gridDim.x - 1;
  }
  __syncthreads();
  if (!s_last) return;
  __threadfence();
  if (power) {
    double acc = 0.0;
    for (int i = tid; i < a.part_total; i += kSegThreads) acc += a.part[i];
    const double tot = block_sum512(acc, sred);
    if (tid == 0) {
      const double L = sqrt(tot);
      ctl->L = L;
      ctl->pw_scale = L > 0.0 ? 1.0 / L : 0.0;
      ctl->iter = it + 1;
      ctl->wg_done = 0u;
    }
    return;
  }
  if (tid == 0) {
    DevCtl* c = ctl;
    const double res = __longlong_as_double((long long)atomicExch(&c->res_bits, 0ull));
    a.hist[it] = res;
    c->last_res = res;
    c->iter = it + 1;
    if (!(res < INFINITY)) {
      c->numeric = 1;
      c->done = 1;
    } else if (c->tol > 0.0 && res <= c->tol) {
      c->converged = 1;
      c->done = 1;
    } else if (it + 1 >= c->max_iter) {
      c->done = 1;
    }
    const double th = c->theta;
    const double t2 = th * th;
    const double thn = 0.5 * (sqrt(t2 * t2 + 4.0 * t2) - t2);
    c->theta_prev = th;
    c->theta = thn;
    c->beta = thn * (1.0 / th - 1.0);
    c->wg_done = 0u;
  }
}

// ---------------------------------------------------------------------------
template <typename T, int NB>
void launch_seg_nb(bool fwd, const SegArgs<T>& a, int n_wg, hipStream_t st) {
  const size_t lds = seg_lds_bytes<T, NB>(a);
  if (fwd)
    hipLaunchKernelGGL((seg_fwd_kernel<T, NB>), dim3(n_wg), dim3(kSegThreads), lds, st, a);
  else
    hipLaunchKernelGGL((seg_bwd_kernel<T, NB>), dim3(n_wg), dim3(kSegThreads), lds, st, a);
}

template <typename T>
void launch_seg(bool fwd, int nbm, const SegArgs<T>& a, int n_wg, hipStream_t st) {
  switch (nbm) {
    case 8: launch_seg_nb<T, 8>(fwd, a, n_wg, st); break;
    case 4: launch_seg_nb<T, 4>(fwd, a, n_wg, st); break;
    case 2: launch_seg_nb<T, 2>(fwd, a, n_wg, st); break;
    default: launch_seg_nb<T, 1>(fwd, a, n_wg, st); break;
  }
}

template <typename T>
size_t seg_lds(int nbm, const SegArgs<T>& a) {
  switch (nbm) {
    case 8: return seg_lds_bytes<T, 8>(a);
    case 4: return seg_lds_bytes<T, 4>(a);
    case 2: return seg_lds_bytes<T, 2>(a);
    default: return seg_lds_bytes<T, 1>(a);
  }
}

template void launch_seg<double>(bool, int, const SegArgs<double>&, int, hipStream_t);
template void launch_seg<float>(bool, int, const SegArgs<float>&, int, hipStream_t);
template size_t seg_lds<double>(int, const SegArgs<double>&);
template size_t seg_lds<float>(int, const SegArgs<float>&);

}  // namespace tapg
