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
#include "seg_device.h"

namespace tapg {

namespace {

constexpr int kRT = 128;   // rows per slice of a register-resident GEMV
constexpr int kKS = kSegThreads / kRT;
constexpr int kKC = 32;    // columns per slice
constexpr int kLDU = 128;  // padded u-dimension of the segment layout

// m[j] = Fbar_s(r, kb + j); the padded stage block makes all 32 loads valid
// and unconditional, so they issue back to back.
template <typename T>
__device__ __forceinline__ void load_factor(const T* __restrict__ F, int r, int kb,
                                            T (&m)[kKC]) {
  const T* base = F + (size_t)kb * kLDU + r;
#pragma unroll
  for (int j = 0; j < kKC; ++j) m[j] = base[j * kLDU];
}

// Four consecutive elements of an LDS vector (one 16-byte read for FP32, two
// for FP64); p is 4-element aligned.
__device__ __forceinline__ void ld4(const double* p, double (&v)[4]) {
  const double2 a = *reinterpret_cast<const double2*>(p);
  const double2 b = *reinterpret_cast<const double2*>(p + 2);
  v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
}
__device__ __forceinline__ void ld4(const float* p, float (&v)[4]) {
  const float4 a = *reinterpret_cast<const float4*>(p);
  v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
}

// Register-resident GEMV slice: red[(ks*NB + b)*128 + r] = sum_{j<32} m[j] X[b*128 + kb + j]
// for the columns b < ncols.  NC columns run together with four partial sums
// each, so the FMAs do not form one dependent chain, and every lane of a wave
// reads the same X addresses (kb is wave-uniform), 4 elements at a time.
template <typename T, int NB, int NC>
__device__ __forceinline__ void gemv_cols(const T (&m)[kKC], const T* X, int kb, int ks, int r,
                                          int ncols, T* red) {
  static_assert(NC == 1 || NC == 2, "one or two columns at a time");
#pragma unroll
  for (int b0 = 0; b0 < NB; b0 += NC) {
    if (b0 < ncols) {
      T acc[NC][4];
#pragma unroll
      for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[c][q] = T(0);
#pragma unroll
      for (int j = 0; j < kKC; j += 4) {
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          T v[4];
          ld4(X + (b0 + c) * kLDU + kb + j, v);
#pragma unroll
          for (int q = 0; q < 4; ++q) acc[c][q] += m[j + q] * v[q];
        }
      }
#pragma unroll
      for (int c = 0; c < NC; ++c)
        if (b0 + c < ncols)
          red[(ks * NB + b0 + c) * kRT + r] = (acc[c][0] + acc[c][1]) + (acc[c][2] + acc[c][3]);
    }
  }
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
  if (a.proj)  // CSR of G and of E', each with a padding int
    b += (size_t)(a.ns + 2 + a.nnzG + a.nu + 2 + a.nnzE) * sizeof(int) +
         (size_t)(a.nnzG + a.nnzE) * sizeof(T) + 16;
  return (b + 15) & ~(size_t)15;
}

// ---------------------------------------------------------------------------
// Backward sweep over one level, stages s_end down to s_begin.  Per node:
//   lambda_n = a_n + A' sum_{c} lambda_c                 (a_n = w1_n + w2_n)
//   v_n      = -(w3_n + B' lambda_n)/2 + W_u sum_{c} j_c
//   j_n      = kappa_n + Fbar_s v_n
// ---------------------------------------------------------------------------
// Backward sweep of one workgroup `wg` of a level in iteration `it` (its
// extrapolation weight beta; scale: 1/|v| in the power iteration).
template <typename T, int NB, bool PROJ>
__device__ __forceinline__ void seg_bwd_body(const SegArgs<T>& a, int wg, int it, T beta,
                                             T scale) {
  constexpr int QX = NB * 128 / kSegThreads > 0 ? NB * 128 / kSegThreads : 1;
  const int tid = threadIdx.x;
  const bool power = a.mode == 1;
  const T* Yc = (it & 1) ? a.Y1 : a.Y0;
  const T* Yo = (it & 1) ? a.Y0 : a.Y1;
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
  int* gRow = reinterpret_cast<int*>(sVal + a.nnzB);  // projector path: CSR of G, then of E'
  int* gCol = gRow + a.ns + 1;
  T* gVal = reinterpret_cast<T*>(gCol + a.nnzG + ((a.ns + 1 + a.nnzG) & 1));
  int* eRow = reinterpret_cast<int*>(gVal + a.nnzG);
  int* eCol = eRow + nu + 1;
  T* eVal = reinterpret_cast<T*>(eCol + a.nnzE + ((nu + 1 + a.nnzE) & 1));
  {
    const int2* rg = a.ranges + (size_t)wg * a.nst;
    for (int i = tid; i < a.nst; i += kSegThreads) {
      sRg[i] = rg[i];
      sFid[i] = a.fid[a.s_begin + i];
    }
    csr_to_lds<T>(a.Btrow, a.Btcol, a.Btval, nu, a.nnzB, sRow, sCol, sVal);
    if constexpr (PROJ) {
      csr_to_lds<T>(a.Grow, a.Gcol, a.Gval, a.ns, a.nnzG, gRow, gCol, gVal);
      csr_to_lds<T>(a.Etrow, a.Etcol, a.Etval, nu, a.nnzE, eRow, eCol, eVal);
    }
    __syncthreads();
  }
  // this thread's rows of B' (one per u-slot)
  RegRow<T, 2> brow[QX];
#pragma unroll
  for (int q = 0; q < QX; ++q) {
    const int i = (tid + q * kSegThreads) % LDU;
    brow[q].load(sRow, sCol, sVal, i, i < nu);
  }
  // projector path: row tid % ns of G for the node column tid / ns, rows of E'
  const int ns = a.ns;
  RegRow<T, 4> grow;
  RegRow<T, 2> erow[QX];
  if constexpr (PROJ) {
    grow.load(gRow, gCol, gVal, ns > 0 ? tid % ns : 0, ns > 0 && tid < NB * ns);
#pragma unroll
    for (int q = 0; q < QX; ++q) {
      const int i = (tid + q * kSegThreads) % LDU;
      erow[q].load(eRow, eCol, eVal, i, i < nu);
    }
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
  if constexpr (!PROJ) load_factor<T>(a.F + (size_t)f_cur * kLDU * kLDU, r, kb, mreg);
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
    const int2 kc = a.wgx[2 * wg];
    lo_c = kc.x;
    const int nc = kc.y - lo_c;
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
    T aval[QX], w3v[QX], kap[QX], lsum[QX];
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
      w3v[q] = power ? scale * C.pu[q][0] : wext(C.pu[q][0], C.pu[q][1], beta);
      kap[q] = power ? T(0) : C.pu[q][2];
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
      if (ok) e = brow[q].apply(e, sLn + b * LDX, sCol, sVal);
      // children's j, summed here (after the barrier above) so that the
      // previous stage needs no closing barrier for its writes to sJ
      T sg = T(0);
      if (ok && kids) {
        for (int c = C.cu[q][0]; c < C.cu[q][1]; ++c) sg += sJ[(c - lo_c) * LDU + i];
      }
      vv[q] = ok ? T(-0.5) * e + (a.wu_scalar ? a.wu * sg : T(0)) : T(0);
      if (idx < NB * LDU) sV[idx] = a.wu_scalar ? vv[q] : sg;
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
    // j = kappa + Fbar_s v: register-resident Fbar_s, or the projector form
    // (v - E'(G v)) / w whose G v goes through red
    if constexpr (PROJ) {
      if (tid < nb * ns) red[tid] = grow.apply(T(0), sV + (tid / ns) * kLDU, gCol, gVal);
    } else {
      gemv_cols<T, NB, (NB >= 2 && sizeof(T) == 4 ? 2 : 1)>(mreg, sV, kb, ks, r, nb, red);
      if (s > a.s_begin) {
        const int fn = __builtin_amdgcn_readfirstlane(sFid[s - 1 - a.s_begin]);
        if (fn != f_cur) {
          f_cur = fn;
          load_factor<T>(a.F + (size_t)fn * kLDU * kLDU, r, kb, mreg);
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < QX; ++q) {
      const int idx = tid + q * kSegThreads;
      const int b = idx / LDU, i = idx - b * LDU;
      dn[q] = -1;
      if (idx < NB * LDU && b < nb && i < nu) {
        T jn;
        if constexpr (PROJ)
          jn = kap[q] + a.winv * (sV[b * kLDU + i] - erow[q].apply(T(0), red + b * ns, eCol, eVal));
        else
          jn = kap[q] + sum_partials<T, NB>(red, b, i);
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
    // No closing barrier: the next stage writes sLn (this stage's sLc, read
    // before this stage's first barrier), sV and red only after barriers of
    // its own that every wave reaches after finishing this stage, and reads
    // this stage's sJ only after its first barrier.
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

template <typename T, int NB, bool PROJ>
__global__ __launch_bounds__(kSegThreads) void seg_bwd_kernel(SegArgs<T> a) {
  const int tree = a.wgtree ? a.wgtree[blockIdx.x] : 0;  // a workgroup never spans two trees
  const DevCtl c = bwd_ctl(a, tree, (int)blockIdx.x);
  if (c.done) return;
  seg_bwd_body<T, NB, PROJ>(a, blockIdx.x, c.iter, (T)c.beta, (T)c.pw_scale);
}

// ---------------------------------------------------------------------------
// Forward sweep over one level, stages s_begin up to s_end, with the fused
// prox / dual update.  Per node:
//   u_n = Fbar_s (W_u u_anc) + j_n / p_n       (= Kbar_s u_anc + k_n)
//   x_n = A x_anc + B u_n + g_n
//   v = w + gamma (x_n, x_n, u_n);  blocks 1, 2: r = v - gamma P_C(v/gamma),
//   y+ = r min(1, W / |r|);  block 3: y+ = v - gamma P_U(v/gamma)
// The product Fbar_s (W_u u_anc) is formed once per parent.  The workgroups
// leave their residual maxima in the tree's control block; the next
// iteration's first backward launch (or a small launch after a run of
// iterations) ends the iteration.
// ---------------------------------------------------------------------------
// Forward sweep of workgroup `wg` of a level (tree `tree`) in iteration `it`
// with the fused prox / dual update.  Returns the workgroup's residual max
// max |y+ - w| / gamma (power iteration: the sum of squares of its part of the
// new iterate); sred is scratch for the workgroup reduction.
template <typename T, int NB, bool PROJ>
__device__ __forceinline__ double seg_fwd_body(const SegArgs<T>& a, int wg, int tree, int it,
                                               T beta, double gam64, double* sred) {
  constexpr int QX = NB * 128 / kSegThreads > 0 ? NB * 128 / kSegThreads : 1;
  const int tid = threadIdx.x;
  const bool power = a.mode == 1;
  const T* Yc = (it & 1) ? a.Y1 : a.Y0;
  T* Yn = (it & 1) ? a.Y0 : a.Y1;  // y^{nu-1} in, y^{nu+1} out
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
  int* gRow = reinterpret_cast<int*>(sVal + a.nnzB);  // projector path: CSR of G, then of E'
  int* gCol = gRow + a.ns + 1;
  T* gVal = reinterpret_cast<T*>(gCol + a.nnzG + ((a.ns + 1 + a.nnzG) & 1));
  int* eRow = reinterpret_cast<int*>(gVal + a.nnzG);
  int* eCol = eRow + nu + 1;
  T* eVal = reinterpret_cast<T*>(eCol + a.nnzE + ((nu + 1 + a.nnzE) & 1));
  {
    const int2* rg = a.ranges + (size_t)wg * a.nst;
    for (int i = tid; i < a.nst; i += kSegThreads) {
      sRg[i] = rg[i];
      sFid[i] = a.fid[a.s_begin + i];
    }
    csr_to_lds<T>(a.Brow, a.Bcol, a.Bval, nx, a.nnzB, sRow, sCol, sVal);
    if constexpr (PROJ) {
      csr_to_lds<T>(a.Grow, a.Gcol, a.Gval, a.ns, a.nnzG, gRow, gCol, gVal);
      csr_to_lds<T>(a.Etrow, a.Etcol, a.Etval, nu, a.nnzE, eRow, eCol, eVal);
    }
  }

  const int r = tid % kRT;
  const int ks = __builtin_amdgcn_readfirstlane(tid / kRT);
  const int kb = ks * kKC;
  // Stage-invariant bounds of this thread's slots, scaled by gamma: for a box
  // C, gamma P_C(v / gamma) = P_{gamma C}(v), so the prox needs no division
  // (and a component inside the box leaves r = v - v = 0 exactly).
  // Kept in LDS (registers are scarce here): [xmin | xmax | xs] by x-slot,
  // [umin | umax] by u-slot, 128 entries each (nx, nu <= 128 on this path).
  // With FP32 sweeps the bounds are kept unscaled and the prox runs in FP64
  // (bnd() scales them there).
  __shared__ T sBnd[5 * kRT];
  const T bscale = sizeof(T) == sizeof(double) ? gam : T(1);
  for (int i = tid; i < kRT; i += kSegThreads) {
    sBnd[i] = bscale * ldm(a.xmin, i, i < nx);
    sBnd[kRT + i] = bscale * ldm(a.xmax, i, i < nx);
    sBnd[2 * kRT + i] = bscale * ldm(a.xs, i, i < nx);
    sBnd[3 * kRT + i] = bscale * ldm(a.umin, i, i < nu);
    sBnd[4 * kRT + i] = bscale * ldm(a.umax, i, i < nu);
  }
  auto bnd = [&](int i) -> double {
    return sizeof(T) == sizeof(double) ? (double)sBnd[i] : gam64 * (double)sBnd[i];
  };
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
  __syncthreads();  // sRg, sFid, CSR ready
  // this thread's rows of B (one per x-slot)
  RegRow<T, 3> brow[QX];
#pragma unroll
  for (int q = 0; q < QX; ++q) {
    const int i = (tid + q * kSegThreads) % LDX;
    brow[q].load(sRow, sCol, sVal, i, i < nx);
  }
  // projector path: row tid % ns of G for the parent column tid / ns, rows of E'
  const int ns = a.ns;
  RegRow<T, 4> grow;
  RegRow<T, 2> erow[QX];
  if constexpr (PROJ) {
    grow.load(gRow, gCol, gVal, ns > 0 ? tid % ns : 0, ns > 0 && tid < NB * ns);
#pragma unroll
    for (int q = 0; q < QX; ++q) {
      const int i = (tid + q * kSegThreads) % LDU;
      erow[q].load(eRow, eCol, eVal, i, i < nu);
    }
  }
  int f_cur = __builtin_amdgcn_readfirstlane(sFid[0]);
  if constexpr (!PROJ) load_factor<T>(a.F + (size_t)f_cur * kLDU * kLDU, r, kb, mreg);
  load_stage(s, PA);
  T* sUp = sU0;  // parents (stage s-1)
  T* sUn = sU1;
  T* sXp = sX0;
  T* sXn = sX1;
  int lo_p = 0, np = 0;
  {  // parents of the first stage come from global memory (or p, q at the root)
    const int2 pp = a.wgx[2 * wg + 1];
    const int par0 = pp.x;
    lo_p = par0 >= 0 ? par0 : 0;
    np = par0 >= 0 ? pp.y - par0 + 1 : 1;
    for (int idx = tid; idx < NB * LDU; idx += kSegThreads) {
      const int b = idx / LDU, i = idx - b * LDU;
      T v = T(0);
      if (b < np && i < nu)
        v = par0 >= 0 ? a.u[(size_t)(lo_p + b) * LDU + i]
                      : (power ? T(0) : a.pq[(size_t)tree * a.pq_stride + LDX + i]);
      sUp[idx] = v;
    }
    for (int idx = tid; idx < NB * LDX; idx += kSegThreads) {
      const int b = idx / LDX, i = idx - b * LDX;
      T v = T(0);
      if (b < np && i < nx)
        v = par0 >= 0 ? a.x[(size_t)(lo_p + b) * LDX + i]
                      : (power ? T(0) : a.pq[(size_t)tree * a.pq_stride + i]);
      sXp[idx] = v;
    }
  }
  __syncthreads();  // the first stage's parents are in LDS
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
    // (the parents in sUp / sXp were written before the previous barrier)
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
    if constexpr (PROJ) {
      // projector form (W_u = w I): Kbar_s u_anc = u_anc - E'(G u_anc); G u_anc via red
      if (tid < np * ns) red[tid] = grow.apply(T(0), V + (tid / ns) * kLDU, gCol, gVal);
    } else {
      // Fbar_s (W_u u_anc), one column per parent
      // (one column at a time in FP64: the forward kernel's registers are scarce)
      gemv_cols<T, NB, (NB >= 2 && NB <= 4 && sizeof(T) == 4 ? 2 : 1)>(mreg, V, kb, ks, r, np, red);
      // this stage's factor is consumed: load the next stage's into the same
      // registers if it is another block
      if (s < a.s_end) {
        const int fn = __builtin_amdgcn_readfirstlane(sFid[s + 1 - a.s_begin]);
        if (fn != f_cur) {
          f_cur = fn;
          load_factor<T>(a.F + (size_t)fn * kLDU * kLDU, r, kb, mreg);
        }
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
        if constexpr (PROJ)
          un = (V[pb * kLDU + i] - erow[q].apply(T(0), red + pb * ns, eCol, eVal)) +
               C.pj[q] * C.pp[q];
        else
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
        xn = brow[q].apply(xn, sUn + b * LDU, sCol, sVal);
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
      // The prox and the residual in FP64 whatever T (FP32 sweeps: w and x
      // widened, y+ rounded to T once, |y+ - w| / gamma the FP64 residual).
      // block 3: box projection, elementwise
#pragma unroll
      for (int q = 0; q < QX; ++q) {
        const int idx = tid + q * kSegThreads;
        const int b = idx / LDU, i = idx - b * LDU;
        if (idx < NB * LDU && b < nb && i < nu) {
          const double w = (double)w3c[q];
          const double v = w + gam64 * (double)uv[q];
          const double y = v - fmin(fmax(v, bnd(3 * kRT + i)), bnd(4 * kRT + i));
          dy3[q] = (T)y;
          double d = fabs(y - w);
          if (!(d <= 1.0e308)) d = INFINITY;
          rmax = fmax(rmax, d);
        }
      }
      // blocks 1, 2: distance prox, needs the Euclidean norm of each node's block
      double r1v[QX], r2v[QX];
      T w1v[QX], w2v[QX];
      double q1v[QX], q2v[QX];
#pragma unroll
      for (int q = 0; q < QX; ++q) {
        const int idx = tid + q * kSegThreads;
        const int b = idx / LDX, i = idx - b * LDX;
        const bool ok = idx < NB * LDX && b < nb && i < nx;
        const T w1 = w1c[q];
        const T w2 = w2c[q];
        const double v1 = (double)w1 + gam64 * (double)xv[q];
        const double v2 = (double)w2 + gam64 * (double)xv[q];
        const double rr1 = v1 - fmin(fmax(v1, bnd(i)), bnd(kRT + i));
        const double rr2 = v2 - fmax(v2, bnd(2 * kRT + i));
        r1v[q] = ok ? rr1 : 0.0;
        r2v[q] = ok ? rr2 : 0.0;
        w1v[q] = w1;
        w2v[q] = w2;
        q1v[q] = r1v[q] * r1v[q];
        q2v[q] = r2v[q] * r2v[q];
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
          const double sc1 = n1 > (double)a.Wx ? (double)a.Wx / n1 : 1.0;
          const double sc2 = n2 > (double)a.Ws ? (double)a.Ws / n2 : 1.0;
          const double y1 = r1v[q] * sc1, y2 = r2v[q] * sc2;
          dy1[q] = (T)y1;
          dy2[q] = (T)y2;
          double d1 = fabs(y1 - (double)w1v[q]);
          double d2 = fabs(y2 - (double)w2v[q]);
          if (!(d1 <= 1.0e308)) d1 = INFINITY;
          if (!(d2 <= 1.0e308)) d2 = INFINITY;
          rmax = fmax(rmax, fmax(d1, d2));
        }
      }
    }
    // Closing barrier only for the LDS norm reduction, which used red as
    // scratch; otherwise the next stage reads sUn / sXn (written before the
    // barrier after u) and writes sUp, sXp and red only after barriers every
    // wave reaches after finishing this stage.
    if (!wave_norm) __syncthreads();
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
  if (power) return block_sum512(zsq, sred);
  // max |y+ - w| / gamma: the division by gamma > 0 is monotone, so dividing
  // the workgroup's max once gives the max of the quotients exactly
  return block_max512(rmax, sred) / gam64;
}

template <typename T, int NB, bool PROJ>
__global__ __launch_bounds__(kSegThreads) void seg_fwd_kernel(SegArgs<T> a) {
  const int tree = a.wgtree ? a.wgtree[blockIdx.x] : 0;  // a workgroup never spans two trees
  DevCtl* ctl = a.ctl + tree;
  __shared__ double sred[kSegThreads];
  if (ctl->done) return;  // this tree has stopped
  const double m = seg_fwd_body<T, NB, PROJ>(a, blockIdx.x, tree, ctl->iter, (T)ctl->beta,
                                             ctl->gamma, sred);
  if (threadIdx.x == 0) {
    if (a.mode == 1)
      a.part[a.part_base + blockIdx.x] = m;
    else
      atomicMax(&ctl->res_bits, (unsigned long long)__double_as_longlong(m));
  }
}

// ---------------------------------------------------------------------------
// Persistent iteration (one tree).
// ---------------------------------------------------------------------------
namespace {

// A hand-over wait is declared stuck after 2 s of the 100 MHz real-time
// counter (an iteration takes well under a millisecond).
constexpr unsigned long long kChainWaitTicks = 200000000ull;

// Thread 0 waits until *p >= target (acquire at device scope; the acquire also
// drops this CU's stale cache lines before the workgroup reads the producer's
// data).  Returns false when the solve was stopped or the wait hit its bound
// (then the error flag and the stop flag are set).
__device__ bool chain_wait(unsigned* p, unsigned target, ChainSync* sync, int* s_flag) {
  if (threadIdx.x == 0) {
    int ok = 1;
    const unsigned long long t0 = __builtin_amdgcn_s_memrealtime();
    while (true) {
      if (__hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) >= target) break;
      if (__hip_atomic_load(&sync->stop, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT)) {
        ok = 0;
        break;
      }
      if (__builtin_amdgcn_s_memrealtime() - t0 > kChainWaitTicks) {
        __hip_atomic_store(&sync->error, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&sync->stop, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    *s_flag = ok;
  }
  __syncthreads();
  return *s_flag != 0;
}

}  // namespace

template <typename T, int NB, bool PROJ>
__global__ __launch_bounds__(kSegThreads) void seg_chain_kernel(ChainArgs<T> c) {
  __shared__ double sred[kSegThreads];
  __shared__ int s_flag;
  const int g = blockIdx.x;
  int l = 0;
  while (l + 1 < c.nlev && g >= c.base[l + 1]) ++l;
  const int wg = g - c.base[l];
  const SegArgs<T>& a = c.lev[l];  // fields read on demand (scalar loads)
  DevCtl* ctl = c.ctl;
  ChainSync* sync = c.sync;
  const int2 par = c.parents[g];  // parent workgroups [par.x, par.y] (par.x < 0: top level)
  const unsigned need = (unsigned)c.nchild[g];
  int it = ctl->iter;
  const int rule = ctl->rule;
  double theta = ctl->theta, theta_prev = ctl->theta_prev, beta = ctl->beta;
  const double gam64 = ctl->gamma;
  // the top workgroup ends iteration `prev` once all forward sweeps of it are in
  auto end_iteration = [&](int prev, unsigned all_target) -> bool {
    if (!chain_wait(&sync->fwd_all, all_target, sync, &s_flag)) return false;
    if (threadIdx.x == 0) {
      const double res = __longlong_as_double(
          (long long)__hip_atomic_exchange(&sync->res[prev & 1], 0ull, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT));
      c.hist[prev] = res;
      ctl->last_res = res;
      ctl->iter = prev + 1;
      if (!(res < INFINITY)) {
        ctl->numeric = 1;
        ctl->done = 1;
      } else if (ctl->tol > 0.0 && res <= ctl->tol) {
        ctl->converged = 1;
        ctl->done = 1;
      } else if (prev + 1 >= ctl->max_iter) {
        ctl->done = 1;
      }
      double th = ctl->theta, thp = ctl->theta_prev, be = ctl->beta;
      theta_update(rule, prev + 1, th, thp, be);
      ctl->theta = th;
      ctl->theta_prev = thp;
      ctl->beta = be;
      s_flag = ctl->done;
      if (ctl->done) __hip_atomic_store(&sync->stop, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    return s_flag == 0;
  };
  int k = 0;
  for (; k < c.iters; ++k) {
    // backward sweep, after the child workgroups' backward sweeps of this iteration
    if (need > 0 && !chain_wait(&c.bwd_cnt[g], need * (unsigned)(k + 1), sync, &s_flag)) break;
    seg_bwd_body<T, NB, PROJ>(a, wg, it, (T)beta, T(1));
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0)
      for (int p = par.x; p >= 0 && p <= par.y; ++p)
        __hip_atomic_fetch_add(&c.bwd_cnt[p], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    // forward sweep: the top workgroup first ends the previous iteration
    if (l == 0) {
      if (k > 0 && !end_iteration(it - 1, (unsigned)c.total * (unsigned)k)) break;
    } else {
      bool ok = true;
      for (int p = par.x; ok && p <= par.y; ++p)
        ok = chain_wait(&c.fwd_flag[p], (unsigned)(k + 1), sync, &s_flag);
      if (!ok) break;
    }
    const double m = seg_fwd_body<T, NB, PROJ>(a, wg, 0, it, (T)beta, gam64, sred);
    if (threadIdx.x == 0)
      __hip_atomic_fetch_max(&sync->res[it & 1], (unsigned long long)__double_as_longlong(m),
                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
      __hip_atomic_store(&c.fwd_flag[g], (unsigned)(k + 1), __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_fetch_add(&sync->fwd_all, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
    ++it;
    theta_update(rule, it, theta, theta_prev, beta);
  }
  // the last iteration of the launch ends here (unless the solve stopped)
  if (l == 0 && k == c.iters) end_iteration(it - 1, (unsigned)c.total * (unsigned)c.iters);
}

// ---------------------------------------------------------------------------
template <typename T, int NB>
void launch_seg_nb(bool fwd, const SegArgs<T>& a, int n_wg, hipStream_t st) {
  const size_t lds = seg_lds_bytes<T, NB>(a);
  if (a.proj) {
    if (fwd)
      hipLaunchKernelGGL((seg_fwd_kernel<T, NB, true>), dim3(n_wg), dim3(kSegThreads), lds, st, a);
    else
      hipLaunchKernelGGL((seg_bwd_kernel<T, NB, true>), dim3(n_wg), dim3(kSegThreads), lds, st, a);
  } else {
    if (fwd)
      hipLaunchKernelGGL((seg_fwd_kernel<T, NB, false>), dim3(n_wg), dim3(kSegThreads), lds, st, a);
    else
      hipLaunchKernelGGL((seg_bwd_kernel<T, NB, false>), dim3(n_wg), dim3(kSegThreads), lds, st, a);
  }
}

template <typename T>
void launch_seg(bool fwd, int nbm, const SegArgs<T>& a, int n_wg, hipStream_t st) {
  if (a.scan) {
    launch_scan<T>(fwd, nbm, a, n_wg, st);
    return;
  }
  switch (nbm) {
    case 4: launch_seg_nb<T, 4>(fwd, a, n_wg, st); break;
    case 2: launch_seg_nb<T, 2>(fwd, a, n_wg, st); break;
    case 1: launch_seg_nb<T, 1>(fwd, a, n_wg, st); break;
    default: throw Fail{TAPG_EINVAL, "segment sweep: unsupported nodes per stage " + std::to_string(nbm)};
  }
}

template <typename T>
size_t seg_lds(int nbm, const SegArgs<T>& a) {
  if (a.scan) return scan_lds<T>(nbm, a);
  switch (nbm) {
    case 4: return seg_lds_bytes<T, 4>(a);
    case 2: return seg_lds_bytes<T, 2>(a);
    case 1: return seg_lds_bytes<T, 1>(a);
    default: throw Fail{TAPG_EINVAL, "segment sweep: unsupported nodes per stage " + std::to_string(nbm)};
  }
}

template <typename T, int NB, bool PROJ>
hipError_t launch_chain_nb(const ChainArgs<T>& c, size_t lds, hipStream_t st) {
  void* args[] = {const_cast<ChainArgs<T>*>(&c)};
  return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&seg_chain_kernel<T, NB, PROJ>),
                                    dim3(c.total), dim3(kSegThreads), args, lds, st);
}

template <typename T>
hipError_t launch_chain(int nbm, bool proj, const ChainArgs<T>& c, size_t lds, hipStream_t st) {
  switch (nbm) {
    case 4: return proj ? launch_chain_nb<T, 4, true>(c, lds, st) : launch_chain_nb<T, 4, false>(c, lds, st);
    case 2: return proj ? launch_chain_nb<T, 2, true>(c, lds, st) : launch_chain_nb<T, 2, false>(c, lds, st);
    case 1: return proj ? launch_chain_nb<T, 1, true>(c, lds, st) : launch_chain_nb<T, 1, false>(c, lds, st);
    default: return hipErrorInvalidValue;
  }
}

template <typename T, int NB, bool PROJ>
int chain_occ(size_t lds) {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &nb, reinterpret_cast<const void*>(&seg_chain_kernel<T, NB, PROJ>), kSegThreads, lds) !=
      hipSuccess)
    return 0;
  return nb;
}

template <typename T>
int chain_blocks_per_cu(int nbm, bool proj, size_t lds) {
  switch (nbm) {
    case 4: return proj ? chain_occ<T, 4, true>(lds) : chain_occ<T, 4, false>(lds);
    case 2: return proj ? chain_occ<T, 2, true>(lds) : chain_occ<T, 2, false>(lds);
    case 1: return proj ? chain_occ<T, 1, true>(lds) : chain_occ<T, 1, false>(lds);
    default: return 0;
  }
}

template hipError_t launch_chain<double>(int, bool, const ChainArgs<double>&, size_t, hipStream_t);
template hipError_t launch_chain<float>(int, bool, const ChainArgs<float>&, size_t, hipStream_t);
template int chain_blocks_per_cu<double>(int, bool, size_t);
template int chain_blocks_per_cu<float>(int, bool, size_t);
template void launch_seg<double>(bool, int, const SegArgs<double>&, int, hipStream_t);
template void launch_seg<float>(bool, int, const SegArgs<float>&, int, hipStream_t);
template size_t seg_lds<double>(int, const SegArgs<double>&);
template size_t seg_lds<float>(int, const SegArgs<float>&);

}  // namespace tapg
