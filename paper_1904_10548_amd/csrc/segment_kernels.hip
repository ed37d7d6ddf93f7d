// Segment sweep kernels for gfx950.
//
// The tree is cut into levels of consecutive stages.  In a level, workgroup w
// owns a group of consecutive nodes at the level's first stage and all their
// descendants down to the level's last stage; by the breadth-first numbering
// these are one contiguous node range per stage (ranges[w][s - s_begin]).  A
// workgroup therefore walks all stages of its level without any grid-wide
// synchronisation: children (backward) and parents (forward) of its nodes are
// its own nodes of the neighbouring stage, kept in LDS.  Only the level
// boundaries go through global memory, between launches.
//
// Per stage, the stage factor Fbar_s (nu x nu, nu <= 128) is held in
// registers: thread t owns row r = t % 128 and the k-slice t / 128 (4 slices
// of ceil(nu/4) <= 32 columns).  While stage s is computed, the loads of the
// next stage's factor and of its node inputs are already in flight, so the
// walk down a chain of stages is not a chain of memory round trips.
//
// Structure used: W_u = w I gives Kbar_s = w Fbar_s, so one matrix per stage
// serves both sweeps (general W_u: Kbar_s v = Fbar_s (W_u v), W_u streamed);
// A = I skips the A products (general A: streamed); B and B' are applied as
// CSR (the flow-network incidence has one or two entries per column).
#include <cmath>

#include "kernels.h"

namespace tapg {

namespace {

constexpr int kRT = 128;  // rows per slice of a register-resident GEMV
constexpr int kKS = kSegThreads / kRT;
constexpr int kKC = 32;   // columns per slice
constexpr int kLDU = 128; // padded u-dimension of the segment layout

template <typename T>
__device__ __forceinline__ T wext(T y, T yp, T beta) {
  return y + beta * (y - yp);
}

// Register-resident block of Fbar_s: m[j] = Fbar_s(r, kb + j).  The segment
// layout pads the u-dimension to 128 (LDU = 128, zero rows/columns beyond
// nu), so every address is inside the stage block and all 32 loads issue
// back to back without conditions.
template <typename T>
__device__ __forceinline__ void load_factor(const T* __restrict__ F, int r, int kb,
                                            T (&m)[kKC]) {
  const T* base = F + (size_t)kb * kLDU + r;
#pragma unroll
  for (int j = 0; j < kKC; ++j) m[j] = base[j * kLDU];
}

// Unconditional load from a clamped index, masked afterwards.
template <typename T>
__device__ __forceinline__ T ldm(const T* __restrict__ p, size_t idx, bool ok) {
  const T v = p[ok ? idx : 0];
  return ok ? v : T(0);
}

// Streamed GEMV partials for a general matrix (A, A' or W_u): thread (r, ks)
// writes red[(ks * NB + b) * 128 + r] = sum_{k in slice} M(r, k) X[b][k].
// Used only when A != I or W_u is not a multiple of I.
template <typename T, int NB>
__device__ __noinline__ void stream_partials(const T* __restrict__ M, int ldm, int R, int K,
                                             const T* X, int ldx, int ncols, T* red) {
  const int r = threadIdx.x % kRT;
  const int ks = __builtin_amdgcn_readfirstlane(threadIdx.x / kRT);
  const int kc = (K + kKS - 1) / kKS;
  const int kb = ks * kc, ke = min(K, kb + kc);
  for (int b = 0; b < ncols && b < NB; ++b) {
    T acc = T(0);
    if (r < R) {
#pragma unroll 8
      for (int k = kb; k < ke; ++k) acc += M[(size_t)k * ldm + r] * X[b * ldx + k];
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

}  // namespace

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
  const int2* rg = a.ranges + (size_t)blockIdx.x * a.nst;

  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* sL0 = reinterpret_cast<T*>(smem_raw);  // lambda ping-pong
  T* sL1 = sL0 + NB * LDX;
  T* sJ = sL1 + NB * LDX;                   // children's j, then this stage's j
  T* sV = sJ + NB * LDU;                    // GEMV input
  T* red = sV + NB * LDU;                   // 4 * NB * 128 partials

  const int r = tid % kRT;
  const int ks = __builtin_amdgcn_readfirstlane(tid / kRT);  // wave-uniform slice
  const int kb = ks * kKC;

  // prefetch registers: x-slots (y1, y1o, y2, y2o), u-slots (y3, y3o, kappa)
  T px[QX][4], pu[QX][3];
  T mreg[kKC], mnext[kKC];

  auto load_nodes = [&](int s) {
    const int2 rr = rg[s - a.s_begin];
    const int lo = rr.x, nb = rr.y - rr.x;
#pragma unroll
    for (int q = 0; q < QX; ++q) {
      const int idx = tid + q * kSegThreads;
      const int b = idx / LDX, i = idx - b * LDX;
      const bool ok = idx < NB * LDX && b < nb && i < nx;
      const size_t o = (size_t)(lo + b) * LDY + i;
      px[q][0] = ldm(Yc, o, ok);
      px[q][1] = ldm(Yo, o, ok && !power);
      px[q][2] = ldm(Yc, o + LDX, ok);
      px[q][3] = ldm(Yo, o + LDX, ok && !power);
    }
#pragma unroll
    for (int q = 0; q < QX; ++q) {
      const int idx = tid + q * kSegThreads;
      const int b = idx / LDU, i = idx - b * LDU;
      const bool ok = idx < NB * LDU && b < nb && i < nu;
      const size_t n = (size_t)(lo + b);
      pu[q][0] = ldm(Yc, n * LDY + 2 * LDX + i, ok);
      pu[q][1] = ldm(Yo, n * LDY + 2 * LDX + i, ok && !power);
      pu[q][2] = ldm(a.kappa, n * LDU + i, ok && !power);
    }
  };

  int s = a.s_end;
  load_factor<T>(a.F + (size_t)s * kLDU * kLDU, r, kb, mreg);
  load_nodes(s);
  T* sLc = sL0;  // children's lambda (stage s+1)
  T* sLn = sL1;  // this stage's lambda
  int lo_c = 0;  // first child node held in LDS

  for (; s >= a.s_begin; --s) {
    const int2 rr = rg[s - a.s_begin];
    const int lo = rr.x, nb = rr.y - rr.x;
    const bool kids_in_lds = s < a.s_end;
    const bool kids_global = !kids_in_lds && s + 1 < a.N;

    // lambda phase (x-slots) and sigma / w3 (u-slots)
    T aval[QX], w3v[QX], sig[QX], kap[QX];
#pragma unroll
    for (int q = 0; q < QX; ++q) {
      const int idx = tid + q * kSegThreads;
      const int b = idx / LDX, i = idx - b * LDX;
      const bool ok = idx < NB * LDX && b < nb && i < nx;
      T av = power ? scale * (px[q][0] + px[q][2])
                   : wext(px[q][0], px[q][1], beta) + wext(px[q][2], px[q][3], beta);
      T ls = T(0);
      if (ok) {
        const int n = lo + b;
        const int ce = a.cend[n];
        for (int c = a.cbeg[n]; c < ce; ++c)
          ls += kids_in_lds ? sLc[(c - lo_c) * LDX + i]
                            : (kids_global ? a.lam[(size_t)c * LDX + i] : T(0));
      }
      aval[q] = ok ? av : T(0);
      if (idx < NB * LDX) sLn[idx] = a.a_ident ? (aval[q] + ls) : ls;
    }
#pragma unroll
    for (int q = 0; q < QX; ++q) {
      const int idx = tid + q * kSegThreads;
      const int b = idx / LDU, i = idx - b * LDU;
      const bool ok = idx < NB * LDU && b < nb && i < nu;
      w3v[q] = power ? scale * pu[q][0] : wext(pu[q][0], pu[q][1], beta);
      kap[q] = pu[q][2];
      T sg = T(0);
      if (ok) {
        const int n = lo + b;
        const int ce = a.cend[n];
        for (int c = a.cbeg[n]; c < ce; ++c)
          sg += kids_in_lds ? sJ[(c - lo_c) * LDU + i]
                            : (kids_global ? a.jv[(size_t)c * LDU + i] : T(0));
      }
      sig[q] = ok ? sg : T(0);
    }
    // next stage's factor and node inputs are loaded while this stage computes
    if (s > a.s_begin) {
      load_factor<T>(a.F + (size_t)(s - 1) * kLDU * kLDU, r, kb, mnext);
      load_nodes(s - 1);
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
        const int pe = a.Btrow[i + 1];
        for (int p = a.Btrow[i]; p < pe; ++p) e += a.Btval[p] * sLn[b * LDX + a.Btcol[p]];
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
    __syncthreads();
#pragma unroll
    for (int q = 0; q < QX; ++q) {
      const int idx = tid + q * kSegThreads;
      const int b = idx / LDU, i = idx - b * LDU;
      if (idx < NB * LDU && b < nb && i < nu) {
        const T jn = kap[q] + sum_partials<T, NB>(red, b, i);
        sJ[b * LDU + i] = jn;
        a.jv[(size_t)(lo + b) * LDU + i] = jn;
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
#pragma unroll
    for (int j = 0; j < kKC; ++j) mreg[j] = mnext[j];
  }
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
  const int2* rg = a.ranges + (size_t)blockIdx.x * a.nst;

  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* sU0 = reinterpret_cast<T*>(smem_raw);
  T* sU1 = sU0 + NB * LDU;
  T* sX0 = sU1 + NB * LDU;
  T* sX1 = sX0 + NB * LDX;
  T* red = sX1 + NB * LDX;  // 4 * NB * 128 partials; reused for the norms
  __shared__ double sred[kSegThreads];
  __shared__ int s_last;

  const int r = tid % kRT;
  const int ks = __builtin_amdgcn_readfirstlane(tid / kRT);  // wave-uniform slice
  const int kb = ks * kKC;
  // prefetch registers: u-slots (j, 1/p), x-slots (g)
  T pj[QX], pp[QX], pg[QX];
  T mreg[kKC], mnext[kKC];

  auto load_nodes = [&](int s) {
    const int2 rr = rg[s - a.s_begin];
    const int lo = rr.x, nb = rr.y - rr.x;
#pragma unroll
    for (int q = 0; q < QX; ++q) {
      const int idx = tid + q * kSegThreads;
      const int b = idx / LDU, i = idx - b * LDU;
      const bool ok = idx < NB * LDU && b < nb && i < nu;
      pj[q] = ldm(a.jv, (size_t)(lo + b) * LDU + i, ok);
      pp[q] = ldm(a.invp, (size_t)(lo + b), ok);
    }
#pragma unroll
    for (int q = 0; q < QX; ++q) {
      const int idx = tid + q * kSegThreads;
      const int b = idx / LDX, i = idx - b * LDX;
      const bool ok = idx < NB * LDX && b < nb && i < nx && !power;
      pg[q] = ldm(a.g, (size_t)(lo + b) * LDX + i, ok);
    }
  };

  int s = a.s_begin;
  load_factor<T>(a.F + (size_t)s * kLDU * kLDU, r, kb, mreg);
  load_nodes(s);
  T* sUp = sU0;  // parents (stage s-1)
  T* sUn = sU1;
  T* sXp = sX0;
  T* sXn = sX1;
  int lo_p = 0, np = 0;
  {  // parents of the first stage come from global memory (or p, q at the root)
    const int2 rr = rg[0];
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

  for (; s <= a.s_end; ++s) {
    const int2 rr = rg[s - a.s_begin];
    const int lo = rr.x, nb = rr.y - rr.x;
    T cj[QX], cp[QX], cg[QX];
#pragma unroll
    for (int q = 0; q < QX; ++q) {
      cj[q] = pj[q];
      cp[q] = pp[q];
      cg[q] = pg[q];
    }
    if (s < a.s_end) {
      load_factor<T>(a.F + (size_t)(s + 1) * kLDU * kLDU, r, kb, mnext);
      load_nodes(s + 1);
    }
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
    __syncthreads();
    const T wsc = a.wu_scalar ? a.wu : T(1);
#pragma unroll
    for (int q = 0; q < QX; ++q) {
      const int idx = tid + q * kSegThreads;
      const int b = idx / LDU, i = idx - b * LDU;
      if (idx < NB * LDU) {
        T un = T(0);
        if (b < nb && i < nu) {
          const int pb = a.anc[lo + b] >= 0 ? a.anc[lo + b] - lo_p : 0;
          un = wsc * sum_partials<T, NB>(red, pb, i) + cj[q] * cp[q];
          a.u[(size_t)(lo + b) * LDU + i] = un;
        }
        sUn[idx] = un;
      }
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
      if (idx < NB * LDX && b < nb && i < nx) {
        const int pb = a.anc[lo + b] >= 0 ? a.anc[lo + b] - lo_p : 0;
        xn = a.a_ident ? sXp[pb * LDX + i] : sum_partials<T, NB>(red, pb, i);
        const int pe = a.Brow[i + 1];
        for (int p = a.Brow[i]; p < pe; ++p) xn += a.Bval[p] * sUn[b * LDU + a.Bcol[p]];
        xn += cg[q];
        a.x[(size_t)(lo + b) * LDX + i] = xn;
      }
      xv[q] = xn;
    }
    __syncthreads();  // red is reused below
#pragma unroll
    for (int q = 0; q < QX; ++q) {
      const int idx = tid + q * kSegThreads;
      if (idx < NB * LDX) sXn[idx] = xv[q];
    }

    // ---- prox / dual update ----
    double* sq = reinterpret_cast<double*>(red);  // [2][NB][LDX] squared block residuals
    T r1v[QX], r2v[QX], w1v[QX], w2v[QX];
#pragma unroll
    for (int q = 0; q < QX; ++q) {
      const int idx = tid + q * kSegThreads;
      const int b = idx / LDX, i = idx - b * LDX;
      const bool ok = idx < NB * LDX && b < nb && i < nx;
      double q1 = 0.0, q2 = 0.0;
      r1v[q] = r2v[q] = w1v[q] = w2v[q] = T(0);
      if (ok) {
        const size_t n = (size_t)(lo + b);
        const T* yc = Yc + n * LDY;
        T* yn = Yn + n * LDY;
        const T xi = xv[q];
        if (power) {
          yn[i] = -xi;
          yn[LDX + i] = -xi;
          zsq += 2.0 * (double)xi * (double)xi;
        } else {
          const T w1 = wext(yc[i], yn[i], beta);
          const T w2 = wext(yc[LDX + i], yn[LDX + i], beta);
          const T v1 = w1 + gam * xi, v2 = w2 + gam * xi;
          const T z1 = v1 / gam, z2 = v2 / gam;
          const T rr1 = v1 - gam * fmin(fmax(z1, a.xmin[i]), a.xmax[i]);
          const T rr2 = v2 - gam * fmax(z2, a.xs[i]);
          r1v[q] = rr1;
          r2v[q] = rr2;
          w1v[q] = w1;
          w2v[q] = w2;
          q1 = (double)rr1 * (double)rr1;
          q2 = (double)rr2 * (double)rr2;
        }
      }
      if (idx < NB * LDX) {
        sq[idx] = q1;
        sq[NB * LDX + idx] = q2;
      }
    }
#pragma unroll
    for (int q = 0; q < QX; ++q) {
      const int idx = tid + q * kSegThreads;
      const int b = idx / LDU, i = idx - b * LDU;
      if (idx < NB * LDU && b < nb && i < nu) {
        const size_t n = (size_t)(lo + b);
        const T* yc = Yc + n * LDY + 2 * LDX;
        T* yn = Yn + n * LDY + 2 * LDX;
        const T ui = sUn[b * LDU + i];
        if (power) {
          yn[i] = -ui;
          zsq += (double)ui * (double)ui;
        } else {
          const T w = wext(yc[i], yn[i], beta);
          const T v = w + gam * ui;
          const T y = v - gam * fmin(fmax(v / gam, a.umin[i]), a.umax[i]);
          yn[i] = y;
          double d = fabs((double)y - (double)w) / gam64;
          if (!(d <= 1.0e308)) d = INFINITY;
          rmax = fmax(rmax, d);
        }
      }
    }
    __syncthreads();
    if (!power) {
      // per-node sums over the LDX entries of each block, fixed tree order
      for (int st = a.LDXR / 2; st > 0; st >>= 1) {
        for (int idx = tid; idx < 2 * NB * st; idx += kSegThreads) {
          const int h = idx / (NB * st), rem = idx - h * NB * st;
          const int b = rem / st, i = rem - b * st;
          if (i + st < LDX) sq[h * NB * LDX + b * LDX + i] += sq[h * NB * LDX + b * LDX + i + st];
        }
        __syncthreads();
      }
#pragma unroll
      for (int q = 0; q < QX; ++q) {
        const int idx = tid + q * kSegThreads;
        const int b = idx / LDX, i = idx - b * LDX;
        if (idx < NB * LDX && b < nb && i < nx) {
          const double n1 = sqrt(sq[b * LDX]), n2 = sqrt(sq[NB * LDX + b * LDX]);
          const T sc1 = n1 > (double)a.Wx ? (T)((double)a.Wx / n1) : T(1);
          const T sc2 = n2 > (double)a.Ws ? (T)((double)a.Ws / n2) : T(1);
          const T y1 = r1v[q] * sc1, y2 = r2v[q] * sc2;
          T* yn = Yn + (size_t)(lo + b) * LDY;
          yn[i] = y1;
          yn[LDX + i] = y2;
          double d1 = fabs((double)y1 - (double)w1v[q]) / gam64;
          double d2 = fabs((double)y2 - (double)w2v[q]) / gam64;
          if (!(d1 <= 1.0e308)) d1 = INFINITY;
          if (!(d2 <= 1.0e308)) d2 = INFINITY;
          rmax = fmax(rmax, fmax(d1, d2));
        }
      }
      __syncthreads();
    }
    // this stage's nodes are the next stage's parents
    T* t = sUp;
    sUp = sUn;
    sUn = t;
    t = sXp;
    sXp = sXn;
    sXn = t;
    lo_p = lo;
    np = nb;
#pragma unroll
    for (int j = 0; j < kKC; ++j) mreg[j] = mnext[j];
  }

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
size_t seg_lds_bytes(const SegArgs<T>& a) {
  return (size_t)(2 * NB * a.LDX + 2 * NB * a.LDU + 4 * NB * kRT) * sizeof(T);
}

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
    case 16: launch_seg_nb<T, 16>(fwd, a, n_wg, st); break;
    case 8: launch_seg_nb<T, 8>(fwd, a, n_wg, st); break;
    case 4: launch_seg_nb<T, 4>(fwd, a, n_wg, st); break;
    case 2: launch_seg_nb<T, 2>(fwd, a, n_wg, st); break;
    default: launch_seg_nb<T, 1>(fwd, a, n_wg, st); break;
  }
}

template void launch_seg<double>(bool, int, const SegArgs<double>&, int, hipStream_t);
template void launch_seg<float>(bool, int, const SegArgs<float>&, int, hipStream_t);

}  // namespace tapg
