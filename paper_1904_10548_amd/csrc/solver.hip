// Device layer of the dual APG solver: HIP kernels for gfx950 and their
// orchestration.
//
// One APG iteration (Sec. 4.3, eqs. apg:1-apg:2) on a tree of N stages is
//   N backward-stage launches  (s = N-1 .. 0)  : costate and the k-recursion
//   N forward-stage launches   (s = 0 .. N-1)  : inputs, states, then the
//                                               prox/dual update and residual
//   1 end-of-iteration launch                  : stop test, theta/beta update
// Every launch processes all nodes of one stage in tiles of NB nodes per
// workgroup, so each factor-matrix column read from L2 serves NB nodes.
// The extrapolated dual w = y + beta (y - y_prev) is recomputed where needed
// and never stored; y^{nu+1} overwrites y^{nu-1} in place.
//
// Node-major layouts: node n's block of a vector quantity of dimension d
// starts at n * LD(d) (LD rounded up to 16 elements).  The dual stores
// (y1 | y2 | y3) at offsets 0, LDX, 2 LDX.  Matrices are column-major so that
// the 64 lanes of a wave, each owning one output row, read 64 consecutive
// elements of a column.
#include <cmath>
#include <cstring>
#include <random>

#include "solver.h"

namespace tapg {

constexpr int kThreads = 256;

template <typename T>
struct SweepArgs {
  int nx, nu, LDX, LDU, LDY;
  int s, node0, count, tile_base;
  int mode;  // 0: APG iteration, 1: power iteration (zero data, no prox)
  const int* anc;
  const int* cbeg;
  const int* cend;
  const T* invp;
  const T* F;   // Fbar_s
  const T* Kb;  // Kbar_s
  const T* At;
  const T* Bt;
  const T* A;
  const T* B;
  const T* xmin;
  const T* xmax;
  const T* xs;
  const T* umin;
  const T* umax;
  T Wx, Ws;
  const T* kappa;
  const T* g;
  const T* pq;
  T* Y0;
  T* Y1;
  T* lam;
  T* jv;
  T* u;
  T* x;
  DevCtl* ctl;
  double* part;
};

// w = y + beta (y - y_prev), the extrapolation of eq. apg:1.
template <typename T>
__device__ __forceinline__ T wext(T y, T yp, T beta) {
  return y + beta * (y - yp);
}

// out[b] = sum_k M1(r, k) X1[b][k] + sum_k M2(r, k) X2[b][k] for the thread's
// output row r.  Threads are split into KS = 256/RT slices of the k range
// (RT = 64, 128 or 256 rows per slice); the slices are summed in a fixed
// order through LDS, so results do not depend on timing.  Every thread of
// the block must call it.  Returns true on the threads that own a row's
// final value (slice 0, r < R).
template <typename T, int NB>
__device__ __forceinline__ bool gemv_tile(const T* __restrict__ M1, int K1, const T* X1, int ldx1,
                                          const T* __restrict__ M2, int K2, const T* X2, int ldx2,
                                          int ldm, int R, T* red, T (&out)[NB], int& row) {
  const int RT = R <= 64 ? 64 : (R <= 128 ? 128 : 256);
  const int KS = kThreads / RT;
  const int tid = threadIdx.x;
  const int r = tid % RT, ks = tid / RT;
  row = r;
  T acc[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) acc[b] = T(0);
  if (r < R) {
    {
      const int c = (K1 + KS - 1) / KS;
      const int kb = ks * c, ke = min(K1, kb + c);
      const T* mp = M1 + (size_t)kb * ldm + r;
#pragma unroll 8
      for (int k = kb; k < ke; ++k) {
        const T m = mp[(size_t)(k - kb) * ldm];
#pragma unroll
        for (int b = 0; b < NB; ++b) acc[b] += m * X1[b * ldx1 + k];
      }
    }
    if (M2 != nullptr) {
      const int c = (K2 + KS - 1) / KS;
      const int kb = ks * c, ke = min(K2, kb + c);
      const T* mp = M2 + (size_t)kb * ldm + r;
#pragma unroll 8
      for (int k = kb; k < ke; ++k) {
        const T m = mp[(size_t)(k - kb) * ldm];
#pragma unroll
        for (int b = 0; b < NB; ++b) acc[b] += m * X2[b * ldx2 + k];
      }
    }
  }
  if (KS == 1) {
#pragma unroll
    for (int b = 0; b < NB; ++b) out[b] = acc[b];
    return r < R;
  }
#pragma unroll
  for (int b = 0; b < NB; ++b) red[(ks * NB + b) * RT + r] = acc[b];
  __syncthreads();
  const bool mine = (ks == 0) && (r < R);
  if (mine) {
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      T s = red[b * RT + r];
      for (int j = 1; j < KS; ++j) s += red[(j * NB + b) * RT + r];
      out[b] = s;
    }
  }
  __syncthreads();
  return mine;
}

// ---------------------------------------------------------------------------
// Backward stage: for every node n of stage s
//   lambda_n = a_n + A' sum_{c in child(n)} lambda_c,       a_n = w1_n + w2_n
//   e_n      = w3_n + B' lambda_n                           (p_n c_n is in kappa)
//   j_n      = kappa_n - Fbar_s e_n / 2 + Kbar_s sum_{c} j_c
// where j_n = p_n k_n is the probability-weighted affine term of the input
// law u_n = Kbar_s u_anc + k_n, and kappa_n = p_n (Gammabar_s ubar_n - Fbar_s c_n / 2).
// ---------------------------------------------------------------------------
template <typename T, int NB>
__global__ __launch_bounds__(kThreads) void bwd_stage_kernel(SweepArgs<T> a) {
  const DevCtl* ctl = a.ctl;
  if (ctl->done) return;
  const int n0 = a.node0 + blockIdx.x * NB;
  const int nb = min(NB, a.node0 + a.count - n0);
  const int it = ctl->iter;
  const T* Yc = (it & 1) ? a.Y1 : a.Y0;
  const T* Yo = (it & 1) ? a.Y0 : a.Y1;
  const bool power = a.mode == 1;
  const T beta = (T)ctl->beta;
  const T scale = (T)ctl->pw_scale;
  const int LDX = a.LDX, LDU = a.LDU, LDY = a.LDY;

  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* sA = reinterpret_cast<T*>(smem_raw);  // a, then lambda
  T* sL = sA + NB * LDX;                   // sum of children's lambda
  T* sE = sL + NB * LDX;                   // w3, then -e/2
  T* sS = sE + NB * LDU;                   // sum of children's j
  T* red = sS + NB * LDU;                  // NB * 256

  for (int idx = threadIdx.x; idx < NB * LDX; idx += kThreads) {
    const int b = idx / LDX, i = idx - b * LDX;
    T av = T(0), ls = T(0);
    if (b < nb && i < a.nx) {
      const int n = n0 + b;
      const T* yc = Yc + (size_t)n * LDY;
      const T* yo = Yo + (size_t)n * LDY;
      const T w1 = power ? scale * yc[i] : wext(yc[i], yo[i], beta);
      const T w2 = power ? scale * yc[LDX + i] : wext(yc[LDX + i], yo[LDX + i], beta);
      av = w1 + w2;
      const int ce = a.cend[n];
      for (int c = a.cbeg[n]; c < ce; ++c) ls += a.lam[(size_t)c * LDX + i];
    }
    sA[idx] = av;
    sL[idx] = ls;
  }
  for (int idx = threadIdx.x; idx < NB * LDU; idx += kThreads) {
    const int b = idx / LDU, i = idx - b * LDU;
    T w3 = T(0), sg = T(0);
    if (b < nb && i < a.nu) {
      const int n = n0 + b;
      const T* yc = Yc + (size_t)n * LDY + 2 * LDX;
      const T* yo = Yo + (size_t)n * LDY + 2 * LDX;
      w3 = power ? scale * yc[i] : wext(yc[i], yo[i], beta);
      const int ce = a.cend[n];
      for (int c = a.cbeg[n]; c < ce; ++c) sg += a.jv[(size_t)c * LDU + i];
    }
    sE[idx] = w3;
    sS[idx] = sg;
  }
  __syncthreads();

  T out[NB];
  int r;
  // lambda = a + A' lambda_sum
  if (gemv_tile<T, NB>(a.At, a.nx, sL, LDX, nullptr, 0, nullptr, 0, LDX, a.nx, red, out, r)) {
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      if (b < nb) {
        const T l = sA[b * LDX + r] + out[b];
        sA[b * LDX + r] = l;
        a.lam[(size_t)(n0 + b) * LDX + r] = l;
      }
    }
  }
  __syncthreads();
  // e = w3 + B' lambda; keep -e/2
  if (gemv_tile<T, NB>(a.Bt, a.nx, sA, LDX, nullptr, 0, nullptr, 0, LDU, a.nu, red, out, r)) {
#pragma unroll
    for (int b = 0; b < NB; ++b) sE[b * LDU + r] = T(-0.5) * (sE[b * LDU + r] + out[b]);
  }
  __syncthreads();
  // j = kappa + Fbar (-e/2) + Kbar sigma
  if (gemv_tile<T, NB>(a.F, a.nu, sE, LDU, a.Kb, a.nu, sS, LDU, LDU, a.nu, red, out, r)) {
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      if (b < nb) {
        const size_t o = (size_t)(n0 + b) * LDU + r;
        const T k0 = power ? T(0) : a.kappa[o];
        a.jv[o] = k0 + out[b];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Forward stage: for every node n of stage s
//   u_n = Kbar_s u_anc + j_n / p_n,    x_n = A x_anc + B u_n + Gd d_n
// then the dual update of eq. apg:2 through the Moreau decomposition:
//   v = w + gamma (x_n, x_n, u_n)
//   blocks 1, 2: r = v - gamma P_C(v / gamma),  y+ = r min(1, W / |r|)
//                (C = [xmin, xmax], W = W_x; C = [xs, inf), W = W_s)
//   block 3:     y+ = v - gamma P_U(v / gamma)
// and the residual max |y+ - w| / gamma in FP64.  In power-iteration mode the
// block writes z = -(x_n, x_n, u_n) and the tile's |z|^2 instead.
// ---------------------------------------------------------------------------
template <typename T, int NB>
__global__ __launch_bounds__(kThreads) void fwd_stage_kernel(SweepArgs<T> a) {
  DevCtl* ctl = a.ctl;
  if (ctl->done) return;
  const int n0 = a.node0 + blockIdx.x * NB;
  const int nb = min(NB, a.node0 + a.count - n0);
  const int it = ctl->iter;
  const T* Yc = (it & 1) ? a.Y1 : a.Y0;
  T* Yn = (it & 1) ? a.Y0 : a.Y1;  // y^{nu-1} in, y^{nu+1} out
  const bool power = a.mode == 1;
  const T beta = (T)ctl->beta;
  const double gam64 = ctl->gamma;
  const T gam = (T)gam64;
  const int LDX = a.LDX, LDU = a.LDU, LDY = a.LDY;

  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* sUp = reinterpret_cast<T*>(smem_raw);  // parent inputs
  T* sXp = sUp + NB * LDU;                  // parent states
  T* sUn = sXp + NB * LDX;                  // u_n
  T* sXn = sUn + NB * LDU;                  // x_n
  T* red = sXn + NB * LDX;                  // NB * 256
  T* sW = red + NB * kThreads;              // w (blocks 1, 2)
  T* sR = sW + NB * LDY;                    // r (blocks 1, 2)
  __shared__ double ps1[kThreads], ps2[kThreads], pmax[kThreads];

  for (int idx = threadIdx.x; idx < NB * LDU; idx += kThreads) {
    const int b = idx / LDU, i = idx - b * LDU;
    T up = T(0);
    if (b < nb && i < a.nu) {
      const int par = a.anc[n0 + b];
      up = par >= 0 ? a.u[(size_t)par * LDU + i] : (power ? T(0) : a.pq[LDX + i]);
    }
    sUp[idx] = up;
    sUn[idx] = T(0);
  }
  for (int idx = threadIdx.x; idx < NB * LDX; idx += kThreads) {
    const int b = idx / LDX, i = idx - b * LDX;
    T xp = T(0);
    if (b < nb && i < a.nx) {
      const int par = a.anc[n0 + b];
      xp = par >= 0 ? a.x[(size_t)par * LDX + i] : (power ? T(0) : a.pq[i]);
    }
    sXp[idx] = xp;
    sXn[idx] = T(0);
  }
  __syncthreads();

  T out[NB];
  int r;
  // u = Kbar u_anc + j / p
  if (gemv_tile<T, NB>(a.Kb, a.nu, sUp, LDU, nullptr, 0, nullptr, 0, LDU, a.nu, red, out, r)) {
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      if (b < nb) {
        const int n = n0 + b;
        const size_t o = (size_t)n * LDU + r;
        const T un = out[b] + a.jv[o] * a.invp[n];
        a.u[o] = un;
        sUn[b * LDU + r] = un;
      }
    }
  }
  __syncthreads();
  // x = A x_anc + B u + g
  if (gemv_tile<T, NB>(a.A, a.nx, sXp, LDX, a.B, a.nu, sUn, LDU, LDX, a.nx, red, out, r)) {
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      if (b < nb) {
        const size_t o = (size_t)(n0 + b) * LDX + r;
        const T xn = out[b] + (power ? T(0) : a.g[o]);
        a.x[o] = xn;
        sXn[b * LDX + r] = xn;
      }
    }
  }
  __syncthreads();

  // ---- prox / dual update, one group of TPN threads per node ----
  constexpr int TPN = kThreads / NB;
  const int b = threadIdx.x / TPN, l = threadIdx.x % TPN;
  double s1 = 0.0, s2 = 0.0, rmax = 0.0;
  if (b < nb) {
    const int n = n0 + b;
    const T* yc = Yc + (size_t)n * LDY;
    T* yn = Yn + (size_t)n * LDY;
    for (int i = l; i < LDY; i += TPN) {
      if (i < 2 * LDX) {
        const int blk = i < LDX ? 0 : 1;
        const int k = i - blk * LDX;
        if (k >= a.nx) continue;
        const T xi = sXn[b * LDX + k];
        if (power) {
          const T z = -xi;
          yn[i] = z;
          s1 += (double)z * (double)z;
          continue;
        }
        const T w = wext(yc[i], yn[i], beta);
        const T v = w + gam * xi;
        const T zz = v / gam;
        const T pz = blk == 0 ? fmin(fmax(zz, a.xmin[k]), a.xmax[k]) : fmax(zz, a.xs[k]);
        const T rr = v - gam * pz;
        if (blk == 0)
          s1 += (double)rr * (double)rr;
        else
          s2 += (double)rr * (double)rr;
        sW[b * LDY + i] = w;
        sR[b * LDY + i] = rr;
      } else {
        const int k = i - 2 * LDX;
        if (k >= a.nu) continue;
        const T ui = sUn[b * LDU + k];
        if (power) {
          const T z = -ui;
          yn[i] = z;
          s1 += (double)z * (double)z;
          continue;
        }
        const T w = wext(yc[i], yn[i], beta);
        const T v = w + gam * ui;
        const T t = fmin(fmax(v / gam, a.umin[k]), a.umax[k]);
        const T y = v - gam * t;
        yn[i] = y;
        double d = fabs((double)y - (double)w) / gam64;
        if (!(d <= 1.0e308)) d = INFINITY;
        rmax = fmax(rmax, d);
      }
    }
  }
  ps1[threadIdx.x] = s1;
  ps2[threadIdx.x] = s2;
  __syncthreads();
  // per-node sums in a fixed tree order (power mode: whole-tile sum)
  const int span = power ? kThreads : TPN;
  const int lane = power ? threadIdx.x : l;
  for (int st = span / 2; st > 0; st >>= 1) {
    if (lane < st) {
      ps1[threadIdx.x] += ps1[threadIdx.x + st];
      ps2[threadIdx.x] += ps2[threadIdx.x + st];
    }
    __syncthreads();
  }
  if (power) {
    if (threadIdx.x == 0) a.part[a.tile_base + blockIdx.x] = ps1[0];
    return;
  }
  if (b < nb) {
    const int n = n0 + b;
    T* yn = Yn + (size_t)n * LDY;
    const double n1 = sqrt(ps1[b * TPN]), n2 = sqrt(ps2[b * TPN]);
    const T sc1 = n1 > (double)a.Wx ? (T)((double)a.Wx / n1) : T(1);
    const T sc2 = n2 > (double)a.Ws ? (T)((double)a.Ws / n2) : T(1);
    for (int i = l; i < 2 * LDX; i += TPN) {
      const int blk = i < LDX ? 0 : 1;
      const int k = i - blk * LDX;
      if (k >= a.nx) continue;
      const T y = sR[b * LDY + i] * (blk == 0 ? sc1 : sc2);
      yn[i] = y;
      double d = fabs((double)y - (double)sW[b * LDY + i]) / gam64;
      if (!(d <= 1.0e308)) d = INFINITY;
      rmax = fmax(rmax, d);
    }
  }
  pmax[threadIdx.x] = rmax;
  __syncthreads();
  for (int st = kThreads / 2; st > 0; st >>= 1) {
    if (threadIdx.x < st) pmax[threadIdx.x] = fmax(pmax[threadIdx.x], pmax[threadIdx.x + st]);
    __syncthreads();
  }
  if (threadIdx.x == 0)
    atomicMax(&ctl->res_bits, (unsigned long long)__double_as_longlong(pmax[0]));
}

// End of one APG iteration: record the residual, test for termination, and
// advance theta_{nu+1} = (sqrt(theta^4 + 4 theta^2) - theta^2) / 2 and
// beta_{nu+1} = theta_{nu+1} (1/theta_nu - 1) (Sec. 4.3).
__global__ void iter_end_kernel(DevCtl* c, double* hist) {
  if (c->done) return;
  const double res = __longlong_as_double((long long)c->res_bits);
  c->res_bits = 0ull;
  hist[c->iter] = res;
  c->last_res = res;
  c->iter += 1;
  if (!(res < INFINITY)) {
    c->numeric = 1;
    c->done = 1;
  } else if (c->tol > 0.0 && res <= c->tol) {
    c->converged = 1;
    c->done = 1;
  } else if (c->iter >= c->max_iter) {
    c->done = 1;
  }
  const double th = c->theta;
  const double t2 = th * th;
  const double thn = 0.5 * (sqrt(t2 * t2 + 4.0 * t2) - t2);
  c->theta_prev = th;
  c->theta = thn;
  c->beta = thn * (1.0 / th - 1.0);
}

// Power iteration step end: |M v| from the per-tile partial sums (fixed order).
__global__ __launch_bounds__(kThreads) void power_end_kernel(DevCtl* c, const double* part, int n) {
  __shared__ double s[kThreads];
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += kThreads) acc += part[i];
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int st = kThreads / 2; st > 0; st >>= 1) {
    if (threadIdx.x < st) s[threadIdx.x] += s[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double L = sqrt(s[0]);
    c->L = L;
    c->pw_scale = L > 0.0 ? 1.0 / L : 0.0;
    c->iter += 1;
  }
}

// ---------------------------------------------------------------------------
// Per-solve data step (FP64), one block per node:
//   ubar_n = -E^+ Ed d_n,  c_n = W_alpha (alpha0 + pi_n c_E),
//   kappa_n = p_n (Gammabar_s ubar_n - Fbar_s c_n / 2),  g_n = Gd d_n.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kThreads) void data_step_kernel(
    int nx, int nu, int nd, int LDX, int LDU, const int* stage, const double* prob,
    const double* demand, const double* price, const double* Pd, const double* Gd,
    const double* Gbar, const double* Fbar, const double* alpha0, const double* cE,
    double W_alpha, T* kappa, T* g) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* sD = reinterpret_cast<double*>(smem_raw);
  double* sUb = sD + nd;
  double* sC = sUb + LDU;
  const int n = blockIdx.x;
  const int s = stage[n];
  for (int k = threadIdx.x; k < nd; k += kThreads) sD[k] = demand[(size_t)n * nd + k];
  __syncthreads();
  const double pi = price[n];
  for (int r = threadIdx.x; r < nu; r += kThreads) {
    double ub = 0.0;
    for (int k = 0; k < nd; ++k) ub += Pd[(size_t)k * LDU + r] * sD[k];
    sUb[r] = ub;
    sC[r] = W_alpha * (alpha0[r] + pi * cE[r]);
  }
  __syncthreads();
  const double pn = prob[n];
  const double* Gs = Gbar + (size_t)s * LDU * LDU;
  const double* Fs = Fbar + (size_t)s * LDU * LDU;
  for (int r = threadIdx.x; r < nu; r += kThreads) {
    double gu = 0.0, fc = 0.0;
    for (int k = 0; k < nu; ++k) {
      gu += Gs[(size_t)k * LDU + r] * sUb[k];
      fc += Fs[(size_t)k * LDU + r] * sC[k];
    }
    kappa[(size_t)n * LDU + r] = (T)(pn * (gu - 0.5 * fc));
  }
  for (int r = threadIdx.x; r < nx; r += kThreads) {
    double gg = 0.0;
    for (int k = 0; k < nd; ++k) gg += Gd[(size_t)k * LDX + r] * sD[k];
    g[(size_t)n * LDX + r] = (T)gg;
  }
}

// Deterministic block reductions (fixed tree order).
__device__ double block_sum(double v, double* s) {
  s[threadIdx.x] = v;
  __syncthreads();
  for (int st = kThreads / 2; st > 0; st >>= 1) {
    if (threadIdx.x < st) s[threadIdx.x] += s[threadIdx.x + st];
    __syncthreads();
  }
  const double r = s[0];
  __syncthreads();
  return r;
}

__device__ double block_max(double v, double* s) {
  s[threadIdx.x] = v;
  __syncthreads();
  for (int st = kThreads / 2; st > 0; st >>= 1) {
    if (threadIdx.x < st) s[threadIdx.x] = fmax(s[threadIdx.x], s[threadIdx.x + st]);
    __syncthreads();
  }
  const double r = s[0];
  __syncthreads();
  return r;
}

// ---------------------------------------------------------------------------
// Primal cost and violations of (u_hat, x_hat), FP64, one block per node:
//   p_n (c_n'u_n + du'W_u du) + W_x dist(x_n|[xmin,xmax]) + W_s dist(x_n|[xs,inf)),
//   max box violation, |E u + Ed d|_inf, dynamics residual.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kThreads) void cost_kernel(
    int nx, int nu, int nd, int ns, int LDX, int LDU, const int* anc, const double* prob,
    const double* demand, const double* price, const T* u, const T* x, const double* pq,
    const double* A, const double* B, const double* Gd, const double* E, const double* Ed,
    const double* Wu, const double* alpha0, const double* cE, const double* xmin,
    const double* xmax, const double* xs, const double* umin, const double* umax,
    double W_alpha, double W_x, double W_s, double* part) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* sU = reinterpret_cast<double*>(smem_raw);
  double* sDu = sU + LDU;
  double* sXp = sDu + LDU;
  double* sD = sXp + LDX;
  __shared__ double red[kThreads];
  const int n = blockIdx.x;
  const int par = anc[n];
  for (int i = threadIdx.x; i < nu; i += kThreads) {
    const double un = (double)u[(size_t)n * LDU + i];
    const double up = par >= 0 ? (double)u[(size_t)par * LDU + i] : pq[LDX + i];
    sU[i] = un;
    sDu[i] = un - up;
  }
  for (int i = threadIdx.x; i < nx; i += kThreads)
    sXp[i] = par >= 0 ? (double)x[(size_t)par * LDX + i] : pq[i];
  for (int k = threadIdx.x; k < nd; k += kThreads) sD[k] = demand[(size_t)n * nd + k];
  __syncthreads();
  double lin = 0.0, quad = 0.0, vbox = 0.0;
  const double pi = price[n];
  for (int r = threadIdx.x; r < nu; r += kThreads) {
    double wd = 0.0;
    for (int k = 0; k < nu; ++k) wd += Wu[(size_t)k * LDU + r] * sDu[k];
    quad += sDu[r] * wd;
    lin += W_alpha * (alpha0[r] + pi * cE[r]) * sU[r];
    vbox = fmax(vbox, fmax(umin[r] - sU[r], sU[r] - umax[r]));
  }
  double d1 = 0.0, d2 = 0.0, dyn = 0.0;
  for (int r = threadIdx.x; r < nx; r += kThreads) {
    const double xr = (double)x[(size_t)n * LDX + r];
    const double e1 = xr - fmin(fmax(xr, xmin[r]), xmax[r]);
    const double e2 = xr - fmax(xr, xs[r]);
    d1 += e1 * e1;
    d2 += e2 * e2;
    double pred = 0.0;
    for (int k = 0; k < nx; ++k) pred += A[(size_t)k * LDX + r] * sXp[k];
    for (int k = 0; k < nu; ++k) pred += B[(size_t)k * LDX + r] * sU[k];
    for (int k = 0; k < nd; ++k) pred += Gd[(size_t)k * LDX + r] * sD[k];
    dyn = fmax(dyn, fabs(xr - pred));
  }
  double mass = 0.0;
  for (int rr = threadIdx.x; rr < ns; rr += kThreads) {
    double e = 0.0;
    for (int k = 0; k < nu; ++k) e += E[(size_t)rr * nu + k] * sU[k];
    for (int k = 0; k < nd; ++k) e += Ed[(size_t)rr * nd + k] * sD[k];
    mass = fmax(mass, fabs(e));
  }
  lin = block_sum(lin, red);
  quad = block_sum(quad, red);
  d1 = block_sum(d1, red);
  d2 = block_sum(d2, red);
  vbox = block_max(fmax(vbox, 0.0), red);
  dyn = block_max(dyn, red);
  mass = block_max(mass, red);
  if (threadIdx.x == 0) {
    part[(size_t)n * 4 + 0] = prob[n] * (lin + quad) + W_x * sqrt(d1) + W_s * sqrt(d2);
    part[(size_t)n * 4 + 1] = vbox;
    part[(size_t)n * 4 + 2] = mass;
    part[(size_t)n * 4 + 3] = dyn;
  }
}

__global__ __launch_bounds__(kThreads) void cost_reduce_kernel(const double* part, int K,
                                                               double* out) {
  __shared__ double red[kThreads];
  double c = 0.0, vb = 0.0, ms = 0.0, dy = 0.0;
  for (int n = threadIdx.x; n < K; n += kThreads) {
    c += part[(size_t)n * 4 + 0];
    vb = fmax(vb, part[(size_t)n * 4 + 1]);
    ms = fmax(ms, part[(size_t)n * 4 + 2]);
    dy = fmax(dy, part[(size_t)n * 4 + 3]);
  }
  c = block_sum(c, red);
  vb = block_max(vb, red);
  ms = block_max(ms, red);
  dy = block_max(dy, red);
  if (threadIdx.x == 0) {
    out[0] = c;
    out[1] = vb;
    out[2] = fmax(ms, dy);
  }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
namespace {

template <typename T>
T* dmalloc(size_t n) {
  void* p = nullptr;
  if (n == 0) n = 1;
  hipError_t e = hipMalloc(&p, n * sizeof(T));
  if (e != hipSuccess) throw Fail{TAPG_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e)};
  return static_cast<T*>(p);
}

template <typename T>
void dfree(T*& p) {
  if (p) (void)hipFree(p);
  p = nullptr;
}

// Column-major padded copy of a row-major rows x cols matrix, optionally transposed.
template <typename T>
std::vector<T> colmajor(const Mat& M, int ld, bool transpose_first) {
  const int R = transpose_first ? M.c : M.r;
  const int C = transpose_first ? M.r : M.c;
  std::vector<T> out((size_t)ld * C, T(0));
  for (int r = 0; r < R; ++r)
    for (int k = 0; k < C; ++k)
      out[(size_t)k * ld + r] = (T)(transpose_first ? M(k, r) : M(r, k));
  return out;
}

// Set-up copies are synchronous: the host vectors are often temporaries.
template <typename T>
T* upload(const std::vector<T>& v, hipStream_t st) {
  T* d = dmalloc<T>(v.size());
  TAPG_HIP(hipStreamSynchronize(st));
  TAPG_HIP(hipMemcpy(d, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  return d;
}

template <typename T>
std::vector<T> padvec(const std::vector<double>& v, int ld) {
  std::vector<T> o(ld, T(0));
  for (size_t i = 0; i < v.size(); ++i) o[i] = (T)v[i];
  return o;
}

template <typename T>
void init_net(tapg_solver_s* S, NetDev<T>& d) {
  const NetworkHost& h = S->net;
  hipStream_t st = S->stream;
  d.At = upload(colmajor<T>(h.A, S->LDX, true), st);
  d.Bt = upload(colmajor<T>(h.B, S->LDU, true), st);
  d.A = upload(colmajor<T>(h.A, S->LDX, false), st);
  d.B = upload(colmajor<T>(h.B, S->LDX, false), st);
  d.xmin = upload(padvec<T>(h.xmin, S->LDX), st);
  d.xmax = upload(padvec<T>(h.xmax, S->LDX), st);
  d.xs = upload(padvec<T>(h.xs, S->LDX), st);
  d.umin = upload(padvec<T>(h.umin, S->LDU), st);
  d.umax = upload(padvec<T>(h.umax, S->LDU), st);
}

template <typename T>
void free_net(NetDev<T>& d) {
  dfree(d.At); dfree(d.Bt); dfree(d.A); dfree(d.B);
  dfree(d.xmin); dfree(d.xmax); dfree(d.xs); dfree(d.umin); dfree(d.umax);
  dfree(d.F); dfree(d.Kb);
}

// Nodes per tile: the largest NB in {8, 4, 2, 1} that keeps at least 256
// tiles in the stage and fits the forward kernel's LDS in 64 KiB.
int pick_nb(int width, size_t elem, int LDX, int LDU, int LDY) {
  for (int nb : {8, 4, 2}) {
    const size_t lds = (size_t)(2 * LDX + 2 * LDU + kThreads + 2 * LDY) * nb * elem;
    if ((width + nb - 1) / nb >= 256 && lds <= 60 * 1024) return nb;
  }
  return 1;
}

template <typename T>
SweepArgs<T> make_args(tapg_solver_s* S, Slot& sl, const NetDev<T>& d, int mode) {
  SweepArgs<T> a{};
  a.nx = S->net.nx;
  a.nu = S->net.nu;
  a.LDX = S->LDX;
  a.LDU = S->LDU;
  a.LDY = S->LDY;
  a.mode = mode;
  a.anc = sl.d_anc;
  a.cbeg = sl.d_cbeg;
  a.cend = sl.d_cend;
  a.invp = static_cast<const T*>(sl.d_invp);
  a.At = d.At;
  a.Bt = d.Bt;
  a.A = d.A;
  a.B = d.B;
  a.xmin = d.xmin;
  a.xmax = d.xmax;
  a.xs = d.xs;
  a.umin = d.umin;
  a.umax = d.umax;
  a.Wx = (T)S->cfg.W_x;
  a.Ws = (T)S->cfg.W_s;
  a.kappa = static_cast<const T*>(sl.d_kappa);
  a.g = static_cast<const T*>(sl.d_g);
  a.pq = static_cast<const T*>(sl.d_pq);
  a.Y0 = static_cast<T*>(sl.d_Y0);
  a.Y1 = static_cast<T*>(sl.d_Y1);
  a.lam = static_cast<T*>(sl.d_lam);
  a.jv = static_cast<T*>(sl.d_j);
  a.u = static_cast<T*>(sl.d_u);
  a.x = static_cast<T*>(sl.d_x);
  a.ctl = sl.d_ctl;
  a.part = sl.d_part;
  return a;
}

template <typename T, int NB>
void launch_bwd(const SweepArgs<T>& a, int tiles, hipStream_t st) {
  const size_t lds = (size_t)(2 * a.LDX + 2 * a.LDU + kThreads) * NB * sizeof(T);
  hipLaunchKernelGGL((bwd_stage_kernel<T, NB>), dim3(tiles), dim3(kThreads), lds, st, a);
}

template <typename T, int NB>
void launch_fwd(const SweepArgs<T>& a, int tiles, hipStream_t st) {
  const size_t lds = (size_t)(2 * a.LDX + 2 * a.LDU + kThreads + 2 * a.LDY) * NB * sizeof(T);
  hipLaunchKernelGGL((fwd_stage_kernel<T, NB>), dim3(tiles), dim3(kThreads), lds, st, a);
}


template <typename T>
void launch_bwd_nb(int nb, const SweepArgs<T>& a, int tiles, hipStream_t st) {
  switch (nb) {
    case 8: launch_bwd<T, 8>(a, tiles, st); break;
    case 4: launch_bwd<T, 4>(a, tiles, st); break;
    case 2: launch_bwd<T, 2>(a, tiles, st); break;
    default: launch_bwd<T, 1>(a, tiles, st); break;
  }
}

template <typename T>
void launch_fwd_nb(int nb, const SweepArgs<T>& a, int tiles, hipStream_t st) {
  switch (nb) {
    case 8: launch_fwd<T, 8>(a, tiles, st); break;
    case 4: launch_fwd<T, 4>(a, tiles, st); break;
    case 2: launch_fwd<T, 2>(a, tiles, st); break;
    default: launch_fwd<T, 1>(a, tiles, st); break;
  }
}

// One APG iteration (mode 0) or one power-iteration step (mode 1) on the
// solver's stream: backward stages, forward stages, end-of-step kernel.
// Event pair index for the timed path (-1: untimed).
struct TimedCursor {
  int next = 0;
  std::vector<int> kind;  // kind of each recorded pair
};

template <typename T>
void enqueue_iteration(tapg_solver_s* S, Slot& sl, const NetDev<T>& d, int mode,
                       TimedCursor* tc = nullptr) {
  SweepArgs<T> a = make_args<T>(S, sl, d, mode);
  if (mode == 1) {
    a.Y0 = static_cast<T*>(sl.d_P0);
    a.Y1 = static_cast<T*>(sl.d_P1);
  }
  const size_t fstride = (size_t)S->LDU * S->LDU;
  hipStream_t st = S->stream;
  for (int pass = 0; pass < 2; ++pass) {
    for (int q = 0; q < sl.N; ++q) {
      const int s = pass == 0 ? sl.N - 1 - q : q;
      a.s = s;
      a.node0 = sl.node_offset[s];
      a.count = sl.node_offset[s + 1] - sl.node_offset[s];
      a.tile_base = sl.tile_offset[s];
      a.F = d.F + s * fstride;
      a.Kb = d.Kb + s * fstride;
      if (tc) (void)hipEventRecord(S->tev[2 * tc->next], st);
      if (pass == 0)
        launch_bwd_nb<T>(sl.nb_of_stage[s], a, sl.tiles_of_stage[s], st);
      else
        launch_fwd_nb<T>(sl.nb_of_stage[s], a, sl.tiles_of_stage[s], st);
      if (tc) {
        (void)hipEventRecord(S->tev[2 * tc->next + 1], st);
        tc->kind.push_back(pass);
        tc->next++;
      }
    }
  }
  if (mode == 0) {
    if (tc) (void)hipEventRecord(S->tev[2 * tc->next], st);
    hipLaunchKernelGGL(iter_end_kernel, dim3(1), dim3(1), 0, st, sl.d_ctl, sl.d_hist);
    if (tc) {
      (void)hipEventRecord(S->tev[2 * tc->next + 1], st);
      tc->kind.push_back(2);
      tc->next++;
    }
  } else
    hipLaunchKernelGGL(power_end_kernel, dim3(1), dim3(kThreads), 0, st, sl.d_ctl,
                       (const double*)sl.d_part, sl.total_tiles);
}

template <typename T>
const NetDev<T>& net_of(tapg_solver_s* S);
template <>
const NetDev<double>& net_of<double>(tapg_solver_s* S) { return S->d64; }
template <>
const NetDev<float>& net_of<float>(tapg_solver_s* S) { return S->d32; }

template <typename T>
std::vector<T> pad_rows(const double* src, int rows, int cols, int ld) {
  std::vector<T> out((size_t)rows * ld, T(0));
  for (int i = 0; i < rows; ++i)
    for (int j = 0; j < cols; ++j) out[(size_t)i * ld + j] = (T)src[(size_t)i * cols + j];
  return out;
}

template <typename T>
void solve_impl(tapg_solver_s* S, const TreeHost& t, Slot& sl, const double* p,
                const double* q, bool warm, double gamma, tapg_result& res) {
  const NetworkHost& h = S->net;
  hipStream_t st = S->stream;
  const int LDX = S->LDX, LDU = S->LDU, LDY = S->LDY;
  const int K = t.K;
  // initial condition
  std::vector<double> pq64(LDX + LDU, 0.0);
  for (int i = 0; i < h.nx; ++i) pq64[i] = p[i];
  for (int i = 0; i < h.nu; ++i) pq64[LDX + i] = q[i];
  std::vector<T> pqT(pq64.begin(), pq64.end());
  TAPG_HIP(hipMemcpyAsync(sl.d_pq64, pq64.data(), pq64.size() * 8, hipMemcpyHostToDevice, st));
  TAPG_HIP(hipMemcpyAsync(sl.d_pq, pqT.data(), pqT.size() * sizeof(T), hipMemcpyHostToDevice, st));
  // control block
  DevCtl c{};
  c.max_iter = S->cfg.max_iter;
  c.tol = S->cfg.tol;
  c.gamma = gamma;
  c.theta = 1.0;
  c.theta_prev = 1.0;
  c.beta = 0.0;
  TAPG_HIP(hipMemcpyAsync(sl.d_ctl, &c, sizeof(c), hipMemcpyHostToDevice, st));
  // dual start
  const size_t ybytes = (size_t)K * LDY * sizeof(T);
  if (warm && sl.has_dual) {
    void* src = sl.last_iter_parity ? sl.d_Y1 : sl.d_Y0;
    void* dst = sl.last_iter_parity ? sl.d_Y0 : sl.d_Y1;
    TAPG_HIP(hipMemcpyAsync(dst, src, ybytes, hipMemcpyDeviceToDevice, st));
  } else {
    TAPG_HIP(hipMemsetAsync(sl.d_Y0, 0, ybytes, st));
    TAPG_HIP(hipMemsetAsync(sl.d_Y1, 0, ybytes, st));
  }
  TAPG_HIP(hipEventRecord(S->ev0, st));
  // data step
  {
    const size_t lds = (size_t)(h.nd + 2 * LDU) * sizeof(double);
    hipLaunchKernelGGL((data_step_kernel<T>), dim3(K), dim3(kThreads), lds, st, h.nx, h.nu, h.nd,
                       LDX, LDU, (const int*)sl.d_stage, (const double*)sl.d_prob64,
                       (const double*)sl.d_demand, (const double*)sl.d_price,
                       (const double*)S->dx.Pd, (const double*)S->dx.Gd,
                       (const double*)S->dx.Gbar, (const double*)S->d64.F,
                       (const double*)S->dx.alpha0, (const double*)S->dx.cE, S->cfg.W_alpha,
                       static_cast<T*>(sl.d_kappa), static_cast<T*>(sl.d_g));
    TAPG_HIP(hipGetLastError());
  }
  // iterations, in chunks of check_every with a host check between chunks
  const int chunk = std::max(1, std::min(S->cfg.check_every, S->cfg.max_iter));
  const NetDev<T>& d = net_of<T>(S);
  if (S->use_graph && !S->time_kernels && (sl.graph == nullptr || sl.graph_iters != chunk)) {
    if (sl.graph) (void)hipGraphExecDestroy(sl.graph);
    sl.graph = nullptr;
    hipGraph_t g = nullptr;
    TAPG_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    for (int i = 0; i < chunk; ++i) enqueue_iteration<T>(S, sl, d, 0);
    TAPG_HIP(hipStreamEndCapture(st, &g));
    hipError_t e = hipGraphInstantiate(&sl.graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) throw Fail{TAPG_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e)};
    sl.graph_iters = chunk;
  }
  DevCtl hc{};
  int launched = 0;
  const bool timed = S->time_kernels;
  if (timed) {
    const size_t need = (size_t)2 * chunk * (2 * sl.N + 1);
    while (S->tev.size() < need) {
      hipEvent_t e;
      TAPG_HIP(hipEventCreate(&e));
      S->tev.push_back(e);
    }
    for (int k = 0; k < 3; ++k) {
      S->kt_ms[k] = 0.0;
      S->kt_n[k] = 0;
    }
  }
  while (true) {
    if (timed) {
      // one iteration per check so that launches after the stop are not timed
      TimedCursor tc;
      for (int i = 0; i < chunk; ++i) {
        enqueue_iteration<T>(S, sl, d, 0, &tc);
        TAPG_HIP(hipMemcpyAsync(&hc, sl.d_ctl, sizeof(hc), hipMemcpyDeviceToHost, st));
        TAPG_HIP(hipStreamSynchronize(st));
        if (hc.done && hc.iter <= launched + i) {  // this iteration was a no-op
          tc.kind.resize(tc.kind.size() - (2 * sl.N + 1));
          tc.next -= 2 * sl.N + 1;
          break;
        }
        if (hc.done) break;
      }
      TAPG_HIP(hipGetLastError());
      for (int k = 0; k < tc.next; ++k) {
        float ms = 0.f;
        TAPG_HIP(hipEventElapsedTime(&ms, S->tev[2 * k], S->tev[2 * k + 1]));
        S->kt_ms[tc.kind[k]] += ms;
        S->kt_n[tc.kind[k]] += 1;
      }
    } else if (S->use_graph) {
      TAPG_HIP(hipGraphLaunch(sl.graph, st));
    } else {
      for (int i = 0; i < chunk; ++i) enqueue_iteration<T>(S, sl, d, 0);
      TAPG_HIP(hipGetLastError());
    }
    launched += chunk;
    TAPG_HIP(hipMemcpyAsync(&hc, sl.d_ctl, sizeof(hc), hipMemcpyDeviceToHost, st));
    TAPG_HIP(hipStreamSynchronize(st));
    if (hc.done || launched >= S->cfg.max_iter) break;
  }
  TAPG_HIP(hipEventRecord(S->ev1, st));
  // cost and violations of the final primal iterate
  {
    const size_t lds = (size_t)(2 * LDU + LDX + h.nd) * sizeof(double);
    hipLaunchKernelGGL((cost_kernel<T>), dim3(K), dim3(kThreads), lds, st, h.nx, h.nu, h.nd, h.ns,
                       LDX, LDU, (const int*)sl.d_anc, (const double*)sl.d_prob64,
                       (const double*)sl.d_demand, (const double*)sl.d_price,
                       (const T*)sl.d_u, (const T*)sl.d_x, (const double*)sl.d_pq64,
                       (const double*)S->d64.A, (const double*)S->d64.B,
                       (const double*)S->dx.Gd, (const double*)S->dx.E,
                       (const double*)S->dx.Ed, (const double*)S->dx.Wu,
                       (const double*)S->dx.alpha0, (const double*)S->dx.cE,
                       (const double*)S->d64.xmin, (const double*)S->d64.xmax,
                       (const double*)S->d64.xs, (const double*)S->d64.umin,
                       (const double*)S->d64.umax, S->cfg.W_alpha, S->cfg.W_x, S->cfg.W_s,
                       sl.d_part);
    hipLaunchKernelGGL(cost_reduce_kernel, dim3(1), dim3(kThreads), 0, st,
                       (const double*)sl.d_part, K, S->dx.red);
    TAPG_HIP(hipGetLastError());
  }
  double red[3];
  TAPG_HIP(hipMemcpyAsync(red, S->dx.red, sizeof(red), hipMemcpyDeviceToHost, st));
  TAPG_HIP(hipStreamSynchronize(st));
  float ms = 0.f;
  TAPG_HIP(hipEventElapsedTime(&ms, S->ev0, S->ev1));
  res.iters = hc.iter;
  res.converged = hc.converged;
  res.primal_res = hc.last_res;
  res.cost = red[0];
  res.viol_box = red[1];
  res.viol_eq = red[2];
  res.gamma = gamma;
  res.solve_ms = ms;
  sl.has_dual = true;
  sl.last_iter_parity = hc.iter & 1;
  sl.last = res;
  sl.has_result = true;
  if (hc.numeric) throw Fail{TAPG_ENUMERIC, "non-finite dual residual (diverging iterates; infeasible data or step size too large)"};
}

template <typename T>
double power_impl(tapg_solver_s* S, const TreeHost& t, Slot& sl, int iters) {
  const NetworkHost& h = S->net;
  hipStream_t st = S->stream;
  const int K = t.K, LDX = S->LDX, LDY = S->LDY;
  if (!sl.d_P0) {
    sl.d_P0 = dmalloc<T>((size_t)K * LDY);
    sl.d_P1 = dmalloc<T>((size_t)K * LDY);
    TAPG_HIP(hipMemsetAsync(sl.d_P1, 0, (size_t)K * LDY * sizeof(T), st));
  }
  std::vector<T> v((size_t)K * LDY, T(0));
  std::mt19937_64 rng(0x5eed1234ull);
  std::normal_distribution<double> nd(0.0, 1.0);
  double nrm2 = 0.0;
  for (int n = 0; n < K; ++n) {
    T* yn = v.data() + (size_t)n * LDY;
    for (int i = 0; i < h.nx; ++i) { yn[i] = (T)nd(rng); nrm2 += (double)yn[i] * yn[i]; }
    for (int i = 0; i < h.nx; ++i) { yn[LDX + i] = (T)nd(rng); nrm2 += (double)yn[LDX + i] * yn[LDX + i]; }
    for (int i = 0; i < h.nu; ++i) { yn[2 * LDX + i] = (T)nd(rng); nrm2 += (double)yn[2 * LDX + i] * yn[2 * LDX + i]; }
  }
  TAPG_HIP(hipMemcpyAsync(sl.d_P0, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, st));
  DevCtl c{};
  c.pw_scale = 1.0 / std::sqrt(nrm2);
  c.max_iter = iters + 1;
  TAPG_HIP(hipMemcpyAsync(sl.d_ctl, &c, sizeof(c), hipMemcpyHostToDevice, st));
  const NetDev<T>& d = net_of<T>(S);
  for (int i = 0; i < iters; ++i) enqueue_iteration<T>(S, sl, d, 1);
  TAPG_HIP(hipGetLastError());
  DevCtl hc{};
  TAPG_HIP(hipMemcpyAsync(&hc, sl.d_ctl, sizeof(hc), hipMemcpyDeviceToHost, st));
  TAPG_HIP(hipStreamSynchronize(st));
  return hc.L;
}

}  // namespace

// ---------------------------------------------------------------------------
// Exported device-layer entry points
// ---------------------------------------------------------------------------
void dev_init(tapg_solver_s* S) {
  TAPG_HIP(hipSetDevice(S->device));
  if (S->stream == nullptr) {
    TAPG_HIP(hipStreamCreateWithFlags(&S->stream, hipStreamNonBlocking));
    S->own_stream = true;
  }
  TAPG_HIP(hipEventCreate(&S->ev0));
  TAPG_HIP(hipEventCreate(&S->ev1));
  const NetworkHost& h = S->net;
  hipStream_t st = S->stream;
  init_net<double>(S, S->d64);
  if (S->fp32) init_net<float>(S, S->d32);
  S->dx.Gd = upload(colmajor<double>(h.Gd, S->LDX, false), st);
  S->dx.Pd = upload(colmajor<double>(h.Pd, S->LDU, false), st);
  S->dx.E = upload(h.E.a.empty() ? std::vector<double>(1, 0.0) : h.E.a, st);
  S->dx.Ed = upload(h.Ed.a.empty() ? std::vector<double>(1, 0.0) : h.Ed.a, st);
  S->dx.Wu = upload(colmajor<double>(Mat::from(S->Wu.data(), h.nu, h.nu), S->LDU, false), st);
  S->dx.alpha0 = upload(padvec<double>(S->alpha0, S->LDU), st);
  S->dx.cE = upload(padvec<double>(S->cE, S->LDU), st);
  S->dx.red = dmalloc<double>(8);
  TAPG_HIP(hipStreamSynchronize(st));
}

void dev_free_slot(Slot& sl) {
  if (sl.graph) (void)hipGraphExecDestroy(sl.graph);
  sl.graph = nullptr;
  dfree(sl.d_anc); dfree(sl.d_cbeg); dfree(sl.d_cend); dfree(sl.d_stage);
  dfree(sl.d_prob64); dfree(sl.d_invp); dfree(sl.d_demand); dfree(sl.d_price);
  dfree(sl.d_kappa); dfree(sl.d_g); dfree(sl.d_pq); dfree(sl.d_pq64);
  dfree(sl.d_P0); dfree(sl.d_P1);
  dfree(sl.d_Y0); dfree(sl.d_Y1); dfree(sl.d_lam); dfree(sl.d_j); dfree(sl.d_u); dfree(sl.d_x);
  dfree(sl.d_ctl); dfree(sl.d_hist); dfree(sl.d_part);
}

void dev_release(tapg_solver_s* S) {
  if (S->device >= 0) (void)hipSetDevice(S->device);
  if (S->stream) (void)hipStreamSynchronize(S->stream);
  for (auto& kv : S->slots) dev_free_slot(kv.second);
  S->slots.clear();
  free_net(S->d64);
  free_net(S->d32);
  dfree(S->dx.Gd); dfree(S->dx.Pd); dfree(S->dx.Gbar); dfree(S->dx.E); dfree(S->dx.Ed);
  dfree(S->dx.Wu); dfree(S->dx.alpha0); dfree(S->dx.cE); dfree(S->dx.red);
  for (hipEvent_t e : S->tev) (void)hipEventDestroy(e);
  S->tev.clear();
  if (S->ev0) (void)hipEventDestroy(S->ev0);
  if (S->ev1) (void)hipEventDestroy(S->ev1);
  S->ev0 = S->ev1 = nullptr;
  if (S->own_stream && S->stream) (void)hipStreamDestroy(S->stream);
  S->stream = nullptr;
}

void dev_upload_factors(tapg_solver_s* S) {
  TAPG_HIP(hipSetDevice(S->device));
  const int nu = S->net.nu, LDU = S->LDU, N = S->N;
  hipStream_t st = S->stream;
  auto pack = [&](const std::vector<double>& src, auto tag) {
    using T = decltype(tag);
    std::vector<T> out((size_t)N * LDU * LDU, T(0));
    for (int s = 0; s < N; ++s)
      for (int r = 0; r < nu; ++r)
        for (int k = 0; k < nu; ++k)
          out[(size_t)s * LDU * LDU + (size_t)k * LDU + r] =
              (T)src[(size_t)s * nu * nu + (size_t)r * nu + k];
    return out;
  };
  dfree(S->d64.F); dfree(S->d64.Kb); dfree(S->dx.Gbar);
  S->d64.F = upload(pack(S->Fbar, double{}), st);
  S->d64.Kb = upload(pack(S->Kbar, double{}), st);
  S->dx.Gbar = upload(pack(S->Gbar, double{}), st);
  if (S->fp32) {
    dfree(S->d32.F); dfree(S->d32.Kb);
    S->d32.F = upload(pack(S->Fbar, float{}), st);
    S->d32.Kb = upload(pack(S->Kbar, float{}), st);
  }
  // every cached iteration graph refers to the old factor buffers
  for (auto& kv : S->slots) {
    if (kv.second.graph) (void)hipGraphExecDestroy(kv.second.graph);
    kv.second.graph = nullptr;
  }
  TAPG_HIP(hipStreamSynchronize(st));
}

Slot& dev_slot(tapg_solver_s* S, const TreeHost& t) {
  TAPG_HIP(hipSetDevice(S->device));
  hipStream_t st = S->stream;
  auto it = S->slots.find(t.uid);
  if (it == S->slots.end()) {
    Slot sl;
    sl.tree_uid = t.uid;
    sl.K = t.K;
    sl.N = t.N;
    sl.elem = S->fp32 ? sizeof(float) : sizeof(double);
    const int K = t.K, LDX = S->LDX, LDU = S->LDU, LDY = S->LDY;
    const size_t e = sl.elem;
    auto dalloc = [&](size_t n) {
      void* p = nullptr;
      hipError_t er = hipMalloc(&p, std::max<size_t>(n, 1) * e);
      if (er != hipSuccess) throw Fail{TAPG_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(er)};
      TAPG_HIP(hipMemsetAsync(p, 0, std::max<size_t>(n, 1) * e, st));
      return p;
    };
    try {
      sl.d_anc = upload(t.anc, st);
      sl.d_cbeg = upload(t.cbeg, st);
      sl.d_cend = upload(t.cend, st);
      sl.d_stage = upload(t.stage, st);
      sl.d_prob64 = upload(t.prob, st);
      if (S->fp32) {
        std::vector<float> ip(K);
        for (int n = 0; n < K; ++n) ip[n] = (float)(1.0 / t.prob[n]);
        sl.d_invp = upload(ip, st);
      } else {
        std::vector<double> ip(K);
        for (int n = 0; n < K; ++n) ip[n] = 1.0 / t.prob[n];
        sl.d_invp = upload(ip, st);
      }
      sl.d_demand = dmalloc<double>((size_t)K * t.nd);
      sl.d_price = dmalloc<double>(K);
      sl.d_kappa = dalloc((size_t)K * LDU);
      sl.d_g = dalloc((size_t)K * LDX);
      sl.d_pq = dalloc(LDX + LDU);
      sl.d_pq64 = dmalloc<double>(LDX + LDU);
      sl.d_Y0 = dalloc((size_t)K * LDY);
      sl.d_Y1 = dalloc((size_t)K * LDY);
      sl.d_lam = dalloc((size_t)K * LDX);
      sl.d_j = dalloc((size_t)K * LDU);
      sl.d_u = dalloc((size_t)K * LDU);
      sl.d_x = dalloc((size_t)K * LDX);
      sl.d_ctl = dmalloc<DevCtl>(1);
      sl.hist_cap = std::max(1, S->cfg.max_iter);
      sl.d_hist = dmalloc<double>(sl.hist_cap);
      sl.node_offset = t.offset;
      sl.nb_of_stage.resize(t.N);
      sl.tiles_of_stage.resize(t.N);
      sl.tile_offset.resize(t.N + 1);
      int tot = 0;
      for (int s = 0; s < t.N; ++s) {
        const int width = t.mu[s];
        const int nb = pick_nb(width, e, LDX, LDU, LDY);
        sl.nb_of_stage[s] = nb;
        sl.tiles_of_stage[s] = (width + nb - 1) / nb;
        sl.tile_offset[s] = tot;
        tot += sl.tiles_of_stage[s];
      }
      sl.tile_offset[t.N] = tot;
      sl.total_tiles = tot;
      sl.part_cap = std::max(tot, 4 * K);
      sl.d_part = dmalloc<double>(sl.part_cap);
    } catch (...) {
      dev_free_slot(sl);
      throw;
    }
    it = S->slots.emplace(t.uid, std::move(sl)).first;
  }
  Slot& sl = it->second;
  if (sl.hist_cap < S->cfg.max_iter) {
    dfree(sl.d_hist);
    sl.hist_cap = S->cfg.max_iter;
    sl.d_hist = dmalloc<double>(sl.hist_cap);
    if (sl.graph) (void)hipGraphExecDestroy(sl.graph);
    sl.graph = nullptr;
  }
  if (sl.data_version != t.version) {
    TAPG_HIP(hipMemcpyAsync(sl.d_demand, t.demand.data(), t.demand.size() * 8,
                            hipMemcpyHostToDevice, st));
    TAPG_HIP(hipMemcpyAsync(sl.d_price, t.price.data(), t.price.size() * 8,
                            hipMemcpyHostToDevice, st));
    sl.data_version = t.version;
  }
  TAPG_HIP(hipStreamSynchronize(st));
  return sl;
}

void dev_solve(tapg_solver_s* S, const TreeHost& t, Slot& sl, const double* p, const double* q,
               bool warm, double gamma, tapg_result& res) {
  TAPG_HIP(hipSetDevice(S->device));
  if (S->fp32)
    solve_impl<float>(S, t, sl, p, q, warm, gamma, res);
  else
    solve_impl<double>(S, t, sl, p, q, warm, gamma, res);
}

double dev_power(tapg_solver_s* S, const TreeHost& t, Slot& sl, int iters) {
  TAPG_HIP(hipSetDevice(S->device));
  return S->fp32 ? power_impl<float>(S, t, sl, iters) : power_impl<double>(S, t, sl, iters);
}

namespace {
template <typename T>
void download_rows(const void* dsrc, int rows, int ld, int cols, double* out, hipStream_t st) {
  std::vector<T> tmp((size_t)rows * ld);
  TAPG_HIP(hipMemcpyAsync(tmp.data(), dsrc, tmp.size() * sizeof(T), hipMemcpyDeviceToHost, st));
  TAPG_HIP(hipStreamSynchronize(st));
  for (int i = 0; i < rows; ++i)
    for (int j = 0; j < cols; ++j) out[(size_t)i * cols + j] = (double)tmp[(size_t)i * ld + j];
}

template <typename T>
void get_dual_impl(tapg_solver_s* S, Slot& sl, double* y) {
  const int nx = S->net.nx, nu = S->net.nu, LDX = S->LDX, LDY = S->LDY;
  const int m = 2 * nx + nu;
  std::vector<T> tmp((size_t)sl.K * LDY);
  const void* src = sl.last_iter_parity ? sl.d_Y1 : sl.d_Y0;
  TAPG_HIP(hipMemcpyAsync(tmp.data(), src, tmp.size() * sizeof(T), hipMemcpyDeviceToHost, S->stream));
  TAPG_HIP(hipStreamSynchronize(S->stream));
  for (int n = 0; n < sl.K; ++n) {
    const T* yn = tmp.data() + (size_t)n * LDY;
    double* o = y + (size_t)n * m;
    for (int i = 0; i < nx; ++i) o[i] = yn[i];
    for (int i = 0; i < nx; ++i) o[nx + i] = yn[LDX + i];
    for (int i = 0; i < nu; ++i) o[2 * nx + i] = yn[2 * LDX + i];
  }
}

template <typename T>
void set_dual_impl(tapg_solver_s* S, Slot& sl, const double* y) {
  const int nx = S->net.nx, nu = S->net.nu, LDX = S->LDX, LDY = S->LDY;
  const int m = 2 * nx + nu;
  std::vector<T> tmp((size_t)sl.K * LDY, T(0));
  for (int n = 0; n < sl.K; ++n) {
    T* yn = tmp.data() + (size_t)n * LDY;
    const double* s = y + (size_t)n * m;
    for (int i = 0; i < nx; ++i) yn[i] = (T)s[i];
    for (int i = 0; i < nx; ++i) yn[LDX + i] = (T)s[nx + i];
    for (int i = 0; i < nu; ++i) yn[2 * LDX + i] = (T)s[2 * nx + i];
  }
  TAPG_HIP(hipMemcpyAsync(sl.d_Y0, tmp.data(), tmp.size() * sizeof(T), hipMemcpyHostToDevice, S->stream));
  TAPG_HIP(hipStreamSynchronize(S->stream));
  sl.has_dual = true;
  sl.last_iter_parity = 0;
}
}  // namespace

void dev_get_primal(tapg_solver_s* S, Slot& sl, double* u, double* x) {
  TAPG_HIP(hipSetDevice(S->device));
  if (S->fp32) {
    if (u) download_rows<float>(sl.d_u, sl.K, S->LDU, S->net.nu, u, S->stream);
    if (x) download_rows<float>(sl.d_x, sl.K, S->LDX, S->net.nx, x, S->stream);
  } else {
    if (u) download_rows<double>(sl.d_u, sl.K, S->LDU, S->net.nu, u, S->stream);
    if (x) download_rows<double>(sl.d_x, sl.K, S->LDX, S->net.nx, x, S->stream);
  }
}

void dev_get_root_input(tapg_solver_s* S, Slot& sl, double* u0) {
  TAPG_HIP(hipSetDevice(S->device));
  if (S->fp32)
    download_rows<float>(sl.d_u, 1, S->LDU, S->net.nu, u0, S->stream);
  else
    download_rows<double>(sl.d_u, 1, S->LDU, S->net.nu, u0, S->stream);
}

void dev_get_dual(tapg_solver_s* S, Slot& sl, double* y) {
  TAPG_HIP(hipSetDevice(S->device));
  if (S->fp32) get_dual_impl<float>(S, sl, y); else get_dual_impl<double>(S, sl, y);
}

void dev_set_dual(tapg_solver_s* S, Slot& sl, const double* y) {
  TAPG_HIP(hipSetDevice(S->device));
  if (S->fp32) set_dual_impl<float>(S, sl, y); else set_dual_impl<double>(S, sl, y);
}

void dev_set_kernel_timing(tapg_solver_s* S, bool on) { S->time_kernels = on; }

int dev_get_history(tapg_solver_s* S, Slot& sl, double* hbuf, int n) {
  TAPG_HIP(hipSetDevice(S->device));
  const int m = std::min(n, sl.has_result ? sl.last.iters : 0);
  if (m > 0) {
    TAPG_HIP(hipMemcpyAsync(hbuf, sl.d_hist, (size_t)m * 8, hipMemcpyDeviceToHost, S->stream));
    TAPG_HIP(hipStreamSynchronize(S->stream));
  }
  return m;
}

}  // namespace tapg
