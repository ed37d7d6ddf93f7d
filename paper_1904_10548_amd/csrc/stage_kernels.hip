// Per-stage sweep kernels for gfx950 and the small per-solve kernels (data
// step, cost, end of iteration, end of a power-iteration step).
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

#include "kernels.h"

namespace tapg {


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
// block writes z = -(x_n, x_n, u_n) and the tile's |z|^2 instead; in
// evaluation mode (2) it stops after u_n and x_n.
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
  const int LDX = a.LDX, LDU = a.LDU, LDY = a.LDY;

  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* sUp = reinterpret_cast<T*>(smem_raw);  // parent inputs
  T* sXp = sUp + NB * LDU;                  // parent states
  T* sUn = sXp + NB * LDX;                  // u_n
  T* sXn = sUn + NB * LDU;                  // x_n
  T* red = sXn + NB * LDX;                  // NB * 256
  // the prox runs in FP64 whatever T (with FP32 sweeps: w and x widened, y+
  // rounded to T once, the residual the FP64 split residual of those inputs)
  double* sW = reinterpret_cast<double*>(red + NB * kThreads);  // w (blocks 1, 2)
  double* sR = sW + NB * LDY;                                   // r (blocks 1, 2)
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
  if (a.mode == 2) return;  // evaluation of x_hat(w) only: no dual update

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
        const double w = (double)wext(yc[i], yn[i], beta);
        const double v = w + gam64 * (double)xi;
        const double zz = v / gam64;
        const double pz = blk == 0 ? fmin(fmax(zz, (double)a.xmin[k]), (double)a.xmax[k])
                                   : fmax(zz, (double)a.xs[k]);
        const double rr = v - gam64 * pz;
        if (blk == 0)
          s1 += rr * rr;
        else
          s2 += rr * rr;
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
        const double w = (double)wext(yc[i], yn[i], beta);
        const double v = w + gam64 * (double)ui;
        const double t = fmin(fmax(v / gam64, (double)a.umin[k]), (double)a.umax[k]);
        const double y = v - gam64 * t;
        yn[i] = (T)y;
        double d = fabs(y - w) / gam64;
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
    const double sc1 = n1 > (double)a.Wx ? (double)a.Wx / n1 : 1.0;
    const double sc2 = n2 > (double)a.Ws ? (double)a.Ws / n2 : 1.0;
    for (int i = l; i < 2 * LDX; i += TPN) {
      const int blk = i < LDX ? 0 : 1;
      const int k = i - blk * LDX;
      if (k >= a.nx) continue;
      const double y = sR[b * LDY + i] * (blk == 0 ? sc1 : sc2);
      yn[i] = (T)y;
      double d = fabs(y - sW[b * LDY + i]) / gam64;
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

// End of one APG iteration (ctl_advance), one thread per tree of the slot, in
// a launch of its own after the last forward launch (the sweep workgroups
// then need no device-wide fence): from the states in prev into out.
__global__ void iter_end_kernel(const DevCtl* prev, DevCtl* out, double* hist, int ntrees,
                                int hist_stride) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= ntrees) return;
  const DevCtl c = prev[k];  // the whole block in one round of loads
  bool record;
  double res = 0.0;
  const DevCtl n = ctl_advance(c, &record, &res);
  if (record) hist[(size_t)k * hist_stride + c.iter] = res;
  out[k] = n;
}

// A bounded wait of `ticks` periods of the device's constant-rate clock (one
// thread): holds a stream while the host enqueues the work behind it.
__global__ void hold_kernel(long long ticks) {
  const long long t0 = wall_clock64();
  while (wall_clock64() - t0 < ticks) __builtin_amdgcn_s_sleep(32);
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
//   kappa_n = p_n (Gammabar_s ubar_n - Fbar_s c_n / 2),  g_n = Gd d_n,
// and, for the scan form of the sweeps (kperp != nullptr), the part of kappa_n
// outside the range of Pi:  kperp_n = kappa_n - Pi kappa_n = E'(G kappa_n)
// with G = (E E')^{-1} E (Gm, ns x nu row-major; E row-major).
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kThreads) void data_step_kernel(
    int nx, int nu, int nd, int LDX, int LDU, const int* stage, const double* prob,
    const double* demand, const double* price, const double* Pd, const double* Gd,
    const double* Gbar, const double* Fbar, const double* alpha0, const double* cE,
    double W_alpha, T* kappa, T* g, int ns, const double* Gm, const double* E, T* kperp) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* sD = reinterpret_cast<double*>(smem_raw);
  double* sUb = sD + nd;
  double* sC = sUb + LDU;
  double* sK = sC + LDU;   // kappa_n in FP64 (scan form only)
  double* sGk = sK + LDU;  // G kappa_n
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
    const double kv = pn * (gu - 0.5 * fc);
    kappa[(size_t)n * LDU + r] = (T)kv;
    if (kperp) sK[r] = kv;
  }
  if (kperp) {
    __syncthreads();
    for (int k = threadIdx.x; k < ns; k += kThreads) {
      double acc = 0.0;
      for (int r = 0; r < nu; ++r) acc += Gm[(size_t)k * nu + r] * sK[r];
      sGk[k] = acc;
    }
    __syncthreads();
    for (int r = threadIdx.x; r < nu; r += kThreads) {
      double acc = 0.0;
      for (int k = 0; k < ns; ++k) acc += E[(size_t)k * nu + r] * sGk[k];
      kperp[(size_t)n * LDU + r] = (T)acc;
    }
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
  // the root of tree k (ancestor -1 - k) starts from that tree's (p, q)
  const double* pqn = pq + (par < 0 ? (size_t)(-par - 1) * (LDX + LDU) : 0);
  for (int i = threadIdx.x; i < nu; i += kThreads) {
    const double un = (double)u[(size_t)n * LDU + i];
    const double up = par >= 0 ? (double)u[(size_t)par * LDU + i] : pqn[LDX + i];
    sU[i] = un;
    sDu[i] = un - up;
  }
  for (int i = threadIdx.x; i < nx; i += kThreads)
    sXp[i] = par >= 0 ? (double)x[(size_t)par * LDX + i] : pqn[i];
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


// Per-tree sums of the per-node cost terms of a forest: block k walks tree
// k's node range of every stage (tstart[s * (ntrees + 1) + k ..]).
__global__ __launch_bounds__(kThreads) void cost_reduce_forest_kernel(const double* part,
                                                                      const int* tstart, int N,
                                                                      int ntrees, double* out) {
  __shared__ double red[kThreads];
  const int k = blockIdx.x;
  double c = 0.0, vb = 0.0, ms = 0.0, dy = 0.0;
  for (int s = 0; s < N; ++s) {
    const int b = tstart[(size_t)s * (ntrees + 1) + k], e = tstart[(size_t)s * (ntrees + 1) + k + 1];
    for (int n = b + threadIdx.x; n < e; n += kThreads) {
      c += part[(size_t)n * 4 + 0];
      vb = fmax(vb, part[(size_t)n * 4 + 1]);
      ms = fmax(ms, part[(size_t)n * 4 + 2]);
      dy = fmax(dy, part[(size_t)n * 4 + 3]);
    }
  }
  c = block_sum(c, red);
  vb = block_max(vb, red);
  ms = block_max(ms, red);
  dy = block_max(dy, red);
  if (threadIdx.x == 0) {
    out[3 * k + 0] = c;
    out[3 * k + 1] = vb;
    out[3 * k + 2] = fmax(ms, dy);
  }
}

// Rows between a tree's own buffers and a forest's: gather (dst row r = src
// row idx[r]) or scatter (dst row idx[r] = src row r), `width` elements a row.
template <typename T>
__global__ __launch_bounds__(kThreads) void copy_rows_kernel(const T* src, int ld_src, T* dst,
                                                             int ld_dst, const int* idx, int rows,
                                                             int width, int scatter) {
  const int r = blockIdx.x;
  if (r >= rows) return;
  const size_t rs = scatter ? (size_t)r : (size_t)idx[r];
  const size_t rd = scatter ? (size_t)idx[r] : (size_t)r;
  for (int i = threadIdx.x; i < width; i += kThreads) dst[rd * ld_dst + i] = src[rs * ld_src + i];
}

__global__ __launch_bounds__(kThreads) void copy_row_sets_kernel(RowCopies c, const int* idx,
                                                                 int rows, int scatter) {
  const int r = blockIdx.x;
  if (r >= rows) return;
  const size_t rs = scatter ? (size_t)r : (size_t)idx[r];
  const size_t rd = scatter ? (size_t)idx[r] : (size_t)r;
  for (int q = 0; q < c.n; ++q) {
    if (c.bytes[q] == 8) {
      const unsigned long long* s = static_cast<const unsigned long long*>(c.src[q]) + rs * c.ld_src[q];
      unsigned long long* d = static_cast<unsigned long long*>(c.dst[q]) + rd * c.ld_dst[q];
      for (int i = threadIdx.x; i < c.width[q]; i += kThreads) d[i] = s[i];
    } else {
      const unsigned* s = static_cast<const unsigned*>(c.src[q]) + rs * c.ld_src[q];
      unsigned* d = static_cast<unsigned*>(c.dst[q]) + rd * c.ld_dst[q];
      for (int i = threadIdx.x; i < c.width[q]; i += kThreads) d[i] = s[i];
    }
  }
}

// Averaged primal iterate (Sec. 4.3; the averaged sequence of accelerated
// dual gradient projection): ua = (1 - theta_nu) ua + theta_nu u_hat(w^nu), the
// same for x, with theta_nu of the iteration that just wrote u and x
// (theta_0 = 1 starts the average at the first iterate).  A stopped tree's
// average is left alone.
template <typename T>
__global__ __launch_bounds__(kThreads) void avg_kernel(const DevCtl* ctl, const T* u, const T* x,
                                                       T* ua, T* xa, size_t nu_el, size_t nx_el) {
  if (ctl->done) return;
  const double th = ctl->theta;
  const size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x;
  const T* src = i < nu_el ? u : x;
  T* dst = i < nu_el ? ua : xa;
  const size_t k = i < nu_el ? i : i - nu_el;
  if (i >= nu_el + nx_el) return;
  if (th >= 1.0)
    dst[k] = src[k];
  else
    dst[k] = (T)((1.0 - th) * (double)dst[k] + th * (double)src[k]);
}

// ---------------------------------------------------------------------------
// Launch wrappers
// ---------------------------------------------------------------------------
template <typename T, int NB>
void launch_bwd(const SweepArgs<T>& a, int tiles, hipStream_t st) {
  const size_t lds = (size_t)(2 * a.LDX + 2 * a.LDU + kThreads) * NB * sizeof(T);
  hipLaunchKernelGGL((bwd_stage_kernel<T, NB>), dim3(tiles), dim3(kThreads), lds, st, a);
}

template <typename T, int NB>
void launch_fwd(const SweepArgs<T>& a, int tiles, hipStream_t st) {
  const size_t lds = (size_t)(2 * a.LDX + 2 * a.LDU + kThreads) * NB * sizeof(T) +
                     (size_t)2 * a.LDY * NB * sizeof(double);
  hipLaunchKernelGGL((fwd_stage_kernel<T, NB>), dim3(tiles), dim3(kThreads), lds, st, a);
}


template <typename T>
void launch_bwd_stage(int nb, const SweepArgs<T>& a, int tiles, hipStream_t st) {
  switch (nb) {
    case 8: launch_bwd<T, 8>(a, tiles, st); break;
    case 4: launch_bwd<T, 4>(a, tiles, st); break;
    case 2: launch_bwd<T, 2>(a, tiles, st); break;
    default: launch_bwd<T, 1>(a, tiles, st); break;
  }
}

template <typename T>
void launch_fwd_stage(int nb, const SweepArgs<T>& a, int tiles, hipStream_t st) {
  switch (nb) {
    case 8: launch_fwd<T, 8>(a, tiles, st); break;
    case 4: launch_fwd<T, 4>(a, tiles, st); break;
    case 2: launch_fwd<T, 2>(a, tiles, st); break;
    default: launch_fwd<T, 1>(a, tiles, st); break;
  }
}


template <typename T>
void launch_avg(const DevCtl* ctl, const T* u, const T* x, T* ua, T* xa, size_t nu_el,
                size_t nx_el, hipStream_t st) {
  const size_t n = nu_el + nx_el;
  if (n == 0) return;
  hipLaunchKernelGGL((avg_kernel<T>), dim3((unsigned)((n + kThreads - 1) / kThreads)),
                     dim3(kThreads), 0, st, ctl, u, x, ua, xa, nu_el, nx_el);
}

void launch_iter_end(DevCtl* c, double* hist, int ntrees, int hist_stride, hipStream_t st) {
  launch_iter_end_from(c, c, hist, ntrees, hist_stride, st);
}

void launch_iter_end_from(const DevCtl* prev, DevCtl* out, double* hist, int ntrees,
                          int hist_stride, hipStream_t st) {
  const int nb = (ntrees + 63) / 64;
  hipLaunchKernelGGL(iter_end_kernel, dim3(nb), dim3(64), 0, st, prev, out, hist, ntrees,
                     hist_stride);
}

void launch_hold(long long ticks, hipStream_t st) {
  hipLaunchKernelGGL(hold_kernel, dim3(1), dim3(1), 0, st, ticks);
}

void launch_power_end(DevCtl* c, const double* part, int n, hipStream_t st) {
  hipLaunchKernelGGL(power_end_kernel, dim3(1), dim3(kThreads), 0, st, c, part, n);
}

template <typename T>
void launch_data_step(int K, int nx, int nu, int nd, int LDX, int LDU, const int* stage,
                      const double* prob, const double* demand, const double* price,
                      const double* Pd, const double* Gd, const double* Gbar, const double* Fbar,
                      const double* alpha0, const double* cE, double W_alpha, T* kappa, T* g,
                      int ns, const double* Gm, const double* E, T* kperp, hipStream_t st) {
  const size_t lds = (size_t)(nd + 3 * LDU + ns) * sizeof(double);
  hipLaunchKernelGGL((data_step_kernel<T>), dim3(K), dim3(kThreads), lds, st, nx, nu, nd, LDX,
                     LDU, stage, prob, demand, price, Pd, Gd, Gbar, Fbar, alpha0, cE, W_alpha,
                     kappa, g, ns, Gm, E, kperp);
}

template <typename T>
void launch_cost(int K, int nx, int nu, int nd, int ns, int LDX, int LDU, const int* anc,
                 const double* prob, const double* demand, const double* price, const T* u,
                 const T* x, const double* pq, const double* A, const double* B,
                 const double* Gd, const double* E, const double* Ed, const double* Wu,
                 const double* alpha0, const double* cE, const double* xmin, const double* xmax,
                 const double* xs, const double* umin, const double* umax, double W_alpha,
                 double W_x, double W_s, double* part, double* out, hipStream_t st) {
  const size_t lds = (size_t)(2 * LDU + LDX + nd) * sizeof(double);
  hipLaunchKernelGGL((cost_kernel<T>), dim3(K), dim3(kThreads), lds, st, nx, nu, nd, ns, LDX,
                     LDU, anc, prob, demand, price, u, x, pq, A, B, Gd, E, Ed, Wu, alpha0, cE,
                     xmin, xmax, xs, umin, umax, W_alpha, W_x, W_s, part);
  hipLaunchKernelGGL(cost_reduce_kernel, dim3(1), dim3(kThreads), 0, st, (const double*)part, K,
                     out);
}

void launch_cost_reduce_forest(const double* part, const int* tstart, int N, int ntrees,
                               double* out, hipStream_t st) {
  hipLaunchKernelGGL(cost_reduce_forest_kernel, dim3(ntrees), dim3(kThreads), 0, st, part, tstart,
                     N, ntrees, out);
}

template <typename T>
void launch_copy_rows(const T* src, int ld_src, T* dst, int ld_dst, const int* idx, int rows,
                      int width, bool scatter, hipStream_t st) {
  if (rows <= 0) return;
  hipLaunchKernelGGL((copy_rows_kernel<T>), dim3(rows), dim3(kThreads), 0, st, src, ld_src, dst,
                     ld_dst, idx, rows, width, scatter ? 1 : 0);
}
void launch_copy_row_sets(const RowCopies& c, const int* idx, int rows, bool scatter,
                          hipStream_t st) {
  if (rows <= 0 || c.n == 0) return;
  hipLaunchKernelGGL(copy_row_sets_kernel, dim3(rows), dim3(kThreads), 0, st, c, idx, rows,
                     scatter ? 1 : 0);
}
template void launch_copy_rows<double>(const double*, int, double*, int, const int*, int, int,
                                       bool, hipStream_t);
template void launch_copy_rows<float>(const float*, int, float*, int, const int*, int, int, bool,
                                      hipStream_t);

#define TAPG_INST(T)                                                                         \
  template void launch_bwd_stage<T>(int, const SweepArgs<T>&, int, hipStream_t);            \
  template void launch_avg<T>(const DevCtl*, const T*, const T*, T*, T*, size_t, size_t,    \
                              hipStream_t);                                                 \
  template void launch_fwd_stage<T>(int, const SweepArgs<T>&, int, hipStream_t);            \
  template void launch_data_step<T>(int, int, int, int, int, int, const int*, const double*, \
                                    const double*, const double*, const double*,             \
                                    const double*, const double*, const double*,             \
                                    const double*, const double*, double, T*, T*, int,       \
                                    const double*, const double*, T*, hipStream_t);          \
  template void launch_cost<T>(int, int, int, int, int, int, int, const int*, const double*, \
                               const double*, const double*, const T*, const T*,             \
                               const double*, const double*, const double*, const double*,   \
                               const double*, const double*, const double*, const double*,   \
                               const double*, const double*, const double*, const double*,   \
                               const double*, const double*, double, double, double,         \
                               double*, double*, hipStream_t);
TAPG_INST(double)
TAPG_INST(float)
#undef TAPG_INST

}  // namespace tapg
