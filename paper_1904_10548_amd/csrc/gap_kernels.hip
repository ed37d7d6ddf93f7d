// Duality gap of a dual iterate (Sec. 4.2, the Fenchel dual and strong
// duality), FP64.
//
// For a dual y (the iterate a solve returns) the gap is evaluated at y and
// at the primal pair that y itself determines:
//   x' = x_hat(y)                      (one dual-gradient sweep at w = y)
//   t  = prox_{g/gamma}(y/gamma + H x') (the split variable of one more step)
//   G  = f(x') + g(t) + F(y),   F(y) = -f(x') - <y, H x'> + g*(y)
// so G = g(t) + g*(y) - <y, H x'>.  The dual objective F(y) is reported with
// it.  Per node n (H x' = (x'_n, x'_n, u'_n)):
//   f part:  p_n (c_n'u'_n + du'_n W_u du'_n)
//   <y,Hx'>: (y1_n + y2_n)'x'_n + y3_n'u'_n
//   g*(y):   sum_i max(y1_i xmax_i, y1_i xmin_i) + xs'y2_n + sum_i max(y3_i umax_i, y3_i umin_i)
//   g(t):    W_x max(0, dist(z1 | [xmin, xmax]) - W_x / gamma)
//          + W_s max(0, dist(z2 | [xs, inf)) - W_s / gamma),   z = y / gamma + H x'
//            (the prox of a distance moves a point towards the set by the
//            weight, so the distance of t is what is left; t3 is in U)
// The sweep itself runs on the per-stage kernels in their evaluation mode.
#include <cmath>

#include "kernels.h"

namespace tapg {

namespace {

__device__ double gap_block_sum(double v, double* s) {
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

template <typename T>
__global__ __launch_bounds__(kThreads) void widen_kernel(const T* src, double* dst, size_t n) {
  const size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x;
  if (i < n) dst[i] = (double)src[i];
}

__global__ __launch_bounds__(kThreads) void gap_node_kernel(
    int nx, int nu, int LDX, int LDU, int LDY, const int* anc, const double* prob,
    const double* price, const double* y, const double* u, const double* x, const double* pq,
    const double* Wu, const double* alpha0, const double* cE, const double* xmin,
    const double* xmax, const double* xs, const double* umin, const double* umax,
    double W_alpha, double W_x, double W_s, double gamma, double* part) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* sDu = reinterpret_cast<double*>(smem_raw);
  __shared__ double red[kThreads];
  const int n = blockIdx.x;
  const int par = anc[n];
  const double* pqn = pq + (par < 0 ? (size_t)(-par - 1) * (LDX + LDU) : 0);
  const double* un = u + (size_t)n * LDU;
  const double* xn = x + (size_t)n * LDX;
  const double* yn = y + (size_t)n * LDY;
  for (int i = threadIdx.x; i < nu; i += kThreads)
    sDu[i] = un[i] - (par >= 0 ? u[(size_t)par * LDU + i] : pqn[LDX + i]);
  __syncthreads();
  const double pi = price[n];
  const double ig = 1.0 / gamma;
  double lin = 0.0, quad = 0.0, yhx = 0.0, gs = 0.0, e1 = 0.0, e2 = 0.0;
  for (int r = threadIdx.x; r < nu; r += kThreads) {
    double wd = 0.0;
    for (int k = 0; k < nu; ++k) wd += Wu[(size_t)k * LDU + r] * sDu[k];
    quad += sDu[r] * wd;
    lin += W_alpha * (alpha0[r] + pi * cE[r]) * un[r];
    const double y3 = yn[2 * LDX + r];
    yhx += y3 * un[r];
    gs += fmax(y3 * umax[r], y3 * umin[r]);
  }
  for (int r = threadIdx.x; r < nx; r += kThreads) {
    const double y1 = yn[r], y2 = yn[LDX + r], xr = xn[r];
    yhx += (y1 + y2) * xr;
    gs += fmax(y1 * xmax[r], y1 * xmin[r]) + xs[r] * y2;
    const double z1 = y1 * ig + xr, z2 = y2 * ig + xr;
    const double d1 = z1 - fmin(fmax(z1, xmin[r]), xmax[r]);
    const double d2 = z2 - fmax(z2, xs[r]);
    e1 += d1 * d1;
    e2 += d2 * d2;
  }
  lin = gap_block_sum(lin, red);
  quad = gap_block_sum(quad, red);
  yhx = gap_block_sum(yhx, red);
  gs = gap_block_sum(gs, red);
  e1 = gap_block_sum(e1, red);
  e2 = gap_block_sum(e2, red);
  if (threadIdx.x == 0) {
    const double gt = W_x * fmax(0.0, sqrt(e1) - W_x * ig) + W_s * fmax(0.0, sqrt(e2) - W_s * ig);
    part[(size_t)n * 4 + 0] = prob[n] * (lin + quad);
    part[(size_t)n * 4 + 1] = yhx;
    part[(size_t)n * 4 + 2] = gs;
    part[(size_t)n * 4 + 3] = gt;
  }
}

// Column sums of the per-node terms, in a fixed order (one block).
__global__ __launch_bounds__(kThreads) void gap_reduce_kernel(const double* part, int K,
                                                              double* out) {
  __shared__ double red[kThreads];
  double c[4] = {0.0, 0.0, 0.0, 0.0};
  for (int n = threadIdx.x; n < K; n += kThreads)
    for (int j = 0; j < 4; ++j) c[j] += part[(size_t)n * 4 + j];
  for (int j = 0; j < 4; ++j) {
    const double s = gap_block_sum(c[j], red);
    if (threadIdx.x == 0) out[j] = s;
  }
}

}  // namespace

template <typename T>
void launch_widen(const T* src, double* dst, size_t n, hipStream_t st) {
  if (n == 0) return;
  const unsigned blocks = (unsigned)((n + kThreads - 1) / kThreads);
  hipLaunchKernelGGL((widen_kernel<T>), dim3(blocks), dim3(kThreads), 0, st, src, dst, n);
}
template void launch_widen<float>(const float*, double*, size_t, hipStream_t);
template void launch_widen<double>(const double*, double*, size_t, hipStream_t);

void launch_gap_terms(int K, int nx, int nu, int LDX, int LDU, int LDY, const int* anc,
                      const double* prob, const double* price, const double* y, const double* u,
                      const double* x, const double* pq, const double* Wu, const double* alpha0,
                      const double* cE, const double* xmin, const double* xmax, const double* xs,
                      const double* umin, const double* umax, double W_alpha, double W_x,
                      double W_s, double gamma, double* part, double* out, hipStream_t st) {
  const size_t lds = (size_t)LDU * sizeof(double);
  hipLaunchKernelGGL(gap_node_kernel, dim3(K), dim3(kThreads), lds, st, nx, nu, LDX, LDU, LDY,
                     anc, prob, price, y, u, x, pq, Wu, alpha0, cE, xmin, xmax, xs, umin, umax,
                     W_alpha, W_x, W_s, gamma, part);
  hipLaunchKernelGGL(gap_reduce_kernel, dim3(1), dim3(kThreads), 0, st, (const double*)part, K,
                     out);
}

}  // namespace tapg
