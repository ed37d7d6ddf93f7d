// Scenario-tree construction from sampled error paths (Sec. 2.3 and 6.2: the
// paper reduces 10^4 Monte-Carlo paths to a tree with the forward scenario
// reduction of Heitsch and Roemisch), stage by stage:
//   stage 0: one root holding every path;
//   stage t: every node of stage t-1 holds a cluster of paths; forward
//   selection picks min(b_t, |cluster|) representatives by the paths' stage-t
//   values, each member joins its nearest representative (ties: the one picked
//   first), and each representative becomes a child (in the order picked) with
//   the representative's value and its members' summed probability.
// Forward selection over a cluster with probabilities p_k and c(k, u) =
// |x_k - x_u|_2: D_k = +inf; n times: u = argmin over unpicked u of
// sum_k p_k min(D_k, c(k, u)) (ties: the lowest position in the cluster),
// then D_k = min(D_k, c(k, u)).  The sums are the transport cost of moving
// every member to its nearest picked point.
//
// Device work per stage: the candidates' transport costs for every cluster at
// once (a tiled kernel: 32 candidates of one cluster per workgroup, the
// cluster's members streamed through LDS in tiles of 32), the argmin per
// cluster, the D update, and the final assignment.  Every distance is the
// same sequence of FP64 operations in every kernel.  The host keeps the tree
// bookkeeping (clusters, node order, probabilities).
#include <algorithm>
#include <cmath>
#include <vector>

#include "kernels.h"

namespace tapg {
namespace {

constexpr int kTU = 32;   // candidates per workgroup
constexpr int kTK = 32;   // members per LDS tile
constexpr int kTB = 256;  // threads per workgroup
constexpr int kGR = kTB / kTU;  // member groups per tile

__device__ __forceinline__ double dist2(const double* a, const double* b, int d) {
#pragma clang fp contract(off)
  double s = 0.0;
  for (int i = 0; i < d; ++i) {
    const double e = a[i] - b[i];
    s += e * e;
  }
  return s;
}

// X row of the member at position k of the stage ordering.
__device__ __forceinline__ const double* xrow(const double* S, const int* perm, int k, int H,
                                              int d, int t) {
  return S + ((size_t)perm[k] * H + t) * d;
}

// total[u] for every candidate position u of every cluster still picking
// (step j < n of its cluster); picked candidates get +inf.  wg_cl / wg_u0:
// the cluster and first candidate of each workgroup.
__global__ __launch_bounds__(kTB) void fs_cost_kernel(const double* S, const int* perm, int H,
                                                     int d, int t, const double* p,
                                                     const double* D, const int* picked,
                                                     const int2* cl, const int* n_pick, int j,
                                                     const int* wg_cl, const int* wg_u0,
                                                     double* total) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* sU = reinterpret_cast<double*>(smem_raw);  // [kTU][d]
  double* sK = sU + kTU * d;                         // [kTK][d]
  double* sPD = sK + kTK * d;                        // [2][kTK]: p, D
  double* sRed = sPD + 2 * kTK;                      // [kTB]
  const int v = wg_cl[blockIdx.x], u0 = wg_u0[blockIdx.x];
  if (j >= n_pick[v]) return;
  const int2 r = cl[v];
  const int tid = threadIdx.x;
  const int nu = min(kTU, r.y - u0);
  for (int e = tid; e < nu * d; e += kTB) {
    const int q = e / d, i = e - q * d;
    sU[q * d + i] = xrow(S, perm, u0 + q, H, d, t)[i];
  }
  const int cu = tid % kTU, grp = tid / kTU;  // candidate; group of each member tile
  double acc = 0.0;
  for (int k0 = r.x; k0 < r.y; k0 += kTK) {
    const int nk = min(kTK, r.y - k0);
    __syncthreads();
    for (int e = tid; e < nk * d; e += kTB) {
      const int q = e / d, i = e - q * d;
      sK[q * d + i] = xrow(S, perm, k0 + q, H, d, t)[i];
    }
    for (int q = tid; q < nk; q += kTB) {
      sPD[q] = p[k0 + q];
      sPD[kTK + q] = D[k0 + q];
    }
    __syncthreads();
    if (cu < nu) {
      const int qb = grp * (kTK / kGR);
      for (int q = qb; q < qb + kTK / kGR && q < nk; ++q) {
        const double c = sqrt(dist2(sK + q * d, sU + cu * d, d));
        acc += sPD[q] * fmin(sPD[kTK + q], c);
      }
    }
  }
  sRed[tid] = acc;
  __syncthreads();
  if (grp == 0 && cu < nu) {
    double s = sRed[cu];
    for (int g = 1; g < kGR; ++g) s += sRed[g * kTU + cu];
    total[u0 + cu] = picked[u0 + cu] ? INFINITY : s;
  }
}

// One workgroup per cluster: the position of the smallest total (the lowest
// position among equal ones) becomes pick j.
__global__ __launch_bounds__(kTB) void fs_argmin_kernel(const double* total, const int2* cl,
                                                       const int* n_pick, int j, int bmax,
                                                       int* sel, int* picked) {
  __shared__ double sv[kTB];
  __shared__ int si[kTB];
  const int v = blockIdx.x;
  if (j >= n_pick[v]) return;
  const int2 r = cl[v];
  double best = INFINITY;
  int bi = r.x;
  for (int u = r.x + threadIdx.x; u < r.y; u += kTB) {
    const double x = total[u];
    if (x < best) {
      best = x;
      bi = u;
    }
  }
  sv[threadIdx.x] = best;
  si[threadIdx.x] = bi;
  __syncthreads();
  for (int s = kTB / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      const double a = sv[threadIdx.x], b = sv[threadIdx.x + s];
      const int ia = si[threadIdx.x], ib = si[threadIdx.x + s];
      if (b < a || (b == a && ib < ia)) {
        sv[threadIdx.x] = b;
        si[threadIdx.x] = ib;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    sel[(size_t)v * bmax + j] = si[0];
    picked[si[0]] = 1;
  }
}

// D_k = min(D_k, c(k, pick j of k's cluster)).
__global__ __launch_bounds__(kTB) void fs_update_kernel(const double* S, const int* perm, int H,
                                                       int d, int t, const int* cl_of,
                                                       const int* n_pick, int j, int bmax,
                                                       const int* sel, int M, double* D) {
  const int k = blockIdx.x * kTB + threadIdx.x;
  if (k >= M) return;
  const int v = cl_of[k];
  if (j >= n_pick[v]) return;
  const int u = sel[(size_t)v * bmax + j];
  const double c = sqrt(dist2(xrow(S, perm, k, H, d, t), xrow(S, perm, u, H, d, t), d));
  D[k] = fmin(D[k], c);
}

// child[k] = the pick of k's cluster nearest to k (ties: the earliest pick).
__global__ __launch_bounds__(kTB) void fs_assign_kernel(const double* S, const int* perm, int H,
                                                       int d, int t, const int* cl_of,
                                                       const int* n_pick, int bmax,
                                                       const int* sel, int M, int* child) {
  const int k = blockIdx.x * kTB + threadIdx.x;
  if (k >= M) return;
  const int v = cl_of[k];
  const double* xk = xrow(S, perm, k, H, d, t);
  double best = INFINITY;
  int bj = 0;
  for (int j = 0; j < n_pick[v]; ++j) {
    const double c = sqrt(dist2(xk, xrow(S, perm, sel[(size_t)v * bmax + j], H, d, t), d));
    if (c < best) {
      best = c;
      bj = j;
    }
  }
  child[k] = bj;
}

template <typename T>
struct DevBuf {
  T* p = nullptr;
  explicit DevBuf(size_t n) {
    if (hipMalloc(&p, std::max<size_t>(n, 1) * sizeof(T)) != hipSuccess)
      throw Fail{TAPG_ENOMEM, "tree build: device allocation failed"};
  }
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
};

}  // namespace
}  // namespace tapg

using namespace tapg;

extern "C" tapg_status tapg_tree_build(int M, int H, int d, const double* samples,
                                       const double* prob, const int* branching, int device,
                                       int cap, int* nodes_per_stage, int* ancestor,
                                       double* node_prob, double* node_value, int* rep,
                                       int* K_out) {
  try {
    clear_error();
    if (M < 1 || H < 1 || d < 1 || d > 128 || !samples || !branching || !nodes_per_stage ||
        !ancestor || !node_prob || !K_out || cap < 1)
      throw Fail{TAPG_EINVAL, "tree build: M, H >= 1, 1 <= d <= 128, non-NULL arrays, cap >= 1"};
    for (int t = 1; t < H; ++t)
      if (branching[t] < 1) throw Fail{TAPG_EINVAL, "tree build: branching[t] >= 1 for t >= 1"};
    std::vector<double> p(M, 1.0 / M);
    if (prob) {
      double s = 0.0;
      for (int k = 0; k < M; ++k) {
        if (!(prob[k] >= 0.0) || !std::isfinite(prob[k]))
          throw Fail{TAPG_EINVAL, "tree build: probabilities must be finite and >= 0"};
        p[k] = prob[k];
        s += prob[k];
      }
      if (!(std::fabs(s - 1.0) <= 1e-9)) throw Fail{TAPG_EINVAL, "tree build: probabilities must add up to 1"};
    }
    for (size_t i = 0; i < (size_t)M * H * d; ++i)
      if (!std::isfinite(samples[i])) throw Fail{TAPG_ENUMERIC, "tree build: non-finite sample"};
    if (hipSetDevice(device) != hipSuccess) throw Fail{TAPG_EDEVICE, "tree build: no such device"};
    hipStream_t st = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess)
      throw Fail{TAPG_EDEVICE, "tree build: stream creation failed"};
    struct StreamGuard {
      hipStream_t s;
      ~StreamGuard() { (void)hipStreamDestroy(s); }
    } sg{st};
    DevBuf<double> dS((size_t)M * H * d), dP(M), dD(M), dTot(M);
    DevBuf<int> dPerm(M), dPicked(M), dClOf(M), dChild(M);
    TAPG_HIP(hipMemcpyAsync(dS.p, samples, (size_t)M * H * d * 8, hipMemcpyHostToDevice, st));

    // the tree so far: per node its members (paths), in breadth-first order
    std::vector<std::vector<int>> mem(1);
    mem[0].resize(M);
    for (int k = 0; k < M; ++k) mem[0][k] = k;
    std::vector<int> anc{-1}, reps{0}, mu{1};
    std::vector<double> pr{1.0};
    if (prob) {
      double s = 0.0;
      for (int k = 0; k < M; ++k) s += p[k];
      pr[0] = s;
    }
    int first = 0;
    for (int t = 1; t < H; ++t) {
      const int nc = mu.back();  // clusters: the nodes of stage t-1
      const int b = branching[t];
      std::vector<int> perm, cl_of(M);
      std::vector<int2> cl(nc);
      std::vector<int> npick(nc), wg_cl, wg_u0;
      for (int v = 0; v < nc; ++v) {
        const std::vector<int>& m = mem[first + v];
        cl[v] = make_int2((int)perm.size(), (int)(perm.size() + m.size()));
        for (int k : m) {
          cl_of[perm.size()] = v;
          perm.push_back(k);
        }
        npick[v] = std::min<int>(b, (int)m.size());
        for (int u0 = cl[v].x; u0 < cl[v].y; u0 += kTU) {
          wg_cl.push_back(v);
          wg_u0.push_back(u0);
        }
      }
      std::vector<double> pp(M), inf(M, INFINITY);
      for (int k = 0; k < M; ++k) pp[k] = p[perm[k]];
      DevBuf<int2> dCl(nc);
      DevBuf<int> dN(nc), dSel((size_t)nc * b), dWc(wg_cl.size()), dWu(wg_u0.size());
      TAPG_HIP(hipMemcpyAsync(dPerm.p, perm.data(), (size_t)M * 4, hipMemcpyHostToDevice, st));
      TAPG_HIP(hipMemcpyAsync(dClOf.p, cl_of.data(), (size_t)M * 4, hipMemcpyHostToDevice, st));
      TAPG_HIP(hipMemcpyAsync(dP.p, pp.data(), (size_t)M * 8, hipMemcpyHostToDevice, st));
      TAPG_HIP(hipMemcpyAsync(dD.p, inf.data(), (size_t)M * 8, hipMemcpyHostToDevice, st));
      TAPG_HIP(hipMemsetAsync(dPicked.p, 0, (size_t)M * 4, st));
      TAPG_HIP(hipMemcpyAsync(dCl.p, cl.data(), (size_t)nc * sizeof(int2), hipMemcpyHostToDevice, st));
      TAPG_HIP(hipMemcpyAsync(dN.p, npick.data(), (size_t)nc * 4, hipMemcpyHostToDevice, st));
      TAPG_HIP(hipMemcpyAsync(dWc.p, wg_cl.data(), wg_cl.size() * 4, hipMemcpyHostToDevice, st));
      TAPG_HIP(hipMemcpyAsync(dWu.p, wg_u0.data(), wg_u0.size() * 4, hipMemcpyHostToDevice, st));
      const int nblk = (M + kTB - 1) / kTB;
      for (int j = 0; j < b; ++j) {
        const size_t lds = ((size_t)(kTU + kTK) * d + 2 * kTK + kTB) * sizeof(double);
        hipLaunchKernelGGL(fs_cost_kernel, dim3((unsigned)wg_cl.size()), dim3(kTB), lds, st, dS.p,
                           dPerm.p, H, d, t, dP.p, dD.p, dPicked.p, dCl.p, dN.p, j, dWc.p, dWu.p,
                           dTot.p);
        hipLaunchKernelGGL(fs_argmin_kernel, dim3(nc), dim3(kTB), 0, st, dTot.p, dCl.p, dN.p, j, b,
                           dSel.p, dPicked.p);
        hipLaunchKernelGGL(fs_update_kernel, dim3(nblk), dim3(kTB), 0, st, dS.p, dPerm.p, H, d, t,
                           dClOf.p, dN.p, j, b, dSel.p, M, dD.p);
      }
      hipLaunchKernelGGL(fs_assign_kernel, dim3(nblk), dim3(kTB), 0, st, dS.p, dPerm.p, H, d, t,
                         dClOf.p, dN.p, b, dSel.p, M, dChild.p);
      TAPG_HIP(hipGetLastError());
      std::vector<int> sel((size_t)nc * b), child(M);
      TAPG_HIP(hipMemcpyAsync(sel.data(), dSel.p, sel.size() * 4, hipMemcpyDeviceToHost, st));
      TAPG_HIP(hipMemcpyAsync(child.data(), dChild.p, (size_t)M * 4, hipMemcpyDeviceToHost, st));
      TAPG_HIP(hipStreamSynchronize(st));
      const int before = (int)anc.size();
      for (int v = 0; v < nc; ++v) {
        for (int j = 0; j < npick[v]; ++j) {
          std::vector<int> m;
          double s = 0.0;
          for (int k = cl[v].x; k < cl[v].y; ++k)
            if (child[k] == j) {
              m.push_back(perm[k]);
              s += p[perm[k]];
            }
          anc.push_back(first + v);
          pr.push_back(s);
          reps.push_back(perm[sel[(size_t)v * b + j]]);
          mem.push_back(std::move(m));
          if ((int)anc.size() > cap)
            throw Fail{TAPG_EDIM, "tree build: more nodes than cap (" + std::to_string(cap) + ")"};
        }
      }
      first += nc;
      mu.push_back((int)anc.size() - before);
    }
    const int K = (int)anc.size();
    for (int t = 0; t < H; ++t) nodes_per_stage[t] = mu[t];
    for (int t = 0, n = 0; t < H; ++t)
      for (int q = 0; q < mu[t]; ++q, ++n) {
        ancestor[n] = anc[n];
        node_prob[n] = pr[n];
        if (rep) rep[n] = reps[n];
        if (node_value)
          for (int i = 0; i < d; ++i)
            node_value[(size_t)n * d + i] = samples[((size_t)reps[n] * H + t) * d + i];
      }
    *K_out = K;
    return TAPG_OK;
  } catch (const Fail& e) {
    set_error(e.msg);
    return e.code;
  } catch (const std::bad_alloc&) {
    set_error("host allocation failed");
    return TAPG_ENOMEM;
  }
}
