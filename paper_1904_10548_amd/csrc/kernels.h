// Kernel argument blocks and launch wrappers shared by the device files.
#pragma once

#include "internal.h"

namespace tapg {

// The extrapolation weights of the next iteration (Sec. 4.3, eq. apg:1):
// beta_{nu+1} = theta_{nu+1} (1/theta_nu - 1) with theta_0 = theta_{-1} = 1 and,
// by `rule` (tapg_config.beta_rule),
//   TAPG_BETA_PAPER  theta_{nu+1} = (sqrt(theta_nu^4 + 4 theta_nu^2) - theta_nu^2) / 2
//   TAPG_BETA_SIMPLE theta_nu = 2 / (nu + 2) for nu >= 1
//   TAPG_BETA_ZERO   beta = 0 (the plain dual proximal gradient); theta_nu =
//                    1 / (nu + 1), the weights of the running primal mean
// `done` is nu + 1, the iterations completed.  Written once, with no FMA
// contraction, so that every workgroup and launch computes the same values.
__device__ inline void theta_update(int rule, int done, double& theta, double& theta_prev,
                                    double& beta) {
#pragma clang fp contract(off)
  const double th = theta;
  double thn;
  if (rule == TAPG_BETA_SIMPLE) {
    thn = 2.0 / (double)(done + 2);
  } else if (rule == TAPG_BETA_ZERO) {
    thn = 1.0 / (double)(done + 1);
  } else {
    const double t2 = th * th;
    thn = 0.5 * (sqrt(t2 * t2 + 4.0 * t2) - t2);
  }
  theta_prev = th;
  theta = thn;
  beta = rule == TAPG_BETA_ZERO ? 0.0 : thn * (1.0 / th - 1.0);
}

// End of one APG iteration for one tree (Sec. 4.3): from its control state
// and the residual max |y+ - w| / gamma that the forward sweep left in
// res_bits, the state of the next iteration: residual recorded (*res, and
// *record when the tree was still running), iteration count, stop flags,
// theta and beta (theta_update).  A stopped tree's state is returned
// unchanged.  Every caller uses this one routine, so the closing launch and
// the workgroups that close an iteration themselves agree bit for bit.
__device__ inline DevCtl ctl_advance(DevCtl c, bool* record, double* res) {
  *record = false;
  if (c.done) return c;
  const double r = __longlong_as_double((long long)c.res_bits);
  *record = true;
  *res = r;
  c.res_bits = 0ull;
  c.last_res = r;
  c.iter += 1;
  if (!(r < INFINITY)) {
    c.numeric = 1;
    c.done = 1;
  } else if (c.tol > 0.0 && r <= c.tol) {
    c.converged = 1;
    c.done = 1;
  } else if (c.iter >= c.max_iter) {
    c.done = 1;
  }
  theta_update(c.rule, c.iter, c.theta, c.theta_prev, c.beta);
  return c;
}

constexpr int kThreads = 256;     // per-stage kernels
constexpr int kSegThreads = 512;  // segment kernels
// static LDS of a segment kernel (reductions, gamma-scaled bounds), reserved
// out of the per-workgroup limit when the dynamic part is checked
constexpr int kSegStaticLds = 16 * 1024;

// Light upper levels (SegArgs::n_main): the static table of one upper
// workgroup, up_plan_stride ints: its nodes (stage by stage), where their
// children are and which upper workgroups are above it.
enum {
  kPlanNw = 0,  // nodes
  kPlanNst,     // stages
  kPlanCb,      // first child of its last stage's nodes (in the level below)
  kPlanNch,     // children of its last stage's nodes
  kPlanSb,      // first stage
  kPlanPar0,    // upper workgroups above it: first, last (-1: none)
  kPlanPar1,
  kPlanTree,    // its tree (a forest's workgroups never span two trees)
  kPlanOff      // nst + 1 entries: first local index per stage; then node[nw],
                // clo[nw], chi[nw]: a node's children as local indices (stages
                // but the last) or as indices from cb (last stage)
};
constexpr int kUpStack = 64;  // pending arrivals of one workgroup (the host checks the bound)

// Arguments of the per-stage sweep kernels.
template <typename T>
struct SweepArgs {
  int nx, nu, LDX, LDU, LDY;
  int s, node0, count, tile_base;
  int mode;  // 0: APG iteration, 1: power iteration (zero data, no prox),
             // 2: evaluation of x_hat(w) only (u, x written; no dual update)
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

// Arguments of the segment sweep kernels (one launch per level and direction).
template <typename T>
struct SegArgs {
  int nx, nu, LDX, LDU, LDY, LDXR;  // LDXR: power of two >= LDX
  int s_begin, s_end, nst, N;
  int mode;        // 0: APG iteration, 1: power iteration
  int a_ident;     // A == I
  int wu_scalar;   // W_u == wu I
  T wu;
  int part_base, part_total;
  int nnzB;        // nonzeros of B (= of B')
  int nch;         // backward: most children of one workgroup below the level's last stage
  const int2* ranges;  // [n_wg][nst] node range [lo, hi) per stage
  // [n_wg][2] per workgroup: the children [cb, ce) of its last stage's nodes
  // (none at the last stage of the tree), then the parents of its first
  // stage's first and last node (-1 at the root)
  const int2* wgx;
  const int* anc;
  const int* cbeg;
  const int* cend;
  const T* invp;
  const T* F;   // Fbar, N blocks of LDU x LDU, column-major
  const int* fid;  // per stage: the block of F that serves it (equal factors share one)
  const T* Wu;  // W_u, LDU x LDU column-major (general W_u only)
  const T* A;   // A, LDX x LDX column-major (general A only)
  const T* At;  // A'
  const int* Brow;  // CSR of B (nx rows)
  const int* Bcol;
  const T* Bval;
  const int* Btrow;  // CSR of B' (nu rows)
  const int* Btcol;
  const T* Btval;
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
  DevCtl* ctl;       // control block of each tree of the forest (one for a tree)
  // With close != 0 (the first backward launch of an iteration after the
  // first of a chunk), the state is advanced from ctl_prev here: every
  // workgroup computes the next state of its tree from ctl_prev and the
  // residual that the previous iteration left in it, and the tree's first
  // workgroup of the launch writes it to ctl (and the residual to the history).
  const DevCtl* ctl_prev;
  int close;
  double* part;
  double* hist;      // residual history, hist_stride entries per tree
  const int* wgtree; // tree of each workgroup of the launch (nullptr: one tree)
  int ntrees;
  int hist_stride;
  int pq_stride;     // (p, q) of tree k at pq + k * pq_stride
  // Projector form of the stage factor (W_u = w I): Fbar v = (v - E'(G v)) / w
  // with G = (E E')^{-1} E, both sparse (CSR of G: ns rows, of E': nu rows).
  int proj, ns, nnzG, nnzE;
  const int* Grow;
  const int* Gcol;
  const T* Gval;
  const int* Etrow;
  const int* Etcol;
  const T* Etval;
  T winv;
  // Scan form of the sweeps (A = I and the projector form): kperp_n = kappa_n
  // - Pi kappa_n per node; zb_n = Pi u_n, written at a level's last stage for
  // the level below; jv holds P_n = Pi j_n instead of j_n.
  int scan;
  const T* kperp;
  T* zb;
  const T* zr;  // Pi q of each tree (the root's parent input), LDU apart
  // forward launch over every stage (scan form): per workgroup and stage the
  // first node the workgroup owns; nodes before it (ancestors shared with a
  // lower-numbered workgroup) are computed but not written (nullptr: all owned)
  const int* own;
  // Light upper levels (scan form): the whole backward sweep in the bottom
  // level's launch.  With n_main > 0 that launch has n_main bottom workgroups
  // and then n_up more, one per upper workgroup j (all levels above
  // the bottom one, numbered from the lowest level up), each writing for the
  // nodes of upper workgroup j a_n = w1_n + w2_n to lam and the local part of
  // m_n, Pi (kappa_n - (w3_n + B' a_n) / (2 w)), to jv.  The upper workgroups'
  // own work (summing the children into lambda_n = a_n + sum_c lambda_c and
  // P_n = local_n - Pi B' (sum_c lambda_c) / (2 w) + sum_c P_c, the same
  // values by the linearity of Pi and B') is run by whichever workgroup of
  // the launch completes its inputs: every bottom or upper workgroup, once
  // done, counts one arrival at each upper workgroup above it (up_par for a
  // bottom workgroup, its table for an upper one) and the local-part
  // workgroup j one at j; the arrival that reaches up_need[u]
  // runs upper workgroup u (and resets its counter), then arrives above it in
  // turn.  No workgroup waits for another.
  int n_main, n_up;
  const int* up_plan;  // [n_up][up_plan_stride] static tables
  int up_plan_stride, up_nw, up_nch;  // most nodes and children below of one upper workgroup
  const int2* up_par;  // [n_main]: upper workgroups above each bottom workgroup
  const int* up_need;  // [n_up]
  unsigned* up_cnt;    // [n_up], zero between launches
};

// Persistent iteration of one tree: every workgroup of every level in one
// cooperative launch, iterating `iters` times.  Levels hand over through
// counters instead of launch boundaries: a workgroup's backward sweep starts
// once its child workgroups have finished theirs, its forward sweep once its
// parent workgroup has finished its own; the top workgroup ends each iteration
// (residual, stop test) once every workgroup has finished its forward sweep.
constexpr int kChainMaxLevels = 8;
struct ChainSync {
  unsigned fwd_all;          // forward sweeps completed by all workgroups
  int stop;                  // set by the top workgroup when the solve stops
  int error;                 // a wait exceeded its bound
  int pad;
  unsigned long long res[2]; // residual max of the last two iterations (double bits)
};
template <typename T>
struct ChainArgs {
  const SegArgs<T>* lev;     // per level, top first (device memory)
  int nlev, total, iters;
  int base[kChainMaxLevels + 1];  // first workgroup of each level
  const int2* parents;       // workgroups [x, y] owning the parents of a workgroup's first stage (x = -1: top)
  const int* nchild;         // child workgroups of each workgroup
  unsigned* bwd_cnt;         // per workgroup: backward sweeps completed by its children
  unsigned* fwd_flag;        // per workgroup: forward sweeps completed
  ChainSync* sync;
  DevCtl* ctl;
  double* hist;
};

// Launch wrappers (segment_kernels.hip).
// Scan-form sweep launches and their dynamic LDS (scan_kernels.hip).
template <typename T>
void launch_scan(bool fwd, int nbm, const SegArgs<T>& a, int n_wg, hipStream_t st);
template <typename T>
size_t scan_lds(int nbm, const SegArgs<T>& a);
template <typename T>
void launch_seg(bool fwd, int nbm, const SegArgs<T>& a, int n_wg, hipStream_t st);
// Dynamic LDS of the work of an upper workgroup (light upper levels, see
// SegArgs::n_main): a table of plan_ints ints, at most nw nodes and nch
// children below.
template <typename T>
size_t scan_up_lds(int plan_ints, int nw, int nch, int nu, int ns, int nnzB, int nnzG, int nnzE);
template <typename T>
size_t seg_lds(int nbm, const SegArgs<T>& a);
// Cooperative launch of the persistent iteration (NB: widest level's
// template, lds: the largest level's dynamic LDS).  hipErrorCooperativeLaunch-
// TooLarge (or any launch error) is returned, not thrown.
template <typename T>
hipError_t launch_chain(int nbm, bool proj, const ChainArgs<T>& c, size_t lds, hipStream_t st);
// Workgroups of the persistent kernel resident per CU (occupancy).
template <typename T>
int chain_blocks_per_cu(int nbm, bool proj, size_t lds);

// Launch wrappers (stage_kernels.hip).
template <typename T>
void launch_bwd_stage(int nb, const SweepArgs<T>& a, int tiles, hipStream_t st);
template <typename T>
void launch_fwd_stage(int nb, const SweepArgs<T>& a, int tiles, hipStream_t st);
// Averaged primal update of one tree (nu_el = K * LDU entries of u, nx_el = K * LDX of x).
template <typename T>
void launch_avg(const DevCtl* ctl, const T* u, const T* x, T* ua, T* xa, size_t nu_el,
                size_t nx_el, hipStream_t st);
// End of an iteration of ntrees trees (per-tree control blocks and histories).
void launch_iter_end(DevCtl* c, double* hist, int ntrees, int hist_stride, hipStream_t st);
// The same from the states in prev into out (out == prev allowed).
void launch_iter_end_from(const DevCtl* prev, DevCtl* out, double* hist, int ntrees,
                          int hist_stride, hipStream_t st);
void launch_power_end(DevCtl* c, const double* part, int n, hipStream_t st);
// Holds the stream for `ticks` periods of the device wall clock (at most 50 ms).
void launch_hold(long long ticks, hipStream_t st);
template <typename T>
void launch_data_step(int K, int nx, int nu, int nd, int LDX, int LDU, const int* stage,
                      const double* prob, const double* demand, const double* price,
                      const double* Pd, const double* Gd, const double* Gbar, const double* Fbar,
                      const double* alpha0, const double* cE, double W_alpha, T* kappa, T* g,
                      int ns, const double* Gm, const double* E, T* kperp, hipStream_t st);
template <typename T>
void launch_cost(int K, int nx, int nu, int nd, int ns, int LDX, int LDU, const int* anc,
                 const double* prob, const double* demand, const double* price, const T* u,
                 const T* x, const double* pq, const double* A, const double* B,
                 const double* Gd, const double* E, const double* Ed, const double* Wu,
                 const double* alpha0, const double* cE, const double* xmin, const double* xmax,
                 const double* xs, const double* umin, const double* umax, double W_alpha,
                 double W_x, double W_s, double* part, double* out, hipStream_t st);
// Per-tree (cost, box violation, equality violation) of a forest from the
// per-node terms written by launch_cost: out[3 k .. 3 k + 2].
void launch_cost_reduce_forest(const double* part, const int* tstart, int N, int ntrees,
                               double* out, hipStream_t st);
// Duality-gap terms of a dual y and its primal (u, x) = x_hat(y), FP64 (gap_kernels.hip):
// out[0..3] = f(x'), <y, H x'>, g*(y), g(t) summed over the K nodes.
void launch_gap_terms(int K, int nx, int nu, int LDX, int LDU, int LDY, const int* anc,
                      const double* prob, const double* price, const double* y, const double* u,
                      const double* x, const double* pq, const double* Wu, const double* alpha0,
                      const double* cE, const double* xmin, const double* xmax, const double* xs,
                      const double* umin, const double* umax, double W_alpha, double W_x,
                      double W_s, double gamma, double* part, double* out, hipStream_t st);
// dst[i] = (double) src[i], i < n.
template <typename T>
void launch_widen(const T* src, double* dst, size_t n, hipStream_t st);
// Row gather (dst[r] = src[idx[r]]) or scatter (dst[idx[r]] = src[r]).
template <typename T>
void launch_copy_rows(const T* src, int ld_src, T* dst, int ld_dst, const int* idx, int rows,
                      int width, bool scatter, hipStream_t st);
// Several arrays gathered or scattered by the same row map in one launch
// (elements of 4 or 8 bytes, copied bit for bit).
constexpr int kRowArrays = 8;
struct RowCopies {
  const void* src[kRowArrays];
  void* dst[kRowArrays];
  int ld_src[kRowArrays], ld_dst[kRowArrays], width[kRowArrays], bytes[kRowArrays];
  int n = 0;
  template <typename E>
  void add(const E* s, int lds, E* d, int ldd, int w) {
    static_assert(sizeof(E) == 4 || sizeof(E) == 8, "row copies move 4- or 8-byte elements");
    if (n >= kRowArrays) throw Fail{TAPG_EINVAL, "row copies: too many arrays in one launch"};
    src[n] = s;
    dst[n] = d;
    ld_src[n] = lds;
    ld_dst[n] = ldd;
    width[n] = w;
    bytes[n] = (int)sizeof(E);
    ++n;
  }
};
void launch_copy_row_sets(const RowCopies& c, const int* idx, int rows, bool scatter,
                          hipStream_t st);

}  // namespace tapg
