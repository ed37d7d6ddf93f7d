// Internal declarations of the tapg library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "tapg.h"

namespace tapg {

// ---------------------------------------------------------------------------
// Errors
// ---------------------------------------------------------------------------
void set_error(const std::string& msg);
void clear_error();

struct Fail {
  tapg_status code;
  std::string msg;
};

#define TAPG_HIP(call)                                                          \
  do {                                                                          \
    hipError_t e_ = (call);                                                     \
    if (e_ != hipSuccess)                                                       \
      throw ::tapg::Fail{TAPG_EDEVICE, std::string(#call) + ": " +              \
                                           hipGetErrorString(e_)};              \
  } while (0)

inline int round_up(int v, int m) { return (v + m - 1) / m * m; }

// ---------------------------------------------------------------------------
// Host dense linear algebra (row-major, FP64), used by the offline factor step
// ---------------------------------------------------------------------------
struct Mat {
  int r = 0, c = 0;
  std::vector<double> a;
  Mat() = default;
  Mat(int rows, int cols) : r(rows), c(cols), a((size_t)rows * cols, 0.0) {}
  double& operator()(int i, int j) { return a[(size_t)i * c + j]; }
  double operator()(int i, int j) const { return a[(size_t)i * c + j]; }
  static Mat eye(int n);
  static Mat from(const double* p, int rows, int cols);
};

Mat matmul(const Mat& A, const Mat& B);
Mat transpose(const Mat& A);
Mat add(const Mat& A, const Mat& B, double beta = 1.0);  // A + beta B
// Householder QR of E' (nu x ns).  Returns false if E is rank deficient.
// Z (nu x m) spans ker E with orthonormal columns; Pd = -E^+ Ed (nu x nd).
bool null_space_and_particular(const Mat& E, const Mat& Ed, Mat& Z, Mat& Pd);
// In-place Cholesky (lower); false if not positive definite.
bool cholesky(Mat& M);
// Solve (L L') X = B in place of B, L from cholesky().
void chol_solve(const Mat& L, Mat& B);

// ---------------------------------------------------------------------------
// Host objects behind the opaque handles
// ---------------------------------------------------------------------------
struct NetworkHost {
  int nx, nu, nd, ns;
  Mat A, B, Gd, E, Ed;
  std::vector<double> xmin, xmax, xs, umin, umax;
  Mat Z, Pd;  // ker E basis and -E^+ Ed
};

struct TreeHost {
  uint64_t uid;       // unique id, never reused
  uint64_t version;   // bumped by set_data
  int N, K, nd;
  std::vector<int> mu, offset, anc, cbeg, cend, stage;
  std::vector<double> prob, demand, price;
  // A forest (a batch of trees sharing the horizon) uses the same layout: the
  // stage-s nodes of tree 0, then those of tree 1, ...; the root of tree k has
  // ancestor -1 - k.  tstart[s * (ntrees + 1) + k] is the first node of tree k
  // at stage s (empty for a single tree).
  int ntrees = 1;
  std::vector<int> tstart;
  // a forest whose demand and price are gathered on the device from its trees'
  // own slots (host arrays left empty, nothing uploaded)
  bool device_data = false;
  int seg_begin(int s, int k) const {
    return tstart.empty() ? offset[s] : tstart[(size_t)s * (ntrees + 1) + k];
  }
  int seg_end(int s, int k) const {
    return tstart.empty() ? offset[s + 1] : tstart[(size_t)s * (ntrees + 1) + k + 1];
  }
};

// Device control block of one tree (read by every kernel; advanced at the end
// of each iteration).  The level launches keep two per tree and use them
// alternately: an iteration's first backward launch advances the state of the
// previous one into the other block.
struct DevCtl {
  int iter;         // iterations completed
  int done;         // stop flag
  int converged;    // residual reached tol
  int numeric;      // non-finite residual seen
  int max_iter;
  int rule;         // theta/beta rule (tapg_config.beta_rule)
  double tol;
  double gamma;
  double theta, theta_prev, beta;
  double last_res;
  unsigned long long res_bits;  // running max |r| of the current iteration (bits of a double >= 0)
  double pw_scale;              // power iteration: 1/|v|
  double L;                     // power iteration: latest |M v| estimate
  unsigned pad1, pad2;
};

// Segment schedule (schedule.cpp).  A workgroup holds at most kSegNbMax nodes
// of one stage (kernel templates NB = 1, 2, 4; wider groups would spill
// registers).  A level covers stages [s_begin, s_end]; its workgroups own
// groups of `group` consecutive nodes of stage s_begin and their descendants.
constexpr int kSegNbMax = 4;
struct LevelPlan {
  int s_begin, s_end, group, nbm, n_wg;
  double cost;
};

// Per-(solver, tree) device buffers.
struct Slot {
  uint64_t tree_uid = 0, data_version = ~0ull;
  int K = 0, N = 0;
  size_t elem = 8;  // sizeof(T) of the sweep buffers
  // structure
  int *d_anc = nullptr, *d_cbeg = nullptr, *d_cend = nullptr, *d_stage = nullptr;
  double* d_prob64 = nullptr;
  void* d_invp = nullptr;  // T[K]
  // data
  double *d_demand = nullptr, *d_price = nullptr;
  void *d_kappa = nullptr, *d_g = nullptr, *d_pq = nullptr;
  double* d_pq64 = nullptr;
  void *d_P0 = nullptr, *d_P1 = nullptr;  // power-iteration vectors
  // iterates
  // scan form: kappa - Pi kappa; Pi u at level ends; Pi q per tree
  void *d_kperp = nullptr, *d_zb = nullptr, *d_zr = nullptr;
  void *d_Y0 = nullptr, *d_Y1 = nullptr, *d_lam = nullptr, *d_j = nullptr, *d_u = nullptr,
       *d_x = nullptr;
  void *d_ua = nullptr, *d_xa = nullptr;  // averaged primal (single-tree solves that ask for it)
  DevCtl* d_ctl = nullptr;
  double* d_hist = nullptr;
  int hist_cap = 0;
  double* d_part = nullptr;  // per-tile partials (power iteration) and per-node cost terms
  int part_cap = 0;
  // tiling per stage: node range [node_offset[s], node_offset[s+1]) in tiles of
  // nb_of_stage[s] nodes; tile_offset[s] numbers the tiles across stages
  std::vector<int> node_offset, nb_of_stage, tiles_of_stage, tile_offset;
  int total_tiles = 0;
  // state
  bool has_dual = false;
  int last_iter_parity = 0;
  double L = 0.0;
  bool L_valid = false;
  tapg_result last{};
  bool has_result = false;
  std::vector<double> last_pq;  // (p | q) of the last solve, LDX + LDU doubles
  bool gap_valid = false;       // last.dual_gap / dual_obj hold the gap of the current dual
  bool numeric = false;  // the last solve hit a non-finite residual
  hipGraphExec_t graph = nullptr;
  int graph_iters = 0;
  // segment schedule: levels top (stage 0) first
  struct Level {
    int s_begin, s_end, n_wg, nbm;
    int nch;  // most children of one workgroup below the level's last stage
    int2* d_ranges;
    int* d_wgtree;  // tree of each workgroup (forests only)
    int2* d_wgx = nullptr;  // children of the last stage, parents of the first
    int nw = 0;             // light upper level: most nodes of one workgroup (all stages)
  };
  std::vector<Level> levels;
  // Scan form: the forward sweep in one launch over stages 0..N-1, each
  // workgroup also walking its nodes' ancestors; its workgroups are those of
  // the bottom level (fwd_group 0) or groups of fwd_group consecutive nodes of
  // the last stage.  d_own: per workgroup and stage, the first node it owns
  // (writes).
  Level fwd_full{0, -1, 0, 1, 0, nullptr, nullptr};
  int* d_own = nullptr;
  int fwd_group = 0;
  // Light upper levels (scan form, one tree): the levels above the bottom one
  // run inside the bottom level's backward launch, which has n_up more
  // workgroups for their nodes' local parts.  d_up_par: per workgroup (bottom
  // ones, then upper ones numbered from the lowest upper level) the upper
  // workgroups above it; d_up_need: arrivals that complete an upper
  // workgroup; d_up_cnt: its arrival counter (zero between launches).
  bool top_light = false;
  int n_up = 0;
  int* d_up_plan = nullptr;  // static table of each upper workgroup (see SegArgs)
  int up_plan_stride = 0, up_nw = 0, up_nch = 0;
  int2* d_up_par = nullptr;
  int* d_up_need = nullptr;
  unsigned* d_up_cnt = nullptr;
  std::vector<LevelPlan> plans;  // the plan the levels were built from
  bool segmented = false;
  bool scan = false;  // sweeps in scan form (the solver allows it; the autotuner may choose)
  int part_total = 0;
  int ntrees = 1;                // trees of the forest held by this slot
  // persistent iteration (one tree): per-level kernel arguments, hand-over
  // tables and counters; chain_state 0: not set up, 1: usable, -1: not usable
  void* d_chain_lev = nullptr;
  int2* d_chain_par = nullptr;
  int* d_chain_nchild = nullptr;
  unsigned* d_chain_cnt = nullptr;  // backward counts, then forward flags
  void* d_chain_sync = nullptr;
  int chain_total = 0, chain_nbm = 0, chain_state = 0;
  std::vector<int> chain_base;  // first workgroup of each level
  size_t chain_lds = 0;
};

// Unique ids of trees and forests (never reused).
uint64_t next_uid();

// A batch of trees as one forest (forest.cpp); map[map_off[k] + n] is the
// forest index of node n of tree k.  host_data = false: demand and price are
// left out (gathered on the device from the trees' slots).
TreeHost build_forest(const std::vector<const TreeHost*>& trees, std::vector<int>& map,
                      std::vector<int>& map_off, bool host_data = true);
// Copy the members' current demand and price into the forest (new version).
void refresh_forest_data(const std::vector<const TreeHost*>& trees, const std::vector<int>& map,
                         const std::vector<int>& map_off, TreeHost& f);

struct SolverState;

// Device-side pieces of a solver (defined in solver.hip).
struct DeviceNet;

}  // namespace tapg

struct tapg_network_s {
  tapg::NetworkHost h;
};

struct tapg_tree_s {
  tapg::TreeHost h;
};
