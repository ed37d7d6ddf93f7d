// Solver object shared by the C-ABI layer (api.cpp) and the device layer
// (solver.hip).
#pragma once

#include "internal.h"

namespace tapg {

template <typename T>
struct NetDev {
  // Sweep operands, column-major (element (r, k) at [k * ld + r]):
  // At = A' (nx x nx, ld LDX), Bt = B' (nu x nx, ld LDU), A (nx x nx, ld LDX),
  // B (nx x nu, ld LDX); stage factors Fbar, Kbar (N blocks of nu x nu, ld LDU).
  T *At = nullptr, *Bt = nullptr, *A = nullptr, *B = nullptr;
  T *xmin = nullptr, *xmax = nullptr, *xs = nullptr, *umin = nullptr, *umax = nullptr;
  T *F = nullptr, *Kb = nullptr;
  // CSR of B (nx rows) and of B' (nu rows); dense W_u (column-major, ld LDU)
  int *Brow = nullptr, *Bcol = nullptr, *Btrow = nullptr, *Btcol = nullptr;
  T *Bval = nullptr, *Btval = nullptr, *Wu = nullptr;
  // projector form of the stage factor (W_u = w I): CSR of G = (E E')^{-1} E
  // (ns rows) and of E' (nu rows)
  int *Grow = nullptr, *Gcol = nullptr, *Etrow = nullptr, *Etcol = nullptr;
  T *Gval = nullptr, *Etval = nullptr;
};

// A cached batch: the forest of its trees (keyed by their ids) and the
// device tables that map every tree's rows into the forest.
struct Batch {
  std::vector<uint64_t> versions;  // member data versions held by the forest
  TreeHost forest;
  std::vector<int> map, map_off;   // forest index of node n of tree k: map[map_off[k] + n]
  int* d_map = nullptr;
  int* d_tstart = nullptr;
  double* d_red = nullptr;         // per tree: cost, box and equality violations
};

struct DevExtra {
  // FP64 operands of the data step and of the cost evaluation.
  double *Gd = nullptr;    // nx x nd, col-major ld LDX
  double *Pd = nullptr;    // nu x nd, col-major ld LDU  (-E^+ Ed)
  double *Gbar = nullptr;  // N x (nu x nu), col-major ld LDU
  double *E = nullptr;     // ns x nu row-major
  double *Ed = nullptr;    // ns x nd row-major
  double *Wu = nullptr;    // nu x nu col-major ld LDU
  double *alpha0 = nullptr, *cE = nullptr;  // LDU
  double *red = nullptr;   // 8 doubles of reduction output
  double *Gm = nullptr;    // G = (E E')^{-1} E, ns x nu row-major (projector form)
};

}  // namespace tapg

struct tapg_solver_s {
  tapg::NetworkHost net;
  tapg_config cfg;
  std::vector<double> alpha0, cE, Wu;
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int LDX = 0, LDU = 0, LDY = 0;
  int N = 0;  // horizon of the factor step, 0 = not factored
  std::vector<double> Fbar, Kbar, Gbar;  // host FP64, N blocks of nu*nu row-major
  // Stage s is served by factor block fid[s]: consecutive stages whose Fbar
  // agree to rounding share the block of the later one (W_u = w I makes every
  // Fbar_s equal to Z Z' / w), so a sweep reloads its factor only on a change.
  std::vector<int> fid;
  int n_factor_blocks = 0;
  int* d_fid = nullptr;
  bool fp32 = false;
  tapg::NetDev<double> d64;
  tapg::NetDev<float> d32;
  tapg::DevExtra dx;
  std::map<uint64_t, tapg::Slot> slots;
  std::map<std::vector<uint64_t>, tapg::Batch> batches;
  std::map<std::string, std::vector<tapg::LevelPlan>> tuned;  // autotuned schedule per tree shape
  std::map<std::string, bool> tuned_scan;  // autotuned sweep form per tree shape
  std::map<std::string, int> tuned_fwd;    // autotuned forward grouping (scan form)
  std::map<std::string, bool> tuned_top;   // autotuned light upper levels (scan form, one tree)
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  bool use_graph = true;
  // structure of the network and weights (detected at creation)
  bool a_ident = false, wu_scalar = false;
  double wu = 1.0;
  bool seg_ok = false;  // segment kernels apply (nx, nu <= 128, B with few nonzeros)
  int nnzB = 0;
  // W_u = w I makes every stage factor Pi / w with Pi = I - E'(E E')^{-1} E;
  // the sweeps then apply it as (v - E'(G v)) / w when G is sparse
  bool proj = false;
  int nnzG = 0, nnzE = 0;
  // A = I as well (and nx <= 64): the sweeps can run in scan form, the
  // recursions unrolled into subtree and root-path sums (TAPG_SCAN=0: never).
  // Untuned slots use the segment form unless TAPG_SCAN=1; the autotuner times
  // both forms and keeps the faster per tree shape.
  bool scan = false;
  bool scan_default = false;
  tapg::Mat G;  // (E E')^{-1} E, ns x nu
  size_t lds_limit = 64 * 1024;  // dynamic LDS per workgroup (device attribute)
  // optional per-launch timing of the sweep kernels (HIP events around each
  // launch; graphs are bypassed while it is on)
  bool time_kernels = false;
  double hold_us = 2000.0;       // kernel timing: device hold ahead of a chunk's launches
  double wall_clock_mhz = 100.0; // rate of the device wall clock
  bool server_active = false;  // a tapg_server drives this solver (other calls refused)
  std::vector<hipEvent_t> tev;      // pairs, reused per chunk
  // backward stages, forward stages, iteration end, persistent iteration
  // (launches; for the persistent one, iterations covered)
  double kt_ms[4] = {0, 0, 0, 0};
  long long kt_n[4] = {0, 0, 0, 0};
};

namespace tapg {


int nb_template(int w);
std::vector<LevelPlan> plan_levels(const TreeHost& t, int nbmax, double node_us,
                                   double c_launch = 3.0, double c_stage = 0.25);
// Distinct plans of the planner under a spread of its cost constants: the
// candidates the autotuner times.
std::vector<std::vector<LevelPlan>> candidate_plans(const TreeHost& t, int nbmax, double node_us);
std::vector<LevelPlan> levels_from_env(const TreeHost& t, const char* spec);
std::vector<std::pair<int, int>> level_ranges(const TreeHost& t, const LevelPlan& L, int& wmax);
// One level over the stages [s, N-1] with groups of g consecutive nodes of stage s.
LevelPlan stage_plan(const TreeHost& t, int s, int g);

// A tree in flight in the serving loop: its iterate state lives in its own
// slot between forests (both dual buffers, control block, history).
struct LiveTree {
  const TreeHost* t = nullptr;
  Slot* own = nullptr;
  std::vector<double> p, q;
  double gamma = 0.0;
  bool warm = false;
  DevCtl ctl{};
  int it0 = 0;            // iterations done when it entered the current forest
  bool finished = false;
  tapg_result res{};
};
// Start a tree: dual (warm: its latest, else zero) and control block.
void dev_live_init(tapg_solver_s* S, LiveTree& j);
// Sweep the given trees as one forest from their current state.
void dev_live_enter(tapg_solver_s* S, const std::vector<LiveTree*>& js);
// One chunk of iterations; returns true if a tree stopped.
bool dev_live_chunk(tapg_solver_s* S, const std::vector<LiveTree*>& js);
// State back into every tree's own slot (results for the stopped ones, which
// are marked finished); the forest is freed.
void dev_live_leave(tapg_solver_s* S, const std::vector<LiveTree*>& js);

// Step size of a tree: cfg.gamma if positive, else 1 / (1.02 L) with L from
// the device power iteration, cached with the tree (api.cpp).
double solver_gamma(tapg_solver_s* solver, const TreeHost& t, Slot& sl);

// Batched solve shared by tapg_batch_solve and the server (api.cpp).
void batch_core(tapg_solver_s* solver, int ntrees, const tapg_tree* trees, const double* const* p,
                const double* const* q, const int* warm_start, double* const* u0_out,
                tapg_result* res, tapg_status* st_out);

// Device layer (solver.hip).
void dev_init(tapg_solver_s* S);             // streams, events, network buffers
void dev_release(tapg_solver_s* S);          // frees everything the solver owns
void dev_upload_factors(tapg_solver_s* S);   // Fbar/Kbar/Gbar to the device
Slot& dev_slot(tapg_solver_s* S, const TreeHost& t);  // allocate/upload as needed
void dev_solve(tapg_solver_s* S, const TreeHost& t, Slot& sl, const double* p,
               const double* q, bool warm, double gamma, tapg_result& res);
// Solve several trees in one set of launches (a forest); results go to each
// tree's own slot as after tapg_solve.
void dev_batch_solve(tapg_solver_s* S, const std::vector<const TreeHost*>& trees,
                     const std::vector<Slot*>& own, const double* const* p,
                     const double* const* q, const int* warm, const std::vector<double>& gamma,
                     tapg_result* res);
double dev_power(tapg_solver_s* S, const TreeHost& t, Slot& sl, int iters);
// Solve in the scratch array (no device allocation); per-stage kernels.
void dev_solve_noalloc(tapg_solver_s* S, const TreeHost& t, const double* p, const double* q,
                       double gamma, tapg_result& res, double* u0, double* u_out, double* x_out);
// Scratch bytes such a solve of the tree needs.
size_t dev_noalloc_bytes(const tapg_solver_s* S, const TreeHost& t);
// Duality gap G and dual objective F of the tree's current dual (FP64).
void dev_gap(tapg_solver_s* S, const TreeHost& t, Slot& sl, double* gap, double* dual_obj);
void dev_get_primal(tapg_solver_s* S, Slot& sl, double* u, double* x);
void dev_get_dual(tapg_solver_s* S, Slot& sl, double* y);
void dev_get_root_input(tapg_solver_s* S, Slot& sl, double* u0);
void dev_set_dual(tapg_solver_s* S, Slot& sl, const double* y);
int dev_get_history(tapg_solver_s* S, Slot& sl, double* h, int n);
void dev_set_kernel_timing(tapg_solver_s* S, bool on);
double dev_event_pair_us(tapg_solver_s* S);
void dev_free_slot(Slot& sl);
// Autotuner: time every candidate schedule of the tree (one tree) or of the
// batch's forest (several trees) and keep the fastest, for this slot and for
// later slots of the same shape.  Returns ms per iteration of the winner.
double dev_autotune(tapg_solver_s* S, const std::vector<const TreeHost*>& trees, int iters,
                    int* ncand);
// Free the forest (slot, graph and maps) cached for this exact batch, if any.
void dev_drop_batch(tapg_solver_s* S, const std::vector<uint64_t>& key);
// Free the device slot of one tree (its buffers, graph and results), if any.
void dev_drop_tree(tapg_solver_s* S, uint64_t uid);

}  // namespace tapg
