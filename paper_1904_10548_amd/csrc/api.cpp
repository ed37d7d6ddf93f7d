// C-ABI entry points: argument validation, host objects, the offline FP64
// factor step, and dispatch to the device layer.  No exception crosses the
// ABI; every failure becomes a tapg_status plus a thread-local message.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <sstream>

#include "solver.h"

namespace tapg {

namespace {
thread_local std::string g_last_error;
std::atomic<uint64_t> g_next_uid{1};
}  // namespace

uint64_t next_uid() { return g_next_uid.fetch_add(1); }

namespace {

bool finite_all(const double* p, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

template <typename F>
tapg_status guarded(F&& f) {
  try {
    clear_error();
    return f();
  } catch (const Fail& e) {
    set_error(e.msg);
    return e.code;
  } catch (const std::bad_alloc&) {
    set_error("host allocation failed");
    return TAPG_ENOMEM;
  } catch (const std::exception& e) {
    set_error(e.what());
    return TAPG_EINVAL;
  } catch (...) {
    set_error("unknown failure");
    return TAPG_EINVAL;
  }
}

[[noreturn]] void fail(tapg_status c, const std::string& m) { throw Fail{c, m}; }

void need(const void* p, const char* what) {
  if (p == nullptr) fail(TAPG_EINVAL, std::string(what) + " is NULL");
}
}  // namespace

void set_error(const std::string& msg) { g_last_error = msg; }
void clear_error() { g_last_error.clear(); }

// Offline factor step (the Engine's factorStep): the per-stage quantities of
// the Riccati-type recursion of the dual-gradient DP, Sec. 4.4.  Because the
// children's probabilities add up to the parent's and W_u, E do not depend on
// the node, the factor of node n is p_n-scaled from one per-stage factor:
//   Qbar_s = W_u + Pbar_{s+1},  Pbar_N = 0
//   Fbar_s = Z (Z' Qbar_s Z)^{-1} Z',  Kbar_s = Fbar_s W_u,
//   Gammabar_s = I - Fbar_s Qbar_s,    Pbar_s = W_u - W_u Fbar_s W_u.
static void factor_step(tapg_solver_s* S, int N) {
  const NetworkHost& h = S->net;
  const int nu = h.nu;
  const Mat Wu = Mat::from(S->Wu.data(), nu, nu);
  const Mat& Z = h.Z;
  const Mat Zt = transpose(Z);
  Mat P(nu, nu);
  S->Fbar.assign((size_t)N * nu * nu, 0.0);
  S->Kbar.assign((size_t)N * nu * nu, 0.0);
  S->Gbar.assign((size_t)N * nu * nu, 0.0);
  const Mat I = Mat::eye(nu);
  for (int s = N - 1; s >= 0; --s) {
    const Mat Q = add(Wu, P);
    Mat M = matmul(matmul(Zt, Q), Z);
    if (!cholesky(M)) fail(TAPG_ENUMERIC, "factor step: Z'(W_u + P)Z is not positive definite");
    Mat X = Zt;  // m x nu
    chol_solve(M, X);
    const Mat F = matmul(Z, X);
    const Mat Kb = matmul(F, Wu);
    const Mat G = add(I, matmul(F, Q), -1.0);
    Mat Pn = add(Wu, matmul(matmul(Wu, F), Wu), -1.0);
    for (int i = 0; i < nu; ++i)
      for (int j = i + 1; j < nu; ++j) {
        const double v = 0.5 * (Pn(i, j) + Pn(j, i));
        Pn(i, j) = v;
        Pn(j, i) = v;
      }
    std::copy(F.a.begin(), F.a.end(), S->Fbar.begin() + (size_t)s * nu * nu);
    std::copy(Kb.a.begin(), Kb.a.end(), S->Kbar.begin() + (size_t)s * nu * nu);
    std::copy(G.a.begin(), G.a.end(), S->Gbar.begin() + (size_t)s * nu * nu);
    if (!finite_all(F.a.data(), F.a.size())) fail(TAPG_ENUMERIC, "factor step: non-finite factor");
    P = Pn;
  }
  S->N = N;
  // Factor ids: stage s shares the block of stage s+1's representative when
  // the two Fbar agree to 16 ulp of the representative's largest entry
  S->fid.assign(N, 0);
  S->n_factor_blocks = N > 0 ? 1 : 0;
  for (int s = N - 1; s >= 0; --s) {
    if (s == N - 1) {
      S->fid[s] = s;
      continue;
    }
    const int rep = S->fid[s + 1];
    const double* Fr = S->Fbar.data() + (size_t)rep * nu * nu;
    const double* Fs = S->Fbar.data() + (size_t)s * nu * nu;
    double mx = 0.0, d = 0.0;
    for (size_t i = 0; i < (size_t)nu * nu; ++i) {
      mx = std::max(mx, std::fabs(Fr[i]));
      d = std::max(d, std::fabs(Fs[i] - Fr[i]));
    }
    if (d <= 16.0 * 2.220446049250313e-16 * mx) {
      S->fid[s] = rep;
    } else {
      S->fid[s] = s;
      S->n_factor_blocks++;
    }
  }
}

}  // namespace tapg

using namespace tapg;

extern "C" {

const char* tapg_last_error(void) { return g_last_error.c_str(); }

const char* tapg_version(void) { return "tapg 0.1 (gfx950)"; }

tapg_status tapg_network_create(int nx, int nu, int nd, int ns, const double* A, const double* B,
                                const double* Gd, const double* E, const double* Ed,
                                const double* xmin, const double* xmax, const double* xs,
                                const double* umin, const double* umax, tapg_network* out) {
  return guarded([&]() -> tapg_status {
    need(out, "out");
    *out = nullptr;
    if (nx < 1 || nu < 1 || nd < 1 || ns < 0 || nx > 256 || nu > 256 || ns >= nu || nd > 4096)
      fail(TAPG_EDIM, "need 1 <= nx, nu <= 256, 1 <= nd <= 4096 and 0 <= ns < nu");
    need(A, "A");
    need(B, "B");
    need(Gd, "Gd");
    if (ns > 0) {
      need(E, "E");
      need(Ed, "Ed");
    }
    need(xmin, "xmin");
    need(xmax, "xmax");
    need(xs, "xs");
    need(umin, "umin");
    need(umax, "umax");
    if (!finite_all(A, (size_t)nx * nx) || !finite_all(B, (size_t)nx * nu) ||
        !finite_all(Gd, (size_t)nx * nd) || (ns > 0 && !finite_all(E, (size_t)ns * nu)) ||
        (ns > 0 && !finite_all(Ed, (size_t)ns * nd)) || !finite_all(xmin, nx) ||
        !finite_all(xmax, nx) || !finite_all(xs, nx) || !finite_all(umin, nu) ||
        !finite_all(umax, nu))
      fail(TAPG_ENUMERIC, "non-finite network data");
    for (int i = 0; i < nu; ++i)
      if (umin[i] > umax[i]) fail(TAPG_EINVAL, "umin > umax at input " + std::to_string(i));
    for (int i = 0; i < nx; ++i)
      if (xmin[i] > xmax[i]) fail(TAPG_EINVAL, "xmin > xmax at state " + std::to_string(i));
    auto net = std::make_unique<tapg_network_s>();
    NetworkHost& h = net->h;
    h.nx = nx;
    h.nu = nu;
    h.nd = nd;
    h.ns = ns;
    h.A = Mat::from(A, nx, nx);
    h.B = Mat::from(B, nx, nu);
    h.Gd = Mat::from(Gd, nx, nd);
    h.E = ns > 0 ? Mat::from(E, ns, nu) : Mat(0, nu);
    h.Ed = ns > 0 ? Mat::from(Ed, ns, nd) : Mat(0, nd);
    h.xmin.assign(xmin, xmin + nx);
    h.xmax.assign(xmax, xmax + nx);
    h.xs.assign(xs, xs + nx);
    h.umin.assign(umin, umin + nu);
    h.umax.assign(umax, umax + nu);
    if (ns > 0) {
      if (!null_space_and_particular(h.E, h.Ed, h.Z, h.Pd))
        fail(TAPG_ENUMERIC, "E does not have full row rank");
    } else {
      h.Z = Mat::eye(nu);
      h.Pd = Mat(nu, nd);
    }
    *out = net.release();
    return TAPG_OK;
  });
}

void tapg_network_destroy(tapg_network net) { delete net; }

static void check_tree(const TreeHost& t) {
  // nodes_per_stage, ancestors (breadth-first, contiguous children), every
  // leaf at stage N-1, probabilities.
  if (t.mu[0] != 1) fail(TAPG_EINVAL, "nodes_per_stage[0] must be 1");
  for (int s = 0; s < t.N; ++s)
    if (t.mu[s] < 1) fail(TAPG_EINVAL, "nodes_per_stage[" + std::to_string(s) + "] < 1");
  if (t.anc[0] != -1) fail(TAPG_EINVAL, "ancestor[0] must be -1");
  for (int s = 1; s < t.N; ++s) {
    int prev = -1;
    for (int n = t.offset[s]; n < t.offset[s + 1]; ++n) {
      const int a = t.anc[n];
      if (a < t.offset[s - 1] || a >= t.offset[s])
        fail(TAPG_EINVAL, "ancestor of node " + std::to_string(n) + " is not in the previous stage");
      if (a < prev)
        fail(TAPG_EINVAL, "children are not contiguous / breadth-first at node " + std::to_string(n));
      prev = a;
    }
  }
  for (int n = 0; n < (t.N > 1 ? t.offset[t.N - 1] : 0); ++n)
    if (t.cend[n] <= t.cbeg[n])
      fail(TAPG_EINVAL, "node " + std::to_string(n) + " has no child but is not at the last stage");
  if (!(std::fabs(t.prob[0] - 1.0) <= 1e-12)) fail(TAPG_EINVAL, "prob[0] must be 1");
  for (int n = 0; n < t.K; ++n) {
    if (!(t.prob[n] > 0.0) || !std::isfinite(t.prob[n]))
      fail(TAPG_EINVAL, "prob[" + std::to_string(n) + "] must be positive and finite");
    if (t.cend[n] > t.cbeg[n]) {
      double s = 0.0;
      for (int c = t.cbeg[n]; c < t.cend[n]; ++c) s += t.prob[c];
      if (!(std::fabs(s - t.prob[n]) <= 1e-12 * t.prob[n] + 1e-300))
        fail(TAPG_EINVAL, "children's probabilities do not add up to node " + std::to_string(n));
    }
  }
}

tapg_status tapg_tree_create(int N, const int* nodes_per_stage, const int* ancestor,
                             const double* prob, int nd, const double* demand, const double* price,
                             tapg_tree* out) {
  return guarded([&]() -> tapg_status {
    need(out, "out");
    *out = nullptr;
    if (N < 1 || N > 100000) fail(TAPG_EDIM, "N must be in [1, 100000]");
    if (nd < 1) fail(TAPG_EDIM, "nd must be >= 1");
    need(nodes_per_stage, "nodes_per_stage");
    need(ancestor, "ancestor");
    need(prob, "prob");
    need(demand, "demand");
    need(price, "price");
    auto tr = std::make_unique<tapg_tree_s>();
    TreeHost& t = tr->h;
    t.uid = g_next_uid.fetch_add(1);
    t.version = 0;
    t.N = N;
    t.nd = nd;
    t.mu.assign(nodes_per_stage, nodes_per_stage + N);
    t.offset.assign(N + 1, 0);
    long long K = 0;
    for (int s = 0; s < N; ++s) {
      if (t.mu[s] < 1) fail(TAPG_EINVAL, "nodes_per_stage[" + std::to_string(s) + "] < 1");
      t.offset[s] = (int)K;
      K += t.mu[s];
      if (K > (1ll << 28)) fail(TAPG_EDIM, "tree too large");
    }
    t.offset[N] = (int)K;
    t.K = (int)K;
    t.anc.assign(ancestor, ancestor + K);
    t.prob.assign(prob, prob + K);
    t.stage.assign(K, 0);
    for (int s = 0; s < N; ++s)
      for (int n = t.offset[s]; n < t.offset[s + 1]; ++n) t.stage[n] = s;
    for (int n = 1; n < K; ++n)
      if (t.anc[n] < 0 || t.anc[n] >= n)
        fail(TAPG_EINVAL, "ancestor of node " + std::to_string(n) + " out of range");
    // first/last child of every node from the ancestors of the next stage
    // (contiguity is checked by check_tree)
    t.cbeg.assign(K, 0);
    t.cend.assign(K, 0);
    for (int s = 1; s < N; ++s) {
      for (int n = t.offset[s]; n < t.offset[s + 1]; ++n) {
        const int a = t.anc[n];
        if (t.cend[a] == 0) t.cbeg[a] = n;
        t.cend[a] = n + 1;
      }
    }
    check_tree(t);
    if (!finite_all(demand, (size_t)K * nd) || !finite_all(price, K))
      fail(TAPG_ENUMERIC, "non-finite demand or price");
    t.demand.assign(demand, demand + (size_t)K * nd);
    t.price.assign(price, price + K);
    *out = tr.release();
    return TAPG_OK;
  });
}

tapg_status tapg_tree_set_data(tapg_tree tree, const double* demand, const double* price) {
  return guarded([&]() -> tapg_status {
    need(tree, "tree");
    need(demand, "demand");
    need(price, "price");
    TreeHost& t = tree->h;
    if (!finite_all(demand, (size_t)t.K * t.nd) || !finite_all(price, t.K))
      fail(TAPG_ENUMERIC, "non-finite demand or price");
    std::copy(demand, demand + (size_t)t.K * t.nd, t.demand.begin());
    std::copy(price, price + t.K, t.price.begin());
    t.version += 1;
    return TAPG_OK;
  });
}

int tapg_tree_num_nodes(tapg_tree tree) { return tree ? tree->h.K : -1; }

tapg_status tapg_tree_dims(tapg_tree tree, int* N, int* K, int* nd) {
  return guarded([&]() -> tapg_status {
    need(tree, "tree");
    if (N) *N = tree->h.N;
    if (K) *K = tree->h.K;
    if (nd) *nd = tree->h.nd;
    return TAPG_OK;
  });
}

tapg_status tapg_network_dims(tapg_network net, int* nx, int* nu, int* nd, int* ns) {
  return guarded([&]() -> tapg_status {
    need(net, "net");
    if (nx) *nx = net->h.nx;
    if (nu) *nu = net->h.nu;
    if (nd) *nd = net->h.nd;
    if (ns) *ns = net->h.ns;
    return TAPG_OK;
  });
}

void tapg_tree_destroy(tapg_tree tree) { delete tree; }

tapg_status tapg_solver_create(tapg_network net, const tapg_config* cfg, tapg_solver* out) {
  return guarded([&]() -> tapg_status {
    need(out, "out");
    *out = nullptr;
    need(net, "net");
    need(cfg, "cfg");
    const NetworkHost& h = net->h;
    need(cfg->alpha0, "cfg->alpha0");
    need(cfg->c_energy, "cfg->c_energy");
    need(cfg->W_u, "cfg->W_u");
    if (!(cfg->W_alpha > 0) || !(cfg->W_s > 0) || !(cfg->W_x > 0))
      fail(TAPG_EINVAL, "W_alpha, W_s and W_x must be positive");
    if (cfg->max_iter < 1) fail(TAPG_EINVAL, "max_iter must be >= 1");
    if (cfg->check_every < 1) fail(TAPG_EINVAL, "check_every must be >= 1");
    if (cfg->precision != TAPG_FP64 && cfg->precision != TAPG_FP32)
      fail(TAPG_EINVAL, "precision must be TAPG_FP64 or TAPG_FP32");
    if (!std::isfinite(cfg->gamma) || !std::isfinite(cfg->tol)) fail(TAPG_EINVAL, "non-finite gamma/tol");
    if (cfg->beta_rule != TAPG_BETA_PAPER && cfg->beta_rule != TAPG_BETA_SIMPLE &&
        cfg->beta_rule != TAPG_BETA_ZERO)
      fail(TAPG_EINVAL, "beta_rule must be TAPG_BETA_PAPER, TAPG_BETA_SIMPLE or TAPG_BETA_ZERO");
    if (cfg->averaged_primal != 0 && cfg->averaged_primal != 1)
      fail(TAPG_EINVAL, "averaged_primal must be 0 or 1");
    if (!std::isfinite(cfg->gap_tol) || cfg->gap_tol < 0) fail(TAPG_EINVAL, "gap_tol must be >= 0");
    if (!finite_all(cfg->W_u, (size_t)h.nu * h.nu) || !finite_all(cfg->alpha0, h.nu) ||
        !finite_all(cfg->c_energy, h.nu))
      fail(TAPG_ENUMERIC, "non-finite weights");
    Mat W = Mat::from(cfg->W_u, h.nu, h.nu);
    for (int i = 0; i < h.nu; ++i)
      for (int j = 0; j < i; ++j)
        if (std::fabs(W(i, j) - W(j, i)) > 1e-12 * (std::fabs(W(i, j)) + std::fabs(W(j, i)) + 1e-300))
          fail(TAPG_EINVAL, "W_u is not symmetric");
    Mat Wc = W;
    if (!cholesky(Wc)) fail(TAPG_ENUMERIC, "W_u is not positive definite");
    auto S = std::make_unique<tapg_solver_s>();
    S->net = h;
    S->cfg = *cfg;
    S->alpha0.assign(cfg->alpha0, cfg->alpha0 + h.nu);
    S->cE.assign(cfg->c_energy, cfg->c_energy + h.nu);
    S->Wu.assign(cfg->W_u, cfg->W_u + (size_t)h.nu * h.nu);
    S->cfg.alpha0 = S->alpha0.data();
    S->cfg.c_energy = S->cE.data();
    S->cfg.W_u = S->Wu.data();
    S->device = cfg->device;
    S->stream = static_cast<hipStream_t>(cfg->hip_stream);
    S->fp32 = cfg->precision == TAPG_FP32;
    // The segment kernels (nx, nu <= 128) use a u-dimension padded to 128.
    const char* seg_env = std::getenv("TAPG_SEGMENTS");
    S->nnzB = 0;
    for (double v : h.B.a) S->nnzB += v != 0.0;
    S->seg_ok = h.nx <= 128 && h.nu <= 128 && S->nnzB <= 1024 &&
                !(seg_env && seg_env[0] == '0');
    S->LDX = round_up(h.nx, 16);
    S->LDU = S->seg_ok ? 128 : round_up(h.nu, 16);
    S->LDY = 2 * S->LDX + S->LDU;
    const char* env = std::getenv("TAPG_USE_GRAPH");
    S->use_graph = !(env && env[0] == '0');
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0)
      fail(TAPG_EDEVICE, "no HIP device available");
    if (cfg->device < 0 || cfg->device >= ndev) fail(TAPG_EDEVICE, "device ordinal out of range");
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, cfg->device) != hipSuccess)
      fail(TAPG_EDEVICE, "hipGetDeviceProperties failed");
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
      fail(TAPG_EDEVICE, std::string("this build targets gfx950; device is ") + prop.gcnArchName);
    try {
      dev_init(S.get());
    } catch (...) {
      dev_release(S.get());
      throw;
    }
    *out = S.release();
    return TAPG_OK;
  });
}

void tapg_solver_destroy(tapg_solver solver) {
  if (!solver) return;
  try {
    dev_release(solver);
  } catch (...) {
  }
  delete solver;
}

tapg_status tapg_factor_step(tapg_solver solver, int N) {
  return guarded([&]() -> tapg_status {
    need(solver, "solver");
    if (solver->server_active) fail(TAPG_ESTATE, "the solver is driven by a server");
    if (N < 1 || N > 100000) fail(TAPG_EDIM, "N must be in [1, 100000]");
    factor_step(solver, N);
    dev_upload_factors(solver);
    return TAPG_OK;
  });
}

tapg_status tapg_get_factors(tapg_solver solver, int stage, double* Fbar, double* Kbar,
                             double* Gbar) {
  return guarded([&]() -> tapg_status {
    need(solver, "solver");
    if (solver->N == 0) fail(TAPG_ESTATE, "factor step not run");
    if (stage < 0 || stage >= solver->N) fail(TAPG_EINVAL, "stage out of range");
    const size_t nn = (size_t)solver->net.nu * solver->net.nu;
    if (Fbar) std::copy_n(solver->Fbar.begin() + stage * nn, nn, Fbar);
    if (Kbar) std::copy_n(solver->Kbar.begin() + stage * nn, nn, Kbar);
    if (Gbar) std::copy_n(solver->Gbar.begin() + stage * nn, nn, Gbar);
    return TAPG_OK;
  });
}

tapg_status tapg_factor_blocks(tapg_solver solver, int* fid, int n, int* n_blocks) {
  return guarded([&]() -> tapg_status {
    need(solver, "solver");
    if (solver->N == 0) fail(TAPG_ESTATE, "factor step not run");
    if (fid) {
      if (n < solver->N) fail(TAPG_EINVAL, "fid holds fewer than N entries");
      std::copy(solver->fid.begin(), solver->fid.end(), fid);
    }
    if (n_blocks) *n_blocks = solver->n_factor_blocks;
    return TAPG_OK;
  });
}

static void check_pair_unserved(tapg_solver solver, tapg_tree tree) {
  need(solver, "solver");
  need(tree, "tree");
  if (solver->N == 0) fail(TAPG_ESTATE, "factor step not run");
  if (tree->h.N != solver->N)
    fail(TAPG_EDIM, "tree horizon " + std::to_string(tree->h.N) + " != factored horizon " +
                        std::to_string(solver->N));
  if (tree->h.nd != solver->net.nd) fail(TAPG_EDIM, "tree nd does not match the network");
}

static void check_pair(tapg_solver solver, tapg_tree tree) {
  need(solver, "solver");
  if (solver->server_active) fail(TAPG_ESTATE, "the solver is driven by a server");
  need(tree, "tree");
  if (solver->N == 0) fail(TAPG_ESTATE, "factor step not run");
  if (tree->h.N != solver->N)
    fail(TAPG_EDIM, "tree horizon " + std::to_string(tree->h.N) + " != factored horizon " +
                        std::to_string(solver->N));
  if (tree->h.nd != solver->net.nd) fail(TAPG_EDIM, "tree nd does not match the network");
}

}  // extern "C"

double tapg::solver_gamma(tapg_solver_s* solver, const TreeHost& t, Slot& sl) {
  if (solver->cfg.gamma > 0) return solver->cfg.gamma;
  if (!sl.L_valid) {
    const int it = solver->cfg.power_iters > 0 ? solver->cfg.power_iters : 100;
    sl.L = dev_power(solver, t, sl, it);
    if (!(sl.L > 0) || !std::isfinite(sl.L)) fail(TAPG_ENUMERIC, "power iteration failed");
    sl.L_valid = true;
  }
  return 1.0 / (1.02 * sl.L);
}

extern "C" {

tapg_status tapg_solve(tapg_solver solver, tapg_tree tree, const double* p, const double* q,
                       int warm_start, double* u0_out, tapg_result* res) {
  return guarded([&]() -> tapg_status {
    check_pair(solver, tree);
    need(p, "p");
    need(q, "q");
    if (!finite_all(p, solver->net.nx) || !finite_all(q, solver->net.nu))
      fail(TAPG_ENUMERIC, "non-finite p or q");
    const TreeHost& t = tree->h;
    Slot& sl = dev_slot(solver, t);
    const double gamma = solver_gamma(solver, t, sl);
    tapg_result r{};
    dev_solve(solver, t, sl, p, q, warm_start != 0, gamma, r);
    if (u0_out) dev_get_root_input(solver, sl, u0_out);  // the root is node 0
    if (res) *res = r;
    return r.converged || solver->cfg.tol <= 0 ? TAPG_OK : TAPG_ENOTCONV;
  });
}

tapg_status tapg_solve_noalloc(tapg_solver solver, tapg_tree tree, const double* p,
                               const double* q, double* u0_out, double* u_out, double* x_out,
                               tapg_result* res) {
  return guarded([&]() -> tapg_status {
    check_pair(solver, tree);
    need(p, "p");
    need(q, "q");
    if (!finite_all(p, solver->net.nx) || !finite_all(q, solver->net.nu))
      fail(TAPG_ENUMERIC, "non-finite p or q");
    if (solver->cfg.averaged_primal || solver->cfg.gap_tol > 0)
      fail(TAPG_EINVAL, "tapg_solve_noalloc: no averaged primal or gap test (they need buffers "
                        "of their own)");
    const TreeHost& t = tree->h;
    double gamma = solver->cfg.gamma;
    if (!(gamma > 0)) {  // the tree's estimate, if one was made (the power iteration allocates)
      auto it = solver->slots.find(t.uid);
      if (it == solver->slots.end() || !it->second.L_valid)
        fail(TAPG_EINVAL, "tapg_solve_noalloc: cfg.gamma <= 0 and no Lipschitz estimate for "
                          "this tree (call tapg_estimate_lipschitz or tapg_solve first)");
      gamma = 1.0 / (1.02 * it->second.L);
    }
    tapg_result r{};
    dev_solve_noalloc(solver, t, p, q, gamma, r, u0_out, u_out, x_out);
    if (res) *res = r;
    return r.converged || solver->cfg.tol <= 0 ? TAPG_OK : TAPG_ENOTCONV;
  });
}

tapg_status tapg_noalloc_bytes(tapg_solver solver, tapg_tree tree, size_t* bytes) {
  return guarded([&]() -> tapg_status {
    need(bytes, "bytes");
    check_pair_unserved(solver, tree);
    *bytes = dev_noalloc_bytes(solver, tree->h);
    return TAPG_OK;
  });
}

}  // extern "C"

namespace tapg {
// Batched solve shared by tapg_batch_solve and the server: validation, the
// step size of every tree, the forest solve and the root inputs.  st_out[k]
// is tree k's status (OK, ENOTCONV or ENUMERIC).
void batch_core(tapg_solver_s* solver, int ntrees, const tapg_tree* trees, const double* const* p,
                const double* const* q, const int* warm_start, double* const* u0_out,
                tapg_result* res, tapg_status* st_out) {
  need(solver, "solver");
  need(trees, "trees");
  need(p, "p");
  need(q, "q");
  if (ntrees < 1) fail(TAPG_EINVAL, "ntrees must be >= 1");
  if (solver->cfg.averaged_primal || solver->cfg.gap_tol > 0)
    fail(TAPG_EINVAL, "the averaged primal and the gap test are for single-tree solves (tapg_solve)");
  std::vector<const TreeHost*> th(ntrees);
  std::vector<Slot*> own(ntrees);
  std::vector<double> gamma(ntrees);
  std::vector<uint64_t> ids;
  for (int k = 0; k < ntrees; ++k) {
    check_pair_unserved(solver, trees[k]);
    need(p[k], "p[k]");
    need(q[k], "q[k]");
    if (!finite_all(p[k], solver->net.nx) || !finite_all(q[k], solver->net.nu))
      fail(TAPG_ENUMERIC, "non-finite p or q of tree " + std::to_string(k));
    th[k] = &trees[k]->h;
    ids.push_back(th[k]->uid);
  }
  std::sort(ids.begin(), ids.end());
  if (std::adjacent_find(ids.begin(), ids.end()) != ids.end())
    fail(TAPG_EINVAL, "a tree appears twice in the batch");
  for (int k = 0; k < ntrees; ++k) {
    own[k] = &dev_slot(solver, *th[k]);
    gamma[k] = solver_gamma(solver, *th[k], *own[k]);
  }
  std::vector<tapg_result> r(ntrees);
  dev_batch_solve(solver, th, own, p, q, warm_start, gamma, r.data());
  for (int k = 0; k < ntrees; ++k) {
    if (u0_out && u0_out[k]) dev_get_root_input(solver, *own[k], u0_out[k]);
    if (res) res[k] = r[k];
    tapg_status sk = TAPG_OK;
    if (own[k]->numeric) sk = TAPG_ENUMERIC;
    else if (!r[k].converged && solver->cfg.tol > 0) sk = TAPG_ENOTCONV;
    if (st_out) st_out[k] = sk;
  }
}
}  // namespace tapg

extern "C" {

tapg_status tapg_autotune(tapg_solver solver, int ntrees, const tapg_tree* trees, int iters,
                          double* ms_per_iter, int* candidates) {
  return guarded([&]() -> tapg_status {
    need(solver, "solver");
    need(trees, "trees");
    if (ntrees < 1) fail(TAPG_EINVAL, "ntrees must be >= 1");
    if (iters < 1 || iters > 100000) fail(TAPG_EINVAL, "iters must be in [1, 100000]");
    std::vector<const TreeHost*> th(ntrees);
    std::vector<uint64_t> ids;
    for (int k = 0; k < ntrees; ++k) {
      check_pair(solver, trees[k]);
      th[k] = &trees[k]->h;
      ids.push_back(th[k]->uid);
    }
    std::sort(ids.begin(), ids.end());
    if (std::adjacent_find(ids.begin(), ids.end()) != ids.end())
      fail(TAPG_EINVAL, "a tree appears twice in the batch");
    const double ms = dev_autotune(solver, th, iters, candidates);
    if (ms_per_iter) *ms_per_iter = ms;
    return TAPG_OK;
  });
}

// The device slot of a tree (ntrees = 1) or of a batch's forest, once solved or tuned.
static const Slot& solved_slot(tapg_solver solver, int ntrees, const tapg_tree* trees) {
  need(trees, "trees");
  if (ntrees < 1) fail(TAPG_EINVAL, "ntrees must be >= 1");
  uint64_t uid = 0;
  if (ntrees == 1) {
    need(trees[0], "tree");
    uid = trees[0]->h.uid;
  } else {
    std::vector<uint64_t> key(ntrees);
    for (int k = 0; k < ntrees; ++k) {
      need(trees[k], "tree");
      key[k] = trees[k]->h.uid;
    }
    auto bit = solver->batches.find(key);
    if (bit == solver->batches.end()) fail(TAPG_ESTATE, "this batch has not been solved or tuned");
    uid = bit->second.forest.uid;
  }
  auto it = solver->slots.find(uid);
  if (it == solver->slots.end()) fail(TAPG_ESTATE, "the tree has not been solved or tuned");
  return it->second;
}

tapg_status tapg_schedule_spec(tapg_solver solver, int ntrees, const tapg_tree* trees, char* buf,
                               int cap) {
  return guarded([&]() -> tapg_status {
    need(solver, "solver");
    need(buf, "buf");
    const Slot& sl = solved_slot(solver, ntrees, trees);
    std::string s;
    if (!sl.segmented) {
      s = "TAPG_SEGMENTS=0";
    } else {
      s = std::string("TAPG_SCAN=") + (sl.scan ? "1" : "0") + " TAPG_LEVELS=";
      for (size_t l = 0; l < sl.plans.size(); ++l)
        s += (l ? "," : "") + std::to_string(sl.plans[l].s_begin) + ":" +
             std::to_string(sl.plans[l].group);
      if (sl.scan) s += " TAPG_FWD_GROUP=" + std::to_string(sl.fwd_group);
      if (sl.scan && sl.top_light) s += " TAPG_TOP=1";
    }
    if ((int)s.size() + 1 > cap) fail(TAPG_EINVAL, "buffer too small for the schedule");
    std::memcpy(buf, s.c_str(), s.size() + 1);
    return TAPG_OK;
  });
}

tapg_status tapg_sweep_form(tapg_solver solver, int ntrees, const tapg_tree* trees, int* form,
                            int* bwd_launches) {
  return guarded([&]() -> tapg_status {
    need(solver, "solver");
    const Slot& sl = solved_slot(solver, ntrees, trees);
    int f = TAPG_FORM_STAGES;
    if (sl.segmented) f = sl.scan ? TAPG_FORM_SCAN : solver->proj ? TAPG_FORM_PROJECTOR : TAPG_FORM_SEGMENT;
    if (form) *form = f;
    if (bwd_launches)
      *bwd_launches = !sl.segmented                  ? sl.N
                      : (sl.top_light && sl.n_up > 0) ? 1  // upper levels in the bottom launch
                                                      : (int)sl.levels.size();
    return TAPG_OK;
  });
}

tapg_status tapg_solver_forget(tapg_solver solver, tapg_tree tree) {
  return guarded([&]() -> tapg_status {
    need(solver, "solver");
    need(tree, "tree");
    if (solver->server_active) fail(TAPG_ESTATE, "the solver is driven by a server");
    const uint64_t uid = tree->h.uid;
    std::vector<std::vector<uint64_t>> keys;
    for (const auto& kv : solver->batches)
      if (std::find(kv.first.begin(), kv.first.end(), uid) != kv.first.end()) keys.push_back(kv.first);
    for (const auto& k : keys) dev_drop_batch(solver, k);
    dev_drop_tree(solver, uid);
    return TAPG_OK;
  });
}

tapg_status tapg_batch_solve(tapg_solver solver, int ntrees, const tapg_tree* trees,
                             const double* const* p, const double* const* q, const int* warm_start,
                             double* const* u0_out, tapg_result* res) {
  return guarded([&]() -> tapg_status {
    if (solver && solver->server_active) fail(TAPG_ESTATE, "the solver is driven by a server");
    std::vector<tapg_status> sk(std::max(ntrees, 1), TAPG_OK);
    batch_core(solver, ntrees, trees, p, q, warm_start, u0_out, res, sk.data());
    tapg_status worst = TAPG_OK;
    for (int k = 0; k < ntrees; ++k) {
      if (sk[k] == TAPG_ENUMERIC) worst = TAPG_ENUMERIC;
      else if (worst == TAPG_OK && sk[k] == TAPG_ENOTCONV) worst = TAPG_ENOTCONV;
    }
    if (worst == TAPG_ENUMERIC) set_error("a tree of the batch has a non-finite dual residual");
    return worst;
  });
}

static Slot& existing_slot(tapg_solver solver, tapg_tree tree) {
  check_pair(solver, tree);
  auto it = solver->slots.find(tree->h.uid);
  if (it == solver->slots.end() || !it->second.has_result)
    fail(TAPG_ESTATE, "tree has not been solved on this solver");
  return it->second;
}

tapg_status tapg_get_primal(tapg_solver solver, tapg_tree tree, double* u, double* x) {
  return guarded([&]() -> tapg_status {
    Slot& sl = existing_slot(solver, tree);
    dev_get_primal(solver, sl, u, x);
    return TAPG_OK;
  });
}

tapg_status tapg_get_dual(tapg_solver solver, tapg_tree tree, double* y) {
  return guarded([&]() -> tapg_status {
    need(y, "y");
    check_pair(solver, tree);
    auto it = solver->slots.find(tree->h.uid);
    if (it == solver->slots.end() || !it->second.has_dual)
      fail(TAPG_ESTATE, "no dual iterate for this tree");
    dev_get_dual(solver, it->second, y);
    return TAPG_OK;
  });
}

tapg_status tapg_set_dual(tapg_solver solver, tapg_tree tree, const double* y) {
  return guarded([&]() -> tapg_status {
    need(y, "y");
    check_pair(solver, tree);
    const size_t m = (size_t)tree->h.K * (2 * solver->net.nx + solver->net.nu);
    if (!finite_all(y, m)) fail(TAPG_ENUMERIC, "non-finite dual");
    Slot& sl = dev_slot(solver, tree->h);
    dev_set_dual(solver, sl, y);
    return TAPG_OK;
  });
}

tapg_status tapg_residual_history(tapg_solver solver, tapg_tree tree, double* hist, int n,
                                  int* written) {
  return guarded([&]() -> tapg_status {
    need(hist, "hist");
    Slot& sl = existing_slot(solver, tree);
    const int w = dev_get_history(solver, sl, hist, std::max(0, n));
    if (written) *written = w;
    return TAPG_OK;
  });
}

tapg_status tapg_residuals(tapg_solver solver, tapg_tree tree, tapg_result* res) {
  return guarded([&]() -> tapg_status {
    need(res, "res");
    Slot& sl = existing_slot(solver, tree);
    if (!sl.gap_valid && !sl.numeric) {  // (a diverged dual has no gap: NaN)
      Slot& cur = dev_slot(solver, tree->h);  // the tree's current data on the device
      double gap = 0.0, F = 0.0;
      dev_gap(solver, tree->h, cur, &gap, &F);
    }
    *res = sl.last;
    return TAPG_OK;
  });
}

tapg_status tapg_estimate_lipschitz(tapg_solver solver, tapg_tree tree, int iters, double* L) {
  return guarded([&]() -> tapg_status {
    need(L, "L");
    check_pair(solver, tree);
    if (iters < 1) fail(TAPG_EINVAL, "iters must be >= 1");
    Slot& sl = dev_slot(solver, tree->h);
    *L = dev_power(solver, tree->h, sl, iters);
    if (!(*L > 0) || !std::isfinite(*L)) fail(TAPG_ENUMERIC, "power iteration failed");
    sl.L = *L;  // used by tapg_solve when cfg.gamma <= 0
    sl.L_valid = true;
    return TAPG_OK;
  });
}

tapg_status tapg_plan_schedule(tapg_tree tree, int precision, const char* levels, int* out,
                               int cap, int* nlevels) {
  return guarded([&]() -> tapg_status {
    need(tree, "tree");
    need(nlevels, "nlevels");
    if (precision != TAPG_FP64 && precision != TAPG_FP32) fail(TAPG_EINVAL, "bad precision");
    const TreeHost& t = tree->h;
    const int nbmax = kSegNbMax;
    std::vector<LevelPlan> plans =
        (levels && levels[0]) ? levels_from_env(t, levels)
                              : plan_levels(t, nbmax, 114.0 * 114.0 / 64.0 / 2400.0);
    *nlevels = (int)plans.size();
    for (size_t l = 0; l < plans.size(); ++l) {
      int wmax = 0;
      level_ranges(t, plans[l], wmax);
      if (wmax > nbmax)
        fail(TAPG_EINVAL, "segment schedule: a workgroup would hold more than " +
                              std::to_string(nbmax) + " nodes of one stage");
      if (out && (int)l < cap) {
        out[5 * l + 0] = plans[l].s_begin;
        out[5 * l + 1] = plans[l].s_end;
        out[5 * l + 2] = plans[l].group;
        out[5 * l + 3] = plans[l].n_wg;
        out[5 * l + 4] = wmax;
      }
    }
    return TAPG_OK;
  });
}

tapg_status tapg_kernel_timing(tapg_solver solver, int enable) {
  return guarded([&]() -> tapg_status {
    need(solver, "solver");
    if (solver->server_active) fail(TAPG_ESTATE, "the solver is driven by a server");
    dev_set_kernel_timing(solver, enable != 0);
    return TAPG_OK;
  });
}

tapg_status tapg_event_pair_overhead(tapg_solver solver, double* us) {
  return guarded([&]() -> tapg_status {
    need(solver, "solver");
    need(us, "us");
    if (solver->server_active) fail(TAPG_ESTATE, "the solver is driven by a server");
    *us = dev_event_pair_us(solver);
    return TAPG_OK;
  });
}

tapg_status tapg_kernel_times(tapg_solver solver, double* ms, long long* launches) {
  return guarded([&]() -> tapg_status {
    need(solver, "solver");
    need(ms, "ms");
    need(launches, "launches");
    for (int k = 0; k < 4; ++k) {
      ms[k] = solver->kt_ms[k];
      launches[k] = solver->kt_n[k];
    }
    return TAPG_OK;
  });
}

}  // extern "C"
