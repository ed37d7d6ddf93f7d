// Host-code checks run under AddressSanitizer + UndefinedBehaviorSanitizer and
// under ThreadSanitizer (the CPU tests build this driver with the library's
// host sources and the stand-in device layer of mock_device.cpp).  It drives
// the C ABI through the host paths: input validation of networks, trees and
// configurations, the JSON reader (the instance files given on the command
// line, every truncation of them and seeded random byte mutations), the
// factor step (host linear algebra), the sweep planner, and the request
// server's worker thread with concurrent clients (the forest builder runs on
// every forest it forms).  Exit status 0 when every check holds.
//
//   driver <dir with network.json controllerconfig.json scenarioTree.json
//           forecaster.json state.json> <scratch dir>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <thread>
#include <vector>

#include "tapg.h"

namespace {

int g_checks = 0, g_failed = 0;

#define CHECK(cond)                                                                      \
  do {                                                                                   \
    ++g_checks;                                                                          \
    if (!(cond)) {                                                                       \
      ++g_failed;                                                                        \
      std::fprintf(stderr, "CHECK failed at line %d: %s (%s)\n", __LINE__, #cond,        \
                   tapg_last_error());                                                   \
    }                                                                                    \
  } while (0)

struct Rng {  // xorshift64*
  uint64_t s;
  explicit Rng(uint64_t seed) : s(seed ? seed : 1) {}
  uint64_t next() {
    s ^= s >> 12;
    s ^= s << 25;
    s ^= s >> 27;
    return s * 2685821657736338717ull;
  }
  double uniform() { return (double)(next() >> 11) * (1.0 / 9007199254740992.0); }
  int below(int n) { return (int)(next() % (uint64_t)n); }
};

std::string slurp(const std::string& p) {
  std::ifstream f(p, std::ios::binary);
  std::stringstream ss;
  ss << f.rdbuf();
  return ss.str();
}

void spit(const std::string& p, const std::string& text) {
  std::ofstream f(p, std::ios::binary | std::ios::trunc);
  f << text;
}

// ------------------------------------------------------------------ JSON --

void check_json_files(const std::string& dir, const std::string& tmp) {
  const std::string net_p = dir + "/network.json", cfg_p = dir + "/controllerconfig.json",
                    tree_p = dir + "/scenarioTree.json", fc_p = dir + "/forecaster.json",
                    st_p = dir + "/state.json";
  tapg_network net = nullptr;
  CHECK(tapg_network_from_json(net_p.c_str(), &net) == TAPG_OK);
  int nx = 0, nu = 0, nd = 0, ns = 0;
  CHECK(tapg_network_dims(net, &nx, &nu, &nd, &ns) == TAPG_OK);
  tapg_tree tree = nullptr;
  CHECK(tapg_tree_from_json(tree_p.c_str(), fc_p.c_str(), &tree) == TAPG_OK);
  int N = 0, K = 0, tnd = 0;
  CHECK(tapg_tree_dims(tree, &N, &K, &tnd) == TAPG_OK && tnd == nd);
  std::vector<double> dem((size_t)K * nd), pr(K), x(nx), q(nu);
  CHECK(tapg_tree_data_from_json(tree_p.c_str(), fc_p.c_str(), K, nd, dem.data(), pr.data()) ==
        TAPG_OK);
  CHECK(tapg_tree_data_from_json(tree_p.c_str(), fc_p.c_str(), K + 1, nd, dem.data(),
                                 pr.data()) == TAPG_EDIM);
  tapg_config cfg;
  std::vector<double> a0(nu), ce(nu), wu((size_t)nu * nu);
  CHECK(tapg_config_from_json(cfg_p.c_str(), nu, &cfg, a0.data(), ce.data(), wu.data()) ==
        TAPG_OK);
  CHECK(tapg_state_from_json(st_p.c_str(), nx, nu, x.data(), q.data()) == TAPG_OK);
  tapg_tree_destroy(tree);
  tapg_network_destroy(net);

  // every truncation of each file is an error, never a crash
  const std::string bad = tmp + "/truncated.json";
  int n_trunc = 0;
  for (const std::string& p : {net_p, tree_p, fc_p, cfg_p, st_p}) {
    const std::string text = slurp(p);
    const size_t step = text.size() > 20000 ? text.size() / 4000 : 1;
    for (size_t len = 0; len < text.size(); len += step) {
      std::string cut = text.substr(0, len);
      while (!cut.empty() && (cut.back() == ' ' || cut.back() == '\n')) cut.pop_back();
      if (cut.size() + 2 >= text.size()) continue;  // only the closing brace missing at most
      spit(bad, cut);
      tapg_network n2 = nullptr;
      tapg_tree t2 = nullptr;
      tapg_status s;
      if (p == net_p) s = tapg_network_from_json(bad.c_str(), &n2);
      else if (p == tree_p) s = tapg_tree_from_json(bad.c_str(), fc_p.c_str(), &t2);
      else if (p == fc_p) s = tapg_tree_from_json(tree_p.c_str(), bad.c_str(), &t2);
      else if (p == cfg_p) s = tapg_config_from_json(bad.c_str(), nu, &cfg, a0.data(), ce.data(),
                                                     wu.data());
      else s = tapg_state_from_json(bad.c_str(), nx, nu, x.data(), q.data());
      CHECK(s != TAPG_OK);
      if (n2) tapg_network_destroy(n2);
      if (t2) tapg_tree_destroy(t2);
      ++n_trunc;
    }
  }
  // seeded random mutations: any status, but memory-safe and no UB
  Rng rng(20190424);
  const char alphabet[] = "{}[],:\"\\-+.eE0123456789 \ntruefalsn\x01\xff";
  int n_mut = 0;
  for (const std::string& p : {net_p, tree_p, cfg_p}) {
    const std::string text = slurp(p);
    for (int m = 0; m < 400; ++m) {
      std::string t = text;
      const int edits = 1 + rng.below(4);
      for (int e = 0; e < edits; ++e) {
        const size_t at = (size_t)rng.below((int)t.size());
        const int op = rng.below(3);
        const char c = alphabet[rng.below((int)sizeof(alphabet) - 1)];
        if (op == 0) t[at] = c;
        else if (op == 1) t.insert(t.begin() + (long)at, c);
        else t.erase(at, 1 + (size_t)rng.below(8));
        if (t.empty()) t = "{";
      }
      spit(bad, t);
      tapg_network n2 = nullptr;
      tapg_tree t2 = nullptr;
      if (p == net_p) (void)tapg_network_from_json(bad.c_str(), &n2);
      else if (p == tree_p) (void)tapg_tree_from_json(bad.c_str(), fc_p.c_str(), &t2);
      else (void)tapg_config_from_json(bad.c_str(), nu, &cfg, a0.data(), ce.data(), wu.data());
      if (n2) tapg_network_destroy(n2);
      if (t2) tapg_tree_destroy(t2);
      ++n_mut;
    }
  }
  std::printf("json: %d truncations, %d mutations\n", n_trunc, n_mut);
}

// ------------------------------------------------- networks and trees --

struct Net {
  int nx = 4, nu = 6, nd = 3, ns = 2;
  std::vector<double> A, B, Gd, E, Ed, xmin, xmax, xs, umin, umax;
  explicit Net(Rng& r) {
    A.assign(nx * nx, 0.0);
    for (int i = 0; i < nx; ++i) A[i * nx + i] = 1.0;
    B.resize(nx * nu);
    for (double& v : B) v = r.uniform() < 0.4 ? r.uniform() - 0.5 : 0.0;
    Gd.resize(nx * nd);
    for (double& v : Gd) v = -r.uniform();
    E.resize(ns * nu);
    for (double& v : E) v = r.uniform() - 0.5;
    Ed.resize(ns * nd);
    for (double& v : Ed) v = r.uniform();
    xmin.assign(nx, 1.0);
    xmax.assign(nx, 10.0);
    xs.assign(nx, 3.0);
    umin.assign(nu, 0.0);
    umax.assign(nu, 5.0);
  }
  tapg_status create(tapg_network* out) const {
    return tapg_network_create(nx, nu, nd, ns, A.data(), B.data(), Gd.data(), E.data(),
                               Ed.data(), xmin.data(), xmax.data(), xs.data(), umin.data(),
                               umax.data(), out);
  }
};

struct Tree {
  int N = 0, nd = 3;
  std::vector<int> mu, anc;
  std::vector<double> prob, dem, price;
  Tree(Rng& r, int N_, int max_children, int nd_) : N(N_), nd(nd_) {
    mu.push_back(1);
    anc.push_back(-1);
    prob.push_back(1.0);
    int first = 0;
    for (int s = 1; s < N; ++s) {
      int cnt = 0;
      for (int v = first; v < first + mu.back(); ++v) {
        const int c = 1 + r.below(max_children);
        for (int k = 0; k < c; ++k) {
          anc.push_back(v);
          prob.push_back(prob[v] / c);
        }
        cnt += c;
      }
      first += mu.back();
      mu.push_back(cnt);
    }
    const int K = (int)anc.size();
    dem.resize((size_t)K * nd);
    for (double& v : dem) v = r.uniform();
    price.resize(K);
    for (double& v : price) v = 0.5 + r.uniform();
  }
  int K() const { return (int)anc.size(); }
  tapg_status create(tapg_tree* out) const {
    return tapg_tree_create(N, mu.data(), anc.data(), prob.data(), nd, dem.data(), price.data(),
                            out);
  }
};

void check_validation(Rng& rng) {
  Net net(rng);
  tapg_network h = nullptr;
  CHECK(net.create(&h) == TAPG_OK);
  tapg_network_destroy(h);
  {
    Net b = net;
    b.E = std::vector<double>(b.ns * b.nu, 0.0);  // rank deficient
    h = nullptr;
    CHECK(b.create(&h) == TAPG_ENUMERIC && h == nullptr);
  }
  {
    Net b = net;
    b.A[3] = NAN;
    CHECK(b.create(&h) != TAPG_OK);
  }
  {
    Net b = net;
    b.umin[2] = 9.0;
    CHECK(b.create(&h) == TAPG_EINVAL);
  }
  {
    Net b = net;
    b.nx = 0;
    CHECK(b.create(&h) != TAPG_OK);
  }
  CHECK(tapg_network_create(4, 6, 3, 2, nullptr, net.B.data(), net.Gd.data(), net.E.data(),
                            net.Ed.data(), net.xmin.data(), net.xmax.data(), net.xs.data(),
                            net.umin.data(), net.umax.data(), &h) == TAPG_EINVAL);

  for (int trial = 0; trial < 30; ++trial) {
    Tree t(rng, 2 + rng.below(10), 1 + rng.below(4), 3);
    tapg_tree th = nullptr;
    CHECK(t.create(&th) == TAPG_OK);
    CHECK(tapg_tree_num_nodes(th) == t.K());
    std::vector<double> d2 = t.dem, p2 = t.price;
    CHECK(tapg_tree_set_data(th, d2.data(), p2.data()) == TAPG_OK);
    tapg_tree_destroy(th);
    if (t.K() > 1) {
      Tree b = t;
      b.anc[b.K() - 1] = b.K() + 5;  // ancestor out of range
      CHECK(b.create(&th) == TAPG_EINVAL);
      Tree c = t;
      c.prob[c.K() - 1] *= 1.5;  // children no longer add up to the parent
      CHECK(c.create(&th) == TAPG_EINVAL);
      Tree d = t;
      d.mu[0] = 0;  // no root (K shrinks, so the arrays still cover it)
      CHECK(d.create(&th) != TAPG_OK);
    }
  }
}

// ------------------------------------------------------------- planner --

void check_planner(Rng& rng) {
  const char* specs[] = {nullptr, "0:1", "0:1,2:1", "0:2,3:1,5:4", "", "1:1", "0:1,0:1",
                         "0:1,2:x", "0:3", "0:1,99:1", "0:1,2:1,4:1,6:1", "0:4,1:2"};
  int out[5 * 64];
  for (int trial = 0; trial < 40; ++trial) {
    Tree t(rng, 2 + rng.below(14), 1 + rng.below(5), 2);
    tapg_tree th = nullptr;
    CHECK(t.create(&th) == TAPG_OK);
    for (const char* spec : specs)
      for (int prec = 0; prec < 2; ++prec) {
        int nl = -1;
        const tapg_status s = tapg_plan_schedule(th, prec, spec, out, 64, &nl);
        if (s == TAPG_OK) {
          CHECK(nl >= 1);
          int covered = 0;
          for (int l = 0; l < nl && l < 64; ++l) {
            CHECK(out[5 * l] == covered);
            CHECK(out[5 * l + 1] >= out[5 * l]);
            covered = out[5 * l + 1] + 1;
          }
          CHECK(covered == t.N);
        } else {
          CHECK(s == TAPG_EINVAL || s == TAPG_EDIM);
        }
      }
    tapg_tree_destroy(th);
  }
}

// --------------------------------------------- solver and factor step --

tapg_config make_cfg(int nu, std::vector<double>& a0, std::vector<double>& ce,
                     std::vector<double>& wu) {
  a0.assign(nu, 1.0);
  ce.assign(nu, 0.5);
  wu.assign((size_t)nu * nu, 0.0);
  for (int i = 0; i < nu; ++i) wu[(size_t)i * nu + i] = 100.0;
  wu[1] = wu[nu] = 3.0;
  tapg_config c;
  std::memset(&c, 0, sizeof(c));
  c.W_alpha = 1.0;
  c.W_s = 50.0;
  c.W_x = 1e3;
  c.alpha0 = a0.data();
  c.c_energy = ce.data();
  c.W_u = wu.data();
  c.gamma = 1e-3;
  c.tol = 1e-4;
  c.max_iter = 1000;
  c.check_every = 10;
  return c;
}

void check_solver(Rng& rng) {
  Net net(rng);
  tapg_network h = nullptr;
  CHECK(net.create(&h) == TAPG_OK);
  std::vector<double> a0, ce, wu;
  tapg_config c = make_cfg(net.nu, a0, ce, wu);
  tapg_solver S = nullptr;
  {
    tapg_config b = c;
    b.W_s = 0.0;
    CHECK(tapg_solver_create(h, &b, &S) == TAPG_EINVAL);
    b = c;
    b.gamma = NAN;
    CHECK(tapg_solver_create(h, &b, &S) == TAPG_EINVAL);
    b = c;
    std::vector<double> w2 = wu;
    w2[1] = 7.0;  // not symmetric
    b.W_u = w2.data();
    CHECK(tapg_solver_create(h, &b, &S) == TAPG_EINVAL);
    b = c;
    b.beta_rule = 9;
    CHECK(tapg_solver_create(h, &b, &S) == TAPG_EINVAL);
  }
  CHECK(tapg_solver_create(h, &c, &S) == TAPG_OK);
  CHECK(tapg_factor_step(S, 0) == TAPG_EDIM);
  const int N = 24;
  CHECK(tapg_factor_step(S, N) == TAPG_OK);
  const int nu = net.nu;
  std::vector<double> F((size_t)nu * nu), Kb((size_t)nu * nu), G((size_t)nu * nu);
  for (int s = 0; s < N; ++s) {
    CHECK(tapg_get_factors(S, s, F.data(), Kb.data(), G.data()) == TAPG_OK);
    bool fin = true;
    for (int i = 0; i < nu * nu; ++i) fin = fin && std::isfinite(F[i]) && std::isfinite(G[i]);
    CHECK(fin);
  }
  CHECK(tapg_get_factors(S, N, F.data(), Kb.data(), G.data()) != TAPG_OK);
  std::vector<int> fid(N);
  int nb = 0;
  CHECK(tapg_factor_blocks(S, fid.data(), N, &nb) == TAPG_OK && nb >= 1 && nb <= N);
  tapg_solver_destroy(S);
  tapg_network_destroy(h);
}

// -------------------------------------------------------------- server --

void check_server(Rng& rng) {
  Net net(rng);
  tapg_network h = nullptr;
  CHECK(net.create(&h) == TAPG_OK);
  std::vector<double> a0, ce, wu;
  tapg_config c = make_cfg(net.nu, a0, ce, wu);
  tapg_solver S = nullptr;
  CHECK(tapg_solver_create(h, &c, &S) == TAPG_OK);
  const int N = 6;
  CHECK(tapg_factor_step(S, N) == TAPG_OK);
  std::vector<Tree> trees;
  std::vector<tapg_tree> th;
  for (int k = 0; k < 6; ++k) {
    trees.emplace_back(rng, N, 1 + rng.below(3), net.nd);
    th.push_back(nullptr);
    CHECK(trees.back().create(&th.back()) == TAPG_OK);
  }
  tapg_server srv = nullptr;
  CHECK(tapg_server_create(S, (size_t)1 << 30, 4, &srv) == TAPG_OK);
  CHECK(tapg_factor_step(S, N) == TAPG_ESTATE);  // the server owns the solver

  const int n_clients = 4, per_client = 40;
  std::vector<int> bad(n_clients, 0);
  std::vector<std::thread> clients;
  for (int cl = 0; cl < n_clients; ++cl)
    clients.emplace_back([&, cl] {
      std::vector<double> p(net.nx, 5.0), q(net.nu), u0(net.nu);
      for (int r = 0; r < per_client; ++r) {
        for (int i = 0; i < net.nu; ++i) q[i] = (double)(cl * 1000 + r) + 0.25 * i;
        long long ticket = 0;
        if (tapg_server_submit(srv, th[(cl + r) % th.size()], p.data(), q.data(), cl % 3,
                               &ticket) != TAPG_OK) {
          ++bad[cl];
          continue;
        }
        tapg_result res;
        double lat = 0.0;
        const tapg_status st = tapg_server_poll(srv, ticket, -1, u0.data(), &res, &lat);
        if (st != TAPG_OK || res.converged != 1 || !(lat >= 0.0)) ++bad[cl];
        for (int i = 0; i < net.nu; ++i)
          if (u0[i] != q[i]) ++bad[cl];  // the result of this request, not another's
        if (r % 7 == 0) {  // a poll of a released ticket
          if (tapg_server_poll(srv, ticket, 0, nullptr, nullptr, nullptr) == TAPG_OK) ++bad[cl];
        }
      }
    });
  for (auto& t : clients) t.join();
  for (int cl = 0; cl < n_clients; ++cl) CHECK(bad[cl] == 0);
  long long batches = 0, solved = 0;
  double busy = 0.0;
  int pending = -1;
  CHECK(tapg_server_stats(srv, &batches, &solved, &busy, &pending) == TAPG_OK);
  CHECK(solved == n_clients * per_client && pending == 0 && batches >= 1);
  tapg_server_destroy(srv);

  // a budget no request fits: every request completes with TAPG_ENOMEM
  CHECK(tapg_server_create(S, 16, 4, &srv) == TAPG_OK);
  {
    std::vector<double> p(net.nx, 5.0), q(net.nu, 1.0), u0(net.nu);
    long long t1 = 0;
    CHECK(tapg_server_submit(srv, th[0], p.data(), q.data(), 0, &t1) == TAPG_OK);
    CHECK(tapg_server_poll(srv, t1, -1, u0.data(), nullptr, nullptr) == TAPG_ENOMEM);
  }
  tapg_server_destroy(srv);

  // a failure while setting up a set completes every request of the set
  CHECK(tapg_server_create(S, (size_t)1 << 30, 8, &srv) == TAPG_OK);
  {
    std::vector<double> p(net.nx, 5.0), q(net.nu, 2.0), u0(net.nu);
    setenv("TAPG_TEST_SERVER_SETUP_FAIL", "2", 1);
    std::vector<long long> tk(3);
    for (int k = 0; k < 3; ++k)
      CHECK(tapg_server_submit(srv, th[k], p.data(), q.data(), k, &tk[k]) == TAPG_OK);
    int failed = 0;
    for (int k = 0; k < 3; ++k) {
      const tapg_status st = tapg_server_poll(srv, tk[k], -1, u0.data(), nullptr, nullptr);
      failed += st == TAPG_EDEVICE;
      CHECK(st == TAPG_OK || st == TAPG_EDEVICE);
    }
    CHECK(failed >= 1);
    unsetenv("TAPG_TEST_SERVER_SETUP_FAIL");
  }
  // destroying the server with requests queued completes them (no leak, no wait)
  {
    std::vector<double> p(net.nx, 5.0), q(net.nu, 4.0);
    for (int k = 0; k < 20; ++k) {
      long long t = 0;
      CHECK(tapg_server_submit(srv, th[k % th.size()], p.data(), q.data(), k, &t) == TAPG_OK);
    }
  }
  tapg_server_destroy(srv);
  for (tapg_tree t : th) tapg_tree_destroy(t);
  tapg_solver_destroy(S);
  tapg_network_destroy(h);
}

void check_control_output(const std::string& tmp) {
  tapg_result r;
  std::memset(&r, 0, sizeof(r));
  r.iters = 3;
  r.dual_gap = NAN;
  const double u[3] = {1.0, -0.0, 1e-300};
  const std::string p = tmp + "/controlOutput.json";
  CHECK(tapg_control_output_write(p.c_str(), 3, u, &r, TAPG_OK) == TAPG_OK);
  CHECK(slurp(p).find("\"dual_gap\": null") != std::string::npos);
  CHECK(tapg_control_output_write((tmp + "/no/such/dir/x.json").c_str(), 3, u, &r, TAPG_OK) ==
        TAPG_EINVAL);
}

}  // namespace

int main(int argc, char** argv) {
  if (argc != 3) {
    std::fprintf(stderr, "usage: %s <instance dir> <scratch dir>\n", argv[0]);
    return 2;
  }
  Rng rng(1904);
  check_json_files(argv[1], argv[2]);
  check_validation(rng);
  check_planner(rng);
  check_solver(rng);
  check_server(rng);
  check_control_output(argv[2]);
  std::printf("host checks: %d, failed: %d\n", g_checks, g_failed);
  return g_failed == 0 ? 0 : 1;
}
