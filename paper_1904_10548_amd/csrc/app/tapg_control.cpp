// tapg_control: one control action from JSON files (Sec. 5.1: the controller
// is set up from the network, the controller configuration and the scenario
// tree; at run time it takes the plant state and the forecasts and writes the
// control action).  Uses only the C ABI of libtapg.
//
//   tapg_control --network network.json --config controllerconfig.json
//                --tree scenarioTree.json [--forecaster forecaster.json]
//                --state state.json --output controlOutput.json
//
// Exit status 0 when the solve reached its tolerance, 2 when it stopped at
// max_iter (the output is written in both cases, with its status), 1 on any
// error (message on stderr, no output written).
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "tapg.h"

namespace {

struct Handles {
  tapg_network net = nullptr;
  tapg_tree tree = nullptr;
  tapg_solver solver = nullptr;
  ~Handles() {
    if (solver) tapg_solver_destroy(solver);
    if (tree) tapg_tree_destroy(tree);
    if (net) tapg_network_destroy(net);
  }
};

int usage(const char* argv0) {
  std::fprintf(stderr,
               "usage: %s --network F --config F --tree F [--forecaster F] --state F "
               "--output F\n",
               argv0);
  return 1;
}

bool ok(tapg_status s, const char* what) {
  if (s == TAPG_OK) return true;
  std::fprintf(stderr, "tapg_control: %s failed (status %d): %s\n", what, (int)s,
               tapg_last_error());
  return false;
}

}  // namespace

int main(int argc, char** argv) {
  const char *network = nullptr, *config = nullptr, *tree = nullptr, *forecaster = nullptr,
             *state = nullptr, *output = nullptr;
  for (int i = 1; i < argc; ++i) {
    const char* a = argv[i];
    const char** slot = std::strcmp(a, "--network") == 0      ? &network
                        : std::strcmp(a, "--config") == 0     ? &config
                        : std::strcmp(a, "--tree") == 0       ? &tree
                        : std::strcmp(a, "--forecaster") == 0 ? &forecaster
                        : std::strcmp(a, "--state") == 0      ? &state
                        : std::strcmp(a, "--output") == 0     ? &output
                                                              : nullptr;
    if (!slot || i + 1 >= argc) return usage(argv[0]);
    *slot = argv[++i];
  }
  if (!network || !config || !tree || !state || !output) return usage(argv[0]);

  Handles h;
  int nx = 0, nu = 0, N = 0;
  if (!ok(tapg_network_from_json(network, &h.net), "network")) return 1;
  if (!ok(tapg_network_dims(h.net, &nx, &nu, nullptr, nullptr), "network sizes")) return 1;
  tapg_config cfg;
  std::vector<double> alpha0(nu), c_energy(nu), W_u((size_t)nu * nu);
  if (!ok(tapg_config_from_json(config, nu, &cfg, alpha0.data(), c_energy.data(), W_u.data()),
          "configuration"))
    return 1;
  if (!ok(tapg_tree_from_json(tree, forecaster, &h.tree), "scenario tree")) return 1;
  if (!ok(tapg_tree_dims(h.tree, &N, nullptr, nullptr), "tree sizes")) return 1;
  std::vector<double> x(nx), u_prev(nu), u0(nu);
  if (!ok(tapg_state_from_json(state, nx, nu, x.data(), u_prev.data()), "state")) return 1;
  if (!ok(tapg_solver_create(h.net, &cfg, &h.solver), "solver")) return 1;
  if (!ok(tapg_factor_step(h.solver, N), "factor step")) return 1;
  tapg_result res;
  const tapg_status st = tapg_solve(h.solver, h.tree, x.data(), u_prev.data(), 0, u0.data(), &res);
  if (st != TAPG_OK && st != TAPG_ENOTCONV) {
    ok(st, "solve");
    return 1;
  }
  if (!ok(tapg_control_output_write(output, nu, u0.data(), &res, st), "control output")) return 1;
  std::printf("tapg_control: %s after %d iterations, residual %.3e, cost %.10g, %.3f ms\n",
              st == TAPG_OK ? "converged" : "max_iter reached", res.iters, res.primal_res,
              res.cost, res.solve_ms);
  return st == TAPG_OK ? 0 : 2;
}
