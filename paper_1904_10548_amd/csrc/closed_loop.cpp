// Closed-loop receding-horizon simulation (Sec. 6.3, closed-loop simulations):
// at every sampling instant k the controller receives the forecast scenario
// tree (its root carries the demand and price observed at k), solves the
// stochastic MPC problem from the plant state, applies the root input to the
// plant, and the plant moves with the observed demand:
//   x_{k+1} = A x_k + B u_k + Gd d_k.
// The next solve starts from x_{k+1} and u_{k-1} = u_k, warm started from the
// previous dual (the tree keeps its shape; only its data change).  The
// performance indices of Sec. 6.3 are accumulated over the H_s steps:
//   KPI_E   = (1/H_s) sum_k (alpha0 + alpha_k)'u_k      (alpha_k = pi_k c_E)
//   KPI_S   = sum_k |max(xs - x_{k+1}, 0)|_1
//   KPI_tau = max_k tau_k                               (wall time of solve k)
#include <algorithm>
#include <chrono>
#include <cmath>
#include <string>
#include <vector>

#include "solver.h"

using namespace tapg;

namespace {

template <typename F>
tapg_status loop_guarded(F&& f) {
  try {
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
  }
}

}  // namespace

extern "C" {

tapg_status tapg_closed_loop(tapg_solver solver, tapg_tree tree, int H_s, const double* x0,
                             const double* u_prev, tapg_forecast_fn forecast, void* ctx,
                             int warm_start, double* x_traj, double* u_traj, double* tau_ms,
                             int* iters, tapg_loop_stats* stats) {
  return loop_guarded([&]() -> tapg_status {
    if (!solver || !tree || !x0 || !u_prev || !forecast)
      throw Fail{TAPG_EINVAL, "closed loop: NULL solver, tree, x0, u_prev or forecast"};
    if (H_s < 1) throw Fail{TAPG_EINVAL, "closed loop: H_s must be >= 1"};
    const NetworkHost& h = solver->net;
    const TreeHost& t = tree->h;
    if (t.nd != h.nd) throw Fail{TAPG_EDIM, "closed loop: tree nd does not match the network"};
    const int nx = h.nx, nu = h.nu, nd = h.nd, K = t.K;
    std::vector<double> demand((size_t)K * nd), price(K);
    std::vector<double> x(x0, x0 + nx), q(u_prev, u_prev + nu), u(nu), xn(nx);
    tapg_loop_stats st{};
    double tau_sum = 0.0;
    if (x_traj) std::copy(x.begin(), x.end(), x_traj);
    for (int k = 0; k < H_s; ++k) {
      if (forecast(ctx, k, demand.data(), price.data()) != 0)
        throw Fail{TAPG_EINVAL, "closed loop: the forecast callback failed at step " +
                                    std::to_string(k)};
      tapg_status s = tapg_tree_set_data(tree, demand.data(), price.data());
      if (s != TAPG_OK) throw Fail{s, std::string("closed loop: ") + tapg_last_error()};
      tapg_result r{};
      const auto t0 = std::chrono::steady_clock::now();
      s = tapg_solve(solver, tree, x.data(), q.data(), warm_start && k > 0, u.data(), &r);
      const double ms =
          std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
      if (s != TAPG_OK && s != TAPG_ENOTCONV)
        throw Fail{s, "closed loop: solve " + std::to_string(k) + ": " + tapg_last_error()};
      // plant step with the observed demand (the root's)
      const double* d = demand.data();
      double eq = 0.0, vb = 0.0, econ = 0.0, safe = 0.0;
      for (int i = 0; i < nx; ++i) {
        double v = 0.0;
        for (int j = 0; j < nx; ++j) v += h.A(i, j) * x[j];
        for (int j = 0; j < nu; ++j) v += h.B(i, j) * u[j];
        for (int j = 0; j < nd; ++j) v += h.Gd(i, j) * d[j];
        xn[i] = v;
        safe += std::max(h.xs[i] - v, 0.0);
      }
      for (int r2 = 0; r2 < h.ns; ++r2) {
        double v = 0.0;
        for (int j = 0; j < nu; ++j) v += h.E(r2, j) * u[j];
        for (int j = 0; j < nd; ++j) v += h.Ed(r2, j) * d[j];
        eq = std::max(eq, std::fabs(v));
      }
      for (int j = 0; j < nu; ++j) {
        econ += (solver->alpha0[j] + price[0] * solver->cE[j]) * u[j];
        vb = std::max(vb, std::max(h.umin[j] - u[j], u[j] - h.umax[j]));
      }
      st.kpi_E += econ / H_s;
      st.kpi_S += safe;
      st.kpi_tau_ms = std::max(st.kpi_tau_ms, ms);
      tau_sum += ms;
      st.max_viol_box = std::max(st.max_viol_box, vb);
      st.max_viol_eq = std::max(st.max_viol_eq, eq);
      st.iters += r.iters;
      st.steps_converged += r.converged ? 1 : 0;
      if (tau_ms) tau_ms[k] = ms;
      if (iters) iters[k] = r.iters;
      if (u_traj) std::copy(u.begin(), u.end(), u_traj + (size_t)k * nu);
      if (x_traj) std::copy(xn.begin(), xn.end(), x_traj + (size_t)(k + 1) * nx);
      x.swap(xn);
      q = u;
    }
    st.mean_tau_ms = tau_sum / H_s;
    if (stats) *stats = st;
    clear_error();
    return TAPG_OK;
  });
}

}  // extern "C"
