// Request server over one solver: a worker thread repeatedly takes the
// pending requests that fit an HBM budget (one request per tree, first come
// first served), solves them as one batch (a forest, one set of launches per
// iteration for all of them) and completes their tickets.  Requests that
// arrive while a batch runs join the next batch.  A session's request is warm
// started when the session's previous request solved the same tree.
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <set>
#include <thread>
#include <unordered_map>

#include "solver.h"

using Clock = std::chrono::steady_clock;

struct tapg_server_s {
  tapg_solver S = nullptr;
  size_t budget = 0;
  int max_batch = 64;
  std::thread worker;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  bool stop = false;
  struct Req {
    long long ticket;
    tapg_tree tree;
    std::vector<double> p, q;
    int session;
    Clock::time_point t_submit;
  };
  struct Done {
    tapg_status st;
    std::vector<double> u0;
    tapg_result res;
    double latency_ms;
    std::string msg;
  };
  std::deque<Req> pending;
  std::unordered_map<long long, Done> done;
  std::unordered_map<int, uint64_t> session_tree;  // tree last solved for each session
  long long next_ticket = 1;
  long long n_batches = 0, n_solved = 0;
  double busy_ms = 0.0;
};

namespace tapg {
namespace {

// Device bytes a request needs while its batch runs: its own slot and its
// share of the forest (iterates, data, tables, residual history), FP64 host
// data uploaded for both.  An estimate, used for admission only.
size_t request_bytes(const tapg_solver_s* S, const TreeHost& t) {
  const size_t e = S->fp32 ? 4 : 8;
  const size_t per_node = (size_t)(2 * S->LDY + 3 * S->LDX + 3 * S->LDU + 1) * e +
                          (size_t)(t.nd + 8) * 8 + 16;
  const size_t hist = (size_t)std::max(1, S->cfg.max_iter) * 8;
  const size_t power = (size_t)2 * S->LDY * e * t.K;
  return 2 * (per_node * t.K + hist) + power;
}

void complete(tapg_server_s* srv, tapg_server_s::Req& r, tapg_status st, const double* u0,
              const tapg_result* res, const std::string& msg) {
  tapg_server_s::Done d;
  d.st = st;
  if (u0) d.u0.assign(u0, u0 + srv->S->net.nu);
  d.res = res ? *res : tapg_result{};
  d.latency_ms = std::chrono::duration<double, std::milli>(Clock::now() - r.t_submit).count();
  d.msg = msg;
  srv->done[r.ticket] = std::move(d);
}

void worker_loop(tapg_server_s* srv) {
  tapg_solver S = srv->S;
  const int nu = S->net.nu;
  while (true) {
    std::vector<tapg_server_s::Req> batch;
    std::vector<int> warm;
    {
      std::unique_lock<std::mutex> lk(srv->mu);
      srv->cv_work.wait(lk, [&] { return srv->stop || !srv->pending.empty(); });
      if (srv->stop) {
        for (auto& r : srv->pending) complete(srv, r, TAPG_ESTATE, nullptr, nullptr, "server stopped");
        srv->pending.clear();
        srv->cv_done.notify_all();
        return;
      }
      size_t used = 0;
      std::set<uint64_t> trees_in;
      for (auto it = srv->pending.begin();
           it != srv->pending.end() && (int)batch.size() < srv->max_batch;) {
        const TreeHost& t = it->tree->h;
        const size_t b = request_bytes(S, t);
        if (b > srv->budget) {
          complete(srv, *it, TAPG_ENOMEM, nullptr, nullptr, "request exceeds the HBM budget");
          it = srv->pending.erase(it);
          continue;
        }
        if (trees_in.count(t.uid) || used + b > srv->budget) {
          ++it;
          continue;
        }
        used += b;
        trees_in.insert(t.uid);
        auto s = srv->session_tree.find(it->session);
        warm.push_back(s != srv->session_tree.end() && s->second == t.uid ? 1 : 0);
        batch.push_back(std::move(*it));
        it = srv->pending.erase(it);
      }
      srv->cv_done.notify_all();  // tickets completed with ENOMEM
      if (batch.empty()) continue;
    }
    // solve outside the lock
    const int n = (int)batch.size();
    std::vector<tapg_tree> trees(n);
    std::vector<const double*> ps(n), qs(n);
    std::vector<std::vector<double>> u0(n, std::vector<double>(nu, 0.0));
    std::vector<double*> u0p(n);
    std::vector<tapg_result> res(n);
    std::vector<tapg_status> st(n, TAPG_OK);
    std::vector<uint64_t> key(n);
    for (int k = 0; k < n; ++k) {
      trees[k] = batch[k].tree;
      ps[k] = batch[k].p.data();
      qs[k] = batch[k].q.data();
      u0p[k] = u0[k].data();
      key[k] = batch[k].tree->h.uid;
    }
    std::string err;
    tapg_status fail_code = TAPG_OK;
    const auto t0 = Clock::now();
    try {
      batch_core(S, n, trees.data(), ps.data(), qs.data(), warm.data(), u0p.data(), res.data(),
                 st.data());
    } catch (const Fail& f) {
      fail_code = f.code;
      err = f.msg;
    } catch (const std::exception& e) {
      fail_code = TAPG_EDEVICE;
      err = e.what();
    }
    try {
      dev_drop_batch(S, key);  // compositions rarely repeat: keep no forest around
    } catch (...) {
    }
    const double ms = std::chrono::duration<double, std::milli>(Clock::now() - t0).count();
    {
      std::lock_guard<std::mutex> lk(srv->mu);
      for (int k = 0; k < n; ++k) {
        if (fail_code != TAPG_OK) {
          complete(srv, batch[k], fail_code, nullptr, nullptr, err);
        } else {
          complete(srv, batch[k], st[k], u0[k].data(), &res[k], "");
          srv->session_tree[batch[k].session] = batch[k].tree->h.uid;
        }
      }
      srv->n_batches++;
      srv->n_solved += n;
      srv->busy_ms += ms;
    }
    srv->cv_done.notify_all();
  }
}

}  // namespace
}  // namespace tapg

using namespace tapg;

extern "C" {

tapg_status tapg_server_create(tapg_solver solver, size_t hbm_budget_bytes, int max_batch,
                               tapg_server* out) {
  if (!out) {
    set_error("out is NULL");
    return TAPG_EINVAL;
  }
  *out = nullptr;
  if (!solver) {
    set_error("solver is NULL");
    return TAPG_EINVAL;
  }
  if (solver->N == 0) {
    set_error("factor step not run");
    return TAPG_ESTATE;
  }
  if (solver->server_active) {
    set_error("the solver already has a server");
    return TAPG_ESTATE;
  }
  if (hbm_budget_bytes == 0 || max_batch < 1) {
    set_error("hbm_budget_bytes and max_batch must be positive");
    return TAPG_EINVAL;
  }
  try {
    auto srv = std::make_unique<tapg_server_s>();
    srv->S = solver;
    srv->budget = hbm_budget_bytes;
    srv->max_batch = max_batch;
    solver->server_active = true;
    tapg_server_s* p = srv.get();
    srv->worker = std::thread([p] { worker_loop(p); });
    *out = srv.release();
    clear_error();
    return TAPG_OK;
  } catch (const std::exception& e) {
    solver->server_active = false;
    set_error(std::string("server start failed: ") + e.what());
    return TAPG_EDEVICE;
  }
}

tapg_status tapg_server_submit(tapg_server srv, tapg_tree tree, const double* p, const double* q,
                               int session, long long* ticket) {
  if (!srv || !tree || !p || !q || !ticket) {
    set_error("NULL argument");
    return TAPG_EINVAL;
  }
  tapg_solver S = srv->S;
  if (tree->h.N != S->N || tree->h.nd != S->net.nd) {
    set_error("tree does not match the solver's horizon / network");
    return TAPG_EDIM;
  }
  for (int i = 0; i < S->net.nx; ++i)
    if (!std::isfinite(p[i])) {
      set_error("non-finite p");
      return TAPG_ENUMERIC;
    }
  for (int i = 0; i < S->net.nu; ++i)
    if (!std::isfinite(q[i])) {
      set_error("non-finite q");
      return TAPG_ENUMERIC;
    }
  tapg_server_s::Req r;
  r.tree = tree;
  r.p.assign(p, p + S->net.nx);
  r.q.assign(q, q + S->net.nu);
  r.session = session;
  r.t_submit = Clock::now();
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    if (srv->stop) {
      set_error("server stopped");
      return TAPG_ESTATE;
    }
    r.ticket = srv->next_ticket++;
    *ticket = r.ticket;
    srv->pending.push_back(std::move(r));
  }
  srv->cv_work.notify_one();
  clear_error();
  return TAPG_OK;
}

tapg_status tapg_server_poll(tapg_server srv, long long ticket, int wait_ms, double* u0_out,
                             tapg_result* res, double* latency_ms) {
  if (!srv) {
    set_error("srv is NULL");
    return TAPG_EINVAL;
  }
  std::unique_lock<std::mutex> lk(srv->mu);
  if (ticket < 1 || ticket >= srv->next_ticket) {
    set_error("unknown ticket");
    return TAPG_EINVAL;
  }
  auto ready = [&] { return srv->done.count(ticket) != 0; };
  if (!ready() && wait_ms != 0) {
    if (wait_ms < 0)
      srv->cv_done.wait(lk, ready);
    else
      srv->cv_done.wait_for(lk, std::chrono::milliseconds(wait_ms), ready);
  }
  auto it = srv->done.find(ticket);
  if (it == srv->done.end()) {
    // pending, or already collected
    bool queued = false;
    for (const auto& r : srv->pending) queued = queued || r.ticket == ticket;
    set_error(queued ? "pending" : "pending (in the running batch) or already collected");
    return TAPG_ESTATE;
  }
  tapg_server_s::Done d = std::move(it->second);
  srv->done.erase(it);
  lk.unlock();
  if (u0_out && !d.u0.empty()) std::copy(d.u0.begin(), d.u0.end(), u0_out);
  if (res) *res = d.res;
  if (latency_ms) *latency_ms = d.latency_ms;
  if (d.st != TAPG_OK) set_error(d.msg);
  else clear_error();
  return d.st;
}

tapg_status tapg_server_stats(tapg_server srv, long long* batches, long long* solved,
                              double* busy_ms, int* pending) {
  if (!srv) {
    set_error("srv is NULL");
    return TAPG_EINVAL;
  }
  std::lock_guard<std::mutex> lk(srv->mu);
  if (batches) *batches = srv->n_batches;
  if (solved) *solved = srv->n_solved;
  if (busy_ms) *busy_ms = srv->busy_ms;
  if (pending) *pending = (int)srv->pending.size();
  clear_error();
  return TAPG_OK;
}

void tapg_server_destroy(tapg_server srv) {
  if (!srv) return;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->stop = true;
  }
  srv->cv_work.notify_all();
  if (srv->worker.joinable()) srv->worker.join();
  srv->S->server_active = false;
  delete srv;
}

}  // extern "C"
