// Request server over one solver: a worker thread keeps the requests in
// flight (one per tree, admitted first come first served while their
// estimated device memory fits an HBM budget) iterating together as one
// forest, and lets requests join and leave between chunks of iterations
// (continuous batching).  A session's request is warm started when the
// session's previous request solved the same tree successfully and no other
// session's request has written that tree's dual since.
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdlib>
#include <deque>
#include <memory>
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
  // Warm starts: the tree each session last solved successfully, and the
  // session whose request last wrote each tree's dual (its slot holds one dual
  // per tree, so a session warm starts only from a dual it wrote itself).
  std::unordered_map<int, uint64_t> session_tree;
  std::unordered_map<uint64_t, int> dual_owner;
  long long next_ticket = 1;
  long long n_batches = 0, n_solved = 0;
  double busy_ms = 0.0;   // chunks of iterations
  double enter_ms = 0.0;  // forming forests (state in, data step, graph)
  double leave_ms = 0.0;  // state back to the trees' slots, results, forest freed
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

// Continuous batching: the trees in flight are iterated as one forest, one
// chunk of iterations at a time.  Between chunks, trees that stopped leave
// (their tickets complete) and pending requests that fit join; whenever the
// set changes, every running tree's exact iterate state (both dual buffers,
// control block, history) goes back to its own slot and the forest is re-formed
// from the new set, so a request's result does not depend on the mix.
// After a failure: free every cached forest of the solver (best effort).
void drop_forests(tapg_solver S) {
  std::vector<std::vector<uint64_t>> keys;
  for (const auto& kv : S->batches) keys.push_back(kv.first);
  for (const auto& k : keys) {
    try {
      dev_drop_batch(S, k);
    } catch (...) {
    }
  }
}

struct Active {
  tapg_server_s::Req req;
  LiveTree lt;
  size_t bytes = 0;
};

void add_ms(tapg_server_s* srv, double tapg_server_s::*field, Clock::time_point t0) {
  const double ms = std::chrono::duration<double, std::milli>(Clock::now() - t0).count();
  std::lock_guard<std::mutex> lk(srv->mu);
  srv->*field += ms;
}

void worker_loop(tapg_server_s* srv) {
  tapg_solver S = srv->S;
  std::vector<std::unique_ptr<Active>> active;
  bool in_forest = false;
  auto live_set = [&] {
    std::vector<LiveTree*> js;
    for (auto& a : active) js.push_back(&a->lt);
    return js;
  };
  // requests taken off the queue but not yet set up (see the admission below)
  std::vector<tapg_server_s::Req> admitted;
  size_t n_setup = 0;
  auto fail_all = [&](tapg_status code, const std::string& msg) {
    std::lock_guard<std::mutex> lk(srv->mu);
    for (auto& a : active) {
      complete(srv, a->req, code, nullptr, nullptr, msg);
      if (a->lt.t) srv->dual_owner.erase(a->lt.t->uid);
    }
    active.clear();
    for (size_t k = n_setup; k < admitted.size(); ++k)
      complete(srv, admitted[k], code, nullptr, nullptr, msg);
    admitted.clear();
    n_setup = 0;
    in_forest = false;
    srv->cv_done.notify_all();
  };
  auto finish = [&] {  // complete the trees that stopped and drop them
    std::lock_guard<std::mutex> lk(srv->mu);
    std::vector<std::unique_ptr<Active>> keep;
    for (auto& a : active) {
      if (!a->lt.finished) {
        keep.push_back(std::move(a));
        continue;
      }
      const tapg_status st = a->lt.own->numeric ? TAPG_ENUMERIC
                             : (!a->lt.res.converged && S->cfg.tol > 0) ? TAPG_ENOTCONV
                                                                        : TAPG_OK;
      std::vector<double> u0(S->net.nu, 0.0);
      try {
        dev_get_root_input(S, *a->lt.own, u0.data());
      } catch (...) {
      }
      complete(srv, a->req, st, u0.data(), &a->lt.res, "");
      // the tree's slot now holds this request's dual; a later request of the
      // session may start from it only if it is finite
      srv->dual_owner[a->lt.t->uid] = a->req.session;
      if (st == TAPG_OK || st == TAPG_ENOTCONV)
        srv->session_tree[a->req.session] = a->lt.t->uid;
      else
        srv->session_tree.erase(a->req.session);
      srv->n_solved++;
    }
    active.swap(keep);
    srv->cv_done.notify_all();
  };
  while (true) {
    admitted.clear();
    n_setup = 0;
    std::vector<int> warm;
    {
      std::unique_lock<std::mutex> lk(srv->mu);
      if (active.empty()) srv->cv_work.wait(lk, [&] { return srv->stop || !srv->pending.empty(); });
      if (srv->stop) break;
      size_t used = 0;
      std::set<uint64_t> trees_in;
      for (auto& a : active) {
        used += a->bytes;
        trees_in.insert(a->lt.t->uid);
      }
      for (auto it = srv->pending.begin();
           it != srv->pending.end() && (int)(active.size() + admitted.size()) < srv->max_batch;) {
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
        auto o = srv->dual_owner.find(t.uid);
        warm.push_back(s != srv->session_tree.end() && s->second == t.uid &&
                               o != srv->dual_owner.end() && o->second == it->session
                           ? 1
                           : 0);
        admitted.push_back(std::move(*it));
        it = srv->pending.erase(it);
      }
      srv->cv_done.notify_all();  // tickets completed with ENOMEM
    }
    try {
      if (!admitted.empty()) {
        if (in_forest) {  // running trees keep their state in their own slots
          std::vector<LiveTree*> js = live_set();
          const auto tl = Clock::now();
          dev_live_leave(S, js);
          add_ms(srv, &tapg_server_s::leave_ms, tl);
          in_forest = false;
          finish();
        }
        for (size_t k = 0; k < admitted.size(); ++k) {
          // into the active set first, so that a failure below completes it
          active.push_back(std::make_unique<Active>());
          Active* a = active.back().get();
          a->req = std::move(admitted[k]);
          n_setup = k + 1;
          a->lt.t = &a->req.tree->h;
          if (const char* f = std::getenv("TAPG_TEST_SERVER_SETUP_FAIL"))
            if (std::atoll(f) == a->req.ticket)
              throw Fail{TAPG_EDEVICE, "request setup failure injected for a test"};
          a->bytes = request_bytes(S, a->req.tree->h);
          a->lt.t = &a->req.tree->h;
          a->lt.own = &dev_slot(S, *a->lt.t);
          a->lt.p = a->req.p;
          a->lt.q = a->req.q;
          a->lt.gamma = solver_gamma(S, *a->lt.t, *a->lt.own);
          a->lt.warm = warm[k] != 0;
          dev_live_init(S, a->lt);
        }
        admitted.clear();
        n_setup = 0;
      }
      if (active.empty()) continue;
      if (!in_forest) {
        const auto te = Clock::now();
        dev_live_enter(S, live_set());
        add_ms(srv, &tapg_server_s::enter_ms, te);
        in_forest = true;
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->n_batches++;
      }
      const auto t0 = Clock::now();
      std::vector<LiveTree*> js = live_set();
      const bool stopped = dev_live_chunk(S, js);
      {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->busy_ms += std::chrono::duration<double, std::milli>(Clock::now() - t0).count();
      }
      if (stopped) {
        const auto tl = Clock::now();
        dev_live_leave(S, js);
        add_ms(srv, &tapg_server_s::leave_ms, tl);
        in_forest = false;
        finish();
      }
    } catch (const Fail& f) {
      fail_all(f.code, f.msg);
      drop_forests(S);
    } catch (const std::exception& e) {
      fail_all(TAPG_EDEVICE, e.what());
      drop_forests(S);
    }
  }
  // stopping: drop the forest, cancel what is left
  try {
    if (in_forest) dev_live_leave(S, live_set());
  } catch (...) {
  }
  std::lock_guard<std::mutex> lk(srv->mu);
  for (auto& a : active) complete(srv, a->req, TAPG_ESTATE, nullptr, nullptr, "server stopped");
  for (auto& r : srv->pending) complete(srv, r, TAPG_ESTATE, nullptr, nullptr, "server stopped");
  srv->pending.clear();
  srv->cv_done.notify_all();
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

tapg_status tapg_server_timing(tapg_server srv, double* enter_ms, double* chunk_ms,
                               double* leave_ms) {
  if (!srv) {
    set_error("srv is NULL");
    return TAPG_EINVAL;
  }
  std::lock_guard<std::mutex> lk(srv->mu);
  if (enter_ms) *enter_ms = srv->enter_ms;
  if (chunk_ms) *chunk_ms = srv->busy_ms;
  if (leave_ms) *leave_ms = srv->leave_ms;
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
