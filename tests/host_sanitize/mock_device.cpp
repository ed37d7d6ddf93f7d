// Host-only stand-ins for the library's device layer, linked only into the
// sanitizer driver of the CPU tests (never into libtapg).  They let the host
// code run under AddressSanitizer, UndefinedBehaviorSanitizer and
// ThreadSanitizer without a GPU: the HIP device query reports one gfx950
// device, buffers are not allocated, and the serving loop's trees "converge"
// after a number of chunks set by their request (q[0]), reporting q as the
// control action so the driver can check that every result reaches its own
// ticket.  No arithmetic of the method happens here.
#include <cstring>
#include <map>
#include <mutex>

#include "solver.h"

namespace tapg {
namespace {

struct MockLive {
  int chunks = 0, need = 1;
  std::vector<double> q;
};
std::mutex g_mu;
std::map<const Slot*, MockLive> g_live;

[[noreturn]] void no_device(const char* what) {
  throw Fail{TAPG_EDEVICE, std::string(what) + ": no device in the host sanitizer build"};
}

}  // namespace

void dev_init(tapg_solver_s*) {}
void dev_release(tapg_solver_s* S) {
  std::lock_guard<std::mutex> lk(g_mu);
  for (auto& kv : S->slots) g_live.erase(&kv.second);
  S->slots.clear();
  S->batches.clear();
}
void dev_upload_factors(tapg_solver_s*) {}

Slot& dev_slot(tapg_solver_s* S, const TreeHost& t) {
  Slot& sl = S->slots[t.uid];
  sl.tree_uid = t.uid;
  sl.K = t.K;
  sl.N = t.N;
  return sl;
}

void dev_live_init(tapg_solver_s*, LiveTree& j) {
  std::lock_guard<std::mutex> lk(g_mu);
  MockLive& m = g_live[j.own];
  m.chunks = 0;
  m.need = 1 + (j.q.empty() ? 0 : (int)j.q[0] % 5);
  m.q = j.q;
  j.finished = false;
  j.res = tapg_result{};
  j.it0 = 0;
}

void dev_live_enter(tapg_solver_s*, const std::vector<LiveTree*>& js) {
  // the real forest builder over the trees in flight, with its invariants
  std::vector<const TreeHost*> trees;
  int K = 0;
  for (const LiveTree* j : js) {
    trees.push_back(j->t);
    K += j->t->K;
  }
  std::vector<int> map, off;
  TreeHost f = build_forest(trees, map, off, true);
  refresh_forest_data(trees, map, off, f);
  if (f.K != K || f.ntrees != (int)js.size() || (int)map.size() != K)
    throw Fail{TAPG_EINVAL, "forest invariants violated"};
  for (int n = 0; n < K; ++n)
    if (map[n] < 0 || map[n] >= K) throw Fail{TAPG_EINVAL, "forest map out of range"};
}

bool dev_live_chunk(tapg_solver_s*, const std::vector<LiveTree*>& js) {
  std::lock_guard<std::mutex> lk(g_mu);
  bool any = false;
  for (LiveTree* j : js) {
    MockLive& m = g_live[j->own];
    if (++m.chunks >= m.need) any = true;
  }
  return any;
}

void dev_live_leave(tapg_solver_s* S, const std::vector<LiveTree*>& js) {
  std::lock_guard<std::mutex> lk(g_mu);
  for (LiveTree* j : js) {
    const MockLive& m = g_live[j->own];
    if (m.chunks < m.need) continue;
    j->finished = true;
    j->res.iters = m.chunks * S->cfg.check_every;
    j->res.converged = 1;
    j->res.gamma = j->gamma;
  }
}

void dev_get_root_input(tapg_solver_s*, Slot& sl, double* u0) {
  std::lock_guard<std::mutex> lk(g_mu);
  const MockLive& m = g_live[&sl];
  std::memcpy(u0, m.q.data(), m.q.size() * sizeof(double));
}

void dev_drop_batch(tapg_solver_s* S, const std::vector<uint64_t>& key) { S->batches.erase(key); }
void dev_drop_tree(tapg_solver_s* S, uint64_t uid) {
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = S->slots.find(uid);
  if (it != S->slots.end()) g_live.erase(&it->second);
  S->slots.erase(uid);
}

void dev_solve(tapg_solver_s*, const TreeHost&, Slot&, const double*, const double*, bool, double,
               tapg_result&) {
  no_device("solve");
}
void dev_batch_solve(tapg_solver_s*, const std::vector<const TreeHost*>&, const std::vector<Slot*>&,
                     const double* const*, const double* const*, const int*,
                     const std::vector<double>&, tapg_result*) {
  no_device("batch solve");
}
double dev_power(tapg_solver_s*, const TreeHost&, Slot&, int) { no_device("power iteration"); }
void dev_solve_noalloc(tapg_solver_s*, const TreeHost&, const double*, const double*, double,
                       tapg_result&, double*, double*, double*) {
  no_device("no-alloc solve");
}
size_t dev_noalloc_bytes(const tapg_solver_s*, const TreeHost&) { no_device("no-alloc bytes"); }
void dev_gap(tapg_solver_s*, const TreeHost&, Slot&, double*, double*) { no_device("gap"); }
void dev_get_primal(tapg_solver_s*, Slot&, double*, double*) { no_device("primal"); }
void dev_get_dual(tapg_solver_s*, Slot&, double*) { no_device("dual"); }
void dev_set_dual(tapg_solver_s*, Slot&, const double*) { no_device("set dual"); }
int dev_get_history(tapg_solver_s*, Slot&, double*, int) { no_device("history"); }
void dev_set_kernel_timing(tapg_solver_s*, bool) { no_device("kernel timing"); }
double dev_event_pair_us(tapg_solver_s*) { no_device("event pair"); }
double dev_autotune(tapg_solver_s*, const std::vector<const TreeHost*>&, int, int*) {
  no_device("autotune");
}

}  // namespace tapg

extern "C" hipError_t hipGetDeviceCount(int* n) {
  *n = 1;
  return hipSuccess;
}

extern "C" hipError_t hipGetDevicePropertiesR0600(hipDeviceProp_tR0600* p, int) {
  std::memset(p, 0, sizeof(*p));
  std::strcpy(p->gcnArchName, "gfx950");
  return hipSuccess;
}
