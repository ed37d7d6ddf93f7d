// A batch of trees as one forest (host).  Every tree keeps its breadth-first
// numbering inside the forest: the forest's stage-s nodes are tree 0's
// stage-s nodes, then tree 1's, ..., so children of consecutive nodes stay
// consecutive and one set of level launches sweeps all trees.  The root of
// tree k has ancestor -1 - k (its parent is that tree's (p, q)).
#include <algorithm>
#include <string>

#include "internal.h"

namespace tapg {

TreeHost build_forest(const std::vector<const TreeHost*>& trees, std::vector<int>& map,
                      std::vector<int>& map_off, bool host_data) {
  const int T = (int)trees.size();
  if (T < 1) throw Fail{TAPG_EINVAL, "empty batch"};
  const TreeHost& t0 = *trees[0];
  TreeHost f;
  f.uid = next_uid();
  f.version = 0;
  f.N = t0.N;
  f.nd = t0.nd;
  f.ntrees = T;
  const int N = f.N;
  for (const TreeHost* t : trees)
    if (t->N != N || t->nd != t0.nd)
      throw Fail{TAPG_EDIM, "the trees of a batch must share the horizon and nd"};
  f.mu.assign(N, 0);
  long long K = 0;
  for (const TreeHost* t : trees) {
    for (int s = 0; s < N; ++s) f.mu[s] += t->mu[s];
    K += t->K;
  }
  if (K > (1ll << 28)) throw Fail{TAPG_EDIM, "batch too large"};
  f.K = (int)K;
  f.offset.assign(N + 1, 0);
  for (int s = 0; s < N; ++s) f.offset[s + 1] = f.offset[s] + f.mu[s];
  f.tstart.assign((size_t)N * (T + 1), 0);
  for (int s = 0; s < N; ++s) {
    int pos = f.offset[s];
    for (int k = 0; k < T; ++k) {
      f.tstart[(size_t)s * (T + 1) + k] = pos;
      pos += trees[k]->mu[s];
    }
    f.tstart[(size_t)s * (T + 1) + T] = pos;
  }
  const int nd = f.nd;
  f.anc.assign(K, 0);
  f.cbeg.assign(K, 0);
  f.cend.assign(K, 0);
  f.stage.assign(K, 0);
  f.prob.assign(K, 0.0);
  f.device_data = !host_data;
  if (host_data) {
    f.price.assign(K, 0.0);
    f.demand.assign((size_t)K * nd, 0.0);
  }
  map.assign(K, 0);
  map_off.assign(T + 1, 0);
  for (int k = 0; k < T; ++k) map_off[k + 1] = map_off[k] + trees[k]->K;
  for (int k = 0; k < T; ++k) {
    const TreeHost& t = *trees[k];
    auto fidx = [&](int n) {
      const int s = t.stage[n];
      return f.tstart[(size_t)s * (T + 1) + k] + (n - t.offset[s]);
    };
    for (int n = 0; n < t.K; ++n) {
      const int fn = fidx(n);
      map[map_off[k] + n] = fn;
      f.anc[fn] = t.anc[n] < 0 ? -1 - k : fidx(t.anc[n]);
      if (t.cend[n] > t.cbeg[n]) {
        f.cbeg[fn] = fidx(t.cbeg[n]);
        f.cend[fn] = fidx(t.cend[n] - 1) + 1;
      }
      f.stage[fn] = t.stage[n];
      f.prob[fn] = t.prob[n];
      if (host_data) {
        f.price[fn] = t.price[n];
        std::copy_n(t.demand.begin() + (size_t)n * nd, nd, f.demand.begin() + (size_t)fn * nd);
      }
    }
  }
  return f;
}

void refresh_forest_data(const std::vector<const TreeHost*>& trees, const std::vector<int>& map,
                         const std::vector<int>& map_off, TreeHost& f) {
  const int nd = f.nd;
  for (size_t k = 0; k < trees.size(); ++k) {
    const TreeHost& t = *trees[k];
    for (int n = 0; n < t.K; ++n) {
      const int fn = map[map_off[k] + n];
      f.price[fn] = t.price[n];
      std::copy_n(t.demand.begin() + (size_t)n * nd, nd, f.demand.begin() + (size_t)fn * nd);
    }
  }
  f.version++;
}

}  // namespace tapg
