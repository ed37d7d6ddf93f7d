// Segment schedule of a tree (host): levels of consecutive stages, each
// split into workgroups that own groups of consecutive nodes of the level's
// first stage and all their descendants within the level.
#include <algorithm>
#include <string>

#include "solver.h"

namespace tapg {

// ---------------------------------------------------------------------------
// Segment schedule.  A level covers stages [s, e]; its workgroups own groups
// of g consecutive nodes of stage s and all their descendants down to e.
// The cut stages and group sizes minimise a simple per-iteration time model
// (per launch, per stage and per node-column costs; workgroups beyond the
// number that fit on the chip at once run in extra rounds) subject to every
// workgroup holding at most NBmax nodes of any stage.
// ---------------------------------------------------------------------------
int nb_template(int w) {
  int t = 1;
  while (t < w) t <<= 1;
  return t;
}

// Groups of g consecutive nodes of stage s, formed tree by tree, so that no
// group (hence no workgroup) holds nodes of two trees of a forest.
static void stage_groups(const TreeHost& t, int s, int g, std::vector<int>& lo,
                         std::vector<int>& hi) {
  lo.clear();
  hi.clear();
  for (int k = 0; k < t.ntrees; ++k) {
    const int a = t.seg_begin(s, k), b = t.seg_end(s, k);
    for (int x = a; x < b; x += g) {
      lo.push_back(x);
      hi.push_back(std::min(x + g, b));
    }
  }
}

// Widest stage-s segment of one tree.
static int widest_tree_stage(const TreeHost& t, int s) {
  int w = 0;
  for (int k = 0; k < t.ntrees; ++k) w = std::max(w, t.seg_end(s, k) - t.seg_begin(s, k));
  return w;
}

std::vector<LevelPlan> plan_levels(const TreeHost& t, int nbmax, double node_us,
                                   double c_launch, double c_stage) {
  const int N = t.N;
  const int conc = 512;  // workgroups resident at once (256 CUs x 2)
  std::vector<double> best(N + 1, 0.0);
  std::vector<LevelPlan> choice(N);
  std::vector<int> lo, hi;
  for (int s = N - 1; s >= 0; --s) {
    best[s] = 1e300;
    const int mu = widest_tree_stage(t, s);
    for (int g = 1; g <= std::max(1, mu); g *= 2) {
      // widths of every group, stage by stage, extended one stage at a time
      stage_groups(t, s, g, lo, hi);
      const int nwg = (int)lo.size();
      double stage_sum = 0.0;
      for (int e = s; e < N; ++e) {
        int wmax = 0;
        for (int w = 0; w < nwg; ++w) wmax = std::max(wmax, hi[w] - lo[w]);
        if (wmax > nbmax) break;
        const int rounds = (nwg + conc - 1) / conc;
        stage_sum += c_stage + node_us * nb_template(wmax);
        const double cost = 2.0 * (c_launch + rounds * stage_sum);
        if (cost + best[e + 1] < best[s]) {
          best[s] = cost + best[e + 1];
          choice[s] = LevelPlan{s, e, g, 0, nwg, cost};
        }
        if (e + 1 < N) {
          for (int w = 0; w < nwg; ++w) {
            const int nlo = t.cbeg[lo[w]], nhi = t.cend[hi[w] - 1];
            lo[w] = nlo;
            hi[w] = nhi;
          }
        }
      }
      if (g >= mu) break;
    }
  }
  std::vector<LevelPlan> out;
  for (int s = 0; s < N;) {
    out.push_back(choice[s]);
    s = choice[s].s_end + 1;
  }
  return out;
}

std::vector<std::vector<LevelPlan>> candidate_plans(const TreeHost& t, int nbmax, double node_us) {
  std::vector<std::vector<LevelPlan>> out;
  auto same = [](const std::vector<LevelPlan>& a, const std::vector<LevelPlan>& b) {
    if (a.size() != b.size()) return false;
    for (size_t i = 0; i < a.size(); ++i)
      if (a[i].s_begin != b[i].s_begin || a[i].s_end != b[i].s_end || a[i].group != b[i].group)
        return false;
    return true;
  };
  for (double cl : {3.0, 0.5, 1.5, 8.0, 20.0})
    for (double cs : {0.25, 0.08, 0.6, 1.5})
      for (double nf : {1.0, 0.4, 2.5}) {
        std::vector<LevelPlan> p = plan_levels(t, nbmax, node_us * nf, cl, cs);
        bool seen = false;
        for (const auto& q : out) seen = seen || same(p, q);
        if (!seen) out.push_back(std::move(p));
      }
  return out;  // the default plan (3.0, 0.25, 1.0) first
}

// Optional override: TAPG_LEVELS="s0:g0,s1:g1,..." (first stage and group size
// of every level, top first).
std::vector<LevelPlan> levels_from_env(const TreeHost& t, const char* spec) {
  std::vector<std::pair<int, int>> cuts;
  std::string str(spec);
  size_t p = 0;
  while (p < str.size()) {
    size_t q = str.find(',', p);
    if (q == std::string::npos) q = str.size();
    const std::string item = str.substr(p, q - p);
    const size_t c = item.find(':');
    cuts.emplace_back(std::stoi(item.substr(0, c)), c == std::string::npos ? 1 : std::stoi(item.substr(c + 1)));
    p = q + 1;
  }
  std::vector<LevelPlan> out;
  for (size_t i = 0; i < cuts.size(); ++i) {
    const int s = cuts[i].first, g = std::max(1, cuts[i].second);
    const int e = i + 1 < cuts.size() ? cuts[i + 1].first - 1 : t.N - 1;
    if (s < 0 || s > e || e >= t.N || (i == 0 && s != 0))
      throw Fail{TAPG_EINVAL, "TAPG_LEVELS does not describe the stages 0..N-1"};
    std::vector<int> lo, hi;
    stage_groups(t, s, g, lo, hi);
    out.push_back(LevelPlan{s, e, g, 0, (int)lo.size(), 0.0});
  }
  return out;
}

LevelPlan stage_plan(const TreeHost& t, int s, int g) {
  std::vector<int> lo, hi;
  stage_groups(t, s, std::max(1, g), lo, hi);
  return LevelPlan{s, t.N - 1, std::max(1, g), 0, (int)lo.size(), 0.0};
}

// Node ranges of every workgroup of a level, stage by stage.
std::vector<std::pair<int, int>> level_ranges(const TreeHost& t, const LevelPlan& L, int& wmax) {
  const int nst = L.s_end - L.s_begin + 1;
  std::vector<std::pair<int, int>> rg((size_t)L.n_wg * nst);
  wmax = 0;
  std::vector<int> glo, ghi;
  stage_groups(t, L.s_begin, L.group, glo, ghi);
  if ((int)glo.size() != L.n_wg) throw Fail{TAPG_EINVAL, "level plan does not match the tree"};
  for (int w = 0; w < L.n_wg; ++w) {
    int lo = glo[w], hi = ghi[w];
    for (int k = 0; k < nst; ++k) {
      rg[(size_t)w * nst + k] = {lo, hi};
      wmax = std::max(wmax, hi - lo);
      if (k + 1 < nst) {
        const int nlo = t.cbeg[lo], nhi = t.cend[hi - 1];
        lo = nlo;
        hi = nhi;
      }
    }
  }
  return rg;
}

}  // namespace tapg
