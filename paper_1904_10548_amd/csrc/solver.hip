// Device-side orchestration of the solver (host code): buffers, schedules,
// iteration graphs, the solve and power-iteration loops, transfers.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <random>
#include <unordered_map>
#include <vector>

#include "kernels.h"
#include "solver.h"

namespace tapg {

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
namespace {

// Optional progress line on stderr every TAPG_PROGRESS seconds of a long solve
// (iterations launched, trees still running).
struct ProgressLine {
  const char* what;
  double every = 0.0;
  std::chrono::steady_clock::time_point t0, last;
  explicit ProgressLine(const char* w) : what(w) {
    const char* e = std::getenv("TAPG_PROGRESS");
    every = e ? std::atof(e) : 0.0;
    t0 = last = std::chrono::steady_clock::now();
  }
  void tick(int iters, int running, int trees) {
    if (!(every > 0.0)) return;
    const auto now = std::chrono::steady_clock::now();
    if (std::chrono::duration<double>(now - last).count() < every) return;
    last = now;
    std::fprintf(stderr, "[tapg] %s: %d iterations, %d of %d trees running, %.1f s\n", what, iters,
                 running, trees, std::chrono::duration<double>(now - t0).count());
    std::fflush(stderr);
  }
};


// Device blocks freed by the solver are kept for reuse, by device and size,
// instead of going back to the driver: hipFree synchronises the device, and
// the server forms and frees a forest every few chunks.  Every path that frees
// a slot has synchronised the solver's stream first, so a reused block is idle.
// The cache is released into the driver when an allocation fails.
class BlockCache {
 public:
  void* get(size_t bytes) {
    int dev = 0;
    (void)hipGetDevice(&dev);
    {
      std::lock_guard<std::mutex> lk(mu_);
      auto& fl = free_[{dev, bytes}];
      if (!fl.empty()) {
        void* p = fl.back();
        fl.pop_back();
        live_[p] = {dev, bytes};
        return p;
      }
    }
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      trim();
      e = hipMalloc(&p, bytes);
    }
    if (e != hipSuccess) throw Fail{TAPG_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e)};
    std::lock_guard<std::mutex> lk(mu_);
    live_[p] = {dev, bytes};
    return p;
  }
  void put(void* p) {
    std::lock_guard<std::mutex> lk(mu_);
    auto it = live_.find(p);
    if (it == live_.end()) {  // not ours
      (void)hipFree(p);
      return;
    }
    free_[it->second].push_back(p);
    live_.erase(it);
  }
  void trim() {  // every cached block back to the driver
    std::lock_guard<std::mutex> lk(mu_);
    int cur = 0;
    (void)hipGetDevice(&cur);
    for (auto& kv : free_) {
      if (kv.second.empty()) continue;
      (void)hipSetDevice(kv.first.first);
      for (void* p : kv.second) (void)hipFree(p);
      kv.second.clear();
    }
    (void)hipSetDevice(cur);
  }

 private:
  std::mutex mu_;
  std::map<std::pair<int, size_t>, std::vector<void*>> free_;
  std::unordered_map<void*, std::pair<int, size_t>> live_;
};

BlockCache& block_cache() {
  static BlockCache* c = new BlockCache();  // lives until the process ends
  return *c;
}

// Device allocations are rounded up to 256 bytes (the cache's size classes).
void* dev_alloc(size_t bytes) {
  return block_cache().get((std::max<size_t>(bytes, 1) + 255) & ~(size_t)255);
}

template <typename T>
T* dmalloc(size_t n) {
  return static_cast<T*>(dev_alloc(std::max<size_t>(n, 1) * sizeof(T)));
}

template <typename T>
void dfree(T*& p) {
  if (p) block_cache().put(p);
  p = nullptr;
}

// Column-major padded copy of a row-major rows x cols matrix, optionally transposed.
template <typename T>
std::vector<T> colmajor(const Mat& M, int ld, bool transpose_first) {
  const int R = transpose_first ? M.c : M.r;
  const int C = transpose_first ? M.r : M.c;
  std::vector<T> out((size_t)ld * C, T(0));
  for (int r = 0; r < R; ++r)
    for (int k = 0; k < C; ++k)
      out[(size_t)k * ld + r] = (T)(transpose_first ? M(k, r) : M(r, k));
  return out;
}

// Set-up copies (tables, structure) go through one pinned staging buffer of
// the process (allocated once, kept to the process's end): the host vector,
// often a temporary, is copied there, the device copy is queued on the
// stream with no wait, and an event recorded behind it.  A staged region is
// written again only after the events of every copy out of the buffer have
// completed (an event stays valid after its stream is gone).  Larger copies
// wait for the stream and copy at once.
struct UploadStage {
  static constexpr size_t kCap = 8u << 20;
  std::mutex mu;
  unsigned char* base = nullptr;
  size_t off = 0;
  std::vector<std::pair<int, hipEvent_t>> pending;  // (device, event) since the last reuse
  std::map<int, std::vector<hipEvent_t>> idle;      // per device (events belong to one)
};

UploadStage& upload_stage() {
  static UploadStage* u = new UploadStage;  // never destroyed: outlives every solver
  return *u;
}

template <typename T>
T* upload(const std::vector<T>& v, hipStream_t st) {
  T* d = dmalloc<T>(v.size());
  const size_t n = v.size() * sizeof(T);
  if (n == 0) return d;
  if (n > UploadStage::kCap / 4) {
    TAPG_HIP(hipStreamSynchronize(st));
    TAPG_HIP(hipMemcpy(d, v.data(), n, hipMemcpyHostToDevice));
    return d;
  }
  UploadStage& u = upload_stage();
  std::lock_guard<std::mutex> lk(u.mu);
  if (u.base == nullptr)
    TAPG_HIP(hipHostMalloc(reinterpret_cast<void**>(&u.base), UploadStage::kCap,
                           hipHostMallocPortable));
  size_t at = (u.off + 255) & ~(size_t)255;
  if (at + n > UploadStage::kCap) {  // reuse: every copy out of the buffer has completed
    for (auto& pe : u.pending) {
      TAPG_HIP(hipEventSynchronize(pe.second));
      u.idle[pe.first].push_back(pe.second);
    }
    u.pending.clear();
    at = 0;
  }
  int dev = 0;
  TAPG_HIP(hipGetDevice(&dev));
  hipEvent_t ev = nullptr;
  auto& pool = u.idle[dev];
  if (pool.empty()) {
    TAPG_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
  } else {
    ev = pool.back();
    pool.pop_back();
  }
  std::memcpy(u.base + at, v.data(), n);
  hipError_t e = hipMemcpyAsync(d, u.base + at, n, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipEventRecord(ev, st);
  if (e != hipSuccess) {  // nothing queued from this region that the event does not cover
    (void)hipStreamSynchronize(st);
    pool.push_back(ev);
    dfree(d);
    throw Fail{TAPG_EDEVICE, std::string("upload: ") + hipGetErrorString(e)};
  }
  u.pending.emplace_back(dev, ev);
  u.off = at + n;
  return d;
}

template <typename T>
std::vector<T> padvec(const std::vector<double>& v, int ld) {
  std::vector<T> o(ld, T(0));
  for (size_t i = 0; i < v.size(); ++i) o[i] = (T)v[i];
  return o;
}

template <typename T>
void init_net(tapg_solver_s* S, NetDev<T>& d) {
  const NetworkHost& h = S->net;
  hipStream_t st = S->stream;
  d.At = upload(colmajor<T>(h.A, S->LDX, true), st);
  d.Bt = upload(colmajor<T>(h.B, S->LDU, true), st);
  d.A = upload(colmajor<T>(h.A, S->LDX, false), st);
  d.B = upload(colmajor<T>(h.B, S->LDX, false), st);
  d.xmin = upload(padvec<T>(h.xmin, S->LDX), st);
  d.xmax = upload(padvec<T>(h.xmax, S->LDX), st);
  d.xs = upload(padvec<T>(h.xs, S->LDX), st);
  d.umin = upload(padvec<T>(h.umin, S->LDU), st);
  d.umax = upload(padvec<T>(h.umax, S->LDU), st);
  // CSR of B (rows = states) and of B' (rows = inputs)
  std::vector<int> row, col;
  std::vector<T> val;
  auto csr = [&](const Mat& M) {
    row.assign(1, 0);
    col.clear();
    val.clear();
    for (int i = 0; i < M.r; ++i) {
      for (int k = 0; k < M.c; ++k)
        if (M(i, k) != 0.0) {
          col.push_back(k);
          val.push_back((T)M(i, k));
        }
      row.push_back((int)col.size());
    }
    if (col.empty()) {
      col.push_back(0);
      val.push_back(T(0));
    }
  };
  csr(h.B);
  d.Brow = upload(row, st);
  d.Bcol = upload(col, st);
  d.Bval = upload(val, st);
  csr(transpose(h.B));
  d.Btrow = upload(row, st);
  d.Btcol = upload(col, st);
  d.Btval = upload(val, st);
  d.Wu = upload(colmajor<T>(Mat::from(S->Wu.data(), h.nu, h.nu), S->LDU, false), st);
  if (S->proj) {
    csr(S->G);
    if (S->G.r == 0) row.assign(1, 0);
    d.Grow = upload(row, st);
    d.Gcol = upload(col, st);
    d.Gval = upload(val, st);
    csr(transpose(h.E));
    d.Etrow = upload(row, st);
    d.Etcol = upload(col, st);
    d.Etval = upload(val, st);
  }
}

template <typename T>
void free_net(NetDev<T>& d) {
  dfree(d.At); dfree(d.Bt); dfree(d.A); dfree(d.B);
  dfree(d.xmin); dfree(d.xmax); dfree(d.xs); dfree(d.umin); dfree(d.umax);
  dfree(d.F); dfree(d.Kb);
  dfree(d.Brow); dfree(d.Bcol); dfree(d.Bval); dfree(d.Btrow); dfree(d.Btcol); dfree(d.Btval);
  dfree(d.Wu);
  dfree(d.Grow); dfree(d.Gcol); dfree(d.Gval); dfree(d.Etrow); dfree(d.Etcol); dfree(d.Etval);
}

// Nodes per tile: the largest NB in {8, 4, 2, 1} that keeps at least 256
// tiles in the stage and fits the forward kernel's LDS in 64 KiB.
int pick_nb(int width, size_t elem, int LDX, int LDU, int LDY) {
  for (int nb : {8, 4, 2}) {  // the forward kernel's LDS (its prox tiles are FP64)
    const size_t lds = (size_t)(2 * LDX + 2 * LDU + kThreads) * nb * elem +
                       (size_t)2 * LDY * nb * sizeof(double);
    if ((width + nb - 1) / nb >= 256 && lds <= 60 * 1024) return nb;
  }
  return 1;
}

template <typename T>
SweepArgs<T> make_args(tapg_solver_s* S, Slot& sl, const NetDev<T>& d, int mode) {
  SweepArgs<T> a{};
  a.nx = S->net.nx;
  a.nu = S->net.nu;
  a.LDX = S->LDX;
  a.LDU = S->LDU;
  a.LDY = S->LDY;
  a.mode = mode;
  a.anc = sl.d_anc;
  a.cbeg = sl.d_cbeg;
  a.cend = sl.d_cend;
  a.invp = static_cast<const T*>(sl.d_invp);
  a.At = d.At;
  a.Bt = d.Bt;
  a.A = d.A;
  a.B = d.B;
  a.xmin = d.xmin;
  a.xmax = d.xmax;
  a.xs = d.xs;
  a.umin = d.umin;
  a.umax = d.umax;
  a.Wx = (T)S->cfg.W_x;
  a.Ws = (T)S->cfg.W_s;
  a.kappa = static_cast<const T*>(sl.d_kappa);
  a.g = static_cast<const T*>(sl.d_g);
  a.pq = static_cast<const T*>(sl.d_pq);
  a.Y0 = static_cast<T*>(sl.d_Y0);
  a.Y1 = static_cast<T*>(sl.d_Y1);
  a.lam = static_cast<T*>(sl.d_lam);
  a.jv = static_cast<T*>(sl.d_j);
  a.u = static_cast<T*>(sl.d_u);
  a.x = static_cast<T*>(sl.d_x);
  a.ctl = sl.d_ctl;
  a.part = sl.d_part;
  return a;
}

// One APG iteration (mode 0) or one power-iteration step (mode 1) on the
// solver's stream: backward stages, forward stages, end-of-step kernel.
template <typename T>
size_t seg_lds_probe(tapg_solver_s* S, int nbm, int nst, int nch, bool scan) {
  SegArgs<T> probe{};
  probe.nch = nch;
  probe.nx = S->net.nx;
  probe.nu = S->net.nu;
  probe.LDX = S->LDX;
  probe.LDU = S->LDU;
  probe.nst = nst;
  probe.nnzB = S->nnzB;
  probe.proj = S->proj ? 1 : 0;
  probe.ns = S->net.ns;
  probe.nnzG = S->nnzG;
  probe.nnzE = S->nnzE;
  probe.scan = scan ? 1 : 0;
  return seg_lds<T>(nbm, probe);
}

template <typename T>
SegArgs<T> make_seg_args(tapg_solver_s* S, Slot& sl, const NetDev<T>& d, int mode) {
  SegArgs<T> a{};
  a.nx = S->net.nx;
  a.nu = S->net.nu;
  a.LDX = S->LDX;
  a.LDU = S->LDU;
  a.LDY = S->LDY;
  int lr = 1;
  while (lr < S->LDX) lr <<= 1;
  a.LDXR = lr;
  a.N = sl.N;
  a.mode = mode;
  a.a_ident = S->a_ident ? 1 : 0;
  a.wu_scalar = S->wu_scalar ? 1 : 0;
  a.wu = (T)S->wu;
  a.part_total = sl.part_total;
  a.nnzB = S->nnzB;
  a.anc = sl.d_anc;
  a.cbeg = sl.d_cbeg;
  a.cend = sl.d_cend;
  a.invp = static_cast<const T*>(sl.d_invp);
  a.F = d.F;
  a.fid = S->d_fid;
  a.proj = S->proj ? 1 : 0;
  a.ns = S->net.ns;
  a.nnzG = S->nnzG;
  a.nnzE = S->nnzE;
  a.Grow = d.Grow;
  a.Gcol = d.Gcol;
  a.Gval = d.Gval;
  a.Etrow = d.Etrow;
  a.Etcol = d.Etcol;
  a.Etval = d.Etval;
  a.winv = (T)(1.0 / S->wu);
  a.scan = sl.scan ? 1 : 0;
  a.kperp = static_cast<const T*>(sl.d_kperp);
  a.zb = static_cast<T*>(sl.d_zb);
  a.zr = static_cast<const T*>(sl.d_zr);
  a.Wu = d.Wu;
  a.A = d.A;
  a.At = d.At;
  a.Brow = d.Brow;
  a.Bcol = d.Bcol;
  a.Bval = d.Bval;
  a.Btrow = d.Btrow;
  a.Btcol = d.Btcol;
  a.Btval = d.Btval;
  a.xmin = d.xmin;
  a.xmax = d.xmax;
  a.xs = d.xs;
  a.umin = d.umin;
  a.umax = d.umax;
  a.Wx = (T)S->cfg.W_x;
  a.Ws = (T)S->cfg.W_s;
  a.kappa = static_cast<const T*>(sl.d_kappa);
  a.g = static_cast<const T*>(sl.d_g);
  a.pq = static_cast<const T*>(sl.d_pq);
  a.Y0 = static_cast<T*>(mode == 1 ? sl.d_P0 : sl.d_Y0);
  a.Y1 = static_cast<T*>(mode == 1 ? sl.d_P1 : sl.d_Y1);
  a.lam = static_cast<T*>(sl.d_lam);
  a.jv = static_cast<T*>(sl.d_j);
  a.u = static_cast<T*>(sl.d_u);
  a.x = static_cast<T*>(sl.d_x);
  a.ctl = sl.d_ctl;
  a.part = sl.d_part;
  a.hist = sl.d_hist;
  a.ntrees = sl.ntrees;
  a.hist_stride = sl.hist_cap;
  a.pq_stride = S->LDX + S->LDU;
  a.wgtree = nullptr;
  return a;
}

// Event pair index for the timed path (-1: untimed).
struct TimedCursor {
  int next = 0;
  std::vector<int> kind;  // kind of each recorded pair
  std::vector<int> it;    // iteration of each pair within the chunk (-1: chunk end)
  int iter = 0;           // iteration being enqueued
};

// One iteration.  Level launches: the control state is read from block blk of
// the slot's two control blocks (block b of tree k at d_ctl[b * ntrees + k]);
// with `close`, the first backward launch first ends the previous iteration,
// advancing the state from the other block into block blk.  The iteration
// itself is not ended here (enqueue_iterations ends a run of them).  Power
// iteration and per-stage kernels: block 0 only, each iteration ended by a
// launch of its own.
template <typename T>
void enqueue_iteration(tapg_solver_s* S, Slot& sl, const NetDev<T>& d, int mode,
                       TimedCursor* tc = nullptr, int blk = 0, bool close = false) {
  hipStream_t st = S->stream;
  if (sl.segmented) {
    SegArgs<T> a = make_seg_args<T>(S, sl, d, mode);
    a.ctl = sl.d_ctl + (size_t)blk * sl.ntrees;
    a.ctl_prev = sl.d_ctl + (size_t)(1 - blk) * sl.ntrees;
    const int nl = (int)sl.levels.size();
    for (int pass = 0; pass < 2; ++pass) {
      int base = 0;
      std::vector<int> bases(nl);
      for (int l = 0; l < nl; ++l) {
        bases[l] = base;
        base += sl.levels[l].n_wg;
      }
      const bool full = pass == 1 && sl.fwd_full.n_wg > 0;
      for (int q = 0; q < (full ? 1 : nl); ++q) {
        const int l = pass == 0 ? nl - 1 - q : q;
        const Slot::Level& L = full ? sl.fwd_full : sl.levels[l];
        a.s_begin = L.s_begin;
        a.s_end = L.s_end;
        a.nst = L.s_end - L.s_begin + 1;
        a.ranges = L.d_ranges;
        a.wgx = L.d_wgx;
        a.wgtree = L.d_wgtree;
        a.part_base = bases[l];
        a.nch = L.nch;
        a.own = full ? sl.d_own : nullptr;
        if (full) {
          a.part_base = 0;
          a.part_total = L.n_wg;
        }
        a.close = (close && mode == 0 && pass == 0 && q == 0) ? 1 : 0;
        const bool light = sl.top_light && sl.n_up > 0 && pass == 0;
        if (light && l != nl - 1) continue;  // the upper levels run in the bottom launch
        a.n_main = a.n_up = 0;
        if (tc) (void)hipEventRecord(S->tev[2 * tc->next], st);
        if (light) {  // bottom level, the upper nodes' local parts and the upper levels
          a.n_main = L.n_wg;
          a.n_up = sl.n_up;
          a.up_plan = sl.d_up_plan;
          a.up_plan_stride = sl.up_plan_stride;
          a.up_nw = sl.up_nw;
          a.up_nch = sl.up_nch;
          a.up_par = sl.d_up_par;
          a.up_need = sl.d_up_need;
          a.up_cnt = sl.d_up_cnt;
          launch_seg<T>(false, L.nbm, a, L.n_wg + sl.n_up, st);
        } else {
          launch_seg<T>(pass == 1, L.nbm, a, L.n_wg, st);
        }
        if (tc) {
          (void)hipEventRecord(S->tev[2 * tc->next + 1], st);
          tc->kind.push_back(pass);
          tc->it.push_back(tc->iter);
          tc->next++;
        }
      }
    }
    if (mode == 0 && sl.d_ua)
      launch_avg<T>(a.ctl, static_cast<const T*>(sl.d_u), static_cast<const T*>(sl.d_x),
                    static_cast<T*>(sl.d_ua), static_cast<T*>(sl.d_xa), (size_t)sl.K * S->LDU,
                    (size_t)sl.K * S->LDX, st);
    // the power iteration's step ends in a launch of its own (the forward
    // workgroups left their partial sums in device memory)
    if (mode == 1)
      launch_power_end(sl.d_ctl, (const double*)sl.d_part,
                       sl.fwd_full.n_wg > 0 ? sl.fwd_full.n_wg : sl.part_total, st);
    return;
  }
  SweepArgs<T> a = make_args<T>(S, sl, d, mode);
  if (mode == 1) {
    a.Y0 = static_cast<T*>(sl.d_P0);
    a.Y1 = static_cast<T*>(sl.d_P1);
  }
  const size_t fstride = (size_t)S->LDU * S->LDU;
  for (int pass = 0; pass < 2; ++pass) {
    for (int q = 0; q < sl.N; ++q) {
      const int s = pass == 0 ? sl.N - 1 - q : q;
      a.s = s;
      a.node0 = sl.node_offset[s];
      a.count = sl.node_offset[s + 1] - sl.node_offset[s];
      a.tile_base = sl.tile_offset[s];
      a.F = d.F + s * fstride;
      a.Kb = d.Kb + s * fstride;
      if (tc) (void)hipEventRecord(S->tev[2 * tc->next], st);
      if (pass == 0)
        launch_bwd_stage<T>(sl.nb_of_stage[s], a, sl.tiles_of_stage[s], st);
      else
        launch_fwd_stage<T>(sl.nb_of_stage[s], a, sl.tiles_of_stage[s], st);
      if (tc) {
        (void)hipEventRecord(S->tev[2 * tc->next + 1], st);
        tc->kind.push_back(pass);
        tc->it.push_back(tc->iter);
        tc->next++;
      }
    }
  }
  if (mode == 0) {
    if (sl.d_ua)
      launch_avg<T>(sl.d_ctl, static_cast<const T*>(sl.d_u), static_cast<const T*>(sl.d_x),
                    static_cast<T*>(sl.d_ua), static_cast<T*>(sl.d_xa), (size_t)sl.K * S->LDU,
                    (size_t)sl.K * S->LDX, st);
    if (tc) (void)hipEventRecord(S->tev[2 * tc->next], st);
    launch_iter_end(sl.d_ctl, sl.d_hist, 1, 0, st);
    if (tc) {
      (void)hipEventRecord(S->tev[2 * tc->next + 1], st);
      tc->kind.push_back(2);
      tc->it.push_back(tc->iter);
      tc->next++;
    }
  } else
    launch_power_end(sl.d_ctl, (const double*)sl.d_part, sl.total_tiles, st);
}

static int launches_per_iter(const Slot& sl) {
  if (sl.segmented)  // backward levels, forward launches (the end is fused or per run)
    return (int)sl.levels.size() + (sl.fwd_full.n_wg > 0 ? 1 : (int)sl.levels.size());
  return 2 * sl.N + 1;
}

// n APG iterations from the state in control block 0 back to block 0.  Level
// launches: iteration i > 0 ends iteration i - 1 in its first backward launch
// (states alternate between the two blocks), and one small launch ends the
// last into block 0; this is what a chunk's graph holds.  Per-stage kernels:
// every iteration ends in a launch of its own.
template <typename T>
void enqueue_iterations(tapg_solver_s* S, Slot& sl, const NetDev<T>& d, int n,
                        TimedCursor* tc = nullptr) {
  for (int i = 0; i < n; ++i) {
    if (tc) tc->iter = i;
    if (sl.segmented)
      enqueue_iteration<T>(S, sl, d, 0, tc, i & 1, i > 0);
    else
      enqueue_iteration<T>(S, sl, d, 0, tc);
  }
  if (!sl.segmented || n < 1) return;
  hipStream_t st = S->stream;
  if (tc) {
    tc->iter = -1;
    (void)hipEventRecord(S->tev[2 * tc->next], st);
  }
  launch_iter_end_from(sl.d_ctl + (size_t)((n - 1) & 1) * sl.ntrees, sl.d_ctl, sl.d_hist,
                       sl.ntrees, sl.hist_cap, st);
  if (tc) {
    (void)hipEventRecord(S->tev[2 * tc->next + 1], st);
    tc->kind.push_back(2);
    tc->it.push_back(-1);
    tc->next++;
  }
}

template <typename T>
const NetDev<T>& net_of(tapg_solver_s* S);
template <>
const NetDev<double>& net_of<double>(tapg_solver_s* S) { return S->d64; }
template <>
const NetDev<float>& net_of<float>(tapg_solver_s* S) { return S->d32; }

template <typename T>
std::vector<T> pad_rows(const double* src, int rows, int cols, int ld) {
  std::vector<T> out((size_t)rows * ld, T(0));
  for (int i = 0; i < rows; ++i)
    for (int j = 0; j < cols; ++j) out[(size_t)i * ld + j] = (T)src[(size_t)i * cols + j];
  return out;
}

// Whether the persistent iteration runs this slot, setting it up the first
// time: asked for with TAPG_CHAIN=1 (it measured slower than the level
// launches on the Barcelona-sized tree: every hand-over is a device-scope
// release / acquire), one tree, the segment schedule with the projector form,
// at most kChainMaxLevels levels, every workgroup resident at once.
template <typename T>
bool chain_usable(tapg_solver_s* S, const TreeHost& t, Slot& sl) {
  if (sl.chain_state) return sl.chain_state > 0;
  sl.chain_state = -1;
  const char* env = std::getenv("TAPG_CHAIN");
  if (!(env && env[0] == '1')) return false;
  const int nl = (int)sl.levels.size();
  if (t.ntrees != 1 || !sl.segmented || !S->proj || sl.scan || nl < 1 || nl > kChainMaxLevels ||
      sl.d_ua)
    return false;
  int total = 0, nbm = 1;
  for (const Slot::Level& L : sl.levels) {
    total += L.n_wg;
    nbm = std::max(nbm, L.nbm);
  }
  size_t lds = 0;
  for (const Slot::Level& L : sl.levels)
    lds = std::max(lds, seg_lds_probe<T>(S, nbm, L.s_end - L.s_begin + 1, L.nch, false));
  if (lds + kSegStaticLds > S->lds_limit) return false;
  int cus = 0;
  TAPG_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, S->device));
  const int bpc = chain_blocks_per_cu<T>(nbm, true, lds);
  if (bpc < 1 || (long long)bpc * cus < total) return false;
  // per-level arguments, and the workgroups that hand over to each other
  hipStream_t st = S->stream;
  const NetDev<T>& d = net_of<T>(S);
  std::vector<SegArgs<T>> lev(nl);
  std::vector<int> base(nl + 1, 0);
  std::vector<std::vector<std::pair<int, int>>> rng(nl);
  for (int l = 0; l < nl; ++l) {
    const Slot::Level& L = sl.levels[l];
    SegArgs<T> a = make_seg_args<T>(S, sl, d, 0);
    a.s_begin = L.s_begin;
    a.s_end = L.s_end;
    a.nst = L.s_end - L.s_begin + 1;
    a.ranges = L.d_ranges;
    a.wgx = L.d_wgx;
    a.wgtree = nullptr;
    a.part_base = base[l];
    a.nch = L.nch;
    lev[l] = a;
    base[l + 1] = base[l] + L.n_wg;
    int wmax = 0;
    rng[l] = level_ranges(t, sl.plans[l], wmax);
  }
  std::vector<int2> par(total, make_int2(-1, -1));
  std::vector<int> nchild(total, 0);
  for (int l = 1; l < nl; ++l) {
    const int nst_p = sl.levels[l - 1].s_end - sl.levels[l - 1].s_begin + 1;
    const int nst = sl.levels[l].s_end - sl.levels[l].s_begin + 1;
    auto owner = [&](int node) {  // workgroup of level l-1 holding `node` at its last stage
      for (int w = 0; w < sl.levels[l - 1].n_wg; ++w) {
        const auto& r = rng[l - 1][(size_t)w * nst_p + nst_p - 1];
        if (node >= r.first && node < r.second) return w;
      }
      throw Fail{TAPG_EINVAL, "persistent iteration: parent workgroup not found"};
    };
    for (int w = 0; w < sl.levels[l].n_wg; ++w) {
      const auto& r = rng[l][(size_t)w * nst];
      const int p0 = owner(t.anc[r.first]), p1 = owner(t.anc[r.second - 1]);
      par[base[l] + w] = make_int2(base[l - 1] + p0, base[l - 1] + p1);
      for (int p = p0; p <= p1; ++p) nchild[base[l - 1] + p]++;
    }
  }
  void* dlev = nullptr;
  TAPG_HIP(hipMalloc(&dlev, sizeof(SegArgs<T>) * nl));
  sl.d_chain_lev = dlev;
  TAPG_HIP(hipMemcpy(dlev, lev.data(), sizeof(SegArgs<T>) * nl, hipMemcpyHostToDevice));
  sl.d_chain_par = upload(par, st);
  sl.d_chain_nchild = upload(nchild, st);
  sl.d_chain_cnt = dmalloc<unsigned>((size_t)2 * total);
  void* dsync = nullptr;
  TAPG_HIP(hipMalloc(&dsync, sizeof(ChainSync)));
  sl.d_chain_sync = dsync;
  sl.chain_total = total;
  sl.chain_nbm = nbm;
  sl.chain_lds = lds;
  sl.chain_state = 1;
  sl.chain_base.assign(base.begin(), base.end());
  return true;
}

// Run `iters` iterations with one cooperative launch of the persistent kernel.
template <typename T>
void chain_run(tapg_solver_s* S, Slot& sl, int iters, bool timed) {
  hipStream_t st = S->stream;
  ChainArgs<T> c{};
  c.lev = static_cast<const SegArgs<T>*>(sl.d_chain_lev);
  c.nlev = (int)sl.levels.size();
  c.total = sl.chain_total;
  c.iters = iters;
  for (int l = 0; l <= c.nlev; ++l) c.base[l] = sl.chain_base[l];
  c.parents = sl.d_chain_par;
  c.nchild = sl.d_chain_nchild;
  c.bwd_cnt = sl.d_chain_cnt;
  c.fwd_flag = sl.d_chain_cnt + sl.chain_total;
  c.sync = static_cast<ChainSync*>(sl.d_chain_sync);
  c.ctl = sl.d_ctl;
  c.hist = sl.d_hist;
  TAPG_HIP(hipMemsetAsync(sl.d_chain_cnt, 0, sizeof(unsigned) * 2 * sl.chain_total, st));
  TAPG_HIP(hipMemsetAsync(sl.d_chain_sync, 0, sizeof(ChainSync), st));
  if (timed) TAPG_HIP(hipEventRecord(S->tev[0], st));
  hipError_t e = launch_chain<T>(sl.chain_nbm, true, c, sl.chain_lds, st);
  if (e != hipSuccess) throw Fail{TAPG_EDEVICE, std::string("persistent iteration launch: ") + hipGetErrorString(e)};
  if (timed) TAPG_HIP(hipEventRecord(S->tev[1], st));
}

// (p, q) of every tree of a slot (FP64 and sweep precision) and, for the scan
// form, Pi q per tree (the root's parent term z = Pi u_prev), formed on the
// host in FP64 from G = (E E')^{-1} E.
template <typename T>
void upload_pq(tapg_solver_s* S, Slot& sl, const std::vector<double>& pq64, hipStream_t st) {
  std::vector<T> pqT(pq64.begin(), pq64.end());
  TAPG_HIP(hipMemcpyAsync(sl.d_pq64, pq64.data(), pq64.size() * 8, hipMemcpyHostToDevice, st));
  TAPG_HIP(hipMemcpyAsync(sl.d_pq, pqT.data(), pqT.size() * sizeof(T), hipMemcpyHostToDevice, st));
  if (!S->scan) return;
  const NetworkHost& h = S->net;
  const int LDX = S->LDX, LDU = S->LDU, PQ = LDX + LDU;
  const int nt = (int)(pq64.size() / PQ);
  std::vector<T> zr((size_t)nt * LDU, T(0));
  std::vector<double> gq(h.ns);
  for (int k = 0; k < nt; ++k) {
    const double* q = pq64.data() + (size_t)k * PQ + LDX;
    for (int r = 0; r < h.ns; ++r) {
      double acc = 0.0;
      for (int i = 0; i < h.nu; ++i) acc += S->G(r, i) * q[i];
      gq[r] = acc;
    }
    for (int i = 0; i < h.nu; ++i) {
      double acc = 0.0;
      for (int r = 0; r < h.ns; ++r) acc += h.E(r, i) * gq[r];
      zr[(size_t)k * LDU + i] = (T)(q[i] - acc);
    }
  }
  TAPG_HIP(hipMemcpyAsync(sl.d_zr, zr.data(), zr.size() * sizeof(T), hipMemcpyHostToDevice, st));
}

// Per-solve data step of a slot's K nodes (kappa, g; kperp for the scan form,
// or with all_forms wherever the solver allows the scan form).
template <typename T>
void data_step(tapg_solver_s* S, Slot& sl, int K, hipStream_t st, bool all_forms = false) {
  const NetworkHost& h = S->net;
  launch_data_step<T>(K, h.nx, h.nu, h.nd, S->LDX, S->LDU, (const int*)sl.d_stage,
                      (const double*)sl.d_prob64, (const double*)sl.d_demand,
                      (const double*)sl.d_price, (const double*)S->dx.Pd,
                      (const double*)S->dx.Gd, (const double*)S->dx.Gbar,
                      (const double*)S->d64.F, (const double*)S->dx.alpha0,
                      (const double*)S->dx.cE, S->cfg.W_alpha, static_cast<T*>(sl.d_kappa),
                      static_cast<T*>(sl.d_g), h.ns, (const double*)S->dx.Gm,
                      (const double*)S->dx.E,
                      (sl.scan || (all_forms && S->scan)) ? static_cast<T*>(sl.d_kperp) : nullptr,
                      st);
}

template <typename T>
void gap_impl(tapg_solver_s* S, const TreeHost& t, Slot& sl, double gamma, double* out);

// Gap G and dual objective F of the slot's current dual (gap_impl's terms).
template <typename T>
void gap_impl_at(tapg_solver_s* S, const TreeHost& t, Slot& sl, double gamma, double* gap,
                 double* dual_obj) {
  double o[4];
  gap_impl<T>(S, t, sl, gamma, o);
  // F(y) = -f(x') - <y, H x'> + g*(y);  G = f(x') + g(t) + F(y)
  const double F = -o[0] - o[1] + o[2];
  *dual_obj = F;
  *gap = o[0] + o[3] + F;
}

template <typename T>
void solve_impl(tapg_solver_s* S, const TreeHost& t, Slot& sl, const double* p,
                const double* q, bool warm, double gamma, tapg_result& res) {
  const NetworkHost& h = S->net;
  hipStream_t st = S->stream;
  const int LDX = S->LDX, LDU = S->LDU, LDY = S->LDY;
  const int K = t.K;
  // initial condition
  std::vector<double> pq64(LDX + LDU, 0.0);
  for (int i = 0; i < h.nx; ++i) pq64[i] = p[i];
  for (int i = 0; i < h.nu; ++i) pq64[LDX + i] = q[i];
  upload_pq<T>(S, sl, pq64, st);
  sl.last_pq = pq64;
  sl.gap_valid = false;
  // averaged primal: its buffers join the iteration's launches (a graph
  // captured without them is rebuilt)
  if (S->cfg.averaged_primal && !sl.d_ua) {
    sl.d_ua = dmalloc<T>((size_t)K * LDU);
    sl.d_xa = dmalloc<T>((size_t)K * LDX);
    if (sl.graph) (void)hipGraphExecDestroy(sl.graph);
    sl.graph = nullptr;
    sl.chain_state = -1;
  }
  // control block
  DevCtl c{};
  c.max_iter = S->cfg.max_iter;
  // with a gap test the host decides the stop (residual and gap together)
  c.tol = S->cfg.gap_tol > 0.0 ? 0.0 : S->cfg.tol;
  c.rule = S->cfg.beta_rule;
  c.gamma = gamma;
  c.theta = 1.0;
  c.theta_prev = 1.0;
  c.beta = 0.0;
  TAPG_HIP(hipMemcpyAsync(sl.d_ctl, &c, sizeof(c), hipMemcpyHostToDevice, st));
  // dual start
  const size_t ybytes = (size_t)K * LDY * sizeof(T);
  if (warm && sl.has_dual) {
    void* src = sl.last_iter_parity ? sl.d_Y1 : sl.d_Y0;
    void* dst = sl.last_iter_parity ? sl.d_Y0 : sl.d_Y1;
    TAPG_HIP(hipMemcpyAsync(dst, src, ybytes, hipMemcpyDeviceToDevice, st));
  } else {
    TAPG_HIP(hipMemsetAsync(sl.d_Y0, 0, ybytes, st));
    TAPG_HIP(hipMemsetAsync(sl.d_Y1, 0, ybytes, st));
  }
  TAPG_HIP(hipEventRecord(S->ev0, st));
  // data step
  data_step<T>(S, sl, K, st);
  TAPG_HIP(hipGetLastError());
  // iterations, in chunks of check_every with a host check between chunks
  const int chunk = std::max(1, std::min(S->cfg.check_every, S->cfg.max_iter));
  const NetDev<T>& d = net_of<T>(S);
  const bool chain = chain_usable<T>(S, t, sl);
  if (!chain && S->use_graph && !S->time_kernels && (sl.graph == nullptr || sl.graph_iters != chunk)) {
    if (sl.graph) (void)hipGraphExecDestroy(sl.graph);
    sl.graph = nullptr;
    hipGraph_t g = nullptr;
    TAPG_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    enqueue_iterations<T>(S, sl, d, chunk);
    TAPG_HIP(hipStreamEndCapture(st, &g));
    hipError_t e = hipGraphInstantiate(&sl.graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) throw Fail{TAPG_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e)};
    sl.graph_iters = chunk;
  }
  DevCtl hc{};
  int launched = 0;
  double gap = NAN, dual_obj = NAN;
  bool gap_valid = false;
  ProgressLine progress("solve");
  const bool timed = S->time_kernels;
  if (timed) {
    const size_t need = (size_t)2 * (chunk * launches_per_iter(sl) + 1);
    while (S->tev.size() < need) {
      hipEvent_t e;
      TAPG_HIP(hipEventCreate(&e));
      S->tev.push_back(e);
    }
    for (int k = 0; k < 4; ++k) {
      S->kt_ms[k] = 0.0;
      S->kt_n[k] = 0;
    }
  }
  while (chain) {  // persistent iteration: one cooperative launch per chunk
    const int before = hc.iter;
    chain_run<T>(S, sl, chunk, timed);
    launched += chunk;
    ChainSync sync{};
    TAPG_HIP(hipMemcpyAsync(&hc, sl.d_ctl, sizeof(hc), hipMemcpyDeviceToHost, st));
    TAPG_HIP(hipMemcpyAsync(&sync, sl.d_chain_sync, sizeof(sync), hipMemcpyDeviceToHost, st));
    TAPG_HIP(hipStreamSynchronize(st));
    if (sync.error)
      throw Fail{TAPG_EDEVICE, "persistent iteration: a hand-over wait exceeded its bound"};
    if (timed) {
      float ms = 0.f;
      TAPG_HIP(hipEventElapsedTime(&ms, S->tev[0], S->tev[1]));
      S->kt_ms[3] += ms;
      S->kt_n[3] += hc.iter - before;
    }
    progress.tick(launched, hc.done ? 0 : 1, 1);
    if (hc.done || launched >= S->cfg.max_iter) break;
  }
  while (!chain) {
    if (timed) {
      // The chunk's launches, each between two events, are queued behind a
      // short hold on the device (sized from the previous chunk's host enqueue
      // time), so that all of them are queued before the first starts and the
      // event pairs time the kernels, not the host.  Launches of iterations
      // after the stop (no-ops) are not counted.
      TAPG_HIP(hipMemcpyAsync(&hc, sl.d_ctl, sizeof(hc), hipMemcpyDeviceToHost, st));
      TAPG_HIP(hipStreamSynchronize(st));
      const int before = hc.iter;
      launch_hold((long long)(std::min(S->hold_us, 50000.0) * S->wall_clock_mhz), st);
      const auto h0 = std::chrono::steady_clock::now();
      TimedCursor tc;
      enqueue_iterations<T>(S, sl, d, chunk, &tc);
      const double enq_us =
          std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - h0).count();
      S->hold_us = 1.5 * enq_us + 200.0;
      TAPG_HIP(hipGetLastError());
      TAPG_HIP(hipMemcpyAsync(&hc, sl.d_ctl, sizeof(hc), hipMemcpyDeviceToHost, st));
      TAPG_HIP(hipStreamSynchronize(st));
      const int ran = hc.iter - before;  // iterations that did work
      for (int k = 0; k < tc.next; ++k) {
        if (tc.it[k] >= ran) continue;  // after the stop: a no-op
        float ms = 0.f;
        TAPG_HIP(hipEventElapsedTime(&ms, S->tev[2 * k], S->tev[2 * k + 1]));
        S->kt_ms[tc.kind[k]] += ms;
        S->kt_n[tc.kind[k]] += 1;
      }
    } else if (S->use_graph) {
      TAPG_HIP(hipGraphLaunch(sl.graph, st));
    } else {
      enqueue_iterations<T>(S, sl, d, chunk);
      TAPG_HIP(hipGetLastError());
    }
    launched += chunk;
    TAPG_HIP(hipMemcpyAsync(&hc, sl.d_ctl, sizeof(hc), hipMemcpyDeviceToHost, st));
    TAPG_HIP(hipStreamSynchronize(st));
    progress.tick(launched, hc.done ? 0 : 1, 1);
    if (!hc.done && S->cfg.gap_tol > 0.0 && (S->cfg.tol <= 0.0 || hc.last_res <= S->cfg.tol)) {
      // stop when the duality gap of the current dual is within gap_tol and
      // the last iteration's residual within tol (tested between chunks)
      sl.last_iter_parity = hc.iter & 1;
      sl.has_dual = true;
      double F = 0.0;
      gap_impl_at<T>(S, t, sl, gamma, &gap, &F);
      dual_obj = F;
      if (std::fabs(gap) <= S->cfg.gap_tol) {
        hc.done = 1;
        hc.converged = 1;
        TAPG_HIP(hipMemcpyAsync(sl.d_ctl, &hc, sizeof(hc), hipMemcpyHostToDevice, st));
        gap_valid = true;
      }
    }
    if (hc.done || launched >= S->cfg.max_iter) break;
  }
  TAPG_HIP(hipEventRecord(S->ev1, st));
  if (sl.d_ua) {  // the averaged primal is the one returned
    TAPG_HIP(hipMemcpyAsync(sl.d_u, sl.d_ua, (size_t)K * LDU * sizeof(T), hipMemcpyDeviceToDevice, st));
    TAPG_HIP(hipMemcpyAsync(sl.d_x, sl.d_xa, (size_t)K * LDX * sizeof(T), hipMemcpyDeviceToDevice, st));
  }
  // cost and violations of the final primal iterate
  launch_cost<T>(K, h.nx, h.nu, h.nd, h.ns, LDX, LDU, (const int*)sl.d_anc,
                 (const double*)sl.d_prob64, (const double*)sl.d_demand,
                 (const double*)sl.d_price, (const T*)sl.d_u, (const T*)sl.d_x,
                 (const double*)sl.d_pq64, (const double*)S->d64.A, (const double*)S->d64.B,
                 (const double*)S->dx.Gd, (const double*)S->dx.E, (const double*)S->dx.Ed,
                 (const double*)S->dx.Wu, (const double*)S->dx.alpha0, (const double*)S->dx.cE,
                 (const double*)S->d64.xmin, (const double*)S->d64.xmax,
                 (const double*)S->d64.xs, (const double*)S->d64.umin,
                 (const double*)S->d64.umax, S->cfg.W_alpha, S->cfg.W_x, S->cfg.W_s, sl.d_part,
                 S->dx.red, st);
  TAPG_HIP(hipGetLastError());
  double red[3];
  TAPG_HIP(hipMemcpyAsync(red, S->dx.red, sizeof(red), hipMemcpyDeviceToHost, st));
  TAPG_HIP(hipStreamSynchronize(st));
  float ms = 0.f;
  TAPG_HIP(hipEventElapsedTime(&ms, S->ev0, S->ev1));
  res.iters = hc.iter;
  res.converged = hc.converged;
  res.primal_res = hc.last_res;
  res.cost = red[0];
  res.viol_box = red[1];
  res.viol_eq = red[2];
  res.gamma = gamma;
  res.solve_ms = ms;
  // the gap is of the dual the solve returns: the one the gap test saw when it
  // stopped the solve, else (a gap test that did not stop it) re-evaluated
  sl.has_dual = true;
  sl.last_iter_parity = hc.iter & 1;
  if (S->cfg.gap_tol > 0.0 && !gap_valid && !hc.numeric) {
    gap_impl_at<T>(S, t, sl, gamma, &gap, &dual_obj);
    gap_valid = true;
  }
  res.dual_gap = gap_valid ? gap : NAN;
  res.dual_obj = gap_valid ? dual_obj : NAN;
  sl.numeric = hc.numeric != 0;
  sl.last = res;
  sl.gap_valid = gap_valid;
  sl.has_result = true;
  if (hc.numeric) throw Fail{TAPG_ENUMERIC, "non-finite dual residual (diverging iterates; infeasible data or step size too large)"};
}

template <typename T>
double power_impl(tapg_solver_s* S, const TreeHost& t, Slot& sl, int iters) {
  const NetworkHost& h = S->net;
  hipStream_t st = S->stream;
  const int K = t.K, LDX = S->LDX, LDY = S->LDY;
  if (!sl.d_P0) {
    sl.d_P0 = dmalloc<T>((size_t)K * LDY);
    sl.d_P1 = dmalloc<T>((size_t)K * LDY);
    TAPG_HIP(hipMemsetAsync(sl.d_P1, 0, (size_t)K * LDY * sizeof(T), st));
  }
  std::vector<T> v((size_t)K * LDY, T(0));
  std::mt19937_64 rng(0x5eed1234ull);
  std::normal_distribution<double> nd(0.0, 1.0);
  double nrm2 = 0.0;
  for (int n = 0; n < K; ++n) {
    T* yn = v.data() + (size_t)n * LDY;
    for (int i = 0; i < h.nx; ++i) { yn[i] = (T)nd(rng); nrm2 += (double)yn[i] * yn[i]; }
    for (int i = 0; i < h.nx; ++i) { yn[LDX + i] = (T)nd(rng); nrm2 += (double)yn[LDX + i] * yn[LDX + i]; }
    for (int i = 0; i < h.nu; ++i) { yn[2 * LDX + i] = (T)nd(rng); nrm2 += (double)yn[2 * LDX + i] * yn[2 * LDX + i]; }
  }
  TAPG_HIP(hipMemcpyAsync(sl.d_P0, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, st));
  DevCtl c{};
  c.pw_scale = 1.0 / std::sqrt(nrm2);
  c.max_iter = iters + 1;
  TAPG_HIP(hipMemcpyAsync(sl.d_ctl, &c, sizeof(c), hipMemcpyHostToDevice, st));
  const NetDev<T>& d = net_of<T>(S);
  for (int i = 0; i < iters; ++i) enqueue_iteration<T>(S, sl, d, 1);
  TAPG_HIP(hipGetLastError());
  DevCtl hc{};
  TAPG_HIP(hipMemcpyAsync(&hc, sl.d_ctl, sizeof(hc), hipMemcpyDeviceToHost, st));
  TAPG_HIP(hipStreamSynchronize(st));
  return hc.L;
}

// Duality gap of the tree's current dual (the iterate its last solve returned),
// FP64 whatever the sweep precision: the dual widened to FP64, one
// dual-gradient evaluation at w = y on the per-stage kernels (FP64 factors and
// data step), then the per-node gap terms.  out[0..3]: f(x'), <y, H x'>,
// g*(y), g(t) (see gap_kernels.hip).
template <typename T>
void gap_impl(tapg_solver_s* S, const TreeHost& t, Slot& sl, double gamma, double* out) {
  const NetworkHost& h = S->net;
  hipStream_t st = S->stream;
  const int K = t.K, N = t.N, LDX = S->LDX, LDU = S->LDU, LDY = S->LDY;
  if (sl.last_pq.size() != (size_t)(LDX + LDU)) throw Fail{TAPG_ESTATE, "no solve of this tree yet"};
  struct Tmp {
    std::vector<void*> p;
    ~Tmp() {  // back to the block cache (the stream has been synchronised)
      for (void* q : p) block_cache().put(q);
    }
    double* get(size_t n) {
      void* q = dev_alloc(std::max<size_t>(n, 1) * sizeof(double));
      p.push_back(q);
      return static_cast<double*>(q);
    }
  } tmp;
  const T* ycur = static_cast<const T*>(sl.last_iter_parity ? sl.d_Y1 : sl.d_Y0);
  const double* y64;
  if (sizeof(T) == sizeof(double)) {
    y64 = reinterpret_cast<const double*>(ycur);
  } else {
    double* w = tmp.get((size_t)K * LDY);
    launch_widen<T>(ycur, w, (size_t)K * LDY, st);
    y64 = w;
  }
  double* lam = tmp.get((size_t)K * LDX);
  double* jv = tmp.get((size_t)K * LDU);
  double* u = tmp.get((size_t)K * LDU);
  double* x = tmp.get((size_t)K * LDX);
  double* kap = tmp.get((size_t)K * LDU);
  double* g = tmp.get((size_t)K * LDX);
  double* invp = tmp.get(K);
  double* pq = tmp.get(LDX + LDU);
  double* part = tmp.get((size_t)K * 4);
  double* red = tmp.get(4);
  DevCtl* ctl = reinterpret_cast<DevCtl*>(tmp.get((sizeof(DevCtl) + 7) / 8));
  std::vector<double> ip(K);
  for (int n = 0; n < K; ++n) ip[n] = 1.0 / t.prob[n];
  TAPG_HIP(hipMemcpyAsync(invp, ip.data(), (size_t)K * 8, hipMemcpyHostToDevice, st));
  TAPG_HIP(hipMemcpyAsync(pq, sl.last_pq.data(), sl.last_pq.size() * 8, hipMemcpyHostToDevice, st));
  DevCtl c{};
  c.gamma = gamma;
  c.max_iter = 1;
  c.theta = c.theta_prev = 1.0;
  TAPG_HIP(hipMemcpyAsync(ctl, &c, sizeof(c), hipMemcpyHostToDevice, st));
  TAPG_HIP(hipMemsetAsync(lam, 0, (size_t)K * LDX * 8, st));
  TAPG_HIP(hipMemsetAsync(jv, 0, (size_t)K * LDU * 8, st));
  launch_data_step<double>(K, h.nx, h.nu, h.nd, LDX, LDU, (const int*)sl.d_stage,
                           (const double*)sl.d_prob64, (const double*)sl.d_demand,
                           (const double*)sl.d_price, (const double*)S->dx.Pd,
                           (const double*)S->dx.Gd, (const double*)S->dx.Gbar,
                           (const double*)S->d64.F, (const double*)S->dx.alpha0,
                           (const double*)S->dx.cE, S->cfg.W_alpha, kap, g, h.ns,
                           (const double*)S->dx.Gm, (const double*)S->dx.E, nullptr, st);
  const NetDev<double>& d = S->d64;
  SweepArgs<double> a{};
  a.nx = h.nx;
  a.nu = h.nu;
  a.LDX = LDX;
  a.LDU = LDU;
  a.LDY = LDY;
  a.mode = 2;
  a.anc = sl.d_anc;
  a.cbeg = sl.d_cbeg;
  a.cend = sl.d_cend;
  a.invp = invp;
  a.At = d.At;
  a.Bt = d.Bt;
  a.A = d.A;
  a.B = d.B;
  a.xmin = d.xmin;
  a.xmax = d.xmax;
  a.xs = d.xs;
  a.umin = d.umin;
  a.umax = d.umax;
  a.Wx = S->cfg.W_x;
  a.Ws = S->cfg.W_s;
  a.kappa = kap;
  a.g = g;
  a.pq = pq;
  a.Y0 = const_cast<double*>(y64);  // read only in evaluation mode; w = y (beta = 0)
  a.Y1 = const_cast<double*>(y64);
  a.lam = lam;
  a.jv = jv;
  a.u = u;
  a.x = x;
  a.ctl = ctl;
  a.part = part;
  const size_t fstride = (size_t)LDU * LDU;
  for (int pass = 0; pass < 2; ++pass) {
    for (int q = 0; q < N; ++q) {
      const int s = pass == 0 ? N - 1 - q : q;
      const int width = t.offset[s + 1] - t.offset[s];
      const int nb = pick_nb(width, sizeof(double), LDX, LDU, LDY);
      a.s = s;
      a.node0 = t.offset[s];
      a.count = width;
      a.tile_base = 0;
      a.F = d.F + s * fstride;
      a.Kb = d.Kb + s * fstride;
      if (pass == 0)
        launch_bwd_stage<double>(nb, a, (width + nb - 1) / nb, st);
      else
        launch_fwd_stage<double>(nb, a, (width + nb - 1) / nb, st);
    }
  }
  launch_gap_terms(K, h.nx, h.nu, LDX, LDU, LDY, sl.d_anc, (const double*)sl.d_prob64,
                   (const double*)sl.d_price, y64, u, x, pq, (const double*)S->dx.Wu,
                   (const double*)S->dx.alpha0, (const double*)S->dx.cE, d.xmin, d.xmax, d.xs,
                   d.umin, d.umax, S->cfg.W_alpha, S->cfg.W_x, S->cfg.W_s, gamma, part, red, st);
  TAPG_HIP(hipGetLastError());
  TAPG_HIP(hipMemcpyAsync(out, red, 4 * sizeof(double), hipMemcpyDeviceToHost, st));
  TAPG_HIP(hipStreamSynchronize(st));
}

// ---------------------------------------------------------------------------
// Solve without allocating (tapg_solve_noalloc): every buffer of the solve
// lives in one file-scope device array, `scratch`, of TAPG_NOALLOC_SCRATCH_BYTES.
// Host code never uses the array's name as an address: its device address is
// looked up once per device at solver creation (hipGetSymbolAddress, with the
// device current) and kept in g_scratch[device].  Each GPU holds its own copy
// until the process ends; calls on one device are serialised by g_scratch_mu,
// and each call overwrites what the previous one left.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[TAPG_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch[kMaxDevices] = {};

__global__ __launch_bounds__(kThreads) void fill_zero_kernel(unsigned* p, size_t n) {
  for (size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x; i < n;
       i += (size_t)gridDim.x * kThreads)
    p[i] = 0u;
}

// Byte offsets of one solve's buffers inside the scratch array.
struct NoallocLayout {
  size_t anc, cbeg, cend, stage, prob, demand, price, pq64, part, red, hist, ctl;
  size_t invp, kappa, g, pq, y0, y1, lam, jv, u, x;
  size_t total;
};

NoallocLayout noalloc_layout(const tapg_solver_s* S, const TreeHost& t, size_t e) {
  NoallocLayout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += (std::max<size_t>(bytes, 1) + 255) & ~(size_t)255;
    return o;
  };
  const size_t K = t.K, LDX = S->LDX, LDU = S->LDU, LDY = S->LDY;
  L.anc = take(K * 4);
  L.cbeg = take(K * 4);
  L.cend = take(K * 4);
  L.stage = take(K * 4);
  L.prob = take(K * 8);
  L.demand = take(K * t.nd * 8);
  L.price = take(K * 8);
  L.pq64 = take((LDX + LDU) * 8);
  L.part = take(4 * K * 8);
  L.red = take(8 * 8);
  L.hist = take((size_t)std::max(1, S->cfg.max_iter) * 8);
  L.ctl = take(2 * sizeof(DevCtl));
  L.invp = take(K * e);
  L.kappa = take(K * LDU * e);
  L.g = take(K * LDX * e);
  L.pq = take((LDX + LDU) * e);
  L.y0 = take(K * LDY * e);
  L.y1 = take(K * LDY * e);
  L.lam = take(K * LDX * e);
  L.jv = take(K * LDU * e);
  L.u = take(K * LDU * e);
  L.x = take(K * LDX * e);
  L.total = off;
  return L;
}

template <typename T>
void noalloc_impl(tapg_solver_s* S, const TreeHost& t, unsigned char* base, const double* p,
                  const double* q, double gamma, tapg_result& res, double* u0, double* u_out,
                  double* x_out) {
  const NetworkHost& h = S->net;
  hipStream_t st = S->stream;
  const int K = t.K, LDX = S->LDX, LDU = S->LDU, LDY = S->LDY;
  const NoallocLayout L = noalloc_layout(S, t, sizeof(T));
  // a local slot whose buffers are views into the scratch array (never freed)
  Slot sl;
  sl.K = K;
  sl.N = t.N;
  sl.elem = sizeof(T);
  sl.d_anc = reinterpret_cast<int*>(base + L.anc);
  sl.d_cbeg = reinterpret_cast<int*>(base + L.cbeg);
  sl.d_cend = reinterpret_cast<int*>(base + L.cend);
  sl.d_stage = reinterpret_cast<int*>(base + L.stage);
  sl.d_prob64 = reinterpret_cast<double*>(base + L.prob);
  sl.d_demand = reinterpret_cast<double*>(base + L.demand);
  sl.d_price = reinterpret_cast<double*>(base + L.price);
  sl.d_pq64 = reinterpret_cast<double*>(base + L.pq64);
  sl.d_part = reinterpret_cast<double*>(base + L.part);
  sl.d_hist = reinterpret_cast<double*>(base + L.hist);
  sl.hist_cap = std::max(1, S->cfg.max_iter);
  sl.d_ctl = reinterpret_cast<DevCtl*>(base + L.ctl);
  sl.d_invp = base + L.invp;
  sl.d_kappa = base + L.kappa;
  sl.d_g = base + L.g;
  sl.d_pq = base + L.pq;
  sl.d_Y0 = base + L.y0;
  sl.d_Y1 = base + L.y1;
  sl.d_lam = base + L.lam;
  sl.d_j = base + L.jv;
  sl.d_u = base + L.u;
  sl.d_x = base + L.x;
  double* red = reinterpret_cast<double*>(base + L.red);
  // per-stage kernels (no schedule tables): tiles as a solver slot would hold them
  sl.segmented = false;
  sl.node_offset = t.offset;
  sl.nb_of_stage.resize(t.N);
  sl.tiles_of_stage.resize(t.N);
  sl.tile_offset.resize(t.N + 1);
  int tot = 0;
  for (int s = 0; s < t.N; ++s) {
    const int nb = pick_nb(t.mu[s], sizeof(T), LDX, LDU, LDY);
    sl.nb_of_stage[s] = nb;
    sl.tiles_of_stage[s] = (t.mu[s] + nb - 1) / nb;
    sl.tile_offset[s] = tot;
    tot += sl.tiles_of_stage[s];
  }
  sl.tile_offset[t.N] = tot;
  sl.total_tiles = tot;
  // tree, data and initial state in (the host arrays stay alive until the sync below)
  std::vector<T> ip(K);
  for (int n = 0; n < K; ++n) ip[n] = (T)(1.0 / t.prob[n]);
  std::vector<double> pq64((size_t)LDX + LDU, 0.0);
  for (int i = 0; i < h.nx; ++i) pq64[i] = p[i];
  for (int i = 0; i < h.nu; ++i) pq64[LDX + i] = q[i];
  std::vector<T> pqT(pq64.begin(), pq64.end());
  DevCtl c{};
  c.max_iter = S->cfg.max_iter;
  c.tol = S->cfg.tol;
  c.rule = S->cfg.beta_rule;
  c.gamma = gamma;
  c.theta = c.theta_prev = 1.0;
  auto h2d = [&](void* dst, const void* src, size_t bytes) {
    TAPG_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st));
  };
  h2d(sl.d_anc, t.anc.data(), (size_t)K * 4);
  h2d(sl.d_cbeg, t.cbeg.data(), (size_t)K * 4);
  h2d(sl.d_cend, t.cend.data(), (size_t)K * 4);
  h2d(sl.d_stage, t.stage.data(), (size_t)K * 4);
  h2d(sl.d_prob64, t.prob.data(), (size_t)K * 8);
  h2d(sl.d_demand, t.demand.data(), (size_t)K * t.nd * 8);
  h2d(sl.d_price, t.price.data(), (size_t)K * 8);
  h2d(sl.d_invp, ip.data(), (size_t)K * sizeof(T));
  h2d(sl.d_pq64, pq64.data(), pq64.size() * 8);
  h2d(sl.d_pq, pqT.data(), pqT.size() * sizeof(T));
  h2d(sl.d_ctl, &c, sizeof(c));
  // cold start: both dual buffers zero (a fill kernel, as the rest of the path)
  const size_t ywords = (L.y1 - L.y0) / 4 * 2;  // Y0 and Y1 are adjacent
  hipLaunchKernelGGL(fill_zero_kernel, dim3(1024), dim3(kThreads), 0, st,
                     reinterpret_cast<unsigned*>(base + L.y0), ywords);
  TAPG_HIP(hipEventRecord(S->ev0, st));
  data_step<T>(S, sl, K, st);
  const int chunk = std::max(1, std::min(S->cfg.check_every, S->cfg.max_iter));
  const NetDev<T>& d = net_of<T>(S);
  DevCtl hc{};
  int launched = 0;
  while (true) {
    enqueue_iterations<T>(S, sl, d, chunk);
    TAPG_HIP(hipGetLastError());
    launched += chunk;
    TAPG_HIP(hipMemcpyAsync(&hc, sl.d_ctl, sizeof(hc), hipMemcpyDeviceToHost, st));
    TAPG_HIP(hipStreamSynchronize(st));
    if (hc.done || launched >= S->cfg.max_iter) break;
  }
  TAPG_HIP(hipEventRecord(S->ev1, st));
  launch_cost<T>(K, h.nx, h.nu, h.nd, h.ns, LDX, LDU, sl.d_anc, sl.d_prob64, sl.d_demand,
                 sl.d_price, (const T*)sl.d_u, (const T*)sl.d_x, sl.d_pq64,
                 (const double*)S->d64.A, (const double*)S->d64.B, (const double*)S->dx.Gd,
                 (const double*)S->dx.E, (const double*)S->dx.Ed, (const double*)S->dx.Wu,
                 (const double*)S->dx.alpha0, (const double*)S->dx.cE,
                 (const double*)S->d64.xmin, (const double*)S->d64.xmax,
                 (const double*)S->d64.xs, (const double*)S->d64.umin,
                 (const double*)S->d64.umax, S->cfg.W_alpha, S->cfg.W_x, S->cfg.W_s, sl.d_part,
                 red, st);
  TAPG_HIP(hipGetLastError());
  double r3[3];
  TAPG_HIP(hipMemcpyAsync(r3, red, sizeof(r3), hipMemcpyDeviceToHost, st));
  std::vector<T> uh, xh;
  if (u0 || u_out) {
    uh.resize((size_t)(u_out ? K : 1) * LDU);
    TAPG_HIP(hipMemcpyAsync(uh.data(), sl.d_u, uh.size() * sizeof(T), hipMemcpyDeviceToHost, st));
  }
  if (x_out) {
    xh.resize((size_t)K * LDX);
    TAPG_HIP(hipMemcpyAsync(xh.data(), sl.d_x, xh.size() * sizeof(T), hipMemcpyDeviceToHost, st));
  }
  TAPG_HIP(hipStreamSynchronize(st));
  float ms = 0.f;
  TAPG_HIP(hipEventElapsedTime(&ms, S->ev0, S->ev1));
  if (u0)
    for (int i = 0; i < h.nu; ++i) u0[i] = (double)uh[i];
  if (u_out)
    for (int n = 0; n < K; ++n)
      for (int i = 0; i < h.nu; ++i) u_out[(size_t)n * h.nu + i] = (double)uh[(size_t)n * LDU + i];
  if (x_out)
    for (int n = 0; n < K; ++n)
      for (int i = 0; i < h.nx; ++i) x_out[(size_t)n * h.nx + i] = (double)xh[(size_t)n * LDX + i];
  res = tapg_result{};
  res.iters = hc.iter;
  res.converged = hc.converged;
  res.primal_res = hc.last_res;
  res.cost = r3[0];
  res.viol_box = r3[1];
  res.viol_eq = r3[2];
  res.gamma = gamma;
  res.solve_ms = ms;
  res.dual_gap = res.dual_obj = NAN;
  if (hc.numeric) throw Fail{TAPG_ENUMERIC, "non-finite dual residual (diverging iterates; infeasible data or step size too large)"};
}

}  // namespace

// ---------------------------------------------------------------------------
// Exported device-layer entry points
// ---------------------------------------------------------------------------
size_t dev_noalloc_bytes(const tapg_solver_s* S, const TreeHost& t) {
  return noalloc_layout(S, t, S->fp32 ? sizeof(float) : sizeof(double)).total;
}

void dev_solve_noalloc(tapg_solver_s* S, const TreeHost& t, const double* p, const double* q,
                       double gamma, tapg_result& res, double* u0, double* u_out, double* x_out) {
  if (S->device < 0 || S->device >= kMaxDevices) throw Fail{TAPG_EDEVICE, "device ordinal out of range"};
  TAPG_HIP(hipSetDevice(S->device));
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  unsigned char* base = static_cast<unsigned char*>(g_scratch[S->device]);
  if (!base) throw Fail{TAPG_ESTATE, "scratch array of this device not set up"};
  const size_t need = dev_noalloc_bytes(S, t);
  if (need > (size_t)TAPG_NOALLOC_SCRATCH_BYTES)
    throw Fail{TAPG_ENOMEM, "tapg_solve_noalloc: the tree needs " + std::to_string(need) +
                                " bytes of scratch; the library holds " +
                                std::to_string((size_t)TAPG_NOALLOC_SCRATCH_BYTES) +
                                " (use tapg_solve)"};
  if (S->fp32)
    noalloc_impl<float>(S, t, base, p, q, gamma, res, u0, u_out, x_out);
  else
    noalloc_impl<double>(S, t, base, p, q, gamma, res, u0, u_out, x_out);
}

void dev_gap(tapg_solver_s* S, const TreeHost& t, Slot& sl, double* gap, double* dual_obj) {
  TAPG_HIP(hipSetDevice(S->device));
  if (!sl.has_dual) throw Fail{TAPG_ESTATE, "no dual for this tree yet"};
  if (S->fp32)
    gap_impl_at<float>(S, t, sl, sl.last.gamma, gap, dual_obj);
  else
    gap_impl_at<double>(S, t, sl, sl.last.gamma, gap, dual_obj);
  sl.last.dual_gap = *gap;
  sl.last.dual_obj = *dual_obj;
  sl.gap_valid = true;
}

void dev_init(tapg_solver_s* S) {
  TAPG_HIP(hipSetDevice(S->device));
  {
    int lds = 0;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, S->device) ==
            hipSuccess &&
        lds > 0)
      S->lds_limit = (size_t)lds;
    int khz = 0;  // the wall clock that the kernel-timing hold counts
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, S->device) == hipSuccess &&
        khz > 0)
      S->wall_clock_mhz = khz / 1000.0;
  }
  {  // structure of A and W_u; segment kernels need nx, nu <= 128
    const NetworkHost& h = S->net;
    bool ai = true;
    for (int i = 0; i < h.nx; ++i)
      for (int j = 0; j < h.nx; ++j)
        if (h.A(i, j) != (i == j ? 1.0 : 0.0)) ai = false;
    S->a_ident = ai;
    const double w0 = S->Wu[0];
    bool ws = w0 > 0.0;
    for (int i = 0; i < h.nu; ++i)
      for (int j = 0; j < h.nu; ++j)
        if (S->Wu[(size_t)i * h.nu + j] != (i == j ? w0 : 0.0)) ws = false;
    S->wu_scalar = ws;
    S->wu = ws ? w0 : 1.0;
    // projector form: G = (E E')^{-1} E by Cholesky of E E' (E has full row
    // rank); used when G is sparse, as for mixing nodes with disjoint inputs
    const char* pe = std::getenv("TAPG_PROJ");
    S->proj = false;
    if (ws && S->seg_ok && !(pe && pe[0] == '0')) {
      Mat G(h.ns, h.nu);
      bool ok = true;
      if (h.ns > 0) {
        Mat EEt = matmul(h.E, transpose(h.E));
        ok = cholesky(EEt);
        if (ok) {
          G = h.E;
          chol_solve(EEt, G);
        }
      }
      int nnz = 0, nnzE = 0;
      for (double v : G.a) nnz += v != 0.0;
      for (double v : h.E.a) nnzE += v != 0.0;
      if (ok && nnz <= 16 * std::max(1, h.ns)) {
        S->proj = true;
        S->G = G;
        S->nnzG = nnz;
        S->nnzE = nnzE;
      }
    }
    const char* se = std::getenv("TAPG_SCAN");
    S->scan = S->proj && ai && h.nx <= 64 && !(se && se[0] == '0');
    S->scan_default = S->scan;  // untuned shapes: the scan form wherever it applies
  }
  if (S->stream == nullptr) {
    TAPG_HIP(hipStreamCreateWithFlags(&S->stream, hipStreamNonBlocking));
    S->own_stream = true;
  }
  TAPG_HIP(hipEventCreate(&S->ev0));
  TAPG_HIP(hipEventCreate(&S->ev1));
  {  // device address of this device's scratch array (tapg_solve_noalloc), once
    if (S->device < 0 || S->device >= kMaxDevices) throw Fail{TAPG_EDEVICE, "device ordinal out of range"};
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch[S->device]) {
      void* ptr = nullptr;
      const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
      if (e != hipSuccess || ptr == nullptr)
        throw Fail{TAPG_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e)};
      g_scratch[S->device] = ptr;
    }
  }
  const NetworkHost& h = S->net;
  hipStream_t st = S->stream;
  init_net<double>(S, S->d64);
  if (S->fp32) init_net<float>(S, S->d32);
  S->dx.Gd = upload(colmajor<double>(h.Gd, S->LDX, false), st);
  S->dx.Pd = upload(colmajor<double>(h.Pd, S->LDU, false), st);
  S->dx.E = upload(h.E.a.empty() ? std::vector<double>(1, 0.0) : h.E.a, st);
  if (S->proj) S->dx.Gm = upload(S->G.a.empty() ? std::vector<double>(1, 0.0) : S->G.a, st);
  S->dx.Ed = upload(h.Ed.a.empty() ? std::vector<double>(1, 0.0) : h.Ed.a, st);
  S->dx.Wu = upload(colmajor<double>(Mat::from(S->Wu.data(), h.nu, h.nu), S->LDU, false), st);
  S->dx.alpha0 = upload(padvec<double>(S->alpha0, S->LDU), st);
  S->dx.cE = upload(padvec<double>(S->cE, S->LDU), st);
  S->dx.red = dmalloc<double>(8);
  TAPG_HIP(hipStreamSynchronize(st));
}

void free_chain(Slot& sl);
void free_up(Slot& sl);

void free_fwd_full(Slot& sl) {
  dfree(sl.fwd_full.d_ranges);
  dfree(sl.fwd_full.d_wgtree);
  dfree(sl.fwd_full.d_wgx);
  dfree(sl.d_own);
  sl.fwd_full = Slot::Level{0, -1, 0, 1, 0, nullptr, nullptr};
  sl.d_own = nullptr;
}

void dev_free_slot(Slot& sl) {
  if (sl.graph) (void)hipGraphExecDestroy(sl.graph);
  sl.graph = nullptr;
  dfree(sl.d_anc); dfree(sl.d_cbeg); dfree(sl.d_cend); dfree(sl.d_stage);
  dfree(sl.d_prob64); dfree(sl.d_invp); dfree(sl.d_demand); dfree(sl.d_price);
  dfree(sl.d_kappa); dfree(sl.d_g); dfree(sl.d_pq); dfree(sl.d_pq64);
  dfree(sl.d_P0); dfree(sl.d_P1);
  dfree(sl.d_Y0); dfree(sl.d_Y1); dfree(sl.d_lam); dfree(sl.d_j); dfree(sl.d_u); dfree(sl.d_x);
  dfree(sl.d_ua); dfree(sl.d_xa);
  dfree(sl.d_kperp); dfree(sl.d_zb); dfree(sl.d_zr);
  dfree(sl.d_ctl); dfree(sl.d_hist); dfree(sl.d_part);
  free_chain(sl);
  free_up(sl);
  for (auto& L : sl.levels) {
    dfree(L.d_ranges);
    dfree(L.d_wgtree);
    dfree(L.d_wgx);
  }
  sl.levels.clear();
  free_fwd_full(sl);
}

void dev_release(tapg_solver_s* S) {
  if (S->device >= 0) (void)hipSetDevice(S->device);
  if (S->stream) (void)hipStreamSynchronize(S->stream);
  for (auto& kv : S->slots) dev_free_slot(kv.second);
  S->slots.clear();
  for (auto& kv : S->batches) {
    dfree(kv.second.d_map);
    dfree(kv.second.d_tstart);
    dfree(kv.second.d_red);
  }
  S->batches.clear();
  free_net(S->d64);
  free_net(S->d32);
  dfree(S->dx.Gd); dfree(S->dx.Pd); dfree(S->dx.Gbar); dfree(S->dx.E); dfree(S->dx.Ed);
  dfree(S->dx.Gm);
  dfree(S->dx.Wu); dfree(S->dx.alpha0); dfree(S->dx.cE); dfree(S->dx.red);
  dfree(S->d_fid);
  for (hipEvent_t e : S->tev) (void)hipEventDestroy(e);
  S->tev.clear();
  if (S->ev0) (void)hipEventDestroy(S->ev0);
  if (S->ev1) (void)hipEventDestroy(S->ev1);
  S->ev0 = S->ev1 = nullptr;
  if (S->own_stream && S->stream) (void)hipStreamDestroy(S->stream);
  S->stream = nullptr;
}

void dev_upload_factors(tapg_solver_s* S) {
  TAPG_HIP(hipSetDevice(S->device));
  const int nu = S->net.nu, LDU = S->LDU, N = S->N;
  hipStream_t st = S->stream;
  auto pack = [&](const std::vector<double>& src, auto tag) {
    using T = decltype(tag);
    std::vector<T> out((size_t)N * LDU * LDU, T(0));
    for (int s = 0; s < N; ++s)
      for (int r = 0; r < nu; ++r)
        for (int k = 0; k < nu; ++k)
          out[(size_t)s * LDU * LDU + (size_t)k * LDU + r] =
              (T)src[(size_t)s * nu * nu + (size_t)r * nu + k];
    return out;
  };
  dfree(S->d_fid);
  S->d_fid = upload(S->fid, st);
  dfree(S->d64.F); dfree(S->d64.Kb); dfree(S->dx.Gbar);
  S->d64.F = upload(pack(S->Fbar, double{}), st);
  S->d64.Kb = upload(pack(S->Kbar, double{}), st);
  S->dx.Gbar = upload(pack(S->Gbar, double{}), st);
  if (S->fp32) {
    dfree(S->d32.F); dfree(S->d32.Kb);
    S->d32.F = upload(pack(S->Fbar, float{}), st);
    S->d32.Kb = upload(pack(S->Kbar, float{}), st);
  }
  // every cached iteration graph refers to the old factor buffers
  for (auto& kv : S->slots) {
    if (kv.second.graph) (void)hipGraphExecDestroy(kv.second.graph);
    kv.second.graph = nullptr;
  }
  TAPG_HIP(hipStreamSynchronize(st));
}

// Cost-model time of one node-column of a stage (us), for the planner.
double seg_node_us(const tapg_solver_s* S) {
  return (double)S->net.nu * S->net.nu / 64.0 / 2400.0 * (S->fp32 ? 0.5 : 1.0);
}

// Shape of a tree or forest: the per-tree stage widths (the schedule depends
// on nothing else).
std::string shape_key(const TreeHost& t) {
  std::string k = std::to_string(t.ntrees) + "|" + std::to_string(t.N);
  for (int s = 0; s < t.N; ++s)
    for (int j = 0; j < t.ntrees; ++j) k += "," + std::to_string(t.seg_end(s, j) - t.seg_begin(s, j));
  return k;
}

// Schedule of a new slot: TAPG_LEVELS, else a plan the autotuner chose for
// this shape, else the planner's.
std::vector<LevelPlan> choose_plans(tapg_solver_s* S, const TreeHost& t) {
  const char* spec = std::getenv("TAPG_LEVELS");
  if (spec && spec[0]) return levels_from_env(t, spec);
  auto it = S->tuned.find(shape_key(t));
  if (it != S->tuned.end()) return it->second;
  return plan_levels(t, kSegNbMax, seg_node_us(S));
}

// Resources of the persistent iteration of a slot (rebuilt on demand).
void free_chain(Slot& sl) {
  if (sl.d_chain_lev) (void)hipFree(sl.d_chain_lev);
  if (sl.d_chain_sync) (void)hipFree(sl.d_chain_sync);
  sl.d_chain_lev = nullptr;
  sl.d_chain_sync = nullptr;
  dfree(sl.d_chain_par);
  dfree(sl.d_chain_nchild);
  dfree(sl.d_chain_cnt);
  sl.chain_state = 0;
}

// The scan form's forward launch: the bottom level's workgroups, each given
// the ancestors of its nodes at every stage above the level (a contiguous
// range no wider than the one below, by the breadth-first numbering), and the
// first node it owns per stage (the nodes past the previous workgroup's range).
// Per workgroup of a level whose node ranges are rg ([nw][nst], stages
// s_begin..s_end): the children [cb, ce) of its last stage's nodes and the
// parents of its first stage's first and last node (the kernels' SegArgs::wgx).
static int2* upload_wgx(const TreeHost& t, const std::vector<int2>& rg, int nw, int nst,
                        int s_end, hipStream_t st) {
  std::vector<int2> x((size_t)2 * nw);
  for (int w = 0; w < nw; ++w) {
    const int2 f = rg[(size_t)w * nst], l = rg[(size_t)w * nst + nst - 1];
    x[2 * w] = s_end + 1 < t.N ? make_int2(t.cbeg[l.x], t.cend[l.y - 1]) : make_int2(0, 0);
    x[2 * w + 1] = make_int2(t.anc[f.x], t.anc[f.y - 1]);
  }
  return upload(x, st);
}

void build_fwd_full(tapg_solver_s* S, const TreeHost& t, Slot& sl, const LevelPlan& B) {
  hipStream_t st = S->stream;
  int wmax = 0;
  const std::vector<std::pair<int, int>> rp = level_ranges(t, B, wmax);
  if (wmax > kSegNbMax)
    throw Fail{TAPG_EINVAL, "scan forward launch: a workgroup would hold " + std::to_string(wmax) +
                                " nodes of one stage (at most " + std::to_string(kSegNbMax) +
                                "; TAPG_FWD_GROUP must be 0, 1, 2 or 4)"};
  const int N = t.N, nstB = B.s_end - B.s_begin + 1, nw = B.n_wg;
  std::vector<int2> rg((size_t)nw * N);
  std::vector<int> own((size_t)nw * N);
  for (int w = 0; w < nw; ++w) {
    for (int s = B.s_begin; s < N; ++s) {
      const auto& q = rp[(size_t)w * nstB + (s - B.s_begin)];
      rg[(size_t)w * N + s] = make_int2(q.first, q.second);
    }
    for (int s = B.s_begin - 1; s >= 0; --s) {
      const int2 c = rg[(size_t)w * N + s + 1];
      rg[(size_t)w * N + s] = make_int2(t.anc[c.x], t.anc[c.y - 1] + 1);
    }
  }
  for (int s = 0; s < N; ++s)
    for (int w = 0; w < nw; ++w) {
      const int2 r = rg[(size_t)w * N + s];
      own[(size_t)w * N + s] = w == 0 ? r.x : std::max(r.x, rg[(size_t)(w - 1) * N + s].y);
    }
  Slot::Level L{0, N - 1, nw, nb_template(wmax), 0, nullptr, nullptr};
  const size_t lds = S->fp32 ? seg_lds_probe<float>(S, L.nbm, N, 0, true)
                             : seg_lds_probe<double>(S, L.nbm, N, 0, true);
  if (lds + kSegStaticLds > S->lds_limit)
    throw Fail{TAPG_EINVAL, "forward launch needs " + std::to_string(lds) + " bytes of LDS"};
  try {
    L.d_ranges = upload(rg, st);
    L.d_wgx = upload_wgx(t, rg, nw, N, N - 1, st);
    sl.d_own = upload(own, st);
    if (t.ntrees > 1) {
      std::vector<int> wt(nw, 0);
      for (int w = 0; w < nw; ++w) {
        const int n0 = rg[(size_t)w * N].x;  // the root of the workgroup's tree
        int k = 0;
        while (k + 1 < t.ntrees && t.seg_begin(0, k + 1) <= n0) ++k;
        wt[w] = k;
      }
      L.d_wgtree = upload(wt, st);
    }
  } catch (...) {
    (void)hipStreamSynchronize(st);  // no queued upload into a block given back
    dfree(L.d_ranges);
    dfree(L.d_wgx);
    dfree(sl.d_own);
    sl.d_own = nullptr;
    throw;
  }
  sl.fwd_full = L;
}

void free_up(Slot& sl) {
  dfree(sl.d_up_plan);
  dfree(sl.d_up_par);
  dfree(sl.d_up_need);
  dfree(sl.d_up_cnt);
  sl.n_up = 0;
}

// Light upper levels, where they apply (scan form, two levels or more, and
// the upper workgroups' work fits the LDS): per upper level the most nodes
// one workgroup holds, and the tables of the bottom launch that runs them
// (SegArgs::n_main): upper workgroups numbered from the lowest upper level
// up, each with its static table (nodes, children, the upper workgroups above
// it, its tree), the upper workgroups above each bottom workgroup, the
// arrivals that complete each upper workgroup (its child workgroups and its
// local part) and their counters.  Otherwise the slot runs every
// level with the full kernel.
void setup_top_light(tapg_solver_s* S, const TreeHost& t, Slot& sl) {
  free_up(sl);
  const int nl = (int)sl.levels.size();
  // a plan whose upper levels are wider than the full kernels take needs them
  auto wide = [&] {
    for (int l = 0; l + 1 < nl; ++l)
      if (sl.levels[l].nbm > kSegNbMax) return true;
    return false;
  };
  auto refuse = [&](const char* why) {
    sl.top_light = false;
    if (wide())
      throw Fail{TAPG_EINVAL, std::string("schedule: upper levels wider than ") +
                                  std::to_string(kSegNbMax) + " nodes per stage need light "
                                  "upper levels, which do not apply here (" + why + ")"};
  };
  if (!sl.top_light || !sl.scan || nl < 2) {
    refuse("scan form, two levels or more");
    return;
  }
  std::vector<std::vector<std::pair<int, int>>> rp(nl);
  for (int l = 0; l < nl; ++l) {
    int wmax = 0;
    rp[l] = level_ranges(t, sl.plans[l], wmax);
  }
  auto nst_of = [&](int l) { return sl.plans[l].s_end - sl.plans[l].s_begin + 1; };
  // upper workgroups, from the lowest upper level up; the owner of each node
  // at an upper level's last stage
  std::vector<int> wg0(nl, 0), owner(t.K, -1);
  int n_up = 0;
  for (int l = nl - 2; l >= 0; --l) {
    wg0[l] = n_up;
    n_up += sl.levels[l].n_wg;
  }
  for (int l = 0; l + 1 < nl; ++l) {
    const int nst = nst_of(l);
    for (int w = 0; w < sl.levels[l].n_wg; ++w) {
      const auto& q = rp[l][(size_t)w * nst + nst - 1];
      for (int n = q.first; n < q.second; ++n) owner[n] = wg0[l] + w;
    }
  }
  // the upper workgroups above workgroup w of level l >= 1: the owners of
  // the parents of its first stage's nodes (consecutive nodes, consecutive
  // owners, every one a parent)
  auto parents_of = [&](int l, int w) {
    const auto& f = rp[l][(size_t)w * nst_of(l)];
    return make_int2(owner[t.anc[f.first]], owner[t.anc[f.second - 1]]);
  };
  // tables: sizes first
  int nw_max = 1, nch_max = 1, nst_max = 1;
  for (int l = 0; l + 1 < nl; ++l) {
    Slot::Level& L = sl.levels[l];
    const int nst = nst_of(l);
    nst_max = std::max(nst_max, nst);
    int nw = 0;
    for (int w = 0; w < L.n_wg; ++w) {
      int c = 0;
      for (int q = 0; q < nst; ++q)
        c += rp[l][(size_t)w * nst + q].second - rp[l][(size_t)w * nst + q].first;
      nw = std::max(nw, c);
      const auto& lq = rp[l][(size_t)w * nst + nst - 1];
      nch_max = std::max(nch_max, t.cend[lq.second - 1] - t.cbeg[lq.first]);
    }
    L.nw = nw;
    nw_max = std::max(nw_max, nw);
  }
  const int PS = kPlanOff + nst_max + 1 + 3 * nw_max;
  if (PS > kSegThreads) {
    refuse("upper workgroups with too many nodes");
    return;
  }
  const size_t lds =
      S->fp32 ? scan_up_lds<float>(PS, nw_max, nch_max, S->net.nu, S->net.ns, S->nnzB, S->nnzG,
                                   S->nnzE)
              : scan_up_lds<double>(PS, nw_max, nch_max, S->net.nu, S->net.ns, S->nnzB, S->nnzG,
                                    S->nnzE);
  if (lds + kSegStaticLds > S->lds_limit) {
    refuse("LDS");
    return;
  }
  std::vector<int> plan((size_t)n_up * PS, 0);
  std::vector<int> need(n_up, 1);  // 1: its local part
  int widest = 1;
  auto count_arrivals = [&](int2 p) {
    if (p.x < 0 || p.y < p.x || p.y >= n_up)
      throw Fail{TAPG_EINVAL, "light upper levels: inconsistent level ranges"};
    for (int u = p.x; u <= p.y; ++u) need[u]++;
    widest = std::max(widest, p.y - p.x + 1);
  };
  for (int l = 0; l + 1 < nl; ++l) {
    const int nst = nst_of(l);
    for (int w = 0; w < sl.levels[l].n_wg; ++w) {
      int* P = plan.data() + (size_t)(wg0[l] + w) * PS;
      const auto* rg = &rp[l][(size_t)w * nst];
      int nw = 0;
      for (int q = 0; q < nst; ++q) nw += rg[q].second - rg[q].first;
      const int cb = t.cbeg[rg[nst - 1].first];
      P[kPlanNw] = nw;
      P[kPlanNst] = nst;
      P[kPlanCb] = cb;
      P[kPlanNch] = t.cend[rg[nst - 1].second - 1] - cb;
      P[kPlanSb] = sl.plans[l].s_begin;
      const int2 par = l > 0 ? parents_of(l, w) : make_int2(-1, -1);
      if (l > 0) count_arrivals(par);
      P[kPlanPar0] = par.x;
      P[kPlanPar1] = par.y;
      {  // the tree of its first node (level ranges never span two trees)
        const int n0 = rg[0].first;
        int k = 0;
        while (k + 1 < t.ntrees && t.seg_begin(sl.plans[l].s_begin, k + 1) <= n0) ++k;
        P[kPlanTree] = k;
      }
      int* off = P + kPlanOff;
      int* node = off + nst + 1;
      int* clo = node + nw;
      int* chi = clo + nw;
      int k = 0;
      for (int q = 0; q < nst; ++q) {
        off[q] = k;
        for (int n = rg[q].first; n < rg[q].second; ++n, ++k) {
          node[k] = n;
          if (q + 1 < nst) {  // children: this workgroup's nodes of the next stage
            clo[k] = off[q] + (rg[q].second - rg[q].first) + (t.cbeg[n] - rg[q + 1].first);
            chi[k] = clo[k] + (t.cend[n] - t.cbeg[n]);
          } else {  // children below, from cb
            clo[k] = t.cbeg[n] - cb;
            chi[k] = t.cend[n] - cb;
          }
        }
      }
      off[nst] = k;
    }
  }
  const int n_main = sl.levels.back().n_wg;
  std::vector<int2> par(n_main);
  for (int w = 0; w < n_main; ++w) {
    par[w] = parents_of(nl - 1, w);
    count_arrivals(par[w]);
  }
  if (widest * nl > kUpStack) {
    refuse("a workgroup below too many upper workgroups");
    return;
  }
  hipStream_t st = S->stream;
  sl.d_up_plan = upload(plan, st);
  sl.d_up_par = upload(par, st);
  sl.d_up_need = upload(need, st);
  sl.d_up_cnt = upload(std::vector<unsigned>(n_up, 0u), st);
  sl.up_plan_stride = PS;
  sl.up_nw = nw_max;
  sl.up_nch = nch_max;
  sl.n_up = n_up;
}

// (Re)build the level launches of a slot from a plan.
void build_levels(tapg_solver_s* S, const TreeHost& t, Slot& sl, const std::vector<LevelPlan>& plans) {
  hipStream_t st = S->stream;
  const int nbmax = kSegNbMax;
  std::vector<Slot::Level> levels;
  int ptot = 0;
  try {
    for (const LevelPlan& P : plans) {
      int wmax = 0;
      std::vector<std::pair<int, int>> rp = level_ranges(t, P, wmax);
      std::vector<int2> rg(rp.size());
      for (size_t k = 0; k < rp.size(); ++k) rg[k] = make_int2(rp[k].first, rp[k].second);
      // (light upper levels hold any number: their kernel takes a stage's
      // nodes one after another; setup_top_light checks that they apply)
      const bool upper_light = sl.top_light && sl.scan && &P != &plans.back();
      if (wmax > nbmax && !upper_light)
        throw Fail{TAPG_EINVAL, "segment schedule: a workgroup would hold more than " +
                                    std::to_string(nbmax) + " nodes of one stage"};
      const int nst = P.s_end - P.s_begin + 1;
      int nch = 0;
      if (P.s_end + 1 < t.N) {
        for (int w = 0; w < P.n_wg; ++w) {
          const auto& q = rp[(size_t)w * nst + nst - 1];
          nch = std::max(nch, t.cend[q.second - 1] - t.cbeg[q.first]);
        }
      }
      Slot::Level L{P.s_begin, P.s_end, P.n_wg, nb_template(wmax), nch, nullptr, nullptr};
      const size_t lds = S->fp32 ? seg_lds_probe<float>(S, L.nbm, nst, nch, sl.scan)
                                 : seg_lds_probe<double>(S, L.nbm, nst, nch, sl.scan);
      if (lds + kSegStaticLds > S->lds_limit)
        throw Fail{TAPG_EINVAL, "segment schedule needs " + std::to_string(lds) +
                                    " bytes of LDS per workgroup (limit " +
                                    std::to_string(S->lds_limit) + ")"};
      L.d_ranges = upload(rg, st);
      levels.push_back(L);
      levels.back().d_wgx = upload_wgx(t, rg, P.n_wg, nst, P.s_end, st);
      if (t.ntrees > 1) {  // the tree of each workgroup, from its first node
        std::vector<int> wt(P.n_wg, 0);
        for (int w = 0; w < P.n_wg; ++w) {
          const int n0 = rp[(size_t)w * nst].first;
          int k = 0;
          while (k + 1 < t.ntrees && t.seg_begin(P.s_begin, k + 1) <= n0) ++k;
          wt[w] = k;
        }
        levels.back().d_wgtree = upload(wt, st);
      }
      ptot += P.n_wg;
    }
  } catch (...) {
    (void)hipStreamSynchronize(st);  // no queued upload into a block given back
    for (auto& L : levels) {
      dfree(L.d_ranges);
      dfree(L.d_wgtree);
      dfree(L.d_wgx);
    }
    throw;
  }
  for (auto& L : sl.levels) {
    dfree(L.d_ranges);
    dfree(L.d_wgtree);
    dfree(L.d_wgx);
  }
  sl.levels = std::move(levels);
  sl.plans = plans;
  setup_top_light(S, t, sl);
  free_fwd_full(sl);
  if (sl.scan)
    build_fwd_full(S, t, sl, sl.fwd_group > 0 ? stage_plan(t, t.N - 1, sl.fwd_group) : plans.back());
  free_chain(sl);
  sl.part_total = ptot;
  sl.segmented = true;
  if (sl.graph) (void)hipGraphExecDestroy(sl.graph);
  sl.graph = nullptr;
}

Slot& dev_slot(tapg_solver_s* S, const TreeHost& t) {
  TAPG_HIP(hipSetDevice(S->device));
  hipStream_t st = S->stream;
  auto it = S->slots.find(t.uid);
  if (it == S->slots.end()) {
    Slot sl;
    sl.tree_uid = t.uid;
    sl.K = t.K;
    {  // sweep form: the tuned one for this shape, else the solver's default
      auto ts = S->tuned_scan.find(shape_key(t));
      sl.scan = S->scan && (ts == S->tuned_scan.end() ? S->scan_default : ts->second);
      auto tf = S->tuned_fwd.find(shape_key(t));
      const char* fg = std::getenv("TAPG_FWD_GROUP");
      sl.fwd_group = (fg && fg[0]) ? std::atoi(fg) : (tf == S->tuned_fwd.end() ? 0 : tf->second);
      if (sl.fwd_group != 0 && sl.fwd_group != 1 && sl.fwd_group != 2 && sl.fwd_group != 4)
        throw Fail{TAPG_EINVAL, "TAPG_FWD_GROUP must be 0, 1, 2 or 4 (got " +
                                    std::to_string(sl.fwd_group) + ")"};
      auto tt = S->tuned_top.find(shape_key(t));
      const char* te = std::getenv("TAPG_TOP");
      sl.top_light = (te && te[0]) ? te[0] == '1' : (tt != S->tuned_top.end() && tt->second);
    }
    sl.N = t.N;
    sl.elem = S->fp32 ? sizeof(float) : sizeof(double);
    const int K = t.K, LDX = S->LDX, LDU = S->LDU, LDY = S->LDY;
    const size_t e = sl.elem;
    auto dalloc = [&](size_t n) {
      void* p = dev_alloc(std::max<size_t>(n, 1) * e);
      TAPG_HIP(hipMemsetAsync(p, 0, std::max<size_t>(n, 1) * e, st));
      return p;
    };
    try {
      sl.d_anc = upload(t.anc, st);
      sl.d_cbeg = upload(t.cbeg, st);
      sl.d_cend = upload(t.cend, st);
      sl.d_stage = upload(t.stage, st);
      sl.d_prob64 = upload(t.prob, st);
      if (S->fp32) {
        std::vector<float> ip(K);
        for (int n = 0; n < K; ++n) ip[n] = (float)(1.0 / t.prob[n]);
        sl.d_invp = upload(ip, st);
      } else {
        std::vector<double> ip(K);
        for (int n = 0; n < K; ++n) ip[n] = 1.0 / t.prob[n];
        sl.d_invp = upload(ip, st);
      }
      sl.d_demand = dmalloc<double>((size_t)K * t.nd);
      sl.d_price = dmalloc<double>(K);
      sl.d_kappa = dalloc((size_t)K * LDU);
      sl.d_g = dalloc((size_t)K * LDX);
      sl.ntrees = t.ntrees;
      sl.d_pq = dalloc((size_t)t.ntrees * (LDX + LDU));
      sl.d_pq64 = dmalloc<double>((size_t)t.ntrees * (LDX + LDU));
      sl.d_Y0 = dalloc((size_t)K * LDY);
      sl.d_Y1 = dalloc((size_t)K * LDY);
      sl.d_lam = dalloc((size_t)K * LDX);
      sl.d_j = dalloc((size_t)K * LDU);
      if (S->scan) {
        sl.d_kperp = dalloc((size_t)K * LDU);
        sl.d_zb = dalloc((size_t)K * LDU);
        sl.d_zr = dalloc((size_t)t.ntrees * LDU);
      }
      sl.d_u = dalloc((size_t)K * LDU);
      sl.d_x = dalloc((size_t)K * LDX);
      sl.d_ctl = dmalloc<DevCtl>(2 * (size_t)t.ntrees);  // two blocks per tree
      sl.hist_cap = std::max(1, S->cfg.max_iter);
      sl.d_hist = dmalloc<double>((size_t)sl.hist_cap * t.ntrees);
      sl.node_offset = t.offset;
      sl.nb_of_stage.resize(t.N);
      sl.tiles_of_stage.resize(t.N);
      sl.tile_offset.resize(t.N + 1);
      int tot = 0;
      for (int s = 0; s < t.N; ++s) {
        const int width = t.mu[s];
        const int nb = pick_nb(width, e, LDX, LDU, LDY);
        sl.nb_of_stage[s] = nb;
        sl.tiles_of_stage[s] = (width + nb - 1) / nb;
        sl.tile_offset[s] = tot;
        tot += sl.tiles_of_stage[s];
      }
      sl.tile_offset[t.N] = tot;
      sl.total_tiles = tot;
      if (S->seg_ok) build_levels(S, t, sl, choose_plans(S, t));
      sl.part_cap = std::max(tot, 4 * K);
      sl.d_part = dmalloc<double>(sl.part_cap);
    } catch (...) {
      (void)hipStreamSynchronize(st);  // no queued upload into a block given back
      dev_free_slot(sl);
      throw;
    }
    it = S->slots.emplace(t.uid, std::move(sl)).first;
  }
  Slot& sl = it->second;
  if (sl.hist_cap < S->cfg.max_iter) {
    dfree(sl.d_hist);
    sl.hist_cap = S->cfg.max_iter;
    sl.d_hist = dmalloc<double>((size_t)sl.hist_cap * sl.ntrees);
    if (sl.graph) (void)hipGraphExecDestroy(sl.graph);
    sl.graph = nullptr;
  }
  if (sl.data_version != t.version && !t.device_data) {
    TAPG_HIP(hipMemcpyAsync(sl.d_demand, t.demand.data(), t.demand.size() * 8,
                            hipMemcpyHostToDevice, st));
    TAPG_HIP(hipMemcpyAsync(sl.d_price, t.price.data(), t.price.size() * 8,
                            hipMemcpyHostToDevice, st));
    sl.data_version = t.version;
  }
  TAPG_HIP(hipStreamSynchronize(st));
  return sl;
}

void dev_solve(tapg_solver_s* S, const TreeHost& t, Slot& sl, const double* p, const double* q,
               bool warm, double gamma, tapg_result& res) {
  TAPG_HIP(hipSetDevice(S->device));
  if (S->fp32)
    solve_impl<float>(S, t, sl, p, q, warm, gamma, res);
  else
    solve_impl<double>(S, t, sl, p, q, warm, gamma, res);
}

namespace {
// The forest of a batch, cached by the member ids (its data refreshed when a
// member's data changed).  host_data = false (the server's forests): demand
// and price are not copied on the host; the caller gathers them on the device
// from the trees' own slots.
Batch& get_batch(tapg_solver_s* S, const std::vector<const TreeHost*>& trees,
                 bool host_data = true) {
  hipStream_t st = S->stream;
  const int nt = (int)trees.size();
  std::vector<uint64_t> key(nt);
  for (int k = 0; k < nt; ++k) key[k] = trees[k]->uid;
  auto bit = S->batches.find(key);
  if (bit == S->batches.end()) {
    Batch b;
    b.forest = build_forest(trees, b.map, b.map_off, host_data);
    for (const TreeHost* t : trees) b.versions.push_back(t->version);
    try {
      b.d_map = upload(b.map, st);
      b.d_tstart = upload(b.forest.tstart, st);
      b.d_red = dmalloc<double>((size_t)3 * nt);
    } catch (...) {
      (void)hipStreamSynchronize(S->stream);  // no queued upload into a block given back
      dfree(b.d_map); dfree(b.d_tstart); dfree(b.d_red);
      throw;
    }
    bit = S->batches.emplace(key, std::move(b)).first;
  } else {
    bool stale = false;
    for (int k = 0; k < nt; ++k) stale = stale || bit->second.versions[k] != trees[k]->version;
    if (stale && !bit->second.forest.device_data) {
      refresh_forest_data(trees, bit->second.map, bit->second.map_off, bit->second.forest);
      for (int k = 0; k < nt; ++k) bit->second.versions[k] = trees[k]->version;
    }
  }
  return bit->second;
}

// Iteration graph of a forest slot (chunk iterations), captured on demand.
template <typename T>
void ensure_graph(tapg_solver_s* S, Slot& sl, int chunk) {
  if (!S->use_graph || (sl.graph != nullptr && sl.graph_iters == chunk)) return;
  hipStream_t st = S->stream;
  if (sl.graph) (void)hipGraphExecDestroy(sl.graph);
  sl.graph = nullptr;
  hipGraph_t g = nullptr;
  const NetDev<T>& d = net_of<T>(S);
  TAPG_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
  enqueue_iterations<T>(S, sl, d, chunk);
  TAPG_HIP(hipStreamEndCapture(st, &g));
  hipError_t e = hipGraphInstantiate(&sl.graph, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) throw Fail{TAPG_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e)};
  sl.graph_iters = chunk;
}

// Iterations per captured graph of a forest formed by the server: the largest
// divisor of the chunk up to 5.  A forest lives for a few chunks only, so a
// short graph replayed chunk / g times beats instantiating a whole chunk.
int live_graph_iters(int chunk) {
  for (int g = 5; g > 1; --g)
    if (chunk % g == 0) return g;
  return 1;
}

// `iters` iterations (a multiple of the slot's graph length) by replaying its
// graph, or by direct launches when graphs are off.
template <typename T>
void run_replays(tapg_solver_s* S, Slot& sl, int iters) {
  if (S->use_graph) {
    for (int i = 0; i < iters; i += sl.graph_iters) TAPG_HIP(hipGraphLaunch(sl.graph, S->stream));
  } else {
    const NetDev<T>& d = net_of<T>(S);
    enqueue_iterations<T>(S, sl, d, iters);
    TAPG_HIP(hipGetLastError());
  }
}

template <typename T>
void run_chunk(tapg_solver_s* S, Slot& sl, int chunk) {
  if (S->use_graph) {
    TAPG_HIP(hipGraphLaunch(sl.graph, S->stream));
  } else {
    const NetDev<T>& d = net_of<T>(S);
    enqueue_iterations<T>(S, sl, d, chunk);
    TAPG_HIP(hipGetLastError());
  }
}

template <typename T>
void forest_data_step(tapg_solver_s* S, const TreeHost& f, Slot& sl) {
  const NetworkHost& h = S->net;
  data_step<T>(S, sl, f.K, S->stream);
  TAPG_HIP(hipGetLastError());
}

template <typename T>
void batch_impl(tapg_solver_s* S, const std::vector<const TreeHost*>& trees,
                const std::vector<Slot*>& own, const double* const* p, const double* const* q,
                const int* warm, const std::vector<double>& gam, tapg_result* res) {
  const NetworkHost& h = S->net;
  hipStream_t st = S->stream;
  const int LDX = S->LDX, LDU = S->LDU, LDY = S->LDY, PQ = LDX + LDU;
  const int nt = (int)trees.size();
  Batch& B = get_batch(S, trees);
  const TreeHost& f = B.forest;
  Slot& sl = dev_slot(S, f);
  if (!sl.segmented)
    throw Fail{TAPG_EINVAL, "batched solves need the segment kernels (nx, nu <= 128, sparse B)"};
  // (p, q) and control block of every tree
  std::vector<double> pq64((size_t)nt * PQ, 0.0);
  std::vector<DevCtl> c(nt);
  for (int k = 0; k < nt; ++k) {
    for (int i = 0; i < h.nx; ++i) pq64[(size_t)k * PQ + i] = p[k][i];
    for (int i = 0; i < h.nu; ++i) pq64[(size_t)k * PQ + LDX + i] = q[k][i];
    c[k] = DevCtl{};
    c[k].max_iter = S->cfg.max_iter;
    c[k].tol = S->cfg.tol;
    c[k].gamma = gam[k];
    c[k].theta = 1.0;
    c[k].theta_prev = 1.0;
    c[k].rule = S->cfg.beta_rule;
    c[k].beta = 0.0;
  }
  upload_pq<T>(S, sl, pq64, st);
  TAPG_HIP(hipMemcpyAsync(sl.d_ctl, c.data(), c.size() * sizeof(DevCtl), hipMemcpyHostToDevice, st));
  // dual start: zero, then the warm trees' latest duals into both buffers
  const size_t ybytes = (size_t)f.K * LDY * sizeof(T);
  TAPG_HIP(hipMemsetAsync(sl.d_Y0, 0, ybytes, st));
  TAPG_HIP(hipMemsetAsync(sl.d_Y1, 0, ybytes, st));
  for (int k = 0; k < nt; ++k) {
    if (!(warm && warm[k] && own[k]->has_dual)) continue;
    const T* src = static_cast<const T*>(own[k]->last_iter_parity ? own[k]->d_Y1 : own[k]->d_Y0);
    const int* idx = B.d_map + B.map_off[k];
    launch_copy_rows<T>(src, LDY, static_cast<T*>(sl.d_Y0), LDY, idx, trees[k]->K, LDY, true, st);
    launch_copy_rows<T>(src, LDY, static_cast<T*>(sl.d_Y1), LDY, idx, trees[k]->K, LDY, true, st);
  }
  TAPG_HIP(hipGetLastError());
  TAPG_HIP(hipEventRecord(S->ev0, st));
  data_step<T>(S, sl, f.K, st);
  TAPG_HIP(hipGetLastError());
  // iterations in graph chunks until every tree has stopped
  const int chunk = std::max(1, std::min(S->cfg.check_every, S->cfg.max_iter));
  const NetDev<T>& d = net_of<T>(S);
  if (S->use_graph && (sl.graph == nullptr || sl.graph_iters != chunk)) {
    if (sl.graph) (void)hipGraphExecDestroy(sl.graph);
    sl.graph = nullptr;
    hipGraph_t g = nullptr;
    TAPG_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    enqueue_iterations<T>(S, sl, d, chunk);
    TAPG_HIP(hipStreamEndCapture(st, &g));
    hipError_t e = hipGraphInstantiate(&sl.graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) throw Fail{TAPG_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e)};
    sl.graph_iters = chunk;
  }
  int launched = 0;
  ProgressLine progress("batch");
  while (true) {
    if (S->use_graph) {
      TAPG_HIP(hipGraphLaunch(sl.graph, st));
    } else {
      enqueue_iterations<T>(S, sl, d, chunk);
      TAPG_HIP(hipGetLastError());
    }
    launched += chunk;
    TAPG_HIP(hipMemcpyAsync(c.data(), sl.d_ctl, c.size() * sizeof(DevCtl), hipMemcpyDeviceToHost, st));
    TAPG_HIP(hipStreamSynchronize(st));
    bool all = true;
    int running = 0;
    for (int k = 0; k < nt; ++k) {
      all = all && c[k].done;
      running += c[k].done ? 0 : 1;
    }
    progress.tick(launched, running, nt);
    if (all || launched >= S->cfg.max_iter) break;
  }
  TAPG_HIP(hipEventRecord(S->ev1, st));
  // cost and violations of every tree's final primal iterate
  launch_cost<T>(f.K, h.nx, h.nu, h.nd, h.ns, LDX, LDU, (const int*)sl.d_anc,
                 (const double*)sl.d_prob64, (const double*)sl.d_demand,
                 (const double*)sl.d_price, (const T*)sl.d_u, (const T*)sl.d_x,
                 (const double*)sl.d_pq64, (const double*)S->d64.A, (const double*)S->d64.B,
                 (const double*)S->dx.Gd, (const double*)S->dx.E, (const double*)S->dx.Ed,
                 (const double*)S->dx.Wu, (const double*)S->dx.alpha0, (const double*)S->dx.cE,
                 (const double*)S->d64.xmin, (const double*)S->d64.xmax,
                 (const double*)S->d64.xs, (const double*)S->d64.umin,
                 (const double*)S->d64.umax, S->cfg.W_alpha, S->cfg.W_x, S->cfg.W_s, sl.d_part,
                 S->dx.red, st);
  launch_cost_reduce_forest(sl.d_part, B.d_tstart, f.N, nt, B.d_red, st);
  TAPG_HIP(hipGetLastError());
  std::vector<double> red((size_t)3 * nt);
  TAPG_HIP(hipMemcpyAsync(red.data(), B.d_red, red.size() * 8, hipMemcpyDeviceToHost, st));
  // every tree's rows, latest dual and history back into its own slot
  for (int k = 0; k < nt; ++k) {
    Slot& o = *own[k];
    const int* idx = B.d_map + B.map_off[k];
    const int Kk = trees[k]->K;
    launch_copy_rows<T>(static_cast<const T*>(sl.d_u), LDU, static_cast<T*>(o.d_u), LDU, idx, Kk,
                        LDU, false, st);
    launch_copy_rows<T>(static_cast<const T*>(sl.d_x), LDX, static_cast<T*>(o.d_x), LDX, idx, Kk,
                        LDX, false, st);
    const T* ysrc = static_cast<const T*>((c[k].iter & 1) ? sl.d_Y1 : sl.d_Y0);
    launch_copy_rows<T>(ysrc, LDY, static_cast<T*>(o.d_Y0), LDY, idx, Kk, LDY, false, st);
    const int m = std::min(c[k].iter, o.hist_cap);
    if (m > 0)
      TAPG_HIP(hipMemcpyAsync(o.d_hist, sl.d_hist + (size_t)k * sl.hist_cap, (size_t)m * 8,
                              hipMemcpyDeviceToDevice, st));
  }
  TAPG_HIP(hipGetLastError());
  TAPG_HIP(hipStreamSynchronize(st));
  float ms = 0.f;
  TAPG_HIP(hipEventElapsedTime(&ms, S->ev0, S->ev1));
  for (int k = 0; k < nt; ++k) {
    tapg_result r{};
    r.dual_gap = r.dual_obj = NAN;  // evaluated on request (tapg_residuals)
    r.iters = c[k].iter;
    r.converged = c[k].converged;
    r.primal_res = c[k].last_res;
    r.cost = red[3 * k + 0];
    r.viol_box = red[3 * k + 1];
    r.viol_eq = red[3 * k + 2];
    r.gamma = gam[k];
    r.solve_ms = ms;
    res[k] = r;
    Slot& o = *own[k];
    o.has_dual = true;
    o.last_iter_parity = 0;
    o.last = r;
    o.has_result = true;
    o.numeric = c[k].numeric != 0;
    o.last_pq.assign(pq64.begin() + (size_t)k * PQ, pq64.begin() + (size_t)(k + 1) * PQ);
    o.gap_valid = false;
  }
}
}  // namespace

namespace {
std::vector<const TreeHost*> live_trees(const std::vector<LiveTree*>& js) {
  std::vector<const TreeHost*> t(js.size());
  for (size_t k = 0; k < js.size(); ++k) t[k] = js[k]->t;
  return t;
}

std::vector<uint64_t> live_key(const std::vector<LiveTree*>& js) {
  std::vector<uint64_t> key(js.size());
  for (size_t k = 0; k < js.size(); ++k) key[k] = js[k]->t->uid;
  return key;
}

// The forest slot of the live set (must exist).
Slot& live_slot(tapg_solver_s* S, const std::vector<LiveTree*>& js, Batch*& B) {
  auto bit = S->batches.find(live_key(js));
  if (bit == S->batches.end()) throw Fail{TAPG_ESTATE, "no forest for this set of trees"};
  B = &bit->second;
  auto sit = S->slots.find(B->forest.uid);
  if (sit == S->slots.end()) throw Fail{TAPG_ESTATE, "forest slot missing"};
  return sit->second;
}

template <typename T>
void live_init_impl(tapg_solver_s* S, LiveTree& j) {
  Slot& o = *j.own;
  hipStream_t st = S->stream;
  const size_t yb = (size_t)j.t->K * S->LDY * sizeof(T);
  if (j.warm && o.has_dual) {
    void* src = o.last_iter_parity ? o.d_Y1 : o.d_Y0;
    void* dst = o.last_iter_parity ? o.d_Y0 : o.d_Y1;
    TAPG_HIP(hipMemcpyAsync(dst, src, yb, hipMemcpyDeviceToDevice, st));
  } else {
    TAPG_HIP(hipMemsetAsync(o.d_Y0, 0, yb, st));
    TAPG_HIP(hipMemsetAsync(o.d_Y1, 0, yb, st));
  }
  o.last_iter_parity = 0;
  o.last_pq.assign((size_t)S->LDX + S->LDU, 0.0);
  for (int i = 0; i < S->net.nx; ++i) o.last_pq[i] = j.p[i];
  for (int i = 0; i < S->net.nu; ++i) o.last_pq[S->LDX + i] = j.q[i];
  // the tree's data step and (p, q) in its own slot, once per request: every
  // forest it runs in gathers the rows, and its cost is evaluated there
  data_step<T>(S, o, j.t->K, st, true);
  TAPG_HIP(hipMemcpyAsync(o.d_pq64, o.last_pq.data(), o.last_pq.size() * sizeof(double),
                          hipMemcpyHostToDevice, st));
  TAPG_HIP(hipStreamSynchronize(st));
  o.gap_valid = false;
  j.ctl = DevCtl{};
  j.ctl.max_iter = S->cfg.max_iter;
  j.ctl.tol = S->cfg.tol;
  j.ctl.gamma = j.gamma;
  j.ctl.theta = 1.0;
  j.ctl.theta_prev = 1.0;
  j.ctl.rule = S->cfg.beta_rule;
  j.ctl.beta = 0.0;
  j.it0 = 0;
  j.finished = false;
  j.res = tapg_result{};
}

template <typename T>
void live_enter_impl(tapg_solver_s* S, const std::vector<LiveTree*>& js) {
  hipStream_t st = S->stream;
  const int LDX = S->LDX, LDU = S->LDU, LDY = S->LDY, PQ = LDX + LDU;
  const int nt = (int)js.size();
  Batch& B = get_batch(S, live_trees(js), false);
  const TreeHost& f = B.forest;
  Slot& sl = dev_slot(S, f);
  if (!sl.segmented)
    throw Fail{TAPG_EINVAL, "batched solves need the segment kernels (nx, nu <= 128, sparse B)"};
  std::vector<double> pq64((size_t)nt * PQ, 0.0);
  std::vector<DevCtl> c(nt);
  for (int k = 0; k < nt; ++k) {
    std::copy(js[k]->p.begin(), js[k]->p.end(), pq64.begin() + (size_t)k * PQ);
    std::copy(js[k]->q.begin(), js[k]->q.end(), pq64.begin() + (size_t)k * PQ + LDX);
    c[k] = js[k]->ctl;
    js[k]->it0 = c[k].iter;
  }
  upload_pq<T>(S, sl, pq64, st);
  TAPG_HIP(hipMemcpyAsync(sl.d_ctl, c.data(), c.size() * sizeof(DevCtl), hipMemcpyHostToDevice, st));
  // each tree's rows from its own slot, one launch per tree: demand and price,
  // both dual buffers as the tree left them, and its data step (kappa, g,
  // kperp)
  for (int k = 0; k < nt; ++k) {
    const int* idx = B.d_map + B.map_off[k];
    const Slot& o = *js[k]->own;
    const int nd = js[k]->t->nd;
    RowCopies rc;
    rc.add(static_cast<const double*>(o.d_demand), nd, static_cast<double*>(sl.d_demand), nd, nd);
    rc.add(static_cast<const double*>(o.d_price), 1, static_cast<double*>(sl.d_price), 1, 1);
    rc.add(static_cast<const T*>(o.d_Y0), LDY, static_cast<T*>(sl.d_Y0), LDY, LDY);
    rc.add(static_cast<const T*>(o.d_Y1), LDY, static_cast<T*>(sl.d_Y1), LDY, LDY);
    rc.add(static_cast<const T*>(o.d_kappa), LDU, static_cast<T*>(sl.d_kappa), LDU, LDU);
    rc.add(static_cast<const T*>(o.d_g), LDX, static_cast<T*>(sl.d_g), LDX, LDX);
    if (sl.scan)
      rc.add(static_cast<const T*>(o.d_kperp), LDU, static_cast<T*>(sl.d_kperp), LDU, LDU);
    launch_copy_row_sets(rc, idx, js[k]->t->K, true, st);
  }
  TAPG_HIP(hipGetLastError());
  const int chunk = std::max(1, std::min(S->cfg.check_every, S->cfg.max_iter));
  ensure_graph<T>(S, sl, live_graph_iters(chunk));
  TAPG_HIP(hipStreamSynchronize(st));
}

template <typename T>
bool live_chunk_impl(tapg_solver_s* S, const std::vector<LiveTree*>& js) {
  Batch* B = nullptr;
  Slot& sl = live_slot(S, js, B);
  hipStream_t st = S->stream;
  const int chunk = std::max(1, std::min(S->cfg.check_every, S->cfg.max_iter));
  TAPG_HIP(hipEventRecord(S->ev0, st));
  run_replays<T>(S, sl, chunk);
  TAPG_HIP(hipEventRecord(S->ev1, st));
  std::vector<DevCtl> c(js.size());
  TAPG_HIP(hipMemcpyAsync(c.data(), sl.d_ctl, c.size() * sizeof(DevCtl), hipMemcpyDeviceToHost, st));
  TAPG_HIP(hipStreamSynchronize(st));
  float ms = 0.f;
  TAPG_HIP(hipEventElapsedTime(&ms, S->ev0, S->ev1));
  bool any = false;
  for (size_t k = 0; k < js.size(); ++k) {
    const bool was_done = js[k]->ctl.done;
    js[k]->ctl = c[k];
    if (!was_done) js[k]->res.solve_ms += ms;  // GPU time of the chunks the tree ran in
    any = any || (c[k].done && !was_done);
  }
  return any;
}

template <typename T>
void live_leave_impl(tapg_solver_s* S, const std::vector<LiveTree*>& js) {
  Batch* B = nullptr;
  Slot& sl = live_slot(S, js, B);
  hipStream_t st = S->stream;
  const int LDX = S->LDX, LDU = S->LDU, LDY = S->LDY;
  const int nt = (int)js.size();
  const NetworkHost& h = S->net;
  bool any_done = false;
  for (LiveTree* j : js) any_done = any_done || j->ctl.done;
  std::vector<double> red((size_t)3 * nt, 0.0);
  for (int k = 0; k < nt; ++k) {
    LiveTree& j = *js[k];
    Slot& o = *j.own;
    const int* idx = B->d_map + B->map_off[k];
    const int Kk = j.t->K;
    {  // both dual buffers and, for a stopped tree, its primal: one launch
      RowCopies rc;
      rc.add(static_cast<const T*>(sl.d_Y0), LDY, static_cast<T*>(o.d_Y0), LDY, LDY);
      rc.add(static_cast<const T*>(sl.d_Y1), LDY, static_cast<T*>(o.d_Y1), LDY, LDY);
      if (j.ctl.done) {
        rc.add(static_cast<const T*>(sl.d_u), LDU, static_cast<T*>(o.d_u), LDU, LDU);
        rc.add(static_cast<const T*>(sl.d_x), LDX, static_cast<T*>(o.d_x), LDX, LDX);
      }
      launch_copy_row_sets(rc, idx, Kk, false, st);
    }
    const int a = std::min(j.it0, o.hist_cap), b = std::min(j.ctl.iter, o.hist_cap);
    if (b > a)
      TAPG_HIP(hipMemcpyAsync(o.d_hist + a, sl.d_hist + (size_t)k * sl.hist_cap + a,
                              (size_t)(b - a) * 8, hipMemcpyDeviceToDevice, st));
    o.last_iter_parity = j.ctl.iter & 1;
    if (j.ctl.done) {  // its cost and violations in its own slot (into B.d_red)
      launch_cost<T>(Kk, h.nx, h.nu, h.nd, h.ns, LDX, LDU, (const int*)o.d_anc,
                     (const double*)o.d_prob64, (const double*)o.d_demand,
                     (const double*)o.d_price, (const T*)o.d_u, (const T*)o.d_x,
                     (const double*)o.d_pq64, (const double*)S->d64.A, (const double*)S->d64.B,
                     (const double*)S->dx.Gd, (const double*)S->dx.E, (const double*)S->dx.Ed,
                     (const double*)S->dx.Wu, (const double*)S->dx.alpha0,
                     (const double*)S->dx.cE, (const double*)S->d64.xmin,
                     (const double*)S->d64.xmax, (const double*)S->d64.xs,
                     (const double*)S->d64.umin, (const double*)S->d64.umax, S->cfg.W_alpha,
                     S->cfg.W_x, S->cfg.W_s, o.d_part, B->d_red + (size_t)3 * k, st);
    }
  }
  TAPG_HIP(hipGetLastError());
  if (any_done)
    TAPG_HIP(hipMemcpyAsync(red.data(), B->d_red, red.size() * 8, hipMemcpyDeviceToHost, st));
  TAPG_HIP(hipStreamSynchronize(st));
  for (int k = 0; k < nt; ++k) {
    LiveTree& j = *js[k];
    if (!j.ctl.done) continue;
    Slot& o = *j.own;
    j.res.iters = j.ctl.iter;
    j.res.converged = j.ctl.converged;
    j.res.primal_res = j.ctl.last_res;
    j.res.cost = red[3 * k + 0];
    j.res.viol_box = red[3 * k + 1];
    j.res.viol_eq = red[3 * k + 2];
    j.res.gamma = j.gamma;
    j.res.dual_gap = j.res.dual_obj = NAN;  // evaluated on request (tapg_residuals)
    o.has_dual = true;
    o.last = j.res;
    o.has_result = true;
    o.numeric = j.ctl.numeric != 0;
    j.finished = true;
  }
  dev_drop_batch(S, live_key(js));
}
}  // namespace

void dev_live_init(tapg_solver_s* S, LiveTree& j) {
  TAPG_HIP(hipSetDevice(S->device));
  if (S->fp32) live_init_impl<float>(S, j); else live_init_impl<double>(S, j);
}

void dev_live_enter(tapg_solver_s* S, const std::vector<LiveTree*>& js) {
  TAPG_HIP(hipSetDevice(S->device));
  if (S->fp32) live_enter_impl<float>(S, js); else live_enter_impl<double>(S, js);
}

bool dev_live_chunk(tapg_solver_s* S, const std::vector<LiveTree*>& js) {
  TAPG_HIP(hipSetDevice(S->device));
  return S->fp32 ? live_chunk_impl<float>(S, js) : live_chunk_impl<double>(S, js);
}

void dev_live_leave(tapg_solver_s* S, const std::vector<LiveTree*>& js) {
  TAPG_HIP(hipSetDevice(S->device));
  if (S->fp32) live_leave_impl<float>(S, js); else live_leave_impl<double>(S, js);
}

namespace {
// Device time of one APG iteration of a slot under its current levels: an
// iteration graph of `iters` iterations, launched once to warm up and twice
// timed (the faster run counts).  The state is synthetic (zero duals, a tiny step size, no stop), so
// the iterates stay finite whatever the tree.
template <typename T>
double time_levels(tapg_solver_s* S, const TreeHost& t, Slot& sl, int iters) {
  hipStream_t st = S->stream;
  const int nt = t.ntrees, PQ = S->LDX + S->LDU;
  if (sl.hist_cap < iters) {  // the timing runs record iters residuals per tree
    TAPG_HIP(hipStreamSynchronize(st));
    dfree(sl.d_hist);
    sl.hist_cap = iters;
    sl.d_hist = dmalloc<double>((size_t)sl.hist_cap * sl.ntrees);
    if (sl.graph) (void)hipGraphExecDestroy(sl.graph);
    sl.graph = nullptr;
  }
  std::vector<DevCtl> c(nt);
  for (int k = 0; k < nt; ++k) {
    c[k] = DevCtl{};
    c[k].max_iter = 1 << 30;
    c[k].tol = 0.0;
    c[k].gamma = 1e-9;
    c[k].theta = c[k].theta_prev = 1.0;
    c[k].rule = S->cfg.beta_rule;
  }
  std::vector<double> pq64((size_t)nt * PQ, 0.0);
  upload_pq<T>(S, sl, pq64, st);
  const size_t yb = (size_t)t.K * S->LDY * sizeof(T);
  TAPG_HIP(hipMemsetAsync(sl.d_Y0, 0, yb, st));
  TAPG_HIP(hipMemsetAsync(sl.d_Y1, 0, yb, st));
  forest_data_step<T>(S, t, sl);
  const NetDev<T>& d = net_of<T>(S);
  auto run = [&](bool timed) {
    TAPG_HIP(hipMemcpyAsync(sl.d_ctl, c.data(), c.size() * sizeof(DevCtl), hipMemcpyHostToDevice, st));
    hipGraph_t g = nullptr;
    hipGraphExec_t ge = nullptr;
    TAPG_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    enqueue_iterations<T>(S, sl, d, iters);
    TAPG_HIP(hipStreamEndCapture(st, &g));
    hipError_t e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) throw Fail{TAPG_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e)};
    if (timed) TAPG_HIP(hipEventRecord(S->ev0, st));
    e = hipGraphLaunch(ge, st);
    if (timed && e == hipSuccess) e = hipEventRecord(S->ev1, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipGraphExecDestroy(ge);
    if (e != hipSuccess) throw Fail{TAPG_EDEVICE, std::string("autotune run: ") + hipGetErrorString(e)};
    float ms = 0.f;
    if (timed) TAPG_HIP(hipEventElapsedTime(&ms, S->ev0, S->ev1));
    return (double)ms;
  };
  run(false);
  // the faster of two timed runs: one run's noise can reorder close candidates
  const double t1 = run(true), t2 = run(true);
  return std::min(t1, t2) / iters;
}

template <typename T>
double autotune_impl(tapg_solver_s* S, const TreeHost& t, Slot& sl, int iters, int* ncand) {
  std::vector<std::vector<LevelPlan>> cands = candidate_plans(t, kSegNbMax, seg_node_us(S));
  const char* te = std::getenv("TAPG_TOP");
  const bool top_forced = te && te[0];
  const bool top_env = top_forced && te[0] == '1';
  sl.top_light = top_env;
  // both sweep forms where the scan form applies: the scan form has fewer
  // launches and shorter chains, the segment form fits more workgroups per
  // compute unit in FP64; which wins depends on the shape
  std::vector<bool> forms = S->scan ? std::vector<bool>{true, false} : std::vector<bool>{false};
  if (ncand) *ncand = (int)(cands.size() * (S->scan ? 5 : 1));
  // the scan form's forward launch: the bottom level's workgroups, or groups
  // of 1, 2 or 4 last-stage nodes (more workgroups, each walking its
  // ancestors); each grouping with every plan, since the best plan differs
  // between groupings and a grouping can reverse the choice of form
  const int fg0 = sl.fwd_group;
  double best = 1e300;
  size_t bi = 0;
  bool bscan = false;
  int bfg = fg0;
  for (bool form : forms) {
    sl.scan = form;
    const std::vector<int> groups = form ? std::vector<int>{0, 1, 2, 4} : std::vector<int>{fg0};
    for (int fg : groups) {
      sl.fwd_group = fg;
      for (size_t i = 0; i < cands.size(); ++i) {
        build_levels(S, t, sl, cands[i]);
        const double ms = time_levels<T>(S, t, sl, iters);
        if (ms < best) {
          best = ms;
          bi = i;
          bscan = form;
          bfg = form ? fg : fg0;
        }
      }
    }
  }
  sl.scan = bscan;
  sl.fwd_group = bfg;
  // light upper levels (scan form): they change what the levels above the
  // bottom one cost, so every plan is timed again with them
  bool btop = top_env;
  if (bscan && !top_forced) {
    for (size_t i = 0; i < cands.size(); ++i) {
      sl.top_light = true;
      build_levels(S, t, sl, cands[i]);
      if (!sl.top_light) continue;  // does not apply to this plan
      const double ms = time_levels<T>(S, t, sl, iters);
      if (ncand) ++*ncand;
      if (ms < best) {
        best = ms;
        bi = i;
        btop = true;
      }
    }
  }
  sl.top_light = btop;
  build_levels(S, t, sl, cands[bi]);
  S->tuned[shape_key(t)] = cands[bi];
  S->tuned_scan[shape_key(t)] = bscan;
  S->tuned_fwd[shape_key(t)] = bfg;
  if (!top_forced) S->tuned_top[shape_key(t)] = sl.top_light;
  sl.has_dual = false;  // the timing runs overwrote the iterates
  sl.has_result = false;
  return best;
}
}  // namespace

double dev_autotune(tapg_solver_s* S, const std::vector<const TreeHost*>& trees, int iters,
                    int* ncand) {
  TAPG_HIP(hipSetDevice(S->device));
  if (!S->seg_ok) throw Fail{TAPG_EINVAL, "the autotuner chooses segment schedules (nx, nu <= 128)"};
  const TreeHost* t = trees[0];
  if (trees.size() > 1) t = &get_batch(S, trees).forest;
  Slot& sl = dev_slot(S, *t);
  return S->fp32 ? autotune_impl<float>(S, *t, sl, iters, ncand)
                 : autotune_impl<double>(S, *t, sl, iters, ncand);
}

void dev_drop_batch(tapg_solver_s* S, const std::vector<uint64_t>& key) {
  auto it = S->batches.find(key);
  if (it == S->batches.end()) return;
  TAPG_HIP(hipSetDevice(S->device));
  TAPG_HIP(hipStreamSynchronize(S->stream));
  dev_drop_tree(S, it->second.forest.uid);
  dfree(it->second.d_map);
  dfree(it->second.d_tstart);
  dfree(it->second.d_red);
  S->batches.erase(it);
}

void dev_drop_tree(tapg_solver_s* S, uint64_t uid) {
  auto it = S->slots.find(uid);
  if (it == S->slots.end()) return;
  TAPG_HIP(hipSetDevice(S->device));
  TAPG_HIP(hipStreamSynchronize(S->stream));
  dev_free_slot(it->second);
  S->slots.erase(it);
}

void dev_batch_solve(tapg_solver_s* S, const std::vector<const TreeHost*>& trees,
                     const std::vector<Slot*>& own, const double* const* p,
                     const double* const* q, const int* warm, const std::vector<double>& gamma,
                     tapg_result* res) {
  TAPG_HIP(hipSetDevice(S->device));
  if (S->fp32)
    batch_impl<float>(S, trees, own, p, q, warm, gamma, res);
  else
    batch_impl<double>(S, trees, own, p, q, warm, gamma, res);
}

double dev_power(tapg_solver_s* S, const TreeHost& t, Slot& sl, int iters) {
  TAPG_HIP(hipSetDevice(S->device));
  return S->fp32 ? power_impl<float>(S, t, sl, iters) : power_impl<double>(S, t, sl, iters);
}

namespace {
template <typename T>
void download_rows(const void* dsrc, int rows, int ld, int cols, double* out, hipStream_t st) {
  std::vector<T> tmp((size_t)rows * ld);
  TAPG_HIP(hipMemcpyAsync(tmp.data(), dsrc, tmp.size() * sizeof(T), hipMemcpyDeviceToHost, st));
  TAPG_HIP(hipStreamSynchronize(st));
  for (int i = 0; i < rows; ++i)
    for (int j = 0; j < cols; ++j) out[(size_t)i * cols + j] = (double)tmp[(size_t)i * ld + j];
}

template <typename T>
void get_dual_impl(tapg_solver_s* S, Slot& sl, double* y) {
  const int nx = S->net.nx, nu = S->net.nu, LDX = S->LDX, LDY = S->LDY;
  const int m = 2 * nx + nu;
  std::vector<T> tmp((size_t)sl.K * LDY);
  const void* src = sl.last_iter_parity ? sl.d_Y1 : sl.d_Y0;
  TAPG_HIP(hipMemcpyAsync(tmp.data(), src, tmp.size() * sizeof(T), hipMemcpyDeviceToHost, S->stream));
  TAPG_HIP(hipStreamSynchronize(S->stream));
  for (int n = 0; n < sl.K; ++n) {
    const T* yn = tmp.data() + (size_t)n * LDY;
    double* o = y + (size_t)n * m;
    for (int i = 0; i < nx; ++i) o[i] = yn[i];
    for (int i = 0; i < nx; ++i) o[nx + i] = yn[LDX + i];
    for (int i = 0; i < nu; ++i) o[2 * nx + i] = yn[2 * LDX + i];
  }
}

template <typename T>
void set_dual_impl(tapg_solver_s* S, Slot& sl, const double* y) {
  const int nx = S->net.nx, nu = S->net.nu, LDX = S->LDX, LDY = S->LDY;
  const int m = 2 * nx + nu;
  std::vector<T> tmp((size_t)sl.K * LDY, T(0));
  for (int n = 0; n < sl.K; ++n) {
    T* yn = tmp.data() + (size_t)n * LDY;
    const double* s = y + (size_t)n * m;
    for (int i = 0; i < nx; ++i) yn[i] = (T)s[i];
    for (int i = 0; i < nx; ++i) yn[LDX + i] = (T)s[nx + i];
    for (int i = 0; i < nu; ++i) yn[2 * LDX + i] = (T)s[2 * nx + i];
  }
  TAPG_HIP(hipMemcpyAsync(sl.d_Y0, tmp.data(), tmp.size() * sizeof(T), hipMemcpyHostToDevice, S->stream));
  TAPG_HIP(hipStreamSynchronize(S->stream));
  sl.has_dual = true;
  sl.last_iter_parity = 0;
  sl.gap_valid = false;
}
}  // namespace

void dev_get_primal(tapg_solver_s* S, Slot& sl, double* u, double* x) {
  TAPG_HIP(hipSetDevice(S->device));
  if (S->fp32) {
    if (u) download_rows<float>(sl.d_u, sl.K, S->LDU, S->net.nu, u, S->stream);
    if (x) download_rows<float>(sl.d_x, sl.K, S->LDX, S->net.nx, x, S->stream);
  } else {
    if (u) download_rows<double>(sl.d_u, sl.K, S->LDU, S->net.nu, u, S->stream);
    if (x) download_rows<double>(sl.d_x, sl.K, S->LDX, S->net.nx, x, S->stream);
  }
}

void dev_get_root_input(tapg_solver_s* S, Slot& sl, double* u0) {
  TAPG_HIP(hipSetDevice(S->device));
  if (S->fp32)
    download_rows<float>(sl.d_u, 1, S->LDU, S->net.nu, u0, S->stream);
  else
    download_rows<double>(sl.d_u, 1, S->LDU, S->net.nu, u0, S->stream);
}

void dev_get_dual(tapg_solver_s* S, Slot& sl, double* y) {
  TAPG_HIP(hipSetDevice(S->device));
  if (S->fp32) get_dual_impl<float>(S, sl, y); else get_dual_impl<double>(S, sl, y);
}

void dev_set_dual(tapg_solver_s* S, Slot& sl, const double* y) {
  TAPG_HIP(hipSetDevice(S->device));
  if (S->fp32) set_dual_impl<float>(S, sl, y); else set_dual_impl<double>(S, sl, y);
}

void dev_set_kernel_timing(tapg_solver_s* S, bool on) { S->time_kernels = on; }

// Median time that an event pair reads around a launch of known length (a
// 10 us hold) queued behind a hold, as the kernel-timing path queues its
// launches, less those 10 us: the dispatch cost that every timed launch
// carries on top of its kernel.
double dev_event_pair_us(tapg_solver_s* S) {
  TAPG_HIP(hipSetDevice(S->device));
  hipStream_t st = S->stream;
  constexpr int n = 64;
  while (S->tev.size() < 2 * n) {
    hipEvent_t e;
    TAPG_HIP(hipEventCreate(&e));
    S->tev.push_back(e);
  }
  launch_hold((long long)(2000.0 * S->wall_clock_mhz), st);
  for (int i = 0; i < n; ++i) {
    TAPG_HIP(hipEventRecord(S->tev[2 * i], st));
    launch_hold((long long)(10.0 * S->wall_clock_mhz), st);
    TAPG_HIP(hipEventRecord(S->tev[2 * i + 1], st));
  }
  TAPG_HIP(hipGetLastError());
  TAPG_HIP(hipStreamSynchronize(st));
  std::vector<double> us(n);
  for (int i = 0; i < n; ++i) {
    float ms = 0.f;
    TAPG_HIP(hipEventElapsedTime(&ms, S->tev[2 * i], S->tev[2 * i + 1]));
    us[i] = 1e3 * ms - 10.0;
  }
  std::nth_element(us.begin(), us.begin() + n / 2, us.end());
  return us[n / 2];
}

int dev_get_history(tapg_solver_s* S, Slot& sl, double* hbuf, int n) {
  TAPG_HIP(hipSetDevice(S->device));
  const int m = std::min(n, sl.has_result ? sl.last.iters : 0);
  if (m > 0) {
    TAPG_HIP(hipMemcpyAsync(hbuf, sl.d_hist, (size_t)m * 8, hipMemcpyDeviceToHost, S->stream));
    TAPG_HIP(hipStreamSynchronize(S->stream));
  }
  return m;
}

}  // namespace tapg
