// Scan-form sweep kernels for gfx950: the dual-gradient sweeps (Sec. 4.4) of a
// network with A = I and W_u = w I, whose stage factors are Fbar_s = Pi / w and
// Kbar_s = Pi with Pi = I - E'(E E')^{-1} E, the orthogonal projector onto the
// null space of E (Pi Pi = Pi).
//
// With these factors the stage-by-stage recursions unroll into sums over
// subtrees (backward) and along root paths (forward).  Writing P_n = Pi j_n
// and z_n = Pi u_n:
//   lambda_n = a_n + sum_c lambda_c                  a_n = w1_n + w2_n
//   m_n      = Pi (kappa_n - (w3_n + B' lambda_n) / (2 w))
//   P_n      = m_n + sum_c P_c
//   j_n      = kperp_n + P_n                         kperp_n = kappa_n - Pi kappa_n
//   u_n      = z_anc + j_n / p_n,   z_n = z_anc + P_n / p_n
//   x_n      = x_anc + B u_n + g_n
// (P_n = Pi j_n follows from j_n = kappa_n + Pi v_n / w and Pi Pi = Pi; then
// j_n = kappa_n - Pi kappa_n + P_n, and z_n = Pi u_anc + Pi j_n / p_n.)
// Only vector additions remain on the chain from stage to stage; the products
// with Pi, B and B' are per node.  A workgroup therefore takes its stages in
// chunks of 8 node-stages (8 / NB stages of NB nodes): each per-node product
// runs over the whole chunk at once, spread over all 512 threads, and each
// chain is walked by one thread per vector component, with the values of the
// neighbouring stage in registers.  A chunk costs five barriers (backward) or
// four (forward) however many stages it holds.  Eight is the fewest the
// thread mapping allows (one x-element per thread); it keeps the next chunk's
// prefetched inputs small enough for FP32 kernels to fit two workgroups per
// compute unit, and shortens the wait on each chunk's loads in FP64 as well.
//
// The workgroups, levels and node ranges are those of the segment kernels, so
// the schedule and the forest layout are shared (the forward launch may also
// take groups of last-stage nodes, each workgroup walking their ancestors).
// The iteration ends in a small launch of its own.  Global
// loads of the next chunk are issued while the current one computes, and a
// chunk's stores are issued at the start of the next, after its one wait.
#include "seg_device.h"

namespace tapg {

namespace {

constexpr int kCN = 8;    // node-stages per chunk
constexpr int kSU = 128;  // padded u-dimension of the segment layout
constexpr int kSX = 64;   // x rows in LDS (nx <= 64 on this path)
constexpr int kQU = kCN * kSU / kSegThreads;  // u-elements per thread and chunk
constexpr int kQX = kCN * kSX / kSegThreads;  // x-elements per thread and chunk
static_assert(kQU * kSegThreads == kCN * kSU && kQX * kSegThreads == kCN * kSX, "chunk shape");

// v[k] for a runtime k < NB, without dynamic register indexing.
template <typename T, int NB>
__device__ __forceinline__ T pick(const T (&v)[NB], int k) {
  T r = v[0];
#pragma unroll
  for (int q = 1; q < NB; ++q) r = k == q ? v[q] : r;
  return r;
}

// sum of v[q] over q in [c0, c1), in increasing q.
template <typename T, int NB>
__device__ __forceinline__ T range_sum(const T (&v)[NB], int c0, int c1) {
  T r = T(0);
#pragma unroll
  for (int q = 0; q < NB; ++q)
    if (q >= c0 && q < c1) r += v[q];
  return r;
}

// Nodes of the element groups of a chunk of stages [s_lo, s_hi]: group j
// covers node-stage kb_j = (tid + 512 j) / W (slot kb % NB of stage s_lo +
// kb / NB); its node, or -1 past the chunk or past the stage's node range.
// kb_j is the same in all lanes of a wave (W = 64 or 128 lanes per
// node-stage), so the results are made wave-uniform: the tests on them compile
// to scalar branches.  All LDS reads are issued before the first is used (one
// wait); with `own` (first node the workgroup writes, per stage) also the
// owned node or -1.
template <int NB, int W, int Q>
__device__ __forceinline__ void chunk_nodes(const int2* sRg, const int* sOwn, int sb, int s_lo,
                                            int s_hi, int (&node)[Q], int (*owned)[Q]) {
  int2 rr[Q];
  int fo[Q];
#pragma unroll
  for (int j = 0; j < Q; ++j) {
    const int kb = (int)(threadIdx.x + j * kSegThreads) / W;
    const int sc = min(s_lo + kb / NB, max(s_hi, sb)) - sb;  // in range for empty chunks too
    rr[j] = sRg[sc];
    if (owned) fo[j] = sOwn[sc];
  }
#pragma unroll
  for (int j = 0; j < Q; ++j) {
    const int kb = (int)(threadIdx.x + j * kSegThreads) / W;
    const int n = rr[j].x + kb % NB;
    const int v = s_lo + kb / NB <= s_hi && n < rr[j].y ? n : -1;
    node[j] = __builtin_amdgcn_readfirstlane(v);
    if (owned) (*owned)[j] = __builtin_amdgcn_readfirstlane(v >= fo[j] ? v : -1);
  }
}

// Layout of a scan launch's dynamic LDS: consecutive arrays, each starting
// on an 8-byte boundary.  Pointers are formed as offsets from the dynamic LDS
// base itself, so the compiler keeps them in the LDS address space (a pointer
// rebuilt from an integer would be a generic one, read with FLAT instructions
// that also wait for every global load in flight).
struct LdsCursor {
  size_t off = 0;
  __host__ __device__ size_t take(size_t bytes) {
    const size_t o = off;
    off = (off + bytes + 7) & ~(size_t)7;
    return o;
  }
};

// The CSR of B', G and E' open a backward launch's dynamic LDS, at the same
// offsets for every role of the launch (bottom level, local parts, upper
// levels), so that a workgroup going on to an upper level keeps them.
template <typename T>
struct CsrLds {
  size_t brow, bcol, bval, grow, gcol, gval, erow, ecol, eval;
  __host__ __device__ void take(LdsCursor& c, int nu, int ns, int nnzB, int nnzG, int nnzE) {
    brow = c.take(sizeof(int) * (nu + 1));
    bcol = c.take(sizeof(int) * nnzB);
    bval = c.take(sizeof(T) * nnzB);
    grow = c.take(sizeof(int) * (ns + 1));
    gcol = c.take(sizeof(int) * nnzG);
    gval = c.take(sizeof(T) * nnzG);
    erow = c.take(sizeof(int) * (nu + 1));
    ecol = c.take(sizeof(int) * nnzE);
    eval = c.take(sizeof(T) * nnzE);
  }
};

template <typename T>
struct BwdLds : CsrLds<T> {  // CSR of B', G and E'; a (then lambda), v (then m), G v;
                             // ranges; packed children slots (two buffers); per-slot
                             // sums of the boundary children (P then lambda, up to 4 slots)
  size_t lam, v, gv, rg, ch, bnd, total;
  __host__ __device__ explicit BwdLds(const SegArgs<T>& a) {
    LdsCursor c;
    this->take(c, a.nu, a.ns, a.nnzB, a.nnzG, a.nnzE);
    lam = c.take(sizeof(T) * kCN * kSX);
    v = c.take(sizeof(T) * kCN * kSU);
    bnd = c.take(sizeof(T) * 4 * (kSU + kSX));
    gv = c.take(sizeof(T) * kCN * a.ns);
    rg = c.take(sizeof(int2) * a.nst);
    ch = c.take(sizeof(int) * 2 * kCN);
    total = c.off;
  }
};

template <typename T>
struct FwdLds {  // c (then u), d, B u + g (then x); ranges; first owned node per
                 // stage; parent slots; CSR of B
  size_t c, d, x, rg, own, par, brow, bcol, bval, total;
  __host__ __device__ explicit FwdLds(const SegArgs<T>& a) {
    LdsCursor k;
    c = k.take(sizeof(T) * kCN * kSU);
    d = k.take(sizeof(T) * kCN * kSU);
    x = k.take(sizeof(T) * kCN * kSX);
    rg = k.take(sizeof(int2) * a.nst);
    own = k.take(sizeof(int) * a.nst);
    par = k.take(sizeof(int) * kCN);
    brow = k.take(sizeof(int) * (a.nx + 1));
    bcol = k.take(sizeof(int) * a.nnzB);
    bval = k.take(sizeof(T) * a.nnzB);
    total = k.off;
  }
};

template <typename T>
size_t scan_lds_bytes(const SegArgs<T>& a, bool fwd) {
  const size_t b = fwd ? FwdLds<T>(a).total : BwdLds<T>(a).total;
  return (b + 15) & ~(size_t)15;
}

// One sparse row held in registers, padded to K entries with (column 0,
// value 0) so that apply() is branch-free: its K reads of X are independent
// and issue together.  Entries past K (none for the rows of a flow network's
// incidence and projector at the sizes used) are read from the LDS copy of the
// CSR.  The products are added in CSR order; a padding term adds exactly 0.
template <typename T, int K>
struct FixRow {
  int col[K];
  T val[K];
  int xb, xe;  // LDS range of the entries past K
  __device__ __forceinline__ void load(const int* srow, const int* scol, const T* sval, int i,
                                       bool ok) {
    const int p0 = ok ? srow[i] : 0, p1 = ok ? srow[i + 1] : 0;
    const int n = min(p1 - p0, K);
#pragma unroll
    for (int k = 0; k < K; ++k) {
      col[k] = k < n ? scol[p0 + k] : 0;
      val[k] = k < n ? sval[p0 + k] : T(0);
    }
    xb = p0 + n;
    xe = p1;
  }
  __device__ __forceinline__ T apply(T acc, const T* X, const int* scol, const T* sval) const {
#pragma unroll
    for (int k = 0; k < K; ++k) acc += val[k] * X[col[k]];
    for (int p = xb; p < xe; ++p) acc += sval[p] * X[scol[p]];
    return acc;
  }
};

// Values handed from one workgroup to another inside a launch (light upper
// levels): agent-scope atomic stores and loads, coherent across the compute
// dies' L2 caches without writing back or invalidating whole caches.
template <typename T>
__device__ __forceinline__ void st_agent(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ T ld_agent(const T* p) {
  return __hip_atomic_load(const_cast<T*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Children slot range (c0, c1) of a node-stage packed into one int.
__device__ __forceinline__ int pack_ch(int c0, int c1) { return c0 | (c1 << 16); }
__device__ __forceinline__ int ch_lo(int v) { return v & 0xFFFF; }
__device__ __forceinline__ int ch_hi(int v) { return v >> 16; }

// ---------------------------------------------------------------------------
// Backward sweep of workgroup `wg` over its level, stages s_end down to
// s_begin, in iteration `it` (extrapolation weight beta; scale: 1/|v| in the
// power iteration, where the data terms are zero).  Writes P_n for every node
// and lambda_n at the level's first stage (read by the level above).
// ---------------------------------------------------------------------------
template <typename T, int NB>
__device__ __forceinline__ void scan_bwd_body(const SegArgs<T>& a, int wg, int it, T beta,
                                              T scale) {
  constexpr int CS = kCN / NB;  // stages per chunk
  const int tid = threadIdx.x;
  const bool power = a.mode == 1;
  const T* Yc = (it & 1) ? a.Y1 : a.Y0;
  const T* Yo = (it & 1) ? a.Y0 : a.Y1;
  const int nx = a.nx, nu = a.nu, LDX = a.LDX, LDY = a.LDY, ns = a.ns;
  const int sb = a.s_begin, se = a.s_end;
  const T hw = T(0.5) * a.winv;  // 1 / (2 w)

  extern __shared__ __align__(16) unsigned char smem_raw[];
  const BwdLds<T> L(a);
  T* sLam = reinterpret_cast<T*>(smem_raw + L.lam);  // [kCN][kSX]: a, then lambda
  T* sV = reinterpret_cast<T*>(smem_raw + L.v);      // [kCN][kSU]: v, then m
  T* sGv = reinterpret_cast<T*>(smem_raw + L.gv);    // [kCN][ns]: G v
  int2* sRg = reinterpret_cast<int2*>(smem_raw + L.rg);  // node range per stage
  int* sCh = reinterpret_cast<int*>(smem_raw + L.ch);    // [2][kCN]: children slots, by chunk parity
  T* sBnd = reinterpret_cast<T*>(smem_raw + L.bnd);      // [NB][kSU] P, then [NB][kSX] lambda
  int* sRow = reinterpret_cast<int*>(smem_raw + L.brow);  // CSR of B' (nu rows)
  int* sCol = reinterpret_cast<int*>(smem_raw + L.bcol);
  T* sVal = reinterpret_cast<T*>(smem_raw + L.bval);
  int* gRow = reinterpret_cast<int*>(smem_raw + L.grow);  // CSR of G (ns rows)
  int* gCol = reinterpret_cast<int*>(smem_raw + L.gcol);
  T* gVal = reinterpret_cast<T*>(smem_raw + L.gval);
  int* eRow = reinterpret_cast<int*>(smem_raw + L.erow);  // CSR of E' (nu rows)
  int* eCol = reinterpret_cast<int*>(smem_raw + L.ecol);
  T* eVal = reinterpret_cast<T*>(smem_raw + L.eval);
  const bool kids_below = se + 1 < a.N;
  // u-elements of a chunk: e = tid + 512 j -> node-stage e / 128, component
  // e % 128 = tid % 128 for every j; x-elements likewise with 64.
  const int iu = tid & (kSU - 1);
  const int ix = tid & (kSX - 1);
  // Children of the level's last stage (in the level below): lambda, P and
  // parent of a batch of kCN of them, loaded unmasked (clamped indices) and
  // masked where stored.  The first batch flies with the first chunk's loads.
  int cb = 0, ce = 0;
  T bl[kQX], bp[kQU];
  int ba = 0;
  auto load_bnd = [&](int c0) {
#pragma unroll
    for (int j = 0; j < kQX; ++j) {
      const int c = c0 + (tid + j * kSegThreads) / kSX;
      bl[j] = ldc(a.lam, (size_t)c * LDX + ix, c < ce && ix < nx);
    }
#pragma unroll
    for (int j = 0; j < kQU; ++j) {
      const int c = c0 + (tid + j * kSegThreads) / kSU;
      bp[j] = ldc((const T*)a.jv, (size_t)c * kSU + iu, c < ce && iu < nu);
    }
    ba = ldc(a.anc, (size_t)(c0 + tid), tid < kCN && c0 + tid < ce);
  };
  if (kids_below) {
    const int2 kc = a.wgx[2 * wg];
    cb = kc.x;
    ce = kc.y;
  }
  {
    const int2* rg = a.ranges + (size_t)wg * a.nst;
    for (int i = tid; i < a.nst; i += kSegThreads) sRg[i] = rg[i];
    csr_to_lds<T>(a.Btrow, a.Btcol, a.Btval, nu, a.nnzB, sRow, sCol, sVal);
    csr_to_lds<T>(a.Grow, a.Gcol, a.Gval, ns, a.nnzG, gRow, gCol, gVal);
    csr_to_lds<T>(a.Etrow, a.Etcol, a.Etval, nu, a.nnzE, eRow, eCol, eVal);
  }
  __syncthreads();

  FixRow<T, 2> btrow, etrow;
  btrow.load(sRow, sCol, sVal, iu, iu < nu);
  etrow.load(eRow, eCol, eVal, iu, iu < nu);
  const bool gfix = kCN * ns <= kSegThreads;  // one row of G per thread
  FixRow<T, 4> grow;
  grow.load(gRow, gCol, gVal, ns > 0 ? tid % ns : 0, gfix && tid < kCN * ns);

  // Children of the level's last stage: the level below left their lambda and
  // P in global memory.  They are staged through LDS kCN at a time (all loads
  // of a batch in flight together) and summed per slot, in child order: thread
  // t sums the P of slot t / 128 (component t % 128) and the lambda of slot
  // t / 64 (component t % 64), adding zero for the other slots' children
  // (x + 0 = x: the same sums as adding each child to its slot).  The sums go
  // to LDS for the chain threads.
  T accL = T(0), accP = T(0);

  const int nchunk = (a.nst + CS - 1) / CS;
  // Inputs of one chunk: per x-element (y1, y1o, y2, y2o), per u-element (y3,
  // y3o, kappa), per node-stage tid < kCN its children range.
  struct Pre {
    T x[kQX][4], u[kQU][3];
    int c0, c1;
    int nx[kQX], nu[kQU];  // node of each element group (-1: none)
  };
  auto chunk_lo = [&](int c) { return max(sb, se - c * CS - CS + 1); };
  auto chunk_hi = [&](int c) { return se - c * CS; };
  auto load_chunk = [&](int c, Pre& P) {
    const int s_lo = chunk_lo(c), s_hi = chunk_hi(c);
    chunk_nodes<NB, kSX, kQX>(sRg, nullptr, sb, s_lo, s_hi, P.nx, nullptr);
    chunk_nodes<NB, kSU, kQU>(sRg, nullptr, sb, s_lo, s_hi, P.nu, nullptr);
#pragma unroll
    for (int j = 0; j < kQX; ++j) {
      const bool ok = P.nx[j] >= 0 && ix < nx;
      const size_t o = (size_t)P.nx[j] * LDY + ix;
      P.x[j][0] = ldc(Yc, o, ok);
      P.x[j][1] = ldc(Yo, o, ok);
      P.x[j][2] = ldc(Yc, o + LDX, ok);
      P.x[j][3] = ldc(Yo, o + LDX, ok);
    }
#pragma unroll
    for (int j = 0; j < kQU; ++j) {
      const bool ok = P.nu[j] >= 0 && iu < nu;
      const size_t n = (size_t)P.nu[j];
      P.u[j][0] = ldc(Yc, n * LDY + 2 * LDX + iu, ok);
      P.u[j][1] = ldc(Yo, n * LDY + 2 * LDX + iu, ok);
      P.u[j][2] = ldc(a.kappa, n * kSU + iu, ok);
    }
    {
      const int kb = tid < kCN ? tid : 0;
      const int s = s_lo + kb / NB, b = kb % NB;
      const int2 rr = sRg[(s <= s_hi ? s : s_lo) - sb];
      const bool ok = tid < kCN && s <= s_hi && b < rr.y - rr.x;
      P.c0 = ldc(a.cbeg, (size_t)(rr.x + b), ok);
      P.c1 = ldc(a.cend, (size_t)(rr.x + b), ok);
    }
  };

  // per chunk, registers of the u-elements: w3 and kappa
  T w3r[kQU], kr[kQU];
  // chain state: the neighbouring stage's lambda / P per slot (component ix / iu)
  T prevL[NB], prevP[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) prevL[b] = prevP[b] = T(0);
  // delayed stores of P (chain threads): the values of the chunk [ps_lo,
  // ps_lo + pcs) that precedes the current one (pcs = 0: none)
  T dP[kCN];
  int ps_lo = 0, pcs = 0;
  auto flush = [&]() {
    if (tid < kSU && iu < nu) {
#pragma unroll
      for (int k = 0; k < CS; ++k) {
        if (k < pcs) {
          const int2 rr = sRg[ps_lo + k - sb];
#pragma unroll
          for (int b = 0; b < NB; ++b)
            if (b < rr.y - rr.x) {
              T* dst = a.jv + (size_t)(rr.x + b) * kSU + iu;
              if (ps_lo + k == sb) st_agent(dst, dP[k * NB + b]);  // read by the level above
              else *dst = dP[k * NB + b];
            }
        }
      }
    }
  };

  auto chunk = [&](int c, Pre& C, Pre& Nx) {
    vm_wait_all();  // this chunk's inputs, the stores issued a chunk ago
    flush();
    const int s_lo = chunk_lo(c), s_hi = chunk_hi(c);
    const int cs = s_hi - s_lo + 1;
    int* ch = sCh + (c & 1) * kCN;
    // inputs into LDS (a) and registers (w3, kappa)
#pragma unroll
    for (int j = 0; j < kQX; ++j) {
      const int e = tid + j * kSegThreads;
      const bool ok = C.nx[j] >= 0 && ix < nx;
      const T av = power ? scale * (C.x[j][0] + C.x[j][2])
                         : wext(C.x[j][0], C.x[j][1], beta) + wext(C.x[j][2], C.x[j][3], beta);
      sLam[e] = ok ? av : T(0);
    }
#pragma unroll
    for (int j = 0; j < kQU; ++j) {
      const bool ok = C.nu[j] >= 0 && iu < nu;
      const T w3 = power ? scale * C.u[j][0] : wext(C.u[j][0], C.u[j][1], beta);
      w3r[j] = ok ? w3 : T(0);
      kr[j] = ok && !power ? C.u[j][2] : T(0);
    }
    if (tid < kCN) {
      const int kb = tid;
      const int s = s_lo + kb / NB, b = kb % NB;
      int r2 = 0;
      if (s <= s_hi && s < se) {
        const int2 rr = sRg[s - sb];
        if (b < rr.y - rr.x) {
          const int lo_c = sRg[s + 1 - sb].x;
          r2 = pack_ch(C.c0 - lo_c, C.c1 - lo_c);
        }
      }
      ch[kb] = r2;
    }
    // the next chunk's loads fly while this one computes (after the last
    // chunk: an empty one, whose clamped loads all read one element)
    load_chunk(c + 1, Nx);
    __syncthreads();

    // lambda chain, bottom stage of the chunk first, in registers
    if (tid < kSX) {
      T av[kCN], bndL[NB];
      int cr[kCN];
#pragma unroll
      for (int q = 0; q < kCN; ++q) {
        av[q] = sLam[q * kSX + ix];
        cr[q] = __builtin_amdgcn_readfirstlane(ch[q]);
      }
#pragma unroll
      for (int b = 0; b < NB; ++b)  // the boundary sums (first chunk only)
        bndL[b] = kids_below && s_hi == se ? sBnd[NB * kSU + b * kSX + ix] : T(0);
#pragma unroll
      for (int k = CS - 1; k >= 0; --k) {
        if (k < cs) {
          const bool bottom = s_lo + k == se;
#pragma unroll
          for (int b = 0; b < NB; ++b) {
            const int v = cr[k * NB + b];
            av[k * NB + b] += bottom ? bndL[b] : range_sum<T, NB>(prevL, ch_lo(v), ch_hi(v));
          }
#pragma unroll
          for (int b = 0; b < NB; ++b) prevL[b] = av[k * NB + b];
        }
      }
#pragma unroll
      for (int q = 0; q < kCN; ++q) sLam[q * kSX + ix] = av[q];
      if (s_lo == sb && sb > 0) {  // the level above reads the first stage's lambda
        const int2 rr = sRg[0];
#pragma unroll
        for (int b = 0; b < NB; ++b)
          if (b < rr.y - rr.x && ix < nx) st_agent(a.lam + (size_t)(rr.x + b) * LDX + ix, av[b]);
      }
    }
    __syncthreads();
    // v = kappa - (w3 + B' lambda) / (2 w), per u-element (all reads first)
    {
      T t[kQU];
#pragma unroll
      for (int j = 0; j < kQU; ++j) {
        const int kb = (tid + j * kSegThreads) / kSU;
        t[j] = btrow.apply(w3r[j], sLam + kb * kSX, sCol, sVal);
      }
#pragma unroll
      for (int j = 0; j < kQU; ++j) {
        const int e = tid + j * kSegThreads;
        // invalid slots have w3 = kappa = 0 and lambda = 0
        sV[e] = e / kSU < cs * NB && iu < nu ? kr[j] - hw * t[j] : T(0);
      }
    }
    __syncthreads();
    // G v, per (node-stage, row of G)
    if (gfix) {
      if (tid < kCN * ns) sGv[tid] = grow.apply(T(0), sV + (tid / ns) * kSU, gCol, gVal);
    } else {
      for (int e = tid; e < kCN * ns; e += kSegThreads) {
        const int kb = e / ns, r = e - kb * ns;
        const T* v = sV + kb * kSU;
        T acc = T(0);
        for (int p = gRow[r]; p < gRow[r + 1]; ++p) acc += gVal[p] * v[gCol[p]];
        sGv[e] = acc;
      }
    }
    __syncthreads();
    // m = v - E'(G v) (all reads first)
    {
      T m[kQU];
#pragma unroll
      for (int j = 0; j < kQU; ++j) {
        const int e = tid + j * kSegThreads;
        m[j] = sV[e] - etrow.apply(T(0), sGv + (e / kSU) * ns, eCol, eVal);
      }
#pragma unroll
      for (int j = 0; j < kQU; ++j) sV[tid + j * kSegThreads] = iu < nu ? m[j] : T(0);
    }
    __syncthreads();
    // P chain, bottom stage first, in registers; P goes to global memory one
    // chunk later
    if (tid < kSU) {
      int cr[kCN];
      T bndP[NB];
#pragma unroll
      for (int q = 0; q < kCN; ++q) {
        dP[q] = sV[q * kSU + iu];
        cr[q] = __builtin_amdgcn_readfirstlane(ch[q]);
      }
#pragma unroll
      for (int b = 0; b < NB; ++b)  // the boundary sums (first chunk only)
        bndP[b] = kids_below && s_hi == se ? sBnd[b * kSU + iu] : T(0);
#pragma unroll
      for (int k = CS - 1; k >= 0; --k) {
        if (k < cs) {
          const bool bottom = s_lo + k == se;
#pragma unroll
          for (int b = 0; b < NB; ++b) {
            const int v = cr[k * NB + b];
            dP[k * NB + b] += bottom ? bndP[b] : range_sum<T, NB>(prevP, ch_lo(v), ch_hi(v));
          }
#pragma unroll
          for (int b = 0; b < NB; ++b) prevP[b] = dP[k * NB + b];
        }
      }
    }
    ps_lo = s_lo;
    pcs = cs;
  };

  if (kids_below) load_bnd(cb);
  Pre PA, PB;
  load_chunk(0, PA);  // in flight while the children of the last stage are summed
  if (kids_below) {
    const int lo_l = sRg[a.nst - 1].x;
    for (int c0 = cb; c0 < ce; c0 += kCN) {
      if (c0 != cb) load_bnd(c0);
#pragma unroll
      for (int j = 0; j < kQX; ++j) {
        const int e = tid + j * kSegThreads;
        const int c = c0 + e / kSX;
        sLam[e] = c < ce && ix < nx ? bl[j] : T(0);
      }
#pragma unroll
      for (int j = 0; j < kQU; ++j) {
        const int e = tid + j * kSegThreads;
        const int c = c0 + e / kSU;
        sV[e] = c < ce && iu < nu ? bp[j] : T(0);
      }
      if (tid < kCN) sCh[tid] = c0 + tid < ce ? ba - lo_l : -1;
      __syncthreads();
      {
        const int sp = tid / kSU, sq = tid / kSX;
        int bq[kCN];  // slot of child c0 + q (-1: past the last child)
#pragma unroll
        for (int q = 0; q < kCN; ++q) bq[q] = __builtin_amdgcn_readfirstlane(sCh[q]);
#pragma unroll
        for (int q = 0; q < kCN; ++q) {
          const T lv = sLam[q * kSX + ix], pv = sV[q * kSU + iu];
          accL += bq[q] == sq ? lv : T(0);
          accP += bq[q] == sp ? pv : T(0);
        }
      }
      __syncthreads();
    }
    if (tid / kSU < NB) sBnd[(tid / kSU) * kSU + iu] = accP;
    if (tid / kSX < NB) sBnd[NB * kSU + (tid / kSX) * kSX + ix] = accL;
  }

  int c = 0;
  while (true) {
    chunk(c, PA, PB);
    if (++c >= nchunk) break;
    chunk(c, PB, PA);
    if (++c >= nchunk) break;
  }
  flush();
}

// ---------------------------------------------------------------------------
// Light upper levels: the whole backward sweep of a tree or a forest in the
// bottom level's launch (SegArgs::n_main).
// ---------------------------------------------------------------------------

// Local parts for the nodes of upper workgroup j (from its table), 4 nodes
// per pass (one per 128 threads): a_n = w1_n + w2_n to lam and Pi (kappa_n -
// (w3_n + B' a_n) / (2 w)) to jv.  Uses the bottom launch's dynamic LDS layout.
template <typename T>
__device__ __forceinline__ void scan_local_up(const SegArgs<T>& a, int j, int it, T beta,
                                              T scale) {
  const bool power = a.mode == 1;  // w = scale y, no data terms
  constexpr int LN = kSegThreads / kSU;  // nodes per pass
  const int tid = threadIdx.x;
  const T* Yc = (it & 1) ? a.Y1 : a.Y0;
  const T* Yo = (it & 1) ? a.Y0 : a.Y1;
  const int nx = a.nx, nu = a.nu, LDX = a.LDX, LDY = a.LDY, ns = a.ns;
  const T hw = T(0.5) * a.winv;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const BwdLds<T> L(a);
  T* sA = reinterpret_cast<T*>(smem_raw + L.lam);  // [LN][kSX]
  T* sV = reinterpret_cast<T*>(smem_raw + L.v);    // [LN][kSU]
  T* sGv = reinterpret_cast<T*>(smem_raw + L.gv);  // [LN][ns]
  int* sRow = reinterpret_cast<int*>(smem_raw + L.brow);
  int* sCol = reinterpret_cast<int*>(smem_raw + L.bcol);
  T* sVal = reinterpret_cast<T*>(smem_raw + L.bval);
  int* gRow = reinterpret_cast<int*>(smem_raw + L.grow);
  int* gCol = reinterpret_cast<int*>(smem_raw + L.gcol);
  T* gVal = reinterpret_cast<T*>(smem_raw + L.gval);
  int* eRow = reinterpret_cast<int*>(smem_raw + L.erow);
  int* eCol = reinterpret_cast<int*>(smem_raw + L.ecol);
  T* eVal = reinterpret_cast<T*>(smem_raw + L.eval);
  const int* plan = a.up_plan + (size_t)j * a.up_plan_stride;
  const int nw = plan[kPlanNw];
  const int* node = plan + kPlanOff + plan[kPlanNst] + 1;
  csr_to_lds<T>(a.Btrow, a.Btcol, a.Btval, nu, a.nnzB, sRow, sCol, sVal);
  csr_to_lds<T>(a.Grow, a.Gcol, a.Gval, ns, a.nnzG, gRow, gCol, gVal);
  csr_to_lds<T>(a.Etrow, a.Etcol, a.Etval, nu, a.nnzE, eRow, eCol, eVal);
  const int b = tid / kSU, i = tid % kSU;
  for (int k0 = 0; k0 < nw; k0 += LN) {
    const bool node_ok = k0 + b < nw;
    const int n = node_ok ? node[k0 + b] : 0;
    T ax = T(0), w3 = T(0), kap = T(0);
    if (node_ok && i < nx) {
      const size_t o = (size_t)n * LDY + i;
      ax = power ? scale * (Yc[o] + Yc[o + LDX])
                 : wext(Yc[o], Yo[o], beta) + wext(Yc[o + LDX], Yo[o + LDX], beta);
    }
    if (node_ok && i < nu) {
      const size_t o = (size_t)n * LDY + 2 * LDX + i;
      w3 = power ? scale * Yc[o] : wext(Yc[o], Yo[o], beta);
      kap = power ? T(0) : a.kappa[(size_t)n * kSU + i];
    }
    if (i < kSX) sA[b * kSX + i] = ax;
    __syncthreads();
    {  // v = kappa - (w3 + B' a) / (2 w)
      T t = w3;
      if (i < nu)
        for (int p = sRow[i]; p < sRow[i + 1]; ++p) t += sVal[p] * sA[b * kSX + sCol[p]];
      sV[b * kSU + i] = node_ok && i < nu ? kap - hw * t : T(0);
    }
    __syncthreads();
    for (int e = tid; e < LN * ns; e += kSegThreads) {  // G v
      const int bb = e / ns, r = e - bb * ns;
      T acc = T(0);
      for (int p = gRow[r]; p < gRow[r + 1]; ++p) acc += gVal[p] * sV[bb * kSU + gCol[p]];
      sGv[bb * ns + r] = acc;
    }
    __syncthreads();
    if (node_ok && i < nu) {  // Pi v = v - E'(G v)
      T acc = T(0);
      for (int p = eRow[i]; p < eRow[i + 1]; ++p) acc += eVal[p] * sGv[b * ns + eCol[p]];
      st_agent(a.jv + (size_t)n * kSU + i, sV[b * kSU + i] - acc);
    }
    if (node_ok && i < nx) st_agent(a.lam + (size_t)n * LDX + i, ax);
  }
}

// Dynamic LDS of an upper workgroup's work: the CSR (as in the backward
// layout), its table, per node lambda, P, the children's lambda sum, B' of
// it and G B' of it, and the children below (lambda and P).
template <typename T>
struct TopLds : CsrLds<T> {
  size_t plan, lam, p, sl, t, g, bl, bp, total;
  __host__ __device__ TopLds(int plan_ints, int nw_, int nch_, int nu, int ns, int nnzB,
                             int nnzG, int nnzE) {
    LdsCursor c;
    this->take(c, nu, ns, nnzB, nnzG, nnzE);
    const size_t nw = (size_t)(nw_ > 0 ? nw_ : 1), nch = (size_t)(nch_ > 0 ? nch_ : 1);
    plan = c.take(sizeof(int) * plan_ints);
    lam = c.take(sizeof(T) * nw * kSX);
    p = c.take(sizeof(T) * nw * kSU);
    sl = c.take(sizeof(T) * nw * kSX);
    t = c.take(sizeof(T) * nw * kSU);
    g = c.take(sizeof(T) * nw * (ns > 0 ? ns : 1));
    bl = c.take(sizeof(T) * nch * kSX);
    bp = c.take(sizeof(T) * nch * kSU);
    total = c.off;
  }
};

// The work of the upper workgroup whose table is in LDS: its nodes' a_n and
// local part of m_n are in lam and jv, and so are the children below its last
// stage (lambda at their stage, P), which the workgroups below left there.
// One batch of loads gathers them all.  The recursions are component-wise,
// so one thread per component walks the stages from the last: lambda_n = a_n
// + sum lambda_c; then the corrections Pi B' (sum lambda_c) / (2 w) of all
// nodes at once; then P_n = (local_n - correction_n) + sum P_c.  Writes P_n
// for its nodes and lambda_n for its first stage.  The CSR of B', G and E'
// are in LDS.
template <typename T>
__device__ void scan_top_body(const SegArgs<T>& a) {
  const int tid = threadIdx.x;
  const int nx = a.nx, nu = a.nu, LDX = a.LDX, ns = a.ns;
  const T hw = T(0.5) * a.winv;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const TopLds<T> L(a.up_plan_stride, a.up_nw, a.up_nch, nu, ns, a.nnzB, a.nnzG, a.nnzE);
  const int* P = reinterpret_cast<const int*>(smem_raw + L.plan);
  T* sL = reinterpret_cast<T*>(smem_raw + L.lam);   // [nw][kSX]: a, then lambda
  T* sP = reinterpret_cast<T*>(smem_raw + L.p);     // [nw][kSU]: local part, then P
  T* sS = reinterpret_cast<T*>(smem_raw + L.sl);    // [nw][kSX]: sum of children's lambda
  T* sT = reinterpret_cast<T*>(smem_raw + L.t);     // [nw][kSU]: B' sum
  T* sG = reinterpret_cast<T*>(smem_raw + L.g);     // [nw][ns]: G B' sum
  T* sBL = reinterpret_cast<T*>(smem_raw + L.bl);   // [nch][kSX]: lambda of the children below
  T* sBP = reinterpret_cast<T*>(smem_raw + L.bp);   // [nch][kSU]: P of the children below
  const int* sRow = reinterpret_cast<const int*>(smem_raw + L.brow);
  const int* sCol = reinterpret_cast<const int*>(smem_raw + L.bcol);
  const T* sVal = reinterpret_cast<const T*>(smem_raw + L.bval);
  const int* gRow = reinterpret_cast<const int*>(smem_raw + L.grow);
  const int* gCol = reinterpret_cast<const int*>(smem_raw + L.gcol);
  const T* gVal = reinterpret_cast<const T*>(smem_raw + L.gval);
  const int* eRow = reinterpret_cast<const int*>(smem_raw + L.erow);
  const int* eCol = reinterpret_cast<const int*>(smem_raw + L.ecol);
  const T* eVal = reinterpret_cast<const T*>(smem_raw + L.eval);
  const int nw = P[kPlanNw], nst = P[kPlanNst], cb = P[kPlanCb], nchl = P[kPlanNch];
  const int* off = P + kPlanOff;
  const int* node = off + nst + 1;
  const int* clo = node + nw;
  const int* chi = clo + nw;
  // Gather: element e of [children lambda | children P | own a | own local
  // part], rows of kSX or kSU; R loads per thread in flight before any wait.
  // Sources and LDS destinations are kept as offsets from global and LDS
  // bases, so that loads stay global and stores stay in LDS.
  {
    constexpr int R = 8;
    const int e1 = nchl * kSX, e2 = e1 + nchl * kSU, e3 = e2 + nw * kSX, e4 = e3 + nw * kSU;
    T* sDst = reinterpret_cast<T*>(smem_raw);  // element offsets below are from here
    const size_t oBL = L.bl / sizeof(T), oBP = L.bp / sizeof(T), oL = L.lam / sizeof(T),
                 oP = L.p / sizeof(T);
    for (int base = 0; base < e4; base += R * kSegThreads) {
      T v[R];
      int dst[R];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int e = base + r * kSegThreads + tid;
        bool ok = false, from_lam = true;
        size_t src = 0;
        dst[r] = -1;
        if (e < e1) {
          const int c = e / kSX, i = e - c * kSX;
          ok = i < nx;
          src = (size_t)(cb + c) * LDX + i;
          dst[r] = (int)(oBL + e);
        } else if (e < e2) {
          const int c = (e - e1) / kSU, i = (e - e1) - c * kSU;
          ok = i < nu;
          from_lam = false;
          src = (size_t)(cb + c) * kSU + i;
          dst[r] = (int)(oBP + (e - e1));
        } else if (e < e3) {
          const int k = (e - e2) / kSX, i = (e - e2) - k * kSX;
          ok = i < nx;
          src = (size_t)node[k] * LDX + i;
          dst[r] = (int)(oL + (e - e2));
        } else if (e < e4) {
          const int k = (e - e3) / kSU, i = (e - e3) - k * kSU;
          ok = i < nu;
          from_lam = false;
          src = (size_t)node[k] * kSU + i;
          dst[r] = (int)(oP + (e - e3));
        }
        const T* base_p = from_lam ? a.lam : a.jv;
        v[r] = ld_agent(base_p + (ok ? src : 0));
        v[r] = ok ? v[r] : T(0);
      }
#pragma unroll
      for (int r = 0; r < R; ++r)
        if (dst[r] >= 0) sDst[dst[r]] = v[r];
    }
  }
  __syncthreads();
  // lambda chain, one thread per component, deepest stage first: the sum of
  // the children's lambda (below the last stage: the gathered ones) and
  // lambda_n = a_n + sum; the first stage's lambda goes out at once
  if (tid < kSX) {
    const int i = tid;
    for (int q = nst - 1; q >= 0; --q) {
      const T* CL = q == nst - 1 ? sBL : sL;
      for (int k = off[q]; k < off[q + 1]; ++k) {
        T acc = T(0);
        for (int c = clo[k]; c < chi[k]; ++c) acc += CL[c * kSX + i];
        sS[k * kSX + i] = acc;
        sL[k * kSX + i] += acc;
      }
    }
    if (P[kPlanSb] > 0 && i < nx)  // the level above reads the first stage's lambda
      for (int k = 0; k < off[1]; ++k) st_agent(a.lam + (size_t)node[k] * LDX + i, sL[k * kSX + i]);
  }
  __syncthreads();
  // the corrections Pi B' (sum lambda) / (2 w) of every node: B' (sum lambda)
  for (int e = tid; e < nw * kSU; e += kSegThreads) {
    const int k = e / kSU, i = e % kSU;
    T acc = T(0);
    if (i < nu)
      for (int p = sRow[i]; p < sRow[i + 1]; ++p) acc += sVal[p] * sS[k * kSX + sCol[p]];
    sT[k * kSU + i] = acc;
  }
  __syncthreads();
  for (int e = tid; e < nw * ns; e += kSegThreads) {  // G B' (sum lambda)
    const int k = e / ns, r = e % ns;
    T acc = T(0);
    for (int p = gRow[r]; p < gRow[r + 1]; ++p) acc += gVal[p] * sT[k * kSU + gCol[p]];
    sG[k * ns + r] = acc;
  }
  __syncthreads();
  for (int e = tid; e < nw * kSU; e += kSegThreads) {  // local part less the correction
    const int k = e / kSU, i = e % kSU;
    if (i < nu) {
      T acc = T(0);
      for (int p = eRow[i]; p < eRow[i + 1]; ++p) acc += eVal[p] * sG[k * ns + eCol[p]];
      sP[k * kSU + i] -= hw * (sT[k * kSU + i] - acc);
    }
  }
  __syncthreads();
  // P chain, one thread per component, deepest stage first: P_n = (local_n -
  // correction_n) + sum of the children's P; every P goes out
  if (tid < kSU && tid < nu) {
    const int i = tid;
    for (int q = nst - 1; q >= 0; --q) {
      const T* CP = q == nst - 1 ? sBP : sP;
      for (int k = off[q]; k < off[q + 1]; ++k) {
        T acc = T(0);
        for (int c = clo[k]; c < chi[k]; ++c) acc += CP[c * kSU + i];
        const T v = sP[k * kSU + i] + acc;
        sP[k * kSU + i] = v;
        st_agent(a.jv + (size_t)node[k] * kSU + i, v);
      }
    }
  }
}

// After a workgroup's stores: one arrival at each upper workgroup p0 .. p1;
// an arrival that completes an upper workgroup's inputs runs it here, then
// arrives above it.  What crosses workgroups (lambda at a level's first
// stage, P there, the local parts, an upper workgroup's results) is written
// and read with agent-scope atomic stores and loads.  Before an arrival every
// wave waits for its stores to complete and the workgroup meets at a
// barrier, so thread 0's arrival (an atomic add) follows them; the runner's
// threads read after the barrier that follows its arrival.  The table of the
// first upper workgroup a workgroup may run is loaded (it is static) while
// the stores complete; the CSR of B', G and E' stay in LDS from the
// workgroup's own work.
template <typename T>
__device__ void scan_cascade(const SegArgs<T>& a, int p0, int p1) {
  __shared__ int sStack[kUpStack];
  __shared__ int sTop, sRun, sHave;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const TopLds<T> L(a.up_plan_stride, a.up_nw, a.up_nch, a.nu, a.ns, a.nnzB, a.nnzG, a.nnzE);
  int* sPlan = reinterpret_cast<int*>(smem_raw + L.plan);
  const int tid = threadIdx.x;
  const int PS = a.up_plan_stride;  // <= kSegThreads (the host checks)
  int pre = p0;  // upper workgroup whose table is prefetched
  int pv = pre >= 0 && tid < PS ? a.up_plan[(size_t)pre * PS + tid] : 0;
  vm_wait_all();
  __syncthreads();  // the workgroup's own work is done with the LDS
  if (pre >= 0 && tid < PS) sPlan[tid] = pv;
  if (tid == 0) {
    int n = 0;
    for (int u = p1; p0 >= 0 && u >= p0 && n < kUpStack; --u) sStack[n++] = u;
    sTop = n;
    sHave = pre;
  }
  __syncthreads();
  while (true) {
    if (tid == 0) {
      int run = -1;
      while (sTop > 0 && run < 0) {
        const int u = sStack[--sTop];
        const unsigned old = __hip_atomic_fetch_add(&a.up_cnt[u], 1u, __ATOMIC_RELAXED,
                                                    __HIP_MEMORY_SCOPE_AGENT);
        if (old + 1u == (unsigned)a.up_need[u]) {
          // every arrival of this launch is in: the counter is free again
          __hip_atomic_store(&a.up_cnt[u], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          run = u;
        }
      }
      sRun = run;
    }
    __syncthreads();
    const int u = sRun;
    if (u < 0) return;
    if (sHave != u) {  // not the prefetched table
      const int v = tid < PS ? a.up_plan[(size_t)u * PS + tid] : 0;
      __syncthreads();
      if (tid < PS) sPlan[tid] = v;
      if (tid == 0) sHave = u;
      __syncthreads();
    }
    scan_top_body<T>(a);
    const int q0 = sPlan[kPlanPar0], q1 = sPlan[kPlanPar1];
    const int nv = q0 >= 0 && tid < PS ? a.up_plan[(size_t)q0 * PS + tid] : 0;  // next table
    vm_wait_all();
    __syncthreads();
    if (q0 >= 0 && tid < PS) sPlan[tid] = nv;
    if (tid == 0) {
      int n = sTop;
      for (int v = q1; q0 >= 0 && v >= q0 && n < kUpStack; --v) sStack[n++] = v;
      sTop = n;
      sHave = q0;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Forward sweep of workgroup `wg` (tree `tree`) over its level, stages
// s_begin up to s_end, in iteration `it`, with the fused prox / dual update
// (as in the segment form).  Returns the workgroup's max |y+ - w| / gamma
// (power iteration: the sum of squares of its part of the new iterate).
// ---------------------------------------------------------------------------
template <typename T, int NB>
__device__ __forceinline__ double scan_fwd_body(const SegArgs<T>& a, int wg, int tree, int it,
                                                T beta, double gam64, double* sred) {
  constexpr int CS = kCN / NB;
  const int tid = threadIdx.x;
  const bool power = a.mode == 1;
  const T* Yc = (it & 1) ? a.Y1 : a.Y0;
  T* Yn = (it & 1) ? a.Y0 : a.Y1;  // y^{nu-1} in, y^{nu+1} out
  const T gam = (T)gam64;
  const int nx = a.nx, nu = a.nu, LDX = a.LDX, LDY = a.LDY;
  const int sb = a.s_begin, se = a.s_end;

  extern __shared__ __align__(16) unsigned char smem_raw[];
  const FwdLds<T> L(a);
  T* sC = reinterpret_cast<T*>(smem_raw + L.c);  // [kCN][kSU]: j / p, then u
  T* sD = reinterpret_cast<T*>(smem_raw + L.d);  // [kCN][kSU]: P / p
  T* sX = reinterpret_cast<T*>(smem_raw + L.x);  // [kCN][kSX]: B u + g, then x
  int2* sRg = reinterpret_cast<int2*>(smem_raw + L.rg);
  int* sOwn = reinterpret_cast<int*>(smem_raw + L.own);  // first node written, per stage
  int* sPar = reinterpret_cast<int*>(smem_raw + L.par);  // [kCN]: parent slot
  int* sRow = reinterpret_cast<int*>(smem_raw + L.brow);  // CSR of B (nx rows)
  int* sCol = reinterpret_cast<int*>(smem_raw + L.bcol);
  T* sVal = reinterpret_cast<T*>(smem_raw + L.bval);
  // bounds xmin, xmax, xs | umin, umax: scaled by gamma in FP64 sweeps (then
  // gamma P_C(v / gamma) = P_{gamma C}(v) needs no division); unscaled with FP32
  // sweeps, whose prox runs in FP64 (bnd() scales them there)
  __shared__ T sBnd[5 * kSU];
  const T bscale = sizeof(T) == sizeof(double) ? gam : T(1);
  auto bnd = [&](int i) -> double {
    return sizeof(T) == sizeof(double) ? (double)sBnd[i] : gam64 * (double)sBnd[i];
  };
  int par0, parl;  // parents of the level's first and last first-stage nodes
  {
    const int2* rg = a.ranges + (size_t)wg * a.nst;
    for (int i = tid; i < a.nst; i += kSegThreads) {
      sRg[i] = rg[i];
      sOwn[i] = a.own ? a.own[(size_t)wg * a.nst + i] : 0;
    }
    csr_to_lds<T>(a.Brow, a.Bcol, a.Bval, nx, a.nnzB, sRow, sCol, sVal);
    for (int i = tid; i < kSU; i += kSegThreads) {
      sBnd[i] = bscale * ldm(a.xmin, i, i < nx);
      sBnd[kSU + i] = bscale * ldm(a.xmax, i, i < nx);
      sBnd[2 * kSU + i] = bscale * ldm(a.xs, i, i < nx);
      sBnd[3 * kSU + i] = bscale * ldm(a.umin, i, i < nu);
      sBnd[4 * kSU + i] = bscale * ldm(a.umax, i, i < nu);
    }
    const int2 pp = a.wgx[2 * wg + 1];
    par0 = pp.x;
    parl = pp.y;
  }
  __syncthreads();
  const int iu = tid & (kSU - 1);
  const int ix = tid & (kSX - 1);
  FixRow<T, 5> brow;
  brow.load(sRow, sCol, sVal, ix, ix < nx);

  // parents of the level's first stage: the level above left x and z = Pi u in
  // global memory; at the root they are (p, Pi q) of the tree (zero in the
  // power iteration)
  const int lo_p = par0 >= 0 ? par0 : 0;
  const int np = par0 >= 0 ? parl - par0 + 1 : 1;
  T xprev[NB], zprev[NB];
  const bool kids_below = se + 1 < a.N;

  const int nchunk = (a.nst + CS - 1) / CS;
  // Inputs of one chunk: per u-element (P, kperp, 1/p, y3, y3o), per x-element
  // (g, y1, y1o, y2, y2o), per node-stage tid < kCN its parent.
  struct Pre {
    T u[kQU][5], x[kQX][5];
    int an;
    int nu[kQU], nx[kQX];  // node of each element group (-1: none)
    int ou[kQU], ox[kQX];  // the same where this workgroup owns (writes) it
  };
  auto load_chunk = [&](int c, Pre& P) {
    const int s_lo = sb + c * CS, s_hi = min(se, s_lo + CS - 1);
    chunk_nodes<NB, kSU, kQU>(sRg, sOwn, sb, s_lo, s_hi, P.nu, &P.ou);
    chunk_nodes<NB, kSX, kQX>(sRg, sOwn, sb, s_lo, s_hi, P.nx, &P.ox);
#pragma unroll
    for (int j = 0; j < kQU; ++j) {
      const bool ok = P.nu[j] >= 0 && iu < nu;
      const size_t n = (size_t)P.nu[j];
      P.u[j][0] = ldc((const T*)a.jv, n * kSU + iu, ok);
      P.u[j][1] = ldc(a.kperp, n * kSU + iu, ok);
      P.u[j][2] = ldc(a.invp, n, ok);
      // FP64: the dual iterates only where this workgroup writes the node (the
      // owner test is the same in every lane of a wave: a scalar branch); an
      // ancestor it only walks needs P, kperp and 1/p for the chains.  (FP32
      // measured faster without the branch.)
      if (sizeof(T) != sizeof(double) || P.ou[j] >= 0) {
        P.u[j][3] = ldc(Yc, n * LDY + 2 * LDX + iu, ok);
        P.u[j][4] = ldc((const T*)Yn, n * LDY + 2 * LDX + iu, ok);
      } else {
        P.u[j][3] = P.u[j][4] = T(0);
      }
    }
#pragma unroll
    for (int j = 0; j < kQX; ++j) {
      const bool ok = P.nx[j] >= 0 && ix < nx;
      const size_t n = (size_t)P.nx[j];
      P.x[j][0] = ldc(a.g, n * LDX + ix, ok);
      if (sizeof(T) != sizeof(double) || P.ox[j] >= 0) {
        P.x[j][1] = ldc(Yc, n * LDY + ix, ok);
        P.x[j][2] = ldc((const T*)Yn, n * LDY + ix, ok);
        P.x[j][3] = ldc(Yc, n * LDY + LDX + ix, ok);
        P.x[j][4] = ldc((const T*)Yn, n * LDY + LDX + ix, ok);
      } else {
        P.x[j][1] = P.x[j][2] = P.x[j][3] = P.x[j][4] = T(0);
      }
    }
    {
      const int kb = tid < kCN ? tid : 0;
      const int s = s_lo + kb / NB, b = kb % NB;
      const int2 rr = sRg[min(s, s_hi) - sb];
      const bool ok = tid < kCN && s <= s_hi && b < rr.y - rr.x;
      P.an = ldc(a.anc, (size_t)(rr.x + b), ok);
    }
  };

  // per chunk, registers of this thread's elements for the prox
  T w3r[kQU], w1r[kQX], w2r[kQX], gr[kQX];
  double rmax = 0.0, zsq = 0.0;
  // delayed stores: u, y3 per u-element; x, y1, y2 per x-element (-1: none)
  T du[kQU], dy3[kQU], dxv[kQX], dy1[kQX], dy2[kQX];
  int dnu[kQU], dnx[kQX];
#pragma unroll
  for (int j = 0; j < kQU; ++j) dnu[j] = -1;
#pragma unroll
  for (int j = 0; j < kQX; ++j) dnx[j] = -1;
  auto flush = [&]() {
#pragma unroll
    for (int j = 0; j < kQU; ++j)
      if (dnu[j] >= 0 && iu < nu) {
        a.u[(size_t)dnu[j] * kSU + iu] = du[j];
        Yn[(size_t)dnu[j] * LDY + 2 * LDX + iu] = dy3[j];
      }
#pragma unroll
    for (int j = 0; j < kQX; ++j)
      if (dnx[j] >= 0 && ix < nx) {
        a.x[(size_t)dnx[j] * LDX + ix] = dxv[j];
        Yn[(size_t)dnx[j] * LDY + ix] = dy1[j];
        Yn[(size_t)dnx[j] * LDY + LDX + ix] = dy2[j];
      }
  };

  auto chunk = [&](int c, Pre& C, Pre& Nx) {
    vm_wait_all();
    flush();
    const int s_lo = sb + c * CS, s_hi = min(se, s_lo + CS - 1);
    const int cs = s_hi - s_lo + 1;
#pragma unroll
    for (int j = 0; j < kQU; ++j) {
      const int e = tid + j * kSegThreads;
      const bool ok = C.nu[j] >= 0 && iu < nu;
      const T d = C.u[j][0] * C.u[j][2];
      const T cj = power ? d : (C.u[j][1] + C.u[j][0]) * C.u[j][2];
      sC[e] = ok ? cj : T(0);
      sD[e] = ok ? d : T(0);
      w3r[j] = ok ? wext(C.u[j][3], C.u[j][4], beta) : T(0);
    }
#pragma unroll
    for (int j = 0; j < kQX; ++j) {
      const bool ok = C.nx[j] >= 0 && ix < nx;
      gr[j] = ok && !power ? C.x[j][0] : T(0);
      w1r[j] = ok ? wext(C.x[j][1], C.x[j][2], beta) : T(0);
      w2r[j] = ok ? wext(C.x[j][3], C.x[j][4], beta) : T(0);
    }
    if (tid < kCN) {
      const int kb = tid;
      const int s = s_lo + kb / NB, b = kb % NB;
      int pb = 0;
      if (s <= s_hi) {
        const int2 rr = sRg[s - sb];
        const int base = s == sb ? lo_p : sRg[s - 1 - sb].x;
        if (b < rr.y - rr.x && C.an >= 0) pb = C.an - base;
      }
      sPar[kb] = pb;
    }
    load_chunk(c + 1, Nx);  // after the last chunk: an empty one
    __syncthreads();

    // u / z chain, top stage first, in registers
    if (tid < kSU) {
      T cv[kCN], dv[kCN];
      int pr[kCN];
#pragma unroll
      for (int q = 0; q < kCN; ++q) {
        cv[q] = sC[q * kSU + iu];
        dv[q] = sD[q * kSU + iu];
        pr[q] = __builtin_amdgcn_readfirstlane(sPar[q]);
      }
#pragma unroll
      for (int k = 0; k < CS; ++k) {
        if (k < cs) {
          T cur[NB];
#pragma unroll
          for (int b = 0; b < NB; ++b) {
            const T zp = pick<T, NB>(zprev, pr[k * NB + b]);
            cv[k * NB + b] += zp;   // u
            cur[b] = zp + dv[k * NB + b];  // z
          }
#pragma unroll
          for (int b = 0; b < NB; ++b) zprev[b] = cur[b];
        }
      }
#pragma unroll
      for (int q = 0; q < kCN; ++q) sC[q * kSU + iu] = cv[q];
      if (s_hi == se && kids_below) {  // the level below reads z of the last stage
        const int2 rr = sRg[se - sb];
#pragma unroll
        for (int b = 0; b < NB; ++b)
          if (b < rr.y - rr.x && iu < nu) a.zb[(size_t)(rr.x + b) * kSU + iu] = zprev[b];
      }
    }
    __syncthreads();
    // B u + g, per x-element (all reads first)
    {
      T v[kQX];
#pragma unroll
      for (int j = 0; j < kQX; ++j) {
        const int kb = (tid + j * kSegThreads) / kSX;
        v[j] = brow.apply(gr[j], sC + kb * kSU, sCol, sVal);
      }
#pragma unroll
      for (int j = 0; j < kQX; ++j) {
        const int e = tid + j * kSegThreads;
        sX[e] = e / kSX < cs * NB && ix < nx ? v[j] : T(0);
      }
    }
    __syncthreads();
    // x chain, top stage first, in registers
    if (tid < kSX) {
      T xv[kCN];
      int pr[kCN];
#pragma unroll
      for (int q = 0; q < kCN; ++q) {
        xv[q] = sX[q * kSX + ix];
        pr[q] = __builtin_amdgcn_readfirstlane(sPar[q]);
      }
#pragma unroll
      for (int k = 0; k < CS; ++k) {
        if (k < cs) {
#pragma unroll
          for (int b = 0; b < NB; ++b) xv[k * NB + b] += pick<T, NB>(xprev, pr[k * NB + b]);
#pragma unroll
          for (int b = 0; b < NB; ++b) xprev[b] = xv[k * NB + b];
        }
      }
#pragma unroll
      for (int q = 0; q < kCN; ++q) sX[q * kSX + ix] = xv[q];
    }
    __syncthreads();

    // ---- prox / dual update, per element; stores held for the next chunk ----
    // (every LDS read first, then the arithmetic; owned elements are written
    // and counted here: an ancestor shared with a lower-numbered workgroup is
    // computed by both and written by that one)
#pragma unroll
    for (int j = 0; j < kQU; ++j) {
      du[j] = sC[tid + j * kSegThreads];
      dnu[j] = C.ou[j];
    }
#pragma unroll
    for (int j = 0; j < kQX; ++j) {
      dxv[j] = sX[tid + j * kSegThreads];  // one node-stage per wave
      dnx[j] = C.ox[j];
    }
    if (power) {
#pragma unroll
      for (int j = 0; j < kQU; ++j) {
        dy3[j] = -du[j];
        if (C.ou[j] >= 0 && iu < nu) zsq += (double)du[j] * (double)du[j];
      }
#pragma unroll
      for (int j = 0; j < kQX; ++j) {
        dy1[j] = dy2[j] = -dxv[j];
        if (C.ox[j] >= 0 && ix < nx) zsq += 2.0 * (double)dxv[j] * (double)dxv[j];
      }
    } else {
      // The prox and the residual in FP64 whatever T (the FP32 sweeps' w and
      // x widened): y+ is rounded to T once, and |y+ - w| / gamma is the FP64
      // split residual |H x_hat - t| of those inputs.
      const double ulo = bnd(3 * kSU + iu), uhi = bnd(4 * kSU + iu);
      const double xlo = bnd(ix), xhi = bnd(kSU + ix), xsf = bnd(2 * kSU + ix);
#pragma unroll
      for (int j = 0; j < kQU; ++j) {
        const double w = (double)w3r[j];
        const double v = w + gam64 * (double)du[j];
        const double y = v - fmin(fmax(v, ulo), uhi);
        dy3[j] = (T)y;
        if (C.ou[j] >= 0 && iu < nu) {
          double d = fabs(y - w);
          if (!(d <= 1.0e308)) d = INFINITY;
          rmax = fmax(rmax, d);
        }
      }
      double r1[kQX], r2[kQX];
      double q1[kQX], q2[kQX];
#pragma unroll
      for (int j = 0; j < kQX; ++j) {
        const bool valid = C.nx[j] >= 0 && ix < nx;
        const double v1 = (double)w1r[j] + gam64 * (double)dxv[j];
        const double v2 = (double)w2r[j] + gam64 * (double)dxv[j];
        r1[j] = valid ? v1 - fmin(fmax(v1, xlo), xhi) : 0.0;
        r2[j] = valid ? v2 - fmax(v2, xsf) : 0.0;
      }
#pragma unroll
      for (int j = 0; j < kQX; ++j) {
        q1[j] = wave_sum(r1[j] * r1[j]);
        q2[j] = wave_sum(r2[j] * r2[j]);
      }
#pragma unroll
      for (int j = 0; j < kQX; ++j) {
        const double n1 = sqrt(q1[j]), n2 = sqrt(q2[j]);
        const double sc1 = n1 > (double)a.Wx ? (double)a.Wx / n1 : 1.0;
        const double sc2 = n2 > (double)a.Ws ? (double)a.Ws / n2 : 1.0;
        const double y1 = r1[j] * sc1, y2 = r2[j] * sc2;
        dy1[j] = (T)y1;
        dy2[j] = (T)y2;
        if (C.ox[j] >= 0 && ix < nx) {
          double d1 = fabs(y1 - (double)w1r[j]);
          double d2 = fabs(y2 - (double)w2r[j]);
          if (!(d1 <= 1.0e308)) d1 = INFINITY;
          if (!(d2 <= 1.0e308)) d2 = INFINITY;
          rmax = fmax(rmax, fmax(d1, d2));
        }
      }
    }
  };

  Pre PA, PB;
  load_chunk(0, PA);  // in flight together with the parents' loads
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const bool okp = par0 >= 0 && b < np;
    xprev[b] = ldm(a.x, (size_t)(lo_p + b) * LDX + ix, okp && ix < nx);
    zprev[b] = ldm((const T*)a.zb, (size_t)(lo_p + b) * kSU + iu, okp && iu < nu);
  }
  if (par0 < 0 && !power) {
    xprev[0] = ldm(a.pq + (size_t)tree * a.pq_stride, ix, ix < nx);
    zprev[0] = ldm(a.zr + (size_t)tree * kSU, iu, iu < nu);
  }
  int c = 0;
  while (true) {
    chunk(c, PA, PB);
    if (++c >= nchunk) break;
    chunk(c, PB, PA);
    if (++c >= nchunk) break;
  }
  flush();
  if (power) return block_sum512(zsq, sred);
  return block_max512(rmax, sred) / gam64;
}

}  // namespace

// UP: the bottom launch of light upper levels (SegArgs::n_main > 0); a
// separate instance, so that the plain backward kernel carries none of it.
template <typename T, int NB, bool UP>
__global__ __launch_bounds__(kSegThreads) void scan_bwd_kernel(SegArgs<T> a) {
  const int wg = (int)blockIdx.x;
  if (UP && wg >= a.n_main) {  // local parts of upper workgroup j
    const int j = wg - a.n_main;
    const int tree = a.up_plan[(size_t)j * a.up_plan_stride + kPlanTree];
    const DevCtl c = a.close ? bwd_ctl_peek(a, tree) : a.ctl[tree];
    if (c.done) return;  // so do the tree's bottom workgroups: no arrivals
    scan_local_up<T>(a, j, c.iter, (T)c.beta, (T)c.pw_scale);
    scan_cascade<T>(a, j, j);
    return;
  }
  const int tree = a.wgtree ? a.wgtree[wg] : 0;  // a workgroup never spans two trees
  const DevCtl c = bwd_ctl(a, tree, wg);
  if (c.done) return;
  scan_bwd_body<T, NB>(a, wg, c.iter, (T)c.beta, (T)c.pw_scale);
  if (UP) {  // the levels above, in this launch
    const int2 p = a.up_par[wg];
    scan_cascade<T>(a, p.x, p.y);
  }
}

template <typename T, int NB>
__global__ __launch_bounds__(kSegThreads) void scan_fwd_kernel(SegArgs<T> a) {
  const int tree = a.wgtree ? a.wgtree[blockIdx.x] : 0;
  DevCtl* ctl = a.ctl + tree;
  __shared__ double sred[kSegThreads];
  if (ctl->done) return;  // this tree has stopped
  const double m = scan_fwd_body<T, NB>(a, blockIdx.x, tree, ctl->iter, (T)ctl->beta,
                                        ctl->gamma, sred);
  if (threadIdx.x == 0) {
    if (a.mode == 1)
      a.part[a.part_base + blockIdx.x] = m;
    else
      atomicMax(&ctl->res_bits, (unsigned long long)__double_as_longlong(m));
  }
}

template <typename T>
size_t scan_up_lds(int plan_ints, int nw, int nch, int nu, int ns, int nnzB, int nnzG, int nnzE) {
  return (TopLds<T>(plan_ints, nw, nch, nu, ns, nnzB, nnzG, nnzE).total + 15) & ~(size_t)15;
}

// Dynamic LDS of a backward launch that also runs the upper levels.
template <typename T>
size_t scan_bwd_lds_with_up(const SegArgs<T>& a) {
  const size_t b = scan_lds_bytes<T>(a, false);
  const size_t t = scan_up_lds<T>(a.up_plan_stride, a.up_nw, a.up_nch, a.nu, a.ns, a.nnzB,
                                  a.nnzG, a.nnzE);
  return t > b ? t : b;
}

template <typename T, int NB>
void launch_scan_nb(bool fwd, const SegArgs<T>& a, int n_wg, hipStream_t st) {
  const size_t lds = !fwd && a.n_main > 0 ? scan_bwd_lds_with_up<T>(a) : scan_lds_bytes<T>(a, fwd);
  if (fwd)
    hipLaunchKernelGGL((scan_fwd_kernel<T, NB>), dim3(n_wg), dim3(kSegThreads), lds, st, a);
  else if (a.n_main > 0)
    hipLaunchKernelGGL((scan_bwd_kernel<T, NB, true>), dim3(n_wg), dim3(kSegThreads), lds, st, a);
  else
    hipLaunchKernelGGL((scan_bwd_kernel<T, NB, false>), dim3(n_wg), dim3(kSegThreads), lds, st, a);
}

template <typename T>
void launch_scan(bool fwd, int nbm, const SegArgs<T>& a, int n_wg, hipStream_t st) {
  switch (nbm) {
    case 4: launch_scan_nb<T, 4>(fwd, a, n_wg, st); break;
    case 2: launch_scan_nb<T, 2>(fwd, a, n_wg, st); break;
    case 1: launch_scan_nb<T, 1>(fwd, a, n_wg, st); break;
    default: throw Fail{TAPG_EINVAL, "scan sweep: unsupported nodes per stage " + std::to_string(nbm)};
  }
}

template <typename T>
size_t scan_lds(int, const SegArgs<T>& a) {
  const size_t f = scan_lds_bytes<T>(a, true), b = scan_lds_bytes<T>(a, false);
  return f > b ? f : b;
}

template void launch_scan<double>(bool, int, const SegArgs<double>&, int, hipStream_t);
template void launch_scan<float>(bool, int, const SegArgs<float>&, int, hipStream_t);
template size_t scan_lds<double>(int, const SegArgs<double>&);
template size_t scan_lds<float>(int, const SegArgs<float>&);
template size_t scan_up_lds<double>(int, int, int, int, int, int, int, int);
template size_t scan_up_lds<float>(int, int, int, int, int, int, int, int);

}  // namespace tapg
