// Solve (Algorithm 3), H^2 matrix-vector product and GMRES-based iterative
// refinement.  After factorization every rank is known on the host, so the
// solve's task lists use static window boundaries only; all instances of a
// batch share one launch per (height, colour step).
#include <algorithm>
#include <atomic>
#include <cmath>
#include <exception>
#include <thread>
#include <cstdio>
#include <cstring>
#include <functional>
#include <memory>
#include <mutex>

#include "h2_driver.h"

namespace h2drv {

using namespace h2k;

namespace {

// a skinny output is split over workgroups into chunks of about kSplitK
// contributor K (at most `maxsplit` chunks when that is set)
constexpr int64_t kSplitK = 192;
// FP32 solves and the product: fewer, longer chunks (fewer partial tiles);
// FP64 solves keep the unlimited split
constexpr int kMaxSplit = 8;
// block products with few right-hand sides use skinny tiles (K split over the
// four waves, long contributor lists over workgroups): 64 x 16 up to 16
// columns, 64 x 32 up to 64; wider blocks use 64 x 64 tiles
constexpr int kSkinnyCols = 64;
inline int product_shape(int nrhs) { return nrhs <= 16 ? 1 : nrhs <= kSkinnyCols ? 3 : 0; }
inline int tile_cols(int shape) { return (shape & 7) == 1 ? 16 : (shape & 7) == 3 ? 32 : 64; }

// Host chunks of recorded descriptor images, kept for later recordings in
// pinned memory: a fresh chunk's first touch (page faults) and a pageable
// upload cost more than the copies themselves.  At most kPoolMax chunks are
// kept; the pool lives until the process ends.
constexpr size_t kImageChunk = (size_t)64 << 20;
struct ChunkPool {
  static constexpr size_t kPoolMax = 16;
  std::mutex m;
  std::vector<char*> free;
  // a pinned chunk of kImageChunk bytes, or nullptr when none can be pinned
  char* get() {
    {
      std::lock_guard<std::mutex> g(m);
      if (!free.empty()) {
        char* p = free.back();
        free.pop_back();
        return p;
      }
    }
    void* p = nullptr;
    if (hipHostMalloc(&p, kImageChunk, hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    return static_cast<char*>(p);
  }
  void put(char* p) {
    {
      std::lock_guard<std::mutex> g(m);
      if (free.size() < kPoolMax) {
        free.push_back(p);
        return;
      }
    }
    (void)hipHostFree(p);
  }
};
ChunkPool& chunk_pool() {
  static ChunkPool* pool = new ChunkPool;  // never destroyed (outlives the runtime's users)
  return *pool;
}

// Append-only host image of descriptor arrays, each 256-byte aligned, kept in
// chunks that are never moved or zero-filled; each chunk covers a contiguous
// range of the device image it is uploaded into.  Chunks of the standard size
// come from the pinned pool and go back to it with the image.
struct HostImage {
  struct Chunk {
    char* h = nullptr;
    bool pooled = false;
    size_t dev_off = 0, used = 0, cap = 0;
  };
  std::vector<Chunk> chunks;
  size_t total = 0;
  bool use_pool = true;  // false: plain host memory only (no HIP call at all)
  HostImage() = default;
  HostImage(const HostImage&) = delete;
  HostImage& operator=(const HostImage&) = delete;
  ~HostImage() {
    for (Chunk& c : chunks) {
      if (c.pooled)
        chunk_pool().put(c.h);
      else
        delete[] c.h;
    }
  }
  bool empty() const { return total == 0; }
  size_t size() const { return total; }
  size_t append(const void* p, size_t bytes) {
    const size_t off = (total + 255) & ~(size_t)255;
    if (chunks.empty() || off - chunks.back().dev_off + bytes > chunks.back().cap) {
      Chunk c;
      if (use_pool && bytes <= kImageChunk) c.h = chunk_pool().get();
      if (c.h) {
        c.pooled = true;
        c.cap = kImageChunk;
      } else {
        c.cap = std::max(kImageChunk, bytes);
        c.h = new char[c.cap];
      }
      c.dev_off = off;
      chunks.push_back(c);
    }
    Chunk& c = chunks.back();
    std::memcpy(c.h + (off - c.dev_off), p, bytes);
    c.used = off - c.dev_off + bytes;
    total = off + bytes;
    return off;
  }
  // copy into the device image dev (at least size() bytes); with a stream the
  // copies are asynchronous and the image must outlive them
  void upload(char* dev, hipStream_t s, bool async) const {
    for (const Chunk& c : chunks) {
      if (c.used == 0) continue;
      if (async)
        H2_HIP(hipMemcpyAsync(dev + c.dev_off, c.h, c.used, hipMemcpyHostToDevice, s));
      else
        H2_HIP(hipMemcpy(dev + c.dev_off, c.h, c.used, hipMemcpyHostToDevice));
    }
  }
};

// Where a solve's launches go: straight to the stream (descriptors staged
// through the context's arena), or into a plan that later solves with the
// same factor and number of right-hand sides replay: descriptors are appended
// to a host image uploaded once, and every launch becomes a replay step that
// receives the image's device address and the plan's partial-tile scratch.
template <class T> struct Emit {
  using Step = std::function<void(hipStream_t, const char*, T*)>;
  h2_context_s* ctx = nullptr;
  hipStream_t s = nullptr;
  bool rec = false;
  HostImage img;
  std::vector<Step> steps;
  int64_t parts_need = 0;  // elements of partial-tile scratch the recorded steps use

  template <class X> size_t stage(const std::vector<X>& v) {
    return img.append(v.data(), sizeof(X) * v.size());
  }
  void strip(const std::vector<STask<T>>& t, int64_t strips, int maxn) {
    if (t.empty()) return;
    const int n = (int)t.size();
    if (!rec) {
      const STask<T>* d = ctx->arena.put(t);
      ctx->arena.flush(s);
      launch_strip<T>(d, n, nullptr, strips, maxn, s);
      return;
    }
    const size_t o = stage(t);
    steps.push_back([=](hipStream_t st, const char* b, T*) {
      launch_strip<T>(reinterpret_cast<const STask<T>*>(b + o), n, nullptr, strips, maxn, st);
    });
  }
  void trsm(const std::vector<TrsmTask<T>>& t, int maxr, int ncols) {
    if (t.empty()) return;
    const int n = (int)t.size();
    if (!rec) {
      const TrsmTask<T>* d = ctx->arena.put(t);
      ctx->arena.flush(s);
      launch_trsm<T>(d, n, nullptr, maxr, ncols, s);
      return;
    }
    const size_t o = stage(t);
    steps.push_back([=](hipStream_t st, const char* b, T*) {
      launch_trsm<T>(reinterpret_cast<const TrsmTask<T>*>(b + o), n, nullptr, maxr, ncols, st);
    });
  }
  void copy(const std::vector<CTask<T, T>>& t, int64_t tiles) {
    if (t.empty()) return;
    const int n = (int)t.size();
    if (!rec) {
      const CTask<T, T>* d = ctx->arena.put(t);
      ctx->arena.flush(s);
      launch_copy<T, T>(d, n, tiles, s);
      return;
    }
    const size_t o = stage(t);
    steps.push_back([=](hipStream_t st, const char* b, T*) {
      launch_copy<T, T>(reinterpret_cast<const CTask<T, T>*>(b + o), n, tiles, st);
    });
  }
  void gemm(const std::vector<GOut<T>>& outs, const std::vector<GCon<T>>& cons, int64_t tiles,
            int shape, int64_t ptiles, const std::vector<GOut<T>>& routs, int64_t rtiles) {
    if (outs.empty()) return;
    const int no = (int)outs.size(), nr = (int)routs.size();
    const int64_t need = ptiles * 64 * tile_cols(shape);
    if (!rec) {
      T* parts = nullptr;
      if (need > 0) {
        DevArray<T>& P = parts_of<T>(ctx);
        if (P.n < need) {
          H2_HIP(hipStreamSynchronize(s));  // earlier launches may still read it
          P.alloc(std::max(need, 2 * P.n), &ctx->tr);
        }
        parts = P.p;
      }
      const GOut<T>* dout = ctx->arena.put(outs);
      const GCon<T>* dcon = ctx->arena.put(cons);
      const GOut<T>* drout = rtiles > 0 ? ctx->arena.put(routs) : nullptr;
      ctx->arena.flush(s);
      launch_gemm<T>(dout, no, dcon, nullptr, tiles, shape, s, parts);
      if (rtiles > 0) launch_gemm_reduce<T>(drout, nr, parts, rtiles, shape, s);
      return;
    }
    const size_t oo = stage(outs), oc = stage(cons);
    const size_t orr = rtiles > 0 ? stage(routs) : 0;
    parts_need = std::max(parts_need, need);
    steps.push_back([=](hipStream_t st, const char* b, T* parts) {
      launch_gemm<T>(reinterpret_cast<const GOut<T>*>(b + oo), no,
                     reinterpret_cast<const GCon<T>*>(b + oc), nullptr, tiles, shape, st, parts);
      if (rtiles > 0)
        launch_gemm_reduce<T>(reinterpret_cast<const GOut<T>*>(b + orr), nr, parts, rtiles, shape,
                              st);
    });
  }
  void laswp(T* A, int64_t lda, int64_t ncols, int nb, const int32_t* piv) {
    if (!rec) {
      launch_laswp<T>(A, lda, ncols, 0, nb, piv, -1, -1, s);
      return;
    }
    steps.push_back([=](hipStream_t st, const char*, T*) {
      launch_laswp<T>(A, lda, ncols, 0, nb, piv, -1, -1, st);
    });
  }
  void trsm_block(const T* A, int64_t lda, T* B, int64_t ldb, int nb, int64_t ncols, int lower) {
    if (!rec) {
      launch_trsm_block<T>(A, lda, B, ldb, nb, ncols, lower, s);
      return;
    }
    steps.push_back([=](hipStream_t st, const char*, T*) {
      launch_trsm_block<T>(A, lda, B, ldb, nb, ncols, lower, st);
    });
  }
};

template <class T> struct GemmBatch {
  std::vector<GOut<T>> outs;
  std::vector<GCon<T>> cons;
  std::vector<int64_t> kss;  // contributor K of every output
  int64_t tiles = 0, ptiles = 0, rtiles = 0;
  int shape, TM, TN;
  bool pending = false;
  bool veck;    // vector loads along k (shape + 8)
  int maxsplit;  // chunks per output at most (0: no limit)
  GemmBatch(int sh, bool vk, int ms)
      : shape(sh), TM(64), TN(tile_cols(sh)), veck(vk), maxsplit(ms) {}
  // begin output C[m0:m, n0:n] = beta C + alpha sum ...
  void out(T* C, int64_t ldc, int m0, int m, int n0, int n, T alpha, T beta) {
    end();
    GOut<T> o{};
    o.C = C;
    o.ldc = ldc;
    o.m = m;
    o.n = n;
    o.m0d = -1;
    o.m0s = m0;
    o.m1d = -1;
    o.n0d = -1;
    o.n0s = n0;
    o.nsplit = 1;
    o.cbeg = o.cend = (int)cons.size();
    o.tm = std::max(0, (m - m0 + TM - 1) / TM);
    o.tn = std::max(0, (n - n0 + TN - 1) / TN);
    o.tile0 = tiles;
    o.alpha = alpha;
    o.beta = beta;
    outs.push_back(o);
    pending = true;
  }
  void con(const T* A, int64_t lda, int transA, const T* B, int64_t ldb, int k0, int k) {
    if (k <= k0) return;
    GCon<T> g{};
    g.A = A;
    g.B = B;
    g.lda = lda;
    g.ldb = ldb;
    g.k = k;
    g.k0d = -1;
    g.k0s = k0;
    g.k1d = -1;
    g.transA = transA;
    cons.push_back(g);
    outs.back().cend = (int)cons.size();
  }
  // close the current output (drops it when it has no tiles); its split is
  // chosen at launch
  void end() {
    if (!pending) return;
    pending = false;
    GOut<T>& o = outs.back();
    const int64_t t = (int64_t)o.tm * o.tn;
    if (t == 0) {
      cons.resize(o.cbeg);
      outs.pop_back();
      return;
    }
    int64_t ks = 0;
    for (int c = o.cbeg; c < o.cend; ++c) ks += cons[c].k - cons[c].k0s;
    kss.push_back(ks);
  }
  // tiles, partial tiles and reduction tiles of every output: skinny outputs
  // with a long contributor list are cut into chunks (the choice depends on
  // the output alone, so batched and single launches round alike)
  void split() {
    tiles = ptiles = rtiles = 0;
    for (size_t q = 0; q < outs.size(); ++q) {
      GOut<T>& o = outs[q];
      const int64_t t = (int64_t)o.tm * o.tn;
      int ns = 1;
      if (shape == 1 || shape == 3) {
        int64_t m = std::min<int64_t>(o.cend - o.cbeg, (kss[q] + kSplitK - 1) / kSplitK);
        if (maxsplit > 0) m = std::min<int64_t>(m, maxsplit);
        ns = (int)std::max<int64_t>(1, m);
      }
      o.nsplit = ns;
      o.tile0 = tiles;
      tiles += t * ns;
      if (ns > 1) {
        o.part0 = ptiles;
        ptiles += t * ns;
        o.rtile0 = rtiles;
        rtiles += t;
      }
    }
  }
  void launch(Emit<T>& em) {
    end();
    if (outs.empty()) return;
    split();
    std::vector<GOut<T>> routs;
    for (auto& o : outs)
      if (o.nsplit > 1) routs.push_back(o);
    em.gemm(outs, cons, tiles, (shape == 1 || shape == 3) && veck ? shape + 8 : shape, ptiles,
            routs, rtiles);
    outs.clear();
    cons.clear();
    kss.clear();
    tiles = ptiles = rtiles = 0;
  }
};

template <class T> struct StripBatch {
  std::vector<STask<T>> tasks;
  int64_t strips = 0;
  int maxn = 1;
  void add(T* X, int64_t ldx, const T* Q, int n, int ext, int side, int trans) {
    if (n <= 0 || ext <= 0) return;
    STask<T> t{};
    t.X = X;
    t.Q = Q;
    t.ldx = ldx;
    t.n = n;
    t.ext = ext;
    t.d0 = -1;
    t.s0 = 0;
    t.side = side;
    t.trans = trans;
    t.strip0 = strips;
    strips += (ext + kStrip - 1) / kStrip;
    maxn = std::max(maxn, n);
    tasks.push_back(t);
  }
  void launch(Emit<T>& em) {
    if (tasks.empty()) return;
    em.strip(tasks, strips, maxn);
    tasks.clear();
    strips = 0;
    maxn = 1;
  }
};

template <class T> struct CopyB {
  std::vector<CTask<T, T>> tasks;
  int64_t tiles = 0;
  void add(const T* src, int64_t lds, T* dst, int64_t ldd, int rows, int cols) {
    if (rows <= 0 || cols <= 0) return;
    CTask<T, T> t{};
    t.src = src;
    t.dst = dst;
    t.lds = lds;
    t.ldd = ldd;
    t.rows = rows;
    t.cols = cols;
    t.add = 0;
    t.tile0 = tiles;
    tiles += ((int64_t)rows * cols + kCopyTile - 1) / kCopyTile;
    tasks.push_back(t);
  }
  void launch(Emit<T>& em) {
    if (tasks.empty()) return;
    em.copy(tasks, tiles);
    tasks.clear();
    tiles = 0;
  }
};

template <class T> LevelStore<T>& store(h2_factor_s* F, size_t li);
template <> LevelStore<double>& store<double>(h2_factor_s* F, size_t li) { return F->st64[li]; }
template <> LevelStore<float>& store<float>(h2_factor_s* F, size_t li) { return F->st32[li]; }
template <class T> DevArray<T>& topM(h2_factor_s* F);
template <> DevArray<double>& topM<double>(h2_factor_s* F) { return F->M64; }
template <> DevArray<float>& topM<float>(h2_factor_s* F) { return F->M32; }

// per-instance solve state
template <class T> struct SolveInst {
  h2_factor_s* F;
  std::vector<DevArray<T>> vec;  // level vectors (leaf level first), plus the top vector
  std::vector<std::vector<int64_t>> voff;
  std::vector<int64_t> vlen;
};

// Work vectors of one instance: per level the cluster segments (leaf level
// first), then the top vector.
template <class T>
void solve_setup(SolveInst<T>& S, h2_factor_s* F, int nrhs, DevTracker* tr) {
  S.F = F;
  const size_t nlev = F->plans.size();
  S.vec = std::vector<DevArray<T>>(nlev + 1);
  S.voff.assign(nlev + 1, {});
  S.vlen.assign(nlev + 1, 0);
  for (size_t li = 0; li < nlev; ++li) {
    const LevelPlan& P = F->plans[li];
    S.voff[li].resize(P.nl);
    int64_t o = 0;
    for (int i = 0; i < P.nl; ++i) {
      S.voff[li][i] = o;
      o += P.n[i];
    }
    S.vlen[li] = o;
    S.vec[li].alloc(std::max<int64_t>(o, 1) * nrhs, tr);
  }
  S.voff[nlev] = F->top_off;
  S.vlen[nlev] = F->n_top;
  S.vec[nlev].alloc(std::max<int64_t>(F->n_top, 1) * nrhs, tr);
}

// one colour's solve tasks (built on a worker thread, emitted in order)
template <class T> struct ColourTasks {
  StripBatch<T> sb;
  std::vector<TrsmTask<T>> trs;
  GemmBatch<T> gb;
  // FP32 products read k-contiguous operands as vectors; FP64 solves keep
  // the ascending k order and the finer split
  explicit ColourTasks(int shape) : gb(shape, sizeof(T) == 4, sizeof(T) == 4 ? kMaxSplit : 0) {}
};

// f(0) .. f(n - 1) on up to 16 threads (the calling thread included), each
// taking the next index
template <class Fn> void parallel_for(int n, Fn f) {
  const int nt = (int)std::max(1u, std::min({16u, std::thread::hardware_concurrency(),
                                             (unsigned)std::max(n, 1)}));
  std::atomic<int> next(0);
  std::vector<std::exception_ptr> errs(nt);
  auto run = [&](int t) {
    try {
      for (int q; (q = next.fetch_add(1)) < n;) f(q);
    } catch (...) {
      errs[t] = std::current_exception();
    }
  };
  std::vector<std::thread> th;
  for (int t = 1; t < nt; ++t) th.emplace_back(run, t);
  run(0);
  for (auto& x : th) x.join();
  for (auto& e : errs)
    if (e) std::rethrow_exception(e);
}

// Algorithm 3 on the work vectors (the right-hand sides already gathered in
// tree order into vec[0]): forward colour by colour and level by level, the
// dense top solve, then backward.
template <class T>
void solve_body(Emit<T>& em, std::vector<SolveInst<T>>& si, int nrhs) {
  const int shape = product_shape(nrhs);
  size_t maxlev = 0;
  for (auto& S : si) maxlev = std::max(maxlev, S.F->plans.size());
  // ---- forward, level by level from the leaves ----
  for (size_t li = 0; li < maxlev; ++li) {
    int maxc = 0;
    for (auto& S : si)
      if (li < S.F->plans.size()) maxc = std::max(maxc, S.F->plans[li].ncolors);
    // each colour's task lists are built on worker threads, then emitted in
    // colour order
    std::vector<ColourTasks<T>> ct;
    ct.reserve(maxc);
    for (int c = 0; c < maxc; ++c) ct.emplace_back(shape);
    parallel_for(maxc, [&](int c) {
      StripBatch<T>& sb = ct[c].sb;
      std::vector<TrsmTask<T>>& trs = ct[c].trs;
      GemmBatch<T>& gb = ct[c].gb;
      for (auto& S : si) {
        h2_factor_s* F = S.F;
        if (li >= F->plans.size()) continue;
        const LevelPlan& P = F->plans[li];
        if (c >= P.ncolors) continue;
        LevelStore<T>& st = store<T>(F, li);
        T* v = S.vec[li].p;
        const int64_t ld = S.vlen[li];
        for (int i : P.members[c]) {
          sb.add(v + S.voff[li][i], ld, st.Q.p + P.offQ[i], P.n[i], nrhs, 0, 1);
          if (P.r[i] > 0) {
            TrsmTask<T> t{};
            t.LU = st.D.p + P.poff[P.find(i, i)];
            t.piv = st.piv.p + P.offPiv[i];
            t.B = v + S.voff[li][i];
            t.ldlu = P.n[i];
            t.ldb = ld;
            t.ncols = nrhs;
            t.ri = -1;
            t.rs = P.r[i];
            t.c0d = -1;
            t.c0s = 0;
            trs.push_back(t);
          }
        }
        // b_j[active rows] -= D_{j,R_i} z_i, grouped by target j
        std::vector<std::pair<int, int>> inc;  // (j, i)
        for (int i : P.members[c])
          if (P.r[i] > 0)
            for (int j : P.nb[i]) inc.push_back({j, i});
        std::sort(inc.begin(), inc.end());
        for (size_t a = 0; a < inc.size();) {
          size_t b = a;
          const int j = inc[a].first;
          const int aj = P.color[j] <= c ? P.r[j] : 0;
          gb.out(v + S.voff[li][j], ld, aj, P.n[j], 0, nrhs, T(-1), T(1));
          for (; b < inc.size() && inc[b].first == j; ++b) {
            const int i = inc[b].second;
            gb.con(st.D.p + P.poff[P.find(j, i)], P.n[j], 0, v + S.voff[li][i], ld, 0, P.r[i]);
          }
          gb.end();
          a = b;
        }
      }
    });
    for (int c = 0; c < maxc; ++c) {
      ct[c].sb.launch(em);
      std::vector<TrsmTask<T>>& trs = ct[c].trs;
      if (!trs.empty()) {
        int maxr = 1;
        for (auto& t : trs) maxr = std::max(maxr, t.rs);
        em.trsm(trs, maxr, nrhs);
      }
      ct[c].gb.launch(em);
    }
    // upsweep: skeleton parts of the children form the parent segments
    CopyB<T> cb;
    for (auto& S : si) {
      h2_factor_s* F = S.F;
      if (li >= F->plans.size()) continue;
      const LevelPlan& P = F->plans[li];
      const size_t nx = li + 1;  // next vector (a level or the top)
      const bool top = nx == F->plans.size();
      const int pa = F->lp[P.lev - 1];
      T* v = S.vec[li].p;
      T* w = S.vec[nx].p;
      const int64_t ldv = S.vlen[li], ldw = S.vlen[nx];
      for (int t = 0; t < F->lp[P.lev] - pa; ++t) {
        const int tau = pa + t;
        int64_t o = top ? F->top_off[t] : S.voff[nx][t];
        for (int cc = F->cp[tau]; cc < F->cp[tau + 1]; ++cc) {
          const int c = cc - P.a;
          const int kt = P.n[c] - P.r[c];
          cb.add(v + S.voff[li][c] + P.r[c], ldv, w + o, ldw, kt, nrhs);
          o += kt;
        }
      }
    }
    cb.launch(em);
  }
  // ---- dense top solve ----
  for (auto& S : si) {
    h2_factor_s* F = S.F;
    const int64_t n = F->n_top;
    if (n == 0) continue;
    const size_t nx = F->plans.size();
    if (nx == 0) {
      // no skeletonized level: b (tree order) is the top vector
      // (vec[0] was allocated with the top size and received the gather)
    }
    T* b = S.vec[nx].p;
    const int64_t ldb2 = S.vlen[nx];
    T* M = topM<T>(F).p;
    em.laswp(b, ldb2, nrhs, (int)n, F->top_piv.p);
    const int nb = 64;
    for (int64_t j0 = 0; j0 < n; j0 += nb) {
      const int w = (int)std::min<int64_t>(nb, n - j0);
      em.trsm_block(M + j0 + j0 * n, n, b + j0, ldb2, w, nrhs, 1);
      if (j0 + w < n) {
        GemmBatch<T> gb(shape, sizeof(T) == 4, sizeof(T) == 4 ? kMaxSplit : 0);
        gb.out(b + j0 + w, ldb2, 0, (int)(n - j0 - w), 0, nrhs, T(-1), T(1));
        gb.con(M + (j0 + w) + j0 * n, n, 0, b + j0, ldb2, 0, w);
        gb.launch(em);
      }
    }
    for (int64_t j0 = ((n - 1) / nb) * nb; j0 >= 0; j0 -= nb) {
      const int w = (int)std::min<int64_t>(nb, n - j0);
      em.trsm_block(M + j0 + j0 * n, n, b + j0, ldb2, w, nrhs, 0);
      if (j0 > 0) {
        GemmBatch<T> gb(shape, sizeof(T) == 4, sizeof(T) == 4 ? kMaxSplit : 0);
        gb.out(b, ldb2, 0, (int)j0, 0, nrhs, T(-1), T(1));
        gb.con(M + j0 * n, n, 0, b + j0, ldb2, 0, w);
        gb.launch(em);
      }
    }
  }
  // ---- backward, from the top level down ----
  for (size_t lj = maxlev; lj-- > 0;) {
    // downsweep into level vectors whose instance has level lj
    CopyB<T> cb;
    for (auto& S : si) {
      h2_factor_s* F = S.F;
      if (lj >= F->plans.size()) continue;
      const LevelPlan& P = F->plans[lj];
      const size_t nx = lj + 1;
      const bool top = nx == F->plans.size();
      const int pa = F->lp[P.lev - 1];
      T* v = S.vec[lj].p;
      T* w = S.vec[nx].p;
      const int64_t ldv = S.vlen[lj], ldw = S.vlen[nx];
      for (int t = 0; t < F->lp[P.lev] - pa; ++t) {
        const int tau = pa + t;
        int64_t o = top ? F->top_off[t] : S.voff[nx][t];
        for (int cc = F->cp[tau]; cc < F->cp[tau + 1]; ++cc) {
          const int c = cc - P.a;
          const int kt = P.n[c] - P.r[c];
          cb.add(w + o, ldw, v + S.voff[lj][c] + P.r[c], ldv, kt, nrhs);
          o += kt;
        }
      }
    }
    cb.launch(em);
    int maxc = 0;
    for (auto& S : si)
      if (lj < S.F->plans.size()) maxc = std::max(maxc, S.F->plans[lj].ncolors);
    std::vector<ColourTasks<T>> ct;
    ct.reserve(maxc);
    for (int c = 0; c < maxc; ++c) ct.emplace_back(shape);
    parallel_for(maxc, [&](int c) {
      GemmBatch<T>& gb = ct[c].gb;
      StripBatch<T>& sb = ct[c].sb;
      for (auto& S : si) {
        h2_factor_s* F = S.F;
        if (lj >= F->plans.size()) continue;
        const LevelPlan& P = F->plans[lj];
        if (c >= P.ncolors) continue;
        LevelStore<T>& st = store<T>(F, lj);
        T* v = S.vec[lj].p;
        const int64_t ld = S.vlen[lj];
        for (int i : P.members[c]) {
          if (P.r[i] > 0) {
            // y_iR -= sum_k Y_k y_k over the columns active when i was eliminated
            gb.out(v + S.voff[lj][i], ld, 0, P.r[i], 0, nrhs, T(-1), T(1));
            for (int k : P.nb[i]) {
              const int ak = P.color[k] <= c ? P.r[k] : 0;
              gb.con(st.D.p + P.poff[P.find(i, k)], P.n[i], 0, v + S.voff[lj][k], ld, ak,
                     P.n[k]);
            }
            gb.end();
          }
          sb.add(v + S.voff[lj][i], ld, st.Q.p + P.offQ[i], P.n[i], nrhs, 0, 0);
        }
      }
    });
    for (int c = maxc - 1; c >= 0; --c) {
      ct[c].gb.launch(em);
      ct[c].sb.launch(em);
    }
  }
}

// A recorded launch sequence: the descriptors in one device image, each
// launch a replay step.  The first use replays the steps launch by launch;
// the second captures them as one HIP graph (kernel nodes only) and later
// uses launch the graph.  If the runtime refuses the capture, the steps keep
// being replayed one by one.
template <class T> struct Replay {
  DevArray<char> img;  // recorded descriptors
  DevArray<T> parts;   // partial tiles of split products
  std::vector<typename Emit<T>::Step> steps;
  hipGraphExec_t gexec = nullptr;
  bool graph_failed = false;
  int64_t uses = 0, graph_uses = 0;
  ~Replay() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
  }
  void take(Emit<T>& em, DevTracker* tr) {
    img.alloc(std::max<int64_t>((int64_t)em.img.size(), 1), tr);
    em.img.upload(img.p, nullptr, false);
    if (em.parts_need > 0) parts.alloc(em.parts_need, tr);
    steps = std::move(em.steps);
  }
  // capture the replay of the steps on stream s; false if the runtime refuses
  bool capture(hipStream_t s) {
    if (hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed) != hipSuccess) {
      (void)hipGetLastError();
      return false;
    }
    for (auto& st : steps) st(s, img.p, parts.p);
    hipGraph_t g = nullptr;
    if (hipStreamEndCapture(s, &g) != hipSuccess || g == nullptr) {
      (void)hipGetLastError();
      return false;
    }
    const hipError_t e = hipGraphInstantiate(&gexec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      gexec = nullptr;
      return false;
    }
    return true;
  }
  void run(hipStream_t s) {
    if (uses > 0 && !gexec && !graph_failed) graph_failed = !capture(s);
    if (gexec) {
      H2_HIP(hipGraphLaunch(gexec, s));
      ++graph_uses;
    } else {
      for (auto& st : steps) st(s, img.p, parts.p);
    }
    ++uses;
  }
};

template <class T> struct SolvePlan : PlanBase {
  int nrhs = 0;
  SolveInst<T> S;
  Replay<T> rp;
  int64_t uses() const override { return rp.uses; }
  int64_t graph_uses() const override { return rp.graph_uses; }
};

template <class T>
void run_solve(h2_context_s* ctx, const std::vector<h2_factor_s*>& Fs,
               const std::vector<const double*>& B, const std::vector<int64_t>& ldb, int nrhs,
               const std::vector<double*>& X, const std::vector<int64_t>& ldx) {
  hipStream_t s = ctx->stream;
  DescArena& ar = ctx->arena;
  ar.s = s;
  if (Fs.size() == 1) {
    // one factor: the launch sequence depends only on the factor and nrhs, so
    // it is recorded once and replayed by later solves
    h2_factor_s* F = Fs[0];
    auto* plan = dynamic_cast<SolvePlan<T>*>(F->splan.get());
    if (!plan || plan->nrhs != nrhs) {
      F->splan.reset();
      auto np = std::make_unique<SolvePlan<T>>();
      np->nrhs = nrhs;
      solve_setup<T>(np->S, F, nrhs, &F->tr);
      Emit<T> em;
      em.ctx = ctx;
      em.s = s;
      em.rec = true;
      std::vector<SolveInst<T>> one(1);
      std::swap(one[0], np->S);
      solve_body<T>(em, one, nrhs);
      std::swap(one[0], np->S);
      np->rp.take(em, &F->tr);
      plan = np.get();
      F->splan = std::move(np);
    }
    SolveInst<T>& S = plan->S;
    launch_gather_rows<T, double>(S.vec[0].p, S.vlen[0], B[0], ldb[0], F->perm_d.p, F->N, nrhs, s);
    plan->rp.run(s);
    launch_scatter_rows<double, T>(X[0], ldx[0], S.vec[0].p, S.vlen[0], F->perm_d.p, F->N, nrhs,
                                   s);
    H2_HIP(hipStreamSynchronize(s));
    return;
  }
  std::vector<SolveInst<T>> si(Fs.size());
  for (size_t q = 0; q < Fs.size(); ++q) {
    solve_setup<T>(si[q], Fs[q], nrhs, &ctx->tr);
    launch_gather_rows<T, double>(si[q].vec[0].p, si[q].vlen[0], B[q], ldb[q], Fs[q]->perm_d.p,
                                  Fs[q]->N, nrhs, s);
  }
  Emit<T> em;
  em.ctx = ctx;
  em.s = s;
  solve_body<T>(em, si, nrhs);
  for (size_t q = 0; q < Fs.size(); ++q) {
    SolveInst<T>& S = si[q];
    launch_scatter_rows<double, T>(X[q], ldx[q], S.vec[0].p, S.vlen[0], S.F->perm_d.p, S.F->N,
                                   nrhs, s);
  }
  H2_HIP(hipStreamSynchronize(s));
  ar.reset();
}

}  // namespace

void solve(h2_context_s* ctx, const std::vector<h2_factor_s*>& Fs,
           const std::vector<const double*>& B, const std::vector<int64_t>& ldb, int nrhs,
           const std::vector<double*>& X, const std::vector<int64_t>& ldx) {
  if (Fs[0]->prec == H2_PREC_FP64)
    run_solve<double>(ctx, Fs, B, ldb, nrhs, X, ldx);
  else
    run_solve<float>(ctx, Fs, B, ldb, nrhs, X, ldx);
}

// ---------------------------------------------------------------------------
// FP64 H^2 matvec: permute, upsweep U^T / E^T, couplings, downsweep E,
// leaf bases U plus dense near blocks, permute back.
// ---------------------------------------------------------------------------
namespace {

// per node offsets into the upsweep / downsweep coefficient vectors
void matvec_layout(h2_matrix_s* H) {
  if (H->mv_ready) return;
  H->hat_off.assign(H->nn, 0);
  int64_t o = 0;
  for (int q = 0; q < H->nn; ++q) {
    H->hat_off[q] = o;
    o += H->rank[q];
  }
  H->hat_total = o;
  H->mv_ready = true;
}

// The product's launches on tree-ordered work vectors: xt (N x nrhs) in,
// yt out, xh / yh the basis coefficients (hat_total x nrhs).
void matvec_body(Emit<double>& em, const h2_matrix_s* H, const double* xt, double* yt, double* xh,
                 double* yh, int nrhs) {
  const int shape = product_shape(nrhs);
  const int64_t N = H->N;
  const double* d = H->data.p;
  auto hx = [&](int q) { return xh + H->hat_off[q] * nrhs; };
  auto hy = [&](int q) { return yh + H->hat_off[q] * nrhs; };
  const int L = H->L;
  if (H->top >= 0) {
    // leaves: xh = U^T x
    GemmBatch<double> gb(shape, true, kMaxSplit);
    for (int q = H->lp[L]; q < H->nn; ++q) {
      if (!H->rank[q]) continue;
      gb.out(hx(q), H->rank[q], 0, H->rank[q], 0, nrhs, 1.0, 0.0);
      gb.con(d + H->offU[q], H->size(q), 1, xt + H->ib[q], N, 0, H->size(q));
      gb.end();
    }
    gb.launch(em);
    for (int l = L - 1; l >= H->top; --l) {
      for (int q = H->lp[l]; q < H->lp[l + 1]; ++q) {
        if (!H->rank[q]) continue;
        gb.out(hx(q), H->rank[q], 0, H->rank[q], 0, nrhs, 1.0, 0.0);
        for (int c = H->cp[q]; c < H->cp[q + 1]; ++c)
          if (H->rank[c]) gb.con(d + H->offE[c], H->rank[c], 1, hx(c), H->rank[c], 0, H->rank[c]);
        gb.end();
      }
      gb.launch(em);
    }
    // couplings
    for (int q = 0; q < H->nn; ++q) {
      if (!H->rank[q]) continue;
      gb.out(hy(q), H->rank[q], 0, H->rank[q], 0, nrhs, 1.0, 0.0);
      for (int64_t e = H->far_ptr[q]; e < H->far_ptr[q + 1]; ++e) {
        const int j = H->far_col[e];
        if (H->rank[j]) gb.con(d + H->offS[e], H->rank[q], 0, hx(j), H->rank[j], 0, H->rank[j]);
      }
      gb.end();
    }
    gb.launch(em);
    for (int l = H->top + 1; l <= L; ++l) {
      for (int q = H->lp[l]; q < H->lp[l + 1]; ++q) {
        const int p = H->parent[q];
        if (!H->rank[q] || !H->rank[p]) continue;
        gb.out(hy(q), H->rank[q], 0, H->rank[q], 0, nrhs, 1.0, 1.0);
        gb.con(d + H->offE[q], H->rank[q], 0, hy(p), H->rank[p], 0, H->rank[p]);
        gb.end();
      }
      gb.launch(em);
    }
  }
  GemmBatch<double> gb(shape, true, kMaxSplit);
  for (int q = H->lp[L]; q < H->nn; ++q) {
    gb.out(yt + H->ib[q], N, 0, H->size(q), 0, nrhs, 1.0, 0.0);
    if (H->top >= 0 && H->rank[q])
      gb.con(d + H->offU[q], H->size(q), 0, hy(q), H->rank[q], 0, H->rank[q]);
    for (int64_t e = H->near_ptr[q]; e < H->near_ptr[q + 1]; ++e) {
      const int j = H->near_col[e];
      gb.con(d + H->offD[e], H->size(q), 0, xt + H->ib[j], N, 0, H->size(j));
    }
    gb.end();
  }
  gb.launch(em);
}

struct MatvecPlan : PlanBase {
  int nrhs = 0;
  DevArray<double> xt, yt, xh, yh;
  Replay<double> rp;
  int64_t uses() const override { return rp.uses; }
  int64_t graph_uses() const override { return rp.graph_uses; }
};

}  // namespace

// ---------------------------------------------------------------------------
// FP64 H^2 matvec: permute, upsweep U^T / E^T, couplings, downsweep E,
// leaf bases U plus dense near blocks, permute back.  The launch sequence is
// recorded once per (matrix, nrhs) with its work vectors and replayed (as one
// graph from the second call on).
// ---------------------------------------------------------------------------
void matvec(h2_context_s* ctx, h2_matrix_s* H, const double* X, int64_t ldx, int nrhs, double* Y,
            int64_t ldy) {
  hipStream_t s = ctx->stream;
  matvec_layout(H);
  auto* plan = dynamic_cast<MatvecPlan*>(H->mvplan.get());
  if (!plan || plan->nrhs != nrhs) {
    H->mvplan.reset();
    auto np = std::make_unique<MatvecPlan>();
    np->nrhs = nrhs;
    const int64_t N = H->N;
    np->xt.alloc(N * nrhs, &H->tr);
    np->yt.alloc(N * nrhs, &H->tr);
    np->xh.alloc(std::max<int64_t>(H->hat_total, 1) * nrhs, &H->tr);
    np->yh.alloc(std::max<int64_t>(H->hat_total, 1) * nrhs, &H->tr);
    Emit<double> em;
    em.ctx = ctx;
    em.s = s;
    em.rec = true;
    matvec_body(em, H, np->xt.p, np->yt.p, np->xh.p, np->yh.p, nrhs);
    np->rp.take(em, &H->tr);
    plan = np.get();
    H->mvplan = std::move(np);
  }
  launch_gather_rows<double, double>(plan->xt.p, H->N, X, ldx, H->perm_d.p, H->N, nrhs, s);
  plan->rp.run(s);
  launch_scatter_rows<double, double>(Y, ldy, plan->yt.p, H->N, H->perm_d.p, H->N, nrhs, s);
}

// The product with every work array in caller-provided device memory
// `scratch` of `cap` bytes (256-byte aligned): [xt | yt | xh | yh | the
// descriptor image | partial tiles].  Allocates no device memory; the
// descriptors are recorded on the host and copied in.  Synchronizes before
// returning.
void matvec_in(h2_context_s* ctx, h2_matrix_s* H, const double* X, int64_t ldx, int nrhs,
               double* Y, int64_t ldy, char* scratch, int64_t cap) {
  hipStream_t s = ctx->stream;
  matvec_layout(H);
  auto up = [](int64_t b) { return (b + 255) & ~(int64_t)255; };
  const int64_t N = H->N, nh = std::max<int64_t>(H->hat_total, 1);
  const int64_t vec = up(8 * (2 * N + 2 * nh) * nrhs);
  if (vec > cap)
    throw H2Error(H2_ERROR_UNSUPPORTED, "the product's vectors need " + std::to_string(vec) +
                                            " bytes of scratch, more than the " +
                                            std::to_string(cap) + " available");
  double* xt = reinterpret_cast<double*>(scratch);
  double* yt = xt + N * nrhs;
  double* xh = yt + N * nrhs;
  double* yh = xh + nh * nrhs;
  Emit<double> em;
  em.ctx = ctx;
  em.s = s;
  em.rec = true;
  em.img.use_pool = false;  // no pinned allocation on this path
  matvec_body(em, H, xt, yt, xh, yh, nrhs);
  const int64_t img = up((int64_t)em.img.size());
  const int64_t need = vec + img + 8 * em.parts_need;
  if (need > cap)
    throw H2Error(H2_ERROR_UNSUPPORTED, "the product needs " + std::to_string(need) +
                                            " bytes of scratch, more than the " +
                                            std::to_string(cap) + " available");
  char* dimg = scratch + vec;
  double* parts = reinterpret_cast<double*>(dimg + img);
  em.img.upload(dimg, s, true);
  launch_gather_rows<double, double>(xt, N, X, ldx, H->perm_d.p, N, nrhs, s);
  for (auto& st : em.steps) st(s, dimg, parts);
  launch_scatter_rows<double, double>(Y, ldy, yt, N, H->perm_d.p, N, nrhs, s);
  // the host image must outlive its copy
  H2_HIP(hipStreamSynchronize(s));
}

// ---------------------------------------------------------------------------
// GMRES-IR: residuals, Krylov basis and updates in FP64; the preconditioner is
// the factor's solve (FP32 or FP64).  Columns share the iteration.
// ---------------------------------------------------------------------------
bool solve_ir(h2_context_s* ctx, h2_matrix_s* H, h2_factor_s* F, const double* B, int64_t ldb,
              int nrhs, double* X, int64_t ldx, const h2_ir_opts& o, h2_ir_report& rep) {
  hipStream_t s = ctx->stream;
  const int64_t N = H->N;
  const int m = o.restart;
  auto precond = [&](const double* in, double* out) {
    solve(ctx, {F}, {in}, {N}, nrhs, {out}, {N});
  };
  auto A = [&](const double* in, double* out) { matvec(ctx, H, in, in == X ? ldx : N, nrhs, out, N); };
  DevArray<double> R, T1, Vb, coef, nrm;
  R.alloc(N * nrhs, &ctx->tr);
  T1.alloc(N * nrhs, &ctx->tr);
  Vb.alloc((int64_t)(m + 1) * N * nrhs, &ctx->tr);
  coef.alloc((int64_t)(m + 2) * nrhs, &ctx->tr);
  nrm.alloc(2 * (int64_t)nrhs, &ctx->tr);
  const int64_t vs = N * nrhs;  // stride between basis vectors
  std::vector<double> bnorm(nrhs), h(nrhs), hcol((size_t)(m + 1) * nrhs);
  // x0 = M^{-1} b
  DevArray<double> Bc;
  Bc.alloc(N * nrhs, &ctx->tr);
  H2_HIP(hipMemcpy2DAsync(Bc.p, N * 8, B, ldb * 8, N * 8, nrhs, hipMemcpyDeviceToDevice, s));
  precond(Bc.p, T1.p);
  H2_HIP(hipMemcpy2DAsync(X, ldx * 8, T1.p, N * 8, N * 8, nrhs, hipMemcpyDeviceToDevice, s));
  launch_colnorms(Bc.p, N, N, nrhs, nrm.p, s);
  H2_HIP(hipMemcpyAsync(bnorm.data(), nrm.p, 8 * nrhs, hipMemcpyDeviceToHost, s));
  H2_HIP(hipStreamSynchronize(s));
  rep = h2_ir_report{};
  auto residual = [&]() {
    // R = B - A X; returns max backward error
    A(X, T1.p);
    launch_sub(R.p, N, Bc.p, N, T1.p, N, N, nrhs, s);
    launch_colnorms(R.p, N, N, nrhs, nrm.p, s);
    std::vector<double> rn(nrhs);
    H2_HIP(hipMemcpyAsync(rn.data(), nrm.p, 8 * nrhs, hipMemcpyDeviceToHost, s));
    H2_HIP(hipStreamSynchronize(s));
    double e = 0;
    for (int c = 0; c < nrhs; ++c) e = std::max(e, bnorm[c] > 0 ? rn[c] / bnorm[c] : rn[c]);
    return e;
  };
  double eb = residual();
  int outer = 0;
  while (eb > o.target_bkwd && outer < o.max_outer) {
    ++outer;
    // z = M^{-1} r, beta = ||z||, v0 = z / beta
    precond(R.p, T1.p);
    launch_colnorms(T1.p, N, N, nrhs, nrm.p, s);
    std::vector<double> beta(nrhs);
    H2_HIP(hipMemcpyAsync(beta.data(), nrm.p, 8 * nrhs, hipMemcpyDeviceToHost, s));
    launch_scale_cols(Vb.p, N, T1.p, N, nrm.p, N, nrhs, 1, s);
    H2_HIP(hipStreamSynchronize(s));
    // per-column Hessenberg / Givens state
    std::vector<std::vector<double>> Hh(nrhs, std::vector<double>((size_t)(m + 1) * m, 0.0));
    std::vector<std::vector<double>> g(nrhs, std::vector<double>(m + 1, 0.0)), cs(nrhs), sn(nrhs);
    for (int c = 0; c < nrhs; ++c) {
      g[c][0] = beta[c];
      cs[c].assign(m, 0);
      sn[c].assign(m, 0);
    }
    int kdone = 0;
    for (int k = 0; k < m; ++k) {
      double* vk = Vb.p + k * vs;
      double* w = Vb.p + (k + 1) * vs;
      A(vk, T1.p);
      precond(T1.p, w);
      // CGS2 against v_0..v_k
      std::vector<double> hk((size_t)(k + 1) * nrhs, 0.0), tmp((size_t)(k + 1) * nrhs);
      for (int pass = 0; pass < 2; ++pass) {
        launch_dots(Vb.p, N, vs, k + 1, w, N, N, nrhs, coef.p, s);
        launch_update(w, N, Vb.p, N, vs, k + 1, coef.p, -1.0, N, nrhs, s);
        H2_HIP(hipMemcpyAsync(tmp.data(), coef.p, 8 * (k + 1) * nrhs, hipMemcpyDeviceToHost, s));
        H2_HIP(hipStreamSynchronize(s));
        for (size_t e = 0; e < tmp.size(); ++e) hk[e] += tmp[e];
      }
      launch_colnorms(w, N, N, nrhs, nrm.p, s);
      std::vector<double> hn(nrhs);
      H2_HIP(hipMemcpyAsync(hn.data(), nrm.p, 8 * nrhs, hipMemcpyDeviceToHost, s));
      launch_scale_cols(w, N, w, N, nrm.p, N, nrhs, 1, s);
      H2_HIP(hipStreamSynchronize(s));
      bool all_done = true;
      for (int c = 0; c < nrhs; ++c) {
        double* col = &Hh[c][(size_t)k * (m + 1)];
        for (int i = 0; i <= k; ++i) col[i] = hk[i + (size_t)c * (k + 1)];
        col[k + 1] = hn[c];
        for (int i = 0; i < k; ++i) {
          const double a = col[i], b = col[i + 1];
          col[i] = cs[c][i] * a + sn[c][i] * b;
          col[i + 1] = -sn[c][i] * a + cs[c][i] * b;
        }
        const double a = col[k], b = col[k + 1];
        const double den = std::hypot(a, b);
        cs[c][k] = den == 0 ? 1.0 : a / den;
        sn[c][k] = den == 0 ? 0.0 : b / den;
        col[k] = cs[c][k] * a + sn[c][k] * b;
        col[k + 1] = 0;
        g[c][k + 1] = -sn[c][k] * g[c][k];
        g[c][k] = cs[c][k] * g[c][k];
        if (std::fabs(g[c][k + 1]) > o.inner_rtol * beta[c] && hn[c] > 0) all_done = false;
      }
      kdone = k + 1;
      rep.inner_iterations++;
      if (all_done) break;
    }
    // back substitution per column, then x += V y
    std::vector<double> y((size_t)kdone * nrhs, 0.0);
    for (int c = 0; c < nrhs; ++c) {
      for (int i = kdone - 1; i >= 0; --i) {
        double acc = g[c][i];
        for (int j = i + 1; j < kdone; ++j) acc -= Hh[c][(size_t)j * (m + 1) + i] * y[j + (size_t)c * kdone];
        const double dii = Hh[c][(size_t)i * (m + 1) + i];
        y[i + (size_t)c * kdone] = dii != 0 ? acc / dii : 0.0;
      }
    }
    H2_HIP(hipMemcpyAsync(coef.p, y.data(), 8 * y.size(), hipMemcpyHostToDevice, s));
    launch_update(X, ldx, Vb.p, N, vs, kdone, coef.p, 1.0, N, nrhs, s);
    H2_HIP(hipStreamSynchronize(s));
    eb = residual();
  }
  rep.outer_iterations = outer;
  rep.max_bkwd = eb;
  return eb <= o.target_bkwd;
}

}  // namespace h2drv
