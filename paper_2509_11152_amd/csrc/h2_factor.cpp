// Factorization driver: strong recursive skeletonization level by level
// (Algorithm 1), colour by colour (Algorithm 2), batched over instances.
//
// Per tree level the host plans everything that depends only on structure and
// on the sizes n_i of the level (colours, fill pattern, block layout, task
// lists); ranks are decided on the device and read by the kernels through the
// level's r array, so a level runs without host synchronisation.  The host
// synchronises once per level to read the ranks, which fix the sizes of the
// next level (n_tau = sum of the children's k~).
#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstdio>
#include <deque>
#include <exception>
#include <future>
#include <memory>
#include <numeric>
#include <thread>
#include <tuple>

#include "h2_driver.h"

namespace h2drv {

using namespace h2k;

namespace {

uint64_t node_hash(uint64_t z) {
  // SplitMix64 output finaliser (Steele, Lea, Flood, OOPSLA 2014)
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

// f(lo, hi) over [0, n) split into contiguous ranges on up to 8 threads (the
// calling thread takes the first)
template <class Fn> void parallel_ranges(int n, Fn f) {
  const int hw = (int)std::max(1u, std::min(8u, std::thread::hardware_concurrency()));
  const int nt = std::max(1, std::min(hw, n / 256));
  if (nt == 1) {
    f(0, n);
    return;
  }
  std::vector<std::thread> th;
  for (int t = 1; t < nt; ++t)
    th.emplace_back(f, (int)((int64_t)n * t / nt), (int)((int64_t)n * (t + 1) / nt));
  f(0, (int)((int64_t)n / nt));
  for (auto& x : th) x.join();
}

// Greedy colouring of the near graph in decreasing (hash(id), id) priority;
// identical to the Jones-Plassmann result for the same priorities.
void color_level(LevelPlan& P) {
  std::vector<int> order(P.nl);
  std::iota(order.begin(), order.end(), 0);
  std::vector<uint64_t> h(P.nl);
  for (int i = 0; i < P.nl; ++i) h[i] = node_hash((uint64_t)(P.a + i));
  std::sort(order.begin(), order.end(), [&](int x, int y) {
    if (h[x] != h[y]) return h[x] > h[y];
    return x > y;
  });
  P.color.assign(P.nl, -1);
  std::vector<int> mark;
  int nc = 0;
  for (int v : order) {
    mark.assign(P.nb[v].size() + 2, 0);
    for (int j : P.nb[v]) {
      const int c = P.color[j];
      if (j != v && c >= 0 && c < (int)mark.size()) mark[c] = 1;
    }
    int c = 0;
    while (mark[c]) ++c;
    P.color[v] = c;
    nc = std::max(nc, c + 1);
  }
  P.ncolors = nc;
  P.members.assign(nc, {});
  for (int i = 0; i < P.nl; ++i) P.members[P.color[i]].push_back(i);
}

}  // namespace

// Build the plan of level `lev` given the sizes n and the lifted fill pairs.
// Structure of level `lev` (colours, fill pattern, first colours, fill pairs)
// given its lifted fill pairs; it does not depend on the cluster sizes.
void plan_level_structure(const h2_matrix_s& H, int lev,
                          const std::vector<std::pair<int, int>>& lifted, LevelPlan& P) {
  P.lev = lev;
  P.a = H.lp[lev];
  P.nl = H.lp[lev + 1] - P.a;
  P.k.resize(P.nl);
  for (int i = 0; i < P.nl; ++i) P.k[i] = H.rank[P.a + i];
  P.nb.assign(P.nl, {});
  for (int i = 0; i < P.nl; ++i)
    for (int64_t e = H.near_ptr[P.a + i]; e < H.near_ptr[P.a + i + 1]; ++e)
      P.nb[i].push_back(H.near_col[e] - P.a);
  color_level(P);
  // fill pattern: lifted pairs plus non-near pairs of neighbours of a common
  // cluster; first colour writing each fill entry
  std::vector<std::vector<std::pair<int, int>>> rows(P.nl);  // (col, firstc)
  parallel_ranges(P.nl, [&](int j0, int j1) {
    std::vector<int> stamp(P.nl, -1), minc(P.nl, INT_MAX);
    std::vector<int> cols;
    for (int j = j0; j < j1; ++j) {
      for (int i : P.nb[j]) stamp[i] = j;  // near of j
      cols.clear();
      for (int i : P.nb[j]) {
        const int ci = P.color[i];
        for (int k : P.nb[i]) {
          if (stamp[k] == j) {
            // near of j or already collected
            if (minc[k] != INT_MAX && ci < minc[k]) minc[k] = ci;
            continue;
          }
          stamp[k] = j;
          minc[k] = ci;
          cols.push_back(k);
        }
      }
      for (int k : cols) {
        rows[j].push_back({k, minc[k]});
        minc[k] = INT_MAX;
      }
      for (int i : P.nb[j]) minc[i] = INT_MAX;
      std::sort(rows[j].begin(), rows[j].end());
    }
  });
  // lifted pairs (sorted): present from the start of the level (firstc -1)
  {
    std::vector<int64_t> lb(P.nl + 1, 0);
    for (auto& pr : lifted) ++lb[pr.first + 1];
    for (int j = 0; j < P.nl; ++j) lb[j + 1] += lb[j];
    parallel_ranges(P.nl, [&](int j0, int j1) {
      for (int j = j0; j < j1; ++j) {
        auto& rw = rows[j];
        const size_t nold = rw.size();
        for (int64_t q = lb[j]; q < lb[j + 1]; ++q) {
          const int c = lifted[q].second;
          auto it = std::lower_bound(rw.begin(), rw.begin() + nold, std::make_pair(c, INT_MIN));
          if (it != rw.begin() + nold && it->first == c)
            it->second = -1;
          else
            rw.push_back({c, -1});
        }
        if (rw.size() != nold) std::sort(rw.begin(), rw.end());
      }
    });
  }
  P.pptr.assign(P.nl + 1, 0);
  P.pcol.clear();
  P.isF.clear();
  P.firstc.clear();
  P.fill_pairs.clear();
  for (int j = 0; j < P.nl; ++j) {
    auto& rw = rows[j];
    // merge near (sorted) and fill (sorted)
    size_t a = 0, b = 0;
    const auto& nbj = P.nb[j];
    while (a < nbj.size() || b < rw.size()) {
      if (b >= rw.size() || (a < nbj.size() && nbj[a] < rw[b].first)) {
        P.pcol.push_back(nbj[a++]);
        P.isF.push_back(0);
        P.firstc.push_back(INT_MAX);
      } else {
        P.pcol.push_back(rw[b].first);
        P.isF.push_back(1);
        P.firstc.push_back(rw[b].second);
        P.fill_pairs.push_back({j, rw[b].first});
        ++b;
      }
    }
    P.pptr[j + 1] = (int64_t)P.pcol.size();
  }
}

// Block layout of a level from its cluster sizes n: D entries and F entries in
// two buffers, CSR order, n_i x n_j column-major.  The fill of the symmetric
// matrix is symmetric (F_kj = F_jk^T), so the F buffer holds one block per
// unordered pair, (j, k) with j < k; the entry (k, j) refers to it.
void plan_level_layout(LevelPlan& P, const std::vector<int>& n) {
  P.n = n;
  P.poff.assign(P.pcol.size(), 0);
  P.nD = P.nF = 0;
  // cur[k]: next entry of row k whose column is still to come; entries (k, j)
  // with j < k are met in ascending j as rows j are visited, so a cursor per
  // row finds the mirror of every stored fill block without a search
  std::vector<int64_t> cur(P.pptr.begin(), P.pptr.end() - 1);
  for (int j = 0; j < P.nl; ++j)
    for (int64_t e = P.pptr[j]; e < P.pptr[j + 1]; ++e) {
      const int k = P.pcol[e];
      const int64_t sz = (int64_t)P.n[j] * P.n[k];
      if (P.isF[e]) {
        if (k > j) {
          P.poff[e] = P.nF;
          P.nF += sz;
          int64_t& m = cur[k];  // the mirror (k, j), after the entries of row k below j
          while (m < P.pptr[k + 1] && P.pcol[m] < j) ++m;
          if (m == P.pptr[k + 1] || P.pcol[m] != j || !P.isF[m])
            throw H2Error(H2_ERROR_FORMAT, "fill pattern is not symmetric");
          P.poff[m] = P.poff[e];
        }
      } else {
        P.poff[e] = P.nD;
        P.nD += sz;
      }
    }
  P.offQ.assign(P.nl, 0);
  P.offV.assign(P.nl, 0);
  P.offPiv.assign(P.nl, 0);
  P.nQ = P.nV = P.nPiv = 0;
  for (int i = 0; i < P.nl; ++i) {
    P.offQ[i] = P.nQ;
    P.nQ += (int64_t)P.n[i] * P.n[i];
    P.offV[i] = P.nV;
    P.nV += (int64_t)P.n[i] * P.k[i];
    P.offPiv[i] = P.nPiv;
    P.nPiv += P.n[i];
  }
  P.r.assign(P.nl, 0);
}

// Build the plan of level `lev` given the sizes n and the lifted fill pairs.
void plan_level(const h2_matrix_s& H, int lev, const std::vector<int>& n,
                const std::vector<std::pair<int, int>>& lifted, LevelPlan& P) {
  plan_level_structure(H, lev, lifted, P);
  plan_level_layout(P, n);
}

// Lifted fill pairs of level plev (sorted, distinct) from the fill pattern of
// the level below it: per parent pt, the parents of its children's fill
// columns that are not near pt.
std::vector<std::pair<int, int>> lifted_pairs(const h2_matrix_s& H, const LevelPlan& P, int plev) {
  const int pa = H.lp[plev];
  const int np = H.lp[plev + 1] - pa;
  auto pnear = [&](int t, int s2) {  // is (t, s2) (global) a near pair of level plev
    const auto b = H.near_col.begin() + H.near_ptr[t], e = H.near_col.begin() + H.near_ptr[t + 1];
    return std::binary_search(b, e, s2);
  };
  std::vector<std::vector<int>> lrow(np);
  parallel_ranges(np, [&](int t0, int t1) {
    std::vector<int> stamp(np, -1);
    for (int t = t0; t < t1; ++t) {
      const int tau = pa + t;
      auto& lr = lrow[t];
      for (int c = H.cp[tau]; c < H.cp[tau + 1]; ++c) {
        const int j = c - P.a;
        for (int64_t e = P.pptr[j]; e < P.pptr[j + 1]; ++e) {
          if (!P.isF[e]) continue;
          const int ps = H.parent[P.a + P.pcol[e]];
          if (stamp[ps - pa] == t) continue;
          stamp[ps - pa] = t;
          if (!pnear(tau, ps)) lr.push_back(ps - pa);
        }
      }
      std::sort(lr.begin(), lr.end());
    }
  });
  std::vector<std::pair<int, int>> lifted;
  for (int t = 0; t < np; ++t)
    for (int x : lrow[t]) lifted.push_back({t, x});
  return lifted;
}

namespace {

template <class T> LevelStore<T>& store_of(h2_factor_s* F, size_t li);
template <> LevelStore<double>& store_of<double>(h2_factor_s* F, size_t li) { return F->st64[li]; }
template <> LevelStore<float>& store_of<float>(h2_factor_s* F, size_t li) { return F->st32[li]; }
template <class T> DevArray<T>& top_of(h2_factor_s* F);
template <> DevArray<double>& top_of<double>(h2_factor_s* F) { return F->M64; }
template <> DevArray<float>& top_of<float>(h2_factor_s* F) { return F->M32; }
template <class T> void add_store(h2_factor_s* F);
template <> void add_store<double>(h2_factor_s* F) { F->st64.emplace_back(); }
template <> void add_store<float>(h2_factor_s* F) { F->st32.emplace_back(); }

template <class T> struct Inst {
  h2_matrix_s* H = nullptr;
  h2_factor_s* F = nullptr;
  const T* data = nullptr;   // H data in the working precision
  DevArray<T> data_conv;     // converted copy (FP32 runs)
  int lev = 0;               // level being processed
  int tlev = -1;             // matrix top level
  bool done = false;
  int rbase = 0;             // offset of this instance's clusters in the height's r array
  size_t li = 0;             // index of the current level in F->plans
  DevArray<T> Fbuf;          // fill blocks of the current level
  DevArray<T> Vbuf;          // bases of the current level
  T* xmul = nullptr;         // the level's multiplier copies (read by the Schur updates)
  double norm = 0;           // ||A||_2 of eps_fill = tol ||A||_2
  double flops = 0;
  double pflops[H2_PHASES] = {0}, pbytes[H2_PHASES] = {0};
};

template <class T> int64_t copy_tiles(int rows, int cols) {
  return ((int64_t)rows * cols + kCopyTile - 1) / kCopyTile;
}

template <class T> struct CopyBatch {
  std::vector<CTask<T, T>> tasks;
  int64_t tiles = 0;
  void add(const T* src, int64_t lds, T* dst, int64_t ldd, int rows, int cols, int add,
           int tr = 0) {
    if (rows <= 0 || cols <= 0) return;
    CTask<T, T> t{};
    t.src = src;
    t.dst = dst;
    t.lds = lds;
    t.ldd = ldd;
    t.rows = rows;
    t.cols = cols;
    t.add = add;
    t.tr = tr;
    t.tile0 = tiles;
    tiles += copy_tiles<T>(rows, cols);
    tasks.push_back(t);
  }
  // append another batch's tasks (its tiles numbered after this one's)
  void append(const CopyBatch& o) {
    const size_t n0 = tasks.size();
    tasks.insert(tasks.end(), o.tasks.begin(), o.tasks.end());
    for (size_t q = n0; q < tasks.size(); ++q) tasks[q].tile0 += tiles;
    tiles += o.tiles;
  }
  void launch(DescArena& ar, hipStream_t s) {
    if (tasks.empty()) return;
    const CTask<T, T>* d = ar.put(tasks);
    ar.flush(s);
    launch_copy<T, T>(d, (int)tasks.size(), tiles, s);
  }
};

// initialise the leaf level: D blocks from the blob, V = U (F is zeroed by
// the caller).  The blob stores the leaf near blocks in CSR order (m_i x m_j
// each) and the leaf bases in leaf order (m_i x k_i), which are exactly the
// orders of the level's D buffer (near entries of the pattern in CSR order)
// and V buffer, so each is one contiguous device-to-device copy.
template <class T> void init_leaf(Inst<T>& I, LevelStore<T>& S, LevelPlan& P, hipStream_t s) {
  const h2_matrix_s& H = *I.H;
  const int q0 = P.a, q1 = P.a + P.nl;
  const int64_t d0 = H.offD[H.near_ptr[q0]];
  const int64_t d1 = H.near_ptr[q1] > H.near_ptr[q0]
                         ? H.offD[H.near_ptr[q1] - 1] +
                               (int64_t)H.size(q1 - 1) * H.size(H.near_col[H.near_ptr[q1] - 1])
                         : d0;
  const int64_t u0 = H.offU[q0];
  const int64_t u1 = H.offU[q1 - 1] + (int64_t)H.size(q1 - 1) * H.rank[q1 - 1];
  if (d1 - d0 != P.nD || u1 - u0 != P.nV)
    throw H2Error(H2_ERROR_FORMAT, "leaf blocks do not match the level layout");
  if (P.nD > 0)
    H2_HIP(hipMemcpyAsync(S.D.p, I.data + d0, sizeof(T) * P.nD, hipMemcpyDeviceToDevice, s));
  if (P.nV > 0)
    H2_HIP(hipMemcpyAsync(I.Vbuf.p, I.data + u0, sizeof(T) * P.nV, hipMemcpyDeviceToDevice, s));
}

// entry kinds of a level's pattern: 0 near, 1 stored fill (j < k), 2 fill
// entry (j, k) with k < j, whose block is the stored (k, j)
std::vector<int8_t> level_kinds(const LevelPlan& P) {
  std::vector<int8_t> kind(P.pcol.size());
  for (int j = 0; j < P.nl; ++j)
    for (int64_t e = P.pptr[j]; e < P.pptr[j + 1]; ++e) kind[e] = P.isF[e] ? (P.tr(j, e) ? 2 : 1) : 0;
  return kind;
}

template <class T> void alloc_level(Inst<T>& I, LevelPlan& P) {
  add_store<T>(I.F);
  LevelStore<T>& S = store_of<T>(I.F, I.F->plans.size() - 1);
  S.D.alloc(P.nD, &I.F->tr);
  S.Q.alloc(P.nQ, &I.F->tr);
  S.piv.alloc(P.nPiv, &I.F->tr);
  I.Fbuf.alloc(P.nF, &I.F->tr);
  I.Vbuf.alloc(P.nV, &I.F->tr);
}

}  // namespace

// Reduction groups of a fill row: consecutive fill blocks holding at most
// `cap` rows of Y^T together (at least one block each; one empty group for an
// empty fill row).
static std::vector<std::pair<int, int>> rf_groups(const std::vector<int>& rows, int cap) {
  std::vector<std::pair<int, int>> g;
  if (rows.empty()) {
    g.push_back({0, 0});
    return g;
  }
  size_t a = 0;
  while (a < rows.size()) {
    size_t b = a;
    int64_t acc = 0;
    while (b < rows.size() && (b == a || acc + rows[b] <= cap)) acc += rows[b++];
    g.push_back({(int)a, (int)b});
    a = b;
  }
  return g;
}

// Scratch elements of the tall-skinny QR of a fill row of order n whose
// blocks have the given widths: one n x n factor per task of every stage
// (groups of blocks, then pairs of factors), plus the global-memory
// reduction space when R does not fit in LDS.
template <class T> static int64_t rf_scratch(int n, const std::vector<int>& rows, int lds) {
  const int64_t per = (int64_t)n * n + (rf_in_lds<T>(n, lds) ? 0 : (int64_t)(n + kAugChunk) * n);
  int64_t g = (int64_t)rf_groups(rows, rf_group_rows(n)).size();
  int64_t tot = g * per;
  for (; g > 1; g = (g + 1) / 2) tot += (g / 2) * per;
  return tot;
}

// Launch descriptors of one colour of one level (all instances).  They are
// built on worker threads from the level's static structure only (window
// starts that depend on earlier colours are read on the device through the
// r array) and consumed in colour order by the launching thread.
template <class T> struct ColourPlan {
  std::vector<AugTask<T>> aug;
  std::vector<std::vector<RTask<T>>> rst;  // per stage of the fill-row QR
  std::vector<std::vector<FillRef<T>>> rrefs;
  std::vector<int> rmaxn;
  std::vector<GramTask<T>> gram;           // FP32: Gram matrices of the fill rows
  std::vector<FillRef<T>> grefs;
  int64_t gram_tiles = 0;
  std::vector<CholTask<T>> chol;           // FP32: their pivoted Cholesky factors
  int cmaxn = 1;
  std::vector<STask<T>> sl, sr;
  int64_t nsl = 0, nsr = 0;
  std::vector<LUTask<T>> lus;
  std::vector<TrsmTask<T>> trs;
  // Schur target lists of the colour per level plan (kept on request)
  std::vector<std::pair<LevelPlan*, std::vector<int64_t>>> owners;
};

// colours planned ahead of the launches
constexpr int kPlanAhead = 8;


template <class T>
static void run_factor(h2_context_s* ctx, std::vector<Inst<T>>& insts, double tol,
                       DevTracker* calltr, int lds) {
  hipStream_t s = ctx->stream;
  // FP32 with the Gram augmentation (Section 2.1, first option): the fill row
  // enters the augmentation as its FP64 Gram matrix (gram_mode: FP64
  // eigendecomposition; chol_mode: pivoted Cholesky factor, then the QR
  // route's SVD); otherwise the QR route
  const h2_prec prec = insts.empty() ? H2_PREC_FP64 : insts[0].F->prec;
  const bool gram_mode = sizeof(T) == 4 && prec == H2_PREC_FP32_GRAM;
  const bool chol_mode = sizeof(T) == 4 && prec == H2_PREC_FP32;
  // chol_mode: this cluster's fill row goes through the Gram factor
  auto use_chol = [&](int n) { return chol_mode && n <= kCholMaxOrder; };
  DescArena& ar = ctx->arena;
  ar.s = s;
  H2_HIP(hipMemsetAsync(ctx->d_err.p, 0, sizeof(int), s));
  const auto t_start = std::chrono::steady_clock::now();
  double plan_ms = 0;
  auto ms_since = [](std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  };
  // events for phase timing
  std::vector<hipEvent_t> evpool;
  auto new_event = [&]() {
    hipEvent_t e;
    H2_HIP(hipEventCreate(&e));
    evpool.push_back(e);
    return e;
  };
  double phase_ms[H2_PHASES] = {0};
  int64_t launches[H2_PHASES] = {0};

  // ---- leaf level plans ----
  {
    const auto t0 = std::chrono::steady_clock::now();
    for (auto& I : insts) {
      const h2_matrix_s& H = *I.H;
      I.lev = H.L;
      I.tlev = H.top;
      std::vector<int> n(H.lp[H.L + 1] - H.lp[H.L]);
      for (size_t i = 0; i < n.size(); ++i) n[i] = H.size(H.lp[H.L] + (int)i);
      if (I.tlev < 0) {
        // no admissible block: the whole leaf level is the dense top block
        I.done = true;
        continue;
      }
      I.F->plans.emplace_back();
      LevelPlan& P = I.F->plans.back();
      plan_level(H, H.L, n, {}, P);
      alloc_level(I, P);
      I.li = I.F->plans.size() - 1;
      LevelStore<T>& S = store_of<T>(I.F, I.li);
      launch_fill<T>(I.Fbuf.p, I.Fbuf.n, T(0), s);
      init_leaf(I, S, P, s);
    }
    plan_ms += ms_since(t0);
  }

  // ---- heights ----
  for (;;) {
    std::vector<Inst<T>*> act;
    for (auto& I : insts)
      if (!I.done) act.push_back(&I);
    if (act.empty()) break;
    const auto t0 = std::chrono::steady_clock::now();
    // structure of each instance's next level (lifted pairs, colours, fill
    // pattern), which needs no rank of this level: planned on worker threads
    // while this level's colours run, taken at the level end
    std::vector<std::future<std::unique_ptr<LevelPlan>>> next_struct(act.size());
    for (size_t q = 0; q < act.size(); ++q) {
      Inst<T>* I = act[q];
      if (I->lev == I->tlev) continue;  // the next level is the dense top block
      const h2_matrix_s* Hp = I->H;
      const LevelPlan* Pp = &I->F->plans[I->li];
      const int plev = I->lev - 1;
      next_struct[q] = std::async(std::launch::async, [Hp, Pp, plev]() {
        auto PN = std::make_unique<LevelPlan>();
        plan_level_structure(*Hp, plev, lifted_pairs(*Hp, *Pp, plev), *PN);
        return PN;
      });
    }
    int total = 0, maxc = 0;
    for (auto* I : act) {
      LevelPlan& P = I->F->plans[I->li];
      I->rbase = total;
      total += P.nl;
      maxc = std::max(maxc, P.ncolors);
    }
    DevArray<int32_t> rdev;
    rdev.alloc(total, calltr);
    launch_fill<int32_t>(rdev.p, total, 0, s);
    // each instance's block pattern on the device, for the Schur and fill-in
    // updates that are enumerated there (staged through the arena, which is
    // reset only after the level's last launch has completed)
    std::vector<SchurLevel<T>> lvh(act.size());
    // kXmulCopy: the multipliers D_RR^{-1} D_{R_i,k} once more, compact
    // (r_i x n_k) in an n_i x n_k region of the colour's copy area: the Schur
    // updates of the colour read them there (the factor keeps them inside D
    // for the solves); the area is reused by every colour
    std::vector<DevArray<T>> xmul(act.size());
    if (kXmulCopy<T>())
      for (size_t q = 0; q < act.size(); ++q) {
        LevelPlan& P = act[q]->F->plans[act[q]->li];
        P.xoff.assign(P.pcol.size(), 0);
        P.nX = 0;
        for (int c = 0; c < P.ncolors; ++c) {
          int64_t off = 0;
          for (int i : P.members[c])
            for (int64_t e = P.pptr[i]; e < P.pptr[i + 1]; ++e)
              if (!P.isF[e]) {
                P.xoff[e] = off;
                off += (int64_t)P.n[i] * P.n[P.pcol[e]];
              }
          P.nX = std::max(P.nX, off);
        }
        xmul[q].alloc(std::max<int64_t>(P.nX, 1), calltr);
      }
    int64_t schur_rows = 0, schur_nnz = 0;
    for (size_t q = 0; q < act.size(); ++q) {
      Inst<T>* I = act[q];
      LevelPlan& P = I->F->plans[I->li];
      SchurLevel<T>& L = lvh[q];
      L.pptr = ar.put(P.pptr);
      L.pcol = ar.put(P.pcol);
      L.poff = ar.put(P.poff);
      L.xoff = kXmulCopy<T>() ? ar.put(P.xoff) : nullptr;
      L.kind = ar.put(level_kinds(P));
      L.color = ar.put(P.color);
      L.n = ar.put(P.n);
      L.r = rdev.p + I->rbase;
      L.D = store_of<T>(I->F, I->li).D.p;
      L.F = I->Fbuf.p;
      L.X = I->xmul = xmul[q].p;
      L.nl = P.nl;
      L.rows0 = schur_rows;
      schur_rows += P.nl;
      schur_nnz += (int64_t)P.pcol.size();
    }
    const SchurLevel<T>* lvdev = ar.put(lvh);
    // the device's Schur target lists: every row's contributors of the colour
    // being processed, and at most one target per pattern entry
    // the contributor entries of a colour's targets: at most the sum over the
    // colour's clusters of |N(i)|^2 (maximum over colours, summed over instances)
    int64_t schur_ncon = 0;
    {
      std::vector<int64_t> per(maxc, 0);
      for (auto* I : act) {
        const LevelPlan& P = I->F->plans[I->li];
        for (int i = 0; i < P.nl; ++i)
          per[P.color[i]] += (int64_t)P.nb[i].size() * (int64_t)P.nb[i].size();
      }
      for (int64_t x : per) schur_ncon = std::max(schur_ncon, x);
    }
    DevArray<SchurRow> schur_rowtab;
    DevArray<SchurTarget> schur_targets;
    DevArray<int64_t> schur_conts, schur_count;
    schur_rowtab.alloc(std::max<int64_t>(schur_rows, 1), calltr);
    schur_targets.alloc(std::max<int64_t>(schur_nnz, 1), calltr);
    schur_conts.alloc(std::max<int64_t>(schur_ncon, 1), calltr);
    schur_count.alloc(2, calltr);
    int maxn_all = 1;
    for (auto* I : act)
      for (int x : I->F->plans[I->li].n) maxn_all = std::max(maxn_all, x);
    if ((int64_t)maxn_all * kStrip * (int64_t)sizeof(T) > 160 * 1024)
      throw H2Error(H2_ERROR_UNSUPPORTED, "cluster of order " + std::to_string(maxn_all) +
                                              " exceeds the strip kernel's LDS capacity");
    if (maxn_all > kMaxAugOrder)
      throw H2Error(H2_ERROR_UNSUPPORTED, "cluster of order " + std::to_string(maxn_all) +
                                              " exceeds the augmentation's limit of " +
                                              std::to_string(kMaxAugOrder));
    // augmentation workspace: max over colours of the sum of per-task scratch
    int64_t wmax = 0;
    int64_t gwmax = 0;
    for (int c = 0; c < maxc; ++c) {
      int64_t w = 0, gw = 0;
      for (auto* I : act) {
        LevelPlan& P = I->F->plans[I->li];
        if (c >= P.ncolors) continue;
        for (int i : P.members[c]) {
          std::vector<int> rows;
          for (int64_t e = P.pptr[i]; e < P.pptr[i + 1]; ++e)
            if (P.isF[e] && P.firstc[e] < c) rows.push_back(P.n[P.pcol[e]]);
          if (gram_mode) {
            w += 2 * aug_work_elems(P.n[i]);  // FP64 arithmetic in FP32 units
            gw += (int64_t)P.n[i] * P.n[i];
          } else if (use_chol(P.n[i])) {
            w += aug_work_elems(P.n[i]) + (int64_t)P.n[i] * P.n[i] + 4;
            gw += (int64_t)P.n[i] * P.n[i] * (int64_t)rf_groups(rows, kGramChunk).size();
          } else {
            w += aug_work_elems(P.n[i]) + rf_scratch<T>(P.n[i], rows, lds);
          }
        }
      }
      wmax = std::max(wmax, w);
      gwmax = std::max(gwmax, gw);
    }
    DevArray<T> work;
    work.alloc(wmax, calltr);
    DevArray<double> gwork;  // Gram matrices of a colour (FP32 path)
    gwork.alloc(gwmax, calltr);
    plan_ms += ms_since(t0);

    // (phase, start, end) events around each phase's launches
    std::vector<std::tuple<int, hipEvent_t, hipEvent_t>> marks;
    auto mark = [&](int ph) {
      hipEvent_t e = new_event();
      H2_HIP(hipEventRecord(e, s));
      return std::make_pair(ph, e);
    };
    auto close_mark = [&](std::pair<int, hipEvent_t> st) {
      hipEvent_t e = new_event();
      H2_HIP(hipEventRecord(e, s));
      marks.emplace_back(st.first, st.second, e);
    };
    auto plan_colour = [&](int c) {
      ColourPlan<T> cp;
      auto& aug = cp.aug;
      auto& rst = cp.rst;
      auto& rrefs = cp.rrefs;
      auto& rmaxn = cp.rmaxn;
      auto& sl = cp.sl;
      auto& sr = cp.sr;
      int64_t& nsl = cp.nsl;
      int64_t& nsr = cp.nsr;
      auto& lus = cp.lus;
      auto& trs = cp.trs;
      int64_t woff = 0, goff = 0;
      for (auto* I : act) {
        LevelPlan& P = I->F->plans[I->li];
        if (c >= P.ncolors) continue;
        LevelStore<T>& S = store_of<T>(I->F, I->li);
        const int rb = I->rbase;
        auto blk = [&](int64_t e) -> T* { return (P.isF[e] ? I->Fbuf.p : S.D.p) + P.poff[e]; };
        // active-window start of neighbour j at colour c: r_j once processed
        auto wdyn = [&](int j, bool incl) -> int {
          return (P.color[j] < c || (incl && P.color[j] == c)) ? rb + j : -1;
        };
        for (int i : P.members[c]) {
          const int ni = P.n[i];
          // ---- augmentation task ----
          AugTask<T> at{};
          at.V = I->Vbuf.p + P.offV[i];
          at.Q = S.Q.p + P.offQ[i];
          at.work = work.p + woff;
          woff += aug_work_elems(ni) * (gram_mode ? 2 : 1);
          at.n = ni;
          at.k = P.k[i];
          at.eps = tol * I->norm;  // eps_fill of the task's own matrix
          std::vector<FillRef<T>> cur;
          for (int64_t e = P.pptr[i]; e < P.pptr[i + 1]; ++e) {
            if (!P.isF[e] || P.firstc[e] >= c) continue;  // zero until a later colour
            const int j = P.pcol[e];
            FillRef<T> fr{};
            fr.F = blk(e);
            fr.tr = P.tr(i, e) ? 1 : 0;
            fr.ld = fr.tr ? P.n[j] : ni;  // the stored block is (j, i) when transposed
            fr.ncols = P.n[j];
            fr.d0 = wdyn(j, false);
            cur.push_back(fr);
          }
          if (gram_mode) {
            GramTask<T> g{};
            g.G = gwork.p + goff;
            goff += (int64_t)ni * ni;
            g.n = ni;
            g.fbeg = (int)cp.grefs.size();
            cp.grefs.insert(cp.grefs.end(), cur.begin(), cur.end());
            g.fend = (int)cp.grefs.size();
            g.tm = (ni + 63) / 64;
            g.tile0 = cp.gram_tiles;
            cp.gram_tiles += (int64_t)g.tm * g.tm;
            cp.gram.push_back(g);
            at.G = g.G;
          }
          const bool chol = use_chol(ni);
          if (chol) {
            // partial Gram matrices over chunks of about kGramChunk fill
            // columns (one workgroup tile each), summed and factored by the
            // pivoted Cholesky
            std::vector<int> rows(cur.size());
            for (size_t q = 0; q < cur.size(); ++q) rows[q] = cur[q].ncols;
            const auto groups = rf_groups(rows, kGramChunk);
            CholTask<T> ct{};
            ct.G = gwork.p + goff;
            for (const auto& gr : groups) {
              GramTask<T> g{};
              g.G = gwork.p + goff;
              goff += (int64_t)ni * ni;
              g.n = ni;
              g.fbeg = (int)cp.grefs.size();
              cp.grefs.insert(cp.grefs.end(), cur.begin() + gr.first, cur.begin() + gr.second);
              g.fend = (int)cp.grefs.size();
              g.tm = (ni + 63) / 64;
              g.tile0 = cp.gram_tiles;
              cp.gram_tiles += (int64_t)g.tm * g.tm;
              cp.gram.push_back(g);
            }
            ct.Rt = work.p + woff;
            woff += (int64_t)ni * ni + 4;  // the factor, its rank, alignment
            ct.n = ni;
            ct.nch = (int)groups.size();
            ct.eps = at.eps;
            cp.chol.push_back(ct);
            cp.cmaxn = std::max(cp.cmaxn, ni);
            at.Rt = ct.Rt;
            at.rgen = 1;
          }
          // stages of the tall-skinny QR: groups of fill blocks, then groups of
          // the previous stage's factors, until one factor remains
          const bool rf_glob = !rf_in_lds<T>(ni, lds);
          for (size_t st = 0; !gram_mode && !chol; ++st) {
            // stage 0: groups of fill blocks; later stages: pairs of factors
            // (an odd one passes to the next stage as it is)
            std::vector<std::pair<int, int>> groups;
            if (st == 0) {
              std::vector<int> rows(cur.size());
              for (size_t q = 0; q < cur.size(); ++q) rows[q] = cur[q].ncols;
              groups = rf_groups(rows, rf_group_rows(ni));
            } else {
              for (int q = 0; q < (int)cur.size(); q += 2)
                groups.push_back({q, std::min(q + 2, (int)cur.size())});
            }
            if (rst.size() <= st) {
              rst.emplace_back();
              rrefs.emplace_back();
              rmaxn.push_back(1);
            }
            std::vector<FillRef<T>> next;
            for (const auto& g : groups) {
              if (st > 0 && g.second - g.first == 1) {
                next.push_back(cur[g.first]);
                continue;
              }
              RTask<T> t{};
              t.tri = st > 0 ? 1 : 0;
              t.out = work.p + woff;
              woff += (int64_t)ni * ni;
              if (rf_glob) {
                t.work = work.p + woff;
                woff += (int64_t)(ni + kAugChunk) * ni;
              }
              t.n = ni;
              t.fbeg = (int)rrefs[st].size();
              for (int q = g.first; q < g.second; ++q) rrefs[st].push_back(cur[q]);
              t.fend = (int)rrefs[st].size();
              rst[st].push_back(t);
              rmaxn[st] = std::max(rmaxn[st], ni);
              FillRef<T> o{};
              o.F = t.out;
              o.ld = ni;
              o.ncols = ni;
              o.d0 = -1;
              next.push_back(o);
            }
            if (groups.size() == 1) {
              at.Rt = next[0].F;
              break;
            }
            cur.swap(next);
          }
          at.ri = rb + i;
          aug.push_back(at);
          // ---- projection: row i (left, Q^T X) and column i (right, X Q) ----
          for (int64_t e = P.pptr[i]; e < P.pptr[i + 1]; ++e) {
            const int j = P.pcol[e];
            if (P.isF[e] && P.firstc[e] >= c && j != i) {
              // still zero: a zero block stays zero under the projection
              continue;
            }
            STask<T> t{};
            t.X = blk(e);
            t.Q = S.Q.p + P.offQ[i];
            t.n = ni;
            t.ext = P.n[j];
            t.d0 = wdyn(j, false);
            t.s0 = 0;
            if (P.tr(i, e)) {
              // fill stored as (j, i): its column side, F_ji <- F_ji Q~ (the
              // one update of the pair's block by cluster i)
              if (P.n[j] > 0 && ni > 0) {
                t.ldx = P.n[j];
                t.side = 1;
                t.trans = 0;
                t.strip0 = nsr;
                nsr += (P.n[j] + kStrip - 1) / kStrip;
                sr.push_back(t);
              }
              continue;
            }
            t.ldx = ni;
            t.side = 0;
            t.trans = 1;
            t.strip0 = nsl;
            nsl += (P.n[j] + kStrip - 1) / kStrip;
            if (P.n[j] > 0 && ni > 0) sl.push_back(t);
            else nsl -= (P.n[j] + kStrip - 1) / kStrip;
          }
          // column i: entries (j, i) for j in the pattern row of i (symmetric
          // pattern); fill blocks are stored once per pair and were updated
          // above
          for (int64_t e = P.pptr[i]; e < P.pptr[i + 1]; ++e) {
            const int j = P.pcol[e];
            const int64_t et = P.find(j, i);
            if (P.isF[et]) continue;
            STask<T> t{};
            t.X = blk(et);
            t.Q = S.Q.p + P.offQ[i];
            t.ldx = P.n[j];
            t.n = ni;
            t.ext = P.n[j];
            t.d0 = wdyn(j, false);
            t.s0 = 0;
            t.side = 1;
            t.trans = 0;
            t.strip0 = nsr;
            const int64_t ns = (P.n[j] + kStrip - 1) / kStrip;
            if (P.n[j] > 0 && ni > 0) {
              sr.push_back(t);
              nsr += ns;
            }
          }
          // ---- LU of D_RR and the U-blocks D_RR^{-1} D_{R,k} ----
          const int64_t eii = P.find(i, i);
          LUTask<T> lt{};
          lt.A = S.D.p + P.poff[eii];
          lt.piv = S.piv.p + P.offPiv[i];
          lt.lda = ni;
          lt.ri = rb + i;
          lus.push_back(lt);
          for (int k : P.nb[i]) {
            const int64_t eik = P.find(i, k);
            TrsmTask<T> tt{};
            tt.LU = lt.A;
            tt.piv = lt.piv;
            tt.B = S.D.p + P.poff[eik];
            tt.Bc = I->xmul ? I->xmul + P.xoff[eik] : nullptr;
            tt.ldlu = ni;
            tt.ldb = ni;
            tt.ncols = P.n[k];
            tt.ri = rb + i;
            tt.rs = 0;
            tt.c0d = wdyn(k, true);
            tt.c0s = 0;
            trs.push_back(tt);
          }
        }
        // ---- Schur complement / fill-in targets ----
        // enumerated on the device (launch_schur); the owner lists are formed
        // here only when they are exported: target (j, k) collects every i of
        // the colour with j, k in N(i), i.e. the colour's clusters i in N(j)
        // whose near list holds k; targets in ascending (j, k) (fill entries
        // when stored, j < k), contributors in ascending i
        if (I->F->keep_owners) {
          std::vector<int64_t> rec;
          std::vector<int> stamp(P.nl, -1), conts, tk;
          for (int j = 0; j < P.nl; ++j) {
            conts.clear();
            tk.clear();
            for (int i : P.nb[j])
              if (P.color[i] == c) conts.push_back(i);
            for (int i : conts)
              for (int k : P.nb[i])
                if (stamp[k] != j) {
                  stamp[k] = j;
                  tk.push_back(k);
                }
            std::sort(tk.begin(), tk.end());
            for (int k : tk) {
              const int64_t e = P.find(j, k);
              if (e < 0) throw H2Error(H2_ERROR_FORMAT, "fill pattern misses a Schur target");
              if (P.tr(j, e)) continue;
              const size_t at = rec.size();
              rec.push_back(c);
              rec.push_back(j + P.a);
              rec.push_back(k + P.a);
              rec.push_back(0);
              for (int i : conts) {
                const int64_t eik = P.find(i, k);
                if (eik >= 0 && !P.isF[eik]) rec.push_back(i + P.a);
              }
              rec[at + 3] = (int64_t)(rec.size() - at - 4);
            }
          }
          cp.owners.push_back({&P, std::move(rec)});
        }
      }
      return cp;
    };
    // planners run up to kPlanAhead colours ahead of the launches
    std::deque<std::future<ColourPlan<T>>> ahead;
    int next_c = 0;
    auto refill = [&]() {
      while (next_c < maxc && (int)ahead.size() < kPlanAhead)
        ahead.push_back(std::async(std::launch::async, plan_colour, next_c++));
    };
    refill();
    for (int c = 0; c < maxc; ++c) {
      const auto tc = std::chrono::steady_clock::now();
      ColourPlan<T> cp = ahead.front().get();
      ahead.pop_front();
      refill();
      plan_ms += ms_since(tc);  // planning the launching thread waited for
      auto& aug = cp.aug;
      auto& rst = cp.rst;
      auto& rrefs = cp.rrefs;
      auto& rmaxn = cp.rmaxn;
      auto& sl = cp.sl;
      auto& sr = cp.sr;
      const int64_t nsl = cp.nsl, nsr = cp.nsr;
      auto& lus = cp.lus;
      auto& trs = cp.trs;
      for (auto& ow : cp.owners)
        ow.first->owners.insert(ow.first->owners.end(), ow.second.begin(), ow.second.end());
      if (aug.empty()) continue;
      int maxn = 1, maxn_aug = 1;
      for (auto& t : aug) maxn_aug = std::max(maxn_aug, t.n);
      for (auto& t : sl) maxn = std::max(maxn, t.n);
      for (auto& t : sr) maxn = std::max(maxn, t.n);
      const int32_t* dyn = rdev.p;
      const bool gram = gram_mode;
      // every descriptor of the colour staged first, then one transfer
      const GramTask<T>* dgram = ar.put(cp.gram);
      const FillRef<T>* dgrefs = ar.put(cp.grefs);
      const CholTask<T>* dchol = ar.put(cp.chol);
      std::vector<const RTask<T>*> drst(rst.size());
      std::vector<const FillRef<T>*> drrefs(rst.size());
      for (size_t st = 0; st < rst.size(); ++st) {
        drst[st] = ar.put(rst[st]);
        drrefs[st] = ar.put(rrefs[st]);
      }
      const AugTask<T>* daug = ar.put(aug);
      const STask<T>* dsl = ar.put(sl);
      const STask<T>* dsr = ar.put(sr);
      const LUTask<T>* dlus = ar.put(lus);
      const TrsmTask<T>* dtrs = ar.put(trs);
      ar.flush(s);
      {
        auto m0 = mark(0);
        launch_gram<T>(dgram, (int)cp.gram.size(), dgrefs, rdev.p, cp.gram_tiles, s);
        launch_pchol<T>(dchol, (int)cp.chol.size(), cp.cmaxn, s);
        for (size_t st = 0; st < rst.size(); ++st)
          launch_rfactor<T>(drst[st], (int)rst[st].size(), drrefs[st], rdev.p, rmaxn[st], s, lds);
        close_mark(m0);
      }
      auto m1 = mark(1);
      launch_augment<T>(daug, (int)aug.size(), rdev.p, ctx->d_err.p, maxn_aug, gram, s, lds);
      close_mark(m1);
      launches[0] += (cp.gram.empty() ? 0 : 1) + (cp.chol.empty() ? 0 : 1) + (int64_t)rst.size();
      launches[1] += 1;
      launches[2] += 2;
      launches[3] += 1;
      launches[4] += 1;
      launches[5] += 1;
      {
        auto m2 = mark(2);
        // the projections of a colour cover many strips: four per workgroup
        launch_strip<T>(dsl, (int)sl.size(), dyn, nsl, maxn, s, 4);
        launch_strip<T>(dsr, (int)sr.size(), dyn, nsr, maxn, s, 4);
        close_mark(m2);
      }
      {
        int maxr = 1;  // r <= n of the cluster (its D block's leading dimension)
        for (auto& t : lus) maxr = std::max(maxr, (int)t.lda);
        auto m3 = mark(3);
        launch_lu<T>(dlus, (int)lus.size(), dyn, ctx->d_err.p, maxr, s, lds);
        close_mark(m3);
      }
      {
        int maxr = 1, maxcols = 1;
        for (auto& t : trs) {
          maxr = std::max(maxr, (int)t.ldlu);
          maxcols = std::max(maxcols, t.ncols);
        }
        auto m4 = mark(4);
        launch_trsm<T>(dtrs, (int)trs.size(), dyn, maxr, maxcols, s, lds);
        close_mark(m4);
      }
      {
        auto m5 = mark(5);
        launch_schur<T>(lvdev, (int)act.size(), schur_rows, c, schur_rowtab.p, schur_targets.p,
                        schur_conts.p, schur_count.p, schur_conts.n, ctx->d_err.p, s);
        close_mark(m5);
      }
      H2_HIP(hipGetLastError());  // a rejected launch configuration
    }
    for (auto* I : act) std::vector<int64_t>().swap(I->F->plans[I->li].xoff);
    // ---- level end: read the ranks ----
    std::vector<int32_t> rh(total);
    H2_HIP(hipMemcpyAsync(rh.data(), rdev.p, sizeof(int32_t) * total, hipMemcpyDeviceToHost, s));
    H2_HIP(hipStreamSynchronize(s));
    {
      int herr = 0;
      H2_HIP(hipMemcpy(&herr, ctx->d_err.p, sizeof(int), hipMemcpyDeviceToHost));
      if (herr & 1) throw H2Error(H2_ERROR_SINGULAR, "zero pivot in a redundant block");
      if (herr & 2) throw H2Error(H2_ERROR_NUMERIC, "non-finite singular value in augmentation");
      if (herr & 4)
        throw H2Error(H2_ERROR_UNSUPPORTED,
                      "a block row has more than " + std::to_string(kSchurMaxContrib) +
                          " Schur contributors of one colour, or the update list overflowed");
      if (herr & 8)
        throw H2Error(H2_ERROR_FORMAT, "close-out destination missing from the next level");
    }
    {
      for (auto& m : marks) {
        float ms = 0;
        H2_HIP(hipEventElapsedTime(&ms, std::get<1>(m), std::get<2>(m)));
        phase_ms[std::get<0>(m)] += ms;
      }
      marks.clear();
    }
    // ---- close-out into the next level (or the dense top block) ----
    for (size_t q = 0; q < act.size(); ++q) {
      Inst<T>* I = act[q];
      const auto tpl = std::chrono::steady_clock::now();
      const h2_matrix_s& H = *I->H;
      h2_factor_s* F = I->F;
      LevelPlan& P = F->plans[I->li];
      for (int i = 0; i < P.nl; ++i) P.r[i] = rh[I->rbase + i];
      // algorithmic flop model of the level, on a worker thread while the
      // close-out is planned (it reads the plan and writes only the instance's
      // counters)
      auto flop_model = std::async(std::launch::async, [I, &P, gmode = gram_mode, cmode = chol_mode]() {
        for (int i = 0; i < P.nl; ++i) {
          const double n = P.n[i], k = P.k[i], r = P.r[i], kt = n - r;
          const bool gm = gmode || (cmode && P.n[i] <= kCholMaxOrder);
          double f = 0, W = kt, Wn = 0;
          for (int64_t e = P.pptr[i]; e < P.pptr[i + 1]; ++e) {
            const int j = P.pcol[e];
            const double w = (P.color[j] < P.color[i]) ? P.n[j] - P.r[j] : P.n[j];
            if (P.isF[e] && P.firstc[e] < P.color[i]) f += w;
            if (!P.isF[e] && j != i) {
              W += w;
              Wn += w;
            }
          }
          // augmentation: projection of the fill row, Householder QR of its
          // transpose (f x n), SVD of the n x n factor (reported as 4 n^3)
          const double qr = f >= n ? 2 * f * n * n - 2 * n * n * n / 3 : 2 * n * f * f - 2 * f * f * f / 3;
          // FP32 path: the Gram matrix Y Y^T (2 n^2 f) replaces the QR
          const double f_qr = gm ? 2 * n * n * f : (4 * n * k * f + qr) * (f > 0);
          const double f_aug = (f_qr + 4 * n * n * n) * (f > 0) +
                               2 * n * kt * kt - 2 * kt * kt * kt / 3 +
                               4 * (n * n * kt - n * kt * kt + kt * kt * kt / 3);
          const double f_proj = 4 * n * n * n + 4 * n * n * Wn + 4 * n * kt * f;
          const double f_lu = 2 * r * r * r / 3 + 2 * r * r * W;
          const double f_schur = 2 * r * W * W;
          I->flops += f_aug + f_proj + f_lu + f_schur;
          const double b = (double)sizeof(T);
          I->pflops[0] += f_qr;
          I->pflops[1] += f_aug - f_qr;
          I->pflops[2] += f_proj;
          I->pflops[3] += 2 * r * r * r / 3;
          I->pflops[4] += 2 * r * r * W;
          I->pflops[5] += f_schur;
          // compulsory bytes: fill row read once (and the group factors
          // written); R, V in and Q~ out; projected blocks read + written;
          // D_RR read + written; panels read + written; Schur targets read +
          // written once per contributor group
          I->pbytes[0] += b * n * f + (gm ? 8.0 : b) * n * n;
          I->pbytes[1] += b * (n * n + n * k + n * n);
          I->pbytes[2] += b * 2 * (n * n + n * Wn + n * f);
          I->pbytes[3] += b * 2 * r * r;
          I->pbytes[4] += b * (r * r + 2 * r * W);
          I->pbytes[5] += b * (2 * r * W + 2 * W * W);
        }
      });
      const int lev = P.lev;
      const int plev = lev - 1;
      // sizes of the next level
      std::vector<int> n2(H.lp[plev + 1] - H.lp[plev]);
      std::vector<int> offc(P.nl);
      for (int t = 0; t < (int)n2.size(); ++t) {
        const int tau = H.lp[plev] + t;
        int o = 0;
        for (int c = H.cp[tau]; c < H.cp[tau + 1]; ++c) {
          offc[c - P.a] = o;
          o += P.n[c - P.a] - P.r[c - P.a];
        }
        n2[t] = o;
      }
      const int pa = H.lp[plev];
      const bool is_top = (lev == I->tlev);
      // destination of a parent pair block: next level D / F, or the dense top
      T* Dn = nullptr;
      T* Fn = nullptr;
      LevelPlan* PN = nullptr;
      int64_t ldtop = 0;
      if (is_top) {
        F->top_level = plev;
        F->top_nodes.clear();
        F->top_off.assign(n2.size(), 0);
        int64_t o = 0;
        for (size_t t = 0; t < n2.size(); ++t) {
          F->top_nodes.push_back(pa + (int)t);
          F->top_off[t] = o;
          o += n2[t];
        }
        F->top_n = n2;
        F->n_top = o;
        ldtop = o;
        DevArray<T>& M = top_of<T>(F);
        M.alloc(o * o, &F->tr);
        launch_fill<T>(M.p, o * o, T(0), s);
        Dn = M.p;
      } else {
        // structure planned during the level's colours; only the layout
        // needed the ranks
        std::unique_ptr<LevelPlan> nxt = next_struct[q].get();
        F->plans.push_back(std::move(*nxt));
        PN = &F->plans.back();
        plan_level_layout(*PN, n2);
      }
      LevelPlan& Pc = F->plans[I->li];
      LevelStore<T>* Sc = &store_of<T>(F, I->li);
      DevArray<T> Vnext;
      if (!is_top) {
        // allocate next level buffers (F and V of the instance move on)
        add_store<T>(F);
        Sc = &store_of<T>(F, I->li);
        LevelStore<T>& SN = store_of<T>(F, F->plans.size() - 1);
        SN.D.alloc(PN->nD, &F->tr);
        SN.Q.alloc(PN->nQ, &F->tr);
        SN.piv.alloc(PN->nPiv, &F->tr);
        launch_fill<T>(SN.D.p, SN.D.n, T(0), s);
        Dn = SN.D.p;
      }
      DevArray<T> Fnext;
      if (!is_top) {
        Fnext.alloc(PN->nF, &F->tr);
        launch_fill<T>(Fnext.p, Fnext.n, T(0), s);
        Fn = Fnext.p;
        Vnext.alloc(PN->nV, &F->tr);
      }
      // close-out on the device from the level's pattern (uploaded at the
      // height start and still staged) and the next level's
      CloseLevel<T> cl{};
      {
        const SchurLevel<T>& SL = lvh[q];
        cl.pptr = SL.pptr;
        cl.pcol = SL.pcol;
        cl.poff = SL.poff;
        cl.kind = SL.kind;
        cl.n = SL.n;
        cl.r = rdev.p + I->rbase;
        cl.D = Sc->D.p;
        cl.F = I->Fbuf.p;
        std::vector<int32_t> par(Pc.nl);
        for (int j = 0; j < Pc.nl; ++j) par[j] = H.parent[Pc.a + j] - pa;
        cl.par = ar.put(par);
        cl.offc = ar.put(offc);
        cl.nl = Pc.nl;
        cl.a = Pc.a;
        cl.pa = pa;
        cl.nnz = (int64_t)Pc.pcol.size();
        cl.far_ptr = H.far_ptr_d.p;
        cl.far_col = H.far_col_d.p;
        cl.offS = H.offS_d.p;
        cl.offE = H.offE_d.p;
        cl.rank = H.rank_d.p;
        cl.data = I->data;
        cl.far0 = H.far_ptr[Pc.a];
        cl.nfar = H.far_ptr[Pc.a + Pc.nl] - cl.far0;
        if (is_top) {
          cl.top = 1;
          cl.top_off = ar.put(F->top_off);
          cl.ldtop = ldtop;
          cl.M = Dn;
        } else {
          cl.top = 0;
          cl.npptr = ar.put(PN->pptr);
          cl.npcol = ar.put(PN->pcol);
          cl.npoff = ar.put(PN->poff);
          cl.nkind = ar.put(level_kinds(*PN));
          cl.nn = ar.put(PN->n);
          cl.noffV = ar.put(PN->offV);
          cl.Dn = Dn;
          cl.Fn = Fn;
          cl.Vn = Vnext.p;
        }
        ar.flush(s);
      }
      flop_model.get();
      F->stats.levels = (int)F->plans.size() - (is_top ? 0 : 1);
      I->F->stats.max_colors = std::max(I->F->stats.max_colors, Pc.ncolors);
      plan_ms += ms_since(tpl);
      if (!is_top) launch_fill<T>(Vnext.p, Vnext.n, T(0), s);  // zero rows of [E_c; 0]
      {
        auto m6 = mark(6);
        launch_closeout<T>(cl, 0, ctx->d_err.p, s);
        launch_closeout<T>(cl, 1, ctx->d_err.p, s);
        close_mark(m6);
      }
      if (!is_top) {
        // the next level's F and V move to the instance; the current ones
        // are released here, stream-ordered after the close-out that reads them
        std::swap(I->Vbuf, Vnext);
        std::swap(I->Fbuf, Fnext);
        I->li = F->plans.size() - 1;
        I->lev = plev;
      } else {
        I->done = true;
        I->Fbuf.release();
        I->Vbuf.release();
      }
    }
    // staged descriptors of the level (patterns included) stay until here
    H2_HIP(hipStreamSynchronize(s));
    ar.reset();
    // the V fills must precede the E copies: the fills above were enqueued
    // before each instance's copy batch launch, so stream order holds.
    H2_HIP(hipGetLastError());
    for (auto& m : marks) {
      float ms = 0;
      H2_HIP(hipEventElapsedTime(&ms, std::get<1>(m), std::get<2>(m)));
      phase_ms[std::get<0>(m)] += ms;
    }
    marks.clear();
  }

  // ---- dense top factorization ----
  {
    CopyBatch<T> cb;
    for (auto& I : insts) {
      h2_factor_s* F = I.F;
      const h2_matrix_s& H = *I.H;
      if (I.tlev < 0) {
        // whole leaf level is the top block: assemble A from the leaf blocks
        const int a = H.lp[H.L], nl = H.lp[H.L + 1] - a;
        F->top_level = H.L;
        F->top_nodes.clear();
        F->top_off.assign(nl, 0);
        F->top_n.assign(nl, 0);
        int64_t o = 0;
        for (int t = 0; t < nl; ++t) {
          F->top_nodes.push_back(a + t);
          F->top_off[t] = o;
          F->top_n[t] = H.size(a + t);
          o += F->top_n[t];
        }
        F->n_top = o;
        DevArray<T>& M = top_of<T>(F);
        M.alloc(o * o, &F->tr);
        launch_fill<T>(M.p, o * o, T(0), s);
        for (int t = 0; t < nl; ++t)
          for (int64_t e = H.near_ptr[a + t]; e < H.near_ptr[a + t + 1]; ++e) {
            const int u = H.near_col[e] - a;
            cb.add(I.data + H.offD[e], F->top_n[t], M.p + F->top_off[t] + F->top_off[u] * o, o,
                   F->top_n[t], F->top_n[u], 0);
          }
      }
    }
    cb.launch(ar, s);
    hipEvent_t et0 = new_event();
    H2_HIP(hipEventRecord(et0, s));
    for (auto& I : insts) {
      h2_factor_s* F = I.F;
      const int64_t n = F->n_top;
      DevArray<T>& M = top_of<T>(F);
      F->top_piv.alloc(std::max<int64_t>(n, 1), &F->tr);
      const int nb = 64;
      for (int64_t j0 = 0; j0 < n; j0 += nb) {
        const int w = (int)std::min<int64_t>(nb, n - j0);
        launch_panel_lu<T>(M.p, n, n, j0, w, F->top_piv.p, ctx->d_err.p, s);
        launch_laswp<T>(M.p, n, n, j0, w, F->top_piv.p, j0, j0 + w, s);
        const int64_t rest = n - j0 - w;
        if (rest > 0) {
          // U12 = L11^{-1} A12
          launch_trsm_block<T>(M.p + j0 + j0 * n, n, M.p + j0 + (j0 + w) * n, n, w, rest, 1, s);
          // A22 -= L21 U12
          std::vector<GOut<T>> outs(1);
          std::vector<GCon<T>> cons(1);
          GOut<T>& o = outs[0];
          o = GOut<T>{};
          o.C = M.p + (j0 + w) + (j0 + w) * n;
          o.ldc = n;
          o.m = (int)rest;
          o.n = (int)rest;
          o.m0d = o.m1d = o.n0d = -1;
          o.cbeg = 0;
          o.cend = 1;
          o.tm = (int)((rest + 63) / 64);
          o.tn = (int)((rest + 63) / 64);
          o.tile0 = 0;
          o.alpha = T(-1);
          o.beta = T(1);
          GCon<T>& g = cons[0];
          g = GCon<T>{};
          g.A = M.p + (j0 + w) + j0 * n;
          g.lda = n;
          g.B = M.p + j0 + (j0 + w) * n;
          g.ldb = n;
          g.k = w;
          g.k0d = g.k1d = -1;
          const GOut<T>* dout = ar.put(outs);
          const GCon<T>* dcon = ar.put(cons);
          ar.flush(s);
          launch_gemm<T>(dout, 1, dcon, nullptr, (int64_t)o.tm * o.tn, 0, s);
        }
      }
      I.flops += 2.0 * (double)n * n * n / 3.0;
      I.pflops[7] += 2.0 * (double)n * n * n / 3.0;
      I.pbytes[7] += 2.0 * sizeof(T) * (double)n * n;
      launches[7] += 4 * ((n + 63) / 64);
    }
    hipEvent_t et1 = new_event();
    H2_HIP(hipEventRecord(et1, s));
    H2_HIP(hipEventSynchronize(et1));
    float ms = 0;
    H2_HIP(hipEventElapsedTime(&ms, et0, et1));
    phase_ms[7] += ms;
    int herr = 0;
    H2_HIP(hipMemcpy(&herr, ctx->d_err.p, sizeof(int), hipMemcpyDeviceToHost));
    if (herr & 1) throw H2Error(H2_ERROR_SINGULAR, "zero pivot in the dense top block");
    if (herr & 8)
      throw H2Error(H2_ERROR_FORMAT, "close-out destination missing from the next level");
    ar.reset();
  }
  phase_ms[8] = plan_ms;
  phase_ms[9] = ms_since(t_start);
  for (auto e : evpool) (void)hipEventDestroy(e);
  for (auto& I : insts) {
    h2_factor_s* F = I.F;
    for (int p = 0; p < H2_PHASES; ++p) {
      F->stats.time_ms[p] = phase_ms[p];
      F->stats.phase_flops[p] = I.pflops[p];
      F->stats.phase_bytes[p] = I.pbytes[p];
      F->stats.launches[p] = launches[p];
    }
    F->stats.n_top = F->n_top;
    F->stats.factor_flops = I.flops;
    F->stats.factor_bytes = F->tr.cur;
    F->stats.peak_bytes = F->tr.peak;
    F->stats.levels = (int)F->plans.size();
  }
}

std::vector<h2_factor_s*> factor(h2_context_s* ctx, const std::vector<h2_matrix_s*>& Hs,
                                 double tol, h2_prec prec, const h2_factor_opts& opts) {
  std::vector<h2_factor_s*> out;
  std::vector<std::unique_ptr<h2_factor_s>> own;
  // the call's byte accounting: every factor's storage and the shared
  // workspaces count against opts.pool_bytes
  DevTracker calltr;
  calltr.mem = &ctx->mem;
  calltr.cap = opts.pool_bytes;
  struct Detach {  // factors outlive the call's tracker
    std::vector<std::unique_ptr<h2_factor_s>>& fs;
    ~Detach() {
      for (auto& f : fs)
        if (f) f->tr.parent = nullptr;
    }
  } detach{own};
  for (auto* H : Hs) {
    own.emplace_back(new h2_factor_s());
    h2_factor_s* F = own.back().get();
    F->ctx = ctx;
    F->prec = prec;
    F->tr.mem = &ctx->mem;
    F->tr.parent = &calltr;
    F->keep_owners = opts.keep_owner_lists != 0;
    F->N = H->N;
    F->L = H->L;
    F->top = H->top;
    F->ib = H->ib;
    F->ie = H->ie;
    F->lp = H->lp;
    F->parent = H->parent;
    F->cp = H->cp;
    F->perm_d.alloc(H->N, &F->tr);
    H2_HIP(hipMemcpyAsync(F->perm_d.p, H->perm_d.p, sizeof(int64_t) * H->N,
                          hipMemcpyDeviceToDevice, ctx->stream));
  }
  auto norm_of = [&](const h2_matrix_s* H) { return opts.norm2 > 0 ? opts.norm2 : H->norm2; };
  // LDS bytes per workgroup the kernels' path choices assume
  const int lds = opts.lds_limit_kib > 0 ? std::min(kLdsBytes, opts.lds_limit_kib * 1024) : kLdsBytes;
  if (prec == H2_PREC_FP64) {
    std::vector<Inst<double>> insts(Hs.size());
    for (size_t i = 0; i < Hs.size(); ++i) {
      insts[i].H = Hs[i];
      insts[i].F = own[i].get();
      insts[i].data = Hs[i]->data.p;
      insts[i].norm = norm_of(Hs[i]);
    }
    run_factor<double>(ctx, insts, tol, &calltr, lds);
  } else {
    std::vector<Inst<float>> insts(Hs.size());
    for (size_t i = 0; i < Hs.size(); ++i) {
      insts[i].H = Hs[i];
      insts[i].F = own[i].get();
      insts[i].data_conv.alloc(Hs[i]->ndata, &calltr);
      launch_convert<float>(insts[i].data_conv.p, Hs[i]->data.p, Hs[i]->ndata, ctx->stream);
      insts[i].data = insts[i].data_conv.p;
      insts[i].norm = norm_of(Hs[i]);
    }
    run_factor<float>(ctx, insts, tol, &calltr, lds);
  }
  H2_HIP(hipStreamSynchronize(ctx->stream));
  for (auto& p : own) {
    p->stats.peak_bytes = calltr.peak;
    p->tr.parent = nullptr;
  }
  for (auto& p : own) out.push_back(p.release());
  return out;
}

}  // namespace h2drv
