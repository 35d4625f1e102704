// Host-side objects of the H^2 library (not part of the ABI).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <deque>
#include <memory>
#include <stdexcept>
#include <string>
#include <vector>

#include "h2.h"
#include "h2_kernels.h"

struct H2Error : std::runtime_error {
  h2_status code;
  H2Error(h2_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define H2_HIP(call)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess)                                                              \
      throw H2Error(e_ == hipErrorOutOfMemory ? H2_ERROR_OUT_OF_MEMORY : H2_ERROR_HIP, \
                    std::string(#call) + ": " + hipGetErrorString(e_));                \
  } while (0)

// Device memory of a context: the caller's allocator callbacks, or the
// device's default stream-ordered memory pool (hipMallocAsync / hipFreeAsync
// on the context's stream, freed blocks kept in the pool for reuse).  Either
// way a block released here may be handed out again to later work of the
// same stream, so releases need no synchronisation.
struct DevMem {
  h2_alloc_fn fa = nullptr;
  h2_free_fn ff = nullptr;
  void* user = nullptr;
  hipStream_t s = nullptr;
  void* get(size_t bytes) {
    void* p = nullptr;
    if (fa) {
      p = fa(bytes, (void*)s, user);
    } else if (hipMallocAsync(&p, bytes, s) != hipSuccess) {
      p = nullptr;
      (void)hipGetLastError();
    }
    if (!p)
      throw H2Error(H2_ERROR_OUT_OF_MEMORY,
                    "device allocation of " + std::to_string(bytes) + " bytes failed");
    return p;
  }
  void put(void* p, size_t bytes) {
    if (!p) return;
    if (ff)
      ff(p, bytes, (void*)s, user);
    else
      (void)hipFreeAsync(p, s);
  }
};

// Byte accounting of one owner (a matrix, a factor, a context's work
// arrays).  `cap` > 0 limits the bytes held at once; a tracker with a parent
// also counts against the parent (one factorization call over several
// instances shares one cap).
struct DevTracker {
  DevMem* mem = nullptr;
  int64_t cur = 0, peak = 0, cap = 0;
  DevTracker* parent = nullptr;
  void add(int64_t b) {
    for (DevTracker* t = this; t; t = t->parent)
      if (t->cap > 0 && t->cur + b > t->cap)
        throw H2Error(H2_ERROR_OUT_OF_MEMORY,
                      "device memory cap of " + std::to_string(t->cap) + " bytes reached (" +
                          std::to_string(t->cur) + " held, " + std::to_string(b) + " requested)");
    for (DevTracker* t = this; t; t = t->parent) {
      t->cur += b;
      if (t->cur > t->peak) t->peak = t->cur;
    }
  }
  void sub(int64_t b) {
    for (DevTracker* t = this; t; t = t->parent) t->cur -= b;
  }
};

template <class T> struct DevArray {
  T* p = nullptr;
  int64_t n = 0;
  DevTracker* tr = nullptr;
  DevArray() = default;
  DevArray(const DevArray&) = delete;
  DevArray& operator=(const DevArray&) = delete;
  DevArray(DevArray&& o) noexcept : p(o.p), n(o.n), tr(o.tr) {
    o.p = nullptr;
    o.n = 0;
  }
  DevArray& operator=(DevArray&& o) noexcept {
    if (this != &o) {
      release();
      p = o.p;
      n = o.n;
      tr = o.tr;
      o.p = nullptr;
      o.n = 0;
    }
    return *this;
  }
  ~DevArray() { release(); }
  void alloc(int64_t count, DevTracker* t) {
    release();
    tr = t;
    if (count > 0) {
      const int64_t b = (int64_t)sizeof(T) * count;
      tr->add(b);
      try {
        p = (T*)tr->mem->get((size_t)b);
      } catch (...) {
        tr->sub(b);
        throw;
      }
      n = count;
    }
  }
  void release() {
    if (p) {
      tr->mem->put(p, (size_t)bytes());
      tr->sub(bytes());
    }
    p = nullptr;
    n = 0;
  }
  int64_t bytes() const { return (int64_t)sizeof(T) * n; }
};

// Descriptor arrays staged through pinned host memory into device memory.
// put() copies an array into the pinned staging chunk and returns the device
// address it will have; flush() issues one asynchronous copy per chunk for
// everything put since the last flush, so a launch group's descriptors
// travel in one transfer (flush before the launches that read them).
// Chunks are only ever added: every array put since the last reset() stays
// valid (several puts feed one launch, and launches queue behind each other),
// so reset() may be called only once the stream has finished all work that
// reads them.
struct DescArena {
  struct Chunk {
    char* h = nullptr;
    char* d = nullptr;
    size_t cap = 0;
    size_t used = 0;     // bytes staged
    size_t flushed = 0;  // bytes whose copy has been issued
  };
  std::vector<Chunk> chunks;
  size_t cur = 0;  // chunk being filled
  hipStream_t s = nullptr;
  DevMem* mem = nullptr;
  ~DescArena() { free_all(); }
  void free_all() {
    for (auto& c : chunks) {
      if (c.h) (void)hipHostFree(c.h);
      if (c.d) mem->put(c.d, c.cap);
    }
    chunks.clear();
    cur = 0;
  }
  void reset() {
    for (auto& c : chunks) c.used = c.flushed = 0;
    cur = 0;
  }
  template <class X> X* put(const std::vector<X>& v) {
    if (v.empty()) return nullptr;
    const size_t bytes = sizeof(X) * v.size();
    const size_t need = (bytes + 255) & ~(size_t)255;
    while (cur < chunks.size() && chunks[cur].used + need > chunks[cur].cap) ++cur;
    if (cur == chunks.size()) {
      Chunk c;
      c.cap = std::max(need, (size_t)64 << 20);
      H2_HIP(hipHostMalloc((void**)&c.h, c.cap, hipHostMallocDefault));
      try {
        c.d = (char*)mem->get(c.cap);
      } catch (...) {
        (void)hipHostFree(c.h);
        throw;
      }
      chunks.push_back(c);
    }
    Chunk& c = chunks[cur];
    std::memcpy(c.h + c.used, v.data(), bytes);
    X* out = reinterpret_cast<X*>(c.d + c.used);
    c.used += need;
    return out;
  }
  // issue the copies of everything staged since the last flush
  void flush(hipStream_t st) {
    for (size_t q = 0; q <= cur && q < chunks.size(); ++q) {
      Chunk& c = chunks[q];
      if (c.used > c.flushed) {
        H2_HIP(hipMemcpyAsync(c.d + c.flushed, c.h + c.flushed, c.used - c.flushed,
                              hipMemcpyHostToDevice, st));
        c.flushed = c.used;
      }
    }
  }
};

// a recorded launch sequence (a solve kept with its factor, a product kept
// with its matrix; h2_solve.cpp)
struct PlanBase {
  virtual ~PlanBase() = default;
  virtual int64_t uses() const = 0;        // calls served by the plan
  virtual int64_t graph_uses() const = 0;  // of those, one graph launch each
};

struct h2_context_s {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;  // created by the context (destroyed with it)
  std::string err;
  DevMem mem;
  DevTracker tr;            // the context's own work arrays
  DevArray<int> d_err;      // device error word: bit0 zero pivot, bit1 non-finite,
                            // bit2 Schur contributors, bit3 close-out destination
  DescArena arena;
  // partial tiles of split skinny GEMMs (grown on demand, after a stream sync)
  DevArray<float> parts32;
  DevArray<double> parts64;
};

template <class T> DevArray<T>& parts_of(h2_context_s* ctx);
template <> inline DevArray<float>& parts_of<float>(h2_context_s* ctx) { return ctx->parts32; }
template <> inline DevArray<double>& parts_of<double>(h2_context_s* ctx) { return ctx->parts64; }

struct h2_matrix_s {
  h2_context_s* ctx = nullptr;
  int64_t N = 0;
  int dim = 0, L = 0, nn = 0, top = -1;
  double norm2 = 0;
  std::vector<int64_t> perm, ib, ie;
  std::vector<int> lp, parent, cp, rank;
  std::vector<int64_t> near_ptr, far_ptr;
  std::vector<int> near_col, far_col;
  std::vector<int64_t> offU, offE, offD, offS;  // element offsets in the data array
  int64_t ndata = 0;
  DevTracker tr;
  DevArray<double> data;
  DevArray<int64_t> perm_d;
  // structure the level close-out reads on the device
  DevArray<int64_t> far_ptr_d, offS_d, offE_d;
  DevArray<int32_t> far_col_d, rank_d;
  int size(int q) const { return (int)(ie[q] - ib[q]); }
  int level_of(int q) const {
    int l = 0;
    while (l + 1 < (int)lp.size() && lp[l + 1] <= q) ++l;
    return l;
  }
  // matvec layout (built lazily) and the last recorded product
  bool mv_ready = false;
  std::vector<int64_t> hat_off;  // per node offset (in units of rank) into the hat vectors
  int64_t hat_total = 0;
  std::unique_ptr<PlanBase> mvplan;
};

// ---- factorization data of one skeletonized level of one matrix ----
struct LevelPlan {
  int lev = 0, a = 0, nl = 0;
  std::vector<int> n, k, color;
  int ncolors = 0;
  std::vector<std::vector<int>> members;  // by colour, ascending local id
  std::vector<std::vector<int>> nb;       // near lists (local, sorted, incl. self)
  // pattern = near U fill, CSR over local rows, sorted columns
  std::vector<int64_t> pptr;
  std::vector<int> pcol;
  std::vector<char> isF;
  std::vector<int64_t> poff;   // element offset in the D or F buffer (a fill entry (j, k)
                               // with k < j: offset of the stored block (k, j))
  std::vector<int> firstc;     // fill entries: first colour that writes it (-1 lifted)
  std::vector<int64_t> offQ, offV, offPiv;
  std::vector<int64_t> xoff;   // near entry (i, k): offset of its multiplier copy in the
                               // colour's copy area (when the Schur update reads copies)
  int64_t nX = 0;              // largest copy area of a colour
  int64_t nD = 0, nF = 0, nQ = 0, nV = 0, nPiv = 0;
  std::vector<int> r;          // redundant counts (host copy after the level)
  std::vector<std::pair<int, int>> fill_pairs;  // (j, k) local, sorted (integer output)
  // Schur target lists, kept on request: records (c, j, k, m, i_1..i_m), global ids
  std::vector<int64_t> owners;
  // fill is stored once per unordered pair, as the block (j, k) with j < k;
  // entry e of row j is then the transpose of its stored block
  bool tr(int j, int64_t e) const { return isF[e] && pcol[e] < j; }
  int64_t find(int i, int j) const {
    int64_t lo = pptr[i], hi = pptr[i + 1];
    while (lo < hi) {
      int64_t mid = (lo + hi) / 2;
      if (pcol[mid] < j) lo = mid + 1; else hi = mid;
    }
    return (lo < pptr[i + 1] && pcol[lo] == j) ? lo : -1;
  }
};

template <class T> struct LevelStore {
  DevArray<T> D, F, Q, V;
  DevArray<int32_t> piv;
};


struct h2_factor_s {
  h2_context_s* ctx = nullptr;
  h2_prec prec = H2_PREC_FP64;
  int64_t N = 0;
  int L = 0, top = -1, top_level = 0;
  std::vector<int64_t> ib, ie;
  std::vector<int> lp, parent, cp;
  DevArray<int64_t> perm_d;
  std::deque<LevelPlan> plans;           // leaf level first (stable references)
  std::vector<LevelStore<double>> st64;  // per level (FP64 factors)
  std::vector<LevelStore<float>> st32;   // per level (FP32 factors)
  // top
  int64_t n_top = 0;
  std::vector<int> top_nodes;
  std::vector<int64_t> top_off;
  std::vector<int> top_n;
  DevArray<double> M64;
  DevArray<float> M32;
  DevArray<int32_t> top_piv;
  DevTracker tr;
  h2_stats stats{};
  bool keep_owners = false;
  std::unique_ptr<PlanBase> splan;  // last recorded solve
};
