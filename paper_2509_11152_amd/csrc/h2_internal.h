// Host-side objects of the H^2 library (not part of the ABI).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
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

// device allocation with byte accounting
struct DevTracker {
  int64_t cur = 0, peak = 0;
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
    n = count;
    if (count > 0) {
      hipError_t e = hipMalloc((void**)&p, sizeof(T) * (size_t)count);
      if (e != hipSuccess) {
        p = nullptr;
        n = 0;
        (void)hipGetLastError();
        throw H2Error(H2_ERROR_OUT_OF_MEMORY,
                      "device allocation of " + std::to_string(sizeof(T) * count) + " bytes failed");
      }
      if (tr) {
        tr->cur += (int64_t)sizeof(T) * count;
        if (tr->cur > tr->peak) tr->peak = tr->cur;
      }
    }
  }
  void release() {
    if (p) {
      (void)hipFree(p);
      if (tr) tr->cur -= (int64_t)sizeof(T) * n;
    }
    p = nullptr;
    n = 0;
  }
  int64_t bytes() const { return (int64_t)sizeof(T) * n; }
};

// Descriptor arrays staged through pinned host memory into device memory.
// Chunks are only ever added: every array put since the last reset() stays
// valid (several puts feed one launch, and launches queue behind each other),
// so reset() may be called only once the stream has finished all work that
// reads them.
struct DescArena {
  struct Chunk {
    char* h = nullptr;
    char* d = nullptr;
    size_t cap = 0;
  };
  std::vector<Chunk> chunks;
  size_t cur = 0, used = 0;  // chunk being filled and bytes used in it
  hipStream_t s = nullptr;
  ~DescArena() { free_all(); }
  void free_all() {
    for (auto& c : chunks) {
      if (c.h) (void)hipHostFree(c.h);
      if (c.d) (void)hipFree(c.d);
    }
    chunks.clear();
    cur = used = 0;
  }
  void reset() { cur = used = 0; }
  template <class X> X* put(const std::vector<X>& v) {
    if (v.empty()) return nullptr;
    const size_t bytes = sizeof(X) * v.size();
    const size_t need = (bytes + 255) & ~(size_t)255;
    while (cur < chunks.size() && used + need > chunks[cur].cap) {
      ++cur;
      used = 0;
    }
    if (cur == chunks.size()) {
      Chunk c;
      c.cap = std::max(need, (size_t)64 << 20);
      H2_HIP(hipHostMalloc((void**)&c.h, c.cap, hipHostMallocDefault));
      hipError_t e = hipMalloc((void**)&c.d, c.cap);
      if (e != hipSuccess) {
        (void)hipHostFree(c.h);
        (void)hipGetLastError();
        throw H2Error(H2_ERROR_OUT_OF_MEMORY, "descriptor arena allocation failed");
      }
      chunks.push_back(c);
      used = 0;
    }
    Chunk& c = chunks[cur];
    std::memcpy(c.h + used, v.data(), bytes);
    H2_HIP(hipMemcpyAsync(c.d + used, c.h + used, bytes, hipMemcpyHostToDevice, s));
    X* out = reinterpret_cast<X*>(c.d + used);
    used += need;
    return out;
  }
};

struct h2_context_s {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;
  int* d_err = nullptr;  // device error word: bit0 zero pivot, bit1 non-finite
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
  int size(int q) const { return (int)(ie[q] - ib[q]); }
  int level_of(int q) const {
    int l = 0;
    while (l + 1 < (int)lp.size() && lp[l + 1] <= q) ++l;
    return l;
  }
  // matvec plan (built lazily)
  bool mv_ready = false;
  std::vector<int64_t> hat_off;  // per node offset (in units of rank) into the hat vectors
  int64_t hat_total = 0;
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
  std::vector<int64_t> poff;   // element offset in the D or F buffer
  std::vector<int> firstc;     // fill entries: first colour that writes it (-1 lifted)
  std::vector<int64_t> offQ, offV, offPiv;
  int64_t nD = 0, nF = 0, nQ = 0, nV = 0, nPiv = 0;
  std::vector<int> r;          // redundant counts (host copy after the level)
  std::vector<std::pair<int, int>> fill_pairs;  // (j, k) local, sorted (integer output)
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

// a solve's recorded launch sequence, kept with its factor (h2_solve.cpp)
struct SolvePlanBase {
  virtual ~SolvePlanBase() = default;
};

struct h2_factor_s {
  h2_context_s* ctx = nullptr;
  h2_prec prec = H2_PREC_FP64;
  int64_t N = 0;
  int L = 0, top = -1, top_level = 0;
  std::vector<int64_t> ib, ie;
  std::vector<int> lp, parent, cp;
  DevArray<int64_t> perm_d;
  std::vector<LevelPlan> plans;          // leaf level first
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
  std::unique_ptr<SolvePlanBase> splan;  // last recorded solve
};
