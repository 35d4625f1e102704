// C-ABI entry points: contexts, loading and validation of the serialized H^2
// matrix, the FP64 H^2 matrix-vector product, statistics and integer exports.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <atomic>
#include <mutex>
#include <thread>

#include "h2_driver.h"
#include "h2_internal.h"

namespace {

template <class F> h2_status guard(h2_context_s* ctx, F&& f) {
  try {
    f();
    return H2_SUCCESS;
  } catch (const H2Error& e) {
    if (ctx) ctx->err = e.what();
    return e.code;
  } catch (const std::bad_alloc&) {
    if (ctx) ctx->err = "host allocation failed";
    return H2_ERROR_OUT_OF_MEMORY;
  } catch (const std::exception& e) {
    if (ctx) ctx->err = e.what();
    return H2_ERROR_HIP;
  }
}

void fail_format(const std::string& m) { throw H2Error(H2_ERROR_FORMAT, m); }

// ---- scratch of the allocation-free product (h2_matvec_noalloc) ----
// A file-scope device array: every GPU the library runs on holds its own copy
// until the process ends.  Host code never passes the array's name to a kernel
// or a copy (on the host it is only a stand-in for the symbol); its device
// address on each device is looked up once, at the first context created on
// that device, and kept in g_scratch.
constexpr int64_t kNoAllocScratchBytes = (int64_t)64 << 20;
static __device__ __align__(256) char scratch[kNoAllocScratchBytes];
constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch[kMaxScratchDevices] = {};
hipError_t g_scratch_err[kMaxScratchDevices] = {};

// with `dev` current: look up this device's copy of the array (once)
void map_scratch(int dev) {
  if (dev < 0 || dev >= kMaxScratchDevices) return;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch[dev]) return;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  g_scratch_err[dev] = e;
  if (e == hipSuccess) g_scratch[dev] = p;
}

void* scratch_of(int dev) {
  if (dev < 0 || dev >= kMaxScratchDevices)
    throw H2Error(H2_ERROR_UNSUPPORTED, "no allocation-free scratch for device " +
                                            std::to_string(dev));
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch[dev])
    throw H2Error(H2_ERROR_HIP, std::string("hipGetSymbolAddress of the scratch array: ") +
                                    hipGetErrorString(g_scratch_err[dev]));
  return g_scratch[dev];
}

struct Reader {
  const uint8_t* p;
  size_t n, off;
  template <class X> std::vector<X> take(int64_t count) {
    if (count < 0) fail_format("negative section length");
    size_t bytes = sizeof(X) * (size_t)count;
    if (off + bytes > n) fail_format("blob truncated");
    std::vector<X> v((size_t)count);
    if (bytes) std::memcpy(v.data(), p + off, bytes);
    off = (off + bytes + 7) & ~(size_t)7;
    return v;
  }
};

template <class X> X rd(const uint8_t* p, size_t off) {
  X v;
  std::memcpy(&v, p + off, sizeof(X));
  return v;
}

// Parse and validate the structure of an H2B1 v1 blob.
void parse(const uint8_t* p, size_t bytes, h2_matrix_s& H) {
  if (bytes < 128) fail_format("blob shorter than its header");
  if (std::memcmp(p, "H2B1", 4) != 0) fail_format("bad magic");
  if (rd<uint32_t>(p, 4) != 1) fail_format("unsupported version");
  if (!(rd<uint32_t>(p, 8) & 1)) fail_format("only symmetric matrices are supported");
  H.dim = (int)rd<uint32_t>(p, 12);
  H.N = rd<int64_t>(p, 16);
  H.L = rd<int32_t>(p, 24);
  H.nn = rd<int32_t>(p, 28);
  H.norm2 = rd<double>(p, 32);
  const int64_t nnz_near = rd<int64_t>(p, 64), nnz_far = rd<int64_t>(p, 72);
  const int64_t total = rd<int64_t>(p, 80);
  if ((size_t)total != bytes) fail_format("blob length does not match its header");
  if (H.N <= 0 || H.L < 0 || H.nn <= 0 || nnz_near <= 0 || nnz_far < 0)
    fail_format("bad sizes in header");
  if (!(H.norm2 > 0) || !std::isfinite(H.norm2)) fail_format("bad norm estimate");
  Reader R{p, bytes, 128};
  H.perm = R.take<int64_t>(H.N);
  H.lp = R.take<int32_t>(H.L + 2);
  H.parent = R.take<int32_t>(H.nn);
  H.cp = R.take<int32_t>(H.nn + 1);
  H.ib = R.take<int64_t>(H.nn);
  H.ie = R.take<int64_t>(H.nn);
  H.rank = R.take<int32_t>(H.nn);
  H.near_ptr = R.take<int64_t>(H.nn + 1);
  H.near_col = R.take<int32_t>(nnz_near);
  H.far_ptr = R.take<int64_t>(H.nn + 1);
  H.far_col = R.take<int32_t>(nnz_far);
  // tree
  if (H.lp[0] != 0 || H.lp[1] != 1 || H.lp[H.L + 1] != H.nn) fail_format("bad level pointers");
  for (int l = 0; l <= H.L; ++l)
    if (H.lp[l + 1] <= H.lp[l]) fail_format("empty level");
  {
    std::vector<char> seen((size_t)H.N, 0);
    for (int64_t v : H.perm) {
      if (v < 0 || v >= H.N || seen[(size_t)v]) fail_format("perm is not a permutation");
      seen[(size_t)v] = 1;
    }
  }
  if (H.parent[0] != -1 || H.ib[0] != 0 || H.ie[0] != H.N) fail_format("bad root");
  for (int l = 0; l <= H.L; ++l) {
    for (int q = H.lp[l]; q < H.lp[l + 1]; ++q) {
      if (H.ib[q] > H.ie[q]) fail_format("bad index range");
      if (q > H.lp[l] && H.ib[q] != H.ie[q - 1]) fail_format("level ranges do not tile");
      if (H.rank[q] < 0 || H.rank[q] > H.ie[q] - H.ib[q]) fail_format("bad rank");
      const int c0 = H.cp[q], c1 = H.cp[q + 1];
      if (l == H.L) {
        if (c1 != c0) fail_format("unbalanced tree: leaf with children");
      } else {
        if (c1 <= c0) fail_format("unbalanced tree: inner node without children");
        if (c0 < H.lp[l + 1] || c1 > H.lp[l + 2]) fail_format("children not on the next level");
        if (H.ib[c0] != H.ib[q] || H.ie[c1 - 1] != H.ie[q]) fail_format("children do not tile");
        for (int c = c0; c < c1; ++c)
          if (H.parent[c] != q) fail_format("parent/child mismatch");
      }
    }
    if (H.ib[H.lp[l]] != 0 || H.ie[H.lp[l + 1] - 1] != H.N) fail_format("level does not cover");
  }
  if (H.cp[0] != 1) fail_format("bad child pointer");
  // lists: sorted, same level, symmetric, diagonal present in near
  auto check_csr = [&](const std::vector<int64_t>& ptr, const std::vector<int32_t>& col,
                       bool is_near) {
    if (ptr[0] != 0 || ptr[H.nn] != (int64_t)col.size()) fail_format("bad CSR pointers");
    for (int q = 0; q < H.nn; ++q) {
      if (ptr[q + 1] < ptr[q]) fail_format("bad CSR pointers");
      const int l = H.level_of(q);
      bool diag = false;
      for (int64_t e = ptr[q]; e < ptr[q + 1]; ++e) {
        const int j = col[e];
        if (j < H.lp[l] || j >= H.lp[l + 1]) fail_format("pair across levels");
        if (e > ptr[q] && col[e - 1] >= j) fail_format("unsorted list");
        if (j == q) diag = true;
        // symmetric pattern
        const auto b = col.begin() + ptr[j], en = col.begin() + ptr[j + 1];
        if (!std::binary_search(b, en, q)) fail_format("pattern is not symmetric");
      }
      if (is_near && !diag && ptr[q + 1] > ptr[q]) fail_format("near list misses the diagonal");
      if (!is_near && diag) fail_format("far list contains the diagonal");
    }
  };
  check_csr(H.near_ptr, H.near_col, true);
  check_csr(H.far_ptr, H.far_col, false);
  if (H.near_ptr[1] - H.near_ptr[0] != 1) fail_format("root must be near itself");
  // data offsets
  int64_t off = 0;
  const int leaf0 = H.lp[H.L];
  H.offU.assign(H.nn, -1);
  for (int q = leaf0; q < H.nn; ++q) {
    H.offU[q] = off;
    off += (int64_t)H.size(q) * H.rank[q];
  }
  H.offE.assign(H.nn, -1);
  for (int c = 1; c < H.nn; ++c) {
    H.offE[c] = off;
    off += (int64_t)H.rank[c] * H.rank[H.parent[c]];
  }
  H.offD.assign(H.near_col.size(), -1);
  for (int q = leaf0; q < H.nn; ++q)
    for (int64_t e = H.near_ptr[q]; e < H.near_ptr[q + 1]; ++e) {
      H.offD[e] = off;
      off += (int64_t)H.size(q) * H.size(H.near_col[e]);
    }
  H.offS.assign(H.far_col.size(), -1);
  for (int q = 0; q < H.nn; ++q)
    for (int64_t e = H.far_ptr[q]; e < H.far_ptr[q + 1]; ++e) {
      H.offS[e] = off;
      off += (int64_t)H.rank[q] * H.rank[H.far_col[e]];
    }
  if ((size_t)R.off + (size_t)off * 8 != bytes) fail_format("data section size mismatch");
  H.ndata = off;
  H.top = -1;
  for (int l = 0; l <= H.L && H.top < 0; ++l)
    if (H.far_ptr[H.lp[l + 1]] > H.far_ptr[H.lp[l]]) H.top = l;
}


// f(lo, hi) over [0, n) in contiguous ranges on up to 8 threads
template <class Fn> void par_ranges(int64_t n, Fn f) {
  const int hw = (int)std::max(1u, std::min(8u, std::thread::hardware_concurrency()));
  const int nt = (int)std::max<int64_t>(1, std::min<int64_t>(hw, n / 64));
  if (nt == 1) {
    f((int64_t)0, n);
    return;
  }
  std::vector<std::thread> th;
  for (int t = 1; t < nt; ++t) th.emplace_back(f, n * t / nt, n * (t + 1) / nt);
  f((int64_t)0, n / nt);
  for (auto& x : th) x.join();
}

// Numerical checks of the data section: finite entries, orthonormal leaf
// bases and stacked transfers, symmetric near blocks and couplings.
void check_data(const double* d, const h2_matrix_s& H) {
  std::atomic<int> bad{0};
  par_ranges(H.ndata, [&](int64_t a, int64_t b) {
    for (int64_t i = a; i < b; ++i)
      if (!std::isfinite(d[i])) {
        bad = 1;
        return;
      }
  });
  if (bad) fail_format("non-finite matrix entry");
  constexpr double kOrth = 1e-10;
  // max |G - I| of G = sum over blocks of B^T B (blocks of `rows` x k, column-major)
  auto gram_dev = [](const std::vector<std::pair<const double*, int>>& blocks, int k) {
    double dev = 0;
    for (int a = 0; a < k; ++a)
      for (int b = 0; b <= a; ++b) {
        double g = 0;
        for (const auto& bl : blocks) {
          const double* x = bl.first + (int64_t)a * bl.second;
          const double* y = bl.first + (int64_t)b * bl.second;
          for (int r = 0; r < bl.second; ++r) g += x[r] * y[r];
        }
        dev = std::max(dev, std::fabs(g - (a == b ? 1.0 : 0.0)));
      }
    return dev;
  };
  const int leaf0 = H.lp[H.L];
  std::atomic<int> which{0};
  par_ranges(H.nn, [&](int64_t a, int64_t b) {
    for (int64_t q = a; q < b && !which; ++q) {
      const int k = H.rank[q];
      if (k == 0) continue;
      std::vector<std::pair<const double*, int>> blocks;
      if (q >= leaf0) {
        blocks.push_back({d + H.offU[q], H.size((int)q)});
      } else {
        for (int c = H.cp[q]; c < H.cp[q + 1]; ++c)
          if (H.rank[c] > 0) blocks.push_back({d + H.offE[c], H.rank[c]});
      }
      if (gram_dev(blocks, k) > kOrth) which = q >= leaf0 ? 1 : 2;
    }
  });
  if (which == 1) fail_format("leaf basis U is not orthonormal (max |U^T U - I| > 1e-10)");
  if (which == 2)
    fail_format("stacked transfers are not orthonormal (max |sum E_c^T E_c - I| > 1e-10)");
  // symmetric values: block (j, i) equals the transpose of block (i, j)
  const double tol = 1e-12 * H.norm2;
  auto sym = [&](const std::vector<int64_t>& ptr, const std::vector<int32_t>& col,
                 const std::vector<int64_t>& off, bool dense, int q0) {
    std::atomic<int> asym{0};
    par_ranges(H.nn - q0, [&](int64_t a, int64_t b) {
      for (int64_t qq = a; qq < b && !asym; ++qq) {
        const int q = q0 + (int)qq;
        for (int64_t e = ptr[q]; e < ptr[q + 1]; ++e) {
          const int j = col[e];
          if (j < q) continue;
          const auto bj = col.begin() + ptr[j], ej = col.begin() + ptr[j + 1];
          const int64_t et = ptr[j] + (std::lower_bound(bj, ej, q) - bj);
          const int m = dense ? H.size(q) : H.rank[q];
          const int n = dense ? H.size(j) : H.rank[j];
          const double* x = d + off[e];   // m x n
          const double* y = d + off[et];  // n x m
          for (int c = 0; c < n; ++c)
            for (int r = 0; r < m; ++r)
              if (std::fabs(x[r + (int64_t)c * m] - y[c + (int64_t)r * n]) > tol) asym = 1;
        }
      }
    });
    return asym != 0;
  };
  if (sym(H.near_ptr, H.near_col, H.offD, true, leaf0))
    fail_format("near blocks are not symmetric (D_ji != D_ij^T)");
  if (sym(H.far_ptr, H.far_col, H.offS, false, 0))
    fail_format("couplings are not symmetric (S_ji != S_ij^T)");
}

}  // namespace

extern "C" {

const char* h2_status_string(h2_status s) {
  switch (s) {
    case H2_SUCCESS: return "success";
    case H2_ERROR_INVALID_ARGUMENT: return "invalid argument";
    case H2_ERROR_FORMAT: return "malformed serialized matrix";
    case H2_ERROR_OUT_OF_MEMORY: return "out of device memory";
    case H2_ERROR_SINGULAR: return "singular pivot";
    case H2_ERROR_NUMERIC: return "non-finite value";
    case H2_ERROR_HIP: return "HIP runtime error";
    case H2_ERROR_NOT_CONVERGED: return "refinement did not converge";
    case H2_ERROR_UNSUPPORTED: return "unsupported size";
  }
  return "unknown status";
}

h2_status h2_context_create(const h2_context_opts* opts, h2_context_t* out) {
  if (!out) return H2_ERROR_INVALID_ARGUMENT;
  *out = nullptr;
  h2_context_opts o{0, nullptr, nullptr, nullptr, nullptr};
  if (opts) o = *opts;
  if ((o.alloc == nullptr) != (o.free == nullptr)) return H2_ERROR_INVALID_ARGUMENT;
  auto* ctx = new (std::nothrow) h2_context_s();
  if (!ctx) return H2_ERROR_OUT_OF_MEMORY;
  h2_status st = guard(nullptr, [&] {
    int count = 0;
    H2_HIP(hipGetDeviceCount(&count));
    if (o.device < 0 || o.device >= count) throw H2Error(H2_ERROR_INVALID_ARGUMENT, "bad device");
    H2_HIP(hipSetDevice(o.device));
    ctx->device = o.device;
    if (o.stream) {
      ctx->stream = (hipStream_t)o.stream;
    } else {
      H2_HIP(hipStreamCreate(&ctx->stream));
      ctx->own_stream = true;
    }
    if (!o.alloc) {
      // keep freed blocks of the default pool cached instead of returning
      // them to the device at every synchronisation
      hipMemPool_t pool = nullptr;
      H2_HIP(hipDeviceGetDefaultMemPool(&pool, o.device));
      uint64_t thr = UINT64_MAX;
      H2_HIP(hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr));
    }
    ctx->mem.fa = o.alloc;
    ctx->mem.ff = o.free;
    ctx->mem.user = o.user;
    ctx->mem.s = ctx->stream;
    ctx->tr.mem = &ctx->mem;
    ctx->arena.s = ctx->stream;
    ctx->arena.mem = &ctx->mem;
    ctx->d_err.alloc(1, &ctx->tr);
    h2k::launch_fill<int32_t>(ctx->d_err.p, 1, 0, ctx->stream);
    H2_HIP(hipStreamSynchronize(ctx->stream));
    map_scratch(o.device);
  });
  if (st != H2_SUCCESS) {
    if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
    delete ctx;
    return st;
  }
  *out = ctx;
  return H2_SUCCESS;
}

h2_status h2_context_destroy(h2_context_t ctx) {
  if (!ctx) return H2_ERROR_INVALID_ARGUMENT;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  ctx->arena.free_all();
  ctx->parts32.release();
  ctx->parts64.release();
  ctx->d_err.release();
  (void)hipStreamSynchronize(ctx->stream);
  const hipStream_t s = ctx->stream;
  const bool own = ctx->own_stream;
  delete ctx;
  if (own) (void)hipStreamDestroy(s);
  return H2_SUCCESS;
}

const char* h2_last_error(h2_context_t ctx) { return ctx ? ctx->err.c_str() : "no context"; }

h2_status h2_sync(h2_context_t ctx) {
  if (!ctx) return H2_ERROR_INVALID_ARGUMENT;
  return guard(ctx, [&] { H2_HIP(hipStreamSynchronize(ctx->stream)); });
}

h2_status h2_blob_check(const void* blob, size_t bytes, char* msg, size_t msgcap) {
  if (msg && msgcap) msg[0] = 0;
  if (!blob) return H2_ERROR_INVALID_ARGUMENT;
  h2_matrix_s H;
  std::string err;
  h2_status st = H2_SUCCESS;
  try {
    const uint8_t* p = (const uint8_t*)blob;
    parse(p, bytes, H);
    check_data((const double*)(p + bytes - (size_t)H.ndata * 8), H);
  } catch (const H2Error& e) {
    st = e.code;
    err = e.what();
  } catch (const std::bad_alloc&) {
    st = H2_ERROR_OUT_OF_MEMORY;
    err = "host allocation failed";
  } catch (const std::exception& e) {
    st = H2_ERROR_FORMAT;
    err = e.what();
  }
  if (msg && msgcap) {
    std::strncpy(msg, err.c_str(), msgcap - 1);
    msg[msgcap - 1] = 0;
  }
  return st;
}

h2_status h2_matrix_load(h2_context_t ctx, const void* blob, size_t bytes, h2_matrix_t* out) {
  if (!ctx || !blob || !out) return H2_ERROR_INVALID_ARGUMENT;
  *out = nullptr;
  auto* H = new (std::nothrow) h2_matrix_s();
  if (!H) return H2_ERROR_OUT_OF_MEMORY;
  H->ctx = ctx;
  H->tr.mem = &ctx->mem;
  h2_status st = guard(ctx, [&] {
    H2_HIP(hipSetDevice(ctx->device));
    const uint8_t* p = (const uint8_t*)blob;
    parse(p, bytes, *H);
    const double* d = (const double*)(p + bytes - (size_t)H->ndata * 8);
    check_data(d, *H);
    H->data.alloc(H->ndata, &H->tr);
    if (H->ndata)
      H2_HIP(hipMemcpyAsync(H->data.p, d, (size_t)H->ndata * 8, hipMemcpyHostToDevice, ctx->stream));
    H->perm_d.alloc(H->N, &H->tr);
    H2_HIP(hipMemcpyAsync(H->perm_d.p, H->perm.data(), (size_t)H->N * 8, hipMemcpyHostToDevice,
                          ctx->stream));
    auto up = [&](auto& dst, const auto& v) {
      dst.alloc((int64_t)v.size(), &H->tr);
      if (!v.empty())
        H2_HIP(hipMemcpyAsync(dst.p, v.data(), v.size() * sizeof(v[0]), hipMemcpyHostToDevice,
                              ctx->stream));
    };
    up(H->far_ptr_d, H->far_ptr);
    up(H->far_col_d, H->far_col);
    up(H->offS_d, H->offS);
    up(H->offE_d, H->offE);
    up(H->rank_d, H->rank);
    H2_HIP(hipStreamSynchronize(ctx->stream));
  });
  if (st != H2_SUCCESS) {
    delete H;
    return st;
  }
  *out = H;
  return H2_SUCCESS;
}

h2_status h2_matrix_destroy(h2_matrix_t H) {
  if (!H) return H2_ERROR_INVALID_ARGUMENT;
  (void)hipSetDevice(H->ctx->device);
  (void)hipStreamSynchronize(H->ctx->stream);
  delete H;
  return H2_SUCCESS;
}

h2_status h2_matrix_get_info(h2_matrix_t H, h2_matrix_info* info) {
  if (!H || !info) return H2_ERROR_INVALID_ARGUMENT;
  info->n = H->N;
  info->dim = H->dim;
  info->depth = H->L;
  info->top_level = H->top;
  info->n_nodes = H->nn;
  info->norm2 = H->norm2;
  info->device_bytes = H->tr.cur;
  return H2_SUCCESS;
}

h2_status h2_matvec(h2_context_t ctx, h2_matrix_t H, const double* X, int64_t ldx, int nrhs,
                    double* Y, int64_t ldy) {
  if (!ctx || !H || !X || !Y || nrhs < 0 || ldx < H->N || ldy < H->N)
    return H2_ERROR_INVALID_ARGUMENT;
  if ((const void*)X == (const void*)Y) return H2_ERROR_INVALID_ARGUMENT;
  if (nrhs == 0) return H2_SUCCESS;
  return guard(ctx, [&] {
    H2_HIP(hipSetDevice(ctx->device));
    h2drv::matvec(ctx, H, X, ldx, nrhs, Y, ldy);
  });
}

h2_status h2_matvec_noalloc(h2_context_t ctx, h2_matrix_t H, const double* X, int64_t ldx,
                            int nrhs, double* Y, int64_t ldy) {
  if (!ctx || !H || !X || !Y || nrhs < 0 || ldx < H->N || ldy < H->N)
    return H2_ERROR_INVALID_ARGUMENT;
  if ((const void*)X == (const void*)Y) return H2_ERROR_INVALID_ARGUMENT;
  if (nrhs == 0) return H2_SUCCESS;
  return guard(ctx, [&] {
    H2_HIP(hipSetDevice(ctx->device));
    h2drv::matvec_in(ctx, H, X, ldx, nrhs, Y, ldy, (char*)scratch_of(ctx->device),
                     kNoAllocScratchBytes);
  });
}

h2_status h2_factor(h2_context_t ctx, h2_matrix_t H, double tol, h2_prec prec,
                    const h2_factor_opts* opts, h2_factor_t* F) {
  return h2_factor_batched(ctx, 1, &H, tol, prec, opts, F);
}

h2_status h2_factor_batched(h2_context_t ctx, int count, const h2_matrix_t* Hs, double tol,
                            h2_prec prec, const h2_factor_opts* opts, h2_factor_t* Fs) {
  if (!ctx || count <= 0 || !Hs || !Fs) return H2_ERROR_INVALID_ARGUMENT;
  if (!(tol >= 0) || !std::isfinite(tol)) return H2_ERROR_INVALID_ARGUMENT;
  if (prec != H2_PREC_FP64 && prec != H2_PREC_FP32 && prec != H2_PREC_FP32_GRAM &&
      prec != H2_PREC_FP32_QR)
    return H2_ERROR_INVALID_ARGUMENT;
  h2_factor_opts o{};
  if (opts) o = *opts;
  if (std::isnan(o.norm2) || !std::isfinite(o.norm2) || o.norm2 < 0 || o.pool_bytes < 0 ||
      o.lds_limit_kib < 0)
    return H2_ERROR_INVALID_ARGUMENT;
  for (int i = 0; i < count; ++i) {
    if (!Hs[i] || Hs[i]->ctx != ctx) return H2_ERROR_INVALID_ARGUMENT;
    Fs[i] = nullptr;
  }
  std::vector<h2_factor_s*> out;
  h2_status st = guard(ctx, [&] {
    H2_HIP(hipSetDevice(ctx->device));
    std::vector<h2_matrix_s*> hs(Hs, Hs + count);
    out = h2drv::factor(ctx, hs, tol, prec, o);
  });
  if (st == H2_SUCCESS)
    for (int i = 0; i < count; ++i) Fs[i] = out[i];
  return st;
}

h2_status h2_factor_destroy(h2_factor_t F) {
  if (!F) return H2_ERROR_INVALID_ARGUMENT;
  (void)hipSetDevice(F->ctx->device);
  (void)hipStreamSynchronize(F->ctx->stream);
  delete F;
  return H2_SUCCESS;
}

h2_status h2_solve(h2_context_t ctx, h2_factor_t F, const double* B, int64_t ldb, int nrhs,
                   double* X, int64_t ldx) {
  return h2_solve_batched(ctx, 1, &F, &B, &ldb, nrhs, &X, &ldx);
}

h2_status h2_solve_batched(h2_context_t ctx, int count, const h2_factor_t* Fs,
                           const double* const* B, const int64_t* ldb, int nrhs,
                           double* const* X, const int64_t* ldx) {
  if (!ctx || count <= 0 || !Fs || !B || !X || !ldb || !ldx || nrhs < 0)
    return H2_ERROR_INVALID_ARGUMENT;
  for (int i = 0; i < count; ++i) {
    if (!Fs[i] || Fs[i]->ctx != ctx || !B[i] || !X[i] || ldb[i] < Fs[i]->N || ldx[i] < Fs[i]->N)
      return H2_ERROR_INVALID_ARGUMENT;
    if (Fs[i]->prec != Fs[0]->prec) return H2_ERROR_INVALID_ARGUMENT;
  }
  if (nrhs == 0) return H2_SUCCESS;
  return guard(ctx, [&] {
    H2_HIP(hipSetDevice(ctx->device));
    std::vector<h2_factor_s*> fs(Fs, Fs + count);
    std::vector<const double*> bs(B, B + count);
    std::vector<double*> xs(X, X + count);
    std::vector<int64_t> lb(ldb, ldb + count), lx(ldx, ldx + count);
    h2drv::solve(ctx, fs, bs, lb, nrhs, xs, lx);
  });
}

h2_status h2_solve_ir(h2_context_t ctx, h2_matrix_t H, h2_factor_t F, const double* B,
                      int64_t ldb, int nrhs, double* X, int64_t ldx, const h2_ir_opts* opts,
                      h2_ir_report* report) {
  if (!ctx || !H || !F || !B || !X || nrhs < 0 || ldb < H->N || ldx < H->N || F->N != H->N)
    return H2_ERROR_INVALID_ARGUMENT;
  if ((const void*)B == (const void*)X) return H2_ERROR_INVALID_ARGUMENT;
  h2_ir_opts o{1e-12, 30, 20, 1e-3};
  if (opts) o = *opts;
  if (o.restart < 1 || o.max_outer < 0 || !(o.target_bkwd > 0)) return H2_ERROR_INVALID_ARGUMENT;
  h2_ir_report rep{};
  bool conv = true;
  h2_status st = guard(ctx, [&] {
    H2_HIP(hipSetDevice(ctx->device));
    conv = h2drv::solve_ir(ctx, H, F, B, ldb, nrhs, X, ldx, o, rep);
  });
  if (report) *report = rep;
  if (st == H2_SUCCESS && !conv) {
    ctx->err = "refinement stopped at backward error " + std::to_string(rep.max_bkwd);
    return H2_ERROR_NOT_CONVERGED;
  }
  return st;
}

h2_status h2_factor_export_ints(h2_factor_t F, int level, h2_int_kind kind, int64_t* buf,
                                int64_t cap, int64_t* len) {
  if (!F || !len || cap < 0 || (cap > 0 && !buf)) return H2_ERROR_INVALID_ARGUMENT;
  std::vector<int64_t> v;
  if (kind == H2_INT_NTOP) {
    v.push_back(F->n_top);
  } else if (kind == H2_INT_LEVELS) {
    for (auto& p : F->plans) v.push_back(p.lev);
  } else {
    const LevelPlan* P = nullptr;
    for (auto& p : F->plans)
      if (p.lev == level) P = &p;
    if (!P) return H2_ERROR_INVALID_ARGUMENT;
    if (kind == H2_INT_SIZES) {
      for (int x : P->n) v.push_back(x);
    } else if (kind == H2_INT_RANKS) {
      for (int i = 0; i < P->nl; ++i) v.push_back(P->n[i] - P->r[i]);
    } else if (kind == H2_INT_COLORS) {
      for (int x : P->color) v.push_back(x);
    } else if (kind == H2_INT_FILL) {
      for (auto& pr : P->fill_pairs) {
        v.push_back(pr.first + P->a);
        v.push_back(pr.second + P->a);
      }
    } else if (kind == H2_INT_OFFSETS) {
      for (int j = 0; j < P->nl; ++j)
        for (int64_t e = P->pptr[j]; e < P->pptr[j + 1]; ++e) {
          v.push_back(j + P->a);
          v.push_back(P->pcol[e] + P->a);
          v.push_back(P->isF[e] ? (P->tr(j, e) ? 2 : 1) : 0);
          v.push_back(P->poff[e]);
        }
    } else if (kind == H2_INT_CLUSTER_OFFSETS) {
      for (int64_t x : P->offQ) v.push_back(x);
    } else if (kind == H2_INT_OWNERS) {
      if (!F->keep_owners) return H2_ERROR_INVALID_ARGUMENT;
      v = P->owners;
    } else {
      return H2_ERROR_INVALID_ARGUMENT;
    }
  }
  *len = (int64_t)v.size();
  for (int64_t i = 0; i < std::min<int64_t>(cap, (int64_t)v.size()); ++i) buf[i] = v[i];
  return H2_SUCCESS;
}

h2_status h2_factor_export_matrix(h2_factor_t F, int level, h2_mat_kind kind, int i, int j,
                                  double* buf, int64_t cap, int64_t* rows, int64_t* cols) {
  if (!F || !rows || !cols || cap < 0 || (cap > 0 && !buf)) return H2_ERROR_INVALID_ARGUMENT;
  return guard(F->ctx, [&] {
    H2_HIP(hipSetDevice(F->ctx->device));
    const void* src = nullptr;
    int64_t m = 0, n = 0;
    if (kind == H2_MAT_TOP) {
      m = n = F->n_top;
      src = F->prec == H2_PREC_FP64 ? (const void*)F->M64.p : (const void*)F->M32.p;
    } else {
      size_t li = F->plans.size();
      for (size_t q = 0; q < F->plans.size(); ++q)
        if (F->plans[q].lev == level) li = q;
      if (li == F->plans.size()) throw H2Error(H2_ERROR_INVALID_ARGUMENT, "no such level");
      const LevelPlan& P = F->plans[li];
      if (i < 0 || i >= P.nl) throw H2Error(H2_ERROR_INVALID_ARGUMENT, "bad cluster index");
      int64_t off = 0;
      if (kind == H2_MAT_Q) {
        m = n = P.n[i];
        off = P.offQ[i];
        src = F->prec == H2_PREC_FP64 ? (const void*)(F->st64[li].Q.p + off)
                                      : (const void*)(F->st32[li].Q.p + off);
      } else if (kind == H2_MAT_BLOCK) {
        if (j < 0 || j >= P.nl) throw H2Error(H2_ERROR_INVALID_ARGUMENT, "bad cluster index");
        const int64_t e = P.find(i, j);
        if (e < 0 || P.isF[e]) throw H2Error(H2_ERROR_INVALID_ARGUMENT, "not a near pair");
        m = P.n[i];
        n = P.n[j];
        src = F->prec == H2_PREC_FP64 ? (const void*)(F->st64[li].D.p + P.poff[e])
                                      : (const void*)(F->st32[li].D.p + P.poff[e]);
      } else {
        throw H2Error(H2_ERROR_INVALID_ARGUMENT, "bad kind");
      }
    }
    *rows = m;
    *cols = n;
    if (m * n > cap || m * n == 0) return;
    H2_HIP(hipStreamSynchronize(F->ctx->stream));
    if (F->prec == H2_PREC_FP64) {
      H2_HIP(hipMemcpy(buf, src, sizeof(double) * m * n, hipMemcpyDeviceToHost));
    } else {
      std::vector<float> tmp((size_t)(m * n));
      H2_HIP(hipMemcpy(tmp.data(), src, sizeof(float) * m * n, hipMemcpyDeviceToHost));
      for (int64_t e = 0; e < m * n; ++e) buf[e] = tmp[(size_t)e];
    }
  });
}

h2_status h2_factor_get_stats(h2_factor_t F, h2_stats* s) {
  if (!F || !s) return H2_ERROR_INVALID_ARGUMENT;
  *s = F->stats;
  s->solves = F->splan ? F->splan->uses() : 0;
  s->solve_graph_launches = F->splan ? F->splan->graph_uses() : 0;
  return H2_SUCCESS;
}

}  // extern "C"
