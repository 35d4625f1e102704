// HIP kernels of the H^2 strong recursive skeletonization solver (gfx950).
//
// Dense contractions (projections by Q~, Schur complement / fill-in updates,
// near-field and coupling products of the H^2 matvec, the trailing update of
// the dense top LU) run on the FP64 / FP32 16x16x4 MFMA instructions.  The
// small per-cluster factorizations (Householder QR of the fill row, one-sided
// Jacobi SVD, complement, partial-pivoting LU) run one workgroup per cluster.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>
#include <cstdint>

#include "h2_kernels.h"

namespace h2k {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

template <class T> struct Acc;
template <> struct Acc<double> { typedef d4 type; };
template <> struct Acc<float> { typedef f4 type; };

__device__ inline d4 mfma16(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ inline f4 mfma16(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Row of accumulator element i held by a lane with kq = lane / 16 (column lane % 16).
// Measured on gfx950: the FP64 16x16x4 instruction interleaves rows
// (kq + 4 i), the FP32 one keeps them contiguous (4 kq + i).
template <class T> __device__ inline int acc_row(int kq, int i);
template <> __device__ inline int acc_row<double>(int kq, int i) { return kq + 4 * i; }
template <> __device__ inline int acc_row<float>(int kq, int i) { return 4 * kq + i; }

// Global-memory view of a pointer taken from a task descriptor (device
// allocations only): accesses through it are global, not flat, so they do
// not count against the LDS wait counter.
template <class T> using gptr = __attribute__((address_space(1))) T*;
template <class T> __device__ inline gptr<T> gmem(T* p) { return (gptr<T>)p; }

// Where the copy of the multipliers of a near block (r x nk) sits inside the
// block's n x nk region of the copy array, and its leading dimension: from
// the first 16-byte boundary with a leading dimension rounded up to 16 bytes
// when that fits the region, else from the region's start with leading
// dimension r.  The triangular solve that writes the copy and the Schur
// update that reads it both place it here.
template <class T, class P> __device__ inline P xmul_at(P base, int r, int n, int nk, int& ld) {
  constexpr int ve = 16 / (int)sizeof(T);
  const int mis = (int)(((uintptr_t)base / sizeof(T)) % ve);
  const int shift = mis ? ve - mis : 0;
  const int ldv = (r + ve - 1) / ve * ve;
  if (shift + (int64_t)ldv * nk <= (int64_t)n * nk) {
    ld = ldv;
    return base + shift;
  }
  ld = r;
  return base;
}

// 16-byte vector of T (one LDS b128 access)
template <class T> struct Vec16;
template <> struct Vec16<float> { typedef float __attribute__((ext_vector_type(4))) type; };
template <> struct Vec16<double> { typedef double __attribute__((ext_vector_type(2))) type; };

template <class T> __device__ inline T eps_of();
template <> __device__ inline double eps_of<double>() { return DBL_EPSILON; }
template <> __device__ inline float eps_of<float>() { return FLT_EPSILON; }

__device__ inline double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ inline float wave_sum(float v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// block-wide sum (same order in every thread); `red` holds >= blockDim.x / 64
// values
template <class T> __device__ inline T block_sum(T v, T* red) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63, nw = blockDim.x >> 6;
  __syncthreads();
  if (l == 0) red[w] = v;
  __syncthreads();
  T s = 0;
  for (int i = 0; i < nw; ++i) s += red[i];
  __syncthreads();
  return s;
}

// ---------------------------------------------------------------------------
// Grouped GEMM with owner-computes accumulation over contributor lists.
// Workgroup = 4 waves arranged WM x WN; each wave owns FM x FN fragments of
// 16 x 16.  Operands are read straight from global memory (L1/L2 cached) in
// the MFMA lane layout: lane l supplies A[row l%16][k l/16] and
// B[k l/16][col l%16].  They enter the MFMA as (B^T, A^T), so it forms the
// transposed block and accumulator element i is C[l%16][acc_row(l/16, i)]:
// the epilogue's loads and stores of the column-major C are coalesced.
// ---------------------------------------------------------------------------
template <class T, int WM, int WN, int FM, int FN>
__global__ __launch_bounds__(256) void k_gemm(const GOut<T>* __restrict__ outs, int nouts,
                                              const GCon<T>* __restrict__ cons,
                                              const int32_t* __restrict__ dyn) {
  constexpr int TM = WM * FM * 16, TN = WN * FN * 16;
  const int64_t tile = blockIdx.x;
  int lo = 0, hi = nouts - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (outs[mid].tile0 <= tile) lo = mid; else hi = mid - 1;
  }
  const GOut<T>& o = outs[lo];
  const int64_t t = tile - o.tile0;
  const int ti = (int)(t % o.tm), tj = (int)(t / o.tm);
  const int m0 = o.m0d >= 0 ? dyn[o.m0d] : o.m0s;
  const int m1 = o.m1d >= 0 ? dyn[o.m1d] : o.m;
  const int n0 = o.n0d >= 0 ? dyn[o.n0d] : o.n0s;
  const int n1 = o.n;
  const int r0 = m0 + ti * TM, c0 = n0 + tj * TN;
  if (r0 >= m1 || c0 >= n1) return;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int wr = r0 + (wave % WM) * FM * 16;
  const int wc = c0 + (wave / WM) * FN * 16;
  typename Acc<T>::type acc[FM][FN];
#pragma unroll
  for (int a = 0; a < FM; ++a)
#pragma unroll
    for (int b = 0; b < FN; ++b) acc[a][b] = (typename Acc<T>::type){0, 0, 0, 0};
  const int l16 = lane & 15, kq = lane >> 4;
  for (int ci = o.cbeg; ci < o.cend; ++ci) {
    const GCon<T> g = cons[ci];
    const int k0 = g.k0d >= 0 ? dyn[g.k0d] : g.k0s;
    const int k1 = g.k1d >= 0 ? dyn[g.k1d] : g.k;
    for (int kk = k0; kk < k1; kk += 4) {
      const int kx = kk + kq;
      const bool kok = kx < k1;
      T av[FM], bv[FN];
#pragma unroll
      for (int a = 0; a < FM; ++a) {
        const int row = wr + a * 16 + l16;
        T v = 0;
        if (kok && row < m1)
          v = g.transA ? g.A[kx + (int64_t)row * g.lda] : g.A[row + (int64_t)kx * g.lda];
        av[a] = v;
      }
#pragma unroll
      for (int b = 0; b < FN; ++b) {
        const int col = wc + b * 16 + l16;
        T v = 0;
        if (kok && col < n1) v = g.B[kx + (int64_t)col * g.ldb];
        bv[b] = v;
      }
      // operands swapped: the accumulator holds the transposed 16 x 16 block,
      // lane l16 owning row l16, so the column-major C is written by
      // consecutive lanes along its contiguous dimension
#pragma unroll
      for (int a = 0; a < FM; ++a)
#pragma unroll
        for (int b = 0; b < FN; ++b) acc[a][b] = mfma16(bv[b], av[a], acc[a][b]);
    }
  }
  const T alpha = o.alpha, beta = o.beta;
#pragma unroll
  for (int a = 0; a < FM; ++a) {
    const int row = wr + a * 16 + l16;
    if (row >= m1) continue;
#pragma unroll
    for (int b = 0; b < FN; ++b)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int col = wc + b * 16 + acc_row<T>(kq, i);
        if (col < n1) {
          T* p = o.C + row + (int64_t)col * o.ldc;
          const T v = alpha * acc[a][b][i];
          *p = beta == T(0) ? v : beta * *p + v;
        }
      }
  }
}

// 16-byte vector of T read from 4- (8-) byte aligned global memory
template <class T> struct VecK;
template <> struct VecK<float> {
  typedef float __attribute__((ext_vector_type(4), aligned(4))) type;
  static constexpr int n = 4;
};
template <> struct VecK<double> {
  typedef double __attribute__((ext_vector_type(2), aligned(8))) type;
  static constexpr int n = 2;
};
template <class T> __device__ inline typename VecK<T>::type ld_veck(gptr<const T> p) {
  return *reinterpret_cast<const __attribute__((address_space(1))) typename VecK<T>::type*>(p);
}

// Skinny variant for outputs of few columns (the solves' right-hand sides):
// a 64 x TN tile (TN = 16 FN) is computed by all four waves, each taking
// every fourth k-step with four row fragments and FN column fragments in
// flight, so every operand element is read once per tile; the waves' partial
// tiles are summed through LDS.  An output with nsplit > 1 has its
// contributor list cut into nsplit chunks, one workgroup each; their partial
// tiles (column-major 64 x TN) go to `parts` and k_gemm_reduce adds them in
// chunk order.
template <class T, int FN, int VK>
__global__ __launch_bounds__(256) void k_gemm_skinny(const GOut<T>* __restrict__ outs, int nouts,
                                                     const GCon<T>* __restrict__ cons,
                                                     const int32_t* __restrict__ dyn,
                                                     T* __restrict__ parts) {
  constexpr int TM = 64, TN = 16 * FN;
  __shared__ T part[2][TM * TN];
  const int64_t tile = blockIdx.x;
  int lo = 0, hi = nouts - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (outs[mid].tile0 <= tile) lo = mid; else hi = mid - 1;
  }
  const GOut<T>& o = outs[lo];
  const int ns = o.nsplit > 1 ? o.nsplit : 1;
  const int64_t trel = tile - o.tile0;
  const int sidx = (int)(trel % ns);
  const int64_t tt = trel / ns;
  const int ti = (int)(tt % o.tm), tj = (int)(tt / o.tm);
  const int m0 = o.m0d >= 0 ? dyn[o.m0d] : o.m0s;
  const int m1 = o.m1d >= 0 ? dyn[o.m1d] : o.m;
  const int n0 = o.n0d >= 0 ? dyn[o.n0d] : o.n0s;
  const int n1 = o.n;
  const int r0 = m0 + ti * TM, c0 = n0 + tj * TN;
  if (ns == 1 && (r0 >= m1 || c0 >= n1)) return;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int l16 = lane & 15, kq = lane >> 4;
  typename Acc<T>::type acc[4][FN];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < FN; ++b) acc[a][b] = (typename Acc<T>::type){0, 0, 0, 0};
  const int ncon = o.cend - o.cbeg;
  const int cps = (ncon + ns - 1) / ns;
  const int cb = o.cbeg + sidx * cps;
  const int ce = min(o.cend, cb + cps);
  // wave w takes blocks w, w + 4, ... of KBLK = 4 VK k-values, NB blocks in
  // flight (64 k per round of the workgroup); in a block, lane group kq
  // holds k = kb + VK kq + s for MFMA step s, so that with VK > 1 operands
  // with k contiguous (B, and A when transposed) are read as one 16-byte
  // vector.  VK = 1 keeps the plain ascending k order of every wave.
  constexpr int KBLK = 4 * VK;
  constexpr int NB = 64 / (4 * KBLK);
  for (int ci = cb; ci < ce; ++ci) {
    const GCon<T> g = cons[ci];
    const int k0 = g.k0d >= 0 ? dyn[g.k0d] : g.k0s;
    const int k1 = g.k1d >= 0 ? dyn[g.k1d] : g.k;
    const gptr<const T> A = gmem(g.A), B = gmem(g.B);
    for (int kb = k0 + wave * KBLK; kb < k1; kb += 4 * KBLK * NB) {
      T av[NB][VK][4], bv[NB][VK][FN];
#pragma unroll
      for (int q = 0; q < NB; ++q) {
        const int kl = kb + q * 4 * KBLK + VK * kq;  // this lane's first k of the block
#pragma unroll
        for (int b = 0; b < FN; ++b) {
          const int col = c0 + b * 16 + l16;
          if (VK > 1 && col < n1 && kl + VK <= k1) {
            const typename VecK<T>::type v = ld_veck<T>(B + kl + (int64_t)col * g.ldb);
#pragma unroll
            for (int s2 = 0; s2 < VK; ++s2) bv[q][s2][b] = v[s2 % VecK<T>::n];
          } else {
#pragma unroll
            for (int s2 = 0; s2 < VK; ++s2)
              bv[q][s2][b] = (col < n1 && kl + s2 < k1) ? B[kl + s2 + (int64_t)col * g.ldb] : T(0);
          }
        }
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          const int row = r0 + a * 16 + l16;
          if (VK > 1 && g.transA && row < m1 && kl + VK <= k1) {
            const typename VecK<T>::type v = ld_veck<T>(A + kl + (int64_t)row * g.lda);
#pragma unroll
            for (int s2 = 0; s2 < VK; ++s2) av[q][s2][a] = v[s2 % VecK<T>::n];
          } else {
#pragma unroll
            for (int s2 = 0; s2 < VK; ++s2) {
              const int kx = kl + s2;
              av[q][s2][a] = (kx < k1 && row < m1)
                                 ? (g.transA ? A[kx + (int64_t)row * g.lda] : A[row + (int64_t)kx * g.lda])
                                 : T(0);
            }
          }
        }
      }
#pragma unroll
      for (int q = 0; q < NB; ++q)
#pragma unroll
        for (int s2 = 0; s2 < VK; ++s2) {
          if (kb + q * 4 * KBLK + s2 >= k1) continue;
#pragma unroll
          for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < FN; ++b) acc[a][b] = mfma16(av[q][s2][a], bv[q][s2][b], acc[a][b]);
        }
    }
  }
  // sum the four waves' tiles: waves 2 and 3 hand theirs to waves 0 and 1,
  // wave 1 to wave 0, which leaves the total in part[1] (column-major)
  auto put = [&](T* dst) {
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < FN; ++b)
#pragma unroll
        for (int i = 0; i < 4; ++i)
          dst[(a * 16 + acc_row<T>(kq, i)) + (b * 16 + l16) * TM] = acc[a][b][i];
  };
  auto take = [&](const T* src) {
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < FN; ++b)
#pragma unroll
        for (int i = 0; i < 4; ++i)
          acc[a][b][i] += src[(a * 16 + acc_row<T>(kq, i)) + (b * 16 + l16) * TM];
  };
  if (wave >= 2) put(part[wave - 2]);
  __syncthreads();
  if (wave < 2) take(part[wave]);
  __syncthreads();
  if (wave == 1) put(part[0]);
  __syncthreads();
  if (wave == 0) {
    take(part[0]);
    put(part[1]);
  }
  __syncthreads();
  const T* sum = part[1];
  if (ns > 1) {
    T* dst = parts + (o.part0 + tt * ns + sidx) * (int64_t)(TM * TN);
    for (int e = threadIdx.x; e < TM * TN; e += blockDim.x) dst[e] = sum[e];
    return;
  }
  const T alpha = o.alpha, beta = o.beta;
  for (int e = threadIdx.x; e < TM * TN; e += blockDim.x) {
    const int rr = e % TM, cc = e / TM;
    const int row = r0 + rr, cl = c0 + cc;
    if (row < m1 && cl < n1) {
      const T v = alpha * sum[e];
      T* p = o.C + row + (int64_t)cl * o.ldc;
      *p = beta == T(0) ? v : beta * *p + v;
    }
  }
}

template <class T, int TN>
__global__ __launch_bounds__(256) void k_gemm_reduce(const GOut<T>* __restrict__ outs, int nouts,
                                                     const T* __restrict__ parts) {
  constexpr int TM = 64;
  const int64_t tile = blockIdx.x;
  int lo = 0, hi = nouts - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (outs[mid].rtile0 <= tile) lo = mid; else hi = mid - 1;
  }
  const GOut<T>& o = outs[lo];
  const int ns = o.nsplit;
  const int64_t tt = tile - o.rtile0;
  const int ti = (int)(tt % o.tm), tj = (int)(tt / o.tm);
  const int r0 = o.m0s + ti * TM, c0 = o.n0s + tj * TN;
  const T* src = parts + (o.part0 + tt * ns) * (int64_t)(TM * TN);
  const T alpha = o.alpha, beta = o.beta;
  for (int e = threadIdx.x; e < TM * TN; e += blockDim.x) {
    const int row = r0 + e % TM, cl = c0 + e / TM;
    if (row < o.m && cl < o.n) {
      T sum = 0;
      for (int q = 0; q < ns; ++q) sum += src[(int64_t)q * (TM * TN) + e];
      T* p = o.C + row + (int64_t)cl * o.ldc;
      const T v = alpha * sum;
      *p = beta == T(0) ? v : beta * *p + v;
    }
  }
}

// One workgroup per output (no tile search), looping over the output's 64 x
// 64 tiles: each wave owns a 32 x 32 quarter.  The tile's C entries are
// fetched before the products and the operands of up to kGemmKB k-steps are
// loaded together, so a tile costs few memory round trips; many workgroups
// per CU hide them.  For outputs of a few tiles (Schur updates of blocks).
constexpr int kGemmKB = 2;
template <class T>
__global__ __launch_bounds__(256) void k_gemm_out(const GOut<T>* __restrict__ outs,
                                                  const GCon<T>* __restrict__ cons,
                                                  const int32_t* __restrict__ dyn) {
  constexpr int FM = 2, FN = 2;
  const GOut<T>& o = outs[blockIdx.x];
  const int m0 = o.m0d >= 0 ? dyn[o.m0d] : o.m0s;
  const int m1 = o.m1d >= 0 ? dyn[o.m1d] : o.m;
  const int n0 = o.n0d >= 0 ? dyn[o.n0d] : o.n0s;
  const int n1 = o.n;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int l16 = lane & 15, kq = lane >> 4;
  const T alpha = o.alpha, beta = o.beta;
  const gptr<T> C = gmem(o.C);
  const int ntile = o.tm * o.tn;
  for (int t = 0; t < ntile; ++t) {
    const int ti = t % o.tm, tj = t / o.tm;
    const int r0 = m0 + ti * 64, c0 = n0 + tj * 64;
    if (r0 >= m1 || c0 >= n1) continue;
    const int wr = r0 + (wave & 1) * 32, wc = c0 + (wave >> 1) * 32;
    // C entries this lane combines in the epilogue
    T cv[FM][FN][4];
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
      for (int b = 0; b < FN; ++b)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int row = wr + a * 16 + l16, col = wc + b * 16 + acc_row<T>(kq, i);
          cv[a][b][i] = (beta != T(0) && row < m1 && col < n1)
                            ? C[row + (int64_t)col * o.ldc] : T(0);
        }
    typename Acc<T>::type acc[FM][FN];
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
      for (int b = 0; b < FN; ++b) acc[a][b] = (typename Acc<T>::type){0, 0, 0, 0};
    for (int ci = o.cbeg; ci < o.cend; ++ci) {
      const GCon<T> g = cons[ci];
      const int k0 = g.k0d >= 0 ? dyn[g.k0d] : g.k0s;
      const int k1 = g.k1d >= 0 ? dyn[g.k1d] : g.k;
      const gptr<const T> A = gmem(g.A), B = gmem(g.B);
      for (int kb = k0; kb < k1; kb += 4 * kGemmKB) {
        T av[kGemmKB][FM], bv[kGemmKB][FN];
#pragma unroll
        for (int q = 0; q < kGemmKB; ++q) {
          const int kx = kb + 4 * q + kq;
          const bool kok = kx < k1;
#pragma unroll
          for (int a = 0; a < FM; ++a) {
            const int row = wr + a * 16 + l16;
            av[q][a] = (kok && row < m1)
                           ? (g.transA ? A[kx + (int64_t)row * g.lda] : A[row + (int64_t)kx * g.lda])
                           : T(0);
          }
#pragma unroll
          for (int b = 0; b < FN; ++b) {
            const int col = wc + b * 16 + l16;
            bv[q][b] = (kok && col < n1) ? B[kx + (int64_t)col * g.ldb] : T(0);
          }
        }
        // operands swapped: the accumulator holds the transposed block, lane
        // l16 owning row l16 (coalesced epilogue)
#pragma unroll
        for (int q = 0; q < kGemmKB; ++q) {
          if (kb + 4 * q >= k1) break;
#pragma unroll
          for (int a = 0; a < FM; ++a)
#pragma unroll
            for (int b = 0; b < FN; ++b) acc[a][b] = mfma16(bv[q][b], av[q][a], acc[a][b]);
        }
      }
    }
#pragma unroll
    for (int a = 0; a < FM; ++a) {
      const int row = wr + a * 16 + l16;
      if (row >= m1) continue;
#pragma unroll
      for (int b = 0; b < FN; ++b)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int col = wc + b * 16 + acc_row<T>(kq, i);
          if (col < n1) C[row + (int64_t)col * o.ldc] = beta * cv[a][b][i] + alpha * acc[a][b][i];
        }
    }
  }
}

// ---------------------------------------------------------------------------
// Schur and fill-in updates enumerated on the device (launch_schur).
// ---------------------------------------------------------------------------
template <class T> __global__ void k_fill(T* p, int64_t n, T v);

// instance of global row g (rows0 ascending)
template <class T> __device__ inline int schur_inst(const SchurLevel<T>* lvs, int ninst, int64_t g) {
  int lo = 0, hi = ninst - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (lvs[mid].rows0 <= g) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// entry (i, k) of row i of the pattern when it is a near entry, else -1
template <class T> __device__ inline int64_t schur_near_entry(const SchurLevel<T>& L, int i, int k) {
  int64_t a = L.pptr[i], b = L.pptr[i + 1];
  const int64_t end = b;
  while (a < b) {
    const int64_t m = (a + b) >> 1;
    if (L.pcol[m] < k) a = m + 1; else b = m;
  }
  return (a < end && L.pcol[a] == k && L.kind[a] == 0) ? a : -1;
}

// workgroup = row g: its contributors (near entries of colour c, in column
// order) to rowtab[g], then its targets, in entry order, appended to the list
template <class T>
__global__ __launch_bounds__(256) void k_schur_enum(const SchurLevel<T>* __restrict__ lvs,
                                                    int ninst, int c, SchurRow* rowtab,
                                                    SchurTarget* targets, int64_t* conts,
                                                    int64_t* count, int64_t ccap, int* err) {
  __shared__ int ci[kSchurMaxContrib];
  __shared__ int64_t eji[kSchurMaxContrib];
  __shared__ int wcnt[4], wcon[4];
  __shared__ int sh_nc;
  __shared__ int64_t sh_base, sh_cbase;
  const int64_t g = blockIdx.x;
  const SchurLevel<T>& L = lvs[schur_inst(lvs, ninst, g)];
  const int j = (int)(g - L.rows0);
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int64_t e0 = L.pptr[j], e1 = L.pptr[j + 1];
  if (tid == 0) sh_nc = 0;
  __syncthreads();
  // contributors, compacted in entry order
  for (int64_t base = e0; base < e1; base += 256) {
    const int64_t e = base + tid;
    const bool f = e < e1 && L.kind[e] == 0 && L.color[L.pcol[e]] == c;
    const unsigned long long bal = __ballot(f);
    if (lane == 0) wcnt[wave] = __popcll(bal);
    __syncthreads();
    int off = sh_nc;
    for (int w = 0; w < wave; ++w) off += wcnt[w];
    off += __popcll(bal & ((1ull << lane) - 1ull));
    if (f) {
      if (off < kSchurMaxContrib) {
        ci[off] = L.pcol[e];
        eji[off] = e;
      } else {
        atomicOr(err, 4);
      }
    }
    __syncthreads();
    if (tid == 0) sh_nc = min(kSchurMaxContrib, sh_nc + wcnt[0] + wcnt[1] + wcnt[2] + wcnt[3]);
    __syncthreads();
  }
  const int nc = sh_nc;
  if (tid == 0) rowtab[g].nc = nc;
  if (tid < nc) {
    rowtab[g].ci[tid] = ci[tid];
    rowtab[g].eji[tid] = eji[tid];
  }
  if (nc == 0) return;
  // targets: entries whose column some contributor is near (fill entries only
  // when stored)
  for (int64_t base = e0; base < e1; base += 256) {
    const int64_t e = base + tid;
    uint32_t mask = 0;
    if (e < e1 && L.kind[e] != 2) {
      const int k = L.pcol[e];
      for (int x = 0; x < nc; ++x)
        if (schur_near_entry(L, ci[x], k) >= 0) mask |= 1u << x;
    }
    const int nb = __popc(mask);
    // exclusive prefix of the contributor counts within the wave
    int incl = nb;
    for (int o = 1; o < 64; o <<= 1) {
      const int v = __shfl_up(incl, o, 64);
      if (lane >= o) incl += v;
    }
    const unsigned long long bal = __ballot(mask != 0);
    if (lane == 63) wcon[wave] = incl;
    if (lane == 0) wcnt[wave] = __popcll(bal);
    __syncthreads();
    if (tid == 0) {
      sh_base = (int64_t)atomicAdd((unsigned long long*)count,
                                   (unsigned long long)(wcnt[0] + wcnt[1] + wcnt[2] + wcnt[3]));
      sh_cbase = (int64_t)atomicAdd((unsigned long long*)(count + 1),
                                    (unsigned long long)(wcon[0] + wcon[1] + wcon[2] + wcon[3]));
    }
    __syncthreads();
    int off = 0, coff = 0;
    for (int w = 0; w < wave; ++w) {
      off += wcnt[w];
      coff += wcon[w];
    }
    off += __popcll(bal & ((1ull << lane) - 1ull));
    coff += incl - nb;
    if (mask) {
      const int k = L.pcol[e];
      SchurTarget t;
      t.e = e;
      t.g = (int32_t)g;
      t.cbeg = sh_cbase + coff;
      const bool fits = t.cbeg + nb <= ccap;
      t.ncont = fits ? nb : 0;
      if (!fits) atomicOr(err, 4);
      targets[sh_base + off] = t;
      int q = 0;
      if (fits)
        for (int x = 0; x < nc; ++x)
          if ((mask >> x) & 1u)
            conts[t.cbeg + q++] = ((int64_t)x << 48) | schur_near_entry(L, ci[x], k);
    }
    __syncthreads();
  }
}

// workgroups loop over the targets: C -= sum of the contributors' products,
// contributors ascending.  The active window of C is cut into
// items of 32 x 32 (2 x 2 fragments of 16 x 16), handed to the four waves in
// turn (from a different wave for each target of a group of four); C of an
// item is read before its products.  A multiplier block
// D(i, k) is column-major with k contiguous, so every lane reads VK
// consecutive k of its column as one 16-byte vector: MFMA step s of a block
// of 4 VK k-values takes k = kb + VK kq + s in lane group kq, for the panel
// D(j, i) as for the multipliers (any assignment of k to the steps gives the
// same sum).
// k-values a lane reads as one vector in the Schur update (FP64 keeps single
// loads: its k order is then the plain ascending one), and the blocks of 4 VK
// k-values of one operand load; a wave issues the loads of its next block
// (next k-values, else the next contribution's first) before the products of
// the current one
template <class T> constexpr int schur_vk() { return sizeof(T) == 4 ? 4 : 1; }
template <class T> constexpr int schur_nb() { return sizeof(T) == 4 ? 1 : 2; }
template <class T>
__global__ __launch_bounds__(256) void k_schur_apply(const SchurLevel<T>* __restrict__ lvs,
                                                     int ninst, int c,
                                                     const SchurRow* __restrict__ rowtab,
                                                     const SchurTarget* __restrict__ targets,
                                                     const int64_t* __restrict__ conts,
                                                     const int64_t* __restrict__ count) {
  constexpr int VK = schur_vk<T>();
  constexpr int KBLK = 4 * VK;
  constexpr int kSchurNB = schur_nb<T>();
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int l16 = lane & 15, kq = lane >> 4;
  const int64_t ntarg = *count;
  // groups of four consecutive targets per workgroup; the items of the q-th
  // target of a group start at wave q, so a run of one-item targets keeps
  // all four waves busy
  for (int64_t g0 = (int64_t)blockIdx.x * 4; g0 < ntarg; g0 += (int64_t)gridDim.x * 4)
  for (int64_t t0 = g0; t0 < min(ntarg, g0 + 4); ++t0) {
    const SchurTarget tg = targets[t0];
    const SchurLevel<T>& L = lvs[schur_inst(lvs, ninst, tg.g)];
    const SchurRow& R = rowtab[tg.g];
    const int j = (int)(tg.g - L.rows0);
    const int k = L.pcol[tg.e];
    const int nj = L.n[j], nk = L.n[k];
    const int m0 = L.color[j] <= c ? L.r[j] : 0;
    const int n0 = L.color[k] <= c ? L.r[k] : 0;
    const gptr<const T> Dg = gmem((const T*)L.D);
    const gptr<const T> Xg = gmem(kXmulCopy<T>() ? L.X : L.D);
    const gptr<T> C = gmem((L.kind[tg.e] == 1 ? L.F : L.D) + L.poff[tg.e]);
    const int nrg = (nj - m0 + 31) / 32;  // row items of the window
    const int ncg = (nk - n0 + 31) / 32;  // column items of the window
    for (int it = (wave - (int)(t0 - g0) + 4) & 3; it < nrg * ncg; it += 4) {
      const int rb = m0 + (it % nrg) * 32;
      const int cb = n0 + (it / nrg) * 32;
      T cv[2][2][4];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int row = rb + a * 16 + l16, col = cb + b * 16 + acc_row<T>(kq, i);
            cv[a][b][i] = (row < nj && col < nk) ? C[row + col * nj] : T(0);
          }
      typename Acc<T>::type acc[2][2];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = (typename Acc<T>::type){0, 0, 0, 0};
      // the item's operand blocks, contributions ascending and k ascending,
      // with the next block's loads issued before the current block's products
      // (the products, and so the rounding, are those of the plain loop)
      struct Blk {
        gptr<const T> A, B;  // D(j, i) (n_j x n_i) and the multipliers of (i, k) (r_i x n_k)
        int k1, kb, ldx;
      };
      auto setup = [&](int q, Blk& bk) {
        const int64_t cv2 = conts[tg.cbeg + q];
        const int x = (int)(cv2 >> 48);
        const int i = R.ci[x];
        bk.k1 = L.r[i];
        bk.A = Dg + L.poff[R.eji[x]];
        if (kXmulCopy<T>()) {
          bk.B = xmul_at<T>(Xg + L.xoff[cv2 & kContEntryMask], bk.k1, L.n[i], nk, bk.ldx);
        } else {
          bk.B = Dg + L.poff[cv2 & kContEntryMask];
          bk.ldx = L.n[i];
        }
        bk.kb = 0;
      };
      auto load = [&](const Blk& bk, T (&av)[kSchurNB][VK][2], T (&bv)[kSchurNB][VK][2]) {
#pragma unroll
        for (int q = 0; q < kSchurNB; ++q) {
          const int kl = bk.kb + q * KBLK + VK * kq;  // this lane's first k of the block
#pragma unroll
          for (int b = 0; b < 2; ++b) {
            const int col = cb + b * 16 + l16;
            if (VK > 1 && col < nk && kl + VK <= bk.k1) {
              const typename VecK<T>::type v = ld_veck<T>(bk.B + (kl + col * bk.ldx));
#pragma unroll
              for (int s2 = 0; s2 < VK; ++s2) bv[q][s2][b] = v[s2 % VecK<T>::n];
            } else {
#pragma unroll
              for (int s2 = 0; s2 < VK; ++s2)
                bv[q][s2][b] = (col < nk && kl + s2 < bk.k1) ? bk.B[kl + s2 + col * bk.ldx] : T(0);
            }
          }
#pragma unroll
          for (int a = 0; a < 2; ++a) {
            const int row = rb + a * 16 + l16;
#pragma unroll
            for (int s2 = 0; s2 < VK; ++s2)
              av[q][s2][a] = (row < nj && kl + s2 < bk.k1) ? bk.A[row + (kl + s2) * nj] : T(0);
          }
        }
      };
      // operands swapped: the accumulator holds the transposed fragment, lane
      // l16 owning row l16 (coalesced epilogue)
      auto prod = [&](const Blk& bk, const T (&av)[kSchurNB][VK][2], const T (&bv)[kSchurNB][VK][2]) {
#pragma unroll
        for (int q = 0; q < kSchurNB; ++q)
#pragma unroll
          for (int s2 = 0; s2 < VK; ++s2) {
            if (bk.kb + q * KBLK + s2 >= bk.k1) continue;
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
              for (int b = 0; b < 2; ++b) acc[a][b] = mfma16(bv[q][s2][b], av[q][s2][a], acc[a][b]);
          }
      };
      // next block after bk (false at the end); q is bk's contribution
      auto advance = [&](int& q, Blk& bk) {
        bk.kb += kSchurNB * KBLK;
        if (bk.kb < bk.k1) return true;
        for (++q; q < tg.ncont; ++q) {
          setup(q, bk);
          if (bk.k1 > 0) return true;
        }
        return false;
      };
      int qc = 0;
      Blk cur;
      bool have = false;
      for (; qc < tg.ncont; ++qc) {
        setup(qc, cur);
        if (cur.k1 > 0) {
          have = true;
          break;
        }
      }
      if (have) {
        T av0[kSchurNB][VK][2], bv0[kSchurNB][VK][2], av1[kSchurNB][VK][2], bv1[kSchurNB][VK][2];
        load(cur, av0, bv0);
        for (;;) {
          Blk nxt = cur;
          int qn = qc;
          const bool more = advance(qn, nxt);
          if (more) load(nxt, av1, bv1);
          prod(cur, av0, bv0);
          if (!more) break;
          cur = nxt;
          qc = qn;
#pragma unroll
          for (int q = 0; q < kSchurNB; ++q)
#pragma unroll
            for (int s2 = 0; s2 < VK; ++s2)
#pragma unroll
              for (int e = 0; e < 2; ++e) {
                av0[q][s2][e] = av1[q][s2][e];
                bv0[q][s2][e] = bv1[q][s2][e];
              }
        }
      }
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const int row = rb + a * 16 + l16;
        if (row >= nj) continue;
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int col = cb + b * 16 + acc_row<T>(kq, i);
            if (col < nk) C[row + col * nj] = cv[a][b][i] - acc[a][b][i];
          }
      }
    }
  }
}

template <class T>
void launch_schur(const SchurLevel<T>* lv, int ninst, int64_t rows, int c, SchurRow* rowtab,
                  SchurTarget* targets, int64_t* conts, int64_t* count, int64_t ccap, int* err,
                  hipStream_t s) {
  if (rows <= 0 || ninst <= 0) return;
  hipLaunchKernelGGL(k_fill<int64_t>, dim3(1), dim3(64), 0, s, count, (int64_t)2, (int64_t)0);
  hipLaunchKernelGGL(k_schur_enum<T>, dim3((unsigned)rows), dim3(256), 0, s, lv, ninst, c, rowtab,
                     targets, conts, count, ccap, err);
  // workgroups loop over however many targets the first launch found
  hipLaunchKernelGGL(k_schur_apply<T>, dim3(8192), dim3(256), 0, s, lv, ninst, c, rowtab, targets,
                     conts, count);
}

template <class T>
void launch_gemm(const GOut<T>* outs, int nouts, const GCon<T>* cons, const int32_t* dyn,
                 int64_t ntiles, int shape, hipStream_t s, T* parts) {
  if (ntiles <= 0 || nouts <= 0) return;
  if (shape == 0)
    hipLaunchKernelGGL((k_gemm<T, 2, 2, 2, 2>), dim3((unsigned)ntiles), dim3(256), 0, s, outs,
                       nouts, cons, dyn);
  else if (shape == 2)
    hipLaunchKernelGGL((k_gemm_out<T>), dim3((unsigned)nouts), dim3(256), 0, s, outs, cons, dyn);
  else if ((shape & 7) == 3) {
    if (shape & 8)
      hipLaunchKernelGGL((k_gemm_skinny<T, 2, VecK<T>::n>), dim3((unsigned)ntiles), dim3(256), 0,
                         s, outs, nouts, cons, dyn, parts);
    else
      hipLaunchKernelGGL((k_gemm_skinny<T, 2, 1>), dim3((unsigned)ntiles), dim3(256), 0, s, outs,
                         nouts, cons, dyn, parts);
  } else {
    if (shape & 8)
      hipLaunchKernelGGL((k_gemm_skinny<T, 1, VecK<T>::n>), dim3((unsigned)ntiles), dim3(256), 0,
                         s, outs, nouts, cons, dyn, parts);
    else
      hipLaunchKernelGGL((k_gemm_skinny<T, 1, 1>), dim3((unsigned)ntiles), dim3(256), 0, s, outs,
                         nouts, cons, dyn, parts);
  }
}

template <class T>
void launch_gemm_reduce(const GOut<T>* routs, int nouts, const T* parts, int64_t ntiles,
                        int shape, hipStream_t s) {
  if (ntiles <= 0 || nouts <= 0) return;
  if ((shape & 7) == 3)
    hipLaunchKernelGGL((k_gemm_reduce<T, 32>), dim3((unsigned)ntiles), dim3(256), 0, s, routs,
                       nouts, parts);
  else
    hipLaunchKernelGGL((k_gemm_reduce<T, 16>), dim3((unsigned)ntiles), dim3(256), 0, s, routs,
                       nouts, parts);
}

// ---------------------------------------------------------------------------
// In-place strip products with a cluster's orthogonal factor Q~.
// ---------------------------------------------------------------------------
template <class T>
__global__ __launch_bounds__(256) void k_strip(const STask<T>* __restrict__ tasks, int ntasks,
                                               const int32_t* __restrict__ dyn, int64_t nstrips,
                                               int group) {
  extern __shared__ char smem_raw[];
  T* xs = reinterpret_cast<T*>(smem_raw);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int l16 = lane & 15, kq = lane >> 4;
  // `group` consecutive strips per workgroup, one after the other
  const int64_t s_end = min(nstrips, (int64_t)(blockIdx.x + 1) * group);
  for (int64_t sid = (int64_t)blockIdx.x * group; sid < s_end; ++sid) {
    int lo = 0, hi = ntasks - 1;
    while (lo < hi) {
      int mid = (lo + hi + 1) >> 1;
      if (tasks[mid].strip0 <= sid) lo = mid; else hi = mid - 1;
    }
    const STask<T>& tk = tasks[lo];
    const int s = (int)(sid - tk.strip0);
    const int c0 = (tk.d0 >= 0 ? dyn[tk.d0] : tk.s0) + s * kStrip;
    if (c0 >= tk.ext) continue;  // the same for the whole workgroup
    const int w = min(kStrip, tk.ext - c0);
    const int n = tk.n;
    // the previous strip's products have read xs
    __syncthreads();
    if (tk.side == 0) {
      // X[:, c0:c0+w] (n x w) -> LDS, layout xs[k + c*n]
      for (int e = threadIdx.x; e < n * kStrip; e += blockDim.x) {
        const int r = e % n, c = e / n;
        xs[e] = c < w ? tk.X[r + (int64_t)(c0 + c) * tk.ldx] : T(0);
      }
      __syncthreads();
      for (int rt = wave; rt * 16 < n; rt += 4) {
        typename Acc<T>::type acc = {0, 0, 0, 0};
        const int row = rt * 16 + l16;
        // four k-steps' operands loaded ahead of their products (the
        // accumulation order is the plain ascending one)
        for (int kk = 0; kk < n; kk += 16) {
          T a[4], b[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int kx = kk + 4 * u + kq;
            a[u] = T(0);
            b[u] = T(0);
            if (kx < n) {
              if (row < n) a[u] = tk.trans ? tk.Q[kx + (int64_t)row * n] : tk.Q[row + (int64_t)kx * n];
              b[u] = xs[kx + l16 * n];
            }
          }
#pragma unroll
          for (int u = 0; u < 4; ++u)
            if (kk + 4 * u < n) acc = mfma16(a[u], b[u], acc);
        }
        const int col = l16;
        if (col < w) {
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int rr = rt * 16 + acc_row<T>(kq, i);
            if (rr < n) tk.X[rr + (int64_t)(c0 + col) * tk.ldx] = acc[i];
          }
        }
      }
    } else {
      // X[c0:c0+w, :] (w x n) -> LDS, layout xs[r + k*16]
      for (int e = threadIdx.x; e < n * kStrip; e += blockDim.x) {
        const int r = e % kStrip, k = e / kStrip;
        xs[e] = r < w ? tk.X[(c0 + r) + (int64_t)k * tk.ldx] : T(0);
      }
      __syncthreads();
      for (int ct = wave; ct * 16 < n; ct += 4) {
        typename Acc<T>::type acc = {0, 0, 0, 0};
        const int col = ct * 16 + l16;
        for (int kk = 0; kk < n; kk += 16) {
          T a[4], b[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int kx = kk + 4 * u + kq;
            a[u] = T(0);
            b[u] = T(0);
            if (kx < n) {
              a[u] = xs[l16 + kx * kStrip];
              if (col < n) b[u] = tk.trans ? tk.Q[col + (int64_t)kx * n] : tk.Q[kx + (int64_t)col * n];
            }
          }
#pragma unroll
          for (int u = 0; u < 4; ++u)
            if (kk + 4 * u < n) acc = mfma16(a[u], b[u], acc);
        }
        if (col < n) {
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int rr = acc_row<T>(kq, i);
            if (rr < w) tk.X[(c0 + rr) + (int64_t)col * tk.ldx] = acc[i];
          }
        }
      }
    }
  }
}

template <class T>
void launch_strip(const STask<T>* tasks, int ntasks, const int32_t* dyn, int64_t nstrips,
                  int maxn, hipStream_t s, int group) {
  if (nstrips <= 0 || ntasks <= 0) return;
  group = std::max(group, 1);
  const size_t lds = (size_t)maxn * kStrip * sizeof(T);
  static bool attr_set = false;
  if (!attr_set) {
    (void)hipFuncSetAttribute((const void*)k_strip<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              160 * 1024);
    attr_set = true;
  }
  const int64_t groups = (nstrips + group - 1) / group;
  hipLaunchKernelGGL(k_strip<T>, dim3((unsigned)groups), dim3(256), lds, s, tasks, ntasks, dyn,
                     nstrips, group);
}

// ---------------------------------------------------------------------------
// Basis augmentation and complement (Section 2.1, QR-based augmentation).
//  1. R = R-factor of Y^T, Y = [F_ij] the fill row, as a tall-skinny QR: the
//     workgroups of k_rfactor reduce groups of fill blocks (Householder on
//     stacked [R; next chunk of Y^T rows], triangle-on-top structured
//     reflectors) and later stages reduce the groups' factors alike;
// then, one workgroup per cluster (k_augment):
//  2. Householder QR of V; its reflectors give V_perp = H_0..H_{k-1} [0; I],
//     an orthonormal basis of the complement of V;
//  3. M' = R V_perp: the projected fill row (I - V V^T) Y equals
//     V_perp M'^T Q_Y^T, so one-sided Jacobi (Hestenes) on the columns of M'
//     with the rotations accumulated in W' yields its singular values (column
//     norms) and left singular vectors V_perp W';
//  4. Vbar = V_perp W'_sel for sigma > eps_fill (largest first) and the
//     complement of V~ = [V, Vbar] is V_perp W'_rest, so
//     Q~ = [V_perp W'_rest, V, V_perp W'_sel] with r = n - k~.
// ---------------------------------------------------------------------------
template <class T>
__device__ void structured_qr(T* R, T* C, int ldw, int n, int m, T* red) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __shared__ T sh_tau, sh_beta;
  for (int j = 0; j < n; ++j) {
    // norm of C[0:m, j]
    T v = (lane < m && wave == 0) ? C[lane + (int64_t)j * ldw] : T(0);
    if (wave == 0) {
      T s2 = wave_sum(v * v);
      if (lane == 0) {
        const T alpha = R[j + (int64_t)j * ldw];
        if (s2 == T(0)) {
          sh_tau = 0;
          sh_beta = alpha;
        } else {
          const T nrm = sqrt(alpha * alpha + s2);
          const T beta = alpha >= T(0) ? -nrm : nrm;
          sh_tau = (beta - alpha) / beta;
          sh_beta = beta;
        }
      }
    }
    __syncthreads();
    const T tau = sh_tau;
    if (tau != T(0)) {
      const T alpha = R[j + (int64_t)j * ldw];
      const T scale = T(1) / (alpha - sh_beta);
      __syncthreads();
      for (int t = threadIdx.x; t < m; t += blockDim.x) C[t + (int64_t)j * ldw] *= scale;
      if (threadIdx.x == 0) R[j + (int64_t)j * ldw] = sh_beta;
      __syncthreads();
      for (int c = j + 1 + wave; c < n; c += (int)(blockDim.x >> 6)) {
        T* Cc = C + (int64_t)c * ldw;
        const T* vj = C + (int64_t)j * ldw;
        T part = 0;
        for (int t = lane; t < m; t += 64) part += vj[t] * Cc[t];
        const T w = R[j + (int64_t)c * ldw] + wave_sum(part);
        const T tw = tau * w;
        for (int t = lane; t < m; t += 64) Cc[t] -= tw * vj[t];
        if (lane == 0) R[j + (int64_t)c * ldw] -= tw;
      }
    }
    __syncthreads();
  }
  (void)red;
}

// Load the next chunk of at most RPT rows of Y^T (fill columns) into the
// registers of the lanes that own columns: cr[u] = Y[col][row u].  (f, c0) is
// the position in the FillRef list (block, first unread column of it); rows
// beyond the end of the fill row are zero.  Returns the rows loaded.
template <class T, int RPT>
__device__ inline int rf_load_chunk(T (&cr)[RPT], const FillRef<T>* __restrict__ refs,
                                    const int32_t* __restrict__ dyn, int fend, int& f, int& c0,
                                    int col, int n) {
#pragma unroll
  for (int u = 0; u < RPT; ++u) cr[u] = T(0);
  int fill = 0;
  while (fill < RPT && f < fend) {
    const FillRef<T> fr = refs[f];
    const int take = min(RPT - fill, fr.ncols - c0);
    if (take > 0 && col < n) {
      const int64_t cs = fr_cs(fr);
      const gptr<const T> src = gmem(fr.F) + col * fr_rs(fr) + (int64_t)(c0 - fill) * cs;
#pragma unroll
      for (int u = 0; u < RPT; ++u)
        if (u >= fill && u < fill + take) cr[u] = src[(int64_t)u * cs];
    }
    fill += max(take, 0);
    c0 += max(take, 0);
    if (c0 >= fr.ncols) {
      ++f;
      c0 = (f < fend && refs[f].d0 >= 0) ? dyn[refs[f].d0] : 0;
    }
  }
  return fill;
}

template <class T> __device__ inline T lane_value(T v, int l);
template <> __device__ inline float lane_value<float>(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
template <> __device__ inline double lane_value<double>(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// ---------------------------------------------------------------------------
// One stage of the tall-skinny QR of fill rows: workgroup = group of fill
// blocks of one cluster, output its R factor as out[col + t n] = R[t][col].
// The fill block of a neighbour already skeletonized at this level is read
// from its active window (first column dyn[d0]).
//
// In LDS (orders up to 256): thread `col` owns column col of the stacked
// [R; chunk] and holds the chunk's rows of that column in registers.  Step j
// of a chunk: the owner of column j publishes it (x), its squared norm and
// alpha = R[j][j]; the reflector with vector [1; x / (alpha - beta)] zeroes
// the chunk's column j, and every column c > j takes w = R[j][c] + v . chunk_c,
// R[j][c] -= tau w, chunk_c -= tau w v.  R[j][c] is touched by its own lane
// only, so a step costs one barrier (a single-wave workgroup's barrier is
// free, and it reads the norm off the owner's lane).
// Otherwise R and the chunk live in `work` (structured_qr above).
// ---------------------------------------------------------------------------
template <class T>
__global__ __launch_bounds__(256) void k_rfactor(const RTask<T>* __restrict__ tasks,
                                                 const FillRef<T>* __restrict__ refs,
                                                 const int32_t* __restrict__ dyn, int lds) {
  extern __shared__ char rf_smem[];
  const RTask<T> tk = tasks[blockIdx.x];
  const int n = tk.n;
  const int tid = threadIdx.x, nthr = blockDim.x;
  __shared__ T red[8];
  if (n == 0) return;
  // same test as the host's (which gives `work` to the others); the launch
  // provides LDS for every in-LDS order of the launch and 64 threads per 64
  // columns
  if (rf_in_lds<T>(n, lds)) {
    constexpr int RPT = rf_chunk<T>();
    const int col = tid, lane = tid & 63;
    const bool one_wave = nthr == 64;
    // reflector buffers first (16-byte aligned vectors), then R
    T* xb = reinterpret_cast<T*>(rf_smem);
    T* Rr = xb + 2 * rf_xstride<T>();
    for (int64_t e = tid; e < (int64_t)n * (n + 1) / 2; e += nthr) Rr[e] = T(0);
    __syncthreads();
    int par = 0;
    T cr[RPT];
    // reflector steps j0..n-1 on the chunk in cr (its columns j < j0 are zero)
    auto run_steps = [&](int j0) {
      for (int j = j0; j < n; ++j, par ^= 1) {
        // the chunk's column j (x), its squared norm and alpha = R[j][j] as
        // wave-uniform values: read off the owner's lane (one wave) or
        // published in LDS, read once per wave (lane u takes x[u]) and
        // spread by lane reads
        T xs[RPT];
        T s2, alpha;
        T d0 = 0, d1 = 0;
        if (one_wave) {
#pragma unroll
          for (int u = 0; u < RPT; ++u) xs[u] = lane_value<T>(cr[u], j);
          alpha = Rr[rf_rowoff(j, n)];
        } else {
          T* x = xb + par * rf_xstride<T>();
          if (col == j) {
            T q0 = 0, q1 = 0;
#pragma unroll
            for (int u = 0; u < RPT; u += 2) {
              x[u] = cr[u];
              x[u + 1] = cr[u + 1];
              q0 += cr[u] * cr[u];
              q1 += cr[u + 1] * cr[u + 1];
            }
            x[RPT] = q0 + q1;
            x[RPT + 1] = Rr[rf_rowoff(j, n)];
          }
          __syncthreads();
          const T mine = x[lane < RPT ? lane : 0];
#pragma unroll
          for (int u = 0; u < RPT; ++u) xs[u] = lane_value<T>(mine, u);
          s2 = x[RPT];
          alpha = x[RPT + 1];
        }
#pragma unroll
        for (int u = 0; u < RPT; u += 2) {
          d0 += xs[u] * cr[u];
          d1 += xs[u + 1] * cr[u + 1];
        }
        const T d = d0 + d1;
        // one wave: the squared norm is the owner's own d (same summation
        // order as the published sum)
        if (one_wave) s2 = lane_value<T>(d, j);
        if (s2 != T(0)) {
          const T nrm = sqrt(alpha * alpha + s2);
          const T beta = alpha >= T(0) ? -nrm : nrm;
          const T tau = (beta - alpha) / beta;
          const T scale = T(1) / (alpha - beta);
          if (col > j && col < n) {
            T* rjc = Rr + rf_rowoff(j, n) + (col - j);
            const T r0 = *rjc;
            const T tw = tau * (r0 + scale * d);
            const T fct = tw * scale;
#pragma unroll
            for (int u = 0; u < RPT; ++u) cr[u] -= fct * xs[u];
            *rjc = r0 - tw;
          }
          if (col == j) Rr[rf_rowoff(j, n)] = beta;
        }
      }
    };
    if (tk.tri) {
      // stacked factors of a previous stage: the first is R itself, the
      // others enter in chunks of RPT rows; rows t0.. of an upper triangular
      // factor are zero in the columns before t0
      if (tk.fend > tk.fbeg) {
        const gptr<const T> F0 = gmem(refs[tk.fbeg].F);
        for (int64_t e = tid; e < (int64_t)n * n; e += nthr) {
          const int t = (int)(e / n), c = (int)(e % n);
          if (t <= c) Rr[rf_rowoff(t, n) + (c - t)] = F0[c + (int64_t)t * n];
        }
      }
      __syncthreads();
      for (int f = tk.fbeg + 1; f < tk.fend; ++f) {
        const gptr<const T> Fb = gmem(refs[f].F);
        for (int t0 = 0; t0 < n; t0 += RPT) {
#pragma unroll
          for (int u = 0; u < RPT; ++u)
            cr[u] = (col < n && t0 + u < n) ? Fb[col + (int64_t)(t0 + u) * n] : T(0);
          run_steps(t0);
        }
      }
    } else {
      int f = tk.fbeg;
      int c0 = (f < tk.fend && refs[f].d0 >= 0) ? dyn[refs[f].d0] : 0;
      for (;;) {
        const int rows = rf_load_chunk<T, RPT>(cr, refs, dyn, tk.fend, f, c0, col, n);
        if (rows == 0) break;
        run_steps(0);
      }
    }
    __syncthreads();
    if (col < n) {
      const gptr<T> out = gmem(tk.out);
      for (int t = 0; t < n; ++t)
        out[col + (int64_t)t * n] = t <= col ? Rr[rf_rowoff(t, n) + (col - t)] : T(0);
    }
  } else {
    const int ldw = n + kAugChunk;
    T* R = tk.work;  // rows 0..n-1 = R, rows n..n+63 = chunk
    T* C = R + n;
    for (int e = tid; e < n * n; e += nthr) R[(e % n) + (int64_t)(e / n) * ldw] = 0;
    __syncthreads();
    int fill = 0;
    for (int f = tk.fbeg; f < tk.fend; ++f) {
      const FillRef<T> fr = refs[f];
      int c = fr.d0 >= 0 ? dyn[fr.d0] : 0;
      while (c < fr.ncols) {
        const int take = min(kAugChunk - fill, fr.ncols - c);
        const int64_t rs = fr_rs(fr), cs = fr_cs(fr);
        for (int e = tid; e < take * n; e += nthr) {
          const int tt = e / n, col = e % n;
          C[(fill + tt) + (int64_t)col * ldw] = fr.F[col * rs + (int64_t)(c + tt) * cs];
        }
        fill += take;
        c += take;
        __syncthreads();
        if (fill == kAugChunk) {
          structured_qr(R, C, ldw, n, fill, red);
          fill = 0;
        }
      }
    }
    if (fill > 0) structured_qr(R, C, ldw, n, fill, red);
    __syncthreads();
    for (int e = tid; e < n * n; e += nthr) {
      const int col = e % n, t = e / n;
      tk.out[e] = t <= col ? R[t + (int64_t)col * ldw] : T(0);
    }
  }
}

template <class T>
void launch_rfactor(const RTask<T>* tasks, int ntasks, const FillRef<T>* refs,
                    const int32_t* dyn, int maxn, hipStream_t s, int lds) {
  if (ntasks <= 0) return;
  lds = std::min(lds, kLdsBytes);
  // every order of the launch fits in LDS: 64 threads per 64 columns of the
  // largest and its LDS; otherwise 256 threads (enough for every in-LDS
  // order) and the full LDS allowance
  const bool in_lds = rf_in_lds<T>(maxn, lds);
  const int threads = in_lds ? 64 * ((maxn + 63) / 64) : 256;
  const int64_t need = in_lds ? rf_lds_elems<T>(maxn) : lds / (int64_t)sizeof(T);
  static bool attr_set = false;
  if (!attr_set) {
    (void)hipFuncSetAttribute((const void*)k_rfactor<T>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBytes);
    attr_set = true;
  }
  hipLaunchKernelGGL(k_rfactor<T>, dim3(ntasks), dim3(threads), (size_t)(need * sizeof(T)), s,
                     tasks, refs, dyn, lds);
}

// ---------------------------------------------------------------------------
// Gram matrix of a cluster's fill row for the FP32 factorization (Section 2.1,
// first augmentation option): G = Y Y^T over the active columns of the fill
// blocks, in FP64 from the FP32 entries (their products are exact), on FP64
// MFMA.  Workgroup = one 64 x 64 tile of G; each wave owns a 32 x 32 quarter
// (2 x 2 fragments) and runs over every fill column, four k-steps at a time.
// ---------------------------------------------------------------------------
template <class T>
__global__ __launch_bounds__(256) void k_gram(const GramTask<T>* __restrict__ tasks, int ntasks,
                                              const FillRef<T>* __restrict__ refs,
                                              const int32_t* __restrict__ dyn) {
  const int64_t tile = blockIdx.x;
  int lo = 0, hi = ntasks - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (tasks[mid].tile0 <= tile) lo = mid; else hi = mid - 1;
  }
  const GramTask<T>& tk = tasks[lo];
  const int n = tk.n;
  const int64_t t = tile - tk.tile0;
  const int ti = (int)(t % tk.tm), tj = (int)(t / tk.tm);
  // G is symmetric: tiles and 32 x 32 quadrants below the diagonal are
  // written as the mirror of the ones above it
  if (ti > tj) return;
  const int r0 = ti * 64, c0 = tj * 64;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int l16 = lane & 15, kq = lane >> 4;
  const int qr = wave & 1, qc = wave >> 1;
  if (ti == tj && qr > qc) return;
  const bool mirror = ti != tj || qr != qc;
  const int wr = r0 + qr * 32, wc = c0 + qc * 32;
  typename Acc<double>::type acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = (typename Acc<double>::type){0, 0, 0, 0};
  for (int f = tk.fbeg; f < tk.fend; ++f) {
    const FillRef<T> fr = refs[f];
    const int k0 = fr.d0 >= 0 ? dyn[fr.d0] : 0;
    const int k1 = fr.ncols;
    const int64_t rs = fr_rs(fr), cs = fr_cs(fr);
    // a block stored transposed has its k index contiguous: each lane then
    // reads four consecutive k of its row as one vector (FP32), and step s4
    // takes k = kk + 4 kq + s4 (any order of k gives the same Gram matrix
    // up to rounding)
    const bool kvec = sizeof(T) == 4 && fr.tr;
    for (int kk = k0; kk < k1; kk += 16) {
      double av[4][2], bv[4][2];
      if (kvec) {
        const int kl = kk + 4 * kq;
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          const int row = (a < 2 ? wr + a * 16 : wc + (a - 2) * 16) + l16;
          double v4[4];
          if (row < n && kl + 4 <= k1) {
            const typename VecK<T>::type v = ld_veck<T>(gmem((const T*)fr.F) + kl + (int64_t)row * rs);
#pragma unroll
            for (int s4 = 0; s4 < 4; ++s4) v4[s4] = double(v[s4 % VecK<T>::n]);
          } else {
#pragma unroll
            for (int s4 = 0; s4 < 4; ++s4)
              v4[s4] = (row < n && kl + s4 < k1) ? double(fr.F[kl + s4 + (int64_t)row * rs]) : 0.0;
          }
#pragma unroll
          for (int s4 = 0; s4 < 4; ++s4) {
            if (a < 2) av[s4][a] = v4[s4]; else bv[s4][a - 2] = v4[s4];
          }
        }
      } else {
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) {
          const int kx = kk + 4 * s4 + kq;
          const bool kok = kx < k1;
          const T* col = fr.F + (int64_t)kx * cs;
#pragma unroll
          for (int a = 0; a < 2; ++a) {
            const int row = wr + a * 16 + l16;
            av[s4][a] = (kok && row < n) ? double(col[row * rs]) : 0.0;
          }
#pragma unroll
          for (int b = 0; b < 2; ++b) {
            const int cc = wc + b * 16 + l16;
            bv[s4][b] = (kok && cc < n) ? double(col[cc * rs]) : 0.0;
          }
        }
      }
      // G = Y Y^T: the "B" operand is Y^T, whose (k, col) entry is Y[col][k];
      // operands enter swapped so the accumulator holds the transposed block
#pragma unroll
      for (int s4 = 0; s4 < 4; ++s4)
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int b = 0; b < 2; ++b) acc[a][b] = mfma16(bv[s4][b], av[s4][a], acc[a][b]);
    }
  }
#pragma unroll
  for (int a = 0; a < 2; ++a) {
    const int row = wr + a * 16 + l16;
    if (row >= n) continue;
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int cc = wc + b * 16 + acc_row<double>(kq, i);
        if (cc < n) {
          tk.G[row + (int64_t)cc * n] = acc[a][b][i];
          if (mirror) tk.G[cc + (int64_t)row * n] = acc[a][b][i];
        }
      }
  }
}

// Cholesky with diagonal pivoting of a summed Gram matrix (CholTask), in LDS,
// one workgroup per task.
template <class T>
__global__ __launch_bounds__(256) void k_pchol(const CholTask<T>* __restrict__ tasks) {
  extern __shared__ char pc_smem[];
  const CholTask<T> tk = tasks[blockIdx.x];
  const int n = tk.n;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  double* Gs = reinterpret_cast<double*>(pc_smem);  // Gs[a + b n]
  int* perm = reinterpret_cast<int*>(Gs + (int64_t)n * n);
  int* iperm = perm + n;
  __shared__ double wv[4];
  __shared__ int wi[4];
  if (n == 0) return;
  // the partial Gram matrices, summed in chunk order
  const gptr<const double> Gg = gmem(tk.G);
  // eight independent loads in flight per thread and chunk
  for (int e0 = tid; e0 < n * n; e0 += 256 * 8) {
    double acc[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) acc[u] = 0;
    for (int c = 0; c < tk.nch; ++c)
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = e0 + 256 * u;
        if (e < n * n) acc[u] += Gg[(int64_t)c * n * n + e];
      }
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (e0 + 256 * u < n * n) Gs[e0 + 256 * u] = acc[u];
  }
  for (int j = tid; j < n; j += 256) perm[j] = j;
  __syncthreads();
  // largest remaining diagonal entry at or after j (ties: the smallest index)
  auto pivot = [&](int j, double& dv, int& di) {
    double v = -1.0;
    int ix = n;
    for (int i = j + tid; i < n; i += 256) {
      const double g = Gs[i + (int64_t)i * n];
      if (g > v) {
        v = g;
        ix = i;
      }
    }
    for (int o = 32; o > 0; o >>= 1) {
      const double v2 = __shfl_xor(v, o, 64);
      const int i2 = __shfl_xor(ix, o, 64);
      if (v2 > v || (v2 == v && i2 < ix)) {
        v = v2;
        ix = i2;
      }
    }
    if (lane == 0) {
      wv[wave] = v;
      wi[wave] = ix;
    }
    __syncthreads();
    dv = wv[0];
    di = wi[0];
    for (int w = 1; w < 4; ++w)
      if (wv[w] > dv || (wv[w] == dv && wi[w] < di)) {
        dv = wv[w];
        di = wi[w];
      }
    __syncthreads();
  };
  double dmax;
  int dummy;
  pivot(0, dmax, dummy);
  const double thr = fmax(1e-6 * tk.eps * tk.eps, 64.0 * n * DBL_EPSILON * dmax);
  int rank = 0;
  for (int j = 0; j < n; ++j) {
    double d;
    int p;
    pivot(j, d, p);
    if (!(d > thr)) break;
    rank = j + 1;
    if (p != j) {
      // symmetric exchange of rows and columns j and p (the computed rows of
      // R take the column exchange too)
      for (int e = tid; e < n; e += 256) {
        const double x = Gs[j + (int64_t)e * n];
        Gs[j + (int64_t)e * n] = Gs[p + (int64_t)e * n];
        Gs[p + (int64_t)e * n] = x;
      }
      __syncthreads();
      for (int e = tid; e < n; e += 256) {
        const double x = Gs[e + (int64_t)j * n];
        Gs[e + (int64_t)j * n] = Gs[e + (int64_t)p * n];
        Gs[e + (int64_t)p * n] = x;
      }
      if (tid == 0) {
        const int x = perm[j];
        perm[j] = perm[p];
        perm[p] = x;
      }
      __syncthreads();
    }
    // row j of R: R[j][i] = G[j][i] / sqrt(G[j][j]), i >= j
    const double rd = sqrt(Gs[j + (int64_t)j * n]);
    __syncthreads();
    for (int i = j + tid; i < n; i += 256) Gs[j + (int64_t)i * n] /= rd;
    __syncthreads();
    // trailing update G[a][b] -= R[j][a] R[j][b], a, b > j
    const int m = n - j - 1;
    for (int e = tid; e < m * m; e += 256) {
      const int a = j + 1 + e % m, b = j + 1 + e / m;
      Gs[a + (int64_t)b * n] -= Gs[j + (int64_t)a * n] * Gs[j + (int64_t)b * n];
    }
    __syncthreads();
  }
  for (int c = tid; c < n; c += 256) iperm[perm[c]] = c;
  __syncthreads();
  // (R P^T)[a][b] = R[a][c] with perm[c] = b
  const gptr<T> Rt = gmem(tk.Rt);
  for (int e = tid; e < n * n; e += 256) {
    const int b = e % n, a = e / n;
    const int c = iperm[b];
    Rt[b + (int64_t)a * n] = (a < rank && c >= a) ? T(Gs[a + (int64_t)c * n]) : T(0);
  }
  if (threadIdx.x == 0) *reinterpret_cast<__attribute__((address_space(1))) int32_t*>(Rt + (int64_t)n * n) = rank;
}

// The same for orders up to 64 with one wave per task: lane l owns column l
// of the working matrix in LDS, the pivot search is a wave reduction and the
// barriers cost next to nothing.
template <class T>
__global__ __launch_bounds__(64) void k_pchol_wave(const CholTask<T>* __restrict__ tasks) {
  extern __shared__ char pc_smem[];
  const CholTask<T> tk = tasks[blockIdx.x];
  const int n = tk.n;
  const int l = threadIdx.x;
  double* Gs = reinterpret_cast<double*>(pc_smem);  // Gs[a + b n], column b of lane b
  int* perm = reinterpret_cast<int*>(Gs + (int64_t)n * n);
  int* iperm = perm + n;
  if (n == 0) return;
  const gptr<const double> Gg = gmem(tk.G);
  // sixteen independent loads in flight per lane and chunk
  for (int e0 = l; e0 < n * n; e0 += 64 * 16) {
    double acc[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) acc[u] = 0;
    for (int c = 0; c < tk.nch; ++c)
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int e = e0 + 64 * u;
        if (e < n * n) acc[u] += Gg[(int64_t)c * n * n + e];
      }
#pragma unroll
    for (int u = 0; u < 16; ++u)
      if (e0 + 64 * u < n * n) Gs[e0 + 64 * u] = acc[u];
  }
  if (l < n) perm[l] = l;
  __syncthreads();
  // largest remaining diagonal entry at or after j (ties: the smallest index)
  auto pivot = [&](int j, double& dv, int& di) {
    double v = (l >= j && l < n) ? Gs[l + (int64_t)l * n] : -1.0;
    int ix = (l >= j && l < n) ? l : n;
    for (int o = 32; o > 0; o >>= 1) {
      const double v2 = __shfl_xor(v, o, 64);
      const int i2 = __shfl_xor(ix, o, 64);
      if (v2 > v || (v2 == v && i2 < ix)) {
        v = v2;
        ix = i2;
      }
    }
    dv = v;
    di = ix;
  };
  double dmax;
  int dummy;
  pivot(0, dmax, dummy);
  const double thr = fmax(1e-6 * tk.eps * tk.eps, 64.0 * n * DBL_EPSILON * dmax);
  int rank = 0;
  for (int j = 0; j < n; ++j) {
    double d;
    int p;
    pivot(j, d, p);
    if (!(d > thr)) break;
    rank = j + 1;
    if (p != j) {
      if (l < n) {  // rows j and p of column l, then columns j and p of row l
        double x = Gs[j + (int64_t)l * n];
        Gs[j + (int64_t)l * n] = Gs[p + (int64_t)l * n];
        Gs[p + (int64_t)l * n] = x;
      }
      __syncthreads();
      if (l < n) {
        double x = Gs[l + (int64_t)j * n];
        Gs[l + (int64_t)j * n] = Gs[l + (int64_t)p * n];
        Gs[l + (int64_t)p * n] = x;
      }
      if (l == 0) {
        const int x = perm[j];
        perm[j] = perm[p];
        perm[p] = x;
      }
      __syncthreads();
    }
    const double rd = sqrt(Gs[j + (int64_t)j * n]);
    __syncthreads();
    if (l >= j && l < n) Gs[j + (int64_t)l * n] /= rd;
    __syncthreads();
    if (l > j && l < n) {
      const double rb = Gs[j + (int64_t)l * n];
      for (int a = j + 1; a < n; ++a) Gs[a + (int64_t)l * n] -= Gs[j + (int64_t)a * n] * rb;
    }
    __syncthreads();
  }
  if (l < n) iperm[perm[l]] = l;
  __syncthreads();
  const gptr<T> Rt = gmem(tk.Rt);
  for (int e = l; e < n * n; e += 64) {
    const int b = e % n, a = e / n;
    const int c = iperm[b];
    Rt[b + (int64_t)a * n] = (a < rank && c >= a) ? T(Gs[a + (int64_t)c * n]) : T(0);
  }
  if (threadIdx.x == 0) *reinterpret_cast<__attribute__((address_space(1))) int32_t*>(Rt + (int64_t)n * n) = rank;
}

template <class T> void launch_pchol(const CholTask<T>* tasks, int ntasks, int maxn, hipStream_t s) {
  if (ntasks <= 0) return;
  if (maxn <= 64) {
    const size_t lds = (size_t)maxn * maxn * sizeof(double) + 2 * (size_t)maxn * sizeof(int);
    hipLaunchKernelGGL(k_pchol_wave<T>, dim3((unsigned)ntasks), dim3(64), lds, s, tasks);
    return;
  }
  const size_t lds = (size_t)maxn * maxn * sizeof(double) + 2 * (size_t)maxn * sizeof(int);
  static bool attr = false;
  if (!attr) {
    (void)hipFuncSetAttribute((const void*)k_pchol<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              kLdsBytes);
    attr = true;
  }
  hipLaunchKernelGGL(k_pchol<T>, dim3((unsigned)ntasks), dim3(256), lds, s, tasks);
}

template <class T>
void launch_gram(const GramTask<T>* tasks, int ntasks, const FillRef<T>* refs,
                 const int32_t* dyn, int64_t ntiles, hipStream_t s) {
  if (ntasks <= 0 || ntiles <= 0) return;
  hipLaunchKernelGGL(k_gram<T>, dim3((unsigned)ntiles), dim3(256), 0, s, tasks, ntasks, refs,
                     dyn);
}

// T: storage type of V, R and Q~; A: arithmetic type.  GRAM: the fill row
// comes as its FP64 Gram matrix G = Y Y^T instead of R (FP32 factorization),
// and Jacobi runs on M = V_perp^T G V_perp (mp x mp), whose column norms after
// convergence are the squared singular values.
template <class T, class A, bool GRAM>
__global__ __launch_bounds__(1024) void k_augment(const AugTask<T>* __restrict__ tasks,
                                                 int32_t* __restrict__ rout, int* err,
                                                 int lds_elems) {
  extern __shared__ char aug_smem[];
  const AugTask<T> tk = tasks[blockIdx.x];
  const A eps_fill = A(tk.eps);
  const int n = tk.n, k = tk.k;
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int wave = tid >> 6, lane = tid & 63, nw = nthr >> 6;
  __shared__ A red[16];
  __shared__ int sh_flag;
  if (n == 0) {
    if (tid == 0) rout[tk.ri] = 0;
    return;
  }
  const T* Rt = tk.Rt;                          // Rt[b + a n] = R[a][b]
  const double* Gy = tk.G;                      // Gram matrix of the fill row (GRAM)
  // global scratch, one region per phase (no phase writes where another
  // phase's data were read): V_perp | reflectors of V | M' (or M) and W' | G V_perp
  A* G = reinterpret_cast<A*>(tk.work);         // n x n (V_perp)
  A* Hr = G + (int64_t)n * n;                   // n^2 (reflectors of V)
  A* Hm = Hr + (int64_t)n * n;                  // 2 n^2 (M' or M, and W')
  A* Hg = Hm + 2 * (int64_t)n * n;              // n^2 (G V_perp)
  A* sig = Hg + (int64_t)n * n;                 // n
  A* tau = sig + n;                             // n
  int* rank = reinterpret_cast<int*>(tau + n);  // n ints (fit in n A's)
  T* Q = tk.Q;
  // barrier between phases; the scratch in global memory is private to the
  // workgroup, whose waves share one CU, so the barrier's workgroup-scope
  // release/acquire orders those accesses as well as LDS.  The Gram variant
  // (glob: the next phase reads global scratch) adds agent-scope fences: its
  // results are wrong without them, for a reason not yet identified.
  auto bsync = [&](bool glob) {
    if (GRAM && glob) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (GRAM && glob) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  };

  // ---- 2. Householder QR of V (n x k): reflectors H_0 .. H_{k-1} ----
  const int mp = n - k;  // dimension of the complement of V
  const int64_t cap = lds_elems;
  A* smem = reinterpret_cast<A*>(aug_smem);
  const bool bc_lds = (int64_t)n * n + 8 <= cap;
  A* Hv = bc_lds ? smem : Hr;                          // n x k reflectors, ld n
  A* Xp = bc_lds ? smem + (int64_t)n * k : G;          // n x mp complement, ld n
  for (int e = tid; e < n * k; e += nthr) Hv[e] = A(tk.V[e]);
  bsync(!bc_lds);
  for (int j = 0; j < k; ++j) {
    A* hj = Hv + (int64_t)j * n;
    A sq = 0;
    for (int t = j + 1 + tid; t < n; t += nthr) sq += hj[t] * hj[t];
    sq = block_sum(sq, red);
    const A alpha = hj[j];
    A tj = 0, beta = alpha;
    if (sq != A(0)) {
      const A nrm = sqrt(alpha * alpha + sq);
      beta = alpha >= A(0) ? -nrm : nrm;
      tj = (beta - alpha) / beta;
    }
    if (tj != A(0)) {
      const A scale = A(1) / (alpha - beta);
      for (int t = j + 1 + tid; t < n; t += nthr) hj[t] *= scale;
    }
    bsync(!bc_lds);
    if (tid == 0) {
      hj[j] = A(1);  // implicit unit of the reflector, stored explicitly
      tau[j] = tj;
    }
    bsync(!bc_lds);
    if (tj != A(0)) {
      for (int c = j + 1 + wave; c < k; c += nw) {
        A* hc = Hv + (int64_t)c * n;
        A d = 0;
        for (int t = j + lane; t < n; t += 64) d += hj[t] * hc[t];
        d = wave_sum(d) * tj;
        for (int t = j + lane; t < n; t += 64) hc[t] -= d * hj[t];
      }
    }
    bsync(!bc_lds);
  }
  // ---- 3. V_perp = H_0 ... H_{k-1} [0; I_mp], the complement of V ----
  for (int e = tid; e < n * mp; e += nthr) {
    const int row = e % n, c = e / n;
    Xp[e] = (row == k + c) ? A(1) : A(0);
  }
  bsync(!bc_lds);
  for (int j = k - 1; j >= 0; --j) {
    const A tj = tau[j];
    if (tj == A(0)) continue;
    const A* hj = Hv + (int64_t)j * n;
    for (int c = wave; c < mp; c += nw) {
      A* xc = Xp + (int64_t)c * n;
      A d = 0;
      for (int t = j + lane; t < n; t += 64) d += hj[t] * xc[t];
      d = wave_sum(d) * tj;
      for (int t = j + lane; t < n; t += 64) xc[t] -= d * hj[t];
    }
    bsync(!bc_lds);
  }
  A* Vp = G;  // keep V_perp in global scratch (n x mp, ld n)
  if (bc_lds)
    for (int e = tid; e < n * mp; e += nthr) Vp[e] = Xp[e];
  bsync(true);

  // ---- 4. the matrix whose columns Jacobi orthogonalizes, and W' = I ----
  // R path: M' = R V_perp (n x mp).  The projected fill row is
  // (I - V V^T) Y = V_perp V_perp^T R^T Q_Y^T, so its nonzero singular values
  // and left singular vectors are those of M'^T mapped by V_perp.
  // GRAM path: M = V_perp^T G V_perp (mp x mp), symmetric positive
  // semidefinite; its right singular vectors are its eigenvectors and its
  // singular values the squares of those of the projected fill row.
  // length of the columns Jacobi rotates: mp for M; n for M' = R V_perp,
  // or the rank of a pivoted Cholesky factor (rows past it are zero), stored
  // after the factor
  const int mrow = GRAM ? mp : tk.rgen ? min(n, *reinterpret_cast<const int32_t*>(Rt + (int64_t)n * n)) : n;
  const bool de_lds = (int64_t)mrow * mp + (int64_t)mp * mp + 8 <= cap;
  A* Ms = de_lds ? smem : Hm;                                       // mrow x mp, ld mrow
  A* Ws = de_lds ? smem + (int64_t)mrow * mp : Hm + (int64_t)mrow * mp;  // mp x mp
  if constexpr (GRAM) {
    A* GV = Hg;  // G V_perp, n x mp
    for (int e = tid; e < n * mp; e += nthr) {
      const int a = e % n, c = e / n;
      A acc = 0;
      for (int b = 0; b < n; ++b) acc += A(Gy[a + (int64_t)b * n]) * Vp[b + (int64_t)c * n];
      GV[e] = acc;
    }
    bsync(true);
    for (int e = tid; e < mp * mp; e += nthr) {
      const int a = e % mp, c = e / mp;
      A acc = 0;
      for (int b = 0; b < n; ++b) acc += Vp[b + (int64_t)a * n] * GV[b + (int64_t)c * n];
      Ms[e] = acc;
    }
  } else {
    for (int e = tid; e < mrow * mp; e += nthr) {
      const int a = e % mrow, c = e / mrow;
      A acc = 0;
      for (int b = tk.rgen ? 0 : a; b < n; ++b) acc += A(Rt[b + (int64_t)a * n]) * Vp[b + (int64_t)c * n];
      Ms[e] = acc;
    }
  }
  for (int e = tid; e < mp * mp; e += nthr) Ws[e] = (e % mp == e / mp) ? A(1) : A(0);
  bsync(!de_lds);

  // ---- 5. one-sided Jacobi on the columns of M' (or M) ----
  // Round-robin ordering: every round rotates ne/2 disjoint column pairs.  A
  // group of LG lanes takes a pair (rows t = gl + LG u staged in registers);
  // LG is chosen per cluster so the pairs of a round spread over the groups.
  constexpr int RJ = 16;
  const int ne = (mp + 1) & ~1;
  const int npair = ne / 2;
  int LG = 8;
  {
    int best = 1 << 30;
    for (int g = 8; g <= 64; g <<= 1) {
      if ((mrow + g - 1) / g > RJ) continue;
      const int passes = (npair + nthr / g - 1) / (nthr / g);
      const int cost = passes * ((mrow + g - 1) / g + 2 * __builtin_ctz(g));
      if (cost < best) {
        best = cost;
        LG = g;
      }
    }
  }
  const int grp = tid / LG, gl = tid % LG, ngrp = nthr / LG;
  const A tolj = eps_of<A>() * A(mrow);
  // FP32 arithmetic: a pair whose inner product is below gabs_min counts as
  // converged.  Off-diagonal entries of the columns' Gram matrix that small
  // move its eigenvalues by at most mp gabs_min = 4e-3 eps_fill^2, so a
  // singular value moves by at most 0.2% of eps_fill near the threshold: the
  // truncation is unaffected, and the noise-level columns below eps_fill stop
  // being rotated sweep after sweep.
  const A gabs_min = sizeof(A) == 4 ? A(4e-3) * eps_fill * eps_fill / A(mp > 40 ? mp : 40) : A(0);
  for (int sweep = 0; sweep < 40 && mp > 1; ++sweep) {
    if (tid == 0) sh_flag = 0;
    __syncthreads();
    for (int rnd = 0; rnd < ne - 1; ++rnd) {
      for (int p = grp; p < npair; p += ngrp) {
        int a, b;
        if (p == 0) {
          a = rnd;
          b = ne - 1;
        } else {
          a = (rnd + p) % (ne - 1);
          b = (rnd - p + ne - 1) % (ne - 1);
        }
        if (a >= mp || b >= mp) continue;
        A* ga = Ms + (int64_t)a * mrow;
        A* gb = Ms + (int64_t)b * mrow;
        A x[RJ], y[RJ];
        A al = 0, be = 0, gab = 0;
#pragma unroll
        for (int u = 0; u < RJ; ++u) {
          const int t = gl + LG * u;
          x[u] = t < mrow ? ga[t] : A(0);
          y[u] = t < mrow ? gb[t] : A(0);
          al += x[u] * x[u];
          be += y[u] * y[u];
          gab += x[u] * y[u];
        }
        for (int o = 1; o < LG; o <<= 1) {
          al += __shfl_xor(al, o, 64);
          be += __shfl_xor(be, o, 64);
          gab += __shfl_xor(gab, o, 64);
        }
        // relative test against sqrt(al) sqrt(be): the product al be can
        // underflow for tiny columns, and a zero there would make every
        // nonzero gab look unconverged
        const A nab = sqrt(al) * sqrt(be);
        if (gab != A(0) && nab > A(0) && fabs(gab) > tolj * nab && fabs(gab) > gabs_min) {
          const A zeta = (be - al) / (A(2) * gab);
          const A tt = (zeta >= A(0) ? A(1) : A(-1)) / (fabs(zeta) + sqrt(A(1) + zeta * zeta));
          const A cs = A(1) / sqrt(A(1) + tt * tt);
          const A sn = cs * tt;
#pragma unroll
          for (int u = 0; u < RJ; ++u) {
            const int t = gl + LG * u;
            if (t < mrow) {
              ga[t] = cs * x[u] - sn * y[u];
              gb[t] = sn * x[u] + cs * y[u];
            }
          }
          A* wa = Ws + (int64_t)a * mp;
          A* wb = Ws + (int64_t)b * mp;
#pragma unroll
          for (int u = 0; u < RJ; ++u) {
            const int t = gl + LG * u;
            const A wu = t < mp ? wa[t] : A(0), wv = t < mp ? wb[t] : A(0);
            if (t < mp) {
              wa[t] = cs * wu - sn * wv;
              wb[t] = sn * wu + cs * wv;
            }
          }
          if (gl == 0) sh_flag = 1;
        }
      }
      bsync(!de_lds);
    }
    const int fl = sh_flag;
    __syncthreads();
    if (!fl) break;
  }
  for (int c = wave; c < mp; c += nw) {
    A sq = 0;
    for (int t = lane; t < mrow; t += 64) sq += Ms[t + (int64_t)c * mrow] * Ms[t + (int64_t)c * mrow];
    sq = wave_sum(sq);
    // R path: the column norm is sigma; GRAM path: it is sigma^2
    if (lane == 0) sig[c] = GRAM ? sqrt(sqrt(sq)) : sqrt(sq);
  }
  bsync(true);

  // ---- 6. selection and Q~ = [V_perp W'_rest, V, V_perp W'_sel] ----
  for (int c = tid; c < mp; c += nthr) {
    int pos = 0;
    const A sc = sig[c];
    for (int i = 0; i < mp; ++i) {
      const A si = sig[i];
      pos += (si > sc) || (si == sc && i < c);
    }
    rank[c] = pos;
  }
  if (tid == 0) {
    int cnt = 0;
    for (int i = 0; i < mp; ++i) cnt += sig[i] > eps_fill;
    sh_flag = cnt;
  }
  __syncthreads();
  const int rbar = sh_flag;
  const int kt = k + rbar;
  const int r = n - kt;
  // column of Q~ receiving the rotated complement vector c: the rbar largest
  // singular directions (in decreasing order) follow V, the others come first
  for (int e = tid; e < n * mp; e += nthr) {
    const int t = e % n, c = e / n;
    const int pos = rank[c];
    const int qcol = pos < rbar ? kt - rbar + pos + r : pos - rbar;
    A acc = 0;
    for (int b = 0; b < mp; ++b) acc += Vp[t + (int64_t)b * n] * Ws[b + (int64_t)c * mp];
    Q[t + (int64_t)qcol * n] = T(acc);
  }
  for (int e = tid; e < n * k; e += nthr) Q[(int64_t)r * n + e] = tk.V[e];
  if (tid == 0) {
    rout[tk.ri] = r;
    for (int i = 0; i < mp; ++i)
      if (!(sig[i] == sig[i])) atomicOr(err, 2);
  }
}

template <class T, class A, bool GRAM>
static void launch_augment_t(const AugTask<T>* tasks, int ntasks, int32_t* r, int* err, int maxn,
                             hipStream_t s, int lds) {
  // LDS: the reflectors of V and V_perp (n^2), then M' and W' (at most 2 n^2)
  const int64_t cap = std::min(lds, kLdsBytes) / (int64_t)sizeof(A);
  const int64_t need = std::min<int64_t>(cap, 2 * (int64_t)maxn * maxn + 8);
  static bool attr_set = false;
  if (!attr_set) {
    (void)hipFuncSetAttribute((const void*)k_augment<T, A, GRAM>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBytes);
    attr_set = true;
  }
  // workgroup size from the largest order: the Jacobi rotates (n - k) / 2
  // column pairs per round, a group of 8 to 64 lanes each, and a round ends
  // with a barrier over every wave, so small clusters take fewer waves
  const int threads = maxn <= 64 ? 128 : maxn <= 128 ? 256 : maxn <= 256 ? 512 : 1024;
  hipLaunchKernelGGL((k_augment<T, A, GRAM>), dim3(ntasks), dim3(threads),
                     (size_t)(need * sizeof(A)), s, tasks, r, err, (int)need);
}

template <class T>
void launch_augment(const AugTask<T>* tasks, int ntasks, int32_t* r, int* err, int maxn, bool gram,
                    hipStream_t s, int lds) {
  if (ntasks <= 0) return;
  if constexpr (sizeof(T) == 4) {
    if (gram) {
      launch_augment_t<T, double, true>(tasks, ntasks, r, err, maxn, s, lds);
      return;
    }
  }
  launch_augment_t<T, T, false>(tasks, ntasks, r, err, maxn, s, lds);
}

// ---------------------------------------------------------------------------
// LU with partial pivoting of the redundant block D_RR, one workgroup each.
// ---------------------------------------------------------------------------
template <class T>
__global__ __launch_bounds__(256) void k_lu(const LUTask<T>* __restrict__ tasks,
                                            const int32_t* __restrict__ dyn, int* err,
                                            int lds_elems) {
  extern __shared__ char lu_smem[];
  const LUTask<T> tk = tasks[blockIdx.x];
  const int r = dyn[tk.ri];
  T* A = tk.A;
  const int64_t ld = tk.lda;
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int wave = tid >> 6, lane = tid & 63;
  __shared__ T wv[4];
  __shared__ int wi[4];
  __shared__ int sh_p;
  if ((int64_t)r * r <= lds_elems) {
    // the r x r block in LDS (ld r); wave 0 takes the pivot, the row swap and
    // the column scaling, all waves the trailing update: two barriers a column
    T* S = reinterpret_cast<T*>(lu_smem);
    for (int e = tid; e < r * r; e += nthr) S[e] = A[(e % r) + (int64_t)(e / r) * ld];
    __syncthreads();
    for (int j = 0; j < r; ++j) {
      if (wave == 0) {
        T best = -1;
        int bi = j;
        for (int i = j + lane; i < r; i += 64) {
          const T v = fabs(S[i + j * r]);
          if (v > best) {
            best = v;
            bi = i;
          }
        }
        for (int o = 32; o > 0; o >>= 1) {
          const T ov = __shfl_xor(best, o, 64);
          const int oi = __shfl_xor(bi, o, 64);
          if (ov > best || (ov == best && oi < bi)) {
            best = ov;
            bi = oi;
          }
        }
        const int p = bi;
        if (lane == 0) {
          tk.piv[j] = p;
          if (!(best > T(0))) atomicOr(err, 1);
        }
        if (p != j)
          for (int c = lane; c < r; c += 64) {
            const T x = S[j + c * r];
            S[j + c * r] = S[p + c * r];
            S[p + c * r] = x;
          }
        // the swap and the scaling touch different rows except through the
        // pivot S[j][j], read after the swap by every lane (same wave)
        const T d = S[j + j * r];
        const T inv = d != T(0) ? T(1) / d : T(0);
        for (int i = j + 1 + lane; i < r; i += 64) S[i + j * r] *= inv;
      }
      __syncthreads();
      const int m = r - j - 1;
      for (int e = tid; e < m * m; e += nthr) {
        const int i = j + 1 + e % m, c = j + 1 + e / m;
        S[i + c * r] -= S[i + j * r] * S[j + c * r];
      }
      __syncthreads();
    }
    for (int e = tid; e < r * r; e += nthr) A[(e % r) + (int64_t)(e / r) * ld] = S[e];
    return;
  }
  for (int j = 0; j < r; ++j) {
    T best = -1;
    int bi = j;
    for (int i = j + tid; i < r; i += nthr) {
      const T v = fabs(A[i + (int64_t)j * ld]);
      if (v > best) {
        best = v;
        bi = i;
      }
    }
    for (int o = 32; o > 0; o >>= 1) {
      const T ov = __shfl_xor(best, o, 64);
      const int oi = __shfl_xor(bi, o, 64);
      if (ov > best || (ov == best && oi < bi)) {
        best = ov;
        bi = oi;
      }
    }
    if (lane == 0) {
      wv[wave] = best;
      wi[wave] = bi;
    }
    __syncthreads();
    if (tid == 0) {
      T b = wv[0];
      int p = wi[0];
      for (int w = 1; w < 4; ++w)
        if (wv[w] > b || (wv[w] == b && wi[w] < p)) {
          b = wv[w];
          p = wi[w];
        }
      sh_p = p;
      tk.piv[j] = p;
      if (!(b > T(0))) atomicOr(err, 1);
    }
    __syncthreads();
    const int p = sh_p;
    if (p != j)
      for (int c = tid; c < r; c += nthr) {
        const T x = A[j + (int64_t)c * ld];
        A[j + (int64_t)c * ld] = A[p + (int64_t)c * ld];
        A[p + (int64_t)c * ld] = x;
      }
    __syncthreads();
    const T d = A[j + (int64_t)j * ld];
    const T inv = d != T(0) ? T(1) / d : T(0);
    for (int i = j + 1 + tid; i < r; i += nthr) A[i + (int64_t)j * ld] *= inv;
    __syncthreads();
    const int m = r - j - 1;
    for (int e = tid; e < m * m; e += nthr) {
      const int i = j + 1 + e % m, c = j + 1 + e / m;
      A[i + (int64_t)c * ld] -= A[i + (int64_t)j * ld] * A[j + (int64_t)c * ld];
    }
    __syncthreads();
  }
}

template <class T>
void launch_lu(const LUTask<T>* tasks, int ntasks, const int32_t* dyn, int* err, int maxr,
               hipStream_t s, int lds) {
  if (ntasks <= 0) return;
  // blocks of order <= maxr factor in LDS when maxr^2 fits, else in place
  const int64_t cap = std::min(lds, kLdsBytes) / (int64_t)sizeof(T);
  const int64_t need = (int64_t)maxr * maxr <= cap ? (int64_t)maxr * maxr : 0;
  static bool attr_set = false;
  if (!attr_set) {
    (void)hipFuncSetAttribute((const void*)k_lu<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              kLdsBytes);
    attr_set = true;
  }
  hipLaunchKernelGGL(k_lu<T>, dim3(ntasks), dim3(256), (size_t)(need * sizeof(T)), s, tasks, dyn,
                     err, (int)need);
}

// ---------------------------------------------------------------------------
// B[0:r, c0:ncols] <- U^{-1} L^{-1} P B with the pivoted LU of the leading
// r x r block (Algorithm 2, the multipliers of the partial LU; Algorithm 3,
// the solves with D_RR).  Workgroup = (task, tile of tc columns): the row-
// permuted tile sits in LDS and every step of the two column-oriented
// substitutions updates rows x columns of the tile in parallel with one
// barrier; row j of the result is final after backward step j and goes
// straight to global memory.
// ---------------------------------------------------------------------------
template <class T>
__global__ __launch_bounds__(256) void k_trsm(const TrsmTask<T>* __restrict__ tasks,
                                              const int32_t* __restrict__ dyn, int tc) {
  extern __shared__ char trsm_smem[];
  const TrsmTask<T> tk = tasks[blockIdx.x];
  const int r = tk.ri >= 0 ? dyn[tk.ri] : tk.rs;
  if (r == 0) return;
  const int c0 = tk.c0d >= 0 ? dyn[tk.c0d] : tk.c0s;
  int ldx = 0;
  T* const xc = tk.Bc ? xmul_at<T>(tk.Bc, r, (int)tk.ldb, tk.ncols, ldx) : nullptr;
  const int cb = c0 + (int)blockIdx.y * tc;
  if (cb >= tk.ncols) return;
  const int ncol = min(tc, tk.ncols - cb);
  T* Bs = reinterpret_cast<T*>(trsm_smem);  // r x ncol, ld r
  int* perm = reinterpret_cast<int*>(Bs + (int64_t)r * tc);
  int* pv = perm + r;  // the pivots, staged
  const T* LU = tk.LU;
  const int64_t ld = tk.ldlu;
  const int tid = threadIdx.x, nthr = blockDim.x;
  for (int j = tid; j < r; j += nthr) {
    pv[j] = tk.piv[j];
    perm[j] = j;
  }
  __syncthreads();
  if (tid == 0)
    for (int j = 0; j < r; ++j) {
      const int p = pv[j];
      const int x = perm[j];
      perm[j] = perm[p];
      perm[p] = x;
    }
  __syncthreads();
  T* B = tk.B + (int64_t)cb * tk.ldb;
  for (int e = tid; e < r * ncol; e += nthr) {
    const int i = e % r, c = e / r;
    Bs[e] = B[perm[i] + (int64_t)c * tk.ldb];
  }
  __syncthreads();
  // thread = (row lane, column): rows rl, rl + RL, ...
  const int RL = nthr / ncol;
  const int rl = tid % RL, col = tid / RL;
  const bool act = col < ncol;
  T* bc = Bs + (int64_t)col * r;
  for (int j = 0; j + 1 < r; ++j) {
    if (act) {
      const T bj = bc[j];
      if (bj != T(0))
        for (int i = j + 1 + rl; i < r; i += RL) bc[i] -= LU[i + (int64_t)j * ld] * bj;
    }
    __syncthreads();
  }
  T* Bg = B + (int64_t)col * tk.ldb;
  for (int j = r - 1; j >= 0; --j) {
    if (act) {
      const T xj = bc[j] / LU[j + (int64_t)j * ld];
      if (xj != T(0))
        for (int i = rl; i < j; i += RL) bc[i] -= LU[i + (int64_t)j * ld] * xj;
      if (rl == j % RL) {
        Bg[j] = xj;
        if (xc) xc[j + (int64_t)(cb + col) * ldx] = xj;
      }
    }
    __syncthreads();
  }
}

// Narrow right-hand sides (the solves): one workgroup per task with the r x r
// factor in LDS; each wave solves whole columns held in registers (row
// lane + 64 u in x[u], r <= 256), pivot values broadcast by lane shuffles.
template <class T>
__global__ __launch_bounds__(256) void k_trsm_wave(const TrsmTask<T>* __restrict__ tasks,
                                                   const int32_t* __restrict__ dyn) {
  extern __shared__ char trw_smem[];
  const TrsmTask<T> tk = tasks[blockIdx.x];
  const int r = tk.ri >= 0 ? dyn[tk.ri] : tk.rs;
  if (r == 0) return;
  const int c0 = tk.c0d >= 0 ? dyn[tk.c0d] : tk.c0s;
  int ldx = 0;
  T* const xc = tk.Bc ? xmul_at<T>(tk.Bc, r, (int)tk.ldb, tk.ncols, ldx) : nullptr;
  T* S = reinterpret_cast<T*>(trw_smem);  // r x r, ld r
  int* perm = reinterpret_cast<int*>(S + (int64_t)r * r);
  int* pv = perm + r;  // the pivots, staged
  const int tid = threadIdx.x, nthr = blockDim.x;
  for (int e = tid; e < r * r; e += nthr) S[e] = tk.LU[(e % r) + (int64_t)(e / r) * tk.ldlu];
  for (int j = tid; j < r; j += nthr) {
    pv[j] = tk.piv[j];
    perm[j] = j;
  }
  __syncthreads();
  if (tid == 0)
    for (int j = 0; j < r; ++j) {
      const int p = pv[j];
      const int x = perm[j];
      perm[j] = perm[p];
      perm[p] = x;
    }
  __syncthreads();
  const int wave = tid >> 6, lane = tid & 63;
  const int nu = (r + 63) >> 6;
  // every wave carries CB right-hand side columns through one sweep: each
  // factor entry read from LDS serves all of them, and the substitution chain
  // is walked once per CB columns
  constexpr int CB = 8;
  for (int col0 = c0 + wave * CB; col0 < tk.ncols; col0 += 4 * CB) {
    const int ncb = min(CB, tk.ncols - col0);
    T* b = tk.B + (int64_t)col0 * tk.ldb;
    T x[4][CB];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int i = lane + 64 * u;
#pragma unroll
      for (int c = 0; c < CB; ++c) x[u][c] = (i < r && c < ncb) ? b[perm[i] + (int64_t)c * tk.ldb] : T(0);
    }
    // L y = P b (unit lower)
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (u >= nu) break;
      const int jn = min(64, r - 64 * u);
      for (int jj = 0; jj < jn; ++jj) {
        const int j = 64 * u + jj;
        T bj[CB];
#pragma unroll
        for (int c = 0; c < CB; ++c) bj[c] = __shfl(x[u][c], jj, 64);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = lane + 64 * v;
          if (v >= u && i > j && i < r) {
            const T l = S[i + j * r];
#pragma unroll
            for (int c = 0; c < CB; ++c) x[v][c] -= l * bj[c];
          }
        }
      }
    }
    // U x = y
#pragma unroll
    for (int u = 3; u >= 0; --u) {
      if (u >= nu) continue;
      const int jn = min(64, r - 64 * u);
      for (int jj = jn - 1; jj >= 0; --jj) {
        const int j = 64 * u + jj;
        const T d = S[j + j * r];
        T xj[CB];
#pragma unroll
        for (int c = 0; c < CB; ++c) {
          xj[c] = __shfl(x[u][c], jj, 64) / d;
          if (lane == jj) x[u][c] = xj[c];
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = lane + 64 * v;
          if (v <= u && i < j) {
            const T uu = S[i + j * r];
#pragma unroll
            for (int c = 0; c < CB; ++c) x[v][c] -= uu * xj[c];
          }
        }
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int i = lane + 64 * u;
      if (i < r)
#pragma unroll
        for (int c = 0; c < CB; ++c)
          if (c < ncb) {
            b[i + (int64_t)c * tk.ldb] = x[u][c];
            if (xc) xc[i + (int64_t)(col0 + c) * ldx] = x[u][c];
          }
    }
  }
}

template <class T>
void launch_trsm(const TrsmTask<T>* tasks, int ntasks, const int32_t* dyn, int maxr, int maxcols,
                 hipStream_t s, int lds) {
  if (ntasks <= 0 || maxr <= 0 || maxcols <= 0) return;
  lds = std::min(lds, kLdsBytes);
  const size_t wlds = (size_t)maxr * maxr * sizeof(T) + 2 * (size_t)maxr * sizeof(int);
  if (maxcols <= 64 && maxr <= 256 && wlds <= (size_t)lds) {
    static bool wattr = false;
    if (!wattr) {
      (void)hipFuncSetAttribute((const void*)k_trsm_wave<T>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBytes);
      wattr = true;
    }
    hipLaunchKernelGGL(k_trsm_wave<T>, dim3(ntasks), dim3(256), wlds, s, tasks, dyn);
    return;
  }
  int tc = 32;
  const int64_t tile_cap = std::min(96 * 1024, lds);
  while (tc > 1 && (int64_t)maxr * tc * (int64_t)sizeof(T) > tile_cap) tc >>= 1;
  tc = std::min(tc, maxcols);
  const size_t tlds = (size_t)maxr * tc * sizeof(T) + 2 * (size_t)maxr * sizeof(int);
  static bool attr_set = false;
  if (!attr_set) {
    (void)hipFuncSetAttribute((const void*)k_trsm<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              kLdsBytes);
    attr_set = true;
  }
  const int tiles = (maxcols + tc - 1) / tc;
  hipLaunchKernelGGL(k_trsm<T>, dim3(ntasks, tiles), dim3(256), tlds, s, tasks, dyn, tc);
}

// ---------------------------------------------------------------------------
// Block copies / accumulations with type conversion.
// ---------------------------------------------------------------------------
template <class T, class S>
__global__ __launch_bounds__(256) void k_copy(const CTask<T, S>* __restrict__ tasks, int ntasks) {
  const int64_t tile = blockIdx.x;
  int lo = 0, hi = ntasks - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (tasks[mid].tile0 <= tile) lo = mid; else hi = mid - 1;
  }
  const CTask<T, S>& tk = tasks[lo];
  const int64_t base = (tile - tk.tile0) * kCopyTile;
  const int64_t tot = (int64_t)tk.rows * tk.cols;
  // a transposed source is read along its columns (element e runs down a
  // destination row) so that both sides of the copy stay coalesced enough
  for (int64_t e = base + threadIdx.x; e < min(base + kCopyTile, tot); e += blockDim.x) {
    int64_t r, c;
    if (tk.tr) {
      c = e % tk.cols;
      r = e / tk.cols;
    } else {
      r = e % tk.rows;
      c = e / tk.rows;
    }
    const T v = (T)(tk.tr ? tk.src[c + r * tk.lds] : tk.src[r + c * tk.lds]);
    T* d = tk.dst + r + c * tk.ldd;
    *d = tk.add ? *d + v : v;
  }
}

template <class T, class S>
void launch_copy(const CTask<T, S>* tasks, int ntasks, int64_t ntiles, hipStream_t s) {
  if (ntasks <= 0 || ntiles <= 0) return;
  hipLaunchKernelGGL((k_copy<T, S>), dim3((unsigned)ntiles), dim3(256), 0, s, tasks, ntasks);
}

// ---------------------------------------------------------------------------
// Level close-out (CloseLevel): one wave per pattern entry (pass 0) or per far
// entry / cluster (pass 1).
// ---------------------------------------------------------------------------
// row of entry e in a CSR row pointer of n rows (largest j with ptr[j] <= e)
__device__ inline int csr_row(const int64_t* ptr, int n, int64_t e) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (ptr[mid] <= e) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// entry (t, s) of a sorted CSR pattern, or -1
__device__ inline int64_t csr_find(const int64_t* ptr, const int32_t* col, int t, int s) {
  int64_t a = ptr[t], b = ptr[t + 1];
  const int64_t end = b;
  while (a < b) {
    const int64_t m = (a + b) >> 1;
    if (col[m] < s) a = m + 1; else b = m;
  }
  return (a < end && col[a] == s) ? a : -1;
}

// dst (ldd) = or += the rows x cols block of src (lds), read transposed when
// srcT (element (r, c) at src[c + r lds]); one wave, the source read along
// its contiguous dimension
template <class T>
__device__ inline void wave_block_copy(const T* src, int64_t lds, bool srcT, T* dst, int64_t ldd,
                                       int rows, int cols, bool add, int lane) {
  const gptr<const T> sg = gmem(src);
  const gptr<T> dg = gmem(dst);
  const int tot = rows * cols;
  for (int e = lane; e < tot; e += 64) {
    int r, c;
    if (srcT) {
      c = e % cols;
      r = e / cols;
    } else {
      r = e % rows;
      c = e / rows;
    }
    const T v = srcT ? sg[c + (int64_t)r * lds] : sg[r + (int64_t)c * lds];
    const gptr<T> d = dg + r + (int64_t)c * ldd;
    *d = add ? *d + v : v;
  }
}

// destination block of parents (pt, ps) and its leading dimension; false
// when the block is written through its mirror (or is missing: err bit 3)
template <class T>
__device__ inline bool close_dest(const CloseLevel<T>& L, int pt, int ps, bool far, T*& d,
                                  int64_t& ld, int* err) {
  if (L.top) {
    ld = L.ldtop;
    d = L.M + L.top_off[pt] + L.top_off[ps] * ld;
    return true;
  }
  const int64_t en = csr_find(L.npptr, L.npcol, pt, ps);
  const int nk = en >= 0 ? L.nkind[en] : -1;
  if (en < 0 || (far && nk != 0)) {
    atomicOr(err, 8);
    return false;
  }
  if (nk == 2) return false;
  ld = L.nn[pt];
  d = (nk == 1 ? L.Fn : L.Dn) + L.npoff[en];
  return true;
}

template <class T>
__global__ __launch_bounds__(256) void k_closeout(CloseLevel<T> L, int pass, int* err) {
  const int lane = threadIdx.x & 63;
  const int64_t w0 = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int64_t nw = (int64_t)gridDim.x * 4;
  if (pass == 0) {
    for (int64_t e = w0; e < L.nnz; e += nw) {
      const int j = csr_row(L.pptr, L.nl, e);
      const int k = L.pcol[e];
      const int nj = L.n[j], nk = L.n[k], rj = L.r[j], rk = L.r[k];
      const int kj = nj - rj, kk = nk - rk;
      if (kj <= 0 || kk <= 0) continue;
      T* d;
      int64_t ld;
      if (!close_dest(L, L.par[j], L.par[k], false, d, ld, err)) continue;
      d += L.offc[j] + (int64_t)L.offc[k] * ld;
      const int kd = L.kind[e];
      if (kd == 2)
        wave_block_copy(L.F + L.poff[e] + rk + (int64_t)rj * nk, nk, true, d, ld, kj, kk, true,
                        lane);
      else
        wave_block_copy((kd == 1 ? L.F : L.D) + L.poff[e] + rj + (int64_t)rk * nj, nj, false, d,
                        ld, kj, kk, kd == 1, lane);
    }
    return;
  }
  const int64_t nq = L.nfar + (L.top ? 0 : L.nl);
  for (int64_t q = w0; q < nq; q += nw) {
    if (q < L.nfar) {
      const int64_t e = L.far0 + q;
      const int j = csr_row(L.far_ptr + L.a, L.nl, e);
      const int gj = L.a + j, gk = L.far_col[e];
      T* d;
      int64_t ld;
      if (!close_dest(L, L.par[j], L.par[gk - L.a], true, d, ld, err)) continue;
      d += L.offc[j] + (int64_t)L.offc[gk - L.a] * ld;
      wave_block_copy(L.data + L.offS[e], L.rank[gj], false, d, ld, L.rank[gj], L.rank[gk], true,
                      lane);
    } else {
      const int j = (int)(q - L.nfar), gj = L.a + j;
      const int pt = L.par[j];
      wave_block_copy(L.data + L.offE[gj], L.rank[gj], false, L.Vn + L.noffV[pt] + L.offc[j],
                      L.nn[pt], L.rank[gj], L.rank[L.pa + pt], false, lane);
    }
  }
}

template <class T> void launch_closeout(const CloseLevel<T>& cl, int pass, int* err, hipStream_t s) {
  const int64_t nq = pass == 0 ? cl.nnz : cl.nfar + (cl.top ? 0 : cl.nl);
  if (nq <= 0) return;
  const int64_t blocks = std::min<int64_t>((nq + 3) / 4, 16384);
  hipLaunchKernelGGL(k_closeout<T>, dim3((unsigned)blocks), dim3(256), 0, s, cl, pass, err);
}

template <class T> __global__ void k_fill(T* p, int64_t n, T v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}
template <class T> void launch_fill(T* p, int64_t n, T v, hipStream_t s) {
  if (n <= 0) return;
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 65536);
  hipLaunchKernelGGL(k_fill<T>, dim3((unsigned)blocks), dim3(256), 0, s, p, n, v);
}

template <class T, class S>
__global__ void k_gather(T* dst, int64_t ldd, const S* src, int64_t lds, const int64_t* perm,
                         int64_t n, int nrhs) {
  const int64_t tot = n * nrhs;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t p = e % n, c = e / n;
    dst[p + c * ldd] = (T)src[perm[p] + c * lds];
  }
}
template <class T, class S>
__global__ void k_scatter(T* dst, int64_t ldd, const S* src, int64_t lds, const int64_t* perm,
                          int64_t n, int nrhs) {
  const int64_t tot = n * nrhs;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t p = e % n, c = e / n;
    dst[perm[p] + c * ldd] = (T)src[p + c * lds];
  }
}
template <class T, class S>
void launch_gather_rows(T* dst, int64_t ldd, const S* src, int64_t lds, const int64_t* perm,
                        int64_t n, int nrhs, hipStream_t s) {
  const int64_t blocks = std::min<int64_t>((n * nrhs + 255) / 256, 65536);
  if (blocks <= 0) return;
  hipLaunchKernelGGL((k_gather<T, S>), dim3((unsigned)blocks), dim3(256), 0, s, dst, ldd, src,
                     lds, perm, n, nrhs);
}
template <class T, class S>
void launch_scatter_rows(T* dst, int64_t ldd, const S* src, int64_t lds, const int64_t* perm,
                         int64_t n, int nrhs, hipStream_t s) {
  const int64_t blocks = std::min<int64_t>((n * nrhs + 255) / 256, 65536);
  if (blocks <= 0) return;
  hipLaunchKernelGGL((k_scatter<T, S>), dim3((unsigned)blocks), dim3(256), 0, s, dst, ldd, src,
                     lds, perm, n, nrhs);
}

template <class T> __global__ void k_convert(T* dst, const double* src, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = (T)src[i];
}
template <class T> void launch_convert(T* dst, const double* src, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 65536);
  hipLaunchKernelGGL(k_convert<T>, dim3((unsigned)blocks), dim3(256), 0, s, dst, src, n);
}

// ---------------------------------------------------------------------------
// Dense top-level LU (blocked right-looking, partial pivoting).
// ---------------------------------------------------------------------------
template <class T>
__global__ __launch_bounds__(256) void k_panel_lu(T* A, int64_t lda, int64_t n, int64_t j0,
                                                  int nb, int32_t* piv, int* err) {
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int wave = tid >> 6, lane = tid & 63;
  __shared__ T wv[4];
  __shared__ int64_t wi[4];
  __shared__ int64_t sh_p;
  for (int jj = 0; jj < nb; ++jj) {
    const int64_t j = j0 + jj;
    T best = -1;
    int64_t bi = j;
    for (int64_t i = j + tid; i < n; i += nthr) {
      const T v = fabs(A[i + j * lda]);
      if (v > best) {
        best = v;
        bi = i;
      }
    }
    for (int o = 32; o > 0; o >>= 1) {
      const T ov = __shfl_xor(best, o, 64);
      const int64_t oi = __shfl_xor(bi, o, 64);
      if (ov > best || (ov == best && oi < bi)) {
        best = ov;
        bi = oi;
      }
    }
    if (lane == 0) {
      wv[wave] = best;
      wi[wave] = bi;
    }
    __syncthreads();
    if (tid == 0) {
      T b = wv[0];
      int64_t p = wi[0];
      for (int w = 1; w < 4; ++w)
        if (wv[w] > b || (wv[w] == b && wi[w] < p)) {
          b = wv[w];
          p = wi[w];
        }
      sh_p = p;
      piv[j] = (int32_t)p;
      if (!(b > T(0))) atomicOr(err, 1);
    }
    __syncthreads();
    const int64_t p = sh_p;
    if (p != j)
      for (int c = tid; c < nb; c += nthr) {
        const int64_t cc = j0 + c;
        const T x = A[j + cc * lda];
        A[j + cc * lda] = A[p + cc * lda];
        A[p + cc * lda] = x;
      }
    __syncthreads();
    const T d = A[j + j * lda];
    const T inv = d != T(0) ? T(1) / d : T(0);
    for (int64_t i = j + 1 + tid; i < n; i += nthr) A[i + j * lda] *= inv;
    __syncthreads();
    // update the remaining panel columns
    for (int c = jj + 1 + wave; c < nb; c += 4) {
      const int64_t cc = j0 + c;
      const T u = A[j + cc * lda];
      for (int64_t i = j + 1 + lane; i < n; i += 64) A[i + cc * lda] -= A[i + j * lda] * u;
    }
    __syncthreads();
  }
}
template <class T>
void launch_panel_lu(T* A, int64_t lda, int64_t n, int64_t j0, int nb, int32_t* piv, int* err,
                     hipStream_t s) {
  hipLaunchKernelGGL(k_panel_lu<T>, dim3(1), dim3(256), 0, s, A, lda, n, j0, nb, piv, err);
}

// apply the row interchanges of rows j0..j0+nb-1 to all columns outside [skip0, skip1)
template <class T>
__global__ void k_laswp(T* A, int64_t lda, int64_t ncols, int64_t j0, int nb, const int32_t* piv,
                        int64_t skip0, int64_t skip1) {
  for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < ncols;
       c += (int64_t)gridDim.x * blockDim.x) {
    if (c >= skip0 && c < skip1) continue;
    for (int jj = 0; jj < nb; ++jj) {
      const int64_t j = j0 + jj, p = piv[j];
      if (p != j) {
        const T x = A[j + c * lda];
        A[j + c * lda] = A[p + c * lda];
        A[p + c * lda] = x;
      }
    }
  }
}
template <class T>
void launch_laswp(T* A, int64_t lda, int64_t ncols, int64_t j0, int nb, const int32_t* piv,
                  int64_t skip0, int64_t skip1, hipStream_t s) {
  if (ncols <= 0) return;
  const int64_t blocks = std::min<int64_t>((ncols + 255) / 256, 4096);
  hipLaunchKernelGGL(k_laswp<T>, dim3((unsigned)blocks), dim3(256), 0, s, A, lda, ncols, j0, nb,
                     piv, skip0, skip1);
}

// triangular solve with an nb x nb diagonal block for ncols right-hand sides:
// unit lower (lower_unit = 1) or upper with diagonal (lower_unit = 0)
// Triangular solve with a diagonal block of order nb <= 64 (the dense top
// solve and the top factorization's panels): the block is staged in LDS and
// each wave solves one column, held one row per lane, with the pivot value
// broadcast by a lane shuffle.
template <class T>
__global__ __launch_bounds__(256) void k_trsm_block(const T* A, int64_t lda, T* B, int64_t ldb,
                                                    int nb, int64_t ncols, int lower_unit) {
  __shared__ T S[64 * 64];
  for (int e = threadIdx.x; e < nb * nb; e += blockDim.x)
    S[e] = A[(e % nb) + (int64_t)(e / nb) * lda];
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int64_t c = (int64_t)blockIdx.x * 4 + wave; c < ncols; c += (int64_t)gridDim.x * 4) {
    T* b = B + c * ldb;
    T x = lane < nb ? b[lane] : T(0);
    if (lower_unit) {
      for (int j = 0; j < nb; ++j) {
        const T bj = __shfl(x, j, 64);
        if (lane > j && lane < nb) x -= S[lane + j * nb] * bj;
      }
    } else {
      for (int j = nb - 1; j >= 0; --j) {
        const T xj = __shfl(x, j, 64) / S[j + j * nb];
        if (lane == j) x = xj;
        else if (lane < j) x -= S[lane + j * nb] * xj;
      }
    }
    if (lane < nb) b[lane] = x;
  }
}
template <class T>
void launch_trsm_block(const T* A, int64_t lda, T* B, int64_t ldb, int nb, int64_t ncols,
                       int lower_unit, hipStream_t s) {
  if (ncols <= 0 || nb <= 0) return;
  const int64_t blocks = std::min<int64_t>((ncols + 3) / 4, 8192);
  hipLaunchKernelGGL(k_trsm_block<T>, dim3((unsigned)blocks), dim3(256), 0, s, A, lda, B, ldb, nb,
                     ncols, lower_unit);
}

// ---------------------------------------------------------------------------
// FP64 column reductions and updates for the refinement loop.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_colnorms(const double* X, int64_t ldx, int64_t n,
                                                  double* out) {
  __shared__ double red[8];
  const double* x = X + blockIdx.x * ldx;
  double s = 0;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) s += x[i] * x[i];
  s = block_sum(s, red);
  if (threadIdx.x == 0) out[blockIdx.x] = sqrt(s);
}
void launch_colnorms(const double* X, int64_t ldx, int64_t n, int nrhs, double* out,
                     hipStream_t s) {
  hipLaunchKernelGGL(k_colnorms, dim3(nrhs), dim3(256), 0, s, X, ldx, n, out);
}

// out[v + c*nvec] = <V_v[:, c], W[:, c]>, V_v = V + v*vstride
__global__ __launch_bounds__(256) void k_dots(const double* V, int64_t ldv, int64_t vstride,
                                              int nvec, const double* W, int64_t ldw, int64_t n,
                                              double* out) {
  __shared__ double red[8];
  const int v = blockIdx.x % nvec, c = blockIdx.x / nvec;
  const double* a = V + v * vstride + c * ldv;
  const double* b = W + c * ldw;
  double s = 0;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) s += a[i] * b[i];
  s = block_sum(s, red);
  if (threadIdx.x == 0) out[v + (int64_t)c * nvec] = s;
}
void launch_dots(const double* V, int64_t ldv, int64_t vstride, int nvec, const double* W,
                 int64_t ldw, int64_t n, int nrhs, double* out, hipStream_t s) {
  if (nvec <= 0) return;
  hipLaunchKernelGGL(k_dots, dim3(nvec * nrhs), dim3(256), 0, s, V, ldv, vstride, nvec, W, ldw, n,
                     out);
}

// W[:, c] += sign * sum_v coef[v + c*nvec] V_v[:, c]
__global__ void k_update(double* W, int64_t ldw, const double* V, int64_t ldv, int64_t vstride,
                         int nvec, const double* coef, double sign, int64_t n, int nrhs) {
  const int64_t tot = n * nrhs;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e % n, c = e / n;
    double s = 0;
    for (int v = 0; v < nvec; ++v) s += coef[v + c * nvec] * V[v * vstride + i + c * ldv];
    W[i + c * ldw] += sign * s;
  }
}
void launch_update(double* W, int64_t ldw, const double* V, int64_t ldv, int64_t vstride, int nvec,
                   const double* coef, double sign, int64_t n, int nrhs, hipStream_t s) {
  if (nvec <= 0) return;
  const int64_t blocks = std::min<int64_t>((n * nrhs + 255) / 256, 65536);
  hipLaunchKernelGGL(k_update, dim3((unsigned)blocks), dim3(256), 0, s, W, ldw, V, ldv, vstride,
                     nvec, coef, sign, n, nrhs);
}

// dst[:, c] = src[:, c] * (invert ? 1/norms[c] : norms[c]) (zero when dividing by zero)
__global__ void k_scale_cols(double* dst, int64_t ldd, const double* src, int64_t lds,
                             const double* norms, int64_t n, int nrhs, int invert) {
  const int64_t tot = n * nrhs;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e % n, c = e / n;
    const double a = norms[c];
    const double f = invert ? (a != 0 ? 1.0 / a : 0.0) : a;
    dst[i + c * ldd] = src[i + c * lds] * f;
  }
}
void launch_scale_cols(double* dst, int64_t ldd, const double* src, int64_t lds,
                       const double* norms, int64_t n, int nrhs, int invert, hipStream_t s) {
  const int64_t blocks = std::min<int64_t>((n * nrhs + 255) / 256, 65536);
  hipLaunchKernelGGL(k_scale_cols, dim3((unsigned)blocks), dim3(256), 0, s, dst, ldd, src, lds,
                     norms, n, nrhs, invert);
}

__global__ void k_axpy_cols(double* Y, int64_t ldy, const double* X, int64_t ldx, const double* a,
                            int64_t n, int nrhs) {
  const int64_t tot = n * nrhs;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e % n, c = e / n;
    Y[i + c * ldy] += (a ? a[c] : 1.0) * X[i + c * ldx];
  }
}
void launch_axpy_cols(double* Y, int64_t ldy, const double* X, int64_t ldx, const double* a,
                      int64_t n, int nrhs, hipStream_t s) {
  const int64_t blocks = std::min<int64_t>((n * nrhs + 255) / 256, 65536);
  hipLaunchKernelGGL(k_axpy_cols, dim3((unsigned)blocks), dim3(256), 0, s, Y, ldy, X, ldx, a, n,
                     nrhs);
}

__global__ void k_sub(double* R, int64_t ldr, const double* B, int64_t ldb, const double* AX,
                      int64_t ldax, int64_t n, int nrhs) {
  const int64_t tot = n * nrhs;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e % n, c = e / n;
    R[i + c * ldr] = B[i + c * ldb] - AX[i + c * ldax];
  }
}
void launch_sub(double* R, int64_t ldr, const double* B, int64_t ldb, const double* AX,
                int64_t ldax, int64_t n, int nrhs, hipStream_t s) {
  const int64_t blocks = std::min<int64_t>((n * nrhs + 255) / 256, 65536);
  hipLaunchKernelGGL(k_sub, dim3((unsigned)blocks), dim3(256), 0, s, R, ldr, B, ldb, AX, ldax, n,
                     nrhs);
}

__global__ void k_check_finite(const double* X, int64_t n, int* flag) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double v = X[i];
    if (!(v - v == 0.0)) atomicOr(flag, 1);
  }
}
void launch_check_finite(const double* X, int64_t n, int* flag, hipStream_t s) {
  if (n <= 0) return;
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 65536);
  hipLaunchKernelGGL(k_check_finite, dim3((unsigned)blocks), dim3(256), 0, s, X, n, flag);
}

// ---- explicit instantiations ----
#define H2K_INST(T)                                                                           \
  template void launch_gemm<T>(const GOut<T>*, int, const GCon<T>*, const int32_t*, int64_t,  \
                               int, hipStream_t, T*);                                         \
  template void launch_gemm_reduce<T>(const GOut<T>*, int, const T*, int64_t, int,             \
                                      hipStream_t);                                           \
  template void launch_strip<T>(const STask<T>*, int, const int32_t*, int64_t, int,           \
                                hipStream_t, int);                                            \
  template void launch_schur<T>(const SchurLevel<T>*, int, int64_t, int, SchurRow*,           \
                                SchurTarget*, int64_t*, int64_t*, int64_t, int*, hipStream_t); \
  template void launch_rfactor<T>(const RTask<T>*, int, const FillRef<T>*, const int32_t*, int, \
                                  hipStream_t, int);                                          \
  template void launch_pchol<T>(const CholTask<T>*, int, int, hipStream_t);                  \
  template void launch_gram<T>(const GramTask<T>*, int, const FillRef<T>*, const int32_t*,    \
                               int64_t, hipStream_t);                                         \
  template void launch_augment<T>(const AugTask<T>*, int, int32_t*, int*, int, bool,          \
                                  hipStream_t, int);                                          \
  template void launch_lu<T>(const LUTask<T>*, int, const int32_t*, int*, int, hipStream_t,   \
                             int);                                                            \
  template void launch_trsm<T>(const TrsmTask<T>*, int, const int32_t*, int, int, hipStream_t, \
                               int);                                                          \
  template void launch_copy<T, double>(const CTask<T, double>*, int, int64_t, hipStream_t);   \
  template void launch_copy<T, float>(const CTask<T, float>*, int, int64_t, hipStream_t);     \
  template void launch_fill<T>(T*, int64_t, T, hipStream_t);                                  \
  template void launch_closeout<T>(const CloseLevel<T>&, int, int*, hipStream_t);            \
  template void launch_gather_rows<T, double>(T*, int64_t, const double*, int64_t,            \
                                              const int64_t*, int64_t, int, hipStream_t);     \
  template void launch_scatter_rows<double, T>(double*, int64_t, const T*, int64_t,           \
                                               const int64_t*, int64_t, int, hipStream_t);    \
  template void launch_panel_lu<T>(T*, int64_t, int64_t, int64_t, int, int32_t*, int*,        \
                                   hipStream_t);                                              \
  template void launch_laswp<T>(T*, int64_t, int64_t, int64_t, int, const int32_t*, int64_t,  \
                                int64_t, hipStream_t);                                        \
  template void launch_trsm_block<T>(const T*, int64_t, T*, int64_t, int, int64_t, int,       \
                                     hipStream_t);                                            \
  template void launch_convert<T>(T*, const double*, int64_t, hipStream_t);

H2K_INST(double)
H2K_INST(float)
template void launch_fill<int32_t>(int32_t*, int64_t, int32_t, hipStream_t);

}  // namespace h2k
