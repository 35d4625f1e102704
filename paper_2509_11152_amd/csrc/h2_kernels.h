// Device task descriptors and kernel launchers of the H^2 factor/solve library.
//
// Every batched operation is a list of small tasks in device memory.  Sizes
// that depend on ranks decided on the device (the redundant count r_i of a
// cluster) are not copied to the host inside a tree level: a descriptor names
// the cluster whose r_i moves a window boundary ("dyn" index into the level's
// r array, -1 = static boundary), and the kernels read it.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace h2k {

// C[rows m0:m1, cols n0:n] = beta * C + alpha * sum_t opA(A_t)[rows, k0:k1] * B_t[k0:k1, cols]
// Column-major everything.  A_t rows and B_t columns use the same indices as
// C's rows and columns; beta = 0 does not read C.
// A boundary is dyn[d] when d >= 0, else the static value.
template <class T> struct GOut {
  T* C;
  int64_t ldc;
  int32_t m, n;         // static row / column end (m is replaced by dyn[m1d] when m1d >= 0)
  int32_t m0d, m0s;     // row start
  int32_t m1d, n0d;     // row end (dynamic), column start (dynamic)
  int32_t n0s;          // column start (static)
  int32_t nsplit;       // skinny kernel: contributor chunks (<= 1: none)
  int32_t cbeg, cend;   // contributor range
  int32_t tm, tn;       // tile counts over the static extent
  int64_t tile0;        // first tile of this output in the launch
  int64_t part0;        // split outputs: first partial tile in the scratch
  int64_t rtile0;       // split outputs: first tile in the reduction launch
  T alpha, beta;
};

template <class T> struct GCon {
  const T* A;
  const T* B;
  int64_t lda, ldb;
  int32_t k;            // static inner end
  int32_t k0d, k0s;     // inner start
  int32_t k1d;          // inner end (dynamic)
  int32_t transA, pad0;
};

// In-place X <- op(Q) X (side 0, X has n rows, columns c0..ext-1 are active)
// or X <- X op(Q) (side 1, X has n columns, rows c0..ext-1 are active).
// op(Q) = Q^T when trans.  One workgroup per strip of 16.
template <class T> struct STask {
  T* X;
  const T* Q;
  int64_t ldx;
  int32_t n;            // order of Q
  int32_t ext;          // static extent of the strip direction
  int32_t d0, s0;       // window start: dyn[d0] or s0
  int32_t side, trans;
  int64_t strip0;       // first strip index in the launch
};

// One column block of the fill row of a cluster: columns c0..ncols-1 of the
// n x ncols block F_ij, c0 = dyn[d0] or 0.  Entry (a, c) is F[a + c ld], or
// F[c + a ld] when `tr` is set (the fill of a symmetric matrix is stored once
// per unordered pair: F_ij is then the transpose of the stored F_ji).
template <class T> struct FillRef {
  const T* F;
  int64_t ld;
  int32_t ncols, d0;
  int32_t tr, pad0;
};
// strides of entry (a, c) of a fill block: a * rs + c * cs
template <class T> __host__ __device__ inline int64_t fr_rs(const FillRef<T>& f) {
  return f.tr ? f.ld : 1;
}
template <class T> __host__ __device__ inline int64_t fr_cs(const FillRef<T>& f) {
  return f.tr ? 1 : f.ld;
}

// One stage of the tall-skinny QR of a fill row Y (Section 2.1, QR-based
// augmentation): the R factor of the rows of Y^T held by a group of fill
// blocks.  It is written as an n x n fill block, out[col + t n] = R[t][col],
// so a later stage can read the factors like fill blocks; later stages merge
// them in pairs (tri).
template <class T> struct RTask {
  T* out;               // n x n, ld n
  T* work;              // (n + kAugChunk) x n, used only when R does not fit in LDS
  int32_t n;
  int32_t fbeg, fend;   // FillRef range
  int32_t tri;          // 1: every block is an n x n factor of a previous stage
                        // (upper triangular in the layout of `out`)
};

// Block pattern of one level of one instance, resident on the device for the
// Schur and fill-in updates (Algorithm 2, partial LU): the level's pattern
// CSR (near and fill entries, rows and columns ascending), each entry's
// element offset in the near (D) or fill (F) buffer and its kind (0 near,
// 1 stored fill block, 2 fill entry stored as the transpose of its mirror),
// and the clusters' colours and orders.  rows0: first global row of the
// instance in a launch over several instances.
// The Schur update reads the multipliers of a near block from a compact copy
// that the triangular solves also write (FP64: its single-element loads touch
// fewer lines there), or in place in D (FP32: its 16-byte loads along k ran
// faster from D than from the copy).
template <class T> constexpr bool kXmulCopy() { return sizeof(T) == 8; }
template <class T> struct SchurLevel {
  const int64_t* pptr;
  const int32_t* pcol;
  const int64_t* poff;
  const int8_t* kind;
  const int32_t* color;
  const int32_t* n;
  const int32_t* r;     // the level's r array (this instance's clusters)
  T* D;
  T* F;
  const T* X;           // kXmulCopy: the multipliers D_RR^{-1} D_{R_i,k} of near entry
                        // (i, k) of the colour being processed, in the n_i x n_k
                        // region at xoff[e] (placed by xmul_at); else unused
  const int64_t* xoff;
  int32_t nl;
  int32_t pad0;
  int64_t rows0;
};
// Close-out of one level into the next level's blocks or the dense top block
// (Section 2.1, level transition), found on the device from the level's
// pattern.  Pass 0: for every pattern entry (j, k) the skeleton part, rows
// [r_j, n_j) x columns [r_k, n_k), of D(j, k) or of the fill (stored, or the
// stored (k, j) read transposed) goes to rows offc[j].., columns offc[k].. of
// the parents' block (p(j), p(k)); a next-level fill entry with p(k) < p(j) is
// written through its stored mirror instead.  Pass 1 (after pass 0): the far
// couplings S_jk are added at the same place (S~ = [S 0; 0 0]) and the
// transfers E_j copied to rows offc[j].. of the parent's next basis.
template <class T> struct CloseLevel {
  // the level being closed (a: its first global cluster, pa: the next level's)
  const int64_t* pptr;
  const int32_t* pcol;
  const int64_t* poff;
  const int8_t* kind;     // 0 near, 1 stored fill, 2 fill read from its mirror
  const int32_t* n;
  const int32_t* r;
  const T* D;
  const T* F;
  const int32_t* par;     // local parent of each cluster
  const int32_t* offc;    // skeleton row offset of each cluster in its parent
  int32_t nl, a, pa, top;
  int64_t nnz;
  // next level (top == 0)
  const int64_t* npptr;
  const int32_t* npcol;
  const int64_t* npoff;
  const int8_t* nkind;
  const int32_t* nn;      // next-level orders
  const int64_t* noffV;   // next-level basis offsets
  T* Dn;
  T* Fn;
  T* Vn;
  // dense top block (top == 1)
  const int64_t* top_off;
  int64_t ldtop;
  T* M;
  // matrix: far lists, couplings, transfers (global cluster ids)
  const int64_t* far_ptr;
  const int32_t* far_col;
  const int64_t* offS;
  const int64_t* offE;
  const int32_t* rank;
  const T* data;
  int64_t far0, nfar;     // far entries of the level's rows
};
constexpr int kSchurMaxContrib = 32;
// one Schur / fill-in target found on the device: global row g (instance row
// offset + j), pattern entry e = (j, k), and its ncont contributions at
// conts[cbeg..]: each (x << 48) | e_ik, x the contributor's slot in row g's
// table, e_ik the entry (i, k) of its multipliers, in ascending x
struct SchurTarget {
  int64_t e;
  int32_t g;
  int32_t ncont;
  int64_t cbeg;
};
constexpr int64_t kContEntryMask = ((int64_t)1 << 48) - 1;
// contributors of one row for the colour being processed: cluster ids and
// their entries (j, i)
struct SchurRow {
  int32_t nc;
  int32_t ci[kSchurMaxContrib];
  int64_t eji[kSchurMaxContrib];
};

// Basis augmentation + complement of one cluster (Algorithm 2, first loop),
// given the R factor of the cluster's fill row.
template <class T> struct AugTask {
  const T* V;           // n x k input basis
  const T* Rt;          // n x n, Rt[b + a n] = R[a][b] (R upper triangular, R^T R = Y Y^T)
  const double* G;      // or n x n FP64 Y Y^T (the FP32 factorization's Gram path)
  T* Q;                 // n x n output Q~ = [V~perp, V~]
  T* work;              // scratch
  int32_t n, k;
  int32_t ri;           // index into the r array (output)
  int32_t rgen;         // Rt holds a general factor (R with permuted columns), not a
                        // triangle, followed by its number of nonzero rows (int32)
  double eps;           // truncation threshold eps_fill = tol ||A||_2 of the task's matrix
};

// Gram matrix of one cluster's fill row (FP32 factorization): G = Y Y^T in
// FP64 over the fill blocks FillRef[fbeg, fend), 64 x 64 tiles.
template <class T> struct GramTask {
  double* G;            // n x n, ld n
  int32_t n;
  int32_t fbeg, fend;
  int32_t tm;           // tiles per dimension
  int64_t tile0;        // first tile of this task in the launch
};

// Factor of a fill row's Gram matrix for the FP32 factorization (the Gram
// option of Section 2.1): G is the sum of nch partial Gram matrices (FP64,
// n x n each, consecutive), factored by Cholesky with diagonal pivoting,
// G = P R^T R P^T, stopped once the largest remaining pivot is at most
// max(1e-6 eps^2, 64 n u maxdiag(G)); Rt receives R P^T (rows past the
// rank zero) as Rt[b + a n] = (R P^T)[a][b], and the rank as an int32 in the
// element after it (Rt holds n^2 + 1 elements).
template <class T> struct CholTask {
  const double* G;
  T* Rt;
  int32_t n, nch;
  double eps;           // eps_fill of the task's matrix
};

// LU with partial pivoting of the leading r x r block of A (r = dyn[ri]).
template <class T> struct LUTask {
  T* A;
  int32_t* piv;
  int64_t lda;
  int32_t ri, pad0;
};

// B[0:r, c0:ncols] <- A_RR^{-1} B[0:r, c0:ncols] with the LU of the leading
// r x r block of A.
template <class T> struct TrsmTask {
  const T* LU;
  const int32_t* piv;
  T* B;
  T* Bc;                // optional: the result again, in a region of ldb x ncols
                        // elements (placed as xmul_at places it)
  int64_t ldlu, ldb;
  int32_t ncols;
  int32_t ri, rs;       // order r: dyn[ri] or rs
  int32_t c0d, c0s;     // first column: dyn[c0d] or c0s
  int32_t pad0;
};

// dst[0:rows, 0:cols] (=|+=) src[0:rows, 0:cols], or the transpose of
// src[0:cols, 0:rows] when `tr` is set; element types may differ.
template <class T, class S> struct CTask {
  const S* src;
  T* dst;
  int64_t lds, ldd;
  int32_t rows, cols;
  int32_t add, tr;
  int64_t tile0;
};

constexpr int kStrip = 16;
constexpr int kCopyTile = 4096;
constexpr int kAugChunk = 64;

constexpr int kLdsBytes = 150 * 1024;  // dynamic LDS a workgroup may request

// Fill-row reduction in LDS, one lane per column: wave w of the workgroup
// owns columns 64 w .. 64 w + 63 and every lane holds rf_chunk<T>() rows of
// its column in registers.  LDS holds R packed upper triangular by rows (row
// j at rf_rowoff(j, n), entries j..n-1) after two reflector buffers.
template <class T> __host__ __device__ constexpr int rf_chunk() { return sizeof(T) == 4 ? 64 : 32; }
__host__ __device__ inline int64_t rf_rowoff(int j, int n) {
  return (int64_t)j * n - (int64_t)j * (j - 1) / 2;
}
// one reflector buffer: the chunk column, its squared norm, R[j][j] (padded
// to 16 bytes)
template <class T> __host__ __device__ constexpr int rf_xstride() {
  return rf_chunk<T>() + (int)(16 / sizeof(T));
}
template <class T> __host__ __device__ inline int64_t rf_lds_elems(int n) {
  return (int64_t)n * (n + 1) / 2 + 2 * (int64_t)rf_xstride<T>();
}
// whether the fill-row reduction of order n runs in LDS (else in `work`)
// with `lds` bytes of LDS per workgroup (kLdsBytes unless a factorization
// asks for less)
template <class T> __host__ __device__ inline bool rf_in_lds(int n, int lds = kLdsBytes) {
  return n <= 256 && rf_lds_elems<T>(n) <= lds / (int64_t)sizeof(T);
}
// largest cluster order the augmentation supports (lanes x registers of a
// Jacobi pair)
constexpr int kMaxAugOrder = 1024;
// rows of Y^T one first-stage group takes (whole fill blocks, at least one)
inline int rf_group_rows(int) { return 256; }
// fill columns per partial Gram matrix (one workgroup tile of G per chunk)
constexpr int kGramChunk = 4096;

// scratch elements of one augmentation task of order n: V_perp (n^2), the
// reflectors of V (n^2), M' or M and W' (2 n^2), G V_perp (n^2), singular
// values, reflector scalars, ranks
inline int64_t aug_work_elems(int n) { return 5 * (int64_t)n * n + 3 * (int64_t)n + 64; }

// ---- launchers (stream-ordered; descriptor arrays are device pointers) ----
// shape 0: 64 x 64 tiles; shape 1: 64 x 16 tiles and shape 3: 64 x 32 tiles
// (outputs of few columns), where outputs with nsplit > 1 leave their chunks'
// partial tiles in `parts` (64 x 16 or 64 x 32 each, column-major) for
// launch_gemm_reduce; shape 2: 64 x 64 tiles, one workgroup per output (for
// outputs of a few tiles).  Shapes 1 and 3 plus 8: operands whose k index is
// contiguous are read as 16-byte vectors, which takes the k-values of an
// MFMA step out of ascending order (the sum is rounded differently)
template <class T>
void launch_gemm(const GOut<T>* outs, int nouts, const GCon<T>* cons, const int32_t* dyn,
                 int64_t ntiles, int shape, hipStream_t s, T* parts = nullptr);
// C = beta C + alpha (sum of the chunks' partial tiles, in chunk order) for the
// split outputs `routs` (tiles numbered by rtile0) of a shape 1 or 3 product
template <class T>
void launch_gemm_reduce(const GOut<T>* routs, int nouts, const T* parts, int64_t ntiles,
                        int shape, hipStream_t s);
// `group`: strips one workgroup takes in turn (fewer, longer workgroups for
// launches of many strips)
template <class T>
void launch_strip(const STask<T>* tasks, int ntasks, const int32_t* dyn, int64_t nstrips,
                  int maxn, hipStream_t s, int group = 1);
// Schur and fill-in updates of colour c over every instance's level, found on
// the device: the targets are the entries (j, k) of row j's pattern whose
// block some cluster i of colour c updates (i near j and k; fill entries
// only when stored, j < k), and each is formed as
// C[active rows, active cols] -= sum over those i, ascending, of
// D_{j, R_i} (D_RR^{-1} D_{R_i, k}).  Fails (err bit 4) when a row has more
// than kSchurMaxContrib contributors.
// Two launches: the first finds every row's contributors (rowtab[g]), the
// targets (appended to `targets`, at most the levels' pattern entries) and
// each target's contributions (appended to `conts`, at most ccap: the
// colour's sum over its clusters of |N(i)|^2; beyond it a target keeps no
// contributions and err bit 4 is set); count[0] and count[1] count them
// (cleared first).  The second forms the targets' updates.
template <class T>
void launch_schur(const SchurLevel<T>* lv, int ninst, int64_t rows, int c, SchurRow* rowtab,
                  SchurTarget* targets, int64_t* conts, int64_t* count, int64_t ccap, int* err,
                  hipStream_t s);
// `lds`: LDS bytes per workgroup the path choices of the fill-row QR, the
// augmentation, the LU and the multipliers may assume (at most kLdsBytes);
// working sets beyond it take the global-memory variants
template <class T>
void launch_rfactor(const RTask<T>* tasks, int ntasks, const FillRef<T>* refs,
                    const int32_t* dyn, int maxn, hipStream_t s, int lds = kLdsBytes);
// pivoted Cholesky factors, one workgroup per task (orders up to kCholMaxOrder)
constexpr int kCholMaxOrder = 128;
template <class T>
void launch_pchol(const CholTask<T>* tasks, int ntasks, int maxn, hipStream_t s);
template <class T>
void launch_gram(const GramTask<T>* tasks, int ntasks, const FillRef<T>* refs,
                 const int32_t* dyn, int64_t ntiles, hipStream_t s);
// gram: the tasks carry G (FP32 storage only), arithmetic in FP64
template <class T>
void launch_augment(const AugTask<T>* tasks, int ntasks, int32_t* r, int* err, int maxn, bool gram,
                    hipStream_t s, int lds = kLdsBytes);
template <class T>
void launch_lu(const LUTask<T>* tasks, int ntasks, const int32_t* dyn, int* err, int maxr,
               hipStream_t s, int lds = kLdsBytes);
template <class T>
void launch_trsm(const TrsmTask<T>* tasks, int ntasks, const int32_t* dyn, int maxr, int maxcols,
                 hipStream_t s, int lds = kLdsBytes);
template <class T, class S>
void launch_copy(const CTask<T, S>* tasks, int ntasks, int64_t ntiles, hipStream_t s);
// pass 0 or 1 of the close-out; err bit 3: a destination missing from the
// next level's pattern
template <class T> void launch_closeout(const CloseLevel<T>& cl, int pass, int* err, hipStream_t s);

template <class T>
void launch_fill(T* p, int64_t n, T v, hipStream_t s);
template <class T, class S>
void launch_gather_rows(T* dst, int64_t ldd, const S* src, int64_t lds, const int64_t* perm,
                        int64_t n, int nrhs, hipStream_t s);
template <class T, class S>
void launch_scatter_rows(T* dst, int64_t ldd, const S* src, int64_t lds, const int64_t* perm,
                         int64_t n, int nrhs, hipStream_t s);
template <class T>
void launch_panel_lu(T* A, int64_t lda, int64_t n, int64_t j0, int nb, int32_t* piv, int* err,
                     hipStream_t s);
template <class T>
void launch_laswp(T* A, int64_t lda, int64_t ncols_total, int64_t j0, int nb,
                  const int32_t* piv, int64_t skip0, int64_t skip1, hipStream_t s);
template <class T>
void launch_trsm_block(const T* A, int64_t lda, T* B, int64_t ldb, int nb, int64_t ncols,
                       int lower_unit, hipStream_t s);
template <class T>
void launch_convert(T* dst, const double* src, int64_t n, hipStream_t s);
void launch_colnorms(const double* X, int64_t ldx, int64_t n, int nrhs, double* out,
                     hipStream_t s);
void launch_dots(const double* V, int64_t ldv, int64_t vstride, int nvec, const double* W,
                 int64_t ldw, int64_t n, int nrhs, double* out, hipStream_t s);
void launch_update(double* W, int64_t ldw, const double* V, int64_t ldv, int64_t vstride,
                   int nvec, const double* coef, double sign, int64_t n, int nrhs,
                   hipStream_t s);
void launch_scale_cols(double* dst, int64_t ldd, const double* src, int64_t lds,
                       const double* norms, int64_t n, int nrhs, int invert, hipStream_t s);
void launch_axpy_cols(double* Y, int64_t ldy, const double* X, int64_t ldx, const double* a,
                      int64_t n, int nrhs, hipStream_t s);
void launch_sub(double* R, int64_t ldr, const double* B, int64_t ldb, const double* AX,
                int64_t ldax, int64_t n, int nrhs, hipStream_t s);
void launch_check_finite(const double* X, int64_t n, int* flag, hipStream_t s);

}  // namespace h2k
