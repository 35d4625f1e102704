/*
 * h2.h -- C ABI of the MI355X H^2 strong recursive skeletonization solver.
 *
 * The library factorizes a symmetric H^2 matrix (Section 1.1 of Boukaram,
 * Keyes, Li, Liu, Turkiyyah, "Linear Complexity H^2 Direct Solver for
 * Fine-Grained Parallel Architectures") with the level-by-level strong
 * recursive skeletonization of Section 2.1 (Algorithms 1 and 2), solves with
 * the factors (Section 2.3, Algorithm 3) and multiplies by the H^2 matrix.
 * All numerical work runs as HIP kernels on one gfx950 GPU.
 *
 * Conventions shared by every entry point:
 *   - Every call returns an h2_status; nothing throws or aborts across the ABI.
 *     On failure h2_last_error(ctx) holds a message.
 *   - Vectors and right-hand sides are DEVICE pointers to column-major float64
 *     arrays with a leading dimension (ld >= N), in ORIGINAL point order; the
 *     tree permutation is applied inside the library.
 *   - Work is enqueued on the context's HIP stream.  Calls return after the
 *     work is enqueued unless stated otherwise; h2_sync waits for it.
 *   - Handles are owned by the caller and released with the matching
 *     *_destroy call.  A factor does not reference its matrix after h2_factor
 *     returns.  Handles are not thread-safe: use one context per host thread.
 */
#ifndef H2_H
#define H2_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  H2_SUCCESS = 0,
  H2_ERROR_INVALID_ARGUMENT = 1, /* bad pointer, size, tolerance or handle */
  H2_ERROR_FORMAT = 2,           /* malformed or unsupported serialized matrix */
  H2_ERROR_OUT_OF_MEMORY = 3,    /* device allocation failed */
  H2_ERROR_SINGULAR = 4,         /* zero pivot in a redundant block or the top block */
  H2_ERROR_NUMERIC = 5,          /* non-finite value produced */
  H2_ERROR_HIP = 6,              /* HIP runtime error */
  H2_ERROR_NOT_CONVERGED = 7,    /* iterative refinement missed its target */
  H2_ERROR_UNSUPPORTED = 8       /* a size beyond what the kernels handle */
} h2_status;

/* Working precision of the factorization.  FP64: the fill row reduced by a
 * Householder QR (Section 2.1, second augmentation option).  The three FP32
 * modes store and compute the factor in FP32 (MFMA with FP32 accumulation)
 * and differ in how the augmentation sees the fill row Y:
 *   FP32: Y Y^T formed in FP64 (Section 2.1, first option) and factored by a
 *     Cholesky with diagonal pivoting, G = P R^T R P^T; the augmentation takes
 *     the SVD of R P^T V_perp in FP32 (clusters of order above 128 take the
 *     QR route);
 *   FP32_GRAM: from the same FP64 Y Y^T, an FP64 eigendecomposition;
 *   FP32_QR: a Householder QR of Y^T, as in FP64. */
typedef enum {
  H2_PREC_FP64 = 0,
  H2_PREC_FP32 = 1,
  H2_PREC_FP32_GRAM = 2,
  H2_PREC_FP32_QR = 3
} h2_prec;

typedef struct h2_context_s* h2_context_t;
typedef struct h2_matrix_s* h2_matrix_t;
typedef struct h2_factor_s* h2_factor_t;

/* Message of a status code (static storage). */
const char* h2_status_string(h2_status s);

/* Device memory callbacks.  `alloc` returns a device pointer to at least
 * `bytes` bytes that work enqueued on `stream` may use from then on, or NULL
 * when it cannot; `free` hands a block back in stream order (work already
 * enqueued on `stream` may still read it; the allocator may give it to later
 * work of the same stream).  Called from the thread that makes the library
 * call, never from inside a kernel or a captured graph. */
typedef void* (*h2_alloc_fn)(size_t bytes, void* stream, void* user);
typedef void (*h2_free_fn)(void* ptr, size_t bytes, void* stream, void* user);

typedef struct {
  int device;        /* HIP device id */
  void* stream;      /* hipStream_t the context enqueues its work on (borrowed).
                        NULL: the context creates its own stream, which orders
                        itself with the legacy default stream like any
                        hipStreamCreate stream, and destroys it with the context. */
  h2_alloc_fn alloc; /* both NULL: hipMallocAsync / hipFreeAsync on the stream,
                        from the device's default memory pool, whose release
                        threshold is raised so that freed blocks stay cached */
  h2_free_fn free;
  void* user;        /* passed to alloc and free */
} h2_context_opts;

/* Create a context (opts NULL = device 0, its own stream, the pool
 * allocator).  Every device byte the library holds for the context, its
 * matrices and its factors comes from the context's allocator: the factor's
 * per-level block buffers (Section 2.2: one buffer per level, offsets from
 * prefix sums of the block dimension products) as well as every temporary
 * workspace (Section 2.2: a memory pool for temporaries).  Matrices and
 * factors must be destroyed before their context. */
h2_status h2_context_create(const h2_context_opts* opts, h2_context_t* ctx);
h2_status h2_context_destroy(h2_context_t ctx);
/* Last error message of the context (valid until the next call on it). */
const char* h2_last_error(h2_context_t ctx);
/* Wait for all work enqueued by the context. */
h2_status h2_sync(h2_context_t ctx);

/*
 * Load a serialized symmetric H^2 matrix (format H2B1 v1: cluster tree,
 * same-level near/far lists, leaf bases U, transfers E, dense near blocks D,
 * couplings S; Section 1.1).  `blob` is a HOST buffer of `bytes` bytes, owned
 * by the caller and not referenced after return.  It is validated as by
 * h2_blob_check, then the data are copied to the device.
 * Errors: H2_ERROR_FORMAT (the message names the failed check).
 */
h2_status h2_matrix_load(h2_context_t ctx, const void* blob, size_t bytes, h2_matrix_t* H);

/*
 * Validate a serialized matrix on the host without a device: magic and
 * version, header sizes, balanced tree (all leaves on one level, children
 * tiling their parent), permutation, sorted same-level near/far CSR lists
 * with a symmetric pattern, the diagonal in every near list, data length,
 * finite entries, orthonormal leaf bases (max |U^T U - I| <= 1e-10),
 * orthonormal stacked transfers of every inner node (max |sum_c E_c^T E_c - I|
 * <= 1e-10), symmetric values (max |D_ji - D_ij^T| and max |S_ji - S_ij^T| at
 * most 1e-12 ||A||_2 with the blob's norm).  Section 1.1 defines the
 * representation; the symmetry is the standing assumption of Section 2.
 * Returns H2_SUCCESS or H2_ERROR_FORMAT; on failure the reason is copied
 * into `msg` (capacity `msgcap` bytes, NUL-terminated; msg may be NULL).
 */
h2_status h2_blob_check(const void* blob, size_t bytes, char* msg, size_t msgcap);
h2_status h2_matrix_destroy(h2_matrix_t H);

typedef struct {
  int64_t n;         /* matrix order N */
  int32_t dim;       /* point dimension recorded in the blob */
  int32_t depth;     /* leaf level L (root = 0) */
  int32_t top_level; /* first level with an admissible block, -1 if none */
  int32_t n_nodes;
  double norm2;      /* ||A||_2 estimate stored in the blob */
  int64_t device_bytes;
} h2_matrix_info;
h2_status h2_matrix_get_info(h2_matrix_t H, h2_matrix_info* info);

/*
 * Y = A X, FP64 H^2 matrix-vector product (the product of Section 1.1:
 * near blocks plus the nested-basis upsweep / coupling / downsweep).
 * X and Y: device, N x nrhs, leading dimensions ldx, ldy >= N; must not alias.
 */
h2_status h2_matvec(h2_context_t ctx, h2_matrix_t H, const double* X, int64_t ldx, int nrhs,
                    double* Y, int64_t ldy);

/*
 * The product of h2_matvec for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same kernels, with every work array (tree-ordered vectors,
 * basis coefficients, launch descriptors, partial tiles) in a library-owned
 * static device array of 64 MiB per device instead of allocated memory.  It
 * calls no device allocator.  Needs about 8 (2 N + 2 K) nrhs bytes for the
 * vectors (K = sum of the cluster ranks) plus the descriptors, about
 * 50 bytes per near and far block; larger problems fail with
 * H2_ERROR_UNSUPPORTED and a message giving the size.  Every call on one
 * device shares that device's array: calls that overlap in time on one GPU
 * (from any context or thread) race and give wrong results.  Synchronizes
 * with the context's stream before returning.  X and Y as for h2_matvec.
 */
h2_status h2_matvec_noalloc(h2_context_t ctx, h2_matrix_t H, const double* X, int64_t ldx,
                            int nrhs, double* Y, int64_t ldy);

/* Options of a factorization call (NULL = all defaults). */
typedef struct {
  double norm2;       /* > 0: ||A||_2 used in eps_fill = tol ||A||_2 in place of
                         the blob's estimate (Section 2.1 leaves the norm to the user) */
  int64_t pool_bytes; /* > 0: cap on the device bytes the call holds at once
                         (factor storage plus workspaces, over all instances);
                         reaching it fails the call with OUT_OF_MEMORY */
  int32_t keep_owner_lists; /* nonzero: keep every colour's Schur target lists for
                               h2_factor_export_ints(H2_INT_OWNERS) (host memory grows
                               with the number of targets) */
  int32_t lds_limit_kib;    /* > 0: on-chip (LDS) bytes per workgroup, in KiB, that the
                               kernels of the fill-row QR, the augmentation, the LU of
                               D_RR and the multipliers may assume, if below the default
                               150; working sets beyond it take the global-memory
                               variants of those kernels (same results up to rounding
                               order).  For exercising those variants at small orders. */
} h2_factor_opts;

/*
 * Factorize (Algorithm 1 with Algorithm 2 per colour): eps_lu = tol, fill
 * truncation threshold eps_fill = tol * ||A||_2 (blob norm unless opts
 * overrides it).  prec selects the arithmetic of the factorization and of
 * its storage (FP64, or FP32 with FP32 accumulation).  Synchronizes with the
 * device once per tree level.  Errors: INVALID_ARGUMENT (tol < 0 or not
 * finite, bad opts), OUT_OF_MEMORY (allocator failure or opts->pool_bytes),
 * SINGULAR (zero pivot), NUMERIC, UNSUPPORTED.
 */
h2_status h2_factor(h2_context_t ctx, h2_matrix_t H, double tol, h2_prec prec,
                    const h2_factor_opts* opts, h2_factor_t* F);
h2_status h2_factor_destroy(h2_factor_t F);

/*
 * X = (LU)^{-1} B with the factors (Algorithm 3).  B, X: device N x nrhs FP64
 * (an FP32 factor converts on the way in and out).  X == B is allowed.
 */
h2_status h2_solve(h2_context_t ctx, h2_factor_t F, const double* B, int64_t ldb, int nrhs,
                   double* X, int64_t ldx);

typedef struct {
  double target_bkwd; /* stop when ||b - A x|| / ||b|| <= target for every column */
  int restart;        /* GMRES restart length */
  int max_outer;      /* refinement steps */
  double inner_rtol;  /* GMRES relative tolerance on the preconditioned residual; every
                         refinement step recomputes the FP64 residual, so a loose value
                         (1e-3) trades inner steps (one solve + one product each) for
                         cheap outer steps */
} h2_ir_opts;

typedef struct {
  int outer_iterations;
  int inner_iterations;   /* total GMRES steps over all refinement steps */
  double max_bkwd;        /* largest achieved backward error over the columns */
} h2_ir_report;

/*
 * GMRES-based iterative refinement (Carson-Higham): x0 = solve(F, b); repeat
 * r = b - A x with the FP64 H^2 product, stop at the target, solve A d = r by
 * GMRES left-preconditioned with the factor, x += d.  Residuals, updates and
 * the Krylov basis are FP64; the factor may be FP32.  Columns are refined
 * together.  B, X: device N x nrhs FP64.  opts NULL = {1e-12, 30, 20, 1e-3}.
 * Returns NOT_CONVERGED (with the report filled) when the target is missed.
 */
h2_status h2_solve_ir(h2_context_t ctx, h2_matrix_t H, h2_factor_t F, const double* B,
                      int64_t ldb, int nrhs, double* X, int64_t ldx, const h2_ir_opts* opts,
                      h2_ir_report* report);

/*
 * Batched factorization of `count` independent matrices: levels are aligned
 * by height above the leaves and every (height, colour step) runs as one set
 * of launches over all instances.  Fs[i] receives the factor of Hs[i] and can
 * be used with h2_solve like any other factor.  opts->norm2, when set,
 * replaces every instance's norm; a failure fails the whole call.
 */
h2_status h2_factor_batched(h2_context_t ctx, int count, const h2_matrix_t* Hs, double tol,
                            h2_prec prec, const h2_factor_opts* opts, h2_factor_t* Fs);

/* Batched solve: one set of launches per (height, colour step) over all instances.
 * B[i], X[i]: device N_i x nrhs FP64 with leading dimensions ldb[i], ldx[i]. */
h2_status h2_solve_batched(h2_context_t ctx, int count, const h2_factor_t* Fs,
                           const double* const* B, const int64_t* ldb, int nrhs,
                           double* const* X, const int64_t* ldx);

typedef enum {
  H2_INT_SIZES = 0,    /* n_i of every cluster of the level */
  H2_INT_RANKS = 1,    /* augmented rank k~_i */
  H2_INT_COLORS = 2,   /* colour of every cluster */
  H2_INT_FILL = 3,     /* fill pattern: pairs (j, k) of global node ids, flattened */
  H2_INT_NTOP = 4,     /* order of the dense top block (level argument ignored) */
  H2_INT_LEVELS = 5,   /* skeletonized levels, leaf level first */
  H2_INT_OFFSETS = 6,  /* block layout of the level (Section 2.2: offsets are prefix sums of
                          the products of block dimensions): for every entry of the level's
                          block pattern (near pairs and fill pairs, rows ascending, columns
                          ascending) the record (j, k, kind, offset) with global node ids;
                          near blocks and fill blocks have a buffer each, n_j x n_k blocks in
                          that order.  kind 0: near block; 1: fill block (j < k); 2: fill
                          entry (j, k) with k < j, stored once as the transpose of the block
                          (k, j) (the fill of a symmetric matrix is symmetric), whose offset
                          it repeats */
  H2_INT_CLUSTER_OFFSETS = 7, /* per cluster of the level: offset of Q~_i (prefix sum of n_i^2) */
  H2_INT_OWNERS = 8    /* Schur/fill-in owner lists (needs opts->keep_owner_lists): for every
                          colour c ascending and every stored target block (j, k) that
                          clusters of colour c update (near pairs, and fill pairs with
                          j < k), targets ascending, the record (c, j, k, m, i_1 .. i_m)
                          with the m contributing clusters ascending (global ids) */
} h2_int_kind;

/* Copy an integer output of the factorization into the host buffer `buf`
 * (capacity `cap` entries); *len receives the full length. */
h2_status h2_factor_export_ints(h2_factor_t F, int level, h2_int_kind kind, int64_t* buf,
                                int64_t cap, int64_t* len);

typedef enum {
  H2_MAT_Q = 0,      /* Q~_i = [V~perp, V~] of cluster i (local index) of the level, n_i x n_i */
  H2_MAT_BLOCK = 1,  /* factored near block (i, j) of the level, n_i x n_j (panels in place) */
  H2_MAT_TOP = 2     /* dense top block after its LU factorization, n_top x n_top */
} h2_mat_kind;

/* Copy one factor matrix to the HOST buffer `buf` (capacity `cap` doubles,
 * column-major); *rows and *cols receive its shape (also when cap is too
 * small, in which case nothing is copied).  Synchronizes with the device.
 * For inspection of the factorization against a reference implementation. */
h2_status h2_factor_export_matrix(h2_factor_t F, int level, h2_mat_kind kind, int i, int j,
                                  double* buf, int64_t cap, int64_t* rows, int64_t* cols);

#define H2_PHASES 10

typedef struct {
  int32_t levels;          /* skeletonized levels */
  int32_t max_colors;
  int64_t n_top;
  int64_t factor_bytes;    /* device bytes held by the factor */
  int64_t peak_bytes;      /* high-water mark of device bytes during h2_factor */
  double factor_flops;     /* algorithmic flop count of the factorization */
  double solve_flops_per_rhs;
  double time_ms[H2_PHASES];     /* device time of the last h2_factor per phase, from
                                    events around the phase's launches:
                                    0 fill-row QR (k_rfactor), 1 augmentation and
                                    complement (k_augment), 2 projection (k_strip),
                                    3 LU of D_RR (k_lu), 4 multipliers (k_trsm),
                                    5 Schur and fill-in (k_gemm), 6 close-out (k_copy),
                                    7 dense top LU; 8 host planning the stream
                                    waited for (wall); 9 total wall */
  double phase_flops[H2_PHASES]; /* algorithmic flops per phase (same indices) */
  double phase_bytes[H2_PHASES]; /* algorithmic HBM bytes per phase (each operand once) */
  int64_t launches[H2_PHASES];   /* kernel launches per phase */
  int64_t solves;                /* h2_solve calls served by the factor's recorded plan */
  int64_t solve_graph_launches;  /* of those, replays as one captured HIP graph launch */
} h2_stats;
h2_status h2_factor_get_stats(h2_factor_t F, h2_stats* stats);

#ifdef __cplusplus
}
#endif
#endif /* H2_H */
