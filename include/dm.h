/*
 * dm.h - implicit distance-matrix matrix-vector products on MI355X (gfx950).
 *
 * For points x_1..x_n in R^d and a distance f, the n x n matrix
 * A_ij = f(x_i, x_j) is never formed; the library answers queries z -> A z
 * (the matrix-vector query model of Section 1 of Indyk & Silwal, "Faster
 * Linear Algebra for Distance Matrices").
 *
 *   DM_L1    f(x, y) = sum_k |x(k) - y(k)|       Algorithms 1 and 2, Section 2
 *   DM_L2SQ  f(x, y) = sum_k (x(k) - y(k))^2     Algorithm 3, Appendix A
 *   DM_TV    f(x, y) = (1/2) sum_k |x(k) - y(k)|  total variation distance of
 *            distributions given as probability vectors (the TV theorem of
 *            Appendix A.3): the l1 path with the result halved.  Float data
 *            only (integer data: DM_ERR_DTYPE); the points are not checked
 *            to lie on the simplex.
 *   DM_L3    f(x, y) = sum_k |x(k) - y(k)|^3     l_p^p for odd p (the odd-p
 *   DM_L5    f(x, y) = sum_k |x(k) - y(k)|^5     theorem of Appendix A.1): the
 *            sort of Algorithm 1 and prefix sums of z x^t, t = 0 .. p, combined
 *            as sum_t C(p, t) (-1)^t x^(p-t) (2 P_t - T_t).  Integer data is
 *            exact under the guard ||z||_1 sum_k range_k^p < 2^62.
 *   DM_L4    f(x, y) = sum_k (x(k) - y(k))^4     l_p^p for even p (Algorithm 5
 *   DM_L6    f(x, y) = sum_k (x(k) - y(k))^6     and the even-p theorem of
 *            Appendix A.1): no sort; the moments F_t(k) = sum_j z_j x~_j(k)^t
 *            of the centred coordinates x~ = x - c (c_k the midpoint of the
 *            coordinate's range), then per point
 *            sum_k sum_t C(p, t) (-1)^t x~_i(k)^(p-t) F_t(k).  Float data in
 *            FP64; integer data exact under the same guard as odd p.
 *   DM_KL    f(x, y) = sum_k x(k) log(x(k) / y(k)), the KL divergence
 *            D(x || y) (Algorithm 4 and the KL theorem of Appendix A):
 *            (A z)_i = -H(x_i) sum_j z_j - sum_k x_i(k) S_k with
 *            S_k = sum_j z_j log x_j(k).  A is not symmetric.
 *   DM_CE    f(x, y) = -sum_k x(k) log y(k), the cross entropy (Appendix
 *            A.3): (A z)_i = -sum_k x_i(k) S_k.  A is not symmetric.
 *            KL and CE: float data only, every coordinate finite and > 0
 *            (dm_prepare returns DM_ERR_ARG otherwise); the points need not
 *            lie on the simplex.  The workspace keeps log x_i(k) in FP64
 *            (n d 8 bytes), formed once at preparation.
 *   DM_MAHA2 f(x, y) = (x - y)^T M (x - y), the squared Mahalanobis distance
 *            for a d x d matrix M (only its symmetric part matters):
 *            (A z)_i = q_i sum_j z_j + sum_j q_j z_j
 *                      - x~_i^T (M + M^T) sum_j z_j x~_j,  q_i = x~_i^T M x~_i.
 *   DM_BILINEAR f(x, y) = x^T M y, the form that the Mahalanobis paragraph of
 *            Appendix A.2 writes down (Algorithms 8 and 9):
 *            (A z)_i = x_i^T M (sum_j z_j x_j).
 *            MAHA2 and BILINEAR: float data only, prepared with
 *            dm_prepare_matrix.  The sort-free metrics accumulate in FP64
 *            and round once to FP32.
 *
 * l1: dm_prepare sorts the n values of every coordinate once (Algorithm 1;
 * stable, ties by ascending point index) and keeps the permutations, their
 * inverses (ranks) and the sorted values.  Each query then walks every
 * coordinate in sorted order with prefix sums P0 = sum z_j and
 * P1 = sum x_j(k) z_j and adds x_ik (2 P0 - T0) - (2 P1 - T1) to row i
 * (Algorithm 2 and the proof of its exactness theorem, Section 2).
 * l2 squared: A z = ||x_i||^2 sum_j z_j + sum_j ||x_j||^2 z_j - 2 X (X^T z)
 * (the decomposition of Section 1.2 and Algorithm 3).
 *
 * Conventions shared by every entry point
 *  - All array arguments named X, Z, Out, U, workspace are DEVICE pointers
 *    (memory on the current HIP device); every other pointer is host memory.
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *  - X is n x d row-major.  Z and Out are n x b row-major (a point's b
 *    right-hand-side values are contiguous).
 *  - Float data (DM_F32, DM_F64): Z is DM_F32, Out is float.  DM_F64 points
 *    are rounded once to FP32 at preparation.  Integer data (DM_I32, DM_I64,
 *    |x| < 2^31): Z is DM_I32 or DM_I64, Out is int64 and exact.
 *  - Argument errors are reported synchronously and before any device work.
 *    Data-dependent errors found on the device during a query (non-finite Z,
 *    an integer result that could exceed int64) are sticky: dm_sync returns
 *    them.  After an error the contents of Out are unspecified.
 *  - Entry points are not thread-safe for one handle; distinct handles are
 *    independent.  Queries on one handle must not overlap in time on
 *    different streams.
 */
#ifndef DM_H
#define DM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dm_handle dm_handle;

typedef enum {
    DM_L1 = 1,
    DM_L2SQ = 2,
    DM_TV = 3,
    DM_L3 = 4,
    DM_L5 = 5,
    DM_L4 = 6,
    DM_L6 = 7,
    DM_KL = 8,
    DM_CE = 9,
    DM_MAHA2 = 10,
    DM_BILINEAR = 11
} dm_metric;
typedef enum { DM_F32 = 1, DM_F64 = 2, DM_I32 = 3, DM_I64 = 4 } dm_dtype;
typedef enum {
    DM_OK = 0,
    DM_ERR_ARG = -1,       /* bad argument (NULL, size < 1, bad enum, short workspace) */
    DM_ERR_NONFINITE = -2, /* NaN or Inf in X (prepare) or Z (query)                     */
    DM_ERR_OVERFLOW = -3,  /* integer query whose exact result may not fit in int64      */
    DM_ERR_NOMEM = -4,     /* device allocation failed                                   */
    DM_ERR_DEVICE = -5,    /* no usable HIP device, or a HIP call failed                 */
    DM_ERR_DTYPE = -6,     /* dtype not allowed here, or integer |x| >= 2^31              */
    DM_ERR_STATE = -7      /* handle used in a way its kind does not support             */
} dm_status;

/* Static text for a status code (never NULL). */
const char* dm_status_string(int32_t status);

/*
 * Bytes of device workspace dm_prepare needs for one dataset: the persistent
 * arrays, the sort's temporary buffers, and everything a later query of any
 * b <= 64 uses (the control block with the sticky status and the chained-scan
 * ticket counters, the query scratch, the look-back record regions of every
 * pass shape and tile variant, and for l1 / TV the single-column group
 * buffer).  The matrix-vector query model of Section 1 prepares once and then
 * answers products only, so with a caller workspace no query allocates.
 * Pure host function.
 * Errors: DM_ERR_ARG for n < 1, d < 1, n * d >= 2^32, bad metric or dtype,
 * bytes == NULL.
 */
dm_status dm_workspace_size(int64_t n, int32_t d, int32_t metric, int32_t dtype, size_t* bytes);

/*
 * Preparation (Algorithm 1 for l1): validates X, and for the sorted metrics
 * (l1, TV, odd p) builds per coordinate k the stable sorted order perm[k][r],
 * its inverse rank[k][i] and the sorted values xs[k][r]; for every metric the
 * FP64 (int64 for integer data) row sums s_i = sum_k x_ik^p and squared norms
 * ||x_i||^2.  For l2 squared, odd p and the sort-free metrics it keeps an FP32
 * (int32) copy of X; for the sort-free metrics also the per-coordinate range
 * midpoints and, for KL, the per-point values sum_k x_ik log x_ik.
 * Float data of the sorted metrics and l2 squared is kept relative to a
 * per-coordinate centre c_k (every such metric is translation invariant): the
 * FP32 midpoint of the coordinate's range when x - c_k is exact for every x of
 * the coordinate (Sterbenz's lemma: all x within a factor two of c_k), else 0.
 * The sorted values, row statistics and the point copy are those of x - c, so
 * the FP32 query keeps its accuracy on points far from the origin.
 * DM_MAHA2 and DM_BILINEAR are prepared with dm_prepare_matrix instead.
 *
 * X: device, n x d row-major of `dtype`; only read during the call.
 * workspace: device memory of at least dm_workspace_size bytes, 256-byte
 *   aligned, owned by the caller, which must outlive the handle; NULL lets the
 *   library allocate (and dm_free release) it.  Either way the handle's device
 *   memory is this one block: dm_matvec, dm_matvec_multi and dm_reserve never
 *   allocate or free device memory.
 * Blocking: returns after the device work finished.
 * Errors: DM_ERR_ARG, DM_ERR_DTYPE (|x| >= 2^31 in integer data),
 * DM_ERR_NONFINITE (NaN/Inf in X, or an FP64 value beyond the FP32 range),
 * DM_ERR_NOMEM, DM_ERR_DEVICE.  DM_ERR_ARG also for DM_KL or DM_CE data with
 * a coordinate <= 0 (after rounding to FP32), and for DM_MAHA2 or
 * DM_BILINEAR.  On error *out is NULL and nothing leaks.
 */
dm_status dm_prepare(const void* X, int64_t n, int32_t d, int32_t metric, int32_t dtype,
                     void* workspace, size_t ws_bytes, void* stream, dm_handle** out);

/*
 * Preparation of a metric that carries a d x d matrix (DM_MAHA2,
 * DM_BILINEAR; the preprocessing of Algorithm 8 in Appendix A.2).  M is HOST
 * memory, d x d row-major FP64, copied during the call.  For DM_MAHA2 the
 * per-point values q_i = (x_i - c)^T M (x_i - c) are formed here (O(n d^2)
 * work, FP64).  Every other argument, the blocking and the errors are those of
 * dm_prepare; additionally DM_ERR_ARG for another metric or M == NULL, and
 * DM_ERR_NONFINITE for a NaN or Inf in M.  dm_prepare itself returns
 * DM_ERR_ARG for these two metrics.
 */
dm_status dm_prepare_matrix(const void* X, int64_t n, int32_t d, int32_t metric, int32_t dtype, const double* M,
                            void* workspace, size_t ws_bytes, void* stream, dm_handle** out);

/*
 * One query: Out = A Z for b right-hand sides at once (b = 1 is the single
 * vector form; b > 1 shares every sorted permutation across the b columns,
 * which is the matrix product of the Appendix C lemma on products AB taken b
 * columns at a time).
 *
 * Z: device n x b of `z_dtype` (DM_F32 for float data; DM_I32 or DM_I64 for
 * integer data).  Out: device n x b, float or int64.  Z and Out must not
 * overlap.  1 <= b <= 64.
 * Stream-ordered and asynchronous: it only enqueues work on `stream`, in the
 * handle's workspace; it neither allocates device memory nor waits.  The
 * first call with a given (Z, Out, b, z_dtype) records the query's launches
 * (totals and one pass per coordinate for l1) in a hipGraph on a private
 * capture stream, and later calls with the same arguments replay it with one
 * hipGraphLaunch; the handle keeps the 4 most recently used graphs (evicting
 * one waits for the handle's last stream).  Replays read Z and write Out at
 * the recorded addresses, so the contents may change between calls.  While
 * profiling is on (dm_profile_enable), or with the environment variable
 * DM_QUERY_GRAPH=0 at preparation, queries are launched eagerly instead.
 * Errors (synchronous): DM_ERR_ARG, DM_ERR_DTYPE, DM_ERR_DEVICE.
 * Errors (sticky, via dm_sync): DM_ERR_NONFINITE, DM_ERR_OVERFLOW.
 */
dm_status dm_matvec(dm_handle* h, const void* Z, int32_t z_dtype, int32_t b, void* Out, void* stream);

/*
 * The same query as dm_matvec, for callers that cannot allocate device memory
 * or do not want to hold the query part of the workspace busy: code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation.  Its
 * scratch (totals partials, the metric's scratch, the look-back records of the
 * pass, and for a single l1 / TV column as many coordinates of the group
 * buffer as fit) comes from the library's static device array of 32 MiB per
 * GPU (held by every GPU the library runs on until the process ends) instead
 * of the workspace.  Z, Out, the stream and the results are exactly those of
 * dm_matvec (same kernels); the handle's workspace still holds the prepared
 * data and the sticky status.  Allocates nothing.
 * The array is shared by every call on a GPU and keeps the last call's
 * contents (each call clears what must start at zero), so calls that overlap
 * in time on one GPU, from any handle or stream, race: serialise them.
 * The handle's device must be the current device.
 * Errors: those of dm_matvec, and DM_ERR_ARG when the call's scratch exceeds
 * the 32 MiB (large n x b shapes: use dm_matvec) or another device is current.
 */
dm_status dm_matvec_static(dm_handle* h, const void* Z, int32_t z_dtype, int32_t b, void* Out, void* stream);

/* Kept for callers that reserved query memory before the workspace held it:
 * checks b (1..64) and does nothing else, since the workspace already holds
 * every query's memory.  Errors: DM_ERR_ARG, DM_ERR_STATE (multi-dataset
 * handle). */
dm_status dm_reserve(dm_handle* h, int32_t b);

/*
 * Tile tuning of the l1 pass (the per-coordinate gather-scan-scatter of
 * Algorithm 2, Section 2).  Each pass configuration (data path, b rounded up
 * to a power of two) has dm_variant_count() tile variants with identical
 * results on integer data and results within the same error bounds on float
 * data; they differ only in speed, which depends on n, b and the device.
 *
 * dm_tune times every variant on this handle's own sorted coordinates
 * (`reps` passes each, after one untimed pass, with a zero right-hand side of
 * n x b `z_dtype` values), keeps the fastest for later dm_matvec calls of the
 * same configuration and stores it in *chosen.  ms_per_pass, if not NULL,
 * receives dm_variant_count() mean pass times in milliseconds.  It allocates
 * and frees temporary device memory (the right-hand side and the result) and
 * synchronises `stream`.  If the environment variable DM_TUNE_CACHE names a
 * file, the choice is appended to it as one text line, and handles prepared
 * later on the same device type with the same metric, dtype, d and
 * floor(log2 n) start from the cached choice instead of variant 0.
 * Errors: DM_ERR_ARG (NULL handle, b outside 1..64, reps outside 1..4096, a
 * metric other than l1), DM_ERR_DTYPE, DM_ERR_STATE (multi-dataset handle),
 * DM_ERR_NOMEM, DM_ERR_DEVICE.
 *
 * dm_set_variant fixes the variant of a configuration (for callers that keep
 * their own tuning results, and for tests); dm_get_variant reports the one in
 * use.  Both are host-only and return the dm_tune argument errors.
 */
int32_t dm_variant_count(void);
dm_status dm_tune(dm_handle* h, int32_t b, int32_t z_dtype, int32_t reps, void* stream, int32_t* chosen,
                  double* ms_per_pass);
dm_status dm_set_variant(dm_handle* h, int32_t b, int32_t z_dtype, int32_t variant);
dm_status dm_get_variant(dm_handle* h, int32_t b, int32_t z_dtype, int32_t* variant);

/* Wait for the handle's last stream, then return and clear the sticky status. */
dm_status dm_sync(dm_handle* h);

/* Shape of a handle.  Any output pointer may be NULL. */
dm_status dm_info(const dm_handle* h, int64_t* n, int32_t* d, int32_t* metric, int32_t* dtype);

/*
 * Copy the preparation results of a sorted-metric handle into caller device buffers
 * (any may be NULL): perm and rank are d x n uint32, xs is d x n float (float
 * data) or int32 (integer data).  perm[k][r] is the point at rank r of
 * coordinate k (ties by ascending point id, Algorithm 1); rank[k][i] is the
 * rank of point i (the positions Algorithm 2 looks up), formed from perm by a
 * kernel on this call, since queries never read it.  Stream-ordered.  Errors: DM_ERR_ARG,
 * DM_ERR_STATE for a handle of a metric that does not sort (l2 squared and
 * the sort-free metrics).
 */
dm_status dm_copy_sorted(const dm_handle* h, uint32_t* perm, uint32_t* rank, void* xs, void* stream);

/*
 * Integer overflow guard (pure, host): nonzero when z_l1 * sum_ranges < 2^62,
 * i.e. when every |(A z)_i| <= sum_j |z_j| * max_ij A_ij is certainly below
 * 2^63 so that wrapping int64 arithmetic returns the exact result.
 * sum_ranges is sum_k (max_k - min_k) for l1 and sum_k (max_k - min_k)^2 for
 * l2 squared.  The device applies the same test during integer queries.
 */
int dm_int_bound_ok(double sum_ranges, double z_l1);

/*
 * Many point sets in one query.  Each dataset is prepared exactly as by
 * dm_prepare (l1 only; all datasets share one segmented sort), and one call
 * of dm_matvec_multi answers A_s Z_s for every dataset s with the same b.
 * The query is captured once per b in a hipGraph (descriptor upload, totals,
 * one launch per coordinate round) and replayed on every call.
 *
 * sets: host array of count descriptors; X device, n x d row-major.
 * Z[s]: device n_s x b, float for float datasets, int32 for integer ones.
 * Out[s]: device n_s x b, float or int64.  Z and Out are host arrays of
 * count device pointers.  1 <= b <= 64.
 * A call that changes any Z/Out pointer waits for the previous call's upload
 * of the pointer table to have run.  The first call with a new b (or with a
 * new choice of 16-byte row access) lays out that b's tile tables and record
 * regions in the workspace's plan area, which dm_workspace_size_multi sizes
 * for every b <= 64, and captures its graph; this synchronises the call's
 * stream.  No call allocates device memory.  Errors as for dm_prepare / dm_matvec;
 * a non-l1 metric is DM_ERR_ARG; dm_matvec_multi on a single-dataset handle
 * (or dm_matvec on a multi-dataset handle) is DM_ERR_STATE.
 */
typedef struct {
    const void* X;
    int64_t n;
    int32_t d;
    int32_t metric;
    int32_t dtype;
} dm_dataset;
dm_status dm_workspace_size_multi(const dm_dataset* sets, int32_t count, size_t* bytes);
dm_status dm_prepare_multi(const dm_dataset* sets, int32_t count, void* workspace, size_t ws_bytes, void* stream,
                           dm_handle** out);
dm_status dm_matvec_multi(dm_handle* h, const void* const* Z, int32_t b, void* const* Out, void* stream);
dm_status dm_multi_count(const dm_handle* h, int32_t* count);

/*
 * Tile tuning of the many-dataset query (the batching of the Appendix C lemma
 * on products AB, taken over many point sets).  Each b has
 * dm_multi_variant_count() tile variants of its coordinate-round launches
 * (ranks per thread R, R / 2, and 2 R for b <= 8 or R / 4 for wider blocks),
 * with identical results on integer datasets and results within the same
 * bounds on float ones.  dm_tune_multi runs the caller's query (Z, Out as for
 * dm_matvec_multi; Out receives A Z) once untimed and `reps` times timed with
 * every variant's plan, keeps the fastest for later calls with this b (its
 * plan stays captured) and stores it in *chosen; ms_per_query, if not NULL,
 * receives dm_multi_variant_count() mean query times in milliseconds.  It
 * synchronises `stream`; it allocates no device memory (every variant's plan
 * fits the workspace's plan area).  dm_set_variant_multi fixes a variant for
 * a b (host only), dm_get_variant_multi reports it.
 * Errors: DM_ERR_ARG (NULL pointers, b outside 1..64, reps outside 1..4096,
 * variant out of range), DM_ERR_STATE (single-dataset handle), DM_ERR_DEVICE.
 */
int32_t dm_multi_variant_count(void);
dm_status dm_tune_multi(dm_handle* h, const void* const* Z, int32_t b, void* const* Out, int32_t reps, void* stream,
                        int32_t* chosen, double* ms_per_query);
dm_status dm_set_variant_multi(dm_handle* h, int32_t b, int32_t variant);
dm_status dm_get_variant_multi(dm_handle* h, int32_t b, int32_t* variant);

/*
 * Rank-k approximation A ~ U diag(lam) U^T by block Krylov iteration, using
 * only products with A (the query model of Section 1; Appendix C.1 cites
 * block Krylov methods for the top singular values, and Table 2 lists the
 * low-rank application).  The paper gives no algorithm; this one:
 *   Q_0 = orth(A Omega), Q_j = orth(A Q_{j-1} against Q_0..Q_{j-1}),
 *   j < iters (block Gram-Schmidt twice, then Cholesky QR twice; columns
 *   numerically dependent on earlier ones are dropped as zero columns);
 *   T = Q^T A Q from the same products plus one more, A Q_{iters-1};
 *   T = V diag(w) V^T by cyclic Jacobi; the `rank` pairs of largest |w|
 *   give lam (in decreasing |lam|) and U = Q V_k.
 * Products with A go through dm_matvec (FP32 in and out, block columns at a
 * time: iters + 1 queries); everything else is FP64 on the device.
 *
 * h: a prepared float handle of a symmetric metric (every metric but DM_KL,
 * DM_CE and a DM_BILINEAR handle whose M is not symmetric).  Omega: device n x block
 * FP64, the start block, drawn by the caller (the library draws no random
 * numbers).  U: device n x rank FP64 (out), orthonormal columns (zero
 * columns only if A has fewer than `rank` independent directions in the
 * basis).  lam: device rank FP64 (out).  sweeps (optional, host): Jacobi
 * sweeps used.  1 <= block <= 64, iters >= 1, block * iters <= 1024,
 * 1 <= rank <= min(64, block * iters).
 * Allocates and frees device memory (about (iters + 2) n block doubles) and
 * synchronises `stream`.
 * Errors: DM_ERR_ARG, DM_ERR_DTYPE (integer handle), DM_ERR_STATE
 * (multi-dataset handle, or A not symmetric), DM_ERR_NOMEM, DM_ERR_DEVICE,
 * DM_ERR_NONFINITE.
 */
dm_status dm_lowrank(dm_handle* h, int32_t rank, int32_t block, int32_t iters, const double* Omega, double* U,
                     double* lam, void* stream, int32_t* sweeps);

/*
 * Approximate l2 distance products (Appendix A.4: the Gaussian embedding
 * theorem, the preprocessing of Algorithm 10 and the approximate l2 theorem).
 * Writes the embedded points
 *     Xout[i][t] = (1 / (beta k)) sum_j G[t][j] X[i][j],  beta = sqrt(2/pi),
 * so that ||Xout_i - Xout_j||_1 approximates ||x_i - x_j||_2 (relative error
 * about 0.76 / sqrt(k) per entry for Gaussian G).  The caller then prepares
 * Xout with the l1 metric (dm_prepare, d = k) and queries it with dm_matvec;
 * that handle answers B z with B_ij = ||Xout_i - Xout_j||_1.
 *
 * X: device n x d, dtype DM_F32 / DM_F64 / DM_I32 / DM_I64 (row-major).
 * G: device k x d FP64 with iid N(0, 1) entries, drawn by the caller (the
 * library draws no random numbers).  Xout: device n x k FP32 (out), must not
 * overlap X.  1 <= k <= 65536.  Accumulation is FP64, rounded once to FP32.
 * Stream-ordered and asynchronous; non-finite X gives non-finite Xout, which
 * dm_prepare then rejects.
 * Errors: DM_ERR_ARG (NULL pointers, sizes, dtype, overlap), DM_ERR_DEVICE.
 */
dm_status dm_embed_l2(const void* X, int64_t n, int32_t d, int32_t dtype, const double* G, int32_t k, float* Xout,
                      void* stream);

/*
 * Measurement support.  While profiling is on, every launch of the listed
 * kernel classes is bracketed by HIP events on the query stream;
 * dm_profile_read waits for them and returns the summed device time and the
 * number of launches since profiling was last switched on.
 * Errors: DM_ERR_ARG (NULL handle, bad class), DM_ERR_DEVICE.
 */
typedef enum { DM_K_L1_PASS = 0, DM_K_TOTALS = 1, DM_K_L2 = 2, DM_K_SORTFREE = 3, DM_K_CLASSES = 4 } dm_kernel_class;
dm_status dm_profile_enable(dm_handle* h, int32_t on);
dm_status dm_profile_read(dm_handle* h, int32_t kernel_class, double* total_ms, int64_t* launches);

/*
 * Streaming copy of `bytes` bytes (a nonzero multiple of 16) from src to dst
 * (device pointers, 16-byte aligned, not overlapping), one 16-byte element per
 * lane, used to calibrate achievable HBM bandwidth and
 * hardware byte counters.  Stream-ordered.  Errors: DM_ERR_ARG, DM_ERR_DEVICE.
 */
dm_status dm_copy_probe(void* dst, const void* src, size_t bytes, void* stream);

/*
 * Random-row probe: Out[perm[r]] += Z[perm[r]] for r = 0 .. n-1, with rows of
 * b FP32 values; the gather and read-modify-write of one coordinate pass of
 * Algorithm 2 in the fused form (the prefix sums left out), used to measure
 * the rate of the pass's random row accesses.  perm: device, n uint32 point
 * indices (a permutation gives the pass's pattern; entries >= n are skipped,
 * repeated entries race).  Z, Out: device n x b FP32 row-major, 16-byte
 * aligned, not overlapping.  b: a power of two, 4..64.  Stream-ordered.
 * Errors: DM_ERR_ARG, DM_ERR_DEVICE.
 */
dm_status dm_gather_probe(const uint32_t* perm, const float* Z, float* Out, int64_t n, int32_t b, void* stream);

/* Release a handle (and its workspace if the library allocated it).  NULL is a no-op. */
void dm_free(dm_handle* h);

#ifdef __cplusplus
}
#endif

#endif /* DM_H */
