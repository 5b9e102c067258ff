// dm_internal.h - host-side declarations shared by the C-ABI layer and the
// kernel translation units.  Not part of the public interface.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace dm {

// element kinds of the point data as seen by the kernels
enum InKind { IN_F32 = 1, IN_F64 = 2, IN_I32 = 3, IN_I64 = 4 };

// prep flags written by the device
// FLAG_DOMAIN: a coordinate outside the metric's domain (KL divergence and
// cross entropy take logarithms and need every coordinate finite and > 0)
enum PrepFlag : uint32_t { FLAG_NONFINITE = 1u, FLAG_INT_RANGE = 2u, FLAG_DOMAIN = 4u };

// sticky query status bits (device side)
// QF_STALL: a chained scan waited too long for a predecessor's record (a
// library fault, not a data error); the query's result is then invalid
enum QueryFlag : uint32_t { QF_NONFINITE = 1u, QF_OVERFLOW = 2u, QF_STALL = 4u };

constexpr int SORT_TILE = 4096;   // keys per sort tile (256 threads x 16)
constexpr int SORT_THREADS = 256;

// Ticket counters of the chained-scan passes, one per tile shape.  A pass of
// a shape with T tiles on a grid of G persistent workgroups consumes exactly
// T + G tickets (each workgroup stops on the first ticket past the last tile),
// so ticket / (T + G) numbers the passes of that shape and, with the shape,
// forms the tag of every word the pass publishes.  Zeroed once when a handle
// is created and never reset; the host never reads them.
constexpr int L1_VARIANTS = 4;      // tile variants per l1 pass configuration (tuned per handle)
constexpr int L1_CLASSES = 96;      // 3 data paths x 8 block widths x L1_VARIANTS
constexpr int LP_CLASSES = 48;      // odd p: 3 data paths x 8 block widths x (p = 3, 5)
constexpr int SINGLE_CLASSES = 12;  // single-column OUT_FRESH passes: 3 data paths x L1_VARIANTS
constexpr int CHAIN_CLASSES = L1_CLASSES + LP_CLASSES + SINGLE_CLASSES;
struct ChainState {
    uint64_t ticket[CHAIN_CLASSES];
};

// Segment tables of a segmented sort: segment s holds keys
// [key_off[s], key_off[s] + key_len[s]) and tiles [tile_off[s], tile_off[s+1]).
struct SegTables {
    const int64_t* key_off;    // S
    const int64_t* key_len;    // S
    const uint32_t* tile_off;  // S + 1
    const uint32_t* tile_seg;  // T
    const uint8_t* seg_int;    // S (integer keys?) or NULL: all segments of one kind
    const float* centre;       // S: subtracted from the sorted float values of a segment, or NULL
    int32_t nseg;
    uint32_t ntiles;
};

// ---- preparation ----------------------------------------------------------
hipError_t launch_prep_transpose(int kind, const void* X, int64_t n, int32_t d,
                                 uint32_t* keys /* d rows of stride ld, or NULL */, int64_t ld,
                                 void* xcopy /* n x d (4-byte) or NULL */,
                                 uint32_t* kmin, uint32_t* kmax, uint32_t* flags,
                                 hipStream_t s);
// row sums of x~^p and squared norms of x~ (x~ = x - centre, float data with
// centre != NULL; x otherwise); with xcopy != NULL also the values x~ as an
// n x d FP32 (int32) copy
hipError_t launch_row_stats(int kind, const void* X, int64_t n, int32_t d,
                            void* rowsum /* n x 8B */, void* rownrm /* n x 8B */, hipStream_t s, int p = 1,
                            const float* centre = nullptr, void* xcopy = nullptr);
// centre[k] for float coordinates from their min/max keys: the FP32 midpoint
// when x - c is exact for the whole range, else 0
hipError_t launch_centre(const uint32_t* kmin, const uint32_t* kmax, int32_t d, float* centre, hipStream_t s);
// xs[k * pitch + r] += centre[k], r < n, k < d
hipError_t launch_add_centre(float* xs, int64_t n, int32_t d, int64_t pitch, const float* centre, hipStream_t s);
hipError_t launch_fill_u32(uint32_t* p, uint32_t v, size_t count, hipStream_t s);
hipError_t launch_copy_probe(void* dst, const void* src, size_t bytes, hipStream_t s);
hipError_t launch_gather_probe(const uint32_t* perm, const float* Z, float* Out, int64_t n, int32_t b,
                               hipStream_t s);

// ---- segmented radix sort (LSD, 4 passes of 8 bits) -----------------------
hipError_t launch_sort_count(const uint32_t* keys, uint32_t* counts, const SegTables& t, int shift,
                             hipStream_t s);
hipError_t launch_sort_scan(uint32_t* counts, const SegTables& t, hipStream_t s);
hipError_t launch_sort_scatter(const uint32_t* kin, const uint32_t* vin, uint32_t* kout, uint32_t* vout,
                               const uint32_t* offs, const SegTables& t, int shift, bool first, bool last,
                               bool is_int, hipStream_t s);
// rank[k * pitch + perm[k * ld + r]] = r for r < n, k < d (the inverse permutations)
hipError_t launch_rank_invert(const uint32_t* perm, int64_t ld, int64_t n, int32_t d, uint32_t* rank, int64_t pitch,
                              hipStream_t s);

// Workgroups of a persistent launch of `fn` on the current device: the
// smaller occupancy of fn and fn2 (two variants of one kernel shape, which
// must share a grid) times the device's compute units, at most ntiles.  The
// occupancy is cached per (device, kernel) under a lock, so concurrent callers
// with distinct handles and devices are safe.
int persistent_grid(const void* fn, const void* fn2, int64_t ntiles);

// The library's static device scratch (k_static.hip): STATIC_SCRATCH_BYTES
// per device, for dm_matvec_static.  *ptr = its address on the current device
// (looked up once per device).
constexpr size_t STATIC_SCRATCH_BYTES = (size_t)32 << 20;
hipError_t static_scratch(char** ptr);

// ---- l1 query --------------------------------------------------------------
// totals: T0[c] = sum_j z_jc, U[c] = sum_j w_j z_jc, |z_c|_1; with guards.
struct TotalsOut {
    void* T0;        // b x (double | int64)
    void* U;         // b x (double | int64)
    double* zl1;     // b
    void* partials;  // scratch
    uint32_t* status;
};
int totals_partial_blocks(int64_t n);
size_t totals_scratch_bytes(int64_t n, int32_t b);
hipError_t launch_totals(bool is_int, int zkind, const void* Z, int64_t n, int32_t b, const void* w,
                         double guard_scale, const TotalsOut& o, hipStream_t s);

// How a pass stores its values: add them into Out[perm[r]] (and, on the
// first pass, U), or write them to Out[perm[r]] without reading Out.
enum { OUT_ADD = 0, OUT_FRESH = 1 };
struct L1PassArgs {
    const uint32_t* perm;   // n (this coordinate)
    const void* xs;         // n (float | int32)
    int64_t n;
    const void* Z;          // n x b
    void* Out;              // n x b (float | int64)
    const void* T0;         // b
    const void* U;          // b (added when first)
    int first;
    ChainState* chain;
    uint64_t* records;      // the shape's own record region (l1_shape)
    size_t record_words;    // its size in 64-bit words; a launch that needs more is refused
    int cls;                // the shape's ticket class (l1_shape)
    int variant;            // tile variant, 0 .. L1_VARIANTS-1
    uint32_t* status;       // sticky query flags (QF_STALL on a stuck chain)
    int out_mode = OUT_ADD; // OUT_FRESH (b = 1 only): write the values, add no U
};
int l1_tile_ranks(int32_t b, bool is_int, int zkind, int variant);
size_t l1_record_words(int64_t n, int32_t b, bool is_int, int zkind, int variant);
// per data path (k_l1_f32.hip, k_l1_i32.hip, k_l1_i64.hip)
hipError_t launch_l1_pass_f32(const L1PassArgs& a, int32_t b, int variant, hipStream_t s);
hipError_t launch_l1_pass_i32(const L1PassArgs& a, int32_t b, int variant, hipStream_t s);
hipError_t launch_l1_pass_i64(const L1PassArgs& a, int32_t b, int variant, hipStream_t s);
int l1_tile_ranks_f32(int32_t b, int variant);
int l1_tile_ranks_i32(int32_t b, int variant);
int l1_tile_ranks_i64(int32_t b, int variant);
// kernel shape of a pass: its ticket class and the words of its record region
// (each shape owns its region, so no shape ever reads another's words)
struct L1Shape {
    int cls;
    size_t record_words;
};
L1Shape l1_shape(int64_t n, int32_t b, bool is_int, int zkind, int variant);
// the single-column OUT_FRESH pass (its own ticket class)
L1Shape l1_single_shape(int64_t n, bool is_int, int zkind, int variant);
// Out[i] = (first ? U : Out[i]) + sum_{k < g} Cs[k * ld + i], b = 1: the sum of
// a group of g passes written in point order (float data: FP64 sum rounded
// once per group; integers: wrapping int64)
hipError_t launch_l1_combine(bool is_int, int64_t ld, const void* Cs, int64_t n, int32_t g, bool first,
                             const void* U, void* Out, hipStream_t s);
// bytes of per-coordinate values per group of a single-column query
constexpr size_t SINGLE_GROUP_BYTES = (size_t)64 << 20;
hipError_t launch_l1_pass(bool is_int, int zkind, int32_t b, const L1PassArgs& a, hipStream_t s);

// ---- many datasets in one query --------------------------------------------
// Per-dataset descriptor read by the multi-dataset kernels; Z and Out are
// refreshed before every query (a captured host-to-device copy).
struct MultiDs {
    const uint32_t* perm;   // d x ld
    const void* xs;         // d x ld (float | int32)
    const void* rowsum;     // n (double | int64): weights of U
    const void* Z;          // n x b (float | int32)
    void* Out;              // n x b (float | int64)
    void* T0;               // b (double | int64)
    void* U;                // b (double | int64)
    int64_t n, ld;
    int32_t d, is_int;
    double guard;           // sum of coordinate ranges (integer overflow guard)
    int64_t tot_blk0;       // first totals block of this dataset
    int32_t tot_nblk, pad;
};
struct MultiTile {
    uint32_t ds;  // dataset
    uint32_t t;   // tile index inside the dataset's coordinate segment
};
// tile variants of the multi-dataset pass (ranks per slot R, R / 2, and 2 R for
// up to 8 columns or R / 4 beyond), chosen per handle and b by dm_tune_multi
constexpr int MULTI_VARIANTS = 3;
int multi_tile_ranks(int32_t b, bool is_int, int variant);
size_t multi_record_words(int64_t ntiles, int32_t b, bool is_int);
int multi_grid(int64_t ntiles, int32_t b, bool is_int, int variant);
int multi_totals_rows();
hipError_t launch_multi_totals(const MultiDs* ds, const uint32_t* blk_ds, int nblocks, int ndatasets, int32_t b,
                               double* partials, uint32_t* status, hipStream_t s);
// vec: 16-byte row accesses; needs b % 4 == 0 and 16-byte aligned Z and Out of every dataset
hipError_t launch_multi_pass(bool is_int, int32_t b, const MultiDs* ds, const MultiTile* tiles, int64_t ntiles,
                             int k, uint64_t* ticket, uint64_t* records, int grid, bool vec, uint32_t* status,
                             int variant, hipStream_t s);

// ---- block-Krylov low rank (k_lowrank.hip) ---------------------------------
int lr_max_block();
int lr_max_basis();
// scratch of lr_gram_blocks for up to nq_max blocks per call
size_t lr_gram_scratch_doubles(int64_t n, int ma, int mb, int nq_max);
// out[(i ma + p) * ldo + q] = scale * sum_r Q_i[r][p] Y[r][q] for i < nq, with
// Q_i = Q + i qstride (n x ma) and Y n x mb (Y may be Q when nq = 1);
// part: lr_gram_scratch_doubles doubles
hipError_t lr_gram_blocks(const double* Q, size_t qstride, int nq, int ma, const double* Y, int mb, int64_t n,
                          double* part, double* out, int ldo, double scale, hipStream_t s);
// Y = beta Y + alpha Q C; Y n x mb, Q n x ma, C ma x ldc (Y may be Q when beta is 0)
hipError_t lr_update_rows(double* Y, int mb, const double* Q, int ma, const double* C, int ldc, double alpha,
                          double beta, int64_t n, hipStream_t s);
// Y = beta Y + alpha sum_(i < nq) Q_i C_i with Q_i = Q + i qstride (n x ma) and
// C_i rows i ma .. of C (leading dimension ldc); Y must not be any Q_i unless nq = 1
hipError_t lr_update_blocks(double* Y, int mb, const double* Q, size_t qstride, int nq, int ma, const double* C,
                            int ldc, double alpha, double beta, int64_t n, hipStream_t s);
hipError_t lr_cholinv(const double* G, int m, double rel, double* X, uint32_t* status, hipStream_t s);
hipError_t lr_symm(double* T, int m, int bw, hipStream_t s);
// FP64 n x B block a <-> FP32 copy b held as two row-major arrays, columns
// 0 .. B1 - 1 (rows x B1) followed by columns B1 .. B - 1 (rows x (B - B1))
hipError_t lr_cvt(const double* a, float* b, int64_t rows, int B, int B1, hipStream_t s);
hipError_t lr_cvt(const float* b, double* a, int64_t rows, int B, int B1, hipStream_t s);
// eigen-decomposition of the symmetric m x m T (destroyed; T2 is a second
// m x m buffer): eigenvalues w (m) and eigenvectors as the rows of V (m x m);
// *sweeps = sweeps used (host value); synchronises s once per sweep
hipError_t lr_eig(double* T, double* T2, double* V, double* w, int m, int max_sweeps, double tol, int* d_done,
                  int* sweeps, hipStream_t s);
hipError_t lr_topk(const double* w, const double* V, int m, int k, double* lam, double* Vk, hipStream_t s);

// ---- l_p^p for odd p >= 3 (k_lp.hip) ---------------------------------------
struct LpPassArgs {
    const uint32_t* perm;   // n (this coordinate)
    const void* xs;         // n (float | int32)
    int64_t n;
    const void* Z;          // n x b
    void* Out;              // n x b (float | int64)
    const void* T0;         // b: sum of z
    const void* Mk;         // moments of this coordinate: Mk[(t - 1) * mstride + c], t = 1 .. p-1
    int64_t mstride;
    const void* U;          // b: sum_j w_j z_j, w_j = sum_k x_jk^p (added when first)
    int first;
    ChainState* chain;
    int cls;                // ticket class (L1_CLASSES + ...)
    uint64_t* records;
    size_t record_words;
    uint32_t* status;       // sticky query flags (QF_STALL on a stuck chain)
};
int lp_tile_ranks(int32_t b, int p);
size_t lp_record_words(int64_t n, int32_t b, bool is_int, int p);
size_t lp_moments_bytes(int64_t n, int32_t d, int32_t b, int p);
// M[t - 1][k][c] = sum_j z_jc x_jk^t (t = 1 .. p-1) from the point copy Xc;
// *M is set inside scratch (lp_moments_bytes)
hipError_t launch_lp_moments(bool is_int, int zkind, int p, const void* Xc, const void* Z, int64_t n, int32_t d,
                             int32_t b, void* scratch, void** M, hipStream_t s);
hipError_t launch_lp_pass(bool is_int, int zkind, int p, int32_t b, const LpPassArgs& a, hipStream_t s);

// ---- Gaussian embedding for approximate l2 queries (k_embed.hip) -----------
// Xout (n x k FP32) = (1 / (beta k)) X G^T, beta = sqrt(2/pi); kind: InKind of X
// p[i] *= s for i < count
hipError_t launch_scale_f32(float* p, size_t count, float s, hipStream_t st);
hipError_t launch_embed_l2(int kind, const void* X, int64_t n, int32_t d, const double* G, int32_t k, float* Xout,
                           hipStream_t s);

// ---- the sort-free family (k_sortfree.hip) ---------------------------------
// SF_EVEN: l_p^p for even p; SF_LOG: moments of log x (KL, cross entropy);
// SF_LIN: moments of the centred coordinates mixed by a d x d matrix
enum SfForm { SF_EVEN = 1, SF_LOG = 2, SF_LIN = 3 };
struct SfQuery {
    const void* X;          // n x d point copy (float | int32)
    const double* LX;       // n x d logarithms of X (SF_LOG) or NULL
    const void* centre;     // d (double | int64) subtracted from every coordinate, or NULL
    const void* Z;          // n x b (float | int32 | int64)
    int64_t n;
    int32_t d, b;
    const void* T0;         // b (double | int64): sum_j z_j
    const double* U;        // b, added to every row, or NULL
    const double* a;        // n: a_i T0 added to row i, or NULL
    const double* W;        // d x d applied to the moments, or NULL
    double alpha;           // scale of the moments when W is NULL
    void* Out;              // n x b (float | int64)
    // Totals formed by the query itself (when sf_fuses_totals holds): the
    // moments kernel also sums z and w z from its loads; T0 and U above are
    // then ignored, and a non-finite z raises QF_NONFINITE in *status.
    uint32_t* status = nullptr;   // NULL: T0 (and U) are given
    const double* wu = nullptr;   // n weights w of U = sum_j w_j z_j, or NULL (no U)
};
// whether launch_sf_query forms the totals itself for this shape (the
// matrix-core moments of float data: 4 <= b <= 16, or even b <= 32 with Z
// 8-byte aligned, or b % 4 == 0 with Z 16-byte aligned; the single-moment
// forms need d % 4 == 0, even p needs b >= 8)
bool sf_fuses_totals(int form, bool is_int, int32_t d, int32_t b, const void* Z);
int sf_moment_count(int form, int p);
size_t sf_scratch_bytes(int64_t n, int32_t d, int32_t b, int form, int p);
hipError_t launch_sf_query(int form, int p, bool is_int, int zkind, const SfQuery& q, void* scratch, hipStream_t s);
// negH[i] = sum_k x_ik log x_ik, LX (n x d) = log X; sets `bad` in *flags for a
// coordinate that is not finite and > 0
hipError_t launch_kl_weights(const float* X, int64_t n, int32_t d, double* negH, double* LX, uint32_t* flags,
                             uint32_t bad, hipStream_t s);
// q[i] = (x_i - c)^T M (x_i - c)
hipError_t launch_maha_weights(const float* X, const double* centre, int64_t n, int32_t d, const double* M, double* q,
                               hipStream_t s);

// ---- l2 squared query ------------------------------------------------------
size_t l2_scratch_bytes(int64_t n, int32_t d, int32_t b);
size_t l2_mfma_scratch_bytes(int64_t n, int32_t d, int32_t b);
hipError_t launch_l2sq(bool is_int, int zkind, const void* Xc, const void* nrm, int64_t n, int32_t d,
                       const void* Z, int32_t b, void* Out, void* scratch, const TotalsOut& tot,
                       double guard_scale, hipStream_t s);

}  // namespace dm
