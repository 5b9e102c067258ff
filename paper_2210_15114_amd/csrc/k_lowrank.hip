// k_lowrank.hip - FP64 building blocks of the block-Krylov low-rank
// approximation (Appendix C.1: the top singular values, and with them a
// rank-k approximation, from matrix-vector queries only).
//
// The products with A run through the l1 / l2-squared query; everything
// here works on tall, skinny FP64 blocks (n x m with m <= 64) and on the
// small projected matrix T = Q^T A Q:
//   * lr_gram_mfma / lr_reduce - C_i = Q_i^T Y for several n x m blocks Q_i
//     against one block Y in one call, on FP64 matrix cores, split over rows
//     into fixed partial sums and reduced in a fixed order (bit-reproducible
//     run to run);
//   * lr_update   - Y = beta Y + alpha sum_i Q_i C_i, row by row on FP64 matrix
//     cores (block Gram-Schmidt updates, Y R^-1 of Cholesky QR, U = Q V);
//   * lr_chol     - the orthonormalising factor of Cholesky QR for a small
//     Gram matrix (column-equilibrated), dropping dependent columns;
//   * lr_jacobi_step - eigenvalues and eigenvectors of the symmetric T by the
//     cyclic Jacobi method with the round-robin pair ordering (all pairs of
//     one step are disjoint, so their rotations are applied together);
//   * lr_select   - the k eigenpairs of largest |lambda|.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "dm_internal.h"

namespace dm {
namespace {

constexpr int GT = 64;     // rows per LDS tile
constexpr int MAXM = 64;   // widest block

// ---------------------------------------------------------------------------
// part[blk][i][p][q] = sum over the rows r of range blk of Q_i[r][p] * Y[r][q]
// for the nq blocks Q_i = Q + i qstride (n x ma, row-major) against one
// n x mb block Y, on FP64 matrix cores.  One wave per (range, i): operands
// are loaded straight into the v_mfma_f64_16x16x4f64 lane layout (A lane l
// holds A[l % 16][l / 16], here Q_i[r + l / 16][16 pt + l % 16]; B lane l
// holds B[l / 16][l % 16], here Y[r + l / 16][16 qt + l % 16]; D lane l,
// element e holds D[4e + l / 16][l % 16]), four rows per product and 16 rows
// per step, so a row of Q_i and of Y is read once by the wave.  Workgroup
// ids go round-robin over the 8 XCDs; ids are decoded so that the nq waves of
// one range sit on the same XCD and start together, and Y's rows are read
// from HBM about once per call and then from that XCD's L2.  The sum over a
// range runs in row order, so the partials, and the fixed-order reduction
// after them, are the same run to run.
// ---------------------------------------------------------------------------
typedef double d4v __attribute__((ext_vector_type(4)));

constexpr int GRAM_PARTS = 4096;   // (range, i) waves per call, at most
constexpr int GRAM_STEP = 16;      // rows per step (four products)

__global__ __launch_bounds__(64) void lr_gram_mfma(const double* __restrict__ Q, size_t qstride, int nq, int ma,
                                                   const double* __restrict__ Y, int mb, int64_t n, int64_t rw,
                                                   int64_t nblk, double* __restrict__ part)
{
    const int id = blockIdx.x;
    const int xcd = id & 7;
    const int slot = id >> 3;
    const int i = slot % nq;
    const int64_t blk = (int64_t)(slot / nq) * 8 + xcd;
    if (blk >= nblk) return;   // the whole wave
    const int lane = threadIdx.x, m = lane & 15, g = lane >> 4;
    const double* __restrict__ A = Q + (size_t)i * qstride;
    const int pt_n = (ma + 15) / 16, qt_n = (mb + 15) / 16;
    d4v acc[MAXM / 16][MAXM / 16];
#pragma unroll
    for (int pt = 0; pt < MAXM / 16; ++pt)
#pragma unroll
        for (int qt = 0; qt < MAXM / 16; ++qt) acc[pt][qt] = d4v{0.0, 0.0, 0.0, 0.0};
    const int64_t r0 = blk * rw;
    const int64_t r1 = r0 + rw < n ? r0 + rw : n;
    for (int64_t r = r0; r < r1; r += GRAM_STEP) {
        double a[GRAM_STEP / 4][MAXM / 16], y[GRAM_STEP / 4][MAXM / 16];
#pragma unroll
        for (int u = 0; u < GRAM_STEP / 4; ++u) {
            const int64_t row = r + 4 * u + g;
            const bool rv = row < r1;
#pragma unroll
            for (int t = 0; t < MAXM / 16; ++t) {
                const int c = 16 * t + m;
                a[u][t] = (t < pt_n && rv && c < ma) ? A[row * ma + c] : 0.0;
                y[u][t] = (t < qt_n && rv && c < mb) ? Y[row * mb + c] : 0.0;
            }
        }
#pragma unroll
        for (int u = 0; u < GRAM_STEP / 4; ++u)
#pragma unroll
            for (int pt = 0; pt < MAXM / 16; ++pt)
#pragma unroll
                for (int qt = 0; qt < MAXM / 16; ++qt)
                    if (pt < pt_n && qt < qt_n)   // the same on every lane
                        acc[pt][qt] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u][pt], y[u][qt], acc[pt][qt], 0, 0, 0);
    }
    double* out = part + ((size_t)blk * nq + i) * ma * mb;
#pragma unroll
    for (int pt = 0; pt < MAXM / 16; ++pt)
#pragma unroll
        for (int qt = 0; qt < MAXM / 16; ++qt) {
            if (pt >= pt_n || qt >= qt_n) continue;
            const int q = 16 * qt + m;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int p = 16 * pt + 4 * e + g;
                if (p < ma && q < mb) out[p * mb + q] = acc[pt][qt][e];
            }
        }
}

// out[p * ldo + q] = scale * sum_blk part[blk][p][q].  A workgroup owns
// RED_E entries; its RED_G thread groups add blocks g, g + RED_G, ... in
// order (four loads in flight), and the group sums are then added in group
// order, so the order is fixed.
constexpr int RED_E = 4, RED_G = 64;

__global__ __launch_bounds__(256) void lr_reduce(const double* __restrict__ part, int nblk, int ma, int mb,
                                                 double* __restrict__ out, int ldo, double scale)
{
    __shared__ double red[RED_G][RED_E];
    const int t = threadIdx.x % RED_E, g = threadIdx.x / RED_E;
    const int e = blockIdx.x * RED_E + t;
    const int cnt = ma * mb;
    double s = 0.0;
    if (e < cnt) {
        int k = g;
        for (; k + 3 * RED_G < nblk; k += 4 * RED_G) {
            const double v0 = part[(size_t)k * cnt + e];
            const double v1 = part[(size_t)(k + RED_G) * cnt + e];
            const double v2 = part[(size_t)(k + 2 * RED_G) * cnt + e];
            const double v3 = part[(size_t)(k + 3 * RED_G) * cnt + e];
            s += v0;
            s += v1;
            s += v2;
            s += v3;
        }
        for (; k < nblk; k += RED_G) s += part[(size_t)k * cnt + e];
    }
    red[g][t] = s;
    __syncthreads();
    if (g == 0 && e < cnt) {
        double v = red[0][t];
        for (int gg = 1; gg < RED_G; ++gg) v += red[gg][t];
        out[(size_t)(e / mb) * ldo + (e % mb)] = scale * v;
    }
}

// ---------------------------------------------------------------------------
// Y = beta Y + alpha sum_(i < nq) Q_i C_i, row by row, on FP64 matrix cores.
// Y is n x mb (leading dimension mb); Q_i = Q + i qstride is n x ma
// row-major; C_i is rows i ma .. i ma + ma - 1 of C (leading dimension ldc).
// A workgroup takes GT rows at a time; for each i it stages the Q_i rows
// (a flat, coalesced copy) and alpha C_i in LDS, and wave w multiplies rows
// 16w .. 16w + 15 by every column with v_mfma_f64_16x16x4f64 (gfx950 lane
// layout: A lane l holds A[l % 16][l / 16], B lane l holds B[l / 16][l % 16],
// D lane l element r holds D[4r + l / 16][l % 16]).  A tile's Q rows are all
// read before its Y rows are written, so Y may be Q when nq = 1 and beta = 0
// (in-place right multiplication).  One call with nq blocks moves Y once,
// where nq single-block calls would move it nq times.
// ---------------------------------------------------------------------------
template <int QPT>
__global__ __launch_bounds__(256) void lr_update(double* Y, int mb, const double* Q, size_t qstride, int nq, int ma,
                                                 const double* __restrict__ C, int ldc, double alpha, double beta,
                                                 int64_t n)
{
    extern __shared__ double lds[];
    const int lq = ma + 1;   // row stride of the Q tile
    double* sQ = lds;        // GT x lq
    double* sC = lds + GT * lq;   // ma x mb
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int m = lane & 15, g = lane >> 4;
    const int ct_n = (mb + 15) / 16;
    // The workgroup's (tile, block) steps in order: tiles blockIdx.x,
    // + gridDim.x, ..., and for each tile the blocks i = 0 .. nq - 1.  The
    // next step's Q rows (QPT doubles per thread, QPT >= GT ma / 256) are
    // loaded into registers while the current step multiplies out of LDS.
    // alpha C_i is staged from L2 at each step, or once when nq = 1.
    const int64_t ntile = (n + GT - 1) / GT;
    const int64_t mine = (int64_t)blockIdx.x < ntile ? (ntile - 1 - blockIdx.x) / gridDim.x + 1 : 0;
    const int64_t steps = mine * nq;
    double rq[QPT];
    auto fetch = [&](int64_t it) {
        const int64_t r0 = ((int64_t)blockIdx.x + (it / nq) * gridDim.x) * GT;
        const int i = (int)(it % nq);
        const int nr = (int)(n - r0 < GT ? n - r0 : GT);
        const double* q0 = Q + (size_t)i * qstride + r0 * ma;
#pragma unroll
        for (int k = 0; k < QPT; ++k) {
            const int e = tid + 256 * k;
            rq[k] = e < nr * ma ? q0[e] : 0.0;
        }
    };
    d4v acc[MAXM / 16];
    if (steps > 0) fetch(0);
    for (int64_t it = 0; it < steps; ++it) {   // uniform
        const int i = (int)(it % nq);
        const int64_t r0 = ((int64_t)blockIdx.x + (it / nq) * gridDim.x) * GT;
        if (i == 0) {
#pragma unroll
            for (int u = 0; u < MAXM / 16; ++u) acc[u] = d4v{0.0, 0.0, 0.0, 0.0};
        }
        __syncthreads();   // the previous step's tiles are no longer read
#pragma unroll
        for (int k = 0; k < QPT; ++k) {
            const int e = tid + 256 * k;
            if (e < GT * ma) sQ[(e / ma) * lq + (e % ma)] = rq[k];
        }
        if (nq > 1 || it == 0)
            for (int e = tid; e < ma * mb; e += 256) sC[e] = alpha * C[(size_t)(i * ma + e / mb) * ldc + (e % mb)];
        __syncthreads();
        if (it + 1 < steps) fetch(it + 1);
        for (int k0 = 0; k0 < ma; k0 += 4) {
            const int kk = k0 + g;
            const double av = kk < ma ? sQ[(16 * w + m) * lq + kk] : 0.0;
#pragma unroll
            for (int u = 0; u < MAXM / 16; ++u) {
                if (u < ct_n) {   // the same on every lane
                    const int c = 16 * u + m;
                    const double bv = (kk < ma && c < mb) ? sC[kk * mb + c] : 0.0;
                    acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[u], 0, 0, 0);
                }
            }
        }
        if (i == nq - 1) {
#pragma unroll
            for (int u = 0; u < MAXM / 16; ++u) {
                const int c = 16 * u + m;
                if (u >= ct_n || c >= mb) continue;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int64_t row = r0 + 16 * w + 4 * r + g;
                    if (row >= n) continue;
                    double* y = Y + row * mb + c;
                    *y = beta == 0.0 ? acc[u][r] : fma(beta, *y, acc[u][r]);
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// X with Y X orthonormal, for the m x m Gram matrix G = Y^T Y (one wave).
// The columns are first scaled to unit norm (D = diag(G)^-1/2, which keeps
// the factorisation accurate when column norms differ by orders of
// magnitude), then D G D = R^T R by Cholesky and X = D R^-1.  A column whose
// remaining pivot is at most rel (it lies in the span of the earlier columns
// to relative accuracy sqrt(rel)), or whose norm is zero, is dropped: its
// rows and columns of R and X are zero, so Y X has a zero column there.  X is
// written m x m.  Non-finite input sets QF_NONFINITE in *status and X = 0.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void lr_chol(const double* __restrict__ G, int m, double rel,
                                              double* __restrict__ X, uint32_t* __restrict__ status)
{
    __shared__ double sG[MAXM][MAXM + 1];
    __shared__ double sR[MAXM][MAXM + 1];
    __shared__ double dsc[MAXM];
    __shared__ int live[MAXM];
    const int l = threadIdx.x;
    bool bad = false;
    if (l < m) {
        const double g = G[l * m + l];
        if (!std::isfinite(g)) bad = true;
        dsc[l] = g > 0.0 && std::isfinite(g) ? 1.0 / sqrt(g) : 0.0;
    }
    __syncthreads();
    for (int i = 0; i < m; ++i) {
        if (l < m) {
            const double v = G[i * m + l];
            if (!std::isfinite(v)) bad = true;
            sG[i][l] = v * dsc[i] * dsc[l];
            sR[i][l] = 0.0;
        }
    }
    if (__any(bad)) {
        if (l == 0) atomicOr(status, (uint32_t)QF_NONFINITE);
        for (int i = 0; i < m; ++i)
            if (l < m) X[i * m + l] = 0.0;
        return;
    }
    __syncthreads();
    for (int j = 0; j < m; ++j) {
        const double d = sG[j][j];
        const bool ok = dsc[j] > 0.0 && d > rel;
        const double rjj = ok ? sqrt(d) : 0.0;
        if (l == 0) live[j] = ok ? 1 : 0;
        if (l < m && l > j) sR[j][l] = ok ? sG[j][l] / rjj : 0.0;
        if (l == j) sR[j][j] = rjj;
        __syncthreads();
        if (l < m && l > j && ok) {
            const double rl = sR[j][l];
            for (int k = j + 1; k < m; ++k) sG[k][l] -= sR[j][k] * rl;
        }
        __syncthreads();
    }
    // R^-1 on the live indices: lane c solves R x = e_c from the bottom up,
    // keeping x in column c of sG (the factorisation no longer needs it);
    // then X = D R^-1
    if (l < m) {
        const int c = l;
        for (int i = 0; i < m; ++i) sG[i][c] = 0.0;
        if (live[c]) {
            sG[c][c] = 1.0 / sR[c][c];
            for (int i = c - 1; i >= 0; --i) {
                if (!live[i]) continue;
                double s = 0.0;
                for (int k = i + 1; k <= c; ++k) s += sR[i][k] * sG[k][c];
                sG[i][c] = -s / sR[i][i];
            }
        }
        for (int i = 0; i < m; ++i) X[i * m + c] = dsc[i] * sG[i][c];
    }
}

// ---------------------------------------------------------------------------
// T[p][q] for p > q: the mirror of T[q][p]; diagonal blocks of width bw
// (both halves computed) are averaged instead.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void lr_symmetrize(double* __restrict__ T, int m, int bw)
{
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= m * m) return;
    const int p = e / m, q = e % m;
    if (p <= q) return;
    if (p / bw == q / bw) {
        const double a = 0.5 * (T[p * m + q] + T[q * m + p]);
        T[p * m + q] = a;
        T[q * m + p] = a;
    } else {
        T[p * m + q] = T[q * m + p];
    }
}

// The FP32 copy of an n x B FP64 block is kept as two row-major arrays, the
// first B1 columns (n x B1) and then the other B - B1 (n x (B - B1)), so that
// each can be queried with rows that fill whole cache lines (B1 = B: one
// array).  Element (r, c) of the block sits at split_index in the copy.
__device__ __forceinline__ size_t split_index(size_t i, int64_t rows, int B, int B1) {
    const size_t r = i / (size_t)B;
    const int c = (int)(i - r * (size_t)B);
    return c < B1 ? r * (size_t)B1 + c : (size_t)rows * B1 + r * (size_t)(B - B1) + (c - B1);
}
__global__ __launch_bounds__(256) void lr_cvt_f64_f32(const double* __restrict__ a, float* __restrict__ b,
                                                      int64_t rows, int B, int B1)
{
    const size_t n = (size_t)rows * B;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256)
        b[split_index(i, rows, B, B1)] = (float)a[i];
}
__global__ __launch_bounds__(256) void lr_cvt_f32_f64(const float* __restrict__ b, double* __restrict__ a,
                                                      int64_t rows, int B, int B1)
{
    const size_t n = (size_t)rows * B;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256)
        a[i] = (double)b[split_index(i, rows, B, B1)];
}

// ---------------------------------------------------------------------------
// Cyclic Jacobi on the symmetric m x m matrix T, one launch per step.
// Step s pairs index 0 with (s mod (m'-1)) + 1 and the other indices around
// a circle (m' = m rounded up to even; a pair with the padding index m is
// left alone), so the m'/2 pairs of a step are disjoint and their rotations
// commute: T' = J^T T J changes each 2 x 2 block (rows of pair i, columns of
// pair j) independently, T'_ij = J_i^T T_ij J_j.  Each rotation is the one
// of the classical Jacobi method that zeroes T[p][q] (Golub and Van Loan,
// symmetric Schur decomposition of a 2 x 2 block).  T is read from Tin and
// written to Tout (every entry, every step), so each workgroup can take all
// rotation angles from Tin while the others write; V accumulates V J in
// place (workgroup j owns columns p_j and q_j).
// ---------------------------------------------------------------------------
constexpr int JMAX = 1024;   // largest m

__device__ __forceinline__ void jacobi_pair(int i, int s, int mp, int& p, int& q) {
    auto pos = [&](int j) { return j == 0 ? 0 : 1 + (j - 1 + s) % (mp - 1); };
    p = pos(i);
    q = pos(mp - 1 - i);
    if (p > q) {
        const int t = p;
        p = q;
        q = t;
    }
}

__global__ __launch_bounds__(256) void lr_jacobi_step(const double* __restrict__ Tin, double* __restrict__ Tout,
                                                      double* __restrict__ V, int m, int s)
{
    __shared__ int sp[JMAX / 2], sq[JMAX / 2];
    __shared__ double sc[JMAX / 2], ss[JMAX / 2];
    const int tid = threadIdx.x;
    const int mp = (m + 1) & ~1;
    const int half = mp / 2;
    for (int i = tid; i < half; i += 256) {
        int p, q;
        jacobi_pair(i, s, mp, p, q);
        double c = 1.0, sn = 0.0;
        if (q < m) {
            const double apq = Tin[p * m + q];
            if (apq != 0.0) {
                const double app = Tin[p * m + p], aqq = Tin[q * m + q];
                const double th = (aqq - app) / (2.0 * apq);
                const double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
                c = 1.0 / sqrt(t * t + 1.0);
                sn = t * c;
            }
        }
        sp[i] = p;
        sq[i] = q;   // q == m marks the padding index
        sc[i] = c;
        ss[i] = sn;
    }
    __syncthreads();
    const int j = blockIdx.x;
    const int pj = sp[j], qj = sq[j];
    const double cj = sc[j], sj = ss[j];
    const bool qv = qj < m;
    // T is symmetric (to rounding), so the block of rows (pi, qi) and columns
    // (pj, qj) is read from, and its rotated values written to, rows pj and qj:
    // a workgroup touches only its own two rows
    for (int i = tid; i < half; i += 256) {
        const int pi = sp[i], qi = sq[i];
        const double ci = sc[i], si = ss[i];
        const bool rv = qi < m;
        // the block [[a, b], [c, d]] = rows (pi, qi) x columns (pj, qj)
        double a = Tin[pj * m + pi];
        double b = qv ? Tin[qj * m + pi] : 0.0;
        double c = rv ? Tin[pj * m + qi] : 0.0;
        double d = (rv && qv) ? Tin[qj * m + qi] : 0.0;
        // rows: J_i^T
        const double a1 = ci * a - si * c, c1 = si * a + ci * c;
        const double b1 = ci * b - si * d, d1 = si * b + ci * d;
        // columns: J_j
        a = cj * a1 - sj * b1;
        b = sj * a1 + cj * b1;
        c = cj * c1 - sj * d1;
        d = sj * c1 + cj * d1;
        Tout[pj * m + pi] = a;
        if (qv) Tout[qj * m + pi] = b;
        if (rv) Tout[pj * m + qi] = c;
        if (rv && qv) Tout[qj * m + qi] = d;
    }
    // V is kept transposed (row j is eigenvector j): rotate rows pj and qj
    if (qv) {
        for (int r = tid; r < m; r += 256) {
            const double va = V[pj * m + r], vb = V[qj * m + r];
            V[pj * m + r] = cj * va - sj * vb;
            V[qj * m + r] = sj * va + cj * vb;
        }
    }
}

// V = I
__global__ __launch_bounds__(256) void lr_identity(double* __restrict__ V, int m)
{
    for (int i = blockIdx.x * 256 + threadIdx.x; i < m * m; i += gridDim.x * 256) V[i] = (i / m == i % m) ? 1.0 : 0.0;
}

// *done = 1 when the off-diagonal mass of T is at most tol^2 times the total;
// w[i] = T[i][i]
__global__ __launch_bounds__(1024) void lr_jacobi_check(const double* __restrict__ T, int m, double tol,
                                                        int* __restrict__ done, double* __restrict__ w)
{
    __shared__ double red[2][1024];
    const int tid = threadIdx.x;
    double off = 0.0, tot = 0.0;
    for (int i = tid; i < m * m; i += 1024) {
        const double v = T[i];
        tot += v * v;
        if (i / m != i % m) off += v * v;
    }
    red[0][tid] = off;
    red[1][tid] = tot;
    __syncthreads();
    for (int st = 512; st > 0; st >>= 1) {
        if (tid < st) {
            red[0][tid] += red[0][tid + st];
            red[1][tid] += red[1][tid + st];
        }
        __syncthreads();
    }
    if (tid == 0) *done = red[0][0] <= tol * tol * red[1][0] ? 1 : 0;
    for (int i = tid; i < m; i += 1024) w[i] = T[i * m + i];
}

// The k eigenpairs of largest |lambda|, in decreasing |lambda| (ties by lower
// index): index i takes place #{j : |w_j| > |w_i|, or equal with j < i}.
__global__ __launch_bounds__(1024) void lr_select(const double* __restrict__ w, const double* __restrict__ V, int m,
                                                  int k, double* __restrict__ lam, double* __restrict__ Vk)
{
    __shared__ int sidx[MAXM];
    for (int i = threadIdx.x; i < m; i += 1024) {
        const double ai = fabs(w[i]);
        int r = 0;
        for (int j = 0; j < m; ++j) {
            const double aj = fabs(w[j]);
            r += (aj > ai || (aj == ai && j < i)) ? 1 : 0;
        }
        if (r < k) {
            sidx[r] = i;
            lam[r] = w[i];
        }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < m * k; e += 1024) {
        const int r = e / k, t = e % k;
        Vk[e] = V[sidx[t] * m + r];   // V holds the eigenvectors as rows
    }
}

}  // namespace

int lr_max_block() { return MAXM; }
int lr_max_basis() { return JMAX; }

// rows per range of lr_gram_blocks: at most GRAM_PARTS (range, block) waves,
// at least 64 rows each, a multiple of the step
static int64_t gram_rows(int64_t n, int nq) {
    const int64_t per = GRAM_PARTS / nq > 0 ? GRAM_PARTS / nq : 1;
    int64_t rw = (n + per - 1) / per;
    if (rw < 64) rw = 64;
    return (rw + GRAM_STEP - 1) / GRAM_STEP * GRAM_STEP;
}

size_t lr_gram_scratch_doubles(int64_t n, int ma, int mb, int nq_max) {
    size_t most = 0;
    for (int nq = 1; nq <= nq_max; ++nq) {
        const int64_t rw = gram_rows(n, nq);
        const size_t c = (size_t)((n + rw - 1) / rw) * nq;
        if (c > most) most = c;
    }
    return most * ma * mb;
}

hipError_t lr_gram_blocks(const double* Q, size_t qstride, int nq, int ma, const double* Y, int mb, int64_t n,
                          double* part, double* out, int ldo, double scale, hipStream_t s)
{
    if (ma < 1 || mb < 1 || ma > MAXM || mb > MAXM || n < 1 || nq < 1) return hipErrorInvalidValue;
    const int64_t rw = gram_rows(n, nq);
    const int64_t nblk = (n + rw - 1) / rw;
    const int64_t grid = (nblk + 7) / 8 * 8 * nq;
    if (grid > 0x7fffffff) return hipErrorInvalidValue;
    lr_gram_mfma<<<(unsigned)grid, 64, 0, s>>>(Q, qstride, nq, ma, Y, mb, n, rw, nblk, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int cnt = nq * ma * mb;
    lr_reduce<<<(cnt + RED_E - 1) / RED_E, 256, 0, s>>>(part, (int)nblk, nq * ma, mb, out, ldo, scale);
    return hipGetLastError();
}

hipError_t lr_update_blocks(double* Y, int mb, const double* Q, size_t qstride, int nq, int ma, const double* C,
                            int ldc, double alpha, double beta, int64_t n, hipStream_t s)
{
    if (ma < 1 || mb < 1 || ma > MAXM || mb > MAXM || n < 1 || nq < 1) return hipErrorInvalidValue;
    const size_t lds = ((size_t)GT * (ma + 1) + (size_t)ma * mb) * sizeof(double);
    int64_t blocks = (n + GT - 1) / GT;
    if (blocks > 2048) blocks = 2048;
    // registers for the prefetched Q rows: 10 per thread up to 40 columns
    if (GT * ma <= 256 * 10)
        lr_update<10><<<(unsigned)blocks, 256, lds, s>>>(Y, mb, Q, qstride, nq, ma, C, ldc, alpha, beta, n);
    else
        lr_update<GT * MAXM / 256><<<(unsigned)blocks, 256, lds, s>>>(Y, mb, Q, qstride, nq, ma, C, ldc, alpha, beta, n);
    return hipGetLastError();
}

hipError_t lr_update_rows(double* Y, int mb, const double* Q, int ma, const double* C, int ldc, double alpha,
                          double beta, int64_t n, hipStream_t s)
{
    return lr_update_blocks(Y, mb, Q, 0, 1, ma, C, ldc, alpha, beta, n, s);
}

hipError_t lr_cholinv(const double* G, int m, double rel, double* X, uint32_t* status, hipStream_t s)
{
    if (m < 1 || m > MAXM) return hipErrorInvalidValue;
    lr_chol<<<1, 64, 0, s>>>(G, m, rel, X, status);
    return hipGetLastError();
}

hipError_t lr_symm(double* T, int m, int bw, hipStream_t s)
{
    lr_symmetrize<<<(m * m + 255) / 256, 256, 0, s>>>(T, m, bw);
    return hipGetLastError();
}

hipError_t lr_cvt(const double* a, float* b, int64_t rows, int B, int B1, hipStream_t s)
{
    size_t blocks = ((size_t)rows * B + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    lr_cvt_f64_f32<<<(unsigned)blocks, 256, 0, s>>>(a, b, rows, B, B1);
    return hipGetLastError();
}
hipError_t lr_cvt(const float* b, double* a, int64_t rows, int B, int B1, hipStream_t s)
{
    size_t blocks = ((size_t)rows * B + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    lr_cvt_f32_f64<<<(unsigned)blocks, 256, 0, s>>>(b, a, rows, B, B1);
    return hipGetLastError();
}

hipError_t lr_eig(double* T, double* T2, double* V, double* w, int m, int max_sweeps, double tol, int* d_done,
                  int* sweeps, hipStream_t s)
{
    if (m < 1 || m > JMAX) return hipErrorInvalidValue;
    lr_identity<<<(m * m + 255) / 256 < 4096 ? (m * m + 255) / 256 : 4096, 256, 0, s>>>(V, m);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int mp = (m + 1) & ~1;
    double* cur = T;
    double* nxt = T2;
    int sweep = 0;
    for (; sweep <= max_sweeps; ++sweep) {
        lr_jacobi_check<<<1, 1024, 0, s>>>(cur, m, tol, d_done, w);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        int done = 0;
        if ((e = hipMemcpyAsync(&done, d_done, sizeof(int), hipMemcpyDeviceToHost, s)) != hipSuccess) return e;
        if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
        if (done || sweep == max_sweeps || mp < 2) break;
        for (int st = 0; st < mp - 1; ++st) {
            lr_jacobi_step<<<mp / 2, 256, 0, s>>>(cur, nxt, V, m, st);
            double* t = cur;
            cur = nxt;
            nxt = t;
        }
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    *sweeps = sweep;
    return hipSuccess;
}

hipError_t lr_topk(const double* w, const double* V, int m, int k, double* lam, double* Vk, hipStream_t s)
{
    if (k < 1 || k > MAXM || k > m) return hipErrorInvalidValue;
    lr_select<<<1, 1024, 0, s>>>(w, V, m, k, lam, Vk);
    return hipGetLastError();
}

}  // namespace dm
