// k_lowrank.hip - FP64 building blocks of the block-Krylov low-rank
// approximation (Appendix C.1: the top singular values, and with them a
// rank-k approximation, from matrix-vector queries only).
//
// The products with A run through the l1 / l2-squared query; everything
// here works on tall, skinny FP64 blocks (n x m with m <= 64) and on the
// small projected matrix T = Q^T A Q:
//   * lr_gram_partial / lr_reduce - C = A^T B of two n x m blocks, split over
//     rows into fixed per-block partial sums and reduced in a fixed order
//     (bit-reproducible run to run);
//   * lr_update   - Y = beta Y + Q C, row by row (block Gram-Schmidt updates,
//     Y R^-1 of Cholesky QR, and U = Q V of the final step);
//   * lr_chol     - the orthonormalising factor of Cholesky QR for a small
//     Gram matrix (column-equilibrated), dropping dependent columns;
//   * lr_jacobi   - eigenvalues and eigenvectors of the symmetric T by the
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
constexpr int64_t LR_ROWS_PER_BLK = 4096;   // rows per partial Gram product

// ---------------------------------------------------------------------------
// C_part[blk] = sum over the block's rows r of A[r][p] * B[r][q]
// A: n x ma, B: n x mb, row-major.  Each thread owns a 4 x 4 block of (p, q)
// entries and a share of the rows of each tile; row shares are added in a
// fixed order at the end.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void lr_gram_partial(const double* __restrict__ A, int ma,
                                                       const double* __restrict__ B, int mb, int64_t n,
                                                       int64_t rows_per_blk, double* __restrict__ part)
{
    __shared__ double sA[GT][MAXM + 4];
    __shared__ double sB[GT][MAXM + 4];
    const int tid = threadIdx.x;
    const int pa = (ma + 3) / 4, pb = (mb + 3) / 4, ne = pa * pb;
    int groups = 256 / ne;
    if (groups > 8) groups = 8;
    if (groups < 1) groups = 1;
    const int e = tid % ne, g = tid / ne;
    const bool active = tid < ne * groups;
    const int p0 = (e / pb) * 4, q0 = (e % pb) * 4;
    double acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
    const int64_t rb = (int64_t)blockIdx.x * rows_per_blk;
    const int64_t re = rb + rows_per_blk < n ? rb + rows_per_blk : n;
    for (int64_t r0 = rb; r0 < re; r0 += GT) {
        const int nr = (int)(re - r0 < GT ? re - r0 : GT);
        for (int i = tid; i < GT * MAXM; i += 256) {
            const int r = i / MAXM, c = i % MAXM;
            sA[r][c] = (r < nr && c < ma) ? A[(r0 + r) * ma + c] : 0.0;
            sB[r][c] = (r < nr && c < mb) ? B[(r0 + r) * mb + c] : 0.0;
        }
        __syncthreads();
        if (active) {
            for (int r = g; r < nr; r += groups) {
                double a[4], bq[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    a[i] = sA[r][p0 + i];
                    bq[i] = sB[r][q0 + i];
                }
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int j = 0; j < 4; ++j) acc[i][j] = fma(a[i], bq[j], acc[i][j]);
            }
        }
        __syncthreads();
    }
    // add the row shares in group order
    double* red = &sA[0][0];   // GT * (MAXM + 4) >= 256 * 16 doubles
    if (active) {
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) red[(g * ne + e) * 16 + i * 4 + j] = acc[i][j];
    }
    __syncthreads();
    if (active && g == 0) {
        for (int gg = 1; gg < groups; ++gg)
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] += red[(gg * ne + e) * 16 + i * 4 + j];
        double* out = part + (size_t)blockIdx.x * ma * mb;
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (p0 + i < ma && q0 + j < mb) out[(p0 + i) * mb + (q0 + j)] = acc[i][j];
    }
}

// out[p * ldo + q] = scale * sum_blk part[blk][p][q], blocks added in order
__global__ __launch_bounds__(256) void lr_reduce(const double* __restrict__ part, int nblk, int ma, int mb,
                                                 double* __restrict__ out, int ldo, double scale)
{
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= ma * mb) return;
    double s = 0.0;
    for (int k = 0; k < nblk; ++k) s += part[(size_t)k * ma * mb + e];
    out[(size_t)(e / mb) * ldo + (e % mb)] = scale * s;
}

// ---------------------------------------------------------------------------
// Y[r][q] = beta * Y[r][q] + sum_p Q[r][p] C[p][q]   (q < mb, p < ma)
// Y: n x ldy (columns 0..mb-1 written), Q: n x ldq, C: ma x ldc.  A workgroup
// owns 64 rows; it stages its Q rows in LDS before writing Y, so Y may be Q
// (in-place right multiplication).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void lr_update(double* Y, int ldy, int mb,
                                                 const double* Q, int ldq, int ma,
                                                 const double* __restrict__ C, int ldc, double beta, int64_t n)
{
    __shared__ double sC[MAXM][MAXM + 1];
    __shared__ double sQ[GT][MAXM + 1];
    const int tid = threadIdx.x;
    const int64_t r0 = (int64_t)blockIdx.x * GT;
    for (int i = tid; i < MAXM * MAXM; i += 256) {
        const int p = i / MAXM, q = i % MAXM;
        sC[p][q] = (p < ma && q < mb) ? C[(size_t)p * ldc + q] : 0.0;
    }
    for (int i = tid; i < GT * MAXM; i += 256) {
        const int r = i / MAXM, c = i % MAXM;
        sQ[r][c] = (r0 + r < n && c < ma) ? Q[(r0 + r) * ldq + c] : 0.0;
    }
    __syncthreads();
    const int rr = tid >> 2, cg = tid & 3;
    const int64_t row = r0 + rr;
    if (row >= n) return;
    double out[MAXM / 4];
#pragma unroll
    for (int k = 0; k < MAXM / 4; ++k) out[k] = 0.0;
    for (int p = 0; p < ma; ++p) {
        const double qv = sQ[rr][p];
#pragma unroll
        for (int k = 0; k < MAXM / 4; ++k) out[k] = fma(qv, sC[p][cg + 4 * k], out[k]);
    }
    double* y = Y + row * ldy;
#pragma unroll
    for (int k = 0; k < MAXM / 4; ++k) {
        const int q = cg + 4 * k;
        if (q < mb) y[q] = beta == 0.0 ? out[k] : fma(beta, y[q], out[k]);
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

__global__ __launch_bounds__(256) void lr_cvt_f64_f32(const double* __restrict__ a, float* __restrict__ b, size_t n)
{
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) b[i] = (float)a[i];
}
__global__ __launch_bounds__(256) void lr_cvt_f32_f64(const float* __restrict__ a, double* __restrict__ b, size_t n)
{
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) b[i] = (double)a[i];
}

// ---------------------------------------------------------------------------
// Cyclic Jacobi on the symmetric m x m matrix T (in place; one workgroup).
// Step s of a sweep pairs index 0 with (s mod (m'-1)) + 1 and the others
// around a circle (m' = m rounded up to even; a pair with the padding index
// is skipped).  Each rotation zeroes T[p][q] (the rotation of the classical
// Jacobi method), and V accumulates the rotations.  Sweeps stop when the
// off-diagonal mass is at most tol^2 times the total, or after max_sweeps.
// On return w[i] = T[i][i]; *sweeps_out is the number of sweeps done.
// ---------------------------------------------------------------------------
constexpr int JMAX = 1024;   // largest m

__global__ __launch_bounds__(1024) void lr_jacobi(double* __restrict__ T, double* __restrict__ V, double* __restrict__ w,
                                                  int m, int max_sweeps, double tol, int* __restrict__ sweeps_out)
{
    __shared__ int sp[JMAX / 2], sq[JMAX / 2];
    __shared__ double sc[JMAX / 2], ss[JMAX / 2];
    __shared__ double red[2][1024];
    const int tid = threadIdx.x;
    const int mp = (m + 1) & ~1;
    const int half = mp / 2;
    for (int i = tid; i < m * m; i += 1024) V[i] = (i / m == i % m) ? 1.0 : 0.0;
    __syncthreads();
    int sweep = 0;
    for (; sweep < max_sweeps; ++sweep) {
        // convergence test: off-diagonal mass against the total
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
        const bool done = red[0][0] <= tol * tol * red[1][0];
        __syncthreads();
        if (done) break;
        for (int s = 0; s < mp - 1; ++s) {
            if (tid < half) {
                auto pos = [&](int j) { return j == 0 ? 0 : 1 + (j - 1 + s) % (mp - 1); };
                int p = pos(tid), q = pos(mp - 1 - tid);
                if (p > q) {
                    const int t = p;
                    p = q;
                    q = t;
                }
                double c = 1.0, sn = 0.0;
                if (q < m) {
                    const double apq = T[p * m + q];
                    if (apq != 0.0) {
                        const double app = T[p * m + p], aqq = T[q * m + q];
                        const double th = (aqq - app) / (2.0 * apq);
                        const double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
                        c = 1.0 / sqrt(t * t + 1.0);
                        sn = t * c;
                    }
                }
                sp[tid] = p;
                sq[tid] = q < m ? q : p;   // a skipped pair rotates nothing
                sc[tid] = c;
                ss[tid] = q < m ? sn : 0.0;
            }
            __syncthreads();
            // rows: T <- J^T T
            for (int idx = tid; idx < half * m; idx += 1024) {
                const int i = idx / m, j = idx % m;
                const int p = sp[i], q = sq[i];
                if (p == q) continue;
                const double c = sc[i], sn = ss[i];
                const double a = T[p * m + j], b = T[q * m + j];
                T[p * m + j] = c * a - sn * b;
                T[q * m + j] = sn * a + c * b;
            }
            __syncthreads();
            // columns: T <- T J, and V <- V J
            for (int idx = tid; idx < m * half; idx += 1024) {
                const int r = idx / half, i = idx % half;
                const int p = sp[i], q = sq[i];
                if (p == q) continue;
                const double c = sc[i], sn = ss[i];
                const double a = T[r * m + p], b = T[r * m + q];
                T[r * m + p] = c * a - sn * b;
                T[r * m + q] = sn * a + c * b;
                const double va = V[r * m + p], vb = V[r * m + q];
                V[r * m + p] = c * va - sn * vb;
                V[r * m + q] = sn * va + c * vb;
            }
            __syncthreads();
        }
    }
    for (int i = tid; i < m; i += 1024) w[i] = T[i * m + i];
    if (tid == 0) *sweeps_out = sweep;
}

// The k eigenpairs of largest |lambda| (ties by lower index), in decreasing
// |lambda|: lam[t] and the columns Vk[:, t] = V[:, idx_t] (m x k).
__global__ __launch_bounds__(256) void lr_select(const double* __restrict__ w, const double* __restrict__ V, int m, int k,
                                                 double* __restrict__ lam, double* __restrict__ Vk)
{
    __shared__ int sidx[MAXM];
    if (threadIdx.x == 0) {
        for (int t = 0; t < k; ++t) {
            int best = -1;
            for (int i = 0; i < m; ++i) {
                bool taken = false;
                for (int u = 0; u < t; ++u) taken = taken || sidx[u] == i;
                if (taken) continue;
                if (best < 0 || fabs(w[i]) > fabs(w[best])) best = i;
            }
            sidx[t] = best;
            lam[t] = w[best];
        }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < m * k; e += 256) {
        const int r = e / k, t = e % k;
        Vk[e] = V[r * m + sidx[t]];
    }
}

}  // namespace

int lr_max_block() { return MAXM; }
int lr_max_basis() { return JMAX; }

size_t lr_gram_scratch_doubles(int64_t n, int ma, int mb) {
    const int64_t nblk = (n + LR_ROWS_PER_BLK - 1) / LR_ROWS_PER_BLK;
    return (size_t)nblk * ma * mb;
}

hipError_t lr_gram(const double* A, int ma, const double* B, int mb, int64_t n, double* part, double* out,
                   int ldo, double scale, hipStream_t s)
{
    if (ma < 1 || mb < 1 || ma > MAXM || mb > MAXM || n < 1) return hipErrorInvalidValue;
    const int64_t nblk = (n + LR_ROWS_PER_BLK - 1) / LR_ROWS_PER_BLK;
    lr_gram_partial<<<(unsigned)nblk, 256, 0, s>>>(A, ma, B, mb, n, LR_ROWS_PER_BLK, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    lr_reduce<<<(ma * mb + 255) / 256, 256, 0, s>>>(part, (int)nblk, ma, mb, out, ldo, scale);
    return hipGetLastError();
}

hipError_t lr_update_rows(double* Y, int ldy, int mb, const double* Q, int ldq, int ma, const double* C, int ldc,
                          double beta, int64_t n, hipStream_t s)
{
    if (ma < 1 || mb < 1 || ma > MAXM || mb > MAXM || n < 1) return hipErrorInvalidValue;
    lr_update<<<(unsigned)((n + GT - 1) / GT), 256, 0, s>>>(Y, ldy, mb, Q, ldq, ma, C, ldc, beta, n);
    return hipGetLastError();
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

hipError_t lr_cvt(const double* a, float* b, size_t n, hipStream_t s)
{
    size_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    lr_cvt_f64_f32<<<(unsigned)blocks, 256, 0, s>>>(a, b, n);
    return hipGetLastError();
}
hipError_t lr_cvt(const float* a, double* b, size_t n, hipStream_t s)
{
    size_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    lr_cvt_f32_f64<<<(unsigned)blocks, 256, 0, s>>>(a, b, n);
    return hipGetLastError();
}

hipError_t lr_eig(double* T, double* V, double* w, int m, int max_sweeps, double tol, int* sweeps, hipStream_t s)
{
    if (m < 1 || m > JMAX) return hipErrorInvalidValue;
    lr_jacobi<<<1, 1024, 0, s>>>(T, V, w, m, max_sweeps, tol, sweeps);
    return hipGetLastError();
}

hipError_t lr_topk(const double* w, const double* V, int m, int k, double* lam, double* Vk, hipStream_t s)
{
    if (k < 1 || k > MAXM || k > m) return hipErrorInvalidValue;
    lr_select<<<1, 256, 0, s>>>(w, V, m, k, lam, Vk);
    return hipGetLastError();
}

}  // namespace dm
