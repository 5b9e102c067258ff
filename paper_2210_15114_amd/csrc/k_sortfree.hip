// k_sortfree.hip - the distance functions whose query needs no sort: per-
// coordinate moments of the right-hand sides, then one pass over the points
// (Appendix A: the KL divergence of Algorithm 4, l_p^p for even p of
// Algorithm 5, the bilinear form of Algorithms 8 and 9, and the squared
// Mahalanobis distance and cross entropy that follow the same pattern).
//
//  even p:     (A z)_i = sum_k sum_(t=0..p) C(p, t) (-1)^t x~_ik^(p-t) F_t(k),
//              F_t(k) = sum_j z_j x~_jk^t,  F_0 = sum z,  x~ = x - c (a
//              per-coordinate centre; the distance is translation invariant)
//  linear:     (A z)_i = sum_k x~_ik V(k) + a_i sum_j z_j + U,
//              V = alpha W F (W a d x d matrix, or the identity),
//              F(k) = sum_j z_j phi(x_jk),  phi = log (KL, cross entropy) or
//              the centred coordinate (Mahalanobis, bilinear form)
//
// Stage 1 (moments) reduces over the points: a workgroup owns a range of
// rows and a range of coordinates and keeps per-thread sums for a few
// coordinates of one column; stage 2 adds the row ranges in a fixed order and
// applies the binomial coefficients (even p) or the scale alpha; an optional
// mix applies W.  The apply stage gives every thread one column and a few
// points, with the moments of a coordinate chunk and the points' coordinates
// staged in LDS.  Float data accumulates in FP64 and rounds once to FP32;
// integer data (even p) runs in wrapping int64, exact whenever the result
// fits.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <type_traits>

#include "dm_internal.h"

namespace dm {
namespace {

constexpr int MSR = 32;   // rows per LDS tile of the moments stage
constexpr int MKG = 4;    // coordinate groups per moments workgroup

template <int NT>
constexpr int moments_kpt() { return NT == 1 ? 16 : NT <= 4 ? 8 : 4; }

template <typename ACC>
__device__ __forceinline__ ACC mul_acc(ACC a, ACC b) {
    if constexpr (std::is_same<ACC, double>::value) return a * b;
    else return (ACC)((uint64_t)a * (uint64_t)b);
}
template <typename ACC>
__device__ __forceinline__ ACC fma_acc(ACC a, ACC b, ACC c) {
    if constexpr (std::is_same<ACC, double>::value) return fma(a, b, c);
    else return (ACC)((uint64_t)a * (uint64_t)b + (uint64_t)c);
}
template <typename ACC>
__device__ __forceinline__ ACC add_acc(ACC a, ACC b) {
    if constexpr (std::is_same<ACC, double>::value) return a + b;
    else return (ACC)((uint64_t)a + (uint64_t)b);
}

// V consecutive values loaded as one vector (16 bytes for V = 4 floats or
// V = 2 doubles); the address must be a multiple of the vector size
template <typename T, int V>
struct alignas(sizeof(T) * V) Vec {
    T v[V];
};

// a Vec loaded with a non-temporal (streaming) load; the elements are copied
// out of the vector by value
template <typename T, int V>
__device__ __forceinline__ Vec<T, V> load_vec_nt(const T* p) {
    Vec<T, V> r;
    if constexpr (V == 1) {
        r.v[0] = __builtin_nontemporal_load(p);
    } else {
        typedef T tv __attribute__((ext_vector_type(V)));
        const tv t = __builtin_nontemporal_load(reinterpret_cast<const tv*>(p));
#pragma unroll
        for (int i = 0; i < V; ++i) r.v[i] = t[i];
    }
    return r;
}
// X rows of the narrow moments: FP64 rows (the logarithms of KL and cross
// entropy) stream faster with non-temporal loads, FP32 rows did not
template <typename XT, int V>
__device__ __forceinline__ Vec<XT, V> load_x_narrow(const XT* p) {
    if constexpr (sizeof(XT) == 8) return load_vec_nt<XT, V>(p);
    else return *reinterpret_cast<const Vec<XT, V>*>(p);
}

// a coordinate value less its centre (none: the value itself)
template <typename XT, typename ACC>
__device__ __forceinline__ ACC feature(XT x, const ACC* centre, int k) {
    return centre ? (ACC)((ACC)x - centre[k]) : (ACC)x;
}

// part[blk][t][k][c] = sum over the workgroup's rows of z_jc phi(x_jk)^(t+1),
// t = 0 .. NT-1.  Threads: column c = tid % BW, coordinate group
// (tid / BW) % MKG, row stripe tid / (BW MKG).
template <typename XT, typename ZT, typename ACC, int NT, int BW>
__global__ __launch_bounds__(256) void sf_moments_kernel(const XT* __restrict__ X, const ACC* __restrict__ centre,
                                                         const ZT* __restrict__ Z, int64_t n, int32_t d, int32_t b,
                                                         int64_t rows_per_blk, ACC* __restrict__ part)
{
    constexpr int KPT = moments_kpt<NT>();
    constexpr int KC = MKG * KPT;
    constexpr int RS = 256 / (BW * MKG) > 0 ? 256 / (BW * MKG) : 1;
    constexpr int XS = KC + 1, ZS = BW + 1;
    constexpr int STAGE = MSR * XS + MSR * ZS;
    constexpr int RED = RS > 1 ? 256 * KPT : 0;
    __shared__ ACC smem[STAGE > RED ? STAGE : RED];
    ACC* sX = smem;
    ACC* sZ = smem + MSR * XS;
    const int tid = threadIdx.x;
    const int c = tid % BW, kg = (tid / BW) % MKG, rs = tid / (BW * MKG);
    const int k0 = blockIdx.y * KC;
    const int64_t rb = (int64_t)blockIdx.x * rows_per_blk;
    const int64_t re = rb + rows_per_blk < n ? rb + rows_per_blk : n;
    ACC acc[KPT][NT];
#pragma unroll
    for (int q = 0; q < KPT; ++q)
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[q][t] = ACC(0);
    for (int64_t r0 = rb; r0 < re; r0 += MSR) {
        const int nr = (int)(re - r0 < MSR ? re - r0 : MSR);
        for (int e = tid; e < MSR * KC; e += 256) {
            const int r = e / KC, kk = e % KC;
            ACC v = ACC(0);
            if (r < nr && k0 + kk < d) v = feature<XT, ACC>(X[(r0 + r) * d + k0 + kk], centre, k0 + kk);
            sX[r * XS + kk] = v;
        }
        for (int e = tid; e < MSR * BW; e += 256) {
            const int r = e / BW, cc = e % BW;
            sZ[r * ZS + cc] = (r < nr && cc < b) ? (ACC)Z[(r0 + r) * b + cc] : ACC(0);
        }
        __syncthreads();
        for (int r = rs; r < nr; r += RS) {
            const ACC z = sZ[r * ZS + c];
#pragma unroll
            for (int q = 0; q < KPT; ++q) {
                const ACC x = sX[r * XS + kg * KPT + q];
                ACC xt = x;
#pragma unroll
                for (int t = 0; t < NT; ++t) {
                    acc[q][t] = fma_acc(xt, z, acc[q][t]);
                    if (t + 1 < NT) xt = mul_acc(xt, x);
                }
            }
        }
        __syncthreads();
    }
    // sum the row stripes (fixed order), one moment at a time
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        if constexpr (RS > 1) {
#pragma unroll
            for (int q = 0; q < KPT; ++q) smem[q * 256 + tid] = acc[q][t];
            __syncthreads();
            if (rs == 0) {
#pragma unroll
                for (int q = 0; q < KPT; ++q) {
                    ACC s = ACC(0);
                    for (int st = 0; st < RS; ++st) s = add_acc(s, smem[q * 256 + st * BW * MKG + tid]);
                    acc[q][t] = s;
                }
            }
            __syncthreads();
        }
        if (rs == 0 && c < b) {
#pragma unroll
            for (int q = 0; q < KPT; ++q) {
                const int k = k0 + kg * KPT + q;
                if (k < d) part[(((size_t)blockIdx.x * NT + t) * d + k) * b + c] = acc[q][t];
            }
        }
    }
}

__host__ __device__ constexpr int64_t binom_sf(int p, int t) {
    int64_t r = 1;
    for (int i = 0; i < t; ++i) r = r * (p - i) / (i + 1);
    return r;
}

// The row-range partials part[blk][e] (e = (t, k, c), count entries) are added
// in a fixed order.  Many entries: two passes; slice s sums blocks [s ks, (s + 1) ks) for every
// entry (threads over consecutive entries, so every load is coalesced), then
// G[e] = coef_t sum over the slices in order, with coef_t = C(p, t + 1)
// (-1)^(t + 1) when p > 0 (even p) and alpha otherwise (float only).
constexpr int SF_SLICES = 32;

template <typename ACC>
__device__ __forceinline__ ACC shfl_xor_acc(ACC v, int off, int width) {
    if constexpr (std::is_same<ACC, double>::value) return __shfl_xor(v, off, width);
    else return (ACC)__shfl_xor((long long)v, off, width);
}

__device__ __forceinline__ int64_t even_coef(int p, int t) { return ((t & 1) ? -1 : 1) * binom_sf(p, t); }

// Few entries (narrow blocks): one launch, one wave per entry; lane l adds
// the partials l, l + 64, ... in order, then a fixed xor tree.
template <typename ACC>
__global__ __launch_bounds__(256) void sf_reduce_waves(const ACC* __restrict__ part, int nblk, int64_t per_t, int nt,
                                                       int p, double alpha, ACC* __restrict__ G)
{
    const int64_t e = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int64_t count = per_t * nt;
    if (e >= count) return;   // whole waves leave together
    ACC s = ACC(0);
    for (int k = lane; k < nblk; k += 64) s = add_acc(s, part[(size_t)k * count + e]);
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) s = add_acc(s, shfl_xor_acc(s, off, 64));
    if (lane != 0) return;
    if (p > 0) G[e] = mul_acc(s, (ACC)even_coef(p, (int)(e / per_t) + 1));
    else G[e] = (ACC)(alpha * (double)s);
}

template <typename ACC>
__global__ __launch_bounds__(256) void sf_reduce_slices(const ACC* __restrict__ part, int nblk, int64_t count, int ks,
                                                        ACC* __restrict__ slices)
{
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= count) return;
    const int k0 = blockIdx.y * ks;
    const int k1 = k0 + ks < nblk ? k0 + ks : nblk;
    ACC acc = ACC(0);
    for (int k = k0; k < k1; ++k) acc = add_acc(acc, part[(size_t)k * count + e]);
    slices[(size_t)blockIdx.y * count + e] = acc;
}

template <typename ACC>
__global__ __launch_bounds__(256) void sf_reduce_kernel(const ACC* __restrict__ slices, int nslice, int64_t per_t,
                                                        int nt, int p, double alpha, ACC* __restrict__ G)
{
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t count = per_t * nt;
    if (e >= count) return;
    ACC s = ACC(0);
    for (int k = 0; k < nslice; ++k) s = add_acc(s, slices[(size_t)k * count + e]);
    if (p > 0) G[e] = mul_acc(s, (ACC)even_coef(p, (int)(e / per_t) + 1));
    else G[e] = (ACC)(alpha * (double)s);
}

// V[k][c] = sum_l W[k][l] F[l][c]
__global__ __launch_bounds__(256) void sf_mix_kernel(const double* __restrict__ W, const double* __restrict__ F,
                                                     int32_t d, int32_t b, double* __restrict__ V)
{
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= (int64_t)d * b) return;
    const int k = (int)(e / b), c = (int)(e % b);
    double s = 0.0;
    for (int l = 0; l < d; ++l) s = fma(W[(size_t)k * d + l], F[(size_t)l * b + c], s);
    V[e] = s;
}

template <int BW> constexpr int apply_ppt() { return BW >= 8 ? BW / 8 : 1; }
template <int NT, int BW> constexpr int apply_kc() { return (BW <= 8 || NT <= 2) ? 32 : 16; }

// Out[i][c] for every point i and column c.  Thread: column c = tid % BW,
// point group tid / BW owning points i0 + q (256 / BW) + group, q < PPT.
//   EVEN (NT = p):  sum_k Horner in x~_ik over G_0 = T0, G_1 .. G_p
//   LIN  (NT = 1):  sum_k x~_ik V(k) + a_i T0 + U
template <typename XT, typename ACC, typename OT, int NT, bool EVEN, int BW>
__global__ __launch_bounds__(256) void sf_apply_kernel(const XT* __restrict__ X, const ACC* __restrict__ centre,
                                                       int64_t n, int32_t d, int32_t b, const ACC* __restrict__ T0,
                                                       const ACC* __restrict__ G, const double* __restrict__ a,
                                                       const double* __restrict__ U, OT* __restrict__ Out)
{
    constexpr int PPT = apply_ppt<BW>();
    constexpr int PG = 256 / BW;
    constexpr int NPB = PG * PPT;
    constexpr int KC = apply_kc<NT, BW>();
    constexpr int XS = KC + 1;
    __shared__ XT sX[NPB * XS];          // raw coordinates; the centre is taken off at use
    __shared__ ACC sC[KC];
    __shared__ ACC sG[NT * KC * BW];
    const int tid = threadIdx.x;
    const int c = tid % BW, pg = tid / BW;
    const int64_t i0 = (int64_t)blockIdx.x * NPB;
    const bool col_ok = c < b;
    const ACC t0 = col_ok ? T0[c] : ACC(0);
    ACC acc[PPT];
#pragma unroll
    for (int q = 0; q < PPT; ++q) acc[q] = ACC(0);
    const size_t per_t = (size_t)d * b;
    for (int k0 = 0; k0 < d; k0 += KC) {
        if (d % 4 == 0) {   // 16-byte loads; a group of 4 lies wholly inside or outside the row
            for (int e = tid; e < NPB * (KC / 4); e += 256) {
                const int p = e / (KC / 4), kk = 4 * (e % (KC / 4));
                const int64_t i = i0 + p;
                Vec<XT, 4> v = {};
                if (i < n && k0 + kk < d) v = *reinterpret_cast<const Vec<XT, 4>*>(X + i * d + k0 + kk);
#pragma unroll
                for (int j = 0; j < 4; ++j) sX[p * XS + kk + j] = v.v[j];
            }
        } else {
            for (int e = tid; e < NPB * KC; e += 256) {
                const int p = e / KC, kk = e % KC;
                const int64_t i = i0 + p;
                sX[p * XS + kk] = (i < n && k0 + kk < d) ? X[i * d + k0 + kk] : XT(0);
            }
        }
        if (tid < KC) sC[tid] = (centre && k0 + tid < d) ? centre[k0 + tid] : ACC(0);
        for (int e = tid; e < NT * KC * BW; e += 256) {
            const int t = e / (KC * BW), rem = e % (KC * BW);
            const int kk = rem / BW, cq = rem % BW;
            sG[e] = (k0 + kk < d && cq < b) ? G[t * per_t + (size_t)(k0 + kk) * b + cq] : ACC(0);
        }
        __syncthreads();
        const int kn = d - k0 < KC ? d - k0 : KC;
        for (int kk = 0; kk < kn; ++kk) {
            ACC g[NT];
#pragma unroll
            for (int t = 0; t < NT; ++t) g[t] = sG[(t * KC + kk) * BW + c];
            const ACC ck = sC[kk];
#pragma unroll
            for (int q = 0; q < PPT; ++q) {
                const ACC x = (ACC)((ACC)sX[(q * PG + pg) * XS + kk] - ck);
                if constexpr (EVEN) {
                    ACC h = t0;
#pragma unroll
                    for (int t = 0; t < NT; ++t) h = fma_acc(h, x, g[t]);
                    acc[q] = add_acc(acc[q], h);
                } else {
                    acc[q] = fma_acc(x, g[0], acc[q]);
                }
            }
        }
        __syncthreads();
    }
    if (!col_ok) return;
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
        const int64_t i = i0 + q * PG + pg;
        if (i >= n) continue;
        ACC s = acc[q];
        if constexpr (!EVEN) {
            if (a) s = fma(a[i], (double)t0, s);
            if (U) s += U[c];
        }
        Out[i * b + c] = (OT)s;
    }
}

// ---- narrow blocks (b <= 8): moments without LDS staging ---------------------
constexpr int NU = 4;   // rows in flight per thread

// part[blk][t][k][c] as sf_moments_kernel.  A workgroup owns a range of rows
// and up to 256 V coordinates; thread (row offset tid / dcv, coordinate group
// tid % dcv) reads V adjacent coordinates of every R-th row (R = 256 / dcv)
// straight from the row-major points, so a wave's loads are contiguous, and
// keeps all NT x BW x V sums in registers; the R row offsets are added in a
// fixed order at the end.  V > 1 needs d to be a multiple of V.
template <typename XT, typename ZT, typename ACC, int NT, int BW, int V>
__global__ __launch_bounds__(256) void sf_moments_narrow(const XT* __restrict__ X, const ACC* __restrict__ centre,
                                                         const ZT* __restrict__ Z, int64_t n, int32_t d, int32_t b,
                                                         int64_t rows_per_blk, ACC* __restrict__ part)
{
    __shared__ ACC red[256 * BW];
    const int tid = threadIdx.x;
    const int k0 = blockIdx.y * 256 * V;
    const int dc = d - k0 < 256 * V ? d - k0 : 256 * V;
    const int dcv = dc / V;
    const int R = 256 / dcv;
    const int kv = tid % dcv, rsub = tid / dcv;
    const bool active = rsub < R;
    const int k = k0 + kv * V;
    const int64_t rb = (int64_t)blockIdx.x * rows_per_blk;
    const int64_t re = rb + rows_per_blk < n ? rb + rows_per_blk : n;
    ACC acc[NT][BW][V];
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int c = 0; c < BW; ++c)
#pragma unroll
            for (int j = 0; j < V; ++j) acc[t][c][j] = ACC(0);
    if (active) {
        ACC cen[V];
#pragma unroll
        for (int j = 0; j < V; ++j) cen[j] = centre ? centre[k + j] : ACC(0);
        auto step = [&](const Vec<XT, V>& xr, const ZT* zr) {
#pragma unroll
            for (int j = 0; j < V; ++j) {
                const ACC x = (ACC)((ACC)xr.v[j] - cen[j]);
                ACC xt = x;
#pragma unroll
                for (int t = 0; t < NT; ++t) {
#pragma unroll
                    for (int c = 0; c < BW; ++c)
                        if (c < b) acc[t][c][j] = fma_acc(xt, (ACC)zr[c], acc[t][c][j]);
                    if (t + 1 < NT) xt = mul_acc(xt, x);
                }
            }
        };
        // a Z row as 16-byte vectors when b and the alignment allow
        constexpr int ZV = 16 / (int)sizeof(ZT);
        const bool zvec = BW >= ZV && b % ZV == 0 && (uintptr_t)Z % 16 == 0;
        auto load_z = [&](int64_t row, ZT (&zr)[BW]) {
            if constexpr (BW >= ZV) {
                if (zvec) {
#pragma unroll
                    for (int c0 = 0; c0 < BW; c0 += ZV) {
                        Vec<ZT, ZV> q = {};
                        if (c0 < b) q = *reinterpret_cast<const Vec<ZT, ZV>*>(Z + row * b + c0);
#pragma unroll
                        for (int v = 0; v < ZV; ++v) zr[c0 + v] = q.v[v];
                    }
                    return;
                }
            }
#pragma unroll
            for (int c = 0; c < BW; ++c) zr[c] = c < b ? Z[row * b + c] : ZT(0);
        };
        int64_t r = rb + rsub;
        for (; r + (int64_t)(NU - 1) * R < re; r += (int64_t)NU * R) {
            Vec<XT, V> xv[NU];
            ZT zv[NU][BW];
#pragma unroll
            for (int u = 0; u < NU; ++u) {
                const int64_t row = r + (int64_t)u * R;
                xv[u] = load_x_narrow<XT, V>(X + row * d + k);
                load_z(row, zv[u]);
            }
#pragma unroll
            for (int u = 0; u < NU; ++u) step(xv[u], zv[u]);
        }
        for (; r < re; r += R) {
            ZT zv[BW];
            load_z(r, zv);
            step(load_x_narrow<XT, V>(X + r * d + k), zv);
        }
    }
#pragma unroll
    for (int t = 0; t < NT; ++t) {
#pragma unroll
        for (int j = 0; j < V; ++j) {
            if (active) {
#pragma unroll
                for (int c = 0; c < BW; ++c) red[tid * BW + c] = acc[t][c][j];
            }
            __syncthreads();
            if (rsub == 0) {
#pragma unroll
                for (int c = 0; c < BW; ++c) {
                    ACC sum = ACC(0);
                    for (int q = 0; q < R; ++q) sum = add_acc(sum, red[(q * dcv + kv) * BW + c]);
                    if (c < b) part[(((size_t)blockIdx.x * NT + t) * d + k + j) * b + c] = sum;
                }
            }
            __syncthreads();
        }
    }
}

// ---- FP64 matrix cores for the single-moment forms (b >= 4) ----------------
// v_mfma_f64_16x16x4f64 lane layout on gfx950 (checked on the GPU with a
// probe): A (16 x 4): lane l holds A[l % 16][l / 16]; B (4 x 16): lane l holds
// B[l / 16][l % 16]; D (16 x 16): lane l, element r holds D[4r + l / 16][l % 16].
typedef double d4v __attribute__((ext_vector_type(4)));

template <typename XT>
__device__ __forceinline__ void load4(const XT* p, double (&v)[4]) {
    if constexpr (sizeof(XT) == 4) {
        const Vec<XT, 4> q = *reinterpret_cast<const Vec<XT, 4>*>(p);
#pragma unroll
        for (int t = 0; t < 4; ++t) v[t] = (double)q.v[t];
    } else {
        const Vec<XT, 2> q0 = *reinterpret_cast<const Vec<XT, 2>*>(p);
        const Vec<XT, 2> q1 = *reinterpret_cast<const Vec<XT, 2>*>(p + 2);
        v[0] = (double)q0.v[0];
        v[1] = (double)q0.v[1];
        v[2] = (double)q1.v[0];
        v[3] = (double)q1.v[1];
    }
}

// part[wg][k][c] = sum over the workgroup's rows j of phi(x_jk) z_jc (phi: the
// centred coordinate, or the stored logarithm).  A wave owns 64 coordinates
// (workgroup column blockIdx.y) and 16 CU columns: 4 x CU tiles of 16 x 16.
// Each step takes 4 rows; lane (m, g) = (l % 16, l / 16) loads coordinates
// k0 + 4m .. +3 of row j + g with one 16-byte load and columns CU m .. +CU-1
// of the same row with one load of 4 CU bytes, so tile t of the coordinates
// holds k = k0 + 4 i + t at tile row i and tile u of the columns holds
// c = CU n + u at tile column n.  CU = 4 serves b <= 64, 2 b <= 32 and 1
// b <= 16 (a step of CU = 1 reads 4 whole rows of Z for b = 16 in one
// coalesced load and takes 4 products instead of the 16 of CU = 4).  Needs
// d % 4 == 0, b % CU == 0 and Z rows aligned to 4 CU bytes.
constexpr int SF_MOM_DEPTH = 4;   // row steps in flight per wave
// TOT: the waves of the first coordinate block also sum z and w z (FP64)
// over their rows into tpart[wave][0 | 1][c] (the totals of the query).
template <typename XT, int P, bool TOT, int CU>
__global__ __launch_bounds__(256) void sf_moments_mfma(const XT* __restrict__ X, const double* __restrict__ centre,
                                                       const float* __restrict__ Z, int64_t n, int32_t d, int32_t b,
                                                       int64_t rows_per_wave, double* __restrict__ part,
                                                       const double* __restrict__ wu, double* __restrict__ tpart)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int m = lane & 15, g = lane >> 4;
    const int64_t xw = (int64_t)blockIdx.x * 4 + w;
    const int k0 = blockIdx.y * 64;
    const int kq = k0 + 4 * m, cq = CU * m;
    const bool kin = kq < d, cin = cq < b;
    // centres apply to FP32 coordinates only (the stored logarithms have none)
    constexpr bool CEN = sizeof(XT) == 4;
    double cen[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) cen[t] = (CEN && centre && kin) ? centre[kq + t] : 0.0;
    d4v acc[4][CU];
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int u = 0; u < CU; ++u) acc[t][u] = d4v{0.0, 0.0, 0.0, 0.0};
    const int64_t r0 = xw * rows_per_wave;
    const int64_t r1 = r0 + rows_per_wave < n ? r0 + rows_per_wave : n;
    // raw values of P row steps in flight: slot p holds step s with s % P == p;
    // a slot is refilled with the step P ahead right after it is consumed
    XT xn[P][4];
    float zn[P][CU];
    double wn[P];
    const bool tw = TOT && blockIdx.y == 0;
    double t0a[CU], ua[CU];
#pragma unroll
    for (int u = 0; u < CU; ++u) { t0a[u] = 0.0; ua[u] = 0.0; }
    auto fetch = [&](int64_t j, XT (&xv)[4], float (&zv)[CU], double& wv) {
#pragma unroll
        for (int t = 0; t < 4; ++t) xv[t] = XT(0);
#pragma unroll
        for (int u = 0; u < CU; ++u) zv[u] = 0.0f;
        wv = 0.0;
        if (j < r1) {
            if (tw && wu) wv = wu[j];
            if (kin) {
                if constexpr (sizeof(XT) == 4) {
                    const Vec<XT, 4> q = *reinterpret_cast<const Vec<XT, 4>*>(X + j * d + kq);
#pragma unroll
                    for (int t = 0; t < 4; ++t) xv[t] = q.v[t];
                } else {
                    const Vec<XT, 2> q0 = *reinterpret_cast<const Vec<XT, 2>*>(X + j * d + kq);
                    const Vec<XT, 2> q1 = *reinterpret_cast<const Vec<XT, 2>*>(X + j * d + kq + 2);
                    xv[0] = q0.v[0]; xv[1] = q0.v[1]; xv[2] = q1.v[0]; xv[3] = q1.v[1];
                }
            }
            if (cin) {
                const Vec<float, CU> q = *reinterpret_cast<const Vec<float, CU>*>(Z + j * b + cq);
#pragma unroll
                for (int u = 0; u < CU; ++u) zv[u] = q.v[u];
            }
        }
    };
#pragma unroll
    for (int p = 0; p < P; ++p) fetch(r0 + 4 * p + g, xn[p], zn[p], wn[p]);
    for (int64_t js = r0; js < r1; js += 4 * P) {   // the same trip count on every lane
#pragma unroll
        for (int p = 0; p < P; ++p) {
            const int64_t j0 = js + 4 * p;
            if (j0 >= r1) break;
            const int64_t j = j0 + g;
            double a[4], z[CU];
#pragma unroll
            for (int t = 0; t < 4; ++t)
                a[t] = (j < r1 && kin) ? (CEN ? (double)xn[p][t] - cen[t] : (double)xn[p][t]) : 0.0;
#pragma unroll
            for (int u = 0; u < CU; ++u) z[u] = (double)zn[p][u];
            if (tw) {
#pragma unroll
                for (int u = 0; u < CU; ++u) {
                    t0a[u] += z[u];
                    ua[u] = fma(wn[p], z[u], ua[u]);
                }
            }
            if (j0 + 4 * P < r1) fetch(j + 4 * P, xn[p], zn[p], wn[p]);
#pragma unroll
            for (int t = 0; t < 4; ++t)
#pragma unroll
                for (int u = 0; u < CU; ++u)
                    acc[t][u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[t], z[u], acc[t][u], 0, 0, 0);
        }
    }
    if (tw) {
        // the four row lanes g of a column group, added in a fixed xor order
#pragma unroll
        for (int u = 0; u < CU; ++u) {
            t0a[u] += __shfl_xor(t0a[u], 16);
            ua[u] += __shfl_xor(ua[u], 16);
            t0a[u] += __shfl_xor(t0a[u], 32);
            ua[u] += __shfl_xor(ua[u], 32);
        }
        if (g == 0) {
#pragma unroll
            for (int u = 0; u < CU; ++u) {
                const int c = cq + u;
                if (c < b) {
                    tpart[((size_t)xw * 2) * b + c] = t0a[u];
                    tpart[((size_t)xw * 2 + 1) * b + c] = ua[u];
                }
            }
        }
    }
    // the workgroup's four waves (disjoint row ranges, the same coordinates)
    // add their sums in LDS in a fixed order, (w0 + w2) + (w1 + w3), and
    // wave 0 writes one partial per workgroup
    __shared__ d4v s_acc[2][4][CU][64];
    if (w >= 2) {
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int u = 0; u < CU; ++u) s_acc[w - 2][t][u][lane] = acc[t][u];
    }
    __syncthreads();
    if (w < 2) {
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int u = 0; u < CU; ++u) acc[t][u] += s_acc[w][t][u][lane];
    }
    __syncthreads();
    if (w == 1) {
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int u = 0; u < CU; ++u) s_acc[0][t][u][lane] = acc[t][u];
    }
    __syncthreads();
    if (w == 0) {
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int u = 0; u < CU; ++u) {
                const d4v v = acc[t][u] + s_acc[0][t][u][lane];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int k = k0 + 4 * (4 * r + g) + t, c = CU * m + u;
                    if (k < d && c < b) part[((size_t)blockIdx.x * d + k) * b + c] = v[r];
                }
            }
    }
}

// Out[i][c] = sum_k x~_ik V[k][c] + a_i T0_c + U_c on matrix cores.  A wave
// takes groups of 16 points and every column (CT tiles of 16); per chunk of
// 16 coordinates lane (m, g) loads coordinates k0 + 4g .. +3 of point m (one
// 16-byte load when d % 4 == 0), and step s of the chunk multiplies the A
// column g = coordinate k0 + 4g + s.  The (group, chunk) pairs of a wave form
// one loop, so the next pair's loads are issued before the current pair's
// products also across group boundaries, and a group's weights a_i when the
// group starts (0.30 -> 0.23 ms at n = 2^20, d = 64, b = 64 against a loop per
// group, which left the first chunk's points and the epilogue's weights
// waiting on memory in every group).  V (d x b FP64) is staged once per
// workgroup in dynamic LDS when it fits (LDS_V), else read through the caches.
// One 16-point group per wave: 2 or 4 groups at a time measured slower (fewer
// waves per SIMD).
template <int CT, bool LDS_V>
__global__ __launch_bounds__(512) void sf_apply_mfma(const float* __restrict__ X, const double* __restrict__ centre,
                                                     int64_t n, int32_t d, int32_t b, const double* __restrict__ T0,
                                                     const double* __restrict__ V, const double* __restrict__ a,
                                                     const double* __restrict__ U, float* __restrict__ Out)
{
    extern __shared__ double sV[];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int m = lane & 15, g = lane >> 4;
    const int wpb = blockDim.x >> 6;   // waves per workgroup (8 share one LDS copy of V)
    if constexpr (LDS_V) {
        for (int e = threadIdx.x; e < d * b; e += blockDim.x) sV[e] = V[e];
        __syncthreads();
    }
    const double* Vs = LDS_V ? sV : V;
    const int64_t ngroup = (n + 15) / 16;
    const int64_t wave = (int64_t)blockIdx.x * wpb + w, nwaves = (int64_t)gridDim.x * wpb;
    const bool vec = d % 4 == 0;
    // column of tile u at tile column m: CT m + u, so that a lane's CT
    // results of a row are adjacent columns (one 16-byte store per row at
    // CT = 4)
    auto colof = [&](int u) { return CT * m + u; };
    double t0[CT], uu[CT];
#pragma unroll
    for (int u = 0; u < CT; ++u) {
        const int c = colof(u);
        t0[u] = c < b ? T0[c] : 0.0;
        uu[u] = (U && c < b) ? U[c] : 0.0;
    }
    // coordinates k0 + 4g .. +3 of point ia, zero outside the data
    auto load_chunk = [&](int64_t ia, int k0, float (&xv)[4]) {
        const int kq = k0 + 4 * g;
#pragma unroll
        for (int s = 0; s < 4; ++s) xv[s] = 0.0f;
        if (ia >= n) return;
        if (vec) {
            if (kq < d) {
                const Vec<float, 4> q = *reinterpret_cast<const Vec<float, 4>*>(X + ia * d + kq);
#pragma unroll
                for (int s = 0; s < 4; ++s) xv[s] = q.v[s];
            }
        } else {
#pragma unroll
            for (int s = 0; s < 4; ++s)
                if (kq + s < d) xv[s] = X[ia * d + kq + s];
        }
    };
    // 16-byte rows of Out: b a multiple of 4 and Out 16-byte aligned
    const bool vec4 = b % 4 == 0 && (uintptr_t)Out % 16 == 0;
    // one flat loop over the wave's (group, chunk) pairs: the next pair's
    // points and centres are loaded before the current pair's products,
    // also across a group boundary, and a group's weights a_i when the
    // group starts, so neither waits at the group's ends
    const int nch = (d + 15) / 16;
    int64_t grp = wave;
    int kc = 0;
    float xn[4];
    double cn[4];
    auto load_centre = [&](int k0, double (&c)[4]) {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int k = k0 + 4 * g + s;
            c[s] = (centre && k < d) ? centre[k] : 0.0;
        }
    };
    if (grp < ngroup) {
        load_chunk(grp * 16 + m, 0, xn);
        load_centre(0, cn);
    }
    d4v acc[CT];
    double aw[4];
    while (grp < ngroup) {
        const int64_t i0 = grp * 16;
        if (kc == 0) {
#pragma unroll
            for (int u = 0; u < CT; ++u) acc[u] = d4v{0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t i = i0 + 4 * r + g;
                aw[r] = (a && i < n) ? a[i] : 0.0;
            }
        }
        float xv[4];
        double cv[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            xv[s] = xn[s];
            cv[s] = cn[s];
        }
        int kc2 = kc + 1;
        int64_t grp2 = grp;
        if (kc2 == nch) {
            kc2 = 0;
            grp2 += nwaves;
        }
        if (grp2 < ngroup) {
            load_chunk(grp2 * 16 + m, 16 * kc2, xn);
            load_centre(16 * kc2, cn);
        }
        const int kq = 16 * kc + 4 * g;
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int k = kq + s;
            const bool kin = k < d;
            double vb[CT];
#pragma unroll
            for (int u = 0; u < CT; ++u) {
                const int c = colof(u);
                vb[u] = (kin && c < b) ? Vs[(size_t)k * b + c] : 0.0;
            }
            const double xa = kin ? (double)xv[s] - cv[s] : 0.0;   // zero for points past n
#pragma unroll
            for (int u = 0; u < CT; ++u) acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(xa, vb[u], acc[u], 0, 0, 0);
        }
        if (kc == nch - 1) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t i = i0 + 4 * r + g;
                if (i >= n) continue;
                float o[CT];
#pragma unroll
                for (int u = 0; u < CT; ++u) {
                    double v = acc[u][r] + uu[u];
                    if (a) v = fma(aw[r], t0[u], v);
                    o[u] = (float)v;
                }
                if (CT == 4 && vec4) {
                    if (CT * m < b)
                        *reinterpret_cast<float4*>(Out + i * b + CT * m) = make_float4(o[0], o[1], o[2], o[3]);
                } else {
#pragma unroll
                    for (int u = 0; u < CT; ++u)
                        if (colof(u) < b) Out[i * b + colof(u)] = o[u];
                }
            }
        }
        kc = kc2;
        grp = grp2;
    }
}

// a non-finite column sum of z means a non-finite z (finite FP32 values
// cannot overflow an FP64 sum)
__global__ void sf_check_finite(const double* __restrict__ T0, int32_t b, uint32_t* __restrict__ status)
{
    const int c = threadIdx.x;
    if (c < b && !isfinite(T0[c])) atomicOr(status, (uint32_t)QF_NONFINITE);
}

// The same product for d <= 16 NCH, d % 4 == 0, with a whole 16-point group
// in flight: a wave loads every coordinate of its next group (NCH 16-byte
// loads per lane) and the group's weights a_i before it multiplies the current
// group, so the 4 NCH product steps of a group cover the memory latency rather
// than the 4 steps of one 16-coordinate chunk.  V and the centres are staged
// once per workgroup in dynamic LDS, zero-padded to 16 NCH rows of 16 CT
// columns, so the product steps read them without bounds tests, and so are the
// column totals T0 and U of the epilogue (which keeps the kernel within the
// registers of 4 waves per SIMD).  The products are taken in the same order as
// in sf_apply_mfma, so the results are the same bit for bit.
template <int CT, int NCH>
__global__ __launch_bounds__(512, 4) void sf_apply_mfma_grp(const float* __restrict__ X,
                                                            const double* __restrict__ centre, int64_t n, int32_t d,
                                                            int32_t b, const double* __restrict__ T0,
                                                            const double* __restrict__ V, const double* __restrict__ a,
                                                            const double* __restrict__ U, float* __restrict__ Out)
{
    constexpr int KP = 16 * NCH, BP = 16 * CT;   // padded rows and columns of V
    extern __shared__ double sV[];               // V (KP x BP), KP centres, BP T0, BP U
    double* const sC = sV + KP * BP;
    double* const sT = sC + KP;
    double* const sU = sT + BP;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int m = lane & 15, g = lane >> 4;
    const int wpb = blockDim.x >> 6;
    for (int e = threadIdx.x; e < KP * BP; e += blockDim.x) {
        const int k = e / BP, c = e % BP;
        sV[e] = (k < d && c < b) ? V[(size_t)k * b + c] : 0.0;
    }
    for (int e = threadIdx.x; e < KP; e += blockDim.x) sC[e] = (centre && e < d) ? centre[e] : 0.0;
    for (int e = threadIdx.x; e < BP; e += blockDim.x) {
        sT[e] = e < b ? T0[e] : 0.0;
        sU[e] = (U && e < b) ? U[e] : 0.0;
    }
    __syncthreads();
    const int64_t ngroup = (n + 15) / 16;
    const int64_t wave = (int64_t)blockIdx.x * wpb + w, nwaves = (int64_t)gridDim.x * wpb;
    // coordinates 16 kc + 4g .. +3 of point grp 16 + m and the weights of the
    // group's rows 4r + g, zero outside the data
    auto load_group = [&](int64_t grp, float (&xg)[NCH][4], double (&ag)[4]) {
        const int64_t ia = grp * 16 + m;
#pragma unroll
        for (int kc = 0; kc < NCH; ++kc) {
            const int kq = 16 * kc + 4 * g;
            Vec<float, 4> q;
#pragma unroll
            for (int s = 0; s < 4; ++s) q.v[s] = 0.0f;
            if (ia < n && kq < d) q = *reinterpret_cast<const Vec<float, 4>*>(X + ia * d + kq);
#pragma unroll
            for (int s = 0; s < 4; ++s) xg[kc][s] = q.v[s];
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int64_t i = grp * 16 + 4 * r + g;
            ag[r] = (a && i < n) ? a[i] : 0.0;
        }
    };
    const bool vec4 = b % 4 == 0 && (uintptr_t)Out % 16 == 0;
    float xn[NCH][4];
    double an[4];
    int64_t grp = wave;
    if (grp < ngroup) load_group(grp, xn, an);
    while (grp < ngroup) {
        const int64_t i0 = grp * 16;
        float xv[NCH][4];
        double aw[4];
#pragma unroll
        for (int kc = 0; kc < NCH; ++kc)
#pragma unroll
            for (int s = 0; s < 4; ++s) xv[kc][s] = xn[kc][s];
#pragma unroll
        for (int r = 0; r < 4; ++r) aw[r] = an[r];
        const int64_t grp2 = grp + nwaves;
        if (grp2 < ngroup) load_group(grp2, xn, an);
        // the lane's V offset, hidden from the optimiser per group so that V
        // is read from LDS at each step instead of being held in registers
        // across the loop (4 NCH CT values per lane)
        int vo = (4 * g) * BP + CT * m;
        asm volatile("" : "+v"(vo));
        d4v acc[CT];
#pragma unroll
        for (int u = 0; u < CT; ++u) acc[u] = d4v{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int kc = 0; kc < NCH; ++kc)
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                // coordinates past d: x, the centre and V are zero (so is the
                // product); points past n only feed output rows that are not stored
                const int k = 16 * kc + 4 * g + s;
                double vb[CT];
#pragma unroll
                for (int u = 0; u < CT; ++u) vb[u] = sV[vo + (16 * kc + s) * BP + u];
                const double xa = (double)xv[kc][s] - sC[k];
#pragma unroll
                for (int u = 0; u < CT; ++u) acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(xa, vb[u], acc[u], 0, 0, 0);
            }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int64_t i = i0 + 4 * r + g;
            if (i >= n) continue;
            float o[CT];
#pragma unroll
            for (int u = 0; u < CT; ++u) {
                double v = acc[u][r] + sU[CT * m + u];
                if (a) v = fma(aw[r], sT[CT * m + u], v);
                o[u] = (float)v;
            }
            if (CT == 4 && vec4) {
                if (CT * m < b) *reinterpret_cast<float4*>(Out + i * b + CT * m) = make_float4(o[0], o[1], o[2], o[3]);
            } else {
#pragma unroll
                for (int u = 0; u < CT; ++u)
                    if (CT * m + u < b) Out[i * b + CT * m + u] = o[u];
            }
        }
        grp = grp2;
    }
}

// Even-p moments on matrix cores: part[blk][t][k][c] = sum over the
// workgroup's rows j of x~_jk^(t+1) z_jc, t = 0 .. NT-1.  A workgroup owns a
// row range and 64 coordinates; wave w owns the 16 coordinates
// k0 + 16w .. +15 (tile row m is coordinate k0 + 16w + m) and 16 CU columns
// (tile u holds column CU n + u at tile column n, from one load of CU values
// of Z per lane and step; CU as in sf_moments_mfma); the powers of x~ are
// formed once per lane and feed NT CU products.  Needs b % CU == 0 and Z rows
// aligned to 4 CU bytes.  TOT: wave 0 of the first coordinate block also sums
// z over the workgroup's rows into tpart[blk][c] (FP64; every wave of a
// workgroup loads the same Z values).
template <int NT, int CU, bool TOT>
__global__ __launch_bounds__(256) void sf_moments_even_mfma(const float* __restrict__ X,
                                                            const double* __restrict__ centre,
                                                            const float* __restrict__ Z, int64_t n, int32_t d,
                                                            int32_t b, int64_t rows_per_blk, double* __restrict__ part,
                                                            double* __restrict__ tpart)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int m = lane & 15, g = lane >> 4;
    const int kt0 = blockIdx.y * 64 + 16 * w;   // the wave's first coordinate
    const int k = kt0 + m;
    const bool kin = k < d, cin = CU * m < b;
    const double ck = kin ? centre[k] : 0.0;
    d4v acc[NT][CU];
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int u = 0; u < CU; ++u) acc[t][u] = d4v{0.0, 0.0, 0.0, 0.0};
    const int64_t r0 = (int64_t)blockIdx.x * rows_per_blk;
    const int64_t r1 = r0 + rows_per_blk < n ? r0 + rows_per_blk : n;
    // two 4-row steps per iteration; the next iteration's raw values are
    // loaded before this iteration's products
    float xn[2], zn[2][CU];
    const bool tw = TOT && blockIdx.y == 0 && w == 0;
    double t0a[CU];
#pragma unroll
    for (int u = 0; u < CU; ++u) t0a[u] = 0.0;
    auto fetch = [&](int64_t j0) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int64_t j = j0 + 4 * h + g;
            xn[h] = 0.0f;
#pragma unroll
            for (int u = 0; u < CU; ++u) zn[h][u] = 0.0f;
            if (j < r1) {
                if (kin) xn[h] = X[j * d + k];
                if (cin) {
                    const Vec<float, CU> q = *reinterpret_cast<const Vec<float, CU>*>(Z + j * b + CU * m);
#pragma unroll
                    for (int u = 0; u < CU; ++u) zn[h][u] = q.v[u];
                }
            }
        }
    };
    fetch(r0);
    for (int64_t j0 = r0; j0 < r1; j0 += 8) {   // the same trip count on every lane
        double x[2], z[2][CU];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            x[h] = (double)xn[h];
#pragma unroll
            for (int u = 0; u < CU; ++u) z[h][u] = (double)zn[h][u];
        }
        if (tw) {   // rows past the range hold z = 0
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int u = 0; u < CU; ++u) t0a[u] += z[h][u];
        }
        if (j0 + 8 < r1) fetch(j0 + 8);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const double xh = (j0 + 4 * h + g < r1 && kin) ? x[h] - ck : 0.0;
            double xt = xh;
#pragma unroll
            for (int t = 0; t < NT; ++t) {
#pragma unroll
                for (int u = 0; u < CU; ++u)
                    acc[t][u] = __builtin_amdgcn_mfma_f64_16x16x4f64(xt, z[h][u], acc[t][u], 0, 0, 0);
                xt *= xh;
            }
        }
    }
    if (tw) {
        // the four row lanes g of a column group, added in a fixed xor order
#pragma unroll
        for (int u = 0; u < CU; ++u) {
            t0a[u] += __shfl_xor(t0a[u], 16);
            t0a[u] += __shfl_xor(t0a[u], 32);
            const int c = CU * m + u;
            if (g == 0 && c < b) tpart[(size_t)blockIdx.x * b + c] = t0a[u];
        }
    }
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int u = 0; u < CU; ++u)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int kk = kt0 + 4 * r + g, c = CU * m + u;
                if (kk < d && c < b) part[(((size_t)blockIdx.x * NT + t) * d + kk) * b + c] = acc[t][u][r];
            }
}

// Even-p point pass on matrix cores: Out[i][c] = sum_k sum_(t=0..P)
// x~_ik^(P-t) G_t[k][c], with G_0[k][c] = T0[c] and G_t (t >= 1) the scaled
// moments.  A workgroup of 8 waves takes 128 points at a time (16 per wave,
// every column in CT tiles of 16); the moments of a chunk of 16 coordinates
// are staged in LDS for all 8 waves between two barriers.  Within a chunk
// lane (m, g) holds coordinates k0 + 4g .. +3 of point i0 + m, and step s
// multiplies the A column g = coordinate k0 + 4g + s, once per power.
template <int P, int CT>
__global__ __launch_bounds__(512) void sf_apply_even_mfma(const float* __restrict__ X,
                                                          const double* __restrict__ centre, int64_t n, int32_t d,
                                                          int32_t b, const double* __restrict__ T0,
                                                          const double* __restrict__ G, float* __restrict__ Out)
{
    __shared__ double sG[P][16][16 * CT];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int m = lane & 15, g = lane >> 4;
    const size_t per_t = (size_t)d * b;
    const bool vec = d % 4 == 0;
    double t0[CT];
#pragma unroll
    for (int u = 0; u < CT; ++u) t0[u] = 16 * u + m < b ? T0[16 * u + m] : 0.0;
    for (int64_t base = (int64_t)blockIdx.x * 128; base < n; base += (int64_t)gridDim.x * 128) {   // uniform
        const int64_t i0 = base + 16 * w, ia = i0 + m;
        d4v acc[CT];
#pragma unroll
        for (int u = 0; u < CT; ++u) acc[u] = d4v{0.0, 0.0, 0.0, 0.0};
        for (int k0 = 0; k0 < d; k0 += 16) {
            __syncthreads();   // every wave is done with the previous chunk
            for (int e = threadIdx.x; e < P * 16 * 16 * CT; e += 512) {
                const int t = e / (16 * 16 * CT), rem = e % (16 * 16 * CT);
                const int kk = rem / (16 * CT), c = rem % (16 * CT);
                sG[t][kk][c] = (k0 + kk < d && c < b) ? G[t * per_t + (size_t)(k0 + kk) * b + c] : 0.0;
            }
            __syncthreads();
            const int kq = k0 + 4 * g;
            float xv[4] = {0.0f, 0.0f, 0.0f, 0.0f};
            if (ia < n) {
                if (vec) {
                    if (kq < d) {
                        const Vec<float, 4> q = *reinterpret_cast<const Vec<float, 4>*>(X + ia * d + kq);
#pragma unroll
                        for (int s2 = 0; s2 < 4; ++s2) xv[s2] = q.v[s2];
                    }
                } else {
#pragma unroll
                    for (int s2 = 0; s2 < 4; ++s2)
                        if (kq + s2 < d) xv[s2] = X[ia * d + kq + s2];
                }
            }
#pragma unroll
            for (int st = 0; st < 4; ++st) {
                const int kk = kq + st;
                const double xa = kk < d ? (double)xv[st] - centre[kk] : 0.0;
                double pw[P + 1];   // pw[e] = xa^e
                pw[0] = 1.0;
#pragma unroll
                for (int e = 1; e <= P; ++e) pw[e] = pw[e - 1] * xa;
#pragma unroll
                for (int u = 0; u < CT; ++u) acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(pw[P], t0[u], acc[u], 0, 0, 0);
#pragma unroll
                for (int t = 1; t <= P; ++t)
#pragma unroll
                    for (int u = 0; u < CT; ++u)
                        acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(pw[P - t], sG[t - 1][4 * g + st][16 * u + m],
                                                                      acc[u], 0, 0, 0);
            }
        }
#pragma unroll
        for (int u = 0; u < CT; ++u) {
            const int c = 16 * u + m;
            if (c >= b) continue;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t i = i0 + 4 * r + g;
                if (i < n) Out[i * b + c] = (float)acc[u][r];
            }
        }
    }
}

// ---- per-point weights at preparation --------------------------------------
// negH[i] = sum_k x_ik log x_ik and LX[i][k] = log x_ik (FP64); flags |= bad
// for a coordinate that is not finite and positive (its logarithm is not finite)
__global__ __launch_bounds__(256) void kl_weights_kernel(const float* __restrict__ X, int64_t n, int32_t d,
                                                         double* __restrict__ negH, double* __restrict__ LX,
                                                         uint32_t* __restrict__ flags, uint32_t bad)
{
    constexpr int PR = 64, KC = 32;
    __shared__ double sT[PR][KC + 1];
    const int tid = threadIdx.x;
    const int64_t i0 = (int64_t)blockIdx.x * PR;
    double s = 0.0;
    bool fault = false;
    for (int k0 = 0; k0 < d; k0 += KC) {
        for (int e = tid; e < PR * KC; e += 256) {
            const int p = e / KC, kk = e % KC;
            const int64_t i = i0 + p;
            double v = 0.0;
            if (i < n && k0 + kk < d) {
                const double x = (double)X[i * d + k0 + kk];
                if (x > 0.0 && x <= 3.4028234663852886e38) {
                    const double lx = log(x);
                    LX[i * d + k0 + kk] = lx;
                    v = x * lx;
                } else {
                    fault = true;
                }
            }
            sT[p][kk] = v;
        }
        __syncthreads();
        if (tid < PR)
            for (int kk = 0; kk < KC; ++kk) s += sT[tid][kk];
        __syncthreads();
    }
    if (tid < PR && i0 + tid < n) negH[i0 + tid] = s;
    if (fault) atomicOr(flags, bad);
}

// q[i] = x~_i^T M x~_i, x~ = x - c.  A workgroup owns 64 points and walks 64
// rows of M at a time: P = X~ M_rows^T from LDS tiles (32 coordinates per
// step, 4 x 4 outputs per thread), then q += sum over the rows of x~_ik P_ik.
__global__ __launch_bounds__(256) void maha_weights_kernel(const float* __restrict__ X, const double* __restrict__ centre,
                                                           int64_t n, int32_t d, const double* __restrict__ M,
                                                           double* __restrict__ q)
{
    constexpr int PR = 64, MR = 64, LC = 32;
    __shared__ double sX[PR][LC + 1];
    __shared__ double sM[MR][LC + 1];
    const int tid = threadIdx.x;
    const int64_t i0 = (int64_t)blockIdx.x * PR;
    const int tr = (tid / 16) * 4, tc = (tid % 16) * 4;
    double qa[4] = {0.0, 0.0, 0.0, 0.0};
    for (int m0 = 0; m0 < d; m0 += MR) {
        double acc[4][4];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
        for (int l0 = 0; l0 < d; l0 += LC) {
            for (int e = tid; e < PR * LC; e += 256) {
                const int p = e / LC, l = e % LC;
                const int64_t i = i0 + p;
                sX[p][l] = (i < n && l0 + l < d) ? (double)X[i * d + l0 + l] - centre[l0 + l] : 0.0;
            }
            for (int e = tid; e < MR * LC; e += 256) {
                const int r = e / LC, l = e % LC;
                sM[r][l] = (m0 + r < d && l0 + l < d) ? M[(size_t)(m0 + r) * d + l0 + l] : 0.0;
            }
            __syncthreads();
#pragma unroll 4
            for (int l = 0; l < LC; ++l) {
                double xa[4], ma[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    xa[i] = sX[tr + i][l];
                    ma[i] = sM[tc + i][l];
                }
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int j = 0; j < 4; ++j) acc[i][j] = fma(xa[i], ma[j], acc[i][j]);
            }
            __syncthreads();
        }
        // acc[i][j] = (M x~_(tr+i))_(m0+tc+j)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int64_t row = i0 + tr + i;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int k = m0 + tc + j;
                if (row < n && k < d) qa[i] = fma((double)X[row * d + k] - centre[k], acc[i][j], qa[i]);
            }
        }
    }
    // the 16 threads of a row group hold disjoint parts of the same 4 sums
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int off = 8; off >= 1; off >>= 1) qa[i] += __shfl_xor(qa[i], off, 16);
    if (tid % 16 == 0) {
#pragma unroll
        for (int i = 0; i < 4; ++i)
            if (i0 + tr + i < n) q[i0 + tr + i] = qa[i];
    }
}

// ---- host side --------------------------------------------------------------
int pad_bw(int32_t b) {
    int w = 1;
    while (w < b) w <<= 1;
    return w;
}

template <int NT>
constexpr int moments_kc() { return MKG * moments_kpt<NT>(); }

int kc_for(int nt) { return nt == 1 ? moments_kc<1>() : nt <= 4 ? moments_kc<4>() : moments_kc<6>(); }

// the narrow moments kernel (all sums of a thread in registers) serves b <= 8
// when the NT x (b rounded up) x V sums fit (b = 16 measured no faster than
// the LDS-tiled kernel)
constexpr bool narrow_fits(int nt, int bw, int v = 1) { return bw <= 8 && nt * bw * v <= 32; }

// coordinates per thread of the narrow moments kernel: 16-byte loads when d
// allows and the sums fit
int narrow_vec(int nt, int32_t b, int32_t d, int xbytes) {
    const int bw = pad_bw(b);
    const int vmax = 16 / xbytes;
    for (int v = vmax; v > 1; v >>= 1)
        if (d % v == 0 && narrow_fits(nt, bw, v)) return v;
    return 1;
}

// Moments launch shape: the kernel family, rows per workgroup (about 2048
// workgroups over the grid; the LDS kernel takes whole tiles) and the number
// of row ranges, which sizes the partial sums.
struct MomentsPlan {
    bool narrow;
    int vec;   // coordinates per thread of the narrow kernel
    int64_t rpb, nblk;
    unsigned kblk;
};
MomentsPlan moments_plan(int64_t n, int32_t d, int32_t b, int nt, int xbytes) {
    MomentsPlan pl;
    pl.narrow = narrow_fits(nt, pad_bw(b));
    pl.vec = pl.narrow ? narrow_vec(nt, b, d, xbytes) : 1;
    const int kc = pl.narrow ? 256 * pl.vec : kc_for(nt);
    pl.kblk = (unsigned)((d + kc - 1) / kc);
    int64_t want = 2048 / (int64_t)pl.kblk;
    if (want < 1) want = 1;
    int64_t r = (n + want - 1) / want;
    if (!pl.narrow) r = (r + MSR - 1) / MSR * MSR;
    if (r < 1) r = 1;
    pl.rpb = r;
    pl.nblk = (n + r - 1) / r;
    return pl;
}

template <typename XT, typename ZT, typename ACC, int NT, int BW>
hipError_t moments_bw(const void* X, const void* centre, const void* Z, int64_t n, int32_t d, int32_t b, void* part,
                      int64_t* nblk_out, hipStream_t s)
{
    const MomentsPlan pl = moments_plan(n, d, b, NT, (int)sizeof(XT));
    *nblk_out = pl.nblk;
    dim3 grid((unsigned)pl.nblk, pl.kblk);
    if constexpr (narrow_fits(NT, BW)) {
        if (pl.narrow) {
            constexpr int V4 = 16 / (int)sizeof(XT);
            if constexpr (V4 >= 4 && narrow_fits(NT, BW, 4)) {
                if (pl.vec == 4) {
                    sf_moments_narrow<XT, ZT, ACC, NT, BW, 4><<<grid, 256, 0, s>>>(
                        (const XT*)X, (const ACC*)centre, (const ZT*)Z, n, d, b, pl.rpb, (ACC*)part);
                    return hipGetLastError();
                }
            }
            if constexpr (V4 >= 2 && narrow_fits(NT, BW, 2)) {
                if (pl.vec == 2) {
                    sf_moments_narrow<XT, ZT, ACC, NT, BW, 2><<<grid, 256, 0, s>>>(
                        (const XT*)X, (const ACC*)centre, (const ZT*)Z, n, d, b, pl.rpb, (ACC*)part);
                    return hipGetLastError();
                }
            }
            sf_moments_narrow<XT, ZT, ACC, NT, BW, 1><<<grid, 256, 0, s>>>(
                (const XT*)X, (const ACC*)centre, (const ZT*)Z, n, d, b, pl.rpb, (ACC*)part);
            return hipGetLastError();
        }
    }
    sf_moments_kernel<XT, ZT, ACC, NT, BW><<<grid, 256, 0, s>>>(
        (const XT*)X, (const ACC*)centre, (const ZT*)Z, n, d, b, pl.rpb, (ACC*)part);
    return hipGetLastError();
}

template <typename XT, typename ZT, typename ACC, int NT>
hipError_t moments_t(int32_t b, const void* X, const void* centre, const void* Z, int64_t n, int32_t d, void* part,
                     int64_t* nblk, hipStream_t s)
{
    switch (pad_bw(b)) {
    case 1: return moments_bw<XT, ZT, ACC, NT, 1>(X, centre, Z, n, d, b, part, nblk, s);
    case 2: return moments_bw<XT, ZT, ACC, NT, 2>(X, centre, Z, n, d, b, part, nblk, s);
    case 4: return moments_bw<XT, ZT, ACC, NT, 4>(X, centre, Z, n, d, b, part, nblk, s);
    case 8: return moments_bw<XT, ZT, ACC, NT, 8>(X, centre, Z, n, d, b, part, nblk, s);
    case 16: return moments_bw<XT, ZT, ACC, NT, 16>(X, centre, Z, n, d, b, part, nblk, s);
    case 32: return moments_bw<XT, ZT, ACC, NT, 32>(X, centre, Z, n, d, b, part, nblk, s);
    case 64: return moments_bw<XT, ZT, ACC, NT, 64>(X, centre, Z, n, d, b, part, nblk, s);
    default: return hipErrorInvalidValue;
    }
}

template <typename XT, typename ACC, typename OT, int NT, bool EVEN, int BW>
hipError_t apply_bw(const void* X, const void* centre, int64_t n, int32_t d, int32_t b, const void* T0, const void* G,
                    const double* a, const double* U, void* Out, hipStream_t s)
{
    constexpr int NPB = (256 / BW) * apply_ppt<BW>();
    const unsigned grid = (unsigned)((n + NPB - 1) / NPB);
    sf_apply_kernel<XT, ACC, OT, NT, EVEN, BW><<<grid, 256, 0, s>>>((const XT*)X, (const ACC*)centre, n, d, b,
                                                                   (const ACC*)T0, (const ACC*)G, a, U, (OT*)Out);
    return hipGetLastError();
}

template <typename XT, typename ACC, typename OT, int NT, bool EVEN>
hipError_t apply_t(const void* X, const void* centre, int64_t n, int32_t d, int32_t b, const void* T0, const void* G,
                   const double* a, const double* U, void* Out, hipStream_t s)
{
    switch (pad_bw(b)) {
    case 1: return apply_bw<XT, ACC, OT, NT, EVEN, 1>(X, centre, n, d, b, T0, G, a, U, Out, s);
    case 2: return apply_bw<XT, ACC, OT, NT, EVEN, 2>(X, centre, n, d, b, T0, G, a, U, Out, s);
    case 4: return apply_bw<XT, ACC, OT, NT, EVEN, 4>(X, centre, n, d, b, T0, G, a, U, Out, s);
    case 8: return apply_bw<XT, ACC, OT, NT, EVEN, 8>(X, centre, n, d, b, T0, G, a, U, Out, s);
    case 16: return apply_bw<XT, ACC, OT, NT, EVEN, 16>(X, centre, n, d, b, T0, G, a, U, Out, s);
    case 32: return apply_bw<XT, ACC, OT, NT, EVEN, 32>(X, centre, n, d, b, T0, G, a, U, Out, s);
    case 64: return apply_bw<XT, ACC, OT, NT, EVEN, 64>(X, centre, n, d, b, T0, G, a, U, Out, s);
    default: return hipErrorInvalidValue;
    }
}

template <typename ACC>
hipError_t reduce_launch(const void* part, int64_t nblk, int64_t per_t, int nt, int p, double alpha, void* G,
                         void* slices, hipStream_t s)
{
    const int64_t count = per_t * nt;
    if (count < 2048) {   // narrow blocks: one launch
        sf_reduce_waves<ACC><<<(unsigned)((count + 3) / 4), 256, 0, s>>>((const ACC*)part, (int)nblk, per_t, nt, p,
                                                                         alpha, (ACC*)G);
        return hipGetLastError();
    }
    const int nsl = (int)(nblk < SF_SLICES ? nblk : SF_SLICES);
    const int ks = (int)((nblk + nsl - 1) / nsl);
    dim3 g1((unsigned)((count + 255) / 256), (unsigned)nsl);
    sf_reduce_slices<ACC><<<g1, 256, 0, s>>>((const ACC*)part, (int)nblk, count, ks, (ACC*)slices);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    sf_reduce_kernel<ACC><<<(unsigned)((count + 255) / 256), 256, 0, s>>>((const ACC*)slices, nsl, per_t, nt, p,
                                                                          alpha, (ACC*)G);
    return hipGetLastError();
}

// Columns per lane of the matrix-core moments for a block of b columns: 1 for
// 4 <= b <= 16, 2 for even b <= 32, 4 for b % 4 == 0 (0: not served).
int mfma_moment_cu(int32_t b) {
    if (b < 4) return 0;
    if (b <= 16) return 1;
    if (b <= 32) return b % 2 == 0 ? 2 : 0;
    return b % 4 == 0 ? 4 : 0;
}
// The matrix-core moments serve the single-moment forms at d % 4 == 0 (16-byte
// loads of X) and the b above; Z must also be aligned to 4 CU bytes.
bool mfma_moments_fit(int form, int32_t d, int32_t b) {
    return form != SF_EVEN && d % 4 == 0 && mfma_moment_cu(b) > 0;
}
bool mfma_moments_aligned(const void* Z, int32_t b) {
    return (uintptr_t)Z % (4 * (uintptr_t)mfma_moment_cu(b)) == 0;
}
// even p (float data) on matrix cores: the b of mfma_moment_cu from b = 8 (Z
// aligned to 4 CU bytes); at b = 4 the vector moments measured faster (l6
// 0.50 against 0.54 ms per query at n = 2^20, d = 64)
bool even_mfma_fit(int32_t b) { return b >= 8 && mfma_moment_cu(b) > 0; }
// row ranges of the even-p matrix-core moments: about 2048 workgroups
int64_t even_mfma_blocks(int64_t n, int32_t d) {
    const int64_t ky = (d + 63) / 64;
    int64_t blk = 2048 / ky;
    const int64_t steps = (n + 3) / 4;
    if (blk > steps) blk = steps;
    return blk < 1 ? 1 : blk;
}
// waves of the matrix-core moments along the rows: about 2048 over the grid
int64_t mfma_row_waves(int64_t n, int32_t d) {
    const int64_t ky = (d + 63) / 64;
    int64_t w = 2048 / ky;
    const int64_t steps = (n + 3) / 4;
    if (w > steps) w = steps;
    return w < 4 ? 4 : (w + 3) / 4 * 4;
}
template <int P>
hipError_t even_query(bool is_int, int zkind, const SfQuery& q, char* part, char* G, char* SL, double* tpart,
                      double* GT, hipStream_t s)
{
    int64_t nblk = 0;
    hipError_t e;
    const int64_t per_t = (int64_t)q.d * q.b;
    // fused totals: the matrix-core moments also sum z (T0 of the query)
    const bool fuse = q.status != nullptr;
    const double* T0q = (const double*)q.T0;
    if (!is_int) {
        if (fuse && !(even_mfma_fit(q.b) && mfma_moments_aligned(q.Z, q.b))) return hipErrorInvalidValue;
        if (even_mfma_fit(q.b) && mfma_moments_aligned(q.Z, q.b)) {
            const int64_t blk = even_mfma_blocks(q.n, q.d);
            const int64_t rpb = ((q.n + blk - 1) / blk + 3) / 4 * 4;
            const int64_t nb = (q.n + rpb - 1) / rpb;
            dim3 grid((unsigned)nb, (unsigned)((q.d + 63) / 64));
            const float* Xf = (const float*)q.X;
            const double* cen = (const double*)q.centre;
            const float* Zf = (const float*)q.Z;
#define SF_EVEN_MOM(CU, TOT)                                                                                        \
    sf_moments_even_mfma<P, CU, TOT><<<grid, 256, 0, s>>>(Xf, cen, Zf, q.n, q.d, q.b, rpb, (double*)part, tpart)
            switch (mfma_moment_cu(q.b) * 2 + (fuse ? 1 : 0)) {
            case 2: SF_EVEN_MOM(1, false); break;
            case 3: SF_EVEN_MOM(1, true); break;
            case 4: SF_EVEN_MOM(2, false); break;
            case 5: SF_EVEN_MOM(2, true); break;
            case 9: SF_EVEN_MOM(4, true); break;
            default: SF_EVEN_MOM(4, false); break;
            }
#undef SF_EVEN_MOM
            e = hipGetLastError();
            nblk = nb;
            if (e == hipSuccess && fuse) {
                // sum z over the row blocks (fixed order), then the finiteness check
                if ((e = reduce_launch<double>(tpart, nb, (int64_t)q.b, 1, 0, 1.0, GT, SL, s)) != hipSuccess)
                    return e;
                sf_check_finite<<<1, 64, 0, s>>>(GT, q.b, q.status);
                e = hipGetLastError();
                T0q = GT;
            }
        } else {
            e = moments_t<float, float, double, P>(q.b, q.X, q.centre, q.Z, q.n, q.d, part, &nblk, s);
        }
        if (e != hipSuccess) return e;
        if ((e = reduce_launch<double>(part, nblk, per_t, P, P, 1.0, G, SL, s)) != hipSuccess) return e;
        // matrix cores for the point pass from b = 8: a 16-column tile costs
        // the same at any b <= 16, the vector pass grows with b (the two meet
        // near b = 6 at n = 2^20, d = 64)
        if (q.b >= 8) {
            int64_t blocks = (q.n + 127) / 128;
            if (blocks > 1024) blocks = 1024;
            const unsigned gb = (unsigned)blocks;
            const float* Xf = (const float*)q.X;
            const double* cen = (const double*)q.centre;
            const double* T0 = T0q;
            const double* Gd = (const double*)G;
            float* O = (float*)q.Out;
            switch ((q.b + 15) / 16) {
            case 1: sf_apply_even_mfma<P, 1><<<gb, 512, 0, s>>>(Xf, cen, q.n, q.d, q.b, T0, Gd, O); break;
            case 2: sf_apply_even_mfma<P, 2><<<gb, 512, 0, s>>>(Xf, cen, q.n, q.d, q.b, T0, Gd, O); break;
            case 3: sf_apply_even_mfma<P, 3><<<gb, 512, 0, s>>>(Xf, cen, q.n, q.d, q.b, T0, Gd, O); break;
            default: sf_apply_even_mfma<P, 4><<<gb, 512, 0, s>>>(Xf, cen, q.n, q.d, q.b, T0, Gd, O); break;
            }
            return hipGetLastError();
        }
        return apply_t<float, double, float, P, true>(q.X, q.centre, q.n, q.d, q.b, T0q, G, nullptr, nullptr, q.Out,
                                                      s);
    }
    if (zkind == IN_I32)
        e = moments_t<int32_t, int32_t, int64_t, P>(q.b, q.X, q.centre, q.Z, q.n, q.d, part, &nblk, s);
    else
        e = moments_t<int32_t, int64_t, int64_t, P>(q.b, q.X, q.centre, q.Z, q.n, q.d, part, &nblk, s);
    if (e != hipSuccess) return e;
    if ((e = reduce_launch<int64_t>(part, nblk, per_t, P, P, 1.0, G, SL, s)) != hipSuccess) return e;
    return apply_t<int32_t, int64_t, int64_t, P, true>(q.X, q.centre, q.n, q.d, q.b, q.T0, G, nullptr, nullptr,
                                                       q.Out, s);
}

}  // namespace

int sf_moment_count(int form, int p) { return form == SF_EVEN ? p : 1; }

namespace {

// row-range partials the moments stage may write
int64_t partial_count(int64_t n, int32_t d, int32_t b, int form, int nt) {
    int64_t nb = moments_plan(n, d, b, nt, form == SF_LOG ? 8 : 4).nblk;
    if (mfma_moments_fit(form, d, b)) nb = std::max(nb, mfma_row_waves(n, d));
    if (form == SF_EVEN && even_mfma_fit(b)) nb = std::max(nb, even_mfma_blocks(n, d));
    return nb;
}

}  // namespace

size_t sf_scratch_bytes(int64_t n, int32_t d, int32_t b, int form, int p) {
    const int nt = sf_moment_count(form, p);
    const int64_t nblk = partial_count(n, d, b, form, nt);
    const size_t cnt = (size_t)nt * d * b;
    // row-range partials, the moments, the mixed moments, slices; then the
    // totals' partials and the totals
    return ((size_t)nblk + 2 + SF_SLICES) * cnt * 8 + ((size_t)nblk + 1) * 2 * (size_t)b * 8;
}

bool sf_fuses_totals(int form, bool is_int, int32_t d, int32_t b, const void* Z) {
    if (form == SF_EVEN) return !is_int && even_mfma_fit(b) && mfma_moments_aligned(Z, b);
    return !is_int && mfma_moments_fit(form, d, b) && mfma_moments_aligned(Z, b);
}

hipError_t launch_sf_query(int form, int p, bool is_int, int zkind, const SfQuery& q, void* scratch, hipStream_t s)
{
    if (q.b < 1 || q.b > 64 || q.n < 1 || q.d < 1) return hipErrorInvalidValue;
    const int nt = sf_moment_count(form, p);
    const int64_t nblk_max = partial_count(q.n, q.d, q.b, form, nt);
    const size_t cnt = (size_t)nt * q.d * q.b;
    char* part = (char*)scratch;
    char* G = part + (size_t)nblk_max * cnt * 8;
    char* V = G + cnt * 8;
    char* SL = V + cnt * 8;
    double* tpart = (double*)(SL + (size_t)SF_SLICES * cnt * 8);
    double* GT = tpart + (size_t)nblk_max * 2 * q.b;
    if (form == SF_EVEN) {
        switch (p) {
        case 2: return even_query<2>(is_int, zkind, q, part, G, SL, tpart, GT, s);
        case 4: return even_query<4>(is_int, zkind, q, part, G, SL, tpart, GT, s);
        case 6: return even_query<6>(is_int, zkind, q, part, G, SL, tpart, GT, s);
        default: return hipErrorInvalidValue;
        }
    }
    if (is_int) return hipErrorInvalidValue;
    int64_t nblk = 0;
    const int64_t per_t = (int64_t)q.d * q.b;
    // KL and cross entropy: moments of the logarithms kept since preparation
    hipError_t e;
    const bool fuse = q.status != nullptr;
    if (fuse && !sf_fuses_totals(form, is_int, q.d, q.b, q.Z)) return hipErrorInvalidValue;
    const double* T0q = (const double*)q.T0;
    const double* Uq = q.U;
    if (mfma_moments_fit(form, q.d, q.b) && mfma_moments_aligned(q.Z, q.b)) {
        const int cu = mfma_moment_cu(q.b);
        const int64_t waves = mfma_row_waves(q.n, q.d);
        const int64_t rpw = ((q.n + waves - 1) / waves + 3) / 4 * 4;
        dim3 grid((unsigned)(waves / 4), (unsigned)((q.d + 63) / 64));
#define SF_MOMENTS_CU(XT, XP, CP, TOT, CU)                                                                         \
    sf_moments_mfma<XT, SF_MOM_DEPTH, TOT, CU><<<grid, 256, 0, s>>>(XP, CP, (const float*)q.Z, q.n, q.d, q.b, rpw, \
                                                                     (double*)part, q.wu, tpart)
#define SF_MOMENTS(XT, XP, CP, TOT)                                                                                \
    do {                                                                                                           \
        if (cu == 1) SF_MOMENTS_CU(XT, XP, CP, TOT, 1);                                                            \
        else if (cu == 2) SF_MOMENTS_CU(XT, XP, CP, TOT, 2);                                                       \
        else SF_MOMENTS_CU(XT, XP, CP, TOT, 4);                                                                    \
    } while (0)
        if (form == SF_LOG) {
            if (fuse) SF_MOMENTS(double, q.LX, nullptr, true);
            else SF_MOMENTS(double, q.LX, nullptr, false);
        } else {
            if (fuse) SF_MOMENTS(float, (const float*)q.X, (const double*)q.centre, true);
            else SF_MOMENTS(float, (const float*)q.X, (const double*)q.centre, false);
        }
#undef SF_MOMENTS
#undef SF_MOMENTS_CU
        e = hipGetLastError();
        nblk = waves / 4;   // one partial per workgroup
        if (e == hipSuccess && fuse) {
            // sum z and sum w z over the waves (fixed order), then the finiteness check
            if ((e = reduce_launch<double>(tpart, waves, 2 * (int64_t)q.b, 1, 0, 1.0, GT, SL, s)) != hipSuccess)
                return e;
            sf_check_finite<<<1, 64, 0, s>>>(GT, q.b, q.status);
            e = hipGetLastError();
            T0q = GT;
            Uq = q.wu ? GT + q.b : nullptr;
        }
    } else {
        e = (form == SF_LOG)
                ? moments_t<double, float, double, 1>(q.b, q.LX, nullptr, q.Z, q.n, q.d, part, &nblk, s)
                : moments_t<float, float, double, 1>(q.b, q.X, q.centre, q.Z, q.n, q.d, part, &nblk, s);
    }
    if (e != hipSuccess) return e;
    const char* Gv = G;
    if (q.W) {
        if ((e = reduce_launch<double>(part, nblk, per_t, 1, 0, 1.0, G, SL, s)) != hipSuccess) return e;
        sf_mix_kernel<<<(unsigned)((per_t + 255) / 256), 256, 0, s>>>(q.W, (const double*)G, q.d, q.b, (double*)V);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        Gv = V;
    } else {
        if ((e = reduce_launch<double>(part, nblk, per_t, 1, 0, q.alpha, G, SL, s)) != hipSuccess) return e;
    }
    const double* cen = form == SF_LOG ? nullptr : (const double*)q.centre;
    if (q.b >= 4) {   // matrix cores: 16 points x every column per wave (masked past b)
        const int64_t groups = (q.n + 15) / 16;
        int64_t blocks = (groups + 7) / 8;
        if (blocks > 1024) blocks = 1024;
        const unsigned gb = (unsigned)blocks;
        const float* Xf = (const float*)q.X;
        const double* T0 = T0q;
        const double* Vd = (const double*)Gv;
        float* O = (float*)q.Out;
        const size_t vbytes = (size_t)q.d * q.b * 8;
        const bool lds = vbytes <= 65536;
        const size_t shm = lds ? vbytes : 0;
        // whole groups in flight where d allows (V and the centres in LDS)
        const bool grp = q.d % 4 == 0 && q.d <= 64;
#define SF_APPLY_GRP(CT, NCH)                                                                                         \
    sf_apply_mfma_grp<CT, NCH><<<gb, 512, ((size_t)16 * (NCH) * (16 * (CT) + 1) + 32 * (CT)) * 8, s>>>(          \
        Xf, cen, q.n, q.d, q.b, T0, Vd, q.a, Uq, O)
#define SF_APPLY_MFMA(CT)                                                                                           \
    do {                                                                                                            \
        if (grp) {                                                                                                  \
            switch ((q.d + 15) / 16) {                                                                              \
            case 1: SF_APPLY_GRP(CT, 1); break;                                                                     \
            case 2: SF_APPLY_GRP(CT, 2); break;                                                                     \
            case 3: SF_APPLY_GRP(CT, 3); break;                                                                     \
            default: SF_APPLY_GRP(CT, 4); break;                                                                    \
            }                                                                                                       \
        } else if (lds)                                                                                             \
            sf_apply_mfma<CT, true><<<gb, 512, shm, s>>>(Xf, cen, q.n, q.d, q.b, T0, Vd, q.a, Uq, O);         \
        else                                                                                                        \
            sf_apply_mfma<CT, false><<<2 * gb, 256, 0, s>>>(Xf, cen, q.n, q.d, q.b, T0, Vd, q.a, Uq, O);      \
    } while (0)
        switch ((q.b + 15) / 16) {
        case 1: SF_APPLY_MFMA(1); break;
        case 2: SF_APPLY_MFMA(2); break;
        case 3: SF_APPLY_MFMA(3); break;
        default: SF_APPLY_MFMA(4); break;
        }
#undef SF_APPLY_MFMA
#undef SF_APPLY_GRP
        return hipGetLastError();
    }
    return apply_t<float, double, float, 1, false>(q.X, cen, q.n, q.d, q.b, T0q, Gv, q.a, Uq, q.Out, s);
}

hipError_t launch_kl_weights(const float* X, int64_t n, int32_t d, double* negH, double* LX, uint32_t* flags,
                             uint32_t bad, hipStream_t s)
{
    if (n < 1 || d < 1) return hipErrorInvalidValue;
    kl_weights_kernel<<<(unsigned)((n + 63) / 64), 256, 0, s>>>(X, n, d, negH, LX, flags, bad);
    return hipGetLastError();
}

hipError_t launch_maha_weights(const float* X, const double* centre, int64_t n, int32_t d, const double* M, double* q,
                               hipStream_t s)
{
    if (n < 1 || d < 1) return hipErrorInvalidValue;
    maha_weights_kernel<<<(unsigned)((n + 63) / 64), 256, 0, s>>>(X, centre, n, d, M, q);
    return hipGetLastError();
}

}  // namespace dm
