// k_lp.hip - the l_p^p query for odd p >= 3 (the odd-p theorem of Appendix
// A.1: the sort of Algorithm 1 plus prefix sums of powers; the paper omits
// the proof).
//
// For odd p, |a - b|^p = sign(a - b) (a - b)^p, and the binomial expansion
// (a - b)^p = sum_t C(p, t) a^(p-t) (-b)^t gives, in coordinate k with the
// sorted order of Algorithm 1 and inclusive prefix sums
//     P_t(r) = sum_{r' <= r} z[perm[r']] xs[r']^t,   T_t = P_t(n - 1),
// the coordinate's share of (A z) at point perm[r] (x = xs[r]):
//     sum_t C(p, t) (-1)^t x^(p-t) (2 P_t(r) - T_t).
// Points before r (and ties, whose difference is 0) enter with a plus sign,
// points after with a minus sign.  For p = 1 this is the l1 pass.  As there,
// the t = p terms summed over k give sum_j w_j z_j with w_j = sum_k x_jk^p
// (added once, by the first pass), while T_0 = sum z is shared by all
// coordinates and T_1 .. T_(p-1) come from a separate moments kernel.
//
// The pass: one persistent launch per coordinate, tiles of NS * R ranks held
// in registers, the p + 1 running sums chained between tiles by the
// decoupled look-back of the l1 pass (records of p + 1 values per column),
// and the combine evaluated by Horner's rule in x.  Float data carries the
// chained sums as double-float pairs; integer data runs in wrapping int64
// (exact modulo 2^64; the overflow guard uses sum_k range_k^p).
#include <hip/hip_runtime.h>

#include <type_traits>

#include "dm_device.h"
#include "dm_internal.h"
#include "l1_common.h"

namespace dm {
namespace {

using namespace l1;

constexpr int64_t binom(int p, int t) {
    int64_t r = 1;
    for (int i = 0; i < t; ++i) r = r * (p - i) / (i + 1);
    return r;
}
// C(p, t) (-1)^t
constexpr int64_t lp_coef(int p, int t) { return (t % 2 ? -1 : 1) * binom(p, t); }

// ---------------------------------------------------------------------------
// moments: M[t-1][k][c] = sum_j z_jc x_jk^t for t = 1 .. p-1.  A workgroup
// takes a range of rows and a group of 16 coordinates; tiles of 64 rows of
// X and Z go through LDS; each thread owns (coordinate, column) pairs and
// keeps their p - 1 sums.  Partial sums per row range are added in order by
// the second stage.  FP64 for float data, wrapping int64 for integer data.
// ---------------------------------------------------------------------------
constexpr int MK = 16;     // coordinates per workgroup
constexpr int MROWS = 64;  // rows per LDS tile
constexpr int MPAIR = 4;   // (coordinate, column) pairs per thread (MK * 64 / 256)

template <typename XT, typename ZT, typename ACC, int PM>
__global__ __launch_bounds__(256) void lp_moments_stage1(const XT* __restrict__ X, const ZT* __restrict__ Z, int64_t n,
                                                         int32_t d, int32_t b, int64_t rows_per_blk,
                                                         ACC* __restrict__ part)
{
    constexpr int NT = PM - 1;   // moments t = 1 .. p-1
    __shared__ ACC sX[MROWS][MK];
    __shared__ ACC sZ[MROWS][65];
    const int tid = threadIdx.x;
    const int k0 = blockIdx.y * MK;
    const int64_t rb = (int64_t)blockIdx.x * rows_per_blk;
    const int64_t re = rb + rows_per_blk < n ? rb + rows_per_blk : n;
    ACC acc[MPAIR][NT];
#pragma unroll
    for (int q = 0; q < MPAIR; ++q)
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[q][t] = ACC(0);
    for (int c0 = 0; c0 < b; c0 += 64) {
        for (int64_t r0 = rb; r0 < re; r0 += MROWS) {
            const int nr = (int)(re - r0 < MROWS ? re - r0 : MROWS);
            for (int e = tid; e < MROWS * MK; e += 256) {
                const int r = e / MK, kk = e % MK;
                sX[r][kk] = (r < nr && k0 + kk < d) ? (ACC)X[(r0 + r) * d + k0 + kk] : ACC(0);
            }
            for (int e = tid; e < MROWS * 64; e += 256) {
                const int r = e / 64, cc = e % 64;
                sZ[r][cc] = (r < nr && c0 + cc < b) ? (ACC)Z[(r0 + r) * b + c0 + cc] : ACC(0);
            }
            __syncthreads();
#pragma unroll
            for (int q = 0; q < MPAIR; ++q) {
                const int pair = tid + 256 * q;   // MK * 64 pairs
                const int kk = pair / 64, cc = pair % 64;
                for (int r = 0; r < nr; ++r) {
                    const ACC x = sX[r][kk], z = sZ[r][cc];
                    ACC xt = x;
#pragma unroll
                    for (int t = 0; t < NT; ++t) {
                        if constexpr (std::is_same<ACC, double>::value) {
                            acc[q][t] = fma(xt, z, acc[q][t]);
                            xt = xt * x;
                        } else {
                            acc[q][t] = (ACC)((uint64_t)acc[q][t] + (uint64_t)xt * (uint64_t)z);
                            xt = (ACC)((uint64_t)xt * (uint64_t)x);
                        }
                    }
                }
            }
            __syncthreads();
        }
        // write this column group's partials: part[blk][t][k][c]
#pragma unroll
        for (int q = 0; q < MPAIR; ++q) {
            const int pair = tid + 256 * q;
            const int kk = pair / 64, cc = pair % 64;
            if (k0 + kk < d && c0 + cc < b) {
#pragma unroll
                for (int t = 0; t < NT; ++t)
                    part[(((size_t)blockIdx.x * NT + t) * d + k0 + kk) * b + c0 + cc] = acc[q][t];
            }
#pragma unroll
            for (int t = 0; t < NT; ++t) acc[q][t] = ACC(0);
        }
    }
}

// M[t][k][c] = sum over row blocks (in order) of part[blk][t][k][c]
template <typename ACC>
__global__ __launch_bounds__(256) void lp_moments_stage2(const ACC* __restrict__ part, int nblk, size_t count,
                                                         ACC* __restrict__ M)
{
    const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= count) return;
    ACC s = ACC(0);
    for (int k = 0; k < nblk; ++k) {
        if constexpr (std::is_same<ACC, double>::value)
            s += part[(size_t)k * count + e];
        else
            s = (ACC)((uint64_t)s + (uint64_t)part[(size_t)k * count + e]);
    }
    M[e] = s;
}

// ---------------------------------------------------------------------------
// arithmetic of the combine: FP32 with the chained sums rounded once from
// double-float to FP32; wrapping int64 for integer data
// ---------------------------------------------------------------------------
__device__ __forceinline__ float lp_mul(float v, float x) { return v * x; }
__device__ __forceinline__ int64_t lp_mul(int64_t v, int32_t x) {
    return (int64_t)((uint64_t)v * (uint64_t)(int64_t)x);
}
template <typename P> __device__ __forceinline__ typename P::O lp_fin(typename P::C bt, typename P::T Tt) {
    if constexpr (std::is_same<P, FloatPath>::value)
        return (float)(2.0 * dd_to_f64(bt) - Tt);
    else
        return (int64_t)(2ull * (uint64_t)bt - (uint64_t)Tt);
}
template <typename P> __device__ __forceinline__ typename P::O lp_u(typename P::T u) {
    return (typename P::O)u;
}
// coef (D + 2 l)
template <typename P> __device__ __forceinline__ typename P::O lp_term(int64_t coef, typename P::O D, typename P::L l) {
    if constexpr (std::is_same<P, FloatPath>::value)
        return (float)coef * fmaf(2.0f, l, D);
    else
        return (int64_t)((uint64_t)coef * ((uint64_t)D + 2ull * (uint64_t)l));
}
// h x + coef (D + 2 l)
template <typename P>
__device__ __forceinline__ typename P::O lp_horner(typename P::O h, typename P::X x, int64_t coef, typename P::O D,
                                                   typename P::L l) {
    if constexpr (std::is_same<P, FloatPath>::value)
        return fmaf(h, x, (float)coef * fmaf(2.0f, l, D));
    else
        return (int64_t)((uint64_t)h * (uint64_t)(int64_t)x + (uint64_t)coef * ((uint64_t)D + 2ull * (uint64_t)l));
}

// ---------------------------------------------------------------------------
// the pass of one coordinate for odd p (NM = p + 1 running sums)
// ---------------------------------------------------------------------------
// VEC: 16-byte accesses to the Z and Out rows (b % 4 == 0, 16-byte aligned
// rows), as in the l1 pass; the same values either way.  p = 3 is held to
// three waves per SIMD (168 registers, one spilled): the pass waits on
// memory and the look-back, and the third wave took it from 3.01 to 2.81 ms
// at n = 2^22, d = 128, b = 64; p = 5 would spill a dozen registers (its pass
// then took 9.90 ms against 8.66 ms) and keeps two.
template <typename P, int BP, int NM, int R, bool VEC>
__global__ __launch_bounds__(256, NM <= 4 ? 3 : 2) void lp_pass_kernel(
    const uint32_t* __restrict__ perm, const typename P::X* __restrict__ xs, int64_t n,
    const typename P::Z* __restrict__ Z, typename P::O* __restrict__ Out, int32_t b,
    const typename P::T* __restrict__ T0, const typename P::T* __restrict__ Mk, int64_t mstride,
    const typename P::T* __restrict__ U, int first, uint64_t* __restrict__ ticket_ctr, int64_t ntiles,
    uint64_t* __restrict__ rec, uint64_t* __restrict__ stat, uint32_t* __restrict__ status)
{
    using L = typename P::L;
    using C = typename P::C;
    using Ly = Lay<BP>;
    constexpr int PW = NM - 1;   // p
    constexpr int CPL = Ly::CPL, LPR = Ly::LPR, RPW = Ly::RPW, NS = Ly::NS;
    constexpr int TILE = NS * R;
    constexpr int WPR = NM * BP * P::WPV;

    __shared__ uint64_t s_ticket;
    __shared__ L s_wtot[4][NM][BP];
    __shared__ C s_wexcl[4][NM][BP];
    __shared__ C s_tot[NM][BP];
    __shared__ C s_carry[NM][BP];
    __shared__ C s_lb[4][NM][BP];

    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int slot = w * RPW + lane / LPR;
    const int col0 = (lane % LPR) * CPL;
    const uint64_t per_pass = (uint64_t)ntiles + gridDim.x;
    if (tid == 0) s_ticket = atomicAdd((unsigned long long*)ticket_ctr, 1ull);
    __syncthreads();
    uint64_t ticket = s_ticket;

    for (;;) {
        const uint64_t tile = ticket % per_pass;
        if (tile >= (uint64_t)ntiles) break;
        const uint32_t tag = (uint32_t)((ticket / per_pass) % 0xffffffffull) + 1u;
        const int64_t r0 = (int64_t)tile * TILE + (int64_t)slot * R;

        uint32_t pr[R];
        typename P::X x[R];
        typename P::Z g[R][CPL];
#pragma unroll
        for (int i = 0; i < R; ++i) {
            const bool valid = r0 + i < n;
            pr[i] = valid ? perm[r0 + i] : 0u;
            x[i] = valid ? xs[r0 + i] : typename P::X(0);
        }
#pragma unroll
        for (int i = 0; i < R; ++i) load_row<CPL, VEC>(Z + (size_t)pr[i] * b, col0, b, r0 + i < n, g[i]);

        // thread sums of z x^t, then the wave's exclusive prefix over slots
        L e[NM][CPL];
#pragma unroll
        for (int j = 0; j < CPL; ++j) {
            L a[NM];
#pragma unroll
            for (int t = 0; t < NM; ++t) a[t] = P::lzero();
#pragma unroll
            for (int i = 0; i < R; ++i) {
                L v = P::ladd(P::lzero(), g[i][j]);   // z x^0
#pragma unroll
                for (int t = 0; t < NM; ++t) {
                    a[t] = P::lsum(a[t], v);
                    v = lp_mul(v, x[i]);
                }
            }
#pragma unroll
            for (int t = 0; t < NM; ++t) {
                L s = a[t];
#pragma unroll
                for (int off = LPR; off < DM_WAVE; off <<= 1) {
                    const L u = P::shfl_up(s, off);
                    if (lane >= off) s = P::lsum(s, u);
                }
                const L xsh = P::shfl_up(s, LPR);
                e[t][j] = lane >= LPR ? xsh : P::lzero();
                if (lane >= DM_WAVE - LPR) s_wtot[w][t][col0 + j] = s;
            }
        }
        __syncthreads();
        // NM * BP entries (up to 384: more than one per thread)
        for (int e = tid; e < NM * BP; e += 256) {
            const int t = e / BP, c = e % BP;
            C acc = P::czero();
#pragma unroll
            for (int ww = 0; ww < 4; ++ww) {
                s_wexcl[ww][t][c] = acc;
                acc = P::caddl(acc, s_wtot[ww][t][c]);
            }
            s_tot[t][c] = acc;
            P::put(rec + ((size_t)tile * 2 + (tile == 0 ? 1 : 0)) * WPR + (c * NM + t) * P::WPV, acc, tag);
        }
        __syncthreads();
        if (tid == 0) publish_word(stat + tile, tag_word(tag, tile == 0 ? 2u : 1u));

        C cc[NM];
        look_back_wg<P, BP, NM, 2>(rec, stat, (int64_t)tile - 1, tag, tid, s_lb, cc, status);
        if (w == 0) {
            const int c = lane;
            if (c < BP) {
#pragma unroll
                for (int t = 0; t < NM; ++t) {
                    s_carry[t][c] = cc[t];
                    if (tile > 0)
                        P::put(rec + ((size_t)tile * 2 + 1) * WPR + (c * NM + t) * P::WPV, P::cadd(cc[t], s_tot[t][c]),
                               tag);
                }
            }
            if (tile > 0 && lane == 0) publish_word(stat + tile, tag_word(tag, 2u));
        }
        __syncthreads();

        // D_t = 2 (prefix before this thread's first rank) - T_t, with T_p
        // left out (it is in U) and T_0 shared by all coordinates
        typename P::O D[NM][CPL];
#pragma unroll
        for (int j = 0; j < CPL; ++j) {
            const int c = col0 + j;
#pragma unroll
            for (int t = 0; t < NM; ++t) {
                if (c < b) {
                    const C bt = P::caddl(P::cadd(s_carry[t][c], s_wexcl[w][t][c]), e[t][j]);
                    const typename P::T Tt = t == 0 ? T0[c] : t < PW ? Mk[(size_t)(t - 1) * mstride + c]
                                                                     : typename P::T(0);
                    D[t][j] = lp_fin<P>(bt, Tt);
                } else {
                    D[t][j] = typename P::O(0);
                }
            }
        }
        L l[NM][CPL];
#pragma unroll
        for (int t = 0; t < NM; ++t)
#pragma unroll
            for (int j = 0; j < CPL; ++j) l[t][j] = P::lzero();
#pragma unroll
        for (int i = 0; i < R; ++i) {
            typename P::O o[CPL];
            if (!first) {
                load_row<CPL, VEC>(Out + (size_t)pr[i] * b, col0, b, r0 + i < n, o);
            } else {
#pragma unroll
                for (int j = 0; j < CPL; ++j) o[j] = col0 + j < b ? lp_u<P>(U[col0 + j]) : typename P::O(0);
            }
            typename P::O res[CPL];
#pragma unroll
            for (int j = 0; j < CPL; ++j) {
                // running sums including rank r0 + i, and the Horner combine
                L v = P::ladd(P::lzero(), g[i][j]);
#pragma unroll
                for (int t = 0; t < NM; ++t) {
                    l[t][j] = P::lsum(l[t][j], v);
                    v = lp_mul(v, x[i]);
                }
                typename P::O h = lp_term<P>(lp_coef(PW, 0), D[0][j], l[0][j]);
#pragma unroll
                for (int t = 1; t < NM; ++t) h = lp_horner<P>(h, x[i], lp_coef(PW, t), D[t][j], l[t][j]);
                res[j] = P::oadd(o[j], h);
            }
            if (r0 + i < n) store_row<CPL, VEC>(Out + (size_t)pr[i] * b, col0, b, res);
        }
        if (tid == 0) s_ticket = atomicAdd((unsigned long long*)ticket_ctr, 1ull);
        __syncthreads();
        ticket = s_ticket;
        __syncthreads();
    }
}

// ranks per slot: NM running sums per column are kept in registers
template <int NM> constexpr int lp_r() { return NM <= 4 ? 4 : 2; }
template <int BP, int NM> constexpr int lp_tile() { return Lay<BP>::NS * lp_r<NM>(); }

inline int lp_bpad(int32_t b) {
    int bp = 1;
    while (bp < b) bp <<= 1;
    return bp;
}

template <typename P, int BP, int NM>
hipError_t lp_launch_bp(const LpPassArgs& a, int32_t b, hipStream_t s) {
    constexpr int R = lp_r<NM>();
    constexpr int TILE = lp_tile<BP, NM>();
    const int64_t ntiles = (a.n + TILE - 1) / TILE;
    if ((size_t)ntiles * (2 * (size_t)NM * P::WPV * BP + 1) > a.record_words) return hipErrorInvalidValue;
    uint64_t* stat = a.records + (size_t)ntiles * 2 * NM * P::WPV * BP;
    // one grid for both row-access forms (the ticket count of a pass is
    // ntiles + grid, so every pass of a shape must launch the same grid)
    const int64_t grid = persistent_grid((const void*)lp_pass_kernel<P, BP, NM, R, false>,
                                         (const void*)lp_pass_kernel<P, BP, NM, R, true>, ntiles);
    const bool vec = (b % 4 == 0) && ((uintptr_t)a.Z % 16 == 0) && ((uintptr_t)a.Out % 16 == 0);
#define LP_PASS(V)                                                                                                  \
    lp_pass_kernel<P, BP, NM, R, V><<<(unsigned)grid, 256, 0, s>>>(                                                  \
        a.perm, (const typename P::X*)a.xs, a.n, (const typename P::Z*)a.Z, (typename P::O*)a.Out, b,               \
        (const typename P::T*)a.T0, (const typename P::T*)a.Mk, a.mstride, (const typename P::T*)a.U, a.first,        \
        &a.chain->ticket[a.cls], ntiles, a.records, stat, a.status)
    if (vec) LP_PASS(true);
    else LP_PASS(false);
#undef LP_PASS
    return hipGetLastError();
}

template <typename P, int NM>
hipError_t lp_launch(const LpPassArgs& a, int32_t b, hipStream_t s) {
    switch (lp_bpad(b)) {
    case 1: return lp_launch_bp<P, 1, NM>(a, b, s);
    case 2: return lp_launch_bp<P, 2, NM>(a, b, s);
    case 4: return lp_launch_bp<P, 4, NM>(a, b, s);
    case 8: return lp_launch_bp<P, 8, NM>(a, b, s);
    case 16: return lp_launch_bp<P, 16, NM>(a, b, s);
    case 32: return lp_launch_bp<P, 32, NM>(a, b, s);
    case 64: return lp_launch_bp<P, 64, NM>(a, b, s);
    default: return hipErrorInvalidValue;
    }
}

template <int NM> int lp_tile_of(int32_t b) {
    switch (lp_bpad(b)) {
    case 1: return lp_tile<1, NM>();
    case 2: return lp_tile<2, NM>();
    case 4: return lp_tile<4, NM>();
    case 8: return lp_tile<8, NM>();
    case 16: return lp_tile<16, NM>();
    case 32: return lp_tile<32, NM>();
    default: return lp_tile<64, NM>();
    }
}

constexpr int64_t LP_MROWS_PER_BLK = 32768;

template <typename XT, typename ZT, typename ACC, int PM>
hipError_t lp_moments_t(const void* Xc, const void* Z, int64_t n, int32_t d, int32_t b, void* part, void* M,
                        hipStream_t s) {
    constexpr int NT = PM - 1;
    const int64_t nblk = (n + LP_MROWS_PER_BLK - 1) / LP_MROWS_PER_BLK;
    dim3 grid((unsigned)nblk, (unsigned)((d + MK - 1) / MK));
    lp_moments_stage1<XT, ZT, ACC, PM><<<grid, 256, 0, s>>>((const XT*)Xc, (const ZT*)Z, n, d, b, LP_MROWS_PER_BLK,
                                                           (ACC*)part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const size_t count = (size_t)NT * d * b;
    lp_moments_stage2<ACC><<<(unsigned)((count + 255) / 256), 256, 0, s>>>((const ACC*)part, (int)nblk, count, (ACC*)M);
    return hipGetLastError();
}

template <int PM>
hipError_t lp_moments_p(bool is_int, int zkind, const void* Xc, const void* Z, int64_t n, int32_t d, int32_t b,
                        void* part, void* M, hipStream_t s) {
    if (!is_int) return lp_moments_t<float, float, double, PM>(Xc, Z, n, d, b, part, M, s);
    if (zkind == IN_I32) return lp_moments_t<int32_t, int32_t, int64_t, PM>(Xc, Z, n, d, b, part, M, s);
    return lp_moments_t<int32_t, int64_t, int64_t, PM>(Xc, Z, n, d, b, part, M, s);
}

}  // namespace

int lp_tile_ranks(int32_t b, int p) { return p == 3 ? lp_tile_of<4>(b) : lp_tile_of<6>(b); }

size_t lp_record_words(int64_t n, int32_t b, bool is_int, int p) {
    const int64_t tile = lp_tile_ranks(b, p);
    const int64_t ntiles = (n + tile - 1) / tile;
    const size_t wpv = is_int ? 2 : 1;
    return (size_t)ntiles * (2 * (size_t)(p + 1) * wpv * (size_t)lp_bpad(b) + 1);
}

size_t lp_moments_bytes(int64_t n, int32_t d, int32_t b, int p) {
    const int64_t nblk = (n + LP_MROWS_PER_BLK - 1) / LP_MROWS_PER_BLK;
    return ((size_t)nblk + 1) * (size_t)(p - 1) * d * b * 8;   // partials, then the moments
}

hipError_t launch_lp_moments(bool is_int, int zkind, int p, const void* Xc, const void* Z, int64_t n, int32_t d,
                             int32_t b, void* scratch, void** M, hipStream_t s) {
    if (b < 1 || b > 64 || (p != 3 && p != 5)) return hipErrorInvalidValue;
    const int64_t nblk = (n + LP_MROWS_PER_BLK - 1) / LP_MROWS_PER_BLK;
    char* part = (char*)scratch;
    *M = part + (size_t)nblk * (p - 1) * d * b * 8;
    if (p == 3) return lp_moments_p<3>(is_int, zkind, Xc, Z, n, d, b, part, *M, s);
    return lp_moments_p<5>(is_int, zkind, Xc, Z, n, d, b, part, *M, s);
}

hipError_t launch_lp_pass(bool is_int, int zkind, int p, int32_t b, const LpPassArgs& a, hipStream_t s) {
    if (b < 1 || b > 64) return hipErrorInvalidValue;
    if (a.cls < 0 || a.cls >= CHAIN_CLASSES) return hipErrorInvalidValue;
    if (p == 3) {
        if (!is_int) return lp_launch<FloatPath, 4>(a, b, s);
        if (zkind == IN_I32) return lp_launch<IntPath<int32_t>, 4>(a, b, s);
        return lp_launch<IntPath<int64_t>, 4>(a, b, s);
    }
    if (p == 5) {
        if (!is_int) return lp_launch<FloatPath, 6>(a, b, s);
        if (zkind == IN_I32) return lp_launch<IntPath<int32_t>, 6>(a, b, s);
        return lp_launch<IntPath<int64_t>, 6>(a, b, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace dm
