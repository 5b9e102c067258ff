// k_l1.hip - the l1 query (Algorithm 2, Section 2) for b right-hand sides.
//
// For one coordinate k with sorted order perm and sorted values xs, and
// inclusive prefix sums in that order
//     P0(r) = sum_{r' <= r} z[perm[r']],   P1(r) = sum_{r' <= r} xs[r'] z[perm[r']],
// the coordinate's share of (A z) at point perm[r] is
//     xs[r] (2 P0(r) - T0) - (2 P1(r) - T1)
// (the S1..S4 split of the exactness proof, with S1 = P1, S2 = T1 - P1,
// S3 = P0 and S4 = T0 - P0; the point's own term is zero, so including it in
// the prefix changes nothing).  Summed over k the T1 terms give
// U = sum_j s_j z_j with s_j = sum_k x_jk, so each pass adds
//     c = xs (2 P0 - T0) - 2 P1
// to Out[perm[r]] and the first pass also adds U.
//
// Algorithm 2 materialises the prefix arrays B_i and C_i and looks positions
// up per point; here the two loops are fused into one pass per coordinate:
// the sorted order is walked once, the prefixes live in registers, and each
// result is scattered to its point's row.  Every pass visits each row of Out
// exactly once (perm is a permutation), so passes are stream-ordered and a
// pass needs no atomics on Out.
//
// One pass = one launch, one tile of TILE consecutive ranks per workgroup.
// Tiles take indices from a ticket counter in dispatch order and chain their
// prefixes with a decoupled look-back over tagged 64-bit words.  Float data
// carries the prefixes between threads, waves and tiles as double-float
// (hi, lo) FP32 pairs; inside a thread the short runs are plain FP32 relative
// to that carry.  Integer data runs in wrapping int64, which is exact modulo
// 2^64.
#include <type_traits>

#include "dm_device.h"
#include "dm_internal.h"
#include "l1_common.h"

namespace dm {
namespace {

using namespace l1;

template <typename P, int BP, int R, int SUB, int OC, bool VEC>
__global__ __launch_bounds__(256, 2) void l1_pass_kernel(
    const uint32_t* __restrict__ perm, const typename P::X* __restrict__ xs, int64_t n,
    const typename P::Z* __restrict__ Z, typename P::O* __restrict__ Out, int32_t b,
    const typename P::T* __restrict__ T0, const typename P::T* __restrict__ U, int first,
    uint64_t* __restrict__ ticket_ctr, int cls, int64_t ntiles,
    uint64_t* __restrict__ rec, uint64_t* __restrict__ stat)
{
    using L = typename P::L;
    using C = typename P::C;
    using Ly = Lay<BP>;
    constexpr int CPL = Ly::CPL, LPR = Ly::LPR, RPW = Ly::RPW, NS = Ly::NS;
    constexpr int CHUNK = NS * R;       // ranks per sub-chunk (one register load per slot)
    constexpr int TILE = CHUNK * SUB;   // ranks per tile
    constexpr int WPR = 2 * BP * P::WPV;   // words per record: (P0, P1) per column, every column of BP
    static_assert(R % OC == 0, "Out chunk must divide the ranks per slot");

    __shared__ uint64_t s_ticket;
    __shared__ C s_red[4][2][BP];
    __shared__ C s_tot[2][BP];
    __shared__ L s_wtot[4][2][BP];
    __shared__ C s_wexcl[4][2][BP];
    __shared__ C s_run[2][BP];

    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int slot = w * RPW + lane / LPR;
    const int col0 = (lane % LPR) * CPL;
    // Each workgroup takes tiles in ticket order until it draws one of the G
    // tickets past the last tile, so a pass consumes ntiles + G tickets.
    const uint64_t per_pass = (uint64_t)ntiles + gridDim.x;
    if (tid == 0) s_ticket = atomicAdd((unsigned long long*)ticket_ctr, 1ull);
    __syncthreads();
    uint64_t ticket = s_ticket;

    for (;;) {
        const uint64_t tile = ticket % per_pass;
        if (tile >= (uint64_t)ntiles) break;
        // nonzero pass tag; every word a pass reads is rewritten by that pass,
        // so only the previous pass's words can be stale and they carry another tag
        const uint32_t tag = (uint32_t)((ticket / per_pass) % 0xffffffffull) + 1u;
        const int64_t tbase = (int64_t)tile * TILE + (int64_t)slot * R;

        // ================= phase 1: the tile's totals =================
        C t0[CPL], t1[CPL];
#pragma unroll
        for (int j = 0; j < CPL; ++j) { t0[j] = P::czero(); t1[j] = P::czero(); }
        for (int s = 0; s < SUB; ++s) {
            const int64_t r0 = tbase + (int64_t)s * CHUNK;
            uint32_t p[R];
            typename P::X x[R];
            typename P::Z g[R][CPL];
#pragma unroll
            for (int i = 0; i < R; ++i) {
                const bool valid = r0 + i < n;
                p[i] = valid ? perm[r0 + i] : 0u;
                x[i] = valid ? xs[r0 + i] : typename P::X(0);
            }
#pragma unroll
            for (int i = 0; i < R; ++i) load_row<CPL, VEC>(Z + (size_t)p[i] * b, col0, b, r0 + i < n, g[i]);
#pragma unroll
            for (int j = 0; j < CPL; ++j) {
                L a0 = P::lzero(), a1 = P::lzero();
#pragma unroll
                for (int i = 0; i < R; ++i) {
                    a0 = P::ladd(a0, g[i][j]);
                    a1 = P::lmac(a1, x[i], g[i][j]);
                }
                t0[j] = P::caddl(t0[j], a0);
                t1[j] = P::caddl(t1[j], a1);
            }
        }
        // sum over the slots of the wave (lanes that share columns), then the waves
#pragma unroll
        for (int j = 0; j < CPL; ++j) {
#pragma unroll
            for (int off = LPR; off < DM_WAVE; off <<= 1) {
                t0[j] = P::cadd(t0[j], P::cshfl_xor(t0[j], off));
                t1[j] = P::cadd(t1[j], P::cshfl_xor(t1[j], off));
            }
            if (lane < LPR) {
                s_red[w][0][col0 + j] = t0[j];
                s_red[w][1][col0 + j] = t1[j];
            }
        }
        __syncthreads();
        if (tid < 2 * BP) {
            const int qt = tid / BP, c = tid % BP;
            const C acc = P::cadd(P::cadd(s_red[0][qt][c], s_red[1][qt][c]), P::cadd(s_red[2][qt][c], s_red[3][qt][c]));
            s_tot[qt][c] = acc;
            // every column of BP is written each pass (padding columns hold zeros),
            // so no word of a record can outlive the pass that wrote it
            P::put(rec + ((size_t)tile * 2 + (tile == 0 ? 1 : 0)) * WPR + (c * 2 + qt) * P::WPV, acc, tag);
        }
        __syncthreads();
        if (tid == 0) publish_word(stat + tile, tag_word(tag, tile == 0 ? 2u : 1u));

        // ================= decoupled look-back (wave 0) =================
        // the exclusive prefix of the tile, then its inclusive record
        C c0, c1;
        look_back_wg<P, BP, WPR>(rec, stat, (int64_t)tile - 1, tag, tid, s_red, c0, c1);
        if (w == 0) {
            const int c = lane;
            const bool act = c < BP;
            if (act) {
                s_run[0][c] = c0;
                s_run[1][c] = c1;
                if (tile > 0) {
                    uint64_t* dst = rec + ((size_t)tile * 2 + 1) * WPR + c * 2 * P::WPV;
                    P::put(dst, P::cadd(c0, s_tot[0][c]), tag);
                    P::put(dst + P::WPV, P::cadd(c1, s_tot[1][c]), tag);
                }
            }
            if (tile > 0 && lane == 0) publish_word(stat + tile, tag_word(tag, 2u));
        }
        __syncthreads();

        // ================= phase 2: scan and scatter, sub-chunk by sub-chunk =================
        // The Z rows are read a second time; they were fetched moments ago in
        // phase 1 and are normally still in the memory-side cache.
        for (int s = 0; s < SUB; ++s) {
            const int64_t r0 = tbase + (int64_t)s * CHUNK;
            uint32_t p[R];
            typename P::X x[R];
            typename P::Z g[R][CPL];
#pragma unroll
            for (int i = 0; i < R; ++i) {
                const bool valid = r0 + i < n;
                p[i] = valid ? perm[r0 + i] : 0u;
                x[i] = valid ? xs[r0 + i] : typename P::X(0);
            }
#pragma unroll
            for (int i = 0; i < R; ++i) load_row<CPL, VEC>(Z + (size_t)p[i] * b, col0, b, r0 + i < n, g[i]);

            L e0[CPL], e1[CPL];
#pragma unroll
            for (int j = 0; j < CPL; ++j) {
                L i0 = P::lzero(), i1 = P::lzero();
#pragma unroll
                for (int i = 0; i < R; ++i) {
                    i0 = P::ladd(i0, g[i][j]);
                    i1 = P::lmac(i1, x[i], g[i][j]);
                }
#pragma unroll
                for (int off = LPR; off < DM_WAVE; off <<= 1) {
                    const L u0 = P::shfl_up(i0, off), u1 = P::shfl_up(i1, off);
                    if (lane >= off) { i0 = P::lsum(i0, u0); i1 = P::lsum(i1, u1); }
                }
                const L x0 = P::shfl_up(i0, LPR), x1 = P::shfl_up(i1, LPR);
                e0[j] = lane >= LPR ? x0 : P::lzero();
                e1[j] = lane >= LPR ? x1 : P::lzero();
                if (lane >= DM_WAVE - LPR) {
                    s_wtot[w][0][col0 + j] = i0;
                    s_wtot[w][1][col0 + j] = i1;
                }
            }
            __syncthreads();
            if (tid < 2 * BP) {
                const int qt = tid / BP, c = tid % BP;
                C acc = s_run[qt][c];
#pragma unroll
                for (int ww = 0; ww < 4; ++ww) {
                    s_wexcl[ww][qt][c] = acc;
                    acc = P::caddl(acc, s_wtot[ww][qt][c]);
                }
                s_run[qt][c] = acc;
            }
            __syncthreads();

            typename P::Fin f[CPL];
#pragma unroll
            for (int j = 0; j < CPL; ++j) {
                const int c = col0 + j;
                if (c < b) {
                    const C b0 = P::caddl(s_wexcl[w][0][c], e0[j]);
                    const C b1 = P::caddl(s_wexcl[w][1][c], e1[j]);
                    f[j] = P::fin(b0, b1, T0[c], first ? U[c] : typename P::T(0));
                } else {
                    f[j] = P::fin(P::czero(), P::czero(), typename P::T(0), typename P::T(0));
                }
            }
            L l0[CPL], l1[CPL];
#pragma unroll
            for (int j = 0; j < CPL; ++j) { l0[j] = P::lzero(); l1[j] = P::lzero(); }
#pragma unroll
            for (int i0 = 0; i0 < R; i0 += OC) {
                typename P::O o[OC][CPL];
#pragma unroll
                for (int i = 0; i < OC; ++i) {
                    if (!first) {
                        load_row<CPL, VEC>(Out + (size_t)p[i0 + i] * b, col0, b, r0 + i0 + i < n, o[i]);
                    } else {
#pragma unroll
                        for (int j = 0; j < CPL; ++j) o[i][j] = P::ufirst(f[j]);
                    }
                }
#pragma unroll
                for (int i = 0; i < OC; ++i) {
                    typename P::O res[CPL];
#pragma unroll
                    for (int j = 0; j < CPL; ++j) {
                        l0[j] = P::ladd(l0[j], g[i0 + i][j]);
                        l1[j] = P::lmac(l1[j], x[i0 + i], g[i0 + i][j]);
                        res[j] = P::oadd(o[i][j], P::out(l0[j], l1[j], x[i0 + i], f[j]));
                    }
                    if (r0 + i0 + i < n) store_row<CPL, VEC>(Out + (size_t)p[i0 + i] * b, col0, b, res);
                }
            }
        }
        if (tid == 0) s_ticket = atomicAdd((unsigned long long*)ticket_ctr, 1ull);
        __syncthreads();
        ticket = s_ticket;
        __syncthreads();
    }
}

// Variant that keeps the whole tile on chip: a tile is two sub-chunks; the
// first is staged in LDS (as per-thread storage) and the second stays in
// registers, so phase 2 reads no Z row twice.  Used where the staging fits.
template <typename P, int BP, int R, int OC, bool VEC>
__global__ __launch_bounds__(256, 2) void l1_pass_keep_kernel(
    const uint32_t* __restrict__ perm, const typename P::X* __restrict__ xs, int64_t n,
    const typename P::Z* __restrict__ Z, typename P::O* __restrict__ Out, int32_t b,
    const typename P::T* __restrict__ T0, const typename P::T* __restrict__ U, int first,
    uint64_t* __restrict__ ticket_ctr, int cls, int64_t ntiles,
    uint64_t* __restrict__ rec, uint64_t* __restrict__ stat)
{
    using L = typename P::L;
    using C = typename P::C;
    using Ly = Lay<BP>;
    constexpr int CPL = Ly::CPL, LPR = Ly::LPR, RPW = Ly::RPW, NS = Ly::NS;
    constexpr int CHUNK = NS * R;       // ranks per sub-chunk (one register load per slot)
    constexpr int SUB = 2;
    constexpr int TILE = CHUNK * SUB;   // ranks per tile
    constexpr int WPR = 2 * BP * P::WPV;   // words per record: (P0, P1) per column, every column of BP
    static_assert(R % OC == 0, "Out chunk must divide the ranks per slot");

    __shared__ uint64_t s_ticket;
    __shared__ C s_red[4][2][BP];   // phase 1 wave sums, then look-back scratch, then phase 2 wave prefixes
    __shared__ C s_tot[2][BP];
    __shared__ L s_wtot[4][2][BP];
    C (*const s_wexcl)[2][BP] = s_red;
    __shared__ C s_run[2][BP];
    __shared__ typename P::Z s_g[R][256][CPL];   // sub-chunk 0 of the tile, per thread
    __shared__ uint32_t s_p[SUB][NS][R];
    __shared__ typename P::X s_x[SUB][NS][R];

    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int slot = w * RPW + lane / LPR;
    const int col0 = (lane % LPR) * CPL;
    // Each workgroup takes tiles in ticket order until it draws one of the G
    // tickets past the last tile, so a pass consumes ntiles + G tickets.
    const uint64_t per_pass = (uint64_t)ntiles + gridDim.x;
    if (tid == 0) s_ticket = atomicAdd((unsigned long long*)ticket_ctr, 1ull);
    __syncthreads();
    uint64_t ticket = s_ticket;

    for (;;) {
        const uint64_t tile = ticket % per_pass;
        if (tile >= (uint64_t)ntiles) break;
        // nonzero pass tag; every word a pass reads is rewritten by that pass,
        // so only the previous pass's words can be stale and they carry another tag
        const uint32_t tag = (uint32_t)((ticket / per_pass) % 0xffffffffull) + 1u;
        const int64_t tbase = (int64_t)tile * TILE + (int64_t)slot * R;

        // ================= phase 1: the tile's totals =================
        C t0[CPL], t1[CPL];
#pragma unroll
        for (int j = 0; j < CPL; ++j) { t0[j] = P::czero(); t1[j] = P::czero(); }
        typename P::Z gk[R][CPL];
#pragma unroll
        for (int s = 0; s < SUB; ++s) {
            const int64_t r0 = tbase + (int64_t)s * CHUNK;
            uint32_t p[R];
            typename P::X x[R];
            typename P::Z g[R][CPL];
#pragma unroll
            for (int i = 0; i < R; ++i) {
                const bool valid = r0 + i < n;
                p[i] = valid ? perm[r0 + i] : 0u;
                x[i] = valid ? xs[r0 + i] : typename P::X(0);
            }
#pragma unroll
            for (int i = 0; i < R; ++i) load_row<CPL, VEC>(Z + (size_t)p[i] * b, col0, b, r0 + i < n, g[i]);
#pragma unroll
            for (int j = 0; j < CPL; ++j) {
                L a0 = P::lzero(), a1 = P::lzero();
#pragma unroll
                for (int i = 0; i < R; ++i) {
                    a0 = P::ladd(a0, g[i][j]);
                    a1 = P::lmac(a1, x[i], g[i][j]);
                }
                t0[j] = P::caddl(t0[j], a0);
                t1[j] = P::caddl(t1[j], a1);
            }
            if (lane % LPR == 0) {
#pragma unroll
                for (int i = 0; i < R; ++i) {
                    s_p[s][slot][i] = p[i];
                    s_x[s][slot][i] = x[i];
                }
            }
            if (s == 0) {
#pragma unroll
                for (int i = 0; i < R; ++i)
#pragma unroll
                    for (int j = 0; j < CPL; ++j) s_g[i][tid][j] = g[i][j];
            } else {
#pragma unroll
                for (int i = 0; i < R; ++i)
#pragma unroll
                    for (int j = 0; j < CPL; ++j) gk[i][j] = g[i][j];
            }
        }
        // sum over the slots of the wave (lanes that share columns), then the waves
#pragma unroll
        for (int j = 0; j < CPL; ++j) {
#pragma unroll
            for (int off = LPR; off < DM_WAVE; off <<= 1) {
                t0[j] = P::cadd(t0[j], P::cshfl_xor(t0[j], off));
                t1[j] = P::cadd(t1[j], P::cshfl_xor(t1[j], off));
            }
            if (lane < LPR) {
                s_red[w][0][col0 + j] = t0[j];
                s_red[w][1][col0 + j] = t1[j];
            }
        }
        __syncthreads();
        if (tid < 2 * BP) {
            const int qt = tid / BP, c = tid % BP;
            const C acc = P::cadd(P::cadd(s_red[0][qt][c], s_red[1][qt][c]), P::cadd(s_red[2][qt][c], s_red[3][qt][c]));
            s_tot[qt][c] = acc;
            // every column of BP is written each pass (padding columns hold zeros),
            // so no word of a record can outlive the pass that wrote it
            P::put(rec + ((size_t)tile * 2 + (tile == 0 ? 1 : 0)) * WPR + (c * 2 + qt) * P::WPV, acc, tag);
        }
        __syncthreads();
        if (tid == 0) publish_word(stat + tile, tag_word(tag, tile == 0 ? 2u : 1u));

        // ================= decoupled look-back (wave 0) =================
        // the exclusive prefix of the tile, then its inclusive record
        C c0, c1;
        look_back_wg<P, BP, WPR>(rec, stat, (int64_t)tile - 1, tag, tid, s_red, c0, c1);
        if (w == 0) {
            const int c = lane;
            const bool act = c < BP;
            if (act) {
                s_run[0][c] = c0;
                s_run[1][c] = c1;
                if (tile > 0) {
                    uint64_t* dst = rec + ((size_t)tile * 2 + 1) * WPR + c * 2 * P::WPV;
                    P::put(dst, P::cadd(c0, s_tot[0][c]), tag);
                    P::put(dst + P::WPV, P::cadd(c1, s_tot[1][c]), tag);
                }
            }
            if (tile > 0 && lane == 0) publish_word(stat + tile, tag_word(tag, 2u));
        }
        __syncthreads();

        // ================= phase 2: scan and scatter, sub-chunk by sub-chunk =================
        // Z rows of sub-chunk 0 come back from LDS, those of sub-chunk 1 from
        // registers; point ids and sorted values of both from LDS
        auto phase2 = [&](const int64_t r0, auto&& getp, auto&& getx, auto&& getg) {
            L e0[CPL], e1[CPL];
#pragma unroll
            for (int j = 0; j < CPL; ++j) {
                L i0 = P::lzero(), i1 = P::lzero();
#pragma unroll
                for (int i = 0; i < R; ++i) {
                    i0 = P::ladd(i0, getg(i, j));
                    i1 = P::lmac(i1, getx(i), getg(i, j));
                }
#pragma unroll
                for (int off = LPR; off < DM_WAVE; off <<= 1) {
                    const L u0 = P::shfl_up(i0, off), u1 = P::shfl_up(i1, off);
                    if (lane >= off) { i0 = P::lsum(i0, u0); i1 = P::lsum(i1, u1); }
                }
                const L x0 = P::shfl_up(i0, LPR), x1 = P::shfl_up(i1, LPR);
                e0[j] = lane >= LPR ? x0 : P::lzero();
                e1[j] = lane >= LPR ? x1 : P::lzero();
                if (lane >= DM_WAVE - LPR) {
                    s_wtot[w][0][col0 + j] = i0;
                    s_wtot[w][1][col0 + j] = i1;
                }
            }
            __syncthreads();
            if (tid < 2 * BP) {
                const int qt = tid / BP, c = tid % BP;
                C acc = s_run[qt][c];
#pragma unroll
                for (int ww = 0; ww < 4; ++ww) {
                    s_wexcl[ww][qt][c] = acc;
                    acc = P::caddl(acc, s_wtot[ww][qt][c]);
                }
                s_run[qt][c] = acc;
            }
            __syncthreads();

            typename P::Fin f[CPL];
#pragma unroll
            for (int j = 0; j < CPL; ++j) {
                const int c = col0 + j;
                if (c < b) {
                    const C b0 = P::caddl(s_wexcl[w][0][c], e0[j]);
                    const C b1 = P::caddl(s_wexcl[w][1][c], e1[j]);
                    f[j] = P::fin(b0, b1, T0[c], first ? U[c] : typename P::T(0));
                } else {
                    f[j] = P::fin(P::czero(), P::czero(), typename P::T(0), typename P::T(0));
                }
            }
            L l0[CPL], l1[CPL];
#pragma unroll
            for (int j = 0; j < CPL; ++j) { l0[j] = P::lzero(); l1[j] = P::lzero(); }
#pragma unroll
            for (int i0 = 0; i0 < R; i0 += OC) {
                typename P::O o[OC][CPL];
#pragma unroll
                for (int i = 0; i < OC; ++i) {
                    if (!first) {
                        load_row<CPL, VEC>(Out + (size_t)getp(i0 + i) * b, col0, b, r0 + i0 + i < n, o[i]);
                    } else {
#pragma unroll
                        for (int j = 0; j < CPL; ++j) o[i][j] = P::ufirst(f[j]);
                    }
                }
#pragma unroll
                for (int i = 0; i < OC; ++i) {
                    typename P::O res[CPL];
#pragma unroll
                    for (int j = 0; j < CPL; ++j) {
                        l0[j] = P::ladd(l0[j], getg(i0 + i, j));
                        l1[j] = P::lmac(l1[j], getx(i0 + i), getg(i0 + i, j));
                        res[j] = P::oadd(o[i][j], P::out(l0[j], l1[j], getx(i0 + i), f[j]));
                    }
                    if (r0 + i0 + i < n) store_row<CPL, VEC>(Out + (size_t)getp(i0 + i) * b, col0, b, res);
                }
            }
        };
        phase2(
            tbase, [&](int i) { return s_p[0][slot][i]; }, [&](int i) { return s_x[0][slot][i]; },
            [&](int i, int j) { return s_g[i][tid][j]; });
        phase2(
            tbase + CHUNK, [&](int i) { return s_p[1][slot][i]; }, [&](int i) { return s_x[1][slot][i]; },
            [&](int i, int j) { return gk[i][j]; });
        if (tid == 0) s_ticket = atomicAdd((unsigned long long*)ticket_ctr, 1ull);
        __syncthreads();
        ticket = s_ticket;
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// totals: T0[c] = sum_j z_jc, U[c] = sum_j w_j z_jc, and ||z_c||_1
// two fixed-order stages (per-block partials, then one block), so FP64
// results are reproducible run to run.
// ---------------------------------------------------------------------------
constexpr int TOT_ROWS = 4096;  // rows per stage-1 block
constexpr int TOT_MAXB = 1024;

template <bool INT, typename ZT, typename WT>
__global__ __launch_bounds__(256) void totals_stage1(const ZT* __restrict__ Z, int64_t n, int32_t b,
                                                     const WT* __restrict__ wgt, void* __restrict__ partials,
                                                     uint32_t* __restrict__ status)
{
    // thread layout: column c = tid % BPc, row lane = tid / BPc
    int bpc = 1;
    while (bpc < b && bpc < 256) bpc <<= 1;
    const int rl = threadIdx.x / bpc, rs = 256 / bpc;
    const int64_t j0 = (int64_t)blockIdx.x * TOT_ROWS;
    const int64_t j1 = min(n, j0 + TOT_ROWS);
    __shared__ double s_f[3][256];
    __shared__ int64_t s_i[2][256];
    uint32_t bad = 0;
    for (int cbase = 0; cbase < b; cbase += bpc) {
        const int c = cbase + (int)(threadIdx.x % bpc);
        double f0 = 0.0, f1 = 0.0, fl = 0.0;
        uint64_t i0 = 0, i1 = 0;
        if (c < b) {
            for (int64_t j = j0 + rl; j < j1; j += rs) {
                const ZT z = Z[j * b + c];
                if constexpr (INT) {
                    i0 += (uint64_t)(int64_t)z;
                    i1 += (uint64_t)(int64_t)wgt[j] * (uint64_t)(int64_t)z;
                    fl += fabs((double)z);
                } else {
                    if (!isfinite(z)) bad = 1;
                    f0 += (double)z;
                    f1 += (double)wgt[j] * (double)z;
                    fl += fabs((double)z);
                }
            }
        }
        s_f[0][threadIdx.x] = f0; s_f[1][threadIdx.x] = f1; s_f[2][threadIdx.x] = fl;
        s_i[0][threadIdx.x] = (int64_t)i0; s_i[1][threadIdx.x] = (int64_t)i1;
        __syncthreads();
        if ((int)threadIdx.x < bpc && c < b) {
            double a0 = 0, a1 = 0, al = 0;
            uint64_t b0 = 0, b1 = 0;
            for (int r = 0; r < rs; ++r) {
                const int t = r * bpc + threadIdx.x;
                a0 += s_f[0][t]; a1 += s_f[1][t]; al += s_f[2][t];
                b0 += (uint64_t)s_i[0][t]; b1 += (uint64_t)s_i[1][t];
            }
            double* pf = (double*)partials + ((size_t)blockIdx.x * b + c) * 3;
            if constexpr (INT) {
                pf[0] = __longlong_as_double((long long)b0);
                pf[1] = __longlong_as_double((long long)b1);
            } else {
                pf[0] = a0;
                pf[1] = a1;
            }
            pf[2] = al;
        }
        __syncthreads();
    }
    if (!INT && bad) atomicOr(status, (uint32_t)QF_NONFINITE);
}

// one block per column: threads take strided slices of the partials, then a
// fixed tree in LDS (reproducible FP64 sums)
template <bool INT>
__global__ __launch_bounds__(256) void totals_stage2(const void* __restrict__ partials, int nblk, int32_t b,
                                                     void* __restrict__ T0, void* __restrict__ U,
                                                     double* __restrict__ zl1, double guard_scale,
                                                     uint32_t* __restrict__ status)
{
    __shared__ double s_f[3][256];
    __shared__ uint64_t s_i[2][256];
    const int c = blockIdx.x, t = threadIdx.x;
    double a0 = 0, a1 = 0, al = 0;
    uint64_t b0 = 0, b1 = 0;
    for (int k = t; k < nblk; k += 256) {
        const double* pf = (const double*)partials + ((size_t)k * b + c) * 3;
        if (INT) {
            b0 += (uint64_t)__double_as_longlong(pf[0]);
            b1 += (uint64_t)__double_as_longlong(pf[1]);
        } else {
            a0 += pf[0];
            a1 += pf[1];
        }
        al += pf[2];
    }
    s_f[0][t] = a0; s_f[1][t] = a1; s_f[2][t] = al;
    s_i[0][t] = b0; s_i[1][t] = b1;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (t < h) {
            s_f[0][t] += s_f[0][t + h];
            s_f[1][t] += s_f[1][t + h];
            s_f[2][t] += s_f[2][t + h];
            s_i[0][t] += s_i[0][t + h];
            s_i[1][t] += s_i[1][t + h];
        }
        __syncthreads();
    }
    if (t == 0) {
        if (INT) {
            ((int64_t*)T0)[c] = (int64_t)s_i[0][0];
            ((int64_t*)U)[c] = (int64_t)s_i[1][0];
            // every |(A z)_i| <= ||z||_1 * max_ij A_ij <= ||z||_1 * guard_scale
            if (!(s_f[2][0] * guard_scale < 4611686018427387904.0)) atomicOr(status, (uint32_t)QF_OVERFLOW);
        } else {
            ((double*)T0)[c] = s_f[0][0];
            ((double*)U)[c] = s_f[1][0];
        }
        zl1[c] = s_f[2][0];
    }
}

}  // namespace

int totals_partial_blocks(int64_t n) { return (int)((n + TOT_ROWS - 1) / TOT_ROWS); }

size_t totals_scratch_bytes(int64_t n, int32_t b) {
    return (size_t)totals_partial_blocks(n) * (size_t)b * 3 * sizeof(double);
}

hipError_t launch_totals(bool is_int, int zkind, const void* Z, int64_t n, int32_t b, const void* w,
                         double guard_scale, const TotalsOut& o, hipStream_t s)
{
    if (b < 1 || b > TOT_MAXB) return hipErrorInvalidValue;
    const int nblk = totals_partial_blocks(n);
    if (!is_int) {
        totals_stage1<false, float, double><<<nblk, 256, 0, s>>>((const float*)Z, n, b, (const double*)w,
                                                                 o.partials, o.status);
    } else if (zkind == IN_I32) {
        totals_stage1<true, int32_t, int64_t><<<nblk, 256, 0, s>>>((const int32_t*)Z, n, b, (const int64_t*)w,
                                                                   o.partials, o.status);
    } else {
        totals_stage1<true, int64_t, int64_t><<<nblk, 256, 0, s>>>((const int64_t*)Z, n, b, (const int64_t*)w,
                                                                   o.partials, o.status);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (is_int)
        totals_stage2<true><<<b, 256, 0, s>>>(o.partials, nblk, b, o.T0, o.U, o.zl1, guard_scale, o.status);
    else
        totals_stage2<false><<<b, 256, 0, s>>>(o.partials, nblk, b, o.T0, o.U, o.zl1, guard_scale, o.status);
    return hipGetLastError();
}

// ranks per slot (R) for each configuration
template <int BP> constexpr int r_float() { return BP >= 32 ? 16 : BP >= 4 ? 8 : 16; }
template <int BP> constexpr int r_int() { return BP >= 4 ? 4 : 8; }
template <int BP, int R> constexpr int out_chunk() { return BP >= 4 ? (R >= 4 ? 4 : R) : R; }
// sub-chunks per tile: tiles of about 1024 ranks for wide blocks, 4 sub-chunks for narrow ones
template <int BP, int R> constexpr int sub_chunks() {
    return (Lay<BP>::NS * R) >= 1024 ? 4 : 1024 / (Lay<BP>::NS * R);
}

static int bpad(int32_t b) {
    int bp = 1;
    while (bp < b) bp <<= 1;
    return bp;
}

// Tiles of the l1 pass kernels: the keep kernel (whole tile on chip, two
// sub-chunks) for float data and for integer blocks of up to 32 columns; the
// re-gathering kernel for 64-column integer blocks, whose int64 rows leave
// room for only 128-rank tiles on chip.  The tile of a configuration is
// defined here once; the launch and the sizing of the record region both
// take it from pass_tile.
template <typename P, int BP> constexpr bool use_keep() { return std::is_same<P, FloatPath>::value || BP <= 32; }
template <typename P, int BP> constexpr int pass_r() {
    return std::is_same<P, FloatPath>::value ? r_float<BP>() : r_int<BP>();
}
template <typename P, int BP> constexpr int pass_sub() {
    return use_keep<P, BP>() ? 2 : sub_chunks<BP, pass_r<P, BP>()>();
}
template <typename P, int BP> constexpr int pass_tile() { return Lay<BP>::NS * pass_r<P, BP>() * pass_sub<P, BP>(); }
// two records of 2*BP values and one status word per tile
template <typename P, int BP> constexpr size_t pass_tile_words() { return 2 * 2 * (size_t)P::WPV * BP + 1; }

template <typename P> static int tile_ranks_p(int32_t b) {
    switch (bpad(b)) {
    case 1: return pass_tile<P, 1>();
    case 2: return pass_tile<P, 2>();
    case 4: return pass_tile<P, 4>();
    case 8: return pass_tile<P, 8>();
    case 16: return pass_tile<P, 16>();
    case 32: return pass_tile<P, 32>();
    default: return pass_tile<P, 64>();
    }
}

int l1_tile_ranks(int32_t b, bool is_int, int zkind) {
    if (!is_int) return tile_ranks_p<FloatPath>(b);
    if (zkind == IN_I32) return tile_ranks_p<IntPath<int32_t>>(b);
    return tile_ranks_p<IntPath<int64_t>>(b);
}

L1Shape l1_shape(int64_t n, int32_t b, bool is_int, int zkind) {
    L1Shape sh;
    const int kind = !is_int ? 0 : zkind == IN_I32 ? 1 : 2;
    int lg = 0;
    while ((1 << lg) < b) ++lg;
    sh.cls = kind * 8 + lg;
    sh.record_words = l1_record_words(n, b, is_int, zkind);
    return sh;
}

size_t l1_record_words(int64_t n, int32_t b, bool is_int, int zkind) {
    const int64_t tile = l1_tile_ranks(b, is_int, zkind);
    const int64_t ntiles = (n + tile - 1) / tile;
    const size_t wpv = is_int ? 2 : 1;
    return (size_t)ntiles * (2 * 2 * wpv * (size_t)bpad(b) + 1);   // two records and one status word per tile
}

template <int BP> constexpr int log2c() { return BP <= 1 ? 0 : 1 + log2c<BP / 2>(); }

// Persistent grid: as many workgroups as fit on the device at once (never more
// than one per tile).  Cached per kernel; every pass of one kernel shape gets
// the same grid, which the ticket arithmetic relies on.
static int persistent_grid_of(int64_t ntiles, const void* fn, const void* fn2) {
    struct Entry { const void* fn; int per_cu; };
    static Entry cache[64];
    static int cached = 0, cus = -1;
    if (cus < 0) {
        int dev = 0;
        (void)hipGetDevice(&dev);
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) cus = 256;
    }
    // the smaller occupancy of the two variants (vector and scalar row access)
    // of one shape, so that every pass of the shape uses the same grid
    int per_cu = 0;
    for (int i = 0; i < cached; ++i)
        if (cache[i].fn == fn) per_cu = cache[i].per_cu;
    if (per_cu == 0) {
        int nb = 0, nb2 = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, 256, 0) != hipSuccess || nb < 1) nb = 1;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb2, fn2, 256, 0) != hipSuccess || nb2 < 1) nb2 = 1;
        per_cu = nb < nb2 ? nb : nb2;
        if (cached < 64) cache[cached++] = Entry{fn, per_cu};
    }
    int64_t g = (int64_t)per_cu * cus;
    if (g > ntiles) g = ntiles;
    return (int)g;
}

template <typename P, int BP>
static hipError_t launch_one(const L1PassArgs& a, int32_t b, hipStream_t s) {
    constexpr bool KEEP = use_keep<P, BP>();
    constexpr int R = pass_r<P, BP>();
    constexpr int SUB = pass_sub<P, BP>();
    constexpr int TILE = pass_tile<P, BP>();
    constexpr int OC = out_chunk<BP, R>();
    // one ticket counter per kernel instantiation family (data path x BP)
    constexpr int kind = std::is_same<P, FloatPath>::value ? 0 : std::is_same<P, IntPath<int32_t>>::value ? 1 : 2;
    const int cls = kind * 8 + log2c<BP>();
    const int64_t ntiles = (a.n + TILE - 1) / TILE;
    // the region must hold every tile's records and status word
    if ((size_t)ntiles * pass_tile_words<P, BP>() > a.record_words) return hipErrorInvalidValue;
    uint64_t* stat = a.records + (size_t)ntiles * 2 * 2 * P::WPV * BP;
    uint64_t* ctr = &a.chain->ticket[cls];
    const bool vec = (b == BP) && ((uintptr_t)a.Z % 16 == 0) && ((uintptr_t)a.Out % 16 == 0);
    // one grid size per tile shape: every pass of a shape must use the same
    // grid, since the ticket count of a pass is ntiles + grid
    if constexpr (KEEP) {
        const int grid = persistent_grid_of(ntiles, (const void*)l1_pass_keep_kernel<P, BP, R, OC, false>,
                                            (const void*)l1_pass_keep_kernel<P, BP, R, OC, true>);
        if (vec)
            l1_pass_keep_kernel<P, BP, R, OC, true><<<grid, 256, 0, s>>>(
                a.perm, (const typename P::X*)a.xs, a.n, (const typename P::Z*)a.Z, (typename P::O*)a.Out, b,
                (const typename P::T*)a.T0, (const typename P::T*)a.U, a.first, ctr, cls, ntiles, a.records, stat);
        else
            l1_pass_keep_kernel<P, BP, R, OC, false><<<grid, 256, 0, s>>>(
                a.perm, (const typename P::X*)a.xs, a.n, (const typename P::Z*)a.Z, (typename P::O*)a.Out, b,
                (const typename P::T*)a.T0, (const typename P::T*)a.U, a.first, ctr, cls, ntiles, a.records, stat);
    } else {
        const int grid = persistent_grid_of(ntiles, (const void*)l1_pass_kernel<P, BP, R, SUB, OC, false>,
                                            (const void*)l1_pass_kernel<P, BP, R, SUB, OC, true>);
        if (vec)
            l1_pass_kernel<P, BP, R, SUB, OC, true><<<grid, 256, 0, s>>>(
                a.perm, (const typename P::X*)a.xs, a.n, (const typename P::Z*)a.Z, (typename P::O*)a.Out, b,
                (const typename P::T*)a.T0, (const typename P::T*)a.U, a.first, ctr, cls, ntiles, a.records, stat);
        else
            l1_pass_kernel<P, BP, R, SUB, OC, false><<<grid, 256, 0, s>>>(
                a.perm, (const typename P::X*)a.xs, a.n, (const typename P::Z*)a.Z, (typename P::O*)a.Out, b,
                (const typename P::T*)a.T0, (const typename P::T*)a.U, a.first, ctr, cls, ntiles, a.records, stat);
    }
    return hipGetLastError();
}

template <typename P>
static hipError_t dispatch_b(const L1PassArgs& a, int32_t b, hipStream_t s) {
    switch (bpad(b)) {
    case 1: return launch_one<P, 1>(a, b, s);
    case 2: return launch_one<P, 2>(a, b, s);
    case 4: return launch_one<P, 4>(a, b, s);
    case 8: return launch_one<P, 8>(a, b, s);
    case 16: return launch_one<P, 16>(a, b, s);
    case 32: return launch_one<P, 32>(a, b, s);
    case 64: return launch_one<P, 64>(a, b, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_l1_pass(bool is_int, int zkind, int32_t b, const L1PassArgs& a, hipStream_t s)
{
    if (b < 1 || b > 64) return hipErrorInvalidValue;
    if (!is_int) return dispatch_b<FloatPath>(a, b, s);
    if (zkind == IN_I32) return dispatch_b<IntPath<int32_t>>(a, b, s);
    return dispatch_b<IntPath<int64_t>>(a, b, s);
}

}  // namespace dm
