// l1_pass.h - the l1 query's coordinate pass (Algorithm 2, Section 2) for b right-hand sides.
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
// pass needs no atomics on Out.  For a single column (OUT_FRESH) a pass writes
// its values to a buffer of its own in point order instead of adding them into
// Out, and the buffers of a group of coordinates are summed afterwards in one
// coalesced sweep: two scattered accesses per rank (the Z gather and the
// store) instead of three, and no scattered load whose latency is exposed.
//
// One pass = one launch, one tile of TILE consecutive ranks per workgroup.
// Tiles take indices from a ticket counter in dispatch order and chain their
// prefixes with a decoupled look-back over tagged 64-bit words.  Float data
// carries the prefixes between threads, waves and tiles as double-float
// (hi, lo) FP32 pairs; inside a thread the short runs are plain FP32 relative
// to that carry.  Integer data runs in wrapping int64, which is exact modulo
// 2^64: only additions, subtractions and multiplications are used, so the
// result is exact whenever |(A z)_i| < 2^63, which the guard
// ||z||_1 sum_k range_k < 2^62 of the totals kernel ensures with a factor of
// two to spare.
//
// This header holds the two pass kernels and their launch; it is compiled
// once per data path (k_l1_f32.hip, k_l1_i32.hip, k_l1_i64.hip).
#pragma once
#include <type_traits>

#include "dm_device.h"
#include "dm_internal.h"
#include "l1_common.h"

namespace dm {
namespace {

using namespace l1;

template <typename P, int BP, int R, int SUB, int OC, bool VEC, int OM = OUT_ADD>
__global__ __launch_bounds__(256, 2) void l1_pass_kernel(
    const uint32_t* __restrict__ perm, const typename P::X* __restrict__ xs, int64_t n,
    const typename P::Z* __restrict__ Z, typename P::O* __restrict__ Out, int32_t b,
    const typename P::T* __restrict__ T0, const typename P::T* __restrict__ U, int first,
    uint64_t* __restrict__ ticket_ctr, int cls, int64_t ntiles,
    uint64_t* __restrict__ rec, uint64_t* __restrict__ stat, uint32_t* __restrict__ status)
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
        C cc[2];
        look_back_wg<P, BP, 2>(rec, stat, (int64_t)tile - 1, tag, tid, s_red, cc, status);
        const C c0 = cc[0], c1 = cc[1];
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
                    f[j] = P::fin(b0, b1, T0[c], (first && OM == OUT_ADD) ? U[c] : typename P::T(0));
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
                    if (!first && OM == OUT_ADD) {
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
                    const size_t orow = (size_t)p[i0 + i];
                    if (r0 + i0 + i < n) store_row<CPL, VEC>(Out + orow * b, col0, b, res);
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
template <typename P, int BP, int R, int OC, bool VEC, int OM = OUT_ADD>
__global__ __launch_bounds__(256, 2) void l1_pass_keep_kernel(
    const uint32_t* __restrict__ perm, const typename P::X* __restrict__ xs, int64_t n,
    const typename P::Z* __restrict__ Z, typename P::O* __restrict__ Out, int32_t b,
    const typename P::T* __restrict__ T0, const typename P::T* __restrict__ U, int first,
    uint64_t* __restrict__ ticket_ctr, int cls, int64_t ntiles,
    uint64_t* __restrict__ rec, uint64_t* __restrict__ stat, uint32_t* __restrict__ status)
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
            // every Z row of the tile is read here once: streaming loads
            for (int i = 0; i < R; ++i) load_row<CPL, VEC, true>(Z + (size_t)p[i] * b, col0, b, r0 + i < n, g[i]);
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
        C cc[2];
        look_back_wg<P, BP, 2>(rec, stat, (int64_t)tile - 1, tag, tid, s_red, cc, status);
        const C c0 = cc[0], c1 = cc[1];
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
                    f[j] = P::fin(b0, b1, T0[c], (first && OM == OUT_ADD) ? U[c] : typename P::T(0));
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
                    if (!first && OM == OUT_ADD) {
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
                    const size_t orow = (size_t)getp(i0 + i);
                    if (r0 + i0 + i < n) store_row<CPL, VEC>(Out + orow * b, col0, b, res);
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
// tile shapes
// ---------------------------------------------------------------------------
// ranks per slot (R) of the default shape
template <int BP> constexpr int r_float() { return BP >= 32 ? 16 : BP >= 4 ? 8 : 16; }
template <int BP> constexpr int r_int() { return BP >= 4 ? 4 : 8; }
// rows of Out read per batch in phase 2: more rows in flight where a thread
// holds 16 or more ranks (measured faster for 32 and 64 columns)
template <int BP, int R> constexpr int out_chunk() { return BP >= 4 ? (R >= 16 ? 8 : R >= 4 ? 4 : R) : R; }
// sub-chunks per tile of the re-gathering kernel: tiles of about 1024 ranks
// for wide blocks, 4 sub-chunks for narrow ones
template <int BP, int R> constexpr int sub_chunks() {
    return (Lay<BP>::NS * R) >= 1024 ? 4 : 1024 / (Lay<BP>::NS * R);
}
// Default kernel family: the keep kernel (whole tile on chip, two
// sub-chunks) for float data and for integer blocks of up to 32 columns; the
// re-gathering kernel for 64-column integer blocks, whose int64 rows leave
// room for only 128-rank tiles on chip.
template <typename P, int BP> constexpr bool default_keep() { return std::is_same<P, FloatPath>::value || BP <= 32; }
template <typename P, int BP> constexpr int default_r() {
    return std::is_same<P, FloatPath>::value ? r_float<BP>() : r_int<BP>();
}

// Variant V of a configuration (P, BP), chosen per handle by the tuner:
//   0 - default family, default R      1 - default family, R halved
//   2 - other family, default R        3 - other family, R halved
// The tile of a variant is defined here once; the launch and the sizing of
// its record region both take it from Shape.
template <typename P, int BP, int V> struct Shape {
    static constexpr bool KEEP = (V < 2) == default_keep<P, BP>();
    static constexpr int R = (V & 1) ? default_r<P, BP>() / 2 : default_r<P, BP>();
    static constexpr int SUB = KEEP ? 2 : sub_chunks<BP, R>();
    static constexpr int TILE = Lay<BP>::NS * R * SUB;
    static constexpr int OC = out_chunk<BP, R>();
    // two records of 2*BP values and one status word per tile
    static constexpr size_t TILE_WORDS = 2 * 2 * (size_t)P::WPV * BP + 1;
};

template <int BP> constexpr int log2c() { return BP <= 1 ? 0 : 1 + log2c<BP / 2>(); }

// Persistent grid: as many workgroups as fit on the device at once (never more
// than one per tile), the same for every pass of one kernel shape on a device,
// which the ticket arithmetic relies on (persistent_grid).
static int persistent_grid_of(int64_t ntiles, const void* fn, const void* fn2) {
    return persistent_grid(fn, fn2, ntiles);
}

// single-column passes that write rather than add (OUT_FRESH): a kernel shape
// of its own with its own ticket class
template <typename P, int BP, int R, int SUB, int OC, bool KEEP, int OM>
hipError_t launch_single(const L1PassArgs& a, int32_t b, hipStream_t s, uint64_t* ctr, int64_t ntiles,
                         uint64_t* stat) {
    if constexpr (KEEP) {
        const int grid = persistent_grid_of(ntiles, (const void*)l1_pass_keep_kernel<P, BP, R, OC, false, OM>,
                                            (const void*)l1_pass_keep_kernel<P, BP, R, OC, false, OM>);
        l1_pass_keep_kernel<P, BP, R, OC, false, OM><<<grid, 256, 0, s>>>(
            a.perm, (const typename P::X*)a.xs, a.n, (const typename P::Z*)a.Z, (typename P::O*)a.Out, b,
            (const typename P::T*)a.T0, (const typename P::T*)a.U, a.first, ctr, a.cls, ntiles, a.records, stat,
            a.status);
    } else {
        const int grid = persistent_grid_of(ntiles, (const void*)l1_pass_kernel<P, BP, R, SUB, OC, false, OM>,
                                            (const void*)l1_pass_kernel<P, BP, R, SUB, OC, false, OM>);
        l1_pass_kernel<P, BP, R, SUB, OC, false, OM><<<grid, 256, 0, s>>>(
            a.perm, (const typename P::X*)a.xs, a.n, (const typename P::Z*)a.Z, (typename P::O*)a.Out, b,
            (const typename P::T*)a.T0, (const typename P::T*)a.U, a.first, ctr, a.cls, ntiles, a.records, stat,
            a.status);
    }
    return hipGetLastError();
}

template <typename P, int BP, int V>
hipError_t launch_shape(const L1PassArgs& a, int32_t b, hipStream_t s) {
    using S = Shape<P, BP, V>;
    constexpr int R = S::R, SUB = S::SUB, TILE = S::TILE, OC = S::OC;
    const int64_t ntiles = (a.n + TILE - 1) / TILE;
    // the region must hold every tile's records and status word
    if ((size_t)ntiles * S::TILE_WORDS > a.record_words) return hipErrorInvalidValue;
    uint64_t* stat = a.records + (size_t)ntiles * 2 * 2 * P::WPV * BP;
    uint64_t* ctr = &a.chain->ticket[a.cls];
    // 16-byte row accesses: whole 4-column groups, 16-byte aligned rows
    const bool vec = (b % 4 == 0) && ((uintptr_t)a.Z % 16 == 0) && ((uintptr_t)a.Out % 16 == 0);
    // one grid size per tile shape: every pass of a shape must use the same
    // grid, since the ticket count of a pass is ntiles + grid (the OUT_FRESH
    // passes are shapes of their own, with their own ticket class)
    if constexpr (BP == 1) {
        if (a.out_mode == OUT_FRESH) return launch_single<P, BP, R, SUB, OC, S::KEEP, OUT_FRESH>(a, b, s, ctr, ntiles, stat);
    }
    if (a.out_mode != OUT_ADD) return hipErrorInvalidValue;   // single columns only
    if constexpr (S::KEEP) {
        const int grid = persistent_grid_of(ntiles, (const void*)l1_pass_keep_kernel<P, BP, R, OC, false>,
                                            (const void*)l1_pass_keep_kernel<P, BP, R, OC, true>);
        if (vec)
            l1_pass_keep_kernel<P, BP, R, OC, true><<<grid, 256, 0, s>>>(
                a.perm, (const typename P::X*)a.xs, a.n, (const typename P::Z*)a.Z, (typename P::O*)a.Out, b,
                (const typename P::T*)a.T0, (const typename P::T*)a.U, a.first, ctr, a.cls, ntiles, a.records, stat, a.status);
        else
            l1_pass_keep_kernel<P, BP, R, OC, false><<<grid, 256, 0, s>>>(
                a.perm, (const typename P::X*)a.xs, a.n, (const typename P::Z*)a.Z, (typename P::O*)a.Out, b,
                (const typename P::T*)a.T0, (const typename P::T*)a.U, a.first, ctr, a.cls, ntiles, a.records, stat, a.status);
    } else {
        const int grid = persistent_grid_of(ntiles, (const void*)l1_pass_kernel<P, BP, R, SUB, OC, false>,
                                            (const void*)l1_pass_kernel<P, BP, R, SUB, OC, true>);
        if (vec)
            l1_pass_kernel<P, BP, R, SUB, OC, true><<<grid, 256, 0, s>>>(
                a.perm, (const typename P::X*)a.xs, a.n, (const typename P::Z*)a.Z, (typename P::O*)a.Out, b,
                (const typename P::T*)a.T0, (const typename P::T*)a.U, a.first, ctr, a.cls, ntiles, a.records, stat, a.status);
        else
            l1_pass_kernel<P, BP, R, SUB, OC, false><<<grid, 256, 0, s>>>(
                a.perm, (const typename P::X*)a.xs, a.n, (const typename P::Z*)a.Z, (typename P::O*)a.Out, b,
                (const typename P::T*)a.T0, (const typename P::T*)a.U, a.first, ctr, a.cls, ntiles, a.records, stat, a.status);
    }
    return hipGetLastError();
}

template <typename P, int BP>
hipError_t launch_bp(const L1PassArgs& a, int32_t b, int v, hipStream_t s) {
    switch (v) {
    case 0: return launch_shape<P, BP, 0>(a, b, s);
    case 1: return launch_shape<P, BP, 1>(a, b, s);
    case 2: return launch_shape<P, BP, 2>(a, b, s);
    case 3: return launch_shape<P, BP, 3>(a, b, s);
    default: return hipErrorInvalidValue;
    }
}

template <typename P, int BP> int tile_bp(int v) {
    switch (v) {
    case 0: return Shape<P, BP, 0>::TILE;
    case 1: return Shape<P, BP, 1>::TILE;
    case 2: return Shape<P, BP, 2>::TILE;
    case 3: return Shape<P, BP, 3>::TILE;
    default: return 0;
    }
}

inline int bpad(int32_t b) {
    int bp = 1;
    while (bp < b) bp <<= 1;
    return bp;
}

// the pass of one data path: block width b (1..64), variant v
template <typename P>
hipError_t launch_pass_p(const L1PassArgs& a, int32_t b, int v, hipStream_t s) {
    switch (bpad(b)) {
    case 1: return launch_bp<P, 1>(a, b, v, s);
    case 2: return launch_bp<P, 2>(a, b, v, s);
    case 4: return launch_bp<P, 4>(a, b, v, s);
    case 8: return launch_bp<P, 8>(a, b, v, s);
    case 16: return launch_bp<P, 16>(a, b, v, s);
    case 32: return launch_bp<P, 32>(a, b, v, s);
    case 64: return launch_bp<P, 64>(a, b, v, s);
    default: return hipErrorInvalidValue;
    }
}

template <typename P> int tile_ranks_p(int32_t b, int v) {
    switch (bpad(b)) {
    case 1: return tile_bp<P, 1>(v);
    case 2: return tile_bp<P, 2>(v);
    case 4: return tile_bp<P, 4>(v);
    case 8: return tile_bp<P, 8>(v);
    case 16: return tile_bp<P, 16>(v);
    case 32: return tile_bp<P, 32>(v);
    case 64: return tile_bp<P, 64>(v);
    default: return 0;
    }
}

}  // namespace
}  // namespace dm
