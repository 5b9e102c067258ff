// k_multi.hip - one query over many point sets of uneven n and d (the
// products AB of the Appendix C lemma, taken for a whole batch of datasets
// at once; every dataset has its own sorted orders from Algorithm 1).
//
// Round k of a query processes coordinate k of every dataset with d > k;
// rounds are stream-ordered, so the Out rows of a dataset are never touched
// by two coordinates at once.  Inside a round every dataset's coordinate is a
// segment of tiles; tiles of all segments are taken in ticket order by
// persistent workgroups, and each tile chains its prefix to the previous
// tiles of its own segment with the windowed look-back (the first tile of a
// segment starts from zero).  A tile stays in registers from its gather to
// its scatter.  The whole query (pointer table upload, totals, all rounds)
// is captured once in a hipGraph and replayed.
#include <type_traits>

#include "dm_device.h"
#include "dm_internal.h"
#include "l1_common.h"

namespace dm {
namespace {

using namespace l1;

constexpr int MT_ROWS = 4096;   // rows per totals block

// ---------------------------------------------------------------------------
// totals of every dataset: T0[c] = sum_j z_jc, U[c] = sum_j s_j z_jc, ||z_c||_1
// stage 1: one block per (dataset, 4096-row chunk); stage 2: one block per
// (dataset, column), fixed-order sums.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void multi_totals_stage1(const MultiDs* __restrict__ ds,
                                                           const uint32_t* __restrict__ blk_ds, int32_t b,
                                                           double* __restrict__ partials,
                                                           uint32_t* __restrict__ status)
{
    const uint32_t s = blk_ds[blockIdx.x];
    const MultiDs D = ds[s];
    const int64_t chunk = (int64_t)blockIdx.x - D.tot_blk0;
    const int64_t j0 = chunk * MT_ROWS, j1 = min(D.n, j0 + MT_ROWS);
    int bpc = 1;
    while (bpc < b && bpc < 256) bpc <<= 1;
    const int rl = threadIdx.x / bpc, rsn = 256 / bpc;
    __shared__ double s_f[3][256];
    __shared__ uint64_t s_i[2][256];
    uint32_t bad = 0;
    for (int cbase = 0; cbase < b; cbase += bpc) {
        const int c = cbase + (int)(threadIdx.x % bpc);
        double f0 = 0.0, f1 = 0.0, fl = 0.0;
        uint64_t i0 = 0, i1 = 0;
        if (c < b) {
            for (int64_t j = j0 + rl; j < j1; j += rsn) {
                if (D.is_int) {
                    const int32_t z = ((const int32_t*)D.Z)[j * b + c];
                    i0 += (uint64_t)(int64_t)z;
                    i1 += (uint64_t)((const int64_t*)D.rowsum)[j] * (uint64_t)(int64_t)z;
                    fl += fabs((double)z);
                } else {
                    const float z = ((const float*)D.Z)[j * b + c];
                    if (!isfinite(z)) bad = 1;
                    f0 += (double)z;
                    f1 += ((const double*)D.rowsum)[j] * (double)z;
                    fl += fabs((double)z);
                }
            }
        }
        s_f[0][threadIdx.x] = f0; s_f[1][threadIdx.x] = f1; s_f[2][threadIdx.x] = fl;
        s_i[0][threadIdx.x] = i0; s_i[1][threadIdx.x] = i1;
        __syncthreads();
        if ((int)threadIdx.x < bpc && c < b) {
            double a0 = 0, a1 = 0, al = 0;
            uint64_t b0 = 0, b1 = 0;
            for (int r = 0; r < rsn; ++r) {
                const int t = r * bpc + threadIdx.x;
                a0 += s_f[0][t]; a1 += s_f[1][t]; al += s_f[2][t];
                b0 += s_i[0][t]; b1 += s_i[1][t];
            }
            double* pf = partials + ((size_t)blockIdx.x * b + c) * 3;
            if (D.is_int) {
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
    if (bad) atomicOr(status, (uint32_t)QF_NONFINITE);
}

__global__ __launch_bounds__(64) void multi_totals_stage2(const MultiDs* __restrict__ ds, int32_t b,
                                                          const double* __restrict__ partials,
                                                          uint32_t* __restrict__ status)
{
    const int s = blockIdx.x / b, c = blockIdx.x % b;
    if (threadIdx.x != 0) return;
    const MultiDs D = ds[s];
    double a0 = 0, a1 = 0, al = 0;
    uint64_t b0 = 0, b1 = 0;
    for (int k = 0; k < D.tot_nblk; ++k) {
        const double* pf = partials + ((size_t)(D.tot_blk0 + k) * b + c) * 3;
        if (D.is_int) {
            b0 += (uint64_t)__double_as_longlong(pf[0]);
            b1 += (uint64_t)__double_as_longlong(pf[1]);
        } else {
            a0 += pf[0];
            a1 += pf[1];
        }
        al += pf[2];
    }
    if (D.is_int) {
        ((int64_t*)D.T0)[c] = (int64_t)b0;
        ((int64_t*)D.U)[c] = (int64_t)b1;
        if (!(al * D.guard < 4611686018427387904.0)) atomicOr(status, (uint32_t)QF_OVERFLOW);
    } else {
        ((double*)D.T0)[c] = a0;
        ((double*)D.U)[c] = a1;
    }
}

// ---------------------------------------------------------------------------
// one round: coordinate k of every dataset in the round's tile table
// ---------------------------------------------------------------------------
template <typename P, int BP, int R, int OC, bool VEC>
__global__ __launch_bounds__(256, 2) void multi_pass_kernel(const MultiDs* __restrict__ ds,
                                                         const MultiTile* __restrict__ tiles, int64_t ntiles,
                                                         int32_t k, int32_t b, uint64_t* __restrict__ ticket_ctr,
                                                         uint64_t* __restrict__ rec, uint64_t* __restrict__ stat,
                                                         uint32_t* __restrict__ status)
{
    using L = typename P::L;
    using C = typename P::C;
    using Ly = Lay<BP>;
    constexpr int CPL = Ly::CPL, LPR = Ly::LPR, RPW = Ly::RPW, NS = Ly::NS;
    constexpr int TILE = NS * R;
    constexpr int WPR = 2 * BP * P::WPV;
    static_assert(R % OC == 0, "Out chunk must divide the ranks per slot");

    __shared__ uint64_t s_ticket;
    __shared__ L s_wtot[4][2][BP];
    __shared__ C s_wexcl[4][2][BP];
    __shared__ C s_tot[2][BP];
    __shared__ C s_carry[2][BP];
    __shared__ C s_lb[4][2][BP];

    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int slot = w * RPW + lane / LPR;
    const int col0 = (lane % LPR) * CPL;
    const uint64_t per_pass = (uint64_t)ntiles + gridDim.x;
    if (tid == 0) s_ticket = atomicAdd((unsigned long long*)ticket_ctr, 1ull);
    __syncthreads();
    uint64_t ticket = s_ticket;
    const bool first = k == 0;

    for (;;) {
        const uint64_t tile = ticket % per_pass;
        if (tile >= (uint64_t)ntiles) break;
        // nonzero pass tag; every word a pass reads is rewritten by that pass
        const uint32_t tag = (uint32_t)((ticket / per_pass) % 0xffffffffull) + 1u;
        const MultiTile mt = tiles[tile];
        const MultiDs& D = ds[mt.ds];
        const int64_t n = D.n;
        const uint32_t* __restrict__ perm = D.perm + (size_t)k * D.ld;
        const typename P::X* __restrict__ xs = (const typename P::X*)D.xs + (size_t)k * D.ld;
        const typename P::Z* __restrict__ Z = (const typename P::Z*)D.Z;
        typename P::O* __restrict__ Out = (typename P::O*)D.Out;
        const typename P::T* __restrict__ T0 = (const typename P::T*)D.T0;
        const typename P::T* __restrict__ U = (const typename P::T*)D.U;
        const bool head = mt.t == 0;   // first tile of its segment
        const int64_t r0 = (int64_t)mt.t * TILE + (int64_t)slot * R;

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
            C acc = P::czero();
#pragma unroll
            for (int ww = 0; ww < 4; ++ww) {
                s_wexcl[ww][qt][c] = acc;
                acc = P::caddl(acc, s_wtot[ww][qt][c]);
            }
            s_tot[qt][c] = acc;
            P::put(rec + ((size_t)tile * 2 + (head ? 1 : 0)) * WPR + (c * 2 + qt) * P::WPV, acc, tag);
        }
        __syncthreads();
        if (tid == 0) publish_word(stat + tile, tag_word(tag, head ? 2u : 1u));

        // windowed look-back inside the segment (its head tile always has an
        // inclusive record, so the walk never leaves the segment)
        C cc[2];
        // two records per wave per round trip: the whole tile is held in registers,
        // and deeper batches would cost occupancy
        look_back_wg<P, BP, 2, 2>(rec, stat, head ? -1 : (int64_t)tile - 1, tag, tid, s_lb, cc, status);
        const C c0 = cc[0], c1 = cc[1];
        if (w == 0) {
            const int c = lane;
            const bool act = c < BP;
            if (act) {
                s_carry[0][c] = c0;
                s_carry[1][c] = c1;
                if (!head) {
                    uint64_t* dst = rec + ((size_t)tile * 2 + 1) * WPR + c * 2 * P::WPV;
                    P::put(dst, P::cadd(c0, s_tot[0][c]), tag);
                    P::put(dst + P::WPV, P::cadd(c1, s_tot[1][c]), tag);
                }
            }
            if (!head && lane == 0) publish_word(stat + tile, tag_word(tag, 2u));
        }
        __syncthreads();

        typename P::Fin f[CPL];
#pragma unroll
        for (int j = 0; j < CPL; ++j) {
            const int c = col0 + j;
            if (c < b) {
                const C b0 = P::caddl(P::cadd(s_carry[0][c], s_wexcl[w][0][c]), e0[j]);
                const C b1 = P::caddl(P::cadd(s_carry[1][c], s_wexcl[w][1][c]), e1[j]);
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
        if (tid == 0) s_ticket = atomicAdd((unsigned long long*)ticket_ctr, 1ull);
        __syncthreads();
        ticket = s_ticket;
        __syncthreads();
    }
}

// ranks per slot of the multi-dataset pass (register-resident tiles): the
// default R, and the tile variants the tuner chooses from (V = 0: R, 1: R / 2,
// 2: 2 R for blocks of up to 8 columns, R / 4 for wider ones)
template <int BP, bool INT> constexpr int mr() { return INT ? (BP >= 16 ? 4 : 8) : (BP >= 32 ? 8 : 16); }
template <int BP, bool INT, int V> constexpr int mrv() {
    return V == 0 ? mr<BP, INT>()
                  : V == 1 ? (mr<BP, INT>() / 2 > 0 ? mr<BP, INT>() / 2 : 1)
                           : (BP <= 8 ? 2 * mr<BP, INT>() : (mr<BP, INT>() / 4 > 0 ? mr<BP, INT>() / 4 : 1));
}
template <int BP, int R> constexpr int moc() { return BP >= 4 ? (R >= 4 ? 4 : R) : R; }

static int bpad2(int32_t b) {
    int bp = 1;
    while (bp < b) bp <<= 1;
    return bp;
}

template <int BP, bool INT, int V> static int mtile() { return Lay<BP>::NS * mrv<BP, INT, V>(); }

template <typename P, int BP, int V, bool VEC>
static const void* kfn() {
    constexpr bool INT = !std::is_same<P, FloatPath>::value;
    constexpr int R = mrv<BP, INT, V>();
    return (const void*)multi_pass_kernel<P, BP, R, moc<BP, R>(), VEC>;
}

// VEC: 16-byte row accesses (b % 4 == 0 and every Z and Out row 16-byte
// aligned, checked by the caller for all datasets)
template <typename P, int BP, int V>
static hipError_t launch_bpv(const MultiDs* ds, const MultiTile* tiles, int64_t ntiles, int k, int32_t b,
                             uint64_t* ctr, uint64_t* rec, int grid, bool vec, uint32_t* status, hipStream_t s) {
    constexpr bool INT = !std::is_same<P, FloatPath>::value;
    constexpr int R = mrv<BP, INT, V>();
    constexpr int TILEW = 2 * 2 * P::WPV * BP;
    uint64_t* stat = rec + (size_t)ntiles * TILEW;
    if (vec)
        multi_pass_kernel<P, BP, R, moc<BP, R>(), true><<<grid, 256, 0, s>>>(ds, tiles, ntiles, k, b, ctr, rec, stat, status);
    else
        multi_pass_kernel<P, BP, R, moc<BP, R>(), false><<<grid, 256, 0, s>>>(ds, tiles, ntiles, k, b, ctr, rec, stat, status);
    return hipGetLastError();
}

template <typename P, int BP>
static hipError_t launch_bp(const MultiDs* ds, const MultiTile* tiles, int64_t ntiles, int k, int32_t b,
                            uint64_t* ctr, uint64_t* rec, int grid, bool vec, uint32_t* status, int v, hipStream_t s) {
    switch (v) {
    case 0: return launch_bpv<P, BP, 0>(ds, tiles, ntiles, k, b, ctr, rec, grid, vec, status, s);
    case 1: return launch_bpv<P, BP, 1>(ds, tiles, ntiles, k, b, ctr, rec, grid, vec, status, s);
    case 2: return launch_bpv<P, BP, 2>(ds, tiles, ntiles, k, b, ctr, rec, grid, vec, status, s);
    default: return hipErrorInvalidValue;
    }
}

template <typename P, int BP> static int grid2(int64_t ntiles, int v) {
    switch (v) {
    case 0: return persistent_grid(kfn<P, BP, 0, false>(), kfn<P, BP, 0, true>(), ntiles);
    case 1: return persistent_grid(kfn<P, BP, 1, false>(), kfn<P, BP, 1, true>(), ntiles);
    default: return persistent_grid(kfn<P, BP, 2, false>(), kfn<P, BP, 2, true>(), ntiles);
    }
}

template <int BP, bool INT> static int mtile_v(int v) {
    return v == 0 ? mtile<BP, INT, 0>() : v == 1 ? mtile<BP, INT, 1>() : mtile<BP, INT, 2>();
}

}  // namespace

int multi_tile_ranks(int32_t b, bool is_int, int v) {
    switch (bpad2(b)) {
    case 1: return is_int ? mtile_v<1, true>(v) : mtile_v<1, false>(v);
    case 2: return is_int ? mtile_v<2, true>(v) : mtile_v<2, false>(v);
    case 4: return is_int ? mtile_v<4, true>(v) : mtile_v<4, false>(v);
    case 8: return is_int ? mtile_v<8, true>(v) : mtile_v<8, false>(v);
    case 16: return is_int ? mtile_v<16, true>(v) : mtile_v<16, false>(v);
    case 32: return is_int ? mtile_v<32, true>(v) : mtile_v<32, false>(v);
    default: return is_int ? mtile_v<64, true>(v) : mtile_v<64, false>(v);
    }
}

size_t multi_record_words(int64_t ntiles, int32_t b, bool is_int) {
    const size_t wpv = is_int ? 2 : 1;
    return (size_t)ntiles * (2 * 2 * wpv * (size_t)bpad2(b) + 1);
}

// the smaller occupancy of the two row-access variants, so that a plan's grid
// does not depend on which one it launches
int multi_grid(int64_t ntiles, int32_t b, bool is_int, int v) {
    switch (bpad2(b)) {
    case 1: return is_int ? grid2<IntPath<int32_t>, 1>(ntiles, v) : grid2<FloatPath, 1>(ntiles, v);
    case 2: return is_int ? grid2<IntPath<int32_t>, 2>(ntiles, v) : grid2<FloatPath, 2>(ntiles, v);
    case 4: return is_int ? grid2<IntPath<int32_t>, 4>(ntiles, v) : grid2<FloatPath, 4>(ntiles, v);
    case 8: return is_int ? grid2<IntPath<int32_t>, 8>(ntiles, v) : grid2<FloatPath, 8>(ntiles, v);
    case 16: return is_int ? grid2<IntPath<int32_t>, 16>(ntiles, v) : grid2<FloatPath, 16>(ntiles, v);
    case 32: return is_int ? grid2<IntPath<int32_t>, 32>(ntiles, v) : grid2<FloatPath, 32>(ntiles, v);
    default: return is_int ? grid2<IntPath<int32_t>, 64>(ntiles, v) : grid2<FloatPath, 64>(ntiles, v);
    }
}

int multi_totals_rows() { return MT_ROWS; }

hipError_t launch_multi_totals(const MultiDs* ds, const uint32_t* blk_ds, int nblocks, int ndatasets, int32_t b,
                               double* partials, uint32_t* status, hipStream_t s)
{
    if (nblocks > 0) multi_totals_stage1<<<nblocks, 256, 0, s>>>(ds, blk_ds, b, partials, status);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    multi_totals_stage2<<<ndatasets * b, 64, 0, s>>>(ds, b, partials, status);
    return hipGetLastError();
}

hipError_t launch_multi_pass(bool is_int, int32_t b, const MultiDs* ds, const MultiTile* tiles, int64_t ntiles,
                             int k, uint64_t* ticket, uint64_t* records, int grid, bool vec, uint32_t* status,
                             int v, hipStream_t s)
{
    if (ntiles <= 0) return hipSuccess;
    if (vec && b % 4 != 0) return hipErrorInvalidValue;
    if (v < 0 || v >= MULTI_VARIANTS) return hipErrorInvalidValue;
    switch (bpad2(b)) {
#define DM_MCASE(BP)                                                                                         \
    case BP:                                                                                                 \
        return is_int ? launch_bp<IntPath<int32_t>, BP>(ds, tiles, ntiles, k, b, ticket, records, grid, vec, status, v, s) \
                      : launch_bp<FloatPath, BP>(ds, tiles, ntiles, k, b, ticket, records, grid, vec, status, v, s);
        DM_MCASE(1) DM_MCASE(2) DM_MCASE(4) DM_MCASE(8) DM_MCASE(16) DM_MCASE(32) DM_MCASE(64)
#undef DM_MCASE
    default: return hipErrorInvalidValue;
    }
}

}  // namespace dm
