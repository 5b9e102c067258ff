// l1_common.h - device code shared by the l1 pass kernels (single dataset
// and multi-dataset): lane layout of a block of b right-hand sides, the two
// data paths (float with double-float carries, integer with wrapping int64)
// and their tagged record words, and row access helpers.
#pragma once
#include "dm_device.h"
#include "dm_internal.h"

namespace dm {
namespace l1 {

template <int BP> struct Lay {
    static constexpr int CPL = BP >= 4 ? 4 : BP;  // columns per lane
    static constexpr int LPR = BP / CPL;          // lanes per row
    static constexpr int RPW = DM_WAVE / LPR;     // rows (slots) per wave
    static constexpr int NS = 4 * RPW;            // slots per workgroup
};

// ---------------------------------------------------------------------------
// arithmetic of the two data kinds
// ---------------------------------------------------------------------------
struct FloatPath {
    using Z = float;
    using O = float;
    using X = float;
    using L = float;   // thread-local partial sums
    using C = dd;      // carries between threads, waves and tiles
    using T = double;  // totals T0 and U
    struct Fin { float d0, e1, u; };

    __device__ static L lzero() { return 0.0f; }
    __device__ static L ladd(L a, Z g) { return a + g; }
    __device__ static L lmac(L a, X x, Z g) { return fmaf(x, g, a); }
    __device__ static L lsum(L a, L b) { return a + b; }
    __device__ static L shfl_up(L v, int o) { return __shfl_up(v, o, 64); }
    __device__ static C czero() { return dd{0.0f, 0.0f}; }
    __device__ static C cshfl_xor(C v, int m) { return dd{__shfl_xor(v.hi, m, 64), __shfl_xor(v.lo, m, 64)}; }
    __device__ static C cadd(C a, C b) { return dd_add(a, b); }
    __device__ static C caddl(C a, L b) { return dd_add_f(a, b); }
    __device__ static void enc(C c, uint32_t& w0, uint32_t& w1) {
        w0 = __float_as_uint(c.hi);
        w1 = __float_as_uint(c.lo);
    }
    __device__ static C dec(uint32_t w0, uint32_t w1) { return dd{__uint_as_float(w0), __uint_as_float(w1)}; }
    // Record words: one 64-bit word per value, hi in the upper half, lo with
    // its 12 low mantissa bits replaced by a 12-bit tag (the carry keeps about
    // 36 significant bits in transit, far more than the FP32 result needs).
    static constexpr int WPV = 1;
    __device__ static uint32_t tag12(uint32_t tag) { return (tag - 1u) % 4095u + 1u; }   // 1..4095
    __device__ static void put(uint64_t* dst, C v, uint32_t tag) {
        const uint32_t lo = (__float_as_uint(v.lo) & 0xfffff000u) | tag12(tag);
        publish_word(dst, ((uint64_t)__float_as_uint(v.hi) << 32) | lo);
    }
    __device__ static bool decode(const uint64_t* w, uint32_t tag, C& v) {
        v = dd{__uint_as_float((uint32_t)(w[0] >> 32)), __uint_as_float((uint32_t)w[0] & 0xfffff000u)};
        return ((uint32_t)w[0] & 0xfffu) == tag12(tag);
    }
    __device__ static Fin fin(C b0, C b1, T t0, T u) {
        Fin f;
        f.d0 = (float)(2.0 * dd_to_f64(b0) - t0);
        f.e1 = (float)(2.0 * dd_to_f64(b1));
        f.u = (float)u;
        return f;
    }
    __device__ static O out(L l0, L l1, X x, const Fin& f) {
        const float a = fmaf(2.0f, l0, f.d0);
        const float e = fmaf(2.0f, l1, f.e1);
        return fmaf(x, a, -e);
    }
    __device__ static O oadd(O a, O b) { return a + b; }
    __device__ static O ufirst(const Fin& f) { return f.u; }
};

template <typename ZT> struct IntPath {
    using Z = ZT;
    using O = int64_t;
    using X = int32_t;
    using L = int64_t;
    using C = int64_t;
    using T = int64_t;
    struct Fin { int64_t d0, e1, u; };

    __device__ static int64_t w(uint64_t v) { return (int64_t)v; }
    __device__ static L lzero() { return 0; }
    __device__ static L ladd(L a, Z g) { return w((uint64_t)a + (uint64_t)(int64_t)g); }
    __device__ static L lmac(L a, X x, Z g) { return w((uint64_t)a + (uint64_t)(int64_t)x * (uint64_t)(int64_t)g); }
    __device__ static L lsum(L a, L b) { return w((uint64_t)a + (uint64_t)b); }
    __device__ static L shfl_up(L v, int o) { return __shfl_up(v, o, 64); }
    __device__ static C czero() { return 0; }
    __device__ static C cshfl_xor(C v, int m) { return __shfl_xor(v, m, 64); }
    __device__ static C cadd(C a, C b) { return w((uint64_t)a + (uint64_t)b); }
    __device__ static C caddl(C a, L b) { return w((uint64_t)a + (uint64_t)b); }
    __device__ static void enc(C c, uint32_t& w0, uint32_t& w1) {
        w0 = (uint32_t)(uint64_t)c;
        w1 = (uint32_t)((uint64_t)c >> 32);
    }
    __device__ static C dec(uint32_t w0, uint32_t w1) { return (int64_t)(((uint64_t)w1 << 32) | w0); }
    // Record words: two 64-bit words per value, each a 32-bit half with the full tag.
    static constexpr int WPV = 2;
    __device__ static void put(uint64_t* dst, C v, uint32_t tag) {
        publish_word(dst, tag_word(tag, (uint32_t)(uint64_t)v));
        publish_word(dst + 1, tag_word(tag, (uint32_t)((uint64_t)v >> 32)));
    }
    __device__ static bool decode(const uint64_t* w, uint32_t tag, C& v) {
        v = (int64_t)(((w[1] & 0xffffffffull) << 32) | (w[0] & 0xffffffffull));
        return (uint32_t)(w[0] >> 32) == tag && (uint32_t)(w[1] >> 32) == tag;
    }
    __device__ static Fin fin(C b0, C b1, T t0, T u) {
        Fin f;
        f.d0 = w(2ull * (uint64_t)b0 - (uint64_t)t0);
        f.e1 = w(2ull * (uint64_t)b1);
        f.u = u;
        return f;
    }
    __device__ static O out(L l0, L l1, X x, const Fin& f) {
        const uint64_t a = (uint64_t)f.d0 + 2ull * (uint64_t)l0;
        const uint64_t e = (uint64_t)f.e1 + 2ull * (uint64_t)l1;
        return w((uint64_t)(int64_t)x * a - e);
    }
    __device__ static O oadd(O a, O b) { return w((uint64_t)a + (uint64_t)b); }
    __device__ static O ufirst(const Fin& f) { return f.u; }
};

// ---------------------------------------------------------------------------
// Decoupled look-back over the tiles of one chained scan.
//
// Tile t keeps two records, each holding NM running sums for every column
// (P0, P1 for l1): the aggregate (the tile's own sums) at record 2t and the
// inclusive prefix at record 2t+1, and a status word (1 = aggregate
// published, 2 = inclusive published).  Starting at tile `hi`, lane l reads
// the status of tile hi-l, so 64 predecessors are examined per round trip.
// The walk sums aggregates back to the nearest tile with an inclusive record
// and adds that record; a run of 64 aggregates with no inclusive record in
// sight is summed and the walk moves on.  Status words are hints only:
// payload words carry their own tags and are checked, and a batch with a
// stale word is read again.  The records of a batch are loaded before any is
// summed, so one round trip to memory covers many predecessors.  Summation
// runs from the nearest predecessor outwards.
// ---------------------------------------------------------------------------
// The same walk run by the whole workgroup of four waves, for records of
// NM running sums per column (P0, P1 for l1; P0..Pp for odd p).  Wave 0 reads
// the status words and decides how many records to take; each wave then
// loads a quarter of them (records j = w, w+4, ...; LB per wave per round
// trip), so one round trip covers 4*LB predecessors.  Wave partials are
// combined in wave order by wave 0.  Every thread of the workgroup must call
// it; the result is valid in wave 0 (lane c holds column c).  s_part is LDS
// scratch of the caller, free for the duration of the call.  Record layout:
// column c's value t at word (c * NM + t) * WPV of a record of NM * BP * WPV
// words.
//
// Every wait is bounded: after LOOK_BACK_SPINS polls without progress (about
// a second; a correct chain waits microseconds) the walk gives up, sets
// QF_STALL in *status and treats the missing prefix as zero, so that the
// kernel always completes and the host sees the fault.
constexpr uint32_t LOOK_BACK_SPINS = 1u << 20;

template <typename P, int BP, int NM, int LB = 8>
__device__ __forceinline__ void look_back_wg(const uint64_t* __restrict__ rec, const uint64_t* __restrict__ stat,
                                             int64_t hi, uint32_t tag, int tid,
                                             typename P::C (*s_part)[NM][BP], typename P::C (&cc)[NM],
                                             uint32_t* __restrict__ status)
{
    using C = typename P::C;
    constexpr int WPR = NM * BP * P::WPV;
    constexpr int W = NM * P::WPV;   // words of one column's NM values
    constexpr int NW = 4;
    __shared__ int s_take, s_cnt;
    __shared__ int64_t s_hi;
    __shared__ uint32_t s_ok[NW];
    const int lane = tid & 63, w = tid >> 6;
    const int c = lane;
    const bool act = c < BP;
#pragma unroll
    for (int t = 0; t < NM; ++t) cc[t] = P::czero();
    bool fin = false;
    uint32_t spins = 0;
    for (;;) {
        if (w == 0) {
            int take = 0, cnt = 0;
            if (hi >= 0) {
                for (;;) {
                    const int64_t q = hi - lane;
                    const uint64_t st = q >= 0 ? peek_word(stat + q) : 0ull;
                    const uint32_t state = (uint32_t)(st >> 32) == tag ? (uint32_t)st : 0u;
                    const uint64_t mI = __ballot(state == 2u);
                    const uint64_t mA = __ballot(state >= 1u);
                    const int la = (~mA) ? __builtin_ctzll(~mA) : 64;
                    const int li = mI ? __builtin_ctzll(mI) : 64;
                    if (li < 64 && li <= la) {
                        fin = true;
                        take = li;
                        break;
                    }
                    if (la > 0) {
                        fin = false;
                        take = la;
                        break;
                    }
                    if (++spins > LOOK_BACK_SPINS) {
                        if (lane == 0) atomicOr(status, (uint32_t)QF_STALL);
                        hi = -1;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(2);
                }
                if (hi >= 0) cnt = take + (fin ? 1 : 0);
            }
            if (lane == 0) {
                s_take = take;
                s_cnt = cnt;
                s_hi = hi;
            }
        }
        __syncthreads();
        const int cnt = s_cnt;
        if (cnt == 0) break;   // hi < 0: nothing (more) to read
        const int take = s_take;
        const int64_t h = s_hi;
        C sum[NM];
#pragma unroll
        for (int t = 0; t < NM; ++t) sum[t] = P::czero();
        bool ok = true;
        if (act) {
            for (int j0 = w; j0 < cnt; j0 += NW * LB) {
                uint64_t wv[LB][W];
#pragma unroll
                for (int u = 0; u < LB; ++u) {
                    const int j = j0 + NW * u;
                    if (j < cnt) {
                        const uint64_t* src = rec + ((size_t)(h - j) * 2 + (j == take ? 1 : 0)) * WPR + c * W;
#pragma unroll
                        for (int k = 0; k < W; ++k) wv[u][k] = peek_word(src + k);
                    }
                }
#pragma unroll
                for (int u = 0; u < LB; ++u) {
                    if (j0 + NW * u < cnt) {
#pragma unroll
                        for (int t = 0; t < NM; ++t) {
                            C v;
                            ok = P::decode(wv[u] + t * P::WPV, tag, v) && ok;
                            sum[t] = P::cadd(sum[t], v);
                        }
                    }
                }
            }
#pragma unroll
            for (int t = 0; t < NM; ++t) s_part[w][t][c] = sum[t];
        }
        const bool wok = __all(ok);
        if (lane == 0) s_ok[w] = wok ? 1u : 0u;
        __syncthreads();
        if (w == 0) {
            if (s_ok[0] & s_ok[1] & s_ok[2] & s_ok[3]) {
                if (act) {
#pragma unroll
                    for (int t = 0; t < NM; ++t)
                        cc[t] = P::cadd(cc[t], P::cadd(P::cadd(s_part[0][t][c], s_part[1][t][c]),
                                                       P::cadd(s_part[2][t][c], s_part[3][t][c])));
                }
                hi = fin ? -1 : hi - take;
                spins = 0;   // progress: the budget counts polls without progress
            } else if (++spins > LOOK_BACK_SPINS) {
                if (lane == 0) atomicOr(status, (uint32_t)QF_STALL);
                hi = -1;
            } else {
                __builtin_amdgcn_s_sleep(1);   // a record was stale: read the same window again
            }
        }
    }
}

// load / store CPL consecutive columns of one row.  VEC: one 16-byte access
// per lane; the caller guarantees b % 4 == 0 and 16-byte aligned rows, so a
// lane with col0 < b owns four whole columns.
// NT marks the load non-temporal (streaming cache policy) for rows that are
// read once per pass; the value read is the same.  The elements of the
// loaded vector are copied out as plain words before the bit casts: this
// clang's __builtin_bit_cast applied to an ext_vector_type element (t.y)
// reads the vector's first element, whatever the index.
typedef uint32_t u32x4_nt __attribute__((ext_vector_type(4)));
template <int CPL, bool VEC, bool NT = false, typename E>
__device__ __forceinline__ void load_row(const E* __restrict__ row, int col0, int b, bool valid, E (&v)[CPL]) {
    if constexpr (VEC && CPL == 4 && sizeof(E) == 4) {
        if (valid && col0 < b) {
            u32x4_nt t;
            if constexpr (NT)
                t = __builtin_nontemporal_load(reinterpret_cast<const u32x4_nt*>(row + col0));
            else
                t = *reinterpret_cast<const u32x4_nt*>(row + col0);
            const uint32_t w[4] = {t[0], t[1], t[2], t[3]};
#pragma unroll
            for (int j = 0; j < 4; ++j) v[j] = __builtin_bit_cast(E, w[j]);
        } else {
#pragma unroll
            for (int j = 0; j < CPL; ++j) v[j] = E(0);
        }
    } else {
#pragma unroll
        for (int j = 0; j < CPL; ++j) v[j] = (valid && col0 + j < b) ? row[col0 + j] : E(0);
    }
}
template <int CPL, bool VEC, typename E>
__device__ __forceinline__ void store_row(E* __restrict__ row, int col0, int b, const E (&v)[CPL]) {
    if constexpr (VEC && CPL == 4 && sizeof(E) == 4) {
        uint4 t;
        t.x = __builtin_bit_cast(uint32_t, v[0]); t.y = __builtin_bit_cast(uint32_t, v[1]);
        t.z = __builtin_bit_cast(uint32_t, v[2]); t.w = __builtin_bit_cast(uint32_t, v[3]);
        if (col0 < b) *reinterpret_cast<uint4*>(row + col0) = t;
    } else {
#pragma unroll
        for (int j = 0; j < CPL; ++j)
            if (col0 + j < b) row[col0 + j] = v[j];
    }
}

}  // namespace l1
}  // namespace dm
