// k_sort.hip - segmented LSD radix sort of 32-bit keys with 32-bit point ids
// (Algorithm 1: every coordinate of every point set is one segment, sorted
// independently; stable, so equal values keep ascending point order).
//
// One pass per 8-bit digit, three kernels per pass:
//   count   - per tile, the 256-bin histogram of the digit;
//   scan    - per segment, exclusive offsets in (digit, tile) order, giving
//             every (tile, digit) pair its first output position;
//   scatter - per tile, a stable local ranking built from wavefront ballots
//             (keys of one wave that share a digit find each other with 8
//             ballots; their order inside the group is the lane order), the
//             tile reordered in LDS, then written out in digit runs.
// The final pass writes the sorted values and the permutation.  Its inverse
// (the rank array Algorithm 2 looks positions up in) is formed on request by
// rank_invert_kernel: the query scatters through perm and never reads it.
#include "dm_device.h"
#include "dm_internal.h"

namespace dm {
namespace {

constexpr int KPT = SORT_TILE / SORT_THREADS;   // keys per thread = 16
constexpr int WAVES = SORT_THREADS / DM_WAVE;   // 4
constexpr int KPW = SORT_TILE / WAVES;          // keys per wave = 1024

struct TileRange {
    int64_t seg_base;  // first key of the segment
    int64_t base;      // first key of the tile
    int32_t count;     // keys in the tile
    uint32_t seg;
};

__device__ __forceinline__ TileRange tile_range(const SegTables& t, uint32_t tile) {
    TileRange r;
    r.seg = t.tile_seg[tile];
    r.seg_base = t.key_off[r.seg];
    int64_t lt = (int64_t)(tile - t.tile_off[r.seg]);
    r.base = r.seg_base + lt * SORT_TILE;
    int64_t end = r.seg_base + t.key_len[r.seg];
    int64_t c = end - r.base;
    r.count = (int32_t)(c < SORT_TILE ? c : SORT_TILE);
    return r;
}

// exclusive scan of one value per thread over a 256-thread block
__device__ __forceinline__ uint32_t block_excl_scan_256(uint32_t v, uint32_t* s_wave /* 4 */) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t incl = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t t = __shfl_up(incl, o, 64);
        if (lane >= o) incl += t;
    }
    if (lane == 63) s_wave[w] = incl;
    __syncthreads();
    uint32_t wbase = 0;
    for (int i = 0; i < w; ++i) wbase += s_wave[i];
    __syncthreads();
    return wbase + incl - v;
}

__global__ __launch_bounds__(SORT_THREADS) void sort_count_kernel(
    const uint32_t* __restrict__ keys, uint32_t* __restrict__ counts, SegTables tb, int shift)
{
    __shared__ uint32_t h[WAVES][256];
    const int w = threadIdx.x >> 6;
    for (int i = threadIdx.x; i < WAVES * 256; i += SORT_THREADS) (&h[0][0])[i] = 0;
    __syncthreads();
    TileRange r = tile_range(tb, blockIdx.x);
    const uint32_t* k = keys + r.base;
    if (r.count == SORT_TILE) {
        // a full tile: all KPT keys of the thread are loaded before any count
        uint32_t kv[KPT];
#pragma unroll
        for (int q = 0; q < KPT; ++q) kv[q] = k[q * SORT_THREADS + threadIdx.x];
        if (shift == 24) {
            // the top digit (sign and exponent bits of float keys) takes few
            // values, so the lanes of a wave that share a digit find each
            // other with 8 ballots and only the first adds their count
#pragma unroll
            for (int q = 0; q < KPT; ++q) {
                const uint32_t dig = (kv[q] >> shift) & 255u;
                uint64_t peers = ~0ull;   // a full tile: every lane holds a key
#pragma unroll
                for (int bit = 0; bit < 8; ++bit) {
                    const bool on = (dig >> bit) & 1u;
                    const uint64_t bb = __ballot(on);
                    peers &= on ? bb : ~bb;
                }
                if (mask_rank(peers) == 0) atomicAdd(&h[w][dig], (uint32_t)__popcll(peers));
            }
        } else {
#pragma unroll
            for (int q = 0; q < KPT; ++q) atomicAdd(&h[w][(kv[q] >> shift) & 255u], 1u);
        }
    } else {
        for (int i = threadIdx.x; i < r.count; i += SORT_THREADS)
            atomicAdd(&h[w][(k[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    const int v = threadIdx.x;
    counts[(size_t)blockIdx.x * 256 + v] = h[0][v] + h[1][v] + h[2][v] + h[3][v];
}

// One block per segment; thread v owns digit v.  Replaces counts[t][v] by
// the absolute output position of tile t's first key with digit v.
__global__ __launch_bounds__(256) void sort_scan_kernel(uint32_t* __restrict__ counts, SegTables tb)
{
    __shared__ uint32_t s_wave[4];
    const uint32_t s = blockIdx.x;
    const uint32_t t0 = tb.tile_off[s], t1 = tb.tile_off[s + 1];
    const int v = threadIdx.x;
    // batches of 8 tiles: 8 independent loads in flight per thread
    constexpr uint32_t B = 8;
    uint32_t total = 0;
    uint32_t t = t0;
    for (; t + B <= t1; t += B) {
        uint32_t c[B];
#pragma unroll
        for (uint32_t q = 0; q < B; ++q) c[q] = counts[(size_t)(t + q) * 256 + v];
#pragma unroll
        for (uint32_t q = 0; q < B; ++q) total += c[q];
    }
    for (; t < t1; ++t) total += counts[(size_t)t * 256 + v];
    uint32_t run = (uint32_t)tb.key_off[s] + block_excl_scan_256(total, s_wave);
    for (t = t0; t + B <= t1; t += B) {
        uint32_t c[B];
#pragma unroll
        for (uint32_t q = 0; q < B; ++q) c[q] = counts[(size_t)(t + q) * 256 + v];
#pragma unroll
        for (uint32_t q = 0; q < B; ++q) {
            counts[(size_t)(t + q) * 256 + v] = run;
            run += c[q];
        }
    }
    for (; t < t1; ++t) {
        const uint32_t c = counts[(size_t)t * 256 + v];
        counts[(size_t)t * 256 + v] = run;
        run += c;
    }
}

// rank[k][perm[k][r]] = r: the position of each point in coordinate k's sorted
// order (the inverse permutation), one coordinate per grid row
__global__ __launch_bounds__(256) void rank_invert_kernel(const uint32_t* __restrict__ perm, int64_t ld, int64_t n,
                                                          uint32_t* __restrict__ rank, int64_t pitch)
{
    const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (r >= n) return;
    const int64_t k = blockIdx.y;
    rank[k * pitch + perm[k * ld + r]] = (uint32_t)r;
}

template <bool FIRST, bool LAST, bool IS_INT>
__global__ __launch_bounds__(SORT_THREADS) void sort_scatter_kernel(
    const uint32_t* __restrict__ kin, const uint32_t* __restrict__ vin,
    uint32_t* __restrict__ kout, uint32_t* __restrict__ vout, const uint32_t* __restrict__ offs, SegTables tb,
    int shift)
{
    __shared__ uint32_t s_keys[SORT_TILE];
    __shared__ uint32_t s_vals[SORT_TILE];
    __shared__ uint32_t s_wcnt[WAVES][256];
    __shared__ uint32_t s_base[256];   // output position of tile index 0 for each digit (mod 2^32)
    __shared__ uint32_t s_wave[4];

    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int i = threadIdx.x; i < WAVES * 256; i += SORT_THREADS) (&s_wcnt[0][0])[i] = 0;
    __syncthreads();
    const TileRange r = tile_range(tb, blockIdx.x);

    uint32_t key[KPT], val[KPT], loc[KPT];
    // wave w ranks the contiguous keys [w*KPW, (w+1)*KPW) of the tile, 64 at a
    // time in order, so (wave, iteration, lane) order is the input order.
    auto rank_key = [&](int j) {
        const int idx = w * KPW + j * 64 + lane;
        const bool valid = idx < r.count;
        const uint32_t dig = (key[j] >> shift) & 255u;
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int bit = 0; bit < 8; ++bit) {
            const bool on = (dig >> bit) & 1u;
            const uint64_t b = __ballot(on);
            peers &= on ? b : ~b;
        }
        const uint32_t before = mask_rank(peers);
        const uint32_t cnt = (uint32_t)__popcll(peers);
        uint32_t base = 0;
        if (valid) base = s_wcnt[w][dig];
        if (valid && before == cnt - 1) s_wcnt[w][dig] = base + cnt;
        loc[j] = base + before;
    };
    if (LAST && r.count == SORT_TILE) {
        // the last pass on a full tile: all KPT keys and values of the thread
        // are loaded before any ranking (2.78 -> 1.77 ms at 2^29 keys); the
        // first and middle passes keep their loads inside the ranking loop,
        // where the same preload measured slower
#pragma unroll
        for (int j = 0; j < KPT; ++j) {
            const int idx = w * KPW + j * 64 + lane;
            key[j] = kin[r.base + idx];
            val[j] = vin[r.base + idx];
        }
#pragma unroll
        for (int j = 0; j < KPT; ++j) rank_key(j);
    } else {
#pragma unroll
        for (int j = 0; j < KPT; ++j) {
            const int idx = w * KPW + j * 64 + lane;
            const bool valid = idx < r.count;
            key[j] = valid ? kin[r.base + idx] : 0u;
            if (FIRST)
                val[j] = (uint32_t)(r.base - r.seg_base + idx);
            else
                val[j] = valid ? vin[r.base + idx] : 0u;
            rank_key(j);
        }
    }
    __syncthreads();
    // per digit: wave prefixes and the tile-local start
    {
        const int v = threadIdx.x;
        const uint32_t c0 = s_wcnt[0][v], c1 = s_wcnt[1][v], c2 = s_wcnt[2][v], c3 = s_wcnt[3][v];
        const uint32_t start = block_excl_scan_256(c0 + c1 + c2 + c3, s_wave);
        // the tile's keys of digit v sit at start .. in LDS and go to offs[v] ..
        s_base[v] = offs[(size_t)blockIdx.x * 256 + v] - start;
        s_wcnt[0][v] = start;
        s_wcnt[1][v] = start + c0;
        s_wcnt[2][v] = start + c0 + c1;
        s_wcnt[3][v] = start + c0 + c1 + c2;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < KPT; ++j) {
        const int idx = w * KPW + j * 64 + lane;
        if (idx < r.count) {
            const uint32_t dig = (key[j] >> shift) & 255u;
            const uint32_t pos = s_wcnt[w][dig] + loc[j];
            s_keys[pos] = key[j];
            s_vals[pos] = val[j];
        }
    }
    __syncthreads();
    const bool as_int = LAST && (tb.seg_int ? tb.seg_int[r.seg] != 0 : IS_INT);
    // float segments are stored relative to their centre (exact, see centre_kernel)
    const float cen = (LAST && !as_int && tb.centre) ? tb.centre[r.seg] : 0.0f;
    for (int i = threadIdx.x; i < r.count; i += SORT_THREADS) {
        const uint32_t k = s_keys[i];
        const uint32_t v = s_vals[i];
        const uint32_t dig = (k >> shift) & 255u;
        const uint32_t gpos = s_base[dig] + (uint32_t)i;
        if (LAST) {
            uint32_t bits = as_int ? (uint32_t)key_i32(k) : __float_as_uint(key_f32(k) - cen);
            kout[gpos] = bits;   // sorted values
            vout[gpos] = v;      // permutation
        } else {
            kout[gpos] = k;
            vout[gpos] = v;
        }
    }
}

}  // namespace

hipError_t launch_sort_count(const uint32_t* keys, uint32_t* counts, const SegTables& t, int shift,
                             hipStream_t s)
{
    sort_count_kernel<<<t.ntiles, SORT_THREADS, 0, s>>>(keys, counts, t, shift);
    return hipGetLastError();
}

hipError_t launch_sort_scan(uint32_t* counts, const SegTables& t, hipStream_t s)
{
    sort_scan_kernel<<<(unsigned)t.nseg, 256, 0, s>>>(counts, t);
    return hipGetLastError();
}

hipError_t launch_sort_scatter(const uint32_t* kin, const uint32_t* vin, uint32_t* kout, uint32_t* vout,
                               const uint32_t* offs, const SegTables& t, int shift, bool first, bool last,
                               bool is_int, hipStream_t s)
{
#define DM_SCATTER(F, L, I) \
    sort_scatter_kernel<F, L, I><<<t.ntiles, SORT_THREADS, 0, s>>>(kin, vin, kout, vout, offs, t, shift)
    if (first && last) return hipErrorInvalidValue;   // four passes always
    if (first) DM_SCATTER(true, false, false);
    else if (!last) DM_SCATTER(false, false, false);
    else if (is_int) DM_SCATTER(false, true, true);
    else DM_SCATTER(false, true, false);
#undef DM_SCATTER
    return hipGetLastError();
}

hipError_t launch_rank_invert(const uint32_t* perm, int64_t ld, int64_t n, int32_t d, uint32_t* rank, int64_t pitch,
                              hipStream_t s)
{
    if (n < 1 || d < 1 || ld < n || pitch < n) return hipErrorInvalidValue;
    const dim3 grid((unsigned)((n + 255) / 256), (unsigned)d);
    rank_invert_kernel<<<grid, 256, 0, s>>>(perm, ld, n, rank, pitch);
    return hipGetLastError();
}

}  // namespace dm
