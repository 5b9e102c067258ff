// k_l1.hip - per-query totals of the l1 query (T0, U and the guard sums)
// and the dispatch of the coordinate passes (l1_pass.h) by data path, block
// width and tuned variant.
#include <mutex>
#include <type_traits>
#include <vector>

#include "dm_device.h"
#include "dm_internal.h"

namespace dm {

int persistent_grid(const void* fn, const void* fn2, int64_t ntiles) {
    struct Entry { int dev; const void* fn; int per_cu; int cus; };
    static std::mutex mu;
    static std::vector<Entry> cache;
    int dev = 0;
    (void)hipGetDevice(&dev);
    int per_cu = 0, cus = 0;
    {
        std::lock_guard<std::mutex> lock(mu);
        for (const Entry& e : cache)
            if (e.dev == dev && e.fn == fn) {
                per_cu = e.per_cu;
                cus = e.cus;
            }
        if (per_cu == 0) {
            if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
                cus = 256;
            int nb = 0, nb2 = 0;
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, 256, 0) != hipSuccess || nb < 1) nb = 1;
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb2, fn2, 256, 0) != hipSuccess || nb2 < 1) nb2 = 1;
            per_cu = nb < nb2 ? nb : nb2;
            cache.push_back(Entry{dev, fn, per_cu, cus});
        }
    }
    int64_t g = (int64_t)per_cu * cus;
    if (g > ntiles) g = ntiles;
    if (g < 1) g = 1;
    return (int)g;
}
namespace {

// ---------------------------------------------------------------------------
// totals: T0[c] = sum_j z_jc, U[c] = sum_j w_j z_jc, and ||z_c||_1
// two fixed-order stages (per-block partials, then one block), so FP64
// results are reproducible run to run.
// ---------------------------------------------------------------------------
constexpr int TOT_ROWS = 4096;  // rows per stage-1 block
constexpr int TOT_MAXB = 1024;

// V adjacent columns per thread, loaded as one vector when V > 1
template <typename T, int V>
struct alignas(sizeof(T) * V) ZVec {
    T v[V];
};

// thread layout: column group (tid % bpc) of V adjacent columns, row lane
// tid / bpc; rows are taken 4 at a time so that 4 loads are in flight
template <bool INT, typename ZT, typename WT, int V>
__global__ __launch_bounds__(256) void totals_stage1(const ZT* __restrict__ Z, int64_t n, int32_t b,
                                                     const WT* __restrict__ wgt, void* __restrict__ partials,
                                                     uint32_t* __restrict__ status)
{
    const int ng = (b + V - 1) / V;   // column groups
    int bpc = 1;
    while (bpc < ng && bpc < 256) bpc <<= 1;
    const int rl = threadIdx.x / bpc, rs = 256 / bpc;
    const int64_t j0 = (int64_t)blockIdx.x * TOT_ROWS;
    const int64_t j1 = min(n, j0 + TOT_ROWS);
    __shared__ double s_f[3][V][256];
    __shared__ int64_t s_i[2][V][256];
    uint32_t bad = 0;
    for (int gbase = 0; gbase < ng; gbase += bpc) {
        const int grp = gbase + (int)(threadIdx.x % bpc);
        const int c0 = grp * V;
        double f0[V], f1[V], fl[V];
        uint64_t i0[V], i1[V];
#pragma unroll
        for (int v = 0; v < V; ++v) {
            f0[v] = f1[v] = fl[v] = 0.0;
            i0[v] = i1[v] = 0;
        }
        auto add = [&](const ZVec<ZT, V>& zr, WT wj) {
#pragma unroll
            for (int v = 0; v < V; ++v) {
                const ZT z = zr.v[v];
                if constexpr (INT) {
                    i0[v] += (uint64_t)(int64_t)z;
                    i1[v] += (uint64_t)(int64_t)wj * (uint64_t)(int64_t)z;
                    fl[v] += fabs((double)z);
                } else {
                    if (!isfinite(z)) bad = 1;
                    f0[v] += (double)z;
                    f1[v] += (double)wj * (double)z;
                    fl[v] += fabs((double)z);
                }
            }
        };
        if (grp < ng) {
            int64_t j = j0 + rl;
            for (; j + 3 * (int64_t)rs < j1; j += 4 * (int64_t)rs) {
                ZVec<ZT, V> zr[4];
                WT wj[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int64_t r = j + u * (int64_t)rs;
                    if (V > 1) {
                        zr[u] = *reinterpret_cast<const ZVec<ZT, V>*>(Z + r * b + c0);
                    } else {
                        zr[u].v[0] = Z[r * b + c0];
                    }
                    wj[u] = wgt[r];
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) add(zr[u], wj[u]);
            }
            for (; j < j1; j += rs) {
                ZVec<ZT, V> zr;
                if (V > 1) {
                    zr = *reinterpret_cast<const ZVec<ZT, V>*>(Z + j * b + c0);
                } else {
                    zr.v[0] = Z[j * b + c0];
                }
                add(zr, wgt[j]);
            }
        }
#pragma unroll
        for (int v = 0; v < V; ++v) {
            s_f[0][v][threadIdx.x] = f0[v];
            s_f[1][v][threadIdx.x] = f1[v];
            s_f[2][v][threadIdx.x] = fl[v];
            s_i[0][v][threadIdx.x] = (int64_t)i0[v];
            s_i[1][v][threadIdx.x] = (int64_t)i1[v];
        }
        __syncthreads();
        if ((int)threadIdx.x < bpc && grp < ng) {
#pragma unroll
            for (int v = 0; v < V; ++v) {
                const int c = c0 + v;
                if (c >= b) continue;
                double a0 = 0, a1 = 0, al = 0;
                uint64_t b0 = 0, b1 = 0;
                for (int r = 0; r < rs; ++r) {
                    const int t = r * bpc + threadIdx.x;
                    a0 += s_f[0][v][t]; a1 += s_f[1][v][t]; al += s_f[2][v][t];
                    b0 += (uint64_t)s_i[0][v][t]; b1 += (uint64_t)s_i[1][v][t];
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
    // 16-byte row loads when every row of Z starts on a 16-byte boundary
    const size_t zb = (!is_int || zkind == IN_I32) ? 4 : 8;
    const int vw = (int)(16 / zb);
    const bool vec = b % vw == 0 && (uintptr_t)Z % 16 == 0;
    if (!is_int) {
        if (vec)
            totals_stage1<false, float, double, 4><<<nblk, 256, 0, s>>>((const float*)Z, n, b, (const double*)w,
                                                                        o.partials, o.status);
        else
            totals_stage1<false, float, double, 1><<<nblk, 256, 0, s>>>((const float*)Z, n, b, (const double*)w,
                                                                        o.partials, o.status);
    } else if (zkind == IN_I32) {
        if (vec)
            totals_stage1<true, int32_t, int64_t, 4><<<nblk, 256, 0, s>>>((const int32_t*)Z, n, b,
                                                                          (const int64_t*)w, o.partials, o.status);
        else
            totals_stage1<true, int32_t, int64_t, 1><<<nblk, 256, 0, s>>>((const int32_t*)Z, n, b,
                                                                          (const int64_t*)w, o.partials, o.status);
    } else {
        if (vec)
            totals_stage1<true, int64_t, int64_t, 2><<<nblk, 256, 0, s>>>((const int64_t*)Z, n, b,
                                                                          (const int64_t*)w, o.partials, o.status);
        else
            totals_stage1<true, int64_t, int64_t, 1><<<nblk, 256, 0, s>>>((const int64_t*)Z, n, b,
                                                                          (const int64_t*)w, o.partials, o.status);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (is_int)
        totals_stage2<true><<<b, 256, 0, s>>>(o.partials, nblk, b, o.T0, o.U, o.zl1, guard_scale, o.status);
    else
        totals_stage2<false><<<b, 256, 0, s>>>(o.partials, nblk, b, o.T0, o.U, o.zl1, guard_scale, o.status);
    return hipGetLastError();
}

static int bpad_i(int32_t b) {
    int bp = 1;
    while (bp < b) bp <<= 1;
    return bp;
}

static int kind_of(bool is_int, int zkind) { return !is_int ? 0 : zkind == IN_I32 ? 1 : 2; }

int l1_tile_ranks(int32_t b, bool is_int, int zkind, int variant) {
    switch (kind_of(is_int, zkind)) {
    case 0: return l1_tile_ranks_f32(b, variant);
    case 1: return l1_tile_ranks_i32(b, variant);
    default: return l1_tile_ranks_i64(b, variant);
    }
}

size_t l1_record_words(int64_t n, int32_t b, bool is_int, int zkind, int variant) {
    const int64_t tile = l1_tile_ranks(b, is_int, zkind, variant);
    if (tile <= 0) return 0;
    const int64_t ntiles = (n + tile - 1) / tile;
    const size_t wpv = is_int ? 2 : 1;
    return (size_t)ntiles * (2 * 2 * wpv * (size_t)bpad_i(b) + 1);   // two records and one status word per tile
}

// Each (data path, block width, variant) has its own ticket class and record
// region, so no shape ever reads another's words.
L1Shape l1_shape(int64_t n, int32_t b, bool is_int, int zkind, int variant) {
    L1Shape sh;
    int lg = 0;
    while ((1 << lg) < b) ++lg;
    sh.cls = (kind_of(is_int, zkind) * 8 + lg) * L1_VARIANTS + variant;
    sh.record_words = l1_record_words(n, b, is_int, zkind, variant);
    return sh;
}

L1Shape l1_single_shape(int64_t n, bool is_int, int zkind, int variant) {
    L1Shape sh;
    sh.cls = L1_CLASSES + LP_CLASSES + kind_of(is_int, zkind) * L1_VARIANTS + variant;
    sh.record_words = l1_record_words(n, 1, is_int, zkind, variant);
    return sh;
}

namespace {

// Out[i] = (first ? U : Out[i]) + sum_k Cs[k][i] over the g coordinates of a
// group (b = 1), coalesced over the points.
template <bool INT>
__global__ __launch_bounds__(256) void l1_combine(int64_t ld, const void* __restrict__ Cs, int64_t n, int32_t g,
                                                  int first, const void* __restrict__ U, void* __restrict__ Out)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    if constexpr (INT) {
        const int64_t* C = (const int64_t*)Cs + i;
        uint64_t acc = (uint64_t)(first ? ((const int64_t*)U)[0] : ((const int64_t*)Out)[i]);
        for (int32_t k = 0; k < g; ++k) acc += (uint64_t)C[(int64_t)k * ld];
        ((int64_t*)Out)[i] = (int64_t)acc;
    } else {
        const float* C = (const float*)Cs + i;
        double acc = first ? ((const double*)U)[0] : (double)((const float*)Out)[i];
        for (int32_t k = 0; k < g; ++k) acc += (double)C[(int64_t)k * ld];
        ((float*)Out)[i] = (float)acc;
    }
}

}  // namespace

hipError_t launch_l1_combine(bool is_int, int64_t ld, const void* Cs, int64_t n, int32_t g, bool first,
                             const void* U, void* Out, hipStream_t s)
{
    if (n < 1 || g < 1 || ld < n) return hipErrorInvalidValue;
    const unsigned grid = (unsigned)((n + 255) / 256);
    if (is_int)
        l1_combine<true><<<grid, 256, 0, s>>>(ld, Cs, n, g, first ? 1 : 0, U, Out);
    else
        l1_combine<false><<<grid, 256, 0, s>>>(ld, Cs, n, g, first ? 1 : 0, U, Out);
    return hipGetLastError();
}

hipError_t launch_l1_pass(bool is_int, int zkind, int32_t b, const L1PassArgs& a, hipStream_t s)
{
    if (b < 1 || b > 64 || a.variant < 0 || a.variant >= L1_VARIANTS) return hipErrorInvalidValue;
    if (a.cls < 0 || a.cls >= CHAIN_CLASSES) return hipErrorInvalidValue;
    switch (kind_of(is_int, zkind)) {
    case 0: return launch_l1_pass_f32(a, b, a.variant, s);
    case 1: return launch_l1_pass_i32(a, b, a.variant, s);
    default: return launch_l1_pass_i64(a, b, a.variant, s);
    }
}

}  // namespace dm
