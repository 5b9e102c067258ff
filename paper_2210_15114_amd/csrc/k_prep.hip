// k_prep.hip - preparation kernels: validation, the coordinate-major key
// arrays that Algorithm 1 sorts, per-coordinate ranges, FP32 copy of X for the
// l2-squared query and the FP64/int64 row statistics.
#include "dm_device.h"
#include "dm_internal.h"

namespace dm {
namespace {

// Value of one input element as the kernels see it (FP32 for float data,
// int32 for integer data) plus validity bits.
template <int KIND> struct In;
template <> struct In<IN_F32> {
    using T = float;
    using V = float;
    __device__ static V conv(T x, uint32_t& bad) {
        if (!isfinite(x)) bad |= FLAG_NONFINITE;
        return x;
    }
    __device__ static uint32_t key(V v) { return f32_key(v); }
};
template <> struct In<IN_F64> {
    using T = double;
    using V = float;
    __device__ static V conv(T x, uint32_t& bad) {
        float v = (float)x;                   // round to nearest even
        if (!isfinite(x) || !isfinite(v)) bad |= FLAG_NONFINITE;
        return v;
    }
    __device__ static uint32_t key(V v) { return f32_key(v); }
};
template <> struct In<IN_I32> {
    using T = int32_t;
    using V = int32_t;
    __device__ static V conv(T x, uint32_t& bad) {
        if (x == INT32_MIN) bad |= FLAG_INT_RANGE;      // |x| < 2^31 required
        return x;
    }
    __device__ static uint32_t key(V v) { return i32_key(v); }
};
template <> struct In<IN_I64> {
    using T = int64_t;
    using V = int32_t;
    __device__ static V conv(T x, uint32_t& bad) {
        if (x <= -(int64_t(1) << 31) || x >= (int64_t(1) << 31)) bad |= FLAG_INT_RANGE;
        return (int32_t)x;
    }
    __device__ static uint32_t key(V v) { return i32_key(v); }
};

constexpr int TT = 64;  // transpose tile: 64 rows x 64 coordinates

// RT consecutive 64 x 64 tiles of X (rows r0 .., coordinates c0 .. +63) per
// workgroup: validates them, writes their keys coordinate-major (coalesced
// both ways through LDS) and their FP32/int32 copy row-major, and folds the
// per-coordinate min/max keys of all RT tiles into kmin/kmax with one atomic
// per coordinate (one per tile contended heavily on the d addresses).
constexpr int RT = 16;
template <int KIND>
__global__ __launch_bounds__(256) void prep_transpose_kernel(
    const typename In<KIND>::T* __restrict__ X, int64_t n, int32_t d,
    uint32_t* __restrict__ keys, int64_t ld, typename In<KIND>::V* __restrict__ xcopy,
    uint32_t* __restrict__ kmin, uint32_t* __restrict__ kmax, uint32_t* __restrict__ flags)
{
    using I = In<KIND>;
    __shared__ uint32_t tile[TT][TT + 1];
    __shared__ uint32_t smin[4][TT], smax[4][TT];
    const int32_t c0 = blockIdx.y * TT;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const int32_t col = c0 + tx;
    uint32_t bad = 0, lo = 0xffffffffu, hi = 0u;
    for (int q = 0; q < RT; ++q) {
        const int64_t r0 = ((int64_t)blockIdx.x * RT + q) * TT;
        if (r0 >= n) break;   // the same on every thread
        __syncthreads();      // the previous tile has been written out
        for (int rr = ty; rr < TT; rr += 4) {
            int64_t row = r0 + rr;
            uint32_t k = 0;
            if (row < n && col < d) {
                typename I::V v = I::conv(X[row * d + col], bad);
                if (xcopy) xcopy[row * d + col] = v;
                k = I::key(v);
                lo = min(lo, k);
                hi = max(hi, k);
            }
            tile[rr][tx] = k;
        }
        __syncthreads();
        if (keys) {
            for (int cc = ty; cc < TT; cc += 4) {
                int32_t c = c0 + cc;
                int64_t row = r0 + tx;
                if (c < d && row < n) keys[(int64_t)c * ld + row] = tile[tx][cc];
            }
        }
    }
    smin[ty][tx] = lo;
    smax[ty][tx] = hi;
    if (bad) atomicOr(flags, bad);
    __syncthreads();
    if (ty == 0 && col < d) {
        uint32_t a = min(min(smin[0][tx], smin[1][tx]), min(smin[2][tx], smin[3][tx]));
        uint32_t b = max(max(smax[0][tx], smax[1][tx]), max(smax[2][tx], smax[3][tx]));
        atomicMin(kmin + col, a);
        atomicMax(kmax + col, b);
    }
}

// Row statistics: rowsum[i] = sum_k x~_ik^p (p = 1: the row sum; p odd >= 3:
// the weights of the l_p^p query's constant term), rownrm[i] = sum_k x~_ik^2,
// where x~_ik = x_ik - c_k for float data with per-coordinate centres c (exact
// in FP32, see centre_kernel) and x~ = x otherwise.  With xcopy set, the
// FP32 (int32) values x~ are also written row-major (n x d).
// G = 2^lg lanes share a row: lane l takes k = l, l + G, ... in ascending order
// (each load instruction reads G consecutive values of the row), and the G
// partial sums are then added by a fixed xor butterfly, so every FP64 sum is
// reproducible.  Integer data runs in wrapping int64 (exact modulo 2^64).
template <int KIND>
__global__ __launch_bounds__(256) void row_stats_kernel(
    const typename In<KIND>::T* __restrict__ X, int64_t n, int32_t d, int p, int lg, void* rowsum, void* rownrm,
    const float* __restrict__ centre, typename In<KIND>::V* __restrict__ xcopy)
{
    using I = In<KIND>;
    const int G = 1 << lg;
    const int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> lg;
    const int l = (int)(threadIdx.x & (G - 1));
    const bool valid = i < n;   // every lane takes part in the butterfly
    const typename I::T* xi = X + (valid ? i : 0) * d;
    uint32_t bad = 0;
    if constexpr (KIND == IN_F32 || KIND == IN_F64) {
        double s = 0.0, q = 0.0;
        if (valid) {
            for (int32_t k = l; k < d; k += G) {
                float t = I::conv(xi[k], bad);
                if (centre) t = t - centre[k];   // exact (Sterbenz)
                if (xcopy) xcopy[i * d + k] = t;
                const double v = (double)t;
                double vp = v;
                for (int e = 1; e < p; ++e) vp *= v;
                s += vp;
                q += v * v;
            }
        }
        for (int off = 1; off < G; off <<= 1) {
            s += __shfl_xor(s, off);
            q += __shfl_xor(q, off);
        }
        if (valid && l == 0) {
            ((double*)rowsum)[i] = s;
            ((double*)rownrm)[i] = q;
        }
    } else {
        uint64_t s = 0, q = 0;
        if (valid) {
            for (int32_t k = l; k < d; k += G) {
                const int32_t t = I::conv(xi[k], bad);
                if (xcopy) xcopy[i * d + k] = t;
                const int64_t v = (int64_t)t;
                uint64_t vp = (uint64_t)v;
                for (int e = 1; e < p; ++e) vp *= (uint64_t)v;
                s += vp;
                q += (uint64_t)v * (uint64_t)v;
            }
        }
        for (int off = 1; off < G; off <<= 1) {
            s += (uint64_t)__shfl_xor((unsigned long long)s, off);
            q += (uint64_t)__shfl_xor((unsigned long long)q, off);
        }
        if (valid && l == 0) {
            ((int64_t*)rowsum)[i] = (int64_t)s;
            ((int64_t*)rownrm)[i] = (int64_t)q;
        }
    }
}

// Centres of float coordinates.  The terms the sorted query forms (x times a
// prefix of z, prefix sums of x z, their totals) grow with |x|, while the
// result only depends on differences of coordinates; for points far from the
// origin (say 10^4 + U[0, 1)) FP32 would lose the differences to cancellation.
// Every metric of the sorted path and l2 squared is invariant under
// translating a coordinate, so the coordinate is shifted by c_k and nothing
// else changes, provided x - c_k is exact for every x of the coordinate.  By
// Sterbenz's lemma it is whenever c_k / 2 <= x <= 2 c_k (or the mirror image
// for negative values): c_k is the FP32 midpoint of [min_k, max_k] when the
// whole range satisfies that, else 0 (a range that reaches zero or spans a
// factor of about three or more: there |x| <= 1.5 (max_k - min_k) already).
__global__ void centre_kernel(const uint32_t* __restrict__ kmin, const uint32_t* __restrict__ kmax, int32_t d,
                              float* __restrict__ centre)
{
    const int32_t k = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
    if (k >= d) return;
    const float lo = key_f32(kmin[k]), hi = key_f32(kmax[k]);
    const float m = 0.5f * lo + 0.5f * hi;
    float c = 0.0f;
    if (lo > 0.0f && m <= 2.0f * lo && hi <= 2.0f * m) c = m;
    if (hi < 0.0f && m >= 2.0f * hi && lo >= 2.0f * m) c = m;
    centre[k] = c;
}

// xs[k * pitch + r] += centre[k] for r < n: the sorted values of coordinate k
// back in the caller's frame (exact: the stored value is x - c_k exactly)
__global__ __launch_bounds__(256) void add_centre_kernel(float* __restrict__ xs, int64_t n, int64_t pitch,
                                                         const float* __restrict__ centre)
{
    const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (r < n) xs[(int64_t)blockIdx.y * pitch + r] += centre[blockIdx.y];
}

__global__ void fill_u32_kernel(uint32_t* p, uint32_t v, size_t count) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i < count; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}

// plain streaming copy, one 16-byte element per lane (a grid-stride loop over
// a capped grid reaches about a quarter less bandwidth on gfx950)
__global__ __launch_bounds__(256) void copy_probe_kernel(uint4* __restrict__ dst, const uint4* __restrict__ src,
                                                         size_t n16) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n16) dst[i] = src[i];
}

// random-row probe: Out[perm[r]] += Z[perm[r]] for every rank r, rows of b
// FP32 values (b a power of two, 4..64) read and written with one 16-byte
// access per lane, GP ranks per row slot in flight; the gather and
// read-modify-write of a coordinate pass without its scan.  Indices >= n are
// skipped.
constexpr int GP = 8;
__global__ __launch_bounds__(256) void gather_probe_kernel(const uint32_t* __restrict__ perm,
                                                           const float* __restrict__ Z, float* __restrict__ Out,
                                                           int64_t n, int32_t b)
{
    const int lpr = b >> 2, slots = 256 / lpr;
    const int slot = threadIdx.x / lpr, col = (threadIdx.x % lpr) * 4;
    const int64_t r0 = ((int64_t)blockIdx.x * slots + slot) * GP;
    uint32_t p[GP];
    float4 g[GP], o[GP];
#pragma unroll
    for (int i = 0; i < GP; ++i) p[i] = r0 + i < n ? perm[r0 + i] : 0xffffffffu;
#pragma unroll
    for (int i = 0; i < GP; ++i)
        if (p[i] < n) g[i] = *reinterpret_cast<const float4*>(Z + (size_t)p[i] * b + col);
#pragma unroll
    for (int i = 0; i < GP; ++i)
        if (p[i] < n) o[i] = *reinterpret_cast<const float4*>(Out + (size_t)p[i] * b + col);
#pragma unroll
    for (int i = 0; i < GP; ++i)
        if (p[i] < n) {
            o[i].x += g[i].x;
            o[i].y += g[i].y;
            o[i].z += g[i].z;
            o[i].w += g[i].w;
            *reinterpret_cast<float4*>(Out + (size_t)p[i] * b + col) = o[i];
        }
}

// p[i] *= s
__global__ __launch_bounds__(256) void scale_f32_kernel(float* __restrict__ p, size_t count, float s)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x)
        p[i] *= s;
}

}  // namespace

hipError_t launch_scale_f32(float* p, size_t count, float s, hipStream_t st)
{
    if (count == 0) return hipSuccess;
    size_t blocks = (count + 255) / 256;
    if (blocks > 256 * 64) blocks = 256 * 64;
    scale_f32_kernel<<<(unsigned)blocks, 256, 0, st>>>(p, count, s);
    return hipGetLastError();
}

hipError_t launch_copy_probe(void* dst, const void* src, size_t bytes, hipStream_t s)
{
    const size_t n16 = bytes / 16;
    // grids of at most 2^30 lanes (16 GiB per launch)
    constexpr size_t CHUNK = (size_t)1 << 30;
    for (size_t at = 0; at < n16; at += CHUNK) {
        const size_t cnt = n16 - at < CHUNK ? n16 - at : CHUNK;
        copy_probe_kernel<<<(unsigned)((cnt + 255) / 256), 256, 0, s>>>((uint4*)dst + at, (const uint4*)src + at, cnt);
    }
    return hipGetLastError();
}

hipError_t launch_gather_probe(const uint32_t* perm, const float* Z, float* Out, int64_t n, int32_t b,
                               hipStream_t s)
{
    const int64_t per = (int64_t)(256 / (b / 4)) * GP;   // ranks per workgroup
    const int64_t grid = (n + per - 1) / per;
    if (grid > 0x7fffffff) return hipErrorInvalidValue;
    gather_probe_kernel<<<(unsigned)grid, 256, 0, s>>>(perm, Z, Out, n, b);
    return hipGetLastError();
}

hipError_t launch_prep_transpose(int kind, const void* X, int64_t n, int32_t d, uint32_t* keys,
                                 int64_t ld, void* xcopy, uint32_t* kmin, uint32_t* kmax, uint32_t* flags,
                                 hipStream_t s)
{
    dim3 grid((unsigned)((n + (int64_t)TT * RT - 1) / ((int64_t)TT * RT)), (unsigned)((d + TT - 1) / TT));
    switch (kind) {
    case IN_F32:
        prep_transpose_kernel<IN_F32><<<grid, 256, 0, s>>>((const float*)X, n, d, keys, ld, (float*)xcopy,
                                                           kmin, kmax, flags);
        break;
    case IN_F64:
        prep_transpose_kernel<IN_F64><<<grid, 256, 0, s>>>((const double*)X, n, d, keys, ld, (float*)xcopy,
                                                           kmin, kmax, flags);
        break;
    case IN_I32:
        prep_transpose_kernel<IN_I32><<<grid, 256, 0, s>>>((const int32_t*)X, n, d, keys, ld,
                                                           (int32_t*)xcopy, kmin, kmax, flags);
        break;
    case IN_I64:
        prep_transpose_kernel<IN_I64><<<grid, 256, 0, s>>>((const int64_t*)X, n, d, keys, ld,
                                                           (int32_t*)xcopy, kmin, kmax, flags);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_row_stats(int kind, const void* X, int64_t n, int32_t d, void* rowsum, void* rownrm,
                            hipStream_t s, int p, const float* centre, void* xcopy)
{
    if (n < 1 || d < 1) return hipErrorInvalidValue;
    // lanes per row: the power of two nearest above d / 4, at most 64
    int lg = 0;
    while ((1 << lg) < 64 && (int64_t)(1 << lg) * 4 < d) ++lg;
    const int64_t threads = n << lg;
    const unsigned grid = (unsigned)((threads + 255) / 256);
    switch (kind) {
    case IN_F32:
        row_stats_kernel<IN_F32><<<grid, 256, 0, s>>>((const float*)X, n, d, p, lg, rowsum, rownrm, centre,
                                                      (float*)xcopy);
        break;
    case IN_F64:
        row_stats_kernel<IN_F64><<<grid, 256, 0, s>>>((const double*)X, n, d, p, lg, rowsum, rownrm, centre,
                                                      (float*)xcopy);
        break;
    case IN_I32:
        row_stats_kernel<IN_I32><<<grid, 256, 0, s>>>((const int32_t*)X, n, d, p, lg, rowsum, rownrm, nullptr,
                                                      (int32_t*)xcopy);
        break;
    case IN_I64:
        row_stats_kernel<IN_I64><<<grid, 256, 0, s>>>((const int64_t*)X, n, d, p, lg, rowsum, rownrm, nullptr,
                                                      (int32_t*)xcopy);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_centre(const uint32_t* kmin, const uint32_t* kmax, int32_t d, float* centre, hipStream_t s)
{
    if (d < 1) return hipErrorInvalidValue;
    centre_kernel<<<(unsigned)((d + 255) / 256), 256, 0, s>>>(kmin, kmax, d, centre);
    return hipGetLastError();
}

hipError_t launch_add_centre(float* xs, int64_t n, int32_t d, int64_t pitch, const float* centre, hipStream_t s)
{
    if (n < 1 || d < 1 || pitch < n) return hipErrorInvalidValue;
    const dim3 grid((unsigned)((n + 255) / 256), (unsigned)d);
    add_centre_kernel<<<grid, 256, 0, s>>>(xs, n, pitch, centre);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, uint32_t v, size_t count, hipStream_t s)
{
    if (count == 0) return hipSuccess;
    size_t blocks = (count + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    fill_u32_kernel<<<(unsigned)blocks, 256, 0, s>>>(p, v, count);
    return hipGetLastError();
}

}  // namespace dm
