// k_l2.hip - the l2-squared query (Algorithm 3, Appendix A):
//     (A z)_i = ||x_i||^2 S0 + R - 2 <x_i, V>,
//     S0 = sum_j z_j,  R = sum_j ||x_j||^2 z_j,  V = X^T z
// (the rank-one terms and the Gram matrix of the decomposition in Section
// 1.2, with the first power of z in S0 and R).
//
// S0 and R come from the totals kernel (weights ||x_j||^2) in FP64.  V is a
// split-K reduction over the points: stage 1 writes one FP64 partial of
// X^T Z per block of rows, stage 2 adds the partials in block order.  The
// apply stage forms <x_i, V> per row and combines the rank-one terms in FP64.
// For float data with at least 16 right-hand sides and d <= 128 both
// contractions run on the BF16 matrix cores (k_l2_mfma.hip).  Other float
// shapes are the linear form of the sort-free kernels (k_sortfree.hip) with
// V = -2 X^T z, weights a_i = ||x_i||^2 on S0 and U = R, all in FP64.  This
// file's vector path serves integer data (wrapping int64, exact modulo 2^64).
#include "dm_device.h"
#include "dm_internal.h"

namespace dm {
namespace {

constexpr int VROWS = 2048;   // rows per stage-1 block
constexpr int CH = 16;        // rows staged in LDS at a time
constexpr int EPT = 32;       // V entries per thread per group

template <bool INT> struct L2T;
template <> struct L2T<false> {
    using X = float;
    using P = double;    // partial / V element
};
template <> struct L2T<true> {
    using X = int32_t;
    using P = int64_t;
};

template <bool INT, typename ZT>
__global__ __launch_bounds__(256) void xtz_stage1(const typename L2T<INT>::X* __restrict__ X, int64_t n,
                                                  int32_t d, const ZT* __restrict__ Z, int32_t b,
                                                  typename L2T<INT>::P* __restrict__ part)
{
    using XT = typename L2T<INT>::X;
    using PT = typename L2T<INT>::P;
    extern __shared__ unsigned char smem[];
    XT* sx = (XT*)smem;                              // CH x d
    ZT* sz = (ZT*)(smem + sizeof(XT) * CH * d);      // CH x b
    const int64_t j0 = (int64_t)blockIdx.x * VROWS;
    const int64_t j1 = min(n, j0 + VROWS);
    const int ent = d * b;
    for (int g0 = 0; g0 < ent; g0 += 256 * EPT) {
        double af[EPT];
        uint64_t ai[EPT];
#pragma unroll
        for (int m = 0; m < EPT; ++m) { af[m] = 0.0; ai[m] = 0; }
        for (int64_t jc = j0; jc < j1; jc += CH) {
            const int rows = (int)min((int64_t)CH, j1 - jc);
            __syncthreads();
            for (int t = threadIdx.x; t < rows * d; t += 256) sx[t] = X[jc * d + t];
            for (int t = threadIdx.x; t < rows * b; t += 256) sz[t] = Z[jc * b + t];
            __syncthreads();
#pragma unroll
            for (int m = 0; m < EPT; ++m) {
                const int e = g0 + threadIdx.x + 256 * m;
                if (e < ent) {
                    const int k = e / b, c = e % b;
                    for (int r = 0; r < rows; ++r) {
                        if constexpr (INT)
                            ai[m] += (uint64_t)(int64_t)sx[r * d + k] * (uint64_t)(int64_t)sz[r * b + c];
                        else
                            af[m] = fma((double)sx[r * d + k], (double)sz[r * b + c], af[m]);
                    }
                }
            }
        }
#pragma unroll
        for (int m = 0; m < EPT; ++m) {
            const int e = g0 + threadIdx.x + 256 * m;
            if (e < ent) {
                if constexpr (INT)
                    part[(size_t)blockIdx.x * ent + e] = (int64_t)ai[m];
                else
                    part[(size_t)blockIdx.x * ent + e] = af[m];
            }
        }
    }
}

template <bool INT>
__global__ __launch_bounds__(256) void xtz_stage2(const typename L2T<INT>::P* __restrict__ part, int nblk,
                                                  int ent, typename L2T<INT>::P* __restrict__ V)
{
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= ent) return;
    if constexpr (INT) {
        uint64_t s = 0;
        for (int k = 0; k < nblk; ++k) s += (uint64_t)part[(size_t)k * ent + e];
        V[e] = (int64_t)s;
    } else {
        double s = 0.0;
        for (int k = 0; k < nblk; ++k) s += part[(size_t)k * ent + e];
        V[e] = s;
    }
}

// Out[i, c] = nrm_i S0_c + R_c - 2 sum_k x_ik V_kc
template <bool INT>
__global__ __launch_bounds__(256) void l2_apply_vec(const typename L2T<INT>::X* __restrict__ X, int64_t n,
                                                    int32_t d, const typename L2T<INT>::P* __restrict__ V,
                                                    int32_t b, const void* __restrict__ nrm,
                                                    const void* __restrict__ S0, const void* __restrict__ R,
                                                    void* __restrict__ Out)
{
    int bpc = 1;
    while (bpc < b && bpc < 256) bpc <<= 1;
    const int rs = 256 / bpc;
    const int c = threadIdx.x % bpc;
    const int64_t i = (int64_t)blockIdx.x * rs + threadIdx.x / bpc;
    if (i >= n) return;
    const typename L2T<INT>::X* xi = X + i * d;
    for (int cc = c; cc < b; cc += bpc) {
        if constexpr (INT) {
            uint64_t acc = 0;
            for (int k = 0; k < d; ++k) acc += (uint64_t)(int64_t)xi[k] * (uint64_t)V[(size_t)k * b + cc];
            const uint64_t r = (uint64_t)((const int64_t*)nrm)[i] * (uint64_t)((const int64_t*)S0)[cc] +
                               (uint64_t)((const int64_t*)R)[cc] - 2ull * acc;
            ((int64_t*)Out)[i * b + cc] = (int64_t)r;
        } else {
            double acc = 0.0;
            for (int k = 0; k < d; ++k) acc = fma((double)xi[k], V[(size_t)k * b + cc], acc);
            const double r = ((const double*)nrm)[i] * ((const double*)S0)[cc] + ((const double*)R)[cc] -
                             2.0 * acc;
            ((float*)Out)[i * b + cc] = (float)r;
        }
    }
}

}  // namespace

size_t l2_scratch_bytes(int64_t n, int32_t d, int32_t b) {
    const size_t nblk = (size_t)((n + VROWS - 1) / VROWS);
    // the integer path's partials; then, for float data, the matrix-core
    // form (d <= 128, 16 <= b <= 64) or else the linear sort-free form
    const size_t vec = (nblk + 1) * (size_t)d * (size_t)b * 8 + 256;
    const bool mfma = d <= 128 && b >= 16 && b <= 64;
    const size_t fl = mfma ? l2_mfma_scratch_bytes(n, d, b) : sf_scratch_bytes(n, d, b, SF_LIN, 1);
    return vec > fl ? vec : fl;
}

hipError_t launch_l2sq_mfma(int zkind, const float* Xc, const double* nrm, int64_t n, int32_t d, const float* Z,
                            int32_t b, float* Out, void* scratch, const TotalsOut& tot, double guard_scale,
                            hipStream_t s, bool* used);

hipError_t launch_l2sq(bool is_int, int zkind, const void* Xc, const void* nrm, int64_t n, int32_t d,
                       const void* Z, int32_t b, void* Out, void* scratch, const TotalsOut& tot,
                       double guard_scale, hipStream_t s)
{
    hipError_t e;
    if (!is_int) {
        // the matrix-core form (it takes its totals itself)
        bool used = false;
        e = launch_l2sq_mfma(zkind, (const float*)Xc, (const double*)nrm, n, d, (const float*)Z, b, (float*)Out,
                             scratch, tot, guard_scale, s, &used);
        if (e != hipSuccess || used) return e;
    }
    // S0 and R (the totals kernel with weights ||x_j||^2)
    e = launch_totals(is_int, zkind, Z, n, b, nrm, guard_scale, tot, s);
    if (e != hipSuccess) return e;
    if (!is_int) {
        // (A z)_i = <x_i, -2 X^T z> + ||x_i||^2 S0 + R: the linear sort-free form
        SfQuery q;
        q.X = Xc;
        q.LX = nullptr;
        q.centre = nullptr;
        q.Z = Z;
        q.n = n;
        q.d = d;
        q.b = b;
        q.T0 = tot.T0;
        q.U = (const double*)tot.U;
        q.a = (const double*)nrm;
        q.W = nullptr;
        q.alpha = -2.0;
        q.Out = Out;
        return launch_sf_query(SF_LIN, 1, false, zkind, q, scratch, s);
    }
    const int nblk = (int)((n + VROWS - 1) / VROWS);
    const int ent = d * b;
    char* base = (char*)scratch;
    void* part = base;
    void* V = base + (size_t)nblk * ent * 8;
    if (is_int) {
        const size_t sm = sizeof(int32_t) * CH * d + (zkind == IN_I32 ? 4 : 8) * CH * b;
        if (zkind == IN_I32)
            xtz_stage1<true, int32_t><<<nblk, 256, sm, s>>>((const int32_t*)Xc, n, d, (const int32_t*)Z, b,
                                                            (int64_t*)part);
        else
            xtz_stage1<true, int64_t><<<nblk, 256, sm, s>>>((const int32_t*)Xc, n, d, (const int64_t*)Z, b,
                                                            (int64_t*)part);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        xtz_stage2<true><<<(ent + 255) / 256, 256, 0, s>>>((const int64_t*)part, nblk, ent, (int64_t*)V);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    } else {
        const size_t sm = sizeof(float) * CH * d + sizeof(float) * CH * b;
        xtz_stage1<false, float><<<nblk, 256, sm, s>>>((const float*)Xc, n, d, (const float*)Z, b, (double*)part);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        xtz_stage2<false><<<(ent + 255) / 256, 256, 0, s>>>((const double*)part, nblk, ent, (double*)V);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    int bpc = 1;
    while (bpc < b && bpc < 256) bpc <<= 1;
    const int rs = 256 / bpc;
    const unsigned grid = (unsigned)((n + rs - 1) / rs);
    if (is_int)
        l2_apply_vec<true><<<grid, 256, 0, s>>>((const int32_t*)Xc, n, d, (const int64_t*)V, b, nrm, tot.T0, tot.U,
                                                Out);
    else
        l2_apply_vec<false><<<grid, 256, 0, s>>>((const float*)Xc, n, d, (const double*)V, b, nrm, tot.T0, tot.U,
                                                 Out);
    return hipGetLastError();
}

}  // namespace dm
