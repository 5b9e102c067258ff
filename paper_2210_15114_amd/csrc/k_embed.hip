// k_embed.hip - the Gaussian embedding that turns the l1 query into an
// approximate l2 query (Appendix A.4: the embedding theorem, the
// preprocessing of Algorithm 10 and the approximate l2 theorem).
//
//   X'[i][t] = (1 / (beta k)) sum_j G[t][j] X[i][j],   beta = sqrt(2/pi),
//
// so that ||X'_i - X'_j||_1 approximates ||x_i - x_j||_2 (the mean of |g.x|
// for a standard Gaussian g is beta ||x||_2).  X' is then prepared and
// queried with the l1 path unchanged.
//
// A tiled product: a workgroup forms 64 rows x 64 columns of X' from LDS
// tiles of X (64 rows) and G (64 rows), 32 coordinates at a time; each
// thread owns 4 x 4 outputs, accumulated in FP64 and rounded once to FP32.
// The work is one-time preparation, bound by writing X' (n k 4 bytes).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "dm_internal.h"

namespace dm {
namespace {

constexpr int ER = 64;   // rows of X' per workgroup
constexpr int EC = 64;   // columns of X' per workgroup
constexpr int EK = 32;   // coordinates per LDS step

template <typename XT>
__global__ __launch_bounds__(256) void embed_kernel(const XT* __restrict__ X, int64_t n, int32_t d,
                                                    const double* __restrict__ G, int32_t k, double scale,
                                                    float* __restrict__ Xout)
{
    __shared__ double sX[ER][EK + 1];
    __shared__ double sG[EC][EK + 1];
    const int tid = threadIdx.x;
    const int64_t r0 = (int64_t)blockIdx.x * ER;
    const int c0 = blockIdx.y * EC;
    const int tr = (tid / 16) * 4, tc = (tid % 16) * 4;   // this thread's 4 x 4 outputs
    double acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
    for (int j0 = 0; j0 < d; j0 += EK) {
        for (int e = tid; e < ER * EK; e += 256) {
            const int r = e / EK, j = e % EK;
            const int64_t row = r0 + r;
            sX[r][j] = (row < n && j0 + j < d) ? (double)X[row * d + j0 + j] : 0.0;
        }
        for (int e = tid; e < EC * EK; e += 256) {
            const int c = e / EK, j = e % EK;
            sG[c][j] = (c0 + c < k && j0 + j < d) ? G[(int64_t)(c0 + c) * d + j0 + j] : 0.0;
        }
        __syncthreads();
#pragma unroll 4
        for (int j = 0; j < EK; ++j) {
            double a[4], g[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                a[i] = sX[tr + i][j];
                g[i] = sG[tc + i][j];
            }
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int t = 0; t < 4; ++t) acc[i][t] = fma(a[i], g[t], acc[i][t]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int64_t row = r0 + tr + i;
        if (row >= n) continue;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int c = c0 + tc + t;
            if (c < k) Xout[row * k + c] = (float)(scale * acc[i][t]);
        }
    }
}

}  // namespace

hipError_t launch_embed_l2(int kind, const void* X, int64_t n, int32_t d, const double* G, int32_t k, float* Xout,
                           hipStream_t s)
{
    if (n < 1 || d < 1 || k < 1) return hipErrorInvalidValue;
    const double beta = std::sqrt(2.0 / M_PI);
    const double scale = 1.0 / (beta * (double)k);
    dim3 grid((unsigned)((n + ER - 1) / ER), (unsigned)((k + EC - 1) / EC));
    switch (kind) {
    case IN_F32: embed_kernel<float><<<grid, 256, 0, s>>>((const float*)X, n, d, G, k, scale, Xout); break;
    case IN_F64: embed_kernel<double><<<grid, 256, 0, s>>>((const double*)X, n, d, G, k, scale, Xout); break;
    case IN_I32: embed_kernel<int32_t><<<grid, 256, 0, s>>>((const int32_t*)X, n, d, G, k, scale, Xout); break;
    case IN_I64: embed_kernel<int64_t><<<grid, 256, 0, s>>>((const int64_t*)X, n, d, G, k, scale, Xout); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace dm
