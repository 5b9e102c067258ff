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
// A tiled product on the FP64 matrix cores (v_mfma_f64_16x16x4f64): a
// workgroup forms 64 rows x 64 columns of X' from LDS tiles of X (64 rows)
// and G (64 rows), 32 coordinates at a time; wave w owns rows 16w .. +15 and
// the four 16-column tiles.  The products are exact FP64 fused operations, the
// sums FP64, rounded once to FP32.  The work is one-time preparation.
//
// Lane layout (checked on the GPU with a probe): A (16 x 4): lane l holds
// A[l % 16][l / 16]; B (4 x 16): lane l holds B[l / 16][l % 16]; D (16 x 16):
// lane l, element r holds D[4r + l / 16][l % 16].
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "dm_internal.h"

namespace dm {
namespace {

constexpr int ER = 64;   // rows of X' per workgroup
constexpr int EC = 64;   // columns of X' per workgroup
constexpr int EK = 32;   // coordinates per LDS step

typedef double d4v __attribute__((ext_vector_type(4)));

template <typename XT>
__global__ __launch_bounds__(256) void embed_kernel(const XT* __restrict__ X, int64_t n, int32_t d,
                                                    const double* __restrict__ G, int32_t k, double scale,
                                                    float* __restrict__ Xout)
{
    __shared__ double sX[ER][EK + 1];
    __shared__ double sG[EC][EK + 1];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int m = lane & 15, g = lane >> 4;
    const int64_t r0 = (int64_t)blockIdx.x * ER;
    const int c0 = blockIdx.y * EC;
    d4v acc[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) acc[u] = d4v{0.0, 0.0, 0.0, 0.0};
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
        // coordinates j0 + 4 kk + g: A[m][g] = X[16w + m][..], B[g][m] = G[16u + m][..]
#pragma unroll
        for (int kk = 0; kk < EK / 4; ++kk) {
            const double a = sX[16 * w + m][4 * kk + g];
#pragma unroll
            for (int u = 0; u < 4; ++u)
                acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, sG[16 * u + m][4 * kk + g], acc[u], 0, 0, 0);
        }
        __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int64_t row = r0 + 16 * w + 4 * r + g;
        if (row >= n) continue;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int c = c0 + 16 * u + m;
            if (c < k) Xout[row * k + c] = (float)(scale * acc[u][r]);
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
