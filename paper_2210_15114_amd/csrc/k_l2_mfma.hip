// k_l2_mfma.hip - matrix-core path of the l2-squared query (Algorithm 3):
//     V = X^T Z            (d x b, split over the points, FP64 partials)
//     Out = ||x_i||^2 S0 + R - 2 X V
// Both contractions run on gfx950 BF16 matrix cores with each FP32 operand
// split into a BF16 high part and a BF16 remainder, x = xh + xl; products
// use xh*yh + xh*yl + xl*yh, which keeps each term to about 2^-16 relative
// (the dropped xl*yl and the remainders of the splits are of that order).
// Accumulation is FP32 inside the matrix cores, flushed into FP64 every 256
// points in the first contraction; the rank-one terms and the final
// combination are FP64.
//
// Shapes: d <= 128 and b >= 16 (other shapes take the vector path).
//
// MFMA v_mfma_f32_32x32x16_bf16 lane layout (wave of 64):
//   A (32 x 16): lane l holds row l%32, k = 8*(l/32) .. +7
//   B (16 x 32): lane l holds column l%32, k = 8*(l/32) .. +7
//   D (32 x 32): acc[r] is row (r/4)*8 + (l/32)*4 + r%4, column l%32
#include "dm_device.h"
#include "dm_internal.h"

namespace dm {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int MAXD = 128;
constexpr int MAXB = 64;
constexpr int ROWS_PER_WG = 4096;

__device__ __forceinline__ void split(float x, __bf16& h, __bf16& l) {
    h = (__bf16)x;
    l = (__bf16)(x - (float)h);
}

// ---------------------------------------------------------------------------
// V partials: workgroup g sums points [g*ROWS_PER_WG, ...) into its own d x b
// FP64 partial.  Wave w owns k-tile (w % kt_n) for every c-tile and takes the
// 16-point steps s with s % rsplit == w / kt_n; operands are loaded straight
// into MFMA lane order (for a fixed t the 32 lanes of a half-wave read 32
// consecutive floats of one row, so every load is coalesced).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void xtz_mfma_kernel(const float* __restrict__ X, int64_t n, int32_t d,
                                                       const float* __restrict__ Z, int32_t b,
                                                       double* __restrict__ part)
{
    __shared__ double s_red[4][2][16][64];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int kt_n = (d + 31) / 32, ct_n = (b + 31) / 32;
    const int rsplit = kt_n >= 4 ? 1 : 4 / kt_n;
    const int kt = w % kt_n, rs = w / kt_n;
    const bool active = rs < rsplit;
    const int kcol = kt * 32 + lane % 32, jg = lane / 32;
    f32x16 acc[2] = {{}, {}};
    double dacc[2][16];
#pragma unroll
    for (int ct = 0; ct < 2; ++ct)
#pragma unroll
        for (int r = 0; r < 16; ++r) dacc[ct][r] = 0.0;
    const int64_t j0 = (int64_t)blockIdx.x * ROWS_PER_WG;
    const int64_t j1 = min(n, j0 + ROWS_PER_WG);
    int since = 0;
    if (active) {
        for (int64_t j = j0 + 16 * rs; j < j1; j += 16 * rsplit) {
            float xv[8], zv[2][8];
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                const int64_t row = j + 8 * jg + t;
                const bool ok = row < j1;
                xv[t] = (ok && kcol < d) ? X[row * d + kcol] : 0.0f;
#pragma unroll
                for (int ct = 0; ct < 2; ++ct) {
                    const int c = ct * 32 + lane % 32;
                    zv[ct][t] = (ok && ct < ct_n && c < b) ? Z[row * b + c] : 0.0f;
                }
            }
            bf16x8 ah, al;
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                __bf16 h, l;
                split(xv[t], h, l);
                ah[t] = h;
                al[t] = l;
            }
#pragma unroll
            for (int ct = 0; ct < 2; ++ct) {
                if (ct < ct_n) {
                    bf16x8 bh, bl;
#pragma unroll
                    for (int t = 0; t < 8; ++t) {
                        __bf16 h, l;
                        split(zv[ct][t], h, l);
                        bh[t] = h;
                        bl[t] = l;
                    }
                    acc[ct] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh, acc[ct], 0, 0, 0);
                    acc[ct] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl, acc[ct], 0, 0, 0);
                    acc[ct] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh, acc[ct], 0, 0, 0);
                }
            }
            // flush the FP32 accumulators into FP64 every 16 steps (256 points)
            if (++since == 16) {
                since = 0;
#pragma unroll
                for (int ct = 0; ct < 2; ++ct)
#pragma unroll
                    for (int r = 0; r < 16; ++r) {
                        dacc[ct][r] += (double)acc[ct][r];
                        acc[ct][r] = 0.0f;
                    }
            }
        }
    }
#pragma unroll
    for (int ct = 0; ct < 2; ++ct)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            dacc[ct][r] += (double)acc[ct][r];
            s_red[w][ct][r][lane] = dacc[ct][r];
        }
    __syncthreads();
    // waves that share a k-tile add their partials in wave order; the first writes
    if (active && rs == 0) {
        double* pb = part + (size_t)blockIdx.x * d * b;
#pragma unroll
        for (int ct = 0; ct < 2; ++ct) {
            if (ct >= ct_n) continue;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                double v = 0.0;
                for (int q = 0; q < rsplit; ++q) v += s_red[kt + q * kt_n][ct][r][lane];
                const int k = kt * 32 + (r / 4) * 8 + (lane / 32) * 4 + (r % 4);
                const int c = ct * 32 + lane % 32;
                if (k < d && c < b) pb[(size_t)k * b + c] = v;
            }
        }
    }
}

// fixed-order sum of the partials: V[e] = sum_g part[g][e].  A block takes 32
// consecutive entries; its 8 row groups each sum the partials g = q, q + 8, ...
// in ascending order (32 lanes read 256 contiguous bytes per load), and the 8
// group sums are added in group order.
__global__ __launch_bounds__(256) void xtz_reduce_kernel(const double* __restrict__ part, int nblk, int ent,
                                                         double* __restrict__ V)
{
    __shared__ double s[8][32];
    const int el = threadIdx.x % 32, q = threadIdx.x / 32;
    const int e = blockIdx.x * 32 + el;
    double acc = 0.0;
    if (e < ent) {
#pragma unroll 8
        for (int g = q; g < nblk; g += 8) acc += part[(size_t)g * ent + e];
    }
    s[q][el] = acc;
    __syncthreads();
    if (q == 0 && e < ent) {
        double v = 0.0;
#pragma unroll
        for (int r = 0; r < 8; ++r) v += s[r][el];
        V[e] = v;
    }
}

// ---------------------------------------------------------------------------
// Out = nrm_i S0_c + R_c - 2 (X V)_ic; each wave computes 32 rows x all b
// columns per step, with the next k-step's X values in flight during the
// current step's products; V is split into BF16 hi/lo once per workgroup in
// LDS.
// ---------------------------------------------------------------------------
template <int KS, bool VEC>
__global__ __launch_bounds__(256) void l2_apply_mfma_kernel(const float* __restrict__ X, int64_t n, int32_t d,
                                                            const double* __restrict__ V, int32_t b,
                                                            const double* __restrict__ nrm,
                                                            const double* __restrict__ S0,
                                                            const double* __restrict__ R,
                                                            float* __restrict__ Out)
{
    __shared__ __bf16 sVh[MAXB][MAXD + 8], sVl[MAXB][MAXD + 8];   // [c][k]
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    for (int e = tid; e < MAXB * MAXD; e += 256) {
        const int c = e / MAXD, k = e % MAXD;
        const float v = (c < b && k < d) ? (float)V[(size_t)k * b + c] : 0.0f;
        __bf16 h, l;
        split(v, h, l);
        sVh[c][k] = h;
        sVl[c][k] = l;
    }
    __syncthreads();
    const int ct_n = (b + 31) / 32;    // 1 or 2
    const int64_t nblk = (n + 31) / 32;
    double s0[2], rr[2];
#pragma unroll
    for (int ct = 0; ct < 2; ++ct) {
        const int c = ct * 32 + lane % 32;
        s0[ct] = (ct < ct_n && c < b) ? S0[c] : 0.0;
        rr[ct] = (ct < ct_n && c < b) ? R[c] : 0.0;
    }
    // X of one k-step (8 values of the lane's A row); the next step's values
    // are loaded before this step's products
    auto load_step = [&](int64_t ir, int ks, float (&xv)[8]) {
        const int kb = ks * 16 + 8 * (lane / 32);
        if (VEC) {
            if (ir < n && kb < d) {
                const float4 a = *reinterpret_cast<const float4*>(X + ir * d + kb);
                const float4 c = *reinterpret_cast<const float4*>(X + ir * d + kb + 4);
                xv[0] = a.x; xv[1] = a.y; xv[2] = a.z; xv[3] = a.w;
                xv[4] = c.x; xv[5] = c.y; xv[6] = c.z; xv[7] = c.w;
            } else {
#pragma unroll
                for (int t = 0; t < 8; ++t) xv[t] = 0.0f;
            }
        } else {
#pragma unroll
            for (int t = 0; t < 8; ++t) xv[t] = (ir < n && kb + t < d) ? X[ir * d + kb + t] : 0.0f;
        }
    };
    for (int64_t blk = (int64_t)blockIdx.x * 4 + w; blk < nblk; blk += (int64_t)gridDim.x * 4) {
        const int64_t i0 = blk * 32;
        const int64_t ir = i0 + lane % 32;       // the A row this lane loads
        float xn[8];
        load_step(ir, 0, xn);
        f32x16 acc0 = {}, acc1 = {};
#pragma unroll 1
        for (int ks = 0; ks < KS; ++ks) {
            const int kb = ks * 16 + 8 * (lane / 32);
            float xv[8];
#pragma unroll
            for (int t = 0; t < 8; ++t) xv[t] = xn[t];
            if (ks + 1 < KS) load_step(ir, ks + 1, xn);
            bf16x8 ah, al;
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                __bf16 h, l;
                split(xv[t], h, l);
                ah[t] = h;
                al[t] = l;
            }
            {
                const bf16x8 bh = *reinterpret_cast<const bf16x8*>(&sVh[lane % 32][kb]);
                const bf16x8 bl = *reinterpret_cast<const bf16x8*>(&sVl[lane % 32][kb]);
                acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh, acc0, 0, 0, 0);
                acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl, acc0, 0, 0, 0);
                acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh, acc0, 0, 0, 0);
            }
            if (ct_n > 1) {
                const bf16x8 bh = *reinterpret_cast<const bf16x8*>(&sVh[32 + lane % 32][kb]);
                const bf16x8 bl = *reinterpret_cast<const bf16x8*>(&sVl[32 + lane % 32][kb]);
                acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh, acc1, 0, 0, 0);
                acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl, acc1, 0, 0, 0);
                acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh, acc1, 0, 0, 0);
            }
        }
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int64_t i = i0 + (r / 4) * 8 + (lane / 32) * 4 + (r % 4);
            if (i >= n) continue;
            const double ni = nrm[i];
            const int c0 = lane % 32;
            if (c0 < b) Out[i * b + c0] = (float)(ni * s0[0] + rr[0] - 2.0 * (double)acc0[r]);
            if (ct_n > 1 && 32 + c0 < b) Out[i * b + 32 + c0] = (float)(ni * s0[1] + rr[1] - 2.0 * (double)acc1[r]);
        }
    }
}

template <int KS>
static void launch_apply(bool vec, unsigned grid, hipStream_t s, const float* X, int64_t n, int32_t d,
                         const double* V, int32_t b, const double* nrm, const double* S0, const double* R, float* Out)
{
    if (vec)
        l2_apply_mfma_kernel<KS, true><<<grid, 256, 0, s>>>(X, n, d, V, b, nrm, S0, R, Out);
    else
        l2_apply_mfma_kernel<KS, false><<<grid, 256, 0, s>>>(X, n, d, V, b, nrm, S0, R, Out);
}

}  // namespace

size_t l2_mfma_partials(int64_t n) { return (size_t)((n + ROWS_PER_WG - 1) / ROWS_PER_WG); }

hipError_t launch_l2sq_mfma(const float* Xc, const double* nrm, int64_t n, int32_t d, const float* Z, int32_t b,
                            float* Out, void* scratch, const TotalsOut& tot, hipStream_t s, bool* used)
{
    *used = false;
    if (d > MAXD || b < 16 || b > MAXB) return hipSuccess;
    const int nblk = (int)l2_mfma_partials(n);
    const int ent = d * b;
    double* part = (double*)scratch;
    double* V = part + (size_t)nblk * ent;
    xtz_mfma_kernel<<<nblk, 256, 0, s>>>(Xc, n, d, Z, b, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    xtz_reduce_kernel<<<(ent + 31) / 32, 256, 0, s>>>(part, nblk, ent, V);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const int64_t blocks = (n + 127) / 128;
    const unsigned grid = (unsigned)(blocks < 256 * 8 ? blocks : 256 * 8);
    const bool vec = (d % 8 == 0) && ((uintptr_t)Xc % 16 == 0);
    const int ks = (d + 15) / 16;
    const double* S0 = (const double*)tot.T0;
    const double* Rr = (const double*)tot.U;
    if (ks <= 1) launch_apply<1>(vec, grid, s, Xc, n, d, V, b, nrm, S0, Rr, Out);
    else if (ks <= 2) launch_apply<2>(vec, grid, s, Xc, n, d, V, b, nrm, S0, Rr, Out);
    else if (ks <= 4) launch_apply<4>(vec, grid, s, Xc, n, d, V, b, nrm, S0, Rr, Out);
    else launch_apply<8>(vec, grid, s, Xc, n, d, V, b, nrm, S0, Rr, Out);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    *used = true;
    return hipSuccess;
}

}  // namespace dm
