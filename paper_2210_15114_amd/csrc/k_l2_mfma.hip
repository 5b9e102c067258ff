// k_l2_mfma.hip - matrix-core path of the l2-squared query (Algorithm 3):
//     V = X^T Z            (d x b, split over the points, FP64 partials)
//     Out = ||x_i||^2 S0 + R - 2 X V
// Both contractions run on gfx950 BF16 matrix cores with each FP32 operand
// split into a BF16 high part and a BF16 remainder, x = xh + xl; products
// use xh*yh + xh*yl + xl*yh, which keeps each term to about 2^-16 relative
// (the dropped xl*yl and the remainders of the splits are of that order).
// Accumulation is FP32 inside the matrix cores, flushed into FP64 every 256
// points in the first contraction; the rank-one terms and the final
// combination are FP64.  The three products of a split go to three
// independent accumulators (hh, hl, lh), added only when they leave the
// matrix cores: a chain of dependent matrix-core products waits out the full
// latency of each one, which made both kernels latency-bound (about half the
// achievable bandwidth) when the three shared one accumulator.
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
// consecutive floats of one row, so every load is coalesced), and the next
// step's operands are loaded before the current step's products.
// FAST: d = 128 and b = 64 (every wave one k-tile, both c-tiles, no checks)
// for the whole steps of a workgroup; the general form checks every access.
// ---------------------------------------------------------------------------
template <bool FAST>
__global__ __launch_bounds__(256) void xtz_mfma_kernel(const float* __restrict__ X, int64_t n, int32_t d,
                                                       const float* __restrict__ Z, int32_t b,
                                                       double* __restrict__ part)
{
    __shared__ double s_red[4][2][16][64];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int kt_n = FAST ? 4 : (d + 31) / 32, ct_n = FAST ? 2 : (b + 31) / 32;
    const int rsplit = kt_n >= 4 ? 1 : 4 / kt_n;
    const int kt = w % kt_n, rs = w / kt_n;
    const bool active = rs < rsplit;
    const int kcol = kt * 32 + lane % 32, jg = lane / 32;
    // FP32 accumulators per c-tile: the main product (hh) and the two
    // remainder products (hl, lh; 2^-8 of it), two independent chains; their
    // FP64 sums live in LDS (s_red, one slot per wave), which keeps the
    // registers of two waves per SIMD
    f32x16 acc[2][2] = {};
#pragma unroll
    for (int ct = 0; ct < 2; ++ct)
#pragma unroll
        for (int r = 0; r < 16; ++r) s_red[w][ct][r][lane] = 0.0;
    const int64_t j0 = (int64_t)blockIdx.x * ROWS_PER_WG;
    const int64_t j1 = min(n, j0 + ROWS_PER_WG);
    auto load = [&](int64_t j, float (&xv)[8], float (&zv)[2][8]) {
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const int64_t row = j + 8 * jg + t;
            if (FAST) {   // d = 128, b = 64 as constants: one base address, immediate offsets
                xv[t] = X[row * MAXD + kcol];
#pragma unroll
                for (int ct = 0; ct < 2; ++ct) zv[ct][t] = Z[row * MAXB + ct * 32 + lane % 32];
            } else {
                const bool ok = row < j1;
                xv[t] = (ok && kcol < d) ? X[row * d + kcol] : 0.0f;
#pragma unroll
                for (int ct = 0; ct < 2; ++ct) {
                    const int c = ct * 32 + lane % 32;
                    zv[ct][t] = (ok && ct < ct_n && c < b) ? Z[row * b + c] : 0.0f;
                }
            }
        }
    };
    int since = 0;
    auto products = [&](const float (&xv)[8], const float (&zv)[2][8]) {
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
            if (FAST || ct < ct_n) {
                bf16x8 bh, bl;
#pragma unroll
                for (int t = 0; t < 8; ++t) {
                    __bf16 h, l;
                    split(zv[ct][t], h, l);
                    bh[t] = h;
                    bl[t] = l;
                }
                acc[ct][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh, acc[ct][0], 0, 0, 0);
                acc[ct][1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl, acc[ct][1], 0, 0, 0);
                acc[ct][1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh, acc[ct][1], 0, 0, 0);
            }
        }
        // flush the FP32 accumulators into FP64 every 16 steps (256 points)
        if (++since == 16) {
            since = 0;
#pragma unroll
            for (int ct = 0; ct < 2; ++ct)
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    s_red[w][ct][r][lane] += (double)(acc[ct][1][r] + acc[ct][0][r]);
                    acc[ct][0][r] = acc[ct][1][r] = 0.0f;
                }
        }
    };
    if (active) {
        // two steps in flight: the operands of steps j + step and j + 2 step
        // are loaded before the products of step j
        const int64_t step = 16 * rsplit;
        int64_t j = j0 + 16 * rs;
        float xa[8], za[2][8], xb[8], zb[2][8];
        if (j < j1) load(j, xa, za);
        if (j + step < j1) load(j + step, xb, zb);
        for (; j < j1; j += 2 * step) {
            float xc[8], zc[2][8], xd[8], zd[2][8];
            if (j + 2 * step < j1) load(j + 2 * step, xc, zc);
            products(xa, za);
            if (j + step >= j1) break;
            if (j + 3 * step < j1) load(j + 3 * step, xd, zd);
            products(xb, zb);
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                xa[t] = xc[t];
                za[0][t] = zc[0][t];
                za[1][t] = zc[1][t];
                xb[t] = xd[t];
                zb[0][t] = zd[0][t];
                zb[1][t] = zd[1][t];
            }
        }
    }
#pragma unroll
    for (int ct = 0; ct < 2; ++ct)
#pragma unroll
        for (int r = 0; r < 16; ++r) s_red[w][ct][r][lane] += (double)(acc[ct][1][r] + acc[ct][0][r]);
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
// columns per block: the lane's whole row segment (every k-step) is loaded
// before the products; V is split into BF16 hi/lo once per workgroup in LDS.
// CHECK = false: the branch-free kernel for whole blocks of 32 rows with
// d = 16 KS, b = 32 CT and 16-byte rows; CHECK = true checks every access
// (other shapes, and the last partial block of the branch-free shapes, which
// a second launch handles).
// ---------------------------------------------------------------------------
template <int KS, int CT, bool CHECK>
__device__ __forceinline__ void l2_apply_block(const float* __restrict__ X, int64_t n, int32_t d, int32_t b,
                                               const __bf16 (*sVh)[MAXD + 8], const __bf16 (*sVl)[MAXD + 8],
                                               const double* __restrict__ nrm, const double* __restrict__ S0,
                                               const double* __restrict__ R, float* __restrict__ Out, int64_t i0,
                                               int lane)
{
    const int64_t ir = i0 + lane % 32;       // the A row this lane loads
    float xv[KS][8];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
        const int kb = ks * 16 + 8 * (lane / 32);
        if (!CHECK) {
            const float4 a = *reinterpret_cast<const float4*>(X + ir * d + kb);
            const float4 c = *reinterpret_cast<const float4*>(X + ir * d + kb + 4);
            xv[ks][0] = a.x; xv[ks][1] = a.y; xv[ks][2] = a.z; xv[ks][3] = a.w;
            xv[ks][4] = c.x; xv[ks][5] = c.y; xv[ks][6] = c.z; xv[ks][7] = c.w;
        } else {
#pragma unroll
            for (int t = 0; t < 8; ++t) xv[ks][t] = (ir < n && kb + t < d) ? X[ir * d + kb + t] : 0.0f;
        }
    }
    f32x16 acc[CT][3] = {};
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
        const int kb = ks * 16 + 8 * (lane / 32);
        bf16x8 ah, al;
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            __bf16 h, l;
            split(xv[ks][t], h, l);
            ah[t] = h;
            al[t] = l;
        }
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) {
            const bf16x8 bh = *reinterpret_cast<const bf16x8*>(&sVh[ct * 32 + lane % 32][kb]);
            const bf16x8 bl = *reinterpret_cast<const bf16x8*>(&sVl[ct * 32 + lane % 32][kb]);
            acc[ct][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh, acc[ct][0], 0, 0, 0);
            acc[ct][1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl, acc[ct][1], 0, 0, 0);
            acc[ct][2] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh, acc[ct][2], 0, 0, 0);
        }
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int64_t i = i0 + (r / 4) * 8 + (lane / 32) * 4 + (r % 4);
        if (CHECK && i >= n) continue;
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) {
            const int c = ct * 32 + lane % 32;
            // the two remainder products are 2^-8 of the main one: their sum
            // in FP32 adds an error below that of the split itself
            const float p = (acc[ct][1][r] + acc[ct][2][r]) + acc[ct][0][r];
            if (!CHECK || c < b) Out[i * b + c] = (float)(nrm[i] * S0[c] + R[c] - 2.0 * (double)p);
        }
    }
}

template <int KS, int CT, bool CHECK>
__global__ __launch_bounds__(256) void l2_apply_mfma_kernel(const float* __restrict__ X, int64_t n, int32_t d,
                                                            const double* __restrict__ V, int32_t b,
                                                            const double* __restrict__ nrm,
                                                            const double* __restrict__ S0,
                                                            const double* __restrict__ R,
                                                            float* __restrict__ Out, int64_t blk0, int64_t nblk)
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
    for (int64_t blk = blk0 + (int64_t)blockIdx.x * 4 + w; blk < nblk; blk += (int64_t)gridDim.x * 4)
        l2_apply_block<KS, CT, CHECK>(X, n, d, b, sVh, sVl, nrm, S0, R, Out, blk * 32, lane);
}

template <int KS, int CT>
static void launch_apply_ct(bool vec, unsigned grid, hipStream_t s, const float* X, int64_t n, int32_t d,
                            const double* V, int32_t b, const double* nrm, const double* S0, const double* R,
                            float* Out)
{
    const int64_t nblk = (n + 31) / 32;
    if (vec && d == KS * 16 && b == CT * 32) {
        // whole blocks branch-free, then the last partial block (if any)
        const int64_t full = n / 32;
        if (full > 0)
            l2_apply_mfma_kernel<KS, CT, false><<<grid, 256, 0, s>>>(X, n, d, V, b, nrm, S0, R, Out, 0, full);
        if (full < nblk)
            l2_apply_mfma_kernel<KS, CT, true><<<1, 256, 0, s>>>(X, n, d, V, b, nrm, S0, R, Out, full, nblk);
    } else {
        l2_apply_mfma_kernel<KS, CT, true><<<grid, 256, 0, s>>>(X, n, d, V, b, nrm, S0, R, Out, 0, nblk);
    }
}

template <int KS>
static void launch_apply(bool vec, unsigned grid, hipStream_t s, const float* X, int64_t n, int32_t d,
                         const double* V, int32_t b, const double* nrm, const double* S0, const double* R, float* Out)
{
    if (b <= 32) launch_apply_ct<KS, 1>(vec, grid, s, X, n, d, V, b, nrm, S0, R, Out);
    else launch_apply_ct<KS, 2>(vec, grid, s, X, n, d, V, b, nrm, S0, R, Out);
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
    // the branch-free form needs d = 128, b = 64 and whole workgroup ranges
    // (the last range is whole when n is a multiple of the range)
    if (d == MAXD && b == MAXB && n % ROWS_PER_WG == 0)
        xtz_mfma_kernel<true><<<nblk, 256, 0, s>>>(Xc, n, d, Z, b, part);
    else
        xtz_mfma_kernel<false><<<nblk, 256, 0, s>>>(Xc, n, d, Z, b, part);
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
