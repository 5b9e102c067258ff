// k_l2_mfma.hip - matrix-core path of the l2-squared query (Algorithm 3):
//     V = X^T Z            (d x b, split over the points, FP64 partials)
//     Out = ||x_i||^2 S0 + R - 2 X V
// Both contractions run on gfx950 BF16 matrix cores with each FP32 operand
// split into a BF16 high part and a BF16 remainder, x = xh + xl; products
// use xh*yh + xh*yl + xl*yh, which keeps each term to about 2^-16 relative
// (the dropped xl*yl and the remainders of the splits are of that order).
// Accumulation is FP32 inside the matrix cores, flushed every 256 points in
// the first contraction (into FP32 sums of at most four flushes, then FP64,
// or straight into FP64 for the general shapes); the rank-one terms and the
// final combination are FP64.  No matrix-core product waits on the one
// before it: the split products go to separate accumulators or are
// interleaved with other tiles' products, since a chain of dependent
// products waits out the full latency of each one (with one accumulator per
// tile both kernels ran at about half the achievable bandwidth).
//
// For d = 128, b = 64 and whole ranges of points the first kernel also forms
// the rank-one totals S0 = sum_j z_j and R = sum_j ||x_j||^2 z_j (FP64) from
// its own loads of Z, so a query reads Z once.
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
// V partials (general shapes): workgroup g sums points [g*ROWS_PER_WG, ...)
// into its own d x b FP64 partial.  Wave w owns k-tile (w % kt_n) for every
// c-tile and takes the 16-point steps s with s % rsplit == w / kt_n; operands
// are loaded straight into MFMA lane order (for a fixed t the 32 lanes of a
// half-wave read 32 consecutive floats of one row, so every load is
// coalesced), two steps ahead of the products, and every access is checked.
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
    // FP32 accumulators per c-tile: the main product (hh) and the two
    // remainder products (hl, lh; 2^-8 of it), two independent chains; their
    // FP64 sums live in LDS (s_red, one slot per wave)
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
            const bool ok = row < j1;
            xv[t] = (ok && kcol < d) ? X[row * d + kcol] : 0.0f;
#pragma unroll
            for (int ct = 0; ct < 2; ++ct) {
                const int c = ct * 32 + lane % 32;
                zv[ct][t] = (ok && ct < ct_n && c < b) ? Z[row * b + c] : 0.0f;
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
            if (ct < ct_n) {
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

// ---------------------------------------------------------------------------
// V partials and the totals for d = 128, b = 64 and whole ranges of points.
// Every wave covers all four k-tiles and both c-tiles (eight independent
// accumulator chains) for the 16-point steps s with s % 4 == w, so each row
// of X and of Z is read once per query.  The FP32 accumulators are flushed
// every 16 steps (256 points) into FP32 sums in LDS: a wave has four flushes
// per range, whose three additions round far below the split products.  The
// four waves' sums are added in FP64 in wave order.  The same loads feed S0
// and R in FP64; the lanes l and l + 32 hold alternate groups of 8 points of
// one column.  Partial layout per workgroup: V (d x b), then S0 (b), R (b).
// ---------------------------------------------------------------------------
constexpr int WIDE_ENT = MAXD * MAXB + 2 * MAXB;

__global__ __launch_bounds__(256) void xtz_wide_kernel(const float* __restrict__ X, const float* __restrict__ Z,
                                                       const double* __restrict__ nrm, double* __restrict__ part)
{
    constexpr int NT = 8;                          // tiles: kt * 2 + ct
    __shared__ float s_sum[4][NT][16][64];         // per wave, FP32 sums of the flushes
    __shared__ double s_tot[4][2][2][64];          // per wave: S0 | R, lane half, column
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int jg = lane >> 5, l32 = lane & 31;
    f32x16 acc[NT] = {};
#pragma unroll
    for (int q = 0; q < NT; ++q)
#pragma unroll
        for (int r = 0; r < 16; ++r) s_sum[w][q][r][lane] = 0.0f;
    double s0[2] = {0.0, 0.0}, r1[2] = {0.0, 0.0};
    // X and Z are streamed once per query here: non-temporal loads (the
    // apply reads X again, but 4nd bytes do not stay cached between the two)
    auto load = [&](int64_t j, float (&xv)[4][8], float (&zv)[2][8], double (&nv)[8]) {
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const int64_t row = j + 8 * jg + t;
#pragma unroll
            for (int kt = 0; kt < 4; ++kt) xv[kt][t] = __builtin_nontemporal_load(&X[row * MAXD + kt * 32 + l32]);
#pragma unroll
            for (int ct = 0; ct < 2; ++ct) zv[ct][t] = __builtin_nontemporal_load(&Z[row * MAXB + ct * 32 + l32]);
            nv[t] = nrm[row];
        }
    };
    auto products = [&](const float (&xv)[4][8], const float (&zv)[2][8], const double (&nv)[8]) {
        bf16x8 ah[4], al[4], bh[2], bl[2];
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            __bf16 h, l;
#pragma unroll
            for (int kt = 0; kt < 4; ++kt) {
                split(xv[kt][t], h, l);
                ah[kt][t] = h;
                al[kt][t] = l;
            }
#pragma unroll
            for (int ct = 0; ct < 2; ++ct) {
                split(zv[ct][t], h, l);
                bh[ct][t] = h;
                bl[ct][t] = l;
            }
        }
        // hh of all eight tiles, then hl, then lh: a tile's next product
        // waits behind seven others
#pragma unroll
        for (int kt = 0; kt < 4; ++kt)
#pragma unroll
            for (int ct = 0; ct < 2; ++ct)
                acc[kt * 2 + ct] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[kt], bh[ct], acc[kt * 2 + ct], 0, 0, 0);
#pragma unroll
        for (int kt = 0; kt < 4; ++kt)
#pragma unroll
            for (int ct = 0; ct < 2; ++ct)
                acc[kt * 2 + ct] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[kt], bl[ct], acc[kt * 2 + ct], 0, 0, 0);
#pragma unroll
        for (int kt = 0; kt < 4; ++kt)
#pragma unroll
            for (int ct = 0; ct < 2; ++ct)
                acc[kt * 2 + ct] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[kt], bh[ct], acc[kt * 2 + ct], 0, 0, 0);
#pragma unroll
        for (int ct = 0; ct < 2; ++ct)
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                s0[ct] += (double)zv[ct][t];
                r1[ct] = fma(nv[t], (double)zv[ct][t], r1[ct]);
            }
    };
    // 4 x 16 steps of 16 points per wave, a flush after every 16; the next
    // step's operands are loaded before the current step's products
    const int64_t jw = (int64_t)blockIdx.x * ROWS_PER_WG + 16 * w;
    float xa[4][8], za[2][8];
    double na[8];
    load(jw, xa, za, na);
    for (int f = 0; f < 4; ++f) {
        for (int u = 0; u < 16; ++u) {
            const int st = f * 16 + u;
            float xb[4][8], zb[2][8];
            double nb[8];
            if (st < 63) load(jw + (int64_t)(st + 1) * 64, xb, zb, nb);
            products(xa, za, na);
#pragma unroll
            for (int t = 0; t < 8; ++t) {
#pragma unroll
                for (int kt = 0; kt < 4; ++kt) xa[kt][t] = xb[kt][t];
                za[0][t] = zb[0][t];
                za[1][t] = zb[1][t];
                na[t] = nb[t];
            }
        }
#pragma unroll
        for (int q = 0; q < NT; ++q)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                s_sum[w][q][r][lane] += acc[q][r];
                acc[q][r] = 0.0f;
            }
    }
#pragma unroll
    for (int ct = 0; ct < 2; ++ct) {
        s_tot[w][0][jg][ct * 32 + l32] = s0[ct];
        s_tot[w][1][jg][ct * 32 + l32] = r1[ct];
    }
    __syncthreads();
    double* pb = part + (size_t)blockIdx.x * WIDE_ENT;
    // wave w writes k-tile w: the four waves' sums in wave order
#pragma unroll
    for (int ct = 0; ct < 2; ++ct)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            double v = 0.0;
#pragma unroll
            for (int q = 0; q < 4; ++q) v += (double)s_sum[q][w * 2 + ct][r][lane];
            const int k = w * 32 + (r / 4) * 8 + jg * 4 + (r % 4);
            pb[(size_t)k * MAXB + ct * 32 + l32] = v;
        }
    if (tid < 2 * MAXB) {
        const int q = tid / MAXB, c = tid % MAXB;
        double v = 0.0;
#pragma unroll
        for (int u = 0; u < 4; ++u) v += s_tot[u][q][0][c] + s_tot[u][q][1][c];
        pb[MAXD * MAXB + tid] = v;
    }
}

// fixed-order sum of the partials: V[e] = sum_g part[g][e].  A block takes 32
// consecutive entries; its 8 row groups each sum the partials g = q, q + 8, ...
// in ascending order (32 lanes read 256 contiguous bytes per load), and the 8
// group sums are added in group order.
// Entries [chk0, chk1) are sums of Z (S0): a non-finite one means a
// non-finite z, which raises the status flag.
__global__ __launch_bounds__(256) void xtz_reduce_kernel(const double* __restrict__ part, int nblk, int ent,
                                                         double* __restrict__ V, int chk0, int chk1,
                                                         uint32_t* __restrict__ status)
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
        if (e >= chk0 && e < chk1 && !isfinite(v)) atomicOr(status, (uint32_t)QF_NONFINITE);
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
            // in FP32 adds an error below that of the split itself; Out is
            // written once and not read here, so its stores bypass the caches'
            // retention (the next query's X^T Z then finds no dirty lines)
            const float p = (acc[ct][1][r] + acc[ct][2][r]) + acc[ct][0][r];
            if (!CHECK || c < b)
                __builtin_nontemporal_store((float)(nrm[i] * S0[c] + R[c] - 2.0 * (double)p), &Out[i * b + c]);
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

size_t l2_mfma_scratch_bytes(int64_t n, int32_t d, int32_t b) {
    return (l2_mfma_partials(n) + 1) * ((size_t)d * b + 2 * (size_t)b) * 8 + 256;
}

hipError_t launch_l2sq_mfma(int zkind, const float* Xc, const double* nrm, int64_t n, int32_t d, const float* Z,
                            int32_t b, float* Out, void* scratch, const TotalsOut& tot, double guard_scale,
                            hipStream_t s, bool* used)
{
    *used = false;
    if (n < 1 || d > MAXD || b < 16 || b > MAXB) return hipSuccess;
    const int nblk = (int)l2_mfma_partials(n);
    // d = 128, b = 64 and whole ranges of points: the totals come with X^T Z
    const bool wide = d == MAXD && b == MAXB && n % ROWS_PER_WG == 0;
    const int ent = wide ? WIDE_ENT : d * b;
    double* part = (double*)scratch;
    double* V = part + (size_t)nblk * ent;
    const double* S0;
    const double* Rr;
    hipError_t e;
    if (wide) {
        xtz_wide_kernel<<<nblk, 256, 0, s>>>(Xc, Z, nrm, part);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        xtz_reduce_kernel<<<(ent + 31) / 32, 256, 0, s>>>(part, nblk, ent, V, d * b, d * b + b, tot.status);
        S0 = V + (size_t)d * b;
        Rr = V + (size_t)d * b + b;
    } else {
        // S0 and R from the totals kernel (weights ||x_j||^2)
        if ((e = launch_totals(false, zkind, Z, n, b, nrm, guard_scale, tot, s)) != hipSuccess) return e;
        xtz_mfma_kernel<<<nblk, 256, 0, s>>>(Xc, n, d, Z, b, part);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        xtz_reduce_kernel<<<(ent + 31) / 32, 256, 0, s>>>(part, nblk, ent, V, 0, 0, tot.status);
        S0 = (const double*)tot.T0;
        Rr = (const double*)tot.U;
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // six workgroups of four waves per compute unit (measured best of 4, 6, 8)
    const int64_t blocks = (n + 127) / 128;
    const unsigned grid = (unsigned)(blocks < 256 * 6 ? blocks : 256 * 6);
    const bool vec = (d % 8 == 0) && ((uintptr_t)Xc % 16 == 0);
    const int ks = (d + 15) / 16;
    if (ks <= 1) launch_apply<1>(vec, grid, s, Xc, n, d, V, b, nrm, S0, Rr, Out);
    else if (ks <= 2) launch_apply<2>(vec, grid, s, Xc, n, d, V, b, nrm, S0, Rr, Out);
    else if (ks <= 4) launch_apply<4>(vec, grid, s, Xc, n, d, V, b, nrm, S0, Rr, Out);
    else launch_apply<8>(vec, grid, s, Xc, n, d, V, b, nrm, S0, Rr, Out);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    *used = true;
    return hipSuccess;
}

}  // namespace dm
