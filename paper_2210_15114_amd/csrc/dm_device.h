// dm_device.h - device-side helpers shared by the gfx950 kernels.
//
// * order-preserving 32-bit keys for the per-coordinate radix sort
//   (Algorithm 1 sorts each coordinate; ties keep ascending point order);
// * double-float ("hi + lo" FP32 pair) arithmetic for the compensated prefix
//   sums of the l1 query (Algorithm 2's partial sums B_i and C_i, carried
//   across tiles without accumulating FP32 rounding);
// * tagged 64-bit words used to publish tile aggregates between workgroups
//   without fences: each word holds 32 payload bits and the 32-bit tag of the
//   pass that wrote it, so a reader accepts a word only when its tag matches.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define DM_WAVE 64

namespace dm {

// ---------------------------------------------------------------------------
// keys
// ---------------------------------------------------------------------------
// FP32 -> unsigned key whose unsigned order is the numeric order.  -0.0 is
// folded onto +0.0 so that the two zeros tie (and stay in point order).
__device__ __forceinline__ uint32_t f32_key(float v) {
    uint32_t u = __float_as_uint(v);
    if (u == 0x80000000u) u = 0u;
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float key_f32(uint32_t k) {
    uint32_t u = (k & 0x80000000u) ? (k & 0x7fffffffu) : ~k;
    return __uint_as_float(u);
}
__device__ __forceinline__ uint32_t i32_key(int32_t v) { return (uint32_t)v ^ 0x80000000u; }
__device__ __forceinline__ int32_t key_i32(uint32_t k) { return (int32_t)(k ^ 0x80000000u); }

// ---------------------------------------------------------------------------
// double-float arithmetic (Knuth's TwoSum, FMA-based TwoProd)
// ---------------------------------------------------------------------------
struct dd { float hi, lo; };

__device__ __forceinline__ dd dd_make(float a) { return dd{a, 0.0f}; }

// exact: a + b = s + e
__device__ __forceinline__ void two_sum(float a, float b, float& s, float& e) {
    s = a + b;
    float bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}
__device__ __forceinline__ void fast_two_sum(float a, float b, float& s, float& e) {
    s = a + b;
    e = b - (s - a);
}
__device__ __forceinline__ dd dd_add(dd a, dd b) {
    float s, e;
    two_sum(a.hi, b.hi, s, e);
    e += a.lo + b.lo;
    dd r;
    fast_two_sum(s, e, r.hi, r.lo);
    return r;
}
__device__ __forceinline__ dd dd_add_f(dd a, float b) {
    float s, e;
    two_sum(a.hi, b, s, e);
    e += a.lo;
    dd r;
    fast_two_sum(s, e, r.hi, r.lo);
    return r;
}
__device__ __forceinline__ double dd_to_f64(dd a) { return (double)a.hi + (double)a.lo; }

// ---------------------------------------------------------------------------
// tagged words: [63:32] tag, [31:0] payload
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t tag_word(uint32_t tag, uint32_t payload) {
    return ((uint64_t)tag << 32) | (uint64_t)payload;
}
__device__ __forceinline__ void publish_word(uint64_t* p, uint64_t w) {
    __hip_atomic_store(p, w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t peek_word(const uint64_t* p) {
    return __hip_atomic_load(const_cast<uint64_t*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// lane id within the wave
__device__ __forceinline__ int lane_id() {
    return (int)__builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}
// number of set bits of `mask` in lanes below this one
__device__ __forceinline__ uint32_t mask_rank(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

}  // namespace dm
