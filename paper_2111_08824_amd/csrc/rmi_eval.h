// Two-level linear RMI evaluation, shared by the host-side builder and the
// GPU probe kernels (Section II-D, "Recursive Model Index").
//
// The root model maps a key to a leaf; the leaf model maps the key to a
// predicted position inside the leaf; the leaf's error bounds, recorded at
// build time, turn that prediction into a search window.  The bounds are
// only valid if the build evaluates exactly the function the probe
// evaluates, so every step here is defined bit-for-bit:
//   * integer differences are exact (u64 arithmetic, saturating at 0);
//   * u64 -> f64 and u64 -> f32 conversions round to nearest even, written
//     out with explicit integer steps and a single rounding;
//   * the affine models use fma / fmaf (one rounding each);
//   * float -> int conversion saturates (NaN -> 0) and truncates.
// Everything is compiled with -ffp-contract=off and without fast-math.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lj {

// Root model: leaf = clamp(floor(a0 + b0 * (x - kmin)), 0, L - 1).
struct RootModel {
    double a0;
    double b0;
    uint64_t kmin;
    uint32_t leaves;
    uint32_t pad;
};

// Leaf record, FP32 model (32 bytes).  Positions are relative to pos0, the
// first position of the leaf's run of R; keys routed to the leaf occupy
// R[pos0 .. pos0 + cnt).  The model predicts rel = slope*(x - base) + icpt,
// the key's offset inside that run; a key of R at offset e has
// e - rel(key) in [lo, hi].
struct alignas(32) LeafF32 {
    uint64_t base;   // smallest key routed to the leaf (R[pos0])
    float slope;
    float icpt;
    uint32_t pos0;
    uint32_t cnt;    // 0 = empty leaf: no key of R routes here
    int32_t lo;
    int32_t hi;
};

// Leaf record, FP64 model (48 bytes).
struct alignas(16) LeafF64 {
    uint64_t base;
    double slope;
    double icpt;
    uint32_t pos0;
    uint32_t cnt;
    int32_t lo;
    int32_t hi;
    uint64_t pad;
};

static_assert(sizeof(LeafF32) == 32, "leaf record layout");
static_assert(sizeof(LeafF64) == 48, "leaf record layout");

__host__ __device__ inline uint64_t sat_sub(uint64_t a, uint64_t b) {
    return a > b ? a - b : 0;
}

// u64 -> f64, round to nearest even: hi*2^32 is exact, the fma rounds once.
__host__ __device__ inline double u64_to_f64(uint64_t v) {
    double hi = (double)(uint32_t)(v >> 32);
    double lo = (double)(uint32_t)v;
    return fma(hi, 4294967296.0, lo);
}

// Leading zeros of a non-zero value.
__host__ __device__ inline int clz64(uint64_t v) { return __builtin_clzll(v); }

// 2^e for 0 <= e <= 64 as a float (exact).
__host__ __device__ inline float pow2f(int e) {
    union { uint32_t u; float f; } c;
    c.u = (uint32_t)(127 + e) << 23;
    return c.f;
}

// u64 -> f32, round to nearest even.  Normalise so the top bit is bit 63,
// keep the top 32 bits and fold the rest into bit 0 as a sticky bit (the
// u32 -> f32 conversion drops 8 bits, so bit 0 only acts as sticky), convert
// once, then scale by an exact power of two.
__host__ __device__ inline float u64_to_f32(uint64_t v) {
    if (v < (1ull << 32)) return (float)(uint32_t)v;
    int lz = clz64(v);
    uint64_t t = v << lz;
    uint32_t top = (uint32_t)(t >> 32) | (uint32_t)((uint32_t)t != 0u);
    return (float)top * pow2f(32 - lz);
}

// Saturating truncation to int32 (NaN -> 0).
__host__ __device__ inline int32_t f32_to_i32_sat(float f) {
    if (!(f == f)) return 0;
    if (f >= 2147483520.0f) return 2147483520;     // largest float below 2^31
    if (f <= -2147483648.0f) return INT32_MIN;
    return (int32_t)f;
}

__host__ __device__ inline int32_t f64_to_i32_sat(double d) {
    if (!(d == d)) return 0;
    if (d >= 2147483647.0) return INT32_MAX;
    if (d <= -2147483648.0) return INT32_MIN;
    return (int32_t)d;
}

// Root routing (FP64): non-decreasing in x because b0 >= 0.
__host__ __device__ inline uint32_t route(const RootModel& rm, uint64_t x) {
    double r = fma(rm.b0, u64_to_f64(sat_sub(x, rm.kmin)), rm.a0);
    if (!(r > 0.0)) return 0;
    if (r >= (double)rm.leaves) return rm.leaves - 1;
    return (uint32_t)r;
}

// Leaf prediction: offset inside the leaf's run, clamped to [0, cnt-1].
// Requires cnt > 0.
__host__ __device__ inline int32_t clamp_rel(int32_t rel, uint32_t cnt) {
    if (rel < 0) return 0;
    if ((uint32_t)rel >= cnt) return (int32_t)(cnt - 1);
    return rel;
}

__host__ __device__ inline int32_t predict_rel(const LeafF32& lf, uint64_t x) {
    float dx = u64_to_f32(sat_sub(x, lf.base));
    return clamp_rel(f32_to_i32_sat(fmaf(lf.slope, dx, lf.icpt)), lf.cnt);
}

__host__ __device__ inline int32_t predict_rel(const LeafF64& lf, uint64_t x) {
    double dx = u64_to_f64(sat_sub(x, lf.base));
    return clamp_rel(f64_to_i32_sat(fma(lf.slope, dx, lf.icpt)), lf.cnt);
}

}  // namespace lj
