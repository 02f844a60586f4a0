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

// Root model, one of two kinds:
//   linear:  leaf = clamp(floor(a0 + b0 * (x - kmin)), 0, L - 1);
//   radix:   a piecewise-linear CDF over a radix table of the key.  The
//            offset x' = x - kmin (0 below kmin) falls in one of kRootBuckets
//            buckets of a float-like code (the exponent of x' and its next
//            kRootSubBits bits; values below 2^kRootSubBits are their own
//            buckets), so bucket widths are powers of two that grow with
//            x'.  tab[b] holds the leaf coordinate (fixed point, frac_bits
//            fraction bits) of bucket b's lower edge: leaves * rank / n,
//            with rank the number of keys of R below it.  Inside a bucket
//            the coordinate is interpolated linearly, in integers only:
//            tab[b] + ((tab[b+1] - tab[b]) * r) >> w, with r the top (at
//            most 32) bits of x' below the bucket's leading bits and 2^w
//            their range.  Non-decreasing in x, exact on host and device.
// The table is read through tab_dev in device code and tab_host on the host.
constexpr uint32_t kRootLinear = 0;
constexpr uint32_t kRootRadix = 1;
constexpr uint32_t kRootSubBits = 6;
constexpr uint32_t kRootBuckets = (64 - kRootSubBits + 1) << kRootSubBits;  // 3776
// Table length: kRootBuckets + 1 edges, padded to a multiple of 4 words
// (the padding repeats the last edge).
constexpr uint32_t kRootTabLen = (kRootBuckets + 1 + 3) & ~3u;
struct RootModel {
    double a0;
    double b0;
    uint64_t kmin;
    uint32_t leaves;
    uint32_t kind;       // kRootLinear or kRootRadix
    uint32_t frac_bits;  // radix: fraction bits of the table's coordinates
    uint32_t pad;
    const uint32_t* tab_host;  // radix: kRootTabLen coordinates
    const uint32_t* tab_dev;
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

// Bucket of the radix root for offset xp, with the offset's bits below the
// bucket's leading bits, cut to their top 32 (*rem), and the number of
// those bits kept (*w; the bucket spans 2^w values of *rem).
__host__ __device__ inline uint32_t root_bucket(uint64_t xp, uint64_t* rem, uint32_t* w) {
    if (xp < (1ull << kRootSubBits)) {
        *rem = 0;
        *w = 0;
        return (uint32_t)xp;
    }
    const uint32_t e = 63u - (uint32_t)clz64(xp);  // >= kRootSubBits
    const uint32_t low = e - kRootSubBits;          // bits below the bucket's leading bits
    const uint32_t sub = (uint32_t)(xp >> low) & ((1u << kRootSubBits) - 1u);
    const uint64_t r = low ? xp & ((1ull << low) - 1ull) : 0ull;
    const uint32_t cut = low > 32u ? low - 32u : 0u;
    *rem = r >> cut;
    *w = low - cut;
    return ((e - kRootSubBits + 1u) << kRootSubBits) | sub;
}

// Radix root with the table at `tab` (global or LDS copy).
__host__ __device__ inline uint32_t route_radix(const RootModel& rm, const uint32_t* tab,
                                                uint64_t x) {
    uint64_t rem;
    uint32_t w;
    const uint32_t b = root_bucket(sat_sub(x, rm.kmin), &rem, &w);
    const uint32_t t0 = tab[b], t1 = tab[b + 1];
    const uint64_t coord = (uint64_t)t0 + (((uint64_t)(t1 - t0) * rem) >> w);
    const uint64_t leaf = coord >> rm.frac_bits;
    return leaf < rm.leaves ? (uint32_t)leaf : rm.leaves - 1;
}

// Root routing: non-decreasing in x (linear: b0 >= 0, FP64; radix: the
// table is non-decreasing).
__host__ __device__ inline uint32_t route(const RootModel& rm, uint64_t x) {
    if (rm.kind == kRootRadix) {
#ifdef __HIP_DEVICE_COMPILE__
        return route_radix(rm, rm.tab_dev, x);
#else
        return route_radix(rm, rm.tab_host, x);
#endif
    }
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
