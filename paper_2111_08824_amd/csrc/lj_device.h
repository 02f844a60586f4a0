// Device helpers shared by the probe and partition kernels: wave
// reductions and the single-pass decoupled look-back scan (Merrill and
// Garland, "Single-pass parallel prefix scan with decoupled look-back",
// NVIDIA TR 2016) over 64-bit status words.
#pragma once

#include <hip/hip_runtime.h>

#include <stdint.h>

namespace lj {
namespace {

constexpr uint64_t kFlagAgg = 1ull << 62;
constexpr uint64_t kFlagInc = 2ull << 62;
constexpr uint64_t kValMask = (1ull << 62) - 1;
constexpr uint32_t kSpinLimit = 1u << 24;  // ~0.5 s of s_sleep before giving up

__device__ inline uint64_t ld_status(const uint64_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void st_status(uint64_t* p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline uint64_t wave_sum(uint64_t v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    return v;
}

__device__ inline uint64_t wave_incl_scan(uint64_t v, int lane) {
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint64_t t = __shfl_up(v, d, 64);
        if (lane >= d) v += t;
    }
    return v;
}

// Decoupled look-back, run by wave 0 of the block.  Publishes the tile's
// aggregate, accumulates the predecessors' values until one with an
// inclusive prefix is found, publishes the tile's inclusive prefix and
// returns its exclusive prefix (valid in every lane of wave 0).
__device__ uint64_t look_back(uint64_t* status, uint32_t tile, uint64_t total,
                              uint32_t* err, int lane) {
    if (tile == 0) {
        if (lane == 0) st_status(&status[0], kFlagInc | total);
        return 0;
    }
    if (lane == 0) st_status(&status[tile], kFlagAgg | total);
    uint64_t excl = 0;
    int64_t base = (int64_t)tile - 1;
    for (;;) {
        int64_t idx = base - lane;
        uint64_t st = idx >= 0 ? ld_status(&status[idx]) : kFlagInc;
        uint32_t spins = 0;
        while (__ballot((st >> 62) == 0)) {
            if ((st >> 62) == 0) st = ld_status(&status[idx]);
            if (++spins > kSpinLimit) {
                // A predecessor never published: report and stop waiting so
                // that the kernel still exits.
                if ((st >> 62) == 0) {
                    __hip_atomic_fetch_or(err, 1u, __ATOMIC_SEQ_CST, __HIP_MEMORY_SCOPE_AGENT);
                    st = kFlagInc;
                }
            }
            __builtin_amdgcn_s_sleep(1);
        }
        uint64_t inc = __ballot((st >> 62) == 2);
        if (inc) {
            int first = __ffsll((unsigned long long)inc) - 1;
            excl += wave_sum(lane <= first ? (st & kValMask) : 0);
            break;
        }
        excl += wave_sum(st & kValMask);
        base -= 64;
    }
    if (lane == 0) st_status(&status[tile], kFlagInc | (excl + total));
    return excl;
}

}  // namespace
}  // namespace lj
