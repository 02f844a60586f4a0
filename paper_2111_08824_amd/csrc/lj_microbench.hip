// Random-gather microbenchmark: the random-access ceiling against which the
// probe's achieved bandwidth is compared.  Every lane issues 8 independent
// 8-byte loads per round, each to a pseudo-random granule of the buffer (a
// SplitMix64 hash of the global load index), the same access shape as one
// step of the probe's search.
#include <hip/hip_runtime.h>

#include "lj_internal.h"

namespace lj {
namespace {

__device__ inline uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

constexpr int kGatherInFlight = 8;

__global__ __launch_bounds__(256) void random_gather_kernel(const uint64_t* buf,
                                                            uint64_t granules,
                                                            uint32_t words_per_granule,
                                                            uint64_t rounds, uint64_t seed,
                                                            uint64_t* sink) {
    const uint64_t gid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t nthreads = (uint64_t)gridDim.x * blockDim.x;
    uint64_t acc = 0;
    for (uint64_t r = 0; r < rounds; ++r) {
        uint64_t v[kGatherInFlight];
#pragma unroll
        for (int k = 0; k < kGatherInFlight; ++k) {
            uint64_t h = mix64(seed + ((r * kGatherInFlight + k) * nthreads + gid));
            v[k] = buf[(h % granules) * words_per_granule];
        }
#pragma unroll
        for (int k = 0; k < kGatherInFlight; ++k) acc ^= v[k];
    }
    if (acc == 0x9e3779b97f4a7c15ull) *sink = acc;  // practically never taken
    if (gid == 0) *sink = acc;
}

}  // namespace

hipError_t launch_random_gather(const void* buf, uint64_t bytes, uint32_t granule,
                                uint64_t reads, uint64_t seed, uint64_t* sink,
                                hipStream_t stream) {
    const uint64_t granules = bytes / granule;
    const unsigned block = 256;
    unsigned grid = 256 * 32;  // 32 blocks per CU
    const uint64_t per_round = (uint64_t)grid * block * kGatherInFlight;
    uint64_t rounds = (reads + per_round - 1) / per_round;
    if (rounds == 0) rounds = 1;
    hipLaunchKernelGGL(random_gather_kernel, dim3(grid), dim3(block), 0, stream,
                       (const uint64_t*)buf, granules, granule / 8u, rounds, seed, sink);
    return hipGetLastError();
}

}  // namespace lj
