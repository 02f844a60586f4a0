// Key-range partition of the outer keys for the binned probe.
//
// The probe's cost on a large R is the last-mile search (Section III and the
// time breakdown of Section VI-B): each key's window lies in a random part of
// R, so its reads miss every cache.  Probing the keys in key order instead
// makes neighbouring keys search neighbouring parts of R, the same locality
// the paper's buffered index gets by queueing requests per node before
// serving them (Section III-B, "Buffered GRMI").  Here the keys of S are put
// into kBins equi-depth key ranges of R (bin(x) = number of fences <= x,
// fence i = R[(i + 1) * n / kBins]) by a stable two-pass LSD partition over
// the two 6-bit digits of the bin number:
//
//   hist   per chunk of kPartChunk keys, the count of each digit (pass 1 also
//          computes and stores every key's bin by binary search over the
//          fences held in LDS);
//   scan   exclusive prefix of the digit-major counts = each chunk's output
//          offset per digit;
//   scatter  stable ranking inside the chunk (ballots per wave, one running
//          count per digit held by lane `digit`), staging in LDS in digit
//          order, then contiguous stores of each digit's run; the output
//          position of every input element is also stored (`dest`) so that
//          the results can be put back in input order with coalesced
//          gathers (`unpermute`).
//
// Chunk layout: element e = wave * 1024 + k * 64 + lane of a chunk, so each
// wave reads 16 runs of 64 consecutive keys.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "lj_device.h"
#include "lj_internal.h"

namespace lj {
namespace {

constexpr int kWaves = kBlock / 64;
constexpr uint32_t kWaveSpan = kPartChunk / kWaves;  // elements per wave per chunk
static_assert(kWaveSpan == kPartItems * 64, "chunk = waves x items x 64 lanes");
static_assert(kDigits == 64, "one running digit count per lane");

__device__ inline uint32_t digit_of(uint32_t bin, uint32_t shift) {
    return (bin >> shift) & (kDigits - 1);
}

// Lane d's count of the valid elements of its wave whose digit is d: six
// ballots on the digit's bits select the lanes that match d.  Counting this
// way needs no LDS atomics (which conflict heavily on 64 counters).
__device__ __forceinline__ uint32_t digit_match_count(uint32_t dg, bool valid, int lane) {
    uint64_t mine = __ballot(valid);
#pragma unroll
    for (int bit = 0; bit < (int)kDigitBits; ++bit) {
        const uint64_t bb = __ballot((dg >> bit) & 1u);
        mine &= ((lane >> bit) & 1) ? bb : ~bb;
    }
    return (uint32_t)__popcll(mine);
}

// Per chunk: digit histogram into hist[digit * nchunks + chunk].  With
// kFromKeys the bins are computed from the keys and stored to `bins`;
// otherwise they are read from `bins`.  A key's bin is the number of fences
// below its bucket (table in LDS) plus a binary search over the fences of
// its own bucket (fences in LDS), usually none or one or two.
template <bool kFromKeys>
__global__ __launch_bounds__(kBlock) void bin_hist_kernel(const uint64_t* __restrict__ keys,
                                                          const uint64_t* __restrict__ fences,
                                                          const uint16_t* __restrict__ bucket_lo,
                                                          uint16_t* __restrict__ bins,
                                                          uint64_t m, uint32_t nchunks,
                                                          uint32_t shift,
                                                          uint32_t* __restrict__ hist) {
    __shared__ uint64_t sf[kFromKeys ? kBins : 1];
    __shared__ uint16_t sb[kFromKeys ? kBuckets + 2 : 2];
    __shared__ uint32_t cnt[kDigits];
    __shared__ uint32_t wcnt[kFromKeys ? 1 : kWaves][kDigits];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if constexpr (kFromKeys) {
        for (uint32_t i = tid; i < kBins - 1; i += kBlock) sf[i] = fences[i];
        for (uint32_t i = tid; i <= kBuckets; i += kBlock) sb[i] = bucket_lo[i];
    }
    for (uint32_t c = blockIdx.x; c < nchunks; c += gridDim.x) {
        if (tid < (int)kDigits) cnt[tid] = 0;
        __syncthreads();
        const uint64_t e0 = (uint64_t)c * kPartChunk + (uint64_t)wave * kWaveSpan + lane;
        uint32_t b[kPartItems];
        if constexpr (kFromKeys) {
            uint64_t x[kPartItems];
            uint32_t len[kPartItems];
#pragma unroll
            for (int k = 0; k < (int)kPartItems; ++k) {
                const uint64_t p = e0 + (uint64_t)k * 64;
                x[k] = keys[p < m ? p : m - 1];
            }
#pragma unroll
            for (int k = 0; k < (int)kPartItems; ++k) {
                const uint32_t bk = key_bucket(x[k]);
                b[k] = sb[bk];
                len[k] = sb[bk + 1] - b[k];
            }
            // Count the bucket's fences <= x: lower bound over
            // sf[b .. b + len), all inside the kBins - 1 fences.
            for (;;) {
                uint32_t act = 0;
#pragma unroll
                for (int k = 0; k < (int)kPartItems; ++k) act |= len[k];
                if (!act) break;
#pragma unroll
                for (int k = 0; k < (int)kPartItems; ++k) {
                    const uint32_t half = len[k] >> 1;
                    const uint32_t at = b[k] + half;
                    const bool le = len[k] != 0 && sf[at < kBins - 1 ? at : kBins - 2] <= x[k];
                    b[k] = le ? at + 1 : b[k];
                    len[k] = le ? len[k] - half - 1 : half;
                }
            }
#pragma unroll
            for (int k = 0; k < (int)kPartItems; ++k) {
                const uint64_t p = e0 + (uint64_t)k * 64;
                if (p < m) bins[p] = (uint16_t)b[k];
            }
        } else {
#pragma unroll
            for (int k = 0; k < (int)kPartItems; ++k) {
                const uint64_t p = e0 + (uint64_t)k * 64;
                b[k] = p < m ? bins[p] : 0u;
            }
        }
        if constexpr (kFromKeys) {
#pragma unroll
            for (int k = 0; k < (int)kPartItems; ++k)
                if (e0 + (uint64_t)k * 64 < m) atomicAdd(&cnt[digit_of(b[k], shift)], 1u);
            __syncthreads();
            if (tid < (int)kDigits) hist[(uint64_t)tid * nchunks + c] = cnt[tid];
        } else {
            uint32_t run = 0;
#pragma unroll
            for (int k = 0; k < (int)kPartItems; ++k)
                run += digit_match_count(digit_of(b[k], shift), e0 + (uint64_t)k * 64 < m, lane);
            wcnt[wave][lane] = run;
            __syncthreads();
            if (tid < (int)kDigits) {
                uint32_t t = 0;
#pragma unroll
                for (int w = 0; w < kWaves; ++w) t += wcnt[w][tid];
                hist[(uint64_t)tid * nchunks + c] = t;
            }
        }
        __syncthreads();
    }
}

// bin_hist_kernel<true> for an index with a radix root and at least kBins
// leaves: a key's bin is its leaf scaled to kBins ranges,
// (leaf * bin_mul) >> 32 with bin_mul = floor(kBins * 2^32 / L), so bin <
// kBins and bins are non-decreasing in the key (the radix root gives leaves
// of about n / L keys each, so these ranges are about equi-depth, like the
// fences; any bin order gives the same pairs).  The root's table is staged
// in LDS; no fence search.
__global__ __launch_bounds__(kBlock) void bin_hist_root_kernel(const uint64_t* __restrict__ keys,
                                                               RootModel root, uint64_t bin_mul,
                                                               uint16_t* __restrict__ bins,
                                                               uint64_t m, uint32_t nchunks,
                                                               uint32_t* __restrict__ hist) {
    __shared__ __align__(16) uint32_t s_root[kRootTabLen];
    __shared__ uint32_t cnt[kDigits];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    {
        const uint4* src = (const uint4*)root.tab_dev;
        uint4* dst = (uint4*)s_root;
        for (uint32_t i = tid; i < kRootTabLen / 4; i += kBlock) dst[i] = src[i];
    }
    for (uint32_t c = blockIdx.x; c < nchunks; c += gridDim.x) {
        if (tid < (int)kDigits) cnt[tid] = 0;
        __syncthreads();
        const uint64_t e0 = (uint64_t)c * kPartChunk + (uint64_t)wave * kWaveSpan + lane;
        uint64_t x[kPartItems];
#pragma unroll
        for (int k = 0; k < (int)kPartItems; ++k) {
            const uint64_t p = e0 + (uint64_t)k * 64;
            x[k] = keys[p < m ? p : m - 1];
        }
#pragma unroll
        for (int k = 0; k < (int)kPartItems; ++k) {
            const uint64_t p = e0 + (uint64_t)k * 64;
            const uint32_t leaf = route_radix(root, s_root, x[k]);
            const uint32_t b = (uint32_t)(((uint64_t)leaf * bin_mul) >> 32);
            if (p < m) {
                bins[p] = (uint16_t)b;
                atomicAdd(&cnt[digit_of(b, 0)], 1u);
            }
        }
        __syncthreads();
        if (tid < (int)kDigits) hist[(uint64_t)tid * nchunks + c] = cnt[tid];
        __syncthreads();
    }
}

// In-place exclusive prefix sum of n counts (total < 2^62, and < 2^32 for
// u32), one tile of kScanTile per block, tiles chained by decoupled
// look-back.
template <class T>
__global__ __launch_bounds__(kBlock) void scan_kernel(T* __restrict__ d, uint64_t n,
                                                      uint64_t* status, uint32_t* tile_ctr,
                                                      uint32_t* err) {
    __shared__ uint32_t s_tile;
    __shared__ uint64_t wsum[kWaves];
    __shared__ uint64_t s_excl;
    constexpr int kPer = kScanTile / kBlock;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (tid == 0) s_tile = atomicAdd(tile_ctr, 1u);
    __syncthreads();
    const uint32_t tile = s_tile;
    const uint64_t base = (uint64_t)tile * kScanTile + (uint64_t)tid * kPer;
    T v[kPer];
    uint64_t tsum = 0;
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
        v[i] = base + i < n ? d[base + i] : (T)0;
        tsum += v[i];
    }
    const uint64_t incl = wave_incl_scan(tsum, lane);
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    uint64_t wpre = 0, total = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
        wpre += w < wave ? wsum[w] : 0;
        total += wsum[w];
    }
    if (wave == 0) {
        const uint64_t e = look_back(status, tile, total, err, lane);
        if (lane == 0) s_excl = e;
    }
    __syncthreads();
    uint64_t run = s_excl + wpre + incl - tsum;
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
        if (base + i < n) d[base + i] = (T)run;
        run += v[i];
    }
}

// One stable partition pass by digit (bin >> shift) & 63.  gofs holds the
// scanned digit-major counts of bin_hist_kernel for the same chunks.
// keys_out[dest] = keys_in[p], bins_out[dest] = bins_in[p] (when bins_out is
// given) and dest_out[p] = dest for every input position p.
// kWriteBins: the pass also stores the bins in their new order (the first
// pass, for the second); without it the LDS stage keeps only the 1-byte
// digit (38 KB of LDS instead of 42 KB), which lets four workgroups share a
// CU instead of three.
template <bool kWriteBins>
__global__ __launch_bounds__(kBlock) void bin_scatter_kernel(
    const uint64_t* __restrict__ keys_in, const uint16_t* __restrict__ bins_in,
    const uint32_t* __restrict__ gofs, uint64_t m, uint32_t nchunks, uint32_t shift,
    uint64_t* __restrict__ keys_out, uint16_t* __restrict__ bins_out,
    uint32_t* __restrict__ dest_out) {
    using StageT = typename std::conditional<kWriteBins, uint16_t, uint8_t>::type;
    __shared__ uint64_t skey[kPartChunk];
    __shared__ StageT sbin[kPartChunk];
    __shared__ uint32_t wbase[kWaves][kDigits];  // wave totals, then wave bases
    __shared__ uint32_t lstart[kDigits];         // chunk-local start of each digit
    __shared__ uint32_t gstart[kDigits];         // global start of each digit's run
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    for (uint32_t c = blockIdx.x; c < nchunks; c += gridDim.x) {
        const uint64_t c0 = (uint64_t)c * kPartChunk;
        const uint32_t e0 = (uint32_t)wave * kWaveSpan + lane;
        uint64_t x[kPartItems];
        uint32_t b[kPartItems], rank[kPartItems];
#pragma unroll
        for (int k = 0; k < (int)kPartItems; ++k) {
            const uint64_t p = c0 + e0 + (uint64_t)k * 64;
            const uint64_t q = p < m ? p : m - 1;
            x[k] = keys_in[q];
            b[k] = bins_in[q];
        }
        // Rank of each element among the earlier elements of its wave with
        // the same digit; lane d keeps the wave's running count of digit d.
        uint32_t run = 0;
#pragma unroll
        for (int k = 0; k < (int)kPartItems; ++k) {
            const bool valid = c0 + e0 + (uint64_t)k * 64 < m;
            const uint32_t dg = digit_of(b[k], shift);
            const uint64_t vb = __ballot(valid);
            uint64_t same = vb, mine = vb;  // lanes with my digit / with digit == my lane
#pragma unroll
            for (int bit = 0; bit < (int)kDigitBits; ++bit) {
                const uint64_t bb = __ballot((dg >> bit) & 1u);
                same &= ((dg >> bit) & 1u) ? bb : ~bb;
                mine &= ((lane >> bit) & 1) ? bb : ~bb;
            }
            rank[k] = (uint32_t)__shfl((int)run, (int)dg, 64) + (uint32_t)__popcll(same & lt);
            run += (uint32_t)__popcll(mine);
        }
        wbase[wave][lane] = run;
        __syncthreads();
        if (wave == 0) {
            uint32_t t[kWaves], tot = 0;
#pragma unroll
            for (int w = 0; w < kWaves; ++w) {
                t[w] = wbase[w][lane];
                tot += t[w];
            }
            const uint32_t excl = (uint32_t)wave_incl_scan(tot, lane) - tot;
            lstart[lane] = excl;
            uint32_t acc = excl;
#pragma unroll
            for (int w = 0; w < kWaves; ++w) {
                wbase[w][lane] = acc;
                acc += t[w];
            }
            gstart[lane] = gofs[(uint64_t)lane * nchunks + c];
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < (int)kPartItems; ++k) {
            const uint64_t p = c0 + e0 + (uint64_t)k * 64;
            if (p < m) {
                const uint32_t dg = digit_of(b[k], shift);
                const uint32_t lpos = wbase[wave][dg] + rank[k];
                skey[lpos] = x[k];
                sbin[lpos] = kWriteBins ? (StageT)b[k] : (StageT)dg;
                dest_out[p] = gstart[dg] + (lpos - lstart[dg]);
            }
        }
        __syncthreads();
        const uint32_t nvalid = m - c0 < kPartChunk ? (uint32_t)(m - c0) : kPartChunk;
        for (uint32_t lp = tid; lp < nvalid; lp += kBlock) {
            const uint32_t v = sbin[lp];
            const uint32_t dg = kWriteBins ? digit_of(v, shift) : v;
            const uint32_t dst = gstart[dg] + (lp - lstart[dg]);
            keys_out[dst] = skey[lp];
            if constexpr (kWriteBins) bins_out[dst] = (uint16_t)v;
        }
        __syncthreads();
    }
}

// out[p] = in[dest[p]] for p < m; one chunk of kPartChunk positions per
// block iteration so that the runs a chunk reads are used whole by one CU.
template <class T>
__global__ __launch_bounds__(kBlock) void unpermute_kernel(const uint32_t* __restrict__ dest,
                                                           const T* __restrict__ in,
                                                           T* __restrict__ out, uint64_t m,
                                                           uint32_t nchunks) {
    const int tid = threadIdx.x;
    for (uint32_t c = blockIdx.x; c < nchunks; c += gridDim.x) {
        const uint64_t c0 = (uint64_t)c * kPartChunk;
        uint32_t dd[kPartItems];
#pragma unroll
        for (int k = 0; k < (int)kPartItems; ++k) {
            const uint64_t p = c0 + (uint64_t)k * kBlock + tid;
            dd[k] = p < m ? dest[p] : 0u;
        }
        T v[kPartItems];
#pragma unroll
        for (int k = 0; k < (int)kPartItems; ++k) v[k] = in[dd[k]];
#pragma unroll
        for (int k = 0; k < (int)kPartItems; ++k) {
            const uint64_t p = c0 + (uint64_t)k * kBlock + tid;
            if (p < m) out[p] = v[k];
        }
    }
}

// unpermute_kernel that also writes the number of pairs of each chunk:
// a 4-byte result is one pair unless ~0u, an 8-byte one holds its pair
// count in the high word.
template <class T>
__global__ __launch_bounds__(kBlock) void unpermute_count_kernel(
    const uint32_t* __restrict__ dest, const T* __restrict__ in, T* __restrict__ out,
    uint64_t m, uint32_t nchunks, uint64_t* __restrict__ counts) {
    __shared__ uint64_t wsum[kWaves];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (uint32_t c = blockIdx.x; c < nchunks; c += gridDim.x) {
        const uint64_t c0 = (uint64_t)c * kPartChunk;
        uint32_t dd[kPartItems];
#pragma unroll
        for (int k = 0; k < (int)kPartItems; ++k) {
            const uint64_t p = c0 + (uint64_t)k * kBlock + tid;
            dd[k] = p < m ? dest[p] : 0u;
        }
        T v[kPartItems];
#pragma unroll
        for (int k = 0; k < (int)kPartItems; ++k) v[k] = in[dd[k]];
        uint64_t pairs = 0;
#pragma unroll
        for (int k = 0; k < (int)kPartItems; ++k) {
            const uint64_t p = c0 + (uint64_t)k * kBlock + tid;
            if (p < m) {
                out[p] = v[k];
                if constexpr (sizeof(T) == 4) pairs += v[k] != ~0u ? 1u : 0u;
                else pairs += (uint64_t)v[k] >> 32;
            }
        }
        pairs = wave_sum(pairs);
        if (lane == 0) wsum[wave] = pairs;
        __syncthreads();
        if (tid == 0) {
            uint64_t t = 0;
#pragma unroll
            for (int w = 0; w < kWaves; ++w) t += wsum[w];
            counts[c] = t;
        }
        __syncthreads();
    }
}

unsigned chunk_grid(uint32_t nchunks, uint32_t cap) {
    return nchunks < cap ? (nchunks ? nchunks : 1u) : cap;
}

}  // namespace

hipError_t launch_partition(const lj_index* idx, const uint64_t* s, uint64_t m, void* ws,
                            const BinnedWs& L, hipStream_t stream) {
    char* w = (char*)ws;
    const uint32_t nchunks = (uint32_t)num_tiles(m, kPartChunk);
    const uint64_t nh = (uint64_t)kDigits * nchunks;
    const unsigned scan_grid = (unsigned)num_tiles(nh, kScanTile);
    uint32_t* err = &((WsHeader*)ws)->err;
    uint32_t* hist1 = (uint32_t*)(w + L.hist1);
    uint32_t* hist2 = (uint32_t*)(w + L.hist2);
    uint16_t* bins_s = (uint16_t*)(w + L.bins_s);
    uint16_t* bins_1 = (uint16_t*)(w + L.bins_1);
    uint64_t* p1 = (uint64_t*)(w + L.p1);
    uint64_t* p2 = (uint64_t*)(w + L.p2);
    uint32_t* ctr = (uint32_t*)(w + L.scan_ctr);

    // Pass 1: low digit.
    if (idx->root.kind == kRootRadix && idx->leaves >= kBins)
        hipLaunchKernelGGL(bin_hist_root_kernel, dim3(chunk_grid(nchunks, 2048)), dim3(kBlock), 0,
                           stream, s, idx->root, ((uint64_t)kBins << 32) / idx->root.leaves,
                           bins_s, m, nchunks, hist1);
    else
        hipLaunchKernelGGL(bin_hist_kernel<true>, dim3(chunk_grid(nchunks, 2048)), dim3(kBlock),
                           0, stream, s, idx->fences_dev, idx->bucket_lo_dev, bins_s, m, nchunks,
                           0u, hist1);
    hipLaunchKernelGGL(scan_kernel<uint32_t>, dim3(scan_grid), dim3(kBlock), 0, stream, hist1,
                       nh, (uint64_t*)(w + L.scan_st1), ctr, err);
    hipLaunchKernelGGL(bin_scatter_kernel<true>, dim3(chunk_grid(nchunks, 65535)), dim3(kBlock),
                       0, stream, s, bins_s, hist1, m, nchunks, 0u, p1, bins_1,
                       (uint32_t*)(w + L.dest1));
    // Pass 2: high digit.
    hipLaunchKernelGGL(bin_hist_kernel<false>, dim3(chunk_grid(nchunks, 4096)), dim3(kBlock), 0,
                       stream, (const uint64_t*)nullptr, (const uint64_t*)nullptr,
                       (const uint16_t*)nullptr, bins_1, m, nchunks, kDigitBits, hist2);
    hipLaunchKernelGGL(scan_kernel<uint32_t>, dim3(scan_grid), dim3(kBlock), 0, stream, hist2,
                       nh, (uint64_t*)(w + L.scan_st2), ctr + 1, err);
    hipLaunchKernelGGL(bin_scatter_kernel<false>, dim3(chunk_grid(nchunks, 65535)), dim3(kBlock),
                       0, stream, p1, bins_1, hist2, m, nchunks, kDigitBits, p2,
                       (uint16_t*)nullptr, (uint32_t*)(w + L.dest2));
    return hipGetLastError();
}

hipError_t launch_scan_u32(uint32_t* d, uint64_t n, uint64_t* status, uint32_t* ctr,
                           uint32_t* err, hipStream_t stream) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(scan_kernel<uint32_t>, dim3((unsigned)num_tiles(n, kScanTile)),
                       dim3(kBlock), 0, stream, d, n, status, ctr, err);
    return hipGetLastError();
}

hipError_t launch_unpermute(const uint32_t* dest, const void* in, void* out, uint64_t m,
                            bool wide, hipStream_t stream) {
    const uint32_t nchunks = (uint32_t)num_tiles(m, kPartChunk);
    const dim3 grid(chunk_grid(nchunks, 65535)), block(kBlock);
    if (wide)
        hipLaunchKernelGGL(unpermute_kernel<uint64_t>, grid, block, 0, stream, dest,
                           (const uint64_t*)in, (uint64_t*)out, m, nchunks);
    else
        hipLaunchKernelGGL(unpermute_kernel<uint32_t>, grid, block, 0, stream, dest,
                           (const uint32_t*)in, (uint32_t*)out, m, nchunks);
    return hipGetLastError();
}

hipError_t launch_unpermute_count(const uint32_t* dest, const void* in, void* out, uint64_t m,
                                  bool wide, void* ws, const BinnedWs& L, hipStream_t stream) {
    char* w = (char*)ws;
    const uint32_t nchunks = (uint32_t)num_tiles(m, kPartChunk);
    const dim3 grid(chunk_grid(nchunks, 65535)), block(kBlock);
    uint64_t* counts = (uint64_t*)(w + L.counts);
    if (wide)
        hipLaunchKernelGGL(unpermute_count_kernel<uint64_t>, grid, block, 0, stream, dest,
                           (const uint64_t*)in, (uint64_t*)out, m, nchunks, counts);
    else
        hipLaunchKernelGGL(unpermute_count_kernel<uint32_t>, grid, block, 0, stream, dest,
                           (const uint32_t*)in, (uint32_t*)out, m, nchunks, counts);
    // counts[nchunks] is 0 (zeroed with the control block): after the scan it
    // holds the total.
    const uint64_t n = (uint64_t)nchunks + 1;
    hipLaunchKernelGGL(scan_kernel<uint64_t>, dim3((unsigned)num_tiles(n, kScanTile)),
                       dim3(kBlock), 0, stream, counts, n, (uint64_t*)(w + L.scan_st3),
                       (uint32_t*)(w + L.scan_ctr) + 2, &((WsHeader*)ws)->err);
    return hipGetLastError();
}

}  // namespace lj
