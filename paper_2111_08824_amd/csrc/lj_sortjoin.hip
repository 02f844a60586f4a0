// Learned sort join (Section IV) of an unsorted R with an unsorted S.
//
// Phases, after Section IV-B..D, on one GPU:
//   model      (IV-B, "Model Building") a strided sample of R is sorted in
//              one block's LDS; every kSjSamplesPerKnot-th sample is a knot
//              of a linear-spline CDF, and a bucket table over the knots
//              (the key bucket of lj_internal.h) locates a key's segment.
//   partition  (IV-B, "Range Partitioning") the model, scaled up by `fan`
//              sub-partitions per segment, gives each key its partition
//              number (pid); per-chunk histograms, their prefix sums and
//              sequential per-digit writes put R in pid order, one stable
//              pass per 6-bit digit of the pid, carrying each key's input
//              position.
//   sort       (IV-C) each partition is sorted on its own by a bitonic
//              network over (key, position): by one wave in registers, or
//              by a block in LDS when larger; since the pids are monotone
//              in the key, R is then globally sorted.
//   join       (IV-D) S is put in order of its pid's high digits by two
//              more passes, and each key of S looks up its run in the one
//              partition of the sorted R that can hold its key (the
//              chunked join's overlap range for a shared model); the runs
//              are put back in S order and emitted, positions mapped back
//              to R's input order.
#include <hip/hip_runtime.h>

#include "lj_device.h"
#include "lj_sortjoin.h"

namespace lj {
namespace {

constexpr int kWaves = kBlock / 64;
constexpr uint32_t kWaveSpan = kPartChunk / kWaves;
constexpr int kModelThreads = 1024;
constexpr int kBigThreads = 1024;
constexpr int kJoinItems = 16;

__device__ inline uint32_t sj_digit(uint32_t pid, uint32_t shift) {
    return (pid >> shift) & (kDigits - 1);
}

// (key, position) order.
__device__ inline bool sj_greater(uint64_t ka, uint32_t pa, uint64_t kb, uint32_t pb) {
    return ka > kb || (ka == kb && pa > pb);
}

// Sample knot t of nk + 1 (equi-depth over the sorted sample s[0..ns)).
__device__ inline uint32_t sj_knot_at(uint32_t t, uint32_t ns, uint32_t nk) {
    return (uint32_t)(((uint64_t)t * (ns - 1)) / nk);
}

// Model of R: sample ns keys at stride n / ns, sort them, write the nk + 1
// knots and, per key bucket b, the number of knots in lower buckets.
__global__ __launch_bounds__(kModelThreads) void sj_model_kernel(
    const uint64_t* __restrict__ keys, uint64_t n, uint32_t ns, uint32_t nk,
    uint64_t* __restrict__ knots, uint16_t* __restrict__ kb_lo) {
    __shared__ uint64_t s[kSjSamples];
    const uint32_t tid = threadIdx.x;
    uint32_t N = 1;
    while (N < ns) N <<= 1;
    for (uint32_t i = tid; i < N; i += kModelThreads)
        s[i] = i < ns ? keys[((uint64_t)i * n) / ns] : ~0ull;
    __syncthreads();
    for (uint32_t k = 2; k <= N; k <<= 1) {
        for (uint32_t d = k >> 1; d > 0; d >>= 1) {
            for (uint32_t c = tid; c < N / 2; c += kModelThreads) {
                const uint32_t a = 2 * c - (c & (d - 1));
                const uint32_t b = a + d;
                const bool up = (a & k) == 0;
                const uint64_t x = s[a], y = s[b];
                if ((x > y) == up) {
                    s[a] = y;
                    s[b] = x;
                }
            }
            __syncthreads();
        }
    }
    for (uint32_t t = tid; t <= nk; t += kModelThreads) knots[t] = s[sj_knot_at(t, ns, nk)];
    // kb_lo[b] = t for the buckets b in (bucket(knot t-1), bucket(knot t)].
    for (uint32_t t = tid; t <= nk + 1; t += kModelThreads) {
        const int hi = t <= nk ? (int)key_bucket(s[sj_knot_at(t, ns, nk)]) : (int)kBuckets;
        const int lo = t ? (int)key_bucket(s[sj_knot_at(t - 1, ns, nk)]) : -1;
        for (int b = lo + 1; b <= hi; ++b) kb_lo[b] = (uint16_t)t;
    }
}

// Sub-partition of fraction f >= 0 of a segment among fan (f >= 1: the last).
__device__ inline uint32_t sj_sub(double f, uint32_t fan) {
    return f < 1.0 ? min((uint32_t)(f * (double)fan), fan - 1) : fan - 1;
}

// Partition number of key x by linear interpolation: inside segment
// [k0, k1), below the first knot over [0, k0), from the last knot k on over
// [k, 2k) (keys beyond in the last one).  Non-decreasing in x.
// b = number of knots <= x.
__device__ inline uint32_t sj_pid_of(uint64_t x, uint32_t b, const uint64_t* kn, uint32_t nk,
                                     uint32_t fan) {
    if (b == 0) return sj_sub((double)x / (double)kn[0], fan);
    if (b > nk) {
        const uint64_t k = kn[nk];
        return (nk + 1) * fan + sj_sub((double)(x - k) / (double)(k ? k : 1), fan);
    }
    const uint64_t k0 = kn[b - 1], k1 = kn[b];
    return b * fan + sj_sub((double)(x - k0) / (double)(k1 - k0), fan);
}

// Per chunk of kPartChunk keys: histogram of the pid digit at `shift`
// into hist[digit * nchunks + chunk].  With kFromKeys the pids are computed
// by the model (knots and bucket table staged in LDS) and stored to pids.
template <bool kFromKeys>
__global__ __launch_bounds__(kBlock) void sj_hist_kernel(
    const uint64_t* __restrict__ keys, const uint64_t* __restrict__ knots,
    const uint16_t* __restrict__ kb_lo, uint32_t nk, uint32_t fan,
    uint32_t* __restrict__ pids, uint64_t m, uint32_t nchunks, uint32_t shift,
    uint32_t* __restrict__ hist) {
    __shared__ uint64_t sk[kFromKeys ? kSjMaxSegments + 1 : 1];
    __shared__ uint16_t sl[kFromKeys ? kBuckets + 1 : 1];
    __shared__ uint32_t cnt[kDigits];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if constexpr (kFromKeys) {
        for (uint32_t i = tid; i <= nk; i += kBlock) sk[i] = knots[i];
        for (uint32_t i = tid; i <= kBuckets; i += kBlock) sl[i] = kb_lo[i];
    }
    for (uint32_t c = blockIdx.x; c < nchunks; c += gridDim.x) {
        if (tid < (int)kDigits) cnt[tid] = 0;
        __syncthreads();
        const uint64_t e0 = (uint64_t)c * kPartChunk + (uint64_t)wave * kWaveSpan + lane;
        uint32_t pid[kPartItems];
        if constexpr (kFromKeys) {
            // Knots <= x: those of lower key buckets plus a lockstep binary
            // search over the knots of x's own bucket.
            uint64_t x[kPartItems];
            uint32_t b[kPartItems], len[kPartItems];
#pragma unroll
            for (int k = 0; k < (int)kPartItems; ++k) {
                const uint64_t p = e0 + (uint64_t)k * 64;
                x[k] = keys[p < m ? p : m - 1];
            }
#pragma unroll
            for (int k = 0; k < (int)kPartItems; ++k) {
                const uint32_t bk = key_bucket(x[k]);
                b[k] = sl[bk];
                len[k] = sl[bk + 1] - b[k];
            }
            for (;;) {
                uint32_t act = 0;
#pragma unroll
                for (int k = 0; k < (int)kPartItems; ++k) act |= len[k];
                if (!act) break;
#pragma unroll
                for (int k = 0; k < (int)kPartItems; ++k) {
                    const uint32_t half = len[k] >> 1;
                    const uint32_t at = b[k] + half;
                    const bool le = len[k] != 0 && sk[at <= nk ? at : nk] <= x[k];
                    b[k] = le ? at + 1 : b[k];
                    len[k] = le ? len[k] - half - 1 : half;
                }
            }
#pragma unroll
            for (int k = 0; k < (int)kPartItems; ++k) {
                pid[k] = sj_pid_of(x[k], b[k], sk, nk, fan);
                const uint64_t p = e0 + (uint64_t)k * 64;
                if (p < m) pids[p] = pid[k];
            }
        } else {
#pragma unroll
            for (int k = 0; k < (int)kPartItems; ++k) {
                const uint64_t p = e0 + (uint64_t)k * 64;
                pid[k] = p < m ? pids[p] : 0u;
            }
        }
#pragma unroll
        for (int k = 0; k < (int)kPartItems; ++k)
            if (e0 + (uint64_t)k * 64 < m) atomicAdd(&cnt[sj_digit(pid[k], shift)], 1u);
        __syncthreads();
        if (tid < (int)kDigits) hist[(uint64_t)tid * nchunks + c] = cnt[tid];
        __syncthreads();
    }
}

// One stable partition pass by pid digit (pid >> shift) & 63; gofs holds
// the scanned digit-major counts of sj_hist_kernel for the same chunks.
// Moves keys and pids; with kPos also the input positions (pos_in null:
// the element's own index); with kDest stores dest_out[p] = output
// position of input p.
template <bool kPos, bool kDest>
__global__ __launch_bounds__(kBlock) void sj_scatter_kernel(
    const uint64_t* __restrict__ keys_in, const uint32_t* __restrict__ pids_in,
    const uint32_t* __restrict__ pos_in, const uint32_t* __restrict__ gofs, uint64_t m,
    uint32_t nchunks, uint32_t shift, uint64_t* __restrict__ keys_out,
    uint32_t* __restrict__ pids_out, uint32_t* __restrict__ pos_out,
    uint32_t* __restrict__ dest_out) {
    __shared__ uint64_t skey[kPartChunk];
    __shared__ uint32_t spid[kPartChunk];
    __shared__ uint32_t spos[kPos ? kPartChunk : 1];
    __shared__ uint32_t wbase[kWaves][kDigits];
    __shared__ uint32_t lstart[kDigits];
    __shared__ uint32_t gstart[kDigits];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    for (uint32_t c = blockIdx.x; c < nchunks; c += gridDim.x) {
        const uint64_t c0 = (uint64_t)c * kPartChunk;
        const uint32_t e0 = (uint32_t)wave * kWaveSpan + lane;
        uint64_t x[kPartItems];
        uint32_t b[kPartItems], rank[kPartItems], ps[kPartItems];
#pragma unroll
        for (int k = 0; k < (int)kPartItems; ++k) {
            const uint64_t p = c0 + e0 + (uint64_t)k * 64;
            const uint64_t q = p < m ? p : m - 1;
            x[k] = keys_in[q];
            b[k] = pids_in[q];
            if constexpr (kPos) ps[k] = pos_in ? pos_in[q] : (uint32_t)q;
        }
        uint32_t run = 0;
#pragma unroll
        for (int k = 0; k < (int)kPartItems; ++k) {
            const bool valid = c0 + e0 + (uint64_t)k * 64 < m;
            const uint32_t dg = sj_digit(b[k], shift);
            const uint64_t vb = __ballot(valid);
            uint64_t same = vb, mine = vb;
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
                const uint32_t dg = sj_digit(b[k], shift);
                const uint32_t lpos = wbase[wave][dg] + rank[k];
                skey[lpos] = x[k];
                spid[lpos] = b[k];
                if constexpr (kPos) spos[lpos] = ps[k];
                if constexpr (kDest) dest_out[p] = gstart[dg] + (lpos - lstart[dg]);
            }
        }
        __syncthreads();
        const uint32_t nvalid = m - c0 < kPartChunk ? (uint32_t)(m - c0) : kPartChunk;
        for (uint32_t lp = tid; lp < nvalid; lp += kBlock) {
            const uint32_t pid = spid[lp];
            const uint32_t dg = sj_digit(pid, shift);
            const uint32_t dst = gstart[dg] + (lp - lstart[dg]);
            keys_out[dst] = skey[lp];
            pids_out[dst] = pid;
            if constexpr (kPos) pos_out[dst] = spos[lp];
        }
        __syncthreads();
    }
}

// start[p] = first position of partition p in the pid-ordered R (p <= parts;
// start[parts] = n), from the sorted pids.
__global__ void sj_bounds_kernel(const uint32_t* __restrict__ pids, uint64_t n, uint32_t parts,
                                 uint32_t* __restrict__ start) {
    for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j <= n;
         j += (uint64_t)gridDim.x * blockDim.x) {
        const int64_t prev = j == 0 ? -1 : (int64_t)pids[j - 1];
        const int64_t cur = j == n ? (int64_t)parts : (int64_t)pids[j];
        for (int64_t p = prev + 1; p <= cur; ++p) start[p] = (uint32_t)j;
    }
}

// Compare-exchange (i, j), i < j, into ascending (key, position) order.
template <class K, class P>
__device__ inline void sj_cmpx(K* key, P* pos, uint32_t i, uint32_t j) {
    const uint64_t ki = key[i], kj = key[j];
    const uint32_t pi = pos[i], pj = pos[j];
    if (sj_greater(ki, pi, kj, pj)) {
        key[i] = kj;
        key[j] = ki;
        pos[i] = pj;
        pos[j] = pi;
    }
}

// Bitonic sort of key/pos[0..sz) by threads [0, nthreads): the network for
// the next power of two N, every comparator ascending (the first step of
// each stage compares mirrored elements), so that the elements past sz act
// as +infinity and every comparator reaching them can be skipped.
template <class K, class P>
__device__ void sj_bitonic(K* key, P* pos, uint32_t sz, uint32_t tid, uint32_t nthreads) {
    uint32_t N = 2;
    while (N < sz) N <<= 1;
    for (uint32_t k = 2; k <= N; k <<= 1) {
        const uint32_t h = k >> 1;
        for (uint32_t c = tid; c < N / 2; c += nthreads) {
            const uint32_t blk = c / h, off = c & (h - 1);
            const uint32_t i = blk * k + off, j = blk * k + k - 1 - off;
            if (j < sz) sj_cmpx(key, pos, i, j);
        }
        __syncthreads();
        for (uint32_t d = k >> 2; d > 0; d >>= 1) {
            for (uint32_t c = tid; c < N / 2; c += nthreads) {
                const uint32_t i = 2 * c - (c & (d - 1)), j = i + d;
                if (j < sz) sj_cmpx(key, pos, i, j);
            }
            __syncthreads();
        }
    }
}

// Wave sort of up to 64 * E (key, position) elements in registers: lane L
// holds elements L * E .. L * E + E - 1, padded past sz with (~0, ~0), which
// orders after every real element (positions are below 2^31).  The same
// all-ascending bitonic network as sj_bitonic: comparators closer than E
// elements are register exchanges, the others a cross-lane shuffle (the
// lower element of each pair keeps the minimum, the upper the maximum).
__device__ inline bool sj_less(uint64_t ka, uint32_t pa, uint64_t kb, uint32_t pb) {
    return ka < kb || (ka == kb && pa < pb);
}

template <int E>
__device__ void sj_sort_wave(uint64_t* __restrict__ keys, uint32_t* __restrict__ pos,
                             uint32_t sz, uint32_t lane, uint32_t a, uint64_t* __restrict__ rs) {
    uint64_t k[E];
    uint32_t p[E];
#pragma unroll
    for (int r = 0; r < E; ++r) {
        const uint32_t e = lane * E + r;
        k[r] = e < sz ? keys[e] : ~0ull;
        p[r] = e < sz ? pos[e] : ~0u;
    }
    // Register comparator (i, j), i < j: ascending.
    auto cx = [&](int i, int j) {
        if (sj_less(k[j], p[j], k[i], p[i])) {
            const uint64_t tk = k[i];
            const uint32_t tp = p[i];
            k[i] = k[j];
            p[i] = p[j];
            k[j] = tk;
            p[j] = tp;
        }
    };
    // Element r against the partner lane's element (the lower lane keeps the
    // minimum).
    auto keep = [&](int r, uint64_t ok, uint32_t op, bool lower) {
        const bool take = lower ? sj_less(ok, op, k[r], p[r]) : sj_less(k[r], p[r], ok, op);
        k[r] = take ? ok : k[r];
        p[r] = take ? op : p[r];
    };
    // Register half-cleaners at distances E/2 .. 1.
    auto local_cleaners = [&]() {
#pragma unroll
        for (int d = E / 2; d > 0; d >>= 1) {
#pragma unroll
            for (int r = 0; r < E; ++r)
                if ((r & d) == 0) cx(r, r | d);
        }
    };
    // Stages up to E: inside each lane.
#pragma unroll
    for (int st = 2; st <= E; st <<= 1) {
#pragma unroll
        for (int r = 0; r < E; ++r) {
            const int r2 = r ^ (st - 1);
            if (r < r2) cx(r, r2);
        }
#pragma unroll
        for (int d = st >> 2; d > 0; d >>= 1) {
#pragma unroll
            for (int r = 0; r < E; ++r)
                if ((r & d) == 0) cx(r, r | d);
        }
    }
    // Stages beyond E: the mirror step and the half-cleaners down to E
    // across lanes, then the rest in registers.
    constexpr uint32_t N = 64u * E;
#pragma unroll 1
    for (uint32_t st = 2 * E; st <= N; st <<= 1) {
        {
            const int src = (int)(lane ^ (st / E - 1));
            const bool lower = (lane & (st / (2 * E))) == 0;
#pragma unroll
            for (int r = 0; r < E / 2; ++r) {
                const int r2 = E - 1 - r;
                const uint64_t ka = __shfl(k[r2], src, 64), kb = __shfl(k[r], src, 64);
                const uint32_t pa = __shfl(p[r2], src, 64), pb = __shfl(p[r], src, 64);
                keep(r, ka, pa, lower);
                keep(r2, kb, pb, lower);
            }
            if constexpr (E == 1) {
                const uint64_t ka = __shfl(k[0], src, 64);
                const uint32_t pa = __shfl(p[0], src, 64);
                keep(0, ka, pa, lower);
            }
        }
#pragma unroll 1
        for (uint32_t d = st >> 2; d >= (uint32_t)E; d >>= 1) {
            const int src = (int)(lane ^ (d / E));
            const bool lower = (lane & (d / E)) == 0;
#pragma unroll
            for (int r = 0; r < E; ++r) {
                const uint64_t ok = __shfl(k[r], src, 64);
                const uint32_t op = __shfl(p[r], src, 64);
                keep(r, ok, op, lower);
            }
        }
        local_cleaners();
    }
#pragma unroll
    for (int r = 0; r < E; ++r) {
        const uint32_t e = lane * E + r;
        if (e < sz) {
            keys[e] = k[r];
            pos[e] = p[r];
            if ((a + e) % kLineKeys == 0) rs[(a + e) / kLineKeys] = k[r];
        }
    }
}

// One wave per partition of kLo + 1 .. kHi keys (kHi <= 1024, or the
// 2048-key sort alone: its 32 elements per lane need about twice the
// registers, which would halve the occupancy of the smaller sorts).  Every
// sort also writes the line samples rs[j] = sorted key kLineKeys * j of its
// partition (the kLo = 0 launch those of one-key partitions too).
constexpr uint32_t kSjWaveCap = 2048;
template <uint32_t kLo, uint32_t kHi>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(kHi > 1024 ? 3 : 5)))
void sj_sort_wave_kernel(uint64_t* __restrict__ keys,
                                                              uint32_t* __restrict__ pos,
                                                              const uint32_t* __restrict__ start,
                                                              uint32_t parts,
                                                              uint64_t* __restrict__ rs) {
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t waves = gridDim.x * (kBlock / 64);
    for (uint32_t p = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6); p < parts; p += waves) {
        const uint32_t a = start[p], sz = start[p + 1] - a;
        if (sz <= kLo || sz > kHi || sz == 0) continue;
        if constexpr (kHi > 1024) {
            sj_sort_wave<32>(keys + a, pos + a, sz, lane, a, rs);
        } else {
            if (sz == 1) {
                if (lane == 0 && a % kLineKeys == 0) rs[a / kLineKeys] = keys[a];
            } else if (sz <= 64) {
                sj_sort_wave<1>(keys + a, pos + a, sz, lane, a, rs);
            } else if (sz <= 128) {
                sj_sort_wave<2>(keys + a, pos + a, sz, lane, a, rs);
            } else if (sz <= 256) {
                sj_sort_wave<4>(keys + a, pos + a, sz, lane, a, rs);
            } else if (sz <= 512) {
                sj_sort_wave<8>(keys + a, pos + a, sz, lane, a, rs);
            } else {
                sj_sort_wave<16>(keys + a, pos + a, sz, lane, a, rs);
            }
        }
    }
}

// Sort every partition of kSjWaveCap + 1 .. kSjSortCap keys in LDS; queue
// the larger ones for sj_sort_big_kernel.
__global__ __launch_bounds__(kBlock) void sj_sort_kernel(uint64_t* __restrict__ keys,
                                                         uint32_t* __restrict__ pos,
                                                         const uint32_t* __restrict__ start,
                                                         uint32_t parts,
                                                         uint32_t* __restrict__ big,
                                                         uint64_t* __restrict__ rs) {
    __shared__ uint64_t sk[kSjSortCap];
    __shared__ uint32_t sp[kSjSortCap];
    const uint32_t tid = threadIdx.x;
    for (uint32_t p = blockIdx.x; p < parts; p += gridDim.x) {
        const uint32_t a = start[p], sz = start[p + 1] - a;
        if (sz <= kSjWaveCap) continue;
        if (sz > kSjSortCap) {
            if (tid == 0) big[1 + atomicAdd(&big[0], 1u)] = p;
            continue;
        }
        for (uint32_t i = tid; i < sz; i += kBlock) {
            sk[i] = keys[a + i];
            sp[i] = pos[a + i];
        }
        __syncthreads();
        sj_bitonic(sk, sp, sz, tid, kBlock);
        for (uint32_t i = tid; i < sz; i += kBlock) {
            keys[a + i] = sk[i];
            pos[a + i] = sp[i];
            if ((a + i) % kLineKeys == 0) rs[(a + i) / kLineKeys] = sk[i];
        }
        __syncthreads();
    }
}

// Partitions larger than kSjSortCap: one block of kBigThreads each, in LDS
// up to kBigCap keys, else in global memory; a partition already in (key,
// position) order (e.g. one repeated key, kept in input order by the stable
// passes) is left as is.
constexpr uint32_t kBigCap = 10240;
__global__ __launch_bounds__(kBigThreads) void sj_sort_big_kernel(
    uint64_t* __restrict__ keys, uint32_t* __restrict__ pos,
    const uint32_t* __restrict__ start, const uint32_t* __restrict__ big,
    uint64_t* __restrict__ rs) {
    __shared__ uint64_t sk[kBigCap];
    __shared__ uint32_t sp[kBigCap];
    __shared__ int unsorted;
    const uint32_t tid = threadIdx.x;
    const uint32_t nbig = big[0];
    for (uint32_t q = blockIdx.x; q < nbig; q += gridDim.x) {
        const uint32_t p = big[1 + q];
        const uint32_t a = start[p], sz = start[p + 1] - a;
        if (tid == 0) unsorted = 0;
        __syncthreads();
        int mine = 0;
        for (uint32_t i = tid + 1; i < sz; i += kBigThreads)
            mine |= sj_greater(keys[a + i - 1], pos[a + i - 1], keys[a + i], pos[a + i]) ? 1 : 0;
        if (mine) atomicOr(&unsorted, 1);
        __syncthreads();
        const bool work = unsorted != 0;
        __syncthreads();
        if (work && sz <= kBigCap) {
            for (uint32_t i = tid; i < sz; i += kBigThreads) {
                sk[i] = keys[a + i];
                sp[i] = pos[a + i];
            }
            __syncthreads();
            sj_bitonic(sk, sp, sz, tid, kBigThreads);
            for (uint32_t i = tid; i < sz; i += kBigThreads) {
                keys[a + i] = sk[i];
                pos[a + i] = sp[i];
                if ((a + i) % kLineKeys == 0) rs[(a + i) / kLineKeys] = sk[i];
            }
        } else {
            if (work) sj_bitonic(keys + a, pos + a, sz, tid, kBigThreads);
            for (uint32_t i = (kLineKeys - a % kLineKeys) % kLineKeys + tid * kLineKeys; i < sz;
                 i += kBigThreads * kLineKeys)
                rs[(a + i) / kLineKeys] = keys[a + i];
        }
        __syncthreads();
    }
}

// Join: S in coarse pid order, each key's run found by lower and upper
// bound inside its own partition of the sorted R; res[q] = v | run length
// << 32 in the same order as the keys, where v is the input position in R
// of a single match (read here, where that part of R is in cache), or
// kSortedPos | the first sorted position of a longer run (then *runs is
// set, and the emitted positions are mapped afterwards).  Blocks are
// mapped XCD-contiguously so that one XCD's L2 serves neighbouring
// partitions.
constexpr uint32_t kSortedPos = 0x80000000u;
__global__ __launch_bounds__(kBlock) void sj_join_kernel(
    const uint64_t* __restrict__ sk, const uint32_t* __restrict__ spid, uint64_t m,
    const uint64_t* __restrict__ rk, const uint64_t* __restrict__ rs,
    const uint32_t* __restrict__ rpos,
    const uint32_t* __restrict__ rstart, uint32_t ntiles, uint32_t tiles_per_xcd,
    uint64_t* __restrict__ res, uint32_t* __restrict__ runs) {
    const uint32_t tile = (blockIdx.x % kXcds) * tiles_per_xcd + blockIdx.x / kXcds;
    if (tile >= ntiles) return;
    const uint64_t base = (uint64_t)tile * kBlock * kJoinItems + threadIdx.x;
    uint64_t x[kJoinItems];
    uint32_t b[kJoinItems], len[kJoinItems], hi[kJoinItems];
#pragma unroll
    for (int k = 0; k < kJoinItems; ++k) {
        const uint64_t q = base + (uint64_t)k * kBlock;
        const bool v = q < m;
        x[k] = v ? sk[q] : 0;
        const uint32_t p = v ? spid[q] : 0;
        b[k] = v ? rstart[p] : 0;
        hi[k] = v ? rstart[p + 1] : 0;
        len[k] = hi[k] - b[k];
    }
    // Lower bound in two lockstep stages: over the line samples
    // rs[j] = rk[kLineKeys * j] that fall in the partition, then inside the
    // one line that holds the bound.
    uint32_t lim[kJoinItems];
#pragma unroll
    for (int k = 0; k < kJoinItems; ++k) {
        const uint32_t j0 = (b[k] + kLineKeys - 1) / kLineKeys;
        lim[k] = j0;  // first sample of the partition
        len[k] = (hi[k] + kLineKeys - 1) / kLineKeys - j0;
    }
    uint32_t c[kJoinItems];
#pragma unroll
    for (int k = 0; k < kJoinItems; ++k) c[k] = lim[k];
    for (;;) {
        uint32_t act = 0;
#pragma unroll
        for (int k = 0; k < kJoinItems; ++k) act |= len[k];
        if (!act) break;
#pragma unroll
        for (int k = 0; k < kJoinItems; ++k) {
            if (len[k]) {
                const uint32_t half = len[k] >> 1, at = c[k] + half;
                if (rs[at] < x[k]) {
                    c[k] = at + 1;
                    len[k] -= half + 1;
                } else {
                    len[k] = half;
                }
            }
        }
    }
    // rk[kLineKeys * (c - 1)] < x <= rk[kLineKeys * c] (where those are in
    // the partition): the bound is in [kLineKeys * (c - 1) + 1, kLineKeys * c].
#pragma unroll
    for (int k = 0; k < kJoinItems; ++k) {
        const uint32_t end = min(hi[k], c[k] * kLineKeys);
        b[k] = c[k] > lim[k] ? (c[k] - 1) * kLineKeys + 1 : b[k];
        len[k] = end - b[k];
    }
    for (;;) {
        uint32_t act = 0;
#pragma unroll
        for (int k = 0; k < kJoinItems; ++k) act |= len[k];
        if (!act) break;
#pragma unroll
        for (int k = 0; k < kJoinItems; ++k) {
            if (len[k]) {
                const uint32_t half = len[k] >> 1, at = b[k] + half;
                if (rk[at] < x[k]) {
                    b[k] = at + 1;
                    len[k] -= half + 1;
                } else {
                    len[k] = half;
                }
            }
        }
    }
    // Run end: usually the next key already differs; else an upper bound.
    uint32_t e[kJoinItems];
#pragma unroll
    for (int k = 0; k < kJoinItems; ++k) {
        const bool hit = b[k] < hi[k] && rk[b[k]] == x[k];
        e[k] = hit ? b[k] + 1 : b[k];
        len[k] = 0;
        if (hit && e[k] < hi[k] && rk[e[k]] == x[k]) {
            e[k] += 1;
            len[k] = hi[k] - e[k];
        }
    }
    for (;;) {
        uint32_t act = 0;
#pragma unroll
        for (int k = 0; k < kJoinItems; ++k) act |= len[k];
        if (!act) break;
#pragma unroll
        for (int k = 0; k < kJoinItems; ++k) {
            if (len[k]) {
                const uint32_t half = len[k] >> 1, at = e[k] + half;
                if (rk[at] <= x[k]) {
                    e[k] = at + 1;
                    len[k] -= half + 1;
                } else {
                    len[k] = half;
                }
            }
        }
    }
    bool longer = false;
#pragma unroll
    for (int k = 0; k < kJoinItems; ++k) {
        const uint64_t q = base + (uint64_t)k * kBlock;
        const uint32_t c = e[k] - b[k];
        uint32_t v = b[k] | kSortedPos;
        if (c == 1) v = rpos[b[k]];
        longer |= q < m && c > 1;
        if (q < m) res[q] = (uint64_t)v | ((uint64_t)c << 32);
    }
    if (__ballot(longer) && (threadIdx.x & 63) == 0) atomicOr(runs, 1u);
}

// Pairs of runs longer than one were emitted with kSortedPos | sorted
// position: map those to R's input positions (written pairs only:
// min(total, cap)); nothing to do unless the join saw such a run.
__global__ void sj_map_kernel(lj_pair* __restrict__ out, uint64_t cap,
                              const uint64_t* __restrict__ count,
                              const uint32_t* __restrict__ runs,
                              const uint32_t* __restrict__ rpos, uint64_t n) {
    if (*runs == 0) return;
    const uint64_t c = *count, lim = c < cap ? c : cap;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < lim;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t r = out[i].r_idx;
        if ((r & kSortedPos) && (r & ~kSortedPos) < n) out[i].r_idx = rpos[r & ~kSortedPos];
    }
}

// Emission from the per-key results in S order (res[q] = v | run length
// << 32), one chunk of kPartChunk keys per block, the chunk's first output
// rank from the scanned per-chunk pair counts; pairs in (s_idx, r_idx)
// order, those of rank >= cap not written.  Without runs longer than one
// (*runs == 0, every R key distinct among the matches) each key emits at
// most one pair, placed by wave ballots; otherwise the chunk's counts are
// scanned in LDS and the pairs emitted by a load-balanced loop, a run's
// k-th pair at v + k.
__global__ __launch_bounds__(kBlock) void sj_emit_kernel(const uint64_t* __restrict__ res,
                                                         uint64_t m,
                                                         const uint64_t* __restrict__ offs,
                                                         lj_pair* __restrict__ out, uint64_t cap,
                                                         const uint32_t* __restrict__ runs) {
    constexpr int kItems = (int)kPartItems;
    __shared__ uint32_t wsum[kItems * kWaves];
    __shared__ uint64_t off[kPartChunk + 1];
    __shared__ uint32_t j0[kPartChunk];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint64_t base = (uint64_t)blockIdx.x * kPartChunk;
    const uint64_t excl = offs[blockIdx.x];
    if (excl >= cap) return;
    uint32_t v[kItems], c[kItems];
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        const uint64_t q = base + (uint64_t)k * kBlock + tid;
        const uint64_t r = q < m ? res[q] : 0ull;
        v[k] = (uint32_t)r;
        c[k] = (uint32_t)(r >> 32);
    }
    if (*runs == 0) {
        const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
        uint32_t lo[kItems];
#pragma unroll
        for (int k = 0; k < kItems; ++k) {
            const uint64_t mask = __ballot(c[k] != 0);
            lo[k] = (uint32_t)__popcll(mask & lt);
            if (lane == 0) wsum[k * kWaves + wave] = (uint32_t)__popcll(mask);
        }
        __syncthreads();
        uint64_t pre = 0;
#pragma unroll
        for (int k = 0; k < kItems; ++k) {
            uint32_t wpre = 0;
            for (int w = 0; w < wave; ++w) wpre += wsum[k * kWaves + w];
            const uint64_t at = excl + pre + wpre + lo[k];
            if (c[k] && at < cap) {
                lj_pair p;
                p.s_idx = (uint32_t)(base + (uint64_t)k * kBlock + tid);
                p.r_idx = v[k];
                out[at] = p;
            }
#pragma unroll
            for (int w = 0; w < kWaves; ++w) pre += wsum[k * kWaves + w];
        }
        return;
    }
    // Chunk order i = k * kBlock + tid: exclusive prefix of the counts.
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        off[k * kBlock + tid] = c[k];
        j0[k * kBlock + tid] = v[k];
    }
    __syncthreads();
    uint64_t loc[kItems], tsum = 0;
#pragma unroll
    for (int i = 0; i < kItems; ++i) {
        loc[i] = tsum;
        tsum += off[tid * kItems + i];
    }
    const uint64_t incl = wave_incl_scan(tsum, lane);
    __shared__ uint64_t wtot[kWaves];
    if (lane == 63) wtot[wave] = incl;
    __syncthreads();
    uint64_t wpre = 0, total = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
        wpre += w < wave ? wtot[w] : 0;
        total += wtot[w];
    }
    const uint64_t texcl = wpre + incl - tsum;
#pragma unroll
    for (int i = 0; i < kItems; ++i) off[tid * kItems + i] = texcl + loc[i];
    if (tid == 0) off[kPartChunk] = total;
    __syncthreads();
    const uint64_t limit = cap - excl < total ? cap - excl : total;
    for (uint64_t o = tid; o < limit; o += kBlock) {
        int a = 0, b = (int)kPartChunk;  // off[kPartChunk] = total > o
        while (b - a > 1) {
            const int mid = (a + b) >> 1;
            if (off[mid] <= o) a = mid;
            else b = mid;
        }
        lj_pair p;
        p.s_idx = (uint32_t)(base + (uint64_t)a);
        p.r_idx = j0[a] + (uint32_t)(o - off[a]);
        out[excl + o] = p;
    }
}

// Total pair count, or UINT64_MAX after a wait error.
__global__ void sj_finish_kernel(const uint64_t* total, const uint32_t* err, uint64_t* count) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *count = *err ? ~0ull : *total;
}

unsigned grid_of(uint64_t items, uint64_t cap) {
    return (unsigned)(items == 0 ? 1 : items < cap ? items : cap);
}

// One relation into pid order: pids from the model, then one stable pass
// per digit from `shift0` up.  Pass k reads the previous pass's output.
struct PassBufs {
    const uint64_t* keys_in;
    uint64_t* keys[2];
    uint32_t* pids[2];
    uint32_t* pos[2];   // null: no positions carried
    uint32_t* dest[2];  // null: no destinations stored
    uint64_t* keys_last;
    uint32_t* pos_last;
};

hipError_t partition_passes(const PassBufs& B, uint64_t n, uint32_t npass, uint32_t shift0,
                            const SortJoinWs& L, char* w, uint32_t* hist, uint32_t st0,
                            uint32_t ctr0, hipStream_t stream) {
    const uint32_t nchunks = (uint32_t)num_tiles(n, kPartChunk);
    const uint64_t nh = (uint64_t)kDigits * nchunks;
    uint32_t* ctr = (uint32_t*)(w + L.scan_ctr);
    uint32_t* err = &((WsHeader*)w)->err;
    const uint64_t* knots = (const uint64_t*)(w + L.knots);
    const uint16_t* kb_lo = (const uint16_t*)(w + L.kb_lo);
    for (uint32_t k = 0; k < npass; ++k) {
        const uint32_t shift = shift0 + k * kDigitBits;
        uint32_t* pin = B.pids[k & 1];
        if (k == 0)
            hipLaunchKernelGGL(sj_hist_kernel<true>, dim3(grid_of(nchunks, 2048)), dim3(kBlock),
                               0, stream, B.keys_in, knots, kb_lo, L.nk, L.fan, pin, n, nchunks,
                               shift, hist);
        else
            hipLaunchKernelGGL(sj_hist_kernel<false>, dim3(grid_of(nchunks, 4096)),
                               dim3(kBlock), 0, stream, (const uint64_t*)nullptr,
                               (const uint64_t*)nullptr, (const uint16_t*)nullptr, 0u, 1u, pin,
                               n, nchunks, shift, hist);
        hipError_t e = launch_scan_u32(hist, nh, (uint64_t*)(w + L.scan_st[st0 + k]),
                                       ctr + ctr0 + k, err, stream);
        if (e != hipSuccess) return e;
        const uint64_t* kin = k == 0 ? B.keys_in : B.keys[(k - 1) & 1];
        const bool last = k + 1 == npass;
        uint64_t* kout = last && B.keys_last ? B.keys_last : B.keys[k & 1];
        uint32_t* pout = B.pos[0] ? (last && B.pos_last ? B.pos_last : B.pos[k & 1]) : nullptr;
        const uint32_t* posin = k == 0 || !B.pos[0] ? nullptr : B.pos[(k - 1) & 1];
        uint32_t* pidout = B.pids[(k + 1) & 1];
        const dim3 grid(grid_of(nchunks, 65535)), block(kBlock);
        if (B.pos[0])
            hipLaunchKernelGGL((sj_scatter_kernel<true, false>), grid, block, 0, stream, kin, pin,
                               posin, (const uint32_t*)hist, n, nchunks, shift, kout, pidout,
                               pout, (uint32_t*)nullptr);
        else
            hipLaunchKernelGGL((sj_scatter_kernel<false, true>), grid, block, 0, stream, kin, pin,
                               (const uint32_t*)nullptr, (const uint32_t*)hist, n, nchunks,
                               shift, kout, pidout, (uint32_t*)nullptr, B.dest[k & 1]);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Model, partition passes, partition starts and sorts of R: the sorted keys
// and their input positions end in (keys_out, pos_out), the partition
// starts and the line samples in the workspace.
hipError_t learned_sort(const uint64_t* keys, uint64_t n, uint64_t* keys_out, uint32_t* pos_out,
                        char* w, const SortJoinWs& L, hipStream_t stream) {
    hipLaunchKernelGGL(sj_model_kernel, dim3(1), dim3(kModelThreads), 0, stream, keys, n, L.ns,
                       L.nk, (uint64_t*)(w + L.knots), (uint16_t*)(w + L.kb_lo));
    PassBufs B{};
    B.keys_in = keys;
    for (int k = 0; k < 2; ++k) {
        B.keys[k] = (uint64_t*)(w + L.r_keys[k]);
        B.pids[k] = (uint32_t*)(w + L.r_bins[k]);
        B.pos[k] = (uint32_t*)(w + L.r_pos[k]);
    }
    B.keys_last = keys_out;
    B.pos_last = pos_out;
    hipError_t e = partition_passes(B, n, L.rpasses, 0, L, w, (uint32_t*)(w + L.r_hist), 0, 0,
                                    stream);
    if (e != hipSuccess) return e;
    const uint32_t* pids = B.pids[L.rpasses & 1];
    uint32_t* start = (uint32_t*)(w + L.r_start);
    hipLaunchKernelGGL(sj_bounds_kernel, dim3(grid_of(num_tiles(n + 1, kBlock), 8192)),
                       dim3(kBlock), 0, stream, pids, n, L.parts, start);
    uint32_t* big = (uint32_t*)(w + L.big_queue);
    uint64_t* rs = (uint64_t*)(w + L.r_rs);
    const dim3 wgrid(grid_of(num_tiles(L.parts, kBlock / 64), 16384));
    hipLaunchKernelGGL((sj_sort_wave_kernel<0, 1024>), wgrid, dim3(kBlock), 0, stream, keys_out,
                       pos_out, (const uint32_t*)start, L.parts, rs);
    hipLaunchKernelGGL((sj_sort_wave_kernel<1024, kSjWaveCap>), wgrid, dim3(kBlock), 0, stream,
                       keys_out, pos_out, (const uint32_t*)start, L.parts, rs);
    hipLaunchKernelGGL(sj_sort_kernel, dim3(grid_of(L.parts, 16384)), dim3(kBlock), 0, stream,
                       keys_out, pos_out, (const uint32_t*)start, L.parts, big, rs);
    hipLaunchKernelGGL(sj_sort_big_kernel, dim3(256), dim3(kBigThreads), 0, stream, keys_out,
                       pos_out, (const uint32_t*)start, (const uint32_t*)big, rs);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_learned_sort(const uint64_t* keys, uint64_t n, uint64_t* keys_out,
                               uint32_t* pos_out, void* ws, const SortJoinWs& L,
                               hipStream_t stream) {
    if (n == 0) return hipSuccess;
    char* w = (char*)ws;
    hipError_t e = launch_zero_words((uint64_t*)ws, L.ctrl_bytes / 8, stream);
    if (e != hipSuccess) return e;
    uint64_t* ko = keys_out ? keys_out : (uint64_t*)(w + L.r_keys[(L.rpasses - 1) & 1]);
    uint32_t* po = pos_out ? pos_out : (uint32_t*)(w + L.r_pos[(L.rpasses - 1) & 1]);
    return learned_sort(keys, n, ko, po, w, L, stream);
}

hipError_t launch_sort_join(const uint64_t* r, uint64_t n, const uint64_t* s, uint64_t m,
                            lj_pair* out, uint64_t cap, uint64_t* count_dev, void* ws,
                            hipStream_t stream, hipEvent_t ev0, hipEvent_t ev1) {
    if (n == 0 || m == 0) return launch_set_u64(count_dev, 0, stream);
    const SortJoinWs L = sort_join_ws(n, m);
    char* w = (char*)ws;
    hipError_t e = launch_zero_words((uint64_t*)ws, L.ctrl_bytes / 8, stream);
    if (e != hipSuccess) return e;
    // Sorted R in the workspace buffers of its last pass.
    uint64_t* rk = (uint64_t*)(w + L.r_keys[(L.rpasses - 1) & 1]);
    uint32_t* rp = (uint32_t*)(w + L.r_pos[(L.rpasses - 1) & 1]);
    e = learned_sort(r, n, rk, rp, w, L, stream);
    if (e != hipSuccess) return e;

    // S into coarse pid order (two passes over the pid's high digits).
    PassBufs B{};
    B.keys_in = s;
    for (int k = 0; k < 2; ++k) {
        B.keys[k] = (uint64_t*)(w + L.s_keys[k]);
        B.pids[k] = (uint32_t*)(w + L.s_bins[k]);
        B.dest[k] = (uint32_t*)(w + L.s_dest[k]);
    }
    e = partition_passes(B, m, L.spasses, L.s_shift, L, w, (uint32_t*)(w + L.s_hist),
                         kSjMaxPasses, kSjMaxPasses, stream);
    if (e != hipSuccess) return e;
    const uint64_t* sk = B.keys[1];
    const uint32_t* spid = B.pids[0];
    uint64_t* res2 = B.keys[0];  // dead after pass 2
    uint64_t* res1 = B.keys[1];  // dead after the join
    uint64_t* res0 = B.keys[0];  // res2 dead after the first put-back

    if (ev0) {
        e = hipEventRecord(ev0, stream);
        if (e != hipSuccess) return e;
    }
    const uint32_t ntiles = (uint32_t)num_tiles(m, (uint64_t)kBlock * kJoinItems);
    const uint32_t tpx = (uint32_t)num_tiles(ntiles, kXcds);
    uint32_t* runs = (uint32_t*)(w + L.big_queue) + 1 + L.parts;
    const uint64_t* rs = (const uint64_t*)(w + L.r_rs);  // written by the sort
    hipLaunchKernelGGL(sj_join_kernel, dim3(tpx * kXcds), dim3(kBlock), 0, stream, sk, spid, m,
                       (const uint64_t*)rk, (const uint64_t*)rs, (const uint32_t*)rp,
                       (const uint32_t*)(w + L.r_start), ntiles, tpx, res2, runs);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (ev1) {
        e = hipEventRecord(ev1, stream);
        if (e != hipSuccess) return e;
    }

    // Put the runs back in S order (pass 2, then pass 1), count per chunk,
    // emit, map positions.
    e = launch_unpermute(B.dest[1], res2, res1, m, true, stream);
    if (e != hipSuccess) return e;
    BinnedWs U{};
    U.scan_ctr = L.scan_ctr + 32;  // its counter: word 2 from here
    U.scan_st3 = L.scan_st[kSjMaxPasses + 2];
    U.counts = L.counts;
    e = launch_unpermute_count(B.dest[0], res1, res0, m, true, ws, U, stream);
    if (e != hipSuccess) return e;
    const uint64_t* offs = (const uint64_t*)(w + L.counts);
    const uint32_t nemit = (uint32_t)num_tiles(m, kPartChunk);
    if (out && cap)
        hipLaunchKernelGGL(sj_emit_kernel, dim3(nemit), dim3(kBlock), 0, stream,
                           (const uint64_t*)res0, m, offs, out, cap, (const uint32_t*)runs);
    hipLaunchKernelGGL(sj_finish_kernel, dim3(1), dim3(64), 0, stream, offs + nemit,
                       (const uint32_t*)&((WsHeader*)ws)->err, count_dev);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (out && cap)
        hipLaunchKernelGGL(sj_map_kernel, dim3(4096), dim3(kBlock), 0, stream, out, cap,
                           (const uint64_t*)count_dev, (const uint32_t*)runs,
                           (const uint32_t*)rp, n);
    return hipGetLastError();
}

}  // namespace lj
