/*
 * Seeded, counter-based random draws for the synthetic join workloads.
 *
 * This file holds no join or index arithmetic: it only turns (stream key,
 * counter) pairs into random numbers, so that the same inputs can be fed to
 * the CPU oracle and to the GPU library.  Every draw is a pure function of
 * its key and counter, so results do not depend on the thread count.
 *
 * Generators used:
 *   - SplitMix64 (Steele, Lea, Flood, "Fast splittable pseudorandom number
 *     generators", OOPSLA 2014): the i-th output of a SplitMix64 stream
 *     started at state k is mix(k + (i+1)*gamma).
 *   - Box-Muller transform for normal deviates.
 *   - Rejection-inversion for the bounded Zipf law (Hormann and Derflinger,
 *     "Rejection-inversion to generate variates from monotone discrete
 *     distributions", ACM TOMACS 1996), specialised to exponent 1.
 *   - A 4-round Feistel network with cycle walking as a keyed bijection on
 *     [0, N) (Black and Rogaway, "Ciphers with arbitrary finite domains",
 *     CT-RSA 2002), used for shuffles and rank scattering.
 */
#include <math.h>
#include <stdint.h>
#include <stddef.h>

#define GAMMA 0x9e3779b97f4a7c15ULL

static inline uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

/* i-th output of the SplitMix64 stream whose state starts at `key`. */
static inline uint64_t draw(uint64_t key, uint64_t i) {
    return mix64(key + (i + 1) * GAMMA);
}

/* Uniform double in (0, 1]: 53 random bits, never zero. */
static inline double unit_open0(uint64_t v) {
    return ((double)(v >> 11) + 1.0) * 0x1.0p-53;
}

/* Uniform double in [0, 1). */
static inline double unit(uint64_t v) {
    return (double)(v >> 11) * 0x1.0p-53;
}

/* Derive a sub-stream key from a seed and a stream label. */
uint64_t wl_stream_key(uint64_t seed, uint64_t label) {
    return mix64(seed ^ mix64(label + GAMMA));
}

/* out[i] = draw(key, start + i) >> shift. */
void wl_draw_u64(uint64_t key, uint64_t start, uint64_t count, uint32_t shift,
                 uint64_t *out) {
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < (int64_t)count; ++i)
        out[i] = draw(key, start + (uint64_t)i) >> shift;
}

/* out[i] = lo + (draw(key, start+i) mod span), span > 0 (64-bit modulo bias
 * is below 2^-40 for the spans used here). */
void wl_draw_range(uint64_t key, uint64_t start, uint64_t count, uint64_t lo,
                   uint64_t span, uint64_t *out) {
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < (int64_t)count; ++i)
        out[i] = lo + draw(key, start + (uint64_t)i) % span;
}

/* out[i] = 1 if the uniform [0,1) draw for counter start+i is below p. */
void wl_draw_bernoulli(uint64_t key, uint64_t start, uint64_t count, double p,
                       uint8_t *out) {
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < (int64_t)count; ++i)
        out[i] = unit(draw(key, start + (uint64_t)i)) < p;
}

/* Lognormal deviates exp(mu + sigma*z), z standard normal by Box-Muller on
 * the draws 2c and 2c+1 of counter c = start + i. */
void wl_draw_lognormal(uint64_t key, uint64_t start, uint64_t count, double mu,
                       double sigma, double *out) {
    const double two_pi = 6.283185307179586476925286766559;
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < (int64_t)count; ++i) {
        uint64_t c = start + (uint64_t)i;
        double u1 = unit_open0(draw(key, 2 * c));
        double u2 = unit(draw(key, 2 * c + 1));
        double z = sqrt(-2.0 * log(u1)) * cos(two_pi * u2);
        out[i] = exp(mu + sigma * z);
    }
}

/* key = min(2^63 - 1, floor(v / vmax * 2^63)). */
void wl_scale_to_u63(const double *v, uint64_t count, double vmax,
                     uint64_t *out) {
    const double top = 9223372036854775808.0; /* 2^63 */
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < (int64_t)count; ++i) {
        double s = floor(v[i] / vmax * top);
        if (!(s >= 0.0)) s = 0.0;
        out[i] = (s >= top) ? 0x7fffffffffffffffULL : (uint64_t)s;
    }
}

/*
 * Bounded Zipf law on ranks 1..nmax with exponent 1: P(k) proportional to
 * 1/k.  Rejection-inversion with hat h(x) = 1/x, whose integral is
 * H(x) = ln x and inverse H^-1(u) = e^u.  Attempt a for sample c uses the
 * uniform draw(wl_stream_key(key, a), c), so every sample is a pure
 * function of (key, c).
 */
void wl_draw_zipf1(uint64_t key, uint64_t start, uint64_t count, uint64_t nmax,
                   uint64_t *out) {
    const double hx1 = log(1.5) - 1.0;          /* H(1.5) - h(1)          */
    const double hn = log((double)nmax + 0.5);  /* H(nmax + 0.5)          */
    const double squeeze = 2.0 - exp(log(2.5) - 0.5); /* 2 - H^-1(H(2.5) - h(2)) */
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < (int64_t)count; ++i) {
        uint64_t c = start + (uint64_t)i;
        uint64_t k = 1;
        for (uint64_t a = 0;; ++a) {
            double u = hn + unit(draw(wl_stream_key(key, a), c)) * (hx1 - hn);
            double x = exp(u);
            double kd = floor(x + 0.5);
            if (kd < 1.0) kd = 1.0;
            if (kd > (double)nmax) kd = (double)nmax;
            k = (uint64_t)kd;
            if (kd - x <= squeeze || u >= log(kd + 0.5) - 1.0 / kd) break;
        }
        out[i] = k;
    }
}

/* Keyed bijection on [0, n): 4 Feistel rounds on an even number of bits
 * b >= 2 with 2^b >= n, cycle-walked until the image falls below n. */
static inline uint64_t feistel(uint64_t x, uint64_t n, uint32_t half,
                               uint64_t mask, const uint64_t rk[4]) {
    do {
        uint64_t l = x >> half, r = x & mask;
        for (int round = 0; round < 4; ++round) {
            uint64_t t = r;
            r = l ^ (mix64(rk[round] ^ r) & mask);
            l = t;
        }
        x = (l << half) | r;
    } while (x >= n);
    return x;
}

static void feistel_setup(uint64_t key, uint64_t n, uint32_t *half,
                          uint64_t *mask, uint64_t rk[4]) {
    uint32_t bits = 2;
    while (bits < 64 && (1ULL << bits) < n) bits += 2;
    *half = bits / 2;
    *mask = (1ULL << *half) - 1;
    for (int r = 0; r < 4; ++r) rk[r] = wl_stream_key(key, 0x1000 + r);
}

/* out[i] = perm(in[i]) for the keyed bijection perm on [0, n); in[i] < n. */
void wl_permute(uint64_t key, uint64_t n, const uint64_t *in, uint64_t count,
                uint64_t *out) {
    uint32_t half; uint64_t mask, rk[4];
    feistel_setup(key, n, &half, &mask, rk);
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < (int64_t)count; ++i)
        out[i] = feistel(in[i], n, half, mask, rk);
}

/* dst[perm(i)] = src[i] for i < n: a keyed shuffle of a u64 array. */
void wl_shuffle_u64(uint64_t key, const uint64_t *src, uint64_t n,
                    uint64_t *dst) {
    uint32_t half; uint64_t mask, rk[4];
    feistel_setup(key, n, &half, &mask, rk);
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < (int64_t)n; ++i)
        dst[feistel((uint64_t)i, n, half, mask, rk)] = src[i];
}

/* Choose k distinct indices of [0, n) with Floyd's algorithm and set their
 * bytes in `mark` (n bytes, zeroed by the caller).  Sequential: the choice
 * depends only on (key, n, k). */
void wl_floyd_mark(uint64_t key, uint64_t n, uint64_t k, uint8_t *mark) {
    for (uint64_t j = n - k; j < n; ++j) {
        uint64_t t = draw(key, j) % (j + 1);
        if (mark[t]) mark[j] = 1;
        else mark[t] = 1;
    }
}
