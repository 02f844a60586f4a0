/*
 * CPU oracle for the indexed nested loop join -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg load
 * this file.  It shares no code, header or table with the GPU library.
 *
 * What it computes (Section II-A, INLJ; Section II-D, RMI; Section VI-B,
 * "Duplicates"): for each tuple of the outer relation S, every tuple of the
 * inner relation R with the same join key.  The learned index is only an
 * access path to that set, so the result has a plain definition:
 *
 *     P = { (i, j) : S[i] == R[j] },  listed in lexicographic (i, j) order,
 *     count = |P|.
 *
 * Three independent routines produce or check P:
 *   orc_brute_join       the definition itself: nested loops over S and R.
 *   orc_sort_merge_join  a plain sort-merge join: sort (S[i], i) pairs with
 *                        the C library's qsort, merge with the sorted R,
 *                        emit the cross product of equal-key runs, then a
 *                        stable counting sort by i.
 *   orc_equal_range      textbook lower/upper-bound binary search on the
 *                        sorted R for single keys (sampled checks at sizes
 *                        where a full join is too slow on the host).
 *
 * For the learned sort join (Section IV) R comes in any order and j is its
 * position as given; the result is the same P:
 *   orc_sort_join        sort (key, position) pairs of both relations with
 *                        qsort, merge, emit, counting sort by i.
 *   orc_sort_positions   the sorted (key, position) pairs of one relation.
 * orc_brute_join takes R in any order and pins both.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    uint64_t key;
    uint64_t idx;
} orc_kv;

/* 1 if R[0..n) is non-decreasing (the INLJ's index on R is ordered). */
int orc_is_nondecreasing(const uint64_t *R, uint64_t n) {
    for (uint64_t j = 1; j < n; ++j)
        if (R[j - 1] > R[j]) return 0;
    return 1;
}

static int cmp_kv(const void *a, const void *b) {
    const orc_kv *x = (const orc_kv *)a, *y = (const orc_kv *)b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    if (x->idx != y->idx) return x->idx < y->idx ? -1 : 1;
    return 0;
}

/* Growable (i, j) list, stored as interleaved uint32 pairs. */
typedef struct {
    uint32_t *p;
    uint64_t len, cap;
} pairvec;

static int push(pairvec *v, uint64_t i, uint64_t j) {
    if (v->len == v->cap) {
        uint64_t nc = v->cap ? 2 * v->cap : 1024;
        uint32_t *np = (uint32_t *)realloc(v->p, nc * 2 * sizeof(uint32_t));
        if (!np) return -1;
        v->p = np;
        v->cap = nc;
    }
    v->p[2 * v->len] = (uint32_t)i;
    v->p[2 * v->len + 1] = (uint32_t)j;
    v->len++;
    return 0;
}

/*
 * Definition of P written out: for i in S order, for j in R order, emit
 * (i, j) when the keys are equal.  The output is in (i, j) order by
 * construction.  *out_pairs is malloc'd (free with orc_free); returns 0, or
 * -1 on allocation failure.
 */
int orc_brute_join(const uint64_t *R, uint64_t n, const uint64_t *S, uint64_t m,
                   uint32_t **out_pairs, uint64_t *out_count) {
    pairvec v = {0, 0, 0};
    for (uint64_t i = 0; i < m; ++i)
        for (uint64_t j = 0; j < n; ++j)
            if (S[i] == R[j] && push(&v, i, j)) { free(v.p); return -1; }
    *out_pairs = v.p;
    *out_count = v.len;
    return 0;
}

/*
 * Sort-merge join of a sorted R with an unsorted S.
 *   1. T = [(S[i], i)], sorted by (key, i).
 *   2. Walk T and R together; on a key present in both, T[a..a2) and
 *      R[b..b2) hold all of its copies: emit (T[k].idx, j) for all k, j.
 *      Otherwise advance the side with the smaller key.
 *   3. Stable counting sort of the emitted pairs by i; within one i the r
 *      indices were emitted in ascending order, so the result is (i, j)
 *      order.
 * Returns 0, -1 on allocation failure, -2 if R is not non-decreasing.
 */
int orc_sort_merge_join(const uint64_t *R, uint64_t n, const uint64_t *S,
                        uint64_t m, uint32_t **out_pairs, uint64_t *out_count) {
    *out_pairs = NULL;
    *out_count = 0;
    if (!orc_is_nondecreasing(R, n)) return -2;
    orc_kv *T = (orc_kv *)malloc((m ? m : 1) * sizeof(orc_kv));
    if (!T) return -1;
    for (uint64_t i = 0; i < m; ++i) {
        T[i].key = S[i];
        T[i].idx = i;
    }
    qsort(T, m, sizeof(orc_kv), cmp_kv);

    pairvec v = {0, 0, 0};
    uint64_t a = 0, b = 0;
    while (a < m && b < n) {
        if (T[a].key < R[b]) {
            ++a;
        } else if (R[b] < T[a].key) {
            ++b;
        } else {
            uint64_t key = R[b], a2 = a, b2 = b;
            while (a2 < m && T[a2].key == key) ++a2;
            while (b2 < n && R[b2] == key) ++b2;
            for (uint64_t k = a; k < a2; ++k)
                for (uint64_t j = b; j < b2; ++j)
                    if (push(&v, T[k].idx, j)) { free(v.p); free(T); return -1; }
            a = a2;
            b = b2;
        }
    }
    free(T);

    /* Stable counting sort by i. */
    uint64_t *start = (uint64_t *)calloc(m + 1, sizeof(uint64_t));
    uint32_t *sorted = (uint32_t *)malloc((v.len ? v.len : 1) * 2 * sizeof(uint32_t));
    if (!start || !sorted) { free(start); free(sorted); free(v.p); return -1; }
    for (uint64_t k = 0; k < v.len; ++k) start[v.p[2 * k] + 1]++;
    for (uint64_t i = 0; i < m; ++i) start[i + 1] += start[i];
    for (uint64_t k = 0; k < v.len; ++k) {
        uint64_t dst = start[v.p[2 * k]]++;
        sorted[2 * dst] = v.p[2 * k];
        sorted[2 * dst + 1] = v.p[2 * k + 1];
    }
    free(start);
    free(v.p);
    *out_pairs = sorted;
    *out_count = v.len;
    return 0;
}

/*
 * (key, position) pairs of keys[0..n) in ascending (key, position) order,
 * by qsort: the sorted relation a sort-based join produces from an
 * unsorted input (Section IV-C), with each key's input position carried.
 * Returns 0, or -1 on allocation failure.
 */
int orc_sort_positions(const uint64_t *keys, uint64_t n, uint64_t *out_keys,
                       uint32_t *out_pos) {
    orc_kv *T = (orc_kv *)malloc((n ? n : 1) * sizeof(orc_kv));
    if (!T) return -1;
    for (uint64_t j = 0; j < n; ++j) {
        T[j].key = keys[j];
        T[j].idx = j;
    }
    qsort(T, n, sizeof(orc_kv), cmp_kv);
    for (uint64_t j = 0; j < n; ++j) {
        out_keys[j] = T[j].key;
        out_pos[j] = (uint32_t)T[j].idx;
    }
    free(T);
    return 0;
}

/*
 * The join of two unsorted relations (Section IV, learned sort join): the
 * same P = {(i, j) : S[i] == R[j]} in (i, j) order, where j is the position
 * in R as given.
 *   1. U = [(R[j], j)] and T = [(S[i], i)], each sorted by (key, position).
 *   2. Merge U and T; on a key present in both, emit (T[k].idx, U[l].idx)
 *      for every copy on each side (U's copies in ascending j).
 *   3. Stable counting sort of the pairs by i.
 * Returns 0, or -1 on allocation failure.
 */
int orc_sort_join(const uint64_t *R, uint64_t n, const uint64_t *S, uint64_t m,
                  uint32_t **out_pairs, uint64_t *out_count) {
    *out_pairs = NULL;
    *out_count = 0;
    orc_kv *U = (orc_kv *)malloc((n ? n : 1) * sizeof(orc_kv));
    orc_kv *T = (orc_kv *)malloc((m ? m : 1) * sizeof(orc_kv));
    if (!U || !T) { free(U); free(T); return -1; }
    for (uint64_t j = 0; j < n; ++j) {
        U[j].key = R[j];
        U[j].idx = j;
    }
    for (uint64_t i = 0; i < m; ++i) {
        T[i].key = S[i];
        T[i].idx = i;
    }
    qsort(U, n, sizeof(orc_kv), cmp_kv);
    qsort(T, m, sizeof(orc_kv), cmp_kv);

    pairvec v = {0, 0, 0};
    uint64_t a = 0, b = 0;
    while (a < m && b < n) {
        if (T[a].key < U[b].key) {
            ++a;
        } else if (U[b].key < T[a].key) {
            ++b;
        } else {
            uint64_t key = U[b].key, a2 = a, b2 = b;
            while (a2 < m && T[a2].key == key) ++a2;
            while (b2 < n && U[b2].key == key) ++b2;
            for (uint64_t k = a; k < a2; ++k)
                for (uint64_t l = b; l < b2; ++l)
                    if (push(&v, T[k].idx, U[l].idx)) {
                        free(v.p); free(T); free(U); return -1;
                    }
            a = a2;
            b = b2;
        }
    }
    free(T);
    free(U);

    uint64_t *start = (uint64_t *)calloc(m + 1, sizeof(uint64_t));
    uint32_t *sorted = (uint32_t *)malloc((v.len ? v.len : 1) * 2 * sizeof(uint32_t));
    if (!start || !sorted) { free(start); free(sorted); free(v.p); return -1; }
    for (uint64_t k = 0; k < v.len; ++k) start[v.p[2 * k] + 1]++;
    for (uint64_t i = 0; i < m; ++i) start[i + 1] += start[i];
    for (uint64_t k = 0; k < v.len; ++k) {
        uint64_t dst = start[v.p[2 * k]]++;
        sorted[2 * dst] = v.p[2 * k];
        sorted[2 * dst + 1] = v.p[2 * k + 1];
    }
    free(start);
    free(v.p);
    *out_pairs = sorted;
    *out_count = v.len;
    return 0;
}

/*
 * For each query key q, the run of R (sorted, non-decreasing) equal to q:
 * first[k] = lower_bound(R, q), count[k] = upper_bound(R, q) - first[k].
 */
void orc_equal_range(const uint64_t *R, uint64_t n, const uint64_t *keys,
                     uint64_t k, uint64_t *first, uint64_t *count) {
    for (uint64_t t = 0; t < k; ++t) {
        uint64_t q = keys[t];
        uint64_t lo = 0, hi = n; /* first index with R[idx] >= q */
        while (lo < hi) {
            uint64_t mid = lo + (hi - lo) / 2;
            if (R[mid] < q) lo = mid + 1;
            else hi = mid;
        }
        uint64_t lo2 = lo, hi2 = n; /* first index with R[idx] > q */
        while (lo2 < hi2) {
            uint64_t mid = lo2 + (hi2 - lo2) / 2;
            if (R[mid] <= q) lo2 = mid + 1;
            else hi2 = mid;
        }
        first[t] = lo;
        count[t] = lo2 - lo;
    }
}

void orc_free(void *p) { free(p); }
