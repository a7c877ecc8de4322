/*
 * omp_hybrid.c -- the paper's method run on the host's CPU cores with OpenMP:
 * a CPU comparison point for the benchmark.
 *
 * BENCHMARK INFRASTRUCTURE ONLY.  This is not the oracle (oracle.c is) and
 * not part of the product: only the CPU-baseline leg of the benchmark and the
 * tests load it.  It shares no code with the GPU library.
 *
 * Paper: Alghamdi & Alaghband, "High Performance Parallel Sort for Shared and
 * Distributed Memory MIMD" (arXiv 2003.01216).  What it runs, for int32 keys:
 *   1. the one-step decimal most-significant-digit partition of Section 3.4
 *      (here on one host instead of a cluster's master): min and max, then the
 *      ten buckets of the fixed-position digit floor(u / 10^(D-1)),
 *      u = k - min(min key, 0), D = decimal digits of max u; every thread
 *      counts its contiguous share of the keys, and a stable scatter moves
 *      them into their buckets;
 *   2. per bucket, the shared-memory hybrid of Sections 3.2-3.3: the bucket is
 *      cut into one partition per thread, each thread quicksorts its own
 *      (Figure 1c), then the sorted partitions are merged pairwise in rounds
 *      (Figure 1b), the pairs of a round on separate threads -- half of the
 *      threads idle in each round, as Section 3.2 describes.
 * Keys only, ascending.
 */
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static void insertion_i32(int32_t* s, int64_t lo, int64_t hi) {
    for (int64_t i = lo + 1; i <= hi; i++) {
        int32_t x = s[i];
        int64_t j = i - 1;
        while (j >= lo && x < s[j]) {
            s[j + 1] = s[j];
            j--;
        }
        s[j + 1] = x;
    }
}

/* Quicksort of s[lo..hi]: median-of-three pivot, partition into smaller and
 * not-smaller elements, recurse on the smaller side, loop on the larger. */
static void quicksort_i32(int32_t* s, int64_t lo, int64_t hi) {
    while (hi - lo + 1 > 16) {
        int64_t mid = lo + (hi - lo) / 2;
        int32_t t;
        if (s[mid] < s[lo]) { t = s[mid]; s[mid] = s[lo]; s[lo] = t; }
        if (s[hi] < s[lo]) { t = s[hi]; s[hi] = s[lo]; s[lo] = t; }
        if (s[mid] < s[hi]) { t = s[mid]; s[mid] = s[hi]; s[hi] = t; }
        const int32_t v = s[hi];
        /* Hoare-style scan from both ends (many equal keys split evenly) */
        int64_t i = lo - 1, j = hi;
        for (;;) {
            do i++; while (s[i] < v);
            do j--; while (j > lo && v < s[j]);
            if (i >= j) break;
            t = s[i]; s[i] = s[j]; s[j] = t;
        }
        t = s[i]; s[i] = s[hi]; s[hi] = t;
        if (i - lo < hi - i) {
            quicksort_i32(s, lo, i - 1);
            lo = i + 1;
        } else {
            quicksort_i32(s, i + 1, hi);
            hi = i - 1;
        }
    }
    insertion_i32(s, lo, hi);
}

static void merge_i32(const int32_t* a, int64_t na, const int32_t* b, int64_t nb, int32_t* out) {
    int64_t i = 0, j = 0, k = 0;
    while (i < na && j < nb) out[k++] = (b[j] < a[i]) ? b[j++] : a[i++];
    while (i < na) out[k++] = a[i++];
    while (j < nb) out[k++] = b[j++];
}

/* Sorts s[0..n) with `threads` threads (tmp holds n keys): partitions
 * quicksorted in parallel, then pairwise merge rounds. */
static void hybrid_bucket(int32_t* s, int32_t* tmp, int64_t n, int threads) {
    if (n < 2) return;
    int parts = threads;
    if (parts > n) parts = (int)n;
    int64_t* st = (int64_t*)malloc(sizeof(int64_t) * (size_t)(parts + 1));
    for (int p = 0; p <= parts; p++) st[p] = n * p / parts;
#pragma omp parallel for num_threads(threads) schedule(static, 1)
    for (int p = 0; p < parts; p++) quicksort_i32(s, st[p], st[p + 1] - 1);
    int32_t* src = s;
    int32_t* dst = tmp;
    int runs = parts;
    while (runs > 1) {
        const int pairs = runs / 2;
#pragma omp parallel for num_threads(threads) schedule(static, 1)
        for (int q = 0; q < pairs; q++) {
            const int64_t a = st[2 * q], m = st[2 * q + 1], e = st[2 * q + 2];
            merge_i32(src + a, m - a, src + m, e - m, dst + a);
        }
        if (runs & 1) memcpy(dst + st[runs - 1], src + st[runs - 1], sizeof(int32_t) * (size_t)(n - st[runs - 1]));
        int w = 0;
        for (int r = 0; r < runs; r += 2) st[w++] = st[r];
        st[w] = n;
        runs = w;
        int32_t* t = src;
        src = dst;
        dst = t;
    }
    if (src != s) memcpy(s, src, sizeof(int32_t) * (size_t)n);
    free(st);
}

/* Returns the number of threads used, or -1 on allocation failure. */
int omp_hybrid_sort_i32(int32_t* k, int64_t n, int threads) {
    if (threads < 1) threads = omp_get_max_threads();
    if (n < 2) return threads;
    int32_t* buf = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    int64_t(*cnt)[10] = (int64_t(*)[10])calloc((size_t)threads, sizeof(int64_t[10]));
    if (!buf || !cnt) {
        free(buf);
        free(cnt);
        return -1;
    }
    /* range */
    int32_t mn = k[0], mx = k[0];
#pragma omp parallel for num_threads(threads) reduction(min : mn) reduction(max : mx)
    for (int64_t i = 0; i < n; i++) {
        if (k[i] < mn) mn = k[i];
        if (k[i] > mx) mx = k[i];
    }
    const int64_t beta = mn < 0 ? mn : 0;
    const uint64_t top = (uint64_t)((int64_t)mx - beta);
    uint64_t p = 1;
    while (p <= top / 10) p *= 10;
    /* stable scatter: thread t owns keys [n*t/T, n*(t+1)/T) */
#pragma omp parallel num_threads(threads)
    {
        const int t = omp_get_thread_num();
        const int64_t a = n * t / threads, e = n * (t + 1) / threads;
        for (int64_t i = a; i < e; i++) cnt[t][(uint64_t)((int64_t)k[i] - beta) / p]++;
#pragma omp barrier
#pragma omp single
        {
            int64_t run = 0;
            for (int d = 0; d < 10; d++)
                for (int q = 0; q < threads; q++) {
                    const int64_t c = cnt[q][d];
                    cnt[q][d] = run;
                    run += c;
                }
        }
        for (int64_t i = a; i < e; i++) buf[cnt[t][(uint64_t)((int64_t)k[i] - beta) / p]++] = k[i];
    }
    /* bucket d now spans [cnt[T-1][d-1], cnt[T-1][d]) (ends after the scatter) */
    int64_t start = 0;
    for (int d = 0; d < 10; d++) {
        const int64_t end = cnt[threads - 1][d];
        hybrid_bucket(buf + start, k + start, end - start, threads);
        memcpy(k + start, buf + start, sizeof(int32_t) * (size_t)(end - start));
        start = end;
    }
    free(buf);
    free(cnt);
    return threads;
}
