/*
 * oracle.c -- plain, slow, obviously-correct CPU implementation of what the
 * hybrid MSD-radix / quicksort / merge sort computes.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or
 * load this file: only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark use it.  It shares no code, header or table with the GPU
 * library.
 *
 * Paper: Alghamdi & Alaghband, "High Performance Parallel Sort for Shared and
 * Distributed Memory MIMD" (arXiv 2003.01216).
 *
 * What it computes (all integer, so every result is exact and unique):
 *   - sorted keys: the ascending rearrangement of the input (Section 3.1,
 *     Figure 1; ascending order is the reading of the garbled quicksort
 *     sentence in Section 3.1);
 *   - stable pairs: keys ascending, equal keys keep their input order
 *     (merge sort's stability, Section 2.1);
 *   - the one-step decimal MSD partition into ten buckets (abstract,
 *     Section 2.1, Section 3.4): the bucket of key k is the decimal digit in
 *     position D-1 of u = k - beta, where beta = min(min key, 0) and D is the
 *     number of decimal digits of max(u) (fixed-position digit reading);
 *   - its finer one-step variants with the two or three most significant
 *     digits (one hundred buckets, floor(u / 10^(D-2)), or one thousand,
 *     floor(u / 10^(D-3)); a u with fewer digits read as its digits followed
 *     by zeros): the next digits the paper's MSD radix would split on
 *     (Sections 2.3, 3.4), taken in the same single step.
 *
 * How it computes the sort (following the paper's algorithms, sequentially):
 *   1. split the array into CHUNKS contiguous partitions, one per "thread" of
 *      the shared-memory hybrid (Section 3.2, power-of-two thread count);
 *   2. quicksort each partition (Figure 1c): choose a pivot (median of
 *      three), partition around it, recurse on the smaller side and loop on
 *      the larger; tiny ranges by insertion;
 *   3. non-recursive (bottom-up) merge (Figure 1b, Section 3.2 merge rounds):
 *      merge neighbouring sorted lists pairwise, carrying an odd last list,
 *      until one list remains; ties are taken from the left list.
 * Every element is ordered by the composite (key, original index), a strict
 * total order, so the result is the stable sort whatever the pivot choice
 * (the paper's quicksort alone is not stable).
 *
 * Other key types and descending order (the key types a sort library is
 * asked for; the paper sorts integers): every key is ordered through an
 * integer order image written out from the type's definition of order --
 * unsigned integers by value, IEEE-754 floats by the standard's total order
 * (sign first, then the magnitude's bit pattern, so -NaN < -inf < ... < -0
 * < +0 < ... < +inf < +NaN), descending order by the image reversed -- and
 * the decimal bucket rule is applied to that image: signed images with
 * beta = min(min image, 0) as above, unsigned keys with beta = 0 in the
 * unsigned domain (u = the key itself).  Outputs are the input keys gathered
 * in the order found, so no image is ever inverted.
 *
 * The "radix mode" runs the paper's fourth model sequentially (Section 3.4):
 * stable counting scatter into the ten buckets, the same sort inside every
 * bucket, then the buckets in digit order.  It must equal the plain mode,
 * which pins that the bucket rule preserves order.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define CHUNKS 16      /* partitions sorted independently before merging */
#define SMALL_RANGE 16 /* ranges below this are sorted by insertion */

typedef struct {
    int64_t key;  /* int32 keys are widened exactly */
    uint64_t idx; /* position in the input: the tie-break */
} item;

static int item_lt(const item* a, const item* b) {
    if (a->key != b->key) return a->key < b->key;
    return a->idx < b->idx;
}

static void item_swap(item* a, item* b) {
    item t = *a;
    *a = *b;
    *b = t;
}

/* ---------------------------------------------------------------- quicksort
 * Figure 1c: pick a pivot V, partition into S1 (< V) and S2 (> V), sort both.
 * Sorts s[low..high] inclusive. */
static void insertion_sort(item* s, int64_t low, int64_t high) {
    for (int64_t i = low + 1; i <= high; i++) {
        item x = s[i];
        int64_t j = i - 1;
        while (j >= low && item_lt(&x, &s[j])) {
            s[j + 1] = s[j];
            j--;
        }
        s[j + 1] = x;
    }
}

static void quicksort(item* s, int64_t low, int64_t high) {
    while (high - low + 1 > SMALL_RANGE) {
        /* median of three, moved to s[high] as the pivot */
        int64_t mid = low + (high - low) / 2;
        if (item_lt(&s[mid], &s[low])) item_swap(&s[mid], &s[low]);
        if (item_lt(&s[high], &s[low])) item_swap(&s[high], &s[low]);
        if (item_lt(&s[mid], &s[high])) item_swap(&s[mid], &s[high]);
        item v = s[high];
        /* partition: everything smaller than v goes left of position p */
        int64_t p = low;
        for (int64_t j = low; j < high; j++) {
            if (item_lt(&s[j], &v)) {
                item_swap(&s[p], &s[j]);
                p++;
            }
        }
        item_swap(&s[p], &s[high]);
        /* S1 = [low, p-1], S2 = [p+1, high]; recurse on the smaller one */
        if (p - low < high - p) {
            quicksort(s, low, p - 1);
            low = p + 1;
        } else {
            quicksort(s, p + 1, high);
            high = p - 1;
        }
    }
    insertion_sort(s, low, high);
}

/* ------------------------------------------------------------------- merge
 * Merge of two sorted lists a[0..na) and b[0..nb) into out; on equal
 * elements the left list goes first (merge sort's stability). */
static void merge_two(const item* a, int64_t na, const item* b, int64_t nb, item* out) {
    int64_t i = 0, j = 0, k = 0;
    while (i < na && j < nb) {
        if (item_lt(&b[j], &a[i]))
            out[k++] = b[j++];
        else
            out[k++] = a[i++];
    }
    while (i < na) out[k++] = a[i++];
    while (j < nb) out[k++] = b[j++];
}

/* Chunked quicksort followed by the bottom-up merge rounds (Figures 1b, 1c;
 * Section 3.2).  Sorts s[0..n). */
static int hybrid_sort(item* s, int64_t n) {
    if (n < 2) return 0;
    int64_t nchunks = CHUNKS;
    if (nchunks > n) nchunks = n;
    int64_t* starts = (int64_t*)malloc(sizeof(int64_t) * (size_t)(nchunks + 1));
    if (!starts) return -1;
    for (int64_t c = 0; c <= nchunks; c++) starts[c] = (n * c) / nchunks;
    for (int64_t c = 0; c < nchunks; c++) quicksort(s, starts[c], starts[c + 1] - 1);

    item* buf = (item*)malloc(sizeof(item) * (size_t)n);
    if (!buf) {
        free(starts);
        return -1;
    }
    item* src = s;
    item* dst = buf;
    int64_t nruns = nchunks;
    while (nruns > 1) {
        int64_t r = 0, w = 0;
        for (; r + 1 < nruns; r += 2) {
            merge_two(src + starts[r], starts[r + 1] - starts[r], src + starts[r + 1],
                      starts[r + 2] - starts[r + 1], dst + starts[r]);
            starts[w++] = starts[r];
        }
        if (r < nruns) { /* odd list carried to the next round */
            memcpy(dst + starts[r], src + starts[r], sizeof(item) * (size_t)(starts[r + 1] - starts[r]));
            starts[w++] = starts[r];
        }
        starts[w] = n;
        nruns = w;
        item* t = src;
        src = dst;
        dst = t;
    }
    if (src != s) memcpy(s, src, sizeof(item) * (size_t)n);
    free(buf);
    free(starts);
    return 0;
}

/* ------------------------------------------------------- decimal digit plan
 * Section 3.4 divides the data into ten parts by the most significant digit.
 * Reading: beta = min(min key, 0); u = k - beta (exact as unsigned 64-bit);
 * D = number of decimal digits of max u (1 for 0); the bucket of k is
 * floor(u / 10^(D-1)), computed here with a real division. */
static const uint64_t POW10[20] = {1ULL,
                                   10ULL,
                                   100ULL,
                                   1000ULL,
                                   10000ULL,
                                   100000ULL,
                                   1000000ULL,
                                   10000000ULL,
                                   100000000ULL,
                                   1000000000ULL,
                                   10000000000ULL,
                                   100000000000ULL,
                                   1000000000000ULL,
                                   10000000000000ULL,
                                   100000000000000ULL,
                                   1000000000000000ULL,
                                   10000000000000000ULL,
                                   100000000000000000ULL,
                                   1000000000000000000ULL,
                                   10000000000000000000ULL};

static int decimal_digits(uint64_t x) {
    int d = 1;
    while (d < 20 && x >= POW10[d]) d++;
    return d;
}

typedef struct {
    int64_t beta;
    int32_t D;
    uint64_t p;
} plan;

static plan make_plan_beta(int64_t beta, int64_t mx) {
    plan pl;
    pl.beta = beta;
    uint64_t top = (uint64_t)mx - (uint64_t)pl.beta;
    pl.D = decimal_digits(top);
    pl.p = POW10[pl.D - 1];
    return pl;
}

static plan make_plan(int64_t mn, int64_t mx) {
    plan pl;
    pl.beta = mn < 0 ? mn : 0;
    uint64_t top = (uint64_t)mx - (uint64_t)pl.beta;
    pl.D = decimal_digits(top);
    pl.p = POW10[pl.D - 1];
    return pl;
}

static int bucket_of(const plan* pl, int64_t k) {
    uint64_t u = (uint64_t)k - (uint64_t)pl->beta;
    return (int)(u / pl->p);
}

/* The finer one-step splitter (a second most significant digit, one hundred
 * buckets): the bucket is the number formed by the first two of the D
 * decimal digits of u, floor(u / 10^(D-2)); a one-digit u reads as its digit
 * followed by a zero (10u).  Bucket b of the ten-bucket rule is the union of
 * buckets 10b .. 10b+9 of this one, so both orders agree with the keys. */
static int bucket2_of(const plan* pl, int64_t k) {
    uint64_t u = (uint64_t)k - (uint64_t)pl->beta;
    if (pl->D == 1) return (int)(10 * u);
    return (int)(u / POW10[pl->D - 2]);
}

/* One thousand buckets: the number formed by the first three of the D
 * digits of u, floor(u / 10^(D-3)); a u of one or two digits reads as its
 * digits followed by zeros (100u, 10u).  Buckets 10c .. 10c+9 of this rule
 * make up bucket c of the hundred-bucket rule. */
static int bucket3_of(const plan* pl, int64_t k) {
    uint64_t u = (uint64_t)k - (uint64_t)pl->beta;
    if (pl->D < 3) return (int)(u * POW10[3 - pl->D]);
    return (int)(u / POW10[pl->D - 3]);
}

/* digits = 1: the ten buckets of Section 3.4; 2 and 3: the finer rules
 * above. */
static int bucket_n(const plan* pl, int64_t k, int digits) {
    if (digits == 3) return bucket3_of(pl, k);
    return digits == 2 ? bucket2_of(pl, k) : bucket_of(pl, k);
}

static int nbuckets(int digits) { return (int)POW10[digits]; }

static int digits_ok(int digits) { return digits >= 1 && digits <= 3; }

/* ------------------------------------------------------- exported: helpers */
static item* load_items_i32(const int32_t* k, int64_t n) {
    item* s = (item*)malloc(sizeof(item) * (size_t)(n > 0 ? n : 1));
    if (!s) return NULL;
    for (int64_t i = 0; i < n; i++) {
        s[i].key = k[i];
        s[i].idx = (uint64_t)i;
    }
    return s;
}

static item* load_items_i64(const int64_t* k, int64_t n) {
    item* s = (item*)malloc(sizeof(item) * (size_t)(n > 0 ? n : 1));
    if (!s) return NULL;
    for (int64_t i = 0; i < n; i++) {
        s[i].key = k[i];
        s[i].idx = (uint64_t)i;
    }
    return s;
}

/* Plan of an array: *beta, *D, *p.  n == 0 gives beta 0, D 1, p 1. */
/* fixed != 0: the keys are unsigned 64-bit values shifted by -2^63 into
 * int64 (order kept); their bias is fixed at that shift, so u is the
 * unsigned value itself (beta = 0 in the unsigned domain). */
static plan plan_of_mode(const item* s, int64_t n, int fixed) {
    if (n == 0) return fixed ? make_plan_beta(INT64_MIN, INT64_MIN) : make_plan(0, 0);
    int64_t mn = s[0].key, mx = s[0].key;
    for (int64_t i = 1; i < n; i++) {
        if (s[i].key < mn) mn = s[i].key;
        if (s[i].key > mx) mx = s[i].key;
    }
    return fixed ? make_plan_beta(INT64_MIN, mx) : make_plan(mn, mx);
}

static plan plan_of(const item* s, int64_t n) { return plan_of_mode(s, n, 0); }

/* bounds[b] = number of keys whose bucket is below b, b = 0..NB (NB = 10,
 * 100 or 1000 buckets) */
static void bounds_of(const item* s, int64_t n, const plan* pl, int digits, int64_t* bounds) {
    int64_t cnt[1000] = {0};
    const int nb = nbuckets(digits);
    for (int64_t i = 0; i < n; i++) cnt[bucket_n(pl, s[i].key, digits)]++;
    bounds[0] = 0;
    for (int b = 0; b < nb; b++) bounds[b + 1] = bounds[b] + cnt[b];
}

/* Stable counting scatter of s[0..n) into the buckets (the master's
 * one-step MSD radix, Section 3.4).  out must hold n items. */
static void stable_scatter(const item* s, int64_t n, const plan* pl, int digits, const int64_t* bounds, item* out) {
    int64_t next[1000];
    for (int b = 0; b < nbuckets(digits); b++) next[b] = bounds[b];
    for (int64_t i = 0; i < n; i++) out[next[bucket_n(pl, s[i].key, digits)]++] = s[i];
}

/* ------------------------------------------------------- exported functions */
int oracle_plan_i32(const int32_t* k, int64_t n, int64_t* beta, int32_t* D, uint64_t* p) {
    item* s = load_items_i32(k, n);
    if (!s) return -1;
    plan pl = plan_of(s, n);
    *beta = pl.beta;
    *D = pl.D;
    *p = pl.p;
    free(s);
    return 0;
}

int oracle_plan_i64(const int64_t* k, int64_t n, int64_t* beta, int32_t* D, uint64_t* p) {
    item* s = load_items_i64(k, n);
    if (!s) return -1;
    plan pl = plan_of(s, n);
    *beta = pl.beta;
    *D = pl.D;
    *p = pl.p;
    free(s);
    return 0;
}

/* bounds[0 .. 10^digits]: the bucket bounds of the array under the one-step
 * rule with `digits` leading digits (1: ten buckets, 2: one hundred, 3: one
 * thousand). */
static int bounds_items_mode(item* s, int64_t n, int digits, int fixed, int64_t* bounds) {
    if (!s) return -1;
    if (!digits_ok(digits)) {
        free(s);
        return -1;
    }
    plan pl = plan_of_mode(s, n, fixed);
    bounds_of(s, n, &pl, digits, bounds);
    free(s);
    return 0;
}

static int bounds_items(item* s, int64_t n, int digits, int64_t* bounds) {
    return bounds_items_mode(s, n, digits, 0, bounds);
}

int oracle_bounds_digits_i32(const int32_t* k, int64_t n, int digits, int64_t* bounds) {
    return bounds_items(load_items_i32(k, n), n, digits, bounds);
}

int oracle_bounds_digits_i64(const int64_t* k, int64_t n, int digits, int64_t* bounds) {
    return bounds_items(load_items_i64(k, n), n, digits, bounds);
}

int oracle_bounds_i32(const int32_t* k, int64_t n, int64_t bounds[11]) {
    return oracle_bounds_digits_i32(k, n, 1, bounds);
}

int oracle_bounds_i64(const int64_t* k, int64_t n, int64_t bounds[11]) {
    return oracle_bounds_digits_i64(k, n, 1, bounds);
}

/* Plain mode: chunked quicksort + bottom-up merge on (key, index). */
int oracle_sort_keys_i32(int32_t* k, int64_t n) {
    item* s = load_items_i32(k, n);
    if (!s) return -1;
    if (hybrid_sort(s, n)) {
        free(s);
        return -1;
    }
    for (int64_t i = 0; i < n; i++) k[i] = (int32_t)s[i].key;
    free(s);
    return 0;
}

int oracle_sort_keys_i64(int64_t* k, int64_t n) {
    item* s = load_items_i64(k, n);
    if (!s) return -1;
    if (hybrid_sort(s, n)) {
        free(s);
        return -1;
    }
    for (int64_t i = 0; i < n; i++) k[i] = s[i].key;
    free(s);
    return 0;
}

/* Stable key + payload sort: the payload travels with its key. */
int oracle_sort_pairs_i32(int32_t* k, uint32_t* v, int64_t n) {
    item* s = load_items_i32(k, n);
    if (!s) return -1;
    uint32_t* v0 = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)(n > 0 ? n : 1));
    if (!v0) {
        free(s);
        return -1;
    }
    memcpy(v0, v, sizeof(uint32_t) * (size_t)n);
    if (hybrid_sort(s, n)) {
        free(s);
        free(v0);
        return -1;
    }
    for (int64_t i = 0; i < n; i++) {
        k[i] = (int32_t)s[i].key;
        v[i] = v0[s[i].idx];
    }
    free(v0);
    free(s);
    return 0;
}

/* Radix mode (Section 3.4 run sequentially): stable scatter into the
 * buckets, the plain sort inside each bucket, buckets in digit order.  Also
 * returns the bucket bounds when bounds != NULL. */
static int radix_mode(item* s, int64_t n, int digits, int64_t* bounds_out) {
    if (!digits_ok(digits)) return -1;
    const int nb = nbuckets(digits);
    plan pl = plan_of(s, n);
    int64_t bounds[1001];
    bounds_of(s, n, &pl, digits, bounds);
    item* t = (item*)malloc(sizeof(item) * (size_t)(n > 0 ? n : 1));
    if (!t) return -1;
    stable_scatter(s, n, &pl, digits, bounds, t);
    for (int b = 0; b < nb; b++) {
        if (hybrid_sort(t + bounds[b], bounds[b + 1] - bounds[b])) {
            free(t);
            return -1;
        }
    }
    memcpy(s, t, sizeof(item) * (size_t)n);
    free(t);
    if (bounds_out)
        for (int b = 0; b <= nb; b++) bounds_out[b] = bounds[b];
    return 0;
}

int oracle_radix_sort_keys_digits_i32(int32_t* k, int64_t n, int digits, int64_t* bounds) {
    item* s = load_items_i32(k, n);
    if (!s) return -1;
    if (radix_mode(s, n, digits, bounds)) {
        free(s);
        return -1;
    }
    for (int64_t i = 0; i < n; i++) k[i] = (int32_t)s[i].key;
    free(s);
    return 0;
}

int oracle_radix_sort_keys_digits_i64(int64_t* k, int64_t n, int digits, int64_t* bounds) {
    item* s = load_items_i64(k, n);
    if (!s) return -1;
    if (radix_mode(s, n, digits, bounds)) {
        free(s);
        return -1;
    }
    for (int64_t i = 0; i < n; i++) k[i] = s[i].key;
    free(s);
    return 0;
}

int oracle_radix_sort_keys_i32(int32_t* k, int64_t n, int64_t* bounds) {
    item* s = load_items_i32(k, n);
    if (!s) return -1;
    if (radix_mode(s, n, 1, bounds)) {
        free(s);
        return -1;
    }
    for (int64_t i = 0; i < n; i++) k[i] = (int32_t)s[i].key;
    free(s);
    return 0;
}

int oracle_radix_sort_keys_i64(int64_t* k, int64_t n, int64_t* bounds) {
    item* s = load_items_i64(k, n);
    if (!s) return -1;
    if (radix_mode(s, n, 1, bounds)) {
        free(s);
        return -1;
    }
    for (int64_t i = 0; i < n; i++) k[i] = s[i].key;
    free(s);
    return 0;
}

int oracle_radix_sort_pairs_digits_i32(int32_t* k, uint32_t* v, int64_t n, int digits, int64_t* bounds) {
    item* s = load_items_i32(k, n);
    if (!s) return -1;
    uint32_t* v0 = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)(n > 0 ? n : 1));
    if (!v0) {
        free(s);
        return -1;
    }
    memcpy(v0, v, sizeof(uint32_t) * (size_t)n);
    if (radix_mode(s, n, digits, bounds)) {
        free(s);
        free(v0);
        return -1;
    }
    for (int64_t i = 0; i < n; i++) {
        k[i] = (int32_t)s[i].key;
        v[i] = v0[s[i].idx];
    }
    free(v0);
    free(s);
    return 0;
}

int oracle_radix_sort_pairs_i32(int32_t* k, uint32_t* v, int64_t n, int64_t* bounds) {
    return oracle_radix_sort_pairs_digits_i32(k, v, n, 1, bounds);
}

/* The intermediate after the one-step MSD radix alone: the stable scatter of
 * the input into bucket order (vals may be NULL).  Writes bounds[NB + 1]. */
static int scatter_only_mode(item* s, int64_t n, int digits, int fixed, int64_t* bounds) {
    if (!digits_ok(digits)) return -1;
    plan pl = plan_of_mode(s, n, fixed);
    bounds_of(s, n, &pl, digits, bounds);
    item* t = (item*)malloc(sizeof(item) * (size_t)(n > 0 ? n : 1));
    if (!t) return -1;
    stable_scatter(s, n, &pl, digits, bounds, t);
    memcpy(s, t, sizeof(item) * (size_t)n);
    free(t);
    return 0;
}

static int scatter_only(item* s, int64_t n, int digits, int64_t* bounds) {
    return scatter_only_mode(s, n, digits, 0, bounds);
}

int oracle_scatter_digits_i32(int32_t* k, uint32_t* v, int64_t n, int digits, int64_t* bounds) {
    item* s = load_items_i32(k, n);
    if (!s) return -1;
    uint32_t* v0 = NULL;
    if (v) {
        v0 = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)(n > 0 ? n : 1));
        if (!v0) {
            free(s);
            return -1;
        }
        memcpy(v0, v, sizeof(uint32_t) * (size_t)n);
    }
    if (scatter_only(s, n, digits, bounds)) {
        free(s);
        free(v0);
        return -1;
    }
    for (int64_t i = 0; i < n; i++) {
        k[i] = (int32_t)s[i].key;
        if (v) v[i] = v0[s[i].idx];
    }
    free(v0);
    free(s);
    return 0;
}

int oracle_scatter_digits_i64(int64_t* k, int64_t n, int digits, int64_t* bounds) {
    item* s = load_items_i64(k, n);
    if (!s) return -1;
    if (scatter_only(s, n, digits, bounds)) {
        free(s);
        return -1;
    }
    for (int64_t i = 0; i < n; i++) k[i] = s[i].key;
    free(s);
    return 0;
}

int oracle_scatter_i32(int32_t* k, uint32_t* v, int64_t n, int64_t bounds[11]) {
    return oracle_scatter_digits_i32(k, v, n, 1, bounds);
}

int oracle_scatter_i64(int64_t* k, int64_t n, int64_t bounds[11]) { return oracle_scatter_digits_i64(k, n, 1, bounds); }

/* The intermediate after the local sorts: the input is scattered into
 * buckets, then every bucket is cut into consecutive partitions of `tile`
 * keys starting at the bucket's first key, and each partition is sorted
 * (stably) on its own (Section 3.4: each thread sorts its partition). */
int oracle_bucket_tiles_digits_i32(int32_t* k, uint32_t* v, int64_t n, int64_t tile, int digits, int64_t* bounds) {
    if (tile < 1) return -1;
    const int nb = nbuckets(digits);
    item* s = load_items_i32(k, n);
    if (!s) return -1;
    uint32_t* v0 = NULL;
    if (v) {
        v0 = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)(n > 0 ? n : 1));
        if (!v0) {
            free(s);
            return -1;
        }
        memcpy(v0, v, sizeof(uint32_t) * (size_t)n);
    }
    if (scatter_only(s, n, digits, bounds)) {
        free(s);
        free(v0);
        return -1;
    }
    for (int b = 0; b < nb; b++) {
        for (int64_t t = bounds[b]; t < bounds[b + 1]; t += tile) {
            int64_t e = t + tile < bounds[b + 1] ? t + tile : bounds[b + 1];
            quicksort(s, t, e - 1);
        }
    }
    for (int64_t i = 0; i < n; i++) {
        k[i] = (int32_t)s[i].key;
        if (v) v[i] = v0[s[i].idx];
    }
    free(v0);
    free(s);
    return 0;
}

int oracle_bucket_tiles_digits_i64(int64_t* k, int64_t n, int64_t tile, int digits, int64_t* bounds) {
    if (tile < 1) return -1;
    const int nb = nbuckets(digits);
    item* s = load_items_i64(k, n);
    if (!s) return -1;
    if (scatter_only(s, n, digits, bounds)) {
        free(s);
        return -1;
    }
    for (int b = 0; b < nb; b++) {
        for (int64_t t = bounds[b]; t < bounds[b + 1]; t += tile) {
            int64_t e = t + tile < bounds[b + 1] ? t + tile : bounds[b + 1];
            quicksort(s, t, e - 1);
        }
    }
    for (int64_t i = 0; i < n; i++) k[i] = s[i].key;
    free(s);
    return 0;
}

int oracle_bucket_tiles_i32(int32_t* k, uint32_t* v, int64_t n, int64_t tile, int64_t bounds[11]) {
    return oracle_bucket_tiles_digits_i32(k, v, n, tile, 1, bounds);
}

int oracle_bucket_tiles_i64(int64_t* k, int64_t n, int64_t tile, int64_t bounds[11]) {
    return oracle_bucket_tiles_digits_i64(k, n, tile, 1, bounds);
}

/* Segmented: every [off[i], off[i+1]) sorted on its own; bounds (may be
 * NULL) receives eleven bucket bounds per segment, relative to its start. */
int oracle_sort_segmented_i32(int32_t* k, const int64_t* off, int64_t nseg, int64_t* bounds) {
    for (int64_t g = 0; g < nseg; g++) {
        int64_t a = off[g], m = off[g + 1] - off[g];
        if (m < 0) return -1;
        if (bounds && oracle_bounds_i32(k + a, m, bounds + 11 * g)) return -1;
        if (oracle_sort_keys_i32(k + a, m)) return -1;
    }
    return 0;
}

int oracle_sort_segmented_i64(int64_t* k, const int64_t* off, int64_t nseg, int64_t* bounds) {
    for (int64_t g = 0; g < nseg; g++) {
        int64_t a = off[g], m = off[g + 1] - off[g];
        if (m < 0) return -1;
        if (bounds && oracle_bounds_i64(k + a, m, bounds + 11 * g)) return -1;
        if (oracle_sort_keys_i64(k + a, m)) return -1;
    }
    return 0;
}

/* ------------------------------------------------------- other key types
 * Key types: 0 int32, 1 uint32, 2 float32, 3 int64, 4 uint64, 5 float64.
 * The order image of key i (an int64 whose signed order is the key order
 * asked for), written from each type's definition:
 *   - signed integers: the value;
 *   - unsigned 32-bit: the value (non-negative, so the signed bucket rule
 *     has beta = 0 and reads the value itself);
 *   - unsigned 64-bit: the value shifted by -2^63 into int64, with the bias
 *     fixed at that shift (u = the value);
 *   - IEEE-754 binary32/binary64: the standard's total order puts every
 *     value with the sign bit set below every value without it, orders
 *     same-sign values by the bit pattern of the magnitude (increasing for
 *     positive, decreasing for negative; NaNs lie beyond the infinities),
 *     and -0 just below +0: image = m for sign 0 and -1 - m for sign 1,
 *     m = the magnitude bits as an integer;
 *   - descending order: the image reversed, -1 - image (unsigned: the
 *     largest value minus the value, so u stays unsigned).
 * Equal images keep their input order (the index tie-break). */
enum { T_I32 = 0, T_U32 = 1, T_F32 = 2, T_I64 = 3, T_U64 = 4, T_F64 = 5 };

static size_t type_size(int t) { return (t == T_I32 || t == T_U32 || t == T_F32) ? 4 : 8; }

static int64_t shift_u64(uint64_t y) { /* y - 2^63 as int64, without overflow */
    const uint64_t h = 0x8000000000000000ull;
    if (y >= h) return (int64_t)(y - h);
    return y == 0 ? INT64_MIN : -(int64_t)(h - y);
}

static int64_t order_image(const void* k, int64_t i, int t, int desc) {
    int64_t img = 0;
    switch (t) {
        case T_I32:
            img = ((const int32_t*)k)[i];
            break;
        case T_I64:
            img = ((const int64_t*)k)[i];
            break;
        case T_U32: {
            const uint32_t x = ((const uint32_t*)k)[i];
            return desc ? (int64_t)(UINT32_MAX - x) : (int64_t)x;
        }
        case T_U64: {
            const uint64_t x = ((const uint64_t*)k)[i];
            return shift_u64(desc ? UINT64_MAX - x : x);
        }
        case T_F32: {
            uint32_t b;
            memcpy(&b, (const char*)k + 4 * i, 4);
            const int64_t m = (int64_t)(b & 0x7FFFFFFFu);
            img = (b >> 31) ? -1 - m : m;
            break;
        }
        case T_F64: {
            uint64_t b;
            memcpy(&b, (const char*)k + 8 * i, 8);
            const int64_t m = (int64_t)(b & 0x7FFFFFFFFFFFFFFFull);
            img = (b >> 63) ? -1 - m : m;
            break;
        }
    }
    return desc ? -1 - img : img;
}

static item* load_items_typed(const void* k, int t, int desc, int64_t n) {
    item* s = (item*)malloc(sizeof(item) * (size_t)(n > 0 ? n : 1));
    if (!s) return NULL;
    for (int64_t i = 0; i < n; i++) {
        s[i].key = order_image(k, i, t, desc);
        s[i].idx = (uint64_t)i;
    }
    return s;
}

/* The input keys (and payload) gathered in the order of s. */
static int gather_typed(void* k, uint32_t* v, int t, const item* s, int64_t n) {
    const size_t w = type_size(t);
    char* k0 = (char*)malloc(w * (size_t)(n > 0 ? n : 1));
    uint32_t* v0 = v ? (uint32_t*)malloc(sizeof(uint32_t) * (size_t)(n > 0 ? n : 1)) : NULL;
    if (!k0 || (v && !v0)) {
        free(k0);
        free(v0);
        return -1;
    }
    memcpy(k0, k, w * (size_t)n);
    if (v) memcpy(v0, v, sizeof(uint32_t) * (size_t)n);
    for (int64_t i = 0; i < n; i++) {
        memcpy((char*)k + w * (size_t)i, k0 + w * (size_t)s[i].idx, w);
        if (v) v[i] = v0[s[i].idx];
    }
    free(k0);
    free(v0);
    return 0;
}

static int valid_type(int t) { return t >= T_I32 && t <= T_F64; }

/* Stable sort of keys of type t (vals may be NULL), ascending or descending. */
int oracle_sort_typed(void* k, uint32_t* v, int t, int desc, int64_t n) {
    if (!valid_type(t)) return -1;
    item* s = load_items_typed(k, t, desc, n);
    if (!s) return -1;
    int rc = hybrid_sort(s, n);
    if (!rc) rc = gather_typed(k, v, t, s, n);
    free(s);
    return rc;
}

int oracle_bounds_typed(const void* k, int t, int desc, int64_t n, int digits, int64_t* bounds) {
    if (!valid_type(t)) return -1;
    return bounds_items_mode(load_items_typed(k, t, desc, n), n, digits, t == T_U64, bounds);
}

int oracle_radix_sort_typed(void* k, uint32_t* v, int t, int desc, int64_t n, int digits, int64_t* bounds) {
    if (!valid_type(t) || !digits_ok(digits)) return -1;
    item* s = load_items_typed(k, t, desc, n);
    if (!s) return -1;
    int rc = 0;
    int64_t b[1001];
    if (scatter_only_mode(s, n, digits, t == T_U64, b)) rc = -1;
    for (int j = 0; !rc && j < nbuckets(digits); j++) rc = hybrid_sort(s + b[j], b[j + 1] - b[j]);
    if (!rc) rc = gather_typed(k, v, t, s, n);
    if (!rc && bounds)
        for (int j = 0; j <= nbuckets(digits); j++) bounds[j] = b[j];
    free(s);
    return rc;
}

/* Intermediates: the stable scatter into buckets (tile <= 0), or that
 * followed by the sort of every `tile`-key partition of every bucket. */
int oracle_stage_typed(void* k, uint32_t* v, int t, int desc, int64_t n, int64_t tile, int digits, int64_t* bounds) {
    if (!valid_type(t) || !digits_ok(digits)) return -1;
    item* s = load_items_typed(k, t, desc, n);
    if (!s) return -1;
    int rc = scatter_only_mode(s, n, digits, t == T_U64, bounds);
    if (!rc && tile > 0) {
        for (int j = 0; j < nbuckets(digits); j++) {
            for (int64_t a = bounds[j]; a < bounds[j + 1]; a += tile) {
                const int64_t e = a + tile < bounds[j + 1] ? a + tile : bounds[j + 1];
                quicksort(s, a, e - 1);
            }
        }
    }
    if (!rc) rc = gather_typed(k, v, t, s, n);
    free(s);
    return rc;
}

/* Order statistic by definition: the j-th smallest key o[j] is the value x
 * with #{k < x} <= j < #{k <= x}.  Returns both counts for a given x. */
void oracle_count_lt_le_i32(const int32_t* k, int64_t n, int32_t x, int64_t* lt, int64_t* le) {
    int64_t a = 0, b = 0;
    for (int64_t i = 0; i < n; i++) {
        a += k[i] < x;
        b += k[i] <= x;
    }
    *lt = a;
    *le = b;
}

void oracle_count_lt_le_i64(const int64_t* k, int64_t n, int64_t x, int64_t* lt, int64_t* le) {
    int64_t a = 0, b = 0;
    for (int64_t i = 0; i < n; i++) {
        a += k[i] < x;
        b += k[i] <= x;
    }
    *lt = a;
    *le = b;
}
