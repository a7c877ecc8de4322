// Host-side check of the GPU library's decimal digit rules (hs_device.h):
// digit_of (ten buckets), bucket2_of (one hundred), bucket3_of (one
// thousand, int32 keys) and bucket_span, for int32 and int64 keys, against
// integer division by powers of ten written out here.  Plans come from make_digit_plan(min, max) of each case; keys
// cover the edges c*q - 1, c*q, c*q + 1 of every bucket and random values.
// Prints the number of mismatches and exits non-zero if there are any.
#include <stdint.h>
#include <stdio.h>

#include "hs_device.h"

static uint64_t g_state = 0x9E3779B97F4A7C15ull;
static uint64_t next_u64() {  // splitmix64
    uint64_t z = (g_state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static int ndigits(uint64_t x) {
    int d = 1;
    while (x >= 10) {
        x /= 10;
        d++;
    }
    return d;
}
static uint64_t pow10u(int e) {
    uint64_t p = 1;
    while (e-- > 0) p *= 10;
    return p;
}

static long long g_bad = 0, g_checked = 0;

template <typename K>
static void check_key(const hs::DigitPlan<K>& pl, K mn, K mx, K k) {
    using U = typename hs::Traits<K>::U;
    const K beta = mn < 0 ? mn : K(0);
    const uint64_t u = (uint64_t)(U)((U)k - (U)beta);
    const uint64_t top = (uint64_t)(U)((U)mx - (U)beta);
    const int D = ndigits(top);
    const uint64_t p = pow10u(D - 1);
    const int want1 = (int)(u / p);
    const int want2 = D == 1 ? (int)(10 * u) : (int)(u / pow10u(D - 2));
    const int got1 = hs::digit_of(pl, k), got2 = hs::bucket2_of(pl, k);
    uint64_t lo1, w1, lo2, w2;
    hs::bucket_span(pl, 10, want1, lo1, w1);
    hs::bucket_span(pl, 100, want2, lo2, w2);
    bool span_ok = u >= lo1 && u - lo1 < w1 && u >= lo2 && u - lo2 < w2;
    int got3 = 0, want3 = 0;
    if constexpr (sizeof(K) == 4) {
        want3 = D <= 2 ? (int)(u * pow10u(3 - D)) : (int)(u / pow10u(D - 3));
        got3 = hs::bucket3_of(pl, k);
        uint64_t lo3, w3;
        hs::bucket_span(pl, 1000, want3, lo3, w3);
        span_ok = span_ok && u >= lo3 && u - lo3 < w3;
    }
    g_checked++;
    if (got1 != want1 || got2 != want2 || got3 != want3 || !span_ok || hs::plan_p(pl) != p) {
        if (g_bad < 10)
            printf("mismatch: %d-bit min %lld max %lld key %lld: digit %d/%d bucket2 %d/%d bucket3 %d/%d span %d\n",
                   (int)(8 * sizeof(K)), (long long)mn, (long long)mx, (long long)k, got1, want1, got2, want2, got3,
                   want3, (int)span_ok);
        g_bad++;
    }
}

template <typename K>
static void check_case(K mn, K mx) {
    using U = typename hs::Traits<K>::U;
    if (mx < mn) {
        K t = mn;
        mn = mx;
        mx = t;
    }
    const hs::DigitPlan<K> pl = hs::make_digit_plan<K>(mn, mx);
    const K beta = mn < 0 ? mn : K(0);
    const U top = (U)mx - (U)beta;
    const U p = (U)pow10u(ndigits((uint64_t)top) - 1);
    const U q = p >= 10 ? p / 10 : 1;
    auto in_range = [&](U u) { return u >= (U)((U)mn - (U)beta) && u <= top; };
    auto key_of = [&](U u) { return (K)(U)(u + (U)beta); };
    check_key<K>(pl, mn, mx, mn);
    check_key<K>(pl, mn, mx, mx);
    for (U c = 0; c <= 99; c++) {
        if (q != 0 && c > (~U(0)) / q) break;
        const U e = c * q;
        for (int dlt = -1; dlt <= 1; dlt++) {
            const U u = e + (U)dlt;
            if ((dlt < 0 && e == 0) || (dlt > 0 && u < e)) continue;
            if (in_range(u)) check_key<K>(pl, mn, mx, key_of(u));
        }
    }
    if constexpr (sizeof(K) == 4) {  // the edges of every three-digit bucket
        const U q3 = p >= 100 ? p / 100 : 1;
        for (U c = 0; c <= 999; c++) {
            if (c > (~U(0)) / q3) break;
            const U e = c * q3;
            for (int dlt = -1; dlt <= 1; dlt++) {
                const U u = e + (U)dlt;
                if ((dlt < 0 && e == 0) || (dlt > 0 && u < e)) continue;
                if (in_range(u)) check_key<K>(pl, mn, mx, key_of(u));
            }
        }
    }
    for (int r = 0; r < 2000; r++) {
        const U span = (U)(top - (U)((U)mn - (U)beta));
        const U u = (U)((U)mn - (U)beta) + (span == ~U(0) ? (U)next_u64() : (U)(next_u64() % ((uint64_t)span + 1)));
        check_key<K>(pl, mn, mx, key_of(u));
    }
}

int main() {
    // int32: maxima at every power of ten and its neighbours, with
    // non-negative and negative minima, and the type's extremes
    const int32_t mins32[] = {0, 5, -1, -7, -1000, INT32_MIN, INT32_MIN + 1};
    for (int e = 0; e <= 9; e++) {
        const int64_t p = (int64_t)pow10u(e);
        for (int64_t m : {p - 1, p, p + 1, 2 * p - 1, 9 * p, 10 * p - 1})
            for (int32_t mn : mins32)
                if (m <= INT32_MAX && m >= 0) check_case<int32_t>(mn, (int32_t)m);
    }
    check_case<int32_t>(INT32_MIN, INT32_MAX);
    check_case<int32_t>(0, INT32_MAX);
    check_case<int32_t>(INT32_MIN, -1);
    check_case<int32_t>(7, 7);
    for (int r = 0; r < 300; r++) check_case<int32_t>((int32_t)next_u64(), (int32_t)next_u64());
    // int64 likewise, up to 10^18 and the full range (D = 20)
    const int64_t mins64[] = {0, 3, -1, -999, INT64_MIN, INT64_MIN + 1};
    for (int e = 0; e <= 18; e++) {
        const uint64_t p = pow10u(e);
        for (uint64_t m : {p - 1, p, p + 1, 2 * p - 1, 9 * p, 10 * p - 1})
            for (int64_t mn : mins64)
                if (m <= (uint64_t)INT64_MAX) check_case<int64_t>(mn, (int64_t)m);
    }
    check_case<int64_t>(INT64_MIN, INT64_MAX);
    check_case<int64_t>(0, INT64_MAX);
    check_case<int64_t>(INT64_MIN, -1);
    for (int r = 0; r < 300; r++) check_case<int64_t>((int64_t)next_u64(), (int64_t)next_u64());
    // d1 = b * 205 >> 11 and d2 = b - 10 d1 for every two-digit bucket
    for (uint32_t b = 0; b < 100; b++) {
        g_checked++;
        if (((b * 205u) >> 11) != b / 10) g_bad++;
    }
    printf("checked %lld, mismatches %lld\n", g_checked, g_bad);
    return g_bad ? 1 : 0;
}
