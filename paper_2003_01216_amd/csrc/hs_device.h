// hs_device.h -- device-side building blocks of the gfx950 hybrid sort.
//
// The sort follows the cluster method of Section 3.4 of Alghamdi & Alaghband
// (arXiv 2003.01216) on one GPU: a one-step decimal MSD partition of the keys
// into ten non-overlapping buckets, a local sort of fixed-size partitions of
// each bucket (here an LDS tile sort, where the paper quicksorts per thread),
// then non-recursive merge rounds of the sorted runs inside each bucket
// (Figure 1b, Section 3.2), each round split over all compute units by
// merge-path co-ranks instead of one thread per pair of lists.
//
// Everything here is integer work; nothing is a dense contraction, so there is
// no MFMA.  Wavefronts are 64 lanes wide.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <limits>
#include <type_traits>

namespace hs {

constexpr int kWave = 64;

// ---------------------------------------------------------------- key traits
template <typename K>
struct Traits;
template <>
struct Traits<int32_t> {
    using U = uint32_t;  // the biased (unsigned) key domain
    static constexpr int32_t kMin = INT32_MIN;
    static constexpr int32_t kMax = INT32_MAX;
};
template <>
struct Traits<int64_t> {
    using U = uint64_t;
    static constexpr int64_t kMin = INT64_MIN;
    static constexpr int64_t kMax = INT64_MAX;
};

// ------------------------------------------------------ decimal digit plan
// Section 3.4: the master divides the keys into ten parts by their most
// significant digit.  Reading used throughout: the digit is the fixed-position
// decimal digit D-1 of u = k - beta, beta = min(min key, 0), D = number of
// decimal digits of max u.  With p = 10^(D-1) (the largest power of ten not
// above max u, or 1), the digit is the number of thresholds b*p, b = 1..9,
// that u reaches -- nine unsigned compares, no division on the hot path.
// thr[b-1] holds b*p - 1 saturated at the type's maximum, so that a threshold
// beyond the unsigned range is never passed: digit = sum_b [u > thr[b-1]].
//
// The finer one-step splitter (a second most significant digit, one hundred
// buckets) reads the first two of the D digits: bucket floor(u / q) with
// q = 10^(D-2), or 10u when D = 1 (a one-digit u read with a trailing zero).
// Bucket b of the ten-bucket rule is the union of buckets 10b .. 10b+9 of
// this one, so both orders agree with the keys.
template <typename K>
struct DigitPlan {
    using U = typename Traits<K>::U;
    U beta;           // (U)beta
    U thr[9];         // b*p - 1, saturated
    uint64_t magic;   // 32-bit keys: ceil(2^64 / p) for p >= 10, 0 for p == 1
    // two-digit rule
    U thr2[9];        // 64-bit keys: c*q - 1 for c = 1..9 (saturated; all-ones when D = 1)
    uint64_t magic2;  // 32-bit keys: ceil(2^64 / q) for q >= 10, else 0
    uint32_t mul2;    // 32-bit keys with magic2 = 0: the bucket is u * mul2 (1 when D = 2, 10 when D = 1)
    // three-digit rule (32-bit keys only)
    uint64_t magic3;  // ceil(2^64 / r), r = p / 100, for r >= 10, else 0
    uint32_t mul3;    // with magic3 = 0: the bucket is u * mul3 (1 when D = 3, 10 when D = 2, 100 when D = 1)
};

// fixed: the keys are images of unsigned keys (the unsigned value x maps
// to x + type minimum, keeping the order), and beta is fixed at the type's
// minimum, so u is the unsigned value itself (no bias, as for non-negative
// signed keys).  Otherwise beta = min(mn, 0).
template <typename K>
__host__ __device__ inline DigitPlan<K> make_digit_plan(K mn, K mx, bool fixed = false) {
    using U = typename Traits<K>::U;
    DigitPlan<K> pl;
    K beta = fixed ? Traits<K>::kMin : (mn < 0 ? mn : K(0));
    pl.beta = (U)beta;
    U top = (U)mx - (U)beta;  // exact: mx >= beta
    U p = 1;
    while (p <= top / 10) p *= 10;  // largest power of ten <= top
    const U umax = ~U(0);
    for (int b = 1; b <= 9; b++) {
        // b*p - 1, or umax when b*p does not fit
        pl.thr[b - 1] = (p > umax / (U)b) ? umax : (U)((U)b * p - 1);
    }
    // p = 10^k does not divide 2^64 for k >= 1, so floor((2^64-1)/p) + 1 is
    // ceil(2^64/p)
    pl.magic = p == 1 ? 0 : ~0ull / (uint64_t)p + 1;
    // two-digit rule: q = p / 10 (none when p = 1)
    const U q = p / 10;
    for (int c = 1; c <= 9; c++) pl.thr2[c - 1] = q == 0 ? umax : (U)((U)c * q - 1);  // c*q < 10q = p: fits
    pl.magic2 = q >= 10 ? ~0ull / (uint64_t)q + 1 : 0;
    pl.mul2 = q == 0 ? 10u : 1u;
    // three-digit rule: r = p / 100 (none when p < 100)
    const U r = p / 100;
    pl.magic3 = r >= 10 ? ~0ull / (uint64_t)r + 1 : 0;
    pl.mul3 = p == 1 ? 100u : p == 10 ? 10u : 1u;
    return pl;
}

// p of a plan (the largest power of ten not above max u, or 1).
template <typename K>
__host__ __device__ inline uint64_t plan_p(const DigitPlan<K>& pl) {
    return (uint64_t)pl.thr[0] + 1;
}

// The key's decimal digit floor(u / p), u = k - beta.  32-bit keys: the high
// word of u * ceil(2^64 / p), exact for every u < 2^32 since p < 2^32 (with
// M = 2^64/p + e, 0 < e < 1, u*M/2^64 exceeds u/p by less than 2^-32 < 1/p,
// too little to cross the next integer); two multiply instructions.  64-bit
// keys: nine compares against the saturated thresholds b*p - 1.
template <typename K>
__host__ __device__ __forceinline__ int digit_of(const DigitPlan<K>& pl, K k) {
    using U = typename Traits<K>::U;
    U u = (U)k - pl.beta;
    if constexpr (sizeof(U) == 4) {
        const uint64_t m = pl.magic;
        const uint64_t mid = (uint64_t)u * (uint32_t)(m >> 32) + (uint32_t)(((uint64_t)u * (uint32_t)m) >> 32);
        return m ? (int)(mid >> 32) : (int)u;
    } else {
        int d = 0;
#pragma unroll
        for (int b = 0; b < 9; b++) d += (u > pl.thr[b]) ? 1 : 0;
        return d;
    }
}

// The key's two-digit bucket (0..99) under the one-hundred-bucket rule.
// 32-bit keys: floor(u / q) by the same multiply-high as digit_of (exact,
// q < 2^32), or u * mul2 for q = 1 and for D = 1.  64-bit keys: the first
// digit d by nine compares, then the second by nine compares of
// u - d*p (< p = 10q) against c*q - 1.
template <typename K>
__host__ __device__ __forceinline__ int bucket2_of(const DigitPlan<K>& pl, K k) {
    using U = typename Traits<K>::U;
    U u = (U)k - pl.beta;
    if constexpr (sizeof(U) == 4) {
        const uint64_t m = pl.magic2;
        const uint64_t mid = (uint64_t)u * (uint32_t)(m >> 32) + (uint32_t)(((uint64_t)u * (uint32_t)m) >> 32);
        return m ? (int)(mid >> 32) : (int)(u * pl.mul2);
    } else {
        int d = 0;
#pragma unroll
        for (int b = 0; b < 9; b++) d += (u > pl.thr[b]) ? 1 : 0;
        const U r = u - (U)d * (pl.thr[0] + 1);
        int e = 0;
#pragma unroll
        for (int c = 0; c < 9; c++) e += (r > pl.thr2[c]) ? 1 : 0;
        return 10 * d + e;
    }
}

// The key's three-digit bucket (0..999) under the one-thousand-bucket rule,
// 32-bit keys: floor(u / r), r = p / 100, by the same exact multiply-high as
// digit_of when r >= 10, else u * mul3 (r = 1, or D < 3: the digits of u
// followed by zeros).
template <typename K>
__host__ __device__ __forceinline__ int bucket3_of(const DigitPlan<K>& pl, K k) {
    using U = typename Traits<K>::U;
    static_assert(sizeof(U) == 4, "one thousand buckets: 32-bit keys");
    U u = (U)k - pl.beta;
    const uint64_t m = pl.magic3;
    const uint64_t mid = (uint64_t)u * (uint32_t)(m >> 32) + (uint32_t)(((uint64_t)u * (uint32_t)m) >> 32);
    return m ? (int)(mid >> 32) : (int)(u * pl.mul3);
}

// Bucket of a key under the rule with NBK buckets (10, 100 or 1000).
template <int NBK, typename K>
__host__ __device__ __forceinline__ int bucket_of(const DigitPlan<K>& pl, K k) {
    static_assert(NBK == 10 || NBK == 100 || NBK == 1000, "ten, one hundred or one thousand buckets");
    if constexpr (NBK == 10)
        return digit_of(pl, k);
    else if constexpr (NBK == 100)
        return bucket2_of(pl, k);
    else
        return bucket3_of(pl, k);
}

// The keys of bucket b (NBK buckets) lie in u in [lo, lo + width): the
// local sorts narrow their words by it.
template <typename K>
__host__ __device__ __forceinline__ void bucket_span(const DigitPlan<K>& pl, int nbk, int b, uint64_t& lo, uint64_t& width) {
    const uint64_t p = plan_p(pl);
    if (nbk == 10) {
        lo = (uint64_t)b * p;
        width = p;
    } else if (nbk == 100 && p >= 10) {
        lo = (uint64_t)b * (p / 10);
        width = p / 10;
    } else if (nbk == 100) {  // D = 1: bucket 10u
        lo = (uint64_t)(b / 10);
        width = 1;
    } else if (p >= 100) {
        lo = (uint64_t)b * (p / 100);
        width = p / 100;
    } else {  // D = 2: bucket 10u; D = 1: bucket 100u
        lo = (uint64_t)(b / (p == 10 ? 10 : 100));
        width = 1;
    }
}

// ----------------------------------------------------------------- sort words
// The LDS sorts work on a "word" W with a plain '<'.  Keys-only sorts use the
// key itself.  Stable key+payload sorts use a 64-bit composite
// (sign-flipped key << 32 | position), which is a strict total order, so any
// correct sorting network or merge produces the stable order; the payload is
// fetched by position afterwards.
__device__ __forceinline__ uint64_t pair_word(int32_t k, uint32_t pos) {
    return ((uint64_t)((uint32_t)k ^ 0x80000000u) << 32) | (uint64_t)pos;
}
__device__ __forceinline__ int32_t pair_key(uint64_t w) { return (int32_t)((uint32_t)(w >> 32) ^ 0x80000000u); }
__device__ __forceinline__ uint32_t pair_pos(uint64_t w) { return (uint32_t)w; }

// Stable 64-bit key + payload sorts: a 128-bit word (sign-flipped key, then
// position), compared lexicographically -- the same strict order.
struct W128 {
    uint64_t lo;  // position
    uint64_t hi;  // key ^ 2^63 (unsigned order = signed key order)
};
__device__ __forceinline__ bool operator<(const W128& a, const W128& b) {
    return a.hi < b.hi || (a.hi == b.hi && a.lo < b.lo);
}
__device__ __forceinline__ W128 pair_word(int64_t k, uint32_t pos) {
    return W128{(uint64_t)pos, (uint64_t)k ^ 0x8000000000000000ull};
}
__device__ __forceinline__ int64_t pair_key(const W128& w) { return (int64_t)(w.hi ^ 0x8000000000000000ull); }
__device__ __forceinline__ uint32_t pair_pos(const W128& w) { return (uint32_t)w.lo; }

// Keeps a loaded word live and unconditional (see lds_corank).
template <typename W>
__device__ __forceinline__ void keep_word(W& x) {
    if constexpr (sizeof(W) == 16) {
        asm volatile("" : "+v"(x.lo), "+v"(x.hi));
    } else {
        asm volatile("" : "+v"(x));
    }
}

template <typename W>
struct WordMin;
template <>
struct WordMin<int32_t> {
    static constexpr int32_t v = INT32_MIN;
};
template <>
struct WordMin<uint32_t> {
    static constexpr uint32_t v = 0u;
};
template <typename W>
struct WordMax;
template <>
struct WordMax<int32_t> {
    static constexpr int32_t v = INT32_MAX;
};
template <>
struct WordMax<int64_t> {
    static constexpr int64_t v = INT64_MAX;
};
template <>
struct WordMax<uint32_t> {
    static constexpr uint32_t v = ~0u;
};
template <>
struct WordMax<uint64_t> {
    static constexpr uint64_t v = ~0ull;
};
template <>
struct WordMax<W128> {
    static constexpr W128 v = {~0ull, ~0ull};
};

// c ? a : b for sort words; 16-byte words select field by field (a
// conditional on two struct lvalues would select an address and move the
// words to scratch memory).
template <typename W>
__device__ __forceinline__ W wsel(bool c, const W& a, const W& b) {
    if constexpr (sizeof(W) == 16) {
        W r;
        r.lo = c ? a.lo : b.lo;
        r.hi = c ? a.hi : b.hi;
        return r;
    } else {
        return c ? a : b;
    }
}

template <typename W>
__device__ __forceinline__ void cas_up(W& a, W& b) {  // a <- min, b <- max
    const bool sw = b < a;
    const W lo = wsel(sw, b, a);
    const W hi = wsel(sw, a, b);
    a = lo;
    b = hi;
}

// LDS index padding: one pad word per 128 bytes, so that lanes reading
// VT-strided positions spread over the banks.
template <typename W>
__device__ __forceinline__ int lds_pad(int i) {
    // i >= 0 always: the unsigned shift is one instruction where a signed
    // division takes four
    constexpr unsigned per = 128 / sizeof(W);
    return i + (int)((unsigned)i / per);
}
// words[lds_pad(i)], with the byte offset formed as (i + (i >> p)) * size:
// a shift and one add-shift instruction.
template <typename W>
__device__ __forceinline__ W lds_at_padded(const W* words, int i) {
    static_assert(sizeof(W) == 4 || sizeof(W) == 8 || sizeof(W) == 16, "4-, 8- or 16-byte words");
    constexpr unsigned size_log2 = sizeof(W) == 16 ? 4 : sizeof(W) == 8 ? 3 : 2;
    constexpr unsigned per_log2 = 7 - size_log2;  // 128-byte pad period
    const unsigned u = (unsigned)i;
    const unsigned off = (u + (u >> per_log2)) << size_log2;
    return *reinterpret_cast<const W*>(reinterpret_cast<const char*>(words) + off);
}
template <typename W>
constexpr int lds_padded_size(int n) {
    return n + n / (128 / (int)sizeof(W)) + 1;
}

// Sorting network over VT registers (VT a power of two), fully unrolled:
// Batcher's odd-even merge sort, every comparator ascending (191
// compare-exchanges for 32 registers, where a bitonic sort takes 240).
template <typename W, int VT>
__device__ __forceinline__ void register_sort(W (&v)[VT]) {
#pragma unroll
    for (int p = 1; p < VT; p <<= 1) {
#pragma unroll
        for (int k = p; k >= 1; k >>= 1) {
#pragma unroll
            for (int j = k % p; j + k < VT; j += 2 * k) {
#pragma unroll
                for (int i = 0; i < k; i++) {
                    if (i < VT - j - k && (i + j) / (2 * p) == (i + j + k) / (2 * p)) cas_up(v[i + j], v[i + j + k]);
                }
            }
        }
    }
}

// Sorts a bitonic sequence of VT registers ascending (half-cleaner cascade).
template <typename W, int VT>
__device__ __forceinline__ void bitonic_merge(W (&v)[VT]) {
#pragma unroll
    for (int j = VT >> 1; j > 0; j >>= 1) {
#pragma unroll
        for (int i = 0; i < VT; i++) {
            const int l = i ^ j;
            if (l > i) cas_up(v[i], v[l]);
        }
    }
}

// ------------------------------------------------ merges across lanes (DPP)
// A 32-bit register's value in lane ^ MASK: a DPP lane permutation where
// one exists (0xB1 = lane ^ 1, 0x4E = lane ^ 2, 0x1B = lane ^ 3 within
// quads, 0x141 = lane ^ 7 within half-rows, 0x140 = lane ^ 15 within rows,
// 0x128 = lane ^ 8 as a rotation by eight within rows), else a bit-mode
// swizzle (xor mask within 32 lanes); masks that cross the two halves of the
// wave go through a backward permute.
template <int MASK>
__device__ __forceinline__ int lane_xor32(int x) {
    if constexpr (MASK == 1) return __builtin_amdgcn_mov_dpp(x, 0xB1, 0xF, 0xF, false);
    else if constexpr (MASK == 2) return __builtin_amdgcn_mov_dpp(x, 0x4E, 0xF, 0xF, false);
    else if constexpr (MASK == 3) return __builtin_amdgcn_mov_dpp(x, 0x1B, 0xF, 0xF, false);
    else if constexpr (MASK == 7) return __builtin_amdgcn_mov_dpp(x, 0x141, 0xF, 0xF, false);
    else if constexpr (MASK == 15) return __builtin_amdgcn_mov_dpp(x, 0x140, 0xF, 0xF, false);
    else if constexpr (MASK == 8) return __builtin_amdgcn_mov_dpp(x, 0x128, 0xF, 0xF, false);
    else if constexpr (MASK < 32) return __builtin_amdgcn_ds_swizzle(x, 0x1F | (MASK << 10));
    else return __shfl_xor(x, MASK, kWave);
}

template <int MASK, typename W>
__device__ __forceinline__ W lane_xor(W x) {
    if constexpr (sizeof(W) == 4) {
        return (W)lane_xor32<MASK>((int)x);
    } else if constexpr (sizeof(W) == 16) {
        return W{lane_xor<MASK>(x.lo), lane_xor<MASK>(x.hi)};
    } else {
        const uint64_t u = (uint64_t)x;
        const uint32_t lo = (uint32_t)lane_xor32<MASK>((int)(uint32_t)u);
        const uint32_t hi = (uint32_t)lane_xor32<MASK>((int)(uint32_t)(u >> 32));
        return (W)(((uint64_t)hi << 32) | lo);
    }
}

// The median of three 32-bit words, one instruction.  With c the smallest
// word it is min(a, b), with c the largest max(a, b): a lane keeps the
// smaller or the larger of its word and its partner's by its own c.
__device__ __forceinline__ int32_t med3_word(int32_t a, int32_t b, int32_t c) {
    int32_t r;
    asm("v_med3_i32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}
__device__ __forceinline__ uint32_t med3_word(uint32_t a, uint32_t b, uint32_t c) {
    uint32_t r;
    asm("v_med3_u32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}

// One compare-exchange stage between lanes: register i meets the partner
// lane's register i (or VT-1-i when FLIP); the lane with `lower` set keeps
// the smaller word.  32-bit words: the partner's word and one median of
// three per register; 64-bit words: compare and selects.
template <typename W, int VT, int MASK, bool FLIP>
__device__ __forceinline__ void lane_stage(W (&v)[VT], bool lower) {
    W p[VT];
#pragma unroll
    for (int i = 0; i < VT; i++) p[i] = lane_xor<MASK>(v[FLIP ? VT - 1 - i : i]);
    if constexpr (sizeof(W) == 4) {
        const W c = lower ? WordMin<W>::v : WordMax<W>::v;
#pragma unroll
        for (int i = 0; i < VT; i++) v[i] = med3_word(v[i], p[i], c);
    } else {
#pragma unroll
        for (int i = 0; i < VT; i++) {
            const bool lt = p[i] < v[i];
            v[i] = wsel(lt == lower, p[i], v[i]);  // lower: the smaller, else the larger
        }
    }
}

// Groups of G lanes (G = 2 .. 32) each holding VT sorted words, the two
// halves of a group sorted runs: merged into one run over the group, lane
// blocked (the group's lane j ends with outputs j*VT .. j*VT+VT-1).  A
// bitonic merge of the two runs: the first stage pairs element e with
// element 2M-1-e (M = G/2*VT; the partner lane is lane ^ (G-1), register
// VT-1-i), then half-cleaners at lane distances G/4 .. 1 and within the
// registers.  No LDS memory, no barrier.
template <typename W, int VT, int D>
__device__ __forceinline__ void lane_half_cleaners(W (&v)[VT], int lane) {
    if constexpr (D >= 1) {
        lane_stage<W, VT, D, false>(v, !(lane & D));
        lane_half_cleaners<W, VT, D / 2>(v, lane);
    }
}

template <typename W, int VT, int G>
__device__ __forceinline__ void lane_merge(W (&v)[VT], int lane) {
    static_assert(G >= 2 && G <= kWave && (G & (G - 1)) == 0, "groups of 2 to 64 lanes");
    lane_stage<W, VT, G - 1, true>(v, !(lane & (G / 2)));
    lane_half_cleaners<W, VT, G / 4>(v, lane);
    bitonic_merge<W, VT>(v);
}

// Branch-free co-rank with log2(STEP0)+1 unrolled probes; STEP0 is a power
// of two not below the largest possible hi - lo.  Probes outside [lo, hi)
// read index 0 of each array instead (always a valid address for callers)
// and are ignored.
template <int STEP0, typename FA, typename FB>
__device__ __forceinline__ int merge_path_fixed(int diag, int na, int nb, FA A, FB B) {
    const int lo = diag > nb ? diag - nb : 0;
    const int hi = diag < na ? diag : na;
    int pos = lo;
#pragma unroll
    for (int step = STEP0; step > 0; step >>= 1) {
        const int m = pos + step - 1;
        const bool inr = m < hi;
        const int ma = inr ? m : 0;
        const int mb = inr ? diag - 1 - m : 0;
        const bool take = inr && !(B(mb) < A(ma));
        pos = take ? pos + step : pos;
    }
    return pos;
}

// Co-rank over padded LDS runs (logical positions; physical lds_pad) A at
// [sa, sa+na) and B at [sb, sb+nb): how many of the first `diag` merged
// outputs come from A (ties to A).  log2(STEP0)+1 probes, STEP0 a power of
// two with 2*STEP0 > hi - lo.  Probe indices are clamped into the runs (B
// may be read one word before sb, or at nb, the first word after it), so
// every read is in bounds and no probe needs a branch.
template <typename W, int STEP0>
__device__ __forceinline__ int lds_corank(const W* lds, int sa, int sb, int diag, int na, int nb) {
    const int lo = diag > nb ? diag - nb : 0;
    const int hi = diag < na ? diag : na;
    const int hic = hi > 0 ? hi - 1 : 0;
    const int kb = sb + diag - 1;  // B[diag - 1 - m] sits at kb - m
    int pos = lo;
#pragma unroll
    for (int step = STEP0; step > 0; step >>= 1) {
        const int m = pos + step - 1;
        const int mc = m < hic ? m : hic;
        W a = lds_at_padded(lds, sa + mc);
        W b = lds_at_padded(lds, kb - mc);
        // both reads are used unconditionally: otherwise the compiler moves
        // them under a branch on m < hi, and every probe pays for the exec
        // mask bookkeeping in scalar instructions
        keep_word(a);
        keep_word(b);
        pos = (m < hi && !(b < a)) ? pos + step : pos;
    }
    return pos;
}

// VT consecutive words from logical position p0 of a padded LDS array
// (VT <= one pad period, so the run crosses at most one pad word): VT+1
// reads at constant offsets, then one select per word.
template <typename W, int VT>
__device__ __forceinline__ void lds_read_padded(const W* lds, int p0, W (&r)[VT]) {
    constexpr int per = 128 / (int)sizeof(W);
    static_assert(VT <= per, "a window crosses at most one pad word");
    const W* base = lds + lds_pad<W>(p0);
    const int cut = per - (p0 & (per - 1));  // words i >= cut lie one further
    W x[VT + 1];
#pragma unroll
    for (int i = 0; i <= VT; i++) x[i] = base[i];
#pragma unroll
    for (int i = 0; i < VT; i++) r[i] = wsel(i >= cut, x[i + 1], x[i]);
}

// The VT outputs that follow co-rank (ai, bi) of a merge: the VT smallest
// of A[ai..ai+VT) and B[bi..bi+VT) (both runs followed by at least VT
// largest-word sentinels).  min(a[i], b[VT-1-i]) is the bitonic sequence of
// those VT words; one bitonic merge sorts it.
template <typename W, int VT>
__device__ __forceinline__ void lds_merge_window(const W* lds, int pa, int pb, W (&v)[VT]) {
    W b[VT];
    lds_read_padded<W, VT>(lds, pa, v);
    lds_read_padded<W, VT>(lds, pb, b);
#pragma unroll
    for (int i = 0; i < VT; i++) v[i] = wsel(b[VT - 1 - i] < v[i], b[VT - 1 - i], v[i]);
    bitonic_merge<W, VT>(v);
}

// --------------------------------------------------------- wave/block helpers
__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

// The dispatcher hands workgroups to the eight XCDs in turn (workgroup b to
// XCD b mod 8), and each XCD has an L2 of its own.  Units (tiles, chunks)
// whose edges share cache lines -- per-tile counts stored tile-minor, runs
// written back to back -- should meet in one L2, so workgroup b takes unit
// x*q + min(x, r) + b/8 (x = b mod 8, q = G/8, r = G mod 8): each XCD works
// through one contiguous range of units in order.  A bijection on [0, G).
__device__ __forceinline__ int64_t xcd_unit(int64_t b, int64_t G) {
    constexpr int64_t kXcd = 8;
    const int64_t q = G / kXcd, r = G % kXcd, x = b % kXcd;
    return x * q + (x < r ? x : r) + b / kXcd;
}

// 32-bit wave scans and reductions by DPP (no LDS traffic): shifts by 1, 2,
// 4 and 8 lanes within each row of 16 (lanes shifted in from outside the
// row take the identity), then rows 1 and 3 combine the last lane of the row
// before them (row_bcast:15) and rows 2 and 3 the last lane of row 1
// (row_bcast:31).  Lane 63 ends with the whole wave's result.
template <int CTRL, int ROWS, typename T>
__device__ __forceinline__ T dpp_from(T x, T id) {
    return (T)__builtin_amdgcn_update_dpp((int)id, (int)x, CTRL, ROWS, 0xF, false);
}
template <typename T, typename Op>
__device__ __forceinline__ T wave_incl_scan_dpp(T x, T id, Op op) {
    static_assert(sizeof(T) == 4, "32-bit lanes");
    x = op(x, dpp_from<0x111, 0xF>(x, id));  // row_shr:1
    x = op(x, dpp_from<0x112, 0xF>(x, id));  // row_shr:2
    x = op(x, dpp_from<0x114, 0xF>(x, id));  // row_shr:4
    x = op(x, dpp_from<0x118, 0xF>(x, id));  // row_shr:8
    x = op(x, dpp_from<0x142, 0xA>(x, id));  // row_bcast:15 into rows 1, 3
    x = op(x, dpp_from<0x143, 0xC>(x, id));  // row_bcast:31 into rows 2, 3
    return x;
}

template <typename T>
__device__ __forceinline__ T wave_incl_scan_add(T x) {
    if constexpr (sizeof(T) == 4) {
        return wave_incl_scan_dpp<T>(x, T(0), [](T a, T b) { return a + b; });
    } else {
        const int lane = lane_id();
#pragma unroll
        for (int d = 1; d < kWave; d <<= 1) {
            T y = __shfl_up(x, d, kWave);
            if (lane >= d) x += y;
        }
        return x;
    }
}

// The wave's total in every lane.
template <typename T>
__device__ __forceinline__ T wave_reduce_add(T x) {
    if constexpr (sizeof(T) == 4) {
        return (T)__builtin_amdgcn_readlane((int)wave_incl_scan_add(x), kWave - 1);
    } else {
#pragma unroll
        for (int d = kWave / 2; d > 0; d >>= 1) x += __shfl_xor(x, d, kWave);
        return x;
    }
}

template <typename T>
__device__ __forceinline__ T wave_reduce_min(T x) {
    if constexpr (sizeof(T) == 4) {
        const T r = wave_incl_scan_dpp<T>(x, std::numeric_limits<T>::max(), [](T a, T b) { return b < a ? b : a; });
        return (T)__builtin_amdgcn_readlane((int)r, kWave - 1);
    } else {
#pragma unroll
        for (int d = kWave / 2; d > 0; d >>= 1) {
            T y = __shfl_xor(x, d, kWave);
            x = y < x ? y : x;
        }
        return x;
    }
}

template <typename T>
__device__ __forceinline__ T wave_reduce_max(T x) {
    if constexpr (sizeof(T) == 4) {
        const T r = wave_incl_scan_dpp<T>(x, std::numeric_limits<T>::lowest(), [](T a, T b) { return b > a ? b : a; });
        return (T)__builtin_amdgcn_readlane((int)r, kWave - 1);
    } else {
#pragma unroll
        for (int d = kWave / 2; d > 0; d >>= 1) {
            T y = __shfl_xor(x, d, kWave);
            x = y > x ? y : x;
        }
        return x;
    }
}

// Index of the last entry of pre[0..n] (non-decreasing, pre[0] = 0) that is
// <= x, i.e. the owner of flat item x in a prefix of per-owner item counts.
template <typename T>
__device__ __forceinline__ int owner_of(const T* pre, int n, T x) {
    int lo = 0, hi = n;  // invariant: pre[lo] <= x < pre[hi] (pre[n] > x)
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (pre[mid] <= x)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

// Number of bottom-up merge rounds a bucket of `size` keys needs when its
// local sort leaves runs of `tile` keys and each round merges `fanin` (2 or
// 4) runs into one.
__host__ __device__ __forceinline__ int merge_rounds(int64_t size, int64_t tile, int fanin = 2) {
    int64_t runs = (size + tile - 1) / tile;
    int r = 0;
    int64_t cover = 1;
    while (cover < runs) {
        cover *= fanin;
        r++;
    }
    return r;
}

// Global-memory searches over long runs by absolute power-of-two steps (top:
// a power of two not below the search range), so that searches of nearby
// values share the cache lines of their early probes.  These searches are
// bound by the cache lines they pull (every deep probe of a search touches
// its own line), not by latency: a 4-ary search, with three probes per
// level, pulls more lines and is slower.

// Co-rank: how many of the first diag outputs of merge(A, B) come from A
// (ties to A).
template <typename FA, typename FB>
__device__ __forceinline__ int64_t merge_path_steps64(int64_t diag, int64_t na, int64_t nb, int64_t top, FA A, FB B) {
    const int64_t lo = diag > nb ? diag - nb : 0;
    const int64_t hi = diag < na ? diag : na;
    int64_t pos = lo;
    for (int64_t step = top; step > 0; step >>= 1) {
        const int64_t m = pos + step - 1;
        if (m < hi && !(B(diag - 1 - m) < A(m))) pos += step;
    }
    return pos;
}

// Searches over runs that start on 32-key block boundaries and come with
// block samples (first key F[b] = R[32b] of every block, last key
// Lst[b] = R[32b + 31] of every full block): a binary search over the dense
// samples, whose lines neighbouring searches share, then at most six probes
// of the keys inside one block.
__device__ __forceinline__ int64_t top_step(int64_t w) {  // largest power of two <= w, 0 for 0
    return w > 0 ? (int64_t)1 << (63 - __builtin_clzll((unsigned long long)w)) : 0;
}

// Co-rank of diag (a multiple of 32) in the stable merge of A[0..na) and
// B[0..nb): how many of the first diag outputs come from A (ties to A).
// Coarse probes m = 32i + 31 compare A's block end la[i] with B's block start
// fb[diag/32 - i - 1] = B[diag - 1 - m].
template <typename K>
__device__ __forceinline__ int64_t merge_path_sampled(int64_t diag, const K* A, int64_t na, const K* la, const K* B,
                                                      int64_t nb, const K* fb) {
    const int64_t lo = diag > nb ? diag - nb : 0;
    const int64_t hi = diag < na ? diag : na;
    const int64_t ilo = lo / 32, ihi = hi >= 32 ? (hi - 32) / 32 : -1;
    int64_t t = 0;  // coarse probes from ilo on at which A's key comes first
    for (int64_t step = top_step(ihi - ilo + 1); step > 0; step >>= 1) {
        const int64_t i = ilo + t + step - 1;
        if (i <= ihi && !(fb[diag / 32 - i - 1] < la[i])) t += step;
    }
    int64_t a = t > 0 ? 32 * (ilo + t) : lo;
    int64_t b = ilo + t <= ihi ? 32 * (ilo + t) + 31 : hi;
    a = a > lo ? a : lo;
    b = b < hi ? b : hi;
    int64_t pos = a;  // b - a < 64
#pragma unroll
    for (int64_t step = 32; step > 0; step >>= 1) {
        const int64_t m = pos + step - 1;
        if (m < b && !(B[diag - 1 - m] < A[m])) pos += step;
    }
    return pos;
}

// Counts of R[0..nr) and Q[0..nq) below v (UPPER: not above v), from their
// block first keys fr and fq; the two searches step together.
template <bool UPPER, typename K>
__device__ __forceinline__ void bound2_sampled(const K* R, int64_t nr, const K* fr, const K* Q, int64_t nq, const K* fq,
                                               K v, int64_t& pr, int64_t& pq) {
    auto in = [&](K x) { return UPPER ? !(v < x) : x < v; };
    const int64_t br = (nr + 31) / 32, bq = (nq + 31) / 32;
    int64_t tr = 0, tq = 0;  // blocks whose first key is in
    for (int64_t step = top_step(br > bq ? br : bq); step > 0; step >>= 1) {
        const int64_t ir = tr + step - 1, iq = tq + step - 1;
        if (ir < br && in(fr[ir])) tr += step;
        if (iq < bq && in(fq[iq])) tq += step;
    }
    // the count lies in [32(t-1) + 1, min(32t, n)] (0 when t = 0)
    pr = tr > 0 ? 32 * (tr - 1) + 1 : 0;
    pq = tq > 0 ? 32 * (tq - 1) + 1 : 0;
    const int64_t er = tr * 32 < nr ? tr * 32 : nr, eq = tq * 32 < nq ? tq * 32 : nq;
#pragma unroll
    for (int64_t step = 16; step > 0; step >>= 1) {
        const int64_t mr = pr + step - 1, mq = pq + step - 1;
        if (mr < er && in(R[mr])) pr += step;
        if (mq < eq && in(Q[mq])) pq += step;
    }
}

}  // namespace hs
