// hs_kernels.hip -- gfx950 kernels of the hybrid MSD-radix / tile-sort /
// merge-path sort, and the host launchers the C ABI calls.
//
// Pipeline for the keys of one call (every array is a segment; a plain sort
// is one segment):
//   k_init, k_classify, scan       per-segment size class and histogram tiles
//   k_range, k_plans               min/max -> decimal digit plan (Section 3.4)
//   k_hist, scan                   per-tile counts of the ten buckets
//   k_btab, scan x2                bucket table, local-sort tiles, merge chunks
//   k_scatter                      stable one-step MSD scatter into buckets
//   k_tilesort                     LDS sort of each T-key partition of a bucket
//   k_partition + k_merge          bottom-up merge rounds (Figure 1b), per round
//   k_small                        segments that fit a tile: one LDS sort each
// The flat work lists (histogram tiles, local-sort partitions, merge chunks)
// live on the device as descriptor arrays written by small kernels (k_tiles,
// k_sdesc, k_partition); every heavy kernel runs one workgroup per list slot
// and reads one descriptor before its data.  Grids are sized by host-side
// upper bounds (unused slots exit at once), so the launch sequence depends
// only on host-side sizes and can be captured in a graph.
#include <hip/hip_runtime.h>

#include "hs_device.h"
#include "hs_io.h"
#include "hs_launch.h"
#include "hs_work.h"

namespace hs {

// ------------------------------------------------------------------ helpers
__device__ __forceinline__ void atomic_min_k(int32_t* p, int32_t v) { atomicMin((int*)p, (int)v); }
__device__ __forceinline__ void atomic_max_k(int32_t* p, int32_t v) { atomicMax((int*)p, (int)v); }
__device__ __forceinline__ void atomic_min_k(int64_t* p, int64_t v) { atomicMin((long long*)p, (long long)v); }
__device__ __forceinline__ void atomic_max_k(int64_t* p, int64_t v) { atomicMax((long long*)p, (long long)v); }

template <typename K, bool PAIRS>
struct WordOf {
    using type = K;
};
template <>
struct WordOf<int32_t, true> {
    using type = uint64_t;
};
template <>
struct WordOf<int64_t, true> {
    using type = W128;
};

// Keys of other types are sorted through a signed-integer image of the same
// width whose order is the order asked for (the same order-preserving maps
// the oracle writes out from each type's definition):
//   unsigned: flip the sign bit (x + type minimum);
//   IEEE-754 float: flip the magnitude bits of negative values (the
//     standard's total order: -NaN < -inf < ... < -0 < +0 < ... < +NaN);
//   descending: the bitwise complement of the image (-1 - image).
// A sort applies the forward map where the partition reads the caller's keys
// and the inverse where a bucket's final output is written (k_image does
// either in place over a whole array, for the debug stage runs).
template <typename K>
__device__ __forceinline__ K image_of(K x, int mode, bool inverse) {
    constexpr K sign = Traits<K>::kMin;
    if (inverse && (mode & kImgDesc)) x = ~x;
    if (mode & kImgUnsigned) x ^= sign;
    if (mode & kImgFloat) x ^= (x >> (8 * sizeof(K) - 1)) & ~sign;  // arithmetic shift: all ones when negative
    if (!inverse && (mode & kImgDesc)) x = ~x;
    return x;
}

// The forward map of a call's mode on one key (0: keys are their own image).
template <typename K>
__device__ __forceinline__ K img_in(const Work<K>& w, K x) {
    return w.img ? image_of(x, w.img, false) : x;
}

// load_run of the caller's keys, f(q, image): with mode != 0 the forward
// map is taken on each key; the mode is tested once, not per key.
template <typename K, int NT, int CAP, typename F>
__device__ __forceinline__ void load_keys_imaged(const K* src, int cnt, int mode, F&& f) {
    if (mode)
        load_run<K, NT, CAP>(src, cnt, [&](int q, K k) { f(q, image_of(k, mode, false)); });
    else
        load_run<K, NT, CAP>(src, cnt, f);
}

// A run of outputs from LDS to memory: keys by key_of, or by key_fin
// (the order image undone) when `fin`; the choice is made once per run,
// so the plain store carries no per-key test.
template <typename K, int NT, int CAP, typename KeyOf, typename KeyFin>
__device__ __forceinline__ void store_chunk_keys(K* dst, int c, bool fin, KeyOf&& key_of, KeyFin&& key_fin) {
    if (fin)
        store_keys<K, NT, CAP>(dst, c, key_fin);
    else
        store_keys<K, NT, CAP>(dst, c, key_of);
}

template <typename K, bool PAIRS>
__device__ __forceinline__ typename WordOf<K, PAIRS>::type make_word(K k, int q) {
    if constexpr (PAIRS)
        return pair_word(k, (uint32_t)q);
    else
        return k;
}
template <typename K, bool PAIRS>
__device__ __forceinline__ K word_key(typename WordOf<K, PAIRS>::type w) {
    if constexpr (PAIRS)
        return pair_key(w);
    else
        return w;
}

// Per-thread digit counters: ten 5-bit fields in one 64-bit word (a thread
// counts at most 16 keys).  Packed words: two 16-bit fields per 32-bit word.
__device__ __forceinline__ void unpack5(uint64_t c, uint32_t (&wd)[5]) {
#pragma unroll
    for (int m = 0; m < 5; m++) {
        uint32_t lo = (uint32_t)(c >> (10 * m)) & 31u;
        uint32_t hi = (uint32_t)(c >> (10 * m + 5)) & 31u;
        wd[m] = lo | (hi << 16);
    }
}
// Field d of the packed words, by mask arithmetic (an indexed select would be
// lowered to a scratch-memory table).
__device__ __forceinline__ uint32_t field16(const uint32_t (&wd)[5], int d) {
    const int h = d >> 1;
    const uint32_t w = (wd[0] & (0u - (uint32_t)(h == 0))) | (wd[1] & (0u - (uint32_t)(h == 1))) |
                       (wd[2] & (0u - (uint32_t)(h == 2))) | (wd[3] & (0u - (uint32_t)(h == 3))) |
                       (wd[4] & (0u - (uint32_t)(h == 4)));
    return (w >> ((d & 1) * 16)) & 0xFFFFu;
}

// Block-wide sum of five packed words; every thread gets the totals.
template <int NT>
__device__ __forceinline__ void block_sum5(uint32_t (&wd)[5], uint32_t (*red)[5]) {
    constexpr int NW = NT / kWave;
    const int lane = lane_id(), wave = threadIdx.x / kWave;
#pragma unroll
    for (int m = 0; m < 5; m++) {
        uint32_t s = wave_reduce_add(wd[m]);
        if (lane == 0) red[wave][m] = s;
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < 5; m++) {
        uint32_t s = 0;
#pragma unroll
        for (int q = 0; q < NW; q++) s += red[q][m];
        wd[m] = s;
    }
    __syncthreads();
}

// Block-wide exclusive scan of five packed words; tot receives the totals.
template <int NT>
__device__ __forceinline__ void block_excl5(uint32_t (&wd)[5], uint32_t (&tot)[5], uint32_t (*red)[5]) {
    constexpr int NW = NT / kWave;
    const int lane = lane_id(), wave = threadIdx.x / kWave;
    uint32_t inc[5];
#pragma unroll
    for (int m = 0; m < 5; m++) {
        inc[m] = wave_incl_scan_add(wd[m]);
        if (lane == kWave - 1) red[wave][m] = inc[m];
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < 5; m++) {
        uint32_t before = 0, all = 0;
#pragma unroll
        for (int q = 0; q < NW; q++) {
            uint32_t r = red[q][m];
            before += (q < wave) ? r : 0u;
            all += r;
        }
        wd[m] = inc[m] - wd[m] + before;
        tot[m] = all;
    }
    __syncthreads();
}

template <typename T, int NT>
__device__ __forceinline__ T block_excl_scan(T x, T& total, T* red) {
    constexpr int NW = NT / kWave;
    const int lane = lane_id(), wave = threadIdx.x / kWave;
    T inc = wave_incl_scan_add(x);
    if (lane == kWave - 1) red[wave] = inc;
    __syncthreads();
    T before = 0, all = 0;
#pragma unroll
    for (int q = 0; q < NW; q++) {
        T r = red[q];
        before += (q < wave) ? r : T(0);
        all += r;
    }
    __syncthreads();
    total = all;
    return inc - x + before;
}

// -------------------------------------------------------- LDS merge blocks
// Gathers this thread's `c` outputs of the merge of A = words[a0 + ai ...]
// (x of them) and B = words[b0 + bi ...] (c - x of them) as an ascending run
// followed by sentinels and the B part reversed -- a bitonic sequence -- and
// sorts it with a half-cleaner cascade.  No data-dependent loop, so the VT
// LDS reads are independent.
template <typename W, int VT>
__device__ __forceinline__ void gather_merge(const W* words, int a0, int b0, int ai, int bi, int x, int c,
                                             W (&v)[VT]) {
    const int gap = VT - c;
#pragma unroll
    for (int i = 0; i < VT; i++) {
        const bool from_a = i < x;
        const bool sentinel = !from_a && i < x + gap;
        int idx = from_a ? (a0 + ai + i) : (b0 + bi + (VT - 1 - i));
        idx = sentinel ? a0 : idx;
        W val = lds_at_padded(words, idx);
        v[i] = wsel(sentinel, WordMax<W>::v, val);
    }
    bitonic_merge<W, VT>(v);
}

// Full-chunk gather: x outputs from A starting at words[a_first], the rest
// from B ending at words[b_last], arranged ascending-then-descending.
template <typename W, int VT>
__device__ __forceinline__ void gather_merge_full(const W* words, int a_first, int b_last, int x, W (&v)[VT]) {
#pragma unroll
    for (int i = 0; i < VT; i++) {
        const int idx = i < x ? a_first + i : b_last - i;
        v[i] = lds_at_padded(words, idx);
    }
    bitonic_merge<W, VT>(v);
}

// One LDS merge level of the block sort: runs of L (one per VT/L... threads)
// merged pairwise; each thread produces VT outputs.  `base` is the padded
// start of this thread's VT-run (runs never straddle a pad word).  Slots at
// or past `cnt` hold the largest word, so a pair of runs that starts there
// is already merged: its threads only keep the barriers.
template <typename W, int NT, int VT, int L>
__device__ __forceinline__ void block_sort_level(W* words, int* sp, W (&v)[VT], int tid, int base, int cnt) {
    __syncthreads();
#pragma unroll
    for (int i = 0; i < VT; i++) words[base + i] = v[i];
    __syncthreads();
    const int gb = (tid * VT) & ~(2 * L - 1);
    const int diag = tid * VT - gb;
    const bool live = gb < cnt;
    auto A = [&](int i) { return lds_at_padded(words, gb + i); };
    auto B = [&](int i) { return lds_at_padded(words, gb + L + i); };
    const int ai = live ? merge_path_fixed<L>(diag, L, L, A, B) : 0;
    sp[tid] = ai;
    __syncthreads();
    if (live) {
        const int an = (diag + VT == 2 * L) ? L : sp[tid + 1];
        gather_merge_full<W, VT>(words, gb + ai, gb + L + (diag - ai) + VT - 1, an - ai, v);
    }
}

// The levels from runs of L up; once L >= cnt (the same on every thread)
// every real key is in the first run, sorted, and the rest is padding.
template <typename W, int NT, int VT, int L>
__device__ __forceinline__ void block_sort_levels(W* words, int* sp, W (&v)[VT], int tid, int base, int cnt) {
    if constexpr (L < NT * VT) {
        if (L >= cnt) return;
        block_sort_level<W, NT, VT, L>(words, sp, v, tid, base, cnt);
        block_sort_levels<W, NT, VT, 2 * L>(words, sp, v, tid, base, cnt);
    }
}

// Sorts words[0..NT*VT) (padded layout) ascending in LDS: a register sorting
// network per thread, merge levels across groups of 2, 4, 8, 16 (and, for
// 32-bit words, 32 and 64) lanes (lane permutations, in registers), then the
// remaining merge levels in LDS, fully unrolled.  Result in blocked layout
// (thread t holds outputs t*VT .. t*VT+VT-1, also in LDS).  Slots at or past
// cnt must hold the largest word: a wave whose slots all lie there has
// nothing to sort in registers, and levels whose runs already cover cnt are
// skipped.
//
// BU (the alternative local sort, the non-recursive merge sort of Figure 1b
// as it stands): each thread sorts its VT words (VT = 2: the pairs of the
// figure's first step), then every merge level runs in LDS, bottom up from
// runs of VT, with no lane merges.
template <typename W, int NT, int VT, bool BU = false>
__device__ __forceinline__ void block_sort(W* words, int* sp, int cnt) {
    static_assert((128 / (int)sizeof(W)) % VT == 0, "a VT-run must not straddle a pad word");
    static_assert(NT >= kWave, "lane merges need whole waves");
    const int tid = threadIdx.x;
    const int base = lds_pad<W>(tid * VT);
    W v[VT];
#pragma unroll
    for (int i = 0; i < VT; i++) v[i] = words[base + i];
    const bool live = (tid / kWave) * kWave * VT < cnt;  // the same on every lane of the wave
    if constexpr (BU) {
        if (live) register_sort<W, VT>(v);
        block_sort_levels<W, NT, VT, VT>(words, sp, v, tid, base, cnt);
        __syncthreads();
#pragma unroll
        for (int i = 0; i < VT; i++) words[base + i] = v[i];
        __syncthreads();
        return;
    }
    if (live) {
        register_sort<W, VT>(v);
        lane_merge<W, VT, 2>(v, tid);
        lane_merge<W, VT, 4>(v, tid);
        lane_merge<W, VT, 8>(v, tid);
        lane_merge<W, VT, 16>(v, tid);
        // 32-bit words: a fifth and a sixth lane level (lane ^ 31 by a
        // swizzle, lane ^ 63 by a backward permute) cost about what the LDS
        // levels they replace do, without their barriers; 64-bit words need
        // two exchanges and a compare-and-select per register, and they do not
        if constexpr (sizeof(W) == 4) {
            lane_merge<W, VT, 32>(v, tid);
            lane_merge<W, VT, 64>(v, tid);
        }
    }
    if constexpr (sizeof(W) == 4) {
        block_sort_levels<W, NT, VT, kWave * VT>(words, sp, v, tid, base, cnt);
    } else {
        block_sort_levels<W, NT, VT, 16 * VT>(words, sp, v, tid, base, cnt);
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < VT; i++) words[base + i] = v[i];
    __syncthreads();
}

// ------------------------------------------------------------- setup kernels
// own_off: where a plain sort's one-segment offsets live (w.off points there).
template <typename K>
__global__ void k_init(Work<K> w, int64_t* own_off, int64_t tiles_bound) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (own_off && t < tiles_bound) {
        // a plain sort's partition-tile list (what k_tiles gives a segmented
        // call): tile t covers [t * ptile, min(n, (t + 1) * ptile))
        const int32_t nt = w.n > w.small_max ? (int32_t)((w.n + w.ptile - 1) / w.ptile) : 0;
        TileDesc d{0, 0, 0, 0, 0, 0, 0, 0};
        if (t < nt) {
            d.base = t * w.ptile;
            d.seg_base = 0;
            d.cnt = (int)min((int64_t)w.ptile, w.n - d.base);
            d.seg = 0;
            d.idx = (int)t;
            d.nt = nt;
            d.grp = (int)(t / kGroupTiles);
            d.pad = 0;
        }
        w.tiles[t] = d;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        *w.err = 0;
        *w.rounds = 0;
        if (own_off) {
            // a plain sort is one segment [0, n): its offsets, partition-tile
            // and group counts and their prefixes are known here (what
            // k_classify and the two scans after it give a segmented call)
            own_off[0] = 0;
            own_off[1] = w.n;
            const int32_t nt = w.n > w.small_max ? (int32_t)((w.n + w.ptile - 1) / w.ptile) : 0;
            const int32_t ng = (nt + kGroupTiles - 1) / kGroupTiles;
            w.tilecnt[0] = nt;
            w.groupcnt[0] = ng;
            w.tilepre[0] = 0;
            w.tilepre[1] = nt;
            w.grouppre[0] = 0;
            w.grouppre[1] = ng;
        }
    }
}

// Size class of every segment, histogram-tile count of the large ones, and
// validation of the offsets (non-decreasing, inside [0, n]) and of the
// caller's bound on the segment length: the host launches only the merge
// rounds that bound needs, so a longer segment would be left partly merged.
// Either error makes every later kernel of the call do nothing.
template <typename K>
__global__ void k_classify(Work<K> w) {
    for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < w.nseg; s += gridDim.x * blockDim.x) {
        const int64_t a = w.off[s], b = w.off[s + 1];
        const bool bad = (b < a) || (s == 0 && a < 0) || (s == w.nseg - 1 && b > w.n);
        if (bad) atomicOr(w.err, kErrOffsets);
        const int64_t m = b - a;
        if (!bad && w.max_seg_len > 0 && m > w.max_seg_len) atomicOr(w.err, kErrSegLen);
        const int32_t nt = (!bad && m > w.small_max) ? (int32_t)((m + w.ptile - 1) / w.ptile) : 0;
        w.tilecnt[s] = nt;
        w.groupcnt[s] = (nt + kGroupTiles - 1) / kGroupTiles;
    }
}

// Materialises the flat histogram-tile list (one thread per tile slot).
template <typename K>
__global__ void k_tiles(Work<K> w, int64_t tiles_bound) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= tiles_bound) return;
    const int total = w.tilepre[w.nseg];
    TileDesc d;
    if (*w.err || t >= total) {
        d = TileDesc{0, 0, 0, 0, 0, 0, 0, 0};
    } else {
        const int s = owner_of(w.tilepre, w.nseg, (int)t);
        const int i = (int)t - w.tilepre[s];
        const int64_t a = w.off[s];
        const int64_t base = a + (int64_t)i * w.ptile;
        d.base = base;
        d.seg_base = a;
        d.cnt = (int)min((int64_t)w.ptile, w.off[s + 1] - base);
        d.seg = s;
        d.idx = i;
        d.nt = w.tilecnt[s];
        d.grp = w.grouppre[s] + i / kGroupTiles;
        d.pad = 0;
    }
    w.tiles[t] = d;
}

// min/max of every histogram tile (one workgroup per tile).
template <typename T, int NT>
__device__ __forceinline__ void block_minmax(T& mn, T& mx, T* rmn, T* rmx) {
    const int lane = lane_id(), wave = threadIdx.x / kWave;
    T a = wave_reduce_min(mn), b = wave_reduce_max(mx);
    if (lane == 0) {
        rmn[wave] = a;
        rmx[wave] = b;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NT / kWave; q++) {
        a = rmn[q] < a ? rmn[q] : a;
        b = rmx[q] > b ? rmx[q] : b;
    }
    mn = a;
    mx = b;
    __syncthreads();
}

// Per tile: min and max, and the bucket counts under the tile's own digit
// plan when the tile holds no negative key (beta 0, p the largest power of
// ten not above the tile's max; images of unsigned keys always, with their
// fixed beta).  If the segment's plan has beta 0 as well,
// it has the same p or a larger one, so the histogram pass only has to fix
// the tiles whose p is smaller (every key then has digit 0) instead of
// reading the keys again.  Keys are read strided (thread t: t, t + NT, ...),
// coalesced per wave, and kept in registers for the count.
template <typename K, int NBK, int HT>
__global__ __launch_bounds__(HT / kHistVT) void k_range(Work<K> w) {
    constexpr int VT = kHistVT, NT = HT / VT;
    __shared__ K rmn[NT / kWave], rmx[NT / kWave];
    __shared__ uint32_t red[NT / kWave][5];
    __shared__ uint32_t h[NBK >= 100 ? NBK : 1];
    const int t = (int)xcd_unit(blockIdx.x, gridDim.x);
    const TileDesc td = w.tiles[t];
    if (td.cnt == 0) return;
    const int tid = threadIdx.x;
    const int cnt = td.cnt;
    const K* src = w.keys + td.base;
    const K k0 = src[0];
    K ks[VT];
    // a full, 16-byte aligned tile is read in 16-byte vectors (consecutive
    // threads on consecutive vectors), any other strided by element (then
    // key v of a thread is element tid + v*NT; the counts need no order)
    using V = typename Vec16<K>::type;
    constexpr int E = Vec16<K>::n;
    const bool vec = cnt == HT && ((uintptr_t)src & 15) == 0;
    if (vec) {
        const V* sv = reinterpret_cast<const V*>(src);
#pragma unroll
        for (int j = 0; j < VT / E; j++) {
            const V x = sv[tid + j * NT];
#pragma unroll
            for (int e = 0; e < E; e++) ks[j * E + e] = (K)Vec16<K>::get(x, e);
        }
    } else {
#pragma unroll
        for (int v = 0; v < VT; v++) {
            const int q = tid + v * NT;
            ks[v] = q < cnt ? src[q] : k0;  // k0 leaves the min and max unchanged
        }
    }
    if (w.img) {
#pragma unroll
        for (int v = 0; v < VT; v++) ks[v] = image_of(ks[v], w.img, false);
    }
    K mn = ks[0], mx = ks[0];
#pragma unroll
    for (int v = 1; v < VT; v++) {
        mn = ks[v] < mn ? ks[v] : mn;
        mx = ks[v] > mx ? ks[v] : mx;
    }
    block_minmax<K, NT>(mn, mx, rmn, rmx);
    if (tid == 0) {
        w.tmin[t] = mn;
        w.tmax[t] = mx;
    }
    if (mn < 0 && !w.ufix) {
        if (tid == 0) w.tp[t] = 0;
        return;
    }
    const DigitPlan<K> pl = make_digit_plan<K>(K(0), mx, w.ufix);
    if constexpr (NBK == 10) {
        uint64_t c = 0;  // at most VT = 16 keys per thread: fits the 5-bit fields
#pragma unroll
        for (int v = 0; v < VT; v++) c += (uint64_t)(vec || tid + v * NT < cnt) << (5 * digit_of(pl, ks[v]));
        uint32_t wd[5];
        unpack5(c, wd);
        block_sum5<NT>(wd, red);
        if (tid < 10) w.counts[10 * (int64_t)t + tid] = field16(wd, tid);
    } else {
        // one hundred or one thousand buckets: LDS atomics (block_minmax
        // ended with a barrier), one per run of equal buckets among a
        // thread's keys -- an LDS atomic serves the lanes on one address one
        // at a time, and in a skewed tile most lanes of a wave share a bucket
        for (int b = tid; b < NBK; b += NT) h[b] = 0;
        __syncthreads();
        uint32_t rb = (uint32_t)bucket_of<NBK>(pl, ks[0]), rn = 0;
#pragma unroll
        for (int v = 0; v < VT; v++) {
            if (vec || tid + v * NT < cnt) {
                const uint32_t b = (uint32_t)bucket_of<NBK>(pl, ks[v]);
                if (b != rb) {
                    atomicAdd(&h[rb], rn);
                    rb = b;
                    rn = 0;
                }
                rn++;
            }
        }
        if (rn) atomicAdd(&h[rb], rn);
        __syncthreads();
        for (int b = tid; b < NBK; b += NT) w.counts[NBK * (int64_t)t + b] = h[b];
    }
    if (tid == 0) w.tp[t] = plan_p(pl);
}

// Per large segment: min/max over its tiles, then the decimal digit plan.
template <typename K>
__global__ __launch_bounds__(1024) void k_plans(Work<K> w) {
    __shared__ K rmn[1024 / kWave], rmx[1024 / kWave];
    if (*w.err) return;
    for (int s = blockIdx.x; s < w.nseg; s += gridDim.x) {
        const int nt = w.tilecnt[s];
        if (nt == 0) continue;
        const int t0 = w.tilepre[s];
        K mn = Traits<K>::kMax, mx = Traits<K>::kMin;
#pragma unroll 8
        for (int t = threadIdx.x; t < nt; t += 1024) {
            const K a = w.tmin[t0 + t], b = w.tmax[t0 + t];
            mn = a < mn ? a : mn;
            mx = b > mx ? b : mx;
        }
        block_minmax<K, 1024>(mn, mx, rmn, rmx);
        if (threadIdx.x == 0) w.plans[s] = make_digit_plan<K>(mn, mx, w.ufix);
    }
}

// ------------------------------------------------------------- histogram
// Per tile: how many keys fall in each of the ten buckets.  Layout: for
// segment s, counts[10*tilepre[s] + d*tilecnt[s] + i] (bucket-major, tile
// minor), so one exclusive scan of the whole array yields every tile's write
// offset inside its bucket.
template <typename K, int NBK, int HT>
__global__ __launch_bounds__(kHistNT) void k_hist(Work<K> w, int64_t tiles_bound) {
    __shared__ uint32_t red[kHistNT / kWave][5];
    __shared__ uint32_t h[NBK >= 100 ? NBK : 1];
    __shared__ int64_t slow[kHistNT];
    __shared__ int nslow;
    const int tid = threadIdx.x;
    const int64_t G = gridDim.x;
    // A fixed grid strides over the tiles (most need no work here, and a
    // workgroup per tile would cost a launch of every one of them).  This
    // workgroup's tiles are blockIdx.x + i*G, checked NT at a time, one per
    // thread; the ones whose keys must be counted are listed in LDS and
    // counted by the whole workgroup, one after the other.
    for (int64_t i0 = 0; blockIdx.x + i0 * G < tiles_bound; i0 += kHistNT) {
        if (tid == 0) nslow = 0;
        __syncthreads();
        const int64_t t = blockIdx.x + (i0 + tid) * G;
        if (t < tiles_bound) {
            const TileDesc td = w.tiles[t];
            if (td.cnt > 0) {
                const DigitPlan<K> pl = w.plans[td.seg];
                const uint64_t tp = w.tp[t];
                // counted by k_range under the tile's own plan: the
                // segment's plan, or one with a smaller p (at most a tenth of
                // the segment's).  Ten buckets: every key then has digit 0.
                // One hundred: every key is in bucket 0 when the tile's p is
                // at most a hundredth of the segment's; at a tenth the keys
                // are counted again.  One thousand: counted again (filling
                // a thousand zeros here would take one thread as long).
                const uint64_t ps = plan_p(pl);
                const bool own = (w.ufix || pl.beta == 0) && tp != 0;
                if (own && tp != ps && (NBK == 10 || (NBK == 100 && tp <= ps / 100))) {
                    uint32_t* out = w.counts + NBK * t;
                    out[0] = (uint32_t)td.cnt;
                    for (int d = 1; d < NBK; d++) out[d] = 0;
                } else if (!own || tp != ps) {
                    slow[atomicAdd(&nslow, 1)] = t;
                }
            }
        }
        __syncthreads();
        const int ns = nslow;
        for (int k = 0; k < ns; k++) {
            const TileDesc td = w.tiles[slow[k]];
            const DigitPlan<K> pl = w.plans[td.seg];
            if constexpr (NBK == 10) {
                uint64_t c = 0;  // a thread sees at most 16 + 3 + 3 keys: fits the 5-bit fields
                load_keys_imaged<K, kHistNT, kHistTile>(w.keys + td.base, td.cnt, w.img,
                                                        [&](int, K k) { c += 1ull << (5 * digit_of(pl, k)); });
                uint32_t wd[5];
                unpack5(c, wd);
                block_sum5<kHistNT>(wd, red);
                if (tid < 10) w.counts[10 * slow[k] + tid] = field16(wd, tid);
            } else {
                for (int b = tid; b < NBK; b += kHistNT) h[b] = 0;
                __syncthreads();
                // one atomic per run of equal buckets, as in k_range
                uint32_t rb = 0, rn = 0;
                load_keys_imaged<K, kHistNT, HT>(w.keys + td.base, td.cnt, w.img, [&](int, K k) {
                    const uint32_t b = (uint32_t)bucket_of<NBK>(pl, k);
                    if (b != rb) {
                        if (rn) atomicAdd(&h[rb], rn);
                        rb = b;
                        rn = 0;
                    }
                    rn++;
                });
                if (rn) atomicAdd(&h[rb], rn);
                __syncthreads();
                for (int b = tid; b < NBK; b += kHistNT) w.counts[NBK * slow[k] + b] = h[b];
                __syncthreads();
            }
        }
        __syncthreads();
    }
}

// Column pass over the tile-major counts: one workgroup per group of up to
// kGroupTiles consecutive tiles of one segment, one thread per bucket,
// walking the group's tiles in order: intra = the bucket's count so far in
// the group, and the group's sum, stored bucket-major inside the segment
// (bucket b of group gi of segment s at nbk*grouppre[s] + b*groupcnt[s] + gi)
// for the scan that follows.
template <int NBK>
constexpr int kColNT = (NBK + kWave - 1) / kWave * kWave;  // one thread per bucket, whole waves
template <int NBK>
__global__ __launch_bounds__(kColNT<NBK>) void k_colsum(const int32_t* tilepre, const int32_t* tilecnt,
                                                                const int32_t* grouppre, const int32_t* groupcnt,
                                                                int32_t nseg, const uint32_t* err,
                                                                const uint32_t* __restrict__ counts,
                                                                uint32_t* __restrict__ intra, uint32_t* __restrict__ gsum) {
    if (*err) return;
    const int g = blockIdx.x;
    if (g >= grouppre[nseg]) return;
    const int b = threadIdx.x;
    if (b >= NBK) return;
    const int s = owner_of(grouppre, nseg, g);
    const int gi = g - grouppre[s];
    const int64_t t0 = tilepre[s] + (int64_t)gi * kGroupTiles;
    const int cnt = min(kGroupTiles, tilecnt[s] - gi * kGroupTiles);
    const uint32_t* src = counts + NBK * t0 + b;
    uint32_t* dst = intra + NBK * t0 + b;
    uint32_t run = 0;
    for (int i0 = 0; i0 < cnt; i0 += 8) {  // eight loads in flight before their stores
        uint32_t c[8];
#pragma unroll
        for (int j = 0; j < 8; j++) c[j] = i0 + j < cnt ? src[(int64_t)NBK * (i0 + j)] : 0u;
#pragma unroll
        for (int j = 0; j < 8; j++) {
            if (i0 + j < cnt) dst[(int64_t)NBK * (i0 + j)] = run;
            run += c[j];
        }
    }
    gsum[(int64_t)NBK * grouppre[s] + (int64_t)b * groupcnt[s] + gi] = run;
}

// Group bases: one thread per (group, bucket), the group's start in the
// bucket relative to its segment's first key, stored tile-major like the
// counts (row g holds buckets 0 .. nbk-1).
template <typename K>
__global__ void k_gbase(Work<K> w, int64_t bound) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= bound || *w.err) return;
    const int nbk = w.nbk;
    const int g = (int)(e / nbk), b = (int)(e - (int64_t)g * nbk);
    if (g >= w.grouppre[w.nseg]) return;
    const int s = owner_of(w.grouppre, w.nseg, g);
    const int64_t base = (int64_t)nbk * w.grouppre[s];
    w.gbase[e] = (int32_t)(w.gpos[base + (int64_t)b * w.groupcnt[s] + (g - w.grouppre[s])] - w.gpos[base]);
}

// Bucket table entry j (bucket d of segment s) from the bucket's start st,
// relative to the segment's first key, and its size sz: start and size, its
// local-sort tiles and merge chunks, the ten-bucket bounds output (with one
// hundred or one thousand buckets, bound b is the start of bucket nbk/10*b)
// and its merge rounds, which it returns.
template <typename K>
__device__ __forceinline__ int btab_entry(const Work<K>& w, int64_t j, int s, int d, int64_t st, int64_t sz) {
    const int nbk = w.nbk;
    const int per = nbk / 10;  // buckets per ten-bucket bound
    const int64_t a = w.off[s];
    w.bstart[j] = a + st;
    w.bsize[j] = sz;
    w.tsc[j] = (int32_t)((sz + w.tile - 1) / w.tile);
    w.mcc[j] = (int32_t)((sz + w.nv - 1) / w.nv);
    if (d % per == 0) w.bounds_out[11 * (int64_t)s + d / per] = st;
    if (d == 0) w.bounds_out[11 * (int64_t)s + 10] = w.off[s + 1] - a;
    // a bucket that spans one key value is in order after the scatter
    uint64_t lo, width;
    bucket_span(w.plans[s], nbk, d, lo, width);
    const bool one = width == 1;
    const int r = one ? 0 : merge_rounds(sz, w.tile, w.fanin);
    w.brounds[j] = r | (one ? kConstBucket : 0);
    return r;
}

// Local-sort descriptor `item` (partitions of all buckets in bucket order,
// then empty slots up to the bound).
template <typename K>
__device__ __forceinline__ void sdesc_item(const Work<K>& w, int64_t item) {
    const int nb = w.nbk * w.nseg;
    SortDesc d{0, 0, 0, 0, 0};
    if (!*w.err && item < w.tsp[nb]) {
        const int j = owner_of(w.tsp, nb, (int)item);
        const int64_t i = item - w.tsp[j];
        const int64_t size = w.bsize[j];
        d.start = w.bstart[j] + i * w.tile;
        d.cnt = (int)min((int64_t)w.tile, size - i * w.tile);
        const int32_t br = w.brounds[j];
        // bit 1: an odd run of its group; bit 2: a bucket of one key value
        d.odd = (bucket_rounds(br) & 1) | (int)(i & 1) << 1 | ((br & kConstBucket) ? 4 : 0) |
                (bucket_rounds(br) == 0 ? 8 : 0);
        d.bucket = j;
        d.sbase = (int32_t)(sample_base(w.bstart[j], w.msp[j]) + i * w.tile / kSampleBlock);
    }
    w.sdesc[item] = d;
}

// Bucket table: btab_entry for every bucket of every segment.
template <typename K>
__global__ void k_btab(Work<K> w) {
    if (*w.err) return;
    // one thread per bucket of every segment
    const int nbk = w.nbk;
    const int64_t nbt = (int64_t)nbk * w.nseg;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < nbt; j += (int64_t)gridDim.x * blockDim.x) {
        const int s = (int)(j / nbk), d = (int)(j - (int64_t)s * nbk);
        const int nt = w.tilecnt[s];
        const int64_t a = w.off[s];
        if (nt == 0) {
            w.bstart[j] = a;
            w.bsize[j] = 0;
            w.tsc[j] = 0;
            w.mcc[j] = 0;
            w.brounds[j] = 0;
            continue;
        }
        // the scan of the group sums, bucket-major inside the segment
        const int ng = w.groupcnt[s];
        const int64_t base = (int64_t)nbk * w.grouppre[s];
        const int64_t p0 = w.gpos[base];
        const int64_t st = w.gpos[base + (int64_t)d * ng] - p0;
        const int64_t en = w.gpos[base + (int64_t)(d + 1) * ng] - p0;
        const int r = btab_entry(w, j, s, d, st, en - st);
        if (r > 0) atomicMax(w.rounds, r);
    }
}

// A plain sort whose partition tiles form one group (at most kGroupTiles
// tiles, so every start fits 32 bits): k_colsum, the scan of the group
// sums, k_gbase, k_btab, the scans of the tile and chunk counts and k_sdesc
// (descriptors 0 .. ts_bound-1) in one workgroup, one thread per bucket.
// Such an array waits on the chain of launches, not on this work.
template <typename K, int NBK>
__global__ __launch_bounds__(kColNT<NBK>) void k_offsets1(Work<K> w, int64_t ts_bound) {
    constexpr int NT = kColNT<NBK>;
    __shared__ int32_t red[NT / kWave];
    const int b = threadIdx.x;
    if (*w.err) {
        for (int64_t item = b; item < ts_bound; item += NT) w.sdesc[item] = SortDesc{0, 0, 0, 0, 0};
        return;
    }
    const int nt = w.tilecnt[0];
    // the bucket's column of counts: each tile's in-group prefix, its size
    int32_t run = 0;
    if (b < NBK) {
        const uint32_t* src = w.counts + b;
        uint32_t* dst = w.intra + b;
        for (int i0 = 0; i0 < nt; i0 += 8) {  // eight loads in flight before their stores
            uint32_t c[8];
#pragma unroll
            for (int j = 0; j < 8; j++) c[j] = i0 + j < nt ? src[NBK * (i0 + j)] : 0u;
#pragma unroll
            for (int j = 0; j < 8; j++) {
                if (i0 + j < nt) dst[NBK * (i0 + j)] = (uint32_t)run;
                run += (int32_t)c[j];
            }
        }
    }
    int32_t all;
    const int32_t st = block_excl_scan<int32_t, NT>(run, all, red);
    int32_t tsc = 0, mcc = 0;
    if (b < NBK) {
        w.gbase[b] = st;
        const int r = btab_entry(w, b, 0, b, st, run);
        if (r > 0) atomicMax(w.rounds, r);
        tsc = w.tsc[b];
        mcc = w.mcc[b];
    }
    int32_t ttot, mtot;
    const int32_t tp = block_excl_scan<int32_t, NT>(tsc, ttot, red);
    const int32_t mp = block_excl_scan<int32_t, NT>(mcc, mtot, red);
    if (b < NBK) {
        w.tsp[b] = tp;
        w.msp[b] = mp;
    }
    if (b == 0) {
        w.tsp[NBK] = ttot;
        w.msp[NBK] = mtot;
    }
    // the bucket table and its scans, written by every thread above, are
    // visible to the whole workgroup after the barrier
    __syncthreads();
    for (int64_t item = b; item < ts_bound; item += NT) sdesc_item(w, item);
}

// ---------------------------------------------------------------- scatter
// One stable counting pass of a tile held in LDS by a decimal digit 0..9:
// every thread ranks its VT consecutive keys (blocked) with packed
// per-thread counters, a block scan gives each thread's start per digit, and
// the keys are staged back grouped by digit, in input order inside a digit.
// dig(key, tag_in) returns the key's digit (bits 0..3) and the byte staged
// with the key in sd (bits 8..15); with TAGIN, tag_in is the byte the key
// carried in (a thread's VT = 16 tags come in 16-byte LDS reads), else 0.
// Tags are bytes, or 16-bit words for one thousand buckets.  tot receives
// the tile's per-digit totals (packed).
template <typename K, bool PAIRS, bool FULL, bool TAGIN, typename T, typename Dig>
__device__ __forceinline__ void digit_pass(K* sk, uint32_t* sv, T* sd, uint32_t (*red)[5],
                                           uint16_t (*offs)[kHistNT], int cnt, Dig&& dig, uint32_t (&tot)[5]) {
    constexpr int NT = kHistNT, VT = kHistVT;
    static_assert(VT == 16, "a thread's tags are whole 16-byte words");
    static_assert(sizeof(T) == 1 || sizeof(T) == 2, "8- or 16-bit tags");
    constexpr int TPW = 4 / (int)sizeof(T);  // tags per 32-bit word
    // each thread's staging start per digit, read back by digit: an indexed
    // LDS read is cheaper than selecting among registers, but the 5 KB cost
    // 64-bit keys and pairs a resident workgroup, so they select instead
    constexpr bool kOffsLds = sizeof(K) == 4 && !PAIRS;
    const int tid = threadIdx.x;
    uint32_t pk[VT];  // tag << 16 | rank << 4 | digit (digit 15 = no key)
    uint32_t tg[VT / TPW];
#pragma unroll
    for (int j = 0; j < VT / TPW; j++) tg[j] = 0;
    if constexpr (TAGIN) {
        const uint4* src = reinterpret_cast<const uint4*>(sd + tid * VT);
#pragma unroll
        for (int j = 0; j < VT / TPW / 4; j++) {
            const uint4 x = src[j];
            tg[4 * j] = x.x;
            tg[4 * j + 1] = x.y;
            tg[4 * j + 2] = x.z;
            tg[4 * j + 3] = x.w;
        }
    }
    uint64_t c = 0;
#pragma unroll
    for (int v = 0; v < VT; v++) {
        const int q = tid * VT + v;
        const bool ok = FULL || q < cnt;
        const int qq = ok ? q : 0;
        constexpr uint32_t kTagMask = sizeof(T) == 1 ? 0xFFu : 0xFFFFu;
        const uint32_t dt = dig(sk[lds_pad<K>(qq)], (tg[v / TPW] >> (8 * (int)sizeof(T) * (v % TPW))) & kTagMask);
        const uint32_t d = dt & 15u;
        const uint32_t r = (((uint32_t)(c >> (5 * d)) & 31u) << 4) | d;
        pk[v] = ok ? (((dt >> 8) & kTagMask) << 16) | r : 15u;
        c += ok ? (1ull << (5 * d)) : 0ull;
    }
    uint32_t wd[5];
    unpack5(c, wd);
    block_excl5<NT>(wd, tot, red);  // ends with a barrier: sk, sv and sd may be overwritten
    // tile-local digit starts folded into the packed prefix
    uint32_t run = 0;
#pragma unroll
    for (int m = 0; m < 5; m++) {
        const uint32_t lo = run;
        run += tot[m] & 0xFFFFu;
        const uint32_t hi = run;
        run += tot[m] >> 16;
        wd[m] += lo | (hi << 16);
    }
    if constexpr (kOffsLds) {
#pragma unroll
        for (int m = 0; m < 5; m++) {
            offs[2 * m][tid] = (uint16_t)(wd[m] & 0xFFFFu);
            offs[2 * m + 1][tid] = (uint16_t)(wd[m] >> 16);
        }
    }
    // the thread's keys (and payload) again, read by every thread before any
    // thread stages its own: holding them in registers across the scan
    // above cost a resident wave per SIMD
    K key[VT];
    uint32_t val[PAIRS ? VT : 1];
#pragma unroll
    for (int v = 0; v < VT; v++) {
        const int q = tid * VT + v;
        const int qq = (FULL || q < cnt) ? q : 0;
        key[v] = sk[lds_pad<K>(qq)];
        if constexpr (PAIRS) val[v] = sv[qq];
    }
    __syncthreads();
#pragma unroll
    for (int v = 0; v < VT; v++) {
        const uint32_t d = pk[v] & 15u;
        if (FULL || d < 10) {  // a full tile has no empty slot: no branch
            const uint32_t start = kOffsLds ? (uint32_t)offs[kOffsLds ? d : 0][tid] : field16(wd, (int)d);
            const int sp = (int)(start + ((pk[v] >> 4) & 31u));
            sk[lds_pad<K>(sp)] = key[v];
            sd[sp] = (T)(pk[v] >> 16);
            if constexpr (PAIRS) sv[sp] = val[v];
        }
    }
}

// Stable one-step MSD scatter (Section 3.4: the master divides the keys into
// ten parts by most significant digit; NBK = 100 and 1000 are the finer two-
// and three-digit splitters, here for stable pairs).  Per tile: the keys are
// grouped by bucket in LDS -- ten buckets by one counting pass on the digit,
// one hundred by two passes and one thousand by three, from the last digit
// of the bucket to the first (each pass stable, so each keeps the previous
// one's order inside a digit) -- and runs of consecutive keys are written to
// their buckets in the scratch copy.  The bucket of a staged key travels
// with it in a byte (16-bit word for one thousand buckets), so each key's
// bucket is computed once.
template <typename K, bool PAIRS, int NBK>
__global__ __launch_bounds__(kHistNT, (PAIRS && NBK >= 100 && sizeof(K) == 4) ? 3 : 1) void k_scatter(Work<K> w) {
    static_assert(NBK == 10 || NBK == 100 || NBK == 1000, "ten, one hundred or one thousand buckets");
    constexpr int NT = kHistNT, VT = kHistVT, HT = kHistTile;
    constexpr int BPT = (NBK + NT - 1) / NT;  // buckets per thread for the counts scan
    using T = std::conditional_t<(NBK > 256), uint16_t, uint8_t>;
    __shared__ K sk[lds_padded_size<K>(HT)];
    __shared__ uint32_t sv[PAIRS ? HT : 1];
    __shared__ __align__(16) T sd[HT];
    __shared__ uint32_t red[NT / kWave][5];
    constexpr bool kOffsLds = sizeof(K) == 4 && !PAIRS;
    __shared__ int32_t dbase[NBK];  // element index (n < 2^31) of bucket d's run, minus its staging start
    __shared__ uint16_t offs[kOffsLds ? 10 : 1][NT];
    const int t = (int)xcd_unit(blockIdx.x, gridDim.x);
    const TileDesc td = w.tiles[t];
    if (td.cnt == 0) return;
    const int tid = threadIdx.x;
    const int64_t base = td.base;
    const int cnt = td.cnt;
    const DigitPlan<K> pl = w.plans[td.seg];
    // the tile's write offset in buckets tid*BPT .. tid*BPT+BPT-1 (and, with
    // one hundred or one thousand buckets, its counts there), loaded before
    // the keys so that both round trips overlap
    uint32_t cb[BPT];
    int64_t gp[BPT];
#pragma unroll
    for (int j = 0; j < BPT; j++) {
        const int b = tid * BPT + j;
        cb[j] = 0;
        gp[j] = 0;
        if (b < NBK) {
            gp[j] = (int64_t)w.gbase[NBK * (int64_t)td.grp + b] + w.intra[NBK * (int64_t)t + b];
            if constexpr (NBK >= 100) cb[j] = w.counts[NBK * (int64_t)t + b];
        }
    }
    // 1. load in natural order (16-byte body)
    load_run<K, NT, HT>(w.keys + base, cnt, [&](int q, K k) { sk[lds_pad<K>(q)] = k; });
    if constexpr (PAIRS) load_run<uint32_t, NT, HT>(w.vals + base, cnt, [&](int q, uint32_t v) { sv[q] = v; });
    if constexpr (NBK == 10) {
        if (tid < 10) dbase[tid] = (int32_t)(td.seg_base + gp[0]);
    } else {
        // the tile's start of each bucket: exclusive scan of its counts
        uint32_t mine = 0;
#pragma unroll
        for (int j = 0; j < BPT; j++) mine += cb[j];
        uint32_t all;
        uint32_t ls = block_excl_scan<uint32_t, NT>(mine, all, &red[0][0]);
#pragma unroll
        for (int j = 0; j < BPT; j++) {
            const int b = tid * BPT + j;
            if (b < NBK) dbase[b] = (int32_t)(td.seg_base + gp[j] - (int64_t)ls);
            ls += cb[j];
        }
    }
    __syncthreads();
    if (w.img) {
        // order images taken in LDS, after the load: the plain load keeps
        // its code
        const int mode = w.img;
        for (int q = tid; q < cnt; q += NT) sk[lds_pad<K>(q)] = image_of(sk[lds_pad<K>(q)], mode, false);
        __syncthreads();
    }
    uint32_t tot[5];
    auto passes = [&](auto full) {
        constexpr bool F = decltype(full)::value;
        if constexpr (NBK == 10) {
            digit_pass<K, PAIRS, F, false>(sk, sv, sd, red, offs, cnt, [&](K k, uint32_t) {
                const uint32_t d = (uint32_t)digit_of(pl, k);
                return d | (d << 8);
            }, tot);
        } else if constexpr (NBK == 1000) {
            // three passes: the last digit of b, the middle one, the first
            // (b / 10 = b * 205 >> 11 and b / 100 = b * 41 >> 12, exact for
            // b < 1000)
            digit_pass<K, PAIRS, F, false>(sk, sv, sd, red, offs, cnt, [&](K k, uint32_t) {
                const uint32_t b = (uint32_t)bucket3_of(pl, k);
                return (b - 10u * ((b * 205u) >> 11)) | (b << 8);
            }, tot);
            __syncthreads();
            digit_pass<K, PAIRS, F, true>(sk, sv, sd, red, offs, cnt, [&](K, uint32_t b) {
                const uint32_t q = (b * 205u) >> 11;
                return (q - 10u * ((q * 205u) >> 11)) | (b << 8);
            }, tot);
            __syncthreads();
            digit_pass<K, PAIRS, F, true>(sk, sv, sd, red, offs, cnt, [&](K, uint32_t b) {
                return ((b * 41u) >> 12) | (b << 8);
            }, tot);
        } else {
            // pass 1 on the second digit, pass 2 on the first; b = 10 d1 + d2
            // (d1 = b * 205 >> 11, exact for b < 100)
            digit_pass<K, PAIRS, F, false>(sk, sv, sd, red, offs, cnt, [&](K k, uint32_t) {
                const uint32_t b = (uint32_t)bucket2_of(pl, k);
                return (b - 10u * ((b * 205u) >> 11)) | (b << 8);
            }, tot);
            __syncthreads();
            digit_pass<K, PAIRS, F, true>(sk, sv, sd, red, offs, cnt, [&](K, uint32_t b) {
                return ((b * 205u) >> 11) | (b << 8);
            }, tot);
        }
    };
    if (cnt == HT)
        passes(std::true_type{});
    else
        passes(std::false_type{});
    if constexpr (NBK == 10) {
        if (tid < 10) {  // dbase[d] -= tile-local start of bucket d
            uint32_t st = 0, r2 = 0;
#pragma unroll
            for (int d = 0; d < 10; d++) {
                st = (d == tid) ? r2 : st;
                r2 += (tot[d >> 1] >> ((d & 1) * 16)) & 0xFFFFu;
            }
            dbase[tid] -= (int32_t)st;
        }
    }
    __syncthreads();
    // 2. coalesced runs out to the buckets (a per-bucket loop of 16-byte
    //    stores measured no faster for keys and slower for pairs)
    auto write_out = [&](auto full) {
#pragma unroll
        for (int j = 0; j < VT; j++) {
            const int q = j * NT + tid;
            if (decltype(full)::value || q < cnt) {
                const K k = sk[lds_pad<K>(q)];
                const int b = sd[q];
                const uint32_t dst = (uint32_t)(dbase[b] + q);
                w.skeys[dst] = k;
                if constexpr (PAIRS) w.svals[dst] = sv[q];
            }
        }
    };
    if (cnt == HT)
        write_out(std::true_type{});
    else
        write_out(std::false_type{});
}

// Keys-only scatter with one hundred or one thousand buckets.  The order of
// the keys inside a bucket cannot be seen in the result (equal keys are
// identical, and the local sorts order the rest), so no stable pass is
// needed: each thread holds its keys in registers (read straight from
// memory), takes the next slots of their buckets from LDS cursors (the tile's
// counts give every bucket exactly its slots), stages them there, and the
// staged runs go out coalesced.  Lanes on one LDS address are served one at
// a time, so in a tile where some bucket is large each run of equal buckets
// among a thread's keys takes all its slots with one atomic add.  One
// hundred buckets keep each staged key's bucket in a byte; one thousand
// recompute it from the key on the way out (two bytes a key would cost the
// second resident workgroup).
template <typename K, int NBK>
__global__ __launch_bounds__(ScatterShape<NBK>::NT) void k_scatter_keys(Work<K> w) {
    static_assert(NBK == 100 || NBK == 1000, "one hundred or one thousand buckets");
    constexpr int NT = ScatterShape<NBK>::NT, VT = ScatterShape<NBK>::VT, HT = NT * VT;
    static_assert(HT == PartShape<NBK>::HT, "the scatter tile is the partition tile");
    constexpr int BPT = (NBK + NT - 1) / NT;  // buckets per thread for the counts scan
    constexpr bool kTag = NBK <= 256;
    using V = typename Vec16<K>::type;
    constexpr int E = Vec16<K>::n;
    __shared__ K sk[lds_padded_size<K>(HT)];
    __shared__ __align__(16) uint8_t sd[kTag ? HT : 1];
    __shared__ uint32_t red[NT / kWave][5];
    __shared__ int32_t dbase[NBK];  // element index (n < 2^31) of bucket b's run, minus its staging start
    __shared__ uint32_t cur[NBK];   // bucket b's next free staging slot
    __shared__ int heavy;           // some bucket holds more than an eighth of the tile
    const int t = (int)xcd_unit(blockIdx.x, gridDim.x);
    const TileDesc td = w.tiles[t];
    if (td.cnt == 0) return;
    const int tid = threadIdx.x;
    const int cnt = td.cnt;
    const DigitPlan<K> pl = w.plans[td.seg];
    // the tile's write offset and count in buckets tid*BPT .. tid*BPT+BPT-1
    uint32_t cb[BPT];
    int64_t gp[BPT];
#pragma unroll
    for (int j = 0; j < BPT; j++) {
        const int b = tid * BPT + j;
        cb[j] = 0;
        gp[j] = 0;
        if (b < NBK) {
            gp[j] = (int64_t)w.gbase[NBK * (int64_t)td.grp + b] + w.intra[NBK * (int64_t)t + b];
            cb[j] = w.counts[NBK * (int64_t)t + b];
        }
    }
    // the keys, straight into registers: a full, 16-byte aligned tile in
    // 16-byte vectors (consecutive threads on consecutive vectors), any other
    // strided by element (key v of a thread is element tid + v*NT)
    const K* src = w.keys + td.base;
    K ks[VT];
    const bool vec = cnt == HT && ((uintptr_t)src & 15) == 0;
    if (vec) {
        const V* sv = reinterpret_cast<const V*>(src);
#pragma unroll
        for (int j = 0; j < VT / E; j++) {
            const V x = sv[tid + j * NT];
#pragma unroll
            for (int e = 0; e < E; e++) ks[j * E + e] = (K)Vec16<K>::get(x, e);
        }
    } else {
#pragma unroll
        for (int v = 0; v < VT; v++) {
            const int q = tid + v * NT;
            ks[v] = q < cnt ? src[q] : src[0];
        }
    }
    if (w.img) {
#pragma unroll
        for (int v = 0; v < VT; v++) ks[v] = image_of(ks[v], w.img, false);
    }
    // the tile's start of each bucket: exclusive scan of its counts (its
    // barriers order the flag's reset before the writes of 1)
    if (tid == 0) heavy = 0;
    {
        uint32_t mine = 0;
#pragma unroll
        for (int j = 0; j < BPT; j++) mine += cb[j];
        uint32_t all;
        uint32_t ls = block_excl_scan<uint32_t, NT>(mine, all, &red[0][0]);
#pragma unroll
        for (int j = 0; j < BPT; j++) {
            const int b = tid * BPT + j;
            if (b < NBK) {
                dbase[b] = (int32_t)(td.seg_base + gp[j] - (int64_t)ls);
                cur[b] = ls;
                if (8 * cb[j] > (uint32_t)cnt) heavy = 1;
            }
            ls += cb[j];
        }
    }
    uint32_t bk[VT];
#pragma unroll
    for (int v = 0; v < VT; v++) bk[v] = (uint32_t)bucket_of<NBK>(pl, ks[v]);
    __syncthreads();
    // key v is real when the tile is full or tid + v*NT < cnt (so the real
    // keys of a thread are its first ones)
    if (heavy) {
        uint32_t len[VT];
        len[VT - 1] = 1;
#pragma unroll
        for (int v = VT - 2; v >= 0; v--)
            len[v] = bk[v] == bk[v + 1] && (vec || tid + (v + 1) * NT < cnt) ? len[v + 1] + 1 : 1u;
        uint32_t slot = 0;
#pragma unroll
        for (int v = 0; v < VT; v++) {
            if (vec || tid + v * NT < cnt) {
                if (v == 0 || bk[v] != bk[v - 1])
                    slot = atomicAdd(&cur[bk[v]], len[v]);
                else
                    slot++;
                sk[lds_pad<K>((int)slot)] = ks[v];
                if constexpr (kTag) sd[slot] = (uint8_t)bk[v];
            }
        }
    } else {
#pragma unroll
        for (int v = 0; v < VT; v++) {
            if (vec || tid + v * NT < cnt) {
                const uint32_t slot = atomicAdd(&cur[bk[v]], 1u);
                sk[lds_pad<K>((int)slot)] = ks[v];
                if constexpr (kTag) sd[slot] = (uint8_t)bk[v];
            }
        }
    }
    __syncthreads();
    // coalesced runs out to the buckets
#pragma unroll
    for (int j = 0; j < VT; j++) {
        const int q = j * NT + tid;
        if (q < cnt) {
            const K k = sk[lds_pad<K>(q)];
            const int b = kTag ? (int)sd[q] : bucket_of<NBK>(pl, k);
            w.skeys[(uint32_t)(dbase[b] + q)] = k;
        }
    }
}

// Materialises the flat list of local-sort partitions (one thread per slot).
template <typename K>
__global__ void k_sdesc(Work<K> w, int64_t bound) {
    const int64_t item = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (item < bound) sdesc_item(w, item);
}

// First and last key of every 32-key block of a sorted partition that starts
// on a block boundary (the split-point searches of fan-in-4 rounds probe
// these dense samples before the keys).
// Block last keys are read only from runs 0 and 2 of a group (the A side of
// its merge paths): `last` is false for the others.
template <typename K, int NT, typename KeyAt>
__device__ __forceinline__ void store_block_samples(const Work<K>& w, int64_t sbase, int cnt, bool last,
                                                    KeyAt&& key_at) {
    for (int b = threadIdx.x; b * kSampleBlock < cnt; b += NT) {
        w.smpf[sbase + b] = key_at(b * kSampleBlock);
        if (last && (b + 1) * kSampleBlock <= cnt) w.smpl[sbase + b] = key_at(b * kSampleBlock + kSampleBlock - 1);
    }
}

// -------------------------------------------------------------- tile sort
// Local sort of each T-key partition of every bucket (Section 3.4: each
// thread of a node sorts its partition; here one workgroup per partition, in
// LDS).  Partitions start at the bucket's first key.  A bucket that needs P
// merge rounds is written to the caller's buffer when P is even and to the
// scratch copy when P is odd, so that its last round lands in the caller's
// buffer with no final copy.
template <typename K, bool PAIRS, int NT, int VT, bool BU>
__global__ __launch_bounds__(NT) void k_tilesort(Work<K> w) {
    using W = typename WordOf<K, PAIRS>::type;
    constexpr int NV = NT * VT;
    __shared__ W words[lds_padded_size<W>(NV)];
    __shared__ uint32_t sv[PAIRS ? NV : 1];
    __shared__ int sp[NT + 1];
    const SortDesc sd = w.sdesc[blockIdx.x];
    if (sd.cnt == 0) return;
    const int tid = threadIdx.x;
    {
        const int64_t start = sd.start;
        const int cnt = sd.cnt;
        K* dk = ((sd.odd & 1) ? w.skeys : w.keys) + start;
        uint32_t* dv = PAIRS ? ((sd.odd & 1) ? w.svals : w.vals) + start : nullptr;
        const K* srck = w.skeys + start;
        const uint32_t* srcv = PAIRS ? w.svals + start : nullptr;
        // the bucket's output is final (no merge round follows) and the keys
        // are order images: undo the image as they are stored
        const int mode = w.img;
        const bool fin = (sd.odd & 8) && mode != 0;
        if (sd.odd & 4) {
            // the bucket's keys all share one value: the scatter left them
            // (and their payload, in input order) as the sort would; copy
            // them to the caller's buffer (no merge round follows)
            if (w.img) {
                for (int q = tid; q < cnt; q += NT) dk[q] = image_of(srck[q], w.img, true);
            } else {
                copy_run<K, NT>(dk, srck, cnt);
            }
            if constexpr (PAIRS) copy_run<uint32_t, NT>(dv, srcv, cnt);
            return;
        }
        if constexpr (PAIRS) {
            // Every key of the partition lies in its bucket's span, so
            // u - lo (u = k - beta) lies in [0, width).  When width fits next
            // to the key's index in a word of the key's width, the sort runs
            // on words (u - lo) << POS | q: the same strict order as the wide
            // composite words, half the LDS traffic and cheaper compares.
            using U = typename Traits<K>::U;
            using NW = U;
            constexpr int BITS = 8 * (int)sizeof(NW);
            constexpr int POS = NV <= 4096 ? 12 : 13;
            static_assert(NV <= (1 << POS), "indices fit the narrow word");
            const DigitPlan<K> pl = w.plans[sd.bucket / w.nbk];
            uint64_t lo, width;
            bucket_span(pl, w.nbk, sd.bucket % w.nbk, lo, width);
            if (width - 1 <= (uint64_t(1) << (BITS - POS)) - 2) {
                const U base = pl.beta + (U)lo;
                NW* wn = reinterpret_cast<NW*>(words);
                load_run<K, NT, NV>(srck, cnt, [&](int q, K k) {
                    wn[lds_pad<NW>(q)] = ((NW)((U)k - base) << POS) | (NW)q;
                });
                load_run<uint32_t, NT, NV>(srcv, cnt, [&](int q, uint32_t v) { sv[q] = v; });
                for (int q = cnt + tid; q < NV; q += NT) wn[lds_pad<NW>(q)] = WordMax<NW>::v;
                __syncthreads();
                block_sort<NW, NT, VT, BU>(wn, sp, cnt);
                auto key_at = [&](int q) { return (K)((U)(lds_at_padded(wn, q) >> POS) + base); };
                store_chunk_keys<K, NT, NV>(dk, cnt, fin, key_at,
                                            [&](int q) { return image_of(key_at(q), mode, true); });
                store_run<uint32_t, NT, NV>(
                    dv, cnt, [&](int q) { return sv[(uint32_t)lds_at_padded(wn, q) & ((1u << POS) - 1)]; });
                if (w.fanin == 4) store_block_samples<K, NT>(w, sd.sbase, cnt, !(sd.odd & 2), key_at);
                return;
            }
        }
        load_run<K, NT, NV>(srck, cnt, [&](int q, K k) { words[lds_pad<W>(q)] = make_word<K, PAIRS>(k, q); });
        if constexpr (PAIRS) load_run<uint32_t, NT, NV>(srcv, cnt, [&](int q, uint32_t v) { sv[q] = v; });
        if (cnt < NV) {  // a bucket's last, shorter partition: pad with the largest word
            for (int q = cnt + tid; q < NV; q += NT) words[lds_pad<W>(q)] = WordMax<W>::v;
        }
        __syncthreads();
        block_sort<W, NT, VT, BU>(words, sp, cnt);
        auto key_at = [&](int q) { return word_key<K, PAIRS>(lds_at_padded(words, q)); };
        store_chunk_keys<K, NT, NV>(dk, cnt, fin, key_at, [&](int q) { return image_of(key_at(q), mode, true); });
        if constexpr (PAIRS)
            store_run<uint32_t, NT, NV>(dv, cnt, [&](int q) { return sv[pair_pos(lds_at_padded(words, q))]; });
        if (w.fanin == 4) store_block_samples<K, NT>(w, sd.sbase, cnt, !(sd.odd & 2), key_at);
    }
}

// ------------------------------------------------------------ merge rounds
// Round `pass` of the non-recursive merge (Figure 1b; Section 3.2 merge
// rounds): inside every bucket still holding more than one run, runs of
// L = T*2^pass keys are merged pairwise (an odd last run is carried).  The
// output of each pair is cut into chunks of NV keys, one workgroup each.
// k_partition (one thread per chunk) finds the co-rank of the chunk's first
// output -- how many of the outputs before it come from the left run, ties
// going to the left run (stable) -- and writes the chunk's descriptor.
template <typename K>
__global__ __launch_bounds__(256) void k_partition(Work<K> w, int pass, int64_t bound) {
    const int64_t item = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (item >= bound) return;
    const int nb = w.nbk * w.nseg;
    MergeDesc d{0, 0, 0, 0, 0, 0, 0};
    if (!*w.err && pass < *w.rounds && item < w.msp[nb]) {
        const int j = owner_of(w.msp, nb, (int)item);
        const int64_t i = item - w.msp[j];
        const int64_t size = w.bsize[j];
        const int64_t T = w.tile, NV = w.nv;
        const int P = bucket_rounds(w.brounds[j]);
        if (P > pass) {
            const int64_t L = T << pass;
            const int64_t o = i * NV;
            const int64_t ps = (o / (2 * L)) * (2 * L);
            const int64_t a_len = min(L, size - ps);
            const int64_t b_len = max((int64_t)0, min(L, size - ps - L));
            const bool odd = (P - pass) & 1;
            const K* src = odd ? w.skeys : w.keys;
            const int64_t base = w.bstart[j] + ps;
            const K* A = src + base;
            const K* B = A + L;
            const int64_t diag = o - ps;
            const int64_t cs = merge_path_steps64(
                diag, a_len, b_len, L, [&](int64_t x) { return A[x]; }, [&](int64_t x) { return B[x]; });
            d.a = base + cs;
            d.b = base + L + (diag - cs);
            d.out = w.bstart[j] + o;
            d.flags = kActive | (odd ? kFromScratch : 0) | (pass + 1 == P ? kLastPass : 0);
            if (o + NV >= min(ps + 2 * L, size)) {
                d.flags |= kLastChunk;
                d.a_end = base + a_len;
                d.b_end = base + L + b_len;
            }
        }
    }
    w.mdesc[item] = d;
}

template <typename K, bool PAIRS, int NT, int VT>
__global__ __launch_bounds__(NT) void k_merge(Work<K> w, int64_t bound) {
    using W = typename WordOf<K, PAIRS>::type;
    constexpr int NV = NT * VT;
    __shared__ W words[lds_padded_size<W>(NV)];
    __shared__ uint32_t sv[PAIRS ? NV : 1];
    __shared__ int sp[NT + 1];
    const int64_t item = blockIdx.x;
    const MergeDesc md = w.mdesc[item];
    const MergeDesc nx = w.mdesc[item + 1 < bound ? item + 1 : item];
    if (!(md.flags & kActive)) return;
    const int tid = threadIdx.x;
    const bool last = md.flags & kLastChunk;
    const int na = (int)((last ? md.a_end : nx.a) - md.a);
    const int tot = na + (int)((last ? md.b_end : nx.b) - md.b);
    const bool odd = md.flags & kFromScratch;
    const K* pa = (odd ? w.skeys : w.keys) + md.a;
    const K* pb = (odd ? w.skeys : w.keys) + md.b;
    const uint32_t* va = PAIRS ? (odd ? w.svals : w.vals) + md.a : nullptr;
    const uint32_t* vb = PAIRS ? (odd ? w.svals : w.vals) + md.b : nullptr;
    K* dk = (odd ? w.keys : w.skeys) + md.out;
    uint32_t* dv = PAIRS ? (odd ? w.vals : w.svals) + md.out : nullptr;
    auto A = [&](int x) { return lds_at_padded(words, x); };
    auto B = [&](int x) { return lds_at_padded(words, na + x); };
    // the two input windows, side by side in LDS (16-byte bodies)
    {
        const K* const ks[2] = {pa, pb};
        const int cs[2] = {na, tot - na}, os[2] = {0, na};
        load_runs<K, NT, NV, 2>(ks, cs, os, [&](int q, K k) { words[lds_pad<W>(q)] = make_word<K, PAIRS>(k, q); });
        if constexpr (PAIRS) {
            const uint32_t* const vs[2] = {va, vb};
            load_runs<uint32_t, NT, NV, 2>(vs, cs, os, [&](int q, uint32_t x) { sv[q] = x; });
        }
    }
    __syncthreads();
    W v[VT];
    if (tot == NV) {
        const int dt = tid * VT;
        const int ai = merge_path_fixed<NV / 2>(dt, na, NV - na, A, B);
        sp[tid] = ai;
        __syncthreads();
        const int an = (tid == NT - 1) ? na : sp[tid + 1];
        gather_merge_full<W, VT>(words, ai, na + (dt - ai) + VT - 1, an - ai, v);
        __syncthreads();
        const int base = lds_pad<W>(tid * VT);
#pragma unroll
        for (int q = 0; q < VT; q++) words[base + q] = v[q];
    } else {  // a bucket's last, shorter chunk
        const int dt = min(tid * VT, tot);
        const int ai = merge_path_fixed<NV / 2>(dt, na, tot - na, A, B);
        sp[tid] = ai;
        __syncthreads();
        const int an = (tid == NT - 1) ? na : sp[tid + 1];
        const int c = min(tid * VT + VT, tot) - dt;
        gather_merge<W, VT>(words, 0, na, ai, dt - ai, an - ai, c, v);
        __syncthreads();
#pragma unroll
        for (int q = 0; q < VT; q++)
            if (q < c) words[lds_pad<W>(tid * VT + q)] = v[q];
    }
    __syncthreads();
    const int mode = w.img;
    store_chunk_keys<K, NT, NV>(
        dk, tot, (md.flags & kLastPass) && mode != 0,
        [&](int q) { return word_key<K, PAIRS>(lds_at_padded(words, q)); },
        [&](int q) { return image_of(word_key<K, PAIRS>(lds_at_padded(words, q)), mode, true); });
    if constexpr (PAIRS)
        store_run<uint32_t, NT, NV>(dv, tot, [&](int q) { return sv[pair_pos(lds_at_padded(words, q))]; });
}

// ------------------------------------------------- fan-in-4 merge rounds
// Round `round` with fan-in 4: runs of L = T*4^round keys, groups of four
// consecutive runs R0..R3 of a bucket.  X = merge(R0, R1) and Y =
// merge(R2, R3) are sampled every S keys (S = w.nv); a sample's place in the
// group's output is exact from two-way searches only:
//   X sample x (X position k*S): rank = k*S + #R2(< x) + #R3(< x)
//   Y sample y (Y position j*S): rank = j*S + #R0(<= y) + #R1(<= y)
// (equal keys keep run order R0 < R1 < R2 < R3: the stable order).  Between
// two consecutive split points lie at most S keys of X and S of Y, so a
// workgroup of capacity 2S merges them in LDS: W0+W1 and W2+W3, then the two.
// One sample per S keys of a bucket, so the chunk list is the fan-in-2 one.
// A sample's place among all samples of its group, in rank order, follows
// from the same counts: the Y samples before x are those at Y positions
// below #R2(< x) + #R3(< x), ceil of that over S; likewise for y.
template <typename K>
__device__ __forceinline__ K elem_at_corank(const K* A, int64_t na, const K* B, int64_t nb, int64_t c, int64_t d) {
    // the output after the first d of merge(A, B), whose co-rank is c (ties -> A)
    const bool has_a = c < na, has_b = d - c < nb;
    if (has_a && (!has_b || !(B[d - c] < A[c]))) return A[c];
    return B[d - c];
}

template <typename K>
__global__ __launch_bounds__(256) void k_part4(Work<K> w, int round, int64_t bound) {
    const int64_t item = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (item >= bound || round >= *w.rounds) return;  // no bucket needs this round: k_merge4 skips it too
    const int nb = w.nbk * w.nseg;
    Split4 d{};
    if (!*w.err && round < *w.rounds && item < w.msp[nb]) {
        const int j = owner_of(w.msp, nb, (int)item);
        const int64_t i = item - w.msp[j];
        const int64_t size = w.bsize[j];
        const int64_t T = w.tile, S = w.nv;
        const int P = bucket_rounds(w.brounds[j]);
        if (P > round) {
            const int64_t L = T << (2 * round);
            const int64_t o = i * S;
            const int64_t q = o / (2 * L);  // half-group: X of group q/2 when even, Y when odd
            const int64_t g = q >> 1;
            const int64_t gbase = g * 4 * L;
            int64_t len[4];
            for (int k = 0; k < 4; k++) len[k] = max((int64_t)0, min(L, size - gbase - k * L));
            const bool odd = (P - round) & 1;
            const K* src = (odd ? w.skeys : w.keys) + w.bstart[j] + gbase;
            const K* R0 = src;
            const K* R1 = src + L;
            const K* R2 = src + 2 * L;
            const K* R3 = src + 3 * L;
            const int64_t pos = o - q * 2 * L;  // position inside X or Y
            int64_t s0, s1, s2, s3, rank, before;  // before: samples of the other half ranked earlier
            // run k's 32-key blocks: samples from gs + k*L/32 (written by the
            // producer of the runs); searches probe them before the keys
            const int64_t gs = sample_base(w.bstart[j], w.msp[j]) + gbase / kSampleBlock, lb = L / kSampleBlock;
            const K* F = w.smpf + gs;
            const K* Lst = w.smpl + gs;
            if (!(q & 1)) {
                const int64_t c = merge_path_sampled(pos, R0, len[0], Lst, R1, len[1], F + lb);
                const K x = elem_at_corank(R0, len[0], R1, len[1], c, pos);
                s0 = c;
                s1 = pos - c;
                bound2_sampled<false>(R2, len[2], F + 2 * lb, R3, len[3], F + 3 * lb, x, s2, s3);
                rank = pos + s2 + s3;
                before = (s2 + s3 + S - 1) / S;
            } else {
                const int64_t e = merge_path_sampled(pos, R2, len[2], Lst + 2 * lb, R3, len[3], F + 3 * lb);
                const K y = elem_at_corank(R2, len[2], R3, len[3], e, pos);
                bound2_sampled<true>(R0, len[0], F, R1, len[1], F + lb, y, s0, s1);
                s2 = e;
                s3 = pos - e;
                rank = pos + s0 + s1;
                before = (s0 + s1 + S - 1) / S;
            }
            const int64_t nx = (len[0] + len[1] + S - 1) / S;
            const int64_t ny = (len[2] + len[3] + S - 1) / S;
            d.base = w.bstart[j] + gbase;
            d.rank = rank;
            d.s[0] = (int32_t)s0;
            d.s[1] = (int32_t)s1;
            d.s[2] = (int32_t)s2;
            d.s[3] = (int32_t)s3;
            for (int k = 0; k < 4; k++) d.len[k] = (int32_t)len[k];
            d.first = (int32_t)(w.msp[j] + gbase / S);
            d.items = (int32_t)(nx + ny);
            d.sbase = (int32_t)gs;
            d.flags = kActive | (odd ? kFromScratch : 0) | (round + 1 == P ? kLastRound : 0) |
                      ((g & 1) ? kOddGroup : 0) | round_tag(round);
            w.ssorted[d.first + pos / S + before] = d;
            return;
        }
    }
    w.ssorted[item] = d;
}

// A workgroup merges the keys between two consecutive split points (at most
// S of X and S of Y) in two LDS levels: W0+W1 -> X' and W2+W3 -> Y', then
// X'+Y'.  Work is counted in jobs of VT outputs (one co-rank and one window
// merge each); a thread runs up to JOBS jobs per level (S = NT*VT*JOBS/2, so
// that NT*JOBS jobs cover the largest chunk, 2S keys), and the cost follows
// the chunk's size (1 to 2S keys), not its capacity.  With one job per
// thread the same LDS carries twice the threads: more waves to hide the LDS
// round trips of the co-rank searches.
//
// LDS is padded (one word per 128 bytes: neighbouring threads' co-ranks lie
// about VT/2 words apart, and the pad spreads them over the banks).  Every
// run is followed by VT largest-word sentinels, so lds_merge_window reads
// VT words past a co-rank without bounds checks.  Level outputs start on
// multiples of VT, so a thread's VT outputs share one pad period and are
// written at constant offsets.

// One chunk of a fan-in-4 round: its four input windows and its output.
template <typename K>
struct Chunk4 {
    bool active;  // false: nothing to do (inactive item, empty chunk or a flagged inconsistency)
    int c[4];     // window lengths
    int at[4];    // logical LDS position of each window
    const K* ks[4];
    const uint32_t* vs[4];
    K* dk;
    uint32_t* dv;
    K* sf;         // block samples of the group's output (first keys), or null in the bucket's last round
    K* sl;         // last keys of full blocks
    bool fin;      // the bucket's last round: the output is final (order images undone)
    int64_t rank;  // group position of the chunk's first output (outputs start blocks where rank + q is a multiple of 32)
};

template <typename K, bool PAIRS, int S, int VT>
__device__ __forceinline__ Chunk4<K> chunk4_of(const Work<K>& w, int round, int64_t item, int64_t bound) {
    // Straight-line code: the split point, its successor and every kernel
    // argument are read before the first decision, so the workgroup waits for
    // one round trip to memory, not for a chain of them, before its loads.
    const Split4 r0 = w.ssorted[item];
    const Split4 nx1 = w.ssorted[item + 1 < bound ? item + 1 : item];
    const bool odd = r0.flags & kFromScratch;
    const K* sk = (odd ? w.skeys : w.keys) + r0.base;
    const uint32_t* svv = PAIRS ? (odd ? w.svals : w.vals) + r0.base : nullptr;
    const int64_t L = (int64_t)w.tile << (2 * round);
    Chunk4<K> g;
    const bool last = item + 1 - r0.first == r0.items;
    int64_t rank_end = last ? 0 : nx1.rank;
    bool neg = false;
#pragma unroll
    for (int k = 0; k < 4; k++) {
        g.c[k] = (last ? r0.len[k] : nx1.s[k]) - r0.s[k];
        rank_end += last ? r0.len[k] : 0;
        neg |= g.c[k] < 0;
    }
    const int c = g.c[0] + g.c[1] + g.c[2] + g.c[3];
    // a split point inconsistent with its successor, or either of them left
    // over from an earlier round (sorted runs map every sample to its own
    // slot, so neither happens), would make the windows run past their runs:
    // flag it and do nothing
    const int32_t tag = round_tag(round), tagmask = ~(int32_t)0xFF;
    const bool stale = (r0.flags & tagmask) != tag || (!last && (nx1.flags & (tagmask | kActive)) != (tag | kActive));
    const bool bad =
        stale || c != rank_end - r0.rank || neg || g.c[0] + g.c[1] > S || g.c[2] + g.c[3] > S;
    g.dk = (odd ? w.keys : w.skeys) + r0.base + r0.rank;
    g.dv = PAIRS ? (odd ? w.vals : w.svals) + r0.base + r0.rank : nullptr;
    g.rank = r0.rank;
    g.sf = (r0.flags & kLastRound) ? nullptr : w.smpf + r0.sbase;
    g.fin = (r0.flags & kLastRound) != 0;
    g.sl = (r0.flags & kOddGroup) ? nullptr : w.smpl + r0.sbase;
    // window r at logical at[r] (>= 1; body vectors on multiples of 4), then
    // VT sentinels and VT + 4 spare words (room for X' and Y' rounded down
    // to multiples of VT)
    int cur = 4;
#pragma unroll
    for (int r = 0; r < 4; r++) {
        g.ks[r] = sk + r * L + r0.s[r];
        g.vs[r] = PAIRS ? svv + r * L + r0.s[r] : nullptr;
        const int h = head_len(g.ks[r], g.c[r]);
        g.at[r] = ((cur + h + 3) & ~3) - h;
        cur = g.at[r] + g.c[r] + 2 * VT + 4;
    }
    // the addresses are needed only past the branch below, but forming them
    // here keeps their argument reads in the first round trip
    asm volatile("" ::"s"(g.ks[0]), "s"(g.ks[3]), "s"(g.dk));
    if constexpr (PAIRS) asm volatile("" ::"s"(g.vs[0]), "s"(g.dv));
    const bool act = r0.flags & kActive;
    if (act && bad && threadIdx.x == 0) atomicOr(w.err, kErrConsistency);
    g.active = act && !bad && c != 0;
    return g;
}

template <typename K, bool PAIRS, int NT, int VT, int JOBS>
struct Merge4Lds {
    using W = typename WordOf<K, PAIRS>::type;
    static constexpr int S = NT * VT * JOBS / 2;
    static constexpr int CAP = 2 * S;
    static constexpr int LOGICAL = CAP + 8 * VT + 32;  // four windows, sentinels, spacing, alignment
    static_assert((128 / sizeof(W)) % VT == 0, "a VT block fits one pad period");
    // Pairs stage the payload after the narrow words, in the half of `words`
    // that narrow sort words (the key's width) leave free, and wide chunks
    // read it from the source windows instead: no separate payload array.
    using U = typename Traits<K>::U;
    static constexpr int kNarrowWords = lds_padded_size<U>(LOGICAL);
    W words[lds_padded_size<W>(LOGICAL)];
    static_assert(!PAIRS || kNarrowWords * (int)sizeof(U) + CAP * 4 <= (int)sizeof(words),
                  "payload fits after the narrow words");
};

template <typename K, bool PAIRS, int NT, int VT, int JOBS>
struct Merge4Loads {
    static constexpr int CAP = NT * VT * JOBS;
    RunsToLds<K, NT, CAP, 4> keys;
    RunsToLds<uint32_t, NT, PAIRS ? CAP : 4, 4> vals;

    __device__ __forceinline__ void issue(const Chunk4<K>& g) {
        const int os[4] = {0, g.c[0], g.c[0] + g.c[1], g.c[0] + g.c[1] + g.c[2]};
        keys.issue(g.ks, g.c, g.at, os);
        if constexpr (PAIRS) vals.issue(g.vs, g.c, os, os);
    }
};

// Windows to LDS as words mk(q, key) (q: index in the concatenated windows),
// from loads issued earlier, plus their sentinels.
template <typename W, typename K, bool PAIRS, int NT, int VT, int JOBS, typename MK>
__device__ __forceinline__ void stage4(W* words, uint32_t* sv, const Merge4Loads<K, PAIRS, NT, VT, JOBS>& ld,
                                       const Chunk4<K>& g, MK&& mk) {
    const int tid = threadIdx.x;
    ld.keys.commit_padded(words, mk);
    if constexpr (PAIRS) {
        if (sv) ld.vals.commit_dense(sv);  // null: the payload is read from the windows at the store
    }
    if (tid < 4 * VT) {
        const int r = tid / VT;
        int p = g.at[0] + g.c[0];
        p = r == 1 ? g.at[1] + g.c[1] : p;
        p = r == 2 ? g.at[2] + g.c[2] : p;
        p = r == 3 ? g.at[3] + g.c[3] : p;
        words[lds_pad<W>(p + tid % VT)] = WordMax<W>::v;
    }
}

// Block samples of a chunk's outputs (for the next round's split points):
// output q is group position rank + q; it starts a block when that is a
// multiple of 32 and ends one when it is 31 past one.
template <int NT, typename K, typename KeyAt>
__device__ __forceinline__ void store_chunk_samples(const Chunk4<K>& g, int c, KeyAt&& key_at) {
    if (g.sf == nullptr) return;
    const int m = (int)(g.rank % kSampleBlock);
    const int64_t b0 = g.rank / kSampleBlock;
    const int qf = (kSampleBlock - m) % kSampleBlock;  // first output that starts a block
    for (int q = qf + kSampleBlock * (int)threadIdx.x; q < c; q += kSampleBlock * NT) g.sf[b0 + (m + q) / kSampleBlock] = key_at(q);
    if (g.sl == nullptr) return;
    const int ql = kSampleBlock - 1 - m;  // first output that ends a block
    for (int q = ql + kSampleBlock * (int)threadIdx.x; q < c; q += kSampleBlock * NT) g.sl[b0 + (m + q) / kSampleBlock] = key_at(q);
}

// The two merge levels and the store, on windows staged in LDS (the caller
// has synchronised after stage4).  key_of turns a word into its key,
// key_fin into the caller's key (the order image undone) when `fin`,
// pos_of into its index in the concatenated windows, and val_at that index
// into its payload.  Ends with the LDS free for reuse only after the
// caller's next barrier.
template <typename W, typename K, bool PAIRS, int NT, int VT, int JOBS, typename KeyOf, typename KeyFin,
          typename PosOf, typename ValAt>
__device__ __forceinline__ void merge4_chunk(W* words, const Chunk4<K>& g, bool fin, KeyOf&& key_of,
                                             KeyFin&& key_fin, PosOf&& pos_of, ValAt&& val_at) {
    constexpr int S = NT * VT * JOBS / 2;
    constexpr int CAP = 2 * S;
    const W wmax = WordMax<W>::v;
    const int tid = threadIdx.x;
    const int c0 = g.c[0], c1 = g.c[1], c2 = g.c[2], c3 = g.c[3];
    const int o2 = c0 + c1, c = o2 + c2 + c3;
    // level 1: X' = merge(W0, W1) at x0, Y' = merge(W2, W3) at y0, in place
    // of the windows (all reads end at the barrier before the writes)
    const int x0 = g.at[0] & ~(VT - 1), y0 = g.at[2] & ~(VT - 1);
    const int jx = (o2 + VT - 1) / VT, jy = (c - o2 + VT - 1) / VT;
    {
        W v[JOBS][VT];
        int dst[JOBS];
#pragma unroll
        for (int h = 0; h < JOBS; h++) {
            const int j = tid + h * NT;
            if (j < jx + jy) {
                const int y = j >= jx;  // arithmetic selects keep these in registers
                const int dt = (j - y * jx) * VT;
                const int sa = g.at[0] + y * (g.at[2] - g.at[0]), sb = g.at[1] + y * (g.at[3] - g.at[1]);
                const int na = c0 + y * (c2 - c0), nb = c1 + y * (c3 - c1);
                const int ai = lds_corank<W, S / 2>(words, sa, sb, dt, na, nb);
                lds_merge_window<W, VT>(words, sa + ai, sb + dt - ai, v[h]);
                dst[h] = lds_pad<W>(x0 + y * (y0 - x0) + dt);
            }
        }
        __syncthreads();
#pragma unroll
        for (int h = 0; h < JOBS; h++) {
            const int j = tid + h * NT;
            if (j < jx + jy) {
#pragma unroll
                for (int q = 0; q < VT; q++) words[dst[h] + q] = v[h][q];
            }
        }
        // sentinels past the last VT group of X' and of Y' (the groups end in
        // sentinels already: their outputs past the end are the windows')
        if (tid < 2 * VT) words[lds_pad<W>((tid < VT ? x0 + jx * VT : y0 + jy * VT - VT) + tid)] = wmax;
        __syncthreads();
    }
    if (o2 == 0 || o2 == c) {  // one side empty (a group short of four runs): X' or Y' is the result
        const int r = o2 == 0 ? y0 : x0;
        store_chunk_keys<K, NT, CAP>(
            g.dk, c, fin, [&](int q) { return key_of(lds_at_padded(words, r + q)); },
            [&](int q) { return key_fin(lds_at_padded(words, r + q)); });
        if constexpr (PAIRS)
            store_run<uint32_t, NT, CAP>(g.dv, c, [&](int q) { return val_at(pos_of(lds_at_padded(words, r + q))); });
        store_chunk_samples<NT>(g, c, [&](int q) { return key_of(lds_at_padded(words, r + q)); });
        return;
    }
    // level 2: merge X' (o2 words) with Y' (c - o2) into logical [0, c)
    {
        const int jc = (c + VT - 1) / VT;
        W v[JOBS][VT];
#pragma unroll
        for (int h = 0; h < JOBS; h++) {
            const int j = tid + h * NT;
            if (j < jc) {
                const int dt = j * VT;
                const int ai = lds_corank<W, S>(words, x0, y0, dt, o2, c - o2);
                lds_merge_window<W, VT>(words, x0 + ai, y0 + dt - ai, v[h]);
            }
        }
        __syncthreads();
#pragma unroll
        for (int h = 0; h < JOBS; h++) {
            const int j = tid + h * NT;
            if (j < jc) {
                W* dst = words + lds_pad<W>(j * VT);
#pragma unroll
                for (int q = 0; q < VT; q++) dst[q] = v[h][q];
            }
        }
        __syncthreads();
    }
    store_chunk_keys<K, NT, CAP>(
        g.dk, c, fin, [&](int q) { return key_of(lds_at_padded(words, q)); },
        [&](int q) { return key_fin(lds_at_padded(words, q)); });
    if constexpr (PAIRS)
        store_run<uint32_t, NT, CAP>(g.dv, c, [&](int q) { return val_at(pos_of(lds_at_padded(words, q))); });
    store_chunk_samples<NT>(g, c, [&](int q) { return key_of(lds_at_padded(words, q)); });
}

// Stable pairs whose chunk spans fewer than 2^(w-13) - 1 key values (w the
// key's width; the keys of each window lie between its first and last, both
// read by every lane) merge words of the key's width ((key - kmin) << 13 |
// q) instead of the wide composite ones: the same strict order (key, then
// index q < 2^13 in the concatenated windows), half the LDS traffic and far
// fewer VALU operations per compare.  The largest word stays below the
// all-ones sentinel.
constexpr int kNarrowPosBits = 13;
template <typename K>
__device__ __forceinline__ bool narrow_chunk(const Chunk4<K>& g, K& kmin) {
    using U = typename Traits<K>::U;
    constexpr U span = (U(1) << (8 * sizeof(K) - kNarrowPosBits)) - 2;
    K lo = Traits<K>::kMax, hi = Traits<K>::kMin;
#pragma unroll
    for (int r = 0; r < 4; r++) {
        if (g.c[r] > 0) {
            const K a = g.ks[r][0], b = g.ks[r][g.c[r] - 1];
            lo = a < lo ? a : lo;
            hi = b > hi ? b : hi;
        }
    }
    kmin = lo;
    return hi >= lo && (U)hi - (U)lo <= span;
}

// One workgroup per chunk.
template <typename K, bool PAIRS, int NT, int VT, int JOBS>
__global__ __launch_bounds__(NT) void k_merge4(Work<K> w, int round, int64_t bound) {
    using W = typename WordOf<K, PAIRS>::type;
    __shared__ Merge4Lds<K, PAIRS, NT, VT, JOBS> sm;
    // The host launches the rounds the whole array could need; a round no
    // bucket needs ends here, on one word every workgroup reads (it stays in
    // the scalar cache), before any descriptor is read.
    if (round >= *w.rounds) return;
    const Chunk4<K> g = chunk4_of<K, PAIRS, NT * VT * JOBS / 2, VT>(w, round, blockIdx.x, bound);
    if (!g.active) return;
    Merge4Loads<K, PAIRS, NT, VT, JOBS> ld;
    ld.issue(g);
    using L = Merge4Lds<K, PAIRS, NT, VT, JOBS>;
    if constexpr (PAIRS) {
        using U = typename Traits<K>::U;
        static_assert(NT * VT * JOBS <= (1 << kNarrowPosBits), "window indices fit the narrow word");
        K kmin;
        const bool narrow = narrow_chunk(g, kmin);  // the same on every lane
        if (narrow) {
            U* words = reinterpret_cast<U*>(sm.words);
            uint32_t* sv = reinterpret_cast<uint32_t*>(reinterpret_cast<U*>(sm.words) + L::kNarrowWords);
            stage4<U>(words, sv, ld, g,
                      [=](int q, K k) { return ((U)((U)k - (U)kmin) << kNarrowPosBits) | (U)q; });
            __syncthreads();
            const int mode = w.img;
            merge4_chunk<U, K, PAIRS, NT, VT, JOBS>(
                words, g, g.fin && mode != 0, [=](U x) { return (K)((U)kmin + (x >> kNarrowPosBits)); },
                [=](U x) { return image_of((K)((U)kmin + (x >> kNarrowPosBits)), mode, true); },
                [](U x) { return (uint32_t)x & ((1u << kNarrowPosBits) - 1); }, [=](uint32_t p) { return sv[p]; });
            return;
        }
    }
    stage4<W>(sm.words, nullptr, ld, g, [](int q, K k) { return make_word<K, PAIRS>(k, q); });
    __syncthreads();
    const int mode = w.img;
    // wide words: the payload of window index p straight from its source
    // window (p lies in window r when o_r <= p < o_(r+1), o_r the windows'
    // prefix of lengths); captured by value, since a reference would keep g
    // in scratch memory, and chosen by selects of the four candidate
    // addresses, which a chain of pointer assignments would turn into a
    // lookup table there
    const int o1 = g.c[0], o2 = o1 + g.c[1], o3 = o2 + g.c[2];
    const uint32_t *v0 = g.vs[0], *v1 = g.vs[1], *v2 = g.vs[2], *v3 = g.vs[3];
    auto val_at = [=](uint32_t p) -> uint32_t {
        const int q = (int)p;
        uint64_t a = (uint64_t)(v0 + q);
        a = q >= o1 ? (uint64_t)(v1 + (q - o1)) : a;
        a = q >= o2 ? (uint64_t)(v2 + (q - o2)) : a;
        a = q >= o3 ? (uint64_t)(v3 + (q - o3)) : a;
        asm volatile("" : "+v"(a));
        return *global_at<uint32_t>((uintptr_t)a);
    };
    merge4_chunk<W, K, PAIRS, NT, VT, JOBS>(
        sm.words, g, g.fin && mode != 0, [](W x) { return word_key<K, PAIRS>(x); },
        [=](W x) { return image_of(word_key<K, PAIRS>(x), mode, true); }, [](W x) { return pair_pos(x); }, val_at);
}

// --------------------------------------------------------- small segments
// A segment with at most NT*VT keys never leaves LDS: one workgroup sorts it
// and writes it back in place.  Its ten buckets are then contiguous ranges of
// the sorted segment (the digit never decreases with the key), so the
// one-step partition is realised by the same sort; the bucket bounds are
// counted from the sorted keys.  Handles segments with lo < size <= hi.
template <typename K, bool PAIRS, int NT, int VT>
__global__ __launch_bounds__(NT) void k_small(Work<K> w, int64_t lo, int64_t hi) {
    using W = typename WordOf<K, PAIRS>::type;
    constexpr int NV = NT * VT;
    static_assert(VT <= 16, "5-bit digit counters");
    __shared__ W words[lds_padded_size<W>(NV)];
    __shared__ uint32_t sv[PAIRS ? NV : 1];
    __shared__ int sp[NT + 1];
    __shared__ uint32_t red[NT / kWave][5];
    const int s = blockIdx.x;
    if (*w.err || s >= w.nseg) return;
    const int tid = threadIdx.x;
    {
        const int64_t a = w.off[s];
        const int64_t m64 = w.off[s + 1] - a;
        if (!(m64 > lo && m64 <= hi)) return;
        const int m = (int)m64;
        if (m > 1) {
            load_keys_imaged<K, NT, NV>(w.keys + a, m, w.img,
                                        [&](int q, K k) { words[lds_pad<W>(q)] = make_word<K, PAIRS>(k, q); });
            if constexpr (PAIRS) load_run<uint32_t, NT, NV>(w.vals + a, m, [&](int q, uint32_t x) { sv[q] = x; });
            for (int q = m + tid; q < NV; q += NT) words[lds_pad<W>(q)] = WordMax<W>::v;
            __syncthreads();
            block_sort<W, NT, VT>(words, sp, m);
            const int mode = w.img;
            store_chunk_keys<K, NT, NV>(
                w.keys + a, m, mode != 0, [&](int q) { return word_key<K, PAIRS>(lds_at_padded(words, q)); },
                [&](int q) { return image_of(word_key<K, PAIRS>(lds_at_padded(words, q)), mode, true); });
            if constexpr (PAIRS)
                store_run<uint32_t, NT, NV>(w.vals + a, m, [&](int q) { return sv[pair_pos(lds_at_padded(words, q))]; });
        } else {
            if (tid == 0 && m == 1) words[lds_pad<W>(0)] = make_word<K, PAIRS>(img_in(w, w.keys[a]), 0);
            __syncthreads();
        }
        // bucket bounds of the segment, from its sorted keys
        uint64_t c = 0;
        if (m > 0) {
            const K mn = word_key<K, PAIRS>(lds_at_padded(words, 0));
            const K mx = word_key<K, PAIRS>(lds_at_padded(words, m - 1));
            const DigitPlan<K> pl = make_digit_plan<K>(mn, mx, w.ufix);
#pragma unroll
            for (int v = 0; v < VT; v++) {
                const int q = tid * VT + v;
                if (q < m) c += 1ull << (5 * digit_of(pl, word_key<K, PAIRS>(lds_at_padded(words, q))));
            }
        }
        uint32_t wd[5];
        unpack5(c, wd);
        block_sum5<NT>(wd, red);
        if (tid == 0) {
            int64_t run = 0;
            for (int d = 0; d < 10; d++) {
                w.bounds_out[11 * (int64_t)s + d] = run;
                run += field16(wd, d);
            }
            w.bounds_out[11 * (int64_t)s + 10] = run;
        }
    }
}

// Brings buckets left in the scratch copy back to the caller's buffer when a
// debug run stops early: stage 1 (after the scatter) copies every large
// segment's keys; stage 2 (after the local sorts) copies the buckets whose
// round count is odd.
template <typename K>
__global__ void k_collect(Work<K> w, int stage) {
    if (*w.err) return;
    const int nb = w.nbk * w.nseg;
    for (int j = blockIdx.x; j < nb; j += gridDim.x) {
        const int64_t size = w.bsize[j];
        if (size == 0) continue;
        if (stage == 2 && !(bucket_rounds(w.brounds[j]) & 1)) continue;
        const int64_t st = w.bstart[j];
        for (int64_t q = threadIdx.x; q < size; q += blockDim.x) {
            w.keys[st + q] = w.skeys[st + q];
            if (w.vals) w.vals[st + q] = w.svals[st + q];
        }
    }
}

// ------------------------------------------------------- other key types
template <typename K>
__global__ __launch_bounds__(256) void k_image(K* keys, int64_t n, int mode, int inverse) {
    using V = typename Vec16<K>::type;
    constexpr int E = Vec16<K>::n;
    const int h = head_len(keys, (int)(n < 16 ? n : 16));
    const int64_t body = (n - h) / E;
    const int64_t tail = h + body * E;
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x, stride = (int64_t)gridDim.x * blockDim.x;
    V* vs = reinterpret_cast<V*>(keys + h);
    for (int64_t i = tid; i < body; i += stride) {
        V x = vs[i];
        K* e = reinterpret_cast<K*>(&x);
#pragma unroll
        for (int j = 0; j < E; j++) e[j] = image_of(e[j], mode, inverse != 0);
        vs[i] = x;
    }
    if (tid < h) keys[tid] = image_of(keys[tid], mode, inverse != 0);
    if (tail + tid < n) keys[tail + tid] = image_of(keys[tail + tid], mode, inverse != 0);
}

// ------------------------------------------------------------ device scan
// Exclusive prefix sum of `in` (length L read on the device as
// len_mul * *len_ptr, or len_const when len_ptr is null); out[L] = total.
// Sums of kScanTile-value blocks are scanned the same way, level by level,
// so a level's length is ceil(L / per) with per = kScanTile^level.
constexpr int kScanNT = 256, kScanVT = 16, kScanTile = kScanNT * kScanVT;
constexpr int kScanTopNT = 1024, kScanTopVT = 16;

__device__ __forceinline__ int64_t scan_len(const ScanSpec& sp, int64_t per) {
    const int64_t L = sp.len_ptr ? sp.len_mul * (int64_t)(*sp.len_ptr) : sp.len_const;
    return (L + per - 1) / per;
}

template <typename Tin, typename Tout>
__global__ __launch_bounds__(kScanNT) void k_scan_reduce(ScanSpec sp, const Tin* in, Tout* partial, int64_t per) {
    __shared__ Tout red[kScanNT / kWave];
    const int64_t L = scan_len(sp, per);
    const int64_t b0 = (int64_t)blockIdx.x * kScanTile;
    if (b0 >= L) return;
    Tout s = 0;
#pragma unroll
    for (int j = 0; j < kScanVT; j++) {
        const int64_t q = b0 + j * kScanNT + threadIdx.x;
        if (q < L) s += (Tout)in[q];
    }
    s = wave_reduce_add(s);
    if (lane_id() == 0) red[threadIdx.x / kWave] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        Tout t = 0;
        for (int q = 0; q < kScanNT / kWave; q++) t += red[q];
        partial[blockIdx.x] = t;
    }
}

// One workgroup: exclusive scan of up to kScanTopNT*kScanTopVT values in
// place (the partials, or a short input when in != out).
template <typename Tin, typename Tout>
__global__ __launch_bounds__(kScanTopNT) void k_scan_single(ScanSpec sp, const Tin* in, Tout* out, int64_t per) {
    __shared__ Tout red[kScanTopNT / kWave];
    const int64_t L = scan_len(sp, per);
    const int tid = threadIdx.x;
    Tout v[kScanTopVT];
    Tout run = 0;
#pragma unroll
    for (int i = 0; i < kScanTopVT; i++) {
        const int64_t q = (int64_t)tid * kScanTopVT + i;
        v[i] = q < L ? (Tout)in[q] : Tout(0);
        run += v[i];
    }
    Tout total;
    Tout pre = block_excl_scan<Tout, kScanTopNT>(run, total, red);
#pragma unroll
    for (int i = 0; i < kScanTopVT; i++) {
        const int64_t q = (int64_t)tid * kScanTopVT + i;
        if (q < L) out[q] = pre;
        pre += v[i];
    }
    if (tid == 0) out[L] = total;
}

// A thread scans kScanVT consecutive values; where they lie wholly inside
// [0, L) and both arrays are 16-byte aligned there, they move in 16-byte
// vectors (the scratch arrays are), else element by element.
template <typename Tin, typename Tout>
__global__ __launch_bounds__(kScanNT) void k_scan_down(ScanSpec sp, const Tin* in, const Tout* partial, Tout* out,
                                                       int64_t per) {
    static_assert(sizeof(Tin) == 4 || sizeof(Tin) == 8, "4- or 8-byte values");
    __shared__ Tout red[kScanNT / kWave];
    const int64_t L = scan_len(sp, per);
    const int64_t b0 = (int64_t)blockIdx.x * kScanTile;
    if (L == 0 && blockIdx.x == 0 && threadIdx.x == 0) out[0] = 0;
    if (b0 >= L) return;
    const int tid = threadIdx.x;
    const int64_t q0 = b0 + (int64_t)tid * kScanVT;
    const bool vec = q0 + kScanVT <= L && ((uintptr_t)(in + q0) & 15) == 0 && ((uintptr_t)(out + q0) & 15) == 0;
    Tout v[kScanVT];
    Tout run = 0;
    if (vec) {
        constexpr int PIN = 16 / sizeof(Tin);  // inputs per 16-byte vector
        const uint4* src = reinterpret_cast<const uint4*>(in + q0);
#pragma unroll
        for (int j = 0; j < kScanVT / PIN; j++) {
            const uint4 x = src[j];
            Tin a[PIN];
            __builtin_memcpy(a, &x, 16);
#pragma unroll
            for (int e = 0; e < PIN; e++) v[PIN * j + e] = (Tout)a[e];
        }
    } else {
#pragma unroll
        for (int i = 0; i < kScanVT; i++) {
            const int64_t q = q0 + i;
            v[i] = q < L ? (Tout)in[q] : Tout(0);
        }
    }
#pragma unroll
    for (int i = 0; i < kScanVT; i++) run += v[i];
    Tout total;
    Tout pre = block_excl_scan<Tout, kScanNT>(run, total, red) + partial[blockIdx.x];
    Tout o[kScanVT];
#pragma unroll
    for (int i = 0; i < kScanVT; i++) {
        o[i] = pre;
        pre += v[i];
    }
    if (vec) {
        constexpr int PER = 16 / sizeof(Tout);  // outputs per 16-byte vector
        uint4* dst = reinterpret_cast<uint4*>(out + q0);
#pragma unroll
        for (int j = 0; j < kScanVT / PER; j++) {
            uint4 x;
            __builtin_memcpy(&x, &o[j * PER], 16);
            dst[j] = x;
        }
    } else {
#pragma unroll
        for (int i = 0; i < kScanVT; i++) {
            const int64_t q = q0 + i;
            if (q < L) out[q] = o[i];
        }
    }
    const int64_t nblk = (L + kScanTile - 1) / kScanTile;
    if (blockIdx.x == nblk - 1 && tid == 0) out[L] = partial[nblk];
}

// Plain copy, used to calibrate the HBM byte counters.
__global__ void k_copy(const uint4* __restrict__ src, uint4* __restrict__ dst, int64_t n16) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

// =================================================================== host
static inline int cdiv64(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

// One level: a single workgroup when the level fits one, else block sums
// into `partial`, their own scan in place (the next level's partials after
// them), and the down-sweep.
template <typename Tin, typename Tout>
static hipError_t scan_impl(const ScanSpec& sp, int64_t len_bound, const Tin* in, Tout* out, Tout* partial,
                            int64_t per, hipStream_t st) {
    if (len_bound <= (int64_t)kScanTopNT * kScanTopVT) {
        k_scan_single<Tin, Tout><<<1, kScanTopNT, 0, st>>>(sp, in, out, per);
        return hipGetLastError();
    }
    const int64_t nblk = cdiv64(len_bound, kScanTile);
    k_scan_reduce<Tin, Tout><<<(unsigned)nblk, kScanNT, 0, st>>>(sp, in, partial, per);
    const hipError_t e = scan_impl<Tout, Tout>(sp, nblk, partial, partial, partial + nblk + 1, per * kScanTile, st);
    if (e != hipSuccess) return e;
    k_scan_down<Tin, Tout><<<(unsigned)nblk, kScanNT, 0, st>>>(sp, in, partial, out, per);
    return hipGetLastError();
}

hipError_t launch_scan_i32(const ScanSpec& sp, int64_t len_bound, const int32_t* in, int32_t* out, int32_t* partial,
                           hipStream_t st) {
    return scan_impl<int32_t, int32_t>(sp, len_bound, in, out, partial, 1, st);
}
hipError_t launch_scan_u32_i64(const ScanSpec& sp, int64_t len_bound, const uint32_t* in, int64_t* out,
                               int64_t* partial, hipStream_t st) {
    return scan_impl<uint32_t, int64_t>(sp, len_bound, in, out, partial, 1, st);
}
// Partials of every level (each level's block sums and its total).
int64_t scan_partial_count(int64_t len_bound) {
    int64_t c = 0;
    while (len_bound > (int64_t)kScanTopNT * kScanTopVT) {
        len_bound = cdiv64(len_bound, kScanTile);
        c += len_bound + 1;
    }
    return c + 1;
}

static int cu_count() {
    static int cus = 0;
    if (!cus) {
        int dev = 0;
        (void)hipGetDevice(&dev);
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) cus = 256;
    }
    return cus;
}

static int grid_of(int64_t items) { return (int)(items < 1 ? 1 : items); }

template <typename K>
hipError_t launch_setup(const Work<K>& w, int64_t* own_off, int64_t tiles_bound, hipStream_t st) {
    const int g = (int)min((int64_t)1024, (int64_t)cdiv64(w.nseg, 256));
    // a plain sort's tile list is written here too (one thread per slot)
    const int64_t ti = own_off ? tiles_bound : 0;
    k_init<K><<<ti > 256 ? cdiv64(ti, 256) : 1, 256, 0, st>>>(w, own_off, ti);
    // a plain sort (own_off) gets its one segment's counts from k_init
    if (!own_off) k_classify<K><<<g < 1 ? 1 : g, 256, 0, st>>>(w);
    return hipGetLastError();
}

template <typename K>
hipError_t launch_range(const Work<K>& w, int64_t tiles_bound, hipStream_t st) {
    if (w.nbk == 1000) {
        // one thousand buckets (32-bit keys only): 16384-key tiles for keys,
        // 4096 for pairs
        if constexpr (sizeof(K) == 4) {
            if (w.ptile == PartShape<1000>::HT)
                k_range<K, 1000, PartShape<1000>::HT><<<grid_of(tiles_bound), PartShape<1000>::NT, 0, st>>>(w);
            else
                k_range<K, 1000, kHistTile><<<grid_of(tiles_bound), kHistNT, 0, st>>>(w);
        } else {
            return hipErrorInvalidValue;
        }
    } else if (w.nbk == 100) {
        k_range<K, 100, kHistTile><<<grid_of(tiles_bound), kHistNT, 0, st>>>(w);
    } else {
        k_range<K, 10, kHistTile><<<grid_of(tiles_bound), kHistNT, 0, st>>>(w);
    }
    return hipGetLastError();
}

template <typename K>
hipError_t launch_plans(const Work<K>& w, hipStream_t st) {
    const int g = (int)min((int64_t)4096, (int64_t)w.nseg);
    k_plans<K><<<g < 1 ? 1 : g, 1024, 0, st>>>(w);
    return hipGetLastError();
}

template <typename K>
hipError_t launch_hist(const Work<K>& w, int64_t tiles_bound, hipStream_t st) {
    const int g = grid_of(tiles_bound < kHistGrid ? tiles_bound : kHistGrid);
    if (w.nbk == 1000) {
        if constexpr (sizeof(K) == 4) {
            if (w.ptile == PartShape<1000>::HT)
                k_hist<K, 1000, PartShape<1000>::HT><<<g, kHistNT, 0, st>>>(w, tiles_bound);
            else
                k_hist<K, 1000, kHistTile><<<g, kHistNT, 0, st>>>(w, tiles_bound);
        } else {
            return hipErrorInvalidValue;
        }
    } else if (w.nbk == 100) {
        k_hist<K, 100, kHistTile><<<g, kHistNT, 0, st>>>(w, tiles_bound);
    } else {
        k_hist<K, 10, kHistTile><<<g, kHistNT, 0, st>>>(w, tiles_bound);
    }
    return hipGetLastError();
}

template <typename K>
hipError_t launch_colsum(const Work<K>& w, int64_t groups_bound, hipStream_t st) {
    const int g = grid_of(groups_bound);
    if (w.nbk == 1000)
        k_colsum<1000><<<g, kColNT<1000>, 0, st>>>(w.tilepre, w.tilecnt, w.grouppre, w.groupcnt, w.nseg, w.err, w.counts,
                                            w.intra, w.gsum);
    else if (w.nbk == 100)
        k_colsum<100><<<g, kColNT<100>, 0, st>>>(w.tilepre, w.tilecnt, w.grouppre, w.groupcnt, w.nseg, w.err, w.counts,
                                         w.intra, w.gsum);
    else
        k_colsum<10><<<g, kColNT<10>, 0, st>>>(w.tilepre, w.tilecnt, w.grouppre, w.groupcnt, w.nseg, w.err, w.counts,
                                       w.intra, w.gsum);
    return hipGetLastError();
}

template <typename K>
hipError_t launch_offsets1(const Work<K>& w, int64_t ts_bound, hipStream_t st) {
    if (w.nbk == 1000) {
        k_offsets1<K, 1000><<<1, kColNT<1000>, 0, st>>>(w, ts_bound);
    } else if (w.nbk == 100) {
        k_offsets1<K, 100><<<1, kColNT<100>, 0, st>>>(w, ts_bound);
    } else {
        k_offsets1<K, 10><<<1, kColNT<10>, 0, st>>>(w, ts_bound);
    }
    return hipGetLastError();
}

template <typename K>
hipError_t launch_gbase(const Work<K>& w, int64_t groups_bound, hipStream_t st) {
    const int64_t bound = (int64_t)w.nbk * groups_bound;
    k_gbase<K><<<cdiv64(bound, 256), 256, 0, st>>>(w, bound);
    return hipGetLastError();
}

template <typename K>
hipError_t launch_btab(const Work<K>& w, hipStream_t st) {
    const int g = (int)min((int64_t)4096, (int64_t)cdiv64((int64_t)w.nbk * w.nseg, 256));
    k_btab<K><<<g < 1 ? 1 : g, 256, 0, st>>>(w);
    return hipGetLastError();
}

template <typename K, bool PAIRS>
hipError_t launch_scatter(const Work<K>& w, int64_t tiles_bound, hipStream_t st) {
    if (w.nbk == 1000) {
        if constexpr (sizeof(K) == 4 && !PAIRS)
            k_scatter_keys<K, 1000><<<grid_of(tiles_bound), ScatterShape<1000>::NT, 0, st>>>(w);
        else if constexpr (sizeof(K) == 4 && PAIRS)
            k_scatter<K, true, 1000><<<grid_of(tiles_bound), kHistNT, 0, st>>>(w);
        else
            return hipErrorInvalidValue;  // one thousand buckets: 32-bit keys only
    } else if (w.nbk == 100) {
        if constexpr (PAIRS)
            k_scatter<K, true, 100><<<grid_of(tiles_bound), kHistNT, 0, st>>>(w);
        else
            k_scatter_keys<K, 100><<<grid_of(tiles_bound), ScatterShape<100>::NT, 0, st>>>(w);
    } else {
        k_scatter<K, PAIRS, 10><<<grid_of(tiles_bound), kHistNT, 0, st>>>(w);
    }
    return hipGetLastError();
}

template <typename K, bool PAIRS, int NT, int VT, bool BU>
hipError_t launch_tilesort(const Work<K>& w, int64_t items_bound, hipStream_t st) {
    k_tilesort<K, PAIRS, NT, VT, BU><<<grid_of(items_bound), NT, 0, st>>>(w);
    return hipGetLastError();
}

template <typename K>
hipError_t launch_tiles(const Work<K>& w, int64_t tiles_bound, hipStream_t st) {
    k_tiles<K><<<cdiv64(tiles_bound, 256), 256, 0, st>>>(w, tiles_bound);
    return hipGetLastError();
}

template <typename K>
hipError_t launch_sdesc(const Work<K>& w, int64_t items_bound, hipStream_t st) {
    k_sdesc<K><<<cdiv64(items_bound, 256), 256, 0, st>>>(w, items_bound);
    return hipGetLastError();
}

template <typename K>
hipError_t launch_partition(const Work<K>& w, int pass, int64_t chunks_bound, hipStream_t st) {
    k_partition<K><<<cdiv64(chunks_bound, 256), 256, 0, st>>>(w, pass, chunks_bound);
    return hipGetLastError();
}

template <typename K, bool PAIRS, int NT, int VT>
hipError_t launch_merge(const Work<K>& w, int64_t chunks_bound, hipStream_t st) {
    k_merge<K, PAIRS, NT, VT><<<grid_of(chunks_bound), NT, 0, st>>>(w, chunks_bound);
    return hipGetLastError();
}

template <typename K>
hipError_t launch_part4(const Work<K>& w, int round, int64_t chunks_bound, hipStream_t st) {
    k_part4<K><<<cdiv64(chunks_bound, 256), 256, 0, st>>>(w, round, chunks_bound);
    return hipGetLastError();
}

template <typename K, bool PAIRS, int NT, int VT, int JOBS>
hipError_t launch_merge4(const Work<K>& w, int round, int64_t chunks_bound, hipStream_t st) {
    k_merge4<K, PAIRS, NT, VT, JOBS><<<grid_of(chunks_bound), NT, 0, st>>>(w, round, chunks_bound);
    return hipGetLastError();
}

template <typename K, bool PAIRS, int NT, int VT>
hipError_t launch_small(const Work<K>& w, int64_t lo, int64_t hi, int64_t segs_bound, hipStream_t st) {
    k_small<K, PAIRS, NT, VT><<<grid_of(segs_bound), NT, 0, st>>>(w, lo, hi);
    return hipGetLastError();
}

template <typename K>
hipError_t launch_collect(const Work<K>& w, int stage, hipStream_t st) {
    const int g = (int)min((int64_t)4096, (int64_t)w.nbk * w.nseg);
    k_collect<K><<<g < 1 ? 1 : g, 256, 0, st>>>(w, stage);
    return hipGetLastError();
}

template <typename K>
hipError_t launch_image(K* keys, int64_t n, int mode, bool inverse, hipStream_t st) {
    if (n <= 0 || mode == 0) return hipSuccess;
    const int64_t vecs = n / Vec16<K>::n + 1;
    const int g = (int)min((int64_t)8 * cu_count(), (vecs + 255) / 256);
    k_image<K><<<g < 1 ? 1 : g, 256, 0, st>>>(keys, n, mode, inverse ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_copy(const void* src, void* dst, int64_t bytes, hipStream_t st) {
    const int64_t n16 = bytes / 16;
    k_copy<<<4 * cu_count(), 256, 0, st>>>((const uint4*)src, (uint4*)dst, n16);
    return hipGetLastError();
}

// ---------------------------------------------------- explicit instances
#define HS_INST_K(K)                                                                 \
    template hipError_t launch_setup<K>(const Work<K>&, int64_t*, int64_t, hipStream_t); \
    template hipError_t launch_range<K>(const Work<K>&, int64_t, hipStream_t);           \
    template hipError_t launch_plans<K>(const Work<K>&, hipStream_t);                    \
    template hipError_t launch_hist<K>(const Work<K>&, int64_t, hipStream_t);            \
    template hipError_t launch_btab<K>(const Work<K>&, hipStream_t);                     \
    template hipError_t launch_colsum<K>(const Work<K>&, int64_t, hipStream_t);          \
    template hipError_t launch_gbase<K>(const Work<K>&, int64_t, hipStream_t);           \
    template hipError_t launch_offsets1<K>(const Work<K>&, int64_t, hipStream_t);        \
    template hipError_t launch_partition<K>(const Work<K>&, int, int64_t, hipStream_t);  \
    template hipError_t launch_tiles<K>(const Work<K>&, int64_t, hipStream_t);           \
    template hipError_t launch_sdesc<K>(const Work<K>&, int64_t, hipStream_t);           \
    template hipError_t launch_part4<K>(const Work<K>&, int, int64_t, hipStream_t);      \
    template hipError_t launch_collect<K>(const Work<K>&, int, hipStream_t);                \
    template hipError_t launch_image<K>(K*, int64_t, int, bool, hipStream_t);
HS_INST_K(int32_t)
HS_INST_K(int64_t)

template hipError_t launch_scatter<int32_t, false>(const Work<int32_t>&, int64_t, hipStream_t);
template hipError_t launch_scatter<int32_t, true>(const Work<int32_t>&, int64_t, hipStream_t);
template hipError_t launch_scatter<int64_t, false>(const Work<int64_t>&, int64_t, hipStream_t);
template hipError_t launch_scatter<int64_t, true>(const Work<int64_t>&, int64_t, hipStream_t);

#define HS_INST_TILE(K, PAIRS, NT, VT) \
    template hipError_t launch_tilesort<K, PAIRS, NT, VT, false>(const Work<K>&, int64_t, hipStream_t);
HS_TILE_VARIANTS(HS_INST_TILE)
#define HS_INST_TILE_BU(K, PAIRS, NT, VT) \
    template hipError_t launch_tilesort<K, PAIRS, NT, VT, true>(const Work<K>&, int64_t, hipStream_t);
HS_TILE_BU_VARIANTS(HS_INST_TILE_BU)
#define HS_INST_SMALL(K, PAIRS, NT, VT) \
    template hipError_t launch_small<K, PAIRS, NT, VT>(const Work<K>&, int64_t, int64_t, int64_t, hipStream_t);
HS_SMALL_VARIANTS(HS_INST_SMALL)
#define HS_INST_MERGE(K, PAIRS, NT, VT) \
    template hipError_t launch_merge<K, PAIRS, NT, VT>(const Work<K>&, int64_t, hipStream_t);
HS_MERGE_VARIANTS(HS_INST_MERGE)
#define HS_INST_MERGE4(K, PAIRS, NT, VT, JOBS) \
    template hipError_t launch_merge4<K, PAIRS, NT, VT, JOBS>(const Work<K>&, int, int64_t, hipStream_t);
HS_MERGE4_VARIANTS(HS_INST_MERGE4)

}  // namespace hs
