// hs_capi.hip -- the C ABI (include/hsort.h): argument checks, the scratch
// layout, the launch sequence of one call, per-kernel timing records.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <type_traits>
#include <string>
#include <vector>

#include "../../include/hsort.h"
#include "hs_launch.h"

using namespace hs;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

// ------------------------------------------------------------- configuration
struct Config {
    int64_t tile;       // local-sort tile (T)
    int64_t tile_vt;    // keys per thread of the local sort
    int64_t merge_nv;   // outputs per merge workgroup
    int64_t merge_vt;   // outputs per thread of the merge
    int64_t small_max;  // segments up to this size never leave LDS
    int64_t fanin;      // runs merged per round: 2 or 4
    int64_t digits = 1;  // decimal digits of the one-step partition: 1 (ten buckets), 2 (one hundred) or 3 (one thousand)
    int64_t local = 0;   // local sort: 0 network + lane merges + LDS levels, 1 bottom-up LDS merge from VT-runs
};

std::mutex g_mu;
// [kind][size class], kind as hsort_kind (0 int32 keys, 1 int64 keys,
// 2 int32 pairs, 3 segmented int32, 4 segmented int64, 5 int64 pairs); size class by the
// number of keys that decides the merge depth (n for a plain sort, the
// longest segment for a segmented one when the caller gives it).
constexpr int kKinds = 6;
constexpr int kClasses = 4;
constexpr int64_t kClassTop[kClasses - 1] = {1 << 18, 1 << 22, 1 << 26};
Config g_cfg[kKinds][kClasses] = {
    {{8192, 16, 4096, 16, 8192, 2}, {8192, 16, 4096, 16, 8192, 2}, {16384, 32, 4096, 16, 8192, 2}, {16384, 32, 4096, 16, 8192, 2}},
    {{4096, 16, 4096, 16, 4096, 2}, {4096, 16, 4096, 16, 4096, 2}, {4096, 16, 4096, 16, 4096, 2}, {4096, 16, 4096, 16, 4096, 2}},
    {{4096, 16, 4096, 16, 4096, 2}, {4096, 16, 4096, 16, 4096, 2}, {4096, 16, 4096, 16, 4096, 2}, {4096, 16, 4096, 16, 4096, 2}},
    {{8192, 16, 4096, 16, 8192, 2}, {8192, 16, 4096, 16, 8192, 2}, {16384, 32, 4096, 16, 8192, 2}, {16384, 32, 4096, 16, 8192, 2}},
    {{4096, 16, 4096, 16, 4096, 2}, {4096, 16, 4096, 16, 4096, 2}, {4096, 16, 4096, 16, 4096, 2}, {4096, 16, 4096, 16, 4096, 2}},
    {{4096, 8, 2048, 8, 4096, 2}, {4096, 8, 2048, 8, 4096, 2}, {4096, 8, 1024, 8, 4096, 4, 2}, {4096, 8, 1024, 8, 4096, 4, 2}},
};

int cfg_index(int kind) { return (kind >= 0 && kind < kKinds) ? kind : -1; }

// key type of a kind: 0 int32 keys, 1 int64 keys, 2 int32 pairs, 3 int64 pairs
int key_type(int kind) {
    return kind == HSORT_KEYS_I64 || kind == HSORT_SEG_I64 ? 1
           : kind == HSORT_PAIRS_I32_U32                 ? 2
           : kind == HSORT_PAIRS_I64_U32                 ? 3
                                                         : 0;
}

int size_class(int64_t n) {
    int c = 0;
    while (c < kClasses - 1 && n > kClassTop[c]) c++;
    return c;
}

// Size that selects the class: n, or for a segmented call the longest
// segment when the caller knows it.
int64_t class_size(int kind, int64_t n, int64_t max_seg_len) {
    const bool seg = kind == HSORT_SEG_I32 || kind == HSORT_SEG_I64;
    return (seg && max_seg_len > 0 && max_seg_len < n) ? max_seg_len : n;
}

Config get_cfg(int kind, int64_t size) {
    std::lock_guard<std::mutex> lk(g_mu);
    return g_cfg[cfg_index(kind)][size_class(size)];
}

template <typename K, bool PAIRS>
bool tile_shape_ok(int64_t nt, int64_t vt) {
#define X(KK, P, NT_, VT_) \
    if constexpr (std::is_same_v<K, KK> && PAIRS == P) \
        if (nt == NT_ && vt == VT_) return true;
    HS_TILE_VARIANTS(X)
#undef X
    return false;
}

template <typename K, bool PAIRS>
bool bu_tile_shape_ok(int64_t nt, int64_t vt) {
#define X(KK, P, NT_, VT_) \
    if constexpr (std::is_same_v<K, KK> && PAIRS == P) \
        if (nt == NT_ && vt == VT_) return true;
    HS_TILE_BU_VARIANTS(X)
#undef X
    return false;
}

template <typename K, bool PAIRS>
bool merge_shape_ok(int64_t nt, int64_t vt) {
#define X(KK, P, NT_, VT_) \
    if constexpr (std::is_same_v<K, KK> && PAIRS == P) \
        if (nt == NT_ && vt == VT_) return true;
    HS_MERGE_VARIANTS(X)
#undef X
    return false;
}

template <typename K, bool PAIRS>
bool merge4_shape_ok(int64_t nv, int64_t vt) {
#define X(KK, P, NT_, VT_, J_) \
    if constexpr (std::is_same_v<K, KK> && PAIRS == P) \
        if (nv == NT_ * VT_ * J_ / 2 && vt == VT_) return true;
    HS_MERGE4_VARIANTS(X)
#undef X
    return false;
}

template <typename K, bool PAIRS>
bool shapes_ok(const Config& c) {
    const int64_t tn = c.tile / c.tile_vt, mn = c.merge_nv / c.merge_vt;
    if (c.local == 1 ? !bu_tile_shape_ok<K, PAIRS>(tn, c.tile_vt) : !tile_shape_ok<K, PAIRS>(tn, c.tile_vt)) return false;
    if (c.fanin == 2) return merge_shape_ok<K, PAIRS>(mn, c.merge_vt);
    return merge4_shape_ok<K, PAIRS>(c.merge_nv, c.merge_vt);
}

bool config_ok(int key_type_index, const Config& c) {
    if (c.tile_vt <= 0 || c.merge_vt <= 0 || c.tile % c.tile_vt || c.merge_nv % c.merge_vt) return false;
    if (c.tile % c.merge_nv) return false;  // merge chunks must tile a run
    if (c.small_max < 0 || c.small_max > 8192) return false;
    if (c.fanin != 2 && c.fanin != 4) return false;
    if (c.digits < 1 || c.digits > 3) return false;
    if (c.digits == 3 && key_type_index != 0 && key_type_index != 2) return false;  // one thousand buckets: 32-bit keys
    if (c.local != 0 && c.local != 1) return false;
    switch (key_type_index) {
        case 0:
            return shapes_ok<int32_t, false>(c);
        case 1:
            return shapes_ok<int64_t, false>(c);
        case 2:
            return shapes_ok<int32_t, true>(c);
        case 3:  // 16-byte words: the whole-segment sort holds at most 4096
            return c.small_max <= 4096 && shapes_ok<int64_t, true>(c);
    }
    return false;
}

// --------------------------------------------------------------- timing
struct Rec {
    std::string name;
    hipEvent_t a, b;
    double bytes;
    // merge rounds: bytes = per_key * keys of the buckets still merging,
    // read from the bucket table left in scratch when the records are read
    const int64_t* bsize = nullptr;
    const int32_t* brounds = nullptr;
    int64_t nb = 0, tile = 0;
    int pass = 0, fanin = 2;
    double per_key = 0;
};
bool g_timing = false;
std::vector<Rec> g_recs;
thread_local bool g_capturing = false;  // no event records inside a captured graph

struct Timer {
    hipStream_t st;
    bool on;
    std::string name;
    double bytes;
    hipEvent_t a = nullptr, b = nullptr;
    Rec deferred{};
    Timer(hipStream_t s, const char* n, double by) : st(s), name(n), bytes(by) {
        {
            std::lock_guard<std::mutex> lk(g_mu);
            on = g_timing && !g_capturing;
        }
        // timing is best effort: a timer whose events cannot be made or
        // recorded is switched off, and the sort goes on untimed
        if (on && (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess ||
                   hipEventRecord(a, st) != hipSuccess)) {
            drop();
            on = false;
        }
    }
    void drop() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
        a = b = nullptr;
    }
    ~Timer() {
        if (!on) return;
        if (hipEventRecord(b, st) != hipSuccess) {
            drop();
            return;
        }
        Rec r = deferred;
        r.name = name;
        r.a = a;
        r.b = b;
        r.bytes = bytes;
        std::lock_guard<std::mutex> lk(g_mu);
        g_recs.push_back(r);
    }
    void per_active_key(const int64_t* bsize, const int32_t* brounds, int64_t nb, int64_t tile, int pass,
                        double per_key, int fanin) {
        deferred.bsize = bsize;
        deferred.brounds = brounds;
        deferred.nb = nb;
        deferred.tile = tile;
        deferred.pass = pass;
        deferred.per_key = per_key;
        deferred.fanin = fanin;
    }
};

// ------------------------------------------------------------ scratch layout
constexpr size_t kAlign = 256;
size_t up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }
int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Buckets per segment and keys per partition tile of a configuration.
int64_t buckets_of(const Config& c) { return c.digits == 3 ? 1000 : c.digits == 2 ? 100 : 10; }
// (pairs with one thousand buckets keep 4096-key tiles: their stable scatter
// stages keys, payload and 16-bit bucket tags in LDS)
int64_t partition_tile(const Config& c, bool pairs) {
    return c.digits == 3 && !pairs ? PartShape<1000>::HT : kHistTile;
}

struct Layout {
    // byte offsets into scratch
    size_t err, own_off, skeys, svals, tmin, tmax, tp, smpf, smpl, rounds, plans, tilecnt, tilepre, groupcnt, grouppre,
        bounds, counts, intra, gsum, gpos, gbase, bstart, bsize, tsc, tsp, mcc, msp, brounds, tiles, sdesc, mdesc, ssorted, part32,
        part64, total;
    // item bounds
    int64_t large_bound, tiles_bound, groups_bound, buckets, ts_bound, chunks_bound;
    int64_t ptile;  // keys per partition tile
};

Layout make_layout(int kind, int64_t n, int64_t nseg, const Config& c) {
    // A plain sort may be forced through the full pipeline (small_max 0), so
    // at least one segment is always counted as large.
    const bool seg = kind == HSORT_SEG_I32 || kind == HSORT_SEG_I64;
    if (!seg) nseg = 1;
    const size_t ksz = (kind == HSORT_KEYS_I64 || kind == HSORT_SEG_I64 || kind == HSORT_PAIRS_I64_U32) ? 8 : 4;
    const bool pairs = kind == HSORT_PAIRS_I32_U32 || kind == HSORT_PAIRS_I64_U32;
    Layout L{};
    L.large_bound = std::min<int64_t>(nseg, std::max<int64_t>(1, n / (c.small_max + 1)));
    const int64_t nbk = buckets_of(c);
    L.ptile = partition_tile(c, pairs);
    L.tiles_bound = cdiv(n, L.ptile) + L.large_bound;
    L.groups_bound = cdiv(L.tiles_bound, kGroupTiles) + L.large_bound;
    L.buckets = nbk * nseg;
    L.ts_bound = cdiv(n, c.tile) + nbk * L.large_bound;
    L.chunks_bound = cdiv(n, c.merge_nv) + nbk * L.large_bound;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o += up(bytes);
        return at;
    };
    L.err = take(8);  // error word at offset 0 (hsort_check reads it there)
    L.own_off = take(16);
    L.bounds = take(sizeof(int64_t) * 11 * nseg);
    L.skeys = take(ksz * n);
    L.svals = pairs ? take(4 * n) : 0;
    L.tmin = take(ksz * L.tiles_bound);
    L.tmax = take(ksz * L.tiles_bound);
    L.tp = take(8 * L.tiles_bound);
    L.smpf = take(ksz * (n / kSampleBlock + L.chunks_bound + 2));
    L.smpl = take(ksz * (n / kSampleBlock + L.chunks_bound + 2));
    L.rounds = take(4);
    L.plans = take((ksz == 8 ? sizeof(DigitPlan<int64_t>) : sizeof(DigitPlan<int32_t>)) * nseg);
    L.tilecnt = take(4 * nseg);
    L.tilepre = take(4 * (nseg + 1));
    L.groupcnt = take(4 * nseg);
    L.grouppre = take(4 * (nseg + 1));
    L.counts = take(4 * nbk * L.tiles_bound);
    L.intra = take(4 * nbk * L.tiles_bound);
    L.gsum = take(4 * nbk * L.groups_bound);
    L.gpos = take(8 * (nbk * L.groups_bound + 1));
    L.gbase = take(4 * nbk * L.groups_bound);
    L.bstart = take(8 * L.buckets);
    L.bsize = take(8 * L.buckets);
    L.tsc = take(4 * L.buckets);
    L.tsp = take(4 * (L.buckets + 1));
    L.mcc = take(4 * L.buckets);
    L.msp = take(4 * (L.buckets + 1));
    L.brounds = take(4 * L.buckets);
    L.tiles = take(sizeof(TileDesc) * L.tiles_bound);
    L.sdesc = take(sizeof(SortDesc) * L.ts_bound);
    L.mdesc = take(sizeof(MergeDesc) * L.chunks_bound);
    L.ssorted = take(sizeof(Split4) * L.chunks_bound);
    const int64_t p32 = std::max(scan_partial_count(nseg), scan_partial_count(L.buckets));
    L.part32 = take(4 * p32);
    L.part64 = take(8 * scan_partial_count(nbk * L.groups_bound));
    L.total = o;
    return L;
}

template <typename K>
Work<K> make_work(const Layout& L, char* scr, K* keys, uint32_t* vals, const int64_t* off, int64_t n, int64_t nseg,
                  const Config& c, int64_t small_max, int64_t max_seg_len) {
    Work<K> w{};
    w.keys = keys;
    w.vals = vals;
    w.skeys = (K*)(scr + L.skeys);
    w.svals = vals ? (uint32_t*)(scr + L.svals) : nullptr;
    w.off = off ? off : (const int64_t*)(scr + L.own_off);
    w.n = n;
    w.nseg = (int32_t)nseg;
    w.tmin = (K*)(scr + L.tmin);
    w.tmax = (K*)(scr + L.tmax);
    w.tp = (uint64_t*)(scr + L.tp);
    w.smpf = (K*)(scr + L.smpf);
    w.smpl = (K*)(scr + L.smpl);
    w.rounds = (int32_t*)(scr + L.rounds);
    w.plans = (DigitPlan<K>*)(scr + L.plans);
    w.tilecnt = (int32_t*)(scr + L.tilecnt);
    w.tilepre = (int32_t*)(scr + L.tilepre);
    w.groupcnt = (int32_t*)(scr + L.groupcnt);
    w.grouppre = (int32_t*)(scr + L.grouppre);
    w.bounds_out = (int64_t*)(scr + L.bounds);
    w.counts = (uint32_t*)(scr + L.counts);
    w.intra = (uint32_t*)(scr + L.intra);
    w.gsum = (uint32_t*)(scr + L.gsum);
    w.gpos = (int64_t*)(scr + L.gpos);
    w.gbase = (int32_t*)(scr + L.gbase);
    w.bstart = (int64_t*)(scr + L.bstart);
    w.bsize = (int64_t*)(scr + L.bsize);
    w.tsc = (int32_t*)(scr + L.tsc);
    w.tsp = (int32_t*)(scr + L.tsp);
    w.mcc = (int32_t*)(scr + L.mcc);
    w.msp = (int32_t*)(scr + L.msp);
    w.brounds = (int32_t*)(scr + L.brounds);
    w.tiles = (TileDesc*)(scr + L.tiles);
    w.sdesc = (SortDesc*)(scr + L.sdesc);
    w.mdesc = (MergeDesc*)(scr + L.mdesc);
    w.ssorted = (Split4*)(scr + L.ssorted);
    w.err = (uint32_t*)(scr + L.err);
    w.nbk = (int32_t)buckets_of(c);
    w.ptile = (int32_t)L.ptile;
    w.tile = (int32_t)c.tile;
    w.fanin = (int32_t)c.fanin;
    w.nv = (int32_t)c.merge_nv;
    w.small_max = small_max;
    w.max_seg_len = max_seg_len;
    return w;
}

// ------------------------------------------------------------- dispatchers
template <typename K, bool PAIRS>
hipError_t tilesort_by_shape(const Config& c, const Work<K>& w, int64_t items, hipStream_t st) {
    const int64_t nt = c.tile / c.tile_vt, vt = c.tile_vt;
    if (c.local == 1) {
#define X(KK, P, NT_, VT_) \
    if constexpr (std::is_same_v<K, KK> && PAIRS == P) \
        if (nt == NT_ && vt == VT_) return launch_tilesort<KK, P, NT_, VT_, true>(w, items, st);
        HS_TILE_BU_VARIANTS(X)
#undef X
        return hipErrorInvalidValue;
    }
#define X(KK, P, NT_, VT_) \
    if constexpr (std::is_same_v<K, KK> && PAIRS == P) \
        if (nt == NT_ && vt == VT_) return launch_tilesort<KK, P, NT_, VT_, false>(w, items, st);
    HS_TILE_VARIANTS(X)
#undef X
    return hipErrorInvalidValue;
}

template <typename K, bool PAIRS>
hipError_t merge_by_shape(const Config& c, const Work<K>& w, int64_t chunks, hipStream_t st) {
    const int64_t nt = c.merge_nv / c.merge_vt, vt = c.merge_vt;
#define X(KK, P, NT_, VT_) \
    if constexpr (std::is_same_v<K, KK> && PAIRS == P) \
        if (nt == NT_ && vt == VT_) return launch_merge<KK, P, NT_, VT_>(w, chunks, st);
    HS_MERGE_VARIANTS(X)
#undef X
    return hipErrorInvalidValue;
}

template <typename K, bool PAIRS>
hipError_t merge4_by_shape(const Config& c, const Work<K>& w, int round, int64_t chunks, hipStream_t st) {
    const int64_t nv = c.merge_nv, vt = c.merge_vt;
#define X(KK, P, NT_, VT_, J_) \
    if constexpr (std::is_same_v<K, KK> && PAIRS == P) \
        if (nv == NT_ * VT_ * J_ / 2 && vt == VT_) return launch_merge4<KK, P, NT_, VT_, J_>(w, round, chunks, st);
    HS_MERGE4_VARIANTS(X)
#undef X
    return hipErrorInvalidValue;
}

template <typename K, bool PAIRS>
hipError_t small_by_shape(int64_t cap, const Work<K>& w, int64_t lo, int64_t hi, int64_t segs, hipStream_t st) {
    if constexpr (PAIRS && sizeof(K) == 8) {  // 16-byte words: at most 8 per thread
        switch (cap) {
            case 4096:
                return launch_small<K, PAIRS, 512, 8>(w, lo, hi, segs, st);
            case 2048:
                return launch_small<K, PAIRS, 256, 8>(w, lo, hi, segs, st);
            case 256:
                return launch_small<K, PAIRS, 64, 4>(w, lo, hi, segs, st);
        }
        return hipErrorInvalidValue;
    }
    switch (cap) {
        case 8192:
            return launch_small<K, PAIRS, 512, 16>(w, lo, hi, segs, st);
        case 4096:
            return launch_small<K, PAIRS, 256, 16>(w, lo, hi, segs, st);
        case 2048:
            return launch_small<K, PAIRS, 256, 8>(w, lo, hi, segs, st);
        case 256:
            return launch_small<K, PAIRS, 64, 4>(w, lo, hi, segs, st);
    }
    return hipErrorInvalidValue;
}

// Small-segment size classes: (lo, hi] -> LDS capacity.
struct SmallClass {
    int64_t lo, hi, cap;
};
std::vector<SmallClass> small_classes(int64_t small_max) {
    std::vector<SmallClass> v;
    int64_t lo = -1;
    for (int64_t cap : {256, 2048, 4096, 8192}) {
        if (lo >= small_max) break;
        const int64_t hi = std::min(cap, small_max);
        if (hi > lo) v.push_back({lo, hi, cap});
        lo = hi;
    }
    return v;
}

#define HS_TRY(expr)                                                                         \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess) return fail(HSORT_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

// The launch sequence of one call: plain (off == nullptr, one segment) or
// segmented.  Every host-side decision depends only on the arguments' sizes
// and the configuration, never on device data, so the sequence can be
// captured into a graph and replayed.
template <typename K, bool PAIRS>
int enqueue_body(int kind, K* keys, uint32_t* vals, int64_t n, const int64_t* off, int64_t nseg, int64_t max_seg_len,
                 void* scratch, size_t scratch_bytes, hipStream_t st, int stage, int64_t small_override, int img) {
    const Config c = get_cfg(kind, class_size(kind, n, max_seg_len));
    const bool seg = off != nullptr;
    if (!seg) nseg = 1;
    const Layout L = make_layout(kind, n, nseg, c);
    if (scratch_bytes < L.total)
        return fail(HSORT_ERR_SCRATCH, "scratch too small: need " + std::to_string(L.total) + " bytes, got " +
                                           std::to_string(scratch_bytes));
    const int64_t small_max = small_override >= 0 ? small_override : c.small_max;
    char* scr = (char*)scratch;
    Work<K> w = make_work<K>(L, scr, keys, vals, off, n, nseg, c, small_max, seg ? max_seg_len : 0);
    w.ufix = (img & kImgUnsigned) ? 1 : 0;
    // a full sort applies the order image where the partition reads the keys
    // and undoes it where each bucket's final output is written; the debug
    // stage runs image the whole array before and after (enqueue)
    w.img = stage == 3 ? img : 0;
    const double kb = sizeof(K) + (PAIRS ? 4.0 : 0.0);
    {
        Timer t(st, "setup", 0);
        HS_TRY(launch_setup<K>(w, seg ? nullptr : (int64_t*)(scr + L.own_off), L.tiles_bound, st));
    }
    const bool any_large = seg ? (n > small_max) : (n > small_max);
    if (!seg && !any_large) {  // a plain sort that fits one tile
        for (const SmallClass& sc : small_classes(small_max)) {
            if (n > sc.lo && n <= sc.hi) {
                Timer t(st, "small", 2 * kb * n);
                HS_TRY((small_by_shape<K, PAIRS>(sc.cap, w, sc.lo, sc.hi, 1, st)));
            }
        }
        return HSORT_OK;
    }
    if (seg) {  // a plain sort's one segment was counted by the setup
        Timer t(st, "scan", 0);
        HS_TRY(launch_scan_i32(ScanSpec{nullptr, 0, nseg}, nseg, w.tilecnt, w.tilepre, (int32_t*)(scr + L.part32), st));
        HS_TRY(launch_scan_i32(ScanSpec{nullptr, 0, nseg}, nseg, w.groupcnt, w.grouppre, (int32_t*)(scr + L.part32), st));
    }
    if (any_large) {
        if (seg) {  // a plain sort's tile list was written by the setup
            Timer t(st, "tiles", 0);
            HS_TRY(launch_tiles<K>(w, L.tiles_bound, st));
        }
        {
            Timer t(st, "range", sizeof(K) * (double)n);
            HS_TRY(launch_range<K>(w, L.tiles_bound, st));
            HS_TRY(launch_plans<K>(w, st));
        }
        {
            // reads keys again only for segments with a negative key (data
            // dependent, so not counted as algorithmic bytes)
            Timer t(st, "hist", 0);
            HS_TRY(launch_hist<K>(w, L.tiles_bound, st));
        }
        const bool one_group = !seg && cdiv(n, L.ptile) <= kGroupTiles;
        if (one_group) {
            // one group of partition tiles: offsets, bucket table and the
            // local-sort descriptors in one workgroup
            Timer t(st, "scan", 0);
            HS_TRY(launch_offsets1<K>(w, L.ts_bound, st));
        } else {
            {
                Timer t(st, "scan", 0);
                HS_TRY(launch_colsum<K>(w, L.groups_bound, st));
                HS_TRY(launch_scan_u32_i64(ScanSpec{w.grouppre + nseg, w.nbk, 0}, w.nbk * L.groups_bound, w.gsum,
                                           w.gpos, (int64_t*)(scr + L.part64), st));
                HS_TRY(launch_gbase<K>(w, L.groups_bound, st));
            }
            {
                Timer t(st, "btab", 0);
                HS_TRY(launch_btab<K>(w, st));
                HS_TRY(launch_scan_i32(ScanSpec{nullptr, 0, L.buckets}, L.buckets, w.tsc, w.tsp,
                                       (int32_t*)(scr + L.part32), st));
                HS_TRY(launch_scan_i32(ScanSpec{nullptr, 0, L.buckets}, L.buckets, w.mcc, w.msp,
                                       (int32_t*)(scr + L.part32), st));
            }
        }
        if (!one_group) {
            Timer t(st, "sdesc", 0);
            HS_TRY(launch_sdesc<K>(w, L.ts_bound, st));
        }
        {
            Timer t(st, "scatter", 2 * kb * n);
            HS_TRY((launch_scatter<K, PAIRS>(w, L.tiles_bound, st)));
        }
        if (stage == 1) {
            HS_TRY(launch_collect<K>(w, 1, st));
            return HSORT_OK;
        }
        {
            Timer t(st, "tilesort", 2 * kb * n);
            HS_TRY((tilesort_by_shape<K, PAIRS>(c, w, L.ts_bound, st)));
        }
        if (stage == 2) {
            HS_TRY(launch_collect<K>(w, 2, st));
            return HSORT_OK;
        }
        int64_t biggest = n;
        if (seg && max_seg_len > 0) biggest = std::min(biggest, max_seg_len);
        const int rounds = merge_rounds(biggest, c.tile, (int)c.fanin);
        for (int p = 0; p < rounds; p++) {
            if (c.fanin == 4) {
                {
                    Timer t(st, "partition", 0);
                    HS_TRY(launch_part4<K>(w, p, L.chunks_bound, st));
                }
                Timer t(st, "merge", 0);
                t.per_active_key(w.bsize, w.brounds, L.buckets, c.tile, p, 2 * kb, 4);
                HS_TRY((merge4_by_shape<K, PAIRS>(c, w, p, L.chunks_bound, st)));
                continue;
            }
            {
                Timer t(st, "partition", 0);
                HS_TRY(launch_partition<K>(w, p, L.chunks_bound, st));
            }
            {
                Timer t(st, "merge", 0);
                t.per_active_key(w.bsize, w.brounds, L.buckets, c.tile, p, 2 * kb, 2);
                HS_TRY((merge_by_shape<K, PAIRS>(c, w, L.chunks_bound, st)));
            }
        }
    }
    if (seg) {
        for (const SmallClass& sc : small_classes(small_max)) {
            Timer t(st, "small", 0);
            HS_TRY((small_by_shape<K, PAIRS>(sc.cap, w, sc.lo, sc.hi, nseg, st)));
        }
    }
    return HSORT_OK;
}

// Keys of other types (img != 0, plain sorts only): a full sort maps them to
// their order image inside the kernels (where the partition reads the keys,
// and back where each bucket's final output is written); the debug stage
// runs map the whole array in place before and after the pipeline.
template <typename K, bool PAIRS>
int enqueue(int kind, K* keys, uint32_t* vals, int64_t n, const int64_t* off, int64_t nseg, int64_t max_seg_len,
            void* scratch, size_t scratch_bytes, hipStream_t st, int stage, int64_t small_override, int img = 0) {
    const bool passes = img && stage != 3;  // debug stage runs: separate image passes
    if (passes) {
        Timer t(st, "image", 2.0 * sizeof(K) * n);
        HS_TRY(launch_image<K>(keys, n, img, false, st));
    }
    const int rc = enqueue_body<K, PAIRS>(kind, keys, vals, n, off, nseg, max_seg_len, scratch, scratch_bytes, st,
                                          stage, small_override, img);
    if (rc == HSORT_OK && passes) {
        Timer t(st, "image", 2.0 * sizeof(K) * n);
        HS_TRY(launch_image<K>(keys, n, img, true, st));
    }
    return rc;
}

// ------------------------------------------------------------ graph cache
// With graph mode on, each distinct call (kind, sizes, pointers, shapes,
// stream) is captured once into a hipGraph and replayed afterwards; the
// kernels read all data-dependent quantities on the device.
struct GraphKey {
    int kind, stage;
    int64_t n, nseg, max_seg_len, small_override;
    int img;
    const void *keys, *vals, *off, *scratch;
    hipStream_t st;
    Config c;
};
struct GraphEntry {
    GraphKey key;
    hipGraph_t graph;
    hipGraphExec_t exec;
    uint64_t last_use;
};
bool g_graph_mode = false;
std::vector<GraphEntry> g_graphs;
uint64_t g_tick = 0;
constexpr size_t kMaxGraphs = 64;

void destroy_entry(GraphEntry& e) {
    (void)hipStreamSynchronize(e.key.st);  // a replay may still be in flight
    (void)hipGraphExecDestroy(e.exec);
    (void)hipGraphDestroy(e.graph);
}

template <typename K, bool PAIRS>
int run(int kind, K* keys, uint32_t* vals, int64_t n, const int64_t* off, int64_t nseg, int64_t max_seg_len,
        void* scratch, size_t scratch_bytes, hipStream_t st, int stage, int64_t small_override, int img = 0) {
    bool graphs;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        graphs = g_graph_mode;
    }
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (graphs && st) (void)hipStreamIsCapturing(st, &cap);
    if (!graphs || !st || cap != hipStreamCaptureStatusNone)
        return enqueue<K, PAIRS>(kind, keys, vals, n, off, nseg, max_seg_len, scratch, scratch_bytes, st, stage,
                                 small_override, img);
    GraphKey key;
    memset(&key, 0, sizeof key);
    key.kind = kind;
    key.stage = stage;
    key.n = n;
    key.nseg = nseg;
    key.max_seg_len = max_seg_len;
    key.small_override = small_override;
    key.img = img;
    key.keys = keys;
    key.vals = vals;
    key.off = off;
    key.scratch = scratch;
    key.st = st;
    key.c = get_cfg(kind, class_size(kind, n, max_seg_len));
    hipGraphExec_t exec = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        for (GraphEntry& e : g_graphs)
            if (!memcmp(&e.key, &key, sizeof key)) {
                e.last_use = ++g_tick;
                exec = e.exec;
                break;
            }
    }
    if (!exec) {
        const Layout L = make_layout(kind, n, off ? nseg : 1, key.c);
        if (scratch_bytes < L.total)
            return fail(HSORT_ERR_SCRATCH, "scratch too small: need " + std::to_string(L.total) + " bytes");
        HS_TRY(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
        g_capturing = true;
        const int rc = enqueue<K, PAIRS>(kind, keys, vals, n, off, nseg, max_seg_len, scratch, scratch_bytes, st,
                                         stage, small_override, img);
        g_capturing = false;
        hipGraph_t graph = nullptr;
        const hipError_t e = hipStreamEndCapture(st, &graph);
        if (rc != HSORT_OK) {
            if (graph) (void)hipGraphDestroy(graph);
            return rc;
        }
        if (e != hipSuccess) return fail(HSORT_ERR_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
        const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        if (ei != hipSuccess) {
            (void)hipGraphDestroy(graph);
            return fail(HSORT_ERR_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(ei));
        }
        std::lock_guard<std::mutex> lk(g_mu);
        if (g_graphs.size() >= kMaxGraphs) {
            auto lru = std::min_element(g_graphs.begin(), g_graphs.end(),
                                        [](const GraphEntry& a, const GraphEntry& b) { return a.last_use < b.last_use; });
            destroy_entry(*lru);
            g_graphs.erase(lru);
        }
        g_graphs.push_back({key, graph, exec, ++g_tick});
    }
    HS_TRY(hipGraphLaunch(exec, st));
    return HSORT_OK;
}

int check_common(const void* keys, int64_t n, const void* scratch) {
    if (n < 0) return fail(HSORT_ERR_INVALID, "n < 0");
    if (n > HSORT_MAX_KEYS) return fail(HSORT_ERR_UNSUPPORTED, "n above HSORT_MAX_KEYS");
    if (n > 0 && (!keys || !scratch)) return fail(HSORT_ERR_INVALID, "null pointer");
    return HSORT_OK;
}

// ------------------------------------------------- library-owned scratch
// hsort_keys_i32_noalloc works in a scratch array the library owns, one per
// GPU (see `scratch` below), found once per device by hipGetSymbolAddress.
constexpr int kMaxDevices = 64;
std::mutex g_static_mu;
void* g_static_ptr[kMaxDevices] = {};

}  // namespace

// The scratch array of hsort_keys_i32_noalloc: file scope, one copy on every
// GPU the library runs on, held until the process ends.  In host code this
// name stands for a host-side shadow, not the device array: the device
// address comes from hipGetSymbolAddress (static_scratch), and only that
// address reaches kernels.
static __device__ __align__(256) unsigned char scratch[HSORT_NOALLOC_SCRATCH_BYTES];

namespace {

// Device address of the current GPU's scratch array (looked up on the first
// call on that GPU, with that GPU current).
int static_scratch(void** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(HSORT_ERR_HIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return fail(HSORT_ERR_UNSUPPORTED, "device ordinal above 63");
    std::lock_guard<std::mutex> lk(g_static_mu);
    if (!g_static_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(HSORT_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_static_ptr[dev] = p;
    }
    *out = g_static_ptr[dev];
    return HSORT_OK;
}

}  // namespace

// ===================================================================== C ABI
extern "C" {

size_t hsort_scratch_bytes(int kind, int64_t n, int64_t nseg) {
    if (cfg_index(kind) < 0 || n < 0 || nseg < 0) return 0;
    // the largest need over the classes a segmented call of n keys may pick
    size_t need = 0;
    const bool seg = kind == HSORT_SEG_I32 || kind == HSORT_SEG_I64;
    for (int c = 0; c < kClasses; c++) {
        if (!seg && c != size_class(n)) continue;
        Config cf;
        {
            std::lock_guard<std::mutex> lk(g_mu);
            cf = g_cfg[cfg_index(kind)][c];
        }
        need = std::max(need, make_layout(kind, n, nseg, cf).total);
    }
    return need;
}

size_t hsort_bounds_offset(int kind, int64_t n, int64_t nseg) {
    if (cfg_index(kind) < 0) return 0;
    return make_layout(kind, n, nseg, get_cfg(kind, n)).bounds;  // does not depend on the shapes
}

int hsort_size_class(int64_t n) { return size_class(n); }

int hsort_keys_i32(int32_t* keys, int64_t n, void* scratch, size_t scratch_bytes, void* stream) {
    g_err.clear();
    int rc = check_common(keys, n, scratch);
    if (rc || n == 0) return rc;
    return run<int32_t, false>(HSORT_KEYS_I32, keys, nullptr, n, nullptr, 1, 0, scratch, scratch_bytes,
                               (hipStream_t)stream, 3, -1);
}

int hsort_keys_i64(int64_t* keys, int64_t n, void* scratch, size_t scratch_bytes, void* stream) {
    g_err.clear();
    int rc = check_common(keys, n, scratch);
    if (rc || n == 0) return rc;
    return run<int64_t, false>(HSORT_KEYS_I64, keys, nullptr, n, nullptr, 1, 0, scratch, scratch_bytes,
                               (hipStream_t)stream, 3, -1);
}

int hsort_pairs(int32_t* keys, uint32_t* vals, int64_t n, void* scratch, size_t scratch_bytes, void* stream) {
    g_err.clear();
    int rc = check_common(keys, n, scratch);
    if (rc || n == 0) return rc;
    if (!vals) return fail(HSORT_ERR_INVALID, "null vals");
    return run<int32_t, true>(HSORT_PAIRS_I32_U32, keys, vals, n, nullptr, 1, 0, scratch, scratch_bytes,
                              (hipStream_t)stream, 3, -1);
}

int hsort_keys_i32_noalloc(int32_t* keys, int64_t n, void* stream) {
    g_err.clear();
    if (n < 0) return fail(HSORT_ERR_INVALID, "n < 0");
    if (n > HSORT_NOALLOC_MAX_KEYS)
        return fail(HSORT_ERR_UNSUPPORTED, "n = " + std::to_string(n) + " above HSORT_NOALLOC_MAX_KEYS (" +
                                               std::to_string(HSORT_NOALLOC_MAX_KEYS) + ")");
    if (n > 0 && !keys) return fail(HSORT_ERR_INVALID, "null keys");
    if (n == 0) return HSORT_OK;
    const Config c = get_cfg(HSORT_KEYS_I32, n);
    const size_t need = make_layout(HSORT_KEYS_I32, n, 1, c).total;
    if (need > (size_t)HSORT_NOALLOC_SCRATCH_BYTES)
        return fail(HSORT_ERR_UNSUPPORTED, "the configured shapes need " + std::to_string(need) +
                                               " bytes of scratch, above HSORT_NOALLOC_SCRATCH_BYTES");
    void* scr = nullptr;
    int rc = static_scratch(&scr);
    if (rc != HSORT_OK) return rc;
    // straight to the launch sequence: no graph cache (its instantiation
    // allocates) and no timing events
    const bool was = g_capturing;
    g_capturing = true;
    rc = enqueue<int32_t, false>(HSORT_KEYS_I32, keys, nullptr, n, nullptr, 1, 0, scr,
                                 (size_t)HSORT_NOALLOC_SCRATCH_BYTES, (hipStream_t)stream, 3, -1);
    g_capturing = was;
    return rc;
}

static int seg_args(const void* keys, int64_t n, const int64_t* offsets, int64_t nseg, int64_t max_seg_len,
                    const void* scratch) {
    if (nseg < 0) return fail(HSORT_ERR_INVALID, "nseg < 0");
    if (nseg > HSORT_MAX_SEGMENTS) return fail(HSORT_ERR_UNSUPPORTED, "nseg above HSORT_MAX_SEGMENTS");
    if (max_seg_len < 0) return fail(HSORT_ERR_INVALID, "max_seg_len < 0");
    if (nseg > 0 && !offsets) return fail(HSORT_ERR_INVALID, "null offsets");
    return check_common(keys, n, scratch);
}

int hsort_segmented(int32_t* keys, int64_t n, const int64_t* offsets, int64_t nseg, int64_t max_seg_len,
                    void* scratch, size_t scratch_bytes, void* stream) {
    g_err.clear();
    int rc = seg_args(keys, n, offsets, nseg, max_seg_len, scratch);
    if (rc || n == 0 || nseg == 0) return rc;
    return run<int32_t, false>(HSORT_SEG_I32, keys, nullptr, n, offsets, nseg, max_seg_len, scratch, scratch_bytes,
                               (hipStream_t)stream, 3, -1);
}

int hsort_segmented_i64(int64_t* keys, int64_t n, const int64_t* offsets, int64_t nseg, int64_t max_seg_len,
                        void* scratch, size_t scratch_bytes, void* stream) {
    g_err.clear();
    int rc = seg_args(keys, n, offsets, nseg, max_seg_len, scratch);
    if (rc || n == 0 || nseg == 0) return rc;
    return run<int64_t, false>(HSORT_SEG_I64, keys, nullptr, n, offsets, nseg, max_seg_len, scratch, scratch_bytes,
                               (hipStream_t)stream, 3, -1);
}

// ------------------------------------------------------- other key types
static int typed_mode(int key_type, int flags, int* img, bool* wide) {
    if (key_type < HSORT_I32 || key_type > HSORT_F64) return fail(HSORT_ERR_INVALID, "unknown key type");
    if (flags & ~HSORT_DESCENDING) return fail(HSORT_ERR_INVALID, "unknown flags");
    const int base = key_type % 3;  // 0 signed, 1 unsigned, 2 float
    *img = (base == 1 ? kImgUnsigned : base == 2 ? kImgFloat : 0) | ((flags & HSORT_DESCENDING) ? kImgDesc : 0);
    *wide = key_type >= HSORT_I64;
    return HSORT_OK;
}

size_t hsort_sort_scratch_bytes(int key_type, int with_vals, int64_t n) {
    if (key_type < HSORT_I32 || key_type > HSORT_F64) return 0;
    const bool wide = key_type >= HSORT_I64;
    const int kind = wide ? (with_vals ? HSORT_PAIRS_I64_U32 : HSORT_KEYS_I64)
                          : (with_vals ? HSORT_PAIRS_I32_U32 : HSORT_KEYS_I32);
    return hsort_scratch_bytes(kind, n, 1);
}

static int sort_typed(void* keys, uint32_t* vals, int64_t n, int key_type, int flags, int stage, void* scratch,
                      size_t scratch_bytes, hipStream_t st) {
    int img = 0;
    bool wide = false;
    int rc = typed_mode(key_type, flags, &img, &wide);
    if (rc) return rc;
    rc = check_common(keys, n, scratch);
    if (rc || n == 0) return rc;
    const int64_t small = stage == 3 ? -1 : 0;  // debug stages run the whole pipeline
    if (!wide) {
        if (vals)
            return run<int32_t, true>(HSORT_PAIRS_I32_U32, (int32_t*)keys, vals, n, nullptr, 1, 0, scratch,
                                      scratch_bytes, st, stage, small, img);
        return run<int32_t, false>(HSORT_KEYS_I32, (int32_t*)keys, nullptr, n, nullptr, 1, 0, scratch, scratch_bytes,
                                   st, stage, small, img);
    }
    if (vals)
        return run<int64_t, true>(HSORT_PAIRS_I64_U32, (int64_t*)keys, vals, n, nullptr, 1, 0, scratch,
                                  scratch_bytes, st, stage, small, img);
    return run<int64_t, false>(HSORT_KEYS_I64, (int64_t*)keys, nullptr, n, nullptr, 1, 0, scratch, scratch_bytes, st,
                               stage, small, img);
}

int hsort_sort(void* keys, uint32_t* vals, int64_t n, int key_type, int flags, void* scratch, size_t scratch_bytes,
               void* stream) {
    g_err.clear();
    return sort_typed(keys, vals, n, key_type, flags, 3, scratch, scratch_bytes, (hipStream_t)stream);
}

int hsort_debug_stage_typed(void* keys, uint32_t* vals, int64_t n, int key_type, int flags, int stage, void* scratch,
                            size_t scratch_bytes, void* stream) {
    g_err.clear();
    if (stage < 1 || stage > 3) return fail(HSORT_ERR_INVALID, "stage must be 1, 2 or 3");
    return sort_typed(keys, vals, n, key_type, flags, stage, scratch, scratch_bytes, (hipStream_t)stream);
}

int hsort_check(const void* scratch, void* stream) {
    g_err.clear();
    if (!scratch) return fail(HSORT_ERR_INVALID, "null scratch");
    hipError_t e = hipStreamSynchronize((hipStream_t)stream);
    if (e != hipSuccess) return fail(HSORT_ERR_HIP, std::string("hipStreamSynchronize: ") + hipGetErrorString(e));
    uint32_t flag = 0;
    e = hipMemcpy(&flag, scratch, sizeof(flag), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return fail(HSORT_ERR_HIP, std::string("hipMemcpy: ") + hipGetErrorString(e));
    if (flag & kErrOffsets) return fail(HSORT_ERR_INVALID, "invalid segment offsets");
    if (flag & kErrSegLen) return fail(HSORT_ERR_INVALID, "a segment is longer than max_seg_len");
    if (flag) return fail(HSORT_ERR_INVALID, "internal consistency check failed on the device");
    return HSORT_OK;
}

const char* hsort_last_error(void) { return g_err.c_str(); }

int hsort_set_config(int kind, int size_cls, int64_t tile, int64_t tile_vt, int64_t merge_nv, int64_t merge_vt,
                     int64_t small_max, int64_t fanin, int64_t digits, int64_t local) {
    g_err.clear();
    const int ci = cfg_index(kind);
    if (ci < 0) return fail(HSORT_ERR_INVALID, "unknown kind");
    if (size_cls < -1 || size_cls >= kClasses) return fail(HSORT_ERR_INVALID, "size class out of range");
    const Config c{tile, tile_vt, merge_nv, merge_vt, small_max, fanin, digits, local};
    if (!config_ok(key_type(kind), c)) return fail(HSORT_ERR_UNSUPPORTED, "tile/merge shape not compiled");
    if (digits == 3 && kind != HSORT_KEYS_I32 && kind != HSORT_PAIRS_I32_U32)
        return fail(HSORT_ERR_UNSUPPORTED, "one thousand buckets: plain int32 sorts (keys only or pairs) only");
    std::lock_guard<std::mutex> lk(g_mu);
    for (int k = 0; k < kClasses; k++)
        if (size_cls < 0 || k == size_cls) g_cfg[ci][k] = c;
    return HSORT_OK;
}

int hsort_get_config(int kind, int size_cls, int64_t* tile, int64_t* tile_vt, int64_t* merge_nv, int64_t* merge_vt,
                     int64_t* small_max, int64_t* fanin, int64_t* digits, int64_t* local) {
    const int ci = cfg_index(kind);
    if (ci < 0 || size_cls < 0 || size_cls >= kClasses || !tile || !tile_vt || !merge_nv || !merge_vt || !small_max ||
        !fanin || !digits || !local)
        return fail(HSORT_ERR_INVALID, "bad arguments");
    Config c;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        c = g_cfg[ci][size_cls];
    }
    *tile = c.tile;
    *tile_vt = c.tile_vt;
    *merge_nv = c.merge_nv;
    *merge_vt = c.merge_vt;
    *small_max = c.small_max;
    *fanin = c.fanin;
    *digits = c.digits;
    *local = c.local;
    return HSORT_OK;
}

int hsort_load_tuning(const char* path) {
    g_err.clear();
    if (!path) return fail(HSORT_ERR_INVALID, "null path");
    FILE* f = fopen(path, "r");
    if (!f) return fail(HSORT_ERR_INVALID, std::string("cannot open ") + path);
    char line[512];
    int lineno = 0, rc = HSORT_OK;
    while (fgets(line, sizeof line, f)) {
        lineno++;
        if (line[0] == '#' || line[0] == '\n') continue;
        int kind = 0, cls = 0;
        long long t, tv, m, mv, sm, fi, dg = 1, lc = 0;
        const int got = sscanf(line, "%d %d %lld %lld %lld %lld %lld %lld %lld %lld", &kind, &cls, &t, &tv, &m, &mv, &sm,
                               &fi, &dg, &lc);
        if (got < 8) {  // the digits (1) and local-sort (0) columns are optional
            rc = fail(HSORT_ERR_INVALID, std::string(path) + ": bad line " + std::to_string(lineno));
            break;
        }
        if ((rc = hsort_set_config(kind, cls, t, tv, m, mv, sm, fi, dg, lc)) != HSORT_OK) break;
    }
    fclose(f);
    return rc;
}

int hsort_debug_stage(int kind, void* keys, uint32_t* vals, int64_t n, int stage, void* scratch,
                      size_t scratch_bytes, void* stream) {
    g_err.clear();
    int rc = check_common(keys, n, scratch);
    if (rc || n == 0) return rc;
    if (stage < 1 || stage > 3) return fail(HSORT_ERR_INVALID, "stage must be 1, 2 or 3");
    hipStream_t st = (hipStream_t)stream;
    switch (kind) {
        case HSORT_KEYS_I32:
            return run<int32_t, false>(kind, (int32_t*)keys, nullptr, n, nullptr, 1, 0, scratch, scratch_bytes, st,
                                       stage, 0);
        case HSORT_KEYS_I64:
            return run<int64_t, false>(kind, (int64_t*)keys, nullptr, n, nullptr, 1, 0, scratch, scratch_bytes, st,
                                       stage, 0);
        case HSORT_PAIRS_I32_U32:
            if (!vals) return fail(HSORT_ERR_INVALID, "null vals");
            return run<int32_t, true>(kind, (int32_t*)keys, vals, n, nullptr, 1, 0, scratch, scratch_bytes, st,
                                      stage, 0);
        case HSORT_PAIRS_I64_U32:
            if (!vals) return fail(HSORT_ERR_INVALID, "null vals");
            return run<int64_t, true>(kind, (int64_t*)keys, vals, n, nullptr, 1, 0, scratch, scratch_bytes, st,
                                      stage, 0);
    }
    return fail(HSORT_ERR_INVALID, "kind must be a plain kind");
}

int hsort_graph_mode(int on) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_graph_mode = on != 0;
    return HSORT_OK;
}

int hsort_graph_clear(void) {
    std::lock_guard<std::mutex> lk(g_mu);
    for (GraphEntry& e : g_graphs) destroy_entry(e);
    g_graphs.clear();
    return HSORT_OK;
}

int64_t hsort_graph_count(void) {
    std::lock_guard<std::mutex> lk(g_mu);
    return (int64_t)g_graphs.size();
}

int hsort_timing_enable(int on) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_timing = on != 0;
    return HSORT_OK;
}

int64_t hsort_timing_read(char* out, int64_t cap) {
    std::vector<Rec> recs;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        recs.swap(g_recs);
    }
    struct Agg {
        std::string name;
        int64_t launches;
        double ms, bytes;
    };
    std::vector<Agg> agg;
    const int64_t* cached_ptr = nullptr;
    std::vector<int64_t> sizes;
    std::vector<int32_t> rounds;
    for (Rec& r : recs) {
        float ms = 0;
        // a record whose events cannot be read is left out
        const bool timed = hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess;
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
        if (!timed) continue;
        if (r.bsize) {
            if (r.bsize != cached_ptr || (int64_t)sizes.size() != r.nb) {
                sizes.assign((size_t)r.nb, 0);
                rounds.assign((size_t)r.nb, 0);
                const bool got =
                    hipMemcpy(sizes.data(), r.bsize, sizeof(int64_t) * r.nb, hipMemcpyDeviceToHost) == hipSuccess &&
                    hipMemcpy(rounds.data(), r.brounds, sizeof(int32_t) * r.nb, hipMemcpyDeviceToHost) == hipSuccess;
                if (!got) {  // bucket sizes unknown: the record keeps its time, with no bytes
                    sizes.clear();
                    rounds.clear();
                }
                cached_ptr = got ? r.bsize : nullptr;
            }
            double active = 0;
            for (size_t b = 0; b < sizes.size(); b++)
                if (bucket_rounds(rounds[b]) > r.pass) active += (double)sizes[b];
            r.bytes = r.per_key * active;
        }
        auto it = std::find_if(agg.begin(), agg.end(), [&](const Agg& a) { return a.name == r.name; });
        if (it == agg.end()) {
            agg.push_back({r.name, 0, 0, 0});
            it = agg.end() - 1;
        }
        it->launches++;
        it->ms += ms;
        it->bytes += r.bytes;
    }
    std::string s;
    for (const Agg& a : agg) {
        char line[256];
        snprintf(line, sizeof line, "%s %lld %.6f %.0f\n", a.name.c_str(), (long long)a.launches, a.ms, a.bytes);
        s += line;
    }
    if (out && cap > 0) {
        const int64_t m = std::min<int64_t>(cap - 1, (int64_t)s.size());
        memcpy(out, s.data(), (size_t)m);
        out[m] = 0;
    }
    return (int64_t)s.size() + 1;
}

int hsort_copy(const void* src, void* dst, int64_t bytes, void* stream) {
    g_err.clear();
    if (!src || !dst || bytes < 0 || bytes % 16) return fail(HSORT_ERR_INVALID, "bad copy arguments");
    Timer t((hipStream_t)stream, "copy", 2.0 * bytes);
    HS_TRY(launch_copy(src, dst, bytes, (hipStream_t)stream));
    return HSORT_OK;
}

}  // extern "C"
