// hs_work.h -- the per-call working set shared by the kernels and the host
// launcher (plain device pointers into the caller's scratch buffer).
#pragma once
#include <stdint.h>

#include "hs_device.h"

namespace hs {

// Keys per histogram / scatter tile (256 threads x 16 keys).
constexpr int kHistNT = 256;
constexpr int kHistVT = 16;
constexpr int kHistTile = kHistNT * kHistVT;
constexpr int64_t kHistGrid = 8192;  // workgroups of the histogram pass (it strides over the tiles)

// Partition tiles (range counts, histogram, scatter) by the number of
// buckets: 256 threads x 16 keys for ten and one hundred; 1024 x 16 for one
// thousand, so that the per-tile counts (one word per bucket and tile) stay
// near a sixteenth of the keys.
template <int NBK>
struct PartShape {
    static constexpr int NT = NBK == 1000 ? 1024 : kHistNT;
    static constexpr int VT = kHistVT;
    static constexpr int HT = NT * VT;
};
// Threads and keys per thread of the keys-only scatter on those tiles (512
// x 32 with one thousand buckets: two workgroups fit a CU's LDS and
// registers).
template <int NBK>
struct ScatterShape {
    static constexpr int NT = NBK == 1000 ? 512 : kHistNT;
    static constexpr int VT = PartShape<NBK>::HT / NT;
};

// Per-tile bucket counts are stored tile-major (one row of nbk words per
// tile, so each pass reads or writes a tile's row in one piece), and their
// offsets are formed in two parts: the exclusive prefix of a tile's counts
// over the earlier tiles of its group of kGroupTiles consecutive tiles of
// one segment, plus the group's start in each bucket (a scan over the group
// sums, bucket-major, and its transpose).
constexpr int kGroupTiles = 64;

// One histogram tile of a large segment (range, histogram and scatter read it).
struct TileDesc {
    int64_t base;      // first key of the tile
    int64_t seg_base;  // first key of its segment
    int32_t cnt;       // keys in the tile
    int32_t seg;       // segment index
    int32_t idx;       // tile index inside the segment
    int32_t nt;        // tiles of the segment
    int32_t grp;       // flat index of the tile's group
    int32_t pad;
};

// One local-sort partition of a bucket.
struct SortDesc {
    int64_t start;   // first key
    int32_t cnt;     // keys (0: no work)
    int32_t odd;     // bit 0: write to the scratch copy (odd number of merge rounds); bit 1: odd partition;
                     // bit 2: the bucket's keys all share one value (copied, not sorted);
                     // bit 3: no merge round follows (this is the bucket's final output)
    int32_t bucket;  // nbk * segment + bucket of the segment
    int32_t sbase;   // sample index of the partition's first 32-key block
};

// One merge workgroup of one round: it merges A[a .. a_end) and
// B[b .. b_end) into out[out ..).  The window ends are the next chunk's
// starts, except for the last chunk of a pair, which carries them itself.
struct MergeDesc {
    int64_t a, b, out;
    int64_t a_end, b_end;  // valid when flags & kLastChunk
    int32_t flags;
    int32_t pad;
};
constexpr int32_t kActive = 1;     // the chunk has work this round
constexpr int32_t kFromScratch = 2;  // source is the scratch copy
constexpr int32_t kLastChunk = 4;  // last chunk of its pair of runs
constexpr int32_t kLastPass = 8;   // the bucket's last merge round (its output is final)

// Fan-in-4 merge rounds: a split point of a group of four runs R0..R3 (the
// first `rank` outputs of the group's stable merge are R0[0..s0), R1[0..s1),
// R2[0..s2), R3[0..s3)).  k_part4 computes one per sample and writes it
// straight to its slot in rank order; a merge workgroup takes the keys
// between two consecutive split points.
struct Split4 {
    int64_t base;   // absolute index of the group's first key (run k starts at base + k*L)
    int64_t rank;   // output position of the split point inside the group
    int32_t s[4];   // keys of each run before the split point
    int32_t len[4]; // run lengths of the group
    int32_t first;  // flat index of the group's first chunk
    int32_t items;  // chunks of the group (= split points)
    int32_t sbase;  // sample index of the group's first 32-key block
    int32_t flags;  // kActive | kFromScratch | kLastRound | round_tag(round)
};
constexpr int32_t kLastRound = 4;  // the bucket's last merge round: its output needs no samples

// brounds[j]: the bucket's merge rounds, with kConstBucket set when the digit
// plan gives the bucket a span of one value (its keys are all equal, so the
// scatter has already left it in order: no local sort, no merge round).
constexpr int32_t kConstBucket = 1 << 30;
__host__ __device__ inline int bucket_rounds(int32_t x) { return x & 0xFFFF; }
constexpr int32_t kOddGroup = 8;   // odd group: its output is run 1 or 3 of the next round's group (no last keys)

// Block samples for the split-point searches of fan-in-4 rounds: the runs a
// round reads are cut into 32-key blocks counted from their bucket's start,
// and the producer of the runs (the local sort, or the previous round)
// stores the first and the last key of every block.  Bucket j's block b
// lives at index bstart/32 + msp[j] + b, msp the prefix of merge chunks
// per bucket: a bucket that merges has at least one chunk, so the term keeps
// its last block and the next such bucket's first apart when a bucket ends
// inside an aligned 32-key window; buckets of small segments have none, so
// the indices stay below n/32 + (chunks bound).
constexpr int kSampleBlock = 32;
__host__ __device__ inline int64_t sample_base(int64_t bstart, int32_t chunks_before) {
    return bstart / kSampleBlock + chunks_before;
}
// A split point records the round that wrote it (bits 8 and up), so that a
// slot left over from an earlier round is recognised instead of trusted.
__host__ __device__ constexpr int32_t round_tag(int round) { return (round + 1) << 8; }

template <typename K>
struct Work {
    K* keys;          // the caller's keys (sorted in place)
    uint32_t* vals;   // the caller's payload (stable pairs) or null
    K* skeys;         // scratch copy of the keys (ping-pong partner)
    uint32_t* svals;  // scratch payload (pairs) or null
    const int64_t* off;  // segment offsets [nseg + 1]
    int64_t n;           // keys addressable through `keys`
    int32_t nseg;

    // per histogram tile, then per segment
    K* tmin;                  // [tiles] min of each tile
    K* tmax;                  // [tiles] max of each tile
    uint64_t* tp;             // [tiles] the tile's own p when it has no negative key (its counts are in), else 0
    K* smpf;                  // [n/32 + buckets + 2] first key of each 32-key block (fan-in-4 rounds)
    K* smpl;                  // [n/32 + buckets + 2] last key of each full 32-key block
    DigitPlan<K>* plans;      // [nseg]
    int32_t* tilecnt;         // [nseg] histogram tiles of a large segment, 0 otherwise
    int32_t* tilepre;         // [nseg + 1] exclusive prefix of tilecnt
    int32_t* groupcnt;        // [nseg] groups of kGroupTiles tiles of a large segment
    int32_t* grouppre;        // [nseg + 1] exclusive prefix of groupcnt
    int64_t* bounds_out;      // [nseg * 11] bucket bounds relative to the segment start

    // per histogram tile, tile-major: [nbk * t + b] (t flat over all large segments)
    uint32_t* counts;  // keys of tile t in bucket b
    uint32_t* intra;   // sum of counts[t'][b] over the earlier tiles t' of t's group
    // per group of tiles
    uint32_t* gsum;    // [nbk * groups] group sums, bucket-major inside a segment (as the scan reads them)
    int64_t* gpos;     // [nbk * groups + 1] exclusive prefix of gsum
    int32_t* gbase;    // [nbk * g + b] group g's start in bucket b, relative to its segment's first key

    // per bucket (nbk per segment)
    int64_t* bstart;  // absolute first key of the bucket
    int64_t* bsize;
    int32_t* tsc;  // local-sort tiles of the bucket
    int32_t* tsp;  // [nbk * nseg + 1] prefix
    int32_t* mcc;  // merge chunks of the bucket
    int32_t* msp;  // [nbk * nseg + 1] prefix
    int32_t* brounds;  // merge rounds of the bucket (0 when its keys all share one value)

    TileDesc* tiles;   // [tiles bound]
    SortDesc* sdesc;   // [local-sort partitions bound]
    MergeDesc* mdesc;  // [merge chunks bound] of the current round (fan-in 2)
    Split4* ssorted;   // [merge chunks bound] split points by rank (fan-in 4)
    int32_t* rounds;  // largest number of merge rounds any bucket needs
    uint32_t* err;   // device-side validation flag (bad offsets)

    int32_t nbk;        // buckets per segment: 10 (one decimal digit), 100 (two) or 1000 (three)
    int32_t ptile;      // keys per partition tile (PartShape<nbk>::HT)
    int32_t ufix;       // keys are images of unsigned keys: beta fixed at the type's minimum
    int32_t img;        // order-image mode of the caller's keys (kImg* bits, 0: none): applied where the
                        // partition reads them, undone where a bucket's final output is written
    int32_t tile;       // keys per local-sort tile (T)
    int32_t fanin;      // runs merged per round: 2 or 4
    int32_t nv;         // outputs per merge workgroup (divides T)
    int64_t small_max;  // segments up to this size are sorted wholly in LDS
    int64_t max_seg_len;  // the caller's bound on the longest segment (merge rounds launched), 0 if none
};

// Order-image modes of other key types (bits; see k_image).
constexpr int kImgUnsigned = 1, kImgFloat = 2, kImgDesc = 4;

// Bits of the device-side error word (read by hsort_check).
constexpr uint32_t kErrOffsets = 1;      // offsets decreasing or outside [0, n]
constexpr uint32_t kErrConsistency = 2;  // a merge chunk inconsistent with its split points
constexpr uint32_t kErrSegLen = 4;       // a segment longer than the caller's max_seg_len

}  // namespace hs
