/*
 * hsort.h -- C ABI of the MI355X (gfx950) hybrid MSD-radix / tile-sort /
 * merge-path integer sort.
 *
 * Method (Alghamdi & Alaghband, "High Performance Parallel Sort for Shared
 * and Distributed Memory MIMD", arXiv 2003.01216, Section 3.4 with Sections
 * 3.1-3.2): a one-step decimal most-significant-digit partition of the keys
 * into ten non-overlapping buckets, a local sort of each bucket's partitions,
 * then non-recursive (bottom-up) merge rounds of the sorted runs inside each
 * bucket.  The buckets' order equals the key order, so the concatenation of
 * the sorted buckets is the sorted array (Section 3.4: every sorted bucket
 * returns to its own position in the array).
 *
 * Conventions for every entry point:
 *   - keys, vals, offsets and scratch are DEVICE pointers (hipMalloc'd or
 *     torch tensors); `stream` is a hipStream_t (NULL = the null stream).
 *   - sorts are in place, ascending, in signed integer order.
 *   - work is enqueued asynchronously on `stream`; the caller synchronises.
 *   - the library allocates no device memory: it works in the caller's
 *     `scratch` buffer of at least hsort_scratch_bytes(...) bytes.  Scratch
 *     contents are undefined after a call, except the bucket bounds (see
 *     hsort_bounds_offset) and the error word read by hsort_check.
 *   - argument errors (null pointer with n > 0, negative sizes, n above
 *     HSORT_MAX_KEYS, nseg above HSORT_MAX_SEGMENTS, scratch too small) are
 *     returned synchronously before anything is enqueued; n == 0 or
 *     nseg == 0 is a no-op returning HSORT_OK.  A failed launch returns
 *     HSORT_ERR_HIP with a message in hsort_last_error().  Invalid segment
 *     offsets, and a segment longer than the caller's max_seg_len, are
 *     detected on the device: every kernel of the call then does nothing
 *     (the keys are left as they were), and hsort_check() reports
 *     HSORT_ERR_INVALID.  No C++ exception crosses this boundary.
 *   - calls on distinct scratch buffers may run concurrently on distinct
 *     streams; the host-side state (configuration, timing records) is
 *     guarded by a mutex.
 */
#ifndef HSORT_H
#define HSORT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    HSORT_OK = 0,
    HSORT_ERR_INVALID = 1,     /* bad argument or bad offsets */
    HSORT_ERR_SCRATCH = 2,     /* scratch buffer too small */
    HSORT_ERR_HIP = 3,         /* a HIP runtime call failed */
    HSORT_ERR_UNSUPPORTED = 4, /* size beyond HSORT_MAX_KEYS */
    HSORT_ERR_BUDGET = 5       /* serving layer: request larger than the memory budget */
} hsort_status;

typedef enum {
    HSORT_KEYS_I32 = 0,      /* int32 keys */
    HSORT_KEYS_I64 = 1,      /* int64 keys */
    HSORT_PAIRS_I32_U32 = 2, /* int32 keys + uint32 payload, stable */
    HSORT_SEG_I32 = 3,       /* segmented int32 keys */
    HSORT_SEG_I64 = 4,       /* segmented int64 keys */
    HSORT_PAIRS_I64_U32 = 5  /* int64 keys + uint32 payload, stable */
} hsort_kind;

/* Key types of hsort_sort (Section 3.4's integers, and the types a sort
 * library is asked for besides). */
typedef enum {
    HSORT_I32 = 0, /* int32 */
    HSORT_U32 = 1, /* uint32 */
    HSORT_F32 = 2, /* IEEE-754 binary32 */
    HSORT_I64 = 3, /* int64 */
    HSORT_U64 = 4, /* uint64 */
    HSORT_F64 = 5  /* IEEE-754 binary64 */
} hsort_key_type;
#define HSORT_DESCENDING 1 /* flag of hsort_sort: largest key first */

/* Largest number of keys in one call (and in one segment). */
#define HSORT_MAX_KEYS ((int64_t)2147483647)
/* Largest number of segments in one segmented call (the per-bucket tables
 * index buckets of all segments with 32-bit integers). */
#define HSORT_MAX_SEGMENTS ((int64_t)16777216)

/* Bytes of scratch a call of `kind` over n keys in nseg segments needs
 * (nseg is ignored for the non-segmented kinds).  Pure host function. */
size_t hsort_scratch_bytes(int kind, int64_t n, int64_t nseg);

/* Sorts keys[0..n) ascending (Section 3.4 method). */
int hsort_keys_i32(int32_t* keys, int64_t n, void* scratch, size_t scratch_bytes, void* stream);
int hsort_keys_i64(int64_t* keys, int64_t n, void* scratch, size_t scratch_bytes, void* stream);

/* For callers that cannot allocate device memory (code under stream
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * sort as hsort_keys_i32, with no scratch argument.  It works in a scratch
 * array of HSORT_NOALLOC_SCRATCH_BYTES that the library owns, one per GPU,
 * held until the process ends; it calls no hipMalloc, hipFree or other
 * allocating routine, and bypasses the graph cache and the timing records.
 * n above HSORT_NOALLOC_MAX_KEYS: HSORT_ERR_UNSUPPORTED at once (also if a
 * tuning table picks shapes whose scratch would not fit).  Every call on one
 * GPU shares that GPU's array, which keeps the last call's contents: calls
 * that overlap on one GPU (concurrent streams or threads) race and must be
 * serialised by the caller. */
#define HSORT_NOALLOC_MAX_KEYS ((int64_t)4194304)
#define HSORT_NOALLOC_SCRATCH_BYTES (24u << 20)
int hsort_keys_i32_noalloc(int32_t* keys, int64_t n, void* stream);

/* Sorts keys[0..n) ascending and permutes vals[0..n) with them.  Stable:
 * equal keys keep their input order (merge sort's stability, Section 2.1). */
int hsort_pairs(int32_t* keys, uint32_t* vals, int64_t n, void* scratch, size_t scratch_bytes, void* stream);

/* Sorts keys[0..n) of any hsort_key_type, ascending or (flags =
 * HSORT_DESCENDING) descending, and permutes vals[0..n) with them when vals
 * is not NULL.  Stable: equal keys keep their input order in both
 * directions.  Floats follow the IEEE-754 total order (-NaN < -inf < ... <
 * -0 < +0 < ... < +inf < +NaN; NaNs by sign and payload), so every bit
 * pattern has one place and the output is unique.  The method is the one of
 * Section 3.4 applied to an order image of the keys: a signed integer of
 * the same width whose order is the order asked for (unsigned: the sign bit
 * flipped; floats: the magnitude bits of negative values flipped;
 * descending: the image complemented), taken where the partition reads
 * the keys and undone where each bucket's final output is written (no
 * extra pass over the array).  The bucket rule reads that image (unsigned
 * keys keep
 * their value: u = k, no bias; the bounds left in scratch are the image's).
 * Scratch: hsort_sort_scratch_bytes(key_type, vals != NULL, n) bytes.
 * Unknown key_type or flags: HSORT_ERR_INVALID at once. */
int hsort_sort(void* keys, uint32_t* vals, int64_t n, int key_type, int flags, void* scratch, size_t scratch_bytes,
               void* stream);
size_t hsort_sort_scratch_bytes(int key_type, int with_vals, int64_t n);

/* Sorts each segment keys[offsets[i] .. offsets[i+1]) independently, for
 * i in [0, nseg) (Section 3.4: the buckets are independent units of work;
 * here every segment gets its own buckets and all buckets of all segments
 * form one flat work list).  Ascending, in place.
 *   keys:        device array of n keys (n bounds the offsets; keys outside
 *                [offsets[0], offsets[nseg]) are untouched).
 *   offsets:     nseg+1 device int64, non-decreasing, with 0 <= offsets[0]
 *                and offsets[nseg] <= n.  Read on the device only, so a
 *                graph replay may change their values.
 *   max_seg_len: 0, or an upper bound on every segment's length.  A bound
 *                lets the call launch only the merge rounds such a segment
 *                needs and selects the tuning class; it is checked on the
 *                device, and a longer segment makes the whole call do
 *                nothing and hsort_check() report HSORT_ERR_INVALID.
 *                Negative: HSORT_ERR_INVALID at once.
 *   nseg:        at most HSORT_MAX_SEGMENTS (else HSORT_ERR_UNSUPPORTED).
 * The bucket bounds of every segment are left in scratch (hsort_bounds_offset). */
int hsort_segmented(int32_t* keys, int64_t n, const int64_t* offsets, int64_t nseg, int64_t max_seg_len,
                    void* scratch, size_t scratch_bytes, void* stream);
int hsort_segmented_i64(int64_t* keys, int64_t n, const int64_t* offsets, int64_t nseg, int64_t max_seg_len,
                        void* scratch, size_t scratch_bytes, void* stream);

/* Byte offset inside scratch of the bucket bounds the last call on that
 * scratch left behind: int64 bounds[nseg][11] (nseg = 1 for the plain
 * kinds), bounds[s][b] = number of keys of segment s whose one-step decimal
 * MSD bucket (Section 3.4) is below b.  Valid after the call completes and
 * until the scratch is reused. */
size_t hsort_bounds_offset(int kind, int64_t n, int64_t nseg);

/* Synchronises `stream` and reads the device-side error word of the last
 * call that used `scratch`: HSORT_ERR_INVALID if its offsets were invalid,
 * a segment was longer than its max_seg_len, or a device-side consistency
 * check failed,
 * HSORT_ERR_HIP if the synchronisation failed, HSORT_OK otherwise. */
int hsort_check(const void* scratch, void* stream);

/* Message for the last error on the calling thread ("" if none). */
const char* hsort_last_error(void);

/* ---------------------------------------------------------------- tuning
 * The shape of the local sort and of the merge, per key kind and size
 * class: tile = keys per local-sort partition (T), tile_vt = keys per thread
 * of that sort (T / tile_vt threads per workgroup); merge_nv = outputs per
 * merge workgroup, merge_vt = outputs per thread; small_max = segments (and
 * plain arrays) up to this size are sorted wholly in LDS; fanin = runs
 * merged per round, 2 (pairwise rounds, Figure 1b) or 4 (each round merges
 * four runs: half as many rounds; a split point is placed by two-way
 * searches only, see the kernels); digits = decimal digits of the one-step
 * partition, 1 (the ten buckets of Section 3.4) or 2 (one hundred buckets by
 * the first two of the D digits, floor(u / 10^(D-2)), or 10u when D = 1: a
 * finer splitter with the same order, so bucket b of the ten is buckets
 * 10b .. 10b+9 of the hundred; smaller buckets need fewer merge rounds)
 * or 3 (one thousand buckets, floor(u / 10^(D-3)), the digits of a shorter u
 * followed by zeros; plain 32-bit sorts only, kinds HSORT_KEYS_I32 and
 * HSORT_PAIRS_I32_U32, and with them the uint32/float32 sorts of
 * hsort_sort; keys-only partition tiles then hold 16384 keys instead of
 * 4096, and a bucket whose digits fix one key value is copied, not
 * sorted).  The exported bounds are
 * the ten-bucket bounds in every case.  local = the
 * local sort: 0 (a register network, merges across lanes, then merge levels
 * in LDS) or 1 (the non-recursive merge sort of Figure 1b: each thread sorts
 * its tile_vt keys -- pairs when tile_vt = 2 -- and every merge level runs
 * bottom up in LDS).  merge_nv must
 * divide tile.  Only compiled shapes are accepted (HSORT_ERR_UNSUPPORTED
 * otherwise).  kind: any hsort_kind; every kind has rows of its own (a
 * segmented kind is tuned apart from the plain sort of its key type, accepts
 * that key type's compiled shapes, and at most two digits).  Size classes
 * 0..3 hold calls whose deciding
 * size -- n, or max_seg_len of a segmented call when given -- is at most
 * 2^18, 2^22, 2^26, or larger (hsort_size_class(n) maps a size to its
 * class); size_cls = -1 sets every class.  The table is process-wide, and
 * scratch sizes depend on it: size scratch after changing it. */
int hsort_set_config(int kind, int size_cls, int64_t tile, int64_t tile_vt, int64_t merge_nv, int64_t merge_vt,
                     int64_t small_max, int64_t fanin, int64_t digits, int64_t local);
int hsort_get_config(int kind, int size_cls, int64_t* tile, int64_t* tile_vt, int64_t* merge_nv, int64_t* merge_vt,
                     int64_t* small_max, int64_t* fanin, int64_t* digits, int64_t* local);
int hsort_size_class(int64_t n);

/* Applies a tuning table written by the autotuner: text lines
 * "kind size_class tile tile_vt merge_nv merge_vt small_max fanin [digits [local]]"
 * (digits 1 and local 0 when left out; '#' starts a comment line).  Stops at the first
 * bad line and returns its error. */
int hsort_load_tuning(const char* path);

/* ----------------------------------------------------- test observability
 * Runs the plain-sort pipeline (kinds HSORT_KEYS_I32, HSORT_KEYS_I64,
 * HSORT_PAIRS_I32_U32) only up to `stage` and leaves that intermediate in
 * keys (and vals): 1 = after the one-step stable bucket scatter (keys in
 * bucket order, input order inside each bucket); 2 = after the local sorts
 * (every `tile`-key partition of every bucket, counted from the bucket's
 * first key, sorted on its own); 3 = the full sort.  vals may be NULL
 * except for pairs. */
int hsort_debug_stage(int kind, void* keys, uint32_t* vals, int64_t n, int stage, void* scratch,
                      size_t scratch_bytes, void* stream);
/* The same for hsort_sort's key types and flags (the intermediate is left
 * in the caller's key values: the order image is undone after the stage). */
int hsort_debug_stage_typed(void* keys, uint32_t* vals, int64_t n, int key_type, int flags, int stage, void* scratch,
                            size_t scratch_bytes, void* stream);

/* ----------------------------------------------------------- hipGraphs
 * With graph mode on, each distinct call -- same entry point, sizes,
 * pointers, shapes and stream -- is captured once into a hipGraph (on the
 * first such call) and replayed on later calls, which removes the per-kernel
 * launch cost of the pass sequence.  The graphs read every data-dependent
 * quantity (segment sizes, bucket sizes, work lists) on the device, so a
 * replay with new key values or new offsets values is exact.  Calls on the
 * null stream, and calls on a stream the caller is already capturing, are
 * launched directly.  At most 64 graphs are cached (least recently used is
 * dropped); hsort_graph_clear() destroys them all (call it before freeing
 * buffers a cached graph refers to, if their addresses may be reused for
 * calls of other sizes). */
int hsort_graph_mode(int on);
int hsort_graph_clear(void);
int64_t hsort_graph_count(void);

/* Per-kernel timing.  While enabled, every group of kernel launches of the
 * library (a pass: "range", "scatter", "tilesort", one "merge" per round,
 * ...) is bracketed by HIP events recorded on the call's stream; launches
 * inside a captured graph (graph mode, or a caller's capture) are not
 * recorded.  hsort_timing_read synchronises those events and writes, for
 * each name, the number of launches, the total milliseconds and the
 * algorithmic HBM bytes those launches had to move (a merge round's from
 * the keys of the buckets still merging in it), as text lines "name
 * launches total_ms bytes"; it returns the number of bytes written (or
 * needed, if cap is too small) and clears the records.  Timing is best
 * effort and never fails a sort: a pass whose events cannot be created or
 * read is left out, and a merge round whose bucket table cannot be read
 * reports zero bytes. */
int hsort_timing_enable(int on);
int64_t hsort_timing_read(char* out, int64_t cap);

/* Plain device-to-device copy of `bytes` (multiple of 16) with the library's
 * copy kernel, used to calibrate hardware byte counters. */
int hsort_copy(const void* src, void* dst, int64_t bytes, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* HSORT_H */
