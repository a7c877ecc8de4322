// hs_launch.h -- host-side launchers of the kernels in hs_kernels.hip.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hs_work.h"

namespace hs {

// Length of a scan: len_mul * (*len_ptr) read on the device, or len_const.
struct ScanSpec {
    const int32_t* len_ptr;
    int64_t len_mul;
    int64_t len_const;
};

// Compiled (key, stable pairs, threads, keys per thread) shapes of the LDS
// sort (local-sort tiles and whole small segments) and of the merge.
#define HS_TILE_VARIANTS(X)                                                                  \
    X(int32_t, false, 1024, 32) X(int32_t, false, 512, 32) X(int32_t, false, 256, 32)        \
    X(int32_t, false, 512, 16)                                                               \
    X(int32_t, false, 256, 16) X(int32_t, false, 256, 8) X(int32_t, false, 64, 4)            \
    X(int64_t, false, 512, 16)                                                               \
    X(int64_t, false, 256, 16) X(int64_t, false, 256, 8) X(int64_t, false, 64, 4)            \
    X(int32_t, true, 512, 16) X(int32_t, true, 256, 16) X(int32_t, true, 256, 8) X(int32_t, true, 64, 4)       \
    X(int64_t, true, 512, 8) X(int64_t, true, 256, 8) X(int64_t, true, 64, 4)
// Shapes of the alternative local sort (bottom-up LDS merge levels from the
// threads' own runs, no lane merges; VT = 2 is the figure's pairs).
#define HS_TILE_BU_VARIANTS(X)                                                               \
    X(int32_t, false, 1024, 2) X(int32_t, false, 512, 8) X(int32_t, true, 1024, 2) X(int64_t, false, 1024, 2)
#define HS_MERGE_VARIANTS(X)                                                                 \
    X(int32_t, false, 256, 16) X(int32_t, false, 256, 32) X(int32_t, false, 512, 16)         \
    X(int64_t, false, 256, 16) X(int32_t, true, 256, 16) X(int64_t, true, 256, 8)
// Fan-in-4 merge: (key, pairs, threads NT, outputs per job VT, jobs per
// thread and level JOBS); sampling stride S = NT*VT*JOBS/2 = merge_nv, a
// workgroup holds up to 2S keys.  One variant per (S, VT): 4096/16, 2048/16
// and 2048/8 for every key kind.
#define HS_MERGE4_VARIANTS(X)                                                                \
    X(int32_t, false, 512, 16, 1) X(int32_t, false, 256, 16, 1) X(int32_t, false, 256, 8, 2)  \
    X(int64_t, false, 256, 16, 2) X(int64_t, false, 256, 16, 1) X(int64_t, false, 512, 8, 1)  \
    X(int32_t, true, 256, 16, 2) X(int32_t, true, 256, 16, 1) X(int32_t, true, 512, 8, 1)    \
    X(int64_t, true, 256, 8, 1) X(int64_t, true, 256, 8, 2)
// Shapes usable by the whole-segment LDS sort (5-bit digit counters: VT <= 16;
// 16-byte words of int64 pairs: VT <= 8).
#define HS_SMALL_VARIANTS(X)                                                                 \
    X(int32_t, false, 512, 16) X(int32_t, false, 256, 16) X(int32_t, false, 256, 8) X(int32_t, false, 64, 4) \
    X(int64_t, false, 512, 16) X(int64_t, false, 256, 16) X(int64_t, false, 256, 8) X(int64_t, false, 64, 4) \
    X(int32_t, true, 512, 16) X(int32_t, true, 256, 16) X(int32_t, true, 256, 8) X(int32_t, true, 64, 4)     \
    X(int64_t, true, 512, 8) X(int64_t, true, 256, 8) X(int64_t, true, 64, 4)

// Each launcher sizes its own (persistent) grid from an upper bound on the
// number of work items it can be handed.
template <typename K>
hipError_t launch_setup(const Work<K>& w, int64_t* own_off, int64_t tiles_bound, hipStream_t st);
template <typename K>
hipError_t launch_range(const Work<K>& w, int64_t tiles_bound, hipStream_t st);
template <typename K>
hipError_t launch_plans(const Work<K>& w, hipStream_t st);
template <typename K>
hipError_t launch_hist(const Work<K>& w, int64_t tiles_bound, hipStream_t st);
template <typename K>
hipError_t launch_btab(const Work<K>& w, hipStream_t st);
template <typename K>
hipError_t launch_colsum(const Work<K>& w, int64_t groups_bound, hipStream_t st);
// A plain sort whose partition tiles form one group: the bucket offsets,
// the bucket table and the scans of its tile and chunk counts in one launch.
template <typename K>
hipError_t launch_offsets1(const Work<K>& w, int64_t ts_bound, hipStream_t st);
template <typename K>
hipError_t launch_gbase(const Work<K>& w, int64_t groups_bound, hipStream_t st);
template <typename K, bool PAIRS>
hipError_t launch_scatter(const Work<K>& w, int64_t tiles_bound, hipStream_t st);
template <typename K, bool PAIRS, int NT, int VT, bool BU>
hipError_t launch_tilesort(const Work<K>& w, int64_t items_bound, hipStream_t st);
template <typename K>
hipError_t launch_partition(const Work<K>& w, int pass, int64_t chunks_bound, hipStream_t st);
template <typename K, bool PAIRS, int NT, int VT>
hipError_t launch_merge(const Work<K>& w, int64_t chunks_bound, hipStream_t st);
template <typename K>
hipError_t launch_tiles(const Work<K>& w, int64_t tiles_bound, hipStream_t st);
template <typename K>
hipError_t launch_sdesc(const Work<K>& w, int64_t items_bound, hipStream_t st);
template <typename K, bool PAIRS, int NT, int VT>
hipError_t launch_small(const Work<K>& w, int64_t lo, int64_t hi, int64_t segs_bound, hipStream_t st);
template <typename K>
hipError_t launch_collect(const Work<K>& w, int stage, hipStream_t st);
template <typename K>
hipError_t launch_part4(const Work<K>& w, int round, int64_t chunks_bound, hipStream_t st);
template <typename K, bool PAIRS, int NT, int VT, int JOBS>
hipError_t launch_merge4(const Work<K>& w, int round, int64_t chunks_bound, hipStream_t st);

hipError_t launch_scan_i32(const ScanSpec& sp, int64_t len_bound, const int32_t* in, int32_t* out, int32_t* partial,
                           hipStream_t st);
hipError_t launch_scan_u32_i64(const ScanSpec& sp, int64_t len_bound, const uint32_t* in, int64_t* out,
                               int64_t* partial, hipStream_t st);
int64_t scan_partial_count(int64_t len_bound);
// In-place order image of other key types (mode: kImg* bits of hs_kernels.hip)
// and its inverse.
template <typename K>
hipError_t launch_image(K* keys, int64_t n, int mode, bool inverse, hipStream_t st);
hipError_t launch_copy(const void* src, void* dst, int64_t bytes, hipStream_t st);

}  // namespace hs
