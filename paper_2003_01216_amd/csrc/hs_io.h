// hs_io.h -- moving runs of keys between HBM and a workgroup with 16-byte
// accesses.  On gfx950 a wavefront's 4-byte loads stream at about two thirds
// of the rate of 16-byte loads, so a run [p, p + cnt) is split into a
// scalar head up to the first 16-byte boundary, a body of aligned 16-byte
// vectors, and a scalar tail.  No vector access is ever misaligned.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hs_device.h"

namespace hs {

template <typename T>
struct Vec16;
template <>
struct Vec16<int32_t> {
    using type = int4;
    static constexpr int n = 4;
    static __device__ __forceinline__ int32_t get(const int4& v, int e) {
        return e == 0 ? v.x : e == 1 ? v.y : e == 2 ? v.z : v.w;
    }
    static __device__ __forceinline__ int4 make(int32_t a, int32_t b, int32_t c, int32_t d) {
        return int4{a, b, c, d};
    }
};
template <>
struct Vec16<uint32_t> {
    using type = uint4;
    static constexpr int n = 4;
    static __device__ __forceinline__ uint32_t get(const uint4& v, int e) {
        return e == 0 ? v.x : e == 1 ? v.y : e == 2 ? v.z : v.w;
    }
    static __device__ __forceinline__ uint4 make(uint32_t a, uint32_t b, uint32_t c, uint32_t d) {
        return uint4{a, b, c, d};
    }
};
template <>
struct Vec16<int64_t> {
    using type = longlong2;
    static constexpr int n = 2;
    static __device__ __forceinline__ int64_t get(const longlong2& v, int e) { return e == 0 ? v.x : v.y; }
};

// A computed address of global memory, typed so that loads through it are
// global loads (an integer cast to a generic pointer gives flat loads, which
// also count against the LDS wait counter).
template <typename V>
__device__ __forceinline__ const V* global_at(uintptr_t a) {
    return (const V*)reinterpret_cast<const __attribute__((address_space(1))) V*>(a);
}

// Elements of [0, cnt) before the first 16-byte boundary of src.
template <typename T>
__device__ __forceinline__ int head_len(const T* src, int cnt) {
    constexpr int E = Vec16<T>::n;
    const int mis = (int)(((uintptr_t)src & 15) / sizeof(T));
    const int h = mis ? E - mis : 0;
    return h < cnt ? h : cnt;
}

// Calls put(q, src[q]) for every q in [0, cnt), cnt <= MAXCNT, reading the
// aligned body with 16-byte loads (all of them issued before any put).
template <typename T, int NT, int MAXCNT, typename F>
__device__ __forceinline__ void load_run(const T* src, int cnt, F&& put) {
    constexpr int E = Vec16<T>::n;
    using V = typename Vec16<T>::type;
    constexpr int PER = (MAXCNT / E + NT - 1) / NT;
    const int tid = threadIdx.x;
    const int head = head_len(src, cnt);
    const int body = (cnt - head) / E;
    const int tail = head + body * E;
    const V* vs = reinterpret_cast<const V*>(src + head);
    V x[PER];
#pragma unroll
    for (int j = 0; j < PER; j++) {
        const int v = j * NT + tid;
        if (v < body) x[j] = vs[v];
    }
    if (tid < head) put(tid, src[tid]);
    if (tid < cnt - tail) put(tail + tid, src[tail + tid]);
#pragma unroll
    for (int j = 0; j < PER; j++) {
        const int v = j * NT + tid;
        if (v < body) {
#pragma unroll
            for (int e = 0; e < E; e++) put(head + v * E + e, Vec16<T>::get(x[j], e));
        }
    }
}

// Several runs at once: calls put(off[r] + q, src[r][q]) for every run r and
// q in [0, cnt[r]), sum of cnt <= MAXTOT.  The runs' aligned bodies form one
// index space of 16-byte vectors shared out over the workgroup, and every
// load (vector, head and tail) is issued before the first put, so the runs'
// memory latencies overlap instead of adding up.
template <typename T, int NT, int MAXTOT, int NR, typename F>
__device__ __forceinline__ void load_runs(const T* const (&src)[NR], const int (&cnt)[NR], const int (&off)[NR],
                                          F&& put) {
    constexpr int E = Vec16<T>::n;
    using V = typename Vec16<T>::type;
    constexpr int PER = (MAXTOT / E + NT - 1) / NT;
    const int tid = threadIdx.x;
    int head[NR], tail[NR], pre[NR + 1];
    uintptr_t vbase[NR];  // address of vector 0 of the shared index space, as seen from run r
    int dbase[NR];        // put index of vector 0, as seen from run r
    pre[0] = 0;
#pragma unroll
    for (int r = 0; r < NR; r++) {
        head[r] = head_len(src[r], cnt[r]);
        const int body = (cnt[r] - head[r]) / E;
        tail[r] = head[r] + body * E;
        pre[r + 1] = pre[r] + body;
        vbase[r] = (uintptr_t)(src[r] + head[r]) - (uintptr_t)pre[r] * sizeof(V);
        dbase[r] = off[r] + head[r] - pre[r] * E;
    }
    V x[PER];
#pragma unroll
    for (int j = 0; j < PER; j++) {
        const int v = j * NT + tid;
        if (v < pre[NR]) {
            uintptr_t b = vbase[0];
#pragma unroll
            for (int r = 1; r < NR; r++) b = v >= pre[r] ? vbase[r] : b;
            x[j] = global_at<V>(b)[v];
        }
    }
    T hv[NR], tv[NR];
#pragma unroll
    for (int r = 0; r < NR; r++) {
        if (tid < head[r]) hv[r] = src[r][tid];
        if (tid < cnt[r] - tail[r]) tv[r] = src[r][tail[r] + tid];
    }
#pragma unroll
    for (int r = 0; r < NR; r++) {
        if (tid < head[r]) put(off[r] + tid, hv[r]);
        if (tid < cnt[r] - tail[r]) put(off[r] + tail[r] + tid, tv[r]);
    }
#pragma unroll
    for (int j = 0; j < PER; j++) {
        const int v = j * NT + tid;
        if (v < pre[NR]) {
            int d = dbase[0];
#pragma unroll
            for (int r = 1; r < NR; r++) d = v >= pre[r] ? dbase[r] : d;
            d += v * E;
#pragma unroll
            for (int e = 0; e < E; e++) put(d + e, Vec16<T>::get(x[j], e));
        }
    }
}

// Runs into LDS in two halves: issue() starts every global load of the runs
// (16-byte body vectors shared out over the workgroup, scalar heads and
// tails) into registers, all before any LDS write; commit() writes them to
// LDS.  commit_padded puts element q of run r into a padded array at logical
// position at[r] + q as xf(off[r] + q, src[r][q]) (off: the element's index
// in the concatenation of the runs).  The caller places each run so that its
// body vectors start on logical multiples of 4, (at[r] + head_len(src[r],
// cnt[r])) % 4 == 0; a vector's words then share one pad period and sit at
// constant offsets from one address.
template <typename K, int NT, int MAXTOT, int NR>
struct RunsToLds {
    static constexpr int E = Vec16<K>::n;
    using V = typename Vec16<K>::type;
    static constexpr int PER = (MAXTOT / E + NT - 1) / NT;
    V x[PER];
    K hv[NR], tv[NR];
    int head[NR], tail[NR], cnt[NR], at[NR], off[NR], pre[NR + 1], wbase[NR], obase[NR];

    __device__ __forceinline__ void issue(const K* const (&src)[NR], const int (&cnt_)[NR], const int (&at_)[NR],
                                          const int (&off_)[NR]) {
        const int tid = threadIdx.x;
        uintptr_t vbase[NR];
        pre[0] = 0;
#pragma unroll
        for (int r = 0; r < NR; r++) {
            cnt[r] = cnt_[r];
            at[r] = at_[r];
            off[r] = off_[r];
            head[r] = head_len(src[r], cnt[r]);
            const int body = (cnt[r] - head[r]) / E;
            tail[r] = head[r] + body * E;
            pre[r + 1] = pre[r] + body;
            vbase[r] = (uintptr_t)(src[r] + head[r]) - (uintptr_t)pre[r] * sizeof(V);
            wbase[r] = at[r] + head[r] - pre[r] * E;  // logical LDS position of vector 0, seen from run r
            obase[r] = off[r] + head[r] - pre[r] * E;  // concatenated index of vector 0, seen from run r
        }
#pragma unroll
        for (int j = 0; j < PER; j++) {
            const int v = j * NT + tid;
            if (v < pre[NR]) {
                uintptr_t b = vbase[0];
#pragma unroll
                for (int r = 1; r < NR; r++) b = v >= pre[r] ? vbase[r] : b;
                x[j] = global_at<V>(b)[v];
            }
        }
#pragma unroll
        for (int r = 0; r < NR; r++) {
            if (tid < head[r]) hv[r] = src[r][tid];
            if (tid < cnt[r] - tail[r]) tv[r] = src[r][tail[r] + tid];
        }
    }

    // put1(pos, idx, key) for single elements, putv(pos, idx, keys[E]) for a
    // body vector (pos = logical position at[r] + q, a multiple of 4 for
    // vectors; idx = off[r] + q).
    template <typename P1, typename PV>
    __device__ __forceinline__ void commit(P1&& put1, PV&& putv) const {
        const int tid = threadIdx.x;
#pragma unroll
        for (int r = 0; r < NR; r++) {
            if (tid < head[r]) put1(at[r] + tid, off[r] + tid, hv[r]);
            if (tid < cnt[r] - tail[r]) put1(at[r] + tail[r] + tid, off[r] + tail[r] + tid, tv[r]);
        }
#pragma unroll
        for (int j = 0; j < PER; j++) {
            const int v = j * NT + tid;
            if (v < pre[NR]) {
                int d = wbase[0], o = obase[0];
#pragma unroll
                for (int r = 1; r < NR; r++) {
                    d = v >= pre[r] ? wbase[r] : d;
                    o = v >= pre[r] ? obase[r] : o;
                }
                K k[E];
#pragma unroll
                for (int e = 0; e < E; e++) k[e] = Vec16<K>::get(x[j], e);
                putv(d + v * E, o + v * E, k);
            }
        }
    }

    // Keys as words of a padded LDS array: words[lds_pad(pos)] = xf(idx, key).
    template <typename W, typename XF>
    __device__ __forceinline__ void commit_padded(W* words, XF&& xf) const {
        commit([&](int pos, int idx, K k) { words[lds_pad<W>(pos)] = xf(idx, k); },
               [&](int pos, int idx, const K (&k)[E]) {
                   W* dst = words + lds_pad<W>(pos);
#pragma unroll
                   for (int e = 0; e < E; e++) dst[e] = xf(idx + e, k[e]);
               });
    }

    // Dense by concatenated index: dst[idx] = key.
    __device__ __forceinline__ void commit_dense(K* dst) const {
        commit([&](int, int idx, K k) { dst[idx] = k; },
               [&](int, int idx, const K (&k)[E]) {
#pragma unroll
                   for (int e = 0; e < E; e++) dst[idx + e] = k[e];
               });
    }
};

// Writes dst[q] = get(q) for every q in [0, cnt), cnt <= MAXCNT, with 16-byte
// stores for the aligned body (4-byte elements only).
template <typename T, int NT, int MAXCNT, typename G>
__device__ __forceinline__ void store_run(T* dst, int cnt, G&& get) {
    static_assert(Vec16<T>::n == 4, "store_run handles 4-byte elements");
    using V = typename Vec16<T>::type;
    constexpr int PER = (MAXCNT / 4 + NT - 1) / NT;
    const int tid = threadIdx.x;
    const int head = head_len(dst, cnt);
    const int body = (cnt - head) / 4;
    const int tail = head + body * 4;
    if (tid < head) dst[tid] = get(tid);
    if (tid < cnt - tail) dst[tail + tid] = get(tail + tid);
    V* vd = reinterpret_cast<V*>(dst + head);
#pragma unroll
    for (int j = 0; j < PER; j++) {
        const int v = j * NT + tid;
        if (v < body) {
            const int q = head + v * 4;
            vd[v] = Vec16<T>::make(get(q), get(q + 1), get(q + 2), get(q + 3));
        }
    }
}

// 8-byte elements: pairs of 16 bytes.
template <int NT, int MAXCNT, typename G>
__device__ __forceinline__ void store_run64(int64_t* dst, int cnt, G&& get) {
    constexpr int PER = (MAXCNT / 2 + NT - 1) / NT;
    const int tid = threadIdx.x;
    const int head = head_len(dst, cnt);
    const int body = (cnt - head) / 2;
    const int tail = head + body * 2;
    if (tid < head) dst[tid] = get(tid);
    if (tid < cnt - tail) dst[tail + tid] = get(tail + tid);
    longlong2* vd = reinterpret_cast<longlong2*>(dst + head);
#pragma unroll
    for (int j = 0; j < PER; j++) {
        const int v = j * NT + tid;
        if (v < body) {
            const int q = head + v * 2;
            vd[v] = longlong2{get(q), get(q + 1)};
        }
    }
}

// dst[q] = src[q] for q in [0, cnt): 16-byte vectors when both pointers
// share their offset inside 16 bytes (equal offsets into two aligned
// arrays), element by element otherwise.
template <typename T, int NT>
__device__ __forceinline__ void copy_run(T* dst, const T* src, int cnt) {
    constexpr int E = 16 / (int)sizeof(T);
    const int tid = threadIdx.x;
    if ((((uintptr_t)dst ^ (uintptr_t)src) & 15) == 0) {
        int head = (int)(((16 - ((uintptr_t)src & 15)) & 15) / sizeof(T));
        head = head < cnt ? head : cnt;
        const int body = (cnt - head) / E;
        const int tail = head + body * E;
        if (tid < head) dst[tid] = src[tid];
        if (tid < cnt - tail) dst[tail + tid] = src[tail + tid];
        const uint4* vs = reinterpret_cast<const uint4*>(src + head);
        uint4* vd = reinterpret_cast<uint4*>(dst + head);
#pragma unroll 4
        for (int v = tid; v < body; v += NT) vd[v] = vs[v];
    } else {
        for (int q = tid; q < cnt; q += NT) dst[q] = src[q];
    }
}

template <typename K, int NT, int MAXCNT, typename G>
__device__ __forceinline__ void store_keys(K* dst, int cnt, G&& get) {
    if constexpr (sizeof(K) == 8)
        store_run64<NT, MAXCNT>(dst, cnt, get);
    else
        store_run<K, NT, MAXCNT>(dst, cnt, get);
}

}  // namespace hs
