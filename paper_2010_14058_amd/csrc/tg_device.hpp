// Device helpers shared by the library's kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tg_internal.hpp"

namespace tg {

// ---------------------------------------------------------------- helpers

static __device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

static __device__ __forceinline__ int lane_id() { return threadIdx.x & (WAVE - 1); }

static __device__ __forceinline__ int64_t lower_bound(const int32_t *a, int64_t lo, int64_t hi,
                                               int32_t key) {
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if (a[mid] < key) lo = mid + 1; else hi = mid;
    }
    return lo;
}

static __device__ __forceinline__ int64_t upper_bound(const int32_t *a, int64_t lo, int64_t hi,
                                               int32_t key) {
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if (a[mid] <= key) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// First index in s[0..len) whose value exceeds f (s inclusive scan, LDS).
static __device__ __forceinline__ int owner_of(const uint32_t *s, int len, uint32_t f) {
    int lo = 0, hi = len;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (s[mid] <= f) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// owner_of for a thread whose item index f only grows: o is the owner of
// the previous f; most steps stay in the same item (one LDS read), else the
// search restarts above o.
static __device__ __forceinline__ int owner_next(const uint32_t *s, int len, uint32_t f, int o) {
    if (s[o] > f) return o;
    int lo = o + 1, hi = len;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (s[mid] <= f) lo = mid + 1; else hi = mid;
    }
    return lo;
}

static __device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
    int lane = lane_id();
#pragma unroll
    for (int d = 1; d < WAVE; d <<= 1) {
        uint32_t o = __shfl_up(v, d, WAVE);
        if (lane >= d) v += o;
    }
    return v;
}

static __device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
#pragma unroll
    for (int d = WAVE / 2; d > 0; d >>= 1) v += (uint64_t)__shfl_xor((unsigned long long)v, d, WAVE);
    return v;
}

static __device__ __forceinline__ uint32_t wave_or(uint32_t v) {
#pragma unroll
    for (int d = WAVE / 2; d > 0; d >>= 1) v |= __shfl_xor(v, d, WAVE);
    return v;
}

static __device__ __forceinline__ uint32_t load_agent(const uint32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// True once an input check has failed (the status word written by earlier
// kernels of the call): later kernels return at once.
static __device__ __forceinline__ bool input_failed(const uint32_t *status) {
    return (__hip_atomic_load(status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & ST_INPUT) != 0;
}

// C(n, r) for r <= 4 (co-lexicographic ranks of type multisets).
static __device__ __forceinline__ int64_t binom_small(int64_t n, int r) {
    if (n < r) return 0;
    switch (r) {
        case 1: return n;
        case 2: return n * (n - 1) / 2;
        case 3: return n * (n - 1) * (n - 2) / 6;
        default: return n * (n - 1) * (n - 2) * (n - 3) / 24;
    }
}

static __device__ __forceinline__ void sort2(int &a, int &b) { if (a > b) { int c = a; a = b; b = c; } }

static __device__ __forceinline__ int rank2(int a, int b) {
    sort2(a, b);
    return (int)(binom_small(a, 1) + binom_small(b + 1, 2));
}

static __device__ __forceinline__ int rank3(int a, int b, int c) {
    sort2(a, b); sort2(b, c); sort2(a, b);
    return (int)(binom_small(a, 1) + binom_small(b + 1, 2) + binom_small(c + 2, 3));
}

static __device__ __forceinline__ int rank4(int a, int b, int c, int d) {
    sort2(a, b); sort2(c, d); sort2(a, c); sort2(b, d); sort2(b, c);
    return (int)(binom_small(a, 1) + binom_small(b + 1, 2) + binom_small(c + 2, 3) +
                 binom_small(d + 3, 4));
}

// Super-hub bitmap probes: bit of node x in the bitmap of super-hub index s,
// and the slot of x inside the super-hub's (sorted) row.
static __device__ __forceinline__ bool sh_bit(const uint64_t *SB, int64_t nw, int s, int32_t x) {
    return (SB[(size_t)s * nw + (x >> 6)] >> (x & 63)) & 1ull;
}

static __device__ __forceinline__ int64_t sh_slot(const uint64_t *SB, const uint32_t *SP, int64_t nw,
                                                  int64_t row_begin, int s, int32_t x) {
    size_t o = (size_t)s * nw + (x >> 6);
    uint64_t below = (x & 63) ? (SB[o] & ((1ull << (x & 63)) - 1)) : 0ull;
    return row_begin + SP[o] + (uint32_t)__popcll(below);
}

}  // namespace tg
