// Prefix sums and radix sorts of the preparation step (hand-written, so
// that a call records no memory-set nodes and needs no library temporary
// buffers when it is captured into a HIP graph).
//
// Exclusive scan of int64 values: per-tile sums, one workgroup scanning the
// tile sums, then each tile rescanning its values from its offset.
// LSD radix sort of 64-bit keys (with optional 32-bit values): per 8-bit
// digit, per-tile digit histograms laid out digit-major, an exclusive scan
// of that table (each digit's tiles in order, so the sort is stable), and a
// scatter in which every key's rank among the equal digits of its tile
// comes from wave ballots.
#include <hip/hip_runtime.h>

#include "tg_device.hpp"

namespace tg {

constexpr int SCAN_THREADS = 256;
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = SCAN_THREADS * SCAN_ITEMS;

// Block-wide exclusive scan of one int64 per thread; *total gets the sum.
__device__ __forceinline__ int64_t block_excl_scan(int64_t v, int64_t *wsum, int64_t *total) {
    const int lane = lane_id(), w = threadIdx.x / WAVE;
    int64_t x = v;
#pragma unroll
    for (int d = 1; d < WAVE; d <<= 1) {
        int64_t o = (int64_t)__shfl_up((unsigned long long)x, d, WAVE);
        if (lane >= d) x += o;
    }
    if (lane == WAVE - 1) wsum[w] = x;
    __syncthreads();
    int64_t before = 0, all = 0;
    for (int q = 0; q < SCAN_THREADS / WAVE; ++q) {
        if (q < w) before += wsum[q];
        all += wsum[q];
    }
    __syncthreads();
    *total = all;
    return before + x - v;
}

__global__ void __launch_bounds__(SCAN_THREADS)
k_scan_tiles(const int64_t *__restrict__ in, int64_t count, int64_t *__restrict__ tile_sum,
             const uint32_t *__restrict__ gate) {
    if (gate && input_failed(gate)) return;
    __shared__ int64_t wsum[SCAN_THREADS / WAVE];
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
    int64_t s = 0;
#pragma unroll
    for (int q = 0; q < SCAN_ITEMS; ++q)
        if (base + q < count) s += in[base + q];
    int64_t total;
    block_excl_scan(s, wsum, &total);
    if (threadIdx.x == 0) tile_sum[blockIdx.x] = total;
}

// One workgroup: exclusive scan of the tile sums in place.
__global__ void __launch_bounds__(SCAN_THREADS)
k_scan_sums(int64_t *__restrict__ sums, int64_t tiles, const uint32_t *__restrict__ gate) {
    if (gate && input_failed(gate)) return;
    __shared__ int64_t wsum[SCAN_THREADS / WAVE];
    int64_t carry = 0;
    for (int64_t b = 0; b < tiles; b += SCAN_THREADS) {
        const int64_t q = b + threadIdx.x;
        const int64_t v = q < tiles ? sums[q] : 0;
        int64_t total;
        const int64_t ex = block_excl_scan(v, wsum, &total);
        if (q < tiles) sums[q] = carry + ex;
        carry += total;
    }
}

__global__ void __launch_bounds__(SCAN_THREADS)
k_scan_apply(const int64_t *__restrict__ in, int64_t count, const int64_t *__restrict__ tile_off,
             int64_t *__restrict__ out, const uint32_t *__restrict__ gate) {
    if (gate && input_failed(gate)) return;
    __shared__ int64_t wsum[SCAN_THREADS / WAVE];
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
    int64_t v[SCAN_ITEMS];
    int64_t s = 0;
#pragma unroll
    for (int q = 0; q < SCAN_ITEMS; ++q) {
        v[q] = base + q < count ? in[base + q] : 0;
        s += v[q];
    }
    int64_t total;
    int64_t run = tile_off[blockIdx.x] + block_excl_scan(s, wsum, &total);
#pragma unroll
    for (int q = 0; q < SCAN_ITEMS; ++q)
        if (base + q < count) {
            out[base + q] = run;
            run += v[q];
        }
}

int64_t scan_tiles(int64_t count) { return (count + SCAN_TILE - 1) / SCAN_TILE; }

hipError_t launch_excl_scan(const int64_t *in, int64_t *out, int64_t count, int64_t *tmp,
                            const uint32_t *gate, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    const int64_t tiles = scan_tiles(count);
    k_scan_tiles<<<(unsigned)tiles, SCAN_THREADS, 0, st>>>(in, count, tmp, gate);
    k_scan_sums<<<1, SCAN_THREADS, 0, st>>>(tmp, tiles, gate);
    k_scan_apply<<<(unsigned)tiles, SCAN_THREADS, 0, st>>>(in, count, tmp, out, gate);
    return hipGetLastError();
}

// ----------------------------------------------------------- radix sort

constexpr int RS_THREADS = 256;
constexpr int RS_ROUNDS = 16;                       // keys per thread per tile
constexpr int RS_TILE = RS_THREADS * RS_ROUNDS;     // keys per tile
constexpr int RS_BINS = 256;

int64_t radix_tiles(int64_t count) { return (count + RS_TILE - 1) / RS_TILE; }

// Digit histogram of one tile, written to hist[digit * tiles + tile].
__global__ void __launch_bounds__(RS_THREADS)
k_rs_hist(const uint64_t *__restrict__ keys, int64_t count, int shift, int64_t tiles,
          int64_t *__restrict__ hist, const uint32_t *__restrict__ gate) {
    if (gate && input_failed(gate)) return;
    __shared__ uint32_t h[RS_BINS];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * RS_TILE;
    for (int r = 0; r < RS_ROUNDS; ++r) {
        const int64_t q = base + (int64_t)r * RS_THREADS + threadIdx.x;
        if (q < count) atomicAdd(&h[(keys[q] >> shift) & (RS_BINS - 1)], 1u);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * tiles + blockIdx.x] = h[threadIdx.x];
}

// Scatter of one tile: keys are taken in tile order (round by round, thread
// by thread); a key's place is its digit's offset for this tile plus the
// number of equal digits before it in the tile.
__global__ void __launch_bounds__(RS_THREADS)
k_rs_scatter(const uint64_t *__restrict__ keys, const uint32_t *__restrict__ vals, int64_t count,
             int shift, int64_t tiles, const int64_t *__restrict__ off,
             uint64_t *__restrict__ keys_out, uint32_t *__restrict__ vals_out,
             const uint32_t *__restrict__ gate) {
    if (gate && input_failed(gate)) return;
    constexpr int NW = RS_THREADS / WAVE;
    __shared__ int64_t base_of[RS_BINS];
    __shared__ uint32_t wave_cnt[NW][RS_BINS];
    const int tid = threadIdx.x, lane = lane_id(), w = tid / WAVE;
    base_of[tid] = off[(int64_t)tid * tiles + blockIdx.x];
    for (int q = 0; q < NW; ++q) wave_cnt[q][tid] = 0;
    __syncthreads();
    const int64_t tile0 = (int64_t)blockIdx.x * RS_TILE;
    const uint64_t below = (1ull << lane) - 1ull;
    for (int r = 0; r < RS_ROUNDS; ++r) {
        const int64_t q = tile0 + (int64_t)r * RS_THREADS + tid;
        const bool valid = q < count;
        const uint64_t k = valid ? keys[q] : 0ull;
        const uint32_t v = valid && vals ? vals[q] : 0u;
        const int dig = (int)((k >> shift) & (RS_BINS - 1));
        // lanes of this wave holding the same digit
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int bit = 0; bit < 8; ++bit) {
            const uint64_t b = __ballot((dig >> bit) & 1);
            peers &= ((dig >> bit) & 1) ? b : ~b;
        }
        const uint32_t rank = (uint32_t)__popcll(peers & below);
        if (valid && rank == 0) wave_cnt[w][dig] = (uint32_t)__popcll(peers);
        __syncthreads();
        if (valid) {
            int64_t pos = base_of[dig] + rank;
            for (int x = 0; x < w; ++x) pos += wave_cnt[x][dig];
            keys_out[pos] = k;
            if (vals) vals_out[pos] = v;
        }
        __syncthreads();
        // advance each digit's base past this round, clear the wave counts
        uint32_t add = 0;
        for (int x = 0; x < NW; ++x) {
            add += wave_cnt[x][tid];
            wave_cnt[x][tid] = 0;
        }
        base_of[tid] += add;
        __syncthreads();
    }
}

// Bytes of temporary storage radix_sort and launch_excl_scan need for
// `count` elements (digit table and its tile sums, or the scan's tile sums).
size_t sort_tmp_need(int64_t count) {
    const int64_t tiles = radix_tiles(count > 0 ? count : 1);
    const int64_t table = tiles * RS_BINS;
    return (size_t)(table + scan_tiles(table) + scan_tiles(count + 1) + 64) * sizeof(int64_t);
}

// Sorts keys[0..count) (and vals alongside when given) by bits [0, end_bit),
// ping-ponging with keys_tmp / vals_tmp; *out_keys / *out_vals receive the
// buffers that hold the result.  tmp: sort_tmp_need(count) bytes.
hipError_t radix_sort(uint64_t *keys, uint64_t *keys_tmp, uint32_t *vals, uint32_t *vals_tmp,
                      int64_t count, int end_bit, void *tmp, const uint32_t *gate,
                      hipStream_t st, uint64_t **out_keys, uint32_t **out_vals) {
    uint64_t *ka = keys, *kb = keys_tmp;
    uint32_t *va = vals, *vb = vals_tmp;
    *out_keys = ka;
    *out_vals = va;
    if (count <= 1) return hipSuccess;
    const int64_t tiles = radix_tiles(count);
    int64_t *table = reinterpret_cast<int64_t *>(tmp);
    int64_t *sums = table + tiles * RS_BINS;
    for (int shift = 0; shift < end_bit; shift += 8) {
        k_rs_hist<<<(unsigned)tiles, RS_THREADS, 0, st>>>(ka, count, shift, tiles, table, gate);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        e = launch_excl_scan(table, table, tiles * RS_BINS, sums, gate, st);
        if (e != hipSuccess) return e;
        k_rs_scatter<<<(unsigned)tiles, RS_THREADS, 0, st>>>(ka, va, count, shift, tiles, table,
                                                            kb, vb, gate);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        uint64_t *tk = ka; ka = kb; kb = tk;
        uint32_t *tv = va; va = vb; vb = tv;
    }
    *out_keys = ka;
    *out_vals = va;
    return hipSuccess;
}

}  // namespace tg
