// Directed typed graphlets (Sec. 4.8): every typed neighbourhood of the
// underlying undirected graph splits by arc direction -- out (the endpoint
// -> k), in (k -> the endpoint) or both (reciprocal arcs) -- and with it the
// sets T_ij, S_i, S_j of Alg. 1.  Per edge (i, j), i < j, the row holds
//   TRI[t][a][b]  at t*9 + a*3 + b   (k in T_ij, type t, direction a at i,
//                                     direction b at j)
//   PATH_I[t][a]  at 9L + t*3 + a    (k in S_i)
//   PATH_J[t][b]  at 12L + t*3 + b   (k in S_j)
// with a, b in {0 out, 1 in, 2 both}.  As in Cor. 2, the 3-path counts come
// from the direction-split typed degrees minus the triangles and the edge
// itself: only the common neighbours are enumerated (one wave per edge,
// each element of the shorter list searched in the longer one).
//
// Global counts are per directed typed graphlet (class of typed digraphs
// under type-preserving isomorphism), named by a canonical key: the
// smallest (types..., pair codes...) over every numbering of the nodes,
// a pair code for nodes x < y being 0 none, 1 x -> y, 2 y -> x, 3 both.
// A row's columns name their classes only through the edge's own class
// (its endpoint types and direction), so the edges are sorted by that
// class, the rows summed per class and column in registers, and only the
// 3L^2 x 15L sums mapped to canonical keys; each 3-node class is then
// divided by its edge count (a triangle is met from its 3 edges, a 3-path
// from its 2).
#include <hip/hip_runtime.h>

#include <vector>

#include "tg_device.hpp"

namespace tg {
namespace {


// Direction code of a CSR slot relative to its row's node: 0 out, 1 in, 2 both.
__device__ __forceinline__ int dir_code(uint8_t d) { return d == 1 ? 0 : d == 2 ? 1 : 2; }

// Checks (sorted rows in range, no self-loops, types in range, direction
// bits 1..3 mirrored by the reverse slot), entries above the diagonal per
// row, and the direction-split typed degrees deg3[v][t*3 + a].  One wave
// per row.
__global__ void __launch_bounds__(256)
k_dir_check(const int64_t *__restrict__ rp, const int32_t *__restrict__ col,
            const uint8_t *__restrict__ dir, const uint8_t *__restrict__ types, int64_t n,
            int64_t nnz, int L, int64_t *__restrict__ ucount, uint32_t *__restrict__ deg3,
            uint32_t *__restrict__ status) {
    __shared__ uint32_t cnt[256 / WAVE][3 * TG_MAX_L];
    const int lane = lane_id(), wv = threadIdx.x / WAVE;
    if (blockIdx.x == 0 && threadIdx.x == 0) ucount[n] = 0;
    const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x / WAVE);
    for (int64_t u = (int64_t)blockIdx.x * (blockDim.x / WAVE) + wv; u < n; u += nwaves) {
        for (int q = lane; q < 3 * L; q += WAVE) cnt[wv][q] = 0;
        wave_sync();
        const int64_t b = rp[u], e = rp[u + 1];
        uint32_t bad = 0;
        uint64_t up = 0;
        if (b < 0 || e < b || e > nnz || (u == 0 && b != 0) || (u == n - 1 && e != nnz)) {
            bad = ST_UNSORTED;
        } else {
            if (types[u] >= L) bad |= ST_TYPE_RANGE;
            for (int64_t s = b + lane; s < e; s += WAVE) {
                const int32_t x = col[s];
                if (x < 0 || x >= n) {
                    bad |= ST_COL_RANGE;
                    continue;
                }
                if (x == u) bad |= ST_SELF_LOOP;
                if (s > b && col[s - 1] >= x) bad |= ST_UNSORTED;
                if (x > u) ++up;
                const uint8_t d = dir[s];
                const int64_t xb = rp[x], xe = rp[x + 1];
                if (d == 0 || d > 3 || xb < 0 || xe < xb || xe > nnz) {
                    bad |= ST_ASYMMETRIC;
                    continue;
                }
                const int64_t r = lower_bound(col, xb, xe, (int32_t)u);
                const uint8_t want = (uint8_t)(((d & 1) << 1) | (d >> 1));
                if (r >= xe || col[r] != (int32_t)u || dir[r] != want) bad |= ST_ASYMMETRIC;
                const int t = types[x];
                if (t < L) atomicAdd(&cnt[wv][t * 3 + dir_code(d)], 1u);
                else bad |= ST_TYPE_RANGE;
            }
        }
        bad = wave_or(bad);
        up = wave_sum_u64(up);
        wave_sync();
        if (lane == 0) {
            ucount[u] = bad ? 0 : (int64_t)up;
            if (bad) atomicOr(status, bad);
        }
        for (int q = lane; q < 3 * L; q += WAVE) deg3[(size_t)u * 3 * L + q] = cnt[wv][q];
        wave_sync();
    }
}

__global__ void k_dir_edge_check(const int64_t *__restrict__ eoff, int64_t n, int64_t m,
                                 uint32_t *__restrict__ status) {
    if (eoff[n] != m) atomicOr(status, ST_EDGE_COUNT);
}

// The canonical edge of each upper slot: esrc[e] = u, eslot[e] = s.
__global__ void k_dir_edges_of(const int64_t *__restrict__ rp, const int32_t *__restrict__ col,
                               const int64_t *__restrict__ eoff, int64_t n,
                               int32_t *__restrict__ esrc, int64_t *__restrict__ eslot) {
    const int lane = lane_id();
    const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x / WAVE);
    for (int64_t u = (int64_t)blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE; u < n;
         u += nwaves) {
        const int64_t e = rp[u + 1], first = e - (eoff[u + 1] - eoff[u]);
        for (int64_t s = first + lane; s < e; s += WAVE) {
            const int64_t id = eoff[u] + (s - first);
            esrc[id] = (int32_t)u;
            eslot[id] = s;
        }
    }
}

// Hubs: nodes of degree >= DIR_HUB_DEG get a bitmap of their neighbours
// (n bits) and the popcount of every bitmap word before it, so that a probe
// into a hub's row is a bitmap word, a prefix count and the direction byte
// of the slot they give (at most DIR_HUB_MAX hubs; others are searched).
constexpr int64_t DIR_HUB_DEG = 256;
constexpr int64_t DIR_HUB_MAX = 8192;

__global__ void k_dir_hub_ids(const int64_t *__restrict__ rp, int64_t n, int64_t hub_max,
                              int32_t *__restrict__ hub_id, int32_t *__restrict__ hub_node,
                              unsigned int *__restrict__ counter) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    int32_t h = -1;
    if (rp[v + 1] - rp[v] >= DIR_HUB_DEG) {
        const unsigned int q = atomicAdd(counter, 1u);
        if ((int64_t)q < hub_max) {
            h = (int32_t)q;
            hub_node[q] = (int32_t)v;
        }
    }
    hub_id[v] = h;
}

// One workgroup per hub: its bitmap, then the exclusive prefix popcounts of
// the bitmap's words.
__global__ void __launch_bounds__(256)
k_dir_hub_bits(const int64_t *__restrict__ rp, const int32_t *__restrict__ col,
               const int32_t *__restrict__ hub_node, const unsigned int *__restrict__ counter,
               int64_t hub_max, int64_t nw, unsigned long long *__restrict__ bits,
               uint32_t *__restrict__ prefix) {
    const int64_t h = blockIdx.x;
    const int64_t cnt = *counter < (unsigned int)hub_max ? (int64_t)*counter : hub_max;
    if (h >= cnt) return;
    const int32_t v = hub_node[h];
    unsigned long long *B = bits + (size_t)h * nw;
    uint32_t *Pf = prefix + (size_t)h * nw;
    const int tid = threadIdx.x;
    for (int64_t q = tid; q < nw; q += 256) B[q] = 0ull;
    __syncthreads();
    for (int64_t s = rp[v] + tid; s < rp[v + 1]; s += 256) {
        const int32_t x = col[s];
        atomicOr(&B[x >> 6], 1ull << (x & 63));
    }
    __syncthreads();
    // prefix popcounts, 256 words at a time (one per thread, coalesced):
    // a scan inside each wave, then over the four wave totals
    __shared__ uint32_t wtot[256 / WAVE];
    const int lane = lane_id(), wv = tid / WAVE;
    uint32_t run = 0;
    for (int64_t base = 0; base < nw; base += 256) {
        const int64_t q = base + tid;
        // the words were set by other threads' atomics: read them from L2
        const uint32_t c =
            q < nw ? (uint32_t)__popcll(__hip_atomic_load(&B[q], __ATOMIC_RELAXED,
                                                          __HIP_MEMORY_SCOPE_AGENT))
                   : 0u;
        const uint32_t incl = wave_incl_scan(c);
        if (lane == WAVE - 1) wtot[wv] = incl;
        __syncthreads();
        uint32_t before = run;
        for (int x = 0; x < wv; ++x) before += wtot[x];
        if (q < nw) Pf[q] = before + incl - c;
        uint32_t all = 0;
        for (int x = 0; x < 256 / WAVE; ++x) all += wtot[x];
        run += all;
        __syncthreads();
    }
}

constexpr int DIR_SAMPLE = 1024;   // LDS sample of a long list (entries per wave)

// One wave per edge (i, j): the common neighbours k by searching each
// element of the shorter list in the longer one, counted per (type of k,
// direction at i, direction at j) in LDS; then the row.  When the shorter
// list fills at least half a wave and the longer one is long, every
// stride-th entry of the longer list is copied to LDS first (at most
// DIR_SAMPLE entries): a probe searches the sample in LDS and then only the
// stride entries between two samples in global memory.
__global__ void __launch_bounds__(256)
k_dir_rows(const int64_t *__restrict__ rp, const int32_t *__restrict__ col,
           const uint8_t *__restrict__ dir, const uint8_t *__restrict__ types,
           const uint32_t *__restrict__ deg3, const int32_t *__restrict__ esrc,
           const int64_t *__restrict__ eslot, int64_t m, int L,
           const int32_t *__restrict__ hub_id, const unsigned long long *__restrict__ hbits,
           const uint32_t *__restrict__ hprefix, int64_t nw, uint64_t *__restrict__ rows) {
    __shared__ uint32_t tri[256 / WAVE][9 * TG_MAX_L];
    __shared__ int32_t samp[256 / WAVE][DIR_SAMPLE];
    const int lane = lane_id(), wv = threadIdx.x / WAVE;
    const int W = 15 * L;
    const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x / WAVE);
    for (int64_t e = (int64_t)blockIdx.x * (blockDim.x / WAVE) + wv; e < m; e += nwaves) {
        const int32_t i = esrc[e];
        const int64_t sij = eslot[e];
        const int32_t j = col[sij];
        for (int q = lane; q < 9 * L; q += WAVE) tri[wv][q] = 0;
        wave_sync();
        const int64_t ib = rp[i], ie = rp[i + 1], jb = rp[j], je = rp[j + 1];
        const bool i_short = ie - ib <= je - jb;
        const int64_t sb = i_short ? ib : jb, se = i_short ? ie : je;
        const int64_t lb = i_short ? jb : ib, le = i_short ? je : ie;
        const int32_t hl = hub_id[i_short ? j : i];     // the longer row's hub index
        int64_t stride = 0;
        int nsamp = 0;
        if (hl >= 0) {
            const unsigned long long *B = hbits + (size_t)hl * nw;
            const uint32_t *Pf = hprefix + (size_t)hl * nw;
            for (int64_t s = sb + lane; s < se; s += WAVE) {
                const int32_t k = col[s];
                const unsigned long long word = B[k >> 6];
                if (!((word >> (k & 63)) & 1ull)) continue;
                const int64_t r = lb + Pf[k >> 6] +
                                  __popcll(word & ((1ull << (k & 63)) - 1ull));
                const int cs = dir_code(dir[s]), cl = dir_code(dir[r]);
                const int a = i_short ? cs : cl, b = i_short ? cl : cs;
                atomicAdd(&tri[wv][types[k] * 9 + a * 3 + b], 1u);
            }
        } else if (se - sb >= WAVE / 2 && le - lb > 2 * WAVE) {
            stride = (le - lb + DIR_SAMPLE - 1) / DIR_SAMPLE;
            nsamp = (int)((le - lb + stride - 1) / stride);
            for (int q = lane; q < nsamp; q += WAVE) samp[wv][q] = col[lb + (int64_t)q * stride];
            wave_sync();
        }
        for (int64_t s = sb + lane; hl < 0 && s < se; s += WAVE) {
            const int32_t k = col[s];
            int64_t lo = lb, hi = le;
            if (stride) {
                int a = 0, b = nsamp;             // first sample above k
                while (a < b) {
                    const int mid = (a + b) >> 1;
                    if (samp[wv][mid] <= k) a = mid + 1; else b = mid;
                }
                if (a == 0) continue;             // k below the whole list
                lo = lb + (int64_t)(a - 1) * stride;
                hi = lo + stride < le ? lo + stride : le;
            }
            const int64_t r = lower_bound(col, lo, hi, k);
            if (r < hi && col[r] == k) {
                const int cs = dir_code(dir[s]), cl = dir_code(dir[r]);
                const int a = i_short ? cs : cl, b = i_short ? cl : cs;
                atomicAdd(&tri[wv][types[k] * 9 + a * 3 + b], 1u);
            }
        }
        wave_sync();
        const int ti = types[i], tj = types[j];
        const int aij = dir_code(dir[sij]);                 // j as seen from i
        const int bji = dir_code((uint8_t)(((dir[sij] & 1) << 1) | (dir[sij] >> 1)));
        uint64_t *row = rows + (size_t)e * W;
        for (int q = lane; q < W; q += WAVE) {
            uint64_t v;
            if (q < 9 * L) {
                v = tri[wv][q];
            } else if (q < 12 * L) {
                const int t = (q - 9 * L) / 3, a = (q - 9 * L) % 3;
                int64_t c = deg3[(size_t)i * 3 * L + t * 3 + a];
                for (int b = 0; b < 3; ++b) c -= tri[wv][t * 9 + a * 3 + b];
                if (t == tj && a == aij) --c;
                v = (uint64_t)c;
            } else {
                const int t = (q - 12 * L) / 3, b = (q - 12 * L) % 3;
                int64_t c = deg3[(size_t)j * 3 * L + t * 3 + b];
                for (int a = 0; a < 3; ++a) c -= tri[wv][t * 9 + a * 3 + b];
                if (t == ti && b == bji) --c;
                v = (uint64_t)c;
            }
            row[q] = v;
        }
        wave_sync();
    }
}

// Canonical key index of a typed digraph on 2 or 3 nodes.  arcs: bit x*3+y
// is the arc x -> y.
__device__ __forceinline__ int pair_code(uint32_t arcs, int x, int y) {
    return (int)((arcs >> (x * 3 + y)) & 1u) | (int)(((arcs >> (y * 3 + x)) & 1u) << 1);
}

__device__ int64_t canon_key3(int t0, int t1, int t2, uint32_t arcs, int L) {
    const int ty[3] = {t0, t1, t2};
    const int perms[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    int64_t best = -1;
    for (int q = 0; q < 6; ++q) {
        const int p0 = perms[q][0], p1 = perms[q][1], p2 = perms[q][2];
        const int64_t key = (((int64_t)ty[p0] * L + ty[p1]) * L + ty[p2]) * 64 +
                            pair_code(arcs, p0, p1) * 16 + pair_code(arcs, p0, p2) * 4 +
                            pair_code(arcs, p1, p2);
        if (best < 0 || key < best) best = key;
    }
    return 4 * (int64_t)L * L + best;
}

__device__ __forceinline__ int64_t canon_key2(int t0, int t1, uint32_t arcs, int L) {
    const int64_t a = ((int64_t)t0 * L + t1) * 4 + pair_code(arcs, 0, 1);
    const int64_t b = ((int64_t)t1 * L + t0) * 4 + pair_code(arcs, 1, 0);
    return a < b ? a : b;
}

// Arcs between endpoint x (0 = i or 1 = j) and node 2 for direction code c.
__device__ __forceinline__ uint32_t end_arcs(int x, int c) {
    const uint32_t out = 1u << (x * 3 + 2), in = 1u << (2 * 3 + x);
    return c == 0 ? out : c == 1 ? in : (out | in);
}

// Edge class of every edge: (type of i, type of j, direction bits of the
// edge) as (ti * L + tj) * 3 + bits - 1; sorted by it, the edges of one class
// are contiguous.
__global__ void k_dir_class(const int32_t *__restrict__ col, const uint8_t *__restrict__ dir,
                            const uint8_t *__restrict__ types, const int32_t *__restrict__ esrc,
                            const int64_t *__restrict__ eslot, int64_t m, int L,
                            uint64_t *__restrict__ key, uint32_t *__restrict__ val) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= m) return;
    const int64_t s = eslot[e];
    key[e] = ((uint64_t)types[esrc[e]] * L + types[col[s]]) * 3 + (dir[s] - 1);
    val[e] = (uint32_t)e;
}

// Column sums of the rows per edge class: each wave walks a contiguous run
// of the class-sorted edges, lanes owning columns, summing in registers and
// adding to csum[class][column] whenever the class changes.
__global__ void __launch_bounds__(256)
k_dir_class_sums(const uint64_t *__restrict__ skey, const uint32_t *__restrict__ sval,
                 const uint64_t *__restrict__ rows, int64_t m, int L, int64_t per_wave,
                 unsigned long long *__restrict__ csum) {
    constexpr int CPL = (15 * TG_MAX_L + WAVE - 1) / WAVE;
    const int lane = lane_id();
    const int W = 15 * L;
    const int64_t wid = (int64_t)blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE;
    const int64_t e0 = wid * per_wave;
    const int64_t e1 = e0 + per_wave < m ? e0 + per_wave : m;
    if (e0 >= e1) return;
    uint64_t acc[CPL];
#pragma unroll
    for (int c = 0; c < CPL; ++c) acc[c] = 0;
    uint64_t cls = skey[e0];
    for (int64_t e = e0; e < e1; ++e) {
        const uint64_t k = skey[e];
        if (k != cls) {
#pragma unroll
            for (int c = 0; c < CPL; ++c) {
                const int q = lane + c * WAVE;
                if (q < W && acc[c]) atomicAdd(&csum[cls * W + q], (unsigned long long)acc[c]);
                acc[c] = 0;
            }
            cls = k;
        }
        const uint64_t *row = rows + (size_t)sval[e] * W;
#pragma unroll
        for (int c = 0; c < CPL; ++c) {
            const int q = lane + c * WAVE;
            if (q < W) acc[c] += row[q];
        }
    }
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
        const int q = lane + c * WAVE;
        if (q < W && acc[c]) atomicAdd(&csum[cls * W + q], (unsigned long long)acc[c]);
    }
}

// Class sums -> canonical keys: one thread per (edge class, column); the
// edge itself is counted once per edge of the class (its 2-node key).
__global__ void k_dir_keys(const unsigned long long *__restrict__ csum,
                           const unsigned long long *__restrict__ ccount, int L,
                           unsigned long long *__restrict__ acc) {
    const int W = 15 * L;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t classes = 3 * (int64_t)L * L;
    if (t >= classes * (W + 1)) return;
    const int64_t cls = t / (W + 1);
    const int q = (int)(t % (W + 1)) - 1;          // -1: the edge's own class
    const int d = (int)(cls % 3) + 1;
    const int ti = (int)(cls / 3 / L), tj = (int)(cls / 3 % L);
    const uint32_t eij = ((d & 1) ? 1u << 1 : 0u) | ((d & 2) ? 1u << 3 : 0u);   // 0->1, 1->0
    if (q < 0) {
        const unsigned long long v = ccount[cls];
        if (v) atomicAdd(&acc[canon_key2(ti, tj, eij, L)], v);
        return;
    }
    const unsigned long long v = csum[cls * W + q];
    if (!v) return;
    int tt;
    uint32_t arcs = eij;
    if (q < 9 * L) {
        tt = q / 9;
        arcs |= end_arcs(0, (q / 3) % 3) | end_arcs(1, q % 3);
    } else if (q < 12 * L) {
        tt = (q - 9 * L) / 3;
        arcs |= end_arcs(0, (q - 9 * L) % 3);
    } else {
        tt = (q - 12 * L) / 3;
        arcs |= end_arcs(1, (q - 12 * L) % 3);
    }
    atomicAdd(&acc[canon_key3(ti, tj, tt, arcs, L)], v);
}

// Number of edges per class (the run lengths of the sorted keys).
__global__ void k_dir_class_count(const uint64_t *__restrict__ skey, int64_t m,
                                  unsigned long long *__restrict__ ccount) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= m) return;
    if (e == m - 1 || skey[e] != skey[e + 1]) {
        // e ends a run: its length is e + 1 minus the start (found by search)
        int64_t lo = 0, hi = e;
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if (skey[mid] < skey[e]) lo = mid + 1; else hi = mid;
        }
        ccount[skey[e]] = (unsigned long long)(e + 1 - lo);
    }
}

// Each 3-node class divided by its edge count (3 for a triangle, 2 for a
// 3-path); a remainder flags ST_NOT_DIVISIBLE.
__global__ void k_dir_finalize(const unsigned long long *__restrict__ acc, int64_t width, int L,
                               uint64_t *__restrict__ out, uint32_t *__restrict__ status) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= width) return;
    uint64_t v = acc[q];
    const int64_t base = 4 * (int64_t)L * L;
    if (q >= base && v) {
        const int c = (int)((q - base) % 64);
        const int edges = (c >> 4 ? 1 : 0) + ((c >> 2) & 3 ? 1 : 0) + (c & 3 ? 1 : 0);
        if (edges < 2 || v % (uint64_t)edges) atomicOr(status, ST_NOT_DIVISIBLE);
        v = edges ? v / (uint64_t)edges : v;
    }
    out[q] = v;
}

struct DirLayout {
    size_t status, ucount, eoff, stmp, deg3, esrc, eslot, rows, acc, ckey, ckey_tmp, cval, cval_tmp,
        sort_tmp, csum, ccount, hub_id, hub_node, hbits, hprefix, total;
    int64_t hub_max, nw;
};

DirLayout dir_layout(int64_t n, int64_t nnz, int L, bool own_rows) {
    DirLayout y{};
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o = (o + bytes + 255) & ~(size_t)255;
        return at;
    };
    const int64_t m = nnz / 2;
    y.status = take(256);
    y.ucount = take(sizeof(int64_t) * (size_t)(n + 1));
    y.eoff = take(sizeof(int64_t) * (size_t)(n + 1));
    y.stmp = take(sizeof(int64_t) * (size_t)(scan_tiles(n + 1) + 1));
    y.deg3 = take(sizeof(uint32_t) * (size_t)(n > 0 ? n : 1) * 3 * L);
    y.esrc = take(sizeof(int32_t) * (size_t)(m > 0 ? m : 1));
    y.eslot = take(sizeof(int64_t) * (size_t)(m > 0 ? m : 1));
    y.rows = take(own_rows ? sizeof(uint64_t) * (size_t)(m > 0 ? m : 1) * 15 * L : 0);
    y.acc = take(sizeof(uint64_t) * (size_t)(4 * L * L + 64 * L * L * L));
    const size_t m1 = (size_t)(m > 0 ? m : 1);
    y.ckey = take(sizeof(uint64_t) * m1);
    y.ckey_tmp = take(sizeof(uint64_t) * m1);
    y.cval = take(sizeof(uint32_t) * m1);
    y.cval_tmp = take(sizeof(uint32_t) * m1);
    y.sort_tmp = take(sort_tmp_need(m > 0 ? m : 1));
    y.csum = take(sizeof(uint64_t) * (size_t)(3 * L * L) * 15 * L);
    y.ccount = take(sizeof(uint64_t) * (size_t)(3 * L * L));
    // at most nnz / DIR_HUB_DEG nodes reach the hub degree
    y.hub_max = nnz / DIR_HUB_DEG < DIR_HUB_MAX ? nnz / DIR_HUB_DEG : DIR_HUB_MAX;
    y.nw = (n + 63) / 64 > 0 ? (n + 63) / 64 : 1;
    y.hub_id = take(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    y.hub_node = take(sizeof(int32_t) * (size_t)(y.hub_max > 0 ? y.hub_max : 1));
    y.hbits = take(sizeof(uint64_t) * (size_t)y.hub_max * y.nw);
    y.hprefix = take(sizeof(uint32_t) * (size_t)y.hub_max * y.nw);
    y.total = o;
    return y;
}

unsigned waves_grid(int64_t items) {
    int64_t b = (items + 3) / 4;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
        cus > 0 && b > (int64_t)cus * 32)
        b = (int64_t)cus * 32;
    return b > 0 ? (unsigned)b : 1u;
}

}  // namespace
}  // namespace tg

using namespace tg;

extern "C" {

int32_t tg_directed_row_width(int32_t L) { return (L < 1 || L > TG_MAX_L) ? 0 : 15 * L; }

int64_t tg_directed_global_width(int32_t L) {
    return (L < 1 || L > TG_MAX_L) ? 0 : 4 * (int64_t)L * L + 64 * (int64_t)L * L * L;
}

size_t tg_directed_workspace_bytes(int64_t n, int64_t nnz, int32_t L) {
    if (n < 0 || nnz < 0 || L < 1 || L > TG_MAX_L) return 0;
    return dir_layout(n, nnz, L, true).total;
}

tg_status tg_count_directed(const int64_t *row_ptr, const int32_t *col, const uint8_t *dir,
                            const uint8_t *types, int64_t n, int64_t nnz, int32_t L,
                            uint64_t *per_edge, uint64_t *global_counts, void *workspace,
                            size_t ws_bytes, void *stream) {
    if (L < 1 || L > TG_MAX_L) return TG_E_L_RANGE;
    if (n < 0 || nnz < 0 || (nnz & 1) || !row_ptr || (n > 0 && !types) ||
        (nnz > 0 && (!col || !dir)) || !workspace || ((uintptr_t)workspace & 255u))
        return TG_E_INVALID_ARG;
    if (n >= (int64_t(1) << 31) || nnz >= (int64_t(1) << 33)) return TG_E_TOO_LARGE;
    const DirLayout y = dir_layout(n, nnz, L, per_edge == nullptr);
    if (ws_bytes < y.total) return TG_E_WORKSPACE;
    hipStream_t st = (hipStream_t)stream;
    char *w = static_cast<char *>(workspace);
    uint32_t *status = reinterpret_cast<uint32_t *>(w + y.status);
    int64_t *ucount = reinterpret_cast<int64_t *>(w + y.ucount);
    int64_t *eoff = reinterpret_cast<int64_t *>(w + y.eoff);
    uint32_t *deg3 = reinterpret_cast<uint32_t *>(w + y.deg3);
    int32_t *esrc = reinterpret_cast<int32_t *>(w + y.esrc);
    int64_t *eslot = reinterpret_cast<int64_t *>(w + y.eslot);
    uint64_t *rows = per_edge ? per_edge : reinterpret_cast<uint64_t *>(w + y.rows);
    unsigned long long *acc = reinterpret_cast<unsigned long long *>(w + y.acc);
    const int64_t m = nnz / 2, width = tg_directed_global_width(L);
#define DIR_CHK(x) do { if ((x) != hipSuccess) return TG_E_DEVICE; } while (0)
    ksum_reset();
    DIR_CHK(launch_fill_u64(reinterpret_cast<uint64_t *>(status), 0, 1, st));
    DIR_CHK(launch_fill_u64(reinterpret_cast<uint64_t *>(acc), 0, width, st));
    if (n > 0) {
        ksum_begin(st);
        k_dir_check<<<waves_grid(n), 256, 0, st>>>(row_ptr, col, dir, types, n, nnz, L, ucount,
                                                    deg3, status);
        ksum_end("dir_check", 0.0, st);
        DIR_CHK(hipGetLastError());
        DIR_CHK(launch_excl_scan(ucount, eoff, n + 1, reinterpret_cast<int64_t *>(w + y.stmp),
                                 nullptr, st));
        k_dir_edge_check<<<1, 1, 0, st>>>(eoff, n, m, status);
        DIR_CHK(hipGetLastError());
    } else if (nnz > 0) {
        return TG_E_INVALID_ARG;
    }
    uint32_t bits = 0;
    DIR_CHK(hipMemcpyAsync(&bits, status, sizeof(bits), hipMemcpyDeviceToHost, st));
    DIR_CHK(hipStreamSynchronize(st));
    ksum_collect();
    if (bits & ST_TYPE_RANGE) return TG_E_TYPE_RANGE;
    if (bits) return TG_E_NOT_SIMPLE;
    if (m > 0) {
        k_dir_edges_of<<<waves_grid(n), 256, 0, st>>>(row_ptr, col, eoff, n, esrc, eslot);
        int32_t *hub_id = reinterpret_cast<int32_t *>(w + y.hub_id);
        int32_t *hub_node = reinterpret_cast<int32_t *>(w + y.hub_node);
        unsigned long long *hbits = reinterpret_cast<unsigned long long *>(w + y.hbits);
        uint32_t *hprefix = reinterpret_cast<uint32_t *>(w + y.hprefix);
        unsigned int *hcount = reinterpret_cast<unsigned int *>(status + 4);   // own 16-byte slot
        ksum_begin(st);
        DIR_CHK(launch_fill_u64(reinterpret_cast<uint64_t *>(hcount), 0, 1, st));
        k_dir_hub_ids<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(row_ptr, n, y.hub_max, hub_id,
                                                                  hub_node, hcount);
        if (y.hub_max > 0)
            k_dir_hub_bits<<<(unsigned)y.hub_max, 256, 0, st>>>(row_ptr, col, hub_node, hcount,
                                                               y.hub_max, y.nw, hbits, hprefix);
        ksum_end("dir_hubs", 0.0, st);
        DIR_CHK(hipGetLastError());
        ksum_begin(st);
        k_dir_rows<<<waves_grid(m), 256, 0, st>>>(row_ptr, col, dir, types, deg3, esrc, eslot, m,
                                                   L, hub_id, hbits, hprefix, y.nw, rows);
        ksum_end("dir_rows", 0.0, st);
        DIR_CHK(hipGetLastError());
        if (global_counts) {
            uint64_t *ckey = reinterpret_cast<uint64_t *>(w + y.ckey);
            uint32_t *cval = reinterpret_cast<uint32_t *>(w + y.cval);
            unsigned long long *csum = reinterpret_cast<unsigned long long *>(w + y.csum);
            unsigned long long *ccount = reinterpret_cast<unsigned long long *>(w + y.ccount);
            const int64_t classes = 3 * (int64_t)L * L;
            ksum_begin(st);
            DIR_CHK(launch_fill_u64(reinterpret_cast<uint64_t *>(csum), 0, classes * 15 * L, st));
            DIR_CHK(launch_fill_u64(reinterpret_cast<uint64_t *>(ccount), 0, classes, st));
            k_dir_class<<<(unsigned)((m + 255) / 256), 256, 0, st>>>(col, dir, types, esrc, eslot, m,
                                                                      L, ckey, cval);
            DIR_CHK(hipGetLastError());
            uint64_t *skey = nullptr;
            uint32_t *sval = nullptr;
            int bits_needed = 1;
            while ((int64_t(1) << bits_needed) < classes) ++bits_needed;
            DIR_CHK(radix_sort(ckey, reinterpret_cast<uint64_t *>(w + y.ckey_tmp), cval,
                               reinterpret_cast<uint32_t *>(w + y.cval_tmp), m, bits_needed,
                               w + y.sort_tmp, nullptr, st, &skey, &sval));
            const int64_t waves = (int64_t)waves_grid(m) * 4;
            const int64_t per_wave = (m + waves - 1) / waves;
            k_dir_class_sums<<<(unsigned)((waves + 3) / 4), 256, 0, st>>>(skey, sval, rows, m, L,
                                                                          per_wave, csum);
            k_dir_class_count<<<(unsigned)((m + 255) / 256), 256, 0, st>>>(skey, m, ccount);
            const int64_t items = classes * (15 * L + 1);
            k_dir_keys<<<(unsigned)((items + 255) / 256), 256, 0, st>>>(csum, ccount, L, acc);
            ksum_end("dir_global", 0.0, st);
            DIR_CHK(hipGetLastError());
        }
    }
    if (global_counts) {
        k_dir_finalize<<<(unsigned)((width + 255) / 256), 256, 0, st>>>(acc, width, L, global_counts,
                                                                        status);
        DIR_CHK(hipGetLastError());
        DIR_CHK(hipMemcpyAsync(&bits, status, sizeof(bits), hipMemcpyDeviceToHost, st));
    }
    DIR_CHK(hipStreamSynchronize(st));
    ksum_collect();
#undef DIR_CHK
    return bits ? TG_E_INTERNAL : TG_OK;
}

}  // extern "C"
