// Device kernels of the typed-graphlet library (gfx950, wave64).
//
// Pipeline for one graph (all integer arithmetic):
//   prep      validate the CSR, relabel nodes by (degree, id) so that a
//             larger internal id means a higher rank, build the relabelled
//             CSR with each slot's canonical edge id, typed degrees.
//   tri       typed triangle counts |T_ij^t| per edge (Cor. 1; intersection
//             of the two neighbour lists).
//   aggr      per node u: A_u(t,t') = sum over type-t neighbours k of
//             |T_uk^t'| and D_u(t,t') = sum over type-t neighbours k of
//             d_k^t'.
//   cycles    non-induced typed 4-cycle counts NC per edge from
//             degree-ordered wedges: every 4-cycle is found once from its
//             highest-ranked vertex (pass A credits the two cycle edges at
//             that vertex, pass B the two far edges).
//   edges     per edge: the triangle set T, ordered typed clique pairs K
//             (Alg. 3's 4-clique branch), gathers X_i, X_j, Y over T; then
//             every orbit of Table 3 by inclusion-exclusion in the spirit of
//             Theorem 1 and Lemmas 1-4, the row write, and the per-workgroup
//             histogram of global counts (Problem 2).
#include <hip/hip_runtime.h>

#include "tg_device.hpp"

namespace tg {

// ------------------------------------------------------------------ prep

__global__ void k_fill_u64(uint64_t *p, uint64_t v, int64_t count) {
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < count; q += stride) p[q] = v;
}

// One wave per input row (grid-stride): row checks, degree, number of larger
// neighbours.
__global__ void k_check_rows(const int64_t *__restrict__ rp, const int32_t *__restrict__ col,
                             const uint8_t *__restrict__ types, int64_t n, int64_t nnz, int L,
                             uint32_t *__restrict__ deg, int64_t *__restrict__ ucount,
                             uint32_t *__restrict__ status, const int32_t *__restrict__ node_graph,
                             const int32_t *__restrict__ gL) {
    const int lane = lane_id();
    if (input_failed(status)) return;  // inconsistent batch descriptor
    if (blockIdx.x == 0 && threadIdx.x == 0) ucount[n] = 0;  // sentinel of the exclusive scan
    const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x / WAVE);
    for (int64_t u = (int64_t)blockIdx.x * (blockDim.x / WAVE) + (threadIdx.x / WAVE); u < n;
         u += nwaves) {
    int64_t b = rp[u], e = rp[u + 1];
    uint32_t bad = 0;
    if (b < 0 || e > nnz || e < b || (u == 0 && b != 0) || (u == n - 1 && e != nnz)) {
        if (lane == 0) {
            atomicOr(status, ST_UNSORTED);
            deg[u] = 0;
            ucount[u] = 0;
        }
        continue;
    }
    uint64_t up = 0;
    const int32_t gu = node_graph ? node_graph[u] : 0;
    for (int64_t s = b + lane; s < e; s += WAVE) {
        int32_t x = col[s];
        if (x < 0 || x >= n) bad |= ST_COL_RANGE;
        else if (node_graph && node_graph[x] != gu) bad |= ST_CROSS_GRAPH;
        if (x == u) bad |= ST_SELF_LOOP;
        if (s > b && col[s - 1] >= x) bad |= ST_UNSORTED;
        if (x > u) ++up;
    }
    up = wave_sum_u64(up);
    bad = wave_or(bad);
    if (lane == 0) {
        if (types[u] >= (node_graph ? gL[gu] : L)) bad |= ST_TYPE_RANGE;
        deg[u] = (uint32_t)(e - b);
        ucount[u] = (int64_t)up;
        if (bad) atomicOr(status, bad);
    }
    }
}

// Batch descriptor checks (one thread per graph) and the node -> graph map
// (one wave per graph, written only for a consistent descriptor).
__global__ void k_batch_graphs(const int64_t *__restrict__ node_ptr, const int32_t *__restrict__ gL,
                               const int64_t *__restrict__ goff, int64_t G, int64_t n, int L_max,
                               int64_t globals_len, int64_t max_nodes,
                               int32_t *__restrict__ node_graph, uint32_t *__restrict__ status,
                               uint64_t *__restrict__ max_gsize) {
    int64_t g = (int64_t)blockIdx.x * (blockDim.x / WAVE) + (threadIdx.x / WAVE);
    int lane = lane_id();
    if (g >= G) return;
    int64_t a = node_ptr[g], b = node_ptr[g + 1];
    int Lg = gL[g];
    bool ok = a >= 0 && b >= a && b <= n && Lg >= 1 && Lg <= L_max;
    if (max_nodes >= 0 && b - a > max_nodes) ok = false;  // above the declared bound
    if (g == 0 && (a != 0 || goff[0] != 0)) ok = false;
    if (g == G - 1 && (b != n || goff[G] != globals_len)) ok = false;
    if (ok) {
        int64_t w = binom_small(Lg + 1, 2) + 2 * binom_small(Lg + 2, 3) + 6 * binom_small(Lg + 3, 4);
        if (goff[g + 1] - goff[g] != w) ok = false;
    }
    if (!ok) {
        if (lane == 0) atomicOr(status, ST_BATCH);
        return;
    }
    for (int64_t v = a + lane; v < b; v += WAVE) node_graph[v] = (int32_t)g;
    if (lane == 0 && b > a) atomicMax((unsigned long long *)max_gsize, (unsigned long long)(b - a));
}

__global__ void k_batch_edges(const int64_t *__restrict__ node_ptr, const int64_t *__restrict__ eoff,
                              int64_t G, int64_t *__restrict__ gedge_ptr,
                              const uint32_t *__restrict__ status) {
    if (input_failed(status)) return;
    int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g <= G) gedge_ptr[g] = eoff[node_ptr[g]];
}

// Per-graph global vectors: divide each graphlet block by its edge count.
__global__ void k_batch_finalize(uint64_t *__restrict__ glob, const int32_t *__restrict__ gL,
                                 const int64_t *__restrict__ goff, int64_t G,
                                 uint32_t *__restrict__ status) {
    if (input_failed(status)) return;
    const uint64_t E[9] = {1, 2, 3, 3, 3, 4, 4, 5, 6};
    for (int64_t g = blockIdx.x; g < G; g += gridDim.x) {
        int Lg = gL[g];
        int n2 = (int)binom_small(Lg + 1, 2), n3 = (int)binom_small(Lg + 2, 3),
            n4 = (int)binom_small(Lg + 3, 4);
        int gw = n2 + 2 * n3 + 6 * n4;
        uint64_t *v = glob + goff[g];
        for (int q = threadIdx.x; q < gw; q += blockDim.x) {
            int h;
            if (q < n2) h = 0;
            else if (q < n2 + n3) h = 1;
            else if (q < n2 + 2 * n3) h = 2;
            else h = 3 + (q - n2 - 2 * n3) / n4;
            if (v[q] % E[h]) atomicOr(status, ST_NOT_DIVISIBLE);
            v[q] /= E[h];
        }
    }
}

// Sort keys of the relabelling: the degree, or for a batch (graph, degree)
// so each graph's nodes stay contiguous (graphlets never span graphs, so a
// per-graph degree order serves the cycle orientation as well); the values
// are the node ids, so a stable sort ranks nodes by (degree, id).
__global__ void k_node_keys(const uint32_t *__restrict__ deg, int64_t n,
                            const int32_t *__restrict__ node_graph, int deg_bits,
                            uint64_t *__restrict__ keys, uint32_t *__restrict__ ids,
                            const uint32_t *__restrict__ status) {
    if (input_failed(status)) return;
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    uint64_t k = (uint64_t)deg[v];
    if (node_graph) k |= (uint64_t)node_graph[v] << deg_bits;
    keys[v] = k;
    ids[v] = (uint32_t)v;
}

__global__ void k_relabel(const uint32_t *__restrict__ sorted_ids, const uint8_t *__restrict__ types,
                          const uint32_t *__restrict__ deg, int64_t n,
                          int32_t *__restrict__ order, int32_t *__restrict__ newid,
                          uint8_t *__restrict__ ntype, int64_t *__restrict__ ndeg,
                          uint64_t *__restrict__ hub_cand, uint32_t sh_deg,
                          const int32_t *__restrict__ node_graph, int32_t *__restrict__ ngraph,
                          const uint32_t *__restrict__ status) {
    if (input_failed(status)) return;
    int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool cand = false;
    if (r < n) {
        int32_t v = (int32_t)sorted_ids[r];
        order[r] = v;
        if (node_graph) ngraph[r] = node_graph[v];
        newid[v] = (int32_t)r;
        ntype[r] = types[v];
        ndeg[r] = deg[v];
        cand = deg[v] >= (uint32_t)HUB_DMIN;
    }
    if (r == 0) ndeg[n] = 0;
    uint64_t bal = __ballot(cand);
    if (lane_id() == 0 && bal)
        atomicAdd((unsigned long long *)hub_cand, (unsigned long long)__popcll(bal));
    uint64_t sbal = __ballot(r < n && ndeg[r] >= (int64_t)sh_deg);
    if (lane_id() == 0 && sbal)
        atomicAdd((unsigned long long *)(hub_cand + 1), (unsigned long long)__popcll(sbal));
}

// One wave per input row (grid-stride): canonical edge id of every slot, the relabelled
// slot key (row << bits | col), and the canonical endpoints of each edge.
__global__ void k_slot_keys(const int64_t *__restrict__ rp, const int32_t *__restrict__ col,
                            const int64_t *__restrict__ ucount, const int64_t *__restrict__ eoff,
                            const int32_t *__restrict__ newid, int64_t n, int bits,
                            uint64_t *__restrict__ keys, uint32_t *__restrict__ vals,
                            int32_t *__restrict__ ei, int32_t *__restrict__ ej,
                            uint32_t *__restrict__ status) {
    if (input_failed(status)) return;  // includes an edge count that is not nnz / 2
    const int lane = lane_id();
    const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x / WAVE);
    for (int64_t u = (int64_t)blockIdx.x * (blockDim.x / WAVE) + (threadIdx.x / WAVE); u < n;
         u += nwaves) {
    int64_t b = rp[u], e = rp[u + 1];
    int64_t ustart = e - ucount[u];
    uint32_t bad = 0;
    uint64_t nu = (uint64_t)newid[u];
    for (int64_t s = b + lane; s < e; s += WAVE) {
        int32_t x = col[s];
        int64_t eid;
        if (x > u) {
            eid = eoff[u] + (s - ustart);
            ei[eid] = (int32_t)nu;
            ej[eid] = newid[x];
        } else {
            int64_t xb = rp[x], xe = rp[x + 1];
            int64_t p = lower_bound(col, xb, xe, (int32_t)u);
            if (p >= xe || col[p] != (int32_t)u) {
                bad |= ST_ASYMMETRIC;
                eid = 0;
            } else {
                eid = eoff[x] + (p - (xe - ucount[x]));
            }
        }
        keys[s] = (nu << bits) | (uint64_t)newid[x];
        vals[s] = (uint32_t)eid;
    }
    bad = wave_or(bad);
    if (lane == 0 && bad) atomicOr(status, bad);
    }
}

// Sorted keys (row << bits | column) to the relabelled CSR, plus the slot of
// every edge in both of its rows: eslot[2e] in the row of its smaller end,
// eslot[2e + 1] in the row of its larger end.
__global__ void k_finish_csr(const uint64_t *__restrict__ keys, const uint32_t *__restrict__ vals,
                             int64_t nnz, int bits, const uint8_t *__restrict__ ntype,
                             uint32_t *__restrict__ eslot, int32_t *__restrict__ ncol,
                             uint32_t *__restrict__ neid, uint8_t *__restrict__ ctype,
                             const uint32_t *__restrict__ status) {
    if (input_failed(status)) return;
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s < nnz) {
        uint64_t k = keys[s];
        int32_t c = (int32_t)(k & ((1ull << bits) - 1));
        int32_t r = (int32_t)(k >> bits);
        uint32_t e = vals[s];
        ncol[s] = c;
        neid[s] = e;
        ctype[s] = ntype[c];
        eslot[2 * (size_t)e + (r < c ? 0 : 1)] = (uint32_t)s;
    }
}

// One wave per internal node: typed degrees d_v^t (rows padded to
// tri_pitch(L) words) and the first slot of the row's hub suffix (neighbours with internal id >= hub_base).
__global__ void k_tdeg(const int64_t *__restrict__ nrp, const int32_t *__restrict__ ncol,
                       const uint8_t *__restrict__ ctype, int64_t n, int L, int32_t hub_base,
                       uint32_t *__restrict__ tdeg, int64_t *__restrict__ hstart,
                       uint32_t *__restrict__ nlow, const uint32_t *__restrict__ status) {
    if (input_failed(status)) return;
    const int lane = lane_id();
    const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x / WAVE);
    for (int64_t v = (int64_t)blockIdx.x * (blockDim.x / WAVE) + (threadIdx.x / WAVE); v < n;
         v += nwaves) {
        if (lane == 0) {
            hstart[v] = lower_bound(ncol, nrp[v], nrp[v + 1], hub_base);
            nlow[v] = (uint32_t)(lower_bound(ncol, nrp[v], nrp[v + 1], (int32_t)v) - nrp[v]);
        }
        uint32_t c = 0;
        for (int64_t base = nrp[v]; base < nrp[v + 1]; base += WAVE) {
            int64_t s = base + lane;
            int t = s < nrp[v + 1] ? (int)ctype[s] : -1;
            for (int tt = 0; tt < L; ++tt) {
                uint64_t bal = __ballot(t == tt);
                if (lane == tt) c += (uint32_t)__popcll(bal);
            }
        }
        const int LP = tri_pitch(L);
        if (lane < LP) tdeg[v * LP + lane] = lane < L ? c : 0u;
    }
}

// ------------------------------------------------------- typed triangles

// Typed triangles: a wave takes TRI_GROUPS consecutive edges, one group of
// WAVE/TRI_GROUPS lanes per edge; a group walks the shorter row and tests each
// node against the longer one (its super-hub bitmap when it has one, the
// hub-core bit matrix when both are hubs, else a binary search), counting
// hits by type.
constexpr int TRI_GROUPS = 8;
constexpr int TRI_LANES = WAVE / TRI_GROUPS;

// A register budget for eight waves per SIMD (two registers spill) hides more
// of the probes' latency than seven waves do.
__global__ void __attribute__((amdgpu_waves_per_eu(8)))
k_tri(const int64_t *__restrict__ nrp, const int32_t *__restrict__ ncol,
                      const uint8_t *__restrict__ ctype, const int32_t *__restrict__ ei,
                      const int32_t *__restrict__ ej, const uint32_t *__restrict__ eslot,
                      uint32_t *__restrict__ tri_slot, int64_t m, int L,
                      uint32_t *__restrict__ tri, uint64_t *__restrict__ tri_sum, int32_t sh_base,
                      int64_t nw, const uint64_t *__restrict__ SB, int32_t hub_base, int Hw,
                      const uint64_t *__restrict__ HB, const uint32_t *__restrict__ status) {
    if (input_failed(status)) return;
    const int64_t wave = (int64_t)blockIdx.x * (blockDim.x / WAVE) + (threadIdx.x / WAVE);
    const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x / WAVE);
    const int lane = lane_id();
    const int grp = lane / TRI_LANES, gl = lane % TRI_LANES;
    uint64_t tot_all = 0;
    // a bounded grid walks the edges: per-edge work is small, so launching
    // one workgroup per 32 edges would leave the dispatcher as the limit
    for (int64_t wv = wave; wv * TRI_GROUPS < m; wv += nwaves) {
        const int64_t e = wv * TRI_GROUPS + grp;
        uint32_t cnt[TG_MAX_L];
#pragma unroll
        for (int t = 0; t < TG_MAX_L; ++t) cnt[t] = 0;
        if (e < m) {
            int32_t i = ei[e], j = ej[e];
            int64_t sb = nrp[i], se = nrp[i + 1], bb = nrp[j], be = nrp[j + 1];
            int32_t big = j;
            if (se - sb > be - bb) {
                int64_t t0 = sb, t1 = se;
                sb = bb; se = be; bb = t0; be = t1;
                big = i;
            }
            const bool probe = big >= sh_base;
            const int sidx = big - sh_base;
            const bool big_hub = big >= hub_base;
            const uint64_t *hrow = big_hub ? HB + (size_t)(big - hub_base) * Hw : nullptr;
            for (int64_t s = sb + gl; s < se; s += TRI_LANES) {
                int32_t x = ncol[s];
                bool found;
                if (probe) {
                    found = sh_bit(SB, nw, sidx, x);
                } else if (big_hub && x >= hub_base) {
                    // both in the hub core: its bit matrix
                    const int hx = x - hub_base;
                    found = (hrow[hx >> 6] >> (hx & 63)) & 1ull;
                } else {
                    int64_t q = lower_bound(ncol, bb, be, x);
                    found = q < be && ncol[q] == x;
                }
                if (found) {
                    int tx = ctype[s];
#pragma unroll
                    for (int t = 0; t < TG_MAX_L; ++t) cnt[t] += (t == tx);
                }
            }
        }
        uint64_t tot = 0;
        // every lane of the group ends with all totals; lane t % 8 stores type t,
        // so a slot's row is written by neighbouring lanes at once
        const int LP = tri_pitch(L);
        const size_t si = e < m ? (size_t)eslot[2 * e] * LP : 0;
        const size_t sj = e < m ? (size_t)eslot[2 * e + 1] * LP : 0;
#pragma unroll
        for (int t = 0; t < TG_MAX_L; ++t) {
            if (t < L) {
                uint32_t v = cnt[t];
#pragma unroll
                for (int d = 1; d < TRI_LANES; d <<= 1) v += __shfl_xor(v, d, WAVE);
                if ((t % TRI_LANES) == gl && e < m) {
                    tri[e * L + t] = v;
                    tri_slot[si + t] = v;
                    tri_slot[sj + t] = v;
                }
                tot += v;
            }
        }
        // one count per group (lanes of a group hold the same totals)
        tot_all += gl == 0 ? tot : 0ull;
    }
    tot_all = wave_sum_u64(tot_all);
    if (lane == 0 && tot_all) atomicAdd((unsigned long long *)tri_sum, (unsigned long long)tot_all);
}

// One workgroup per super-hub: bitmap of its neighbours over all nodes and
// the per-word exclusive prefix popcounts (slot of a neighbour in the row).
__global__ void __launch_bounds__(256) k_superhubs(const int64_t *__restrict__ nrp,
                                                   const int32_t *__restrict__ ncol, int64_t n,
                                                   int S, int64_t nw, uint64_t *__restrict__ SB,
                                                   uint32_t *__restrict__ SP) {
    __shared__ uint32_t part[256];
    const int s = blockIdx.x;
    if (s >= S) return;
    const int tid = threadIdx.x;
    const int64_t v = n - S + s;
    uint64_t *bits = SB + (size_t)s * nw;
    uint32_t *pre = SP + (size_t)s * nw;
    for (int64_t q = tid; q < nw; q += 256) bits[q] = 0ull;
    __syncthreads();
    for (int64_t p = nrp[v] + tid; p < nrp[v + 1]; p += 256) {
        int32_t x = ncol[p];
        __hip_atomic_fetch_or((unsigned long long *)&bits[x >> 6], 1ull << (x & 63),
                              __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
    __syncthreads();
    // contiguous word segments per thread, then a block scan of their sums
    const int64_t seg = (nw + 255) / 256;
    const int64_t q0 = tid * seg, q1 = q0 + seg < nw ? q0 + seg : nw;
    uint32_t sum = 0;
    for (int64_t q = q0; q < q1; ++q)
        sum += (uint32_t)__popcll(__hip_atomic_load((unsigned long long *)&bits[q], __ATOMIC_RELAXED,
                                                    __HIP_MEMORY_SCOPE_WORKGROUP));
    part[tid] = sum;
    __syncthreads();
    if (tid == 0) {
        uint32_t run = 0;
        for (int q = 0; q < 256; ++q) {
            uint32_t c = part[q];
            part[q] = run;
            run += c;
        }
    }
    __syncthreads();
    uint32_t run = part[tid];
    for (int64_t q = q0; q < q1; ++q) {
        pre[q] = run;
        run += (uint32_t)__popcll(__hip_atomic_load((unsigned long long *)&bits[q], __ATOMIC_RELAXED,
                                                    __HIP_MEMORY_SCOPE_WORKGROUP));
    }
}

// ------------------------------------------------------ node aggregates

// One wave per internal node u; LDS holds A_u and D_u (L x L uint64 each).
// An entry of A_u sums at most d_u triangle counts of at most d_u, one of
// D_u at most d_u degrees, so with every degree below 2^16 both are stored
// as uint32 (ad_u32).
__global__ void k_node_aggr(const int64_t *__restrict__ nrp, const int32_t *__restrict__ ncol,
                            const uint8_t *__restrict__ ctype, const uint32_t *__restrict__ tri_slot,
                            const uint32_t *__restrict__ tdeg,
                            int64_t n, int L, uint64_t *__restrict__ A, uint64_t *__restrict__ D,
                            int ad_u32, const uint32_t *__restrict__ status) {
    if (input_failed(status)) return;
    extern __shared__ uint64_t sm_aggr[];
    int w = threadIdx.x / WAVE;
    int lane = lane_id();
    int LL = L * L;
    uint64_t *sA = sm_aggr + (size_t)w * 2 * LL;
    uint64_t *sD = sA + LL;
    const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x / WAVE);
    for (int64_t u = (int64_t)blockIdx.x * (blockDim.x / WAVE) + w; u < n; u += nwaves) {
        for (int q = lane; q < LL; q += WAVE) { sA[q] = 0; sD[q] = 0; }
        wave_sync();
        for (int64_t s = nrp[u] + lane; s < nrp[u + 1]; s += WAVE) {
            int32_t k = ncol[s];
            int t = ctype[s];
            const uint32_t *ts = tri_slot + (size_t)s * tri_pitch(L);
            const uint32_t *dk = tdeg + (size_t)k * tri_pitch(L);
            for (int t2 = 0; t2 < L; ++t2) {
                uint32_t a = ts[t2];
                uint32_t d = dk[t2];
                if (a) atomicAdd((unsigned long long *)&sA[t * L + t2], (unsigned long long)a);
                if (d) atomicAdd((unsigned long long *)&sD[t * L + t2], (unsigned long long)d);
            }
        }
        wave_sync();
        if (ad_u32) {
            uint32_t *A32 = reinterpret_cast<uint32_t *>(A), *D32 = reinterpret_cast<uint32_t *>(D);
            for (int q = lane; q < LL; q += WAVE) {
                A32[(size_t)u * LL + q] = (uint32_t)sA[q];
                D32[(size_t)u * LL + q] = (uint32_t)sD[q];
            }
        } else {
            for (int q = lane; q < LL; q += WAVE) {
                A[(size_t)u * LL + q] = sA[q];
                D[(size_t)u * LL + q] = sD[q];
            }
        }
        wave_sync();
    }
}

// ------------------------------------------------------------ 4-cycles
//
// A wedge is a path x - g - ... seen from a "group" vertex.  Pass A groups by
// the cycle's top vertex v (largest internal id): items are v's lower
// neighbours u, targets are u's neighbours w < v, the map counts, per w, the
// centres u by type.  Every pair of centres sharing (v, w) closes the 4-cycle
// v-u1-w-u2; its two edges at v, oriented (v, u), get +1 at (type u2, type w).
// Pass B groups by the vertex a opposite the top: items are all neighbours c
// of a, targets are c's neighbours v above both a and c, the map counts, per
// v, the centres c by type; the far edge oriented (c, a) gets +1 at
// (type v, type of the other centre).  NC is kept in canonical orientation.



template <int PASS>
__device__ __forceinline__ void item_range(const CycleArgs &a, int32_t g, int64_t &ib, int64_t &ie) {
    ib = a.nrp[g];
    if (PASS == 0) ie = ib + a.nlow[g];
    else ie = a.nrp[g + 1];
}

// Slot of g in the row of its neighbour x, for the item at a slot of g's row
// holding edge e.
__device__ __forceinline__ int64_t slot_in_row_of(const CycleArgs &a, int32_t g, int32_t x,
                                                  uint32_t e) {
    return (int64_t)a.eslot[2 * (size_t)e + (x < g ? 0 : 1)];
}

// Targets of item x (edge e) in group g: pass A, x's neighbours below g;
// pass B, x's neighbours above both g and x.  The row is sorted, so both
// are contiguous, bounded by g's own slot in x's row or x's split point.
template <int PASS>
__device__ __forceinline__ void target_range(const CycleArgs &a, int32_t g, int32_t x, uint32_t e,
                                             int64_t &tb, int64_t &te) {
    const int64_t xb = a.nrp[x];
    if (PASS == 0) {
        tb = xb;
        te = slot_in_row_of(a, g, x, e);
    } else {
        tb = g > x ? slot_in_row_of(a, g, x, e) + 1 : xb + a.nlow[x];
        te = a.nrp[x + 1];
    }
}

// flip = 1 when the pass orientation is the reverse of the canonical one.
template <int PASS>
__device__ __forceinline__ int orient_flip(const CycleArgs &a, int32_t g, int32_t x, uint32_t e) {
    int32_t ci = a.ei[e];
    return PASS == 0 ? (ci != g) : (ci != x);
}

// Matrix index (pass orientation) of the count for centre type t, target type ty.
template <int PASS>
__device__ __forceinline__ int pass_entry(int t, int ty, int L) {
    return PASS == 0 ? t * L + ty : ty * L + t;
}

constexpr uint32_t EMPTY_KEY = 0xffffffffu;

__device__ __forceinline__ int hash_slot(uint32_t y, int log2_slots) {
    return (int)((y * 0x9E3779B1u) >> (32 - log2_slots));
}

// Adds v to NC entry idx.  An entry counts 4-cycles through one edge, at
// most (d_i - 1)(d_j - 1), so with every degree below 2^16 NC holds uint32.
__device__ __forceinline__ void nc_add(const CycleArgs &a, size_t idx, uint64_t v) {
    if (a.nc_u32)
        atomicAdd(reinterpret_cast<unsigned int *>(a.NC) + idx, (unsigned int)v);
    else
        atomicAdd((unsigned long long *)&a.NC[idx], (unsigned long long)v);
}

// Light groups: one 64-thread workgroup per group, LDS open-addressing map
// keyed by target with 16-bit counters per type (group wedges at most the
// light bucket bound, itself at most LIGHT_MAXW); the map has the smallest
// power-of-two slot count above that bound, so smaller buckets take less LDS
// and fit more workgroups on a CU.
template <int PASS>
__global__ void __launch_bounds__(64) k_cyc_light(CycleArgs a) {
    extern __shared__ uint32_t sm_light[];
    const int L = a.L;
    const int LW = (L + 1) / 2;
    uint32_t *keys = sm_light;
    // slots: the smallest power of two above the light bucket, so a group's
    // distinct targets (at most its wedges) always find a free slot
    const int HC = 1 << a.light_log2;
    uint32_t *cnt = keys + HC;
    __shared__ int32_t it_tx[WAVE];  // type of each staged item (the centre)
    __shared__ int64_t it_tb[WAVE];
    __shared__ uint32_t it_scan[WAVE];
    __shared__ uint32_t it_eid[WAVE];
    __shared__ int it_flip[WAVE];
    int lane = threadIdx.x;
    if (input_failed(a.status)) return;
    uint64_t count = a.counters[a.count_idx];
    for (int q = lane; q < HC; q += WAVE) keys[q] = EMPTY_KEY;
    for (int q = lane; q < HC * LW; q += WAVE) cnt[q] = 0;
    __syncthreads();
    for (uint64_t idx = blockIdx.x; idx < count; idx += gridDim.x) {
        int32_t g = (int32_t)a.list[idx];
        int64_t ib, ie;
        item_range<PASS>(a, g, ib, ie);
        for (int phase = 0; phase < 2; ++phase) {
            for (int64_t cb = ib; cb < ie; cb += WAVE) {
                int64_t s = cb + lane;
                uint32_t len = 0;
                if (s < ie) {
                    int32_t x = a.ncol[s];
                    uint32_t e = a.neid[s];
                    int64_t tb, te;
                    target_range<PASS>(a, g, x, e, tb, te);
                    len = (uint32_t)(te - tb);
                    it_tx[lane] = a.ntype[x];
                    it_tb[lane] = tb;
                    it_eid[lane] = e;
                    it_flip[lane] = phase ? orient_flip<PASS>(a, g, x, e) : 0;
                }
                uint32_t incl = wave_incl_scan(len);
                it_scan[lane] = incl;
                uint32_t total = __shfl(incl, WAVE - 1, WAVE);
                int nitems = (int)((ie - cb) < WAVE ? (ie - cb) : WAVE);
                __syncthreads();
                int o = 0;
                for (uint32_t f = lane; f < total; f += WAVE) {
                    o = owner_next(it_scan, nitems, f, o);
                    uint32_t excl = o ? it_scan[o - 1] : 0;
                    const int tx = it_tx[o];
                    const int64_t ys = it_tb[o] + (f - excl);
                    uint32_t y = (uint32_t)a.ncol[ys];
                    int h = hash_slot(y, a.light_log2);
                    if (phase == 0) {
                        // the group has fewer distinct keys than slots, so the
                        // probe ends; the bound only guards corrupted input
                        bool ok = false;
                        for (int probe = 0; probe < HC; ++probe) {
                            uint32_t old = atomicCAS(&keys[h], EMPTY_KEY, y);
                            if (old == EMPTY_KEY || old == y) { ok = true; break; }
                            h = (h + 1) & (HC - 1);
                        }
                        if (ok) atomicAdd(&cnt[h * LW + (tx >> 1)], 1u << ((tx & 1) * 16));
                        else atomicOr(a.status, ST_INTERNAL);
                    } else {
                        int probe = 0;
                        while (keys[h] != y && probe < HC) {
                            h = (h + 1) & (HC - 1);
                            ++probe;
                        }
                        if (probe == HC) {
                            atomicOr(a.status, ST_INTERNAL);
                            continue;
                        }
                        int ty = a.ctype[ys];
                        uint32_t e = it_eid[o];
                        int flip = it_flip[o];
                        const size_t nc0 = (size_t)e * L * L;
                        for (int t = 0; t < L; ++t) {
                            uint32_t c = (cnt[h * LW + (t >> 1)] >> ((t & 1) * 16)) & 0xffffu;
                            uint32_t val = c - (t == tx ? 1u : 0u);
                            if (val) {
                                int pq = pass_entry<PASS>(t, ty, L);
                                int p = pq / L, q = pq - p * L;
                                int canon = flip ? q * L + p : pq;
                                nc_add(a, nc0 + canon, val);
                            }
                        }
                    }
                }
                __syncthreads();
            }
        }
        for (int q = lane; q < HC; q += WAVE) keys[q] = EMPTY_KEY;
        for (int q = lane; q < HC * LW; q += WAVE) cnt[q] = 0;
        __syncthreads();
    }
}

// Block-wide inclusive scan of up to NT/2 values held by threads [0, NT/2);
// result in s[0..NT/2).
template <int NT>
__device__ __forceinline__ void block_scan_chunk(uint32_t v, uint32_t *s, uint32_t *wave_tot) {
    int tid = threadIdx.x;
    int w = tid / WAVE;
    uint32_t incl = wave_incl_scan(v);
    if ((tid & (WAVE - 1)) == WAVE - 1) wave_tot[w] = incl;
    __syncthreads();
    uint32_t add = 0;
    for (int q = 0; q < w; ++q) add += wave_tot[q];
    if (tid < NT / 2) s[tid] = incl + add;
    __syncthreads();
}

// Boundary k of a split of target ids [rb, re) into `parts` ranges: the
// first id c with mass(rb, c) / mass(rb, re) + (c - rb) / (re - rb) >=
// 2k / parts, where mass is adjacency (row starts are nondecreasing).  Each
// range then holds at most 2 / parts of the adjacency mass (targets are met
// in proportion to their degree) and at most 2 / parts of the ids (the map
// entries a range touches).
__device__ __forceinline__ int32_t range_cut(const int64_t *nrp, int32_t rb, int32_t re, uint32_t k,
                                             uint32_t parts) {
    if (k == 0) return rb;
    if (k >= parts) return re;
    const int64_t base = nrp[rb];
    const double inv_mass = 1.0 / (double)(nrp[re] - base > 0 ? nrp[re] - base : 1);
    const double inv_ids = 1.0 / (double)(re - rb);
    const double target = 2.0 * (double)k / (double)parts;
    int32_t lo = rb, hi = re;
    while (lo < hi) {
        int32_t mid = lo + ((hi - lo) >> 1);
        double f = (double)(nrp[mid] - base) * inv_mass + (double)(mid - rb) * inv_ids;
        if (f < target) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// Copies of the task kernel's 32-bit tallies (every degree below 2^16).
constexpr int TALLY_COPIES = 2;   // (4 measured slower)

// Map entries by target degree class.  The count of centres of one type at
// target w never exceeds w's degree, so targets of degree < 16 keep 4-bit
// counts, < 64 6-bit, < 256 8-bit, < 1024 10-bit, < 65536 16-bit and the
// rest 32-bit.  A word holds F = 32 / bits fields (none crosses a word), so
// an entry takes ceil(L / F) words.  With ids ranked by degree each class is
// one id range; the classes are laid out one after the other (class c: ids
// [s[c], s[c+1]) from word o[c]), so a task's entries are one contiguous word
// range.
constexpr int MAP_CLASSES = 6;

struct MapClasses {
    int32_t s[MAP_CLASSES];     // first id of each class (s[0] = 0)
    uint64_t o[MAP_CLASSES];    // first word of each class
};

__device__ __forceinline__ int class_bits(int c) {
    return c == 0 ? 4 : c == 1 ? 6 : c == 2 ? 8 : c == 3 ? 10 : c == 4 ? 16 : 32;
}

__device__ __forceinline__ int class_words(int c, int L) {
    const int F = 32 / class_bits(c);
    return (L + F - 1) / F;
}

__device__ __forceinline__ int map_class(const MapClasses &m, int32_t w) {
    int c = 0;
#pragma unroll
    for (int q = 1; q < MAP_CLASSES; ++q) c += w >= m.s[q];
    return c;
}

// First word of target w's entry in class c (w may be n: the layout's end).
__device__ __forceinline__ uint64_t map_word(const MapClasses &m, int32_t w, int c, int L) {
    int32_t st = 0;
    uint64_t of = 0;
#pragma unroll
    for (int q = 0; q < MAP_CLASSES; ++q)
        if (q == c) {
            st = m.s[q];
            of = m.o[q];
        }
    return of + (uint64_t)(w - st) * (uint64_t)class_words(c, L);
}

// First node id of degree >= d (degrees nondecreasing in id).
__device__ __forceinline__ int32_t first_of_degree(const int64_t *nrp, int64_t n, int64_t d) {
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (nrp[mid + 1] - nrp[mid] < d) lo = mid + 1; else hi = mid;
    }
    return (int32_t)lo;
}

__device__ MapClasses map_classes(const CycleArgs &a) {
    MapClasses m;
    const int32_t n = (int32_t)a.n;
    m.s[0] = 0;
    if (a.deg_sorted) {
        const int64_t lim[MAP_CLASSES - 1] = {16, 64, 256, 1024, 65536};
        for (int c = 1; c < MAP_CLASSES; ++c) m.s[c] = first_of_degree(a.nrp, a.n, lim[c - 1]);
    } else {
        // degrees are not ordered by id: one class (16- or 32-bit) for every id
        for (int c = 1; c < MAP_CLASSES - 1; ++c) m.s[c] = 0;
        m.s[MAP_CLASSES - 1] = a.max_deg >= 65536 ? 0 : n;
    }
    m.o[0] = 0;
    for (int c = 1; c < MAP_CLASSES; ++c)
        m.o[c] = m.o[c - 1] + (uint64_t)(m.s[c] - m.s[c - 1]) * class_words(c - 1, a.L);
    return m;
}

// Heavy tasks: one NT-thread workgroup per task, pulled from a queue.  A
// task is a heavy group restricted to one range of target ids; a group with
// many wedges is split into ranges of about equal adjacency mass (targets are
// met in proportion to their degree), so its work spreads over workgroups and
// each range has every wedge that reaches its targets.  The map is a dense
// uint32 array private to the workgroup, indexed by target, with L counts per
// target sized by the target's degree class (above).  The entries of the
// range are cleared by streaming zeros over its word range when that is
// cheaper than a walk over the wedges; then a count walk and an emit walk.
template <int PASS, int NT>
__global__ void __launch_bounds__(NT) k_cyc_heavy(CycleArgs a) {
    constexpr int HEAVY_THREADS = NT;
    constexpr int HEAVY_CHUNK = NT / 2;
    extern __shared__ uint64_t sm_heavy[];
    const int L = a.L;
    const int LL = L * L;
    const int CH = a.chunk;
    uint64_t *acc = sm_heavy;  // CH * L * L
    // every degree below 2^16: a round's tally of one item (its targets in
    // the task, each count below 2^16) stays below 2^32, so the tallies are
    // 32-bit words in TALLY_COPIES interleaved copies (fewer conflicts)
    uint32_t *acc32 = reinterpret_cast<uint32_t *>(sm_heavy);
    const bool t32 = a.nc_u32 != 0;
    uint32_t *hub_after = reinterpret_cast<uint32_t *>(acc + (size_t)CH * LL * (t32 ? TALLY_COPIES / 2 : 1));
    // hub targets (the top hub_ids ids) are counted in LDS as 16-bit fields
    // per (target, centre type) after the tallies; the rest in the map
    uint32_t *hub = hub_after;
    const int32_t hub_lo = a.hub_ids > 0 ? (int32_t)(a.n - a.hub_ids) : (int32_t)a.n;
    const int hub_words = (a.hub_ids * L + 1) / 2;
    __shared__ int32_t it_tx[HEAVY_CHUNK];  // type of each staged item (the centre)
    __shared__ int64_t it_tb[HEAVY_CHUNK];
    __shared__ uint32_t it_scan[HEAVY_CHUNK];
    __shared__ uint32_t it_eid[HEAVY_CHUNK];
    __shared__ int it_flip[HEAVY_CHUNK];
    __shared__ uint32_t wave_tot[HEAVY_THREADS / WAVE];
    __shared__ int32_t s_task[4];  // group, first target, end target, streamed clear
    __shared__ MapClasses s_mc;
    int tid = threadIdx.x;
    if (input_failed(a.status)) return;
    uint32_t *map = a.maps + (size_t)blockIdx.x * (size_t)a.n * L;
    uint64_t count = a.counters[a.count_idx];
    if (tid == 0) s_mc = map_classes(a);
    __syncthreads();
    while (true) {
        if (tid == 0) {
            uint64_t idx = atomicAdd((unsigned long long *)&a.counters[a.next_idx], 1ull);
            s_task[0] = -1;
            if (idx < count) {
                // groups were queued by increasing id, and the largest groups
                // belong to the highest-ranked nodes: take them first so the
                // longest tasks do not form the tail
                uint4 tk = a.tasks[count - 1 - idx];
                int32_t g = (int32_t)tk.x;
                if (a.blk_flag && a.blk_flag[g]) tk.z = 0;   // counted by the blocked path
                int32_t rb = PASS == 0 ? 0 : g + 1;
                int32_t re = PASS == 0 ? g : (int32_t)a.n;
                int32_t lo = rb, hi = re;
                if (tk.z == 0) {
                    hi = lo;
                    tk.z = 1;
                } else if (tk.z > 1) {
                    lo = range_cut(a.nrp, rb, re, tk.y, tk.z);
                    hi = range_cut(a.nrp, rb, re, tk.y + 1, tk.z);
                }
                const MapClasses mc = s_mc;
                // hub targets live in LDS: only [lo, min(hi, hub_lo)) of the map is used
                const int32_t mhi = hi < hub_lo ? hi : (lo > hub_lo ? lo : hub_lo);
                const uint64_t w0 = map_word(mc, lo, map_class(mc, lo), L);
                const uint64_t w1 = map_word(mc, mhi, map_class(mc, mhi), L);
                uint64_t wt = tk.w / tk.z;
                s_task[0] = g;
                s_task[1] = lo;
                s_task[2] = hi;
                s_task[3] = (w1 - w0) * 4 <= wt * a.clear_bytes ? 1 : 0;
            }
        }
        __syncthreads();
        const int32_t g = s_task[0];
        const int32_t lo = s_task[1], hi = s_task[2];
        const bool streamed = s_task[3] != 0;
        const bool whole = PASS == 0 ? (lo == 0 && hi == g) : (lo == g + 1 && hi == a.n);
        __syncthreads();
        if (g < 0) break;
        int64_t ib, ie;
        item_range<PASS>(a, g, ib, ie);
        const MapClasses mc = s_mc;
        if (hi <= lo) continue;
        if (hub_words > 0 && hi > hub_lo) {
            for (int q = tid; q < hub_words; q += HEAVY_THREADS) hub[q] = 0u;
            __syncthreads();
        }
        if (streamed) {
            const int32_t mhi = hi < hub_lo ? hi : (lo > hub_lo ? lo : hub_lo);
            const uint64_t w0 = map_word(mc, lo, map_class(mc, lo), L);
            uint32_t *p0 = map + w0;
            size_t cnt = (size_t)(map_word(mc, mhi, map_class(mc, mhi), L) - w0);
            size_t head = ((16 - ((uintptr_t)p0 & 15)) & 15) / 4;
            if (head > cnt) head = cnt;
            if ((size_t)tid < head) p0[tid] = 0u;
            uint4 *pv = reinterpret_cast<uint4 *>(p0 + head);
            size_t nv = (cnt - head) / 4;
            for (size_t q = tid; q < nv; q += HEAVY_THREADS) pv[q] = make_uint4(0u, 0u, 0u, 0u);
            size_t done = head + nv * 4;
            if ((size_t)tid < cnt - done) p0[done + tid] = 0u;
            __syncthreads();
        }
        for (int phase = streamed ? 1 : 0; phase < 3; ++phase) {
            for (int64_t cb = ib; cb < ie; cb += CH) {
                int nitems = (int)((ie - cb) < CH ? (ie - cb) : CH);
                uint32_t len = 0;
                if (tid < nitems) {
                    int64_t s = cb + tid;
                    int32_t x = a.ncol[s];
                    uint32_t e = a.neid[s];
                    int64_t tb, te;
                    target_range<PASS>(a, g, x, e, tb, te);
                    if (!whole) {
                        // clip to the task's target range [lo, hi)
                        if (tb < te && a.ncol[tb] < lo) tb = lower_bound(a.ncol, tb, te, lo);
                        if (tb < te && a.ncol[te - 1] >= hi) te = lower_bound(a.ncol, tb, te, hi);
                    }
                    len = (uint32_t)(te > tb ? te - tb : 0);
                    it_tx[tid] = a.ntype[x];
                    it_tb[tid] = tb;
                    it_eid[tid] = e;
                    it_flip[tid] = orient_flip<PASS>(a, g, x, e);
                }
                block_scan_chunk<NT>(len, it_scan, wave_tot);
                uint32_t total = it_scan[nitems - 1];
                if (phase == 2) {
                    const int words = t32 ? nitems * LL * TALLY_COPIES / 2 : nitems * LL;
                    for (int q = tid; q < words; q += HEAVY_THREADS) acc[q] = 0;
                    __syncthreads();
                }
                int o = 0;
                for (uint32_t f = tid; f < total; f += HEAVY_THREADS) {
                    o = owner_next(it_scan, nitems, f, o);
                    uint32_t excl = o ? it_scan[o - 1] : 0;
                    const int tx = it_tx[o];
                    const int64_t ys = it_tb[o] + (f - excl);
                    const int32_t y = a.ncol[ys];
                    if (y >= hub_lo) {
                        // a count never exceeds the target's degree (below
                        // 2^16 whenever hub targets are on)
                        const uint32_t base = (uint32_t)(y - hub_lo) * (uint32_t)L;
                        if (phase == 1) {
                            const uint32_t idx = base + (uint32_t)tx;
                            atomicAdd(&hub[idx >> 1], 1u << ((idx & 1u) * 16u));
                        } else if (phase == 2) {
                            const int ty = a.ctype[ys];
                            uint64_t *ac = acc + (size_t)o * LL;
                            uint32_t *ac32 = acc32 + (size_t)o * LL * TALLY_COPIES + (tid & (TALLY_COPIES - 1));
                            for (int t = 0; t < L; ++t) {
                                const uint32_t idx = base + (uint32_t)t;
                                const uint32_t c = (hub[idx >> 1] >> ((idx & 1u) * 16u)) & 0xffffu;
                                const uint32_t val = c - (t == tx ? 1u : 0u);
                                if (!val) continue;
                                if (t32)
                                    atomicAdd(&ac32[pass_entry<PASS>(t, ty, L) * TALLY_COPIES], val);
                                else
                                    atomicAdd((unsigned long long *)&ac[pass_entry<PASS>(t, ty, L)],
                                              (unsigned long long)val);
                            }
                        }
                        continue;
                    }
                    const int cls = map_class(mc, y);
                    const int bits = class_bits(cls);
                    const int F = 32 / bits;
                    uint32_t *my = map + map_word(mc, y, cls, L);
                    if (phase == 0) {
                        const int ew = class_words(cls, L);
                        for (int q = 0; q < ew; ++q) my[q] = 0u;
                    } else if (phase == 1) {
                        // the map is private to this workgroup: workgroup scope
                        // keeps the update in the XCD's L2
                        __hip_atomic_fetch_add(&my[tx / F], 1u << ((tx % F) * bits),
                                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                    } else {
                        int ty = a.ctype[ys];
                        uint64_t *ac = acc + (size_t)o * LL;
                        uint32_t *ac32 = acc32 + (size_t)o * LL * TALLY_COPIES + (tid & (TALLY_COPIES - 1));
                        // one load per map word (atomic loads are not merged by
                        // the compiler), the counts of its types extracted
                        const uint32_t mask = bits == 32 ? 0xffffffffu : (1u << bits) - 1u;
                        int wq = -1;
                        uint32_t word = 0;
                        for (int t = 0; t < L; ++t) {
                            if (t / F != wq) {
                                wq = t / F;
                                word = __hip_atomic_load(&my[wq], __ATOMIC_RELAXED,
                                                         __HIP_MEMORY_SCOPE_WORKGROUP);
                            }
                            const uint32_t c = (word >> ((t % F) * bits)) & mask;
                            const uint32_t val = c - (t == tx ? 1u : 0u);
                            if (!val) continue;
                            if (t32)
                                atomicAdd(&ac32[pass_entry<PASS>(t, ty, L) * TALLY_COPIES], val);
                            else
                                atomicAdd((unsigned long long *)&ac[pass_entry<PASS>(t, ty, L)],
                                          (unsigned long long)val);
                        }
                    }
                }
                __syncthreads();
                if (phase == 2) {
                    for (int q = tid; q < nitems * LL; q += HEAVY_THREADS) {
                        uint64_t v = 0;
                        if (t32) {
#pragma unroll
                            for (int r = 0; r < TALLY_COPIES; ++r) v += acc32[TALLY_COPIES * q + r];
                        } else {
                            v = acc[q];
                        }
                        if (!v) continue;
                        int o = q / LL;
                        int pq = q - o * LL;
                        int p = pq / L, r = pq - p * L;
                        int canon = it_flip[o] ? r * L + p : pq;
                        nc_add(a, (size_t)it_eid[o] * LL + canon, v);
                    }
                    __syncthreads();
                }
            }
            // all map traffic of a task stays inside this workgroup, so a
            // workgroup barrier orders the clear, count and emit walks
            __syncthreads();
        }
    }
}

// ------------------------------------------------ blocked heavy 4-cycle groups
//
// A large heavy group is counted without a private map per workgroup and
// without global atomics in its count:
//   select  the largest candidate groups whose maps and records fit (the
//           task kernel skips their tasks);
//   setup   per group: items, walk tasks of a fixed wedge count, target
//           blocks (exclusive prefixes over the pass's blocked groups);
//   items   per group: exclusive wedge prefix over its items, so a walk task
//           (a wedge range) finds its first item by binary search;
//   hist    per walk task: wedges per target block (LDS), added to the
//           bucket (group, block) counts and kept as the task's row of a
//           histogram matrix;
//   part    per walk task: that row reserves a run of each bucket, then
//           every wedge writes a 16-bit record (target offset in the
//           block, centre type) into its run (without the matrix the task
//           is walked once more for the row);
//   count   per bucket: the records counted in LDS per (target, centre
//           type), written as the group map's entries of that block (the
//           degree-class layout of the task maps; only reached targets are
//           written, and only reached targets are read);
//   emit    per walk task: every wedge reads its target's entry from the
//           group's map (read-only now, shared by all tasks of the group)
//           and adds the counts to the item's LDS tallies, flushed to NC.
// Every wedge of a blocked group is thus read three times as a target id
// (streaming) and written and read once as a record; the only random
// accesses are the LDS counts and the emit reads of one map per group.

constexpr int BLK_UNROLL = 4;   // wedges per thread and step of the walks
constexpr int BLK_COUNT_THREADS = 512;   // threads of the block-count kernel (measured best of 256, 512, 1024)
constexpr int BLK_EMIT_UNROLL = 4;       // wedges per thread and step of the emit walk
constexpr int BLK_COPIES = 1;   // copies of each item's emit tallies (more copies measured no faster)
constexpr int BLK_HOLD = 2;     // 16-byte record loads a count thread keeps for its second pass

// Largest k < K with start[k] <= t (start[0] = 0 <= t).
__device__ __forceinline__ int blk_find(const uint32_t *start, int K, uint32_t t) {
    int lo = 0, hi = K;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (start[mid] <= t) lo = mid + 1; else hi = mid;
    }
    return lo - 1;
}

// Size bin of a group of w >= 1 wedges: 4 bins per octave (the octave and
// the two bits below its leading one), nondecreasing in w.
__device__ __forceinline__ int blk_bin(uint64_t w) {
    const int e = 63 - __clzll((long long)w);
    const int frac = e >= 2 ? (int)((w >> (e - 2)) & 3u) : (e == 1 ? (int)((w & 1u) << 1) : 0);
    return 4 * e + frac;
}

// Selection of the pass's blocked groups (one workgroup): the packed map
// stride of the degree-class layout sets how many group maps fit the map
// region; the largest size bins are taken from the top while the groups
// fit those slots and their wedges the records; the chosen candidates are
// listed and flagged (the task kernel skips their tasks).
template <int PASS>
__global__ void __launch_bounds__(1024) k_blk_select(CycleArgs a, BlkArgs b) {
    __shared__ int s_bin;
    __shared__ uint32_t s_cnt;
    if (input_failed(a.status)) return;
    const int tid = threadIdx.x;
    if (tid == 0) {
        const MapClasses mc = map_classes(a);
        uint64_t stride = map_word(mc, (int32_t)a.n, map_class(mc, (int32_t)a.n), a.L);
        if (stride < 1) stride = 1;
        uint64_t slots = b.maps_words / stride;
        if (slots > (uint64_t)b.max_groups) slots = (uint64_t)b.max_groups;
        uint64_t cnt = 0, wsum = 0;
        int bin = BLK_BINS;
        for (int q = BLK_BINS - 1; q >= 0; --q) {
            const uint64_t c = b.hist[2 * q], ws = b.hist[2 * q + 1];
            if (!c) continue;
            if (cnt + c > slots || wsum + ws > b.max_wedges) break;
            cnt += c;
            wsum += ws;
            bin = q;
        }
        s_bin = bin;
        s_cnt = 0;
        a.counters[C_BLK_STRIDE] = stride;
    }
    __syncthreads();
    const int bin = s_bin;
    const uint64_t ncand = a.counters[b.c_cand];
    for (uint64_t i = tid; i < ncand; i += 1024) {
        const uint2 e = b.cand[i];
        if (blk_bin(e.y) >= bin) {
            const uint32_t k = atomicAdd(&s_cnt, 1u);
            b.list[k] = e;
            b.flag[e.x] = 1;
        }
    }
    __syncthreads();
    if (tid == 0) a.counters[b.c_count] = s_cnt;
}

// One walk task: the wedges [f0, f1) of blocked group k (group node g).
struct BlkWalk {
    int32_t g;
    int k;
    uint32_t t;            // walk task index
    uint32_t f0, f1;
    uint32_t first;        // item holding wedge f0
    uint32_t ni;           // items of the group
    int64_t ib;            // slot of the first item in g's row
};

// Takes the next walk task from the queue at counters[next]; g < 0 when
// the queue is empty.  Called by one thread.
template <int PASS>
__device__ BlkWalk blk_take(const CycleArgs &a, const BlkArgs &b, int next) {
    BlkWalk w;
    w.g = -1;
    const uint32_t total = (uint32_t)a.counters[C_BLK_TASKS];
    const uint32_t t = (uint32_t)atomicAdd((unsigned long long *)&a.counters[next], 1ull);
    if (t >= total) return w;
    const int K = (int)a.counters[C_BLK_GROUPS];
    const int k = blk_find(b.tstart, K, t);
    const uint2 e = b.list[k];
    w.g = (int32_t)e.x;
    w.k = k;
    w.t = t;
    w.f0 = (t - b.tstart[k]) * b.task;
    w.f1 = e.y - w.f0 < b.task ? e.y : w.f0 + b.task;
    w.ni = b.ioff[k + 1] - b.ioff[k] - 1;
    int64_t ie;
    item_range<PASS>(a, w.g, w.ib, ie);
    // last item whose prefix is at most f0 (items without wedges skipped)
    const uint32_t *pre = b.ipre + b.ioff[k];
    uint32_t lo = 0, hi = w.ni;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (pre[mid] <= w.f0) lo = mid + 1; else hi = mid;
    }
    w.first = lo - 1;
    return w;
}

// Takes the next emit task: from the queue of XCD x + q (mod 8), moving q
// on when that queue is empty (q = 8: every queue is empty).  Called by one
// thread; q lives across calls.
template <int PASS>
__device__ BlkWalk blk_take_emit(const CycleArgs &a, const BlkArgs &b, int x, int &q) {
    BlkWalk w;
    w.g = -1;
    const int K = (int)a.counters[C_BLK_GROUPS];
    const int pitch = b.max_groups / 8 + 1;
    while (q < 8) {
        const int xx = (x + q) & 7;
        const int nx = K > xx ? (K - xx + 7) / 8 : 0;
        const uint32_t *xs = b.xstart + (size_t)xx * pitch;
        const uint32_t total = xs[nx];
        const uint32_t p = total ? (uint32_t)atomicAdd(
                                       (unsigned long long *)&a.counters[C_BLK_NEXT_E + xx], 1ull)
                                 : 0u;
        if (p >= total) {
            ++q;
            continue;
        }
        const int i = blk_find(xs, nx, p);
        const int k = xx + 8 * i;
        const uint2 e = b.list[k];
        w.g = (int32_t)e.x;
        w.k = k;
        w.f0 = (p - xs[i]) * b.task;
        w.f1 = e.y - w.f0 < b.task ? e.y : w.f0 + b.task;
        w.ni = b.ioff[k + 1] - b.ioff[k] - 1;
        int64_t ie;
        item_range<PASS>(a, w.g, w.ib, ie);
        const uint32_t *pre = b.ipre + b.ioff[k];
        uint32_t lo = 0, hi = w.ni;
        while (lo < hi) {
            const uint32_t mid = (lo + hi) >> 1;
            if (pre[mid] <= w.f0) lo = mid + 1; else hi = mid;
        }
        w.first = lo - 1;
        return w;
    }
    return w;
}

// Stages the items first + [0, CH) of a walk task that have wedges before
// f1: per item its first target slot inside the task, its type, edge and
// orientation flip, and the inclusive scan of its target counts inside the
// task in scan[].  Returns how many were staged (the same in every thread).
template <int PASS, int NT>
__device__ int blk_stage(const CycleArgs &a, const BlkArgs &b, const BlkWalk &w, uint32_t first,
                         int CH, int64_t *it_tb, uint32_t *it_scan, int32_t *it_tx,
                         uint32_t *it_eid, int *it_flip, uint32_t *wave_tot) {
    const int tid = threadIdx.x;
    const uint32_t *pre = b.ipre + b.ioff[w.k];
    const uint32_t i = first + (uint32_t)tid;
    const bool ok = tid < CH && i < w.ni && pre[i] < w.f1;
    uint32_t len = 0;
    if (ok) {
        const uint32_t p0 = pre[i], p1 = pre[i + 1];
        const uint32_t lo = p0 > w.f0 ? p0 : w.f0;
        const uint32_t hi = p1 < w.f1 ? p1 : w.f1;
        len = hi > lo ? hi - lo : 0u;
        const int64_t s = w.ib + i;
        const int32_t x = a.ncol[s];
        const uint32_t e = a.neid[s];
        int64_t tb, te;
        target_range<PASS>(a, w.g, x, e, tb, te);
        it_tb[tid] = tb + (lo - p0);
        it_tx[tid] = a.ntype[x];
        it_eid[tid] = e;
        it_flip[tid] = orient_flip<PASS>(a, w.g, x, e);
    }
    const int cnt = __syncthreads_count(ok);
    block_scan_chunk<NT>(len, it_scan, wave_tot);
    return cnt;
}

// Per group: items, walk tasks and blocks, with exclusive prefixes over the
// pass's blocked groups; resets the queues.  One workgroup.
template <int PASS>
__global__ void __launch_bounds__(1024) k_blk_setup(CycleArgs a, BlkArgs b) {
    constexpr int NT = 1024;
    __shared__ uint32_t wt[4][NT / WAVE];
    __shared__ uint32_t carry[4];
    __shared__ unsigned long long s_mtot;
    if (input_failed(a.status)) return;
    const int tid = threadIdx.x, lane = tid & (WAVE - 1), wv = tid / WAVE;
    const uint64_t listed = a.counters[b.c_count];
    const int K = (int)(listed < (uint64_t)b.max_groups ? listed : (uint64_t)b.max_groups);
    if (tid < 4) carry[tid] = 0;
    if (tid == 0) s_mtot = 0;
    __syncthreads();
    uint32_t *out[4] = {b.ioff, b.tstart, b.boff, b.moff};
    for (int c0 = 0; c0 < K; c0 += NT) {
        const int k = c0 + tid;
        uint32_t v[4] = {0u, 0u, 0u, 0u};
        if (k < K) {
            const uint2 e = b.list[k];
            const int32_t g = (int32_t)e.x;
            int64_t ib, ie;
            item_range<PASS>(a, g, ib, ie);
            const int64_t span = PASS == 0 ? (int64_t)g : a.n - 1 - g;
            v[0] = (uint32_t)(ie - ib) + 1u;
            v[1] = (e.y + b.task - 1) / b.task;
            v[2] = (uint32_t)((span + BLK_IDS - 1) >> BLK_SHIFT);
            // histogram-matrix rows: tasks x blocks (saturated; a total
            // beyond the capacity turns the matrix off for the pass)
            const uint64_t mw = (uint64_t)v[1] * v[2];
            v[3] = mw > 0xffffffffull ? 0xffffffffu : (uint32_t)mw;
            atomicAdd(&s_mtot, (unsigned long long)v[3]);
        }
        uint32_t incl[4];
        for (int q = 0; q < 4; ++q) {
            incl[q] = wave_incl_scan(v[q]);
            if (lane == WAVE - 1) wt[q][wv] = incl[q];
        }
        __syncthreads();
        uint32_t add[4];
        for (int q = 0; q < 4; ++q) {
            add[q] = carry[q];
            for (int r = 0; r < wv; ++r) add[q] += wt[q][r];
            if (k < K) out[q][k] = add[q] + incl[q] - v[q];
        }
        __syncthreads();
        if (tid == NT - 1)
            for (int q = 0; q < 4; ++q) carry[q] = add[q] + incl[q];
        __syncthreads();
    }
    if (tid == 0) {
        for (int q = 0; q < 4; ++q) out[q][K] = carry[q];
        a.counters[C_BLK_MAT] = b.mat_cap > 0 && s_mtot <= (unsigned long long)b.mat_cap ? 1u : 0u;
        a.counters[C_BLK_GROUPS] = (uint64_t)K;
        a.counters[C_BLK_TASKS] = carry[1];
        a.counters[C_BLK_BUCKETS] = carry[2];
        a.counters[C_BLK_NEXT_H] = 0;
        a.counters[C_BLK_NEXT_P] = 0;
        a.counters[C_BLK_NEXT_C] = 0;
    }
    // emit queues: XCD x walks the tasks of groups x, x + 8, x + 16, ...
    // (their maps then stay in that XCD's L2); thread x scans them
    __syncthreads();
    if (tid < 8) {
        const int x = tid;
        const int pitch = b.max_groups / 8 + 1;
        uint32_t *xs = b.xstart + (size_t)x * pitch;
        uint32_t acc = 0;
        int i = 0;
        for (int k = x; k < K; k += 8, ++i) {
            xs[i] = acc;
            acc += b.tstart[k + 1] - b.tstart[k];
        }
        xs[i] = acc;
        a.counters[C_BLK_NEXT_E + x] = 0;
    }
}

// Per group: exclusive wedge prefix of its items (their target counts), the
// total checked against the wedge count of the selection; clears the
// group's bucket counts.
template <int PASS>
__global__ void __launch_bounds__(256) k_blk_items(CycleArgs a, BlkArgs b) {
    constexpr int NT = 256;
    __shared__ uint32_t wt[NT / WAVE];
    __shared__ uint32_t s_carry;
    if (input_failed(a.status)) return;
    const int tid = threadIdx.x, lane = tid & (WAVE - 1), wv = tid / WAVE;
    const int K = (int)a.counters[C_BLK_GROUPS];
    for (int k = blockIdx.x; k < K; k += gridDim.x) {
        const uint2 e = b.list[k];
        const int32_t g = (int32_t)e.x;
        int64_t ib, ie;
        item_range<PASS>(a, g, ib, ie);
        const uint32_t ni = (uint32_t)(ie - ib);
        uint32_t *pre = b.ipre + b.ioff[k];
        if (tid == 0) s_carry = 0;
        __syncthreads();
        for (uint32_t c0 = 0; c0 < ni; c0 += NT) {
            const uint32_t i = c0 + (uint32_t)tid;
            uint32_t len = 0;
            if (i < ni) {
                const int64_t s = ib + i;
                int64_t tb, te;
                target_range<PASS>(a, g, a.ncol[s], a.neid[s], tb, te);
                len = te > tb ? (uint32_t)(te - tb) : 0u;
            }
            const uint32_t incl = wave_incl_scan(len);
            if (lane == WAVE - 1) wt[wv] = incl;
            __syncthreads();
            uint32_t add = s_carry;
            for (int r = 0; r < wv; ++r) add += wt[r];
            if (i < ni) pre[i] = add + incl - len;
            __syncthreads();
            if (tid == NT - 1) s_carry = add + incl;
            __syncthreads();
        }
        if (tid == 0) {
            pre[ni] = s_carry;
            if (s_carry != e.y) atomicOr(a.status, ST_INTERNAL);
            atomicAdd((unsigned long long *)&a.counters[PASS == 0 ? C_BLK_A_DONE : C_BLK_B_DONE],
                      (unsigned long long)e.y);
        }
        for (uint32_t j = b.boff[k] + tid; j < b.boff[k + 1]; j += NT) {
            b.bcount[j] = 0;
            b.pcur[j] = 0u;
            b.bgroup[j] = (uint32_t)k;
        }
        __syncthreads();
    }
}

// Adds the task's wedges per target block to hist[] (LDS); with RECORDS,
// writes each wedge's record at the position hist[] holds for its block
// instead (and advances it).
template <int PASS, int NT, bool RECORDS>
__device__ void blk_walk_blocks(const CycleArgs &a, const BlkArgs &b, const BlkWalk &w,
                                uint32_t *hist, int64_t *it_tb, uint32_t *it_scan, int32_t *it_tx,
                                uint32_t *it_eid, int *it_flip, uint32_t *wave_tot) {
    constexpr int CH = NT / 2;
    const int tid = threadIdx.x;
    const int lane = tid & (WAVE - 1);
    const int32_t rbase = PASS == 0 ? 0 : w.g + 1;
    for (uint32_t first = w.first;; first += CH) {
        const int cnt = blk_stage<PASS, NT>(a, b, w, first, CH, it_tb, it_scan, it_tx, it_eid,
                                            it_flip, wave_tot);
        if (cnt == 0) break;
        const uint32_t total = it_scan[cnt - 1];
        int o = 0;
        // BLK_UNROLL wedges per thread and step: their target loads are
        // issued together
        for (uint32_t f0 = tid; f0 < total; f0 += NT * BLK_UNROLL) {
            int32_t y[BLK_UNROLL];
            int ow[BLK_UNROLL];
#pragma unroll
            for (int u = 0; u < BLK_UNROLL; ++u) {
                const uint32_t f = f0 + (uint32_t)u * NT;
                ow[u] = -1;
                if (f < total) {
                    o = owner_next(it_scan, cnt, f, o);
                    const uint32_t excl = o ? it_scan[o - 1] : 0u;
                    ow[u] = o;
                    y[u] = a.ncol[it_tb[o] + (f - excl)];
                }
            }
#pragma unroll
            for (int u = 0; u < BLK_UNROLL; ++u) {
                // the lanes of a wave hold consecutive wedges, mostly of one
                // item with ascending targets: runs of lanes share a block,
                // and the first lane of each run counts the whole run (one
                // LDS atomic per run instead of one per wedge)
                const bool act = ow[u] >= 0;
                const uint32_t rel = act ? (uint32_t)(y[u] - rbase) : 0u;
                const int key = act ? (int)(rel >> BLK_SHIFT) : -1;
                const int prev = __shfl_up(key, 1, WAVE);
                const bool lead = act && (lane == 0 || prev != key);
                const uint64_t leads = __ballot(lead);
                const uint64_t acts = __ballot(act);
                const int nact = __popcll(acts);   // active lanes are a prefix
                const uint64_t above = lane == WAVE - 1 ? 0ull : leads >> (lane + 1);
                const int run = above ? __ffsll((long long)above) : nact - lane;
                const int head = WAVE - 1 - __clzll((long long)(leads & ((2ull << lane) - 1ull)));
                if (RECORDS) {
                    uint32_t pos = 0;
                    if (lead) pos = atomicAdd(&hist[key], (uint32_t)run);
                    pos = (uint32_t)__shfl((int)pos, act ? head : lane, WAVE) + (uint32_t)(lane - head);
                    if (act)
                        b.rec[pos] = (uint16_t)((rel & (BLK_IDS - 1)) |
                                                ((uint32_t)it_tx[ow[u]] << BLK_SHIFT));
                } else if (lead) {
                    atomicAdd(&hist[key], (uint32_t)run);
                }
            }
        }
        __syncthreads();
        if (cnt < CH) break;
    }
}

// Bucket counts: one walk task at a time, wedges per block in LDS, then
// added to the group's bucket counts.
template <int PASS, int NT>
__global__ void __launch_bounds__(NT) k_blk_hist(CycleArgs a, BlkArgs b) {
    extern __shared__ uint32_t sm_hist[];  // nb_max counts
    constexpr int CH = NT / 2;
    __shared__ int64_t it_tb[CH];
    __shared__ uint32_t it_scan[CH];
    __shared__ int32_t it_tx[CH];
    __shared__ uint32_t it_eid[CH];
    __shared__ int it_flip[CH];
    __shared__ uint32_t wave_tot[NT / WAVE];
    __shared__ BlkWalk s_w;
    if (input_failed(a.status)) return;
    const int tid = threadIdx.x;
    const bool mat_on = a.counters[C_BLK_MAT] != 0;
    while (true) {
        if (tid == 0) s_w = blk_take<PASS>(a, b, C_BLK_NEXT_H);
        __syncthreads();
        const BlkWalk w = s_w;
        if (w.g < 0) break;
        const uint32_t b0 = b.boff[w.k], nb = b.boff[w.k + 1] - b0;
        for (uint32_t j = tid; j < nb; j += NT) sm_hist[j] = 0u;
        __syncthreads();
        blk_walk_blocks<PASS, NT, false>(a, b, w, sm_hist, it_tb, it_scan, it_tx, it_eid, it_flip,
                                         wave_tot);
        uint32_t *row = mat_on ? b.mat + b.moff[w.k] + (size_t)(w.t - b.tstart[w.k]) * nb : nullptr;
        for (uint32_t j = tid; j < nb; j += NT) {
            const uint32_t c = sm_hist[j];
            if (row) row[j] = c;
            if (c) atomicAdd((unsigned long long *)&b.bcount[b0 + j], (unsigned long long)c);
        }
        __syncthreads();
    }
}

// Record partition: one walk task at a time; its wedges per block reserve
// a run of each bucket, then every wedge writes its record into the run.
template <int PASS, int NT>
__global__ void __launch_bounds__(NT) k_blk_part(CycleArgs a, BlkArgs b) {
    extern __shared__ uint32_t sm_hist[];  // nb_max counts, then record positions
    constexpr int CH = NT / 2;
    __shared__ int64_t it_tb[CH];
    __shared__ uint32_t it_scan[CH];
    __shared__ int32_t it_tx[CH];
    __shared__ uint32_t it_eid[CH];
    __shared__ int it_flip[CH];
    __shared__ uint32_t wave_tot[NT / WAVE];
    __shared__ BlkWalk s_w;
    if (input_failed(a.status)) return;
    const int tid = threadIdx.x;
    const bool mat_on = a.counters[C_BLK_MAT] != 0;
    while (true) {
        if (tid == 0) s_w = blk_take<PASS>(a, b, C_BLK_NEXT_P);
        __syncthreads();
        const BlkWalk w = s_w;
        if (w.g < 0) break;
        const uint32_t b0 = b.boff[w.k], nb = b.boff[w.k + 1] - b0;
        if (mat_on) {
            // the histogram kernel left this task's row of block counts
            const uint32_t *row = b.mat + b.moff[w.k] + (size_t)(w.t - b.tstart[w.k]) * nb;
            for (uint32_t j = tid; j < nb; j += NT) sm_hist[j] = row[j];
            __syncthreads();
        } else {
            for (uint32_t j = tid; j < nb; j += NT) sm_hist[j] = 0u;
            __syncthreads();
            blk_walk_blocks<PASS, NT, false>(a, b, w, sm_hist, it_tb, it_scan, it_tx, it_eid,
                                             it_flip, wave_tot);
        }
        for (uint32_t j = tid; j < nb; j += NT) {
            const uint32_t c = sm_hist[j];
            if (c)
                sm_hist[j] = (uint32_t)b.bstart[b0 + j] + atomicAdd(&b.pcur[b0 + j], c);
        }
        __syncthreads();
        blk_walk_blocks<PASS, NT, true>(a, b, w, sm_hist, it_tb, it_scan, it_tx, it_eid, it_flip,
                                        wave_tot);
    }
}

// Block counts: one bucket (group, block) at a time; its records counted in
// LDS as 16-bit fields per (target, centre type) (a count never exceeds the
// target's degree, below 2^16 on this path); then a second pass over the
// records lets the first record of each target (a claim bit) write the
// target's entry to the group's map in the degree-class layout and clear
// its fields, so the counts are zero again for the next bucket.  Only
// reached targets are written, and only reached targets are read.
template <int PASS>
__global__ void __launch_bounds__(BLK_COUNT_THREADS) k_blk_count(CycleArgs a, BlkArgs b) {
    constexpr int NT = BLK_COUNT_THREADS;
    extern __shared__ uint32_t sm_cnt[];  // BLK_IDS * L 16-bit fields, then BLK_IDS claim bits
    __shared__ int s_k;
    __shared__ uint32_t s_j;
    __shared__ int64_t s_r[2];
    __shared__ MapClasses s_mc;
    if (input_failed(a.status)) return;
    const int tid = threadIdx.x;
    const int L = a.L;
    const uint32_t total = (uint32_t)a.counters[C_BLK_BUCKETS];
    const size_t stride = (size_t)a.counters[C_BLK_STRIDE];
    const int words = (BLK_IDS * L + 1) / 2;
    uint32_t *claim = sm_cnt + words;
    for (int q = tid; q < words + BLK_IDS / 32; q += NT) sm_cnt[q] = 0u;
    if (tid == 0) s_mc = map_classes(a);
    __syncthreads();
    const MapClasses mc = s_mc;
    // thread 0 takes the next bucket while the workgroup counts the current
    // one (the queue position is only read at the next step)
    uint32_t next = 0;
    if (tid == 0) next = (uint32_t)atomicAdd((unsigned long long *)&a.counters[C_BLK_NEXT_C], 1ull);
    while (true) {
        if (tid == 0) {
            // empty buckets are passed over here, without a barrier
            uint32_t j = next;
            int64_t r0 = 0, r1 = 0;
            while (j < total) {
                r0 = b.bstart[j];
                r1 = b.bstart[j + 1];
                if (r1 != r0) break;
                j = (uint32_t)atomicAdd((unsigned long long *)&a.counters[C_BLK_NEXT_C], 1ull);
            }
            s_j = j;
            s_k = j < total ? (int)b.bgroup[j] : -1;
            s_r[0] = r0;
            s_r[1] = r1;
            if (j < total)
                next = (uint32_t)atomicAdd((unsigned long long *)&a.counters[C_BLK_NEXT_C], 1ull);
        }
        __syncthreads();
        const uint32_t j = s_j;
        const int k = s_k;
        if (k < 0) break;
        const int64_t r0 = s_r[0], r1 = s_r[1];
        // records 8 at a time (16-byte loads of the 16-byte aligned runs
        // covering [r0, r1); the record region is padded to 256 bytes); a
        // bucket of at most NT * 8 * BLK_HOLD records stays in registers
        // for the second pass
        const int64_t v0 = r0 >> 3, v1 = (r1 + 7) >> 3;
        const uint4 *rv = reinterpret_cast<const uint4 *>(b.rec);
        const bool hold = v1 - v0 <= (int64_t)NT * BLK_HOLD;
        uint4 held[BLK_HOLD];
#pragma unroll
        for (int h = 0; h < BLK_HOLD; ++h) held[h] = make_uint4(0u, 0u, 0u, 0u);
        for (int64_t v = v0 + tid, h = 0; v < v1; v += NT, ++h) {
            const uint4 q = rv[v];
            if (hold) {
#pragma unroll
                for (int hh = 0; hh < BLK_HOLD; ++hh)
                    if (hh == h) held[hh] = q;
            }
            const uint32_t wv[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int64_t r = v * 8 + e;
                if (r < r0 || r >= r1) continue;
                const uint32_t rc = (wv[e >> 1] >> ((e & 1) * 16)) & 0xffffu;
                const uint32_t idx = (rc & (BLK_IDS - 1)) * (uint32_t)L + (rc >> BLK_SHIFT);
                atomicAdd(&sm_cnt[idx >> 1], 1u << ((idx & 1u) * 16u));
            }
        }
        __syncthreads();
        const int32_t g = (int32_t)b.list[k].x;
        const int64_t rbase = PASS == 0 ? 0 : (int64_t)g + 1;
        const int64_t id0 = rbase + (int64_t)(j - b.boff[k]) * BLK_IDS;
        uint32_t *map = a.maps + (size_t)k * stride;
        for (int64_t v = v0 + tid, h = 0; v < v1; v += NT, ++h) {
          uint4 q;
          if (hold) {
              q = held[0];
#pragma unroll
              for (int hh = 1; hh < BLK_HOLD; ++hh)
                  if (hh == h) q = held[hh];
          } else {
              q = rv[v];
          }
          const uint32_t wv[4] = {q.x, q.y, q.z, q.w};
          for (int e = 0; e < 8; ++e) {
            const int64_t r = v * 8 + e;
            if (r < r0 || r >= r1) continue;
            const uint32_t off = ((wv[e >> 1] >> ((e & 1) * 16)) & 0xffffu) & (BLK_IDS - 1);
            // claim bit of target off: word off % 128, bit off / 128, so
            // that consecutive targets (dense hub blocks) use different banks
            const uint32_t bit = 1u << (off >> 7);
            if (atomicOr(&claim[off & (BLK_IDS / 32 - 1)], bit) & bit) continue;
            const int32_t wid = (int32_t)(id0 + off);
            const uint32_t base = off * (uint32_t)L;
            const int cls = map_class(mc, wid);
            const int bits = class_bits(cls);
            const int F = 32 / bits;
            uint32_t *my = map + map_word(mc, wid, cls, L);
            for (int q = 0; q * F < L; ++q) {
                uint32_t word = 0;
                for (int t = q * F; t < L && t < (q + 1) * F; ++t) {
                    const uint32_t idx = base + t;
                    const uint32_t sh = (idx & 1u) * 16u;
                    const uint32_t c = (sm_cnt[idx >> 1] >> sh) & 0xffffu;
                    word |= c << ((t - q * F) * bits);
                    // this target's fields belong to this thread now
                    atomicAnd(&sm_cnt[idx >> 1], ~(0xffffu << sh));
                }
                my[q] = word;
            }
          }
        }
        __syncthreads();
        for (int q = tid; q < BLK_IDS / 32; q += NT) claim[q] = 0u;
        __syncthreads();
    }
}

// Emit walk: one walk task at a time; each wedge reads its target's entry
// from the group's map and adds count - [same type as the centre] to the
// item's 32-bit tallies in LDS (a task has at most BLK_TASK wedges of
// counts below 2^16), flushed to NC after each staging round.
template <int PASS, int NT>
__global__ void __launch_bounds__(NT) k_blk_emit(CycleArgs a, BlkArgs b) {
    extern __shared__ uint32_t sm_acc[];  // emit_chunk * L * L tallies
    constexpr int CHMAX = NT / 2;
    __shared__ int64_t it_tb[CHMAX];
    __shared__ uint32_t it_scan[CHMAX];
    __shared__ int32_t it_tx[CHMAX];
    __shared__ uint32_t it_eid[CHMAX];
    __shared__ int it_flip[CHMAX];
    __shared__ uint32_t wave_tot[NT / WAVE];
    __shared__ BlkWalk s_w;
    __shared__ MapClasses s_mc;
    if (input_failed(a.status)) return;
    const int tid = threadIdx.x;
    const int L = a.L, LL = L * L;
    const int CH = b.emit_chunk;
    const size_t stride = (size_t)a.counters[C_BLK_STRIDE];
    // workgroups are dispatched to the eight XCDs in turn
    const int xcd = (int)(blockIdx.x & 7u);
    int q = 0;   // thread 0's queue position
    if (tid == 0) s_mc = map_classes(a);
    __syncthreads();
    const MapClasses mc = s_mc;
    while (true) {
        if (tid == 0) s_w = blk_take_emit<PASS>(a, b, xcd, q);
        __syncthreads();
        const BlkWalk w = s_w;
        if (w.g < 0) break;
        const uint32_t *map = a.maps + (size_t)w.k * stride;
        for (uint32_t first = w.first;; first += CH) {
            const int cnt = blk_stage<PASS, NT>(a, b, w, first, CH, it_tb, it_scan, it_tx, it_eid,
                                                it_flip, wave_tot);
            if (cnt == 0) break;
            for (int q = tid; q < cnt * LL * BLK_COPIES; q += NT) sm_acc[q] = 0u;
            __syncthreads();
            const uint32_t total = it_scan[cnt - 1];
            int o = 0;
            // BLK_EMIT_UNROLL wedges per thread and step: target loads issued
            // together, then the first map word of each target together
            for (uint32_t f0 = tid; f0 < total; f0 += NT * BLK_EMIT_UNROLL) {
                int ow[BLK_EMIT_UNROLL], ty[BLK_EMIT_UNROLL];
                int32_t y[BLK_EMIT_UNROLL];
                uint32_t w0[BLK_EMIT_UNROLL];
#pragma unroll
                for (int u = 0; u < BLK_EMIT_UNROLL; ++u) {
                    const uint32_t f = f0 + (uint32_t)u * NT;
                    ow[u] = -1;
                    if (f < total) {
                        o = owner_next(it_scan, cnt, f, o);
                        const uint32_t excl = o ? it_scan[o - 1] : 0u;
                        ow[u] = o;
                        const int64_t ys = it_tb[o] + (f - excl);
                        y[u] = a.ncol[ys];
                        ty[u] = a.ctype[ys];
                    }
                }
#pragma unroll
                for (int u = 0; u < BLK_EMIT_UNROLL; ++u) {
                    if (ow[u] < 0) continue;
                    w0[u] = map[map_word(mc, y[u], map_class(mc, y[u]), L)];
                }
#pragma unroll
                for (int u = 0; u < BLK_EMIT_UNROLL; ++u) {
                    if (ow[u] < 0) continue;
                    const int tx = it_tx[ow[u]];
                    const int cls = map_class(mc, y[u]);
                    const int bits = class_bits(cls);
                    const int F = 32 / bits;
                    const uint32_t mask = bits == 32 ? 0xffffffffu : (1u << bits) - 1u;
                    // BLK_COPIES interleaved copies of each item's tallies:
                    // lanes of one item and target type spread over banks
                    uint32_t *ac = sm_acc + (size_t)ow[u] * LL * BLK_COPIES + (tid & (BLK_COPIES - 1));
                    int wq = 0;
                    uint32_t word = w0[u];
                    for (int t = 0; t < L; ++t) {
                        if (t / F != wq) {
                            wq = t / F;
                            word = map[map_word(mc, y[u], cls, L) + wq];
                        }
                        const uint32_t c = (word >> ((t % F) * bits)) & mask;
                        const uint32_t val = c - (t == tx ? 1u : 0u);
                        if (val) atomicAdd(&ac[pass_entry<PASS>(t, ty[u], L) * BLK_COPIES], val);
                    }
                }
            }
            __syncthreads();
            for (int q = tid; q < cnt * LL; q += NT) {
                uint32_t v = 0;
#pragma unroll
                for (int r = 0; r < BLK_COPIES; ++r) v += sm_acc[q * BLK_COPIES + r];
                if (!v) continue;
                const int oo = q / LL;
                const int pq = q - oo * LL;
                const int p = pq / L, r = pq - p * L;
                const int canon = it_flip[oo] ? r * L + p : pq;
                nc_add(a, (size_t)it_eid[oo] * LL + canon, v);
            }
            __syncthreads();
            if (cnt < CH) break;
        }
    }
}

// Bytes of one target's map entry assumed by the id-range splits (the
// 16-bit class; targets of smaller degree take less, of degree >= 2^16 more).
__device__ __forceinline__ uint64_t map_bytes_per_id(int L) { return (uint64_t)((L + 1) / 2) * 4; }

// Wave-wide list appends of the groups found by the lanes of a wave (one
// counter update per wave and list).  Every lane of the wave calls this with
// its own node v and wedge count w (0: no group).  Light groups go to
// `light`; a heavy group gets one queue entry per target range, the splits
// beyond one entry per group drawing on a shared budget of extra slots (a
// wave whose splits do not fit keeps its groups whole).
__device__ void push_groups(int32_t v, uint64_t w, uint32_t *light, uint4 *heavy,
                            uint64_t *counters, int c_light, int c_heavy, int c_wedges,
                            int c_wedges_heavy, uint64_t task_wedges, int64_t range_ids,
                            uint64_t map_bytes_per_id, uint64_t range_bytes, uint64_t light_max,
                            uint2 *cand, uint64_t *chist, int c_cand, uint64_t cand_min) {
    const int lane = lane_id();
    const uint64_t below = (1ull << lane) - 1ull;
    const bool is_light = w && w <= light_max;
    const bool is_heavy = w > light_max;
    // candidates of the blocked path (a node is one group per pass, so the
    // list holds at most n entries); the selection takes the largest later
    if (cand && is_heavy && w >= cand_min && w < (1ull << 31)) {
        const uint64_t k = atomicAdd((unsigned long long *)&counters[c_cand], 1ull);
        cand[k] = make_uint2((uint32_t)v, (uint32_t)w);
        const int bin = blk_bin(w);
        atomicAdd((unsigned long long *)&chist[2 * bin], 1ull);
        atomicAdd((unsigned long long *)&chist[2 * bin + 1], (unsigned long long)w);
    }
    uint64_t bl = __ballot(is_light);
    if (bl) {
        uint64_t base = 0;
        if (lane == 0)
            base = atomicAdd((unsigned long long *)&counters[c_light], (unsigned long long)__popcll(bl));
        base = __shfl(base, 0, WAVE);
        if (is_light) light[base + __popcll(bl & below)] = (uint32_t)v;
    }
    uint64_t tot = wave_sum_u64(w);
    uint64_t tot_heavy = wave_sum_u64(is_heavy ? w : 0ull);
    if (lane == 0 && tot) atomicAdd((unsigned long long *)&counters[c_wedges], (unsigned long long)tot);
    uint64_t bh = __ballot(is_heavy);
    if (!bh) return;
    if (lane == 0) {
        atomicAdd((unsigned long long *)&counters[c_wedges_heavy], (unsigned long long)tot_heavy);
        atomicAdd((unsigned long long *)&counters[C_HEAVY_GROUPS], (unsigned long long)__popcll(bh));
    }
    uint32_t parts = 0;
    if (is_heavy) {
        uint64_t q = (w + task_wedges - 1) / task_wedges;
        // a group with at least one wedge per target id reuses map lines:
        // split its id range so one task's map entries stay within
        // range_bytes (and so in cache between its count and emit walks)
        if (range_bytes && range_ids > 0 && w >= (uint64_t)range_ids) {
            uint64_t rb = ((uint64_t)range_ids * map_bytes_per_id + range_bytes - 1) / range_bytes;
            if (rb > q) q = rb;
        }
        parts = (uint32_t)(q > (uint64_t)TASK_MAX_PARTS ? TASK_MAX_PARTS : q);
    }
    uint32_t extra = wave_incl_scan(parts ? parts - 1 : 0u);
    uint32_t extra_tot = __shfl(extra, WAVE - 1, WAVE);
    if (extra_tot) {
        int ok = 1;
        if (lane == 0) {
            uint64_t old = atomicAdd((unsigned long long *)&counters[C_TASK_EXTRA],
                                     (unsigned long long)extra_tot);
            ok = old + extra_tot <= (uint64_t)TASK_EXTRA;
        }
        if (!__shfl(ok, 0, WAVE) && parts) parts = 1;
    }
    uint32_t incl = wave_incl_scan(parts);
    uint32_t all = __shfl(incl, WAVE - 1, WAVE);
    uint64_t base = 0;
    if (lane == 0) base = atomicAdd((unsigned long long *)&counters[c_heavy], (unsigned long long)all);
    base = __shfl(base, 0, WAVE) + (incl - parts);
    uint32_t wc = w > 0xffffffffull ? 0xffffffffu : (uint32_t)w;
    for (uint32_t k = 0; k < parts; ++k) heavy[base + k] = make_uint4((uint32_t)v, k, parts, wc);
}

// Wedges of node v in both passes from its own row: for a neighbour x below
// v, v's slot in x's row splits x's row into pass-A targets (below v) and
// pass-B targets (above v); for x above v, pass B takes x's neighbours above
// x (x's split point).
__device__ __forceinline__ void node_wedges(const int64_t *__restrict__ nrp,
                                            const int32_t *__restrict__ ncol,
                                            const uint32_t *__restrict__ neid,
                                            const uint32_t *__restrict__ eslot,
                                            const uint32_t *__restrict__ nlow, int32_t v, int64_t s,
                                            uint64_t &wa, uint64_t &wb) {
    int32_t x = ncol[s];
    int64_t xb = nrp[x], xe = nrp[x + 1];
    if (x < v) {
        int64_t r = (int64_t)eslot[2 * (size_t)neid[s] + 0];
        wa += (uint64_t)(r - xb);
        wb += (uint64_t)(xe - r - 1);
    } else {
        wb += (uint64_t)(xe - xb - nlow[x]);
    }
}

// Wedge counts of both passes per node, bucketed into light and heavy lists.
// Node ids are ranked by degree, so nodes below the first one of degree >=
// 64 are taken one per lane (64 nodes of similar degree per wave) and the
// rest one per wave.
__global__ void __launch_bounds__(256) k_cyc_work(
    const int64_t *__restrict__ nrp, const int32_t *__restrict__ ncol,
    const uint32_t *__restrict__ neid, const uint32_t *__restrict__ eslot,
    const uint32_t *__restrict__ nlow, int64_t n, uint32_t *__restrict__ listA_light,
    uint4 *__restrict__ listA_heavy, uint32_t *__restrict__ listB_light,
    uint4 *__restrict__ listB_heavy, uint64_t *__restrict__ counters, uint64_t task_wedges,
    int L, uint64_t range_bytes, uint64_t light_max, BlkSelect bs,
    const uint32_t *__restrict__ status) {
    if (input_failed(status)) return;
    __shared__ int64_t s_thr;
    if (threadIdx.x == 0) {
        int64_t lo = 0, hi = n;
        while (lo < hi) {
            int64_t mid = (lo + hi) >> 1;
            if (nrp[mid + 1] - nrp[mid] < WAVE) lo = mid + 1; else hi = mid;
        }
        s_thr = lo;
    }
    __syncthreads();
    const int64_t thr = s_thr;
    const int lane = lane_id();
    const int64_t wid = (int64_t)blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE;
    const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x / WAVE);
    const int64_t chunks = (thr + WAVE - 1) / WAVE;
    for (int64_t c = wid; c < chunks; c += nwaves) {
        const int64_t v = c * WAVE + lane;
        uint64_t wa = 0, wb = 0;
        if (v < thr)
            for (int64_t s = nrp[v]; s < nrp[v + 1]; ++s)
                node_wedges(nrp, ncol, neid, eslot, nlow, (int32_t)v, s, wa, wb);
        push_groups((int32_t)v, wa, listA_light, listA_heavy, counters, C_A_LIGHT, C_A_HEAVY,
                    C_WEDGES_A, C_WEDGES_A_HEAVY, task_wedges, v,
                    map_bytes_per_id(L), range_bytes, light_max, bs.cand_a, bs.hist_a, C_BLK_CAND_A,
                    bs.min_wedges_a);
        push_groups((int32_t)v, wb, listB_light, listB_heavy, counters, C_B_LIGHT, C_B_HEAVY,
                    C_WEDGES_B, C_WEDGES_B_HEAVY, task_wedges, n - 1 - v,
                    map_bytes_per_id(L), range_bytes, light_max, bs.cand_b, bs.hist_b, C_BLK_CAND_B,
                    bs.min_wedges_b);
    }
    for (int64_t v = thr + wid; v < n; v += nwaves) {
        uint64_t wa = 0, wb = 0;
        for (int64_t s = nrp[v] + lane; s < nrp[v + 1]; s += WAVE)
            node_wedges(nrp, ncol, neid, eslot, nlow, (int32_t)v, s, wa, wb);
        wa = wave_sum_u64(wa);
        wb = wave_sum_u64(wb);
        push_groups((int32_t)v, lane == 0 ? wa : 0ull, listA_light, listA_heavy, counters,
                    C_A_LIGHT, C_A_HEAVY, C_WEDGES_A, C_WEDGES_A_HEAVY, task_wedges, v,
                    map_bytes_per_id(L), range_bytes, light_max, bs.cand_a, bs.hist_a, C_BLK_CAND_A,
                    bs.min_wedges_a);
        push_groups((int32_t)v, lane == 0 ? wb : 0ull, listB_light, listB_heavy, counters,
                    C_B_LIGHT, C_B_HEAVY, C_WEDGES_B, C_WEDGES_B_HEAVY, task_wedges, n - 1 - v,
                    map_bytes_per_id(L), range_bytes, light_max, bs.cand_b, bs.hist_b, C_BLK_CAND_B,
                    bs.min_wedges_b);
    }
}

// Global counts: divide each graphlet block by its edge count.
__global__ void k_global_finalize(const uint64_t *__restrict__ gacc, int L,
                                  uint64_t *__restrict__ out, uint32_t *__restrict__ status) {
    if (input_failed(status)) return;
    int q = blockIdx.x * blockDim.x + threadIdx.x;
    int n2 = (int)binom_small(L + 1, 2), n3 = (int)binom_small(L + 2, 3),
        n4 = (int)binom_small(L + 3, 4);
    int gw = n2 + 2 * n3 + 6 * n4;
    if (q >= gw) return;
    int h;
    if (q < n2) h = 0;
    else if (q < n2 + n3) h = 1;
    else if (q < n2 + 2 * n3) h = 2;
    else h = 3 + (q - n2 - 2 * n3) / n4;
    const uint64_t E[9] = {1, 2, 3, 3, 3, 4, 4, 5, 6};
    uint64_t v = gacc[q];
    if (v % E[h]) atomicOr(status, ST_NOT_DIVISIBLE);
    out[q] = v / E[h];
}

// The number of entries above the diagonal must be half the adjacency (a
// symmetric graph); otherwise the edge numbering would leave [0, m).
__global__ void k_check_edge_count(const int64_t *__restrict__ eoff, int64_t n, int64_t m,
                                   uint32_t *__restrict__ status) {
    if (input_failed(status)) return;
    if (eoff[n] != m) atomicOr(status, ST_EDGE_COUNT);
}

// The call's status code from the status bits (the same mapping as the
// host side's), for calls that never read the status back themselves.
__global__ void k_status_code(const uint32_t *__restrict__ status, int32_t *__restrict__ out) {
    const uint32_t b = *status;
    tg_status s = TG_OK;
    if (b & (ST_BATCH | ST_CROSS_GRAPH)) s = TG_E_BATCH;
    else if (b & ST_TYPE_RANGE) s = TG_E_TYPE_RANGE;
    else if (b & (ST_COL_RANGE | ST_UNSORTED | ST_SELF_LOOP | ST_ASYMMETRIC | ST_EDGE_COUNT))
        s = TG_E_NOT_SIMPLE;
    else if (b) s = TG_E_INTERNAL;
    *out = (int32_t)s;
}

// ------------------------------------------------------ launch wrappers

#define LAUNCH_CHECK() do { hipError_t e_ = hipGetLastError(); if (e_ != hipSuccess) return e_; } while (0)

static inline unsigned blocks_for(int64_t items, int per_block) {
    return (unsigned)((items + per_block - 1) / per_block);
}

// Blocks for a grid-stride kernel: enough to fill the device, no more (per
// item work that is small leaves the workgroup dispatcher as the limit
// when every few items get a workgroup of their own).
static inline unsigned blocks_bounded(int64_t items, int per_block, int per_cu) {
    unsigned b = blocks_for(items, per_block);
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
        cus > 0 && b > (unsigned)cus * per_cu)
        b = (unsigned)cus * per_cu;
    return b > 0 ? b : 1;
}

hipError_t launch_fill_u64(uint64_t *p, uint64_t v, int64_t count, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    int64_t b = (count + 255) / 256;
    if (b > 4096) b = 4096;
    k_fill_u64<<<(unsigned)b, 256, 0, st>>>(p, v, count);
    LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_check_rows(const int64_t *rp, const int32_t *col, const uint8_t *types, int64_t n,
                             int64_t nnz, int L, uint32_t *deg, int64_t *ucount, uint32_t *status,
                             const int32_t *node_graph, const int32_t *gL, hipStream_t st) {
    k_check_rows<<<blocks_bounded(n > 0 ? n : 1, 4, 32), 256, 0, st>>>(rp, col, types, n, nnz, L, deg, ucount, status,
                                                       node_graph, gL);
    LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_check_edge_count(const int64_t *eoff, int64_t n, int64_t m, uint32_t *status,
                                   hipStream_t st) {
    k_check_edge_count<<<1, 1, 0, st>>>(eoff, n, m, status);
    LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_status_code(const uint32_t *status, int32_t *out, hipStream_t st) {
    k_status_code<<<1, 1, 0, st>>>(status, out);
    LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_node_keys(const uint32_t *deg, int64_t n, const int32_t *node_graph, int deg_bits,
                            uint64_t *keys, uint32_t *ids, const uint32_t *status, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    k_node_keys<<<blocks_for(n, 256), 256, 0, st>>>(deg, n, node_graph, deg_bits, keys, ids, status);
    LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_relabel(const uint32_t *sorted_ids, const uint8_t *types, const uint32_t *deg,
                          int64_t n, int32_t *order, int32_t *newid, uint8_t *ntype, int64_t *ndeg,
                          uint64_t *hub_cand, uint32_t sh_deg, const int32_t *node_graph,
                          int32_t *ngraph, const uint32_t *status, hipStream_t st) {
    k_relabel<<<blocks_for(n > 0 ? n : 1, 256), 256, 0, st>>>(sorted_ids, types, deg, n, order,
                                                              newid, ntype, ndeg, hub_cand, sh_deg,
                                                              node_graph, ngraph, status);
    LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_slot_keys(const int64_t *rp, const int32_t *col, const int64_t *ucount,
                            const int64_t *eoff, const int32_t *newid, int64_t n, int bits,
                            uint64_t *keys, uint32_t *vals, int32_t *ei, int32_t *ej,
                            uint32_t *status, hipStream_t st) {
    k_slot_keys<<<blocks_bounded(n, 4, 32), 256, 0, st>>>(rp, col, ucount, eoff, newid, n, bits, keys, vals,
                                                  ei, ej, status);
    LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_finish_csr(const uint64_t *keys, const uint32_t *vals, int64_t nnz, int bits,
                             const uint8_t *ntype, uint32_t *eslot, int32_t *ncol, uint32_t *neid,
                             uint8_t *ctype, const uint32_t *status, hipStream_t st) {
    if (nnz == 0) return hipSuccess;
    k_finish_csr<<<blocks_for(nnz, 256), 256, 0, st>>>(keys, vals, nnz, bits, ntype, eslot, ncol,
                                                       neid, ctype, status);
    LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_tdeg(const int64_t *nrp, const int32_t *ncol, const uint8_t *ctype, int64_t n,
                       int L, int32_t hub_base, uint32_t *tdeg, int64_t *hstart, uint32_t *nlow,
                       const uint32_t *status, hipStream_t st) {
    k_tdeg<<<blocks_bounded(n, 4, 32), 256, 0, st>>>(nrp, ncol, ctype, n, L, hub_base, tdeg,
                                                     hstart, nlow, status);
    LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_tri(const int64_t *nrp, const int32_t *ncol, const uint8_t *ctype,
                      const int32_t *ei, const int32_t *ej, const uint32_t *eslot,
                      uint32_t *tri_slot, int64_t m, int L, uint32_t *tri,
                      uint64_t *tri_sum, int32_t sh_base, int64_t nw, const uint64_t *SB,
                      int32_t hub_base, int Hw, const uint64_t *HB, const uint32_t *status,
                      hipStream_t st) {
    if (m == 0) return hipSuccess;
    k_tri<<<blocks_bounded(m, 4 * TRI_GROUPS, 32), 256, 0, st>>>(
        nrp, ncol, ctype, ei, ej, eslot, tri_slot, m, L, tri, tri_sum, sh_base, nw, SB, hub_base,
        Hw, HB, status);
    LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_node_aggr(const int64_t *nrp, const int32_t *ncol, const uint8_t *ctype,
                            const uint32_t *tri_slot, const uint32_t *tdeg,
                            int64_t n, int L, uint64_t *A, uint64_t *D, bool ad_u32,
                            const uint32_t *status, hipStream_t st) {
    size_t sh = (size_t)4 * 2 * L * L * sizeof(uint64_t);
    k_node_aggr<<<blocks_bounded(n, 4, 32), 256, sh, st>>>(nrp, ncol, ctype, tri_slot, tdeg, n, L,
                                                           A, D, ad_u32 ? 1 : 0, status);
    LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_cyc_work(const int64_t *nrp, const int32_t *ncol, const uint32_t *neid,
                           const uint32_t *eslot, const uint32_t *nlow, int64_t n, uint32_t *la_l,
                           uint4 *la_h, uint32_t *lb_l, uint4 *lb_h, uint64_t *counters,
                           uint64_t task_wedges, int L, uint64_t range_bytes,
                           uint64_t light_max, const BlkSelect &blk, const uint32_t *status,
                           hipStream_t st) {
    if (n <= 0) return hipSuccess;
    int dev = 0, cus = 0;
    hipError_t err = hipGetDevice(&dev);
    if (err != hipSuccess) return err;
    err = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (err != hipSuccess) return err;
    int64_t want = (n + 4 * WAVE - 1) / (4 * WAVE) + 1;
    int64_t cap = (int64_t)(cus > 0 ? cus : 256) * 16;
    unsigned grid = (unsigned)(want < cap ? want : cap);
    k_cyc_work<<<grid, 256, 0, st>>>(nrp, ncol, neid, eslot, nlow, n, la_l, la_h, lb_l, lb_h,
                                     counters, task_wedges, L, range_bytes, light_max, blk, status);
    LAUNCH_CHECK();
    return hipSuccess;
}

// Items per staging round: at most threads / 2, with LDS accumulators of
// L^2 words per item within 32 KB (256 threads) or 50 KB (512 or more), so
// a workgroup stays under 64 KB of LDS for every L.
int heavy_chunk_for(int L, int threads, int hub_ids, bool t32) {
    // LDS for the per-item tallies: a 1024-thread workgroup runs alone on
    // its CU (registers), so it may take twice the budget of smaller ones;
    // with hub targets in LDS the tallies and the hub fields share it
    int budget = threads >= 1024 ? 102400 : threads >= 512 ? 51200 : 32768;
    if (hub_ids > 0) {
        // four workgroups per CU while the hub fields leave room, else the
        // tallies keep 8 KB
        budget = 36864 - ((hub_ids * L + 1) / 2) * 4;
        if (budget < 8192) budget = 8192;
    }
    int ch = budget / (L * L * (t32 ? 4 * TALLY_COPIES : 8));
    if (ch > threads / 2) ch = threads / 2;
    if (ch < 1) ch = 1;
    return ch;
}

// Hub targets of the pass-B task kernel: the top ids whose 16-bit fields
// (L per target) fit `bytes` of LDS, a power of two, at most n (0: none).
int heavy_hub_ids(int L, int64_t n, int64_t bytes) {
    if ((int64_t)L * 2 > bytes) return 0;
    int h = 1;
    while ((int64_t)(2 * h) * L * 2 <= bytes) h *= 2;
    return (int64_t)h > n ? (int)n : h;
}

hipError_t launch_cycles(int pass, bool heavy, const CycleArgs &args, unsigned grid, hipStream_t st) {
    if (grid == 0) return hipSuccess;
    if (!heavy) {
        size_t sh = ((size_t)1 << args.light_log2) * (1 + (args.L + 1) / 2) * sizeof(uint32_t);
        if (pass == 0) k_cyc_light<0><<<grid, 64, sh, st>>>(args);
        else k_cyc_light<1><<<grid, 64, sh, st>>>(args);
    } else {
        size_t sh = (size_t)args.chunk * args.L * args.L *
                        (args.nc_u32 ? sizeof(uint32_t) * TALLY_COPIES : sizeof(uint64_t)) +
                    (size_t)((args.hub_ids * args.L + 1) / 2) * sizeof(uint32_t);
        if (pass == 0) k_cyc_heavy<0, HEAVY_THREADS_A><<<grid, HEAVY_THREADS_A, sh, st>>>(args);
        else k_cyc_heavy<1, HEAVY_THREADS_B><<<grid, HEAVY_THREADS_B, sh, st>>>(args);
    }
    LAUNCH_CHECK();
    return hipSuccess;
}

// Threads of the blocked walk kernels (hist, part, emit).
constexpr int BLK_WALK_THREADS = 512;
constexpr int BLK_EMIT_THREADS = 512;

// Items per emit staging round: at most a quarter of the emit threads,
// with BLK_COPIES copies of 32-bit tallies of L^2 words per item within
// 64 KB of LDS.
int blk_emit_chunk(int L) {
    int ch = 65536 / (L * L * (int)sizeof(uint32_t) * BLK_COPIES);
    if (ch > BLK_EMIT_THREADS / 4) ch = BLK_EMIT_THREADS / 4;
    if (ch < 1) ch = 1;
    return ch;
}

template <int PASS>
static hipError_t launch_blk_pass(const CycleArgs &a, const BlkArgs &b, int64_t *scan_tmp,
                                  unsigned wide, hipStream_t st) {
    constexpr int NT = BLK_WALK_THREADS;
    const size_t sh_hist = (size_t)b.nb_max * sizeof(uint32_t);
    const size_t sh_cnt = (size_t)((BLK_IDS * a.L + 1) / 2 + BLK_IDS / 32) * sizeof(uint32_t);
    const size_t sh_acc = (size_t)b.emit_chunk * a.L * a.L * sizeof(uint32_t) * BLK_COPIES;
    k_blk_select<PASS><<<1, 1024, 0, st>>>(a, b);
    LAUNCH_CHECK();
    k_blk_setup<PASS><<<1, 1024, 0, st>>>(a, b);
    LAUNCH_CHECK();
    k_blk_items<PASS><<<(unsigned)b.max_groups, 256, 0, st>>>(a, b);
    LAUNCH_CHECK();
    k_blk_hist<PASS, NT><<<wide, NT, sh_hist, st>>>(a, b);
    LAUNCH_CHECK();
    hipError_t err = launch_excl_scan(b.bcount, b.bstart, b.nbk + 1, scan_tmp, a.status, st);
    if (err != hipSuccess) return err;
    k_blk_part<PASS, NT><<<wide, NT, sh_hist, st>>>(a, b);
    LAUNCH_CHECK();
    k_blk_count<PASS><<<wide, BLK_COUNT_THREADS, sh_cnt, st>>>(a, b);
    LAUNCH_CHECK();
    k_blk_emit<PASS, BLK_EMIT_THREADS><<<wide, BLK_EMIT_THREADS, sh_acc, st>>>(a, b);
    LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_blk(int pass, const CycleArgs &a, const BlkArgs &b, int64_t *scan_tmp,
                      hipStream_t st) {
    if (b.max_groups <= 0 || a.L > 16 || b.emit_chunk < 1 || b.emit_chunk > BLK_EMIT_THREADS / 2 ||
        b.task < 1 || b.task > BLK_TASK)
        return hipErrorInvalidValue;
    int dev = 0, cus = 0;
    hipError_t err = hipGetDevice(&dev);
    if (err != hipSuccess) return err;
    err = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (err != hipSuccess) return err;
    const unsigned wide = (unsigned)(cus > 0 ? cus : 256) * 4;
    return pass == 0 ? launch_blk_pass<0>(a, b, scan_tmp, wide, st)
                     : launch_blk_pass<1>(a, b, scan_tmp, wide, st);
}

hipError_t launch_global_finalize(const uint64_t *gacc, int L, int gw, uint64_t *out, uint32_t *status,
                                  hipStream_t st) {
    k_global_finalize<<<blocks_for(gw, 256), 256, 0, st>>>(gacc, L, out, status);
    LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_batch_graphs(const int64_t *node_ptr, const int32_t *gL, const int64_t *goff,
                               int64_t G, int64_t n, int L_max, int64_t globals_len,
                               int64_t max_nodes, int32_t *node_graph, uint32_t *status,
                               uint64_t *max_gsize, hipStream_t st) {
    if (G <= 0) return hipSuccess;
    k_batch_graphs<<<blocks_for(G, 4), 256, 0, st>>>(node_ptr, gL, goff, G, n, L_max, globals_len,
                                                     max_nodes, node_graph, status, max_gsize);
    LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_batch_edges(const int64_t *node_ptr, const int64_t *eoff, int64_t G,
                              int64_t *gedge_ptr, const uint32_t *status, hipStream_t st) {
    k_batch_edges<<<blocks_for(G + 1, 256), 256, 0, st>>>(node_ptr, eoff, G, gedge_ptr, status);
    LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_batch_finalize(uint64_t *globals, const int32_t *gL, const int64_t *goff, int64_t G,
                                 uint32_t *status, hipStream_t st) {
    if (G <= 0) return hipSuccess;
    unsigned grid = (unsigned)(G < 8192 ? G : 8192);
    k_batch_finalize<<<grid, 256, 0, st>>>(globals, gL, goff, G, status);
    LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_superhubs(const int64_t *nrp, const int32_t *ncol, int64_t n, int S, int64_t nw,
                            uint64_t *SB, uint32_t *SP, hipStream_t st) {
    if (S <= 0) return hipSuccess;
    k_superhubs<<<(unsigned)S, 256, 0, st>>>(nrp, ncol, n, S, nw, SB, SP);
    LAUNCH_CHECK();
    return hipSuccess;
}

}  // namespace tg
