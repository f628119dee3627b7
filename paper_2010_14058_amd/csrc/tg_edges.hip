// Per-edge kernels: triangle set, typed 4-clique pairs, gathers, the
// derivation of every orbit, the row write and the global histogram.
//
// Hub core.  The H highest-ranked nodes (internal ids base..n-1, base = n-H)
// keep a dense H x H adjacency bit-matrix HB with a per-word exclusive
// prefix popcount and per-type hub masks TM.  For an edge (i, j) the
// triangle set T = Gamma_i cap Gamma_j splits into hub members (kept as a
// bit mask Tm over hub indices and a list) and low members (a sorted list).
// Hub members of two hub endpoints come from AND-ing their bit rows; the
// slot of a hub k inside a hub row is its prefix popcount.  Ordered typed
// clique pairs K(u, v) = #{(k, r) in T^u x T^v : k ~ r} (the 4-clique test of
// Alg. 3) are counted as popcounts of AND-ed hub words for hub-hub pairs and
// by scanning the short rows of low members for the rest.
#include <hip/hip_runtime.h>
#include <type_traits>

#include "tg_device.hpp"

namespace tg {

// One wave per hub: its bit row over hub neighbours and the prefix popcounts.
__global__ void k_hub_rows(const int64_t *__restrict__ nrp, const int32_t *__restrict__ ncol,
                           const int64_t *__restrict__ hstart, int64_t n, int H, int Hw,
                           uint64_t *__restrict__ HB, uint32_t *__restrict__ pre) {
    extern __shared__ uint64_t sm_hub[];
    int w = threadIdx.x / WAVE, lane = lane_id();
    int h = blockIdx.x * (blockDim.x / WAVE) + w;
    if (h >= H) return;
    uint64_t *row = sm_hub + (size_t)w * Hw;
    for (int q = lane; q < Hw; q += WAVE) row[q] = 0;
    wave_sync();
    const int32_t base = (int32_t)(n - H);
    const int32_t v = base + h;
    for (int64_t s = hstart[v] + lane; s < nrp[v + 1]; s += WAVE) {
        int32_t x = ncol[s] - base;
        atomicOr((unsigned long long *)&row[x >> 6], 1ull << (x & 63));
    }
    wave_sync();
    uint32_t carry = 0;
    for (int q0 = 0; q0 < Hw; q0 += WAVE) {
        int q = q0 + lane;
        uint64_t word = q < Hw ? row[q] : 0ull;
        uint32_t c = (uint32_t)__popcll(word);
        uint32_t incl = wave_incl_scan(c);
        if (q < Hw) {
            HB[(size_t)h * Hw + q] = word;
            pre[(size_t)h * Hw + q] = carry + incl - c;
        }
        carry += __shfl(incl, WAVE - 1, WAVE);
    }
}

// TM[q][t] (t < tm_pitch(L)): bit b set iff hub 64q+b has type t, for
// t < L - 1; the padding entry is zero.  A word's masks are adjacent, so the
// hub-pair count reads them 16 bytes at a time.
__global__ void k_hub_types(const uint8_t *__restrict__ ntype, int64_t n, int H, int Hw, int L,
                            uint64_t *__restrict__ TM) {
    const int TP = tm_pitch(L);
    int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= TP * Hw) return;
    int q = idx / TP, t = idx - q * TP;
    uint64_t m = 0;
    if (t < L - 1)
        for (int b = 0; b < 64; ++b) {
            int h = q * 64 + b;
            if (h < H && ntype[n - H + h] == t) m |= 1ull << b;
        }
    TM[idx] = m;
}

// Index of global entry idx (layout of L types) in the layout of Lg <= L
// types, or -1 if the entry involves a type >= Lg.  Co-lexicographic ranks
// of multisets over {0..Lg-1} are the same in both layouts.
__device__ __forceinline__ int remap_global(int idx, int L, int Lg) {
    int n2 = (int)binom_small(L + 1, 2), n3 = (int)binom_small(L + 2, 3),
        n4 = (int)binom_small(L + 3, 4);
    int m2 = (int)binom_small(Lg + 1, 2), m3 = (int)binom_small(Lg + 2, 3),
        m4 = (int)binom_small(Lg + 3, 4);
    if (idx < n2) return idx < m2 ? idx : -1;
    idx -= n2;
    if (idx < n3) return idx < m3 ? m2 + idx : -1;
    idx -= n3;
    if (idx < n3) return idx < m3 ? m2 + m3 + idx : -1;
    idx -= n3;
    int h = idx / n4, r = idx - h * n4;
    return r < m4 ? m2 + 2 * m3 + h * m4 + r : -1;
}

// Add v to global entry idx of the edge's graph g (always 0 for one graph).
// uint64 words of the LDS histogram (0 when it lives in global memory).
__device__ __forceinline__ int hist_words(const EdgeArgs &a) {
    return a.hist_in_lds == 2 ? (a.gw + 1) / 2 : a.hist_in_lds ? a.gw : 0;
}

// Entry q of the LDS histogram, read and cleared.
__device__ __forceinline__ uint64_t hist_take(const EdgeArgs &a, uint64_t *hist, int q) {
    if (a.hist_in_lds == 2) {
        uint32_t *h = reinterpret_cast<uint32_t *>(hist);
        uint32_t v = h[q];
        if (v) h[q] = 0u;
        return v;
    }
    uint64_t v = hist[q];
    if (v) hist[q] = 0ull;
    return v;
}

__device__ __forceinline__ void hist_add(const EdgeArgs &a, uint64_t *hist, int idx, uint64_t v,
                                         int64_t g) {
    if (!v) return;
    if (a.hist_in_lds == 2) {
        // 32-bit entries: the host allows them only when a flush interval's
        // sum fits (batch chunks of small-degree graphs)
        atomicAdd(reinterpret_cast<uint32_t *>(hist) + idx, (uint32_t)v);
    } else if (a.hist_in_lds) {
        atomicAdd((unsigned long long *)&hist[idx], (unsigned long long)v);
    } else if (a.batch) {
        int j = remap_global(idx, a.L, a.gL[g]);
        if (j < 0) atomicOr(a.status, ST_INTERNAL);
        else atomicAdd((unsigned long long *)&a.gacc[a.goff[g] + j], (unsigned long long)v);
    } else {
        atomicAdd((unsigned long long *)&a.gacc[idx], (unsigned long long)v);
    }
}

template <int NT>
__device__ __forceinline__ void group_sync() {
    if (NT == WAVE) wave_sync(); else __syncthreads();
}

// Position of hub x (index hx) inside the row of hub y (index hy).
__device__ __forceinline__ int64_t hub_slot(const EdgeArgs &a, int32_t y, int hy, int hx) {
    size_t o = (size_t)hy * a.Hw + (hx >> 6);
    uint64_t below = (hx & 63) ? (a.HB[o] & ((1ull << (hx & 63)) - 1)) : 0ull;
    return a.hstart[y] + a.hpre[o] + (uint32_t)__popcll(below);
}

__device__ __forceinline__ bool hub_adj(const EdgeArgs &a, int hy, int hx) {
    return (a.HB[(size_t)hy * a.Hw + (hx >> 6)] >> (hx & 63)) & 1ull;
}

// Accumulate the triangle-set gathers of member k of type t: X_i(t, .) += |T_ik^.|,
// X_j(t, .) += |T_jk^.|, Y(t, .) += d_k^.
// The three rows have tri_pitch(L) words (a multiple of 4, 16-byte aligned),
// read four words per load.
__device__ __forceinline__ void gather_member(const EdgeArgs &a, int32_t k, int t, int64_t s_i,
                                              int64_t s_j, uint64_t *Xi, uint64_t *Xj,
                                              uint64_t *Y) {
    const int L = a.L;
    const int LP = tri_pitch(L);
    const uint4 *ri = reinterpret_cast<const uint4 *>(a.tri_slot + (size_t)s_i * LP);
    const uint4 *rj = reinterpret_cast<const uint4 *>(a.tri_slot + (size_t)s_j * LP);
    const uint4 *ry = reinterpret_cast<const uint4 *>(a.tdeg + (size_t)k * LP);
    for (int c = 0; c < LP; c += 4) {
        const uint4 vi = ri[c >> 2], vj = rj[c >> 2], vy = ry[c >> 2];
        const uint32_t wi[4] = {vi.x, vi.y, vi.z, vi.w};
        const uint32_t wj[4] = {vj.x, vj.y, vj.z, vj.w};
        const uint32_t wy[4] = {vy.x, vy.y, vy.z, vy.w};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int t2 = c + q;
            if (t2 >= L) break;
            if (wi[q]) atomicAdd((unsigned long long *)&Xi[t * L + t2], (unsigned long long)wi[q]);
            if (wj[q]) atomicAdd((unsigned long long *)&Xj[t * L + t2], (unsigned long long)wj[q]);
            if (wy[q]) atomicAdd((unsigned long long *)&Y[t * L + t2], (unsigned long long)wy[q]);
        }
    }
}

// Copies of the workgroup kernel's 32-bit gather sums per wave: lanes of a
// wave gathering members of one type add into different copies.
constexpr int GATHER_COPIES = 4;

// gather_member into 32-bit copies (every degree below 2^16: a sum over the
// members of an edge's triangle set, each below 2^16, stays below 2^32);
// entry e of lane copy c is word e * GATHER_COPIES + c.
__device__ __forceinline__ void gather_member32(const EdgeArgs &a, int32_t k, int t, int64_t s_i,
                                                int64_t s_j, uint32_t *Xi) {
    const int L = a.L;
    uint32_t *Xj = Xi + L * L * GATHER_COPIES;
    uint32_t *Y = Xi + 2 * L * L * GATHER_COPIES;
    const int LP = tri_pitch(L);
    const uint4 *ri = reinterpret_cast<const uint4 *>(a.tri_slot + (size_t)s_i * LP);
    const uint4 *rj = reinterpret_cast<const uint4 *>(a.tri_slot + (size_t)s_j * LP);
    const uint4 *ry = reinterpret_cast<const uint4 *>(a.tdeg + (size_t)k * LP);
    for (int c = 0; c < LP; c += 4) {
        const uint4 vi = ri[c >> 2], vj = rj[c >> 2], vy = ry[c >> 2];
        const uint32_t wi[4] = {vi.x, vi.y, vi.z, vi.w};
        const uint32_t wj[4] = {vj.x, vj.y, vj.z, vj.w};
        const uint32_t wy[4] = {vy.x, vy.y, vy.z, vy.w};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int t2 = c + q;
            if (t2 >= L) break;
            const int e = (t * L + t2) * GATHER_COPIES;
            if (wi[q]) atomicAdd(&Xi[e], wi[q]);
            if (wj[q]) atomicAdd(&Xj[e], wj[q]);
            if (wy[q]) atomicAdd(&Y[e], wy[q]);
        }
    }
}

// Ordered append of flagged items across the NT threads; returns each
// flagged thread's position (order = thread order) and advances *count.
template <int NT>
__device__ __forceinline__ uint32_t ordered_append(bool flag, uint32_t &count, uint32_t *wave_cnt) {
    uint64_t bal = __ballot(flag);
    int lane = lane_id();
    uint32_t within = (uint32_t)__popcll(bal & ((1ull << lane) - 1));
    if (NT == WAVE) {
        uint32_t pos = count + within;
        count += (uint32_t)__popcll(bal);
        return pos;
    }
    int w = threadIdx.x / WAVE;
    if (lane == 0) wave_cnt[w] = (uint32_t)__popcll(bal);
    __syncthreads();
    uint32_t off = 0, tot = 0;
    for (int q = 0; q < NT / WAVE; ++q) {
        if (q < w) off += wave_cnt[q];
        tot += wave_cnt[q];
    }
    __syncthreads();
    uint32_t pos = count + off + within;
    count += tot;
    return pos;
}

// LDS scratch of one edge.
struct EdgeShared {
    uint64_t *Xi, *Xj, *Y, *K;
    uint64_t *Tm;           // hub members as bits over hub indices
    uint32_t *Th;           // hub members' hub indices; member q at Th[q * th_step]
                            // (uint16 words, step 1, in the workgroup kernel)
    int th_step;            // +1, or -1 when Th grows down from the end of Tl's buffer
    uint32_t *Tl;           // low members, ascending
    uint32_t *meta;         // [0] |Tl| [1] |Th| [2] first word of Tm [3] last word
    uint32_t *wave_cnt;     // ordered_append scratch
    uint64_t *Gw;           // per-wave copies of Xi, Xj, Y (3 L^2 words each) or null
};

// Hub-member list: hub index (below HUB_MAX <= 2^16) of member q.  The
// one-wave kernel shares a uint32 buffer with the low members (Th grows down
// from its end); the workgroup kernel keeps a uint16 list of its own, half
// the LDS, so that one more workgroup fits on a CU.
template <int NT>
__device__ __forceinline__ void th_put(const EdgeShared &S, uint32_t q, int hk) {
    if constexpr (NT == WAVE) S.Th[(ptrdiff_t)q * S.th_step] = (uint32_t)hk;
    else reinterpret_cast<uint16_t *>(S.Th)[q] = (uint16_t)hk;
}

template <int NT>
__device__ __forceinline__ int th_get(const EdgeShared &S, uint32_t q) {
    if constexpr (NT == WAVE) return (int)S.Th[(ptrdiff_t)q * S.th_step];
    else return (int)reinterpret_cast<const uint16_t *>(S.Th)[q];
}

// Inclusive scan of one value per thread over the NT threads; *total (if
// given) receives the sum over all of them.
template <int NT>
__device__ __forceinline__ uint32_t group_incl_scan(uint32_t v, uint32_t *wave_cnt,
                                                    uint32_t *total = nullptr) {
    uint32_t incl = wave_incl_scan(v);
    if (NT == WAVE) {
        if (total) *total = __shfl(incl, WAVE - 1, WAVE);
        return incl;
    }
    int w = threadIdx.x / WAVE;
    if (lane_id() == WAVE - 1) wave_cnt[w] = incl;
    __syncthreads();
    uint32_t add = 0, all = 0;
    for (int q = 0; q < NT / WAVE; ++q) {
        if (q < w) add += wave_cnt[q];
        all += wave_cnt[q];
    }
    __syncthreads();
    if (total) *total = all;
    return incl + add;
}

// Build T (hub mask/list and sorted low list) and the gathers X_i, X_j, Y.
// With G32 (every degree below 2^16, workgroup kernel) the per-wave gather
// copies are GATHER_COPIES 32-bit lane copies.
template <int NT, bool G32 = false>
__device__ void edge_build(const EdgeArgs &a, int32_t i, int32_t j, const EdgeShared &S, int tid) {
    const int L = a.L, LL = L * L;
    const int Hw = a.Hw;
    const int32_t base = a.hub_base;
    for (int q = tid; q < 4 * LL; q += NT) S.Xi[q] = 0;
    if (S.Gw) {
        const int gwords = (NT / WAVE) * 3 * LL * (G32 ? GATHER_COPIES / 2 : 1);
        for (int q = tid; q < gwords; q += NT) S.Gw[q] = 0;
    }
    for (int q = tid; q < Hw; q += NT) S.Tm[q] = 0;
    // gathers go to this wave's private copy when there is one (fewer
    // conflicting LDS atomics), summed into Xi, Xj, Y at the end
    uint64_t *gXi = S.Gw ? S.Gw + (size_t)(tid / WAVE) * 3 * LL : S.Xi;
    uint64_t *gXj = S.Gw ? gXi + LL : S.Xj;
    uint64_t *gY = S.Gw ? gXi + 2 * LL : S.Y;
    // 32-bit lane copies: wave w's block of 3 L^2 entries x GATHER_COPIES
    uint32_t *hXi = G32 ? reinterpret_cast<uint32_t *>(S.Gw) +
                              (size_t)(tid / WAVE) * 3 * LL * GATHER_COPIES +
                              (lane_id() & (GATHER_COPIES - 1))
                        : nullptr;

    if (tid == 0) {
        S.meta[0] = 0;
        S.meta[1] = 0;
        S.meta[2] = 0xffffffffu;
        S.meta[3] = 0;
    }
    group_sync<NT>();
    const int64_t ib = a.nrp[i], ie = a.nrp[i + 1], jb = a.nrp[j], je = a.nrp[j + 1];
    const int64_t ih = a.hstart[i], jh = a.hstart[j];

    // low members: walk the shorter low prefix, test each node against the
    // other endpoint (its super-hub bitmap, else a binary search)
    {
        bool i_small = (ih - ib) <= (jh - jb);
        int64_t sb = i_small ? ib : jb, se = i_small ? ih : jh;
        int64_t lb = i_small ? jb : ib, le = i_small ? jh : ih;
        const int32_t other = i_small ? j : i;
        const bool probe = other >= a.sh_base;
        const int so = other - a.sh_base;
        // the low list must be sorted only for the binary searches of the
        // clique walk, which both endpoints being super-hubs avoid; then
        // waves append on their own, with no barrier per chunk
        const bool unordered = NT > WAVE && i >= a.sh_base && j >= a.sh_base;
        uint32_t count = 0;
        // software pipeline over the chunks: candidate ids are loaded two
        // chunks ahead and the other endpoint's bitmap words one chunk ahead,
        // so the dependent loads of a chunk overlap the work of the previous
        const uint64_t *sbrow = probe ? a.SB + (size_t)so * a.nw : nullptr;
        const int64_t orow = a.nrp[other];
        int32_t x1 = sb + tid < se ? a.ncol[sb + tid] : 0;
        uint64_t w1 = probe && sb + tid < se ? sbrow[x1 >> 6] : 0ull;
        int32_t x2 = sb + NT + tid < se ? a.ncol[sb + NT + tid] : 0;
        for (int64_t p0 = sb; p0 < se; p0 += NT) {
            const int64_t p = p0 + tid;
            const int32_t x = x1;
            const uint64_t w = w1;
            x1 = x2;
            w1 = probe && p + NT < se ? sbrow[x1 >> 6] : 0ull;
            x2 = p + 2 * NT < se ? a.ncol[p + 2 * NT] : 0;
            bool found = false;
            int64_t q = 0;
            if (p < se) {
                if (probe) {
                    found = (w >> (x & 63)) & 1ull;
                    if (found) {
                        const uint64_t below = (x & 63) ? (w & ((1ull << (x & 63)) - 1)) : 0ull;
                        q = orow + a.SP[(size_t)so * a.nw + (x >> 6)] + (uint32_t)__popcll(below);
                    }
                } else {
                    q = lower_bound(a.ncol, lb, le, x);
                    found = q < le && a.ncol[q] == x;
                }
            }
            uint32_t pos;
            if (unordered) {
                const uint64_t bal = __ballot(found);
                uint32_t at = 0;
                if (bal) {
                    if (lane_id() == 0) at = atomicAdd(&S.meta[0], (uint32_t)__popcll(bal));
                    at = __shfl(at, 0, WAVE);
                }
                pos = at + (uint32_t)__popcll(bal & ((1ull << lane_id()) - 1ull));
            } else {
                pos = ordered_append<NT>(found, count, S.wave_cnt);
            }
            if (found) {
                S.Tl[pos] = (uint32_t)x;
                if constexpr (G32)
                    gather_member32(a, x, a.ctype[p], i_small ? p : q, i_small ? q : p, hXi);
                else
                    gather_member(a, x, a.ctype[p], i_small ? p : q, i_small ? q : p, gXi, gXj, gY);
            }
        }
        if (tid == 0 && !unordered) S.meta[0] = count;
    }

    // hub members
    const bool hi = i >= base, hj = j >= base;
    if (hi && hj) {
        // T's hub mask is the AND of the two bit rows: its members are listed
        // in hub order (a scan of the words' popcounts gives each word its
        // place), then gathered one member per thread, so every thread has
        // independent loads however the members fall into words
        const int hx_i = i - base, hx_j = j - base;
        uint32_t nh = 0;
        for (int q0 = 0; q0 < Hw; q0 += NT) {
            const int q = q0 + tid;
            uint64_t m = q < Hw ? a.HB[(size_t)hx_i * Hw + q] & a.HB[(size_t)hx_j * Hw + q] : 0ull;
            if (q < Hw) S.Tm[q] = m;
            if (m) {
                atomicMin(&S.meta[2], (uint32_t)q);
                atomicMax(&S.meta[3], (uint32_t)q);
            }
            const uint32_t c = (uint32_t)__popcll(m);
            uint32_t all = 0;
            uint32_t pos = nh + group_incl_scan<NT>(c, S.wave_cnt, &all) - c;
            while (m) {
                const int b = __ffsll((unsigned long long)m) - 1;
                m &= m - 1;
                th_put<NT>(S, pos, q * 64 + b);
                ++pos;
            }
            nh += all;
        }
        if (tid == 0) S.meta[1] = nh;
        group_sync<NT>();
        for (uint32_t f = tid; f < nh; f += NT) {
            const int hk = th_get<NT>(S, f);
            const int32_t k = base + hk;
            if constexpr (G32)
                gather_member32(a, k, a.ntype[k], hub_slot(a, i, hx_i, hk), hub_slot(a, j, hx_j, hk),
                                hXi);
            else
                gather_member(a, k, a.ntype[k], hub_slot(a, i, hx_i, hk), hub_slot(a, j, hx_j, hk),
                              gXi, gXj, gY);
        }
    } else {
        // scan the shorter hub suffix; test the other endpoint by its bit row
        // when it is a hub, else by binary search in its hub suffix
        bool i_small = (ie - ih) <= (je - jh);
        int64_t sb = i_small ? ih : jh, se = i_small ? ie : je;
        int32_t other = i_small ? j : i;
        int64_t ob = i_small ? jh : ih, oe = i_small ? je : ie;
        bool other_hub = other >= base;
        for (int64_t p = sb + tid; p < se; p += NT) {
            int32_t x = a.ncol[p];
            int hk = x - base;
            int64_t q;
            bool found;
            if (other_hub) {
                found = hub_adj(a, other - base, hk);
                q = found ? hub_slot(a, other, other - base, hk) : 0;
            } else {
                q = lower_bound(a.ncol, ob, oe, x);
                found = q < oe && a.ncol[q] == x;
            }
            if (!found) continue;
            atomicOr((unsigned long long *)&S.Tm[hk >> 6], 1ull << (hk & 63));
            atomicMin(&S.meta[2], (uint32_t)(hk >> 6));
            atomicMax(&S.meta[3], (uint32_t)(hk >> 6));
            uint32_t pos = atomicAdd(&S.meta[1], 1u);
            th_put<NT>(S, pos, hk);
            if constexpr (G32)
                gather_member32(a, x, a.ctype[p], i_small ? p : q, i_small ? q : p, hXi);
            else
                gather_member(a, x, a.ctype[p], i_small ? p : q, i_small ? q : p, gXi, gXj, gY);
        }
    }
    group_sync<NT>();
    if (S.Gw) {
        const uint32_t *gw32 = reinterpret_cast<const uint32_t *>(S.Gw);
        for (int q = tid; q < 3 * LL; q += NT) {
            uint64_t v = 0;
            if constexpr (G32) {
                for (int w = 0; w < NT / WAVE; ++w)
#pragma unroll
                    for (int c = 0; c < GATHER_COPIES; ++c)
                        v += gw32[((size_t)w * 3 * LL + q) * GATHER_COPIES + c];
            } else {
                for (int w = 0; w < NT / WAVE; ++w) v += S.Gw[(size_t)w * 3 * LL + q];
            }
            S.Xi[q] = v;  // Xi, Xj, Y are consecutive
        }
        group_sync<NT>();
    }
}

// Scratch of the flattened low-member scans (NT entries each).
struct ScanScratch {
    uint32_t *r;       // member
    int64_t *start;    // first slot scanned in its row
    uint32_t *scan;    // inclusive scan of the scanned lengths
};

// Ordered typed clique pairs K over the triangle set built by edge_build.
// Hub-hub pairs: per hub member, its bit row AND the hub mask of T, counted
// by type (popcounts against the type masks TMs), or bit tests when T has
// few hub members.  Pairs with a low member r: the neighbours x > r of r are
// walked (flattened over all threads) and each x in T adds both orders, so
// every such pair is seen once.
template <int NT>
__device__ void edge_cliques(const EdgeArgs &a, int32_t i, int32_t j, const EdgeShared &S,
                             const uint64_t *TMs, const ScanScratch &F, int tid) {
    const int L = a.L;
    const int Hw = a.Hw;
    const int TP = tm_pitch(L);
    const int32_t base = a.hub_base;
    const uint32_t nTl = S.meta[0], nTh = S.meta[1];
    // both endpoints super-hubs: low membership of T by two bitmap probes
    const bool both_sh = i >= a.sh_base && j >= a.sh_base;
    const int si = i - a.sh_base, sj = j - a.sh_base;
    if (nTh >= 2) {
        // each unordered hub pair {k, x} once, from its lower member, adding
        // both orders; the work is spread over all threads
        const uint32_t b0 = S.meta[2] >> 3, b1 = (S.meta[3] >> 3) + 1;  // 64-byte blocks
        const uint32_t nb = b1 - b0;
        if (nTh <= 8 * nb + 1) {
            // few members: test every pair's bit
            const uint32_t P = nTh * (nTh - 1) / 2;
            for (uint32_t f = tid; f < P; f += NT) {
                // f = bb (bb - 1) / 2 + aa with aa < bb
                uint32_t bb = (uint32_t)((1.0 + sqrt(1.0 + 8.0 * (double)f)) * 0.5);
                while (bb * (bb - 1) / 2 > f) --bb;
                while ((bb + 1) * bb / 2 <= f) ++bb;
                const uint32_t aa = f - bb * (bb - 1) / 2;
                const int hk = th_get<NT>(S, aa), hx = th_get<NT>(S, bb);
                const int32_t k = base + hk, x = base + hx;
                if ((a.HB[(size_t)hk * Hw + (hx >> 6)] >> (hx & 63)) & 1ull) {
                    const int tk = a.ntype[k], tx = a.ntype[x];
                    atomicAdd((unsigned long long *)&S.K[tk * L + tx], 1ull);
                    atomicAdd((unsigned long long *)&S.K[tx * L + tk], 1ull);
                }
            }
        } else {
            // member k's bit row from its own block on (bits above k), AND
            // the hub mask of T, counted by type; items (member, block) are
            // laid out member by member and each thread takes a contiguous
            // run of them, so counts of one member add up in registers
            for (uint32_t c0 = 0; c0 < nTh; c0 += NT) {
                const uint32_t members = nTh - c0 < (uint32_t)NT ? nTh - c0 : (uint32_t)NT;
                uint32_t len = 0;
                if ((uint32_t)tid < members) {
                    const int32_t k = base + th_get<NT>(S, c0 + tid);
                    const uint32_t kb = (uint32_t)(k - base) >> 9;
                    const uint32_t sb = kb > b0 ? kb : b0;
                    len = sb < b1 ? b1 - sb : 0;
                    F.r[tid] = (uint32_t)k;
                    F.start[tid] = sb;
                }
                uint32_t incl = group_incl_scan<NT>(len, S.wave_cnt);
                F.scan[tid] = incl;
                group_sync<NT>();
                const uint32_t total = F.scan[members - 1];
                const uint32_t per = (total + NT - 1) / NT;
                uint32_t f = (uint32_t)tid * per;
                const uint32_t fe = f + per < total ? f + per : total;
                int o = f < fe ? owner_of(F.scan, (int)members, f) : 0;
                while (f < fe) {
                    const int32_t k = (int32_t)F.r[o];
                    const int hk = k - base;
                    const int tk = a.ntype[k];
                    const uint32_t oend = F.scan[o] < fe ? F.scan[o] : fe;
                    const uint32_t excl = o ? F.scan[o - 1] : 0;
                    const uint64_t *rowk = a.HB + (size_t)hk * Hw;
                    if constexpr (NT == WAVE) {
                        // one wave per edge: registers decide how many waves fit
                        // two 16-bit tallies per register: a member's run covers at
                        // most 16 blocks of 512 bits, so a tally stays below 2^13
                        uint32_t cnt[TG_MAX_L / 2];
#pragma unroll
                        for (int t = 0; t < TG_MAX_L / 2; ++t) cnt[t] = 0;
                        for (; f < oend; ++f) {
                            const uint32_t q = ((uint32_t)F.start[o] + (f - excl)) * 8;
                            const ulonglong2 *rp = reinterpret_cast<const ulonglong2 *>(rowk + q);
#pragma unroll 1
                            for (int half = 0; half < 2; ++half) {
                                ulonglong2 r0 = rp[2 * half], r1 = rp[2 * half + 1];
                                uint64_t w[4] = {r0.x, r0.y, r1.x, r1.y};
#pragma unroll
                                for (int bq = 0; bq < 4; ++bq) {
                                    const int word = (int)q + 4 * half + bq;
                                    uint64_t v = w[bq] & S.Tm[word];
                                    // keep members above k only
                                    if (word < (hk >> 6)) v = 0;
                                    else if (word == (hk >> 6))
                                        v &= (hk & 63) == 63 ? 0ull : (~0ull << ((hk & 63) + 1));
                                    if (!v) continue;
                                    // types 0..L-2 by their masks, type L-1 by
                                    // what they leave
                                    uint32_t rest = (uint32_t)__popcll(v);
                                    const ulonglong2 *tw =
                                        reinterpret_cast<const ulonglong2 *>(TMs + (size_t)word * TP);
#pragma unroll
                                    for (int t = 0; t < TG_MAX_L - 1; t += 2) {
                                        if (t >= TP) break;
                                        const ulonglong2 m2 = tw[t >> 1];
                                        const uint32_t c0 = (uint32_t)__popcll(v & m2.x);
                                        const uint32_t c1 = (uint32_t)__popcll(v & m2.y);
                                        cnt[t >> 1] += c0 | (c1 << 16);
                                        rest -= c0 + c1;
                                    }
#pragma unroll
                                    for (int t = 0; t < TG_MAX_L; ++t)
                                        if (t == L - 1) cnt[t >> 1] += rest << (16 * (t & 1));
                                }
                            }
                        }
#pragma unroll
                        for (int t = 0; t < TG_MAX_L; ++t) {
                            const uint32_t c = (cnt[t >> 1] >> (16 * (t & 1))) & 0xffffu;
                            if (t < L && c) {
                                unsigned long long *Kp = (unsigned long long *)S.K;
                                atomicAdd(&Kp[tk * L + t], (unsigned long long)c);
                                atomicAdd(&Kp[t * L + tk], (unsigned long long)c);
                            }
                        }
                    } else {
                        uint32_t cnt[TG_MAX_L];
#pragma unroll
                        for (int t = 0; t < TG_MAX_L; ++t) cnt[t] = 0;
                        for (; f < oend; ++f) {
                            const uint32_t q = ((uint32_t)F.start[o] + (f - excl)) * 8;
                            const ulonglong2 *rp = reinterpret_cast<const ulonglong2 *>(rowk + q);
                            ulonglong2 r0 = rp[0], r1 = rp[1], r2 = rp[2], r3 = rp[3];
                            uint64_t w[8] = {r0.x, r0.y, r1.x, r1.y, r2.x, r2.y, r3.x, r3.y};
#pragma unroll
                            for (int bq = 0; bq < 8; ++bq) {
                                const int word = (int)q + bq;
                                uint64_t v = w[bq] & S.Tm[word];
                                // keep members above k only
                                if (word < (hk >> 6)) v = 0;
                                else if (word == (hk >> 6))
                                    v &= (hk & 63) == 63 ? 0ull : (~0ull << ((hk & 63) + 1));
                                if (!v) continue;
                                // types 0..L-2 by their masks, type L-1 by what
                                // they leave
                                uint32_t rest = (uint32_t)__popcll(v);
                                const ulonglong2 *tw =
                                    reinterpret_cast<const ulonglong2 *>(TMs + (size_t)word * TP);
#pragma unroll
                                for (int t = 0; t < TG_MAX_L - 1; t += 2) {
                                    if (t >= TP) break;
                                    const ulonglong2 m2 = tw[t >> 1];
                                    const uint32_t c0 = (uint32_t)__popcll(v & m2.x);
                                    const uint32_t c1 = (uint32_t)__popcll(v & m2.y);
                                    cnt[t] += c0;
                                    cnt[t + 1] += c1;
                                    rest -= c0 + c1;
                                }
#pragma unroll
                                for (int t = 0; t < TG_MAX_L; ++t)
                                    if (t == L - 1) cnt[t] += rest;
                            }
                        }
#pragma unroll
                        for (int t = 0; t < TG_MAX_L; ++t)
                            if (t < L && cnt[t]) {
                                unsigned long long *Kp = (unsigned long long *)S.K;
                                atomicAdd(&Kp[tk * L + t], (unsigned long long)cnt[t]);
                                atomicAdd(&Kp[t * L + tk], (unsigned long long)cnt[t]);
                            }
                    }
                    ++o;
                }
                group_sync<NT>();
            }
        }
    }
    for (uint32_t c0 = 0; c0 < nTl; c0 += NT) {
        const uint32_t items = nTl - c0 < (uint32_t)NT ? nTl - c0 : (uint32_t)NT;
        uint32_t len = 0;
        if ((uint32_t)tid < items) {
            int32_t r = (int32_t)S.Tl[c0 + tid];
            int64_t b = a.nrp[r] + a.nlow[r];
            len = (uint32_t)(a.nrp[r + 1] - b);
            F.r[tid] = (uint32_t)r;
            F.start[tid] = b;
        }
        uint32_t incl = group_incl_scan<NT>(len, S.wave_cnt);
        F.scan[tid] = incl;
        group_sync<NT>();
        const uint32_t total = F.scan[items - 1];
        int o = 0;
        for (uint32_t f = tid; f < total; f += NT) {
            o = owner_next(F.scan, (int)items, f, o);
            uint32_t excl = o ? F.scan[o - 1] : 0;
            int32_t r = (int32_t)F.r[o];
            int32_t x = a.ncol[F.start[o] + (f - excl)];
            bool in;
            if (x >= base) {
                int hx = x - base;
                in = (S.Tm[hx >> 6] >> (hx & 63)) & 1ull;
            } else if (both_sh) {
                in = sh_bit(a.SB, a.nw, si, x) && sh_bit(a.SB, a.nw, sj, x);
            } else {
                uint32_t lo = 0, hi2 = nTl;
                while (lo < hi2) {
                    uint32_t mid = (lo + hi2) >> 1;
                    if ((int32_t)S.Tl[mid] < x) lo = mid + 1; else hi2 = mid;
                }
                in = lo < nTl && (int32_t)S.Tl[lo] == x;
            }
            if (!in) continue;
            int tr = a.ntype[r], tx = a.ntype[x];
            atomicAdd((unsigned long long *)&S.K[tr * L + tx], 1ull);
            atomicAdd((unsigned long long *)&S.K[tx * L + tr], 1ull);
        }
        group_sync<NT>();
    }
    // K is read by every thread next, also when T has no low member
    group_sync<NT>();
}

// One edge's Xi, Xj, Y, K (4 L^2 words in LDS) to its xyk row.  Each entry
// is at most max_deg^2 (a sum over at most max_deg common neighbours of a
// count at most max_deg), so with every degree below 2^16 it fits 32 bits.
__device__ __forceinline__ void store_xyk(const EdgeArgs &a, int64_t e, const uint64_t *src,
                                          int tid, int nt) {
    const int n = 4 * a.L * a.L;
    if (a.xyk_u32) {
        uint32_t *dst = reinterpret_cast<uint32_t *>(a.xyk) + (size_t)e * n;
        for (int q = tid; q < n; q += nt) dst[q] = (uint32_t)src[q];
    } else {
        uint64_t *dst = a.xyk + (size_t)e * n;
        for (int q = tid; q < n; q += nt) dst[q] = src[q];
    }
}

// Every orbit of Table 3 for edge e from the triangle, clique, cycle and
// aggregate quantities (inclusion-exclusion in the spirit of Theorem 1;
// Lemmas 1-4 for g4, g5, g9, g11), the row write and the histogram.
// Derivation (Sec. 4 identities, Lemmas 1-4) of one edge's 3-node entries
// for type t, and of its 4-node orbits for type pair p; xyk holds the edge's
// Xi, Xj, Y, K (4 L^2 words, in LDS or global memory).
__device__ __forceinline__ void derive_three(const EdgeArgs &a, int64_t e, int32_t i, int32_t j,
                                             int t, uint64_t *hist, uint32_t &bad, uint64_t *row) {
    const int L = a.L;
    const int n2 = (int)binom_small(L + 1, 2);
    const int n3 = (int)binom_small(L + 2, 3);
    const int64_t gid = a.batch ? (int64_t)a.ngraph[i] : 0;
    const int ta = a.ntype[i], tb = a.ntype[j];
    int64_t nTt = a.tri[(size_t)e * L + t];
    const int LP = tri_pitch(L);
    int64_t si = (int64_t)a.tdeg[(size_t)i * LP + t] - nTt - (tb == t);
    int64_t sj = (int64_t)a.tdeg[(size_t)j * LP + t] - nTt - (ta == t);
    if (si < 0 || sj < 0) bad |= ST_INTERNAL;
    if (row) {
        row[t] = (uint64_t)nTt;
        row[L + t] = (uint64_t)(si + sj);
    }
    int r3 = rank3(ta, tb, t);
    hist_add(a, hist, n2 + r3, (uint64_t)(si + sj), gid);
    hist_add(a, hist, n2 + n3 + r3, (uint64_t)nTt, gid);
}

// XT: word of the xyk entries; NARROW: A, D and NC held as uint32.
template <typename XT, bool NARROW>
__device__ __forceinline__ void derive_pair(const EdgeArgs &a, int64_t e, int32_t i, int32_t j,
                                            int p, const XT *xyk, uint64_t *hist,
                                            uint32_t &bad, uint64_t *row) {
    using AT = typename std::conditional<NARROW, uint32_t, uint64_t>::type;
    const int L = a.L;
    const int LL = L * L;
    const int P = L * (L + 1) / 2;
    const int n2 = (int)binom_small(L + 1, 2);
    const int n3 = (int)binom_small(L + 2, 3);
    const int n4 = (int)binom_small(L + 3, 4);
    const int hbase = n2 + 2 * n3;
    const int64_t gid = a.batch ? (int64_t)a.ngraph[i] : 0;
    const int ta = a.ntype[i], tb = a.ntype[j];
    const XT *Xi = xyk, *Xj = Xi + LL, *Y = Xi + 2 * LL, *K = Xi + 3 * LL;
    const uint32_t *tri_e = a.tri + (size_t)e * L;
    const uint32_t *di = a.tdeg + (size_t)i * tri_pitch(L);
    const uint32_t *dj = a.tdeg + (size_t)j * tri_pitch(L);
    const AT *Ab = reinterpret_cast<const AT *>(a.A), *Db = reinterpret_cast<const AT *>(a.D);
    const AT *Ai = Ab + (size_t)i * LL, *Aj = Ab + (size_t)j * LL;
    const AT *Di = Db + (size_t)i * LL, *Dj = Db + (size_t)j * LL;
    const AT *NC = reinterpret_cast<const AT *>(a.NC) + (size_t)e * LL;
    // pair (t, u), t <= u, from its lexicographic index
    int t = 0, rem = p;
    while (rem >= L - t) { rem -= L - t; ++t; }
    const int u = t + rem;
    const bool same = t == u;
    const int r4 = rank4(ta, tb, t, u);
    const int qa = t * L + u, qb = u * L + t;   // ordered (t,u) and (u,t)
    const int64_t nTt = tri_e[t], nTu = tri_e[u];
    const int64_t Sit = (int64_t)di[t] - nTt - (tb == t), Siu = (int64_t)di[u] - nTu - (tb == u);
    const int64_t Sjt = (int64_t)dj[t] - nTt - (ta == t), Sju = (int64_t)dj[u] - nTu - (ta == u);
    auto emit = [&](int o, int64_t v) {
        if (v < 0) bad |= ST_INTERNAL;
        if (row) row[2 * L + (o - 3) * P + p] = (uint64_t)v;
        // graphlet of each orbit (Sec. 4.4): h3 = g3+g4, h4 = g5,
        // h5 = g6, h6 = g7+g8+g9, h7 = g10+g11, h8 = g12
        const int h = o <= 4 ? 3 : o == 5 ? 4 : o == 6 ? 5 : o <= 9 ? 6 : o <= 11 ? 7 : 8;
        hist_add(a, hist, hbase + (h - 3) * n4 + r4, (uint64_t)v, gid);
    };
    // cliques and chordal cycles
    const int64_t K0 = (int64_t)K[qa], K1 = (int64_t)K[qb];
    if (same && (K0 & 1)) bad |= ST_INTERNAL;
    if (!same && K0 != K1) bad |= ST_INTERNAL;
    const int64_t g12 = same ? K0 / 2 : K0;
    emit(12, g12);
    emit(11, (same ? nTt * (nTt - 1) / 2 : nTt * nTu) - g12);                 // Lemma 4
    const int64_t Xi0 = (int64_t)Xi[qa], Xi1 = (int64_t)Xi[qb];
    const int64_t Xj0 = (int64_t)Xj[qa], Xj1 = (int64_t)Xj[qb];
    // C_i(x,y): pairs k in T^x, r in S_i^y adjacent; likewise C_j
    const int64_t Ci0 = Xi0 - nTt * (tb == u) - K0, Ci1 = Xi1 - nTu * (tb == t) - K1;
    const int64_t Cj0 = Xj0 - nTt * (ta == u) - K0, Cj1 = Xj1 - nTu * (ta == t) - K1;
    const int64_t g10 = same ? Ci0 + Cj0 : Ci0 + Cj0 + Ci1 + Cj1;
    emit(10, g10);
    emit(9, (same ? nTt * (Sit + Sjt) : nTt * (Siu + Sju) + nTu * (Sit + Sjt)) - g10);  // Lemma 3
    // 4-cycles: non-induced cycles minus chordal and clique instances
    const int64_t Cyc0 = (int64_t)NC[qa] - Ci1 - Cj0 - K0;
    const int64_t Cyc1 = (int64_t)NC[qb] - Ci0 - Cj1 - K1;
    const int64_t g6 = same ? Cyc0 : Cyc0 + Cyc1;
    emit(6, g6);
    emit(4, (same ? Sit * Sjt : Sit * Sju + Siu * Sjt) - g6);                 // Lemma 1
    // tailed-triangle tails: adjacent pairs inside S_i (resp. S_j)
    const int64_t sgi0 = (int64_t)Ai[qa] - Xi0 - (tb == t) * nTu;
    const int64_t sgi1 = (int64_t)Ai[qb] - Xi1 - (tb == u) * nTt;
    const int64_t sgj0 = (int64_t)Aj[qa] - Xj0 - (ta == t) * nTu;
    const int64_t sgj1 = (int64_t)Aj[qb] - Xj1 - (ta == u) * nTt;
    const int64_t Ei0 = sgi0 - Ci1, Ei1 = sgi1 - Ci0;
    const int64_t Ej0 = sgj0 - Cj1, Ej1 = sgj1 - Cj0;
    if (same && ((Ei0 + Ej0) & 1)) bad |= ST_INTERNAL;
    if (!same && (Ei0 != Ei1 || Ej0 != Ej1)) bad |= ST_INTERNAL;
    const int64_t g7 = same ? (Ei0 + Ej0) / 2 : Ei0 + Ej0;
    emit(7, g7);
    emit(5, (same ? Sit * (Sit - 1) / 2 + Sjt * (Sjt - 1) / 2 : Sit * Siu + Sjt * Sju) - g7);  // Lemma 2
    // 4-path end edges: neighbours of S_i / S_j outside the edge's sets
    const int64_t Y0 = (int64_t)Y[qa], Y1 = (int64_t)Y[qb];
    const int64_t dli0 = (int64_t)Di[qa] - Y0 - (tb == t) * (int64_t)dj[u];
    const int64_t dli1 = (int64_t)Di[qb] - Y1 - (tb == u) * (int64_t)dj[t];
    const int64_t dlj0 = (int64_t)Dj[qa] - Y0 - (ta == t) * (int64_t)di[u];
    const int64_t dlj1 = (int64_t)Dj[qb] - Y1 - (ta == u) * (int64_t)di[t];
    const int64_t Pi0 = dli0 - Sit * (ta == u) - sgi0 - Cyc0;
    const int64_t Pi1 = dli1 - Siu * (ta == t) - sgi1 - Cyc1;
    const int64_t Pj0 = dlj0 - Sjt * (tb == u) - sgj0 - Cyc1;
    const int64_t Pj1 = dlj1 - Sju * (tb == t) - sgj1 - Cyc0;
    emit(3, same ? Pi0 + Pj0 : Pi0 + Pi1 + Pj0 + Pj1);
    // tailed-triangle edges opposite the tail's node
    const int64_t Q0 = Y0 - Xi0 - Cj0 - nTt * (ta == u);
    const int64_t Q1 = Y1 - Xi1 - Cj1 - nTu * (ta == t);
    emit(8, same ? Q0 : Q0 + Q1);
}

template <int NT, bool NARROW>
__device__ void edge_derive(const EdgeArgs &a, int nb, const int64_t *slot_e, const int32_t *slot_i,
                            const int32_t *slot_j, const uint64_t *xyk, uint64_t *hist, int tid,
                            uint32_t &bad) {
    // nb edges at once (their Xi, Xj, Y, K in consecutive LDS slots of
    // 4 L^2 words), so that the per-pair work of several edges fills a wave
    const int L = a.L;
    const int LL = L * L;
    const int P = L * (L + 1) / 2;
    const int W = 2 * L + 10 * P;
    for (int b = tid; b < nb; b += NT) {
        const int32_t i = slot_i[b], j = slot_j[b];
        const int64_t gid = a.batch ? (int64_t)a.ngraph[i] : 0;
        hist_add(a, hist, rank2(a.ntype[i], a.ntype[j]), 1, gid);
    }
    for (int it = tid; it < nb * L; it += NT) {
        const int b = it / L;
        derive_three(a, slot_e[b], slot_i[b], slot_j[b], it - b * L, hist, bad,
                     a.rows ? a.rows + (size_t)slot_e[b] * W : nullptr);
    }
    for (int it = tid; it < nb * P; it += NT) {
        const int b = it / P;
        derive_pair<uint64_t, NARROW>(a, slot_e[b], slot_i[b], slot_j[b], it - b * P,
                                      xyk + (size_t)b * 4 * LL, hist, bad,
                                      a.rows ? a.rows + (size_t)slot_e[b] * W : nullptr);
    }
}

// LDS layout shared by both edge kernels (dynamic part), in uint64 words:
// [Xi Xj Y K : 4 L^2 per derive slot][hist][Tm : Hw] then uint32 lists.
__device__ __forceinline__ EdgeShared carve(const EdgeArgs &a, uint64_t *sm, uint32_t *meta,
                                            uint32_t *wave_cnt, uint64_t **hist, uint32_t *Th,
                                            int th_step, uint32_t *Tl) {
    const int LL = a.L * a.L;
    EdgeShared S;
    S.Xi = sm;
    S.Xj = sm + LL;
    S.Y = sm + 2 * LL;
    S.K = sm + 3 * LL;
    *hist = sm + 4 * LL * a.derive_batch;
    S.Tm = *hist + hist_words(a);
    S.Th = Th;
    S.th_step = th_step;
    S.Tl = Tl;
    S.meta = meta;
    S.wave_cnt = wave_cnt;
    S.Gw = nullptr;
    return S;
}

// Light edges: one wave per edge (|T| <= min degree <= tcap, lists in LDS).
// DEFER: the edge's Xi, Xj, Y, K go to a.xyk and k_derive does the rest, so
// this kernel carries no derivation state (fewer registers, more waves).
// NARROW: A, D and NC held as uint32 (used by the fused derivation only).
template <bool DEFER, bool NARROW>
__device__ __forceinline__ void edges_light_body(const EdgeArgs &a) {
    extern __shared__ uint64_t sm_edge[];
    __shared__ uint32_t meta[4];
    __shared__ uint32_t wave_cnt[1];
    __shared__ uint32_t fl_r[WAVE], fl_scan[WAVE];
    __shared__ int64_t fl_start[WAVE];
    const ScanScratch F{fl_r, fl_start, fl_scan};
    const int LL = a.L * a.L;
    uint64_t *hist;
    const int EB = a.derive_batch;
    uint64_t *after = sm_edge + 4 * LL * EB + hist_words(a) + a.Hw;
    // one list of tcap entries: low members from the front, hub members from
    // the back (|T| <= min degree <= tcap)
    uint32_t *Tl = (uint32_t *)after;
    uint32_t *Th = Tl + (a.tcap - 1);
    EdgeShared S = carve(a, sm_edge, meta, wave_cnt, &hist, Th, -1, Tl);
    int lane = threadIdx.x;
    if (input_failed(a.status)) return;
    uint32_t bad = 0;
    for (int q = lane; q < hist_words(a); q += WAVE) hist[q] = 0;
    __syncthreads();
    __shared__ int64_t slot_e[4];
    __shared__ int32_t slot_i[4], slot_j[4];
    int nb = 0;  // edges waiting for their derivation
    // build T, the gathers and the cliques of edge e into derive slot nb;
    // edges of the heavy path are queued instead
    auto one_edge = [&](int64_t e) {
        int32_t i = a.ei[e], j = a.ej[e];
        int64_t di = a.nrp[i + 1] - a.nrp[i], dj = a.nrp[j + 1] - a.nrp[j];
        if ((di < dj ? di : dj) > a.tcap) {
            if (lane == 0)
                a.heavy_list[atomicAdd((unsigned long long *)&a.counters[C_EDGE_HEAVY], 1ull)] =
                    (uint32_t)e;
            return;
        }
        EdgeShared Sb = S;
        Sb.Xi = S.Xi + (size_t)nb * 4 * LL;
        Sb.Xj = Sb.Xi + LL;
        Sb.Y = Sb.Xi + 2 * LL;
        Sb.K = Sb.Xi + 3 * LL;
        edge_build<WAVE>(a, i, j, Sb, lane);
        edge_cliques<WAVE>(a, i, j, Sb, a.TM, F, lane);
        if constexpr (DEFER) {
            store_xyk(a, e, Sb.Xi, lane, WAVE);
            return;
        }
        if (lane == 0) {
            slot_e[nb] = e;
            slot_i[nb] = i;
            slot_j[nb] = j;
        }
        ++nb;
    };
    auto derive_all = [&]() {
        if constexpr (DEFER) return;
        if (!nb) return;
        __syncthreads();
        edge_derive<WAVE, NARROW>(a, nb, slot_e, slot_i, slot_j, S.Xi, hist, lane, bad);
        __syncthreads();
        nb = 0;
    };
    if (!a.batch) {
        for (int64_t e = blockIdx.x; e < a.m; e += gridDim.x) {
            one_edge(e);
            if (nb == EB) derive_all();
        }
        derive_all();
        if (a.hist_in_lds)
            for (int q = lane; q < a.gw; q += WAVE) {
                uint64_t v = hist_take(a, hist, q);
                if (v) atomicAdd((unsigned long long *)&a.gacc[q], (unsigned long long)v);
            }
    } else {
        // chunks of consecutive edges (the edges of one graph are
        // contiguous); the histogram is flushed into a graph's own vector
        // whenever the graph changes and at the end of each chunk
        auto flush = [&](int64_t g) {
            if (!a.hist_in_lds) return;
            const int Lg = a.gL[g];
            uint64_t *dst = a.gacc + a.goff[g];
            for (int q = lane; q < a.gw; q += WAVE) {
                uint64_t v = hist_take(a, hist, q);
                if (!v) continue;
                int jq = remap_global(q, a.L, Lg);
                if (jq < 0) bad |= ST_INTERNAL;
                else atomicAdd((unsigned long long *)&dst[jq], (unsigned long long)v);
            }
            __syncthreads();
        };
        const int64_t nchunks = (a.m + BATCH_EDGE_CHUNK - 1) / BATCH_EDGE_CHUNK;
        for (int64_t c = blockIdx.x; c < nchunks; c += gridDim.x) {
            int64_t e0 = c * BATCH_EDGE_CHUNK;
            int64_t e1 = e0 + BATCH_EDGE_CHUNK < a.m ? e0 + BATCH_EDGE_CHUNK : a.m;
            int64_t cur = a.ngraph[a.ei[e0]];
            for (int64_t e = e0; e < e1; ++e) {
                int64_t g = a.ngraph[a.ei[e]];
                if (g != cur) {
                    flush(cur);
                    cur = g;
                }
                one_edge(e);
                derive_all();
            }
            flush(cur);
        }
    }
    bad = wave_or(bad);
    if (lane == 0 && bad) atomicOr(a.status, bad);
}

// The deferred variant holds no derivation state; a register budget for six
// waves per SIMD keeps more edges in flight (a few spilled registers cost
// less than the fifth-to-sixth wave gains; seven or eight spill too much).
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(6)))
k_edges_light_deferred(EdgeArgs a) {
    edges_light_body<true, false>(a);
}

template <bool NARROW>
__global__ void __launch_bounds__(64) k_edges_light_fused(EdgeArgs a) {
    edges_light_body<false, NARROW>(a);
}

// Heavy edges: one 256-thread workgroup per edge, pulled from a queue; the
// low list lives in a global buffer of n entries private to the workgroup,
// the hub list (at most H entries) in LDS.  MODE 0 stores each edge's Xi,
// Xj, Y, K for the separate derivation (MODE 3 the same with 32-bit gather
// copies, every degree below 2^16); 1 and 2 derive in place with 32-bit
// and 64-bit A, D and NC (one instance each, so that the deferred one holds
// no derivation state).
// The deferred instance runs under a register budget for five waves per SIMD
// (some registers spill): with the uint16 hub list, five workgroups fit a
// CU's LDS.
template <int MODE>
__global__ void __launch_bounds__(EDGE_THREADS_HEAVY)
__attribute__((amdgpu_waves_per_eu(MODE == 0 || MODE == 3 ? 5 : 1))) k_edges_heavy(EdgeArgs a) {
    extern __shared__ uint64_t sm_edgeh[];
    __shared__ uint32_t meta[4];
    __shared__ uint32_t wave_cnt[EDGE_THREADS_HEAVY / WAVE];
    __shared__ uint64_t s_idx;
    __shared__ int64_t slot_e[1];
    __shared__ int32_t slot_i[1], slot_j[1];
    __shared__ uint32_t fl_r[EDGE_THREADS_HEAVY], fl_scan[EDGE_THREADS_HEAVY];
    __shared__ int64_t fl_start[EDGE_THREADS_HEAVY];
    const ScanScratch F{fl_r, fl_start, fl_scan};
    const int NT = EDGE_THREADS_HEAVY;
    const int LL = a.L * a.L;
    uint64_t *hist;
    uint64_t *after = sm_edgeh + 4 * LL * a.derive_batch + hist_words(a) + a.Hw;
    // type masks of the hub core, 16-byte aligned for their paired loads
    uint64_t *TMs =
        reinterpret_cast<uint64_t *>((reinterpret_cast<uintptr_t>(after) + 15) & ~uintptr_t(15));
    const int TMw = tm_pitch(a.L) * a.Hw;
    uint64_t *Gw = TMs + TMw;                     // per-wave gather copies
    uint32_t *Th = (uint32_t *)(Gw + (size_t)(NT / WAVE) * 3 * LL * (GATHER_COPIES / 2));
    uint32_t *Tl = a.tbuf + (size_t)blockIdx.x * (size_t)a.n;
    EdgeShared S = carve(a, sm_edgeh, meta, wave_cnt, &hist, Th, 1, Tl);
    S.Gw = Gw;
    int tid = threadIdx.x;
    if (input_failed(a.status)) return;
    for (int q = tid; q < TMw; q += NT) TMs[q] = a.TM[q];
    uint32_t bad = 0;
    for (int q = tid; q < hist_words(a); q += NT) hist[q] = 0;
    uint64_t count = a.counters[C_EDGE_HEAVY];
    __syncthreads();
    while (true) {
        if (tid == 0) s_idx = atomicAdd((unsigned long long *)&a.counters[C_EDGE_NEXT], 1ull);
        __syncthreads();
        uint64_t idx = s_idx;
        __syncthreads();
        if (idx >= count) break;
        int64_t e = a.heavy_list[idx];
        int32_t i = a.ei[e], j = a.ej[e];
        edge_build<NT, MODE == 3>(a, i, j, S, tid);
        __threadfence_block();
        __syncthreads();
        edge_cliques<NT>(a, i, j, S, TMs, F, tid);
        if constexpr (MODE == 0 || MODE == 3) {
            store_xyk(a, e, S.Xi, tid, NT);
        } else {
            if (tid == 0) {
                slot_e[0] = e;
                slot_i[0] = i;
                slot_j[0] = j;
            }
            __syncthreads();
            edge_derive<NT, MODE == 1>(a, 1, slot_e, slot_i, slot_j, S.Xi, hist, tid, bad);
        }
        __threadfence_block();
        __syncthreads();
    }
    if (a.hist_in_lds)
        for (int q = tid; q < a.gw; q += NT) {
            uint64_t v = hist_take(a, hist, q);
            if (v) atomicAdd((unsigned long long *)&a.gacc[q], (unsigned long long)v);
        }
    if (bad) atomicOr(a.status, bad);
}

// Deferred derivation: one thread per (edge, type pair) over the whole
// edge set, reading each edge's Xi, Xj, Y, K from a.xyk; the 3-node entries
// ride on the pairs p < L and the 2-node entry on p = 0.
// A block takes EB = blockDim / P consecutive edges at a time, one thread per
// (edge, type pair); their rows are assembled in LDS (rbuf, EB rows) and then
// written out whole, so the table is written in full lines.
template <typename XT, bool NARROW>
__device__ void derive_edges(const EdgeArgs &a, uint64_t *hist, uint64_t *rbuf, uint32_t &bad) {
    const int L = a.L;
    const int LL = L * L;
    const int P = L * (L + 1) / 2;
    const int W = 2 * L + 10 * P;
    const int EB = (int)blockDim.x / P;
    const XT *xyk = reinterpret_cast<const XT *>(a.xyk);
    const int tid = threadIdx.x;
    const int b = tid / P, p = tid - b * P;
    for (int64_t e0 = (int64_t)blockIdx.x * EB; e0 < a.m; e0 += (int64_t)gridDim.x * EB) {
        const int nb = a.m - e0 < EB ? (int)(a.m - e0) : EB;
        if (b < nb) {
            const int64_t e = e0 + b;
            const int32_t i = a.ei[e], j = a.ej[e];
            uint64_t *row = rbuf ? rbuf + (size_t)b * W : nullptr;
            if (p == 0) hist_add(a, hist, rank2(a.ntype[i], a.ntype[j]), 1, 0);
            if (p < L) derive_three(a, e, i, j, p, hist, bad, row);
            derive_pair<XT, NARROW>(a, e, i, j, p, xyk + (size_t)e * 4 * LL, hist, bad, row);
        }
        if (rbuf) {  // the same for the whole block
            __syncthreads();
            uint64_t *dst = a.rows + (size_t)e0 * W;
            for (int q = tid; q < nb * W; q += blockDim.x) dst[q] = rbuf[q];
            __syncthreads();
        }
    }
}

// One instance per word width (chosen at launch), so each keeps the
// registers of a single derivation loop.
template <typename XT, bool NARROW>
__global__ void __launch_bounds__(256) k_derive(EdgeArgs a) {
    extern __shared__ uint64_t sm_der[];
    if (input_failed(a.status)) return;
    uint64_t *hist = sm_der;
    for (int q = threadIdx.x; q < hist_words(a); q += blockDim.x) hist[q] = 0;
    __syncthreads();
    uint32_t bad = 0;
    derive_edges<XT, NARROW>(a, hist, a.rows ? sm_der + hist_words(a) : nullptr, bad);
    __syncthreads();
    if (a.hist_in_lds)
        for (int q = threadIdx.x; q < a.gw; q += blockDim.x) {
            uint64_t v = hist_take(a, hist, q);
            if (v) atomicAdd((unsigned long long *)&a.gacc[q], (unsigned long long)v);
        }
    if (bad) atomicOr(a.status, bad);
}

// ------------------------------------------------------ launch wrappers

hipError_t launch_hub_build(const int64_t *nrp, const int32_t *ncol, const int64_t *hstart,
                            const uint8_t *ntype, int64_t n, int H, int Hw, int L, uint64_t *HB,
                            uint32_t *pre, uint64_t *TM, hipStream_t st) {
    if (H <= 0) return hipSuccess;
    size_t sh = (size_t)4 * Hw * sizeof(uint64_t);
    k_hub_rows<<<(unsigned)((H + 3) / 4), 256, sh, st>>>(nrp, ncol, hstart, n, H, Hw, HB, pre);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (tm_pitch(L) > 0)
        k_hub_types<<<(unsigned)((tm_pitch(L) * Hw + 255) / 256), 256, 0, st>>>(ntype, n, H, Hw, L,
                                                                              TM);
    return hipGetLastError();
}

size_t edge_lds_bytes(const EdgeArgs &args, bool heavy) {
    int LL = args.L * args.L;
    const int hw = args.hist_in_lds == 2 ? (args.gw + 1) / 2 : args.hist_in_lds ? args.gw : 0;
    size_t sh = (size_t)(4 * LL * args.derive_batch + hw + args.Hw) * sizeof(uint64_t);
    if (!heavy) sh += (size_t)args.tcap * sizeof(uint32_t);
    else sh += (size_t)(tm_pitch(args.L) * args.Hw + 1) * sizeof(uint64_t) +
               (size_t)(EDGE_THREADS_HEAVY / WAVE) * 3 * LL * sizeof(uint64_t) * (GATHER_COPIES / 2) +
               (size_t)(args.hub_base < args.n ? (args.n - args.hub_base) : 0) * sizeof(uint16_t);
    return sh;
}

hipError_t launch_edges(bool heavy, const EdgeArgs &args, unsigned grid, hipStream_t st) {
    if (grid == 0) return hipSuccess;
    size_t sh = edge_lds_bytes(args, heavy);
    if (heavy) {
        if (args.xyk && args.agg_u32) k_edges_heavy<3><<<grid, EDGE_THREADS_HEAVY, sh, st>>>(args);
        else if (args.xyk) k_edges_heavy<0><<<grid, EDGE_THREADS_HEAVY, sh, st>>>(args);
        else if (args.agg_u32) k_edges_heavy<1><<<grid, EDGE_THREADS_HEAVY, sh, st>>>(args);
        else k_edges_heavy<2><<<grid, EDGE_THREADS_HEAVY, sh, st>>>(args);
    } else if (args.xyk) {
        k_edges_light_deferred<<<grid, 64, sh, st>>>(args);
    } else if (args.agg_u32) {
        k_edges_light_fused<true><<<grid, 64, sh, st>>>(args);
    } else {
        k_edges_light_fused<false><<<grid, 64, sh, st>>>(args);
    }
    return hipGetLastError();
}

hipError_t launch_derive(const EdgeArgs &args, unsigned grid, hipStream_t st) {
    if (grid == 0 || args.m == 0) return hipSuccess;
    const int hw = args.hist_in_lds == 2 ? (args.gw + 1) / 2 : args.hist_in_lds ? args.gw : 0;
    // LDS: the histogram, then the rows of blockDim / P edges
    const int P = args.L * (args.L + 1) / 2;
    const int W = 2 * args.L + 10 * P;
    const size_t rw = args.rows ? (size_t)(256 / P) * W : 0;
    const size_t sh = ((size_t)hw + rw) * sizeof(uint64_t);
    // the 32-bit xyk words come with 32-bit A, D and NC (both follow from
    // the largest degree)
    if (args.xyk_u32 && args.agg_u32) k_derive<uint32_t, true><<<grid, 256, sh, st>>>(args);
    else if (args.agg_u32) k_derive<uint64_t, true><<<grid, 256, sh, st>>>(args);
    else k_derive<uint64_t, false><<<grid, 256, sh, st>>>(args);
    return hipGetLastError();
}

}  // namespace tg
