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

// TM[t][q]: bit b set iff hub 64q+b has type t.
__global__ void k_hub_types(const uint8_t *__restrict__ ntype, int64_t n, int H, int Hw, int L,
                            uint64_t *__restrict__ TM) {
    int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= L * Hw) return;
    int t = idx / Hw, q = idx - t * Hw;
    uint64_t m = 0;
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
__device__ __forceinline__ void hist_add(const EdgeArgs &a, uint64_t *hist, int idx, uint64_t v,
                                         int64_t g) {
    if (!v) return;
    if (a.hist_in_lds) {
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

// Accumulate the triangle-set gathers of member k: X_i(t, .) += |T_ik^.|,
// X_j(t, .) += |T_jk^.|, Y(t, .) += d_k^.
__device__ __forceinline__ void gather_member(const EdgeArgs &a, int32_t k, int64_t s_i, int64_t s_j,
                                              uint64_t *Xi, uint64_t *Xj, uint64_t *Y) {
    const int L = a.L;
    uint32_t eik = a.neid[s_i], ejk = a.neid[s_j];
    int t = a.ntype[k];
    for (int t2 = 0; t2 < L; ++t2) {
        uint32_t vi = a.tri[(size_t)eik * L + t2];
        uint32_t vj = a.tri[(size_t)ejk * L + t2];
        uint32_t vy = a.tdeg[(size_t)k * L + t2];
        if (vi) atomicAdd((unsigned long long *)&Xi[t * L + t2], (unsigned long long)vi);
        if (vj) atomicAdd((unsigned long long *)&Xj[t * L + t2], (unsigned long long)vj);
        if (vy) atomicAdd((unsigned long long *)&Y[t * L + t2], (unsigned long long)vy);
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
    uint32_t *Th;           // hub members, unordered
    uint32_t *Tl;           // low members, ascending
    uint32_t *meta;         // [0] |Tl| [1] |Th| [2] first word of Tm [3] last word
    uint32_t *wave_cnt;     // ordered_append scratch
};

// Build T (hub mask/list and sorted low list) and the gathers X_i, X_j, Y.
template <int NT>
__device__ void edge_build(const EdgeArgs &a, int32_t i, int32_t j, const EdgeShared &S, int tid) {
    const int L = a.L, LL = L * L;
    const int Hw = a.Hw;
    const int32_t base = a.hub_base;
    for (int q = tid; q < 4 * LL; q += NT) S.Xi[q] = 0;
    for (int q = tid; q < Hw; q += NT) S.Tm[q] = 0;
    if (tid == 0) {
        S.meta[0] = 0;
        S.meta[1] = 0;
        S.meta[2] = 0xffffffffu;
        S.meta[3] = 0;
    }
    group_sync<NT>();
    const int64_t ib = a.nrp[i], ie = a.nrp[i + 1], jb = a.nrp[j], je = a.nrp[j + 1];
    const int64_t ih = a.hstart[i], jh = a.hstart[j];

    // low members: probe the shorter low prefix in the longer one
    {
        bool i_small = (ih - ib) <= (jh - jb);
        int64_t sb = i_small ? ib : jb, se = i_small ? ih : jh;
        int64_t lb = i_small ? jb : ib, le = i_small ? jh : ih;
        uint32_t count = 0;
        for (int64_t p0 = sb; p0 < se; p0 += NT) {
            int64_t p = p0 + tid;
            bool found = false;
            int64_t q = 0;
            int32_t x = 0;
            if (p < se) {
                x = a.ncol[p];
                q = lower_bound(a.ncol, lb, le, x);
                found = q < le && a.ncol[q] == x;
            }
            uint32_t pos = ordered_append<NT>(found, count, S.wave_cnt);
            if (found) {
                S.Tl[pos] = (uint32_t)x;
                gather_member(a, x, i_small ? p : q, i_small ? q : p, S.Xi, S.Xj, S.Y);
            }
        }
        if (tid == 0) S.meta[0] = count;
    }

    // hub members
    const bool hi = i >= base, hj = j >= base;
    if (hi && hj) {
        const int hx_i = i - base, hx_j = j - base;
        for (int q = tid; q < Hw; q += NT) {
            uint64_t m = a.HB[(size_t)hx_i * Hw + q] & a.HB[(size_t)hx_j * Hw + q];
            S.Tm[q] = m;
            if (!m) continue;
            atomicMin(&S.meta[2], (uint32_t)q);
            atomicMax(&S.meta[3], (uint32_t)q);
            while (m) {
                int b = __ffsll((unsigned long long)m) - 1;
                m &= m - 1;
                int hk = q * 64 + b;
                int32_t k = base + hk;
                uint32_t pos = atomicAdd(&S.meta[1], 1u);
                S.Th[pos] = (uint32_t)k;
                gather_member(a, k, hub_slot(a, i, hx_i, hk), hub_slot(a, j, hx_j, hk), S.Xi, S.Xj, S.Y);
            }
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
            S.Th[pos] = (uint32_t)x;
            gather_member(a, x, i_small ? p : q, i_small ? q : p, S.Xi, S.Xj, S.Y);
        }
    }
    group_sync<NT>();
}

// Ordered typed clique pairs K over the triangle set built by edge_build.
template <int NT>
__device__ void edge_cliques(const EdgeArgs &a, const EdgeShared &S, int tid) {
    const int L = a.L;
    const int Hw = a.Hw;
    const int32_t base = a.hub_base;
    const uint32_t nTl = S.meta[0], nTh = S.meta[1];
    if (nTh) {
        const uint32_t wlo = S.meta[2], whi = S.meta[3];
        const uint32_t range = whi - wlo + 1;
        const bool pair_mode = nTh <= range;
        for (uint32_t idx = tid; idx < nTh; idx += NT) {
            int32_t k = (int32_t)S.Th[idx];
            int hk = k - base;
            int tk = a.ntype[k];
            uint32_t cnt[TG_MAX_L];
#pragma unroll
            for (int t = 0; t < TG_MAX_L; ++t) cnt[t] = 0;
            const uint64_t *rowk = a.HB + (size_t)hk * Hw;
            if (pair_mode) {
                for (uint32_t jdx = 0; jdx < nTh; ++jdx) {
                    int hx = (int)S.Th[jdx] - base;
                    if ((rowk[hx >> 6] >> (hx & 63)) & 1ull) {
                        int tx = a.ntype[base + hx];
#pragma unroll
                        for (int t = 0; t < TG_MAX_L; ++t) cnt[t] += (t == tx);
                    }
                }
            } else {
                for (uint32_t q = wlo; q <= whi; ++q) {
                    uint64_t v = rowk[q] & S.Tm[q];
                    if (!v) continue;
#pragma unroll
                    for (int t = 0; t < TG_MAX_L; ++t)
                        if (t < L) cnt[t] += (uint32_t)__popcll(v & a.TM[(size_t)t * Hw + q]);
                }
            }
#pragma unroll
            for (int t = 0; t < TG_MAX_L; ++t)
                if (t < L && cnt[t])
                    atomicAdd((unsigned long long *)&S.K[tk * L + t], (unsigned long long)cnt[t]);
        }
    }
    for (uint32_t idx = tid; idx < nTl; idx += NT) {
        int32_t r = (int32_t)S.Tl[idx];
        int tr = a.ntype[r];
        uint32_t cnt[TG_MAX_L], rev[TG_MAX_L];
#pragma unroll
        for (int t = 0; t < TG_MAX_L; ++t) { cnt[t] = 0; rev[t] = 0; }
        for (int64_t s = a.nrp[r]; s < a.nrp[r + 1]; ++s) {
            int32_t x = a.ncol[s];
            bool in;
            bool hubx = x >= base;
            if (hubx) {
                int hx = x - base;
                in = (S.Tm[hx >> 6] >> (hx & 63)) & 1ull;
            } else {
                uint32_t lo = 0, hi2 = nTl;
                while (lo < hi2) {
                    uint32_t mid = (lo + hi2) >> 1;
                    if ((int32_t)S.Tl[mid] < x) lo = mid + 1; else hi2 = mid;
                }
                in = lo < nTl && (int32_t)S.Tl[lo] == x;
            }
            if (!in) continue;
            int tx = a.ntype[x];
#pragma unroll
            for (int t = 0; t < TG_MAX_L; ++t) {
                cnt[t] += (t == tx);
                rev[t] += (hubx && t == tx);
            }
        }
#pragma unroll
        for (int t = 0; t < TG_MAX_L; ++t) {
            if (t >= L) continue;
            if (cnt[t]) atomicAdd((unsigned long long *)&S.K[tr * L + t], (unsigned long long)cnt[t]);
            if (rev[t]) atomicAdd((unsigned long long *)&S.K[t * L + tr], (unsigned long long)rev[t]);
        }
    }
    group_sync<NT>();
}

// Every orbit of Table 3 for edge e from the triangle, clique, cycle and
// aggregate quantities (inclusion-exclusion in the spirit of Theorem 1;
// Lemmas 1-4 for g4, g5, g9, g11), the row write and the histogram.
template <int NT>
__device__ void edge_derive(const EdgeArgs &a, int64_t e, int32_t i, int32_t j, const EdgeShared &S,
                            uint64_t *hist, int tid, uint32_t &bad) {
    const int64_t gid = a.batch ? (int64_t)a.ngraph[i] : 0;
    const int L = a.L;
    const uint64_t *Xi = S.Xi, *Xj = S.Xj, *Y = S.Y, *K = S.K;
    const int ta = a.ntype[i], tb = a.ntype[j];
    const int LL = L * L;
    const int P = L * (L + 1) / 2;
    const int W = 2 * L + 10 * P;
    const uint32_t *tri_e = a.tri + (size_t)e * L;
    const uint32_t *di = a.tdeg + (size_t)i * L;
    const uint32_t *dj = a.tdeg + (size_t)j * L;
    const uint64_t *Ai = a.A + (size_t)i * LL, *Aj = a.A + (size_t)j * LL;
    const uint64_t *Di = a.D + (size_t)i * LL, *Dj = a.D + (size_t)j * LL;
    const uint64_t *NC = a.NC + (size_t)e * LL;
    uint64_t *row = a.rows ? a.rows + (size_t)e * W : nullptr;
    const int n2 = (int)binom_small(L + 1, 2);
    const int n3 = (int)binom_small(L + 2, 3);
    const int n4 = (int)binom_small(L + 3, 4);

    if (tid == 0) hist_add(a, hist, rank2(ta, tb), 1, gid);
    for (int t = tid; t < L; t += NT) {
        int64_t nTt = tri_e[t];
        int64_t si = (int64_t)di[t] - nTt - (tb == t);
        int64_t sj = (int64_t)dj[t] - nTt - (ta == t);
        if (si < 0 || sj < 0) bad |= ST_INTERNAL;
        if (row) {
            row[t] = (uint64_t)nTt;
            row[L + t] = (uint64_t)(si + sj);
        }
        int r3 = rank3(ta, tb, t);
        hist_add(a, hist, n2 + r3, (uint64_t)(si + sj), gid);
        hist_add(a, hist, n2 + n3 + r3, (uint64_t)nTt, gid);
    }
    for (int p = tid; p < P; p += NT) {
        // pair (t, u), t <= u, from its lexicographic index
        int t = 0, rem = p;
        while (rem >= L - t) { rem -= L - t; ++t; }
        int u = t + rem;
        int64_t nT_[2] = {(int64_t)tri_e[t], (int64_t)tri_e[u]};
        int64_t Si[2], Sj[2];
        int xs[2] = {t, u};
        for (int z = 0; z < 2; ++z) {
            int x = xs[z];
            Si[z] = (int64_t)di[x] - nT_[z] - (tb == x);
            Sj[z] = (int64_t)dj[x] - nT_[z] - (ta == x);
        }
        // ordered quantities for (x, y) = (t, u) [z=0] and (u, t) [z=1]
        int64_t Ci[2], Cj[2], sgi[2], sgj[2], dli[2], dlj[2], Kx[2], Yx[2], Xix[2], NCx[2];
        for (int z = 0; z < 2; ++z) {
            int x = z ? u : t, y = z ? t : u;
            int zx = z, zy = 1 - z;  // index of x / y inside nT_, Si, Sj
            int q = x * L + y;
            int64_t xi = (int64_t)Xi[q], xj = (int64_t)Xj[q], kk = (int64_t)K[q], yy = (int64_t)Y[q];
            Ci[z] = xi - nT_[zx] * (tb == y) - kk;
            Cj[z] = xj - nT_[zx] * (ta == y) - kk;
            sgi[z] = (int64_t)Ai[q] - xi - (tb == x) * nT_[zy];
            sgj[z] = (int64_t)Aj[q] - xj - (ta == x) * nT_[zy];
            dli[z] = (int64_t)Di[q] - yy - (tb == x) * (int64_t)dj[y];
            dlj[z] = (int64_t)Dj[q] - yy - (ta == x) * (int64_t)di[y];
            Kx[z] = kk;
            Yx[z] = yy;
            Xix[z] = xi;
            NCx[z] = (int64_t)NC[q];
        }
        int64_t Cyc[2], Ei[2], Ej[2], Pi[2], Pj[2], Q[2];
        for (int z = 0; z < 2; ++z) Cyc[z] = NCx[z] - Ci[1 - z] - Cj[z] - Kx[z];
        for (int z = 0; z < 2; ++z) {
            int zb = 1 - z;
            int y = z ? t : u;
            int zx = z;
            Ei[z] = sgi[z] - Ci[zb];
            Ej[z] = sgj[z] - Cj[zb];
            Pi[z] = dli[z] - Si[zx] * (ta == y) - sgi[z] - Cyc[z];
            Pj[z] = dlj[z] - Sj[zx] * (tb == y) - sgj[z] - Cyc[zb];
            Q[z] = Yx[z] - Xix[z] - Cj[z] - nT_[zx] * (ta == y);
        }
        int64_t g[13];
        if (t == u) {
            if (Kx[0] & 1) bad |= ST_INTERNAL;
            if ((Ei[0] + Ej[0]) & 1) bad |= ST_INTERNAL;
            g[12] = Kx[0] / 2;
            g[6] = Cyc[0];
            g[10] = Ci[0] + Cj[0];
            g[7] = (Ei[0] + Ej[0]) / 2;
            g[3] = Pi[0] + Pj[0];
            g[8] = Q[0];
            g[4] = Si[0] * Sj[0] - g[6];
            g[5] = Si[0] * (Si[0] - 1) / 2 + Sj[0] * (Sj[0] - 1) / 2 - g[7];
            g[9] = nT_[0] * (Si[0] + Sj[0]) - g[10];
            g[11] = nT_[0] * (nT_[0] - 1) / 2 - g[12];
        } else {
            if (Ei[0] != Ei[1] || Ej[0] != Ej[1] || Kx[0] != Kx[1]) bad |= ST_INTERNAL;
            g[12] = Kx[0];
            g[6] = Cyc[0] + Cyc[1];
            g[10] = Ci[0] + Cj[0] + Ci[1] + Cj[1];
            g[7] = Ei[0] + Ej[0];
            g[3] = Pi[0] + Pi[1] + Pj[0] + Pj[1];
            g[8] = Q[0] + Q[1];
            g[4] = Si[0] * Sj[1] + Si[1] * Sj[0] - g[6];
            g[5] = Si[0] * Si[1] + Sj[0] * Sj[1] - g[7];
            g[9] = nT_[0] * (Si[1] + Sj[1]) + nT_[1] * (Si[0] + Sj[0]) - g[10];
            g[11] = nT_[0] * nT_[1] - g[12];
        }
        int r4 = rank4(ta, tb, t, u);
        // graphlet of each orbit (Sec. 4.4): h3 = g3+g4, h4 = g5, h5 = g6,
        // h6 = g7+g8+g9, h7 = g10+g11, h8 = g12
        const int hof[13] = {0, 0, 0, 3, 3, 4, 5, 6, 6, 6, 7, 7, 8};
        for (int o = 3; o <= 12; ++o) {
            if (g[o] < 0) bad |= ST_INTERNAL;
            uint64_t v = (uint64_t)g[o];
            if (row) row[2 * L + (o - 3) * P + p] = v;
            hist_add(a, hist, n2 + 2 * n3 + (hof[o] - 3) * n4 + r4, v, gid);
        }
    }
}

// LDS layout shared by both edge kernels (dynamic part), in uint64 words:
// [Xi Xj Y K : 4 L^2][hist : gw if in LDS][Tm : Hw] then uint32 lists.
__device__ __forceinline__ EdgeShared carve(const EdgeArgs &a, uint64_t *sm, uint32_t *meta,
                                            uint32_t *wave_cnt, uint64_t **hist, uint32_t *Th,
                                            uint32_t *Tl) {
    const int LL = a.L * a.L;
    EdgeShared S;
    S.Xi = sm;
    S.Xj = sm + LL;
    S.Y = sm + 2 * LL;
    S.K = sm + 3 * LL;
    *hist = sm + 4 * LL;
    S.Tm = *hist + (a.hist_in_lds ? a.gw : 0);
    S.Th = Th;
    S.Tl = Tl;
    S.meta = meta;
    S.wave_cnt = wave_cnt;
    return S;
}

// Light edges: one wave per edge (|T| <= min degree <= TCAP, lists in LDS).
__global__ void __launch_bounds__(64) k_edges_light(EdgeArgs a) {
    extern __shared__ uint64_t sm_edge[];
    __shared__ uint32_t meta[4];
    __shared__ uint32_t wave_cnt[1];
    const int LL = a.L * a.L;
    uint64_t *hist;
    uint64_t *after = sm_edge + 4 * LL + (a.hist_in_lds ? a.gw : 0) + a.Hw;
    uint32_t *Th = (uint32_t *)after;
    uint32_t *Tl = Th + TCAP;
    EdgeShared S = carve(a, sm_edge, meta, wave_cnt, &hist, Th, Tl);
    int lane = threadIdx.x;
    uint32_t bad = 0;
    if (a.hist_in_lds)
        for (int q = lane; q < a.gw; q += WAVE) hist[q] = 0;
    __syncthreads();
    auto one_edge = [&](int64_t e) {
        int32_t i = a.ei[e], j = a.ej[e];
        int64_t di = a.nrp[i + 1] - a.nrp[i], dj = a.nrp[j + 1] - a.nrp[j];
        if ((di < dj ? di : dj) > TCAP) {
            if (lane == 0)
                a.heavy_list[atomicAdd((unsigned long long *)&a.counters[C_EDGE_HEAVY], 1ull)] =
                    (uint32_t)e;
            return;
        }
        edge_build<WAVE>(a, i, j, S, lane);
        edge_cliques<WAVE>(a, S, lane);
        edge_derive<WAVE>(a, e, i, j, S, hist, lane, bad);
        __syncthreads();
    };
    if (!a.batch) {
        for (int64_t e = blockIdx.x; e < a.m; e += gridDim.x) one_edge(e);
        if (a.hist_in_lds)
            for (int q = lane; q < a.gw; q += WAVE)
                if (hist[q]) atomicAdd((unsigned long long *)&a.gacc[q], (unsigned long long)hist[q]);
    } else {
        // chunks of consecutive edges (the edges of one graph are
        // contiguous); the histogram is flushed into a graph's own vector
        // whenever the graph changes and at the end of each chunk
        auto flush = [&](int64_t g) {
            if (!a.hist_in_lds) return;
            const int Lg = a.gL[g];
            uint64_t *dst = a.gacc + a.goff[g];
            for (int q = lane; q < a.gw; q += WAVE) {
                uint64_t v = hist[q];
                if (!v) continue;
                int jq = remap_global(q, a.L, Lg);
                if (jq < 0) bad |= ST_INTERNAL;
                else atomicAdd((unsigned long long *)&dst[jq], (unsigned long long)v);
                hist[q] = 0;
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
            }
            flush(cur);
        }
    }
    bad = wave_or(bad);
    if (lane == 0 && bad) atomicOr(a.status, bad);
}

// Heavy edges: one 256-thread workgroup per edge, pulled from a queue; the
// low list lives in a global buffer of n entries private to the workgroup,
// the hub list (at most H entries) in LDS.
__global__ void __launch_bounds__(EDGE_THREADS_HEAVY) k_edges_heavy(EdgeArgs a) {
    extern __shared__ uint64_t sm_edgeh[];
    __shared__ uint32_t meta[4];
    __shared__ uint32_t wave_cnt[EDGE_THREADS_HEAVY / WAVE];
    __shared__ uint64_t s_idx;
    const int NT = EDGE_THREADS_HEAVY;
    const int LL = a.L * a.L;
    uint64_t *hist;
    uint64_t *after = sm_edgeh + 4 * LL + (a.hist_in_lds ? a.gw : 0) + a.Hw;
    uint32_t *Th = (uint32_t *)after;
    uint32_t *Tl = a.tbuf + (size_t)blockIdx.x * (size_t)a.n;
    EdgeShared S = carve(a, sm_edgeh, meta, wave_cnt, &hist, Th, Tl);
    int tid = threadIdx.x;
    uint32_t bad = 0;
    if (a.hist_in_lds)
        for (int q = tid; q < a.gw; q += NT) hist[q] = 0;
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
        edge_build<NT>(a, i, j, S, tid);
        __threadfence_block();
        __syncthreads();
        edge_cliques<NT>(a, S, tid);
        edge_derive<NT>(a, e, i, j, S, hist, tid, bad);
        __threadfence_block();
        __syncthreads();
    }
    if (a.hist_in_lds)
        for (int q = tid; q < a.gw; q += NT)
            if (hist[q]) atomicAdd((unsigned long long *)&a.gacc[q], (unsigned long long)hist[q]);
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
    k_hub_types<<<(unsigned)((L * Hw + 255) / 256), 256, 0, st>>>(ntype, n, H, Hw, L, TM);
    return hipGetLastError();
}

size_t edge_lds_bytes(const EdgeArgs &args, bool heavy) {
    int LL = args.L * args.L;
    size_t sh = (size_t)(4 * LL + (args.hist_in_lds ? args.gw : 0) + args.Hw) * sizeof(uint64_t);
    if (!heavy) sh += (size_t)2 * TCAP * sizeof(uint32_t);
    else sh += (size_t)(args.hub_base < args.n ? (args.n - args.hub_base) : 0) * sizeof(uint32_t);
    return sh;
}

hipError_t launch_edges(bool heavy, const EdgeArgs &args, unsigned grid, hipStream_t st) {
    if (grid == 0) return hipSuccess;
    size_t sh = edge_lds_bytes(args, heavy);
    if (!heavy) k_edges_light<<<grid, 64, sh, st>>>(args);
    else k_edges_heavy<<<grid, EDGE_THREADS_HEAVY, sh, st>>>(args);
    return hipGetLastError();
}

}  // namespace tg
