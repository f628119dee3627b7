// Position-aware typed graphlets (Sec. 5): the per-edge counts keep the
// role each of the two other nodes plays relative to the oriented edge
// (i, j) (i the edge's canonical first endpoint), and the global counts are
// kept per class of typed graphlets under type-preserving isomorphism (the
// Definition of a position-aware typed graphlet instance).  The kernels
// reuse everything the typed path computes up to the per-edge gathers
// (triangle sets, cliques K, gathers X_i, X_j, Y, node aggregates A, D and
// the non-induced 4-cycle counts NC); only the derivation differs: the
// oriented quantities of the typed derivation are written role by role
// instead of being summed over the two orders of a type pair (Sec. 5.2: the
// position-aware counts are what the enumeration finds before the lookup
// table merges type orders).
#include <hip/hip_runtime.h>

#include "tg_device.hpp"

namespace tg {

// co-lexicographic rank of the unordered pair {x, y} over any alphabet
__device__ __forceinline__ int64_t pair_rank(int64_t x, int64_t y) {
    if (x > y) { int64_t z = x; x = y; y = z; }
    return x + y * (y + 1) / 2;
}

__device__ __forceinline__ void pa_hist_add(const EdgeArgs &a, uint64_t *hist, int64_t idx,
                                            int64_t v) {
    if (!v) return;
    if (idx < 0 || idx >= a.gw) {  // a class index outside the layout: never expected
        atomicOr(a.status, ST_INTERNAL);
        return;
    }
    if (a.hist_in_lds) atomicAdd((unsigned long long *)&hist[idx], (unsigned long long)v);
    else atomicAdd((unsigned long long *)&a.gacc[idx], (unsigned long long)v);
}

// Global class indices (layout in include/tg.h): labellings are given as
// types by node position of each graphlet's drawing.
struct PaClass {
    int L, P;
    int64_t c3;            // C(L+2, 3)
    const PaLayout *pl;
    __device__ int64_t edge(int a, int b) const { return pl->gstart[0] + rank2(a, b); }
    __device__ int64_t path3(int c, int x, int y) const {
        return pl->gstart[1] + (int64_t)c * P + rank2(x, y);
    }
    __device__ int64_t tri(int a, int b, int c) const { return pl->gstart[2] + rank3(a, b, c); }
    __device__ int64_t path4(int t0, int t1, int t2, int t3) const {
        return pl->gstart[3] + pair_rank((int64_t)t0 * L + t1, (int64_t)t3 * L + t2);
    }
    __device__ int64_t star(int c, int x, int y, int z) const {
        return pl->gstart[4] + (int64_t)c * c3 + rank3(x, y, z);
    }
    __device__ int64_t cycle(int t0, int t1, int t2, int t3) const {
        return pl->gstart[5] + pair_rank(rank2(t0, t2), rank2(t1, t3));
    }
    __device__ int64_t tailed(int t0, int t1, int t2, int t3) const {
        return pl->gstart[6] + ((int64_t)t3 * L + t2) * P + rank2(t0, t1);
    }
    __device__ int64_t diamond(int t0, int t1, int t2, int t3) const {
        return pl->gstart[7] + (int64_t)rank2(t0, t2) * P + rank2(t1, t3);
    }
    __device__ int64_t clique(int a, int b, int c, int d) const {
        return pl->gstart[8] + rank4(a, b, c, d);
    }
};

// 3-node entries of type t: |T^t|, |S_i^t|, |S_j^t|.
__device__ __forceinline__ void pa_three(const EdgeArgs &a, const PaLayout &pl, const PaClass &C,
                                         int64_t e, int32_t i, int32_t j, int t, uint64_t *hist,
                                         uint32_t &bad, uint64_t *row) {
    const int L = a.L;
    const int ta = a.ntype[i], tb = a.ntype[j];
    const int64_t nT = a.tri[(size_t)e * L + t];
    const int LP = tri_pitch(L);
    const int64_t si = (int64_t)a.tdeg[(size_t)i * LP + t] - nT - (tb == t);
    const int64_t sj = (int64_t)a.tdeg[(size_t)j * LP + t] - nT - (ta == t);
    if (si < 0 || sj < 0) bad |= ST_INTERNAL;
    if (row) {
        row[pl.start[PB_TRI] + t] = (uint64_t)nT;
        row[pl.start[PB_PATH_I] + t] = (uint64_t)si;
        row[pl.start[PB_PATH_J] + t] = (uint64_t)sj;
    }
    pa_hist_add(a, hist, C.tri(ta, tb, t), nT);
    pa_hist_add(a, hist, C.path3(ta, t, tb), si);   // 3-path t-i-j, centre i
    pa_hist_add(a, hist, C.path3(tb, ta, t), sj);   // 3-path i-j-t, centre j
}

// 4-node entries of the unordered type pair p = {t <= u}: the ordered role
// pairs (t, u) and (u, t) of the ordered blocks and the entry of the
// unordered blocks.  The intermediate quantities are those of the typed
// derivation (with the same checks): C_i(x, y) = #{k in T^x, r in S_i^y,
// k ~ r}, Cyc(x, y) = #{k in S_i^x, r in S_j^y, k ~ r}, E_i(x, y) =
// #{k in S_i^x, r in S_i^y, k ~ r} (ordered), P_i(x, y) = #{k in S_i^x,
// r in I^y, k ~ r}, Q(x, y) = #{k in T^x, r in I^y, k ~ r}, K ordered
// clique pairs; g4, g5, g9, g11 follow from Lemmas 1-4 role by role.
template <typename XT, bool NARROW>
__device__ __forceinline__ void pa_pair(const EdgeArgs &a, const PaLayout &pl, const PaClass &C,
                                        int64_t e, int32_t i, int32_t j, int p, const XT *xyk,
                                        uint64_t *hist, uint32_t &bad, uint64_t *row) {
    using AT = typename std::conditional<NARROW, uint32_t, uint64_t>::type;
    const int L = a.L;
    const int LL = L * L;
    const int ta = a.ntype[i], tb = a.ntype[j];
    const XT *Xi = xyk, *Xj = Xi + LL, *Y = Xi + 2 * LL, *K = Xi + 3 * LL;
    const uint32_t *tri_e = a.tri + (size_t)e * L;
    const uint32_t *di = a.tdeg + (size_t)i * tri_pitch(L);
    const uint32_t *dj = a.tdeg + (size_t)j * tri_pitch(L);
    const AT *Ab = reinterpret_cast<const AT *>(a.A), *Db = reinterpret_cast<const AT *>(a.D);
    const AT *Ai = Ab + (size_t)i * LL, *Aj = Ab + (size_t)j * LL;
    const AT *Di = Db + (size_t)i * LL, *Dj = Db + (size_t)j * LL;
    const AT *NC = reinterpret_cast<const AT *>(a.NC) + (size_t)e * LL;
    int t = 0, rem = p;
    while (rem >= L - t) { rem -= L - t; ++t; }
    const int u = t + rem;
    const bool same = t == u;
    const int qa = t * L + u, qb = u * L + t;
    const int64_t nTt = tri_e[t], nTu = tri_e[u];
    const int64_t Sit = (int64_t)di[t] - nTt - (tb == t), Siu = (int64_t)di[u] - nTu - (tb == u);
    const int64_t Sjt = (int64_t)dj[t] - nTt - (ta == t), Sju = (int64_t)dj[u] - nTu - (ta == u);
    // ordered block entry (x, y) with its class index
    auto put = [&](int b, int x, int y, int64_t v, int64_t cls) {
        if (v < 0) bad |= ST_INTERNAL;
        if (row) row[pl.start[b] + x * L + y] = (uint64_t)v;
        pa_hist_add(a, hist, cls, v);
    };
    auto put_pair = [&](int b, int64_t v, int64_t cls) {
        if (v < 0) bad |= ST_INTERNAL;
        if (row) row[pl.start[b] + p] = (uint64_t)v;
        pa_hist_add(a, hist, cls, v);
    };
    const int64_t K0 = (int64_t)K[qa], K1 = (int64_t)K[qb];
    if (same && (K0 & 1)) bad |= ST_INTERNAL;
    if (!same && K0 != K1) bad |= ST_INTERNAL;
    const int64_t Xi0 = (int64_t)Xi[qa], Xi1 = (int64_t)Xi[qb];
    const int64_t Xj0 = (int64_t)Xj[qa], Xj1 = (int64_t)Xj[qb];
    const int64_t Ci0 = Xi0 - nTt * (tb == u) - K0, Ci1 = Xi1 - nTu * (tb == t) - K1;
    const int64_t Cj0 = Xj0 - nTt * (ta == u) - K0, Cj1 = Xj1 - nTu * (ta == t) - K1;
    const int64_t Cyc0 = (int64_t)NC[qa] - Ci1 - Cj0 - K0;
    const int64_t Cyc1 = (int64_t)NC[qb] - Ci0 - Cj1 - K1;
    const int64_t sgi0 = (int64_t)Ai[qa] - Xi0 - (tb == t) * nTu;
    const int64_t sgi1 = (int64_t)Ai[qb] - Xi1 - (tb == u) * nTt;
    const int64_t sgj0 = (int64_t)Aj[qa] - Xj0 - (ta == t) * nTu;
    const int64_t sgj1 = (int64_t)Aj[qb] - Xj1 - (ta == u) * nTt;
    const int64_t Ei0 = sgi0 - Ci1, Ei1 = sgi1 - Ci0;
    const int64_t Ej0 = sgj0 - Cj1, Ej1 = sgj1 - Cj0;
    if (same && ((Ei0 & 1) || (Ej0 & 1))) bad |= ST_INTERNAL;
    if (!same && (Ei0 != Ei1 || Ej0 != Ej1)) bad |= ST_INTERNAL;
    const int64_t Y0 = (int64_t)Y[qa], Y1 = (int64_t)Y[qb];
    const int64_t dli0 = (int64_t)Di[qa] - Y0 - (tb == t) * (int64_t)dj[u];
    const int64_t dli1 = (int64_t)Di[qb] - Y1 - (tb == u) * (int64_t)dj[t];
    const int64_t dlj0 = (int64_t)Dj[qa] - Y0 - (ta == t) * (int64_t)di[u];
    const int64_t dlj1 = (int64_t)Dj[qb] - Y1 - (ta == u) * (int64_t)di[t];
    const int64_t Pi0 = dli0 - Sit * (ta == u) - sgi0 - Cyc0;
    const int64_t Pi1 = dli1 - Siu * (ta == t) - sgi1 - Cyc1;
    const int64_t Pj0 = dlj0 - Sjt * (tb == u) - sgj0 - Cyc1;
    const int64_t Pj1 = dlj1 - Sju * (tb == t) - sgj1 - Cyc0;
    const int64_t Q0 = Y0 - Xi0 - Cj0 - nTt * (ta == u);
    const int64_t Q1 = Y1 - Xi1 - Cj1 - nTu * (ta == t);

    // ordered role pairs: (x, y) = (t, u), and (u, t) unless t == u
    for (int o = 0; o < (same ? 1 : 2); ++o) {
        const int x = o ? u : t, y = o ? t : u;
        const int64_t nTx = o ? nTu : nTt;
        const int64_t Six = o ? Siu : Sit, Siy = o ? Sit : Siu;
        const int64_t Sjy = o ? Sjt : Sju;
        const int64_t Ci = o ? Ci1 : Ci0, Cj = o ? Cj1 : Cj0, Cyc = o ? Cyc1 : Cyc0;
        const int64_t Pi = o ? Pi1 : Pi0, Pj = o ? Pj1 : Pj0, Q = o ? Q1 : Q0;
        put(PB_G3I, x, y, Pi, C.path4(y, x, ta, tb));               // r-k-i-j
        put(PB_G3J, x, y, Pj, C.path4(ta, tb, x, y));               // i-j-k-r
        put(PB_G4, x, y, Six * Sjy - Cyc, C.path4(x, ta, tb, y));   // Lemma 1; k-i-j-r
        put(PB_G6, x, y, Cyc, C.cycle(ta, tb, y, x));               // i-j-r-k-i
        put(PB_G8, x, y, Q, C.tailed(ta, tb, x, y));                // tail r at k
        put(PB_G9I, x, y, nTx * Siy - Ci, C.tailed(tb, x, ta, y));  // Lemma 3; tail at i
        put(PB_G9J, x, y, nTx * Sjy - Cj, C.tailed(ta, x, tb, y));  // tail at j
        put(PB_G10I, x, y, Ci, C.diamond(ta, tb, x, y));            // chord i-k
        put(PB_G10J, x, y, Cj, C.diamond(tb, ta, x, y));            // chord j-k
    }
    // unordered role pairs
    const int64_t g12 = same ? K0 / 2 : K0;
    const int64_t g7i = same ? Ei0 / 2 : Ei0, g7j = same ? Ej0 / 2 : Ej0;
    put_pair(PB_G5I, (same ? Sit * (Sit - 1) / 2 : Sit * Siu) - g7i, C.star(ta, tb, t, u));  // Lemma 2
    put_pair(PB_G5J, (same ? Sjt * (Sjt - 1) / 2 : Sjt * Sju) - g7j, C.star(tb, ta, t, u));
    put_pair(PB_G7I, g7i, C.tailed(t, u, ta, tb));
    put_pair(PB_G7J, g7j, C.tailed(t, u, tb, ta));
    put_pair(PB_G11, (same ? nTt * (nTt - 1) / 2 : nTt * nTu) - g12, C.diamond(ta, t, tb, u));  // Lemma 4
    put_pair(PB_G12, g12, C.clique(ta, tb, t, u));
}

// One thread per (edge, unordered type pair) over consecutive edges, rows
// assembled in LDS and written whole; the 3-node entries ride on the pairs
// p < L and the edge's own class on p = 0.
template <typename XT, bool NARROW>
__global__ void __launch_bounds__(256) k_derive_pa(EdgeArgs a, PaLayout pl) {
    extern __shared__ uint64_t sm_pa[];
    if (input_failed(a.status)) return;
    const int L = a.L;
    const int LL = L * L;
    const int P = L * (L + 1) / 2;
    const int W = pl.start[PB_NUM];
    const int hw = a.hist_in_lds ? a.gw : 0;
    uint64_t *hist = sm_pa;
    uint64_t *rbuf = a.rows ? sm_pa + hw : nullptr;
    for (int q = threadIdx.x; q < hw; q += blockDim.x) hist[q] = 0;
    __syncthreads();
    PaClass C{L, P, binom_small(L + 2, 3), &pl};
    uint32_t bad = 0;
    const XT *xyk = reinterpret_cast<const XT *>(a.xyk);
    const int EB = (int)blockDim.x / P;
    const int tid = threadIdx.x;
    const int b = tid / P, p = tid - b * P;
    for (int64_t e0 = (int64_t)blockIdx.x * EB; e0 < a.m; e0 += (int64_t)gridDim.x * EB) {
        const int nb = a.m - e0 < EB ? (int)(a.m - e0) : EB;
        if (b < nb) {
            const int64_t e = e0 + b;
            const int32_t i = a.ei[e], j = a.ej[e];
            uint64_t *row = rbuf ? rbuf + (size_t)b * W : nullptr;
            if (p == 0) pa_hist_add(a, hist, C.edge(a.ntype[i], a.ntype[j]), 1);
            if (p < L) pa_three(a, pl, C, e, i, j, p, hist, bad, row);
            pa_pair<XT, NARROW>(a, pl, C, e, i, j, p, xyk + (size_t)e * 4 * LL, hist, bad, row);
        }
        if (rbuf) {
            __syncthreads();
            uint64_t *dst = a.rows + (size_t)e0 * W;
            for (int q = tid; q < nb * W; q += blockDim.x) dst[q] = rbuf[q];
            __syncthreads();
        }
    }
    __syncthreads();
    for (int q = tid; q < hw; q += blockDim.x) {
        const uint64_t v = hist[q];
        if (v) atomicAdd((unsigned long long *)&a.gacc[q], (unsigned long long)v);
    }
    if (bad) atomicOr(a.status, bad);
}

// Global position-aware counts: each class's per-edge sum divided by its
// graphlet's edge count (each instance is met once from each of its edges).
__global__ void k_pa_finalize(const uint64_t *__restrict__ acc, PaLayout pl,
                              uint64_t *__restrict__ out, uint32_t *__restrict__ status) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= pl.gstart[9] || input_failed(status)) return;
    int h = 0;
    while (q >= pl.gstart[h + 1]) ++h;
    const uint64_t E[9] = {1, 2, 3, 3, 3, 4, 4, 5, 6};
    const uint64_t v = acc[q];
    if (v % E[h]) atomicOr(status, ST_NOT_DIVISIBLE);
    out[q] = v / E[h];
}

static int64_t binom_h(int64_t n, int r) {
    if (n < r) return 0;
    int64_t v = 1;
    for (int k = 1; k <= r; ++k) v = v * (n - r + k) / k;
    return v;
}

PaLayout pa_layout(int L) {
    PaLayout pl;
    const int P = L * (L + 1) / 2, LL = L * L;
    int s = 0;
    for (int b = 0; b < PB_NUM; ++b) {
        pl.start[b] = s;
        const bool pair = b == PB_G5I || b == PB_G5J || b == PB_G7I || b == PB_G7J ||
                          b == PB_G11 || b == PB_G12;
        s += b <= PB_PATH_J ? L : pair ? P : LL;
    }
    pl.start[PB_NUM] = s;
    const int64_t sizes[9] = {P,
                              (int64_t)L * P,
                              binom_h(L + 2, 3),
                              binom_h((int64_t)LL + 1, 2),
                              (int64_t)L * binom_h(L + 2, 3),
                              binom_h((int64_t)P + 1, 2),
                              (int64_t)LL * P,
                              (int64_t)P * P,
                              binom_h(L + 3, 4)};
    pl.gstart[0] = 0;
    for (int h = 0; h < 9; ++h) pl.gstart[h + 1] = pl.gstart[h] + sizes[h];
    return pl;
}

hipError_t launch_derive_pa(const EdgeArgs &args, const PaLayout &pl, unsigned grid,
                            hipStream_t st) {
    if (grid == 0 || args.m == 0) return hipSuccess;
    const int P = args.L * (args.L + 1) / 2;
    const size_t hw = args.hist_in_lds ? (size_t)args.gw : 0;
    const size_t rw = args.rows ? (size_t)(256 / P) * pl.start[PB_NUM] : 0;
    const size_t sh = (hw + rw) * sizeof(uint64_t);
    if (args.xyk_u32 && args.agg_u32) k_derive_pa<uint32_t, true><<<grid, 256, sh, st>>>(args, pl);
    else if (args.agg_u32) k_derive_pa<uint64_t, true><<<grid, 256, sh, st>>>(args, pl);
    else k_derive_pa<uint64_t, false><<<grid, 256, sh, st>>>(args, pl);
    return hipGetLastError();
}

hipError_t launch_pa_finalize(const uint64_t *acc, const PaLayout &pl, uint64_t *out,
                              uint32_t *status, hipStream_t st) {
    const int64_t w = pl.gstart[9];
    if (w <= 0) return hipSuccess;
    k_pa_finalize<<<(unsigned)((w + 255) / 256), 256, 0, st>>>(acc, pl, out, status);
    return hipGetLastError();
}

}  // namespace tg
