// Typed-graphlet spectral node embeddings (Alg. 5).  For a typed graphlet
// H, each edge weighs the number of instances of H that contain it
// (`k_graphlet_weights`, read off the per-edge typed rows).  Sec. 8.8 runs
// the algorithm on every connected component of the typed-graphlet graph
// G^H (the edges of nonzero weight): a component's embedding is the
// eigenvectors of the dim smallest eigenvalues of its normalised Laplacian
// L = I - D^{-1/2} W D^{-1/2}, rows scaled to unit length.
//
// Components come from a hook-and-compress pass (each root hooks onto the
// smaller root of an edge's other end, so every component ends up named by
// its smallest node id), then a stable sort of the nodes by component.
// Components of at most DENSE_MAX nodes -- on power-law inputs nearly all
// but the giant one -- are solved together, one workgroup each: the dense
// S = D^{-1/2} W D^{-1/2} of the component in LDS and a cyclic Jacobi
// eigensolver.  A larger component runs Chebyshev-filtered subspace
// iteration on M = (S + I) / 2 (spectrum in [0, 1]; its largest
// eigenvalues are the wanted ones) with a block of p = dim + oversample
// vectors: each iteration filters the block with a Chebyshev polynomial
// of M that damps [0, b] (b the block's smallest Ritz value) and keeps the
// top of the spectrum, orthonormalises it (eigen-decomposition of its Gram
// matrix, twice), and takes Ritz vectors (eigen-decomposition of its
// projection of M), until the dim wanted residuals ||M x - theta x|| fall
// below the tolerance.  All of it runs in this file's kernels: a weighted
// SpMM over the CSR restricted to the component (one wave per row, the
// block stored row-major so a neighbour's row is one coalesced read),
// tiled tall-skinny Gram products with a fixed-order reduction, and a
// one-workgroup Jacobi eigensolver for the p x p matrices.  Nodes of zero
// weighted degree are in no instance of H and no component: their rows
// stay zero.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <vector>

#include "tg_device.hpp"

namespace tg {
namespace {

constexpr int EMB_MAX_P = 256;     // largest block (dim + oversample)
constexpr int DENSE_MAX = 64;      // largest component solved densely in LDS
constexpr int GRAM_ROWS = 2048;    // rows per Gram partial
constexpr int GRAM_TILE = 32;

// ------------------------------------------------------ edge weights

// W_e = instances of the typed graphlet (h, sorted type multiset ms) that
// contain edge e: the orbits of h at the type pair (or type) that completes
// the edge's endpoint types to ms.
__global__ void k_graphlet_weights(const uint64_t *__restrict__ rows, int64_t m, int L,
                                   const int64_t *__restrict__ uv, const uint8_t *__restrict__ types,
                                   int h, int k, int4 ms, uint64_t *__restrict__ w) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= m) return;
    const int a = types[uv[2 * e]], b = types[uv[2 * e + 1]];
    int rest[4] = {ms.x, ms.y, ms.z, ms.w};
    int cnt = k;
    // remove a and b from the multiset
    bool ok = true;
    for (int x = 0; x < 2 && ok; ++x) {
        const int v = x == 0 ? a : b;
        int at = -1;
        for (int q = 0; q < cnt; ++q)
            if (rest[q] == v) { at = q; break; }
        if (at < 0) ok = false;
        else {
            for (int q = at; q + 1 < cnt; ++q) rest[q] = rest[q + 1];
            --cnt;
        }
    }
    uint64_t v = 0;
    if (ok) {
        const uint64_t *row = rows + (size_t)e * (2 * L + 10 * (L * (L + 1) / 2));
        if (h == 0) {
            v = 1;
        } else if (h <= 2) {
            v = row[(h == 1 ? L : 0) + rest[0]];
        } else {
            const int t = rest[0] < rest[1] ? rest[0] : rest[1];
            const int u = rest[0] < rest[1] ? rest[1] : rest[0];
            const int P = L * (L + 1) / 2;
            const int p = t * L - t * (t - 1) / 2 + (u - t);
            const int first = h == 3 ? 3 : h == 4 ? 5 : h == 5 ? 6 : h == 6 ? 7 : h == 7 ? 10 : 12;
            const int last = h == 3 ? 4 : h == 4 ? 5 : h == 5 ? 6 : h == 6 ? 9 : h == 7 ? 11 : 12;
            for (int o = first; o <= last; ++o) v += row[2 * L + (o - 3) * P + p];
        }
    }
    w[e] = v;
}

// ------------------------------------------------ weighted CSR, degrees

// Entries above the diagonal per row (cnt[n] = 0 closes the scan); a row
// pointer that is not monotone inside [0, nnz] flags the status word.
__global__ void k_emb_upper(const int64_t *__restrict__ rp, const int32_t *__restrict__ col,
                            int64_t n, int64_t nnz, int64_t *__restrict__ cnt,
                            uint32_t *__restrict__ status) {
    const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u == 0) {
        cnt[n] = 0;
        if (rp[0] != 0 || rp[n] != nnz) atomicOr(status, ST_UNSORTED);
    }
    if (u >= n) return;
    const int64_t b = rp[u], e = rp[u + 1];
    if (b < 0 || e < b || e > nnz) {
        cnt[u] = 0;
        atomicOr(status, ST_UNSORTED);
        return;
    }
    cnt[u] = e - upper_bound(col, b, e, (int32_t)u);
}

// One wave per row: the weight of every slot (its canonical edge's weight),
// the row's weighted degree and its scale D^{-1/2} (0 for degree 0).
__global__ void k_emb_slots(const int64_t *__restrict__ rp, const int32_t *__restrict__ col,
                            int64_t n, int64_t m, const int64_t *__restrict__ eoff,
                            const uint64_t *__restrict__ w, double *__restrict__ wslot,
                            double *__restrict__ sc, uint64_t *__restrict__ deg,
                            uint32_t *__restrict__ status) {
    const int lane = lane_id();
    const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x / WAVE);
    for (int64_t u = (int64_t)blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE; u < n;
         u += nwaves) {
        const int64_t b = rp[u], end = rp[u + 1];
        const int64_t first_up = end - (eoff[u + 1] - eoff[u]);
        uint64_t d = 0;
        uint32_t bad = 0;
        for (int64_t s = b + lane; s < end; s += WAVE) {
            const int32_t x = col[s];
            int64_t e;
            if (x < 0 || x >= n || x == u || (s > b && col[s - 1] >= x)) {
                bad = 1;
                e = -1;
            } else if (x > u) {
                e = eoff[u] + (s - first_up);
            } else {
                const int64_t xb = rp[x], xe = rp[x + 1];
                const int64_t pos = lower_bound(col, xb, xe, (int32_t)u);
                if (pos >= xe || col[pos] != (int32_t)u) { bad = 1; e = -1; }
                else e = eoff[x] + (pos - (xe - (eoff[x + 1] - eoff[x])));
            }
            if (e >= m) e = -1;     // only after a failed check elsewhere
            if (e < 0) bad = 1;
            const uint64_t we = e >= 0 ? w[e] : 0;
            wslot[s] = (double)we;
            d += we;
        }
        d = wave_sum_u64(d);
        bad = wave_or(bad);
        if (lane == 0) {
            deg[u] = d;
            sc[u] = d > 0 ? 1.0 / sqrt((double)d) : 0.0;
            if (bad) atomicOr(status, ST_ASYMMETRIC);
        }
    }
}

__global__ void k_emb_edge_check(const int64_t *__restrict__ eoff, int64_t n, int64_t m,
                                 uint32_t *__restrict__ status) {
    if (eoff[n] != m) *status |= ST_EDGE_COUNT;
}

// --------------------------------------------------- components of G^H

__device__ __forceinline__ int32_t cc_find(const int32_t *parent, int32_t r) {
    // parents only ever decrease, so the walk ends
    for (;;) {
        const int32_t q = __hip_atomic_load(parent + r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (q == r) return r;
        r = q;
    }
}

__global__ void k_cc_init(int32_t *__restrict__ parent, int64_t n) {
    const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u < n) parent[u] = (int32_t)u;
}

// Every edge of nonzero weight whose ends have different roots hooks the
// larger root onto the smaller one; *changed records that some did.  One
// wave per row, lanes over its slots (each edge from its smaller end).
__global__ void k_cc_hook(const int64_t *__restrict__ rp, const int32_t *__restrict__ col,
                          const double *__restrict__ wslot, int64_t n, int32_t *parent,
                          uint32_t *__restrict__ changed) {
    const int lane = lane_id();
    const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x / WAVE);
    for (int64_t u = (int64_t)blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE; u < n;
         u += nwaves) {
        uint32_t hooked = 0;
        for (int64_t s = rp[u + 1] - 1 - lane; s >= rp[u]; s -= WAVE) {
            const int32_t x = col[s];
            if (x <= u) break;                       // the rest of the row is below u
            if (wslot[s] == 0.0) continue;
            const int32_t a = cc_find(parent, (int32_t)u), b = cc_find(parent, x);
            if (a != b) {
                atomicMin(parent + (a > b ? a : b), a < b ? a : b);
                hooked = 1;
            }
        }
        hooked = wave_or(hooked);
        if (lane == 0 && hooked) atomicOr(changed, 1u);
    }
}

__global__ void k_cc_compress(int32_t *parent, int64_t n) {
    const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u < n) parent[u] = cc_find(parent, (int32_t)u);
}

constexpr uint64_t CC_NONE = 0xFFFFFFFFull;   // sort key of a node in no component

// Sort keys: a node's component (its root), or CC_NONE; values: node ids.
// Also the per-node outputs that need no solve: component ids (-1 outside
// every component) and zero embedding rows outside every component.
__global__ void k_cc_keys(const int32_t *__restrict__ parent, const uint64_t *__restrict__ deg,
                          int64_t n, int dim, uint64_t *__restrict__ keys,
                          uint32_t *__restrict__ ids, int32_t *__restrict__ comp,
                          double *__restrict__ Z) {
    const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= n) return;
    const bool act = deg[u] > 0;
    keys[u] = act ? (uint64_t)parent[u] : CC_NONE;
    ids[u] = (uint32_t)u;
    if (comp) comp[u] = act ? parent[u] : -1;
    if (!act)
        for (int j = 0; j < dim; ++j) Z[(size_t)u * dim + j] = 0.0;
}

// flag[i] = 1 where sorted position i starts a component (flag[n] = 0).
__global__ void k_cc_flags(const uint64_t *__restrict__ key, int64_t n, int64_t *__restrict__ flag) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i > n) return;
    flag[i] = (i < n && key[i] != CC_NONE && (i == 0 || key[i] != key[i - 1])) ? 1 : 0;
}

// seg_start[c] = first sorted position of component c (seg_start[#c] =
// nact); loc[u] = u's position inside its component.  segx is the
// exclusive scan of the flags: position i is in component segx[i+1] - 1.
__global__ void k_cc_segments(const int64_t *__restrict__ flag, const int64_t *__restrict__ segx,
                              int64_t n, int64_t nact, int64_t *__restrict__ seg_start) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) seg_start[segx[n]] = nact;
    if (i < nact && flag[i]) seg_start[segx[i]] = i;
}

__global__ void k_cc_loc(const int64_t *__restrict__ segx, const int64_t *__restrict__ seg_start,
                         const uint32_t *__restrict__ order, int64_t nact,
                         int32_t *__restrict__ loc) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nact) loc[order[i]] = (int32_t)(i - seg_start[segx[i + 1] - 1]);
}

// ------------------------------------------------------------- blocks

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    // SplitMix64 finaliser (Steele, Lea and Flood, 2014)
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Random start block in [-1, 1) (s rows of a component, counter-based).
__global__ void k_emb_random(double *__restrict__ X, int64_t s, int p, uint64_t seed) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= s * p) return;
    const uint64_t r = mix64(seed ^ mix64((uint64_t)q));
    X[q] = (double)(r >> 11) * (1.0 / 9007199254740992.0) * 2.0 - 1.0;
}

// out = alpha * (S X) + beta * X + gamma * Z, S = D^{-1/2} W D^{-1/2}
// restricted to one component: local row r is node nodes[r], a neighbour x
// is local row loc[x].  One wave per row, each lane a set of the p columns.
__global__ void __launch_bounds__(256)
k_emb_spmm(const int64_t *__restrict__ rp, const int32_t *__restrict__ col,
           const double *__restrict__ wslot, const double *__restrict__ sc,
           const uint32_t *__restrict__ nodes, const int32_t *__restrict__ loc, int64_t n, int p,
           const double *__restrict__ X, const double *__restrict__ Z, double alpha, double beta,
           double gamma, double *__restrict__ out) {
    constexpr int CPL = EMB_MAX_P / WAVE;   // columns per lane
    const int lane = lane_id();
    const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x / WAVE);
    for (int64_t r = (int64_t)blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE; r < n;
         r += nwaves) {
        const int64_t u = nodes[r];
        double acc[CPL];
#pragma unroll
        for (int c = 0; c < CPL; ++c) acc[c] = 0.0;
        const double su = sc[u];
        {
            for (int64_t s = rp[u]; s < rp[u + 1]; ++s) {
                const int32_t x = col[s];
                const double coef = wslot[s] * sc[x];
                if (coef == 0.0) continue;
                const double *xr = X + (size_t)loc[x] * p;
#pragma unroll
                for (int c = 0; c < CPL; ++c) {
                    const int j = lane + c * WAVE;
                    if (j < p) acc[c] += coef * xr[j];
                }
            }
        }
        const double *xu = X + (size_t)r * p;
        const double *zu = Z ? Z + (size_t)r * p : nullptr;
        double *ou = out + (size_t)r * p;
#pragma unroll
        for (int c = 0; c < CPL; ++c) {
            const int j = lane + c * WAVE;
            if (j < p) {
                double v = alpha * su * acc[c] + beta * xu[j];
                if (zu) v += gamma * zu[j];
                ou[j] = v;
            }
        }
    }
}

// Partial Gram tiles: part[chunk][i][j] = sum over the chunk's rows r of
// A[r][i] * B[r][j], one 32 x 32 output tile per workgroup.
__global__ void __launch_bounds__(256)
k_emb_gram_part(const double *__restrict__ A, const double *__restrict__ B, int64_t n, int p,
                double *__restrict__ part) {
    __shared__ double sa[GRAM_TILE][GRAM_TILE + 1];
    __shared__ double sb[GRAM_TILE][GRAM_TILE + 1];
    const int tiles = (p + GRAM_TILE - 1) / GRAM_TILE;
    const int ti = blockIdx.y / tiles, tj = blockIdx.y % tiles;
    const int64_t r0 = (int64_t)blockIdx.x * GRAM_ROWS;
    const int64_t r1 = r0 + GRAM_ROWS < n ? r0 + GRAM_ROWS : n;
    const int tid = threadIdx.x;
    // each thread: 4 outputs (i = tid / 8, j = (tid % 8) * 4 + 0..3)
    const int oi = tid / 8, oj = (tid % 8) * 4;
    double acc[4] = {0, 0, 0, 0};
    for (int64_t rb = r0; rb < r1; rb += GRAM_TILE) {
        for (int q = tid; q < GRAM_TILE * GRAM_TILE; q += 256) {
            const int rr = q / GRAM_TILE, cc = q % GRAM_TILE;
            const int64_t r = rb + rr;
            const int ca = ti * GRAM_TILE + cc, cb = tj * GRAM_TILE + cc;
            sa[rr][cc] = (r < r1 && ca < p) ? A[(size_t)r * p + ca] : 0.0;
            sb[rr][cc] = (r < r1 && cb < p) ? B[(size_t)r * p + cb] : 0.0;
        }
        __syncthreads();
#pragma unroll 4
        for (int rr = 0; rr < GRAM_TILE; ++rr) {
            const double av = sa[rr][oi];
#pragma unroll
            for (int x = 0; x < 4; ++x) acc[x] += av * sb[rr][oj + x];
        }
        __syncthreads();
    }
    double *dst = part + (size_t)blockIdx.x * p * p;
    const int gi = ti * GRAM_TILE + oi;
#pragma unroll
    for (int x = 0; x < 4; ++x) {
        const int gj = tj * GRAM_TILE + oj + x;
        if (gi < p && gj < p) dst[(size_t)gi * p + gj] = acc[x];
    }
}

// C = sum of the partials, chunk by chunk in order (a fixed order: the same
// inputs give the same bits).
__global__ void k_emb_gram_sum(const double *__restrict__ part, int64_t chunks, int p,
                               double *__restrict__ C) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= p * p) return;
    double s = 0.0;
    for (int64_t c = 0; c < chunks; ++c) s += part[(size_t)c * p * p + q];
    C[q] = s;
}

// ----------------------------------------------- small symmetric eigen

template <int MAXP>
struct JacobiShared {
    int slot[MAXP];
    double rc[MAXP / 2], rs[MAXP / 2];
    int ri[MAXP / 2], rj[MAXP / 2];
    int order[MAXP];
    int rotated;
};

// Cyclic Jacobi on the p x p symmetric A (row-major, destroyed; LDS or
// global memory), the whole workgroup (256 threads) taking part: V gets
// the eigenvectors as columns and sh.order the column order that sorts the
// eigenvalues (A's final diagonal) descending.  Each rotation is the
// symmetric Schur step (Golub and Van Loan, Sec. 8.5.2) that annihilates
// a_ij; the p / 2 disjoint pairs of a round-robin step rotate together,
// rows first, then columns.  A pair is skipped once |a_ij| <= 1e-17
// sqrt(|a_ii a_jj|) (or a_ij = 0), and the sweeps stop after one that
// rotates nothing (at most max_sweeps).
template <int MAXP>
__device__ void jacobi_solve(double *A, double *V, int p, int max_sweeps, JacobiShared<MAXP> &sh) {
    const int tid = threadIdx.x;
    const int pe = p + (p & 1);              // even count (index p is a dummy when p is odd)
    const int half = pe / 2;
    for (int q = tid; q < p * p; q += 256) V[q] = (q / p == q % p) ? 1.0 : 0.0;
    for (int q = tid; q < pe; q += 256) sh.slot[q] = q;
    __syncthreads();
    for (int sweep = 0; sweep < max_sweeps; ++sweep) {
        if (tid == 0) sh.rotated = 0;
        __syncthreads();
        for (int step = 0; step < pe - 1; ++step) {
            // the pairs of this step: slot[k] with slot[pe - 1 - k]
            for (int k = tid; k < half; k += 256) {
                int i = sh.slot[k], j = sh.slot[pe - 1 - k];
                if (i > j) { const int t = i; i = j; j = t; }
                double c = 1.0, sn = 0.0;
                if (j < p) {
                    const double aij = A[i * p + j];
                    const double aii = A[i * p + i], ajj = A[j * p + j];
                    if (aij != 0.0 && fabs(aij) > 1e-17 * sqrt(fabs(aii) * fabs(ajj))) {
                        const double tau = (ajj - aii) / (2.0 * aij);
                        const double t = (tau >= 0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                        c = 1.0 / sqrt(1.0 + t * t);
                        sn = t * c;
                        sh.rotated = 1;
                    }
                }
                sh.ri[k] = i; sh.rj[k] = j; sh.rc[k] = c; sh.rs[k] = sn;
            }
            __syncthreads();
            // rows i, j of A <- J^T A
            for (int q = tid; q < half * p; q += 256) {
                const int k = q / p, x = q % p;
                if (sh.rs[k] == 0.0) continue;
                const int i = sh.ri[k], j = sh.rj[k];
                const double ai = A[i * p + x], aj = A[j * p + x];
                A[i * p + x] = sh.rc[k] * ai - sh.rs[k] * aj;
                A[j * p + x] = sh.rs[k] * ai + sh.rc[k] * aj;
            }
            __syncthreads();
            // columns i, j of A <- A J and of V <- V J
            for (int q = tid; q < half * p; q += 256) {
                const int k = q / p, x = q % p;
                if (sh.rs[k] == 0.0) continue;
                const int i = sh.ri[k], j = sh.rj[k];
                const double ai = A[x * p + i], aj = A[x * p + j];
                A[x * p + i] = sh.rc[k] * ai - sh.rs[k] * aj;
                A[x * p + j] = sh.rs[k] * ai + sh.rc[k] * aj;
                const double vi = V[x * p + i], vj = V[x * p + j];
                V[x * p + i] = sh.rc[k] * vi - sh.rs[k] * vj;
                V[x * p + j] = sh.rs[k] * vi + sh.rc[k] * vj;
            }
            __syncthreads();
            // the rotation annihilates a_ij: store the zero it stands for
            for (int k = tid; k < half; k += 256) {
                if (sh.rs[k] == 0.0) continue;
                A[sh.ri[k] * p + sh.rj[k]] = 0.0;
                A[sh.rj[k] * p + sh.ri[k]] = 0.0;
            }
            // round robin: slot 0 stays, the others move one place
            if (tid == 0) {
                const int last = sh.slot[pe - 1];
                for (int q = pe - 1; q > 1; --q) sh.slot[q] = sh.slot[q - 1];
                sh.slot[1] = last;
            }
            __syncthreads();
        }
        const int any = sh.rotated;
        __syncthreads();
        if (!any) break;
    }
    // sort descending by the diagonal (stable insertion sort, one thread)
    if (tid == 0) {
        for (int q = 0; q < p; ++q) sh.order[q] = q;
        for (int a = 1; a < p; ++a) {
            const int v = sh.order[a];
            const double dv = A[v * p + v];
            int b = a - 1;
            while (b >= 0 && A[sh.order[b] * p + sh.order[b]] < dv) {
                sh.order[b + 1] = sh.order[b];
                --b;
            }
            sh.order[b + 1] = v;
        }
    }
    __syncthreads();
}

// The p x p matrices of the subspace iteration (global memory, L2-resident,
// p <= 256): eigenvalues descending to w, matching eigenvectors to the
// columns of Vs (V is the unsorted accumulator).  One workgroup.
__global__ void __launch_bounds__(256)
k_emb_jacobi(double *__restrict__ A, double *__restrict__ V, double *__restrict__ w,
             double *__restrict__ Vs, int p, int max_sweeps) {
    __shared__ JacobiShared<EMB_MAX_P> sh;
    jacobi_solve<EMB_MAX_P>(A, V, p, max_sweeps, sh);
    for (int q = threadIdx.x; q < p; q += 256) w[q] = A[sh.order[q] * p + sh.order[q]];
    for (int q = threadIdx.x; q < p * p; q += 256) Vs[q] = V[(q / p) * p + sh.order[q % p]];
}

// Components of at most DENSE_MAX nodes, one workgroup each: the dense S of
// the component in LDS, its Jacobi eigen-decomposition, and the embedding
// rows of its nodes (the eigenvectors of the min(dim, s) largest
// eigenvalues of S, i.e. the smallest of L = I - S), with the eigenvalues
// of L to the root's row of evals.  Larger components return at once.
__global__ void __launch_bounds__(256)
k_emb_dense(const int64_t *__restrict__ rp, const int32_t *__restrict__ col,
            const double *__restrict__ wslot, const double *__restrict__ sc,
            const int64_t *__restrict__ seg_start, const uint32_t *__restrict__ order,
            const int32_t *__restrict__ loc, int dim, int raw, double *__restrict__ Z,
            double *__restrict__ evals) {
    __shared__ double A[DENSE_MAX * DENSE_MAX];
    __shared__ double V[DENSE_MAX * DENSE_MAX];
    __shared__ double nrm[DENSE_MAX];
    __shared__ JacobiShared<DENSE_MAX> sh;
    const int64_t start = seg_start[blockIdx.x];
    const int s = (int)(seg_start[blockIdx.x + 1] - start);
    if (s > DENSE_MAX) return;
    const uint32_t *nodes = order + start;
    const int tid = threadIdx.x, lane = lane_id(), wv = tid / WAVE;
    for (int q = tid; q < s * s; q += 256) A[q] = 0.0;
    __syncthreads();
    for (int r = wv; r < s; r += 256 / WAVE) {
        const int64_t u = nodes[r];
        const double su = sc[u];
        for (int64_t q = rp[u] + lane; q < rp[u + 1]; q += WAVE) {
            const int32_t x = col[q];
            const double coef = wslot[q] * su * sc[x];
            if (coef != 0.0) A[r * s + loc[x]] = coef;
        }
    }
    __syncthreads();
    jacobi_solve<DENSE_MAX>(A, V, s, 60, sh);
    const int k = dim < s ? dim : s;
    for (int r = tid; r < s; r += 256) {
        double q = 0.0;
        for (int j = 0; j < k; ++j) {
            const double v = V[r * s + sh.order[j]];
            q += v * v;
        }
        nrm[r] = raw ? 1.0 : q > 0 ? 1.0 / sqrt(q) : 0.0;
    }
    __syncthreads();
    for (int q = tid; q < s * dim; q += 256) {
        const int r = q / dim, j = q % dim;
        Z[(size_t)nodes[r] * dim + j] = j < k ? V[r * s + sh.order[j]] * nrm[r] : 0.0;
    }
    if (evals)
        for (int j = tid; j < k; j += 256)
            evals[(size_t)nodes[0] * dim + j] = 1.0 - A[sh.order[j] * s + sh.order[j]];
}

// Columns scaled: Q[:, j] = V[:, j] * f(sigma_j) with f = 1/sqrt (to
// orthonormalise by the Gram matrix's eigen-decomposition); columns whose
// sigma is not above 1e-24 sigma_max (singular values 1e-12 apart) are
// zeroed.
__global__ void k_emb_scale_cols(double *__restrict__ V, const double *__restrict__ sigma, int p) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= p * p) return;
    const int j = q % p;
    const double smax = sigma[0];
    const double sj = sigma[j];
    V[q] = (sj > 1e-24 * smax && sj > 0) ? V[q] / sqrt(sj) : 0.0;
}

// Y = X Q (n x p times p x p); a workgroup keeps a 32-column tile of Q in
// LDS and takes 8 rows at a time.
__global__ void __launch_bounds__(256)
k_emb_apply(const double *__restrict__ X, const double *__restrict__ Q, int64_t n, int p,
            double *__restrict__ Y) {
    extern __shared__ double sq[];   // p x 32
    const int tiles = (p + 31) / 32;
    const int tj = blockIdx.y;
    const int tid = threadIdx.x;
    for (int q = tid; q < p * 32; q += 256) {
        const int k = q / 32, c = q % 32;
        const int j = tj * 32 + c;
        sq[q] = j < p ? Q[(size_t)k * p + j] : 0.0;
    }
    __syncthreads();
    (void)tiles;
    const int ri = tid / 32, c = tid % 32;
    const int j = tj * 32 + c;
    for (int64_t r0 = (int64_t)blockIdx.x * 64; r0 < n && r0 < (int64_t)blockIdx.x * 64 + 64;
         r0 += 8) {
        const int64_t r = r0 + ri;
        if (r >= n) continue;
        const double *xr = X + (size_t)r * p;
        double acc = 0.0;
        for (int k = 0; k < p; ++k) acc += xr[k] * sq[k * 32 + c];
        if (j < p) Y[(size_t)r * p + j] = acc;
    }
}

// res[j] = ||MX[:, j] - theta_j X[:, j]||^2 partial sums per chunk, then
// summed: one wave per row range.
__global__ void __launch_bounds__(256)
k_emb_residual_part(const double *__restrict__ X, const double *__restrict__ MX,
                    const double *__restrict__ theta, int64_t n, int p,
                    double *__restrict__ part) {
    constexpr int CPL = EMB_MAX_P / WAVE;
    const int lane = lane_id();
    const int w = threadIdx.x / WAVE;
    __shared__ double red[4][EMB_MAX_P];
    double acc[CPL];
#pragma unroll
    for (int c = 0; c < CPL; ++c) acc[c] = 0.0;
    const int64_t r0 = (int64_t)blockIdx.x * GRAM_ROWS;
    const int64_t r1 = r0 + GRAM_ROWS < n ? r0 + GRAM_ROWS : n;
    for (int64_t r = r0 + w; r < r1; r += 4) {
#pragma unroll
        for (int c = 0; c < CPL; ++c) {
            const int j = lane + c * WAVE;
            if (j < p) {
                const double d = MX[(size_t)r * p + j] - theta[j] * X[(size_t)r * p + j];
                acc[c] += d * d;
            }
        }
    }
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
        const int j = lane + c * WAVE;
        if (j < p) red[w][j] = acc[c];
    }
    __syncthreads();
    for (int j = threadIdx.x; j < p; j += 256)
        part[(size_t)blockIdx.x * p + j] = red[0][j] + red[1][j] + red[2][j] + red[3][j];
}

__global__ void k_emb_residual_sum(const double *__restrict__ part, int64_t chunks, int p,
                                   double *__restrict__ res) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= p) return;
    double s = 0.0;
    for (int64_t c = 0; c < chunks; ++c) s += part[(size_t)c * p + j];
    res[j] = sqrt(s);
}

// Z[nodes[r]][0..dim) = X[r][0..dim) / its length (unscaled when raw);
// the component's eigenvalues of L (2 - 2 theta) to evals (its root's row).
__global__ void k_emb_output(const double *__restrict__ X, const uint32_t *__restrict__ nodes,
                             int64_t s, int p, int dim, int raw, const double *__restrict__ theta,
                             double *__restrict__ Z, double *__restrict__ evals) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r == 0 && evals)
        for (int j = 0; j < dim && j < p; ++j) evals[j] = 2.0 - 2.0 * theta[j];
    if (r >= s) return;
    const double *xr = X + (size_t)r * p;
    double q = 0.0;
    for (int j = 0; j < dim && j < p; ++j) q += xr[j] * xr[j];
    const double inv = raw ? 1.0 : q > 0 ? 1.0 / sqrt(q) : 0.0;
    double *zr = Z + (size_t)nodes[r] * dim;
    for (int j = 0; j < dim; ++j) zr[j] = j < p ? xr[j] * inv : 0.0;
}

// Workspace layout of the embedding.
struct EmbLayout {
    int p;
    int64_t chunks;
    size_t cnt, eoff, stmp, status, wslot, sc, deg, parent, keys, keys_tmp, ids, ids_tmp, sort_tmp,
        seg_start, loc, X, Y, Yp, Yn, MX, part, G, V, Vs, H, theta, sigma, res, total;
};

EmbLayout emb_layout(int64_t n, int64_t nnz, int dim) {
    EmbLayout y{};
    int p = dim + (dim / 4 > 8 ? dim / 4 : 8);
    if (p > EMB_MAX_P) p = EMB_MAX_P;
    y.p = p;
    y.chunks = (n + GRAM_ROWS - 1) / GRAM_ROWS;
    if (y.chunks < 1) y.chunks = 1;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o = (o + bytes + 255) & ~(size_t)255;
        return at;
    };
    y.cnt = take(sizeof(int64_t) * (size_t)(n + 1));
    y.eoff = take(sizeof(int64_t) * (size_t)(n + 1));
    y.stmp = take(sizeof(int64_t) * (size_t)(scan_tiles(n + 1) + 1));
    y.status = take(256);
    y.wslot = take(sizeof(double) * (size_t)(nnz > 0 ? nnz : 1));
    y.sc = take(sizeof(double) * (size_t)(n > 0 ? n : 1));
    y.deg = take(sizeof(uint64_t) * (size_t)(n > 0 ? n : 1));
    y.parent = take(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    y.keys = take(sizeof(uint64_t) * (size_t)(n > 0 ? n : 1));
    y.keys_tmp = take(sizeof(uint64_t) * (size_t)(n > 0 ? n : 1));
    y.ids = take(sizeof(uint32_t) * (size_t)(n > 0 ? n : 1));
    y.ids_tmp = take(sizeof(uint32_t) * (size_t)(n > 0 ? n : 1));
    y.sort_tmp = take(sort_tmp_need(n > 0 ? n : 1));
    y.seg_start = take(sizeof(int64_t) * (size_t)(n + 1));
    y.loc = take(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    const size_t blk = sizeof(double) * (size_t)(n > 0 ? n : 1) * p;
    y.X = take(blk);
    y.Y = take(blk);
    y.Yp = take(blk);
    y.Yn = take(blk);
    y.MX = take(blk);
    y.part = take(sizeof(double) * (size_t)y.chunks * p * p);
    y.G = take(sizeof(double) * (size_t)p * p);
    y.V = take(sizeof(double) * (size_t)p * p);
    y.Vs = take(sizeof(double) * (size_t)p * p);
    y.H = take(sizeof(double) * (size_t)p * p);
    y.theta = take(sizeof(double) * p);
    y.sigma = take(sizeof(double) * p);
    y.res = take(sizeof(double) * p);
    y.total = o;
    return y;
}

uint64_t mix64_host(uint64_t z) {
    // SplitMix64 finaliser (Steele, Lea and Flood, 2014), as mix64
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

unsigned row_grid(int64_t n) {
    int64_t b = (n + 3) / 4;
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

tg_status tg_graphlet_weights(const uint64_t *per_edge, int64_t m, int32_t L,
                              const int64_t *edge_uv, const uint8_t *types, int32_t graphlet,
                              const int32_t types_sorted[4], uint64_t *weights, void *stream) {
    if (L < 1 || L > TG_MAX_L) return TG_E_L_RANGE;
    if (m < 0 || graphlet < 0 || graphlet > 8 || !types_sorted || (m > 0 && (!per_edge || !edge_uv ||
                                                                          !types || !weights)))
        return TG_E_INVALID_ARG;
    const int k = graphlet == 0 ? 2 : graphlet <= 2 ? 3 : 4;
    int t[4] = {0, 0, 0, 0};
    for (int q = 0; q < k; ++q) {
        t[q] = types_sorted[q];
        if (t[q] < 0 || t[q] >= L || (q > 0 && t[q] < t[q - 1])) return TG_E_TYPE_RANGE;
    }
    if (m == 0) return TG_OK;
    hipStream_t st = (hipStream_t)stream;
    k_graphlet_weights<<<(unsigned)((m + 255) / 256), 256, 0, st>>>(
        per_edge, m, L, edge_uv, types, graphlet, k, make_int4(t[0], t[1], t[2], t[3]), weights);
    if (hipGetLastError() != hipSuccess) return TG_E_DEVICE;
    return hipStreamSynchronize(st) == hipSuccess ? TG_OK : TG_E_DEVICE;
}

size_t tg_embedding_workspace_bytes(int64_t n, int64_t nnz, int32_t dim) {
    if (n < 0 || nnz < 0 || dim < 1 || dim > EMB_MAX_P) return 0;
    return emb_layout(n, nnz, dim).total;
}

tg_status tg_graphlet_embedding(const int64_t *row_ptr, const int32_t *col, int64_t n, int64_t nnz,
                                const uint64_t *weights, int32_t dim, const tg_embed_opts *opts,
                                double *Z, double *eigenvalues, int32_t *component,
                                int32_t *iterations, void *workspace, size_t ws_bytes,
                                void *stream) {
    if (n < 1 || nnz < 0 || (nnz & 1) || dim < 1 || dim > EMB_MAX_P || !row_ptr || !Z ||
        (nnz > 0 && (!col || !weights)) || !workspace || ((uintptr_t)workspace & 255u))
        return TG_E_INVALID_ARG;
    if (n >= (int64_t(1) << 31)) return TG_E_TOO_LARGE;
    const EmbLayout y = emb_layout(n, nnz, dim);
    if (ws_bytes < y.total) return TG_E_WORKSPACE;
    int max_iter = opts && opts->max_iter > 0 ? opts->max_iter : 500;
    int degree = opts && opts->degree > 0 ? opts->degree : 10;
    const double tol = opts && opts->tol > 0 ? opts->tol : 1e-10;
    const uint64_t seed = opts ? opts->seed : 0;
    const int raw = opts && opts->raw ? 1 : 0;
    hipStream_t st = (hipStream_t)stream;
    char *w = static_cast<char *>(workspace);
    auto D = [&](size_t off) { return reinterpret_cast<double *>(w + off); };
    int64_t *cnt = reinterpret_cast<int64_t *>(w + y.cnt);
    int64_t *eoff = reinterpret_cast<int64_t *>(w + y.eoff);
    uint32_t *status = reinterpret_cast<uint32_t *>(w + y.status);
    uint64_t *deg = reinterpret_cast<uint64_t *>(w + y.deg);
    const int p0 = y.p;
    const int64_t m = nnz / 2;
#define EMB_CHK(x) do { if ((x) != hipSuccess) return TG_E_DEVICE; } while (0)
    // weighted CSR: canonical edge ids of the slots, their weights, degrees
    EMB_CHK(launch_fill_u64(reinterpret_cast<uint64_t *>(status), 0, 1, st));
    k_emb_upper<<<(unsigned)((n + 256) / 256), 256, 0, st>>>(row_ptr, col, n, nnz, cnt, status);
    EMB_CHK(hipGetLastError());
    EMB_CHK(launch_excl_scan(cnt, eoff, n + 1, reinterpret_cast<int64_t *>(w + y.stmp), nullptr, st));
    k_emb_edge_check<<<1, 1, 0, st>>>(eoff, n, m, status);
    EMB_CHK(hipGetLastError());
    uint32_t bits = 0;
    EMB_CHK(hipMemcpyAsync(&bits, status, sizeof(bits), hipMemcpyDeviceToHost, st));
    EMB_CHK(hipStreamSynchronize(st));
    if (bits) return TG_E_NOT_SIMPLE;
    k_emb_slots<<<row_grid(n), 256, 0, st>>>(row_ptr, col, n, m, eoff, weights, D(y.wslot), D(y.sc),
                                             deg, status);
    EMB_CHK(hipGetLastError());
    // active nodes (nonzero weighted degree) bound the block size
    std::vector<uint64_t> hdeg((size_t)n);
    EMB_CHK(hipMemcpyAsync(hdeg.data(), deg, sizeof(uint64_t) * (size_t)n, hipMemcpyDeviceToHost, st));
    EMB_CHK(hipMemcpyAsync(&bits, status, sizeof(bits), hipMemcpyDeviceToHost, st));
    EMB_CHK(hipStreamSynchronize(st));
    if (bits) return TG_E_NOT_SIMPLE;
    int64_t active = 0;
    for (uint64_t d : hdeg) active += d > 0;
    const unsigned rg_n = row_grid(n);
    auto grid_of = [](int64_t count) { return (unsigned)((count + 255) / 256); };
    int32_t *parent = reinterpret_cast<int32_t *>(w + y.parent);
    int32_t *loc = reinterpret_cast<int32_t *>(w + y.loc);
    int64_t *seg_start = reinterpret_cast<int64_t *>(w + y.seg_start);
    uint32_t *changed = status + 2;         // its own 8-byte word
    if (eigenvalues) EMB_CHK(launch_fill_u64(reinterpret_cast<uint64_t *>(eigenvalues), 0,
                                             n * (int64_t)dim, st));
    // components of G^H: hook and compress until no edge joins two roots
    k_cc_init<<<grid_of(n), 256, 0, st>>>(parent, n);
    EMB_CHK(hipGetLastError());
    for (int round = 0;; ++round) {
        if (round > 64) return TG_E_INTERNAL;    // parents strictly decrease: never reached
        uint32_t flag = 0;
        EMB_CHK(launch_fill_u64(reinterpret_cast<uint64_t *>(changed), 0, 1, st));
        k_cc_hook<<<rg_n, 256, 0, st>>>(row_ptr, col, D(y.wslot), n, parent, changed);
        k_cc_compress<<<grid_of(n), 256, 0, st>>>(parent, n);
        EMB_CHK(hipGetLastError());
        EMB_CHK(hipMemcpyAsync(&flag, changed, sizeof(flag), hipMemcpyDeviceToHost, st));
        EMB_CHK(hipStreamSynchronize(st));
        if (!flag) break;
    }
    // nodes sorted by component (stable: ascending ids inside one), the
    // components' start positions and each node's place in its component
    uint64_t *keys = reinterpret_cast<uint64_t *>(w + y.keys);
    uint32_t *ids = reinterpret_cast<uint32_t *>(w + y.ids);
    k_cc_keys<<<grid_of(n), 256, 0, st>>>(parent, deg, n, dim, keys, ids, component, Z);
    EMB_CHK(hipGetLastError());
    uint64_t *skeys = nullptr;
    uint32_t *order = nullptr;
    EMB_CHK(radix_sort(keys, reinterpret_cast<uint64_t *>(w + y.keys_tmp), ids,
                       reinterpret_cast<uint32_t *>(w + y.ids_tmp), n, 32, w + y.sort_tmp, nullptr,
                       st, &skeys, &order));
    int64_t *flags = cnt, *segx = eoff;    // both free once the slots are weighed
    k_cc_flags<<<grid_of(n + 1), 256, 0, st>>>(skeys, n, flags);
    EMB_CHK(hipGetLastError());
    EMB_CHK(launch_excl_scan(flags, segx, n + 1, reinterpret_cast<int64_t *>(w + y.stmp), nullptr, st));
    k_cc_segments<<<grid_of(n), 256, 0, st>>>(flags, segx, n, active, seg_start);
    k_cc_loc<<<grid_of(n), 256, 0, st>>>(segx, seg_start, order, active, loc);
    EMB_CHK(hipGetLastError());
    int64_t nseg = 0;
    EMB_CHK(hipMemcpyAsync(&nseg, segx + n, sizeof(nseg), hipMemcpyDeviceToHost, st));
    EMB_CHK(hipStreamSynchronize(st));
    if (iterations) *iterations = 0;
    if (nseg == 0) {
        EMB_CHK(hipStreamSynchronize(st));
        return TG_OK;
    }
    std::vector<int64_t> hseg((size_t)nseg + 1);
    EMB_CHK(hipMemcpyAsync(hseg.data(), seg_start, sizeof(int64_t) * (size_t)(nseg + 1),
                           hipMemcpyDeviceToHost, st));
    // every small component at once
    k_emb_dense<<<(unsigned)nseg, 256, 0, st>>>(row_ptr, col, D(y.wslot), D(y.sc), seg_start, order,
                                                loc, dim, raw, Z, eigenvalues);
    EMB_CHK(hipGetLastError());
    EMB_CHK(hipStreamSynchronize(st));

    // the large components, one after another
    double *X = D(y.X), *Y = D(y.Y), *Yp = D(y.Yp), *Yn = D(y.Yn), *MX = D(y.MX);
    double *G = D(y.G), *V = D(y.V), *Vs = D(y.Vs), *H = D(y.H);
    double *theta = D(y.theta), *sigma = D(y.sigma), *res = D(y.res), *part = D(y.part);
    bool all_converged = true;
    int most_iterations = 0;
    for (int64_t c = 0; c < nseg; ++c) {
        const int64_t cs = hseg[(size_t)c], ns = hseg[(size_t)c + 1] - cs;
        if (ns <= DENSE_MAX) continue;
        const uint32_t *nodes = order + cs;
        uint32_t root = 0;
        EMB_CHK(hipMemcpyAsync(&root, nodes, sizeof(root), hipMemcpyDeviceToHost, st));
        EMB_CHK(hipStreamSynchronize(st));
        const int p = (int)(ns < p0 ? ns : p0);
        const int64_t chunks = (ns + GRAM_ROWS - 1) / GRAM_ROWS;
        const unsigned rg = row_grid(ns);
        const int tiles = (p + GRAM_TILE - 1) / GRAM_TILE;
        auto gram = [&](const double *A, const double *B, double *C) -> hipError_t {
            k_emb_gram_part<<<dim3((unsigned)chunks, (unsigned)(tiles * tiles)), 256, 0, st>>>(
                A, B, ns, p, part);
            k_emb_gram_sum<<<(unsigned)((p * p + 255) / 256), 256, 0, st>>>(part, chunks, p, C);
            return hipGetLastError();
        };
        auto eig = [&](double *A) -> hipError_t {   // A destroyed; Vs, sigma filled
            k_emb_jacobi<<<1, 256, 0, st>>>(A, V, sigma, Vs, p, 60);
            return hipGetLastError();
        };
        auto apply = [&](const double *A, const double *Q, double *out) -> hipError_t {
            k_emb_apply<<<dim3((unsigned)((ns + 63) / 64), (unsigned)tiles), 256,
                          (size_t)p * 32 * sizeof(double), st>>>(A, Q, ns, p, out);
            return hipGetLastError();
        };
        auto spmm = [&](const double *A, const double *Zb, double alpha, double beta, double gamma,
                        double *out) -> hipError_t {
            k_emb_spmm<<<rg, 256, 0, st>>>(row_ptr, col, D(y.wslot), D(y.sc), nodes, loc, ns, p, A,
                                           Zb, alpha, beta, gamma, out);
            return hipGetLastError();
        };
        // orthonormalise A into out through the eigen-decomposition of A^T A
        auto orth = [&](const double *A, double *out) -> hipError_t {
            hipError_t e = gram(A, A, G);
            if (e != hipSuccess) return e;
            if ((e = eig(G)) != hipSuccess) return e;
            k_emb_scale_cols<<<(unsigned)((p * p + 255) / 256), 256, 0, st>>>(Vs, sigma, p);
            if ((e = hipGetLastError()) != hipSuccess) return e;
            return apply(A, Vs, out);
        };
        // Three rotating blocks (the Chebyshev recurrence needs two inputs
        // and an output), plus Yp (first orthonormalisation pass) and MX.
        double *R[3] = {X, Y, Yn};
        std::vector<double> h_theta((size_t)p), h_res((size_t)p);
        const int want = dim < p ? dim : p;
        // Rayleigh-Ritz on the orthonormal block Q: Ritz vectors to xo, M
        // times them to mo, Ritz values to theta (descending), residual
        // norms read back.
        auto rayleigh_ritz = [&](const double *Q, double *xo, double *mo) -> hipError_t {
            hipError_t e;
            if ((e = spmm(Q, nullptr, 0.5, 0.5, 0.0, MX)) != hipSuccess) return e;
            if ((e = gram(Q, MX, H)) != hipSuccess) return e;
            if ((e = eig(H)) != hipSuccess) return e;
            if ((e = apply(Q, Vs, xo)) != hipSuccess) return e;
            if ((e = apply(MX, Vs, mo)) != hipSuccess) return e;
            if ((e = hipMemcpyAsync(theta, sigma, sizeof(double) * p, hipMemcpyDeviceToDevice,
                                    st)) != hipSuccess)
                return e;
            k_emb_residual_part<<<(unsigned)chunks, 256, 0, st>>>(xo, mo, theta, ns, p, part);
            k_emb_residual_sum<<<1, 256, 0, st>>>(part, chunks, p, res);
            if ((e = hipGetLastError()) != hipSuccess) return e;
            if ((e = hipMemcpyAsync(h_theta.data(), theta, sizeof(double) * p,
                                    hipMemcpyDeviceToHost, st)) != hipSuccess)
                return e;
            if ((e = hipMemcpyAsync(h_res.data(), res, sizeof(double) * p, hipMemcpyDeviceToHost,
                                    st)) != hipSuccess)
                return e;
            return hipStreamSynchronize(st);
        };
        auto done = [&]() {
            for (int j = 0; j < want; ++j)
                if (!(h_res[(size_t)j] <= tol)) return false;
            return true;
        };
        // start: a random block, orthonormalised twice, and its Ritz vectors
        k_emb_random<<<(unsigned)((ns * p + 255) / 256), 256, 0, st>>>(R[0], ns, p,
                                                                      seed ^ mix64_host(root));
        EMB_CHK(hipGetLastError());
        EMB_CHK(orth(R[0], Yp));
        EMB_CHK(orth(Yp, R[1]));
        EMB_CHK(rayleigh_ritz(R[1], R[0], R[2]));
        int it = 0;
        bool converged = done();
        while (!converged && it < max_iter) {
            ++it;
            // Damp [0, bnd], bnd the block's smallest Ritz value: by
            // interlacing it is at most the p-th largest eigenvalue of M, so
            // no wanted one is damped.  The filter is scaled to 1 at the top
            // of the spectrum (1); its degree is capped so that its growth
            // stays below 1e6, which bounds the block's condition number.
            double bnd = h_theta[(size_t)p - 1];
            bnd = bnd < 1e-3 ? 1e-3 : bnd > 1.0 - 1e-9 ? 1.0 - 1e-9 : bnd;
            const double e = bnd / 2, cc = bnd / 2;
            const double t1 = (1.0 - cc) / e;
            int deg_f = degree;
            const double cap = std::acosh(1e6) / std::acosh(t1);
            if (cap < deg_f) deg_f = cap < 1 ? 1 : (int)cap;
            double *prev = R[0], *cur = R[1], *nxt = R[2];
            double rho_prev = 1.0, rho = t1;
            EMB_CHK(spmm(prev, nullptr, 0.5 / (e * t1), (0.5 - cc) / (e * t1), 0.0, cur));
            for (int j = 1; j < deg_f; ++j) {
                const double rho_next = 2 * t1 * rho - rho_prev;
                const double k1 = 2 * rho / (rho_next * e);
                EMB_CHK(spmm(cur, prev, k1 * 0.5, k1 * (0.5 - cc), -rho_prev / rho_next, nxt));
                rho_prev = rho;
                rho = rho_next;
                double *t = prev;
                prev = cur;
                cur = nxt;
                nxt = t;
            }
            // cur: the filtered block; prev and nxt are free
            EMB_CHK(orth(cur, Yp));
            EMB_CHK(orth(Yp, prev));
            EMB_CHK(rayleigh_ritz(prev, cur, nxt));
            R[0] = cur;
            R[1] = prev;
            R[2] = nxt;
            converged = done();
        }
        all_converged = all_converged && converged;
        most_iterations = it > most_iterations ? it : most_iterations;
        k_emb_output<<<grid_of(ns), 256, 0, st>>>(R[0], nodes, ns, p, dim, raw, theta, Z,
                                                  eigenvalues ? eigenvalues + (size_t)root * dim
                                                              : nullptr);
        EMB_CHK(hipGetLastError());
    }
    if (iterations) *iterations = most_iterations;
    EMB_CHK(hipStreamSynchronize(st));
#undef EMB_CHK
    return all_converged ? TG_OK : TG_E_NO_CONVERGENCE;
}

}  // extern "C"
