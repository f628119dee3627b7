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
// top of the spectrum, orthonormalises it (Cholesky QR, twice), and takes
// Ritz vectors (eigen-decomposition of its projection of M), until the dim
// wanted residuals ||M x - theta x|| fall below the tolerance; a block
// whose residuals stall (a cut inside an eigenvalue cluster) is widened.
// All of it runs in this file's kernels: an SpMM over the component's own
// CSR of S (a wave per row, long rows split into fixed items summed in
// order, the block stored row-major so a neighbour's row is one coalesced
// read), Gram products and block-times-matrix products on the fp64 matrix
// cores with a fixed-order reduction over row chunks, and one-workgroup
// Cholesky and block-Jacobi kernels for the p x p matrices (the packed
// upper triangle in LDS up to p = 192).  Nodes of zero weighted degree are
// in no instance of H and no component: their rows stay zero.
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

// A block widened from p to q columns: the old columns, then random ones.
__global__ void k_emb_widen(const double *__restrict__ X, int64_t s, int p, int q, uint64_t seed,
                            double *__restrict__ Y) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= s * q) return;
    const int64_t r = t / q;
    const int j = (int)(t % q);
    if (j < p) {
        Y[t] = X[(size_t)r * p + j];
    } else {
        const uint64_t z = mix64(seed ^ mix64((uint64_t)t));
        Y[t] = (double)(z >> 11) * (1.0 / 9007199254740992.0) * 2.0 - 1.0;
    }
}

// ------------------------------------------- S of one large component

// The component's own CSR of S = D^{-1/2} W D^{-1/2}, built once and read
// by every product: local row r is node nodes[r], only nonzero entries,
// columns as local rows.  A row of more than SPMM_CH nonzeros (a hub) is
// cut into items of SPMM_CH, each a wave's work in the products.
constexpr int SPMM_CH = 512;

__global__ void k_loc_len(const int64_t *__restrict__ rp, const double *__restrict__ wslot,
                          const uint32_t *__restrict__ nodes, int64_t ns, int64_t *__restrict__ len,
                          int64_t *__restrict__ hcnt) {
    const int lane = lane_id();
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        len[ns] = 0;
        hcnt[ns] = 0;
    }
    const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x / WAVE);
    for (int64_t r = (int64_t)blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE; r < ns;
         r += nwaves) {
        const int64_t u = nodes[r];
        uint64_t c = 0;
        for (int64_t q = rp[u] + lane; q < rp[u + 1]; q += WAVE) c += wslot[q] != 0.0;
        c = wave_sum_u64(c);
        if (lane == 0) {
            len[r] = (int64_t)c;
            hcnt[r] = c > (uint64_t)SPMM_CH ? (int64_t)((c + SPMM_CH - 1) / SPMM_CH) : 0;
        }
    }
}

__global__ void k_loc_fill(const int64_t *__restrict__ rp, const int32_t *__restrict__ col,
                           const double *__restrict__ wslot, const double *__restrict__ sc,
                           const uint32_t *__restrict__ nodes, const int32_t *__restrict__ loc,
                           int64_t ns, const int64_t *__restrict__ lrp, int32_t *__restrict__ lcol,
                           double *__restrict__ lval) {
    const int lane = lane_id();
    const uint64_t below = (1ull << lane) - 1;
    const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x / WAVE);
    for (int64_t r = (int64_t)blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE; r < ns;
         r += nwaves) {
        const int64_t u = nodes[r];
        const double su = sc[u];
        int64_t out = lrp[r];
        for (int64_t base = rp[u]; base < rp[u + 1]; base += WAVE) {
            const int64_t q = base + lane;
            const bool nz = q < rp[u + 1] && wslot[q] != 0.0;
            const uint64_t bal = __ballot(nz);
            if (nz) {
                const int32_t x = col[q];
                const int64_t at = out + __popcll(bal & below);
                lcol[at] = loc[x];
                lval[at] = wslot[q] * su * sc[x];
            }
            out += __popcll(bal);
        }
    }
}

__global__ void k_loc_items(const int64_t *__restrict__ hptr, int64_t ns, int32_t *__restrict__ hrow) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= ns) return;
    for (int64_t i = hptr[r]; i < hptr[r + 1]; ++i) hrow[i] = (int32_t)r;
}

// acc += the nonzeros [k0, k1) of S times X, a wave split into WAVE / GS
// groups that take every (WAVE / GS)-th nonzero, each lane CPL columns
// (j = lane % GS + c * GS); then the groups are summed in a fixed tree.
template <int GS, int CPL>
__device__ __forceinline__ void spmm_range(const int32_t *__restrict__ lcol,
                                           const double *__restrict__ lval, int64_t k0, int64_t k1,
                                           int p, const double *__restrict__ X, double (&acc)[CPL]) {
    constexpr int NG = WAVE / GS;
    const int lane = lane_id(), g = lane / GS, li = lane % GS;
#pragma unroll
    for (int c = 0; c < CPL; ++c) acc[c] = 0.0;
    int64_t k = k0 + g;
    for (; k + NG < k1; k += 2 * NG) {
        const int32_t c0 = lcol[k], c1 = lcol[k + NG];
        const double v0 = lval[k], v1 = lval[k + NG];
        const double *x0 = X + (size_t)c0 * p, *x1 = X + (size_t)c1 * p;
#pragma unroll
        for (int c = 0; c < CPL; ++c) {
            const int j = li + c * GS;
            if (j < p) {
                acc[c] += v0 * x0[j];
                acc[c] += v1 * x1[j];
            }
        }
    }
    if (k < k1) {
        const double v0 = lval[k];
        const double *x0 = X + (size_t)lcol[k] * p;
#pragma unroll
        for (int c = 0; c < CPL; ++c) {
            const int j = li + c * GS;
            if (j < p) acc[c] += v0 * x0[j];
        }
    }
#pragma unroll
    for (int c = 0; c < CPL; ++c)
        for (int off = GS; off < WAVE; off <<= 1) acc[c] += __shfl_xor(acc[c], off, WAVE);
}

// out = alpha * (S X) + beta * X + gamma * Zb on the rows of at most
// SPMM_CH nonzeros, one wave per row.
template <int GS, int CPL>
__global__ void __launch_bounds__(256)
k_spmm_rows(const int64_t *__restrict__ lrp, const int32_t *__restrict__ lcol,
            const double *__restrict__ lval, int64_t ns, int p, const double *__restrict__ X,
            const double *__restrict__ Zb, double alpha, double beta, double gamma,
            double *__restrict__ out) {
    const int lane = lane_id();
    const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x / WAVE);
    for (int64_t r = (int64_t)blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE; r < ns;
         r += nwaves) {
        const int64_t k0 = lrp[r], k1 = lrp[r + 1];
        if (k1 - k0 > SPMM_CH) continue;
        double acc[CPL];
        spmm_range<GS, CPL>(lcol, lval, k0, k1, p, X, acc);
        if (lane < GS) {
#pragma unroll
            for (int c = 0; c < CPL; ++c) {
                const int j = lane + c * GS;
                if (j < p) {
                    const size_t o = (size_t)r * p + j;
                    double v = alpha * acc[c] + beta * X[o];
                    if (Zb) v += gamma * Zb[o];
                    out[o] = v;
                }
            }
        }
    }
}

// Partial products of the items of the long rows: part[i][0..p).
template <int GS, int CPL>
__global__ void __launch_bounds__(256)
k_spmm_items(const int64_t *__restrict__ lrp, const int32_t *__restrict__ lcol,
             const double *__restrict__ lval, const int64_t *__restrict__ hptr,
             const int32_t *__restrict__ hrow, int64_t nitems, int p, const double *__restrict__ X,
             double *__restrict__ part) {
    const int lane = lane_id();
    const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x / WAVE);
    for (int64_t i = (int64_t)blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE; i < nitems;
         i += nwaves) {
        const int32_t r = hrow[i];
        const int64_t k0 = lrp[r] + (i - hptr[r]) * SPMM_CH;
        const int64_t k1 = k0 + SPMM_CH < lrp[r + 1] ? k0 + SPMM_CH : lrp[r + 1];
        double acc[CPL];
        spmm_range<GS, CPL>(lcol, lval, k0, k1, p, X, acc);
        if (lane < GS) {
#pragma unroll
            for (int c = 0; c < CPL; ++c) {
                const int j = lane + c * GS;
                if (j < p) part[(size_t)i * p + j] = acc[c];
            }
        }
    }
}

// The long rows: their items' partials summed in item order.
__global__ void __launch_bounds__(256)
k_spmm_finish(const int64_t *__restrict__ hptr, int64_t ns, int p, const double *__restrict__ X,
              const double *__restrict__ Zb, double alpha, double beta, double gamma,
              const double *__restrict__ part, double *__restrict__ out) {
    const int lane = lane_id();
    const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x / WAVE);
    for (int64_t r = (int64_t)blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE; r < ns;
         r += nwaves) {
        const int64_t i0 = hptr[r], i1 = hptr[r + 1];
        if (i0 == i1) continue;
        for (int j = lane; j < p; j += WAVE) {
            double acc = 0.0;
            for (int64_t i = i0; i < i1; ++i) acc += part[(size_t)i * p + j];
            const size_t o = (size_t)r * p + j;
            double v = alpha * acc + beta * X[o];
            if (Zb) v += gamma * Zb[o];
            out[o] = v;
        }
    }
}

// fp64 matrix cores: v_mfma_f64_16x16x4f64 multiplies a 16 x 4 by a 4 x 16
// block; lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16] and holds
// D[l / 16 + 4r][l % 16] in register r of its 4-wide accumulator.
typedef double dbl4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ dbl4 mfma_f64(double a, double b, dbl4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

constexpr int MT = 64;     // output tile edge of the dense products
constexpr int MK = 32;     // depth staged in LDS per step

// Partial Gram tiles: part[chunk][i][j] = sum over the chunk's rows r of
// A[r][i] * B[r][j], for the tiles on and above the diagonal (A^T B is
// symmetric wherever it is used: A^T A, and Q^T M Q with M symmetric).  A
// workgroup (4 waves) takes a 64 x 64 tile of the p x p result, each wave
// 16 of its rows against all 64 columns; the rows
// of the chunk are staged 32 at a time in LDS (coalesced row segments) and
// fed to the fp64 matrix cores, the rows being the contraction index.
__global__ void __launch_bounds__(256)
k_emb_gram_part(const double *__restrict__ A, const double *__restrict__ B, int64_t n, int p,
                double *__restrict__ part) {
    __shared__ double as[MK][MT + 1];
    __shared__ double bs[MK][MT + 1];
    // blockIdx.y enumerates the tiles (ti, tj) with ti <= tj: the products
    // are symmetric, k_emb_gram_sum mirrors the rest
    const int tiles = (p + MT - 1) / MT;
    int ti = 0, rest = blockIdx.y;
    while (rest >= tiles - ti) {
        rest -= tiles - ti;
        ++ti;
    }
    const int i0 = ti * MT, j0 = (ti + rest) * MT;
    const int64_t r0 = (int64_t)blockIdx.x * GRAM_ROWS;
    const int64_t r1 = r0 + GRAM_ROWS < n ? r0 + GRAM_ROWS : n;
    const int tid = threadIdx.x, lane = tid & (WAVE - 1), wv = tid / WAVE;
    dbl4 acc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = dbl4{0.0, 0.0, 0.0, 0.0};
    for (int64_t rb = r0; rb < r1; rb += MK) {
        for (int q = tid; q < MK * MT; q += 256) {
            const int rr = q / MT, cc = q % MT;
            const int64_t r = rb + rr;
            as[rr][cc] = (r < r1 && i0 + cc < p) ? A[(size_t)r * p + i0 + cc] : 0.0;
            bs[rr][cc] = (r < r1 && j0 + cc < p) ? B[(size_t)r * p + j0 + cc] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < MK; kk += 4) {
            const double a = as[kk + lane / 16][wv * 16 + lane % 16];
#pragma unroll
            for (int t = 0; t < 4; ++t) acc[t] = mfma_f64(a, bs[kk + lane / 16][t * 16 + lane % 16], acc[t]);
        }
        __syncthreads();
    }
    double *dst = part + (size_t)blockIdx.x * p * p;
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int i = i0 + wv * 16 + lane / 16 + 4 * r, j = j0 + t * 16 + lane % 16;
            if (i < p && j < p) dst[(size_t)i * p + j] = acc[t][r];
        }
}

// C = sum of the partials, chunk by chunk in order (a fixed order: the same
// inputs give the same bits); an entry below the diagonal in a tile below
// the diagonal tiles takes its mirror image.
__global__ void k_emb_gram_sum(const double *__restrict__ part, int64_t chunks, int p,
                               double *__restrict__ C) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= p * p) return;
    const int i = q / p, j = q % p;
    const int src = (i / MT > j / MT) ? j * p + i : q;
    double s = 0.0;
    for (int64_t c = 0; c < chunks; ++c) s += part[(size_t)c * p * p + src];
    C[q] = s;
}

// ----------------------------------------------- small symmetric eigen

// Round-robin pairing of pe (even) indices: at step t, slot 0 holds index
// 0 and slot q >= 1 holds 1 + ((q - 1 - t) mod (pe - 1)); pair k of the step
// is (slot k, slot pe - 1 - k).  Over pe - 1 steps every two indices meet
// once.
__device__ __forceinline__ int rr_slot(int q, int t, int pe) {
    if (q == 0) return 0;
    int r = (q - 1 - t) % (pe - 1);
    return 1 + (r < 0 ? r + pe - 1 : r);
}

template <int MAXP>
struct JacobiShared {
    double rc[MAXP / 2], rs[MAXP / 2];
    int ri[MAXP / 2], rj[MAXP / 2];
    int order[MAXP];
    int rotated;
};

// Cyclic Jacobi on the p x p symmetric A (row-major, destroyed; LDS or
// global memory), the whole workgroup (NT threads) taking part: V gets
// the eigenvectors as columns and sh.order the column order that sorts the
// eigenvalues (A's final diagonal) descending.  Each rotation is the
// symmetric Schur step (Golub and Van Loan, Sec. 8.5.2) that annihilates
// a_ij; the p / 2 disjoint pairs of a round-robin step rotate together,
// rows first, then columns.  A pair is skipped once |a_ij| <= 1e-15
// sqrt(|a_ii a_jj|) (or a_ij = 0), and the sweeps stop after one that
// rotates nothing (at most max_sweeps).
template <int MAXP, int NT>
__device__ void jacobi_solve(double *A, double *V, int p, int max_sweeps, JacobiShared<MAXP> &sh) {
    const int tid = threadIdx.x;
    const int pe = p + (p & 1);              // even count (index p is a dummy when p is odd)
    const int half = pe / 2;
    for (int q = tid; q < p * p; q += NT) V[q] = (q / p == q % p) ? 1.0 : 0.0;
    __syncthreads();
    for (int sweep = 0; sweep < max_sweeps; ++sweep) {
        if (tid == 0) sh.rotated = 0;
        __syncthreads();
        for (int step = 0; step < pe - 1; ++step) {
            for (int k = tid; k < half; k += NT) {
                int i = rr_slot(k, step, pe), j = rr_slot(pe - 1 - k, step, pe);
                if (i > j) { const int t = i; i = j; j = t; }
                double c = 1.0, sn = 0.0;
                if (j < p) {
                    const double aij = A[i * p + j];
                    const double aii = A[i * p + i], ajj = A[j * p + j];
                    if (aij != 0.0 && fabs(aij) > 1e-15 * sqrt(fabs(aii) * fabs(ajj))) {
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
            for (int q = tid; q < half * p; q += NT) {
                const int k = q / p, x = q % p;
                if (sh.rs[k] == 0.0) continue;
                const int i = sh.ri[k], j = sh.rj[k];
                const double ai = A[i * p + x], aj = A[j * p + x];
                A[i * p + x] = sh.rc[k] * ai - sh.rs[k] * aj;
                A[j * p + x] = sh.rs[k] * ai + sh.rc[k] * aj;
            }
            __syncthreads();
            // columns i, j of A <- A J and of V <- V J
            for (int q = tid; q < half * p; q += NT) {
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
            for (int k = tid; k < half; k += NT) {
                if (sh.rs[k] == 0.0) continue;
                A[sh.ri[k] * p + sh.rj[k]] = 0.0;
                A[sh.rj[k] * p + sh.ri[k]] = 0.0;
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

// The Rayleigh-Ritz matrix of the subspace iteration (p <= 256, global
// memory, L2-resident): cyclic Jacobi as in jacobi_solve, but each thread
// applies the two-sided rotation to whole 2 x 2 blocks, one pair of pairs
// (k, l) at a time -- the block of rows (i_k, j_k) and columns (i_l, j_l)
// becomes J_k^T B J_l, its mirror image the transpose -- so a step costs
// two barriers.  The rotations are logged (rot_cs, rot_ij, *nsteps steps of
// p / 2 pairs) for k_jacobi_vecs; the eigenvalues, sorted descending, go to
// w and their column order to order.  One workgroup of 1024.
constexpr int RR_SWEEPS = 30;
constexpr int LDS_P = 192;                              // widest block kept in LDS
constexpr int LDS_PACKED = LDS_P * (LDS_P + 1) / 2;     // its upper triangle

// Symmetric p x p storage: full row-major (both halves written) or the
// packed upper triangle (row-major, LDS).
template <bool PACKED>
struct Sym {
    double *a;
    int p;
    __device__ __forceinline__ int at(int i, int j) const {
        if (!PACKED) return i * p + j;
        if (i > j) { const int t = i; i = j; j = t; }
        return i * p - i * (i - 1) / 2 + (j - i);
    }
    __device__ __forceinline__ double get(int i, int j) const { return a[at(i, j)]; }
    __device__ __forceinline__ void set(int i, int j, double v) const {
        a[at(i, j)] = v;
        if (!PACKED && i != j) a[at(j, i)] = v;
    }
};

template <bool PACKED>
__device__ void jacobi_rr_body(Sym<PACKED> A, int p, double2 *__restrict__ rot_cs,
                               short2 *__restrict__ rot_ij, int *__restrict__ nsteps,
                               int *__restrict__ order, double *__restrict__ w) {
    __shared__ double rc[EMB_MAX_P / 2], rs[EMB_MAX_P / 2];
    __shared__ int ri[EMB_MAX_P / 2], rj[EMB_MAX_P / 2];
    __shared__ double dg[EMB_MAX_P];
    __shared__ int rotated;
    const int tid = threadIdx.x;
    const int pe = p + (p & 1);
    const int half = pe / 2;
    // the update: thread (kg, l) takes the pairs of pairs (k, l), k = kg,
    // kg + groups, ... up to l
    const int groups = 1024 / half;
    const int my_l = tid % half, my_kg = tid / half;
    int steps = 0;
    for (int sweep = 0; sweep < RR_SWEEPS; ++sweep) {
        if (tid == 0) rotated = 0;
        __syncthreads();
        for (int step = 0; step < pe - 1; ++step, ++steps) {
            for (int k = tid; k < half; k += 1024) {
                int i = rr_slot(k, step, pe), j = rr_slot(pe - 1 - k, step, pe);
                if (i > j) { const int t = i; i = j; j = t; }
                double c = 1.0, sn = 0.0;
                if (j < p) {
                    const double aij = A.get(i, j);
                    const double aii = A.get(i, i), ajj = A.get(j, j);
                    if (aij != 0.0 && fabs(aij) > 1e-15 * sqrt(fabs(aii) * fabs(ajj))) {
                        const double tau = (ajj - aii) / (2.0 * aij);
                        const double t = (tau >= 0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                        c = 1.0 / sqrt(1.0 + t * t);
                        sn = t * c;
                        rotated = 1;
                    }
                }
                ri[k] = i; rj[k] = j; rc[k] = c; rs[k] = sn;
                rot_cs[(size_t)steps * half + k] = make_double2(c, sn);
                rot_ij[(size_t)steps * half + k] = make_short2((short)i, (short)j);
            }
            __syncthreads();
            for (int k = my_kg, l = my_l; my_kg < groups && k <= l; k += groups) {
                const double ck = rc[k], sk = rs[k], cl = rc[l], sl = rs[l];
                const int ik = ri[k], jk = rj[k], il = ri[l], jl = rj[l];
                if (k == l) {
                    if (sk == 0.0) continue;
                    const double aii = A.get(ik, ik), ajj = A.get(jk, jk), aij = A.get(ik, jk);
                    A.set(ik, ik, ck * ck * aii - 2.0 * ck * sk * aij + sk * sk * ajj);
                    A.set(jk, jk, sk * sk * aii + 2.0 * ck * sk * aij + ck * ck * ajj);
                    A.set(ik, jk, 0.0);     // annihilated
                    continue;
                }
                if (sk == 0.0 && sl == 0.0) continue;
                const bool hk = jk < p, hl = jl < p;    // false: the dummy index of odd p
                const double b00 = A.get(ik, il);
                const double b01 = hl ? A.get(ik, jl) : 0.0;
                const double b10 = hk ? A.get(jk, il) : 0.0;
                const double b11 = hk && hl ? A.get(jk, jl) : 0.0;
                const double r00 = ck * b00 - sk * b10, r01 = ck * b01 - sk * b11;
                const double r10 = sk * b00 + ck * b10, r11 = sk * b01 + ck * b11;
                A.set(ik, il, cl * r00 - sl * r01);
                if (hl) A.set(ik, jl, sl * r00 + cl * r01);
                if (hk) A.set(jk, il, cl * r10 - sl * r11);
                if (hk && hl) A.set(jk, jl, sl * r10 + cl * r11);
            }
            __syncthreads();
        }
        const int any = rotated;
        __syncthreads();
        if (!any) break;
    }
    for (int q = tid; q < p; q += 1024) dg[q] = A.get(q, q);
    __syncthreads();
    // descending order, ties by index
    for (int j = tid; j < p; j += 1024) {
        const double d = dg[j];
        int r = 0;
        for (int i = 0; i < p; ++i) r += dg[i] > d || (dg[i] == d && i < j);
        order[r] = j;
        w[r] = d;
    }
    if (tid == 0) *nsteps = steps;
}

// p <= LDS_P: the packed upper triangle of H in LDS.
__global__ void __launch_bounds__(1024)
k_jacobi_rr_lds(const double *__restrict__ H, int p, double2 *__restrict__ rot_cs,
                short2 *__restrict__ rot_ij, int *__restrict__ nsteps, int *__restrict__ order,
                double *__restrict__ w) {
    __shared__ double a[LDS_PACKED];
    const Sym<true> A{a, p};
    for (int q = threadIdx.x; q < p * p; q += 1024) {
        const int i = q / p, j = q % p;
        if (i <= j) a[A.at(i, j)] = H[q];
    }
    __syncthreads();
    jacobi_rr_body<true>(A, p, rot_cs, rot_ij, nsteps, order, w);
}

// Wider blocks: H itself, in global memory (L2-resident), destroyed.
__global__ void __launch_bounds__(1024)
k_jacobi_rr(double *__restrict__ H, int p, double2 *__restrict__ rot_cs,
            short2 *__restrict__ rot_ij, int *__restrict__ nsteps, int *__restrict__ order,
            double *__restrict__ w) {
    jacobi_rr_body<false>(Sym<false>{H, p}, p, rot_cs, rot_ij, nsteps, order, w);
}

// Eigenvectors of the logged rotations: row x of V = e_x^T J_1 J_2 ...,
// one wave per row held in LDS, the pairs of a step in parallel; written
// with the columns sorted (Vs[x][q] = V[x][order[q]]).
__global__ void __launch_bounds__(256)
k_jacobi_vecs(const double2 *__restrict__ rot_cs, const short2 *__restrict__ rot_ij,
              const int *__restrict__ nsteps, const int *__restrict__ order, int p,
              double *__restrict__ Vs) {
    __shared__ double rows[256 / WAVE][EMB_MAX_P];
    const int lane = lane_id(), wv = threadIdx.x / WAVE;
    const int x = blockIdx.x * (256 / WAVE) + wv;
    if (x >= p) return;                      // whole waves only: no workgroup barrier below
    double *v = rows[wv];
    const int half = (p + (p & 1)) / 2;
    for (int q = lane; q < p; q += WAVE) v[q] = q == x ? 1.0 : 0.0;
    wave_sync();
    const int T = *nsteps;
    for (int t = 0; t < T; ++t) {
        for (int k = lane; k < half; k += WAVE) {
            const double2 cs = rot_cs[(size_t)t * half + k];
            if (cs.y == 0.0) continue;
            const short2 ij = rot_ij[(size_t)t * half + k];
            const double vi = v[ij.x], vj = v[ij.y];
            v[ij.x] = cs.x * vi - cs.y * vj;
            v[ij.y] = cs.y * vi + cs.x * vj;
        }
        wave_sync();
    }
    for (int q = lane; q < p; q += WAVE) Vs[(size_t)x * p + q] = v[order[q]];
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
    jacobi_solve<DENSE_MAX, 256>(A, V, s, 60, sh);
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

// Cholesky QR step: G = R^T R (R upper, right-looking) and Rinv = R^{-1},
// so that A Rinv has orthonormal columns when G = A^T A.  A pivot below
// 1e-30 of the largest diagonal is raised to it (a rank-deficient block
// keeps finite values).  One workgroup; Rinv's column j is solved by thread
// j by back substitution.  R lives in the packed upper triangle in LDS
// (p <= LDS_P) or in G's upper triangle.
template <bool PACKED>
__device__ void chol_body(Sym<PACKED> R, const double *__restrict__ G, double *__restrict__ Rinv,
                          int p) {
    __shared__ double floor_v;
    const int tid = threadIdx.x;
    if (PACKED) {
        for (int q = tid; q < p * p; q += 1024) {
            const int i = q / p, j = q % p;
            if (i <= j) R.a[R.at(i, j)] = G[q];
        }
        __syncthreads();
    }
    if (tid == 0) {
        double mx = 0.0;
        for (int i = 0; i < p; ++i) mx = R.get(i, i) > mx ? R.get(i, i) : mx;
        floor_v = mx > 0 ? 1e-30 * mx : 1e-300;
    }
    __syncthreads();
    for (int k = 0; k < p; ++k) {
        if (tid == 0) {
            const double d = R.get(k, k);
            R.a[R.at(k, k)] = sqrt(d > floor_v ? d : floor_v);
        }
        __syncthreads();
        const double rkk = R.get(k, k);
        for (int j = k + 1 + tid; j < p; j += 1024) R.a[R.at(k, j)] /= rkk;
        __syncthreads();
        const int wd = p - k - 1;
        for (int q = tid; q < wd * wd; q += 1024) {
            const int i = k + 1 + q / wd, j = k + 1 + q % wd;
            if (j >= i) R.a[R.at(i, j)] -= R.get(k, i) * R.get(k, j);
        }
        __syncthreads();
    }
    for (int j = tid; j < p; j += 1024) {
        for (int i = p - 1; i >= 0; --i) {
            if (i > j) {
                Rinv[i * p + j] = 0.0;
                continue;
            }
            double sum = i == j ? 1.0 : 0.0;
            for (int l = i + 1; l <= j; ++l) sum -= R.get(i, l) * Rinv[l * p + j];
            Rinv[i * p + j] = sum / R.get(i, i);
        }
    }
}

__global__ void __launch_bounds__(1024)
k_emb_chol_lds(const double *__restrict__ G, double *__restrict__ Rinv, int p) {
    __shared__ double a[LDS_PACKED];
    chol_body<true>(Sym<true>{a, p}, G, Rinv, p);
}

__global__ void __launch_bounds__(1024)
k_emb_chol(double *__restrict__ G, double *__restrict__ Rinv, int p) {
    chol_body<false>(Sym<false>{G, p}, G, Rinv, p);
}

// Y = X Q (n x p times p x p) on the fp64 matrix cores: a workgroup (4
// waves) takes a 64-row x 64-column tile of Y, each wave 16 rows; X's rows
// and Q's rows are staged 32 deep in LDS.
__global__ void __launch_bounds__(256)
k_emb_apply(const double *__restrict__ X, const double *__restrict__ Q, int64_t n, int p,
            double *__restrict__ Y) {
    __shared__ double xs[MT][MK + 1];
    __shared__ double qs[MK][MT + 1];
    const int64_t r0 = (int64_t)blockIdx.x * MT;
    const int c0 = blockIdx.y * MT;
    const int tid = threadIdx.x, lane = tid & (WAVE - 1), wv = tid / WAVE;
    dbl4 acc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = dbl4{0.0, 0.0, 0.0, 0.0};
    for (int k0 = 0; k0 < p; k0 += MK) {
        for (int q = tid; q < MT * MK; q += 256) {
            const int rr = q / MK, kk = q % MK;
            const int64_t r = r0 + rr;
            xs[rr][kk] = (r < n && k0 + kk < p) ? X[(size_t)r * p + k0 + kk] : 0.0;
            const int kq = q / MT, cc = q % MT;
            qs[kq][cc] = (k0 + kq < p && c0 + cc < p) ? Q[(size_t)(k0 + kq) * p + c0 + cc] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < MK; kk += 4) {
            const double a = xs[wv * 16 + lane % 16][kk + lane / 16];
#pragma unroll
            for (int t = 0; t < 4; ++t) acc[t] = mfma_f64(a, qs[kk + lane / 16][t * 16 + lane % 16], acc[t]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int64_t row = r0 + wv * 16 + lane / 16 + 4 * r;
            const int col = c0 + t * 16 + lane % 16;
            if (row < n && col < p) Y[(size_t)row * p + col] = acc[t][r];
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

// Workspace layout of the embedding.  p0 is the starting block width,
// pmax the widest a stalled component may grow to; blocks hold the largest
// possible component (n rows) at pmax columns.
struct EmbLayout {
    int p0, pmax;
    int64_t chunks, max_items;
    size_t cnt, eoff, stmp, status, wslot, sc, deg, parent, keys, keys_tmp, ids, ids_tmp, sort_tmp,
        seg_start, loc, lrp, hptr, lcol, lval, hrow, spart, X, Y, Yp, Yn, MX, part, G, Vs, H,
        theta, sigma, res, rot_cs, rot_ij, rr_misc, total;
};

EmbLayout emb_layout(int64_t n, int64_t nnz, int dim) {
    EmbLayout y{};
    int p = dim + (dim / 4 > 8 ? dim / 4 : 8);
    if (p > EMB_MAX_P) p = EMB_MAX_P;
    y.p0 = p;
    y.pmax = 4 * p < EMB_MAX_P ? 4 * p : EMB_MAX_P;
    const int pm = y.pmax;
    y.chunks = (n + GRAM_ROWS - 1) / GRAM_ROWS;
    if (y.chunks < 1) y.chunks = 1;
    // a row of more than SPMM_CH nonzeros has at most twice len / SPMM_CH items
    y.max_items = 2 * (nnz / SPMM_CH) + 1;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o = (o + bytes + 255) & ~(size_t)255;
        return at;
    };
    const size_t n1 = (size_t)(n > 0 ? n : 1), nz1 = (size_t)(nnz > 0 ? nnz : 1);
    y.cnt = take(sizeof(int64_t) * (size_t)(n + 1));
    y.eoff = take(sizeof(int64_t) * (size_t)(n + 1));
    y.stmp = take(sizeof(int64_t) * (size_t)(scan_tiles(n + 1) + 1));
    y.status = take(256);
    y.wslot = take(sizeof(double) * nz1);
    y.sc = take(sizeof(double) * n1);
    y.deg = take(sizeof(uint64_t) * n1);
    y.parent = take(sizeof(int32_t) * n1);
    y.keys = take(sizeof(uint64_t) * n1);
    y.keys_tmp = take(sizeof(uint64_t) * n1);
    y.ids = take(sizeof(uint32_t) * n1);
    y.ids_tmp = take(sizeof(uint32_t) * n1);
    y.sort_tmp = take(sort_tmp_need(n > 0 ? n : 1));
    y.seg_start = take(sizeof(int64_t) * (size_t)(n + 1));
    y.loc = take(sizeof(int32_t) * n1);
    y.lrp = take(sizeof(int64_t) * (size_t)(n + 1));
    y.hptr = take(sizeof(int64_t) * (size_t)(n + 1));
    y.lcol = take(sizeof(int32_t) * nz1);
    y.lval = take(sizeof(double) * nz1);
    y.hrow = take(sizeof(int32_t) * (size_t)y.max_items);
    y.spart = take(sizeof(double) * (size_t)y.max_items * pm);
    const size_t blk = sizeof(double) * n1 * pm;
    y.X = take(blk);
    y.Y = take(blk);
    y.Yp = take(blk);
    y.Yn = take(blk);
    y.MX = take(blk);
    y.part = take(sizeof(double) * (size_t)y.chunks * pm * pm);
    y.G = take(sizeof(double) * (size_t)pm * pm);
    y.Vs = take(sizeof(double) * (size_t)pm * pm);
    y.H = take(sizeof(double) * (size_t)pm * pm);
    y.theta = take(sizeof(double) * pm);
    y.sigma = take(sizeof(double) * pm);
    y.res = take(sizeof(double) * pm);
    const size_t rots = (size_t)RR_SWEEPS * (pm + 1) * ((pm + 1) / 2);
    y.rot_cs = take(sizeof(double2) * rots);
    y.rot_ij = take(sizeof(short2) * rots);
    y.rr_misc = take(sizeof(int) * (pm + 1));     // step count, then the column order
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
    const int p0 = y.p0;
    const int64_t m = nnz / 2;
#define EMB_CHK(x) do { if ((x) != hipSuccess) return TG_E_DEVICE; } while (0)
    ksum_reset();
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
    ksum_begin(st);
    k_emb_dense<<<(unsigned)nseg, 256, 0, st>>>(row_ptr, col, D(y.wslot), D(y.sc), seg_start, order,
                                                loc, dim, raw, Z, eigenvalues);
    ksum_end("dense", 0.0, st);
    EMB_CHK(hipGetLastError());
    EMB_CHK(hipStreamSynchronize(st));
    ksum_collect();

    // the large components, one after another
    double *X = D(y.X), *Y = D(y.Y), *Yp = D(y.Yp), *Yn = D(y.Yn), *MX = D(y.MX);
    double *G = D(y.G), *Vs = D(y.Vs), *H = D(y.H);
    double *theta = D(y.theta), *sigma = D(y.sigma), *res = D(y.res), *part = D(y.part);
    int64_t *lrp = reinterpret_cast<int64_t *>(w + y.lrp);
    int64_t *hptr = reinterpret_cast<int64_t *>(w + y.hptr);
    int32_t *lcol = reinterpret_cast<int32_t *>(w + y.lcol);
    double *lval = D(y.lval);
    int32_t *hrow = reinterpret_cast<int32_t *>(w + y.hrow);
    double *spart = D(y.spart);
    double2 *rot_cs = reinterpret_cast<double2 *>(w + y.rot_cs);
    short2 *rot_ij = reinterpret_cast<short2 *>(w + y.rot_ij);
    int *rr_misc = reinterpret_cast<int *>(w + y.rr_misc);
    bool all_converged = true;
    int most_iterations = 0;
    for (int64_t c = 0; c < nseg; ++c) {
        const int64_t cs = hseg[(size_t)c], ns = hseg[(size_t)c + 1] - cs;
        if (ns <= DENSE_MAX) continue;
        const uint32_t *nodes = order + cs;
        const unsigned rg = row_grid(ns);
        // the component's S as its own CSR, and the items of its long rows
        k_loc_len<<<rg, 256, 0, st>>>(row_ptr, D(y.wslot), nodes, ns, cnt, eoff);
        EMB_CHK(hipGetLastError());
        EMB_CHK(launch_excl_scan(cnt, lrp, ns + 1, reinterpret_cast<int64_t *>(w + y.stmp), nullptr, st));
        EMB_CHK(launch_excl_scan(eoff, hptr, ns + 1, reinterpret_cast<int64_t *>(w + y.stmp), nullptr,
                                 st));
        k_loc_fill<<<rg, 256, 0, st>>>(row_ptr, col, D(y.wslot), D(y.sc), nodes, loc, ns, lrp, lcol,
                                       lval);
        k_loc_items<<<grid_of(ns), 256, 0, st>>>(hptr, ns, hrow);
        EMB_CHK(hipGetLastError());
        uint32_t root = 0;
        int64_t nitems = 0, nnz_c = 0;
        EMB_CHK(hipMemcpyAsync(&root, nodes, sizeof(root), hipMemcpyDeviceToHost, st));
        EMB_CHK(hipMemcpyAsync(&nitems, hptr + ns, sizeof(nitems), hipMemcpyDeviceToHost, st));
        EMB_CHK(hipMemcpyAsync(&nnz_c, lrp + ns, sizeof(nnz_c), hipMemcpyDeviceToHost, st));
        EMB_CHK(hipStreamSynchronize(st));
        if (nitems > y.max_items) return TG_E_INTERNAL;
        const int pcap = (int)(ns < y.pmax ? ns : y.pmax);
        int p = (int)(ns < p0 ? ns : p0);
        const int want = dim < p ? dim : p;
        const int64_t chunks = (ns + GRAM_ROWS - 1) / GRAM_ROWS;
        // flops of an s x p by p x p product, and of a symmetric Gram product
        // (one triangle)
        auto dense_flops = [&]() { return 2.0 * (double)ns * (double)p * (double)p; };
        auto gram_flops = [&]() { return (double)ns * (double)p * (double)(p + 1); };
        auto gram = [&](const double *A, const double *B, double *C) -> hipError_t {
            const int mt = (p + MT - 1) / MT;
            ksum_begin(st);
            k_emb_gram_part<<<dim3((unsigned)chunks, (unsigned)(mt * (mt + 1) / 2)), 256, 0, st>>>(
                A, B, ns, p, part);
            ksum_end("gram", gram_flops(), st);
            k_emb_gram_sum<<<(unsigned)((p * p + 255) / 256), 256, 0, st>>>(part, chunks, p, C);
            return hipGetLastError();
        };
        auto apply = [&](const double *A, const double *Q, double *out) -> hipError_t {
            ksum_begin(st);
            k_emb_apply<<<dim3((unsigned)((ns + MT - 1) / MT), (unsigned)((p + MT - 1) / MT)), 256,
                          0, st>>>(A, Q, ns, p, out);
            ksum_end("apply", dense_flops(), st);
            return hipGetLastError();
        };
        // out = alpha S A + beta A + gamma Zb
        // algorithmic bytes of one product: every nonzero's column and value
        // and the neighbour's block row, each row's own block row read (and
        // Zb's) and the output row written
        auto spmm_bytes = [&](bool zb) {
            return (double)nnz_c * (12.0 + 8.0 * p) + (double)ns * 8.0 * p * (zb ? 3.0 : 2.0);
        };
        auto spmm = [&](const double *A, const double *Zb, double alpha, double beta, double gamma,
                        double *out) -> hipError_t {
            ksum_begin(st);
#define EMB_SPMM(GSV, CPLV)                                                                       \
    do {                                                                                          \
        k_spmm_rows<GSV, CPLV><<<rg, 256, 0, st>>>(lrp, lcol, lval, ns, p, A, Zb, alpha, beta,     \
                                                   gamma, out);                                   \
        if (nitems)                                                                               \
            k_spmm_items<GSV, CPLV><<<row_grid(nitems), 256, 0, st>>>(lrp, lcol, lval, hptr, hrow, \
                                                                      nitems, p, A, spart);       \
    } while (0)
            if (p <= 16) EMB_SPMM(16, 1);
            else if (p <= 32) EMB_SPMM(32, 1);
            else if (p <= 64) EMB_SPMM(64, 1);
            else if (p <= 128) EMB_SPMM(64, 2);
            else if (p <= 192) EMB_SPMM(64, 3);
            else EMB_SPMM(64, 4);
#undef EMB_SPMM
            if (nitems)
                k_spmm_finish<<<rg, 256, 0, st>>>(hptr, ns, p, A, Zb, alpha, beta, gamma, spart, out);
            ksum_end("spmm", spmm_bytes(Zb != nullptr), st);
            return hipGetLastError();
        };
        // Cholesky QR: out = A R^{-1}, A^T A = R^T R
        auto orth = [&](const double *A, double *out) -> hipError_t {
            hipError_t e = gram(A, A, G);
            if (e != hipSuccess) return e;
            ksum_begin(st);
            if (p <= LDS_P) k_emb_chol_lds<<<1, 1024, 0, st>>>(G, Vs, p);
            else k_emb_chol<<<1, 1024, 0, st>>>(G, Vs, p);
            ksum_end("chol", 0.0, st);
            if ((e = hipGetLastError()) != hipSuccess) return e;
            return apply(A, Vs, out);
        };
        // Three rotating blocks (the Chebyshev recurrence needs two inputs
        // and an output), plus Yp (first orthonormalisation pass) and MX.
        double *R[3] = {X, Y, Yn};
        std::vector<double> h_theta, h_res;
        // Rayleigh-Ritz on the orthonormal block Q: Ritz vectors to xo, M
        // times them to mo, Ritz values to theta (descending), residual
        // norms read back.
        auto rayleigh_ritz = [&](const double *Q, double *xo, double *mo) -> hipError_t {
            hipError_t e;
            h_theta.assign((size_t)p, 0.0);
            h_res.assign((size_t)p, 0.0);
            if ((e = spmm(Q, nullptr, 0.5, 0.5, 0.0, MX)) != hipSuccess) return e;
            if ((e = gram(Q, MX, H)) != hipSuccess) return e;
            ksum_begin(st);
            if (p <= LDS_P)
                k_jacobi_rr_lds<<<1, 1024, 0, st>>>(H, p, rot_cs, rot_ij, rr_misc, rr_misc + 1, sigma);
            else
                k_jacobi_rr<<<1, 1024, 0, st>>>(H, p, rot_cs, rot_ij, rr_misc, rr_misc + 1, sigma);
            k_jacobi_vecs<<<(unsigned)((p + 3) / 4), 256, 0, st>>>(rot_cs, rot_ij, rr_misc, rr_misc + 1,
                                                                   p, Vs);
            ksum_end("jacobi", 0.0, st);
            if ((e = hipGetLastError()) != hipSuccess) return e;
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
            if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
            ksum_collect();
            return hipSuccess;
        };
        auto worst = [&]() {
            double r = 0.0;
            for (int j = 0; j < want; ++j)
                r = !(h_res[(size_t)j] <= r) ? h_res[(size_t)j] : r;   // NaN counts as worst
            return r;
        };
        // start: a random block, orthonormalised twice, and its Ritz vectors
        k_emb_random<<<(unsigned)((ns * p + 255) / 256), 256, 0, st>>>(R[0], ns, p,
                                                                      seed ^ mix64_host(root));
        EMB_CHK(hipGetLastError());
        EMB_CHK(orth(R[0], Yp));
        EMB_CHK(orth(Yp, R[1]));
        EMB_CHK(rayleigh_ritz(R[1], R[0], R[2]));
        int it = 0;
        double chk = worst();       // worst wanted residual at the last checkpoint
        int chk_it = 0;
        bool converged = chk <= tol;
        while (!converged && it < max_iter) {
            ++it;
            // Every 25 iterations: a worst wanted residual that fell by less
            // than 100x means the cut sits in a cluster of eigenvalues wider
            // than the block; widen the block (its Ritz vectors and fresh
            // random columns) by half.
            bool widen = false;
            if (it - chk_it >= 25) {
                widen = worst() > 1e-2 * chk && p < pcap;
                chk = worst();
                chk_it = it;
            }
            if (widen) {
                const int q = p + (p / 2 > 16 ? p / 2 : 16) < pcap ? p + (p / 2 > 16 ? p / 2 : 16)
                                                                  : pcap;
                k_emb_widen<<<(unsigned)((ns * q + 255) / 256), 256, 0, st>>>(
                    R[0], ns, p, q, seed ^ mix64_host(root + (uint64_t)it), R[1]);
                EMB_CHK(hipGetLastError());
                p = q;
                        EMB_CHK(orth(R[1], Yp));
                EMB_CHK(orth(Yp, R[2]));
                EMB_CHK(rayleigh_ritz(R[2], R[0], R[1]));
                chk = worst();
                converged = chk <= tol;
                continue;
            }
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
            converged = worst() <= tol;
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
    ksum_collect();
#undef EMB_CHK
    return all_converged ? TG_OK : TG_E_NO_CONVERGENCE;
}

}  // extern "C"
