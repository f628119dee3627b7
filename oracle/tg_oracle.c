/*
 * CPU oracle for per-edge typed graphlet counts (test infrastructure).
 *
 * This file is the slow, plain reference that the GPU library is checked
 * against.  Only the tests, the smoke check and the benchmark's CPU-baseline
 * leg load it; the product path never does.  It shares no code, header or
 * table with the GPU library.
 *
 * What is counted (Rossi et al., "Heterogeneous Graphlets"):
 *   G = (V, E, phi) simple undirected, phi : V -> {0..L-1}  (Def. 1).
 *   For every edge e = (i, j):
 *     tri[t]   = |T_ij^t|,  T_ij^t = Gamma_i^t  cap Gamma_j^t        (Cor. 1)
 *     path3[t] = |S_i^t| + |S_j^t|,
 *                S_i^t = Gamma_i^t \ (Gamma_j^t cup {j})             (Cor. 2, 3)
 *     f_e(g, {t, t'}) for the ten 4-node orbits g3..g12 of Table 3: the
 *       number of node pairs {k, r} (k != r, both outside {i, j}) whose
 *       induced subgraph with i, j is the graphlet of orbit g with edge ij in
 *       that orbit, and whose type multiset is {t, t'}.  The key is the type
 *       multiset, so the two assignments of t, t' to k, r are summed
 *       (Def. of typed graphlet instance; multiset hashing, Sec. 4.5).
 *
 * Two independent ways of computing one edge's row are given:
 *   tgo_edge_definition  the definition itself: every connected induced
 *                        4-node subgraph around the edge is classified by its
 *                        edge count and degrees;
 *   tgo_edge_paper       the paper's Algorithms 1-3 (typed sets, path-based
 *                        and triangle-based enumeration) with the remaining
 *                        orbits derived by Lemmas 1-4.
 * Global counts follow Problem 2 and the orbit-to-graphlet sums of Sec. 4.4:
 * C_H = (1/|E(H)|) sum_e x_e(H).
 *
 * Row layout (shared convention with the library, written out separately
 * here): [tri t=0..L-1][path3 t=0..L-1] then for g = 3..12 one block of
 * P = L(L+1)/2 unordered type pairs (t <= t') in lexicographic order.
 * Global layout: h0 (edges, C(L+1,2)), h1 (3-paths, C(L+2,3)), h2
 * (triangles, C(L+2,3)), h3..h8 (4-path, 4-star, 4-cycle, tailed triangle,
 * chordal cycle, 4-clique; C(L+3,4) each); inside a block a sorted type
 * multiset sits at its position in co-lexicographic order.  The oracle finds
 * that position through a table built by enumerating the multisets in that
 * order (the precomputed type-vector table of Sec. 4.5), not by formula.
 *
 * Readings where the paper is loose (listed in the design notes):
 *   - S_i excludes j and S_j excludes i (Cor. 2 says so explicitly; the
 *     shorter form Gamma_i^t \ T_ij^t in Alg. 1 would keep j).
 *   - the symmetry-breaking test "w_r <= w_k" of Alg. 2/3 is strict, since
 *     w_r is a neighbour of w_k and the graph has no self-loops.
 *   - types are 0-based.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define TGO_MAX_L 16

enum { TGO_OK = 0, TGO_EINVAL = 1, TGO_ENOMEM = 2, TGO_ENOTDIV = 3, TGO_ENEG = 4 };

/* ---------------------------------------------------------------- layout */

static int64_t binom(int64_t a, int64_t b) {
    if (b < 0 || a < b) return 0;
    int64_t r = 1;
    for (int64_t k = 1; k <= b; ++k) r = r * (a - b + k) / k;
    return r;
}

int tgo_num_pairs(int L) { return L * (L + 1) / 2; }
int tgo_row_width(int L) { return 2 * L + 10 * tgo_num_pairs(L); }
int tgo_global_width(int L) {
    return (int)(binom(L + 1, 2) + 2 * binom(L + 2, 3) + 6 * binom(L + 3, 4));
}

/* pair index of unordered (t, t'), built by walking pairs in order */
static int pair_table(int L, int t, int u) {
    if (t > u) { int x = t; t = u; u = x; }
    int idx = 0;
    for (int a = 0; a < L; ++a)
        for (int b = a; b < L; ++b) {
            if (a == t && b == u) return idx;
            ++idx;
        }
    return -1;
}

int tgo_pair_index(int L, int t, int u) { return pair_table(L, t, u); }

/* column of orbit g (3..12) and pair (t, t') inside a row */
static int col_of(int L, int g, int t, int u) {
    return 2 * L + (g - 3) * tgo_num_pairs(L) + pair_table(L, t, u);
}

/* Co-lexicographic position tables for sorted multisets of size K=2,3,4,
 * indexed by the mixed-radix code of the sorted tuple. */
typedef struct {
    int L;
    int32_t *r2, *r3, *r4;
} rank_tables;

static void sort_small(int *a, int k) {
    for (int x = 1; x < k; ++x) {
        int v = a[x], y = x - 1;
        while (y >= 0 && a[y] > v) { a[y + 1] = a[y]; --y; }
        a[y + 1] = v;
    }
}

static int build_rank_tables(rank_tables *rt, int L) {
    rt->L = L;
    rt->r2 = (int32_t *)malloc(sizeof(int32_t) * L * L);
    rt->r3 = (int32_t *)malloc(sizeof(int32_t) * L * L * L);
    rt->r4 = (int32_t *)malloc(sizeof(int32_t) * L * L * L * L);
    if (!rt->r2 || !rt->r3 || !rt->r4) return TGO_ENOMEM;
    int c = 0;
    for (int b = 0; b < L; ++b)
        for (int a = 0; a <= b; ++a) rt->r2[a * L + b] = c++;
    c = 0;
    for (int d = 0; d < L; ++d)
        for (int b = 0; b <= d; ++b)
            for (int a = 0; a <= b; ++a) rt->r3[(a * L + b) * L + d] = c++;
    c = 0;
    for (int e = 0; e < L; ++e)
        for (int d = 0; d <= e; ++d)
            for (int b = 0; b <= d; ++b)
                for (int a = 0; a <= b; ++a) rt->r4[((a * L + b) * L + d) * L + e] = c++;
    return TGO_OK;
}

static void free_rank_tables(rank_tables *rt) {
    free(rt->r2); free(rt->r3); free(rt->r4);
}

static int rank_of(const rank_tables *rt, int *ty, int k) {
    int L = rt->L;
    sort_small(ty, k);
    if (k == 2) return rt->r2[ty[0] * L + ty[1]];
    if (k == 3) return rt->r3[(ty[0] * L + ty[1]) * L + ty[2]];
    return rt->r4[((ty[0] * L + ty[1]) * L + ty[2]) * L + ty[3]];
}

/* ----------------------------------------------------------------- graph */

typedef struct {
    int64_t n;
    const int64_t *row_ptr;
    const int32_t *col;
    const uint8_t *types;
    int L;
} graph;

static int adjacent(const graph *g, int32_t a, int32_t b) {
    int64_t lo = g->row_ptr[a], hi = g->row_ptr[a + 1];
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        int32_t x = g->col[mid];
        if (x == b) return 1;
        if (x < b) lo = mid + 1; else hi = mid;
    }
    return 0;
}

/* --------------------------------------------------- definition (brute) */

/* Orbit of edge (i, j) inside the connected induced subgraph {i, j, k, r};
 * Table 3 read as graph shapes.  adj[x][y] over local indices 0=i 1=j 2=k 3=r. */
static int classify(int adj[4][4]) {
    int deg[4] = {0, 0, 0, 0}, m = 0;
    for (int x = 0; x < 4; ++x)
        for (int y = x + 1; y < 4; ++y)
            if (adj[x][y]) { ++deg[x]; ++deg[y]; ++m; }
    if (m == 3) {
        for (int x = 0; x < 4; ++x) if (deg[x] == 3) return 5;  /* 4-star */
        if (deg[0] == 1 || deg[1] == 1) return 3;                /* 4-path, end edge */
        return 4;                                                /* 4-path, centre edge */
    }
    if (m == 4) {
        int all2 = 1;
        for (int x = 0; x < 4; ++x) if (deg[x] != 2) all2 = 0;
        if (all2) return 6;                                      /* 4-cycle */
        /* tailed triangle: one node of degree 3 (where the tail hangs),
         * one of degree 1 (the tail end) */
        int hub = -1, tail = -1;
        for (int x = 0; x < 4; ++x) {
            if (deg[x] == 3) hub = x;
            if (deg[x] == 1) tail = x;
        }
        if ((hub == 0 && tail == 1) || (hub == 1 && tail == 0)) return 7; /* tail edge */
        if (hub == 0 || hub == 1) return 9;  /* triangle edge touching the hub */
        return 8;                            /* triangle edge opposite the hub */
    }
    if (m == 5) {
        if (deg[0] == 3 && deg[1] == 3) return 11;               /* chord */
        return 10;                                               /* outer edge */
    }
    return 12;                                                   /* 4-clique */
}

static void count_quad(const graph *g, int32_t i, int32_t j, int32_t k, int32_t r,
                       uint64_t *row) {
    int32_t v[4] = {i, j, k, r};
    int adj[4][4];
    memset(adj, 0, sizeof(adj));
    for (int x = 0; x < 4; ++x)
        for (int y = x + 1; y < 4; ++y)
            adj[x][y] = adj[y][x] = adjacent(g, v[x], v[y]);
    int orb = classify(adj);
    row[col_of(g->L, orb, g->types[k], g->types[r])] += 1;
}

/* Union of Gamma_i and Gamma_j minus {i, j}, sorted; returns its length. */
static int64_t candidate_union(const graph *g, int32_t i, int32_t j, int32_t *out) {
    int64_t a = g->row_ptr[i], ae = g->row_ptr[i + 1];
    int64_t b = g->row_ptr[j], be = g->row_ptr[j + 1];
    int64_t c = 0;
    while (a < ae || b < be) {
        int32_t x;
        if (b >= be || (a < ae && g->col[a] < g->col[b])) x = g->col[a++];
        else if (a >= ae || g->col[b] < g->col[a]) x = g->col[b++];
        else { x = g->col[a]; ++a; ++b; }
        if (x != i && x != j) out[c++] = x;
    }
    return c;
}

int tgo_edge_definition_g(const graph *g, int32_t i, int32_t j, uint64_t *row,
                          int32_t *scratch) {
    int L = g->L;
    memset(row, 0, sizeof(uint64_t) * tgo_row_width(L));
    int64_t c = candidate_union(g, i, j, scratch);
    /* 3-node: every k in the union closes a triangle or forms a 3-path */
    for (int64_t x = 0; x < c; ++x) {
        int32_t k = scratch[x];
        int t = g->types[k];
        if (adjacent(g, i, k) && adjacent(g, j, k)) row[t] += 1;
        else row[L + t] += 1;
    }
    /* 4-node, both extra nodes next to i or j */
    for (int64_t x = 0; x < c; ++x)
        for (int64_t y = x + 1; y < c; ++y)
            count_quad(g, i, j, scratch[x], scratch[y], row);
    /* 4-node, r reachable only through k */
    for (int64_t x = 0; x < c; ++x) {
        int32_t k = scratch[x];
        for (int64_t s = g->row_ptr[k]; s < g->row_ptr[k + 1]; ++s) {
            int32_t r = g->col[s];
            if (r == i || r == j) continue;
            if (adjacent(g, i, r) || adjacent(g, j, r)) continue;
            count_quad(g, i, j, k, r, row);
        }
    }
    return TGO_OK;
}

/* ------------------------------------------------------- paper (Alg 1-4) */

enum { PSI_NONE = 0, PSI_SI = 1, PSI_SJ = 2, PSI_T = 3 };

int tgo_edge_paper_g(const graph *g, int32_t i, int32_t j, uint64_t *row, uint8_t *psi) {
    const int L = g->L;
    const uint8_t *phi = g->types;
    const int64_t *rp = g->row_ptr;
    const int32_t *col = g->col;
    int64_t nT[TGO_MAX_L], nSi[TGO_MAX_L], nSj[TGO_MAX_L];
    /* per-edge count vector x over (orbit, unordered type pair), Alg. 4 */
    int64_t x[13][TGO_MAX_L][TGO_MAX_L];
    memset(x, 0, sizeof(x));
    for (int t = 0; t < L; ++t) nT[t] = nSi[t] = nSj[t] = 0;

    /* Alg. 1: typed triangles and typed 3-stars, by marking Gamma_i then
     * scanning Gamma_j (the hashing argument of Thm. 2). */
    for (int64_t s = rp[i]; s < rp[i + 1]; ++s)
        if (col[s] != j) psi[col[s]] = PSI_SI;
    for (int64_t s = rp[j]; s < rp[j + 1]; ++s) {
        int32_t w = col[s];
        if (w == i) continue;
        psi[w] = (psi[w] == PSI_SI) ? PSI_T : PSI_SJ;
    }
    for (int64_t s = rp[i]; s < rp[i + 1]; ++s) {
        int32_t w = col[s];
        if (w == j) continue;
        if (psi[w] == PSI_T) nT[phi[w]]++; else nSi[phi[w]]++;
    }
    for (int64_t s = rp[j]; s < rp[j + 1]; ++s) {
        int32_t w = col[s];
        if (w != i && psi[w] == PSI_SJ) nSj[phi[w]]++;
    }

#define BUMP(orb, tk, tr) do {                                   \
        int a_ = (tk), b_ = (tr);                                \
        if (a_ > b_) { int c_ = a_; a_ = b_; b_ = c_; }          \
        x[orb][a_][b_] += 1;                                     \
    } while (0)

    /* Alg. 2: path-based graphlets, from S_i then from S_j */
    for (int64_t s = rp[i]; s < rp[i + 1]; ++s) {
        int32_t wk = col[s];
        if (wk == j || psi[wk] != PSI_SI) continue;
        for (int64_t q = rp[wk]; q < rp[wk + 1]; ++q) {
            int32_t wr = col[q];
            if (wr == i || wr == j) continue;
            if (psi[wr] == PSI_NONE) BUMP(3, phi[wk], phi[wr]);
            else if (psi[wr] == PSI_SI && wr < wk) BUMP(7, phi[wk], phi[wr]);
        }
    }
    for (int64_t s = rp[j]; s < rp[j + 1]; ++s) {
        int32_t wk = col[s];
        if (wk == i || psi[wk] != PSI_SJ) continue;
        for (int64_t q = rp[wk]; q < rp[wk + 1]; ++q) {
            int32_t wr = col[q];
            if (wr == i || wr == j) continue;
            if (psi[wr] == PSI_NONE) BUMP(3, phi[wk], phi[wr]);
            else if (psi[wr] == PSI_SJ && wr < wk) BUMP(7, phi[wk], phi[wr]);
            else if (psi[wr] == PSI_SI) BUMP(6, phi[wk], phi[wr]);
        }
    }
    /* Alg. 3: triangle-based graphlets, from T_ij */
    for (int64_t s = rp[i]; s < rp[i + 1]; ++s) {
        int32_t wk = col[s];
        if (wk == j || psi[wk] != PSI_T) continue;
        for (int64_t q = rp[wk]; q < rp[wk + 1]; ++q) {
            int32_t wr = col[q];
            if (wr == i || wr == j) continue;
            if (psi[wr] == PSI_T && wr < wk) BUMP(12, phi[wk], phi[wr]);
            else if (psi[wr] == PSI_SI || psi[wr] == PSI_SJ) BUMP(10, phi[wk], phi[wr]);
            else if (psi[wr] == PSI_NONE) BUMP(8, phi[wk], phi[wr]);
        }
    }
#undef BUMP

    /* Alg. 1, loop over type pairs t <= t': Lemmas 1-4 give the orbits that
     * were not enumerated. */
    int rc = TGO_OK;
    for (int t = 0; t < L; ++t)
        for (int u = t; u < L; ++u) {
            int64_t g4, g5, g9, g11;
            if (t == u) {
                g4 = nSi[t] * nSj[t] - x[6][t][u];                               /* Lemma 1 */
                g5 = nSi[t] * (nSi[t] - 1) / 2 + nSj[t] * (nSj[t] - 1) / 2
                     - x[7][t][u];                                               /* Lemma 2 */
                g9 = nT[t] * (nSi[t] + nSj[t]) - x[10][t][u];                    /* Lemma 3 */
                g11 = nT[t] * (nT[t] - 1) / 2 - x[12][t][u];                     /* Lemma 4 */
            } else {
                g4 = nSi[t] * nSj[u] + nSi[u] * nSj[t] - x[6][t][u];
                g5 = nSi[t] * nSi[u] + nSj[t] * nSj[u] - x[7][t][u];
                g9 = nT[t] * (nSi[u] + nSj[u]) + nT[u] * (nSi[t] + nSj[t]) - x[10][t][u];
                g11 = nT[t] * nT[u] - x[12][t][u];
            }
            if (g4 < 0 || g5 < 0 || g9 < 0 || g11 < 0) rc = TGO_ENEG;
            x[4][t][u] = g4; x[5][t][u] = g5; x[9][t][u] = g9; x[11][t][u] = g11;
        }

    memset(row, 0, sizeof(uint64_t) * tgo_row_width(L));
    for (int t = 0; t < L; ++t) {
        row[t] = (uint64_t)nT[t];
        row[L + t] = (uint64_t)(nSi[t] + nSj[t]);   /* Cor. 3 */
    }
    for (int orb = 3; orb <= 12; ++orb)
        for (int t = 0; t < L; ++t)
            for (int u = t; u < L; ++u) row[col_of(L, orb, t, u)] = (uint64_t)x[orb][t][u];

    /* clear the marks left on Gamma_i and Gamma_j */
    for (int64_t s = rp[i]; s < rp[i + 1]; ++s) psi[col[s]] = PSI_NONE;
    for (int64_t s = rp[j]; s < rp[j + 1]; ++s) psi[col[s]] = PSI_NONE;
    return rc;
}

/* --------------------------------------------------- public entry points */

int tgo_edge_definition(int64_t n, const int64_t *row_ptr, const int32_t *col,
                        const uint8_t *types, int L, int32_t i, int32_t j, uint64_t *row) {
    if (L < 1 || L > TGO_MAX_L || i < 0 || j < 0 || i >= n || j >= n) return TGO_EINVAL;
    graph g = {n, row_ptr, col, types, L};
    int64_t cap = (row_ptr[i + 1] - row_ptr[i]) + (row_ptr[j + 1] - row_ptr[j]) + 1;
    int32_t *scratch = (int32_t *)malloc(sizeof(int32_t) * cap);
    if (!scratch) return TGO_ENOMEM;
    int rc = tgo_edge_definition_g(&g, i, j, row, scratch);
    free(scratch);
    return rc;
}

int tgo_edge_paper(int64_t n, const int64_t *row_ptr, const int32_t *col,
                   const uint8_t *types, int L, int32_t i, int32_t j, uint64_t *row) {
    if (L < 1 || L > TGO_MAX_L || i < 0 || j < 0 || i >= n || j >= n) return TGO_EINVAL;
    graph g = {n, row_ptr, col, types, L};
    uint8_t *psi = (uint8_t *)calloc((size_t)n, 1);
    if (!psi) return TGO_ENOMEM;
    int rc = tgo_edge_paper_g(&g, i, j, row, psi);
    free(psi);
    return rc;
}

typedef struct {
    const graph *g;
    const int64_t *uv;
    uint64_t *rows;
    int64_t begin, end;
    int method;
    int rc;
} job;

static void *worker(void *arg) {
    job *jb = (job *)arg;
    const graph *g = jb->g;
    int W = tgo_row_width(g->L);
    jb->rc = TGO_OK;
    uint8_t *psi = NULL;
    int32_t *scratch = NULL;
    if (jb->method == 1) {
        psi = (uint8_t *)calloc((size_t)g->n, 1);
        if (!psi) { jb->rc = TGO_ENOMEM; return NULL; }
    } else {
        int64_t maxd = 0;
        for (int64_t v = 0; v < g->n; ++v) {
            int64_t d = g->row_ptr[v + 1] - g->row_ptr[v];
            if (d > maxd) maxd = d;
        }
        scratch = (int32_t *)malloc(sizeof(int32_t) * (2 * maxd + 1));
        if (!scratch) { jb->rc = TGO_ENOMEM; return NULL; }
    }
    for (int64_t e = jb->begin; e < jb->end; ++e) {
        int32_t i = (int32_t)jb->uv[2 * e], j = (int32_t)jb->uv[2 * e + 1];
        int rc = jb->method == 1 ? tgo_edge_paper_g(g, i, j, jb->rows + e * W, psi)
                                 : tgo_edge_definition_g(g, i, j, jb->rows + e * W, scratch);
        if (rc != TGO_OK) jb->rc = rc;
    }
    free(psi);
    free(scratch);
    return NULL;
}

/* Rows for a list of edges uv[k][2]; method 0 = definition, 1 = paper.
 * Work is split into contiguous ranges, one per thread. */
int tgo_edges(int64_t n, const int64_t *row_ptr, const int32_t *col, const uint8_t *types,
              int L, const int64_t *uv, int64_t k, int method, int nthreads, uint64_t *rows) {
    if (L < 1 || L > TGO_MAX_L || nthreads < 1 || (method != 0 && method != 1)) return TGO_EINVAL;
    for (int64_t e = 0; e < k; ++e) {
        int64_t i = uv[2 * e], j = uv[2 * e + 1];
        if (i < 0 || j < 0 || i >= n || j >= n || i == j) return TGO_EINVAL;
    }
    graph g = {n, row_ptr, col, types, L};
    if (nthreads > k) nthreads = k > 0 ? (int)k : 1;
    pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * nthreads);
    job *jobs = (job *)malloc(sizeof(job) * nthreads);
    if (!th || !jobs) { free(th); free(jobs); return TGO_ENOMEM; }
    for (int t = 0; t < nthreads; ++t) {
        jobs[t].g = &g; jobs[t].uv = uv; jobs[t].rows = rows; jobs[t].method = method;
        jobs[t].begin = k * t / nthreads; jobs[t].end = k * (t + 1) / nthreads;
        pthread_create(&th[t], NULL, worker, &jobs[t]);
    }
    int rc = TGO_OK;
    for (int t = 0; t < nthreads; ++t) {
        pthread_join(th[t], NULL);
        if (jobs[t].rc != TGO_OK) rc = jobs[t].rc;
    }
    free(th); free(jobs);
    return rc;
}

/* Global typed graphlet counts from the rows of ALL edges uv[m][2]
 * (Problem 2; orbit-to-graphlet sums of Sec. 4.4; division by |E(H)|). */
int tgo_global_from_rows(const uint8_t *types, int L, const int64_t *uv, int64_t m,
                         const uint64_t *rows, uint64_t *global) {
    if (L < 1 || L > TGO_MAX_L) return TGO_EINVAL;
    rank_tables rt;
    if (build_rank_tables(&rt, L) != TGO_OK) { free_rank_tables(&rt); return TGO_ENOMEM; }
    int W = tgo_row_width(L);
    int64_t n2 = binom(L + 1, 2), n3 = binom(L + 2, 3), n4 = binom(L + 3, 4);
    int64_t off_h1 = n2, off_h2 = n2 + n3, off_h3 = n2 + 2 * n3;
    int Gw = tgo_global_width(L);
    memset(global, 0, sizeof(uint64_t) * Gw);
    /* graphlet of each orbit (Sec. 4.4): h3 = g3+g4, h4 = g5, h5 = g6,
     * h6 = g7+g8+g9, h7 = g10+g11, h8 = g12 */
    static const int graphlet_of[13] = {0, 0, 0, 3, 3, 4, 5, 6, 6, 6, 7, 7, 8};
    for (int64_t e = 0; e < m; ++e) {
        int a = types[uv[2 * e]], b = types[uv[2 * e + 1]];
        const uint64_t *row = rows + e * W;
        int ty[4];
        ty[0] = a; ty[1] = b;
        global[rank_of(&rt, ty, 2)] += 1;
        for (int t = 0; t < L; ++t) {
            ty[0] = a; ty[1] = b; ty[2] = t;
            int r3 = rank_of(&rt, ty, 3);
            global[off_h1 + r3] += row[L + t];
            global[off_h2 + r3] += row[t];
        }
        for (int orb = 3; orb <= 12; ++orb)
            for (int t = 0; t < L; ++t)
                for (int u = t; u < L; ++u) {
                    ty[0] = a; ty[1] = b; ty[2] = t; ty[3] = u;
                    int r4 = rank_of(&rt, ty, 4);
                    int h = graphlet_of[orb];
                    global[off_h3 + (h - 3) * n4 + r4] += row[col_of(L, orb, t, u)];
                }
    }
    /* each instance was seen once from each of its edges */
    static const int edges_of[9] = {1, 2, 3, 3, 3, 4, 4, 5, 6};
    int rc = TGO_OK;
    int64_t starts[10] = {0, off_h1, off_h2, off_h3, off_h3 + n4, off_h3 + 2 * n4,
                          off_h3 + 3 * n4, off_h3 + 4 * n4, off_h3 + 5 * n4, Gw};
    for (int h = 0; h < 9; ++h)
        for (int64_t q = starts[h]; q < starts[h + 1]; ++q) {
            if (global[q] % edges_of[h]) rc = TGO_ENOTDIV;
            global[q] /= edges_of[h];
        }
    free_rank_tables(&rt);
    return rc;
}

/* ====================================================================
 * Position-aware typed graphlets (Sec. 5; Def. of a position-aware typed
 * graphlet instance): the types must coincide via the isomorphism, so a
 * per-edge count keeps the role each node plays relative to the oriented
 * edge (i, j), and a global count is kept per class of typed graphlets
 * under type-preserving isomorphism.
 *
 * Per-edge row (edge oriented (i, j); node classes S_i, S_j, T, I as in
 * Alg. 1; ordered pairs (x, y) at column x*L + y of their block, unordered
 * pairs {t <= u} at the lexicographic pair index):
 *   TRI    [t]      |T^t|
 *   PATH_I [t]      |S_i^t|                  (3-path k-i-j)
 *   PATH_J [t]      |S_j^t|                  (3-path i-j-k)
 *   G3I  (x, y)     k in S_i^x, r in I^y, k~r      4-path r-k-i-j
 *   G3J  (x, y)     k in S_j^x, r in I^y, k~r      4-path i-j-k-r
 *   G4   (x, y)     k in S_i^x, r in S_j^y, k!~r   4-path k-i-j-r
 *   G5I  {t, u}     k, r in S_i, k!~r              4-star centred at i
 *   G5J  {t, u}     k, r in S_j, k!~r              4-star centred at j
 *   G6   (x, y)     k in S_i^x, r in S_j^y, k~r    4-cycle i-j-r-k
 *   G7I  {t, u}     k, r in S_i, k~r               triangle i-k-r, tail j
 *   G7J  {t, u}     k, r in S_j, k~r               triangle j-k-r, tail i
 *   G8   (x, y)     k in T^x, r in I^y, k~r        triangle i-j-k, tail r at k
 *   G9I  (x, y)     k in T^x, r in S_i^y, k!~r     triangle i-j-k, tail r at i
 *   G9J  (x, y)     k in T^x, r in S_j^y, k!~r     triangle i-j-k, tail r at j
 *   G10I (x, y)     k in T^x, r in S_i^y, k~r      diamond, chord i-k
 *   G10J (x, y)     k in T^x, r in S_j^y, k~r      diamond, chord j-k
 *   G11  {t, u}     k, r in T, k!~r                diamond, chord i-j
 *   G12  {t, u}     k, r in T, k~r                 4-clique
 * Summing each block's columns over the roles gives the typed row
 * (Def. of a typed graphlet instance), so every typed count splits into
 * position-aware ones (the property P_H >= T_H of Sec. 5.2).
 * ==================================================================== */

enum { PB_TRI, PB_PATH_I, PB_PATH_J, PB_G3I, PB_G3J, PB_G4, PB_G5I, PB_G5J, PB_G6, PB_G7I,
       PB_G7J, PB_G8, PB_G9I, PB_G9J, PB_G10I, PB_G10J, PB_G11, PB_G12, PB_NUM };

static int pa_block_width(int L, int b) {
    if (b <= PB_PATH_J) return L;
    if (b == PB_G5I || b == PB_G5J || b == PB_G7I || b == PB_G7J || b == PB_G11 || b == PB_G12)
        return tgo_num_pairs(L);
    return L * L;
}

static int pa_block_start(int L, int b) {
    int s = 0;
    for (int q = 0; q < b; ++q) s += pa_block_width(L, q);
    return s;
}

int tgo_pa_row_width(int L) { return pa_block_start(L, PB_NUM); }

static int pa_col_ord(int L, int b, int x, int y) { return pa_block_start(L, b) + x * L + y; }
static int pa_col_pair(int L, int b, int t, int u) { return pa_block_start(L, b) + pair_table(L, t, u); }

/* --------------------------------------------- PA: the definition itself */

/* One pair {k, r} around oriented edge (i, j): the roles follow from the
 * adjacencies of k and r to i and j (the sets of Alg. 1) and k ~ r. */
static void pa_count_pair(const graph *g, int32_t i, int32_t j, int32_t k, int32_t r,
                          uint64_t *row) {
    const int L = g->L;
    int ki = adjacent(g, i, k), kj = adjacent(g, j, k);
    int ri = adjacent(g, i, r), rj = adjacent(g, j, r);
    int kr = adjacent(g, k, r);
    /* class codes: 0 = I, 1 = S_i, 2 = S_j, 3 = T */
    int ck = (ki ? 1 : 0) | (kj ? 2 : 0), cr = (ri ? 1 : 0) | (rj ? 2 : 0);
    int tk = g->types[k], tr = g->types[r];
    if (ck > cr || (ck == cr && k > r)) {   /* order the pair by class */
        int c = ck; ck = cr; cr = c;
        int t = tk; tk = tr; tr = t;
    }
    int col = -1;
    if (ck == 0) {                               /* k in I */
        if (!kr || cr == 0) return;              /* not connected to the edge */
        if (cr == 1) col = pa_col_ord(L, PB_G3I, tr, tk);
        else if (cr == 2) col = pa_col_ord(L, PB_G3J, tr, tk);
        else col = pa_col_ord(L, PB_G8, tr, tk);
    } else if (ck == 1 && cr == 1) {
        col = pa_col_pair(L, kr ? PB_G7I : PB_G5I, tk, tr);
    } else if (ck == 1 && cr == 2) {
        col = pa_col_ord(L, kr ? PB_G6 : PB_G4, tk, tr);
    } else if (ck == 1 && cr == 3) {
        col = pa_col_ord(L, kr ? PB_G10I : PB_G9I, tr, tk);
    } else if (ck == 2 && cr == 2) {
        col = pa_col_pair(L, kr ? PB_G7J : PB_G5J, tk, tr);
    } else if (ck == 2 && cr == 3) {
        col = pa_col_ord(L, kr ? PB_G10J : PB_G9J, tr, tk);
    } else {                                     /* both in T */
        col = pa_col_pair(L, kr ? PB_G12 : PB_G11, tk, tr);
    }
    row[col] += 1;
}

int tgo_pa_edge_definition_g(const graph *g, int32_t i, int32_t j, uint64_t *row,
                             int32_t *scratch) {
    int L = g->L;
    memset(row, 0, sizeof(uint64_t) * tgo_pa_row_width(L));
    int64_t c = candidate_union(g, i, j, scratch);
    for (int64_t x = 0; x < c; ++x) {
        int32_t k = scratch[x];
        int t = g->types[k];
        int ai = adjacent(g, i, k), aj = adjacent(g, j, k);
        if (ai && aj) row[pa_block_start(L, PB_TRI) + t] += 1;
        else if (ai) row[pa_block_start(L, PB_PATH_I) + t] += 1;
        else row[pa_block_start(L, PB_PATH_J) + t] += 1;
    }
    for (int64_t x = 0; x < c; ++x)
        for (int64_t y = x + 1; y < c; ++y) pa_count_pair(g, i, j, scratch[x], scratch[y], row);
    for (int64_t x = 0; x < c; ++x) {
        int32_t k = scratch[x];
        for (int64_t s = g->row_ptr[k]; s < g->row_ptr[k + 1]; ++s) {
            int32_t r = g->col[s];
            if (r == i || r == j) continue;
            if (adjacent(g, i, r) || adjacent(g, j, r)) continue;
            pa_count_pair(g, i, j, k, r, row);
        }
    }
    return TGO_OK;
}

/* ------------------------- PA: Alg. 1-3 without the type-multiset table */

/* Sec. 5.2: the same enumeration as tgo_edge_paper_g with the keys kept in
 * role order (the lookup table that merges orderings is left out), and the
 * remaining orbits from Lemmas 1-4 applied per role. */
int tgo_pa_edge_paper_g(const graph *g, int32_t i, int32_t j, uint64_t *row, uint8_t *psi) {
    const int L = g->L;
    const uint8_t *phi = g->types;
    const int64_t *rp = g->row_ptr;
    const int32_t *col = g->col;
    int64_t nT[TGO_MAX_L], nSi[TGO_MAX_L], nSj[TGO_MAX_L];
    const int W = tgo_pa_row_width(L);
    int64_t *x = (int64_t *)calloc((size_t)W, sizeof(int64_t));
    if (!x) return TGO_ENOMEM;
    for (int t = 0; t < L; ++t) nT[t] = nSi[t] = nSj[t] = 0;

    for (int64_t s = rp[i]; s < rp[i + 1]; ++s)
        if (col[s] != j) psi[col[s]] = PSI_SI;
    for (int64_t s = rp[j]; s < rp[j + 1]; ++s) {
        int32_t w = col[s];
        if (w == i) continue;
        psi[w] = (psi[w] == PSI_SI) ? PSI_T : PSI_SJ;
    }
    for (int64_t s = rp[i]; s < rp[i + 1]; ++s) {
        int32_t w = col[s];
        if (w == j) continue;
        if (psi[w] == PSI_T) nT[phi[w]]++; else nSi[phi[w]]++;
    }
    for (int64_t s = rp[j]; s < rp[j + 1]; ++s) {
        int32_t w = col[s];
        if (w != i && psi[w] == PSI_SJ) nSj[phi[w]]++;
    }
    /* Alg. 2 from S_i: 4-paths r-k-i-j and triangles i-k-r */
    for (int64_t s = rp[i]; s < rp[i + 1]; ++s) {
        int32_t wk = col[s];
        if (wk == j || psi[wk] != PSI_SI) continue;
        for (int64_t q = rp[wk]; q < rp[wk + 1]; ++q) {
            int32_t wr = col[q];
            if (wr == i || wr == j) continue;
            if (psi[wr] == PSI_NONE) x[pa_col_ord(L, PB_G3I, phi[wk], phi[wr])] += 1;
            else if (psi[wr] == PSI_SI && wr < wk) x[pa_col_pair(L, PB_G7I, phi[wk], phi[wr])] += 1;
        }
    }
    /* Alg. 2 from S_j: 4-paths i-j-k-r, triangles j-k-r, 4-cycles */
    for (int64_t s = rp[j]; s < rp[j + 1]; ++s) {
        int32_t wk = col[s];
        if (wk == i || psi[wk] != PSI_SJ) continue;
        for (int64_t q = rp[wk]; q < rp[wk + 1]; ++q) {
            int32_t wr = col[q];
            if (wr == i || wr == j) continue;
            if (psi[wr] == PSI_NONE) x[pa_col_ord(L, PB_G3J, phi[wk], phi[wr])] += 1;
            else if (psi[wr] == PSI_SJ && wr < wk) x[pa_col_pair(L, PB_G7J, phi[wk], phi[wr])] += 1;
            else if (psi[wr] == PSI_SI) x[pa_col_ord(L, PB_G6, phi[wr], phi[wk])] += 1;
        }
    }
    /* Alg. 3 from T: 4-cliques, chordal cycles, tailed triangles at k */
    for (int64_t s = rp[i]; s < rp[i + 1]; ++s) {
        int32_t wk = col[s];
        if (wk == j || psi[wk] != PSI_T) continue;
        for (int64_t q = rp[wk]; q < rp[wk + 1]; ++q) {
            int32_t wr = col[q];
            if (wr == i || wr == j) continue;
            if (psi[wr] == PSI_T && wr < wk) x[pa_col_pair(L, PB_G12, phi[wk], phi[wr])] += 1;
            else if (psi[wr] == PSI_SI) x[pa_col_ord(L, PB_G10I, phi[wk], phi[wr])] += 1;
            else if (psi[wr] == PSI_SJ) x[pa_col_ord(L, PB_G10J, phi[wk], phi[wr])] += 1;
            else if (psi[wr] == PSI_NONE) x[pa_col_ord(L, PB_G8, phi[wk], phi[wr])] += 1;
        }
    }
    /* Lemmas 1-4 per role */
    int rc = TGO_OK;
    for (int a = 0; a < L; ++a)
        for (int b = 0; b < L; ++b) {
            int64_t g4 = nSi[a] * nSj[b] - x[pa_col_ord(L, PB_G6, a, b)];          /* Lemma 1 */
            int64_t g9i = nT[a] * nSi[b] - x[pa_col_ord(L, PB_G10I, a, b)];       /* Lemma 3 */
            int64_t g9j = nT[a] * nSj[b] - x[pa_col_ord(L, PB_G10J, a, b)];
            if (g4 < 0 || g9i < 0 || g9j < 0) rc = TGO_ENEG;
            x[pa_col_ord(L, PB_G4, a, b)] = g4;
            x[pa_col_ord(L, PB_G9I, a, b)] = g9i;
            x[pa_col_ord(L, PB_G9J, a, b)] = g9j;
        }
    for (int t = 0; t < L; ++t)
        for (int u = t; u < L; ++u) {
            int64_t g5i, g5j, g11;
            if (t == u) {
                g5i = nSi[t] * (nSi[t] - 1) / 2 - x[pa_col_pair(L, PB_G7I, t, u)];  /* Lemma 2 */
                g5j = nSj[t] * (nSj[t] - 1) / 2 - x[pa_col_pair(L, PB_G7J, t, u)];
                g11 = nT[t] * (nT[t] - 1) / 2 - x[pa_col_pair(L, PB_G12, t, u)];    /* Lemma 4 */
            } else {
                g5i = nSi[t] * nSi[u] - x[pa_col_pair(L, PB_G7I, t, u)];
                g5j = nSj[t] * nSj[u] - x[pa_col_pair(L, PB_G7J, t, u)];
                g11 = nT[t] * nT[u] - x[pa_col_pair(L, PB_G12, t, u)];
            }
            if (g5i < 0 || g5j < 0 || g11 < 0) rc = TGO_ENEG;
            x[pa_col_pair(L, PB_G5I, t, u)] = g5i;
            x[pa_col_pair(L, PB_G5J, t, u)] = g5j;
            x[pa_col_pair(L, PB_G11, t, u)] = g11;
        }
    for (int t = 0; t < L; ++t) {
        x[pa_block_start(L, PB_TRI) + t] = nT[t];
        x[pa_block_start(L, PB_PATH_I) + t] = nSi[t];
        x[pa_block_start(L, PB_PATH_J) + t] = nSj[t];
    }
    for (int q = 0; q < W; ++q) row[q] = (uint64_t)x[q];
    free(x);
    for (int64_t s = rp[i]; s < rp[i + 1]; ++s) psi[col[s]] = PSI_NONE;
    for (int64_t s = rp[j]; s < rp[j + 1]; ++s) psi[col[s]] = PSI_NONE;
    return rc;
}

typedef struct {
    const graph *g;
    const int64_t *uv;
    uint64_t *rows;
    int64_t begin, end;
    int method;
    int rc;
} pa_job;

static void *pa_worker(void *arg) {
    pa_job *jb = (pa_job *)arg;
    const graph *g = jb->g;
    int W = tgo_pa_row_width(g->L);
    jb->rc = TGO_OK;
    uint8_t *psi = (uint8_t *)calloc((size_t)g->n, 1);
    int64_t maxd = 0;
    for (int64_t v = 0; v < g->n; ++v) {
        int64_t d = g->row_ptr[v + 1] - g->row_ptr[v];
        if (d > maxd) maxd = d;
    }
    int32_t *scratch = (int32_t *)malloc(sizeof(int32_t) * (2 * maxd + 1));
    if (!psi || !scratch) { free(psi); free(scratch); jb->rc = TGO_ENOMEM; return NULL; }
    for (int64_t e = jb->begin; e < jb->end; ++e) {
        int32_t i = (int32_t)jb->uv[2 * e], j = (int32_t)jb->uv[2 * e + 1];
        int rc = jb->method == 1 ? tgo_pa_edge_paper_g(g, i, j, jb->rows + e * W, psi)
                                 : tgo_pa_edge_definition_g(g, i, j, jb->rows + e * W, scratch);
        if (rc != TGO_OK) jb->rc = rc;
    }
    free(psi);
    free(scratch);
    return NULL;
}

/* Position-aware rows for edges uv[k][2], each oriented as given; method 0
 * = definition, 1 = paper. */
int tgo_pa_edges(int64_t n, const int64_t *row_ptr, const int32_t *col, const uint8_t *types,
                 int L, const int64_t *uv, int64_t k, int method, int nthreads, uint64_t *rows) {
    if (L < 1 || L > TGO_MAX_L || nthreads < 1 || (method != 0 && method != 1)) return TGO_EINVAL;
    for (int64_t e = 0; e < k; ++e) {
        int64_t i = uv[2 * e], j = uv[2 * e + 1];
        if (i < 0 || j < 0 || i >= n || j >= n || i == j) return TGO_EINVAL;
    }
    graph g = {n, row_ptr, col, types, L};
    if (nthreads > k) nthreads = k > 0 ? (int)k : 1;
    pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * nthreads);
    pa_job *jobs = (pa_job *)malloc(sizeof(pa_job) * nthreads);
    if (!th || !jobs) { free(th); free(jobs); return TGO_ENOMEM; }
    for (int t = 0; t < nthreads; ++t) {
        jobs[t].g = &g; jobs[t].uv = uv; jobs[t].rows = rows; jobs[t].method = method;
        jobs[t].begin = k * t / nthreads; jobs[t].end = k * (t + 1) / nthreads;
        pthread_create(&th[t], NULL, pa_worker, &jobs[t]);
    }
    int rc = TGO_OK;
    for (int t = 0; t < nthreads; ++t) {
        pthread_join(th[t], NULL);
        if (jobs[t].rc != TGO_OK) rc = jobs[t].rc;
    }
    free(th); free(jobs);
    return rc;
}

/* ------------------------------------------ PA: global counts per class
 *
 * A class is a typed graphlet up to type-preserving isomorphism.  Node
 * positions of each graphlet (the labelling used to describe a class):
 *   h0 edge (0, 1); h1 3-path 1-0-2 (0 the centre); h2 triangle 0, 1, 2;
 *   h3 4-path 0-1-2-3; h4 4-star, 0 the centre; h5 4-cycle 0-1-2-3-0;
 *   h6 tailed triangle: triangle 0, 1, 2, tail 2-3; h7 chordal cycle
 *   0-1-2-3-0 with chord 0-2; h8 4-clique.
 * Class order inside each block (each class listed once, by the
 * representative labelling named):
 *   h0  {t0 <= t1} co-lexicographic                      (multisets)
 *   h1  centre c, then ends {t1 <= t2} co-lexicographic
 *   h2  multiset co-lexicographic
 *   h3  halves A = (t0, t1), B = (t3, t2) read as numbers t*L + t': pairs
 *       A <= B, co-lexicographic (B outer, A inner)
 *   h4  centre c, then leaves {t1 <= t2 <= t3} co-lexicographic
 *   h5  diagonals D1 = {t0, t2}, D2 = {t1, t3}, each a pair index p =
 *       co-lexicographic rank of the unordered pair; pairs of pair indices
 *       p(D1) <= p(D2), co-lexicographic
 *   h6  tail tip t3 outer, attachment t2, then {t0 <= t1} co-lexicographic
 *   h7  chord {t0 <= t2} co-lexicographic outer, rim {t1 <= t3} inner
 *   h8  multiset co-lexicographic
 * The oracle enumerates these representatives in that order and maps every
 * labelling to its class through the graphlet's automorphisms (a table
 * over all L^k labellings), not by a rank formula.
 * ==================================================================== */

#define PA_NG 9

static const int pa_k[PA_NG] = {2, 3, 3, 4, 4, 4, 4, 4, 4};

/* automorphism groups as position permutations (image of position q) */
static const int aut_h0[][4] = {{0, 1}, {1, 0}};
static const int aut_h1[][4] = {{0, 1, 2}, {0, 2, 1}};
static const int aut_h2[][4] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
static const int aut_h3[][4] = {{0, 1, 2, 3}, {3, 2, 1, 0}};
static const int aut_h4[][4] = {{0, 1, 2, 3}, {0, 1, 3, 2}, {0, 2, 1, 3},
                                {0, 2, 3, 1}, {0, 3, 1, 2}, {0, 3, 2, 1}};
static const int aut_h5[][4] = {{0, 1, 2, 3}, {1, 2, 3, 0}, {2, 3, 0, 1}, {3, 0, 1, 2},
                                {3, 2, 1, 0}, {0, 3, 2, 1}, {1, 0, 3, 2}, {2, 1, 0, 3}};
static const int aut_h6[][4] = {{0, 1, 2, 3}, {1, 0, 2, 3}};
static const int aut_h7[][4] = {{0, 1, 2, 3}, {2, 1, 0, 3}, {0, 3, 2, 1}, {2, 3, 0, 1}};

typedef struct {
    int L;
    int64_t width;            /* total classes */
    int64_t start[PA_NG + 1]; /* first class of each graphlet */
    int32_t *cls[PA_NG];      /* labelling code (base L, position 0 most significant) -> class */
} pa_tables;

static int64_t pa_code(const int *t, int k, int L) {
    int64_t c = 0;
    for (int q = 0; q < k; ++q) c = c * L + t[q];
    return c;
}

/* Give the representative labelling rep and all its automorphic images
 * class `id` (if not given yet); returns 1 if rep was new. */
static int pa_assign(pa_tables *pt, int h, const int *rep, int64_t id) {
    const int k = pa_k[h], L = pt->L;
    const int(*aut)[4];
    int na;
    switch (h) {
        case 0: aut = aut_h0; na = 2; break;
        case 1: aut = aut_h1; na = 2; break;
        case 2: aut = aut_h2; na = 6; break;
        case 3: aut = aut_h3; na = 2; break;
        case 4: aut = aut_h4; na = 6; break;
        case 5: aut = aut_h5; na = 8; break;
        case 6: aut = aut_h6; na = 2; break;
        case 7: aut = aut_h7; na = 4; break;
        default: aut = NULL; na = 0; break;
    }
    if (h == 8) {
        /* the 4-clique: every permutation of the positions */
        int p[4];
        int fresh = pt->cls[h][pa_code(rep, 4, L)] < 0;
        for (p[0] = 0; p[0] < 4; ++p[0])
            for (p[1] = 0; p[1] < 4; ++p[1])
                for (p[2] = 0; p[2] < 4; ++p[2])
                    for (p[3] = 0; p[3] < 4; ++p[3]) {
                        if (p[0] == p[1] || p[0] == p[2] || p[0] == p[3] || p[1] == p[2] ||
                            p[1] == p[3] || p[2] == p[3]) continue;
                        int img[4];
                        for (int q = 0; q < 4; ++q) img[p[q]] = rep[q];
                        pt->cls[h][pa_code(img, 4, L)] = (int32_t)id;
                    }
        return fresh;
    }
    int fresh = pt->cls[h][pa_code(rep, k, L)] < 0;
    for (int a = 0; a < na; ++a) {
        int img[4];
        for (int q = 0; q < k; ++q) img[aut[a][q]] = rep[q];
        pt->cls[h][pa_code(img, k, L)] = (int32_t)id;
    }
    return fresh;
}

static void pa_free_tables(pa_tables *pt) {
    for (int h = 0; h < PA_NG; ++h) free(pt->cls[h]);
}

static int pa_build_tables(pa_tables *pt, int L) {
    memset(pt, 0, sizeof(*pt));
    pt->L = L;
    for (int h = 0; h < PA_NG; ++h) {
        int64_t sz = 1;
        for (int q = 0; q < pa_k[h]; ++q) sz *= L;
        pt->cls[h] = (int32_t *)malloc(sizeof(int32_t) * sz);
        if (!pt->cls[h]) { pa_free_tables(pt); return TGO_ENOMEM; }
        for (int64_t q = 0; q < sz; ++q) pt->cls[h][q] = -1;
    }
    int64_t id = 0;
    int r[4];
    int dup = 0;  /* a representative met twice: the class order is not a listing */
    for (int h = 0; h < PA_NG; ++h) {
        pt->start[h] = id;
        int64_t local = 0;
        switch (h) {
            case 0:
                for (int b = 0; b < L; ++b)
                    for (int a = 0; a <= b; ++a) { r[0] = a; r[1] = b; if (!pa_assign(pt, h, r, id + local++)) dup = 1; }
                break;
            case 1:
                for (int c = 0; c < L; ++c)
                    for (int b = 0; b < L; ++b)
                        for (int a = 0; a <= b; ++a) {
                            r[0] = c; r[1] = a; r[2] = b;
                            if (!pa_assign(pt, h, r, id + local++)) dup = 1;
                        }
                break;
            case 2:
            case 8: {
                int k = pa_k[h];
                if (k == 3) {
                    for (int c = 0; c < L; ++c)
                        for (int b = 0; b <= c; ++b)
                            for (int a = 0; a <= b; ++a) {
                                r[0] = a; r[1] = b; r[2] = c;
                                if (!pa_assign(pt, h, r, id + local++)) dup = 1;
                            }
                } else {
                    for (int d = 0; d < L; ++d)
                        for (int c = 0; c <= d; ++c)
                            for (int b = 0; b <= c; ++b)
                                for (int a = 0; a <= b; ++a) {
                                    r[0] = a; r[1] = b; r[2] = c; r[3] = d;
                                    if (!pa_assign(pt, h, r, id + local++)) dup = 1;
                                }
                }
                break;
            }
            case 3:
                for (int B = 0; B < L * L; ++B)
                    for (int A = 0; A <= B; ++A) {
                        r[0] = A / L; r[1] = A % L; r[3] = B / L; r[2] = B % L;
                        if (!pa_assign(pt, h, r, id + local++)) dup = 1;
                    }
                break;
            case 4:
                for (int c = 0; c < L; ++c)
                    for (int z = 0; z < L; ++z)
                        for (int y = 0; y <= z; ++y)
                            for (int x = 0; x <= y; ++x) {
                                r[0] = c; r[1] = x; r[2] = y; r[3] = z;
                                if (!pa_assign(pt, h, r, id + local++)) dup = 1;
                            }
                break;
            case 5: {
                int P = tgo_num_pairs(L);
                for (int p2 = 0; p2 < P; ++p2)
                    for (int p1 = 0; p1 <= p2; ++p1) {
                        /* pair index -> (lo, hi), walking pairs co-lexicographically */
                        int q = 0, d1lo = 0, d1hi = 0, d2lo = 0, d2hi = 0;
                        for (int hi = 0; hi < L; ++hi)
                            for (int lo = 0; lo <= hi; ++lo, ++q) {
                                if (q == p1) { d1lo = lo; d1hi = hi; }
                                if (q == p2) { d2lo = lo; d2hi = hi; }
                            }
                        r[0] = d1lo; r[2] = d1hi; r[1] = d2lo; r[3] = d2hi;
                        if (!pa_assign(pt, h, r, id + local++)) dup = 1;
                    }
                break;
            }
            case 6:
                for (int z = 0; z < L; ++z)
                    for (int a = 0; a < L; ++a)
                        for (int y = 0; y < L; ++y)
                            for (int x = 0; x <= y; ++x) {
                                r[0] = x; r[1] = y; r[2] = a; r[3] = z;
                                if (!pa_assign(pt, h, r, id + local++)) dup = 1;
                            }
                break;
            case 7:
                for (int cb = 0; cb < L; ++cb)
                    for (int ca = 0; ca <= cb; ++ca)
                        for (int rb = 0; rb < L; ++rb)
                            for (int ra = 0; ra <= rb; ++ra) {
                                r[0] = ca; r[2] = cb; r[1] = ra; r[3] = rb;
                                if (!pa_assign(pt, h, r, id + local++)) dup = 1;
                            }
                break;
        }
        id += local;
    }
    pt->start[PA_NG] = id;
    pt->width = id;
    if (dup) { pa_free_tables(pt); return TGO_EINVAL; }
    /* every labelling must have a class */
    for (int h = 0; h < PA_NG; ++h) {
        int64_t sz = 1;
        for (int q = 0; q < pa_k[h]; ++q) sz *= L;
        for (int64_t q = 0; q < sz; ++q)
            if (pt->cls[h][q] < 0) { pa_free_tables(pt); return TGO_EINVAL; }
    }
    return TGO_OK;
}

int64_t tgo_pa_global_width(int L) {
    if (L < 1 || L > TGO_MAX_L) return 0;
    pa_tables pt;
    if (pa_build_tables(&pt, L) != TGO_OK) return 0;
    int64_t w = pt.width;
    pa_free_tables(&pt);
    return w;
}

/* Representative labelling (types by position) of class idx and its
 * graphlet h (0..8); returns the node count, or 0 if idx is out of range. */
int tgo_pa_global_describe(int L, int64_t idx, int *graphlet, int *types_by_position) {
    if (L < 1 || L > TGO_MAX_L) return 0;
    pa_tables pt;
    if (pa_build_tables(&pt, L) != TGO_OK) return 0;
    int found = 0;
    for (int h = 0; h < PA_NG && !found; ++h) {
        if (idx < pt.start[h] || idx >= pt.start[h + 1]) continue;
        const int k = pa_k[h];
        int64_t sz = 1;
        for (int q = 0; q < k; ++q) sz *= L;
        /* the smallest labelling code of the class */
        for (int64_t c = 0; c < sz; ++c)
            if (pt.cls[h][c] == idx) {
                int64_t v = c;
                for (int q = k - 1; q >= 0; --q) { types_by_position[q] = (int)(v % L); v /= L; }
                *graphlet = h;
                found = k;
                break;
            }
    }
    pa_free_tables(&pt);
    return found;
}

static const int pa_edges_of[PA_NG] = {1, 2, 3, 3, 3, 4, 4, 5, 6};

static void pa_add(const pa_tables *pt, uint64_t *global, int h, const int *lab, uint64_t v) {
    if (!v) return;
    global[pt->cls[h][pa_code(lab, pa_k[h], pt->L)]] += v;
}

/* Global position-aware counts from the position-aware rows of ALL edges
 * uv[m][2] (each row oriented as its uv entry): every column names the full
 * labelling of its instance, each instance is met once per edge, and the
 * sums are divided by the graphlet's edge count (Problem 2). */
int tgo_pa_global_from_rows(const uint8_t *types, int L, const int64_t *uv, int64_t m,
                            const uint64_t *rows, uint64_t *global) {
    if (L < 1 || L > TGO_MAX_L) return TGO_EINVAL;
    pa_tables pt;
    int rc = pa_build_tables(&pt, L);
    if (rc != TGO_OK) return rc;
    const int W = tgo_pa_row_width(L);
    memset(global, 0, sizeof(uint64_t) * pt.width);
    for (int64_t e = 0; e < m; ++e) {
        const int a = types[uv[2 * e]], b = types[uv[2 * e + 1]];
        const uint64_t *row = rows + e * W;
        int lab[4];
        lab[0] = a; lab[1] = b;
        pa_add(&pt, global, 0, lab, 1);
        for (int t = 0; t < L; ++t) {
            lab[0] = a; lab[1] = b; lab[2] = t;                 /* triangle */
            pa_add(&pt, global, 2, lab, row[pa_block_start(L, PB_TRI) + t]);
            lab[0] = a; lab[1] = t; lab[2] = b;                 /* 3-path t-i-j, centre i */
            pa_add(&pt, global, 1, lab, row[pa_block_start(L, PB_PATH_I) + t]);
            lab[0] = b; lab[1] = a; lab[2] = t;                 /* 3-path i-j-t, centre j */
            pa_add(&pt, global, 1, lab, row[pa_block_start(L, PB_PATH_J) + t]);
        }
        for (int x = 0; x < L; ++x)
            for (int y = 0; y < L; ++y) {
                int l3[4];
                l3[0] = y; l3[1] = x; l3[2] = a; l3[3] = b;      /* r-k-i-j */
                pa_add(&pt, global, 3, l3, row[pa_col_ord(L, PB_G3I, x, y)]);
                l3[0] = a; l3[1] = b; l3[2] = x; l3[3] = y;      /* i-j-k-r */
                pa_add(&pt, global, 3, l3, row[pa_col_ord(L, PB_G3J, x, y)]);
                l3[0] = x; l3[1] = a; l3[2] = b; l3[3] = y;      /* k-i-j-r */
                pa_add(&pt, global, 3, l3, row[pa_col_ord(L, PB_G4, x, y)]);
                l3[0] = a; l3[1] = b; l3[2] = y; l3[3] = x;      /* cycle i-j-r-k */
                pa_add(&pt, global, 5, l3, row[pa_col_ord(L, PB_G6, x, y)]);
                l3[0] = a; l3[1] = b; l3[2] = x; l3[3] = y;      /* triangle i, j, k; tail r at k */
                pa_add(&pt, global, 6, l3, row[pa_col_ord(L, PB_G8, x, y)]);
                l3[0] = b; l3[1] = x; l3[2] = a; l3[3] = y;      /* tail r at i */
                pa_add(&pt, global, 6, l3, row[pa_col_ord(L, PB_G9I, x, y)]);
                l3[0] = a; l3[1] = x; l3[2] = b; l3[3] = y;      /* tail r at j */
                pa_add(&pt, global, 6, l3, row[pa_col_ord(L, PB_G9J, x, y)]);
                l3[0] = a; l3[1] = b; l3[2] = x; l3[3] = y;      /* chord i-k, rim j, r */
                pa_add(&pt, global, 7, l3, row[pa_col_ord(L, PB_G10I, x, y)]);
                l3[0] = b; l3[1] = a; l3[2] = x; l3[3] = y;      /* chord j-k, rim i, r */
                pa_add(&pt, global, 7, l3, row[pa_col_ord(L, PB_G10J, x, y)]);
            }
        for (int t = 0; t < L; ++t)
            for (int u = t; u < L; ++u) {
                int l4[4];
                l4[0] = a; l4[1] = b; l4[2] = t; l4[3] = u;      /* star at i: leaves j, k, r */
                pa_add(&pt, global, 4, l4, row[pa_col_pair(L, PB_G5I, t, u)]);
                l4[0] = b; l4[1] = a;
                pa_add(&pt, global, 4, l4, row[pa_col_pair(L, PB_G5J, t, u)]);
                l4[0] = t; l4[1] = u; l4[2] = a; l4[3] = b;      /* triangle i, k, r; tail j at i */
                pa_add(&pt, global, 6, l4, row[pa_col_pair(L, PB_G7I, t, u)]);
                l4[2] = b; l4[3] = a;
                pa_add(&pt, global, 6, l4, row[pa_col_pair(L, PB_G7J, t, u)]);
                l4[0] = a; l4[1] = t; l4[2] = b; l4[3] = u;      /* chord i-j, rim k, r */
                pa_add(&pt, global, 7, l4, row[pa_col_pair(L, PB_G11, t, u)]);
                l4[0] = a; l4[1] = b; l4[2] = t; l4[3] = u;
                pa_add(&pt, global, 8, l4, row[pa_col_pair(L, PB_G12, t, u)]);
            }
    }
    rc = TGO_OK;
    for (int h = 0; h < PA_NG; ++h)
        for (int64_t q = pt.start[h]; q < pt.start[h + 1]; ++q) {
            if (global[q] % pa_edges_of[h]) rc = TGO_ENOTDIV;
            global[q] /= pa_edges_of[h];
        }
    pa_free_tables(&pt);
    return rc;
}
