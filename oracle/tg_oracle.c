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
