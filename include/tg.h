/*
 * tg.h - C ABI of the MI355X typed-graphlet counting library (libtg.so).
 *
 * Computes, for every edge of a simple undirected graph whose nodes carry one
 * of L types, the counts of all typed 2-, 3- and 4-node graphlets that
 * contain the edge (local typed graphlet counting, Problem 1 of Rossi et al.,
 * "Heterogeneous Graphlets"), and the global count of every typed graphlet
 * (Problem 2).  Algorithm 1 of the paper requires a graph and ensures the
 * counts for each edge; this library produces them as a dense table.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Graph: CSR over n nodes with int64 row offsets row_ptr[n+1] and int32
 *   neighbour ids col[nnz], nnz = 2M.  Every row is strictly ascending
 *   (no duplicates), contains no self-loop, and the adjacency is symmetric.
 *   types[n] (uint8) holds each node's type in [0, L), 1 <= L <= TG_MAX_L.
 * Memory: graph, types, outputs and workspace are DEVICE pointers on the
 *   current HIP device.  The caller allocates and owns all of them; the
 *   library allocates no device memory and frees nothing.
 * Stream: every kernel runs on the given hipStream_t (passed as void*, NULL
 *   means the null stream).  The call synchronises that stream once during
 *   the input checks (twice for a batch) and once at the end, to read back
 *   the device-side checks, so the counts are complete when it returns
 *   (tg_count_batch_async: never).
 * Errors: every call returns tg_status.  Input checks run before any output
 *   is written; on an input error the outputs are left untouched.  Device
 *   faults reported by HIP map to TG_E_DEVICE; a failed internal check
 *   (TG_E_INTERNAL) leaves the outputs unspecified.
 * Determinism: all counts are exact unsigned 64-bit integers; identical
 *   inputs give identical outputs regardless of scheduling.
 *
 * Per-edge row layout (row_width(L) = 2L + 10 P columns, P = L(L+1)/2):
 *   [ tri[t], t = 0..L-1 ]        |T_ij^t|: type-t nodes adjacent to both
 *                                  i and j (typed triangles, Cor. 1)
 *   [ path3[t], t = 0..L-1 ]      |S_i^t| + |S_j^t|, S_i^t the type-t
 *                                  neighbours of i that are neither j nor
 *                                  adjacent to j (typed 3-paths, Cor. 2-3)
 *   [ g3 | g4 | ... | g12 ]       ten blocks of P columns, one per 4-node
 *                                  orbit of Table 3; inside a block the
 *                                  unordered type pair {t, t'} (t <= t') of
 *                                  the two nodes outside the edge, in
 *                                  lexicographic order: index
 *                                  t*L - t(t-1)/2 + (t'-t).
 *   Orbits: g3 4-path end edge, g4 4-path centre edge, g5 4-star, g6 4-cycle,
 *   g7 tailed-triangle tail, g8 tailed-triangle edge opposite the tail's
 *   node, g9 tailed-triangle edge at the tail's node, g10 chordal-cycle outer
 *   edge, g11 chordal-cycle chord, g12 4-clique.
 * Edge order: row e belongs to the e-th undirected edge (u, v), u < v, in
 *   lexicographic order of (u, v) (the unique edge id of the parallel
 *   scheme, Sec. 4.7).
 * Global layout (global_width(L) = C(L+1,2) + 2 C(L+2,3) + 6 C(L+3,4)):
 *   blocks h0 (edges), h1 (3-paths), h2 (triangles), h3 (4-paths),
 *   h4 (4-stars), h5 (4-cycles), h6 (tailed triangles), h7 (chordal cycles),
 *   h8 (4-cliques); inside a block, the sorted type multiset of the
 *   graphlet's nodes at its co-lexicographic rank
 *   sum_k C(s_k + k, k + 1) over the sorted types s_0 <= s_1 <= ....
 *   Each entry is the number of instances (per-edge sums divided by the
 *   graphlet's edge count, Problem 2 / Sec. 6).
 */
#ifndef TG_H
#define TG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TG_MAX_L 16

typedef enum tg_status {
    TG_OK = 0,
    TG_E_INVALID_ARG = 1, /* null pointer, negative size, odd nnz, ... */
    TG_E_NOT_SIMPLE = 2,  /* unsorted row, duplicate, self-loop, asymmetric, id out of range */
    TG_E_TYPE_RANGE = 3,  /* some types[v] >= L */
    TG_E_L_RANGE = 4,     /* L < 1 or L > TG_MAX_L */
    TG_E_WORKSPACE = 5,   /* workspace smaller than tg_workspace_bytes() */
    TG_E_DEVICE = 6,      /* a HIP call failed */
    TG_E_INTERNAL = 7,    /* an internal consistency check failed */
    TG_E_TOO_LARGE = 8,   /* n or nnz beyond the supported range (see below) */
    TG_E_BATCH = 9,       /* batch descriptor inconsistent, or an edge joins two graphs */
    TG_E_OOM = 10,        /* the request can never fit the serving arena or a worker's region */
    TG_E_TIMEOUT = 11,    /* tg_server_wait: the request is not finished yet */
    TG_E_NO_CONVERGENCE = 12 /* tg_graphlet_embedding: iteration limit reached */
} tg_status;

/* Human-readable name of a status code (static string). */
const char *tg_status_str(tg_status s);

/* Number of uint64 columns of a per-edge row, 2L + 10 L(L+1)/2; 0 if L is
 * out of range. */
int32_t tg_row_width(int32_t L);

/* Number of uint64 entries of the global table; 0 if L is out of range. */
int32_t tg_global_width(int32_t L);

/* Bytes of device workspace tg_count_typed_graphlets needs for a graph of n
 * nodes, nnz adjacency entries and L types.  Returns 0 for invalid sizes.
 * Supported range: n < 2^31, nnz < 2^32. */
size_t tg_workspace_bytes(int64_t n, int64_t nnz, int32_t L);

/* Count typed 2-, 3- and 4-node graphlets for every edge (Problem 1,
 * Algorithm 1) and globally (Problem 2).
 *   row_ptr, col, types   device CSR and node types as described above.
 *   per_edge              device uint64 [nnz/2][tg_row_width(L)] or NULL to
 *                         skip the per-edge table (global counts only).
 *   global_counts         device uint64 [tg_global_width(L)], or NULL.
 *   workspace             device buffer of ws_bytes >= tg_workspace_bytes(),
 *                         256-byte aligned (TG_E_INVALID_ARG otherwise).
 *   stream                hipStream_t as void*.
 * Returns when the counts are complete (see Stream above). */
tg_status tg_count_typed_graphlets(const int64_t *row_ptr, const int32_t *col,
                                   const uint8_t *types, int64_t n, int64_t nnz, int32_t L,
                                   uint64_t *per_edge, uint64_t *global_counts,
                                   void *workspace, size_t ws_bytes, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * counts as tg_count_typed_graphlets, with the workspace taken from a
 * static device array of TG_NOALLOC_SCRATCH_BYTES bytes that the library
 * holds on each device it runs on until the process ends.  The call
 * allocates nothing (no hipMalloc, no hipFree, no allocating library
 * routine).
 *   row_ptr, col, types, n, nnz, L, per_edge, global_counts, stream
 *                         as for tg_count_typed_graphlets (device pointers,
 *                         caller-owned outputs).
 * The workspace layout of the graph must fit the array: a graph whose
 * per-node and per-edge regions (with one heavy 4-cycle map and one
 * heavy-edge list) exceed it gives TG_E_TOO_LARGE before any device work;
 * smaller graphs run with as many heavy workgroups and super-hub bitmaps as
 * the rest of the array holds.  Every call on a device shares that
 * device's array and finds the previous call's contents there (the library
 * clears what must start at zero): calls that overlap on one device, on any
 * streams or host threads, race and give undefined results; serialise them.
 * Other errors as for tg_count_typed_graphlets. */
#define TG_NOALLOC_SCRATCH_BYTES (256u << 20)
tg_status tg_count_typed_graphlets_noalloc(const int64_t *row_ptr, const int32_t *col,
                                           const uint8_t *types, int64_t n, int64_t nnz,
                                           int32_t L, uint64_t *per_edge,
                                           uint64_t *global_counts, void *stream);

/* Batched counting of many graphs in one call.  The graphs are given as one
 * CSR over all their nodes (a disjoint union): graph g owns the nodes
 * [graph_node_ptr[g], graph_node_ptr[g+1]) and no edge joins two graphs;
 * its node types lie in [0, graph_L[g]), 1 <= graph_L[g] <= L_max.  Graphlets
 * are connected, so every edge's counts are those of its own graph.
 *   graph_node_ptr    device int64 [G+1], graph_node_ptr[0] = 0,
 *                     graph_node_ptr[G] = n, non-decreasing.
 *   graph_L           device int32 [G].
 *   graph_global_off  device int64 [G+1]: graph g's global vector occupies
 *                     graph_globals[off[g] .. off[g+1]), which must be
 *                     tg_global_width(graph_L[g]) entries (its own layout);
 *                     off[0] = 0, off[G] = globals_len.
 *   graph_globals     device uint64 [globals_len]: per-graph global counts.
 *   per_edge          NULL, or device uint64 [nnz/2][tg_row_width(L_max)]
 *                     rows of the union's edges in canonical order (the
 *                     edges of graph g are contiguous), laid out for L_max.
 *   workspace         at least tg_batch_workspace_bytes(n, nnz, G, L_max),
 *                     256-byte aligned.
 * Validation, streams and errors as for tg_count_typed_graphlets; an
 * inconsistent descriptor or a cross-graph edge gives TG_E_BATCH. */
size_t tg_batch_workspace_bytes(int64_t n, int64_t nnz, int64_t G, int32_t L_max);
tg_status tg_count_batch(const int64_t *row_ptr, const int32_t *col, const uint8_t *types,
                         int64_t n, int64_t nnz, const int64_t *graph_node_ptr,
                         const int32_t *graph_L, int64_t G, int32_t L_max,
                         const int64_t *graph_global_off, int64_t globals_len,
                         uint64_t *per_edge, uint64_t *graph_globals, void *workspace,
                         size_t ws_bytes, void *stream);

/* tg_count_batch without any host synchronisation, so that a caller can
 * record it into a HIP graph (stream capture) and replay it: a batch of many
 * small graphs as one graph launch (the task-parallel scheme of Sec. 4.7
 * scheduled by the device's own work queues).  Arguments as for
 * tg_count_batch, plus:
 *   max_graph_nodes   1 <= max_graph_nodes <= n: an upper bound on every
 *                     graph's node count, given by the caller (it sizes the
 *                     kernels' word widths and sort keys without a read-back);
 *                     a graph above it gives TG_E_BATCH.
 *   status_out        device int32: receives the call's tg_status on the
 *                     stream, after the counts.  The outputs are valid only
 *                     if it reads TG_OK once the stream has reached that
 *                     point.
 * The function returns TG_OK once every kernel is enqueued (host-side
 * argument errors are returned directly, before any device work); device-side
 * input errors (not simple, type range, batch descriptor) go to *status_out
 * only, and every kernel after a failed check does nothing.  It records no
 * memory-set operation, no allocation and no host copy, and it enqueues the
 * same kernels with the same arguments for the same inputs, so a recorded
 * graph can be replayed as long as the inputs, outputs and workspace stay at
 * the same addresses.  Work statistics (tg_last_stats) and phase timing are
 * not collected. */
tg_status tg_count_batch_async(const int64_t *row_ptr, const int32_t *col, const uint8_t *types,
                               int64_t n, int64_t nnz, const int64_t *graph_node_ptr,
                               const int32_t *graph_L, int64_t G, int32_t L_max,
                               int64_t max_graph_nodes, const int64_t *graph_global_off,
                               int64_t globals_len, uint64_t *per_edge, uint64_t *graph_globals,
                               void *workspace, size_t ws_bytes, int32_t *status_out,
                               void *stream);

/* Serving with continuous batching.  A server counts a stream of requests,
 * each one typed graph (the local counts of Problem 1 reduced to its global
 * counts, Problem 2), with the global vector of each request left in device
 * memory until the caller releases it.  All device memory is the caller's
 * `arena` (256-byte aligned, arena_bytes): `workers` regions of
 * worker_bytes each (one batch's union CSR, descriptor, outputs and
 * workspace), the rest a pool from which each admitted request takes one
 * block (its CSR, types and global vector) until it is released.
 *   Admission: requests are admitted in arrival order when their block fits
 *     the pool (by HBM footprint); a request waits while it does not.
 *   Batching: each worker (a host thread with its own HIP stream) takes the
 *     admitted requests not yet started as one batched call (up to its region
 *     and max_batch_edges edges), so requests that arrive while others run
 *     join the next batch and workers overlap on the device; a request of at
 *     least single_edges edges runs alone as a single-graph call.  A failing
 *     batch is re-run request by request: only the offending request fails.
 *   Knobs: the workers use the scheduling knobs of the creating thread
 *     (tg_set_tuning), with the heavy-map and heavy-list budgets cut to a
 *     quarter and an eighth of worker_bytes.
 * Results are exact and independent of the batch a request lands in. */
typedef struct tg_server tg_server;

typedef enum { TG_MEM_HOST = 0, TG_MEM_DEVICE = 1 } tg_mem;

/* One request's graph: CSR and types as for tg_count_typed_graphlets, in
 * host memory (copied at submission; the caller may free it on return) or
 * in device memory (read when the request runs: it must stay valid until the
 * request is done). */
typedef struct {
    const int64_t *row_ptr;
    const int32_t *col;
    const uint8_t *types;
    int64_t n, nnz;
    int32_t L;
    int32_t mem;            /* tg_mem */
} tg_graph_desc;

typedef struct {
    int32_t state;          /* 0 waiting, 1 admitted, 2 running, 3 done */
    int32_t status;         /* tg_status once done, else -1 */
    const uint64_t *global_counts;  /* device, tg_global_width(L) entries, once
                                       done with TG_OK, until released */
    double t_submit, t_admit, t_start, t_done;  /* seconds since creation, -1 if not yet */
    int64_t batch;          /* batch that ran it (-1 before) */
} tg_request_info;

/* Starts the workers.  TG_E_INVALID_ARG: null or unaligned arena, workers
 * outside 1..64, worker_bytes < 4096, single_edges or max_batch_edges < 1;
 * TG_E_OOM: the worker regions leave no pool; TG_E_DEVICE: no current
 * device. */
tg_status tg_server_create(void *arena, size_t arena_bytes, int32_t workers, size_t worker_bytes,
                           int64_t single_edges, int64_t max_batch_edges, tg_server **out);
/* Queues a request and returns its ticket; TG_E_OOM if its block is larger
 * than the whole pool (it could never be admitted); a request whose
 * workspace cannot fit a worker's region finishes with TG_E_OOM. */
tg_status tg_server_submit(tg_server *s, const tg_graph_desc *g, int64_t *ticket);
/* State, status, result pointer and timestamps of a ticket (non-blocking). */
tg_status tg_server_poll(tg_server *s, int64_t ticket, tg_request_info *info);
/* Blocks until the request is done or timeout_s seconds have passed
 * (TG_E_TIMEOUT). */
tg_status tg_server_wait(tg_server *s, int64_t ticket, double timeout_s);
/* Hands out up to max_tickets tickets of requests that finished since the
 * previous call (each ticket once, in completion order), waiting up to
 * timeout_s seconds when there is none; returns how many were written. */
int32_t tg_server_take_done(tg_server *s, int64_t *tickets, int32_t max_tickets,
                            double timeout_s);
/* Frees a finished request's block (its CSR and result); the ticket is then
 * invalid.  TG_E_INVALID_ARG for an unknown, released or unfinished ticket. */
tg_status tg_server_release(tg_server *s, int64_t ticket);
/* Counters: [0] submitted, [1] finished, [2] rejected (TG_E_OOM), [3]
 * batches, [4] single-graph calls, [5] pool bytes in use, [6] peak pool
 * bytes, [7] pool size, [8] microseconds workers spent running batches (sum
 * over workers), [9] waiting, [10] admitted not started, [11] first device
 * error (tg_status) of a worker.  Returns the number written. */
#define TG_SERVER_NUM_STATS 12
int32_t tg_server_stats(tg_server *s, int64_t *stats, int32_t max_stats);
/* Finishes every submitted request (results not yet released become
 * invalid and their memory serves the remaining requests), stops the
 * workers and frees the server; returns the first device error of a
 * worker, or TG_OK. */
tg_status tg_server_destroy(tg_server *s);

/* The canonical edge list (the edge of each per-edge row): edge_uv (device
 * int64 [nnz/2][2]) receives (u, v), u < v, in lexicographic order, the
 * order of the rows of tg_count_typed_graphlets (the unique edge ids of the
 * parallel scheme, Sec. 4.7).  For a graph that call accepts (sorted rows);
 * TG_E_NOT_SIMPLE if the entries above the diagonal are not half of nnz
 * (nothing is written then).  Workspace: tg_edge_list_workspace_bytes(n)
 * bytes, 256-byte aligned.  Returns when the list is complete on `stream`. */
size_t tg_edge_list_workspace_bytes(int64_t n);
tg_status tg_edge_list(const int64_t *row_ptr, const int32_t *col, int64_t n, int64_t nnz,
                       int64_t *edge_uv, void *workspace, size_t ws_bytes, void *stream);

/* Directed typed graphlets of 2 and 3 nodes (Sec. 4.8: every typed
 * neighbourhood, and with it T_ij, S_i and S_j of Alg. 1, splits into out-
 * and in-neighbours; nodes joined both ways form a third case).
 * Input: the underlying undirected graph as for tg_count_typed_graphlets
 * (row_ptr, col, types, n, nnz, L; an edge wherever at least one arc is)
 * and dir (device uint8 [nnz]): for CSR slot s of row u (u -> col[s]), bit
 * 0 is the arc u -> col[s] and bit 1 the arc col[s] -> u; every slot has
 * at least one bit and its reverse slot the mirrored bits
 * (TG_E_NOT_SIMPLE otherwise, as for an unsorted or asymmetric CSR).
 * Per-edge rows (device uint64 [nnz/2][tg_directed_row_width(L) = 15L], or
 * NULL), edges in canonical order (i < j), with a, b in {0: out, the
 * endpoint -> k; 1: in, k -> the endpoint; 2: both}:
 *   TRI[t][a][b]  at t*9 + a*3 + b   k adjacent to both i and j, of type t,
 *                                    direction a at i and b at j
 *   PATH_I[t][a]  at 9L + t*3 + a    k adjacent to i only (k != j)
 *   PATH_J[t][b]  at 12L + t*3 + b   k adjacent to j only (k != i)
 * Global counts (device uint64 [tg_directed_global_width(L) = 4L^2 +
 * 64L^3], or NULL): instances per directed typed graphlet, i.e. per class
 * of typed digraphs under type-preserving isomorphism, each class at its
 * canonical key: over every numbering of its nodes, the smallest tuple
 * (types..., pair codes...), the code of nodes x < y being 0 (no arc), 1
 * (x -> y), 2 (y -> x) or 3 (both).  2-node classes at (t0*L + t1)*4 +
 * c01; 3-node classes (3-paths and triangles) at 4L^2 + ((t0*L + t1)*L +
 * t2)*64 + c01*16 + c02*4 + c12.  Entries that are not canonical keys are
 * 0.  Workspace: tg_directed_workspace_bytes(n, nnz, L) bytes, device,
 * 256-byte aligned.  Errors as for tg_count_typed_graphlets; n >= 2^31 or
 * nnz >= 2^33 gives TG_E_TOO_LARGE.  Returns when the results are complete
 * on `stream`. */
int32_t tg_directed_row_width(int32_t L);
int64_t tg_directed_global_width(int32_t L);
size_t tg_directed_workspace_bytes(int64_t n, int64_t nnz, int32_t L);
tg_status tg_count_directed(const int64_t *row_ptr, const int32_t *col, const uint8_t *dir,
                            const uint8_t *types, int64_t n, int64_t nnz, int32_t L,
                            uint64_t *per_edge, uint64_t *global_counts, void *workspace,
                            size_t ws_bytes, void *stream);

/* Typed-graphlet spectral embeddings (Alg. 5), in two calls.
 *
 * tg_graphlet_weights: W_e, the number of instances of one typed graphlet
 * that contain edge e, for every edge, read off the per-edge rows: the
 * graphlet's orbits (Sec. 4.4: h1 path3; h2 tri; h3 g3+g4; h4 g5; h5 g6;
 * h6 g7+g8+g9; h7 g10+g11; h8 g12) at the type (pair) that completes the
 * edge's endpoint types to the graphlet's type multiset; 0 where the
 * endpoint types are not part of it (h0, the edge itself: 1 or 0).
 *   per_edge      device uint64 [m][tg_row_width(L)] (tg_count_typed_graphlets)
 *   edge_uv       device int64 [m][2] (tg_edge_list): the edge of each row
 *   types         device uint8 [n]
 *   graphlet      0..8 (h0..h8); types_sorted (host int32 [4]) its sorted
 *                 type multiset, 2, 3 or 4 entries as the graphlet has nodes
 *   weights       device uint64 [m], written
 * TG_E_L_RANGE, TG_E_INVALID_ARG (m < 0, graphlet out of range, missing
 * pointers), TG_E_TYPE_RANGE (multiset entries unsorted or outside [0, L)),
 * TG_E_DEVICE.  Returns when the weights are complete on `stream`.
 *
 * tg_graphlet_embedding: Alg. 5 on every connected component of the
 * typed-graphlet graph G^H (the edges with W > 0), as Sec. 8.8 prescribes
 * for graphs with several components.  For a component C of s nodes, with
 * D_ii = sum_j W_ij the typed-graphlet degree, its nodes' rows of Z are the
 * eigenvectors of the min(dim, s) smallest eigenvalues of C's normalised
 * Laplacian I - D^{-1/2} W D^{-1/2}, each row scaled to unit length, zero
 * past column min(dim, s).  Nodes with D_ii = 0 are in no instance and no
 * component: zero rows.  Eigenvectors of a repeated eigenvalue are any
 * orthonormal basis of its eigenspace; signs are arbitrary.
 *   row_ptr, col  the graph (device CSR as for tg_count_typed_graphlets:
 *                 sorted rows, symmetric, no self-loops; TG_E_NOT_SIMPLE
 *                 otherwise)
 *   weights       device uint64 [nnz/2], per canonical edge (the order of
 *                 tg_edge_list)
 *   dim           1..256
 *   opts          NULL for the defaults, else read (see tg_embed_opts)
 *   Z             device float64 [n][dim], written
 *   eigenvalues   device float64 [n][dim] or NULL: row r holds, ascending,
 *                 the min(dim, s) eigenvalues of the component whose
 *                 smallest node id is r; every other entry is 0
 *   component     device int32 [n] or NULL: the smallest node id of each
 *                 node's component, -1 for nodes in none
 *   iterations    host int32 or NULL: the most filter iterations any one
 *                 component took (0 when every component was solved densely)
 *   workspace     tg_embedding_workspace_bytes(n, nnz, dim) bytes, device,
 *                 256-byte aligned, caller-owned
 * Method: components by hook-and-compress; those of at most 64 nodes by a
 * dense Jacobi eigensolver, one workgroup each; larger ones by
 * Chebyshev-filtered subspace iteration on (S + I) / 2, S = D^{-1/2} W
 * D^{-1/2}, with a block of p = dim + max(8, dim / 4) vectors (at most 256
 * and at most s), in float64, until every wanted Ritz pair has residual
 * norm ||M x - theta x|| <= tol.  TG_E_NO_CONVERGENCE when some component
 * reached max_iter (its rows then hold its last Ritz vectors).
 * Deterministic: the same inputs and seed give the same bits.  Returns when
 * the results are complete on `stream` (the call synchronises the stream
 * several times). */
typedef struct tg_embed_opts {
    int32_t max_iter;   /* iteration limit (<= 0: 500) */
    int32_t degree;     /* Chebyshev filter degree (<= 0: 10) */
    double tol;         /* residual tolerance (<= 0: 1e-10) */
    uint64_t seed;      /* seed of the random start block */
    int32_t raw;        /* nonzero: Z receives the eigenvectors themselves
                           (orthonormal columns), rows not rescaled */
    int32_t reserved;   /* set to 0 */
} tg_embed_opts;
tg_status tg_graphlet_weights(const uint64_t *per_edge, int64_t m, int32_t L,
                              const int64_t *edge_uv, const uint8_t *types, int32_t graphlet,
                              const int32_t types_sorted[4], uint64_t *weights, void *stream);
size_t tg_embedding_workspace_bytes(int64_t n, int64_t nnz, int32_t dim);
tg_status tg_graphlet_embedding(const int64_t *row_ptr, const int32_t *col, int64_t n, int64_t nnz,
                                const uint64_t *weights, int32_t dim, const tg_embed_opts *opts,
                                double *Z, double *eigenvalues, int32_t *component,
                                int32_t *iterations, void *workspace, size_t ws_bytes,
                                void *stream);

/* Sparse per-edge output (Sec. 4.6: an edge keeps only its nonzero typed
 * graphlet counts, with a lookup table from key to description, here
 * tg_key_describe).  Built from a dense per-edge table `rows` (device uint64
 * [m][tg_row_width(L)], as written by tg_count_typed_graphlets) in two calls:
 *   tg_sparse_offsets   writes edge_off (device int64 [m+1]): edge e's pairs
 *                       are entries [edge_off[e], edge_off[e+1]) and
 *                       edge_off[m] is their total; needs a workspace of
 *                       tg_sparse_workspace_bytes(m) bytes.
 *   tg_sparse_fill      writes keys (device uint16) and counts (device
 *                       uint64), each of edge_off[m] entries: the column id
 *                       and the count of every nonzero entry, edges in
 *                       canonical order, columns ascending within an edge.
 * The caller owns every buffer and sizes keys/counts from edge_off[m].
 * Both calls return when their results are complete on `stream`.  Errors:
 * TG_E_L_RANGE, TG_E_INVALID_ARG (m < 0, missing pointers), TG_E_WORKSPACE
 * (workspace too small), TG_E_DEVICE. */
size_t tg_sparse_workspace_bytes(int64_t m);
tg_status tg_sparse_offsets(const uint64_t *rows, int64_t m, int32_t L, int64_t *edge_off,
                            void *workspace, size_t ws_bytes, void *stream);
tg_status tg_sparse_fill(const uint64_t *rows, int64_t m, int32_t L, const int64_t *edge_off,
                         uint16_t *keys, uint64_t *counts, void *stream);

/* Position-aware typed graphlets (Sec. 5; Def. of a position-aware typed
 * graphlet instance: node types must coincide via the isomorphism).  The
 * per-edge counts keep the role each of the two other nodes k, r plays
 * relative to the edge (i, j), oriented with i the edge's first endpoint in
 * canonical order (i < j in the input's ids); the global counts are kept per
 * class of typed graphlets under type-preserving isomorphism.  Folding the
 * roles of each block gives the typed row of tg_count_typed_graphlets.
 *
 * Per-edge row (tg_pa_row_width(L) = 3L + 9 L^2 + 6 P columns), blocks in
 * this order; an ordered block holds (x, y) at x*L + y, an unordered block
 * {t <= u} at the lexicographic pair index, a 3-node block t at t.  With
 * S_i the neighbours of i that are neither j nor adjacent to j, S_j
 * likewise, T the common neighbours and I the nodes adjacent to neither:
 *   0 TRI [t]     |T^t|              1 PATH_I [t]  |S_i^t| (3-path k-i-j)
 *   2 PATH_J [t]  |S_j^t| (i-j-k)
 *   3 G3I (x,y)   k in S_i^x, r in I^y, k~r: 4-path r-k-i-j
 *   4 G3J (x,y)   k in S_j^x, r in I^y, k~r: 4-path i-j-k-r
 *   5 G4 (x,y)    k in S_i^x, r in S_j^y, not k~r: 4-path k-i-j-r
 *   6 G5I {t,u}   k, r in S_i, not k~r: 4-star centred at i
 *   7 G5J {t,u}   the same at j
 *   8 G6 (x,y)    k in S_i^x, r in S_j^y, k~r: 4-cycle i-j-r-k
 *   9 G7I {t,u}   k, r in S_i, k~r: triangle i-k-r with tail j
 *  10 G7J {t,u}   the same at j
 *  11 G8 (x,y)    k in T^x, r in I^y, k~r: triangle i-j-k, tail r at k
 *  12 G9I (x,y)   k in T^x, r in S_i^y, not k~r: tail r at i
 *  13 G9J (x,y)   k in T^x, r in S_j^y, not k~r: tail r at j
 *  14 G10I (x,y)  k in T^x, r in S_i^y, k~r: chordal cycle, chord i-k
 *  15 G10J (x,y)  k in T^x, r in S_j^y, k~r: chordal cycle, chord j-k
 *  16 G11 {t,u}   k, r in T, not k~r: chordal cycle, chord i-j
 *  17 G12 {t,u}   k, r in T, k~r: 4-clique
 * Global layout (tg_pa_global_width(L) classes): graphlets h0..h8 in order,
 * each class described by the types at the positions of a drawing: h0 edge
 * (0,1); h1 3-path 1-0-2 (0 the centre); h2 triangle; h3 4-path 0-1-2-3;
 * h4 4-star with centre 0; h5 4-cycle 0-1-2-3-0; h6 tailed triangle with
 * triangle 0,1,2 and tail 2-3; h7 chordal cycle 0-1-2-3-0 with chord 0-2;
 * h8 4-clique.  With rk2(x, y) = min + max(max+1)/2 (co-lexicographic rank
 * of an unordered pair over any alphabet), rk3 / rk4 the co-lexicographic
 * ranks of sorted multisets and P = L(L+1)/2, the index inside each block:
 *   h0 rk2(t0,t1); h1 t0*P + rk2(t1,t2); h2 rk3; h3 rk2(t0*L+t1, t3*L+t2);
 *   h4 t0*C(L+2,3) + rk3(t1,t2,t3); h5 rk2(rk2(t0,t2), rk2(t1,t3));
 *   h6 (t3*L + t2)*P + rk2(t0,t1); h7 rk2(t0,t2)*P + rk2(t1,t3); h8 rk4.
 * Each entry counts instances (per-edge sums divided by the graphlet's
 * edge count). */
int32_t tg_pa_row_width(int32_t L);
int64_t tg_pa_global_width(int32_t L);

/* Position-aware counts of one graph, arguments, workspace
 * (tg_workspace_bytes), streams and errors as for tg_count_typed_graphlets;
 * per_edge is device uint64 [nnz/2][tg_pa_row_width(L)] or NULL,
 * global_counts device uint64 [tg_pa_global_width(L)] or NULL.  The
 * position-aware derivation runs as its own pass over per-edge inputs
 * held in the workspace: a graph whose (nnz/2) * 32 L^2 bytes exceed 16 GiB
 * gives TG_E_TOO_LARGE before any device work. */
tg_status tg_count_position_aware(const int64_t *row_ptr, const int32_t *col,
                                  const uint8_t *types, int64_t n, int64_t nnz, int32_t L,
                                  uint64_t *per_edge, uint64_t *global_counts, void *workspace,
                                  size_t ws_bytes, void *stream);

/* Meaning of position-aware column `col`: *block 0..17 as listed above,
 * *t, *t2 the role types (x, y), the unordered pair t <= t2, or the type
 * and -1 for the 3-node blocks. */
tg_status tg_pa_key_describe(int32_t L, int32_t col, int32_t *block, int32_t *t, int32_t *t2);

/* Meaning of position-aware global entry `idx`: *graphlet 0..8, *k its node
 * count and types_by_position[0..k-1] the types at the drawing's positions
 * of one member of the class (the rest set to -1). */
tg_status tg_pa_global_key_describe(int32_t L, int64_t idx, int32_t *graphlet,
                                    int32_t types_by_position[4], int32_t *k);

/* Meaning of per-edge column `col` for L types: orbit 1 = tri, 2 = path3
 * (with *t the third node's type and *t2 = -1), else the orbit number 3..12
 * of Table 3 with the unordered type pair (*t <= *t2). */
tg_status tg_key_describe(int32_t L, int32_t col, int32_t *orbit, int32_t *t, int32_t *t2);

/* Meaning of global entry `idx`: *graphlet in 0..8 (h0..h8), *k its node
 * count (2, 3 or 4) and types_sorted[0..k-1] the sorted type multiset. */
tg_status tg_global_key_describe(int32_t L, int32_t idx, int32_t *graphlet,
                                 int32_t types_sorted[4], int32_t *k);

/* Per-kernel-class device time of the most recent tg_count_directed or
 * tg_graphlet_embedding call on this host thread, recorded while timing is
 * on (tg_set_timing): for each class, its name (owned by the library),
 * the summed milliseconds of its launches (HIP events on the caller's
 * stream), their number, and the class's algorithmic units over those
 * launches -- bytes for the bandwidth-bound classes, flops for the
 * matrix-core classes, 0 where the library does not price the class
 * (embedding: "spmm" bytes = nonzeros x (12 + 8p) + rows x 8p x (2 or 3),
 * "gram" flops = s p (p + 1) (a symmetric product), "apply" flops = 2 s p^2,
 * "chol", "jacobi" 0; directed:
 * "dir_check", "dir_rows", "dir_global" 0, priced by the caller).  Returns
 * the number of classes written (at most max_classes); any output may be
 * NULL. */
int32_t tg_kernel_sums(const char **names, double *ms, double *units, int64_t *calls,
                       int32_t max_classes);

/* Text naming the HIP call and error behind the most recent TG_E_DEVICE
 * returned by a counting call on this host thread ("" if that call had no
 * HIP failure).  The string is owned by the library and valid until the
 * next counting call on the thread. */
const char *tg_last_error(void);

/* Scheduling knobs (work splits, workgroup counts, degree buckets), kept
 * per host thread and applied to later calls on that thread.  They change how work is scheduled, never
 * the counts.
 *   TG_TUNE_TASK_WEDGES  (default 262144, >= 1): a heavy wedge group is split
 *       into target-id ranges of about this many wedges each (at most 64).
 *   TG_TUNE_CLEAR_BYTES  (default 64, >= 0): a task clears its map range by
 *       streaming zeros when the range costs at most this many bytes per
 *       wedge of the task, else by a walk over its wedges; 0 never streams.
 *   TG_TUNE_CYCLE_SLOTS  (default 2048, 1..65536): most workgroups of the heavy
 *       4-cycle kernels; each owns a dense map of n*L*4 bytes of workspace.
 *   TG_TUNE_MAP_BYTES    (default 32 GiB, >= 1): workspace bytes for those
 *       maps; the slot count is cut to fit (at least one slot).
 *   TG_TUNE_EDGE_SLOTS   (default 1280, 1..65536): most workgroups of the
 *       heavy-edge kernel; each owns a list of n*4 bytes of workspace.
 *   TG_TUNE_TBUF_BYTES   (default 8 GiB, >= 1): workspace bytes for those
 *       lists; the slot count is cut to fit (at least one slot).
 *   TG_TUNE_RANGE_BYTES  (default 0, >= 0): a heavy group with at least
 *       one wedge per target id is also split so that one task's map entries
 *       take at most this many bytes; 0 turns this off.
 *   TG_TUNE_DERIVE_EDGES (default 0 = automatic, 0..4): edges of the light
 *       kernel whose per-type-pair derivation runs together in one wave.
 *   TG_TUNE_LIGHT_WEDGES (default 512, 1..512): degree bucket of the 4-cycle
 *       groups: a group of at most this many wedges is counted by one wave
 *       with a map in LDS, a larger one by the heavy (task) kernel.
 *   TG_TUNE_EDGE_DEG     (default 1024, 1..1024): degree bucket of the edges:
 *       an edge whose smaller endpoint degree is at most this is counted by
 *       one wave with its triangle set in LDS, else by a 256-thread
 *       workgroup of the heavy-edge kernel.
 *   TG_TUNE_SH_MAX       (default 2048, 0..2048): most super-hubs, the
 *       highest-ranked nodes of degree >= TG_TUNE_SH_DEG that get a bitmap
 *       over all nodes (constant-time membership and slot lookups); the
 *       workspace budget for the bitmaps (512 MiB) may cut it further.  A
 *       node of that degree without a bitmap is probed by binary search.
 *   TG_TUNE_SH_DEG       (default 1024, 32..2^31-1): smallest degree of a
 *       super-hub.
 *   TG_TUNE_BLK_WEDGES   (default 2^16, >= 1): smallest heavy pass-A
 *       4-cycle group (grouped by top vertex) that may be counted by the
 *       blocked path (single graphs with every
 *       degree below 2^16, L <= 16 and at most 2^25 nodes): its wedges are
 *       written once as 2-byte records grouped by target block, counted per
 *       block in LDS into one map per group, then walked in tasks that read
 *       that map.  The largest such groups are taken while their maps fit
 *       the cycle map region (at most 4096 groups per pass) and their wedges
 *       the records; the rest go to the task kernel.
 *   TG_TUNE_BLK_TASK     (default 65536, 1024..65536): wedges per walk task
 *       of the blocked path.
 *   TG_TUNE_BLK_WEDGES_B (default 2^31 = off, >= 1): the same bound for
 *       pass-B groups (grouped by the vertex opposite the top), which are
 *       many and small on power-law graphs.
 *   TG_TUNE_HUB_LDS      (default 20480, 0..65536): LDS bytes of the pass-B
 *       task kernel for 16-bit counts of targets among the top-ranked ids
 *       (single graphs with every degree below 2^16; pass-B targets lie
 *       above both ends of their wedge, so they concentrate there); 0 keeps
 *       every target in the workgroup's map.
 *   TG_TUNE_BLK_BYTES    (default 4 GiB, 0..2^33): workspace bytes for the
 *       blocked path's records (two bytes per wedge of the blocked groups of
 *       one pass); 0 turns the blocked path off.
 * CYCLE_SLOTS, MAP_BYTES, EDGE_SLOTS, TBUF_BYTES, SH_MAX and BLK_BYTES change
 * tg_workspace_bytes and tg_batch_workspace_bytes, so they must be set
 * before the workspace is sized.
 * tg_set_tuning returns TG_E_INVALID_ARG for an unknown knob or a value out
 * of range; tg_get_tuning returns the current value (-1 if unknown). */
typedef enum {
    TG_TUNE_TASK_WEDGES = 0,
    TG_TUNE_CLEAR_BYTES = 1,
    TG_TUNE_CYCLE_SLOTS = 2,
    TG_TUNE_MAP_BYTES = 3,
    TG_TUNE_EDGE_SLOTS = 4,
    TG_TUNE_TBUF_BYTES = 5,
    TG_TUNE_RANGE_BYTES = 6,
    TG_TUNE_DERIVE_EDGES = 7,
    TG_TUNE_LIGHT_WEDGES = 8,
    TG_TUNE_EDGE_DEG = 9,
    TG_TUNE_SH_MAX = 10,
    TG_TUNE_SH_DEG = 11,
    TG_TUNE_BLK_WEDGES = 12,
    TG_TUNE_BLK_BYTES = 13,
    TG_TUNE_BLK_TASK = 14,
    TG_TUNE_BLK_WEDGES_B = 15,
    TG_TUNE_HUB_LDS = 16
} tg_tune;
#define TG_NUM_TUNE 17
tg_status tg_set_tuning(int32_t knob, int64_t value);
int64_t tg_get_tuning(int32_t knob);

/* Timing of the phases of the most recent tg_count_typed_graphlets call on
 * this host thread, measured with HIP events on the caller's stream when
 * timing is enabled.  tg_set_timing(1) turns it on (off by default).
 * tg_phase_times writes up to max_phases durations in milliseconds into ms
 * and their names into names (static strings); returns the phase count.
 * It synchronises on the recorded events. */
void tg_set_timing(int32_t enable);
int32_t tg_phase_times(float *ms, const char **names, int32_t max_phases);

/* Work statistics of the most recent call on this host thread (for
 * bandwidth accounting), up to max_stats of: [0] wedges of 4-cycle pass A,
 * [1] groups on the light cycle path (both passes), [2] groups on the heavy
 * cycle path, [3] edges on the heavy clique path, [4] wedges of pass B,
 * [5] pass-A wedges in heavy groups, [6] pass-B wedges in heavy groups,
 * [7] sum over edges of |T_ij| (three times the triangle count),
 * [8] nodes of at least the super-hub degree, [9] super-hubs given a bitmap
 * (the rest of [8] is probed by binary search), [10] hub-core size,
 * [11] groups on the blocked cycle path (both passes), [12] pass-A wedges
 * in blocked groups, [13] pass-B wedges in blocked groups.
 * Returns the number written (at most TG_NUM_STATS). */
#define TG_NUM_STATS 14
int32_t tg_last_stats(int64_t *stats, int32_t max_stats);

#ifdef __cplusplus
}
#endif

#endif /* TG_H */
