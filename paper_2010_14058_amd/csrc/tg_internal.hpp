// Internal declarations shared by the library's HIP sources.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/tg.h"

namespace tg {

constexpr int WAVE = 64;

// Status bits raised on the device by the input checks and the counters.
enum : uint32_t {
    ST_COL_RANGE = 1u << 0,
    ST_UNSORTED = 1u << 1,
    ST_SELF_LOOP = 1u << 2,
    ST_TYPE_RANGE = 1u << 3,
    ST_ASYMMETRIC = 1u << 4,
    ST_INTERNAL = 1u << 5,
    ST_NOT_DIVISIBLE = 1u << 6,
    ST_BATCH = 1u << 7,       // inconsistent batch descriptor
    ST_CROSS_GRAPH = 1u << 8, // an edge joins two graphs of a batch
    ST_EDGE_COUNT = 1u << 9,  // entries above the diagonal are not half the adjacency
};

// Bits that mean the input is unusable: every kernel after the input checks
// returns at once when one is set (so a call that never reads the status
// back on the host stays in bounds).
constexpr uint32_t ST_INPUT = ST_COL_RANGE | ST_UNSORTED | ST_SELF_LOOP | ST_TYPE_RANGE |
                              ST_ASYMMETRIC | ST_BATCH | ST_CROSS_GRAPH | ST_EDGE_COUNT;

// Tunables of the cycle and clique passes.
constexpr int64_t LIGHT_MAXW = 512;   // a group is light if it has at most this many wedges
// Threads of a heavy 4-cycle workgroup, per pass: pass A's maps are spread
// over all ids, so fewer, larger workgroups (fewer maps sharing an XCD's L2)
// pay; pass B's targets are compact.  A workgroup stages up to half as many
// items per round as it has threads.
constexpr int HEAVY_THREADS_A = 1024;
constexpr int HEAVY_THREADS_B = 256;
constexpr int64_t TASK_WEDGES = 1 << 18;  // default wedges per heavy task (target range)
constexpr int TASK_MAX_PARTS = 64;        // most target ranges per heavy group
constexpr int64_t TASK_EXTRA = 1 << 16;   // task slots beyond one per node, shared by both passes
constexpr int SEQ_CLEAR_BYTES = 64;       // default bytes per wedge below which a range is cleared by streaming
constexpr int64_t TASK_RANGE_BYTES = 0;  // default map-byte bound per task of a dense heavy group (0: off)
constexpr int TCAP = 1024;            // triangle set kept in LDS by the light edge kernel
constexpr int EDGE_THREADS_HEAVY = 256;
constexpr int64_t BATCH_EDGE_CHUNK = 256;  // consecutive edges per work item in batches
constexpr int HUB_DMIN = 32;          // smallest degree of a hub-core node
constexpr int HUB_MAX = 8192;         // largest hub core (bit-matrix HUB_MAX^2 bits)
constexpr int SH_DMIN = 1024;         // default smallest degree of a super-hub (full-row bitmap)
constexpr int SH_MAX = 2048;          // most super-hubs (the default cap)
constexpr size_t SH_BUDGET = size_t(512) << 20;  // bytes of super-hub bitmaps and prefixes
// Blocked heavy 4-cycle groups: the wedges of a group are partitioned by
// target block (BLK_IDS ids) into 16-bit records (offset in the block, centre
// type in the top 4 bits, so L <= 16), counted block by block in LDS into one
// map per group, then walked again in tasks of BLK_TASK wedges that read it.
constexpr int BLK_SHIFT = 12;
constexpr int BLK_IDS = 1 << BLK_SHIFT;
constexpr uint32_t BLK_TASK = 1u << 16;      // default and largest wedges per walk task
                                             // (32-bit tallies stay exact)
constexpr int BLK_MAX_GROUPS = 4096;         // blocked groups per pass (each owns one map)
constexpr int BLK_BINS = 128;                // group-size histogram: 4 bins per octave
constexpr int64_t BLK_MAX_NODES = int64_t(BLK_IDS) * 8192;  // at most 8192 blocks per group
constexpr int64_t BLK_MIN_WEDGES = 1 << 16;  // default smallest blocked group (pass A)
// pass B's groups (many, and small) run faster on the task kernel: off by
// default (no group reaches 2^31 wedges on this path)
constexpr int64_t BLK_MIN_WEDGES_B = int64_t(1) << 31;
constexpr int64_t HUB_LDS_BYTES = 20480;   // default LDS for the pass-B kernel's hub targets
constexpr size_t BLK_BUDGET = size_t(4) << 30;  // default bytes of records

// Device-side layout of everything the library keeps in the caller's
// workspace.  All offsets are byte offsets from the workspace base.
struct Layout {
    int64_t n, nnz, m;
    int L;
    int heavy_slots;          // dense cycle maps (one per heavy workgroup)
    int heavy_edge_slots;     // global triangle buffers of the heavy edge kernel
    bool defer;               // derivation in its own pass (off_xyk valid)
    size_t sort_tmp_bytes;
    size_t off_status, off_counters;
    size_t off_deg, off_ucount, off_eoff, off_order, off_newid, off_ntype, off_nrp, off_ndeg;
    size_t off_key_a, off_key_b, off_val_a, off_val_b;
    size_t off_ncol, off_neid, off_ei, off_ej, off_ctype;
    size_t off_tdeg, off_tri, off_tri_slot, off_A, off_D, off_NC;
    size_t off_listA_light, off_listA_heavy, off_listB_light, off_listB_heavy, off_list_edge;
    size_t off_maps, off_tbuf, off_gacc, off_sort_tmp;
    size_t off_hstart, off_HB, off_hpre, off_TM, off_eslot, off_nlow, off_xyk;
    size_t off_node_graph, off_ngraph, off_gedge;   // batched graphs only
    size_t off_SB, off_SP;                          // super-hub bitmaps
    size_t off_pacc;                                // position-aware global accumulators
    // blocked heavy 4-cycle groups (single graphs; blk_groups = 0: none)
    int blk_groups;                                 // most blocked groups per pass
    int blk_nb;                                     // blocks of the widest target range
    int64_t blk_records;                            // record capacity
    int64_t blk_nbk;                                // bucket capacity
    size_t off_blk_list_a, off_blk_list_b, off_blk_meta, off_blk_ipre;
    size_t off_blk_cand_a, off_blk_cand_b, off_blk_flag, off_blk_hist;
    size_t off_blk_bcount, off_blk_bstart, off_blk_pcur, off_blk_rec, off_blk_bgroup, off_blk_mat;
    int64_t blk_mat;                                // histogram matrix capacity (0: none)
    int sh_max;
    int64_t G;
    size_t total;
};

// Counters block (uint64 each) at off_counters.
enum Counter {
    C_A_LIGHT = 0, C_A_HEAVY, C_B_LIGHT, C_B_HEAVY, C_EDGE_HEAVY,
    C_A_NEXT, C_B_NEXT, C_EDGE_NEXT, C_WEDGES_A, C_WEDGES_B,
    C_WEDGES_A_HEAVY, C_WEDGES_B_HEAVY, C_TRI_SUM, C_HUB_CAND, C_SH_CAND,
    C_TASK_EXTRA, C_HEAVY_GROUPS, C_MAX_GSIZE,
    // blocked groups: list lengths and wedges per pass, then the current
    // pass's group count, walk tasks, buckets and queue positions
    C_BLK_A, C_BLK_CAND_A, C_BLK_B, C_BLK_CAND_B, C_BLK_GROUPS, C_BLK_TASKS, C_BLK_BUCKETS,
    C_BLK_NEXT_H, C_BLK_NEXT_P, C_BLK_NEXT_C, C_BLK_A_DONE, C_BLK_B_DONE, C_BLK_STRIDE,
    C_BLK_MAT,                              // 1: this pass's histogram rows are in the matrix
    C_BLK_NEXT_E,                           // eight emit queues, one per XCD
    C_BLK_NEXT_E_END = C_BLK_NEXT_E + 8,
    C_NUM = C_BLK_NEXT_E_END
};

// Workspace budgets of the per-workgroup scratch regions: the heavy 4-cycle
// maps (n L words each), the heavy-edge member lists (n words each), the
// super-hub bitmaps and the per-edge inputs of the separate derivation pass.
struct Budget {
    size_t map_bytes;
    int64_t cycle_slots;
    size_t tbuf_bytes;
    int64_t edge_slots;
    int64_t sh_max;
    size_t sh_bytes;
    size_t xyk_bytes;
    size_t blk_bytes;     // records of the blocked 4-cycle groups (0: no blocked path)
    int64_t blk_task;     // wedges per blocked walk task (sizes the histogram matrix)
};

// The budgets the scheduling knobs of the calling thread give.
Budget budget_from_tuning();

tg_status plan_layout(int64_t n, int64_t nnz, int L, Layout *lay, int64_t G, const Budget &b);
inline tg_status plan_layout(int64_t n, int64_t nnz, int L, Layout *lay, int64_t G = 0) {
    return plan_layout(n, nnz, L, lay, G, budget_from_tuning());
}

// Batch descriptor (device pointers) of tg_count_batch.
struct BatchIn {
    const int64_t *node_ptr;   // [G+1]
    const int32_t *gL;         // [G]
    const int64_t *goff;       // [G+1]
    int64_t G;
    int64_t globals_len;
    int64_t max_nodes;         // declared bound on a graph's node count (checked), or -1
};

// Arguments of the 4-cycle passes.
struct CycleArgs {
    const int64_t *nrp;
    const int32_t *ncol;
    const uint8_t *ntype;
    const uint32_t *neid;
    const uint8_t *ctype;      // type of the neighbour at each adjacency slot
    const int32_t *ei;
    const uint32_t *list;      // light groups
    const uint4 *tasks;        // heavy tasks: group, part, parts, wedges of the group
    const uint32_t *eslot;     // [2e] slot of edge e in the row of its smaller end, [2e+1] larger end
    const uint32_t *nlow;      // neighbours below the node itself, per node
    uint64_t clear_bytes;      // streamed-clear threshold (bytes per wedge)
    uint64_t *counters;
    int count_idx;
    int next_idx;
    int L;
    int64_t n;
    uint64_t *NC;
    int nc_u32;                  // NC stored as uint32 (every degree below 2^16)
    uint32_t *maps;
    int chunk;
    uint32_t *status;
    int light_log2;            // log2 of the light kernel's hash slots (> light bucket)
    int deg_sorted;            // node ids ranked by degree (not the graph-major batch order)
    int64_t max_deg;           // largest degree (or a bound)
    const uint8_t *blk_flag;   // groups counted by the blocked path (skipped by the tasks), or null
    int hub_ids;               // task kernel: targets among the top hub_ids ids counted in LDS (0: none)
};

// Blocked heavy 4-cycle groups of one pass (see BLK_SHIFT).
struct BlkArgs {
    uint2 *list;            // (group, wedges) of the pass's blocked groups
    int c_count;            // counter holding the list length
    int max_groups;
    const uint2 *cand;      // candidate groups (heavy, at least the smallest blocked size)
    int c_cand;             // counter holding the candidate count
    const uint64_t *hist;   // [BLK_BINS][2] candidates and their wedges per size bin
    uint8_t *flag;          // per node: 1 if its group is blocked
    uint64_t max_wedges;    // record capacity
    uint64_t maps_words;    // words of the map region
    uint32_t task;          // wedges per walk task (at most BLK_TASK)
    uint32_t *ioff;         // [max_groups + 1] first item prefix of each group
    uint32_t *tstart;       // [max_groups + 1] first walk task of each group
    uint32_t *boff;         // [max_groups + 1] first bucket of each group
    uint32_t *moff;         // [max_groups + 1] first histogram-matrix entry of each group
    uint32_t *mat;          // per walk task its wedges per block (rows of the group's block count)
    int64_t mat_cap;        // matrix capacity (0: the partition walks its task twice)
    uint32_t *xstart;       // [8][max_groups / 8 + 1] first walk task of group x + 8 i
                            // within the emit queue of XCD x
    uint32_t *ipre;         // per group: exclusive wedge prefix of its items, then the total
    int64_t *bcount;        // [nbk + 1] records per bucket (group, block)
    int64_t *bstart;        // [nbk + 1] exclusive prefix of bcount
    uint32_t *pcur;         // [nbk + 1] records placed per bucket
    uint32_t *bgroup;       // [nbk + 1] group of each bucket
    uint16_t *rec;          // records grouped by bucket
    int nb_max;             // blocks of the widest target range
    int64_t nbk;            // bucket capacity
    int emit_chunk;         // items per staging round of the emit walk
};

// Arguments of the per-edge clique / derivation kernels.
struct EdgeArgs {
    const int64_t *nrp;
    const int32_t *ncol;
    const uint8_t *ntype;
    const uint32_t *neid;
    const int32_t *ei, *ej;
    const uint32_t *tri;
    const uint32_t *tdeg;        // typed degrees per node, rows of tri_pitch(L)
    const uint8_t *ctype;        // type of the neighbour at each adjacency slot
    const uint32_t *tri_slot;    // typed triangle counts per slot, rows of tri_pitch(L)
    const uint64_t *A, *D, *NC;
    int agg_u32;                 // A, D and NC stored as uint32 (every degree below 2^16)
    int64_t m;
    int L;
    uint64_t *rows;      // may be null
    uint64_t *gacc;      // global accumulators
    int gw;
    int hist_in_lds;             // 0: global atomics, 1: uint64 LDS histogram, 2: uint32 LDS histogram
    int tcap;                    // light/heavy edge cut on the smaller degree = LDS list size
    int derive_batch;            // edges whose derivation runs together (LDS slots of 4 L^2 words)
    uint64_t *xyk;               // deferred derivation: Xi, Xj, Y, K per edge ([m][4 L^2]), or null
    int xyk_u32;                 // xyk entries stored as uint32 (every degree below 2^16)
    uint32_t *heavy_list;
    uint64_t *counters;
    uint32_t *tbuf;      // heavy: per-workgroup low-member buffers of n entries
    int64_t n;
    uint32_t *status;
    // hub core: internal ids hub_base..n-1
    int32_t hub_base;
    int Hw;                      // 64-bit words per bit row
    const int64_t *hstart;       // first slot of each row's hub suffix
    const uint32_t *nlow;        // neighbours below the node itself, per node
    const uint64_t *HB;          // [H][Hw] hub adjacency bits
    const uint32_t *hpre;        // [H][Hw] exclusive prefix popcounts
    const uint64_t *TM;          // [Hw][tm_pitch(L)] hubs of types 0..L-2 per word, zero padded
    // super-hubs: internal ids sh_base..n-1 with a bitmap over all nodes
    int32_t sh_base;
    int64_t nw;                  // 64-bit words per super-hub bitmap
    const uint64_t *SB;          // [S][nw]
    const uint32_t *SP;          // [S][nw] exclusive prefix popcounts
    // batched graphs: per-graph global vectors at goff[g], in graph g's own
    // L layout; the kernels compute in the layout of L (= max over graphs)
    int batch;
    const int32_t *ngraph;       // internal node -> graph
    const int64_t *gedge_ptr;    // [G+1] canonical edge range of each graph
    const int32_t *gL;           // [G]
    const int64_t *goff;         // [G+1]
    int64_t G;
};

// Position-aware rows (tg_position.hip): blocks in row order; a block is L
// wide (3-node), L^2 (ordered role pairs) or L(L+1)/2 (unordered pairs).
enum PaBlock {
    PB_TRI, PB_PATH_I, PB_PATH_J, PB_G3I, PB_G3J, PB_G4, PB_G5I, PB_G5J, PB_G6, PB_G7I, PB_G7J,
    PB_G8, PB_G9I, PB_G9J, PB_G10I, PB_G10J, PB_G11, PB_G12, PB_NUM
};

struct PaLayout {
    int start[PB_NUM + 1];   // first column of each block; start[PB_NUM] = row width
    int64_t gstart[10];      // first global class of graphlets h0..h8; gstart[9] = width
};

PaLayout pa_layout(int L);
hipError_t launch_derive_pa(const EdgeArgs &args, const PaLayout &pl, unsigned grid,
                            hipStream_t st);
hipError_t launch_pa_finalize(const uint64_t *acc, const PaLayout &pl, uint64_t *out,
                              uint32_t *status, hipStream_t st);

// Per-class kernel timing of the directed and embedding calls (tg_api.hip),
// active while tg_set_timing is on: ksum_reset at the start of a call,
// ksum_begin / ksum_end around the launches of a class (units: the class's
// algorithmic bytes or flops for those launches), ksum_collect once the
// stream has been synchronised.
void ksum_reset();
void ksum_begin(hipStream_t st);
void ksum_end(const char *cls, double units, hipStream_t st);
void ksum_collect();

// Prefix sums and radix sorts (tg_sort.hip).  `gate` is the status word:
// they do nothing once an input check has failed.
int64_t scan_tiles(int64_t count);
size_t sort_tmp_need(int64_t count);
hipError_t launch_excl_scan(const int64_t *in, int64_t *out, int64_t count, int64_t *tmp,
                            const uint32_t *gate, hipStream_t st);
hipError_t radix_sort(uint64_t *keys, uint64_t *keys_tmp, uint32_t *vals, uint32_t *vals_tmp,
                      int64_t count, int end_bit, void *tmp, const uint32_t *gate,
                      hipStream_t st, uint64_t **out_keys, uint32_t **out_vals);

// Launch wrappers (tg_kernels.hip).
hipError_t launch_fill_u64(uint64_t *p, uint64_t v, int64_t count, hipStream_t st);
hipError_t launch_check_rows(const int64_t *rp, const int32_t *col, const uint8_t *types, int64_t n,
                             int64_t nnz, int L, uint32_t *deg, int64_t *ucount, uint32_t *status,
                             const int32_t *node_graph, const int32_t *gL, hipStream_t st);
hipError_t launch_check_edge_count(const int64_t *eoff, int64_t n, int64_t m, uint32_t *status,
                                   hipStream_t st);
hipError_t launch_status_code(const uint32_t *status, int32_t *out, hipStream_t st);
hipError_t launch_batch_graphs(const int64_t *node_ptr, const int32_t *gL, const int64_t *goff,
                               int64_t G, int64_t n, int L_max, int64_t globals_len,
                               int64_t max_nodes, int32_t *node_graph, uint32_t *status,
                               uint64_t *max_gsize, hipStream_t st);
hipError_t launch_batch_edges(const int64_t *node_ptr, const int64_t *eoff, int64_t G,
                              int64_t *gedge_ptr, const uint32_t *status, hipStream_t st);
hipError_t launch_batch_finalize(uint64_t *globals, const int32_t *gL, const int64_t *goff, int64_t G,
                                 uint32_t *status, hipStream_t st);
hipError_t launch_node_keys(const uint32_t *deg, int64_t n, const int32_t *node_graph, int deg_bits,
                            uint64_t *keys, uint32_t *ids, const uint32_t *status, hipStream_t st);
hipError_t launch_relabel(const uint32_t *sorted_ids, const uint8_t *types, const uint32_t *deg,
                          int64_t n, int32_t *order, int32_t *newid, uint8_t *ntype, int64_t *ndeg,
                          uint64_t *hub_cand, uint32_t sh_deg, const int32_t *node_graph,
                          int32_t *ngraph, const uint32_t *status, hipStream_t st);
hipError_t launch_slot_keys(const int64_t *rp, const int32_t *col, const int64_t *ucount,
                            const int64_t *eoff, const int32_t *newid, int64_t n, int bits,
                            uint64_t *keys, uint32_t *vals, int32_t *ei, int32_t *ej,
                            uint32_t *status, hipStream_t st);
hipError_t launch_finish_csr(const uint64_t *keys, const uint32_t *vals, int64_t nnz, int bits,
                             const uint8_t *ntype, uint32_t *eslot, int32_t *ncol, uint32_t *neid,
                             uint8_t *ctype, const uint32_t *status, hipStream_t st);
hipError_t launch_tdeg(const int64_t *nrp, const int32_t *ncol, const uint8_t *ctype, int64_t n,
                       int L, int32_t hub_base, uint32_t *tdeg, int64_t *hstart, uint32_t *nlow,
                       const uint32_t *status, hipStream_t st);
hipError_t launch_hub_build(const int64_t *nrp, const int32_t *ncol, const int64_t *hstart,
                            const uint8_t *ntype, int64_t n, int H, int Hw, int L, uint64_t *HB,
                            uint32_t *pre, uint64_t *TM, hipStream_t st);
// Row pitch (uint32 words) of per-slot typed triangle counts: L rounded up
// to a multiple of 4, for 16-byte loads.
__host__ __device__ inline int tri_pitch(int L) { return (L + 3) & ~3; }
// Words per hub-core word in the type-mask table: masks of types 0..L-2
// (the last type is what the others leave), padded to an even count.
__host__ __device__ inline int tm_pitch(int L) { return L & ~1; }

hipError_t launch_tri(const int64_t *nrp, const int32_t *ncol, const uint8_t *ctype,
                      const int32_t *ei, const int32_t *ej, const uint32_t *eslot,
                      uint32_t *tri_slot, int64_t m, int L, uint32_t *tri,
                      uint64_t *tri_sum, int32_t sh_base, int64_t nw, const uint64_t *SB,
                      int32_t hub_base, int Hw, const uint64_t *HB, const uint32_t *status,
                      hipStream_t st);
hipError_t launch_superhubs(const int64_t *nrp, const int32_t *ncol, int64_t n, int S, int64_t nw,
                            uint64_t *SB, uint32_t *SP, hipStream_t st);
hipError_t launch_node_aggr(const int64_t *nrp, const int32_t *ncol, const uint8_t *ctype,
                            const uint32_t *tri_slot, const uint32_t *tdeg,
                            int64_t n, int L, uint64_t *A, uint64_t *D, bool ad_u32,
                            const uint32_t *status, hipStream_t st);
// Blocked-group candidates of the wedge-count kernel: heavy groups of at
// least min_wedges wedges (and below 2^31) are appended to cand_a / cand_b
// and counted in a size histogram (all heavy groups still get their tasks);
// null lists turn the blocked path off.
struct BlkSelect {
    uint2 *cand_a, *cand_b;
    uint64_t *hist_a, *hist_b;
    uint64_t min_wedges_a, min_wedges_b;
};
hipError_t launch_cyc_work(const int64_t *nrp, const int32_t *ncol, const uint32_t *neid,
                           const uint32_t *eslot, const uint32_t *nlow, int64_t n, uint32_t *la_l,
                           uint4 *la_h, uint32_t *lb_l, uint4 *lb_h, uint64_t *counters,
                           uint64_t task_wedges, int L, uint64_t range_bytes,
                           uint64_t light_max, const BlkSelect &blk, const uint32_t *status,
                           hipStream_t st);
// The blocked groups of one pass: selection bookkeeping, item prefixes,
// record partition, block counts into the group maps and the emit walk.
hipError_t launch_blk(int pass, const CycleArgs &args, const BlkArgs &blk, int64_t *scan_tmp,
                      hipStream_t st);
int blk_emit_chunk(int L);
int heavy_chunk_for(int L, int threads, int hub_ids = 0, bool t32 = false);
int heavy_hub_ids(int L, int64_t n, int64_t bytes);
hipError_t launch_cycles(int pass, bool heavy, const CycleArgs &args, unsigned grid, hipStream_t st);
hipError_t launch_edges(bool heavy, const EdgeArgs &args, unsigned grid, hipStream_t st);
hipError_t launch_derive(const EdgeArgs &args, unsigned grid, hipStream_t st);
hipError_t launch_global_finalize(const uint64_t *gacc, int L, int gw, uint64_t *out,
                                  uint32_t *status, hipStream_t st);


}  // namespace tg
