// Host side of the typed-graphlet library: workspace planning, the input
// checks, the launch sequence and the C ABI declared in include/tg.h.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstring>
#include <mutex>
#include <vector>

#include "tg_internal.hpp"


namespace tg {

static int64_t binom_host(int64_t a, int64_t b) {
    if (b < 0 || a < b) return 0;
    int64_t r = 1;
    for (int64_t k = 1; k <= b; ++k) r = r * (a - b + k) / k;
    return r;
}

static int bits_for(int64_t n) {
    int b = 1;
    while ((int64_t(1) << b) < n) ++b;
    return b;
}

static size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }
// Workspace regions start at multiples of 256 bytes from the base, and some
// are read 16 bytes at a time, so the base must be 256-byte aligned.
static bool ws_aligned(const void *p) { return ((uintptr_t)p & 255u) == 0; }

// Bytes of dense cycle maps allowed; the number of heavy workgroups follows.
static const size_t MAP_BUDGET = size_t(32) << 30;
static const size_t TBUF_BUDGET = size_t(8) << 30;
static const int MAX_HEAVY_SLOTS = 1280;   // heavy-edge workgroups (5 per CU)
static const int MAX_CYCLE_SLOTS = 2048;   // heavy 4-cycle workgroups (map budget permitting)
// Largest per-edge buffer of triangle-set sums for a separate derivation pass.
static const size_t XYK_BUDGET = size_t(16) << 30;

// Scheduling knobs (tg_set_tuning), per host thread.
thread_local int64_t g_tune[TG_NUM_TUNE] = {
    TASK_WEDGES, SEQ_CLEAR_BYTES, MAX_CYCLE_SLOTS, (int64_t)MAP_BUDGET, MAX_HEAVY_SLOTS,
    (int64_t)TBUF_BUDGET, TASK_RANGE_BYTES, 0, LIGHT_MAXW, TCAP, SH_MAX, SH_DMIN,
    BLK_MIN_WEDGES, (int64_t)BLK_BUDGET, BLK_TASK, BLK_MIN_WEDGES_B, HUB_LDS_BYTES};

// Temporary storage of the preparation's sorts and prefix sums.
static size_t sort_tmp_bytes(int64_t n, int64_t nnz) {
    return sort_tmp_need((n > nnz ? n : nnz) + 1);
}

Budget budget_from_tuning() {
    Budget b;
    b.map_bytes = (size_t)g_tune[TG_TUNE_MAP_BYTES];
    b.cycle_slots = g_tune[TG_TUNE_CYCLE_SLOTS];
    b.tbuf_bytes = (size_t)g_tune[TG_TUNE_TBUF_BYTES];
    b.edge_slots = g_tune[TG_TUNE_EDGE_SLOTS];
    b.sh_max = g_tune[TG_TUNE_SH_MAX];
    b.sh_bytes = SH_BUDGET;
    b.xyk_bytes = XYK_BUDGET;
    b.blk_bytes = (size_t)g_tune[TG_TUNE_BLK_BYTES];
    b.blk_task = g_tune[TG_TUNE_BLK_TASK];
    return b;
}

tg_status plan_layout(int64_t n, int64_t nnz, int L, Layout *lay, int64_t G, const Budget &bud) {
    if (L < 1 || L > TG_MAX_L) return TG_E_L_RANGE;
    if (n < 0 || nnz < 0 || (nnz & 1)) return TG_E_INVALID_ARG;
    if (n >= (int64_t(1) << 31) || nnz >= (int64_t(1) << 32)) return TG_E_TOO_LARGE;
    Layout &y = *lay;
    memset(&y, 0, sizeof(y));
    y.n = n;
    y.nnz = nnz;
    y.m = nnz / 2;
    y.L = L;
    int64_t LL = (int64_t)L * L;
    size_t per_map = (size_t)(n > 0 ? n : 1) * L * sizeof(uint32_t);
    int64_t slots = (int64_t)(bud.map_bytes / per_map);
    if (slots > bud.cycle_slots) slots = bud.cycle_slots;
    if (slots < 1) slots = 1;
    y.heavy_slots = (int)slots;
    size_t per_t = (size_t)(n > 0 ? n : 1) * sizeof(uint32_t);
    int64_t eslots = (int64_t)(bud.tbuf_bytes / per_t);
    if (eslots > bud.edge_slots) eslots = bud.edge_slots;
    if (eslots < 1) eslots = 1;
    y.heavy_edge_slots = (int)eslots;
    // blocked heavy 4-cycle groups: single graphs within the record format
    // (4-bit centre types, at most 8192 blocks per group); one map per group
    // from the task maps' slots
    if (G == 0 && bud.blk_bytes >= 2 && L <= 16 && n > 0 && n <= BLK_MAX_NODES) {
        // group maps in the degree-class layout take far less than the n L
        // words of a task map: the selection fits as many as the map
        // region holds, at most BLK_MAX_GROUPS
        y.blk_groups = BLK_MAX_GROUPS;
        y.blk_nb = (int)((n + BLK_IDS - 1) / BLK_IDS);
        int64_t rec = (int64_t)(bud.blk_bytes / sizeof(uint16_t));
        if (rec > (int64_t)0xffffffffll) rec = (int64_t)0xffffffffll;
        // a pass has at most sum over nodes of d^2 <= nnz^2 / 2 wedges
        // (nnz < 2^32): small graphs need no more records than that
        const double cap = 0.5 * (double)nnz * (double)nnz + 8.0;
        if ((double)rec > cap) rec = (int64_t)cap;
        y.blk_records = rec;
        y.blk_nbk = (int64_t)y.blk_groups * y.blk_nb;
        // histogram matrix: one row of block counts per walk task, at most
        // (records / task + groups) tasks of blk_nb blocks; kept within 1 GiB
        const int64_t task = bud.blk_task > 0 ? bud.blk_task : BLK_TASK;
        const int64_t mat = (rec / task + y.blk_groups + 1) * (int64_t)y.blk_nb;
        y.blk_mat = mat * (int64_t)sizeof(uint32_t) <= (int64_t(1) << 30) ? mat : 0;
    }
    {
        int64_t scan_len = nnz > y.blk_nbk ? nnz : y.blk_nbk;
        y.sort_tmp_bytes = sort_tmp_bytes(n, scan_len);
    }
    if (y.sort_tmp_bytes == 0) return TG_E_INTERNAL;
    int gw = (int)(binom_host(L + 1, 2) + 2 * binom_host(L + 2, 3) + 6 * binom_host(L + 3, 4));

    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align_up(off + bytes);
        return o;
    };
    y.off_status = take(64);
    y.off_counters = take(sizeof(uint64_t) * C_NUM);
    y.off_deg = take(sizeof(uint32_t) * (n + 1));
    y.off_ucount = take(sizeof(int64_t) * (n + 1));
    y.off_eoff = take(sizeof(int64_t) * (n + 1));
    y.off_order = take(sizeof(int32_t) * (n + 1));
    y.off_newid = take(sizeof(int32_t) * (n + 1));
    y.off_ntype = take(n + 1);
    y.off_nrp = take(sizeof(int64_t) * (n + 1));
    y.off_ndeg = take(sizeof(int64_t) * (n + 1));
    int64_t nk = nnz > n ? nnz : n;
    y.off_key_a = take(sizeof(uint64_t) * (nk + 1));
    y.off_key_b = take(sizeof(uint64_t) * (nk + 1));
    y.off_val_a = take(sizeof(uint32_t) * (nk + 1));
    y.off_val_b = take(sizeof(uint32_t) * (nk + 1));
    y.off_ncol = take(sizeof(int32_t) * (nnz + 1));
    y.off_ctype = take((size_t)nnz + 1);
    y.off_neid = take(sizeof(uint32_t) * (nnz + 1));
    y.off_ei = take(sizeof(int32_t) * (y.m + 1));
    y.off_ej = take(sizeof(int32_t) * (y.m + 1));
    y.off_tdeg = take(sizeof(uint32_t) * (size_t)(n + 1) * tri_pitch(L));
    y.off_tri = take(sizeof(uint32_t) * (y.m + 1) * L);
    y.off_tri_slot = take(sizeof(uint32_t) * (size_t)(nnz + 1) * tri_pitch(L));
    y.off_A = take(sizeof(uint64_t) * (n + 1) * LL);
    y.off_D = take(sizeof(uint64_t) * (n + 1) * LL);
    y.off_NC = take(sizeof(uint64_t) * (y.m + 1) * LL);
    y.off_listA_light = take(sizeof(uint32_t) * (n + 1));
    y.off_listA_heavy = take(sizeof(uint4) * (n + 1 + TASK_EXTRA));
    y.off_listB_light = take(sizeof(uint32_t) * (n + 1));
    y.off_listB_heavy = take(sizeof(uint4) * (n + 1 + TASK_EXTRA));
    y.off_list_edge = take(sizeof(uint32_t) * (y.m + 1));
    y.off_maps = take(per_map * (size_t)y.heavy_slots);
    y.off_tbuf = take(per_t * (size_t)y.heavy_edge_slots);
    y.off_gacc = take(sizeof(uint64_t) * gw);
    y.off_sort_tmp = take(y.sort_tmp_bytes);
    y.off_hstart = take(sizeof(int64_t) * (n + 1));
    y.off_eslot = take(sizeof(uint32_t) * (2 * y.m + 1));
    // deferred derivation (single graphs): Xi, Xj, Y, K of every edge
    y.defer = G == 0 && (size_t)y.m * 4 * LL * sizeof(uint64_t) <= bud.xyk_bytes;
    if (y.defer) y.off_xyk = take(sizeof(uint64_t) * (size_t)(y.m + 1) * 4 * LL);
    y.off_nlow = take(sizeof(uint32_t) * (n + 1));
    const size_t hw = HUB_MAX / 64;
    y.off_HB = take(sizeof(uint64_t) * HUB_MAX * hw);
    y.off_hpre = take(sizeof(uint32_t) * HUB_MAX * hw);
    y.off_TM = take(sizeof(uint64_t) * TG_MAX_L * hw);
    y.G = G;
    {
        const int64_t nw = (n + 63) / 64;
        const size_t per_sh = (size_t)nw * (sizeof(uint64_t) + sizeof(uint32_t));
        int64_t shm = (int64_t)(bud.sh_bytes / (per_sh > 0 ? per_sh : 1));
        if (shm > bud.sh_max) shm = bud.sh_max;
        y.sh_max = (int)shm;
        y.off_SB = take(sizeof(uint64_t) * (size_t)nw * (size_t)(shm > 0 ? shm : 1));
        y.off_SP = take(sizeof(uint32_t) * (size_t)nw * (size_t)(shm > 0 ? shm : 1));
    }
    y.off_node_graph = take(sizeof(int32_t) * (G > 0 ? n + 1 : 1));
    y.off_ngraph = take(sizeof(int32_t) * (G > 0 ? n + 1 : 1));
    y.off_gedge = take(sizeof(int64_t) * (G + 1));
    y.off_pacc = take(sizeof(uint64_t) * (size_t)pa_layout(L).gstart[9]);
    if (y.blk_groups > 0) {
        const size_t kg = (size_t)y.blk_groups;
        y.off_blk_list_a = take(sizeof(uint2) * kg);
        y.off_blk_list_b = take(sizeof(uint2) * kg);
        y.off_blk_meta = take(sizeof(uint32_t) * (4 * (kg + 1) + 8 * (kg / 8 + 1)));
        y.off_blk_mat = take(sizeof(uint32_t) * (size_t)(y.blk_mat > 0 ? y.blk_mat : 1));
        // items of distinct groups: at most one per adjacency slot, plus a
        // total per group
        y.off_blk_ipre = take(sizeof(uint32_t) * ((size_t)nnz + kg + 1));
        y.off_blk_bcount = take(sizeof(int64_t) * (size_t)(y.blk_nbk + 1));
        y.off_blk_bstart = take(sizeof(int64_t) * (size_t)(y.blk_nbk + 1));
        y.off_blk_pcur = take(sizeof(uint32_t) * (size_t)(y.blk_nbk + 1));
        y.off_blk_bgroup = take(sizeof(uint32_t) * (size_t)(y.blk_nbk + 1));
        // padded for the count kernel's 16-byte loads past the last record
        y.off_blk_rec = take(sizeof(uint16_t) * (size_t)y.blk_records + 16);
        y.off_blk_cand_a = take(sizeof(uint2) * (size_t)(n + 1));
        y.off_blk_cand_b = take(sizeof(uint2) * (size_t)(n + 1));
        y.off_blk_flag = take(2 * (size_t)(n + 8));
        y.off_blk_hist = take(sizeof(uint64_t) * 2 * 2 * BLK_BINS);
    }
    y.total = off;
    return TG_OK;
}

// --------------------------------------------------------------- timing

namespace {
struct Timing {
    bool enabled = false;
    std::vector<hipEvent_t> ev;
    std::vector<const char *> names;
    int used = 0;
    hipStream_t stream = nullptr;
    int64_t stats[TG_NUM_STATS] = {0};
};
thread_local Timing g_timing;

void timing_reset(hipStream_t st) {
    g_timing.used = 0;
    g_timing.names.clear();
    g_timing.stream = st;
}

// Per-class device time of the instrumented calls (directed counts,
// embeddings): launches of one class are bracketed by two events on the
// caller's stream; the elapsed times are added to the class's sums when
// the call has synchronised the stream (ksum_collect).
struct KSum {
    const char *name;
    double ms, units;
    int64_t calls;
};
struct KPending {
    int cls;
    double units;
    int ev;
};
thread_local std::vector<KSum> g_ksums;
thread_local std::vector<hipEvent_t> g_kev;
thread_local std::vector<KPending> g_kpend;
thread_local int g_kev_used = 0;
thread_local int g_kopen = -1;

}  // namespace

void ksum_reset() {
    g_ksums.clear();
    g_kpend.clear();
    g_kev_used = 0;
    g_kopen = -1;
}

void ksum_begin(hipStream_t st) {
    if (!g_timing.enabled) return;
    if ((int)g_kev.size() < g_kev_used + 2) {
        hipEvent_t a, b;
        if (hipEventCreate(&a) != hipSuccess) return;
        if (hipEventCreate(&b) != hipSuccess) {
            (void)hipEventDestroy(a);
            return;
        }
        g_kev.push_back(a);
        g_kev.push_back(b);
    }
    if (hipEventRecord(g_kev[g_kev_used], st) != hipSuccess) return;
    g_kopen = g_kev_used;
    g_kev_used += 2;
}

void ksum_end(const char *cls, double units, hipStream_t st) {
    if (!g_timing.enabled || g_kopen < 0) return;
    if (hipEventRecord(g_kev[g_kopen + 1], st) != hipSuccess) return;
    int c = -1;
    for (int q = 0; q < (int)g_ksums.size(); ++q)
        if (std::strcmp(g_ksums[q].name, cls) == 0) c = q;
    if (c < 0) {
        g_ksums.push_back({cls, 0.0, 0.0, 0});
        c = (int)g_ksums.size() - 1;
    }
    g_kpend.push_back({c, units, g_kopen});
    g_kopen = -1;
}

void ksum_collect() {
    if (!g_timing.enabled) return;
    for (const KPending &k : g_kpend) {
        float v = 0.f;
        if (hipEventElapsedTime(&v, g_kev[k.ev], g_kev[k.ev + 1]) != hipSuccess) continue;
        g_ksums[k.cls].ms += v;
        g_ksums[k.cls].units += k.units;
        g_ksums[k.cls].calls += 1;
    }
    g_kpend.clear();
    g_kev_used = 0;
}

namespace {

void timing_mark(const char *name) {
    if (!g_timing.enabled) return;
    Timing &T = g_timing;
    if ((int)T.ev.size() <= T.used) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return;
        T.ev.push_back(e);
    }
    if (hipEventRecord(T.ev[T.used], T.stream) != hipSuccess) return;
    T.names.push_back(name);
    ++T.used;
}
}  // namespace

static tg_status status_from_bits(uint32_t bits) {
    if (bits & (ST_BATCH | ST_CROSS_GRAPH)) return TG_E_BATCH;
    if (bits & ST_TYPE_RANGE) return TG_E_TYPE_RANGE;
    if (bits & (ST_COL_RANGE | ST_UNSORTED | ST_SELF_LOOP | ST_ASYMMETRIC | ST_EDGE_COUNT))
        return TG_E_NOT_SIMPLE;
    if (bits) return TG_E_INTERNAL;
    return TG_OK;
}

thread_local char g_last_error[256];

static tg_status hip_failed(hipError_t e, const char *what) {
    snprintf(g_last_error, sizeof(g_last_error), "%s: %s (%d)", what, hipGetErrorString(e), (int)e);
    return TG_E_DEVICE;
}

#define HIPCHK(x) do { hipError_t e_ = (x); if (e_ != hipSuccess) return hip_failed(e_, #x); } while (0)

template <class T>
static T *at(void *base, size_t off) {
    return reinterpret_cast<T *>(static_cast<char *>(base) + off);
}

// One counting call.  pa: per_edge and global_counts receive the
// position-aware layout (needs the separate derivation pass, y.defer).
// status_out (batches only): the call does not synchronise with the host at
// all; it needs the batch's declared largest graph (batch->max_nodes, checked
// on the device) and writes its tg_status to status_out on the device.
static tg_status run(const int64_t *row_ptr, const int32_t *col, const uint8_t *types, int64_t n,
                     int64_t nnz, int L, uint64_t *per_edge, uint64_t *global_counts, void *ws,
                     const Layout &y, hipStream_t st, const BatchIn *batch, bool pa = false,
                     int32_t *status_out = nullptr) {
    if (pa && (batch || !y.defer)) return TG_E_INTERNAL;
    const bool async = status_out != nullptr;
    if (async && (!batch || batch->max_nodes < 1)) return TG_E_INTERNAL;
    const int64_t m = y.m;
    const int LL = L * L;
    const int gw = tg_global_width(L);
    g_last_error[0] = 0;
    uint32_t *status = at<uint32_t>(ws, y.off_status);
    uint64_t *counters = at<uint64_t>(ws, y.off_counters);
    uint32_t *deg = at<uint32_t>(ws, y.off_deg);
    int64_t *ucount = at<int64_t>(ws, y.off_ucount);
    int64_t *eoff = at<int64_t>(ws, y.off_eoff);
    int32_t *order = at<int32_t>(ws, y.off_order);
    int32_t *newid = at<int32_t>(ws, y.off_newid);
    uint8_t *ntype = at<uint8_t>(ws, y.off_ntype);
    int64_t *nrp = at<int64_t>(ws, y.off_nrp);
    int64_t *ndeg = at<int64_t>(ws, y.off_ndeg);
    uint64_t *key_a = at<uint64_t>(ws, y.off_key_a);
    uint64_t *key_b = at<uint64_t>(ws, y.off_key_b);
    uint32_t *val_a = at<uint32_t>(ws, y.off_val_a);
    uint32_t *val_b = at<uint32_t>(ws, y.off_val_b);
    int32_t *ncol = at<int32_t>(ws, y.off_ncol);
    uint32_t *neid = at<uint32_t>(ws, y.off_neid);
    int32_t *ei = at<int32_t>(ws, y.off_ei);
    int32_t *ej = at<int32_t>(ws, y.off_ej);
    uint32_t *tdeg = at<uint32_t>(ws, y.off_tdeg);
    uint32_t *tri = at<uint32_t>(ws, y.off_tri);
    uint32_t *tri_slot = at<uint32_t>(ws, y.off_tri_slot);
    uint64_t *A = at<uint64_t>(ws, y.off_A);
    uint64_t *D = at<uint64_t>(ws, y.off_D);
    uint64_t *NC = at<uint64_t>(ws, y.off_NC);
    uint32_t *la_l = at<uint32_t>(ws, y.off_listA_light);
    uint4 *la_h = at<uint4>(ws, y.off_listA_heavy);
    uint32_t *lb_l = at<uint32_t>(ws, y.off_listB_light);
    uint4 *lb_h = at<uint4>(ws, y.off_listB_heavy);
    uint32_t *le = at<uint32_t>(ws, y.off_list_edge);
    uint32_t *maps = at<uint32_t>(ws, y.off_maps);
    uint32_t *tbuf = at<uint32_t>(ws, y.off_tbuf);
    uint64_t *gacc = at<uint64_t>(ws, y.off_gacc);
    void *stmp = at<void>(ws, y.off_sort_tmp);
    int64_t *stmp64 = static_cast<int64_t *>(stmp);
    if (sort_tmp_bytes(n, nnz) > y.sort_tmp_bytes) return TG_E_INTERNAL;

    int32_t *node_graph = batch ? at<int32_t>(ws, y.off_node_graph) : nullptr;
    int32_t *ngraph = batch ? at<int32_t>(ws, y.off_ngraph) : nullptr;
    int64_t *gedge = at<int64_t>(ws, y.off_gedge);

    timing_reset(st);
    timing_mark("start");
    // status, counters and global accumulators start at zero
    HIPCHK(launch_fill_u64(reinterpret_cast<uint64_t *>(status), 0, 8, st));
    HIPCHK(launch_fill_u64(counters, 0, C_NUM, st));
    if (batch) HIPCHK(launch_fill_u64(global_counts, 0, batch->globals_len, st));
    else HIPCHK(launch_fill_u64(gacc, 0, gw, st));

    // ---- input checks: batch descriptor, rows, degrees, edge numbering.
    // Every kernel after a check returns at once once an input check has
    // failed, so the host needs to look at the status only where it sizes
    // later launches (hub core, super-hubs, largest degree).
    uint64_t max_gsize = 0;
    if (batch) {
        HIPCHK(launch_batch_graphs(batch->node_ptr, batch->gL, batch->goff, batch->G, n, L,
                                   batch->globals_len, batch->max_nodes, node_graph, status,
                                   counters + C_MAX_GSIZE, st));
        if (async) {
            max_gsize = (uint64_t)batch->max_nodes;
        } else {
            uint32_t bst = 0;
            HIPCHK(hipMemcpyAsync(&bst, status, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
            HIPCHK(hipMemcpyAsync(&max_gsize, counters + C_MAX_GSIZE, sizeof(uint64_t),
                                  hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            if (bst) return status_from_bits(bst);
        }
    }
    HIPCHK(launch_check_rows(row_ptr, col, types, n, nnz, L, deg, ucount, status, node_graph,
                             batch ? batch->gL : nullptr, st));
    HIPCHK(launch_excl_scan(ucount, eoff, n + 1, stmp64, status, st));
    HIPCHK(launch_check_edge_count(eoff, n, m, status, st));
    if (batch) HIPCHK(launch_batch_edges(batch->node_ptr, eoff, batch->G, gedge, status, st));

    // ---- relabel by (degree, id), or (graph, degree, id) for a batch
    //      (each graph's nodes contiguous): rank order = internal id order.
    //      Degrees are below the node count (of the largest graph).
    const int deg_bits = bits_for(batch ? (int64_t)max_gsize : n);
    const int key_bits = deg_bits + (batch ? bits_for(batch->G) : 0);
    HIPCHK(launch_node_keys(deg, n, node_graph, deg_bits, key_a, val_a, status, st));
    uint64_t *sk = nullptr;
    uint32_t *sv = nullptr;
    HIPCHK(radix_sort(key_a, key_b, val_a, val_b, n, key_bits, stmp, status, st, &sk, &sv));
    HIPCHK(launch_relabel(sv, types, deg, n, order, newid, ntype, ndeg, counters + C_HUB_CAND,
                          (uint32_t)g_tune[TG_TUNE_SH_DEG], node_graph, ngraph, status, st));
    HIPCHK(launch_excl_scan(ndeg, nrp, n + 1, stmp64, status, st));
    const int bits = bits_for(n);
    HIPCHK(launch_slot_keys(row_ptr, col, ucount, eoff, newid, n, bits, key_a, val_a, ei, ej, status,
                            st));
    // hub core and super-hubs: single graphs only (in a batch the top ids are
    // not the top degrees); the largest degree sizes the word widths
    uint64_t cand[2] = {0, 0};
    int64_t max_deg = 0;
    if (batch) {
        max_deg = max_gsize > 0 ? (int64_t)max_gsize - 1 : 0;  // a bound
    }
    if (!async) {
        uint32_t bits_now = 0;
        HIPCHK(hipMemcpyAsync(&bits_now, status, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
        if (!batch) {
            HIPCHK(hipMemcpyAsync(cand, counters + C_HUB_CAND, 2 * sizeof(uint64_t),
                                  hipMemcpyDeviceToHost, st));
            // in degree order the top-ranked node has the largest degree
            if (n > 0)
                HIPCHK(hipMemcpyAsync(&max_deg, ndeg + (n - 1), sizeof(int64_t),
                                      hipMemcpyDeviceToHost, st));
        }
        HIPCHK(hipStreamSynchronize(st));
        if (bits_now) return status_from_bits(bits_now);
    }
    // hub core: the highest-ranked nodes of degree >= HUB_DMIN, at most HUB_MAX
    const uint64_t hub_cand = batch ? 0 : cand[0], sh_cand = batch ? 0 : cand[1];
    const int H = (int)(hub_cand < (uint64_t)HUB_MAX ? hub_cand : (uint64_t)HUB_MAX);
    // super-hubs: the highest-ranked nodes of degree >= the super-hub degree
    // (tuning knob) that fit; nodes of that degree beyond them are probed by
    // binary search like any other
    const int S = (int)(sh_cand < (uint64_t)y.sh_max ? sh_cand : (uint64_t)y.sh_max);
    const int32_t sh_base = (int32_t)(n - S);
    const int64_t nw = (n + 63) / 64;
    uint64_t *SB = at<uint64_t>(ws, y.off_SB);
    uint32_t *SP = at<uint32_t>(ws, y.off_SP);
    // bit rows padded to whole 64-byte blocks (8 words) for vector loads
    const int Hw = H > 0 ? (((H + 63) / 64 + 7) / 8) * 8 : 0;
    const int32_t hub_base = (int32_t)(n - H);
    HIPCHK(radix_sort(key_a, key_b, val_a, val_b, nnz, 2 * bits, stmp, status, st, &sk, &sv));
    uint32_t *eslot = at<uint32_t>(ws, y.off_eslot);
    uint32_t *nlow = at<uint32_t>(ws, y.off_nlow);
    uint8_t *ctype = at<uint8_t>(ws, y.off_ctype);
    HIPCHK(launch_finish_csr(sk, sv, nnz, bits, ntype, eslot, ncol, neid, ctype, status, st));
    int64_t *hstart = at<int64_t>(ws, y.off_hstart);
    uint64_t *HB = at<uint64_t>(ws, y.off_HB);
    uint32_t *hpre = at<uint32_t>(ws, y.off_hpre);
    uint64_t *TM = at<uint64_t>(ws, y.off_TM);
    HIPCHK(launch_tdeg(nrp, ncol, ctype, n, L, hub_base, tdeg, hstart, nlow, status, st));
    HIPCHK(launch_hub_build(nrp, ncol, hstart, ntype, n, H, Hw, L, HB, hpre, TM, st));
    HIPCHK(launch_superhubs(nrp, ncol, n, S, nw, SB, SP, st));
    timing_mark("prep");

    // ---- typed triangles and node aggregates
    HIPCHK(launch_tri(nrp, ncol, ctype, ei, ej, eslot, tri_slot, m, L, tri, counters + C_TRI_SUM,
                      sh_base, nw, SB, hub_base, Hw, HB, status, st));
    timing_mark("tri");
    // every degree below 2^16: node aggregates, per-edge 4-cycle counts and
    // derivation inputs stay below 2^32 and are held as 32-bit words
    const bool words32 = max_deg < 65536;
    HIPCHK(launch_node_aggr(nrp, ncol, ctype, tri_slot, tdeg, n, L, A, D, words32, status, st));
    timing_mark("aggr");

    // ---- 4-cycles from degree-ordered wedges
    HIPCHK(launch_fill_u64(NC, 0, words32 ? (m * LL + 1) / 2 : m * LL, st));
    // blocked path: counts of a blocked group's targets never exceed their
    // degree, held in 16-bit fields
    const bool blk_on = y.blk_groups > 0 && !batch && words32 && L <= 16;
    // a group has at most min(d_max^2, nnz) wedges: a pass whose smallest
    // blocked group cannot occur launches nothing of the blocked path
    const uint64_t wedge_cap = (uint64_t)(max_deg * max_deg < nnz ? max_deg * max_deg : nnz);
    const bool blk_pass[2] = {blk_on && wedge_cap >= (uint64_t)g_tune[TG_TUNE_BLK_WEDGES],
                              blk_on && wedge_cap >= (uint64_t)g_tune[TG_TUNE_BLK_WEDGES_B] &&
                                  g_tune[TG_TUNE_BLK_WEDGES_B] < (int64_t(1) << 31)};
    BlkSelect bsel;
    bsel.cand_a = blk_pass[0] ? at<uint2>(ws, y.off_blk_cand_a) : nullptr;
    bsel.cand_b = blk_pass[1] ? at<uint2>(ws, y.off_blk_cand_b) : nullptr;
    bsel.hist_a = blk_on ? at<uint64_t>(ws, y.off_blk_hist) : nullptr;
    bsel.hist_b = blk_on ? bsel.hist_a + 2 * BLK_BINS : nullptr;
    bsel.min_wedges_a = (uint64_t)g_tune[TG_TUNE_BLK_WEDGES];
    bsel.min_wedges_b = (uint64_t)g_tune[TG_TUNE_BLK_WEDGES_B];
    uint8_t *blk_flag = blk_on ? at<uint8_t>(ws, y.off_blk_flag) : nullptr;
    if (blk_pass[0] || blk_pass[1]) {
        // flags of both passes and the histograms start at zero
        HIPCHK(launch_fill_u64(at<uint64_t>(ws, y.off_blk_flag), 0, (2 * (n + 8) + 7) / 8, st));
        HIPCHK(launch_fill_u64(bsel.hist_a, 0, 4 * BLK_BINS, st));
    }
    HIPCHK(launch_cyc_work(nrp, ncol, neid, eslot, nlow, n, la_l, la_h, lb_l, lb_h, counters,
                           (uint64_t)g_tune[TG_TUNE_TASK_WEDGES], L,
                           (uint64_t)g_tune[TG_TUNE_RANGE_BYTES],
                           (uint64_t)g_tune[TG_TUNE_LIGHT_WEDGES], bsel, status, st));
    timing_mark("cyc_work");
    CycleArgs ca;
    ca.tasks = nullptr;
    ca.eslot = eslot;
    ca.nlow = nlow;
    ca.clear_bytes = (uint64_t)g_tune[TG_TUNE_CLEAR_BYTES];
    ca.nrp = nrp; ca.ncol = ncol; ca.ntype = ntype; ca.neid = neid; ca.ctype = ctype; ca.ei = ei;
    ca.counters = counters; ca.L = L; ca.n = n; ca.NC = NC; ca.nc_u32 = words32 ? 1 : 0; ca.maps = maps;
    ca.status = status;
    {
        // hash slots: the smallest power of two above the light bucket
        int lg = 1;
        while ((int64_t(1) << lg) <= g_tune[TG_TUNE_LIGHT_WEDGES]) ++lg;
        ca.light_log2 = lg;
    }
    ca.deg_sorted = batch ? 0 : 1;
    ca.blk_flag = nullptr;
    ca.hub_ids = 0;
    ca.max_deg = max_deg;
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    int cus = 0;
    HIPCHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    // light groups differ in size up to 512 wedges: many small workgroups
    // balance them (each clears its LDS map per group anyway)
    unsigned light_grid = (unsigned)((cus > 0 ? cus : 256) * 1024);
    for (int pass = 0; pass < 2; ++pass) {
        ca.list = pass == 0 ? la_l : lb_l;
        ca.count_idx = pass == 0 ? C_A_LIGHT : C_B_LIGHT;
        ca.next_idx = 0;
        HIPCHK(launch_cycles(pass, false, ca, light_grid, st));
        timing_mark(pass == 0 ? "cycA_light" : "cycB_light");
        if (blk_pass[pass]) {
            BlkArgs bk;
            bk.list = at<uint2>(ws, pass == 0 ? y.off_blk_list_a : y.off_blk_list_b);
            bk.c_count = pass == 0 ? C_BLK_A : C_BLK_B;
            bk.max_groups = y.blk_groups;
            bk.cand = pass == 0 ? bsel.cand_a : bsel.cand_b;
            bk.c_cand = pass == 0 ? C_BLK_CAND_A : C_BLK_CAND_B;
            bk.hist = pass == 0 ? bsel.hist_a : bsel.hist_b;
            bk.flag = blk_flag + (pass == 0 ? 0 : (size_t)(n + 8));
            bk.max_wedges = (uint64_t)y.blk_records;
            bk.maps_words = (uint64_t)y.heavy_slots * (uint64_t)n * (uint64_t)L;
            bk.task = (uint32_t)g_tune[TG_TUNE_BLK_TASK];
            uint32_t *meta = at<uint32_t>(ws, y.off_blk_meta);
            bk.ioff = meta;
            bk.tstart = meta + (y.blk_groups + 1);
            bk.boff = meta + 2 * (size_t)(y.blk_groups + 1);
            bk.moff = meta + 3 * (size_t)(y.blk_groups + 1);
            bk.xstart = meta + 4 * (size_t)(y.blk_groups + 1);
            bk.mat = at<uint32_t>(ws, y.off_blk_mat);
            bk.mat_cap = y.blk_mat;
            bk.ipre = at<uint32_t>(ws, y.off_blk_ipre);
            bk.bcount = at<int64_t>(ws, y.off_blk_bcount);
            bk.bstart = at<int64_t>(ws, y.off_blk_bstart);
            bk.pcur = at<uint32_t>(ws, y.off_blk_pcur);
            bk.bgroup = at<uint32_t>(ws, y.off_blk_bgroup);
            bk.rec = at<uint16_t>(ws, y.off_blk_rec);
            bk.nb_max = y.blk_nb;
            bk.nbk = y.blk_nbk;
            bk.emit_chunk = blk_emit_chunk(L);
            HIPCHK(launch_blk(pass, ca, bk, stmp64, st));
            timing_mark(pass == 0 ? "cycA_blk" : "cycB_blk");
        }
        ca.blk_flag = blk_pass[pass] ? blk_flag + (pass == 0 ? 0 : (size_t)(n + 8)) : nullptr;
        ca.tasks = pass == 0 ? la_h : lb_h;
        ca.count_idx = pass == 0 ? C_A_HEAVY : C_B_HEAVY;
        ca.next_idx = pass == 0 ? C_A_NEXT : C_B_NEXT;
        // pass B's targets lie above both ends of the wedge and concentrate
        // on the top-ranked nodes (single graphs: ids ranked by degree):
        // those are counted in LDS (16-bit fields, so only when every degree
        // is below 2^16)
        ca.hub_ids = pass == 1 && !batch && words32 && L <= 16
                         ? heavy_hub_ids(L, n, g_tune[TG_TUNE_HUB_LDS]) : 0;
        ca.chunk = heavy_chunk_for(L, pass == 0 ? HEAVY_THREADS_A : HEAVY_THREADS_B, ca.hub_ids,
                                   words32);
        HIPCHK(launch_cycles(pass, true, ca, (unsigned)y.heavy_slots, st));
        timing_mark(pass == 0 ? "cycA_heavy" : "cycB_heavy");
    }

    // ---- cliques, derivation, rows and global counts
    EdgeArgs ea;
    ea.nrp = nrp; ea.ncol = ncol; ea.ntype = ntype; ea.neid = neid; ea.ei = ei; ea.ej = ej;
    ea.ctype = ctype;
    ea.tri = tri; ea.tdeg = tdeg; ea.tri_slot = tri_slot; ea.A = A; ea.D = D; ea.NC = NC; ea.m = m; ea.L = L;
    ea.agg_u32 = words32 ? 1 : 0;  // A, D and NC entries below 2^32
    ea.rows = per_edge; ea.gacc = gacc; ea.gw = gw;
    ea.hist_in_lds = (size_t)gw * sizeof(uint64_t) <= 32768 ? 1 : 0;
    // a batch chunk flushes after at most BATCH_EDGE_CHUNK (256) edges, each
    // adding at most 6 * max_deg^2 to one entry (three orbits of a graphlet,
    // each at most 2 * max_deg^2): 32-bit entries hold that sum when
    // max_deg <= 1024
    if (batch && max_deg <= 1024 && (size_t)gw * sizeof(uint32_t) <= 32768) ea.hist_in_lds = 2;
    // light edges: smaller endpoint degree at most tcap (the LDS list size)
    const int64_t ecut = g_tune[TG_TUNE_EDGE_DEG];
    ea.tcap = (int)(max_deg < ecut ? (max_deg > 0 ? max_deg : 1) : ecut);
    // derive several edges together when their type pairs leave lanes idle
    // (a batch flushes its histogram per graph, so it derives edge by edge)
    {
        const int P = L * (L + 1) / 2;
        // automatic: up to 3 edges (measured best on the power-law graph
        // with L = 5; a fourth slot costs more occupancy than it gains)
        int eb = g_tune[TG_TUNE_DERIVE_EDGES] > 0 ? (int)g_tune[TG_TUNE_DERIVE_EDGES] : 64 / P;
        if (g_tune[TG_TUNE_DERIVE_EDGES] == 0 && eb > 3) eb = 3;
        if (eb > 4) eb = 4;
        if (eb < 1 || batch) eb = 1;
        ea.derive_batch = eb;
    }
    ea.heavy_list = le; ea.counters = counters; ea.tbuf = tbuf; ea.n = n; ea.status = status;
    ea.hub_base = hub_base; ea.Hw = Hw; ea.hstart = hstart; ea.nlow = nlow; ea.HB = HB; ea.hpre = hpre; ea.TM = TM;
    ea.sh_base = sh_base; ea.nw = nw; ea.SB = SB; ea.SP = SP;
    ea.batch = batch ? 1 : 0;
    ea.ngraph = ngraph;
    ea.gedge_ptr = gedge;
    ea.gL = batch ? batch->gL : nullptr;
    ea.goff = batch ? batch->goff : nullptr;
    ea.G = batch ? batch->G : 1;
    if (batch) ea.gacc = global_counts;
    uint64_t *xyk = y.defer ? at<uint64_t>(ws, y.off_xyk) : nullptr;
    ea.xyk = xyk;
    ea.xyk_u32 = words32 ? 1 : 0;
    EdgeArgs ed = ea;  // the separate derivation pass keeps the histogram
    if (xyk) {
        ea.hist_in_lds = 0;
        ea.derive_batch = 1;
    }
    // edge costs are very uneven: many small workgroups balance the light
    // kernel far better than a few long grid-stride loops, except where each
    // workgroup ends by flushing a whole global histogram (fused, one graph)
    const int64_t per_cu = (xyk || batch) ? 2048 : 24;
    unsigned edge_grid = (unsigned)((cus > 0 ? cus : 256) * per_cu);
    int64_t units = batch ? (m + BATCH_EDGE_CHUNK - 1) / BATCH_EDGE_CHUNK : m;
    if ((int64_t)edge_grid > units) edge_grid = (unsigned)(units > 0 ? units : 1);
    HIPCHK(launch_edges(false, ea, edge_grid, st));
    timing_mark("edges_light");
    EdgeArgs eh = ea;
    if (batch) eh.hist_in_lds = 0;  // heavy edges of many graphs: direct per-graph atomics
    else eh.hist_in_lds = ea.hist_in_lds ? 1 : 0;
    eh.derive_batch = 1;
    if (xyk) eh.hist_in_lds = 0;
    HIPCHK(launch_edges(true, eh, (unsigned)y.heavy_edge_slots, st));
    timing_mark("edges_heavy");
    if (pa) {
        const PaLayout pl = pa_layout(L);
        uint64_t *pacc = at<uint64_t>(ws, y.off_pacc);
        HIPCHK(launch_fill_u64(pacc, 0, pl.gstart[9], st));
        ed.gacc = pacc;
        ed.gw = (int)pl.gstart[9];
        ed.hist_in_lds = (size_t)ed.gw * sizeof(uint64_t) <= 32768 ? 1 : 0;
        HIPCHK(launch_derive_pa(ed, pl, (unsigned)(cus > 0 ? cus * 8 : 2048), st));
        timing_mark("derive");
        if (global_counts) HIPCHK(launch_pa_finalize(pacc, pl, global_counts, status, st));
        timing_mark("global");
    } else if (xyk) {
        ed.hist_in_lds = (size_t)gw * sizeof(uint64_t) <= 32768 ? 1 : 0;
        HIPCHK(launch_derive(ed, (unsigned)(cus > 0 ? cus * 8 : 2048), st));
        timing_mark("derive");
    }
    if (pa) {
        // position-aware globals done above
    } else if (batch)
        HIPCHK(launch_batch_finalize(global_counts, batch->gL, batch->goff, batch->G, status, st));
    else if (global_counts)
        HIPCHK(launch_global_finalize(gacc, L, gw, global_counts, status, st));
    if (!pa) timing_mark("global");

    if (async) {
        HIPCHK(launch_status_code(status, status_out, st));
        return TG_OK;
    }
    uint32_t end_bits = 0;
    HIPCHK(hipMemcpyAsync(&end_bits, status, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    uint64_t cnt_host[C_NUM];
    HIPCHK(hipMemcpyAsync(cnt_host, counters, sizeof(cnt_host), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    g_timing.stats[0] = (int64_t)cnt_host[C_WEDGES_A];
    g_timing.stats[1] = (int64_t)(cnt_host[C_A_LIGHT] + cnt_host[C_B_LIGHT]);
    g_timing.stats[2] = (int64_t)cnt_host[C_HEAVY_GROUPS];
    g_timing.stats[3] = (int64_t)cnt_host[C_EDGE_HEAVY];
    g_timing.stats[4] = (int64_t)cnt_host[C_WEDGES_B];
    g_timing.stats[5] = (int64_t)cnt_host[C_WEDGES_A_HEAVY];
    g_timing.stats[6] = (int64_t)cnt_host[C_WEDGES_B_HEAVY];
    g_timing.stats[7] = (int64_t)cnt_host[C_TRI_SUM];
    g_timing.stats[8] = (int64_t)sh_cand;
    g_timing.stats[9] = (int64_t)S;
    {
        const uint64_t kg = (uint64_t)y.blk_groups;
        const uint64_t ka = cnt_host[C_BLK_A] < kg ? cnt_host[C_BLK_A] : kg;
        const uint64_t kb = cnt_host[C_BLK_B] < kg ? cnt_host[C_BLK_B] : kg;
        g_timing.stats[11] = blk_on ? (int64_t)(ka + kb) : 0;
        g_timing.stats[12] = (int64_t)cnt_host[C_BLK_A_DONE];
        g_timing.stats[13] = (int64_t)cnt_host[C_BLK_B_DONE];
    }
    g_timing.stats[10] = (int64_t)H;
    if (end_bits) return status_from_bits(end_bits) == TG_OK ? TG_E_INTERNAL
                                                              : status_from_bits(end_bits);
    return TG_OK;
}

// --------------------------------------------------- allocation-free entry

// Scratch of tg_count_typed_graphlets_noalloc: a file-scope device array,
// one copy per device (at its own address), held until the process ends.
// Host code never passes `scratch` itself to a kernel: it is a host-side
// stand-in; the device address comes from hipGetSymbolAddress, once per
// device, and every use goes through that pointer.
static __device__ __align__(256) unsigned char scratch[TG_NOALLOC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[MAX_DEVICES] = {};

// Device address of the current device's scratch (looked up on the first
// call on that device, with the device current).
static tg_status scratch_for_current_device(void **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_failed(e, "hipGetDevice");
    if (dev < 0 || dev >= MAX_DEVICES) return TG_E_DEVICE;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_failed(e, "hipGetSymbolAddress(scratch)");
        if (!p || !ws_aligned(p)) return TG_E_INTERNAL;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return TG_OK;
}

// Workspace layout inside the scratch: the per-node and per-edge regions
// with one heavy 4-cycle map, one heavy-edge list and no super-hub bitmaps
// must fit; what is left goes to the separate derivation pass's inputs
// (when they take at most half of it), then half of the rest to more
// cycle maps, a quarter to heavy-edge lists and a quarter to super-hub
// bitmaps, each also capped by the calling thread's knobs.
static tg_status plan_noalloc(int64_t n, int64_t nnz, int L, Layout *y) {
    if (L < 1 || L > TG_MAX_L) return TG_E_L_RANGE;
    if (n < 0 || nnz < 0 || (nnz & 1)) return TG_E_INVALID_ARG;
    const size_t cap = (size_t)TG_NOALLOC_SCRATCH_BYTES;
    const size_t slack = size_t(1) << 16;  // region alignment
    const size_t nn = (size_t)(n > 0 ? n : 1);
    const size_t per_map = nn * L * sizeof(uint32_t), per_t = nn * sizeof(uint32_t);
    const size_t per_sh = (size_t)((n + 63) / 64) * (sizeof(uint64_t) + sizeof(uint32_t));
    Budget b{per_map, 1, per_t, 1, 0, 0, 0};
    tg_status s = plan_layout(n, nnz, L, y, 0, b);
    if (s != TG_OK) return s;
    if (y->total + slack > cap) return TG_E_TOO_LARGE;
    size_t rem = cap - y->total - slack;
    const size_t xyk = (size_t)(nnz / 2) * 4 * L * L * sizeof(uint64_t);
    if (xyk <= rem / 2) {
        b.xyk_bytes = xyk;
        rem -= xyk;
    }
    int64_t cs = 1 + (int64_t)(rem / 2 / per_map);
    if (cs > g_tune[TG_TUNE_CYCLE_SLOTS]) cs = g_tune[TG_TUNE_CYCLE_SLOTS];
    int64_t es = 1 + (int64_t)(rem / 4 / per_t);
    if (es > g_tune[TG_TUNE_EDGE_SLOTS]) es = g_tune[TG_TUNE_EDGE_SLOTS];
    int64_t sh = (int64_t)(rem / 4 / per_sh);
    if (sh > g_tune[TG_TUNE_SH_MAX]) sh = g_tune[TG_TUNE_SH_MAX];
    b.cycle_slots = cs;
    b.map_bytes = (size_t)cs * per_map;
    b.edge_slots = es;
    b.tbuf_bytes = (size_t)es * per_t;
    b.sh_max = sh;
    b.sh_bytes = (size_t)sh * per_sh;
    s = plan_layout(n, nnz, L, y, 0, b);
    if (s != TG_OK) return s;
    return y->total <= cap ? TG_OK : TG_E_INTERNAL;
}

}  // namespace tg

// ================================================================ C ABI

extern "C" {

const char *tg_status_str(tg_status s) {
    switch (s) {
        case TG_OK: return "ok";
        case TG_E_INVALID_ARG: return "invalid argument";
        case TG_E_NOT_SIMPLE: return "graph is not a simple symmetric sorted CSR";
        case TG_E_TYPE_RANGE: return "node type out of range";
        case TG_E_L_RANGE: return "number of types out of range";
        case TG_E_WORKSPACE: return "workspace too small";
        case TG_E_DEVICE: return "HIP error";
        case TG_E_INTERNAL: return "internal consistency check failed";
        case TG_E_TOO_LARGE: return "graph too large";
        case TG_E_BATCH: return "inconsistent batch descriptor or an edge between two graphs";
        case TG_E_OOM: return "request does not fit the serving memory";
        case TG_E_TIMEOUT: return "request not finished";
        case TG_E_NO_CONVERGENCE: return "eigensolver did not converge";
    }
    return "unknown status";
}

int32_t tg_row_width(int32_t L) {
    if (L < 1 || L > TG_MAX_L) return 0;
    return 2 * L + 10 * (L * (L + 1) / 2);
}

int32_t tg_global_width(int32_t L) {
    if (L < 1 || L > TG_MAX_L) return 0;
    return (int32_t)(tg::binom_host(L + 1, 2) + 2 * tg::binom_host(L + 2, 3) +
                     6 * tg::binom_host(L + 3, 4));
}

size_t tg_workspace_bytes(int64_t n, int64_t nnz, int32_t L) {
    tg::Layout y;
    if (tg::plan_layout(n, nnz, L, &y) != TG_OK) return 0;
    return y.total;
}

tg_status tg_count_typed_graphlets(const int64_t *row_ptr, const int32_t *col,
                                   const uint8_t *types, int64_t n, int64_t nnz, int32_t L,
                                   uint64_t *per_edge, uint64_t *global_counts, void *workspace,
                                   size_t ws_bytes, void *stream) {
    tg::Layout y;
    tg_status s = tg::plan_layout(n, nnz, L, &y);
    if (s != TG_OK) return s;
    if (n > 0 && (!row_ptr || !types)) return TG_E_INVALID_ARG;
    if (nnz > 0 && !col) return TG_E_INVALID_ARG;
    if (!workspace || !tg::ws_aligned(workspace)) return TG_E_INVALID_ARG;
    if (ws_bytes < y.total) return TG_E_WORKSPACE;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (n == 0) {
        if (global_counts && tg::launch_fill_u64(global_counts, 0, tg_global_width(L), st) !=
                                 hipSuccess)
            return TG_E_DEVICE;
        return hipStreamSynchronize(st) == hipSuccess ? TG_OK : TG_E_DEVICE;
    }
    return tg::run(row_ptr, col, types, n, nnz, L, per_edge, global_counts, workspace, y, st,
                   nullptr);
}

tg_status tg_count_typed_graphlets_noalloc(const int64_t *row_ptr, const int32_t *col,
                                           const uint8_t *types, int64_t n, int64_t nnz,
                                           int32_t L, uint64_t *per_edge,
                                           uint64_t *global_counts, void *stream) {
    tg::Layout y;
    tg_status s = tg::plan_noalloc(n, nnz, L, &y);
    if (s != TG_OK) return s;
    if (n > 0 && (!row_ptr || !types)) return TG_E_INVALID_ARG;
    if (nnz > 0 && !col) return TG_E_INVALID_ARG;
    void *ws = nullptr;
    s = tg::scratch_for_current_device(&ws);
    if (s != TG_OK) return s;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (n == 0) {
        if (global_counts && tg::launch_fill_u64(global_counts, 0, tg_global_width(L), st) !=
                                 hipSuccess)
            return TG_E_DEVICE;
        return hipStreamSynchronize(st) == hipSuccess ? TG_OK : TG_E_DEVICE;
    }
    // no phase events (their creation is not needed by the counts)
    const bool timing = tg::g_timing.enabled;
    tg::g_timing.enabled = false;
    s = tg::run(row_ptr, col, types, n, nnz, L, per_edge, global_counts, ws, y, st, nullptr);
    tg::g_timing.enabled = timing;
    return s;
}

int32_t tg_pa_row_width(int32_t L) {
    if (L < 1 || L > TG_MAX_L) return 0;
    return tg::pa_layout(L).start[tg::PB_NUM];
}

int64_t tg_pa_global_width(int32_t L) {
    if (L < 1 || L > TG_MAX_L) return 0;
    return tg::pa_layout(L).gstart[9];
}

tg_status tg_count_position_aware(const int64_t *row_ptr, const int32_t *col,
                                  const uint8_t *types, int64_t n, int64_t nnz, int32_t L,
                                  uint64_t *per_edge, uint64_t *global_counts, void *workspace,
                                  size_t ws_bytes, void *stream) {
    tg::Layout y;
    tg_status s = tg::plan_layout(n, nnz, L, &y);
    if (s != TG_OK) return s;
    if (n > 0 && (!row_ptr || !types)) return TG_E_INVALID_ARG;
    if (nnz > 0 && !col) return TG_E_INVALID_ARG;
    if (!workspace || !tg::ws_aligned(workspace)) return TG_E_INVALID_ARG;
    if (ws_bytes < y.total) return TG_E_WORKSPACE;
    if (!y.defer) return TG_E_TOO_LARGE;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (n == 0) {
        if (global_counts && tg::launch_fill_u64(global_counts, 0, tg_pa_global_width(L), st) !=
                                 hipSuccess)
            return TG_E_DEVICE;
        return hipStreamSynchronize(st) == hipSuccess ? TG_OK : TG_E_DEVICE;
    }
    return tg::run(row_ptr, col, types, n, nnz, L, per_edge, global_counts, workspace, y, st,
                   nullptr, true);
}

namespace {
// Unordered pair {lo <= hi} at co-lexicographic rank r.
void unrank_pair(int64_t r, int64_t *lo, int64_t *hi) {
    int64_t h = 0;
    while ((h + 1) * (h + 2) / 2 <= r) ++h;
    *hi = h;
    *lo = r - h * (h + 1) / 2;
}

// Sorted multiset of k <= 4 types at co-lexicographic rank r.
void unrank_multiset(int64_t r, int k, int32_t *out) {
    for (int pos = k - 1; pos >= 0; --pos) {
        int64_t c = pos;
        while (tg::binom_host(c + 1, pos + 1) <= r) ++c;
        r -= tg::binom_host(c, pos + 1);
        out[pos] = (int32_t)(c - pos);
    }
}
}  // namespace

tg_status tg_pa_key_describe(int32_t L, int32_t c, int32_t *block, int32_t *t, int32_t *t2) {
    if (L < 1 || L > TG_MAX_L) return TG_E_L_RANGE;
    if (!block || !t || !t2 || c < 0 || c >= tg_pa_row_width(L)) return TG_E_INVALID_ARG;
    const tg::PaLayout pl = tg::pa_layout(L);
    int b = 0;
    while (c >= pl.start[b + 1]) ++b;
    const int q = c - pl.start[b];
    *block = b;
    const int w = pl.start[b + 1] - pl.start[b];
    if (b <= tg::PB_PATH_J) {
        *t = q;
        *t2 = -1;
    } else if (w == L * L) {
        *t = q / L;
        *t2 = q % L;
    } else {
        int p = q, a = 0;
        while (p >= L - a) { p -= L - a; ++a; }
        *t = a;
        *t2 = a + p;
    }
    return TG_OK;
}

tg_status tg_pa_global_key_describe(int32_t L, int64_t idx, int32_t *graphlet,
                                    int32_t types_by_position[4], int32_t *k) {
    if (L < 1 || L > TG_MAX_L) return TG_E_L_RANGE;
    if (!graphlet || !types_by_position || !k || idx < 0 || idx >= tg_pa_global_width(L))
        return TG_E_INVALID_ARG;
    const tg::PaLayout pl = tg::pa_layout(L);
    int h = 0;
    while (idx >= pl.gstart[h + 1]) ++h;
    const int64_t r = idx - pl.gstart[h];
    const int64_t P = L * (L + 1) / 2, c3 = tg::binom_host(L + 2, 3);
    int32_t *o = types_by_position;
    for (int q = 0; q < 4; ++q) o[q] = -1;
    int64_t lo, hi, lo2, hi2;
    switch (h) {
        case 0: unrank_pair(r, &lo, &hi); o[0] = (int32_t)lo; o[1] = (int32_t)hi; *k = 2; break;
        case 1:
            o[0] = (int32_t)(r / P);
            unrank_pair(r % P, &lo, &hi);
            o[1] = (int32_t)lo; o[2] = (int32_t)hi; *k = 3;
            break;
        case 2: unrank_multiset(r, 3, o); *k = 3; break;
        case 3:
            unrank_pair(r, &lo, &hi);   // halves A = lo, B = hi
            o[0] = (int32_t)(lo / L); o[1] = (int32_t)(lo % L);
            o[3] = (int32_t)(hi / L); o[2] = (int32_t)(hi % L); *k = 4;
            break;
        case 4: o[0] = (int32_t)(r / c3); unrank_multiset(r % c3, 3, o + 1); *k = 4; break;
        case 5: {
            int64_t p1, p2;
            unrank_pair(r, &p1, &p2);
            unrank_pair(p1, &lo, &hi);
            unrank_pair(p2, &lo2, &hi2);
            o[0] = (int32_t)lo; o[2] = (int32_t)hi; o[1] = (int32_t)lo2; o[3] = (int32_t)hi2;
            *k = 4;
            break;
        }
        case 6: {
            const int64_t zq = r / P;
            unrank_pair(r % P, &lo, &hi);
            o[0] = (int32_t)lo; o[1] = (int32_t)hi;
            o[2] = (int32_t)(zq % L); o[3] = (int32_t)(zq / L); *k = 4;
            break;
        }
        case 7:
            unrank_pair(r / P, &lo, &hi);
            unrank_pair(r % P, &lo2, &hi2);
            o[0] = (int32_t)lo; o[2] = (int32_t)hi; o[1] = (int32_t)lo2; o[3] = (int32_t)hi2;
            *k = 4;
            break;
        default: unrank_multiset(r, 4, o); *k = 4; break;
    }
    *graphlet = h;
    return TG_OK;
}

size_t tg_batch_workspace_bytes(int64_t n, int64_t nnz, int64_t G, int32_t L_max) {
    tg::Layout y;
    if (G < 1 || tg::plan_layout(n, nnz, L_max, &y, G) != TG_OK) return 0;
    return y.total;
}

tg_status tg_count_batch(const int64_t *row_ptr, const int32_t *col, const uint8_t *types, int64_t n,
                         int64_t nnz, const int64_t *graph_node_ptr, const int32_t *graph_L,
                         int64_t G, int32_t L_max, const int64_t *graph_global_off,
                         int64_t globals_len, uint64_t *per_edge, uint64_t *graph_globals,
                         void *workspace, size_t ws_bytes, void *stream) {
    if (G < 1) return TG_E_INVALID_ARG;
    tg::Layout y;
    tg_status s = tg::plan_layout(n, nnz, L_max, &y, G);
    if (s != TG_OK) return s;
    if (!row_ptr || !types || !graph_node_ptr || !graph_L || !graph_global_off || !graph_globals ||
        !workspace || !tg::ws_aligned(workspace) || (nnz > 0 && !col) || n < 1 || globals_len < 1)
        return TG_E_INVALID_ARG;
    if (ws_bytes < y.total) return TG_E_WORKSPACE;
    tg::BatchIn b{graph_node_ptr, graph_L, graph_global_off, G, globals_len, -1};
    return tg::run(row_ptr, col, types, n, nnz, L_max, per_edge, graph_globals, workspace, y,
                   reinterpret_cast<hipStream_t>(stream), &b);
}

tg_status tg_count_batch_async(const int64_t *row_ptr, const int32_t *col, const uint8_t *types,
                               int64_t n, int64_t nnz, const int64_t *graph_node_ptr,
                               const int32_t *graph_L, int64_t G, int32_t L_max,
                               int64_t max_graph_nodes, const int64_t *graph_global_off,
                               int64_t globals_len, uint64_t *per_edge, uint64_t *graph_globals,
                               void *workspace, size_t ws_bytes, int32_t *status_out,
                               void *stream) {
    if (G < 1 || max_graph_nodes < 1 || max_graph_nodes > n) return TG_E_INVALID_ARG;
    tg::Layout y;
    tg_status s = tg::plan_layout(n, nnz, L_max, &y, G);
    if (s != TG_OK) return s;
    if (!row_ptr || !types || !graph_node_ptr || !graph_L || !graph_global_off || !graph_globals ||
        !workspace || !tg::ws_aligned(workspace) || (nnz > 0 && !col) || n < 1 || globals_len < 1 ||
        !status_out)
        return TG_E_INVALID_ARG;
    if (ws_bytes < y.total) return TG_E_WORKSPACE;
    tg::BatchIn b{graph_node_ptr, graph_L, graph_global_off, G, globals_len, max_graph_nodes};
    // no phase events: the call may be recorded into a graph
    const bool timing = tg::g_timing.enabled;
    tg::g_timing.enabled = false;
    s = tg::run(row_ptr, col, types, n, nnz, L_max, per_edge, graph_globals, workspace, y,
                reinterpret_cast<hipStream_t>(stream), &b, false, status_out);
    tg::g_timing.enabled = timing;
    return s;
}

tg_status tg_key_describe(int32_t L, int32_t c, int32_t *orbit, int32_t *t, int32_t *t2) {
    if (L < 1 || L > TG_MAX_L) return TG_E_L_RANGE;
    if (!orbit || !t || !t2 || c < 0 || c >= tg_row_width(L)) return TG_E_INVALID_ARG;
    if (c < 2 * L) {
        *orbit = c < L ? 1 : 2;
        *t = c % L;
        *t2 = -1;
        return TG_OK;
    }
    int P = L * (L + 1) / 2;
    int q = c - 2 * L;
    *orbit = 3 + q / P;
    int p = q % P, a = 0;
    while (p >= L - a) { p -= L - a; ++a; }
    *t = a;
    *t2 = a + p;
    return TG_OK;
}

tg_status tg_global_key_describe(int32_t L, int32_t idx, int32_t *graphlet, int32_t types_sorted[4],
                                 int32_t *k) {
    if (L < 1 || L > TG_MAX_L) return TG_E_L_RANGE;
    if (!graphlet || !types_sorted || !k || idx < 0 || idx >= tg_global_width(L))
        return TG_E_INVALID_ARG;
    int64_t n2 = tg::binom_host(L + 1, 2), n3 = tg::binom_host(L + 2, 3),
            n4 = tg::binom_host(L + 3, 4);
    int64_t r;
    int h, kk;
    if (idx < n2) { h = 0; kk = 2; r = idx; }
    else if (idx < n2 + n3) { h = 1; kk = 3; r = idx - n2; }
    else if (idx < n2 + 2 * n3) { h = 2; kk = 3; r = idx - n2 - n3; }
    else { int64_t q = idx - n2 - 2 * n3; h = 3 + (int)(q / n4); kk = 4; r = q % n4; }
    // invert the co-lexicographic rank: largest element first
    int32_t out[4] = {0, 0, 0, 0};
    for (int pos = kk - 1; pos >= 0; --pos) {
        int64_t c = pos;  // s_pos + pos is the largest c with C(c, pos+1) <= r
        while (tg::binom_host(c + 1, pos + 1) <= r) ++c;
        r -= tg::binom_host(c, pos + 1);
        out[pos] = (int32_t)(c - pos);
    }
    *graphlet = h;
    *k = kk;
    for (int q = 0; q < 4; ++q) types_sorted[q] = q < kk ? out[q] : -1;
    return TG_OK;
}

void tg_set_timing(int32_t enable) { tg::g_timing.enabled = enable != 0; }

int32_t tg_kernel_sums(const char **names, double *ms, double *units, int64_t *calls,
                       int32_t max_classes) {
    const int cnt = (int)tg::g_ksums.size() < max_classes ? (int)tg::g_ksums.size() : max_classes;
    for (int q = 0; q < cnt; ++q) {
        if (names) names[q] = tg::g_ksums[q].name;
        if (ms) ms[q] = tg::g_ksums[q].ms;
        if (units) units[q] = tg::g_ksums[q].units;
        if (calls) calls[q] = tg::g_ksums[q].calls;
    }
    return cnt < 0 ? 0 : cnt;
}

int32_t tg_phase_times(float *ms, const char **names, int32_t max_phases) {
    tg::Timing &T = tg::g_timing;
    if (T.used < 2) return 0;
    if (hipEventSynchronize(T.ev[T.used - 1]) != hipSuccess) return -1;
    int cnt = 0;
    for (int q = 1; q < T.used && cnt < max_phases; ++q, ++cnt) {
        float v = 0.f;
        if (hipEventElapsedTime(&v, T.ev[q - 1], T.ev[q]) != hipSuccess) v = -1.f;
        if (ms) ms[cnt] = v;
        if (names) names[cnt] = T.names[q];
    }
    return cnt;
}

tg_status tg_set_tuning(int32_t knob, int64_t value) {
    switch (knob) {
    case TG_TUNE_TASK_WEDGES:
        if (value < 1) return TG_E_INVALID_ARG;
        break;
    case TG_TUNE_CLEAR_BYTES:
        if (value < 0 || value > (int64_t(1) << 30)) return TG_E_INVALID_ARG;
        break;
    case TG_TUNE_CYCLE_SLOTS:
    case TG_TUNE_EDGE_SLOTS:
        if (value < 1 || value > 65536) return TG_E_INVALID_ARG;
        break;
    case TG_TUNE_MAP_BYTES:
    case TG_TUNE_TBUF_BYTES:
        if (value < 1) return TG_E_INVALID_ARG;
        break;
    case TG_TUNE_RANGE_BYTES:
        if (value < 0) return TG_E_INVALID_ARG;
        break;
    case TG_TUNE_DERIVE_EDGES:
        if (value < 0 || value > 4) return TG_E_INVALID_ARG;
        break;
    case TG_TUNE_LIGHT_WEDGES:
        if (value < 1 || value > tg::LIGHT_MAXW) return TG_E_INVALID_ARG;
        break;
    case TG_TUNE_EDGE_DEG:
        if (value < 1 || value > tg::TCAP) return TG_E_INVALID_ARG;
        break;
    case TG_TUNE_SH_MAX:
        if (value < 0 || value > tg::SH_MAX) return TG_E_INVALID_ARG;
        break;
    case TG_TUNE_SH_DEG:
        // at least the hub-core degree, so that super-hubs stay inside the core
        if (value < tg::HUB_DMIN || value > INT32_MAX) return TG_E_INVALID_ARG;
        break;
    case TG_TUNE_BLK_WEDGES:
    case TG_TUNE_BLK_WEDGES_B:
        if (value < 1) return TG_E_INVALID_ARG;
        break;
    case TG_TUNE_HUB_LDS:
        if (value < 0 || value > 65536) return TG_E_INVALID_ARG;
        break;
    case TG_TUNE_BLK_TASK:
        if (value < 1024 || value > tg::BLK_TASK) return TG_E_INVALID_ARG;
        break;
    case TG_TUNE_BLK_BYTES:
        // record positions are 32-bit: at most 2^32 records
        if (value < 0 || value > (int64_t(1) << 33)) return TG_E_INVALID_ARG;
        break;
    default:
        return TG_E_INVALID_ARG;
    }
    tg::g_tune[knob] = value;
    return TG_OK;
}

int64_t tg_get_tuning(int32_t knob) {
    if (knob < 0 || knob >= TG_NUM_TUNE) return -1;
    return tg::g_tune[knob];
}

const char *tg_last_error(void) { return tg::g_last_error; }

int32_t tg_last_stats(int64_t *stats, int32_t max_stats) {
    int cnt = max_stats < TG_NUM_STATS ? max_stats : TG_NUM_STATS;
    for (int q = 0; q < cnt; ++q) stats[q] = tg::g_timing.stats[q];
    return cnt;
}

}  // extern "C"
