// Serving loop with continuous batching (native): requests carrying one
// typed graph each are admitted by their HBM footprint into a caller-owned
// device arena, keep their CSR and their global counts there until the
// caller releases them, and are counted by worker threads, each with its
// own HIP stream and a fixed region of the arena for one batch: a free
// worker takes every admitted request not yet started (up to its region
// and an edge budget) as one batched call, so requests that arrive while
// others are on the GPU join the next batch and the workers' batches
// overlap on the device.  Requests of at least `single_edges` edges run as
// single-graph calls (the hub core and super-hub bitmaps that a batch's
// graph-major order gives up).  A failing batch is re-run request by
// request so that only the offending request gets the error.
#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "tg_arena.hpp"
#include "tg_internal.hpp"

namespace tg {

// One request's graph inside the union CSR of a batch.
struct UnionPart {
    const int64_t *rp;
    const int32_t *col;
    const uint8_t *types;
    int64_t n, nnz, node_off, slot_off;
    const uint64_t *src_glob;  // its global vector in the batch's output
    uint64_t *dst_glob;        // its own result slot
    int32_t gw;
};

// One workgroup per part: rows and types of the union.
__global__ void k_union_nodes(const UnionPart *__restrict__ parts, int P, int64_t n_total,
                              int64_t nnz_total, int64_t *__restrict__ urp,
                              uint8_t *__restrict__ utypes) {
    for (int p = blockIdx.x; p < P; p += gridDim.x) {
        const UnionPart q = parts[p];
        for (int64_t v = threadIdx.x; v < q.n; v += blockDim.x) {
            urp[q.node_off + v] = q.rp[v] + q.slot_off;
            utypes[q.node_off + v] = q.types[v];
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) urp[n_total] = nnz_total;
}

// One workgroup per part: neighbour ids shifted by the part's first node.
__global__ void k_union_cols(const UnionPart *__restrict__ parts, int P,
                             int32_t *__restrict__ ucol) {
    for (int p = blockIdx.x; p < P; p += gridDim.x) {
        const UnionPart q = parts[p];
        for (int64_t s = threadIdx.x; s < q.nnz; s += blockDim.x)
            ucol[q.slot_off + s] = q.col[s] + (int32_t)q.node_off;
    }
}

// One workgroup per part: its global vector from the batch output to its slot.
__global__ void k_scatter_globals(const UnionPart *__restrict__ parts, int P) {
    for (int p = blockIdx.x; p < P; p += gridDim.x) {
        const UnionPart q = parts[p];
        for (int c = threadIdx.x; c < q.gw; c += blockDim.x) q.dst_glob[c] = q.src_glob[c];
    }
}

namespace {

using Clock = std::chrono::steady_clock;

enum { ST_WAITING = 0, ST_ADMITTED = 1, ST_RUNNING = 2, ST_DONE = 3 };

struct Req {
    int64_t id = 0;
    int64_t n = 0, nnz = 0;
    int32_t L = 0;
    int mem = TG_MEM_HOST;
    // inputs: host copies (host requests) or the caller's device pointers
    std::vector<int64_t> h_rp;
    std::vector<int32_t> h_col;
    std::vector<uint8_t> h_types;
    const int64_t *d_rp = nullptr;
    const int32_t *d_col = nullptr;
    const uint8_t *d_types = nullptr;
    // device-resident copy and result inside the arena
    int64_t block = -1;
    int64_t *rp = nullptr;
    int32_t *col = nullptr;
    uint8_t *types = nullptr;
    uint64_t *glob = nullptr;
    int state = ST_WAITING;
    tg_status status = TG_OK;
    double t_submit = 0, t_admit = -1, t_start = -1, t_done = -1;
    int64_t batch = -1;
    bool released = false;
    int64_t edges() const { return nnz / 2; }
};

// Bytes of one request's block: CSR, types and its global vector.
size_t block_layout(int64_t n, int64_t nnz, int L, size_t off[4]) {
    size_t o = 0;
    off[0] = o; o = Arena::round(o + sizeof(int64_t) * (size_t)(n + 1));
    off[1] = o; o = Arena::round(o + sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
    off[2] = o; o = Arena::round(o + (size_t)(n > 0 ? n : 1));
    off[3] = o; o = Arena::round(o + sizeof(uint64_t) * (size_t)tg_global_width(L));
    return o;
}

// Layout of a worker's region for a batch of G graphs with n nodes and nnz
// adjacency entries in all: union CSR, batch descriptor, parts, the batch's
// global output, then the workspace.
struct BatchLayout {
    size_t rp, col, types, node_ptr, gL, goff, parts, glob, ws, ws_bytes, total;
};

BatchLayout batch_layout(int64_t n, int64_t nnz, int64_t G, int L_max, int64_t glen) {
    BatchLayout b{};
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o = Arena::round(o + bytes);
        return at;
    };
    b.rp = take(sizeof(int64_t) * (size_t)(n + 1));
    b.col = take(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
    b.types = take((size_t)(n > 0 ? n : 1));
    b.node_ptr = take(sizeof(int64_t) * (size_t)(G + 1));
    b.gL = take(sizeof(int32_t) * (size_t)G);
    b.goff = take(sizeof(int64_t) * (size_t)(G + 1));
    b.parts = take(sizeof(UnionPart) * (size_t)G);
    b.glob = take(sizeof(uint64_t) * (size_t)glen);
    b.ws_bytes = tg_batch_workspace_bytes(n, nnz, G, L_max);
    b.ws = take(b.ws_bytes);
    b.total = o;
    return b;
}

}  // namespace

struct Server {
    char *arena = nullptr;
    size_t arena_bytes = 0, worker_bytes = 0;
    int workers = 0;
    int64_t single_edges = 0, max_batch_edges = 0;
    int device = 0;
    int64_t knobs[TG_NUM_TUNE];
    Arena pool;                       // request blocks: the arena after the worker regions
    size_t pool_base = 0;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<std::unique_ptr<Req>> reqs;   // by ticket
    std::deque<Req *> waiting, admitted;
    std::deque<int64_t> finished;     // tickets done and not yet handed out by take_done
    bool stop = false;
    int64_t batches = 0, done = 0, rejected = 0, single_calls = 0;
    size_t peak_pool = 0;
    double busy_s = 0;
    Clock::time_point t0 = Clock::now();
    std::vector<std::thread> threads;
    tg_status fatal = TG_OK;
    char fatal_msg[256] = {0};

    double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }
    Req *get(int64_t ticket) {
        if (ticket < 0 || ticket >= (int64_t)reqs.size()) return nullptr;
        Req *r = reqs[(size_t)ticket].get();
        return r && !r->released ? r : nullptr;
    }

    // FIFO admission: a waiting request is admitted when its block fits.
    void admit_locked() {
        while (!waiting.empty()) {
            Req *r = waiting.front();
            size_t off[4];
            const size_t bytes = block_layout(r->n, r->nnz, r->L, off);
            const int64_t at = pool.alloc(bytes);
            if (at < 0) return;
            char *base = arena + pool_base + at;
            r->block = at;
            r->rp = reinterpret_cast<int64_t *>(base + off[0]);
            r->col = reinterpret_cast<int32_t *>(base + off[1]);
            r->types = reinterpret_cast<uint8_t *>(base + off[2]);
            r->glob = reinterpret_cast<uint64_t *>(base + off[3]);
            r->state = ST_ADMITTED;
            r->t_admit = now();
            admitted.push_back(r);
            waiting.pop_front();
            if (pool.in_use() > peak_pool) peak_pool = pool.in_use();
        }
    }

    void finish_locked(Req *r, tg_status s) {
        r->status = s;
        r->state = ST_DONE;
        r->t_done = now();
        ++done;
        finished.push_back(r->id);
    }

    // The next batch for a worker: the first admitted request alone if it
    // is large, else the admitted small requests in arrival order while the
    // batch fits the worker's region and the edge budget.
    std::vector<Req *> pick_locked() {
        std::vector<Req *> out;
        while (!admitted.empty()) {
            Req *r0 = admitted.front();
            if (r0->edges() >= single_edges) {
                if (tg_workspace_bytes(r0->n, r0->nnz, r0->L) > worker_bytes) {
                    admitted.pop_front();
                    finish_locked(r0, TG_E_OOM);
                    ++rejected;
                    cv.notify_all();
                    continue;
                }
                admitted.pop_front();
                out.push_back(r0);
                return out;
            }
            break;
        }
        int64_t n = 0, nnz = 0, edges = 0, glen = 0;
        int L_max = 1;
        auto it = admitted.begin();
        while (it != admitted.end()) {
            Req *r = *it;
            if (r->edges() >= single_edges) break;
            const int64_t n2 = n + r->n, nnz2 = nnz + r->nnz;
            const int L2 = r->L > L_max ? r->L : L_max;
            const int64_t glen2 = glen + tg_global_width(r->L);
            const BatchLayout b = batch_layout(n2, nnz2, (int64_t)out.size() + 1, L2, glen2);
            const bool fits = b.ws_bytes > 0 && b.total <= worker_bytes &&
                              (out.empty() || edges + r->edges() <= max_batch_edges);
            if (!fits) {
                if (out.empty()) {   // alone it can never run
                    it = admitted.erase(it);
                    finish_locked(r, TG_E_OOM);
                    ++rejected;
                    cv.notify_all();
                    continue;
                }
                break;
            }
            n = n2; nnz = nnz2; L_max = L2; glen = glen2; edges += r->edges();
            out.push_back(r);
            it = admitted.erase(it);
        }
        return out;
    }

    void worker_main(int w);
    tg_status run_batch(const std::vector<Req *> &batch, char *region, hipStream_t st,
                        UnionPart *staging, size_t staging_parts, std::vector<int64_t> &hbuf,
                        std::vector<int32_t> &hL);
};

namespace {
tg_status upload(Req *r, hipStream_t st) {
    const hipMemcpyKind k = r->mem == TG_MEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
    const void *rp = r->mem == TG_MEM_HOST ? (const void *)r->h_rp.data() : (const void *)r->d_rp;
    const void *col = r->mem == TG_MEM_HOST ? (const void *)r->h_col.data() : (const void *)r->d_col;
    const void *ty = r->mem == TG_MEM_HOST ? (const void *)r->h_types.data()
                                           : (const void *)r->d_types;
    if (hipMemcpyAsync(r->rp, rp, sizeof(int64_t) * (size_t)(r->n + 1), k, st) != hipSuccess)
        return TG_E_DEVICE;
    if (r->nnz > 0 &&
        hipMemcpyAsync(r->col, col, sizeof(int32_t) * (size_t)r->nnz, k, st) != hipSuccess)
        return TG_E_DEVICE;
    if (r->n > 0 && hipMemcpyAsync(r->types, ty, (size_t)r->n, k, st) != hipSuccess)
        return TG_E_DEVICE;
    return TG_OK;
}
}  // namespace

// Counts a batch on the worker's stream; every request gets its status.
tg_status Server::run_batch(const std::vector<Req *> &batch, char *region, hipStream_t st,
                            UnionPart *staging, size_t staging_parts,
                            std::vector<int64_t> &hbuf, std::vector<int32_t> &hL) {
    for (Req *r : batch) {
        tg_status s = upload(r, st);
        if (s != TG_OK) return s;
    }
    if (batch.size() == 1 && batch[0]->edges() >= single_edges) {
        Req *r = batch[0];
        r->status = tg_count_typed_graphlets(r->rp, r->col, r->types, r->n, r->nnz, r->L, nullptr,
                                             r->glob, region, worker_bytes, st);
        return TG_OK;
    }
    const int64_t G = (int64_t)batch.size();
    int64_t n = 0, nnz = 0, glen = 0;
    int L_max = 1;
    for (Req *r : batch) {
        n += r->n;
        nnz += r->nnz;
        glen += tg_global_width(r->L);
        if (r->L > L_max) L_max = r->L;
    }
    const BatchLayout b = batch_layout(n, nnz, G, L_max, glen);
    if ((size_t)G > staging_parts || b.total > worker_bytes) return TG_E_INTERNAL;
    int64_t *urp = reinterpret_cast<int64_t *>(region + b.rp);
    int32_t *ucol = reinterpret_cast<int32_t *>(region + b.col);
    uint8_t *utypes = reinterpret_cast<uint8_t *>(region + b.types);
    int64_t *node_ptr = reinterpret_cast<int64_t *>(region + b.node_ptr);
    int32_t *gL = reinterpret_cast<int32_t *>(region + b.gL);
    int64_t *goff = reinterpret_cast<int64_t *>(region + b.goff);
    UnionPart *parts = reinterpret_cast<UnionPart *>(region + b.parts);
    uint64_t *bglob = reinterpret_cast<uint64_t *>(region + b.glob);
    // descriptor: node_ptr [G+1], goff [G+1] then the L values, in host memory
    hbuf.assign((size_t)(2 * (G + 1)), 0);
    hL.assign((size_t)G, 0);
    int64_t no = 0, so = 0, go = 0;
    for (int64_t g = 0; g < G; ++g) {
        Req *r = batch[(size_t)g];
        hbuf[(size_t)g] = no;
        hbuf[(size_t)(G + 1 + g)] = go;
        hL[(size_t)g] = r->L;
        staging[g] = UnionPart{r->rp, r->col, r->types, r->n, r->nnz, no, so, bglob + go, r->glob,
                               tg_global_width(r->L)};
        no += r->n;
        so += r->nnz;
        go += tg_global_width(r->L);
    }
    hbuf[(size_t)G] = no;
    hbuf[(size_t)(2 * G + 1)] = go;
    if (hipMemcpyAsync(node_ptr, hbuf.data(), sizeof(int64_t) * (size_t)(G + 1),
                       hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(goff, hbuf.data() + G + 1, sizeof(int64_t) * (size_t)(G + 1),
                       hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(gL, hL.data(), sizeof(int32_t) * (size_t)G, hipMemcpyHostToDevice, st) !=
            hipSuccess ||
        hipMemcpyAsync(parts, staging, sizeof(UnionPart) * (size_t)G, hipMemcpyHostToDevice, st) !=
            hipSuccess)
        return TG_E_DEVICE;
    const unsigned grid = (unsigned)(G < 4096 ? G : 4096);
    k_union_nodes<<<grid, 256, 0, st>>>(parts, (int)G, n, nnz, urp, utypes);
    k_union_cols<<<grid, 256, 0, st>>>(parts, (int)G, ucol);
    if (hipGetLastError() != hipSuccess) return TG_E_DEVICE;
    tg_status s = tg_count_batch(urp, ucol, utypes, n, nnz, node_ptr, gL, G, L_max, goff, glen,
                                 nullptr, bglob, region + b.ws, b.ws_bytes, st);
    if (s == TG_OK) {
        k_scatter_globals<<<grid, 256, 0, st>>>(parts, (int)G);
        if (hipGetLastError() != hipSuccess) return TG_E_DEVICE;
        for (Req *r : batch) r->status = TG_OK;
        return TG_OK;
    }
    if (s == TG_E_DEVICE) return s;
    // isolate the failing request(s): each one alone
    for (Req *r : batch)
        r->status = tg_count_typed_graphlets(r->rp, r->col, r->types, r->n, r->nnz, r->L, nullptr,
                                             r->glob, region, worker_bytes, st);
    return TG_OK;
}

void Server::worker_main(int w) {
    if (hipSetDevice(device) != hipSuccess) {
        std::lock_guard<std::mutex> lk(mu);
        fatal = TG_E_DEVICE;
        return;
    }
    // the creating thread's scheduling knobs, with the per-workgroup
    // scratch budgets kept within this worker's region
    for (int k = 0; k < TG_NUM_TUNE; ++k) tg_set_tuning(k, knobs[k]);
    if ((size_t)knobs[TG_TUNE_MAP_BYTES] > worker_bytes / 4)
        tg_set_tuning(TG_TUNE_MAP_BYTES, (int64_t)(worker_bytes / 4 > 0 ? worker_bytes / 4 : 1));
    if ((size_t)knobs[TG_TUNE_TBUF_BYTES] > worker_bytes / 8)
        tg_set_tuning(TG_TUNE_TBUF_BYTES, (int64_t)(worker_bytes / 8 > 0 ? worker_bytes / 8 : 1));
    if ((size_t)knobs[TG_TUNE_BLK_BYTES] > worker_bytes / 16)
        tg_set_tuning(TG_TUNE_BLK_BYTES, (int64_t)(worker_bytes / 16));
    hipStream_t st = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
        std::lock_guard<std::mutex> lk(mu);
        fatal = TG_E_DEVICE;
        return;
    }
    char *region = arena + (size_t)w * worker_bytes;
    const size_t staging_parts = 1 << 16;
    std::vector<UnionPart> staging(staging_parts);
    std::vector<int64_t> hbuf;   // host sources of the descriptor copies, kept
    std::vector<int32_t> hL;     // until the stream has consumed them
    std::unique_lock<std::mutex> lk(mu);
    while (true) {
        admit_locked();
        std::vector<Req *> batch = pick_locked();
        if (batch.empty()) {
            if (stop && waiting.empty() && admitted.empty()) break;
            cv.wait(lk);
            continue;
        }
        const int64_t id = batches++;
        const double t_start = now();
        for (Req *r : batch) {
            r->state = ST_RUNNING;
            r->t_start = t_start;
            r->batch = id;
        }
        if (batch.size() == 1 && batch[0]->edges() >= single_edges) ++single_calls;
        lk.unlock();
        tg_status s = run_batch(batch, region, st, staging.data(), staging_parts, hbuf, hL);
        if (hipStreamSynchronize(st) != hipSuccess) s = TG_E_DEVICE;
        lk.lock();
        busy_s += now() - t_start;
        for (Req *r : batch) finish_locked(r, s == TG_OK ? r->status : s);
        if (s == TG_E_DEVICE && fatal == TG_OK) {
            fatal = s;
            snprintf(fatal_msg, sizeof(fatal_msg), "%s", tg_last_error());
        }
        cv.notify_all();
    }
    lk.unlock();
    (void)hipStreamDestroy(st);
}

}  // namespace tg

struct tg_server {
    tg::Server s;
};

extern "C" {

tg_status tg_server_create(void *arena, size_t arena_bytes, int32_t workers, size_t worker_bytes,
                           int64_t single_edges, int64_t max_batch_edges, tg_server **out) {
    if (!out) return TG_E_INVALID_ARG;
    *out = nullptr;
    if (!arena || ((uintptr_t)arena & 255u) || workers < 1 || workers > 64 || worker_bytes < 4096 ||
        single_edges < 1 || max_batch_edges < 1)
        return TG_E_INVALID_ARG;
    worker_bytes &= ~(size_t)255;
    if ((size_t)workers * worker_bytes >= arena_bytes) return TG_E_OOM;
    tg_server *h = new (std::nothrow) tg_server;
    if (!h) return TG_E_OOM;
    tg::Server &s = h->s;
    s.arena = static_cast<char *>(arena);
    s.arena_bytes = arena_bytes;
    s.workers = workers;
    s.worker_bytes = worker_bytes;
    s.single_edges = single_edges;
    s.max_batch_edges = max_batch_edges;
    if (hipGetDevice(&s.device) != hipSuccess) {
        delete h;
        return TG_E_DEVICE;
    }
    for (int k = 0; k < TG_NUM_TUNE; ++k) s.knobs[k] = tg_get_tuning(k);
    s.pool_base = (size_t)workers * worker_bytes;
    s.pool.reset(arena_bytes - s.pool_base);
    for (int w = 0; w < workers; ++w) s.threads.emplace_back([&s, w] { s.worker_main(w); });
    *out = h;
    return TG_OK;
}

tg_status tg_server_submit(tg_server *h, const tg_graph_desc *g, int64_t *ticket) {
    if (!h || !g || !ticket) return TG_E_INVALID_ARG;
    if (g->L < 1 || g->L > TG_MAX_L) return TG_E_L_RANGE;
    if (g->n < 1 || g->nnz < 0 || (g->nnz & 1) || (g->nnz > 0 && !g->col) || !g->row_ptr ||
        !g->types || (g->mem != TG_MEM_HOST && g->mem != TG_MEM_DEVICE))
        return TG_E_INVALID_ARG;
    if (g->n >= (int64_t(1) << 31) || g->nnz >= (int64_t(1) << 32)) return TG_E_TOO_LARGE;
    tg::Server &s = h->s;
    size_t off[4];
    if (tg::block_layout(g->n, g->nnz, g->L, off) > s.pool.size()) return TG_E_OOM;
    std::unique_ptr<tg::Req> r(new (std::nothrow) tg::Req);
    if (!r) return TG_E_OOM;
    r->n = g->n;
    r->nnz = g->nnz;
    r->L = g->L;
    r->mem = g->mem;
    if (g->mem == TG_MEM_HOST) {
        r->h_rp.assign(g->row_ptr, g->row_ptr + g->n + 1);
        r->h_col.assign(g->col, g->col + g->nnz);
        r->h_types.assign(g->types, g->types + g->n);
    } else {
        r->d_rp = g->row_ptr;
        r->d_col = g->col;
        r->d_types = g->types;
    }
    std::lock_guard<std::mutex> lk(s.mu);
    if (s.stop) return TG_E_INVALID_ARG;
    r->id = (int64_t)s.reqs.size();
    r->t_submit = s.now();
    s.waiting.push_back(r.get());
    *ticket = r->id;
    s.reqs.push_back(std::move(r));
    s.cv.notify_all();
    return TG_OK;
}

tg_status tg_server_poll(tg_server *h, int64_t ticket, tg_request_info *info) {
    if (!h || !info) return TG_E_INVALID_ARG;
    tg::Server &s = h->s;
    std::lock_guard<std::mutex> lk(s.mu);
    tg::Req *r = s.get(ticket);
    if (!r) return TG_E_INVALID_ARG;
    info->state = r->state;
    info->status = r->state == tg::ST_DONE ? (int32_t)r->status : -1;
    info->global_counts = r->state == tg::ST_DONE && r->status == TG_OK ? r->glob : nullptr;
    info->t_submit = r->t_submit;
    info->t_admit = r->t_admit;
    info->t_start = r->t_start;
    info->t_done = r->t_done;
    info->batch = r->batch;
    return TG_OK;
}

tg_status tg_server_wait(tg_server *h, int64_t ticket, double timeout_s) {
    if (!h) return TG_E_INVALID_ARG;
    tg::Server &s = h->s;
    std::unique_lock<std::mutex> lk(s.mu);
    tg::Req *r = s.get(ticket);
    if (!r) return TG_E_INVALID_ARG;
    const auto until = std::chrono::steady_clock::now() +
                       std::chrono::duration_cast<std::chrono::steady_clock::duration>(
                           std::chrono::duration<double>(timeout_s > 0 ? timeout_s : 0));
    while (r->state != tg::ST_DONE) {
        if (timeout_s <= 0) return TG_E_TIMEOUT;
        if (s.cv.wait_until(lk, until) == std::cv_status::timeout && r->state != tg::ST_DONE)
            return TG_E_TIMEOUT;
    }
    return TG_OK;
}

int32_t tg_server_take_done(tg_server *h, int64_t *tickets, int32_t max_tickets,
                            double timeout_s) {
    if (!h || !tickets || max_tickets < 1) return 0;
    tg::Server &s = h->s;
    std::unique_lock<std::mutex> lk(s.mu);
    if (s.finished.empty() && timeout_s > 0)
        s.cv.wait_for(lk, std::chrono::duration<double>(timeout_s),
                      [&] { return !s.finished.empty(); });
    int32_t cnt = 0;
    while (cnt < max_tickets && !s.finished.empty()) {
        tickets[cnt++] = s.finished.front();
        s.finished.pop_front();
    }
    return cnt;
}

tg_status tg_server_release(tg_server *h, int64_t ticket) {
    if (!h) return TG_E_INVALID_ARG;
    tg::Server &s = h->s;
    std::lock_guard<std::mutex> lk(s.mu);
    tg::Req *r = s.get(ticket);
    if (!r || r->state != tg::ST_DONE) return TG_E_INVALID_ARG;
    if (r->block >= 0) s.pool.release(r->block);
    r->block = -1;
    r->released = true;
    r->h_rp.clear();
    r->h_rp.shrink_to_fit();
    r->h_col.clear();
    r->h_col.shrink_to_fit();
    r->h_types.clear();
    r->h_types.shrink_to_fit();
    s.cv.notify_all();   // memory freed: admission may proceed
    return TG_OK;
}

int32_t tg_server_stats(tg_server *h, int64_t *stats, int32_t max_stats) {
    if (!h || !stats) return 0;
    tg::Server &s = h->s;
    std::lock_guard<std::mutex> lk(s.mu);
    const int64_t v[TG_SERVER_NUM_STATS] = {
        (int64_t)s.reqs.size(), s.done, s.rejected, s.batches, s.single_calls,
        (int64_t)s.pool.in_use(), (int64_t)s.peak_pool, (int64_t)s.pool.size(),
        (int64_t)(s.busy_s * 1e6), (int64_t)s.waiting.size(), (int64_t)s.admitted.size(),
        (int64_t)s.fatal};
    int cnt = max_stats < TG_SERVER_NUM_STATS ? max_stats : TG_SERVER_NUM_STATS;
    for (int q = 0; q < cnt; ++q) stats[q] = v[q];
    return cnt;
}

tg_status tg_server_destroy(tg_server *h) {
    if (!h) return TG_E_INVALID_ARG;
    tg::Server &s = h->s;
    {
        std::lock_guard<std::mutex> lk(s.mu);
        s.stop = true;
        // finished results become invalid now; their memory lets the
        // remaining requests through
        for (auto &r : s.reqs)
            if (r && r->state == tg::ST_DONE && !r->released && r->block >= 0) {
                s.pool.release(r->block);
                r->block = -1;
                r->released = true;
            }
        s.cv.notify_all();
    }
    for (auto &t : s.threads) t.join();
    tg_status f = s.fatal;
    delete h;
    return f;
}

}  // extern "C"
