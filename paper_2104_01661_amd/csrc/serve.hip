// Continuous-batching query server over a resident set of graphs.
//
// Queries (triangle count, single-source BFS, up-to-8-source betweenness)
// carry a scheduled arrival time on the server clock; a query becomes
// visible to the workers once the clock passes it, so an open-loop arrival
// stream is replayed exactly.  Each worker thread owns a HIP stream and a
// context (its own workspace).  A free worker takes the oldest visible
// query and every other visible query of the same kind on the same graph,
// up to the batch limits:
//   * BFS: up to 64 queries share one multi-source BFS, one wavefront lane
//     per query (the lane-mask frontier of the betweenness kernels);
//   * BC: up to 8 queries of up to 8 sources share one 64-lane batch of
//     Algorithm 3, the dependencies summed per group of 8 lanes;
//   * TC: every visible count on the graph is answered by one count.
// A batch starts only if its working-set estimate fits the memory budget
// next to the batches already running.  A lane's arithmetic does not
// depend on the other lanes, so every result is the same alone and in a
// mix (BC group sums use a fixed reduction tree).
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>

#include "internal.h"

namespace {

__global__ void k_lane_levels(const uint16_t *__restrict__ lev, int64_t n, int k, int64_t *__restrict__ out)
{
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x) {
        const uint16_t x = lev[v * 64 + k];
        out[v] = x == 0xFFFF ? -1 : (int64_t)x;
    }
}

// ------------------------------------------------------ BC group digests

constexpr int DG_BLOCK = 256;
constexpr int DG_TILE = 4096;

// per tile of vertices: sum and max of each of the 8 group columns, in a
// fixed order (a column's result depends on that column alone)
__global__ __launch_bounds__(DG_BLOCK) void k_group_tiles(const double *__restrict__ cent, int64_t n,
                                                          double *__restrict__ psum,
                                                          double *__restrict__ pmax)
{
    __shared__ double ss[8][DG_BLOCK];
    __shared__ double sm[8][DG_BLOCK];
    const int64_t base = (int64_t)blockIdx.x * DG_TILE;
    double s[8], m[8];
    for (int g = 0; g < 8; g++) {
        s[g] = 0.0;
        m[g] = 0.0;
    }
    for (int64_t v = base + threadIdx.x; v < base + DG_TILE && v < n; v += DG_BLOCK)
        for (int g = 0; g < 8; g++) {
            const double x = cent[v * 8 + g];
            s[g] += x;
            m[g] = x > m[g] ? x : m[g];
        }
    for (int g = 0; g < 8; g++) {
        ss[g][threadIdx.x] = s[g];
        sm[g][threadIdx.x] = m[g];
    }
    __syncthreads();
    for (int w = DG_BLOCK / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int g = 0; g < 8; g++) {
                ss[g][threadIdx.x] += ss[g][threadIdx.x + w];
                const double y = sm[g][threadIdx.x + w];
                sm[g][threadIdx.x] = y > sm[g][threadIdx.x] ? y : sm[g][threadIdx.x];
            }
        __syncthreads();
    }
    if (threadIdx.x < 8) {
        psum[blockIdx.x * 8 + threadIdx.x] = ss[threadIdx.x][0];
        pmax[blockIdx.x * 8 + threadIdx.x] = sm[threadIdx.x][0];
    }
}

__global__ void k_group_final(const double *__restrict__ psum, const double *__restrict__ pmax,
                              int64_t tiles, double *__restrict__ out)
{
    const int g = threadIdx.x;
    if (g < 8) {
        double s = 0.0, m = 0.0;
        for (int64_t t = 0; t < tiles; t++) {
            s += psum[t * 8 + g];
            const double y = pmax[t * 8 + g];
            m = y > m ? y : m;
        }
        out[g] = s;
        out[8 + g] = m;
    }
}

__global__ void k_group_col(const double *__restrict__ cent, int64_t n, int g, double *__restrict__ out)
{
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x)
        out[v] = cent[v * 8 + g];
}

}  // namespace

// ============================================================ host side

namespace {

struct Slot {
    lagr_query q;
    int64_t ticket;
};

struct Kept {
    void *p;
    size_t bytes;
    int64_t n;
    lagr_type type;
};

// a context-owned scratch buffer that grows on demand
struct Grow {
    void *p = nullptr;
    size_t bytes = 0;
    void *get(size_t want)
    {
        if (want <= bytes) return p;
        if (p) dev_free(p, bytes);
        p = dev_alloc(want);
        bytes = p ? want : 0;
        return p;
    }
    void release()
    {
        if (p) dev_free(p, bytes);
        p = nullptr;
        bytes = 0;
    }
    ~Grow()
    {
        if (p) dev_free(p, bytes);
    }
};

}  // namespace

struct lagr_server_s {
    std::vector<lagr_graph> graphs;
    int device = 0;
    lagr_server_config cfg{};
    std::chrono::steady_clock::time_point t0;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Slot> pending;
    std::vector<lagr_result> done;
    size_t polled = 0;
    std::unordered_map<int64_t, Kept> kept;
    int64_t kept_bytes = 0;
    int64_t next_ticket = 0;
    int64_t completed = 0;
    // device memory: per worker, what its context and buffers hold between
    // batches (measured after each batch) and the estimate of its running
    // batch (0 when idle); in_use = kept vectors + the sum over workers of
    // the larger of the two
    std::vector<int64_t> held, fp_run;
    std::vector<int64_t> bc_levels;   // per graph: the most BC levels a batch needed
    int64_t in_use = 0, peak = 0, dev_peak = 0;
    int running = 0, running_bc = 0;
    int bc_cap = 1;           // workers that may run betweenness batches at once
    bool trim_all = false;    // idle workers free their workspaces
    bool stop = false;
    int64_t batches[3] = {0, 0, 0}, queries[3] = {0, 0, 0}, rejected = 0;
    std::vector<std::thread> workers;

    double now() const
    {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
};

namespace {

// Device working set of one batch, in bytes (an estimate; the admission
// also counts what each worker measurably holds): for a multi-source BFS
// the unreached masks and two active lists (16n) and two level buffers of
// lane masks and vertex lists (24n), plus, when results are kept, the 64 x
// 16-bit level lanes and one int64 vector per query; for BC the 64-lane
// sigma and W arrays (2 x 512n), one level buffer of 12n per level (8
// levels until a batch on the graph has shown its depth), the unreached
// masks and lists, the 8 group sums, the 64 partial sums of every hub-row
// chunk, and the kept vectors; for a count the work partials.
int64_t footprint(const lagr_server_s *S, int kind, int graph, int nq)
{
    const lagr_graph G = S->graphs[graph];
    const int64_t n = G->A->nrows;
    const bool keep = S->cfg.keep_vectors != 0;
    if (kind == LAGR_QUERY_TC) return 16 * (n + 1);
    if (kind == LAGR_QUERY_BFS) return 40 * n + (keep ? (128 + 8 * (int64_t)nq) * n : 0);
    const int64_t levels = std::max<int64_t>(8, S->bc_levels[graph]);
    const int64_t chunks = G->chunks.n > 0 ? G->chunks.n : 0;
    return (1024 + 12 * levels + 16 + 64) * n + 512 * chunks + (keep ? 8 * (int64_t)nq * n : 0);
}

struct Worker {
    lagr_server_s *S;
    int index = 0;
    int device;
    hipStream_t stream = nullptr;
    lagr_ctx ctx = nullptr;
    Grow lev, cent, digest;
    int64_t retained() const
    {
        return (int64_t)(ctx_retained_bytes(ctx) + lev.bytes + cent.bytes + digest.bytes);
    }
    void trim()
    {
        ctx_trim(ctx);
        lev.release();
        cent.release();
        digest.release();
    }
};

// Memory the server would hold with worker w running a batch of estimate
// fp (under S->mu).
int64_t projected(const lagr_server_s *S, int w, int64_t fp)
{
    int64_t t = S->kept_bytes;
    for (size_t o = 0; o < S->held.size(); o++)
        t += (int)o == w ? std::max(S->held[o], fp) : std::max(S->held[o], S->fp_run[o]);
    return t;
}

// run one batch; fills res (same order as batch)
int run_batch(Worker &W, const std::vector<Slot> &batch, std::vector<lagr_result> &res, char *msg)
{
    lagr_server_s *S = W.S;
    const lagr_query &q0 = batch[0].q;
    const lagr_graph G = S->graphs[q0.graph];
    const int64_t n = G->A->nrows;
    const bool keep = S->cfg.keep_vectors != 0;
    std::vector<std::pair<int64_t, Kept>> kept;
    if (q0.kind == LAGR_QUERY_TC) {
        int64_t t = 0;
        TRY(lagr_tc_adv(&t, G, W.ctx, msg));
        for (auto &r : res) r.triangles = t;
    } else if (q0.kind == LAGR_QUERY_BFS) {
        int64_t src[64];
        for (int k = 0; k < 64; k++) src[k] = k < (int)batch.size() ? batch[k].q.sources[0] : -1;
        uint16_t *lev = nullptr;
        if (keep) {
            lev = (uint16_t *)W.lev.get(2 * 64 * (size_t)(n > 0 ? n : 1));
            if (!lev) return lagr_fail(msg, LAGR_OUT_OF_MEMORY, "level lanes");
        }
        int64_t st[3 * 64];
        TRY(msbfs_compute(W.ctx, G, src, lev, st, msg));
        for (size_t k = 0; k < batch.size(); k++) {
            res[k].reached = st[k];
            res[k].level_sum = st[64 + k];
            res[k].depth = st[128 + k];
            if (keep) {
                Kept kv{dev_alloc(8 * (size_t)(n > 0 ? n : 1)), 8 * (size_t)(n > 0 ? n : 1), n, LAGR_INT64};
                if (!kv.p) return lagr_fail(msg, LAGR_OUT_OF_MEMORY, "result vector");
                hipLaunchKernelGGL(k_lane_levels, dim3(grid_for(n, 256, 4096)), dim3(256), 0, W.ctx->stream,
                                   lev, n, (int)k, (int64_t *)kv.p);
                LAUNCH_CHECK();
                kept.push_back({batch[k].ticket, kv});
            }
        }
    } else {
        int64_t src[64];
        for (int k = 0; k < 64; k++) src[k] = -1;
        for (size_t q = 0; q < batch.size(); q++)
            for (int i = 0; i < batch[q].q.nsources; i++) src[8 * q + i] = batch[q].q.sources[i];
        double *cent = (double *)W.cent.get(8 * 8 * (size_t)(n > 0 ? n : 1));
        const int64_t tiles = (n + DG_TILE - 1) / DG_TILE;
        double *dg = (double *)W.digest.get(8 * (16 * (size_t)(tiles > 0 ? tiles : 1) + 16));
        if (!cent || !dg) return lagr_fail(msg, LAGR_OUT_OF_MEMORY, "bc buffers");
        TRY(bc_compute(W.ctx, G, src, 1, 3, cent, msg));
        double *psum = dg, *pmax = dg + 8 * (tiles > 0 ? tiles : 1), *fin = pmax + 8 * (tiles > 0 ? tiles : 1);
        if (n > 0) {
            hipLaunchKernelGGL(k_group_tiles, dim3((unsigned)tiles), dim3(DG_BLOCK), 0, W.ctx->stream, cent, n,
                               psum, pmax);
            LAUNCH_CHECK();
            hipLaunchKernelGGL(k_group_final, dim3(1), dim3(64), 0, W.ctx->stream, psum, pmax, tiles, fin);
            LAUNCH_CHECK();
        } else {
            TRY(fill_i64(W.ctx, (int64_t *)fin, 16, 0, msg));
        }
        double h[16];
        TRY(read_back(W.ctx, h, fin, sizeof(h), msg));
        for (size_t q = 0; q < batch.size(); q++) {
            res[q].bc_sum = h[q];
            res[q].bc_max = h[8 + q];
            if (keep) {
                Kept kv{dev_alloc(8 * (size_t)(n > 0 ? n : 1)), 8 * (size_t)(n > 0 ? n : 1), n, LAGR_FP64};
                if (!kv.p) return lagr_fail(msg, LAGR_OUT_OF_MEMORY, "result vector");
                hipLaunchKernelGGL(k_group_col, dim3(grid_for(n, 256, 4096)), dim3(256), 0, W.ctx->stream, cent,
                                   n, (int)q, (double *)kv.p);
                LAUNCH_CHECK();
                kept.push_back({batch[q].ticket, kv});
            }
        }
    }
    HIP_TRY(hipStreamSynchronize(W.ctx->stream));
    if (!kept.empty()) {
        std::lock_guard<std::mutex> lk(S->mu);
        for (auto &kv : kept) {
            S->kept[kv.first] = kv.second;
            S->kept_bytes += (int64_t)kv.second.bytes;
        }
    }
    return LAGR_SUCCESS;
}

void worker_main(Worker *W)
{
    lagr_server_s *S = W->S;
    char msg[LAGR_MSG_LEN];
    (void)hipSetDevice(W->device);
    set_thread_native_alloc(true);
    for (;;) {
        std::vector<Slot> batch;
        int64_t fp = 0;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            for (;;) {
                if (S->stop) return;
                if (S->trim_all && S->fp_run[W->index] == 0 && S->held[W->index] > 0) {
                    lk.unlock();
                    W->trim();
                    lk.lock();
                    S->held[W->index] = W->retained();
                    S->in_use = projected(S, -1, 0);
                    S->cv_work.notify_all();
                    continue;
                }
                if (S->trim_all && S->running == 0) {
                    bool all = true;
                    for (int64_t h : S->held) all = all && h == 0;
                    if (all) S->trim_all = false;
                }
                if (S->pending.empty()) {
                    S->cv_work.wait(lk);
                    continue;
                }
                const double t = S->now();
                const Slot &front = S->pending.front();
                if (front.q.arrival > t) {
                    S->cv_work.wait_for(lk, std::chrono::duration<double>(front.q.arrival - t));
                    continue;
                }
                // the oldest visible query and its visible companions; while
                // max_bc_workers workers run betweenness batches, the oldest
                // visible query of another kind instead (BFS and counts take
                // a few milliseconds, a betweenness batch on a large graph
                // tens of them)
                size_t hi = 0;
                if (front.q.kind == LAGR_QUERY_BC && S->running_bc >= S->bc_cap) {
                    hi = S->pending.size();
                    for (size_t i = 1; i < S->pending.size() && S->pending[i].q.arrival <= t; i++)
                        if (S->pending[i].q.kind != LAGR_QUERY_BC) {
                            hi = i;
                            break;
                        }
                    if (hi == S->pending.size()) {
                        S->cv_work.wait(lk);      // a running batch ends first
                        continue;
                    }
                }
                const Slot &head = S->pending[hi];
                const int kind = head.q.kind, graph = head.q.graph;
                const size_t cap = kind == LAGR_QUERY_BFS ? (size_t)S->cfg.max_bfs_batch
                                 : kind == LAGR_QUERY_BC ? (size_t)S->cfg.max_bc_batch
                                                         : (size_t)1 << 30;
                std::vector<size_t> take;
                for (size_t i = hi; i < S->pending.size() && take.size() < cap; i++) {
                    const Slot &s = S->pending[i];
                    if (s.q.arrival > t) break;
                    if (s.q.kind == kind && s.q.graph == graph) take.push_back(i);
                }
                fp = footprint(S, kind, graph, (int)take.size());
                if (fp > S->cfg.budget_bytes) {
                    // larger than the whole budget: refuse these queries
                    for (size_t j = take.size(); j-- > 0;) {
                        lagr_result r{};
                        r.ticket = S->pending[take[j]].ticket;
                        r.kind = kind;
                        r.graph = graph;
                        r.status = LAGR_BUDGET_EXCEEDED;
                        r.arrival = S->pending[take[j]].q.arrival;
                        r.start = r.done = t;
                        S->done.push_back(r);
                        S->pending.erase(S->pending.begin() + (long)take[j]);
                        S->completed++;
                        S->rejected++;
                    }
                    S->cv_done.notify_all();
                    continue;
                }
                // memory: the estimate beside what every worker holds
                if (projected(S, W->index, fp) > S->cfg.budget_bytes) {
                    if (S->running > 0) {
                        S->cv_work.wait(lk);   // admitted again when memory frees up
                        continue;
                    }
                    // nothing runs: the workspaces held from earlier batches
                    // are freed -- this worker's now, the idle workers' when
                    // they wake -- and the batch is looked at again; with
                    // only kept result vectors beside it, it runs
                    if (S->held[W->index] > 0) {
                        lk.unlock();
                        W->trim();
                        lk.lock();
                        S->held[W->index] = W->retained();
                        continue;
                    }
                    bool others = false;
                    for (size_t o = 0; o < S->held.size(); o++) others = others || S->held[o] > 0;
                    if (others) {
                        S->trim_all = true;
                        S->cv_work.notify_all();
                        S->cv_work.wait(lk);
                        continue;
                    }
                }
                for (size_t j = take.size(); j-- > 0;) {
                    batch.push_back(S->pending[take[j]]);
                    S->pending.erase(S->pending.begin() + (long)take[j]);
                }
                std::reverse(batch.begin(), batch.end());
                S->fp_run[W->index] = fp;
                S->in_use = projected(S, -1, 0);
                S->peak = std::max(S->peak, S->in_use);
                S->trim_all = false;
                S->running++;
                if (kind == LAGR_QUERY_BC) S->running_bc++;
                S->batches[kind]++;
                S->queries[kind] += (int64_t)batch.size();
                break;
            }
        }
        std::vector<lagr_result> res(batch.size());
        const double start = S->now();
        for (size_t k = 0; k < batch.size(); k++) {
            res[k] = lagr_result{};
            res[k].ticket = batch[k].ticket;
            res[k].kind = batch[k].q.kind;
            res[k].graph = batch[k].q.graph;
            res[k].arrival = batch[k].q.arrival;
            res[k].start = start;
            res[k].batch_size = (int32_t)batch.size();
        }
        const int rc = run_batch(*W, batch, res, msg);
        const double done = S->now();
        // measured: what this worker now holds, and the device's use
        const int64_t held = W->retained();
        size_t dfree = 0, dtotal = 0;
        const bool have_info = hipMemGetInfo(&dfree, &dtotal) == hipSuccess;
        {
            std::lock_guard<std::mutex> lk(S->mu);
            for (auto &r : res) {
                r.status = rc < 0 ? rc : LAGR_SUCCESS;
                r.done = done;
                S->done.push_back(r);
            }
            S->completed += (int64_t)res.size();
            S->fp_run[W->index] = 0;
            S->held[W->index] = held;
            S->in_use = projected(S, -1, 0);
            if (batch[0].q.kind == LAGR_QUERY_BC && rc >= 0)
                S->bc_levels[batch[0].q.graph] = std::max(S->bc_levels[batch[0].q.graph], W->ctx->last_bc_levels);
            if (have_info) S->dev_peak = std::max(S->dev_peak, (int64_t)(dtotal - dfree));
            S->running--;
            if (batch[0].q.kind == LAGR_QUERY_BC) S->running_bc--;
        }
        S->cv_done.notify_all();
        S->cv_work.notify_all();
    }
}

}  // namespace

// ================================================================= API

extern "C" int lagr_server_new(lagr_server *Sp, const lagr_graph *graphs, int32_t ngraphs,
                               const lagr_server_config *cfg, lagr_ctx ctx, char *msg)
{
    if (!Sp || !graphs || !cfg || !ctx) return lagr_fail(msg, LAGR_NULL_POINTER, "NULL argument");
    *Sp = nullptr;
    if (ngraphs < 1) return lagr_fail(msg, LAGR_INVALID_VALUE, "the server needs at least one graph");
    if (cfg->workers < 1 || cfg->workers > 16 || cfg->max_bfs_batch < 1 || cfg->max_bfs_batch > 64 ||
        cfg->max_bc_batch < 1 || cfg->max_bc_batch > 8 || cfg->budget_bytes <= 0 || cfg->max_bc_workers < 0 ||
        cfg->max_bc_workers > cfg->workers)
        return lagr_fail(msg, LAGR_INVALID_VALUE, "server configuration out of range");
    for (int32_t g = 0; g < ngraphs; g++) {
        if (!graphs[g]) return lagr_fail(msg, LAGR_NULL_POINTER, "graph %d is NULL", g);
        if (graphs[g]->kind != LAGR_ADJACENCY_UNDIRECTED)
            return lagr_fail(msg, LAGR_NOT_IMPLEMENTED, "served graphs must be undirected");
    }
    // every cached property the workers read is built now, on this thread
    for (int32_t g = 0; g < ngraphs; g++) {
        TRY(lagr_property_tc_lower(graphs[g], ctx, msg));
        RowChunks ch;
        TRY(graph_chunks(graphs[g], ctx, &ch, msg));
    }
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    lagr_server_s *S = new (std::nothrow) lagr_server_s();
    if (!S) return lagr_fail(msg, LAGR_OUT_OF_MEMORY, "server");
    S->graphs.assign(graphs, graphs + ngraphs);
    S->device = ctx->device;
    S->cfg = *cfg;
    S->held.assign((size_t)cfg->workers, 0);
    S->bc_levels.assign((size_t)ngraphs, 0);
    S->fp_run.assign((size_t)cfg->workers, 0);
    S->bc_cap = cfg->max_bc_workers > 0 ? cfg->max_bc_workers : std::max(1, cfg->workers - 2);
    S->t0 = std::chrono::steady_clock::now();
    std::vector<Worker *> ws;
    for (int w = 0; w < cfg->workers; w++) {
        Worker *W = new (std::nothrow) Worker();
        if (!W) break;
        W->S = S;
        W->index = w;
        W->device = ctx->device;
        if (hipStreamCreateWithFlags(&W->stream, hipStreamNonBlocking) != hipSuccess ||
            lagr_ctx_new(&W->ctx, ctx->device, W->stream, msg) < 0) {
            delete W;
            break;
        }
        ws.push_back(W);
    }
    if ((int)ws.size() != cfg->workers) {
        for (Worker *W : ws) {
            lagr_ctx_free(&W->ctx);
            (void)hipStreamDestroy(W->stream);
            delete W;
        }
        delete S;
        return lagr_fail(msg, LAGR_OUT_OF_MEMORY, "server workers");
    }
    for (Worker *W : ws) S->workers.emplace_back([W]() {
        worker_main(W);
        // still on the worker thread (native allocation), which took the
        // worker's device memory with hipMalloc
        lagr_ctx_free(&W->ctx);
        (void)hipStreamDestroy(W->stream);
        delete W;
    });
    *Sp = S;
    return lagr_ok(msg);
}

extern "C" int lagr_server_clock(const lagr_server S, double *now, char *msg)
{
    if (!S || !now) return lagr_fail(msg, LAGR_NULL_POINTER, "NULL argument");
    *now = S->now();
    return lagr_ok(msg);
}

extern "C" int lagr_server_submit(lagr_server S, const lagr_query *q, int64_t *ticket, char *msg)
{
    if (!S || !q) return lagr_fail(msg, LAGR_NULL_POINTER, "NULL argument");
    if (q->kind < LAGR_QUERY_TC || q->kind > LAGR_QUERY_BC)
        return lagr_fail(msg, LAGR_INVALID_VALUE, "unknown query kind %d", q->kind);
    if (q->graph < 0 || q->graph >= (int32_t)S->graphs.size())
        return lagr_fail(msg, LAGR_INVALID_INDEX, "graph %d is not resident", q->graph);
    const int64_t n = S->graphs[q->graph]->A->nrows;
    const int need = q->kind == LAGR_QUERY_TC ? 0 : 1;
    const int most = q->kind == LAGR_QUERY_BFS ? 1 : q->kind == LAGR_QUERY_BC ? 8 : 0;
    if (q->nsources < need || q->nsources > most)
        return lagr_fail(msg, LAGR_INVALID_VALUE, "%d sources for a query of kind %d", q->nsources, q->kind);
    for (int i = 0; i < q->nsources; i++)
        if (q->sources[i] < 0 || q->sources[i] >= n)
            return lagr_fail(msg, LAGR_INVALID_INDEX, "source %lld out of range", (long long)q->sources[i]);
    {
        std::lock_guard<std::mutex> lk(S->mu);
        Slot s{*q, S->next_ticket++};
        // keep arrival order (a late-stamped query goes behind earlier ones)
        auto it = S->pending.end();
        while (it != S->pending.begin() && (it - 1)->q.arrival > q->arrival) --it;
        S->pending.insert(it, s);
        if (ticket) *ticket = s.ticket;
    }
    S->cv_work.notify_all();
    return lagr_ok(msg);
}

extern "C" int lagr_server_poll(lagr_server S, lagr_result *out, int32_t max, int32_t *n, char *msg)
{
    if (!S || !n || (max > 0 && !out)) return lagr_fail(msg, LAGR_NULL_POINTER, "NULL argument");
    std::lock_guard<std::mutex> lk(S->mu);
    int32_t k = 0;
    while (k < max && S->polled < S->done.size()) out[k++] = S->done[S->polled++];
    *n = k;
    return lagr_ok(msg);
}

extern "C" int lagr_server_wait(lagr_server S, int64_t n_completed, double timeout_s, char *msg)
{
    if (!S) return lagr_fail(msg, LAGR_NULL_POINTER, "NULL argument");
    std::unique_lock<std::mutex> lk(S->mu);
    const bool ok = S->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s),
                                        [&]() { return S->completed >= n_completed; });
    if (!ok) {
        if (msg) snprintf(msg, LAGR_MSG_LEN, "%lld of %lld queries completed", (long long)S->completed,
                          (long long)n_completed);
        return LAGR_NO_VALUE;
    }
    return lagr_ok(msg);
}

extern "C" int lagr_server_result_vector(lagr_server S, int64_t ticket, lagr_vector *v, lagr_ctx ctx,
                                         char *msg)
{
    if (!S || !v || !ctx) return lagr_fail(msg, LAGR_NULL_POINTER, "NULL argument");
    *v = nullptr;
    Kept kv;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        auto it = S->kept.find(ticket);
        if (it == S->kept.end())
            return lagr_fail(msg, LAGR_INVALID_INDEX, "no kept vector for ticket %lld", (long long)ticket);
        kv = it->second;
        S->kept.erase(it);
        S->kept_bytes -= (int64_t)kv.bytes;
    }
    lagr_vector x = new (std::nothrow) lagr_vector_s();
    void *p = x ? dev_alloc(kv.bytes) : nullptr;
    int rc = LAGR_SUCCESS;
    if (!x || !p) rc = lagr_fail(msg, LAGR_OUT_OF_MEMORY, "result vector");
    else if (hipMemcpyAsync(p, kv.p, kv.bytes, hipMemcpyDeviceToDevice, ctx->stream) != hipSuccess ||
             hipStreamSynchronize(ctx->stream) != hipSuccess)
        rc = lagr_fail(msg, LAGR_DEVICE_ERROR, "result copy");
    set_thread_native_alloc(true);
    dev_free(kv.p, kv.bytes);
    set_thread_native_alloc(false);
    if (rc < 0) {
        if (p) dev_free(p, kv.bytes);
        delete x;
        return rc;
    }
    x->type = kv.type;
    x->n = kv.n;
    x->fmt = LAGR_VEC_FULL;
    x->nvals = kv.n;
    x->values = p;
    x->values_bytes = kv.bytes;
    *v = x;
    return lagr_ok(msg);
}

extern "C" int lagr_server_stats(const lagr_server S, lagr_server_counts *st, char *msg)
{
    if (!S || !st) return lagr_fail(msg, LAGR_NULL_POINTER, "NULL argument");
    std::lock_guard<std::mutex> lk(S->mu);
    st->completed = S->completed;
    for (int k = 0; k < 3; k++) {
        st->batches[k] = S->batches[k];
        st->queries[k] = S->queries[k];
    }
    st->rejected = S->rejected;
    st->peak_bytes = S->peak;
    st->pending = (int64_t)S->pending.size();
    st->device_peak_bytes = S->dev_peak;
    st->held_bytes = S->in_use;
    return lagr_ok(msg);
}

extern "C" int lagr_server_free(lagr_server *Sp)
{
    if (!Sp || !*Sp) return LAGR_SUCCESS;
    lagr_server_s *S = *Sp;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
    }
    S->cv_work.notify_all();
    for (auto &t : S->workers) t.join();
    set_thread_native_alloc(true);
    for (auto &kv : S->kept) dev_free(kv.second.p, kv.second.bytes);
    set_thread_native_alloc(false);
    delete S;
    *Sp = nullptr;
    return LAGR_SUCCESS;
}
