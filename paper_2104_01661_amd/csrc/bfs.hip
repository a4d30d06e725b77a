// Direction-optimising parents BFS (Section IV-A, Algorithms 1 and 2).
//
// One level is q<!s(p), r> = q any.secondi A, fused with p<s(q)> = q (the
// vxm + assign fusion Section VI-B describes for GAP's bfs.cc): the kernel
// that discovers v writes its parent, its level and its bit in the next
// frontier bitmap in the same pass.
//   push: a wavefront per frontier vertex u scans N(u) with coalesced loads
//         (hub rows, longer than GRAPH_LONG_ROW, chunk by chunk);
//   pull: one lane per unvisited vertex v scans its in-neighbours (row v
//         of AT; of A itself for an undirected graph) in ascending order
//         and stops at the first one in the frontier bitmap.
// A compaction pass then lists the next frontier, counts it and its degree
// sum and adds it to the visited set.  The level loop runs on the device:
// a one-thread kernel folds the counters into the level state and picks
// the next level's direction, and every kernel of a level returns at once
// when the search is done.  Two levels (the two
// buffer parities) are captured once into a hipGraph per context and
// replayed; the host looks at the done flag only every few levels.
#include "internal.h"

namespace {

constexpr int BFS_ALPHA = 14;
constexpr int BFS_BETA = 24;
constexpr unsigned BFS_EXPAND_MAX = 2048;   // expansion workgroups at most

__device__ __forceinline__ bool bit_test(const uint32_t *bm, int64_t v)
{
    return (bm[v >> 5] >> (v & 31)) & 1u;
}

}  // namespace

// Everything a level needs, in device memory: the kernels of a level take
// only this struct's address and the buffer parity, so one captured
// hipGraph of two levels serves every call (the host refreshes the
// struct before each search).  Buffers [par] hold the current frontier,
// [par ^ 1] the next one.
struct BfsDev {
    const int64_t *rp;        // out-edges (push)
    const int32_t *ci;
    const int64_t *rpT;       // in-edges (pull): AT, or A when undirected
    const int32_t *ciT;
    int64_t n, W;
    int32_t *level;
    unsigned long long *parent;
    uint32_t *visited;
    uint32_t *bm[2];
    int32_t *list[2];
    RowChunks ch;
    int32_t any_parent, push_only;
    // level state: lev, direction, termination, frontier size / degree sum,
    // unexplored degree sum, and the compaction counters of the last level
    int32_t lev, pull, done, pad_;
    int32_t *done_host;       // pinned host word set when the search ends
    // a pull level's new frontier per expansion workgroup: size in blk[g],
    // degree sum in blk[BFS_EXPAND_MAX + g], for the eg workgroups
    unsigned long long *blk;
    int64_t eg;
    int64_t nq, mf, mu;
    unsigned long long nnext, enext;
};

namespace {


// Start of a level: fold the last compaction's counters into the state,
// stop when the frontier is empty, and pick the direction (Beamer, Asanovic
// and Patterson, SC 2012, the heuristic the paper cites): pull when the
// frontier's edges exceed the unexplored edges / BFS_ALPHA, back to push
// when the frontier has fewer than n / BFS_BETA vertices.  One thread runs
// it: in the start kernel for the first level, then in a one-thread kernel
// after each compaction.  (Folding it into the compaction's last workgroup
// by a ticket counter measured no faster than the separate node.)
__device__ void bfs_decide(BfsDev *d)
{
    const int64_t nq = (int64_t)d->nnext, mf = (int64_t)d->enext;
    d->nq = nq;
    d->mf = mf;
    d->mu -= mf;
    d->lev += 1;
    if (nq == 0 || d->lev == INT32_MAX) {
        d->done = 1;
        __hip_atomic_store(d->done_host, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        __threadfence_system();
        return;
    }
    if (!d->push_only) {
        if (!d->pull && mf > d->mu / BFS_ALPHA) d->pull = 1;
        else if (d->pull && nq < d->n / BFS_BETA) d->pull = 0;
    }
    d->nnext = 0;
    d->enext = 0;
}

// The per-search start in one launch: the level state from the kernel
// argument h into d, levels and parents to -1 and the three bitmaps
// (visited, two frontiers) to 0, except the source's entries; then the
// first level's decision, with the source as the frontier.
__global__ void k_bfs_start(BfsDev h, BfsDev *d, int32_t *__restrict__ level, int64_t *__restrict__ parent,
                            int64_t n, uint32_t *__restrict__ bms, int64_t W, int64_t src)
{
    const int64_t step = (int64_t)gridDim.x * blockDim.x;
    const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int64_t i = t0; i < n; i += step) {
        level[i] = i == src ? 0 : -1;
        parent[i] = i == src ? src : -1;
    }
    const int64_t sw = src >> 5;
    const uint32_t sbit = 1u << (src & 31);
    for (int64_t i = t0; i < 3 * W; i += step) bms[i] = (i == sw || i == W + sw) ? sbit : 0u;
    if (t0 == 0) {
        *d = h;
        d->list[0][0] = (int32_t)src;
        d->nnext = 1;
        d->enext = (unsigned long long)(d->rp[src + 1] - d->rp[src]);
        bfs_decide(d);
    }
}

// Push the neighbours rp-range [b, e) of frontier vertex u, one per lane.
__device__ __forceinline__ void push_range(const BfsDev &d, int32_t u, int64_t b, int64_t e, unsigned lane,
                                           int32_t lev, uint32_t *__restrict__ next_bm)
{
    for (int64_t p = b + lane; p < e; p += 64) {
        const int32_t v = d.ci[p];
        if (bit_test(d.visited, v)) continue;
        const int32_t old = atomicCAS(&d.level[v], -1, lev);
        if (old == -1) {
            if (d.any_parent) d.parent[v] = (unsigned long long)u;
            else atomicMin(&d.parent[v], (unsigned long long)u);
            atomicOr(&next_bm[v >> 5], 1u << (v & 31));
        } else if (old == lev && !d.any_parent) {
            atomicMin(&d.parent[v], (unsigned long long)u);
        }
    }
}

// Push: a wavefront per frontier vertex u (rows of at most GRAPH_LONG_ROW)
// scans N(u) with coalesced loads; a vertex is claimed by a 32-bit CAS on
// its level.  The parent is the smallest frontier neighbour (atomicMin on
// the unsigned parent, whose "absent" value -1 is the largest), or, with
// LAGR_BFS_ANY_PARENT, the CAS winner.
__device__ __forceinline__ void bfs_push(const BfsDev &d, int par)
{
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / 64;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / 64;
    const unsigned lane = lane_id();
    const int32_t lev = d.lev;
    const int32_t *frontier = d.list[par];
    uint32_t *next_bm = d.bm[par ^ 1];
    for (int64_t f = wave; f < d.nq; f += nw) {
        const int32_t u = frontier[f];
        const int64_t b = d.rp[u], e = d.rp[u + 1];
        if (e - b > GRAPH_LONG_ROW) continue;   // bfs_push_chunks
        push_range(d, u, b, e, lane, lev, next_bm);
    }
}

// The frontier's hub vertices: every chunk of a long row whose vertex is in
// the frontier bitmap is pushed by a whole wave.
__device__ __forceinline__ void bfs_push_chunks(const BfsDev &d, int par)
{
    const unsigned lane = lane_id();
    const int32_t lev = d.lev;
    uint32_t *next_bm = d.bm[par ^ 1];
    for_marked_chunks(d.ch, d.bm[par], [&](int32_t u, int64_t b, int64_t e) {
        push_range(d, u, b, e, lane, lev, next_bm);
    });
}

// Pull: one lane per unvisited vertex scans its in-neighbours (row v of AT)
// in ascending order and stops at the first one in the frontier bitmap,
// the smallest valid parent.  Neighbours are taken PULL_BATCH at a time (independent
// loads, then independent bitmap probes) so a lane waits for two round
// trips per batch rather than two per neighbour.
constexpr int PULL_BATCH = 8;

__device__ __forceinline__ void bfs_pull(const BfsDev &d, int par)
{
    const int64_t n = d.n;
    const int32_t lev = d.lev;
    const uint32_t *cur_bm = d.bm[par];
    uint32_t *next_bm = d.bm[par ^ 1];
    int64_t *parent = (int64_t *)d.parent;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    __shared__ unsigned long long s_cnt, s_deg;
    if (threadIdx.x == 0) {
        s_cnt = 0;
        s_deg = 0;
    }
    __syncthreads();
    unsigned long long cnt = 0, deg = 0;
    // every lane runs the same trip count, so the ballot sees the whole wave
    for (int64_t v0 = (int64_t)blockIdx.x * blockDim.x; v0 < n; v0 += stride) {
        const int64_t v = v0 + threadIdx.x;
        int32_t par_v = -1;
        if (v < n && !bit_test(d.visited, v)) {
            const int64_t b = d.rpT[v], e = d.rpT[v + 1];
            for (int64_t p0 = b; p0 < e && par_v < 0; p0 += PULL_BATCH) {
                int32_t u[PULL_BATCH];
#pragma unroll
                for (int t = 0; t < PULL_BATCH; t++) u[t] = p0 + t < e ? d.ciT[p0 + t] : -1;
#pragma unroll
                for (int t = PULL_BATCH - 1; t >= 0; t--)
                    if (u[t] >= 0 && bit_test(cur_bm, u[t])) par_v = u[t];
            }
        }
        if (par_v >= 0) {
            parent[v] = par_v;
            d.level[v] = lev;
            cnt += 1;
            deg += (unsigned long long)(d.rp[v + 1] - d.rp[v]);
        }
        // the wave's 64 vertices are 64-aligned: they own two bitmap words,
        // which no other wave writes or reads in this kernel.  Every word of
        // the next bitmap is written (so it needs no clearing), and the new
        // vertices join the visited set here.
        const uint64_t m = __ballot(par_v >= 0);
        const unsigned lane = lane_id();
        const int64_t w0 = (v - lane) >> 5;
        if ((lane == 0 || lane == 32) && w0 + (lane >> 5) < d.W) {
            const int64_t w = w0 + (lane >> 5);
            const uint32_t x = (uint32_t)(m >> lane);
            next_bm[w] = x;
            if (x) d.visited[w] |= x;
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        cnt += __shfl_xor(cnt, o, 64);
        deg += __shfl_xor(deg, o, 64);
    }
    if (lane_id() == 0 && cnt) {
        atomicAdd(&s_cnt, cnt);
        atomicAdd(&s_deg, deg);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        d.blk[blockIdx.x] = s_cnt;
        d.blk[BFS_EXPAND_MAX + blockIdx.x] = s_deg;
    }
}

// The level's expansion in one launch (2048 workgroups at most: all of
// them resident at once, and a level past the end dispatches half as many
// as a grid of one thread per vertex): pull, or push over the frontier
// list and then over the hub chunks marked in the frontier bitmap.  One
// kernel node per level instead of three: a node whose work the direction
// skips still costs its dispatch (a few microseconds at thousands of
// workgroups).
__global__ __launch_bounds__(256) void k_bfs_expand(BfsDev *dp, int par)
{
    const BfsDev &d = *dp;
    if (d.done) return;
    if (d.pull) {
        bfs_pull(d, par);
    } else {
        bfs_push(d, par);
        bfs_push_chunks(d, par);
    }
}

__global__ void k_bfs_decide(BfsDev *d)
{
    if (threadIdx.x == 0 && !d->done) bfs_decide(d);
}

// End of a level: the next frontier from its bitmap, a thread per 32-bit
// word.  Each workgroup scans its words' popcounts, reserves its range of
// the list with one atomic (atomics on one address from every wavefront
// would serialise), writes its vertices in ascending order, adds its
// degree sum with one more atomic, ORs its words into the visited set and
// clears the words of the consumed frontier bitmap.
__global__ __launch_bounds__(256) void k_bfs_compact(BfsDev *dp, int par)
{
    const BfsDev &d = *dp;
    if (d.done) return;
    __shared__ unsigned scan[256];
    __shared__ unsigned long long base_s, deg_s, nq_s;
    if (d.pull) {
        // After a pull level: its workgroups counted the new frontier.  When
        // the next level pulls again (the test of bfs_decide), it needs
        // neither the list nor a cleared bitmap: skip the pass.
        unsigned long long c = 0, g = 0;
        for (int64_t b = threadIdx.x; b < d.eg; b += blockDim.x) {
            c += d.blk[b];
            g += d.blk[BFS_EXPAND_MAX + b];
        }
        for (int o = 32; o > 0; o >>= 1) {
            c += __shfl_xor(c, o, 64);
            g += __shfl_xor(g, o, 64);
        }
        if (threadIdx.x == 0) {
            nq_s = 0;
            deg_s = 0;
        }
        __syncthreads();
        if (lane_id() == 0 && c) {
            atomicAdd(&nq_s, c);
            atomicAdd(&deg_s, g);
        }
        __syncthreads();
        const int64_t nq = (int64_t)nq_s;
        if (nq > 0 && nq >= d.n / BFS_BETA) {
            if (blockIdx.x == 0 && threadIdx.x == 0) {
                dp->nnext = nq_s;
                dp->enext = deg_s;
            }
            return;
        }
        __syncthreads();
    }
    const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t *next_bm = d.bm[par ^ 1];
    int32_t *next_list = d.list[par ^ 1];
    const uint32_t x = w < d.W ? next_bm[w] : 0u;
    if (w < d.W) d.bm[par][w] = 0u;
    if (x) d.visited[w] |= x;
    const unsigned c = (unsigned)__popc(x);
    unsigned long long deg = 0;
    for (uint32_t y = x; y; y &= y - 1) {
        const int64_t v = w * 32 + __ffs(y) - 1;
        deg += (unsigned long long)(d.rp[v + 1] - d.rp[v]);
    }
    scan[threadIdx.x] = c;
    if (threadIdx.x == 0) deg_s = 0;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
        const unsigned y = (int)threadIdx.x >= o ? scan[threadIdx.x - o] : 0u;
        __syncthreads();
        scan[threadIdx.x] += y;
        __syncthreads();
    }
    for (int o = 32; o > 0; o >>= 1) deg += __shfl_xor(deg, o, 64);
    if (lane_id() == 0 && deg) atomicAdd(&deg_s, deg);
    if (threadIdx.x == 255) base_s = scan[255] ? atomicAdd(&dp->nnext, (unsigned long long)scan[255]) : 0;
    __syncthreads();
    if (threadIdx.x == 0 && deg_s) atomicAdd(&dp->enext, deg_s);
    unsigned long long pos = base_s + scan[threadIdx.x] - c;
    for (uint32_t y = x; y; y &= y - 1) next_list[pos++] = (int32_t)(w * 32 + __ffs(y) - 1);
}

__global__ void k_level_to_i64(const int32_t *__restrict__ in, int64_t *__restrict__ out, int64_t n)
{
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x)
        out[v] = in[v];
}

// One level on stream s with buffer parity par.
int enqueue_level(BfsDev *d, int par, int64_t n, int64_t W, hipStream_t s, char *msg)
{
    hipLaunchKernelGGL(k_bfs_expand, dim3(grid_for(n, 256, BFS_EXPAND_MAX)), dim3(256), 0, s, d, par);
    hipLaunchKernelGGL(k_bfs_compact, dim3(grid_for(W, 256, 1 << 30)), dim3(256), 0, s, d, par);
    hipLaunchKernelGGL(k_bfs_decide, dim3(1), dim3(64), 0, s, d);
    LAUNCH_CHECK();
    return LAGR_SUCCESS;
}

}  // namespace

// The context's captured two-level graph for graphs of n vertices.
static int bfs_graph(lagr_ctx ctx, BfsDev *d, int64_t n, int64_t W, hipGraphExec_t *exec, char *msg)
{
    if (ctx->bfs_exec && ctx->bfs_key == n && ctx->bfs_state == (void *)d) {
        *exec = ctx->bfs_exec;
        return LAGR_SUCCESS;
    }
    if (ctx->bfs_exec) (void)hipGraphExecDestroy(ctx->bfs_exec);
    ctx->bfs_exec = nullptr;
    if (!ctx->capture_stream) HIP_TRY(hipStreamCreateWithFlags(&ctx->capture_stream, hipStreamNonBlocking));
    HIP_TRY(hipStreamBeginCapture(ctx->capture_stream, hipStreamCaptureModeThreadLocal));
    int rc = enqueue_level(d, 0, n, W, ctx->capture_stream, msg);
    if (rc >= 0) rc = enqueue_level(d, 1, n, W, ctx->capture_stream, msg);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(ctx->capture_stream, &g);
    if (rc < 0 || e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return rc < 0 ? rc : lagr_fail(msg, LAGR_DEVICE_ERROR, "bfs capture: %s", hipGetErrorString(e));
    }
    const hipError_t ei = hipGraphInstantiate(&ctx->bfs_exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ei != hipSuccess) {
        ctx->bfs_exec = nullptr;
        return lagr_fail(msg, LAGR_DEVICE_ERROR, "bfs graph: %s", hipGetErrorString(ei));
    }
    ctx->bfs_key = n;
    ctx->bfs_state = (void *)d;
    *exec = ctx->bfs_exec;
    return LAGR_SUCCESS;
}

static int new_full_i64(lagr_vector *out, int64_t n, int64_t **values, char *msg)
{
    lagr_vector v = new (std::nothrow) lagr_vector_s();
    if (!v) return lagr_fail(msg, LAGR_OUT_OF_MEMORY, "vector");
    v->type = LAGR_INT64;
    v->n = n;
    v->fmt = LAGR_VEC_FULL;
    v->nvals = n;
    v->values_bytes = sizeof(int64_t) * (size_t)(n > 0 ? n : 1);
    v->values = dev_alloc(v->values_bytes);
    if (!v->values) {
        delete v;
        return lagr_fail(msg, LAGR_OUT_OF_MEMORY, "vector values");
    }
    *values = (int64_t *)v->values;
    *out = v;
    return LAGR_SUCCESS;
}

extern "C" int lagr_bfs(lagr_vector *level_out, lagr_vector *parent_out, const lagr_graph G,
                        int64_t source, uint32_t flags, lagr_ctx ctx, char *msg)
{
    if (!G || !ctx) return lagr_fail(msg, LAGR_NULL_POINTER, "NULL argument");
    if (level_out) *level_out = nullptr;
    if (parent_out) *parent_out = nullptr;
    const lagr_matrix A = G->A;
    const int64_t n = A->nrows;
    if (source < 0 || source >= n)
        return lagr_fail(msg, LAGR_INVALID_INDEX, "source %lld out of range", (long long)source);
    // pull steps read in-edges: a directed graph needs its transpose
    if (!(flags & LAGR_BFS_PUSH_ONLY)) TRY(graph_ensure_at(G, ctx, msg));
    const lagr_matrix AT = (flags & LAGR_BFS_PUSH_ONLY) ? A : graph_in_edges(G);
    const int64_t W = (n + 31) / 32;
    int32_t *lev32 = (int32_t *)ws_get(ctx, WS_BFS_A, sizeof(int32_t) * n);
    int32_t *lists = (int32_t *)ws_get(ctx, WS_BFS_B, sizeof(int32_t) * 2 * n);
    // three bitmaps, then the pull levels' per-workgroup counters
    const size_t bm_bytes = (sizeof(uint32_t) * 3 * W + 255) & ~(size_t)255;
    uint32_t *bms = (uint32_t *)ws_get(ctx, WS_BFS_C, bm_bytes + sizeof(unsigned long long) * 2 * BFS_EXPAND_MAX);
    BfsDev *d = (BfsDev *)ws_get(ctx, WS_BFS_D, sizeof(BfsDev));
    int64_t *parent_scratch = nullptr;
    if (!parent_out) parent_scratch = (int64_t *)ws_get(ctx, WS_BFS_E, sizeof(int64_t) * n);
    if (!lev32 || !lists || !bms || !d || (!parent_out && !parent_scratch))
        return lagr_fail(msg, LAGR_OUT_OF_MEMORY, "bfs workspace");
    RowChunks ch;
    TRY(graph_chunks(G, ctx, &ch, msg));
    lagr_vector pv = nullptr, lv = nullptr;
    int64_t *parent = parent_scratch;
    if (parent_out) TRY(new_full_i64(&pv, n, &parent, msg));

    int rc = LAGR_SUCCESS;
    auto cleanup = [&]() {
        if (pv) lagr_vector_free(&pv);
        if (lv) lagr_vector_free(&lv);
    };
#define BFS_TRY(expr)            \
    do {                         \
        rc = (expr);             \
        if (rc < 0) {            \
            cleanup();           \
            return rc;           \
        }                        \
    } while (0)

    // the level state goes to the device as the start kernel's argument
    BfsDev h{};
    h.rp = A->rowptr;
    h.ci = A->colidx;
    h.rpT = AT->rowptr;
    h.ciT = AT->colidx;
    h.n = n;
    h.W = W;
    h.level = lev32;
    h.parent = (unsigned long long *)parent;
    h.visited = bms;
    h.bm[0] = bms + W;
    h.bm[1] = bms + 2 * W;
    h.list[0] = lists;
    h.list[1] = lists + n;
    h.ch = ch;
    h.blk = (unsigned long long *)((char *)bms + bm_bytes);
    h.eg = grid_for(n, 256, BFS_EXPAND_MAX);
    h.any_parent = (flags & LAGR_BFS_ANY_PARENT) ? 1 : 0;
    h.push_only = (flags & LAGR_BFS_PUSH_ONLY) ? 1 : 0;
    h.lev = 0;
    h.mu = A->nvals;
    // the decision kernel stores 1 to this pinned word when the search
    // ends; the host clears it first (nothing else writes it: the last
    // search on this context drained before it returned)
    volatile int32_t *done_flag = (volatile int32_t *)((char *)ctx->pinned + LAGR_PINNED_STAGE);
    h.done_host = (int32_t *)((char *)ctx->pinned_dev + LAGR_PINNED_STAGE);
    *done_flag = 0;
    static_assert(sizeof(BfsDev) <= 1024, "BfsDev is passed as a kernel argument");
    hipLaunchKernelGGL(k_bfs_start, dim3(grid_for(n, 256, 4096)), dim3(256), 0, ctx->stream, h, d, lev32, parent,
                       n, bms, W, source);
    if (hipGetLastError() != hipSuccess) BFS_TRY(lagr_fail(msg, LAGR_DEVICE_ERROR, "bfs start launch"));
    hipGraphExec_t exec = nullptr;
    BFS_TRY(bfs_graph(ctx, d, n, W, &exec, msg));
    // replay two levels at a time; look at the done flag after 8 levels and
    // then after every 4 (each look is a host round trip; a level past the
    // end costs only kernels that return at once).  An R-MAT graph of 2^20
    // vertices is 5 to 6 levels deep, which the search finishes in 7 to 8
    // steps: one look.
    int64_t levels = 0;
    for (int64_t replays = 4;; replays = 2) {
        for (int64_t r = 0; r < replays; r++)
            if (hipGraphLaunch(exec, ctx->stream) != hipSuccess)
                BFS_TRY(lagr_fail(msg, LAGR_DEVICE_ERROR, "bfs graph launch"));
        levels += 2 * replays;
        BFS_TRY(host_wait(ctx, msg));
        if (*done_flag) break;
        if (levels > n + 2) BFS_TRY(lagr_fail(msg, LAGR_DEVICE_ERROR, "bfs did not terminate"));
    }
    if (level_out) {
        int64_t *lvals = nullptr;
        BFS_TRY(new_full_i64(&lv, n, &lvals, msg));
        hipLaunchKernelGGL(k_level_to_i64, dim3(grid_for(n, 256, 8192)), dim3(256), 0, ctx->stream,
                           lev32, lvals, n);
        if (hipGetLastError() != hipSuccess) BFS_TRY(lagr_fail(msg, LAGR_DEVICE_ERROR, "bfs level export"));
        *level_out = lv;
        lv = nullptr;
    }
    if (parent_out) {
        *parent_out = pv;
        pv = nullptr;
    }
#undef BFS_TRY
    return lagr_ok(msg);
}
