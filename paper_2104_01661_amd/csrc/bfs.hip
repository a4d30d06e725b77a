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
// The frontier is a bitmap.  A push writes no returning atomic: every lane
// that finds an unvisited neighbour v stores v's level (the same value from
// every finder), lowers v's parent with atomicMin and sets v's bit, so a
// push step waits for two memory round trips (the neighbour ids, then the
// visited and frontier words) instead of four.
//
// A level is ONE kernel.  Its workgroups first read the counters the
// previous levels left and each takes the level's decisions itself -- stop
// when the frontier is empty, push or pull by Beamer's test -- from the
// same inputs, so they agree without synchronising; workgroup 0 records the
// level state for the next kernel.  Rotating bitmaps replace the compaction
// and decision passes of a three-kernel level: level k reads frontier slot
// k mod 3, writes slot k+1 and clears slot k+2, and the visited set takes
// F_k in at the end of level k (level k tests "visited or in F_k").  The
// levels are nodes of a hipGraph built once per context; the host watches
// pinned words that the kernels store and queues further levels only when
// the first ones did not finish the search.
#include <algorithm>
#include <atomic>
#include <chrono>

#include "internal.h"

namespace {

constexpr unsigned BFS_GRID = 2048;        // workgroups of a level kernel
constexpr int BFS_SPREAD = 16;             // vertex, degree and hub counters
constexpr int BFS_NCTR = 3 * BFS_SPREAD;
constexpr int BFS_CTR_STRIDE = 16;         // 128 bytes between counters

__device__ __forceinline__ bool bit_test(const uint32_t *bm, int64_t v)
{
    return (bm[v >> 5] >> (v & 31)) & 1u;
}

}  // namespace

// The state of one level: k (the frontier F_k being expanded), its
// direction, the frontier's size, degree sum and hub rows, the edges not
// yet explored, and the search's running counter totals at its start.
struct BfsLevel {
    int32_t lev, pull, done, pad_;
    int64_t mu, nq, mf, nhub;
    unsigned long long cnt_tot, deg_tot, hub_tot;
};

// Everything a level needs, in device memory (the start node copies the
// search's arguments in).
//
// The counters only grow during a search: every level adds the vertices it
// finds, their degrees and the number of them whose rows are hub rows
// (longer than GRAPH_LONG_ROW, pushed chunk by chunk).  A level's frontier
// is the difference between the totals at its start and at the previous
// level's start, so no counter is reset between levels.  A pull finds each
// vertex once; a push counts every (frontier vertex, new neighbour) pair,
// so its count and degree sum may include a vertex more than once.  They
// steer only the direction choice, and a count is zero exactly when the
// level found nothing.
struct BfsDev {
    const int64_t *rp;        // out-edges (push)
    const int32_t *ci;
    const int64_t *rpT;       // in-edges (pull): AT, or A when undirected
    const int32_t *ciT;
    const int64_t *deg;       // out-degrees (the cached row-degree property)
    int64_t n, W;
    int32_t *level;
    unsigned long long *parent;
    uint32_t *visited;
    uint32_t *bm[3];          // F_k in bm[k % 3]
    unsigned long long *ctr;  // BFS_NCTR counters, BFS_CTR_STRIDE words apart
    RowChunks ch;
    int32_t any_parent, push_only;
    int32_t alpha, beta;      // direction thresholds
    int64_t src;
    int32_t *done_host;       // pinned host word set when the search ends
    int32_t *level_host;      // pinned host word: the last level started
    BfsLevel st[2];           // level k's state in st[k & 1]
};

namespace {

// Level k's state from level k-1's and the counters (Beamer, Asanovic and
// Patterson, SC 2012, the heuristic the paper cites): pull when the
// frontier's edges exceed the unexplored edges / alpha, back to push when
// the frontier has fewer than n / beta vertices (14 and 24 by default, the
// graph's tuned values after lagr_bfs_autotune).  Every workgroup
// of level k evaluates it from the same inputs.  Wave 0 of the workgroup
// calls it with the previous state and the counters (both loaded at once);
// the result goes to *ns.
__device__ void bfs_level_state(const BfsLevel *__restrict__ psp, const unsigned long long *__restrict__ ctr,
                                int64_t n, int push_only, int alpha, int beta, BfsLevel *ns)
{
    const unsigned lane = lane_id();
    // lanes 0..15: vertex counts; 16..31: degree sums; 32..47: hub counts
    const unsigned long long v = lane < BFS_NCTR ? ctr[(size_t)lane * BFS_CTR_STRIDE] : 0ull;
    const BfsLevel ps = *psp;
    const unsigned long long cnt = wave_sum64(lane < BFS_SPREAD ? v : 0ull);
    const unsigned long long deg = wave_sum64((lane >= BFS_SPREAD && lane < 2 * BFS_SPREAD) ? v : 0ull);
    const unsigned long long hub = wave_sum64((lane >= 2 * BFS_SPREAD && lane < BFS_NCTR) ? v : 0ull);
    if (lane != 0) return;
    if (ps.done) {
        ns->done = 2;   // finished before this level
        return;
    }
    const int k = ps.lev + 1;
    ns->lev = k;
    ns->cnt_tot = cnt;
    ns->deg_tot = deg;
    ns->hub_tot = hub;
    ns->nq = (int64_t)(cnt - ps.cnt_tot);
    ns->mf = (int64_t)(deg - ps.deg_tot);
    ns->nhub = (int64_t)(hub - ps.hub_tot);
    ns->mu = ps.mu - ns->mf;
    ns->done = (ns->nq == 0 || k >= INT32_MAX - 1) ? 1 : 0;
    int pull = ps.pull;
    if (!push_only) {
        if (!pull && ns->mf > ns->mu / alpha) pull = 1;
        else if (pull && ns->nq < n / beta) pull = 0;
    }
    ns->pull = pull;
}

// The arguments of a level kept in registers (loaded once at the kernel's
// start, beside the state).
struct LevelArgs {
    const int64_t *rp, *rpT, *deg;
    const int32_t *ci, *ciT;
    int64_t n, W;
    int32_t *level;
    unsigned long long *parent;
    uint32_t *visited;
    uint32_t *bm0, *bm1, *bm2;
    RowChunks ch;
    int any_parent, push_only;
};

// Push the neighbours rp-range [b, e) of frontier vertex u, up to four per
// lane at a time: every neighbour in neither the visited set nor F_k gets
// its level and its bit in the next frontier, and the parent u unless it
// already has a smaller one (atomicMin on the unsigned parent, whose
// "absent" value -1 is the largest); with LAGR_BFS_ANY_PARENT the parent is
// whichever finder stores last.  The new neighbours' degrees, loaded beside
// these stores, are added while the next step's loads are in flight.
constexpr int PUSH_DEPTH = 4;

__device__ __forceinline__ void push_range(const LevelArgs &a, const uint32_t *__restrict__ cur,
                                           uint32_t *__restrict__ next, int32_t u, int64_t b, int64_t e,
                                           unsigned lane, int32_t lev, unsigned long long &cnt,
                                           unsigned long long &deg, unsigned long long &hub)
{
    int64_t pend[PUSH_DEPTH] = {0, 0, 0, 0};
    for (int64_t p0 = b; p0 < e; p0 += 64 * PUSH_DEPTH) {
        int32_t v[PUSH_DEPTH];
#pragma unroll
        for (int t = 0; t < PUSH_DEPTH; t++) {
            const int64_t p = p0 + 64 * t + lane;
            v[t] = p < e ? a.ci[p] : -1;
        }
        // the previous step's degrees (their loads were issued before this
        // step's ids)
#pragma unroll
        for (int t = 0; t < PUSH_DEPTH; t++) {
            deg += (unsigned long long)pend[t];
            hub += pend[t] > GRAPH_LONG_ROW ? 1ull : 0ull;
            pend[t] = 0;
        }
        uint32_t vis[PUSH_DEPTH], cw[PUSH_DEPTH];
#pragma unroll
        for (int t = 0; t < PUSH_DEPTH; t++) {
            vis[t] = v[t] >= 0 ? a.visited[v[t] >> 5] : ~0u;
            cw[t] = v[t] >= 0 ? cur[v[t] >> 5] : ~0u;
        }
#pragma unroll
        for (int t = 0; t < PUSH_DEPTH; t++) {
            if (v[t] >= 0 && !(((vis[t] | cw[t]) >> (v[t] & 31)) & 1u)) {
                a.level[v[t]] = lev;
                if (a.any_parent) a.parent[v[t]] = (unsigned long long)u;
                else atomicMin(&a.parent[v[t]], (unsigned long long)u);
                atomicOr(&next[v[t] >> 5], 1u << (v[t] & 31));
                pend[t] = a.deg[v[t]];
                cnt += 1;
            }
        }
    }
#pragma unroll
    for (int t = 0; t < PUSH_DEPTH; t++) {
        deg += (unsigned long long)pend[t];
        hub += pend[t] > GRAPH_LONG_ROW ? 1ull : 0ull;
    }
}

// The frontier's hub rows: the chunks of rows longer than GRAPH_LONG_ROW
// whose vertex is in bitmap bm, each split in CHUNK_SPLIT pieces so that
// more wavefronts share a hub (as for_marked_chunks, with virtual chunk c
// = piece c % CHUNK_SPLIT of chunk c / CHUNK_SPLIT).
constexpr int CHUNK_SPLIT = 2;

template <typename Body>
__device__ __forceinline__ void for_marked_pieces(const RowChunks &ch, const uint32_t *__restrict__ bm, Body body)
{
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / 64;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / 64;
    const unsigned lane = lane_id();
    const int64_t nv = ch.n * CHUNK_SPLIT;
    for (int64_t k0 = 0; wave + k0 * nw < nv; k0 += 64) {
        const int64_t c = wave + (k0 + lane) * nw;
        bool hit = false;
        if (c < nv) {
            const int32_t u = ch.row[c / CHUNK_SPLIT];
            hit = (bm[u >> 5] >> (u & 31)) & 1u;
        }
        for (uint64_t m = __ballot(hit); m; m &= m - 1) {
            const int64_t cc = wave + (k0 + (int64_t)__ffsll((unsigned long long)m) - 1) * nw;
            const int64_t r = cc / CHUNK_SPLIT, q = cc % CHUNK_SPLIT;
            const int64_t b = ch.beg[r], e = ch.end[r];
            const int64_t len = e - b, piece = (len + CHUNK_SPLIT - 1) / CHUNK_SPLIT;
            const int64_t pb = b + q * piece, pe = pb + piece < e ? pb + piece : e;
            if (pb < pe) body(ch.row[r], pb, pe);
        }
    }
}

// The frontier's other vertices: vertex v belongs to wavefront v mod nw
// (lane l of wave w tests vertices w + (l + 64 j) nw), so that a run of
// consecutive frontier vertices spreads over many wavefronts; body(u)
// runs with the whole wave for each vertex in the bitmap.
template <typename Body>
__device__ __forceinline__ void for_marked_vertices(const uint32_t *__restrict__ bm, int64_t n, Body body)
{
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / 64;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / 64;
    const unsigned lane = lane_id();
    for (int64_t k0 = 0; wave + k0 * nw < n; k0 += 64) {
        const int64_t v = wave + (k0 + lane) * nw;
        const bool hit = v < n && bit_test(bm, v);
        for (uint64_t m = __ballot(hit); m; m &= m - 1)
            body((int32_t)(wave + (k0 + (int64_t)__ffsll((unsigned long long)m) - 1) * nw));
    }
}

// Pull: one lane per unvisited vertex scans its in-neighbours (row v of AT)
// in ascending order and stops at the first one in the frontier bitmap,
// the smallest valid parent.  Neighbours are taken PULL_BATCH at a time
// (independent loads, then independent bitmap probes) so a lane waits for
// two round trips per batch rather than two per neighbour.
constexpr int PULL_BATCH = 8;

__device__ __forceinline__ void bfs_pull(const LevelArgs &a, const uint32_t *__restrict__ cur,
                                         uint32_t *__restrict__ next, int32_t lev, unsigned long long &cnt,
                                         unsigned long long &deg, unsigned long long &hub)
{
    const int64_t n = a.n;
    int64_t *parent = (int64_t *)a.parent;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const unsigned lane = lane_id();
    // every lane runs the same trip count, so the ballot sees the whole wave
    for (int64_t v0 = (int64_t)blockIdx.x * blockDim.x; v0 < n; v0 += stride) {
        const int64_t v = v0 + threadIdx.x;
        int32_t par_v = -1;
        if (v < n && !bit_test(a.visited, v) && !bit_test(cur, v)) {
            const int64_t b = a.rpT[v], e = a.rpT[v + 1];
            for (int64_t p0 = b; p0 < e && par_v < 0; p0 += PULL_BATCH) {
                int32_t u[PULL_BATCH];
#pragma unroll
                for (int t = 0; t < PULL_BATCH; t++) u[t] = p0 + t < e ? a.ciT[p0 + t] : -1;
#pragma unroll
                for (int t = PULL_BATCH - 1; t >= 0; t--)
                    if (u[t] >= 0 && bit_test(cur, u[t])) par_v = u[t];
            }
        }
        if (par_v >= 0) {
            parent[v] = par_v;
            a.level[v] = lev;
            const int64_t dv = a.deg[v];
            cnt += 1;
            deg += (unsigned long long)dv;
            hub += dv > GRAPH_LONG_ROW ? 1ull : 0ull;
        }
        // the wave's 64 vertices are 64-aligned: they own two bitmap words,
        // which no other wave writes in this kernel.  Every word of the
        // next bitmap is written, so a pull needs no cleared bitmap.
        const uint64_t m = __ballot(par_v >= 0);
        const int64_t w0 = (v - lane) >> 5;
        if ((lane == 0 || lane == 32) && w0 + (lane >> 5) < a.W) next[w0 + (lane >> 5)] = (uint32_t)(m >> lane);
    }
}

// One level: expand F_k (the level after the one whose state is in
// st[par ^ 1]).  dp, st and ctr are the device struct, its st array and the
// counters (passed apart so that the state and counter loads go out first).
// Grid: BFS_GRID workgroups of 256.
__global__ __launch_bounds__(256, 8) void k_bfs_level(const BfsDev *__restrict__ dp, BfsLevel *st,
                                                      unsigned long long *ctr, int par)
{
    __shared__ BfsLevel S;
    __shared__ unsigned long long s_cnt, s_deg, s_hub;
    if (threadIdx.x < 64) bfs_level_state(st + (par ^ 1), ctr, dp->n, dp->push_only, dp->alpha, dp->beta, &S);
    LevelArgs a;
    a.rp = dp->rp;
    a.rpT = dp->rpT;
    a.deg = dp->deg;
    a.ci = dp->ci;
    a.ciT = dp->ciT;
    a.n = dp->n;
    a.W = dp->W;
    a.level = dp->level;
    a.parent = dp->parent;
    a.visited = dp->visited;
    a.bm0 = dp->bm[0];
    a.bm1 = dp->bm[1];
    a.bm2 = dp->bm[2];
    a.ch = dp->ch;
    a.any_parent = dp->any_parent;
    if (threadIdx.x == 0) {
        s_cnt = 0;
        s_deg = 0;
        s_hub = 0;
    }
    __syncthreads();
    if (S.done == 2) {
        // keep the finished state moving through the parities
        if (blockIdx.x == 0 && threadIdx.x == 0) st[par] = st[par ^ 1];
        return;
    }
    const int k = S.lev;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st[par] = S;
        if (S.done) __hip_atomic_store(dp->done_host, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
        else __hip_atomic_store(dp->level_host, k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
    if (S.done) return;
    const int r = k % 3;
    const uint32_t *cur = r == 0 ? a.bm0 : (r == 1 ? a.bm1 : a.bm2);
    uint32_t *next = r == 0 ? a.bm1 : (r == 1 ? a.bm2 : a.bm0);
    uint32_t *stale = r == 0 ? a.bm2 : (r == 1 ? a.bm0 : a.bm1);
    const int64_t gt = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t gstride = (int64_t)gridDim.x * blockDim.x;
    // F_k joins the visited set at the end of the level: the first word of
    // each thread is loaded now and or-ed in at the end
    const uint32_t fold0 = gt < a.W ? cur[gt] : 0u;
    // F_{k-1}'s bitmap is cleared for F_{k+2}
    for (int64_t w = gt; w < a.W; w += gstride) stale[w] = 0u;
    const int32_t lev = k + 1;   // the level of the vertices found now
    unsigned long long cnt = 0, deg = 0, hub = 0;
    const unsigned lane = lane_id();
    if (S.pull) {
        bfs_pull(a, cur, next, lev, cnt, deg, hub);
    } else {
        for_marked_vertices(cur, a.n, [&](int32_t u) {
            const int64_t b = a.rp[u], e = a.rp[u + 1];
            if (e - b <= GRAPH_LONG_ROW) push_range(a, cur, next, u, b, e, lane, lev, cnt, deg, hub);
        });
        // the frontier's hub rows (when it has any): every piece of a chunk
        // whose row is in the bitmap
        if (S.nhub > 0)
            for_marked_pieces(a.ch, cur, [&](int32_t u, int64_t b, int64_t e) {
                push_range(a, cur, next, u, b, e, lane, lev, cnt, deg, hub);
            });
    }
    if (fold0) atomicOr(&a.visited[gt], fold0);
    for (int64_t w = gt + gstride; w < a.W; w += gstride) {
        const uint32_t x = cur[w];
        if (x) atomicOr(&a.visited[w], x);
    }
    // the level's vertex count, degree sum and hub count: one atomic per
    // workgroup on one of BFS_SPREAD counters
    cnt = wave_sum64(cnt);
    deg = wave_sum64(deg);
    hub = wave_sum64(hub);
    if (lane == 0 && (cnt | deg | hub)) {
        atomicAdd(&s_cnt, cnt);
        atomicAdd(&s_deg, deg);
        atomicAdd(&s_hub, hub);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const int sp = (int)(blockIdx.x % BFS_SPREAD);
        if (s_cnt) atomicAdd(ctr + (size_t)sp * BFS_CTR_STRIDE, s_cnt);
        if (s_deg) atomicAdd(ctr + (size_t)(BFS_SPREAD + sp) * BFS_CTR_STRIDE, s_deg);
        if (s_hub) atomicAdd(ctr + (size_t)(2 * BFS_SPREAD + sp) * BFS_CTR_STRIDE, s_hub);
    }
}

// The per-search start: the search's arguments h (the graph's first node,
// whose argument the host sets before each launch) into the device struct,
// levels and parents to -1, the four bitmaps (visited, three frontiers) and
// the counters to 0, except the source's entries: F_0 = {src} in bm[0]
// and the source in the counters.
__global__ void k_bfs_start(BfsDev h, BfsDev *__restrict__ dp)
{
    const int64_t n = h.n, W = h.W, src = h.src;
    const int64_t step = (int64_t)gridDim.x * blockDim.x;
    const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int64_t i = t0; i < n; i += step) {
        h.level[i] = i == src ? 0 : -1;
        h.parent[i] = i == src ? (unsigned long long)src : ~0ull;
    }
    uint32_t *bms = h.visited;   // visited, then bm[0..2], contiguous
    const int64_t sw = W + (src >> 5);
    const uint32_t sbit = 1u << (src & 31);
    for (int64_t i = t0; i < 4 * W; i += step) bms[i] = i == sw ? sbit : 0u;
    // the struct and the counters, by thread 0 alone (it then sets the
    // source's)
    if (t0 == 0) {
        *dp = h;
        for (int i = 0; i < BFS_NCTR; i++) h.ctr[(size_t)i * BFS_CTR_STRIDE] = 0ull;
        const int64_t ds = h.deg[src];
        h.ctr[0] = 1ull;
        h.ctr[(size_t)BFS_SPREAD * BFS_CTR_STRIDE] = (unsigned long long)ds;
        if (ds > GRAPH_LONG_ROW) h.ctr[(size_t)2 * BFS_SPREAD * BFS_CTR_STRIDE] = 1ull;
    }
}

__global__ void k_level_to_i64(const int32_t *__restrict__ in, int64_t *__restrict__ out, int64_t n)
{
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x)
        out[v] = in[v];
}

}  // namespace

// Levels in the first graph of a search (the start, then levels 0..7: an
// R-MAT graph of 2^20 vertices is 5 to 7 levels deep, and one more level
// finds the frontier empty) and in each further graph (4).
constexpr int BFS_FIRST_LEVELS = 8;
constexpr int BFS_MORE_LEVELS = 4;

static int add_level_nodes(hipGraph_t g, hipGraphNode_t prev, BfsDev *d, unsigned long long *ctr, int first_par,
                           int count, char *msg)
{
    BfsLevel *st = d->st;   // address arithmetic only: d is a device address
    for (int l = 0; l < count; l++) {
        int par = (first_par + l) & 1;
        const BfsDev *dc = d;
        void *args[] = {&dc, &st, &ctr, &par};
        hipKernelNodeParams p{};
        p.func = (void *)k_bfs_level;
        p.gridDim = dim3(BFS_GRID);
        p.blockDim = dim3(256);
        p.sharedMemBytes = 0;
        p.kernelParams = args;
        p.extra = nullptr;
        hipGraphNode_t node = nullptr;
        HIP_TRY(hipGraphAddKernelNode(&node, g, prev ? &prev : nullptr, prev ? 1 : 0, &p));
        prev = node;
    }
    return LAGR_SUCCESS;
}

static hipKernelNodeParams start_params(void **args, int64_t n)
{
    hipKernelNodeParams p{};
    p.func = (void *)k_bfs_start;
    p.gridDim = dim3(grid_for(n, 256, 4096));
    p.blockDim = dim3(256);
    p.sharedMemBytes = 0;
    p.kernelParams = args;
    p.extra = nullptr;
    return p;
}

// The context's graphs for graphs of n vertices and the state struct d:
// the start and levels 0..BFS_FIRST_LEVELS-1, and BFS_MORE_LEVELS further
// levels (level k has parity k & 1).  The start node's argument is set
// before each launch.
static int bfs_graphs(lagr_ctx ctx, BfsDev *d, unsigned long long *ctr, int64_t n, char *msg)
{
    if (ctx->bfs_exec && ctx->bfs_exec_more && ctx->bfs_key == n && ctx->bfs_state == (void *)d &&
        ctx->bfs_ctr == (void *)ctr)
        return LAGR_SUCCESS;
    if (ctx->bfs_exec) (void)hipGraphExecDestroy(ctx->bfs_exec);
    if (ctx->bfs_exec_more) (void)hipGraphExecDestroy(ctx->bfs_exec_more);
    if (ctx->bfs_graph) (void)hipGraphDestroy(ctx->bfs_graph);
    ctx->bfs_exec = ctx->bfs_exec_more = nullptr;
    ctx->bfs_graph = nullptr;
    ctx->bfs_start_node = nullptr;
    ctx->bfs_key = -1;
    BfsDev h{};
    void *sargs[] = {&h, &d};
    const hipKernelNodeParams sp = start_params(sargs, n);
    hipGraph_t g = nullptr;
    HIP_TRY(hipGraphCreate(&g, 0));
    ctx->bfs_graph = g;
    HIP_TRY(hipGraphAddKernelNode(&ctx->bfs_start_node, g, nullptr, 0, &sp));
    TRY(add_level_nodes(g, ctx->bfs_start_node, d, ctr, 0, BFS_FIRST_LEVELS, msg));
    HIP_TRY(hipGraphInstantiate(&ctx->bfs_exec, g, nullptr, nullptr, 0));
    hipGraph_t g2 = nullptr;
    HIP_TRY(hipGraphCreate(&g2, 0));
    int rc = add_level_nodes(g2, nullptr, d, ctr, BFS_FIRST_LEVELS & 1, BFS_MORE_LEVELS, msg);
    const hipError_t ei = rc >= 0 ? hipGraphInstantiate(&ctx->bfs_exec_more, g2, nullptr, nullptr, 0) : hipSuccess;
    (void)hipGraphDestroy(g2);
    if (rc < 0) return rc;
    if (ei != hipSuccess) {
        ctx->bfs_exec_more = nullptr;
        return lagr_fail(msg, LAGR_DEVICE_ERROR, "bfs graph: %s", hipGetErrorString(ei));
    }
    ctx->bfs_key = n;
    ctx->bfs_state = (void *)d;
    ctx->bfs_ctr = (void *)ctr;
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
    // four bitmaps (visited, three frontiers), then the counters
    const size_t bm_bytes = (sizeof(uint32_t) * 4 * W + 255) & ~(size_t)255;
    uint32_t *bms = (uint32_t *)ws_get(ctx, WS_BFS_C, bm_bytes + sizeof(unsigned long long) * BFS_NCTR * BFS_CTR_STRIDE);
    BfsDev *d = (BfsDev *)ws_get(ctx, WS_BFS_D, sizeof(BfsDev));
    int64_t *parent_scratch = nullptr;
    if (!parent_out) parent_scratch = (int64_t *)ws_get(ctx, WS_BFS_E, sizeof(int64_t) * n);
    if (!lev32 || !bms || !d || (!parent_out && !parent_scratch))
        return lagr_fail(msg, LAGR_OUT_OF_MEMORY, "bfs workspace");
    RowChunks ch;
    TRY(graph_chunks(G, ctx, &ch, msg));
    TRY(lagr_property_row_degree(G, ctx, msg));
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

    // the search's arguments go to the device as the start node's argument
    static_assert(sizeof(BfsDev) <= 2048, "BfsDev is passed as a kernel argument");
    BfsDev h{};
    h.rp = A->rowptr;
    h.ci = A->colidx;
    h.rpT = AT->rowptr;
    h.ciT = AT->colidx;
    h.deg = G->row_degree;
    h.n = n;
    h.W = W;
    h.level = lev32;
    h.parent = (unsigned long long *)parent;
    h.visited = bms;
    h.bm[0] = bms + W;
    h.bm[1] = bms + 2 * W;
    h.bm[2] = bms + 3 * W;
    h.ctr = (unsigned long long *)((char *)bms + bm_bytes);
    h.ch = ch;
    h.any_parent = (flags & LAGR_BFS_ANY_PARENT) ? 1 : 0;
    h.push_only = (flags & LAGR_BFS_PUSH_ONLY) ? 1 : 0;
    h.alpha = G->bfs_alpha;
    h.beta = G->bfs_beta;
    h.src = source;
    // the state "before level 0", which level 0 (parity 0) reads from st[1]
    h.st[1].lev = -1;
    h.st[1].pull = 0;
    h.st[1].done = 0;
    h.st[1].mu = A->nvals;
    // the level kernel that finds the frontier empty stores 1 to the done
    // word, and every other level stores its index to the level word; the
    // host clears both first.  Nothing else writes them: the last search on
    // this context had stored its done word before that call returned, and
    // its levels left in flight only pass the finished state on.
    volatile int32_t *done_flag = (volatile int32_t *)((char *)ctx->pinned + LAGR_PINNED_STAGE);
    volatile int32_t *level_flag = (volatile int32_t *)((char *)ctx->pinned + LAGR_PINNED_LEVEL);
    h.done_host = (int32_t *)((char *)ctx->pinned_dev + LAGR_PINNED_STAGE);
    h.level_host = (int32_t *)((char *)ctx->pinned_dev + LAGR_PINNED_LEVEL);
    BFS_TRY(bfs_graphs(ctx, d, h.ctr, n, msg));
    {
        // the previous search's start node has run: its done word came
        // from a later node
        void *sargs[] = {&h, &d};
        const hipKernelNodeParams sp = start_params(sargs, n);
        if (hipGraphExecKernelNodeSetParams(ctx->bfs_exec, ctx->bfs_start_node, &sp) != hipSuccess)
            BFS_TRY(lagr_fail(msg, LAGR_DEVICE_ERROR, "bfs start arguments"));
    }
    *done_flag = 0;
    *level_flag = -1;
    std::atomic_thread_fence(std::memory_order_seq_cst);
    if (hipGraphLaunch(ctx->bfs_exec, ctx->stream) != hipSuccess)
        BFS_TRY(lagr_fail(msg, LAGR_DEVICE_ERROR, "bfs graph launch"));
    // poll the pinned words: return at the done word, and queue more
    // levels whenever the last queued level has started without finding the
    // frontier empty.  Every 64 polls the runtime is asked whether the stream
    // failed or drained.
    int64_t queued = BFS_FIRST_LEVELS;
    for (unsigned it = 1;; it++) {
        if (*done_flag) break;
        if (*level_flag >= queued - 1) {
            if (queued > n + 2) BFS_TRY(lagr_fail(msg, LAGR_DEVICE_ERROR, "bfs did not terminate"));
            if (hipGraphLaunch(ctx->bfs_exec_more, ctx->stream) != hipSuccess)
                BFS_TRY(lagr_fail(msg, LAGR_DEVICE_ERROR, "bfs graph launch"));
            queued += BFS_MORE_LEVELS;
            continue;
        }
        if ((it & 63u) == 0) {
            const hipError_t e = hipStreamQuery(ctx->stream);
            if (e != hipSuccess && e != hipErrorNotReady)
                BFS_TRY(lagr_fail(msg, LAGR_DEVICE_ERROR, "bfs stream: %s", hipGetErrorString(e)));
            if (e == hipSuccess && !*done_flag && *level_flag < queued - 1)
                BFS_TRY(lagr_fail(msg, LAGR_DEVICE_ERROR, "bfs stream drained before the search ended"));
        }
    }
    std::atomic_thread_fence(std::memory_order_acquire);
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

// The BFS direction thresholds for this graph: every (alpha, beta) of a
// small grid around Beamer's (14, 24) times lagr_bfs from the given
// sources (host clock, the sum over the sources of the median of 3
// searches each); the fastest pair is kept in G for later searches.
extern "C" int lagr_bfs_autotune(int32_t *alpha, int32_t *beta, lagr_graph G, const int64_t *sources, int32_t ns,
                                 lagr_ctx ctx, char *msg)
{
    if (!G || !ctx || (ns > 0 && !sources)) return lagr_fail(msg, LAGR_NULL_POINTER, "NULL argument");
    if (ns <= 0) return lagr_fail(msg, LAGR_INVALID_VALUE, "no sources to time");
    if (ctx->device < 0) return lagr_fail(msg, LAGR_DEVICE_ERROR, "validation-only context");
    const int32_t as[] = {6, 10, 14, 20, 32};
    const int32_t bs[] = {12, 24, 48};
    int32_t ba = G->bfs_alpha, bb = G->bfs_beta;
    double best = -1.0;
    for (const int32_t a : as)
        for (const int32_t b : bs) {
            G->bfs_alpha = a;
            G->bfs_beta = b;
            std::vector<double> per;
            for (int32_t k = 0; k < ns; k++) {
                double ts[3];
                for (int r = 0; r < 3; r++) {
                    // no outputs: the search runs in the context's workspace
                    const auto t0 = std::chrono::steady_clock::now();
                    int rc = lagr_bfs(nullptr, nullptr, G, sources[k], 0, ctx, msg);
                    if (rc >= 0) rc = host_wait(ctx, msg);
                    ts[r] = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
                    if (rc < 0) {
                        G->bfs_alpha = ba;
                        G->bfs_beta = bb;
                        return rc;
                    }
                }
                std::sort(ts, ts + 3);
                per.push_back(ts[1]);
            }
            double tot = 0.0;
            for (const double t : per) tot += t;
            if (best < 0 || tot < best) {
                best = tot;
                ba = a;
                bb = b;
            }
        }
    G->bfs_alpha = ba;
    G->bfs_beta = bb;
    if (alpha) *alpha = ba;
    if (beta) *beta = bb;
    return lagr_ok(msg);
}
