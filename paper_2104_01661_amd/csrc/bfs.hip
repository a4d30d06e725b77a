// Direction-optimising parents BFS (Section IV-A, Algorithms 1 and 2).
//
// One level is q<!s(p), r> = q any.secondi A, fused with p<s(q)> = q (the
// vxm + assign fusion Section VI-B describes for GAP's bfs.cc): the kernel
// that discovers v writes its parent, its level, the next frontier list
// and the next frontier bitmap in the same pass.
//   push: a wavefront per frontier vertex u scans N(u) with coalesced loads;
//         a vertex is claimed by a 32-bit CAS on its level.  The parent is
//         the smallest frontier neighbour (atomicMin on the unsigned
//         parent, whose "absent" value -1 is the largest), or, with
//         LAGR_BFS_ANY_PARENT, the CAS winner.
//   pull: one lane per unvisited vertex v scans N(v) in ascending order
//         and stops at the first neighbour in the frontier bitmap, which is
//         the smallest valid parent.
//   The frontier's hub vertices (rows longer than GRAPH_LONG_ROW) are
//   pushed chunk by chunk by separate waves, so no wave walks a whole hub.
// Direction (Beamer, Asanovic and Patterson, SC 2012, the heuristic the
// paper cites): pull when the frontier's edges exceed the unexplored edges
// / ALPHA, back to push when the frontier has fewer than n / BETA vertices.
#include "internal.h"

namespace {

__device__ __forceinline__ int64_t bcast64(int64_t x, int src)
{
    const int lo = __shfl((int)(x & 0xffffffff), src, 64);
    const int hi = __shfl((int)(x >> 32), src, 64);
    return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

constexpr int BFS_ALPHA = 14;
constexpr int BFS_BETA = 24;

struct BfsCounters {
    unsigned long long nnext;   // vertices discovered this level
    unsigned long long enext;   // sum of their degrees
};

__device__ __forceinline__ bool bit_test(const uint32_t *bm, int64_t v)
{
    return (bm[v >> 5] >> (v & 31)) & 1u;
}

// `visited` holds the vertices of earlier levels only; it absorbs the
// level's discoveries after the level, so every frontier neighbour of a
// vertex found in this level still reaches the parent update.
// The level kernels only write levels, parents and the next frontier's
// bitmap.  k_bfs_compact then turns the bitmap into the next frontier list
// (ascending within each workgroup's range), counts it and its degree sum,
// and adds it to the visited set: one global atomic per workgroup, since
// atomics on one address from every wavefront serialise.

__global__ __launch_bounds__(256) void k_bfs_init(int64_t src, int32_t *level, int64_t *parent,
                                                  int32_t *list, uint32_t *visited, uint32_t *bm)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        level[src] = 0;
        parent[src] = src;
        list[0] = (int32_t)src;
        visited[src >> 5] |= 1u << (src & 31);
        bm[src >> 5] |= 1u << (src & 31);
    }
}

// Push the neighbours rp-range [b, e) of frontier vertex u, one per lane.
__device__ __forceinline__ void push_range(const int32_t *__restrict__ ci, int32_t u, int64_t b, int64_t e,
                                           unsigned lane, int32_t lev, int any_parent,
                                           int32_t *__restrict__ level, unsigned long long *__restrict__ parent,
                                           const uint32_t *__restrict__ visited, uint32_t *__restrict__ next_bm)
{
    for (int64_t p = b + lane; p < e; p += 64) {
        const int32_t v = ci[p];
        if (bit_test(visited, v)) continue;
        const int32_t old = atomicCAS(&level[v], -1, lev);
        if (old == -1) {
            if (any_parent) parent[v] = (unsigned long long)u;
            else atomicMin(&parent[v], (unsigned long long)u);
            atomicOr(&next_bm[v >> 5], 1u << (v & 31));
        } else if (old == lev && !any_parent) {
            atomicMin(&parent[v], (unsigned long long)u);
        }
    }
}

__global__ __launch_bounds__(256) void k_bfs_push(const int64_t *__restrict__ rp,
                                                  const int32_t *__restrict__ ci,
                                                  const int32_t *__restrict__ frontier, int64_t nq,
                                                  int32_t lev, int any_parent,
                                                  int32_t *__restrict__ level,
                                                  unsigned long long *__restrict__ parent,
                                                  const uint32_t *__restrict__ visited,
                                                  uint32_t *__restrict__ next_bm)
{
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / 64;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / 64;
    const unsigned lane = lane_id();
    for (int64_t f = wave; f < nq; f += nw) {
        const int32_t u = frontier[f];
        const int64_t b = rp[u], e = rp[u + 1];
        if (e - b > GRAPH_LONG_ROW) continue;   // k_bfs_push_chunks
        push_range(ci, u, b, e, lane, lev, any_parent, level, parent, visited, next_bm);
    }
}

// The frontier's hub vertices: every chunk of a long row whose vertex is in
// the frontier bitmap is pushed by its own wave.
__global__ __launch_bounds__(256) void k_bfs_push_chunks(const int32_t *__restrict__ ci, RowChunks ch,
                                                         const uint32_t *__restrict__ cur_bm,
                                                         int32_t lev, int any_parent,
                                                         int32_t *__restrict__ level,
                                                         unsigned long long *__restrict__ parent,
                                                         const uint32_t *__restrict__ visited,
                                                         uint32_t *__restrict__ next_bm)
{
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / 64;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / 64;
    const unsigned lane = lane_id();
    for (int64_t c = wave; c < ch.n; c += nw) {
        const int32_t u = ch.row[c];
        if (!bit_test(cur_bm, u)) continue;
        push_range(ci, u, ch.beg[c], ch.end[c], lane, lev, any_parent, level, parent, visited, next_bm);
    }
}

// One lane per unvisited vertex: scan its neighbours in ascending order and
// stop at the first one in the frontier bitmap, the smallest valid parent.
// Neighbours are taken PULL_BATCH at a time (independent loads, then
// independent bitmap probes) so a lane waits for two round trips per batch
// rather than two per neighbour.
constexpr int PULL_BATCH = 8;

__global__ __launch_bounds__(256) void k_bfs_pull(const int64_t *__restrict__ rp,
                                                  const int32_t *__restrict__ ci, int64_t n,
                                                  int32_t lev, const uint32_t *__restrict__ cur_bm,
                                                  int32_t *__restrict__ level,
                                                  int64_t *__restrict__ parent,
                                                  const uint32_t *__restrict__ visited,
                                                  uint32_t *__restrict__ next_bm)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    // every lane runs the same trip count, so the ballot sees the whole wave
    for (int64_t v0 = (int64_t)blockIdx.x * blockDim.x; v0 < n; v0 += stride) {
        const int64_t v = v0 + threadIdx.x;
        int32_t par = -1;
        if (v < n && !bit_test(visited, v)) {
            const int64_t b = rp[v], e = rp[v + 1];
            for (int64_t p0 = b; p0 < e && par < 0; p0 += PULL_BATCH) {
                int32_t u[PULL_BATCH];
#pragma unroll
                for (int t = 0; t < PULL_BATCH; t++) u[t] = p0 + t < e ? ci[p0 + t] : -1;
#pragma unroll
                for (int t = PULL_BATCH - 1; t >= 0; t--)
                    if (u[t] >= 0 && bit_test(cur_bm, u[t])) par = u[t];
            }
        }
        if (par >= 0) {
            parent[v] = par;
            level[v] = lev;
        }
        // the wave's 64 vertices are 64-aligned: they own two bitmap words,
        // which no other wave writes in this kernel
        const uint64_t m = __ballot(par >= 0);
        const unsigned lane = lane_id();
        const int64_t w0 = (v - lane) >> 5;
        if (lane == 0 && (uint32_t)m) next_bm[w0] = (uint32_t)m;
        if (lane == 32 && (uint32_t)(m >> 32)) next_bm[w0 + 1] = (uint32_t)(m >> 32);
    }
}

// Next frontier from its bitmap: a thread per 32-bit word.  Each workgroup
// scans its words' popcounts, reserves its range of the list with one
// atomic, writes its vertices in ascending order, adds its degree sum with
// one more atomic and ORs its words into the visited set.
__global__ __launch_bounds__(256) void k_bfs_compact(const int64_t *__restrict__ rp, int64_t n,
                                                     const uint32_t *__restrict__ next_bm, int64_t W,
                                                     uint32_t *__restrict__ visited,
                                                     int32_t *__restrict__ next_list,
                                                     BfsCounters *__restrict__ cnt)
{
    __shared__ unsigned scan[256];
    __shared__ unsigned long long base_s, deg_s;
    const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t x = w < W ? next_bm[w] : 0u;
    if (x) visited[w] |= x;
    const unsigned c = (unsigned)__popc(x);
    unsigned long long deg = 0;
    for (uint32_t y = x; y; y &= y - 1) {
        const int64_t v = w * 32 + __ffs(y) - 1;
        deg += (unsigned long long)(rp[v + 1] - rp[v]);
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
    if (threadIdx.x == 255) base_s = scan[255] ? atomicAdd(&cnt->nnext, (unsigned long long)scan[255]) : 0;
    __syncthreads();
    if (threadIdx.x == 0 && deg_s) atomicAdd(&cnt->enext, deg_s);
    unsigned long long pos = base_s + scan[threadIdx.x] - c;
    for (uint32_t y = x; y; y &= y - 1) next_list[pos++] = (int32_t)(w * 32 + __ffs(y) - 1);
}

__global__ void k_level_to_i64(const int32_t *__restrict__ in, int64_t *__restrict__ out, int64_t n)
{
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x)
        out[v] = in[v];
}

}  // namespace

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
    if (G->kind != LAGR_ADJACENCY_UNDIRECTED && !(flags & LAGR_BFS_PUSH_ONLY))
        return lagr_fail(msg, LAGR_NOT_IMPLEMENTED,
                         "pull steps on a directed graph need its transpose; use LAGR_BFS_PUSH_ONLY");
    const int64_t W = (n + 31) / 32;
    int32_t *lev32 = (int32_t *)ws_get(ctx, WS_BFS_A, sizeof(int32_t) * n);
    int32_t *lists = (int32_t *)ws_get(ctx, WS_BFS_B, sizeof(int32_t) * 2 * n);
    uint32_t *bms = (uint32_t *)ws_get(ctx, WS_BFS_C, sizeof(uint32_t) * 3 * W);
    BfsCounters *cnt = (BfsCounters *)ws_get(ctx, WS_BFS_D, sizeof(BfsCounters));
    int64_t *parent_scratch = nullptr;
    if (!parent_out) parent_scratch = (int64_t *)ws_get(ctx, WS_BFS_E, sizeof(int64_t) * n);
    if (!lev32 || !lists || !bms || !cnt || (!parent_out && !parent_scratch))
        return lagr_fail(msg, LAGR_OUT_OF_MEMORY, "bfs workspace");
    lagr_vector pv = nullptr, lv = nullptr;
    int64_t *parent = parent_scratch;
    if (parent_out) TRY(new_full_i64(&pv, n, &parent, msg));
    uint32_t *visited = bms, *bm_cur = bms + W, *bm_next = bms + 2 * W;
    int32_t *list_cur = lists, *list_next = lists + n;

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

    BFS_TRY(fill_u32(ctx, (uint32_t *)lev32, n, 0xFFFFFFFFu, msg));
    BFS_TRY(fill_i64(ctx, parent, n, -1, msg));
    BFS_TRY(fill_u32(ctx, bms, 3 * W, 0u, msg));
    hipLaunchKernelGGL(k_bfs_init, dim3(1), dim3(64), 0, ctx->stream, source, lev32, parent,
                       list_cur, visited, bm_cur);
    if (hipGetLastError() != hipSuccess) {
        cleanup();
        return lagr_fail(msg, LAGR_DEVICE_ERROR, "bfs init launch");
    }
    const int64_t *rp = A->rowptr;
    const int32_t *ci = A->colidx;
    RowChunks ch;
    {
        int rc2 = graph_chunks(G, ctx, &ch, msg);
        if (rc2 < 0) {
            cleanup();
            return rc2;
        }
    }
    // host copies of the per-level counters drive the direction choice
    int64_t hdeg_src = 0;
    {
        int64_t two[2];
        BFS_TRY(read_back(ctx, two, rp + source, 2 * sizeof(int64_t), msg));
        hdeg_src = two[1] - two[0];
    }
    int64_t nq = 1, mf = hdeg_src, mu = A->nvals - hdeg_src;
    bool pull = false;
    const bool push_only = (flags & LAGR_BFS_PUSH_ONLY) != 0;
    const int any_parent = (flags & LAGR_BFS_ANY_PARENT) ? 1 : 0;
    for (int32_t lev = 1; nq > 0 && lev < INT32_MAX; lev++) {
        if (!push_only) {
            if (!pull && mf > mu / BFS_ALPHA) pull = true;
            else if (pull && nq < n / BFS_BETA) pull = false;
        }
        BFS_TRY(fill_i64(ctx, (int64_t *)cnt, 2, 0, msg));
        if (pull) {
            TIMED(ctx, "bfs_pull",
                  hipLaunchKernelGGL(k_bfs_pull, dim3(grid_for(n, 256, 8192)), dim3(256), 0,
                                     ctx->stream, rp, ci, n, lev, bm_cur, lev32, parent, visited,
                                     bm_next));
        } else {
            TIMED(ctx, "bfs_push",
                  hipLaunchKernelGGL(k_bfs_push, dim3(grid_for(nq * 64, 256, 8192)), dim3(256), 0,
                                     ctx->stream, rp, ci, list_cur, nq, lev, any_parent, lev32,
                                     (unsigned long long *)parent, visited, bm_next));
            if (ch.n > 0)
                TIMED(ctx, "bfs_push",
                      hipLaunchKernelGGL(k_bfs_push_chunks, dim3(grid_for(ch.n * 64, 256, 4096)),
                                         dim3(256), 0, ctx->stream, ci, ch, bm_cur, lev, any_parent,
                                         lev32, (unsigned long long *)parent, visited, bm_next));
        }
        if (hipGetLastError() != hipSuccess) {
            cleanup();
            return lagr_fail(msg, LAGR_DEVICE_ERROR, "bfs level launch");
        }
        TIMED(ctx, "bfs_compact",
              hipLaunchKernelGGL(k_bfs_compact, dim3(grid_for(W, 256, 1 << 30)), dim3(256), 0, ctx->stream,
                                 rp, n, bm_next, W, visited, list_next, cnt));
        BfsCounters h;
        BFS_TRY(read_back(ctx, &h, cnt, sizeof(h), msg));
        nq = (int64_t)h.nnext;
        mf = (int64_t)h.enext;
        mu -= mf;
        // the consumed frontier bitmap becomes the next level's output
        BFS_TRY(fill_u32(ctx, bm_cur, W, 0u, msg));
        uint32_t *tb = bm_cur;
        bm_cur = bm_next;
        bm_next = tb;
        int32_t *tl = list_cur;
        list_cur = list_next;
        list_next = tl;
    }
    if (level_out) {
        int64_t *lvals = nullptr;
        BFS_TRY(new_full_i64(&lv, n, &lvals, msg));
        hipLaunchKernelGGL(k_level_to_i64, dim3(grid_for(n, 256, 8192)), dim3(256), 0, ctx->stream,
                           lev32, lvals, n);
        if (hipGetLastError() != hipSuccess) {
            cleanup();
            return lagr_fail(msg, LAGR_DEVICE_ERROR, "bfs level export");
        }
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
