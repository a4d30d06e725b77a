// Batched betweenness centrality (Section IV-B, Algorithm 3).
//
// Layout: a batch holds up to 64 sources, one per wavefront lane.  Path
// counts sigma and the backward quantity W = (1 + delta) / sigma are
// n x 64 FP64 arrays, vertex-major (the 64 lanes of a vertex are 512
// contiguous bytes, so a wave reads a neighbour's row in one coalesced
// load).  The frontier S[d] of Algorithm 3 is kept as one 64-bit lane mask
// per vertex and level (bit k = vertex is at depth d from source k) plus
// the list of vertices whose mask is not empty; the visited mask P's
// pattern is the per-vertex mask of lanes not yet reached, with a list of
// the vertices that still have such lanes ("active").
//
// Forward level d (F<!s(P), r> = F plus.first A, then P += F), in the
// direction that touches fewer edges (the choice the paper describes for
// BC, after Beamer):
//   pull: a wave per active vertex v gathers, in ascending neighbour order,
//         sigma(u, k) of the neighbours u at depth d in lane k;
//   push: a wave per frontier vertex u adds sigma(u, k) to every neighbour
//         v still unreached in lane k (FP64 atomics).
// Path counts are integers below 2^53, so every FP64 sum is exact and the
// result does not depend on the order of the additions.  A compaction pass
// then folds the new masks into the unreached masks and lists the next
// frontier and the active vertices.
// Backward level i (Algorithm 3's backtrack, read as i = d down to 1 so the
// deepest level contributes): for v at depth i-1 in lane k (the level's
// list),
//   delta(v,k) = sigma(v,k) * sum over neighbours w at depth i in lane k of
//                W(w,k),   W(w,k) = (1 + delta(w,k)) / sigma(w,k),
// summed in ascending neighbour order; the kernel writes W(v,k) for the
// next level and adds the lane sum of delta(v,.) to centrality(v).  A
// source contributes nothing to itself (depth 0 is never a target).
#include <vector>

#include "internal.h"

namespace {

// Vertices with more neighbours than BC_LONG are split into BC_CHUNK-long
// pieces (hub vertices would otherwise hold one wave for the whole level).
constexpr int64_t BC_LONG = GRAPH_LONG_ROW;
constexpr int64_t BC_CHUNK = GRAPH_LONG_ROW;
// push a forward level when the frontier's edges are fewer than the active
// vertices' edges / BC_PUSH_RATIO
constexpr int64_t BC_PUSH_RATIO = 10;

__global__ __launch_bounds__(256) void k_bc_init(int64_t n, uint64_t lanes,
                                                 uint64_t *__restrict__ unvis,
                                                 uint64_t *__restrict__ mask0)
{
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x) {
        unvis[v] = lanes;
        mask0[v] = 0;
    }
}

// src[k] is lane k's source, or -1 for an idle lane
__global__ void k_bc_sources(const int64_t *__restrict__ src, uint64_t *__restrict__ unvis,
                             uint64_t *__restrict__ mask0, double *__restrict__ sigma)
{
    const int k = threadIdx.x;
    if (k < 64 && src[k] >= 0) {
        const int64_t s = src[k];
        atomicAnd((unsigned long long *)&unvis[s], ~(1ull << k));
        atomicOr((unsigned long long *)&mask0[s], 1ull << k);
        sigma[s * 64 + k] = 1.0;
    }
}

// Add the sum of delta over each group of 2^gshift lanes (a fixed tree, so
// a group's sum does not depend on the other lanes) to centrality
// [v * groups + group]; gshift = 6 sums all 64 lanes into centrality[v].
__device__ __forceinline__ void group_add(double delta, int gshift, unsigned lane,
                                          double *__restrict__ centrality, int64_t v)
{
    double t = delta;
    for (int o = (1 << gshift) >> 1; o > 0; o >>= 1) t += __shfl_xor(t, o, 64);
    if ((lane & ((1u << gshift) - 1)) == 0) centrality[v * (64 >> gshift) + (lane >> gshift)] += t;
}

__device__ __forceinline__ int64_t bcast64(int64_t x, int src)
{
    const int lo = __shfl((int)(x & 0xffffffff), src, 64);
    const int hi = __shfl((int)(x >> 32), src, 64);
    return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

__device__ __forceinline__ uint64_t shfl64(uint64_t x, int src)
{
    const unsigned lo = __shfl((unsigned)(x & 0xffffffffu), src, 64);
    const unsigned hi = __shfl((unsigned)(x >> 32), src, 64);
    return ((uint64_t)hi << 32) | lo;
}

// acc += val[u_t * 64 + lane] for every hit t of the ballot `hits` (in
// ascending t) whose mask m_t has this lane, where u_t and m_t are lane t's
// neighbour and mask.  Eight rows are loaded before any is added, and the
// additions keep the ascending order (adding 0.0 for a lane without the bit
// leaves the sum unchanged), so the result is that of the one-at-a-time
// loop.
constexpr int BC_GATHER = 8;

__device__ __forceinline__ double gather_hits(uint64_t hits, int32_t u, uint64_t m, const double *__restrict__ val,
                                              unsigned lane, double acc)
{
    while (hits) {
        int32_t uu[BC_GATHER];
        bool on[BC_GATHER];
#pragma unroll
        for (int j = 0; j < BC_GATHER; j++) {
            on[j] = false;
            uu[j] = 0;
            if (hits) {
                const int t = __ffsll((unsigned long long)hits) - 1;
                hits &= hits - 1;
                uu[j] = __shfl(u, t, 64);
                on[j] = (shfl64(m, t) >> lane) & 1ull;
            }
        }
        double x[BC_GATHER];
#pragma unroll
        for (int j = 0; j < BC_GATHER; j++) x[j] = on[j] ? val[(int64_t)uu[j] * 64 + lane] : 0.0;
#pragma unroll
        for (int j = 0; j < BC_GATHER; j++) acc += x[j];
    }
    return acc;
}

// Pull: one wave per active vertex (rows of at most BC_LONG neighbours);
// writes next[v] (zero on entry) and sigma of the lanes it reaches.
__device__ __forceinline__ void bc_pull_rows(const int64_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                                 const int32_t *__restrict__ act, int64_t na,
                                                 const uint64_t *__restrict__ cur, uint64_t *__restrict__ next,
                                                 const uint64_t *__restrict__ unvis, double *__restrict__ sigma)
{
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / 64;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / 64;
    const unsigned lane = lane_id();
    for (int64_t q = wave; q < na; q += nw) {
        const int64_t v = act[q];
        const int64_t b = rp[v], e = rp[v + 1];
        if (e - b > BC_LONG) continue;   // bc_forward_chunks
        const uint64_t uv = unvis[v];
        double acc = 0.0;
        for (int64_t p0 = b; p0 < e; p0 += 64) {
            const int64_t p = p0 + lane;
            int32_t u = 0;
            uint64_t fm = 0;
            if (p < e) {
                u = ci[p];
                fm = cur[u] & uv;
            }
            acc = gather_hits(__ballot(fm != 0), u, fm, sigma, lane, acc);
        }
        const uint64_t nw_mask = __ballot(acc > 0.0) & uv;
        if ((nw_mask >> lane) & 1ull) sigma[v * 64 + lane] = acc;
        if (lane == 0 && nw_mask) next[v] = nw_mask;
    }
}

// Push from frontier vertex u (lanes fm, this lane's sigma su) over the
// neighbour range [b, e), 64 neighbours per step.
__device__ __forceinline__ void bc_push_range(const int32_t *__restrict__ ci, int64_t b, int64_t e, uint64_t fm,
                                              double su, const uint64_t *__restrict__ unvis,
                                              double *__restrict__ sigma, uint64_t *__restrict__ next,
                                              unsigned lane)
{
    for (int64_t p0 = b; p0 < e; p0 += 64) {
        const int64_t p = p0 + lane;
        int32_t v = 0;
        uint64_t m = 0;
        if (p < e) {
            v = ci[p];
            m = unvis[v] & fm;
        }
        uint64_t hits = __ballot(m != 0);
        while (hits) {
            const int t = __ffsll((unsigned long long)hits) - 1;
            hits &= hits - 1;
            const int32_t vv = __shfl(v, t, 64);
            const uint64_t mm = shfl64(m, t);
            if ((mm >> lane) & 1ull) unsafeAtomicAdd(&sigma[(int64_t)vv * 64 + lane], su);
            if (lane == 0) atomicOr((unsigned long long *)&next[vv], (unsigned long long)mm);
        }
    }
}

// Push: one wave per frontier vertex (rows of at most BC_LONG neighbours).
__device__ __forceinline__ void bc_push_rows(const int64_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                                 const int32_t *__restrict__ front, int64_t nf,
                                                 const uint64_t *__restrict__ cur, uint64_t *__restrict__ next,
                                                 const uint64_t *__restrict__ unvis, double *__restrict__ sigma)
{
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / 64;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / 64;
    const unsigned lane = lane_id();
    for (int64_t q = wave; q < nf; q += nw) {
        const int64_t u = front[q];
        const int64_t b = rp[u], e = rp[u + 1];
        if (e - b > BC_LONG) continue;   // bc_push_chunks
        bc_push_range(ci, b, e, cur[u], sigma[u * 64 + lane], unvis, sigma, next, lane);
    }
}

// Push for the frontier's hub vertices, one wave per chunk.
__device__ __forceinline__ void bc_push_chunks(const int32_t *__restrict__ ci, const RowChunks &ch,
                                                        const uint64_t *__restrict__ cur,
                                                        uint64_t *__restrict__ next,
                                                        const uint64_t *__restrict__ unvis,
                                                        double *__restrict__ sigma)
{
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / 64;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / 64;
    const unsigned lane = lane_id();
    for (int64_t c = wave; c < ch.n; c += nw) {
        const int64_t u = ch.row[c];
        const uint64_t fm = cur[u];
        if (fm == 0) continue;
        bc_push_range(ci, ch.beg[c], ch.end[c], fm, sigma[u * 64 + lane], unvis, sigma, next, lane);
    }
}

// After a level: unvis &= ~next; the vertices with a new mask form the next
// frontier list and those with unreached lanes and in-edges (rows of rpT,
// the pull side) the active list; cnt[0..3] += frontier size, its
// out-degree sum (rp), active size, its in-degree sum.  Workgroup g owns the g-th contiguous share of the vertices: it
// counts, reserves its ranges with one atomic per counter and writes its
// vertices in ascending order.
__global__ __launch_bounds__(256) void k_bc_compact(const int64_t *__restrict__ rp,
                                                    const int64_t *__restrict__ rpT, int64_t n,
                                                    const uint64_t *__restrict__ next, uint64_t *__restrict__ unvis,
                                                    int32_t *__restrict__ flist, int32_t *__restrict__ alist,
                                                    unsigned long long *__restrict__ cnt)
{
    __shared__ unsigned sf[256], sa[256];
    __shared__ unsigned long long base_f, base_a, sum_ef, sum_ea;
    const int64_t share = (n + gridDim.x - 1) / gridDim.x;
    const int64_t v0 = (int64_t)blockIdx.x * share, v1 = min(n, v0 + share);
    unsigned cf = 0, ca = 0;
    unsigned long long ef = 0, ea = 0;
    for (int64_t v = v0 + threadIdx.x; v < v1; v += 256) {
        const uint64_t nm = next[v];
        uint64_t uv = unvis[v];
        if (nm) {
            uv &= ~nm;
            unvis[v] = uv;
        }
        const int64_t deg = rp[v + 1] - rp[v], din = rpT[v + 1] - rpT[v];
        if (nm) {
            cf++;
            ef += (unsigned long long)deg;
        }
        if (uv && din) {
            ca++;
            ea += (unsigned long long)din;
        }
    }
    sf[threadIdx.x] = cf;
    sa[threadIdx.x] = ca;
    if (threadIdx.x == 0) sum_ef = sum_ea = 0;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
        const unsigned yf = (int)threadIdx.x >= o ? sf[threadIdx.x - o] : 0u;
        const unsigned ya = (int)threadIdx.x >= o ? sa[threadIdx.x - o] : 0u;
        __syncthreads();
        sf[threadIdx.x] += yf;
        sa[threadIdx.x] += ya;
        __syncthreads();
    }
    for (int o = 32; o > 0; o >>= 1) {
        ef += __shfl_xor(ef, o, 64);
        ea += __shfl_xor(ea, o, 64);
    }
    if (lane_id() == 0) {
        if (ef) atomicAdd(&sum_ef, ef);
        if (ea) atomicAdd(&sum_ea, ea);
    }
    if (threadIdx.x == 255) {
        base_f = sf[255] ? atomicAdd(&cnt[0], (unsigned long long)sf[255]) : 0;
        base_a = sa[255] ? atomicAdd(&cnt[2], (unsigned long long)sa[255]) : 0;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        if (sum_ef) atomicAdd(&cnt[1], sum_ef);
        if (sum_ea) atomicAdd(&cnt[3], sum_ea);
    }
    unsigned long long pf = base_f + sf[threadIdx.x] - cf, pa = base_a + sa[threadIdx.x] - ca;
    for (int64_t v = v0 + threadIdx.x; v < v1; v += 256) {
        const uint64_t nm = next[v], uv = unvis[v];
        if (nm) flist[pf++] = (int32_t)v;
        if (uv && rpT[v + 1] > rpT[v]) alist[pa++] = (int32_t)v;
    }
}

// Backward targets: one wave per vertex of level i-1's list (rows of at
// most BC_LONG neighbours).
__device__ __forceinline__ void bc_backward_rows(const int64_t *__restrict__ rp,
                                                     const int32_t *__restrict__ ci,
                                                     const int32_t *__restrict__ tlist, int64_t nt,
                                                     const uint64_t *__restrict__ at_i,   // depth i
                                                     const uint64_t *__restrict__ at_im1, // depth i-1
                                                     int has_deeper, int gshift,
                                                     const double *__restrict__ sigma,
                                                     double *__restrict__ W,
                                                     double *__restrict__ centrality)
{
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / 64;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / 64;
    const unsigned lane = lane_id();
    for (int64_t q = wave; q < nt; q += nw) {
        const int64_t v = tlist[q];
        const int64_t b = rp[v], e = rp[v + 1];
        if (e - b > BC_LONG) continue;   // bc_backward_chunks
        const uint64_t dm = at_im1[v];
        double acc = 0.0;
        if (has_deeper) {
            for (int64_t p0 = b; p0 < e; p0 += 64) {
                const int64_t p = p0 + lane;
                int32_t w = 0;
                uint64_t fm = 0;
                if (p < e) {
                    w = ci[p];
                    fm = at_i[w] & dm;
                }
                acc = gather_hits(__ballot(fm != 0), w, fm, W, lane, acc);
            }
        }
        const bool mine = (dm >> lane) & 1ull;
        double delta = 0.0;
        if (mine) {
            const double s = sigma[v * 64 + lane];
            delta = s * acc;
            W[v * 64 + lane] = (1.0 + delta) / s;
        }
        group_add(delta, gshift, lane, centrality, v);
    }
}

// Hub vertices (more than BC_LONG neighbours): every chunk of the neighbour
// list is gathered by its own wave into partial[chunk][lane]; the combine
// kernels add a vertex's chunk partials in chunk order and finish the
// level exactly as the per-vertex kernels do.
__device__ __forceinline__ double gather_lanes(const int32_t *__restrict__ ci, int64_t b, int64_t e,
                                               const uint64_t *__restrict__ lvl, uint64_t want,
                                               const double *__restrict__ val, unsigned lane)
{
    double acc = 0.0;
    for (int64_t p0 = b; p0 < e; p0 += 64) {
        const int64_t p = p0 + lane;
        int32_t u = 0;
        uint64_t fm = 0;
        if (p < e) {
            u = ci[p];
            fm = lvl[u] & want;
        }
        acc = gather_hits(__ballot(fm != 0), u, fm, val, lane, acc);
    }
    return acc;
}

__device__ __forceinline__ void bc_forward_chunks(const int32_t *__restrict__ ci, const RowChunks &ch,
                                                           const uint64_t *__restrict__ cur,
                                                           const uint64_t *__restrict__ unvis,
                                                           const double *__restrict__ sigma,
                                                           double *__restrict__ partial)
{
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / 64;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / 64;
    const unsigned lane = lane_id();
    for (int64_t c = wave; c < ch.n; c += nw) {
        const uint64_t uv = unvis[ch.row[c]];
        if (uv == 0) continue;
        partial[c * 64 + lane] = gather_lanes(ci, ch.beg[c], ch.end[c], cur, uv, sigma, lane);
    }
}

__global__ __launch_bounds__(256) void k_bc_forward_combine(const int64_t *__restrict__ rp, RowChunks ch,
                                                            const double *__restrict__ partial,
                                                            uint64_t *__restrict__ next,
                                                            const uint64_t *__restrict__ unvis,
                                                            double *__restrict__ sigma)
{
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / 64;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / 64;
    const unsigned lane = lane_id();
    for (int64_t c = wave; c < ch.n; c += nw) {
        const int64_t v = ch.row[c];
        if (ch.beg[c] != rp[v]) continue;   // first chunk of its vertex only
        const uint64_t uv = unvis[v];
        if (uv == 0) continue;
        const int64_t k = (rp[v + 1] - rp[v] + BC_CHUNK - 1) / BC_CHUNK;
        double acc = 0.0;
        for (int64_t q = 0; q < k; q++) acc += partial[(c + q) * 64 + lane];
        const uint64_t nw_mask = __ballot(acc > 0.0) & uv;
        if ((nw_mask >> lane) & 1ull) sigma[v * 64 + lane] = acc;
        if (lane == 0 && nw_mask) next[v] = nw_mask;
    }
}

__device__ __forceinline__ void bc_backward_chunks(const int32_t *__restrict__ ci, const RowChunks &ch,
                                                            const uint64_t *__restrict__ at_i,
                                                            const uint64_t *__restrict__ at_im1,
                                                            const double *__restrict__ W,
                                                            double *__restrict__ partial)
{
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / 64;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / 64;
    const unsigned lane = lane_id();
    for (int64_t c = wave; c < ch.n; c += nw) {
        const uint64_t dm = at_im1[ch.row[c]];
        if (dm == 0) continue;
        partial[c * 64 + lane] = gather_lanes(ci, ch.beg[c], ch.end[c], at_i, dm, W, lane);
    }
}

// A push level in one launch: the frontier's hub chunks, then its short
// rows.  Both read sigma of frontier vertices and add into sigma of
// unvisited ones (atomically): for each source lane the sets are disjoint.
__global__ __launch_bounds__(256) void k_bc_push(const int64_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                                 const int32_t *__restrict__ front, int64_t nf,
                                                 const uint64_t *__restrict__ cur, uint64_t *next,
                                                 const uint64_t *__restrict__ unvis, double *sigma, RowChunks ch)
{
    bc_push_chunks(ci, ch, cur, next, unvis, sigma);
    bc_push_rows(rp, ci, front, nf, cur, next, unvis, sigma);
}

// A pull level in one launch: the hub rows' chunks (a wave each, into
// partial), then the short rows.  The chunks read sigma of frontier
// vertices; the short rows write sigma of unvisited ones: for each source
// lane the two sets are disjoint.
__global__ __launch_bounds__(256) void k_bc_pull(const int64_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                                 const int32_t *__restrict__ act, int64_t na,
                                                 const uint64_t *__restrict__ cur, uint64_t *__restrict__ next,
                                                 const uint64_t *__restrict__ unvis, double *sigma, RowChunks ch,
                                                 double *__restrict__ partial)
{
    bc_forward_chunks(ci, ch, cur, unvis, sigma, partial);
    bc_pull_rows(rp, ci, act, na, cur, next, unvis, sigma);
}

// A backward level in one launch: the hub rows' chunks (with has_chunks),
// then the short rows.  Both read W of depth-i vertices; the short rows
// write W of depth-(i-1) ones: for each source lane the sets are disjoint.
__global__ __launch_bounds__(256) void k_bc_backward(const int64_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                                     const int32_t *__restrict__ tlist, int64_t nt,
                                                     const uint64_t *__restrict__ at_i,
                                                     const uint64_t *__restrict__ at_im1, int has_deeper,
                                                     int gshift, const double *__restrict__ sigma, double *W,
                                                     double *__restrict__ centrality, RowChunks ch, int has_chunks,
                                                     double *__restrict__ partial)
{
    if (has_chunks) bc_backward_chunks(ci, ch, at_i, at_im1, W, partial);
    bc_backward_rows(rp, ci, tlist, nt, at_i, at_im1, has_deeper, gshift, sigma, W, centrality);
}

__global__ __launch_bounds__(256) void k_bc_backward_combine(const int64_t *__restrict__ rp, RowChunks ch,
                                                             const uint64_t *__restrict__ at_im1,
                                                             int has_deeper, int gshift,
                                                             const double *__restrict__ partial,
                                                             const double *__restrict__ sigma,
                                                             double *__restrict__ W,
                                                             double *__restrict__ centrality)
{
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / 64;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / 64;
    const unsigned lane = lane_id();
    for (int64_t c = wave; c < ch.n; c += nw) {
        const int64_t v = ch.row[c];
        if (ch.beg[c] != rp[v]) continue;
        const uint64_t dm = at_im1[v];
        if (dm == 0) continue;
        double acc = 0.0;
        if (has_deeper) {
            const int64_t k = (rp[v + 1] - rp[v] + BC_CHUNK - 1) / BC_CHUNK;
            for (int64_t q = 0; q < k; q++) acc += partial[(c + q) * 64 + lane];
        }
        double delta = 0.0;
        if ((dm >> lane) & 1ull) {
            const double s = sigma[v * 64 + lane];
            delta = s * acc;
            W[v * 64 + lane] = (1.0 + delta) / s;
        }
        group_add(delta, gshift, lane, centrality, v);
    }
}


// ------------------------------------------------ multi-source BFS lanes
//
// Up to 64 breadth-first searches at once, one per lane, with the forward
// machinery of the betweenness batches but no path counts: a vertex
// reaches lane k at depth d + 1 when a neighbour is at depth d in lane k.

// Pull over the active list (rows of at most BC_LONG neighbours): OR of the
// neighbours' depth-d masks within the vertex's unreached lanes, stopping
// once every unreached lane is found.
__global__ __launch_bounds__(256) void k_ms_pull(const int64_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                                 const int32_t *__restrict__ act, int64_t na,
                                                 const uint64_t *__restrict__ cur, uint64_t *__restrict__ next,
                                                 const uint64_t *__restrict__ unvis)
{
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / 64;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / 64;
    const unsigned lane = lane_id();
    for (int64_t q = wave; q < na; q += nw) {
        const int64_t v = act[q];
        const int64_t b = rp[v], e = rp[v + 1];
        if (e - b > BC_LONG) continue;   // k_ms_pull_chunks
        const uint64_t uv = unvis[v];
        uint64_t acc = 0;
        for (int64_t p0 = b; p0 < e && acc != uv; p0 += 64) {
            const int64_t p = p0 + lane;
            uint64_t m = p < e ? (cur[ci[p]] & uv) : 0;
            for (int o = 32; o > 0; o >>= 1) m |= shfl64(m, (int)(lane ^ o));
            acc |= m;
        }
        if (lane == 0 && acc) next[v] = acc;
    }
}

// Pull for hub vertices with unreached lanes, one wave per chunk (OR-ed in).
__global__ __launch_bounds__(256) void k_ms_pull_chunks(const int32_t *__restrict__ ci, RowChunks ch,
                                                        const uint64_t *__restrict__ cur,
                                                        uint64_t *__restrict__ next,
                                                        const uint64_t *__restrict__ unvis)
{
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / 64;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / 64;
    const unsigned lane = lane_id();
    for (int64_t c = wave; c < ch.n; c += nw) {
        const int64_t v = ch.row[c];
        const uint64_t uv = unvis[v];
        if (uv == 0) continue;
        uint64_t acc = 0;
        for (int64_t p0 = ch.beg[c]; p0 < ch.end[c] && acc != uv; p0 += 64) {
            const int64_t p = p0 + lane;
            uint64_t m = p < ch.end[c] ? (cur[ci[p]] & uv) : 0;
            for (int o = 32; o > 0; o >>= 1) m |= shfl64(m, (int)(lane ^ o));
            acc |= m;
        }
        if (lane == 0 && acc) atomicOr((unsigned long long *)&next[v], (unsigned long long)acc);
    }
}

// Push from the frontier over the neighbour range [b, e) of u (lanes fm).
__device__ __forceinline__ void ms_push_range(const int32_t *__restrict__ ci, int64_t b, int64_t e, uint64_t fm,
                                              const uint64_t *__restrict__ unvis, uint64_t *__restrict__ next,
                                              unsigned lane)
{
    for (int64_t p = b + lane; p < e; p += 64) {
        const int32_t v = ci[p];
        const uint64_t m = unvis[v] & fm;
        if (m) atomicOr((unsigned long long *)&next[v], (unsigned long long)m);
    }
}

__global__ __launch_bounds__(256) void k_ms_push(const int64_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                                 const int32_t *__restrict__ front, int64_t nf,
                                                 const uint64_t *__restrict__ cur, uint64_t *__restrict__ next,
                                                 const uint64_t *__restrict__ unvis)
{
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / 64;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / 64;
    const unsigned lane = lane_id();
    for (int64_t q = wave; q < nf; q += nw) {
        const int64_t u = front[q];
        const int64_t b = rp[u], e = rp[u + 1];
        if (e - b > BC_LONG) continue;   // k_ms_push_chunks
        ms_push_range(ci, b, e, cur[u], unvis, next, lane);
    }
}

__global__ __launch_bounds__(256) void k_ms_push_chunks(const int32_t *__restrict__ ci, RowChunks ch,
                                                        const uint64_t *__restrict__ cur,
                                                        uint64_t *__restrict__ next,
                                                        const uint64_t *__restrict__ unvis)
{
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / 64;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / 64;
    const unsigned lane = lane_id();
    for (int64_t c = wave; c < ch.n; c += nw) {
        const uint64_t fm = cur[ch.row[c]];
        if (fm) ms_push_range(ci, ch.beg[c], ch.end[c], fm, unvis, next, lane);
    }
}

// Per lane k, over the vertices reached at depth d (the frontier list and
// their masks): stats[k] += count, stats[64 + k] += count * d, stats[128 +
// k] = max depth; with lev, lev[v * 64 + k] = d.  64 list entries per
// wave step; one set of atomics per workgroup.
__global__ __launch_bounds__(256) void k_ms_stats(const int32_t *__restrict__ front, int64_t nf,
                                                  const uint64_t *__restrict__ mask, int64_t d,
                                                  uint16_t *__restrict__ lev, unsigned long long *__restrict__ stats)
{
    __shared__ unsigned long long cnt[64];
    if (threadIdx.x < 64) cnt[threadIdx.x] = 0;
    __syncthreads();
    const unsigned lane = lane_id();
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / 64;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / 64;
    unsigned long long mine = 0;
    for (int64_t q0 = wave * 64; q0 < nf; q0 += nw * 64) {
        const int64_t q = q0 + lane;
        const int64_t v = q < nf ? front[q] : -1;
        const uint64_t x = v >= 0 ? mask[v] : 0;
        for (int k = 0; k < 64; k++) {
            const uint64_t bal = __ballot((x >> k) & 1ull);
            if ((int)lane == k) mine += (unsigned long long)__popcll(bal);
        }
        if (lev)
            for (int t = 0; t < 64; t++) {
                const int64_t vt = bcast64(v, t);
                if (vt < 0) break;
                const uint64_t xt = shfl64(x, t);
                if ((xt >> lane) & 1ull) lev[vt * 64 + lane] = (uint16_t)d;
            }
    }
    if (mine) atomicAdd(&cnt[lane], mine);
    __syncthreads();
    if (threadIdx.x < 64 && cnt[threadIdx.x]) {
        const unsigned long long c = cnt[threadIdx.x];
        atomicAdd(&stats[threadIdx.x], c);
        atomicAdd(&stats[64 + threadIdx.x], c * (unsigned long long)d);
        atomicMax(&stats[128 + threadIdx.x], (unsigned long long)d);
    }
}

__global__ void k_ms_sources(const int64_t *__restrict__ src, uint64_t *__restrict__ unvis,
                             uint64_t *__restrict__ mask0, unsigned long long *__restrict__ stats)
{
    const int k = threadIdx.x;
    if (k < 64) {
        stats[k] = 0;
        stats[64 + k] = 0;
        stats[128 + k] = 0;
        if (src[k] >= 0) {
            atomicAnd((unsigned long long *)&unvis[src[k]], ~(1ull << k));
            atomicOr((unsigned long long *)&mask0[src[k]], 1ull << k);
        }
    }
}

}  // namespace


// Betweenness of the 64-lane batches described by lane_src (HOST, 64
// entries per batch, -1 = idle lane), summed into cent: with gshift = 6 one
// value per vertex over every batch; with gshift = 3 one value per group of
// 8 lanes (cent is n x 8) -- the serving path, where each group is one
// query.  cent is zeroed here.
int bc_compute(lagr_ctx ctx, const lagr_graph G, const int64_t *lane_src, int nbatches, int gshift,
               double *cent, char *msg)
{
    const lagr_matrix A = G->A;
    const int64_t n = A->nrows;
    const size_t n1 = (size_t)(n > 0 ? n : 1);
    const int groups = 64 >> gshift;
    double *sigma = (double *)ws_get(ctx, WS_BC_SIGMA, sizeof(double) * 64 * n1);
    double *Wv = (double *)ws_get(ctx, WS_BC_W, sizeof(double) * 64 * n1);
    uint64_t *unvis = (uint64_t *)ws_get(ctx, WS_BC_UNVIS, sizeof(uint64_t) * n1);
    int32_t *acts = (int32_t *)ws_get(ctx, WS_BC_ACT, sizeof(int32_t) * 2 * n1);
    unsigned long long *cnt = (unsigned long long *)ws_get(ctx, WS_BC_CNT, 64);
    int64_t *dsrc = (int64_t *)ws_get(ctx, WS_BFS_D, sizeof(int64_t) * 64 + 64);
    if (!sigma || !Wv || !unvis || !acts || !cnt || !dsrc) return lagr_fail(msg, LAGR_OUT_OF_MEMORY, "bc workspace");
    int rc = LAGR_SUCCESS;
    // level d's lane masks (8 bytes per vertex) and vertex list (4 bytes per
    // vertex) share one context-owned buffer, reused across calls, so the
    // steady state allocates nothing per level
    const size_t mask_bytes = sizeof(uint64_t) * n1;
    const size_t lv_bytes = mask_bytes + sizeof(int32_t) * n1;
    if (ctx->lv_bytes < lv_bytes) {
        (void)hipStreamSynchronize(ctx->stream);
        for (void *p : ctx->lvpool) dev_free(p, ctx->lv_bytes);
        ctx->lvpool.clear();
        ctx->lv_bytes = lv_bytes;
    }
    std::vector<void *> &pool = ctx->lvpool;
    auto level_buf = [&](size_t d) -> uint64_t * {
        while (pool.size() <= d) {
            void *p = dev_alloc(ctx->lv_bytes);
            if (!p) return nullptr;
            pool.push_back(p);
        }
        return (uint64_t *)pool[d];
    };
    auto levels = [&](size_t d) { return (uint64_t *)pool[d]; };
    auto lists = [&](size_t d) { return (int32_t *)((char *)pool[d] + mask_bytes); };
    auto cleanup = [&]() { (void)hipStreamSynchronize(ctx->stream); };
#define BC_TRY(expr)       \
    do {                   \
        rc = (expr);       \
        if (rc < 0) {      \
            cleanup();     \
            return rc;     \
        }                  \
    } while (0)
#define BC_LAUNCHED()                                                               \
    do {                                                                            \
        if (hipGetLastError() != hipSuccess)                                        \
            BC_TRY(lagr_fail(msg, LAGR_DEVICE_ERROR, "bc kernel launch failed"));   \
    } while (0)

    BC_TRY(fill_i64(ctx, (int64_t *)cent, n * groups, 0, msg));   // 0.0 has all-zero bits
    // push and the backward sweep read out-edges (A); pull reads in-edges
    // (AT, which is A itself for an undirected graph)
    const lagr_matrix AT = graph_in_edges(G);
    if (!AT) BC_TRY(lagr_fail(msg, LAGR_PROPERTY_MISSING, "the transpose of a directed graph is missing"));
    RowChunks ch, chT;
    BC_TRY(graph_chunks(G, ctx, &ch, msg));
    BC_TRY(graph_chunks_in(G, ctx, &chT, msg));
    double *partial = nullptr;
    unsigned cblocks = 1, cblocksT = 1;
    if (ch.n > 0 || chT.n > 0) {
        const int64_t most = ch.n > chT.n ? ch.n : chT.n;
        partial = (double *)ws_get(ctx, WS_BC_MASKS, sizeof(double) * 64 * (size_t)most);
        if (!partial) BC_TRY(lagr_fail(msg, LAGR_OUT_OF_MEMORY, "bc chunk partials"));
        cblocks = grid_for(ch.n * 64, 256, 16384);
        cblocksT = grid_for(chT.n * 64, 256, 16384);
    }
    const unsigned compact_blocks = (unsigned)(n > 0 ? (ctx->num_cus < n ? ctx->num_cus : n) : 1);
    int32_t *act_cur = acts, *act_next = acts + n1;
    // compaction after a level: returns frontier size / degree sum, active
    // size / degree sum
    unsigned long long h[4];
    auto compact = [&](const uint64_t *next, int32_t *flist) -> int {
        TRY(fill_i64(ctx, (int64_t *)cnt, 4, 0, msg));
        if (n > 0) {
            hipLaunchKernelGGL(k_bc_compact, dim3(compact_blocks), dim3(256), 0, ctx->stream, A->rowptr, AT->rowptr, n, next,
                               unvis, flist, act_next, cnt);
            LAUNCH_CHECK();
        }
        TRY(read_back(ctx, h, cnt, sizeof(h), msg));
        std::swap(act_cur, act_next);
        return LAGR_SUCCESS;
    };
    auto wgrid = [](int64_t items) { return grid_for(items * 64, 256, 16384); };
    std::vector<int64_t> nlev;
    for (int b = 0; b < nbatches; b++) {
        const int64_t *src = lane_src + 64 * b;
        uint64_t lanes = 0;
        for (int k = 0; k < 64; k++)
            if (src[k] >= 0) lanes |= 1ull << k;
        if (!lanes) continue;
        uint64_t *m0 = level_buf(0);
        if (!m0) BC_TRY(lagr_fail(msg, LAGR_OUT_OF_MEMORY, "bc level buffers"));
        if (hipMemcpyAsync(dsrc, src, sizeof(int64_t) * 64, hipMemcpyHostToDevice, ctx->stream) !=
            hipSuccess)
            BC_TRY(lagr_fail(msg, LAGR_DEVICE_ERROR, "bc sources copy"));
        // push adds into sigma, so every unreached (vertex, lane) starts at 0
        BC_TRY(fill_i64(ctx, (int64_t *)sigma, n * 64, 0, msg));
        hipLaunchKernelGGL(k_bc_init, dim3(grid_for(n, 256, 8192)), dim3(256), 0, ctx->stream, n,
                           lanes, unvis, m0);
        BC_LAUNCHED();
        hipLaunchKernelGGL(k_bc_sources, dim3(1), dim3(64), 0, ctx->stream, dsrc, unvis, m0, sigma);
        BC_LAUNCHED();
        BC_TRY(compact(m0, lists(0)));
        nlev.assign(1, (int64_t)h[0]);
        // forward sweep: depth d -> d + 1 until no lane advances
        size_t depth = 0;
        while (true) {
            const int64_t nf = (int64_t)h[0], ef = (int64_t)h[1], na = (int64_t)h[2], ea = (int64_t)h[3];
            uint64_t *next = level_buf(depth + 1);
            if (!next) BC_TRY(lagr_fail(msg, LAGR_OUT_OF_MEMORY, "bc level buffers"));
            BC_TRY(fill_i64(ctx, (int64_t *)next, n, 0, msg));
            const bool push = ef * BC_PUSH_RATIO < ea;
            if (push) {
                const unsigned qg = ch.n > 0 && cblocks > wgrid(nf) ? cblocks : wgrid(nf);
                TIMED(ctx, "bc_forward",
                      hipLaunchKernelGGL(k_bc_push, dim3(qg), dim3(256), 0, ctx->stream, A->rowptr, A->colidx,
                                         lists(depth), nf, levels(depth), next, unvis, sigma, ch));
                BC_LAUNCHED();
            } else if (na > 0) {
                const unsigned pg = chT.n > 0 && cblocksT > wgrid(na) ? cblocksT : wgrid(na);
                TIMED(ctx, "bc_forward",
                      hipLaunchKernelGGL(k_bc_pull, dim3(pg), dim3(256), 0, ctx->stream, AT->rowptr, AT->colidx,
                                         act_cur, na, levels(depth), next, unvis, sigma, chT, partial));
                BC_LAUNCHED();
                if (chT.n > 0) {
                    hipLaunchKernelGGL(k_bc_forward_combine, dim3(cblocksT), dim3(256), 0, ctx->stream,
                                       AT->rowptr, chT, partial, next, unvis, sigma);
                    BC_LAUNCHED();
                }
            }
            BC_TRY(compact(next, lists(depth + 1)));
            if (h[0] == 0) break;
            depth++;
            nlev.push_back((int64_t)h[0]);
        }
        // backward sweep: targets at depth i-1 gather from depth i
        for (size_t i = depth + 1; i >= 2; i--) {
            const int has_deeper = i <= depth ? 1 : 0;
            const uint64_t *at_i = has_deeper ? levels(i) : levels(i - 1);
            const int64_t nt = nlev[i - 1];
            const int has_chunks = ch.n > 0 && has_deeper ? 1 : 0;
            const unsigned bg = has_chunks && cblocks > wgrid(nt) ? cblocks : wgrid(nt);
            TIMED(ctx, "bc_backward",
                  hipLaunchKernelGGL(k_bc_backward, dim3(bg), dim3(256), 0, ctx->stream, A->rowptr, A->colidx,
                                     lists(i - 1), nt, at_i, levels(i - 1), has_deeper, gshift, sigma, Wv, cent,
                                     ch, has_chunks, partial));
            BC_LAUNCHED();
            if (ch.n > 0) {
                hipLaunchKernelGGL(k_bc_backward_combine, dim3(cblocks), dim3(256), 0, ctx->stream,
                                   A->rowptr, ch, levels(i - 1), has_deeper, gshift, partial, sigma,
                                   Wv, cent);
                BC_LAUNCHED();
            }
        }
    }
    cleanup();
#undef BC_TRY
#undef BC_LAUNCHED
    return LAGR_SUCCESS;
}


// Multi-source BFS over the lanes of lane_src (HOST, 64, -1 idle): per lane
// the number of reached vertices (the source included), the sum of their
// levels and the largest level into stats[3][64] (host); with lev
// (n x 64 uint16), every reached (vertex, lane)'s level, 0xFFFF elsewhere.
int msbfs_compute(lagr_ctx ctx, const lagr_graph G, const int64_t *lane_src, uint16_t *lev, int64_t *stats,
                  char *msg)
{
    const lagr_matrix A = G->A;
    const int64_t n = A->nrows;
    const size_t n1 = (size_t)(n > 0 ? n : 1);
    uint64_t *unvis = (uint64_t *)ws_get(ctx, WS_BC_UNVIS, sizeof(uint64_t) * n1);
    int32_t *acts = (int32_t *)ws_get(ctx, WS_BC_ACT, sizeof(int32_t) * 2 * n1);
    unsigned long long *cnt = (unsigned long long *)ws_get(ctx, WS_BC_CNT, 64);
    int64_t *dsrc = (int64_t *)ws_get(ctx, WS_BFS_D, sizeof(int64_t) * 64 + 64);
    unsigned long long *dstats = (unsigned long long *)ws_get(ctx, WS_BFS_E, sizeof(int64_t) * 3 * 64);
    if (!unvis || !acts || !cnt || !dsrc || !dstats) return lagr_fail(msg, LAGR_OUT_OF_MEMORY, "msbfs workspace");
    // two (mask, list) buffers of the context's level pool, used in turn
    const size_t mask_bytes = sizeof(uint64_t) * n1;
    const size_t lv_bytes = mask_bytes + sizeof(int32_t) * n1;
    if (ctx->lv_bytes < lv_bytes) {
        TRY(hipStreamSynchronize(ctx->stream) == hipSuccess ? LAGR_SUCCESS
                                                            : lagr_fail(msg, LAGR_DEVICE_ERROR, "sync"));
        for (void *p : ctx->lvpool) dev_free(p, ctx->lv_bytes);
        ctx->lvpool.clear();
        ctx->lv_bytes = lv_bytes;
    }
    while (ctx->lvpool.size() < 2) {
        void *p = dev_alloc(ctx->lv_bytes);
        if (!p) return lagr_fail(msg, LAGR_OUT_OF_MEMORY, "msbfs level buffers");
        ctx->lvpool.push_back(p);
    }
    auto mask_of = [&](int b) { return (uint64_t *)ctx->lvpool[b]; };
    auto list_of = [&](int b) { return (int32_t *)((char *)ctx->lvpool[b] + mask_bytes); };
    uint64_t lanes = 0;
    for (int k = 0; k < 64; k++)
        if (lane_src[k] >= 0) lanes |= 1ull << k;
    RowChunks ch;
    TRY(graph_chunks(G, ctx, &ch, msg));
    const unsigned cblocks = ch.n > 0 ? grid_for(ch.n * 64, 256, 16384) : 1;
    const unsigned compact_blocks = (unsigned)(n > 0 ? (ctx->num_cus < n ? ctx->num_cus : n) : 1);
    int32_t *act_cur = acts, *act_next = acts + n1;
    unsigned long long h[4];
    auto compact = [&](const uint64_t *next, int32_t *flist) -> int {
        TRY(fill_i64(ctx, (int64_t *)cnt, 4, 0, msg));
        if (n > 0) {
            hipLaunchKernelGGL(k_bc_compact, dim3(compact_blocks), dim3(256), 0, ctx->stream, A->rowptr, A->rowptr, n, next,
                               unvis, flist, act_next, cnt);
            LAUNCH_CHECK();
        }
        TRY(read_back(ctx, h, cnt, sizeof(h), msg));
        std::swap(act_cur, act_next);
        return LAGR_SUCCESS;
    };
    auto wgrid = [](int64_t items) { return grid_for(items * 64, 256, 16384); };
    auto stats_of = [&](const int32_t *flist, int64_t nf, const uint64_t *mask, int64_t d) -> int {
        if (nf > 0) {
            hipLaunchKernelGGL(k_ms_stats, dim3(grid_for(nf, 256, 256)), dim3(256), 0, ctx->stream, flist, nf, mask,
                               d, lev, dstats);
            LAUNCH_CHECK();
        }
        return LAGR_SUCCESS;
    };
    HIP_TRY(hipMemcpyAsync(dsrc, lane_src, sizeof(int64_t) * 64, hipMemcpyHostToDevice, ctx->stream));
    if (lev) TRY(fill_u32(ctx, (uint32_t *)lev, n * 32, 0xFFFFFFFFu, msg));
    uint64_t *m0 = mask_of(0);
    hipLaunchKernelGGL(k_bc_init, dim3(grid_for(n, 256, 8192)), dim3(256), 0, ctx->stream, n, lanes, unvis, m0);
    hipLaunchKernelGGL(k_ms_sources, dim3(1), dim3(64), 0, ctx->stream, dsrc, unvis, m0, dstats);
    LAUNCH_CHECK();
    TRY(compact(m0, list_of(0)));
    TRY(stats_of(list_of(0), (int64_t)h[0], m0, 0));
    int b = 0;
    for (int64_t d = 1; d < 65535; d++) {
        const int64_t nf = (int64_t)h[0], ef = (int64_t)h[1], na = (int64_t)h[2], ea = (int64_t)h[3];
        uint64_t *cur = mask_of(b), *next = mask_of(b ^ 1);
        TRY(fill_i64(ctx, (int64_t *)next, n, 0, msg));
        if (ef * BC_PUSH_RATIO < ea) {
            hipLaunchKernelGGL(k_ms_push, dim3(wgrid(nf)), dim3(256), 0, ctx->stream, A->rowptr, A->colidx,
                               list_of(b), nf, cur, next, unvis);
            if (ch.n > 0)
                hipLaunchKernelGGL(k_ms_push_chunks, dim3(cblocks), dim3(256), 0, ctx->stream, A->colidx, ch, cur,
                                   next, unvis);
        } else if (na > 0) {
            hipLaunchKernelGGL(k_ms_pull, dim3(wgrid(na)), dim3(256), 0, ctx->stream, A->rowptr, A->colidx,
                               act_cur, na, cur, next, unvis);
            if (ch.n > 0)
                hipLaunchKernelGGL(k_ms_pull_chunks, dim3(cblocks), dim3(256), 0, ctx->stream, A->colidx, ch, cur,
                                   next, unvis);
        }
        LAUNCH_CHECK();
        TRY(compact(next, list_of(b ^ 1)));
        if (h[0] == 0) break;
        TRY(stats_of(list_of(b ^ 1), (int64_t)h[0], next, d));
        b ^= 1;
    }
    TRY(stage_to_host(ctx, 0, dstats, 8 * 3 * 64, true, msg));
    memcpy(stats, ctx->pinned, 8 * 3 * 64);
    return LAGR_SUCCESS;
}

extern "C" int lagr_bc(lagr_vector *centrality_out, const lagr_graph G, const int64_t *sources,
                       int32_t ns, lagr_ctx ctx, char *msg)
{
    if (!centrality_out || !G || !ctx) return lagr_fail(msg, LAGR_NULL_POINTER, "NULL argument");
    *centrality_out = nullptr;
    if (ns < 0 || (ns > 0 && !sources)) return lagr_fail(msg, LAGR_INVALID_VALUE, "bad sources");
    const int64_t n = G->A->nrows;
    for (int32_t k = 0; k < ns; k++)
        if (sources[k] < 0 || sources[k] >= n)
            return lagr_fail(msg, LAGR_INVALID_INDEX, "source %lld out of range", (long long)sources[k]);
    // pull steps of a directed graph read its transpose
    TRY(graph_ensure_at(G, ctx, msg));
    // one source per lane, batches of 64 summed in order
    const int nbatches = (ns + 63) / 64;
    std::vector<int64_t> lane_src((size_t)64 * (nbatches > 0 ? nbatches : 1), -1);
    for (int32_t k = 0; k < ns; k++) lane_src[k] = sources[k];
    lagr_vector cv = new (std::nothrow) lagr_vector_s();
    if (!cv) return lagr_fail(msg, LAGR_OUT_OF_MEMORY, "vector");
    cv->type = LAGR_FP64;
    cv->n = n;
    cv->fmt = LAGR_VEC_FULL;
    cv->nvals = n;
    cv->values_bytes = sizeof(double) * (size_t)(n > 0 ? n : 1);
    cv->values = dev_alloc(cv->values_bytes);
    if (!cv->values) {
        delete cv;
        return lagr_fail(msg, LAGR_OUT_OF_MEMORY, "centrality");
    }
    const int rc = bc_compute(ctx, G, lane_src.data(), nbatches, 6, (double *)cv->values, msg);
    if (rc < 0) {
        lagr_vector_free(&cv);
        return rc;
    }
    *centrality_out = cv;
    return lagr_ok(msg);
}
