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
// BC, after Beamer), taken on the device from the counts the previous
// level's compaction left, so the host queues a chunk of levels at once and
// reads the frontier sizes once per chunk instead of once per level:
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
// A backward level pushes (BC_BACKWARD_AUTO) when its edges are fewer than
// the next shallower level's / BC_BACK_PUSH_RATIO (its atomics cost more
// per edge than the gather's loads).
constexpr int64_t BC_BACK_PUSH_RATIO = 4;
// forward levels: the fixed grid, the levels queued before the host first
// reads the frontier sizes, then per further read, and the ring of level
// counters (larger than a chunk plus one)
constexpr unsigned BC_FORWARD_GRID = 8192;
constexpr size_t BC_FIRST_LEVELS = 8;
constexpr size_t BC_MORE_LEVELS = 4;
constexpr size_t BC_RING = 16;

// A forward level's direction from its counts c = {frontier size, its
// out-degree sum, active size, its in-degree sum}, which the compaction of
// the previous level left on the device: 0 the frontier is empty (the sweep
// is over), 1 push (the frontier's edges are fewer than the active
// vertices' edges / BC_PUSH_RATIO), 2 pull, 3 nothing (no active vertex).
__device__ __forceinline__ int bc_direction(const unsigned long long *__restrict__ c)
{
    const unsigned long long nf = c[0], ef = c[1], na = c[2], ea = c[3];
    if (nf == 0) return 0;
    if (ef * (unsigned long long)BC_PUSH_RATIO < ea) return 1;
    return na > 0 ? 2 : 3;
}


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
// With cin (the counts of the level that wrote next), a level whose
// frontier was empty compacts nothing.
__global__ __launch_bounds__(256) void k_bc_compact(const int64_t *__restrict__ rp,
                                                    const int64_t *__restrict__ rpT, int64_t n,
                                                    const uint64_t *__restrict__ next, uint64_t *__restrict__ unvis,
                                                    int32_t *__restrict__ flist, int32_t *__restrict__ alist,
                                                    unsigned long long *__restrict__ cnt,
                                                    const unsigned long long *__restrict__ cin)
{
    if (cin && cin[0] == 0) return;
    __shared__ unsigned wf[4], wa[4];
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
    if (threadIdx.x == 0) sum_ef = sum_ea = 0;
    unsigned tf, ta;
    const unsigned xf = block_excl_scan256(cf, wf, tf);
    const unsigned xa = block_excl_scan256(ca, wa, ta);
    ef = wave_sum64(ef);
    ea = wave_sum64(ea);
    if (lane_id() == 0) {
        if (ef) atomicAdd(&sum_ef, ef);
        if (ea) atomicAdd(&sum_ea, ea);
    }
    if (threadIdx.x == 0) {
        base_f = tf ? atomicAdd(&cnt[0], (unsigned long long)tf) : 0;
        base_a = ta ? atomicAdd(&cnt[2], (unsigned long long)ta) : 0;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        if (sum_ef) atomicAdd(&cnt[1], sum_ef);
        if (sum_ea) atomicAdd(&cnt[3], sum_ea);
    }
    unsigned long long pf = base_f + xf, pa = base_a + xa;
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
                                                            double *__restrict__ sigma,
                                                            const unsigned long long *__restrict__ c)
{
    if (bc_direction(c) != 2) return;   // only after a pull
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

// A forward level in one launch, its direction taken on the device: push
// over the frontier list (rows of A, hub chunks first), or pull over the
// active list (rows of AT, the hub rows' chunks into partial first).
__global__ __launch_bounds__(256) void k_bc_forward(const int64_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                                    const int64_t *__restrict__ rpT, const int32_t *__restrict__ ciT,
                                                    const int32_t *__restrict__ front,
                                                    const int32_t *__restrict__ act,
                                                    const uint64_t *__restrict__ cur, uint64_t *next,
                                                    const uint64_t *__restrict__ unvis, double *sigma, RowChunks ch,
                                                    RowChunks chT, double *__restrict__ partial,
                                                    const unsigned long long *__restrict__ c)
{
    const int dir = bc_direction(c);
    if (dir == 1) {
        bc_push_chunks(ci, ch, cur, next, unvis, sigma);
        bc_push_rows(rp, ci, front, (int64_t)c[0], cur, next, unvis, sigma);
    } else if (dir == 2) {
        bc_forward_chunks(ciT, chT, cur, unvis, sigma, partial);
        bc_pull_rows(rpT, ciT, act, (int64_t)c[2], cur, next, unvis, sigma);
    }
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

// ---------------------------------------------- backward sweep, push form
//
// The push form of a backward level (W = W B, Section IV-B): every vertex
// w at depth i scatters its W(w) into the accumulators of its in-neighbours
// v at depth i-1, lane by lane, with FP64 atomics -- so the order of the
// additions, and the last bits of the result, vary from run to run (the
// pull form above adds in a fixed order).  The accumulators are the W
// slots of the depth-(i-1) lanes, cleared first; a finishing pass then
// turns each into delta = sigma * sum and W = (1 + delta) / sigma, as the
// pull form does in one pass.

// W[v][lanes at depth i-1] = 0 for the vertices of level i-1.
__global__ __launch_bounds__(256) void k_bc_back_clear(const int32_t *__restrict__ tlist, int64_t nt,
                                                       const uint64_t *__restrict__ at_im1, double *__restrict__ W)
{
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / 64;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / 64;
    const unsigned lane = lane_id();
    for (int64_t q = wave; q < nt; q += nw) {
        const int64_t v = tlist[q];
        if ((at_im1[v] >> lane) & 1ull) W[v * 64 + lane] = 0.0;
    }
}

// Scatter of the in-neighbour range [b, e) of w (lanes fm, this lane's
// value wl): 64 neighbours loaded at once, then every one with a lane
// at depth i-1 taken in turn by the whole wave.
__device__ __forceinline__ void back_push_range(const int32_t *__restrict__ ciT, int64_t b, int64_t e, uint64_t fm,
                                                double wl, const uint64_t *__restrict__ at_im1, double *W,
                                                unsigned lane)
{
    for (int64_t p0 = b; p0 < e; p0 += 64) {
        const int64_t p = p0 + lane;
        int32_t v = 0;
        uint64_t hm = 0;
        if (p < e) {
            v = ciT[p];
            hm = at_im1[v] & fm;
        }
        uint64_t hits = __ballot(hm != 0);
        while (hits) {
            const int t = __ffsll((unsigned long long)hits) - 1;
            hits &= hits - 1;
            const int32_t vv = __shfl(v, t, 64);
            const uint64_t mm = shfl64(hm, t);
            if ((mm >> lane) & 1ull)
                __hip_atomic_fetch_add(W + (int64_t)vv * 64 + lane, wl, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// One wave per vertex of level i (rows of at most BC_LONG in-neighbours),
// then one wave per chunk of the longer rows.
__global__ __launch_bounds__(256) void k_bc_back_push(const int64_t *__restrict__ rpT, const int32_t *__restrict__ ciT,
                                                      const int32_t *__restrict__ slist, int64_t ns,
                                                      const uint64_t *__restrict__ at_i,
                                                      const uint64_t *__restrict__ at_im1, double *W, RowChunks chT)
{
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / 64;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / 64;
    const unsigned lane = lane_id();
    for (int64_t q = wave; q < ns; q += nw) {
        const int64_t w = slist[q];
        const int64_t b = rpT[w], e = rpT[w + 1];
        if (e - b > BC_LONG) continue;   // its chunks below
        const uint64_t fm = at_i[w];
        const double wl = (fm >> lane) & 1ull ? W[w * 64 + lane] : 0.0;
        back_push_range(ciT, b, e, fm, wl, at_im1, W, lane);
    }
    for (int64_t c = wave; c < chT.n; c += nw) {
        const int64_t w = chT.row[c];
        const uint64_t fm = at_i[w];
        if (fm == 0) continue;
        const double wl = (fm >> lane) & 1ull ? W[w * 64 + lane] : 0.0;
        back_push_range(ciT, chT.beg[c], chT.end[c], fm, wl, at_im1, W, lane);
    }
}

// delta and W of the vertices of level i-1 from their accumulated sums.
__global__ __launch_bounds__(256) void k_bc_back_finish(const int32_t *__restrict__ tlist, int64_t nt,
                                                        const uint64_t *__restrict__ at_im1, int gshift,
                                                        const double *__restrict__ sigma, double *__restrict__ W,
                                                        double *__restrict__ centrality)
{
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / 64;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / 64;
    const unsigned lane = lane_id();
    for (int64_t q = wave; q < nt; q += nw) {
        const int64_t v = tlist[q];
        const uint64_t dm = at_im1[v];
        double delta = 0.0;
        if ((dm >> lane) & 1ull) {
            const double s = sigma[v * 64 + lane];
            delta = s * W[v * 64 + lane];
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

// A multi-source level in one launch, its direction taken on the device
// from its counts c (bc_direction): push over the frontier list (hub
// chunks, then short rows) or pull over the active list (short rows, then
// the hub rows' chunks).
__global__ __launch_bounds__(256) void k_ms_forward(const int64_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                                    const int32_t *__restrict__ front,
                                                    const int32_t *__restrict__ act,
                                                    const uint64_t *__restrict__ cur, uint64_t *__restrict__ next,
                                                    const uint64_t *__restrict__ unvis, RowChunks ch,
                                                    const unsigned long long *__restrict__ c)
{
    const int dir = bc_direction(c);
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / 64;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / 64;
    const unsigned lane = lane_id();
    if (dir == 1) {
        for (int64_t k = wave; k < ch.n; k += nw) {
            const uint64_t fm = cur[ch.row[k]];
            if (fm) ms_push_range(ci, ch.beg[k], ch.end[k], fm, unvis, next, lane);
        }
        const int64_t nf = (int64_t)c[0];
        for (int64_t q = wave; q < nf; q += nw) {
            const int64_t u = front[q];
            const int64_t b = rp[u], e = rp[u + 1];
            if (e - b > BC_LONG) continue;   // its chunks above
            ms_push_range(ci, b, e, cur[u], unvis, next, lane);
        }
    } else if (dir == 2) {
        const int64_t na = (int64_t)c[2];
        for (int64_t q = wave; q < na; q += nw) {
            const int64_t v = act[q];
            const int64_t b = rp[v], e = rp[v + 1];
            if (e - b > BC_LONG) continue;   // its chunks below
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
        for (int64_t k = wave; k < ch.n; k += nw) {
            const int64_t v = ch.row[k];
            const uint64_t uv = unvis[v];
            if (uv == 0) continue;
            uint64_t acc = 0;
            for (int64_t p0 = ch.beg[k]; p0 < ch.end[k] && acc != uv; p0 += 64) {
                const int64_t p = p0 + lane;
                uint64_t m = p < ch.end[k] ? (cur[ci[p]] & uv) : 0;
                for (int o = 32; o > 0; o >>= 1) m |= shfl64(m, (int)(lane ^ o));
                acc |= m;
            }
            if (lane == 0 && acc) atomicOr((unsigned long long *)&next[v], (unsigned long long)acc);
        }
    }
}

// Per lane k, over the vertices reached at depth d (the frontier list and
// their masks): stats[k] += count, stats[64 + k] += count * d, stats[128 +
// k] = max depth; with lev, lev[v * 64 + k] = d.  64 list entries per
// wave step; one set of atomics per workgroup.
__global__ __launch_bounds__(256) void k_ms_stats(const int32_t *__restrict__ front,
                                                  const unsigned long long *__restrict__ c,
                                                  const uint64_t *__restrict__ mask, int64_t d,
                                                  uint16_t *__restrict__ lev, unsigned long long *__restrict__ stats)
{
    const int64_t nf = (int64_t)c[0];   // the level's size, from its counts
    if (nf == 0) return;
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
               double *cent, char *msg, int backward)
{
    ctx->last_bc_levels = 0;
    const lagr_matrix A = G->A;
    const int64_t n = A->nrows;
    const size_t n1 = (size_t)(n > 0 ? n : 1);
    const int groups = 64 >> gshift;
    double *sigma = (double *)ws_get(ctx, WS_BC_SIGMA, sizeof(double) * 64 * n1);
    double *Wv = (double *)ws_get(ctx, WS_BC_W, sizeof(double) * 64 * n1);
    uint64_t *unvis = (uint64_t *)ws_get(ctx, WS_BC_UNVIS, sizeof(uint64_t) * n1);
    int32_t *acts = (int32_t *)ws_get(ctx, WS_BC_ACT, sizeof(int32_t) * 2 * n1);
    unsigned long long *cnt = (unsigned long long *)ws_get(ctx, WS_BC_CNT, sizeof(unsigned long long) * 4 * BC_RING);
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
    // the active list of level d is acts + (d & 1) n1; the counts of level d
    // (frontier size and out-degree sum, active size and in-degree sum) are
    // slot d % BC_RING of the counter ring, written by the compaction of
    // level d - 1 and read on the device by level d's kernels
    auto act_of = [&](size_t d) { return acts + (d & 1) * n1; };
    auto slot = [&](size_t d) { return cnt + 4 * (d % BC_RING); };
    auto compact = [&](const uint64_t *next, size_t d_next, const unsigned long long *cin) -> int {
        if (n > 0) {
            hipLaunchKernelGGL(k_bc_compact, dim3(compact_blocks), dim3(256), 0, ctx->stream, A->rowptr, AT->rowptr,
                               n, next, unvis, lists(d_next), act_of(d_next), slot(d_next), cin);
            LAUNCH_CHECK();
        }
        return LAGR_SUCCESS;
    };
    auto wgrid = [](int64_t items) { return grid_for(items * 64, 256, 16384); };
    // forward levels run with a fixed grid (their loops stride over the
    // lists), so the host queues them without knowing the counts
    unsigned fgrid = BC_FORWARD_GRID;
    if (cblocks > fgrid) fgrid = cblocks;
    if (cblocksT > fgrid) fgrid = cblocksT;
    std::vector<int64_t> nlev, elev;
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
        BC_TRY(fill_i64(ctx, (int64_t *)cnt, 4 * BC_RING, 0, msg));
        hipLaunchKernelGGL(k_bc_init, dim3(grid_for(n, 256, 8192)), dim3(256), 0, ctx->stream, n,
                           lanes, unvis, m0);
        BC_LAUNCHED();
        hipLaunchKernelGGL(k_bc_sources, dim3(1), dim3(64), 0, ctx->stream, dsrc, unvis, m0, sigma);
        BC_LAUNCHED();
        BC_TRY(compact(m0, 0, nullptr));
        // forward sweep: depth d -> d + 1 until no lane advances, queued a
        // chunk of levels at a time (BC_FIRST_LEVELS, then BC_MORE_LEVELS);
        // after each chunk one read of its levels' frontier sizes
        nlev.clear();
        elev.clear();
        size_t d0 = 0;
        size_t depth = 0;
        bool done = false;
        for (size_t chunk = BC_FIRST_LEVELS; !done; chunk = BC_MORE_LEVELS) {
            if (d0 + chunk > (size_t)n + 2) BC_TRY(lagr_fail(msg, LAGR_DEVICE_ERROR, "bc forward sweep did not end"));
            // the slots the chunk's compactions add to start from zero
            for (size_t d = d0 + 1; d <= d0 + chunk; d++)
                if (d >= BC_RING) BC_TRY(fill_i64(ctx, (int64_t *)slot(d), 4, 0, msg));
            for (size_t d = d0; d < d0 + chunk; d++) {
                uint64_t *next = level_buf(d + 1);
                if (!next) BC_TRY(lagr_fail(msg, LAGR_OUT_OF_MEMORY, "bc level buffers"));
                BC_TRY(fill_i64(ctx, (int64_t *)next, n, 0, msg));
                TIMED(ctx, "bc_forward",
                      hipLaunchKernelGGL(k_bc_forward, dim3(fgrid), dim3(256), 0, ctx->stream, A->rowptr, A->colidx,
                                         AT->rowptr, AT->colidx, lists(d), act_of(d), levels(d), next, unvis, sigma,
                                         ch, chT, partial, slot(d)));
                BC_LAUNCHED();
                if (chT.n > 0) {
                    hipLaunchKernelGGL(k_bc_forward_combine, dim3(cblocksT), dim3(256), 0, ctx->stream,
                                       AT->rowptr, chT, partial, next, unvis, sigma, slot(d));
                    BC_LAUNCHED();
                }
                BC_TRY(compact(next, d + 1, slot(d)));
            }
            // the frontier sizes of levels d0 .. d0 + chunk: one read of the ring
            unsigned long long ring[4 * BC_RING];
            BC_TRY(stage_to_host(ctx, 0, cnt, sizeof(ring), true, msg));
            memcpy(ring, ctx->pinned, sizeof(ring));
            for (size_t d = d0; d <= d0 + chunk; d++) {
                if (d < nlev.size()) continue;   // level d0 was read with the previous chunk
                const unsigned long long nf = ring[4 * (d % BC_RING)];
                if (nf == 0) {
                    done = true;
                    break;
                }
                nlev.push_back((int64_t)nf);
                elev.push_back((int64_t)ring[4 * (d % BC_RING) + 1]);
            }
            d0 += chunk;
        }
        depth = nlev.size() - 1;   // the deepest non-empty level
        if ((int64_t)nlev.size() > ctx->last_bc_levels) ctx->last_bc_levels = (int64_t)nlev.size();
        // backward sweep: targets at depth i-1 gather from depth i (pull),
        // or depth i scatters to them (push: by request, on every level or
        // where level i has fewer edges than level i-1 / BC_BACK_PUSH_RATIO)
        for (size_t i = depth + 1; i >= 2; i--) {
            const int has_deeper = i <= depth ? 1 : 0;
            const bool push = has_deeper && (backward == BC_BACKWARD_PUSH ||
                                             (backward == BC_BACKWARD_AUTO &&
                                              elev[i] * BC_BACK_PUSH_RATIO < elev[i - 1]));
            if (push) {
                const int64_t nt = nlev[i - 1], nsrc = nlev[i];
                hipLaunchKernelGGL(k_bc_back_clear, dim3(wgrid(nt)), dim3(256), 0, ctx->stream, lists(i - 1), nt,
                                   levels(i - 1), Wv);
                BC_LAUNCHED();
                const unsigned pg = chT.n > 0 && cblocksT > wgrid(nsrc) ? cblocksT : wgrid(nsrc);
                TIMED(ctx, "bc_backward_push",
                      hipLaunchKernelGGL(k_bc_back_push, dim3(pg), dim3(256), 0, ctx->stream, AT->rowptr, AT->colidx,
                                         lists(i), nsrc, levels(i), levels(i - 1), Wv, chT));
                BC_LAUNCHED();
                hipLaunchKernelGGL(k_bc_back_finish, dim3(wgrid(nt)), dim3(256), 0, ctx->stream, lists(i - 1), nt,
                                   levels(i - 1), gshift, sigma, Wv, cent);
                BC_LAUNCHED();
                continue;
            }
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
//
// The levels' directions and their end are decided on the device (each
// level's kernels read the counts the previous compaction left), so the
// host queues the start and the first MS_FIRST_LEVELS levels at once --
// replayed from a hipGraph captured once per context and buffer set -- and
// reads the frontier sizes once; deeper searches continue MS_MORE_LEVELS
// levels per read.
constexpr size_t MS_FIRST_LEVELS = 8;
constexpr size_t MS_MORE_LEVELS = 4;

namespace {
// k_bc_init with the lane mask from src[64] (the sources' copy carries it,
// so a captured start serves any set of lanes)
__global__ __launch_bounds__(256) void k_ms_init(int64_t n, const int64_t *__restrict__ src,
                                                 uint64_t *__restrict__ unvis, uint64_t *__restrict__ mask0)
{
    const uint64_t lanes = (uint64_t)src[64];
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        unvis[v] = lanes;
        mask0[v] = 0;
    }
}

template <class T>
__global__ void k_set(T *__restrict__ p, int64_t n, T v)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

struct MsBufs {
    const int64_t *rp;
    const int32_t *ci;
    int64_t n;
    uint64_t lanes;
    uint64_t *unvis;
    int32_t *acts;
    unsigned long long *cnt;
    int64_t *dsrc;
    unsigned long long *dstats;
    uint64_t *mask[2];
    int32_t *list[2];
    uint16_t *lev;
    RowChunks ch;
    unsigned compact_blocks;
};

// Queue levels d0 .. d0 + count - 1 (and, with start, the search's start)
// on stream s.
int ms_enqueue(const MsBufs &B, hipStream_t s, bool start, size_t d0, size_t count, char *msg)
{
    const int64_t n = B.n;
    const size_t n1 = (size_t)(n > 0 ? n : 1);
    auto slot = [&](size_t d) { return B.cnt + 4 * (d % BC_RING); };
    auto act_of = [&](size_t d) { return B.acts + (d & 1) * n1; };
    if (start) {
        hipLaunchKernelGGL(k_set<int64_t>, dim3(1), dim3(64), 0, s, (int64_t *)B.cnt, (int64_t)(4 * BC_RING), (int64_t)0);
        if (B.lev)
            hipLaunchKernelGGL(k_set<uint32_t>, dim3(grid_for(n * 32, 256, 16384)), dim3(256), 0, s,
                               (uint32_t *)B.lev, n * 32, 0xFFFFFFFFu);
        hipLaunchKernelGGL(k_ms_init, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, n, B.dsrc, B.unvis, B.mask[0]);
        hipLaunchKernelGGL(k_ms_sources, dim3(1), dim3(64), 0, s, B.dsrc, B.unvis, B.mask[0], B.dstats);
        if (n > 0)
            hipLaunchKernelGGL(k_bc_compact, dim3(B.compact_blocks), dim3(256), 0, s, B.rp, B.rp, n, B.mask[0],
                               B.unvis, B.list[0], act_of(0), slot(0), (const unsigned long long *)nullptr);
        hipLaunchKernelGGL(k_ms_stats, dim3(256), dim3(256), 0, s, B.list[0], slot(0), B.mask[0], (int64_t)0, B.lev,
                           B.dstats);
        LAUNCH_CHECK();
    } else {
        // the slots these levels' compactions add to start from zero
        for (size_t d = d0 + 1; d <= d0 + count; d++)
            hipLaunchKernelGGL(k_set<int64_t>, dim3(1), dim3(64), 0, s, (int64_t *)slot(d), (int64_t)4, (int64_t)0);
    }
    for (size_t d = d0; d < d0 + count; d++) {
        const int b = (int)(d & 1);
        uint64_t *cur = B.mask[b], *next = B.mask[b ^ 1];
        hipLaunchKernelGGL(k_set<int64_t>, dim3(grid_for(n, 256, 16384)), dim3(256), 0, s, (int64_t *)next, n,
                           (int64_t)0);
        hipLaunchKernelGGL(k_ms_forward, dim3(BC_FORWARD_GRID), dim3(256), 0, s, B.rp, B.ci, B.list[b], act_of(d),
                           cur, next, B.unvis, B.ch, slot(d));
        if (n > 0)
            hipLaunchKernelGGL(k_bc_compact, dim3(B.compact_blocks), dim3(256), 0, s, B.rp, B.rp, n, next, B.unvis,
                               B.list[b ^ 1], act_of(d + 1), slot(d + 1), slot(d));
        hipLaunchKernelGGL(k_ms_stats, dim3(256), dim3(256), 0, s, B.list[b ^ 1], slot(d + 1), next,
                           (int64_t)(d + 1), B.lev, B.dstats);
        LAUNCH_CHECK();
    }
    return LAGR_SUCCESS;
}
}  // namespace

int msbfs_compute(lagr_ctx ctx, const lagr_graph G, const int64_t *lane_src, uint16_t *lev, int64_t *stats,
                  char *msg)
{
    const lagr_matrix A = G->A;
    const int64_t n = A->nrows;
    const size_t n1 = (size_t)(n > 0 ? n : 1);
    uint64_t *unvis = (uint64_t *)ws_get(ctx, WS_BC_UNVIS, sizeof(uint64_t) * n1);
    int32_t *acts = (int32_t *)ws_get(ctx, WS_BC_ACT, sizeof(int32_t) * 2 * n1);
    unsigned long long *cnt = (unsigned long long *)ws_get(ctx, WS_BC_CNT, sizeof(unsigned long long) * 4 * BC_RING);
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
    MsBufs B;
    B.rp = A->rowptr;
    B.ci = A->colidx;
    B.n = n;
    B.lanes = 0;
    for (int k = 0; k < 64; k++)
        if (lane_src[k] >= 0) B.lanes |= 1ull << k;
    B.unvis = unvis;
    B.acts = acts;
    B.cnt = cnt;
    B.dsrc = dsrc;
    B.dstats = dstats;
    for (int b = 0; b < 2; b++) {
        B.mask[b] = (uint64_t *)ctx->lvpool[b];
        B.list[b] = (int32_t *)((char *)ctx->lvpool[b] + mask_bytes);
    }
    B.lev = lev;
    TRY(graph_chunks(G, ctx, &B.ch, msg));
    B.compact_blocks = (unsigned)(n > 0 ? (ctx->num_cus < n ? ctx->num_cus : n) : 1);
    // the sources and the lane mask; the copy is from pinned staging
    int64_t *stage = (int64_t *)((char *)ctx->pinned + 2048);
    HIP_TRY(hipStreamSynchronize(ctx->stream));   // the staging area is free
    memcpy(stage, lane_src, sizeof(int64_t) * 64);
    stage[64] = (int64_t)B.lanes;
    HIP_TRY(hipMemcpyAsync(dsrc, stage, sizeof(int64_t) * 65, hipMemcpyHostToDevice, ctx->stream));
    // the start and the first levels: the context's captured graph for this
    // buffer set (every argument of its nodes), captured on first use
    const std::vector<uintptr_t> key = {(uintptr_t)B.rp, (uintptr_t)B.ci, (uintptr_t)n,
                                        (uintptr_t)unvis, (uintptr_t)acts, (uintptr_t)cnt, (uintptr_t)dsrc,
                                        (uintptr_t)dstats, (uintptr_t)B.mask[0], (uintptr_t)B.mask[1],
                                        (uintptr_t)lev, (uintptr_t)B.ch.n, (uintptr_t)B.ch.row,
                                        (uintptr_t)B.compact_blocks};
    if (!ctx->ms_exec || ctx->ms_key != key) {
        if (ctx->ms_exec) (void)hipGraphExecDestroy(ctx->ms_exec);
        ctx->ms_exec = nullptr;
        ctx->ms_key.clear();
        if (!ctx->capture_stream) HIP_TRY(hipStreamCreateWithFlags(&ctx->capture_stream, hipStreamNonBlocking));
        HIP_TRY(hipStreamBeginCapture(ctx->capture_stream, hipStreamCaptureModeThreadLocal));
        const int rc = ms_enqueue(B, ctx->capture_stream, true, 0, MS_FIRST_LEVELS, msg);
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(ctx->capture_stream, &g);
        if (rc < 0 || e != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return rc < 0 ? rc : lagr_fail(msg, LAGR_DEVICE_ERROR, "msbfs capture: %s", hipGetErrorString(e));
        }
        const hipError_t ei = hipGraphInstantiate(&ctx->ms_exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ei != hipSuccess) {
            ctx->ms_exec = nullptr;
            return lagr_fail(msg, LAGR_DEVICE_ERROR, "msbfs graph: %s", hipGetErrorString(ei));
        }
        ctx->ms_key = key;
    }
    HIP_TRY(hipGraphLaunch(ctx->ms_exec, ctx->stream));
    // read the frontier sizes (one read of the counter ring per chunk)
    size_t d0 = 0;
    for (size_t chunk = MS_FIRST_LEVELS;; chunk = MS_MORE_LEVELS) {
        unsigned long long ring[4 * BC_RING];
        TRY(stage_to_host(ctx, 0, cnt, sizeof(ring), true, msg));
        memcpy(ring, ctx->pinned, sizeof(ring));
        bool done = false;
        for (size_t d = d0 + 1; d <= d0 + chunk; d++)
            if (ring[4 * (d % BC_RING)] == 0) done = true;
        if (done) break;
        d0 += chunk;
        if (d0 + MS_MORE_LEVELS >= 65535) return lagr_fail(msg, LAGR_DEVICE_ERROR, "msbfs did not end");
        TRY(ms_enqueue(B, ctx->stream, false, d0, MS_MORE_LEVELS, msg));
    }
    TRY(stage_to_host(ctx, 0, dstats, 8 * 3 * 64, true, msg));
    memcpy(stats, ctx->pinned, 8 * 3 * 64);
    return LAGR_SUCCESS;
}

namespace {
// levels[k * n + v] = level of v from lane k's source (-1 unreached), for
// lanes k < nl, from the lane-major 16-bit levels lev[v * 64 + k]
__global__ __launch_bounds__(256) void k_lanes_to_rows(const uint16_t *__restrict__ lev, int64_t n, int nl,
                                                       int32_t *__restrict__ levels)
{
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / 64;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / 64;
    const unsigned lane = lane_id();
    // a wave reads 64 vertices' 64 lanes (8 KB) and writes 64 consecutive
    // vertices of each row
    for (int64_t v0 = wave * 64; v0 < n; v0 += nw * 64) {
        for (int k = 0; k < nl; k++) {
            const int64_t v = v0 + lane;
            if (v < n) {
                const uint16_t x = lev[v * 64 + k];
                levels[(int64_t)k * n + v] = x == 0xFFFF ? -1 : (int32_t)x;
            }
        }
    }
}
}  // namespace

extern "C" int lagr_bfs_batch(int32_t *levels, int64_t *reached, int64_t *level_sum, int64_t *depth,
                              const lagr_graph G, const int64_t *sources, int32_t ns, lagr_ctx ctx, char *msg)
{
    if (!G || !ctx) return lagr_fail(msg, LAGR_NULL_POINTER, "NULL argument");
    if (ns < 0 || (ns > 0 && !sources)) return lagr_fail(msg, LAGR_INVALID_VALUE, "bad sources");
    if (G->kind != LAGR_ADJACENCY_UNDIRECTED)
        return lagr_fail(msg, LAGR_INVALID_VALUE, "the batched search needs an undirected graph");
    const int64_t n = G->A->nrows;
    for (int32_t k = 0; k < ns; k++)
        if (sources[k] < 0 || sources[k] >= n)
            return lagr_fail(msg, LAGR_INVALID_INDEX, "source %lld out of range", (long long)sources[k]);
    uint16_t *lev = nullptr;
    if (levels) {
        lev = (uint16_t *)ws_get(ctx, WS_GEN_A, sizeof(uint16_t) * 64 * (size_t)(n > 0 ? n : 1));
        if (!lev) return lagr_fail(msg, LAGR_OUT_OF_MEMORY, "level lanes");
    }
    for (int32_t b0 = 0; b0 < ns; b0 += 64) {
        const int nl = ns - b0 < 64 ? ns - b0 : 64;
        int64_t src[64];
        for (int k = 0; k < 64; k++) src[k] = k < nl ? sources[b0 + k] : -1;
        int64_t st[3 * 64];
        TRY(msbfs_compute(ctx, G, src, lev, st, msg));
        for (int k = 0; k < nl; k++) {
            if (reached) reached[b0 + k] = st[k];
            if (level_sum) level_sum[b0 + k] = st[64 + k];
            if (depth) depth[b0 + k] = st[128 + k];
        }
        if (levels && n > 0) {
            hipLaunchKernelGGL(k_lanes_to_rows, dim3(grid_for(n, 256, 4096)), dim3(256), 0, ctx->stream, lev, n, nl,
                               levels + (int64_t)b0 * n);
            LAUNCH_CHECK();
        }
    }
    if (levels) HIP_TRY(hipStreamSynchronize(ctx->stream));
    return lagr_ok(msg);
}

extern "C" int lagr_bc(lagr_vector *centrality_out, const lagr_graph G, const int64_t *sources,
                       int32_t ns, lagr_ctx ctx, char *msg)
{
    return lagr_bc_dir(centrality_out, G, sources, ns, 0, ctx, msg);
}

extern "C" int lagr_bc_dir(lagr_vector *centrality_out, const lagr_graph G, const int64_t *sources,
                           int32_t ns, uint32_t flags, lagr_ctx ctx, char *msg)
{
    if (!centrality_out || !G || !ctx) return lagr_fail(msg, LAGR_NULL_POINTER, "NULL argument");
    if (flags & ~(uint32_t)(LAGR_BC_BACKWARD_PUSH_PULL | LAGR_BC_BACKWARD_PUSH_ONLY))
        return lagr_fail(msg, LAGR_INVALID_VALUE, "unknown flags 0x%x", flags);
    const int backward = (flags & LAGR_BC_BACKWARD_PUSH_ONLY)   ? BC_BACKWARD_PUSH
                         : (flags & LAGR_BC_BACKWARD_PUSH_PULL) ? BC_BACKWARD_AUTO
                                                                : BC_BACKWARD_PULL;
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
    const int rc = bc_compute(ctx, G, lane_src.data(), nbatches, 6, (double *)cv->values, msg, backward);
    if (rc < 0) {
        lagr_vector_free(&cv);
        return rc;
    }
    *centrality_out = cv;
    return lagr_ok(msg);
}
