// Single-source shortest paths by delta-stepping (Section IV-D, Algorithm 5)
// over the min.plus semiring.  Algorithm 5 splits A into light edges
// (0 < w <= delta) and heavy edges (w > delta) and settles the buckets
// [i delta, (i+1) delta) of tentative distances in increasing order:
//   light phase: t_Req = A_L' min.plus t restricted to the vertices of the
//     bucket whose distance changed, folded into t with min; repeated
//     until no vertex of the bucket improves (a light edge can land in the
//     same bucket);
//   heavy phase: once the bucket is settled, one product with A_H' from
//     every vertex of the bucket (a heavy edge always lands in a later
//     bucket);
//   then the next bucket that holds a reached, unsettled vertex.
// The printed listing is damaged where it forms t_Req and the next
// bucket's vector; the steps here follow the cited method (Meyer and
// Sanders' delta-stepping), which the listing abbreviates.
//
// On the device, every min.plus product is a push over the frontier's
// rows fused with the min accumulation: t(v) is the FP64 bit pattern in a
// 64-bit word, and for non-negative doubles the unsigned order of the bit
// patterns is the numeric order, so atomicMin on the word is the min
// monoid.  The bucket loop runs on the device: a one-thread kernel moves
// the phase state, every kernel of a step returns at once when its phase
// is not active, and two steps (the two frontier buffer parities) are
// captured once per context into a hipGraph that the host replays.
#include "internal.h"

namespace {

constexpr int SSSP_LIGHT = 0;
constexpr int SSSP_HEAVY = 1;
constexpr unsigned long long SSSP_INF = 0x7FF0000000000000ull;   // +inf

__device__ __forceinline__ bool bit_test(const uint32_t *bm, int64_t v)
{
    return (bm[v >> 5] >> (v & 31)) & 1u;
}

__device__ __forceinline__ double as_f64(unsigned long long b)
{
    return __longlong_as_double((long long)b);
}

__device__ __forceinline__ unsigned long long as_bits(double x)
{
    return (unsigned long long)__double_as_longlong(x);
}

}  // namespace

// Everything a step needs, in device memory (the captured kernels take only
// this struct's address and the parity).  list[par] / bm[par]: the light
// frontier of this step; bm[par ^ 1]: the vertices improved into the
// bucket, which become the next frontier; sbm / slist: the vertices settled
// in the bucket, whose heavy edges the heavy phase relaxes.
struct SsspDev {
    const int64_t *rp;
    const int32_t *ci;
    const double *w;
    int64_t n, W;
    unsigned long long *dist;
    uint32_t *bm[2];
    uint32_t *sbm;
    int32_t *list[2];
    int32_t *slist;
    RowChunks ch;
    double delta;
    // phase state: bucket [lo, hi), phase, termination, frontier and settled
    // sizes; nnext / nsettled / nmin are the counters the kernels fill
    double lo, hi;
    int64_t bucket, nq, steps;
    int32_t phase, done, heavy_now, pad_;
    unsigned long long nnext, nsettled, nmin;
};

namespace {

__global__ void k_sssp_init(SsspDev *d, int64_t src)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        d->dist[src] = 0ull;
        d->list[0][0] = (int32_t)src;
        d->bm[0][src >> 5] |= 1u << (src & 31);
    }
}

// Start of a step: take the frontier the last step left (nnext); an empty
// frontier ends the bucket's light phase.
__global__ void k_sssp_decide(SsspDev *d)
{
    if (threadIdx.x != 0 || d->done) return;
    d->steps += 1;
    d->heavy_now = 0;
    if (d->phase == SSSP_LIGHT) {
        d->nq = (int64_t)d->nnext;
        d->nnext = 0;
        if (d->nq == 0) {
            d->phase = SSSP_HEAVY;
            d->heavy_now = 1;
            d->nsettled = 0;
            d->nmin = SSSP_INF;
        }
    }
}

// The block's minimum of x into *out with one atomic (256 threads).
__device__ __forceinline__ void block_min_to(unsigned long long x, unsigned long long *out)
{
    __shared__ unsigned long long wmin[4];
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long y = __shfl_xor(x, o, 64);
        x = y < x ? y : x;
    }
    if (lane_id() == 0) wmin[threadIdx.x / 64] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long m = wmin[0];
        for (int k = 1; k < 4; k++) m = wmin[k] < m ? wmin[k] : m;
        if (m != SSSP_INF) atomicMin(out, m);
    }
}

// Relax one edge per lane whose weight class matches (light: w <= delta,
// marking the target for the next frontier when it improves inside the
// bucket; heavy: w > delta, which always leaves the bucket).  RELAX_BATCH
// edges per lane go through each stage together (their loads, then their
// t reads, then their atomics), so a lane waits for each round trip once
// per batch rather than once per edge.  Returns the lane's smallest improved
// distance at or above hi.
constexpr int RELAX_BATCH = 4;

template <bool HEAVY>
__device__ __forceinline__ unsigned long long relax_batch(const SsspDev &d, const double *du, const int64_t *p,
                                                          uint32_t *__restrict__ next_bm)
{
    double w[RELAX_BATCH];
    int32_t v[RELAX_BATCH];
    bool ok[RELAX_BATCH];
#pragma unroll
    for (int k = 0; k < RELAX_BATCH; k++) {
        ok[k] = p[k] >= 0;
        w[k] = ok[k] ? d.w[p[k]] : 0.0;
        v[k] = ok[k] ? d.ci[p[k]] : 0;
    }
    unsigned long long nb[RELAX_BATCH], cur[RELAX_BATCH];
#pragma unroll
    for (int k = 0; k < RELAX_BATCH; k++) {
        ok[k] = ok[k] && (HEAVY ? (w[k] > d.delta) : !(w[k] > d.delta));
        nb[k] = as_bits(du[k] + w[k]);
        cur[k] = ok[k] ? d.dist[v[k]] : 0ull;
    }
    // The atomic's old value is not waited for: a lane whose value is below
    // the one it read has lowered t(v) or lost to a lower value stored in
    // this step, whose own lane marks v too (a lower value is inside the
    // bucket whenever this one is) and reports a value no larger; so the
    // marks and the smallest value are those of the winners alone.
#pragma unroll
    for (int k = 0; k < RELAX_BATCH; k++) {
        ok[k] = ok[k] && nb[k] < cur[k];
        if (ok[k]) atomicMin(&d.dist[v[k]], nb[k]);
    }
    unsigned long long far = SSSP_INF;
#pragma unroll
    for (int k = 0; k < RELAX_BATCH; k++) {
        if (!ok[k]) continue;
        if (!HEAVY && as_f64(nb[k]) < d.hi) atomicOr(&next_bm[v[k] >> 5], 1u << (v[k] & 31));
        else far = nb[k] < far ? nb[k] : far;
    }
    return far;
}

// The edges rp-range [b, e) of one vertex (distance du), over the wave.
template <bool HEAVY>
__device__ __forceinline__ unsigned long long relax_range(const SsspDev &d, double du, int64_t b, int64_t e,
                                                          unsigned lane, uint32_t *__restrict__ next_bm)
{
    unsigned long long far = SSSP_INF;
    const double dus[RELAX_BATCH] = {du, du, du, du};
    static_assert(RELAX_BATCH == 4, "dus initialiser");
    for (int64_t p0 = b + lane; p0 < e; p0 += 64 * RELAX_BATCH) {
        int64_t p[RELAX_BATCH];
#pragma unroll
        for (int k = 0; k < RELAX_BATCH; k++) p[k] = p0 + 64 * k < e ? p0 + 64 * k : -1;
        const unsigned long long x = relax_batch<HEAVY>(d, dus, p, next_bm);
        far = x < far ? x : far;
    }
    return far;
}

// Vertices per wavefront: the frontier spread over all wavefronts, at
// least 1 and at most 64 (a power of two).
__device__ __forceinline__ int group_size(int64_t nq, int64_t nw)
{
    int g = 1;
    while (g < 64 && (int64_t)g * nw < nq) g <<= 1;
    return g;
}

// Relax the edges of the g vertices list[f0 .. f0 + g) (rows of at most
// GRAPH_LONG_ROW entries) with the whole wave: an inclusive scan of the row
// lengths over the lanes lays the g rows end to end, and lane l takes edge
// t0 + l of that sequence.  The rows' ends, starts and distances go to the
// wave's LDS, and each lane walks them forward to the owner of its edge
// (its edges only increase: about one step per row boundary crossed),
// keeping the owner's start and distance in registers.  Every lane of the
// wave must call it (256-thread workgroups).
struct RelaxRows {
    int end[64];
    int64_t start[64];
    double du[64];
};
template <bool HEAVY>
__device__ __forceinline__ unsigned long long relax_group(const SsspDev &d, const int32_t *__restrict__ list,
                                                          int64_t f0, int g, int64_t nq, unsigned lane,
                                                          uint32_t *__restrict__ next_bm)
{
    const int64_t f = f0 + lane;
    int64_t b = 0;
    int len = 0;
    double du = 0.0;
    if ((int)lane < g && f < nq) {
        const int32_t u = list[f];
        b = d.rp[u];
        const int64_t e = d.rp[u + 1];
        if (e - b <= GRAPH_LONG_ROW) {
            len = (int)(e - b);
            du = as_f64(d.dist[u]);
        }
    }
    const int incl = wave_incl_sum(len);
    const int total = __builtin_amdgcn_readlane(incl, 63);
    const int64_t start = b - (incl - len);   // row start minus the row's offset in the sequence
    __shared__ RelaxRows rows[4];
    RelaxRows &R = rows[threadIdx.x >> 6];
    // (the wave's LDS operations run in order; the fences keep the compiler
    // from moving them across: the previous call's reads, then these writes)
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    R.end[lane] = incl;
    R.start[lane] = start;
    R.du[lane] = du;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    int r = 0, rend = R.end[0];
    int64_t sr = R.start[0];
    double dr = R.du[0];
    unsigned long long far = SSSP_INF;
    for (int t0 = 0; t0 < total; t0 += 64 * RELAX_BATCH) {
        int64_t p[RELAX_BATCH];
        double dk[RELAX_BATCH];
#pragma unroll
        for (int k = 0; k < RELAX_BATCH; k++) {
            const int t = t0 + 64 * k + (int)lane;
            p[k] = -1;
            dk[k] = 0.0;
            if (t < total) {
                if (rend <= t) {
                    do {
                        ++r;
                        rend = R.end[r];
                    } while (rend <= t);
                    sr = R.start[r];
                    dr = R.du[r];
                }
                p[k] = sr + t;
                dk[k] = dr;
            }
        }
        const unsigned long long x = relax_batch<HEAVY>(d, dk, p, next_bm);
        far = x < far ? x : far;
    }
    return far;
}

// Light phase: groups of frontier vertices per wavefront (rows of at most
// GRAPH_LONG_ROW entries; longer rows in sssp_light_chunks).
__device__ __forceinline__ void sssp_light(const SsspDev &d, int par)
{
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / 64;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / 64;
    const unsigned lane = lane_id();
    const int64_t nq = d.nq;
    const int g = group_size(nq, nw);
    if (g == 1) {
        for (int64_t f = wave; f < nq; f += nw) {
            const int32_t u = d.list[par][f];
            const int64_t b = d.rp[u], e = d.rp[u + 1];
            if (e - b > GRAPH_LONG_ROW) continue;
            (void)relax_range<false>(d, as_f64(d.dist[u]), b, e, lane, d.bm[par ^ 1]);
        }
        return;
    }
    for (int64_t f0 = wave * g; f0 < nq; f0 += nw * g)
        (void)relax_group<false>(d, d.list[par], f0, g, nq, lane, d.bm[par ^ 1]);
}

__device__ __forceinline__ void sssp_light_chunks(const SsspDev &d, int par)
{
    const unsigned lane = lane_id();
    uint32_t *next_bm = d.bm[par ^ 1];
    for_marked_chunks(d.ch, d.bm[par], [&](int32_t u, int64_t b, int64_t e) {
        (void)relax_range<false>(d, as_f64(d.dist[u]), b, e, lane, next_bm);
    });
}

// One light step in one launch: the frontier's short rows, then the chunks
// of its long rows (a kernel node with nothing to do still costs its
// dispatch).
__global__ __launch_bounds__(256) void k_sssp_light(SsspDev *dp, int par)
{
    const SsspDev &d = *dp;
    if (d.done || d.phase != SSSP_LIGHT) return;
    sssp_light(d, par);
    sssp_light_chunks(d, par);
}

// A 32-vertex word per thread: the workgroup scans the words' popcounts,
// reserves its range of out_list with one atomic on *counter and writes its
// vertices in ascending order.
__device__ __forceinline__ void block_list_words(uint32_t x, int64_t w, int32_t *__restrict__ out_list,
                                                 unsigned long long *counter)
{
    __shared__ unsigned wtot[4];
    __shared__ unsigned long long base_s;
    const unsigned c = (unsigned)__popc(x);
    unsigned total;
    const unsigned before = block_excl_scan256(c, wtot, total);
    if (threadIdx.x == 0) base_s = total ? atomicAdd(counter, (unsigned long long)total) : 0;
    __syncthreads();
    unsigned long long pos = base_s + before;
    for (uint32_t y = x; y; y &= y - 1) out_list[pos++] = (int32_t)(w * 32 + __ffs(y) - 1);
}

// End of a light step: the next frontier from bm[par ^ 1] (its bits stay
// for the next step's chunk kernel); the consumed bm[par] is cleared.
__device__ __forceinline__ void sssp_compact(SsspDev *dp, int par)
{
    const SsspDev &d = *dp;
    const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t x = w < d.W ? d.bm[par ^ 1][w] : 0u;
    if (w < d.W) d.bm[par][w] = 0u;
    block_list_words(x, w, d.list[par ^ 1], &dp->nnext);
}

// Settled set of the bucket: the vertices with lo <= t < hi (their t is
// final once the light phase is over), as a bitmap and a list; and the
// smallest t at or above hi (the next bucket, unless the heavy phase
// lowers it).
__device__ __forceinline__ void sssp_settled(SsspDev *dp)
{
    const SsspDev &d = *dp;
    const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const unsigned long long lo = as_bits(d.lo), hi = as_bits(d.hi);
    uint32_t x = 0u;
    unsigned long long far = SSSP_INF;
    if (w < d.W) {
        const int64_t v0 = w * 32;
        const int cnt = (int)min((int64_t)32, d.n - v0);
        for (int k = 0; k < cnt; k++) {
            const unsigned long long t = d.dist[v0 + k];
            if (t >= lo && t < hi) x |= 1u << k;
            else if (t >= hi && t < far) far = t;
        }
        d.sbm[w] = x;
    }
    block_list_words(x, w, d.slist, &dp->nsettled);
    block_min_to(far, &dp->nmin);
}

// The bitmap pass of a step, one launch for both kinds (a step is either a
// light one or the heavy one, never both): the next frontier after a light
// step, or the settled set before the heavy phase.
__global__ __launch_bounds__(256) void k_sssp_words(SsspDev *dp, int par)
{
    const SsspDev &d = *dp;
    if (d.done) return;
    if (d.phase == SSSP_LIGHT) sssp_compact(dp, par);
    else if (d.heavy_now) sssp_settled(dp);
}

// Heavy phase in one launch: groups of settled vertices per wavefront
// (short rows), then the chunks of the long rows; improved distances fold
// into nmin.
__global__ __launch_bounds__(256) void k_sssp_heavy(SsspDev *dp)
{
    const SsspDev &d = *dp;
    if (d.done || !d.heavy_now) return;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / 64;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / 64;
    const unsigned lane = lane_id();
    const int64_t ns = (int64_t)d.nsettled;
    const int g = group_size(ns, nw);
    unsigned long long far = SSSP_INF;
    if (g == 1) {
        for (int64_t f = wave; f < ns; f += nw) {
            const int32_t u = d.slist[f];
            const int64_t b = d.rp[u], e = d.rp[u + 1];
            if (e - b > GRAPH_LONG_ROW) continue;
            const unsigned long long x = relax_range<true>(d, as_f64(d.dist[u]), b, e, lane, nullptr);
            far = x < far ? x : far;
        }
    } else {
        for (int64_t f0 = wave * g; f0 < ns; f0 += nw * g) {
            const unsigned long long x = relax_group<true>(d, d.slist, f0, g, ns, lane, nullptr);
            far = x < far ? x : far;
        }
    }
    for_marked_chunks(d.ch, d.sbm, [&](int32_t u, int64_t b, int64_t e) {
        const unsigned long long x = relax_range<true>(d, as_f64(d.dist[u]), b, e, lane, nullptr);
        far = x < far ? x : far;
    });
    block_min_to(far, &dp->nmin);
}

// After the heavy phase: the bucket of the smallest unsettled distance (or
// the end of the search when no reached vertex is left unsettled) and its
// vertices as the next frontier.  Every workgroup derives the bucket from
// the final nmin itself; workgroup 0 records it.  (nnext is zero here: the
// decision that started the heavy phase cleared it.)
__global__ __launch_bounds__(256) void k_sssp_bucket(SsspDev *dp, int par)
{
    const SsspDev &d = *dp;
    if (d.done || !d.heavy_now) return;
    const unsigned long long nmin = d.nmin;
    const bool first = blockIdx.x == 0 && threadIdx.x == 0;
    if (nmin == SSSP_INF) {
        if (first) dp->done = 1;
        return;
    }
    const double m = as_f64(nmin), delta = d.delta;
    double bk = floor(m / delta);
    if (bk * delta > m) bk -= 1.0;
    if ((bk + 1.0) * delta <= m) bk += 1.0;
    const double lod = bk * delta, hid = (bk + 1.0) * delta;
    if (first) {
        dp->bucket = (int64_t)bk;
        dp->lo = lod;
        dp->hi = hid;
        dp->phase = SSSP_LIGHT;
    }
    const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const unsigned long long lo = as_bits(lod), hi = as_bits(hid);
    uint32_t x = 0u;
    if (w < d.W) {
        const int64_t v0 = w * 32;
        const int cnt = (int)min((int64_t)32, d.n - v0);
        for (int k = 0; k < cnt; k++) {
            const unsigned long long t = d.dist[v0 + k];
            if (t >= lo && t < hi) x |= 1u << k;
        }
        d.bm[par ^ 1][w] = x;
    }
    block_list_words(x, w, d.list[par ^ 1], &dp->nnext);
}

// Weights must be positive and finite: flag any other value.
__global__ void k_sssp_check_weights(const double *__restrict__ w, int64_t nnz, unsigned *__restrict__ bad)
{
    bool b = false;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < nnz;
         p += (int64_t)gridDim.x * blockDim.x) {
        const double x = w[p];
        if (!(x > 0.0) || !(x < INFINITY)) b = true;
    }
    if (__ballot(b) && lane_id() == 0) *bad = 1u;
}

// One step with buffer parity par.
int enqueue_step(SsspDev *d, int par, int64_t W, int num_cus, hipStream_t s, char *msg)
{
    const unsigned wgrid = grid_for(W, 256, 1 << 30);
    hipLaunchKernelGGL(k_sssp_decide, dim3(1), dim3(64), 0, s, d);
    hipLaunchKernelGGL(k_sssp_light, dim3((unsigned)(num_cus * 8)), dim3(256), 0, s, d, par);
    hipLaunchKernelGGL(k_sssp_words, dim3(wgrid), dim3(256), 0, s, d, par);
    hipLaunchKernelGGL(k_sssp_heavy, dim3((unsigned)(num_cus * 8)), dim3(256), 0, s, d);
    hipLaunchKernelGGL(k_sssp_bucket, dim3(wgrid), dim3(256), 0, s, d, par);
    LAUNCH_CHECK();
    return LAGR_SUCCESS;
}

}  // namespace

// The context's captured two-step graph for graphs of n vertices.
static int sssp_graph(lagr_ctx ctx, SsspDev *d, int64_t n, int64_t W, hipGraphExec_t *exec, char *msg)
{
    if (ctx->sssp_exec && ctx->sssp_key == n && ctx->sssp_state == (void *)d) {
        *exec = ctx->sssp_exec;
        return LAGR_SUCCESS;
    }
    if (ctx->sssp_exec) (void)hipGraphExecDestroy(ctx->sssp_exec);
    ctx->sssp_exec = nullptr;
    if (!ctx->capture_stream) HIP_TRY(hipStreamCreateWithFlags(&ctx->capture_stream, hipStreamNonBlocking));
    HIP_TRY(hipStreamBeginCapture(ctx->capture_stream, hipStreamCaptureModeThreadLocal));
    int rc = enqueue_step(d, 0, W, ctx->num_cus, ctx->capture_stream, msg);
    if (rc >= 0) rc = enqueue_step(d, 1, W, ctx->num_cus, ctx->capture_stream, msg);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(ctx->capture_stream, &g);
    if (rc < 0 || e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return rc < 0 ? rc : lagr_fail(msg, LAGR_DEVICE_ERROR, "sssp capture: %s", hipGetErrorString(e));
    }
    const hipError_t ei = hipGraphInstantiate(&ctx->sssp_exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ei != hipSuccess) {
        ctx->sssp_exec = nullptr;
        return lagr_fail(msg, LAGR_DEVICE_ERROR, "sssp graph: %s", hipGetErrorString(ei));
    }
    ctx->sssp_key = n;
    ctx->sssp_state = (void *)d;
    *exec = ctx->sssp_exec;
    return LAGR_SUCCESS;
}

extern "C" int lagr_sssp(lagr_vector *dist_out, const lagr_graph G, int64_t source, double delta,
                         lagr_ctx ctx, char *msg)
{
    if (!dist_out || !G || !ctx) return lagr_fail(msg, LAGR_NULL_POINTER, "NULL argument");
    *dist_out = nullptr;
    const lagr_matrix A = G->A;
    const int64_t n = A->nrows;
    if (A->type != LAGR_FP64 || (A->nvals > 0 && !A->values))
        return lagr_fail(msg, LAGR_DOMAIN_MISMATCH, "sssp needs FP64 edge weights");
    if (source < 0 || source >= n)
        return lagr_fail(msg, LAGR_INVALID_INDEX, "source %lld out of range", (long long)source);
    if (!(delta > 0.0) || !(delta < INFINITY))
        return lagr_fail(msg, LAGR_INVALID_VALUE, "delta must be positive and finite");
    const int64_t W = (n + 31) / 32;
    int32_t *lists = (int32_t *)ws_get(ctx, WS_BFS_B, sizeof(int32_t) * 3 * n);
    uint32_t *bms = (uint32_t *)ws_get(ctx, WS_BFS_C, sizeof(uint32_t) * 3 * W);
    SsspDev *d = (SsspDev *)ws_get(ctx, WS_SSSP, sizeof(SsspDev));
    unsigned *bad = (unsigned *)ws_get(ctx, WS_COUNTERS, 64);
    if (!lists || !bms || !d || !bad) return lagr_fail(msg, LAGR_OUT_OF_MEMORY, "sssp workspace");
    if (A->nvals > 0) {
        TRY(fill_u32(ctx, bad, 1, 0u, msg));
        hipLaunchKernelGGL(k_sssp_check_weights, dim3(grid_for(A->nvals, 256, 2048)), dim3(256), 0, ctx->stream,
                           (const double *)A->values, A->nvals, bad);
        LAUNCH_CHECK();
        unsigned hbad = 0;
        TRY(read_back(ctx, &hbad, bad, sizeof(hbad), msg));
        if (hbad) return lagr_fail(msg, LAGR_INVALID_VALUE, "sssp weights must be positive and finite");
    }
    RowChunks ch;
    TRY(graph_chunks(G, ctx, &ch, msg));
    lagr_vector dv = new (std::nothrow) lagr_vector_s();
    if (!dv) return lagr_fail(msg, LAGR_OUT_OF_MEMORY, "vector");
    dv->type = LAGR_FP64;
    dv->n = n;
    dv->fmt = LAGR_VEC_FULL;
    dv->nvals = n;
    dv->values_bytes = sizeof(double) * (size_t)(n > 0 ? n : 1);
    dv->values = dev_alloc(dv->values_bytes);
    if (!dv->values) {
        delete dv;
        return lagr_fail(msg, LAGR_OUT_OF_MEMORY, "vector values");
    }
    int rc = LAGR_SUCCESS;
#define SSSP_TRY(expr)               \
    do {                             \
        rc = (expr);                 \
        if (rc < 0) {                \
            lagr_vector_free(&dv);   \
            return rc;               \
        }                            \
    } while (0)

    SsspDev h{};
    h.rp = A->rowptr;
    h.ci = A->colidx;
    h.w = (const double *)A->values;
    h.n = n;
    h.W = W;
    h.dist = (unsigned long long *)dv->values;
    h.bm[0] = bms;
    h.bm[1] = bms + W;
    h.sbm = bms + 2 * W;
    h.list[0] = lists;
    h.list[1] = lists + n;
    h.slist = lists + 2 * n;
    h.ch = ch;
    h.delta = delta;
    h.lo = 0.0;
    h.hi = delta;
    h.phase = SSSP_LIGHT;
    h.nnext = 1;   // the source
    h.nmin = SSSP_INF;
    static_assert(sizeof(SsspDev) <= 4096, "SsspDev must fit the pinned staging buffer");
    memcpy(ctx->pinned, &h, sizeof(h));
    if (hipMemcpyAsync(d, ctx->pinned, sizeof(h), hipMemcpyHostToDevice, ctx->stream) != hipSuccess)
        SSSP_TRY(lagr_fail(msg, LAGR_DEVICE_ERROR, "sssp state copy"));
    SSSP_TRY(fill_i64(ctx, (int64_t *)dv->values, n, (int64_t)SSSP_INF, msg));
    SSSP_TRY(fill_u32(ctx, bms, 3 * W, 0u, msg));
    hipLaunchKernelGGL(k_sssp_init, dim3(1), dim3(64), 0, ctx->stream, d, source);
    if (hipGetLastError() != hipSuccess) SSSP_TRY(lagr_fail(msg, LAGR_DEVICE_ERROR, "sssp init launch"));
    hipGraphExec_t exec = nullptr;
    SSSP_TRY(sssp_graph(ctx, d, n, W, &exec, msg));
    // two steps per replay; the done flag is read after every SSSP_REPLAYS
    // replays (each look is a host round trip).  A bucket of k vertices is
    // settled after at most k + 1 light steps (within the bucket this is
    // Bellman-Ford over light edges) and one heavy step, and every vertex
    // settles in exactly one bucket, so 3n + 2 steps bound a correct run.
    constexpr int SSSP_REPLAYS = 2;
    const double limit = 4.0 * (double)n + 64.0;
    double steps = 0.0;
    for (;;) {
        for (int r = 0; r < SSSP_REPLAYS; r++)
            if (hipGraphLaunch(exec, ctx->stream) != hipSuccess)
                SSSP_TRY(lagr_fail(msg, LAGR_DEVICE_ERROR, "sssp graph launch"));
        steps += 2.0 * SSSP_REPLAYS;
        int32_t done = 0;
        SSSP_TRY(read_back(ctx, &done, &d->done, sizeof(done), msg));
        if (done) break;
        if (steps > limit) SSSP_TRY(lagr_fail(msg, LAGR_DEVICE_ERROR, "sssp did not terminate"));
    }
#undef SSSP_TRY
    *dist_out = dv;
    return lagr_ok(msg);
}
