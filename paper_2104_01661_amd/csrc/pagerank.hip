// PageRank as GAP specifies it (Section IV-C, Algorithm 4), in FP64:
//   teleport = (1 - damping) / n;  r = 1 / n;  d = d_out / damping;
//   each iteration: t = r;  w = t / d where d_out > 0 (a vertex without
//   out-edges sends nothing);  r = teleport + AT plus.second w;  stop when
//   the 1-norm of t - r is below tol, or after itermax iterations.
// AT plus.second w is a pull over the rows of AT (the in-edges; A itself
// for an undirected graph): a row of at most PR_THREAD_ROW in-edges is
// summed by one lane in ascending order, the order of the listing's sum;
// longer rows are cut into chunks of GRAPH_LONG_ROW entries, each reduced by
// a wavefront in a fixed order (lane-strided partial sums, then a fixed
// butterfly), and the chunks of a row are added in chunk order, so every
// run gives the same bits.  One dense pass then forms |t - r| with
// per-workgroup partial sums, and the next iteration's w; a one-workgroup
// kernel adds the partials in a fixed order and decides termination on the
// device, and every kernel of an iteration returns at once after that, so
// the host reads the done flag only every few iterations.
#include "internal.h"

namespace {

constexpr int PR_THREAD_ROW = 32;
constexpr int PR_BATCH = 8;         // gathers in flight per lane; the adds keep their order
constexpr int PR_BLOCK = 256;
constexpr int PR_PARTIALS = 1024;   // workgroups of the dense pass (grid-stride)

struct PrDev {
    int32_t done, pad_;
    int64_t iters;
    double diff;
};

// r = 1/n, w = r / d (d = d_out / damping, where d_out > 0), state reset.
__global__ void k_pr_init(const int64_t *__restrict__ rp, int64_t n, double damping, double *__restrict__ r,
                          double *__restrict__ w, PrDev *st)
{
    const double r0 = 1.0 / (double)n;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x) {
        const int64_t dout = rp[v + 1] - rp[v];
        r[v] = r0;
        w[v] = dout > 0 ? r0 / ((double)dout / damping) : 0.0;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->done = 0;
        st->iters = 0;
        st->diff = 0.0;
    }
}

// Rows of at most PR_THREAD_ROW in-edges: r(j) = teleport + sum in
// ascending order.  Longer rows are left to the chunk kernels.
__device__ __forceinline__ void pr_rows(const int64_t *__restrict__ rpT, const int32_t *__restrict__ ciT, int64_t n,
                                        double teleport, const double *__restrict__ w, double *__restrict__ r)
{
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n;
         j += (int64_t)gridDim.x * blockDim.x) {
        const int64_t b = rpT[j], e = rpT[j + 1];
        if (e - b > PR_THREAD_ROW) continue;
        double s = 0.0;
        for (int64_t p0 = b; p0 < e; p0 += PR_BATCH) {
            double x[PR_BATCH];
#pragma unroll
            for (int k = 0; k < PR_BATCH; k++) x[k] = p0 + k < e ? w[ciT[p0 + k]] : 0.0;
#pragma unroll
            for (int k = 0; k < PR_BATCH; k++)
                if (p0 + k < e) s += x[k];
        }
        r[j] = teleport + s;
    }
}

// A chunk of a long row per wavefront: lane l adds entries l, l + 64, ...
// in order, then a fixed butterfly adds the lanes.
__device__ __forceinline__ void pr_chunks(const int32_t *__restrict__ ciT, const RowChunks &ch,
                                          const double *__restrict__ w, double *__restrict__ part)
{
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / 64;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / 64;
    const unsigned lane = lane_id();
    for (int64_t c = wave; c < ch.n; c += nw) {
        double s = 0.0;
        const int64_t e = ch.end[c];
        for (int64_t p0 = ch.beg[c] + lane; p0 < e; p0 += 64 * PR_BATCH) {
            double x[PR_BATCH];
#pragma unroll
            for (int k = 0; k < PR_BATCH; k++) x[k] = p0 + 64 * k < e ? w[ciT[p0 + 64 * k]] : 0.0;
#pragma unroll
            for (int k = 0; k < PR_BATCH; k++)
                if (p0 + 64 * k < e) s += x[k];
        }
        for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
        if (lane == 0) part[c] = s;
    }
}

// One gather pass per iteration: the chunks of the long rows (a wave
// each), then the short rows (a lane each), in one launch, so the short
// rows fill the machine while the chunk work drains.  Each row's and each
// chunk's summation order is fixed, whatever the grid.
__global__ __launch_bounds__(PR_BLOCK) void k_pr_gather(const int64_t *__restrict__ rpT,
                                                        const int32_t *__restrict__ ciT, int64_t n, double teleport,
                                                        const double *__restrict__ w, double *__restrict__ r,
                                                        RowChunks ch, double *__restrict__ part, const PrDev *st)
{
    if (st->done) return;
    pr_chunks(ciT, ch, w, part);
    pr_rows(rpT, ciT, n, teleport, w, r);
}

// r(j) of a long row: its chunks' sums in chunk order (a row's chunks are
// consecutive in the list; the thread of its first chunk adds them).
__global__ __launch_bounds__(PR_BLOCK) void k_pr_combine(const int64_t *__restrict__ rpT, RowChunks ch,
                                                         double teleport, const double *__restrict__ part,
                                                         double *__restrict__ r, const PrDev *st)
{
    if (st->done) return;
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < ch.n;
         c += (int64_t)gridDim.x * blockDim.x) {
        const int32_t j = ch.row[c];
        if (ch.beg[c] != rpT[j]) continue;
        double s = 0.0;
        for (int64_t k = c; k < ch.n && ch.row[k] == j; k++) s += part[k];
        r[j] = teleport + s;
    }
}

// |t - r| summed per workgroup (lanes in vertex order, then a fixed tree),
// and the next iteration's w = r / d.
__global__ __launch_bounds__(PR_BLOCK) void k_pr_diff(const int64_t *__restrict__ rp, int64_t n, double damping,
                                                      const double *__restrict__ t, const double *__restrict__ r,
                                                      double *__restrict__ w, double *__restrict__ partial,
                                                      const PrDev *st)
{
    if (st->done) return;
    __shared__ double red[PR_BLOCK];
    double s = 0.0;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x) {
        const double rv = r[v];
        s += fabs(t[v] - rv);
        const int64_t dout = rp[v + 1] - rp[v];
        w[v] = dout > 0 ? rv / ((double)dout / damping) : 0.0;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = PR_BLOCK / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// The iteration's change: the partials in a fixed tree; done when it is
// below tol or when itermax iterations have run.
__global__ __launch_bounds__(PR_PARTIALS) void k_pr_decide(const double *__restrict__ partial, double tol,
                                                           int64_t itermax, PrDev *st)
{
    if (st->done) return;
    __shared__ double red[PR_PARTIALS];
    red[threadIdx.x] = partial[threadIdx.x];
    __syncthreads();
    for (int o = PR_PARTIALS / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        st->iters += 1;
        st->diff = red[0];
        if (red[0] < tol || st->iters >= itermax) st->done = 1;
    }
}

}  // namespace

extern "C" int lagr_pagerank(lagr_vector *rank_out, int64_t *iters_out, const lagr_graph G, double damping,
                             double tol, int64_t itermax, lagr_ctx ctx, char *msg)
{
    if (!rank_out || !G || !ctx) return lagr_fail(msg, LAGR_NULL_POINTER, "NULL argument");
    *rank_out = nullptr;
    if (iters_out) *iters_out = 0;
    if (!(damping >= 0.0) || !(damping <= 1.0))
        return lagr_fail(msg, LAGR_INVALID_VALUE, "damping must lie in [0, 1]");
    if (!(tol >= 0.0) || !(tol < INFINITY) || itermax < 0)
        return lagr_fail(msg, LAGR_INVALID_VALUE, "tol must be finite and >= 0, itermax >= 0");
    const lagr_matrix A = G->A;
    const int64_t n = A->nrows;
    TRY(graph_ensure_at(G, ctx, msg));
    const lagr_matrix AT = graph_in_edges(G);
    lagr_vector rv = new (std::nothrow) lagr_vector_s();
    if (!rv) return lagr_fail(msg, LAGR_OUT_OF_MEMORY, "vector");
    rv->type = LAGR_FP64;
    rv->n = n;
    rv->fmt = LAGR_VEC_FULL;
    rv->nvals = n;
    rv->values_bytes = sizeof(double) * (size_t)(n > 0 ? n : 1);
    rv->values = dev_alloc(rv->values_bytes);
    if (!rv->values) {
        delete rv;
        return lagr_fail(msg, LAGR_OUT_OF_MEMORY, "vector values");
    }
    int rc = LAGR_SUCCESS;
#define PR_TRY(expr)              \
    do {                          \
        rc = (expr);              \
        if (rc < 0) {             \
            lagr_vector_free(&rv); \
            return rc;            \
        }                         \
    } while (0)
    if (n == 0) {
        *rank_out = rv;
        return lagr_ok(msg);
    }
    const size_t n1 = (size_t)n;
    double *bufs = (double *)ws_get(ctx, WS_GEN_F, sizeof(double) * 2 * n1);
    double *partial = (double *)ws_get(ctx, WS_GEN_G, sizeof(double) * PR_PARTIALS);
    PrDev *st = (PrDev *)ws_get(ctx, WS_COUNTERS, sizeof(PrDev));
    if (!bufs || !partial || !st) PR_TRY(lagr_fail(msg, LAGR_OUT_OF_MEMORY, "pagerank workspace"));
    double *w = bufs, *t = bufs + n1;
    double *r = (double *)rv->values;
    RowChunks ch;
    PR_TRY(row_chunks(ctx, AT->rowptr, n, PR_THREAD_ROW, GRAPH_LONG_ROW, WS_CHUNK_A, WS_CHUNK_B, &ch, msg));
    double *part = nullptr;
    if (ch.n > 0) {
        part = (double *)ws_get(ctx, WS_GEN_H, sizeof(double) * (size_t)ch.n);
        if (!part) PR_TRY(lagr_fail(msg, LAGR_OUT_OF_MEMORY, "pagerank chunk sums"));
    }
    PR_TRY(fill_i64(ctx, (int64_t *)partial, PR_PARTIALS, 0, msg));
    hipLaunchKernelGGL(k_pr_init, dim3(grid_for(n, PR_BLOCK, 4096)), dim3(PR_BLOCK), 0, ctx->stream, A->rowptr, n,
                       damping, r, w, st);
    if (hipGetLastError() != hipSuccess) PR_TRY(lagr_fail(msg, LAGR_DEVICE_ERROR, "pagerank launch"));
    const double teleport = (1.0 - damping) / (double)n;
    const unsigned rgrid = grid_for(n, PR_BLOCK, 8192);
    const unsigned cgrid = grid_for(ch.n * 64, PR_BLOCK, 4096);
    const unsigned bgrid = grid_for(ch.n, PR_BLOCK, 1024);
    const unsigned ggrid = rgrid > cgrid ? rgrid : cgrid;
    // r and t trade places every iteration; after k iterations the rank is
    // in r when k is even (counting from the buffer r starts in)
    double *cur = r, *prev = t;
    int64_t launched = 0;
    constexpr int PR_GROUP = 4;   // iterations queued between looks at the done flag
    while (launched < itermax) {
        for (int g = 0; g < PR_GROUP && launched < itermax; g++, launched++) {
            std::swap(cur, prev);   // prev: the prior rank t; cur receives the new r
            hipLaunchKernelGGL(k_pr_gather, dim3(ggrid), dim3(PR_BLOCK), 0, ctx->stream, AT->rowptr, AT->colidx,
                               n, teleport, w, cur, ch, part, st);
            if (ch.n > 0) {
                hipLaunchKernelGGL(k_pr_combine, dim3(bgrid), dim3(PR_BLOCK), 0, ctx->stream, AT->rowptr, ch,
                                   teleport, part, cur, st);
            }
            hipLaunchKernelGGL(k_pr_diff, dim3(PR_PARTIALS), dim3(PR_BLOCK), 0, ctx->stream, A->rowptr, n, damping,
                               prev, cur, w, partial, st);
            hipLaunchKernelGGL(k_pr_decide, dim3(1), dim3(PR_PARTIALS), 0, ctx->stream, partial, tol, itermax,
                               st);
            if (hipGetLastError() != hipSuccess) PR_TRY(lagr_fail(msg, LAGR_DEVICE_ERROR, "pagerank launch"));
        }
        int32_t done = 0;
        PR_TRY(read_back(ctx, &done, &st->done, sizeof(done), msg));
        if (done) break;
    }
    PrDev hs{};
    PR_TRY(read_back(ctx, &hs, st, sizeof(hs), msg));
    // the rank after hs.iters iterations sits in r for an even count, in t
    // for an odd one
    if (hs.iters % 2 == 1)
        if (hipMemcpyAsync(r, t, sizeof(double) * n1, hipMemcpyDeviceToDevice, ctx->stream) != hipSuccess)
            PR_TRY(lagr_fail(msg, LAGR_DEVICE_ERROR, "pagerank copy"));
#undef PR_TRY
    if (iters_out) *iters_out = hs.iters;
    *rank_out = rv;
    return lagr_ok(msg);
}
