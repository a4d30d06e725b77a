// Connected components by FastSV (Section IV-F, Algorithm 7, the variant
// over the whole graph): a parent vector f, its grandparents gf, and mngf,
// the smallest grandparent seen among each vertex's neighbours.  Reading of
// the listing's damaged hooking lines: step 1 is mngf<min>= A min.second
// gf followed by f(x)<min>= mngf with x = f as it stood at the end of the
// previous iteration; step 2 is f = min(f, mngf); step 3 is f = min(f, gf);
// step 4 is gf = f(f); the loop ends when no grandparent changes.
//
// On the device the three hooking steps are one kernel: each is a min into
// f whose inputs (mngf, x, gf) do not change while they run, so the order
// of the atomicMin updates does not matter.  A second kernel forms the
// grandparents, compares them with the last ones and counts the changes
// with one atomic per workgroup.  For a directed graph the neighbours are
// taken both ways (A and AT): weakly connected components.  FastSV only
// lowers f, so it ends with every vertex labelled by the smallest vertex
// id of its component.
#include "internal.h"

namespace {

constexpr int CC_THREAD_ROW = 64;
constexpr int CC_BLOCK = 256;

__global__ void k_cc_init(int64_t n, int32_t *__restrict__ f, int32_t *__restrict__ gf, int32_t *__restrict__ dup,
                          int32_t *__restrict__ mngf, int32_t *__restrict__ x)
{
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x) {
        const int32_t i = (int32_t)v;
        f[v] = gf[v] = dup[v] = mngf[v] = x[v] = i;
    }
}

// mngf(u) = min(mngf(u), min over neighbours v of gf(v)) for rows of at most
// CC_THREAD_ROW entries (one lane each, loads batched); longer rows are left
// to k_cc_mngf_chunks.
__device__ __forceinline__ void cc_mngf_rows(const int64_t *__restrict__ rp, const int32_t *__restrict__ ci, int64_t n,
                                             const int32_t *__restrict__ gf, int32_t *__restrict__ mngf)
{
    for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n;
         u += (int64_t)gridDim.x * blockDim.x) {
        const int64_t b = rp[u], e = rp[u + 1];
        if (e - b > CC_THREAD_ROW) continue;
        int32_t m = mngf[u];
        for (int64_t p0 = b; p0 < e; p0 += 8) {
            int32_t v[8];
#pragma unroll
            for (int k = 0; k < 8; k++) v[k] = p0 + k < e ? ci[p0 + k] : -1;
#pragma unroll
            for (int k = 0; k < 8; k++)
                if (v[k] >= 0) m = min(m, gf[v[k]]);
        }
        if (m < mngf[u]) atomicMin(&mngf[u], m);
    }
}

// A chunk of a long row per wavefront: the wave's minimum, one atomic.
__device__ __forceinline__ void cc_mngf_chunks(const int32_t *__restrict__ ci, const RowChunks &ch,
                                               const int32_t *__restrict__ gf, int32_t *__restrict__ mngf)
{
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / 64;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / 64;
    const unsigned lane = lane_id();
    for (int64_t c = wave; c < ch.n; c += nw) {
        int32_t m = INT32_MAX;
        for (int64_t p = ch.beg[c] + lane; p < ch.end[c]; p += 64) m = min(m, gf[ci[p]]);
        for (int o = 32; o > 0; o >>= 1) m = min(m, __shfl_xor(m, o, 64));
        if (lane == 0 && m < INT32_MAX) atomicMin(&mngf[ch.row[c]], m);
    }
}

// One launch per side: the long rows' chunks (a wave each), then the short
// rows (a lane each); they touch disjoint entries of mngf.
__global__ __launch_bounds__(CC_BLOCK) void k_cc_mngf(const int64_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                                      int64_t n, const int32_t *__restrict__ gf,
                                                      int32_t *__restrict__ mngf, RowChunks ch)
{
    cc_mngf_chunks(ci, ch, gf, mngf);
    cc_mngf_rows(rp, ci, n, gf, mngf);
}

// Steps 1 to 3: f(x(u)) = min(f(x(u)), mngf(u)); f(u) = min(f(u), mngf(u), gf(u)).
// Most vertices of a large component share their parent x(u), so the
// atomic is made only when it would lower f (f only decreases, so a stale
// read can only cause a needless atomic): atomics from many threads on one
// address are serialised.
__global__ void k_cc_hook(int64_t n, const int32_t *__restrict__ x, const int32_t *__restrict__ mngf,
                          const int32_t *__restrict__ gf, int32_t *f)
{
    for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n;
         u += (int64_t)gridDim.x * blockDim.x) {
        const int32_t m = mngf[u], xu = x[u];
        if (m < f[xu]) atomicMin(&f[xu], m);
        const int32_t h = min(m, gf[u]);
        if (h < f[u]) atomicMin(&f[u], h);
    }
}

// Steps 4 and 5: gf = f(f), x = f; count the grandparents that changed.
__global__ __launch_bounds__(CC_BLOCK) void k_cc_grand(int64_t n, const int32_t *__restrict__ f,
                                                       int32_t *__restrict__ gf, int32_t *__restrict__ dup,
                                                       int32_t *__restrict__ x, unsigned long long *changed)
{
    __shared__ unsigned long long cnt;
    if (threadIdx.x == 0) cnt = 0;
    __syncthreads();
    unsigned long long c = 0;
    for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n;
         u += (int64_t)gridDim.x * blockDim.x) {
        const int32_t fu = f[u];
        const int32_t g = f[fu];
        x[u] = fu;
        gf[u] = g;
        if (dup[u] != g) {
            dup[u] = g;
            c++;
        }
    }
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
    if (lane_id() == 0 && c) atomicAdd(&cnt, c);
    __syncthreads();
    if (threadIdx.x == 0 && cnt) atomicAdd(changed, cnt);
}

__global__ void k_cc_label(int64_t n, const int32_t *__restrict__ f, int64_t *__restrict__ out)
{
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x)
        out[v] = f[v];
}

}  // namespace

extern "C" int lagr_cc(lagr_vector *component, int64_t *iters_out, const lagr_graph G, lagr_ctx ctx, char *msg)
{
    if (!component || !G || !ctx) return lagr_fail(msg, LAGR_NULL_POINTER, "NULL argument");
    *component = nullptr;
    if (iters_out) *iters_out = 0;
    const lagr_matrix A = G->A;
    const int64_t n = A->nrows;
    const bool directed = G->kind == LAGR_ADJACENCY_DIRECTED;
    if (directed) TRY(graph_ensure_at(G, ctx, msg));
    lagr_vector lv = new (std::nothrow) lagr_vector_s();
    if (!lv) return lagr_fail(msg, LAGR_OUT_OF_MEMORY, "vector");
    lv->type = LAGR_INT64;
    lv->n = n;
    lv->fmt = LAGR_VEC_FULL;
    lv->nvals = n;
    lv->values_bytes = sizeof(int64_t) * (size_t)(n > 0 ? n : 1);
    lv->values = dev_alloc(lv->values_bytes);
    if (!lv->values) {
        delete lv;
        return lagr_fail(msg, LAGR_OUT_OF_MEMORY, "vector values");
    }
    int rc = LAGR_SUCCESS;
#define CC_TRY(expr)              \
    do {                          \
        rc = (expr);              \
        if (rc < 0) {             \
            lagr_vector_free(&lv); \
            return rc;            \
        }                         \
    } while (0)
    if (n == 0) {
        *component = lv;
        return lagr_ok(msg);
    }
    const size_t n1 = (size_t)n;
    int32_t *buf = (int32_t *)ws_get(ctx, WS_GEN_F, sizeof(int32_t) * 5 * n1);
    unsigned long long *changed = (unsigned long long *)ws_get(ctx, WS_COUNTERS, 64);
    if (!buf || !changed) CC_TRY(lagr_fail(msg, LAGR_OUT_OF_MEMORY, "cc workspace"));
    int32_t *f = buf, *gf = buf + n1, *dup = buf + 2 * n1, *mngf = buf + 3 * n1, *x = buf + 4 * n1;
    // neighbour sides: A, and AT for a directed graph; each with the chunk
    // list of its rows longer than CC_THREAD_ROW (the two lists live in
    // separate workspace slots)
    const lagr_matrix sides[2] = {A, directed ? G->AT : nullptr};
    RowChunks chs[2];
    const WsSlot cslots[2][2] = {{WS_CHUNK_A, WS_CHUNK_B}, {WS_GEN_G, WS_GEN_H}};
    for (int k = 0; k < 2; k++)
        if (sides[k])
            CC_TRY(row_chunks(ctx, sides[k]->rowptr, n, CC_THREAD_ROW, GRAPH_LONG_ROW, cslots[k][0], cslots[k][1],
                              &chs[k], msg));
    const unsigned vgrid = grid_for(n, CC_BLOCK, 8192);
    hipLaunchKernelGGL(k_cc_init, dim3(vgrid), dim3(CC_BLOCK), 0, ctx->stream, n, f, gf, dup, mngf, x);
    if (hipGetLastError() != hipSuccess) CC_TRY(lagr_fail(msg, LAGR_DEVICE_ERROR, "cc launch"));
    int64_t iters = 0;
    for (;;) {
        iters++;
        for (int k = 0; k < 2; k++) {
            if (!sides[k]) continue;
            const unsigned cgrid = chs[k].n > 0 ? grid_for(chs[k].n * 64, CC_BLOCK, 4096) : 0u;
            hipLaunchKernelGGL(k_cc_mngf, dim3(vgrid > cgrid ? vgrid : cgrid), dim3(CC_BLOCK), 0, ctx->stream,
                               sides[k]->rowptr, sides[k]->colidx, n, gf, mngf, chs[k]);
        }
        hipLaunchKernelGGL(k_cc_hook, dim3(vgrid), dim3(CC_BLOCK), 0, ctx->stream, n, x, mngf, gf, f);
        CC_TRY(fill_i64(ctx, (int64_t *)changed, 1, 0, msg));
        hipLaunchKernelGGL(k_cc_grand, dim3(grid_for(n, CC_BLOCK, 2048)), dim3(CC_BLOCK), 0, ctx->stream, n, f, gf,
                           dup, x, changed);
        if (hipGetLastError() != hipSuccess) CC_TRY(lagr_fail(msg, LAGR_DEVICE_ERROR, "cc launch"));
        unsigned long long h = 0;
        CC_TRY(read_back(ctx, &h, changed, sizeof(h), msg));
        if (h == 0) break;
        if (iters > n + 2) CC_TRY(lagr_fail(msg, LAGR_DEVICE_ERROR, "cc did not converge"));
    }
    hipLaunchKernelGGL(k_cc_label, dim3(vgrid), dim3(CC_BLOCK), 0, ctx->stream, n, f, (int64_t *)lv->values);
    if (hipGetLastError() != hipSuccess) CC_TRY(lagr_fail(msg, LAGR_DEVICE_ERROR, "cc launch"));
#undef CC_TRY
    if (iters_out) *iters_out = iters;
    *component = lv;
    return lagr_ok(msg);
}
