// Many-graph triangle counting in one launch.
//
// Each graph's degree-ordered strictly lower part L_g and its min-side
// count plan (tc_device.h) are packed back to back: local int32 column
// ids, int64 row offsets into one shared id array, segment descriptors
// re-based onto that array, work items re-based onto the packed
// descriptors and onto global rows, and the graph of every item.  One
// kernel (the plan's wave loop, taking items from per-XCD work counters)
// covers every item of every graph and adds each graph's count to its own
// counter.  The launch -- counter reset and count kernel -- is captured once
// into a hipGraph on a stream the batch owns and replayed on every call; the
// grid size and the number of items taken per grab are picked by timing a
// small grid of candidates (lagr_batch_autotune).
#include <new>
#include <vector>

#include "internal.h"
#include "tc_device.h"

struct lagr_batch_s {
    int device = 0;
    int num_cus = 256;
    int64_t ng = 0, R = 0, E = 0, NE = 0, K = 0, NB = 0;
    int64_t *rp = nullptr;          // R + 1 packed row offsets
    int32_t *ci = nullptr;          // E packed local column ids
    uint64_t *ent = nullptr;        // NE packed segment descriptors
    uint32_t *bits = nullptr;       // NB packed bitmap words
    uint64_t *item = nullptr;       // K packed items
    int32_t *item_row = nullptr;    // K global rows
    int32_t *item_graph = nullptr;  // K graph ids
    unsigned long long *counts = nullptr;   // ng per-graph counts, then the work counters
    int64_t *host_counts = nullptr;         // pinned, ng
    hipStream_t stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    lagr_tune exec_tune{};
    lagr_tune tune{8, (int32_t)TC_DYN_ITEMS, 1};
    hipEvent_t ready = nullptr;
};

namespace {

// kernel used inside the capture (a plain fill: no memset node)
__global__ void k_fill_u64_batch(unsigned long long *__restrict__ p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0ull;
}

__global__ void k_pack_rowptr(const int64_t *__restrict__ rp, int64_t n, int64_t ebase,
                              int64_t *__restrict__ out)
{
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n;
         r += (int64_t)gridDim.x * blockDim.x)
        out[r] = rp[r] + ebase;
}

// out[i] = in[i] + add (re-bases packed descriptors: the offset fields sit
// in the high bits, so adding a shifted base moves them)
__global__ void k_pack_add_u64(const uint64_t *__restrict__ in, int64_t n, uint64_t add,
                               uint64_t *__restrict__ out)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        out[i] = in[i] + add;
}

// Plan entries: segment descriptors move by add_seg, bitmap entries
// (TC_PLAN_BITS set) by add_bits.
__global__ void k_pack_ent(const uint64_t *__restrict__ in, int64_t n, uint64_t add_seg, uint64_t add_bits,
                           uint64_t *__restrict__ out)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t x = in[i];
        out[i] = x + ((x & TC_PLAN_BITS) ? add_bits : add_seg);
    }
}

__global__ void k_pack_items(const int32_t *__restrict__ row, int64_t n, int32_t rbase, int32_t g,
                             int32_t *__restrict__ row_out, int32_t *__restrict__ graph_out)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        row_out[i] = row[i] + rbase;
        graph_out[i] = g;
    }
}

// Items taken `grain` at a time from per-XCD counters (ctr, zeroed with
// the per-graph counts before each launch), as in the single-graph count;
// OFF32 when the packed ids and bitmap words each number below 2^30.
template <bool OFF32>
__global__ __launch_bounds__(TC_BLOCK, 8) void k_tc_batched(PlanArgs a, unsigned long long *ctr, int64_t grain)
{
    __shared__ TcWaveLds lds[TC_WAVES];
    tc_dyn_wave<true, OFF32>(a, lds[threadIdx.x / 64], ctr, (int)(blockIdx.x % TC_DYN_PARTS), grain);
}

constexpr int64_t BATCH_CTRS = (int64_t)TC_DYN_STRIDE * TC_DYN_PARTS;   // after the ng counts

PlanArgs batch_args(const lagr_batch B)
{
    PlanArgs a;
    a.nitems = B->K;
    a.Lrp = B->rp;
    a.Lci = B->ci;
    a.ent = B->ent;
    a.bits = B->bits;
    a.item = B->item;
    a.item_row = B->item_row;
    a.item_graph = B->item_graph;
    a.per_graph = B->counts;
    return a;
}

int check_tune(const lagr_tune &t, char *msg)
{
    if (t.blocks_per_cu < 1 || t.blocks_per_cu > 16 || t.row_charge < 1 || t.row_charge > (1 << 20))
        return lagr_fail(msg, LAGR_INVALID_VALUE, "tune out of range (blocks_per_cu %d, row_charge %d)",
                         t.blocks_per_cu, t.row_charge);
    return LAGR_SUCCESS;
}

// counter reset + count kernel on stream s (what the hipGraph holds)
int enqueue_count(lagr_batch B, hipStream_t s, const lagr_tune &t, char *msg)
{
    hipLaunchKernelGGL(k_fill_u64_batch, dim3(grid_for(B->ng + BATCH_CTRS, 256, 1024)), dim3(256), 0, s, B->counts,
                       B->ng + BATCH_CTRS);
    LAUNCH_CHECK();
    if (B->K > 0) {
        // a multiple of 8 workgroups, so every XCD gets the same number
        const unsigned blocks = (unsigned)(B->num_cus * t.blocks_per_cu);
        const int64_t lim = (int64_t)1 << 30;
        if (B->E < lim && B->NB < lim)
            hipLaunchKernelGGL(k_tc_batched<true>, dim3(blocks), dim3(TC_BLOCK), 0, s, batch_args(B), B->counts + B->ng,
                               (int64_t)t.row_charge);
        else
            hipLaunchKernelGGL(k_tc_batched<false>, dim3(blocks), dim3(TC_BLOCK), 0, s, batch_args(B),
                               B->counts + B->ng, (int64_t)t.row_charge);
        LAUNCH_CHECK();
    }
    return LAGR_SUCCESS;
}

void drop_graph(lagr_batch B)
{
    if (B->exec) (void)hipGraphExecDestroy(B->exec);
    if (B->graph) (void)hipGraphDestroy(B->graph);
    B->exec = nullptr;
    B->graph = nullptr;
}

}  // namespace

extern "C" int lagr_batch_new(lagr_batch *Bout, const lagr_graph *graphs, int64_t ngraphs, lagr_ctx ctx,
                              char *msg)
{
    if (!Bout || !ctx || (ngraphs > 0 && !graphs)) return lagr_fail(msg, LAGR_NULL_POINTER, "NULL argument");
    *Bout = nullptr;
    if (ngraphs < 1) return lagr_fail(msg, LAGR_INVALID_VALUE, "a batch needs at least one graph");
    for (int64_t g = 0; g < ngraphs; g++)
        if (!graphs[g]) return lagr_fail(msg, LAGR_NULL_POINTER, "graph %lld is NULL", (long long)g);
    // Basic mode: compute every missing triangle-count operand
    std::vector<int64_t> gb(ngraphs + 1), eb(ngraphs + 1), nb(ngraphs + 1), kb(ngraphs + 1), bb(ngraphs + 1);
    gb[0] = eb[0] = nb[0] = kb[0] = bb[0] = 0;
    for (int64_t g = 0; g < ngraphs; g++) {
        TRY(lagr_property_tc_lower(graphs[g], ctx, msg));
        gb[g + 1] = gb[g] + graphs[g]->L->nrows;
        eb[g + 1] = eb[g] + graphs[g]->L->nvals;
        nb[g + 1] = nb[g] + graphs[g]->tcplan->ent_cap;
        kb[g + 1] = kb[g] + graphs[g]->tcplan->nitems;
        bb[g + 1] = bb[g] + graphs[g]->tcplan->nbits;
    }
    if (gb[ngraphs] >= ((int64_t)1 << 31))
        return lagr_fail(msg, LAGR_NOT_IMPLEMENTED, "a batch holds fewer than 2^31 rows");
    if (eb[ngraphs] >= ((int64_t)1 << (64 - TC_PLAN_LEN_BITS)) ||
        nb[ngraphs] >= ((int64_t)1 << (64 - TC_PLAN_CNT_BITS)))
        return lagr_fail(msg, LAGR_NOT_IMPLEMENTED, "batch too large for the packed plan");
    lagr_batch B = new (std::nothrow) lagr_batch_s();
    if (!B) return lagr_fail(msg, LAGR_OUT_OF_MEMORY, "batch");
    B->device = ctx->device;
    B->num_cus = ctx->num_cus;
    B->ng = ngraphs;
    B->R = gb[ngraphs];
    B->E = eb[ngraphs];
    B->NE = nb[ngraphs];
    B->K = kb[ngraphs];
    B->NB = bb[ngraphs];
    auto one = [](int64_t x) { return (size_t)(x > 0 ? x : 1); };
    B->rp = (int64_t *)dev_alloc(8 * (B->R + 1));
    B->ci = (int32_t *)dev_alloc(4 * one(B->E));
    B->ent = (uint64_t *)dev_alloc(8 * one(B->NE));
    B->bits = (uint32_t *)dev_alloc(4 * one(B->NB));
    B->item = (uint64_t *)dev_alloc(8 * one(B->K));
    B->item_row = (int32_t *)dev_alloc(4 * one(B->K));
    B->item_graph = (int32_t *)dev_alloc(4 * one(B->K));
    B->counts = (unsigned long long *)dev_alloc(8 * (ngraphs + BATCH_CTRS));
    int rc = LAGR_SUCCESS;
    if (!B->rp || !B->ci || !B->ent || !B->bits || !B->item || !B->item_row || !B->item_graph || !B->counts ||
        hipHostMalloc(&B->host_counts, 8 * ngraphs, hipHostMallocDefault) != hipSuccess ||
        hipStreamCreateWithFlags(&B->stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&B->ready, hipEventDisableTiming) != hipSuccess) {
        lagr_batch_free(&B);
        return lagr_fail(msg, LAGR_OUT_OF_MEMORY, "batch arrays");
    }
    for (int64_t g = 0; g < ngraphs && rc >= 0; g++) {
        const lagr_matrix L = graphs[g]->L;
        const TcPlan *P = graphs[g]->tcplan;
        if (L->nrows > 0)
            hipLaunchKernelGGL(k_pack_rowptr, dim3(grid_for(L->nrows, 256, 4096)), dim3(256), 0, ctx->stream,
                               L->rowptr, L->nrows, eb[g], B->rp + gb[g]);
        // the whole entry array (each virtual row's region), unused slots too
        if (P->ent_cap > 0)
            hipLaunchKernelGGL(k_pack_ent, dim3(grid_for(P->ent_cap, 256, 4096)), dim3(256), 0, ctx->stream,
                               P->ent, P->ent_cap, (uint64_t)eb[g] << TC_PLAN_LEN_BITS, (uint64_t)bb[g],
                               B->ent + nb[g]);
        if (P->nitems > 0) {
            hipLaunchKernelGGL(k_pack_add_u64, dim3(grid_for(P->nitems, 256, 4096)), dim3(256), 0, ctx->stream,
                               P->item, P->nitems, (uint64_t)nb[g] << TC_PLAN_CNT_BITS, B->item + kb[g]);
            hipLaunchKernelGGL(k_pack_items, dim3(grid_for(P->nitems, 256, 4096)), dim3(256), 0, ctx->stream,
                               P->item_row, P->nitems, (int32_t)gb[g], (int32_t)g, B->item_row + kb[g],
                               B->item_graph + kb[g]);
        }
        if (hipGetLastError() != hipSuccess) rc = lagr_fail(msg, LAGR_DEVICE_ERROR, "pack launch");
        if (rc >= 0 && L->nvals > 0 &&
            hipMemcpyAsync(B->ci + eb[g], L->colidx, 4 * L->nvals, hipMemcpyDeviceToDevice, ctx->stream) !=
                hipSuccess)
            rc = lagr_fail(msg, LAGR_DEVICE_ERROR, "pack copy");
        if (rc >= 0 && P->nbits > 0 &&
            hipMemcpyAsync(B->bits + bb[g], P->bits, 4 * P->nbits, hipMemcpyDeviceToDevice, ctx->stream) !=
                hipSuccess)
            rc = lagr_fail(msg, LAGR_DEVICE_ERROR, "pack copy");
    }
    if (rc >= 0) rc = fill_i64(ctx, B->rp + B->R, 1, B->E, msg);
    if (rc < 0) {
        lagr_batch_free(&B);
        return rc;
    }
    *Bout = B;
    return lagr_ok(msg);
}

extern "C" int lagr_batch_info(const lagr_batch B, int64_t *ngraphs, int64_t *rows, int64_t *entries,
                               char *msg)
{
    if (!B) return lagr_fail(msg, LAGR_NULL_POINTER, "batch is NULL");
    if (ngraphs) *ngraphs = B->ng;
    if (rows) *rows = B->R;
    if (entries) *entries = B->E;
    return lagr_ok(msg);
}

extern "C" int lagr_tc_batched(int64_t *counts, lagr_batch B, const lagr_tune *tune, lagr_ctx ctx, char *msg)
{
    if (!counts || !B || !ctx) return lagr_fail(msg, LAGR_NULL_POINTER, "NULL argument");
    const lagr_tune t = tune ? *tune : B->tune;
    TRY(check_tune(t, msg));
    if (t.use_graph) {
        const bool stale = !B->exec || B->exec_tune.blocks_per_cu != t.blocks_per_cu ||
                           B->exec_tune.row_charge != t.row_charge;
        if (stale) {
            drop_graph(B);
            HIP_TRY(hipStreamBeginCapture(B->stream, hipStreamCaptureModeThreadLocal));
            const int rc = enqueue_count(B, B->stream, t, msg);
            hipGraph_t gr = nullptr;
            const hipError_t e = hipStreamEndCapture(B->stream, &gr);
            if (rc < 0) {
                if (gr) (void)hipGraphDestroy(gr);
                return rc;
            }
            if (e != hipSuccess) return lagr_fail(msg, LAGR_DEVICE_ERROR, "capture: %s", hipGetErrorString(e));
            B->graph = gr;
            HIP_TRY(hipGraphInstantiate(&B->exec, B->graph, nullptr, nullptr, 0));
            B->exec_tune = t;
        }
        // the replay follows all work already queued on the caller's stream
        HIP_TRY(hipEventRecord(B->ready, ctx->stream));
        HIP_TRY(hipStreamWaitEvent(B->stream, B->ready, 0));
        HIP_TRY(hipGraphLaunch(B->exec, B->stream));
        HIP_TRY(hipMemcpyAsync(B->host_counts, B->counts, 8 * B->ng, hipMemcpyDeviceToHost, B->stream));
        HIP_TRY(hipStreamSynchronize(B->stream));
    } else {
        TRY(enqueue_count(B, ctx->stream, t, msg));
        HIP_TRY(hipMemcpyAsync(B->host_counts, B->counts, 8 * B->ng, hipMemcpyDeviceToHost, ctx->stream));
        HIP_TRY(hipStreamSynchronize(ctx->stream));
    }
    memcpy(counts, B->host_counts, 8 * B->ng);
    return lagr_ok(msg);
}

extern "C" int lagr_batch_autotune(lagr_tune *best, lagr_batch B, lagr_ctx ctx, char *msg)
{
    if (!best || !B || !ctx) return lagr_fail(msg, LAGR_NULL_POINTER, "NULL argument");
    static const int bpc[] = {2, 4, 8};
    static const int charge[] = {2, 4, 8};   // items per grab
    std::vector<int64_t> scratch(B->ng);
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    float best_ms = 1e30f;
    lagr_tune pick = B->tune;
    int rc = LAGR_SUCCESS;
    for (int c : charge) {
        for (int b : bpc) {
            lagr_tune t{b, c, 0};
            rc = lagr_tc_batched(scratch.data(), B, &t, ctx, msg);   // warm
            if (rc < 0) break;
            float ms_min = 1e30f;
            for (int rep = 0; rep < 2 && rc >= 0; rep++) {
                (void)hipEventRecord(e0, ctx->stream);
                rc = enqueue_count(B, ctx->stream, t, msg);
                (void)hipEventRecord(e1, ctx->stream);
                if (hipEventSynchronize(e1) != hipSuccess) rc = lagr_fail(msg, LAGR_DEVICE_ERROR, "autotune");
                float ms = 0.f;
                (void)hipEventElapsedTime(&ms, e0, e1);
                ms_min = ms < ms_min ? ms : ms_min;
            }
            if (rc < 0) break;
            if (ms_min < best_ms) {
                best_ms = ms_min;
                pick = t;
            }
        }
        if (rc < 0) break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc < 0) return rc;
    pick.use_graph = 1;
    B->tune = pick;
    *best = pick;
    return lagr_ok(msg);
}

extern "C" int lagr_batch_free(lagr_batch *Bp)
{
    if (!Bp || !*Bp) return LAGR_SUCCESS;
    lagr_batch B = *Bp;
    if (B->stream) (void)hipStreamSynchronize(B->stream);
    drop_graph(B);
    auto one = [](int64_t x) { return (size_t)(x > 0 ? x : 1); };
    dev_free(B->rp, 8 * (B->R + 1));
    dev_free(B->ci, 4 * one(B->E));
    dev_free(B->ent, 8 * one(B->NE));
    dev_free(B->bits, 4 * one(B->NB));
    dev_free(B->item, 8 * one(B->K));
    dev_free(B->item_row, 4 * one(B->K));
    dev_free(B->item_graph, 4 * one(B->K));
    dev_free(B->counts, 8 * (B->ng + BATCH_CTRS));
    if (B->host_counts) (void)hipHostFree(B->host_counts);
    if (B->ready) (void)hipEventDestroy(B->ready);
    if (B->stream) (void)hipStreamDestroy(B->stream);
    delete B;
    *Bp = nullptr;
    return LAGR_SUCCESS;
}
