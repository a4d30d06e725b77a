// Many-graph triangle counting in one launch.
//
// The degree-ordered strictly lower parts L_g of many graphs are packed
// back to back: local int32 column ids, int64 row offsets into one shared
// id array, and a table of each graph's first row.  One work-balanced
// kernel (the row kernel of tc_device.h) covers every row of every graph
// and adds each graph's count to its own counter.  The launch -- counter
// reset and count kernel -- is captured once into a hipGraph on a stream
// the batch owns and replayed on every call; the grid size and the fixed
// per-row charge of the balanced partition are picked by timing a small
// grid of candidates (lagr_batch_autotune).
#include <new>
#include <vector>

#include "internal.h"
#include "tc_device.h"

struct lagr_batch_s {
    int device = 0;
    int num_cus = 256;
    int64_t ng = 0, R = 0, E = 0;
    int64_t *gbase = nullptr;      // ng + 1
    int64_t *rp = nullptr;         // R + 1
    int32_t *ci = nullptr;         // E
    int64_t *prefix = nullptr;     // R + 1, work prefix for prefix_charge
    int64_t prefix_charge = -1;
    unsigned long long *counts = nullptr;   // ng
    int64_t *host_counts = nullptr;         // pinned, ng
    hipStream_t stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    lagr_tune exec_tune{};
    lagr_tune tune{4, 64, 1};
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

__global__ __launch_bounds__(256) void k_batch_work(TcArgs a, int64_t charge, int64_t *__restrict__ work)
{
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / 64;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / 64;
    for (int64_t r0 = wave * 64; r0 < a.nrows; r0 += nw * 64) tc_row_work_wave(a, r0, work, charge);
}

__global__ __launch_bounds__(TC_BLOCK) void k_tc_batched(TcArgs a, const int64_t *__restrict__ prefix,
                                                         unsigned long long *__restrict__ per_graph)
{
    __shared__ TcWaveLds lds[TC_WAVES];
    const unsigned wave = threadIdx.x / 64;
    const int64_t w = (int64_t)blockIdx.x * TC_WAVES + wave;
    tc_rows_balanced<false>(a, lds[wave], nullptr, prefix, w, (int64_t)gridDim.x * TC_WAVES, per_graph);
}

TcArgs batch_args(const lagr_batch B)
{
    TcArgs a;
    a.nrows = B->R;
    a.Mrp = a.Arp = a.Brp = B->rp;
    a.Mci = a.Aci = a.Bci = B->ci;
    a.tc_form = 1;
    a.gbase = B->gbase;
    a.ngraphs = B->ng;
    return a;
}

int check_tune(const lagr_tune &t, char *msg)
{
    if (t.blocks_per_cu < 1 || t.blocks_per_cu > 16 || t.row_charge < 0 || t.row_charge > (1 << 20))
        return lagr_fail(msg, LAGR_INVALID_VALUE, "tune out of range (blocks_per_cu %d, row_charge %d)",
                         t.blocks_per_cu, t.row_charge);
    return LAGR_SUCCESS;
}

// work prefix for the given charge, on stream s
int batch_prefix(lagr_ctx ctx, lagr_batch B, int64_t charge, char *msg)
{
    if (B->prefix_charge == charge) return LAGR_SUCCESS;
    TRY(fill_i64(ctx, B->prefix + B->R, 1, 0, msg));
    if (B->R > 0) {
        hipLaunchKernelGGL(k_batch_work, dim3(grid_for(B->R, 256, 16384)), dim3(256), 0, ctx->stream,
                           batch_args(B), charge, B->prefix);
        LAUNCH_CHECK();
    }
    TRY(scan_exclusive_i64(ctx, B->prefix, B->prefix, B->R + 1, nullptr, msg));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    B->prefix_charge = charge;
    return LAGR_SUCCESS;
}

// counter reset + count kernel on stream s (what the hipGraph holds)
int enqueue_count(lagr_batch B, hipStream_t s, const lagr_tune &t, char *msg)
{
    hipLaunchKernelGGL(k_fill_u64_batch, dim3(grid_for(B->ng, 256, 1024)), dim3(256), 0, s, B->counts,
                       B->ng);
    LAUNCH_CHECK();
    if (B->R > 0) {
        hipLaunchKernelGGL(k_tc_batched, dim3((unsigned)(B->num_cus * t.blocks_per_cu)), dim3(TC_BLOCK), 0,
                           s, batch_args(B), (const int64_t *)B->prefix, B->counts);
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
    std::vector<int64_t> gb(ngraphs + 1), eb(ngraphs + 1);
    gb[0] = eb[0] = 0;
    for (int64_t g = 0; g < ngraphs; g++) {
        TRY(lagr_property_tc_lower(graphs[g], ctx, msg));
        gb[g + 1] = gb[g] + graphs[g]->L->nrows;
        eb[g + 1] = eb[g] + graphs[g]->L->nvals;
    }
    lagr_batch B = new (std::nothrow) lagr_batch_s();
    if (!B) return lagr_fail(msg, LAGR_OUT_OF_MEMORY, "batch");
    B->device = ctx->device;
    B->num_cus = ctx->num_cus;
    B->ng = ngraphs;
    B->R = gb[ngraphs];
    B->E = eb[ngraphs];
    B->gbase = (int64_t *)dev_alloc(8 * (ngraphs + 1));
    B->rp = (int64_t *)dev_alloc(8 * (B->R + 1));
    B->ci = (int32_t *)dev_alloc(4 * (B->E > 0 ? B->E : 1));
    B->prefix = (int64_t *)dev_alloc(8 * (B->R + 1));
    B->counts = (unsigned long long *)dev_alloc(8 * ngraphs);
    int rc = LAGR_SUCCESS;
    if (!B->gbase || !B->rp || !B->ci || !B->prefix || !B->counts ||
        hipHostMalloc(&B->host_counts, 8 * ngraphs, hipHostMallocDefault) != hipSuccess ||
        hipStreamCreateWithFlags(&B->stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&B->ready, hipEventDisableTiming) != hipSuccess) {
        lagr_batch_free(&B);
        return lagr_fail(msg, LAGR_OUT_OF_MEMORY, "batch arrays");
    }
    if (hipMemcpyAsync(B->gbase, gb.data(), 8 * (ngraphs + 1), hipMemcpyHostToDevice, ctx->stream) !=
        hipSuccess)
        rc = lagr_fail(msg, LAGR_DEVICE_ERROR, "batch table copy");
    for (int64_t g = 0; g < ngraphs && rc >= 0; g++) {
        const lagr_matrix L = graphs[g]->L;
        if (L->nrows > 0) {
            hipLaunchKernelGGL(k_pack_rowptr, dim3(grid_for(L->nrows, 256, 4096)), dim3(256), 0, ctx->stream,
                               L->rowptr, L->nrows, eb[g], B->rp + gb[g]);
            if (hipGetLastError() != hipSuccess) rc = lagr_fail(msg, LAGR_DEVICE_ERROR, "pack launch");
        }
        if (rc >= 0 && L->nvals > 0 &&
            hipMemcpyAsync(B->ci + eb[g], L->colidx, 4 * L->nvals, hipMemcpyDeviceToDevice, ctx->stream) !=
                hipSuccess)
            rc = lagr_fail(msg, LAGR_DEVICE_ERROR, "pack copy");
    }
    if (rc >= 0) rc = fill_i64(ctx, B->rp + B->R, 1, B->E, msg);
    if (rc >= 0) rc = batch_prefix(ctx, B, B->tune.row_charge, msg);
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
    TRY(batch_prefix(ctx, B, t.row_charge, msg));
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
    static const int bpc[] = {1, 2, 4, 8};
    static const int charge[] = {16, 64, 256};
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
    dev_free(B->gbase, 8 * (B->ng + 1));
    dev_free(B->rp, 8 * (B->R + 1));
    dev_free(B->ci, 4 * (B->E > 0 ? B->E : 1));
    dev_free(B->prefix, 8 * (B->R + 1));
    dev_free(B->counts, 8 * B->ng);
    if (B->host_counts) (void)hipHostFree(B->host_counts);
    if (B->ready) (void)hipEventDestroy(B->ready);
    if (B->stream) (void)hipStreamDestroy(B->stream);
    delete B;
    *Bp = nullptr;
    return LAGR_SUCCESS;
}
