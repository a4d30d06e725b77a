// Masked plus.pair dot product and its fusion with reduce: triangle
// counting (Section IV-E, Algorithm 6) as C<s(L)> = L plus.pair L^T and
// t = sum(C), computed without forming C (the fusion Section VI-B asks
// for).  The row kernel is described in tc_device.h.
#include "internal.h"
#include "tc_device.h"

namespace {

__global__ __launch_bounds__(256) void k_tc_row_work(TcArgs a, int64_t *__restrict__ work)
{
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / 64;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / 64;
    for (int64_t r0 = wave * 64; r0 < a.nrows; r0 += nw * 64) tc_row_work_wave(a, r0, work);
}

template <bool PER_ENTRY>
__global__ __launch_bounds__(TC_BLOCK) void k_tc_rows(TcArgs a, const int64_t *__restrict__ prefix,
                                                      unsigned long long *__restrict__ total,
                                                      int64_t *__restrict__ entry_counts)
{
    __shared__ TcWaveLds lds[TC_WAVES];
    const unsigned wave = threadIdx.x / 64;
    const int64_t w = (int64_t)blockIdx.x * TC_WAVES + wave;
    unsigned long long acc = tc_rows_balanced<PER_ENTRY>(a, lds[wave], entry_counts, prefix, w,
                                                         (int64_t)gridDim.x * TC_WAVES);
    if (!PER_ENTRY) {
        // one atomic per workgroup (atomics on one address serialise)
        for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
        __shared__ unsigned long long wsum[TC_WAVES];
        if (lane_id() == 0) wsum[wave] = acc;
        __syncthreads();
        if (threadIdx.x == 0) {
            unsigned long long t = 0;
            for (int i = 0; i < TC_WAVES; i++) t += wsum[i];
            if (t) atomicAdd(total, t);
        }
    }
}

// ------------------------------------------------- min-side count plan

__device__ __forceinline__ uint64_t plan_pack(int64_t off, int64_t len)
{
    return ((uint64_t)off << TC_PLAN_LEN_BITS) | (uint64_t)len;
}

// B-side rows j below PLAN_HOT (the highest-degree vertices after the
// relabel) receive most B entries; a workgroup first gathers their counts
// in LDS, so each takes one global atomic per workgroup instead of one per
// entry (same-address atomics serialise).  The kernels read the row of
// every entry of L (rowid), so every thread knows its entry's row and
// column directly; workgroup g takes the g-th contiguous share of the
// entries, which keeps its hot counts dense.  The count kernel's atomic
// returns the workgroup's offset inside each hot row (boff, PLAN_GRID x
// PLAN_HOT), which the fill kernel, run on the same partition, starts from.
// The kernels chain dependent loads (row, row start, column, column's row),
// so they run 512-thread workgroups, four per CU (the 32 KiB LDS table
// allows it), for more loads in flight.
constexpr int PLAN_HOT = 8192;
constexpr int PLAN_BLOCK = 512;
constexpr unsigned PLAN_GRID = 1024;

struct PlanEntry {
    int64_t i, j, p, si;   // row, column, position in row i, start of row i
};

// rowpk[r] = plan_pack(start of row r, length of row r): one gather gives
// both (the plan kernels gather it for the row and for the column of every
// entry, at random columns).
__device__ __forceinline__ PlanEntry plan_entry(const int32_t *__restrict__ rowid, const int32_t *__restrict__ ci,
                                                const uint64_t *__restrict__ rowpk, int64_t e)
{
    PlanEntry x;
    x.i = rowid[e];
    x.j = ci[e];
    x.si = (int64_t)(rowpk[x.i] >> TC_PLAN_LEN_BITS);
    x.p = e - x.si;
    return x;
}

__global__ void k_row_pack(const int64_t *__restrict__ rp, int64_t n, uint64_t *__restrict__ rowpk)
{
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n;
         r += (int64_t)gridDim.x * blockDim.x)
        rowpk[r] = plan_pack(rp[r], rp[r + 1] - rp[r]);
}

// Entries per virtual row (cnt: 2n+1 entries, zero on entry).  The loops
// step whole wavefronts, so every lane of a wave takes part in each
// iteration's ballots and shuffles.
__global__ __launch_bounds__(PLAN_BLOCK) void k_plan_count(const int32_t *__restrict__ rowid,
                                                           const int32_t *__restrict__ ci, int64_t nnz,
                                                           const uint64_t *__restrict__ rowpk, int64_t n,
                                                           unsigned long long *__restrict__ cnt,
                                                           unsigned *__restrict__ boff)
{
    __shared__ unsigned hot[PLAN_HOT];
    for (int x = threadIdx.x; x < PLAN_HOT; x += PLAN_BLOCK) hot[x] = 0u;
    __syncthreads();
    const int64_t share = (nnz + gridDim.x - 1) / gridDim.x;
    const int64_t e0 = (int64_t)blockIdx.x * share, e1 = min(nnz, e0 + share);
    const unsigned lane = lane_id();
    for (int64_t w0 = e0 + (threadIdx.x & ~63u); w0 < e1; w0 += PLAN_BLOCK) {
        const int64_t e = w0 + lane;
        bool a_side = false;
        int32_t key = -1;
        if (e < e1) {
            const PlanEntry x = plan_entry(rowid, ci, rowpk, e);
            key = (int32_t)x.i;
            const int64_t lj = (int64_t)(rowpk[x.j] & ((1ull << TC_PLAN_LEN_BITS) - 1));
            if (x.p > 0 && lj > 0) {
                if (lj <= x.p) a_side = true;
                else if (x.j < PLAN_HOT) atomicAdd(&hot[x.j], 1u);
                else atomicAdd(&cnt[n + x.j], 1ull);
            }
        }
        const WaveRun w = wave_run(key);
        const uint64_t take = __ballot(a_side) & w.run;
        if (lane == w.head && take) atomicAdd(&cnt[key], (unsigned long long)__popcll(take));
    }
    __syncthreads();
    unsigned *mine = boff + (size_t)blockIdx.x * PLAN_HOT;
    for (int x = threadIdx.x; x < PLAN_HOT && x < n; x += PLAN_BLOCK)
        mine[x] = hot[x] ? (unsigned)atomicAdd(&cnt[n + x], (unsigned long long)hot[x]) : 0u;
}

// cur (a copy of the first 2n offsets) holds the write cursor of each
// virtual row; the order of the entries within a row is immaterial.  Hot
// B rows hand out positions from LDS as offsets from bstart, the first
// B-side offset (the host checks that the B side spans fewer than 2^32
// entries), starting at the workgroup's range from the count kernel.
__global__ __launch_bounds__(PLAN_BLOCK) void k_plan_fill(const int32_t *__restrict__ rowid,
                                                          const int32_t *__restrict__ ci, int64_t nnz,
                                                          const uint64_t *__restrict__ rowpk, int64_t n,
                                                          const int64_t *__restrict__ trp, int64_t bstart,
                                                          const unsigned *__restrict__ boff,
                                                          unsigned long long *__restrict__ cur,
                                                          uint64_t *__restrict__ ent)
{
    __shared__ unsigned hot[PLAN_HOT];
    const unsigned *mine = boff + (size_t)blockIdx.x * PLAN_HOT;
    for (int x = threadIdx.x; x < PLAN_HOT && x < n; x += PLAN_BLOCK)
        hot[x] = (unsigned)(trp[n + x] - bstart) + mine[x];
    __syncthreads();
    const int64_t share = (nnz + gridDim.x - 1) / gridDim.x;
    const int64_t e0 = (int64_t)blockIdx.x * share, e1 = min(nnz, e0 + share);
    const unsigned lane = lane_id();
    for (int64_t w0 = e0 + (threadIdx.x & ~63u); w0 < e1; w0 += PLAN_BLOCK) {
        const int64_t e = w0 + lane;
        bool a_side = false;
        int32_t key = -1;
        uint64_t packed = 0;
        if (e < e1) {
            const PlanEntry x = plan_entry(rowid, ci, rowpk, e);
            key = (int32_t)x.i;
            const uint64_t pj = rowpk[x.j];
            const int64_t lj = (int64_t)(pj & ((1ull << TC_PLAN_LEN_BITS) - 1));
            if (x.p > 0 && lj > 0) {
                if (lj <= x.p) {
                    a_side = true;
                    packed = pj;
                } else if (x.j < PLAN_HOT) {
                    ent[bstart + atomicAdd(&hot[x.j], 1u)] = plan_pack(x.si, x.p);
                } else {
                    ent[atomicAdd(&cur[n + x.j], 1ull)] = plan_pack(x.si, x.p);
                }
            }
        }
        const WaveRun w = wave_run(key);
        const uint64_t take = __ballot(a_side) & w.run;
        unsigned long long base = 0;
        if (lane == w.head && take) base = atomicAdd(&cur[key], (unsigned long long)__popcll(take));
        base = (unsigned long long)__shfl((long long)base, (int)w.head, 64);
        if (a_side) ent[base + __popcll(take & w.before)] = packed;
    }
}

__global__ void k_plan_items(const int64_t *__restrict__ trp, int64_t nv, int64_t *__restrict__ irp)
{
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < nv;
         r += (int64_t)gridDim.x * blockDim.x)
        irp[r] = (trp[r + 1] - trp[r] + 63) / 64;
}

// First virtual row r in [0, nv) with irp[r + 1] > k.
__device__ __forceinline__ int64_t plan_row_of(const int64_t *__restrict__ irp, int64_t nv, int64_t k)
{
    int64_t lo = 0, hi = nv - 1;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (irp[mid + 1] > k) hi = mid;
        else lo = mid + 1;
    }
    return lo;
}

__global__ void k_plan_item_work(const int64_t *__restrict__ Lrp, int64_t n,
                                 const int64_t *__restrict__ trp, const int64_t *__restrict__ irp,
                                 const uint64_t *__restrict__ ent, int64_t nitems,
                                 uint64_t *__restrict__ item, int32_t *__restrict__ item_row,
                                 int64_t *__restrict__ work)
{
    const uint64_t lmask = (1ull << TC_PLAN_LEN_BITS) - 1;
    const int64_t nv = 2 * n;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nitems;
         k += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = plan_row_of(irp, nv, k);
        const int64_t e0 = trp[r] + 64 * (k - irp[r]);
        const int64_t e1 = min(trp[r + 1], e0 + 64);
        const int64_t m = r < n ? r : r - n;
        int64_t ids = 0;
        for (int64_t e = e0; e < e1; e++) ids += (int64_t)(ent[e] & lmask);
        const int64_t units = (ids + 63) >> 6;
        int64_t w = TC_COST_ITEM + TC_COST_BATCH * ((units + TC_FLAT_INFLIGHT - 1) / TC_FLAT_INFLIGHT);
        if (k == irp[r]) w += TC_COST_MARK * ((Lrp[m + 1] - Lrp[m] + 63) >> 6);
        item[k] = ((uint64_t)e0 << TC_PLAN_CNT_BITS) | (uint64_t)(e1 - e0);
        item_row[k] = (int32_t)m;
        work[k] = w;
    }
}

// Each workgroup writes its count to partial[blockIdx.x]; k_sum_partials
// adds them (atomics on one address from every wavefront would serialise).
// Workgroups are dispatched to the 8 XCDs in turn (workgroup b runs on XCD
// b mod 8), and each XCD has its own L2: the waves of workgroup b take their
// items from the counter of eighth b mod 8 first (tc_dyn_wave).  Each
// workgroup writes its count to partial[blockIdx.x].
__global__ __launch_bounds__(TC_BLOCK, 8) void k_tc_split(PlanArgs a, unsigned long long *__restrict__ partial,
                                                          unsigned long long *__restrict__ ctr)
{
    __shared__ TcWaveLds lds[TC_WAVES];
    unsigned long long acc = tc_dyn_wave(a, lds[threadIdx.x / 64], ctr, (int)(blockIdx.x % TC_DYN_PARTS));
    __shared__ unsigned long long wsum[TC_WAVES];
    if (lane_id() == 0) wsum[threadIdx.x / 64] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int i = 0; i < TC_WAVES; i++) t += wsum[i];
        partial[blockIdx.x] = t;
    }
}

__global__ __launch_bounds__(256) void k_sum_partials(const unsigned long long *__restrict__ partial, int64_t n,
                                                      unsigned long long *__restrict__ out)
{
    __shared__ unsigned long long s[256];
    unsigned long long t = 0;
    for (int64_t i = threadIdx.x; i < n; i += 256) t += partial[i];
    s[threadIdx.x] = t;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = s[0];
}

}  // namespace

void tc_plan_free(lagr_graph G)
{
    TcPlan *P = G->tcplan;
    if (!P) return;
    const size_t nv1 = (size_t)(2 * P->n + 1);
    dev_free(P->trp, 8 * nv1);
    dev_free(P->irp, 8 * nv1);
    dev_free(P->iprefix, 8 * (size_t)(P->nitems + 1));
    dev_free(P->ent, 8 * (size_t)(P->nent > 0 ? P->nent : 1));
    dev_free(P->item, 8 * (size_t)(P->nitems > 0 ? P->nitems : 1));
    dev_free(P->item_row, 4 * (size_t)(P->nitems > 0 ? P->nitems : 1));
    delete P;
    G->tcplan = nullptr;
}

int tc_plan_build(lagr_ctx ctx, lagr_graph G, const int32_t *rowid, char *msg)
{
    const lagr_matrix Lm = G->L;
    const int64_t n = Lm->nrows, nv = 2 * n;
    if (Lm->nvals >= ((int64_t)1 << (64 - TC_PLAN_LEN_BITS)))
        return lagr_fail(msg, LAGR_NOT_IMPLEMENTED, "L too large for the count plan");
    TcPlan *P = new (std::nothrow) TcPlan();
    if (!P) return lagr_fail(msg, LAGR_OUT_OF_MEMORY, "count plan");
    P->n = n;
    G->tcplan = P;
    auto fail = [&](int rc) {
        tc_plan_free(G);
        return rc;
    };
    P->trp = (int64_t *)dev_alloc(8 * (size_t)(nv + 1));
    P->irp = (int64_t *)dev_alloc(8 * (size_t)(nv + 1));
    if (!P->trp || !P->irp) return fail(lagr_fail(msg, LAGR_OUT_OF_MEMORY, "count plan"));
    int rc;
    if ((rc = fill_i64(ctx, P->trp, nv + 1, 0, msg)) < 0) return fail(rc);
    const int64_t nnz = Lm->nvals;
    if (G->L_maxrow >= ((int64_t)1 << TC_PLAN_LEN_BITS))
        return fail(lagr_fail(msg, LAGR_NOT_IMPLEMENTED, "rows of L too long for the count plan"));
    unsigned *boff = (unsigned *)ws_get(ctx, WS_GEN_H, sizeof(unsigned) * (size_t)PLAN_GRID * PLAN_HOT);
    uint64_t *rowpk = (uint64_t *)ws_get(ctx, WS_GEN_E, sizeof(uint64_t) * (size_t)(n > 0 ? n : 1));
    if (!boff || !rowpk) return fail(lagr_fail(msg, LAGR_OUT_OF_MEMORY, "count plan"));
    if (n > 0) {
        hipLaunchKernelGGL(k_row_pack, dim3(grid_for(n, 256, 16384)), dim3(256), 0, ctx->stream, Lm->rowptr, n,
                           rowpk);
        if (hipGetLastError() != hipSuccess) return fail(lagr_fail(msg, LAGR_DEVICE_ERROR, "plan launch"));
    }
    if (nnz > 0) {
        hipLaunchKernelGGL(k_plan_count, dim3(PLAN_GRID), dim3(PLAN_BLOCK), 0, ctx->stream, rowid, Lm->colidx, nnz,
                           rowpk, n, (unsigned long long *)P->trp, boff);
        if (hipGetLastError() != hipSuccess) return fail(lagr_fail(msg, LAGR_DEVICE_ERROR, "plan launch"));
    }
    if ((rc = scan_exclusive_i64(ctx, P->trp, P->trp, nv + 1, &P->nent, msg)) < 0) return fail(rc);
    int64_t bstart = 0;
    if (n > 0 && (rc = read_back(ctx, &bstart, P->trp + n, sizeof(bstart), msg)) < 0) return fail(rc);
    if (P->nent - bstart >= ((int64_t)1 << 32))
        return fail(lagr_fail(msg, LAGR_NOT_IMPLEMENTED, "L too large for the count plan"));
    P->ent = (uint64_t *)dev_alloc(8 * (size_t)(P->nent > 0 ? P->nent : 1));
    unsigned long long *cur = (unsigned long long *)ws_get(ctx, WS_TC_WORK, 8 * (size_t)(nv > 0 ? nv : 1));
    if (!P->ent || !cur) return fail(lagr_fail(msg, LAGR_OUT_OF_MEMORY, "count plan"));
    if (n > 0) {
        if (hipMemcpyAsync(cur, P->trp, 8 * (size_t)nv, hipMemcpyDeviceToDevice, ctx->stream) != hipSuccess)
            return fail(lagr_fail(msg, LAGR_DEVICE_ERROR, "plan copy"));
        if (nnz > 0)
            hipLaunchKernelGGL(k_plan_fill, dim3(PLAN_GRID), dim3(PLAN_BLOCK), 0, ctx->stream, rowid, Lm->colidx,
                               nnz, rowpk, n, P->trp, bstart, boff, cur, P->ent);
        hipLaunchKernelGGL(k_plan_items, dim3(grid_for(nv, 256, 16384)), dim3(256), 0, ctx->stream, P->trp,
                           nv, P->irp);
        if (hipGetLastError() != hipSuccess) return fail(lagr_fail(msg, LAGR_DEVICE_ERROR, "plan launch"));
    }
    if ((rc = fill_i64(ctx, P->irp + nv, 1, 0, msg)) < 0) return fail(rc);
    if ((rc = scan_exclusive_i64(ctx, P->irp, P->irp, nv + 1, &P->nitems, msg)) < 0) return fail(rc);
    P->iprefix = (int64_t *)dev_alloc(8 * (size_t)(P->nitems + 1));
    P->item = (uint64_t *)dev_alloc(8 * (size_t)(P->nitems > 0 ? P->nitems : 1));
    P->item_row = (int32_t *)dev_alloc(4 * (size_t)(P->nitems > 0 ? P->nitems : 1));
    if (!P->iprefix || !P->item || !P->item_row) return fail(lagr_fail(msg, LAGR_OUT_OF_MEMORY, "count plan"));
    if (P->nitems > 0) {
        hipLaunchKernelGGL(k_plan_item_work, dim3(grid_for(P->nitems, 256, 16384)), dim3(256), 0, ctx->stream,
                           Lm->rowptr, n, P->trp, P->irp, P->ent, P->nitems, P->item, P->item_row, P->iprefix);
        if (hipGetLastError() != hipSuccess) return fail(lagr_fail(msg, LAGR_DEVICE_ERROR, "plan launch"));
    }
    if ((rc = fill_i64(ctx, P->iprefix + P->nitems, 1, 0, msg)) < 0) return fail(rc);
    if ((rc = scan_exclusive_i64(ctx, P->iprefix, P->iprefix, P->nitems + 1, nullptr, msg)) < 0) return fail(rc);
    return LAGR_SUCCESS;
}

// total_dev[0] (zeroed here) receives the sum in the fused form.
int tc_masked_dot(lagr_ctx ctx, const TcArgs &a, bool per_entry, unsigned long long *total_dev,
                  int64_t *entry_counts, char *msg)
{
    TRY(fill_i64(ctx, (int64_t *)total_dev, 1, 0, msg));
    if (a.nrows <= 0) return LAGR_SUCCESS;
    int64_t *prefix = (int64_t *)ws_get(ctx, WS_TC_WORK, sizeof(int64_t) * (a.nrows + 1));
    if (!prefix) return lagr_fail(msg, LAGR_OUT_OF_MEMORY, "tc work prefix");
    TRY(fill_i64(ctx, prefix + a.nrows, 1, 0, msg));
    hipLaunchKernelGGL(k_tc_row_work, dim3(grid_for(a.nrows, 256, 16384)), dim3(256), 0, ctx->stream,
                       a, prefix);
    LAUNCH_CHECK();
    TRY(scan_exclusive_i64(ctx, prefix, prefix, a.nrows + 1, nullptr, msg));
    // four resident waves per SIMD: the balanced partition needs no more
    const unsigned blocks = (unsigned)(ctx->num_cus * 4);
    if (per_entry)
        TIMED(ctx, "tc_rows_entries",
              hipLaunchKernelGGL(k_tc_rows<true>, dim3(blocks), dim3(TC_BLOCK), 0, ctx->stream, a,
                                 prefix, total_dev, entry_counts));
    else
        TIMED(ctx, "tc_rows",
              hipLaunchKernelGGL(k_tc_rows<false>, dim3(blocks), dim3(TC_BLOCK), 0, ctx->stream, a,
                                 prefix, total_dev, entry_counts));
    LAUNCH_CHECK();
    return LAGR_SUCCESS;
}

// ------------------------------------------------------------------- TC

static int tc_on_lower(lagr_ctx ctx, const lagr_graph G, int64_t *ntri, char *msg)
{
    const lagr_matrix L = G->L;
    const TcPlan *P = G->tcplan;
    // eight resident waves per SIMD (the LDS and register budgets of
    // k_tc_split allow it); the work counters follow the partials
    const unsigned blocks = (unsigned)(ctx->num_cus * 8);
    const size_t nctr = (size_t)TC_DYN_STRIDE * TC_DYN_PARTS;
    unsigned long long *tot = (unsigned long long *)ws_get(ctx, WS_TC, 8 * ((size_t)blocks + 1 + nctr));
    if (!tot) return lagr_fail(msg, LAGR_OUT_OF_MEMORY, "tc counter");
    if (P->nitems > 0) {
        unsigned long long *ctr = tot + 1 + blocks;
        TRY(fill_i64(ctx, (int64_t *)ctr, (int64_t)nctr, 0, msg));
        PlanArgs a{P->nitems, L->rowptr, L->colidx, P->iprefix, P->ent, P->item, P->item_row};
        TIMED(ctx, "tc_split",
              hipLaunchKernelGGL(k_tc_split, dim3(blocks), dim3(TC_BLOCK), 0, ctx->stream, a, tot + 1, ctr));
        LAUNCH_CHECK();
        hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, ctx->stream, tot + 1, (int64_t)blocks, tot);
        LAUNCH_CHECK();
    } else {
        TRY(fill_i64(ctx, (int64_t *)tot, 1, 0, msg));
    }
    unsigned long long h = 0;
    TRY(read_back(ctx, &h, tot, sizeof(h), msg));
    *ntri = (int64_t)h;
    return LAGR_SUCCESS;
}

extern "C" int lagr_tc_adv(int64_t *ntriangles, const lagr_graph G, lagr_ctx ctx, char *msg)
{
    if (!ntriangles || !G || !ctx) return lagr_fail(msg, LAGR_NULL_POINTER, "NULL argument");
    if (!G->L || !G->tcplan) return lagr_fail(msg, LAGR_PROPERTY_MISSING, "tc_lower property not computed");
    TRY(tc_on_lower(ctx, G, ntriangles, msg));
    return lagr_ok(msg);
}

extern "C" int lagr_tc(int64_t *ntriangles, lagr_graph G, lagr_ctx ctx, char *msg)
{
    if (!ntriangles || !G || !ctx) return lagr_fail(msg, LAGR_NULL_POINTER, "NULL argument");
    TRY(lagr_property_tc_lower(G, ctx, msg));
    return lagr_tc_adv(ntriangles, G, ctx, msg);
}
