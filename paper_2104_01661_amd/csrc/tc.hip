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

// The entries of rows [r0, r0 + 64) of L, flattened over the wave: f(i,
// p, start of row i, e) for entry e at position p of row i.  The row of an
// entry is found by a binary search over the 64 row starts held one per
// lane.  Every lane runs the same trip count (the shuffles need the whole
// wave); lanes past the end pass valid = false.
template <class F>
__device__ __forceinline__ void plan_walk_rows(const int64_t *__restrict__ rp, int64_t n, int64_t r0,
                                               unsigned lane, F f)
{
    const int64_t rl = r0 + lane;
    const int64_t st = rp[rl < n ? rl : n];
    const int64_t first = bcast64(st, 0);
    const int64_t last = rp[r0 + 64 < n ? r0 + 64 : n];
    for (int64_t base = first; base < last; base += 64) {
        const int64_t e = base + lane;
        int t = 0;
#pragma unroll
        for (int b = 32; b > 0; b >>= 1) {
            const int c = t + b;
            const int lo = __shfl((int)(st & 0xffffffff), c, 64);
            const int hi = __shfl((int)(st >> 32), c, 64);
            const int64_t sc = (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
            if (sc <= e) t = c;
        }
        const int lo = __shfl((int)(st & 0xffffffff), t, 64);
        const int hi = __shfl((int)(st >> 32), t, 64);
        const int64_t si = (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
        if (e < last) f(r0 + t, e - si, si, e);
    }
}

// B-side rows j below PLAN_HOT (the highest-degree vertices after the
// relabel) receive most B entries; a workgroup first gathers their counts
// in LDS, so each takes one global atomic per workgroup instead of one per
// entry (same-address atomics serialise).  A workgroup owns PLAN_ROWS
// consecutive rows of L, 64 per wavefront.
constexpr int PLAN_HOT = 8192;
constexpr int PLAN_ROWS = 256;

// Entries per virtual row (cnt: 2n+1 entries, zero on entry).
__global__ __launch_bounds__(PLAN_ROWS) void k_plan_count(const int64_t *__restrict__ rp,
                                                          const int32_t *__restrict__ ci, int64_t n,
                                                          unsigned long long *__restrict__ cnt)
{
    __shared__ unsigned hot[PLAN_HOT];
    for (int x = threadIdx.x; x < PLAN_HOT; x += PLAN_ROWS) hot[x] = 0u;
    __syncthreads();
    const int64_t r0 = (int64_t)blockIdx.x * PLAN_ROWS + (threadIdx.x / 64) * 64;
    if (r0 < n)
        plan_walk_rows(rp, n, r0, lane_id(), [&](int64_t i, int64_t p, int64_t, int64_t e) {
            if (p == 0) return;
            const int32_t j = ci[e];
            const int64_t lj = rp[j + 1] - rp[j];
            if (lj == 0) return;
            if (lj <= p) atomicAdd(&cnt[i], 1ull);
            else if (j < PLAN_HOT) atomicAdd(&hot[j], 1u);
            else atomicAdd(&cnt[n + j], 1ull);
        });
    __syncthreads();
    for (int x = threadIdx.x; x < PLAN_HOT && x < n; x += PLAN_ROWS)
        if (hot[x]) atomicAdd(&cnt[n + x], (unsigned long long)hot[x]);
}

// cur (a copy of the first 2n offsets) holds the write cursor of each
// virtual row; the order of the entries within a row is immaterial.  Hot
// B rows reserve one range per workgroup and hand out positions from LDS
// as offsets from bstart, the first B-side offset (the host checks that
// the B side spans fewer than 2^32 entries).
__global__ __launch_bounds__(PLAN_ROWS) void k_plan_fill(const int64_t *__restrict__ rp,
                                                         const int32_t *__restrict__ ci, int64_t n,
                                                         int64_t bstart, unsigned long long *__restrict__ cur,
                                                         uint64_t *__restrict__ ent)
{
    __shared__ unsigned hot[PLAN_HOT];
    for (int x = threadIdx.x; x < PLAN_HOT; x += PLAN_ROWS) hot[x] = 0u;
    __syncthreads();
    const int64_t r0 = (int64_t)blockIdx.x * PLAN_ROWS + (threadIdx.x / 64) * 64;
    const unsigned lane = lane_id();
    if (r0 < n)
        plan_walk_rows(rp, n, r0, lane, [&](int64_t, int64_t p, int64_t, int64_t e) {
            if (p == 0) return;
            const int32_t j = ci[e];
            if (j >= PLAN_HOT) return;
            const int64_t lj = rp[j + 1] - rp[j];
            if (lj > p) atomicAdd(&hot[j], 1u);
        });
    __syncthreads();
    for (int x = threadIdx.x; x < PLAN_HOT && x < n; x += PLAN_ROWS)
        if (hot[x]) hot[x] = (unsigned)((int64_t)atomicAdd(&cur[n + x], (unsigned long long)hot[x]) - bstart);
    __syncthreads();
    if (r0 < n)
        plan_walk_rows(rp, n, r0, lane, [&](int64_t i, int64_t p, int64_t si, int64_t e) {
            if (p == 0) return;
            const int32_t j = ci[e];
            const int64_t sj = rp[j], lj = rp[j + 1] - sj;
            if (lj == 0) return;
            if (lj <= p) ent[atomicAdd(&cur[i], 1ull)] = plan_pack(sj, lj);
            else if (j < PLAN_HOT) ent[bstart + atomicAdd(&hot[j], 1u)] = plan_pack(si, p);
            else ent[atomicAdd(&cur[n + j], 1ull)] = plan_pack(si, p);
        });
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

struct PlanArgs {
    int64_t nitems;
    const int64_t *Lrp;
    const int32_t *Lci;
    const int64_t *iprefix;
    const uint64_t *ent;
    const uint64_t *item;
    const int32_t *item_row;
};

// Each workgroup writes its count to partial[blockIdx.x]; k_sum_partials
// adds them (atomics on one address from every wavefront would serialise).
__global__ __launch_bounds__(TC_BLOCK, 8) void k_tc_split(PlanArgs a, unsigned long long *__restrict__ partial)
{
    __shared__ TcWaveLds lds[TC_WAVES];
    TcWaveLds &L = lds[threadIdx.x / 64];
    const unsigned lane = lane_id();
    const int64_t w = (int64_t)blockIdx.x * TC_WAVES + threadIdx.x / 64;
    const int64_t nw = (int64_t)gridDim.x * TC_WAVES;
    for (int x = lane; x < TC_BM_WORDS; x += 64) L.bm[x] = 0u;
    wave_sync();
    const int64_t T = a.iprefix[a.nitems];
    const int64_t lo = (int64_t)((__int128)T * w / nw), hi = (int64_t)((__int128)T * (w + 1) / nw);
    const int64_t k0 = tc_lower_bound(a.iprefix, a.nitems, lo);
    const int64_t k1 = tc_lower_bound(a.iprefix, a.nitems, hi);
    const uint64_t lmask = (1ull << TC_PLAN_LEN_BITS) - 1;
    unsigned long long acc = 0;
    int32_t marked = -1, first_id = -1;
    int64_t alen = 0;
    const int32_t *Arow = nullptr;
    bool use_hash = false;
    for (int64_t k = k0; k < k1; k++) {
        const uint64_t it = a.item[k];
        const int32_t m = a.item_row[k];
        const int64_t e0 = (int64_t)(it >> TC_PLAN_CNT_BITS);
        const int cnt = (int)(it & ((1u << TC_PLAN_CNT_BITS) - 1));
        int64_t s = 0;
        int len = 0;
        if ((int)lane < cnt) {
            const uint64_t x = a.ent[e0 + lane];
            s = (int64_t)(x >> TC_PLAN_LEN_BITS);
            len = (int)(x & lmask);
        }
        if (m != marked) {
            if (marked >= 0) tc_unmark_kept(L, first_id, alen, lane);
            Arow = a.Lci + a.Lrp[m];
            alen = a.Lrp[m + 1] - a.Lrp[m];
            use_hash = tc_mark(L, Arow, alen, lane, &first_id);
            marked = m;
        }
        acc += tc_stream_flat(L, use_hash, Arow, alen, a.Lci, s, len, cnt, lane);
    }
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    __shared__ unsigned long long wsum[TC_WAVES];
    if (lane == 0) wsum[threadIdx.x / 64] = acc;
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

int tc_plan_build(lagr_ctx ctx, lagr_graph G, char *msg)
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
    const unsigned wgrid = (unsigned)((n + PLAN_ROWS - 1) / PLAN_ROWS);
    if (n > 0) {
        hipLaunchKernelGGL(k_plan_count, dim3(wgrid), dim3(PLAN_ROWS), 0, ctx->stream, Lm->rowptr, Lm->colidx, n,
                           (unsigned long long *)P->trp);
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
        hipLaunchKernelGGL(k_plan_fill, dim3(wgrid), dim3(PLAN_ROWS), 0, ctx->stream, Lm->rowptr, Lm->colidx, n,
                           bstart, cur, P->ent);
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
    // k_tc_split allow it): the static partition assumes all resident
    const unsigned blocks = (unsigned)(ctx->num_cus * 8);
    unsigned long long *tot = (unsigned long long *)ws_get(ctx, WS_TC, 8 * ((size_t)blocks + 1));
    if (!tot) return lagr_fail(msg, LAGR_OUT_OF_MEMORY, "tc counter");
    if (P->nitems > 0) {
        PlanArgs a{P->nitems, L->rowptr, L->colidx, P->iprefix, P->ent, P->item, P->item_row};
        TIMED(ctx, "tc_split",
              hipLaunchKernelGGL(k_tc_split, dim3(blocks), dim3(TC_BLOCK), 0, ctx->stream, a, tot + 1));
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
