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
        for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
        if (lane_id() == 0 && acc) atomicAdd(total, acc);
    }
}

}  // namespace

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
    unsigned long long *tot = (unsigned long long *)ws_get(ctx, WS_TC, 64);
    if (!tot) return lagr_fail(msg, LAGR_OUT_OF_MEMORY, "tc counter");
    TcArgs a;
    a.nrows = L->nrows;
    a.Mrp = a.Arp = a.Brp = L->rowptr;
    a.Mci = a.Aci = a.Bci = L->colidx;
    a.tc_form = 1;
    TRY(tc_masked_dot(ctx, a, false, tot, nullptr, msg));
    unsigned long long h = 0;
    TRY(read_back(ctx, &h, tot, sizeof(h), msg));
    *ntri = (int64_t)h;
    return LAGR_SUCCESS;
}

extern "C" int lagr_tc_adv(int64_t *ntriangles, const lagr_graph G, lagr_ctx ctx, char *msg)
{
    if (!ntriangles || !G || !ctx) return lagr_fail(msg, LAGR_NULL_POINTER, "NULL argument");
    if (!G->L) return lagr_fail(msg, LAGR_PROPERTY_MISSING, "tc_lower property not computed");
    TRY(tc_on_lower(ctx, G, ntriangles, msg));
    return lagr_ok(msg);
}

extern "C" int lagr_tc(int64_t *ntriangles, lagr_graph G, lagr_ctx ctx, char *msg)
{
    if (!ntriangles || !G || !ctx) return lagr_fail(msg, LAGR_NULL_POINTER, "NULL argument");
    TRY(lagr_property_tc_lower(G, ctx, msg));
    return lagr_tc_adv(ntriangles, G, ctx, msg);
}
