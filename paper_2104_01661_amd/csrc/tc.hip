// Masked plus.pair dot product and its fusion with reduce: triangle
// counting (Section IV-E, Algorithm 6) as C<s(L)> = L plus.pair L^T and
// t = sum(C), computed without forming C (the fusion Section VI-B asks
// for).
//
// General form: for every mask entry (i, j) in M, C(i,j) = |A_i and B_j|,
// the number of column ids the two sorted rows share (B_j is row j of B,
// i.e. column j of B^T, so this is A plus.pair B^T under the mask).
//
// Device design (gfx950): one wavefront per row i.  The wave hashes A_i
// into a private open-addressing table in LDS, then streams the rows B_j of
// the mask row's column ids j as one flattened sequence: each of the 64
// lanes takes one position, finds its segment j by a binary search over
// the chunk's segment offsets (held in LDS), loads one column id with a
// coalesced read and probes the table.  Rows whose A_i is too long for the
// table go to a block-per-row kernel that binary-searches A_i in memory.
#include "internal.h"
#include "tc_device.h"

namespace {

template <bool PER_ENTRY>
__global__ __launch_bounds__(TC_BLOCK) void k_tc_rows(TcArgs a, unsigned long long *__restrict__ total,
                                                      int64_t *__restrict__ entry_counts)
{
    __shared__ TcWaveLds lds[TC_WAVES];
    const unsigned wave = threadIdx.x / 64;
    const int64_t gw = (int64_t)blockIdx.x * TC_WAVES + wave;
    const int64_t nw = (int64_t)gridDim.x * TC_WAVES;
    unsigned long long acc = 0;
    for (int64_t i = gw; i < a.nrows; i += nw)
        acc += tc_row<PER_ENTRY>(a, i, lds[wave], entry_counts);
    if (!PER_ENTRY) {
        for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
        if (lane_id() == 0 && acc) atomicAdd(total, acc);
    }
}

template <bool PER_ENTRY>
__global__ __launch_bounds__(256) void k_tc_bigrows(TcArgs a, unsigned long long *__restrict__ total,
                                                    int64_t *__restrict__ entry_counts)
{
    __shared__ unsigned long long part[4];
    unsigned long long acc = 0;
    for (int64_t i = blockIdx.x; i < a.nrows; i += gridDim.x) {
        const int64_t a0 = a.Arp[i], alen = a.Arp[i + 1] - a0;
        if (alen <= TC_HASH_MAX_ROW) continue;
        for (int64_t q = a.Mrp[i]; q < a.Mrp[i + 1]; q++) {
            const int32_t j = a.Mci[q];
            const int64_t b0 = a.Brp[j], b1 = a.Brp[j + 1];
            unsigned long long c = 0;
            for (int64_t p = b0 + threadIdx.x; p < b1; p += blockDim.x) {
                const int32_t k = a.Bci[p];
                int64_t lo = a0, hi = a0 + alen;
                while (lo < hi) {
                    int64_t mid = (lo + hi) >> 1;
                    if (a.Aci[mid] < k) lo = mid + 1;
                    else hi = mid;
                }
                c += (lo < a0 + alen && a.Aci[lo] == k) ? 1 : 0;
            }
            for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
            if (PER_ENTRY) {
                if (lane_id() == 0) part[threadIdx.x / 64] = c;
                __syncthreads();
                if (threadIdx.x == 0) entry_counts[q] = (int64_t)(part[0] + part[1] + part[2] + part[3]);
                __syncthreads();
            } else {
                acc += c;
            }
        }
    }
    if (!PER_ENTRY && lane_id() == 0 && acc) atomicAdd(total, acc);
}

}  // namespace

int tc_masked_dot(lagr_ctx ctx, const TcArgs &a, int64_t max_arow, bool per_entry,
                  unsigned long long *total_dev, int64_t *entry_counts, char *msg)
{
    if (a.nrows <= 0) return LAGR_SUCCESS;
    // enough waves to fill 256 CUs several times over, each striding rows
    const int64_t blocks = grid_for(a.nrows, TC_WAVES, 2048L * 8);
    if (per_entry)
        TIMED(ctx, "tc_rows_entries",
              hipLaunchKernelGGL(k_tc_rows<true>, dim3((unsigned)blocks), dim3(TC_BLOCK), 0,
                                 ctx->stream, a, total_dev, entry_counts));
    else
        TIMED(ctx, "tc_rows",
              hipLaunchKernelGGL(k_tc_rows<false>, dim3((unsigned)blocks), dim3(TC_BLOCK), 0,
                                 ctx->stream, a, total_dev, entry_counts));
    LAUNCH_CHECK();
    if (max_arow > TC_HASH_MAX_ROW) {
        const unsigned g = grid_for(a.nrows, 1, 4096);
        if (per_entry)
            hipLaunchKernelGGL(k_tc_bigrows<true>, dim3(g), dim3(256), 0, ctx->stream, a, total_dev,
                               entry_counts);
        else
            hipLaunchKernelGGL(k_tc_bigrows<false>, dim3(g), dim3(256), 0, ctx->stream, a, total_dev,
                               entry_counts);
        LAUNCH_CHECK();
    }
    return LAGR_SUCCESS;
}

// ------------------------------------------------------------------- TC

static int tc_on_lower(lagr_ctx ctx, lagr_matrix L, int64_t maxrow, int64_t *ntri, char *msg)
{
    unsigned long long *tot = (unsigned long long *)ws_get(ctx, WS_TC, 64);
    if (!tot) return lagr_fail(msg, LAGR_OUT_OF_MEMORY, "tc counter");
    TRY(fill_i64(ctx, (int64_t *)tot, 1, 0, msg));
    TcArgs a;
    a.nrows = L->nrows;
    a.Mrp = a.Arp = a.Brp = L->rowptr;
    a.Mci = a.Aci = a.Bci = L->colidx;
    a.skip_short = 1;
    TRY(tc_masked_dot(ctx, a, maxrow, false, tot, nullptr, msg));
    unsigned long long h = 0;
    TRY(read_back(ctx, &h, tot, sizeof(h), msg));
    *ntri = (int64_t)h;
    return LAGR_SUCCESS;
}

extern "C" int lagr_tc_adv(int64_t *ntriangles, const lagr_graph G, lagr_ctx ctx, char *msg)
{
    if (!ntriangles || !G || !ctx) return lagr_fail(msg, LAGR_NULL_POINTER, "NULL argument");
    if (!G->L) return lagr_fail(msg, LAGR_PROPERTY_MISSING, "tc_lower property not computed");
    TRY(tc_on_lower(ctx, G->L, G->L_maxrow, ntriangles, msg));
    return lagr_ok(msg);
}

extern "C" int lagr_tc(int64_t *ntriangles, lagr_graph G, lagr_ctx ctx, char *msg)
{
    if (!ntriangles || !G || !ctx) return lagr_fail(msg, LAGR_NULL_POINTER, "NULL argument");
    TRY(lagr_property_tc_lower(G, ctx, msg));
    return lagr_tc_adv(ntriangles, G, ctx, msg);
}
