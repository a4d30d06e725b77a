// Matrix build from tuples, strictly lower select, the graph object with
// its cached properties (Listing 1; Section V), and CheckGraph.
#include <new>

#include "internal.h"

namespace {

// Make a wave's LDS writes visible to the whole wave.
__device__ __forceinline__ void wave_barrier_lds()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Rows of at most this many entries are scanned by one thread; longer ones
// are cut into chunks that whole wavefronts take (see row_chunks).
constexpr int64_t LANE_ROW_MAX = 64;
constexpr int64_t ROW_CHUNK = 2048;

__global__ void k_build_keys(const int32_t *__restrict__ src, const int32_t *__restrict__ dst,
                             int64_t nedges, int64_t nrows, int64_t ncols, int cbits, int sym,
                             int drop, uint64_t *__restrict__ keys, unsigned *__restrict__ err)
{
    const uint64_t sent = (uint64_t)nrows << cbits;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nedges;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t u = src[e], v = dst[e];
        const bool ok = u >= 0 && u < nrows && v >= 0 && v < ncols &&
                        (!sym || (v < nrows && u < ncols));
        if (!ok) atomicOr(err, 1u);
        const bool dead = !ok || (drop && u == v);
        if (sym) {
            keys[2 * e] = dead ? sent : (((uint64_t)u << cbits) | (uint64_t)v);
            keys[2 * e + 1] = dead ? sent : (((uint64_t)v << cbits) | (uint64_t)u);
        } else {
            keys[e] = dead ? sent : (((uint64_t)u << cbits) | (uint64_t)v);
        }
    }
}

// flag[p] = 1 if sorted key p is the first copy of a live entry.
__global__ void k_unique_flags(const uint64_t *__restrict__ keys, int64_t n, uint64_t sent,
                               int64_t *__restrict__ flag)
{
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n;
         p += (int64_t)gridDim.x * blockDim.x)
        flag[p] = (keys[p] < sent && (p == 0 || keys[p] != keys[p - 1])) ? 1 : 0;
}

__global__ void k_compact_keys(const uint64_t *__restrict__ keys, int64_t n, uint64_t sent,
                               const int64_t *__restrict__ pos, uint64_t *__restrict__ out_keys,
                               int32_t *__restrict__ colidx, uint64_t cmask)
{
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n;
         p += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t k = keys[p];
        if (k < sent && (p == 0 || k != keys[p - 1])) {
            out_keys[pos[p]] = k;
            colidx[pos[p]] = (int32_t)(k & cmask);
        }
    }
}

__global__ void k_keys_to_cols(const uint64_t *__restrict__ keys, int64_t n, uint64_t cmask,
                               int32_t *__restrict__ colidx)
{
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n;
         p += (int64_t)gridDim.x * blockDim.x)
        colidx[p] = (int32_t)(keys[p] & cmask);
}

// ------------------------------------------------ strictly lower select

__global__ void k_count_lower(const int64_t *__restrict__ rp, const int32_t *__restrict__ ci,
                              int64_t n, int64_t *__restrict__ cnt)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        // columns are sorted: the lower part is a prefix of the row
        int64_t lo = rp[i], hi = rp[i + 1];
        while (lo < hi) {
            int64_t mid = (lo + hi) >> 1;
            if (ci[mid] < i) lo = mid + 1;
            else hi = mid;
        }
        cnt[i] = lo - rp[i];
    }
}

__global__ void k_copy_lower(const int64_t *__restrict__ rp, const int32_t *__restrict__ ci,
                             const void *__restrict__ va, int64_t n,
                             const int64_t *__restrict__ orp, int32_t *__restrict__ oci,
                             void *__restrict__ ova)
{
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / 64;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / 64;
    const unsigned lane = lane_id();
    for (int64_t i = wave; i < n; i += nw) {
        const int64_t len = orp[i + 1] - orp[i];
        for (int64_t t = lane; t < len; t += 64) {
            oci[orp[i] + t] = ci[rp[i] + t];
            if (va) ((uint64_t *)ova)[orp[i] + t] = ((const uint64_t *)va)[rp[i] + t];
        }
    }
}

// ------------------------------------------------------- CheckGraph

// One entry (i, p) of the check: in range, after its predecessor, on the
// diagonal, mirrored.
__device__ __forceinline__ void check_entry(const int64_t *rp, const int32_t *ci, int64_t nrows,
                                            int64_t ncols, int want_sym, int64_t i, int64_t a,
                                            int64_t p, unsigned &e, unsigned long long &diag)
{
    const int64_t j = ci[p];
    if (j < 0 || j >= ncols) {
        e |= 1u;
        return;
    }
    if (p > a && ci[p - 1] >= j) e |= 2u;
    if (j == i) diag++;
    if (want_sym) {
        if (j >= nrows) {
            e |= 4u;
            return;
        }
        int64_t lo = rp[j], hi = rp[j + 1];
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if (ci[mid] < i) lo = mid + 1;
            else hi = mid;
        }
        if (lo >= rp[j + 1] || ci[lo] != i) e |= 4u;
    }
}

// Rows of at most LANE_ROW_MAX entries: one thread each; longer rows are
// left to k_check_chunks.
__global__ void k_check(const int64_t *__restrict__ rp, const int32_t *__restrict__ ci,
                        int64_t nrows, int64_t ncols, int want_sym,
                        unsigned *__restrict__ err, unsigned long long *__restrict__ ndiag)
{
    unsigned long long diag = 0;
    unsigned e = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nrows;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t a = rp[i], b = rp[i + 1];
        if (b < a) {
            e |= 8u;
            continue;
        }
        if (b - a > LANE_ROW_MAX) continue;
        for (int64_t p = a; p < b; p++) check_entry(rp, ci, nrows, ncols, want_sym, i, a, p, e, diag);
    }
    if (e) atomicOr(err, e);
    if (diag) atomicAdd(ndiag, diag);
}

__global__ void k_check_chunks(const int64_t *__restrict__ rp, const int32_t *__restrict__ ci,
                               int64_t nrows, int64_t ncols, int want_sym, RowChunks ch,
                               unsigned *__restrict__ err, unsigned long long *__restrict__ ndiag)
{
    unsigned long long diag = 0;
    unsigned e = 0;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / 64;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / 64;
    const unsigned lane = lane_id();
    for (int64_t c = wave; c < ch.n; c += nw) {
        const int64_t i = ch.row[c];
        for (int64_t p = ch.beg[c] + lane; p < ch.end[c]; p += 64)
            check_entry(rp, ci, nrows, ncols, want_sym, i, rp[i], p, e, diag);
    }
    if (e) atomicOr(err, e);
    if (diag) atomicAdd(ndiag, diag);
}

// ---------------------------------------- degree order and relabel (TC)

// key of vertex v: (v << dbits) | (maxdeg - deg(v)), dbits a multiple of 8
// (the radix passes take whole 8-bit digits, which must not reach v).  A
// stable sort on the low dbits bits alone orders by descending degree and,
// since the keys start in ascending v, keeps ties in ascending id: two
// passes at 2^20 instead of five over (degree, id).  The vertex with new
// label p is order[p] >> dbits.
__global__ void k_order_keys(const int64_t *__restrict__ deg, int64_t n, int64_t maxdeg, int dbits,
                             uint64_t *__restrict__ keys)
{
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x)
        keys[v] = ((uint64_t)v << dbits) | (uint64_t)(maxdeg - deg[v]);
}

// inv[v] = the new label of vertex v; also clears the emit's row counters
// (cur, n of them) and the last slot of the lengths to be scanned (cnt_end).
__global__ void k_inverse_perm(const uint64_t *__restrict__ keys, int64_t n, int dbits, int32_t *__restrict__ inv,
                               unsigned long long *__restrict__ cur, int64_t *__restrict__ cnt_end)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) *cnt_end = 0;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n;
         p += (int64_t)gridDim.x * blockDim.x) {
        inv[keys[p] >> dbits] = (int32_t)p;
        cur[p] = 0ull;
    }
}

// rowA[e] = the row of entry e of L (the sorts and the plan read it).  A
// wave takes 64 consecutive rows and writes them one after the other, its
// lanes over the row's entries (coalesced stores; a lane per row would
// scatter every store).  The rows of L are short (at most a few thousand
// ids after the degree order), so no wave is left with a hub row.
__global__ void k_row_ids(const int64_t *__restrict__ rp, int64_t n, int32_t *__restrict__ rowA)
{
    const unsigned lane = lane_id();
    const int64_t step = (int64_t)gridDim.x * blockDim.x;
    for (int64_t r0 = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63u); r0 < n; r0 += step) {
        const int64_t r = r0 + lane;
        const int64_t mb = r < n ? rp[r] : 0, me = r < n ? rp[r + 1] : 0;
        // four 16-lane groups, each writing one row at a time: most rows
        // of L are shorter than 16 entries
        const int rows = (int)min((int64_t)64, n - r0);
        const unsigned g = lane >> 4, sub = lane & 15u;
        for (int k0 = 0; k0 < rows; k0 += 4) {
            const int k = k0 + (int)g;
            const int64_t b = __shfl(mb, k & 63, 64), e = __shfl(me, k & 63, 64);
            if (k < rows)
                for (int64_t p = b + sub; p < e; p += 16) rowA[p] = (int32_t)(r0 + k);
        }
    }
}

// wrow[w] = the row holding entry 64w of A (the first entry of window w).
// A wave takes 64 consecutive rows and writes, row after row, the windows
// that start in each, its lanes over them (a hub row starts many; a lane
// per row would write a hub's windows alone).
__global__ void k_window_rows(const int64_t *__restrict__ rp, int64_t n, int32_t *__restrict__ wrow)
{
    const unsigned lane = lane_id();
    const int64_t step = (int64_t)gridDim.x * blockDim.x;
    for (int64_t r0 = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63u); r0 < n; r0 += step) {
        const int64_t r = r0 + lane;
        const int64_t mb = r < n ? (rp[r] + 63) >> 6 : 0, me = r < n ? (rp[r + 1] + 63) >> 6 : 0;
        // a row that starts at most 4 windows writes them itself (nearly
        // every row); the wave writes the longer ones together
        if (me - mb <= 4)
            for (int64_t w = mb; w < me; w++) wrow[w] = (int32_t)r;
        uint64_t todo = __ballot(me - mb > 4);
        while (todo) {
            const int k = __ffsll((unsigned long long)todo) - 1;
            todo &= todo - 1;
            const int64_t wb = (int64_t)__shfl((long long)mb, k, 64), we = (int64_t)__shfl((long long)me, k, 64);
            for (int64_t w = wb + lane; w < we; w += 64) wrow[w] = (int32_t)(r0 + k);
        }
    }
}

// The strictly lower part of the relabelled A, written in A's own layout:
// the ids inv[v] < inv[u] of row u go, unsorted, to P[rpA[u] ..), and
// cur[u] (zero on entry) ends as their number, the length of row inv[u] of
// L.  Emitting into the space of the source row needs no counting pass
// first.  Waves take windows of 64 consecutive entries of A in turn (grid
// stride: the waves at work at once cover neighbouring windows), one lane
// per entry, and need no stored row id per entry: a lane finds its row
// from the window's first row (wrow) by a binary search, over shuffles, of
// the next 64 row ends held one per lane (again 64 rows on while a lane's
// entry lies past them, as after a run of empty rows).  The lanes of one
// row make one atomic.  An entry's id and its label depend on the window
// alone, and the labels of the 64 candidate rows are read with their ends,
// so a window waits for three round trips (first row and ids; row ends,
// row labels and id labels; the atomic) instead of five.  (Contiguous runs
// of windows per wave, each found by a search of the row offsets, took
// 343 us at 2^20 against 253 us.)
constexpr int EMIT_ILP = 2;   // windows per wavefront in flight

__global__ void k_emit_windows(const int32_t *__restrict__ wrow, const int32_t *__restrict__ ci,
                               const int64_t *__restrict__ rpA, int64_t n, const int32_t *__restrict__ inv,
                               int64_t nnz, unsigned long long *__restrict__ cur, int32_t *__restrict__ P)
{
    const unsigned lane = lane_id();
    const int64_t nwin = (nnz + 63) >> 6;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    // rows of the 64 after rc whose end is at or before e; sets u, ub and
    // the row's label ivu (from lab, the label of row rc + lane) of a lane
    // whose row is among them
    auto search = [&](int64_t rc, int64_t end, int64_t start0, int32_t lab, int64_t e, bool &need, int32_t &u,
                      int64_t &ub, int32_t &ivu) {
        int cntr = 0;
#pragma unroll
        for (int sft = 32; sft >= 1; sft >>= 1) {
            const int64_t y = (int64_t)__shfl((long long)end, cntr + sft - 1, 64);
            if (y <= e) cntr += sft;
        }
        const int64_t last = (int64_t)__shfl((long long)end, 63, 64);
        if (cntr == 63 && last <= e) cntr = 64;
        const int64_t prev = (int64_t)__shfl((long long)end, cntr > 0 ? cntr - 1 : 0, 64);
        const int32_t lr = __shfl(lab, cntr & 63, 64);
        if (need && cntr < 64) {
            u = (int32_t)(rc + cntr);
            ub = cntr > 0 ? prev : start0;
            ivu = lr;
            need = false;
        }
    };
    for (int64_t w0 = wave; w0 < nwin; w0 += EMIT_ILP * nwaves) {
        int64_t e[EMIT_ILP], rc[EMIT_ILP], ub[EMIT_ILP], end[EMIT_ILP], start0[EMIT_ILP];
        int32_t u[EMIT_ILP], cj[EMIT_ILP], iv[EMIT_ILP], ivu[EMIT_ILP], lab[EMIT_ILP];
        bool need[EMIT_ILP];
        // the windows' first rows and the entries' ids: both known from the
        // window alone
#pragma unroll
        for (int k = 0; k < EMIT_ILP; k++) {
            const int64_t w = w0 + k * nwaves;
            e[k] = (w << 6) + lane;
            u[k] = -1;
            ub[k] = 0;
            ivu[k] = 0;
            need[k] = w < nwin && e[k] < nnz;
            rc[k] = w < nwin ? wrow[w] : 0;
            cj[k] = need[k] ? ci[e[k]] : 0;
        }
        // then the next 64 row ends and their rows' labels, and the ids'
        // labels, together
#pragma unroll
        for (int k = 0; k < EMIT_ILP; k++) {
            const int64_t ri = rc[k] + 1 + lane;
            end[k] = ri <= n ? rpA[ri] : INT64_MAX;   // end of row rc + lane
            start0[k] = rc[k] < n ? rpA[rc[k]] : 0;
            lab[k] = rc[k] + lane < n ? inv[rc[k] + lane] : 0;
            iv[k] = need[k] ? inv[cj[k]] : 0;
        }
#pragma unroll
        for (int k = 0; k < EMIT_ILP; k++) {
            search(rc[k], end[k], start0[k], lab[k], e[k], need[k], u[k], ub[k], ivu[k]);
            rc[k] += 64;
            // a window that spans more than 64 rows searches on
            while (__ballot(need[k])) {
                const int64_t ri = rc[k] + 1 + lane;
                const int64_t en = ri <= n ? rpA[ri] : INT64_MAX;
                const int32_t lb = rc[k] + lane < n ? inv[rc[k] + lane] : 0;
                search(rc[k], en, rpA[rc[k]], lb, e[k], need[k], u[k], ub[k], ivu[k]);
                rc[k] += 64;
            }
        }
        bool take[EMIT_ILP];
#pragma unroll
        for (int k = 0; k < EMIT_ILP; k++) take[k] = u[k] >= 0 && iv[k] < ivu[k];
        WaveRun wr[EMIT_ILP];
        uint64_t t[EMIT_ILP];
        unsigned long long base[EMIT_ILP];
#pragma unroll
        for (int k = 0; k < EMIT_ILP; k++) {
            wr[k] = wave_run(u[k]);
            t[k] = __ballot(take[k]) & wr[k].run;
            base[k] = 0;
            if (lane == wr[k].head && t[k]) base[k] = atomicAdd(&cur[u[k]], (unsigned long long)__popcll(t[k]));
        }
#pragma unroll
        for (int k = 0; k < EMIT_ILP; k++) {
            base[k] = (unsigned long long)__shfl((long long)base[k], (int)wr[k].head, 64);
            if (take[k]) P[ub[k] + (int64_t)base[k] + __popcll(t[k] & wr[k].before)] = iv[k];
        }
    }
}

// cnt[inv[u]] = cur[u], the row lengths of L by new label, and
// cnt[n + inv[u]] = deg(u) - cur[u], the column lengths of L (A is
// symmetric without self-loops: u's neighbours above it in the order).
__global__ void k_lower_lengths(const unsigned long long *__restrict__ cur, const int32_t *__restrict__ inv,
                                const int64_t *__restrict__ rpA, int64_t n, int64_t *__restrict__ cnt,
                                unsigned long long *__restrict__ status)
{
    if (blockIdx.x == 0 && threadIdx.x < 8) status[threadIdx.x] = 0ull;   // the preparation's status words
    for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n;
         u += (int64_t)gridDim.x * blockDim.x) {
        const int64_t k = (int64_t)cur[u], r = inv[u];
        cnt[r] = k;
        cnt[n + r] = rpA[u + 1] - rpA[u] - k;
    }
}

// Rows of at most SORT_SHORT ids: each entry's place in its row of L is the
// number of smaller ids in the row (the ids of a row are distinct), read
// from the row's unsorted copy in P, at the offset in A of the row's vertex
// (order[r] >> oshift is the vertex with new label r).  One thread per entry
// of L; rowL, the row of every entry of L, is already written.
constexpr int64_t SORT_SHORT = 64;

__global__ void k_sort_short(const int32_t *__restrict__ rowL, const int64_t *__restrict__ Lrp,
                             const uint64_t *__restrict__ order, int oshift, const int64_t *__restrict__ rpA,
                             const int32_t *__restrict__ P, int64_t nnz, int32_t *__restrict__ Lci)
{
    for (int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; o < nnz;
         o += (int64_t)gridDim.x * blockDim.x) {
        const int32_t r = rowL[o];
        const int64_t b = Lrp[r], c = Lrp[r + 1] - b;
        if (c > SORT_SHORT) continue;   // k_sort_long
        const int32_t *src = P + rpA[order[r] >> oshift];
        const int32_t x = src[o - b];
        int rank = 0;
#pragma unroll 8
        for (int t = 0; t < (int)c; t++) rank += src[t] < x ? 1 : 0;
        Lci[b + rank] = x;
    }
}

// Rows of SORT_SHORT + 1 .. SORT_LONG ids (listed as records, below): one
// wave per row.  The row, padded with INT32_MAX to N = 64R ids (R a power
// of two), sits in registers as R chunks of 64 (id lane + 64k in register
// k of lane `lane`).  Each chunk is sorted by a bitonic network across the
// lanes (shuffles, no memory); then runs of 64, 128, ... are merged in
// pairs through the wave's LDS: an id's place in the merged run is its
// place in its own run plus the number of ids of the partner run below it
// (ids of the right run count equal ids as below, so the places form a
// permutation even among the pads), found by a binary search of the
// partner run.  This does O(N log^2 64 + N log^2 N / 2) work instead of
// O(len^2) compares for ranking.  Longer rows set *too_long and stay
// unsorted.
constexpr int SORT_MID = 512;
constexpr int SORT_LONG = (int)TC_SORT_LONG;

// Rows of L longer than min_len, listed as records rec[2c] = start of the
// row in L, rec[2c + 1] = (offset of its unsorted copy in P << 16) |
// min(length, 0xffff), so that the sort reads one 16-byte record per row
// instead of a chain of dependent loads: rows of at most mid_len ids in
// rec1[0 .. count[0]), longer ones in rec2[0 .. count[1]) (counts zero on
// entry), so that the launch for either class reads only its own rows.
// Each workgroup reserves its ranges with one atomic per class.
__global__ __launch_bounds__(256) void k_list_long_rows(const int64_t *__restrict__ Lrp, int64_t n, int64_t min_len,
                                                        int64_t mid_len, const uint64_t *__restrict__ order,
                                                        int oshift, const int64_t *__restrict__ rpA,
                                                        int64_t *__restrict__ rec1, int64_t *__restrict__ rec2,
                                                        unsigned long long *count)
{
    __shared__ unsigned long long sc[256];
    __shared__ unsigned long long base_s[2];
    const int64_t share = (n + gridDim.x - 1) / gridDim.x;
    const int64_t v0 = (int64_t)blockIdx.x * share, v1 = min(n, v0 + share);
    // per-thread counts of both classes, packed 32 bits each (n < 2^31)
    unsigned long long c = 0;
    for (int64_t v = v0 + threadIdx.x; v < v1; v += 256) {
        const int64_t len = Lrp[v + 1] - Lrp[v];
        c += len > mid_len ? (1ull << 32) : len > min_len ? 1ull : 0ull;
    }
    sc[threadIdx.x] = c;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
        const unsigned long long y = (int)threadIdx.x >= o ? sc[threadIdx.x - o] : 0ull;
        __syncthreads();
        sc[threadIdx.x] += y;
        __syncthreads();
    }
    if (threadIdx.x == 255) {
        const unsigned long long t1 = sc[255] & 0xffffffffull, t2 = sc[255] >> 32;
        base_s[0] = t1 ? atomicAdd(&count[0], t1) : 0;
        base_s[1] = t2 ? atomicAdd(&count[1], t2) : 0;
    }
    __syncthreads();
    const unsigned long long before = sc[threadIdx.x] - c;
    unsigned long long p1 = base_s[0] + (before & 0xffffffffull), p2 = base_s[1] + (before >> 32);
    for (int64_t v = v0 + threadIdx.x; v < v1; v += 256) {
        const int64_t b = Lrp[v], len = Lrp[v + 1] - b;
        if (len > min_len) {
            int64_t *rec = len > mid_len ? rec2 + 2 * p2++ : rec1 + 2 * p1++;
            rec[0] = b;
            rec[1] = (rpA[order[v] >> oshift] << 16) | (len < 0xffff ? len : 0xffff);
        }
    }
}

template <int R>
__device__ __forceinline__ void sort_row_wave(const int32_t *__restrict__ src, int len, int32_t *x,
                                              int32_t *__restrict__ out, unsigned lane)
{
    int32_t v[R];
#pragma unroll
    for (int k = 0; k < R; k++) {
        const int i = (int)lane + 64 * k;
        v[k] = i < len ? src[i] : INT32_MAX;
    }
    // bitonic sort of each chunk across the 64 lanes, ascending
#pragma unroll
    for (int size = 2; size <= 64; size <<= 1)
#pragma unroll
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            const bool keep_min = ((lane & (unsigned)size) == 0) == ((lane & (unsigned)stride) == 0);
#pragma unroll
            for (int k = 0; k < R; k++) {
                const int32_t y = __shfl_xor(v[k], stride, 64);
                v[k] = keep_min ? min(v[k], y) : max(v[k], y);
            }
        }
    // merge rounds: id lane + 64k lies in run 64k / L (lane < 64 <= L), so
    // the run, its partner and the side are known per register k; the R
    // binary searches advance together, one LDS read each per step
#pragma unroll
    for (int L = 64; L < 64 * R; L <<= 1) {
        if (L == 64) {
#pragma unroll
            for (int k = 0; k < R; k++) x[lane + 64 * k] = v[k];
        }
        wave_barrier_lds();
        int base[R];
#pragma unroll
        for (int k = 0; k < R; k++) base[k] = 0;
#pragma unroll
        for (int half = L >> 1; half >= 1; half >>= 1)
#pragma unroll
            for (int k = 0; k < R; k++) {
                const int run = 64 * k / L;
                const int32_t y = x[(run ^ 1) * L + base[k] + half - 1];
                if ((run & 1) ? y <= v[k] : y < v[k]) base[k] += half;
            }
        int pos[R];
#pragma unroll
        for (int k = 0; k < R; k++) {
            const int run = 64 * k / L;
            const int32_t y = x[(run ^ 1) * L + base[k]];
            const int below = base[k] + (((run & 1) ? y <= v[k] : y < v[k]) ? 1 : 0);
            pos[k] = (run & ~1) * L + ((int)lane + 64 * k - run * L) + below;
        }
        wave_barrier_lds();
#pragma unroll
        for (int k = 0; k < R; k++) x[pos[k]] = v[k];
        wave_barrier_lds();
#pragma unroll
        for (int k = 0; k < R; k++) v[k] = x[lane + 64 * k];
        if (2 * L == 64 * R) wave_barrier_lds();
    }
#pragma unroll
    for (int k = 0; k < R; k++) {
        const int i = (int)lane + 64 * k;
        if (i < len) out[i] = v[k];
    }
}

// The rows of one list (lengths up to HI), so that each launch takes only
// the LDS its rows need (HI ids per wave) and shorter rows keep many waves
// resident; the launch with HI = SORT_LONG flags the rows past it.
template <int HI>
__global__ __launch_bounds__(256) void k_sort_long(const longlong2 *__restrict__ rec,
                                                   const unsigned long long *__restrict__ count,
                                                   const int32_t *__restrict__ P, int32_t *__restrict__ Lci,
                                                   unsigned long long *__restrict__ too_long)
{
    __shared__ int32_t buf[4][HI];
    int32_t *x = buf[threadIdx.x / 64];
    const unsigned lane = lane_id();
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / 64;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / 64;
    const int64_t nrows = (int64_t)*count;
    longlong2 next = wave < nrows ? rec[wave] : make_longlong2(0, 0);
    for (int64_t c = wave; c < nrows; c += nw) {
        const longlong2 cur = next;
        if (c + nw < nrows) next = rec[c + nw];   // the next row's record, in flight meanwhile
        const int64_t b = cur.x;
        const int len = (int)(cur.y & 0xffff);
        if (len > HI) {   // left to the radix sort (status[1])
            if (HI == SORT_LONG && lane == 0) too_long[0] = 1ull;
            continue;
        }
        const int32_t *src = P + (cur.y >> 16);
        if (HI <= 512) {
            if (len <= 128) sort_row_wave<2>(src, len, x, Lci + b, lane);
            else if (len <= 256) sort_row_wave<4>(src, len, x, Lci + b, lane);
            else sort_row_wave<(HI >= 512 ? 8 : 4)>(src, len, x, Lci + b, lane);
        } else {
            if (len <= 1024) sort_row_wave<16>(src, len, x, Lci + b, lane);
            else sort_row_wave<(HI >= 2048 ? 32 : 16)>(src, len, x, Lci + b, lane);
        }
    }
}

// Rows longer than SORT_LONG: a (row, id) key for every entry of L, then a
// global radix sort.
__global__ void k_row_keys(const int32_t *__restrict__ rowL, const int64_t *__restrict__ Lrp,
                           const uint64_t *__restrict__ order, int oshift, const int64_t *__restrict__ rpA,
                           const int32_t *__restrict__ P, int64_t nnz, int vbits, uint64_t *__restrict__ keys)
{
    for (int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; o < nnz;
         o += (int64_t)gridDim.x * blockDim.x) {
        const int32_t r = rowL[o];
        const int32_t x = P[rpA[order[r] >> oshift] + (o - Lrp[r])];
        keys[o] = ((uint64_t)r << vbits) | (uint64_t)x;
    }
}

// L's row offsets, rp_out[0..n] = rp[0..n] (the first n+1 scanned lengths),
// and status[0] = the longest row of L (one atomic per workgroup); also
// clears the two long-row list counts (nlong).
__global__ __launch_bounds__(256) void k_row_max(const int64_t *__restrict__ rp, int64_t n,
                                                 int64_t *__restrict__ rp_out,
                                                 unsigned long long *__restrict__ status,
                                                 unsigned long long *__restrict__ nlong)
{
    __shared__ unsigned long long m_s;
    if (threadIdx.x == 0) m_s = 0;
    if (blockIdx.x == 0 && threadIdx.x < 2) nlong[threadIdx.x] = 0ull;
    __syncthreads();
    unsigned long long m = 0;
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r <= n; r += (int64_t)gridDim.x * blockDim.x) {
        const int64_t b = rp[r];
        rp_out[r] = b;
        if (r < n) {
            const unsigned long long len = (unsigned long long)(rp[r + 1] - b);
            m = len > m ? len : m;
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long y = __shfl_xor(m, o, 64);
        m = y > m ? y : m;
    }
    if (lane_id() == 0 && m) atomicMax(&m_s, m);
    __syncthreads();
    if (threadIdx.x == 0 && m_s) atomicMax(&status[0], m_s);
}

__global__ void k_keys_split(const uint64_t *__restrict__ keys, int64_t nnz, int vbits, uint64_t vmask,
                             int32_t *__restrict__ ci, int32_t *__restrict__ rowid)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz;
         e += (int64_t)gridDim.x * blockDim.x) {
        ci[e] = (int32_t)(keys[e] & vmask);
        rowid[e] = (int32_t)(keys[e] >> vbits);
    }
}

}  // namespace

// ------------------------------------------------------------------ API

extern "C" int lagr_matrix_build(lagr_matrix *A, int64_t nrows, int64_t ncols, int64_t nedges,
                                 const int32_t *src, const int32_t *dst, uint32_t flags,
                                 lagr_ctx ctx, char *msg)
{
    if (!A || !ctx) return lagr_fail(msg, LAGR_NULL_POINTER, "NULL argument");
    *A = nullptr;
    if (nrows < 0 || ncols < 0 || nrows >= INT32_MAX || ncols >= INT32_MAX || nedges < 0)
        return lagr_fail(msg, LAGR_INVALID_VALUE, "bad sizes");
    if (nedges > 0 && (!src || !dst)) return lagr_fail(msg, LAGR_NULL_POINTER, "edge arrays");
    const int sym = (flags & LAGR_BUILD_SYMMETRIZE) ? 1 : 0;
    const int drop = (flags & LAGR_BUILD_DROP_LOOPS) ? 1 : 0;
    if (sym && nrows != ncols)
        return lagr_fail(msg, LAGR_DIMENSION_MISMATCH, "symmetrize needs a square matrix");
    const int64_t nk = sym ? 2 * nedges : nedges;
    const int cbits = bits_for((uint64_t)(ncols > 0 ? ncols - 1 : 0));
    const int nbits = cbits + bits_for((uint64_t)nrows);
    const uint64_t sent = (uint64_t)nrows << cbits;

    lagr_matrix M = new (std::nothrow) lagr_matrix_s();
    if (!M) return lagr_fail(msg, LAGR_OUT_OF_MEMORY, "matrix");
    M->type = LAGR_BOOL;
    M->nrows = nrows;
    M->ncols = ncols;
    int rc = LAGR_SUCCESS;
    uint64_t *keys = (uint64_t *)ws_get(ctx, WS_KEYS, sizeof(uint64_t) * (nk > 0 ? nk : 1));
    int64_t *pos = (int64_t *)ws_get(ctx, WS_FLAGS, sizeof(int64_t) * (nk > 0 ? nk : 1));
    unsigned *err = (unsigned *)ws_get(ctx, WS_COUNTERS, 64);
    int64_t nnz = 0;
    unsigned herr = 0;
    if (!keys || !pos || !err) {
        delete M;
        return lagr_fail(msg, LAGR_OUT_OF_MEMORY, "build workspace");
    }
    HIP_TRY(hipMemsetAsync(err, 0, sizeof(unsigned), ctx->stream));
    if (nedges > 0) {
        hipLaunchKernelGGL(k_build_keys, dim3(grid_for(nedges, 256, 65536)), dim3(256), 0,
                           ctx->stream, src, dst, nedges, nrows, ncols, cbits, sym, drop, keys, err);
        LAUNCH_CHECK();
    }
    rc = read_back(ctx, &herr, err, sizeof(unsigned), msg);
    if (rc < 0 || herr) {
        delete M;
        return rc < 0 ? rc : lagr_fail(msg, LAGR_INVALID_INDEX, "edge endpoint out of range");
    }
    if ((rc = radix_sort_u64(ctx, keys, nk, nbits, msg)) < 0) goto fail;
    if (nk > 0) {
        hipLaunchKernelGGL(k_unique_flags, dim3(grid_for(nk, 256, 65536)), dim3(256), 0,
                           ctx->stream, keys, nk, sent, pos);
        LAUNCH_CHECK();
    }
    if ((rc = scan_exclusive_i64(ctx, pos, pos, nk, &nnz, msg)) < 0) goto fail;
    if ((rc = matrix_alloc(M, nnz, msg)) < 0) goto fail;
    {
        uint64_t *ukeys = (uint64_t *)ws_get(ctx, WS_SORT_TMP, sizeof(uint64_t) * (nnz > 0 ? nnz : 1));
        if (!ukeys) {
            rc = lagr_fail(msg, LAGR_OUT_OF_MEMORY, "build workspace");
            goto fail;
        }
        if (nk > 0) {
            hipLaunchKernelGGL(k_compact_keys, dim3(grid_for(nk, 256, 65536)), dim3(256), 0,
                               ctx->stream, keys, nk, sent, pos, ukeys, M->colidx,
                               (cbits ? ((1ull << cbits) - 1) : 0ull));
            LAUNCH_CHECK();
        }
        if ((rc = rowptr_from_sorted_keys(ctx, ukeys, nnz, cbits, nrows, M->rowptr, msg)) < 0)
            goto fail;
    }
    *A = M;
    return lagr_ok(msg);
fail:
    matrix_release_arrays(M);
    delete M;
    return rc;
}

extern "C" int lagr_select_tril(lagr_matrix *C, const lagr_matrix A, lagr_ctx ctx, char *msg)
{
    if (!C || !A || !ctx) return lagr_fail(msg, LAGR_NULL_POINTER, "NULL argument");
    *C = nullptr;
    const int64_t n = A->nrows;
    int64_t *cnt = (int64_t *)ws_get(ctx, WS_GEN_A, sizeof(int64_t) * (n + 1));
    if (!cnt) return lagr_fail(msg, LAGR_OUT_OF_MEMORY, "select workspace");
    if (n > 0) {
        hipLaunchKernelGGL(k_count_lower, dim3(grid_for(n, 256, 65536)), dim3(256), 0, ctx->stream,
                           A->rowptr, A->colidx, n, cnt);
        LAUNCH_CHECK();
    }
    TRY(fill_i64(ctx, cnt + n, 1, 0, msg));
    int64_t nnz = 0;
    TRY(scan_exclusive_i64(ctx, cnt, cnt, n + 1, &nnz, msg));
    lagr_matrix M = new (std::nothrow) lagr_matrix_s();
    if (!M) return lagr_fail(msg, LAGR_OUT_OF_MEMORY, "matrix");
    M->type = A->type;
    M->nrows = A->nrows;
    M->ncols = A->ncols;
    int rc = matrix_alloc(M, nnz, msg);
    if (rc < 0) {
        delete M;
        return rc;
    }
    HIP_TRY(hipMemcpyAsync(M->rowptr, cnt, sizeof(int64_t) * (n + 1), hipMemcpyDeviceToDevice,
                           ctx->stream));
    if (n > 0) {
        hipLaunchKernelGGL(k_copy_lower, dim3(grid_for(n * 64, 256, 16384)), dim3(256), 0,
                           ctx->stream, A->rowptr, A->colidx, A->values, n, M->rowptr, M->colidx,
                           M->values);
        LAUNCH_CHECK();
    }
    *C = M;
    return lagr_ok(msg);
}

// ----------------------------------------------------------------- graph

extern "C" int lagr_graph_new(lagr_graph *G, lagr_matrix *A, lagr_kind kind, lagr_ctx ctx,
                              char *msg)
{
    if (!G || !A || !*A || !ctx) return lagr_fail(msg, LAGR_NULL_POINTER, "NULL argument");
    *G = nullptr;
    if (kind != LAGR_ADJACENCY_UNDIRECTED && kind != LAGR_ADJACENCY_DIRECTED)
        return lagr_fail(msg, LAGR_INVALID_VALUE, "unknown graph kind");
    if ((*A)->nrows != (*A)->ncols)
        return lagr_fail(msg, LAGR_DIMENSION_MISMATCH, "adjacency matrix must be square");
    lagr_graph g = new (std::nothrow) lagr_graph_s();
    if (!g) return lagr_fail(msg, LAGR_OUT_OF_MEMORY, "graph");
    g->A = *A;
    g->kind = kind;
    *A = nullptr;
    *G = g;
    return lagr_ok(msg);
}

extern "C" int lagr_graph_check(lagr_graph G, lagr_ctx ctx, char *msg)
{
    if (!G || !ctx) return lagr_fail(msg, LAGR_NULL_POINTER, "NULL argument");
    lagr_matrix A = G->A;
    unsigned *err = (unsigned *)ws_get(ctx, WS_COUNTERS, 64);
    if (!err) return lagr_fail(msg, LAGR_OUT_OF_MEMORY, "counters");
    HIP_TRY(hipMemsetAsync(err, 0, 16, ctx->stream));
    unsigned long long *nd = (unsigned long long *)(err + 2);
    const int want_sym = G->kind == LAGR_ADJACENCY_UNDIRECTED;
    if (A->nrows > 0) {
        hipLaunchKernelGGL(k_check, dim3(grid_for(A->nrows, 256, 4096)), dim3(256), 0, ctx->stream,
                           A->rowptr, A->colidx, A->nrows, A->ncols, want_sym, err, nd);
        LAUNCH_CHECK();
        RowChunks ch;
        TRY(row_chunks(ctx, A->rowptr, A->nrows, LANE_ROW_MAX, ROW_CHUNK, WS_CHUNK_A, WS_CHUNK_B, &ch,
                       msg));
        if (ch.n > 0) {
            hipLaunchKernelGGL(k_check_chunks, dim3(grid_for(ch.n * 64, 256, 8192)), dim3(256), 0,
                               ctx->stream, A->rowptr, A->colidx, A->nrows, A->ncols, want_sym, ch,
                               err, nd);
            LAUNCH_CHECK();
        }
    }
    unsigned h[4] = {0, 0, 0, 0};
    TRY(read_back(ctx, h, err, 16, msg));
    unsigned long long hd;
    memcpy(&hd, &h[2], 8);
    if (h[0] & 8u) return lagr_fail(msg, LAGR_INVALID_OBJECT, "row offsets decrease");
    if (h[0] & 1u) return lagr_fail(msg, LAGR_INVALID_OBJECT, "column id out of range");
    if (h[0] & 2u) return lagr_fail(msg, LAGR_INVALID_OBJECT, "row not sorted or has duplicates");
    if (h[0] & 4u) return lagr_fail(msg, LAGR_INVALID_OBJECT, "undirected graph is not symmetric");
    G->ndiag = (int64_t)hd;
    if (want_sym) G->symmetric = 1;
    return lagr_ok(msg);
}

extern "C" int lagr_property_row_degree(lagr_graph G, lagr_ctx ctx, char *msg)
{
    if (!G || !ctx) return lagr_fail(msg, LAGR_NULL_POINTER, "NULL argument");
    if (G->row_degree) return lagr_ok(msg);
    const int64_t n = G->A->nrows;
    int64_t *deg = (int64_t *)dev_alloc(sizeof(int64_t) * (n > 0 ? n : 1));
    if (!deg) return lagr_fail(msg, LAGR_OUT_OF_MEMORY, "row degree");
    int64_t mx = 0, nbig = 0;
    int rc = row_degrees(ctx, G->A->rowptr, n, deg, &mx, msg, TC_SORT_LONG, &nbig);
    if (rc < 0) {
        dev_free(deg, sizeof(int64_t) * (n > 0 ? n : 1));
        return rc;
    }
    G->row_degree = deg;
    G->max_degree = mx;
    G->deg_over_sort = nbig;
    return lagr_ok(msg);
}

extern "C" int lagr_property_tc_lower(lagr_graph G, lagr_ctx ctx, char *msg)
{
    TRY(tc_lower_build(G, ctx, false, msg));
    return lagr_ok(msg);
}

int tc_lower_build(lagr_graph G, lagr_ctx ctx, bool defer, char *msg)
{
    if (!G || !ctx) return lagr_fail(msg, LAGR_NULL_POINTER, "NULL argument");
    if (G->L) return LAGR_SUCCESS;
    if (G->kind != LAGR_ADJACENCY_UNDIRECTED)
        return lagr_fail(msg, LAGR_INVALID_VALUE, "triangle counting needs an undirected graph");
    if (G->ndiag < 0 || G->symmetric < 0) TRY(lagr_graph_check(G, ctx, msg));
    if (G->ndiag != 0)
        return lagr_fail(msg, LAGR_INVALID_VALUE, "graph has %lld self-loops", (long long)G->ndiag);
    lagr_matrix A = G->A;
    const int64_t n = A->nrows;
    const int64_t nnzA = A->nvals;
    const int64_t nwin = (nnzA + 63) >> 6;
    int32_t *wrow = (int32_t *)ws_get(ctx, WS_GEN_D, sizeof(int32_t) * (nwin > 0 ? nwin : 1));
    if (!wrow) return lagr_fail(msg, LAGR_OUT_OF_MEMORY, "tc workspace");
    // the first row of every 64-entry window of A (step 2 below): it reads
    // A only, so it is queued before the degrees, whose largest value the
    // host reads back (the radix sort's digit count depends on it)
    if (nnzA > 0) {
        hipLaunchKernelGGL(k_window_rows, dim3(grid_for(n, 256, 8192)), dim3(256), 0, ctx->stream, A->rowptr, n,
                           wrow);
        LAUNCH_CHECK();
    }
    TRY(lagr_property_row_degree(G, ctx, msg));
    const int vbits = bits_for((uint64_t)(n > 0 ? n - 1 : 0));
    const uint64_t vmask = vbits ? ((1ull << vbits) - 1) : 0ull;

    // 1. descending-degree order, ties by id (Algorithm 6 sorts by degree;
    //    descending keeps the rows of L short for the row-by-row form)
    uint64_t *okeys = (uint64_t *)ws_get(ctx, WS_PERM, sizeof(uint64_t) * (n > 0 ? n : 1));
    int32_t *inv = (int32_t *)ws_get(ctx, WS_DEG, sizeof(int32_t) * (n > 0 ? n : 1));
    int64_t *cnt = (int64_t *)ws_get(ctx, WS_FLAGS, sizeof(int64_t) * (2 * n + 1));
    if (!okeys || !inv || !cnt) return lagr_fail(msg, LAGR_OUT_OF_MEMORY, "tc workspace");
    const int dbits = (bits_for((uint64_t)G->max_degree) + 7) / 8 * 8;
    if (n > 0) {
        hipLaunchKernelGGL(k_order_keys, dim3(grid_for(n, 256, 65536)), dim3(256), 0, ctx->stream,
                           G->row_degree, n, G->max_degree, dbits, okeys);
        LAUNCH_CHECK();
    }
    TRY(radix_sort_u64(ctx, okeys, n, dbits, msg));
    int32_t *P = (int32_t *)ws_get(ctx, WS_GEN_C, sizeof(int32_t) * (nnzA > 0 ? nnzA : 1));
    unsigned long long *cur = (unsigned long long *)ws_get(ctx, WS_GEN_B, sizeof(int64_t) * (n > 0 ? n : 1));
    unsigned long long *status = (unsigned long long *)ws_get(ctx, WS_COUNTERS, 64);
    if (!P || !cur || !status) return lagr_fail(msg, LAGR_OUT_OF_MEMORY, "tc workspace");
    // (with n = 0 the kernel still clears cnt[2n], the scan's only entry)
    hipLaunchKernelGGL(k_inverse_perm, dim3(grid_for(n, 256, 65536)), dim3(256), 0, ctx->stream, okeys, n, dbits,
                       inv, cur, cnt + 2 * n);
    LAUNCH_CHECK();
    if (nnzA > 0) {
        // 2. with the first row of every 64-entry window of A (above), the
        //    relabelled strictly lower part lands unsorted in A's layout,
        //    counting its row lengths
        hipLaunchKernelGGL(k_emit_windows, dim3(grid_for(nnzA, 256, 8192)), dim3(256), 0, ctx->stream, wrow,
                           A->colidx, A->rowptr, n, inv, nnzA, cur, P);
        LAUNCH_CHECK();
    }
    hipLaunchKernelGGL(k_lower_lengths, dim3(grid_for(n, 256, 8192)), dim3(256), 0, ctx->stream, cur, inv,
                       A->rowptr, n, cnt, status);
    LAUNCH_CHECK();
    // A is symmetric without self-loops (checked above), so L holds exactly
    // half of its entries: no host round trip for the count (checked
    // against the scan's total with the status read below).  One scan of
    // [row lengths | column lengths | 0] gives L's row offsets (its first
    // n+1 entries) and the regions of the count plan's 2n virtual rows.
    if (nnzA % 2 != 0) return lagr_fail(msg, LAGR_INVALID_OBJECT, "odd entry count in a symmetric matrix");
    const int64_t nnz = nnzA / 2;
    TRY(scan_exclusive_i64(ctx, cnt, cnt, 2 * n + 1, nullptr, msg));
    lagr_matrix L = new (std::nothrow) lagr_matrix_s();
    if (!L) return lagr_fail(msg, LAGR_OUT_OF_MEMORY, "matrix");
    L->type = LAGR_BOOL;
    L->nrows = n;
    L->ncols = n;
    int rc = matrix_alloc(L, nnz, msg);
    if (rc < 0) {
        delete L;
        return rc;
    }
    int32_t *rowid = (int32_t *)ws_get(ctx, WS_GEN_A, sizeof(int32_t) * (nnz > 0 ? nnz : 1));
    // two record lists of up to n rows each
    int64_t *lrows = (int64_t *)ws_get(ctx, WS_CHUNK_A, 4 * sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    unsigned long long *nlong = (unsigned long long *)ws_get(ctx, WS_CHUNK_B, 64);
    if (!rowid || !lrows || !nlong) {
        rc = lagr_fail(msg, LAGR_OUT_OF_MEMORY, "tc workspace");
        goto fail;
    }
    // 3. the rows are sorted from P into L: rows of at most SORT_SHORT ids
    //    by rank, rows up to SORT_LONG by a wave sort in registers and LDS (listed
    //    on the device), longer rows (flagged in status[1]) by a radix sort
    hipLaunchKernelGGL(k_row_max, dim3(grid_for(n + 1, 256, 256)), dim3(256), 0, ctx->stream, cnt, n, L->rowptr,
                       status, nlong);
    if (hipGetLastError() != hipSuccess) {
        rc = lagr_fail(msg, LAGR_DEVICE_ERROR, "row offsets launch failed");
        goto fail;
    }
    if (n > 0) {
        // the row of every entry of L (the plan reads it too)
        hipLaunchKernelGGL(k_row_ids, dim3(grid_for(n, 256, 8192)), dim3(256), 0, ctx->stream, L->rowptr, n,
                           rowid);
        if (nnz > 0)
            hipLaunchKernelGGL(k_sort_short, dim3(grid_for(nnz, 256, 65536)), dim3(256), 0, ctx->stream, rowid,
                               L->rowptr, okeys, dbits, A->rowptr, P, nnz, L->colidx);
        if (hipGetLastError() != hipSuccess) {
            rc = lagr_fail(msg, LAGR_DEVICE_ERROR, "row sort launch failed");
            goto fail;
        }
        hipLaunchKernelGGL(k_list_long_rows, dim3(grid_for(n, 256, 1024)), dim3(256), 0, ctx->stream, L->rowptr, n,
                           SORT_SHORT, SORT_MID, okeys, dbits, A->rowptr, lrows, lrows + 2 * n, nlong);
        hipLaunchKernelGGL(k_sort_long<SORT_MID>, dim3((unsigned)(ctx->num_cus * 16)), dim3(256), 0, ctx->stream,
                           (const longlong2 *)lrows, nlong, P, L->colidx, status + 1);
        hipLaunchKernelGGL(k_sort_long<SORT_LONG>, dim3((unsigned)(ctx->num_cus * 2)), dim3(256), 0, ctx->stream,
                           (const longlong2 *)(lrows + 2 * n), nlong + 1, P, L->colidx, status + 1);
        if (hipGetLastError() != hipSuccess) {
            rc = lagr_fail(msg, LAGR_DEVICE_ERROR, "row sort launch failed");
            goto fail;
        }
    }
    G->L = L;
    // A row of L holds neighbours of its vertex ranked before it, so at most
    // its degree.  Let C be the number of vertices with more than SORT_LONG
    // neighbours: a vertex with at most SORT_LONG neighbours has a row of at
    // most SORT_LONG ids, and one with more is ranked among the first C
    // (the order is by descending degree), so its row holds at most C - 1
    // ids.  With C <= SORT_LONG + 1 every row is therefore sorted in LDS,
    // and with the largest degree below the plan's length field every row
    // fits it: the plan's status can then wait for the count.
    if (defer && G->deg_over_sort >= 0 && G->deg_over_sort <= SORT_LONG + 1 && tc_plan_fits(G->max_degree)) {
        if ((rc = tc_plan_build(ctx, G, rowid, cnt, msg)) >= 0 && (rc = tc_plan_status(ctx, G, status, msg)) >= 0) {
            G->tc_status_pending = true;
            return LAGR_SUCCESS;
        }
        tc_plan_free(G);
        G->L = nullptr;
        G->L_maxrow = -1;
        goto fail;
    }
    for (int attempt = 0;; attempt++) {
        if ((rc = tc_plan_build(ctx, G, rowid, cnt, msg)) < 0) break;
        bool unsorted = false;
        if ((rc = tc_plan_settle(ctx, G, status, nnz, &unsorted, msg)) < 0) break;
        if (!unsorted || attempt > 0) break;
        // a row longer than SORT_LONG: sort every row with a global radix
        // sort of (row, id) keys and build the plan again
        tc_plan_free(G);
        uint64_t *keys = (uint64_t *)ws_get(ctx, WS_KEYS, sizeof(uint64_t) * nnz);
        if (!keys) {
            rc = lagr_fail(msg, LAGR_OUT_OF_MEMORY, "tc workspace");
            break;
        }
        hipLaunchKernelGGL(k_row_keys, dim3(grid_for(nnz, 256, 65536)), dim3(256), 0, ctx->stream, rowid,
                           L->rowptr, okeys, dbits, A->rowptr, P, nnz, vbits, keys);
        if (hipGetLastError() != hipSuccess) {
            rc = lagr_fail(msg, LAGR_DEVICE_ERROR, "row sort launch failed");
            break;
        }
        if ((rc = radix_sort_u64(ctx, keys, nnz, 2 * vbits, msg)) < 0) break;
        hipLaunchKernelGGL(k_keys_split, dim3(grid_for(nnz, 256, 65536)), dim3(256), 0, ctx->stream, keys, nnz,
                           vbits, vmask, L->colidx, rowid);
        if (hipGetLastError() != hipSuccess) {
            rc = lagr_fail(msg, LAGR_DEVICE_ERROR, "row sort launch failed");
            break;
        }
    }
    if (rc < 0) {
        tc_plan_free(G);
        G->L = nullptr;
        G->L_maxrow = -1;
        goto fail;
    }
    return LAGR_SUCCESS;
fail:
    matrix_release_arrays(L);
    delete L;
    return rc;
}

extern "C" int lagr_graph_matrix(lagr_matrix *A, const lagr_graph G, char *msg)
{
    if (!A || !G) return lagr_fail(msg, LAGR_NULL_POINTER, "NULL argument");
    *A = G->A;
    return lagr_ok(msg);
}

static int cached_chunks(ChunkCache &cc, const lagr_matrix M, lagr_ctx ctx, RowChunks *out, char *msg)
{
    if (cc.n < 0) {
        RowChunks tmp;
        TRY(row_chunks(ctx, M->rowptr, M->nrows, GRAPH_LONG_ROW, GRAPH_LONG_ROW, WS_CHUNK_A, WS_CHUNK_B, &tmp,
                       msg));
        const size_t nc = (size_t)(tmp.n > 0 ? tmp.n : 1);
        int32_t *row = (int32_t *)dev_alloc(nc * 4);
        int64_t *beg = (int64_t *)dev_alloc(nc * 8);
        int64_t *end = (int64_t *)dev_alloc(nc * 8);
        if (!row || !beg || !end) {
            dev_free(row, nc * 4);
            dev_free(beg, nc * 8);
            dev_free(end, nc * 8);
            return lagr_fail(msg, LAGR_OUT_OF_MEMORY, "chunk list");
        }
        if (tmp.n > 0) {
            HIP_TRY(hipMemcpyAsync(row, tmp.row, nc * 4, hipMemcpyDeviceToDevice, ctx->stream));
            HIP_TRY(hipMemcpyAsync(beg, tmp.beg, nc * 8, hipMemcpyDeviceToDevice, ctx->stream));
            HIP_TRY(hipMemcpyAsync(end, tmp.end, nc * 8, hipMemcpyDeviceToDevice, ctx->stream));
        }
        cc.row = row;
        cc.beg = beg;
        cc.end = end;
        cc.n = tmp.n;
    }
    out->n = cc.n;
    out->row = cc.row;
    out->beg = cc.beg;
    out->end = cc.end;
    return LAGR_SUCCESS;
}

static void free_chunks(ChunkCache &cc)
{
    if (cc.n >= 0) {
        const size_t nc = (size_t)(cc.n > 0 ? cc.n : 1);
        dev_free(cc.row, nc * 4);
        dev_free(cc.beg, nc * 8);
        dev_free(cc.end, nc * 8);
    }
    cc = ChunkCache();
}

int graph_chunks(lagr_graph G, lagr_ctx ctx, RowChunks *out, char *msg)
{
    return cached_chunks(G->chunks, G->A, ctx, out, msg);
}

int graph_chunks_in(lagr_graph G, lagr_ctx ctx, RowChunks *out, char *msg)
{
    if (G->kind != LAGR_ADJACENCY_DIRECTED) return graph_chunks(G, ctx, out, msg);
    if (!G->AT) return lagr_fail(msg, LAGR_PROPERTY_MISSING, "the transpose of a directed graph is missing");
    return cached_chunks(G->chunks_t, G->AT, ctx, out, msg);
}

int graph_ensure_at(lagr_graph G, lagr_ctx ctx, char *msg)
{
    if (G->kind != LAGR_ADJACENCY_DIRECTED || G->AT) return LAGR_SUCCESS;
    return matrix_transpose(ctx, G->A, &G->AT, msg);
}

extern "C" int lagr_property_at(lagr_graph G, lagr_ctx ctx, char *msg)
{
    if (!G || !ctx) return lagr_fail(msg, LAGR_NULL_POINTER, "NULL argument");
    TRY(graph_ensure_at(G, ctx, msg));
    return lagr_ok(msg);
}

extern "C" int lagr_graph_at(lagr_matrix *AT, const lagr_graph G, char *msg)
{
    if (!AT || !G) return lagr_fail(msg, LAGR_NULL_POINTER, "NULL argument");
    *AT = graph_in_edges(G);
    if (!*AT) return lagr_fail(msg, LAGR_PROPERTY_MISSING, "the transpose has not been computed");
    return lagr_ok(msg);
}

extern "C" int lagr_graph_tc_lower(lagr_matrix *L, const lagr_graph G, char *msg)
{
    if (!L || !G) return lagr_fail(msg, LAGR_NULL_POINTER, "NULL argument");
    *L = G->L;
    return lagr_ok(msg);
}

extern "C" int lagr_graph_delete_properties(lagr_graph G, lagr_ctx ctx, char *msg)
{
    if (!G || !ctx) return lagr_fail(msg, LAGR_NULL_POINTER, "NULL argument");
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    const int64_t n = G->A ? G->A->nrows : 0;
    if (G->row_degree) dev_free(G->row_degree, sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    G->row_degree = nullptr;
    G->max_degree = -1;
    G->deg_over_sort = -1;
    lagr_matrix_free(&G->L);
    tc_plan_free(G);
    G->L_maxrow = -1;
    G->tc_status_pending = false;
    lagr_matrix_free(&G->AT);
    free_chunks(G->chunks_t);
    // ndiag and the symmetry flag describe A, which a graph never changes:
    // the results of lagr_graph_check stay valid and are kept
    return lagr_ok(msg);
}

extern "C" int lagr_graph_set_tuning(lagr_graph G, int64_t tc_hubs, int32_t bfs_alpha, int32_t bfs_beta,
                                     lagr_ctx ctx, char *msg)
{
    if (!G || !ctx) return lagr_fail(msg, LAGR_NULL_POINTER, "NULL argument");
    if (tc_hubs < -1 || bfs_alpha == 0 || bfs_beta == 0 || bfs_alpha < -1 || bfs_beta < -1)
        return lagr_fail(msg, LAGR_INVALID_VALUE, "tuning values out of range");
    if (tc_hubs != G->tc_hubs) {
        // the count operand was planned for the old hub count: drop it
        HIP_TRY(hipStreamSynchronize(ctx->stream));
        lagr_matrix_free(&G->L);
        tc_plan_free(G);
        G->L_maxrow = -1;
        G->tc_status_pending = false;
        G->tc_hubs = tc_hubs;
    }
    if (bfs_alpha > 0) G->bfs_alpha = bfs_alpha;
    if (bfs_beta > 0) G->bfs_beta = bfs_beta;
    return lagr_ok(msg);
}

extern "C" int lagr_graph_get_tuning(int64_t *tc_hubs, int32_t *bfs_alpha, int32_t *bfs_beta, const lagr_graph G,
                                     char *msg)
{
    if (!G) return lagr_fail(msg, LAGR_NULL_POINTER, "NULL argument");
    if (tc_hubs) *tc_hubs = G->tc_hubs;
    if (bfs_alpha) *bfs_alpha = G->bfs_alpha;
    if (bfs_beta) *bfs_beta = G->bfs_beta;
    return lagr_ok(msg);
}

extern "C" int lagr_graph_ndiag(int64_t *ndiag, const lagr_graph G, char *msg)
{
    if (!ndiag || !G) return lagr_fail(msg, LAGR_NULL_POINTER, "NULL argument");
    *ndiag = G->ndiag;
    return lagr_ok(msg);
}

extern "C" int lagr_graph_free(lagr_graph *G)
{
    if (!G || !*G) return LAGR_SUCCESS;
    lagr_graph g = *G;
    const int64_t n = g->A ? g->A->nrows : 0;
    if (g->row_degree) dev_free(g->row_degree, sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    free_chunks(g->chunks);
    free_chunks(g->chunks_t);
    lagr_matrix_free(&g->A);
    lagr_matrix_free(&g->AT);
    lagr_matrix_free(&g->L);
    tc_plan_free(g);
    delete g;
    *G = nullptr;
    return LAGR_SUCCESS;
}
