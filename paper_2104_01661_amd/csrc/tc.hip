// Masked plus.pair dot product and its fusion with reduce: triangle
// counting (Section IV-E, Algorithm 6) as C<s(L)> = L plus.pair L^T and
// t = sum(C), computed without forming C (the fusion Section VI-B asks
// for).  The row kernel is described in tc_device.h.
#include <algorithm>
#include <chrono>
#include <mutex>

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

// Every virtual row has a region of the entry array whose size is known
// before the plan is built: A-side row i at most len(L_i) entries (the
// region of row i in L's own layout) and B-side row j at most the number
// of rows of L holding j (the column length of L, from A's degrees), so
// the fill needs no counting pass: each row hands out slots from a cursor
// that starts at its region's start, and the cursor's end is the row's
// entry count.
//
// B-side rows j below PLAN_HOT (the highest-degree vertices after the
// relabel) receive most B entries, and atomics on one address serialise,
// so their slots are taken in two steps.  k_plan_hot counts, per
// workgroup, the B entries of each hot row in LDS and reserves them with
// one global atomic per (workgroup, row); it needs the row length of L
// only for hot columns (held in LDS), so it reads just the entry's row,
// column and row start.  k_plan_fill, run on the same partition of the
// entries (workgroup g takes the g-th contiguous share), hands out the
// reserved slots from LDS.  The fill chains dependent loads (row, row
// start, column, column's row), so it runs 512-thread workgroups, four per
// CU, for more loads in flight.
constexpr int PLAN_HOT = 4096;
constexpr int PLAN_BLOCK = 512;
constexpr unsigned PLAN_GRID = 1024;

// The plan's set-up, in one pass over the virtual rows r <= 2n:
//  * rowpk[r] = plan_pack(start of row r, length of row r) for r < n: one
//    gather gives both (the plan kernels gather it for the row and for the
//    column of every entry, at random columns);
//  * trp = the regions (2n + 1 starts), and cur, the rows' write cursors,
//    = their first 2n;
//  * bw (n + 1 bitmap word counts, raised by k_plan_hot) = 0, and the
//    bitmap row list's count *nbrows = 0;
//  * hubw[x] (x < nh) = the words of hub row x's bitmap up to its largest
//    id (0 for an empty row): what a hub pair reading L_x as bits costs.
__global__ void k_row_pack(const int64_t *__restrict__ rp, const int32_t *__restrict__ Lci, int64_t n,
                           uint64_t *__restrict__ rowpk, const int64_t *__restrict__ regions,
                           int64_t *__restrict__ trp, unsigned long long *__restrict__ cur,
                           int64_t *__restrict__ bw, unsigned long long *__restrict__ nbrows, int64_t nh,
                           unsigned *__restrict__ hubw)
{
    const int64_t nv = 2 * n;
    if (blockIdx.x == 0 && threadIdx.x == 0) *nbrows = 0ull;
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r <= nv;
         r += (int64_t)gridDim.x * blockDim.x) {
        const int64_t g = regions[r];
        trp[r] = g;
        if (r < nv) cur[r] = (unsigned long long)g;
        if (r <= n) bw[r] = 0;
        if (r < n) {
            const int64_t b = rp[r], e = rp[r + 1];
            rowpk[r] = plan_pack(b, e - b);
            if (r < nh) hubw[r] = e > b ? (unsigned)((Lci[e - 1] >> 5) + 1) : 0u;
        }
    }
}

// The hub columns: j < plan_hubs(n), a 1/256 share of the vertices (the
// highest-degree ones after the relabel) and at most PLAN_HOT, in graphs
// of 2^18 vertices or more.  Keeping hub pairs in row i trades count time
// for a smaller transpose; that pays where the hub columns' B rows are
// large (at 2^20: 44 us less in all), not in small graphs (a batch of
// 2,000 graphs of 2^8 to 2^16 vertices, whose preparation is not in its
// count, counted 25% slower with hubs).
static inline int64_t plan_hubs(int64_t n)
{
    if (n < ((int64_t)1 << 18)) return 0;
    const int64_t h = n >> 8;
    return h < PLAN_HOT ? h : PLAN_HOT;
}

// A hub pair (column j < plan_hubs(n)) goes to B row j only when p is below
// both len(L_j) and L_j's bitmap words; otherwise row i reads L_j's ids or
// bitmap, whichever is shorter.
__host__ __device__ __forceinline__ bool plan_hub_b(int64_t p, int64_t lj, int64_t words)
{
    return p < lj && p < words;
}

// Any other pair goes to B row j when L_j is longer than the prefix
// L_i[0, p), and in a graph with hub columns only when L_j is more than
// twice as long: there a pair whose sides are closer streams L_j from row
// i, at most p more ids, and spares the fill a cursor atomic and a
// scattered write in B row j (at 2^20: 1.0 million of the 6.1 million such
// pairs, 14 million more ids and bitmap words read, the whole count 1.5%
// faster; in graphs of 2^16 vertices or fewer the extra ids cost more than
// the fill saves).
__host__ __device__ __forceinline__ bool plan_cold_b(int64_t p, int64_t lj, int64_t nhub)
{
    return nhub > 0 ? lj > 2 * p : lj > p;
}

// One pass over the entries of L, on the fill's partition (workgroup g
// takes the g-th contiguous share):
//  * per workgroup, the B entries of each hot row, reserved in the row's
//    region: boff[g * PLAN_HOT + x] = offset of workgroup g's first slot in
//    row n + x, relative to bstart = trp[n] (fewer than 2^32 entries);
//  * bw[i] = the bitmap words row i needs (0 for none; zero on entry):
//    ceil(j / 32) for its largest id j that tc_bitmap_pair accepts at its
//    position (row i streamed by a B pair), and all of the row: for a hub
//    row every word up to its largest id, else tc_full_words(last id,
//    length) when that is worth reading instead of the row's ids (row i
//    streamed whole by an A pair).  The lanes of one row take their maximum
//    within the wave (the words grow with the id along the row, so the
//    last lane that asks for any holds it) and the run head makes the
//    row's one atomic.
// Waves step whole (wave_run needs every lane).
__global__ __launch_bounds__(PLAN_BLOCK) void k_plan_hot(const int32_t *__restrict__ rowid,
                                                         const int32_t *__restrict__ ci, int64_t nnz,
                                                         const uint64_t *__restrict__ rowpk,
                                                         const unsigned *__restrict__ hubw, int64_t nhub, int64_t n,
                                                         const int64_t *__restrict__ trp,
                                                         unsigned long long *__restrict__ cur,
                                                         unsigned *__restrict__ boff, unsigned long long *__restrict__ bw)
{
    // hot row x: its counter, and its length and hub bitmap words as two
    // 16-bit halves (0xFFFF: read the global value).  32 KiB of LDS keep
    // four workgroups on a CU, so the whole grid is resident at once.
    __shared__ unsigned hot[PLAN_HOT];
    __shared__ unsigned hmeta[PLAN_HOT];
    const uint64_t lmask = (1ull << TC_PLAN_LEN_BITS) - 1;
    const int64_t nh = n < PLAN_HOT ? n : PLAN_HOT;
    for (int x = threadIdx.x; x < PLAN_HOT; x += PLAN_BLOCK) {
        hot[x] = 0u;
        const uint64_t len = x < nh ? (rowpk[x] & lmask) : 0u;
        const unsigned words = x < nhub ? hubw[x] : 0u;
        hmeta[x] = (unsigned)min(len, (uint64_t)0xFFFF) | min(words, 0xFFFFu) << 16;
    }
    __syncthreads();
    const unsigned lane = lane_id();
    const int64_t share = (nnz + gridDim.x - 1) / gridDim.x;
    const int64_t e0 = (int64_t)blockIdx.x * share, e1 = min(nnz, e0 + share);
    for (int64_t base = e0 + (threadIdx.x & ~63u); base < e1; base += PLAN_BLOCK) {
        const int64_t e = base + lane;
        int32_t i = -1;
        unsigned v = 0;
        if (e < e1) {
            i = rowid[e];
            const int32_t j = ci[e];
            const uint64_t pk = rowpk[i];
            const int64_t p = e - (int64_t)(pk >> TC_PLAN_LEN_BITS), len = (int64_t)(pk & lmask);
            if (j < PLAN_HOT) {
                const unsigned m = hmeta[j];
                const int64_t lj = (m & 0xFFFFu) != 0xFFFFu ? (int64_t)(m & 0xFFFFu) : (int64_t)(rowpk[j] & lmask);
                if (lj > 0 && p > 0) {
                    bool b_side = plan_cold_b(p, lj, nhub);
                    if (j < nhub) b_side = plan_hub_b(p, lj, (m >> 16) != 0xFFFFu ? (int64_t)(m >> 16) : hubw[j]);
                    if (b_side) atomicAdd(&hot[j], 1u);
                }
            }
            if (j >= nhub && tc_bitmap_pair(j, p)) v = (unsigned)((j + 31) >> 5);   // hub pairs: plan_hub_b
            if (p == len - 1 && i <= TC_BM_IDS)   // the row's last (largest) id
                v = max(v, i < nhub ? (unsigned)((j >> 5) + 1) : tc_full_words(j, len));
        }
        const WaveRun w = wave_run(i);
        const uint64_t acc = __ballot(v > 0) & w.run;
        if (acc) {
            const int last = 63 - __clzll((unsigned long long)acc);
            const unsigned m = (unsigned)__shfl((int)v, last, 64);
            if (lane == w.head) atomicMax(&bw[i], (unsigned long long)m);
        }
    }
    __syncthreads();
    const int64_t bstart = trp[n];
    unsigned *mine = boff + (size_t)blockIdx.x * PLAN_HOT;
    for (int x = threadIdx.x; x < nh; x += PLAN_BLOCK)
        mine[x] = hot[x] ? (unsigned)((int64_t)atomicAdd(&cur[n + x], (unsigned long long)hot[x]) - bstart) : 0u;
}

// The rows with bitmap words (off[r + 1] > off[r]), listed in
// rows[0 .. *count) (count zero on entry): they are contiguous runs of
// labels, so the build below spreads them over all waves through this list.
// Each workgroup reserves its range with one atomic.  The same launch
// writes lowpk (see low_pack below) for the rows j < nd.
__device__ void low_pack(const int64_t *__restrict__ Lrp, const int32_t *__restrict__ Lci,
                         const int64_t *__restrict__ boff, int64_t nd, int64_t nhub, ulonglong2 *__restrict__ lowpk);

__global__ __launch_bounds__(256) void k_bitmap_list(const int64_t *__restrict__ off, int64_t n,
                                                     int32_t *__restrict__ rows, unsigned long long *count,
                                                     const int64_t *__restrict__ Lrp,
                                                     const int32_t *__restrict__ Lci, int64_t nd, int64_t nhub,
                                                     ulonglong2 *__restrict__ lowpk)
{
    low_pack(Lrp, Lci, off, nd, nhub, lowpk);
    __shared__ unsigned sc[256];
    __shared__ unsigned long long base_s;
    const int64_t share = (n + gridDim.x - 1) / gridDim.x;
    const int64_t v0 = (int64_t)blockIdx.x * share, v1 = min(n, v0 + share);
    unsigned c = 0;
    for (int64_t v = v0 + threadIdx.x; v < v1; v += 256) c += off[v + 1] > off[v] ? 1u : 0u;
    sc[threadIdx.x] = c;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
        const unsigned y = (int)threadIdx.x >= o ? sc[threadIdx.x - o] : 0u;
        __syncthreads();
        sc[threadIdx.x] += y;
        __syncthreads();
    }
    if (threadIdx.x == 255) base_s = sc[255] ? atomicAdd(count, (unsigned long long)sc[255]) : 0;
    __syncthreads();
    unsigned long long pos = base_s + sc[threadIdx.x] - c;
    for (int64_t v = v0 + threadIdx.x; v < v1; v += 256)
        if (off[v + 1] > off[v]) rows[pos++] = (int32_t)v;
}

// One listed row per wave: the bits of the row's ids below 32 words (a
// prefix of the sorted row) gathered in the wave's LDS, then written out.
constexpr int BITMAP_BLOCK = 256;

__global__ __launch_bounds__(BITMAP_BLOCK) void k_bitmap_build(const int32_t *__restrict__ rows,
                                                               const unsigned long long *__restrict__ count,
                                                               const int64_t *__restrict__ Lrp,
                                                               const int32_t *__restrict__ Lci,
                                                               const int64_t *__restrict__ off,
                                                               uint32_t *__restrict__ bits)
{
    __shared__ uint32_t buf[BITMAP_BLOCK / 64][TC_BM_WORDS];
    uint32_t *wb = buf[threadIdx.x / 64];
    const unsigned lane = lane_id();
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / 64;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / 64;
    const int64_t nrows = (int64_t)*count;
    for (int64_t c = wave; c < nrows; c += nw) {
        const int32_t r = rows[c];
        const int64_t ob = off[r];
        const int nwr = (int)(off[r + 1] - ob);
        const int64_t b = Lrp[r], e = Lrp[r + 1];
        for (int x = lane; x < nwr; x += 64) wb[x] = 0u;
        wave_sync();
        const int32_t lim = 32 * nwr;
        for (int64_t t0 = b; t0 < e; t0 += 64) {
            const int64_t t = t0 + lane;
            const int32_t x = t < e ? Lci[t] : INT32_MAX;
            if (x < lim) atomicOr(&wb[x >> 5], 1u << (x & 31));
            if (__shfl(x, 63, 64) >= lim) break;   // the row ascends
        }
        wave_sync();
        for (int x = lane; x < nwr; x += 64) bits[ob + x] = wb[x];
        wave_sync();
    }
}

// For the rows j < nd (the lowest ids, whose columns hold most entries of
// L): lowpk[j] = {rowpk[j], TC_PLAN_BITS | (words << TC_PLAN_WORDS_SHIFT)
// | offset of row j's bitmap when an A pair should read row j as bits
// (tc_full_words > 0), else 0}.  The fill gathers this 16-byte entry (the
// table, 0.4 MB at nd = 24,577, stays in L2) instead of rowpk for those
// columns.
// (grid-stride over the launch of k_bitmap_list)
__device__ void low_pack(const int64_t *__restrict__ Lrp, const int32_t *__restrict__ Lci,
                         const int64_t *__restrict__ boff, int64_t nd, int64_t nhub, ulonglong2 *__restrict__ lowpk)
{
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < nd; j += (int64_t)gridDim.x * blockDim.x) {
        const int64_t b = Lrp[j], len = Lrp[j + 1] - b;
        const int64_t last = len > 0 ? Lci[b + len - 1] : 0;
        const unsigned w = len == 0 ? 0u : j < nhub ? (unsigned)((last >> 5) + 1) : tc_full_words(last, len);
        lowpk[j] = make_ulonglong2(plan_pack(b, len),
                                   w ? TC_PLAN_BITS | ((uint64_t)w << TC_PLAN_WORDS_SHIFT) | (uint64_t)boff[j] : 0ull);
    }
}

// Each wave takes PLAN_ILP windows of 64 consecutive entries per iteration
// and runs them stage by stage (their loads, then their gathers, then
// their atomics), so a wave waits for each round trip once per PLAN_ILP
// windows: the kernel is bound by the latency of gathers and atomics that
// miss L2.  Every lane of a wave runs every iteration (the loop bound is
// uniform), as wave_run's ballots and shuffles need.
constexpr int PLAN_ILP = 2;

// cur (the region starts, hot rows already advanced by k_plan_hot) holds
// the write cursor of each virtual row; the order of the entries within a
// row is immaterial.  Hot B rows hand out positions from LDS as offsets
// from bstart = trp[n], the first B-side slot, starting at the workgroup's
// reservation.  A B pair that tc_bitmap_pair accepts gets the entry
// TC_PLAN_BITS | (offset of row i's bitmap) in the same slot, and an A
// pair whose row j reads better as bits gets lowpk[j].y.
__global__ __launch_bounds__(PLAN_BLOCK) void k_plan_fill(const int32_t *__restrict__ rowid,
                                                          const int32_t *__restrict__ ci, int64_t nnz,
                                                          const uint64_t *__restrict__ rowpk, int64_t n,
                                                          const int64_t *__restrict__ trp,
                                                          const unsigned *__restrict__ boff,
                                                          const int64_t *__restrict__ bitoff,
                                                          const ulonglong2 *__restrict__ lowpk, int64_t nd,
                                                          int64_t nhub,
                                                          unsigned long long *__restrict__ cur,
                                                          uint64_t *__restrict__ ent)
{
    __shared__ unsigned hot[PLAN_HOT];
    const int64_t bstart = trp[n];
    const unsigned *mine = boff + (size_t)blockIdx.x * PLAN_HOT;
    for (int x = threadIdx.x; x < PLAN_HOT && x < n; x += PLAN_BLOCK)
        hot[x] = mine[x];
    __syncthreads();
    const int64_t share = (nnz + gridDim.x - 1) / gridDim.x;
    const int64_t e0 = (int64_t)blockIdx.x * share, e1 = min(nnz, e0 + share);
    const unsigned lane = lane_id();
    const uint64_t lmask = (1ull << TC_PLAN_LEN_BITS) - 1;
    const int64_t first = (int64_t)(threadIdx.x / 64) * PLAN_ILP * 64 + lane;
    for (int64_t base = e0; base < e1; base += (int64_t)PLAN_BLOCK * PLAN_ILP) {
        int32_t i[PLAN_ILP], j[PLAN_ILP];
        uint64_t pi[PLAN_ILP], pj[PLAN_ILP], fb[PLAN_ILP];
#pragma unroll
        for (int k = 0; k < PLAN_ILP; k++) {
            const int64_t e = base + first + 64 * k;
            i[k] = e < e1 ? rowid[e] : -1;
            j[k] = e < e1 ? ci[e] : 0;
        }
#pragma unroll
        for (int k = 0; k < PLAN_ILP; k++) {
            pi[k] = i[k] >= 0 ? rowpk[i[k]] : 0ull;
            pj[k] = 0ull;
            fb[k] = 0ull;
            if (i[k] >= 0 && j[k] < nd) {
                const ulonglong2 lp = lowpk[j[k]];
                pj[k] = lp.x;
                fb[k] = lp.y;
            } else if (i[k] >= 0) {
                pj[k] = rowpk[j[k]];
            }
        }
        // row i's region (A pairs, hub pairs that read L_j) or B row j:
        // positions from LDS (hub rows) or the row's cursor
        bool a_side[PLAN_ILP];
        int64_t bpos[PLAN_ILP];
        uint64_t aval[PLAN_ILP], bval[PLAN_ILP];
#pragma unroll
        for (int k = 0; k < PLAN_ILP; k++) {
            const int64_t e = base + first + 64 * k;
            const int64_t si = (int64_t)(pi[k] >> TC_PLAN_LEN_BITS), p = e - si, lj = (int64_t)(pj[k] & lmask);
            const bool valid = i[k] >= 0 && p > 0 && lj > 0;
            bpos[k] = -1;
            bval[k] = plan_pack(si, p);
            if (j[k] < nhub) {
                const int64_t words = (int64_t)((fb[k] & ~TC_PLAN_BITS) >> TC_PLAN_WORDS_SHIFT);
                a_side[k] = valid && !plan_hub_b(p, lj, words);
                aval[k] = lj <= words ? pj[k] : fb[k];
                if (valid && !a_side[k]) bpos[k] = bstart + (int64_t)atomicAdd(&hot[j[k]], 1u);
            } else {
                a_side[k] = valid && !plan_cold_b(p, lj, nhub);
                aval[k] = fb[k] ? fb[k] : pj[k];
                if (valid && !a_side[k]) {
                    if (tc_bitmap_pair(j[k], p)) bval[k] = TC_PLAN_BITS | (uint64_t)bitoff[i[k]];
                    if (j[k] < PLAN_HOT) bpos[k] = bstart + (int64_t)atomicAdd(&hot[j[k]], 1u);
                    else bpos[k] = (int64_t)atomicAdd(&cur[n + j[k]], 1ull);
                }
            }
        }
        // A side: one cursor atomic per row run
#pragma unroll
        for (int k = 0; k < PLAN_ILP; k++) {
            const WaveRun w = wave_run(i[k]);
            const uint64_t take = __ballot(a_side[k]) & w.run;
            unsigned long long abase = 0;
            if (lane == w.head && take) abase = atomicAdd(&cur[i[k]], (unsigned long long)__popcll(take));
            abase = (unsigned long long)__shfl((long long)abase, (int)w.head, 64);
            if (a_side[k]) ent[abase + __popcll(take & w.before)] = aval[k];
            if (bpos[k] >= 0) ent[bpos[k]] = bval[k];
        }
    }
}

// irp[r] = items of virtual row r (its entries, cur[r] - trp[r], in runs of
// up to 64), r < nv, and irp[nv] = 0.
__global__ void k_plan_items(const int64_t *__restrict__ trp, const unsigned long long *__restrict__ cur, int64_t nv,
                             int64_t *__restrict__ irp)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) irp[nv] = 0;   // the scan's last slot
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < nv;
         r += (int64_t)gridDim.x * blockDim.x)
        irp[r] = ((int64_t)cur[r] - trp[r] + 63) / 64;
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

// Item descriptors over a capacity; the item count is irp[nv], on the
// device (the plan is built without a host round trip).
__global__ void k_plan_item_work(int64_t n, const int64_t *__restrict__ trp,
                                 const unsigned long long *__restrict__ cur, const int64_t *__restrict__ irp,
                                 uint64_t *__restrict__ item, int32_t *__restrict__ item_row)
{
    const int64_t nv = 2 * n, nitems = irp[nv];
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nitems;
         k += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = plan_row_of(irp, nv, k);
        const int64_t e0 = trp[r] + 64 * (k - irp[r]);
        const int64_t e1 = min((int64_t)cur[r], e0 + 64);
        item[k] = ((uint64_t)e0 << TC_PLAN_CNT_BITS) | (uint64_t)(e1 - e0);
        item_row[k] = (int32_t)(r < n ? r : r - n);
    }
}

// Workgroups are dispatched to the 8 XCDs in turn (workgroup b runs on XCD
// b mod 8), and each XCD has its own L2: the waves of workgroup b take their
// items from the counter of eighth b mod 8 first (tc_dyn_wave).  Each
// workgroup writes its count to partial[blockIdx.x].
template <bool OFF32>
__global__ __launch_bounds__(TC_BLOCK, 8) void k_tc_split(PlanArgs a, unsigned long long *__restrict__ partial,
                                                          unsigned long long *__restrict__ ctr)
{
    __shared__ TcWaveLds lds[TC_WAVES];
    unsigned long long acc =
        tc_dyn_wave<false, OFF32>(a, lds[threadIdx.x / 64], ctr, (int)(blockIdx.x % TC_DYN_PARTS), TC_DYN_ITEMS);
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
    const size_t nv = (size_t)(2 * P->n);
    dev_free(P->trp, 8 * (nv + 1));
    dev_free(P->irp, 8 * (nv + 1));
    dev_free(P->ent, 8 * (size_t)(P->ent_cap > 0 ? P->ent_cap : 1));
    dev_free(P->item, 8 * (size_t)(P->item_cap > 0 ? P->item_cap : 1));
    dev_free(P->item_row, 4 * (size_t)(P->item_cap > 0 ? P->item_cap : 1));
    dev_free(P->boff, 8 * (size_t)(P->n + 1));
    dev_free(P->bits, 4 * (size_t)(P->bits_cap > 0 ? P->bits_cap : 1));
    dev_free(P->status, 64);
    delete P;
    G->tcplan = nullptr;
}

// Built without a host round trip: the entries go to regions of known size
// (2 nnz slots in all), the items take at most nnz/64 + one per non-empty
// virtual row and the bitmaps fewer words than L has entries (a row's
// words stay below its length), so every array is allocated at its bound.
// The item and bitmap word counts are irp[2n] and boff[n] on the device;
// the caller reads them back (with the rest of its status) and sets
// P->nitems and P->nbits.
int tc_plan_build(lagr_ctx ctx, lagr_graph G, const int32_t *rowid, const int64_t *regions, char *msg)
{
    const lagr_matrix Lm = G->L;
    const int64_t n = Lm->nrows, nv = 2 * n;
    const int64_t nnz = Lm->nvals;
    if (2 * nnz >= ((int64_t)1 << 32))
        return lagr_fail(msg, LAGR_NOT_IMPLEMENTED, "L too large for the count plan");
    TcPlan *P = new (std::nothrow) TcPlan();
    if (!P) return lagr_fail(msg, LAGR_OUT_OF_MEMORY, "count plan");
    P->n = n;
    P->nitems = -1;
    P->ent_cap = 2 * nnz;
    P->item_cap = nnz / 64 + (nv < nnz ? nv : nnz) + 1;
    // rows' words stay below their lengths, except hub rows' (at most
    // PLAN_HOT / 32 words each)
    P->bits_cap = nnz + (int64_t)PLAN_HOT * (PLAN_HOT / 32);
    G->tcplan = P;
    auto fail = [&](int rc) {
        tc_plan_free(G);
        return rc;
    };
    P->trp = (int64_t *)dev_alloc(8 * (size_t)(nv + 1));
    P->irp = (int64_t *)dev_alloc(8 * (size_t)(nv + 1));
    P->ent = (uint64_t *)dev_alloc(8 * (size_t)(P->ent_cap > 0 ? P->ent_cap : 1));
    P->item = (uint64_t *)dev_alloc(8 * (size_t)P->item_cap);
    P->item_row = (int32_t *)dev_alloc(4 * (size_t)P->item_cap);
    P->boff = (int64_t *)dev_alloc(8 * (size_t)(n + 1));
    P->bits = (uint32_t *)dev_alloc(4 * (size_t)P->bits_cap);
    P->status = (unsigned long long *)dev_alloc(64);
    if (!P->trp || !P->irp || !P->ent || !P->item || !P->item_row || !P->boff || !P->bits || !P->status)
        return fail(lagr_fail(msg, LAGR_OUT_OF_MEMORY, "count plan"));
    int rc;
    // per-workgroup hub reservations, then the hub rows' bitmap words
    unsigned *boff = (unsigned *)ws_get(ctx, WS_GEN_H, sizeof(unsigned) * ((size_t)PLAN_GRID + 1) * PLAN_HOT);
    unsigned *hubw = boff + (size_t)PLAN_GRID * PLAN_HOT;
    int64_t nhub = plan_hubs(n);
    if (G->tc_hubs >= 0) nhub = G->tc_hubs < PLAN_HOT ? (G->tc_hubs < n ? G->tc_hubs : n) : PLAN_HOT;
    uint64_t *rowpk = (uint64_t *)ws_get(ctx, WS_GEN_E, sizeof(uint64_t) * (size_t)(n > 0 ? n : 1));
    unsigned long long *cur = (unsigned long long *)ws_get(ctx, WS_TC_WORK, 8 * (size_t)(nv > 0 ? nv : 1));
    if (!boff || !rowpk || !cur) return fail(lagr_fail(msg, LAGR_OUT_OF_MEMORY, "count plan"));
    // rows needing bitmaps are listed below (n ids, then the count)
    int32_t *brows = (int32_t *)ws_get(ctx, WS_GEN_F, sizeof(int32_t) * (size_t)n + 64);
    if (!brows) return fail(lagr_fail(msg, LAGR_OUT_OF_MEMORY, "count plan"));
    unsigned long long *nbrows = (unsigned long long *)(brows + n + (n & 1));
    // regions and cursors, the bitmap words' clear, rowpk and the hub rows'
    // words (with n = 0: trp[0] and the clears)
    hipLaunchKernelGGL(k_row_pack, dim3(grid_for(nv + 1, 256, 16384)), dim3(256), 0, ctx->stream, Lm->rowptr,
                       Lm->colidx, n, rowpk, regions, P->trp, cur, P->boff, nbrows, nnz > 0 ? nhub : 0, hubw);
    if (n > 0) {
        if (nnz > 0) {
            hipLaunchKernelGGL(k_plan_hot, dim3(PLAN_GRID), dim3(PLAN_BLOCK), 0, ctx->stream, rowid, Lm->colidx,
                               nnz, rowpk, hubw, nhub, n, P->trp, cur, boff, (unsigned long long *)P->boff);
        }
        if (hipGetLastError() != hipSuccess) return fail(lagr_fail(msg, LAGR_DEVICE_ERROR, "plan launch"));
        if ((rc = scan_exclusive_i64(ctx, P->boff, P->boff, n + 1, nullptr, msg)) < 0) return fail(rc);
        // the rows needing bitmaps, listed, then one wave each; the list's
        // launch also packs the lowest rows (lowpk)
        const int64_t nd = n < TC_BM_IDS + 1 ? n : TC_BM_IDS + 1;   // rows whose ids all lie below TC_BM_IDS
        ulonglong2 *lowpk = (ulonglong2 *)ws_get(ctx, WS_GEN_G, sizeof(ulonglong2) * (size_t)nd);
        if (!lowpk) return fail(lagr_fail(msg, LAGR_OUT_OF_MEMORY, "count plan"));
        hipLaunchKernelGGL(k_bitmap_list, dim3(grid_for(n, 256, 1024)), dim3(256), 0, ctx->stream, P->boff, n, brows,
                           nbrows, Lm->rowptr, Lm->colidx, nd, nhub, lowpk);
        hipLaunchKernelGGL(k_bitmap_build, dim3((unsigned)(ctx->num_cus * 8)), dim3(BITMAP_BLOCK), 0, ctx->stream,
                           brows, nbrows, Lm->rowptr, Lm->colidx, P->boff, P->bits);
        if (nnz > 0)
            hipLaunchKernelGGL(k_plan_fill, dim3(PLAN_GRID), dim3(PLAN_BLOCK), 0, ctx->stream, rowid, Lm->colidx,
                               nnz, rowpk, n, P->trp, boff, P->boff, lowpk, nd, nhub, cur, P->ent);
    }
    hipLaunchKernelGGL(k_plan_items, dim3(grid_for(nv, 256, 16384)), dim3(256), 0, ctx->stream, P->trp, cur, nv,
                       P->irp);
    if (hipGetLastError() != hipSuccess) return fail(lagr_fail(msg, LAGR_DEVICE_ERROR, "plan launch"));
    if ((rc = scan_exclusive_i64(ctx, P->irp, P->irp, nv + 1, nullptr, msg)) < 0) return fail(rc);
    if (n > 0) {
        hipLaunchKernelGGL(k_plan_item_work, dim3(grid_for(P->item_cap, 256, 16384)), dim3(256), 0, ctx->stream,
                           n, P->trp, cur, P->irp, P->item, P->item_row);
        if (hipGetLastError() != hipSuccess) return fail(lagr_fail(msg, LAGR_DEVICE_ERROR, "plan launch"));
    }
    return LAGR_SUCCESS;
}

namespace {

// The plan's status: out[0..1] = in[0..1] (L's longest row, the unsorted
// flag, from the preparation's kernels), out[3..5] = plan items, entries of
// L, bitmap words.
__global__ void k_tc_status(const int64_t *__restrict__ nitems, const int64_t *__restrict__ nnzL,
                            const int64_t *__restrict__ nbits, const unsigned long long *__restrict__ in,
                            unsigned long long *__restrict__ out)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        out[0] = in[0];
        out[1] = in[1];
        out[2] = 0;
        out[3] = (unsigned long long)*nitems;
        out[4] = (unsigned long long)*nnzL;
        out[5] = (unsigned long long)*nbits;
    }
}

}  // namespace

int tc_plan_status(lagr_ctx ctx, lagr_graph G, unsigned long long *status, char *msg)
{
    TcPlan *P = G->tcplan;
    const int64_t n = G->L->nrows;
    hipLaunchKernelGGL(k_tc_status, dim3(1), dim3(64), 0, ctx->stream, P->irp + 2 * n, G->L->rowptr + n,
                       P->boff + n, status, P->status);
    LAUNCH_CHECK();
    return LAGR_SUCCESS;
}

bool tc_plan_fits(int64_t max_row) { return max_row < ((int64_t)1 << TC_PLAN_LEN_BITS); }

int tc_plan_settle(lagr_ctx ctx, lagr_graph G, unsigned long long *status, int64_t nnz, bool *unsorted, char *msg)
{
    TRY(tc_plan_status(ctx, G, status, msg));
    unsigned long long st[6] = {0, 0, 0, 0, 0, 0};
    TRY(read_back(ctx, st, G->tcplan->status, sizeof(st), msg));
    return tc_plan_settle_host(G, st, nnz, unsorted, msg);
}

int tc_plan_settle_host(lagr_graph G, const unsigned long long *st, int64_t nnz, bool *unsorted, char *msg)
{
    TcPlan *P = G->tcplan;
    if ((int64_t)st[4] != nnz)
        return lagr_fail(msg, LAGR_INVALID_OBJECT, "L has %lld entries, expected %lld", (long long)st[4],
                         (long long)nnz);
    *unsorted = st[1] != 0;
    if (st[0] >= ((unsigned long long)1 << TC_PLAN_LEN_BITS))
        return lagr_fail(msg, LAGR_NOT_IMPLEMENTED, "rows of L too long for the count plan");
    G->L_maxrow = (int64_t)st[0];
    P->nitems = (int64_t)st[3];
    P->nbits = (int64_t)st[5];
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

// The count's ids sit below 2^30 entries of L, and its bitmap words below
// 2^30 words (the bitmaps hold fewer words than L has entries, plus at most
// PLAN_HOT / 32 words for each of PLAN_HOT hub rows): 32-bit byte offsets
// reach them.
static inline bool tc_off32(const lagr_matrix L)
{
    return L->nvals < ((int64_t)1 << 30) - ((int64_t)1 << 20);
}

// With the plan's status still on the device (G->tc_status_pending), the
// count reads the item count there, its grid is sized from the item
// capacity, and the status comes back with the count in one read.
static int tc_on_lower(lagr_ctx ctx, const lagr_graph G, int64_t *ntri, char *msg)
{
    const lagr_matrix L = G->L;
    TcPlan *P = G->tcplan;
    const bool pending = G->tc_status_pending;
    const int64_t items = pending ? P->item_cap : P->nitems;
    // up to eight resident waves per SIMD (the LDS and register budgets of
    // k_tc_split allow it), fewer for a small plan, and a multiple of 8
    // workgroups (one eighth of the items per XCD); the work counters follow
    // the partials
    const int64_t want = (items + TC_DYN_ITEMS * TC_WAVES - 1) / (TC_DYN_ITEMS * TC_WAVES);
    const int64_t most = (int64_t)ctx->num_cus * 8;
    const unsigned blocks = (unsigned)(((want < most ? want : most) + TC_DYN_PARTS - 1) / TC_DYN_PARTS * TC_DYN_PARTS);
    const size_t nctr = (size_t)TC_DYN_STRIDE * TC_DYN_PARTS;
    unsigned long long *tot = (unsigned long long *)ws_get(ctx, WS_TC, 8 * ((size_t)blocks + 1 + nctr));
    if (!tot) return lagr_fail(msg, LAGR_OUT_OF_MEMORY, "tc counter");
    if (items > 0) {
        unsigned long long *ctr = tot + 1 + blocks;
        TRY(fill_i64(ctx, (int64_t *)ctr, (int64_t)nctr, 0, msg));
        PlanArgs a{P->nitems, pending ? P->irp + 2 * L->nrows : nullptr, L->rowptr, L->colidx, P->ent, P->item,
                   P->item_row, P->bits};
        if (tc_off32(L))
            TIMED(ctx, "tc_split",
                  hipLaunchKernelGGL(k_tc_split<true>, dim3(blocks), dim3(TC_BLOCK), 0, ctx->stream, a, tot + 1, ctr));
        else
            TIMED(ctx, "tc_split",
                  hipLaunchKernelGGL(k_tc_split<false>, dim3(blocks), dim3(TC_BLOCK), 0, ctx->stream, a, tot + 1, ctr));
        LAUNCH_CHECK();
        hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, ctx->stream, tot + 1, (int64_t)blocks, tot);
        LAUNCH_CHECK();
    } else {
        TRY(fill_i64(ctx, (int64_t *)tot, 1, 0, msg));
    }
    unsigned long long h = 0;
    if (!pending) {
        TRY(read_back(ctx, &h, tot, sizeof(h), msg));
    } else {
        // the count and the plan's status in one wait
        unsigned long long st[6];
        TRY(stage_to_host(ctx, 0, tot, sizeof(h), false, msg));
        TRY(stage_to_host(ctx, 8, P->status, sizeof(st), true, msg));
        memcpy(&h, ctx->pinned, sizeof(h));
        memcpy(st, (char *)ctx->pinned + 8, sizeof(st));
        bool unsorted = false;
        TRY(tc_plan_settle_host(G, st, L->nvals, &unsorted, msg));
        if (unsorted) return lagr_fail(msg, LAGR_DEVICE_ERROR, "a row of L was left unsorted");
        G->tc_status_pending = false;
    }
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

// ------------------------------------------------------------ autotuning

// The count plan's hub columns for this graph: each candidate share of the
// vertices (none, then n / 1024 .. n / 128, at most PLAN_HOT) rebuilds the
// preparation and times the whole count (host clock around lagr_tc, median
// of 3); the fastest is kept in G and its plan left built.
extern "C" int lagr_tc_autotune(int64_t *hubs, lagr_graph G, lagr_ctx ctx, char *msg)
{
    if (!G || !ctx) return lagr_fail(msg, LAGR_NULL_POINTER, "NULL argument");
    if (ctx->device < 0) return lagr_fail(msg, LAGR_DEVICE_ERROR, "validation-only context");
    const int64_t n = G->A->nrows;
    std::vector<int64_t> cand = {0};
    for (int sh = 10; sh >= 7; sh--) {
        int64_t h = n >> sh;
        if (h > PLAN_HOT) h = PLAN_HOT;
        if (h > cand.back()) cand.push_back(h);
    }
    int64_t best = -1;
    double best_t = 0.0;
    int64_t t_ref = -1;
    for (const int64_t h : cand) {
        G->tc_hubs = h;
        double ts[3];
        for (int r = 0; r < 3; r++) {
            TRY(lagr_graph_delete_properties(G, ctx, msg));
            const auto t0 = std::chrono::steady_clock::now();
            int64_t t = 0;
            TRY(lagr_tc(&t, G, LAGR_TC_DEFAULT, ctx, msg));
            ts[r] = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
            if (t_ref < 0) t_ref = t;
            if (t != t_ref) return lagr_fail(msg, LAGR_DEVICE_ERROR, "tuning candidates counted differently");
        }
        std::sort(ts, ts + 3);
        if (best < 0 || ts[1] < best_t) {
            best = h;
            best_t = ts[1];
        }
    }
    G->tc_hubs = best;
    TRY(lagr_graph_delete_properties(G, ctx, msg));
    TRY(lagr_property_tc_lower(G, ctx, msg));
    if (hubs) *hubs = best;
    return lagr_ok(msg);
}

// ---------------------------------------------- allocation-free count

// Scratch of the allocation-free count: one partial per workgroup, the
// total, and the per-XCD work counters, in a fixed device array (each GPU
// the library runs on holds its own copy until the process ends).  Host
// code never passes the array's name to a kernel: its device address comes
// from hipGetSymbolAddress, taken once per device.
constexpr int TC_NOALLOC_MAX_BLOCKS = 4096;
constexpr size_t TC_NOALLOC_WORDS =
    (size_t)TC_NOALLOC_MAX_BLOCKS + 1 + (size_t)TC_DYN_STRIDE * TC_DYN_PARTS;
static __device__ __align__(256) unsigned long long scratch[TC_NOALLOC_WORDS];

constexpr int TC_NOALLOC_MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static unsigned long long *g_scratch_dev[TC_NOALLOC_MAX_DEVICES];

// The device address of `scratch` on ctx's device (looked up on the first
// call there, with that device current).
static int scratch_address(lagr_ctx ctx, unsigned long long **out, char *msg)
{
    const int dev = ctx->device;
    if (dev < 0 || dev >= TC_NOALLOC_MAX_DEVICES)
        return lagr_fail(msg, LAGR_INVALID_VALUE, "device %d has no scratch slot", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        int cur = -1;
        HIP_TRY(hipGetDevice(&cur));
        if (cur != dev) HIP_TRY(hipSetDevice(dev));
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != dev) (void)hipSetDevice(cur);
        if (e != hipSuccess || !p)
            return lagr_fail(msg, LAGR_DEVICE_ERROR, "scratch address: %s", hipGetErrorString(e));
        g_scratch_dev[dev] = (unsigned long long *)p;
    }
    *out = g_scratch_dev[dev];
    return LAGR_SUCCESS;
}

extern "C" int lagr_tc_adv_noalloc(int64_t *ntriangles_dev, const lagr_graph G, lagr_ctx ctx, char *msg)
{
    if (!ntriangles_dev || !G || !ctx) return lagr_fail(msg, LAGR_NULL_POINTER, "NULL argument");
    if (ctx->device < 0) return lagr_fail(msg, LAGR_DEVICE_ERROR, "validation-only context");
    if (!G->L || !G->tcplan || G->tc_status_pending)
        return lagr_fail(msg, LAGR_PROPERTY_MISSING, "tc_lower property not computed");
    const lagr_matrix L = G->L;
    const TcPlan *P = G->tcplan;
    // the grid of lagr_tc_adv, which must fit the scratch
    const int64_t want = (P->nitems + TC_DYN_ITEMS * TC_WAVES - 1) / (TC_DYN_ITEMS * TC_WAVES);
    const int64_t most = (int64_t)ctx->num_cus * 8;
    const int64_t blocks = ((want < most ? want : most) + TC_DYN_PARTS - 1) / TC_DYN_PARTS * TC_DYN_PARTS;
    if (blocks > TC_NOALLOC_MAX_BLOCKS)
        return lagr_fail(msg, LAGR_INVALID_VALUE,
                         "the count needs %lld workgroup partials; the fixed scratch holds %d",
                         (long long)blocks, TC_NOALLOC_MAX_BLOCKS);
    unsigned long long *sp = nullptr;
    TRY(scratch_address(ctx, &sp, msg));
    if (P->nitems > 0) {
        unsigned long long *part = sp;
        unsigned long long *ctr = sp + TC_NOALLOC_MAX_BLOCKS + 1;
        // the counters keep the previous call's values: clear them (a fill
        // kernel, so the call may also be captured into a graph)
        TRY(fill_i64(ctx, (int64_t *)ctr, (int64_t)TC_DYN_STRIDE * TC_DYN_PARTS, 0, msg));
        PlanArgs a{P->nitems, nullptr, L->rowptr, L->colidx, P->ent, P->item, P->item_row, P->bits};
        if (tc_off32(L))
            hipLaunchKernelGGL(k_tc_split<true>, dim3((unsigned)blocks), dim3(TC_BLOCK), 0, ctx->stream, a, part, ctr);
        else
            hipLaunchKernelGGL(k_tc_split<false>, dim3((unsigned)blocks), dim3(TC_BLOCK), 0, ctx->stream, a, part, ctr);
        LAUNCH_CHECK();
        hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, ctx->stream, part, blocks,
                           (unsigned long long *)ntriangles_dev);
        LAUNCH_CHECK();
    } else {
        TRY(fill_i64(ctx, ntriangles_dev, 1, 0, msg));
    }
    return lagr_ok(msg);
}

// The three methods count the same C<s(L)> = L plus.pair L^T, reduced
// (Algorithm 6): the count plan (the default), the fused masked dot of
// lagr_mxm_reduce over L, or Algorithm 6 as written -- C formed by
// lagr_mxm, then reduced by lagr_reduce_scalar.
extern "C" int lagr_tc(int64_t *ntriangles, lagr_graph G, int method, lagr_ctx ctx, char *msg)
{
    if (!ntriangles || !G || !ctx) return lagr_fail(msg, LAGR_NULL_POINTER, "NULL argument");
    if (method < LAGR_TC_DEFAULT || method > LAGR_TC_MXM)
        return lagr_fail(msg, LAGR_INVALID_VALUE, "unknown triangle-count method %d", method);
    if (method == LAGR_TC_DEFAULT) {
        // the plan's status read once, with the count
        TRY(tc_lower_build(G, ctx, true, msg));
        const int rc = lagr_tc_adv(ntriangles, G, ctx, msg);
        if (rc < 0 && G->tc_status_pending) {
            // a failed count leaves no half-known operand behind
            (void)hipStreamSynchronize(ctx->stream);
            tc_plan_free(G);
            lagr_matrix_free(&G->L);
            G->L_maxrow = -1;
            G->tc_status_pending = false;
        }
        return rc;
    }
    TRY(lagr_property_tc_lower(G, ctx, msg));
    const lagr_matrix Lm = G->L;
    const uint32_t desc = LAGR_DESC_STRUCT | LAGR_DESC_TRAN1;
    if (method == LAGR_TC_DOT) {
        int64_t t = 0;
        TRY(lagr_mxm_reduce(&t, Lm, LAGR_PLUS_PAIR, Lm, Lm, desc, ctx, msg));
        *ntriangles = t;
        return lagr_ok(msg);
    }
    lagr_matrix C = nullptr;
    TRY(lagr_matrix_new(&C, LAGR_INT64, Lm->nrows, Lm->ncols, ctx, msg));
    int rc = lagr_mxm(C, Lm, LAGR_NOOP, LAGR_PLUS_PAIR, Lm, Lm, desc, ctx, msg);
    int64_t t = 0;
    if (rc >= 0) rc = lagr_reduce_scalar(&t, LAGR_NOOP, LAGR_PLUS, C, ctx, msg);
    lagr_matrix_free(&C);
    if (rc < 0) return rc;
    *ntriangles = t;          // no entry (LAGR_NO_VALUE): no triangle
    return lagr_ok(msg);
}
